"""Launch-shape autotuner for a Simulation.

Every option it touches (3D plane kernels and 2D tile kernels and their tile rows, tile depths,
the interleaved chunk schedule, tile rows, rows per thread, marching chunk, persistent grid)
changes only the work decomposition -- results are bitwise
identical -- so candidates are timed on the live state: the state is saved,
each candidate runs a few steps with per-kernel HIP events, and the state is
restored.  The winner is applied and stored in a JSON cache keyed by the
problem class (dimension, mechanisms, size bucket, domain-count bucket,
device architecture).
"""
import json
import math
import os

from .native import (FW_OPT_MARCH_CHUNK, FW_OPT_PERSISTENT, FW_OPT_PLANE_KERNELS, FW_OPT_PLANE_ROWS,
                     FW_OPT_PRS_PLANES, FW_OPT_ROWS_PER_THREAD, FW_OPT_STEP_CHUNK, FW_OPT_TILE_ROWS,
                     FW_OPT_VEL_PLANES)

CACHE_PATH = os.path.join(os.path.expanduser("~"), ".cache", "fw25_autotune.json")

# the library's defaults (3D with N >= 3; 2D grids default to 8-row tile
# kernels, 3D grids with N <= 2 to 8-row tiles of 2 velocity planes)
DEFAULT = {"plane_kernels": -1, "plane_rows": 4, "tile_rows": 4, "rows_per_thread": 1, "march_chunk": 0,
           "persistent": 0, "vel_planes": 1, "prs_planes": 0,    # prs_planes 0: the library's default for N
           "step_chunk": -1}


def candidates(ndim):
    out = []
    if ndim == 3:
        # the plane kernels ignore the marching shape
        for plane in (-1,):
            for prow in (4, 8):
                for vp in (1, 2, 4):
                    for pp in (2, 4, 8):
                        # interleaved chunks: the library's choice for the grid, or whole-grid launches
                        for sc in (-1, 0):
                            out.append({"plane_kernels": plane, "plane_rows": prow, "tile_rows": 4,
                                        "rows_per_thread": 1, "march_chunk": 0, "persistent": 0,
                                        "vel_planes": vp, "prs_planes": pp, "step_chunk": sc})
        for rows, rpt in ((4, 1), (8, 1), (16, 1), (16, 2), (8, 2)):
            for persistent in (0, 4):
                for chunk in (0, 24, 96):
                    out.append({"plane_kernels": 0, "tile_rows": rows, "rows_per_thread": rpt, "march_chunk": chunk,
                                "persistent": persistent})
    else:
        if ndim == 2:
            # 2D tile kernels (64 x R tiles, one per block) ignore the marching shape
            for prow in (4, 8, 16):
                out.append({"plane_kernels": 1, "plane_rows": prow, "tile_rows": 4, "rows_per_thread": 1,
                            "march_chunk": 0, "persistent": 0})
        for persistent in (0, 2, 4, 8):
            for chunk in ((0, 16, 32) if ndim == 2 else (0,)):
                out.append({"plane_kernels": 0, "tile_rows": 4, "rows_per_thread": 1, "march_chunk": chunk,
                            "persistent": persistent})
    return out


def _default_rows_planes(sim):
    """The library's default tile rows and velocity planes for this grid."""
    if sim.ndim == 2:
        return 8, 1
    return (8, 2) if (sim.ndim == 3 and sim.n_mech <= 2) else (4, 1)


def apply(sim, cfg):
    rows, vp = _default_rows_planes(sim)
    sim.set_option(FW_OPT_PLANE_KERNELS, cfg.get("plane_kernels", -1))
    sim.set_option(FW_OPT_PLANE_ROWS, cfg.get("plane_rows", rows))
    sim.set_option(FW_OPT_VEL_PLANES, cfg.get("vel_planes", vp))
    pp = cfg.get("prs_planes", 0)
    sim.set_option(FW_OPT_PRS_PLANES, pp if pp else (2 if sim.n_mech >= 3 else 8))
    sim.set_option(FW_OPT_STEP_CHUNK, cfg.get("step_chunk", -1))
    # rows per thread first when shrinking to 4-row tiles is requested
    sim.set_option(FW_OPT_ROWS_PER_THREAD, 1)
    sim.set_option(FW_OPT_TILE_ROWS, cfg["tile_rows"])
    sim.set_option(FW_OPT_ROWS_PER_THREAD, cfg["rows_per_thread"])
    sim.set_option(FW_OPT_MARCH_CHUNK, cfg["march_chunk"])
    sim.set_option(FW_OPT_PERSISTENT, cfg["persistent"])


def problem_key(sim):
    import torch
    cells = sum(int(math.prod(s)) for s in sim.shapes)
    arch = torch.cuda.get_device_properties(sim.device).gcnArchName.split(":")[0]
    return "ndim=%d|N=%d|cells~2^%d|domains~2^%d|%s" % (sim.ndim, sim.n_mech, round(math.log2(max(cells, 1))),
                                                       round(math.log2(max(sim.n_domains, 1))), arch)


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune(sim, steps=3, cands=None, cache_path=CACHE_PATH, use_cache=True):
    """Pick the fastest launch shape for sim (total ms of `steps` steps), apply
    it and return (config, {label: ms})."""
    key = problem_key(sim)
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        apply(sim, cache[key]["config"])
        return cache[key]["config"], cache[key].get("timings", {})
    cands = cands or candidates(sim.ndim)
    snap = sim.save_state()
    timings = {}
    best, best_ms = None, float("inf")
    for cfg in cands:
        apply(sim, cfg)
        sim.load_state(snap)
        sim.time_kernels(1)                  # warm the launch shape
        sim.load_state(snap)
        ms = float(sum(sim.time_kernels(steps)))
        timings[json.dumps(cfg, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = cfg, ms
    apply(sim, best)
    sim.load_state(snap)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = {"config": best, "ms_per_step": best_ms / steps, "timings": timings}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, timings
