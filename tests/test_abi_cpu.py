"""The C ABI without a GPU: the library loads, exports every declared entry
point, and its host-side validation returns the documented error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fw25.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2606_11103_amd import native
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(native.lib, n), n
        assert n in native.SIGNATURES, n
    assert native.lib.fw_abi_version() == 2


def _create(ndim=2, shapes=((64, 48, 1),), dx=1e-4, dt=1e-8, nmech=2, pml=6, params=None):
    from paper_2606_11103_amd import native
    h = ctypes.c_void_p()
    shp = np.ascontiguousarray(np.array(shapes, dtype=np.int64).reshape(-1))
    pp = None
    if params is not None:
        params = np.ascontiguousarray(np.array(params, dtype=np.float64))
        pp = ctypes.c_void_p(params.ctypes.data)
    rc = native.lib.fw_create_grid(ctypes.byref(h), ndim, len(shapes), ctypes.c_void_p(shp.ctypes.data),
                                   dx, dt, nmech, pml, pp)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=0), -1), (dict(ndim=4), -1), (dict(nmech=0), -1), (dict(nmech=5), -1),
    (dict(shapes=((20, 48, 1),)), -1),            # 20 <= 2*6 + 8
    (dict(shapes=((64, 48, 2),)), -1),            # unused dim must be 1
    (dict(dx=0.0), -1), (dict(dt=-1.0), -1), (dict(pml=-1), -1),
    (dict(params=(2.0, 1e6, 0.0)), -1),           # R0 must be < 1
])
def test_create_grid_rejects(kw, code):
    rc, h = _create(**kw)
    assert rc == code
    assert not h.value


def test_workspace_bytes_and_state_order():
    from paper_2606_11103_amd import native
    lib = native.lib
    rc, h = _create()
    assert rc == 0
    nb = lib.fw_workspace_bytes(h)
    cells = 64 * 48
    # p, vx, vy, 2 x 2 psi1 and 2 psi2 (N = 2) and 2 + 2 CPML fields, plus the class map
    assert nb >= cells * 4 * (1 + 2 + 2 * 2 + 2 + 4) + cells
    assert lib.fw_state_bytes(h) > 0
    # stepping before anything is set up
    assert lib.fw_step(h, 1, None) == native.FW_ESTATE
    assert lib.fw_prepare(h) == native.FW_ESTATE
    assert lib.fw_prepare(None) == native.FW_EINVAL
    k = np.ones(4)
    assert lib.fw_set_relaxation_table(h, 2, ctypes.c_void_p(k.ctypes.data), ctypes.c_void_p(k.ctypes.data),
                                       ctypes.c_void_p(k.ctypes.data)) == native.FW_ESTATE
    assert b"media" in lib.fw_last_error()
    assert lib.fw_destroy(h) == 0


def _media(h, cls, base, c, rho, beta, amp=0.0):
    from paper_2606_11103_amd import native
    arrs = [np.ascontiguousarray(np.asarray(a, dt)) for a, dt in
            ((cls, np.uint8), (base, np.int32), (c, np.float64), (rho, np.float64), (beta, np.float64))]
    ptrs = [ctypes.c_void_p(a.ctypes.data) for a in arrs]
    return native.lib.fw_set_media(h, ptrs[0], ptrs[1], len(arrs[2]), ptrs[2], ptrs[3], ptrs[4], amp,
                                   ctypes.c_uint64(1))


def test_adjoint_calls_validate_without_gpu():
    """The adjoint's entry points check their arguments and the call order on
    the host: NULL pointers (FW_EINVAL), the class alpha0 values before the
    media (FW_ESTATE), and a workspace request with n_steps < 1 (-1)."""
    from paper_2606_11103_amd import native
    lib = native.lib
    rc, h = _create()
    assert rc == 0
    a0 = np.ones(2)
    assert lib.fw_set_class_alpha0(h, 2, ctypes.c_void_p(a0.ctypes.data)) == native.FW_ESTATE
    assert lib.fw_set_class_alpha0(h, 2, None) == native.FW_EINVAL
    assert lib.fw_adjoint_workspace_bytes(h, 0, 10) == -1
    nb = lib.fw_adjoint_workspace_bytes(h, 100, 10)
    assert nb > 10 * lib.fw_state_bytes(h)
    buf = ctypes.c_void_p(256)
    assert lib.fw_adjoint(h, 100, 10, None, nb, buf, buf, buf, None) == native.FW_EINVAL
    assert lib.fw_adjoint(h, 100, 10, buf, nb, buf, None, buf, None) == native.FW_EINVAL
    assert lib.fw_adjoint_modulus(h, 100, 10, buf, nb, buf, buf, None, None) == native.FW_EINVAL
    # dJ/dalpha0 requested before fw_set_class_alpha0
    assert lib.fw_adjoint(h, 100, 10, buf, nb, buf, buf, buf, None) == native.FW_ESTATE
    assert lib.fw_destroy(h) == 0


def test_set_media_validation_without_gpu():
    from paper_2606_11103_amd import native
    rc, h = _create(dt=1e-8)
    cls = np.zeros(64 * 48, np.uint8)
    # class index beyond n_classes
    bad = cls.copy()
    bad[5] = 2
    assert _media(h, bad, [0], [1500.0, 1600.0], [1000.0, 1000.0], [0.0, 0.0]) == native.FW_EINVAL
    # non-positive density
    assert _media(h, cls, [0], [1500.0], [0.0], [0.0]) == native.FW_EINVAL
    # noise amplitude out of range
    assert _media(h, cls, [0], [1500.0], [1000.0], [0.0], amp=0.7) == native.FW_EINVAL
    # stability bound: 2D limit is c dt / dx < 0.5497
    assert _media(h, cls, [0], [6000.0], [1000.0], [0.0]) == native.FW_EUNSTABLE
    assert b"time step" in native.lib.fw_last_error()
    # valid arguments but no workspace bound yet
    assert _media(h, cls, [0], [1500.0], [1000.0], [0.0]) == native.FW_ESTATE
    native.lib.fw_destroy(h)


def test_sources_and_receivers_validation_without_gpu():
    from paper_2606_11103_amd import native
    lib = native.lib
    rc, h = _create()
    dom = np.zeros(2, np.int32)
    P = lambda a: ctypes.c_void_p(a.ctypes.data)
    cells = np.array([10, 64 * 48], np.int64)           # second is outside the domain
    widx = np.zeros(2, np.int32)
    waves = np.zeros((1, 8), np.float32)
    assert lib.fw_set_sources(h, 2, P(dom), P(cells), P(widx), 1, P(waves), 8) == native.FW_EINVAL
    cells = np.array([10, 10], np.int64)                 # duplicate cell
    assert lib.fw_set_sources(h, 2, P(dom), P(cells), P(widx), 1, P(waves), 8) == native.FW_EINVAL
    cells = np.array([10, 11], np.int64)
    widx2 = np.array([0, 1], np.int32)                   # wave index out of range
    assert lib.fw_set_sources(h, 2, P(dom), P(cells), P(widx2), 1, P(waves), 8) == native.FW_EINVAL
    waves[0, 3] = np.nan
    assert lib.fw_set_sources(h, 2, P(dom), P(cells), P(widx), 1, P(waves), 8) == native.FW_ENONFINITE
    dom_bad = np.array([0, 1], np.int32)                 # only one domain
    assert lib.fw_set_receivers(h, 2, P(dom_bad), P(cells), 10) == native.FW_EINVAL
    assert lib.fw_set_receivers(h, 2, P(dom), P(cells), 10) == native.FW_ESTATE   # no workspace
    # caller-owned trace buffer: NULL or too small is rejected before anything else
    assert lib.fw_set_receivers_into(h, 2, P(dom), P(cells), 10, None, 20) == native.FW_EINVAL
    fake = ctypes.c_void_p(0x1000)                       # never dereferenced: the call stops first
    assert lib.fw_set_receivers_into(h, 2, P(dom), P(cells), 10, fake, 19) == native.FW_EINVAL
    assert lib.fw_set_receivers_into(h, 2, P(dom), P(cells), 10, fake, 20) == native.FW_ESTATE
    assert lib.fw_set_option(h, native.FW_OPT_TILE_ROWS, 12) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_ROWS_PER_THREAD, 3) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_MARCH_CHUNK, -1) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_TILE_ORDER, 3) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_PLANE_KERNELS, 2) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_PLANE_ROWS, 12) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_PLANE_ROWS, 16) == 0      # 2D tile kernels only
    assert lib.fw_set_option(h, native.FW_OPT_PLANE_ROWS, 8) == 0
    assert lib.fw_set_option(h, native.FW_OPT_STEP_CHUNK, 3) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_STEP_CHUNK, -2) == native.FW_EINVAL
    for v in (-1, 0, 4, 120):
        assert lib.fw_set_option(h, native.FW_OPT_STEP_CHUNK, v) == 0
    for v in (-1, 0, 1):
        assert lib.fw_set_option(h, native.FW_OPT_RESIDENT_1D, v) == 0
    for v in (-2, 2):
        assert lib.fw_set_option(h, native.FW_OPT_RESIDENT_1D, v) == native.FW_EINVAL
    assert lib.fw_set_option(h, native.FW_OPT_GRAPH_STEPS, 8) == 0
    lib.fw_destroy(h)


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    import paper_2606_11103_amd.native as nat
    monkeypatch.setattr(nat, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        nat._load()
    importlib.reload(nat)


def test_binding_shares_the_hip_runtime_torch_loads():
    """Importing the binding before torch still loads a single HIP runtime
    (torch's): a second one beside it would not know torch's device memory
    and would report no device from the library's calls."""
    import subprocess
    import sys
    code = ("import paper_2606_11103_amd.native\n"
            "libs = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})\n"
            "print(len(libs), libs)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[0] == "1", out.stdout


def test_time_space_stencil_host_setup():
    """fw_set_time_space_stencil computes the time-space set on the host: the
    same coefficients as the oracle's exact rational solution, the Taylor set
    back with c_ref = 0, and documented errors for invalid speeds."""
    from oracle import fdcoef
    from paper_2606_11103_amd import native
    lib = native.lib
    dx, dt = 1e-4, 2e-8
    rc, h = _create(dx=dx, dt=dt)
    assert rc == 0
    buf = np.zeros(5)
    out = buf[:4]
    p = ctypes.c_void_p(buf.ctypes.data)
    assert lib.fw_get_stencil(h, p) == 0
    assert np.array_equal(out, np.array(fdcoef.staggered_coefficients(4))) and buf[4] == 0.0
    for c_ref in (800.0, 1540.0, 3000.0, 4900.0):
        assert lib.fw_set_time_space_stencil(h, c_ref) == 0
        assert lib.fw_get_stencil(h, p) == 0
        ref = np.array(fdcoef.time_space_coefficients(c_ref * dt / dx, 4))
        assert np.max(np.abs(out - ref) / np.abs(ref)) < 1e-13, (c_ref, out, ref)
    assert lib.fw_set_time_space_stencil(h, -1.0) == native.FW_EINVAL
    assert lib.fw_set_time_space_stencil(h, float("nan")) == native.FW_EINVAL
    assert lib.fw_set_time_space_stencil(h, dx / dt) == native.FW_EINVAL      # r = 1
    assert lib.fw_get_stencil(h, p) == 0                                       # unchanged by the failures
    assert np.max(np.abs(out - ref) / np.abs(ref)) < 1e-13
    assert lib.fw_set_time_space_stencil(h, 0.0) == 0
    assert lib.fw_get_stencil(h, p) == 0
    assert np.array_equal(out, np.array(fdcoef.staggered_coefficients(4)))
    assert lib.fw_set_time_space_stencil(None, 1500.0) == native.FW_EINVAL
    assert lib.fw_destroy(h) == 0


def test_widened_stencil_host_setup():
    """fw_set_widened_stencil: 2D only; c_1..c_4 and b equal the oracle's exact
    rationals; fw_set_time_space_stencil and c_ref = 0 clear b."""
    from oracle import fdcoef
    from paper_2606_11103_amd import native
    lib = native.lib
    dx, dt = 1e-4, 2e-8
    buf = np.zeros(5)
    p = ctypes.c_void_p(buf.ctypes.data)
    rc, h3 = _create(ndim=3, shapes=((40, 36, 30),), dx=dx, dt=dt)
    assert rc == 0
    assert lib.fw_set_widened_stencil(h3, 1500.0) == native.FW_EUNSUPPORTED
    assert lib.fw_destroy(h3) == 0
    rc, h = _create(dx=dx, dt=dt)
    assert rc == 0
    for c_ref in (900.0, 1540.0, 3500.0):
        assert lib.fw_set_widened_stencil(h, c_ref) == 0
        assert lib.fw_get_stencil(h, p) == 0
        c, b = fdcoef.isotropic_time_space_coefficients(c_ref * dt / dx, 2, 4)
        assert np.max(np.abs(buf[:4] - c) / np.abs(c)) < 1e-13
        assert abs(buf[4] - b) <= 1e-15 * b
    assert lib.fw_set_widened_stencil(h, -5.0) == native.FW_EINVAL
    assert lib.fw_set_widened_stencil(h, dx / dt) == native.FW_EINVAL
    assert lib.fw_set_time_space_stencil(h, 1540.0) == 0
    assert lib.fw_get_stencil(h, p) == 0
    assert buf[4] == 0.0
    assert lib.fw_set_widened_stencil(h, 1540.0) == 0
    assert lib.fw_set_widened_stencil(h, 0.0) == 0
    assert lib.fw_get_stencil(h, p) == 0
    assert np.array_equal(buf[:4], np.array(fdcoef.staggered_coefficients(4))) and buf[4] == 0.0
    assert lib.fw_destroy(h) == 0
