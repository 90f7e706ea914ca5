"""Fill the relaxation-table cache (data/relax_tables.json) for the named
workloads by running the FP64 calibration (relax.fit_class) on every class
that is not cached yet.  Usage: python -m paper_2606_11103_amd.relax_cache
[--adjoint] [--sweep] [--sweep4] [--library] [--tissues] [--pml-reference]
[--procs=N]"""
import sys
import time

from . import relax


def main():
    sys.path.insert(0, __file__.rsplit("/paper_2606_11103_amd/", 1)[0])
    from workloads import configs
    jobs = [
        ("2d_homogeneous", configs.homogeneous_2d(64, 10), 2),
        ("2d_two_layer", configs.two_layer_2d(64, 10, n_rec=2), 4),
        ("3d_heterogeneous", configs.heterogeneous_3d(shape=(64, 64, 64), steps=10, n_elem=4), 4),
        ("3d_heterogeneous_N2", configs.heterogeneous_3d(shape=(64, 64, 64), steps=10, n_elem=4, nmech=2), 2),
    ]
    if "--adjoint" in sys.argv:
        jobs = [("2d_adjoint", configs.adjoint_2d(n=64, n_shots=1, steps=10, n_rec=4, pml=8), 4)]
    if "--sweep" in sys.argv:
        jobs.append(("1d_sweep", configs.sweep_1d(n_cells=64, steps=10, pml=8), 2))
    if "--sweep4" in sys.argv:
        jobs.append(("1d_sweep_N4", configs.sweep_1d(n_cells=64, steps=10, pml=8, nmech=4), 4))
    if "--tissues" in sys.argv:
        class _Tissues:      # muscle, fat, liver of the two-layer validation (Sec. 4)
            c, alpha0, y = [1540.0] * 3, [0.15, 0.40, 0.50], [1.0, 1.1, 1.1]
        jobs = [("tissue_layers", _Tissues, 2)]
    if "--pml-reference" in sys.argv:
        class _Ref:          # the fixed tissue of the homogeneous absorbing layers (Sec. 4.6)
            c, alpha0, y = [1540.0], [0.5], [1.0]
        jobs = [("pml_reference", _Ref, 2), ("pml_reference", _Ref, 4)]
    if "--library" in sys.argv:
        lib = configs.library_classes()

        class _Lib:
            c, alpha0, y = lib["c"], lib["alpha0"], lib["y"]
        jobs.append(("library", _Lib, 2))
    for name, case, N in jobs:
        t = time.time()
        _, _, _, fits = relax.tables_for(dict(c=case.c, alpha0=case.alpha0, y=case.y), N, processes=int(next((a.split('=')[1] for a in sys.argv if a.startswith('--procs=')), 6)))
        print("%-18s N=%d classes=%d  %.1f s  model NRMSE %s" % (
            name, N, len(fits), time.time() - t, ["%.4f" % f["nrmse"] for f in fits]), flush=True)


if __name__ == "__main__":
    main()
