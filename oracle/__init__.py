"""FP64 CPU oracle for the attenuating nonlinear acoustic FDTD step.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package.  It shares no code with the product library
``paper_2606_11103_amd`` and never imports it.

Modules
-------
fdcoef    exact staggered finite-difference coefficients (Sec. 3.3)
analytic  closed forms: power law, Kramers-Kronig, k_pred, discrete
          dispersion of the scheme, measurement formulas (Secs. 2.2, 3.1, 4)
solver    per-voxel FP64 set-up + literal C stepping engine and its
          discrete adjoint (Secs. 2.1, 3.3)

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
