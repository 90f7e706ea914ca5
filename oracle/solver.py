"""FP64 oracle solver: per-voxel set-up in numpy, literal stepping in C.

Test infrastructure (the oracle): only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import anything under
``oracle/``.  It shares no code with the product library.

Set-up follows the paper and the readings recorded with the project docs:

* Sec. 2.1, Eqs. (relaxation_a)/(relaxation_b): each class row (kappa_i,
  d_i^nu, alpha_i^nu) becomes per-voxel FP64 arrays a, b with
  b = exp(-(d/kappa + alpha) dt) and a = d/(kappa (d + kappa alpha)) (b - 1).
* Sec. 2.1, Eq. (wave2): K = 1/kappa = rho c^2.  An optional per-voxel speed
  perturbation c (1 + eps) uses SplitMix64 (Steele, Lea & Flood 2014) of
  seed XOR the domain-local linear index: eps = amp (2u - 1),
  u = (SplitMix64 >> 40) * 2^-24.
* Nonlinearity (named in Sec. 1): bulk modulus K + 2 beta p, beta = 1 + B/(2A).
* CPML (Sec. 2.1 says the boundary uses the same relaxation form): one extra
  memory variable per axis with kappa = 1, d(delta) = d0 delta^2,
  alpha(delta) = pi f_alpha (1 - delta), d0 = 3 c_ref ln(1/R0) / (2 P dx),
  delta = depth into a P-cell slab, measured from the slab's inner edge at
  positions P - 1/2 and n - P - 1/2 (cells at integers, faces at half-integers).
"""
import ctypes
import os

import numpy as np

from . import fdcoef
from .analytic import recursion_coefficients

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_libs = {}


def build(force=False):
    """Compile the C stepping engine with gcc (-O2, no FP contraction)."""
    import subprocess
    src = os.path.join(_HERE, "fdtd_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-std=c11", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load(path=None):
    """The compiled stepping engine: the library built from fdtd_oracle.c, or
    another build of that source named by path (tests that plant a mistake
    in a copy of the engine load it this way) or by the environment variable
    ORACLE_ENGINE (the sanitizer test runs the oracle pins on an
    instrumented build this way)."""
    path = path or os.environ.get("ORACLE_ENGINE") or None
    key = path or LIB_PATH
    lib = _libs.get(key)
    if lib is None:
        if path is None:
            build()
        lib = ctypes.CDLL(key)
        lib.oracle_steps.restype = ctypes.c_int
        lib.oracle_adjoint_step.restype = ctypes.c_int
        _libs[key] = lib
    return lib


class _Sim(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nmech", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("fd", ctypes.c_double * 4), ("fd_b", ctypes.c_double)] + \
               [(nm, ctypes.c_void_p) for nm in ("rho", "K", "beta", "ik1", "ik2",
                                                  "a1", "b1", "a2", "b2",
                                                  "pml_aF", "pml_bF", "pml_aC", "pml_bC")] + \
               [("nmax", ctypes.c_int64)] + \
               [(nm, ctypes.c_void_p) for nm in ("p", "v", "psi1", "psi2", "psiP1", "psiP2")]


def splitmix64(x):
    """SplitMix64 output for state x (uint64 numpy array), published constants."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def speed_noise(ncell, amp, seed):
    """eps[i] = amp * (2u - 1), u = (SplitMix64(seed ^ i) >> 40) * 2^-24."""
    idx = np.arange(ncell, dtype=np.uint64)
    u = (splitmix64(idx ^ np.uint64(seed)) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    return amp * (2.0 * u - 1.0)


def crop_noise(index, amp, seed):
    """speed_noise at arbitrary (full-domain) linear indices."""
    idx = np.asarray(index, dtype=np.uint64)
    u = (splitmix64(idx ^ np.uint64(seed)) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    return amp * (2.0 * u - 1.0)


def pml_profile(n, P, dx, dt, R0, f_alpha, c_ref, staggered):
    """CPML recursion coefficients (a, b) along one axis of n points.
    staggered=True gives the faces (positions i + 1/2), else the cells."""
    a = np.zeros(n)
    b = np.zeros(n)
    if P <= 0:
        return a, b
    x = np.arange(n, dtype=np.float64) + (0.5 if staggered else 0.0)
    delta = np.maximum.reduce([(P - 0.5 - x) / P, (x - (n - P - 0.5)) / P, np.zeros(n)])
    delta = np.minimum(delta, 1.0)
    d0 = 3.0 * c_ref * np.log(1.0 / R0) / (2.0 * P * dx)
    d = d0 * delta ** 2
    al = np.pi * f_alpha * (1.0 - delta)
    b = np.exp(-(d + al) * dt)
    with np.errstate(invalid="ignore", divide="ignore"):
        a = np.where(d > 0, d / (d + al) * (b - 1.0), 0.0)
    return a, b


def recursion_scale_derivatives(kappa, d, alpha, dt):
    """d a / d s and d b / d s at s = 1 when d is replaced by s d
    (kappa and alpha fixed), from differentiating Eqs. (relaxation_a/b)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    b = np.exp(-(d / kappa + alpha) * dt)
    b_s = -(d / kappa) * dt * b
    a_s = d * alpha / (d + kappa * alpha) ** 2 * (b - 1.0) + d / (kappa * (d + kappa * alpha)) * b_s
    return a_s, b_s


def beta_from_b_over_a(b_over_a):
    """Coefficient of nonlinearity beta = 1 + B/(2A) of a fluid with
    parameter B/A."""
    return 1.0 + np.asarray(b_over_a, dtype=np.float64) / 2.0


class OracleSim:
    """One domain of the FP64 oracle.

    shape = (nx, ny, nz) with unused trailing dims 1; class_map is uint8 with
    shape (nz, ny, nx); per-class arrays c, rho, beta [C] (beta = 0 is the
    linear medium, see beta_from_b_over_a); kappa [C][2],
    d and alpha [C][2][N] (index 0 for the gradient operator, 1 for the
    divergence operator).  a_scale (per voxel, optional) multiplies both
    operators' recursion coefficients a of the voxel (its relaxation
    strength; b, the relaxation times, unchanged).  fd_c_ref (optional, a
    speed) selects the time-space-domain staggered coefficients for the
    Courant number fd_c_ref dt / dx instead of the Taylor ones; with
    off_axis (2D/3D) the widened stencil of fdcoef.isotropic_time_space_coefficients.
    """

    def __init__(self, ndim, shape, dx, dt, nmech, class_map, c, rho, beta,
                 kappa, d, alpha, pml_cells=0, pml_R0=1e-4, pml_f_alpha=1e6, pml_c_ref=None,
                 noise_amp=0.0, noise_seed=0, d_scale=None, noise_index=None, axis_full=None,
                 engine=None, a_scale=None, fd_c_ref=None, off_axis=False):
        self.engine = engine
        self.ndim = int(ndim)
        nx, ny, nz = (list(shape) + [1, 1, 1])[:3]
        self.shape = (int(nx), int(ny), int(nz))
        self.nc = nx * ny * nz
        self.dx, self.dt, self.N = float(dx), float(dt), int(nmech)
        cls = np.asarray(class_map, dtype=np.int64).reshape(-1)
        assert cls.size == self.nc
        c = np.asarray(c, dtype=np.float64)
        rho = np.asarray(rho, dtype=np.float64)
        beta = np.asarray(beta, dtype=np.float64)
        kappa = np.asarray(kappa, dtype=np.float64).reshape(-1, 2)
        d = np.asarray(d, dtype=np.float64).reshape(-1, 2, self.N)
        alpha = np.asarray(alpha, dtype=np.float64).reshape(-1, 2, self.N)
        # a crop of a larger domain: noise keyed by the full-domain linear
        # index, CPML profiles of the full axes restricted to the crop
        if noise_amp and noise_index is not None:
            eps = crop_noise(np.asarray(noise_index).reshape(-1), noise_amp, noise_seed)
        else:
            eps = speed_noise(self.nc, noise_amp, noise_seed) if noise_amp else np.zeros(self.nc)
        cv = c[cls] * (1.0 + eps)
        self.rho = np.ascontiguousarray(rho[cls])
        self.c_voxel = cv
        self.K = np.ascontiguousarray(self.rho * cv * cv)
        self.beta = np.ascontiguousarray(beta[cls])
        self.ik1 = np.ascontiguousarray(1.0 / kappa[cls, 0])
        self.ik2 = np.ascontiguousarray(1.0 / kappa[cls, 1])
        # per-voxel d scale s(x) (1 = the class table); used by the adjoint checks
        s = np.ones(self.nc) if d_scale is None else np.asarray(d_scale, dtype=np.float64).reshape(-1)
        self.coef = {}
        for i, nm in ((0, "1"), (1, "2")):
            kv = kappa[cls, i][None, :]
            dv = d[cls, i, :].T * s[None, :]
            av = alpha[cls, i, :].T
            a_, b_ = recursion_coefficients(kv, dv, av, self.dt)
            if a_scale is not None:
                # per-voxel relaxation strength: both operators' coefficients a
                # of the voxel scaled by s(x), the relaxation times (b) kept
                a_ = a_ * np.asarray(a_scale, dtype=np.float64).reshape(1, -1)
            # derivative with respect to s of a(s d), b(s d): (1/s) * [d da/dd]
            as_, bs_ = recursion_scale_derivatives(kv, dv, av, self.dt)
            self.coef["a" + nm] = np.ascontiguousarray(a_)
            self.coef["b" + nm] = np.ascontiguousarray(b_)
            self.coef["as" + nm] = np.ascontiguousarray(as_ / s[None, :])
            self.coef["bs" + nm] = np.ascontiguousarray(bs_ / s[None, :])
        # staggered coefficients: the Taylor set, or the time-space set for
        # the Courant number of the speed fd_c_ref (fdcoef)
        # off_axis: the widened stencil of fdcoef.isotropic_time_space_coefficients
        # (fourth order in time in every direction of a 2D/3D grid)
        self.fd_b = 0.0
        if fd_c_ref and off_axis and self.ndim > 1:
            self.fd, self.fd_b = fdcoef.isotropic_time_space_coefficients(
                float(fd_c_ref) * self.dt / self.dx, self.ndim, 4)
        elif fd_c_ref:
            self.fd = fdcoef.time_space_coefficients(float(fd_c_ref) * self.dt / self.dx, 4)
        else:
            self.fd = fdcoef.staggered_coefficients(4)
        cref = float(np.max(c)) if pml_c_ref is None else float(pml_c_ref)
        self.nmax = max(self.shape)
        pm = {k: np.zeros((3, self.nmax)) for k in ("aF", "bF", "aC", "bC")}
        for a in range(self.ndim):
            n_a = self.shape[a]
            n_full, o = (n_a, 0) if axis_full is None else axis_full[a]
            aF, bF = pml_profile(n_full, pml_cells, dx, dt, pml_R0, pml_f_alpha, cref, True)
            aC, bC = pml_profile(n_full, pml_cells, dx, dt, pml_R0, pml_f_alpha, cref, False)
            pm["aF"][a, :n_a], pm["bF"][a, :n_a] = aF[o:o + n_a], bF[o:o + n_a]
            pm["aC"][a, :n_a], pm["bC"][a, :n_a] = aC[o:o + n_a], bC[o:o + n_a]
        self.pml = {k: np.ascontiguousarray(v) for k, v in pm.items()}
        self.reset()

    # ------------------------------------------------------------ state --
    def reset(self):
        nc, N = self.nc, self.N
        self.p = np.zeros(nc)
        self.v = np.zeros((3, nc))
        self.psi1 = np.zeros((3, N, nc))
        self.psi2 = np.zeros((3, N, nc))
        self.psiP1 = np.zeros((3, nc))
        self.psiP2 = np.zeros((3, nc))
        self.step = 0

    STATE_FIELDS = ("p", "v", "psi1", "psi2", "psiP1", "psiP2")

    def get_state(self):
        st = {k: getattr(self, k).copy() for k in self.STATE_FIELDS}
        st["step"] = self.step
        return st

    def set_state(self, st):
        for k in self.STATE_FIELDS:
            getattr(self, k)[...] = st[k]
        self.step = st["step"]

    def _struct(self):
        st = _Sim()
        st.ndim, st.nmech = self.ndim, self.N
        st.n[0], st.n[1], st.n[2] = self.shape
        st.dx, st.dt = self.dx, self.dt
        for i in range(4):
            st.fd[i] = self.fd[i]
        st.fd_b = self.fd_b
        ptr = lambda arr: arr.ctypes.data
        st.rho, st.K, st.beta = ptr(self.rho), ptr(self.K), ptr(self.beta)
        st.ik1, st.ik2 = ptr(self.ik1), ptr(self.ik2)
        st.a1, st.b1 = ptr(self.coef["a1"]), ptr(self.coef["b1"])
        st.a2, st.b2 = ptr(self.coef["a2"]), ptr(self.coef["b2"])
        st.pml_aF, st.pml_bF = ptr(self.pml["aF"]), ptr(self.pml["bF"])
        st.pml_aC, st.pml_bC = ptr(self.pml["aC"]), ptr(self.pml["bC"])
        st.nmax = self.nmax
        st.p, st.v, st.psi1, st.psi2 = ptr(self.p), ptr(self.v), ptr(self.psi1), ptr(self.psi2)
        st.psiP1, st.psiP2 = ptr(self.psiP1), ptr(self.psiP2)
        return st

    # ---------------------------------------------------------- stepping --
    def run(self, n_steps, src_cell=(), src_wave=None, rec_cell=(), energy=False):
        """Advance n_steps.  src_wave is [n_src][n_t] (sample t is added at the
        end of global step t).  Returns (receivers [n_steps][n_rec], energy or None)."""
        lib = _load(self.engine)
        src_cell = np.ascontiguousarray(np.asarray(src_cell, dtype=np.int64).reshape(-1))
        rec_cell = np.ascontiguousarray(np.asarray(rec_cell, dtype=np.int64).reshape(-1))
        n_src = src_cell.size
        if n_src:
            wave = np.ascontiguousarray(np.asarray(src_wave, dtype=np.float64).reshape(n_src, -1))
            n_t = wave.shape[1]
        else:
            wave = np.zeros((0, 1))
            n_t = 0
        rec = np.zeros((n_steps, rec_cell.size))
        en = np.zeros(n_steps) if energy else None
        st = self._struct()
        rc = lib.oracle_steps(ctypes.byref(st), ctypes.c_int(n_steps), ctypes.c_int(self.step),
                              ctypes.c_int64(n_src), ctypes.c_void_p(src_cell.ctypes.data),
                              ctypes.c_void_p(wave.ctypes.data), ctypes.c_int(n_t),
                              ctypes.c_int64(rec_cell.size), ctypes.c_void_p(rec_cell.ctypes.data),
                              ctypes.c_void_p(rec.ctypes.data),
                              ctypes.c_void_p(en.ctypes.data if en is not None else None))
        self.step += n_steps
        self.last_status = rc
        return rec, en

    def adjoint_step(self, lam, gK, gs):
        """Apply the transposed step to lam (dict of adjoint arrays shaped like
        the state), using the forward state currently held (u^n)."""
        lib = _load(self.engine)
        st = self._struct()
        c = self.coef
        rc = lib.oracle_adjoint_step(ctypes.byref(st),
                                     *[ctypes.c_void_p(lam[k].ctypes.data) for k in
                                       ("p", "v", "psi1", "psiP1", "psi2", "psiP2")],
                                     *[ctypes.c_void_p(c[k].ctypes.data) for k in ("as1", "bs1", "as2", "bs2")],
                                     ctypes.c_void_p(gK.ctypes.data), ctypes.c_void_p(gs.ctypes.data))
        assert rc == 0


def misfit_gradient(sim, n_steps, src_cell, src_wave, rec_cell, observed):
    """FP64 discrete adjoint of the whole run (beta = 0), literal.

    J = 1/2 sum_n dt sum_r (rec[n][r] - observed[n][r])^2, rec[n] = p^{n+1}
    at rec_cell.  Every forward state is stored (no checkpointing).  Returns
    (J, gK, gs, rec) where gK = dJ/dK per voxel and gs = dJ/ds per voxel for
    the scale s of every d coefficient owned by the voxel (d -> s d)."""
    sim.reset()
    states = []
    recs = []
    for n in range(n_steps):
        states.append(sim.get_state())
        r, _ = sim.run(1, src_cell, src_wave, rec_cell)
        recs.append(r[0])
    rec = np.array(recs)
    res = rec - np.asarray(observed, dtype=np.float64)
    J = 0.5 * sim.dt * float(np.sum(res * res))
    lam = {k: np.zeros_like(getattr(sim, k)) for k in sim.STATE_FIELDS}
    gK = np.zeros(sim.nc)
    gs = np.zeros(sim.nc)
    rc = np.asarray(rec_cell, dtype=np.int64).reshape(-1)
    for n in range(n_steps - 1, -1, -1):
        np.add.at(lam["p"], rc, sim.dt * res[n])
        sim.set_state(states[n])
        sim.adjoint_step(lam, gK, gs)
    sim.set_state(states[0])
    return J, gK, gs, rec
