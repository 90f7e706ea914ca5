"""Relaxation-parameter calibration (host, FP64): the paper's Sec. 3.

For one tissue class (c, alpha0, y) and N mechanisms this fits the 2 + 4N
parameters (kappa_1, kappa_2, d_i^nu, alpha_i^nu; Sec. 2.1) so that the
model wavenumber of Eq. (dispersion_relations) matches the power law of
Eq. (power_law_attenuation) and the Kramers-Kronig phase velocity of
Eq. (kk_relation):

* objective J = mean |k'_GT - k'_pred|^2 over log-spaced frequencies in the
  band (Sec. 3.2), each wavenumber normalised by the ranges of the real and
  imaginary parts of k_GT and weighted by (1 - w) and w;
* adaptive Nelder-Mead (SciPy ``minimize``), maximum 5e4 iterations,
  absolute tolerances 1e-25 (Sec. 3.2);
* variables and bounds of Table 2: kappa in [0.98, 1] (linear, start 1),
  d in [1e2, 1e10] and alpha in [1e5, 1e12] optimised as log10 (start 1e6
  and 1e9), which keeps d >= 0 and alpha > 0;
* w swept over {0.1, 0.3, 0.5, 0.7, 0.9}; the winner has the lowest
  attenuation NRMSE (Sec. 4.1 definition) at the eight measurement
  frequencies 1 + 2.714 k MHz among the candidates that pass both bars of the
  failure label (10 % NRMSE, 5 m/s dispersion error, Sec. 3.2), else among
  all; ties broken by the dispersion error.

Conventions: e^{+iwt} time dependence, so attenuation is -Im k_pred and the
comparison uses conj(k_pred); alpha0 in dB/(MHz^y cm) converted with
20 log10(e) dB per neper; phase velocity referenced to c at f_ref = 1 MHz.
"""
import json
import math
import os

import numpy as np

NEPER_DB = 20.0 / math.log(10.0)
WEIGHTS = (0.1, 0.3, 0.5, 0.7, 0.9)
FAIL_NRMSE = 0.10                # failure label of Sec. 3.2: attenuation NRMSE
FAIL_DISP = 5.0                  # and dispersion error (m/s)
MEASURE_FREQS = 1e6 + 2.714e6 * np.arange(8)


def _alpha_np(f_hz, alpha0_db, y):
    return alpha0_db * 100.0 / NEPER_DB * (np.asarray(f_hz) / 1e6) ** y


def target_wavenumber(f_hz, c0, alpha0_db, y, f_ref=1e6):
    """k_GT = w / c(w) + i alpha(w) with the Kramers-Kronig c(w)."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    w0 = 2.0 * np.pi * f_ref
    a0 = alpha0_db * 100.0 / NEPER_DB / (2.0 * np.pi * 1e6) ** y
    if abs(y - 1.0) < 1e-12:
        inv_c = 1.0 / c0 - 2.0 / np.pi * a0 * np.log(w / w0)
    else:
        inv_c = 1.0 / c0 + a0 * math.tan(math.pi * y / 2.0) * (w ** (y - 1.0) - w0 ** (y - 1.0))
    return w * inv_c + 1j * a0 * w ** y


def model_wavenumber(f_hz, c, kappa, d, alpha):
    """k_pred of Eq. (dispersion_relations); kappa [2], d and alpha [2][N]."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    S = []
    for i in range(2):
        g = np.zeros_like(w, dtype=np.complex128)
        for dn, an in zip(d[i], alpha[i]):
            g += dn / kappa[i] ** 2 / (dn / kappa[i] + an + 1j * w)
        S.append(1.0 / kappa[i] - g)
    return w / c / np.sqrt(S[0] * S[1])


def step_matched(kappa, d, alpha, dt):
    """Mechanisms for a run at time step dt with the relaxation response of
    the fitted (continuous) ones.

    The recursion of Eq. (relaxation_psi) with b = exp(-R dt),
    R = d/kappa + alpha, behaves at frequencies w dt << 1 like a relaxation
    with the same DC gain a / (1 - b) = -d / (kappa (d + kappa alpha)) but the
    rate (e^{R dt} - 1) / dt instead of R.  A fitted mechanism of rate
    r = d/kappa + alpha and strength g = (d/kappa) / r therefore becomes
    R = ln(1 + r dt) / dt, d' = kappa g R, alpha' = (1 - g) R: kappa, every
    DC gain and every low-frequency pole are kept, and b = 1 / (1 + r dt)
    (a backward-Euler step of the relaxation equation).  Rates far below
    1/dt are left almost unchanged; rates at or above it -- which a fit of the
    continuous model uses freely, and which the recursion would otherwise
    turn into a frequency-independent term with no attenuation -- are
    pulled below it.  kappa [..][2], d and alpha [..][2][N]."""
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    k = kappa[..., None]
    r = d / k + alpha
    g = (d / k) / r
    R = np.log1p(r * dt) / dt
    return kappa.copy(), k * g * R, (1.0 - g) * R


def _unpack(x, N):
    kappa = np.array([x[0], x[1]])
    d = 10.0 ** np.asarray(x[2:2 + 2 * N]).reshape(2, N)
    al = 10.0 ** np.asarray(x[2 + 2 * N:2 + 4 * N]).reshape(2, N)
    return kappa, d, al


def _objective_factory(f, kgt, w, c, N):
    rr = np.ptp(kgt.real)
    ri = np.ptp(kgt.imag)
    gt = (1.0 - w) * kgt.real / rr + 1j * w * kgt.imag / ri

    def J(x):
        kappa, d, al = _unpack(x, N)
        kp = np.conj(model_wavenumber(f, c, kappa, d, al))
        pr = (1.0 - w) * kp.real / rr + 1j * w * kp.imag / ri
        val = np.mean(np.abs(gt - pr) ** 2)
        return val if np.isfinite(val) else 1e30
    return J


def model_errors(c, alpha0_db, y, kappa, d, alpha, f_ref=1e6):
    """(attenuation NRMSE, dispersion RMSE in m/s) of the closed-form model at
    the eight measurement frequencies."""
    f = MEASURE_FREQS
    kp = model_wavenumber(f, c, kappa, d, alpha)
    kt = target_wavenumber(f, c, alpha0_db, y, f_ref)
    at = kt.imag
    am = -kp.imag
    nr = math.sqrt(np.mean((am - at) ** 2)) / (at.max() - at.min())
    w = 2.0 * np.pi * f
    disp = math.sqrt(np.mean((w / kp.real - w / kt.real) ** 2))
    return nr, disp


def passes(nrmse, disp):
    """Both bars of the failure label."""
    return nrmse <= FAIL_NRMSE and disp <= FAIL_DISP


def choose(cands, nrmse=None, disp=None):
    """The weight's candidate to keep: the lowest attenuation NRMSE among the
    candidates that pass both bars, else the lowest NRMSE of all; ties to the
    lower dispersion error, then the smaller w.  nrmse / disp override the
    candidates' own (closed-form) figures, e.g. with simulated ones.
    Returns the index into cands."""
    nr = [cd["nrmse"] for cd in cands] if nrmse is None else list(nrmse)
    dp = [cd["disp"] for cd in cands] if disp is None else list(disp)
    return min(range(len(cands)), key=lambda j: (not passes(nr[j], dp[j]), nr[j], dp[j], cands[j]["w"]))


def effective(fit):
    """A cached fit with its kept candidate chosen by choose() (fits stored
    before candidates were kept are returned as they are)."""
    if "cands" not in fit:
        return fit
    out = dict(fit)
    out.update(fit["cands"][choose(fit["cands"])])
    out["failed"] = not passes(out["nrmse"], out["disp"])
    return out


def fit_class(c, alpha0_db, y, nmech=2, weights=WEIGHTS, n_freq=64, band=(1e6, 20e6),
              f_ref=1e6, maxiter=50000, tol=1e-25):
    """Fit one class; returns a dict with kappa [2], d [2][N], alpha [2][N],
    the chosen weight and the model errors, plus every weight's candidate
    under "cands" (for selection by simulated attenuation)."""
    from scipy.optimize import minimize
    N = int(nmech)
    f = np.logspace(math.log10(band[0]), math.log10(band[1]), n_freq)
    kgt = target_wavenumber(f, c, alpha0_db, y, f_ref)
    x0 = np.array([1.0, 1.0] + [6.0] * (2 * N) + [9.0] * (2 * N))
    bounds = [(0.98, 1.0)] * 2 + [(2.0, 10.0)] * (2 * N) + [(5.0, 12.0)] * (2 * N)
    cands = []
    for w in weights:
        J = _objective_factory(f, kgt, w, c, N)
        res = minimize(J, x0, method="Nelder-Mead", bounds=bounds,
                       options=dict(adaptive=True, maxiter=int(maxiter), maxfev=int(maxiter) * 4,
                                    xatol=tol, fatol=tol))
        kappa, d, al = _unpack(res.x, N)
        nr, disp = model_errors(c, alpha0_db, y, kappa, d, al, f_ref)
        cand = dict(kappa=kappa.tolist(), d=d.tolist(), alpha=al.tolist(), w=w, J=float(res.fun),
                    nrmse=nr, disp=disp)
        cands.append(cand)
    best = dict(cands[choose(cands)])
    best.update(c=float(c), alpha0=float(alpha0_db), y=float(y), nmech=N,
                failed=not passes(best["nrmse"], best["disp"]), cands=cands)
    return best


# ------------------------------------------------------------ table cache --
CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "relax_tables.json")


def _key(c, alpha0_db, y, nmech, maxiter):
    return "c=%.6f|a0=%.8g|y=%.6f|N=%d|it=%d" % (c, alpha0_db, y, nmech, maxiter)


def _fit_job(args):
    c, a0, y, N, maxiter = args
    return _key(c, a0, y, N, maxiter), fit_class(c, a0, y, N, maxiter=maxiter)


def load_cache(path=CACHE_PATH):
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def tables_for(classes, nmech, maxiter=50000, allow_fit=True, processes=None, path=CACHE_PATH, dt=None):
    """Return (kappa [C][2], d [C][2][N], alpha [C][2][N], fits) for classes =
    dict(c=[...], alpha0=[...], y=[...]).  Rows come from the cache when
    present; otherwise they are fitted (in parallel) and the cache is updated.
    With dt the tables are step_matched to that time step (the fits
    themselves, in `fits`, stay those of the continuous model)."""
    cache = load_cache(path)
    items = list(zip(classes["c"], classes["alpha0"], classes["y"]))
    keys = [_key(c, a0, y, nmech, maxiter) for c, a0, y in items]
    todo = sorted({k: (c, a0, y, nmech, maxiter) for k, (c, a0, y) in zip(keys, items) if k not in cache}.items())
    if todo:
        if not allow_fit:
            raise KeyError("relaxation tables missing from cache: %d classes" % len(todo))
        jobs = [v for _, v in todo]
        nproc = processes or min(8, os.cpu_count() or 1)
        # fit in chunks and write the cache after each, so that an interrupted
        # run keeps what it has finished
        chunk = max(1, 4 * nproc)
        for start in range(0, len(jobs), chunk):
            part = jobs[start:start + chunk]
            if len(part) > 1:
                import multiprocessing as mp
                with mp.get_context("fork").Pool(min(nproc, len(part))) as pool:
                    out = pool.map(_fit_job, part)
            else:
                out = [_fit_job(part[0])]
            cache = load_cache(path)
            cache.update(dict(out))
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=0, sort_keys=True)
            os.replace(tmp, path)
    fits = [effective(cache[k]) for k in keys]
    kappa = np.array([f["kappa"] for f in fits], dtype=np.float64)
    d = np.array([f["d"] for f in fits], dtype=np.float64)
    al = np.array([f["alpha"] for f in fits], dtype=np.float64)
    if dt is not None:
        kappa, d, al = step_matched(kappa, d, al, dt)
    return kappa, d, al, fits
