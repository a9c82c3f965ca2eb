"""Thin ctypes binding of the C ABI in include/fpt.h (argument marshalling only).

Every step of the method runs in the HIP kernels of libfpt.so; this module only
converts Python/numpy/torch arguments to the C structures and back.  It fails
loudly when the library has not been built: there is no fallback path.

torch is imported first so that the HIP runtime torch ships with is the one the
library binds to (both carry the soname libamdhip64.so.7); device buffers and
streams are torch's.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

try:  # torch supplies device memory and streams; import it before loading the library
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libfpt.so")
HEADER = os.path.join(ROOT, "include", "fpt.h")

FPT_OK, FPT_EINVAL, FPT_ENOMEM, FPT_EHIP, FPT_ESTATE, FPT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FPT_POT_PIECEWISE_LINEAR, FPT_POT_EXPONENTIAL, FPT_POT_GAUSSIAN_BUMP = 0, 1, 2
FPT_BIAS_NONE, FPT_BIAS_CONST, FPT_BIAS_MLP = 0, 1, 2
FPT_FP64, FPT_FP32_STATE = 0, 1
FPT_BINS_LINEAR, FPT_BINS_LOG = 0, 1
FPT_AXIS_PHI, FPT_AXIS_TIME = 0, 1
FPT_FLAG_CENSORED = 0x80000000
FPT_FLAG_ENDED_EARLY = 0x40000000
FPT_STEP_MASK = 0x3FFFFFFF
FPT_MAX_STEPS = 0x3FFFFFFF
FPT_MAX_TABLE = 4096
FPT_MAX_BINS = 1024
FPT_MLP_NPARAM = 4482
FPT_MLP_MAX_GRID = 1024
FPT_MLP_OBJ_J, FPT_MLP_OBJ_LOG_J = 0, 1
FPT_MLP_GRAD_NOALLOC_MAX = 1 << 18

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class fpt_potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("V0", ctypes.c_double), ("phi_T", ctypes.c_double),
                ("A_plus", ctypes.c_double), ("A_minus", ctypes.c_double), ("phi_in", ctypes.c_double),
                ("pi_in", ctypes.c_double), ("phi_end", ctypes.c_double), ("bump_m", ctypes.c_double),
                ("bump_K", ctypes.c_double), ("bump_Sigma", ctypes.c_double)]


class fpt_noise_table(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("phi_lo", ctypes.c_double), ("phi_hi", ctypes.c_double),
                ("S", _dp), ("tan_theta", _dp), ("dim", ctypes.c_int32), ("Xi_pp", _dp), ("Xi_pq", _dp),
                ("Xi_qq", _dp), ("axis", ctypes.c_int32)]


class fpt_bias(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("A", ctypes.c_double), ("mlp_params", _fp),
                ("norm", ctypes.c_double * 4), ("mlp_every", ctypes.c_int32), ("grid_n", ctypes.c_int32 * 2),
                ("grid_range", ctypes.c_double * 4)]


class fpt_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("bins_kind", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("N_ref", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("instance", ctypes.c_uint32), ("block_size", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("chunk", ctypes.c_int32)]


class fpt_hist(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_uint64), ("n_censored", ctypes.c_uint64), ("n_ended_early", ctypes.c_uint64),
                ("n_steps_total", ctypes.c_uint64), ("sum_w", ctypes.c_double), ("sum_w2", ctypes.c_double),
                ("sum_wN", ctypes.c_double), ("sum_wN2", ctypes.c_double), ("count", _u64p),
                ("sum_w_bin", _dp), ("sum_w2_bin", _dp), ("sum_lnw_bin", _dp), ("sum_lnw2_bin", _dp)]


class fpt_moments(ctypes.Structure):
    _fields_ = [("mean_w", ctypes.c_double), ("mean_N", ctypes.c_double), ("var_N", ctypes.c_double),
                ("ess", ctypes.c_double), ("mass_under", ctypes.c_double), ("mass_over", ctypes.c_double)]


class fpt_tail(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_int32), ("x_star", ctypes.c_double), ("P", ctypes.c_double),
                ("P_err", ctypes.c_double), ("P_err_lognormal", ctypes.c_double), ("ess", ctypes.c_double),
                ("count", ctypes.c_uint64)]


class fpt_batch_options(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("chunk", ctypes.c_int32), ("item_size", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class FptError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


_lib = None


def header_functions() -> list[str]:
    """Names of the functions include/fpt.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpt_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libfpt.so (raises if it is missing: the product has no CPU path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.fpt_create.argtypes = [P(fpt_potential), P(fpt_noise_table), P(fpt_bias), P(fpt_options),
                             P(ctypes.c_void_p)]
    L.fpt_run.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fpt_histogram.argtypes = [ctypes.c_void_p, P(fpt_hist)]
    L.fpt_reset.argtypes = [ctypes.c_void_p]
    L.fpt_destroy.argtypes = [ctypes.c_void_p]
    L.fpt_destroy.restype = None
    L.fpt_last_kernel_ms.argtypes = [ctypes.c_void_p, _dp]
    L.fpt_strerror.argtypes = [ctypes.c_int]
    L.fpt_strerror.restype = ctypes.c_char_p
    L.fpt_last_error.argtypes = []
    L.fpt_last_error.restype = ctypes.c_char_p
    L.fpt_noise_table_bessel.argtypes = [P(fpt_potential), ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, _dp, _dp]
    L.fpt_noise_table_bessel2d.argtypes = [P(fpt_potential), ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, _dp, _dp, _dp]
    L.fpt_noise_table_matched.argtypes = [P(fpt_potential), ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    L.fpt_noise_table_matched_time.argtypes = [P(fpt_potential), ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               _dp, _dp, _dp, _dp]
    L.fpt_noise_table_bessel2d_time.argtypes = [P(fpt_potential), ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                _dp, _dp, _dp, _dp]
    L.fpt_jackknife.argtypes = [ctypes.c_int32, ctypes.c_int32, _u64p, _dp, _dp, _dp]
    L.fpt_lognormal_bins.argtypes = [ctypes.c_int32, ctypes.c_uint64, _u64p, _dp, _dp, _dp, _dp, _dp]
    L.fpt_merge_bins.argtypes = [ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp, _dp]
    L.fpt_density.argtypes = [P(fpt_hist), ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp,
                              _dp, P(fpt_moments)]
    L.fpt_tail_at.argtypes = [P(fpt_hist), ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int32, P(fpt_tail)]
    L.fpt_tail_find.argtypes = [P(fpt_hist), ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, P(fpt_tail)]
    L.fpt_batch_create.argtypes = [P(ctypes.c_void_p), ctypes.c_int32, P(fpt_batch_options), P(ctypes.c_void_p)]
    L.fpt_batch_run.argtypes = [ctypes.c_void_p, _u64p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_void_p]
    L.fpt_batch_autotune.argtypes = [ctypes.c_void_p, _u64p, ctypes.c_double, ctypes.c_uint64, ctypes.c_char_p,
                                     ctypes.c_void_p]
    L.fpt_batch_config.argtypes = [ctypes.c_void_p, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.fpt_batch_last_ms.argtypes = [ctypes.c_void_p, _dp]
    L.fpt_batch_destroy.argtypes = [ctypes.c_void_p]
    L.fpt_batch_destroy.restype = None
    L.fpt_mlp_set.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fpt_mlp_get.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fpt_mlp_table.argtypes = [ctypes.c_void_p, _dp]
    L.fpt_mlp_grad.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _dp,
                               _u64p]
    L.fpt_mlp_grad_noalloc.argtypes = L.fpt_mlp_grad.argtypes
    L.fpt_mlp_adam.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_void_p]
    for name in ("fpt_create", "fpt_run", "fpt_histogram", "fpt_reset", "fpt_last_kernel_ms",
                 "fpt_noise_table_bessel", "fpt_noise_table_bessel2d", "fpt_noise_table_matched",
                 "fpt_noise_table_matched_time", "fpt_noise_table_bessel2d_time", "fpt_jackknife", "fpt_lognormal_bins",
                 "fpt_merge_bins", "fpt_density", "fpt_tail_at", "fpt_tail_find", "fpt_batch_create", "fpt_batch_run", "fpt_batch_autotune",
                 "fpt_batch_config", "fpt_batch_last_ms", "fpt_mlp_set", "fpt_mlp_get", "fpt_mlp_table",
                 "fpt_mlp_grad", "fpt_mlp_grad_noalloc", "fpt_mlp_adam"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != FPT_OK:
        L = load()
        raise FptError(rc, where, f"{L.fpt_strerror(rc).decode()}: {L.fpt_last_error().decode()}")


def _ptr(t):
    """Device pointer of a torch tensor (or None / an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_potential(kind, V0, phi_T, A_plus, A_minus, phi_in, pi_in, phi_end, bump=(0.0, 0.0, 0.0)) -> fpt_potential:
    """bump = (m, K, Sigma) of the Gaussian bump (its centre phi_0 is phi_T)."""
    return fpt_potential(kind, V0, phi_T, A_plus, A_minus, phi_in, pi_in, phi_end, *bump)


def fpt_noise_table_bessel(pot: fpt_potential, sigma: float, n: int, phi_lo: float, phi_hi: float):
    """Noise table of eq. (covariance_constant_nu) computed by the library's device kernel."""
    S = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    _check(load().fpt_noise_table_bessel(ctypes.byref(pot), sigma, n, phi_lo, phi_hi,
                                         S.ctypes.data_as(_dp), t.ctypes.data_as(_dp)), "fpt_noise_table_bessel")
    return S, t


def fpt_noise_table_bessel2d(pot: fpt_potential, sigma: float, n: int, phi_lo: float, phi_hi: float):
    """2D noise covariance (Xi_pp, Xi_pq, Xi_qq) of eq. (covariance_matrix_direct), device kernel."""
    X = [np.empty(n, dtype=np.float64) for _ in range(3)]
    _check(load().fpt_noise_table_bessel2d(ctypes.byref(pot), sigma, n, phi_lo, phi_hi, *[x.ctypes.data_as(_dp) for x in X]),
           "fpt_noise_table_bessel2d")
    return tuple(X)


def fpt_noise_table_matched(pot: fpt_potential, sigma: float, n: int, phi_lo: float, phi_hi: float,
                            phi_start: float, pi_start: float):
    """(S, tan_theta, 4|B_k|^2/pi) of the Bessel-matched table, eq. (covariance_constant_nu_bessel_matched),
    along the classical trajectory from (phi_start, pi_start); device kernels."""
    S = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    fac = np.empty(n, dtype=np.float64)
    _check(load().fpt_noise_table_matched(ctypes.byref(pot), sigma, n, phi_lo, phi_hi, phi_start, pi_start,
                                          S.ctypes.data_as(_dp), t.ctypes.data_as(_dp), fac.ctypes.data_as(_dp)),
           "fpt_noise_table_matched")
    return S, t, fac


def fpt_noise_table_matched_time(pot: fpt_potential, sigma: float, n: int, t_lo: float, t_hi: float,
                                 phi_start: float, pi_start: float, phi_ref: float):
    """(S, tan_theta, 4|B_k|^2/pi, phi_j) of the Bessel-matched table on time nodes t_lo + j h after the
    classical trajectory passes phi_ref; device kernels."""
    out = [np.empty(n, dtype=np.float64) for _ in range(4)]
    _check(load().fpt_noise_table_matched_time(ctypes.byref(pot), sigma, n, t_lo, t_hi, phi_start, pi_start, phi_ref,
                                               *[a.ctypes.data_as(_dp) for a in out]),
           "fpt_noise_table_matched_time")
    return tuple(out)


def fpt_noise_table_bessel2d_time(pot: fpt_potential, sigma: float, n: int, t_lo: float, t_hi: float,
                                  phi_start: float, pi_start: float, phi_ref: float):
    """(Xi_pp, Xi_pq, Xi_qq, phi_j) of the 2D covariance on time nodes t_lo + j h after the classical
    trajectory passes phi_ref; device kernels."""
    out = [np.empty(n, dtype=np.float64) for _ in range(4)]
    _check(load().fpt_noise_table_bessel2d_time(ctypes.byref(pot), sigma, n, t_lo, t_hi, phi_start, pi_start,
                                                phi_ref, *[a.ctypes.data_as(_dp) for a in out]),
           "fpt_noise_table_bessel2d_time")
    return tuple(out)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def fpt_jackknife(n_traj_blocks, sum_w_blocks):
    """(mass, error) per histogram slot from blocks of trajectories: delete-one jackknife."""
    n = np.ascontiguousarray(n_traj_blocks, dtype=np.uint64)
    sw = _f64(sum_w_blocks)
    B, ns = sw.shape
    p, e = np.empty(ns), np.empty(ns)
    _check(load().fpt_jackknife(ns, B, n.ctypes.data_as(_u64p), sw.ctypes.data_as(_dp), p.ctypes.data_as(_dp),
                                e.ctypes.data_as(_dp)), "fpt_jackknife")
    return p, e


def fpt_lognormal_bins(n_traj, count, sum_lnw, sum_lnw2):
    """(mass, lo, hi) per slot: the lognormal mean of the slot's weights and Cox's one-sigma interval."""
    c = np.ascontiguousarray(count, dtype=np.uint64)
    a, b = _f64(sum_lnw), _f64(sum_lnw2)
    ns = len(c)
    p, lo, hi = np.empty(ns), np.empty(ns), np.empty(ns)
    _check(load().fpt_lognormal_bins(ns, int(n_traj), c.ctypes.data_as(_u64p), a.ctypes.data_as(_dp),
                                     b.ctypes.data_as(_dp), p.ctypes.data_as(_dp), lo.ctypes.data_as(_dp),
                                     hi.ctypes.data_as(_dp)), "fpt_lognormal_bins")
    return p, lo, hi


def fpt_merge_bins(p_runs, err_runs):
    """Inverse-variance merge per slot over runs (rows)."""
    P, E = _f64(p_runs), _f64(err_runs)
    R, ns = P.shape
    p, e = np.empty(ns), np.empty(ns)
    _check(load().fpt_merge_bins(ns, R, P.ctypes.data_as(_dp), E.ctypes.data_as(_dp), p.ctypes.data_as(_dp),
                                 e.ctypes.data_as(_dp)), "fpt_merge_bins")
    return p, e


def _hist_struct(hist: dict):
    """An fpt_hist over the arrays of a histogram dict (as Context.histogram returns); the arrays
    are kept alive by the returned tuple."""
    arrs = [np.ascontiguousarray(hist["count"], dtype=np.uint64)] + [
        _f64(hist[k]) for k in ("sum_w", "sum_w2", "sum_lnw", "sum_lnw2")]
    h = fpt_hist(int(hist["n_traj"]), int(hist.get("n_censored", 0)), int(hist.get("n_ended_early", 0)),
                 int(hist.get("n_steps_total", 0)), float(hist.get("sum_w_total", 0.0)),
                 float(hist.get("sum_w2_total", 0.0)), float(hist.get("sum_wN", 0.0)),
                 float(hist.get("sum_wN2", 0.0)), arrs[0].ctypes.data_as(_u64p),
                 *[a.ctypes.data_as(_dp) for a in arrs[1:]])
    return h, arrs


def fpt_density(hist: dict, bins_kind: int, n_bins: int, lo: float, hi: float, moments: bool = True):
    """(density per bin, bin edges, whole-run figures or None) of a histogram dict."""
    h, keep = _hist_struct(hist)
    dens, edges = np.empty(n_bins), np.empty(n_bins + 1)
    m = fpt_moments()
    _check(load().fpt_density(ctypes.byref(h), bins_kind, n_bins, lo, hi, dens.ctypes.data_as(_dp),
                              edges.ctypes.data_as(_dp), ctypes.byref(m) if moments else None), "fpt_density")
    del keep
    mo = {f: getattr(m, f) for f, _ in fpt_moments._fields_} if moments else None
    return dens, edges, mo


def _tail_dict(t: fpt_tail) -> dict:
    return {f: getattr(t, f) for f, _ in fpt_tail._fields_}


def fpt_tail_at(hist: dict, bins_kind: int, n_bins: int, lo: float, hi: float, slot: int) -> dict:
    """The tail set of slots slot .. n_bins + 1: slot, x_star, P, P_err, ess, count."""
    h, keep = _hist_struct(hist)
    t = fpt_tail()
    _check(load().fpt_tail_at(ctypes.byref(h), bins_kind, n_bins, lo, hi, slot, ctypes.byref(t)), "fpt_tail_at")
    del keep
    return _tail_dict(t)


def fpt_tail_find(hist: dict, bins_kind: int, n_bins: int, lo: float, hi: float, p_target: float) -> dict:
    """The tail set whose probability is the largest at or below p_target (slot -1 if none)."""
    h, keep = _hist_struct(hist)
    t = fpt_tail()
    _check(load().fpt_tail_find(ctypes.byref(h), bins_kind, n_bins, lo, hi, p_target, ctypes.byref(t)),
           "fpt_tail_find")
    del keep
    return _tail_dict(t)


class Context:
    """Owns one fpt_ctx; mirrors fpt_run / fpt_histogram / fpt_reset / fpt_destroy.  S, tan_theta give a
    1D noise table; Xi = (Xi_pp, Xi_pq, Xi_qq) a 2D one (S and tan_theta are then ignored).  axis
    FPT_AXIS_TIME puts the nodes in time (phi_lo, phi_hi then hold N)."""

    def __init__(self, pot: fpt_potential, S, tan_theta, phi_lo: float, phi_hi: float, *, bias_kind=FPT_BIAS_NONE,
                 A=0.0, mlp_params=None, norm=(0.0, 1.0, 0.0, 1.0), mlp_every=0, grid_n=(2, 2),
                 grid_range=(-1.0, 1.0, -1.0, 1.0), precision=FPT_FP64,
                 bins_kind=FPT_BINS_LINEAR, n_bins=64, lo=-1.0, hi=1.0, N_ref=0.0, max_steps=FPT_MAX_STEPS,
                 instance=0, block_size=0, blocks_per_cu=0, chunk=0, Xi=None, axis=FPT_AXIS_PHI):
        L = load()
        if Xi is not None:
            self._X = [np.ascontiguousarray(x, dtype=np.float64) for x in Xi]
            n_tab = len(self._X[0])
            table = fpt_noise_table(n_tab, phi_lo, phi_hi, None, None, 2, *[x.ctypes.data_as(_dp) for x in self._X])
            table.axis = axis
        else:
            self._S = np.ascontiguousarray(S, dtype=np.float64)
            self._t = np.ascontiguousarray(tan_theta, dtype=np.float64)
            table = fpt_noise_table(len(self._S), phi_lo, phi_hi, self._S.ctypes.data_as(_dp),
                                    self._t.ctypes.data_as(_dp))
        table.axis = axis
        self._mlp = (np.ascontiguousarray(mlp_params, dtype=np.float32) if mlp_params is not None else None)
        bias = fpt_bias(bias_kind, A, self._mlp.ctypes.data_as(_fp) if self._mlp is not None else None,
                        (ctypes.c_double * 4)(*norm), mlp_every, (ctypes.c_int32 * 2)(*grid_n),
                        (ctypes.c_double * 4)(*grid_range))
        self.grid_n = (int(grid_n[0]), int(grid_n[1]))
        self.n_bins = int(n_bins)
        opts = fpt_options(precision, bins_kind, n_bins, lo, hi, N_ref, max_steps, instance, block_size,
                           blocks_per_cu, chunk)
        h = ctypes.c_void_p()
        _check(L.fpt_create(ctypes.byref(pot), ctypes.byref(table), ctypes.byref(bias), ctypes.byref(opts),
                            ctypes.byref(h)), "fpt_create")
        self._h = h
        self._lib = L

    @property
    def handle(self):
        return self._h

    def run(self, n_traj: int, dN: float, seed: int, traj_offset: int = 0, stream=None, d_N=None, d_lnw=None,
            d_steps=None):
        _check(self._lib.fpt_run(self._h, n_traj, dN, seed, traj_offset, _stream_handle(stream), _ptr(d_N),
                                 _ptr(d_lnw), _ptr(d_steps)), "fpt_run")

    def histogram(self) -> dict:
        nb = self.n_bins + 2
        arrs = {"count": np.zeros(nb, dtype=np.uint64), "sum_w": np.zeros(nb), "sum_w2": np.zeros(nb),
                "sum_lnw": np.zeros(nb), "sum_lnw2": np.zeros(nb)}
        h = fpt_hist()
        h.count = arrs["count"].ctypes.data_as(_u64p)
        h.sum_w_bin = arrs["sum_w"].ctypes.data_as(_dp)
        h.sum_w2_bin = arrs["sum_w2"].ctypes.data_as(_dp)
        h.sum_lnw_bin = arrs["sum_lnw"].ctypes.data_as(_dp)
        h.sum_lnw2_bin = arrs["sum_lnw2"].ctypes.data_as(_dp)
        _check(self._lib.fpt_histogram(self._h, ctypes.byref(h)), "fpt_histogram")
        arrs.update(n_traj=h.n_traj, n_censored=h.n_censored, n_ended_early=h.n_ended_early,
                    n_steps_total=h.n_steps_total, sum_w_total=h.sum_w, sum_w2_total=h.sum_w2, sum_wN=h.sum_wN,
                    sum_wN2=h.sum_wN2)
        return arrs

    def reset(self):
        _check(self._lib.fpt_reset(self._h), "fpt_reset")

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double()
        _check(self._lib.fpt_last_kernel_ms(self._h, ctypes.byref(ms)), "fpt_last_kernel_ms")
        return ms.value

    # ---- learned bias -------------------------------------------------------
    def mlp_set(self, params, stream=None):
        """params: a device tensor, or host values (copied through a float32 array)."""
        if torch is not None and isinstance(params, torch.Tensor) and params.is_cuda:
            src = params.contiguous()
            _check(self._lib.fpt_mlp_set(self._h, src.data_ptr(), _stream_handle(stream)), "fpt_mlp_set")
            return
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != FPT_MLP_NPARAM:
            raise ValueError(f"need {FPT_MLP_NPARAM} parameters")
        _check(self._lib.fpt_mlp_set(self._h, a.ctypes.data, _stream_handle(stream)), "fpt_mlp_set")
        torch.cuda.synchronize()     # the host array must outlive the copy

    def mlp_get(self, stream=None) -> np.ndarray:
        a = np.empty(FPT_MLP_NPARAM, dtype=np.float32)
        _check(self._lib.fpt_mlp_get(self._h, a.ctypes.data, _stream_handle(stream)), "fpt_mlp_get")
        return a

    def mlp_table(self) -> np.ndarray:
        a = np.empty(self.grid_n[0] * self.grid_n[1], dtype=np.float64)
        _check(self._lib.fpt_mlp_table(self._h, a.ctypes.data_as(_dp)), "fpt_mlp_table")
        return a.reshape(self.grid_n)

    def mlp_grad(self, n_traj: int, dN: float, seed: int, tail_lo: float, d_grad, traj_offset: int = 0, stream=None,
                 d_G=None, want_J: bool = True, objective: int = FPT_MLP_OBJ_J, noalloc: bool = False):
        """Fill d_grad (device, 4482 float32) with dJ/dtheta (or d ln J/dtheta); returns (J, n_tail)
        when want_J.  noalloc selects fpt_mlp_grad_noalloc (no device allocation; n_traj at most
        FPT_MLP_GRAD_NOALLOC_MAX)."""
        J = ctypes.c_double()
        nt = ctypes.c_uint64()
        name = "fpt_mlp_grad_noalloc" if noalloc else "fpt_mlp_grad"
        _check(getattr(self._lib, name)(self._h, n_traj, dN, seed, traj_offset, tail_lo, objective,
                                        _stream_handle(stream),
                                        _ptr(d_grad), _ptr(d_G), ctypes.byref(J) if want_J else None,
                                        ctypes.byref(nt) if want_J else None), name)
        return (J.value, int(nt.value)) if want_J else None

    def mlp_adam(self, d_grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 stream=None):
        _check(self._lib.fpt_mlp_adam(self._h, _ptr(d_grad), lr, beta1, beta2, eps, _stream_handle(stream)),
               "fpt_mlp_adam")

    def destroy(self):
        if getattr(self, "_h", None):
            self._lib.fpt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Owns one fpt_batch over a list of Contexts (which must outlive it)."""

    def __init__(self, contexts, *, block_size=0, chunk=0, item_size=0, use_graph=True):
        L = load()
        self._ctxs = list(contexts)
        arr = (ctypes.c_void_p * len(self._ctxs))(*[c.handle.value for c in self._ctxs])
        opts = fpt_batch_options(block_size, chunk, item_size, 1 if use_graph else 0)
        h = ctypes.c_void_p()
        _check(L.fpt_batch_create(arr, len(self._ctxs), ctypes.byref(opts), ctypes.byref(h)), "fpt_batch_create")
        self._h = h
        self._lib = L

    def _counts(self, n_traj):
        a = np.ascontiguousarray(n_traj, dtype=np.uint64)
        if a.shape != (len(self._ctxs),):
            raise ValueError("one trajectory count per instance")
        return a

    def run(self, n_traj, dN: float, seed: int, traj_offset: int = 0, stream=None):
        a = self._counts(n_traj)
        _check(self._lib.fpt_batch_run(self._h, a.ctypes.data_as(_u64p), dN, seed, traj_offset,
                                       _stream_handle(stream)), "fpt_batch_run")

    def autotune(self, n_traj, dN: float, seed: int, cache_path=None, stream=None):
        a = self._counts(n_traj)
        path = cache_path.encode() if cache_path else None
        _check(self._lib.fpt_batch_autotune(self._h, a.ctypes.data_as(_u64p), dN, seed, path,
                                            _stream_handle(stream)), "fpt_batch_autotune")

    def config(self):
        b, c = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.fpt_batch_config(self._h, ctypes.byref(b), ctypes.byref(c)), "fpt_batch_config")
        return b.value, c.value

    def last_ms(self) -> float:
        ms = ctypes.c_double()
        _check(self._lib.fpt_batch_last_ms(self._h, ctypes.byref(ms)), "fpt_batch_last_ms")
        return ms.value

    def destroy(self):
        if getattr(self, "_h", None):
            self._lib.fpt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
