"""Test infrastructure, not part of the product.

Python access to the FP64 CPU oracle in ``fpt_oracle.c`` plus the closed forms
the tests pin it against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module.  It never imports the GPU
package, and the GPU package never imports it.

Paper: Jackson et al., "Stochastic inflation beyond slow roll: noise modelling
and importance sampling", arXiv:2410.13683.  The oracle follows Sec. 4.1
(Euler-Maruyama with 1D noise, diffusion-based bias, weights of the Mazonka
form), Sec. 3.2 (constant-nu noise, eq. covariance_constant_nu) and Sec. 3.4
(nu^2 as a function of phi, eq. nu_squared_approximation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

POT_PIECEWISE_LINEAR = 0
POT_EXPONENTIAL = 1
POT_GAUSSIAN_BUMP = 2
BIAS_NONE = 0
BIAS_CONST = 1
BIAS_MLP = 2
FLAG_CENSORED = 0x80000000
FLAG_ENDED_EARLY = 0x40000000
STEP_MASK = 0x3FFFFFFF
MLP_NPARAM = 4482


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = f"{_LIB}.{os.getpid()}.tmp"      # per process: concurrent builds (test workers) do not collide
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64, dp]
        L.orc_normals.restype = None
        L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, dp]
        L.orc_uniforms.restype = None
        for name in ("orc_V", "orc_dV", "orc_d2V"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int, dp, ctypes.c_double]
            f.restype = ctypes.c_double
        L.orc_noise_table_bessel.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_noise_table_bessel.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_run.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, ctypes.c_double, fp, dp, ctypes.c_int, ip, dp,
                              ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_int64, dp, dp, u32p, dp, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_mlp_eval.argtypes = [fp, dp, ctypes.c_double, ctypes.c_double]
        L.orc_mlp_eval.restype = ctypes.c_double
        L.orc_mlp_replay_grad.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          fp, fp, dp, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int]
        L.orc_mlp_replay_grad.restype = ctypes.c_int
        L.orc_mlp_tabulate.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp]
        L.orc_mlp_tabulate.restype = ctypes.c_int
        L.orc_grid_replay_grad.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           fp, fp, dp, ip, dp, ctypes.c_double, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        L.orc_grid_replay_grad.restype = ctypes.c_int
        L.orc_adam_step.argtypes = [fp, fp, fp, fp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double]
        L.orc_adam_step.restype = None
        L.orc_noise_table_bessel2d.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                               ctypes.c_double, dp, dp, dp]
        L.orc_noise_table_bessel2d.restype = ctypes.c_int
        L.orc_sqrt_sym2.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc_sqrt_sym2.restype = ctypes.c_int
        L.orc_normals2d.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, dp]
        L.orc_normals2d.restype = None
        L.orc_run2d.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_int64, dp, dp, u32p, dp, ctypes.c_int]
        L.orc_run2d.restype = ctypes.c_int
        L.orc_principal_axis.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_principal_axis.restype = None
        L.orc_bessel_match.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.orc_bessel_match.restype = None
        L.orc_noise_table_matched.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp,
                                              ctypes.c_int]
        L.orc_noise_table_matched.restype = ctypes.c_int
        L.orc_noise_table_matched_time.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, dp, dp, dp, dp, ctypes.c_int]
        L.orc_noise_table_matched_time.restype = ctypes.c_int
        L.orc_noise_table_bessel2d_time.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, dp, dp, dp, dp]
        L.orc_noise_table_bessel2d_time.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_u32p(c), _u32p(k), _u32p(out))
    return out


def normals(seed: int, instance: int, traj: int, n0: int, count: int) -> np.ndarray:
    z = np.empty(count, dtype=np.float64)
    lib().orc_normals(seed, instance, traj, n0, count, _dp(z))
    return z


def uniforms(seed: int, instance: int, traj: int, call: int) -> np.ndarray:
    u = np.empty(4, dtype=np.float64)
    lib().orc_uniforms(seed, instance, traj, call, _dp(u))
    return u


# --------------------------------------------------------------------------
# problem description
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """One first-passage problem (Sec. 4.1): potential, noise table, bias, start/end."""
    kind: int
    V0: float
    phi_T: float
    A_plus: float
    A_minus: float
    phi_in: float
    pi_in: float
    phi_end: float
    S: np.ndarray              # noise amplitude S_phiphi at the table nodes
    tan_theta: np.ndarray      # tan(theta_n) at the table nodes
    phi_lo: float = 0.0
    phi_hi: float = 0.0
    bias_kind: int = BIAS_NONE
    A_bias: float = 0.0
    mlp_params: np.ndarray | None = None
    mlp_norm: np.ndarray | None = None
    mlp_every: int = 1                # >= 1: the network every k steps; 0: the tabulated network
    grid_n: tuple = (2, 2)            # tabulation grid over the normalised inputs (x0, x1)
    grid_range: tuple = (-1.0, 1.0, -1.0, 1.0)
    bump: tuple = (0.0, 0.0, 0.0)     # (m, K, Sigma) of the Gaussian bump (phi_0 = phi_T)
    tab_axis: int = 0                 # 0: table nodes in phi; 1: in the run's time N = n dN

    def pot(self) -> np.ndarray:
        return _pot_array(self.V0, self.phi_T, self.A_plus, self.A_minus, self.bump)


def _pot_array(V0, phi_T, A_plus, A_minus, bump=(0.0, 0.0, 0.0)) -> np.ndarray:
    """{V0, phi_T, A_plus, A_minus, m, K, Sigma}, the oracle's potential parameters."""
    return np.array([V0, phi_T, A_plus, A_minus, *bump], dtype=np.float64)


def potential(kind, V0, phi_T, A_plus, A_minus, phi, bump=(0.0, 0.0, 0.0)):
    p = _pot_array(V0, phi_T, A_plus, A_minus, bump)
    L = lib()
    return L.orc_V(kind, _dp(p), phi), L.orc_dV(kind, _dp(p), phi), L.orc_d2V(kind, _dp(p), phi)


def noise_table_bessel(kind, V0, phi_T, A_plus, A_minus, sigma, n, phi_lo, phi_hi, bump=(0.0, 0.0, 0.0)):
    """Eq. (covariance_constant_nu) with nu(phi) from eq. (nu_squared_approximation)."""
    p = _pot_array(V0, phi_T, A_plus, A_minus, bump)
    S = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    rc = lib().orc_noise_table_bessel(kind, _dp(p), sigma, n, phi_lo, phi_hi, _dp(S), _dp(t))
    if rc != 0:
        raise ValueError("invalid noise-table parameters")
    return S, t


def bessel_match(nu: float, y: float, pref: float, dphi: complex, ddphi: complex):
    """(A_k, B_k) of eq. (bessel_matching) from the mode and its N-derivative at -k eta = y, with
    pref = a/sqrt(-eta)."""
    f = np.array([dphi.real, dphi.imag]); g = np.array([ddphi.real, ddphi.imag])
    A = np.zeros(2); B = np.zeros(2)
    lib().orc_bessel_match(nu, y, pref, _dp(f), _dp(g), _dp(A), _dp(B))
    return complex(A[0], A[1]), complex(B[0], B[1])


def noise_table_matched(kind, V0, phi_T, A_plus, A_minus, sigma, n, phi_lo, phi_hi, phi_start, pi_start,
                        n_threads: int = 0, bump=(0.0, 0.0, 0.0)):
    """Eq. (covariance_constant_nu_bessel_matched) on the nodes: (S, tan_theta, 4|B_k|^2/pi), with B_k
    from the mode equation solved along the classical trajectory from (phi_start, pi_start)."""
    p = _pot_array(V0, phi_T, A_plus, A_minus, bump)
    S = np.empty(n); t = np.empty(n); fac = np.empty(n)
    rc = lib().orc_noise_table_matched(kind, _dp(p), sigma, n, phi_lo, phi_hi, phi_start, pi_start,
                                       _dp(S), _dp(t), _dp(fac), n_threads)
    if rc != 0:
        raise ValueError("invalid matched noise-table parameters (or phi_start too late for a node)")
    return S, t, fac


def noise_table_matched_time(kind, V0, phi_T, A_plus, A_minus, sigma, n, t_lo, t_hi, phi_start, pi_start,
                             phi_ref, n_threads: int = 0, bump=(0.0, 0.0, 0.0)):
    """The matched table on nodes in time after the classical trajectory passes phi_ref:
    (S, tan_theta, 4|B_k|^2/pi, phi at the nodes)."""
    p = _pot_array(V0, phi_T, A_plus, A_minus, bump)
    S = np.empty(n); t = np.empty(n); fac = np.empty(n); ph = np.empty(n)
    rc = lib().orc_noise_table_matched_time(kind, _dp(p), sigma, n, t_lo, t_hi, phi_start, pi_start, phi_ref,
                                            _dp(S), _dp(t), _dp(fac), _dp(ph), n_threads)
    if rc != 0:
        raise ValueError("invalid time-node matched table (start too late, phi_ref not passed, or a node "
                         "outside the trajectory)")
    return S, t, fac, ph


def run(prob: Problem, dN: float, seed: int, n_traj: int, traj_offset: int = 0, instance: int = 0,
        max_steps: int = STEP_MASK, n_threads: int = 0, last_phi: bool = False):
    """Per-trajectory (N, ln w, steps|flags) for trajectories traj_offset .. +n_traj-1; with
    last_phi also an (n_traj, 2) array of phi before and after each trajectory's last step."""
    S = np.ascontiguousarray(prob.S, dtype=np.float64)
    t = np.ascontiguousarray(prob.tan_theta, dtype=np.float64)
    N = np.empty(n_traj, dtype=np.float64)
    lnw = np.empty(n_traj, dtype=np.float64)
    steps = np.empty(n_traj, dtype=np.uint32)
    phi2 = np.empty((n_traj, 2)) if last_phi else None
    mlp = (np.ascontiguousarray(prob.mlp_params, dtype=np.float32)
           if prob.mlp_params is not None else np.zeros(MLP_NPARAM, dtype=np.float32))
    norm = (np.ascontiguousarray(prob.mlp_norm, dtype=np.float64)
            if prob.mlp_norm is not None else np.array([0.0, 1.0, 0.0, 1.0]))
    pot = prob.pot()
    gn = (ctypes.c_int * 2)(*prob.grid_n)
    gr = np.ascontiguousarray(prob.grid_range, dtype=np.float64)
    rc = lib().orc_run(prob.kind, _dp(pot), len(S), prob.phi_lo, prob.phi_hi, _dp(S), _dp(t), int(prob.tab_axis),
                       prob.phi_in, prob.pi_in, prob.phi_end, prob.bias_kind, prob.A_bias,
                       _fp(mlp), _dp(norm), prob.mlp_every, gn, _dp(gr), dN, seed, instance, traj_offset,
                       n_traj, max_steps, _dp(N), _dp(lnw), _u32p(steps), _dp(phi2) if last_phi else None,
                       n_threads)
    if rc != 0:
        raise ValueError("invalid oracle problem")
    return (N, lnw, steps, phi2) if last_phi else (N, lnw, steps)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def mlp_eval(params: np.ndarray, norm, phi: float, pi_: float) -> float:
    p = np.ascontiguousarray(params, dtype=np.float32)
    nrm = np.ascontiguousarray(norm, dtype=np.float64)
    return float(lib().orc_mlp_eval(_fp(p), _dp(nrm), phi, pi_))


def mlp_replay_grad(prob: Problem, theta_old: np.ndarray, theta: np.ndarray, dN: float, seed: int,
                    n_traj: int, N_ref: float, tail_lo: float, traj_offset: int = 0, instance: int = 0,
                    max_steps: int = STEP_MASK, n_threads: int = 0):
    """Gradient and value of J(theta) = (1/n) sum_T w_old w_theta on replayed paths."""
    S = np.ascontiguousarray(prob.S, dtype=np.float64)
    t = np.ascontiguousarray(prob.tan_theta, dtype=np.float64)
    told = np.ascontiguousarray(theta_old, dtype=np.float32)
    tnew = np.ascontiguousarray(theta, dtype=np.float32)
    norm = np.ascontiguousarray(prob.mlp_norm, dtype=np.float64)
    grad = np.empty(MLP_NPARAM, dtype=np.float64)
    J = np.zeros(1, dtype=np.float64)
    pot = prob.pot()
    rc = lib().orc_mlp_replay_grad(prob.kind, _dp(pot), len(S), prob.phi_lo, prob.phi_hi, _dp(S), _dp(t),
                                   prob.phi_in, prob.pi_in, prob.phi_end, _fp(told), _fp(tnew), _dp(norm),
                                   dN, seed, instance, traj_offset, n_traj, max_steps, N_ref, tail_lo,
                                   _dp(grad), _dp(J), n_threads)
    if rc != 0:
        raise ValueError("invalid oracle problem")
    return grad, float(J[0])


def mlp_tabulate(params: np.ndarray, grid_n, grid_range) -> np.ndarray:
    """Network output 0 on the grid (x0_i, x1_j), row-major [n0, n1]."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    out = np.empty(grid_n[0] * grid_n[1], dtype=np.float64)
    rc = lib().orc_mlp_tabulate(_fp(p), grid_n[0], grid_n[1], *[float(v) for v in grid_range], _dp(out))
    if rc != 0:
        raise ValueError("invalid grid")
    return out.reshape(grid_n[0], grid_n[1])


def grid_replay_grad(prob: Problem, theta_old: np.ndarray, theta: np.ndarray, dN: float, seed: int,
                     n_traj: int, N_ref: float, tail_lo: float, traj_offset: int = 0, instance: int = 0,
                     max_steps: int = STEP_MASK, n_threads: int = 0):
    """J(theta), its gradient and the grid-node weights G for paths drawn with the tabulated theta_old."""
    S = np.ascontiguousarray(prob.S, dtype=np.float64)
    t = np.ascontiguousarray(prob.tan_theta, dtype=np.float64)
    told = np.ascontiguousarray(theta_old, dtype=np.float32)
    tnew = np.ascontiguousarray(theta, dtype=np.float32)
    norm = np.ascontiguousarray(prob.mlp_norm, dtype=np.float64)
    gn = (ctypes.c_int * 2)(*prob.grid_n)
    gr = np.ascontiguousarray(prob.grid_range, dtype=np.float64)
    grad = np.empty(MLP_NPARAM, dtype=np.float64)
    G = np.empty(prob.grid_n[0] * prob.grid_n[1], dtype=np.float64)
    J = np.zeros(1, dtype=np.float64)
    pot = prob.pot()
    rc = lib().orc_grid_replay_grad(prob.kind, _dp(pot), len(S), prob.phi_lo, prob.phi_hi, _dp(S), _dp(t),
                                    prob.phi_in, prob.pi_in, prob.phi_end, _fp(told), _fp(tnew), _dp(norm),
                                    gn, _dp(gr), dN, seed, instance, traj_offset, n_traj, max_steps, N_ref,
                                    tail_lo, _dp(grad), _dp(J), _dp(G), n_threads)
    if rc != 0:
        raise ValueError("invalid oracle problem")
    return grad, float(J[0]), G.reshape(prob.grid_n[0], prob.grid_n[1])


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, grad: np.ndarray, t: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """Step t (1-based) of Adam on float32 arrays, updated in place."""
    for a in (theta, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float32)
    lib().orc_adam_step(_fp(theta), _fp(m), _fp(v), _fp(g), len(theta), t, lr, b1, b2, eps)


# --------------------------------------------------------------------------
# two-dimensional noise
# --------------------------------------------------------------------------
@dataclass
class Problem2D:
    """A first-passage problem with 2D noise: node covariances Xi (phi-phi, phi-pi, pi-pi)."""
    kind: int
    V0: float
    phi_T: float
    A_plus: float
    A_minus: float
    phi_in: float
    pi_in: float
    phi_end: float
    Xpp: np.ndarray
    Xpq: np.ndarray
    Xqq: np.ndarray
    phi_lo: float = 0.0
    phi_hi: float = 0.0
    bias_kind: int = BIAS_NONE
    A_bias: float = 0.0
    tab_axis: int = 0                # 1: the nodes are in the run's time (phi_lo, phi_hi hold N)

    def pot(self) -> np.ndarray:
        return _pot_array(self.V0, self.phi_T, self.A_plus, self.A_minus)


def noise_table_bessel2d(kind, V0, phi_T, A_plus, A_minus, sigma, n, phi_lo, phi_hi, bump=(0.0, 0.0, 0.0)):
    """(Xi_pp, Xi_pq, Xi_qq) at the nodes: both homogeneous modes of eq. (bessel_matched_homogeneous)."""
    p = _pot_array(V0, phi_T, A_plus, A_minus, bump)
    X = [np.empty(n, dtype=np.float64) for _ in range(3)]
    rc = lib().orc_noise_table_bessel2d(kind, _dp(p), sigma, n, phi_lo, phi_hi, *[_dp(x) for x in X])
    if rc != 0:
        raise ValueError("invalid noise-table parameters")
    return tuple(X)


def noise_table_bessel2d_time(kind, V0, phi_T, A_plus, A_minus, sigma, n, t_lo, t_hi, phi_start, pi_start, phi_ref):
    """(Xi_pp, Xi_pq, Xi_qq, phi at the nodes) of the 2D table on nodes in time after the classical
    trajectory from (phi_start, pi_start) passes phi_ref."""
    p = _pot_array(V0, phi_T, A_plus, A_minus)
    X = [np.empty(n, dtype=np.float64) for _ in range(4)]
    rc = lib().orc_noise_table_bessel2d_time(kind, _dp(p), sigma, n, t_lo, t_hi, phi_start, pi_start, phi_ref,
                                             *[_dp(x) for x in X])
    if rc != 0:
        raise ValueError("invalid 2D time-node table (phi_ref not passed, a node outside the trajectory, or a "
                         "node the covariance rejects)")
    return tuple(X)


def sqrt_sym2(a: float, b: float, c: float):
    out = [np.zeros(1) for _ in range(3)]
    if lib().orc_sqrt_sym2(a, b, c, *[_dp(x) for x in out]) != 0:
        raise ValueError("not positive semi-definite")
    return tuple(float(x[0]) for x in out)


def principal_axis(a: float, b: float, c: float):
    e = [np.zeros(1), np.zeros(1)]
    lib().orc_principal_axis(a, b, c, _dp(e[0]), _dp(e[1]))
    return float(e[0][0]), float(e[1][0])


def normals2d(seed: int, instance: int, traj: int, n0: int, count: int) -> np.ndarray:
    """(xi_1, xi_2) of steps n0 .. n0+count-1 of one trajectory with 2D noise, shape (count, 2)."""
    z = np.empty(2 * count, dtype=np.float64)
    lib().orc_normals2d(seed, instance, traj, n0, count, _dp(z))
    return z.reshape(count, 2)


def run2d(prob: Problem2D, dN: float, seed: int, n_traj: int, traj_offset: int = 0, instance: int = 0,
          max_steps: int = STEP_MASK, n_threads: int = 0, last_phi: bool = False):
    """As run, with 2D noise."""
    X = [np.ascontiguousarray(x, dtype=np.float64) for x in (prob.Xpp, prob.Xpq, prob.Xqq)]
    N = np.empty(n_traj, dtype=np.float64)
    lnw = np.empty(n_traj, dtype=np.float64)
    steps = np.empty(n_traj, dtype=np.uint32)
    phi2 = np.empty((n_traj, 2)) if last_phi else None
    pot = prob.pot()
    rc = lib().orc_run2d(prob.kind, _dp(pot), len(X[0]), prob.phi_lo, prob.phi_hi, *[_dp(x) for x in X],
                         int(prob.tab_axis), prob.phi_in, prob.pi_in, prob.phi_end, prob.bias_kind, prob.A_bias, dN, seed, instance,
                         traj_offset, n_traj, max_steps, _dp(N), _dp(lnw), _u32p(steps),
                         _dp(phi2) if last_phi else None, n_threads)
    if rc != 0:
        raise ValueError("invalid oracle problem")
    return (N, lnw, steps, phi2) if last_phi else (N, lnw, steps)


# --------------------------------------------------------------------------
# weighted histogram of deltaN = N - N_ref (Sec. 4.1: P(deltaN) from the
# sampled first-passage times, each weighted by w = exp(ln w))
# --------------------------------------------------------------------------
BINS_LINEAR = 0
BINS_LOG = 1


def bin_index(x: np.ndarray, bins_kind: int, n_bins: int, lo: float, hi: float) -> np.ndarray:
    """Index into an array of n_bins + 2: 0 = underflow, 1..n_bins, n_bins+1 = overflow.

    Linear bins: t = (x - lo) * (n_bins / (hi - lo)); log bins: t = ln(x / lo) * (n_bins / ln(hi / lo))
    (x <= 0 is underflow); bin = floor(t) + 1, clamped to the under/overflow slots.  Bins are half-open.
    """
    x = np.asarray(x, dtype=np.float64)
    if bins_kind == BINS_LINEAR:
        t = (x - lo) * (n_bins / (hi - lo))
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(x > 0, np.log(np.where(x > 0, x, 1.0) / lo) * (n_bins / np.log(hi / lo)), -1.0)
    j = np.floor(t)
    idx = np.where(t < 0, 0, np.where(j >= n_bins, n_bins + 1, j + 1))
    return idx.astype(np.int64)


def bin_edges(bins_kind: int, n_bins: int, lo: float, hi: float) -> np.ndarray:
    if bins_kind == BINS_LINEAR:
        return lo + (hi - lo) * np.arange(n_bins + 1) / n_bins
    return lo * (hi / lo) ** (np.arange(n_bins + 1) / n_bins)


def histogram(N, lnw, steps, N_ref, bins_kind, n_bins, lo, hi):
    """Accumulators per bin: count, sum w, sum w^2, sum ln w, sum (ln w)^2, plus totals."""
    N = np.asarray(N, dtype=np.float64)
    lnw = np.asarray(lnw, dtype=np.float64)
    steps = np.asarray(steps, dtype=np.uint32)
    crossed = (steps & (FLAG_CENSORED | FLAG_ENDED_EARLY)) == 0
    x = N[crossed] - N_ref
    lw = lnw[crossed]
    w = np.exp(lw)
    idx = bin_index(x, bins_kind, n_bins, lo, hi)
    nb = n_bins + 2
    out = {
        "count": np.bincount(idx, minlength=nb).astype(np.uint64),
        "sum_w": np.bincount(idx, weights=w, minlength=nb),
        "sum_w2": np.bincount(idx, weights=w * w, minlength=nb),
        "sum_lnw": np.bincount(idx, weights=lw, minlength=nb),
        "sum_lnw2": np.bincount(idx, weights=lw * lw, minlength=nb),
        "n_traj": int(len(N)),
        "n_censored": int(np.count_nonzero(steps & FLAG_CENSORED)),
        "n_ended_early": int(np.count_nonzero(steps & FLAG_ENDED_EARLY)),
        "n_steps_total": int(np.sum((steps & STEP_MASK).astype(np.uint64))),
        "sum_w_total": float(np.sum(w)),
        "sum_w2_total": float(np.sum(w * w)),
        "sum_wN": float(np.sum(w * N[crossed])),
        "sum_wN2": float(np.sum(w * N[crossed] ** 2)),
    }
    return out
