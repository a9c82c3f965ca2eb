"""Seeded, synthetic workload definitions shared by the tests, the benchmark
and the smoke check.

This module holds parameters only: potentials, start/end points, table grids,
time steps, trajectory counts, seeds and histogram layouts.  It performs none
of the method's arithmetic (no noise model, no drift, no stepping) and imports
neither the GPU binding nor the CPU oracle, so both can be fed from it.

The paper's numerical experiments (Sec. 4.2) use the piecewise-linear
potential V = V0 + A_+-(phi - phi_T) of eq. (potential_starobinsky) with
A_- = 1e-3 A_+.  The workloads below use V0 = 1e-10 and slope parameters
eps_V = (A/V0)^2/2 of 0.01 (steep side) and 1e-8 (flat side), which give the
same ratio A_-/A_+ = 1e-3.  No dataset is involved anywhere.

Derived constants are stored rather than recomputed at import time:
NOISE_S_HUBBLE (H/2pi with H^2 = V0/3), DELTA_E (the distance phi_e - phi_end for which the noise-free Euler-Maruyama
passage time from phi_e is 10 e-folds at dN = 1e-4) and the noise-free
reference times N_REF_*.  They were written by ``oracle/derive_constants.py``,
which calls only the CPU oracle; ``tests/test_workloads.py`` re-derives them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

POT_PIECEWISE_LINEAR = 0
POT_EXPONENTIAL = 1
POT_GAUSSIAN_BUMP = 2
BIAS_NONE = 0
BIAS_CONST = 1
BIAS_MLP = 2
BINS_LINEAR = 0
BINS_LOG = 1

V0 = 1e-10
EPS_PLUS = 0.01        # slope parameter on the slow-roll side, eps_V = (A_+/V0)^2 / 2
EPS_MINUS = 1e-8       # slope parameter on the ultra-slow-roll side
A_PLUS = V0 * math.sqrt(2.0 * EPS_PLUS)
A_MINUS = V0 * math.sqrt(2.0 * EPS_MINUS)

# Written by oracle/derive_constants.py (noise-free oracle runs).
NOISE_S_HUBBLE = 9.188814923696534e-07  # H/2pi with H^2 = V0/3 (de Sitter noise amplitude)
DELTA_E = 0.04857416112949248        # phi_e - phi_end giving N = 10 at dN = 1e-4
N_REF_SRUSR = 9.999999999999952       # noise-free N for the SR->USR workloads at dN = 1e-4
N_REF_LINEAR = 7.612929983590818       # noise-free N for the linear slow-roll workload at dN = 1e-3
SIGMA_LIN_LINEAR = 1.918e-5          # linear-theory spread of N for the linear workload
SIGMA_LIN_SRUSR = 0.0205             # linear-theory spread of N for the SR->USR workloads

# Dyadic noise-table grid: phi_j = (j - 3300) 2^-16 for j = 0..4095, so every
# node, including the transition phi_T = 0, is an exact double.
TABLE_N = 4096
TABLE_H = 2.0 ** -16
TABLE_J_T = 3300
TABLE_PHI_LO = -TABLE_J_T * TABLE_H
TABLE_PHI_HI = (TABLE_N - 1 - TABLE_J_T) * TABLE_H


@dataclass
class Workload:
    """One first-passage problem with its run and histogram settings."""
    name: str
    kind: int
    V0: float
    phi_T: float
    A_plus: float
    A_minus: float
    phi_in: float
    pi_in: float
    phi_end: float
    noise: str                      # "const": S = noise_S, tan = noise_tan (one table node);
                                    # "bessel": eq. (covariance_constant_nu) table on the grid below;
                                    # "xi_const": 2D noise with covariance noise_Xi (one node);
                                    # "bessel2d": 2D noise of eq. (covariance_matrix_direct) on the grid;
                                    # "bessel2d_time": the same on nodes in time (as "matched_time");
                                    # "matched": eq. (covariance_constant_nu_bessel_matched) on the grid,
                                    # B_k from the classical trajectory started at match_start;
                                    # "matched_time": the same noise on nodes in time, table_lo and
                                    # table_hi the times after the trajectory passes phi_in
    dN: float
    n_traj: int
    seed: int
    noise_S: float = 0.0
    noise_tan: float = 0.0
    noise_Xi: tuple = (0.0, 0.0, 0.0)   # (Xi_pp, Xi_pq, Xi_qq) for "xi_const"
    sigma: float = 1.0              # coarse-graining ratio k_sigma / aH
    match_start: tuple = (0.0, 0.0)  # (phi, pi) at which the "matched" table's classical trajectory starts
    noise_cut_below: bool = False    # the table's lowest node carries no noise: none below the table
    noise_cut_end: bool = False      # the table's last node carries no noise: none after the table
    bump: tuple = (0.0, 0.0, 0.0)    # (m, K, Sigma) of the Gaussian bump (centre phi_0 = phi_T)
    table_n: int = 1
    table_lo: float = 0.0
    table_hi: float = 0.0
    bias_kind: int = BIAS_NONE
    A_bias: float = 0.0
    precision: int = 0              # 0 FP64, 1 FP32 state
    bins_kind: int = BINS_LINEAR
    n_bins: int = 64
    lo: float = -1.0
    hi: float = 1.0
    N_ref: float = 0.0
    max_steps: int = 1 << 24         # far above every workload here (<= 1.2e5 steps per trajectory)
    # learned control (bias_kind == BIAS_MLP): network parameters (4482 float32), input
    # normalisation (c0, s0, c1, s1) and the tabulation grid over the normalised inputs
    mlp_params: Optional[np.ndarray] = None
    mlp_norm: tuple = (0.0, 1.0, 0.0, 1.0)
    grid_n: tuple = (2, 2)
    grid_range: tuple = (-1.0, 1.0, -1.0, 1.0)
    extra: dict = field(default_factory=dict)

    def with_(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def linear_slow_roll(n_traj: int = 10_000, seed: int = 1) -> Workload:
    """V = V0 (1 + sqrt(2 * 0.01) (phi - phi_end)), phi_in = phi_end + 1, pi_in = -V'/V(phi_in),
    constant noise H/2pi, dN = 1e-3, 64 linear bins over deltaN in [-5, 5] sigma."""
    alpha = math.sqrt(2.0 * EPS_PLUS)
    return Workload(
        name="linear_slow_roll", kind=POT_PIECEWISE_LINEAR, V0=V0, phi_T=0.0,
        A_plus=V0 * alpha, A_minus=V0 * alpha, phi_in=1.0, pi_in=-alpha / (1.0 + alpha), phi_end=0.0,
        noise="const", noise_S=NOISE_S_HUBBLE, noise_tan=0.0, dN=1e-3, n_traj=n_traj, seed=seed,
        bins_kind=BINS_LINEAR, n_bins=64, lo=-5 * SIGMA_LIN_LINEAR, hi=5 * SIGMA_LIN_LINEAR,
        N_ref=N_REF_LINEAR)


def exponential_ig(n_traj: int = 20_000, seed: int = 7, alpha: float = 0.5, S: float = 0.05,
                   delta_phi: float = 1.0, dN: float = 1e-4, A_bias: float = 0.0) -> Workload:
    """V = V0 exp(alpha (phi - phi_end)) with pi_in = -alpha (an exact fixed point of the
    drift) and constant noise S along phi only: phi is a Brownian motion with drift -alpha,
    so N is inverse-Gaussian with mean delta_phi/alpha and shape delta_phi^2/S^2."""
    return Workload(
        name="exponential_ig", kind=POT_EXPONENTIAL, V0=V0, phi_T=0.0, A_plus=alpha, A_minus=0.0,
        phi_in=delta_phi, pi_in=-alpha, phi_end=0.0, noise="const", noise_S=S, noise_tan=0.0,
        dN=dN, n_traj=n_traj, seed=seed, bias_kind=BIAS_CONST if A_bias else BIAS_NONE,
        A_bias=A_bias, bins_kind=BINS_LINEAR, n_bins=64,
        lo=-1.0, hi=3.0, N_ref=delta_phi / alpha)


def srusr_bessel(n_traj: int = 1_000_000, seed: int = 2) -> Workload:
    """Piecewise-linear slow roll -> ultra-slow roll, phi_T = phi_e = 0 = phi_in,
    pi_in = -sqrt(2 eps_+) (the slow-roll value at phi_e), phi_end = -DELTA_E,
    Bessel-ansatz noise table (4096 nodes, sigma = 1), FP64, dN = 1e-4, no bias."""
    return Workload(
        name="srusr_bessel_fp64", kind=POT_PIECEWISE_LINEAR, V0=V0, phi_T=0.0,
        A_plus=A_PLUS, A_minus=A_MINUS, phi_in=0.0, pi_in=-math.sqrt(2.0 * EPS_PLUS),
        phi_end=-DELTA_E, noise="bessel", sigma=1.0, table_n=TABLE_N,
        table_lo=TABLE_PHI_LO, table_hi=TABLE_PHI_HI, dN=1e-4, n_traj=n_traj, seed=seed,
        bins_kind=BINS_LINEAR, n_bins=64, lo=-5 * SIGMA_LIN_SRUSR, hi=5 * SIGMA_LIN_SRUSR,
        N_ref=N_REF_SRUSR)


def srusr_is_fp32(A_bias: float = 2.0, n_traj: int = 100_000_000, seed: int = 3) -> Workload:
    """The SR->USR problem with FP32 state and FP64 log-weights, constant IS bias, weighted
    P(deltaN) on 256 log-spaced bins over deltaN in [sigma/2, 8 sigma]."""
    return srusr_bessel(n_traj=n_traj, seed=seed).with_(
        name=f"srusr_is_fp32_A{A_bias:g}", precision=1, bias_kind=BIAS_CONST, A_bias=A_bias,
        bins_kind=BINS_LOG, n_bins=256, lo=0.5 * SIGMA_LIN_SRUSR, hi=8 * SIGMA_LIN_SRUSR)


# The matched table's classical trajectory starts 7 e-folds of slow roll above the transition,
# on the steep branch's attractor, so every node's mode can start at k = 100 aH with sigma = 1.
MATCH_PHI_START = 1.0


def srusr_matched(n_traj: int = 1_000_000, seed: int = 7, sigma: float = 1.0) -> Workload:
    """The SR -> USR problem with the Bessel-matched noise of eq. (covariance_constant_nu_bessel_matched)
    on the 4096-node grid: B_k from the mode equation solved along the classical trajectory from
    phi = 1 (pi = -V'/V there), FP64, dN = 1e-4, no bias."""
    pi0 = -A_PLUS / (V0 + A_PLUS * MATCH_PHI_START)
    return srusr_bessel(n_traj=n_traj, seed=seed).with_(
        name=f"srusr_matched_sigma{sigma:g}", noise="matched", sigma=sigma, match_start=(MATCH_PHI_START, pi0))


# Noise indexed by time: the runs start on the matched table's classical trajectory, at the
# transition, with the momentum it has there.  Written by `python -m oracle.derive_constants --time`
# (scipy solve from MATCH_PHI_START; oracle Euler-Maruyama passage): 7.61 e-folds from phi = 1,
# pi there is 0.65 % below -sqrt(2 eps_+) in magnitude, and the slow final phase turns that into
# a noise-free passage of 12.18 e-folds to phi_end.
TIME_PI_IN = -0.14049970258869465
N_REF_TIME = 12.179564152175258


def srusr_time(n_traj: int = 1_000_000, seed: int = 13, tau_hi: float = 12.5, table_n: int = TABLE_N,
               sigma: float = 1.0) -> Workload:
    """The SR -> USR problem with the Bessel-matched noise indexed by time, the paper's scheme
    (Sec. 4.1): table_n nodes over tau in [0, tau_hi] after the classical trajectory from phi = 1
    passes phi_in = 0, the runs started on it (TIME_PI_IN), the last node zero, so the noise (and
    the bias) stop at tau_hi and the run goes on classically to phi_end.  tau_hi = 12.5 keeps the
    noise on past the classical passage (12.18 e-folds); a smaller tau_hi switches it off earlier."""
    return srusr_matched(n_traj=n_traj, seed=seed, sigma=sigma).with_(
        name=f"srusr_time_tau{tau_hi:g}", noise="matched_time", pi_in=TIME_PI_IN, N_ref=N_REF_TIME,
        table_n=table_n, table_lo=0.0, table_hi=tau_hi, noise_cut_end=True)


def srusr_is_fp32_time(A_bias: float = 2.0, n_traj: int = 100_000_000, seed: int = 17) -> Workload:
    """srusr_is_fp32 on the time-indexed problem of srusr_time."""
    t = srusr_time()
    return srusr_is_fp32(A_bias=A_bias, n_traj=n_traj, seed=seed).with_(
        name=f"srusr_is_fp32_time_A{A_bias:g}", noise="matched_time", match_start=t.match_start, pi_in=t.pi_in,
        N_ref=t.N_ref, table_lo=0.0, table_hi=t.table_hi, noise_cut_end=True)


def srusr_is_fp32_matched(A_bias: float = 2.0, n_traj: int = 100_000_000, seed: int = 3) -> Workload:
    """srusr_is_fp32 with the Bessel-matched noise table."""
    m = srusr_matched()
    return srusr_is_fp32(A_bias=A_bias, n_traj=n_traj, seed=seed).with_(
        name=f"srusr_is_fp32_matched_A{A_bias:g}", noise="matched", match_start=m.match_start)


# Gaussian bump, eq. (potential_swagat), with the paper's K, m, Sigma and phi_0.  Written by
# `python -m oracle.derive_constants --bump` (oracle potential, scipy background from phi = 3.2
# on the slow-roll attractor): the transition N_T (first eps2 < -3) is 42.1417 e-folds after
# phi = 3.2 and ultra-slow roll ends at 44.5506.  The noise acts (sigma = 1) from the middle of
# ultra-slow roll, N = 43.346 (phi_in, pi_in), to N_T + 4.7 (BUMP_PHI_LO), where eps2 = 0.7316 in
# the constant-eps2 phase.  V0 is set by P_R = V/(24 pi^2 eps_V) = 2.1e-9 at 55 e-folds before eps1 = 1.
BUMP = (0.5, 1.17e-3, 1.59e-2)
BUMP_PHI0 = 2.18812
BUMP_V0 = 8.885867165645307e-11
BUMP_PHI_IN = 2.2034255935977227
BUMP_PI_IN = -0.0010119120161906673
BUMP_PHI_LO = 2.20304329338396
BUMP_EPS2 = 0.7316306386485752      # eps2 at N_T + 4.7 (the last mode's coarse-graining crossing)
BUMP_PHI_END = 2.0                  # on the slow-roll attractor again, ~16 e-folds after phi_in
BUMP_N_REF = 16.010232287737356     # noise-free passage to BUMP_PHI_END at dN = 1e-3
BUMP_MATCH_START = 2.5              # the matched table's classical trajectory starts here
BUMP_TAU_HI = 3.4955927519341046    # the same window in e-folds: N_T + 4.7 - (N_T + N_USR_END)/2


def gaussian_bump(n_traj: int = 1_000_000, seed: int = 11, A_bias: float = 0.0, dN: float = 1e-3) -> Workload:
    """The Gaussian-bump model of eq. (potential_swagat) (K = 1.17e-3, m = 0.5, Sigma = 1.59e-2,
    phi_0 = 2.18812), FP64 state.  Bessel-matched noise (sigma = 1) on 4096 nodes over the window
    [BUMP_PHI_LO, BUMP_PHI_IN]; none below it.  From (phi_in, pi_in) on the classical trajectory to
    phi_end = 2.0; constant bias A_bias.  64 linear bins over deltaN in [-0.5, 1.5)."""
    dlnV0 = 2 * 0.25 / (BUMP_MATCH_START * (0.25 + BUMP_MATCH_START ** 2))   # V'/V at phi = 2.5 (bump ~ 0)
    return Workload(
        name=f"gaussian_bump_A{A_bias:g}", kind=POT_GAUSSIAN_BUMP, V0=BUMP_V0, phi_T=BUMP_PHI0, A_plus=0.0,
        A_minus=0.0, phi_in=BUMP_PHI_IN, pi_in=BUMP_PI_IN, phi_end=BUMP_PHI_END, noise="matched", sigma=1.0,
        table_n=TABLE_N, table_lo=BUMP_PHI_LO, table_hi=BUMP_PHI_IN, match_start=(BUMP_MATCH_START, -dlnV0),
        noise_cut_below=True, bump=BUMP, dN=dN, n_traj=n_traj, seed=seed,
        bias_kind=BIAS_CONST if A_bias else BIAS_NONE, A_bias=A_bias, bins_kind=BINS_LINEAR, n_bins=64,
        lo=-0.5, hi=1.5, N_ref=BUMP_N_REF)


def gaussian_bump_is(A_bias: float = 3.0, n_traj: int = 10_000_000, seed: int = 12) -> Workload:
    """gaussian_bump with a constant bias and 96 log-spaced bins over deltaN in [0.02, 3): the far
    tail, where the classical constant-eps2 form of eq. (delta_N_pdf_constant_epsilon_2) applies."""
    return gaussian_bump(n_traj=n_traj, seed=seed, A_bias=A_bias).with_(
        name=f"gaussian_bump_is_A{A_bias:g}", bins_kind=BINS_LOG, n_bins=96, lo=0.02, hi=3.0)


def gaussian_bump_time(n_traj: int = 1_000_000, seed: int = 11, A_bias: float = 0.0, dN: float = 1e-3,
                       table_n: int = TABLE_N) -> Workload:
    """gaussian_bump with the noise indexed by time, the paper's scheme (Sec. 4.1): table_n nodes over
    tau in [0, BUMP_TAU_HI] after the classical trajectory passes phi_in, the same window of modes in
    e-folds, the last node zero, so the noise (and the bias) stop after BUMP_TAU_HI e-folds whatever
    phi a trajectory has reached."""
    return gaussian_bump(n_traj=n_traj, seed=seed, A_bias=A_bias, dN=dN).with_(
        name=f"gaussian_bump_time_A{A_bias:g}", noise="matched_time", table_n=table_n, table_lo=0.0,
        table_hi=BUMP_TAU_HI, noise_cut_below=False, noise_cut_end=True)


def gaussian_bump_time_is(A_bias: float = 3.0, n_traj: int = 10_000_000, seed: int = 12) -> Workload:
    """gaussian_bump_time with a constant bias and the far-tail bins of gaussian_bump_is."""
    return gaussian_bump_time(n_traj=n_traj, seed=seed, A_bias=A_bias).with_(
        name=f"gaussian_bump_time_is_A{A_bias:g}", bins_kind=BINS_LOG, n_bins=96, lo=0.02, hi=3.0)


def batched_instances(n_inst: int = 64, seed: int = 4, n_min: float = 1e5, n_max: float = 1e7,
                      max_steps: int = 1 << 20) -> list[Workload]:
    """Instances of the SR->USR problem with eps_- log-uniform in [1e-10, 1e-6] and
    phi_e - phi_end uniform in [0.1, 1]; trajectory counts log-uniform in [n_min, n_max];
    a per-instance step cap censors the (very long) flat-branch runs.  The noise table
    uses 4096 nodes phi_j = (j - 2100) 2^-11, covering [-1.03, 0.97] with a node at phi_T."""
    rng = np.random.default_rng(seed)
    eps_m = 10.0 ** rng.uniform(-10, -6, n_inst)
    delta = rng.uniform(0.1, 1.0, n_inst)
    counts = np.round(10.0 ** rng.uniform(math.log10(n_min), math.log10(n_max), n_inst)).astype(np.int64)
    out = []
    for i in range(n_inst):
        w = srusr_bessel(n_traj=int(counts[i]), seed=seed).with_(
            name=f"batched_{i}", A_minus=V0 * math.sqrt(2.0 * eps_m[i]), phi_end=-float(delta[i]),
            table_lo=-2100 * 2.0 ** -11, table_hi=(4095 - 2100) * 2.0 ** -11,
            max_steps=int(max_steps), extra={"instance": i, "eps_minus": float(eps_m[i])})
        out.append(w)
    return out


# ---------------------------------------------------------------------------
# learned control
# ---------------------------------------------------------------------------
MLP_NPARAM = 4482
MLP_HIDDEN = 64


def mlp_constant_init(A: float, seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """Initial parameters whose output 0 is the constant A: W1, W2 drawn N(0, gain^2/fan_in)
    (seeded), biases 0, W3 = 0, b3 = (A, 0).  Training starts from the constant-bias control."""
    rng = np.random.default_rng(seed)
    p = np.zeros(MLP_NPARAM, dtype=np.float32)
    p[:128] = rng.standard_normal(128) * gain / math.sqrt(2.0)
    p[192:4288] = rng.standard_normal(4096) * gain / math.sqrt(MLP_HIDDEN)
    p[4480] = A
    return p


def mlp_random(seed: int, scale: float = 0.2, out_bias: float = 1.0) -> np.ndarray:
    """Random parameters (every entry N(0, scale^2)) with output bias b3[0] = out_bias: a
    smoothly varying amplitude around out_bias, for parity tests."""
    p = (np.random.default_rng(seed).standard_normal(MLP_NPARAM) * scale).astype(np.float32)
    p[4480] = out_bias
    return p


def srusr_learned(n_traj: int = 10_000_000, seed: int = 5, A_init: float = 1.0,
                  grid_n: tuple = (32, 32)) -> Workload:
    """The SR->USR problem with FP32 state and a learned control: inputs
    x0 = (phi - phi_mid)/(DELTA_E/2) (phi_mid halfway between phi_end and phi_in) and
    x1 = (ln|pi| - c1)/s1 mapping ln|pi| from ln sqrt(2 eps_+) (start) to ln sqrt(2 eps_-)
    (the flat-branch attractor) onto [1, -1]; tabulated on grid_n nodes over
    x0 in [-1.05, 1.05], x1 in [-1.2, 1.2]; the network starts as the constant A_init."""
    ln_hi, ln_lo = 0.5 * math.log(2.0 * EPS_PLUS), 0.5 * math.log(2.0 * EPS_MINUS)
    return srusr_is_fp32(A_bias=0.0, n_traj=n_traj, seed=seed).with_(
        name="srusr_learned_fp32", bias_kind=BIAS_MLP, A_bias=0.0,
        mlp_params=mlp_constant_init(A_init, seed=seed),
        mlp_norm=(-0.5 * DELTA_E, 0.5 * DELTA_E, 0.5 * (ln_hi + ln_lo), 0.5 * (ln_hi - ln_lo)),
        grid_n=tuple(grid_n), grid_range=(-1.05, 1.05, -1.2, 1.2))


def exponential_ig_learned(n_traj: int = 4000, seed: int = 29, dN: float = 2e-3, params=None,
                           grid_n: tuple = (24, 12)) -> Workload:
    """The inverse-Gaussian companion with a learned control: x0 = (phi - 0.5)/0.5 (phi from
    phi_in = 1 to phi_end = 0 maps to [1, -1]), x1 = ln|pi| - ln 0.5 (pi stays at -alpha = -0.5
    without bias; the bias moves only phi, so x1 = 0), grid over x0 in [-1.05, 1.05] and
    x1 in [-1.5, 1.5]."""
    return exponential_ig(n_traj=n_traj, seed=seed, dN=dN).with_(
        name="exponential_ig_learned", bias_kind=BIAS_MLP, mlp_params=params,
        mlp_norm=(0.5, 0.5, math.log(0.5), 1.0), grid_n=tuple(grid_n), grid_range=(-1.05, 1.05, -1.5, 1.5))


# ---------------------------------------------------------------------------
# two-dimensional noise
# ---------------------------------------------------------------------------
TABLE2D_N = 2048
TABLE2D_H = 2.0 ** -15
TABLE2D_J_T = 1650          # node at phi_T = 0; same range as the 1D grid


def srusr_2d(n_traj: int = 1_000_000, seed: int = 6, sigma: float = 0.1, A_bias: float = 0.0) -> Workload:
    """The SR -> USR problem with 2D noise: the covariance of the full Bunch-Davies mode at
    -k eta = sigma (eq. covariance_matrix_direct; sigma << 1 as that approach requires) on 2048
    nodes phi_j = (j - 1650) 2^-15, FP64 state, dN = 1e-4, optional constant bias."""
    return srusr_bessel(n_traj=n_traj, seed=seed).with_(
        name=f"srusr_2d_sigma{sigma:g}", noise="bessel2d", sigma=sigma, table_n=TABLE2D_N,
        table_lo=-TABLE2D_J_T * TABLE2D_H, table_hi=(TABLE2D_N - 1 - TABLE2D_J_T) * TABLE2D_H,
        bias_kind=BIAS_CONST if A_bias else BIAS_NONE, A_bias=A_bias)


def srusr_2d_time(n_traj: int = 1_000_000, seed: int = 6, sigma: float = 0.1, A_bias: float = 0.0,
                  tau_hi: float = 12.5, table_n: int = TABLE2D_N) -> Workload:
    """srusr_2d with the covariance indexed by time, the paper's scheme (Sec. 4.1): table_n nodes over
    tau in [0, tau_hi] after the matched table's reference trajectory (from phi = 1) passes phi_in = 0,
    the runs started on it (TIME_PI_IN), the last node zero, so the noise and the bias stop at tau_hi."""
    t = srusr_time()
    return srusr_2d(n_traj=n_traj, seed=seed, sigma=sigma, A_bias=A_bias).with_(
        name=f"srusr_2d_time_sigma{sigma:g}_tau{tau_hi:g}", noise="bessel2d_time", pi_in=TIME_PI_IN,
        N_ref=N_REF_TIME, match_start=t.match_start, table_n=table_n, table_lo=0.0, table_hi=tau_hi,
        noise_cut_end=True)


def exponential_2d(n_traj: int = 4000, seed: int = 9, S: float = 0.05, rho: float = 0.8, ratio: float = 1.0,
                   dN: float = 1e-3, A_bias: float = 0.0) -> Workload:
    """The exponential companion with a constant, correlated 2D noise: Xi = S^2 [[1, rho r], [rho r, r^2]]
    (r = ratio of the pi to the phi amplitude), acting on phi and pi."""
    return exponential_ig(n_traj=n_traj, seed=seed, S=S, dN=dN).with_(
        name="exponential_2d", noise="xi_const", noise_Xi=(S * S, rho * ratio * S * S, ratio * ratio * S * S),
        bias_kind=BIAS_CONST if A_bias else BIAS_NONE, A_bias=A_bias)
