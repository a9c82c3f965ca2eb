"""MI355X (gfx950) first-passage-time library for the stochastic-deltaN method of
arXiv:2410.13683: batched Euler-Maruyama Langevin trajectories in (phi, pi) with
importance sampling, reduced to a weighted histogram of P(deltaN).

The compute path is the HIP library libfpt.so (C ABI in include/fpt.h); the
module ``fpt`` is its ctypes binding.
"""
__all__ = ["fpt", "workloads"]
