"""fpt_mlp_grad_noalloc (the gradient entry point that allocates no device memory; its
per-trajectory scratch is a fixed device array of the library) against fpt_mlp_grad, through the
C ABI: two calls in a row, the second with fewer trajectories, each equal to the allocating entry
point's result on the same trajectories (J and the tail count exactly up to the order of atomic
additions, the grid-node weights G to 1e-10, the FP32 gradient to FP32 rounding), and a size
beyond the array rejected on the host."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2410_13683_amd import fpt  # noqa: E402
from paper_2410_13683_amd import runner  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _grad(ctx, w, n, off, tail_lo, noalloc):
    g = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    G = torch.zeros(w.grid_n[0] * w.grid_n[1], dtype=torch.float64, device="cuda")
    J, n_tail = ctx.mlp_grad(n, w.dN, w.seed, tail_lo, g, traj_offset=off, d_G=G, noalloc=noalloc,
                             objective=fpt.FPT_MLP_OBJ_LOG_J)
    torch.cuda.synchronize()
    return J, n_tail, G.cpu().numpy(), g.cpu().numpy()


def test_noalloc_gradient_equals_allocating_entry_point():
    w = W.exponential_ig_learned(n_traj=4000, seed=31, dN=2e-3,
                                 params=W.mlp_random(12, scale=0.2, out_bias=1.0))
    ctx = runner.context_for(w)
    tail_lo = 0.0                                   # deltaN >= 0: about half the paths
    for n, off in ((4000, 0), (1500, 10_000)):
        say(f"no-alloc gradient: n={n} offset={off}")
        ref = _grad(ctx, w, n, off, tail_lo, noalloc=False)
        got = _grad(ctx, w, n, off, tail_lo, noalloc=True)
        assert got[1] == ref[1] and ref[1] > 100
        assert abs(got[0] / ref[0] - 1.0) < 1e-12
        np.testing.assert_allclose(got[2], ref[2], rtol=1e-10, atol=1e-13 * np.abs(ref[2]).max())
        np.testing.assert_allclose(got[3], ref[3], rtol=2e-6, atol=1e-7 * np.abs(ref[3]).max())
        assert np.count_nonzero(ref[3]) > 4000
    with pytest.raises(fpt.FptError):
        _grad(ctx, w, fpt.FPT_MLP_GRAD_NOALLOC_MAX + 1, 0, tail_lo, noalloc=True)
    ctx.destroy()
