"""GPU tests of the batched persistent launch (many instances in one kernel),
its hipGraph replay and the autotuner: every instance's histogram must equal the
one a single-context fpt_run produces for the same seed and trajectories
(counts and step totals exactly; FP64 sums up to the order of atomic adds)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2410_13683_amd import fpt  # noqa: E402
from paper_2410_13683_amd import runner  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _instances(precision):
    ws = [
        W.srusr_bessel(seed=0).with_(bias_kind=W.BIAS_CONST, A_bias=1.5, extra={"instance": 3}),
        W.linear_slow_roll().with_(extra={"instance": 1}),
        W.exponential_ig(dN=1e-3).with_(extra={"instance": 7}, bias_kind=W.BIAS_CONST, A_bias=0.7),
        W.srusr_bessel().with_(A_minus=W.V0 * 2e-4, phi_end=-0.05, n_bins=32, lo=-0.5, hi=0.5,
                               extra={"instance": 2}),
        W.srusr_bessel().with_(max_steps=40_000, extra={"instance": 5}),   # all censored
    ]
    return [w.with_(precision=precision) for w in ws]


def _compare(h_batch, h_single):
    assert h_batch["n_traj"] == h_single["n_traj"]
    for k in ("n_censored", "n_ended_early", "n_steps_total"):
        assert h_batch[k] == h_single[k], k
    assert np.array_equal(h_batch["count"], h_single["count"])
    for k in ("sum_w", "sum_w2", "sum_lnw", "sum_lnw2"):
        np.testing.assert_allclose(h_batch[k], h_single[k], rtol=1e-11, atol=1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_runs(precision):
    ws = _instances(precision)
    counts = [3000, 1500, 2600, 700, 400]
    seed, dN_of = 99, [w.dN for w in ws]
    assert len(set(dN_of)) > 1
    # one dN per batch: run the batch per distinct dN group
    for dN in sorted(set(dN_of)):
        group = [i for i, w in enumerate(ws) if w.dN == dN]
        say(f"batch prec={precision} dN={dN} instances={group}")
        singles = []
        for i in group:
            c = runner.context_for(ws[i])
            c.run(counts[i], dN, seed, 0, torch.cuda.current_stream())
            singles.append(c.histogram())
            c.destroy()
        ctxs = [runner.context_for(ws[i]) for i in group]
        b = fpt.Batch(ctxs, block_size=256, item_size=512, use_graph=False)
        b.run([counts[i] for i in group], dN, seed, 0, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for c, hs in zip(ctxs, singles):
            _compare(c.histogram(), hs)
        b.destroy()
        for c in ctxs:
            c.destroy()


def test_graph_replays_match_eager_runs():
    """Capture on a side stream, replay with new seeds, offsets and counts; each replay's
    accumulated histograms equal eager single runs."""
    ws = [w for w in _instances(1) if w.dN == 1e-4]
    stream = torch.cuda.Stream()
    ctxs = [runner.context_for(w) for w in ws]
    b = fpt.Batch(ctxs, use_graph=True)
    ref = [runner.context_for(w) for w in ws]
    plan = [(5, 0, [900, 400, 300]), (6, 10_000, [1200, 50, 0]), (7, 20_000, [64, 640, 333])]
    for k, (seed, off, counts) in enumerate(plan):
        say(f"graph replay {k}: seed={seed} offset={off} counts={counts}")
        b.run(counts, 1e-4, seed, off, stream)
        stream.synchronize()
        for c, n in zip(ref, counts):
            c.run(n, 1e-4, seed, off, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for c, r in zip(ctxs, ref):
            _compare(c.histogram(), r.histogram())
    assert b.last_ms() > 0
    b.destroy()
    for c in ctxs + ref:
        c.destroy()


def test_autotune_picks_a_valid_config_and_caches_it(tmp_path):
    ws = [w for w in _instances(1) if w.dN == 1e-4]
    counts = [4000, 2000, 1000]
    cache = str(tmp_path / "tune.txt")
    ctxs = [runner.context_for(w) for w in ws]
    b = fpt.Batch(ctxs, use_graph=True)
    say("autotune")
    b.autotune(counts, 1e-4, 3, cache, torch.cuda.current_stream())
    blk, chk = b.config()
    assert blk in (256, 512, 1024) and chk in (32, 64, 128, 256)
    line = open(cache).read().split()
    assert line[1:] == [str(blk), str(chk)]
    # tuning left the contexts' histograms untouched
    for c in ctxs:
        assert int(c.histogram()["count"].sum()) == 0
    stream = torch.cuda.Stream()
    b.run(counts, 1e-4, 3, 0, stream)
    stream.synchronize()
    for w, c, n in zip(ws, ctxs, counts):
        r = runner.context_for(w)
        r.run(n, 1e-4, 3, 0, torch.cuda.current_stream())
        _compare(c.histogram(), r.histogram())
        r.destroy()
    b2 = fpt.Batch(ctxs, use_graph=False)
    b2.autotune(counts, 1e-4, 3, cache, torch.cuda.current_stream())
    assert b2.config() == (blk, chk)
    b.destroy()
    b2.destroy()
    for c in ctxs:
        c.destroy()


def test_batched_instances_workload_totals():
    """The 64-instance workload (scaled counts): every trajectory is binned, censored or ended."""
    ws = W.batched_instances(n_min=200, n_max=2000, max_steps=1 << 14)
    ws = [w.with_(precision=1) for w in ws]
    ctxs = [runner.context_for(w) for w in ws]
    b = fpt.Batch(ctxs, use_graph=True)
    stream = torch.cuda.Stream()
    counts = [w.n_traj for w in ws]
    say(f"64 instances, {sum(counts)} trajectories")
    b.run(counts, 1e-4, 4, 0, stream)
    stream.synchronize()
    for c, n in zip(ctxs, counts):
        h = c.histogram()
        assert h["n_traj"] == n
        assert int(h["count"].sum()) + h["n_censored"] + h["n_ended_early"] == n
    b.destroy()
    for c in ctxs:
        c.destroy()


def test_bench_batched_configuration_matches_single_runs(tmp_path):
    """The bench's batched configuration as it times it (64 FP32 instances, trajectory counts scaled
    by 0.1, step cap 2^20, autotuned, hipGraph): one pass, then four instances (the largest, the
    smallest, the most censored and the median) rerun as single-context launches over the same
    trajectories give the same histograms."""
    ws = [w.with_(precision=1) for w in W.batched_instances()]
    counts = np.array([max(1, int(round(w.n_traj * 0.1))) for w in ws], dtype=np.uint64)
    ctxs = [runner.context_for(w) for w in ws]
    stream = torch.cuda.Stream()
    b = fpt.Batch(ctxs, use_graph=True)
    dN, seed, off = ws[0].dN, ws[0].seed, 1 << 32
    b.autotune(counts, dN, seed, cache_path=str(tmp_path / "tune.txt"), stream=stream)
    say(f"bench batch configuration: {int(counts.sum())} trajectories, config {b.config()}")
    for c in ctxs:
        c.reset()
    b.run(counts, dN, seed, off, stream)
    stream.synchronize()
    hb = [c.histogram() for c in ctxs]
    for c, n, h in zip(ctxs, counts, hb):
        assert h["n_traj"] == n and int(h["count"].sum()) + h["n_censored"] + h["n_ended_early"] == n
    cens = [h["n_censored"] / h["n_traj"] for h in hb]
    pick = sorted({int(np.argmax(counts)), int(np.argmin(counts)), int(np.argmax(cens)),
                   int(np.argsort(counts)[len(counts) // 2])})
    assert max(cens) > 0                        # the step cap is exercised
    for i in pick:
        ctxs[i].reset()
        ctxs[i].run(int(counts[i]), dN, seed, off, None)
        torch.cuda.synchronize()
        _compare(hb[i], ctxs[i].histogram())
    say(f"  instances {pick} equal to single launches")
    b.destroy()
    for c in ctxs:
        c.destroy()
