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


def test_batch_equals_single_runs_with_eps1_ends_on_a_phi_table():
    """FP32 state, constant bias A = 1, on a smooth 256-node phi table where every path starts at
    |pi| = 1 and ends at eps_1 = 1 (|pi| = sqrt 2) about 200 steps later (exponential potential,
    V'/V = 2, dN = 1e-3): its groups run on the table record both with the end test (near sqrt 2)
    and without it (the early groups, whose lanes the bound clears).  Batched with a single-node
    instance of the same dN, the histogram must equal the single launch's."""
    lo, hi, n_nodes = 0.4, 1.2, 256
    phi = np.linspace(lo, hi, n_nodes)
    S = 2e-3 * (1.0 + 0.3 * (phi - 0.8))
    t = 0.05 + 0.05 * phi
    w = W.exponential_ig(seed=21, alpha=2.0, S=0.0, delta_phi=1.0, dN=1e-3).with_(
        pi_in=-1.0, precision=1, bias_kind=W.BIAS_CONST, A_bias=1.0)
    other = W.exponential_ig(dN=1e-3).with_(precision=1, extra={"instance": 7}, bias_kind=W.BIAS_CONST, A_bias=0.7)
    assert other.dN == w.dN
    pot = fpt.make_potential(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.phi_in, w.pi_in, w.phi_end)

    def eps1_ctx():
        return fpt.Context(pot, S, t, lo, hi, bias_kind=w.bias_kind, A=w.A_bias, precision=1,
                           bins_kind=w.bins_kind, n_bins=w.n_bins, lo=w.lo, hi=w.hi, N_ref=w.N_ref,
                           max_steps=w.max_steps)

    counts, seed = [3000, 1000], 123
    say(f"batch fp32 eps_1 ends on a phi table, counts {counts}")
    singles = []
    for make, n in ((eps1_ctx, counts[0]), (lambda: runner.context_for(other), counts[1])):
        c = make()
        c.run(n, w.dN, seed, 0, torch.cuda.current_stream())
        singles.append(c.histogram())
        c.destroy()
    assert singles[0]["n_ended_early"] == counts[0]
    ctxs = [eps1_ctx(), runner.context_for(other)]
    b = fpt.Batch(ctxs, block_size=256, item_size=512, use_graph=False)
    b.run(counts, w.dN, seed, 0, torch.cuda.current_stream())
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


@pytest.mark.parametrize("use_graph", [False, True])
def test_more_instances_than_blocks(use_graph):
    """300 instances (more than the resident blocks, so blocks take several instances and, once the
    tickets are used up, join instances that still have trajectories), counts from 0 to 20000 with
    one large instance: every instance's totals add up, and a sample of instances (the large one,
    small ones, one with a single trajectory) equals single-context launches over the same
    trajectories."""
    rng = np.random.default_rng(12)
    n_inst = 300
    ws = [W.linear_slow_roll(seed=3).with_(extra={"instance": 100 + i}, precision=1) for i in range(n_inst)]
    counts = rng.integers(0, 200, n_inst)
    counts[7], counts[11], counts[13] = 20_000, 1, 0
    ctxs = [runner.context_for(w) for w in ws]
    b = fpt.Batch(ctxs, block_size=256, item_size=256, use_graph=use_graph)
    stream = torch.cuda.Stream()
    say(f"{n_inst} instances, {int(counts.sum())} trajectories, graph {use_graph}")
    b.run(counts.astype(np.uint64), 1e-3, 21, 5000, stream)
    stream.synchronize()
    hb = [c.histogram() for c in ctxs]
    for h, n in zip(hb, counts):
        assert h["n_traj"] == n and int(h["count"].sum()) + h["n_censored"] + h["n_ended_early"] == n
    for i in (7, 11, 13, 0, 150, 299):
        r = runner.context_for(ws[i])
        r.run(int(counts[i]), 1e-3, 21, 5000, torch.cuda.current_stream())
        _compare(hb[i], r.histogram())
        r.destroy()
    b.destroy()
    for c in ctxs:
        c.destroy()


def test_batch_with_no_trajectories():
    """All counts zero: the run launches nothing and leaves every histogram empty; a later run
    with counts still works (the graph is captured then)."""
    ws = [w for w in _instances(1) if w.dN == 1e-4]
    ctxs = [runner.context_for(w) for w in ws]
    b = fpt.Batch(ctxs, use_graph=True)
    stream = torch.cuda.Stream()
    b.run([0] * len(ws), 1e-4, 5, 0, stream)
    stream.synchronize()
    for c in ctxs:
        h = c.histogram()
        assert h["n_traj"] == 0 and int(h["count"].sum()) == 0 and h["n_steps_total"] == 0
    b.run([100] * len(ws), 1e-4, 5, 0, stream)
    stream.synchronize()
    for c in ctxs:
        h = c.histogram()
        assert h["n_traj"] == 100 and int(h["count"].sum()) + h["n_censored"] + h["n_ended_early"] == 100
    b.destroy()
    for c in ctxs:
        c.destroy()


def _ks_binned(ca, cb):
    """KS distance of two binned laws (cumulative masses compared at every slot edge)."""
    fa, fb = np.cumsum(ca) / np.sum(ca), np.cumsum(cb) / np.sum(cb)
    return float(np.max(np.abs(fa - fb)))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_oracle(precision):
    """The batched kernel against the CPU oracle (not against single-context runs): the instances
    of _instances (a biased SR -> USR run, the linear problem, a biased inverse-Gaussian companion
    at another dN, a second SR -> USR potential, an all-censored instance) plus one instance of the
    64-instance workload under its own step cap, at most 3e3 trajectories each.  FP64: each
    instance's histogram equals the oracle's histogram of the oracle's own trajectories (counts
    exactly up to 2 bin-edge near-ties, sums to 1e-9, censored and step totals).  FP32 (coupled
    streams, the FP32 rounding only): the same censoring; for the SR -> USR instances the binned
    law of deltaN and the weighted binned law within KS 1e-3 of the oracle's.  The linear and
    inverse-Gaussian problems spread N by only 2.5e-6 of its value, less than the FP32 state's
    rounding of the drift over a path (a few 1e-7 of N): there the weighted mean of N must agree
    within 1e-6 relative and the KS bar does not apply."""
    from oracle import oracle as orc
    from tests._glue import oracle_run
    ws = _instances(precision)
    counts = [3000, 1500, 2600, 700, 400]
    wb = min(W.batched_instances(), key=lambda w: -w.extra["eps_minus"])    # shortest runs
    ws.append(wb.with_(precision=precision, max_steps=1 << 16))
    counts.append(500)
    seed, off = 1234, 77
    for dN in sorted({w.dN for w in ws}):
        group = [i for i, w in enumerate(ws) if w.dN == dN]
        say(f"batch vs oracle prec={precision} dN={dN} instances={group}")
        ctxs = [runner.context_for(ws[i]) for i in group]
        b = fpt.Batch(ctxs, block_size=256, item_size=512, use_graph=False)
        b.run([counts[i] for i in group], dN, seed, off, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for i, c in zip(group, ctxs):
            w = ws[i].with_(seed=seed)
            hb = c.histogram()
            N, lnw, st = oracle_run(w, n_traj=counts[i], traj_offset=off)
            ho = orc.histogram(N, lnw, st, w.N_ref, w.bins_kind, w.n_bins, w.lo, w.hi)
            assert hb["n_traj"] == ho["n_traj"] and hb["n_censored"] == ho["n_censored"], i
            assert hb["n_ended_early"] == ho["n_ended_early"], i
            cb, co = hb["count"].astype(np.int64), ho["count"].astype(np.int64)
            if precision == 0:
                assert np.abs(cb - co).sum() <= 2, (i, np.abs(cb - co).sum())
                assert abs(int(hb["n_steps_total"]) - int(ho["n_steps_total"])) <= 2, i
                same = cb == co
                np.testing.assert_allclose(hb["sum_w"][same], ho["sum_w"][same], rtol=1e-9, atol=1e-300)
                np.testing.assert_allclose(hb["sum_lnw"][same], ho["sum_lnw"][same], rtol=1e-9, atol=1e-9)
            elif cb.sum() > 0:
                mean_b = hb["sum_wN"] / hb["sum_w_total"]
                mean_o = ho["sum_wN"] / ho["sum_w_total"]
                ks = _ks_binned(cb, co)
                ksw = _ks_binned(hb["sum_w"], ho["sum_w"])
                say(f"  instance {i}: KS {ks:.2e}, weighted KS {ksw:.2e}, mean N rel. diff "
                    f"{abs(mean_b / mean_o - 1):.1e}")
                assert abs(mean_b / mean_o - 1.0) < 1e-6, (i, mean_b, mean_o)
                if ws[i].name.startswith(("srusr", "batched")):
                    assert ks < 1e-3 and ksw < 1e-3, (i, ks, ksw)
            say(f"  instance {i}: {int(cb.sum())} binned, {hb['n_censored']} censored, equal to the oracle")
        b.destroy()
        for c in ctxs:
            c.destroy()
