"""Batched analysis + synthesis captured in one HIP graph: every replay, with
eager work between replays, equals the eager calls bit for bit; the
autotuner returns a valid, timed choice."""
import numpy as np
import pytest

from workloads import PRESETS, pink_plus_tones

pytestmark = pytest.mark.gpu


def c3_kw():
    p = PRESETS["c3"]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


def test_graph_replays_equal_eager(dev):
    import torch
    import paper_1210_0084_amd as sq
    from paper_1210_0084_amd.tuning import BatchGraph
    plan = sq.Plan(**c3_kw())
    lens = [50000, 0, 123457, 70000, 1]
    lay = plan.batch_layout(lens)
    g = np.random.default_rng(3)
    x = torch.tensor(np.concatenate([pink_plus_tones(n, 44100.0, 40 + i) for i, n in enumerate(lens)]),
                     dtype=torch.float32, device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    graph = BatchGraph(plan, x, coef, y, lay)
    for r in range(4):
        x.copy_(torch.tensor(g.standard_normal(x.numel()), dtype=torch.float32, device=dev))
        graph.replay()
        torch.cuda.synchronize()
        gc, gy = coef.clone(), y.clone()
        ce = plan.analyze_batched(x, layout=lay)          # eager work between replays
        ye = plan.synthesize_batched(ce, layout=lay)
        torch.cuda.synchronize()
        assert torch.equal(gc, ce) and torch.equal(gy, ye), r
        assert (gy - x).abs().max().item() < 1e-4


def test_graph_survives_larger_eager_calls(dev):
    # the graph owns its workspace: an eager call on the same plan that needs a
    # larger workspace (and replaces the plan's own) leaves replays unchanged
    import torch
    import paper_1210_0084_amd as sq
    from paper_1210_0084_amd.tuning import BatchGraph
    plan = sq.Plan(**c3_kw())
    lens = [60000, 90001]
    lay = plan.batch_layout(lens)
    x = torch.tensor(np.concatenate([pink_plus_tones(n, 44100.0, 80 + i) for i, n in enumerate(lens)]),
                     dtype=torch.float32, device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    graph = BatchGraph(plan, x, coef, y, lay)
    graph.replay()
    torch.cuda.synchronize()
    c0, y0 = coef.clone(), y.clone()
    big = torch.tensor(pink_plus_tones(2_000_000, 44100.0, 99), dtype=torch.float32, device=dev)
    for _ in range(2):
        cb = plan.analyze(big)                      # grows the plan's workspace
        yb = plan.synthesize(cb, big.numel())
        coef.zero_()
        y.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(coef, c0) and torch.equal(y, y0)
        assert (yb - big).abs().max().item() < 1e-4


def test_autotuner_picks_a_valid_option(dev, tmp_path):
    import paper_1210_0084_amd as sq
    from paper_1210_0084_amd.tuning import autotune
    kw = c3_kw()
    cache = str(tmp_path / "tune.json")
    cands = [dict(group_cap=1024, pass_cap=4096, lds_cap=9216, layout="band"),
             dict(group_cap=2048, pass_cap=4096, lds_cap=9216, layout="band")]
    best = autotune(kw, [200000, 300000], "f32", cache=cache, reps=2, candidates=cands)
    assert best["options"] in cands and best["ms"] > 0 and len(best["all"]) == 2
    again = autotune(kw, [200000, 300000], "f32", cache=cache, reps=2, candidates=cands)
    assert again == best
    sq.Plan(**kw, **best["options"])
