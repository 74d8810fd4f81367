"""Streaming service on the GPU: per-slice coefficients against the oracle's
linear (streaming) analysis, reconstruction, identical results alone and in
the mix, admission by memory budget, snapshot/restore, gaps and closing."""
import numpy as np
import pytest

from oracle import OraclePlan, analyze_stream
from workloads import PRESETS, pink_plus_tones

pytestmark = pytest.mark.gpu


def c5_kw():
    p = PRESETS["c5"]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


@pytest.fixture(scope="module")
def sq():
    import paper_1210_0084_amd as m
    return m


@pytest.fixture(scope="module")
def plan(sq, dev):
    return sq.Plan(**c5_kw(), layout="slice")


HOP = 4096


def feed(server, ids, signals, hop=HOP, coefs_of=None):
    """Round-robin hops, one tick per round, then a zero flush; returns outputs
    (first T samples of each stream) and, for stream coefs_of, {m: c^m}."""
    plan = server.plan
    flush = plan.N + plan.transition
    outs = {i: [] for i in ids}
    caps = {}
    fed = {i: 0 for i in ids}
    total = {i: len(s) + flush for i, s in zip(ids, signals)}
    sig = dict(zip(ids, signals))
    while any(fed[i] < total[i] for i in ids):
        for i in ids:
            if fed[i] >= total[i]:
                continue
            n = min(hop, total[i] - fed[i])
            h = np.zeros(n)
            lo, hi = fed[i], min(fed[i] + n, len(sig[i]))
            if hi > lo:
                h[:hi - lo] = sig[i][lo:hi]
            server.push(i, h)
            fed[i] += n
        server.tick()
        if coefs_of is not None:
            m, c = server.last_coefs(coefs_of)
            if m >= 0:
                caps[m] = c
        for i in ids:
            outs[i].append(server.poll(i))
    return {i: np.concatenate(outs[i])[:len(sig[i])] for i in ids}, caps


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_stream_coefficients_and_reconstruction(sq, plan):
    srv = sq.StreamServer(plan, "f32", max_streams=8, max_batch=64)
    sigs = [pink_plus_tones(96000, 48000.0, 5_000_000 + i) for i in range(4)]
    ids = [srv.open() for _ in sigs]
    outs, caps = feed(srv, ids, sigs, coefs_of=ids[0])
    for i, s in zip(ids, sigs):
        assert rel(outs[i], s) <= 1e-5
    opl = OraclePlan(**c5_kw())
    ref = analyze_stream(opl, sigs[0], max(caps) + 1)
    for m, c in caps.items():
        r = np.concatenate([ck[m] for ck in ref])
        assert rel(c, r) <= 1e-5, m
    st = srv.stats()
    assert st["slices"] > 0 and st["latency_count"] > 0 and st["latency_p99_s"] >= st["latency_p50_s"] > 0


def test_alone_equals_in_the_mix_bitwise(sq, plan):
    sigs = [pink_plus_tones(70000 + 3000 * i, 48000.0, 5_000_100 + i) for i in range(6)]
    mix = sq.StreamServer(plan, "f32", max_streams=8, max_batch=64)
    ids = [mix.open() for _ in sigs]
    outs, caps_mix = feed(mix, ids, sigs, coefs_of=ids[3])
    alone = sq.StreamServer(plan, "f32", max_streams=8, max_batch=64)
    a = alone.open()
    out_a, caps_a = feed(alone, [a], [sigs[3]], coefs_of=a)
    assert np.array_equal(out_a[a], outs[ids[3]])
    assert caps_a.keys() == caps_mix.keys()
    for m in caps_a:
        assert np.array_equal(caps_a[m], caps_mix[m])


def test_admission_by_memory_budget(sq, plan):
    # every device buffer counts against the budget: per stream two rings of
    # 4N float32 samples plus its 4N-sample share of the staging buffer (and
    # two 32-byte copy records); fixed: the workspace and coefficients of
    # max_batch slices
    import torch
    probe = sq.StreamServer(plan, "f32", max_streams=1, max_batch=8)
    st0 = probe.stats()
    per, fixed = st0["bytes_per_stream"], st0["fixed_bytes"]
    assert per == 3 * 4 * plan.N * 4 + 64
    assert fixed >= plan.workspace_bytes(0, 8) + 8 * plan.coefs_per_slice * 8
    del probe
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    budget = fixed + 3 * per + per // 2
    srv = sq.StreamServer(plan, "f32", max_streams=16, max_batch=8, hbm_budget_bytes=budget)
    assert srv.stats()["slots"] == 3
    used = before - torch.cuda.mem_get_info()[0]
    # the driver rounds allocations up to its page size: allow 2 MiB per buffer
    assert used <= budget + 8 * (2 << 20), (used, budget)
    with pytest.raises(sq.SlicqBusy):
        sq.StreamServer(plan, "f32", max_streams=16, max_batch=8, hbm_budget_bytes=fixed + per - 1)
    ids = [srv.open() for _ in range(3)]
    with pytest.raises(sq.SlicqBusy):
        srv.open()
    srv.close(ids[1])
    srv.tick()
    assert srv.open() == ids[1]
    st = srv.stats()
    assert st["admitted"] == 4 and st["rejected"] == 1 and st["closed"] == 1


def test_snapshot_restore_bitwise(sq, plan):
    srv = sq.StreamServer(plan, "f32", max_streams=4, max_batch=16)
    x = pink_plus_tones(120000, 48000.0, 5_000_200)
    a = srv.open()
    head = 40960
    for lo in range(0, head, HOP):
        srv.push(a, x[lo:lo + HOP])
        srv.tick()
    first = srv.poll(a)
    blob = srv.snapshot(a)
    rest = x[head:]
    for lo in range(0, len(rest), HOP):
        srv.push(a, rest[lo:lo + HOP])
        srv.tick()
    cont = srv.poll(a)
    b = srv.open()
    srv.restore(b, blob)
    for lo in range(0, len(rest), HOP):
        srv.push(b, rest[lo:lo + HOP])
        srv.tick()
    replay = srv.poll(b)
    assert len(first) > 0 and np.array_equal(cont, replay)


def test_gap_and_close_midstream(sq, plan):
    srv = sq.StreamServer(plan, "f32", max_streams=2, max_batch=16)
    x = pink_plus_tones(90000, 48000.0, 5_000_300)
    a = srv.open()
    expect = x.copy()
    fed = 0
    out = []
    for k in range(0, len(x) // HOP):
        if k == 5:
            srv.push_gap(a, HOP)               # the hop never arrived
            expect[fed:fed + HOP] = 0.0
        else:
            srv.push(a, x[fed:fed + HOP])
        fed += HOP
        srv.tick()
        out.append(srv.poll(a))
    y = np.concatenate(out)
    assert len(y) > 6 * HOP
    assert rel(y, expect[:len(y)]) <= 1e-5
    assert srv.stats()["gap_samples"] == HOP
    srv.close(a)                               # mid-slice: queued input is dropped
    srv.tick()
    b = srv.open()
    z = pink_plus_tones(50000, 48000.0, 5_000_301)
    outs, _ = feed(srv, [b], [z])
    assert rel(outs[b], z) <= 1e-5


def test_push_many_and_poll_many_match_single_calls(sq, plan):
    # a whole round of hops in one call gives the same output as one call per stream
    sigs = [pink_plus_tones(60000 + 1000 * i, 48000.0, 5_000_400 + i) for i in range(5)]
    one = sq.StreamServer(plan, "f32", max_streams=8, max_batch=64)
    ids1 = [one.open() for _ in sigs]
    ref, _ = feed(one, ids1, sigs)
    many = sq.StreamServer(plan, "f32", max_streams=8, max_batch=64)
    ids = [many.open() for _ in sigs]
    flush = plan.N + plan.transition
    total = [len(s) + flush for s in sigs]
    fed = [0] * len(sigs)
    outs = [[] for _ in sigs]
    while any(f < t for f, t in zip(fed, total)):
        live, hops = [], []
        for i, s in enumerate(sigs):
            if fed[i] >= total[i]:
                continue
            n = min(HOP, total[i] - fed[i])
            h = np.zeros(n)
            lo, hi = fed[i], min(fed[i] + n, len(s))
            if hi > lo:
                h[:hi - lo] = s[lo:hi]
            live.append(ids[i])
            hops.append(h)
            fed[i] += n
        many.push_many(live, hops)
        many.tick()
        for i, y in zip(range(len(sigs)), many.poll_many(ids)):
            outs[i].append(y.copy())
    for i, s in enumerate(sigs):
        y = np.concatenate(outs[i])[:len(s)]
        assert np.array_equal(y, ref[ids1[i]])
    with pytest.raises(sq.SlicqError):
        many.push_many([ids[0], 99], [np.zeros(4), np.zeros(4)])   # 99 is not open: nothing is appended


def test_churn_alone_equals_in_a_large_mix_bitwise(sq, plan):
    # 64 streams, with streams closing and new ones opening mid-run: a
    # stream's output and coefficients are bit-identical alone and in the mix
    rng = np.random.default_rng(11)
    mix = sq.StreamServer(plan, "f32", max_streams=80, max_batch=256)
    n0 = 64
    lens = [int(rng.integers(30000, 60000)) for _ in range(n0 + 8)]
    sigs = [pink_plus_tones(n, 48000.0, 5_001_000 + i) for i, n in enumerate(lens)]
    flush = plan.N + plan.transition
    ids = {i: mix.open() for i in range(n0)}
    fed = {i: 0 for i in ids}
    outs = {i: [] for i in ids}
    watch = 3                                   # compared alone below
    caps_mix = {}
    late = list(range(n0, n0 + 8))
    closed = set()
    rnd = 0
    while any(fed[i] < lens[i] + flush for i in ids if i not in closed):
        rnd += 1
        if rnd == 4:                            # churn: close 8 streams, open 8 new ones
            for i in range(10, 18):
                mix.close(ids[i])
                closed.add(i)
            for i in late:
                ids[i] = mix.open()
                fed[i] = 0
                outs[i] = []
        for i, sid in ids.items():
            if i in closed or fed[i] >= lens[i] + flush:
                continue
            h = np.zeros(HOP)
            lo, hi = fed[i], min(fed[i] + HOP, lens[i])
            if hi > lo:
                h[:hi - lo] = sigs[i][lo:hi]
            mix.push(sid, h)
            fed[i] += HOP
        mix.tick()
        m, c = mix.last_coefs(ids[watch])
        if m >= 0:
            caps_mix[m] = c
        for i, sid in ids.items():
            if i not in closed:
                outs[i].append(mix.poll(sid))
    for i in [watch, n0 + 2]:                   # one stream from the start, one opened mid-run
        alone = sq.StreamServer(plan, "f32", max_streams=2, max_batch=16)
        a = alone.open()
        out_a, caps_a = feed(alone, [a], [sigs[i]], coefs_of=a if i == watch else None)
        y = np.concatenate(outs[i])[:lens[i]]
        assert np.array_equal(out_a[a], y), i
        if i == watch:
            assert caps_a.keys() == caps_mix.keys()
            for m in caps_a:
                assert np.array_equal(caps_a[m], caps_mix[m])
    assert rel(np.concatenate(outs[n0 + 5])[:lens[n0 + 5]], sigs[n0 + 5]) <= 1e-5


def test_full_size_service_sampled(sq, plan):
    # the bench's service configuration (512 streams, 576 slots, batches of up
    # to 1024 slices), every stream fed 0.5 s: every stream reconstructs its
    # input, and one stream's coefficients match the oracle's linear analysis
    srv = sq.StreamServer(plan, "f32", max_streams=576, max_batch=1024)
    sigs = [pink_plus_tones(24000, 48000.0, 5_000_000 + i) for i in range(512)]
    ids = [srv.open() for _ in sigs]
    outs, caps = feed(srv, ids, sigs, coefs_of=ids[300])
    worst = max(rel(outs[i], s) for i, s in zip(ids, sigs))
    print(f"512 streams: worst reconstruction rel-L2 {worst:.2e}", flush=True)
    assert worst <= 1e-5
    opl = OraclePlan(**c5_kw())
    ref = analyze_stream(opl, sigs[300], max(caps) + 1)
    for m, c in caps.items():
        r = np.concatenate([ck[m] for ck in ref])
        assert rel(c, r) <= 1e-5, m
