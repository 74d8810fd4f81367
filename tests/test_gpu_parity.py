"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative L2 over all stored coefficients / all output samples):
FP32 1e-5 and FP64 1e-12 for coefficients, reconstruction and adjoint.
Every coefficient check also bounds the worst band: the relative L2 of each
band k over its S x M_k coefficients stays within BAND_TOL (1e-4 FP32,
1e-10 FP64), so a wrong low-energy band cannot hide behind the global norm.
"""
import numpy as np
import pytest

from oracle import OraclePlan, analyze, synthesize, adjoint, pack, unpack, num_slices
from workloads import PRESETS, noise_plus_sines, pink_plus_tones

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
BAND_TOL = {"f32": 1e-4, "f64": 1e-10}
TINY = dict(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0)
TINY2 = dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)


def preset(name):
    p = PRESETS[name]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0)


def worst_band(opl, got, ref, S):
    """Largest per-band relative L2 error of band-major packed coefficients
    (band k occupies [S off_k, S off_k + S M_k)); bands that are zero in the
    reference are compared by their absolute error against the global norm."""
    got = np.asarray(got)
    scale = np.linalg.norm(ref) / np.sqrt(max(len(ref), 1))
    worst = 0.0
    for off, b in zip(opl.offsets, opl.bands):
        sl = slice(S * off, S * (off + b.M))
        nb = np.linalg.norm(ref[sl])
        den = nb if nb > 1e-3 * scale * np.sqrt(S * b.M) else scale * np.sqrt(S * b.M)
        if den > 0:
            worst = max(worst, np.linalg.norm(got[sl] - ref[sl]) / den)
    return worst


def check_coefs(opl, got, ref, S, dt, tol=None):
    e, eb = rel(got, ref), worst_band(opl, got, ref, S)
    assert e <= (tol or TOL[dt]), ("global", e)
    assert eb <= BAND_TOL[dt], ("worst band", eb)
    return e, eb


@pytest.fixture(scope="module")
def sq():
    import paper_1210_0084_amd as m
    return m


def torch_dtype(name):
    import torch
    return torch.float32 if name == "f32" else torch.float64


_plans = {}


def gpu_plan(sq, kw):
    key = tuple(sorted(kw.items()))
    if key not in _plans:
        okw = {k: v for k, v in kw.items() if k != "fused"}
        _plans[key] = (sq.Plan(**kw), OraclePlan(**okw))
    return _plans[key]


def check_roundtrip(sq, dev, kw, x, dt, check_adjoint=True, seed=0):
    import torch
    plan, opl = gpu_plan(sq, kw)
    T = len(x)
    print(f"case 2N={kw['slice_len']} B={kw['bins_per_octave']} T={T} {dt}", flush=True)
    ref = pack(opl, analyze(opl, x))
    xd = torch.tensor(x, dtype=torch_dtype(dt), device=dev)
    c = plan.analyze(xd)
    y = plan.synthesize(c, T)
    torch.cuda.synchronize()
    S = num_slices(T, opl.two_n)
    check_coefs(opl, c.cpu().numpy(), ref, S, dt)
    assert rel(y.cpu().numpy(), x) <= TOL[dt], rel(y.cpu().numpy(), x)
    if check_adjoint and T > 0:
        g = np.random.default_rng(seed)
        cr = g.standard_normal(len(ref)) + 1j * g.standard_normal(len(ref))
        ctype = torch.complex64 if dt == "f32" else torch.complex128
        crd = torch.tensor(cr, dtype=ctype, device=dev)
        ya = plan.adjoint(crd, T).cpu().numpy()
        ys = plan.synthesize(crd, T).cpu().numpy()
        assert rel(ya, adjoint(opl, unpack(opl, cr, S), T)) <= TOL[dt]
        assert rel(ys, synthesize(opl, unpack(opl, cr, S), T)) <= TOL[dt]
    return c


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("T", [1, 63, 64, 65, 128, 300, 1000])
@pytest.mark.parametrize("kw", [TINY, TINY2], ids=["tiny64", "tiny128"])
def test_tiny_plans(sq, dev, kw, T, dt):
    x = np.random.default_rng(T).standard_normal(T)
    check_roundtrip(sq, dev, kw, x, dt, seed=T)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_c1_full(sq, dev, dt):
    from workloads import make_c1
    check_roundtrip(sq, dev, preset("c1"), make_c1(), dt)


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "pipeline"])
@pytest.mark.parametrize("name,T", [("c3", 100000), ("c4", 264600), ("c5", 60000), ("c2", 150000)])
def test_preset_shapes_f32(sq, dev, name, T, fused):
    # fused: one workgroup per slice where the half spectrum fits in LDS (2N <=
    # 32768 in FP32); pipeline: the multi-kernel path (the only one for c2)
    p = PRESETS[name]
    x = pink_plus_tones(T, p.fs, 77) if name != "c4" else noise_plus_sines(T, p.fs, 5)
    kw = dict(preset(name), fused=fused)
    plan, _ = gpu_plan(sq, kw)
    assert (0 in plan.fused_dtypes) == (fused and name != "c2")
    check_roundtrip(sq, dev, kw, x, "f32", check_adjoint=(name in ("c4", "c5")))


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("name,T", [("c2", 150000), ("c5", 60000), ("c3", 100000)])
def test_smooth_policy_presets(sq, dev, name, T, dt):
    # M_k the smallest even 2^a, 3 2^a or 5 2^a (radix-3/5 band transforms,
    # fractional hops): coefficients per band, reconstruction, adjoint and
    # synthesis of random coefficients against the oracle
    p = PRESETS[name]
    kw = dict(preset(name), m_policy="smooth")
    plan, opl = gpu_plan(sq, kw)
    assert any(m % 3 == 0 or m % 5 == 0 for m in plan.M)
    x = pink_plus_tones(T, p.fs, 78)
    check_roundtrip(sq, dev, kw, x, dt)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("T", [1, 63, 64, 65, 300, 1000])
def test_smooth_policy_tiny(sq, dev, T, dt):
    kw = dict(TINY2, m_policy="smooth")
    x = np.random.default_rng(T + 7).standard_normal(T)
    check_roundtrip(sq, dev, kw, x, dt, seed=T)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_fused_and_pipeline_agree(sq, dev, dt):
    # the two kernel paths compute the same transform (to rounding): 2N = 8192
    # fits one workgroup in both FP32 and FP64
    import torch
    kw = preset("c1")
    fused = sq.Plan(**kw, fused=True)
    pipe = sq.Plan(**kw, fused=False)
    assert {0, 1} <= fused.fused_dtypes and not pipe.fused_dtypes
    x = torch.tensor(noise_plus_sines(50000, 44100.0, 12), dtype=torch_dtype(dt), device=dev)
    cf, cp = fused.analyze(x), pipe.analyze(x)
    yf, yp = fused.synthesize(cf, 50000), pipe.synthesize(cp, 50000)
    af, ap = fused.adjoint(cf, 50000), pipe.adjoint(cp, 50000)
    torch.cuda.synchronize()
    t = TOL[dt]
    assert rel(cf.cpu().numpy(), cp.cpu().numpy()) <= t
    assert rel(yf.cpu().numpy(), yp.cpu().numpy()) <= t
    assert rel(af.cpu().numpy(), ap.cpu().numpy()) <= t


OPTION_SETS = [
    dict(group_cap=64, lds_cap=512, pass_cap=256),        # many small items; large synthesis items alone
    dict(group_cap=4096, lds_cap=16384, pass_cap=1024),   # the largest items; wide slice-pass items
    dict(group_cap=512, lds_cap=2048, pass_cap=4096, layout="slice"),
]


@pytest.mark.parametrize("opts", OPTION_SETS, ids=["small", "large", "slice-major"])
@pytest.mark.parametrize("name,T,dt", [("c4", 100000, "f32"), ("c5", 60000, "f32"), ("c1", 70000, "f64")])
def test_tuning_options(sq, dev, opts, name, T, dt):
    # every work-item decomposition gives the oracle's coefficients (in its layout),
    # reconstruction and adjoint
    import torch
    kw = preset(name)
    _, opl = gpu_plan(sq, kw)
    plan = sq.Plan(**kw, **opts, fused=False)     # the options cut the pipeline's work items
    print(f"case {name} T={T} {dt} {opts}", flush=True)
    x = pink_plus_tones(T, kw["fs"], 91)
    c_ref = analyze(opl, x)
    S = num_slices(T, opl.two_n)
    slice_major = opts.get("layout") == "slice"
    ref = (np.concatenate([np.concatenate([ck[m] for ck in c_ref]) for m in range(S)]) if slice_major
           else pack(opl, c_ref))
    xd = torch.tensor(x, dtype=torch_dtype(dt), device=dev)
    c = plan.analyze(xd)
    y = plan.synthesize(c, T)
    if slice_major:
        assert rel(c.cpu().numpy(), ref) <= TOL[dt]
        check_coefs(opl, plan.to_band_major(c, S).cpu().numpy(), pack(opl, c_ref), S, dt)
    else:
        check_coefs(opl, c.cpu().numpy(), ref, S, dt)
    assert rel(y.cpu().numpy(), x) <= TOL[dt]
    if not slice_major:
        g = np.random.default_rng(5)
        cr = g.standard_normal(len(ref)) + 1j * g.standard_normal(len(ref))
        crd = torch.tensor(cr, dtype=torch.complex64 if dt == "f32" else torch.complex128, device=dev)
        assert rel(plan.adjoint(crd, T).cpu().numpy(), adjoint(opl, unpack(opl, cr, S), T)) <= TOL[dt]


def test_c2_full_stereo_f32(sq, dev):
    # the benchmarked workload at its full size: 60 s stereo, batched launch
    import torch
    from workloads import make_c2
    kw = preset("c2")
    plan, opl = gpu_plan(sq, kw)
    xs = make_c2()
    T = xs.shape[1]
    xd = torch.tensor(xs.reshape(-1), dtype=torch.float32, device=dev)
    c = plan.analyze_batched(xd, [T, T])
    y = plan.synthesize_batched(c, [T, T])
    torch.cuda.synchronize()
    cc = c.cpu().numpy()
    half = len(cc) // 2
    S = plan.num_slices(T)
    for ch in range(2):
        ref = pack(opl, analyze(opl, xs[ch]))
        e, eb = check_coefs(opl, cc[ch * half:(ch + 1) * half], ref, S, "f32")
        print(f"c2 channel {ch}: rel-L2 {e:.2e}, worst band {eb:.2e}", flush=True)
    assert rel(y.cpu().numpy(), xs.reshape(-1)) <= 1e-5


def test_c3_full_batch_graph_vs_oracle(sq, dev):
    # the whole ragged batch (256 signals of 5-30 s, 2N = 32768) through one
    # graph replay, as timed: eight signals (the shortest, the longest and six
    # seeded ones) against the oracle band by band, reconstruction of every
    # sample of every signal
    import torch
    from paper_1210_0084_amd.tuning import BatchGraph
    from workloads import make_c3_cut
    kw = preset("c3")
    plan, opl = gpu_plan(sq, kw)
    lens, offs, base = make_c3_cut()
    lay = plan.batch_layout(lens)
    print(f"case c3 full batch: {len(lens)} signals, {sum(lens)} samples, {lay.total_slices} slices", flush=True)
    x = torch.tensor(np.concatenate([base[o:o + t] for o, t in zip(offs, lens)]), dtype=torch.float32, device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    graph = BatchGraph(plan, x, coef, y, lay)
    coef.zero_()
    y.zero_()
    graph.replay()
    torch.cuda.synchronize()
    err = (torch.linalg.vector_norm((y - x).double()) / torch.linalg.vector_norm(x.double())).item()
    assert err <= 1e-5, err
    pick = {int(np.argmin(lens)), int(np.argmax(lens))}
    g = np.random.default_rng(44)
    while len(pick) < 8:
        pick.add(int(g.integers(0, len(lens))))
    for b in sorted(pick):
        xb = x[lay.x_off[b]:lay.x_off[b + 1]].cpu().numpy().astype(np.float64)
        S = int(lay.slices[b])
        got = coef[lay.coef_off[b]:lay.coef_off[b] + S * plan.coefs_per_slice].cpu().numpy()
        e, eb = check_coefs(opl, got, pack(opl, analyze(opl, xb)), S, "f32")
        print(f"signal {b}: T={lens[b]} rel-L2 {e:.2e}, worst band {eb:.2e}", flush=True)


def test_c3_f64_full_slice_length(sq, dev):
    # the FP64 path at 2N = 32768 (four-step slice FFT of 16384 points)
    x = pink_plus_tones(100000, 44100.0, 78)
    check_roundtrip(sq, dev, preset("c3"), x, "f64", check_adjoint=True)


def test_batched_offsets_out_of_range_are_reported(sq, dev):
    # a signal whose samples fall outside x_len is refused by a prepared batch
    # and flagged by the plain batched call (read back by slicq_batched_status)
    import ctypes
    import torch
    plan, _ = gpu_plan(sq, TINY2)
    lib = plan._lib
    P = ctypes.c_void_p
    st = P(torch.cuda.current_stream(dev).cuda_stream)
    x_off = torch.tensor([0, 300, 900], dtype=torch.int64, device=dev)       # second signal ends at 900
    S = [plan.num_slices(300), plan.num_slices(600)]
    c_off = torch.tensor([0, S[0] * plan.coefs_per_slice], dtype=torch.int64, device=dev)
    coef_len = sum(S) * plan.coefs_per_slice
    nb = lib.slicq_batch_tasks_bytes(sum(S))
    tasks = torch.empty(nb, dtype=torch.uint8, device=dev)
    h = P()
    for x_len, want in ((800, -4), (900, 0)):
        rc = lib.slicq_batch_create(plan._h, P(x_off.data_ptr()), P(c_off.data_ptr()), 2, sum(S), x_len, coef_len,
                                    P(tasks.data_ptr()), nb, st, ctypes.byref(h))
        assert rc == want, (x_len, rc)
        if rc == 0:
            lib.slicq_batch_destroy(h)
    # a wrong total_slices is refused too
    assert lib.slicq_batch_create(plan._h, P(x_off.data_ptr()), P(c_off.data_ptr()), 2, sum(S) + 1, 900, coef_len,
                                  P(tasks.data_ptr()), lib.slicq_batch_tasks_bytes(sum(S) + 1), st,
                                  ctypes.byref(h)) == -4
    xp = torch.zeros(900, dtype=torch.float32, device=dev)
    coef = torch.empty(coef_len, dtype=torch.complex64, device=dev)
    plan._ensure_tables(0, dev)
    w, wb = plan._workspace(0, sum(S), dev, None)
    for x_len, want in ((800, -4), (900, 0)):
        rc = lib.slicq_analyze_batched(plan._h, 0, P(xp.data_ptr()), x_len, P(x_off.data_ptr()), 2, sum(S),
                                       P(coef.data_ptr()), coef_len, P(c_off.data_ptr()), P(w.data_ptr()), wb, st)
        assert rc == 0                                # enqueue-only: cannot see device offsets
        bad = ctypes.c_int32()
        n = ctypes.c_int64()
        assert lib.slicq_batched_status(plan._h, 0, sum(S), P(w.data_ptr()), wb, ctypes.byref(bad),
                                        ctypes.byref(n), st) == want
        assert bad.value == (1 if want else 0)
    assert plan.batched_status(0, sum(S), dev) == sum(S)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batch_invariance_bitwise(sq, dev, dt):
    # each signal's result inside a ragged batch equals its single-signal result bit for bit
    import torch
    kw = TINY2
    plan, _ = gpu_plan(sq, kw)
    lens = [300, 0, 128, 1, 777, 64]
    xs = [np.random.default_rng(i + 40).standard_normal(n) for i, n in enumerate(lens)]
    tdt = torch_dtype(dt)
    xp = torch.tensor(np.concatenate(xs), dtype=tdt, device=dev)
    cb = plan.analyze_batched(xp, lens)
    yb = plan.synthesize_batched(cb, lens)
    lay = plan.batch_layout(lens)
    x_off, coef_off = lay.x_off, lay.coef_off
    for i, n in enumerate(lens):
        if n == 0:
            continue
        ci = plan.analyze(torch.tensor(xs[i], dtype=tdt, device=dev))
        yi = plan.synthesize(ci, n)
        assert torch.equal(cb[coef_off[i]:coef_off[i] + ci.numel()], ci)
        assert torch.equal(yb[x_off[i]:x_off[i + 1]], yi)


def test_determinism_bitwise(sq, dev):
    import torch
    kw = preset("c4")
    plan, _ = gpu_plan(sq, kw)
    x = torch.tensor(noise_plus_sines(100000, 44100.0, 3), dtype=torch.float32, device=dev)
    c1 = plan.analyze(x).clone()
    y1 = plan.synthesize(c1, 100000).clone()
    c2 = plan.analyze(x)
    y2 = plan.synthesize(c2, 100000)
    assert torch.equal(c1, c2) and torch.equal(y1, y2)


def test_small_workspace_runs_in_chunks(sq, dev):
    # a workspace for 3 slices processes a 40-slice signal in 14 passes, same result
    import torch
    kw = preset("c5")
    plan, _ = gpu_plan(sq, kw)
    T = 160000
    x = torch.tensor(pink_plus_tones(T, 48000.0, 9), dtype=torch.float32, device=dev)
    S = plan.num_slices(T)
    small = plan.workspace_bytes(0, S) - (S - 3) * (2 * plan.N + 64) * 8
    work = torch.empty(small, dtype=torch.uint8, device=dev)
    c_full = plan.analyze(x).clone()
    y_full = plan.synthesize(c_full, T).clone()
    c_chunk = plan.analyze(x, work=work)
    y_chunk = plan.synthesize(c_chunk, T, work=work)
    assert torch.equal(c_full, c_chunk) and torch.equal(y_full, y_chunk)
    # one slice per pass, two slices: both shared overlaps span two launches
    T2 = plan.N
    x2 = torch.tensor(pink_plus_tones(T2, 48000.0, 10), dtype=torch.float32, device=dev)
    assert plan.num_slices(T2) == 2
    one = plan.workspace_bytes(0, 2) - (2 * plan.N + 64) * 8
    w1 = torch.empty(one, dtype=torch.uint8, device=dev)
    c2 = plan.analyze(x2).clone()
    y2 = plan.synthesize(c2, T2).clone()
    assert torch.equal(plan.synthesize(c2, T2, work=w1), y2)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_prepared_batch_equals_batched_calls(sq, dev, dt):
    # a reused layout runs on its prepared task table (slicq_*_batch); results are
    # bitwise those of the calls that rebuild the table, also with a chunked workspace
    import torch
    for kw, lens in ((TINY2, [300, 0, 128, 1, 777, 64]), (preset("c4"), [20000, 70001, 44100])):
        plan, _ = gpu_plan(sq, kw)
        tdt = torch_dtype(dt)
        xs = [np.random.default_rng(i + 60).standard_normal(n) for i, n in enumerate(lens)]
        xp = torch.tensor(np.concatenate(xs), dtype=tdt, device=dev)
        c_ref = plan.analyze_batched(xp, lens).clone()           # rebuilds the task table
        y_ref = plan.synthesize_batched(c_ref, lens).clone()
        a_ref = plan.synthesize_batched(c_ref, lens, adjoint=True).clone()
        lay = plan.batch_layout(lens)
        c = plan.analyze_batched(xp, layout=lay)
        y = plan.synthesize_batched(c, layout=lay)
        adj = plan.synthesize_batched(c, layout=lay, adjoint=True)
        assert torch.equal(c, c_ref) and torch.equal(y, y_ref) and torch.equal(adj, a_ref)
        S = lay.total_slices
        cb = 16 if dt == "f64" else 8
        small = plan.workspace_bytes(0 if dt == "f32" else 1, S) - max(S - 2, 0) * (2 * plan.N + 64) * cb
        work = torch.empty(small, dtype=torch.uint8, device=dev)
        c2 = plan.analyze_batched(xp, layout=lay, work=work)
        y2 = plan.synthesize_batched(c2, layout=lay, work=work)
        assert torch.equal(c2, c_ref) and torch.equal(y2, y_ref)


def test_prepared_batch_rejects_short_buffers(sq, dev):
    import ctypes
    import torch
    plan, _ = gpu_plan(sq, TINY2)
    lens = [300, 500]
    lay = plan.batch_layout(lens)
    xp = torch.zeros(800, dtype=torch.float32, device=dev)
    c = plan.analyze_batched(xp, layout=lay)
    h = lay.prepared(plan, xp.device)
    w, wb = plan._workspace(0, lay.total_slices, xp.device, None)
    lib = plan._lib
    P = ctypes.c_void_p
    st = P(torch.cuda.current_stream(dev).cuda_stream)
    assert lib.slicq_analyze_batch(h, 0, P(xp.data_ptr()), 799, P(c.data_ptr()), c.numel(), P(w.data_ptr()), wb,
                                   st) == -4
    assert lib.slicq_synthesize_batch(h, 0, P(c.data_ptr()), c.numel() - 1, P(xp.data_ptr()), 800,
                                      P(w.data_ptr()), wb, st) == -4
    assert lib.slicq_analyze_batch(h, 0, P(xp.data_ptr()), 800, P(c.data_ptr()), c.numel(), P(w.data_ptr()), 64,
                                   st) == -4
    torch.cuda.synchronize()


def test_size_errors(sq, dev):
    import torch
    plan, _ = gpu_plan(sq, TINY2)
    x = torch.zeros(300, dtype=torch.float32, device=dev)
    out = torch.empty(10, dtype=torch.complex64, device=dev)
    with pytest.raises(sq.SlicqError, match="-4"):
        plan.analyze(x, out=out)
    with pytest.raises(sq.SlicqError, match="-4"):
        plan.analyze(x, work=torch.empty(64, dtype=torch.uint8, device=dev))


@pytest.mark.parametrize("name,T", [("c2", 150000), ("c4", 100000), ("c5", 60000)])
def test_slice_major_layout(sq, dev, name, T):
    import torch
    kw = preset(name)
    plan = sq.Plan(**kw, layout="slice")
    opl = OraclePlan(**kw)
    p = PRESETS[name]
    x = pink_plus_tones(T, p.fs, 31)
    ref = pack(opl, analyze(opl, x))
    c = plan.analyze(torch.tensor(x, dtype=torch.float32, device=dev))
    y = plan.synthesize(c, T)
    S = plan.num_slices(T)
    check_coefs(opl, plan.to_band_major(c, S).cpu().numpy(), ref, S, "f32")
    assert rel(y.cpu().numpy(), x) <= 1e-5
    k = plan.nbands // 2
    assert torch.equal(plan.band(c, k, S), c.view(S, plan.coefs_per_slice)[:, plan.offsets[k]:plan.offsets[k] + plan.M[k]])
