"""Differentiable sliCQ on the GPU: the adjoint kernel behind
torch.autograd (SliCQFunction) against FP64 central finite differences, the
oracle's adjoint and the dot-product identity.

Loss (reading of the differentiable workload): sum over stored coefficients of
(log(1 + |c(x)|^2) - log(1 + |c(y)|^2))^2 with a fixed second batch y.
"""
import numpy as np
import pytest

from oracle import OraclePlan, adjoint, unpack, num_slices
from workloads import PRESETS, noise_plus_sines

pytestmark = pytest.mark.gpu


def c4_kw():
    p = PRESETS["c4"]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


@pytest.fixture(scope="module")
def sq():
    import paper_1210_0084_amd as m
    return m


@pytest.fixture(scope="module")
def plan(sq):
    return sq.Plan(**c4_kw())


def loss_terms(c, cy):
    import torch
    return (torch.log1p(c.real ** 2 + c.imag ** 2) - torch.log1p(cy.real ** 2 + cy.imag ** 2)) ** 2


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_dot_product_identity(sq, dev, plan, dt):
    import torch
    tdt = torch.float32 if dt == "f32" else torch.float64
    ctype = torch.complex64 if dt == "f32" else torch.complex128
    T = 50000
    g = np.random.default_rng(1)
    x = torch.tensor(g.standard_normal(T), dtype=tdt, device=dev)
    S = plan.num_slices(T)
    n = S * plan.coefs_per_slice
    c = torch.tensor(g.standard_normal(n) + 1j * g.standard_normal(n), dtype=ctype, device=dev)
    lhs = torch.real(torch.vdot(c.to(torch.complex128), plan.analyze(x).to(torch.complex128))).item()
    rhs = torch.dot(x.double(), plan.adjoint(c, T).double()).item()
    assert abs(lhs - rhs) <= (1e-5 if dt == "f32" else 1e-12) * abs(lhs)


def test_adjoint_matches_oracle_f64(sq, dev, plan):
    import torch
    T = 40000
    opl = OraclePlan(**c4_kw())
    S = num_slices(T, opl.two_n)
    g = np.random.default_rng(2)
    n = S * opl.coefs_per_slice
    c = g.standard_normal(n) + 1j * g.standard_normal(n)
    ya = plan.adjoint(torch.tensor(c, dtype=torch.complex128, device=dev), T).cpu().numpy()
    ref = adjoint(opl, unpack(opl, c, S), T)
    assert np.linalg.norm(ya - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_gradient_against_central_differences(sq, dev, plan, dt):
    # 64 random coordinates of a batch of 2 signals of 6 s (264600 samples)
    import torch
    B, T = 2, 264600
    x64 = np.stack([noise_plus_sines(T, 44100.0, 5 + 1000 * b) for b in range(B)])
    y64 = np.stack([noise_plus_sines(T, 44100.0, 1005 + 1000 * b) for b in range(B)])
    tdt = torch.float32 if dt == "f32" else torch.float64
    x = torch.tensor(x64, dtype=tdt, device=dev, requires_grad=True)
    y = torch.tensor(y64, dtype=tdt, device=dev)
    with torch.no_grad():
        cy = sq.slicq(y, plan)
    loss = loss_terms(sq.slicq(x, plan), cy).sum()
    loss.backward()
    grad = x.grad.detach().double().cpu().numpy()

    # FP64 central differences, Richardson-extrapolated (error O(h^4)); each
    # loss difference is summed term by term so that coefficients the
    # coordinate does not reach cancel exactly
    xd = torch.tensor(x64, dtype=torch.float64, device=dev)
    cy64 = sq.slicq(torch.tensor(y64, dtype=torch.float64, device=dev), plan)
    g = np.random.default_rng(6)
    coords = [(int(g.integers(B)), int(g.integers(T))) for _ in range(64)]

    def central(b, t, h):
        xp = xd.clone()
        xm = xd.clone()
        xp[b, t] += h
        xm[b, t] -= h
        dterm = loss_terms(sq.slicq(xp, plan), cy64) - loss_terms(sq.slicq(xm, plan), cy64)
        return dterm.sum().item() / (2 * h)

    h = 2e-4
    fd = np.array([(4 * central(b, t, h / 2) - central(b, t, h)) / 3 for b, t in coords])
    got = np.array([grad[b, t] for b, t in coords])
    err = np.linalg.norm(got - fd) / np.linalg.norm(fd)
    print(f"gradient vs central differences ({dt}): rel-L2 {err:.2e}", flush=True)
    assert err <= (1e-4 if dt == "f32" else 1e-7)


def test_batched_autograd_equals_per_signal(sq, dev, plan):
    import torch
    B, T = 3, 70000
    g = np.random.default_rng(4)
    xs = torch.tensor(g.standard_normal((B, T)), dtype=torch.float32, device=dev, requires_grad=True)
    c = sq.slicq(xs, plan)
    w = torch.randn(c.shape, dtype=torch.float32, device=dev)
    ((c.real ** 2 + c.imag ** 2) * w).sum().backward()
    gb = xs.grad.clone()
    for b in range(B):
        xb = xs.detach()[b].clone().requires_grad_(True)
        cb = sq.slicq(xb, plan)
        assert torch.equal(cb.detach(), c.detach()[b])
        ((cb.real ** 2 + cb.imag ** 2) * w[b]).sum().backward()
        assert torch.equal(xb.grad, gb[b])


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_loss_kernel_matches_torch_and_is_deterministic(sq, dev, dt):
    # the one-pass loss kernel (value and gradient) against the same loss in
    # FP64 torch operations; two runs give identical results
    import torch
    ctype = torch.complex64 if dt == "f32" else torch.complex128
    g = np.random.default_rng(31)
    n = 1_000_003
    c = torch.tensor(g.standard_normal(n) + 1j * g.standard_normal(n), dtype=ctype, device=dev, requires_grad=True)
    t = torch.tensor(g.uniform(0, 2, n), dtype=c.real.dtype, device=dev)
    loss = sq.logmag_loss(c, t)
    loss.backward()
    cd = c.detach().to(torch.complex128).requires_grad_(True)
    ref = ((torch.log1p(cd.real ** 2 + cd.imag ** 2) - t.double()) ** 2).sum()
    ref.backward()
    tol = 1e-5 if dt == "f32" else 1e-12
    assert abs(loss.item() - ref.item()) <= tol * abs(ref.item())
    gd = c.grad.to(torch.complex128)
    assert (torch.linalg.vector_norm(gd - cd.grad) / torch.linalg.vector_norm(cd.grad)).item() <= tol
    again = sq.logmag_loss(c.detach(), t)
    assert again.item() == loss.item()


def test_gradient_through_loss_kernel_fd(sq, dev, plan):
    # analysis -> loss kernel -> adjoint: gradient against FP64 central differences
    import torch
    T = 20000
    x0 = noise_plus_sines(T, 44100.0, 41)
    y = noise_plus_sines(T, 44100.0, 1041)
    xd = torch.tensor(x0, dtype=torch.float64, device=dev, requires_grad=True)
    with torch.no_grad():
        cy = plan.analyze(torch.tensor(y, dtype=torch.float64, device=dev))
        ty = torch.log1p(cy.real ** 2 + cy.imag ** 2)
    sq.logmag_loss(sq.slicq(xd, plan), ty).backward()
    grad = xd.grad.cpu().numpy()

    def f(v):
        with torch.no_grad():
            return sq.logmag_loss(plan.analyze(torch.tensor(v, dtype=torch.float64, device=dev)), ty).item()
    g = np.random.default_rng(6)
    for i in g.integers(0, T, 8):
        h = 1e-4
        e = np.zeros(T)
        e[i] = h
        fd = (f(x0 + e) - f(x0 - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_full_c4_batch_sampled_against_oracle(sq, dev, plan):
    # the differentiable workload at full size (32 x 264600 samples, 1088
    # slices) through SliCQFunction as the bench runs it: the coefficients and
    # the input gradient of a linear loss of three sampled signals (first,
    # middle, last) against the FP64 oracle, band by band
    import torch
    from oracle import analyze, pack
    from workloads import make_c4
    xb = make_c4(32)
    B, T = xb.shape
    x = torch.tensor(xb, dtype=torch.float32, device=dev, requires_grad=True)
    c = sq.slicq(x, plan)
    g = np.random.default_rng(61)
    w = torch.tensor(g.standard_normal(tuple(c.shape)) + 1j * g.standard_normal(tuple(c.shape)),
                     dtype=torch.complex64, device=dev)
    (c.real * w.real + c.imag * w.imag).sum().backward()
    torch.cuda.synchronize()
    opl = OraclePlan(**c4_kw())
    S = num_slices(T, opl.two_n)
    for b in (0, 16, 31):
        print(f"case c4 full batch, signal {b}", flush=True)
        ref = pack(opl, analyze(opl, xb[b]))
        got = c[b].detach().cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
        for k in range(opl.K + 2):
            o, M = int(plan.offsets[k]) * S, int(plan.M[k])
            r = ref[o:o + S * M]
            assert np.linalg.norm(got[o:o + S * M] - r) <= 1e-4 * np.linalg.norm(r), (b, k)
        gref = adjoint(opl, unpack(opl, w[b].cpu().numpy().astype(np.complex128), S), T)
        gg = x.grad[b].cpu().numpy()
        assert np.linalg.norm(gg - gref) <= 1e-5 * np.linalg.norm(gref), b
