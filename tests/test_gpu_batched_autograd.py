"""GPU tests of the batched form (many uneven transforms in one plan, HIP-graph capture) and of
the differentiable form (autograd Functions whose backward is the adjoint transform)."""
import numpy as np
import pytest

from gpu_util import require_gpu, assert_close
from oracle import mr1l as O
from workloads import batched_c4, rng_for, transform_problem, cn01

pytestmark = pytest.mark.gpu


def _t(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", {"c64": torch.complex64,
                                                                   "c128": torch.complex128}[dtype])


def _small_batch():
    # same recipe as the 512-transform workload (d = 15, box [-32,32], L = ceil(log2 n),
    # primes in [n, 2n]) with sizes log-uniform in [2^6, 2^12] so that the oracle stays fast
    return batched_c4(count=24, seed_extra=1, log2_lo=6.0, log2_hi=12.0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batched_matches_oracle_and_plain(dtype):
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan, Plan
    probs = _small_batch()
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype=dtype, device=0)
    y = np.concatenate([p.samples[0] for p in probs])[None, :]
    c = np.concatenate([p.coeffs[0] for p in probs])[None, :]
    cb = bp.forward(_t(torch, y, dtype)).cpu().numpy()[0]
    yb = bp.adjoint(_t(torch, c, dtype)).cpu().numpy()[0]
    res, uniq, cnt = bp.alias()
    res, cnt = res.cpu().numpy(), cnt.cpu().numpy()
    fo, so = bp.freq_offsets, np.concatenate([[0], np.cumsum([p.M.sum() for p in probs])])
    for b, p in enumerate(probs):
        f0, f1 = fo[b], fo[b + 1]
        r0, _, c0 = O.unaliased_sets(p.freqs, p.M, p.z)
        assert np.array_equal(res[: len(p.M), f0:f1], r0)
        assert np.array_equal(cnt[f0:f1].astype(np.int64), c0)
        assert_close(cb[f0:f1], O.forward(p.freqs, p.M, p.z, p.samples[0]), dtype, f"batched fwd {b}")
        assert_close(yb[so[b]:so[b + 1]], O.adjoint(p.freqs, p.M, p.z, p.coeffs[0]), dtype, f"batched adj {b}")
        # the plain per-transform plan runs the same arithmetic
        pp = Plan(p.freqs, p.M, p.z, dtype=dtype, device=0)
        cp = pp.forward(_t(torch, p.samples, dtype)).cpu().numpy()[0]
        yp = pp.adjoint(_t(torch, p.coeffs, dtype)).cpu().numpy()[0]
        assert np.array_equal(cp, cb[f0:f1])
        assert np.array_equal(yp, yb[so[b]:so[b + 1]])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batched_inblock_kernel_matches_stage_sweep(dtype):
    """The persistent in-block kernel (small transforms whole in one workgroup, from a work queue)
    gives the bits of the stage sweep, in both directions, on a batch that mixes in-block and swept
    transforms; two calls in a row (the queue is reset by the launch itself)."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan, batch_inblock
    probs = batched_c4(count=40, seed_extra=2, log2_lo=6.0, log2_hi=13.5)
    y = _t(torch, np.concatenate([p.samples[0] for p in probs])[None, :], dtype)
    c = _t(torch, np.concatenate([p.coeffs[0] for p in probs])[None, :], dtype)
    assert batch_inblock() == 1
    try:
        batch_inblock(0)
        swept = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype=dtype, device=0)
    finally:
        batch_inblock(1)
    mixed = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype=dtype, device=0)
    ref = (swept.forward(y), swept.adjoint(c))
    n_small = sum(1 for p in probs if p.n <= 2048 and (2 * p.M.max() - 1) <= 4096)
    print(f"{n_small} of {len(probs)} transforms in-block", flush=True)
    assert 0 < n_small < len(probs)
    for _ in range(2):
        got = (mixed.forward(y), mixed.adjoint(c))
        for a, b in zip(got, ref):
            assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def test_batched_graph_replay():
    """Forward and adjoint captured into HIP graphs (torch.cuda.CUDAGraph) and replayed several
    times with eager work in between: every replay equals the eager result."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan
    probs = _small_batch()
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
    y = _t(torch, np.concatenate([p.samples[0] for p in probs])[None, :], "c64")
    c = _t(torch, np.concatenate([p.coeffs[0] for p in probs])[None, :], "c64")
    c_out = bp.empty_coeffs()
    y_out = bp.empty_samples()
    ref_c = bp.forward(y).clone()
    ref_y = bp.adjoint(c).clone()
    gf = bp.capture("forward", y, c_out)
    ga = bp.capture("adjoint", c, y_out)
    for rep in range(3):
        c_out.zero_()
        y_out.zero_()
        junk = bp.forward(y) * 2 + 1            # eager work between replays
        torch.cuda.synchronize()
        gf.replay()
        ga.replay()
        torch.cuda.synchronize()
        assert torch.equal(c_out, ref_c), rep
        assert torch.equal(y_out, ref_y), rep
        del junk


def test_batched_group_streams_graph_replay():
    """A batch large enough (over 2^25 Bluestein points, three length groups) that the groups' stage
    pipelines run on concurrent streams: forward and adjoint equal the transforms' own plans bit for
    bit, and graph replays (with eager work and synchronisation between them) equal the eager call."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan, Plan
    rng = rng_for(506)
    probs = [transform_problem(rng, 1 << 15, 6, 40, 12, lo, 2 * lo, with_data=False)
             for lo in (1 << 17, 1 << 18, 1 << 19)]
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
    assert sum(int(v) for v in bp.fft_lengths) >= 1 << 25
    g = torch.Generator(device="cuda:0").manual_seed(506)
    y = torch.randn((1, bp.sum_M), dtype=torch.complex64, device="cuda:0", generator=g)
    c = torch.randn((1, bp.n), dtype=torch.complex64, device="cuda:0", generator=g)
    ref_c = bp.forward(y).clone()
    ref_y = bp.adjoint(c).clone()
    fo = bp.freq_offsets
    so = np.concatenate([[0], np.cumsum([int(p.M.sum()) for p in probs])])
    for b, p in enumerate(probs):
        pp = Plan(p.freqs, p.M, p.z, dtype="c64", device=0)
        assert torch.equal(torch.view_as_real(pp.forward(y[:, so[b]:so[b + 1]].contiguous())),
                           torch.view_as_real(ref_c[:, fo[b]:fo[b + 1]])), b
        assert torch.equal(torch.view_as_real(pp.adjoint(c[:, fo[b]:fo[b + 1]].contiguous())),
                           torch.view_as_real(ref_y[:, so[b]:so[b + 1]])), b
        pp.close()
    c_out = bp.empty_coeffs()
    y_out = bp.empty_samples()
    gf = bp.capture("forward", y, c_out)
    ga = bp.capture("adjoint", c, y_out)
    for rep in range(3):
        c_out.zero_()
        y_out.zero_()
        junk = bp.forward(y) * 2 + 1            # eager work between replays
        torch.cuda.synchronize()
        gf.replay()
        ga.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(c_out), torch.view_as_real(ref_c)), rep
        assert torch.equal(torch.view_as_real(y_out), torch.view_as_real(ref_y)), rep
        del junk


def test_autograd_gradcheck_double():
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    from paper_1711_05152_amd.autograd import Mr1lFFT, Mr1lSynth, Mr1lFFTAdj, Mr1lAnalysis
    p = transform_problem(rng_for(500), 24, 3, 5, 3, 29, 61, n_rhs=1)
    fp = Plan(p.freqs, p.M, p.z, dtype="c128", weights="paper", device=0)
    ep = Plan(p.freqs, p.M, p.z, dtype="c128", weights="eval", device=0)
    y = _t(torch, p.samples, "c128").requires_grad_(True)
    c = _t(torch, p.coeffs, "c128").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v: Mr1lFFT.apply(v, fp), (y,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda v: Mr1lFFTAdj.apply(v, fp), (c,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda v: Mr1lSynth.apply(v, ep), (c,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda v: Mr1lAnalysis.apply(v, ep), (y,), eps=1e-6, atol=1e-8)


def _lsq_loss(torch, c, plan, y, w):
    from paper_1711_05152_amd.autograd import Mr1lSynth
    r = Mr1lSynth.apply(c, plan) - y
    return 0.5 * (w * (r.real ** 2 + r.imag ** 2)).sum()


def test_lsq_gradient_dense_fp64_reference():
    """Sample-domain least squares L(c) = 1/2 sum_l (1/M_l) ||A_l c - y_l||^2: the autograd
    gradient (A^H W (A c - y) in PyTorch's convention) against the dense FP64 Fourier matrix."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    p = transform_problem(rng_for(501), 200, 30, 16, 4, 200, 400, n_rhs=2)
    A = np.concatenate([O.fourier_matrix(O.lattice_nodes(p.z[l], p.M[l]), p.freqs) for l in range(len(p.M))])
    wv = np.concatenate([np.full(m, 1.0 / m) for m in p.M])
    for dtype in ("c128", "c64"):
        ep = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="eval", n_rhs=2, device=0)
        c = _t(torch, p.coeffs, dtype).requires_grad_(True)
        y = _t(torch, p.samples, dtype)
        w = torch.from_numpy(wv).to("cuda:0", torch.float64 if dtype == "c128" else torch.float32)
        loss = _lsq_loss(torch, c, ep, y, w)
        loss.backward()
        ref = (A.conj().T @ (wv[:, None] * (A @ p.coeffs.T - p.samples.T))).T
        assert_close(c.grad.detach().cpu().numpy(), ref, dtype, f"lsq grad {dtype}")


def test_lsq_gradient_finite_differences_subset():
    """Directional finite differences along random directions supported on 1024 frequencies of a
    2^14-frequency, d = 30 problem (FP64 plan) match the autograd gradient."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    p = transform_problem(rng_for(502), 1 << 14, 30, 16, 8, 1 << 14, 1 << 15, n_rhs=1)
    ep = Plan(p.freqs, p.M, p.z, dtype="c128", weights="eval", device=0)
    wv = torch.from_numpy(np.concatenate([np.full(m, 1.0 / m) for m in p.M])).to("cuda:0")
    y = _t(torch, p.samples, "c128")
    c = _t(torch, p.coeffs, "c128").requires_grad_(True)
    _lsq_loss(torch, c, ep, y, wv).backward()
    g = c.grad.detach()
    rng = rng_for(503)
    for _ in range(3):
        sub = rng.choice(p.n, size=1024, replace=False)
        v = np.zeros((1, p.n), np.complex128)
        v[0, sub] = cn01(rng, 1024)
        vt = _t(torch, v, "c128")
        eps = 1e-5
        with torch.no_grad():
            lp = _lsq_loss(torch, c + eps * vt, ep, y, wv).item()
            lm = _lsq_loss(torch, c - eps * vt, ep, y, wv).item()
        fd = (lp - lm) / (2 * eps)
        an = torch.real(torch.sum(torch.conj(g) * vt)).item()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_gradient_descent_decreases_loss():
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    p = transform_problem(rng_for(504), 1 << 12, 30, 16, 6, 1 << 12, 1 << 13, n_rhs=4)
    ep = Plan(p.freqs, p.M, p.z, dtype="c64", weights="eval", n_rhs=4, device=0)
    c_true = _t(torch, p.coeffs, "c64")
    with torch.no_grad():
        y = ep.adjoint(c_true)
    res, _, _ = ep.alias()
    step = 1.0 / sum(int(torch.bincount(res[l]).max()) for l in range(ep.L))
    wv = torch.from_numpy(np.concatenate([np.full(m, 1.0 / m) for m in p.M]).astype(np.float32)).to("cuda:0")
    c = torch.zeros_like(c_true, requires_grad=True)
    losses = []
    for _ in range(20):
        loss = _lsq_loss(torch, c, ep, y, wv)
        losses.append(loss.item())
        c.grad = None
        loss.backward()
        with torch.no_grad():
            c -= step * c.grad
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:])), losses
    assert losses[-1] < 0.5 * losses[0]


def test_fused_lsq_loss_and_gradient():
    """WeightedLsq (one library pass each way) gives the loss 1/2 sum_l (1/M_l)||s_l - y_l||^2 and
    the gradient of the elementwise autograd formulation; composed with Mr1lSynth it reproduces the
    dense FP64 gradient A^H W (A c - y); the in-place gradient (grad = s) and the scale work."""
    torch = require_gpu()
    from paper_1711_05152_amd.autograd import Mr1lSynth, WeightedLsq
    from paper_1711_05152_amd.mr1l import Plan
    p = transform_problem(rng_for(505), 300, 12, 16, 5, 300, 700, n_rhs=3)
    A = np.concatenate([O.fourier_matrix(O.lattice_nodes(p.z[l], p.M[l]), p.freqs) for l in range(len(p.M))])
    wv = np.concatenate([np.full(m, 1.0 / m) for m in p.M])
    for dtype in ("c128", "c64"):
        ep = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="eval", n_rhs=3, device=0)
        y = _t(torch, p.samples, dtype)
        s_np = cn01(rng_for(506), p.samples.shape)
        s = _t(torch, s_np, dtype).requires_grad_(True)
        loss = WeightedLsq.apply(s, y, ep)
        ref_loss = 0.5 * float(np.sum(wv[None, :] * np.abs(s_np - p.samples) ** 2))
        assert abs(loss.item() - ref_loss) <= (1e-13 if dtype == "c128" else 1e-6) * ref_loss
        (3.0 * loss).backward()
        ref_grad = 3.0 * wv[None, :] * (s_np - p.samples)
        assert_close(s.grad.cpu().numpy(), ref_grad, dtype, f"fused lsq grad {dtype}")
        # in place, with a device scale
        g = s.detach().clone()
        ep.lsq_residual(g, y, grad=g, scale=torch.tensor(2.0, dtype=torch.float64, device="cuda:0"))
        assert_close(g.cpu().numpy(), 2.0 * wv[None, :] * (s_np - p.samples), dtype, f"in-place grad {dtype}")
        # through the synthesis: gradient with respect to c
        c = _t(torch, p.coeffs, dtype).requires_grad_(True)
        WeightedLsq.apply(Mr1lSynth.apply(c, ep), y, ep).backward()
        ref = (A.conj().T @ (wv[:, None] * (A @ p.coeffs.T - p.samples.T))).T
        assert_close(c.grad.detach().cpu().numpy(), ref, dtype, f"composed lsq grad {dtype}")
