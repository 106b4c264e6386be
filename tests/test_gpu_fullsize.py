"""Parity of the batched and differentiable forms at the sizes of their workloads.

* The 512-transform batch (|I_b| log-uniform in [2^8, 2^18], d = 15, L_b = ceil(log2 |I_b|), primes
  in [|I_b|, 2|I_b|], complex64): every transform of the batched plan is bit-identical to its own
  plain plan in both directions, and 8 transforms drawn at random agree with the oracle (R15).
* The least-squares workload (|I| = 2^20 in [-16,16]^30, L = 20 primes in [2^20, 2^21]) in a
  complex128 plan: directional finite differences of the sample-domain loss along directions
  supported on 1024 frequencies equal the autograd gradient (A^* of the weighted residual).
"""
import numpy as np
import pytest

from gpu_util import require_gpu, assert_close
from oracle import mr1l as O
from workloads import batched_c4, lsq_c5, rng_for

pytestmark = pytest.mark.gpu


def test_batched_512_full_size():
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan, Plan
    probs = batched_c4(with_data=False)
    assert len(probs) == 512
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
    g = torch.Generator(device="cuda:0").manual_seed(4004)
    y = torch.randn((1, bp.sum_M), dtype=torch.complex64, device="cuda:0", generator=g)
    c = torch.randn((1, bp.n), dtype=torch.complex64, device="cuda:0", generator=g)
    cb = bp.forward(y)
    yb = bp.adjoint(c)
    torch.cuda.synchronize()
    fo = bp.freq_offsets
    so = np.concatenate([[0], np.cumsum([int(p.M.sum()) for p in probs])])
    pick = set(rng_for(4005).choice(len(probs), size=8, replace=False).tolist())
    print(f"batched 512: sum n {bp.n}, sum M {bp.sum_M}; oracle on transforms {sorted(pick)}", flush=True)
    for b, p in enumerate(probs):
        pp = Plan(p.freqs, p.M, p.z, dtype="c64", device=0)
        yv = y[:, so[b]:so[b + 1]].contiguous()
        cv = c[:, fo[b]:fo[b + 1]].contiguous()
        cp = pp.forward(yv)
        yp = pp.adjoint(cv)
        assert torch.equal(torch.view_as_real(cp), torch.view_as_real(cb[:, fo[b]:fo[b + 1]])), b
        assert torch.equal(torch.view_as_real(yp), torch.view_as_real(yb[:, so[b]:so[b + 1]])), b
        if b in pick:
            yh = yv.cpu().numpy()[0].astype(np.complex128)
            ch = cv.cpu().numpy()[0].astype(np.complex128)
            assert_close(cp.cpu().numpy()[0], O.forward(p.freqs, p.M, p.z, yh), "c64", f"forward {b}")
            assert_close(yp.cpu().numpy()[0], O.adjoint(p.freqs, p.M, p.z, ch), "c64", f"adjoint {b}")
        pp.close()


def test_lsq_full_size_finite_differences():
    torch = require_gpu()
    from paper_1711_05152_amd.autograd import Mr1lSynth, WeightedLsq
    from paper_1711_05152_amd.mr1l import Plan
    freqs, M, z, seed = lsq_c5()
    ep = Plan(freqs, M, z, dtype="c128", weights="eval", n_rhs=1, device=0)
    print(f"least squares: n {ep.n}, L {ep.L}, sum M {ep.sum_M}", flush=True)
    g = torch.Generator(device="cuda:0").manual_seed(seed % (1 << 62))
    with torch.no_grad():
        c_true = torch.randn((1, ep.n), dtype=torch.complex128, device="cuda:0", generator=g)
        y = ep.adjoint(c_true)
        y += 1e-3 * torch.randn(y.shape, dtype=torch.complex128, device="cuda:0", generator=g)
        c0 = c_true + 0.1 * torch.randn(c_true.shape, dtype=torch.complex128, device="cuda:0", generator=g)
        del c_true

    def loss_of(cc):
        return WeightedLsq.apply(Mr1lSynth.apply(cc, ep), y, ep)

    c = c0.clone().requires_grad_(True)
    loss_of(c).backward()
    grad = c.grad.detach()
    rng = rng_for(5005)
    for _ in range(3):
        sub = rng.choice(ep.n, size=1024, replace=False)
        v = torch.zeros_like(c0)
        vals = rng.standard_normal(1024) + 1j * rng.standard_normal(1024)
        v[0, torch.from_numpy(sub).to("cuda:0")] = torch.from_numpy(vals).to("cuda:0")
        eps = 1e-2
        with torch.no_grad():
            lp = loss_of(c0 + eps * v).item()
            lm = loss_of(c0 - eps * v).item()
        # the loss is quadratic in c, so the central difference has no truncation error: what is
        # left is the rounding of the two losses (about 1e-12 relative in double over 3e7 samples)
        fd = (lp - lm) / (2 * eps)
        an = torch.real(torch.sum(torch.conj(grad) * v)).item()
        tol = 1e-7 * abs(an) + 1e-12 * max(abs(lp), abs(lm)) / eps
        print(f"directional derivative: fd {fd:.12e} autograd {an:.12e} (tol {tol:.2e})", flush=True)
        assert abs(fd - an) <= tol, (fd, an, tol)
