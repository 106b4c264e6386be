"""mr1l_lsq_residual_noalloc (the allocation-free variant of mr1l_lsq_residual) against the
allocating entry point, through the C ABI: the same loss and gradient, bit for bit, on two calls in
a row (the second on a smaller plan, so the fixed partials array keeps the first call's larger
contents beyond what the second writes), and a clear error beyond the array's limit."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import require_gpu
from workloads import cn01, rng_for, transform_problem

pytestmark = pytest.mark.gpu


def _call(fn, plan, s, y, scale, grad, loss):
    import torch
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: C.c_void_p(0 if t is None else t.data_ptr())  # noqa: E731
    return fn(plan._h, ptr(s), ptr(y), ptr(scale), ptr(grad), ptr(loss), stream)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_matches_allocating_entry_point(dtype):
    torch = require_gpu()
    from paper_1711_05152_amd import _lib
    from paper_1711_05152_amd.mr1l import Plan
    lib = _lib.lib()
    tdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]
    # second call smaller: fewer lattices and right-hand sides (fewer block partials)
    for rep, (n, L, n_rhs) in enumerate(((4000, 12, 9), (900, 3, 2))):
        p = transform_problem(rng_for(960, rep), n, 5, 20, L, n, 3 * n, n_rhs=n_rhs)
        plan = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="eval", n_rhs=n_rhs, device=0)
        s = torch.from_numpy(p.samples).to("cuda:0", tdt)
        y = torch.from_numpy(cn01(rng_for(961, rep), p.samples.shape)).to("cuda:0", tdt)
        scale = torch.tensor([0.75], dtype=torch.float64, device="cuda:0")
        outs = []
        for fn in (lib.mr1l_lsq_residual, lib.mr1l_lsq_residual_noalloc):
            grad = torch.empty_like(s)
            loss = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
            assert _call(fn, plan, s, y, scale, grad, loss) == 0, lib.mr1l_last_error()
            torch.cuda.synchronize()
            outs.append((grad.cpu(), loss.cpu()))
        (g0, l0), (g1, l1) = outs
        assert torch.equal(torch.view_as_real(g0), torch.view_as_real(g1))
        assert l0.item() == l1.item() and np.isfinite(l1.item()), (l0.item(), l1.item())
        # against the formula in double: loss = 1/2 sum_l (1/M_l) |s - y|^2
        off = np.concatenate([[0], np.cumsum(p.M)])
        dy = p.samples - y.cpu().numpy().astype(np.complex128)
        want = sum(0.5 / p.M[l] * np.sum(np.abs(dy[:, off[l]:off[l + 1]]) ** 2) for l in range(L))
        tol = 1e-12 if dtype == "c128" else 1e-5
        assert abs(l1.item() - want) <= tol * want, (l1.item(), want)
        # gradient only (no loss, no scale): the array is not touched, same bits as the allocating call
        grads = []
        for fn in (lib.mr1l_lsq_residual, lib.mr1l_lsq_residual_noalloc):
            grad = torch.empty_like(s)
            assert _call(fn, plan, s, y, None, grad, None) == 0
            torch.cuda.synchronize()
            grads.append(torch.view_as_real(grad.cpu()))
        assert torch.equal(grads[0], grads[1])
        plan.close()


def test_noalloc_rejects_plans_beyond_its_array():
    torch = require_gpu()
    from paper_1711_05152_amd import _lib
    from paper_1711_05152_amd.mr1l import Plan
    lib = _lib.lib()
    # 64 L n_rhs = 64 * 3 * 700 = 134400 > 131072 block partials
    p = transform_problem(rng_for(962), 40, 3, 6, 3, 17, 60, n_rhs=1)
    plan = Plan(p.freqs, p.M, p.z, dtype="c64", weights="eval", n_rhs=700, device=0)
    s = torch.zeros((700, plan.sum_M), dtype=torch.complex64, device="cuda:0")
    loss = torch.zeros((1,), dtype=torch.float64, device="cuda:0")
    assert _call(lib.mr1l_lsq_residual_noalloc, plan, s, s, None, None, loss) == 6   # MR1L_ERR_UNSUPPORTED
    assert b"131072" in lib.mr1l_last_error()
    # the gradient alone needs no partials and is accepted
    grad = torch.empty_like(s)
    assert _call(lib.mr1l_lsq_residual_noalloc, plan, s, s, None, grad, None) == 0
    torch.cuda.synchronize()
    assert torch.count_nonzero(grad).item() == 0
    plan.close()
