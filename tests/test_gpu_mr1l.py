"""GPU parity of the HIP multiple rank-1 lattice FFT against the CPU oracle (through the C ABI).

Integer outputs (residues, unaliased sets, counters) must be bit-exact; coefficients and samples
follow the tolerances in gpu_util.assert_close.  Sizes span the one-block Bluestein path
(2M - 1 <= 4096), the four-step path, ragged tails, several right-hand sides and the full
standalone workload (|I| = 2^16, d = 10, L = 16).
"""
import zlib

import numpy as np
import pytest

from gpu_util import require_gpu, assert_close
from oracle import mr1l as O
from workloads import rng_for, transform_problem, standalone_c2, cn01

pytestmark = pytest.mark.gpu


def _plan(p, dtype, weights="paper", n_rhs=None):
    from paper_1711_05152_amd.mr1l import Plan
    return Plan(p.freqs, p.M, p.z, dtype=dtype, weights=weights,
                n_rhs=n_rhs if n_rhs is not None else p.samples.shape[0], device=0)


def _to(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", {"c64": torch.complex64,
                                                                   "c128": torch.complex128}[dtype])


class _pow2_only:
    """Plans created inside take power-of-two Bluestein lengths only (mr1l_fft_smooth(0))."""

    def __enter__(self):
        from paper_1711_05152_amd.mr1l import fft_smooth
        self.prev = fft_smooth(-1)
        fft_smooth(0)

    def __exit__(self, *exc):
        from paper_1711_05152_amd.mr1l import fft_smooth
        fft_smooth(self.prev)


CASES = [
    # name, n, d, box, L, mlo, mhi, n_rhs
    ("tiny_small_path", 30, 3, 5, 3, 17, 60, 1),
    ("small_path_ragged", 700, 4, 12, 5, 700, 1400, 2),
    ("fourstep_lg13_14", 2500, 6, 20, 4, 2500, 5000, 1),
    ("fourstep_multi_rhs", 6000, 5, 30, 6, 6000, 12000, 5),
    ("mixed_paths", 1500, 3, 40, 6, 1500, 6000, 3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_alias_bit_exact(case, dtype):
    torch = require_gpu()
    name, n, d, box, L, mlo, mhi, n_rhs = case
    p = transform_problem(rng_for(300, zlib.crc32(name.encode())), n, d, box, L, mlo, mhi, n_rhs=n_rhs)
    plan = _plan(p, dtype)
    res, uniq, cnt = plan.alias()
    torch.cuda.synchronize()
    r0, u0, c0 = O.unaliased_sets(p.freqs, p.M, p.z)
    assert np.array_equal(res.cpu().numpy(), r0)
    assert np.array_equal(uniq.cpu().numpy().astype(bool), u0)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), np.minimum(c0, 255))
    assert plan.n_uncovered() == int((c0 == 0).sum())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("weights", ["paper", "eval"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_forward_adjoint_parity(case, weights, dtype):
    torch = require_gpu()
    name, n, d, box, L, mlo, mhi, n_rhs = case
    p = transform_problem(rng_for(301, zlib.crc32(name.encode())), n, d, box, L, mlo, mhi, n_rhs=n_rhs)
    plan = _plan(p, dtype, weights)
    print(f"case {name} dtype {dtype} weights {weights}", flush=True)
    y = _to(torch, p.samples, dtype)
    c = plan.forward(y)
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples, weights)
    yy = plan.adjoint(_to(torch, p.coeffs, dtype))
    y_ref = O.adjoint(p.freqs, p.M, p.z, p.coeffs, weights)
    torch.cuda.synchronize()
    assert_close(c.cpu().numpy(), c_ref, dtype, f"forward {name}")
    assert_close(yy.cpu().numpy(), y_ref, dtype, f"adjoint {name}")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_standalone_full_size(dtype):
    """|I| = 2^16 frequencies in [-64,64]^10, L = 16 primes in [2^16, 2^17]: elementwise parity of
    forward and adjoint with the oracle, bit-exact integers, and the adjoint identity."""
    torch = require_gpu()
    p = standalone_c2()
    plan = _plan(p, dtype)
    res, uniq, cnt = plan.alias()
    y = _to(torch, p.samples, dtype)
    c = plan.forward(y)
    yy = plan.adjoint(_to(torch, p.coeffs, dtype))
    torch.cuda.synchronize()
    r0, u0, c0 = O.unaliased_sets(p.freqs, p.M, p.z)
    assert np.array_equal(res.cpu().numpy(), r0)
    assert np.array_equal(uniq.cpu().numpy().astype(bool), u0)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), c0)
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples)
    y_ref = O.adjoint(p.freqs, p.M, p.z, p.coeffs)
    c_np = c.cpu().numpy()
    assert_close(c_np, c_ref, dtype, "forward full")
    assert_close(yy.cpu().numpy(), y_ref, dtype, "adjoint full")
    # adjoint identity <F y, c> = <y, F* c> on the GPU results alone
    lhs = np.vdot(p.coeffs[0], c_np[0])
    rhs = np.vdot(yy.cpu().numpy()[0], p.samples[0])
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0)


MANY_LAT_CASES = [
    # name, n, d, box, L, mlo, mhi: one transform, one right-hand side, Alg. 2's weights
    ("L8_one_pass_half", 3000, 5, 20, 8, 3000, 6000),
    ("L11_ragged_slots", 1777, 4, 30, 11, 1777, 3554),
    ("L19_fourstep", 5001, 6, 25, 19, 5001, 10002),
    ("L64_four_passes", 700, 3, 40, 64, 700, 1400),
    ("L65_ragged_pass", 700, 3, 40, 65, 700, 1400),
]


@pytest.mark.parametrize("case", MANY_LAT_CASES, ids=[c[0] for c in MANY_LAT_CASES])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_many_lattices_plain_and_batched(case, dtype):
    """One transform of 8 to 65 lattices (several passes of the gather's lattice slots): parity
    with the oracle, and forward and adjoint bit-identical to the same transform twice inside a
    batched plan (whose gather and scatter find each frequency's transform by search)."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan
    name, n, d, box, L, mlo, mhi = case
    p = transform_problem(rng_for(307, zlib.crc32(name.encode())), n, d, box, L, mlo, mhi)
    print(f"case {name} dtype {dtype}", flush=True)
    plan = _plan(p, dtype)
    c = plan.forward(_to(torch, p.samples, dtype))
    yy = plan.adjoint(_to(torch, p.coeffs, dtype))
    bp = BatchedPlan([(p.freqs, p.M, p.z), (p.freqs, p.M, p.z)], dtype=dtype, device=0)
    cb = bp.forward(_to(torch, np.concatenate([p.samples, p.samples], axis=1), dtype))
    yb = bp.adjoint(_to(torch, np.concatenate([p.coeffs, p.coeffs], axis=1), dtype))
    torch.cuda.synchronize()
    c_np, y_np = c.cpu().numpy(), yy.cpu().numpy()
    assert_close(c_np, O.forward(p.freqs, p.M, p.z, p.samples), dtype, f"forward {name}")
    assert_close(y_np, O.adjoint(p.freqs, p.M, p.z, p.coeffs), dtype, f"adjoint {name}")
    sm = int(p.M.sum())
    cb, yb = cb.cpu().numpy()[0], yb.cpu().numpy()[0]
    assert np.array_equal(c_np[0], cb[:n]) and np.array_equal(c_np[0], cb[n:])
    assert np.array_equal(y_np[0], yb[:sm]) and np.array_equal(y_np[0], yb[sm:])


def test_standalone_dense_ndft_subset():
    """Coefficients of 64 covered frequencies of the full workload against the term-by-term sum
    of Alg. 2 (tier 0 of the oracle, no FFT)."""
    torch = require_gpu()
    p = standalone_c2()
    plan = _plan(p, "c64")
    c = plan.forward(_to(torch, p.samples, "c64")).cpu().numpy()[0]
    _, _, counter = O.unaliased_sets(p.freqs, p.M, p.z)
    cov = np.nonzero(counter > 0)[0]
    sub = rng_for(302).choice(cov, size=64, replace=False)
    ref = O.forward_direct(p.freqs, p.M, p.z, p.samples[0], subset=sub)
    assert_close(c[sub], ref, "c64", "dense subset")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_exact_recovery_planted(dtype):
    """Samples of a polynomial supported on I (synthesised on the GPU by the EVAL adjoint, i.e. the
    Fourier matrix) are inverted exactly by the PAPER forward on covered frequencies."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    p = transform_problem(rng_for(303), 3000, 8, 25, 12, 6001, 9000, n_rhs=1)
    synth = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="eval", device=0)
    inv = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="paper", device=0)
    c_true = _to(torch, p.coeffs, dtype)
    c_back = inv.forward(synth.adjoint(c_true)).cpu().numpy()[0]
    _, _, counter = O.unaliased_sets(p.freqs, p.M, p.z)
    cov = counter > 0
    assert_close(c_back[cov], p.coeffs[0][cov], dtype, "recovery")
    assert np.all(c_back[~cov] == 0)


def test_edge_cases():
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    rng = rng_for(304)
    # M = 1 and M = 2 lattices, z = 0, a single frequency, uncovered frequencies
    freqs = np.array([[0, 0], [1, 0], [0, 1], [2, 3]], np.int32)
    M = np.array([1, 2, 3, 5, 7], np.int64)
    z = np.array([[0, 0], [1, 1], [1, 2], [0, 0], [3, 5]], np.int64)
    y = cn01(rng, (1, int(M.sum())))
    for dtype in ("c64", "c128"):
        plan = Plan(freqs, M, z, dtype=dtype, device=0)
        got = plan.forward(_to(torch, y, dtype)).cpu().numpy()
        assert_close(got, O.forward(freqs, M, z, y), dtype, "edge forward")
        c = cn01(rng, (1, 4))
        got = plan.adjoint(_to(torch, c, dtype)).cpu().numpy()
        assert_close(got, O.adjoint(freqs, M, z, c), dtype, "edge adjoint")
    one = Plan(np.array([[3]], np.int32), [11], [[2]], dtype="c128", device=0)
    yy = cn01(rng, (1, 11))
    assert_close(one.forward(_to(torch, yy, "c128")).cpu().numpy(), O.forward([[3]], [11], [[2]], yy), "c128")


def test_invalid_arguments_raise():
    require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    from paper_1711_05152_amd import Mr1lError
    with pytest.raises(Mr1lError) as e:
        Plan(np.array([[1, 2], [1, 2]], np.int32), [5], [[1, 1]], device=0)
    assert e.value.status == 1
    with pytest.raises(Mr1lError) as e:
        Plan(np.array([[1, 2]], np.int32), [1 << 24], [[1, 1]], device=0)
    assert e.value.status == 6


def test_exact_modulo_path():
    """|k| ~ 2^30 with M ~ 2^22 puts d max|k| max M above 2^52, where residues use the exact
    int64 remainder instead of the double-precision quotient estimate."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan
    rng = rng_for(305)
    freqs = np.unique(rng.integers(-(1 << 30), 1 << 30, size=(200, 2)), axis=0).astype(np.int32)
    M = np.array([4194301, 4194287], np.int64)           # primes just below 2^22
    z = rng.integers(0, 4194287, size=(2, 2)).astype(np.int64)
    plan = Plan(freqs, M, z, dtype="c64", device=0)
    res, uniq, cnt = plan.alias()
    torch.cuda.synchronize()
    r0, u0, c0 = O.unaliased_sets(freqs, M, z)
    assert np.array_equal(res.cpu().numpy(), r0)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), c0)


@pytest.mark.parametrize("weights", ["paper", "eval"])
def test_cache_alias_matches_recompute(weights):
    """Plan-cached index work (residues and bitmaps reused between calls) gives the results of
    recomputing them in every call, across several calls: bit-identical where the kernels are
    deterministic; the Fourier-matrix adjoint accumulates bins with floating-point atomics, whose
    order (and so the last bits) may change from call to call, so it is compared to 1e-5."""
    torch = require_gpu()
    p = transform_problem(rng_for(310), 5000, 7, 25, 9, 5000, 10000, n_rhs=2)
    ref = _plan(p, "c64", weights)
    cached = _plan(p, "c64", weights)
    cached.cache_alias(True)
    y = _to(torch, p.samples, "c64")
    c = _to(torch, p.coeffs, "c64")

    def same_adj():
        a, b = cached.adjoint(c), ref.adjoint(c)
        if weights == "paper":
            return torch.equal(a, b)
        return float((a - b).abs().max()) <= 1e-5 * float(b.abs().max())

    for _ in range(3):
        assert torch.equal(cached.forward(y), ref.forward(y))
        assert same_adj()
    cached.cache_alias(False)
    assert same_adj()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_eval_adjoint_counting_sort(dtype):
    """Fourier-matrix adjoint on plans with many (k, l) pairs (counting-sort path: bins summed in
    ascending k, no atomics): parity with the oracle, bit-identical repeated calls, and the same
    results with plan-cached index work."""
    torch = require_gpu()
    p = transform_problem(rng_for(320), 12000, 6, 30, 8, 9000, 20000, n_rhs=3)
    plan = _plan(p, dtype, "eval")
    c = _to(torch, p.coeffs, dtype)
    y1 = plan.adjoint(c)
    y2 = plan.adjoint(c)
    assert torch.equal(y1, y2)
    assert_close(y1.cpu().numpy(), O.adjoint(p.freqs, p.M, p.z, p.coeffs, "eval"), dtype, "eval adjoint")
    plan.cache_alias(True)
    for _ in range(2):
        assert torch.equal(plan.adjoint(c), y1)


def test_eval_adjoint_crowded_bins():
    """A lattice with z = 0 puts every frequency into bin 0 (more frequencies per bin than the
    in-register sort takes): still the oracle's sum."""
    torch = require_gpu()
    p = transform_problem(rng_for(321), 20000, 4, 20, 5, 20000, 40000, n_rhs=1)
    p.z[2] = 0
    plan = _plan(p, "c128", "eval")
    y = plan.adjoint(_to(torch, p.coeffs, "c128"))
    assert_close(y.cpu().numpy(), O.adjoint(p.freqs, p.M, p.z, p.coeffs, "eval"), "c128", "crowded eval adjoint")


def test_memory_cache_reuse_and_release():
    """Plans created one after another reuse the library's cached device blocks (stale contents
    included) and cached filter spectra, and give the same results; the cache gives its idle blocks
    back on request and can be switched off."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import memory_cache
    name, n, d, box, L, mlo, mhi, n_rhs = CASES[3]
    p = transform_problem(rng_for(302, 7), n, d, box, L, mlo, mhi, n_rhs=n_rhs)
    y = _to(torch, p.samples, "c128")
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples, "paper")
    memory_cache(0)
    outs = []
    for _ in range(3):
        plan = _plan(p, "c128")
        outs.append(plan.forward(y).cpu().numpy())
        del plan
    assert memory_cache(0) > 0          # the destroyed plans' buffers were held for reuse
    assert memory_cache(0) == 0
    for o in outs:
        assert_close(o, c_ref, "c128", "forward after reuse")
    # the later plans copy the first one's filter spectra from the library's spectrum cache
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    default_cap = torch.cuda.get_device_properties(0).total_memory // 4
    try:
        memory_cache(0, 0)
        plan = _plan(p, "c128")
        assert_close(plan.forward(y).cpu().numpy(), c_ref, "c128", "forward without caching")
        del plan
        assert memory_cache(0) == 0
    finally:
        memory_cache(0, default_cap)


LARGE = [
    # Bluestein lengths 2^21 .. 2^23: stage-1/3 tiles of 8192 or 16384 elements (fp32) and of 8192
    # elements (fp64) hold 128-byte row segments; 2^24 keeps shorter segments
    ("lg21", 3000, 5, 30, 2, (1 << 19) + 1, 1 << 20),
    ("lg22", 3000, 5, 30, 2, (1 << 20) + 1, 1 << 21),
    ("lg23", 3000, 5, 30, 1, (1 << 21) + 1, 1 << 22),
]


@pytest.mark.parametrize("case", LARGE, ids=[c[0] for c in LARGE])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_large_bluestein_lengths(case, dtype):
    torch = require_gpu()
    name, n, d, box, L, mlo, mhi = case
    p = transform_problem(rng_for(303, zlib.crc32(name.encode())), n, d, box, L, mlo, mhi, n_rhs=2)
    print(f"large {name} {dtype} M={list(p.M)}", flush=True)
    with _pow2_only():
        plan = _plan(p, dtype)
    assert all(int(v) & (int(v) - 1) == 0 for v in plan.fft_lengths)
    c = plan.forward(_to(torch, p.samples, dtype))
    yy = plan.adjoint(_to(torch, p.coeffs, dtype))
    torch.cuda.synchronize()
    assert_close(c.cpu().numpy(), O.forward(p.freqs, p.M, p.z, p.samples, "paper"), dtype, f"forward {name}")
    assert_close(yy.cpu().numpy(), O.adjoint(p.freqs, p.M, p.z, p.coeffs, "paper"), dtype, f"adjoint {name}")


SPLIT_CASES = [(13, "c64"), (13, "c128"), (15, "c64"), (15, "c128"), (16, "c128"), (18, "c64"), (21, "c64"),
               (22, "c128")]


@pytest.mark.parametrize("lgn,dtype", SPLIT_CASES, ids=[f"lg{a}_{b}" for a, b in SPLIT_CASES])
def test_every_compiled_split_matches_oracle(lgn, dtype):
    """Every four-step schedule compiled for a Bluestein length (the autotuner's candidates: each
    split, and for each split every stage-2 variant, i.e. radix schedule, values per thread and tile
    size) gives the oracle's forward and adjoint; the schedule overrides are restored afterwards."""
    torch = require_gpu()
    import ctypes
    from paper_1711_05152_amd import _lib
    from paper_1711_05152_amd.tune_fft import candidates, describe, p2_variants
    lo, hi = (1 << (lgn - 2)) + 1, 1 << (lgn - 1)
    p = transform_problem(rng_for(304, lgn), 1500, 6, 40, 2, lo + (hi - lo) // 2, hi, n_rhs=1)
    ref_c = O.forward(p.freqs, p.M, p.z, p.samples, "paper")
    ref_y = O.adjoint(p.freqs, p.M, p.z, p.coeffs, "paper")
    dt = {"c64": _lib.C64, "c128": _lib.C128}[dtype]
    cur = ctypes.c_int(0)
    pow2 = _pow2_only()
    pow2.__enter__()
    try:
        for s in candidates(lgn):
            _lib.check(_lib.lib().mr1l_fft_split(dt, lgn, s, ctypes.byref(cur)), "mr1l_fft_split")
            assert cur.value == s
            for v in p2_variants(lgn, s):
                _lib.check(_lib.lib().mr1l_fft_p2_variant(dt, lgn, v, ctypes.byref(cur)), "mr1l_fft_p2_variant")
                assert cur.value == v
                print(f"schedule lg{lgn} {dtype} {describe(lgn, s, v)}", flush=True)
                plan = _plan(p, dtype)
                c = plan.forward(_to(torch, p.samples, dtype))
                yy = plan.adjoint(_to(torch, p.coeffs, dtype))
                torch.cuda.synchronize()
                assert_close(c.cpu().numpy(), ref_c, dtype, f"forward {describe(lgn, s, v)}")
                assert_close(yy.cpu().numpy(), ref_y, dtype, f"adjoint {describe(lgn, s, v)}")
                del plan
            _lib.lib().mr1l_fft_p2_variant(dt, lgn, -2, None)
        with pytest.raises(_lib.Mr1lError):
            _lib.check(_lib.lib().mr1l_fft_split(dt, lgn, 2, None), "mr1l_fft_split")
        for bad in (5, 7):   # 8 values per thread never combine with the radix-16-major schedule; 7 is out of range
            with pytest.raises(_lib.Mr1lError):
                _lib.check(_lib.lib().mr1l_fft_p2_variant(dt, lgn, bad, None), "mr1l_fft_p2_variant")
    finally:
        _lib.lib().mr1l_fft_p2_variant(dt, lgn, -2, None)
        _lib.lib().mr1l_fft_split(dt, lgn, -1, None)
        pow2.__exit__()


def test_smooth_length_class_rule():
    """A power-of-two length class turns into 3 * 2^k only when all of the plan's lattices in it fit:
    sizes 5000 and 7000 share the class 2^14 (3 * 2^12 = 12288 covers 2 * 5000 - 1 but not
    2 * 7000 - 1), so both keep 2^14; 3000 (class 2^13, too short for a factor-3 length) keeps 2^13;
    sizes 20000 and 21000 (class 2^16, both within 3 * 2^14) both take 49152."""
    require_gpu()
    from paper_1711_05152_amd.mr1l import Plan, fft_smooth
    prev = fft_smooth(-1)
    fft_smooth(2)
    rng = np.random.default_rng(7)
    M = np.array([5003, 7001, 3001, 20011, 21001], np.int64)
    freqs = rng.integers(-20, 21, size=(300, 3)).astype(np.int32)
    freqs = np.unique(freqs, axis=0)
    z = np.stack([rng.integers(0, m, size=3) for m in M]).astype(np.int64)
    try:
        plan = Plan(freqs, M, z, dtype="c64", weights="paper", n_rhs=1, device=0)
        assert [int(v) for v in plan.fft_lengths] == [1 << 14, 1 << 14, 1 << 13, 3 << 14, 3 << 14]
    finally:
        fft_smooth(prev)


def test_large_transform_splits_length_class():
    """A transform of at least 2^25 power-of-two points times right-hand sides splits a class: of the
    sizes 1200007 (2M - 1 within 3 * 2^20) and 1900009 (not) in the class 2^22, the first takes
    3 * 2^20 with four right-hand sides (2 x 2^22 x 4 = 2^25) and 2^22 with one; forward and
    adjoint of the split plan agree with the oracle."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import Plan, fft_smooth
    prev = fft_smooth(-1)
    fft_smooth(2)
    from workloads import distinct_freqs
    rng = rng_for(307)
    freqs = distinct_freqs(rng, 600, 4, -20, 20)
    M = np.array([1200007, 1900009], np.int64)
    z = np.stack([rng.integers(0, m, size=4) for m in M]).astype(np.int64)
    samples = cn01(rng, (4, int(M.sum())))
    coeffs = cn01(rng, (4, freqs.shape[0]))
    try:
        one = Plan(freqs, M, z, dtype="c64", weights="paper", n_rhs=1, device=0)
        assert [int(v) for v in one.fft_lengths] == [1 << 22, 1 << 22]
        one.close()
        plan = Plan(freqs, M, z, dtype="c64", weights="paper", n_rhs=4, device=0)
        assert [int(v) for v in plan.fft_lengths] == [3 << 20, 1 << 22]
    finally:
        fft_smooth(prev)
    got_c = plan.forward(_to(torch, samples, "c64")).cpu().numpy()
    got_y = plan.adjoint(_to(torch, coeffs, "c64")).cpu().numpy()
    assert_close(got_c, O.forward(freqs, M, z, samples, "paper"), "c64", "forward, split class")
    assert_close(got_y, O.adjoint(freqs, M, z, coeffs, "paper"), "c64", "adjoint, split class")


SMOOTH_CASES = [(g, dt, w) for g in range(12, 23) for dt in ("c64", "c128")
                for w in (("paper", "eval") if g in (14, 18) else ("paper",))]


@pytest.mark.parametrize("g,dtype,weights", SMOOTH_CASES, ids=[f"3x2p{g}_{dt}_{w}" for g, dt, w in SMOOTH_CASES])
def test_smooth_lengths_match_oracle(g, dtype, weights):
    """Bluestein lengths N = 3 * 2^g for g = 12 .. 22 (lattice sizes M in [2^g + 1, 1.5 * 2^g], so
    2^(g+1) < 2M - 1 <= 3 * 2^g): with every class allowed (mode 2) the plan takes that length for
    every lattice, its forward and
    adjoint agree with the oracle on two right-hand sides (unaligned lattice offsets, so stages 1
    to 3 run with their column rotation), and a power-of-two plan of the same problem agrees with
    it to rounding."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import fft_smooth
    lo, hi = (1 << g) + 1, 3 << (g - 1)
    L = 2 if g <= 20 else 1
    p = transform_problem(rng_for(305, g), 1200, 5, 30, L, lo, hi, n_rhs=2)
    print(f"smooth 3*2^{g} {dtype} {weights} M={list(p.M)}", flush=True)
    prev = fft_smooth(-1)
    fft_smooth(2)
    try:
        plan = _plan(p, dtype, weights)
    finally:
        fft_smooth(prev)
    assert [int(v) for v in plan.fft_lengths] == [3 << g] * L
    x, c = _to(torch, p.samples, dtype), _to(torch, p.coeffs, dtype)
    got_c = plan.forward(x).cpu().numpy()
    got_y = plan.adjoint(c).cpu().numpy()
    assert_close(got_c, O.forward(p.freqs, p.M, p.z, p.samples, weights), dtype, f"forward 3*2^{g}")
    assert_close(got_y, O.adjoint(p.freqs, p.M, p.z, p.coeffs, weights), dtype, f"adjoint 3*2^{g}")
    del plan
    with _pow2_only():
        plan2 = _plan(p, dtype, weights)
    assert [int(v) for v in plan2.fft_lengths] == [4 << g] * L
    assert_close(got_c, plan2.forward(x).cpu().numpy().astype(np.complex128), dtype, "3*2^g against 2^(g+2)")
    assert_close(got_y, plan2.adjoint(c).cpu().numpy().astype(np.complex128), dtype, "3*2^g against 2^(g+2)")


def test_graft_smoke_entry_point():
    """The smoke entry point (one small forward + adjoint per precision against the oracle) runs."""
    require_gpu()
    import __graft_entry__
    __graft_entry__.smoke()


@pytest.mark.parametrize("weights", ["paper", "eval"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_several_rhs_match_one_at_a_time(weights, dtype):
    """With several right-hand sides per pass the gather reads its bins, and the Fourier-matrix
    adjoint its coefficients, through 64-byte slots that hold a block of right-hand sides side by
    side (9 right-hand sides: blocks of 8 and 1 in complex64, 4, 4 and 1 in complex128, the last
    block padded).  Forward and adjoint, of a plain plan and of a batched plan of two transforms
    (one of them on the in-block kernel), are bit-identical to a one-right-hand-side plan called
    column by column, and agree with the oracle."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import BatchedPlan, rhs_interleave
    fview = np.float32 if dtype == "c64" else np.float64
    p = transform_problem(rng_for(977), 3000, 5, 16, 6, 3000, 9000, n_rhs=9)
    q = transform_problem(rng_for(978), 200, 5, 16, 3, 200, 400, n_rhs=9)
    probs = [(p.freqs, p.M, p.z), (q.freqs, q.M, q.z)]
    prev = rhs_interleave(-1)
    try:
        assert rhs_interleave(2) == 2   # these sizes stay in cache: interleave by request
        plans = [(_plan(p, dtype, weights), _plan(p, dtype, weights, n_rhs=1), p.samples, p.coeffs),
                 (BatchedPlan(probs, dtype=dtype, weights=weights, n_rhs=9, device=0),
                  BatchedPlan(probs, dtype=dtype, weights=weights, n_rhs=1, device=0),
                  np.concatenate([p.samples, q.samples], axis=1),
                  np.concatenate([p.coeffs, q.coeffs], axis=1))]
    finally:
        rhs_interleave(prev)
    for many, one, ys, cs in plans:
        y = _to(torch, ys, dtype)
        c = _to(torch, cs, dtype)
        fm = many.forward(y).cpu().numpy()
        am = many.adjoint(c).cpu().numpy()
        f1 = np.concatenate([one.forward(y[i:i + 1].contiguous()).cpu().numpy() for i in range(9)])
        a1 = np.concatenate([one.adjoint(c[i:i + 1].contiguous()).cpu().numpy() for i in range(9)])
        torch.cuda.synchronize()
        assert np.array_equal(fm.view(fview), f1.view(fview))
        assert np.array_equal(am.view(fview), a1.view(fview))
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples, weights)
    y_ref = O.adjoint(p.freqs, p.M, p.z, p.coeffs, weights)
    n, sm = len(p.freqs), int(np.sum(p.M))
    assert_close(fm[:, :n], c_ref, dtype, "forward, several right-hand sides")
    assert_close(am[:, :sm], y_ref, dtype, "adjoint, several right-hand sides")


@pytest.mark.parametrize("weights", ["paper", "eval"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_rhs_chunking_matches_one_pass(weights, dtype):
    """A work-area bound that holds three right-hand sides makes the plan loop over passes of 3, 3
    and 1 of its 7 right-hand sides (offset chunks, a short last one; the Fourier-matrix adjoint
    sums its bins per chunk after one counting sort): forward and adjoint are bit-identical to a
    plan that does all seven in one pass, and agree with the oracle."""
    torch = require_gpu()
    from paper_1711_05152_amd.mr1l import work_limit
    p = transform_problem(rng_for(951), 3000, 5, 16, 6, 3000, 9000, n_rhs=7)
    one = _plan(p, dtype, weights)
    esz = 8 if dtype == "c64" else 16
    region = int(one.fft_lengths.sum()) * esz
    default = work_limit(0)
    try:
        assert work_limit(3 * region + esz) == 3 * region + esz
        chunked = _plan(p, dtype, weights)
    finally:
        assert work_limit(-1) == default
    y = _to(torch, p.samples, dtype)
    c = _to(torch, p.coeffs, dtype)
    outs = []
    for plan in (one, chunked):
        outs.append((plan.forward(y).cpu().numpy(), plan.adjoint(c).cpu().numpy()))
    torch.cuda.synchronize()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a.view(np.float32 if dtype == "c64" else np.float64),
                              b.view(np.float32 if dtype == "c64" else np.float64))
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples, weights)
    y_ref = O.adjoint(p.freqs, p.M, p.z, p.coeffs, weights)
    assert_close(outs[1][0], c_ref, dtype, "chunked forward")
    assert_close(outs[1][1], y_ref, dtype, "chunked adjoint")
