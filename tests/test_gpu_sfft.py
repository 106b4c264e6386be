"""GPU parity of sfft_detect (Alg. 3 on the device) against the CPU oracle.

Detected frequency sets, per-step lattice sizes and sample counts must be bit-identical to the
oracle run with the same seed (same SplitMix64 streams on both sides); coefficients follow the
precision of the transforms.  The full-size d = 20 workload is checked through properties that
hold at any size (exact support recovery, coefficient error against the planted values).
"""
import importlib.util
import math
import os

import numpy as np
import pytest

from gpu_util import require_gpu, assert_close
from oracle.sfft import sfft as oracle_sfft, PlantedBlackBox
from workloads import S0, rng_for, random_planted, planted_c1, planted_c3, sweep_t52, sweep_t54

pytestmark = pytest.mark.gpu

SEED1 = 1711051521


def _lex(f):
    return np.lexsort(np.asarray(f).T[::-1])


def _run(p, dtype, delta, s, r, b=10, seed=SEED1, s_local=0, zero_anchors=False):
    from paper_1711_05152_amd.sfft import sfft_detect
    return sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed), delta=delta, s=s,
                       s_local=s_local, r=r, b=b, seed=seed, dtype=dtype, zero_anchors=zero_anchors, cap=max(s, 1))


def _compare_with_oracle(p, dtype, delta, s, r, b=10, seed=SEED1, s_local=0, zero_anchors=False):
    got = _run(p, dtype, delta, s, r, b, seed, s_local, zero_anchors)
    bb = PlantedBlackBox(p.freqs, p.coeffs, p.sigma, p.noise_seed)
    ref = oracle_sfft(p.lo, p.hi, bb, delta, s, s_local if s_local else s, r=r, b=b, seed=seed,
                      zero_anchors=zero_anchors)
    assert np.array_equal(got.freqs, ref.freqs), (got.freqs.shape, ref.freqs.shape)
    st = got.stats
    for step in ref.steps[1:]:
        t = step["t"]
        assert st["L"][t - 1] == step["L"], t
        assert st["sumM"][t - 1] == step["sumM"], t
        assert st["calls"][t - 1] == step["calls"], t
        assert st["n_J"][t - 1] == step["n_J"], t
    assert st["samples"] == ref.samples
    assert_close(got.coeffs, ref.coeffs, dtype, "sfft coefficients vs oracle")
    return got, ref


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_plain_d5_box8_s50(dtype):
    """d = 5, box [-8,8]^5, s = 50 unit-modulus coefficients, r = 1, delta = 1e-12 (complex128
    is the plain form; complex64 run for parity of the single-precision path)."""
    require_gpu()
    p = planted_c1()
    delta = 1e-12 if dtype == "c128" else 1e-4
    got, ref = _compare_with_oracle(p, dtype, delta, 50, 1)
    order = _lex(p.freqs)
    assert np.array_equal(got.freqs, p.freqs[order])
    if dtype == "c128":
        assert np.abs(got.coeffs - p.coeffs[order]).max() <= 1e-11


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noisy_repetitions_parity(dtype):
    """r = 3 detection iterations with complex Gaussian noise (Sec. 5.2 noise model)."""
    require_gpu()
    p = random_planted(rng_for(400), 5, 10, 120, "u1_10", sigma=1e-2, noise_seed=77)
    _compare_with_oracle(p, dtype, 1e-3 if dtype == "c128" else 2e-3, 120, 3, seed=5)


def test_selection_binds_s_local():
    """s_local smaller than the number of candidates above delta: top-s selection with ties by
    position decides the sets (same decision on both sides)."""
    require_gpu()
    p = random_planted(rng_for(401), 4, 6, 60, "u1_10")
    _compare_with_oracle(p, "c128", 1e-9, 40, 2, s_local=25, seed=6)


def test_zero_anchors_d1_and_empty():
    require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    # real parts of one sign: the r = 1 setting with anchors fixed to 0
    rng = rng_for(402)
    p = random_planted(rng, 4, 5, 30, "unit")
    p.coeffs = np.abs(p.coeffs.real) + 0.1 + 1j * p.coeffs.imag
    _compare_with_oracle(p, "c128", 1e-9, 30, 1, zero_anchors=True, seed=7)
    # d = 1
    p1 = random_planted(rng, 1, 20, 6, "unit")
    _compare_with_oracle(p1, "c128", 1e-9, 6, 2, seed=8)
    # empty black box -> empty output
    res = sfft_detect([-3, -3, -3], [3, 3, 3], planted=(np.zeros((0, 3), np.int32), np.zeros(0), 0.0, 0),
                      delta=1e-6, s=10, r=1, b=3, seed=1)
    assert res.freqs.shape == (0, 3)


def test_callback_sampler_matches_planted():
    """A caller-supplied black box (explicit nodes, evaluated here with torch on the device)
    detects the same set as the built-in planted black box."""
    torch = require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    p = random_planted(rng_for(403), 4, 5, 25, "unit")
    hf = torch.tensor(p.freqs, dtype=torch.float64, device="cuda:0")
    hc = torch.tensor(p.coeffs, dtype=torch.complex128, device="cuda:0")

    def sampler(x):
        ph = (x @ hf.T) % 1.0
        return torch.exp(2j * np.pi * ph) @ hc

    cb = sfft_detect(p.lo, p.hi, sampler=sampler, delta=1e-9, s=25, r=1, b=10, seed=9, dtype="c128")
    pl = _run(p, "c128", 1e-9, 25, 1, seed=9)
    assert np.array_equal(cb.freqs, pl.freqs)
    assert np.abs(cb.coeffs - pl.coeffs).max() < 1e-10
    assert np.array_equal(cb.freqs, p.freqs[_lex(p.freqs)])


_GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_module():
    spec = importlib.util.spec_from_file_location(
        "make_sfft_oracle_golden", os.path.join(_GOLDEN_DIR, "make_sfft_oracle_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _compare_with_golden(name, p, got, dtype, min_margin):
    """The library's solve against the oracle's stored solve of the same inputs (written by
    tests/golden/make_sfft_oracle_golden.py): detected set, per-step |I^(t)|, |J_t|, lattices,
    sizes, Alg. 1 calls and uncovered counts, sample count (all exact) and coefficients (R15).
    The oracle's smallest decision margin must leave room for the transform's rounding."""
    gm = _golden_module()
    g = np.load(gm.path(name))
    assert str(g["digest"]) == gm.input_digest(p), "golden file was made from other inputs"
    margin = float(g["margin"])
    print(f"{name}: oracle decision margin {margin:.3e}", flush=True)
    assert margin >= min_margin, f"oracle decision margin {margin:.3e} too close to rounding"
    assert np.array_equal(got.freqs, g["freqs"]), (got.freqs.shape, g["freqs"].shape)
    keys = [str(k) for k in g["step_keys"]]
    st = got.stats
    for row in g["steps"]:
        step = dict(zip(keys, (int(v) for v in row)))
        t = step["t"]
        assert st["n_It"][t - 1] == step["n_It"], (name, t)
        if t == 1:
            continue
        for k in ("n_J", "L", "sumM", "calls", "uncovered"):
            assert st[k][t - 1] == step[k], (name, t, k, st[k][t - 1], step[k])
    assert st["samples"] == int(g["samples"])
    assert st["samples_full"] == int(g["samples_full"])
    assert_close(got.coeffs, g["coeffs"], dtype, f"{name} coefficients vs oracle")


@pytest.mark.parametrize("sigma", [0.0, 1e-2])
def test_scale_d20_box32_s1000(sigma):
    """d = 20, box [-32,32]^20, s = 1000, |c| in [1,10], r = 5, delta = 1e-3, complex64 transforms:
    the oracle's solve of the same inputs (stored) is reproduced exactly (set, every step's
    lattices and counts, samples; coefficients within R15), the planted support is recovered
    exactly and the coefficient error against the planted values stays within the noise level."""
    require_gpu()
    p = planted_c3(sigma)
    got = _run(p, "c64", 1e-3, 1000, 5, seed=1711051523)
    _compare_with_golden("c3_sigma0" if sigma == 0 else "c3_sigma1e-2", p, got, "c64", 1e-2)
    order = _lex(p.freqs)
    assert np.array_equal(got.freqs, p.freqs[order])
    err = np.abs(got.coeffs - p.coeffs[order])
    print(f"sigma {sigma}: max coeff err {err.max():.3e}, samples {got.stats['samples']}, "
          f"ms {got.stats['ms_total']:.1f}", flush=True)
    assert err.max() <= (1e-4 * 10 if sigma == 0 else 1e-3)


def test_table52_setting_matches_oracle():
    """Setting of Table 5.2 (d = 5, N = 32, s = 1000, unit moduli, r = 2, delta = 0.1), complex128:
    the solve reproduces the oracle's stored solve of the same instance exactly."""
    require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    p = sweep_t52(0)
    got = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=0.1, s=1000, r=2, b=10,
                      seed=S0 + 52000, dtype="c128", cap=1000)
    _compare_with_golden("t52_r2_delta0.1", p, got, "c128", 1e-9)


def test_table54_setting_matches_oracle():
    """Setting of Table 5.4 (d = 10, N = 32, s = 1000, unit moduli, SNR 30 dB noise, r = 2,
    delta = 1e-12), complex128: the solve reproduces the oracle's stored solve exactly."""
    require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    p = sweep_t54(0, 30.0)
    got = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed), delta=1e-12, s=1000, r=2,
                      b=10, seed=S0 + 54000, dtype="c128", cap=1000)
    _compare_with_golden("t54_snr30_r2", p, got, "c128", 1e-9)


# ---- exhausted Alg. 1 retries (reading R4), failing black box, streams, reproducibility --------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("seed", [5, 42])
def test_uncovered_step_matches_oracle(seed, dtype):
    """Alg. 3 step 2b with a single Alg. 1 call (b = 1) that does not reconstruct J_t (c = 4 and
    gamma = 0.999 leave two to four lattices): the kept lattices, the per-step uncovered counts
    and the output (the uncovered frequency has counter 0, so it is never detected) equal the
    oracle's, and the library reports MR1L_WARN_UNCOVERED.  Seed 5 leaves a frequency uncovered at
    step 2 and misses a planted one; seed 42 at the last step."""
    require_gpu()
    from paper_1711_05152_amd import _lib
    from paper_1711_05152_amd.sfft import sfft_detect
    p = random_planted(rng_for(404), 3, 4, 8, "unit")
    delta = 1e-9 if dtype == "c128" else 1e-4     # above the rounding level of the transforms
    got = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=delta, s=8, r=1, b=1, seed=seed,
                      dtype=dtype, c=4.0, gamma=0.999, cap=8)
    ref = oracle_sfft(p.lo, p.hi, PlantedBlackBox(p.freqs, p.coeffs), delta, 8, r=1, b=1, seed=seed, c=4.0,
                      gamma=0.999)
    assert sum(step["uncovered"] for step in ref.steps[1:]) > 0
    assert got.status == _lib.MR1L_WARN_UNCOVERED
    assert np.array_equal(got.freqs, ref.freqs)
    assert got.freqs.shape[0] < 8 or seed != 5
    for step in ref.steps[1:]:
        t = step["t"]
        for k in ("L", "sumM", "calls", "uncovered", "n_J"):
            assert got.stats[k][t - 1] == step[k], (seed, t, k)
    assert got.stats["samples"] == ref.samples
    assert_close(got.coeffs, ref.coeffs, dtype, "coefficients after an uncovered step")


def test_failing_sampler_reports_callback_error():
    """A caller black box that fails (on the 1-D lines, or later on the lattice nodes) makes
    sfft_detect return MR1L_ERR_CALLBACK; the library stays usable afterwards."""
    torch = require_gpu()
    from paper_1711_05152_amd import _lib
    from paper_1711_05152_amd.sfft import sfft_detect
    p = planted_c1()
    hf = torch.tensor(p.freqs, dtype=torch.float64, device="cuda:0")
    hc = torch.tensor(p.coeffs, dtype=torch.complex128, device="cuda:0")
    K = int(p.hi[0] - p.lo[0] + 1)

    def fails_always(x):
        raise RuntimeError("black box failed")

    def fails_on_lattices(x):
        if x.shape[0] > K:
            raise RuntimeError("black box failed on a lattice")
        return torch.exp(2j * np.pi * ((x @ hf.T) % 1.0)) @ hc

    for sampler in (fails_always, fails_on_lattices):
        with pytest.raises(_lib.Mr1lError) as ei:
            sfft_detect(p.lo, p.hi, sampler=sampler, delta=1e-12, s=50, r=1, b=10, seed=SEED1, dtype="c128")
        assert ei.value.status == 5, ei.value
    res = _run(p, "c128", 1e-12, 50, 1)
    assert np.array_equal(res.freqs, p.freqs[_lex(p.freqs)])


def test_callback_sampler_on_non_default_stream():
    """The caller's black box runs on the library's stream (the one that wrote the nodes), also
    when torch's current stream is another one: same result as the built-in black box."""
    torch = require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    p = random_planted(rng_for(406), 4, 6, 40, "unit")
    hf = torch.tensor(p.freqs, dtype=torch.float64, device="cuda:0")
    hc = torch.tensor(p.coeffs, dtype=torch.complex128, device="cuda:0")

    def sampler(x):
        return torch.exp(2j * np.pi * ((x @ hf.T) % 1.0)) @ hc

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        cb = sfft_detect(p.lo, p.hi, sampler=sampler, delta=1e-9, s=40, r=2, b=10, seed=12, dtype="c128")
    torch.cuda.synchronize()
    pl = _run(p, "c128", 1e-9, 40, 2, seed=12)
    assert np.array_equal(cb.freqs, pl.freqs)
    assert np.abs(cb.coeffs - pl.coeffs).max() < 1e-10
    assert np.array_equal(cb.freqs, p.freqs[_lex(p.freqs)])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_solves_are_bit_reproducible(dtype):
    """Two identical solves (built-in noisy black box, repetitions as right-hand sides) give
    bit-identical coefficients and identical statistics: the synthesis of the samples sums every
    bin in a fixed order."""
    require_gpu()
    p = random_planted(rng_for(405), 5, 8, 50, "unit", sigma=1e-3, noise_seed=3)
    runs = [_run(p, dtype, 1e-2, 50, 2, seed=11) for _ in range(2)]
    a, b = runs
    assert np.array_equal(a.freqs, b.freqs)
    assert np.array_equal(a.coeffs.view(np.float64), b.coeffs.view(np.float64))
    for k in ("n_It", "n_J", "n_detected", "L", "sumM", "calls", "uncovered", "samples"):
        assert a.stats[k] == b.stats[k], k


# ---- construction variant with redraws, component order --------------------------------------------

def test_construct_redraw_matches_oracle():
    """mr1l_construct with redraws: lattice sizes and generating vectors identical to the oracle's
    variant (same streams, redraw a >= 1 keyed separately), and every lattice adds a frequency."""
    require_gpu()
    from paper_1711_05152_amd.mr1l import mr1l_construct
    from oracle import construct as Cn
    from oracle import mr1l as O
    from workloads import distinct_freqs
    hits = 0
    for rep in range(4):
        f = distinct_freqs(rng_for(340, rep), 900, 3, -40, 40)
        M, z, calls, unc = mr1l_construct(f, b=10, seed=40 + rep, t=2, redraw=64)
        stats: dict = {}
        Mo, zo, cov, callso = Cn.construct_retry(f, b=10, seed=40 + rep, t=2, redraw=64, stats=stats)
        assert np.array_equal(M, Mo) and np.array_equal(z, zo) and calls == callso and unc == 0
        hits += stats.get("redraws", 0)
    assert hits > 0   # the variant actually redrew on these sets


@pytest.mark.parametrize("n", [3000, 200_000, 270_000],
                         ids=["lds_bitmaps", "lds_bitmaps_above_64KiB", "global_atomics_above_2p19_bins"])
def test_construct_matches_oracle(n):
    """mr1l_construct (Alg. 1 itself, rounds of trial lattices): lattice sizes, generating vectors
    and the number of calls identical to the oracle's.  The sizes cover the three histogram paths
    of a round: LDS bitmaps, LDS bitmaps beyond 64 KiB (lattices of 2^18..2^19 bins) and global
    atomics (lattices above 2^19 bins, lambda = 2 (n - 1) > 2^19)."""
    require_gpu()
    from paper_1711_05152_amd.mr1l import mr1l_construct
    from oracle import construct as Cn
    from workloads import distinct_freqs
    f = distinct_freqs(rng_for(342, n), n, 6, -40, 40)
    print(f"construct n={n}", flush=True)
    M, z, calls, unc = mr1l_construct(f, b=10, seed=41, t=3)
    Mo, zo, cov, callso = Cn.construct_retry(f, b=10, seed=41, t=3)
    assert np.array_equal(M, Mo) and np.array_equal(z, zo) and calls == callso
    assert unc == 0 and cov


def test_sfft_redraw_and_order_match_oracle():
    """sfft_detect with the redraw variant and with a component order: detected sets, per-step
    lattices, redraw counts and sample counts identical to the oracle's runs; a caller-supplied
    sampler sees nodes in its own component order."""
    torch = require_gpu()
    from paper_1711_05152_amd.sfft import sfft_detect
    p = random_planted(rng_for(341), 5, 16, 400, "box")
    bb = PlantedBlackBox(p.freqs, p.coeffs)
    for redraw, order in ((64, None), (0, [3, 0, 4, 2, 1]), (64, [1, 2, 0, 4, 3])):
        got = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=1e-12, s=400, r=1, b=10, seed=77,
                          dtype="c128", redraw=redraw, order=order, cap=400)
        ref = oracle_sfft(p.lo, p.hi, bb, 1e-12, 400, r=1, b=10, seed=77, redraw=redraw, order=order)
        assert np.array_equal(got.freqs, ref.freqs), (redraw, order)
        for step in ref.steps[1:]:
            t = step["t"]
            assert got.stats["L"][t - 1] == step["L"] and got.stats["sumM"][t - 1] == step["sumM"]
            assert got.stats["redraws"][t - 1] == step["redraws"], (redraw, order, t)
        assert got.stats["samples"] == ref.samples
        assert_close(got.coeffs, ref.coeffs, "c128", f"sfft redraw {redraw} order {order}")
    # caller sampler, permuted order: same result as the built-in black box
    hf = torch.from_numpy(p.freqs.astype(np.float64)).to("cuda:0")
    hc = torch.from_numpy(p.coeffs).to("cuda:0")

    def sampler(x):
        return torch.exp(2j * np.pi * ((x @ hf.T) % 1.0)) @ hc

    order = [2, 4, 0, 1, 3]
    cb = sfft_detect(p.lo, p.hi, sampler=sampler, delta=1e-9, s=400, r=1, b=10, seed=78, dtype="c128", order=order)
    pl = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=1e-9, s=400, r=1, b=10, seed=78,
                     dtype="c128", order=order)
    assert np.array_equal(cb.freqs, pl.freqs)
    assert np.abs(cb.coeffs - pl.coeffs).max() < 1e-10
    assert set(map(tuple, cb.freqs.tolist())) == set(map(tuple, p.freqs.tolist()))


def _binomial_ok(k, n, p, slack=0.05):
    """k successes of n consistent with rate p (3 standard deviations plus slack)."""
    return abs(k / n - p) <= 3.0 * math.sqrt(max(p * (1 - p), 1e-12) / n) + slack


def test_success_rates_match_table_5_2():
    """Success rate of Alg. 3 on the setting of Table 5.2 (d = 5, N = 32, s = 1000, unit-modulus
    coefficients) for cells where the paper's rate is strictly between 0 and 1 or at an end:
    30 seeded instances per cell agree with the printed rates (1000 repetitions) within binomial
    error.  This checks the readings of the detection steps (e.g. the 1/K factor of the 1-D
    projections) against the paper's own runs."""
    require_gpu()
    import bench
    cells = {(1, 3e-1), (1, 1e-2), (2, 3e-1), (2, 1e-1), (3, 1e-2)}
    rows = bench.sweep_table52(30, cells)
    assert len(rows) == len(cells)
    for row in rows:
        print(row, flush=True)
        assert _binomial_ok(round(row["success_rate"] * 30), 30, row["paper_success_rate"]), row


def test_noise_success_rates_match_table_5_4():
    """Alg. 3 with complex Gaussian noise (setting of Table 5.4: d = 10, s = 1000, delta = 1e-12):
    success rates over 20 instances agree with the printed ones within binomial error, and the
    largest relative l2 error of the coefficients stays below three times the printed maximum."""
    require_gpu()
    import bench
    rows = bench.sweep_table54(20, {(30, 1), (50, 1), (30, 2), (0, 5)})
    assert len(rows) == 4
    for row in rows:
        print(row, flush=True)
        assert _binomial_ok(round(row["success_rate"] * 20), 20, row["paper_success_rate"], slack=0.1), row
        assert row["max_rel_l2_error"] <= 3 * row["paper_max_rel_l2_error"], row


def test_repeated_solves_reuse_staging_safely():
    """Many solves in a row: each call creates and destroys its own stream, while the pinned
    staging of step tables and the cached device blocks carry over between calls.  Every solve
    returns the same result."""
    require_gpu()
    p = planted_c1()
    first = None
    for i in range(30):
        res = _run(p, "c128" if i % 2 == 0 else "c64", 1e-12 if i % 2 == 0 else 1e-4, 50, 1)
        if first is None:
            first = res.freqs
        assert np.array_equal(res.freqs, first), i


def test_concurrent_solves_match_serial():
    """Independent solves on several host threads (each sfft_detect on its own stream, several
    in flight on the device) give bit-identical results to the same solves one after another."""
    require_gpu()
    import bench
    from paper_1711_05152_amd.sfft import sfft_detect
    probs = [random_planted(rng_for(407, i), 5, 16, 300, "unit", sigma=1e-3 * (i % 2), noise_seed=i)
             for i in range(8)]
    jobs = [lambda p=p, i=i: sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed),
                                         delta=1e-2, s=300, r=2, b=10, seed=100 + i,
                                         dtype="c64" if i % 3 == 0 else "c128", cap=300)
            for i, p in enumerate(probs)]
    serial = bench.solve_all(jobs, 1)
    concurrent = bench.solve_all(jobs, 4)
    for i, (a, b) in enumerate(zip(serial, concurrent)):
        assert np.array_equal(a.freqs, b.freqs), i
        assert np.array_equal(a.coeffs.view(np.float64), b.coeffs.view(np.float64)), i
        assert a.stats["samples"] == b.stats["samples"], i
