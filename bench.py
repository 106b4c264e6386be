"""Benchmark: multiple rank-1 lattice FFT, forward + adjoint, on one MI355X.

Workload (one "step"): the standalone transform pair on |I| = 2^16 frequencies drawn uniformly
from [-64,64]^10, L = 16 lattices with prime sizes uniform in [2^16, 2^17], complex64 samples
(CN(0,1)) already resident in HBM.  A step runs every stage of the hot path twice (forward:
residues, alias histograms, prime-length DFTs, gather; adjoint: residues, alias histograms,
scatter, prime-length DFTs).  value = |I| / (time of forward + adjoint) in frequencies per second.

Prints ONE JSON line (rank 0).  Extra fields: per-stage device times (HIP events on the launch
stream), the roofline of the dominant kernel, and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The CPU oracle legs run in spawned worker processes with one BLAS / OpenMP thread each (set here,
# before numpy is imported anywhere in this process, and inherited by every worker).
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
    os.environ[_v] = "1"

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak
FP64_VECTOR_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="budget of each standalone-workload leg of the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sparse-FFT, batched and gradient-descent workloads")
    ap.add_argument("--gd-steps", type=int, default=5)
    ap.add_argument("--only", choices=["sfft", "batched", "batched_plan", "autograd", "throughput"],
                    help="run only this extra workload and print its figures (for profiling it alone)")
    ap.add_argument("--sweeps", type=int, default=0, metavar="REPS",
                    help="also run the success-rate (Table 5.2 setting) and noise (Table 5.4 setting) "
                         "sweeps with REPS seeded instances per cell")
    ap.add_argument("--bspline-sweeps", type=int, default=0, metavar="REPS",
                    help="also run the B-spline test function sweeps (settings of Tables 5.7 and 5.8) with REPS "
                         "seeds per row")
    ap.add_argument("--bspline-max-N", type=int, default=256,
                    help="largest expansion N of the threshold-truncation rows")
    ap.add_argument("--emit-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="no GPU: turn the counter files of two rocprofv3 --pmc runs of this script "
                         "(FETCH_SIZE, then WRITE_SIZE, both with --copy-calibration) into the "
                         "per-launch HBM traffic file read by the roofline")
    return ap.parse_args()


# ---- HBM traffic from hardware counters ----------------------------------------------------------
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_mr1l_n65536_d10_L16_c64.json")
COPY_BYTES = 1 << 28            # the calibration copy (--copy-calibration): 256 MiB read + written
STAGE_OF_KERNEL = [("k_res_hist", "alias_hist"), ("k_hist_merge", "alias_hist"), ("k_p1<", "bluestein_p1"),
                   ("k_p2<", "bluestein_p2"), ("k_p3<", "bluestein_p3"), ("k_small<", "bluestein_small"),
                   ("k_gather", "gather"), ("k_scatter", "scatter")]


def kernel_sources_digest() -> str:
    """SHA-256 over every file of the HIP sources: the stored traffic is valid for this digest only."""
    import hashlib
    d = os.path.join(ROOT, "paper_1711_05152_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def emit_traffic(fetch_csv: str, write_csv: str, out_json: str) -> None:
    """Per-launch HBM bytes of each stage: counter KiB per dispatch of the fp32 workload kernels,
    scaled by (bytes moved / counter bytes) of the 256 MiB calibration copy measured in the same
    run; stages with two kernels add theirs."""
    import csv
    import collections

    def load(path, counter):
        per = collections.defaultdict(list)
        copy = 0.0
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            name = r["Kernel_Name"]
            if "copyBuffer" in name:
                copy = max(copy, v)
                continue
            if "<double" in name:       # plan-time filter construction
                continue
            for key, stage in STAGE_OF_KERNEL:
                if key in name:
                    per[(stage, name)].append(v)
                    break
        return per, copy

    fetch, fcopy = load(fetch_csv, "FETCH_SIZE")
    write, wcopy = load(write_csv, "WRITE_SIZE")
    if fcopy <= 0 or wcopy <= 0:
        raise SystemExit("no calibration copy in the counter files (run with --copy-calibration)")
    fs, ws = COPY_BYTES / fcopy, COPY_BYTES / wcopy
    # a stage launch runs one kernel per role (k_res_hist + k_hist_merge for the alias stage);
    # template variants of one role (e.g. stage 1 reading samples or bins) are averaged
    roles = collections.defaultdict(lambda: {"f": [], "w": [], "kernels": []})
    for (stage, name), vals in fetch.items():
        role = roles[(stage, name.split("<")[0].split("(")[0])]
        role["f"].extend(vals)
        role["w"].extend(write.get((stage, name), []))
        role["kernels"].append(name.split("(")[0])
    stages = collections.defaultdict(lambda: {"fetch_bytes": 0.0, "write_bytes": 0.0, "kernels": []})
    for (stage, _), role in roles.items():
        st = stages[stage]
        st["fetch_bytes"] += fs * sum(role["f"]) / len(role["f"])
        if role["w"]:
            st["write_bytes"] += ws * sum(role["w"]) / len(role["w"])
        st["kernels"] += role["kernels"]
    for st in stages.values():
        st["traffic_bytes"] = st["fetch_bytes"] + st["write_bytes"]
    out = {"source_sha256": kernel_sources_digest(),
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_counter_bytes": fcopy, "write_counter_bytes": wcopy,
                           "fetch_scale": fs, "write_scale": ws},
           "stages": dict(stages)}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({"written": out_json, "fetch_scale": fs, "write_scale": ws}))


def stored_traffic(stage: str):
    """HBM bytes per launch of ``stage`` from the stored counter file, or None when absent or
    taken from other kernel sources than the ones built here."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_sources_digest() or stage not in t.get("stages", {}):
        return None
    return t["stages"][stage]["traffic_bytes"]


def _sync():
    import torch
    torch.cuda.synchronize()


def extra_sfft():
    """Sparse FFT solves (Alg. 3 on the device): repetitions batched as right-hand sides vs one
    transform call per repetition ("plain")."""
    import numpy as np
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import planted_c1, planted_c3
    out = {}
    cases = [("d5_box8_s50_r1_c128", planted_c1(), "c128", 1e-12, 50, 1, 1711051521),
             ("d20_box32_s1000_r5_c64", planted_c3(0.0), "c64", 1e-3, 1000, 5, 1711051523),
             ("d20_box32_s1000_r5_c64_sigma1e-2", planted_c3(1e-2), "c64", 1e-3, 1000, 5, 1711051523)]
    for name, p, dt, delta, s, r, seed in cases:
        row = {}
        for mode in ("batched", "plain"):
            times, res = [], None
            for _ in range(3):
                res = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed), delta=delta,
                                  s=s, r=r, b=10, seed=seed, dtype=dt, plain=(mode == "plain"))
                times.append(res.stats["ms_total"])
            order = np.lexsort(p.freqs.T[::-1])
            ok = bool(np.array_equal(res.freqs, p.freqs[order]))
            st = res.stats
            row[mode] = {"ms_total_median": float(np.median(times)), "ms_excl_sampling": st["ms_total"] - st["ms_sampling"],
                         "ms_sampling": st["ms_sampling"], "ms_transform": st["ms_transform"],
                         "ms_construct": st["ms_construct"], "ms_select": st["ms_select"],
                         "samples": st["samples"], "support_recovered": ok,
                         "max_coeff_err": float(np.abs(res.coeffs - p.coeffs[order]).max()) if ok else None}
        row["batched_over_plain_time"] = row["batched"]["ms_total_median"] / row["plain"]["ms_total_median"]
        out[name] = row
    return out


def _golden(name):
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    return rows


def _recovery(res, p):
    """(number of planted frequencies detected, relative l2 error of the coefficient vector over
    the union of planted and detected frequencies)."""
    import numpy as np
    want = {tuple(k): c for k, c in zip(p.freqs.tolist(), p.coeffs)}
    got = {tuple(k): c for k, c in zip(res.freqs.tolist(), res.coeffs)}
    correct = sum(1 for k in got if k in want)
    err2 = sum(abs(got.get(k, 0.0) - c) ** 2 for k, c in want.items())
    err2 += sum(abs(c) ** 2 for k, c in got.items() if k not in want)
    return correct, math.sqrt(err2) / float(np.linalg.norm(p.coeffs))


def solve_all(jobs, workers: int = 1):
    """Run independent sparse-FFT solves: ``jobs`` is a list of zero-argument callables, each one
    solve.  With workers > 1 they run on that many host threads, each solve on its own HIP stream
    (sfft_detect creates one per call and releases the interpreter while it runs), so several
    solves are in flight on the device at once.  Results keep the order of ``jobs``."""
    if workers <= 1:
        return [job() for job in jobs]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda job: job(), jobs))


def sweep_table52(reps: int, cells=None, dtype: str = "c128", workers: int = 1):
    """Success rate and minimal number of correctly detected frequencies of Alg. 3 (setting of
    Table 5.2: d = 5, N = 32, s = 1000, unit-modulus coefficients) for each (r, delta) cell, over
    ``reps`` seeded instances (``workers`` solves in flight at once), beside the paper's values from
    1000 repetitions."""
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import S0, sweep_t52
    out = []
    for r, delta, pmin, prate in _golden("table52_mlfft_success.txt"):
        r = int(r)
        if cells is not None and (r, delta) not in cells:
            continue
        probs = [sweep_t52(rep) for rep in range(reps)]

        def job(rep, r=r, delta=delta):
            p = probs[rep]
            return sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=delta, s=1000, r=r, b=10,
                               seed=S0 + 52000 + rep, dtype=dtype, cap=1000)
        t0 = time.perf_counter()
        results = solve_all([lambda rep=rep: job(rep) for rep in range(reps)], workers)
        secs = time.perf_counter() - t0
        ok, mins = 0, []
        for p, res in zip(probs, results):
            correct, _ = _recovery(res, p)
            mins.append(correct)
            ok += correct == 1000
        out.append({"r": r, "delta": delta, "reps": reps, "success_rate": ok / max(1, reps),
                    "min_correct": min(mins) if mins else None, "paper_success_rate": prate,
                    "paper_min_correct": int(pmin), "paper_reps": 1000, "workers": workers,
                    "solves_per_s": reps / secs})
        print("sweep table 5.2 cell", json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def sweep_table54(reps: int, rows=None, dtype: str = "c128", workers: int = 1):
    """Alg. 3 on noisy samples (setting of Table 5.4: d = 10, N = 32, s = 1000, delta = 1e-12,
    sigma = sqrt(s / SNR)) for each (SNR dB, r) row over ``reps`` seeded instances (``workers``
    solves in flight at once): maximal sample count, minimal number of correctly detected
    frequencies, success rate, maximal relative l2 error, beside the paper's values from 1000
    repetitions."""
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import S0, sweep_t54
    out = []
    for snr, _sig, r, psamp, pmin, prate, perr in _golden("table54_mlfft_noise.txt"):
        r = int(r)
        if rows is not None and (int(snr), r) not in rows:
            continue
        probs = [sweep_t54(rep, snr) for rep in range(reps)]

        def job(rep, r=r):
            p = probs[rep]
            return sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed), delta=1e-12, s=1000,
                               r=r, b=10, seed=S0 + 54000 + rep, dtype=dtype, cap=1000)
        t0 = time.perf_counter()
        results = solve_all([lambda rep=rep: job(rep) for rep in range(reps)], workers)
        secs = time.perf_counter() - t0
        ok, mins, errs, samples = 0, [], [], []
        for p, res in zip(probs, results):
            correct, err = _recovery(res, p)
            mins.append(correct)
            errs.append(err)
            samples.append(res.stats["samples"])
            ok += correct == 1000
        out.append({"snr_db": int(snr), "sigma": math.sqrt(1000.0 / 10.0 ** (snr / 10.0)), "r": r, "reps": reps,
                    "max_samples": max(samples) if samples else None, "min_correct": min(mins) if mins else None,
                    "success_rate": ok / max(1, reps), "max_rel_l2_error": max(errs) if errs else None,
                    "paper_max_samples": int(psamp), "paper_min_correct": int(pmin), "paper_success_rate": prate,
                    "paper_max_rel_l2_error": perr, "paper_reps": 1000, "workers": workers,
                    "solves_per_s": reps / secs})
        print("sweep table 5.4 row", json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def sweep_table57(reps: int, rows=None, dtype: str = "c128"):
    """Alg. 3 on the 10-variate B-spline test function of Sec. 5.3 with s-sparse truncation (setting
    of Table 5.7: search space [-N,N]^10, r = 5, delta = 1e-12, s_local = 2s) for each (N, s) row
    over ``reps`` seeds: maximal sample count and maximal relative L2 error (the library's Parseval
    formula), median solve time, beside the paper's Alg. 3 values from 10 runs."""
    import numpy as np
    from paper_1711_05152_amd.sfft import paper_f10, sfft_detect
    from workloads import S0
    f = paper_f10(dtype)
    out = []
    for N, s, a5s, a5e, a3s, a3e, a4s, a4e in _golden("table57_bspline_ssparse.txt"):
        N, s = int(N), int(s)
        if rows is not None and (N, s) not in rows:
            continue
        errs, samples, ms, sizes = [], [], [], []
        for rep in range(reps):
            res = sfft_detect([-N] * 10, [N] * 10, bspline=f, delta=1e-12, s=s, s_local=2 * s, r=5, b=10,
                              seed=S0 + 57000 + rep, dtype=dtype, cap=s)
            errs.append(f.rel_l2_error(res.freqs, res.coeffs)[0])
            samples.append(res.stats["samples"])
            ms.append(res.stats["ms_total"])
            sizes.append(len(res.freqs))
        out.append({"N": N, "s": s, "reps": reps, "max_samples": max(samples), "max_rel_l2_error": max(errs),
                    "max_I": max(sizes), "ms_total_median": float(np.median(ms)),
                    "paper_alg3_max_samples": int(a3s), "paper_alg3_max_rel_l2_error": a3e,
                    "paper_alg5_max_samples": int(a5s), "paper_alg4_max_samples": int(a4s), "paper_reps": 10})
        print("sweep table 5.7 row", json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def sweep_table58(reps: int, rows=None, dtype: str = "c128", max_N: int = 1 << 30):
    """Alg. 3 on the B-spline test function with threshold truncation (setting of Table 5.8: search
    space [-N,N]^10, r = 10, s = |Gamma| (no sparsity cut), delta = threshold / 10 in the 1-D
    detections and delta = threshold elsewhere) over ``reps`` seeds: maximal |I|, maximal sample
    count, maximal relative L2 error and median solve time.  The paper prints Alg. 5 and Alg. 4
    columns for this table (no Alg. 3 column); both are carried along for context."""
    import numpy as np
    from paper_1711_05152_amd.sfft import paper_f10, sfft_detect
    from workloads import S0
    f = paper_f10(dtype)
    out = []
    for N, thr, a5i, a5s, a5e, a4i, a4s, a4e in _golden("table58_bspline_threshold.txt"):
        N = int(N)
        if N > max_N or (rows is not None and (N, thr) not in rows):
            continue
        errs, samples, ms, sizes = [], [], [], []
        for rep in range(reps):
            res = sfft_detect([-N] * 10, [N] * 10, bspline=f, delta=thr, delta_1d=thr / 10, s=1 << 62, r=10, b=10,
                              seed=S0 + 58000 + rep, dtype=dtype, cap=1 << 19)
            errs.append(f.rel_l2_error(res.freqs, res.coeffs)[0])
            samples.append(res.stats["samples"])
            ms.append(res.stats["ms_total"])
            sizes.append(len(res.freqs))
        out.append({"N": N, "threshold": thr, "reps": reps, "max_I": max(sizes), "max_samples": max(samples),
                    "max_rel_l2_error": max(errs), "ms_total_median": float(np.median(ms)),
                    "paper_alg5": {"max_I": int(a5i), "max_samples": int(a5s), "max_rel_l2_error": a5e},
                    "paper_alg4": {"max_I": int(a4i), "max_samples": int(a4s), "max_rel_l2_error": a4e},
                    "paper_reps": 10})
        print("sweep table 5.8 row", json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def extra_batched(with_plain: bool = True):
    """512 independent transforms (d=15, |I_b| log-uniform in [2^8,2^18], L_b = ceil(log2 |I_b|),
    primes in [|I_b|, 2|I_b|]), forward + adjoint per step, three ways: one batched plan whose small
    transforms (one-block Bluestein lengths, at most 2048 frequencies) run whole in the persistent
    in-block launch and the rest in the stage sweep (eager, and captured in a HIP graph); the same
    plan with every transform in the stage sweep; one plan per transform, launched one after
    another."""
    import numpy as np
    import torch
    from paper_1711_05152_amd.mr1l import BatchedPlan, Plan, batch_inblock
    from workloads import batched_c4
    probs = batched_c4(with_data=False)
    ntot = sum(p.n for p in probs)
    g = torch.Generator(device="cuda:0").manual_seed(4)
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
    try:
        batch_inblock(0)
        bs = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
    finally:
        batch_inblock(1)
    y = torch.randn(bp.sum_M, dtype=torch.complex64, device="cuda:0", generator=g)[None, :]
    c = torch.randn(bp.n, dtype=torch.complex64, device="cuda:0", generator=g)[None, :]
    co, yo = bp.empty_coeffs(), bp.empty_samples()

    def timeit(fn, reps=10):
        fn()
        _sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        _sync()
        return (time.perf_counter() - t0) * 1e3 / reps

    t_sweep = timeit(lambda: (bs.forward(y, out=co), bs.adjoint(c, out=yo)))
    t_batched = timeit(lambda: (bp.forward(y, out=co), bp.adjoint(c, out=yo)))
    gf = bp.capture("forward", y, co)
    ga = bp.capture("adjoint", c, yo)
    t_graph = timeit(lambda: (gf.replay(), ga.replay()))
    small = [b for b, p in enumerate(probs) if p.n <= 2048 and 2 * int(p.M.max()) - 1 <= 4096]
    out = {"transforms": len(probs), "sum_n": int(ntot), "sum_M": int(bp.sum_M),
           "inblock_transforms": len(small), "inblock_frequencies": int(sum(probs[b].n for b in small)),
           "ms_fwd_adj_stage_sweep": t_sweep, "ms_fwd_adj_batched": t_batched,
           "ms_fwd_adj_batched_graph": t_graph, "freqs_per_s_batched_graph": ntot / (t_graph * 1e-3),
           "stage_sweep_over_inblock": t_sweep / t_batched}
    del bs
    if not with_plain:
        return out
    plans = [Plan(p.freqs, p.M, p.z, dtype="c64", device=0) for p in probs]
    fo = np.concatenate([[0], np.cumsum([p.n for p in probs])])
    so = np.concatenate([[0], np.cumsum([int(p.M.sum()) for p in probs])])
    views = [(y[:, so[b]:so[b + 1]], c[:, fo[b]:fo[b + 1]], co[:, fo[b]:fo[b + 1]], yo[:, so[b]:so[b + 1]])
             for b in range(len(probs))]
    cos = [pl.empty_coeffs() for pl in plans]
    yos = [pl.empty_samples() for pl in plans]
    ys = [v[0].contiguous() for v in views]
    cs = [v[1].contiguous() for v in views]

    def plain():
        for b, pl in enumerate(plans):
            pl.forward(ys[b], out=cos[b])
            pl.adjoint(cs[b], out=yos[b])
    t_plain = timeit(plain, reps=3)
    out.update({"ms_fwd_adj_plain": t_plain, "freqs_per_s_plain": ntot / (t_plain * 1e-3),
                "plain_over_batched_graph": t_plain / t_graph})
    return out


def extra_sweep_throughput(reps: int = 16, workers: int = 8):
    """Independent solves of one sweep cell (Table 5.2 setting, r = 2, delta = 0.1, complex128):
    solves per second one after another and with ``workers`` solves in flight; the two runs give
    bit-identical results."""
    import numpy as np
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import S0, sweep_t52
    probs = [sweep_t52(rep) for rep in range(reps)]
    jobs = [lambda rep=rep: sfft_detect(probs[rep].lo, probs[rep].hi,
                                        planted=(probs[rep].freqs, probs[rep].coeffs, 0.0, 0), delta=0.1, s=1000,
                                        r=2, b=10, seed=S0 + 52000 + rep, dtype="c128", cap=1000)
            for rep in range(reps)]
    solve_all(jobs[:2], 1)   # warm-up
    out = {"cell": "d=5 N=32 s=1000 r=2 delta=0.1 complex128", "solves": reps}
    res = {}
    for w in (1, workers):
        t0 = time.perf_counter()
        res[w] = solve_all(jobs, w)
        out[f"solves_per_s_{w}_in_flight"] = reps / (time.perf_counter() - t0)
    out["identical"] = all(np.array_equal(a.freqs, b.freqs) and np.array_equal(a.coeffs, b.coeffs)
                           for a, b in zip(res[1], res[workers]))
    out["concurrent_over_serial"] = out[f"solves_per_s_{workers}_in_flight"] / out["solves_per_s_1_in_flight"]
    return out


def extra_autograd(steps: int):
    """Gradient descent on L(c) = 1/2 sum_l (1/M_l) ||A_l c - y_l||^2 with the differentiable
    Fourier-matrix transform: |I| = 2^20 in [-16,16]^30, L = 20 primes in [2^20, 2^21], 64
    right-hand sides, y = A c_true + complex Gaussian noise sigma = 1e-3, complex64."""
    import numpy as np
    import torch
    from paper_1711_05152_amd.autograd import Mr1lSynth, WeightedLsq
    from paper_1711_05152_amd.mr1l import Plan
    from workloads import lsq_c5
    freqs, M, z, seed = lsq_c5()
    n_rhs = 64
    ep = Plan(freqs, M, z, dtype="c64", weights="eval", n_rhs=n_rhs, device=0)
    g = torch.Generator(device="cuda:0").manual_seed(seed % (1 << 62))
    with torch.no_grad():
        c_true = torch.randn((n_rhs, ep.n), dtype=torch.complex64, device="cuda:0", generator=g)
        y = ep.adjoint(c_true)
        y += 1e-3 * torch.randn(y.shape, dtype=torch.complex64, device="cuda:0", generator=g)
        del c_true
        res, _, _ = ep.alias()
        step = 1.0 / sum(int(torch.bincount(res[l]).max()) for l in range(ep.L))
        del res
    c = torch.zeros((n_rhs, ep.n), dtype=torch.complex64, device="cuda:0", requires_grad=True)
    losses = []

    def gd_step():
        # fused residual, loss and loss gradient (one library pass over the samples each way)
        loss = WeightedLsq.apply(Mr1lSynth.apply(c, ep), y, ep)
        c.grad = None
        loss.backward()
        with torch.no_grad():
            c.add_(c.grad, alpha=-step)   # one fused elementwise pass
        return loss.detach()

    losses.append(float(gd_step()))
    _sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        losses.append(float(gd_step()))
    _sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"n": ep.n, "d": 30, "L": ep.L, "n_rhs": n_rhs, "sum_M": ep.sum_M, "ms_per_gd_step": ms,
            "steps_timed": steps, "loss_first": losses[0], "loss_last": losses[-1],
            "loss_monotone": all(b <= a for a, b in zip(losses, losses[1:]))}


# ---- CPU oracle baseline -----------------------------------------------------------------------------
# The oracle as it stands (FP64 NumPy, tier 1) on the host cores, in spawned worker processes with one
# thread each: a single-core leg (one worker, the paper's one-thread protocol) and an all-core leg
# (a pool over lattices or transforms, one process per core of the allowed set).  Every worker builds
# the seeded workloads itself; nothing GPU-side runs in them.
_CPU_STATE: dict = {}


def _cpu_c2():
    if "c2" not in _CPU_STATE:
        from workloads import standalone_c2
        _CPU_STATE["c2"] = standalone_c2()
    return _CPU_STATE["c2"]


def _cpu_c2_pairs(seconds: float):
    """Single core: forward + adjoint of the standalone workload, repeated for ``seconds``."""
    from oracle import mr1l as O
    p = _cpu_c2()
    iters, t0 = 0, time.perf_counter()
    while True:
        O.forward(p.freqs, p.M, p.z, p.samples)
        O.adjoint(p.freqs, p.M, p.z, p.coeffs)
        iters += 1
        if time.perf_counter() - t0 > seconds:
            break
    return iters, (time.perf_counter() - t0) / iters


def _cpu_c2_alias(l: int):
    from oracle import mr1l as O
    p = _cpu_c2()
    return O.unaliased_sets(p.freqs, p.M[l:l + 1], p.z[l:l + 1])[1][0]


def _cpu_c2_fwd(l: int):
    """Lattice l's term of Alg. 2: DFT_{M_l}(y_l)/M_l at the residues of I_l (0 elsewhere)."""
    from oracle import mr1l as O
    p = _cpu_c2()
    off = O.sample_offsets(p.M)
    return O.forward(p.freqs, p.M[l:l + 1], p.z[l:l + 1], p.samples[0, off[l]:off[l + 1]])


def _cpu_c2_adj(args):
    """Lattice l's slice of the adjoint for coefficients already divided by counter_k."""
    from oracle import mr1l as O
    l, cprime = args
    p = _cpu_c2()
    return O.adjoint(p.freqs, p.M[l:l + 1], p.z[l:l + 1], cprime)


def _cpu_c2_pair_pool(pool):
    """One forward + adjoint of the standalone workload with the lattices spread over the pool:
    alias sets per lattice, lattice terms summed in ascending l and divided by counter_k (forward);
    alias sets again, then each lattice's slice (adjoint)."""
    import numpy as np
    p = _cpu_c2()
    L = len(p.M)
    uniq = pool.map(_cpu_c2_alias, range(L))
    counter = np.sum(uniq, axis=0)
    terms = pool.map(_cpu_c2_fwd, range(L))
    c = np.zeros(p.n, np.complex128)
    for t in terms:
        c += t
    cov = counter > 0
    c[cov] /= counter[cov]
    c[~cov] = 0.0
    uniq = pool.map(_cpu_c2_alias, range(L))
    counter = np.sum(uniq, axis=0)
    cp = np.where(counter > 0, p.coeffs[0] / np.maximum(counter, 1), 0.0)
    y = np.concatenate(pool.map(_cpu_c2_adj, [(l, cp) for l in range(L)]))
    return c, y


class _TimedBlackBox:
    """The oracle's planted black box with the time spent sampling accumulated (the paper reports
    its solve times without it)."""

    def __init__(self, bb):
        self.bb, self.d, self.seconds = bb, bb.d, 0.0

    def sample_1d(self, *a, **k):
        t0 = time.perf_counter()
        y = self.bb.sample_1d(*a, **k)
        self.seconds += time.perf_counter() - t0
        return y

    def sample_lattice(self, *a, **k):
        t0 = time.perf_counter()
        y = self.bb.sample_lattice(*a, **k)
        self.seconds += time.perf_counter() - t0
        return y


def _cpu_solve(case: str):
    """One oracle solve (Alg. 3) of the plain (d = 5) or at-scale (d = 20) workload."""
    from oracle.sfft import PlantedBlackBox, sfft
    from workloads import planted_c1, planted_c3
    if case == "d5_box8_s50_r1":
        p, kw = planted_c1(), dict(delta=1e-12, s=50, r=1, seed=1711051521)
    else:
        p = planted_c3(1e-2 if case.endswith("sigma1e-2") else 0.0)
        kw = dict(delta=1e-3, s=1000, r=5, seed=1711051523)
    bb = _TimedBlackBox(PlantedBlackBox(p.freqs, p.coeffs, p.sigma, p.noise_seed))
    t0 = time.perf_counter()
    res = sfft(p.lo, p.hi, bb, kw["delta"], kw["s"], kw["s"], r=kw["r"], b=10, seed=kw["seed"])
    total = time.perf_counter() - t0
    return {"s_total": total, "s_excl_sampling": total - bb.seconds, "s_sampling": bb.seconds,
            "detected": int(res.freqs.shape[0]), "samples": int(res.samples)}


_C4_SUBSET = 16


def _cpu_c4_problem(b: int):
    key = ("c4", b)
    if key not in _CPU_STATE:
        import numpy as np
        from workloads import batched_c4, cn01, rng_for
        q = batched_c4(count=_C4_SUBSET, with_data=False)[b]
        rng = rng_for(4, 1000 + b)
        _CPU_STATE[key] = (q, cn01(rng, (int(q.M.sum()),)), cn01(rng, (q.n,)))
    return _CPU_STATE[key]


def _cpu_c4_pair(b: int):
    """Forward + adjoint of transform b of the 512-transform batch (the first 16 are the subset)."""
    from oracle import mr1l as O
    q, y, c = _cpu_c4_problem(b)
    t0 = time.perf_counter()
    O.forward(q.freqs, q.M, q.z, y)
    O.adjoint(q.freqs, q.M, q.z, c)
    return q.n, time.perf_counter() - t0


_C5_LATS = 2


def _cpu_c5_part(l: int):
    """Lattice l's share of one right-hand side of a gradient step of the least-squares workload:
    synthesis A_l c, weighted residual (1/M_l)(A_l c - y_l), and A_l^* of it (Fourier-matrix
    weighting)."""
    import numpy as np
    from oracle import mr1l as O
    if "c5" not in _CPU_STATE:
        from workloads import cn01, lsq_c5, rng_for
        freqs, M, z, _ = lsq_c5()
        _CPU_STATE["c5"] = (freqs, M, z, cn01(rng_for(5, 1000), (freqs.shape[0],)))
    freqs, M, z, c = _CPU_STATE["c5"]
    rng = np.random.default_rng(l)
    y = rng.standard_normal(int(M[l])) + 1j * rng.standard_normal(int(M[l]))
    t0 = time.perf_counter()
    s_l = O.adjoint(freqs, M[l:l + 1], z[l:l + 1], c, "eval")
    r_l = (s_l - y) / float(M[l])
    O.forward(freqs, M[l:l + 1], z[l:l + 1], r_l, "eval")
    return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(seconds: float):
    """All CPU oracle figures of the bench line (see the module docstring for the workloads)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import mr1l as O
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    P = max(1, min(16, allowed))
    ctx = mp.get_context("spawn")
    out = {"cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(), "cores_allowed": allowed,
           "threads_per_process": 1}
    with ctx.Pool(P) as pool:
        # the headline single-core leg alone, then the other single-core legs side by side (one
        # process each): the two d = 20 solves, the d = 5 solve, the batch and gradient-step subsets
        iters, t_pair = pool.apply_async(_cpu_c2_pairs, (seconds,)).get()
        jobs = {name: pool.apply_async(_cpu_solve, (name,))
                for name in ("d20_box32_s1000_r5", "d20_box32_s1000_r5_sigma1e-2", "d5_box8_s50_r1")}
        c4_one = pool.apply_async(_cpu_c4_all, ())
        c5_one = pool.apply_async(_cpu_c5_sequential, ())
        n4, t4 = c4_one.get()
        t5 = c5_one.get()
        solves = {k: j.get() for k, j in jobs.items()}
        _progress("cpu oracle single-core legs done")
        # all-core legs (the pool is idle now)
        p = _cpu_c2()
        c, y = _cpu_c2_pair_pool(pool)          # warm-up and check against the oracle's own call
        assert np.allclose(c, O.forward(p.freqs, p.M, p.z, p.samples)[0], atol=1e-12)
        assert np.allclose(y, O.adjoint(p.freqs, p.M, p.z, p.coeffs)[0], atol=1e-12)
        k, t0 = 0, time.perf_counter()
        while True:
            _cpu_c2_pair_pool(pool)
            k += 1
            if time.perf_counter() - t0 > seconds:
                break
        t_pair_all = (time.perf_counter() - t0) / k
        t0 = time.perf_counter()
        r4 = pool.map(_cpu_c4_pair, range(_C4_SUBSET))
        t4_all = time.perf_counter() - t0
        t0 = time.perf_counter()
        nl5 = min(P, 20)
        pool.map(_cpu_c5_part, range(nl5))
        t5_all = time.perf_counter() - t0
        _progress("cpu oracle all-core legs done")
    n = _cpu_c2().n
    out["standalone"] = {
        "single_core": {"freqs_per_s": n / t_pair, "s_per_pair": t_pair, "pairs": iters},
        "all_cores": {"freqs_per_s": n / t_pair_all, "s_per_pair": t_pair_all, "pairs": k, "processes": P,
                      "split": "lattices over processes"}}
    out["sfft_solves"] = solves
    out["batched_512_subset"] = {
        "sample": f"first {_C4_SUBSET} of the 512 transforms ({n4} frequencies), forward + adjoint each",
        "single_core_freqs_per_s": n4 / t4, "all_cores_freqs_per_s": sum(r[0] for r in r4) / t4_all,
        "all_cores_processes": P}
    out["gd_step_subset"] = {
        "sample": f"{_C5_LATS} of 20 lattices of 1 of 64 right-hand sides (single core), {nl5} lattices of 1 "
                  f"right-hand side (all cores); scaled to the whole step",
        "single_core_s_per_step_est": t5 * (20 / _C5_LATS) * 64,
        "all_cores_s_per_step_est": t5_all * (20 / nl5) * 64, "all_cores_processes": P}
    return out, P, t_pair, t_pair_all


def _cpu_c4_all():
    tot_n, tot_t = 0, 0.0
    for b in range(_C4_SUBSET):
        nb, tb = _cpu_c4_pair(b)
        tot_n += nb
        tot_t += tb
    return tot_n, tot_t


def _cpu_c5_sequential():
    return sum(_cpu_c5_part(l) for l in range(_C5_LATS))


def measure_standalone(p, dtype: str, steps: int, warmup: int) -> dict:
    """Forward + adjoint steps of one plan of the standalone workload: the headline loop (HIP events
    on the launch stream around all steps), the plan-cached loop, and a loop with the library's
    per-stage events (its own step time reported beside the plain one)."""
    import torch
    from paper_1711_05152_amd.mr1l import Plan
    dev = torch.device("cuda", 0)
    tdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]
    plan = Plan(p.freqs, p.M, p.z, dtype=dtype, weights="paper", n_rhs=1, device=0)
    y = torch.from_numpy(p.samples).to(dev, tdt)
    c_in = torch.from_numpy(p.coeffs).to(dev, tdt)
    c_out = plan.empty_coeffs()
    y_out = plan.empty_samples()

    def step():
        plan.forward(y, out=c_out)
        plan.adjoint(c_in, out=y_out)

    stream = torch.cuda.current_stream(dev)

    def loop():
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, (time.perf_counter() - t0) * 1e3 / steps

    ms_event, ms_wall = loop()
    plan.cache_alias(True)
    ms_cached, _ = loop()
    plan.cache_alias(False)
    plan.timing(True)
    ms_event_timed, _ = loop()
    stages = plan.timing_read()
    plan.timing(False)
    # timing_read covers the warm-up calls of the last loop as well
    calls = steps + warmup
    out = {"ms_event": ms_event, "ms_wall": ms_wall, "ms_cached": ms_cached, "ms_event_timed": ms_event_timed,
           "per_launch": {k: v[0] / v[1] for k, v in stages.items()},
           "per_step": {k: v[0] / calls for k, v in stages.items()},
           "fft_lengths": [int(v) for v in plan.fft_lengths]}
    plan.close()
    return out


def bluestein_alu(stage: str, ms: float, Ns, dtype: str):
    """Nominal FFT flops (5 N log2 N per transform) a Bluestein stage launch executes, with the
    four-step split the library uses for each length, over the launch time, against the vector peak
    (diagnostic: Bluestein's padded lengths are not the method's algorithmic work)."""
    import ctypes as C
    from paper_1711_05152_amd import _lib
    code = _lib.C64 if dtype == "c64" else _lib.C128
    flops = 0.0
    for N in Ns:
        if stage == "bluestein_small":
            flops += 2 * fft_flops(N)
            continue
        if N % 3 == 0:
            # N = 3 * 2^lg: one compiled split, the factor 3 in the stage-2 rows
            lg = int(round(math.log2(N // 3)))
            lg1 = max(lg - 10, min((lg + 1) // 2, 8))
        else:
            lg = int(round(math.log2(N)))
            cur = C.c_int(0)
            if _lib.lib().mr1l_fft_split(code, lg, 0, C.byref(cur)) != 0:
                return None
            lg1 = cur.value
        n1, n2 = 1 << lg1, N >> lg1
        if stage == "bluestein_p2":
            flops += 2 * fft_flops(n2) * n1
        elif stage in ("bluestein_p1", "bluestein_p3"):
            flops += fft_flops(n1) * n2
        else:
            return None
    peak = FP32_VECTOR_TFLOPS if dtype == "c64" else FP64_VECTOR_TFLOPS
    achieved = flops / (ms * 1e-3) / 1e12
    return {"achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "flops": flops}


def _progress(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def fft_flops(N: int) -> float:
    """Nominal cost of a complex FFT of length N (5 N log2 N)."""
    return 5.0 * N * math.log2(N) if N > 1 else 0.0


def main():
    args = parse()
    if args.emit_traffic:
        emit_traffic(*args.emit_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1 (multi-GPU sharding "
                                   "is described in DESIGN.md, not implemented)"}))
        sys.exit(2)
    import torch

    from workloads import standalone_c2

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only:
        fn = {"sfft": extra_sfft, "batched": extra_batched, "batched_plan": lambda: extra_batched(False),
              "autograd": lambda: extra_autograd(args.gd_steps),
              "throughput": extra_sweep_throughput}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    p = standalone_c2()
    n, d, L = p.n, p.d, len(p.M)
    sumM = int(p.M.sum())
    m64 = measure_standalone(p, "c64", args.steps, args.warmup)
    _progress(f"headline timed: {m64['ms_event']:.4f} ms/step, plan-cached {m64['ms_cached']:.4f} ms/step")
    ms_event, ms_wall, ms_cached = m64["ms_event"], m64["ms_wall"], m64["ms_cached"]
    per_launch, per_step, Ns = m64["per_launch"], m64["per_step"], m64["fft_lengths"]

    # ---- roofline of the dominant kernel ------------------------------------------------------------
    # Every stage launch processes one direction of the whole transform (all L lattices), whose
    # algorithmic bytes are 8 sum M_l (samples) + n d (packed int8 frequencies) + 8 n (coefficients).
    alg_dir = 8 * sumM + n * d * 1 + 8 * n
    dom = max(per_step, key=per_step.get)
    dom_ms = per_launch[dom]
    achieved = alg_dir / (dom_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom), "avg_launch_ms": dom_ms,
            "work_per_launch": alg_dir,
            "work_note": "algorithmic bytes of one direction (8 sum M + n d + 8 n), the units one launch of "
                         "any stage processes; avg_launch_ms from HIP events around each launch",
            "alu_diagnostic": bluestein_alu(dom, dom_ms, Ns, "c64")}

    # measured memory traffic (stored counter file of these sources) over each stage's launch time
    kernel_traffic = {}
    for k, t_ms in per_launch.items():
        b = stored_traffic(k)
        if b is not None:
            kernel_traffic[k] = {"bytes_per_launch": b, "GBs": b / (t_ms * 1e-3) / 1e9,
                                 "frac_hbm_peak": b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "traffic_over_algorithmic": b / alg_dir}

    # end-to-end algorithmic bytes (samples + packed frequencies + coefficients, both directions)
    alg_bytes = 2 * alg_dir
    e2e = {"alg_bytes_per_step": alg_bytes, "GBs": alg_bytes / (ms_event * 1e-3) / 1e9,
           "frac_hbm": alg_bytes / (ms_event * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if kernel_traffic and len(kernel_traffic) == len(per_launch):
        step_traffic = sum(kernel_traffic[k]["bytes_per_launch"] * (per_step[k] / per_launch[k])
                           for k in per_launch)
        e2e["measured_traffic_per_step"] = step_traffic
        e2e["traffic_over_algorithmic"] = step_traffic / alg_bytes

    # complex128 companion of the same workload (the paper computes in IEEE double)
    m128 = measure_standalone(p, "c128", args.steps, args.warmup)
    alg_dir128 = 16 * sumM + n * d * 1 + 16 * n
    dom128 = max(m128["per_step"], key=m128["per_step"].get)
    c128 = {"value": n / (m128["ms_event"] * 1e-3), "unit": "freqs/s", "ms_per_step": m128["ms_event"],
            "plan_cached_ms_per_step": m128["ms_cached"], "stages_ms_per_launch": m128["per_launch"],
            "dominant_kernel": dom128,
            "roofline_frac_hbm": alg_dir128 / (m128["per_launch"][dom128] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "alg_bytes_per_direction": alg_dir128,
            "end_to_end_frac_hbm": 2 * alg_dir128 / (m128["ms_event"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    _progress(f"complex128 companion timed: {m128['ms_event']:.4f} ms/step")

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    # ---- CPU oracle baseline ------------------------------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        detail, P, t_one, t_all = cpu_baseline(args.cpu_seconds)
        _progress(f"cpu oracle baseline: {t_one:.3f} s per pair on one core, {t_all:.3f} s on {P}")
        cpu = {"value": n / t_all, "unit": "freqs/s", "cores": P, "kind": "oracle",
               "sample": f"forward+adjoint pairs of the same |I|=2^16 workload for {args.cpu_seconds:.0f} s "
                         f"(numpy FFT tier, FP64), lattices spread over {P} single-threaded processes; "
                         f"one core: {n / t_one:.4g} freqs/s",
               "single_core_value": n / t_one, **detail}

    line = {
        "metric": "mr1l-FFT freqs/s fwd+adj (|I|=2^16,d=10)",
        "value": n / (ms_event * 1e-3),
        "unit": "freqs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_event,
        "ms_per_step_wall": ms_wall,
        "ms_per_step_stage_timed": m64["ms_event_timed"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "standalone mr1l-FFT forward+adjoint: |I|=2^16 uniform in [-64,64]^10, "
                               "L=16 prime M_l uniform in [2^16,2^17], complex64 samples CN(0,1)",
                   "n": n, "d": d, "L": L, "sum_M": sumM, "fft_lengths": sorted(set(Ns)),
                   "residues": "exact (int32 when d max|k| max M < 2^31, else int64)"},
        "plan_cached": {"value": n / (ms_cached * 1e-3), "unit": "freqs/s", "ms_per_step": ms_cached,
                        "note": "residues and alias bitmaps computed once per plan, not per call"},
        "roofline": roof,
        "end_to_end": e2e,
        "stages_ms_per_step": per_step,
        "stages_ms_per_launch": per_launch,
        "stages_measured_traffic": kernel_traffic or None,
        "c128": c128,
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        extra = {"sfft": extra_sfft()}
        _progress("sparse FFT solve timed")
        extra["batched_512"] = extra_batched()
        _progress("batched transforms timed")
        extra["autograd_lsq"] = extra_autograd(args.gd_steps)
        _progress("gradient-descent steps timed")
        extra["sweep_throughput"] = extra_sweep_throughput()
        _progress("independent solves timed")
        line["extra"] = extra
    if args.sweeps > 0:
        t0 = time.perf_counter()
        line["sweeps"] = {"table52_success": sweep_table52(args.sweeps), "table54_noise": sweep_table54(args.sweeps)}
        line["sweeps"]["seconds"] = time.perf_counter() - t0
    if args.bspline_sweeps > 0:
        t0 = time.perf_counter()
        line["bspline_sweeps"] = {"table57_ssparse": sweep_table57(args.bspline_sweeps),
                                  "table58_threshold": sweep_table58(args.bspline_sweeps, max_N=args.bspline_max_N)}
        line["bspline_sweeps"]["seconds"] = time.perf_counter() - t0
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
