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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak
FP64_VECTOR_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sparse-FFT, batched and gradient-descent workloads")
    ap.add_argument("--gd-steps", type=int, default=5)
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


def sweep_table52(reps: int, cells=None, dtype: str = "c128"):
    """Success rate and minimal number of correctly detected frequencies of Alg. 3 (setting of
    Table 5.2: d = 5, N = 32, s = 1000, unit-modulus coefficients) for each (r, delta) cell, over
    ``reps`` seeded instances, beside the paper's values from 1000 repetitions."""
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import S0, sweep_t52
    out = []
    for r, delta, pmin, prate in _golden("table52_mlfft_success.txt"):
        r = int(r)
        if cells is not None and (r, delta) not in cells:
            continue
        ok, mins = 0, []
        for rep in range(reps):
            p = sweep_t52(rep)
            res = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, 0.0, 0), delta=delta, s=1000, r=r, b=10,
                              seed=S0 + 52000 + rep, dtype=dtype, cap=1000)
            correct, _ = _recovery(res, p)
            mins.append(correct)
            ok += correct == 1000
        out.append({"r": r, "delta": delta, "reps": reps, "success_rate": ok / max(1, reps),
                    "min_correct": min(mins) if mins else None, "paper_success_rate": prate,
                    "paper_min_correct": int(pmin), "paper_reps": 1000})
        print("sweep table 5.2 cell", json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def sweep_table54(reps: int, rows=None, dtype: str = "c128"):
    """Alg. 3 on noisy samples (setting of Table 5.4: d = 10, N = 32, s = 1000, delta = 1e-12,
    sigma = sqrt(s / SNR)) for each (SNR dB, r) row over ``reps`` seeded instances: maximal sample
    count, minimal number of correctly detected frequencies, success rate, maximal relative l2
    error, beside the paper's values from 1000 repetitions."""
    from paper_1711_05152_amd.sfft import sfft_detect
    from workloads import S0, sweep_t54
    out = []
    for snr, _sig, r, psamp, pmin, prate, perr in _golden("table54_mlfft_noise.txt"):
        r = int(r)
        if rows is not None and (int(snr), r) not in rows:
            continue
        ok, mins, errs, samples = 0, [], [], []
        for rep in range(reps):
            p = sweep_t54(rep, snr)
            res = sfft_detect(p.lo, p.hi, planted=(p.freqs, p.coeffs, p.sigma, p.noise_seed), delta=1e-12, s=1000,
                              r=r, b=10, seed=S0 + 54000 + rep, dtype=dtype, cap=1000)
            correct, err = _recovery(res, p)
            mins.append(correct)
            errs.append(err)
            samples.append(res.stats["samples"])
            ok += correct == 1000
        out.append({"snr_db": int(snr), "sigma": math.sqrt(1000.0 / 10.0 ** (snr / 10.0)), "r": r, "reps": reps,
                    "max_samples": max(samples) if samples else None, "min_correct": min(mins) if mins else None,
                    "success_rate": ok / max(1, reps), "max_rel_l2_error": max(errs) if errs else None,
                    "paper_max_samples": int(psamp), "paper_min_correct": int(pmin), "paper_success_rate": prate,
                    "paper_max_rel_l2_error": perr, "paper_reps": 1000})
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


def extra_batched():
    """512 independent transforms (d=15, |I_b| log-uniform in [2^8,2^18], L_b = ceil(log2 |I_b|),
    primes in [|I_b|, 2|I_b|]): one batched plan (eager and HIP-graph replay) vs one plan per
    transform launched one after another.  Forward + adjoint per step."""
    import numpy as np
    import torch
    from paper_1711_05152_amd.mr1l import BatchedPlan, Plan
    from workloads import batched_c4
    probs = batched_c4(with_data=False)
    ntot = sum(p.n for p in probs)
    g = torch.Generator(device="cuda:0").manual_seed(4)
    bp = BatchedPlan([(p.freqs, p.M, p.z) for p in probs], dtype="c64", device=0)
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

    t_batched = timeit(lambda: (bp.forward(y, out=co), bp.adjoint(c, out=yo)))
    gf = bp.capture("forward", y, co)
    ga = bp.capture("adjoint", c, yo)
    t_graph = timeit(lambda: (gf.replay(), ga.replay()))
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
    return {"transforms": len(probs), "sum_n": int(ntot), "sum_M": int(bp.sum_M),
            "ms_fwd_adj_batched": t_batched, "ms_fwd_adj_batched_graph": t_graph, "ms_fwd_adj_plain": t_plain,
            "freqs_per_s_batched_graph": ntot / (t_graph * 1e-3), "freqs_per_s_plain": ntot / (t_plain * 1e-3),
            "plain_over_batched_graph": t_plain / t_graph}


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
            c.sub_(step * c.grad)
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
    import numpy as np
    import torch

    from paper_1711_05152_amd.mr1l import Plan
    from workloads import standalone_c2

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = standalone_c2()
    n, d, L = p.n, p.d, len(p.M)
    sumM = int(p.M.sum())
    plan = Plan(p.freqs, p.M, p.z, dtype="c64", weights="paper", n_rhs=1, device=0)
    y = torch.from_numpy(p.samples).to(dev, torch.complex64)
    c_in = torch.from_numpy(p.coeffs).to(dev, torch.complex64)
    c_out = plan.empty_coeffs()
    y_out = plan.empty_samples()

    def step():
        plan.forward(y, out=c_out)
        plan.adjoint(c_in, out=y_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_wall = (t1 - t0) * 1e3 / args.steps
    ms_event = ev0.elapsed_time(ev1) / args.steps

    # plan-cached variant: residues and alias bitmaps computed once and reused by every call
    plan.cache_alias(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev4 = torch.cuda.Event(enable_timing=True)
    ev5 = torch.cuda.Event(enable_timing=True)
    ev4.record(stream)
    for _ in range(args.steps):
        step()
    ev5.record(stream)
    torch.cuda.synchronize()
    ms_cached = ev4.elapsed_time(ev5) / args.steps
    plan.cache_alias(False)
    _progress(f"headline timed: {ms_event:.4f} ms/step, plan-cached {ms_cached:.4f} ms/step")

    # per-stage device time: HIP events recorded by the library on the stream of each launch, over
    # a second timed loop of the same steps (its own step time is reported beside the plain one)
    plan.timing(True)
    ev2 = torch.cuda.Event(enable_timing=True)
    ev3 = torch.cuda.Event(enable_timing=True)
    ev2.record(stream)
    for _ in range(args.steps):
        step()
    ev3.record(stream)
    torch.cuda.synchronize()
    ms_event_timed = ev2.elapsed_time(ev3) / args.steps
    stages = plan.timing_read()
    plan.timing(False)
    per_launch = {k: v[0] / v[1] for k, v in stages.items()}
    per_step = {k: v[0] / args.steps for k, v in stages.items()}

    # ---- roofline of the dominant kernel ------------------------------------------------------------
    Ns = [int(v) for v in plan.fft_lengths]
    dom = max(per_step, key=per_step.get)
    lg = [int(round(math.log2(N))) for N in Ns]
    # four-step split of the library: N = N1 N2, N1 = 2^max(lgN - 12, min(lgN // 2, 8))
    lg1 = [max(g - 12, min(g // 2, 8)) for g in lg]
    if dom == "bluestein_p2":
        # row FFTs (forward + inverse) of length N2 on N1 rows, per lattice, nominal 5 N log2 N each
        flops = sum(2 * fft_flops(1 << (g - g1)) * (1 << g1) for g, g1 in zip(lg, lg1))
    elif dom in ("bluestein_p1", "bluestein_p3"):
        flops = sum(fft_flops(1 << g1) * (1 << (g - g1)) for g, g1 in zip(lg, lg1))
    elif dom == "bluestein_small":
        flops = sum(2 * fft_flops(N) for N in Ns)
    else:
        flops = None
    dom_ms = per_launch[dom]
    if flops is not None:
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_TFLOPS, "traffic": stored_traffic(dom),
                "avg_launch_ms": dom_ms, "work_per_launch": flops}
    else:
        nbytes = 8 * sumM + n * d + 8 * n
        achieved = nbytes / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom), "avg_launch_ms": dom_ms,
                "work_per_launch": nbytes}

    # measured memory traffic (stored counter file of these sources) over each stage's launch time
    kernel_traffic = {}
    for k, t_ms in per_launch.items():
        b = stored_traffic(k)
        if b is not None:
            kernel_traffic[k] = {"bytes_per_launch": b, "GBs": b / (t_ms * 1e-3) / 1e9,
                                 "frac_hbm_peak": b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # end-to-end algorithmic bytes (samples + packed frequencies + coefficients, both directions)
    alg_bytes = 2 * (8 * sumM + n * d * 1 + 8 * n)
    e2e = {"alg_bytes_per_step": alg_bytes, "GBs": alg_bytes / (ms_event * 1e-3) / 1e9,
           "frac_hbm": alg_bytes / (ms_event * 1e-3) / 1e9 / HBM_PEAK_GBS}

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
        from oracle import mr1l as O
        threads = 1
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        iters = 0
        tc0 = time.perf_counter()
        while True:
            O.forward(p.freqs, p.M, p.z, p.samples)
            O.adjoint(p.freqs, p.M, p.z, p.coeffs)
            iters += 1
            if time.perf_counter() - tc0 > args.cpu_seconds:
                break
        tcpu = (time.perf_counter() - tc0) / iters
        _progress(f"cpu oracle baseline: {iters} pairs, {tcpu:.3f} s each")
        cpu = {"value": n / tcpu, "unit": "freqs/s", "cores": threads, "kind": "oracle",
               "sample": f"{iters} forward+adjoint pairs of the same |I|=2^16 workload (numpy FFT tier, "
                         f"FP64), {tcpu:.3f} s each"}

    line = {
        "metric": "mr1l-FFT freqs/s fwd+adj (|I|=2^16,d=10)",
        "value": n / (ms_event * 1e-3),
        "unit": "freqs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_event,
        "ms_per_step_wall": ms_wall,
        "ms_per_step_stage_timed": ms_event_timed,
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
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        extra = {"sfft": extra_sfft()}
        _progress("sparse FFT solve timed")
        extra["batched_512"] = extra_batched()
        _progress("batched transforms timed")
        extra["autograd_lsq"] = extra_autograd(args.gd_steps)
        _progress("gradient-descent steps timed")
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
