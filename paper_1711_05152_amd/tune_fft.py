"""Autotuner of the four-step Bluestein schedule; rewrites csrc/fft_schedule_table.h.

Every Bluestein length 2^lgN from 2^13 to 2^24 has three splits compiled (the rule's
2^lgN1 x 2^(lgN - lgN1) and its neighbours, where both factors stay within 2^4 .. 2^12).  For each
precision and length this script builds a synthetic plan whose lattices all have that length
(distinct primes M with 2M - 1 in (2^(lgN-1), 2^lgN], about 2^22 Bluestein points in total),
times forward + adjoint under every split (mr1l_fft_split), and keeps the fastest one when it
beats the rule's by more than ``--margin``.  It writes the table, prints one JSON line per length
and, with ``--report``, a Markdown summary.  Run it on the GPU, then rebuild the library
(``__graft_entry__.build()``): plans read the table when they are created.

    python -m paper_1711_05152_amd.tune_fft [--lengths 13-24] [--dtypes c64,c128] [--report FILE]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

import numpy as np

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fft_schedule_table.h")
TILE_LG, SMALL_MAX_LG = 12, 12


def rule_split(lgn: int) -> int:
    return max(lgn - TILE_LG, min(lgn // 2, TILE_LG - 4))


def candidates(lgn: int) -> list[int]:
    r = rule_split(lgn)
    return [s for s in (r - 1, r, r + 1) if 4 <= s <= TILE_LG and 4 <= lgn - s <= TILE_LG]


def _primes_in(lo: int, hi: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """``count`` distinct primes drawn from [lo, hi] (trial division on random odd candidates)."""
    out: set[int] = set()
    while len(out) < count:
        m = int(rng.integers(lo, hi + 1)) | 1
        if m < 3 or m > hi:
            continue
        if all(m % q for q in range(3, int(m ** 0.5) + 1, 2)):
            out.add(m)
    return np.array(sorted(out), np.int64)


def workload(lgn: int, rng: np.random.Generator):
    """Lattices of Bluestein length exactly 2^lgn: M in [2^(lgn-2) + 1, 2^(lgn-1)] so 2M - 1 lies
    in (2^(lgn-1), 2^lgn); about 2^22 Bluestein points over at most 64 lattices."""
    L = max(1, min(64, 1 << max(0, 22 - lgn)))
    lo, hi = (1 << (lgn - 2)) + 1, 1 << (lgn - 1)
    M = _primes_in(lo + (hi - lo) // 2, hi, L, rng)
    n = int(min(M.min() // 2, 1 << 16))
    d = 4
    freqs = np.unique(rng.integers(-1000, 1001, size=(2 * n, d)), axis=0)[:n].astype(np.int32)
    z = np.stack([rng.integers(0, m, size=d) for m in M]).astype(np.int64)
    return freqs, M, z


def time_split(freqs, M, z, dtype: str, reps: int) -> float:
    import torch
    from .mr1l import Plan
    plan = Plan(freqs, M, z, dtype=dtype, weights="paper", n_rhs=1, device=0)
    tdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]
    g = torch.Generator(device="cuda:0").manual_seed(1)
    y = torch.randn((1, plan.sum_M), dtype=tdt, device="cuda:0", generator=g)
    c = torch.randn((1, plan.n), dtype=tdt, device="cuda:0", generator=g)
    co, yo = plan.empty_coeffs(), plan.empty_samples()
    for _ in range(3):
        plan.forward(y, out=co)
        plan.adjoint(c, out=yo)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.forward(y, out=co)
            plan.adjoint(c, out=yo)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    del plan
    return best


def set_split(dtype: str, lgn: int, s: int) -> int:
    from . import _lib
    cur = C.c_int(0)
    _lib.check(_lib.lib().mr1l_fft_split({"c64": _lib.C64, "c128": _lib.C128}[dtype], lgn, s, C.byref(cur)),
               "mr1l_fft_split")
    return cur.value


def write_table(chosen: dict, path: str = TABLE) -> None:
    rows = []
    for dt in ("c64", "c128"):
        vals = [chosen.get((dt, lg), -1) for lg in range(25)]
        rows.append("    {" + ", ".join(str(v) for v in vals) + "},")
    src = ("// Four-step splits of the Bluestein lengths, as measured on MI355X by\n"
           "// paper_1711_05152_amd/tune_fft.py (which rewrites this file): kTunedSplit[dtype][lgN] is lgN1 of\n"
           "// 2^lgN = 2^lgN1 * 2^(lgN - lgN1) for dtype 0 = complex64, 1 = complex128; -1 keeps the rule.\n"
           "#pragma once\n#include <stdint.h>\nstatic const int8_t kTunedSplit[2][25] = {\n" + "\n".join(rows) + "\n};\n")
    with open(path, "w") as fh:
        fh.write(src)


def parse_lengths(spec: str) -> list[int]:
    out = []
    for part in spec.split(","):
        a, _, b = part.partition("-")
        out += list(range(int(a), int(b or a) + 1))
    return [lg for lg in out if SMALL_MAX_LG < lg <= 24]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--lengths", default="13-24")
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--margin", type=float, default=0.02, help="relative gain needed to leave the rule")
    ap.add_argument("--report", default=None, help="also write a Markdown summary to this file")
    ap.add_argument("--no-write", action="store_true", help="measure only; leave the table alone")
    ap.add_argument("--table", default=TABLE, help="where to write the table (default: the library's source)")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    chosen, results = {}, []
    rng = np.random.default_rng(1711051524)
    for dtype in args.dtypes.split(","):
        for lgn in parse_lengths(args.lengths):
            freqs, M, z = workload(lgn, rng)
            ms = {}
            for s in candidates(lgn):
                set_split(dtype, lgn, s)
                ms[s] = time_split(freqs, M, z, dtype, args.reps)
            set_split(dtype, lgn, -1)
            r = rule_split(lgn)
            best = min(ms, key=ms.get)
            pick = best if ms[best] < (1.0 - args.margin) * ms[r] else r
            if pick != r:
                chosen[(dtype, lgn)] = pick
            row = {"dtype": dtype, "lgN": lgn, "L": len(M), "M_range": [int(M.min()), int(M.max())],
                   "ms_fwd_adj": {str(k): round(v, 5) for k, v in ms.items()}, "rule": r, "chosen": pick,
                   "gain_vs_rule": round(1.0 - ms[pick] / ms[r], 4)}
            results.append(row)
            print(json.dumps(row), flush=True)
    if not args.no_write:
        write_table(chosen, args.table)
    if args.report:
        lines = ["# Four-step split autotuning (Bluestein FFT of the multiple rank-1 lattice transform)", "",
                 "Command (from the repository root on one MI355X):", "", "```",
                 "python -m paper_1711_05152_amd.tune_fft " + " ".join(argv if argv is not None else sys.argv[1:]),
                 "```", "",
                 "Forward + adjoint of one plan per row (lattices of exactly that Bluestein length, about 2^22 "
                 "Bluestein points in total), best of 3 x %d calls, in ms per call pair, for every compiled "
                 "split lgN1 (2^lgN = 2^lgN1 columns x 2^(lgN - lgN1) rows).  A split other than the rule's is "
                 "kept when it is at least %.0f %% faster." % (args.reps, 100 * args.margin), "",
                 "| dtype | lgN | L | ms per split | rule | chosen | gain |", "|---|---:|---:|---|---:|---:|---:|"]
        for r in results:
            cells = ", ".join(f"{k}: {v:.4f}" for k, v in r["ms_fwd_adj"].items())
            lines.append(f"| {r['dtype']} | {r['lgN']} | {r['L']} | {cells} | {r['rule']} | {r['chosen']} | "
                         f"{100 * r['gain_vs_rule']:.1f} % |")
        with open(args.report, "w") as fh:
            fh.write("\n".join(lines) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
