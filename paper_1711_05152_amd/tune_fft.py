"""Autotuner of the four-step Bluestein schedule; rewrites csrc/fft_schedule_table.h.

Every Bluestein length 2^lgN from 2^13 to 2^24 has three splits compiled (the rule's
2^lgN1 x 2^(lgN - lgN1) and its neighbours, where both factors stay within 2^4 .. 2^12), and
stage 2 (row DFTs, filter, inverse row DFTs) has up to six variants per split: its radix schedule
(bits spread evenly over the stages, e.g. 8 8 16 for 1024-point rows, or radix 16 in every stage
but one, 4 16 16), its values per thread (16, or 8 with radices up to 8, e.g. 4 4 8 8, and twice
the threads) and its tile size (2048- or 4096-element tiles for rows of up to 2^10 points); a
variant exists only where it changes the kernel.  For each precision and length this script
builds a synthetic plan whose lattices all have that length (distinct primes M with 2M - 1 in
(2^(lgN-1), 2^lgN], about 2^22 Bluestein points in total), times forward + adjoint under every
(split, variant) (mr1l_fft_split, mr1l_fft_p2_variant), and keeps the fastest when it beats the
rule's split with variant 0 by more than ``--margin``.  Where the class 2^lgN also has a factor-3
length 3 * 2^(lgN - 2) (lgN - 2 in 12 .. 22), a second synthetic plan with lattices that all fit it
(M in [2^(lgN-2) + 1, 3 * 2^(lgN-3)]) is timed with the chosen power-of-two schedule and with the
factor-3 length (mr1l_fft_smooth), which the class then takes when it is faster by the margin.  It
writes the tables, prints one JSON line per length and, with ``--report``, a Markdown summary.  Run it on the GPU, then rebuild the library
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


P2_TILE_LG = 11


def _lgv(order: int) -> int:
    return 3 if order >= 4 else 4


def _n_stages(lg: int, order: int = 1) -> int:
    return (lg + _lgv(order) - 1) // _lgv(order)


def _stage_lr(lg: int, i: int, order: int) -> int:
    """Radix (log2) of stage i of a 2^lg-point tile DFT under radix order ``order`` (the library's
    rule: 1 = bits spread evenly, ascending, 16 values per thread; 3 = radix 16 but the first
    stage; 5 = bits spread evenly, ascending, 8 values per thread)."""
    ns = _n_stages(lg, order)
    if order in (2, 3):
        return lg - 4 * (ns - 1) if i == (0 if order == 3 else ns - 1) else 4
    return lg // ns + 1 if i >= ns - lg % ns else lg // ns


def p2_variants(lgn: int, split: int) -> list[int]:
    """Stage-2 variants compiled for this length and split (bit 0 radix schedule, bit 1 big tile,
    bit 2 eight values per thread)."""
    lg2 = lgn - split
    sched = any(_stage_lr(lg2, i, 1) != _stage_lr(lg2, i, 3) for i in range(_n_stages(lg2)))
    big = lg2 + 1 <= P2_TILE_LG
    return [v for v in range(7)
            if not ((v & 4) and (v & 1)) and (not (v & 1) or sched) and (not (v & 2) or big)]


def describe(lgn: int, split: int, v: int) -> str:
    lg2 = lgn - split
    order = 5 if v & 4 else (3 if v & 1 else 1)
    radices = "x".join(str(1 << _stage_lr(lg2, i, order)) for i in range(_n_stages(lg2, order)))
    tile = 4096 if (v & 2) or lg2 + 1 > P2_TILE_LG else 2048
    return f"{split}/{radices}/{tile}" + ("/8v" if v & 4 else "")


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
    in (2^(lgn-1), 2^lgn), spread over the whole class as primes drawn from an octave are; about
    2^22 Bluestein points over at most 64 lattices.  (Timed with powers of two only.)"""
    L = max(1, min(64, 1 << max(0, 22 - lgn)))
    lo, hi = (1 << (lgn - 2)) + 1, 1 << (lgn - 1)
    M = _primes_in(lo, hi, L, rng)
    n = int(min(M.min() // 2, 1 << 16))
    d = 4
    freqs = np.unique(rng.integers(-1000, 1001, size=(2 * n, d)), axis=0)[:n].astype(np.int32)
    z = np.stack([rng.integers(0, m, size=d) for m in M]).astype(np.int64)
    return freqs, M, z


def workload3(lgn: int, rng: np.random.Generator):
    """Lattices that all fit the factor-3 length 3 * 2^(lgn-2) of the class 2^lgn:
    M in [2^(lgn-2) + 1, 3 * 2^(lgn-3)], about 2^22 power-of-two points as in ``workload``."""
    L = max(1, min(64, 1 << max(0, 22 - lgn)))
    lo, hi = (1 << (lgn - 2)) + 1, 3 << (lgn - 3)
    M = _primes_in(lo, hi, L, rng)
    n = int(min(M.min() // 2, 1 << 16))
    d = 4
    freqs = np.unique(rng.integers(-1000, 1001, size=(2 * n, d)), axis=0)[:n].astype(np.int32)
    z = np.stack([rng.integers(0, m, size=d) for m in M]).astype(np.int64)
    return freqs, M, z


def set_smooth(mode: int) -> int:
    from .mr1l import fft_smooth
    return fft_smooth(mode)


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


def set_p2_variant(dtype: str, lgn: int, v: int) -> int:
    from . import _lib
    cur = C.c_int(0)
    _lib.check(_lib.lib().mr1l_fft_p2_variant({"c64": _lib.C64, "c128": _lib.C128}[dtype], lgn, v, C.byref(cur)),
               "mr1l_fft_p2_variant")
    return cur.value


def write_table(chosen: dict, chosen_p2: dict, chosen3: dict = None, path: str = TABLE) -> None:
    def rows(tab):
        out = []
        for dt in ("c64", "c128"):
            vals = [tab.get((dt, lg), -1) for lg in range(25)]
            out.append("    {" + ", ".join(str(v) for v in vals) + "},")
        return "\n".join(out)
    src = ("// Four-step splits of the Bluestein lengths, as measured on MI355X by\n"
           "// paper_1711_05152_amd/tune_fft.py (which rewrites this file): kTunedSplit[dtype][lgN] is lgN1 of\n"
           "// 2^lgN = 2^lgN1 * 2^(lgN - lgN1) for dtype 0 = complex64, 1 = complex128; -1 keeps the rule.\n"
           "#pragma once\n#include <stdint.h>\nstatic const int8_t kTunedSplit[2][25] = {\n" + rows(chosen) + "\n};\n"
           "// Stage-2 variants (bit 0: radix schedule of orders 3 / 2; bit 1: 4096-element row tiles; bit 2:\n"
           "// 8 values per thread) chosen by the same tuner: kTunedP2[dtype][lgN] for the split of kTunedSplit;\n"
           "// -1 keeps variant 0.\n"
           "static const int8_t kTunedP2[2][25] = {\n" + rows(chosen_p2) + "\n};\n"
           "// Bluestein length classes 2^lg whose lattices take 3 * 2^(lg - 2) when all of them fit, chosen by\n"
           "// the same tuner (1: the factor-3 length measured faster; 0 or -1: powers of two).\n"
           "static const int8_t kTunedSmooth[2][25] = {\n" + rows(chosen3 or {}) + "\n};\n")
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
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--margin", type=float, default=0.015, help="relative gain needed to leave the rule")
    ap.add_argument("--report", default=None, help="also write a Markdown summary to this file")
    ap.add_argument("--no-write", action="store_true", help="measure only; leave the table alone")
    ap.add_argument("--table", default=TABLE, help="where to write the table (default: the library's source)")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    chosen, chosen_p2, chosen3, results = {}, {}, {}, []
    rng = np.random.default_rng(1711051524)
    prev_smooth = set_smooth(-1)
    for dtype in args.dtypes.split(","):
        for lgn in parse_lengths(args.lengths):
            freqs, M, z = workload(lgn, rng)
            set_smooth(0)
            ms = {}
            for s in candidates(lgn):
                set_split(dtype, lgn, s)
                for v in p2_variants(lgn, s):
                    set_p2_variant(dtype, lgn, v)
                    ms[(s, v)] = time_split(freqs, M, z, dtype, args.reps)
                set_p2_variant(dtype, lgn, -2)
            set_split(dtype, lgn, -1)
            r = (rule_split(lgn), 0)
            best = min(ms, key=ms.get)
            pick = best if ms[best] < (1.0 - args.margin) * ms[r] else r
            if pick[0] != r[0]:
                chosen[(dtype, lgn)] = pick[0]
            if pick[1] != 0:
                chosen_p2[(dtype, lgn)] = pick[1]
            row = {"dtype": dtype, "lgN": lgn, "L": len(M), "M_range": [int(M.min()), int(M.max())],
                   "ms_fwd_adj": {describe(lgn, *k): round(v, 5) for k, v in ms.items()},
                   "rule": describe(lgn, *r), "chosen": describe(lgn, *pick),
                   "gain_vs_rule": round(1.0 - ms[pick] / ms[r], 4)}
            if 12 <= lgn - 2 <= 22:
                # factor-3 length of the class against the power-of-two schedule just chosen
                f3, M3, z3 = workload3(lgn, rng)
                set_split(dtype, lgn, pick[0])
                set_p2_variant(dtype, lgn, pick[1])
                set_smooth(0)
                t_pow2 = time_split(f3, M3, z3, dtype, args.reps)
                set_smooth(2)
                t_3 = time_split(f3, M3, z3, dtype, args.reps)
                set_smooth(0)
                set_p2_variant(dtype, lgn, -2)
                set_split(dtype, lgn, -1)
                use3 = t_3 < (1.0 - args.margin) * t_pow2
                if use3:
                    chosen3[(dtype, lgn)] = 1
                row["factor3"] = {"M_range": [int(M3.min()), int(M3.max())], "ms_pow2": round(t_pow2, 5),
                                  "ms_3x": round(t_3, 5), "chosen": "3x2^%d" % (lgn - 2) if use3 else "2^%d" % lgn}
            results.append(row)
            print(json.dumps(row), flush=True)
    set_smooth(prev_smooth)
    if not args.no_write:
        write_table(chosen, chosen_p2, chosen3, args.table)
    if args.report:
        lines = ["# Four-step split autotuning (Bluestein FFT of the multiple rank-1 lattice transform)", "",
                 "Command (from the repository root on one MI355X):", "", "```",
                 "python -m paper_1711_05152_amd.tune_fft " + " ".join(argv if argv is not None else sys.argv[1:]),
                 "```", "",
                 "Forward + adjoint of one plan per row (lattices of exactly that Bluestein length, about 2^22 "
                 "Bluestein points in total), best of 3 x %d calls, in ms per call pair, for every compiled "
                 "schedule split/radices/tile: the split lgN1 (2^lgN = 2^lgN1 columns x 2^(lgN - lgN1) rows), "
                 "the radices of stage 2's forward row DFT (the inverse runs them in reverse order) and "
                 "stage 2's tile in elements; /8v marks 8 values per thread instead of 16.  A schedule other than the rule's split with evenly spread "
                 "radices and the default tile is kept when it is at least %.0f %% faster."
                 % (args.reps, 100 * args.margin), "",
                 "| dtype | lgN | L | ms per schedule | rule | chosen | gain |", "|---|---:|---:|---|---|---|---:|"]
        for r in results:
            cells = ", ".join(f"{k}: {v:.4f}" for k, v in r["ms_fwd_adj"].items())
            lines.append(f"| {r['dtype']} | {r['lgN']} | {r['L']} | {cells} | {r['rule']} | {r['chosen']} | "
                         f"{100 * r['gain_vs_rule']:.1f} % |")
        lines += ["", "Factor-3 lengths: a plan whose lattices all fit 3 * 2^(lgN-2) (sizes below), forward + "
                  "adjoint in ms with the chosen power-of-two schedule and with the factor-3 length; the class "
                  "takes the factor-3 length when it is at least %.0f %% faster." % (100 * args.margin), "",
                  "| dtype | lgN | M range | 2^lgN | 3 * 2^(lgN-2) | chosen |", "|---|---:|---|---:|---:|---|"]
        for r in results:
            f = r.get("factor3")
            if f:
                lines.append(f"| {r['dtype']} | {r['lgN']} | {f['M_range'][0]} .. {f['M_range'][1]} | "
                             f"{f['ms_pow2']:.4f} | {f['ms_3x']:.4f} | {f['chosen']} |")
        with open(args.report, "w") as fh:
            fh.write("\n".join(lines) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
