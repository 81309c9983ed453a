"""Summaries of rocprofv3 results (SQLite ``*_results.db``) for ``profiles/``.

``python -m paper_2511_06788_amd.profiling trace <db> --cmd "<rocprofv3 command>"``
prints a per-kernel table (calls, total and average duration) as Markdown.

``python -m paper_2511_06788_amd.profiling pmc --fetch <db> --write <db>
--copy-fetch <db> --copy-write <db> --kernel <regex> --n N_POINTS --N N_COLS
--source <file> --cmd ...`` prints the byte counters of the kernels matching
``regex`` per dispatch, scaled by the factor that makes a plain device copy of
known size read its own size, and writes the JSON record ``bench.py`` uses for
its ``traffic`` field.

``python -m paper_2511_06788_amd.profiling mfma --pmc-db <db> --trace-db <db>
--kernel LABEL=REGEX --flop LABEL=FLOP ...`` prints, per kernel, the matrix-core
utilisation (``MfmaUtil``: MFMA-busy cycles over active cycles of every SIMD),
the MFMA flops the counters saw per dispatch (``MfmaFlopsF64``/``BF16``) next to
the algorithmic count, and the rate from the trace's average duration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import sqlite3
import sys


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    # rocprofv3's top_kernels view reports durations in microseconds
    return [{"name": r[0], "calls": int(r[1]), "total_ms": r[2] / 1e3, "avg_us": r[3], "pct": r[4]}
            for r in rows]


def counter_per_dispatch(db: str, counter: str, pattern: str, min_frac: float = 0.0):
    """Mean of `counter` over the dispatches of kernels matching `pattern`
    whose value is at least min_frac of the largest (a CG sweep launched after
    every column converged returns at once and moves next to nothing; such
    launches are left out of a per-sweep figure).  Returns (mean, used, all)."""
    con = sqlite3.connect(db)
    rx = re.compile(pattern)
    vals = [r[1] for r in con.execute("select kernel_name, value from counters_collection where counter_name=?",
                                      (counter,)) if rx.search(r[0])]
    if not vals:
        return None, 0, 0
    top = max(vals)
    used = [v for v in vals if v >= min_frac * top]
    return sum(used) / len(used), len(used), len(vals)


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    m = re.match(r"(void )?([\w:]+)(<[^()]*>)?", name)
    return (m.group(2) + (m.group(3) or "")) if m else name[:60]


def cmd_trace(args):
    st = kernel_stats(args.db)
    out = [f"# Kernel trace: {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
           "| kernel | calls | total (ms) | average (us) | share |", "|---|---:|---:|---:|---:|"]
    for r in st[: args.top]:
        out.append(f"| `{short_name(r['name'])}` | {r['calls']} | {r['total_ms']:.2f} | {r['avg_us']:.1f} | {r['pct']:.1f}% |")
    if args.note:
        out += ["", args.note]
    print("\n".join(out))


def cmd_pmc(args):
    cf, _, _ = counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", args.copy_kernel)
    cw, _, _ = counter_per_dispatch(args.copy_write, "WRITE_SIZE", args.copy_kernel)
    copy_kib = args.copy_bytes / 1024.0
    fscale = copy_kib / cf
    wscale = copy_kib / cw
    # several --kernel patterns: kernels that alternate one launch per
    # iteration (the two forms of a sweep); the figures are their mean
    fs_, ws_ = [], []
    nf = af = nw = aw = 0
    for pat in args.kernel:
        f1, n1, a1 = counter_per_dispatch(args.fetch, "FETCH_SIZE", pat, args.min_frac)
        w1, n2, a2 = counter_per_dispatch(args.write, "WRITE_SIZE", pat, args.min_frac)
        fs_.append(f1)
        ws_.append(w1)
        nf, af, nw, aw = nf + n1, af + a1, nw + n2, aw + a2
    f = sum(fs_) / len(fs_)
    w = sum(ws_) / len(ws_)
    blk = args.n * args.N * args.esz
    algo_read = args.reads * blk + args.esz * args.n
    algo_write = args.writes * blk
    per_kernel = [{"kernel_regex": k, "fetch_kib": a * fscale, "write_kib": b * wscale}
                  for k, a, b in zip(args.kernel, fs_, ws_)]
    rec = {
        "kernel_regex": args.kernel, "per_kernel": per_kernel, "n": args.n, "N": args.N,
        "fetch_kib_per_dispatch": f * fscale, "write_kib_per_dispatch": w * wscale, "copy_scale": 1.0,
        "raw_fetch_kib": f, "raw_write_kib": w, "fetch_scale": fscale, "write_scale": wscale,
        "dispatches": [nf, nw], "dispatches_all": [af, aw], "min_frac": args.min_frac,
        "algorithmic_read_bytes": algo_read, "algorithmic_write_bytes": algo_write,
        "source_sha256": hashlib.sha256(open(args.source, "rb").read()).hexdigest(), "command": args.cmd,
    }
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rec, fh, indent=1)
    print("\n".join([
        f"# HBM traffic: {args.title}", "", "Commands:", "", "```", args.cmd, "```", "",
        f"Copy calibration: a plain device copy of {args.copy_bytes} bytes reads as {cf:.1f} KiB FETCH_SIZE and "
        f"{cw:.1f} KiB WRITE_SIZE per dispatch: fetch scale {fscale:.4f}, write scale {wscale:.4f}.", "",
        "| quantity | per dispatch |", "|---|---:|",
        f"| FETCH_SIZE raw (KiB) | {f:.1f} |", f"| WRITE_SIZE raw (KiB) | {w:.1f} |",
        f"| read bytes, scaled | {f * fscale * 1024:.4g} |", f"| written bytes, scaled | {w * wscale * 1024:.4g} |",
        f"| algorithmic read bytes | {algo_read:.4g} |", f"| algorithmic written bytes | {algo_write:.4g} |",
        f"| read / algorithmic | {f * fscale * 1024 / algo_read:.2f} |",
        f"| written / algorithmic | {w * wscale * 1024 / max(algo_write, 1):.2f} |",
        f"| dispatches averaged (of all) | {nf} of {af} / {nw} of {aw} |",
        "",
    ] + ([f"Per kernel (the table gives their mean): " + "; ".join(
        f"`{k['kernel_regex']}` reads {k['fetch_kib'] * 1024:.4g} B, writes {k['write_kib'] * 1024:.4g} B"
        for k in per_kernel), ""] if len(per_kernel) > 1 else []) + [
        f"Averaged: the dispatches whose counter is at least {args.min_frac:g} of the largest (launches past the last "
        "converged column of a CG chunk return at once and move almost nothing).",
    ] + ([""] + [args.note] if args.note else [])))


# Dense matrix-core peaks of the MI355X (TFLOP/s)
MFMA_PEAK = {"F64": 78.6, "BF16": 2500.0}


def trace_avg_us(db: str, pattern: str):
    """Call-weighted average duration (us) of the kernels matching `pattern`."""
    rx = re.compile(pattern)
    st = [r for r in kernel_stats(db) if rx.search(r["name"])]
    calls = sum(r["calls"] for r in st)
    return (sum(r["total_ms"] for r in st) * 1e3 / calls, calls) if calls else (None, 0)


def cmd_mfma(args):
    flop = dict(kv.split("=", 1) for kv in args.flop)
    out = [f"# Matrix-core use: {args.title}", "", "Commands:", "", "```", args.cmd, "```", "",
           "| kernel | dispatches | MfmaUtil (%) | MFMA flop per dispatch (counters) | algorithmic flop | "
           "average (us, trace) | algorithmic TFLOP/s | of peak |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for kv in args.kernel:
        label, pat = kv.split("=", 1)
        util, nu, _ = counter_per_dispatch(args.pmc_db, "MfmaUtil", pat)
        kind = args.kind
        fl, _, _ = counter_per_dispatch(args.pmc_db, "MfmaFlops" + kind, pat)
        avg, _ = trace_avg_us(args.trace_db, pat)
        algo = float(flop[label]) if label in flop else None
        rate = algo / (avg * 1e-6) / 1e12 if (algo and avg) else None
        out.append(f"| `{label}` | {nu} | {util:.1f} | {fl:.4g} | "
                   f"{algo:.4g} | {avg:.1f} | {rate:.1f} | {rate / MFMA_PEAK[kind]:.2f} |"
                   if None not in (util, fl, algo, avg) else f"| `{label}` | {nu} | n/a | n/a | n/a | n/a | n/a | n/a |")
    out += ["", f"Peak: {MFMA_PEAK[args.kind]} TFLOP/s dense {args.kind} (MI355X). MfmaUtil is rocprofv3's derived "
            "metric, SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs)."]
    if args.note:
        out += ["", args.note]
    print("\n".join(out))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--top", type=int, default=20)
    t.add_argument("--note", default="", help="text appended to the summary")
    p = sub.add_parser("pmc")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        p.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    p.add_argument("--kernel", required=True, action="append",
                   help="kernel name pattern; repeat for kernels that alternate per iteration (mean taken)")
    p.add_argument("--copy-kernel", default="copyBuffer")
    p.add_argument("--copy-bytes", type=int, default=1 << 30)
    p.add_argument("--n", type=int, required=True)
    p.add_argument("--N", type=int, required=True)
    p.add_argument("--esz", type=int, default=8, help="bytes per element of the blocks (8 FP64, 4 FP32)")
    p.add_argument("--reads", type=float, default=3)
    p.add_argument("--writes", type=float, default=2)
    p.add_argument("--source", required=True)
    p.add_argument("--cmd", required=True)
    p.add_argument("--title", default="")
    p.add_argument("--json", default=None)
    p.add_argument("--min-frac", type=float, default=0.1)
    p.add_argument("--note", default="")
    m = sub.add_parser("mfma")
    m.add_argument("--pmc-db", required=True)
    m.add_argument("--trace-db", required=True)
    m.add_argument("--kernel", required=True, action="append", help="LABEL=REGEX")
    m.add_argument("--flop", default=[], action="append", help="LABEL=algorithmic flop per dispatch")
    m.add_argument("--kind", default="F64", choices=sorted(MFMA_PEAK))
    m.add_argument("--cmd", required=True)
    m.add_argument("--title", default="")
    m.add_argument("--note", default="")
    args = ap.parse_args(argv)
    {"trace": cmd_trace, "pmc": cmd_pmc, "mfma": cmd_mfma}[args.what](args)


if __name__ == "__main__":
    sys.exit(main())
