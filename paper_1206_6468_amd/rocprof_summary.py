"""Summaries of rocprofv3 output for the committed profile records.

Reads the SQLite databases rocprofv3 writes (``*_results.db``) and produces
short text records:

  kernels   per-kernel dispatch statistics of a ``--kernel-trace --stats`` run
            (calls, total and average duration, share of GPU time);
  traffic   HBM bytes per dispatch from two ``--pmc`` runs (FETCH_SIZE, then
            WRITE_SIZE) of the benchmark, each scaled by what the same counter
            reads for a plain device copy of known size (two more runs of
            ``bench.py --copy-calibration``).

The traffic record carries a hash of the kernel sources so that a reader can
tell whether it still describes the kernels in the tree.

    python -m paper_1206_6468_amd.rocprof_summary kernels DB --command CMD --out FILE.md
    python -m paper_1206_6468_amd.rocprof_summary traffic --fetch DB --write DB \
        --copy-fetch DB --copy-write DB --workload NAME --commands CMD... --out FILE.json
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sqlite3
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


KERNEL_SOURCES = ("nfhmm_kernels.hip", "special.h", "wave.h", "jobdesc.h", "launch.h")


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    """SHA-256 prefix over device-side sources (by default the iteration kernels
    and the headers they include; the host runtime is not part of it)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    """'void nfhmm::k_counts<false>(nfhmm::WorkList)' -> 'k_counts';
    the BF16 instantiation (template argument true) gets a '_bf16' suffix;
    other template arguments are kept ('k_chain_fb<40>', 'k_stft<1024>');
    kernels from outside the library keep their bare name and their namespace's
    first part ('distribution_elementwise_grid_stride_kernel (at)')."""
    m = re.search(r"nfhmm::(?:\(anonymous namespace\)::)?(\w+)(<([^>]*)>)?\(", full)
    if not m:
        q = re.match(r"(?:void )?([\w:]+)", full.replace("(anonymous namespace)::", ""))
        if not q:
            return full
        parts = q.group(1).split("::")
        return f"{parts[-1]} ({parts[0]})" if len(parts) > 1 else parts[-1]
    base, targ = m.group(1), m.group(3)
    if targ is None:
        return base
    if targ in ("true", "false"):
        return base + ("_bf16" if targ == "true" else "")
    return f"{base}<{targ}>"


def _db(path: str) -> str:
    if os.path.isdir(path):
        found = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
        if not found:
            raise FileNotFoundError(f"no *_results.db under {path}")
        return found[0]
    return path


def kernel_stats(db: str):
    """[(name, calls, total ns, average ns, share)] by total time, and the GPU's name."""
    con = sqlite3.connect(_db(db))
    rows = con.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows) or 1
    rows = [(n, c, t, a, 100.0 * t / tot) for n, c, t, a in rows]
    gpu = con.execute("select name from rocpd_info_agent where type = 'GPU' limit 1").fetchone()
    return rows, (gpu[0] if gpu else "?")


def counter_per_kernel(db: str, counter: str):
    con = sqlite3.connect(_db(db))
    acc = defaultdict(list)
    for name, val in con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                                 (counter,)):
        acc[name].append(float(val))
    return acc


def cmd_kernels(a):
    rows, gpu = kernel_stats(a.db)
    lines = [f"# Kernel dispatch statistics: {a.title}", "",
             f"Command (run from /tmp with TMPDIR=/tmp; `$R` is the repository root):", "",
             f"    {a.command}", "",
             f"GPU: {gpu}; kernel sources {kernel_source_hash(tuple(a.sources))}"
             + ("" if tuple(a.sources) == KERNEL_SOURCES else f" ({', '.join(a.sources)})") + ".", "",
             "| kernel | calls | total ms | average us | share of GPU time |",
             "|---|---:|---:|---:|---:|"]
    for name, calls, total, avg, pct in rows:
        lines.append(f"| `{short_name(name)}` | {calls} | {total / 1e6:.3f} | {avg / 1e3:.1f} | {pct:.1f}% |")
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}")


def cmd_traffic(a):
    fetch = counter_per_kernel(a.fetch, "FETCH_SIZE")
    write = counter_per_kernel(a.write, "WRITE_SIZE")
    cf = counter_per_kernel(a.copy_fetch, "FETCH_SIZE")
    cw = counter_per_kernel(a.copy_write, "WRITE_SIZE")
    copy_bytes = a.copy_bytes

    def copy_factor(d):
        # the copy dispatches are the ones that move about copy_bytes
        vals = [v for vs in d.values() for v in vs if v * 1024 > 0.25 * copy_bytes]
        if not vals:
            raise SystemExit("no copy-sized dispatch found in the calibration run")
        return copy_bytes / (1024 * sum(vals) / len(vals)), len(vals)

    f_fac, nf = copy_factor(cf)
    w_fac, nw = copy_factor(cw)
    kernels = {}
    for full in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(full, []), write.get(full, [])
        if not fv or not wv:
            continue
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        kernels[short_name(full)] = {
            "workload": a.workload, "dispatches": len(fv),
            "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
            "fetch_bytes_per_launch": fk * 1024 * f_fac, "write_bytes_per_launch": wk * 1024 * w_fac,
            "bytes_per_launch": fk * 1024 * f_fac + wk * 1024 * w_fac,
        }
    out = {"kernel_source_hash": kernel_source_hash(tuple(a.sources)), "kernel_sources": a.sources,
           "workload": a.workload,
           "calibration": {"copy_bytes": copy_bytes, "fetch_scale": f_fac, "write_scale": w_fac,
                           "copy_dispatches": [nf, nw]},
           "commands": a.commands, "kernels": kernels}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {a.out}")
    if a.md:
        lines = [f"# HBM traffic per launch: {a.workload}", "",
                 "Commands (run from /tmp with TMPDIR=/tmp; `$R` is the repository root):", ""]
        lines += [f"    {c}" for c in a.commands]
        lines += ["", f"Kernel sources {out['kernel_source_hash']} ({', '.join(a.sources)}).  Calibration: a {copy_bytes / 2**20:.0f} MiB "
                  f"device copy reads FETCH_SIZE x {f_fac:.4f} and WRITE_SIZE x {w_fac:.4f} of its true bytes; "
                  "the figures below are scaled by those factors.", "",
                  "| kernel | dispatches | fetched MB / launch | written MB / launch | total MB / launch |",
                  "|---|---:|---:|---:|---:|"]
        for name, e in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"] * kv[1]["dispatches"]):
            if e["bytes_per_launch"] * e["dispatches"] < 1e6:
                continue
            lines.append(f"| `{name}` | {e['dispatches']} | {e['fetch_bytes_per_launch'] / 1e6:.1f} | "
                         f"{e['write_bytes_per_launch'] / 1e6:.1f} | {e['bytes_per_launch'] / 1e6:.1f} |")
        with open(a.md, "w") as f:
            f.write("\n".join(lines) + "\n")
        print(f"wrote {a.md}")


def cmd_counters(a):
    """Per-kernel averages of every counter of one --pmc run, with MFMA busy
    fraction (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE of one XCD times the
    SIMDs) and LDS bank-conflict ratio where their counters are present."""
    con = sqlite3.connect(_db(a.db))
    acc = defaultdict(lambda: defaultdict(list))
    for name, cn, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
        acc[name][cn].append(float(v))
    lines = [f"# Hardware counters per dispatch: {a.title}", "",
             "Command (run from /tmp with TMPDIR=/tmp; `$R` is the repository root):", "", f"    {a.command}", "",
             f"Kernel sources {kernel_source_hash(tuple(a.sources))}"
             + ("" if tuple(a.sources) == KERNEL_SOURCES else f" ({', '.join(a.sources)})")
             + f".  GRBM_GUI_ACTIVE is summed over the {a.xcds} XCDs; MFMA busy = "
             f"SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {a.xcds} x {a.simds} SIMDs).", ""]
    names = sorted({c for d in acc.values() for c in d})
    lines += ["| kernel | dispatches | " + " | ".join(names) + " | MFMA busy | LDS conflict / access |",
              "|---|---:|" + "---:|" * len(names) + "---:|---:|"]
    rows = []
    for k, d in acc.items():
        avg = {c: sum(v) / len(v) for c, v in d.items()}
        util = ""
        if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and avg.get("GRBM_GUI_ACTIVE"):
            util = f"{avg['SQ_VALU_MFMA_BUSY_CYCLES'] / (avg['GRBM_GUI_ACTIVE'] / a.xcds * a.simds):.3f}"
        lds = ""
        if "SQ_LDS_BANK_CONFLICT" in avg and avg.get("SQ_LDS_IDX_ACTIVE"):
            lds = f"{avg['SQ_LDS_BANK_CONFLICT'] / max(1.0, avg['SQ_LDS_IDX_ACTIVE'] - avg['SQ_LDS_BANK_CONFLICT']):.3f}"
        ndisp = len(next(iter(d.values())))
        rows.append((avg.get("GRBM_GUI_ACTIVE", 0.0) * ndisp,
                     f"| `{short_name(k)}` | {ndisp} | "
                     + " | ".join(f"{avg.get(c, float('nan')):.4g}" for c in names) + f" | {util} | {lds} |"))
    lines += [r for _, r in sorted(rows, key=lambda x: -x[0])]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--command", required=True)
    k.add_argument("--title", default="")
    k.add_argument("--note", default="")
    k.add_argument("--sources", nargs="+", default=list(KERNEL_SOURCES),
                   help="files under csrc/ whose hash the record carries")
    k.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for n in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + n.replace("_", "-"), dest=n, required=True)
    t.add_argument("--copy-bytes", type=float, default=float(256 << 20))
    t.add_argument("--workload", required=True)
    t.add_argument("--commands", nargs="+", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--md", default="", help="also write a markdown table here")
    t.add_argument("--sources", nargs="+", default=list(KERNEL_SOURCES),
                   help="files under csrc/ whose hash the record carries")
    q = sub.add_parser("counters")
    q.add_argument("db")
    q.add_argument("--command", required=True)
    q.add_argument("--title", default="")
    q.add_argument("--xcds", type=int, default=8)
    q.add_argument("--simds", type=int, default=1024)
    q.add_argument("--sources", nargs="+", default=list(KERNEL_SOURCES),
                   help="files under csrc/ whose hash the record carries")
    q.add_argument("--out", required=True)
    a = ap.parse_args()
    {"kernels": cmd_kernels, "traffic": cmd_traffic, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
