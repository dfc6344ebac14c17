"""Summaries of rocprofv3 output for the library's kernels (host-side text processing).

Commands (each reads the directory rocprofv3 wrote with ``--output-format csv -d <dir>``):

  python -m paper_2401_06841_amd.profiling trace <dir>
      kernel table (calls, average / min / max microseconds, share) from the kernel trace
  python -m paper_2401_06841_amd.profiling counters <dir> [<dir> ...]
      per-kernel averages per dispatch of every counter collected with --pmc
  python -m paper_2401_06841_amd.profiling traffic --kernel NAME --workload W --precision P
          --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR [--out FILE]
      HBM bytes per launch of one kernel: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
      scaled by what the same counter reads for a plain device copy of known size
  python -m paper_2401_06841_amd.profiling flops --kernel NAME --workload W --precision P
          --pmc DIR [--out FILE]
      executed floating-point operations per launch: 64 lanes x (ADD + MUL + TRANS + 2 FMA)
      VALU instructions of the kernel's precision (SQ_INSTS_VALU_*_F64 or _F32)

The JSON records carry the hash of the step kernels' sources; the benchmark uses a record
only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources that define and launch the step kernels
STEP_SOURCES = ("dg_api.hip", "dg_basis.hpp", "dg_ctx.hpp", "dg_kernels.hpp")
# bytes a plain device copy of the calibration moves per dispatch (bench.py --copy-calibration)
COPY_BYTES = 4 * (1 << 27)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _files(d: str, suffix: str):
    out = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not out:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return out


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def kernel_stats(d: str):
    """Rows of the kernel-statistics files: name, calls, total / average / min / max ns."""
    rows = []
    for f in _files(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append({"name": _col(r, "Name", "KernelName"), "calls": int(_col(r, "Calls")),
                             "total_ns": float(_col(r, "TotalDurationNs")), "avg_ns": float(_col(r, "AverageNs")),
                             "min_ns": float(_col(r, "MinNs")), "max_ns": float(_col(r, "MaxNs"))})
    return rows


def counters(d: str):
    """{kernel: {"dispatches": n, counter: average value per dispatch}} from --pmc output
    (values of one dispatch and counter are summed first, over any per-instance rows)."""
    per = collections.defaultdict(float)
    names = {}
    for f in _files(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = _col(r, "Kernel_Name", "Kernel-Name", "KernelName")
                disp = (f, _col(r, "Dispatch_Id", "Dispatch-Id", "DispatchId"))
                c = _col(r, "Counter_Name", "Counter-Name", "CounterName")
                per[(k, disp, c)] += float(_col(r, "Counter_Value", "Counter-Value", "CounterValue"))
                names[(k, disp)] = {"vgpr": r.get("VGPR_Count") or r.get("Arch_VGPR_Count"),
                                    "agpr": r.get("Accum_VGPR_Count"), "scratch": r.get("Scratch_Size"),
                                    "lds": r.get("LDS_Block_Size")}
    out = collections.defaultdict(lambda: collections.defaultdict(float))
    disps = collections.defaultdict(set)
    for (k, disp, c), v in per.items():
        out[k][c] += v
        disps[k].add(disp)
    res = {}
    for k, cs in out.items():
        n = len(disps[k])
        res[k] = {"dispatches": n}
        for c, v in cs.items():
            res[k][c] = v / n
        res[k]["resources"] = names[(k, next(iter(disps[k])))] if disps[k] else {}
    return res


def _match(table, kernel: str):
    hits = [k for k in table if kernel in k]
    if len(hits) != 1:
        raise KeyError(f"kernel {kernel!r} matches {hits}")
    return hits[0]


def traffic(kernel, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    f, w = counters(fetch_dir), counters(write_dir)
    cf, cw = counters(copy_fetch_dir), counters(copy_write_dir)
    copy = "copyBuffer"
    ff = COPY_BYTES / (1024.0 * cf[_match(cf, copy)]["FETCH_SIZE"])
    wf = COPY_BYTES / (1024.0 * cw[_match(cw, copy)]["WRITE_SIZE"])
    kf, kw = _match(f, kernel), _match(w, kernel)
    read = f[kf]["FETCH_SIZE"] * 1024.0 * ff
    written = w[kw]["WRITE_SIZE"] * 1024.0 * wf
    return {"kernel": kf, "bytes_per_launch": read + written, "read_bytes": read, "written_bytes": written,
            "fetch_factor": ff, "write_factor": wf, "dispatches": f[kf]["dispatches"]}


def flops(kernel, pmc_dir, precision):
    c = counters(pmc_dir)
    k = _match(c, kernel)
    sfx = "F64" if precision == "fp64" else "F32"
    g = lambda n: c[k].get(f"SQ_INSTS_VALU_{n}_{sfx}", 0.0)    # noqa: E731
    inst = {n: g(n) for n in ("ADD", "MUL", "FMA", "TRANS")}
    return {"kernel": k, "flops_per_launch": 64.0 * (inst["ADD"] + inst["MUL"] + inst["TRANS"] + 2.0 * inst["FMA"]),
            "valu_instructions": inst, "dispatches": c[k]["dispatches"]}


def _print_trace(d):
    rows = sorted(kernel_stats(d), key=lambda r: -r["total_ns"])
    tot = sum(r["total_ns"] for r in rows) or 1.0
    print("| kernel | calls | avg us | min us | max us | share % |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['name']} | {r['calls']} | {r['avg_ns'] / 1e3:.1f} | {r['min_ns'] / 1e3:.1f} | "
              f"{r['max_ns'] / 1e3:.1f} | {100 * r['total_ns'] / tot:.1f} |")


def _print_counters(dirs):
    merged = collections.defaultdict(dict)
    for d in dirs:
        for k, v in counters(d).items():
            merged[k].update(v)
    cols = sorted({c for v in merged.values() for c in v if c not in ("dispatches", "resources")})
    print("| kernel | dispatches | " + " | ".join(cols) + " |")
    print("|---|---|" + "---|" * len(cols))
    for k, v in sorted(merged.items()):
        print(f"| {k} | {v['dispatches']} | " + " | ".join(f"{v.get(c, float('nan')):.4g}" for c in cols) + " |")


def main(argv=None):
    p = argparse.ArgumentParser(prog="python -m paper_2401_06841_amd.profiling")
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    for name in ("traffic", "flops"):
        q = sub.add_parser(name)
        q.add_argument("--kernel", required=True)
        q.add_argument("--workload", required=True)
        q.add_argument("--precision", required=True, choices=["fp64", "fp32"])
        q.add_argument("--out")
        if name == "traffic":
            for a in ("--fetch", "--write", "--copy-fetch", "--copy-write"):
                q.add_argument(a, required=True)
        else:
            q.add_argument("--pmc", required=True)
    a = p.parse_args(argv)
    if a.cmd == "trace":
        _print_trace(a.dir)
        return
    if a.cmd == "counters":
        _print_counters(a.dirs)
        return
    if a.cmd == "traffic":
        rec = traffic(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write)
    else:
        rec = flops(a.kernel, a.pmc, a.precision)
    rec.update({"workload": a.workload, "precision": a.precision, "source_hash": source_hash()})
    text = json.dumps(rec, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main(sys.argv[1:])
