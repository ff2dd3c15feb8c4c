"""Turn rocprofv3 outputs into the short text summaries kept under profiles/.

    python bench_profile.py stats  --dir D --out F --command C
    python bench_profile.py valu --dir D --kernel k_render --pairs-log P --out F --command C
    python bench_profile.py util --dir D --kernel k_render --out F --command C
    python bench_profile.py traffic --fetch-dir D1 --write-dir D2
           --kernel k_render --source paper_2603_00145_amd/csrc/render.hip --calib-mib 1024
           --out F --command-fetch C1 --command-write C2

`valu` takes one `--pmc` run of VALU instruction counters (SQ_INSTS_VALU_*) of bench.py with
`--pairs-log`, and records their mean per dispatch of one kernel with the mean contributing
pairs per dispatch and the kernel's assembly digest.

`util` takes one `--pmc` run of LDS and issue counters (SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT,
SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_SCA, SQ_WAIT_INST_LDS, SQ_WAIT_INST_ANY, GRBM_GUI_ACTIVE) and
records the busy fractions rocprofv3's derived metrics define (LdsUtil, VALUBusy) for one kernel.

`stats` summarises a `--kernel-trace --stats` run (per-kernel calls and durations of this
library's kernels).  `traffic` takes one `--pmc FETCH_SIZE` run and one `--pmc WRITE_SIZE`
run of the same program (which ran a plain streaming kernel, torch.neg over calib-mib MiB,
before its timed steps), scales the kernel's per-dispatch counters by what the counters read
for that streaming kernel (which reads and writes exactly calib-mib MiB), and records the
SHA-256 of the kernel's gfx950 assembly in the build that was profiled (kernel_digests.json,
written by the build), so that a reader can tell whether the figure still applies.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
OUR_KERNELS = ("k_", "(anonymous namespace)::k_")


DIGESTS = os.path.join(ROOT, "paper_2603_00145_amd", "kernel_digests.json")


def kernel_digest(kernel):
    """SHA-256 of the kernel's assembly in the current build (None without a build); a
    template kernel is recorded under its name without arguments (the build digests the
    instantiation the benchmark runs)."""
    try:
        with open(DIGESTS) as f:
            return json.load(f).get(kernel.split("<")[0])
    except (OSError, ValueError):
        return None


def _short(name: str) -> str:
    """Kernel name without return type, namespace and argument list (template arguments
    kept)."""
    n = name[5:] if name.startswith("void ") else name
    if n.startswith("(anonymous namespace)::"):
        n = n[len("(anonymous namespace)::"):]
    return n.split("(")[0].strip()


def _rows(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        sys.exit(f"no {pattern} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def counters(d, counter):
    """{dispatch id: (kernel name, value)} of one counter."""
    out = {}
    for r in _rows(d, "*counter_collection.csv"):
        if r["Counter_Name"] == counter:
            out[r["Dispatch_Id"]] = (r["Kernel_Name"], float(r["Counter_Value"]))
    return out


def per_kernel(vals, kernel):
    x = [v for (n, v) in vals.values() if _short(n) == kernel]
    if not x:
        sys.exit(f"kernel {kernel} not found")
    return statistics.mean(x), len(x)


def calib(vals):
    """Counter value of the calibration kernel (the largest neg kernel dispatch)."""
    x = [v for (n, v) in vals.values() if "neg" in n.lower()]
    if not x:
        sys.exit("calibration kernel (torch.neg) not found")
    return max(x)


def cmd_traffic(a):
    f_vals = counters(a.fetch_dir, "FETCH_SIZE")
    w_vals = counters(a.write_dir, "WRITE_SIZE")
    fk, nf = per_kernel(f_vals, a.kernel)
    wk, nw = per_kernel(w_vals, a.kernel)
    cal_bytes = a.calib_mib * 1024.0 * 1024.0
    cf, cw = calib(f_vals), calib(w_vals)         # KiB
    sf, sw = cal_bytes / (cf * 1024.0), cal_bytes / (cw * 1024.0)
    traffic = fk * 1024.0 * sf + wk * 1024.0 * sw
    digest = kernel_digest(a.kernel)
    if digest is None:
        sys.exit("no kernel_digests.json entry: build first")
    txt = f"""# HBM traffic of {a.kernel} ({a.workload})

Commands (from the repository root on the GPU machine, run after `cd /tmp`):

    {a.command_fetch}
    {a.command_write}

| counter | {a.kernel}, KiB per dispatch (mean of {min(nf, nw)}) | calibration kernel (torch.neg, {a.calib_mib} MiB in + out), KiB | scale |
|---|---|---|---|
| FETCH_SIZE | {fk:.1f} | {cf:.1f} | {sf:.4f} |
| WRITE_SIZE | {wk:.1f} | {cw:.1f} | {sw:.4f} |

HBM bytes per launch = FETCH x scale + WRITE x scale:

traffic_bytes: {traffic:.0f}
kernel: {a.kernel}
kernel_asm_sha256: {digest}
source: {a.source}
"""
    with open(a.out, "w") as f:
        f.write(txt)
    print(txt)


def cmd_valu(a):
    rows = _rows(a.dir, "*counter_collection.csv")
    per = {}
    names = {}
    for r in rows:
        if _short(r["Kernel_Name"]) != a.kernel:
            continue
        d = int(r["Dispatch_Id"])
        per.setdefault(d, {})[r["Counter_Name"]] = \
            per.get(d, {}).get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names[r["Counter_Name"]] = 1
    if not per:
        sys.exit(f"kernel {a.kernel} not found")
    with open(a.pairs_log) as f:
        pairs = json.load(f)
    disp = sorted(per)
    if len(disp) != len(pairs):
        sys.exit(f"{len(disp)} dispatches of {a.kernel} but {len(pairs)} logged steps")
    digest = kernel_digest(a.kernel)
    if digest is None:
        sys.exit("no kernel_digests.json entry: build first")
    means = {c: statistics.mean(per[d].get(c, 0.0) for d in disp) for c in sorted(names)}
    mp = statistics.mean(pairs)
    txt = f"""# VALU instruction mix of {a.kernel} ({a.workload})

Command (from the repository root on the GPU machine, run after `cd /tmp`):

    {a.command}

Wave-level instruction counts per dispatch (mean of {len(disp)} dispatches, one per training
iteration; each covers up to 64 lanes), and the contributing (Gaussian, voxel) pairs gm_bin
reported for the same iterations.

| counter | per dispatch | per contributing pair |
|---|---|---|
"""
    for c, v in means.items():
        txt += f"| {c} | {v:.4g} | {v / mp:.4f} |\n"
    txt += f"\npairs_per_launch: {mp:.0f}\n"
    for c, v in means.items():
        txt += f"{c}: {v:.0f}\n"
    txt += f"kernel: {a.kernel}\nkernel_asm_sha256: {digest}\nsource: {a.source}\n"
    if a.note:
        txt += "\n" + a.note + "\n"
    with open(a.out, "w") as f:
        f.write(txt)
    print(txt)


def cmd_util(a):
    rows = _rows(a.dir, "*counter_collection.csv")
    per = {}
    for r in rows:
        if _short(r["Kernel_Name"]) != a.kernel:
            continue
        d = per.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    if not per:
        sys.exit(f"kernel {a.kernel} not found")
    names = sorted({c for d in per.values() for c in d})
    m = {c: statistics.mean(d.get(c, 0.0) for d in per.values()) for c in names}
    need = ("GRBM_GUI_ACTIVE", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_VALU",
            "SQ_ACTIVE_INST_SCA", "SQ_WAIT_INST_LDS", "SQ_WAIT_INST_ANY")
    for c in need:
        if c not in m:
            sys.exit(f"counter {c} missing")
    digest = kernel_digest(a.kernel)
    if digest is None:
        sys.exit("no kernel_digests.json entry: build first")
    # GRBM_GUI_ACTIVE comes summed over the XCDs: per XCD it is the dispatch's GPU clocks
    clocks = m["GRBM_GUI_ACTIVE"] / a.xcds
    cu_clocks = clocks * a.cus
    rows_out = [
        ("LDS busy (LdsUtil: SQ_LDS_IDX_ACTIVE / (clocks x CUs))", m["SQ_LDS_IDX_ACTIVE"] / cu_clocks),
        ("LDS stalled on bank conflicts (SQ_LDS_BANK_CONFLICT / (clocks x CUs))",
         m["SQ_LDS_BANK_CONFLICT"] / cu_clocks),
        ("vector issue busy (VALUBusy: SQ_ACTIVE_INST_VALU / (clocks x CUs))",
         m["SQ_ACTIVE_INST_VALU"] / cu_clocks),
        ("scalar issue busy (SQ_ACTIVE_INST_SCA / (clocks x CUs))", m["SQ_ACTIVE_INST_SCA"] / cu_clocks),
        ("share of issue waits that wait on LDS (SQ_WAIT_INST_LDS / SQ_WAIT_INST_ANY)",
         m["SQ_WAIT_INST_LDS"] / m["SQ_WAIT_INST_ANY"]),
    ]
    txt = f"""# LDS and issue utilisation of {a.kernel} ({a.workload})

Command (from the repository root on the GPU machine, run after `cd /tmp`):

    {a.command}

Counters per dispatch (mean of {len(per)} dispatches), summed over the chip; clocks =
GRBM_GUI_ACTIVE / {a.xcds} XCDs = {clocks:.0f}, CUs = {a.cus}.

| fraction | value |
|---|---|
"""
    for k, v in rows_out:
        txt += f"| {k} | {v:.3f} |\n"
    txt += "\n"
    for c in names:
        txt += f"{c}: {m[c]:.0f}\n"
    txt += f"kernel: {a.kernel}\nkernel_asm_sha256: {digest}\nsource: {a.source}\n"
    if a.note:
        txt += "\n" + a.note + "\n"
    with open(a.out, "w") as f:
        f.write(txt)
    print(txt)


def cmd_stats(a):
    rows = _rows(a.dir, "*kernel_stats.csv")
    lines = []
    for r in rows:
        name = _short(r["Name"])
        if not name.startswith("k_"):
            continue
        lines.append((float(r["TotalDurationNs"]), name, int(r["Calls"]),
                      float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    lines.sort(reverse=True)
    txt = f"# Kernel time summary: {a.workload}\n\nCommand (from the repository root on the GPU " \
          f"machine, run after `cd /tmp`):\n\n    {a.command}\n\nLibrary kernels only.\n\n" \
          "| kernel | calls | avg us | min us | max us |\n|---|---|---|---|---|\n"
    for _, name, calls, avg, mn, mx in lines:
        txt += f"| {name} | {calls} | {avg:.1f} | {mn:.1f} | {mx:.1f} |\n"
    if a.note:
        txt += "\n" + a.note + "\n"
    with open(a.out, "w") as f:
        f.write(txt)
    print(txt)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch-dir", required=True)
    t.add_argument("--write-dir", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--source", required=True, help="the kernel's source file (for the reader)")
    t.add_argument("--calib-mib", type=int, default=1024)
    t.add_argument("--workload", default="training iteration, 256^3 workload")
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--out", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--dir", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--source", required=True)
    v.add_argument("--pairs-log", required=True)
    v.add_argument("--workload", default="training iteration, 256^3 workload")
    v.add_argument("--command", required=True)
    v.add_argument("--note", default="")
    v.add_argument("--out", required=True)
    u = sub.add_parser("util")
    u.add_argument("--dir", required=True)
    u.add_argument("--kernel", required=True)
    u.add_argument("--source", required=True)
    u.add_argument("--xcds", type=int, default=8)
    u.add_argument("--cus", type=int, default=256)
    u.add_argument("--workload", default="training iteration, 256^3 workload")
    u.add_argument("--command", required=True)
    u.add_argument("--note", default="")
    u.add_argument("--out", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--workload", default="training iteration, 256^3 workload")
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    a = ap.parse_args()
    {"traffic": cmd_traffic, "stats": cmd_stats, "valu": cmd_valu, "util": cmd_util}[a.cmd](a)


if __name__ == "__main__":
    main()
