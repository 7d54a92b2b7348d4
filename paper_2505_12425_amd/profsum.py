"""Summarise rocprofv3 output of the benchmark into short text records.

    python -m paper_2505_12425_amd.profsum stats --dir D --out F.md --cmd "..."
        kernel-trace statistics (``rocprofv3 --kernel-trace --stats -f csv``)
        of every kernel, with readable labels.
    python -m paper_2505_12425_amd.profsum traffic --fetch D1 --write D2 \\
            --copy-bytes N --out F.json --md F.md --cmd-fetch "..." --cmd-write "..." \\
            [--only warp_f32,warp_u8]
        HBM bytes per launch from one ``--pmc FETCH_SIZE`` and one
        ``--pmc WRITE_SIZE`` run: each counter's mean per dispatch, scaled by
        the factor that maps the same counter on the plain copy kernel
        (N bytes read and N written per dispatch) to N bytes.

The JSON record carries the hash of the kernel sources it was taken on (runs
on the same sources merge into it); the benchmark reports a kernel's traffic
only while that hash still matches.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")


def kernel_source_sha() -> str:
    """Hash of every kernel and host source file of libkr."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


_TPL = re.compile(r"kr::k_(tiled|batch)<(\d+), (\d+), (true|false), (\d+), (\d+), (\d+), (\d+), \d+>")


def label(name: str) -> str:
    """Readable label: e.g. 'warp_u8 c3 tiled 4x16x1x4' for a k_tiled instance."""
    m = _TPL.search(name)
    if m:
        kind, op, c, f32, px, txt, cpt, rpt = m.groups()
        opn = "warp" if op == "1" else "resize"
        dt = "f32" if f32 == "true" else "u8"
        pre = "batch_" if kind == "batch" else ""
        return f"{pre}{opn}_{dt} c{c} {px}x{txt}x{cpt}x{rpt}"
    if "k_copy" in name:
        return "copy"
    if "k_generic" in name:
        return "generic " + name.split("(")[0].split("k_generic")[-1]
    return name.split("(")[0][:60]


def bench_key(name: str) -> str | None:
    """The benchmark's name for a kernel ('warp_f32', 'batch_resize_f32', ...)."""
    m = _TPL.search(name)
    if not m:
        return "copy" if "k_copy" in name else None
    kind, op, c, f32 = m.groups()[:4]
    if c != "3":
        return None
    return ("batch_" if kind == "batch" else "") + ("warp" if op == "1" else "resize") + \
        ("_f32" if f32 == "true" else "_u8")


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def stats(dir_: str, out: str, cmd: str) -> None:
    path = _one(os.path.join(dir_, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", cmd, "```", "",
             "| kernel | calls | avg us | min us | max us | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append("| {} | {} | {:.2f} | {:.2f} | {:.2f} | {:.3f} | {:.1f} |".format(
            label(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    lines += ["", "Full kernel names:", ""]
    lines += [f"- `{label(r['Name'])}`: `{r['Name'].split('(')[0]}`" for r in rows]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_means(dir_: str, counter: str):
    path = _one(os.path.join(dir_, "**", "*counter_collection.csv"))
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def traffic(fetch_dir, write_dir, copy_bytes, out, md, cmd_fetch, cmd_write, only=None) -> None:
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    copy_f = [v for k, v in fetch.items() if bench_key(k) == "copy"]
    copy_w = [v for k, v in write.items() if bench_key(k) == "copy"]
    if not copy_f or not copy_w:
        raise SystemExit("the profiled run has no copy-kernel dispatch to calibrate against")
    f_fac = copy_bytes / (copy_f[0][0] * 1024.0)
    w_fac = copy_bytes / (copy_w[0][0] * 1024.0)
    # per benchmark kernel: the instantiation with the most dispatches
    best = {}
    for name, (fk, n) in fetch.items():
        key = bench_key(name)
        if key in (None, "copy") or name not in write or (only and key not in only):
            continue
        if key not in best or n > best[key][1]:
            best[key] = (name, n)
    kernels = {}
    for key, (name, n) in sorted(best.items()):
        fk, wk = fetch[name][0], write[name][0]
        kernels[key] = {"kernel": label(name), "dispatches": n, "fetch_kib": round(fk, 1),
                        "write_kib": round(wk, 1), "fetch_bytes": round(fk * 1024 * f_fac),
                        "write_bytes": round(wk * 1024 * w_fac),
                        "bytes_per_launch": round(fk * 1024 * f_fac + wk * 1024 * w_fac)}
    calib = {"copy_bytes_each_way": copy_bytes, "fetch_kib_per_copy": round(copy_f[0][0], 1),
             "write_kib_per_copy": round(copy_w[0][0], 1), "fetch_factor": round(f_fac, 4),
             "write_factor": round(w_fac, 4)}
    for k in kernels.values():
        k.update(command_fetch=cmd_fetch, command_write=cmd_write, calibration=calib)
    sha = kernel_source_sha()
    rec = {"source_sha": sha, "kernels": {}}
    if os.path.exists(out):  # merge with entries taken on the same sources
        old = json.load(open(out))
        if old.get("source_sha") == sha:
            rec["kernels"].update(old.get("kernels", {}))
    rec["kernels"].update(kernels)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    if md:
        lines = ["# HBM traffic per launch (rocprofv3 --pmc)", "", "Commands:", "", "```", cmd_fetch, cmd_write,
                 "```", "",
                 f"Calibration: the copy kernel moves {copy_bytes} B each way per dispatch; FETCH_SIZE reads "
                 f"{copy_f[0][0]:.1f} KiB (factor {f_fac:.4f}), WRITE_SIZE {copy_w[0][0]:.1f} KiB "
                 f"(factor {w_fac:.4f}).", "",
                 "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB | total MB |",
                 "|---|---:|---:|---:|---:|---:|---:|"]
        for key, k in kernels.items():
            lines.append(f"| {key} ({k['kernel']}) | {k['dispatches']} | {k['fetch_kib']} | {k['write_kib']} | "
                         f"{k['fetch_bytes'] / 1e6:.2f} | {k['write_bytes'] / 1e6:.2f} | "
                         f"{k['bytes_per_launch'] / 1e6:.2f} |")
        lines += ["", f"Kernel sources hash: {sha}"]
        with open(md, "w") as f:
            f.write("\n".join(lines) + "\n")


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--md", default=None)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--only", default=None, help="comma-separated benchmark kernel names to record")
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.dir, a.out, a.cmd)
    else:
        traffic(a.fetch, a.write, a.copy_bytes, a.out, a.md, a.cmd_fetch, a.cmd_write,
                a.only.split(",") if a.only else None)


if __name__ == "__main__":
    main()
