"""Summarise rocprofv3 output of the benchmark into short text records.

    python -m paper_2505_12425_amd.profsum stats --dir D --out F.md --cmd "..."
        kernel-trace statistics (``rocprofv3 --kernel-trace --stats -f csv``)
        of every kernel, with readable labels.
    python -m paper_2505_12425_amd.profsum counters --dir D --out F.md --cmd "..." --px warp_u8=8294400,...
        shader-sequencer counters of one --pmc pass per benchmark kernel
        (instructions per output pixel, or the split of wave time).
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
import json
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")


def kernel_source_sha() -> str:
    """Hash of every kernel and host source file of libkr (the same hash the
    library carries in its build key)."""
    from .build import source_sha
    return source_sha()


_TPL = re.compile(r"kr::k_(tiled|batch)<(\d+), (\d+), (true|false), (\d+), (\d+), (\d+), (\d+), \d+"
                  r"(?:, (?:true|false))?>")
_OPS = {"0": "resize", "1": "warp", "2": "perspective"}
_POINT = re.compile(r"kr::(?:\(anonymous namespace\)::)?k_(nearest|flip_u8|flip_f32|gray|half|permute)<([^>]*)>")


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").split("(")[0]


def label(name: str) -> str:
    """Readable label: e.g. 'warp_u8 c3 4x16x1x4' for a k_tiled instance."""
    m = _TPL.search(name)
    if m:
        kind, op, c, f32, px, txt, cpt, rpt = m.groups()
        dt = "f32" if f32 == "true" else "u8"
        pre = "batch_" if kind == "batch" else ""
        src = " c1 f32-source" if c == "5" else f" c{c}"  # channel code 5: one-channel f32 source
        return f"{pre}{_OPS[op]}_{dt}{src} {px}x{txt}x{cpt}x{rpt}"
    if "k_copy" in name:
        return "copy"
    if "k_stream" in name:
        return "stream probe"
    if "k_generic" in name:
        return "generic " + _short(name).split("k_generic")[-1]
    m = _POINT.search(name)
    if m:
        if m.group(1) == "half":  # <C, DST_F32>: the exact 2x downscale kernel
            c, f32 = [t.strip() for t in m.group(2).split(",")]
            return f"resize_{'f32' if f32 == 'true' else 'u8'} c{c} half"
        return f"{m.group(1)}<{m.group(2)}>"
    return _short(name)[:60]


def _point_key(kind: str, args: str) -> str | None:
    a = [t.strip() for t in args.split(",")]
    if kind == "permute":  # <C, F32>
        return None if a[0] != "3" else ("permute_f32" if a[1] == "true" else "permute_u8")
    if kind in ("flip_u8", "flip_f32"):
        return kind if a[0] == "3" else None
    if kind == "half":  # <C, DST_F32>
        return None if a[0] != "3" else ("resize_f32" if a[1] == "true" else "resize_u8")
    if kind == "gray":  # <SRC_F32, DST_F32>
        return None if a[0] == "true" else ("gray_f32" if a[1] == "true" else "gray_u8")
    # nearest <C, SRC_F32, DST_F32>; the direction is told apart by grid size
    if a[0] != "3" or a[1] == "true":
        return None
    return "nearest_{}_" + ("f32" if a[2] == "true" else "u8")


def bench_key(name: str) -> str | None:
    """The benchmark's name for a kernel ('warp_f32', 'resize_tiled_u8', 'batch_resize_f32', ...).
    Nearest-resize kernels give a pattern with '{}' for the direction."""
    m = _TPL.search(name)
    if not m:
        if "k_copy" in name:
            return "copy"
        p = _POINT.search(name)
        return _point_key(*p.groups()) if p else None
    kind, op, c, f32 = m.groups()[:4]
    if c != "3":
        return None
    # per-image resizes: 'resize_u8' names the exact-2x kernel of the 4K
    # step, 'resize_tiled_u8' the LDS-tiled kernel of every other ratio
    name = _OPS[op] + ("_tiled" if op == "0" and kind != "batch" else "")
    return ("batch_" if kind == "batch" else "") + name + ("_f32" if f32 == "true" else "_u8")


def _overlap_stats(ev) -> dict:
    """Overlap figures of time-sorted dispatches (start, end, queue, label)."""
    n = len(ev)
    overl = [False] * n
    active = []  # (end, queue, index) of dispatches still running
    busy = total = 0
    cur_end = -1
    cur_start = 0
    peak = 0
    for i, (t0, t1, q, _) in enumerate(ev):
        active = [a for a in active if a[0] > t0]
        for a in active:
            if a[1] != q:
                overl[i] = True
                overl[a[2]] = True
        active.append((t1, q, i))
        peak = max(peak, len(active))
        total += t1 - t0
        if t0 > cur_end:
            busy += cur_end - cur_start if cur_end > 0 else 0
            cur_start, cur_end = t0, t1
        else:
            cur_end = max(cur_end, t1)
    busy += cur_end - cur_start if n else 0
    return {"dispatches": n, "queues": len({e[2] for e in ev}), "overlapping_another_queue": int(sum(overl)),
            "kernel_time_ms": round(total / 1e6, 3), "busy_time_ms": round(busy / 1e6, 3),
            "mean_concurrency": round(total / busy, 3) if busy else 0.0, "peak_concurrency": peak}


def overlap(dir_: str, out: str, cmd: str, gap_ms: float = 2.0) -> dict:
    """Concurrency of kernel executions across hardware queues, from a
    rocprofv3 kernel trace: how many dispatches overlap in time with a
    dispatch of another queue, the summed kernel time over the time any
    kernel runs (mean concurrency), and the most kernels running at once.
    The trace is also cut into segments at idle gaps of gap_ms or more (one
    segment per server run of a benchmark that runs several), each with the
    same figures."""
    path = _one(os.path.join(dir_, "**", "*kernel_trace.csv"))
    rows = list(csv.DictReader(open(path)))
    qcol = "Stream_Id" if rows and "Stream_Id" in rows[0] and any(r["Stream_Id"] not in ("", "0") for r in rows) \
        else "Queue_Id"
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r[qcol], label(r["Kernel_Name"])) for r in rows)
    res = _overlap_stats(ev)
    segs, cur, last_end = [], [], None
    for e in ev:
        if cur and e[0] - last_end >= gap_ms * 1e6:
            segs.append(cur)
            cur = []
        cur.append(e)
        last_end = e[1] if last_end is None or not cur[:-1] else max(last_end, e[1])
    if cur:
        segs.append(cur)
    res["segments"] = [_overlap_stats(sg) for sg in segs]
    row = ("| {dispatches} | {queues} | {overlapping_another_queue} | {kernel_time_ms} | {busy_time_ms} "
           "| {mean_concurrency} | {peak_concurrency} |")
    head = ("| dispatches | queues | overlapping a dispatch of another queue | kernel time (ms) "
            "| time any kernel runs (ms) | mean concurrency | peak concurrency |")
    lines = ["# Kernel overlap across queues (rocprofv3 kernel trace)", "", "Command:", "", "```", cmd, "```", "",
             f"Queues identified by {qcol}.", "", "Whole trace:", "", head, "|---:|---:|---:|---:|---:|---:|---:|",
             row.format(**res), "",
             f"Segments (the trace cut at idle gaps of {gap_ms:g} ms or more):", "", "| segment " + head,
             "|---:|---:|---:|---:|---:|---:|---:|---:|"]
    lines += [f"| {i} " + row.format(**sg) for i, sg in enumerate(res["segments"])]
    with open(out, "w") as f:
        f.write("\n".join(lines + [""]))
    return res


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
    lines += [f"- `{label(r['Name'])}`: `{_short(r['Name'])}`" for r in rows]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_means(dir_: str, counter: str):
    """Mean counter value per (kernel, grid size), with the dispatch count."""
    path = _one(os.path.join(dir_, "**", "*counter_collection.csv"))
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    out = {}
    for k, v in acc.items():
        if bench_key(k[0]) == "copy":
            # copies of several sizes share one grid; the calibration copy is
            # the largest, so keep the dispatches within 2x of the biggest
            top = max(v)
            v = [x for x in v if x >= 0.5 * top]
        out[k] = (sum(v) / len(v), len(v))
    return out


def _keyed(means):
    """Benchmark key -> the (kernel, grid) entries it covers.  A per-image key
    takes the entry with the most dispatches; a batch key ('batch_...') takes
    every entry, since one batch launches one kernel per group and the groups
    together make one step.  A nearest kernel seen at two grid sizes is the
    downscale at the smaller grid and the upscale at the larger."""
    grids = defaultdict(set)
    for (name, grid) in means:
        grids[name].add(grid)
    sel = defaultdict(list)
    for (name, grid), (_, n) in means.items():
        key = bench_key(name)
        if key is None:
            continue
        if "{}" in key:
            g = sorted(grids[name])
            if len(g) != 2:
                continue
            key = key.format("down" if grid == g[0] else "up")
        if key.startswith("batch_"):
            sel[key].append((name, grid))
        elif not sel[key] or n > means[sel[key][0]][1]:
            sel[key] = [(name, grid)]
    return dict(sel)


def traffic(fetch_dir, write_dir, copy_bytes, out, md, cmd_fetch, cmd_write, only=None) -> None:
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    fkeys, wkeys = _keyed(fetch), _keyed(write)
    if "copy" not in fkeys or "copy" not in wkeys:
        raise SystemExit("the profiled run has no copy-kernel dispatch to calibrate against")
    copy_f, copy_w = fetch[fkeys["copy"][0]], write[wkeys["copy"][0]]
    f_fac = copy_bytes / (copy_f[0] * 1024.0)
    w_fac = copy_bytes / (copy_w[0] * 1024.0)
    kernels = {}
    for key in sorted(fkeys):
        if key == "copy" or key not in wkeys or (only and key not in only):
            continue
        fk = sum(fetch[e][0] for e in fkeys[key])
        wk = sum(write[e][0] for e in wkeys[key])
        n = min(fetch[e][1] for e in fkeys[key])
        kernels[key] = {"kernel": " + ".join(label(e[0]) for e in fkeys[key]),
                        "grid": [e[1] for e in fkeys[key]], "dispatches": n,
                        "fetch_kib": round(fk, 1),
                        "write_kib": round(wk, 1), "fetch_bytes": round(fk * 1024 * f_fac),
                        "write_bytes": round(wk * 1024 * w_fac),
                        "bytes_per_launch": round(fk * 1024 * f_fac + wk * 1024 * w_fac)}
    calib = {"copy_bytes_each_way": copy_bytes, "fetch_kib_per_copy": round(copy_f[0], 1),
             "write_kib_per_copy": round(copy_w[0], 1), "fetch_factor": round(f_fac, 4),
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
                 f"{copy_f[0]:.1f} KiB (factor {f_fac:.4f}), WRITE_SIZE {copy_w[0]:.1f} KiB "
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


def _all_counter_means(dir_: str):
    """Mean value per dispatch of every counter, per (kernel, grid size)."""
    path = _one(os.path.join(dir_, "**", "*counter_collection.csv"))
    acc = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        acc[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: ({c: sum(v) / len(v) for c, v in cs.items()}, max(len(v) for v in cs.values()))
            for k, cs in acc.items()}


def counters(dir_: str, out: str, cmd: str, px: dict) -> dict:
    """Shader-sequencer counters of the benchmark's kernels, one --pmc pass:
    instructions per output pixel (SQ_INSTS_*: wave instructions, x 64 /
    output pixels) and LDS bank-conflict cycles per LDS instruction, or the
    split of wave time (SQ_WAVE_CYCLES) into waiting, issue-blocked and
    active.  px maps a benchmark key to the kernel's output pixels."""
    means = _all_counter_means(dir_)
    keyed = _keyed({k: (0.0, n) for k, (_, n) in means.items()})
    rows = {}
    for key, ents in sorted(keyed.items()):
        if key not in px:
            continue
        cs, n = means[ents[0]]
        rows[key] = {"kernel": label(ents[0][0]), "dispatches": n, **{c: round(v, 1) for c, v in cs.items()}}
    lines = ["# Shader-sequencer counters of the benchmark kernels (rocprofv3 --pmc)", "", "Command:", "", "```",
             cmd, "```", ""]
    if any("SQ_INSTS_VALU" in r for r in rows.values()):
        lines += ["Per dispatch, averaged over the run's dispatches of each kernel.  Instruction counts are wave",
                  "instructions, so `x 64 / output pixels` gives instructions per output pixel.",
                  "SQ_LDS_BANK_CONFLICT counts cycles the LDS stalls on bank conflicts.", "",
                  "| kernel | dispatches | waves | VALU / px | SALU / px | LDS instr / px | conflict cycles / LDS instr |",
                  "|---|---:|---:|---:|---:|---:|---:|"]
        for key, r in rows.items():
            f = 64.0 / px[key]
            lds = r.get("SQ_INSTS_LDS", 0.0)
            conf = f"{r.get('SQ_LDS_BANK_CONFLICT', 0.0) / lds:.2f}" if lds else "-"
            lines.append(f"| {key} ({r['kernel']}) | {r['dispatches']} | {r.get('SQ_WAVES', 0):.0f} | "
                         f"{r.get('SQ_INSTS_VALU', 0) * f:.1f} | {r.get('SQ_INSTS_SALU', 0) * f:.1f} | "
                         f"{lds * f:.2f} | {conf} |")
    if any("SQ_WAVE_CYCLES" in r for r in rows.values()):
        lines += ["Fractions of SQ_WAVE_CYCLES (summed over waves), averaged over each kernel's dispatches.",
                  "wait = waiting on a dependency (s_waitcnt, barrier); issue = ready but waiting for an",
                  "instruction slot; active = issuing, of which VALU, LDS and VMEM are shown.", "",
                  "| kernel | wait | issue | active | VALU | LDS | VMEM |", "|---|---:|---:|---:|---:|---:|---:|"]
        for key, r in rows.items():
            wc = r.get("SQ_WAVE_CYCLES", 0.0) or 1.0
            lines.append(f"| {key} ({r['kernel']}) | {r.get('SQ_WAIT_ANY', 0) / wc:.2f} | "
                         f"{r.get('SQ_WAIT_INST_ANY', 0) / wc:.2f} | {r.get('SQ_ACTIVE_INST_ANY', 0) / wc:.2f} | "
                         f"{r.get('SQ_ACTIVE_INST_VALU', 0) / wc:.2f} | {r.get('SQ_ACTIVE_INST_LDS', 0) / wc:.2f} | "
                         f"{r.get('SQ_ACTIVE_INST_VMEM', 0) / wc:.2f} |")
    lines += ["", f"Kernel sources hash: {kernel_source_sha()}"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--cmd", required=True)
    o = sub.add_parser("overlap")
    o.add_argument("--dir", required=True)
    o.add_argument("--out", required=True)
    o.add_argument("--cmd", required=True)
    o.add_argument("--gap-ms", type=float, default=2.0)
    q = sub.add_parser("counters")
    q.add_argument("--dir", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--cmd", required=True)
    q.add_argument("--px", required=True, help="key=pixels,... output pixels of each benchmark kernel")
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
    elif a.what == "counters":
        counters(a.dir, a.out, a.cmd, {k: int(v) for k, v in (e.split("=") for e in a.px.split(","))})
    elif a.what == "overlap":
        print(json.dumps(overlap(a.dir, a.out, a.cmd, a.gap_ms)))
    else:
        traffic(a.fetch, a.write, a.copy_bytes, a.out, a.md, a.cmd_fetch, a.cmd_write,
                a.only.split(",") if a.only else None)


if __name__ == "__main__":
    main()
