"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

  python -m paper_2111_02912_amd.profsummary stats KERNEL_STATS_CSV --cmd "..."
  python -m paper_2111_02912_amd.profsummary bench BENCH_OUTPUT --cmd "..." --title "..."
  python -m paper_2111_02912_amd.profsummary pmc FETCH_CSV WRITE_CSV --calib-bytes N
         --cmd-fetch "..." --cmd-write "..." [--json OUT.json]
  python -m paper_2111_02912_amd.profsummary timeline KERNEL_TRACE_CSV --cmd "..."
         [--after-gap-ms 20] [--steps K]

The timeline mode reads a kernel trace, keeps the dispatches after the
last idle gap of at least --after-gap-ms (a host pause placed before the
timed steps), and reports where the GPU is busy and where it idles: the
union of kernel intervals, the time with 0, 1, 2, 3+ kernels in flight, the
busy time per kernel class and the longest idle gaps with the kernels on
either side.

The pmc mode scales each kernel's FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
by the ratio "known bytes / counter reading" of the calibration copy kernel
(a device-to-device copy of N bytes in the same run) and reports bytes per
dispatch.  --json writes {kernel class: {fetch, write, sources}} where
sources is a hash of the HIP sources, so a reader can tell whether the
counters still describe the current kernels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# kernel name -> timing class of the library
_INDEX = ("k_points_hist", "k_tile_scatter", "k_scan", "k_subproblems", "k_owner_")


def _targs(name: str):
    """Template arguments of a kernel symbol, e.g. 'k_cols<512, 16, false, 512>'."""
    if "<" not in name:
        return []
    inner = name[name.index("<") + 1:name.rindex(">")] if ">" in name else ""
    return [t.strip() for t in inner.split(",")]


def kernel_class(name: str):
    # the short name: no return type, namespace or argument list (argument
    # types may carry namespaces of their own)
    base = short(name).split("<")[0].split("::")[-1].strip()
    if any(base.startswith(k) for k in _INDEX):
        return "index"
    ta = _targs(name)
    if base in ("k_first_pass", "k_rows_first"):
        return "fft_first"
    if base in ("k_last_adj", "k_rows_last_adj"):
        return "fft_last_adj"
    if base in ("k_cols", "k_cols_pf", "k_mid_pass"):
        # k_cols[_pf]<L, E, INV, NT[, DER]>, k_mid_pass<MAXE, INV>
        inv = ta[2] if base.startswith("k_cols") and len(ta) > 2 else (ta[1] if len(ta) > 1 else "false")
        return "fft_mid_inv" if inv == "true" else "fft_mid_fwd"
    if base in ("k_gather_staged", "k_gather"):
        # <D, J, MODE, ...>
        return "gather_jac" if len(ta) > 2 and ta[2] == "1" else "gather"
    if base == "k_reduce_parts":
        return "gather_jac"
    if base.startswith("k_spread") or base == "k_permute":
        return "spread"
    return None


# sources of the NUFFT kernels, their launch configuration and the plan
# (the CG, off-resonance and batch sources do not affect those kernels)
NUFFT_SOURCES = ("kbn_internal.h", "kbn_window.h", "plan.cpp", "points.hip", "fft.hip", "fft_fast.hip",
                 "interp.hip")


def sources_hash() -> str:
    h = hashlib.sha256()
    for name in NUFFT_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0] if "(" in name else name


def stats(path: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {cmd}",
           f"# source hash: {sources_hash()}", "",
           f"{'kernel':58s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"{short(r['Name'])[:58]:58s} {int(r['Calls']):6d} "
                   f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['MinNs']) / 1e3:10.1f} "
                   f"{float(r['MaxNs']) / 1e3:10.1f} {100 * float(r['TotalDurationNs']) / total:6.2f}")
    return "\n".join(out) + "\n"


def _per_kernel(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def pmc(fetch_csv, write_csv, calib_bytes, cmd_f, cmd_w, json_out=None, steps=1) -> str:
    fa = _per_kernel(fetch_csv)
    wa = _per_kernel(write_csv)

    def calib(agg):
        # the calibration copy is the largest single dispatch of a copy kernel
        best = None
        for name, vals in agg.items():
            if "elementwise" in name or "copyBuffer" in name:
                v = max(vals)
                best = v if best is None or v > best else best
        return best

    cf, cw = calib(fa), calib(wa)
    sf = calib_bytes / (cf * 1024.0) if cf else float("nan")
    sw = calib_bytes / (cw * 1024.0) if cw else float("nan")
    out = ["# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE per dispatch (mean over dispatches)",
           f"# fetch command: {cmd_f}", f"# write command: {cmd_w}",
           f"# calibration: device copy of {calib_bytes} bytes read FETCH_SIZE={cf:.0f} KiB, "
           f"WRITE_SIZE={cw:.0f} KiB -> scale fetch x{sf:.4f}, write x{sw:.4f}",
           f"# source hash: {sources_hash()}", "",
           f"{'kernel':58s} {'n':>4s} {'fetch_MB':>10s} {'write_MB':>10s}"]
    classes = {}
    for name in sorted(set(fa) | set(wa)):
        f = sum(fa.get(name, [0])) / max(len(fa.get(name, [])), 1) * 1024.0 * sf
        w = sum(wa.get(name, [0])) / max(len(wa.get(name, [])), 1) * 1024.0 * sw
        out.append(f"{short(name)[:58]:58s} {len(fa.get(name, [])):4d} {f / 1e6:10.2f} {w / 1e6:10.2f}")
        cls = kernel_class(name)
        if cls is not None:
            # totals over all dispatches of the run, divided per step below
            c = classes.setdefault(cls, {"fetch_per_step": 0.0, "write_per_step": 0.0})
            c["fetch_per_step"] += sum(fa.get(name, [])) * 1024.0 * sf / steps
            c["write_per_step"] += sum(wa.get(name, [])) * 1024.0 * sw / steps
    out.append("")
    out.append(f"per step ({steps} steps in the run), by kernel class:")
    for cls, c in sorted(classes.items()):
        out.append(f"  {cls:14s} fetch {c['fetch_per_step'] / 1e6:10.2f} MB  write {c['write_per_step'] / 1e6:10.2f} MB")
    if json_out:
        with open(json_out, "w") as fh:
            json.dump({"sources": sources_hash(), "calib_bytes": calib_bytes, "steps": steps,
                       "classes": classes}, fh, indent=1)
    return "\n".join(out) + "\n"


def _dims(r, name):
    """'x' or 'x*y*z' of a size column (one column or one per axis)."""
    if name in r:
        return r[name]
    d = [r.get(f"{name}_{a}", "") for a in "XYZ"]
    d = [v for v in d if v not in ("", "1", "0")]
    return "*".join(d) if d else "1"


def timeline(path: str, cmd: str, after_gap_ms: float = 20.0, steps: int = 1) -> str:
    rows = []
    shape = {}
    for r in csv.DictReader(open(path)):
        key = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]))
        rows.append(key)
        shape[key] = (_dims(r, "Grid_Size"), _dims(r, "Workgroup_Size"), r.get("LDS_Block_Size", "?"))
    rows.sort()
    if not rows:
        return "no dispatches\n"
    # the timed window starts after the last long idle gap
    first = 0
    end_so_far = rows[0][1]
    for i in range(1, len(rows)):
        if rows[i][0] - end_so_far >= after_gap_ms * 1e6:
            first = i
        end_so_far = max(end_so_far, rows[i][1])
    win = rows[first:]
    t0 = win[0][0]
    t1 = max(e for _, e, _ in win)
    span = t1 - t0
    # sweep: time with n kernels in flight, idle gaps
    ev = sorted([(s, 1) for s, _, _ in win] + [(e, -1) for _, e, _ in win])
    level = 0
    last = t0
    at = collections.Counter()
    gaps = []
    for t, d in ev:
        if t > last:
            at[min(level, 3)] += t - last
            if level == 0:
                gaps.append((t - last, last, t))
        level += d
        last = t
    busy = span - at[0]
    # busy time per class (intervals of the class, merged)
    per = collections.defaultdict(list)
    for s_, e_, n in win:
        per[kernel_class(n) or n.split("<")[0]].append((s_, e_))
    cls_busy = {}
    for c, iv in per.items():
        iv.sort()
        tot, cs, ce = 0, iv[0][0], iv[0][1]
        for s_, e_ in iv[1:]:
            if s_ > ce:
                tot += ce - cs
                cs, ce = s_, e_
            else:
                ce = max(ce, e_)
        cls_busy[c] = (tot + ce - cs, len(iv))

    def near(t, before):
        # kernel ending at t (before) or starting at t (after)
        for s_, e_, n in win:
            if (before and e_ == t) or (not before and s_ == t):
                return n[:40]
        return "?"

    out = ["# rocprofv3 --kernel-trace timeline of the timed window", f"# command: {cmd}",
           f"# source hash: {sources_hash()}",
           f"# window: dispatches after the last idle gap >= {after_gap_ms} ms ({len(win)} dispatches, "
           f"{steps} step(s))", "",
           f"window {span / 1e6:.3f} ms ({span / 1e6 / steps:.3f} ms per step); GPU busy {busy / 1e6:.3f} ms "
           f"({100 * busy / span:.1f} %), idle {at[0] / 1e6:.3f} ms ({100 * at[0] / span:.1f} %)",
           "kernels in flight: " + ", ".join(f"{k if k < 3 else '3+'}: {100 * at[k] / span:.1f} %"
                                            for k in range(4)), "",
           f"{'class':28s} {'dispatches':>10s} {'busy_ms':>9s} {'pct_of_window':>14s}"]
    for c, (t, n) in sorted(cls_busy.items(), key=lambda kv: -kv[1][0]):
        out.append(f"{c[:28]:28s} {n:10d} {t / 1e6:9.3f} {100 * t / span:14.1f}")
    gaps.sort(reverse=True)
    out += ["", f"idle gaps: {len(gaps)}, longest:", f"{'gap_us':>8s}  after -> before"]
    for g, a, b in gaps[:10]:
        out.append(f"{g / 1e3:8.1f}  {near(a, True)} -> {near(b, False)}")
    out += ["", "longest dispatches (grid size, workgroup size, LDS bytes):"]
    for r in sorted(win, key=lambda r: r[0] - r[1])[:15]:
        gs, ws, lds = shape[r]
        out.append(f"{(r[1] - r[0]) / 1e3:8.1f} us  {r[2][:50]:50s} grid {gs} wg {ws} lds {lds}")
    return "\n".join(out) + "\n"


def _fmt(v, indent=2):
    pad = " " * indent
    if isinstance(v, dict):
        lines = []
        for k, x in v.items():
            if isinstance(x, dict):
                lines.append(f"{pad}{k}:")
                lines.extend(_fmt(x, indent + 2))
            else:
                lines.append(f"{pad}{k}: {_num(x)}")
        return lines
    return [f"{pad}{_num(v)}"]


def _num(x):
    if isinstance(x, float):
        return f"{x:.6g}"
    if isinstance(x, list):
        return "[" + ", ".join(_num(e) for e in x) + "]"
    return str(x)


def bench(path: str, cmd: str, title: str) -> str:
    """Text summary of the last JSON line a bench.py run printed."""
    lines = [ln for ln in open(path).read().splitlines() if ln.strip().startswith("{")]
    d = json.loads(lines[-1])
    out = [title, f"command: {cmd}", f"source hash: {sources_hash()}", ""]
    head = ("metric", "value", "unit", "ms_per_step", "steps", "warmup", "dtype", "vs_baseline")
    for k in head:
        if k in d:
            out.append(f"{k}: {_num(d[k])}")
    for k, v in d.items():
        if k in head or k in ("n_gpus", "higher_is_better", "scaling", "data"):
            continue
        if isinstance(v, dict):
            out.append(f"{k}:")
            out.extend(_fmt(v))
        else:
            out.append(f"{k}: {_num(v)}")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    bsub = sub.add_parser("bench")
    bsub.add_argument("json")
    bsub.add_argument("--cmd", required=True)
    bsub.add_argument("--title", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--calib-bytes", type=int, required=True)
    p.add_argument("--cmd-fetch", required=True)
    p.add_argument("--cmd-write", required=True)
    p.add_argument("--json")
    p.add_argument("--steps", type=int, default=1, help="steps (incl. warm-up) in the counted run")
    t = sub.add_parser("timeline")
    t.add_argument("csv")
    t.add_argument("--cmd", required=True)
    t.add_argument("--after-gap-ms", type=float, default=20.0)
    t.add_argument("--steps", type=int, default=1, help="steps in the timed window")
    a = ap.parse_args()
    if a.mode == "bench":
        sys.stdout.write(bench(a.json, a.cmd, a.title))
    elif a.mode == "stats":
        sys.stdout.write(stats(a.csv, a.cmd))
    elif a.mode == "timeline":
        sys.stdout.write(timeline(a.csv, a.cmd, a.after_gap_ms, a.steps))
    else:
        sys.stdout.write(pmc(a.fetch_csv, a.write_csv, a.calib_bytes, a.cmd_fetch, a.cmd_write, a.json,
                             a.steps))


if __name__ == "__main__":
    main()
