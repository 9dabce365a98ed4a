"""Summaries of rocprofv3 result databases for the profiles/ folder, and the
lookup bench.py uses to report a kernel's measured HBM traffic.

A summary is a short markdown file: the commands that produced the databases,
the kernel-trace statistics, the per-dispatch FETCH_SIZE / WRITE_SIZE readings
and the plain-copy calibration, and two machine-readable footer lines:

    kernel-source-sha256: <hash of the sources the kernel is built from>
    traffic-per-launch-bytes <kernel filter> <f64|f32>: <bytes>

The traffic is (FETCH_SIZE * fetch scale + WRITE_SIZE * write scale) * 1024,
averaged over the kernel's dispatches, where each scale is the copy's known
byte count over what the counter reads for it.  bench.py reports it only while
the hash still matches the sources (otherwise the kernel has changed since the
counters were taken and the figure is stale).

    python -m paper_2410_19075_amd.profsum --out profiles/X.md --filter k_ring_stage \
        --sources ring.hip,models.h,nd_dev.h,runtime.hip --trace kt.db \
        --fetch f.db --write w.db --copy-fetch cf.db --copy-write cw.db \
        --copy-bytes 1073741824 --cmd "..." [--cmd "..."]
"""
import argparse
import collections
import hashlib
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def read_traffic(md_path, kfilter, dtype, files):
    """Measured bytes per launch from a summary, or None when the summary is
    missing or was taken on other kernel sources."""
    if not os.path.exists(md_path):
        return None
    txt = open(md_path).read()
    m = re.search(r"^kernel-source-sha256: (\w+)$", txt, re.M)
    if not m or m.group(1) != source_hash(files):
        return None
    m = re.search(r"^traffic-per-launch-bytes %s %s: ([0-9.eE+]+)$" % (re.escape(kfilter), dtype), txt, re.M)
    return float(m.group(1)) if m else None


def _kernels(db):
    con = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for name, dur in con.execute("select name, duration from kernels"):
        agg[name].append(dur)
    return agg


def _counters(db):
    con = sqlite3.connect(db)
    cur = con.execute("select * from counters_collection limit 1")
    cols = {d[0]: i for i, d in enumerate(cur.description)}
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in con.execute("select * from counters_collection"):
        agg[r[cols["kernel_name"]]][r[cols["counter_name"]]].append(r[cols["value"]])
    return agg


def _short(n):
    n = n.replace("nd::", "").split("(")[0]
    return n.replace("void ", "")[:70]


def _dtype(name):
    return "f32" if re.search(r"<[^>]*\bfloat\b", name) else "f64"


def _sq_section(a):
    """Per-dispatch averages of every counter of the --sq pass for the filtered
    kernels, and figures derived from them with the kernel's average duration
    from --trace in place of the GPU-busy cycles of the profiler's own derived
    metrics: VALU busy = SQ_ACTIVE_INST_VALU (quad-cycles) / (CUs x cycles);
    VALU issue share = SQ_INSTS_VALU x 4 cycles / (SIMDs x cycles) (a wave64
    VALU instruction holds its SIMD for 4 cycles, transcendental ones longer);
    LDS conflict share = SQ_LDS_BANK_CONFLICT / (CUs x cycles); conflicts per
    LDS access = SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)."""
    c = _counters(a.sq)
    sel = {n: d for n, d in c.items() if any(f in n for f in a.filter.split("|"))}
    names = sorted({cn for d in sel.values() for cn in d})
    L = ["## SQ counters per dispatch (`--pmc " + " ".join(names) + "`)", "",
         "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    avg = {}
    for n, d in sorted(sel.items()):
        avg[n] = {cn: sum(v) / len(v) for cn, v in d.items() if v}
        L.append(f"| `{_short(n)}` | " + " | ".join(f"{avg[n][cn]:.4g}" if cn in avg[n] else "-" for cn in names) + " |")
    L.append("")
    dur = {}
    if a.trace:
        for n, v in _kernels(a.trace).items():
            dur[n] = sum(v) / len(v) * 1e-9
    cus = a.simds // 4

    def fmt(x, f="%.2f"):
        return "-" if x is None else f % x

    rows = []
    for n, m in sorted(avg.items()):
        cyc = dur.get(n, 0.0) * a.clock_ghz * 1e9
        busy = m["SQ_ACTIVE_INST_VALU"] / (cus * cyc) if cyc and "SQ_ACTIVE_INST_VALU" in m else None
        share = m["SQ_INSTS_VALU"] * 4 / (a.simds * cyc) if cyc and "SQ_INSTS_VALU" in m else None
        conf = m["SQ_LDS_BANK_CONFLICT"] / (cus * cyc) if cyc and "SQ_LDS_BANK_CONFLICT" in m else None
        idx = m.get("SQ_LDS_IDX_ACTIVE", 0.0) - m.get("SQ_LDS_BANK_CONFLICT", 0.0)
        per = m["SQ_LDS_BANK_CONFLICT"] / idx if idx > 0 and "SQ_LDS_BANK_CONFLICT" in m else None
        rows.append(f"| `{_short(n)}` | {dur.get(n, 0) * 1e6:.2f} | {fmt(busy)} | {fmt(share)} | {fmt(conf)} | "
                    f"{fmt(per, '%.3f')} |")
    L += ["Derived (%d CUs, %d SIMDs, %.1f GHz; durations from the kernel trace):" % (cus, a.simds, a.clock_ghz), "",
          "| kernel | avg us | VALU busy | VALU issue share | LDS conflict share | conflicts per LDS access |",
          "|---|---|---|---|---|---|"] + rows + [""]
    return L


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--filter", required=True,
                    help="substring naming the kernel the traffic is for ('a|b': either, e.g. two kernels of one stage)")
    ap.add_argument("--sources", required=True, help="comma-separated files under csrc/ the kernel is built from")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=0)
    ap.add_argument("--group", type=int, default=1, help="dispatches of the filtered kernels per launch unit")
    ap.add_argument("--sq", help="counter database of an --pmc pass over SQ_* (and GRBM_*) counters")
    ap.add_argument("--clock-ghz", type=float, default=2.4, help="shader clock for the issue-time estimate")
    ap.add_argument("--simds", type=int, default=1024, help="SIMDs of the chip (256 CUs x 4)")
    ap.add_argument("--cmd", action="append", default=[])
    a = ap.parse_args()
    L = [f"# {a.title or a.filter}", "", "Commands (run from the repository root):", "", "```"] + a.cmd + ["```", ""]
    if a.trace:
        k = _kernels(a.trace)
        tot = sum(sum(v) for v in k.values())
        L += ["## Kernel trace (`--kernel-trace --stats`)", "", "| kernel | calls | avg us | total ms | share |",
              "|---|---|---|---|---|"]
        for n, v in sorted(k.items(), key=lambda kv: -sum(kv[1]))[:12]:
            L.append(f"| `{_short(n)}` | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {sum(v) / 1e6:.2f} | "
                     f"{100 * sum(v) / tot:.1f}% |")
        L.append("")
    scale = {}
    for cname, db in (("FETCH_SIZE", a.copy_fetch), ("WRITE_SIZE", a.copy_write)):
        if db and a.copy_bytes:
            c = _counters(db)
            vals = [v for n, d in c.items() if "copyBuffer" in n or "elementwise" in n for v in d.get(cname, [])]
            big = max(vals)
            scale[cname] = a.copy_bytes / (big * 1024.0)
    if scale:
        L += ["## Counter calibration (plain device copy of %.0f bytes)" % a.copy_bytes, "",
              "| counter | reads (KiB) | scale |", "|---|---|---|"]
        for cname, s in scale.items():
            L.append(f"| {cname} | {a.copy_bytes / 1024.0 / s:.6g} | {s:.4g} |")
        L.append("")
    per = collections.defaultdict(lambda: [0.0, 0])
    for cname, db in (("FETCH_SIZE", a.fetch), ("WRITE_SIZE", a.write)):
        if not db:
            continue
        c = _counters(db)
        L += [f"## {cname} per dispatch (KiB)", "", "| kernel | avg | dispatches |", "|---|---|---|"]
        for n, d in sorted(c.items()):
            if "nd::" not in n:
                continue
            v = d.get(cname, [])
            if not v:
                continue
            L.append(f"| `{_short(n)}` | {sum(v) / len(v):.6g} | {len(v)} |")
            if any(f in n for f in a.filter.split("|")):
                acc = per[(_dtype(n), cname)]
                acc[0] += sum(v) * 1024.0 * scale.get(cname, 1.0)
                acc[1] += len(v)
        L.append("")
    if a.sq:
        L += _sq_section(a)
    L += ["kernel-source-sha256: " + source_hash(a.sources.split(","))]
    for dt in ("f64", "f32"):
        f, w = per.get((dt, "FETCH_SIZE")), per.get((dt, "WRITE_SIZE"))
        if f and w and f[1] and w[1]:
            L.append(f"traffic-per-launch-bytes {a.filter} {dt}: {a.group * (f[0] / f[1] + w[0] / w[1]):.6g}")
    with open(a.out, "w") as fh:
        fh.write("\n".join(L) + "\n")
    print("\n".join(L))


if __name__ == "__main__":
    main()
