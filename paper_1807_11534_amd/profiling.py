"""Summaries of rocprofv3 result databases (rocpd SQLite) for the profiles/ notes.

    python -m paper_1807_11534_amd.profiling [--trace T.db] [--fetch F.db] [--write W.db]
        [--kernel SUBSTRING] [--copy-mib N] [--bench-json B.json] [--traced-json T.out]
        [--fetch-json F.out] [--write-json W.out]
    python -m paper_1807_11534_amd.profiling --combine PART.md [PART.md ...]
    python -m paper_1807_11534_amd.profiling --sq S.db --sq-json S.out

--trace    database of `rocprofv3 --kernel-trace --stats`
--fetch    database of `rocprofv3 --pmc FETCH_SIZE`   (KiB per dispatch)
--write    database of `rocprofv3 --pmc WRITE_SIZE`   (KiB per dispatch)
--copy-mib size of the plain buffer copy run first in the counter passes; the
           ratio (copy bytes) / (counter bytes of that copy) calibrates both
           counters.
--traced-json output of the benchmark run under the trace: its roofline pass is
           the last GPU work of the run, so the last `launches` dispatches of
           the kernel are the launches its HIP events timed
--fetch-json, --write-json  the same for the two counter runs (their roofline
           pass gives the dispatches averaged)
--sq, --sq-json  database and benchmark output of a run of instruction
           counters (SQ_INSTS_VALU, ...): their per-launch averages over the
           roofline pass, as the record bench.py reads for roofline.valu
Prints a short markdown report: per-kernel duration table, and for the kernel
matching --kernel its average duration, calibrated HBM bytes per launch and,
with --bench-json, the benchmark's live figures beside them.  Each counter
run also prints a `counter_bytes_per_launch:` line; --combine reads such
partial reports (from separate profiler runs) and prints the traffic record
(FETCH_SIZE + WRITE_SIZE bytes per launch of one kernel).
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sqlite3

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# sources that define the iteration kernels: a change to any voids a
# recorded traffic figure
KERNEL_SOURCES = ("iterate.hip", "rdseg_device.h", "components_device.h")


def kernel_source_digest():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(_CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, profiles_dir):
    """HBM bytes per launch of `kernel` recorded in a summary under
    profiles_dir, or None when none was taken from the current kernel sources."""
    want = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(profiles_dir, "*.md"))):
        text = open(path).read()
        k = re.search(r"^traffic_kernel: (.+)$", text, re.M)
        b = re.search(r"^traffic_bytes_per_launch: ([0-9.eE+]+)$", text, re.M)
        d = re.search(r"^traffic_source_digest: ([0-9a-f]+)$", text, re.M)
        if k and b and d and k.group(1).strip() == kernel and d.group(1) == want:
            return float(b.group(1)), os.path.basename(path)
    return None


def recorded_counters(kernel, profiles_dir):
    """Instruction-counter averages per launch of `kernel` ({counter: value})
    recorded in a summary under profiles_dir, or None when none was taken
    from the current kernel sources."""
    want = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(profiles_dir, "*.md"))):
        text = open(path).read()
        k = re.search(r"^counters_kernel: (.+)$", text, re.M)
        d = re.search(r"^counters_source_digest: ([0-9a-f]+)$", text, re.M)
        if not (k and d and k.group(1).strip() == kernel and d.group(1) == want):
            continue
        vals = {c: float(v) for c, v in
                re.findall(r"^counter_per_launch: (\S+) ([0-9.eE+-]+)$", text, re.M)}
        if vals:
            return vals, os.path.basename(path)
    return None


def kernel_stats(db):
    con = sqlite3.connect(db)
    # durations of the top_kernels view are in microseconds
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels order by total_duration desc").fetchall()
    con.close()
    return rows


def _dispatch_source(con):
    """(relation, name column, start column, end column) of the per-dispatch
    kernel records in a rocpd database."""
    rels = [r[0] for r in con.execute(
        "select name from sqlite_master where type in ('view', 'table')").fetchall()]
    order = sorted(rels, key=lambda r: (r != "kernels", "kernel" not in r.lower(), r))
    for rel in order:
        cols = [c[1] for c in con.execute(f"pragma table_info('{rel}')").fetchall()]
        start = next((c for c in ("start", "start_ns", "begin") if c in cols), None)
        end = next((c for c in ("end", "end_ns", "stop") if c in cols), None)
        name = next((c for c in ("name", "kernel_name") if c in cols), None)
        if start and end and name and "kernel" in rel.lower():
            return rel, name, start, end
    raise RuntimeError("no per-dispatch kernel relation among " + ", ".join(rels))


def last_dispatches(db, substring, n):
    """Durations (us) of the last n dispatches, by start time, of the kernel
    whose name contains substring, and the total number of its dispatches."""
    con = sqlite3.connect(db)
    rel, name, start, end = _dispatch_source(con)
    rows = con.execute(f'select "{start}", "{end}" from "{rel}" where "{name}" like ? '
                       f'order by "{start}"', ("%" + substring + "%",)).fetchall()
    con.close()
    return [(e - b) * 1e-3 for b, e in rows[-n:]], len(rows)


def counter_by_kernel(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, count(*), avg(value), sum(value) from counters_collection "
                       "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    con.close()
    return {r[0]: dict(dispatches=r[1], avg_kib=r[2], sum_kib=r[3]) for r in rows}


def last_counter_values(db, counter, substring, n):
    """Counter values (KiB) of the last n dispatches of the kernel whose name
    contains substring, in dispatch order, or None when the table has no
    ordering column."""
    con = sqlite3.connect(db)
    cols = [c[1] for c in con.execute("pragma table_info('counters_collection')").fetchall()]
    key = next((c for c in ("dispatch_id", "start", "correlation_id", "id") if c in cols), None)
    if key is None:
        con.close()
        return None
    # one value per dispatch (rows split by hardware dimension are summed)
    group = f'group by "{key}" ' if key in ("dispatch_id", "correlation_id") else ""
    rows = con.execute(f'select sum(value) from counters_collection where counter_name = ? and '
                       f'kernel_name like ? {group}order by "{key}"',
                       (counter, "%" + substring + "%")).fetchall()
    con.close()
    return [r[0] for r in rows[-n:]]


def counters_in(db):
    con = sqlite3.connect(db)
    rows = con.execute("select distinct counter_name from counters_collection").fetchall()
    con.close()
    return sorted(r[0] for r in rows)


def copy_reading(db, counter):
    """Counter KiB per dispatch of the runtime's buffer-copy kernel (largest)."""
    con = sqlite3.connect(db)
    rows = con.execute("select value from counters_collection where counter_name = ? and "
                       "kernel_name like '%copyBuffer%' order by value desc", (counter,)).fetchall()
    con.close()
    return rows[0][0] if rows else None


def short(name):
    name = name.replace("rdseg::(anonymous namespace)::", "")
    return name.split("(")[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--combine", nargs="+", metavar="PART.md")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", help="substring of the kernel name (default: the "
                    "benchmark's dominant kernel)")
    ap.add_argument("--copy-mib", type=float, default=0.0)
    ap.add_argument("--bench-json")
    ap.add_argument("--traced-json", help="benchmark output of the traced run itself")
    ap.add_argument("--fetch-json", help="benchmark output of the FETCH_SIZE run")
    ap.add_argument("--write-json", help="benchmark output of the WRITE_SIZE run")
    ap.add_argument("--sq", help="database of a `rocprofv3 --pmc` run of instruction "
                    "counters (SQ_*, GRBM_*): per-launch averages over the roofline pass")
    ap.add_argument("--sq-json", help="benchmark output of the --sq run")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args()

    if a.combine:
        combine(a.combine)
        return
    if a.sq:
        sq_report(a)
        return
    if not a.kernel:
        src = a.traced_json or a.bench_json or a.fetch_json or a.write_json
        if not src:
            ap.error("--kernel or a benchmark output is needed")
        lines = [l for l in open(src).read().splitlines() if l.strip().startswith("{")]
        a.kernel = json.loads(lines[-1])["roofline"]["kernel"].replace(",", ", ").rstrip(">")
    name = a.kernel
    if a.trace:
        rows = kernel_stats(a.trace)
        print("| kernel | calls | total us | avg us | % |")
        print("|---|---:|---:|---:|---:|")
        for name, calls, tot, avg, pct in rows[: a.top]:
            print(f"| `{short(name)}` | {calls} | {tot:.1f} | {avg:.3f} | {pct:.1f} |")
        sel = [r for r in rows if a.kernel in r[0]]
        if not sel:
            print(f"\nno kernel matches {a.kernel!r}")
            return
        name, calls, tot, avg, pct = sel[0]
        print(f"\nselected kernel `{short(name)}`: {calls} dispatches in the trace (tuning probes "
              f"included), average {avg:.3f} us")

    def bench_line(path):
        lines = [l for l in open(path).read().splitlines() if l.strip().startswith("{")]
        return json.loads(lines[-1])

    bench = None
    if a.traced_json and a.trace:
        r = bench_line(a.traced_json)["roofline"]
        durs, total = last_dispatches(a.trace, a.kernel, r["launches"])
        mean = sum(durs) / len(durs)
        print(f"\nthe benchmark's roofline pass = the last {len(durs)} of {total} dispatches: "
              f"rocprof average {mean:.3f} us; the same run's HIP-event average "
              f"{r['avg_launch_ms'] * 1e3:.3f} us (ratio {r['avg_launch_ms'] * 1e3 / mean:.4f})")
        flops = r["flops_per_update"] * r["updates_per_launch"]
        print(f"algorithmic FP32 operations per launch {flops:.4g} "
              f"({r['flops_per_update']} per active pixel-update x {r['updates_per_launch']:.6g}) -> "
              f"{flops / (mean * 1e-6) / 1e12:.2f} TFLOP/s at the rocprof average "
              f"({flops / (mean * 1e-6) / 1e12 / r['peak']:.4f} of the {r['peak']:.1f} TFLOP/s peak); "
              f"unblocked-equivalent bytes per launch {r['hbm']['alg_bytes_per_launch']:.4g}")
    if a.bench_json:
        bench = bench_line(a.bench_json)
        r = bench["roofline"]
        print(f"unprofiled benchmark (HIP events): average {r['avg_launch_ms'] * 1e3:.3f} us over "
              f"{r['launches']} launches, achieved {r['achieved']:.2f} {r['unit']} "
              f"({r['frac']:.4f} of peak)")
    total = 0.0
    n_counters = 0
    if a.fetch or a.write:
        src = a.fetch_json or a.write_json or a.bench_json
        kname = bench_line(src)["roofline"]["kernel"] if src else record_name(None, name)
        print(f"\ncombine_kernel: {kname}")
    runs = {"fetch": a.fetch_json, "write": a.write_json}
    for label, db, counter in [("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")]:
        if not db:
            continue
        per = counter_by_kernel(db, counter)
        k = [v for n, v in per.items() if a.kernel in n]
        cal = copy_reading(db, counter)
        factor = (a.copy_mib * 1024.0 / cal) if (cal and a.copy_mib) else 1.0
        print(f"\n{counter}: copy of {a.copy_mib:g} MiB reads {cal} KiB -> factor {factor:.4f}")
        if k:
            v = k[0]
            print(f"{counter} of the selected kernel: {v['dispatches']} dispatches, average "
                  f"{v['avg_kib']:.1f} KiB raw, {v['avg_kib'] * factor * 1024 / 1e6:.3f} MB calibrated per dispatch")
            kib = v["avg_kib"]
            n_last = 0
            if runs[label]:
                r = bench_line(runs[label])["roofline"]
                n_last = r["launches"] if r["kernel"].replace(",", ", ").rstrip(">") == a.kernel else 0
            if n_last:
                vals = last_counter_values(db, counter, a.kernel, n_last)
                if vals:
                    kib = sum(vals) / len(vals)
                    print(f"{counter} over the roofline pass (last {len(vals)} dispatches): "
                          f"average {kib:.1f} KiB raw, {kib * factor * 1024 / 1e6:.3f} MB calibrated")
            total += kib * factor * 1024
            n_counters += 1
            print(f"counter_bytes_per_launch: {counter} {kib * factor * 1024:.0f}")
    if n_counters == 2:
        print("\nmachine-readable record (read by bench.py for roofline.traffic):\n")
        print("```")
        print(f"traffic_kernel: {record_name(bench, name)}")
        print(f"traffic_bytes_per_launch: {total:.0f}")
        print(f"traffic_source_digest: {kernel_source_digest()}")
        print("```")


def sq_report(a):
    """Per-launch averages of every counter in an instruction-counter run, over
    the benchmark's roofline pass (the last `launches` dispatches of its
    dominant kernel), as a machine-readable record."""
    lines = [l for l in open(a.sq_json).read().splitlines() if l.strip().startswith("{")]
    r = json.loads(lines[-1])["roofline"]
    kname = r["kernel"]
    sub = a.kernel or kname.replace(",", ", ").rstrip(">")
    print(f"benchmark roofline pass: {r['launches']} launches of {kname}, HIP-event average "
          f"{r['avg_launch_ms'] * 1e3:.3f} us, {r['updates_per_launch']:.6g} active pixel-updates "
          f"per launch\n")
    print("| counter | per launch (average over the roofline pass) |")
    print("|---|---:|")
    out = {}
    for c in counters_in(a.sq):
        vals = last_counter_values(a.sq, c, sub, r["launches"])
        if not vals:
            continue
        out[c] = sum(vals) / len(vals)
        print(f"| {c} | {out[c]:.6g} |")
    print("\nmachine-readable record (read by bench.py for roofline.valu):\n")
    print("```")
    print(f"counters_kernel: {kname}")
    for c, v in out.items():
        print(f"counter_per_launch: {c} {v:.6g}")
    print(f"counters_source_digest: {kernel_source_digest()}")
    print("```")


def record_name(bench, name):
    """Kernel name as the benchmark's roofline reports it (no spaces)."""
    if bench:
        return bench["roofline"]["kernel"]
    return short(name).replace(" ", "").split(",false")[0].split(",true")[0].rstrip(">") + ">"


def combine(parts):
    """Traffic record from partial reports of separate counter runs of one
    kernel (each holding `counter_bytes_per_launch:` lines and a
    `combine_kernel:` line)."""
    got, kernels = {}, set()
    for path in parts:
        text = open(path).read()
        for c, v in re.findall(r"^counter_bytes_per_launch: (\S+) ([0-9.eE+]+)$", text, re.M):
            got[c] = float(v)
        kernels.update(k.strip() for k in re.findall(r"^combine_kernel: (.+)$", text, re.M))
    if set(got) != {"FETCH_SIZE", "WRITE_SIZE"} or len(kernels) != 1:
        raise SystemExit("need one FETCH_SIZE and one WRITE_SIZE report of the same kernel")
    print("machine-readable record (read by bench.py for roofline.traffic):\n")
    print("```")
    print(f"traffic_kernel: {kernels.pop()}")
    print(f"traffic_bytes_per_launch: {got['FETCH_SIZE'] + got['WRITE_SIZE']:.0f}")
    print(f"traffic_source_digest: {kernel_source_digest()}")
    print("```")


if __name__ == "__main__":
    main()
