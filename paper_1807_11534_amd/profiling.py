"""Summaries of rocprofv3 result databases (rocpd SQLite) for the profiles/ notes.

    python -m paper_1807_11534_amd.profiling --trace T.db [--fetch F.db --write W.db]
        [--kernel SUBSTRING] [--copy-mib N] [--bench-json B.json]

--trace    database of `rocprofv3 --kernel-trace --stats`
--fetch    database of `rocprofv3 --pmc FETCH_SIZE`   (KiB per dispatch)
--write    database of `rocprofv3 --pmc WRITE_SIZE`   (KiB per dispatch)
--copy-mib size of the plain buffer copy run first in the counter passes; the
           ratio (copy bytes) / (counter bytes of that copy) calibrates both
           counters.
Prints a short markdown report: per-kernel duration table, and for the kernel
matching --kernel its average duration, calibrated HBM bytes per launch and,
with --bench-json, the benchmark's live figures beside them.
"""
import argparse
import json
import sqlite3


def kernel_stats(db):
    con = sqlite3.connect(db)
    # durations of the top_kernels view are in microseconds
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels order by total_duration desc").fetchall()
    con.close()
    return rows


def counter_by_kernel(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, count(*), avg(value), sum(value) from counters_collection "
                       "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    con.close()
    return {r[0]: dict(dispatches=r[1], avg_kib=r[2], sum_kib=r[3]) for r in rows}


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
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", default="k_iterate<64, 64, 8, 1024")
    ap.add_argument("--copy-mib", type=float, default=0.0)
    ap.add_argument("--bench-json")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args()

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
    print(f"\nselected kernel `{short(name)}`: {calls} dispatches, average {avg:.3f} us")
    bench = None
    if a.bench_json:
        lines = [l for l in open(a.bench_json).read().splitlines() if l.strip().startswith("{")]
        bench = json.loads(lines[-1])
        r = bench["roofline"]
        print(f"benchmark (HIP events): average {r['avg_launch_ms'] * 1e3:.3f} us over "
              f"{r['launches']} launches, algorithmic bytes per launch {r['alg_bytes_per_launch']:.4g}, "
              f"achieved {r['achieved']:.1f} GB/s")
        print(f"algorithmic GB/s at the rocprof average: "
              f"{r['alg_bytes_per_launch'] / (avg * 1e-6) / 1e9:.1f}")
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


if __name__ == "__main__":
    main()
