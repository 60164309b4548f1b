"""Host logic of the measurement tooling: the HBM-traffic record that the
benchmark attaches to its roofline is taken only from a summary written for
the current kernel sources, and the two counter runs combine by summing."""
import os
import subprocess
import sys

from paper_1807_11534_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL = "k_resident<64,64,8,1024>"


def _record(kernel, nbytes, digest):
    return (f"# summary\n\n```\ntraffic_kernel: {kernel}\ntraffic_bytes_per_launch: {nbytes}\n"
            f"traffic_source_digest: {digest}\n```\n")


def test_record_needs_matching_kernel_and_sources(tmp_path):
    cur = profiling.kernel_source_digest()
    assert len(cur) == 16
    (tmp_path / "a_stale.md").write_text(_record(KERNEL, 111, "0" * 16))
    assert profiling.recorded_traffic(KERNEL, str(tmp_path)) is None
    (tmp_path / "b_other_kernel.md").write_text(_record("k_iterate<8,8,32,512>", 222, cur))
    assert profiling.recorded_traffic(KERNEL, str(tmp_path)) is None
    (tmp_path / "c_current.md").write_text(_record(KERNEL, 333, cur))
    assert profiling.recorded_traffic(KERNEL, str(tmp_path)) == (333.0, "c_current.md")


def test_combine_sums_fetch_and_write(tmp_path):
    fetch = tmp_path / "fetch.md"
    write = tmp_path / "write.md"
    fetch.write_text(f"combine_kernel: {KERNEL}\ncounter_bytes_per_launch: FETCH_SIZE 700\n")
    write.write_text(f"combine_kernel: {KERNEL}\ncounter_bytes_per_launch: WRITE_SIZE 300\n")
    out = subprocess.run([sys.executable, "-m", "paper_1807_11534_amd.profiling", "--combine",
                          str(fetch), str(write)], capture_output=True, text=True, cwd=ROOT,
                         check=True).stdout
    (tmp_path / "rec.md").write_text(out)
    assert profiling.recorded_traffic(KERNEL, str(tmp_path)) == (1000.0, "rec.md")


def test_counter_record_needs_matching_kernel_and_sources(tmp_path):
    cur = profiling.kernel_source_digest()

    def rec(kernel, digest, vals):
        body = "".join(f"counter_per_launch: {c} {v}\n" for c, v in vals.items())
        return f"```\ncounters_kernel: {kernel}\n{body}counters_source_digest: {digest}\n```\n"

    (tmp_path / "a_stale.md").write_text(rec(KERNEL, "0" * 16, {"SQ_INSTS_VALU": 5}))
    assert profiling.recorded_counters(KERNEL, str(tmp_path)) is None
    (tmp_path / "b_other.md").write_text(rec("k_iterate<8,8,32,512>", cur, {"SQ_INSTS_VALU": 6}))
    assert profiling.recorded_counters(KERNEL, str(tmp_path)) is None
    (tmp_path / "c_cur.md").write_text(rec(KERNEL, cur, {"SQ_INSTS_VALU": 7.5e8,
                                                         "SQ_INSTS_LDS": 2e8}))
    assert profiling.recorded_counters(KERNEL, str(tmp_path)) == (
        {"SQ_INSTS_VALU": 7.5e8, "SQ_INSTS_LDS": 2e8}, "c_cur.md")
