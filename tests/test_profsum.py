"""The rocprofv3 summaries behind the benchmark's traffic figure and the
matrix-core flop profile, on small hand-made counter files: per-dispatch
means, the copy-kernel scaling of FETCH_SIZE / WRITE_SIZE, the source-hash
guard of a stored traffic figure, and the 512-flop unit of the MFMA counters."""
import csv

from paper_2205_14741_amd import profsum

GEMM = "void sm::ns_gemm_kernel<4, 1, 2, true>(float*, long, int const*, sm::TileRec const*, double*)"
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>(int, float*)"


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Counter_Name", "Counter_Value"], r)))
    return str(path)


def test_counter_means_per_kernel(tmp_path):
    p = _csv(tmp_path / "c.csv", [(GEMM, "FETCH_SIZE", 10), (GEMM, "FETCH_SIZE", 30), (GEMM, "WRITE_SIZE", 7),
                                  (COPY, "FETCH_SIZE", 4)])
    m = profsum.counter_means(p, "FETCH_SIZE")
    assert m["sm::ns_gemm_kernel<4, 1, 2, true>"] == (2, 20.0)
    assert m["at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>"] == (1, 4.0)


def test_traffic_scaled_by_copy_kernel_and_hash_guard(tmp_path):
    # the copy kernel moves 1 MiB each way but FETCH reads half of it: the
    # fetch factor is 2, the write factor 1
    fe = _csv(tmp_path / "f.csv", [(COPY, "FETCH_SIZE", 512), (GEMM, "FETCH_SIZE", 100), (GEMM, "FETCH_SIZE", 300)])
    wr = _csv(tmp_path / "w.csv", [(COPY, "WRITE_SIZE", 1024), (GEMM, "WRITE_SIZE", 50)])
    text = profsum.traffic_summary(fe, wr, 2 ** 20, "cmd-f", "cmd-w")
    assert "copy_fetch_factor 2.0000" in text and "copy_write_factor 1.0000" in text
    out = tmp_path / "t.txt"
    out.write_text(text)
    want = 200 * 1024 * 2 + 50 * 1024
    assert profsum.read_traffic(str(out), "sm::ns_gemm_kernel<4, 1, 2, true>") == want
    # a summary taken for other GEMM sources is not used
    out.write_text(text.replace(profsum.gemm_source_hash(), "0000000000000000"))
    assert profsum.read_traffic(str(out), "sm::ns_gemm_kernel<4, 1, 2, true>") is None


def test_mfma_summary_units(tmp_path):
    p = _csv(tmp_path / "m.csv", [(GEMM, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 2), (GEMM, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 4),
                                  (GEMM, "SQ_INSTS_VALU_MFMA_MOPS_F64", 0), (COPY, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 0)])
    text = profsum.mfma_summary(p, "cmd")
    lines = [l for l in text.splitlines() if l.startswith("mfma ")]
    assert len(lines) == 1                       # the copy kernel issues none
    assert lines[0] == "mfma sm::ns_gemm_kernel<4, 1, 2, true> | 2 | 1536 | 0 | 0 | 0"


def test_tail_averages_the_last_dispatches(tmp_path):
    """A benchmark's timed launches come last: --tail averages only the last
    N dispatches, and a stored tail figure is the one the benchmark reads."""
    fe = _csv(tmp_path / "f.csv", [(COPY, "FETCH_SIZE", 512), (GEMM, "FETCH_SIZE", 100), (GEMM, "FETCH_SIZE", 300),
                                   (GEMM, "FETCH_SIZE", 500)])
    wr = _csv(tmp_path / "w.csv", [(COPY, "WRITE_SIZE", 1024), (GEMM, "WRITE_SIZE", 50), (GEMM, "WRITE_SIZE", 50),
                                   (GEMM, "WRITE_SIZE", 80)])
    name = "sm::ns_gemm_kernel<4, 1, 2, true>"
    text = profsum.traffic_summary(fe, wr, 2 ** 20, "cmd-f", "cmd-w", [(name, 2)])
    out = tmp_path / "t.txt"
    out.write_text(text)
    assert profsum.read_traffic(str(out), name) == 400 * 1024 * 2 + 65 * 1024
    trace = tmp_path / "trace.csv"
    with open(trace, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for t0, d in [(0, 1000), (5000, 3000), (9000, 5000)]:
            w.writerow([GEMM, t0, t0 + d])
    stats = tmp_path / "s.csv"
    with open(stats, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"])
        w.writerow([GEMM, 3, 3000, 9000, 100.0])
    text = profsum.stats_summary(str(stats), "cmd", trace=str(trace), tails=profsum.parse_tails([f"{name}=2"]))
    assert f"tail {name} | 2 | 4.00" in text
