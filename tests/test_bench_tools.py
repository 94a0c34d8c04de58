"""The bench's measurement helpers on small synthetic rocprofv3 outputs (CPU):
counter tables and records, last-N trace means, source hashes, model bytes."""
import csv
import os

import pytest

import bench


def _counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


@pytest.fixture
def pmc_dir(tmp_path):
    base = str(tmp_path)
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<double>>(int)"
    # a 1 GiB copy reads 2^20 KiB and writes 2^20 KiB; the counters read half / all of it
    _counters(f"{base}/copy_fetch", [(copy, "FETCH_SIZE", 524288)] * 3)
    _counters(f"{base}/copy_write", [(copy, "WRITE_SIZE", 1048576)] * 3)
    # two steps: kernel A twice per step, kernel B once; an input kernel once
    a, b, gen = "cf::k_a<double>(int)", "cf::k_b(int)", "cf::k_gen(int)"
    _counters(f"{base}/fetch", [(a, "FETCH_SIZE", 100)] * 4 + [(b, "FETCH_SIZE", 50)] * 2 + [(gen, "FETCH_SIZE", 7)])
    _counters(f"{base}/write", [(a, "WRITE_SIZE", 200)] * 4 + [(b, "WRITE_SIZE", 30)] * 2 + [(gen, "WRITE_SIZE", 9)])
    return base


def test_pmc_record_sums_a_path_per_unit(pmc_dir):
    rec = dict(l.split(": ", 1) for l in bench.pmc_record(pmc_dir, "step_fp64", "step550", 2, ["k_gen"]).splitlines())
    assert rec["kernel"] == "step_fp64" and rec["workload"] == "step550"
    assert float(rec["fetch_kib"]) == (4 * 100 + 2 * 50) / 2
    assert float(rec["write_kib"]) == (4 * 200 + 2 * 30) / 2
    assert float(rec["fetch_factor"]) == 2.0 and float(rec["write_factor"]) == 1.0
    assert rec["source_sha256"] == bench.kernel_source_hash("step_fp64")


def test_summarize_pmc_scales_by_the_copy(pmc_dir):
    txt = bench.summarize_pmc(pmc_dir)
    assert "factor 2.000" in txt and "factor 1.000" in txt
    row = [l for l in txt.splitlines() if "`cf::k_a<double>`" in l][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "100" and cells[2] == "200"
    assert float(cells[3]) == pytest.approx(100 * 2 * 1024 / 1e9, abs=1e-3)


def test_trace_last_takes_each_kernels_last_dispatches(tmp_path):
    path = tmp_path / "run_kernel_trace.csv"
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        # k_x: 10 us warm-up then 2 and 4 us; k_y: 3 us; a non-library kernel
        w.writerows([("cf::k_x(int)", 0, 10000), ("cf::k_x(int)", 20000, 22000), ("cf::k_x(int)", 30000, 34000),
                     ("cf::k_y(int)", 5000, 8000), ("at::native::copy(int)", 0, 99999)])
    txt = bench.summarize_trace_last(str(path), 2)
    rows = {l.split("|")[1].strip(): l for l in txt.splitlines() if l.startswith("| `")}
    assert "`at::native::copy`" not in rows
    assert rows["`cf::k_x`"].rstrip(" |").endswith("3.0")
    assert rows["`cf::k_y`"].rstrip(" |").endswith("3.0")
    assert "| 3 |" in rows["`cf::k_x`"]


def test_source_hash_follows_the_sources_and_flags():
    h = bench.kernel_source_hash("rk2_fused")
    assert h and len(h) == 64 and h == bench.kernel_source_hash("rk2_fused")
    assert bench.kernel_source_hash("poisson_mixed") != bench.kernel_source_hash("step_fp64")
    assert bench.kernel_source_hash("no_such_kernel") is None


def test_measured_traffic_needs_a_matching_record(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_x.txt").write_text("kernel: rk2_fused\nworkload: w\nsource_sha256: stale\n"
                                        "fetch_kib: 1\nwrite_kib: 1\nfetch_factor: 2\nwrite_factor: 1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("rk2_fused", "w") is None
    (prof / "traffic_x.txt").write_text(f"kernel: rk2_fused\nworkload: w\nsource_sha256: "
                                        f"{bench.kernel_source_hash('rk2_fused')}\n"
                                        "fetch_kib: 3\nwrite_kib: 5\nfetch_factor: 2\nwrite_factor: 1\n")
    assert bench.measured_traffic("rk2_fused", "w") == (3 * 2 + 5) * 1024


def test_model_bytes_of_the_mixed_solve():
    """The mixed solve with one refinement: 100 B per point, as the sum of its
    passes (FP32 spectra 4 B per point, FP64 right-hand side and result)."""
    x, zyz = 8 + 4, 3 * (4 + 4)
    first_out, resid, accum = 4 + 4, 4 + 8 + 4, 4 + 4 + 8
    assert bench.MODEL_BYTES_PER_POINT["poisson_mixed_refine1"] == x + zyz + first_out + resid + zyz + accum


def test_summarize_counters_means_per_kernel_and_counter(tmp_path):
    base = str(tmp_path)
    a, b = "void cf::k_a<double, 64>(int)", "void cf::k_b(int)"
    _counters(f"{base}/p1", [(a, "SQ_INSTS_VALU", 10), (a, "SQ_INSTS_VALU", 30), (b, "SQ_INSTS_VALU", 7)])
    _counters(f"{base}/p2", [(a, "GRBM_GUI_ACTIVE", 8), (a, "GRBM_GUI_ACTIVE", 16)])
    rows = [l for l in bench.summarize_counters(base, "k_a").splitlines() if l.startswith("| `")]
    assert rows == ["| `cf::k_a<double, 64>` | GRBM_GUI_ACTIVE | 2 | 12 |",
                    "| `cf::k_a<double, 64>` | SQ_INSTS_VALU | 2 | 20 |"]
