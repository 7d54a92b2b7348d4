"""Host logic of the rocprofv3 summariser: kernel labels, benchmark keys and
the HBM-traffic calibration, on small synthetic counter files."""
import csv
import json
import os

from paper_2505_12425_amd import profsum

TILED_W = "void kr::k_tiled<1, 3, true, 1, 64, 1, 16, 3, true>(kr::TiledJob, kr::Epilogue, kr::TileGeom)"
TILED_P = "void kr::k_tiled<2, 3, false, 4, 16, 1, 4, 3, false>(kr::TiledJob, kr::Epilogue, kr::TileGeom)"
BATCH_A = "void kr::k_batch<1, 3, false, 4, 16, 1, 2, 3>(kr::TiledJob const*, int, int)"
BATCH_B = "void kr::k_batch<1, 3, false, 4, 8, 1, 1, 3>(kr::TiledJob const*, int, int)"
NEAR = "void kr::(anonymous namespace)::k_nearest<3, false, true>(kr::NearestJob, kr::Epilogue)"
GRAY = "void kr::(anonymous namespace)::k_gray<false, false>(void const*, void*, int)"
COPY = "kr::k_copy(unsigned int __vector(4)*, unsigned int __vector(4) const*, unsigned long)"
HALF = "void kr::(anonymous namespace)::k_half<3, true>(kr::ImageJob, kr::Epilogue)"


def test_labels_and_keys():
    assert profsum.label(TILED_W) == "warp_f32 c3 1x64x1x16"
    assert profsum.label(TILED_P) == "perspective_u8 c3 4x16x1x4"
    assert profsum.label(BATCH_A) == "batch_warp_u8 c3 4x16x1x2"
    assert profsum.label(COPY) == "copy"
    assert profsum.label("kr::k_stream(unsigned int __vector(4)*, unsigned int __vector(4) const*, unsigned long, "
                         "int, int)") == "stream probe"
    assert profsum.label(NEAR) == "nearest<3, false, true>"
    assert profsum.bench_key(TILED_W) == "warp_f32"
    assert profsum.bench_key(TILED_P) == "perspective_u8"
    assert profsum.bench_key(BATCH_B) == "batch_warp_u8"
    assert profsum.bench_key(GRAY) == "gray_u8"
    assert profsum.bench_key(NEAR) == "nearest_{}_f32"
    assert profsum.bench_key(HALF) == "resize_f32" and profsum.label(HALF) == "resize_f32 c3 half"
    tiled_r = "void kr::k_tiled<0, 3, false, 4, 16, 1, 1, 3, false>(kr::TiledJob, kr::Epilogue, kr::TileGeom)"
    assert profsum.bench_key(tiled_r) == "resize_tiled_u8" and profsum.label(tiled_r) == "resize_u8 c3 4x16x1x1"
    assert profsum.bench_key("void kr::k_batch<0, 3, true, 1, 64, 1, 4, 3, false>(x)") == "batch_resize_f32"
    f32src = "void kr::k_tiled<1, 5, true, 4, 16, 1, 2, 3, false>(kr::TiledJob, kr::Epilogue, kr::TileGeom)"
    assert profsum.label(f32src) == "warp_f32 c1 f32-source 4x16x1x2" and profsum.bench_key(f32src) is None
    assert profsum.bench_key(TILED_W.replace("<1, 3,", "<1, 4,")) is None  # only 3-channel kernels are benchmarked


def _write(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "r_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for name, grid, val in rows:
            w.writerow([name, grid, counter, val])


def test_traffic_calibration_and_grouping(tmp_path):
    gib = 1 << 30
    # FETCH_SIZE reads half the bytes on the copy, WRITE_SIZE all of them;
    # a 100 MiB copy on the same grid must not enter the calibration
    fetch = [(COPY, 524288, gib / 2048), (COPY, 524288, gib / 2048), (COPY, 524288, 100 * 2 ** 20 / 2048),
             (BATCH_A, 1000, 300.0), (BATCH_B, 500, 100.0),
             (NEAR, 1000, 10.0), (NEAR, 4000, 20.0), (GRAY, 64, 7.0)]
    write = [(COPY, 524288, gib / 1024), (COPY, 524288, gib / 1024), (COPY, 524288, 100 * 2 ** 20 / 1024),
             (BATCH_A, 1000, 400.0), (BATCH_B, 500, 50.0),
             (NEAR, 1000, 30.0), (NEAR, 4000, 120.0), (GRAY, 64, 8.0)]
    _write(tmp_path / "f", "FETCH_SIZE", fetch)
    _write(tmp_path / "w", "WRITE_SIZE", write)
    out = tmp_path / "t.json"
    profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), gib, str(out), str(tmp_path / "t.md"), "cf", "cw")
    k = json.load(open(out))["kernels"]
    assert k["batch_warp_u8"]["fetch_bytes"] == 2 * 400 * 1024  # both groups of the batch, factor 2
    assert k["batch_warp_u8"]["write_bytes"] == 450 * 1024
    assert k["nearest_down_f32"]["bytes_per_launch"] == (2 * 10 + 30) * 1024  # smaller grid
    assert k["nearest_up_f32"]["bytes_per_launch"] == (2 * 20 + 120) * 1024
    assert k["gray_u8"]["bytes_per_launch"] == (2 * 7 + 8) * 1024
    assert k["gray_u8"]["calibration"]["fetch_factor"] == 2.0


def test_overlap_counts_concurrent_dispatches_of_other_queues(tmp_path):
    import csv
    rows = [("0", 100, 200, "kr::k_batch<1, 3, false, 4, 16, 1, 2, 3, false>(x)"),
            ("1", 150, 260, "kr::k_batch<1, 3, false, 4, 16, 1, 2, 3, false>(x)"),
            ("0", 300, 400, "kr::k_copy(x)"),          # alone
            ("0", 500, 600, "kr::k_copy(x)"),
            ("2", 550, 580, "kr::k_copy(x)"),
            ("2", 590, 595, "kr::k_copy(x)")]          # same queue as the one before: still overlaps queue 0
    with open(tmp_path / "r_kernel_trace.csv", "w") as f:
        w = csv.writer(f)
        w.writerow(["Queue_Id", "Start_Timestamp", "End_Timestamp", "Kernel_Name"])
        w.writerows(rows)
    r = profsum.overlap(str(tmp_path), str(tmp_path / "o.md"), "cmd")
    assert r["dispatches"] == 6 and r["queues"] == 3
    assert r["overlapping_another_queue"] == 5
    assert r["peak_concurrency"] == 2
    assert abs(r["mean_concurrency"] - 445 / 360) < 1e-3
    assert profsum.label(rows[0][3]) == "batch_warp_u8 c3 4x16x1x2"


def test_overlap_segments_split_at_idle_gaps(tmp_path):
    import csv
    rows = [("0", 100, 200, "kr::k_copy(x)"), ("1", 150, 260, "kr::k_copy(x)"), ("0", 300, 400, "kr::k_copy(x)"),
            ("0", 500, 600, "kr::k_copy(x)"), ("2", 550, 580, "kr::k_copy(x)"), ("2", 590, 595, "kr::k_copy(x)")]
    with open(tmp_path / "r_kernel_trace.csv", "w") as f:
        w = csv.writer(f)
        w.writerow(["Queue_Id", "Start_Timestamp", "End_Timestamp", "Kernel_Name"])
        w.writerows(rows)
    # 100 ns: the 100 ns gap before the fourth dispatch splits, the 40 ns gap does not
    r = profsum.overlap(str(tmp_path), str(tmp_path / "o.md"), "cmd", gap_ms=1e-4)
    a, b = r["segments"]
    assert (a["dispatches"], a["queues"], a["overlapping_another_queue"]) == (3, 2, 2)
    assert (b["dispatches"], b["queues"], b["overlapping_another_queue"]) == (3, 2, 3)
    assert "| 1 | 3 | 2 | 3 |" in (tmp_path / "o.md").read_text()
    assert len(profsum.overlap(str(tmp_path), str(tmp_path / "o.md"), "cmd")["segments"]) == 1


def test_counters_per_pixel_and_wave_states(tmp_path):
    rows = []
    for c, v in (("SQ_INSTS_VALU", 1000.0), ("SQ_INSTS_SALU", 500.0), ("SQ_INSTS_LDS", 40.0),
                 ("SQ_LDS_BANK_CONFLICT", 80.0), ("SQ_WAVES", 16.0)):
        rows += [(TILED_W, 4096, c, v), (TILED_W, 4096, c, v * 3)]  # two dispatches: mean = 2 v
    path = tmp_path / "c"
    os.makedirs(path)
    with open(path / "r_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writerows(rows)
    r = profsum.counters(str(path), str(tmp_path / "c.md"), "cmd", {"warp_f32": 64 * 10})
    assert r["warp_f32"]["SQ_INSTS_VALU"] == 2000.0 and r["warp_f32"]["dispatches"] == 2
    text = (tmp_path / "c.md").read_text()
    assert "| 32 | 200.0 | 100.0 | 8.00 | 2.00 |" in text  # 2000 x 64 / 640 VALU per pixel
    rows = [(TILED_W, 4096, "SQ_WAVE_CYCLES", 100.0), (TILED_W, 4096, "SQ_WAIT_ANY", 40.0),
            (TILED_W, 4096, "SQ_WAIT_INST_ANY", 30.0), (TILED_W, 4096, "SQ_ACTIVE_INST_ANY", 30.0),
            (TILED_W, 4096, "SQ_ACTIVE_INST_VALU", 20.0)]
    with open(path / "r_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writerows(rows)
    profsum.counters(str(path), str(tmp_path / "s.md"), "cmd", {"warp_f32": 640})
    assert "| 0.40 | 0.30 | 0.30 | 0.20 | 0.00 | 0.00 |" in (tmp_path / "s.md").read_text()
