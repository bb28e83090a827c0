"""The rocprofv3 summariser behind the committed profile records, on small
hand-made CSV files: stage mapping, copy-probe scaling of the byte counters,
per-launch averages without the first launch, and the CNN application
split at the first CLAMP iteration kernel."""

import csv
import json

import pytest

from paper_2406_13651_amd import profsum


def _counter_csv(path, counter, rows):
    """rows: (dispatch id, kernel name, value)."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for d, k, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Grid_Size": 256, "Counter_Name": counter,
                        "Counter_Value": v})


def test_stage_names():
    assert profsum.stage_of("void clampk::k_row_upd_mann<256>(clampk::RowArgs, clampk::FuseArgs)") == \
        "row_update_mann"
    assert profsum.stage_of("void clampk::k_row_grad<256>(clampk::RowArgs)") == "row_grad"
    assert profsum.stage_of("void clampk::k_col_inv_compact<256>(clampk::ColArgs)") == "col_inv"
    assert profsum.stage_of("clampk::k_mace_final(double const*, int, double*)") == "mace_step"
    assert profsum.stage_of("__amd_rocclr_copyBuffer") is None


def test_traffic_scales_by_the_copy_probe_and_skips_first_launches(tmp_path):
    """A 1 MiB probe reads FETCH_SIZE 512 (KiB units of 2 KiB) and writes
    WRITE_SIZE 1024: bytes = FETCH_SIZE x 2048, WRITE_SIZE x 1024.  The
    update pass's first launch (a cold outlier) is left out of the mean."""
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    upd = "void clampk::k_row_upd_mann<256>(clampk::RowArgs, clampk::FuseArgs)"
    _counter_csv(fetch, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 512.0), (2, upd, 9999.0), (3, upd, 100.0),
                                       (4, upd, 300.0)])
    _counter_csv(write, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 1024.0), (2, upd, 1.0), (3, upd, 50.0),
                                       (4, upd, 70.0)])
    per, fk, wk = profsum.traffic(str(fetch), str(write), 1, skip_first=1)
    assert fk == pytest.approx(2.0) and wk == pytest.approx(1.0)
    assert per["row_update_mann"]["read_bytes"] == pytest.approx(200.0 * 2048)
    assert per["row_update_mann"]["write_bytes"] == pytest.approx(60.0 * 1024)


def test_cnn_application_bytes_from_the_evaluation_phase(tmp_path):
    """CNN kernels before the first CLAMP iteration kernel are training;
    after it, two applications (two output layers) of 10 + 30 + 20 fetched
    units each: one opening with the packed input, one with the first layer
    read from the fp32 volume."""
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    conv, fin = "void clampk::k_conv<32, 0>(clampk::ConvArgs)", "clampk::k_conv_final(clampk::ConvArgs)"
    rows = [(1, "__amd_rocclr_copyBuffer", 512.0), (2, conv, 777.0), (3, fin, 777.0),
            (4, "void clampk::k_row_grad<256>(clampk::RowArgs)", 5.0),
            (5, "clampk::k_pack(float const*, float const*, long, unsigned short*)", 10.0), (6, conv, 30.0),
            (7, fin, 20.0), (8, "clampk::k_conv_first(clampk::ConvArgs)", 10.0),
            (9, conv, 30.0), (10, fin, 20.0)]
    _counter_csv(fetch, "FETCH_SIZE", rows)
    _counter_csv(write, "WRITE_SIZE", [(d, k, 1024.0 if "copy" in k else v) for d, k, v in rows])
    r = profsum.cnn_traffic(str(fetch), str(write), 1)
    assert r["applications"] == 2
    assert r["read_bytes"] == pytest.approx(60.0 * 2048)
    assert r["write_bytes"] == pytest.approx(60.0 * 1024)


def test_traffic_record_is_written_with_the_source_hash(tmp_path):
    fetch, write, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "rec.json"
    upd = "void clampk::k_row_grad<256>(clampk::RowArgs)"
    _counter_csv(fetch, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 512.0), (2, upd, 1.0), (3, upd, 3.0)])
    _counter_csv(write, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 1024.0), (2, upd, 1.0), (3, upd, 2.0)])
    profsum.main(["traffic", "--fetch", str(fetch), "--write", str(write), "--probe-mib", "1", "--workload", "w",
                  "--out", str(out)])
    rec = json.load(open(out))["w"]
    assert rec["source_sha256"] == profsum.kernel_source_hash("fwd")
    assert rec["stages"]["row_grad"]["read_bytes"] == pytest.approx(3.0 * 2048)


def test_phase_table_splits_at_the_first_clamp_kernel_and_names_unet_kernels(tmp_path):
    """Kernel-duration table by phase: prior-agent kernels (the CNN's and the
    U-Net's) before the first CLAMP iteration kernel are training, after it
    evaluation; anonymous-namespace prefixes are dropped; rows by total time."""
    trace = tmp_path / "trace.csv"
    rows = [("void clampk::k_conv<32, 0, 2>(clampk::ConvArgs)", 0, 100),
            ("clampk::(anonymous namespace)::k_upconv(clampk::UpArgs)", 200, 250),
            ("void clampk::k_row_grad<256>(clampk::RowArgs)", 300, 310),
            ("void clampk::k_conv<32, 0, 2>(clampk::ConvArgs)", 400, 420),
            ("void clampk::k_conv<32, 0, 2>(clampk::ConvArgs)", 500, 540),
            ("clampk::(anonymous namespace)::k_upconv(clampk::UpArgs)", 600, 605)]
    with open(trace, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for k, t0, t1 in rows:
            w.writerow({"Kernel_Name": k, "Start_Timestamp": t0 * 1000, "End_Timestamp": t1 * 1000})
    table = profsum.phases_trace(str(trace)).splitlines()
    assert table[0] == "| kernel | phase | launches | avg us | total us |"
    body = table[2:]
    assert body[0] == "| `k_conv<32, 0, 2>` | training | 1 | 100.0 | 100 |"
    assert "| `k_upconv` | training | 1 | 50.0 | 50 |" in body
    assert "| `k_conv<32, 0, 2>` | evaluation | 2 | 30.0 | 60 |" in body
    assert "| `k_upconv` | evaluation | 1 | 5.0 | 5 |" in body
    assert not any("k_row_grad" in r for r in body)
