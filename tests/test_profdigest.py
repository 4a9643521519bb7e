"""Host tests of the rocprofv3 summary tool: the counter calibration takes the copy dispatch."""
import csv
import json

from paper_2205_11935_amd import profdigest

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_copy_calibration_ignores_library_kernels(tmp_path):
    # a library kernel that reads far more than the 1 MiB copy must not be taken for it; the copy's
    # counters are split over two dimensions (summed per dispatch)
    fetch = [(1, "void ctl::k_mac_limb<6>(ctl::X)", 4096, "FETCH_SIZE", 9000.0),
             (2, "__amd_rocclr_copyBuffer", 1024, "FETCH_SIZE", 256.0),
             (2, "__amd_rocclr_copyBuffer", 1024, "FETCH_SIZE", 256.0),
             (3, "__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", 1.0)]
    write = [(1, "void ctl::k_mac_limb<6>(ctl::X)", 4096, "WRITE_SIZE", 5000.0),
             (2, "__amd_rocclr_copyBuffer", 1024, "WRITE_SIZE", 1024.0),
             (3, "__amd_rocclr_copyBuffer", 64, "WRITE_SIZE", 2.0)]
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    js, md = tmp_path / "t.json", tmp_path / "t.md"
    profdigest.main(["counters", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
                     "--copy-mib", "1", "--cmd-fetch", "a", "--cmd-write", "b",
                     "--site", "k_mac_limb<6> grid 4096", "k_mac @ layer 0 mac",
                     "--json", str(js), "--md", str(md)])
    rec = json.loads(js.read_text())
    cal = rec["copy_calibration"]
    assert cal["fetch_kernel"] == cal["write_kernel"] == "__amd_rocclr_copyBuffer"
    assert cal["fetch_scale"] == 2.0 and cal["write_scale"] == 1.0
    e = rec["instances"]["k_mac_limb<6> grid 4096"]
    assert e["fetch_bytes_per_launch"] == 9000.0 * 1024 * 2.0
    assert e["write_bytes_per_launch"] == 5000.0 * 1024
    assert rec["instances"]["k_mac @ layer 0 mac"] == e
