"""The counter post-processing (paper_2112_06396_amd.traffic) on synthetic
rocprofv3 CSVs: calibration by the largest copy and per-launch medians."""
import csv
import os

from paper_2112_06396_amd import traffic

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for did, name, grid, val in rows:
            # two counter instances per dispatch (summed by the loader)
            for part in (val / 2, val / 2):
                w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                            "Counter_Value": part})


def test_calibration_and_medians(tmp_path):
    names = ["ntt_pass_kernel<a>", "conv_kernel<b>", "ksk_rows_kernel<c>"]
    fetch, write = [], []
    did = 0
    # a 1 GiB copy: FETCH_SIZE counts half its bytes, WRITE_SIZE all of them
    fetch.append((did, "__amd_rocclr_copyBuffer", 1, 524288.0))
    write.append((did, "__amd_rocclr_copyBuffer", 1, 1048576.0))
    did += 1
    for step in range(12):
        for i, nm in enumerate(names):
            fetch.append((did, nm, 1000 + i, 1024.0 * (i + 1) + step))   # KiB, uncalibrated
            write.append((did, nm, 1000 + i, 2048.0 * (i + 1)))
            did += 1
    _write(str(tmp_path / "F"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "W"), "WRITE_SIZE", write)
    (cf, cw, sf, sw), rows = traffic.per_launch(traffic.load(str(tmp_path / "F"), "FETCH_SIZE"),
                                               traffic.load(str(tmp_path / "W"), "WRITE_SIZE"), 3, 10)
    assert (cf, cw, sf, sw) == (524288.0, 1048576.0, 2.0, 1.0)
    for i, (name, grid, rd, wr) in enumerate(rows):
        assert name == names[i] and grid == 1000 + i
        # steps 2..11 are the last ten; median of (1024 (i+1) + step) * 2 / 1024 MiB
        assert abs(rd - 2 * (1024.0 * (i + 1) + 6.5) / 1024) < 1e-9
        assert wr == 2.0 * (i + 1)
