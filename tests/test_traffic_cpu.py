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


def test_sq_summary_merges_runs_per_launch(tmp_path):
    """Two SQ counter runs over the same steps: per launch position, the
    median of each counter over the last `steps` steps, both runs merged."""
    names = ["ntt_pass_kernel<a>", "ksk_rows_kernel<c>"]
    runs = {"S1": ("SQ_WAVE_CYCLES", lambda i, st: 1000.0 * (i + 1) + st),
            "S2": ("SQ_WAIT_ANY", lambda i, st: 100.0 * (i + 1) + 2 * st)}
    for d, (counter, val) in runs.items():
        rows = [(0, "__amd_rocclr_copyBuffer", 1, 5.0)]
        did = 1
        for st in range(12):
            for i, nm in enumerate(names):
                rows.append((did, nm, 64 + i, val(i, st)))
                did += 1
        _write(str(tmp_path / d), counter, rows)
    out = traffic.sq_summary([str(tmp_path / "S1"), str(tmp_path / "S2")], 2, 10)
    for i, (name, grid, c) in enumerate(out):
        assert name == names[i] and grid == 64 + i
        # the last ten steps are 2..11: median step 6.5
        assert c["SQ_WAVE_CYCLES"] == 1000.0 * (i + 1) + 6.5
        assert c["SQ_WAIT_ANY"] == 100.0 * (i + 1) + 13.0
