"""HBM traffic per kernel launch from two rocprofv3 counter runs.

Input: the CSV directories of `rocprofv3 --pmc FETCH_SIZE` and
`rocprofv3 --pmc WRITE_SIZE` (KiB per dispatch, one counter per run) over
`bench.py --no-extras --batch 1 --calib-copy-mib 256` (the plain Rotate).
The largest plain device copy of each run calibrates the counters: its
WRITE_SIZE is its size, and FETCH_SIZE is scaled to the same size.  The
medians over the last `steps` Rotates (each `launches` library kernels)
give every launch's read and write MiB.  Printed last are the two lines the
committed counter summary of the key-switch kernel carries (the hash of the
kernel sources the counters were taken on, HBM bytes per launch), which
bench.py checks before it reports `traffic`:

    python -m paper_2112_06396_amd.traffic gpurun_out/pmcF gpurun_out/pmcW
"""
import argparse
import collections
import csv
import os
import statistics

LIBRARY_KERNELS = ("ntt_pass", "conv_kernel", "ksk_rows")


def load(directory: str, counter: str):
    """[(dispatch id, kernel name, grid size, value)] summed over the
    counter's instances, in dispatch order."""
    path = os.path.join(directory, "p_counter_collection.csv")
    agg = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]))
            agg[key] = agg.get(key, 0.0) + float(r["Counter_Value"])
    return [(d, k, g, v) for (d, k, g), v in sorted(agg.items())]


def per_launch(fetch, write, launches: int, steps: int):
    """Calibration factors and, per launch position of a step, (kernel, grid,
    median read MiB, median write MiB)."""
    cf = max(v for _, k, _, v in fetch if "copyBuffer" in k)
    cw = max(v for _, k, _, v in write if "copyBuffer" in k)
    sf, sw = cw / cf, 1.0
    lib_f = [x for x in fetch if x[1].startswith(LIBRARY_KERNELS)][-launches * steps:]
    lib_w = [x for x in write if x[1].startswith(LIBRARY_KERNELS)][-launches * steps:]
    if len(lib_f) != launches * steps or len(lib_w) != len(lib_f):
        raise ValueError("fewer library dispatches than launches * steps")
    rows = []
    for i in range(launches):
        rd = [lib_f[j][3] * sf / 1024 for j in range(i, len(lib_f), launches)]
        wr = [lib_w[j][3] * sw / 1024 for j in range(i, len(lib_w), launches)]
        rows.append((lib_f[i][1], lib_f[i][2], statistics.median(rd), statistics.median(wr)))
    return (cf, cw, sf, sw), rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--launches", type=int, default=9, help="library kernels per Rotate")
    ap.add_argument("--steps", type=int, default=10, help="Rotates to take the median over")
    ap.add_argument("--kernel", default="ksk_rows", help="the kernel whose bytes per launch are printed")
    args = ap.parse_args(argv)
    from .build import source_hash
    (cf, cw, sf, sw), rows = per_launch(load(args.fetch_dir, "FETCH_SIZE"), load(args.write_dir, "WRITE_SIZE"),
                                        args.launches, args.steps)
    print(f"calibration: the largest copy ({cw / 1024:.0f} MiB) reads FETCH_SIZE {cf:.0f} KiB (x{sf:.3f}) and "
          f"writes WRITE_SIZE {cw:.0f} KiB (x{sw:.3f})")
    dom = None
    for i, (k, g, r, w) in enumerate(rows):
        print(f"{i} {k[:60]:60s} grid {g:8d}  read {r:7.1f} MiB  write {w:6.1f} MiB")
        if k.startswith(args.kernel):
            dom = (r + w) * 2 ** 20
    if dom is not None:
        print(f"source_hash: {source_hash()}")
        print(f"hbm_bytes_per_launch: {dom:.0f}")


if __name__ == "__main__":
    main()
