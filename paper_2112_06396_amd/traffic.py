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

With --sq, the arguments are instead directories of `rocprofv3 --pmc` runs
of SQ counters over the same command, and the medians per launch position
of every counter they hold are printed, with the wait and activity
counters as fractions of SQ_WAVE_CYCLES:

    python -m paper_2112_06396_amd.traffic --sq gpurun_out/sq1 gpurun_out/sq2
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


def load_all(directory: str):
    """{dispatch id: (kernel name, grid size, {counter: value summed over
    its instances})} of a counter run."""
    path = os.path.join(directory, "p_counter_collection.csv")
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            if d not in out:
                out[d] = (r["Kernel_Name"], int(r["Grid_Size"]), collections.Counter())
            out[d][2][r["Counter_Name"]] += float(r["Counter_Value"])
    return out


def sq_summary(dirs, launches: int, steps: int):
    """Per launch position of a step: (kernel, grid, {counter: median over
    the last `steps` steps}), every counter of every run merged."""
    rows = [dict() for _ in range(launches)]
    names = [None] * launches
    for d in dirs:
        lib = [v for _, v in sorted(load_all(d).items()) if v[0].startswith(LIBRARY_KERNELS)]
        lib = lib[-launches * steps:]
        if len(lib) != launches * steps:
            raise ValueError(f"{d}: fewer library dispatches than launches * steps")
        for i in range(launches):
            sel = lib[i::launches]
            names[i] = (sel[0][0], sel[0][1])
            for c in sel[0][2]:
                rows[i][c] = statistics.median(x[2][c] for x in sel)
    return [(names[i][0], names[i][1], rows[i]) for i in range(launches)]


SQ_FRACTIONS = ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_ANY")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir", nargs="?")
    ap.add_argument("more", nargs="*", help="--sq: further counter directories")
    ap.add_argument("--sq", action="store_true", help="summarize SQ counter runs instead")
    ap.add_argument("--launches", type=int, default=9, help="library kernels per Rotate")
    ap.add_argument("--steps", type=int, default=10, help="Rotates to take the median over")
    ap.add_argument("--kernel", default="ksk_rows", help="the kernel whose bytes per launch are printed")
    args = ap.parse_args(argv)
    from .build import source_hash
    if args.sq:
        dirs = [args.fetch_dir] + ([args.write_dir] if args.write_dir else []) + list(args.more)
        print(f"source_hash: {source_hash()}")
        for i, (k, g, c) in enumerate(sq_summary(dirs, args.launches, args.steps)):
            print(f"{i} {k[:60]} grid {g}")
            print("    " + ", ".join(f"{n} {v:.0f}" for n, v in sorted(c.items())))
            wc = c.get("SQ_WAVE_CYCLES")
            if wc:
                print("    per SQ_WAVE_CYCLES: " + ", ".join(f"{n[3:]} {c[n] / wc:.3f}" for n in SQ_FRACTIONS if n in c))
        return
    if not args.write_dir:
        ap.error("the WRITE_SIZE run's directory is missing")
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
