"""Launch-plan tuner.

Times a workload (a callable that enqueues library calls on one stream)
under candidate launch plans (include/hks.h, ``hks_plan``) and keeps the
fastest.  No plan field changes a result, so the tuner only trades launch
shapes: the NTT's tile shapes (the split N = 2^n1 x 2^n2 between the column
and row passes, columns per column-pass block, rows per row-pass block),
elements per thread of each NTT pass class, the grouping of NewLimb's
target limbs, and the XCD-aware block order of batched launches.  Before a
plan is kept, the workload's outputs under it are compared word for word
with those under the starting plan.

The search is coordinate descent from the context's current plan: each field
in turn takes each of its candidate values with the others held; a value is
kept when it is faster than the incumbent by more than ``min_gain`` (timing
noise is about half a percent); passes repeat until one keeps nothing, at
most ``rounds`` times.

Results are cached as JSON, keyed by device architecture and workload shape
(``cache_key``), so that a context can start from the tuned plan without
timing anything (``apply_cached``).  The package's ``plans.json`` holds the
plans tuned on MI355X (gfx950) for the shapes the benchmark runs:

    python -m paper_2112_06396_amd.tune --workload rotate
    python -m paper_2112_06396_amd.tune --workload batch --size 16
    python -m paper_2112_06396_amd.tune --workload hrotate --size 64
    python -m paper_2112_06396_amd.tune --workload dft_trace --L 35 --K 12 --level 35
    (likewise trace, hoisted_trace)
"""
import argparse
import json
import os
import sys
import tempfile

ALWAYS8 = 0xFFFFFFFF
_E16 = (0, 2048, 4096, 6144, 12288, ALWAYS8)

# candidate values of each plan field (include/hks.h, hks_plan)
CANDIDATES = {
    "e16_fwd_cols": _E16,
    "e16_fwd_rows": _E16,
    "e16_inv_rows": _E16,
    "e16_inv_cols": _E16,
    "conv_group_limbs": (4, 8, 16, 64),
    "conv_group_max_batch": (0, 1, 2, 4, 16),
    "row_xcd_order": (0, 1),
    "ksk_xcd_order": (0, 1),
    "n1": (0,),  # the default split; candidates_for() adds the neighbouring ones
    "col_lines": (8, 16, 32),
    "row_lines": (4, 8, 16),
}


def candidates_for(log_n: int) -> dict:
    """CANDIDATES with the NTT splits valid at ring degree 2^log_n: the
    default (0 = log_n // 2) and one stage more or fewer in the column pass,
    within 5..9 stages per pass."""
    c = dict(CANDIDATES)
    h = log_n // 2
    c["n1"] = (0,) + tuple(v for v in (h - 1, h + 1) if 5 <= v <= 9 and 5 <= log_n - v <= 9)
    return c

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans.json")


def coordinate_descent(measure, start: dict, candidates=None, rounds: int = 2, min_gain: float = 0.01,
                       log=None, verbose: bool = False):
    """Minimise measure(plan) (seconds) over the candidate values, one field
    at a time, from `start`.  Returns (best plan, its time, the time of
    `start`, the list of (plan, time) measured)."""
    candidates = CANDIDATES if candidates is None else candidates
    best = dict(start)
    t_start = t_best = measure(best)
    trace = [(dict(best), t_best)]
    for _ in range(rounds):
        changed = False
        for field, values in candidates.items():
            for v in values:
                if v == best.get(field):
                    continue
                trial = dict(best)
                trial[field] = v
                t = measure(trial)
                trace.append((trial, t))
                if log and verbose:
                    log(f"[tune]   {field} = {v}: {t * 1e6:.1f} us (incumbent {t_best * 1e6:.1f})")
                if t < t_best * (1.0 - min_gain):
                    if log:
                        log(f"[tune] {field} {best.get(field)} -> {v}: {t_best * 1e6:.1f} -> {t * 1e6:.1f} us")
                    best, t_best, changed = trial, t, True
        if not changed:
            break
    return best, t_best, t_start, trace


def cache_key(arch: str, log_n: int, L: int, K: int, dnum: int, workload: str) -> str:
    """`workload` names the call and its shape, e.g. "rotate_l24",
    "batch16_l24", "hrotate64_l24"."""
    return f"{arch.split(':')[0]}/n{log_n}/L{L}/K{K}/d{dnum}/{workload}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_entry(key: str, entry: dict, path: str = DEFAULT_CACHE):
    """Adds or replaces one entry (atomic replace of the file)."""
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def apply_cached(ctx, key: str, path: str = DEFAULT_CACHE):
    """Sets the cached plan for `key` on the context; returns the entry, or
    None (plan unchanged) when the cache has none."""
    from . import hks
    entry = load_cache(path).get(key)
    if entry is None:
        return None
    hks.hks_set_plan(ctx, entry["plan"])
    return entry


def event_measure(ctx, run, stream, reps: int, trials: int = 3):
    """measure(plan) for coordinate_descent: sets the plan, runs the workload
    once untimed, then `trials` times `reps` calls bracketed by HIP events on
    `stream` (a torch stream, the one the workload launches on); returns the
    median seconds per call."""
    import torch
    from . import hks

    def measure(plan):
        hks.hks_set_plan(ctx, plan)
        run(0)
        torch.cuda.synchronize()
        times = []
        for tr in range(trials):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(reps):
                run(1 + tr * reps + i)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3 / reps)
        return sorted(times)[len(times) // 2]

    return measure


def tune(ctx, run, outputs, stream, reps: int, rounds: int = 2, min_gain: float = 0.01, log=None,
         verbose: bool = False):
    """Tunes the context's plan for `run`.  `outputs()` returns the tensors
    run(0) writes; the plan the search keeps must reproduce them exactly
    (else the starting plan stays).  Returns the entry for the cache."""
    import torch
    from . import hks
    start = hks.hks_get_plan(ctx)
    run(0)
    torch.cuda.synchronize()
    ref = [t.view(torch.int64).clone() for t in outputs()]
    best, t_best, t_start, trace = coordinate_descent(event_measure(ctx, run, stream, reps), start,
                                                      candidates=candidates_for(ctx.log_n), rounds=rounds,
                                                      min_gain=min_gain, log=log, verbose=verbose)
    hks.hks_set_plan(ctx, best)
    for o in outputs():
        o.view(torch.int64).zero_()
    run(0)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b.view(torch.int64)) for a, b in zip(ref, outputs()))
    if not same:
        hks.hks_set_plan(ctx, start)
        best, t_best = start, t_start
    return {"plan": best, "us": t_best * 1e6, "default_us": t_start * 1e6, "plans_timed": len(trace),
            "outputs_equal": same}


def _workload(args, hks, synth, ctx, key_mods, n, stream):
    """The benchmark's shapes: plain Rotate, a batch of `size` ciphertexts
    with distinct keys, HRotate over `size` rotations, and the
    bootstrapping-shaped traces; synthetic residues."""
    level = args.level
    gals = [hks.hks_galois_for_rotation(k + 1, args.log_n) for k in range(max(args.size, 1))]
    if args.workload == "rotate":
        pool = 4
        cts = [synth.device_residues(key_mods[:level], (2,), n, 7000 + i) for i in range(pool)]
        keys = [synth.device_residues(key_mods, (args.dnum, 2), n, 5000 + i) for i in range(pool)]
        outs = [hks.empty((2, level, n)) for _ in range(pool)]

        def run(i):
            j = i % pool
            hks.hks_rotate(ctx, cts[j], level, gals[0], keys[j], outs[j], stream)
        return run, (lambda: outs[:1]), 200, f"rotate_l{level}"
    if args.workload == "batch":
        b = args.size
        cts = [synth.device_residues(key_mods[:level], (2,), n, 7000 + i) for i in range(b)]
        keys = [synth.device_residues(key_mods, (args.dnum, 2), n, 5000 + i) for i in range(b)]
        outs = [hks.empty((2, level, n)) for _ in range(b)]

        def run(i):
            hks.hks_batch_rotate(ctx, cts, level, gals[:b], keys, outs, stream)
        return run, (lambda: outs), max(4, 200 // b), f"batch{b}_l{level}"
    if args.workload == "hrotate":
        r = args.size
        ct = synth.device_residues(key_mods[:level], (2,), n, 7000)
        keys = [synth.device_residues(key_mods, (args.dnum, 2), n, 5000 + i) for i in range(r)]
        outs = [hks.empty((2, level, n)) for _ in range(r)]

        def run(i):
            hks.hks_hrotate(ctx, ct, level, gals[:r], keys, outs, stream)
        return run, (lambda: outs), max(3, 100 // r), f"hrotate{r}_l{level}"
    if args.workload in ("trace", "hoisted_trace", "dft_trace"):
        # bootstrapping-shaped traces (trace.bootstrap_plan) run eagerly from
        # the top level: synthetic stages, the same with hoisted PtMatVecMult
        # stages and NewMult, or the factored DFT's own offsets
        from . import trace
        kw = {"trace": {}, "hoisted_trace": {"hoisted": True, "new_mult": True},
              "dft_trace": {"hoisted": True, "new_mult": True, "dft": (args.log_n - 1, 3)}}[args.workload]
        plan = trace.bootstrap_plan(level, **kw)
        bufs = trace.TraceBuffers(plan, n)
        bufs.view("x0", level).copy_(synth.device_residues(key_mods[:level], (2,), n, 11))
        keys = {k: synth.device_residues(key_mods, (args.dnum, 2), n, 2000 + i) for i, k in enumerate(plan.rotations)}
        rlk = synth.device_residues(key_mods, (args.dnum, 2), n, 1999)
        dmods = key_mods if kw else key_mods[:level]
        diag = {d: synth.device_residues(dmods, (), n, 100 + i) for i, d in enumerate(plan.diagonals)}
        ext = trace.ext_diagonals(plan, diag, args.L) if kw else None

        def run(i):
            trace.run_plan(ctx, plan, bufs, diag, keys, rlk, stream=stream, diag_ext=ext)
        outs = [bufs.ct[name] for name in sorted(plan.buffers) if name != "x0"]
        return run, (lambda: outs), 3, f"{args.workload}_l{level}"
    raise ValueError(args.workload)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=("rotate", "batch", "hrotate", "trace", "hoisted_trace", "dft_trace"),
                    default="rotate")
    ap.add_argument("--size", type=int, default=16, help="ciphertexts (batch) or rotations (hrotate)")
    ap.add_argument("--log-n", type=int, default=16)
    ap.add_argument("--L", type=int, default=24)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--dnum", type=int, default=3)
    ap.add_argument("--level", type=int, default=24)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--verbose", action="store_true", help="log the time of every plan timed")
    args = ap.parse_args(argv)
    import torch
    from . import hks, synth

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    pq = hks.hks_gen_primes(50, args.log_n + 1, args.L + args.K)
    ctx = hks.Context(args.log_n, pq[:args.L], pq[args.L:], args.dnum, max_batch=16)
    n = 1 << args.log_n
    stream = torch.cuda.current_stream()
    run, outputs, reps, wl = _workload(args, hks, synth, ctx, pq, n, stream)
    torch.cuda.synchronize()
    arch = torch.cuda.get_device_properties(0).gcnArchName
    key = cache_key(arch, args.log_n, args.L, args.K, args.dnum, wl)
    log(f"[tune] {key}: {reps} calls per timing")
    entry = tune(ctx, run, outputs, stream, reps, rounds=args.rounds, log=log, verbose=args.verbose)
    log(f"[tune] {key}: {entry['default_us']:.1f} us (start) -> {entry['us']:.1f} us, "
        f"{entry['plans_timed']} plans timed, outputs equal: {entry['outputs_equal']}")
    save_entry(key, entry, args.cache)
    print(json.dumps({"key": key, **entry}))
    torch.cuda.synchronize()
    ctx.close()


if __name__ == "__main__":
    main()
