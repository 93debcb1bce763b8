"""A bootstrapping-shaped sequence of key-switching calls, run through the C
ABI eagerly or captured as one hipGraph.

The sequence follows the structure of CKKS bootstrapping's linear layers and
polynomial evaluation (Sec. 3: CoeffToSlot, EvalMod, SlotToCoeff):
  - CoeffToSlot: hoisted stages (Algorithm 4), each rotating the current
    ciphertext by `count` baby-step indices k = stride * (i + 1), multiplying
    every rotation by a plaintext diagonal (Algorithm 1 without Rescale),
    summing, then one Rescale; one level per stage;
  - EvalMod-like: per level, two Mult + relinearization + Rescale
    (Algorithm 2), or two NewMult (Sec. 5.1), x' = x y and y' = x x,
    issued as one batched call (the level's two key-switches share every
    launch);
  - SlotToCoeff: the CoeffToSlot stages again with negated indices.
Levels fall by one per stage or EvalMod level, so the limb count is uneven
along the trace.  The plan is plain data; `run_plan` issues it through the
binding (every step runs in the library's kernels).
"""
from dataclasses import dataclass, field

import torch

from . import hks


@dataclass
class Plan:
    top: int                    # level of the input ciphertext "x0"
    ops: list = field(default_factory=list)
    rotations: list = field(default_factory=list)  # rotation indices needing keys
    diagonals: list = field(default_factory=list)  # plaintext names
    buffers: set = field(default_factory=set)
    key_switches: int = 0
    out: str = ""
    out_level: int = 0


def dft_offsets(log_slots: int, iters: int, inverse: bool) -> list:
    """Rotation offsets of the factored homomorphic DFT over n = 2^log_slots
    slots, per PtMatVecMult in application order (Sec. 3).  The DFT is a
    product of log_slots radix-2 stages whose butterflies pair slots m/2
    apart (m = 2, 4, ..., n; SlotToCoeff applies them upward, CoeffToSlot the
    inverses downward); `iters` groups of consecutive stages, balanced with
    the larger groups last, are multiplied out.  A group whose stages pair
    slots h_1, ..., h_r apart has non-zero diagonals exactly at the offsets
    sum_t e_t h_t mod n, e_t in {-1, 0, 1}; offset d is the rotation right by
    d, offset 0 the diagonal without rotation."""
    n = 1 << log_slots
    base, extra = divmod(log_slots, iters)
    sizes = [base] * (iters - extra) + [base + 1] * extra
    halves = [1 << s for s in range(log_slots)]  # m/2 for m = 2 .. n
    if inverse:
        halves = halves[::-1]
    out, pos = [], 0
    for r in sizes:
        offs = {0}
        for h in halves[pos:pos + r]:
            offs = {(o + e * h) % n for o in offs for e in (-1, 0, 1)}
        out.append(sorted(offs))
        pos += r
    return out


def bootstrap_plan(top: int, counts=(12, 12, 16), strides=(1, 32, 1024), evalmod_levels: int = 20,
                   hoisted: bool = False, new_mult: bool = False, dft=None) -> Plan:
    """Ops (kind, ...) over ciphertext buffers named by strings:
      ("hrotate", src, level, [k...], [dst...])
      ("ptmult", src, diag, level, dst)
      ("add", a, b, level, dst)
      ("ptmatvec", src, level, [k...], [diag...], dst)   sum_i M_i Rotate_k_i(src), one ModDown
      ("rescale", src, level, dst)        -> level - 1
      ("mult", a, b, level, dst)          -> level - 1 (relinearized, rescaled)
      ("newmult", a, b, level, dst)       -> level - 1 (Sec. 5.1, one ModDown by P q_(level-1))
      ("mults", [(a, b, dst), ...], level)    the products of one level in one batched call
      ("newmults", [(a, b, dst), ...], level)
    With `hoisted`, each linear stage is one ptmatvec (Sec. 5.2) instead of
    an HRotate followed by PtMult and Add per rotation; with `new_mult`, the
    EvalMod products are NewMult instead of Mult + Rescale.  With
    dft = (log_slots, iters), the linear stages have the factored DFT's
    rotation offsets (dft_offsets: CoeffToSlot, then SlotToCoeff) instead of
    `counts` x `strides`; offset 0 is a diagonal without rotation (a PtMult
    of the input, no key)."""
    p = Plan(top=top)
    level, x = top, "x0"
    p.buffers.add(x)
    nxt = iter(f"s{i}" for i in range(10 ** 6))

    if dft is not None:
        groups_c = dft_offsets(dft[0], dft[1], True)
        groups_s = dft_offsets(dft[0], dft[1], False)
    else:
        groups_c = [[stride * (i + 1) for i in range(cnt)] for cnt, stride in zip(counts, strides)]
        groups_s = [[-k for k in ks] for ks in groups_c]

    def linear_stage(groups, stage_id):
        nonlocal level, x
        for si, ks in enumerate(groups):
            cnt = len(ks)
            rot = [k for k in ks if k != 0]
            rs = {k: f"r{i}" for i, k in enumerate(rot)}
            ds = [f"{stage_id}{si}_{i}" for i in range(cnt)]
            p.diagonals.extend(ds)
            p.key_switches += len(rot)
            for k in rot:
                if k not in p.rotations:
                    p.rotations.append(k)
            if hoisted:
                p.ops.append(("ptmatvec", x, level, list(ks), ds, "acc"))
            else:
                if rot:
                    p.ops.append(("hrotate", x, level, rot, [rs[k] for k in rot]))
                for i, k in enumerate(ks):
                    p.ops.append(("ptmult", rs[k] if k else x, ds[i], level, "acc" if i == 0 else "t"))
                    if i:
                        p.ops.append(("add", "acc", "t", level, "acc"))
                p.buffers.update(list(rs.values()) + ["t"])
            y = next(nxt)
            p.ops.append(("rescale", "acc", level, y))
            p.buffers.update(["acc", y])
            x, level = y, level - 1

    linear_stage(groups_c, "c")
    y = x
    for _ in range(evalmod_levels):
        a, b = next(nxt), next(nxt)
        p.ops.append(("newmults" if new_mult else "mults", [(x, y, a), (x, x, b)], level))
        p.key_switches += 2
        p.buffers.update([a, b])
        x, y, level = a, b, level - 1
    linear_stage(groups_s, "s")
    p.out, p.out_level = x, level
    return p


class TraceBuffers:
    """Device buffers of a plan: one flat [2 * top * N] tensor per
    ciphertext name, viewed as [2][level][N] at the level an op uses."""

    def __init__(self, plan: Plan, n: int, device="cuda"):
        self.n = n
        self.top = plan.top
        self.ct = {name: hks.empty((2 * plan.top * n,), device) for name in sorted(plan.buffers)}

    def view(self, name, level):
        return self.ct[name][: 2 * level * self.n].view(2, level, self.n)


def ext_diagonals(plan: Plan, diag, L: int) -> dict:
    """For the ptmatvec ops: (diagonal, level) -> the diagonal over
    Q_level U P, [level + K][N] contiguous, from diag[name] given over all
    L + K primes (q_0..q_{L-1}, p_0..p_{K-1})."""
    import torch
    out = {}
    for op in plan.ops:
        if op[0] == "ptmatvec":
            _, _, level, _, ds, _ = op
            for d in ds:
                t = diag[d]
                out[(d, level)] = torch.cat([t[:level], t[L:]]).contiguous()
    return out


def run_plan(ctx, plan: Plan, bufs: TraceBuffers, diag, keys, rlk, stream=None, diag_ext=None):
    """Issue every op of the plan on `stream` (default: torch's current
    stream, which is the capture stream under torch.cuda.graph).  diag maps
    a diagonal name to a [>= level][N] device tensor (over all L + K primes
    for a hoisted plan, with diag_ext from ext_diagonals), keys maps a
    rotation index to its switching key, rlk is the relinearization key."""
    n = bufs.n
    for op in plan.ops:
        kind = op[0]
        if kind == "ptmatvec":
            _, src, level, ks, ds, dst = op
            gals = [hks.hks_galois_for_rotation(k, ctx.log_n) if k else 1 for k in ks]
            hks.hks_ptmatvec(ctx, bufs.view(src, level), level, gals, [keys[k] if k else None for k in ks],
                             [diag_ext[(d, level)] for d in ds], bufs.view(dst, level), stream)
            continue
        if kind == "hrotate":
            _, src, level, ks, dsts = op
            gals = [hks.hks_galois_for_rotation(k, ctx.log_n) for k in ks]
            hks.hks_hrotate(ctx, bufs.view(src, level), level, gals, [keys[k] for k in ks],
                            [bufs.view(d, level) for d in dsts], stream)
        elif kind == "ptmult":
            _, src, d, level, dst = op
            hks.hks_ptmult(ctx, bufs.view(src, level), diag[d][:level], level, False, bufs.view(dst, level), stream)
        elif kind == "add":
            _, a, b, level, dst = op
            hks.hks_add(ctx, bufs.view(a, level), bufs.view(b, level), level, 2, bufs.view(dst, level), stream)
        elif kind == "rescale":
            _, src, level, dst = op
            hks.hks_rescale(ctx, bufs.view(src, level), level, bufs.view(dst, level - 1), stream)
        elif kind == "mult":
            _, a, b, level, dst = op
            hks.hks_mult_relin(ctx, bufs.view(a, level), bufs.view(b, level), level, rlk, True,
                               bufs.view(dst, level - 1), stream)
        elif kind == "newmult":
            _, a, b, level, dst = op
            hks.hks_new_mult(ctx, bufs.view(a, level), bufs.view(b, level), level, rlk, bufs.view(dst, level - 1),
                             stream)
        elif kind in ("mults", "newmults"):
            _, prods, level = op
            c1 = [bufs.view(a, level) for a, _, _ in prods]
            c2 = [bufs.view(b, level) for _, b, _ in prods]
            outs = [bufs.view(d, level - 1) for _, _, d in prods]
            if kind == "mults":
                hks.hks_batch_mult_relin(ctx, c1, c2, level, [rlk] * len(prods), True, outs, stream)
            else:
                hks.hks_batch_new_mult(ctx, c1, c2, level, [rlk] * len(prods), outs, stream)
        else:
            raise ValueError(f"unknown op {kind}")
    return bufs.view(plan.out, plan.out_level)


def capture(ctx, plan: Plan, bufs: TraceBuffers, diag, keys, rlk, diag_ext=None) -> torch.cuda.CUDAGraph:
    """The whole plan as one hipGraph (replay with g.replay() on the current
    stream).  The library allocates nothing and sets no memory inside calls,
    so every node is a kernel launch."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run_plan(ctx, plan, bufs, diag, keys, rlk, diag_ext=diag_ext)
    return g
