"""A bootstrapping-shaped sequence of key-switching calls, run through the C
ABI eagerly or captured as one hipGraph.

The sequence follows the structure of CKKS bootstrapping's linear layers and
polynomial evaluation (Sec. 3: CoeffToSlot, EvalMod, SlotToCoeff):
  - CoeffToSlot: hoisted stages (Algorithm 4), each rotating the current
    ciphertext by `count` baby-step indices k = stride * (i + 1), multiplying
    every rotation by a plaintext diagonal (Algorithm 1 without Rescale),
    summing, then one Rescale; one level per stage;
  - EvalMod-like: per level, two Mult + relinearization + Rescale
    (Algorithm 2), x' = x y and y' = x x;
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


def bootstrap_plan(top: int, counts=(12, 12, 16), strides=(1, 32, 1024), evalmod_levels: int = 20) -> Plan:
    """Ops (kind, ...) over ciphertext buffers named by strings:
      ("hrotate", src, level, [k...], [dst...])
      ("ptmult", src, diag, level, dst)
      ("add", a, b, level, dst)
      ("rescale", src, level, dst)        -> level - 1
      ("mult", a, b, level, dst)          -> level - 1 (relinearized, rescaled)
    """
    p = Plan(top=top)
    level, x = top, "x0"
    p.buffers.add(x)
    nxt = iter(f"s{i}" for i in range(10 ** 6))

    def linear_stage(sign, stage_id):
        nonlocal level, x
        for si, (cnt, stride) in enumerate(zip(counts, strides)):
            ks = [sign * stride * (i + 1) for i in range(cnt)]
            rs = [f"r{i}" for i in range(cnt)]
            p.ops.append(("hrotate", x, level, ks, rs))
            p.key_switches += cnt
            for k in ks:
                if k not in p.rotations:
                    p.rotations.append(k)
            for i in range(cnt):
                d = f"{stage_id}{si}_{i}"
                p.diagonals.append(d)
                p.ops.append(("ptmult", rs[i], d, level, "acc" if i == 0 else "t"))
                if i:
                    p.ops.append(("add", "acc", "t", level, "acc"))
            y = next(nxt)
            p.ops.append(("rescale", "acc", level, y))
            p.buffers.update(rs + ["acc", "t", y])
            x, level = y, level - 1

    linear_stage(+1, "c")
    y = x
    for _ in range(evalmod_levels):
        a, b = next(nxt), next(nxt)
        p.ops.append(("mult", x, y, level, a))
        p.ops.append(("mult", x, x, level, b))
        p.key_switches += 2
        p.buffers.update([a, b])
        x, y, level = a, b, level - 1
    linear_stage(-1, "s")
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


def run_plan(ctx, plan: Plan, bufs: TraceBuffers, diag, keys, rlk, stream=None):
    """Issue every op of the plan on `stream` (default: torch's current
    stream, which is the capture stream under torch.cuda.graph).  diag maps
    a diagonal name to a [>= level][N] device tensor, keys maps a rotation
    index to its switching key, rlk is the relinearization key."""
    n = bufs.n
    for op in plan.ops:
        kind = op[0]
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
        else:
            raise ValueError(f"unknown op {kind}")
    return bufs.view(plan.out, plan.out_level)


def capture(ctx, plan: Plan, bufs: TraceBuffers, diag, keys, rlk) -> torch.cuda.CUDAGraph:
    """The whole plan as one hipGraph (replay with g.replay() on the current
    stream).  The library allocates nothing and sets no memory inside calls,
    so every node is a kernel launch."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run_plan(ctx, plan, bufs, diag, keys, rlk)
    return g
