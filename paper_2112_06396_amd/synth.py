"""Seeded synthetic inputs (numpy PCG64).

This module only draws random numbers; it holds none of the key-switching
arithmetic.  Both the HIP path's tests/benchmark and the CPU oracle take their
inputs from here, so the two sides see identical bits.

Seed rule: workload ``c`` uses base seed ``0x4B530000 + c``; an object of kind
``k`` and index ``i`` uses ``base + 1000*k + i``.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 0x4B530000

# object kinds for seed derivation
KIND_CT = 0      # ciphertext residues
KIND_KEY = 1     # switching-key residues (uniform rows / uniform synthetic keys)
KIND_SECRET = 2  # ternary secret
KIND_ERROR = 3   # error polynomials
KIND_MSG = 4     # message polynomials
KIND_PT = 5      # plaintext residues


def seed_for(workload: int, kind: int, index: int = 0) -> int:
    return BASE_SEED + workload + 1000 * kind + index


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_residues(g: np.random.Generator, mods, n: int) -> np.ndarray:
    """[len(mods)][n] uint64, row i uniform in [0, mods[i])."""
    mods = [int(m) for m in mods]
    out = np.empty((len(mods), n), dtype=np.uint64)
    for i, m in enumerate(mods):
        out[i] = g.integers(0, m, size=n, dtype=np.uint64)
    return out


def ternary(g: np.random.Generator, n: int) -> np.ndarray:
    """n coefficients uniform in {-1, 0, 1} (int64)."""
    return g.integers(-1, 2, size=n, dtype=np.int64)


def cbd(g: np.random.Generator, n: int, eta: int = 21) -> np.ndarray:
    """Centered binomial samples: sum of eta coin flips minus sum of eta coin flips."""
    a = g.integers(0, 2, size=(n, eta), dtype=np.int8).sum(axis=1, dtype=np.int64)
    b = g.integers(0, 2, size=(n, eta), dtype=np.int8).sum(axis=1, dtype=np.int64)
    return a - b


def small_uniform(g: np.random.Generator, n: int, bound: int) -> np.ndarray:
    """n coefficients uniform in [-bound, bound) (int64)."""
    return g.integers(-bound, bound, size=n, dtype=np.int64)


def device_residues(mods, lead_shape, n: int, seed: int, device="cuda"):
    """[*lead_shape][len(mods)][n] residues drawn on the GPU (torch's seeded
    generator): for benchmark-scale keys and ciphertexts whose values only
    need to be valid residues of the right moduli.  Values are 62-bit
    uniform words reduced mod q (relative bias below 2^-12)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    qs = torch.tensor([int(m) for m in mods], dtype=torch.int64, device=device).view(-1, 1)
    x = torch.randint(0, 1 << 62, (*lead_shape, len(mods), n), generator=gen, dtype=torch.int64, device=device)
    return (x % qs).view(torch.uint64)
