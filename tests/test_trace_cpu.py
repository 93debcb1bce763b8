"""Host logic of the bootstrapping-shaped plans: the factored DFT's rotation
offsets computed combinatorially by the package equal the non-zero diagonals
of the oracle's factor matrices, and plans are consistent."""
import pytest

from oracle import encoding as C
from paper_2112_06396_amd import trace


@pytest.mark.parametrize("log_slots", [1, 2, 3, 5, 8, 9, 11])
def test_dft_offsets_equal_the_oracle_factors_diagonals(log_slots):
    n = 1 << log_slots
    for iters in sorted({1, min(3, log_slots), log_slots}):
        for inverse in (True, False):
            f = C.coeff_to_slot_factors(n, iters) if inverse else C.slot_to_coeff_factors(n, iters)
            assert trace.dft_offsets(log_slots, iters, inverse) == [sorted(G) for G in f]


def test_dft_plan_shape_at_the_benchmark_size():
    """N = 2^16 (2^15 slots), three iterations: CoeffToSlot 32, 63, 63
    diagonals and SlotToCoeff 63, 63, 32; 155 distinct non-zero rotations."""
    assert [len(g) for g in trace.dft_offsets(15, 3, True)] == [32, 63, 63]
    assert [len(g) for g in trace.dft_offsets(15, 3, False)] == [63, 63, 32]
    p = trace.bootstrap_plan(35, dft=(15, 3), hoisted=True, new_mult=True)
    assert len(p.rotations) == 155 and 0 not in p.rotations
    assert p.key_switches == 2 * (31 + 62 + 62) + 40
    assert p.out_level == 35 - 3 - 20 - 3
    levels = [op[2] for op in p.ops if op[0] == "ptmatvec"]
    assert levels == [35, 34, 33, 12, 11, 10]


def test_unhoisted_dft_plan_uses_the_input_for_offset_zero():
    p = trace.bootstrap_plan(8, dft=(3, 3), evalmod_levels=1)
    first = [op for op in p.ops if op[0] == "ptmult"][0]
    assert first[1] == "x0"  # offset 0 of the first factor multiplies the input itself
    assert all(0 not in op[3] for op in p.ops if op[0] == "hrotate")
