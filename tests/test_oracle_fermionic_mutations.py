"""Plant plausible mistakes in the complex / fermionic oracle (on the CPU) and
check that a pin of test_oracle_fermionic.py fails for each."""

import numpy as np
import pytest

import oracle
from oracle import blocksparse as B
from oracle import fermionic as F
from tests import test_oracle_fermionic as P

CAUGHT = (AssertionError, KeyError, ValueError, IndexError, TypeError, oracle.OracleError)


def _run_pins():
    for case in P.CASES:
        P.test_complex_tensordot_matches_dense_and_real_parts(*case)
        P.test_conjugation_identity(*case)
        P.test_conj_gives_the_squared_norm(*case)
        for l1, l2 in (((0,), (1,)), ((0, 2), (3,)), ((1,), (2, 3))):
            P.test_swap_gate_is_the_dense_sign_pattern(*case, l1, l2)
        P.test_swap_gate_involution_and_commutation(*case)
    P.test_swap_gate_hand_example_z2()
    P.test_real_values_reduce_to_the_real_oracle()


def test_fermionic_pins_pass_unmutated():
    _run_pins()


def _mut_conj_keeps_values(monkeypatch):
    monkeypatch.setattr(F, "conj", lambda t: B.dual(t))


def _mut_parity_first_component(monkeypatch):
    monkeypatch.setattr(F, "parity", lambda q, fer: int(q[0]) % 2)


def _mut_swap_either_odd(monkeypatch):
    """Sign flipped where either group (not both) is odd."""
    def bad(t, legs1, legs2, fer):
        out = t.copy()
        for b in range(t.nblocks):
            p1 = sum(F.parity(t.charges[b, i], fer) for i in legs1) % 2
            p2 = sum(F.parity(t.charges[b, j], fer) for j in legs2) % 2
            if p1 or p2:
                o, sz = int(t.offsets[b]), int(np.prod(t.shapes[b]))
                out.data[o:o + sz] = -np.asarray(t.data)[o:o + sz]
        return out
    monkeypatch.setattr(F, "swap_gate", bad)


def _mut_real_accumulator(monkeypatch):
    """Block sums accumulated in float64 (imaginary parts lost)."""
    monkeypatch.setattr(B, "_value_type", lambda a, b: np.float64)


def _mut_conj_b_only(monkeypatch):
    orig = F.tensordot_c
    monkeypatch.setattr(F, "tensordot_c", lambda a, b, ax, bx, conj_a=False, conj_b=False:
                        orig(a, b, ax, bx, False, conj_b))


MUTATIONS = [_mut_conj_keeps_values, _mut_parity_first_component, _mut_swap_either_odd, _mut_real_accumulator,
             _mut_conj_b_only]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m.__name__ for m in MUTATIONS])
def test_each_fermionic_mutation_is_caught(mut, monkeypatch):
    mut(monkeypatch)
    with pytest.raises(CAUGHT):
        _run_pins()
