"""Plant plausible mistakes in the CTM-move oracle (on the CPU) and check that
a pin of test_oracle_ctm.py fails for each."""

import numpy as np
import pytest

import oracle
from oracle import ctm as OC
from tests import test_oracle_ctm as P

CAUGHT = (AssertionError, KeyError, ValueError, IndexError, oracle.OracleError)


def _run_pins(cases=("u1", "z2")):
    for name in cases:
        env, dense, spaces = P._dense_env(name)
        chi = env["chi"]
        mv = (name, env, dense, spaces, OC.left_move(env, 10 ** 6), OC.left_move(env, max(1, chi - 2)))
        P.test_enlarged_corners_and_halves_match_the_dense_network(mv)
        P.test_untruncated_projectors_keep_every_value_above_the_floor(mv)
        P.test_truncated_projectors_give_the_best_rank_chi_approximation(mv)
        P.test_renormalised_tensors_match_the_dense_network(mv)
        P.test_renormalisation_divides_by_the_largest_entry(mv)
        P.test_factors_follow_the_svd_gauge(mv)
    P.test_one_element_network_closed_form()


def test_ctm_pins_pass_unmutated():
    _run_pins()


def _mut_projector_power(monkeypatch):
    """S^+1/2 in the projectors instead of S^-1/2."""
    orig = OC.scale_new_leg
    monkeypatch.setattr(OC, "scale_new_leg", lambda t, s, p, leg: orig(t, s, -p, leg))


def _mut_v_side_unscaled(monkeypatch):
    """S^-1/2 applied to U only (V^T left unscaled)."""
    orig = OC.scale_new_leg
    monkeypatch.setattr(OC, "scale_new_leg", lambda t, s, p, leg: orig(t, s, p if leg else 0.0, leg))


def _mut_corner_axes(monkeypatch):
    """The bottom-right corner's A step pairs T3.k with A.r and T2.k with A.b
    (legs of equal signature classes and dims: no structural error)."""
    chains = dict(OC.CORNER_CHAINS)
    q3 = list(chains["Q3"])
    q3[2] = (None, "A", (1, 4), (3, 2))
    chains["Q3"] = q3
    monkeypatch.setattr(OC, "CORNER_CHAINS", chains)


def _mut_frobenius_normalisation(monkeypatch):
    def bad(t):
        f = float(np.linalg.norm(t.data))
        return type(t)(t.sym_mod, t.sig, t.n, t.charges, t.shapes, t.offsets, t.data / f)
    monkeypatch.setattr(OC, "normalise_max", bad)


def _mut_projectors_exchanged(monkeypatch):
    """P_dn used for C1' and P_up for C4'."""
    orig = OC.left_move

    def bad(env, chi, tol=0.0, deg_tol=1e-10):
        r = orig(env, chi, tol, deg_tol)
        r["C1n"] = OC._td(r["Pdn"], r["C1T1"], (0, 1, 2), (0, 1, 2))
        return r
    monkeypatch.setattr(OC, "left_move", bad)


def _mut_no_gauge(monkeypatch):
    """Every singular pair with the opposite sign."""
    monkeypatch.setattr(oracle.svd, "sign_gauge", lambda U, Vt: (-U, -Vt))


MUTATIONS = [_mut_projector_power, _mut_v_side_unscaled, _mut_corner_axes, _mut_frobenius_normalisation,
             _mut_projectors_exchanged, _mut_no_gauge]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m.__name__ for m in MUTATIONS])
def test_each_ctm_mutation_is_caught(mut, monkeypatch):
    mut(monkeypatch)
    with pytest.raises(CAUGHT):
        _run_pins()
