"""Plant plausible mistakes in the truncated-SVD oracle (on the CPU) and check
that a pin of test_oracle_svd.py fails for each."""

import numpy as np
import pytest

import oracle.svd as OS
from tests import test_oracle_svd as P

CAUGHT = (AssertionError, KeyError, ValueError, IndexError)


def _run_pins():
    for case in P.CASES:
        P.test_sector_values_are_the_dense_matrix_values(*case)
        P.test_full_rank_reconstruction_and_orthonormality(*case)
        P.test_sign_gauge_largest_entry_positive(*case)
    P.test_block_diagonal_closed_form()
    P.test_truncation_rule_hand_made_spectra()


def test_svd_pins_pass_unmutated():
    _run_pins()


def _mut_sector_unsigned(monkeypatch):
    """The sector charge summed without the leg signatures."""
    def bad(t, b, legs):
        tot = [0] * t.nsym
        for x in legs:
            for c in range(t.nsym):
                tot[c] += int(t.charges[b, x, c])
        return tuple(OS._nq(tot, t.sym_mod))
    monkeypatch.setattr(OS, "_sector_of", bad)


def _mut_block_transposed(monkeypatch):
    """A block placed with its column legs first (a transposed sub-matrix,
    reshaped into the slot)."""
    orig = OS.sector_matrices

    def bad(t, row_legs):
        out = orig(t, row_legs)
        res = {}
        for X, (M, rl, cl) in out.items():
            M = M.copy()
            for _, rd, ro in rl[:1]:
                for _, cd, co in cl[:1]:
                    m, n = int(np.prod(rd)), int(np.prod(cd))
                    M[ro:ro + m, co:co + n] = M[ro:ro + m, co:co + n].T.reshape(m, n)
            res[X] = (M, rl, cl)
        return res
    monkeypatch.setattr(OS, "sector_matrices", bad)


def _mut_truncation_keeps_one_more(monkeypatch):
    orig = OS.truncation

    def bad(svals, chi, tol=0.0, deg_tol=1e-10):
        return orig(svals, chi + 1, tol, deg_tol)
    monkeypatch.setattr(OS, "truncation", bad)


def _mut_truncation_splits_multiplets(monkeypatch):
    """Ties at the cut resolved by order instead of dropped whole."""
    def bad(svals, chi, tol=0.0, deg_tol=1e-10):
        allv = sorted(((float(v), X, i) for X, s in svals.items() for i, v in enumerate(s)), reverse=True)
        smax = allv[0][0] if allv else 0.0
        kept = {X: 0 for X in svals}
        for v, X, i in allv[:chi]:
            if v > tol * smax:
                kept[X] += 1
        return kept
    monkeypatch.setattr(OS, "truncation", bad)


def _mut_u_without_last_column(monkeypatch):
    """The kept U columns cut one short (an off-by-one in the slice)."""
    orig = OS.svd_truncated

    def bad(t, row_legs, chi, tol=0.0, deg_tol=1e-10):
        u, S, vt, kept = orig(t, row_legs, chi, tol, deg_tol)
        data = u.data.copy()
        for b in range(u.nblocks):
            o, sh = int(u.offsets[b]), tuple(int(x) for x in u.shapes[b])
            blk = data[o:o + int(np.prod(sh))].reshape(sh)
            blk[..., -1] = 0.0
            data[o:o + blk.size] = blk.ravel()
        return type(u)(u.sym_mod, u.sig, u.n, u.charges, u.shapes, u.offsets, data), S, vt, kept
    monkeypatch.setattr(OS, "svd_truncated", bad)


def _mut_values_ascending(monkeypatch):
    """Singular values reported in ascending order (a reversed sort)."""
    orig = OS.svd_sectors

    def bad(t, row_legs):
        return {X: (U[:, ::-1], s[::-1], Vt[::-1]) for X, (U, s, Vt) in orig(t, row_legs).items()}
    monkeypatch.setattr(OS, "svd_sectors", bad)


def _mut_no_sign_gauge(monkeypatch):
    """The raw LAPACK signs kept."""
    monkeypatch.setattr(OS, "sign_gauge", lambda U, Vt: (U, Vt))


def _mut_gauge_flips_u_only(monkeypatch):
    """The sign fixed on u_k but not carried to v_k."""
    orig = OS.sign_gauge
    monkeypatch.setattr(OS, "sign_gauge", lambda U, Vt: (orig(U, Vt)[0], Vt))


MUTATIONS = [_mut_no_sign_gauge, _mut_gauge_flips_u_only, _mut_sector_unsigned, _mut_block_transposed, _mut_truncation_keeps_one_more,
             _mut_truncation_splits_multiplets, _mut_u_without_last_column, _mut_values_ascending]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m.__name__ for m in MUTATIONS])
def test_each_svd_mutation_is_caught(mut, monkeypatch):
    mut(monkeypatch)
    with pytest.raises(CAUGHT):
        _run_pins()
