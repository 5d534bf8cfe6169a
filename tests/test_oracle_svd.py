"""Pins of the block-sparse truncated SVD oracle (oracle/svd.py).

None re-types the oracle's own steps: the singular values are checked against
the SVD of the dense matrix the block tensor embeds into (rows = the row legs'
dense index space, columns = the column legs'), the factors by reconstructing
the tensor and by orthonormality, a block-diagonal tensor against its closed
form, and the truncation rule against hand-made spectra whose kept sets are
worked out by hand.
"""

import numpy as np
import pytest

import oracle
from oracle import svd as OS
from workloads import Leg, rand

SYMS = {"U1": (0,), "Z2": (2,), "U1xU1": (0, 0)}


CHARGES = {"U1": [(-1,), (0,), (1,)], "Z2": [(0,), (1,)],
           "U1xU1": [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1)]}


def _random_tensor(seed, sym, rank, n=None):
    """Legs whose 1-3 sectors come from a small common charge set (so many
    charge tuples conserve), dims 1-4, i.i.d. N(0,1) blocks."""
    rng = np.random.default_rng(seed)
    sm = SYMS[sym]
    pool = CHARGES[sym]
    legs = []
    for _ in range(rank):
        k = int(rng.integers(min(2, len(pool)), min(3, len(pool)) + 1))
        ts = sorted(pool[i] for i in rng.choice(len(pool), size=k, replace=False))
        legs.append(Leg(int(rng.choice([-1, 1])), tuple(ts), tuple(int(rng.integers(1, 5)) for _ in ts)))
    if n is None:
        n = tuple(0 for _ in sm)
    return rand(legs, n, sm, seed + 1000)


def _dense_matrix(t, row_legs):
    maps = oracle.leg_index_maps(t)
    d = oracle.to_dense(t, maps)
    col_legs = [x for x in range(t.rank) if x not in row_legs]
    m = int(np.prod([maps[x]["D"] for x in row_legs])) if row_legs else 1
    return np.transpose(d, list(row_legs) + col_legs).reshape(m, -1)


CASES = [(1, "U1", 4, (0, 2), None), (2, "U1", 4, (0, 1), (1,)), (3, "Z2", 3, (1,), (1,)),
         (4, "U1xU1", 4, (0, 3), None), (5, "U1", 5, (4, 0), None), (6, "Z2", 4, (2, 3), None),
         (12, "U1xU1", 3, (0,), (1, 0))]


@pytest.mark.parametrize("seed,sym,rank,rows,n", CASES)
def test_sector_values_are_the_dense_matrix_values(seed, sym, rank, rows, n):
    """The block-diagonal structure: the union of the sectors' singular values
    is the spectrum of the dense embedded matrix (which adds only zeros)."""
    t = _random_tensor(seed, sym, rank, n)
    assert t.nblocks > 0
    sv = OS.svd_sectors(t, rows)
    union = np.sort(np.concatenate([s for _, s, _ in sv.values()]))[::-1]
    dense = np.linalg.svd(_dense_matrix(t, rows), compute_uv=False)
    smax = float(dense[0])
    assert union.size <= dense.size
    assert np.max(np.abs(union - dense[:union.size])) <= 1e-12 * smax
    assert np.all(dense[union.size:] <= 1e-12 * smax)


@pytest.mark.parametrize("seed,sym,rank,rows,n", CASES)
def test_full_rank_reconstruction_and_orthonormality(seed, sym, rank, rows, n):
    """Keeping every value: U diag(S) V^T contracted over the new leg and put
    back in the tensor's leg order is the tensor itself; U and V have
    orthonormal columns in every sector."""
    t = _random_tensor(seed, sym, rank, n)
    assert t.nblocks > 0
    u, S, vt, kept = OS.svd_truncated(t, rows, chi=10 ** 9, tol=0.0)
    assert sum(kept.values()) == sum(len(s) for _, s, _ in OS.svd_sectors(t, rows).values())
    # scale U's columns: multiply each block's last axis by the sector's S
    us = u.copy() if hasattr(u, "copy") else u
    data = us.data.copy()
    for b in range(us.nblocks):
        X = tuple(int(v) for v in us.charges[b, -1])
        o, sz = int(us.offsets[b]), int(np.prod(us.shapes[b]))
        blk = data[o:o + sz].reshape(tuple(us.shapes[b])) * S[X]
        data[o:o + sz] = blk.ravel()
    us = type(u)(u.sym_mod, u.sig, u.n, u.charges, u.shapes, u.offsets, data)
    rec = oracle.tensordot_dense(us, vt, (u.rank - 1,), (0,))
    col_legs = [x for x in range(t.rank) if x not in rows]
    order = list(rows) + col_legs
    back = oracle.transpose(rec, [order.index(x) for x in range(t.rank)])
    maps = oracle.leg_index_maps(t)
    assert np.allclose(oracle.to_dense(back, maps) if back.nblocks else 0.0, oracle.to_dense(t, maps),
                       rtol=0, atol=1e-12 * max(1.0, float(np.abs(t.data).max())))
    for X, (U, s, Vt) in OS.svd_sectors(t, rows).items():
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
        assert np.allclose(Vt @ Vt.T, np.eye(Vt.shape[0]), atol=1e-13)
        assert np.all(np.diff(s) <= 0)


def test_block_diagonal_closed_form():
    """A rank-2 U(1) tensor on legs (l, l*) whose blocks are diagonal with
    known entries: the sectors' singular values are the sorted absolute
    entries, and chi = 4 keeps exactly the four largest."""
    leg = Leg(1, ((-1,), (0,), (1,)), (2, 3, 1))
    t = rand([leg, leg.conj()], (0,), (0,), 5)
    vals = {(-1,): [3.0, -7.0], (0,): [0.5, 6.0, -2.0], (1,): [-4.0]}
    data = np.zeros_like(t.data)
    for b in range(t.nblocks):
        q = (int(t.charges[b, 0, 0]),)
        o = int(t.offsets[b])
        d = int(t.shapes[b, 0])
        data[o:o + d * d] = np.diag(vals[q]).ravel()
    t = type(t)(t.sym_mod, t.sig, t.n, t.charges, t.shapes, t.offsets, data)
    sv = OS.svd_sectors(t, (0,))
    for q, v in vals.items():
        assert np.allclose(sv[q][1], sorted(np.abs(v), reverse=True), rtol=0, atol=1e-14)
    u, S, vt, kept = OS.svd_truncated(t, (0,), chi=4)
    assert kept == {(-1,): 2, (0,): 1, (1,): 1}   # 7, 6, 4, 3 kept; 2, 0.5 dropped
    assert sorted(np.concatenate(list(S.values())).tolist()) == [3.0, 4.0, 6.0, 7.0]
    # U and V^T carry the new leg: U (l, v) with v of signature -1, n = 0
    assert u.sig.tolist() == [1, -1] and vt.sig.tolist() == [1, -1]
    assert u.nblocks == 3 and vt.nblocks == 3


# ------------------------------------------------------ truncation rule
def test_truncation_rule_hand_made_spectra():
    s = {"a": np.array([5.0, 3.0, 1.0]), "b": np.array([4.0, 3.0, 0.5])}
    # chi = 3: the 3rd and 4th largest are both 3 (a degenerate pair across
    # sectors): the pair is dropped whole, leaving 5 and 4
    assert OS.truncation(s, 3) == {"a": 1, "b": 1}
    # chi = 4: 5, 4, 3, 3 kept (the 5th largest is 1)
    assert OS.truncation(s, 4) == {"a": 2, "b": 2}
    # chi at or above the number of values: everything above the floor
    assert OS.truncation(s, 6) == {"a": 3, "b": 3}
    assert OS.truncation(s, 100) == {"a": 3, "b": 3}
    # tol: values at or below tol * 5 are dropped first
    assert OS.truncation(s, 100, tol=0.2) == {"a": 2, "b": 2}   # 1 and 0.5 <= 1.0
    assert OS.truncation(s, 100, tol=0.19) == {"a": 3, "b": 2}  # 0.95 floor keeps 1
    # chi = 0 keeps nothing
    assert OS.truncation(s, 0) == {"a": 0, "b": 0}
    # near-degenerate within deg_tol of the first dropped value: dropped too
    s2 = {"a": np.array([2.0, 1.0 + 1e-12]), "b": np.array([1.0])}
    assert OS.truncation(s2, 2) == {"a": 1, "b": 0}
    assert OS.truncation(s2, 2, deg_tol=0.0) == {"a": 2, "b": 0}
    # exact zeros never survive the floor
    assert OS.truncation({"a": np.array([1.0, 0.0])}, 5) == {"a": 1}


@pytest.mark.parametrize("seed,sym,rank,rows,n", CASES)
def test_sign_gauge_largest_entry_positive(seed, sym, rank, rows, n):
    """The sign of each singular pair: u_k's entry of largest magnitude is
    positive (the factors are then unique for distinct values), and the
    flip is applied to both factors (reconstruction above still holds)."""
    t = _random_tensor(seed, sym, rank, n)
    for X, (U, s, Vt) in OS.svd_sectors(t, rows).items():
        for k in range(U.shape[1]):
            col = np.abs(U[:, k])
            i = int(np.flatnonzero(col == col.max())[0])
            assert U[i, k] > 0.0
