"""Pins of the complex and fermionic oracle (oracle/fermionic.py).

Complex tensordot: against the dense embedding in complex arithmetic (O1),
against its four real parts computed with the real oracle, and the
conjugation identity conj(A).conj(B) = conj(A.B).  Swap gates: against the
dense tensor multiplied by the sign of each dense index (the parity of the
charge sector it lies in, on each swapped leg), a hand-made Z2 example, the
involution, and commutation with a contraction that leaves both groups free.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import fermionic as F
from workloads import Leg

CASES = [  # (sym_mod, legs, n, axes_a, axes_b) for A and B built on the same legs
    ((W.U1,), "u1", (0,)),
    ((2,), "z2", (1,)),
    ((W.U1, W.U1), "u1xu1", (0, 0)),
]


def _legs(kind):
    if kind == "u1":
        v = Leg(1, ((-1,), (0,), (1,)), (2, 3, 1))
        w = Leg(1, ((0,), (1,), (2,)), (1, 2, 2))
    elif kind == "z2":
        v = Leg(1, ((0,), (1,)), (2, 3))
        w = Leg(1, ((0,), (1,)), (1, 2))
    else:
        v = Leg(1, ((0, 0), (1, 0), (0, 1)), (2, 1, 2))
        w = Leg(1, ((0, 0), (1, 1), (-1, 0)), (1, 2, 1))
    return v, w


def _pair(sym, kind, n, seed):
    v, w = _legs(kind)
    a = W.rand_complex([v, w, v.conj(), w], n, sym, seed)
    b = W.rand_complex([v, w.conj(), v], tuple(0 for _ in sym), sym, seed + 1)
    return a, b


def _real_part(t, part):
    out = t.copy()
    out.data = np.ascontiguousarray(getattr(np.asarray(t.data), part)).astype(np.float64)
    return out


@pytest.mark.parametrize("sym,kind,n", CASES)
def test_complex_tensordot_matches_dense_and_real_parts(sym, kind, n):
    a, b = _pair(sym, kind, n, 11)
    ax, bx = (2, 3), (0, 1)
    c = oracle.tensordot_blockpair(a, b, ax, bx)
    assert c.data.dtype == np.complex128 and c.nblocks > 0
    d = oracle.tensordot_dense(a, b, ax, bx)
    assert oracle.same_structure(c, d)
    assert np.max(np.abs(c.data - d.data)) <= 1e-13 * np.max(np.abs(d.data))
    # (Ar + i Ai)(Br + i Bi) from four real contractions
    ar, ai, br, bi = _real_part(a, "real"), _real_part(a, "imag"), _real_part(b, "real"), _real_part(b, "imag")
    rr, ii = oracle.tensordot_blockpair(ar, br, ax, bx), oracle.tensordot_blockpair(ai, bi, ax, bx)
    ri, ir = oracle.tensordot_blockpair(ar, bi, ax, bx), oracle.tensordot_blockpair(ai, br, ax, bx)
    assert np.allclose(c.data.real, rr.data - ii.data, rtol=0, atol=1e-13 * np.max(np.abs(c.data)))
    assert np.allclose(c.data.imag, ri.data + ir.data, rtol=0, atol=1e-13 * np.max(np.abs(c.data)))


@pytest.mark.parametrize("sym,kind,n", CASES)
def test_conjugation_identity(sym, kind, n):
    """conj(A).conj(B) = conj(A.B): the same blocks with flipped signatures
    and total charge, conjugated values; conj twice is the identity."""
    a, b = _pair(sym, kind, n, 21)
    ax, bx = (1, 2), (1, 0)
    ab = oracle.tensordot_blockpair(a, b, ax, bx)
    cc = F.tensordot_c(a, b, ax, bx, conj_a=True, conj_b=True)
    ref = F.conj(ab)
    assert cc.sig.tolist() == (-ab.sig).tolist() and cc.n.tolist() == ref.n.tolist()
    assert np.array_equal(cc.charges, ref.charges) and np.array_equal(cc.shapes, ref.shapes)
    assert np.allclose(cc.data, ref.data, rtol=0, atol=1e-13 * np.max(np.abs(ab.data)))
    back = F.conj(F.conj(a))
    assert np.array_equal(back.data, a.data) and back.sig.tolist() == a.sig.tolist()


@pytest.mark.parametrize("sym,kind,n", CASES)
def test_conj_gives_the_squared_norm(sym, kind, n):
    """<A|A> = tensordot(conj(A), A) over every leg = sum |a|^2, a real
    positive number (conjugation maps each leg to its dual, so every leg of
    conj(A) contracts with the same leg of A)."""
    a, _ = _pair(sym, kind, n, 61)
    legs = tuple(range(a.rank))
    s = oracle.tensordot_blockpair(F.conj(a), a, legs, legs)
    assert s.rank == 0 and s.nblocks == 1
    ref = float(np.sum(np.abs(a.data) ** 2))
    assert abs(s.data[0] - ref) <= 1e-13 * ref and s.data[0].imag == 0.0


def test_real_values_reduce_to_the_real_oracle():
    a, b = _pair((W.U1,), "u1", (0,), 31)
    a.data = a.data.real.astype(np.complex128)
    b.data = b.data.real.astype(np.complex128)
    c = oracle.tensordot_blockpair(a, b, (2, 3), (0, 1))
    r = oracle.tensordot_blockpair(_real_part(a, "real"), _real_part(b, "real"), (2, 3), (0, 1))
    assert np.array_equal(c.data.real, r.data) and not np.any(c.data.imag)


# ---------------------------------------------------------------- swap gates
def _dense_signs(t, maps, legs1, legs2, fermionic):
    """(-1)^(P1 P2) at every dense index, P_k the parity of the summed
    charges of group k at that index (every charge component fermionic here:
    the parity of a charge is the sum of its components mod 2)."""
    assert all(f == 1 for f in fermionic)
    par = []
    for l, m in enumerate(maps):
        p = np.zeros(m["D"], dtype=np.int64)
        for q in m["charges"]:
            p[m["start"][q]:m["start"][q] + m["dims"][q]] = sum(int(v) for v in q) % 2
        par.append(p)
    grids = np.meshgrid(*par, indexing="ij")
    p1 = sum(grids[i] for i in legs1) % 2 if legs1 else 0
    p2 = sum(grids[j] for j in legs2) % 2 if legs2 else 0
    return np.where((p1 * p2) % 2 == 1, -1.0, 1.0)


@pytest.mark.parametrize("sym,kind,n", CASES)
@pytest.mark.parametrize("legs1,legs2", [((0,), (1,)), ((0, 2), (3,)), ((1,), (2, 3)), ((0,), (0,))])
def test_swap_gate_is_the_dense_sign_pattern(sym, kind, n, legs1, legs2):
    a, _ = _pair(sym, kind, n, 41)
    fer = W.FERMIONIC[tuple(sym)]
    maps = oracle.leg_index_maps(a)
    got = oracle.to_dense(F.swap_gate(a, legs1, legs2, fer), maps)
    ref = oracle.to_dense(a, maps) * _dense_signs(a, maps, legs1, legs2, fer)
    assert np.array_equal(got, ref)


def test_swap_gate_hand_example_z2():
    """Legs V = Z2 {0: dim 1, 1: dim 1} and its dual, n = 0: blocks (0, 0)
    and (1, 1); the swap gate negates (1, 1) only."""
    v = Leg(1, ((0,), (1,)), (1, 1))
    t = W.rand([v, v.conj()], (0,), (2,), 3)
    assert t.nblocks == 2
    s = F.swap_gate(t, (0,), (1,), (1,))
    assert s.data[0] == t.data[0] and s.data[1] == -t.data[1]


@pytest.mark.parametrize("sym,kind,n", CASES)
def test_swap_gate_involution_and_commutation(sym, kind, n):
    a, b = _pair(sym, kind, n, 51)
    fer = W.FERMIONIC[tuple(sym)]
    s = F.swap_gate(a, (0,), (1,), fer)
    assert np.array_equal(F.swap_gate(s, (0,), (1,), fer).data, a.data)
    assert np.array_equal(F.swap_gate(a, (), (1,), fer).data, a.data)
    # a swap of A's free legs 0, 1 commutes with contracting legs 2, 3
    left = oracle.tensordot_blockpair(s, b, (2, 3), (0, 1))
    right = F.swap_gate(oracle.tensordot_blockpair(a, b, (2, 3), (0, 1)), (0,), (1,), fer)
    assert np.allclose(left.data, right.data, rtol=0, atol=1e-13 * np.max(np.abs(right.data)))
