"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: they use closed forms
(convolution counts of the D = 18 contraction), the paper's worked example with its physical
values, brute force over dense indices, special cases that reduce to plain
numpy.tensordot, and bitwise invariants.
"""

import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import random_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------- rank-4 U(1), D = 18
def test_u1_d18_closed_form_structure():
    # Leg {-2:2,-1:4,0:6,1:4,2:2}, signature (+,+,-,-), n=0.  A block (q0,q1,q2,q3)
    # is allowed iff q0+q1 = q2+q3 =: s.  For each s the number of (q0,q1) pairs is
    # c_s = (1,2,3,4,5,4,3,2,1) and the elements per side conv_s = (d*d)[s]
    # (self-convolution of the dims).
    dims = [2, 4, 6, 4, 2]
    conv = np.convolve(dims, dims)
    cnt = np.convolve([1] * 5, [1] * 5)
    assert conv.tolist() == [4, 16, 40, 64, 76, 64, 40, 16, 4]
    assert cnt.tolist() == [1, 2, 3, 4, 5, 4, 3, 2, 1]
    (p,) = W.u1_d18()
    a, b = p.a, p.b
    assert a.nblocks == int(np.sum(cnt ** 2)) == 85
    assert int(a.block_sizes.sum()) == int(np.sum(conv ** 2)) == 17712
    st = oracle.structure_stats(a, b, p.axes_a, p.axes_b)
    assert st["pairs"] == int(np.sum(cnt ** 3)) == 325
    assert st["sectors"] == 9
    mkn = [st["mkn"][k] for k in sorted(st["mkn"])]
    assert [m for m, k, n in mkn] == conv.tolist()
    assert all(m == k == n for m, k, n in mkn)
    assert st["flops"] == 2 * int(np.sum(conv ** 3)) == 2199168
    assert st["c_blocks"] == 85
    c = oracle.output_structure(a, b, p.axes_a, p.axes_b)
    # C's legs are A's free legs (+,+) then B's free legs (-,-): same tuples as A
    assert np.array_equal(c.charges, a.charges)
    assert int(c.block_sizes.sum()) == 17712


def test_u1_d18_dense_equals_blockpair():
    (p,) = W.u1_d18()
    c1 = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    c2 = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
    assert oracle.same_structure(c1, c2)
    assert oracle.rel_frobenius(c2.data, c1.data) < 1e-13


# ------------------------------------------------------- the worked example
def _gold():
    rows = []
    with open(os.path.join(GOLD, "h_squared.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.append((tuple(int(x) for x in v[:4]), float(v[4]), float(v[5])))
    return rows


def test_paper_example_h_structure_and_fusion():
    H = W.spin_half_pair_hamiltonian()
    assert H.nblocks == 6
    vals = {tuple(int(q) for q in H.charges[b, :, 0]): float(H.block(b).ravel()[0])
            for b in range(H.nblocks)}
    for key, h, _ in _gold():
        assert vals[key] == h
    Hm, rec = oracle.fuse_legs(H, ((0, 1), (2, 3)))
    # fused charges {-2:1, 0:2, 2:1} on both legs: a 4x4 block-diagonal matrix
    assert Hm.rank == 2
    assert [int(q) for q in Hm.charges[:, 0, 0]] == [-2, 0, 2]
    assert Hm.shapes.tolist() == [[1, 1], [2, 2], [1, 1]]
    back = oracle.unfuse_legs(Hm, rec)
    assert oracle.same_structure(back, H) and np.array_equal(back.data, H.data)


@pytest.mark.parametrize("impl", ["dense", "blockpair", "brute"])
def test_paper_example_h_squared_exact(impl):
    H = W.spin_half_pair_hamiltonian()
    if impl == "brute":
        cd = oracle.tensordot_brute(H, H, (2, 3), (0, 1))
        idx = {-1: 0, 1: 1}
        for key, _, h2 in _gold():
            assert cd[tuple(idx[q] for q in key)] == h2
        return
    f = oracle.tensordot_dense if impl == "dense" else oracle.tensordot_blockpair
    H2 = f(H, H, (2, 3), (0, 1))
    got = {tuple(int(q) for q in H2.charges[b, :, 0]): float(H2.block(b).ravel()[0])
           for b in range(H2.nblocks)}
    assert len(got) == 6
    for key, _, h2 in _gold():
        assert got[key] == h2  # bitwise: dyadic values


def test_paper_example_fused_matmul_identity():
    # tensordot(H,H,((2,3),(0,1))) == (H_mat @ H_mat).unfuse  (Sec. II.B listing)
    H = W.spin_half_pair_hamiltonian()
    Hm, rec = oracle.fuse_legs(H, ((0, 1), (2, 3)))
    H2m = oracle.tensordot_blockpair(Hm, Hm, (1,), (0,))
    H2 = oracle.unfuse_legs(H2m, [rec[0], rec[1]])
    ref = oracle.tensordot_blockpair(H, H, (2, 3), (0, 1))
    assert oracle.same_structure(H2, ref) and np.array_equal(H2.data, ref.data)


def test_norms_closed_form():
    H = W.spin_half_pair_hamiltonian()
    fro, mx = oracle.norms(H)
    assert fro == pytest.approx(np.sqrt(3) / 2, rel=1e-15)  # 4/16 + 2/4 = 3/4
    assert mx == 0.5


# ----------------------------------------------------- O1 vs O2 vs O3
@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("sym", ["U1", "Z2", "U1xZ2"])
def test_brute_dense_blockpair_agree(seed, sym):
    a, b, xa, xb = random_problem(seed, sym, max_sectors=2, max_dim=2,
                                  keep=0.8 if seed % 3 == 0 else None,
                                  drop_partner=seed % 4 == 1)
    c1, cd = oracle.tensordot_dense(a, b, xa, xb, return_dense=True)
    cd3 = oracle.tensordot_brute(a, b, xa, xb)
    assert cd3.shape == cd.shape
    assert np.allclose(cd3, cd, rtol=0, atol=1e-13)
    c2 = oracle.tensordot_blockpair(a, b, xa, xb)
    assert oracle.same_structure(c1, c2)
    np.testing.assert_allclose(c2.data, c1.data, rtol=1e-13, atol=1e-13)
    for k in range(c1.nblocks):  # output blocks obey sum s*rho = n_C
        tot = np.zeros(c1.nsym, dtype=np.int64)
        for i in range(c1.rank):
            tot += int(c1.sig[i]) * c1.charges[k, i, :].astype(np.int64)
        for cc, m in enumerate(c1.sym_mod):
            assert (tot[cc] % m if m else tot[cc]) == c1.n[cc]


@pytest.mark.parametrize("seed", range(30))
def test_larger_random_dense_vs_blockpair(seed):
    sym = ["U1", "Z3", "U1xU1"][seed % 3]
    a, b, xa, xb = random_problem(seed + 1000, sym, rank_a=int(2 + seed % 4), rank_b=int(2 + (seed // 4) % 4),
                                  max_sectors=4, max_dim=4, keep=0.7 if seed % 2 else None,
                                  shuffle=seed % 5 == 0)
    c1 = oracle.tensordot_dense(a, b, xa, xb)
    c2 = oracle.tensordot_blockpair(a, b, xa, xb)
    assert oracle.same_structure(c1, c2)
    assert oracle.rel_frobenius(c2.data, c1.data) < 1e-13


# ------------------------------------------------------ special cases
def test_single_sector_reduces_to_numpy_tensordot():
    rng = np.random.default_rng(5)
    legs = [W.Leg(s, ((0,),), (d,)) for s, d in zip((1, 1, -1, -1, 1), (3, 4, 5, 2, 3))]
    a = W.rand(legs, (0,), (0,), 1)
    legs_b = [legs[2].conj(), W.Leg(1, ((0,),), (6,)), legs[1].conj()]
    b = W.rand(legs_b, (0,), (0,), 2)
    c = oracle.tensordot_blockpair(a, b, (2, 1), (0, 2))
    ref = np.tensordot(a.block(0), b.block(0), axes=((2, 1), (0, 2)))
    assert c.nblocks == 1 and np.array_equal(c.block(0), ref)
    del rng


def test_all_z2_charge_zero_reduces_to_numpy_tensordot():
    legs = [W.Leg(s, ((0,),), (d,)) for s, d in zip((1, -1, 1), (4, 3, 5))]
    a = W.rand(legs, (0,), (2,), 7)
    b = W.rand([legs[1].conj(), W.Leg(-1, ((0,),), (2,))], (0,), (2,), 8)
    c = oracle.tensordot_dense(a, b, (1,), (0,))
    ref = np.tensordot(a.block(0), b.block(0), axes=((1,), (0,)))
    assert np.array_equal(c.block(0), ref)


def test_empty_and_full_contraction():
    # tensor with no blocks -> empty C; contraction over all legs -> scalar block
    legs = [W.Leg(1, ((0,), (1,)), (2, 3)), W.Leg(-1, ((0,), (1,)), (2, 3))]
    a = W.rand(legs, (0,), (0,), 1)
    b = W.rand([l.conj() for l in legs], (0,), (0,), 2)
    c = oracle.tensordot_dense(a, b, (0, 1), (0, 1))
    assert c.rank == 0 and c.nblocks == 1
    ref = sum(float(np.sum(a.block(i) * b.block(i))) for i in range(2))
    assert c.data[0] == pytest.approx(ref, rel=1e-14)
    empty = W.rand(legs, (5,), (0,), 3)  # no block can carry n=5
    assert empty.nblocks == 0
    c0 = oracle.tensordot_blockpair(empty, b, (1,), (1,))
    assert c0.nblocks == 0 and c0.data.size == 0


# ---------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(12))
def test_power_of_two_gauge_is_bitwise(seed):
    a, b, xa, xb = random_problem(seed + 50, "U1", rank_a=3, rank_b=3, ncon=2, max_sectors=3, max_dim=3)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    # scale contracted sector rho of the first contracted leg by 2^k in A, 2^-k in B
    q = a.charges[0, xa[0], :].copy() if a.nblocks else None
    if q is None:
        return
    a2, b2 = a.copy(), b.copy()
    for i in range(a2.nblocks):
        if np.array_equal(a2.charges[i, xa[0], :], q):
            a2.data[a2.offsets[i]:a2.offsets[i] + a2.block_sizes[i]] *= 8.0
    for j in range(b2.nblocks):
        if np.array_equal(b2.charges[j, xb[0], :], q):
            b2.data[b2.offsets[j]:b2.offsets[j] + b2.block_sizes[j]] *= 0.125
    got = oracle.tensordot_blockpair(a2, b2, xa, xb)
    assert np.array_equal(got.data, ref.data)


@pytest.mark.parametrize("seed", range(12))
def test_swap_operands_is_transpose(seed):
    a, b, xa, xb = random_problem(seed + 80, "U1xZ2", max_sectors=3, max_dim=3)
    ab = oracle.tensordot_blockpair(a, b, xa, xb)
    ba = oracle.tensordot_blockpair(b, a, xb, xa)
    nfa = a.rank - len(xa)
    nfb = b.rank - len(xb)
    perm = tuple(range(nfb, nfb + nfa)) + tuple(range(nfb))
    t = oracle.transpose(ba, perm)
    assert oracle.same_structure(t, ab)
    np.testing.assert_allclose(t.data, ab.data, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(12))
def test_fusion_invariance(seed):
    a, b, xa, xb = random_problem(seed + 120, "U1", rank_a=4, rank_b=3, ncon=2, max_sectors=3, max_dim=3,
                                  keep=0.8, drop_partner=True)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    fa = tuple(i for i in range(a.rank) if i not in xa)
    fb = tuple(i for i in range(b.rank) if i not in xb)
    # constituents of the fused contracted leg: union of both partners' tuples
    def cons(t, legs):
        out = {}
        for k in range(t.nblocks):
            key = tuple(tuple(int(v) for v in t.charges[k, x, :]) for x in legs)
            out[key] = tuple(int(t.shapes[k, x]) for x in legs)
        return out
    tmpl = {**cons(a, xa), **cons(b, xb)}
    A, ra = oracle.fuse_legs(a, (fa, xa), templates=[None, tmpl])
    B, rb = oracle.fuse_legs(b, (xb, fb), templates=[tmpl, None])
    C = oracle.tensordot_blockpair(A, B, (1,), (0,))
    back = oracle.unfuse_legs(C, [ra[0], rb[1]])
    idx = {tuple(back.charges[k].ravel()): k for k in range(back.nblocks)}
    seen = set()
    for k in range(ref.nblocks):
        kk = idx[tuple(ref.charges[k].ravel())]
        seen.add(kk)
        np.testing.assert_allclose(back.block(kk), ref.block(k), rtol=1e-13, atol=1e-13)
    for kk in range(back.nblocks):  # sub-blocks outside rule R are exactly zero
        if kk not in seen:
            assert not np.any(back.block(kk))


# ------------------------------------------------------------ validation
def _u1_d18():
    (p,) = W.u1_d18()
    return p.a, p.b


def test_validation_status_classes():
    a, b = _u1_d18()
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(a, b, (2, 3), (0,))
    assert e.value.status == oracle.ERR_ARG
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(a, b, (2, 2), (0, 1))
    assert e.value.status == oracle.ERR_ARG
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(a, b, (0, 1), (0, 1))  # (+,+) with (+,+)
    assert e.value.status == oracle.ERR_SIGNATURE
    bad = a.copy(); bad.charges[3, 0, 0] += 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(bad, b, (2, 3), (0, 1))
    assert e.value.status in (oracle.ERR_CHARGE, oracle.ERR_DUPLICATE)
    bad = a.copy(); bad.shapes[0, 0] = 0
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(bad, b, (2, 3), (0, 1))
    assert e.value.status == oracle.ERR_SHAPE
    bad = a.copy(); bad.charges[1] = bad.charges[0]; bad.shapes[1] = bad.shapes[0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(bad, b, (2, 3), (0, 1))
    assert e.value.status == oracle.ERR_DUPLICATE
    bad = b.copy(); bad.sym_mod = (2,)
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(a, bad, (2, 3), (0, 1))
    assert e.value.status == oracle.ERR_SYM
    # a contracted charge with a different dim in B
    legs = [W._u1_leg(s, [(-1, 2), (0, 3), (1, 2)]) for s in (1, -1)]
    x = W.rand(legs, (0,), (0,), 1)
    legs_b = [W._u1_leg(s, [(-1, 2), (0, 4), (1, 2)]) for s in (1, -1)]
    y = W.rand(legs_b, (0,), (0,), 2)
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(x, y, (1,), (0,))
    assert e.value.status == oracle.ERR_SHAPE
    # overlapping blocks in the buffer
    bad = a.copy(); bad.offsets[1] = bad.offsets[0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.validate_pair(bad, b, (2, 3), (0, 1))
    assert e.value.status == oracle.ERR_ARG


def test_z_m_charges_normalised():
    legs = [W.Leg(1, ((0,), (1,)), (2, 1)), W.Leg(-1, ((0,), (1,)), (2, 1))]
    a = W.rand(legs, (0,), (2,), 1)
    a2 = a.copy()
    a2.charges[:, :, 0] += 2 * np.array([[1, -3]] * a2.nblocks, dtype=np.int32)  # same classes mod 2
    c1 = oracle.tensordot_dense(a, a, (1,), (0,)) if False else None
    del c1
    b = W.rand([legs[1].conj(), legs[0]], (0,), (2,), 2)
    r1 = oracle.tensordot_blockpair(a, b, (1,), (0,))
    r2 = oracle.tensordot_blockpair(a2, b, (1,), (0,))
    assert oracle.same_structure(r1, r2) and np.array_equal(r1.data, r2.data)


@pytest.mark.parametrize("step", [0, 1, 2])
def test_sampled_blocks_equal_full_blockpair(step):
    """tensordot_blocks (O2 on chosen output blocks) gives exactly the blocks
    of the full O2 result: same pairs, same order."""
    import workloads as W
    t = W.ctm()
    steps = [("C", "T1"), (None, "T4"), (None, "A")]
    cur = None
    for i, ((an, bn), (ax, bx)) in enumerate(zip(steps, t["axes"])):
        a = t[an] if an else cur
        if i == step:
            full = oracle.tensordot_blockpair(a, t[bn], ax, bx)
            rng = np.random.default_rng(step)
            ids = sorted(set(rng.integers(0, full.nblocks, size=12).tolist()) | {0, full.nblocks - 1})
            s, blocks = oracle.tensordot_blocks(a, t[bn], ax, bx, ids)
            assert np.array_equal(s.charges, full.charges) and np.array_equal(s.offsets, full.offsets)
            for k in ids:
                assert np.array_equal(blocks[k], full.block(k))
            return
        cur = oracle.tensordot_blockpair(a, t[bn], ax, bx)


# ---------------------------------------------------------- transpose, gradient
def _inner(x, y):
    """Sum over the blocks the two tensors share (matched by charge tuple) of
    the elementwise products."""
    xn, yn = oracle.normalize(x), oracle.normalize(y)
    ky = {tuple(yn.charges[b].ravel().tolist()): b for b in range(yn.nblocks)}
    s = 0.0
    for b in range(xn.nblocks):
        k = tuple(xn.charges[b].ravel().tolist())
        if k in ky:
            s += float(np.sum(xn.block(b) * yn.block(ky[k])))
    return s


def _with_data(t, rng):
    out = t.copy()
    out.data = rng.standard_normal(int(t.block_sizes.sum()))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_transpose_equals_dense_transpose(seed):
    a, _, _, _ = random_problem(seed + 7100, ["U1", "Z2", "U1xU1"][seed % 3], rank_a=2 + seed % 3, rank_b=1,
                                max_sectors=3, max_dim=3, shuffle=True)
    perm = list(np.random.default_rng(seed).permutation(a.rank))
    t = oracle.transpose(a, perm)
    oracle.validate_tensor(t)
    da = oracle.to_dense(a, oracle.leg_index_maps(a))
    dt = oracle.to_dense(t, oracle.leg_index_maps(t))
    assert np.array_equal(np.transpose(da, perm), dt)


@pytest.mark.parametrize("wrt", [0, 1])
@pytest.mark.parametrize("seed", range(8))
def test_grad_adjoint_identity(seed, wrt):
    """<E, dA> = <dC, tensordot(E, B)> for any E with A's structure (and the
    same for B): the defining property of the gradient of a linear map,
    checked with the dense contraction (O1) on the right-hand side."""
    sym = ["U1", "Z2", "U1xZ2", "Z3"][seed % 4]
    a, b, xa, xb = random_problem(seed + 7200, sym, rank_a=1 + seed % 4, rank_b=1 + (seed // 2) % 4,
                                  max_sectors=3, max_dim=3, shuffle=seed % 2 == 0)
    rng = np.random.default_rng(seed)
    dc = _with_data(oracle.tensordot_dense(a, b, xa, xb), rng)
    g = oracle.tensordot_grad(a, b, xa, xb, dc, wrt)
    op = a if wrt == 0 else b
    oracle.validate_tensor(g)
    assert g.rank == op.rank and list(g.sig) == list(op.sig)
    assert list(g.n) == list(oracle.normalize(op).n)
    e = _with_data(op, rng)
    ce = oracle.tensordot_dense(e, b, xa, xb) if wrt == 0 else oracle.tensordot_dense(a, e, xa, xb)
    lhs, rhs = _inner(e, g), _inner(ce, dc)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs))


def test_grad_u1_d18_matches_matrix_form():
    """The D = 18 contraction (A's contracted legs trail, B's lead): the gradient is the
    plain matrix product in each sector, dA = dC B^T, checked densely."""
    (p,) = W.u1_d18()
    rng = np.random.default_rng(1)
    c = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    dc = _with_data(c, rng)
    ga = oracle.tensordot_grad(p.a, p.b, p.axes_a, p.axes_b, dc, 0)
    ma = oracle.leg_index_maps(ga)
    dd = oracle.to_dense(dc, oracle.leg_index_maps(dc))
    db = oracle.to_dense(p.b, oracle.leg_index_maps(p.b))
    ref = np.tensordot(dd, db, axes=([2, 3], [2, 3]))
    assert np.allclose(oracle.to_dense(ga, ma), ref, rtol=0, atol=1e-12)
