"""Pins of the CTM left-move oracle (oracle/ctm.py).

None re-uses the oracle's axis tuples: every tensor of the move is
recomputed densely with numpy.einsum from the lattice picture (each bond one
index letter, written from the leg lists of ``workloads.ctm_env``), the
projectors are checked against what they must do (the identity on the
product of the halves when nothing is truncated, the best rank-chi
approximation of the four-corner product when something is: Eckart-Young),
and a one-element network against its closed form.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import ctm as OC
from oracle import svd as OS


def _space(pairs, sym_mod):
    dims = {tuple(int(v) % m if m else int(v) for v, m in zip(q, sym_mod)): int(d) for q, d in pairs}
    start, pos = {}, 0
    for q in sorted(dims):
        start[q] = pos
        pos += dims[q]
    return {"charges": sorted(dims), "dims": dims, "start": start, "D": pos}


def _dense_env(name):
    E, V, P, sm = W.CTM_SMALL[name]
    e, v, p = _space(E, sm), _space(V, sm), _space(P, sm)
    env = W.ctm_move_small(name)
    legs = {"C1": [e, e], "C2": [e, e], "C3": [e, e], "C4": [e, e], "T1": [e, v, v, e], "T2": [e, v, v, e],
            "T3": [e, v, v, e], "T4": [e, v, v, e], "A": [v, v, v, v, p], "Ac": [v, v, v, v, p]}
    dense = {k: oracle.to_dense(env[k], legs[k]) for k in legs}
    return env, dense, (e, v, p)


def _kspace(kept, sym_mod):
    return _space([(X, k) for X, k in kept.items() if k > 0], sym_mod)


def _dense_corners(d):
    def ein(spec, *ops):
        return np.einsum(spec, *ops, optimize=True)
    return {
        "Q1": ein("ac,ckbR,aqwB,kqXYp,bwZVp->RBXYZV", d["C1"], d["T1"], d["T4"], d["A"], d["Ac"]),
        "Q2": ein("ca,aqwB,Lkbc,kXYqp,bZVwp->BLXYZV", d["C2"], d["T2"], d["T1"], d["A"], d["Ac"]),
        "Q3": ein("ac,Lkbc,Tqwa,XYkqp,ZVbwp->LTXYZV", d["C3"], d["T3"], d["T2"], d["A"], d["Ac"]),
        "Q4": ein("ac,Tqwa,ckbR,XqkYp,ZwbVp->TRXYZV", d["C4"], d["T4"], d["T3"], d["A"], d["Ac"]),
    }


CASES = ["u1", "z2", "u1xu1", "u1_mid"]


@pytest.fixture(scope="module", params=CASES)
def move(request):
    env, dense, spaces = _dense_env(request.param)
    chi = env["chi"]
    full = OC.left_move(env, 10 ** 6)            # nothing truncated
    trunc = OC.left_move(env, max(1, chi - 2))   # a few values dropped
    return request.param, env, dense, spaces, full, trunc


def _close(a, b, rel=1e-12):
    scale = max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    assert a.shape == b.shape
    assert float(np.max(np.abs(a - b))) <= rel * scale if a.size else True


def test_enlarged_corners_and_halves_match_the_dense_network(move):
    name, env, d, (e, v, p), full, _ = move
    q = _dense_corners(d)
    maps6 = [e, e, v, v, v, v]
    for k in ("Q1", "Q2", "Q3", "Q4"):
        _close(oracle.to_dense(full[k], maps6), q[k])
    rup = np.einsum("pijqkr,istjuk->pqrstu", q["Q2"], q["Q1"], optimize=True)
    rdn = np.einsum("ipqjrk,sitjuk->pqrstu", q["Q3"], q["Q4"], optimize=True)
    m = np.einsum("abcijk,defijk->abcdef", rup, rdn, optimize=True)
    maps = [e, v, v, e, v, v]
    _close(oracle.to_dense(full["Rup"], maps), rup)
    _close(oracle.to_dense(full["Rdn"], maps), rdn)
    _close(oracle.to_dense(full["M"], maps), m, 1e-11)


def _mat(x):
    s = x.shape
    return x.reshape(int(np.prod(s[:3])), -1)


def _dense_projectors(r, e, v, sym_mod):
    ks = _kspace(r["kept"], sym_mod)
    pup = oracle.to_dense(r["Pup"], [e, v, v, ks])
    pdn = oracle.to_dense(r["Pdn"], [e, v, v, ks])
    return pup, pdn, ks


def test_untruncated_projectors_keep_every_value_above_the_floor(move):
    """chi unbounded: every value of every sector is kept, and the projectors
    are the identity on the product of the halves,
    R_up (P_up P_dn^T) R_dn^T = M.  The four-corner product's spectrum spans
    7-10 decades here and the projectors divide by the smallest kept value,
    so the identity is checked with a floor (tol = 1e-5: values at or below
    1e-5 of the largest dropped): it then misses M by exactly the dropped
    values' root sum of squares (and by rounding of order 1e-16 x 1e5)."""
    name, env, d, (e, v, p), full, _ = move
    nsv = sum(min(Mx.shape) for Mx, _, _ in OS.sector_matrices(full["M"], OC.M_ROWS).values())
    assert sum(full["kept"].values()) == nsv
    floored = OC.left_move(env, 10 ** 6, tol=1e-5)
    maps = [e, v, v, e, v, v]
    rup, rdn, m = (_mat(oracle.to_dense(floored[k], maps)) for k in ("Rup", "Rdn", "M"))
    sv = np.linalg.svd(m, compute_uv=False)
    assert np.all(sv[nsv:] <= 1e-12 * sv[0])
    kept = sum(floored["kept"].values())
    assert kept == int(np.count_nonzero(sv > 1e-5 * sv[0]))
    pup, pdn, _ = _dense_projectors(floored, e, v, env["A"].sym_mod)
    got = rup @ _mat(pup) @ _mat(pdn).T @ rdn.T
    miss = np.linalg.norm(got - m)
    assert abs(miss - np.sqrt(np.sum(sv[kept:] ** 2))) <= 1e-9 * sv[0]


def test_truncated_projectors_give_the_best_rank_chi_approximation(move):
    """Eckart-Young: R_up P_up P_dn^T R_dn^T has the chi largest singular
    values of M and misses M by the root sum of squares of the others."""
    name, env, d, (e, v, p), _, trunc = move
    maps = [e, v, v, e, v, v]
    rup, rdn, m = (_mat(oracle.to_dense(trunc[k], maps)) for k in ("Rup", "Rdn", "M"))
    pup, pdn, _ = _dense_projectors(trunc, e, v, env["A"].sym_mod)
    approx = rup @ _mat(pup) @ _mat(pdn).T @ rdn.T
    sv = np.linalg.svd(m, compute_uv=False)
    kept = sum(trunc["kept"].values())
    assert 0 < kept <= env["chi"] - 2
    got = np.linalg.svd(approx, compute_uv=False)
    assert np.allclose(got[:kept], sv[:kept], rtol=1e-9, atol=1e-9 * sv[0])
    assert np.all(got[kept:] <= 1e-9 * sv[0])
    miss = np.linalg.norm(m - approx)
    assert abs(miss - np.sqrt(np.sum(sv[kept:] ** 2))) <= 1e-9 * sv[0]


def test_renormalised_tensors_match_the_dense_network(move):
    """C1', T4', C4' from the projectors (the oracle's own, embedded densely)
    and the dense environment, each written from the lattice picture; the new
    tensors have the old ones' legs and signatures."""
    name, env, d, (e, v, p), _, r = move
    pup, pdn, ks = _dense_projectors(r, e, v, env["A"].sym_mod)
    c1t1 = np.einsum("ac,ckbR->akbR", d["C1"], d["T1"], optimize=True)
    t4aa = np.einsum("tqwB,XqYZp,xwyzp->tBXYZxyz", d["T4"], d["A"], d["Ac"], optimize=True)
    c4t3 = np.einsum("ac,ckbR->akbR", d["C4"], d["T3"], optimize=True)
    c1n = np.einsum("akbx,akbR->xR", pup, c1t1, optimize=True)
    t4n = np.einsum("tXxk,tBXYZxyz,BYyl->kZzl", pdn, t4aa, pup, optimize=True)
    c4n = np.einsum("akbx,akbR->xR", pdn, c4t3, optimize=True)
    _close(oracle.to_dense(r["C1n"], [ks, e]), c1n, 1e-10)
    _close(oracle.to_dense(r["T4n"], [ks, v, v, ks]), t4n, 1e-10)
    _close(oracle.to_dense(r["C4n"], [ks, e]), c4n, 1e-10)
    for k, ref in (("C1n", "C1"), ("T4n", "T4"), ("C4n", "C4")):
        assert r[k].sig.tolist() == env[ref].sig.tolist()
        assert r[k].n.tolist() == env[ref].n.tolist()


def test_renormalisation_divides_by_the_largest_entry(move):
    _, _, _, _, _, r = move
    for k in ("C1n", "T4n", "C4n"):
        a, b = r[k].data, r[k + "_norm"].data
        mx = float(np.max(np.abs(a)))
        assert float(np.max(np.abs(b))) == pytest.approx(1.0, abs=1e-15)
        assert np.allclose(b * mx, a, rtol=1e-15, atol=1e-15 * mx)


def test_one_element_network_closed_form():
    """Every leg one charge of dim 1: every tensor is a number.  With
    q_i the corners' values, M = q1 q2 q3 q4, S = |M|, U = +1 (the gauge),
    V^T = sign(M), so P_up = q3 q4 sign(M) / sqrt|M|, P_dn = q1 q2 / sqrt|M|,
    C1' = P_up c1 t1, C4' = P_dn c4 t3 and T4' = t4 a^2 (the projectors
    cancel exactly)."""
    one = [((0,), 1)]
    env = W.ctm_env(one, one, one, (W.U1,), tuple(range(31, 40)))
    x = {k: float(env[k].data[0]) for k in W.ENV_NAMES}
    r = OC.left_move(env, 1)
    a = x["A"]
    q1 = x["C1"] * x["T1"] * x["T4"] * a * a
    q2 = x["C2"] * x["T2"] * x["T1"] * a * a
    q3 = x["C3"] * x["T3"] * x["T2"] * a * a
    q4 = x["C4"] * x["T4"] * x["T3"] * a * a
    m = q1 * q2 * q3 * q4
    assert float(r["M"].data[0]) == pytest.approx(m, rel=1e-14)
    assert float(r["U"].data[0]) == 1.0 and float(r["Vt"].data[0]) == np.sign(m)
    pup = q3 * q4 * np.sign(m) / np.sqrt(abs(m))
    pdn = q1 * q2 / np.sqrt(abs(m))
    assert float(r["Pup"].data[0]) == pytest.approx(pup, rel=1e-14)
    assert float(r["Pdn"].data[0]) == pytest.approx(pdn, rel=1e-14)
    assert float(r["C1n"].data[0]) == pytest.approx(pup * x["C1"] * x["T1"], rel=1e-14)
    assert float(r["C4n"].data[0]) == pytest.approx(pdn * x["C4"] * x["T3"], rel=1e-14)
    assert float(r["T4n"].data[0]) == pytest.approx(x["T4"] * a * a, rel=1e-13)
    assert float(r["T4n_norm"].data[0]) == np.sign(x["T4"])


def test_factors_follow_the_svd_gauge(move):
    """The move's U: in every sector, each kept column's entry of largest
    magnitude is positive (the gauge that makes the new tensors unique), and
    its columns are orthonormal."""
    _, _, _, _, _, r = move
    for X, (Ux, rl, cl) in OS.sector_matrices(r["U"], (0, 1, 2)).items():
        assert Ux.shape[1] == r["kept"][X]
        assert np.allclose(Ux.T @ Ux, np.eye(Ux.shape[1]), atol=1e-12)
        for k in range(Ux.shape[1]):
            col = np.abs(Ux[:, k])
            assert Ux[int(np.flatnonzero(col == col.max())[0]), k] > 0.0
