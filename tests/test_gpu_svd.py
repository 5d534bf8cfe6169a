"""Parity of the block-sparse truncated SVD (yastn_svd_*) with the oracle
(oracle/svd.py): every singular value of every sector within 1e-12 of the
largest, the kept counts exactly, the kept factors' structure bit for bit,
the truncated product U_X diag(S_X) V_X^T of every sector within 1e-11, and
orthonormal kept columns.  Singular vectors are unique up to sign (and
rotations inside a multiplet), so the vectors are compared through that
product, which the truncation rule keeps unique (it never splits a multiplet).
"""

import numpy as np
import pytest

import oracle
from oracle import svd as OS
import workloads as W
from tests.test_oracle_svd import CASES, _random_tensor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts deselect -m gpu
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_12196_amd as Y  # noqa: E402
from tests import gpu_util as G  # noqa: E402


def gpu_svd(t, rows, chi, tol=0.0, deg_tol=1e-10, pu=0.0, pv=0.0, flags=0):
    sv = Y.Svd(t, rows)
    if flags:
        sv.set_flags(flags)
    tdev = G.upload(t)
    ws = torch.empty(max(256, sv.workspace_bytes), dtype=torch.uint8, device=G.DEV)
    svals = torch.full((max(1, sv.nsv),), float("nan"), dtype=torch.float64, device=G.DEV)
    kept, sweeps = sv.run(tdev, svals, ws, chi, tol, deg_tol)
    us, vs = sv.output()
    u = torch.full((max(1, us.numel),), float("nan"), dtype=torch.float64, device=G.DEV)
    vt = torch.full((max(1, vs.numel),), float("nan"), dtype=torch.float64, device=G.DEV)
    sv.factors(u, vt, ws, pu=pu, pv=pv)
    torch.cuda.synchronize()
    return sv, svals.cpu().numpy()[:sv.nsv], kept, sweeps, (us, u.cpu().numpy()[:us.numel]), \
        (vs, vt.cpu().numpy()[:vs.numel])


def _blocks(s, vals):
    out = {}
    for b in range(s.nblocks):
        key = tuple(tuple(int(v) for v in s.charges[b, l]) for l in range(s.charges.shape[1]))
        o, sh = int(s.offsets[b]), tuple(int(x) for x in s.shapes[b])
        out[key] = vals[o:o + int(np.prod(sh))].reshape(sh)
    return out


def check_svd(t, rows, chi, tol=0.0, deg_tol=1e-10, tol_sv=1e-12, tol_rec=1e-11, flags=0):
    sv, svals, kept, sweeps, (us, u), (vs, vt) = gpu_svd(t, rows, chi, tol, deg_tol, flags=flags)
    mats = OS.sector_matrices(t, rows)
    dec = OS.svd_sectors(t, rows)
    assert [X for X, *_ in sv.sectors] == list(mats), "sector order differs from the oracle"
    smax = max(float(d[1][0]) for d in dec.values())
    # every singular value
    for (X, m, n, s0), (Xr, (M, rl, cl)) in zip(sv.sectors, mats.items()):
        assert (m, n) == M.shape
        ref = dec[X][1]
        got = svals[s0:s0 + min(m, n)]
        assert np.all(np.diff(got) <= 0), f"sector {X}: not descending"
        err = float(np.max(np.abs(got - ref)))
        assert err <= tol_sv * smax, f"sector {X}: singular values off by {err:.3e} (max {smax:.3e})"
    # kept counts: the oracle's rule on the oracle's values
    ref_kept = OS.truncation({X: d[1] for X, d in dec.items()}, chi, tol, deg_tol)
    assert kept == [ref_kept[X] for X in mats], "kept counts differ"
    # structure of the factors
    u_ref, S_ref, vt_ref, _ = OS.svd_truncated(t, rows, chi, tol, deg_tol)
    assert G.structure_equal(us, u_ref), "U structure differs"
    assert G.structure_equal(vs, vt_ref), "V^T structure differs"
    ub, vb = _blocks(us, u), _blocks(vs, vt)
    for k, (X, (M, rl, cl)) in enumerate(mats.items()):
        kx = kept[k]
        if kx == 0:
            continue
        Uk = np.concatenate([ub[tuple(key) + (X,)].reshape(-1, kx) for key, dims, o in rl], axis=0)
        Vk = np.concatenate([vb[(X,) + tuple(key)].reshape(kx, -1) for key, dims, o in cl], axis=1)
        s0 = sv.sectors[k][3]
        Sk = svals[s0:s0 + kx]
        U, s, Vt = dec[X]
        ref = (U[:, :kx] * s[:kx]) @ Vt[:kx]
        got = (Uk * Sk) @ Vk
        den = max(float(np.linalg.norm(ref)), 1e-300)
        assert float(np.linalg.norm(got - ref)) / den <= tol_rec, f"sector {X}: truncated product"
        assert np.allclose(Uk.T @ Uk, np.eye(kx), atol=tol_rec)
        assert np.allclose(Vk @ Vk.T, np.eye(kx), atol=tol_rec)
    # with the sign rule on both sides the factors themselves agree, where the
    # rule's margin (largest vs second-largest |u|) and the kept values' gaps
    # leave no room for rounding to decide differently
    if _margins_ok(dec, kept, list(mats)):
        compare_blocks(us, u, u_ref, 1e-9)
        compare_blocks(vs, vt, vt_ref, 1e-9)
    return sv, kept, sweeps


def _margins_ok(dec, kept, order):
    for k, X in enumerate(order):
        U, s, _ = dec[X]
        kx = kept[k]
        if kx == 0:
            continue
        if kx < s.size and (s[kx - 1] - s[kx]) <= 1e-6 * s[0]:
            return False
        if np.any(np.diff(s[:kx]) >= -1e-6 * s[0]):
            return False
        for j in range(kx):
            col = np.sort(np.abs(U[:, j]))[::-1]
            if col.size > 1 and col[0] - col[1] <= 1e-6 * col[0]:
                return False
    return True


def compare_blocks(s, vals, ref, tol):
    assert G.structure_equal(s, ref)
    if ref.data.size:
        err = float(np.max(np.abs(vals - ref.data)))
        assert err <= tol * max(1.0, float(np.max(np.abs(ref.data)))), f"factor values off by {err:.3e}"


@pytest.mark.parametrize("seed,sym,rank,rows,n", CASES)
def test_svd_small_random(seed, sym, rank, rows, n):
    t = _random_tensor(seed, sym, rank, n)
    total = sum(min(M.shape) for M, _, _ in OS.sector_matrices(t, rows).values())
    for chi in (0, 1, max(1, total // 2), total, total + 5):
        check_svd(t, rows, chi)


def test_svd_wide_and_tall_sectors_and_tol():
    """Sectors with fewer rows than columns (stored transposed) next to tall
    ones, several column blocks of 8 (dims up to 40), and a tol floor."""
    from workloads import Leg, rand
    l1 = Leg(1, ((-1,), (0,), (1,)), (3, 9, 2))
    l2 = Leg(1, ((0,), (1,)), (5, 4))
    l3 = Leg(-1, ((-1,), (0,), (1,), (2,)), (7, 11, 6, 3))
    t = rand([l1, l2, l3], (0,), (0,), 909)
    for rows in ((0, 1), (2,), (0,), (1, 2)):
        check_svd(t, rows, chi=17)
        check_svd(t, rows, chi=1000, tol=1e-2)


def test_svd_recover_v_wide_and_tall_sectors():
    """The formed-vector mode (QR of each sector, sweeps on R^T) on sectors
    stored transposed next to tall ones: values, kept counts and factors
    against the oracle, with and without a tol floor."""
    from workloads import Leg, rand
    l1 = Leg(1, ((-1,), (0,), (1,)), (3, 9, 2))
    l2 = Leg(1, ((0,), (1,)), (5, 4))
    l3 = Leg(-1, ((-1,), (0,), (1,), (2,)), (7, 11, 6, 3))
    t = rand([l1, l2, l3], (0,), (0,), 909)
    for rows in ((0, 1), (2,), (0,), (1, 2)):
        check_svd(t, rows, chi=17, flags=Y.SVD_RECOVER_V)
        check_svd(t, rows, chi=1000, tol=1e-2, flags=Y.SVD_RECOVER_V)


def _corner():
    """The chi = 128, D = 8 enlarged corner (the oracle's chain output)."""
    from bench import STEPS
    t = W.ctm()
    cur = None
    for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
        cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
    return cur


def test_svd_ctm_corner_chi128():
    """The chi = 128, D = 8 enlarged corner split as rows (r1, A_r, A*_r) x
    columns (bot4, A_b, A*_b): 51 sectors up to 924 x 924, truncated to
    chi = 128."""
    cur = _corner()
    dec = OS.svd_sectors(cur, (0, 3, 5))
    allv = np.sort(np.concatenate([d[1] for d in dec.values()]))[::-1]
    assert (allv[127] - allv[128]) / allv[127] > 1e-6  # a clean cut: the kept set is unique
    sv, kept, sweeps = check_svd(cur, (0, 3, 5), chi=128)
    assert sum(kept) == 128
    print(f"corner SVD: {sv.nsectors} sectors, {sv.nsv} values, {sweeps} sweeps", flush=True)


def test_svd_scaled_factors():
    """U's kept column t times S_t^pu and V^T's row t times S_t^pv (the CTM
    projectors take -1/2 and -1/2)."""
    from oracle import ctm as OC
    t = _random_tensor(4, "U1xU1", 4, None)
    rows = (0, 3)
    u_ref, S_ref, vt_ref, _ = OS.svd_truncated(t, rows, 12)
    dec = OS.svd_sectors(t, rows)
    for pu, pv in ((-0.5, -0.5), (1.0, 0.25)):
        sv, svals, kept, sweeps, (us, u), (vs, vt) = gpu_svd(t, rows, 12, pu=pu, pv=pv)
        assert _margins_ok(dec, kept, [X for X, *_ in sv.sectors])
        compare_blocks(us, u, OC.scale_new_leg(u_ref, S_ref, pu, u_ref.rank - 1), 1e-9)
        compare_blocks(vs, vt, OC.scale_new_leg(vt_ref, S_ref, pv, 0), 1e-9)


def test_svd_repeat_bitwise():
    """Two runs on the same input give the same bits (no atomics in the
    arithmetic, fixed reduction orders)."""
    t = _random_tensor(5, "U1", 5, None)
    a = gpu_svd(t, (4, 0), 10)
    b = gpu_svd(t, (4, 0), 10)
    assert np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert np.array_equal(a[4][1], b[4][1]) and np.array_equal(a[5][1], b[5][1])


def test_svd_recover_v_corner_chi128():
    """Right vectors recovered after the sweeps on the chi = 128 corner: the
    kept values lie far above eps s_max, so the mode is used (the sweeps run
    on R^T of a QR factorisation of each sector, fewer of them than the
    default mode's); the factors pass the oracle checks and the values and
    factors agree with the default mode's within rounding."""
    cur = _corner()
    base = gpu_svd(cur, (0, 3, 5), 128)
    sv, kept, sweeps = check_svd(cur, (0, 3, 5), chi=128, flags=Y.SVD_RECOVER_V)
    rec = gpu_svd(cur, (0, 3, 5), 128, flags=Y.SVD_RECOVER_V)
    assert rec[3] < base[3], f"no fewer sweeps with the QR preconditioning ({rec[3]} vs {base[3]})"
    smax = float(np.max(base[1]))
    assert float(np.max(np.abs(rec[1] - base[1]))) <= 1e-12 * smax
    assert rec[2] == base[2]
    for i in (4, 5):
        err = float(np.max(np.abs(rec[i][1] - base[i][1])))
        assert err <= 1e-9, f"factor {i - 4} off the default mode's by {err:.3e}"
    print(f"recovered mode: {rec[3]} sweeps (default {base[3]})", flush=True)


def test_svd_recover_v_tall_sector_without_qr():
    """Formed vectors on a sector taller than the QR panel step holds (1100 x
    40, plus a small one): the sweeps run on W itself and the right vectors
    are formed as W^T u / s; factors against the oracle."""
    from workloads import Leg, rand
    rows = Leg(1, ((0,), (1,)), (1100, 6))
    cols = Leg(-1, ((0,), (1,)), (40, 5))
    t = rand([rows, cols], (0,), (0,), 77)
    sv, kept, sweeps = check_svd(t, (0,), chi=30, flags=Y.SVD_RECOVER_V)
    assert sum(kept) == 30 and sweeps >= 1


def test_svd_recover_v_falls_back_on_small_kept_values():
    """One sector scaled by 1e-10 and every value kept: recovered right
    vectors there would carry ~1e-5 relative error, so the call runs again
    with accumulated rotations (more sweeps in total) and returns bitwise the
    default mode's result."""
    from oracle.blocksparse import normalize
    t = _random_tensor(4, "U1xU1", 4, None)
    rows = (0, 3)
    tn = normalize(t)
    sec = [OS._sector_of(tn, b, rows) for b in range(t.nblocks)]
    small = sorted(set(sec))[len(set(sec)) // 2]
    for b in range(t.nblocks):
        if sec[b] == small:
            o = int(t.offsets[b])
            t.data[o:o + int(np.prod(t.shapes[b]))] *= 1e-10
    dec = OS.svd_sectors(t, rows)
    allv = np.concatenate([d[1] for d in dec.values()])
    assert allv.min() < 1e-9 * allv.max()
    chi = int(allv.size)  # keep every value
    base = gpu_svd(t, rows, chi, deg_tol=0.0)
    assert sum(base[2]) == chi
    rec = gpu_svd(t, rows, chi, deg_tol=0.0, flags=Y.SVD_RECOVER_V)
    assert rec[3] > base[3], "no second pass"
    assert np.array_equal(rec[1], base[1]) and rec[2] == base[2]
    assert np.array_equal(rec[4][1], base[4][1]) and np.array_equal(rec[5][1], base[5][1])


def test_svd_set_flags_rejects_unknown():
    t = _random_tensor(2, "U1", 3, None)
    sv = Y.Svd(t, (0,))
    with pytest.raises(RuntimeError):
        sv.set_flags(2)
    sv.set_flags(0)
