"""Parity of the HIP path with the CPU oracle (run on an MI355X).

Structure (block list, shapes, offsets, signature, total charge) must match
the oracle bit for bit; FP64 values within 1e-12 relative Frobenius error
(per output tensor, and 1e-11 relative per block); reduced precisions within
the tolerances stated in each test.  Every output element is pre-filled with
NaN, so an element the kernels fail to write shows up as NaN.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import random_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts deselect -m gpu
    pytest.skip("no GPU", allow_module_level=True)

from tests import gpu_util as G  # noqa: E402

TOL_F64 = 1e-12
TOL = {"f32": 1e-6, "bf16x3": 2e-5, "bf16x6": 1e-6}


def check_f64(s, vals, ref, tol=TOL_F64):
    assert G.structure_equal(s, ref), "structure differs from the oracle"
    assert not np.any(np.isnan(vals)), "unwritten output elements"
    err = oracle.rel_frobenius(vals, ref.data)
    assert err <= tol, f"relative Frobenius error {err:.3e}"
    for k in range(ref.nblocks):
        o, n = int(ref.offsets[k]), int(ref.block_sizes[k])
        r = ref.data[o:o + n]
        den = max(float(np.sqrt(np.sum(r * r))), 1e-300)
        assert float(np.sqrt(np.sum((vals[o:o + n] - r) ** 2))) / den <= 1e-11 or np.allclose(vals[o:o + n], r, atol=1e-14)
    return err


# ------------------------------------------------- rank-4 U(1), D = 18
def test_u1_d18_f64():
    (p,) = W.u1_d18()
    ref = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    pl, (s,), (v,) = G.run([(p.a, p.b, p.axes_a, p.axes_b)])
    check_f64(s, v, ref)
    st = pl.stats(0)
    assert (st["pairs"], st["sectors"], st["c_blocks"], st["c_numel"]) == (325, 9, 85, 17712)
    assert st["useful_flops"] == 2199168


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6"])
def test_paper_example_exact_all_precisions(prec):
    H = W.spin_half_pair_hamiltonian()
    ref = oracle.tensordot_blockpair(H, H, (2, 3), (0, 1))
    _, (s,), (v,) = G.run([(H, H, (2, 3), (0, 1))], precision=prec)
    assert G.structure_equal(s, ref)
    assert np.array_equal(v, ref.data)  # dyadic values: exact in every precision


# ------------------------------------------------------- random structures
FLAGS = {"auto": 0, "mfma": 1, "rows": 2}


@pytest.mark.parametrize("kind", list(FLAGS))
@pytest.mark.parametrize("seed", range(48))
def test_random_structures_f64(seed, kind):
    sym = ["U1", "Z2", "U1xZ2", "Z3", "U1xU1"][seed % 5]
    a, b, xa, xb = random_problem(seed + 2000, sym, rank_a=1 + seed % 5, rank_b=1 + (seed // 5) % 5,
                                  max_sectors=4, max_dim=5 + seed % 7, keep=0.75 if seed % 3 else None,
                                  shuffle=seed % 4 == 0, drop_partner=seed % 6 == 1)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    _, (s,), (v,) = G.run([(a, b, xa, xb)], flags=FLAGS[kind])
    check_f64(s, v, ref)


@pytest.mark.parametrize("seed", range(6))
def test_random_batch_one_launch(seed):
    probs = []
    for i in range(7):
        a, b, xa, xb = random_problem(seed * 100 + i + 4000, ["U1", "Z2", "U1xZ2"][i % 3],
                                      max_sectors=4, max_dim=6, keep=0.8)
        probs.append((a, b, xa, xb))
    _, S, V = G.run(probs)
    for (a, b, xa, xb), s, v in zip(probs, S, V):
        check_f64(s, v, oracle.tensordot_blockpair(a, b, xa, xb))


# ---------------------------------------------------------- edge cases
def _u1(s, pairs):
    return W.Leg(s, tuple((q,) for q, _ in pairs), tuple(d for _, d in pairs))


def test_large_k_several_chunks_and_tiles():
    # one big sector: K = 300 (> one 128-entry offset table), M, N > 64 (several tiles)
    l1 = _u1(1, [(0, 70), (1, 3)])
    l2 = _u1(1, [(0, 20), (1, 15)])
    a = W.rand([l1, l2, l2.conj()], (0,), (0,), 5)
    b = W.rand([l2, l2.conj(), _u1(-1, [(0, 90), (1, 2)])], (0,), (0,), 6)
    ref = oracle.tensordot_blockpair(a, b, (1, 2), (1, 0))
    _, (s,), (v,) = G.run([(a, b, (1, 2), (1, 0))])
    check_f64(s, v, ref)


def test_outer_product_and_full_contraction():
    l = _u1(1, [(-1, 3), (0, 5), (1, 2)])
    a = W.rand([l, l.conj()], (0,), (0,), 1)
    b = W.rand([l, l.conj(), l], (1,), (0,), 2)
    ref = oracle.tensordot_blockpair(a, b, (), ())          # no contracted legs
    _, (s,), (v,) = G.run([(a, b, (), ())])
    check_f64(s, v, ref)
    c = W.rand([l.conj(), l], (0,), (0,), 3)
    ref = oracle.tensordot_blockpair(a, c, (0, 1), (0, 1))  # rank-0 result
    _, (s,), (v,) = G.run([(a, c, (0, 1), (0, 1))])
    check_f64(s, v, ref)


def test_empty_inputs_and_no_matches():
    l = _u1(1, [(0, 2), (1, 3)])
    a = W.rand([l, l], (7,), (0,), 1)   # no block can carry n = 7: empty tensor
    b = W.rand([l.conj(), l], (0,), (0,), 2)
    _, (s,), (v,) = G.run([(a, b, (1,), (0,))])
    assert s.nblocks == 0 and s.numel == 0
    a = W.rand([l, _u1(1, [(5, 2)])], (5,), (0,), 3)  # contracted charges never shared
    b = W.rand([_u1(-1, [(4, 2)]), l], (-4,), (0,), 4)
    _, (s,), (v,) = G.run([(a, b, (1,), (0,))])
    assert s.nblocks == 0


def test_permuted_legs_and_gapped_buffers():
    a, b, xa, xb = random_problem(77, "U1xU1", rank_a=6, rank_b=4, ncon=3, max_sectors=3, max_dim=4,
                                  shuffle=True)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    _, (s,), (v,) = G.run([(a, b, xa, xb)])
    check_f64(s, v, ref)


# ------------------------------------------------ CTM enlarged corner
@pytest.mark.parametrize("kind", list(FLAGS))
def test_ctm_chain_f64(kind):
    t = W.ctm()
    steps = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]
    cur_ref, cur_gpu = None, None
    for (an, bn), (ax, bx) in zip(steps, t["axes"]):
        a_ref = t[an] if an else cur_ref
        ref = oracle.tensordot_blockpair(a_ref, t[bn], ax, bx)
        a_in = t[an] if an else cur_gpu
        _, (s,), (v,) = G.run([(a_in, t[bn], ax, bx)], flags=FLAGS[kind])
        check_f64(s, v, ref)
        cur_ref, cur_gpu = ref, G.as_block_tensor(s, v)


# ------------------------------------------- 64 uneven U(1) problems
def test_u1_uneven_batched_one_launch():
    probs = [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_uneven()]
    pl, S, V = G.run(probs)
    for (a, b, xa, xb), s, v in zip(probs, S, V):
        check_f64(s, v, oracle.tensordot_blockpair(a, b, xa, xb))
    assert sum(pl.stats(i)["sectors"] for i in range(len(probs))) == 664


def test_k_chunked_shared_b_fused_norm():
    """The K-chunked shared-B kernel's fused-norm instance on the D = 18
    contraction (K = 76: three chunks of 32, the last one partial): C and
    both norms against the oracle, and bitwise on a second run."""
    import paper_2405_12196_amd as Y
    (p,) = W.u1_d18()
    ref = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b)])
    pl.set_variant(CHUNK_VARIANT)
    A, B = G.upload(p.a), G.upload(p.b)
    c, s = G.alloc_out(pl, 0)
    ws = G.workspace(pl)
    got = []
    for _ in range(2):
        nout = torch.full((2,), float("nan"), dtype=torch.float64, device=G.DEV)
        pl.contract_norm([A], [B], [c], ws, nout)
        torch.cuda.synchronize()
        got.append(nout.cpu().numpy())
    check_f64(s, c.cpu().numpy()[:s.numel], ref)
    rf, rm = oracle.norms(ref)
    assert abs(got[0][0] - rf) <= 1e-13 * rf and abs(got[0][1] - rm) <= 1e-13 * rm
    assert np.array_equal(got[0], got[1])


def test_u1_uneven_k_chunked_shared_b():
    """The K-chunked shared-B kernel (variant 24) on the 64 uneven problems:
    K up to 404 (13 chunks of 32, the last one partial), N up to 404 (seven
    column ranges of a sector), every problem against the oracle."""
    import paper_2405_12196_amd as Y
    probs = [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_uneven()]
    pl = Y.plan(probs)
    pl.set_variant(CHUNK_VARIANT)
    assert max(pl.stats(i)["max_k"] for i in range(len(probs))) > 32 * 12
    A = [G.upload(a) for a, _, _, _ in probs]
    B = [G.upload(b) for _, b, _, _ in probs]
    outs = [G.alloc_out(pl, i) for i in range(len(probs))]
    pl.contract(A, B, [c for c, _ in outs], G.workspace(pl))
    torch.cuda.synchronize()
    for (a, b, xa, xb), (c, s) in zip(probs, outs):
        check_f64(s, c.cpu().numpy()[:s.numel], oracle.tensordot_blockpair(a, b, xa, xb))


# ------------------------------------------------------- reduced precision
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("in_f32", [True, False])
def test_reduced_precision_u1_d18(prec, in_f32):
    import paper_2405_12196_amd as Y
    (p,) = W.u1_d18()
    ref = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    _, (s,), (v,) = G.run([(p.a, p.b, p.axes_a, p.axes_b)], precision=prec,
                          in_dtype=Y.DTYPE_F32 if in_f32 else Y.DTYPE_F64, out_dtype=Y.DTYPE_F64)
    assert G.structure_equal(s, ref)
    err = oracle.rel_frobenius(v, ref.data)
    assert err <= TOL[prec], f"{prec}: {err:.3e}"


@pytest.mark.parametrize("kind", ["auto", "mfma"])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16x6"])
def test_reduced_precision_ctm_step3(prec, kind):
    t = W.ctm()
    a = oracle.tensordot_blockpair(oracle.tensordot_blockpair(t["C"], t["T1"], (1,), (0,)), t["T4"], (0,), (0,))
    ref = oracle.tensordot_blockpair(a, t["A"], (0, 3), (0, 1))
    _, (s,), (v,) = G.run([(a, t["A"], (0, 3), (0, 1))], precision=prec, flags=FLAGS[kind])
    assert G.structure_equal(s, ref)
    assert oracle.rel_frobenius(v, ref.data) <= TOL[prec]


@pytest.mark.parametrize("in_f32,out_f32", [(False, False), (True, False), (True, True)])
def test_fp32_shared_b_kernel(in_f32, out_f32):
    """FP32 arithmetic on the shared-B kernel (variant 22): the D = 18
    contraction and every corner step, each within the FP32 tolerance of the
    FP64 oracle; the fused norm of the last step against the oracle's."""
    import paper_2405_12196_amd as Y
    ind = Y.DTYPE_F32 if in_f32 else Y.DTYPE_F64
    outd = Y.DTYPE_F32 if out_f32 else Y.DTYPE_F64
    t = W.ctm()
    (p1,) = W.u1_d18()
    cases, cur = [(p1.a, p1.b, p1.axes_a, p1.axes_b)], None
    for (an, bn), (ax, bx) in zip([("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")], t["axes"]):
        a = t[an] if an else cur
        cases.append((a, t[bn], ax, bx))
        cur = oracle.tensordot_blockpair(a, t[bn], ax, bx)
    for i, (a, b, xa, xb) in enumerate(cases):
        ref = oracle.tensordot_blockpair(a, b, xa, xb)
        pl = Y.plan([(a, b, xa, xb)], precision="f32", in_dtype=ind, out_dtype=outd)
        pl.set_variant(22)
        A, B = G.upload(a, ind), G.upload(b, ind)
        c = torch.empty(max(1, pl.output(0).numel), dtype=torch.float32 if out_f32 else torch.float64, device=G.DEV)
        ws = G.workspace(pl)
        last = i == len(cases) - 1
        nout = torch.full((2,), float("nan"), dtype=torch.float64, device=G.DEV)
        if last:
            pl.contract_norm([A], [B], [c], ws, nout)
        else:
            pl.contract([A], [B], [c], ws)
        torch.cuda.synchronize()
        v = c.double().cpu().numpy()[:pl.output(0).numel]
        assert not np.any(np.isnan(v))
        err = oracle.rel_frobenius(v, ref.data)
        assert err <= TOL["f32"], f"case {i}: {err:.3e}"
        if last:
            rf, rm = oracle.norms(ref)
            got = nout.cpu().numpy()
            assert abs(got[0] - rf) <= TOL["f32"] * rf and abs(got[1] - rm) <= TOL["f32"] * rm


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("variant", [1, 8])
def test_bf16_tile_kinds_ctm_steps(prec, variant):
    """Split-BF16 with FP32 operand buffers: the packed-B tiles (variant 1)
    and the register-resident tiles (variant 8, K <= 64) on every corner
    step, each within the stated error of the FP64 oracle."""
    import paper_2405_12196_amd as Y
    t = W.ctm()
    cur = None
    for i, ((an, bn), (ax, bx)) in enumerate(zip([("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")], t["axes"])):
        a = t[an] if an else cur
        ref = oracle.tensordot_blockpair(a, t[bn], ax, bx)
        pl = Y.plan([(a, t[bn], ax, bx)], precision=prec, in_dtype=Y.DTYPE_F32, out_dtype=Y.DTYPE_F64)
        pl.set_variant(variant)
        A, B = G.upload(a, Y.DTYPE_F32), G.upload(t[bn], Y.DTYPE_F32)
        c, s = G.alloc_out(pl, 0)
        pl.contract([A], [B], [c], G.workspace(pl))
        torch.cuda.synchronize()
        v = c.cpu().numpy()[:s.numel]
        assert G.structure_equal(s, ref) and not np.any(np.isnan(v))
        err = oracle.rel_frobenius(v, ref.data)
        assert err <= TOL[prec], f"step {i + 1}: {err:.3e}"
        cur = ref


# ------------------------------------------------------------ invariants
@pytest.mark.parametrize("kind", ["mfma", "rows"])
def test_repeat_runs_bitwise_identical(kind):
    t = W.ctm()
    a = oracle.tensordot_blockpair(t["C"], t["T1"], (1,), (0,))
    _, _, (v1,) = G.run([(a, t["T4"], (0,), (0,))], flags=FLAGS[kind])
    _, _, (v2,) = G.run([(a, t["T4"], (0,), (0,))], repeat=3, flags=FLAGS[kind])
    assert np.array_equal(v1, v2)


def test_power_of_two_gauge_bitwise():
    (p,) = W.u1_d18()
    a, b = p.a.copy(), p.b.copy()
    for i in range(a.nblocks):  # contracted sector rho = 1 on A's leg 2 (and B's leg 0)
        if a.charges[i, 2, 0] == 1:
            a.data[a.offsets[i]:a.offsets[i] + a.block_sizes[i]] *= 4.0
    for j in range(b.nblocks):
        if b.charges[j, 0, 0] == 1:
            b.data[b.offsets[j]:b.offsets[j] + b.block_sizes[j]] *= 0.25
    _, _, (v0,) = G.run([(p.a, p.b, p.axes_a, p.axes_b)])
    _, _, (v1,) = G.run([(a, b, p.axes_a, p.axes_b)])
    assert np.array_equal(v0, v1)


def test_fusion_invariance_on_gpu():
    a, b, xa, xb = random_problem(321, "U1", rank_a=4, rank_b=3, ncon=2, max_sectors=3, max_dim=4, keep=0.8)
    fa = tuple(i for i in range(a.rank) if i not in xa)
    fb = tuple(i for i in range(b.rank) if i not in xb)

    def cons(t, legs):
        return {tuple(tuple(int(v) for v in t.charges[k, x, :]) for x in legs):
                tuple(int(t.shapes[k, x]) for x in legs) for k in range(t.nblocks)}
    tmpl = {**cons(a, xa), **cons(b, xb)}
    A, ra = oracle.fuse_legs(a, (fa, xa), templates=[None, tmpl])
    B, rb = oracle.fuse_legs(b, (xb, fb), templates=[tmpl, None])
    _, (s,), (v,) = G.run([(A, B, (1,), (0,))])
    back = oracle.unfuse_legs(G.as_block_tensor(s, v), [ra[0], rb[1]])
    _, (s2,), (v2,) = G.run([(a, b, xa, xb)])
    direct = G.as_block_tensor(s2, v2)
    idx = {tuple(back.charges[k].ravel()): k for k in range(back.nblocks)}
    for k in range(direct.nblocks):
        kk = idx[tuple(direct.charges[k].ravel())]
        np.testing.assert_allclose(back.block(kk), direct.block(k), rtol=1e-12, atol=1e-13)


def test_multi_plan_launch_equals_separate():
    import paper_2405_12196_amd as Y
    probs = [random_problem(900 + i, ["U1", "Z2", "U1xU1"][i], max_sectors=4, max_dim=6) for i in range(3)]
    sep = [G.run([p])[2][0] for p in probs]
    plans = [Y.plan([p]) for p in probs]
    jobs, outs = [], []
    for pl, (a, b, _, _) in zip(plans, probs):
        c, o = G.alloc_out(pl, 0)
        jobs.append((pl, [G.upload(a)], [G.upload(b)], [c], G.workspace(pl)))
        outs.append((c, o))
    Y.contract_jobs(jobs)
    torch.cuda.synchronize()
    for (c, o), v in zip(outs, sep):
        assert np.array_equal(c.cpu().numpy()[:o.numel], v)


def test_multi_plan_launch_with_pointer_table_plan():
    """A merged launch list holding a plan of 70 problems (its pointers go
    through the workspace table, in a launch of its own) between two small
    plans: every problem of every plan against the oracle."""
    import paper_2405_12196_amd as Y
    small = [random_problem(950 + i, ["U1", "Z2"][i], max_sectors=4, max_dim=6) for i in range(2)]
    big = [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_d18(70)]
    groups = [[small[0]], big, [small[1]]]
    jobs, outs = [], []
    for probs in groups:
        pl = Y.plan(probs)
        cs = [G.alloc_out(pl, i) for i in range(len(probs))]
        jobs.append((pl, [G.upload(p[0]) for p in probs], [G.upload(p[1]) for p in probs], [c for c, _ in cs],
                     G.workspace(pl)))
        outs.append((probs, cs))
    Y.contract_jobs(jobs)
    torch.cuda.synchronize()
    for probs, cs in outs:
        for (a, b, xa, xb), (c, s) in zip(probs, cs):
            check_f64(s, c.cpu().numpy()[:s.numel], oracle.tensordot_blockpair(a, b, xa, xb))


# ----------------------------------------------------------------- norms
@pytest.mark.parametrize("n", [0, 1, 1000, 3994616])
def test_norm_f64(n):
    import paper_2405_12196_amd as Y
    x = np.random.default_rng(n).standard_normal(max(n, 1))[:n]
    xd = torch.from_numpy(x.copy() if n else np.zeros(1)).to(G.DEV)
    out = torch.zeros(2, dtype=torch.float64, device=G.DEV)
    ws = torch.empty(Y.norm_workspace_bytes(), dtype=torch.uint8, device=G.DEV)
    Y.norm(xd, n, out, ws)
    torch.cuda.synchronize()
    fro, mx = out.cpu().numpy()
    t = W.BlockTensor((0,), np.zeros(1, np.int8), np.zeros(1, np.int32), np.zeros((1, 1, 1), np.int32),
                      np.array([[max(n, 1)]], np.int64), np.zeros(1, np.int64), x if n else np.zeros(1))
    rf, rm = oracle.norms(t) if n else (0.0, 0.0)
    assert abs(fro - rf) <= 1e-13 * max(rf, 1.0)
    assert mx == rm


# ------------------------------------------------------ kernel variants
NUM_VARIANTS = 25  # yastn.h YASTN_NUM_VARIANTS
PAIR_VARIANT = 23  # paired-row loads: only plans whose A rows allow them
CHUNK_VARIANT = 24  # K in chunks through LDS: any K, tiles of at most 32 rows


@pytest.mark.parametrize("variant", range(1, NUM_VARIANTS))
@pytest.mark.parametrize("seed", range(10))
def test_every_variant_matches_oracle(seed, variant):
    import paper_2405_12196_amd as Y
    sym = ["U1", "Z2", "U1xZ2", "U1xU1", "Z3"][seed % 5]
    a, b, xa, xb = random_problem(seed + 5100, sym, rank_a=2 + seed % 4, rank_b=2 + (seed // 4) % 3,
                                  max_sectors=4, max_dim=6 + seed % 5, keep=0.8, shuffle=seed % 3 == 0)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    pl = Y.plan([(a, b, xa, xb)])
    try:
        pl.set_variant(variant)
    except Y.YastnError as e:
        if variant == PAIR_VARIANT:  # needs K <= 40 and A rows in even contiguous runs
            assert e.status == "ERR_STATE"
            return
        assert variant != CHUNK_VARIANT, "the K-chunked kernel fits every small plan"
        # the row kernel needs K, N <= 64, the register-resident B kernels
        # K <= 64 (variant 16 and the shared-B variants 20-22: K <= 80)
        assert e.status == "ERR_STATE" and variant >= 7 and not 17 <= variant <= 19
        limit = 80 if variant == 16 or variant >= 20 else 64
        assert max(pl.stats(0)["max_k"], pl.stats(0)["max_n"] if variant == 7 else 0) > limit
        return
    A, B = G.upload(a), G.upload(b)
    c, s = G.alloc_out(pl, 0)
    pl.contract([A], [B], [c], G.workspace(pl))
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)


@pytest.mark.parametrize("variant", [20, 21, 22])
def test_shared_b_kernel_interleaved_legs_in_one_batch(variant):
    """The shared-B kernel on a batch mixing rank-7 operands with contracted
    legs spread out (up to four free-leg classes of A), Z2 and U(1)xU(1)
    problems and the D = 18 contraction, in one launch: every problem
    against the oracle."""
    import paper_2405_12196_amd as Y
    probs = [random_problem(seed, sym, rank_a=7, rank_b=4, ncon=3, max_sectors=2, max_dim=3)
             for sym, seed in [("Z2", 7100), ("Z2", 7103), ("Z2", 7105), ("Z2", 7108), ("Z3", 7103), ("Z3", 7107)]]
    probs += [random_problem(seed + 7200, sym, rank_a=4, rank_b=3, ncon=2, max_sectors=3, max_dim=5, keep=0.7)
              for seed, sym in enumerate(["Z2", "U1xU1", "U1xZ2"])]
    c1 = W.u1_d18(2)
    probs += [(p.a, p.b, p.axes_a, p.axes_b) for p in c1]
    pl = Y.plan(probs)
    if max(pl.stats(i)["max_k"] for i in range(len(probs))) > 80:
        pytest.skip("a sector with K > 80 (the kernel's limit)")
    pl.set_variant(variant)
    A = [G.upload(p[0]) for p in probs]
    B = [G.upload(p[1]) for p in probs]
    outs = [G.alloc_out(pl, i) for i in range(len(probs))]
    pl.contract(A, B, [c for c, _ in outs], G.workspace(pl))
    torch.cuda.synchronize()
    for (a, b, xa, xb), (c, s) in zip(probs, outs):
        check_f64(s, c.cpu().numpy()[:s.numel], oracle.tensordot_blockpair(a, b, xa, xb))


@pytest.mark.parametrize("variant", range(0, NUM_VARIANTS))
def test_u1_d18_every_variant(variant):
    """The D = 18 contraction (K = 76 in its largest sector): every variant that fits,
    including the occupancy-1 register-resident tiles that take K <= 80."""
    import paper_2405_12196_amd as Y
    (p,) = W.u1_d18()
    ref = oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b)
    pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b)])
    if variant:
        try:
            pl.set_variant(variant)
        except Y.YastnError as e:
            assert e.status == "ERR_STATE" and (7 <= variant <= 15 or variant == PAIR_VARIANT)
            return
    A, B = G.upload(p.a), G.upload(p.b)
    c, s = G.alloc_out(pl, 0)
    pl.contract([A], [B], [c], G.workspace(pl))
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)


@pytest.mark.parametrize("variant", range(0, NUM_VARIANTS))
def test_missing_a_blocks_every_variant(variant):
    """The D = 18 contraction with every fifth A block absent (lazy storage): rows of a
    sector then lack A data for part of its k range, which must count as
    zeros in every kernel."""
    import paper_2405_12196_amd as Y
    from workloads import BlockTensor
    (p,) = W.u1_d18()
    keep = np.arange(p.a.nblocks) % 5 != 2
    a = BlockTensor(p.a.sym_mod, p.a.sig, p.a.n, p.a.charges[keep], p.a.shapes[keep], p.a.offsets[keep], p.a.data)
    ref = oracle.tensordot_dense(a, p.b, p.axes_a, p.axes_b)
    pl = Y.plan([(a, p.b, p.axes_a, p.axes_b)])
    if variant:
        try:
            pl.set_variant(variant)
        except Y.YastnError as e:
            assert e.status == "ERR_STATE" and (7 <= variant <= 15 or variant == PAIR_VARIANT)
            return
    A, B = G.upload(a), G.upload(p.b)
    c, s = G.alloc_out(pl, 0)
    pl.contract([A], [B], [c], G.workspace(pl))
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)


def test_autotune_ctm_step3_picks_a_correct_variant():
    import paper_2405_12196_amd as Y
    t = W.ctm()
    a = oracle.tensordot_blockpair(oracle.tensordot_blockpair(t["C"], t["T1"], (1,), (0,)), t["T4"], (0,), (0,))
    ref = oracle.tensordot_blockpair(a, t["A"], (0, 3), (0, 1))
    pl = Y.plan([(a, t["A"], (0, 3), (0, 1))])
    A, B = G.upload(a), G.upload(t["A"])
    c, s = G.alloc_out(pl, 0)
    ws = G.workspace(pl)
    v, times = pl.autotune([A], [B], [c], ws, reps=2)
    assert 1 <= v < Y.NUM_VARIANTS and times[v] > 0 and times[0] == min(x for x in times[1:] if x > 0)
    c.fill_(float("nan"))
    pl.contract([A], [B], [c], ws)
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)


# ------------------------------------------------------------ HIP graphs
@pytest.mark.parametrize("kind", ["auto", "mfma"])
def test_graph_replays_equal_eager_chain(kind):
    """The enlarged-corner chain (four contractions + FP64 norm) captured in one HIP
    graph: every replay, with eager work and synchronisations between
    replays, must reproduce the eager results bitwise."""
    import paper_2405_12196_amd as Y
    t = W.ctm()
    steps = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]
    plans, cur = [], None
    for (an, bn), (ax, bx) in zip(steps, t["axes"]):
        pl = Y.plan([(t[an] if an else cur, t[bn], ax, bx)], flags=FLAGS[kind])
        plans.append(pl)
        cur = pl.output(0)
    inp = {k: G.upload(t[k]) for k in ("C", "T1", "T4", "A", "Ac")}
    outs = [torch.full((max(1, pl.output(0).numel),), float("nan"), dtype=torch.float64, device=G.DEV) for pl in plans]
    wss = [G.workspace(pl) for pl in plans]
    nout = torch.zeros(2, dtype=torch.float64, device=G.DEV)

    def chain(st):
        for i, ((an, bn), pl) in enumerate(zip(steps, plans)):
            a = inp[an] if an else outs[i - 1]
            if i == len(steps) - 1:  # the last output's FP64 norm, fused into its contraction
                pl.contract_norm([a], [inp[bn]], [outs[i]], wss[i], nout, stream=st)
            else:
                pl.contract([a], [inp[bn]], [outs[i]], wss[i], stream=st)

    chain(int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    ref_norm = nout.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        chain(int(s.cuda_stream))
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        nout.zero_()
        junk = torch.randn(1 << 16, device=G.DEV, dtype=torch.float64).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), f"replay {rep} differs from the eager chain"
        assert torch.equal(nout, ref_norm)
        del junk


# ------------------------------------------------------------ fused norm
@pytest.mark.parametrize("kind", ["auto", "mfma", "rows", 8, 17, 20, 21, 22])
def test_fused_norm_matches_oracle_and_repeats_bitwise(kind):
    """The FP64 norm of the step-4 output, from the contraction's epilogue
    (register-resident, shared-B and pipelined kernels) or from the separate
    pass (other kernels); an int kind is a kernel variant."""
    import paper_2405_12196_amd as Y
    t = W.ctm()
    a = oracle.tensordot_blockpair(t["C"], t["T1"], (1,), (0,))
    a = oracle.tensordot_blockpair(a, t["T4"], (0,), (0,))
    a = oracle.tensordot_blockpair(a, t["A"], (0, 3), (0, 1))
    ref = oracle.tensordot_blockpair(a, t["Ac"], (0, 2, 6), (0, 1, 4))
    pl = Y.plan([(a, t["Ac"], (0, 2, 6), (0, 1, 4))], flags=FLAGS[kind] if isinstance(kind, str) else 0)
    if not isinstance(kind, str):
        pl.set_variant(kind)
    A, B = G.upload(a), G.upload(t["Ac"])
    c, s = G.alloc_out(pl, 0)
    ws = G.workspace(pl)
    nout = torch.full((2,), float("nan"), dtype=torch.float64, device=G.DEV)
    pl.contract_norm([A], [B], [c], ws, nout)
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)
    rf, rm = oracle.norms(ref)
    got = nout.cpu().numpy()
    # C itself differs from the oracle's by rounding: both norms to 1e-13 relative,
    # and the max is exactly the max of the library's own output
    assert abs(got[0] - rf) <= 1e-13 * rf and abs(got[1] - rm) <= 1e-13 * rm
    assert got[1] == float(c[:s.numel].abs().max())
    first = nout.clone()
    for _ in range(3):
        nout.fill_(float("nan"))
        pl.contract_norm([A], [B], [c], ws, nout)
    torch.cuda.synchronize()
    assert torch.equal(nout, first)


def test_fused_norm_empty_output():
    import paper_2405_12196_amd as Y
    l = _u1(1, [(0, 2), (1, 3)])
    a = W.rand([l, _u1(1, [(5, 2)])], (5,), (0,), 3)  # contracted charges never shared
    b = W.rand([_u1(-1, [(4, 2)]), l], (-4,), (0,), 4)
    xa, xb = (1,), (0,)
    pl = Y.plan([(a, b, xa, xb)])
    assert pl.output(0).numel == 0
    nout = torch.full((2,), float("nan"), dtype=torch.float64, device=G.DEV)
    c = torch.zeros(1, dtype=torch.float64, device=G.DEV)
    pl.contract_norm([G.upload(a)], [G.upload(b)], [c], G.workspace(pl), nout)
    torch.cuda.synchronize()
    assert nout.cpu().tolist() == [0.0, 0.0]


# ------------------------------------------------------------------ split-K
def _long_k_problem(seed):
    """A(i, k1, k2) . B(k1, k2, j), U(1): small M and N (i, j: 2 sectors of
    dims 4 and 3), K per sector up to 3 x 60 x 60 = 10,800 (split into k
    ranges, summed by the reduction kernel)."""
    from workloads import Leg, rand
    li = Leg(1, ((0,), (1,)), (4, 3))
    lk = Leg(1, ((-1,), (0,), (1,)), (60, 60, 60))
    lj = Leg(-1, ((0,), (1,)), (3, 4))
    a = rand([li, lk.conj(), lk.conj()], (0,), (0,), seed)
    b = rand([lk, lk, lj], (0,), (0,), seed + 1)
    return a, b, (1, 2), (0, 1)


@pytest.mark.parametrize("variant", [0, 17, 18, 19])
def test_split_k_long_sectors(variant):
    import paper_2405_12196_amd as Y
    a, b, xa, xb = _long_k_problem(77)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    pl = Y.plan([(a, b, xa, xb)])
    assert pl.stats(0)["max_k"] > 4096 and pl.stats(0)["tiles"] > pl.stats(0)["sectors"]
    if variant:
        pl.set_variant(variant)
    else:
        with pytest.raises(Y.YastnError) as e:
            pl.set_variant(8)  # no register-resident tiles for split sectors
        assert e.value.status == "ERR_STATE"
    A, B = G.upload(a), G.upload(b)
    c, s = G.alloc_out(pl, 0)
    ws = G.workspace(pl)
    for _ in range(2):  # partial slots are fully rewritten by every call
        pl.contract([A], [B], [c], ws)
    torch.cuda.synchronize()
    check_f64(s, c.cpu().numpy()[:s.numel], ref)


def test_split_k_fp32_and_norm():
    import paper_2405_12196_amd as Y
    a, b, xa, xb = _long_k_problem(78)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    _, (s,), (v,) = G.run([(a, b, xa, xb)], precision="f32", in_dtype=Y.DTYPE_F32, out_dtype=Y.DTYPE_F64)
    assert G.structure_equal(s, ref)
    assert oracle.rel_frobenius(v, ref.data) <= 1e-6
    pl = Y.plan([(a, b, xa, xb)])
    A, B = G.upload(a), G.upload(b)
    c, s = G.alloc_out(pl, 0)
    nout = torch.zeros(2, dtype=torch.float64, device=G.DEV)
    pl.contract_norm([A], [B], [c], G.workspace(pl), nout)
    torch.cuda.synchronize()
    rf, rm = oracle.norms(ref)
    assert abs(float(nout[0]) / rf - 1) <= 1e-13


@pytest.mark.parametrize("flags", ["mfma", "rows"])
def test_long_k_with_forced_kernel_family(flags):
    """A plan that forces a kernel family (packed-B MFMA tiles, or the row
    kernel request) is not split into k ranges (only the pipelined kernel
    writes partial slots): it contracts without error and matches the oracle."""
    import paper_2405_12196_amd as Y
    a, b, xa, xb = _long_k_problem(79)
    ref = oracle.tensordot_blockpair(a, b, xa, xb)
    f = Y.FLAG_MFMA if flags == "mfma" else Y.FLAG_ROWS
    pl, (s,), (v,) = G.run([(a, b, xa, xb)], flags=f)
    assert pl.stats(0)["max_k"] > 4096 and pl.stats(0)["tiles"] == pl.stats(0)["sectors"]
    check_f64(s, v, ref)


def test_long_k_wide_sector_not_split():
    """K > 4096 with an output sector of more than 16 64 x 64 tiles: computed
    without k ranges (no partial-slot workspace), still exact."""
    import paper_2405_12196_amd as Y
    from workloads import Leg, rand
    li = Leg(1, ((0,),), (300,))
    lk = Leg(1, ((-1,), (0,), (1,)), (50, 60, 50))
    lj = Leg(-1, ((0,),), (260,))
    a = rand([li, lk.conj(), lk.conj()], (0,), (0,), 81)
    b = rand([lk, lk, lj], (0,), (0,), 82)
    ref = oracle.tensordot_blockpair(a, b, (1, 2), (0, 1))
    pl, (s,), (v,) = G.run([(a, b, (1, 2), (0, 1))])
    st = pl.stats(0)
    assert st["max_k"] > 4096 and st["max_m"] * st["max_n"] > 64 * 64 * 16
    # packed B (K x N FP64) and the norm parts only: no partial slots
    assert pl.workspace_bytes < st["max_k"] * st["max_n"] * 8 + (1 << 20)
    check_f64(s, v, ref)


# ------------------------------------------------------------ structure cache
def test_structure_cache_handles_and_tuning():
    """An identical request returns a handle to the cached plan (same
    structure, same bits); FLAG_NOCACHE plans afresh; a handle's variant is
    its own; a tuned structure hands its choice to later handles at once."""
    import paper_2405_12196_amd as Y
    Y.plan_cache_clear()
    (p,) = W.u1_d18()
    prob = [(p.a, p.b, p.axes_a, p.axes_b)]
    pl1 = Y.plan(prob)
    ms1, c1 = pl1.profile()
    assert not c1 and len(ms1) == 4 and all(v >= 0 for v in ms1)
    pl2 = Y.plan(prob)
    assert pl2.profile()[1], "an identical request should hit the cache"
    pl3 = Y.plan(prob, flags=Y.FLAG_NOCACHE)
    assert not pl3.profile()[1]
    A, B = G.upload(p.a), G.upload(p.b)
    outs = []
    for pl in (pl1, pl2, pl3):
        c, s = G.alloc_out(pl, 0)
        pl.contract([A], [B], [c], G.workspace(pl))
        outs.append(c)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    # per-handle variants: setting one handle's leaves the other on the heuristic
    pl1.set_variant(1)
    c1_, _ = G.alloc_out(pl1, 0)
    c2_, _ = G.alloc_out(pl2, 0)
    pl1.contract([A], [B], [c1_], G.workspace(pl1))
    pl2.contract([A], [B], [c2_], G.workspace(pl2))
    torch.cuda.synchronize()
    ref = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
    for c in (c1_, c2_):
        assert oracle.rel_frobenius(c.cpu().numpy()[:ref.data.size], ref.data) <= TOL_F64
    # tuning: the first autotune times, a later handle gets the choice at once
    c, _ = G.alloc_out(pl2, 0)
    v, times = pl2.autotune([A], [B], [c], G.workspace(pl2), reps=2)
    pl4 = Y.plan(prob)
    v4, times4 = pl4.autotune([A], [B], [c], G.workspace(pl4), reps=2)
    assert v4 == v and times4 == times
    # a different structure misses
    (q,) = W.u1_d18(1)
    pl5 = Y.plan([(q.a, q.b, (2, 3), (0, 1))], precision="f32")
    assert not pl5.profile()[1]
    Y.plan_cache_clear()
    assert not Y.plan(prob).profile()[1]
