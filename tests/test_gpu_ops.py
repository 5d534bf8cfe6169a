"""Leg permutation and the reverse-mode gradient of a tensordot on an MI355X,
against the CPU oracle (structure bit for bit; a permutation moves values, so
they match exactly; gradients within 1e-12 relative Frobenius error in FP64).
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

import paper_2405_12196_amd as Y  # noqa: E402
from tests import gpu_util as G  # noqa: E402


def run_perm(t, perm, dtype=Y.DTYPE_F64):
    p = Y.Perm(t, perm)
    s = p.output()
    x = G.upload(t, dtype)
    y = torch.full((max(1, s.numel),), float("nan"), dtype=G.torch_dtype(dtype), device=G.DEV)
    p.permute(x, y, dtype)
    torch.cuda.synchronize()
    return s, y.cpu().numpy()[:s.numel].astype(np.float64)


@pytest.mark.parametrize("seed", range(12))
def test_permute_matches_oracle(seed):
    sym = ["U1", "Z2", "U1xU1", "Z3", "U1xZ2"][seed % 5]
    a, _, _, _ = random_problem(seed + 9100, sym, rank_a=1 + seed % 6, rank_b=1, max_sectors=4,
                                max_dim=5, shuffle=seed % 2 == 0, keep=0.8)
    perm = [int(v) for v in np.random.default_rng(seed).permutation(a.rank)]
    ref = oracle.transpose(a, perm)
    for dt in (Y.DTYPE_F64, Y.DTYPE_F32):
        s, v = run_perm(a, perm, dt)
        assert G.structure_equal(s, ref)
        want = ref.data if dt == Y.DTYPE_F64 else ref.data.astype(np.float32).astype(np.float64)
        assert np.array_equal(v, want)


def test_permute_ctm_intermediate():
    """The chi = 128 step-3 output (rank 7, 15,643 blocks): reverse its legs."""
    t = W.ctm()
    cur = None
    for (an, bn), (ax, bx) in zip([("C", "T1"), (None, "T4"), (None, "A")], t["axes"][:3]):
        cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
    perm = list(range(cur.rank))[::-1]
    s, v = run_perm(cur, perm)
    ref = oracle.transpose(cur, perm)
    assert G.structure_equal(s, ref) and np.array_equal(v, ref.data)


@pytest.mark.parametrize("perm", [[1, 3, 4, 5, 0, 2, 6], [4, 0, 5, 1, 2, 3, 6]])
def test_permute_ctm_blocks_gradient_order(perm):
    """The chi = 128 step-3 output with its contracted legs (b1, b4, p) moved
    behind the free ones (the leg order the last contraction's gradient
    produces), and back, in FP64 and FP32: large blocks whose output runs
    are strided in the input."""
    t = W.ctm()
    cur = None
    for (an, bn), (ax, bx) in zip([("C", "T1"), (None, "T4"), (None, "A")], t["axes"][:3]):
        cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
    ref = oracle.transpose(cur, perm)
    for dt in (Y.DTYPE_F64, Y.DTYPE_F32):
        s, v = run_perm(cur, perm, dt)
        want = ref.data if dt == Y.DTYPE_F64 else ref.data.astype(np.float32).astype(np.float64)
        assert G.structure_equal(s, ref) and np.array_equal(v, want)


@pytest.mark.parametrize("seed", range(6))
def test_permute_large_blocks(seed):
    """Large blocks (dims up to 70, dims of 1 anywhere) under random
    permutations, in FP64 and FP32."""
    from workloads import Leg
    rng = np.random.default_rng(seed + 77)
    while True:  # at most 4 M elements
        legs = []
        for _ in range(3 + seed % 3):
            d = [int(v) for v in rng.choice([1, 2, 5, 33, 70], size=2)]
            legs.append(Leg(int(rng.choice([1, -1])), ((0,), (1,)), tuple(d)))
        a = W.rand(legs, (0,), (2,), seed + 5)
        if a.data.size <= 4_000_000:
            break
    perm = [int(v) for v in rng.permutation(a.rank)]
    ref = oracle.transpose(a, perm)
    for dt in (Y.DTYPE_F64, Y.DTYPE_F32):
        s, v = run_perm(a, perm, dt)
        want = ref.data if dt == Y.DTYPE_F64 else ref.data.astype(np.float32).astype(np.float64)
        assert G.structure_equal(s, ref) and np.array_equal(v, want)


def test_permute_empty_and_bad_perm():
    a, _, _, _ = random_problem(9300, "U1", rank_a=3, rank_b=1)
    empty = a.copy()
    empty.charges, empty.shapes = a.charges[:0], a.shapes[:0]
    empty.offsets, empty.data = a.offsets[:0], a.data[:0]
    s, v = run_perm(empty, [2, 0, 1])
    assert s.nblocks == 0 and s.numel == 0
    with pytest.raises(Y.YastnError) as e:
        Y.Perm(a, [0, 0, 1])
    assert e.value.status == "ERR_ARG"


def run_grad(a, b, xa, xb, dc, wrt, precision="f64"):
    g = Y.Grad(a, b, xa, xb, wrt, precision=precision)
    s = g.output()
    other = b if wrt == 0 else a
    out = torch.full((max(1, s.numel),), float("nan"), dtype=G.torch_dtype(g.out_dtype), device=G.DEV)
    ws = torch.empty(max(256, g.workspace_bytes), dtype=torch.uint8, device=G.DEV)
    g.run(G.upload(dc, g.in_dtype), G.upload(other, g.in_dtype), out, ws)
    torch.cuda.synchronize()
    return s, out.cpu().numpy()[:s.numel].astype(np.float64)


def _dc(a, b, xa, xb, seed):
    c = oracle.output_structure(a, b, xa, xb)
    c.data = np.random.default_rng(seed).standard_normal(int(c.block_sizes.sum()))
    return c


@pytest.mark.parametrize("wrt", [0, 1])
@pytest.mark.parametrize("seed", range(10))
def test_grad_random_matches_oracle(seed, wrt):
    sym = ["U1", "Z2", "U1xZ2", "U1xU1", "Z3"][seed % 5]
    a, b, xa, xb = random_problem(seed + 9400, sym, rank_a=2 + seed % 4, rank_b=2 + (seed // 3) % 3,
                                  max_sectors=4, max_dim=6, keep=0.85, shuffle=seed % 3 == 0)
    dc = _dc(a, b, xa, xb, seed)
    ref = oracle.tensordot_grad(a, b, xa, xb, dc, wrt)
    s, v = run_grad(a, b, xa, xb, dc, wrt)
    assert G.structure_equal(s, ref)
    assert not np.any(np.isnan(v))
    assert oracle.rel_frobenius(v, ref.data) <= 1e-12


@pytest.mark.parametrize("wrt", [0, 1])
@pytest.mark.parametrize("step", [2, 3])
def test_grad_ctm_steps(step, wrt):
    """Corner steps 3 (A's contracted legs 0, 3) and 4 (0, 2, 6): gradients
    that need the permutation back to the operand's leg order."""
    t = W.ctm()
    cur = None
    steps = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]
    for i, ((an, bn), (ax, bx)) in enumerate(zip(steps, t["axes"])):
        a = t[an] if an else cur
        if i == step:
            dc = _dc(a, t[bn], ax, bx, step)
            ref = oracle.tensordot_grad(a, t[bn], ax, bx, dc, wrt)
            s, v = run_grad(a, t[bn], ax, bx, dc, wrt)
            assert G.structure_equal(s, ref)
            assert oracle.rel_frobenius(v, ref.data) <= 1e-12
            return
        cur = oracle.tensordot_blockpair(a, t[bn], ax, bx)


def test_grad_u1_d18_fp32():
    (p,) = W.u1_d18()
    dc = _dc(p.a, p.b, p.axes_a, p.axes_b, 5)
    ref = oracle.tensordot_grad(p.a, p.b, p.axes_a, p.axes_b, dc, 0)
    s, v = run_grad(p.a, p.b, p.axes_a, p.axes_b, dc, 0, precision="f32")
    assert G.structure_equal(s, ref)
    assert oracle.rel_frobenius(v, ref.data) <= 1e-6
