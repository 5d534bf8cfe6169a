"""Parity of the complex128 tensordot (yastn_zplan_*) and the fermionic swap
gate (yastn_swap_*) with the oracle (oracle/fermionic.py).

Complex: structures bit for bit; values within 1e-12 of the output's largest
|entry| (FP64 MFMA on the real form, the same products as the complex ones,
summed in another order), for every conjugation of the operands, several
symmetries, a grouped multi-problem plan, and the enlarged-corner chain at
chi = 128 with complex tensors (A* = conj(A) as the last step's conjugated
B), autotuned as the benchmark runs it.  Swap gates: bitwise (negation is
exact) for FP64, FP32 and complex buffers, the negated counts against the
oracle's, and a swap gate on a complex contraction's output.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import fermionic as F

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts deselect -m gpu
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_12196_amd as Y  # noqa: E402
from tests import gpu_util as G  # noqa: E402
from tests.test_oracle_fermionic import CASES, _pair  # noqa: E402


def up(t):
    x = torch.from_numpy(np.ascontiguousarray(t.data))
    if x.numel() == 0:
        x = torch.zeros(1, dtype=x.dtype)
    return x.to(G.DEV)


def zrun(problems, conj=0, autotune=False):
    zp = Y.ZPlan(problems, conj=conj)
    A = [up(a) for a, _, _, _ in problems]
    B = [up(b) for _, b, _, _ in problems]
    outs = []
    for p in range(len(problems)):
        s = zp.output(p)
        outs.append((torch.full((max(1, s.numel),), complex("nan+nanj"), dtype=torch.complex128, device=G.DEV), s))
    ws = torch.empty(max(256, zp.workspace_bytes), dtype=torch.uint8, device=G.DEV)
    if autotune:
        zp.autotune(A, B, [c for c, _ in outs], ws, reps=2)
    zp.contract(A, B, [c for c, _ in outs], ws)
    torch.cuda.synchronize()
    return zp, [(s, c.cpu().numpy()[:s.numel]) for c, s in outs]


def check(s, vals, ref, tol=1e-12):
    assert G.structure_equal(s, ref), "structure differs from the oracle"
    if ref.data.size:
        assert np.all(np.isfinite(vals)), "unwritten elements"
        err = float(np.max(np.abs(vals - ref.data))) / float(np.max(np.abs(ref.data)))
        assert err <= tol, f"max error {err:.3e} of the largest |entry|"


@pytest.mark.parametrize("sym,kind,n", CASES)
@pytest.mark.parametrize("conj", [0, Y.CONJ_A, Y.CONJ_B, Y.CONJ_A | Y.CONJ_B])
def test_zcontract_small(sym, kind, n, conj):
    a, b = _pair(sym, kind, n, 71)
    # A (v, w, v*, w) . B (v, w*, v): with neither or both conjugated A's
    # v*, w meet B's v, w*; conjugating one operand flips its signatures, so
    # then A's v meets B's v
    ax, bx = ((2, 3), (0, 1)) if conj in (0, Y.CONJ_A | Y.CONJ_B) else ((0,), (0,))
    ca, cb = bool(conj & Y.CONJ_A), bool(conj & Y.CONJ_B)
    ref = F.tensordot_c(a, b, ax, bx, conj_a=ca, conj_b=cb)
    zp, [(s, vals)] = zrun([(a, b, ax, bx)], conj=conj)
    check(s, vals, ref)
    flops = oracle.structure_stats(F.conj(a) if ca else a, F.conj(b) if cb else b, ax, bx)["flops"]
    assert zp.stats(0)["useful_flops"] == 4 * flops


def test_zcontract_grouped_problems():
    probs = []
    for seed in (81, 83, 85):
        a, b = _pair((W.U1,), "u1", (0,), seed)
        probs.append((a, b, (2, 3), (0, 1)))
    a, b = _pair((W.U1,), "u1", (0,), 87)
    probs.append((a, b, (2,), (0,)))
    zp, got = zrun(probs)
    for (a, b, ax, bx), (s, vals) in zip(probs, got):
        check(s, vals, oracle.tensordot_blockpair(a, b, ax, bx))


def test_zcontract_ctm_chain_chi128_autotuned():
    """The enlarged-corner chain with complex tensors: C.T1, .T4, .A, .A*
    (the last as A with CONJ_B), each step's output in full."""
    t = W.complex_ctm()
    cur_ref, cur_dev, cur_s = None, None, None
    for i, ((an, bn), (ax, bx)) in enumerate(zip([("C", "T1"), (None, "T4"), (None, "A"), (None, "A")],
                                                 t["axes"])):
        conj = Y.CONJ_B if i == 3 else 0
        a_ref = t[an] if an else cur_ref
        ref = F.tensordot_c(a_ref, t[bn], ax, bx, conj_b=bool(conj))
        a_struct = t[an] if an else G.as_block_tensor(cur_s, np.zeros(1))
        zp = Y.ZPlan([(a_struct, t[bn], ax, bx)], conj=conj)
        s = zp.output(0)
        out = torch.full((max(1, s.numel),), complex("nan+nanj"), dtype=torch.complex128, device=G.DEV)
        ws = torch.empty(max(256, zp.workspace_bytes), dtype=torch.uint8, device=G.DEV)
        A = [up(t[an])] if an else [cur_dev]
        zp.autotune(A, [up(t[bn])], [out], ws, reps=2)
        zp.contract(A, [up(t[bn])], [out], ws)
        torch.cuda.synchronize()
        check(s, out.cpu().numpy()[:s.numel], ref)
        cur_ref, cur_dev, cur_s = ref, out, s
        print(f"complex step {i + 1}: {s.nblocks} blocks, {s.numel} elements", flush=True)


@pytest.mark.parametrize("sym,kind,n", CASES)
@pytest.mark.parametrize("legs1,legs2", [((0,), (1,)), ((0, 2), (3,)), ((1,), (2, 3))])
def test_swap_gate_bitwise(sym, kind, n, legs1, legs2):
    a, _ = _pair(sym, kind, n, 91)
    fer = W.FERMIONIC[tuple(sym)]
    ref = F.swap_gate(a, legs1, legs2, fer)
    sg = Y.SwapGate(a, legs1, legs2, fer)
    odd = [b for b in range(a.nblocks)
           if sum(F.parity(a.charges[b, i], fer) for i in legs1) % 2 and
           sum(F.parity(a.charges[b, j], fer) for j in legs2) % 2]
    assert sg.blocks == len(odd) and sg.elements == sum(int(np.prod(a.shapes[b])) for b in odd)
    # complex, FP64 (real part), FP32
    x = up(a)
    sg.apply(x, Y.DTYPE_C128)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy()[:a.data.size], ref.data)
    xr = torch.from_numpy(np.ascontiguousarray(a.data.real)).to(G.DEV)
    sg.apply(xr, Y.DTYPE_F64)
    xf = torch.from_numpy(np.ascontiguousarray(a.data.real.astype(np.float32))).to(G.DEV)
    sg.apply(xf, Y.DTYPE_F32)
    torch.cuda.synchronize()
    assert np.array_equal(xr.cpu().numpy(), ref.data.real)
    assert np.array_equal(xf.cpu().numpy(), ref.data.real.astype(np.float32))


def test_swap_gate_on_a_complex_contraction_output():
    a, b = _pair((W.U1, W.U1), "u1xu1", (0, 0), 95)
    zp, [(s, vals)] = zrun([(a, b, (2, 3), (0, 1))])
    c = G.as_block_tensor(s, np.zeros(1))
    sg = Y.SwapGate(c, (0,), (2,), (1, 1))
    x = torch.from_numpy(np.ascontiguousarray(vals)).to(G.DEV)
    sg.apply(x, Y.DTYPE_C128)
    torch.cuda.synchronize()
    ref = F.swap_gate(oracle.tensordot_blockpair(a, b, (2, 3), (0, 1)), (0,), (2,), (1, 1))
    check(s, x.cpu().numpy(), ref)
