"""yastn_contract_noalloc: the contraction with its workspace in the library's
fixed per-GPU scratch array (no device allocation), against yastn_contract
with a caller workspace on the same plan and inputs.

Two calls in a row, the second with a smaller problem, so the second runs on
what the first left in the scratch; each result must be bitwise the
workspace form's (same kernels, same summation order) and within 1e-12 of the
oracle (the sum over matched block pairs, Sec. II.B).  Plans whose workspace
exceeds the scratch are refused.
"""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts deselect -m gpu
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_12196_amd as Y  # noqa: E402
from tests import gpu_util as G  # noqa: E402


def _setup(probs, flags=0):
    pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b) for p in probs], flags=flags)
    A = [G.upload(p.a) for p in probs]
    B = [G.upload(p.b) for p in probs]
    return pl, A, B


def _outs(pl):
    return [torch.full((max(1, pl.output(i).numel),), float("nan"), dtype=torch.float64, device=G.DEV)
            for i in range(pl.nprob)]


def _check(pl, probs, A, B):
    """noalloc vs the workspace form (bitwise) and vs the oracle (1e-12)."""
    assert pl.workspace_bytes <= Y.SCRATCH_BYTES
    c_ws = _outs(pl)
    pl.contract(A, B, c_ws, G.workspace(pl))
    c_na = _outs(pl)
    pl.contract_noalloc(A, B, c_na)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        n = pl.output(i).numel
        assert torch.equal(c_na[i][:n], c_ws[i][:n]), f"problem {i}: noalloc differs from the workspace form"
    rng = np.random.default_rng(11)
    pick = sorted(set(rng.integers(0, len(probs), size=min(8, len(probs))).tolist()) | {0, len(probs) - 1})
    for i in pick:
        p = probs[i]
        ref = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
        s = pl.output(i)
        assert G.structure_equal(s, ref)
        err = oracle.rel_frobenius(c_na[i][:s.numel].cpu().numpy(), ref.data)
        assert err <= 1e-12, f"problem {i}: {err:.3e}"


def test_noalloc_two_calls_second_smaller():
    """64 uneven U(1) problems (packed B of ~41 MiB and the pipelined kernel in
    the scratch), then one D = 18 problem on the packed-B MFMA tiles."""
    big = W.u1_uneven()
    pl, A, B = _setup(big)
    assert pl.workspace_bytes > 32 << 20  # the scratch is really used
    print(f"noalloc call 1: {len(big)} problems, workspace {pl.workspace_bytes} bytes", flush=True)
    _check(pl, big, A, B)
    small = W.u1_d18(1)
    pl2, A2, B2 = _setup(small, flags=Y.FLAG_MFMA)
    assert 0 < pl2.workspace_bytes < pl.workspace_bytes
    print(f"noalloc call 2: 1 problem, workspace {pl2.workspace_bytes} bytes", flush=True)
    _check(pl2, small, A2, B2)


def test_noalloc_ctm_chain_steps():
    """The chi = 128 enlarged-corner steps, each through the scratch."""
    t = W.ctm()
    cur, cur_dev = None, None
    from bench import STEPS
    for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
        a = t[an] if an else cur
        a_dev = G.upload(t[an]) if an else cur_dev
        pl = Y.plan([(a, t[bn], ax, bx)])
        b_dev = G.upload(t[bn])
        (c,) = _outs(pl)
        pl.contract_noalloc([a_dev], [b_dev], [c])
        (cw,) = _outs(pl)
        pl.contract([a_dev], [b_dev], [cw], G.workspace(pl))
        torch.cuda.synchronize()
        n = pl.output(0).numel
        assert torch.equal(c[:n], cw[:n])
        cur, cur_dev = G.as_block_tensor(pl.output(0), c[:n].cpu().numpy()), c


def test_noalloc_refuses_plan_larger_than_scratch():
    probs = W.u1_d18(512)  # packed B of 512 x 17,712 FP64 elements: 72.6 MB
    pl, A, B = _setup(probs)
    assert pl.workspace_bytes > Y.SCRATCH_BYTES
    C = _outs(pl)
    with pytest.raises(Y.YastnError) as e:
        pl.contract_noalloc(A, B, C)
    assert e.value.status == "ERR_STATE"
