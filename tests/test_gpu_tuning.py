"""The tuning store on the device: a plan autotuned, the store saved to a
file, emptied with the structure cache, and loaded again: a new plan of the
same request starts at the saved variant (its autotune returns the saved
choice and times without timing again) and its results match the oracle."""

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


def _buffers(pl, probs):
    A = [G.upload(p.a) for p in probs]
    B = [G.upload(p.b) for p in probs]
    C = [G.alloc_out(pl, i)[0] for i in range(len(probs))]
    return A, B, C, G.workspace(pl)


def test_tuning_store_roundtrip(tmp_path):
    probs = W.u1_d18(8)
    desc = [(p.a, p.b, p.axes_a, p.axes_b) for p in probs]
    Y.tune_clear()
    Y.plan_cache_clear()
    pl = Y.plan(desc)
    A, B, C, ws = _buffers(pl, probs)
    v, times = pl.autotune(A, B, C, ws, reps=2)
    assert v >= 1
    path = tmp_path / "tuning.json"
    Y.tune_save(str(path))
    Y.tune_clear()
    Y.plan_cache_clear()
    assert Y.tune_load(str(path)) >= 1
    pl2 = Y.plan(desc)
    A2, B2, C2, ws2 = _buffers(pl2, probs)
    v2, times2 = pl2.autotune(A2, B2, C2, ws2, reps=2)
    assert v2 == v
    fits = [t for t in times if t >= 0]
    assert np.allclose([t for t in times2 if t >= 0], fits, rtol=1e-5, atol=0)  # the stored times
    pl2.contract(A2, B2, C2, ws2)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        ref = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
        got = C2[i].cpu().numpy()[:ref.data.size]
        assert np.max(np.abs(got - ref.data)) <= 1e-12 * np.max(np.abs(ref.data))
    # a different request is not matched: a new plan of it starts untuned
    other = [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_d18(2)]
    pl3 = Y.plan(other)
    A3, B3, C3, ws3 = _buffers(pl3, W.u1_d18(2))
    v3, times3 = pl3.autotune(A3, B3, C3, ws3, reps=1)
    assert v3 >= 1
    Y.tune_clear()
