"""Parity at the full workload sizes, in the launch configuration the benchmark
times (plans built and autotuned as there, the FP64 norm fused into the last
contraction, grouped launches over many problems, the serving loop).

The corner chains at chi = 128 and chi = 256 are compared element by element
with the oracle's chain (block-pair form), in FP64 and in the reduced
precisions; where an output is too large for the oracle in full (the serving
mix's largest runs) it computes sampled output blocks one by one (every
matched block pair of those blocks, Sec. II.B) from the GPU's own input of
that step.  The structure of every output is compared in full, bit for bit.
Properties that hold at any size cover the rest: every output element is
written (outputs are pre-filled with NaN) and the fused norm agrees with an
independent reduction.
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
from bench import STEPS, Chain  # noqa: E402
from tests import gpu_util as G  # noqa: E402

TOL_F64 = 1e-12
TOL = {"f32": 1e-6, "bf16x3": 2e-5, "bf16x6": 1e-6}


def sample_ids(s, n, seed):
    """n seeded block indices plus the smallest and the largest block."""
    sizes = np.prod(s.shapes, axis=1)
    rng = np.random.default_rng(seed)
    ids = set(rng.integers(0, s.nblocks, size=min(n, s.nblocks)).tolist())
    ids |= {int(np.argmin(sizes)), int(np.argmax(sizes))}
    return sorted(ids)


def check_sampled(a, b, ax, bx, s, vals, nsample, seed, tol=TOL_F64):
    """Structure in full, values on sampled blocks, against the oracle."""
    ids = sample_ids(s, nsample, seed)
    ref_s, blocks = oracle.tensordot_blocks(a, b, ax, bx, ids)
    assert G.structure_equal(s, ref_s), "structure differs from the oracle"
    worst = 0.0
    for k in ids:
        o = int(s.offsets[k])
        shp = tuple(int(x) for x in s.shapes[k])
        got = vals[o:o + int(np.prod(shp))].reshape(shp)
        err = oracle.rel_frobenius(got, blocks[k])
        assert err <= tol, f"block {k} {shp}: relative Frobenius error {err:.3e}"
        worst = max(worst, err)
    return worst


def all_written(x, n):
    return bool(torch.isfinite(x[:n]).all())


def test_headline_chain_autotuned_full_oracle():
    """chi = 128, D = 8: the timed chain, every element against the oracle."""
    t = W.ctm()
    ch = Chain(torch, Y, t)
    for o in ch.outs:
        o.fill_(float("nan"))
    ch.step(0)
    torch.cuda.synchronize()
    cur = None
    for i, ((an, bn), (ax, bx), pl, o) in enumerate(zip(STEPS, t["axes"], ch.plans, ch.outs)):
        cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
        s = pl.output(0)
        assert G.structure_equal(s, cur)
        vals = o[:s.numel].cpu().numpy()
        assert not np.any(np.isnan(vals))
        assert oracle.rel_frobenius(vals, cur.data) <= TOL_F64, f"step {i + 1}"
    assert abs(float(ch.nout[0]) / float(np.linalg.norm(cur.data)) - 1) <= 1e-13


@pytest.fixture(scope="module")
def chi256_oracle():
    """The oracle's chain at chi = 256, D = 10: every output of the four steps
    in full (block-pair form; the largest output has 69.2 M elements)."""
    t = W.ctm_chi256()
    refs, cur = [], None
    for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
        cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
        refs.append(cur)
    return t, refs


def _full_step_check(i, pl, out, ref, tol):
    s = pl.output(0)
    assert G.structure_equal(s, ref), f"step {i + 1}: structure differs from the oracle"
    assert all_written(out, s.numel), f"step {i + 1}: unwritten output elements"
    err = oracle.rel_frobenius(out[:s.numel].double().cpu().numpy(), ref.data)
    assert err <= tol, f"step {i + 1}: relative Frobenius error {err:.3e} > {tol:.0e}"
    return err


def test_chi256_D10_f64_full_oracle(chi256_oracle):
    """chi = 256, D = 10, FP64: the benchmark's autotuned chain, every element
    of every step against the oracle's chain, and the fused norm."""
    t, refs = chi256_oracle
    ch = Chain(torch, Y, t)
    for o in ch.outs:
        o.fill_(float("nan"))
    ch.step(0)
    torch.cuda.synchronize()
    for i, (pl, o, ref) in enumerate(zip(ch.plans, ch.outs, refs)):
        _full_step_check(i, pl, o, ref, TOL_F64)
    nrm = float(np.linalg.norm(refs[-1].data))
    assert abs(float(ch.nout[0]) / nrm - 1) <= 1e-13
    mx = float(np.abs(refs[-1].data).max())
    assert abs(float(ch.nout[1]) / mx - 1) <= TOL_F64
    assert float(ch.nout[1]) == float(ch.outs[-1][:ch.n_last].abs().max())


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16x6"])
def test_chi256_D10_reduced_precision_chain(chi256_oracle, prec):
    """The reduced-precision chains (FP32 intermediates, the last output and
    its norm in FP64) end to end: every step's output against the oracle's
    FP64 chain, within the precision's stated tolerance."""
    t, refs = chi256_oracle
    ch = Chain(torch, Y, t, prec=prec)
    for o in ch.outs:
        o.fill_(float("nan"))
    ch.step(0)
    torch.cuda.synchronize()
    for i, (pl, o, ref) in enumerate(zip(ch.plans, ch.outs, refs)):
        _full_step_check(i, pl, o, ref, TOL[prec])
    got = ch.outs[-1][:ch.n_last]
    assert abs(float(ch.nout[0]) / float(torch.linalg.vector_norm(got)) - 1) <= 1e-13


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16x6"])
def test_chi256_D10_reduced_precision_isolated_steps(chi256_oracle, prec):
    """Each step alone on the oracle's FP64 input of that step (rounded to
    FP32 for the operand buffers), against the oracle's output of that step."""
    t, refs = chi256_oracle
    for i, ((an, bn), (ax, bx)) in enumerate(zip(STEPS, t["axes"])):
        a = t[an] if an else refs[i - 1]
        last = i == len(STEPS) - 1
        pl = Y.plan([(a, t[bn], ax, bx)], precision=prec, in_dtype=Y.DTYPE_F32,
                    out_dtype=Y.DTYPE_F64 if last else Y.DTYPE_F32)
        c, _ = G.alloc_out(pl, 0)
        pl.contract([G.upload(a, Y.DTYPE_F32)], [G.upload(t[bn], Y.DTYPE_F32)], [c], G.workspace(pl))
        torch.cuda.synchronize()
        _full_step_check(i, pl, c, refs[i], TOL[prec])
        del pl, c
        torch.cuda.empty_cache()


def test_u1_d18_x4096_batch():
    """The benchmark's 4096-problem batch of the rank-4 U(1) D = 18 contraction
    in one grouped launch: the structure of all 4096 outputs against the
    oracle's, every element written, and 66 problems (64 seeded, the first and
    the last) in full against the oracle."""
    probs = W.u1_d18(4096)
    pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b) for p in probs])
    A = [G.upload(p.a) for p in probs]
    B = [G.upload(p.b) for p in probs]
    C = [G.alloc_out(pl, i)[0] for i in range(len(probs))]
    pl.contract(A, B, C, G.workspace(pl))
    torch.cuda.synchronize()
    ref_s = oracle.output_structure(probs[0].a, probs[0].b, probs[0].axes_a, probs[0].axes_b, with_data=False)
    for i in range(len(probs)):
        s = pl.output(i)
        assert G.structure_equal(s, ref_s), f"problem {i}: structure"
        assert all_written(C[i], s.numel), f"problem {i}: unwritten output elements"
    rng = np.random.default_rng(4096)
    pick = sorted(set(rng.choice(len(probs), size=64, replace=False).tolist()) | {0, len(probs) - 1})
    for i in pick:
        p = probs[i]
        ref = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
        err = oracle.rel_frobenius(C[i][:ref.data.size].cpu().numpy(), ref.data)
        assert err <= TOL_F64, f"problem {i}: {err:.3e}"


@pytest.mark.parametrize("name", ["u1_d18_x64", "u1_d18_x512", "u1_uneven", "u1_uneven_f32"])
def test_grouped_batches(name):
    """The grouped launches of the batch workloads (autotuned up to 64
    problems, as timed): sampled problems in full against the oracle."""
    probs = {"u1_d18_x64": lambda: W.u1_d18(64), "u1_d18_x512": lambda: W.u1_d18(512),
             "u1_uneven": W.u1_uneven, "u1_uneven_f32": W.u1_uneven}[name]()
    prec = "f32" if name.endswith("f32") else "f64"
    dt = torch.float32 if prec == "f32" else torch.float64
    pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b) for p in probs], precision=prec)
    A = [torch.from_numpy(p.a.data).to(G.DEV).to(dt) for p in probs]
    B = [torch.from_numpy(p.b.data).to(G.DEV).to(dt) for p in probs]
    C = [torch.full((max(1, pl.output(i).numel),), float("nan"), dtype=dt, device=G.DEV) for i in range(len(probs))]
    ws = G.workspace(pl)
    if len(probs) <= 64:
        pl.autotune(A, B, C, ws, reps=3)
    for c in C:
        c.fill_(float("nan"))
    pl.contract(A, B, C, ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    pick = sorted(set(rng.integers(0, len(probs), size=16).tolist()) | {0, len(probs) - 1})
    for i in range(len(probs)):
        assert all_written(C[i], pl.output(i).numel), f"problem {i}: unwritten output elements"
    for i in pick:
        p = probs[i]
        ref = oracle.tensordot_blockpair(p.a, p.b, p.axes_a, p.axes_b)
        s = pl.output(i)
        assert G.structure_equal(s, ref)
        err = oracle.rel_frobenius(C[i][:s.numel].double().cpu().numpy(), ref.data)
        assert err <= (TOL["f32"] if prec == "f32" else TOL_F64), f"problem {i}: {err:.3e}"


def test_serving_mix_full_sizes():
    """All 32 serving runs (Z2 and U(1), D up to 10, chi up to 256) through the
    server with the benchmark's memory budget: each result bitwise equal to
    the same plans run alone, and every run checked against the oracle on
    sampled blocks of every step."""
    runs = []
    for r in range(32):
        t = W.serving_run(r)
        plans, cur = [], None
        for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
            pl = Y.plan([(t[an] if an else cur, t[bn], ax, bx)])
            plans.append(pl)
            cur = pl.output(0)
        runs.append((r, t, plans))
    srv = Y.Server(pool_bytes=32 << 30, max_ahead=2)
    reqs = []
    for r, t, plans in runs:
        inp = {k: G.upload(t[k]) for k in ("C", "T1", "T4", "A", "Ac")}
        n = plans[-1].output(0).numel
        out = torch.full((max(1, n),), float("nan"), dtype=torch.float64, device=G.DEV)
        rid = srv.submit(plans, inp["C"], [inp[bn] for _, bn in STEPS], out)
        reqs.append((rid, inp, out, n))
        srv.step()
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 32 and st["pool_peak"] <= st["pool_bytes"]
    for (r, t, plans), (rid, inp, out, n) in zip(runs, reqs):
        assert srv.query(rid)[0] == Y.REQ_DONE
        outs = []
        for i, ((an, bn), pl) in enumerate(zip(STEPS, plans)):
            c = torch.full((max(1, pl.output(0).numel),), float("nan"), dtype=torch.float64, device=G.DEV)
            pl.contract([inp[an] if an else outs[-1]], [inp[bn]], [c], G.workspace(pl))
            outs.append(c)
        torch.cuda.synchronize()
        assert torch.equal(out[:n], outs[-1][:n]), f"run {r}: result in the mix differs from alone"
        # every run, every step: structure in full and sampled blocks against
        # the oracle (on the GPU's input of that step; the D = 10 runs' largest
        # intermediates are too large for the oracle in full)
        cur = None
        for i, ((an, bn), (ax, bx), pl, c) in enumerate(zip(STEPS, t["axes"], plans, outs)):
            s = pl.output(0)
            assert all_written(c, s.numel)
            vals = c[:s.numel].cpu().numpy()
            check_sampled(t[an] if an else cur, t[bn], ax, bx, s, vals, 4, 100 * r + i)
            cur = G.as_block_tensor(s, vals)
            del vals
        del outs, inp
        torch.cuda.empty_cache()
    srv.close()
