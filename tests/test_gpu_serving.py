"""Serving runtime (continuous batching) on an MI355X.

Requests from several concurrent CTM runs (the serving mix's geometry at small
bond and environment dimensions, Z2 and U(1)) go through yastn_server_*; every
result must be bitwise the one the same chain gives alone through
yastn_contract (the kernels are deterministic and the merged launch keeps each
plan's tiles), and the chain must match the CPU oracle.
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

STEPS = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]
# (run, repeats): runs 0, 1, 4 are Z2 (D = 4, chi = 64 / 128; D = 6, chi = 64),
# runs 16, 17 are U(1) (D = 4, chi = 64 / 128)
RUNS = [0, 1, 4, 16, 17]


class Run:
    """One CTM run: resident tensors, cached plans, its chain alone as reference."""

    def __init__(self, run):
        self.t = W.serving_run(run)
        self.plans, cur = [], None
        for (an, bn), (ax, bx) in zip(STEPS, self.t["axes"]):
            pl = Y.plan([(self.t[an] if an else cur, self.t[bn], ax, bx)])
            self.plans.append(pl)
            cur = pl.output(0)
        self.inp = {k: G.upload(self.t[k]) for k in ("C", "T1", "T4", "A", "Ac")}
        self.n_out = self.plans[-1].output(0).numel

    def alone(self):
        outs = [G.alloc_out(pl, 0)[0] for pl in self.plans]
        for i, ((an, bn), pl) in enumerate(zip(STEPS, self.plans)):
            a = self.inp[an] if an else outs[i - 1]
            pl.contract([a], [self.inp[bn]], [outs[i]], G.workspace(pl))
        torch.cuda.synchronize()
        return outs[-1][:self.n_out].clone()

    def submit(self, srv, out):
        return srv.submit(self.plans, self.inp["C"], [self.inp[bn] for _, bn in STEPS], out)


@pytest.fixture(scope="module")
def runs():
    return [Run(r) for r in RUNS]


def test_chain_alone_matches_oracle(runs):
    r = runs[3]  # U(1), D = 4, chi = 64
    cur = None
    for (an, bn), (ax, bx) in zip(STEPS, r.t["axes"]):
        cur = oracle.tensordot_blockpair(r.t[an] if an else cur, r.t[bn], ax, bx)
    got = r.alone().cpu().numpy()
    assert oracle.rel_frobenius(got, cur.data) <= 1e-12


def test_mix_equals_alone_bitwise(runs):
    ref = [r.alone() for r in runs]
    srv = Y.Server(pool_bytes=1 << 30, max_ahead=2)
    reqs = []
    # staggered arrivals: two requests of every run, submitted while earlier ones run
    for rep in range(2):
        for i, r in enumerate(runs):
            out = torch.full((max(1, r.n_out),), float("nan"), dtype=torch.float64, device=G.DEV)
            reqs.append((i, r.submit(srv, out), out))
            srv.step()
    srv.drain()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert st["max_batch"] > 1, "no launch merged steps of several requests"
    for i, rid, out in reqs:
        state, lat = srv.query(rid)
        assert state == Y.REQ_DONE and lat > 0
        assert torch.equal(out[:runs[i].n_out], ref[i]), f"run {RUNS[i]}: result in the mix differs from alone"
    srv.close()


def test_admission_waits_for_memory(runs):
    """A pool that holds one request at a time: later requests queue, are
    admitted as memory frees up, and still give the alone results."""
    r = runs[1]  # Z2, D = 4, chi = 128
    ref = r.alone()
    need = 0
    for i, pl in enumerate(r.plans):
        if i + 1 < len(r.plans):
            need += (pl.output(0).numel * 8 + 255) // 256 * 256
        need += (pl.workspace_bytes + 255) // 256 * 256
    srv = Y.Server(pool_bytes=need + 256, max_ahead=3)
    outs = [torch.full((r.n_out,), float("nan"), dtype=torch.float64, device=G.DEV) for _ in range(3)]
    ids = [r.submit(srv, o) for o in outs]
    srv.step()
    st = srv.stats()
    assert st["running"] == 1 and st["queued"] == 2
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 3 and st["pool_peak"] <= st["pool_bytes"]
    for rid, o in zip(ids, outs):
        assert srv.query(rid)[0] == Y.REQ_DONE
        assert torch.equal(o, ref)
    srv.close()


def test_oversized_request_rejected(runs):
    r = runs[0]
    srv = Y.Server(pool_bytes=4096)
    out = torch.empty(max(1, r.n_out), dtype=torch.float64, device=G.DEV)
    with pytest.raises(Y.YastnError) as e:
        r.submit(srv, out)
    assert e.value.status == "ERR_NOMEM"
    srv.close()


def _footprint(plans):
    al = lambda b: (b + 255) // 256 * 256
    f = 0
    for i, pl in enumerate(plans):
        if i + 1 < len(plans):
            f += al(pl.output(0).numel * 8)
        f += al(pl.workspace_bytes)
    return f


def test_bounded_bypass_admission():
    """A request that does not fit is passed by later ones that do, at most
    16 times; then admission waits for it (no starvation), and every request
    still completes with its alone-result."""
    small, med, big = Run(16), Run(5), Run(21)  # U(1) D=4 chi=64; Z2 D=6 chi=128; U(1) D=6 chi=128
    fs, fm, fb = _footprint(small.plans), _footprint(med.plans), _footprint(big.plans)
    # memory alone would admit a 17th small request next to M; after M, B fits
    # next to 16 small ones
    assert fb - 256 >= 17 * fs and fm - 256 >= 16 * fs, (fs, fm, fb)
    srv = Y.Server(pool_bytes=fm + fb - 256, max_ahead=2)
    o_m = torch.empty(max(1, med.n_out), dtype=torch.float64, device=G.DEV)
    o_b = torch.empty(max(1, big.n_out), dtype=torch.float64, device=G.DEV)
    o_s = [torch.empty(max(1, small.n_out), dtype=torch.float64, device=G.DEV) for _ in range(30)]
    rm = med.submit(srv, o_m)
    rb = big.submit(srv, o_b)
    rs = [small.submit(srv, o) for o in o_s]
    srv.step()  # admission: M fits, B waits, S1..S16 pass B, S17.. wait behind B
    assert srv.query(rm)[0] != Y.REQ_QUEUED
    assert srv.query(rb)[0] == Y.REQ_QUEUED
    states = [srv.query(r)[0] for r in rs]
    assert all(s != Y.REQ_QUEUED for s in states[:16]), states
    assert all(s == Y.REQ_QUEUED for s in states[16:]), states
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 32 and st["bypasses"] == 16 and st["queued_peak"] >= 31
    assert torch.equal(o_m[:med.n_out], med.alone())
    assert torch.equal(o_b[:big.n_out], big.alone())
    ref = small.alone()
    for o in o_s:
        assert torch.equal(o[:small.n_out], ref)
    srv.close()
