"""Plant plausible mistakes in the oracle (on the CPU) and check a pin fails.

Each mutation is a small, realistic slip (a dropped term, a wrong index or
sign, a transposed operand, a skipped normalisation); the pins of
test_oracle_pins.py must catch every one of them.
"""

import numpy as np
import pytest

import oracle
import oracle.blocksparse as ob
import workloads as W
from tests import test_oracle_pins as P

CAUGHT = (AssertionError, oracle.OracleError, KeyError, ValueError, IndexError)


def _run_pins():
    P.test_u1_d18_closed_form_structure()
    P.test_u1_d18_dense_equals_blockpair()
    P.test_paper_example_h_squared_exact("dense")
    P.test_paper_example_h_squared_exact("blockpair")
    P.test_paper_example_h_squared_exact("brute")
    P.test_paper_example_fused_matmul_identity()
    P.test_z_m_charges_normalised()
    for seed in range(8):
        for sym in ("U1", "Z2", "U1xZ2"):
            P.test_brute_dense_blockpair_agree(seed, sym)
    for seed in range(4):
        P.test_fusion_invariance(seed)
        P.test_swap_operands_is_transpose(seed)


def test_pins_pass_unmutated():
    _run_pins()


def _mut_matched_wrong_axes(monkeypatch):
    orig = ob.matched_pairs

    def bad(a, b, axes_a, axes_b):
        return orig(a, b, axes_a, axes_a if len(axes_a) and max(axes_a) < b.rank else axes_b)
    monkeypatch.setattr(ob, "matched_pairs", bad)


def _mut_blockpair_drop_term(monkeypatch):
    """O2 overwrites instead of accumulating: only the last matched pair of
    each output block survives."""
    orig = ob.tensordot_blockpair

    def bad(a, b, axes_a, axes_b):
        c = orig(a, b, axes_a, axes_b)
        aa, bb = ob.normalize(a), ob.normalize(b)
        fa, fb = ob._free(aa.rank, axes_a), ob._free(bb.rank, axes_b)
        idx = {ob._block_key(c, k): k for k in range(c.nblocks)}
        for i, j in ob.matched_pairs(aa, bb, axes_a, axes_b):
            k = idx[ob._block_key(aa, i, fa) + ob._block_key(bb, j, fb)]
            r = np.tensordot(aa.block(i), bb.block(j), (tuple(axes_a), tuple(axes_b)))
            c.data[c.offsets[k]:c.offsets[k] + r.size] = r.ravel()
        return c
    monkeypatch.setattr(ob, "tensordot_blockpair", bad)
    monkeypatch.setattr(oracle, "tensordot_blockpair", bad)


def _mut_output_order(monkeypatch):
    monkeypatch.setattr(ob, "_flat", lambda key: tuple(-v for q in key for v in q))


def _mut_n_sign(monkeypatch):
    orig = ob.output_structure

    def bad(a, b, axes_a, axes_b):
        c = orig(a, b, axes_a, axes_b)
        c.n = np.array(ob._nq([int(p) - int(q) for p, q in zip(a.n, b.n)], a.sym_mod), dtype=np.int32)
        return c
    monkeypatch.setattr(ob, "output_structure", bad)


def _mut_no_mod(monkeypatch):
    monkeypatch.setattr(ob, "_nq", lambda q, sym_mod: tuple(int(v) for v in q))


def _mut_dense_transposed(monkeypatch):
    """O1 contracts B with A (operands swapped), then reads C in A-then-B
    order as if nothing happened."""
    orig = np.tensordot

    class FakeNP:
        def __getattr__(self, k):
            return getattr(np, k)

        @staticmethod
        def tensordot(x, y, axes):
            r = orig(y, x, (axes[1], axes[0]))
            return r.reshape(orig(x, y, axes).shape)
    monkeypatch.setattr(ob, "np", FakeNP())


def _mut_fuse_sign(monkeypatch):
    orig = ob.fuse_legs

    def bad(t, groups, templates=None):
        out, rec = orig(t, groups, templates)
        out = out.copy()
        out.sig = (-out.sig).astype(np.int8)  # signature of the fused leg flipped
        return out, rec
    monkeypatch.setattr(ob, "fuse_legs", bad)
    monkeypatch.setattr(oracle, "fuse_legs", bad)


MUTATIONS = {
    "matched_pairs uses A's axes for B": _mut_matched_wrong_axes,
    "block-pair sum keeps one term": _mut_blockpair_drop_term,
    "output blocks in reversed order": _mut_output_order,
    "n_C = n_A - n_B": _mut_n_sign,
    "Z_m charges not reduced": _mut_no_mod,
    "dense contraction transposed": _mut_dense_transposed,
    "fused leg signature flipped": _mut_fuse_sign,
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    with pytest.raises(CAUGHT):
        _run_pins()


def test_ctm_structure_counts():
    """Counts of the four enlarged-corner steps at chi=128, D=8, derived by
    an independent enumeration of the workload recipe."""
    t = W.ctm()
    steps = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]
    expect = [(255, 15, 255), (4489, 15, 4489), (33145, 13, 15643), (32647, 13, 5113)]
    cur = None
    for (an, bn), (ax, bx), (npair, nsec, ncb) in zip(steps, t["axes"], expect):
        a = t[an] if an else cur
        st = oracle.structure_stats(a, t[bn], ax, bx)
        assert (st["pairs"], st["sectors"], st["c_blocks"]) == (npair, nsec, ncb)
        cur = oracle.output_structure(a, t[bn], ax, bx)
