"""Plain FP64 reference for one CTM move (test infrastructure only).

The paper's CTM iteration (Sec. III, Fig. 3) builds enlarged corners from
the environment tensors C, T and the site tensor (panels b, b', c), forms the
product of four enlarged corners and decomposes it by SVD (panel d); the
truncated SVD gives the projections from the enlarged virtual spaces back to
dimension chi.  The paper prints no formulas for these steps; the reading
taken here is the directional (left) move of the corner-transfer-matrix
method for a 1x1 unit cell, written out below in this module's notation.
Every contraction is ``tensordot_blockpair`` (O2) and the SVD is
``svd.svd_truncated``; nothing is fused, blocked or reordered beyond that.

Tensors (legs and signatures as ``workloads.ctm_env`` builds them):
C1..C4 corners, T1..T4 edges, A the site tensor, A* its conjugate.

1. Enlarged corners, each a chain of four contractions (corner . edge,
   . the other edge, . A, . A*), with two cuts of three legs each:
     Q1 top-left     legs (T1.r, T4.bot, A.b, A.r, A*.b, A*.r)
                     right cut (0, 3, 5), bottom cut (1, 2, 4)
     Q2 top-right    legs (T2.bot, T1.l, A.l, A.b, A*.l, A*.b)
                     left cut (1, 2, 4), bottom cut (0, 3, 5)
     Q3 bottom-right legs (T3.l, T2.t, A.t, A.l, A*.t, A*.l)
                     top cut (1, 2, 4), left cut (0, 3, 5)
     Q4 bottom-left  legs (T4.t, T3.r, A.t, A.r, A*.t, A*.r)
                     top cut (0, 2, 4), right cut (1, 3, 5)
2. Half systems across the horizontal cut:
     R_up = Q2 . Q1 over (Q2 left cut, Q1 right cut)
            legs (x: Q2 bottom cut, b: Q1 bottom cut)
     R_dn = Q3 . Q4 over (Q3 left cut, Q4 right cut)
            legs (x': Q3 top cut, b': Q4 top cut)
3. The four-corner product M = R_up . R_dn over (b, b'): the 2x2 system cut
   open on the right vertical bond, legs (x, x').
4. Truncated SVD M = U S V^T with rows x (``svd.svd_truncated``, its sign
   gauge and truncation rule), kept values S (at most chi); U has legs
   (x, k) with k of signature -1, V^T legs (k, x') with k of signature +1.
5. Projectors onto the left vertical bond.  A factor's legs carry M's
   signatures, so a half contracts with the factor's dual F* (every
   signature flipped, total charge negated, the same real values):
     P_up = R_dn . (S^-1/2 V^T)* over x'  legs (b', k), k of signature -1
     P_dn = R_up . (U S^-1/2)* over x     legs (b, k),  k of signature +1
   As matrices, P_up = R_dn^T V S^-1/2 and P_dn = R_up^T U S^-1/2, so with
   nothing truncated P_up P_dn^T inserted on the bond between the halves is
   the identity on their product: R_up (P_up P_dn^T) R_dn^T = M; truncated,
   it gives M's best rank-chi approximation U S V^T (the pins of
   tests/test_oracle_ctm.py).
6. The left column absorbs the next one, a projector on each vertical bond
   (P_up below the upper tensor, P_dn above the lower one):
     C1' = P_up . (C1 . T1)               legs (k, T1.r)         = C1's form
     T4' = P_dn^T (T4 . A . A*) P_up      legs (k, A.r, A*.r, k) = T4's form
     C4' = P_dn . (C4 . T3)               legs (k, T3.r)         = C4's form
   T4' is contracted as (((P_dn . T4) . A) . A*) . P_up, the order of an
   enlarged corner's chain (T4 . A . A* alone would hold D^8 chi^2 numbers).
7. Renormalisation: each new tensor divided by its largest |entry|.
"""

from __future__ import annotations

import numpy as np

from workloads import BlockTensor

from . import svd as S
from .blocksparse import dual, norms, tensordot_blockpair

# (left operand or None = the running result, right operand, axes_left, axes_right)
CORNER_CHAINS = {
    "Q1": [("C1", "T1", (1,), (0,)), (None, "T4", (0,), (0,)),
           (None, "A", (0, 3), (0, 1)), (None, "Ac", (0, 2, 6), (0, 1, 4))],
    "Q2": [("C2", "T2", (1,), (0,)), (None, "T1", (0,), (3,)),
           (None, "A", (0, 4), (3, 0)), (None, "Ac", (0, 3, 6), (3, 0, 4))],
    "Q3": [("C3", "T3", (1,), (3,)), (None, "T2", (0,), (3,)),
           (None, "A", (1, 4), (2, 3)), (None, "Ac", (1, 3, 6), (2, 3, 4))],
    "Q4": [("C4", "T4", (0,), (3,)), (None, "T3", (0,), (0,)),
           (None, "A", (1, 3), (1, 2)), (None, "Ac", (1, 2, 6), (1, 2, 4))],
}
# halves and the four-corner product: (left, right, axes_left, axes_right)
HALF_UP = ("Q2", "Q1", (1, 2, 4), (0, 3, 5))
HALF_DN = ("Q3", "Q4", (0, 3, 5), (1, 3, 5))
PRODUCT = ("Rup", "Rdn", (3, 4, 5), (3, 4, 5))
M_ROWS = (0, 1, 2)
# the column's own pieces before projection
C1T1 = ("C1", "T1", (1,), (0,))          # legs (C1.d, T1.k, T1.b, T1.r)
C4T3 = ("C4", "T3", (1,), (0,))          # legs (C4.u, T3.k, T3.b, T3.r)
# T4' as a chain from P_dn (legs (T4.bot-, A.b-, A*.b-type, k)):
T4_CHAIN = [("Pdn", "T4", (0,), (0,)),           # Z1 (A.b', A*.b', k, T4.k, T4.b, T4.bot)
            ("Z1", "A", (0, 3), (0, 1)),          # Z2 (A*.b', k, T4.b, T4.bot, A.b, A.r, A.p)
            ("Z2", "Ac", (0, 2, 6), (0, 1, 4)),   # Z3 (k, T4.bot, A.b, A.r, A*.b, A*.r)
            ("Z3", "Pup", (1, 2, 4), (0, 1, 2))]  # T4' (k, A.r, A*.r, k)


def _td(x, y, ax, bx):
    return tensordot_blockpair(x, y, ax, bx)


def enlarged_corner(env: dict, name: str) -> BlockTensor:
    cur = None
    for left, right, ax, bx in CORNER_CHAINS[name]:
        cur = _td(env[left] if left else cur, env[right], ax, bx)
    return cur


def scale_new_leg(t: BlockTensor, svals: dict, power: float, leg: int) -> BlockTensor:
    """Multiply a factor's new leg (last leg of U, first of V^T) by S^power:
    block entries along that leg scaled by the sector's kept values."""
    data = t.data.copy()
    for b in range(t.nblocks):
        X = tuple(int(v) for v in t.charges[b, leg])
        sh = tuple(int(x) for x in t.shapes[b])
        o = int(t.offsets[b])
        blk = data[o:o + int(np.prod(sh))].reshape(sh)
        f = np.asarray(svals[X], dtype=np.float64) ** power
        shape = [1] * len(sh)
        shape[leg] = f.size
        data[o:o + blk.size] = (blk * f.reshape(shape)).ravel()
    return BlockTensor(t.sym_mod, t.sig, t.n, t.charges, t.shapes, t.offsets, data)


def normalise_max(t: BlockTensor) -> BlockTensor:
    """Step 7: divide by the largest |entry| (a tensor of zeros is left as is)."""
    _, mx = norms(t)
    if mx == 0.0:
        return t.copy()
    return BlockTensor(t.sym_mod, t.sig, t.n, t.charges, t.shapes, t.offsets, t.data / mx)


def left_move(env: dict, chi: int, tol: float = 0.0, deg_tol: float = 1e-10) -> dict:
    """All intermediate and final tensors of one left move (steps 1-7)."""
    r = {}
    for q in ("Q1", "Q2", "Q3", "Q4"):
        r[q] = enlarged_corner(env, q)
    r["Rup"] = _td(r[HALF_UP[0]], r[HALF_UP[1]], HALF_UP[2], HALF_UP[3])
    r["Rdn"] = _td(r[HALF_DN[0]], r[HALF_DN[1]], HALF_DN[2], HALF_DN[3])
    r["M"] = _td(r[PRODUCT[0]], r[PRODUCT[1]], PRODUCT[2], PRODUCT[3])
    u, svals, vt, kept = S.svd_truncated(r["M"], M_ROWS, chi, tol, deg_tol)
    r["U"], r["S"], r["Vt"], r["kept"] = u, svals, vt, kept
    r["Us"] = scale_new_leg(u, svals, -0.5, u.rank - 1)
    r["Vts"] = scale_new_leg(vt, svals, -0.5, 0)
    r["Pup"] = _td(r["Rdn"], dual(r["Vts"]), (0, 1, 2), (1, 2, 3))
    r["Pdn"] = _td(r["Rup"], dual(r["Us"]), (0, 1, 2), (0, 1, 2))
    r["C1T1"] = _td(env[C1T1[0]], env[C1T1[1]], C1T1[2], C1T1[3])
    r["C4T3"] = _td(env[C4T3[0]], env[C4T3[1]], C4T3[2], C4T3[3])
    r["C1n"] = _td(r["Pup"], r["C1T1"], (0, 1, 2), (0, 1, 2))
    r["C4n"] = _td(r["Pdn"], r["C4T3"], (0, 1, 2), (0, 1, 2))
    both = dict(env, **r)
    for out, (left, right, ax, bx) in zip(("Z1", "Z2", "Z3", "T4n"), T4_CHAIN):
        both[out] = r[out] = _td(both[left], both[right], ax, bx)
    for k in ("C1n", "T4n", "C4n"):
        r[k + "_norm"] = normalise_max(r[k])
    return r
