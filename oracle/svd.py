"""Plain FP64 reference for the block-sparse truncated SVD (test infrastructure).

The CTM step of the paper (Sec. III, Fig. 3 (c)-(d)) fuses the enlarged corner
into a block-diagonal matrix and truncates its singular value decomposition
to the environment dimension chi.  Here, for a block tensor T and a split of
its legs into row legs and column legs:

  * sector X = sum over the row legs of s_i rho_i (normalised; by the block
    form of charge conservation the column legs then carry n - X), one dense
    matrix M_X per sector: Sec. II.B fusion of the row legs into one leg and
    of the column legs into another, the constituent charge tuples of a
    sector in ascending order (as ``fuse_legs``), each block's row index in C
    order over its row legs and its column index in C order over its column
    legs;
  * M_X = U_X diag(S_X) V_X^T by numpy.linalg.svd, S_X descending, with the
    sign of every singular pair fixed (the reading taken, the paper fixes
    none): (u_k, v_k) and (-u_k, -v_k) are equally valid, and the pair kept
    is the one whose u_k has its entry of largest magnitude (the first such
    in row order) positive, so the factors, and what is built from them, are
    unique when the values are distinct;
  * one global truncation over all sectors (``truncation``): the rule below;
  * the kept factors as block tensors: U with legs (row legs..., v), the new
    leg v of charge X and signature -1, so U has total charge 0; V^T with
    legs (v', column legs...), v' of charge X and signature +1, so V^T has
    the total charge of T.  A sector with no kept value has no blocks.

Truncation (the paper fixes none; the reading taken): values at or below
tol * (largest singular value) are dropped; of the rest, if more than chi
remain, with c the (chi+1)-th largest, a value is kept iff it exceeds
c * (1 + deg_tol).  So at most chi values are kept and a multiplet of values
within the relative gap deg_tol of the first dropped value is dropped whole,
never split.  Kept values of a sector are a prefix of its descending list.
"""

from __future__ import annotations

import numpy as np

from workloads import BlockTensor

from .blocksparse import _block_key, _flat, _nq, normalize


def _sector_of(t: BlockTensor, b: int, legs) -> tuple:
    tot = [0] * t.nsym
    for x in legs:
        for c in range(t.nsym):
            tot[c] += int(t.sig[x]) * int(t.charges[b, x, c])
    return tuple(_nq(tot, t.sym_mod))


def sector_matrices(t: BlockTensor, row_legs):
    """{X: (M_X, rows, cols)} in ascending X.  rows / cols: the sector's
    constituent tuples in order, each (charges, dims, offset in M_X)."""
    t = normalize(t)
    row_legs = tuple(row_legs)
    col_legs = tuple(x for x in range(t.rank) if x not in row_legs)
    rows, cols = {}, {}
    for b in range(t.nblocks):
        X = _sector_of(t, b, row_legs)
        rows.setdefault(X, {})[_block_key(t, b, row_legs)] = tuple(int(t.shapes[b, x]) for x in row_legs)
        cols.setdefault(X, {})[_block_key(t, b, col_legs)] = tuple(int(t.shapes[b, x]) for x in col_legs)
    out = {}
    for X in sorted(rows):
        rl, cl, r0, c0 = [], [], 0, 0
        for key in sorted(rows[X], key=_flat):
            dims = rows[X][key]
            rl.append((key, dims, r0))
            r0 += int(np.prod(dims))
        for key in sorted(cols[X], key=_flat):
            dims = cols[X][key]
            cl.append((key, dims, c0))
            c0 += int(np.prod(dims))
        out[X] = [np.zeros((r0, c0)), rl, cl]
    rpos = {X: {k: (d, o) for k, d, o in v[1]} for X, v in out.items()}
    cpos = {X: {k: (d, o) for k, d, o in v[2]} for X, v in out.items()}
    for b in range(t.nblocks):
        X = _sector_of(t, b, row_legs)
        rd, ro = rpos[X][_block_key(t, b, row_legs)]
        cd, co = cpos[X][_block_key(t, b, col_legs)]
        m, n = int(np.prod(rd)), int(np.prod(cd))
        blk = np.transpose(t.block(b), row_legs + col_legs).reshape(m, n)
        out[X][0][ro:ro + m, co:co + n] = blk
    return {X: tuple(v) for X, v in out.items()}


def sign_gauge(U, Vt):
    """Flip (u_k, v_k) to (-u_k, -v_k) where u_k's entry of largest magnitude
    (the first such) is negative."""
    if U.size == 0:
        return U, Vt
    i = np.argmax(np.abs(U), axis=0)
    f = np.where(U[i, np.arange(U.shape[1])] < 0.0, -1.0, 1.0)
    return U * f, Vt * f[:, None]


def svd_sectors(t: BlockTensor, row_legs):
    """{X: (U_X, S_X, Vt_X)}: the SVD of every sector matrix (full_matrices
    off, S_X descending, signs by ``sign_gauge``)."""
    res = {}
    for X, (M, _, _) in sector_matrices(t, row_legs).items():
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        U, Vt = sign_gauge(U, Vt)
        res[X] = (U, S, Vt)
    return res


def truncation(svals: dict, chi: int, tol: float = 0.0, deg_tol: float = 1e-10) -> dict:
    """Kept count per sector for singular values {X: S_X (descending)} under
    the global rule of the module docstring."""
    allv = np.concatenate([np.asarray(s, dtype=np.float64) for s in svals.values()]) if svals else np.zeros(0)
    if allv.size == 0:
        return {X: 0 for X in svals}
    smax = float(allv.max())
    floor = tol * smax
    alive = np.sort(allv[allv > floor])[::-1]
    cut = floor
    if alive.size > chi:
        cut = max(floor, float(alive[chi]) * (1.0 + deg_tol))
    return {X: int(np.count_nonzero(np.asarray(s) > cut)) for X, s in svals.items()}


def _pack(sym_mod, sig, n, items):
    """Block tensor from [(charge tuple of tuples, array)] in ascending order."""
    items = sorted(items, key=lambda kv: _flat(kv[0]))
    rank = len(sig)
    nsym = len(sym_mod)
    charges = np.zeros((len(items), rank, nsym), dtype=np.int32)
    shapes = np.zeros((len(items), rank), dtype=np.int64)
    datas = []
    for k, (key, arr) in enumerate(items):
        charges[k] = np.array(key, dtype=np.int32).reshape(rank, nsym)
        shapes[k] = arr.shape
        datas.append(np.ascontiguousarray(arr).ravel())
    sizes = np.array([d.size for d in datas], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if items else np.zeros(0, np.int64)
    return BlockTensor(tuple(sym_mod), np.array(sig, dtype=np.int8), np.array(n, dtype=np.int32), charges,
                       shapes, offsets, np.concatenate(datas) if datas else np.zeros(0))


def svd_truncated(t: BlockTensor, row_legs, chi: int, tol: float = 0.0, deg_tol: float = 1e-10):
    """(U, S, Vt, kept): U and Vt as block tensors (legs as in the module
    docstring), S = {X: kept singular values}, kept = {X: count}."""
    t = normalize(t)
    row_legs = tuple(row_legs)
    col_legs = tuple(x for x in range(t.rank) if x not in row_legs)
    mats = sector_matrices(t, row_legs)
    dec = {}
    for X, (M, _, _) in mats.items():
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        U, Vt = sign_gauge(U, Vt)
        dec[X] = (U, s, Vt)
    kept = truncation({X: d[1] for X, d in dec.items()}, chi, tol, deg_tol)
    u_items, v_items, S = [], [], {}
    for X, (M, rl, cl) in mats.items():
        k = kept[X]
        U, s, Vt = dec[X]
        S[X] = s[:k].copy()
        if k == 0:
            continue
        for key, dims, o in rl:
            m = int(np.prod(dims))
            u_items.append((tuple(key) + (X,), U[o:o + m, :k].reshape(dims + (k,))))
        for key, dims, o in cl:
            n = int(np.prod(dims))
            v_items.append(((X,) + tuple(key), Vt[:k, o:o + n].reshape((k,) + dims)))
    u = _pack(t.sym_mod, [int(t.sig[x]) for x in row_legs] + [-1], [0] * t.nsym, u_items)
    vt = _pack(t.sym_mod, [1] + [int(t.sig[x]) for x in col_legs], [int(v) for v in t.n], v_items)
    return u, S, vt, kept
