"""Plain FP64 reference for the block-sparse tensordot (test infrastructure).

Paper references are to "YASTN: Yet another symmetric tensor networks"
(arXiv:2405.12196): Sec. II.A (abelian-symmetric tensor, block form of charge
conservation, lazy 1D storage), Sec. II.B (fusion, fused charges and sector
dims, the fuse -> multiply -> unfuse contraction identity and its footnote on
charges missing from one partner).
"""

from __future__ import annotations

import itertools

import numpy as np

from workloads import BlockTensor

# status classes shared by meaning (not by code) with the C library
ERR_ARG, ERR_SYM, ERR_CHARGE, ERR_SIGNATURE, ERR_SHAPE, ERR_DUPLICATE = (
    "ERR_ARG", "ERR_SYM", "ERR_CHARGE", "ERR_SIGNATURE", "ERR_SHAPE", "ERR_DUPLICATE")


class OracleError(Exception):
    def __init__(self, status, msg=""):
        super().__init__(f"{status}: {msg}")
        self.status = status


# ---------------------------------------------------------------------------
# charges
# ---------------------------------------------------------------------------
def _nq(q, sym_mod):
    """Normalise one charge vector: Z_m components into [0, m) (Sec. II.A:
    Z_m charges are elements of Z_m, U(1) charges of Z)."""
    return tuple(int(v) % m if m else int(v) for v, m in zip(q, sym_mod))


def normalize(t: BlockTensor) -> BlockTensor:
    out = t.copy()
    for c, m in enumerate(t.sym_mod):
        if m:
            out.charges[:, :, c] = np.mod(out.charges[:, :, c], m)
    out.n = np.array(_nq(t.n, t.sym_mod), dtype=np.int32)
    return out


def _block_key(t: BlockTensor, b: int, legs=None):
    """Charge tuple of block b restricted to ``legs`` (tuple of tuples)."""
    legs = range(t.rank) if legs is None else legs
    return tuple(_nq(t.charges[b, i, :], t.sym_mod) for i in legs)


def _flat(key):
    return tuple(v for q in key for v in q)


# ---------------------------------------------------------------------------
# validation (Sec. II.A block conservation; Sec. II.B contraction compatibility)
# ---------------------------------------------------------------------------
def validate_tensor(t: BlockTensor):
    if t.charges.ndim != 3 or t.shapes.ndim != 2:
        raise OracleError(ERR_ARG, "bad descriptor arrays")
    if t.charges.shape[1] != t.rank or t.shapes.shape[1] != t.rank:
        raise OracleError(ERR_ARG, "rank mismatch")
    if t.charges.shape[2] != t.nsym or t.n.shape[0] != t.nsym:
        raise OracleError(ERR_ARG, "nsym mismatch")
    if any(int(s) not in (1, -1) for s in t.sig):
        raise OracleError(ERR_ARG, "signature must be +1 or -1")
    if t.nblocks and np.any(t.shapes < 1):
        raise OracleError(ERR_SHAPE, "dims must be >= 1")
    seen = set()
    leg_dims = [dict() for _ in range(t.rank)]
    n = _nq(t.n, t.sym_mod)
    for b in range(t.nblocks):
        key = _block_key(t, b)
        if key in seen:
            raise OracleError(ERR_DUPLICATE, f"block {key} repeated")
        seen.add(key)
        tot = [0] * t.nsym
        for i in range(t.rank):
            for c in range(t.nsym):
                tot[c] += int(t.sig[i]) * key[i][c]
        if _nq(tot, t.sym_mod) != n:
            raise OracleError(ERR_CHARGE, f"block {key} violates sum s*rho = n")
    for b in range(t.nblocks):
        key = _block_key(t, b)
        for i in range(t.rank):
            d = int(t.shapes[b, i])
            if leg_dims[i].setdefault(key[i], d) != d:
                raise OracleError(ERR_SHAPE, f"leg {i} charge {key[i]} has two dims")
    if t.nblocks:
        if np.any(t.offsets < 0):
            raise OracleError(ERR_ARG, "negative offset")
        order = np.argsort(t.offsets, kind="stable")
        ends = t.offsets[order] + t.block_sizes[order]
        if np.any(ends[:-1] > t.offsets[order][1:]):
            raise OracleError(ERR_ARG, "blocks overlap in the 1D buffer")
    return leg_dims


def validate_pair(a: BlockTensor, b: BlockTensor, axes_a, axes_b):
    axes_a, axes_b = tuple(axes_a), tuple(axes_b)
    if len(axes_a) != len(axes_b):
        raise OracleError(ERR_ARG, "axes of different length")
    for ax, r in ((axes_a, a.rank), (axes_b, b.rank)):
        if any(x < 0 or x >= r for x in ax) or len(set(ax)) != len(ax):
            raise OracleError(ERR_ARG, "axes out of range or repeated")
    if tuple(a.sym_mod) != tuple(b.sym_mod):
        raise OracleError(ERR_SYM, "different symmetry")
    if any(m < 0 or m == 1 for m in a.sym_mod):
        raise OracleError(ERR_SYM, "sym_mod must be 0 (U(1)) or >= 2 (Z_m)")
    dims_a = validate_tensor(a)
    dims_b = validate_tensor(b)
    for x, y in zip(axes_a, axes_b):
        if int(a.sig[x]) == int(b.sig[y]):
            raise OracleError(ERR_SIGNATURE, f"legs {x} and {y} have equal signature")
    for x, y in zip(axes_a, axes_b):
        for q, d in dims_a[x].items():
            if q in dims_b[y] and dims_b[y][q] != d:
                raise OracleError(ERR_SHAPE, f"contracted charge {q} has dims {d} vs {dims_b[y][q]}")
    return dims_a, dims_b


# ---------------------------------------------------------------------------
# output structure (rule R)
# ---------------------------------------------------------------------------
def _free(rank, axes):
    return tuple(i for i in range(rank) if i not in axes)


def matched_pairs(a: BlockTensor, b: BlockTensor, axes_a, axes_b):
    """All (i, j) with block i of A and block j of B whose charges agree on
    every contracted leg pair (Sec. II.B: contracted legs carry the same
    charge on both partners; a charge present on one side only contributes
    nothing, per the footnote on missing partner charges)."""
    bykey = {}
    for j in range(b.nblocks):
        bykey.setdefault(_block_key(b, j, axes_b), []).append(j)
    out = []
    for i in range(a.nblocks):
        for j in bykey.get(_block_key(a, i, axes_a), []):
            out.append((i, j))
    return out


def output_structure(a: BlockTensor, b: BlockTensor, axes_a, axes_b, with_data=True):
    """Rule R: C's legs are A's free legs then B's free legs (numpy tensordot
    order, as in the paper's listing), n_C = n_A + n_B, and C holds exactly the
    blocks (a_free, b_free) reached by at least one matched pair, sorted in
    ascending lexicographic order, stored contiguously."""
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    pairs = matched_pairs(a, b, axes_a, axes_b)
    keys = {}
    for i, j in pairs:
        ka, kb = _block_key(a, i, fa), _block_key(b, j, fb)
        k = ka + kb
        if k not in keys:
            shp = tuple(int(a.shapes[i, x]) for x in fa) + tuple(int(b.shapes[j, y]) for y in fb)
            keys[k] = shp
    order = sorted(keys, key=_flat)
    nsym = a.nsym
    rank = len(fa) + len(fb)
    charges = np.zeros((len(order), rank, nsym), dtype=np.int32)
    shapes = np.zeros((len(order), rank), dtype=np.int64)
    for bi, k in enumerate(order):
        charges[bi] = np.array(k, dtype=np.int32).reshape(rank, nsym)
        shapes[bi] = keys[k]
    sizes = np.prod(shapes, axis=1).astype(np.int64) if len(order) else np.zeros(0, np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if len(order) else np.zeros(0, np.int64)
    sig = np.array([a.sig[x] for x in fa] + [b.sig[y] for y in fb], dtype=np.int8)
    n = np.array(_nq([int(p) + int(q) for p, q in zip(a.n, b.n)], a.sym_mod), dtype=np.int32)
    return BlockTensor(tuple(a.sym_mod), sig, n, charges, shapes, offsets,
                       np.zeros(int(sizes.sum()) if with_data else 0, dtype=_value_type(a, b)))


def _value_type(a, b):
    """float64, or complex128 when either operand holds complex values."""
    return np.result_type(np.asarray(a.data).dtype, np.asarray(b.data).dtype, np.float64)


# ---------------------------------------------------------------------------
# O1: dense embedding (the definition)
# ---------------------------------------------------------------------------
def leg_index_maps(t: BlockTensor, extra=None):
    """Per leg: charges present (ascending lexicographic), their dims and the
    first dense index of each sector (basis ordered by charge, Sec. II.A).
    ``extra[i]`` adds charges (with dims) to leg i, e.g. a contraction
    partner's charges so both dense index spaces coincide."""
    maps = []
    for i in range(t.rank):
        dims = {}
        for b in range(t.nblocks):
            dims[_nq(t.charges[b, i, :], t.sym_mod)] = int(t.shapes[b, i])
        if extra is not None and extra[i]:
            for q, d in extra[i].items():
                dims.setdefault(q, d)
        qs = sorted(dims)
        start, pos = {}, 0
        for q in qs:
            start[q] = pos
            pos += dims[q]
        maps.append({"charges": qs, "dims": dims, "start": start, "D": pos})
    return maps


def to_dense(t: BlockTensor, maps):
    full = np.zeros(tuple(m["D"] for m in maps), dtype=np.result_type(np.asarray(t.data).dtype, np.float64))
    for b in range(t.nblocks):
        key = _block_key(t, b)
        sl = tuple(slice(maps[i]["start"][key[i]], maps[i]["start"][key[i]] + int(t.shapes[b, i]))
                   for i in range(t.rank))
        full[sl] = t.block(b)
    return full


def _contracted_extra(a, b, axes_a, axes_b):
    ea = [None] * a.rank
    eb = [None] * b.rank
    for x, y in zip(axes_a, axes_b):
        da = {_nq(a.charges[i, x, :], a.sym_mod): int(a.shapes[i, x]) for i in range(a.nblocks)}
        db = {_nq(b.charges[j, y, :], b.sym_mod): int(b.shapes[j, y]) for j in range(b.nblocks)}
        ea[x], eb[y] = db, da
    return ea, eb


def tensordot_dense(a: BlockTensor, b: BlockTensor, axes_a, axes_b, *, return_dense=False):
    """O1.  Embed A and B densely (contracted legs share the union of both
    partners' charges), contract with numpy.tensordot in float64 (complex128
    for complex values), read C's
    blocks back at rule-R positions, and check that every dense entry outside
    those blocks is exactly zero (Sec. II.A element-wise conservation)."""
    validate_pair(a, b, axes_a, axes_b)
    a, b = normalize(a), normalize(b)
    ea, eb = _contracted_extra(a, b, axes_a, axes_b)
    ma, mb = leg_index_maps(a, ea), leg_index_maps(b, eb)
    ad, bd = to_dense(a, ma), to_dense(b, mb)
    cd = np.tensordot(ad, bd, axes=(tuple(axes_a), tuple(axes_b)))
    c = output_structure(a, b, axes_a, axes_b)
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    cmaps = [ma[x] for x in fa] + [mb[y] for y in fb]
    mask = np.zeros(cd.shape, dtype=bool)
    for k in range(c.nblocks):
        key = _block_key(c, k)
        sl = tuple(slice(cmaps[i]["start"][key[i]], cmaps[i]["start"][key[i]] + int(c.shapes[k, i]))
                   for i in range(c.rank))
        c.data[c.offsets[k]:c.offsets[k] + int(np.prod(c.shapes[k]))] = cd[sl].ravel()
        mask[sl] = True
    outside = cd[~mask]
    if outside.size and np.any(outside != 0.0):
        raise AssertionError("dense result has non-zero entries outside the rule-R blocks")
    if return_dense:
        return c, cd
    return c


# ---------------------------------------------------------------------------
# O2: block pairs
# ---------------------------------------------------------------------------
def tensordot_blockpair(a: BlockTensor, b: BlockTensor, axes_a, axes_b):
    """O2.  For each rule-R output block, sum numpy.tensordot of its matched
    block pairs in ascending lexicographic order of the contracted charges
    (the fuse -> multiply -> unfuse identity of Sec. II.B, block by block)."""
    validate_pair(a, b, axes_a, axes_b)
    a, b = normalize(a), normalize(b)
    c = output_structure(a, b, axes_a, axes_b)
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    index = {_block_key(c, k): k for k in range(c.nblocks)}
    groups = {}
    for i, j in matched_pairs(a, b, axes_a, axes_b):
        k = index[_block_key(a, i, fa) + _block_key(b, j, fb)]
        groups.setdefault(k, []).append((_flat(_block_key(a, i, axes_a)), i, j))
    for k, lst in groups.items():
        lst.sort()
        acc = np.zeros(tuple(int(x) for x in c.shapes[k]), dtype=c.data.dtype)
        for _, i, j in lst:
            acc += np.tensordot(a.block(i), b.block(j), axes=(tuple(axes_a), tuple(axes_b)))
        c.data[c.offsets[k]:c.offsets[k] + acc.size] = acc.ravel()
    return c


def tensordot_blocks(a: BlockTensor, b: BlockTensor, axes_a, axes_b, block_ids):
    """O2 restricted to some output blocks: returns (structure of C without
    values, {block index: dense block}) for the rule-R output block indices in
    block_ids, each the sum of numpy.tensordot over its matched block pairs in
    ascending lexicographic order of the contracted charges -- the same terms
    in the same order as tensordot_blockpair, for outputs too large to hold on
    the host (Sec. II.B, block by block)."""
    validate_pair(a, b, axes_a, axes_b)
    a, b = normalize(a), normalize(b)
    c = output_structure(a, b, axes_a, axes_b, with_data=False)
    want = {int(k) for k in block_ids}
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    index = {_block_key(c, k): k for k in range(c.nblocks)}
    groups = {}
    for i, j in matched_pairs(a, b, axes_a, axes_b):
        k = index[_block_key(a, i, fa) + _block_key(b, j, fb)]
        if k in want:
            groups.setdefault(k, []).append((_flat(_block_key(a, i, axes_a)), i, j))
    out = {}
    for k in sorted(want):
        acc = np.zeros(tuple(int(x) for x in c.shapes[k]), dtype=_value_type(a, b))
        for _, i, j in sorted(groups.get(k, [])):
            acc += np.tensordot(a.block(i), b.block(j), axes=(tuple(axes_a), tuple(axes_b)))
        out[k] = acc
    return c, out


# ---------------------------------------------------------------------------
# O3: brute force over dense indices (tiny inputs only)
# ---------------------------------------------------------------------------
def tensordot_brute(a: BlockTensor, b: BlockTensor, axes_a, axes_b):
    """O3.  Pure-Python loops.  Every dense index gets its charge from the leg
    maps; every stored non-zero element is checked against the element form
    of charge conservation (eq. elemchargecon, Sec. II.A); C is formed by
    explicit sums over the contracted dense indices.  Returns the dense C."""
    a, b = normalize(a), normalize(b)
    ea, eb = _contracted_extra(a, b, axes_a, axes_b)
    ma, mb = leg_index_maps(a, ea), leg_index_maps(b, eb)

    def charge_of(maps, leg, idx):
        for q in maps[leg]["charges"]:
            s = maps[leg]["start"][q]
            if s <= idx < s + maps[leg]["dims"][q]:
                return q, idx - s
        raise IndexError

    def lookup(t, maps):
        blocks = {_block_key(t, k): k for k in range(t.nblocks)}
        vals = {}
        for idx in itertools.product(*[range(m["D"]) for m in maps]):
            qs, loc = zip(*[charge_of(maps, i, x) for i, x in enumerate(idx)])
            k = blocks.get(tuple(qs))
            v = 0.0 if k is None else float(t.block(k)[tuple(loc)])
            if v != 0.0:
                tot = [0] * t.nsym
                for i, q in enumerate(qs):
                    for c_ in range(t.nsym):
                        tot[c_] += int(t.sig[i]) * q[c_]
                if _nq(tot, t.sym_mod) != _nq(t.n, t.sym_mod):
                    raise AssertionError("non-zero element violates charge conservation")
            vals[idx] = v
        return vals

    va, vb = lookup(a, ma), lookup(b, mb)
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    cshape = tuple(ma[x]["D"] for x in fa) + tuple(mb[y]["D"] for y in fb)
    ctr_ranges = [range(ma[x]["D"]) for x in axes_a]
    out = np.zeros(cshape, dtype=np.float64)
    for ci in itertools.product(*[range(d) for d in cshape]):
        ia_free, ib_free = ci[:len(fa)], ci[len(fa):]
        s = 0.0
        for xs in itertools.product(*ctr_ranges):
            ia = [0] * a.rank
            ib = [0] * b.rank
            for p, x in enumerate(fa):
                ia[x] = ia_free[p]
            for p, y in enumerate(fb):
                ib[y] = ib_free[p]
            for p, (x, y) in enumerate(zip(axes_a, axes_b)):
                ia[x] = xs[p]
                ib[y] = xs[p]
            s += va[tuple(ia)] * vb[tuple(ib)]
        out[ci] = s
    return out


# ---------------------------------------------------------------------------
# O-fuse: fusion and unfusion (Sec. II.B, fused charges and sector dims)
# ---------------------------------------------------------------------------
def fuse_legs(t: BlockTensor, groups, templates=None):
    """Fuse each group of legs into one leg; new legs in group order.

    Fused signature s_r = signature of the group's first leg.  A constituent
    charge tuple (rho_i)_{i in group} maps to the fused charge
    nu = s_r * sum_i s_i rho_i; the fused sector dim is the sum over its
    constituents of prod_i D_i.  Only constituents that occur in some block
    are kept (lazy fusion), plus those listed in ``templates[g]`` (charges of
    a contraction partner).  Constituents of a sector are ordered ascending
    lexicographically.  Returns (fused tensor, record for unfuse_legs).
    """
    t = normalize(t)
    groups = [tuple(g) for g in groups]
    assert sorted(x for g in groups for x in g) == list(range(t.rank))
    sm = t.sym_mod
    record = []
    for gi, g in enumerate(groups):
        s_r = int(t.sig[g[0]])
        cons = {}
        for b in range(t.nblocks):
            key = _block_key(t, b, g)
            cons[key] = tuple(int(t.shapes[b, x]) for x in g)
        if templates is not None and templates[gi]:
            for key, dims in templates[gi].items():
                cons.setdefault(key, dims)
        sectors = {}
        for key in sorted(cons, key=_flat):
            tot = [0] * t.nsym
            for x, q in zip(g, key):
                for c in range(t.nsym):
                    tot[c] += int(t.sig[x]) * q[c]
            nu = _nq([s_r * v for v in tot], sm)
            sectors.setdefault(nu, []).append(key)
        layout = {}
        for nu, keys in sectors.items():
            pos = 0
            for key in keys:
                dims = cons[key]
                layout[key] = (nu, pos, dims)
                pos += int(np.prod(dims))
        sector_dim = {}
        for key, (nu, pos, dims) in layout.items():
            sector_dim[nu] = max(sector_dim.get(nu, 0), pos + int(np.prod(dims)))
        record.append({"legs": g, "s": s_r, "layout": layout, "dim": sector_dim,
                       "sig": tuple(int(t.sig[x]) for x in g)})
    fblocks = {}
    for b in range(t.nblocks):
        fkey = []
        places = []
        for gi, g in enumerate(groups):
            nu, pos, dims = record[gi]["layout"][_block_key(t, b, g)]
            fkey.append(nu)
            places.append((pos, int(np.prod(dims))))
        fkey = tuple(fkey)
        if fkey not in fblocks:
            fblocks[fkey] = np.zeros(tuple(record[gi]["dim"][fkey[gi]] for gi in range(len(groups))))
        perm = [x for g in groups for x in g]
        blk = np.transpose(t.block(b), perm).reshape(tuple(p[1] for p in places))
        fblocks[fkey][tuple(slice(p, p + s) for p, s in places)] = blk
    order = sorted(fblocks, key=lambda k: _flat(k))
    rank = len(groups)
    charges = np.zeros((len(order), rank, t.nsym), dtype=np.int32)
    shapes = np.zeros((len(order), rank), dtype=np.int64)
    datas = []
    for k, key in enumerate(order):
        charges[k] = np.array(key, dtype=np.int32).reshape(rank, t.nsym)
        shapes[k] = fblocks[key].shape
        datas.append(fblocks[key].ravel())
    sizes = np.array([d.size for d in datas], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if len(order) else np.zeros(0, np.int64)
    data = np.concatenate(datas) if datas else np.zeros(0)
    out = BlockTensor(tuple(sm), np.array([r["s"] for r in record], dtype=np.int8),
                      t.n.copy(), charges, shapes, offsets, data)
    return out, record


def unfuse_legs(t: BlockTensor, records):
    """Inverse of fuse_legs: ``records[i]`` describes fused leg i (a record
    from fuse_legs).  Every constituent sub-block of every stored fused block
    becomes an original-structure block (zero-valued ones included)."""
    sm = t.sym_mod
    out = {}
    for k in range(t.nblocks):
        fkey = _block_key(t, k)
        fblk = t.block(k)
        per_leg = []
        for i, rec in enumerate(records):
            items = [(key, pos, dims) for key, (nu, pos, dims) in rec["layout"].items() if nu == fkey[i]]
            per_leg.append(items)
        for combo in itertools.product(*per_leg):
            sub = fblk[tuple(slice(pos, pos + int(np.prod(dims))) for key, pos, dims in combo)]
            shape = tuple(d for key, pos, dims in combo for d in dims)
            key = tuple(q for kk, pos, dims in combo for q in kk)
            out[key] = sub.reshape(shape)
    sig = [s for rec in records for s in rec["sig"]]
    order = sorted(out, key=_flat)
    rank = len(sig)
    nsym = len(sm)
    charges = np.zeros((len(order), rank, nsym), dtype=np.int32)
    shapes = np.zeros((len(order), rank), dtype=np.int64)
    for k, key in enumerate(order):
        charges[k] = np.array(key, dtype=np.int32).reshape(rank, nsym)
        shapes[k] = out[key].shape
    datas = [out[key].ravel() for key in order]
    sizes = np.array([d.size for d in datas], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if order else np.zeros(0, np.int64)
    return BlockTensor(tuple(sm), np.array(sig, dtype=np.int8), t.n.copy(), charges, shapes,
                       offsets, np.concatenate(datas) if datas else np.zeros(0))


def transpose(t: BlockTensor, perm):
    """Permute the legs of a block tensor; blocks re-sorted lexicographically."""
    t = normalize(t)
    perm = tuple(perm)
    keys = []
    for b in range(t.nblocks):
        key = _block_key(t, b)
        keys.append((_flat(tuple(key[p] for p in perm)), b))
    keys.sort()
    charges = np.zeros_like(t.charges)
    shapes = np.zeros_like(t.shapes)
    datas = []
    for k, (_, b) in enumerate(keys):
        charges[k] = t.charges[b][list(perm)]
        shapes[k] = t.shapes[b][list(perm)]
        datas.append(np.transpose(t.block(b), perm).ravel())
    sizes = np.array([d.size for d in datas], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if keys else np.zeros(0, np.int64)
    return BlockTensor(tuple(t.sym_mod), t.sig[list(perm)].copy(), t.n.copy(), charges, shapes,
                       offsets, np.concatenate(datas) if datas else np.zeros(0))


def dual(t: BlockTensor) -> BlockTensor:
    """The conjugate of a real block tensor: the same blocks and data with
    every signature and the total charge flipped (Sec. II.A, conjugation), so
    each of its legs contracts with the matching leg of t."""
    out = t.copy()
    out.sig = (-np.asarray(t.sig)).astype(np.int8)
    out.n = np.array(_nq(-np.asarray(t.n, dtype=np.int64), t.sym_mod), dtype=np.int32)
    return out


def tensordot_grad(a: BlockTensor, b: BlockTensor, axes_a, axes_b, dc: BlockTensor, wrt: int) -> BlockTensor:
    """Reverse mode of C = tensordot(A, B, axes) for real data: with dC the
    gradient of a scalar loss with respect to C, dA[i, k] = sum_j dC[i, j]
    B[k, j] and dB[k, j] = sum_i A[i, k] dC[i, j] (i: free legs of A, j:
    free legs of B, k: contracted).  Each is a tensordot against the dual of
    the other operand (Sec. II.B), with its legs then put back in the
    operand's order."""
    axes_a, axes_b = list(axes_a), list(axes_b)
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    if wrt == 0:
        r = tensordot_blockpair(dc, dual(b), [len(fa) + i for i in range(len(fb))], fb)
        # legs of r: A's free legs, then B's contracted legs in B's leg order
        legs = list(fa) + [axes_a[axes_b.index(l)] for l in sorted(axes_b)]
    else:
        r = tensordot_blockpair(dual(a), dc, list(fa), list(range(len(fa))))
        # legs of r: A's contracted legs in A's leg order (as B's), then B's free legs
        legs = [axes_b[axes_a.index(l)] for l in sorted(axes_a)] + list(fb)
    perm = [legs.index(l) for l in range(len(legs))]
    return transpose(r, perm)


# ---------------------------------------------------------------------------
# norms, comparisons, counts
# ---------------------------------------------------------------------------
def norms(t: BlockTensor):
    """(Frobenius norm, max |x|) over all stored blocks, in float64."""
    if t.nblocks == 0:
        return 0.0, 0.0
    vals = np.concatenate([t.block(b).ravel() for b in range(t.nblocks)])
    if vals.size == 0:
        return 0.0, 0.0
    return float(np.sqrt(np.sum(vals * vals))), float(np.max(np.abs(vals)))


def same_structure(x: BlockTensor, y: BlockTensor) -> bool:
    x, y = normalize(x), normalize(y)
    return (x.sig.tolist() == y.sig.tolist() and x.n.tolist() == y.n.tolist()
            and np.array_equal(x.charges, y.charges) and np.array_equal(x.shapes, y.shapes)
            and np.array_equal(x.offsets, y.offsets))


def rel_frobenius(got: np.ndarray, ref: np.ndarray) -> float:
    """||got - ref||_F / ||ref||_F over the concatenated blocks."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(ref * ref)))
    num = float(np.sqrt(np.sum((got - ref) ** 2)))
    return num / den if den > 0 else num


def structure_stats(a: BlockTensor, b: BlockTensor, axes_a, axes_b, elem_bytes=8):
    """Matched pairs, sectors (fused contracted charge X = sum over A's
    contracted legs of s_i rho_i), per-sector M/K/N of the fused matrices,
    useful flops (sum over matched pairs of 2 m k n) and algorithmic bytes
    (|A| + |B| + |C| stored elements, each moved once)."""
    a, b = normalize(a), normalize(b)
    fa, fb = _free(a.rank, axes_a), _free(b.rank, axes_b)
    pairs = matched_pairs(a, b, axes_a, axes_b)
    sect = {}
    flops = 0
    for i, j in pairs:
        kx = _block_key(a, i, axes_a)
        tot = [0] * a.nsym
        for x, q in zip(axes_a, kx):
            for c in range(a.nsym):
                tot[c] += int(a.sig[x]) * q[c]
        X = _nq(tot, a.sym_mod)
        m = int(np.prod([a.shapes[i, x] for x in fa])) if fa else 1
        k = int(np.prod([a.shapes[i, x] for x in axes_a])) if axes_a else 1
        n = int(np.prod([b.shapes[j, y] for y in fb])) if fb else 1
        flops += 2 * m * k * n
        s = sect.setdefault(X, {"rows": {}, "ks": {}, "cols": {}})
        s["rows"][_block_key(a, i, fa)] = m
        s["ks"][kx] = k
        s["cols"][_block_key(b, j, fb)] = n
    c = output_structure(a, b, axes_a, axes_b)
    mkn = {X: (sum(v["rows"].values()), sum(v["ks"].values()), sum(v["cols"].values()))
           for X, v in sect.items()}
    nA, nB, nC = int(a.block_sizes.sum()), int(b.block_sizes.sum()), int(c.block_sizes.sum())
    return {"pairs": len(pairs), "sectors": len(sect), "mkn": mkn, "flops": flops,
            "c_blocks": c.nblocks, "numel": (nA, nB, nC),
            "bytes": (nA + nB + nC) * elem_bytes}
