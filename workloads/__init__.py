"""Seeded synthetic inputs for the abelian-symmetric block-sparse tensordot.

This module only *builds inputs*: leg definitions for the workloads below, the
list of blocks a symmetric tensor holds, and i.i.d. N(0,1) values drawn from a
fixed seed.  It performs no matching, fusion, contraction or accumulation; both
the CPU oracle and the HIP library consume what it returns and each re-checks
the structure on its own.

Conventions (paper, Sec. II.A "Abelian-symmetric tensor"):
  * a leg is V(s, t, D): signature s = +1/-1, charge sectors t, sector dims D;
  * charges have ``nsym`` integer components; component c belongs to U(1)
    (``sym_mod[c] == 0``, charges in Z) or to Z_m (``sym_mod[c] == m >= 2``,
    charges reduced into [0, m));
  * a rank-N tensor with total charge n holds only blocks whose charge tuple
    obeys  sum_i s_i rho_i = n  (the block form of charge conservation);
  * all blocks are serialised in one 1D array (lazy storage); each block is a
    C-order dense array; ``offsets`` gives its first element.

Values: ``numpy.random.default_rng(seed).standard_normal`` fills the blocks in
ascending lexicographic order of their (normalised) charge tuples, each block
in C order.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

U1 = 0  # sym_mod entry for a U(1) component


# --------------------------------------------------------------------------
# plain containers
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Leg:
    """V(s, t, D): signature, charge sectors (tuples of nsym ints), dims."""

    s: int
    t: tuple
    D: tuple

    def conj(self) -> "Leg":
        # conjugating a leg flips its signature (paper, footnote in Sec. II.A)
        return Leg(-self.s, self.t, self.D)


@dataclass
class BlockTensor:
    """Block-sparse tensor as the C-ABI describes it (plain arrays only)."""

    sym_mod: tuple            # [nsym]
    sig: np.ndarray           # int8  [rank]
    n: np.ndarray             # int32 [nsym]
    charges: np.ndarray       # int32 [nblocks, rank, nsym]
    shapes: np.ndarray        # int64 [nblocks, rank]
    offsets: np.ndarray       # int64 [nblocks]
    data: np.ndarray          # float64 [numel]
    meta: dict = field(default_factory=dict)

    @property
    def rank(self) -> int:
        return int(self.sig.shape[0])

    @property
    def nsym(self) -> int:
        return len(self.sym_mod)

    @property
    def nblocks(self) -> int:
        return int(self.charges.shape[0])

    @property
    def block_sizes(self) -> np.ndarray:
        if self.nblocks == 0:
            return np.zeros(0, dtype=np.int64)
        return np.prod(self.shapes, axis=1).astype(np.int64)

    @property
    def numel(self) -> int:
        """Length of the 1D buffer (end of the last block)."""
        if self.nblocks == 0:
            return 0
        return int(np.max(self.offsets + self.block_sizes))

    def block(self, i: int) -> np.ndarray:
        off = int(self.offsets[i])
        shp = tuple(int(x) for x in self.shapes[i])
        size = int(np.prod(shp)) if shp else 1
        return self.data[off:off + size].reshape(shp)

    def copy(self) -> "BlockTensor":
        return BlockTensor(tuple(self.sym_mod), self.sig.copy(), self.n.copy(),
                           self.charges.copy(), self.shapes.copy(),
                           self.offsets.copy(), self.data.copy(), dict(self.meta))


def _norm_charge(q, sym_mod):
    return tuple(int(v) % m if m else int(v) for v, m in zip(q, sym_mod))


def allowed_tuples(legs, n, sym_mod):
    """Every sector-index tuple whose charges satisfy sum_i s_i rho_i = n.

    Returned in ascending lexicographic order of the normalised charge tuple.
    """
    nsym = len(sym_mod)
    n = _norm_charge(n, sym_mod)
    per_leg = []
    for leg in legs:
        items = sorted(((_norm_charge(q, sym_mod), d) for q, d in zip(leg.t, leg.D)))
        per_leg.append(items)
    out = []
    for combo in itertools.product(*per_leg):
        tot = [0] * nsym
        for leg, (q, _) in zip(legs, combo):
            for c in range(nsym):
                tot[c] += leg.s * q[c]
        if _norm_charge(tot, sym_mod) == n:
            out.append(combo)
    return out


def rand(legs, n, sym_mod, seed, *, keep=None, shuffle_seed=None, gap=0):
    """Random symmetric tensor on ``legs`` with total charge ``n``.

    ``keep``: optional fraction in (0, 1]; a seeded subset of the allowed blocks
    is kept (lazy storage holds any subset).  ``shuffle_seed``: permute the
    order of blocks in the 1D buffer (block table stays lexicographic).
    ``gap``: number of unused elements between consecutive blocks in the
    buffer (the layout need not be dense).
    """
    sym_mod = tuple(sym_mod)
    combos = allowed_tuples(legs, n, sym_mod)
    if keep is not None and keep < 1.0 and combos:
        sel = np.random.default_rng(seed + 7919).random(len(combos)) < keep
        combos = [c for c, k in zip(combos, sel) if k]
    rank, nsym = len(legs), len(sym_mod)
    nb = len(combos)
    charges = np.zeros((nb, rank, nsym), dtype=np.int32)
    shapes = np.zeros((nb, rank), dtype=np.int64)
    for b, combo in enumerate(combos):
        for i, (q, d) in enumerate(combo):
            charges[b, i, :] = q
            shapes[b, i] = d
    sizes = np.prod(shapes, axis=1).astype(np.int64) if nb else np.zeros(0, np.int64)
    order = np.arange(nb)
    if shuffle_seed is not None and nb:
        order = np.random.default_rng(shuffle_seed).permutation(nb)
    offsets = np.zeros(nb, dtype=np.int64)
    pos = 0
    for b in order:
        offsets[b] = pos
        pos += int(sizes[b]) + gap
    total = pos
    data = np.zeros(total, dtype=np.float64)
    vals = np.random.default_rng(seed).standard_normal(int(sizes.sum()) if nb else 0)
    v = 0
    for b in range(nb):  # fill in lexicographic block order, each in C order
        sz = int(sizes[b])
        data[offsets[b]:offsets[b] + sz] = vals[v:v + sz]
        v += sz
    return BlockTensor(sym_mod, np.array([l.s for l in legs], dtype=np.int8),
                       np.array(_norm_charge(n, sym_mod), dtype=np.int32),
                       charges, shapes, offsets, data, {"seed": seed})


def conj(t: BlockTensor) -> BlockTensor:
    """Conjugate of a real tensor: flip every signature, n -> -n, same data."""
    out = t.copy()
    out.sig = (-t.sig).astype(np.int8)
    out.n = np.array(_norm_charge([-int(v) for v in t.n], t.sym_mod), dtype=np.int32)
    return out


# --------------------------------------------------------------------------
# workload definitions
# --------------------------------------------------------------------------
@dataclass
class Contraction:
    """One tensordot: C = A . B over axes (axes_a, axes_b)."""

    a: BlockTensor
    b: BlockTensor
    axes_a: tuple
    axes_b: tuple
    name: str = ""


def _u1_leg(s, pairs):
    return Leg(s, tuple((q,) for q, _ in pairs), tuple(d for _, d in pairs))


def _leg2(s, pairs):
    return Leg(s, tuple(tuple(q) for q, _ in pairs), tuple(d for _, d in pairs))


# ---- single U(1) rank-4 tensordot (D = 18) -------------------------------
D18_LEG = [(-2, 2), (-1, 4), (0, 6), (1, 4), (2, 2)]
SIG_PPMM = (1, 1, -1, -1)


def rank4_u1_problem(leg_pairs, seed_a, seed_b, name=""):
    legs = [_u1_leg(s, leg_pairs) for s in SIG_PPMM]
    a = rand(legs, (0,), (U1,), seed_a)
    b = rand(legs, (0,), (U1,), seed_b)
    return Contraction(a, b, (2, 3), (0, 1), name)


def u1_d18(batch: int = 1):
    """U(1) rank-4, signature (+,+,-,-), legs {-2:2,-1:4,0:6,1:4,2:2};
    A seed 101+2i, B seed 102+2i; contract A's legs (2,3) with B's (0,1)."""
    return [rank4_u1_problem(D18_LEG, 101 + 2 * i, 102 + 2 * i, f"u1_d18[{i}]")
            for i in range(batch)]


# ---- CTMRG enlarged corner, U(1)xU(1), chi = 128 / 256 ------------------------
def _ctm_legs_u1u1(chi):
    if chi == 128:
        e = [((0, 0), 20)]
        e += [(q, 14) for q in [(1, 0), (-1, 0), (0, 1), (0, -1)]]
        e += [(q, 8) for q in [(1, 1), (1, -1), (-1, 1), (-1, -1)]]
        e += [(q, 6) for q in [(0, 2), (0, -2)]]
        e += [(q, 2) for q in [(1, 2), (1, -2), (-1, 2), (-1, -2)]]
        v = [((0, 0), 4)] + [(q, 1) for q in [(1, 0), (-1, 0), (0, 1), (0, -1)]]
    elif chi == 256:
        e = []
        for q1 in range(-2, 3):
            for q2 in range(-2, 3):
                l1 = abs(q1) + abs(q2)
                if (q1, q2) == (0, 0):
                    d = 20
                elif l1 == 1:
                    d = 18
                elif abs(q1) == 1 and abs(q2) == 1:
                    d = 14
                elif l1 == 2:
                    d = 12
                elif l1 == 3:
                    d = 6
                else:
                    d = 3
                e.append(((q1, q2), d))
        v = [(q, 2) for q in [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]]
    else:
        raise ValueError("chi must be 128 or 256")
    p = [(q, 1) for q in [(0, 0), (1, 0), (0, 1), (1, 1)]]
    return e, v, p


CTM_AXES = [((1,), (0,)), ((0,), (0,)), ((0, 3), (0, 1)), ((0, 2, 6), (0, 1, 4))]


def ctm_tensors(E, V, P, sym_mod, seeds, mk):
    """C(d,r), T1(l,k,b,r), T4(t,k,b,bot), A(t,l,b,r,p), A* for an enlarged
    corner.  ``mk(s, pairs)`` builds a leg; signatures as in the workload."""
    C = rand([mk(-1, E), mk(1, E)], (0,) * len(sym_mod), sym_mod, seeds[0])
    T1 = rand([mk(-1, E), mk(-1, V), mk(1, V), mk(1, E)], (0,) * len(sym_mod), sym_mod, seeds[1])
    T4 = rand([mk(1, E), mk(-1, V), mk(1, V), mk(-1, E)], (0,) * len(sym_mod), sym_mod, seeds[2])
    A = rand([mk(1, V), mk(1, V), mk(-1, V), mk(-1, V), mk(1, P)], (0,) * len(sym_mod), sym_mod, seeds[3])
    return {"C": C, "T1": T1, "T4": T4, "A": A, "Ac": conj(A)}


def ctm(chi: int = 128, seeds=(201, 202, 203, 204)):
    """CTMRG enlarged-corner step, U(1)xU(1), FP64: chi=128 (15 sectors),
    D=8 (5 sectors), d=4.  Returns the tensors; the four chained steps are
    C.T1 ((1),(0)), .T4 ((0),(0)), .A ((0,3),(0,1)), .A* ((0,2,6),(0,1,4))."""
    E, V, P = _ctm_legs_u1u1(chi)
    t = ctm_tensors(E, V, P, (U1, U1), seeds, _leg2)
    t["axes"] = CTM_AXES
    t["name"] = f"ctm_u1xu1_chi{chi}"
    return t


def ctm_chi256():
    """The enlarged-corner step at chi=256, D=10 (precision sweep), seeds 401-404."""
    return ctm(256, seeds=(401, 402, 403, 404))


# ---- 64 independent U(1) contractions, uneven D ----------------------------
def u1_uneven(nprob: int = 64, seed: int = 3):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(nprob):
        D = int(rng.integers(12, 41))
        k = int(rng.integers(3, 10))
        dims = [1] * k
        for _ in range(D - k):
            j = int(rng.choice([j for j in range(k) if dims[j] < 16]))
            dims[j] += 1
        q0 = -((k - 1) // 2)
        pairs = [(q0 + j, dims[j]) for j in range(k)]
        probs.append(rank4_u1_problem(pairs, 3000 + 2 * i, 3001 + 2 * i, f"u1_uneven[{i}]"))
    return probs


# ---- serving mix of 32 CTMRG runs -------------------------------------------------
U1_E = {64: [2, 4, 7, 11, 16, 11, 7, 4, 2], 128: [4, 8, 15, 22, 30, 22, 15, 8, 4],
        192: [6, 11, 23, 33, 46, 33, 23, 11, 6], 256: [8, 15, 30, 45, 60, 45, 30, 15, 8]}
U1_V = {4: [(-1, 1), (0, 2), (1, 1)], 6: [(-1, 2), (0, 2), (1, 2)],
        8: [(-2, 1), (-1, 2), (0, 2), (1, 2), (2, 1)],
        10: [(-2, 1), (-1, 2), (0, 4), (1, 2), (2, 1)]}


def serving_run(run: int):
    """Run ``run`` of the 32-run serving mix: runs 0-15 Z2, 16-31 U(1); each
    symmetry cycles D in {4,6,8,10} x chi in {64,128,192,256}."""
    sym = "Z2" if run < 16 else "U1"
    r = run % 16
    D = (4, 6, 8, 10)[r // 4]
    chi = (64, 128, 192, 256)[r % 4]
    base = (5000 + run) * 10
    seeds = (base + 1, base + 2, base + 3, base + 4)
    if sym == "Z2":
        E = [((0,), chi // 2), ((1,), chi // 2)]
        V = [((0,), D // 2), ((1,), D // 2)]
        P = [((0,), 2), ((1,), 2)]
        t = ctm_tensors(E, V, P, (2,), seeds, _leg2)
    else:
        E = [((q,), d) for q, d in zip(range(-4, 5), U1_E[chi])]
        V = [((q,), d) for q, d in U1_V[D]]
        P = [((0,), 1), ((1,), 2), ((2,), 1)]
        t = ctm_tensors(E, V, P, (U1,), seeds, _leg2)
    t["axes"] = CTM_AXES
    t["name"] = f"serve_{sym}_D{D}_chi{chi}"
    t["sym"], t["D"], t["chi"] = sym, D, chi
    return t


# ---- the paper's worked example --------------------------------------------
def spin_half_pair_hamiltonian():
    """H = S1.S2 for two spin-1/2 as a U(1) tensor on legs (l, l, l*, l*),
    l = V(+1, t=(-1, 1), D=(1, 1)), charge = 2 S^z, H[t0,t1,t2,t3] =
    <t0 t1|H|t2 t3>  (paper, Sec. II.A listing and the remark after it)."""
    l = _u1_leg(1, [(-1, 1), (1, 1)])
    legs = [l, l, l.conj(), l.conj()]
    t = rand(legs, (0,), (U1,), seed=0)
    val = {(1, 1, 1, 1): 0.25, (-1, -1, -1, -1): 0.25,
           (1, -1, 1, -1): -0.25, (-1, 1, -1, 1): -0.25,
           (1, -1, -1, 1): 0.5, (-1, 1, 1, -1): 0.5}
    for b in range(t.nblocks):
        key = tuple(int(q) for q in t.charges[b, :, 0])
        t.data[t.offsets[b]] = val[key]
    return t


# ---- a 1x1 unit cell of the CTM environment: the left move ------------------
def ctm_env(E, V, P, sym_mod, seeds, mk=_leg2):
    """Corners C1 (top-left), C2 (top-right), C3 (bottom-right), C4 (bottom-left),
    edges T1 (top), T2 (right), T3 (bottom), T4 (left), the site tensor A and
    its conjugate, all of total charge 0, on legs E (environment), V (virtual)
    and P (physical).  Leg order and signatures (every bond joins a +1 leg to a
    -1 leg of the same space):
        C1 (d -, r +)  C2 (l -, d -)  C3 (u +, l -)  C4 (u +, r +)
        T1 (l -, k -, b +, r +)   T2 (t +, k +, b -, bot -)
        T3 (l -, k +, b -, r +)   T4 (t +, k -, b +, bot -)
        A  (t +, l +, b -, r -, p +),  A* = A with every signature flipped
    where k / b are an edge's legs to the ket / bra layer of the site.
    ``seeds``: nine seeds, for C1, T1, T4, A, C2, C3, C4, T2, T3 in that order
    (so C1, T1, T4, A coincide with ``ctm_tensors`` for the same first four)."""
    z = (0,) * len(sym_mod)
    s = dict(zip(("C1", "T1", "T4", "A", "C2", "C3", "C4", "T2", "T3"), seeds))
    env = {
        "C1": rand([mk(-1, E), mk(1, E)], z, sym_mod, s["C1"]),
        "C2": rand([mk(-1, E), mk(-1, E)], z, sym_mod, s["C2"]),
        "C3": rand([mk(1, E), mk(-1, E)], z, sym_mod, s["C3"]),
        "C4": rand([mk(1, E), mk(1, E)], z, sym_mod, s["C4"]),
        "T1": rand([mk(-1, E), mk(-1, V), mk(1, V), mk(1, E)], z, sym_mod, s["T1"]),
        "T2": rand([mk(1, E), mk(1, V), mk(-1, V), mk(-1, E)], z, sym_mod, s["T2"]),
        "T3": rand([mk(-1, E), mk(1, V), mk(-1, V), mk(1, E)], z, sym_mod, s["T3"]),
        "T4": rand([mk(1, E), mk(-1, V), mk(1, V), mk(-1, E)], z, sym_mod, s["T4"]),
        "A": rand([mk(1, V), mk(1, V), mk(-1, V), mk(-1, V), mk(1, P)], z, sym_mod, s["A"]),
    }
    env["Ac"] = conj(env["A"])
    return env


ENV_NAMES = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4", "A")


def ctm_move_u1xu1(chi: int = 128):
    """The left move at chi = 128, D = 8, d = 4 (U(1)xU(1), the legs of the
    enlarged-corner workload; C1, T1, T4, A are its tensors), new chi = chi."""
    E, V, P = _ctm_legs_u1u1(chi)
    base = (201, 202, 203, 204) if chi == 128 else (401, 402, 403, 404)
    env = ctm_env(E, V, P, (U1, U1), base + tuple(base[0] + 4 + i for i in range(5)))
    env["chi"] = chi
    env["name"] = f"ctm_move_u1xu1_chi{chi}"
    return env


CTM_SMALL = {
    # name: (E, V, P, sym_mod); charges as tuples of one or two components
    "u1": ([((-1,), 2), ((0,), 3), ((1,), 2)], [((-1,), 1), ((0,), 1), ((1,), 1)],
           [((-1,), 1), ((1,), 1)], (U1,)),
    "z2": ([((0,), 4), ((1,), 3)], [((0,), 2), ((1,), 1)], [((0,), 1), ((1,), 1)], (2,)),
    "u1xu1": ([((0, 0), 3), ((1, 0), 1), ((-1, 0), 1), ((0, 1), 1), ((0, -1), 1)],
              [((0, 0), 1), ((1, 0), 1), ((0, -1), 1)], [((0, 0), 1), ((1, 1), 1)], (U1, U1)),
    "u1_mid": ([((-2,), 3), ((-1,), 6), ((0,), 8), ((1,), 6), ((2,), 3)],
               [((-1,), 1), ((0,), 2), ((1,), 1)], [((-1,), 1), ((1,), 1)], (U1,)),
}


def ctm_move_small(name: str, seed: int = 700):
    """Small left-move cases for exact checks (dense arrays of a few MB at most)."""
    E, V, P, sm = CTM_SMALL[name]
    env = ctm_env(E, V, P, sm, tuple(seed + i for i in range(9)))
    env["chi"] = sum(d for _, d in E)
    env["name"] = f"ctm_move_{name}"
    return env


# ---- complex values and fermionic charges ------------------------------------
def rand_complex(legs, n, sym_mod, seed, **kw):
    """As ``rand`` with complex128 values: one N(0,1) stream from ``seed``
    gives each element's real and imaginary parts in turn (blocks in ascending
    charge order, each in C order)."""
    t = rand(legs, n, sym_mod, seed, **kw)
    nb = t.nblocks
    sizes = np.prod(t.shapes, axis=1).astype(np.int64) if nb else np.zeros(0, np.int64)
    vals = np.random.default_rng(seed).standard_normal(2 * int(sizes.sum()))
    data = np.zeros(t.data.size, dtype=np.complex128)
    v = 0
    for b in range(nb):
        sz = int(sizes[b])
        data[t.offsets[b]:t.offsets[b] + sz] = vals[v:v + 2 * sz:2] + 1j * vals[v + 1:v + 2 * sz:2]
        v += 2 * sz
    t.data = data
    return t


def complex_ctm(chi: int = 128):
    """The enlarged-corner workload (``ctm``) with complex128 values on every
    tensor (seeds 201-204 as there; A* = conj(A): flipped signatures and
    conjugated values)."""
    E, V, P = _ctm_legs_u1u1(chi)
    z = (0, 0)
    sm = (U1, U1)
    t = {"C": rand_complex([_leg2(-1, E), _leg2(1, E)], z, sm, 201),
         "T1": rand_complex([_leg2(-1, E), _leg2(-1, V), _leg2(1, V), _leg2(1, E)], z, sm, 202),
         "T4": rand_complex([_leg2(1, E), _leg2(-1, V), _leg2(1, V), _leg2(-1, E)], z, sm, 203),
         "A": rand_complex([_leg2(1, V), _leg2(1, V), _leg2(-1, V), _leg2(-1, V), _leg2(1, P)], z, sm, 204)}
    t["axes"] = CTM_AXES
    t["name"] = f"ctm_u1xu1_chi{chi}_c128"
    return t


# fermionic charge components per symmetry: parity = sum of those mod 2
FERMIONIC = {(2,): (1,), (U1,): (1,), (U1, U1): (1, 1)}
