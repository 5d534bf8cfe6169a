"""Seeded random block-sparse problems for tests (input construction only)."""

import numpy as np

from workloads import Leg, rand

SYMS = {"U1": (0,), "Z2": (2,), "Z3": (3,), "U1xU1": (0, 0), "U1xZ2": (0, 2)}


def random_leg(rng, sym_mod, s, max_sectors=3, max_dim=3):
    nsec = int(rng.integers(1, max_sectors + 1))
    seen = set()
    t, D = [], []
    for _ in range(nsec * 3):
        q = tuple(int(rng.integers(0, m)) if m else int(rng.integers(-2, 3)) for m in sym_mod)
        if q in seen:
            continue
        seen.add(q)
        t.append(q)
        D.append(int(rng.integers(1, max_dim + 1)))
        if len(t) == nsec:
            break
    return Leg(s, tuple(t), tuple(D))


def random_problem(seed, sym="U1", rank_a=None, rank_b=None, ncon=None, keep=None,
                   max_sectors=3, max_dim=3, shuffle=False, drop_partner=False):
    """A and B with random legs; contracted legs of B are the conjugates of the
    matching legs of A (same charges and dims, opposite signature).  With
    ``drop_partner`` some contracted charges exist on one side only."""
    rng = np.random.default_rng(seed)
    sym_mod = SYMS[sym]
    ra = int(rng.integers(1, 5)) if rank_a is None else rank_a
    rb = int(rng.integers(1, 5)) if rank_b is None else rank_b
    nc = int(rng.integers(0, min(ra, rb) + 1)) if ncon is None else ncon
    legs_a = [random_leg(rng, sym_mod, int(rng.choice([-1, 1])), max_sectors, max_dim) for _ in range(ra)]
    axes_a = tuple(int(x) for x in rng.permutation(ra)[:nc])
    axes_b = tuple(int(x) for x in rng.permutation(rb)[:nc])
    legs_b = [random_leg(rng, sym_mod, int(rng.choice([-1, 1])), max_sectors, max_dim) for _ in range(rb)]
    for x, y in zip(axes_a, axes_b):
        la = legs_a[x]
        lb = la.conj()
        if drop_partner and len(la.t) > 1 and rng.random() < 0.5:
            lb = Leg(lb.s, lb.t[1:], lb.D[1:])
        legs_b[y] = lb
    n_a = tuple(int(rng.integers(0, m)) if m else int(rng.integers(-1, 2)) for m in sym_mod)
    n_b = tuple(int(rng.integers(0, m)) if m else int(rng.integers(-1, 2)) for m in sym_mod)
    a = rand(legs_a, n_a, sym_mod, seed * 2 + 11, keep=keep,
             shuffle_seed=(seed + 5) if shuffle else None, gap=1 if shuffle else 0)
    b = rand(legs_b, n_b, sym_mod, seed * 2 + 12, keep=keep,
             shuffle_seed=(seed + 6) if shuffle else None)
    return a, b, axes_a, axes_b
