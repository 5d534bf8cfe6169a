"""Complex conjugation, fermionic parity and swap gates (test infrastructure).

  * ``conj``: the conjugate of a block tensor -- every leg mapped to its dual
    space, which flips the leg's signature and complex-conjugates the elements
    (Sec. II.A, footnote on conjugation); the total charge flips with the
    signatures.  For real values it is ``dual``.
  * ``parity``: the fermionic parity of a charge, the sum of its fermionic
    components mod 2 (Z2 parity itself; for U(1) or U(1)xU(1) particle
    numbers, the total particle number mod 2).
  * ``swap_gate``: the swap gate between two groups of legs of one tensor
    (Sec. III, fermionic Hubbard example: the fermionic order is imposed by
    swap gates on every line crossing, and a swap gate changes the sign of
    the blocks whose charges have odd parity on both swapped legs).  For
    groups G1 and G2 each block is multiplied by (-1)^(P1 P2), P_k the parity
    of the summed charge of group k -- the product of the swap gates of every
    pair (i in G1, j in G2).
  * ``tensordot_c``: tensordot of complex tensors, either operand optionally
    conjugated first (the block-pair oracle O2 in complex arithmetic).
"""

from __future__ import annotations

import numpy as np

from workloads import BlockTensor

from .blocksparse import dual, tensordot_blockpair


def conj(t: BlockTensor) -> BlockTensor:
    out = dual(t)
    out.data = np.conj(np.asarray(t.data))
    return out


def parity(q, fermionic) -> int:
    return int(sum(int(f) * int(v) for v, f in zip(q, fermionic))) % 2


def swap_gate(t: BlockTensor, legs1, legs2, fermionic) -> BlockTensor:
    out = t.copy()
    for b in range(t.nblocks):
        p1 = sum(parity(t.charges[b, i], fermionic) for i in legs1) % 2
        p2 = sum(parity(t.charges[b, j], fermionic) for j in legs2) % 2
        if p1 and p2:
            o = int(t.offsets[b])
            sz = int(np.prod(t.shapes[b]))
            out.data[o:o + sz] = -np.asarray(t.data)[o:o + sz]
    return out


def tensordot_c(a: BlockTensor, b: BlockTensor, axes_a, axes_b, conj_a=False, conj_b=False) -> BlockTensor:
    return tensordot_blockpair(conj(a) if conj_a else a, conj(b) if conj_b else b, axes_a, axes_b)
