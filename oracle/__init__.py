"""CPU FP64 oracle for the abelian-symmetric block-sparse tensordot.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the test-suite, the smoke check and the benchmark's CPU-baseline leg may call
it.  It is slow and obviously correct by construction, and shares no code with
the HIP path (the only common module is the seeded input generator
``workloads``, which holds no contraction arithmetic).

Implementations (each cites the passage of the paper it follows):
  * ``tensordot_dense``    (O1) embed every block in a dense array, contract
                           with numpy.tensordot, read the blocks back;
  * ``tensordot_blockpair`` (O2) sum numpy.tensordot over matched block pairs;
  * ``tensordot_blocks``   O2 for chosen output blocks only (full-size samples);
  * ``tensordot_brute``    (O3) pure-Python loops over every dense index;
  * ``fuse_legs`` / ``unfuse_legs`` (O-fuse) leg fusion and its inverse;
  * ``transpose``          leg permutation of a block tensor;
  * ``dual`` / ``tensordot_grad`` the conjugate and the reverse-mode gradient
                           of a tensordot with respect to either operand;
  * ``validate_*``         structural checks with the library's status classes;
  * ``norms``              Frobenius norm and max-abs of a block tensor;
  * ``structure_stats``    matched pairs, sectors, useful flops, bytes;
  * ``svd.*``              the block-sparse truncated SVD of a block tensor
                           (sector matrices, per-sector SVD, the global
                           truncation rule, the kept factors as block tensors);
  * ``ctm.left_move``      one CTM move on a 1x1 unit cell: four enlarged
                           corners, the halves and their product, its
                           truncated SVD, the projectors, the renormalised
                           left column;
  * ``fermionic.*``        complex conjugation, fermionic parity, swap gates,
                           and the complex tensordot (O2 in complex128).

Every function is pinned by tests that do not re-use its own formula (closed
forms, the paper's worked example, brute force, special cases that reduce to
plain numpy.tensordot, invariants); see tests/test_oracle_*.py.
"""

from .blocksparse import (  # noqa: F401
    OracleError, ERR_ARG, ERR_SYM, ERR_CHARGE, ERR_SIGNATURE, ERR_SHAPE,
    ERR_DUPLICATE, normalize, validate_tensor, validate_pair, output_structure,
    tensordot_dense, tensordot_blockpair, tensordot_blocks, tensordot_brute, to_dense,
    leg_index_maps, fuse_legs, unfuse_legs, transpose, dual, tensordot_grad, norms, structure_stats,
    rel_frobenius, same_structure,
)
from . import svd  # noqa: F401
from . import ctm  # noqa: F401
from . import fermionic  # noqa: F401
