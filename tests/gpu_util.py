"""Helpers for GPU tests: upload block tensors, run the library, read back."""

import numpy as np

import paper_2405_12196_amd as Y

DEV = "cuda:0"


def torch_dtype(code):
    import torch
    return torch.float64 if code == Y.DTYPE_F64 else torch.float32


def upload(t, dtype_code=Y.DTYPE_F64):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(t.data, dtype=np.float64))
    if x.numel() == 0:
        x = torch.zeros(1, dtype=torch.float64)
    return x.to(DEV).to(torch_dtype(dtype_code))


def alloc_out(pl, p, fill=float("nan")):
    import torch
    o = pl.output(p)
    return torch.full((max(1, o.numel),), fill, dtype=torch_dtype(pl.out_dtype), device=DEV), o


def workspace(pl):
    import torch
    return torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device=DEV)


def run(problems, precision="f64", in_dtype=None, out_dtype=None, tile_rows=0, repeat=1, flags=0):
    """problems: list of (A, B, axes_a, axes_b) BlockTensors.  Returns
    (plan, [Structure], [np.float64 arrays of C values])."""
    import torch
    pl = Y.plan(problems, precision=precision, in_dtype=in_dtype, out_dtype=out_dtype, tile_rows=tile_rows,
                flags=flags)
    A = [upload(a, pl.in_dtype) for a, _, _, _ in problems]
    B = [upload(b, pl.in_dtype) for _, b, _, _ in problems]
    outs = [alloc_out(pl, p) for p in range(len(problems))]
    ws = workspace(pl)
    for _ in range(repeat):
        pl.contract(A, B, [c for c, _ in outs], ws)
    torch.cuda.synchronize()
    vals = [c.cpu().numpy()[:o.numel].astype(np.float64) for c, o in outs]
    return pl, [o for _, o in outs], vals


def structure_equal(s, ref):
    """Library output structure vs an oracle BlockTensor (bit-exact)."""
    return (s.sig.tolist() == ref.sig.tolist() and s.n.tolist() == ref.n.tolist()
            and np.array_equal(s.charges, ref.charges) and np.array_equal(s.shapes, ref.shapes)
            and np.array_equal(s.offsets, ref.offsets) and s.numel == int(ref.block_sizes.sum()))


def as_block_tensor(s, vals):
    """Library output (structure + values) as a workloads.BlockTensor."""
    from workloads import BlockTensor
    return BlockTensor(tuple(s.sym_mod), s.sig.copy(), s.n.copy(), s.charges.copy(), s.shapes.copy(),
                       s.offsets.copy(), np.asarray(vals, dtype=np.float64).copy())
