"""CPU replay of the kernels' indexing against the oracle (no GPU).

tests/emu/emu.cpp compiles the library's planner (host.cpp) and address
helpers (index.hpp) with g++ and replays the pack and GEMM loops on the CPU,
checking every read and write against its buffer and that each output element
is written exactly once.  Its results must match the oracle, so a wrong
offset formula or tiling is caught here before any kernel runs on a GPU.
"""

import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import paper_2405_12196_amd as Y
import workloads as W
from tests.helpers import random_problem

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "emu", "libemu.so")


@pytest.fixture(scope="module")
def emu():
    src = [os.path.join(HERE, "emu", "emu.cpp"), os.path.join(ROOT, "paper_2405_12196_amd", "csrc", "host.cpp")]
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-o", SO] + src,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    L = C.CDLL(SO)
    L.emu_plan.restype = C.c_void_p
    L.emu_plan.argtypes = [C.POINTER(Y.Problem), C.c_int, C.c_int, C.c_int]
    L.emu_output.argtypes = [C.c_void_p, C.c_int, C.POINTER(Y.TensorDesc), C.POINTER(C.c_int64)]
    L.emu_contract.argtypes = [C.c_void_p] + [C.POINTER(C.c_void_p), C.POINTER(C.c_int64)] * 3
    L.emu_contract.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                               C.POINTER(C.c_int64), C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]
    L.emu_error.restype = C.c_char_p
    L.emu_set_pack_gather.argtypes = [C.c_int]
    L.emu_free.argtypes = [C.c_void_p]
    return L


def run_emu(L, problems, cb=4, rb=4):
    keep = Y._Keep()
    arr = (Y.Problem * len(problems))()
    for i, (a, b, xa, xb) in enumerate(problems):
        arr[i].a = Y._desc(a, keep)
        arr[i].b = Y._desc(b, keep)
        arr[i].ncontract = len(xa)
        arr[i].axes_a = keep.ptr(np.array(xa, np.int32), C.c_int32)
        arr[i].axes_b = keep.ptr(np.array(xb, np.int32), C.c_int32)
    h = L.emu_plan(arr, len(problems), rb, cb)
    assert h, L.emu_error().decode()
    outs = []
    for p in range(len(problems)):
        d, n = Y.TensorDesc(), C.c_int64()
        L.emu_output(h, p, C.byref(d), C.byref(n))
        nb, r, s = d.nblocks, d.rank, d.nsym
        cp = (lambda ptr, cnt, dt: np.ctypeslib.as_array(ptr, shape=(cnt,)).astype(dt) if cnt else np.zeros(0, dt))
        outs.append((cp(d.charges, nb * r * s, np.int32).reshape(nb, r, s), cp(d.shapes, nb * r, np.int64).reshape(nb, r),
                     cp(d.offsets, nb, np.int64), int(n.value)))
    np_ = len(problems)
    A = [np.ascontiguousarray(a.data if a.data.size else np.zeros(1)) for a, _, _, _ in problems]
    B = [np.ascontiguousarray(b.data if b.data.size else np.zeros(1)) for _, b, _, _ in problems]
    Cc = [np.full(max(1, o[3]), np.nan) for o in outs]
    ptrs = lambda xs: (C.c_void_p * np_)(*[x.ctypes.data for x in xs])
    lens = lambda xs, real: (C.c_int64 * np_)(*real)
    rc = L.emu_contract(h, ptrs(A), lens(A, [a.data.size for a, _, _, _ in problems]), ptrs(B),
                        lens(B, [b.data.size for _, b, _, _ in problems]), ptrs(Cc), lens(Cc, [o[3] for o in outs]))
    msg = L.emu_error().decode()
    L.emu_free(h)
    assert rc == 0, msg
    return [(o, c[:o[3]]) for o, c in zip(outs, Cc)]


def check(res, ref):
    (charges, shapes, offsets, numel), vals = res
    assert np.array_equal(charges, ref.charges) and np.array_equal(shapes, ref.shapes)
    assert np.array_equal(offsets, ref.offsets) and numel == int(ref.block_sizes.sum())
    assert oracle.rel_frobenius(vals, ref.data) <= 1e-12


def test_emu_u1_d18(emu):
    (p,) = W.u1_d18()
    (res,) = run_emu(emu, [(p.a, p.b, p.axes_a, p.axes_b)])
    check(res, oracle.tensordot_dense(p.a, p.b, p.axes_a, p.axes_b))


@pytest.mark.parametrize("rb", [1, 2, 4])
@pytest.mark.parametrize("cb", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", range(12))
def test_emu_random(emu, seed, cb, rb):
    sym = ["U1", "Z2", "U1xZ2", "Z3", "U1xU1"][seed % 5]
    a, b, xa, xb = random_problem(seed + 2000, sym, rank_a=1 + seed % 5, rank_b=1 + (seed // 5) % 5,
                                  max_sectors=4, max_dim=5 + seed % 7, keep=0.75 if seed % 3 else None,
                                  shuffle=seed % 4 == 0, drop_partner=seed % 6 == 1)
    (res,) = run_emu(emu, [(a, b, xa, xb)], cb, rb)
    check(res, oracle.tensordot_blockpair(a, b, xa, xb))


def test_emu_interleaved_legs(emu):
    # rank-7 A with contracted legs spread out: four free-leg classes
    for seed in range(6):
        a, b, xa, xb = random_problem(seed + 7000, "U1", rank_a=7, rank_b=4, ncon=3, max_sectors=2, max_dim=3)
        (res,) = run_emu(emu, [(a, b, xa, xb)])
        check(res, oracle.tensordot_blockpair(a, b, xa, xb))


def test_emu_ctm_steps_1_to_3(emu):
    t = W.ctm()
    cur = None
    for (an, bn), (ax, bx) in zip([("C", "T1"), (None, "T4"), (None, "A")], t["axes"][:3]):
        a = t[an] if an else cur
        ref = oracle.tensordot_blockpair(a, t[bn], ax, bx)
        (res,) = run_emu(emu, [(a, t[bn], ax, bx)], 3)
        check(res, ref)
        cur = ref


def test_emu_u1_uneven_batch(emu):
    probs = [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_uneven(12)]
    for res, (a, b, xa, xb) in zip(run_emu(emu, probs), probs):
        check(res, oracle.tensordot_blockpair(a, b, xa, xb))


@pytest.mark.parametrize("seed", range(6))
def test_emu_subblock_pack(emu, seed):
    # the stride-computed pack items (taken when B offsets overflow int32)
    emu.emu_set_pack_gather(0)
    try:
        sym = ["U1", "Z2", "U1xU1"][seed % 3]
        a, b, xa, xb = random_problem(seed + 4000, sym, rank_a=2 + seed % 3, rank_b=2 + (seed // 3) % 3,
                                      max_sectors=4, max_dim=6, keep=0.75 if seed % 2 else None,
                                      shuffle=seed % 2 == 0, drop_partner=seed == 3)
        probs = [(a, b, xa, xb)] + [(p.a, p.b, p.axes_a, p.axes_b) for p in W.u1_uneven(3, seed=seed)]
        for res, (a, b, xa, xb) in zip(run_emu(emu, probs), probs):
            check(res, oracle.tensordot_blockpair(a, b, xa, xb))
    finally:
        emu.emu_set_pack_gather(1)
