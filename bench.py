#!/usr/bin/env python3
"""Benchmark: one CTMRG enlarged-corner step on one MI355X.

Workload (FP64, U(1)xU(1)): environment chi = 128 in 15 sectors, bond D = 8
in 5 sectors, physical d = 4; four chained block-sparse tensordots
    C.T1 ((1),(0)),  .T4 ((0),(0)),  .A ((0,3),(0,1)),  .A* ((0,2,6),(0,1,4))
followed by the FP64 Frobenius/max norm of the last output (the input of the
CTM truncation).  Synthetic i.i.d. N(0,1) blocks, fixed seeds.  Plans are
built once before timing (the block structure repeats across CTM iterations).

A step = the four contractions + the norm.  value = useful TFLOP/s
(sum over matched block pairs of 2 m k n, over the four contractions) per
step time.  Also reported: p50/p99 step latency, the same step in the plain
per-sector FP64 form on the same GPU (gather each operand into its fused
sector matrices, one torch.matmul per sector, scatter back), the roofline of
the dominant kernel (HIP events on the launch stream), and the CPU oracle
(block-pair form) timed on the host cores on a bounded sample.
"""

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6      # MI355X dense FP64 matrix
STEPS = [("C", "T1"), (None, "T4"), (None, "A"), (None, "Ac")]


# ------------------------------------------------------------------ HIP events
class HipEvents:
    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.made = []

    def new(self):
        e = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
        self.made.append(e.value)
        return e.value

    def record(self, e, stream):
        assert self.hip.hipEventRecord(ctypes.c_void_p(e), ctypes.c_void_p(stream)) == 0

    def ms(self, a, b):
        f = ctypes.c_float()
        assert self.hip.hipEventElapsedTime(ctypes.byref(f), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return float(f.value)

    def close(self):
        for e in self.made:
            self.hip.hipEventDestroy(ctypes.c_void_p(e))


# ------------------------------------------------------- measured traffic
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ctm_corner_chi128_D8_f64_hbm_traffic.json")


# the sources that define the contraction kernels, their instances, tables
# and launches (the counters in profiles/ are valid while these are unchanged)
CONTRACTION_SOURCES = ("device.hip", "dispatch.hpp", "host.cpp", "index.hpp", "inst_f64.hip", "inst_lds.hip",
                       "inst_lds_norm.hip", "inst_ldsk.hip", "kernels.hpp", "lds_select.hpp", "plan.hpp",
                       "planner.hpp")


def kernel_source_hash():
    """sha256 over the contraction kernels' sources."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2405_12196_amd", "csrc")
    for f in CONTRACTION_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(step, variant):
    """HBM bytes per launch of contraction `step` (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy), from the committed counter summary; None when the
    kernels changed since the counters were taken or another variant runs."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = rec.get("per_launch", {}).get(f"step{step}_v{variant}")
    return int(e["fetch_bytes"] + e["write_bytes"]) if e else None


def steps_timed(torch, ev, sp, fn, K):
    """(ms per step, per-step latencies in ms): K steps back to back between
    two synchronisations, wall clock (a HIP event recorded between steps
    stalls the queue for ~10 us, so none is recorded in this pass); then K
    more steps, each bracketed by HIP events on the launch stream, for the
    latency percentiles."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / K
    evs = [(ev.new(), ev.new()) for _ in range(K)]
    for k in range(K):
        ev.record(evs[k][0], sp)
        fn()
        ev.record(evs[k][1], sp)
    torch.cuda.synchronize()
    return ms, np.array([ev.ms(a, b) for a, b in evs])


# ------------------------------------------------------------ HIP graphs
def capture(torch, fn):
    """Capture fn(stream_handle) into a torch CUDAGraph (HIP graph) on a side
    stream; returns (graph, None) or (None, error text) if capture fails."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(g, stream=s):
            fn(int(s.cuda_stream))
    except Exception as e:  # noqa: BLE001 - reported in the JSON line
        torch.cuda.synchronize()
        return None, f"{type(e).__name__}: {e}"
    torch.cuda.current_stream().wait_stream(s)
    return g, None


# ------------------------------------------------- plain per-sector FP64 form
def _key(t, b, legs):
    return tuple(int(v) for x in legs for v in t.charges[b, x, :])


def plain_maps(A, B, xa, xb, Cs):
    """Index maps of the plain per-sector form (benchmark harness, host numpy):
    for every sector X, gather indices of the fused A_X (M x K) and B_X (K x N)
    and scatter indices of C_X into C's blocks.  Index len(data) is a zero slot
    (absent sub-blocks); for C it is a dump slot."""
    fa = [i for i in range(A.sig.shape[0]) if i not in xa]
    fb = [i for i in range(B.sig.shape[0]) if i not in xb]
    sm = tuple(A.sym_mod)

    def sector(t, b, legs, sig):
        out = []
        for c in range(len(sm)):
            v = sum(int(sig[x]) * int(t.charges[b, x, c]) for x in legs)
            out.append(v % sm[c] if sm[c] else v)
        return tuple(out)
    bk = {}
    for j in range(B.charges.shape[0]):
        bk.setdefault(_key(B, j, xb), []).append(j)
    sect = {}
    for i in range(A.charges.shape[0]):
        kc = _key(A, i, xa)
        if kc not in bk:
            continue
        X = sector(A, i, xa, A.sig)
        s = sect.setdefault(X, {"rows": {}, "ks": {}, "cols": {}, "a": {}, "b": {}})
        s["rows"][_key(A, i, fa)] = i
        s["ks"][kc] = i
        s["a"][(_key(A, i, fa), kc)] = i
        for j in bk[kc]:
            s["cols"][_key(B, j, fb)] = j
            s["b"][(kc, _key(B, j, fb))] = j
    cidx = {tuple(int(v) for v in Cs.charges[k].ravel()): k for k in range(Cs.charges.shape[0])}
    nA = int(np.max(A.offsets + np.prod(A.shapes, axis=1))) if A.charges.shape[0] else 0
    nB = int(np.max(B.offsets + np.prod(B.shapes, axis=1))) if B.charges.shape[0] else 0
    nC = int(Cs.numel)
    gA, gB, sC, mats = [], [], [], []
    oa = ob = 0
    for X in sorted(sect):
        s = sect[X]
        rows, ks, cols = sorted(s["rows"]), sorted(s["ks"]), sorted(s["cols"])
        mdim = [int(np.prod([A.shapes[s["rows"][r], x] for x in fa])) for r in rows]
        kdim = [int(np.prod([A.shapes[s["ks"][k], x] for x in xa])) for k in ks]
        ndim = [int(np.prod([B.shapes[s["cols"][c], y] for y in fb])) for c in cols]
        M, K, N = sum(mdim), sum(kdim), sum(ndim)
        ia = np.full((M, K), nA, dtype=np.int64)
        ib = np.full((K, N), nB, dtype=np.int64)
        ic = np.full((M, N), nC, dtype=np.int64)
        r0 = 0
        for r, m in zip(rows, mdim):
            k0 = 0
            for k, kk in zip(ks, kdim):
                i = s["a"].get((r, k))
                if i is not None:
                    shp = tuple(int(v) for v in A.shapes[i])
                    blk = np.arange(int(np.prod(shp)), dtype=np.int64).reshape(shp)
                    ia[r0:r0 + m, k0:k0 + kk] = blk.transpose(fa + list(xa)).reshape(m, kk) + int(A.offsets[i])
                k0 += kk
            c0 = 0
            for c, n in zip(cols, ndim):
                k = cidx.get(r + c)
                if k is not None:
                    ic[r0:r0 + m, c0:c0 + n] = np.arange(m * n, dtype=np.int64).reshape(m, n) + int(Cs.offsets[k])
                c0 += n
            r0 += m
        k0 = 0
        for k, kk in zip(ks, kdim):
            c0 = 0
            for c, n in zip(cols, ndim):
                j = s["b"].get((k, c))
                if j is not None:
                    shp = tuple(int(v) for v in B.shapes[j])
                    blk = np.arange(int(np.prod(shp)), dtype=np.int64).reshape(shp)
                    ib[k0:k0 + kk, c0:c0 + n] = blk.transpose(list(xb) + fb).reshape(kk, n) + int(B.offsets[j])
                c0 += n
            k0 += kk
        mats.append((oa, M, K, ob, N))
        gA.append(ia.ravel())
        gB.append(ib.ravel())
        sC.append(ic.ravel())
        oa += M * K
        ob += K * N
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.int64)
    return cat(gA), cat(gB), cat(sC), mats, nA, nB, nC


class PlainStep:
    """One contraction in the plain per-sector form on the GPU (torch FP64)."""

    def __init__(self, A, B, xa, xb, Cs, dev):
        import torch
        gA, gB, sC, self.mats, self.nA, self.nB, self.nC = plain_maps(A, B, xa, xb, Cs)
        self.gA = torch.from_numpy(gA).to(dev)
        self.gB = torch.from_numpy(gB).to(dev)
        self.sC = torch.from_numpy(sC).to(dev)
        self.pc = torch.empty(len(sC), dtype=torch.float64, device=dev)

    def run(self, a_ext, b_ext, c_ext):
        import torch
        pa = a_ext[self.gA]                                   # fuse: gather into A_X
        pb = b_ext[self.gB]                                   # fuse: gather into B_X
        oc = 0
        for oa, M, K, ob, N in self.mats:                     # one matmul per sector
            torch.matmul(pa[oa:oa + M * K].view(M, K), pb[ob:ob + K * N].view(K, N),
                         out=self.pc[oc:oc + M * N].view(M, N))
            oc += M * N
        c_ext.index_copy_(0, self.sC, self.pc)                # unfuse: scatter into C's blocks


# ------------------------------------------------------------ chained step
class Chain:
    """The four chained contractions of an enlarged-corner step plus the FP64
    norm of the last output, with resident buffers and plans built (and
    autotuned) once.  Reduced precisions keep FP32 buffers between steps and
    write the last output (the truncation input) in FP64."""

    def __init__(self, torch, Y, t, prec="f64", tile_rows=0, tune=True, sp=0):
        self.torch, self.Y, self.sp = torch, Y, sp
        f64 = prec == "f64"
        dt = lambda d: torch.float64 if d == Y.DTYPE_F64 else torch.float32
        self.plans, cur = [], None
        tp0 = time.perf_counter()
        for i, ((an, bn), (ax, bx)) in enumerate(zip(STEPS, t["axes"])):
            out_dt = Y.DTYPE_F64 if (f64 or i == len(STEPS) - 1) else Y.DTYPE_F32
            pl = Y.plan([(t[an] if an else cur, t[bn], ax, bx)], precision=prec, stream=sp, tile_rows=tile_rows,
                        in_dtype=Y.DTYPE_F64 if f64 else Y.DTYPE_F32, out_dtype=out_dt)
            self.plans.append(pl)
            cur = pl.output(0)
        torch.cuda.synchronize()
        self.plan_ms = (time.perf_counter() - tp0) * 1e3
        self.stats = [pl.stats(0) for pl in self.plans]
        self.useful = sum(st["useful_flops"] for st in self.stats)
        in_dt = torch.float64 if f64 else torch.float32
        up = lambda x: torch.from_numpy(np.ascontiguousarray(x.data)).to("cuda:0").to(in_dt)
        self.inp = {k: up(t[k]) for k in ("C", "T1", "T4", "A", "Ac")}
        self.outs = [torch.empty(max(1, pl.output(0).numel), dtype=dt(pl.out_dtype), device="cuda:0")
                     for pl in self.plans]
        self.wss = [torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device="cuda:0") for pl in self.plans]
        self.nws = torch.empty(Y.norm_workspace_bytes(), dtype=torch.uint8, device="cuda:0")
        self.nout = torch.zeros(2, dtype=torch.float64, device="cuda:0")
        self.n_last = self.plans[-1].output(0).numel
        self.ops = [(self.inp[an] if an else self.outs[i - 1], self.inp[bn], self.outs[i], self.wss[i])
                    for i, (an, bn) in enumerate(STEPS)]
        self.tuned = []
        if tune:
            for i, (pl, (a, b, c, w)) in enumerate(zip(self.plans, self.ops)):
                v, times = pl.autotune([a], [b], [c], w, reps=5, stream=sp)
                self.tuned.append({"step": i + 1, "variant": v, "ms": [round(x, 4) for x in times]})
            torch.cuda.synchronize()

    def step(self, st):
        n = len(self.plans)
        for i, (pl, (a, b, c, w)) in enumerate(zip(self.plans, self.ops)):
            if i == n - 1:  # the truncation input's FP64 norm, fused into its contraction
                pl.contract_norm([a], [b], [c], w, self.nout, stream=st)
            else:
                pl.contract([a], [b], [c], w, stream=st)

    def timed(self, ev, K, warmup=3):
        """ms per step over K steps, eager and graph-replayed; the faster wins."""
        torch = self.torch
        for _ in range(warmup):
            self.step(self.sp)
        torch.cuda.synchronize()
        ref = self.outs[-1][:self.n_last].clone()
        graph, err = capture(torch, self.step)

        def run(fn):
            return steps_timed(torch, ev, self.sp, fn, K)

        modes = {"eager": run(lambda: self.step(self.sp))}
        if graph is not None:
            modes["graph"] = run(graph.replay)
            del graph
        assert torch.equal(self.outs[-1][:self.n_last], ref), "timed steps changed the result"
        mode = min(modes, key=lambda m: modes[m][0])
        return modes[mode][0], modes[mode][1], mode, {m: round(v[0], 5) for m, v in modes.items()}, err


def rel_err(torch, got, ref):
    d = got.to(torch.float64) - ref.to(torch.float64)
    return float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref.to(torch.float64)))


# ------------------------------------------------------- other workloads
FP32_MFMA_PEAK_TFS = 157.3     # MI355X dense FP32 matrix


def graph_time(torch, ev, sp, fn, R=10, REP=5):
    """ms per call of fn(stream), from HIP events around REP replays of a
    graph of R calls (eager calls if capture fails)."""
    def rep(st):
        for _ in range(R):
            fn(st)
    rep(sp)
    torch.cuda.synchronize()
    g, _ = capture(torch, rep)
    e0, e1 = ev.new(), ev.new()
    torch.cuda.synchronize()
    ev.record(e0, sp)
    for _ in range(REP):
        g.replay() if g is not None else rep(sp)
    ev.record(e1, sp)
    torch.cuda.synchronize()
    return ev.ms(e0, e1) / (R * REP)


def precision_section(torch, Y, W, ev, sp, K, plain_value):
    """FP64 / FP32 / split-BF16 x3 / x6 chains on the corner step at chi = 128
    and at chi = 256, D = 10: throughput and relative Frobenius error of each
    step's output against this GPU's FP64 chain.  The benchmark does not run
    the oracle here; tests/test_gpu_fullsize.py holds the FP64 chain and each
    reduced-precision chain to the oracle's chain element by element."""
    out = {}
    for name, t in (("chi128_D8", W.ctm()), ("chi256_D10", W.ctm_chi256())):
        ref, rows = None, {}
        for prec in ("f64", "f32", "bf16x3", "bf16x6"):
            ch = Chain(torch, Y, t, prec=prec, sp=sp)
            ms, lat, mode, _, _ = ch.timed(ev, K)
            val = ch.useful / (ms * 1e-3) / 1e12
            row = {"ms_per_step": round(ms, 4), "useful_TFs": round(val, 3), "timing": mode,
                   "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4)}
            if prec == "f64":
                ref = [o.clone() for o in ch.outs]
            else:
                row["rel_err_per_step"] = [float("%.3e" % rel_err(torch, o[:r.numel()], r)) for o, r in zip(ch.outs, ref)]
                row["rel_err_reference"] = "this GPU's FP64 chain (held to the oracle's chain at 1e-12 by the tests)"
                row["norm_rel_err"] = float("%.3e" % abs(float(ch.nout[0]) / float(torch.linalg.vector_norm(ref[-1])) - 1))
            if plain_value and name == "chi128_D8":
                row["vs_plain_per_sector_f64"] = round(val / plain_value, 2)
            rows[prec] = row
            del ch
            torch.cuda.empty_cache()
        out[name] = rows
    return out


def cold_time(torch, ev, sp, fn, reps=10):
    """Median ms of fn(stream) with the 256 MB Infinity Cache flushed first:
    a 512 MiB fill runs on the same stream before each timed call."""
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
    evs = [(ev.new(), ev.new()) for _ in range(reps)]
    for r, (a, b) in enumerate(evs):
        flush.fill_(r & 0xFF)
        ev.record(a, sp)
        fn(sp)
        ev.record(b, sp)
    torch.cuda.synchronize()
    del flush
    return float(np.median([ev.ms(a, b) for a, b in evs]))


def batch_section(torch, Y, W, ev, sp):
    """Config-1 batches (N copies of the U(1) rank-4 tensordot, D = 18) and the
    64 independent U(1) problems of uneven D in grouped launches; warm (inputs
    resident in the caches from the previous launch) and cold (Infinity Cache
    flushed before each launch)."""
    res = {}
    cases = [("u1_d18_x1", lambda: W.u1_d18(1), "f64"), ("u1_d18_x64", lambda: W.u1_d18(64), "f64"),
             ("u1_d18_x512", lambda: W.u1_d18(512), "f64"), ("u1_d18_x4096", lambda: W.u1_d18(4096), "f64"),
             ("u1_uneven_x64", W.u1_uneven, "f64"), ("u1_uneven_x64_f32", W.u1_uneven, "f32")]
    for name, make, prec in cases:
        probs = make()
        f64 = prec == "f64"
        dt = torch.float64 if f64 else torch.float32
        pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b) for p in probs], precision=prec, stream=sp)
        A = [torch.from_numpy(p.a.data).to("cuda:0").to(dt) for p in probs]
        B = [torch.from_numpy(p.b.data).to("cuda:0").to(dt) for p in probs]
        C = [torch.empty(max(1, pl.output(i).numel), dtype=dt, device="cuda:0") for i in range(len(probs))]
        ws = torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device="cuda:0")
        _, tune_ms = pl.autotune(A, B, C, ws, reps=3, stream=sp)
        st = [pl.stats(i) for i in range(len(probs))]
        useful = sum(x["useful_flops"] for x in st)
        byts = sum(x["alg_bytes"] for x in st)
        ms = graph_time(torch, ev, sp, lambda s_: pl.contract(A, B, C, ws, stream=s_))
        cold = cold_time(torch, ev, sp, lambda s_: pl.contract(A, B, C, ws, stream=s_))
        tf = useful / (ms * 1e-3) / 1e12
        peak = FP64_MFMA_PEAK_TFS if f64 else FP32_MFMA_PEAK_TFS
        res[name] = {"problems": len(probs), "precision": prec, "us_per_launch": round(ms * 1e3, 2),
                     "useful_TFs": round(tf, 3), "frac_of_mfma_peak": round(tf / peak, 4),
                     "achieved_GBs": round(byts / (ms * 1e-3) / 1e9, 1), "useful_flop": int(useful),
                     "alg_bytes": int(byts), "launch_groups": 1 + (len(probs) - 1) // 65536,
                     "cold_us_per_launch": round(cold * 1e3, 2),
                     "cold_useful_TFs": round(useful / (cold * 1e-3) / 1e12, 3),
                     "variant": pl.variant_id, "inputs": "resident; warm = repeated launches, cold = MALL flushed",
                     "autotune_ms": [round(x, 4) for x in tune_ms] if tune_ms else None}
        del pl, A, B, C, ws
        torch.cuda.empty_cache()
    return res


def grad_section(torch, Y, W, ev, sp):
    """Reverse mode of the chi = 128 corner steps 3 and 4: dA and dB (one
    contraction with the dual of the other operand, then the permutation back
    to the operand's leg order), timed as graphs of repeated calls; the step
    inputs come from the library's own forward chain."""
    t = W.ctm()
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x.data)).to("cuda:0")
    res, cur, cur_dev = {}, None, None
    for i, ((an, bn), (ax, bx)) in enumerate(zip(STEPS, t["axes"])):
        a, a_dev = (t[an], up(t[an])) if an else (cur, cur_dev)
        b_dev = up(t[bn])
        pl = Y.plan([(a, t[bn], ax, bx)], stream=sp)
        c = torch.empty(max(1, pl.output(0).numel), dtype=torch.float64, device="cuda:0")
        ws = torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device="cuda:0")
        pl.contract([a_dev], [b_dev], [c], ws, stream=sp)
        if i >= 2:
            flop = pl.stats(0)["useful_flops"]
            dc = torch.randn(c.numel(), dtype=torch.float64, device="cuda:0")
            for wrt in (0, 1):
                g = Y.Grad(a, t[bn], ax, bx, wrt, stream=sp)
                o = g.output()
                out = torch.empty(max(1, o.numel), dtype=torch.float64, device="cuda:0")
                gws = torch.empty(max(256, g.workspace_bytes), dtype=torch.uint8, device="cuda:0")
                other = b_dev if wrt == 0 else a_dev
                ms = graph_time(torch, ev, sp, lambda s_: g.run(dc, other, out, gws, stream=s_))
                res[f"step{i + 1}_d{'AB'[wrt]}"] = {"us": round(ms * 1e3, 2),
                                                   "useful_TFs": round(flop / (ms * 1e-3) / 1e12, 3),
                                                   "grad_numel": int(o.numel)}
                del g, out, gws
        torch.cuda.synchronize()
        cur, cur_dev = pl.output(0), c
    torch.cuda.empty_cache()
    return res


def complex_section(torch, Y, W, ev, sp, reps=5):
    """The chi = 128 enlarged-corner chain with complex128 tensors
    (yastn_zplan: C.T1, .T4, .A, .A* with A* = A under CONJ_B), each plan
    autotuned, the four contractions timed as one graph per step as the real
    chain is; useful flops = 8 m k n per matched block pair.  Then the
    fermionic swap gate between the last output's legs (A.b, A*.b) and
    (A.r, A*.r) in place (bytes = read + write of the negated blocks)."""
    t = W.complex_ctm()
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x.data)).to("cuda:0")
    plans, args, cur_s, cur_dev = [], [], None, None
    for i, ((an, bn), (ax, bx)) in enumerate(zip([("C", "T1"), (None, "T4"), (None, "A"), (None, "A")],
                                                 t["axes"])):
        a_s = t[an] if an else cur_s
        zp = Y.ZPlan([(a_s, t[bn], ax, bx)], conj=Y.CONJ_B if i == 3 else 0, stream=sp)
        o = zp.output(0)
        c = torch.empty(max(1, o.numel), dtype=torch.complex128, device="cuda:0")
        ws = torch.empty(max(256, zp.workspace_bytes), dtype=torch.uint8, device="cuda:0")
        a_dev = up(t[an]) if an else cur_dev
        b_dev = up(t[bn])
        zp.autotune([a_dev], [b_dev], [c], ws, reps=3, stream=sp)
        plans.append(zp)
        args.append(([a_dev], [b_dev], [c], ws))
        cur_s, cur_dev = o, c
    flop = sum(zp.stats(0)["useful_flops"] for zp in plans)

    def step(s_):
        for zp, (a, b, c, ws) in zip(plans, args):
            zp.contract(a, b, c, ws, stream=s_)
    ms = graph_time(torch, ev, sp, step)
    sg = Y.SwapGate(cur_s, (2, 4), (3, 5), W.FERMIONIC[tuple(cur_s.sym_mod)])
    sw_ms = graph_time(torch, ev, sp, lambda s_: sg.apply(cur_dev, Y.DTYPE_C128, stream=s_))
    res = {"step_ms": round(ms, 4), "useful_GFLOP": round(flop / 1e9, 3),
           "useful_TFs": round(flop / (ms * 1e-3) / 1e12, 3),
           "swap_gate": {"us": round(sw_ms * 1e3, 2), "blocks_negated": sg.blocks,
                         "bytes": 2 * 16 * sg.elements,
                         "GBs": round(2 * 16 * sg.elements / (sw_ms * 1e-3) / 1e9, 1),
                         "output_numel": int(cur_s.numel)},
           "timing": "graph of the four contractions replayed; swap gate as a graph of one launch"}
    del plans, args
    torch.cuda.empty_cache()
    return res


SPLIT = ("validate", "join", "host_tables", "upload")


def plan_costs(torch, Y, W, descs, plans, first_ms, sp, tile_rows, reps=5):
    """Planning cost of the four corner contractions: the first plans (code
    objects loaded then, the structure cache empty), the same requests again
    (structure-cache hits: a CTM iteration after the first), and afresh with
    the cache bypassed (median of reps), each split into validation, the
    device join, the host tables and the upload; then the same at chi = 256."""
    def split(pls):
        tot = [0.0] * 4
        for pl in pls:
            for i, v in enumerate(pl.profile()[0]):
                tot[i] += v
        return {k: round(v, 3) for k, v in zip(SPLIT, tot)}

    def timed(ds, flags):
        t0 = time.perf_counter()
        pls = [Y.plan([d], stream=sp, tile_rows=tile_rows, flags=flags) for d in ds]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, pls

    rec = {"first_ms": round(first_ms, 2), "first_split_ms": split(plans)}
    cached = [timed(descs, 0) for _ in range(reps)]
    rec["cached_ms"] = round(float(np.median([c[0] for c in cached])), 3)
    rec["cached_hits"] = all(pl.profile()[1] for pl in cached[-1][1])
    fresh = [timed(descs, Y.FLAG_NOCACHE) for _ in range(reps)]
    k = int(np.argsort([f[0] for f in fresh])[reps // 2])
    rec["uncached_ms"] = round(fresh[k][0], 2)
    rec["uncached_split_ms"] = split(fresh[k][1])
    t = W.ctm_chi256()
    d256, cur = [], None
    for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
        a = t[an] if an else cur
        pl = Y.plan([(a, t[bn], ax, bx)], stream=sp, flags=Y.FLAG_NOCACHE)
        d256.append((a, t[bn], ax, bx))
        cur = pl.output(0)
    f256 = [timed(d256, Y.FLAG_NOCACHE) for _ in range(3)]
    k = int(np.argsort([f[0] for f in f256])[1])
    rec["chi256_uncached_ms"] = round(f256[k][0], 2)
    rec["chi256_uncached_split_ms"] = split(f256[k][1])
    rec["what"] = ("four single-problem plans; first = cold process; cached = the same requests again "
                   "(structure cache); uncached = planned afresh (FLAG_NOCACHE), median")
    return rec


def svd_section(torch, Y, last, last_struct, sp, chi=128, reps=5):
    """The CTM truncation of the chi = 128 step's output (the enlarged corner,
    FP64): rows (r1, A_r, A*_r) x columns (bot4, A_b, A*_b), block-sparse SVD
    on the GPU (yastn_svd: fuse, Jacobi sweeps, sort, global truncation to
    chi) and the kept factors (yastn_svd_factors); median wall time of
    ``reps`` runs on resident data, synchronised (the SVD syncs per sweep)."""
    rows = (0, 3, 5)
    sv = Y.Svd(last_struct, rows, stream=sp)
    ws = torch.empty(max(256, sv.workspace_bytes), dtype=torch.uint8, device="cuda:0")
    svals = torch.empty(max(1, sv.nsv), dtype=torch.float64, device="cuda:0")
    kept, sweeps = sv.run(last, svals, ws, chi, stream=sp)
    us, vs = sv.output()
    u = torch.empty(max(1, us.numel), dtype=torch.float64, device="cuda:0")
    vt = torch.empty(max(1, vs.numel), dtype=torch.float64, device="cuda:0")
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kept, sweeps = sv.run(last, svals, ws, chi, stream=sp)
        sv.factors(u, vt, ws, stream=sp)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(times))
    # MFMA work of the sweeps: per block pair and round, the 16 x 16 Gram
    # matrix over the W rows and the rotation of W's and V's 16 columns
    flop = 0.0
    for X, m, n, s0 in sv.sectors:
        r, c = max(m, n), min(m, n)
        nb = max(2, -(-c // 8))
        nb += nb & 1
        per_round = (nb // 2) * 2.0 * 16 * 16 * (2 * r + c)
        flop += per_round * (nb - 1) * sweeps
    # the same with the kept right vectors recovered after the sweeps (the
    # mode the CTM move uses): the sweeps rotate W only
    sv.set_flags(Y.SVD_RECOVER_V)
    rtimes = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rkept, rsweeps = sv.run(last, svals, ws, chi, stream=sp)
        sv.factors(u, vt, ws, stream=sp)
        torch.cuda.synchronize()
        rtimes.append((time.perf_counter() - t0) * 1e3)
    rms = float(np.median(rtimes))
    rflop = 0.0
    for X, m, n, s0 in sv.sectors:
        r, c = max(m, n), min(m, n)
        nb = max(2, -(-c // 8))
        nb += nb & 1
        rflop += (nb // 2) * 2.0 * 16 * 16 * (2 * r) * (nb - 1) * rsweeps
    dims = sorted(((max(m, n), min(m, n)) for _, m, n, _ in sv.sectors), reverse=True)
    res = {"ms": round(ms, 3), "sweeps": sweeps, "sectors": sv.nsectors, "singular_values": sv.nsv,
           "largest_sectors": dims[:4], "chi": chi, "kept": int(sum(kept)),
           "jacobi_mfma_GFLOP": round(flop / 1e9, 2), "jacobi_mfma_TFs": round(flop / (ms * 1e-3) / 1e12, 3),
           "frac_of_fp64_mfma_peak": round(flop / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFS, 4),
           "recover_v": {"ms": round(rms, 3), "sweeps": rsweeps, "kept": int(sum(rkept)),
                         "jacobi_mfma_GFLOP": round(rflop / 1e9, 2),
                         "jacobi_mfma_TFs": round(rflop / (rms * 1e-3) / 1e12, 3)},
           "timing": f"median of {reps} synchronised runs (fuse, sweeps, sort, truncation, factors)"}
    del sv, ws, svals, u, vt
    torch.cuda.empty_cache()
    return res


def ctm_section(torch, Y, W, sp, chi=128, reps=5):
    """One CTM left move (yastn_ctm_move) at chi = 128, D = 8, U(1)xU(1): four
    enlarged corners, halves, four-corner product, truncated SVD to chi,
    projectors, the new left column, FP64 normalisation, all on the device
    from resident inputs.  The first move plans what follows the SVD and
    autotunes every contraction plan; the timed moves repeat it with the
    plans cached (the steady state of CTM, whose structure repeats).
    Median wall time of ``reps`` moves, each returning when done (the move
    waits for the SVD's kept counts), and the median per-phase event times."""
    env = W.ctm_move_u1xu1(chi)
    ctm = Y.Ctm([env[k] for k in Y.CTM_INPUTS], stream=sp)
    dev = [torch.from_numpy(env[k].data).to("cuda:0") for k in Y.CTM_INPUTS]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctm.move(dev, chi, autotune=True, stream=sp)
    first = (time.perf_counter() - t0) * 1e3
    walls, phases = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctm.move(dev, chi, stream=sp)
        walls.append((time.perf_counter() - t0) * 1e3)
        kept, sweeps, ms, flops = ctm.info()
        phases.append(ms)
    med = np.median(np.array(phases), axis=0)
    names = ("corners", "halves_and_product", "svd", "plans_after_svd_and_factors", "projectors_and_column",
             "normalisation")
    contr_ms = float(med[0] + med[1] + med[4])
    res = {"ms": round(float(np.median(walls)), 3), "first_move_ms_with_autotune": round(first, 1),
           "phases_ms": {n: round(float(v), 3) for n, v in zip(names, med)},
           "chi": chi, "kept": kept, "sweeps": sweeps,
           "useful_GFLOP": {"before_svd": round(flops[0] / 1e9, 3), "after_svd": round(flops[1] / 1e9, 3)},
           "contractions_TFs": round((flops[0] + flops[1]) / (contr_ms * 1e-3) / 1e12, 3),
           "svd_to_contractions": round(float(med[2]) / contr_ms, 2),
           "contraction_launches": 11,
           "timing": f"median of {reps} moves after one autotuned move; wall time per move, phases from HIP events"}
    ctm.free()
    del dev
    torch.cuda.empty_cache()
    return res


def serving_section(torch, Y, W, sp, nreq=2000, warm=200, budget_gib=32, seed=5):
    """32 concurrent CTM runs (16 Z2, 16 U(1); D in {4,6,8,10} x chi in
    {64,128,192,256}) submit enlarged-corner requests with Poisson arrivals to
    the continuous-batching server (HBM budget for intermediates); the rate is
    0.7x the closed-loop saturation rate of a calibration pass.  ``warm``
    requests first, then ``nreq`` measured ones (latency percentiles and
    throughput over those)."""
    runs = []
    for r in range(32):
        t = W.serving_run(r)
        plans, cur = [], None
        for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
            pl = Y.plan([(t[an] if an else cur, t[bn], ax, bx)], stream=sp)
            plans.append(pl)
            cur = pl.output(0)
        inp = {k: torch.from_numpy(t[k].data).to("cuda:0") for k in ("C", "T1", "T4", "A", "Ac")}
        out = torch.empty(max(1, plans[-1].output(0).numel), dtype=torch.float64, device="cuda:0")
        flops = sum(pl.stats(0)["useful_flops"] for pl in plans)
        runs.append({"plans": plans, "inp": inp, "out": out, "flops": flops, "name": t["name"]})
    srv = Y.Server(pool_bytes=budget_gib << 30, max_ahead=2, stream=sp)

    def submit(i):
        r = runs[i]
        return srv.submit(r["plans"], r["inp"]["C"], [r["inp"][bn] for _, bn in STEPS], r["out"])

    # calibration: one request of every run, closed loop (all submitted at once)
    for i in range(32):
        submit(i)
    srv.drain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(32):
        submit(i)
    srv.drain()
    torch.cuda.synchronize()
    sat = 32 / (time.perf_counter() - t0)           # requests per second
    lam = 0.7 * sat
    rng = np.random.default_rng(seed)
    ntot = warm + nreq
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=ntot))
    which = rng.integers(0, 32, size=ntot)
    ids, flop = [], 0.0
    queued_at_submit = []
    torch.cuda.synchronize()
    st0 = srv.stats()
    base = time.perf_counter()
    t_meas = None
    k = 0
    while k < ntot or srv.stats()["completed"] < srv.stats()["submitted"]:
        now = time.perf_counter() - base
        while k < ntot and arrivals[k] <= now:
            if k == warm:
                t_meas = time.perf_counter()
                st0 = srv.stats()
            rid = submit(int(which[k]))
            if k >= warm:
                ids.append(rid)
                flop += runs[int(which[k])]["flops"]
                queued_at_submit.append(srv.stats()["queued"])
            k += 1
        srv.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - (t_meas if t_meas is not None else base)
    lat = np.array([srv.query(i)[1] for i in ids])
    st = srv.stats()
    srv.close()
    del runs
    torch.cuda.empty_cache()
    q = np.array(queued_at_submit)
    return {"requests": nreq, "warmup_requests": warm, "runs": 32, "arrival_rate_per_s": round(lam, 2),
            "saturation_rate_per_s": round(sat, 2), "hbm_budget_GiB": budget_gib,
            "useful_TFs": round(flop / wall / 1e12, 3), "wall_s": round(wall, 3),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_steps_per_launch": int(st["max_batch"]), "launches": int(st["ticks"] - st0["ticks"]),
            "admitted": int(st["admitted"] - st0["admitted"]), "completed": int(st["completed"] - st0["completed"]),
            "bypasses": int(st["bypasses"] - st0["bypasses"]), "queued_peak": int(st["queued_peak"]),
            "queued_at_submit_p50": float(np.percentile(q, 50)), "queued_at_submit_max": int(q.max()),
            "pool_peak_GiB": round(st["pool_peak"] / 2 ** 30, 2),
            "latency": "submit to the host observing the completion event; percentiles over the measured requests",
            "admission": "arrival order; a request that fits may pass a waiting one at most 16 times"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(t, useful, reps):
    """The oracle on the host cores (the only place the benchmark runs it)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle
    import workloads as W

    def o2_step():
        cur = None
        for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
            cur = oracle.tensordot_blockpair(t[an] if an else cur, t[bn], ax, bx)
        oracle.norms(cur)

    def med(fn, n):
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    with threadpool_limits(1):
        s1 = med(o2_step, reps)
    with threadpool_limits(ncpu):
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        sall = med(o2_step, reps)
        (p1,) = W.u1_d18()
        f1 = 2199168.0
        d1 = med(lambda: oracle.tensordot_dense(p1.a, p1.b, p1.axes_a, p1.axes_b), reps)

        def o1_step():
            cur = None
            for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
                cur = oracle.tensordot_dense(t[an] if an else cur, t[bn], ax, bx)
        d2 = med(o1_step, 1)
    return {"value": round(useful / sall / 1e12, 6), "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"median of {reps} full enlarged-corner steps (4 block-pair tensordots + norm, chi = 128, "
                      f"D = 8) at {threads} BLAS threads: {sall * 1e3:.0f} ms per step",
            "cpu_model": _cpu_model(), "host_cpus": ncpu,
            "o2_one_thread": {"value": round(useful / s1 / 1e12, 6), "ms_per_step": round(s1 * 1e3, 1)},
            "o1_dense_u1_d18": {"GFLOPs_useful": round(f1 / d1 / 1e9, 3), "ms": round(d1 * 1e3, 2)},
            "o1_dense_corner_step": {"GFLOPs_useful": round(useful / d2 / 1e9, 3), "ms": round(d2 * 1e3, 1),
                                     "note": "dense-embed form, one run"}}


# --------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="f64", choices=["f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--tile-rows", type=int, default=0, help="rows per wave tile: 64, 128, 256, 512 or 0 (plan's choice)")
    ap.add_argument("--no-tune", action="store_true", help="skip the kernel-variant autotuner")
    ap.add_argument("--variants", default="",
                    help="comma-separated kernel variant per contraction (skips the autotuner), e.g. 8,8,13,8")
    ap.add_argument("--separate-norm", action="store_true",
                    help="norm of the last output as its own two-pass kernel instead of fused into the contraction")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision sweep, the batched configs and the serving loop")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--batch-only", default="", choices=["", "u1_d18_x64", "u1_d18_x512", "u1_uneven_x64"],
                    help="run only this grouped launch (autotuned, then --steps launches) and print its time; "
                         "for profiling")
    ap.add_argument("--svd-only", action="store_true",
                    help="run only the truncated SVD of the chi = 128 corner and print its record; for profiling")
    ap.add_argument("--tune-file", default="",
                    help="tuning store (JSON): loaded before planning if it exists (known requests start at "
                         "their tuned variant), saved after autotuning")
    ap.add_argument("--complex-only", action="store_true",
                    help="run only the complex128 corner chain and the swap gate and print their record")
    ap.add_argument("--ctm-only", action="store_true",
                    help="run only the CTM left move at chi = 128 and print its record; for profiling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (scale for HBM byte counters)")
    args = ap.parse_args()
    ws_env = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws_env != 1:
        print("bench.py measures one GPU only: the block-sparse tensordot of this library runs on a single "
              "MI355X (sharding over several GPUs is not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        x = torch.randn(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": x.numel() * 8, "copies": 3}))
        return

    import paper_2405_12196_amd as Y
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batch_only:
        probs = {"u1_d18_x64": lambda: W.u1_d18(64), "u1_d18_x512": lambda: W.u1_d18(512),
                 "u1_uneven_x64": W.u1_uneven}[args.batch_only]()
        sp = int(torch.cuda.current_stream().cuda_stream)
        pl = Y.plan([(p.a, p.b, p.axes_a, p.axes_b) for p in probs], stream=sp, tile_rows=args.tile_rows)
        A = [torch.from_numpy(p.a.data).to("cuda:0") for p in probs]
        B = [torch.from_numpy(p.b.data).to("cuda:0") for p in probs]
        C = [torch.empty(max(1, pl.output(i).numel), dtype=torch.float64, device="cuda:0") for i in range(len(probs))]
        ws = torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device="cuda:0")
        _, tune_ms = pl.autotune(A, B, C, ws, reps=3, stream=sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pl.contract(A, B, C, ws, stream=sp)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) * 1e6 / args.steps
        flop = sum(pl.stats(i)["useful_flops"] for i in range(len(probs)))
        print(json.dumps({"batch": args.batch_only, "variant": pl.variant_id, "us_per_launch_host": round(us, 2),
                          "useful_flop": flop, "launches": args.steps,
                          "autotune_ms": [round(x, 4) for x in tune_ms]}))
        return
    if args.svd_only:
        sp = int(torch.cuda.current_stream().cuda_stream)
        t = W.ctm()
        ch = Chain(torch, Y, t, tune=False, sp=sp)
        ch.step(sp)
        torch.cuda.synchronize()
        print(json.dumps({"svd": svd_section(torch, Y, ch.outs[-1], ch.plans[-1].output(0), sp)}))
        return
    if args.ctm_only:
        sp = int(torch.cuda.current_stream().cuda_stream)
        print(json.dumps({"ctm_move": ctm_section(torch, Y, W, sp, reps=max(1, args.steps))}))
        return
    if args.complex_only:
        sp = int(torch.cuda.current_stream().cuda_stream)
        print(json.dumps({"complex128": complex_section(torch, Y, W, HipEvents(), sp)}))
        return
    dev = "cuda:0"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sp = int(stream.cuda_stream)
    t = W.ctm()
    # ---- plans (once; structure is fixed across CTM iterations)
    tp0 = time.perf_counter()
    tune_loaded = None
    if args.tune_file and os.path.exists(args.tune_file):
        tune_loaded = Y.tune_load(args.tune_file)  # plans of known requests start at their tuned variant
    plans, descs = [], []
    cur = None
    for (an, bn), (ax, bx) in zip(STEPS, t["axes"]):
        a = t[an] if an else cur
        pl = Y.plan([(a, t[bn], ax, bx)], stream=sp, tile_rows=args.tile_rows)
        plans.append(pl)
        descs.append((a, t[bn], ax, bx))
        cur = pl.output(0)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - tp0) * 1e3
    plan_rec = plan_costs(torch, Y, W, descs, plans, plan_ms, sp, args.tile_rows)
    stats = [pl.stats(0) for pl in plans]
    useful = sum(s["useful_flops"] for s in stats)
    alg_bytes = [s["alg_bytes"] for s in stats]

    # ---- device buffers (resident before timing)
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x.data)).to(dev)
    inp = {k: up(t[k]) for k in ("C", "T1", "T4", "A", "Ac")}
    outs = [torch.empty(max(1, pl.output(0).numel), dtype=torch.float64, device=dev) for pl in plans]
    wss = [torch.empty(max(256, pl.workspace_bytes), dtype=torch.uint8, device=dev) for pl in plans]
    nws = torch.empty(Y.norm_workspace_bytes(), dtype=torch.uint8, device=dev)
    nout = torch.zeros(2, dtype=torch.float64, device=dev)
    n_last = plans[-1].output(0).numel
    ops = []
    for i, ((an, bn), _) in enumerate(zip(STEPS, t["axes"])):
        ops.append((inp[an] if an else outs[i - 1], inp[bn], outs[i], wss[i]))

    # ---- autotune each contraction's kernel variant (outside the timed region)
    tuned = []
    if args.variants:
        for pl, v in zip(plans, [int(x) for x in args.variants.split(",")]):
            pl.set_variant(v)
    elif not args.no_tune:
        for i, (pl, (a, b, c, w)) in enumerate(zip(plans, ops)):
            v, times = pl.autotune([a], [b], [c], w, reps=5, stream=sp)
            tuned.append({"step": i + 1, "variant": v, "ms": [round(x, 4) for x in times]})
        torch.cuda.synchronize()
        if args.tune_file:
            Y.tune_save(args.tune_file)

    ev = HipEvents()

    def step(st):
        for i, (pl, (a, b, c, w)) in enumerate(zip(plans, ops)):
            if i == len(plans) - 1 and not args.separate_norm:
                pl.contract_norm([a], [b], [c], w, nout, stream=st)  # the truncation input's FP64 norm, fused
            else:
                pl.contract([a], [b], [c], w, stream=st)
        if args.separate_norm:
            Y.norm(outs[-1], n_last, nout, nws, stream=st)

    for _ in range(args.warmup):
        step(sp)
    torch.cuda.synchronize()
    ref_last = outs[-1][:n_last].clone()

    # ---- the step captured once into a HIP graph (no host work per replay);
    # the graph's result must be bitwise the eager one
    graph, graph_err = capture(torch, lambda st: step(st))
    if graph is not None:
        for _ in range(max(1, args.warmup // 2)):
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(outs[-1][:n_last], ref_last), "graph replay differs from the eager step"

    # ---- timed region: K steps, either as graph replays or as eager launches
    # (one host call per kernel); both are timed and the faster is reported
    K = args.steps

    def timed(run):
        return steps_timed(torch, ev, sp, run, K)

    modes = {"eager": timed(lambda: step(sp))}
    if graph is not None:
        modes["graph"] = timed(graph.replay)
    mode = min(modes, key=lambda m: modes[m][0])
    ms_per_step, lat = modes[mode]
    assert torch.equal(outs[-1][:n_last], ref_last), "timed steps changed the result"

    # ---- per-contraction kernel time: R launches of one contraction in one
    # graph, HIP events around the replays on the launch stream
    R, REP = 20, 5
    per_kernel, gemm_avg = [], []
    for i, (pl, (a, b, c, w)) in enumerate(zip(plans, ops)):
        def rep(st, pl=pl, a=a, b=b, c=c, w=w):
            for _ in range(R):
                pl.contract([a], [b], [c], w, stream=st)
        g, _ = capture(torch, rep)
        e0, e1 = ev.new(), ev.new()
        torch.cuda.synchronize()
        ev.record(e0, sp)
        for _ in range(REP):
            g.replay() if g is not None else rep(sp)
        ev.record(e1, sp)
        torch.cuda.synchronize()
        ms = ev.ms(e0, e1) / (R * REP)
        gemm_avg.append(ms)
        per_kernel.append({"step": i + 1, "us_per_launch": round(ms * 1e3, 2), "alg_bytes": int(alg_bytes[i]),
                           "achieved_GBs": round(alg_bytes[i] / (ms * 1e-3) / 1e9, 1),
                           "useful_TFs": round(stats[i]["useful_flops"] / (ms * 1e-3) / 1e12, 2),
                           "tiles": int(stats[i]["tiles"]), "variant": pl.variant_id})
        del g
    step(sp)  # restore the chain's outputs
    torch.cuda.synchronize()
    gemm_avg = np.array(gemm_avg)
    dom = int(np.argmax(gemm_avg))
    ach = alg_bytes[dom] / (gemm_avg[dom] * 1e-3) / 1e9
    value = useful / (ms_per_step * 1e-3) / 1e12

    # ---- plain per-sector FP64 form on the same GPU
    plain = None
    if not args.no_plain:
        cur_structs = [d[0] for d in descs]
        psteps = []
        for i, (a, b, ax, bx) in enumerate(descs):
            psteps.append(PlainStep(a if i == 0 else plans[i - 1].output(0), b, ax, bx, plans[i].output(0), dev))
        del cur_structs
        ext = lambda n: torch.zeros(n + 1, dtype=torch.float64, device=dev)
        a_ext = [ext(p.nA) for p in psteps]
        b_ext = [ext(p.nB) for p in psteps]
        c_ext = [ext(p.nC) for p in psteps]
        keys = ["C", "T1", "T4", "A", "Ac"]
        a_ext[0][:psteps[0].nA].copy_(inp["C"][:psteps[0].nA])
        for i, (an, bn) in enumerate(STEPS):
            b_ext[i][:psteps[i].nB].copy_(inp[bn][:psteps[i].nB])
        del keys

        def pstep(st=None):
            for i, p in enumerate(psteps):
                if i > 0:
                    a_ext[i][:p.nA].copy_(c_ext[i - 1][:p.nA])
                p.run(a_ext[i], b_ext[i], c_ext[i])
            Y.norm(c_ext[-1], psteps[-1].nC, nout, nws, stream=st)

        for _ in range(3):
            pstep()
        torch.cuda.synchronize()
        maxdiff = float((c_ext[-1][:n_last] - outs[-1][:n_last]).abs().max()) / float(outs[-1][:n_last].abs().max())
        KP = max(5, min(50, K // 4))
        torch.cuda.synchronize()
        tq = time.perf_counter()
        for _ in range(KP):
            pstep()
        torch.cuda.synchronize()
        pms_eager = (time.perf_counter() - tq) * 1e3 / KP
        # the same form captured in a graph (launch overhead removed): the
        # faster of the two is the denominator
        pg, pg_err = capture(torch, pstep)
        pms_graph = None
        if pg is not None:
            pg.replay()
            torch.cuda.synchronize()
            tq = time.perf_counter()
            for _ in range(KP):
                pg.replay()
            torch.cuda.synchronize()
            pms_graph = (time.perf_counter() - tq) * 1e3 / KP
            del pg
        pms = min(pms_eager, pms_graph) if pms_graph is not None else pms_eager
        plain = {"value": round(useful / (pms * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "ms_per_step": round(pms, 4),
                 "ms_per_step_eager": round(pms_eager, 4),
                 "ms_per_step_graph": round(pms_graph, 4) if pms_graph is not None else None,
                 "graph_error": pg_err, "steps": KP, "max_rel_diff_vs_library": maxdiff,
                 "form": "gather into fused sector matrices, one torch.matmul (FP64) per sector, scatter"}

    # ---- CPU oracle baseline, bounded sample: the block-pair form (O2) of the
    # step at one BLAS thread and at all host cores (median of cpu_reps each),
    # and the dense-embed form (O1) of the D = 18 contraction and of the step
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(t, useful, args.cpu_reps)

    # ---- the other workloads (not the headline value)
    extras = None
    if not args.no_extras:
        del graph
        torch.cuda.empty_cache()
        extras = {"precision": precision_section(torch, Y, W, ev, sp, max(10, K // 10), plain["value"] if plain else None),
                  "batched": batch_section(torch, Y, W, ev, sp),
                  "gradient": grad_section(torch, Y, W, ev, sp),
                  "svd": svd_section(torch, Y, outs[-1], plans[-1].output(0), sp),
                  "ctm_move": ctm_section(torch, Y, W, sp),
                  "complex128": complex_section(torch, Y, W, ev, sp),
                  "serving": serving_section(torch, Y, W, sp, nreq=args.serve_requests, warm=args.serve_warmup)}

    rec = {
        "metric": "useful TFLOP/s per block-sparse tensordot vs plain per-sector FP64; p50/p99 latency",
        "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ctmrg_enlarged_corner_u1xu1_chi128_D8_d4", "contractions_per_step": 4,
                   "useful_flop_per_step": int(useful), "plus": "fp64 norm of the step-4 output" + (" (separate kernel)" if args.separate_norm else " (fused into its contraction)"),
                   "parallelism": "single GPU"},
        "p50_ms": round(float(np.percentile(lat, 50)), 5), "p99_ms": round(float(np.percentile(lat, 99)), 5),
        "plan_ms": round(plan_ms, 2), "plan": plan_rec, "tuning_entries_loaded": tune_loaded,
        "timing": {"graph": "step captured in one HIP graph, one replay per step",
                   "eager": "one host launch per kernel"}[mode],
        "ms_per_step_by_mode": {m: round(v[0], 5) for m, v in modes.items()}, "graph_error": graph_err,
        "vs_plain_per_sector_f64": round(value / plain["value"], 3) if plain else None,
        "plain_per_sector_f64": plain,
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom + 1, plans[dom].variant_id),
                     "kernel": f"grouped gather GEMM of contraction {dom + 1}",
                     "launch_us": round(float(gemm_avg[dom]) * 1e3, 2),
                     "timing": f"HIP events on the launch stream around {REP} replays of a graph of {R} launches"},
        "kernels": per_kernel,
        "autotune": tuned,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    ev.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
