// HIP kernels of the block-sparse tensordot for gfx950 (CDNA4), as templates.
// Instantiated in the inst_*.hip translation units (one per arithmetic), so
// the many tile shapes compile in parallel.
//
//  k_pack_b     fuses B's legs into the per-sector matrices B_X (K_X x N_X,
//               row-major; absent sub-blocks zero) -- the "fuse" step of the
//               fuse -> multiply -> unfuse contraction of paper Sec. II.B,
//               applied to the small operand only.
//  k_gemm4      grouped GEMM C_X = A_X B_X over every sector of every problem
//               in one launch, FP64 / FP32 MFMA 16x16x4.  One wave owns a tile
//               of up to 64 rows of one A free tuple x up to 64 columns of B_X.
//               A is never materialised: each element is gathered from its
//               block through the factorised offsets of plan.hpp (the leg
//               permute is fused into the load).  The epilogue writes each
//               element straight into its output block (the "unfuse" step),
//               exactly once: no atomics, deterministic results.
//  k_gemm_res   as k_gemm4 for sectors with K_X <= 64, with the tile's B
//               values and k metadata held in registers and B read straight
//               from its blocks (no pack kernel).
//  k_gemm_lds   as k_gemm_res, the B tile loaded once per workgroup job of
//               up to eight tiles of one sector column range and read from LDS.
//  k_gemm_pf    sectors of any K, k loop software-pipelined (loads of the
//               next k batch in flight while the MFMAs of this one run).
//  k_rows       tall-skinny sectors (K, N <= 64): one row of C_X per lane.
//  k_gemm_bf16  split-BF16 products on bf16 MFMA 16x16x32, FP32 accumulation.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "index.hpp"

namespace yastn {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Wave-uniform reads of plan tables go through the constant address space:
// the tables are read-only while kernels run, so the compiler may use scalar
// loads (reads only) and keep the values in SGPRs.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
__device__ __forceinline__ T cst(const T *p) {
  return *(const __attribute__((address_space(4))) T *)(p);
}
#else
template <typename T> __device__ __forceinline__ T cst(const T *p) { return *p; }  // host pass: unused
#endif

// The plan's table of pointers, one field at a time: copying the whole
// struct in one aggregate load loses the constant address space of the
// pointers inside it, and every table read behind them then becomes a
// per-lane flat load instead of a scalar load.
__device__ __forceinline__ DevPlan load_plan(const DevPlan *p) {
  DevPlan d;
  d.probs = cst(&p->probs);
  d.sectors = cst(&p->sectors);
  d.rows = cst(&p->rows);
  d.ctrs = cst(&p->ctrs);
  d.cols = cst(&p->cols);
  d.agrid = cst(&p->agrid);
  d.aoff = cst(&p->aoff);
  d.cgrid = cst(&p->cgrid);
  d.bblocks = cst(&p->bblocks);
  d.tiles = cst(&p->tiles);
  d.items = cst(&p->items);
  d.kofs = cst(&p->kofs);
  d.kp = cst(&p->kp);
  d.colmap = cst(&p->colmap);
  d.bofs = cst(&p->bofs);
  d.ntiles = cst(&p->ntiles);
  d.nitems = cst(&p->nitems);
  return d;
}

// The pointers of launch problem i (kernel arguments or the device table).
__device__ __forceinline__ ProbPtrs prob_ptrs(const LaunchArgs &a, int i) {
  return a.ptab ? cst(a.ptab + i) : a.p[i];
}

// LDS written by one lane and read by another lane of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fused output norm: a lane's running sum of squares and max |x| of the
// values it stored; at the end of a tile the wave combines them in a fixed
// butterfly order and lane 0 files the tile's part (a small kernel then
// reduces the parts in tile order: deterministic, no atomics).
struct NormAcc {
  double ss = 0.0, mx = 0.0;
  __device__ void add(double v) {
    ss = fma(v, v, ss);
    mx = fmax(mx, fabs(v));
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void norm_file_tile(const NormArgs &na, int t, int lane, NormAcc &acc) {
  const double ss = wave_sum(acc.ss), mx = wave_max(acc.mx);
  acc = NormAcc{};
  if (lane == 0) {
    na.parts[2 * (int64_t)t] = ss;
    na.parts[2 * (int64_t)t + 1] = mx;
  }
}

// A value the compiler cannot prove wave-uniform but that is.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T *uniptr(T *p) {
  return reinterpret_cast<T *>(uni64(reinterpret_cast<int64_t>(p)));
}


// ---------------------------------------------------------------------------
// numeric helpers
// ---------------------------------------------------------------------------
// round-to-nearest-even float -> bf16 bits (finite inputs)
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ---------------------------------------------------------------------------
// B pack: per-sector matrices B_X in the workspace
// ---------------------------------------------------------------------------
// One workgroup per item.  A gather item copies up to 2048 consecutive
// elements of B_X, 8 per thread: the offset-table reads, then every B read,
// then the stores (no load waits on a store); an absent entry reads B[0] and
// stores zero.  A sub-block item writes up to 256 elements of one (s, j)
// sub-block; consecutive threads write consecutive elements of a B_X row.
template <typename In, typename Cmp>
__global__ void __launch_bounds__(256) k_pack_b(LaunchArgs args) {
  for (int g = blockIdx.x; g < args.nitems; g += gridDim.x) {
    int jb = 0;
    while (jb + 1 < args.njobs && g >= args.jobs[jb + 1].item0) ++jb;
    const JobArg &job = args.jobs[jb];
    const DevPlan P = load_plan(job.plan);
    const DevPackItem it = cst(P.items + (g - job.item0 + job.pitem0));
    const DevSector sec = cst(P.sectors + it.sector);
    if (it.s < 0) {
      constexpr int R = kGatherItem / 256;
      const int32_t *bo = P.bofs + sec.bofs0 + it.e0;
      Cmp *dst = reinterpret_cast<Cmp *>(job.ws) + sec.bpack + it.e0;
      const In *src = reinterpret_cast<const In *>(prob_ptrs(args, job.prob0 + sec.prob - job.plo).b);
      const int32_t last = it.j - 1;
      int32_t o[R];
      In v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) o[r] = bo[min((int32_t)threadIdx.x + 256 * r, last)];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[max(o[r], 0)];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int32_t e = (int32_t)threadIdx.x + 256 * r;
        if (e <= last) dst[e] = o[r] >= 0 ? Cmp(v[r]) : Cmp(0);
      }
      continue;
    }
    const DevCtrTuple ct = cst(P.ctrs + (sec.ctr0 + it.s));
    const DevColTuple cl = cst(P.cols + (sec.col0 + it.j));
    const int32_t e = it.e0 + (int32_t)threadIdx.x;
    if (e >= ct.k * cl.n) continue;
    const int32_t kd = e / cl.n, cb = e - kd * cl.n;
    Cmp *dst = reinterpret_cast<Cmp *>(job.ws) + sec.bpack + (int64_t)(ct.ko + kd) * sec.N + cl.no + cb;
    if (it.bblk < 0) {
      *dst = Cmp(0);
    } else {
      const In *src = reinterpret_cast<const In *>(prob_ptrs(args, job.prob0 + sec.prob - job.plo).b);
      const DevBBlock bb = cst(P.bblocks + it.bblk);
      const DevProb pr = cst(P.probs + sec.prob);
      *dst = Cmp(src[b_offset(bb, ct, cl, pr, kd, cb)]);
    }
  }
}

// ---------------------------------------------------------------------------
// operand access: buffer resources or 64-bit pointers
// ---------------------------------------------------------------------------
// BUF = true: A and C are reached through buffer resources (scalar base,
// 32-bit byte offsets; the hardware returns 0 for reads past num_records and
// drops such writes).  Used when both buffers are below 2 GiB.  BUF = false:
// plain 64-bit addresses, any size.
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
constexpr int kBufFlags = 0x00020000;  // raw buffer, gfx9-family descriptor word 3

// Cache policy of the streaming operands (A read once, C written once).  The
// non-temporal hint (bit 1 of the buffer instructions' cache-policy operand)
// would keep them from evicting the plan tables, but on gfx950 it makes these
// kernels about 1.5x slower (the C stores are partial lines that the L2 no
// longer merges), so the default policy is kept.
constexpr int kStream = 0;

template <typename T> struct BufIo;
template <> struct BufIo<double> {
  template <int CP> __device__ static double ld(__amdgpu_buffer_rsrc_t r, int32_t byte) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte, 0, CP));
  }
  template <int CP> __device__ static void st(__amdgpu_buffer_rsrc_t r, int32_t byte, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), r, byte, 0, CP);
  }
};
template <> struct BufIo<float> {
  template <int CP> __device__ static float ld(__amdgpu_buffer_rsrc_t r, int32_t byte) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte, 0, CP));
  }
  template <int CP> __device__ static void st(__amdgpu_buffer_rsrc_t r, int32_t byte, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte, 0, CP);
  }
};

template <typename T, bool BUF, int CP = 0> struct Src;
template <typename T, int CP> struct Src<T, true, CP> {
  __amdgpu_buffer_rsrc_t r;
  __device__ void init(const void *p, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc(uniptr(const_cast<void *>(p)), (short)0, uni((int)(n * (int64_t)sizeof(T))),
                                          kBufFlags);
  }
  __device__ T operator()(int32_t i) const { return BufIo<T>::template ld<CP>(r, i * (int32_t)sizeof(T)); }
  // element i if v, else 0 (read at a byte offset past any buffer below 2 GiB)
  __device__ T ld_z(bool v, int32_t i) const {
    return BufIo<T>::template ld<CP>(r, v ? i * (int32_t)sizeof(T) : (int32_t)(0x80000000u - sizeof(T)));
  }
  // the element at byte offset `byte` if v, else 0
  __device__ T ldb_z(bool v, int32_t byte) const {
    return BufIo<T>::template ld<CP>(r, v ? byte : (int32_t)(0x80000000u - sizeof(T)));
  }
  // elements i and i + 1 in one load if v, else two zeros
  __device__ void ld2_z(bool v, int32_t i, T &x0, T &x1) const {
    ld2b_z(v, i * (int32_t)sizeof(T), x0, x1);
  }
  // the two elements at byte offset `byte` if v, else two zeros
  __device__ void ld2b_z(bool v, int32_t byte_in, T &x0, T &x1) const {
    const int32_t byte = v ? byte_in : (int32_t)(0x80000000u - 2 * sizeof(T));
    if constexpr (sizeof(T) == 8) {
      const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, byte, 0, CP);
      x0 = __builtin_bit_cast(T, u2v{w[0], w[1]});
      x1 = __builtin_bit_cast(T, u2v{w[2], w[3]});
    } else {
      const u2v w = __builtin_amdgcn_raw_buffer_load_b64(r, byte, 0, CP);
      x0 = __builtin_bit_cast(T, w[0]);
      x1 = __builtin_bit_cast(T, w[1]);
    }
  }
};
template <typename T, int CP> struct Src<T, false, CP> {
  const T *__restrict__ p;
  __device__ void init(const void *q, int64_t) { p = reinterpret_cast<const T *>(q); }
  __device__ T operator()(int64_t i) const { return p[i]; }
  __device__ T ld_z(bool v, int64_t i) const { return v ? p[i] : T(0); }
};
template <typename T, bool BUF, int CP = 0> struct Dst;
template <typename T, int CP> struct Dst<T, true, CP> {
  __amdgpu_buffer_rsrc_t r;
  __device__ void init(void *p, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc(uniptr(p), (short)0, uni((int)(n * (int64_t)sizeof(T))), kBufFlags);
  }
  __device__ void put(int64_t i, T v) const { BufIo<T>::template st<CP>(r, (int32_t)i * (int32_t)sizeof(T), v); }
  // element i if v, else a byte offset past any buffer below 2 GiB (the
  // store is dropped): no per-lane branch around the store
  __device__ void put_if(bool v, int32_t i, T x) const {
    BufIo<T>::template st<CP>(r, v ? i * (int32_t)sizeof(T) : (int32_t)(0x80000000u - sizeof(T)), x);
  }
};
template <typename T, int CP> struct Dst<T, false, CP> {
  T *__restrict__ p;
  __device__ void init(void *q, int64_t) { p = reinterpret_cast<T *>(q); }
  __device__ void put(int64_t i, T v) const { p[i] = v; }
  __device__ void put_if(bool v, int64_t i, T x) const {
    if (v) p[i] = x;
  }
};

// Tile context shared by every precision: the tile's row tuple and sector,
// the problem's operands, and the lane's output columns.
template <typename In, typename Out, bool BUF, int CB> struct TileCtx {
  DevTile tile;
  DevRowTuple rt;
  DevSector sec;
  Src<In, BUF> A, B;
  Dst<Out, BUF> C;
  const char *ws;
  int64_t cbase[CB];        // output block offset of the lane's columns (-1: none)
  int32_t cnj[CB], ccl[CB];
  int cbn;
};

template <typename In, typename Out, bool BUF, int CB, bool COLS = true>
__device__ __forceinline__ DevPlan tile_setup(const LaunchArgs &args, int t, int lane, TileCtx<In, Out, BUF, CB> &x) {
  int jb = 0;
  while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
  const JobArg &job = args.jobs[jb];
  const DevPlan P = load_plan(job.plan);
  x.tile = cst(P.tiles + (t - job.tile0 + job.ptile0));
  x.rt = cst(P.rows + x.tile.rowtuple);
  x.sec = cst(P.sectors + x.tile.sector);
  const ProbPtrs pp = prob_ptrs(args, job.prob0 + x.sec.prob - job.plo);
  const DevProb pr = cst(P.probs + x.sec.prob);
  x.A.init(pp.a, pr.a_span);
  x.B.init(pp.b, pr.b_span);
  x.C.init(pp.c, pr.c_numel);
  x.ws = job.ws;
  x.cbn = (x.tile.ncols + 15) >> 4;
  if (!COLS) return P;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int lc = 16 * cb + (lane & 15);
    x.cbase[cb] = -1;
    x.cnj[cb] = 0;
    x.ccl[cb] = 0;
    if (lc < x.tile.ncols) {
      const DevColMap cm = P.colmap[x.sec.cm0 + x.tile.n0 + lc];
      x.cbase[cb] = P.cgrid[x.rt.cgrid + cm.j];
      x.cnj[cb] = cm.nj;
      x.ccl[cb] = cm.cl;
    }
  }
  return P;
}

// ---------------------------------------------------------------------------
// grouped gather GEMM (FP64 / FP32 MFMA, K = 4 per instruction)
// ---------------------------------------------------------------------------
template <typename Cmp> struct Mfma4;
template <> struct Mfma4<double> {
  typedef d4 acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // accumulator element v of lane l holds row (l>>4) + 4v, column l&15
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma4<float> {
  typedef f4 acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // accumulator element v of lane l holds row 4(l>>4) + v, column l&15
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// One wave tile: rows are processed in chunks of 16*RB; the tile's metadata
// and output columns are set up once.  Within a chunk, KB k-steps of loads
// are issued before the MFMAs that consume them.
template <typename In, typename Cmp, typename Out, bool BUF, int RB, int CB, int KB>
__global__ void __launch_bounds__(256) k_gemm4(LaunchArgs args) {
  typedef typename std::conditional<BUF, int32_t, int64_t>::type Off;
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int W = gridDim.x * 4;
  for (int t = gw; t < args.ntiles; t += W) {
    TileCtx<In, Out, BUF, CB> x;
    const DevPlan P = tile_setup<In, Out, BUF, CB>(args, t, lane, x);
    const Cmp *__restrict__ Bp = reinterpret_cast<const Cmp *>(x.ws) + x.sec.bpack;
    const int64_t *__restrict__ kofs = P.kofs + x.rt.kofs;
    const DevKP *__restrict__ kp = P.kp + x.sec.kp0;
    const int K = x.sec.K, N = x.sec.N;
    for (int mc = 0; mc < x.tile.nrows; mc += 16 * RB) {
      const int rows = min(16 * RB, x.tile.nrows - mc);
      const int rbn = (rows + 15) >> 4;
      int32_t rg[RB][kMaxAct];
      bool rv[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int lr = 16 * rb + (lane & 15);
        rv[rb] = lr < rows;
        a_rowparts(x.rt, x.sec.nact, x.tile.m0 + mc + lr, rg[rb]);
      }
      acc_t acc[RB][CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};
      // k metadata of the next batch is fetched while this batch's A loads fly
      int64_t kon[KB];
      DevKP pn[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const int k = 4 * q + (lane >> 4);
        kon[q] = k < K ? kofs[k] : -1;
        pn[q] = k < K ? kp[k] : DevKP{};
      }
      for (int kk0 = 0; kk0 < K; kk0 += 4 * KB) {
        Cmp av[KB][RB], bv[KB][CB];
        int64_t ko[KB];
        DevKP pc[KB];
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          ko[q] = kon[q];
          pc[q] = pn[q];
        }
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          const int k = kk0 + 4 * q + (lane >> 4);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            av[q][rb] = (ko[q] >= 0 && rv[rb]) ? Cmp(x.A(a_offset_t<Off>(ko[q], pc[q].p, rg[rb]))) : Cmp(0);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int c = x.tile.n0 + 16 * cb + (lane & 15);
            bv[q][cb] = (k < K && c < N) ? Bp[(int64_t)k * N + c] : Cmp(0);
          }
        }
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          const int k = kk0 + 4 * KB + 4 * q + (lane >> 4);
          kon[q] = k < K ? kofs[k] : -1;
          pn[q] = k < K ? kp[k] : DevKP{};
        }
#pragma unroll
        for (int q = 0; q < KB; ++q)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (rb < rbn)
#pragma unroll
              for (int cb = 0; cb < CB; ++cb)
                if (cb < x.cbn) acc[rb][cb] = M::run(av[q][rb], bv[q][cb], acc[rb][cb]);
      }
      // element (row, col) of C_X -> output block (i, j_col), row-major m_i x n_j
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= x.cbn || x.cbase[cb] < 0) continue;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + M::row(lane, v);
            if (lr < rows)
              x.C.put(x.cbase[cb] + (int64_t)(x.tile.m0 + mc + lr) * x.cnj[cb] + x.ccl[cb], Out(acc[rb][cb][v]));
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// tall-skinny sectors (K, N <= 64): one row of C_X per lane, VALU FMA
// ---------------------------------------------------------------------------
// HBM-bound shapes (tens of thousands of rows, K and N of a few tens): each
// lane gathers its row of A_X (all K values at once, coalesced across the
// wave's consecutive rows) and accumulates 16 columns at a time with B_X
// values that are uniform across the wave, so the k offsets, P factors and
// B_X come from scalar loads.  No padding of K or N.
template <typename In, typename Cmp, typename Out, bool BUF, int KMAX>
__global__ void __launch_bounds__(256) k_rows(LaunchArgs args) {
  typedef typename std::conditional<BUF, int32_t, int64_t>::type Off;
  __shared__ Cmp bs_all[4][KMAX][16];  // per wave: B_X rows 0..K-1, the 16 columns of one pass
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Cmp (*bs)[16] = bs_all[wid];
  const int gw = blockIdx.x * 4 + wid;  // wave-uniform
  const int W = gridDim.x * 4;
  for (int t = gw; t < args.ntiles; t += W) {
    TileCtx<In, Out, BUF, 1> x;
    const DevPlan P = tile_setup<In, Out, BUF, 1>(args, t, lane, x);
    const Cmp *__restrict__ Bp = reinterpret_cast<const Cmp *>(x.ws) + x.sec.bpack;
    const int64_t *kofs = P.kofs + x.rt.kofs;
    const DevKP *kp = P.kp + x.sec.kp0;
    const DevColMap *cmap = P.colmap + x.sec.cm0 + x.tile.n0;
    const int64_t *cgrid = P.cgrid + x.rt.cgrid;
    const int K = uni(x.sec.K), N = uni(x.sec.N), ncols = uni(x.tile.ncols), nrows = uni(x.tile.nrows);
    for (int mc = 0; mc < nrows; mc += 64) {
      const int lr = mc + lane;
      const bool valid = lr < nrows;
      const int32_t ra = x.tile.m0 + lr;
      int32_t rg[kMaxAct];
      a_rowparts(x.rt, x.sec.nact, ra, rg);
      Cmp a[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        a[k] = Cmp(0);
        if (k < K) {
          const int64_t ko = cst(kofs + k);
          const DevKP p = cst(kp + k);
          if (valid && ko >= 0) a[k] = Cmp(x.A(a_offset_t<Off>(ko, p.p, rg)));
        }
      }
      for (int cc = 0; cc < ncols; cc += 16) {
        const int nc = min(16, ncols - cc);
        // stage B_X[k][n0 + cc + c] (zero beyond K and the tile's columns)
        for (int e = lane; e < KMAX * 16; e += 64) {
          const int k = e >> 4, c = e & 15;
          bs[k][c] = (k < K && c < nc) ? Bp[(int64_t)k * N + x.tile.n0 + cc + c] : Cmp(0);
        }
        wave_lds_sync();
        Cmp acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = Cmp(0);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < K) {
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[c] = fma(a[k], bs[k][c], acc[c]);
          }
        }
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < nc) {
            const DevColMap cm = cst(cmap + cc + c);
            const int64_t cbase = cst(cgrid + cm.j);
            if (valid && cbase >= 0) x.C.put(cbase + (int64_t)ra * cm.nj + cm.cl, Out(acc[c]));
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// grouped gather GEMM, split-BF16 products on bf16 MFMA (K = 32 per instruction)
// ---------------------------------------------------------------------------
// x = hi + mid + lo with hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid)
// (round to nearest even).  NT = 3: hi*hi + hi*mid + mid*hi;  NT = 6 adds
// mid*mid + hi*lo + lo*hi.  FP32 accumulation.
template <int NT>
__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
  const uint16_t hb = bf16_rne(x);
  const float r = x - bf16_to_f(hb);
  const uint16_t mb = bf16_rne(r);
  uint16_t lb = 0;
  if (NT > 3) lb = bf16_rne(r - bf16_to_f(mb));
  h = __builtin_bit_cast(__bf16, hb);
  m = __builtin_bit_cast(__bf16, mb);
  l = __builtin_bit_cast(__bf16, lb);
}

template <typename In, typename Out, bool BUF, int RB, int CB, int NT>
__global__ void __launch_bounds__(256) k_gemm_bf16(LaunchArgs args) {
  typedef typename std::conditional<BUF, int32_t, int64_t>::type Off;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int W = gridDim.x * 4;
  for (int t = gw; t < args.ntiles; t += W) {
    TileCtx<In, Out, BUF, CB> x;
    const DevPlan P = tile_setup<In, Out, BUF, CB>(args, t, lane, x);
    const float *__restrict__ Bp = reinterpret_cast<const float *>(x.ws) + x.sec.bpack;
    const int64_t *__restrict__ kofs = P.kofs + x.rt.kofs;
    const DevKP *__restrict__ kp = P.kp + x.sec.kp0;
    const int K = x.sec.K, N = x.sec.N;
    for (int mc = 0; mc < x.tile.nrows; mc += 16 * RB) {
      const int rows = min(16 * RB, x.tile.nrows - mc);
      const int rbn = (rows + 15) >> 4;
      int32_t rg[RB][kMaxAct];
      bool rv[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int lr = 16 * rb + (lane & 15);
        rv[rb] = lr < rows;
        a_rowparts(x.rt, x.sec.nact, x.tile.m0 + mc + lr, rg[rb]);
      }
      f4 acc[RB][CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f4{0, 0, 0, 0};
      for (int kk = 0; kk < K; kk += 32) {
        bf8 ah[RB], am[RB], al[RB], bh[CB], bm[CB], bl[CB];
        float av[8][RB], bv[8][CB];
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {  // this lane's 8 consecutive k
          const int k = kk + 8 * (lane >> 4) + e8;
          int64_t ko = -1;
          DevKP p{};
          if (k < K) {
            ko = kofs[k];
            p = kp[k];
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            av[e8][rb] = (ko >= 0 && rv[rb]) ? float(x.A(a_offset_t<Off>(ko, p.p, rg[rb]))) : 0.f;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int c = x.tile.n0 + 16 * cb + (lane & 15);
            bv[e8][cb] = (k < K && c < N) ? Bp[(int64_t)k * N + c] : 0.f;
          }
        }
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            __bf16 h, m, l;
            split3<NT>(av[e8][rb], h, m, l);
            ah[rb][e8] = h;
            am[rb][e8] = m;
            al[rb][e8] = l;
          }
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            __bf16 h, m, l;
            split3<NT>(bv[e8][cb], h, m, l);
            bh[cb][e8] = h;
            bm[cb][e8] = m;
            bl[cb][e8] = l;
          }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            if (cb >= x.cbn) continue;
            f4 c = acc[rb][cb];
            // small terms first, largest last
            if (NT > 3) {
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rb], bh[cb], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bl[cb], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[rb], bm[cb], c, 0, 0, 0);
            }
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[rb], bh[cb], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bm[cb], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bh[cb], c, 0, 0, 0);
            acc[rb][cb] = c;
          }
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= x.cbn || x.cbase[cb] < 0) continue;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + 4 * (lane >> 4) + v;
            if (lr < rows)
              x.C.put(x.cbase[cb] + (int64_t)(x.tile.m0 + mc + lr) * x.cnj[cb] + x.ccl[cb], Out(acc[rb][cb][v]));
          }
        }
      }
    }
  }
}


// x * y for a row index (or row part) and a per-row factor (class factor,
// output block width): with 32-bit offsets both are below 2^24 (plans check
// the row counts and widths for the kernels that use this), so the product is
// a full-rate 24-bit multiply; 64-bit offsets multiply in 64 bits.
template <typename Off> __device__ __forceinline__ Off mul_rows(int32_t x, int32_t y) {
  if constexpr (sizeof(Off) == 4)
    return (Off)__umul24((uint32_t)x, (uint32_t)y);
  else
    return (Off)x * (Off)y;
}

// ---------------------------------------------------------------------------
// grouped gather GEMM with the tile's B columns resident in registers
// ---------------------------------------------------------------------------
// For sectors with K_X <= 4*KQ.  A wave loads, once per tile, the k offsets
// and class factors of its k slots and the B_X values of its k slots and
// columns (straight from B's blocks through the plan's per-sector offset
// table, so no packed copy of B is needed), then walks the tile's rows in
// chunks of 16*RB.  The A loads of chunk c+1 are issued before the MFMAs and
// stores of chunk c, so every wave keeps a chunk of loads in flight while it
// computes.  NA = free-leg classes supported (nact <= NA).
template <typename In, typename Off, bool BUF, int RB, int KQ, int NA>
__device__ __forceinline__ void res_load_chunk(const Src<In, BUF, kStream> &A, const DevRowTuple &rt, int nact, int K,
                                               int32_t row0, int rows, int lane, const Off (&ko)[KQ],
                                               const int32_t (&pk)[KQ][NA], In (&av)[KQ][RB]) {
  // Loads only (no per-lane branch, no use of a loaded value), so the chunk's
  // loads stay in flight until its MFMAs: padding rows and k slots past K
  // read 0 from past the end of the buffer; k quads past K (wave-uniform)
  // are skipped, their MFMAs too.
  int32_t rg[RB][NA];
  bool rv[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int lr = 16 * rb + (lane & 15);
    rv[rb] = lr < rows;
    a_rowparts_fast<NA, true>(rt, nact, row0 + (rv[rb] ? lr : 0), rg[rb]);
  }
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (4 * q < K) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        Off o = ko[q];
#pragma unroll
        for (int a = 0; a < NA; ++a) o += mul_rows<Off>(pk[q][a], rg[rb][a]);
        av[q][rb] = A.ld_z(ko[q] >= 0 && rv[rb], o);
      }
    }
}

// The lane's output columns of a tile (MFMA layout: column lane & 15 of each
// 16-column block): base offset of the column's output block, its width n_j
// and the column within it; base -1 for padding columns.  Both table reads
// of every column are issued together.
template <typename Off, int CB>
__device__ __forceinline__ void tile_columns(const DevColMap *cmap, const int64_t *cgrid, int ncols, int lane,
                                             Off (&cbase)[CB], int32_t (&cnj)[CB], int32_t (&ccl)[CB]) {
  DevColMap cm[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int lc = 16 * cb + (lane & 15);
    cm[cb] = cmap[lc < ncols ? lc : 0];
  }
  int64_t g[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) g[cb] = cgrid[cm[cb].j];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const bool v = 16 * cb + (lane & 15) < ncols;
    cbase[cb] = v ? (Off)g[cb] : (Off)-1;
    cnj[cb] = cm[cb].nj;
    ccl[cb] = cm[cb].cl;
  }
}

// One tile's record and operands, read field by field with scalar loads.
template <typename In, typename Out, bool BUF> struct RecCtx {
  const int64_t *kofs;
  const DevKP *kp;
  const int32_t *bofs;
  const DevColMap *cmap;
  const int64_t *cgrid;
  const DevColRes *colres;  // resolved output columns (null: use cmap and cgrid)
  int32_t m0, nrows, n0, ncols, K, N, nact;
  int32_t split;   // 1: split-K tile, accumulators go to the partial slot at `part`
  int64_t part;    // workspace byte offset of the partial slot
  int64_t bpack;   // the sector's packed B_X in the workspace (elements)
  DevRowTuple rt;  // only lsuf / lmag / lsh of classes 1..kRecAct are filled
  Src<In, BUF, kStream> A;
  Src<In, BUF> B;
  Dst<Out, BUF, kStream> C;
};

template <typename In, typename Out, bool BUF>
__device__ __forceinline__ void rec_setup(const LaunchArgs &args, const JobArg &job, const DevTileRec *r,
                                          RecCtx<In, Out, BUF> &x);

template <typename In, typename Out, bool BUF>
__device__ __forceinline__ void rec_setup(const LaunchArgs &args, int t, RecCtx<In, Out, BUF> &x) {
  int jb = 0;
  while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
  const JobArg &job = args.jobs[jb];
  rec_setup<In, Out, BUF>(args, job, cst(&job.recs) + (t - job.tile0 + job.ptile0), x);
}

// The record r of a tile of `job`.
template <typename In, typename Out, bool BUF>
__device__ __forceinline__ void rec_setup(const LaunchArgs &args, const JobArg &job, const DevTileRec *r,
                                          RecCtx<In, Out, BUF> &x) {
  x.kofs = cst(&r->kofs);
  x.kp = cst(&r->kp);
  x.bofs = cst(&r->bofs);
  x.cmap = cst(&r->cmap);
  x.cgrid = cst(&r->cgrid);
  x.colres = cst(&r->colres);
  const int64_t a_span = cst(&r->a_span), b_span = cst(&r->b_span), c_numel = cst(&r->c_numel);
  x.m0 = cst(&r->m0);
  x.nrows = cst(&r->nrows);
  x.n0 = cst(&r->n0);
  x.ncols = cst(&r->ncols);
  x.K = cst(&r->K);
  x.N = cst(&r->N);
  x.nact = cst(&r->nact);
  x.bpack = cst(&r->bpack);
  x.split = cst(&r->split);
  x.part = cst(&r->part);
  const int32_t prob = cst(&r->prob);
#pragma unroll
  for (int a = 0; a < kRecAct; ++a) {
    x.rt.lsuf[a + 1] = cst(&r->lsuf[a]);
    x.rt.lmag[a + 1] = cst(&r->lmag[a]);
    x.rt.lsh[a + 1] = cst(&r->lsh[a]);
  }
  const ProbPtrs pp = prob_ptrs(args, job.prob0 + prob - job.plo);
  x.A.init(pp.a, a_span);
  x.B.init(pp.b, b_span);
  x.C.init(pp.c, c_numel);
}

// NT = 0: products in Cmp on the FP64 / FP32 MFMA 16x16x4.  NT = 3 or 6:
// split-BF16 products (Cmp = float values split into 2 or 3 bf16 terms) on
// the bf16 MFMA 16x16x32 with FP32 accumulation; eight of the lane's k slots
// form one instruction's k group (slot q = 8s + j holds k = kl + 4q, the same
// for A and B, so each group covers k = 32s .. 32s + 31 once).
template <typename In, typename Cmp, typename Out, bool BUF, int RB, int CB, int KQ, int NA, int PD, int OCC,
          int NT = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) k_gemm_res(LaunchArgs args) {
  static_assert(NA <= kRecAct + 1, "tile records carry kRecAct class boundaries");
  static_assert(NT == 0 || (std::is_same<Cmp, float>::value && KQ % 8 == 0), "split-BF16 tiles: FP32 values, 8k slots");
  constexpr int NS = NT > 3 ? 3 : 2;  // bf16 terms per value
  typedef typename std::conditional<BUF, int32_t, int64_t>::type Off;
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4;
  const int gw = blockIdx.x * 4 + uni(threadIdx.x >> 6);  // wave-uniform
  const int W = gridDim.x * 4;
  const bool do_norm = args.norm.parts != nullptr;
  NormAcc nacc;
  for (int t = gw; t < args.ntiles; t += W) {
    RecCtx<In, Out, BUF> x;
    rec_setup<In, Out, BUF>(args, t, x);
    const int K = x.K, N = x.N, nact = x.nact, nrows = x.nrows;
    const int cbn = (x.ncols + 15) >> 4;
    Off cbase[CB];
    int32_t cnj[CB], ccl[CB];
    tile_columns<Off, CB>(x.cmap, x.cgrid, x.ncols, lane, cbase, cnj, ccl);
    // k slots of this lane: offset of (row 0, k), class factors, and the B
    // values of its columns; every table read is issued before any is used
    // (k slots past K read entry 0 and are masked afterwards)
    Off ko[KQ];
    int32_t pk[KQ][NA];
    Cmp bv[KQ][CB];
    {
      int32_t bo[KQ][CB];
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int k = 4 * q + kl;
        const int kk = k < K ? k : 0;
        ko[q] = (Off)x.kofs[kk];
#pragma unroll
        for (int a = 0; a < NA; ++a) pk[q][a] = x.kp[kk].p[a];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int c = x.n0 + 16 * cb + (lane & 15);
          bo[q][cb] = x.bofs[(k < K && c < N) ? (int64_t)kk * N + c : 0];
        }
      }
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        ko[q] = 4 * q + kl < K ? ko[q] : (Off)-1;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int c = x.n0 + 16 * cb + (lane & 15);
          bv[q][cb] = Cmp(x.B.ld_z(4 * q + kl < K && c < N && bo[q][cb] >= 0, bo[q][cb]));
        }
      }
    }
    // split-BF16: the B terms of each k group, once per tile
    bf8 bs[NT ? KQ / 8 : 1][CB][NS];
    if constexpr (NT > 0) {
#pragma unroll
      for (int g = 0; g < KQ / 8; ++g)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            __bf16 h, m, l;
            split3<NT>(bv[8 * g + j][cb], h, m, l);
            bs[g][cb][0][j] = h;
            bs[g][cb][1][j] = m;
            if constexpr (NS > 2) bs[g][cb][NS - 1][j] = l;
          }
    }
    // rows in chunks of 16 * RB; the A loads of chunk c + PD are issued
    // before the MFMAs of chunk c (a ring of PD + 1 register buffers)
    const int nch = (nrows + 16 * RB - 1) / (16 * RB);
    In ab[PD + 1][KQ][RB];
    auto load_chunk = [&](int c, In (&dst)[KQ][RB]) {
      res_load_chunk<In, Off, BUF, RB, KQ, NA>(x.A, x.rt, nact, K, x.m0 + c * 16 * RB,
                                               min(16 * RB, nrows - c * 16 * RB), lane, ko, pk, dst);
    };
    auto compute_chunk = [&](int c, const In (&av)[KQ][RB]) {
      const int mc = c * 16 * RB;
      const int rows = min(16 * RB, nrows - mc);
      const int rbn = (rows + 15) >> 4;
      acc_t acc[RB][CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};
      if constexpr (NT == 0) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
          if (4 * q < K) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
              if (rb < rbn)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                  if (cb < cbn) acc[rb][cb] = M::run(Cmp(av[q][rb]), bv[q][cb], acc[rb][cb]);
          }
        }
      } else {
#pragma unroll
        for (int g = 0; g < KQ / 8; ++g) {
          if (32 * g < K) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              if (rb >= rbn) continue;
              bf8 as[NS];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                __bf16 h, m, l;
                split3<NT>(Cmp(av[8 * g + j][rb]), h, m, l);
                as[0][j] = h;
                as[1][j] = m;
                if constexpr (NS > 2) as[NS - 1][j] = l;
              }
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                if (cb >= cbn) continue;
                acc_t c = acc[rb][cb];
                // small terms first, the leading product last
                if constexpr (NS > 2) {
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[2], bs[g][cb][0], c, 0, 0, 0);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[0], bs[g][cb][2], c, 0, 0, 0);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[1], bs[g][cb][1], c, 0, 0, 0);
                }
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[1], bs[g][cb][0], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[0], bs[g][cb][1], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[0], bs[g][cb][0], c, 0, 0, 0);
                acc[rb][cb] = c;
              }
            }
          }
        }
      }
      // stores without per-lane branches (padding rows and columns: dropped)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= cbn) continue;
        const bool cv = cbase[cb] >= 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + M::row(lane, v);
            const bool ok = cv && lr < rows;
            const Out val = Out(acc[rb][cb][v]);
            x.C.put_if(ok, cbase[cb] + mul_rows<Off>(x.m0 + mc + lr, cnj[cb]) + (Off)ccl[cb], val);
            if (do_norm) nacc.add(ok ? (double)val : 0.0);
          }
        }
      }
    };
#pragma unroll
    for (int u = 0; u < PD; ++u)
      if (u < nch) load_chunk(u, ab[u]);
    for (int c0 = 0; c0 < nch; c0 += PD + 1) {
#pragma unroll
      for (int u = 0; u <= PD; ++u) {
        const int c = c0 + u;
        if (c < nch) {
          if (c + PD < nch) load_chunk(c + PD, ab[(u + PD) % (PD + 1)]);
          compute_chunk(c, ab[u]);
        }
      }
    }
    if (do_norm) norm_file_tile(args.norm, t, lane, nacc);
  }
}

// ---------------------------------------------------------------------------
// grouped gather GEMM with the B tile shared in LDS by a workgroup
// ---------------------------------------------------------------------------
// For sectors with K_X <= 4*KQ.  A workgroup takes a job of up to eight wave
// tiles of one (sector, column range): its 256 threads load the B_X tile
// (4*KQ k rows x 16*CB columns, zero past K and N, straight from B's blocks
// through the offset table) into LDS once, then each wave computes its tiles
// as k_gemm_res does, reading the B operand of every MFMA from LDS.  The B
// load is paid once per job instead of once per tile, and the registers it
// held in k_gemm_res are free for more resident waves.
// res_load_chunk with the k metadata read from the wave's LDS slice
// (kw[k] = {A byte offset of (row 0, k) or -1, class factors in bytes}).
// Row parts are below 2^24 (plans check the row counts) and the class
// factors are at most K_X * 8, so every product is a full-rate 24-bit
// multiply-add (a 32-bit integer multiply issues at a quarter of the rate).
template <typename In, int RB, int KQ, int NA>
__device__ __forceinline__ void lds_load_chunk(const Src<In, true, kStream> &A, const DevRowTuple &rt, int nact,
                                               int K, int32_t row0, int rows, int lane, const int32_t (*kw)[1 + NA],
                                               In (&av)[KQ][RB]) {
  int32_t rg[RB][NA];
  bool rv[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int lr = 16 * rb + (lane & 15);
    rv[rb] = lr < rows;
    a_rowparts_fast<NA, true>(rt, nact, row0 + (rv[rb] ? lr : 0), rg[rb]);
  }
  const int kl = lane >> 4;
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (4 * q < K) {
      const int32_t *m = kw[4 * q + kl];
      const int32_t ko = m[0];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        int32_t o = ko;
#pragma unroll
        for (int a = 0; a < NA; ++a) o += (int32_t)__umul24((uint32_t)m[1 + a], (uint32_t)rg[rb][a]);
        av[q][rb] = A.ldb_z(ko >= 0 && rv[rb], o);
      }
    }
}

// lds_load_chunk for paired rows (RB = 2): lane i of a 16-lane group loads
// rows 2i and 2i + 1 of the chunk in one 2-element load, into av[q][0] and
// av[q][1].  Valid when the innermost free-leg class of every row tuple has
// an even run length with unit stride (rows 2i, 2i + 1 adjacent in memory)
// and every chunk starts at an even row; then a tile's row count is even, so
// both rows of a pair are valid or both are padding.
template <typename In, int KQ, int NA>
__device__ __forceinline__ void lds_load_chunk_pair(const Src<In, true, kStream> &A, const DevRowTuple &rt, int nact,
                                                    int K, int32_t row0, int rows, int lane,
                                                    const int32_t (*kw)[1 + NA], In (&av)[KQ][2]) {
  int32_t rg[NA];
  const int lr = 2 * (lane & 15);
  const bool rv = lr < rows;
  a_rowparts_fast<NA, true>(rt, nact, row0 + (rv ? lr : 0), rg);
  const int kl = lane >> 4;
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (4 * q < K) {
      const int32_t *m = kw[4 * q + kl];
      const int32_t ko = m[0];
      int32_t o = ko;
#pragma unroll
      for (int a = 0; a < NA; ++a) o += (int32_t)__umul24((uint32_t)m[1 + a], (uint32_t)rg[a]);
      A.ld2b_z(ko >= 0 && rv, o, av[q][0], av[q][1]);
    }
}

// The tile's output columns from its resolved column table (one 16-byte
// load per column block instead of the column map and then the output block
// offsets).
template <typename Off, int CB>
__device__ __forceinline__ void tile_columns_res(const DevColRes *cr, int ncols, int lane, Off (&cbase)[CB],
                                                 int32_t (&cnj)[CB], int32_t (&ccl)[CB]) {
  DevColRes e[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int lc = 16 * cb + (lane & 15);
    e[cb] = cr[lc < ncols ? lc : 0];
  }
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const bool v = 16 * cb + (lane & 15) < ncols;
    cbase[cb] = v ? (Off)e[cb].cbase : (Off)-1;
    cnj[cb] = e[cb].nj;
    ccl[cb] = e[cb].cl;
  }
}

// NORM: the instance that files the fused output norm (the others carry none
// of its code).  PAIR (RB = 2): rows loaded in adjacent pairs, row block 0 of
// the MFMA holds the chunk's even rows and block 1 its odd rows.
//
// A workgroup job is one B tile (a sector's k range x column range) and one
// tile of rows per wave.  Its start is arranged as few dependent round trips
// as the data allows: the job's fields and the wave's tile record (stored in
// job order, so its address needs no load) are read together; then the B
// tile's offsets, the tile's output columns and its k metadata; then the B
// values and, once the k metadata is in the wave's LDS slice, the A loads of
// the tile's first row chunk, which are in flight while the B tile is
// written to LDS and the workgroup waits for it.
template <typename In, typename Cmp, typename Out, int RB, int CB, int KQ, int NA, int PD, int OCC, bool NORM,
          bool PAIR = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) k_gemm_lds(LaunchArgs args) {
  static_assert(NA <= kRecAct + 1, "tile records carry kRecAct class boundaries");
  static_assert(!PAIR || RB == 2, "paired rows fill two row blocks");
  static_assert(kLdsJobTiles == 4, "one tile per wave of a job");
  constexpr bool BUF = true;
  typedef int32_t Off;
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  constexpr int BW = 16 * CB;                  // tile columns
  constexpr int BE = 4 * KQ * BW;              // B tile elements
  constexpr int BR = (BE + 255) / 256;         // per thread
  __shared__ Cmp bl[4 * KQ][BW];
  __shared__ int32_t kls[4][4 * KQ][1 + NA];  // per wave: A offset of (row 0, k) (-1 past K), class factors
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4;
  const int w = uni(threadIdx.x >> 6);
  NormAcc nacc;
  struct Tile {
    RecCtx<In, Out, BUF> x;
    Off cbase[CB];
    int32_t cnj[CB], ccl[CB];
  };
  auto load_chunk = [&](const Tile &T, int c, In (&dst)[KQ][RB]) {
    const RecCtx<In, Out, BUF> &x = T.x;
    if constexpr (PAIR)
      lds_load_chunk_pair<In, KQ, NA>(x.A, x.rt, x.nact, x.K, x.m0 + c * 16 * RB, min(16 * RB, x.nrows - c * 16 * RB),
                                      lane, kls[w], dst);
    else
      lds_load_chunk<In, RB, KQ, NA>(x.A, x.rt, x.nact, x.K, x.m0 + c * 16 * RB, min(16 * RB, x.nrows - c * 16 * RB),
                                     lane, kls[w], dst);
  };
  // the tile's rows in chunks of 16 * RB, A loads PD chunks ahead; chunk 0
  // is already in ab[0]
  auto run = [&](int32_t tl, const Tile &T, In (&ab)[PD + 1][KQ][RB]) {
    const RecCtx<In, Out, BUF> &x = T.x;
    const int K = x.K, nrows = x.nrows;
    const int cbn = (x.ncols + 15) >> 4;
    const int nch = (nrows + 16 * RB - 1) / (16 * RB);
    auto compute_chunk = [&](int c, const In (&av)[KQ][RB]) {
      const int mc = c * 16 * RB;
      const int rows = min(16 * RB, nrows - mc);
      // paired rows: both row blocks hold rows of any chunk (even, odd rows)
      const int rbn = PAIR ? RB : (rows + 15) >> 4;
      acc_t acc[RB][CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        if (4 * q < K) {
          Cmp b[CB];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) b[cb] = bl[4 * q + kl][16 * cb + (lane & 15)];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (rb < rbn)
#pragma unroll
              for (int cb = 0; cb < CB; ++cb)
                if (cb < cbn) acc[rb][cb] = M::run(Cmp(av[q][rb]), b[cb], acc[rb][cb]);
        }
      }
      // stores without per-lane branches: padding rows and columns store past
      // the end of C (dropped) and add 0 to the norm
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= cbn) continue;
        const bool cv = T.cbase[cb] >= 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = PAIR ? 2 * M::row(lane, v) + rb : 16 * rb + M::row(lane, v);
            const bool ok = cv && lr < rows;
            const Out val = Out(acc[rb][cb][v]);
            x.C.put_if(ok, T.cbase[cb] + (Off)__umul24((uint32_t)(x.m0 + mc + lr), (uint32_t)T.cnj[cb]) + (Off)T.ccl[cb],
                       val);
            if constexpr (NORM) nacc.add(ok ? (double)val : 0.0);
          }
        }
      }
    };
#pragma unroll
    for (int u = 1; u < PD; ++u)
      if (u < nch) load_chunk(T, u, ab[u]);
    for (int c0 = 0; c0 < nch; c0 += PD + 1) {
#pragma unroll
      for (int u = 0; u <= PD; ++u) {
        const int c = c0 + u;
        if (c < nch) {
          if (c + PD < nch && c + PD > 0) load_chunk(T, c + PD, ab[(u + PD) % (PD + 1)]);
          compute_chunk(c, ab[u]);
        }
      }
    }
    // single-problem launches: plan-local tile index = part index
    if constexpr (NORM) norm_file_tile(args.norm, tl, lane, nacc);
  };
  for (int j = blockIdx.x; j < args.ntiles; j += gridDim.x) {
    int jb = 0;
    while (jb + 1 < args.njobs && j >= args.jobs[jb + 1].tile0) ++jb;
    const JobArg &job = args.jobs[jb];
    const int32_t jl = j - job.tile0 + job.ptile0;
    const DevLdsJob *lj = cst(&job.ljobs) + jl;
    Tile T;
    rec_setup<In, Out, BUF>(args, job, cst(&job.ljrecs) + (int64_t)jl * kLdsJobTiles + w, T.x);
    const int32_t tl = uni(cst(&lj->t[w]));
    const int32_t *bofs = cst(&lj->bofs);
    const int32_t K = cst(&lj->K), N = cst(&lj->N), n0 = cst(&lj->n0);
    Src<In, BUF> B;
    B.init(prob_ptrs(args, job.prob0 + cst(&lj->prob) - job.plo).b, cst(&lj->b_span));
    // B tile offsets, the tile's output columns and its k metadata
    int32_t bo[BR];
    bool bv[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int e = min((int)threadIdx.x + 256 * i, BE - 1);
      const int k = e / BW, c = n0 + e % BW;
      bv[i] = k < K && c < N;
      bo[i] = bofs[bv[i] ? k * N + c : 0];
    }
    if (T.x.colres)
      tile_columns_res<Off, CB>(T.x.colres, T.x.ncols, lane, T.cbase, T.cnj, T.ccl);
    else
      tile_columns<Off, CB>(T.x.cmap, T.x.cgrid, T.x.ncols, lane, T.cbase, T.cnj, T.ccl);
    int32_t ko[(4 * KQ + 63) / 64], pk[(4 * KQ + 63) / 64][NA];
#pragma unroll
    for (int k0 = 0; k0 < 4 * KQ; k0 += 64) {
      const int k = k0 + lane;
      const int kk = k < T.x.K ? k : 0;
      ko[k0 / 64] = k < T.x.K ? (int32_t)T.x.kofs[kk] : -1;
#pragma unroll
      for (int a = 0; a < NA; ++a) pk[k0 / 64][a] = T.x.kp[kk].p[a];
    }
    // B values
    In v[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) v[i] = B.ld_z(bv[i] && bo[i] >= 0, bo[i]);
    // k metadata into the wave's LDS slice, then the first chunk's A loads
#pragma unroll
    for (int k0 = 0; k0 < 4 * KQ; k0 += 64) {
      const int k = k0 + lane;
      if (k < 4 * KQ) {
        kls[w][k][0] = ko[k0 / 64] >= 0 ? ko[k0 / 64] * (int32_t)sizeof(In) : -1;
#pragma unroll
        for (int a = 0; a < NA; ++a) kls[w][k][1 + a] = pk[k0 / 64][a] * (int32_t)sizeof(In);
      }
    }
    wave_lds_sync();
    In ab[PD + 1][KQ][RB];
    const bool live = T.x.nrows > 0;  // empty job slot: a copy of slot 0 with no rows
    if (live) load_chunk(T, 0, ab[0]);
    // the B tile into LDS
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      const int e = (int)threadIdx.x + 256 * i;
      if (e < BE) bl[e / BW][e % BW] = Cmp(v[i]);
    }
    __syncthreads();
    if (live) run(tl, T, ab);
    __syncthreads();  // the next job overwrites the B tile and the k metadata
  }
}

// ---------------------------------------------------------------------------
// shared-B grouped GEMM for sectors of any K, k in chunks through LDS
// ---------------------------------------------------------------------------
// The shared-B kernel's jobs (four tiles of 16 * RB rows of one sector column
// range, one per wave) with K walked in chunks of 4 * KQ: the workgroup
// stages each chunk of the B tile in LDS (two buffers, alternating, so the
// workgroup meets once per chunk) straight from B's blocks through
// the plan's offset table (no packed copy of B, so no pack pass), each wave
// stages the chunk's k metadata in its LDS slice (two slices, alternating)
// and keeps its accumulators across the chunks.  While the MFMAs of chunk c
// run, the loads of chunk c + 1 (B values, A) and the offsets of chunk c + 2
// (B offsets, k metadata) are in flight.  Tiles hold at most 16 * RB rows.
template <typename In, typename Cmp, typename Out, int RB, int CB, int KQ, int NA, int OCC, bool NORM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) k_gemm_ldsk(LaunchArgs args) {
  static_assert(NA <= kRecAct + 1, "tile records carry kRecAct class boundaries");
  static_assert(kLdsJobTiles == 4, "one tile per wave of a job");
  static_assert(4 * KQ <= 64, "one k of a chunk per lane");
  constexpr bool BUF = true;
  typedef int32_t Off;
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  constexpr int BW = 16 * CB;       // tile columns
  constexpr int KC = 4 * KQ;        // k of a chunk
  constexpr int BE = KC * BW;       // B chunk elements
  constexpr int BR = (BE + 255) / 256;
  __shared__ Cmp bl[2][KC][BW];  // two chunks, alternating
  __shared__ int32_t kls[4][2][KC][1 + NA];  // per wave, two chunks: A byte offset of (row 0, k) or -1, factors
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4;
  const int w = uni(threadIdx.x >> 6);
  NormAcc nacc;
  for (int j = blockIdx.x; j < args.ntiles; j += gridDim.x) {
    int jb = 0;
    while (jb + 1 < args.njobs && j >= args.jobs[jb + 1].tile0) ++jb;
    const JobArg &job = args.jobs[jb];
    const int32_t jl = j - job.tile0 + job.ptile0;
    const DevLdsJob *lj = cst(&job.ljobs) + jl;
    RecCtx<In, Out, BUF> x;
    rec_setup<In, Out, BUF>(args, job, cst(&job.ljrecs) + (int64_t)jl * kLdsJobTiles + w, x);
    const int32_t tl = uni(cst(&lj->t[w]));
    const int32_t *bofs = cst(&lj->bofs);
    const int32_t K = cst(&lj->K), N = cst(&lj->N), n0 = cst(&lj->n0);
    Src<In, BUF> B;
    B.init(prob_ptrs(args, job.prob0 + cst(&lj->prob) - job.plo).b, cst(&lj->b_span));
    Off cbase[CB];
    int32_t cnj[CB], ccl[CB];
    if (x.colres)
      tile_columns_res<Off, CB>(x.colres, x.ncols, lane, cbase, cnj, ccl);
    else
      tile_columns<Off, CB>(x.cmap, x.cgrid, x.ncols, lane, cbase, cnj, ccl);
    const bool live = x.nrows > 0;  // empty job slot: a copy of slot 0 with no rows
    const int nk = (K + KC - 1) / KC;
    // per-chunk loads: the B tile's offsets, the tile's k metadata (one k per
    // lane), the B values, the A values
    auto load_bofs = [&](int c, int32_t (&bo)[BR], bool (&bv)[BR]) {
#pragma unroll
      for (int i = 0; i < BR; ++i) {
        const int e = min((int)threadIdx.x + 256 * i, BE - 1);
        const int k = c * KC + e / BW, col = n0 + e % BW;
        bv[i] = k < K && col < N;
        bo[i] = bofs[bv[i] ? k * N + col : 0];
      }
    };
    auto load_kmeta = [&](int c, int32_t &ko, int32_t (&pk)[NA]) {
      const int k = c * KC + lane;
      const bool v = lane < KC && k < x.K;
      const int kk = v ? k : 0;
      ko = v ? (int32_t)x.kofs[kk] : -1;
#pragma unroll
      for (int a = 0; a < NA; ++a) pk[a] = x.kp[kk].p[a];
    };
    auto load_b = [&](const int32_t (&bo)[BR], const bool (&bv)[BR], In (&v)[BR]) {
#pragma unroll
      for (int i = 0; i < BR; ++i) v[i] = B.ld_z(bv[i] && bo[i] >= 0, bo[i]);
    };
    auto put_kmeta = [&](int buf, int32_t ko, const int32_t (&pk)[NA]) {
      if (lane < KC) {
        kls[w][buf][lane][0] = ko >= 0 ? ko * (int32_t)sizeof(In) : -1;
#pragma unroll
        for (int a = 0; a < NA; ++a) kls[w][buf][lane][1 + a] = pk[a] * (int32_t)sizeof(In);
      }
      wave_lds_sync();
    };
    auto load_a = [&](int c, int buf, In (&av)[KQ][RB]) {
      lds_load_chunk<In, RB, KQ, NA>(x.A, x.rt, x.nact, min(KC, K - c * KC), x.m0, x.nrows, lane, kls[w][buf], av);
    };
    auto put_b = [&](int buf, const In (&v)[BR]) {
#pragma unroll
      for (int i = 0; i < BR; ++i) {
        const int e = (int)threadIdx.x + 256 * i;
        if (e < BE) bl[buf][e / BW][e % BW] = Cmp(v[i]);
      }
    };
    const int cbn = (x.ncols + 15) >> 4;
    const int rbn = (x.nrows + 15) >> 4;
    acc_t acc[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};
    auto mfma_chunk = [&](int c, const In (&av)[KQ][RB]) {
      const int Kc = min(KC, K - c * KC);
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        if (4 * q < Kc) {
          Cmp b[CB];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) b[cb] = bl[c & 1][4 * q + kl][16 * cb + (lane & 15)];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (rb < rbn)
#pragma unroll
              for (int cb = 0; cb < CB; ++cb)
                if (cb < cbn) acc[rb][cb] = M::run(Cmp(av[q][rb]), b[cb], acc[rb][cb]);
        }
      }
    };
    // prologue: chunk 0's metadata, B values and A loads; chunk 1's offsets
    int32_t bo[BR];
    bool bv[BR];
    int32_t ko, pk[NA];
    In v[BR];
    In av0[KQ][RB], av1[KQ][RB];
    load_bofs(0, bo, bv);
    load_kmeta(0, ko, pk);
    load_b(bo, bv, v);
    put_kmeta(0, ko, pk);
    if (live) load_a(0, 0, av0);
    if (nk > 1) {
      load_bofs(1, bo, bv);
      load_kmeta(1, ko, pk);
    }
    put_b(0, v);
    __syncthreads();
    // chunk c: the loads of chunk c + 1 and the offsets of chunk c + 2 go out
    // before chunk c's MFMAs; chunk c + 1's B values then go to the other LDS
    // buffer (every wave finished chunk c - 1, which used it, before the
    // previous barrier) and the workgroup meets once
    auto step = [&](int c, const In (&acur)[KQ][RB], In (&anext)[KQ][RB]) {
      const int nb = (c + 1) & 1;
      if (c + 1 < nk) {
        load_b(bo, bv, v);
        put_kmeta(nb, ko, pk);
        if (live) load_a(c + 1, nb, anext);
        if (c + 2 < nk) {
          load_bofs(c + 2, bo, bv);
          load_kmeta(c + 2, ko, pk);
        }
      }
      if (live) mfma_chunk(c, acur);
      if (c + 1 < nk) put_b(nb, v);
      __syncthreads();  // chunk c + 1's B tile is in LDS; every wave is done with chunk c
    };
    for (int c = 0; c < nk; c += 2) {
      step(c, av0, av1);
      if (c + 1 < nk) step(c + 1, av1, av0);
    }
    if (live) {
      // stores without per-lane branches: padding rows and columns store
      // past the end of C (dropped) and add 0 to the norm
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= cbn) continue;
        const bool cv = cbase[cb] >= 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            const int lr = 16 * rb + M::row(lane, vv);
            const bool ok = cv && lr < x.nrows;
            const Out val = Out(acc[rb][cb][vv]);
            x.C.put_if(ok, cbase[cb] + (Off)__umul24((uint32_t)(x.m0 + lr), (uint32_t)cnj[cb]) + (Off)ccl[cb], val);
            if constexpr (NORM) nacc.add(ok ? (double)val : 0.0);
          }
        }
      }
      if constexpr (NORM) norm_file_tile(args.norm, tl, lane, nacc);
    }
    __syncthreads();  // the next job overwrites the B chunk and the k metadata
  }
}

// ---------------------------------------------------------------------------
// grouped gather GEMM for sectors of any K, software-pipelined over k
// ---------------------------------------------------------------------------
// Tiles start from the flat tile record (as k_gemm_res); B comes from the
// packed B_X in the workspace.  The k loop runs in batches of KB MFMA k-steps.
// The tile's k metadata (offset of (row 0, k), -1 where the row tuple has no
// A block, and the class factors) is staged in LDS once per tile (in segments
// of kPfSeg entries), so reading it never waits on the operand loads; the A
// and B loads of batch n + PD are issued before the MFMAs of batch n, from a
// ring of PD + 1 register buffers, with no load under a branch (reads past K,
// past the tile's rows or past N return 0 from past the end of the buffer).
constexpr int kPfSeg = 256;

template <typename In, typename Cmp, typename Out, bool BUF, int RB, int CB, int KB, int NA, int PD>
__global__ void __launch_bounds__(256) k_gemm_pf(LaunchArgs args) {
  static_assert(NA <= kRecAct + 1, "tile records carry kRecAct class boundaries");
  static_assert(BUF, "pipelined tiles address every operand through buffer resources");
  constexpr int R = PD + 1;
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  __shared__ int32_t meta_lds[4][kPfSeg * (1 + NA)];
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4;
  const int gw = blockIdx.x * 4 + uni(threadIdx.x >> 6);  // wave-uniform
  const int W = gridDim.x * 4;
  int32_t *const ml = meta_lds[threadIdx.x >> 6];  // this wave's slice
  const bool do_norm = args.norm.parts != nullptr;
  NormAcc nacc;
  for (int t = gw; t < args.ntiles; t += W) {
    RecCtx<In, Out, BUF> x;
    rec_setup<In, Out, BUF>(args, t, x);
    int jb = 0;
    while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
    // the sector's packed B_X (K x N, row-major) in the workspace
    Src<Cmp, true> Bq;
    Bq.init(reinterpret_cast<const Cmp *>(cst(&args.jobs[jb].ws)) + x.bpack, (int64_t)x.K * x.N);
    const int K = x.K, N = x.N, nact = x.nact, nrows = x.nrows;
    const int cbn = (x.ncols + 15) >> 4;
    int32_t cbase[CB], cnj[CB], ccl[CB];
    tile_columns<int32_t, CB>(x.cmap, x.cgrid, x.ncols, lane, cbase, cnj, ccl);
    // k metadata of k = s0 .. s0 + ks - 1 into LDS (lanes stride the entries;
    // every lane of the wave reads them after the wave-local fence)
    auto stage = [&](int s0, int ks) {
      for (int i = lane; i < ks; i += 64) {
        ml[i] = (int32_t)x.kofs[s0 + i];
#pragma unroll
        for (int a = 0; a < NA; ++a) ml[kPfSeg * (1 + a) + i] = x.kp[s0 + i].p[a];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const bool one_seg = K <= kPfSeg;
    if (one_seg) stage(0, K);
    for (int mc = 0; mc < nrows; mc += 16 * RB) {
      const int rows = min(16 * RB, nrows - mc);
      const int rbn = (rows + 15) >> 4;
      int32_t rg[RB][NA];
      bool rv[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int lr = 16 * rb + (lane & 15);
        rv[rb] = lr < rows;
        a_rowparts_fast<NA>(x.rt, nact, x.m0 + mc + (rv[rb] ? lr : 0), rg[rb]);
      }
      acc_t acc[RB][CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};
      for (int s0 = 0; s0 < K; s0 += kPfSeg) {
        const int ks = min(kPfSeg, K - s0);
        if (!one_seg) stage(s0, ks);
        const int nb = (ks + 4 * KB - 1) / (4 * KB);
        In ad[R][KB][RB];
        Cmp bd[R][KB][CB];
        // operands of batch n (k = s0 + 4 KB n + 4 q + kl)
        auto load = [&](int n, In (&av)[KB][RB], Cmp (&bv)[KB][CB]) {
#pragma unroll
          for (int q = 0; q < KB; ++q) {
            const int ki = 4 * KB * n + 4 * q + kl;  // index within the segment
            const bool kv = ki < ks;
            const int kc = kv ? ki : 0;
            const int32_t o = ml[kc];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              int32_t off = o;
#pragma unroll
              for (int a = 0; a < NA; ++a) off += ml[kPfSeg * (1 + a) + kc] * rg[rb][a];
              av[q][rb] = x.A.ld_z(kv && o >= 0 && rv[rb], off);
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int c = x.n0 + 16 * cb + (lane & 15);
              bv[q][cb] = Bq.ld_z(kv && c < N, (s0 + ki) * N + c);
            }
          }
        };
        auto mfma = [&](int n, const In (&av)[KB][RB], const Cmp (&bv)[KB][CB]) {
#pragma unroll
          for (int q = 0; q < KB; ++q)
            if (4 * KB * n + 4 * q < ks)
#pragma unroll
              for (int rb = 0; rb < RB; ++rb)
                if (rb < rbn)
#pragma unroll
                  for (int cb = 0; cb < CB; ++cb)
                    if (cb < cbn) acc[rb][cb] = M::run(Cmp(av[q][rb]), bv[q][cb], acc[rb][cb]);
        };
#pragma unroll
        for (int u = 0; u < PD; ++u) load(u, ad[u], bd[u]);
        int n = 0;
        for (; n + R <= nb; n += R) {
#pragma unroll
          for (int u = 0; u < R; ++u) {
            load(n + u + PD, ad[(u + PD) % R], bd[(u + PD) % R]);
            mfma(n + u, ad[u], bd[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
          if (n + u < nb) mfma(n + u, ad[u], bd[u]);
      }
      if (x.split) {
        // split-K tile: the accumulators, row r and column c of the tile at
        // r * 64 + c of its partial slot (summed into C by k_split_reduce)
        Cmp *pt = reinterpret_cast<Cmp *>(cst(&args.jobs[jb].ws) + x.part);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lr = 16 * rb + M::row(lane, v);
              if (lr < rows) pt[(mc + lr) * 64 + 16 * cb + (lane & 15)] = acc[rb][cb][v];
            }
        continue;
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (cb >= cbn) continue;
        const bool cv = cbase[cb] >= 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbn) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + M::row(lane, v);
            const bool ok = cv && lr < rows;
            const Out val = Out(acc[rb][cb][v]);
            x.C.put_if(ok, cbase[cb] + (x.m0 + mc + lr) * cnj[cb] + ccl[cb], val);
            if (do_norm) nacc.add(ok ? (double)val : 0.0);
          }
        }
      }
    }
    if (do_norm) norm_file_tile(args.norm, t, lane, nacc);
  }
}

// ---------------------------------------------------------------------------
// split-K reduction: the output tile of each group is the sum of its partial
// slots, taken in slot order (a fixed order, so results are reproducible),
// written into C's blocks through the column map as the GEMM epilogue does
// ---------------------------------------------------------------------------
template <typename Acc, typename Out>
__global__ void __launch_bounds__(256) k_split_reduce(RedArgs args) {
  for (int i = blockIdx.x; i < args.nitems; i += gridDim.x) {
    const DevRedItem &it = args.items[i];
    Out *C = reinterpret_cast<Out *>((args.ptab ? cst(args.ptab + (it.prob - args.plo)) : args.p[it.prob - args.plo]).c);
    const int n = it.nrows * 64;
    for (int e = threadIdx.x; e < n; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (c >= it.ncols) continue;
      const DevColMap cm = it.cmap[c];
      const int64_t base = it.cgrid[cm.j];
      if (base < 0) continue;
      // sixteen slots' loads in flight at a time, summed in slot order
      Acc sum = 0;
      const char *slot = args.ws + it.off0;
      int s = 0;
      for (; s + 16 <= it.nslots; s += 16, slot += 16 * (int64_t)it.slot_bytes) {
        Acc v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = reinterpret_cast<const Acc *>(slot + (int64_t)u * it.slot_bytes)[e];
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += v[u];
      }
      for (; s < it.nslots; ++s, slot += it.slot_bytes) sum += reinterpret_cast<const Acc *>(slot)[e];
      C[base + (int64_t)(it.m0 + r) * cm.nj + cm.cl] = Out(sum);
    }
  }
}

}  // namespace yastn
