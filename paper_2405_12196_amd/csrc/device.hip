// HIP kernels (gfx950 / CDNA4) and the C ABI of the block-sparse tensordot.
//
//  k_join_*   charge-hash join: B blocks are inserted into an open-addressing
//             table keyed by their contracted charges; every A block probes it
//             and emits its matches (count, scan, emit).  Two blocks meet iff
//             their charges agree on every contracted leg pair (paper Sec.
//             II.B: contracted legs carry the same charges on both partners).
//  k_pack_b   fuses B's legs into the per-sector matrices B_X (K_X x N_X,
//             row-major; absent sub-blocks zero) -- the "fuse" step of the
//             fuse -> multiply -> unfuse contraction of Sec. II.B, applied to
//             the small operand only.
//  k_gemm     grouped GEMM C_X = A_X B_X over every sector of every problem
//             in one launch.  One wave owns a tile of up to 64 rows of one A
//             free tuple x up to 64 columns of B_X.  A is never materialised:
//             each element is gathered from its block through the factorised
//             offsets of plan.hpp (the leg permute is fused into the load).
//             The epilogue writes each element straight into its output block
//             (the "unfuse" step), exactly once: C need not be zeroed and no
//             atomics are used, so results are deterministic.
//  k_norm_*   FP64 Frobenius norm and max |x|, two fixed-order passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <type_traits>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "index.hpp"
#include "planner.hpp"

namespace yastn {

const char *last_error_cstr();

#define YASTN_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return set_error(YASTN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

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
  d.ntiles = cst(&p->ntiles);
  d.nitems = cst(&p->nitems);
  return d;
}

// LDS written by one lane and read by another lane of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// charge-hash join
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t key_hash(const int32_t *k, int len) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  for (int i = 0; i < len; ++i) {
    h ^= (uint64_t)(uint32_t)k[i] + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h *= 0xFF51AFD7ED558CCDull;
  }
  return h ^ (h >> 33);
}

__device__ __forceinline__ bool key_eq(const int32_t *a, const int32_t *b, int len) {
  for (int i = 0; i < len; ++i)
    if (a[i] != b[i]) return false;
  return true;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_join_build(const int32_t *keyb, int64_t nb, int klen, int32_t *owner, int32_t *head,
                             int32_t *next, uint64_t mask) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const int32_t *kj = keyb + j * klen;
  uint64_t h = key_hash(kj, klen) & mask;
  for (;;) {
    int32_t o = atomicCAS(&owner[h], -1, (int32_t)j);
    if (o == -1 || key_eq(keyb + (int64_t)o * klen, kj, klen)) {
      next[j] = atomicExch(&head[h], (int32_t)j);
      return;
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int64_t probe_slot(const int32_t *ki, const int32_t *keyb, int klen,
                                              const int32_t *owner, uint64_t mask) {
  uint64_t h = key_hash(ki, klen) & mask;
  for (;;) {
    int32_t o = owner[h];
    if (o < 0) return -1;
    if (key_eq(keyb + (int64_t)o * klen, ki, klen)) return (int64_t)h;
    h = (h + 1) & mask;
  }
}

__global__ void k_join_count(const int32_t *keya, int64_t na, const int32_t *keyb, int klen, const int32_t *owner,
                             const int32_t *head, const int32_t *next, uint64_t mask, int64_t *cnt) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= na) return;
  int64_t slot = probe_slot(keya + i * klen, keyb, klen, owner, mask);
  int64_t c = 0;
  if (slot >= 0)
    for (int32_t j = head[slot]; j >= 0; j = next[j]) ++c;
  cnt[i] = c;
}

// exclusive scan of n counts by one workgroup of 1024 threads; out[n] = total
__global__ void __launch_bounds__(1024) k_scan_one(const int64_t *cnt, int64_t n, int64_t *out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b0 = std::min<int64_t>(n, t * per), b1 = std::min<int64_t>(n, b0 + per);
  int64_t s = 0;
  for (int64_t i = b0; i < b1; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b0; i < b1; ++i) {
    out[i] = run;
    run += cnt[i];
  }
  if (t == 1023) out[n] = part[1023];
}

__global__ void k_join_emit(const int32_t *keya, int64_t na, const int32_t *keyb, int klen, const int32_t *owner,
                            const int32_t *head, const int32_t *next, uint64_t mask, const int64_t *off,
                            int32_t *pa, int32_t *pb) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= na) return;
  int64_t slot = probe_slot(keya + i * klen, keyb, klen, owner, mask);
  if (slot < 0) return;
  int64_t p = off[i];
  for (int32_t j = head[slot]; j >= 0; j = next[j]) {
    pa[p] = (int32_t)i;
    pb[p] = j;
    ++p;
  }
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
// One workgroup per item of up to 256 elements of one (s, j) sub-block;
// consecutive threads write consecutive elements of a B_X row.
template <typename In, typename Cmp>
__global__ void __launch_bounds__(256) k_pack_b(LaunchArgs args) {
  for (int g = blockIdx.x; g < args.nitems; g += gridDim.x) {
    int jb = 0;
    while (jb + 1 < args.njobs && g >= args.jobs[jb + 1].item0) ++jb;
    const JobArg &job = args.jobs[jb];
    const DevPlan P = load_plan(job.plan);
    const DevPackItem it = cst(P.items + (g - job.item0 + job.pitem0));
    const DevSector sec = cst(P.sectors + it.sector);
    const DevCtrTuple ct = cst(P.ctrs + (sec.ctr0 + it.s));
    const DevColTuple cl = cst(P.cols + (sec.col0 + it.j));
    const int32_t e = it.e0 + (int32_t)threadIdx.x;
    if (e >= ct.k * cl.n) continue;
    const int32_t kd = e / cl.n, cb = e - kd * cl.n;
    Cmp *dst = reinterpret_cast<Cmp *>(job.ws) + sec.bpack + (int64_t)(ct.ko + kd) * sec.N + cl.no + cb;
    if (it.bblk < 0) {
      *dst = Cmp(0);
    } else {
      const In *src = reinterpret_cast<const In *>(args.p[job.prob0 + sec.prob - job.plo].b);
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

template <typename T> struct BufIo;
template <> struct BufIo<double> {
  __device__ static double ld(__amdgpu_buffer_rsrc_t r, int32_t byte) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, int32_t byte, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), r, byte, 0, 0);
  }
};
template <> struct BufIo<float> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, int32_t byte) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, int32_t byte, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte, 0, 0);
  }
};

template <typename T, bool BUF> struct Src;
template <typename T> struct Src<T, true> {
  __amdgpu_buffer_rsrc_t r;
  __device__ void init(const void *p, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc(uniptr(const_cast<void *>(p)), (short)0, uni((int)(n * (int64_t)sizeof(T))),
                                          kBufFlags);
  }
  __device__ T operator()(int32_t i) const { return BufIo<T>::ld(r, i * (int32_t)sizeof(T)); }
};
template <typename T> struct Src<T, false> {
  const T *__restrict__ p;
  __device__ void init(const void *q, int64_t) { p = reinterpret_cast<const T *>(q); }
  __device__ T operator()(int64_t i) const { return p[i]; }
};
template <typename T, bool BUF> struct Dst;
template <typename T> struct Dst<T, true> {
  __amdgpu_buffer_rsrc_t r;
  __device__ void init(void *p, int64_t n) {
    r = __builtin_amdgcn_make_buffer_rsrc(uniptr(p), (short)0, uni((int)(n * (int64_t)sizeof(T))), kBufFlags);
  }
  __device__ void put(int64_t i, T v) const { BufIo<T>::st(r, (int32_t)i * (int32_t)sizeof(T), v); }
};
template <typename T> struct Dst<T, false> {
  T *__restrict__ p;
  __device__ void init(void *q, int64_t) { p = reinterpret_cast<T *>(q); }
  __device__ void put(int64_t i, T v) const { p[i] = v; }
};

// Tile context shared by every precision: the tile's row tuple and sector,
// the problem's operands, and the lane's output columns.
template <typename In, typename Out, bool BUF, int CB> struct TileCtx {
  DevTile tile;
  DevRowTuple rt;
  DevSector sec;
  Src<In, BUF> A;
  Dst<Out, BUF> C;
  const char *ws;
  int64_t cbase[CB];        // output block offset of the lane's columns (-1: none)
  int32_t cnj[CB], ccl[CB];
  int cbn;
};

template <typename In, typename Out, bool BUF, int CB>
__device__ __forceinline__ DevPlan tile_setup(const LaunchArgs &args, int t, int lane, TileCtx<In, Out, BUF, CB> &x) {
  int jb = 0;
  while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
  const JobArg &job = args.jobs[jb];
  const DevPlan P = load_plan(job.plan);
  x.tile = cst(P.tiles + (t - job.tile0 + job.ptile0));
  x.rt = cst(P.rows + x.tile.rowtuple);
  x.sec = cst(P.sectors + x.tile.sector);
  const ProbPtrs pp = args.p[job.prob0 + x.sec.prob - job.plo];
  const DevProb pr = cst(P.probs + x.sec.prob);
  x.A.init(pp.a, pr.a_span);
  x.C.init(pp.c, pr.c_numel);
  x.ws = job.ws;
  x.cbn = (x.tile.ncols + 15) >> 4;
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

// ---------------------------------------------------------------------------
// FP64 norm: Frobenius and max |x|
// ---------------------------------------------------------------------------
constexpr int kNormBlocks = 512;

template <typename T>
__global__ void __launch_bounds__(256) k_norm_partial(const T *x, int64_t n, double *part) {
  __shared__ double ss[256], sm[256];
  double s = 0.0, m = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double v = (double)x[i];
    s = fma(v, v, s);
    m = fmax(m, fabs(v));
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ss[0];
    part[2 * blockIdx.x + 1] = sm[0];
  }
}

__global__ void __launch_bounds__(256) k_norm_final(const double *part, int np, double *out) {
  __shared__ double ss[256], sm[256];
  double s = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    s += part[2 * i];
    m = fmax(m, part[2 * i + 1]);
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(ss[0]);
    out[1] = sm[0];
  }
}

// ---------------------------------------------------------------------------
// host: join driver
// ---------------------------------------------------------------------------
namespace {

template <typename T> yastn_status dmalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? YASTN_ERR_NOMEM : YASTN_ERR_HIP,
                     std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return YASTN_OK;
}

struct DevBufs {  // frees whatever it holds
  std::vector<void *> ptrs;
  ~DevBufs() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <typename T> yastn_status alloc(T **p, size_t count) {
    yastn_status s = dmalloc(p, count);
    if (s == YASTN_OK) ptrs.push_back(*p);
    return s;
  }
};

unsigned grid_for(int64_t n, int block) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 65535)); }

yastn_status gpu_join(const HostProblem &hp, hipStream_t st, std::vector<std::pair<int32_t, int32_t>> &pairs) {
  pairs.clear();
  const int64_t na = hp.a.nblocks, nb = hp.b.nblocks;
  if (na == 0 || nb == 0) return YASTN_OK;
  const int klen = hp.nc * hp.a.nsym;
  std::vector<int32_t> ka, kb;
  contracted_keys(hp.a, hp.axes_a, hp.nc, ka);
  contracted_keys(hp.b, hp.axes_b, hp.nc, kb);
  uint64_t tsize = 64;
  while (tsize < 2 * (uint64_t)nb) tsize <<= 1;
  DevBufs bufs;
  int32_t *d_ka, *d_kb, *owner, *head, *next;
  int64_t *cnt, *off;
  yastn_status s;
  if ((s = bufs.alloc(&d_ka, ka.size())) || (s = bufs.alloc(&d_kb, kb.size())) || (s = bufs.alloc(&owner, tsize)) ||
      (s = bufs.alloc(&head, tsize)) || (s = bufs.alloc(&next, nb)) || (s = bufs.alloc(&cnt, na)) ||
      (s = bufs.alloc(&off, na + 1)))
    return s;
  if (!ka.empty()) YASTN_HIP(hipMemcpyAsync(d_ka, ka.data(), ka.size() * 4, hipMemcpyHostToDevice, st));
  if (!kb.empty()) YASTN_HIP(hipMemcpyAsync(d_kb, kb.data(), kb.size() * 4, hipMemcpyHostToDevice, st));
  k_fill_i32<<<grid_for(tsize, 256), 256, 0, st>>>(owner, tsize, -1);
  k_fill_i32<<<grid_for(tsize, 256), 256, 0, st>>>(head, tsize, -1);
  k_join_build<<<grid_for(nb, 256), 256, 0, st>>>(d_kb, nb, klen, owner, head, next, tsize - 1);
  k_join_count<<<grid_for(na, 256), 256, 0, st>>>(d_ka, na, d_kb, klen, owner, head, next, tsize - 1, cnt);
  k_scan_one<<<1, 1024, 0, st>>>(cnt, na, off);
  YASTN_HIP(hipGetLastError());
  int64_t total = 0;
  YASTN_HIP(hipMemcpyAsync(&total, off + na, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  YASTN_HIP(hipStreamSynchronize(st));
  if (total == 0) return YASTN_OK;
  int32_t *pa, *pb;
  if ((s = bufs.alloc(&pa, total)) || (s = bufs.alloc(&pb, total))) return s;
  k_join_emit<<<grid_for(na, 256), 256, 0, st>>>(d_ka, na, d_kb, klen, owner, head, next, tsize - 1, off, pa, pb);
  YASTN_HIP(hipGetLastError());
  std::vector<int32_t> ha(total), hb(total);
  YASTN_HIP(hipMemcpyAsync(ha.data(), pa, total * 4, hipMemcpyDeviceToHost, st));
  YASTN_HIP(hipMemcpyAsync(hb.data(), pb, total * 4, hipMemcpyDeviceToHost, st));
  YASTN_HIP(hipStreamSynchronize(st));
  pairs.resize(total);
  for (int64_t i = 0; i < total; ++i) pairs[i] = {ha[i], hb[i]};
  return YASTN_OK;
}

template <typename T> size_t bytes_of(const std::vector<T> &v) { return v.size() * sizeof(T); }

yastn_status upload(Plan &pl) {
  PlanTables &t = pl.t;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  size_t o_probs = take(bytes_of(t.probs)), o_sec = take(bytes_of(t.sectors)), o_rows = take(bytes_of(t.rows)),
         o_ctrs = take(bytes_of(t.ctrs)), o_cols = take(bytes_of(t.cols)), o_agrid = take(bytes_of(t.agrid)),
         o_aoff = take(bytes_of(t.aoff)), o_cgrid = take(bytes_of(t.cgrid)), o_bb = take(bytes_of(t.bblocks)),
         o_tiles = take(bytes_of(t.tiles)), o_items = take(bytes_of(t.items)), o_kofs = take(bytes_of(t.kofs)),
         o_kp = take(bytes_of(t.kp)), o_cm = take(bytes_of(t.colmap)), o_plan = take(sizeof(DevPlan));
  char *base;
  yastn_status s = dmalloc(&base, off);
  if (s) return s;
  pl.dev_mem = base;
  std::vector<char> host(off, 0);
  auto put = [&](size_t o, const void *src, size_t b) {
    if (b) std::memcpy(host.data() + o, src, b);
  };
  put(o_probs, t.probs.data(), bytes_of(t.probs));
  put(o_sec, t.sectors.data(), bytes_of(t.sectors));
  put(o_rows, t.rows.data(), bytes_of(t.rows));
  put(o_ctrs, t.ctrs.data(), bytes_of(t.ctrs));
  put(o_cols, t.cols.data(), bytes_of(t.cols));
  put(o_agrid, t.agrid.data(), bytes_of(t.agrid));
  put(o_aoff, t.aoff.data(), bytes_of(t.aoff));
  put(o_cgrid, t.cgrid.data(), bytes_of(t.cgrid));
  put(o_bb, t.bblocks.data(), bytes_of(t.bblocks));
  put(o_tiles, t.tiles.data(), bytes_of(t.tiles));
  put(o_items, t.items.data(), bytes_of(t.items));
  put(o_kofs, t.kofs.data(), bytes_of(t.kofs));
  put(o_kp, t.kp.data(), bytes_of(t.kp));
  put(o_cm, t.colmap.data(), bytes_of(t.colmap));
  DevPlan dp{};
  dp.probs = reinterpret_cast<const DevProb *>(base + o_probs);
  dp.sectors = reinterpret_cast<const DevSector *>(base + o_sec);
  dp.rows = reinterpret_cast<const DevRowTuple *>(base + o_rows);
  dp.ctrs = reinterpret_cast<const DevCtrTuple *>(base + o_ctrs);
  dp.cols = reinterpret_cast<const DevColTuple *>(base + o_cols);
  dp.agrid = reinterpret_cast<const int32_t *>(base + o_agrid);
  dp.aoff = reinterpret_cast<const int64_t *>(base + o_aoff);
  dp.cgrid = reinterpret_cast<const int64_t *>(base + o_cgrid);
  dp.bblocks = reinterpret_cast<const DevBBlock *>(base + o_bb);
  dp.tiles = reinterpret_cast<const DevTile *>(base + o_tiles);
  dp.items = reinterpret_cast<const DevPackItem *>(base + o_items);
  dp.kofs = reinterpret_cast<const int64_t *>(base + o_kofs);
  dp.kp = reinterpret_cast<const DevKP *>(base + o_kp);
  dp.colmap = reinterpret_cast<const DevColMap *>(base + o_cm);
  dp.ntiles = (int32_t)t.tiles.size();
  dp.nitems = (int32_t)t.items.size();
  put(o_plan, &dp, sizeof(dp));
  pl.dplan = reinterpret_cast<DevPlan *>(base + o_plan);
  YASTN_HIP(hipMemcpy(base, host.data(), off, hipMemcpyHostToDevice));
  return YASTN_OK;
}

// ---- kernel dispatch -------------------------------------------------------
// Kernel variants of one plan: 0 = the plan's heuristic choice; 1..kVariants-1
// = MFMA tiles with (rows per chunk, k-steps per load batch) from kMfmaShapes,
// or the row-per-lane kernel.  yastn_plan_autotune times the candidates.
// RB only tunes speed (a tile of any height is walked in chunks); CB must
// cover the plan's tile width.  Without buffer addressing (buffers of 2 GiB
// or more) one general MFMA shape is compiled.
typedef void (*KernelFn)(LaunchArgs);

struct Shape {
  int rb, kb;
};
constexpr Shape kMfmaShapes[] = {{4, 2}, {4, 1}, {4, 4}, {2, 2}, {2, 4}, {1, 4}};
constexpr int kNumMfma = sizeof(kMfmaShapes) / sizeof(Shape);
constexpr int kVariantRows = kNumMfma + 1;  // variant ids: 1..kNumMfma MFMA, kVariantRows rows
constexpr int kVariants = kVariantRows + 1;
static_assert(kVariants == YASTN_NUM_VARIANTS, "variant count must match the header");

template <typename In, typename Cmp, typename Out, int RB, int KB>
KernelFn pick_mfma_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm4<In, Cmp, Out, true, RB, 1, KB>;
    case 2: return k_gemm4<In, Cmp, Out, true, RB, 2, KB>;
    case 3: return k_gemm4<In, Cmp, Out, true, RB, 3, KB>;
    default: return k_gemm4<In, Cmp, Out, true, RB, 4, KB>;
  }
}
template <typename In, typename Cmp, typename Out>
KernelFn pick_gemm4(bool buf, int shape, int cb) {
  if (!buf) return k_gemm4<In, Cmp, Out, false, 4, 4, 2>;
  if (std::is_same<Cmp, double>::value) {
    switch (shape) {
      case 1: return pick_mfma_cb<In, Cmp, Out, 4, 1>(cb);
      case 2: return pick_mfma_cb<In, Cmp, Out, 4, 4>(cb);
      case 3: return pick_mfma_cb<In, Cmp, Out, 2, 2>(cb);
      case 4: return pick_mfma_cb<In, Cmp, Out, 2, 4>(cb);
      case 5: return pick_mfma_cb<In, Cmp, Out, 1, 4>(cb);
      default: break;
    }
  } else if (shape == 3 || shape == 4 || shape == 5) {
    return pick_mfma_cb<In, Cmp, Out, 2, 4>(cb);
  }
  return pick_mfma_cb<In, Cmp, Out, 4, 2>(cb);
}
template <typename In, typename Out, int NT>
KernelFn pick_bf16(bool buf, int cb) {
  if (!buf) return k_gemm_bf16<In, Out, false, 4, 4, NT>;
  switch (cb) {
    case 1: return k_gemm_bf16<In, Out, true, 4, 1, NT>;
    case 2: return k_gemm_bf16<In, Out, true, 4, 2, NT>;
    case 3: return k_gemm_bf16<In, Out, true, 4, 3, NT>;
    default: return k_gemm_bf16<In, Out, true, 4, 4, NT>;
  }
}
template <typename In, typename Out>
KernelFn pick_gemm(yastn_precision p, bool buf, int shape, int cb) {
  switch (p) {
    case YASTN_F32: return pick_gemm4<In, float, Out>(buf, shape, cb);
    case YASTN_BF16X3: return pick_bf16<In, Out, 3>(buf, cb);
    default: return pick_bf16<In, Out, 6>(buf, cb);
  }
}
KernelFn gemm_kernel(const yastn_options &o, bool buf, int shape, int cb) {
  if (o.in_dtype == YASTN_DTYPE_F64) {
    if (o.precision == YASTN_F64) return pick_gemm4<double, double, double>(buf, shape, cb);
    return o.out_dtype == YASTN_DTYPE_F64 ? pick_gemm<double, double>(o.precision, buf, shape, cb)
                                          : pick_gemm<double, float>(o.precision, buf, shape, cb);
  }
  return o.out_dtype == YASTN_DTYPE_F64 ? pick_gemm<float, double>(o.precision, buf, shape, cb)
                                        : pick_gemm<float, float>(o.precision, buf, shape, cb);
}
template <typename In, typename Cmp, typename Out>
KernelFn pick_rows(bool buf, int kmax) {
  if (!buf) return k_rows<In, Cmp, Out, false, 64>;
  if (kmax <= 16) return k_rows<In, Cmp, Out, true, 16>;
  if (kmax <= 32) return k_rows<In, Cmp, Out, true, 32>;
  if (kmax <= 48) return k_rows<In, Cmp, Out, true, 48>;
  return k_rows<In, Cmp, Out, true, 64>;
}
KernelFn rows_kernel(const yastn_options &o, bool buf, int kmax) {
  if (o.in_dtype == YASTN_DTYPE_F64) {
    if (o.precision == YASTN_F64) return pick_rows<double, double, double>(buf, kmax);
    return o.out_dtype == YASTN_DTYPE_F64 ? pick_rows<double, float, double>(buf, kmax)
                                          : pick_rows<double, float, float>(buf, kmax);
  }
  return o.out_dtype == YASTN_DTYPE_F64 ? pick_rows<float, float, double>(buf, kmax)
                                        : pick_rows<float, float, float>(buf, kmax);
}

KernelFn pack_kernel(const yastn_options &o) {
  const bool f64cmp = o.precision == YASTN_F64;
  if (o.in_dtype == YASTN_DTYPE_F64) return f64cmp ? k_pack_b<double, double> : k_pack_b<double, float>;
  return k_pack_b<float, float>;
}

int g_num_cu = 0;
std::once_flag g_cu_once;
int num_cus() {
  std::call_once(g_cu_once, [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      g_num_cu = n;
    if (g_num_cu <= 0) g_num_cu = 256;
  });
  return g_num_cu;
}

struct JobRef {
  const Plan *plan;
  const Group *g;
  const void *const *a;
  const void *const *b;
  void *const *c;
  void *ws;
};

yastn_status launch(const std::vector<JobRef> &jobs, hipStream_t st, void *const *events = nullptr) {
  if (events && events[0]) YASTN_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(events[0]), st));
  if (jobs.empty()) {
    if (events && events[1]) YASTN_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(events[1]), st));
    if (events && events[2]) YASTN_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(events[2]), st));
    return YASTN_OK;
  }
  const yastn_options &o = jobs[0].plan->opts;
  int cb = 1, kmax = 0, variant = jobs[0].plan->variant;
  bool buf = true, rows_fit = true, rows_pick = true;
  for (auto &j : jobs) {
    cb = std::max(cb, j.plan->cb);
    kmax = std::max(kmax, j.plan->kmax);
    buf = buf && j.plan->buf_ok;
    rows_fit = rows_fit && j.plan->rows_fit;
    rows_pick = rows_pick && j.plan->rows_kernel;
    if (j.plan->variant != variant) variant = 0;
  }
  bool rows = variant == 0 ? rows_pick : (variant == kVariantRows && rows_fit);
  const int shape = (variant >= 1 && variant <= kNumMfma) ? variant - 1 : 0;
  KernelFn gemm = rows ? rows_kernel(o, buf, kmax) : gemm_kernel(o, buf, shape, cb), pack = pack_kernel(o);
  size_t ji = 0;
  while (ji < jobs.size()) {
    LaunchArgs la;
    std::memset(&la, 0, sizeof(la));
    int np = 0;
    while (ji < jobs.size() && la.njobs < kMaxJobs) {
      const JobRef &j = jobs[ji];
      const int n = j.g->phi - j.g->plo;
      if (np + n > kMaxProbs) break;
      JobArg &ja = la.jobs[la.njobs++];
      ja.plan = j.plan->dplan;
      ja.ws = reinterpret_cast<char *>(j.ws);
      ja.tile0 = la.ntiles;
      ja.item0 = la.nitems;
      ja.ptile0 = j.g->t0;
      ja.pitem0 = j.g->i0;
      ja.prob0 = np;
      ja.plo = j.g->plo;
      for (int p = j.g->plo; p < j.g->phi; ++p) {
        la.p[np].a = j.a[p];
        la.p[np].b = j.b[p];
        la.p[np].c = j.c[p];
        ++np;
      }
      la.ntiles += j.g->t1 - j.g->t0;
      la.nitems += j.g->i1 - j.g->i0;
      ++ji;
    }
    const int max_wg = num_cus() * 4;
    void *kargs[] = {&la};
    if (la.nitems > 0) {
      unsigned g = (unsigned)std::min<int64_t>(la.nitems, 16 * max_wg);
      YASTN_HIP(hipLaunchKernel(reinterpret_cast<const void *>(pack), dim3(g), dim3(256), kargs, 0, st));
    }
    if (events && events[1]) YASTN_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(events[1]), st));
    if (la.ntiles > 0) {
      unsigned g = (unsigned)std::min<int64_t>((la.ntiles + 3) / 4, max_wg);
      YASTN_HIP(hipLaunchKernel(reinterpret_cast<const void *>(gemm), dim3(g), dim3(256), kargs, 0, st));
    }
    if (events && events[2]) YASTN_HIP(hipEventRecord(reinterpret_cast<hipEvent_t>(events[2]), st));
  }
  return YASTN_OK;
}

yastn_status check_job_ptrs(const Plan *pl, const void *const *a, const void *const *b, void *const *c, void *ws) {
  const int np = (int)pl->probs.size();
  if (np > 0 && (!a || !b || !c)) return set_error(YASTN_ERR_ARG, "null buffer array");
  for (int p = 0; p < np; ++p) {
    const HostProblem &hp = pl->probs[p];
    if (hp.c_numel > 0 && (!a[p] || !b[p] || !c[p])) return set_error(YASTN_ERR_ARG, "null device buffer");
  }
  if (pl->ws_bytes > 0 && !ws) return set_error(YASTN_ERR_ARG, "null workspace");
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255u)) return set_error(YASTN_ERR_ARG, "workspace must be 256-byte aligned");
  return YASTN_OK;
}

}  // namespace
}  // namespace yastn

// ===========================================================================
// C ABI
// ===========================================================================
using namespace yastn;

struct yastn_plan_s {
  Plan p;
};

extern "C" {

int32_t yastn_abi_version(void) { return YASTN_ABI_VERSION; }

const char *yastn_last_error(void) { return last_error_cstr(); }

const char *yastn_status_string(yastn_status s) {
  switch (s) {
    case YASTN_OK: return "YASTN_OK";
    case YASTN_ERR_ARG: return "YASTN_ERR_ARG";
    case YASTN_ERR_SYM: return "YASTN_ERR_SYM";
    case YASTN_ERR_CHARGE: return "YASTN_ERR_CHARGE";
    case YASTN_ERR_SIGNATURE: return "YASTN_ERR_SIGNATURE";
    case YASTN_ERR_SHAPE: return "YASTN_ERR_SHAPE";
    case YASTN_ERR_DUPLICATE: return "YASTN_ERR_DUPLICATE";
    case YASTN_ERR_NOMEM: return "YASTN_ERR_NOMEM";
    case YASTN_ERR_HIP: return "YASTN_ERR_HIP";
    case YASTN_ERR_STATE: return "YASTN_ERR_STATE";
  }
  return "unknown status";
}

yastn_status yastn_plan(const yastn_problem *probs, int32_t nprob, const yastn_options *opts, void *hip_stream,
                        yastn_plan_t *out) {
  if (!out) return set_error(YASTN_ERR_ARG, "null plan output");
  *out = nullptr;
  if (nprob < 0 || (nprob > 0 && !probs)) return set_error(YASTN_ERR_ARG, "bad problem array");
  yastn_options o;
  yastn_status s = check_options(opts, &o);
  if (s) return s;
  yastn_plan_s *h = new (std::nothrow) yastn_plan_s();
  if (!h) return set_error(YASTN_ERR_NOMEM, "host allocation");
  Plan &pl = h->p;
  pl.opts = o;
  try {
    pl.probs.resize(nprob);
    for (int p = 0; p < nprob; ++p)
      if ((s = validate_problem(probs[p], pl.probs[p])) != YASTN_OK) {
        delete h;
        return s;
      }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&pl.device) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return set_error(YASTN_ERR_HIP, "no HIP device");
    }
    std::vector<std::vector<std::pair<int32_t, int32_t>>> allpairs(nprob);
    for (int p = 0; p < nprob; ++p)
      if ((s = gpu_join(pl.probs[p], st, allpairs[p])) != YASTN_OK) {
        delete h;
        return s;
      }
    // Pass 0 builds 64 x 64 tiles to learn the sector shapes; then the plan
    // picks the kernel family and, for MFMA, the tile width, and rebuilds if
    // the tiling changed.
    int64_t a_base = 0, b_base = 0;
    auto build_all = [&](int rb, int cb, int nch) -> yastn_status {
      pl.t = PlanTables{};
      pl.prob_t0.clear();
      pl.prob_i0.clear();
      a_base = b_base = 0;
      pl.rb = rb;
      pl.cb = cb;
      pl.nch = nch;
      for (int p = 0; p < nprob; ++p) {
        pl.prob_t0.push_back((int32_t)pl.t.tiles.size());
        pl.prob_i0.push_back((int32_t)pl.t.items.size());
        yastn_status st2 = build_structure(pl.probs[p], p, allpairs[p], a_base, b_base, pl.t, rb, cb, nch);
        if (st2 != YASTN_OK) return st2;
        a_base += pl.probs[p].a.nblocks;
        b_base += pl.probs[p].b.nblocks;
      }
      return YASTN_OK;
    };
    if ((s = build_all(4, 4, 1)) != YASTN_OK) {
      delete h;
      return s;
    }
    int64_t maxn = 1, maxk = 0, rows = 0, rows64 = 0;
    for (auto &sec : pl.t.sectors) {
      maxn = std::max<int64_t>(maxn, sec.N);
      maxk = std::max<int64_t>(maxk, sec.K);
    }
    for (auto &rt : pl.t.rows) {
      rows += rt.m;
      rows64 += (rt.m + 63) / 64 * 64;
    }
    pl.kmax = (int)maxk;
    const bool bf16 = o.precision == YASTN_BF16X3 || o.precision == YASTN_BF16X6;
    pl.rows_fit = !bf16 && maxk <= 64 && maxn <= 64;
    pl.rows_kernel = pl.rows_fit && o.flags == YASTN_FLAG_ROWS;
    pl.variant = 0;
    // tiles: 64 rows (walked in chunks by every kernel) x the narrowest column
    // width that covers the widest sector (at most 64)
    const int cb = (int)std::min<int64_t>(4, (maxn + 15) / 16);
    if (cb != 4 && (s = build_all(4, cb, 1)) != YASTN_OK) {
      delete h;
      return s;
    }
    if (o.tile_rows) pl.variant = o.tile_rows == 64 ? 1 : (o.tile_rows == 32 ? 4 : 6);
    (void)rows;
    (void)rows64;
    if (a_base > INT32_MAX || b_base > INT32_MAX) {
      delete h;
      return set_error(YASTN_ERR_ARG, "too many blocks in one plan");
    }
    finish_tiles(pl);
    // buffer addressing needs every A span and C size below 2 GiB
    const int64_t in_b = o.in_dtype == YASTN_DTYPE_F64 ? 8 : 4, out_b = o.out_dtype == YASTN_DTYPE_F64 ? 8 : 4;
    pl.buf_ok = true;
    for (const DevProb &dp : pl.t.probs)
      if (dp.a_span * in_b >= (int64_t(1) << 31) || dp.c_numel * out_b >= (int64_t(1) << 31)) pl.buf_ok = false;
    if ((s = upload(pl)) != YASTN_OK) {
      yastn_free(h);
      return s;
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_plan_output(yastn_plan_t plan, int32_t prob, yastn_tensor_desc *c, int64_t *c_numel) {
  if (!plan || !c) return set_error(YASTN_ERR_ARG, "null argument");
  if (prob < 0 || prob >= (int32_t)plan->p.probs.size()) return set_error(YASTN_ERR_ARG, "problem index out of range");
  HostProblem &hp = plan->p.probs[prob];
  c->rank = hp.c_rank;
  c->nsym = hp.a.nsym;
  c->sym_mod = hp.a.sym_mod;
  c->sig = hp.c_sig;
  c->n = hp.c_n;
  c->nblocks = (int64_t)hp.c_offsets.size();
  c->charges = hp.c_charges.data();
  c->shapes = hp.c_shapes.data();
  c->offsets = hp.c_offsets.data();
  if (c_numel) *c_numel = hp.c_numel;
  return YASTN_OK;
}

yastn_status yastn_plan_workspace(yastn_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return set_error(YASTN_ERR_ARG, "null argument");
  *bytes = plan->p.ws_bytes;
  return YASTN_OK;
}

yastn_status yastn_plan_stats(yastn_plan_t plan, int32_t prob, yastn_stats *st) {
  if (!plan || !st) return set_error(YASTN_ERR_ARG, "null argument");
  if (prob < 0 || prob >= (int32_t)plan->p.probs.size()) return set_error(YASTN_ERR_ARG, "problem index out of range");
  *st = plan->p.probs[prob].stats;
  return YASTN_OK;
}

yastn_status yastn_contract(yastn_plan_t plan, const void *const *a, const void *const *b, void *const *c,
                            void *workspace, void *hip_stream) {
  if (!plan) return set_error(YASTN_ERR_ARG, "null plan");
  yastn_status s = check_job_ptrs(&plan->p, a, b, c, workspace);
  if (s) return s;
  std::vector<JobRef> jobs;
  for (const Group &g : plan->p.groups) jobs.push_back(JobRef{&plan->p, &g, a, b, c, workspace});
  return launch(jobs, reinterpret_cast<hipStream_t>(hip_stream));
}

yastn_status yastn_contract_timed(yastn_plan_t plan, const void *const *a, const void *const *b, void *const *c,
                                  void *workspace, void *hip_stream, void *const *events) {
  if (!plan) return set_error(YASTN_ERR_ARG, "null plan");
  if (plan->p.groups.size() > 1) return set_error(YASTN_ERR_STATE, "timed contraction needs a plan of one launch");
  yastn_status s = check_job_ptrs(&plan->p, a, b, c, workspace);
  if (s) return s;
  std::vector<JobRef> jobs;
  for (const Group &g : plan->p.groups) jobs.push_back(JobRef{&plan->p, &g, a, b, c, workspace});
  return launch(jobs, reinterpret_cast<hipStream_t>(hip_stream), events);
}

yastn_status yastn_plan_set_variant(yastn_plan_t plan, int32_t variant) {
  if (!plan) return set_error(YASTN_ERR_ARG, "null plan");
  if (variant < 0 || variant >= kVariants) return set_error(YASTN_ERR_ARG, "variant out of range");
  if (variant == kVariantRows && !plan->p.rows_fit) return set_error(YASTN_ERR_STATE, "row kernel does not fit this plan");
  plan->p.variant = variant;
  return YASTN_OK;
}

yastn_status yastn_plan_autotune(yastn_plan_t plan, const void *const *a, const void *const *b, void *const *c,
                                 void *workspace, void *hip_stream, int32_t reps, int32_t *chosen, float *times_ms) {
  if (!plan || reps < 1) return set_error(YASTN_ERR_ARG, "bad argument");
  yastn_status s = check_job_ptrs(&plan->p, a, b, c, workspace);
  if (s) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  std::vector<JobRef> jobs;
  for (const Group &g : plan->p.groups) jobs.push_back(JobRef{&plan->p, &g, a, b, c, workspace});
  hipEvent_t e0, e1;
  YASTN_HIP(hipEventCreate(&e0));
  YASTN_HIP(hipEventCreate(&e1));
  const int keep = plan->p.variant;
  const bool bf16 = plan->p.opts.precision == YASTN_BF16X3 || plan->p.opts.precision == YASTN_BF16X6;
  const bool f32 = plan->p.opts.precision == YASTN_F32;
  int best = 1;
  float best_ms = 1e30f;
  for (int v = 1; v < kVariants; ++v) {
    float ms = -1.f;
    const bool applicable = v == 1 || (v == kVariantRows ? plan->p.rows_fit
                                                         : (!bf16 && plan->p.buf_ok && (!f32 || v == 4)));
    if (applicable) {
      plan->p.variant = v;
      s = launch(jobs, st);  // warm-up
      if (!s) s = (hipEventRecord(e0, st) == hipSuccess) ? YASTN_OK : YASTN_ERR_HIP;
      for (int r = 0; r < reps && !s; ++r) s = launch(jobs, st);
      if (!s && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
          hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
        ms /= reps;
        if (ms < best_ms) {
          best_ms = ms;
          best = v;
        }
      }
      if (s) break;
    }
    if (times_ms) times_ms[v] = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) {
    plan->p.variant = keep;
    return s;
  }
  plan->p.variant = best;
  if (chosen) *chosen = best;
  if (times_ms) times_ms[0] = best_ms;
  return YASTN_OK;
}

yastn_status yastn_contract_jobs(const yastn_job *jobs, int32_t njobs, void *hip_stream) {
  if (njobs < 0 || (njobs > 0 && !jobs)) return set_error(YASTN_ERR_ARG, "bad job array");
  std::vector<JobRef> refs;
  for (int i = 0; i < njobs; ++i) {
    if (!jobs[i].plan) return set_error(YASTN_ERR_ARG, "null plan in job");
    const Plan &p = jobs[i].plan->p;
    const Plan &p0 = jobs[0].plan->p;
    if (p.opts.precision != p0.opts.precision || p.opts.in_dtype != p0.opts.in_dtype || p.opts.out_dtype != p0.opts.out_dtype)
      return set_error(YASTN_ERR_STATE, "jobs of one launch must share precision and dtypes");
    yastn_status s = check_job_ptrs(&p, jobs[i].a, jobs[i].b, jobs[i].c, jobs[i].workspace);
    if (s) return s;
    for (const Group &g : p.groups) refs.push_back(JobRef{&p, &g, jobs[i].a, jobs[i].b, jobs[i].c, jobs[i].workspace});
  }
  return launch(refs, reinterpret_cast<hipStream_t>(hip_stream));
}

size_t yastn_norm_workspace(void) { return 2 * kNormBlocks * sizeof(double); }

yastn_status yastn_norm(const void *x, int64_t n, yastn_dtype dtype, double *out, void *workspace, void *hip_stream) {
  if (!out || !workspace || (n > 0 && !x) || n < 0) return set_error(YASTN_ERR_ARG, "bad argument");
  if (dtype != YASTN_DTYPE_F64 && dtype != YASTN_DTYPE_F32) return set_error(YASTN_ERR_ARG, "unknown dtype");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  double *part = reinterpret_cast<double *>(workspace);
  int nb = (int)std::min<int64_t>(kNormBlocks, std::max<int64_t>(1, (n + 255) / 256));
  if (dtype == YASTN_DTYPE_F64)
    k_norm_partial<double><<<nb, 256, 0, st>>>(reinterpret_cast<const double *>(x), n, part);
  else
    k_norm_partial<float><<<nb, 256, 0, st>>>(reinterpret_cast<const float *>(x), n, part);
  k_norm_final<<<1, 256, 0, st>>>(part, nb, out);
  YASTN_HIP(hipGetLastError());
  return YASTN_OK;
}

void yastn_free(yastn_plan_t plan) {
  if (!plan) return;
  if (plan->p.dev_mem) (void)hipFree(plan->p.dev_mem);
  delete plan;
}

}  // extern "C"
