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

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
template <typename In, typename Cmp>
__global__ void __launch_bounds__(256) k_pack_b(LaunchArgs args) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int W = gridDim.x * 4;
  for (int g = gw; g < args.nitems; g += W) {
    int jb = 0;
    while (jb + 1 < args.njobs && g >= args.jobs[jb + 1].item0) ++jb;
    const JobArg &job = args.jobs[jb];
    const DevPlan &P = *job.plan;
    const DevPackItem it = P.items[g - job.item0 + job.pitem0];
    const DevSector sec = P.sectors[it.sector];
    const DevCtrTuple &ct = P.ctrs[sec.ctr0 + it.s];
    const DevColTuple &cl = P.cols[sec.col0 + it.j];
    const DevProb pr = P.probs[sec.prob];
    Cmp *dst = reinterpret_cast<Cmp *>(job.ws) + sec.bpack + (int64_t)ct.ko * sec.N + cl.no;
    const In *src = reinterpret_cast<const In *>(args.p[job.prob0 + sec.prob - job.plo].b);
    const int64_t total = (int64_t)ct.k * cl.n;
    if (it.bblk < 0) {
      for (int64_t e = lane; e < total; e += 64) dst[(e / cl.n) * sec.N + (e % cl.n)] = Cmp(0);
      continue;
    }
    const DevBBlock bb = P.bblocks[it.bblk];
    for (int64_t e = lane; e < total; e += 64) {
      const int64_t kd = e / cl.n, cb = e - kd * cl.n;
      const int64_t o = b_offset(bb, ct, cl, pr, kd, cb);
      dst[kd * sec.N + cb] = Cmp(src[o]);
    }
  }
}

// ---------------------------------------------------------------------------
// grouped gather GEMM (FP64 / FP32 MFMA, K = 4 per instruction)
// ---------------------------------------------------------------------------
struct KInfo {
  int64_t off;        // element offset of A(row 0 of the tuple, k) plus the k part; -1: block absent
  int32_t p[kMaxAct]; // P_a of k's contracted tuple
};

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

// Per-wave tile prologue shared by every precision: locate the tile and
// fill the wave's k-offset table for contracted indices [k0, kend).
__device__ __forceinline__ void build_kinfo(const DevPlan &P, const DevRowTuple &rt, const DevSector &sec,
                                            const DevProb &pr, int k0, int kend, int lane, KInfo *ki) {
  for (int k = k0 + lane; k < kend; k += 64) {
    KInfo e;
    e.off = a_koffset(P, rt, sec, pr, k, e.p);
    ki[k - k0] = e;
  }
}

template <typename In, typename Cmp, typename Out, int CB>
__global__ void __launch_bounds__(256) k_gemm4(LaunchArgs args) {
  typedef Mfma4<Cmp> M;
  typedef typename M::acc_t acc_t;
  __shared__ KInfo kinfo_all[4][kKChunk];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  KInfo *kinfo = kinfo_all[wid];
  const int gw = blockIdx.x * 4 + wid;
  const int W = gridDim.x * 4;
  for (int t = gw; t < args.ntiles; t += W) {
    int jb = 0;
    while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
    const JobArg &job = args.jobs[jb];
    const DevPlan &P = *job.plan;
    const DevTile tile = P.tiles[t - job.tile0 + job.ptile0];
    const DevRowTuple rt = P.rows[tile.rowtuple];
    const DevSector sec = P.sectors[rt.sector];
    const DevProb pr = P.probs[sec.prob];
    const ProbPtrs pp = args.p[job.prob0 + sec.prob - job.plo];
    const In *__restrict__ A = reinterpret_cast<const In *>(pp.a);
    Out *__restrict__ C = reinterpret_cast<Out *>(pp.c);
    const Cmp *__restrict__ Bp = reinterpret_cast<const Cmp *>(job.ws) + sec.bpack;
    const int rbn = (tile.nrows + 15) >> 4, cbn = (tile.ncols + 15) >> 4;

    // per-row factorised offsets RG_a(ra) of the lane's 4 rows
    int32_t rg[4][kMaxAct];
    bool rv[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int lr = 16 * rb + (lane & 15);
      rv[rb] = lr < tile.nrows;
      const int32_t ra = tile.m0 + lr;
      a_rowparts(rt, pr.nact, ra, rg[rb]);
    }
    acc_t acc[4][CB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = acc_t{0, 0, 0, 0};

    for (int k0 = 0; k0 < sec.K; k0 += kKChunk) {
      const int kend = min(sec.K, k0 + kKChunk);
      build_kinfo(P, rt, sec, pr, k0, kend, lane, kinfo);
      wave_sync();
      for (int kk = k0; kk < kend; kk += 4) {
        const int k = kk + (lane >> 4);
        Cmp av[4], bv[CB];
        KInfo e;
        e.off = -1;
        if (k < kend) e = kinfo[k - k0];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          av[rb] = Cmp(0);
          if (e.off >= 0 && rv[rb]) {
            av[rb] = Cmp(A[a_offset(e.off, e.p, rg[rb])]);
          }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int c = tile.n0 + 16 * cb + (lane & 15);
          bv[cb] = (k < kend && c < sec.N) ? Bp[(int64_t)k * sec.N + c] : Cmp(0);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          if (rb < rbn)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
              if (cb < cbn) acc[rb][cb] = M::run(av[rb], bv[cb], acc[rb][cb]);
      }
      wave_sync();
    }
    // epilogue: element (row, col) of C_X -> output block (i, j_col), row-major m_i x n_j
    const DevColTuple *cols = P.cols + sec.col0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      if (cb >= cbn) continue;
      const int c = tile.n0 + 16 * cb + (lane & 15);
      if (c >= sec.N || c >= tile.n0 + tile.ncols) continue;
      const int j = find_col(cols, sec.Q, c);
      const int64_t cbase = P.cgrid[rt.cgrid + j];
      if (cbase < 0) continue;
      const int64_t nj = cols[j].n;
      const int64_t cl = c - cols[j].no;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        if (rb >= rbn) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int lr = 16 * rb + M::row(lane, v);
          if (lr < tile.nrows) C[cbase + (int64_t)(tile.m0 + lr) * nj + cl] = Out(acc[rb][cb][v]);
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
__device__ __forceinline__ void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
  h = bf16_rne(x);
  float r = x - bf16_to_f(h);
  m = bf16_rne(r);
  if (NT > 3) {
    float r2 = r - bf16_to_f(m);
    l = bf16_rne(r2);
  } else {
    l = 0;
  }
}

template <typename In, typename Out, int CB, int NT>
__global__ void __launch_bounds__(256) k_gemm_bf16(LaunchArgs args) {
  __shared__ KInfo kinfo_all[4][kKChunk];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  KInfo *kinfo = kinfo_all[wid];
  const int gw = blockIdx.x * 4 + wid;
  const int W = gridDim.x * 4;
  for (int t = gw; t < args.ntiles; t += W) {
    int jb = 0;
    while (jb + 1 < args.njobs && t >= args.jobs[jb + 1].tile0) ++jb;
    const JobArg &job = args.jobs[jb];
    const DevPlan &P = *job.plan;
    const DevTile tile = P.tiles[t - job.tile0 + job.ptile0];
    const DevRowTuple rt = P.rows[tile.rowtuple];
    const DevSector sec = P.sectors[rt.sector];
    const DevProb pr = P.probs[sec.prob];
    const ProbPtrs pp = args.p[job.prob0 + sec.prob - job.plo];
    const In *__restrict__ A = reinterpret_cast<const In *>(pp.a);
    Out *__restrict__ C = reinterpret_cast<Out *>(pp.c);
    const float *__restrict__ Bp = reinterpret_cast<const float *>(job.ws) + sec.bpack;
    const int rbn = (tile.nrows + 15) >> 4, cbn = (tile.ncols + 15) >> 4;
    int32_t rg[4][kMaxAct];
    bool rv[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int lr = 16 * rb + (lane & 15);
      rv[rb] = lr < tile.nrows;
      const int32_t ra = tile.m0 + lr;
      a_rowparts(rt, pr.nact, ra, rg[rb]);
    }
    f4 acc[4][CB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f4{0, 0, 0, 0};
    for (int k0 = 0; k0 < sec.K; k0 += kKChunk) {
      const int kend = min(sec.K, k0 + kKChunk);
      build_kinfo(P, rt, sec, pr, k0, kend, lane, kinfo);
      wave_sync();
      for (int kk = k0; kk < kend; kk += 32) {
        const int kb = kk + 8 * (lane >> 4);  // this lane's 8 consecutive k
        uint16_t ah[4][8], am[4][8], al[4][8], bh[CB][8], bm[CB][8], bl[CB][8];
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
          const int k = kb + e8;
          KInfo e;
          e.off = -1;
          if (k < kend) e = kinfo[k - k0];
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            float x = 0.f;
            if (e.off >= 0 && rv[rb]) {
              x = float(A[a_offset(e.off, e.p, rg[rb])]);
            }
            split3<NT>(x, ah[rb][e8], am[rb][e8], al[rb][e8]);
          }
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int c = tile.n0 + 16 * cb + (lane & 15);
            float y = (k < kend && c < sec.N) ? Bp[(int64_t)k * sec.N + c] : 0.f;
            split3<NT>(y, bh[cb][e8], bm[cb][e8], bl[cb][e8]);
          }
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          if (rb >= rbn) continue;
          bf8 a_h, a_m, a_l;
#pragma unroll
          for (int e8 = 0; e8 < 8; ++e8) {
            a_h[e8] = __builtin_bit_cast(__bf16, ah[rb][e8]);
            a_m[e8] = __builtin_bit_cast(__bf16, am[rb][e8]);
            a_l[e8] = __builtin_bit_cast(__bf16, al[rb][e8]);
          }
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            if (cb >= cbn) continue;
            bf8 b_h, b_m, b_l;
#pragma unroll
            for (int e8 = 0; e8 < 8; ++e8) {
              b_h[e8] = __builtin_bit_cast(__bf16, bh[cb][e8]);
              b_m[e8] = __builtin_bit_cast(__bf16, bm[cb][e8]);
              b_l[e8] = __builtin_bit_cast(__bf16, bl[cb][e8]);
            }
            f4 c = acc[rb][cb];
            // small terms first, largest last
            if (NT > 3) {
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, b_h, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, b_l, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_m, b_m, c, 0, 0, 0);
            }
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_m, b_h, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, b_m, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, b_h, c, 0, 0, 0);
            acc[rb][cb] = c;
          }
        }
      }
      wave_sync();
    }
    const DevColTuple *cols = P.cols + sec.col0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      if (cb >= cbn) continue;
      const int c = tile.n0 + 16 * cb + (lane & 15);
      if (c >= sec.N || c >= tile.n0 + tile.ncols) continue;
      const int j = find_col(cols, sec.Q, c);
      const int64_t cbase = P.cgrid[rt.cgrid + j];
      if (cbase < 0) continue;
      const int64_t nj = cols[j].n;
      const int64_t cl = c - cols[j].no;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        if (rb >= rbn) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int lr = 16 * rb + 4 * (lane >> 4) + v;
          if (lr < tile.nrows) C[cbase + (int64_t)(tile.m0 + lr) * nj + cl] = Out(acc[rb][cb][v]);
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
         o_tiles = take(bytes_of(t.tiles)), o_items = take(bytes_of(t.items)), o_plan = take(sizeof(DevPlan));
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
  dp.ntiles = (int32_t)t.tiles.size();
  dp.nitems = (int32_t)t.items.size();
  put(o_plan, &dp, sizeof(dp));
  pl.dplan = reinterpret_cast<DevPlan *>(base + o_plan);
  YASTN_HIP(hipMemcpy(base, host.data(), off, hipMemcpyHostToDevice));
  return YASTN_OK;
}

// ---- kernel dispatch -------------------------------------------------------
typedef void (*KernelFn)(LaunchArgs);

template <typename In, typename Cmp, typename Out>
KernelFn pick_gemm4(int cb) {
  switch (cb) {
    case 1: return k_gemm4<In, Cmp, Out, 1>;
    case 2: return k_gemm4<In, Cmp, Out, 2>;
    case 3: return k_gemm4<In, Cmp, Out, 3>;
    default: return k_gemm4<In, Cmp, Out, 4>;
  }
}
template <typename In, typename Out, int NT>
KernelFn pick_bf16(int cb) {
  switch (cb) {
    case 1: return k_gemm_bf16<In, Out, 1, NT>;
    case 2: return k_gemm_bf16<In, Out, 2, NT>;
    case 3: return k_gemm_bf16<In, Out, 3, NT>;
    default: return k_gemm_bf16<In, Out, 4, NT>;
  }
}
template <typename In, typename Out>
KernelFn pick_gemm(yastn_precision p, int cb) {
  switch (p) {
    case YASTN_F64: return pick_gemm4<In, double, Out>(cb);
    case YASTN_F32: return pick_gemm4<In, float, Out>(cb);
    case YASTN_BF16X3: return pick_bf16<In, Out, 3>(cb);
    default: return pick_bf16<In, Out, 6>(cb);
  }
}
KernelFn gemm_kernel(const yastn_options &o, int cb) {
  if (o.in_dtype == YASTN_DTYPE_F64)
    return o.out_dtype == YASTN_DTYPE_F64 ? pick_gemm<double, double>(o.precision, cb) : pick_gemm<double, float>(o.precision, cb);
  return o.out_dtype == YASTN_DTYPE_F64 ? pick_gemm<float, double>(o.precision, cb) : pick_gemm<float, float>(o.precision, cb);
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

yastn_status launch(const std::vector<JobRef> &jobs, hipStream_t st) {
  if (jobs.empty()) return YASTN_OK;
  const yastn_options &o = jobs[0].plan->opts;
  int cb = 1;
  for (auto &j : jobs) cb = std::max(cb, j.plan->cb);
  KernelFn gemm = gemm_kernel(o, cb), pack = pack_kernel(o);
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
      unsigned g = (unsigned)std::min<int64_t>((la.nitems + 3) / 4, max_wg);
      YASTN_HIP(hipLaunchKernel(reinterpret_cast<const void *>(pack), dim3(g), dim3(256), kargs, 0, st));
    }
    if (la.ntiles > 0) {
      unsigned g = (unsigned)std::min<int64_t>((la.ntiles + 3) / 4, max_wg);
      YASTN_HIP(hipLaunchKernel(reinterpret_cast<const void *>(gemm), dim3(g), dim3(256), kargs, 0, st));
    }
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
    // column blocks per wave tile: enough for the widest sector, at most 4 (64 columns)
    std::vector<std::vector<std::pair<int32_t, int32_t>>> allpairs(nprob);
    for (int p = 0; p < nprob; ++p)
      if ((s = gpu_join(pl.probs[p], st, allpairs[p])) != YASTN_OK) {
        delete h;
        return s;
      }
    // first pass: widest sector decides the tile width of the plan
    int64_t a_base = 0, b_base = 0;
    pl.cb = 4;
    for (int pass = 0; pass < 2; ++pass) {
      pl.t = PlanTables{};
      pl.prob_t0.clear();
      pl.prob_i0.clear();
      a_base = b_base = 0;
      for (int p = 0; p < nprob; ++p) {
        pl.prob_t0.push_back((int32_t)pl.t.tiles.size());
        pl.prob_i0.push_back((int32_t)pl.t.items.size());
        if ((s = build_structure(pl.probs[p], p, allpairs[p], a_base, b_base, pl.t, pl.cb)) != YASTN_OK) {
          delete h;
          return s;
        }
        a_base += pl.probs[p].a.nblocks;
        b_base += pl.probs[p].b.nblocks;
      }
      if (pass == 0) {
        int64_t maxn = 1;
        for (auto &sec : pl.t.sectors) maxn = std::max<int64_t>(maxn, sec.N);
        int cb = (int)std::min<int64_t>(4, (maxn + 15) / 16);
        if (cb == pl.cb) break;
        pl.cb = cb;
      }
    }
    if (a_base > INT32_MAX || b_base > INT32_MAX) {
      delete h;
      return set_error(YASTN_ERR_ARG, "too many blocks in one plan");
    }
    finish_tiles(pl);
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
