// Block-sparse truncated SVD of a block tensor viewed as a matrix (row legs x
// column legs): the truncation step of the CTM move (paper Sec. III, Fig. 3
// (c)-(d): the enlarged corner fused into a block-diagonal matrix, its SVD
// truncated to the environment dimension chi).  gfx950 / CDNA4, FP64.
//
//  k_svd_init    W = 0 and V = identity for every sector.
//  k_svd_gather  fuse the blocks into one dense matrix per sector X (X = sum
//                over the row legs of s_i rho_i), Sec. II.B fusion: the
//                constituent tuples of a sector in ascending charge order,
//                each block's row index in C order over its row legs, its
//                column index over its column legs.  One thread per block
//                element: contiguous reads, each element's place in W from
//                per-leg strides.  A sector with fewer rows than columns is
//                stored transposed, so every working matrix W is tall.
//  k_svd_round   one round of a block one-sided Jacobi sweep, all sectors in
//                one launch: W's columns form blocks of 8; the round pairs
//                the blocks of each sector (round-robin: every pair once per
//                sweep), and one workgroup per block pair forms the 16 x 16
//                Gram matrix of its 16 columns on the FP64 MFMA, diagonalises
//                it with cyclic Jacobi rotations in LDS, and applies the
//                rotation to those columns of W and of V on the MFMA (V
//                accumulates the rotations, so W V stays M V with M the
//                sector matrix).  The largest scaled off-diagonal Gram entry
//                seen in a sweep decides convergence.
//  k_svd_qr_*    with the singular vectors formed after the sweeps
//                (YASTN_SVD_RECOVER_V): W = Q R by Householder panel steps,
//                the sweeps then run on R^T (Q is never formed), and
//                k_svd_recover_qr forms the left vectors as W v / s.
//  k_svd_colsort before each sweep, the columns of each sector in order of
//  k_svd_colperm descending norm (de Rijk's ordering).
//  k_svd_norms   singular values = column norms of the converged W; W's
//                columns scaled to unit norm (the left vectors).
//  k_svd_sort    each sector's values in descending order (rank by count).
//  k_svd_*       the global truncation: values at or below tol x max are
//                dropped; if more than chi remain and c is the (chi+1)-th
//                largest, a value is kept iff it exceeds c (1 + deg_tol).
//  k_svd_gauge   the sign of each kept pair (u_t, v_t): the one whose u_t
//                has its entry of largest magnitude (the first such in row
//                order) positive, so the factors are unique for distinct
//                values.
//  k_svd_write   the kept columns of U and rows of V^T as block tensors, with
//                that sign and, on request, column / row t scaled by S_t^p
//                (p = -1/2 gives the CTM projector factors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/yastn.h"
#include "index.hpp"
#include "planner.hpp"

#define SVD_HIP(call)                                                                                            \
  do {                                                                                                           \
    hipError_t e_ = (call);                                                                                      \
    if (e_ != hipSuccess) return set_error(YASTN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace yastn {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kSvdW = 8;           // columns per block (a block pair is 16 columns: one MFMA tile)
constexpr int kSvdMaxSweeps = 40;  // outer sweeps before giving up
constexpr int kSvdInnerSweeps = 1; // cyclic Jacobi sweeps on a pair's 16 x 16 Gram matrix per round
constexpr int kSvdWaves = 8;       // waves of a round's workgroup (one workgroup per block pair)
constexpr int kSvdGramGroups = 16; // 4-row groups of a wave's Gram loads in flight
constexpr int kSvdRotChunks = 2;   // 16-row chunks of a wave's rotation loads in flight
                                   // (78 VGPRs: three workgroups per CU; 4 chunks take 94
                                   // and 8 take 156, fewer workgroups and slower rounds)

// W (rows x ld) and V (ld x ld) are stored in panels of 8 columns: panel p
// holds columns 8p .. 8p + 7 of every row, row after row, so a column block
// of the Jacobi sweep is one contiguous array and every load and store of a
// round touches whole runs of 64-byte rows
struct DevSvdSector {
  int64_t w_off;   // W: rows x ld in 8-column panels, elements from the workspace base
  int64_t v_off;   // V: ld x ld in 8-column panels
  int64_t m_off;   // a copy of the sector matrix (W's layout), for right vectors recovered at the end
  int64_t s_off;   // scratch for the column reordering: W's layout, then V's
  int32_t rows;    // W's rows (>= cols)
  int32_t cols;    // W's columns
  int32_t ld;      // kSvdW * nb
  int32_t nb;      // column blocks, even, >= 2
  int32_t npairs;  // nb / 2: the sector's workgroups in a round
  int32_t sv0;     // first of the sector's cols singular values (global index)
  int32_t trans;   // 1: W = M^T
  int32_t pad;
};

struct DevSvdGather {  // one block of T: element e (C order over T's legs) -> W
  int64_t t_off;       // first element in T's buffer
  int64_t w_off;       // the sector's W
  int64_t wr0, wc0;    // W row and column of the block's element 0
  int32_t numel, rank;
  int32_t wrows;       // W's rows
  uint32_t colmask;    // bit l: leg l's index moves along W's columns (else rows)
  int32_t dim[YASTN_MAX_RANK];
  uint32_t mag[YASTN_MAX_RANK];
  int32_t sh[YASTN_MAX_RANK];
  int64_t wstr[YASTN_MAX_RANK];  // W row or column step of each leg's index
};
struct DevSvdTile {
  int32_t blk, start;
};
constexpr int kSvdTile = 1024;

struct DevSvdOut {     // one output block: U (kind 0) or V^T (kind 1)
  int64_t out_off;     // first element in the output buffer
  int64_t base;        // workspace offset of the source matrix (W or V)
  int32_t a, b;        // U: m_i x t; V^T: t x n_j
  int32_t r0, rows;    // the source row of the block's first row (U) / column (V^T); the source's rows
  int32_t sv0, kind;   // the sector's first sorted index (perm); 0 = U, 1 = V^T
};

// element (r, c) of a matrix of R rows in 8-column panels
__device__ __forceinline__ int64_t pix(int64_t r, int c, int64_t R) {
  return (int64_t)(c >> 3) * (R << 3) + (r << 3) + (c & 7);
}

// 1 / y and 1 / sqrt(x) from the hardware estimates refined by two Newton
// steps each (the error of the estimate squared per step): the rotation
// parameters need no correct rounding, only c^2 (1 + t^2) = 1 to working
// precision, which the refined 1 / sqrt gives for any t
__device__ __forceinline__ double rcp_nr(double y) {
  double r = __builtin_amdgcn_rcp(y);
  r = fma(r, fma(-y, r, 1.0), r);
  r = fma(r, fma(-y, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
  r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
  return r;
}

// ------------------------------------------------------------------ kernels
__global__ void __launch_bounds__(256) k_svd_init(const DevSvdSector *sec, int nsec, double *ws) {
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector s = sec[k];
    const int64_t nw = (int64_t)s.rows * s.ld, nv = (int64_t)s.ld * s.ld;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < nw + nv; i += (int64_t)gridDim.x * 256) {
      if (i < nw) {
        ws[s.w_off + i] = 0.0;
      } else {
        const int64_t j = i - nw;  // panel p = j / (8 ld), row (j mod 8 ld) / 8, column 8 p + j mod 8
        const int64_t pnl = j / (8 * (int64_t)s.ld), in = j - pnl * 8 * s.ld;
        ws[s.v_off + j] = ((in >> 3) == 8 * pnl + (in & 7)) ? 1.0 : 0.0;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_svd_gather(const DevSvdGather *__restrict__ blocks,
                                                    const DevSvdTile *__restrict__ tiles, int ntiles,
                                                    const double *__restrict__ t, double *__restrict__ ws) {
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const DevSvdTile tl = tiles[ti];
    const DevSvdGather &b = blocks[tl.blk];
    const int end = min(tl.start + kSvdTile, b.numel);
    for (int e = tl.start + (int)threadIdx.x; e < end; e += 256) {
      uint32_t r = (uint32_t)e;
      int64_t wr = b.wr0, wc = b.wc0;
      for (int d = b.rank - 1; d >= 0; --d) {
        const uint32_t q = (uint32_t)(((uint64_t)r * b.mag[d]) >> b.sh[d]);
        const int64_t step = (int64_t)(r - q * (uint32_t)b.dim[d]) * b.wstr[d];
        if ((b.colmask >> d) & 1u) wc += step;
        else wr += step;
        r = q;
      }
      ws[b.w_off + pix(wr, (int)wc, b.wrows)] = t[b.t_off + e];
    }
  }
}

// workgroup -> (sector, block pair) of a round; the largest sectors' pairs
// first, so the longest workgroups start first
struct DevSvdWg {
  int32_t sec, p;
};

struct SvdRoundArgs {
  const DevSvdSector *sec;
  const DevSvdWg *wg;
  double *ws;
  unsigned long long *conv;  // per sector: largest scaled off-diagonal Gram entry this sweep (bits of a double >= 0)
  const int32_t *done;       // per sector: converged, skip
  int32_t nsec, round;
  double rot_tol;            // rotate a pair only above this scaled off-diagonal entry
  int32_t with_v;            // 0: V is not accumulated (right vectors recovered after the sweeps)
  double *nrm2;              // per column: its squared norm after the round that last rotated it
};

// The round-robin pairing of nb blocks (nb even): round rr in [0, nb - 1),
// pair p in [0, nb / 2); every unordered pair of blocks once per nb - 1 rounds.
__device__ __forceinline__ void rr_pair(int nb, int rr, int p, int &P, int &Q) {
  const int n1 = nb - 1;
  if (p == 0) {
    P = n1;
    Q = rr;
  } else {
    P = (rr + p) % n1;
    Q = (rr - p + n1) % n1;
  }
}

__global__ void __launch_bounds__(64 * kSvdWaves) k_svd_round(SvdRoundArgs a) {
  __shared__ double gpart[kSvdWaves][16][16];
  __shared__ double g[16][17];
  __shared__ double q[16][17];
  __shared__ int rotated;
  const DevSvdWg wgi = a.wg[blockIdx.x];
  const int lo = wgi.sec, p = wgi.p;
  const DevSvdSector S = a.sec[lo];  // loaded together with the flag
  if (a.done[lo]) return;
  int P, Q;
  rr_pair(S.nb, a.round % (S.nb - 1), p, P, Q);
  double *W = a.ws + S.w_off;
  double *V = a.ws + S.v_off;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int c16 = lane & 15, kq = lane >> 4;
  auto colof = [&](int c) { return c < kSvdW ? kSvdW * P + c : kSvdW * Q + c - kSvdW; };
  // ---- Gram matrix of the 16 columns: wave w takes the 4-row groups w,
  // w + kSvdWaves, ...; kSvdGramGroups groups' loads are issued before their
  // MFMAs (row indices clamped, values past the last row zeroed after the
  // load, so no load sits under a branch)
  {
    const int col = colof(c16);
    constexpr int kStride = 4 * kSvdWaves;
    d4v acc = {0, 0, 0, 0};
    for (int r0 = 4 * wid; r0 < S.rows; r0 += kStride * kSvdGramGroups) {
      double x[kSvdGramGroups];
#pragma unroll
      for (int u = 0; u < kSvdGramGroups; ++u) x[u] = W[pix(min(r0 + kStride * u + kq, S.rows - 1), col, S.rows)];
#pragma unroll
      for (int u = 0; u < kSvdGramGroups; ++u) {
        const double xv = r0 + kStride * u + kq < S.rows ? x[u] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, xv, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) gpart[wid][kq + 4 * v][c16] = acc[v];
  }
  __syncthreads();
  // W's rows, then V's rows (the same row stride), are rotated in 16-row
  // chunks, kSvdRotChunks chunks of a wave in flight at once (clamped loads;
  // stores past the last row skipped), so V's loads overlap W's.  The loads
  // do not depend on the rotation: each wave issues its first chunks now,
  // and they arrive while wave 0 runs the Jacobi.
  const int nw = S.rows, nt = S.rows + (a.with_v ? S.cols : 0);
  const int cout = colof(c16);
  int cin[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) cin[kk] = colof(4 * kk + kq);
  auto at = [&](int r, int c) { return r < nw ? W + pix(r, c, nw) : V + pix(r - nw, c, S.ld); };
  constexpr int kChunk = 16 * kSvdWaves;
  const int rb0 = 16 * wid;
  double x[kSvdRotChunks][4];
  auto load_chunks = [&](int rb) {
#pragma unroll
    for (int u = 0; u < kSvdRotChunks; ++u) {
      const int r = min(rb + kChunk * u + c16, nt - 1);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) x[u][kk] = *at(r, cin[kk]);
    }
  };
  if (rb0 < nt) load_chunks(rb0);
  if (wid == 0) {
    // sum the waves' parts in a fixed order, Q = I
    for (int e = lane; e < 256; e += 64) {
      const int i = e >> 4, j = e & 15;
      double sum = gpart[0][i][j];
#pragma unroll
      for (int w = 1; w < kSvdWaves; ++w) sum += gpart[w][i][j];
      g[i][j] = sum;
      q[i][j] = i == j ? 1.0 : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // convergence measure: largest |g_ij| / sqrt(g_ii g_jj) over i != j
    // (the largest square, one square root at the end)
    double off2 = 0.0;
    for (int e = lane; e < 256; e += 64) {
      const int i = e >> 4, j = e & 15;
      const double d = g[i][i] * g[j][j];
      // (the estimate of 1 / d: the measure only decides convergence)
      if (i != j && d > 0.0) off2 = fmax(off2, g[i][j] * g[i][j] * __builtin_amdgcn_rcp(d));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) off2 = fmax(off2, __shfl_xor(off2, o, 64));
    const double off = off2 > 0.0 ? off2 * rsq_nr(off2) : 0.0;
    if (lane == 0) atomicMax(a.conv + lo, (unsigned long long)__double_as_longlong(off));
    int any = 0;
    if (off > a.rot_tol) {
      // cyclic Jacobi on g (16 x 16): 15 rounds of 8 disjoint rotations.  Lane
      // (rx, ry) owns the 2 x 2 block of g on the index pairs of rotations rx
      // (rows) and ry (columns) and the same block of q: it reads the block
      // and rotation ry's diagonal and off-diagonal entries together (one
      // LDS round trip per round), forms rotation ry, takes rotation rx from
      // lane rx, and writes g <- J^T g J and q <- q J on its block.  Lanes
      // with the same ry compute the same (c, s).
      const int rx = lane >> 3, ry = lane & 7;
      const double tol2 = a.rot_tol * a.rot_tol;
      // J = [[c, s], [-s, c]] on (i, j) zeroing g_ij of J^T g J: with
      // a = g_jj - g_ii and b = 2 g_ij, t = tan = sign(a) b / (|a| + sqrt(a^2 + b^2))
      // (the smaller root; |t| <= 1), c = 1 / sqrt(1 + t^2), s = t c; no rotation when
      // g_ij is below rot_tol sqrt(g_ii g_jj) (compared squared)
      auto rot_of = [&](double gii, double gjj, double gij, double &c, double &sn) {
        const double d = gii * gjj;
        const bool go = gij != 0.0 && d > 0.0 && gij * gij > tol2 * d;
        // formed without a branch; a lane without rotation takes c = 1,
        // s = 0 (what it formed, possibly not finite, is discarded by the
        // select).  t needs no full precision (one Newton step on each
        // estimate), c does (two).
        const double aa = gjj - gii, bb = 2.0 * gij;
        const double h = fma(aa, aa, bb * bb);
        double r = __builtin_amdgcn_rsq(h);
        r = fma(0.5 * r, fma(-h * r, r, 1.0), r);
        const double den = fma(h, r, fabs(aa));
        double rd = __builtin_amdgcn_rcp(den);
        rd = fma(rd, fma(-den, rd, 1.0), rd);
        const double t = (aa < 0.0 ? -bb : bb) * rd;
        const double cc = rsq_nr(fma(t, t, 1.0));
        c = go ? cc : 1.0;
        sn = go ? t * cc : 0.0;
        return go;
      };
      for (int sw = 0; sw < kSvdInnerSweeps; ++sw) {
        int applied = 0;
        for (int rr = 0; rr < 15; ++rr) {
          // round-robin pair of 16 indices without a division
          auto pair_of = [&](int r, int &i, int &j) {
            i = 15;
            j = rr;
            if (r != 0) {
              i = rr + r;
              i -= i >= 15 ? 15 : 0;
              j = rr - r;
              j += j < 0 ? 15 : 0;
            }
          };
          int ix, jx, iy, jy;
          pair_of(rx, ix, jx);
          pair_of(ry, iy, jy);
          const double yii = g[iy][iy], yjj = g[jy][jy], yij = g[iy][jy];
          const double b00 = g[ix][iy], b01 = g[ix][jy], b10 = g[jx][iy], b11 = g[jx][jy];
          const double q00 = q[ix][iy], q01 = q[ix][jy], q10 = q[jx][iy], q11 = q[jx][jy];
          double cy, sy;
          applied |= rot_of(yii, yjj, yij, cy, sy);
          // rotation rx as formed by lane rx (whose column rotation it is)
          const double cx = __shfl(cy, rx, 64), sx = __shfl(sy, rx, 64);
          // C = B J_y (columns), then J_x^T C (rows)
          const double c00 = cy * b00 - sy * b01, c01 = sy * b00 + cy * b01;
          const double c10 = cy * b10 - sy * b11, c11 = sy * b10 + cy * b11;
          // every lane has read this round's entries before any lane writes
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          g[ix][iy] = cx * c00 - sx * c10;
          g[jx][iy] = sx * c00 + cx * c10;
          g[ix][jy] = cx * c01 - sx * c11;
          g[jx][jy] = sx * c01 + cx * c11;
          q[ix][iy] = cy * q00 - sy * q01;
          q[ix][jy] = sy * q00 + cy * q01;
          q[jx][iy] = cy * q10 - sy * q11;
          q[jx][jy] = sy * q10 + cy * q11;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        applied = __any(applied);
        any |= applied;
        if (!applied) break;
      }
    }
    if (lane == 0) rotated = any;
    // the squared column norms after this round (the diagonal of the rotated
    // Gram matrix): the next sweep orders the columns by them
    if (lane < 16) {
      const int col = colof(lane);
      if (col < S.cols) a.nrm2[S.sv0 + col] = g[lane][lane];
    }
  }
  __syncthreads();
  if (!rotated) return;
  // ---- [W_P W_Q] <- [W_P W_Q] q and [V_P V_Q] <- [V_P V_Q] q: wave w takes
  // 16-row chunks w, w + kSvdWaves, ...; A operand = 16 rows x 4 of the 16
  // columns, B operand = 4 rows of q
  double qb[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) qb[kk] = q[4 * kk + kq][c16];
  for (int rb = rb0; rb < nt; rb += kChunk * kSvdRotChunks) {
    if (rb != rb0) load_chunks(rb);
    d4v acc[kSvdRotChunks];
#pragma unroll
    for (int u = 0; u < kSvdRotChunks; ++u) {
      acc[u] = d4v{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u][kk], qb[kk], acc[u], 0, 0, 0);
    }
    // every lane has read its rows before any lane of the wave writes them
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < kSvdRotChunks; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb + kChunk * u + kq + 4 * v;
        if (r < nt) *at(r, cout) = acc[u][v];
      }
  }
}

// ---- QR preconditioning of the sweeps (right vectors recovered) ----------
// W = Q R by Householder reflections, then the sweeps run on X = R^T (n x n:
// its columns are nearly orthogonal and graded, and one-sided Jacobi on it
// needs about half the sweeps); the right vectors of W are X's converged
// normalised columns and the left ones are recovered as W v / s.  Q itself
// is never formed.
constexpr int kSvdQrMaxRows = 1024;  // rows of a sector's panel held in LDS
constexpr bool kSvdUseQr = true;     // precondition the sweeps when the right vectors are recovered
constexpr int kSvdQrGroup = 1;       // trailing panels per workgroup of a panel step (4: longer chains, slower)
constexpr int kSvdRecChunk = 256, kSvdRecT = 8;  // right-vector recovery: rows per LDS chunk, pairs per pass

// sums of 8 per-thread values over a 256-thread workgroup, in a fixed order;
// every thread returns the 8 sums.  Within a wave a transposing butterfly:
// the xor-32, -16 and -8 exchanges each halve the values a lane keeps (4, 2,
// then 1: value ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3)
// & 1)), the xor-4, -2 and -1 exchanges finish that value's sum: 10
// exchanges instead of 48.
__device__ __forceinline__ void qr_sum8(double (&v)[8], double (*red)[8], double *out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double w[4], x[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b5 ? v[i] : v[i + 4];
    const double keep = b5 ? v[i + 4] : v[i];
    w[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b4 ? w[i] : w[i + 2];
    const double keep = b4 ? w[i + 2] : w[i];
    x[i] = keep + __shfl_xor(send, 16, 64);
  }
  double y = (b3 ? x[1] : x[0]) + __shfl_xor(b3 ? x[0] : x[1], 8, 64);
  y += __shfl_xor(y, 4, 64);
  y += __shfl_xor(y, 2, 64);
  y += __shfl_xor(y, 1, 64);
  if ((lane & 7) == 0) red[wid][(b5 ? 4 : 0) + (b4 ? 2 : 0) + (b3 ? 1 : 0)] = y;
  __syncthreads();
  if (threadIdx.x < 8) out[threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = out[i];
}

// One panel step p (columns 8p .. 8p + 7) for every sector that has it.
// Workgroup (x, y): sector y; x = 0 the panel itself, x >= 1 the trailing
// panels p + 1 + (x - 1) G .. p + x G (G = kSvdQrGroup).  Every workgroup of a sector
// factors panel p (rows 8p .. m - 1) in LDS with the same arithmetic, so all
// hold the same reflectors (v with v_0 = 1, tau; beta on the diagonal).
// x = 0 writes the panel's triangle of R, transposed, into X; x > 0 applies
// the eight reflectors in order to each of its panels of W (rows 8p .. m - 1)
// in place, each thread holding four rows of it.  Panel p itself is only read, so the
// workgroups of a step do not race.
__global__ void __launch_bounds__(256) k_svd_qr_step(const DevSvdSector *sec, const DevSvdSector *qsec, int nsec,
                                                     double *ws, int p) {
  __shared__ double P[kSvdQrMaxRows][8];
  __shared__ double red[4][8];
  __shared__ double sums[8];
  __shared__ double tau[8];
  const int tid = threadIdx.x;
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k];
    const int npan = (S.cols + 7) >> 3;
    // x = 0: the panel itself; x >= 1: trailing panels q0 .. q0 + kSvdQrGroup - 1
    const int q0 = blockIdx.x == 0 ? p : p + 1 + ((int)blockIdx.x - 1) * kSvdQrGroup;
    if (p >= npan || q0 >= npan) continue;  // uniform across the workgroup
    const int m = S.rows, r0 = 8 * p, mt = m - r0;
    double *W = ws + S.w_off;
    const double *Wp = W + (int64_t)p * m * 8 + (int64_t)r0 * 8;  // panel p, row r0
    // the panel into LDS, sixteen loads of a thread in flight at a time
    for (int e0 = 0; e0 < mt * 8; e0 += 256 * 16) {
      double buf[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = e0 + tid + 256 * i;
        buf[i] = e < mt * 8 ? Wp[e] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int e = e0 + tid + 256 * i;
        if (e < mt * 8) P[e >> 3][e & 7] = buf[i];
      }
    }
    __syncthreads();
    for (int c = 0; c < 8; ++c) {
      // the reflector of column c from rows c .. mt - 1, and its effect on
      // the panel's columns c + 1 .. 7, from one reduction: d_j = sum over
      // rows r > c of x_r P[r][j] (d_c = |x_tail|^2), then with v_r =
      // x_r / (alpha - beta) the dot v^T P[:, j] = P[c][j] + d_j / (alpha -
      // beta).  Row c is read before the reduction's barriers, written after.
      double v8[8], pc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        v8[i] = 0.0;
        pc[i] = P[c][i];
      }
      for (int r = c + 1 + tid; r < mt; r += 256) {
        const double xr = P[r][c];
#pragma unroll
        for (int j = 0; j < 8; ++j) v8[j] = fma(xr, P[r][j], v8[j]);
      }
      qr_sum8(v8, red, sums);
      const double s = v8[c], alpha = pc[c];
      double t = 0.0, beta = alpha, scale = 0.0;
      if (s > 0.0) {
        beta = -copysign(sqrt(fma(alpha, alpha, s)), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      double dot[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) dot[j] = fma(scale, v8[j], pc[j]);
      for (int r = c + tid; r < mt; r += 256) {
        const double vr = r == c ? 1.0 : P[r][c] * scale;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j > c) P[r][j] -= t * vr * dot[j];
        if (r > c) P[r][c] = vr;
      }
      if (tid == 0) {
        P[c][c] = beta;
        tau[c] = t;
      }
      __syncthreads();
    }
    if (blockIdx.x == 0) {
      // R's diagonal block, transposed: X[8p + j][8p + c] = R[8p + c][8p + j], c <= j
      const DevSvdSector Q = qsec[k];
      double *X = ws + Q.w_off;
      if (tid < 64) {
        const int c = tid >> 3, j = tid & 7;
        if (c <= j && r0 + j < S.cols) X[pix(r0 + j, r0 + c, Q.rows)] = P[c][j];
      }
      __syncthreads();  // P is reused by the next sector
      continue;
    }
    // apply the reflectors to panels q0 .. q0 + kSvdQrGroup - 1, rows
    // r0 .. m - 1 (four rows per thread)
    for (int q = q0; q < min(npan, q0 + kSvdQrGroup); ++q) {
      double *Wq = W + (int64_t)q * m * 8 + (int64_t)r0 * 8;
      double a[4][8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = tid + 256 * u;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[u][j] = r < mt ? Wq[r * 8 + j] : 0.0;
      }
      for (int c = 0; c < 8; ++c) {
        double v8[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v8[j] = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = tid + 256 * u;
          const double vr = r < c || r >= mt ? 0.0 : (r == c ? 1.0 : P[r][c]);
#pragma unroll
          for (int j = 0; j < 8; ++j) v8[j] = fma(vr, a[u][j], v8[j]);
        }
        qr_sum8(v8, red, sums);
        const double t = tau[c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = tid + 256 * u;
          const double vr = r < c || r >= mt ? 0.0 : (r == c ? 1.0 : P[r][c]);
#pragma unroll
          for (int j = 0; j < 8; ++j) a[u][j] -= t * vr * v8[j];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = tid + 256 * u;
        if (r < mt)
#pragma unroll
          for (int j = 0; j < 8; ++j) Wq[r * 8 + j] = a[u][j];
      }
    }
    __syncthreads();  // P is reused by the next sector
  }
}

// X = R^T below the diagonal blocks (R[b][a] from row b of W for panel(b) <
// panel(a)) and zeros above the diagonal and in the padding columns; the
// diagonal blocks were written by the panel steps
__global__ void __launch_bounds__(256) k_svd_qr_finish(const DevSvdSector *sec, const DevSvdSector *qsec, int nsec,
                                                       double *ws) {
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k], Q = qsec[k];
    const double *W = ws + S.w_off;
    double *X = ws + Q.w_off;
    const int n = S.cols;
    const int64_t ne = (int64_t)n * S.ld;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < ne; e += (int64_t)gridDim.x * 256) {
      const int b = (int)((e / ((int64_t)n * 8)) * 8 + (e & 7));  // column of X
      const int a = (int)((e % ((int64_t)n * 8)) >> 3);            // row of X
      if (b < n && b <= a && (a >> 3) == (b >> 3)) continue;      // a diagonal block entry
      X[e] = b < n && b <= a ? W[pix(b, a, S.rows)] : 0.0;
    }
  }
}

// Kept pair t of sector k after sweeps on X: v = X's normalised column j
// (j = perm[t]) into column j of V, and the left vector w = M0 v / s_j into
// column j of W.  A workgroup takes kSvdRecT pairs and 256 rows of W, v in
// LDS in chunks, each sum in ascending column order.
__global__ void __launch_bounds__(256) k_svd_recover_qr(const DevSvdSector *sec, const DevSvdSector *qsec, int nsec,
                                                        double *ws, const int32_t *perm, const double *sv,
                                                        const int32_t *kept) {
  __shared__ double x[kSvdRecT][kSvdRecChunk];
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k], Q = qsec[k];
    const double *X = ws + Q.w_off;
    const double *M0 = ws + S.m_off;
    double *W = ws + S.w_off;
    double *V = ws + S.v_off;
    const int nk = kept[k], n = S.cols;
    const int ntc = (nk + kSvdRecT - 1) / kSvdRecT, nrc = (S.rows + 255) / 256;
    for (int item = blockIdx.x; item < ntc * nrc; item += gridDim.x) {
      const int t0 = (item / nrc) * kSvdRecT, r = (item % nrc) * 256 + (int)threadIdx.x;
      int jt[kSvdRecT];
#pragma unroll
      for (int q = 0; q < kSvdRecT; ++q) jt[q] = t0 + q < nk ? perm[S.sv0 + t0 + q] : -1;
      double acc[kSvdRecT];
#pragma unroll
      for (int q = 0; q < kSvdRecT; ++q) acc[q] = 0.0;
      for (int c0 = 0; c0 < n; c0 += kSvdRecChunk) {
        const int nc = min(kSvdRecChunk, n - c0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSvdRecT; ++q)
          if ((int)threadIdx.x < nc) {
            const double xv = jt[q] >= 0 ? X[pix(c0 + (int)threadIdx.x, jt[q], Q.rows)] : 0.0;
            x[q][threadIdx.x] = xv;
            // the right vector, once per pair (the row chunk 0 workgroup)
            if (jt[q] >= 0 && item % nrc == 0) V[pix(c0 + (int)threadIdx.x, jt[q], S.ld)] = xv;
          }
        __syncthreads();
        if (r < S.rows)
          for (int c = 0; c < nc; ++c) {
            const double mv = M0[pix(r, c0 + c, S.rows)];
#pragma unroll
            for (int q = 0; q < kSvdRecT; ++q) acc[q] = fma(mv, x[q][c], acc[q]);
          }
      }
      if (r < S.rows)
#pragma unroll
        for (int q = 0; q < kSvdRecT; ++q)
          if (jt[q] >= 0) W[pix(r, jt[q], S.rows)] = acc[q] * (1.0 / sv[S.sv0 + t0 + q]);
    }
  }
}

// M0 = W for every sector (the fused matrix, kept for the recovery of the
// right vectors)
__global__ void __launch_bounds__(256) k_svd_copy_m(const DevSvdSector *sec, int nsec, double *ws) {
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector s = sec[k];
    const int64_t nw = (int64_t)s.rows * s.ld;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < nw; i += (int64_t)gridDim.x * 256)
      ws[s.m_off + i] = ws[s.w_off + i];
  }
}

// The right vectors of the kept pairs of a sector without accumulated
// rotations: with W = M0 V converged and u_j = w_j / s_j (column j = perm[t]
// of the normalised W), M0^T u_j = s_j v_j, so v_j = M0^T u_j / s_j, written
// into column j of V.  Its error is about (rows)^1/2 eps s_max / s_j
// relative, so the mode suits truncations that keep the large values only.
// A workgroup takes kSvdRecT kept pairs and 256 columns: the pairs' u in
// LDS in chunks of kSvdRecChunk rows, one thread per column, M0 read once
// per kSvdRecT pairs, each sum in ascending row order.
__global__ void __launch_bounds__(256) k_svd_recover(const DevSvdSector *sec, int nsec, double *ws,
                                                     const int32_t *perm, const double *sv, const int32_t *kept) {
  __shared__ double u[kSvdRecT][kSvdRecChunk];
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k];
    const double *W = ws + S.w_off;
    const double *M0 = ws + S.m_off;
    double *V = ws + S.v_off;
    const int nk = kept[k];
    const int ntc = (nk + kSvdRecT - 1) / kSvdRecT, ncc = (S.cols + 255) / 256;
    for (int item = blockIdx.x; item < ntc * ncc; item += gridDim.x) {
      const int t0 = (item / ncc) * kSvdRecT, c = (item % ncc) * 256 + (int)threadIdx.x;
      int jt[kSvdRecT];
#pragma unroll
      for (int q = 0; q < kSvdRecT; ++q) jt[q] = t0 + q < nk ? perm[S.sv0 + t0 + q] : -1;
      double acc[kSvdRecT];
#pragma unroll
      for (int q = 0; q < kSvdRecT; ++q) acc[q] = 0.0;
      for (int r0 = 0; r0 < S.rows; r0 += kSvdRecChunk) {
        const int nr = min(kSvdRecChunk, S.rows - r0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSvdRecT; ++q)
          if ((int)threadIdx.x < nr) u[q][threadIdx.x] = jt[q] >= 0 ? W[pix(r0 + (int)threadIdx.x, jt[q], S.rows)] : 0.0;
        __syncthreads();
        if (c < S.cols)
          for (int r = 0; r < nr; ++r) {
            const double m = M0[pix(r0 + r, c, S.rows)];
#pragma unroll
            for (int q = 0; q < kSvdRecT; ++q) acc[q] = fma(m, u[q][r], acc[q]);
          }
      }
      if (c < S.cols)
#pragma unroll
        for (int q = 0; q < kSvdRecT; ++q)
          if (jt[q] >= 0) V[pix(c, jt[q], S.ld)] = acc[q] * (1.0 / sv[S.sv0 + t0 + q]);
    }
  }
}

// Squared column norms of W before the first sweep (one wave per 8-column
// panel, lanes over 8 rows x 8 columns, fixed summation order); later sweeps
// take them from the rounds.
__global__ void __launch_bounds__(256) k_svd_colnorm2(const DevSvdSector *sec, int nsec, const double *ws,
                                                      double *nrm2) {
  const int lane = threadIdx.x & 63;
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k];
    const int npan = S.ld >> 3;
    for (int p = blockIdx.x * 4 + (threadIdx.x >> 6); p < npan; p += gridDim.x * 4) {
      const double *pan = ws + S.w_off + (int64_t)p * S.rows * 8;
      double ss = 0.0;
      for (int r = lane >> 3; r < S.rows; r += 8) {
        const double x = pan[(int64_t)r * 8 + (lane & 7)];
        ss = fma(x, x, ss);
      }
      ss += __shfl_xor(ss, 8, 64);
      ss += __shfl_xor(ss, 16, 64);
      ss += __shfl_xor(ss, 32, 64);
      const int col = 8 * p + (lane & 7);
      if (lane < 8 && col < S.cols) nrm2[S.sv0 + col] = ss;
    }
  }
}

// Column order of each sector at the start of a sweep: descending norm
// (ties by index), the order that sorting the columns of a one-sided Jacobi
// before each sweep (de Rijk) uses; it cuts the sweeps of graded matrices.
// Workgroup (x, y) ranks columns 256 y .. 256 y + 255 of sector x by
// counting over the sector's squared norms, staged in LDS as FP32 (the order
// is a heuristic: FP32 keys compare at the full VALU rate, and ties still
// go by index, so the ranks are a permutation): perm[sv0 + rank] = column;
// chg[k] (zeroed at the sweep's start) is set when a column moves.
// Converged sectors and sectors wider than kSvdSortMax keep their order.
constexpr int kSvdSortMax = 4096, kSvdSortSlice = 256;
__global__ void __launch_bounds__(256) k_svd_colsort(const DevSvdSector *sec, int nsec, const double *nrm2,
                                                     const int32_t *done, int32_t *perm, int32_t *chg) {
  __shared__ float nrm[kSvdSortMax];
  for (int k = blockIdx.x; k < nsec; k += gridDim.x) {
    const DevSvdSector S = sec[k];
    const int j0 = (int)blockIdx.y * kSvdSortSlice;
    if (done[k] || S.cols > kSvdSortMax || j0 >= S.cols) continue;  // uniform across the workgroup
    for (int j = threadIdx.x; j < S.cols; j += 256) nrm[j] = (float)nrm2[S.sv0 + j];
    __syncthreads();
    const int j = j0 + (int)threadIdx.x;
    int moved = 0;
    if (j < S.cols) {
      const float v = nrm[j];
      int rank = 0, i = 0;
      // sixteen LDS reads in flight per batch (one read per step waits on
      // the LDS latency every time); bitwise, not short-circuit, logic, so
      // the compares stay branch-free
      for (; i + 16 <= S.cols; i += 16) {
        float u[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) u[q] = nrm[i + q];
#pragma unroll
        for (int q = 0; q < 16; ++q) rank += (int)(u[q] > v) | ((int)(u[q] == v) & (int)(i + q < j));
      }
      for (; i < S.cols; ++i) {
        const float u = nrm[i];
        rank += (int)(u > v) | ((int)(u == v) & (int)(i < j));
      }
      perm[S.sv0 + rank] = j;
      moved = rank != j;
    }
    // one atomic per workgroup (the barrier also keeps nrm until every
    // thread has ranked: the next sector reuses it)
    if (__syncthreads_or(moved) && threadIdx.x == 0) atomicOr(chg + k, 1);
  }
}

// Reordered columns, for the sectors whose order changed: back = 0 gathers
// W[:, perm[t]] (and V[:, perm[t]] when with_v) into the sector's scratch,
// back = 1 copies the scratch over W (and V); only the columns that move
// (perm[t] != t) are touched, and padding columns keep their (zero) values.
__global__ void __launch_bounds__(256) k_svd_colperm(const DevSvdSector *sec, int nsec, double *ws, const int32_t *perm,
                                                     const int32_t *chg, int with_v, int back) {
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    if (!chg[k]) continue;
    const DevSvdSector S = sec[k];
    const int64_t nw = (int64_t)S.rows * S.ld, nv = with_v ? (int64_t)S.ld * S.ld : 0;
    double *scr = ws + S.s_off;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < nw + nv; e += (int64_t)gridDim.x * 256) {
      const bool inw = e < nw;
      const int64_t i = inw ? e : e - nw;           // element in W's or V's panel layout
      const int64_t R = inw ? S.rows : S.ld;        // rows of that matrix
      double *M = ws + (inw ? S.w_off : S.v_off);
      const int t = (int)((i / (R * 8)) * 8 + (i & 7));  // column of element i
      if (t >= S.cols) continue;
      const int src = perm[S.sv0 + t];
      if (src == t) continue;
      if (back) {
        M[i] = scr[e];
      } else {
        const int64_t r = (i % (R * 8)) >> 3;
        scr[e] = M[pix(r, src, R)];
      }
    }
  }
}

// conv[k] = 0 (every sweep); done[k] = 0 too when done is given (first
// sweep), chg[k] = 0 when chg is given
__global__ void k_svd_sweep_begin(unsigned long long *conv, int32_t *done, int nsec, int32_t *chg) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nsec; k += gridDim.x * blockDim.x) {
    conv[k] = 0ull;
    if (done) done[k] = 0;
    if (chg) chg[k] = 0;
  }
}

// done[k] = 1 once sector k's sweep saw no scaled off-diagonal entry above
// tol; *alldone = every sector done (one workgroup)
__global__ void __launch_bounds__(256) k_svd_sweep_end(const unsigned long long *conv, int32_t *done, int nsec,
                                                       const DevSvdSector *sec, double eps_scale, int32_t *alldone) {
  __shared__ int notdone;
  if (threadIdx.x == 0) notdone = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nsec; k += 256) {
    const double off = __longlong_as_double((long long)conv[k]);
    const double tol = fmax(1e-14, eps_scale * sqrt((double)sec[k].rows));
    if (!done[k] && off <= tol) done[k] = 1;
    if (!done[k]) atomicOr(&notdone, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *alldone = notdone ? 0 : 1;
}

// singular value j of a sector = norm of W's column j; the column scaled to
// unit norm.  One wave per 8-column panel: lanes over 8 rows x 8 columns
// (64-byte row segments), a fixed summation order.
__global__ void __launch_bounds__(256) k_svd_norms(const DevSvdSector *sec, int nsec, double *ws, double *sv_raw) {
  const int lane = threadIdx.x & 63;
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k];
    const int npan = S.ld >> 3;
    for (int p = blockIdx.x * 4 + (threadIdx.x >> 6); p < npan; p += gridDim.x * 4) {
      double *pan = ws + S.w_off + (int64_t)p * S.rows * 8;
      double ss = 0.0;
      for (int r = lane >> 3; r < S.rows; r += 8) {
        const double x = pan[(int64_t)r * 8 + (lane & 7)];
        ss = fma(x, x, ss);
      }
      ss += __shfl_xor(ss, 8, 64);
      ss += __shfl_xor(ss, 16, 64);
      ss += __shfl_xor(ss, 32, 64);
      const int col = 8 * p + (lane & 7);
      const double sig = sqrt(ss);
      const double inv = sig > 0.0 ? 1.0 / sig : 0.0;
      if (col < S.cols) {
        for (int r = lane >> 3; r < S.rows; r += 8) pan[(int64_t)r * 8 + (lane & 7)] *= inv;
        if (lane < 8) sv_raw[S.sv0 + col] = sig;
      }
    }
  }
}

// descending order within each sector: rank of value j = values that are
// larger, or equal with a smaller index; sv[sv0 + rank] and perm.
// Workgroup (x, y) ranks values 256 y .. 256 y + 255 of sector x, from LDS
// when the sector has at most kSvdSortMax values, else from memory.
__global__ void __launch_bounds__(256) k_svd_sort(const DevSvdSector *sec, int nsec, const double *sv_raw, double *sv,
                                                  int32_t *perm) {
  __shared__ double xs[kSvdSortMax];
  for (int k = blockIdx.x; k < nsec; k += gridDim.x) {
    const DevSvdSector S = sec[k];
    const double *x = sv_raw + S.sv0;
    const bool lds = S.cols <= kSvdSortMax;
    for (int j0 = (int)blockIdx.y * 256; j0 < S.cols; j0 += (int)gridDim.y * 256) {  // uniform
      if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < S.cols; i += 256) xs[i] = x[i];
        __syncthreads();
      }
      const double *src = lds ? xs : x;
      const int j = j0 + (int)threadIdx.x;
      if (j < S.cols) {
        const double v = src[j];
        int rank = 0, i = 0;
        for (; i + 16 <= S.cols; i += 16) {
          double w[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) w[q] = src[i + q];
#pragma unroll
          for (int q = 0; q < 16; ++q) rank += (int)(w[q] > v) | ((int)(w[q] == v) & (int)(i + q < j));
        }
        for (; i < S.cols; ++i) rank += (int)(src[i] > v) | ((int)(src[i] == v) & (int)(i < j));
        sv[S.sv0 + rank] = v;
        perm[S.sv0 + rank] = j;
      }
    }
  }
}

// largest value and how many exceed tol x largest (one workgroup)
__global__ void __launch_bounds__(1024) k_svd_stats(const double *sv, int n, double tol, double *stat) {
  __shared__ double mx[1024];
  __shared__ int cnt[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) m = fmax(m, sv[i]);
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
    __syncthreads();
  }
  const double floor_v = tol * mx[0];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 1024) c += sv[i] > floor_v;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stat[0] = mx[0];
    stat[1] = floor_v;
    stat[2] = (double)cnt[0];
    stat[3] = floor_v;  // the cut, raised by k_svd_cut when more than chi remain
  }
}

// the (chi+1)-th largest value c among those above the floor: the value v
// with (# larger) <= chi < (# larger or equal); cut = c (1 + deg_tol)
__global__ void __launch_bounds__(256) k_svd_cut(const double *sv, int n, int chi, double deg_tol, double *stat) {
  __shared__ double tile[256];
  const double floor_v = stat[1];
  const bool need = stat[2] > (double)chi;
  if (!need) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double v = i < n ? sv[i] : -1.0;
  int gt = 0, ge = 0;
  for (int j0 = 0; j0 < n; j0 += 256) {
    __syncthreads();
    tile[threadIdx.x] = j0 + (int)threadIdx.x < n ? sv[j0 + threadIdx.x] : -1.0;
    __syncthreads();
    const int m = min(256, n - j0);
    // bitwise logic (no branch per compare), sixteen LDS reads in flight
    int j = 0;
    for (; j + 16 <= m; j += 16) {
      double w[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) w[q] = tile[j + q];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int above = (int)(w[q] > floor_v);
        gt += above & (int)(w[q] > v);
        ge += above & (int)(w[q] >= v);
      }
    }
    for (; j < m; ++j) {
      const double w = tile[j];
      const int above = (int)(w > floor_v);
      gt += above & (int)(w > v);
      ge += above & (int)(w >= v);
    }
  }
  if (i < n && v > floor_v && gt <= chi && chi < ge) stat[3] = v * (1.0 + deg_tol);
}

// kept[k] = how many of sector k's values exceed the cut: its values are
// in descending order, so a binary search for the first one at or below it
__global__ void __launch_bounds__(256) k_svd_kept(const DevSvdSector *sec, int nsec, const double *sv,
                                                  const double *stat, int32_t *kept) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < nsec; k += gridDim.x * 256) {
    const DevSvdSector S = sec[k];
    const double cut = stat[3];
    int lo = 0, hi = S.cols;  // sv[sv0 + i] > cut for i < lo, <= cut for i >= hi
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sv[S.sv0 + mid] > cut) lo = mid + 1;
      else hi = mid;
    }
    kept[k] = lo;
  }
}

// sign of kept pair t of a sector: u_t = column perm[t] of U (W, or V for a
// sector stored transposed), rows 0 .. mU-1; the entry of largest |u| (the
// first in row order on ties) decides.  One wave per kept pair, lanes stride
// the rows, then a butterfly over (|u|, row) that keeps the larger magnitude
// and, at equal magnitude, the smaller row.
__global__ void __launch_bounds__(256) k_svd_gauge(const DevSvdSector *sec, int nsec, const double *ws,
                                                   const int32_t *perm, const int32_t *kept, double *sign) {
  const int lane = threadIdx.x & 63;
  for (int k = blockIdx.y; k < nsec; k += gridDim.y) {
    const DevSvdSector S = sec[k];
    const double *U = ws + (S.trans ? S.v_off : S.w_off);
    const int mU = S.trans ? S.cols : S.rows;     // U's rows: m
    const int64_t RU = S.trans ? S.ld : S.rows;   // rows of the matrix that holds U
    const int nk = kept[k];
    for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < nk; t += gridDim.x * 4) {
      const int j = perm[S.sv0 + t];
      double best = -1.0, val = 0.0;
      int row = 0x7fffffff;
      for (int r = lane; r < mU; r += 64) {
        const double x = U[pix(r, j, RU)];
        if (fabs(x) > best) {  // rows ascend per lane: the first maximum stays
          best = fabs(x);
          val = x;
          row = r;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64), ov = __shfl_xor(val, o, 64);
        const int orow = __shfl_xor(row, o, 64);
        if (ob > best || (ob == best && orow < row)) {
          best = ob;
          val = ov;
          row = orow;
        }
      }
      if (lane == 0) sign[S.sv0 + t] = val < 0.0 ? -1.0 : 1.0;
    }
  }
}

__device__ __forceinline__ double sv_power(double s, double p) {
  if (p == 0.0) return 1.0;
  if (p == -0.5) return 1.0 / sqrt(s);
  if (p == 0.5) return sqrt(s);
  return pow(s, p);
}

// U block (kind 0): element (r, t) = sign_t S_t^pu src(r0 + r, perm[t]), out
// row-major a x b (b = t kept); V^T block (kind 1): element (t, c) = sign_t
// S_t^pv src(r0 + c, perm[t]), out row-major a x b (a = kept).  S_t is the
// sector's t-th largest value, sv_raw[sv0 + perm[sv0 + t]].
__global__ void __launch_bounds__(256) k_svd_write(const DevSvdOut *__restrict__ items, int nitems,
                                                   const double *__restrict__ ws, const int32_t *__restrict__ perm,
                                                   const double *__restrict__ sv_raw,
                                                   const double *__restrict__ sign, double pu, double pv,
                                                   double *__restrict__ u, double *__restrict__ vt) {
  __shared__ double fac[512];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const DevSvdOut o = items[it];
    const int64_t n = (int64_t)o.a * o.b;
    double *out = o.kind == 0 ? u : vt;
    const int nt = o.kind == 0 ? o.b : o.a;
    const double p = o.kind == 0 ? pu : pv;
    __syncthreads();
    for (int t = threadIdx.x; t < nt && t < 512; t += 256)
      fac[t] = sign[o.sv0 + t] * sv_power(sv_raw[o.sv0 + perm[o.sv0 + t]], p);
    __syncthreads();
    for (int64_t e = threadIdx.x; e < n; e += 256) {
      const int32_t x = (int32_t)(e / o.b), y = (int32_t)(e - (int64_t)x * o.b);
      const int32_t r = o.kind == 0 ? x : y, t = o.kind == 0 ? y : x;
      const double f = t < 512 ? fac[t] : sign[o.sv0 + t] * sv_power(sv_raw[o.sv0 + perm[o.sv0 + t]], p);
      out[o.out_off + e] = f * ws[o.base + pix(o.r0 + r, perm[o.sv0 + t], o.rows)];
    }
  }
}

unsigned grid1(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65535)); }

using Key = std::vector<int32_t>;

}  // namespace

struct SvdPlanImpl {
  HostTensor t;
  std::vector<int32_t> row_legs, col_legs;
  struct Tuple {
    Key key;
    std::vector<int64_t> dims;
    int64_t size, off;  // elements (product of dims) and first row / column in the sector matrix
  };
  struct Sector {
    Key x;
    std::vector<Tuple> rows, cols;
    int64_t m = 0, n = 0;
  };
  std::vector<Sector> sectors;
  std::vector<DevSvdSector> dsec;
  int64_t nsv = 0;
  int max_rounds = 1, total_pairs = 0, max_cols = 1;
  int max_panels = 0;   // 8-column panels of the widest sector (QR steps)
  bool qr_ok = true;    // every sector's rows fit the QR panel step
  int32_t flags = 0;  // YASTN_SVD_RECOVER_V
  size_t ws_bytes = 0;
  size_t off_sv_raw = 0, off_perm = 0, off_conv = 0, off_done = 0, off_stat = 0, off_flag = 0, off_sign = 0,
         off_chg = 0;
  void *dev_mem = nullptr;  // sectors, gather blocks and tiles
  DevSvdSector *d_sec = nullptr;
  DevSvdGather *d_gather = nullptr;
  DevSvdTile *d_tiles = nullptr;
  DevSvdWg *d_wg = nullptr;
  DevSvdSector *d_secqr = nullptr;  // the sectors as the sweeps on X = R^T see them
  int ngather = 0, ntiles = 0;
  int device = 0;
  // after yastn_svd: kept counts and the output structures
  std::vector<int32_t> kept;
  bool have_kept = false;
  std::vector<int32_t> u_q, v_q;
  std::vector<int64_t> u_sh, v_sh, u_off, v_off;
  std::vector<int8_t> u_sig, v_sig;
  std::vector<int32_t> u_n, v_n;
  int64_t u_numel = 0, v_numel = 0;
  std::vector<DevSvdOut> outs;
  void *out_mem = nullptr;
  int sweeps = 0;
};

}  // namespace yastn

using namespace yastn;

struct yastn_svd_s {
  SvdPlanImpl p;
};

namespace {

int64_t norm_q(int64_t v, int32_t m) {
  if (m == 0) return v;
  int64_t r = v % m;
  return r < 0 ? r + m : r;
}

}  // namespace

extern "C" {

yastn_status yastn_svd_plan(const yastn_tensor_desc *t, int32_t nrow, const int32_t *row_legs, void *hip_stream,
                            yastn_svd_t *out) {
  if (!t || !out || (nrow > 0 && !row_legs)) return set_error(YASTN_ERR_ARG, "null argument");
  *out = nullptr;
  yastn_svd_t h = nullptr;
  try {
    h = new yastn_svd_s;
    SvdPlanImpl &P = h->p;
    yastn_status st = validate_tensor(*t, "T", P.t);
    if (st != YASTN_OK) {
      delete h;
      return st;
    }
    const HostTensor &T = P.t;
    const int r = T.rank, ns = T.nsym;
    if (nrow < 1 || nrow >= r) {
      delete h;
      return set_error(YASTN_ERR_ARG, "row legs must be a non-empty proper subset of the legs");
    }
    bool isrow[YASTN_MAX_RANK] = {false};
    for (int i = 0; i < nrow; ++i) {
      if (row_legs[i] < 0 || row_legs[i] >= r || isrow[row_legs[i]]) {
        delete h;
        return set_error(YASTN_ERR_ARG, "row legs out of range or repeated");
      }
      isrow[row_legs[i]] = true;
      P.row_legs.push_back(row_legs[i]);
    }
    for (int i = 0; i < r; ++i)
      if (!isrow[i]) P.col_legs.push_back(i);
    // ---- sectors: X = sum over row legs of s_i rho_i; tuples ascending
    std::map<Key, std::map<Key, std::vector<int64_t>>> rows, cols;
    std::vector<Key> bx(size_t(T.nblocks)), brk(size_t(T.nblocks)), bck(size_t(T.nblocks));
    for (int64_t b = 0; b < T.nblocks; ++b) {
      Key x(ns, 0);
      for (int c = 0; c < ns; ++c) {
        int64_t v = 0;
        for (int l : P.row_legs) v += int64_t(T.sig[l]) * T.q(b, l)[c];
        x[c] = (int32_t)norm_q(v, T.sym_mod[c]);
      }
      Key rk, ck;
      std::vector<int64_t> rd, cd;
      for (int l : P.row_legs) {
        rk.insert(rk.end(), T.q(b, l), T.q(b, l) + ns);
        rd.push_back(T.dim(b, l));
      }
      for (int l : P.col_legs) {
        ck.insert(ck.end(), T.q(b, l), T.q(b, l) + ns);
        cd.push_back(T.dim(b, l));
      }
      rows[x][rk] = rd;
      cols[x][ck] = cd;
      bx[b] = x;
      brk[b] = rk;
      bck[b] = ck;
    }
    std::map<Key, int> sec_id;
    for (auto &kv : rows) {
      SvdPlanImpl::Sector s;
      s.x = kv.first;
      for (auto &rv : kv.second) {
        int64_t sz = 1;
        for (int64_t d : rv.second) sz *= d;
        s.rows.push_back({rv.first, rv.second, sz, s.m});
        s.m += sz;
      }
      for (auto &cv : cols[kv.first]) {
        int64_t sz = 1;
        for (int64_t d : cv.second) sz *= d;
        s.cols.push_back({cv.first, cv.second, sz, s.n});
        s.n += sz;
      }
      if (std::max(s.m, s.n) > (int64_t(1) << 15)) {
        delete h;
        return set_error(YASTN_ERR_ARG, "sector matrix side above 32768");
      }
      sec_id[kv.first] = (int)P.sectors.size();
      P.sectors.push_back(std::move(s));
    }
    // ---- device sector table and workspace layout
    int64_t welems = 0;
    int wg = 0;
    for (auto &s : P.sectors) {
      DevSvdSector d{};
      d.trans = s.m < s.n;
      d.rows = (int32_t)std::max(s.m, s.n);
      d.cols = (int32_t)std::min(s.m, s.n);
      int nb = (d.cols + kSvdW - 1) / kSvdW;
      nb = std::max(2, nb + (nb & 1));
      d.nb = nb;
      d.ld = kSvdW * nb;
      d.w_off = welems;
      welems += int64_t(d.rows) * d.ld;
      d.v_off = welems;
      welems += int64_t(d.ld) * d.ld;
      d.m_off = welems;
      welems += int64_t(d.rows) * d.ld;
      d.s_off = welems;
      welems += int64_t(d.rows) * d.ld + int64_t(d.ld) * d.ld;
      d.npairs = nb / 2;
      wg += nb / 2;
      d.sv0 = (int32_t)P.nsv;
      P.nsv += d.cols;
      P.max_rounds = std::max(P.max_rounds, nb - 1);
      P.max_cols = std::max(P.max_cols, (int)d.cols);
      P.max_panels = std::max(P.max_panels, ((int)d.cols + 7) / 8);
      P.qr_ok = P.qr_ok && d.rows <= kSvdQrMaxRows;
      P.dsec.push_back(d);
    }
    P.total_pairs = wg;
    const int nsec = (int)P.sectors.size();
    // the round's workgroups: sectors by descending rows (then index), pairs in order
    std::vector<DevSvdWg> wgs;
    {
      std::vector<int> ord(static_cast<size_t>(nsec), 0);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return P.dsec[size_t(x)].rows > P.dsec[size_t(y)].rows; });
      for (int k : ord)
        for (int q = 0; q < P.dsec[size_t(k)].npairs; ++q) wgs.push_back(DevSvdWg{k, q});
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = al(size_t(welems) * 8);
    P.off_sv_raw = off;
    off += al(size_t(std::max<int64_t>(1, P.nsv)) * 8);
    P.off_perm = off;
    off += al(size_t(std::max<int64_t>(1, P.nsv)) * 4);
    P.off_conv = off;
    off += al(size_t(std::max(1, nsec)) * 8);
    P.off_done = off;
    off += al(size_t(std::max(1, nsec)) * 4);
    P.off_stat = off;
    off += al(4 * 8);
    P.off_flag = off;
    off += al(8);
    P.off_sign = off;
    off += al(size_t(std::max<int64_t>(1, P.nsv)) * 8);
    P.off_chg = off;
    off += al(size_t(std::max(1, nsec)) * 4);
    P.ws_bytes = off;
    // ---- gather items: one per block of T, W strides per leg
    std::vector<DevSvdGather> gat;
    std::vector<DevSvdTile> tiles;
    for (int64_t b = 0; b < T.nblocks; ++b) {
      const int k = sec_id.at(bx[b]);
      const SvdPlanImpl::Sector &s = P.sectors[k];
      const DevSvdSector &d = P.dsec[k];
      int64_t ro = -1, co = -1;
      for (auto &tp : s.rows)
        if (tp.key == brk[b]) ro = tp.off;
      for (auto &tp : s.cols)
        if (tp.key == bck[b]) co = tp.off;
      DevSvdGather g{};
      g.t_off = T.offsets[b];
      g.numel = (int32_t)T.size(b);
      g.rank = r;
      // index weights within the block's row (column) of the sector matrix
      int64_t wrow[YASTN_MAX_RANK] = {0}, wcol[YASTN_MAX_RANK] = {0};
      int64_t acc = 1;
      for (int i = (int)P.row_legs.size() - 1; i >= 0; --i) {
        wrow[P.row_legs[i]] = acc;
        acc *= T.dim(b, P.row_legs[i]);
      }
      acc = 1;
      for (int i = (int)P.col_legs.size() - 1; i >= 0; --i) {
        wcol[P.col_legs[i]] = acc;
        acc *= T.dim(b, P.col_legs[i]);
      }
      // M[ro + rowidx][co + colidx]; W = M or W = M^T (rows and columns swapped)
      g.w_off = d.w_off;
      g.wrows = d.rows;
      g.wr0 = d.trans ? co : ro;
      g.wc0 = d.trans ? ro : co;
      g.colmask = 0;
      for (int l = 0; l < r; ++l) {
        g.dim[l] = (int32_t)T.dim(b, l);
        div_magic((uint32_t)g.dim[l], &g.mag[l], &g.sh[l]);
        const bool rl = wrow[l] != 0;  // leg l indexes M's rows
        g.wstr[l] = rl ? wrow[l] : wcol[l];
        if (rl == (d.trans != 0)) g.colmask |= 1u << l;  // a W column: M's column, or M's row when transposed
      }
      for (int32_t s0 = 0; s0 < g.numel; s0 += kSvdTile) tiles.push_back(DevSvdTile{(int32_t)gat.size(), s0});
      gat.push_back(g);
    }
    P.ngather = (int)gat.size();
    P.ntiles = (int)tiles.size();
    // the sectors for sweeps on X = R^T: n rows, X in the scratch region,
    // the column reordering's scratch after it
    std::vector<DevSvdSector> dsq(P.dsec);
    for (auto &d : dsq) {
      d.w_off = d.s_off;
      d.s_off += int64_t(d.cols) * d.ld;
      d.rows = d.cols;
    }
    const size_t o_sec = 0, o_gat = al(P.dsec.size() * sizeof(DevSvdSector)),
                 o_til = o_gat + al(gat.size() * sizeof(DevSvdGather)), o_wg = o_til + al(tiles.size() * sizeof(DevSvdTile)),
                 o_sq = o_wg + al(wgs.size() * sizeof(DevSvdWg)), tot = o_sq + al(dsq.size() * sizeof(DevSvdSector));
    std::vector<char> host(std::max<size_t>(tot, 256), 0);
    if (!P.dsec.empty()) std::memcpy(host.data() + o_sec, P.dsec.data(), P.dsec.size() * sizeof(DevSvdSector));
    if (!gat.empty()) std::memcpy(host.data() + o_gat, gat.data(), gat.size() * sizeof(DevSvdGather));
    if (!tiles.empty()) std::memcpy(host.data() + o_til, tiles.data(), tiles.size() * sizeof(DevSvdTile));
    if (!wgs.empty()) std::memcpy(host.data() + o_wg, wgs.data(), wgs.size() * sizeof(DevSvdWg));
    if (!dsq.empty()) std::memcpy(host.data() + o_sq, dsq.data(), dsq.size() * sizeof(DevSvdSector));
    if (hipGetDevice(&P.device) != hipSuccess || hipMalloc(&P.dev_mem, host.size()) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return set_error(YASTN_ERR_NOMEM, "device tables of the SVD plan");
    }
    char *base = reinterpret_cast<char *>(P.dev_mem);
    P.d_sec = reinterpret_cast<DevSvdSector *>(base + o_sec);
    P.d_gather = reinterpret_cast<DevSvdGather *>(base + o_gat);
    P.d_tiles = reinterpret_cast<DevSvdTile *>(base + o_til);
    P.d_wg = reinterpret_cast<DevSvdWg *>(base + o_wg);
    P.d_secqr = reinterpret_cast<DevSvdSector *>(base + o_sq);
    hipStream_t stm = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(P.dev_mem, host.data(), host.size(), hipMemcpyHostToDevice, stm) != hipSuccess ||
        hipStreamSynchronize(stm) != hipSuccess) {
      (void)hipGetLastError();
      yastn_svd_free(h);
      return set_error(YASTN_ERR_HIP, "upload of the SVD plan");
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_svd_set_flags(yastn_svd_t h, int32_t flags) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (flags & ~YASTN_SVD_RECOVER_V) return set_error(YASTN_ERR_ARG, "unknown SVD flag");
  h->p.flags = flags;
  return YASTN_OK;
}

yastn_status yastn_svd_info(yastn_svd_t h, int32_t *nsectors, int64_t *nsv, size_t *workspace_bytes) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (nsectors) *nsectors = (int32_t)h->p.sectors.size();
  if (nsv) *nsv = h->p.nsv;
  if (workspace_bytes) *workspace_bytes = h->p.ws_bytes;
  return YASTN_OK;
}

yastn_status yastn_svd_sector(yastn_svd_t h, int32_t k, int32_t *charge, int64_t *m, int64_t *n, int64_t *sv0) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (k < 0 || k >= (int32_t)h->p.sectors.size()) return set_error(YASTN_ERR_ARG, "sector index out of range");
  const auto &s = h->p.sectors[k];
  if (charge)
    for (size_t c = 0; c < s.x.size(); ++c) charge[c] = s.x[c];
  if (m) *m = s.m;
  if (n) *n = s.n;
  if (sv0) *sv0 = h->p.dsec[k].sv0;
  return YASTN_OK;
}

yastn_status yastn_svd(yastn_svd_t h, const void *t, int32_t chi, double tol, double deg_tol, double *sv,
                       int32_t *kept, int32_t *sweeps, void *workspace, void *hip_stream) {
  if (!h || !kept || (h->p.nsv > 0 && (!t || !sv || !workspace))) return set_error(YASTN_ERR_ARG, "null argument");
  if (chi < 0 || !(tol >= 0.0) || !(deg_tol >= 0.0)) return set_error(YASTN_ERR_ARG, "chi, tol and deg_tol must be >= 0");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u) return set_error(YASTN_ERR_ARG, "workspace must be 256-byte aligned");
  SvdPlanImpl &P = h->p;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int nsec = (int)P.sectors.size();
  P.have_kept = false;
  P.kept.assign(size_t(nsec), 0);
  if (sweeps) *sweeps = 0;
  if (nsec == 0) return YASTN_OK;
  char *ws = reinterpret_cast<char *>(workspace);
  double *W = reinterpret_cast<double *>(ws);
  double *sv_raw = reinterpret_cast<double *>(ws + P.off_sv_raw);
  int32_t *perm = reinterpret_cast<int32_t *>(ws + P.off_perm);
  unsigned long long *conv = reinterpret_cast<unsigned long long *>(ws + P.off_conv);
  int32_t *done = reinterpret_cast<int32_t *>(ws + P.off_done);
  double *stat = reinterpret_cast<double *>(ws + P.off_stat);
  int32_t *flag = reinterpret_cast<int32_t *>(ws + P.off_flag);
  int32_t *chg = reinterpret_cast<int32_t *>(ws + P.off_chg);
  // one pass: fuse, sweeps, values, truncation, factors; with recover set, the
  // right vectors are formed at the end if that is accurate enough
  auto attempt = [&](bool recover, bool &accurate) -> yastn_status {
    accurate = true;
    // ---- W = fused sector matrices, V = I, no sector done
    hipLaunchKernelGGL(k_svd_init, dim3(64, std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec, nsec, W);
    hipLaunchKernelGGL(k_svd_sweep_begin, dim3(grid1(nsec, 256)), dim3(256), 0, st, conv, done, nsec,
                       (int32_t *)nullptr);
    if (P.ntiles > 0)
      hipLaunchKernelGGL(k_svd_gather, dim3(std::min(P.ntiles, 65535)), dim3(256), 0, st, P.d_gather, P.d_tiles,
                         P.ntiles, reinterpret_cast<const double *>(t), W);
    if (recover)
      hipLaunchKernelGGL(k_svd_copy_m, dim3(64, std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec, nsec, W);
    // with the right vectors recovered, the sweeps run on X = R^T of W = Q R
    const bool qr = recover && kSvdUseQr && P.qr_ok;
    const DevSvdSector *swsec = qr ? P.d_secqr : P.d_sec;
    if (qr) {
      for (int p = 0; p < P.max_panels; ++p)
        hipLaunchKernelGGL(k_svd_qr_step, dim3(1 + (P.max_panels - p - 1 + kSvdQrGroup - 1) / kSvdQrGroup,
                                               std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec,
                           (const DevSvdSector *)P.d_secqr, nsec, W, p);
      hipLaunchKernelGGL(k_svd_qr_finish, dim3(256, std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec,
                         (const DevSvdSector *)P.d_secqr, nsec, W);
    }
    SVD_HIP(hipGetLastError());
    // ---- sweeps of rounds until every sector is converged
    SvdRoundArgs ra{};
    ra.with_v = recover ? 0 : 1;
    ra.nrm2 = sv_raw;  // free until the values are formed after the sweeps
    hipLaunchKernelGGL(k_svd_colnorm2, dim3(64, std::min(nsec, 65535)), dim3(256), 0, st, swsec, nsec,
                       (const double *)W, sv_raw);
    ra.sec = swsec;
    ra.wg = P.d_wg;
    ra.ws = W;
    ra.conv = conv;
    ra.done = done;
    ra.nsec = nsec;
    const double eps = 2.220446049250313e-16;
    const double eps_scale = 64.0 * eps;  // convergence: off <= max(1e-14, 64 eps sqrt(rows))
    ra.rot_tol = 4.0 * eps;
    int32_t all = 0;
    int sw = 0;
    for (; sw < kSvdMaxSweeps && !all; ++sw) {
      hipLaunchKernelGGL(k_svd_sweep_begin, dim3(grid1(nsec, 256)), dim3(256), 0, st, conv, (int32_t *)nullptr, nsec,
                         chg);
      // columns by descending norm (the order is recomputed every sweep)
      hipLaunchKernelGGL(k_svd_colsort,
                         dim3(std::min(nsec, 65535), std::min(P.max_cols + kSvdSortSlice - 1, kSvdSortMax) / kSvdSortSlice),
                         dim3(256), 0, st, swsec, nsec, (const double *)sv_raw, (const int32_t *)done, perm, chg);
      for (int back = 0; back < 2; ++back)
        hipLaunchKernelGGL(k_svd_colperm, dim3(256, std::min(nsec, 65535)), dim3(256), 0, st, swsec, nsec, W,
                           (const int32_t *)perm, (const int32_t *)chg, ra.with_v, back);
      for (int rr = 0; rr < P.max_rounds; ++rr) {
        ra.round = rr;
        hipLaunchKernelGGL(k_svd_round, dim3(P.total_pairs), dim3(64 * kSvdWaves), 0, st, ra);
      }
      hipLaunchKernelGGL(k_svd_sweep_end, dim3(1), dim3(256), 0, st, conv, done, nsec, swsec, eps_scale, flag);
      SVD_HIP(hipGetLastError());
      SVD_HIP(hipMemcpyAsync(&all, flag, 4, hipMemcpyDeviceToHost, st));
      SVD_HIP(hipStreamSynchronize(st));
    }
    P.sweeps += sw;
    if (!all) return set_error(YASTN_ERR_STATE, "Jacobi sweeps did not converge");
    // ---- singular values, sorted per sector; global truncation
    hipLaunchKernelGGL(k_svd_norms, dim3(64, std::min(nsec, 65535)), dim3(256), 0, st, swsec, nsec, W, sv_raw);
    hipLaunchKernelGGL(k_svd_sort, dim3(std::min(nsec, 65535), std::min((P.max_cols + 255) / 256, 64)), dim3(256), 0, st,
                       P.d_sec, nsec, sv_raw, sv, perm);
    hipLaunchKernelGGL(k_svd_stats, dim3(1), dim3(1024), 0, st, sv, (int)P.nsv, tol, stat);
    hipLaunchKernelGGL(k_svd_cut, dim3(grid1(P.nsv, 256)), dim3(256), 0, st, sv, (int)P.nsv, chi, deg_tol, stat);
    int32_t *dkept = reinterpret_cast<int32_t *>(ws + P.off_done);  // done[] is free again
    hipLaunchKernelGGL(k_svd_kept, dim3(grid1(nsec, 256)), dim3(256), 0, st, P.d_sec, nsec, sv, stat, dkept);
    if (recover) {
      // the recovered right vectors carry about sqrt(rows) eps s_max / s_t of
      // relative error: only when the smallest kept value keeps that below
      // 1e-11 is the mode used; else the caller runs the SVD again with the
      // rotations accumulated
      std::vector<double> hsv(size_t(P.nsv));
      SVD_HIP(hipMemcpyAsync(P.kept.data(), dkept, size_t(nsec) * 4, hipMemcpyDeviceToHost, st));
      SVD_HIP(hipMemcpyAsync(hsv.data(), sv, size_t(P.nsv) * 8, hipMemcpyDeviceToHost, st));
      SVD_HIP(hipStreamSynchronize(st));
      double smax = 0.0, smin = 0.0;
      int rows_max = 1;
      bool any = false;
      for (int k = 0; k < nsec; ++k) {
        const DevSvdSector &d = P.dsec[size_t(k)];
        if (d.cols > 0) smax = std::max(smax, hsv[size_t(d.sv0)]);
        if (P.kept[size_t(k)] > 0) {
          const double v = hsv[size_t(d.sv0 + P.kept[size_t(k)] - 1)];
          smin = any ? std::min(smin, v) : v;
          any = true;
          rows_max = std::max(rows_max, (int)d.rows);
        }
      }
      if (any && !(smin > 0.0 && 4.0 * std::sqrt((double)rows_max) * eps * smax <= 1e-11 * smin)) {
        accurate = false;
        return YASTN_OK;
      }
      if (qr)
        hipLaunchKernelGGL(k_svd_recover_qr, dim3(256, std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec,
                           (const DevSvdSector *)P.d_secqr, nsec, W, perm, sv, dkept);
      else
        hipLaunchKernelGGL(k_svd_recover, dim3(256, std::min(nsec, 65535)), dim3(256), 0, st,
                           P.d_sec, nsec, W, perm, sv, dkept);
    }
    hipLaunchKernelGGL(k_svd_gauge, dim3(8, std::min(nsec, 65535)), dim3(256), 0, st, P.d_sec, nsec, W, perm, dkept,
                       reinterpret_cast<double *>(ws + P.off_sign));
    SVD_HIP(hipGetLastError());
    SVD_HIP(hipMemcpyAsync(P.kept.data(), dkept, size_t(nsec) * 4, hipMemcpyDeviceToHost, st));
    SVD_HIP(hipStreamSynchronize(st));
    return YASTN_OK;
  };
  P.sweeps = 0;
  bool accurate = true;
  yastn_status ss = attempt((P.flags & YASTN_SVD_RECOVER_V) != 0, accurate);
  if (ss == YASTN_OK && !accurate) ss = attempt(false, accurate);
  if (sweeps) *sweeps = P.sweeps;
  if (ss != YASTN_OK) return ss;
  std::memcpy(kept, P.kept.data(), size_t(nsec) * 4);
  P.have_kept = true;
  // ---- output structures for these kept counts
  const HostTensor &T = P.t;
  const int ns = T.nsym;
  P.u_sig.clear();
  P.v_sig.clear();
  for (int l : P.row_legs) P.u_sig.push_back(T.sig[l]);
  P.u_sig.push_back(-1);
  P.v_sig.push_back(1);
  for (int l : P.col_legs) P.v_sig.push_back(T.sig[l]);
  P.u_n.assign(size_t(ns), 0);
  P.v_n.assign(T.n, T.n + ns);
  struct Blk {
    Key key;
    std::vector<int64_t> shape;
    DevSvdOut o;
  };
  std::vector<Blk> ub, vb;
  for (int k = 0; k < nsec; ++k) {
    const int32_t tk = P.kept[k];
    if (tk == 0) continue;
    const auto &s = P.sectors[k];
    const DevSvdSector &d = P.dsec[k];
    // U = W (normalised) or V (transposed sector); V^T's source the other
    const int64_t usrc = d.trans ? d.v_off : d.w_off, vsrc = d.trans ? d.w_off : d.v_off;
    for (auto &tp : s.rows) {
      Blk b;
      b.key = tp.key;
      b.key.insert(b.key.end(), s.x.begin(), s.x.end());
      b.shape = tp.dims;
      b.shape.push_back(tk);
      b.o = DevSvdOut{0, usrc, (int32_t)tp.size, tk, (int32_t)tp.off, d.trans ? d.ld : d.rows, d.sv0, 0};
      ub.push_back(std::move(b));
    }
    for (auto &tp : s.cols) {
      Blk b;
      b.key = s.x;
      b.key.insert(b.key.end(), tp.key.begin(), tp.key.end());
      b.shape.push_back(tk);
      b.shape.insert(b.shape.end(), tp.dims.begin(), tp.dims.end());
      b.o = DevSvdOut{0, vsrc, tk, (int32_t)tp.size, (int32_t)tp.off, d.trans ? d.rows : d.ld, d.sv0, 1};
      vb.push_back(std::move(b));
    }
  }
  auto lay = [&](std::vector<Blk> &bs, std::vector<int32_t> &q, std::vector<int64_t> &sh, std::vector<int64_t> &of,
                 int64_t &numel) {
    std::sort(bs.begin(), bs.end(), [](const Blk &x, const Blk &y) { return x.key < y.key; });
    q.clear();
    sh.clear();
    of.clear();
    numel = 0;
    for (auto &b : bs) {
      q.insert(q.end(), b.key.begin(), b.key.end());
      sh.insert(sh.end(), b.shape.begin(), b.shape.end());
      of.push_back(numel);
      b.o.out_off = numel;
      numel += int64_t(b.o.a) * b.o.b;
    }
  };
  lay(ub, P.u_q, P.u_sh, P.u_off, P.u_numel);
  lay(vb, P.v_q, P.v_sh, P.v_off, P.v_numel);
  P.outs.clear();
  for (auto &b : ub) P.outs.push_back(b.o);
  for (auto &b : vb) P.outs.push_back(b.o);
  // Charge tuples are compared as stored (normalised); ascending order.
  if (P.out_mem) {
    (void)hipFree(P.out_mem);
    P.out_mem = nullptr;
  }
  if (!P.outs.empty()) {
    if (hipMalloc(&P.out_mem, P.outs.size() * sizeof(DevSvdOut)) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(YASTN_ERR_NOMEM, "output table of the SVD");
    }
    SVD_HIP(hipMemcpyAsync(P.out_mem, P.outs.data(), P.outs.size() * sizeof(DevSvdOut), hipMemcpyHostToDevice, st));
    SVD_HIP(hipStreamSynchronize(st));
  }
  return YASTN_OK;
}

yastn_status yastn_svd_output(yastn_svd_t h, yastn_tensor_desc *u, int64_t *u_numel, yastn_tensor_desc *vt,
                              int64_t *vt_numel) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  SvdPlanImpl &P = h->p;
  if (!P.have_kept) return set_error(YASTN_ERR_STATE, "no yastn_svd result yet");
  const int ns = P.t.nsym;
  if (u) {
    u->rank = (int32_t)P.u_sig.size();
    u->nsym = ns;
    u->sym_mod = P.t.sym_mod;
    u->sig = P.u_sig.data();
    u->n = P.u_n.data();
    u->nblocks = (int64_t)P.u_off.size();
    u->charges = P.u_q.data();
    u->shapes = P.u_sh.data();
    u->offsets = P.u_off.data();
  }
  if (u_numel) *u_numel = P.u_numel;
  if (vt) {
    vt->rank = (int32_t)P.v_sig.size();
    vt->nsym = ns;
    vt->sym_mod = P.t.sym_mod;
    vt->sig = P.v_sig.data();
    vt->n = P.v_n.data();
    vt->nblocks = (int64_t)P.v_off.size();
    vt->charges = P.v_q.data();
    vt->shapes = P.v_sh.data();
    vt->offsets = P.v_off.data();
  }
  if (vt_numel) *vt_numel = P.v_numel;
  return YASTN_OK;
}

yastn_status yastn_svd_factors_scaled(yastn_svd_t h, void *u, void *vt, double pu, double pv, const void *workspace,
                                      void *hip_stream) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  SvdPlanImpl &P = h->p;
  if (!P.have_kept) return set_error(YASTN_ERR_STATE, "no yastn_svd result yet");
  if ((P.u_numel > 0 && !u) || (P.v_numel > 0 && !vt) || (!P.outs.empty() && !workspace))
    return set_error(YASTN_ERR_ARG, "null buffer");
  if (!std::isfinite(pu) || !std::isfinite(pv)) return set_error(YASTN_ERR_ARG, "powers must be finite");
  if (P.outs.empty()) return YASTN_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const char *ws = reinterpret_cast<const char *>(workspace);
  hipLaunchKernelGGL(k_svd_write, dim3(std::min<int>((int)P.outs.size(), 65535)), dim3(256), 0, st,
                     reinterpret_cast<const DevSvdOut *>(P.out_mem), (int)P.outs.size(),
                     reinterpret_cast<const double *>(ws), reinterpret_cast<const int32_t *>(ws + P.off_perm),
                     reinterpret_cast<const double *>(ws + P.off_sv_raw),
                     reinterpret_cast<const double *>(ws + P.off_sign), pu, pv, reinterpret_cast<double *>(u),
                     reinterpret_cast<double *>(vt));
  SVD_HIP(hipGetLastError());
  return YASTN_OK;
}

yastn_status yastn_svd_factors(yastn_svd_t h, void *u, void *vt, const void *workspace, void *hip_stream) {
  return yastn_svd_factors_scaled(h, u, vt, 0.0, 0.0, workspace, hip_stream);
}

void yastn_svd_free(yastn_svd_t h) {
  if (!h) return;
  if (h->p.dev_mem) (void)hipFree(h->p.dev_mem);
  if (h->p.out_mem) (void)hipFree(h->p.out_mem);
  delete h;
}

}  // extern "C"
