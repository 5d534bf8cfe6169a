// Internal plan layout shared by the host planner (host.cpp) and the HIP
// kernels (device.hip).  Plain structs of fixed-width fields so host and
// device agree on the layout.
//
// Vocabulary (paper Sec. II.B, contraction identity sum_X A_IX B_XJ):
//   sector X      fused contracted charge, X = sum over A's contracted legs of
//                 s_i rho_i; one dense GEMM C_X = A_X B_X per sector;
//   row tuple i   charges on A's free legs (one block-row of A_X / C_X);
//   ctr tuple s   charges on the contracted legs (one block-column of A_X);
//   col tuple j   charges on B's free legs (one block-column of B_X / C_X).
// Output block (i, j) is a C-order array of m_i x n_j elements (A's free legs
// first, then B's), so the sub-block (i, j) of C_X *is* an output block.
//
// A-operand address factorisation.  For A block (i, s) with legs in storage
// order, the offset of element (row ra, contracted index kd) is
//     sum_f x_f(ra) * stride_f  +  sum_c y_c(kd) * stride_c,
// stride_l = product of the dims of the legs after l.  Group the free legs by
// how many contracted legs follow them ("class" g); legs of one class are
// contiguous and the class index falls along storage order.  Then
//     sum_f x_f stride_f = sum_a P_a(s) * RG_a(ra),
//     RG_a(ra) = (ra mod Lsuf_a) - (ra mod Lsuf_{a+1}),
// with Lsuf_a = product of the free dims of classes a..end (Lsuf_0 = m_i,
// Lsuf_nact = 1) and P_a(s) = product of the dims of the last g_a contracted
// legs (1 for g_a = 0).  The contracted part is
//     sum_c y_c(kd) * FAc_c(i) * CAc_c(s),
// FAc_c = product of free dims after leg c, CAc_c = product of contracted
// dims after leg c.  So every element costs nact multiply-adds on top of a
// per-(row tuple, k) offset table the plan builds once (kofs).
#pragma once
#include <cstdint>

namespace yastn {

constexpr int kMaxRank = 8;
constexpr int kMaxAct = 4;     // free-leg classes of A (<= min(#free, #contracted + 1))
constexpr int kMaxJobs = 32;   // plans per launch
constexpr int kMaxProbs = 64;  // problems per launch with the pointer triples in kernel args
constexpr int kMaxTableProbs = 1 << 16;  // problems per launch group with a device pointer table
constexpr int kPackItem = 256; // packed-B elements per sub-block pack work item
constexpr int kGatherItem = 2048;  // packed-B elements per gather pack work item (8 per thread)

struct DevProb {               // one problem of a plan
  int32_t nact;                // active free-leg classes of A
  int32_t nc;                  // contracted legs
  int32_t nfb;                 // free legs of B
  int32_t pad;
  int64_t a_span;              // elements of A's buffer that blocks reach (max offset + size)
  int64_t c_numel;             // elements of C
  int64_t b_span;              // elements of B's buffer that blocks reach
};

struct DevSector {             // one (problem, sector)
  int32_t prob;
  int32_t S, Q;                // contracted tuples, col tuples
  int32_t K, N;                // K_X, N_X
  int32_t ctr0, col0;          // first ctr tuple / col tuple (plan-global index)
  int32_t nact;                // active free-leg classes of A (copy of the problem's)
  int64_t bpack;               // element offset of packed B_X (K_X x N_X, row-major) in workspace
  int64_t kp0;                 // first of K_X entries in kp (P_a of each contracted index)
  int64_t cm0;                 // first of N_X entries in colmap
  int64_t bofs0;               // first of K_X * N_X entries in bofs
};

struct DevRowTuple {           // one (problem, sector, A free tuple)
  int32_t sector;              // plan-global sector index
  int32_t m;                   // rows
  int64_t agrid;               // first of S entries in agrid (A block or -1)
  int64_t cgrid;               // first of Q entries in cgrid (C element offset or -1)
  int64_t kofs;                // first of K_X entries in kofs (A offset of (row 0, k), -1 absent)
  int32_t lsuf[kMaxAct + 1];   // Lsuf_a, a = 0..nact
  uint32_t lmag[kMaxAct + 1];  // floor(r / Lsuf_a) = (r * lmag_a) >> lsh_a for 0 <= r < 2^31
  int32_t lsh[kMaxAct + 1];
  int32_t fac[kMaxRank];       // FAc_c, contracted legs in axes order
};

struct DevColMap {             // one column of a sector's C_X / B_X
  int32_t j;                   // column tuple (sector-local)
  int32_t cl;                  // column within the tuple
  int32_t nj;                  // n_j
  int32_t pad;
};

// One column of a sector's C_X with the output block of one row tuple
// resolved (the column map and the row tuple's output block offsets in one
// 16-byte entry, so a tile's columns take one load instead of two dependent
// ones).
struct alignas(16) DevColRes {
  int32_t cbase;               // C element offset of output block (i, j), -1 if absent
  int32_t nj;                  // n_j
  int32_t cl;                  // column within tuple j
  int32_t pad;
};

struct DevKP {                 // P_a of one contracted index
  int32_t p[kMaxAct];
};

struct DevCtrTuple {           // one (problem, sector, contracted tuple)
  int32_t k, ko;               // k_s and its first index in the sector's K space
  int32_t dims[kMaxRank];      // contracted dims in axes order
  int32_t cac[kMaxRank];       // CAc_c in axes order
  int32_t p[kMaxAct];          // P_a
};

struct DevColTuple {           // one (problem, sector, B free tuple)
  int32_t n, no;               // n_j and its first column in the sector
  int32_t dims[kMaxRank];      // B free dims (B storage order)
};

struct DevBBlock {             // one B block, strides for the pack kernel
  int64_t off;
  int32_t sc[kMaxRank];        // strides of contracted legs (axes order)
  int32_t sf[kMaxRank];        // strides of free legs (storage order)
};

struct DevTile {               // one wave tile: rows [m0, m0 + nrows) of a row tuple, in chunks
  int32_t rowtuple;            // plan-global row tuple
  int32_t sector;              // its sector (saves a dependent load)
  int32_t m0;                  // first row within the row tuple
  int32_t n0;                  // first column within the sector
  int32_t nrows;               // rows (a multiple of the chunk height except at the tuple's end)
  int32_t ncols;               // columns (<= 16 * column blocks of the kernel)
  int32_t k0, kn;              // k range [k0, k0 + kn) of the sector (all of K unless split)
  int32_t red;                 // split-K group (index into the plan's groups) or -1
  int32_t part;                // this tile's partial slot within its split-K group
};

// A split-K group: the k ranges of one output tile, computed by separate
// tiles into partial slots of the workspace and summed in slot order into C.
struct DevRedItem {
  const DevColMap *cmap;       // the sector's column map, from the tile's first column
  const int64_t *cgrid;        // the row tuple's output block offsets
  int64_t off0;                // workspace byte offset of slot 0
  int64_t slot_bytes;          // bytes of one slot (nrows x 64 accumulators)
  int32_t prob, m0, nrows, ncols, nslots, pad;
};

// Everything one wave needs to start a tile, in one record of absolute
// addresses read with a few scalar loads (no chain of dependent table reads).
// Built at upload time, when the tables' device addresses are known.
constexpr int kRecAct = 3;     // class boundaries a record carries (nact <= kRecAct + 1)
struct DevTileRec {
  const int64_t *kofs;         // the row tuple's A offsets of (row 0, k), K_X entries
  const DevKP *kp;             // the sector's class factors, K_X entries
  const int32_t *bofs;         // the sector's B offsets, K_X x N_X row-major
  const DevColMap *cmap;       // the sector's column map, from column n0
  const int64_t *cgrid;        // the row tuple's output block offsets, Q_X entries
  int64_t a_span, b_span, c_numel;  // element bounds of the problem's buffers
  int32_t m0, nrows, n0, ncols;
  int32_t K, N, nact, prob;    // prob: plan-local problem index
  int32_t lsuf[kRecAct];       // Lsuf_1 .. Lsuf_kRecAct of the row tuple
  int32_t lsh[kRecAct];
  uint32_t lmag[kRecAct];
  int32_t split;               // 1: a split-K tile, accumulators go to its partial slot; 0: to C
  int64_t bpack;               // the sector's packed B_X from k0 on, in the workspace (elements)
  int64_t part;                // split-K tiles: workspace byte offset of the partial slot
  const struct DevColRes *colres;  // the tile's columns from n0, output blocks resolved for its
                                   // row tuple (plans whose buffers fit 32-bit offsets; else null)
};
static_assert(sizeof(DevTileRec) == 160, "tile record layout");

// One pack work item, in one of two forms.
//  s >= 0: up to kPackItem elements of the (sector, s, j) sub-block of packed
//          B_X, B offsets computed from the block's strides;
//  s <  0: a gather of j (<= kGatherItem) consecutive elements of packed B_X
//          starting at e0, the B offset of each read from the bofs table (used
//          when every offset of the sector fits int32 and K_X * N_X does too).
struct DevPackItem {
  int32_t sector;
  int32_t s, j;
  int32_t bblk;                // B block (plan-global) or -1 (absent: zeros); unused by gathers
  int32_t e0;                  // first element (row-major over k_s x n_j, or over K_X x N_X)
  int32_t pad;
};

struct DevPlan {               // device-resident table of the plan's arrays
  const DevProb *probs;
  const DevSector *sectors;
  const DevRowTuple *rows;
  const DevCtrTuple *ctrs;
  const DevColTuple *cols;
  const int32_t *agrid;        // A block (plan-global) or -1
  const int64_t *aoff;         // element offset of each A block (plan-global)
  const int64_t *cgrid;        // C element offset or -1
  const DevBBlock *bblocks;
  const DevTile *tiles;
  const DevPackItem *items;
  const int64_t *kofs;         // per row tuple, per contracted index
  const DevKP *kp;             // per sector, per contracted index
  const DevColMap *colmap;     // per sector, per column
  const int32_t *bofs;         // per sector, K_X x N_X row-major: element offset in B's buffer, -1 absent
  const DevTileRec *recs;      // per tile (same order as tiles)
  int32_t ntiles, nitems;
};

// A shared-B workgroup job: wave tiles of one (sector, column range) of one
// problem (plan-local tile indices; -1 = none, t[0] always a tile).  Wave w of
// the workgroup computes t[w], t[w + 4], ...
// The B tile's fields (those of the first tile's record) are copied in at
// upload, so the B loads start one dependent read earlier.
constexpr int kLdsJobTiles = 4;
static_assert(kLdsJobTiles % 4 == 0, "four waves per job");
struct DevLdsJob {
  int32_t t[kLdsJobTiles];
  const int32_t *bofs;         // the sector's B offsets from the tiles' k0, K x N row-major
  int64_t b_span;              // element bound of the problem's B buffer
  int32_t K, N, n0, prob;      // the tiles' K range length, N_X, first column, plan-local problem
};

struct ProbPtrs {
  const void *a, *b;
  void *c;
};

struct JobArg {                // a range of one plan's problems inside a launch
  const DevPlan *plan;
  const DevTileRec *recs;      // the plan's tile records (device)
  const DevLdsJob *ljobs;      // the plan's shared-B jobs (device)
  const DevTileRec *ljrecs;    // the records of those jobs' tiles, kLdsJobTiles per job in
                               // slot order (an empty slot: a copy of slot 0 with no rows)
  char *ws;                    // job workspace (packed B)
  int32_t tile0, item0;        // first launch-global tile (shared-B job) / pack item of this job
  int32_t ptile0, pitem0;      // first plan-local tile (shared-B job) / pack item of this job
  int32_t prob0;               // entry of LaunchArgs::p for the plan's problem plo
  int32_t plo;                 // first plan problem covered by this job
};

// Norm of the output fused into the GEMM epilogue (single-problem launches):
// every tile writes its sum of squares and max |x| to parts[tile].
struct NormArgs {
  double *parts;               // [ntiles][2] in the workspace, null = no norm
};

// Problem pointers: p[] in the kernel arguments, or (a launch of one group of
// more than kMaxProbs problems) the table ptab in the job's workspace, written
// by k_put_ptrs before the launch.
struct LaunchArgs {
  int32_t njobs, ntiles, nitems, pad;
  NormArgs norm;
  const ProbPtrs *ptab;
  JobArg jobs[kMaxJobs];
  ProbPtrs p[kMaxProbs];
};
static_assert(sizeof(LaunchArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// The split-K reduction of one job: its groups' slots summed into C.
struct RedArgs {
  const DevRedItem *items;
  int32_t nitems, plo;         // plo: plan problem of p[0]
  const char *ws;
  const ProbPtrs *ptab;        // as LaunchArgs::ptab
  ProbPtrs p[kMaxProbs];
};

// One chunk of a device pointer table, written by k_put_ptrs.
constexpr int kPtrChunk = 160;
struct PtrChunk {
  ProbPtrs *dst;
  int32_t n, pad;
  ProbPtrs p[kPtrChunk];
};
static_assert(sizeof(PtrChunk) <= 4096, "kernel arguments are limited to 4 KiB");
static_assert(sizeof(RedArgs) <= 4096, "kernel arguments are limited to 4 KiB");

}  // namespace yastn
