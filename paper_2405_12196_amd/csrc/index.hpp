// Address arithmetic of the pack and GEMM kernels, usable on host and device
// (the host build lets the indexing be exercised on the CPU).  See plan.hpp
// for the factorisation of A offsets.
#pragma once
#include <cstdint>

#include "plan.hpp"

#ifndef __HIPCC__
#define YASTN_HD inline
#else
#define YASTN_HD __host__ __device__ __forceinline__
#endif

namespace yastn {

// last contracted tuple s of a sector with ko_s <= k
YASTN_HD int find_ctr(const DevCtrTuple *ct, int S, int k) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ct[mid].ko <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// last column tuple j of a sector with no_j <= c
YASTN_HD int find_col(const DevColTuple *cl, int Q, int c) {
  int lo = 0, hi = Q - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cl[mid].no <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Offset of A(row 0, contracted index k) of row tuple rt, or -1 when the block
// (rt, tuple of k) is absent; fills P_a of k's tuple.
YASTN_HD int64_t a_koffset(const DevPlan &P, const DevRowTuple &rt, const DevSector &sec, const DevProb &pr, int k,
                           int32_t *p_out) {
  const DevCtrTuple *ctrs = P.ctrs + sec.ctr0;
  const int s = find_ctr(ctrs, sec.S, k);
  const DevCtrTuple &ct = ctrs[s];
  for (int a = 0; a < kMaxAct; ++a) p_out[a] = ct.p[a];
  const int32_t blk = P.agrid[rt.agrid + s];
  if (blk < 0) return -1;
  int64_t r = k - ct.ko, koff = 0;
  for (int c = pr.nc - 1; c >= 0; --c) {
    const int64_t d = ct.dims[c];
    koff += (r % d) * (int64_t)rt.fac[c] * ct.cac[c];
    r /= d;
  }
  return P.aoff[blk] + koff;
}

// RG_a(ra) for a = 0..kMaxAct-1 (zero past nact)
YASTN_HD void a_rowparts(const DevRowTuple &rt, int nact, int32_t ra, int32_t *rg) {
  for (int a = 0; a < kMaxAct; ++a) rg[a] = 0;
  for (int a = 0; a < nact; ++a) rg[a] = (ra % rt.lsuf[a]) - (ra % rt.lsuf[a + 1]);
}

YASTN_HD int64_t a_offset(int64_t koff, const int32_t *p, const int32_t *rg) {
  int64_t o = koff;
  for (int a = 0; a < kMaxAct; ++a) o += (int64_t)p[a] * rg[a];
  return o;
}

// Source offset in B of element (kd, cb) of block bb (contracted tuple ct,
// column tuple cl).
YASTN_HD int64_t b_offset(const DevBBlock &bb, const DevCtrTuple &ct, const DevColTuple &cl, const DevProb &pr,
                          int64_t kd, int64_t cb) {
  int64_t o = bb.off, r = cb;
  for (int q = pr.nfb - 1; q >= 0; --q) {
    const int64_t d = cl.dims[q];
    o += (r % d) * bb.sf[q];
    r /= d;
  }
  r = kd;
  for (int c = pr.nc - 1; c >= 0; --c) {
    const int64_t d = ct.dims[c];
    o += (r % d) * bb.sc[c];
    r /= d;
  }
  return o;
}

}  // namespace yastn
