// Address arithmetic of the pack and GEMM kernels, usable on host and device
// (the host build lets the indexing be exercised on the CPU).  See plan.hpp
// for the factorisation of A offsets.
#pragma once
#include <cstdint>

#include "plan.hpp"

#ifndef __HIPCC__
#define YASTN_HD inline
#else
#include <hip/hip_runtime.h>
#define YASTN_HD __host__ __device__ __forceinline__
#endif

namespace yastn {

// RG_a(ra) for a = 0..kMaxAct-1 (zero past nact)
// (fixed trip count, so the array stays in registers)
YASTN_HD void a_rowparts(const DevRowTuple &rt, int nact, int32_t ra, int32_t *rg) {
#pragma unroll
  for (int a = 0; a < kMaxAct; ++a) rg[a] = a < nact ? (ra % rt.lsuf[a]) - (ra % rt.lsuf[a + 1]) : 0;
}

// The same RG_a with one multiply-high division per class boundary instead of
// two modulo operations per class: RG_a = (r mod Lsuf_a) - (r mod Lsuf_{a+1}),
// r mod Lsuf_0 = r (rows of a tuple are below Lsuf_0 = m_i), Lsuf_nact = 1.
// U24: the row count of the tuple is below 2^24 (so are the quotient and
// Lsuf), and the device multiplies them at full rate in 24 bits.
template <int NA, bool U24 = false>
YASTN_HD void a_rowparts_fast(const DevRowTuple &rt, int nact, int32_t ra, int32_t *rg) {
  int32_t prev = ra;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    int32_t next = 0;
    if (a + 1 < nact) {
      const uint32_t q = (uint32_t)(((uint64_t)(uint32_t)ra * rt.lmag[a + 1]) >> rt.lsh[a + 1]);
#if defined(__HIP_DEVICE_COMPILE__)
      if constexpr (U24)
        next = ra - (int32_t)__umul24(q, (uint32_t)rt.lsuf[a + 1]);
      else
        next = ra - (int32_t)q * rt.lsuf[a + 1];
#else
      next = ra - (int32_t)q * rt.lsuf[a + 1];
#endif
    }
    rg[a] = a < nact ? prev - next : 0;
    prev = next;
  }
}

// Magic multiplier for floor(n / d), 0 <= n < 2^31, 1 <= d < 2^31 (round-up
// method: l = ceil(log2 d), m = ceil(2^(31 + l) / d) < 2^32).
inline void div_magic(uint32_t d, uint32_t *mag, int32_t *sh) {
  int l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  *sh = 31 + l;
  *mag = (uint32_t)(((uint64_t(1) << (31 + l)) + d - 1) / d);
}

// Same sum in the offset type of the kernel (32-bit when buffers are small).
template <typename Off>
YASTN_HD Off a_offset_t(int64_t koff, const int32_t *p, const int32_t *rg) {
  Off o = (Off)koff;
  for (int a = 0; a < kMaxAct; ++a) o += (Off)p[a] * (Off)rg[a];
  return o;
}

YASTN_HD int64_t a_offset(int64_t koff, const int32_t *p, const int32_t *rg) {
  int64_t o = koff;
  for (int a = 0; a < kMaxAct; ++a) o += (int64_t)p[a] * rg[a];
  return o;
}

// Source offset in B of element (kd, cb) of block bb (contracted tuple ct,
// column tuple cl).
// (fixed trip counts, so the dims and strides stay in registers)
YASTN_HD int64_t b_offset(const DevBBlock &bb, const DevCtrTuple &ct, const DevColTuple &cl, const DevProb &pr,
                          int32_t kd, int32_t cb) {
  int64_t o = bb.off;
  int32_t r = cb;
#pragma unroll
  for (int q = kMaxRank - 1; q >= 0; --q)
    if (q < pr.nfb) {
      const int32_t d = cl.dims[q];
      o += (int64_t)(r % d) * bb.sf[q];
      r /= d;
    }
  r = kd;
#pragma unroll
  for (int c = kMaxRank - 1; c >= 0; --c)
    if (c < pr.nc) {
      const int32_t d = ct.dims[c];
      o += (int64_t)(r % d) * bb.sc[c];
      r /= d;
    }
  return o;
}

}  // namespace yastn
