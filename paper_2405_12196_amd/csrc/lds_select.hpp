// Instance selection of the FP64 shared-B kernel (k_gemm_lds), included by
// the two translation units that instantiate it (without / with the fused
// norm), so the instances compile in parallel.
#pragma once
#include "dispatch.hpp"
#include "kernels.hpp"

namespace yastn {
namespace lds_inst {
typedef double D;
template <int RB, int KQ, int NA, int PD, int OCC, bool NORM, bool PAIR = false> KernelFn lds_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_lds<D, D, D, RB, 1, KQ, NA, PD, OCC, NORM, PAIR>;
    case 2: return k_gemm_lds<D, D, D, RB, 2, KQ, NA, PD, OCC, NORM, PAIR>;
    case 3: return k_gemm_lds<D, D, D, RB, 3, KQ, NA, PD, OCC, NORM, PAIR>;
    default: return k_gemm_lds<D, D, D, RB, 4, KQ, NA, PD, OCC, NORM, PAIR>;
  }
}
// paired-row loads: shape {rb 2, pd 0, occ 2}, K <= 40
template <bool NORM> KernelFn lds_pair(int cb, int kq, int na) {
  if (kq > 10) return nullptr;
  if (na <= 2) return kq <= 5 ? lds_cb<2, 5, 2, 0, 2, NORM, true>(cb) : lds_cb<2, 10, 2, 0, 2, NORM, true>(cb);
  return kq <= 5 ? lds_cb<2, 5, 4, 0, 2, NORM, true>(cb) : lds_cb<2, 10, 4, 0, 2, NORM, true>(cb);
}
template <int RB, int NA, int PD, int OCC, bool NORM> KernelFn lds_kq(int kq, int cb) {
  if (kq <= 5) return lds_cb<RB, 5, NA, PD, OCC, NORM>(cb);
  if (kq <= 10) return lds_cb<RB, 10, NA, PD, OCC, NORM>(cb);
  if (kq <= 16) return lds_cb<RB, 16, NA, PD, OCC, NORM>(cb);
  return lds_cb<RB, 20, NA, PD, OCC, NORM>(cb);
}
template <int RB, int PD, int OCC, bool NORM> KernelFn lds_na(int na, int kq, int cb) {
  return na <= 2 ? lds_kq<RB, 2, PD, OCC, NORM>(kq, cb) : lds_kq<RB, 4, PD, OCC, NORM>(kq, cb);
}
template <bool NORM> KernelFn lds_shape(int shape, int cb, int kq, int na) {
  if (kq > 20) return nullptr;
  switch (shape) {  // kLdsShapes {rb, pd, occ}
    case 1: return lds_na<1, 0, 3, NORM>(na, kq, cb);
    case 2: return lds_na<2, 0, 2, NORM>(na, kq, cb);
    case 3: return lds_pair<NORM>(cb, kq, na);
    default: return lds_na<1, 1, 2, NORM>(na, kq, cb);
  }
}
}  // namespace lds_inst
}  // namespace yastn
