// Template instances of the FP64 kernels.
#include "dispatch.hpp"
#include "kernels.hpp"

namespace yastn {
namespace {
typedef double D;

template <int RB, int KB> KernelFn g4_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm4<D, D, D, true, RB, 1, KB>;
    case 2: return k_gemm4<D, D, D, true, RB, 2, KB>;
    case 3: return k_gemm4<D, D, D, true, RB, 3, KB>;
    default: return k_gemm4<D, D, D, true, RB, 4, KB>;
  }
}
template <int RB, int KQ, int NA, int PD, int OCC> KernelFn res_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_res<D, D, D, true, RB, 1, KQ, NA, PD, OCC>;
    case 2: return k_gemm_res<D, D, D, true, RB, 2, KQ, NA, PD, OCC>;
    case 3: return k_gemm_res<D, D, D, true, RB, 3, KQ, NA, PD, OCC>;
    default: return k_gemm_res<D, D, D, true, RB, 4, KQ, NA, PD, OCC>;
  }
}
template <int RB, int NA, int PD, int OCC> KernelFn res_kq(int kq, int cb) {
  if (kq <= 5) return res_cb<RB, 5, NA, PD, OCC>(cb);
  if (kq <= 10) return res_cb<RB, 10, NA, PD, OCC>(cb);
  if (kq <= 16) return res_cb<RB, 16, NA, PD, OCC>(cb);
  if constexpr (OCC == 1) {
    if (kq <= 20) return res_cb<RB, 20, NA, PD, OCC>(cb);
  }
  return nullptr;
}
template <int RB, int PD, int OCC> KernelFn res_na(int na, int kq, int cb) {
  return na <= 2 ? res_kq<RB, 2, PD, OCC>(kq, cb) : res_kq<RB, 4, PD, OCC>(kq, cb);
}
}  // namespace

KernelFn gemm4_f64(bool buf, int shape, int cb) {
  if (!buf) return k_gemm4<D, D, D, false, 4, 4, 2>;
  switch (shape) {
    case 1: return g4_cb<4, 1>(cb);
    case 2: return g4_cb<4, 4>(cb);
    case 3: return g4_cb<2, 2>(cb);
    case 4: return g4_cb<2, 4>(cb);
    case 5: return g4_cb<1, 4>(cb);
    default: return g4_cb<4, 2>(cb);
  }
}

KernelFn res_f64(bool buf, int shape, int cb, int kq, int na) {
  if (!buf) return nullptr;
  switch (shape) {  // kResShapes {rb, pd, occ}
    case 0: return res_na<1, 1, 3>(na, kq, cb);
    case 1: return res_na<2, 0, 3>(na, kq, cb);
    case 2: return res_na<1, 2, 3>(na, kq, cb);
    case 3: return res_na<2, 1, 3>(na, kq, cb);
    case 4: return res_na<1, 1, 4>(na, kq, cb);
    case 5: return res_na<1, 2, 2>(na, kq, cb);
    case 6: return res_na<1, 1, 2>(na, kq, cb);
    case 7: return res_na<2, 1, 2>(na, kq, cb);
    default: return res_na<1, 1, 1>(na, kq, cb);
  }
}

namespace {
template <int RB, int KB, int NA, int PD> KernelFn pf_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_pf<D, D, D, true, RB, 1, KB, NA, PD>;
    case 2: return k_gemm_pf<D, D, D, true, RB, 2, KB, NA, PD>;
    case 3: return k_gemm_pf<D, D, D, true, RB, 3, KB, NA, PD>;
    default: return k_gemm_pf<D, D, D, true, RB, 4, KB, NA, PD>;
  }
}
template <int RB, int KB, int PD> KernelFn pf_na(int na, int cb) {
  return na <= 2 ? pf_cb<RB, KB, 2, PD>(cb) : pf_cb<RB, KB, 4, PD>(cb);
}
}  // namespace

KernelFn pf_f64(bool buf, int shape, int cb, int na) {
  if (!buf) return nullptr;
  switch (shape) {  // kPfShapes {rb, kb, pd}
    case 1: return pf_na<2, 2, 3>(na, cb);
    case 2: return pf_na<4, 1, 3>(na, cb);
    default: return pf_na<2, 2, 2>(na, cb);
  }
}

ReduceFn split_reduce(yastn_precision precision, yastn_dtype out) {
  if (precision == YASTN_F64) return k_split_reduce<double, double>;
  return out == YASTN_DTYPE_F64 ? k_split_reduce<float, double> : k_split_reduce<float, float>;
}

KernelFn rows_f64(bool buf, int kmax) {
  if (!buf) return k_rows<D, D, D, false, 64>;
  if (kmax <= 16) return k_rows<D, D, D, true, 16>;
  if (kmax <= 32) return k_rows<D, D, D, true, 32>;
  if (kmax <= 48) return k_rows<D, D, D, true, 48>;
  return k_rows<D, D, D, true, 64>;
}

KernelFn pack_f64() { return k_pack_b<D, D>; }

}  // namespace yastn
