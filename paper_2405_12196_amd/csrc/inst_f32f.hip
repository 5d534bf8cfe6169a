// Template instances of the FP32-arithmetic kernels with FP32 input buffers.
#include "dispatch.hpp"
#include "kernels.hpp"

namespace yastn {
namespace {
typedef float In;
typedef float F;

template <typename Out, int RB, int KB> KernelFn g4_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm4<In, F, Out, true, RB, 1, KB>;
    case 2: return k_gemm4<In, F, Out, true, RB, 2, KB>;
    case 3: return k_gemm4<In, F, Out, true, RB, 3, KB>;
    default: return k_gemm4<In, F, Out, true, RB, 4, KB>;
  }
}
template <typename Out> KernelFn g4(bool buf, int shape, int cb) {
  if (!buf) return k_gemm4<In, F, Out, false, 4, 4, 2>;
  if (shape == 3 || shape == 4 || shape == 5) return g4_cb<Out, 2, 4>(cb);
  return g4_cb<Out, 4, 2>(cb);
}
template <typename Out, int KQ> KernelFn res_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_res<In, F, Out, true, 2, 1, KQ, 4, 0, 3>;
    case 2: return k_gemm_res<In, F, Out, true, 2, 2, KQ, 4, 0, 3>;
    case 3: return k_gemm_res<In, F, Out, true, 2, 3, KQ, 4, 0, 3>;
    default: return k_gemm_res<In, F, Out, true, 2, 4, KQ, 4, 0, 3>;
  }
}
template <typename Out> KernelFn res(bool buf, int cb, int kq) {
  if (!buf) return nullptr;
  if (kq <= 5) return res_cb<Out, 5>(cb);
  if (kq <= 10) return res_cb<Out, 10>(cb);
  if (kq <= 16) return res_cb<Out, 16>(cb);
  return nullptr;
}
template <typename Out> KernelFn rows(bool buf, int kmax) {
  if (!buf) return k_rows<In, F, Out, false, 64>;
  if (kmax <= 16) return k_rows<In, F, Out, true, 16>;
  if (kmax <= 32) return k_rows<In, F, Out, true, 32>;
  if (kmax <= 48) return k_rows<In, F, Out, true, 48>;
  return k_rows<In, F, Out, true, 64>;
}
template <typename Out> KernelFn pf(bool buf, int cb) {
  if (!buf) return nullptr;
  switch (cb) {
    case 1: return k_gemm_pf<In, F, Out, true, 2, 1, 2, 4, 2>;
    case 2: return k_gemm_pf<In, F, Out, true, 2, 2, 2, 4, 2>;
    case 3: return k_gemm_pf<In, F, Out, true, 2, 3, 2, 4, 2>;
    default: return k_gemm_pf<In, F, Out, true, 2, 4, 2, 4, 2>;
  }
}
// shared-B tiles: one shape (rows per chunk 32, no chunk prefetch, 2+ waves per SIMD)
template <typename Out, int KQ, bool NORM> KernelFn lds_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_lds<In, F, Out, 2, 1, KQ, 4, 0, 2, NORM>;
    case 2: return k_gemm_lds<In, F, Out, 2, 2, KQ, 4, 0, 2, NORM>;
    case 3: return k_gemm_lds<In, F, Out, 2, 3, KQ, 4, 0, 2, NORM>;
    default: return k_gemm_lds<In, F, Out, 2, 4, KQ, 4, 0, 2, NORM>;
  }
}
template <typename Out, bool NORM> KernelFn lds(int cb, int kq) {
  if (kq <= 5) return lds_cb<Out, 5, NORM>(cb);
  if (kq <= 10) return lds_cb<Out, 10, NORM>(cb);
  if (kq <= 16) return lds_cb<Out, 16, NORM>(cb);
  if (kq <= 20) return lds_cb<Out, 20, NORM>(cb);
  return nullptr;
}
}  // namespace

KernelFn lds_f32f(yastn_dtype out, int cb, int kq, bool norm) {
  if (out == YASTN_DTYPE_F64) return norm ? lds<double, true>(cb, kq) : lds<double, false>(cb, kq);
  return norm ? lds<float, true>(cb, kq) : lds<float, false>(cb, kq);
}
KernelFn pf_f32f(yastn_dtype out, bool buf, int cb) {
  return out == YASTN_DTYPE_F64 ? pf<double>(buf, cb) : pf<float>(buf, cb);
}
KernelFn gemm4_f32f(yastn_dtype out, bool buf, int shape, int cb) {
  return out == YASTN_DTYPE_F64 ? g4<double>(buf, shape, cb) : g4<float>(buf, shape, cb);
}
KernelFn res_f32f(yastn_dtype out, bool buf, int cb, int kq) {
  return out == YASTN_DTYPE_F64 ? res<double>(buf, cb, kq) : res<float>(buf, cb, kq);
}
KernelFn rows_f32f(yastn_dtype out, bool buf, int kmax) {
  return out == YASTN_DTYPE_F64 ? rows<double>(buf, kmax) : rows<float>(buf, kmax);
}
KernelFn pack_f32f() { return k_pack_b<In, F>; }

}  // namespace yastn
