// Template instances of the split-BF16 kernels.
#include "dispatch.hpp"
#include "kernels.hpp"

namespace yastn {
namespace {
template <typename In, typename Out, int NT> KernelFn pick(bool buf, int cb) {
  if (!buf) return k_gemm_bf16<In, Out, false, 4, 4, NT>;
  switch (cb) {
    case 1: return k_gemm_bf16<In, Out, true, 4, 1, NT>;
    case 2: return k_gemm_bf16<In, Out, true, 4, 2, NT>;
    case 3: return k_gemm_bf16<In, Out, true, 4, 3, NT>;
    default: return k_gemm_bf16<In, Out, true, 4, 4, NT>;
  }
}
template <typename In, typename Out> KernelFn pick_nt(int nt, bool buf, int cb) {
  return nt == 3 ? pick<In, Out, 3>(buf, cb) : pick<In, Out, 6>(buf, cb);
}
// register-resident tiles with split-BF16 products (FP32 operand buffers):
// 16 rows per chunk, one chunk of A loads ahead, occupancy 2 (1 for K > 32)
template <typename Out, int NT, int KQ, int NA> KernelFn res_cb(int cb) {
  constexpr int OCC = KQ > 8 ? 1 : 2;
  switch (cb) {
    case 1: return k_gemm_res<float, float, Out, true, 1, 1, KQ, NA, 1, OCC, NT>;
    case 2: return k_gemm_res<float, float, Out, true, 1, 2, KQ, NA, 1, OCC, NT>;
    case 3: return k_gemm_res<float, float, Out, true, 1, 3, KQ, NA, 1, OCC, NT>;
    default: return k_gemm_res<float, float, Out, true, 1, 4, KQ, NA, 1, OCC, NT>;
  }
}
template <typename Out, int NT> KernelFn res_kq(int kq, int na, int cb) {
  if (kq <= 8) return na <= 2 ? res_cb<Out, NT, 8, 2>(cb) : res_cb<Out, NT, 8, 4>(cb);
  if (kq <= 16) return na <= 2 ? res_cb<Out, NT, 16, 2>(cb) : res_cb<Out, NT, 16, 4>(cb);
  return nullptr;
}
}  // namespace

KernelFn res_bf16(yastn_dtype out, int nt, int cb, int kq, int na) {
  if (out == YASTN_DTYPE_F64) return nt == 3 ? res_kq<double, 3>(kq, na, cb) : res_kq<double, 6>(kq, na, cb);
  return nt == 3 ? res_kq<float, 3>(kq, na, cb) : res_kq<float, 6>(kq, na, cb);
}

KernelFn bf16_gemm(yastn_dtype in, yastn_dtype out, int nt, bool buf, int cb) {
  if (in == YASTN_DTYPE_F64)
    return out == YASTN_DTYPE_F64 ? pick_nt<double, double>(nt, buf, cb) : pick_nt<double, float>(nt, buf, cb);
  return out == YASTN_DTYPE_F64 ? pick_nt<float, double>(nt, buf, cb) : pick_nt<float, float>(nt, buf, cb);
}

}  // namespace yastn
