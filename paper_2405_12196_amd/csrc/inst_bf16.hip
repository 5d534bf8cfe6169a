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
}  // namespace

KernelFn bf16_gemm(yastn_dtype in, yastn_dtype out, int nt, bool buf, int cb) {
  if (in == YASTN_DTYPE_F64)
    return out == YASTN_DTYPE_F64 ? pick_nt<double, double>(nt, buf, cb) : pick_nt<double, float>(nt, buf, cb);
  return out == YASTN_DTYPE_F64 ? pick_nt<float, double>(nt, buf, cb) : pick_nt<float, float>(nt, buf, cb);
}

}  // namespace yastn
