// Template instances of the K-chunked shared-B kernel (k_gemm_ldsk), FP64:
// tiles of 32 rows, 1-4 column blocks, 32 k per chunk, with and without the
// fused norm.
#include "dispatch.hpp"
#include "kernels.hpp"

namespace yastn {
namespace {
typedef double D;
template <int NA, bool NORM> KernelFn ldsk_cb(int cb) {
  switch (cb) {
    case 1: return k_gemm_ldsk<D, D, D, kLdskRb, 1, kLdskKq, NA, 2, NORM>;
    case 2: return k_gemm_ldsk<D, D, D, kLdskRb, 2, kLdskKq, NA, 2, NORM>;
    case 3: return k_gemm_ldsk<D, D, D, kLdskRb, 3, kLdskKq, NA, 2, NORM>;
    case 4: return k_gemm_ldsk<D, D, D, kLdskRb, 4, kLdskKq, NA, 2, NORM>;
    default: return nullptr;
  }
}
}  // namespace

KernelFn ldsk_f64(int cb, int na, bool norm) {
  if (norm) return na <= 2 ? ldsk_cb<2, true>(cb) : ldsk_cb<4, true>(cb);
  return na <= 2 ? ldsk_cb<2, false>(cb) : ldsk_cb<4, false>(cb);
}

}  // namespace yastn
