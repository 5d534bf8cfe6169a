// Template instances of the FP64 shared-B kernel (k_gemm_lds) without the
// fused norm, and the selection between the two instance sets.
#include "lds_select.hpp"

namespace yastn {

KernelFn lds_f64(int shape, int cb, int kq, int na, bool norm) {
  return norm ? lds_f64_norm(shape, cb, kq, na) : lds_inst::lds_shape<false>(shape, cb, kq, na);
}

}  // namespace yastn
