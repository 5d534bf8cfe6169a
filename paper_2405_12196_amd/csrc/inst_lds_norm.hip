// Template instances of the FP64 shared-B kernel (k_gemm_lds) that file the
// fused output norm.
#include "lds_select.hpp"

namespace yastn {

KernelFn lds_f64_norm(int shape, int cb, int kq, int na) { return lds_inst::lds_shape<true>(shape, cb, kq, na); }

}  // namespace yastn
