// Kernel selection: which template instance of kernels.hpp runs a launch.
// Each arithmetic's instances live in their own translation unit
// (inst_f64.hip, inst_f32d.hip, inst_f32f.hip, inst_bf16.hip).
#pragma once
#include "../../include/yastn.h"
#include "plan.hpp"

namespace yastn {

typedef void (*KernelFn)(LaunchArgs);
typedef void (*ReduceFn)(RedArgs);

// the split-K reduction of an arithmetic (FP64, or FP32 accumulators) into out
ReduceFn split_reduce(yastn_precision precision, yastn_dtype out);

// k_gemm4 tile shapes: rows per chunk = 16 * rb, k-steps per load batch = kb.
struct Shape {
  int rb, kb;
};
constexpr Shape kMfmaShapes[] = {{4, 2}, {4, 1}, {4, 4}, {2, 2}, {2, 4}, {1, 4}};
constexpr int kNumMfma = sizeof(kMfmaShapes) / sizeof(Shape);
// k_gemm_res: rows per chunk = 16 * rb, A loads issued pd chunks ahead of the
// MFMAs (a ring of pd + 1 register buffers), occupancy hint (occ waves per
// SIMD); k slots held = 4 * kq.  A higher occupancy hint caps the registers
// per wave, and wide tiles (more columns, more k slots, deeper rings) then
// spill to scratch; the autotuner measures the trade.  Occupancy 1 leaves the
// register file to one wave per SIMD and also takes K up to 80.
struct ResShape {
  int rb, pd, occ;
};
constexpr ResShape kResShapes[] = {{1, 1, 3}, {2, 0, 3}, {1, 2, 3}, {2, 1, 3}, {1, 1, 4},
                                   {1, 2, 2}, {1, 1, 2}, {2, 1, 2}, {1, 1, 1}};
constexpr int kNumRes = sizeof(kResShapes) / sizeof(ResShape);
constexpr int kResKq[] = {5, 10, 16, 20};
// k_gemm_pf: rows per chunk = 16 * rb, k-steps per pipelined batch = kb,
// operand loads issued pd batches ahead of the MFMAs
struct PfShape {
  int rb, kb, pd;
};
constexpr PfShape kPfShapes[] = {{2, 2, 2}, {2, 2, 3}, {4, 1, 3}};
constexpr int kNumPf = sizeof(kPfShapes) / sizeof(PfShape);
// k_gemm_lds: rows per chunk = 16 * rb, A loads pd chunks ahead, occupancy
// hint occ; K <= 80.  The fourth shape loads rows in adjacent pairs (FP64,
// K <= 40, plans whose row tuples allow it: Plan::pair_ok).
struct LdsShape {
  int rb, pd, occ;
};
constexpr LdsShape kLdsShapes[] = {{1, 1, 2}, {1, 0, 3}, {2, 0, 2}, {2, 0, 2}};
constexpr int kLdsPairShape = 3;
constexpr int kPairMaxK = 40;
constexpr int kNumLds = sizeof(kLdsShapes) / sizeof(LdsShape);
// k_gemm_ldsk: the shared-B jobs with K in chunks of 4 * kLdskKq, tiles of
// at most 16 * kLdskRb rows (any K; FP64)
constexpr int kLdskRb = 2;
constexpr int kLdskKq = 8;
constexpr int kResMaxK = 64;      // K limit of the shapes with occ > 1
constexpr int kResMaxKWide = 80;  // K limit of the occupancy-1 shape
constexpr int res_max_k(int shape) { return kResShapes[shape].occ == 1 ? kResMaxKWide : kResMaxK; }

// FP64 arithmetic (F64 buffers)
KernelFn gemm4_f64(bool buf, int shape, int cb);
KernelFn res_f64(bool buf, int shape, int cb, int kq, int na);
KernelFn rows_f64(bool buf, int kmax);
KernelFn pf_f64(bool buf, int shape, int cb, int na);
KernelFn pack_f64();
KernelFn lds_f64(int shape, int cb, int kq, int na, bool norm);  // kq <= 20; norm: files the fused norm
KernelFn lds_f64_norm(int shape, int cb, int kq, int na);
KernelFn ldsk_f64(int cb, int na, bool norm);  // cb <= 4; norm: files the fused norm
// FP32 arithmetic with FP64 input buffers (out: F64 or F32)
KernelFn gemm4_f32d(yastn_dtype out, bool buf, int shape, int cb);
KernelFn res_f32d(yastn_dtype out, bool buf, int cb, int kq);
KernelFn rows_f32d(yastn_dtype out, bool buf, int kmax);
KernelFn pf_f32d(yastn_dtype out, bool buf, int cb);
KernelFn pack_f32d();
KernelFn lds_f32d(yastn_dtype out, int cb, int kq, bool norm);  // shape kLdsShapes[2], kq <= 20
// FP32 arithmetic with FP32 input buffers
KernelFn gemm4_f32f(yastn_dtype out, bool buf, int shape, int cb);
KernelFn res_f32f(yastn_dtype out, bool buf, int cb, int kq);
KernelFn rows_f32f(yastn_dtype out, bool buf, int kmax);
KernelFn pf_f32f(yastn_dtype out, bool buf, int cb);
KernelFn pack_f32f();
KernelFn lds_f32f(yastn_dtype out, int cb, int kq, bool norm);  // shape kLdsShapes[2], kq <= 20
// split-BF16 products (nt = 3 or 6), FP32 accumulation
KernelFn bf16_gemm(yastn_dtype in, yastn_dtype out, int nt, bool buf, int cb);
// split-BF16 register-resident tiles, FP32 operand buffers, K <= 64 (nullptr otherwise)
KernelFn res_bf16(yastn_dtype out, int nt, int cb, int kq, int na);

}  // namespace yastn
