// One CTM move on the device: the left move of the corner-transfer-matrix
// method for a 1x1 unit cell (paper Sec. III, Fig. 3: enlarged corners from
// the environment and the site tensors, the SVD of the product of four of
// them, projections back to chi).  gfx950, FP64 throughout.
//
// The move is a DAG of 28 block-sparse contractions, one truncated SVD and
// three normalisations.  Contractions that do not depend on each other run
// in one grouped launch (a plan with several problems): the four corners'
// first steps with C4.T3 (C1.T1 is the first corner's first step), then the
// corners' remaining steps, the two halves, the four-corner product; after
// the SVD the two projectors, then C1', C4' and the first step of T4' (from
// P_dn.T4 on, T4' is contracted in the order of a corner's chain, never
// forming T4.A.A*).  Eleven contraction launches in all, plus the SVD's and
// the normalisation's kernels.  The SVD's kept
// counts decide the projectors' structure, so the host waits for them once;
// the later plans come from the structure cache when the structure repeats
// (as it does move after move once CTM settles).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/yastn.h"
#include "planner.hpp"

#define CTM_HIP(call)                                                                                            \
  do {                                                                                                           \
    hipError_t e_ = (call);                                                                                      \
    if (e_ != hipSuccess) return set_error(YASTN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CTM_TRY(call)                  \
  do {                                 \
    yastn_status s_ = (call);          \
    if (s_ != YASTN_OK) return s_;     \
  } while (0)

namespace yastn {
namespace {

// tensors of the move: the nine inputs, A*, then every intermediate
enum : int {
  kC1, kC2, kC3, kC4, kT1, kT2, kT3, kT4, kA, kAc,
  kQ1a, kQ1b, kQ1c, kQ1, kQ2a, kQ2b, kQ2c, kQ2, kQ3a, kQ3b, kQ3c, kQ3, kQ4a, kQ4b, kQ4c, kQ4,
  kC4T3, kRup, kRdn, kM,
  kUs, kVts, kUsD, kVtsD, kPup, kPdn, kC1n, kZ1, kZ2, kZ3, kT4n, kC4n, kC1o, kT4o, kC4o,
  kNumIds
};

// one contraction: out = tensordot(left, right, axes)
struct Step {
  int out, left, right;
  std::vector<int32_t> ax, bx;
};

// the grouped launches before the SVD, in order (Q1a is C1.T1 itself)
const std::vector<std::vector<Step>> &pre_levels() {
  static const std::vector<std::vector<Step>> L = {
      {{kQ1a, kC1, kT1, {1}, {0}}, {kQ2a, kC2, kT2, {1}, {0}}, {kQ3a, kC3, kT3, {1}, {3}},
       {kQ4a, kC4, kT4, {0}, {3}}, {kC4T3, kC4, kT3, {1}, {0}}},
      {{kQ1b, kQ1a, kT4, {0}, {0}}, {kQ2b, kQ2a, kT1, {0}, {3}}, {kQ3b, kQ3a, kT2, {0}, {3}},
       {kQ4b, kQ4a, kT3, {0}, {0}}},
      {{kQ1c, kQ1b, kA, {0, 3}, {0, 1}}, {kQ2c, kQ2b, kA, {0, 4}, {3, 0}}, {kQ3c, kQ3b, kA, {1, 4}, {2, 3}},
       {kQ4c, kQ4b, kA, {1, 3}, {1, 2}}},
      {{kQ1, kQ1c, kAc, {0, 2, 6}, {0, 1, 4}}, {kQ2, kQ2c, kAc, {0, 3, 6}, {3, 0, 4}},
       {kQ3, kQ3c, kAc, {1, 3, 6}, {2, 3, 4}}, {kQ4, kQ4c, kAc, {1, 2, 6}, {1, 2, 4}}},
      {{kRup, kQ2, kQ1, {1, 2, 4}, {0, 3, 5}}, {kRdn, kQ3, kQ4, {0, 3, 5}, {1, 3, 5}}},
      {{kM, kRup, kRdn, {3, 4, 5}, {3, 4, 5}}},
  };
  return L;
}
constexpr int kCornerLevels = 4;  // levels 0-3 build the corners

const std::vector<std::vector<Step>> &post_levels() {
  static const std::vector<std::vector<Step>> L = {
      {{kPup, kRdn, kVtsD, {0, 1, 2}, {1, 2, 3}}, {kPdn, kRup, kUsD, {0, 1, 2}, {0, 1, 2}}},
      {{kC1n, kPup, kQ1a, {0, 1, 2}, {0, 1, 2}}, {kC4n, kPdn, kC4T3, {0, 1, 2}, {0, 1, 2}},
       {kZ1, kPdn, kT4, {0}, {0}}},
      {{kZ2, kZ1, kA, {0, 3}, {0, 1}}},
      {{kZ3, kZ2, kAc, {0, 2, 6}, {0, 1, 4}}},
      {{kT4n, kZ3, kPup, {1, 2, 4}, {0, 1, 2}}},
  };
  return L;
}

// a descriptor with its own arrays
struct OwnedDesc {
  int32_t rank = 0, nsym = 0;
  std::vector<int32_t> sym_mod, n, charges;
  std::vector<int8_t> sig;
  std::vector<int64_t> shapes, offsets;
  int64_t nblocks = 0;

  void assign(const yastn_tensor_desc &d) {
    rank = d.rank;
    nsym = d.nsym;
    nblocks = d.nblocks;
    sym_mod.assign(d.sym_mod, d.sym_mod + d.nsym);
    n.assign(d.n, d.n + d.nsym);
    sig.assign(d.sig, d.sig + d.rank);
    charges.assign(d.charges, d.charges + size_t(d.nblocks) * d.rank * d.nsym);
    shapes.assign(d.shapes, d.shapes + size_t(d.nblocks) * d.rank);
    offsets.assign(d.offsets, d.offsets + size_t(d.nblocks));
  }
  yastn_tensor_desc view() const {
    yastn_tensor_desc d{};
    d.rank = rank;
    d.nsym = nsym;
    d.sym_mod = sym_mod.data();
    d.sig = sig.data();
    d.n = n.data();
    d.nblocks = nblocks;
    d.charges = charges.data();
    d.shapes = shapes.data();
    d.offsets = offsets.data();
    return d;
  }
  // the conjugate of a real tensor: signatures and total charge flipped
  OwnedDesc dual() const {
    OwnedDesc o = *this;
    for (auto &s : o.sig) s = int8_t(-s);
    for (int c = 0; c < nsym; ++c) {
      const int64_t m = sym_mod[c];
      int64_t v = -int64_t(n[c]);
      if (m) v = ((v % m) + m) % m;
      o.n[c] = int32_t(v);
    }
    return o;
  }
};

// elements spanned by a descriptor's blocks (inputs may leave gaps)
bool desc_span(const yastn_tensor_desc &d, int64_t *numel) {
  if (d.rank < 0 || d.rank > YASTN_MAX_RANK || d.nblocks < 0) return false;
  if (d.nblocks > 0 && (!d.shapes || !d.offsets)) return false;
  int64_t span = 0;
  for (int64_t b = 0; b < d.nblocks; ++b) {
    int64_t sz = 1;
    for (int i = 0; i < d.rank; ++i) sz *= std::max<int64_t>(0, d.shapes[b * d.rank + i]);
    span = std::max(span, d.offsets[b] + sz);
  }
  *numel = span;
  return true;
}

struct Slot {
  OwnedDesc d;
  int64_t numel = 0;
  double *buf = nullptr;
};

__global__ void __launch_bounds__(256) k_ctm_divide(const double *__restrict__ x, double *__restrict__ y, int64_t n,
                                                    const double *__restrict__ norm2) {
  const double mx = norm2[1];
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double v = x[i];
    y[i] = mx > 0.0 ? v / mx : v;
  }
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace yastn

using namespace yastn;

struct yastn_ctm_s {
  std::array<Slot, kNumIds> s;
  std::vector<yastn_plan_t> pre, post;
  yastn_svd_t svd = nullptr;
  void *pre_mem = nullptr, *post_mem = nullptr, *ws = nullptr, *svd_ws = nullptr;
  size_t post_cap = 0, ws_cap = 0;
  double *sv = nullptr, *norms = nullptr;
  void *norm_ws = nullptr;
  int64_t nsv = 0;
  std::vector<int32_t> kept;
  int32_t kept_total = 0, sweeps = 0;
  double ms[6] = {0, 0, 0, 0, 0, 0};
  double flops[2] = {0, 0};
  std::array<hipEvent_t, 7> ev{};
  bool have_result = false;
  int device = 0;
};

namespace {

// plan one grouped launch; fills the output slots' structures
yastn_status plan_level(yastn_ctm_s &h, const std::vector<Step> &lv, hipStream_t st, yastn_plan_t *out) {
  std::vector<yastn_problem> probs(lv.size());
  std::vector<yastn_tensor_desc> views(2 * lv.size());
  for (size_t i = 0; i < lv.size(); ++i) {
    views[2 * i] = h.s[lv[i].left].d.view();
    views[2 * i + 1] = h.s[lv[i].right].d.view();
    probs[i].a = views[2 * i];
    probs[i].b = views[2 * i + 1];
    probs[i].ncontract = (int32_t)lv[i].ax.size();
    probs[i].axes_a = lv[i].ax.data();
    probs[i].axes_b = lv[i].bx.data();
  }
  CTM_TRY(yastn_plan(probs.data(), (int32_t)probs.size(), nullptr, st, out));
  for (size_t i = 0; i < lv.size(); ++i) {
    yastn_tensor_desc c{};
    int64_t numel = 0;
    CTM_TRY(yastn_plan_output(*out, (int32_t)i, &c, &numel));
    Slot &o = h.s[lv[i].out];
    o.d.assign(c);
    o.numel = numel;
  }
  return YASTN_OK;
}

yastn_status grow_workspace(yastn_ctm_s &h, const std::vector<yastn_plan_t> &plans) {
  size_t need = 256;
  for (auto p : plans) {
    size_t b = 0;
    CTM_TRY(yastn_plan_workspace(p, &b));
    need = std::max(need, b);
  }
  if (need <= h.ws_cap) return YASTN_OK;
  if (h.ws) CTM_HIP(hipFree(h.ws));
  h.ws = nullptr;
  h.ws_cap = 0;
  if (hipMalloc(&h.ws, need) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(YASTN_ERR_NOMEM, "CTM contraction workspace");
  }
  h.ws_cap = need;
  return YASTN_OK;
}

// place the buffers of the given slots in one allocation
yastn_status place(yastn_ctm_s &h, const std::vector<int> &ids, void **mem, size_t *cap) {
  size_t need = 256;
  for (int id : ids) need += al256(size_t(std::max<int64_t>(1, h.s[id].numel)) * 8);
  if (need > *cap) {
    if (*mem) CTM_HIP(hipFree(*mem));
    *mem = nullptr;
    *cap = 0;
    if (hipMalloc(mem, need) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(YASTN_ERR_NOMEM, "CTM intermediates");
    }
    *cap = need;
  }
  char *p = reinterpret_cast<char *>(*mem);
  for (int id : ids) {
    h.s[id].buf = reinterpret_cast<double *>(p);
    p += al256(size_t(std::max<int64_t>(1, h.s[id].numel)) * 8);
  }
  return YASTN_OK;
}

yastn_status run_level(yastn_ctm_s &h, yastn_plan_t plan, const std::vector<Step> &lv, bool tune, hipStream_t st) {
  std::vector<const void *> a(lv.size()), b(lv.size());
  std::vector<void *> c(lv.size());
  for (size_t i = 0; i < lv.size(); ++i) {
    a[i] = h.s[lv[i].left].buf;
    b[i] = h.s[lv[i].right].buf;
    c[i] = h.s[lv[i].out].buf;
  }
  if (tune) CTM_TRY(yastn_plan_autotune(plan, a.data(), b.data(), c.data(), h.ws, st, 3, nullptr, nullptr));
  return yastn_contract(plan, a.data(), b.data(), c.data(), h.ws, st);
}

void release_post(yastn_ctm_s &h) {
  for (auto p : h.post) yastn_free(p);
  h.post.clear();
}

}  // namespace

extern "C" {

yastn_status yastn_ctm_plan(const yastn_tensor_desc *env, void *hip_stream, yastn_ctm_t *out) {
  if (!env || !out) return set_error(YASTN_ERR_ARG, "null argument");
  *out = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  yastn_ctm_t h = nullptr;
  try {
    h = new yastn_ctm_s;
  } catch (const std::bad_alloc &) {
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  auto fail = [&](yastn_status s) {
    yastn_ctm_free(h);
    return s;
  };
  for (int i = 0; i < 9; ++i) {
    int64_t span = 0;
    if (!desc_span(env[i], &span) || !env[i].sig || !env[i].sym_mod || !env[i].n ||
        (env[i].nblocks > 0 && !env[i].charges))
      return fail(set_error(YASTN_ERR_ARG, "CTM input " + std::to_string(i) + ": bad descriptor"));
    if (env[i].rank != (i < 4 ? 2 : i < 8 ? 4 : 5))
      return fail(set_error(YASTN_ERR_ARG, "CTM input " + std::to_string(i) + ": wrong rank"));
    h->s[i].d.assign(env[i]);
    h->s[i].numel = span;
  }
  h->s[kAc].d = h->s[kA].d.dual();
  h->s[kAc].numel = h->s[kA].numel;
  if (hipGetDevice(&h->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(set_error(YASTN_ERR_HIP, "no device"));
  }
  for (auto &lv : pre_levels()) {
    yastn_plan_t p = nullptr;
    yastn_status s = plan_level(*h, lv, st, &p);
    if (s != YASTN_OK) return fail(s);
    h->pre.push_back(p);
  }
  std::vector<int> ids;
  for (auto &lv : pre_levels())
    for (auto &stp : lv) ids.push_back(stp.out);
  size_t cap = 0;
  yastn_status s = place(*h, ids, &h->pre_mem, &cap);
  if (s == YASTN_OK) s = grow_workspace(*h, h->pre);
  if (s != YASTN_OK) return fail(s);
  // the SVD of the four-corner product, rows = R_up's remaining legs
  const int32_t rows[3] = {0, 1, 2};
  yastn_tensor_desc m = h->s[kM].d.view();
  s = yastn_svd_plan(&m, 3, rows, hip_stream, &h->svd);
  if (s != YASTN_OK) return fail(s);
  int32_t nsec = 0;
  size_t svd_ws = 0;
  // the move keeps chi values of the four-corner product, far above eps
  // times its largest: the singular vectors are formed after QR-
  // preconditioned sweeps (yastn_svd falls back to accumulated rotations
  // when they would not be accurate)
  if (s == YASTN_OK) s = yastn_svd_set_flags(h->svd, YASTN_SVD_RECOVER_V);
  s = s == YASTN_OK ? yastn_svd_info(h->svd, &nsec, &h->nsv, &svd_ws) : s;
  if (s != YASTN_OK) return fail(s);
  h->kept.assign(size_t(std::max(0, nsec)), 0);
  const size_t extra = al256(size_t(std::max<int64_t>(1, h->nsv)) * 8) + 256 + al256(yastn_norm_workspace());
  if (hipMalloc(&h->svd_ws, al256(std::max<size_t>(256, svd_ws)) + extra) != hipSuccess) {
    (void)hipGetLastError();
    return fail(set_error(YASTN_ERR_NOMEM, "CTM SVD workspace"));
  }
  char *e = reinterpret_cast<char *>(h->svd_ws) + al256(std::max<size_t>(256, svd_ws));
  h->sv = reinterpret_cast<double *>(e);
  e += al256(size_t(std::max<int64_t>(1, h->nsv)) * 8);
  h->norms = reinterpret_cast<double *>(e);
  e += 256;
  h->norm_ws = e;
  for (auto &ev : h->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      (void)hipGetLastError();
      return fail(set_error(YASTN_ERR_HIP, "event creation"));
    }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_ctm_move(yastn_ctm_t h, const void *const *env, int32_t chi, double tol, double deg_tol,
                            int32_t flags, void *hip_stream) {
  if (!h || !env) return set_error(YASTN_ERR_ARG, "null argument");
  for (int i = 0; i < 9; ++i)
    if (!env[i] && h->s[i].numel > 0) return set_error(YASTN_ERR_ARG, "null CTM input buffer");
  if (chi < 0 || !(tol >= 0.0) || !(deg_tol >= 0.0)) return set_error(YASTN_ERR_ARG, "chi, tol and deg_tol must be >= 0");
  if (flags & ~YASTN_CTM_AUTOTUNE) return set_error(YASTN_ERR_ARG, "unknown CTM flags");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device) {
    (void)hipGetLastError();
    return set_error(YASTN_ERR_STATE, "current device is not the CTM plan's device");
  }
  const bool tune = (flags & YASTN_CTM_AUTOTUNE) != 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  h->have_result = false;
  for (int i = 0; i < 9; ++i) h->s[i].buf = const_cast<double *>(reinterpret_cast<const double *>(env[i]));
  h->s[kAc].buf = h->s[kA].buf;
  // ---- corners, halves, the four-corner product
  CTM_HIP(hipEventRecord(h->ev[0], st));
  const auto &pre = pre_levels();
  for (size_t l = 0; l < pre.size(); ++l) {
    CTM_TRY(run_level(*h, h->pre[l], pre[l], tune, st));
    if ((int)l == kCornerLevels - 1) CTM_HIP(hipEventRecord(h->ev[1], st));
  }
  CTM_HIP(hipEventRecord(h->ev[2], st));
  // ---- truncated SVD (waits for the kept counts), scaled factors
  CTM_TRY(yastn_svd(h->svd, h->s[kM].buf, chi, tol, deg_tol, h->sv, h->kept.data(), &h->sweeps, h->svd_ws,
                    hip_stream));
  CTM_HIP(hipEventRecord(h->ev[3], st));
  h->kept_total = 0;
  for (int32_t k : h->kept) h->kept_total += k;
  yastn_tensor_desc u{}, vt{};
  int64_t un = 0, vn = 0;
  CTM_TRY(yastn_svd_output(h->svd, &u, &un, &vt, &vn));
  h->s[kUs].d.assign(u);
  h->s[kUs].numel = un;
  h->s[kVts].d.assign(vt);
  h->s[kVts].numel = vn;
  h->s[kUsD].d = h->s[kUs].d.dual();
  h->s[kUsD].numel = un;
  h->s[kVtsD].d = h->s[kVts].d.dual();
  h->s[kVtsD].numel = vn;
  // ---- plans after the SVD (structure cache), their buffers
  release_post(*h);
  const auto &post = post_levels();
  for (auto &lv : post) {
    yastn_plan_t p = nullptr;
    CTM_TRY(plan_level(*h, lv, st, &p));
    h->post.push_back(p);
  }
  h->s[kC1o].d = h->s[kC1n].d;
  h->s[kC1o].numel = h->s[kC1n].numel;
  h->s[kT4o].d = h->s[kT4n].d;
  h->s[kT4o].numel = h->s[kT4n].numel;
  h->s[kC4o].d = h->s[kC4n].d;
  h->s[kC4o].numel = h->s[kC4n].numel;
  CTM_TRY(place(*h, {kUs, kVts, kPup, kPdn, kC1n, kZ1, kZ2, kZ3, kT4n, kC4n, kC1o, kT4o, kC4o}, &h->post_mem,
                &h->post_cap));
  h->s[kUsD].buf = h->s[kUs].buf;
  h->s[kVtsD].buf = h->s[kVts].buf;
  CTM_TRY(grow_workspace(*h, h->post));
  CTM_TRY(yastn_svd_factors_scaled(h->svd, h->s[kUs].buf, h->s[kVts].buf, -0.5, -0.5, h->svd_ws, hip_stream));
  CTM_HIP(hipEventRecord(h->ev[4], st));
  // ---- projectors and the new left column
  for (size_t l = 0; l < post.size(); ++l) CTM_TRY(run_level(*h, h->post[l], post[l], tune, st));
  CTM_HIP(hipEventRecord(h->ev[5], st));
  // ---- each new tensor divided by its largest |entry|
  const int src[3] = {kC1n, kT4n, kC4n}, dst[3] = {kC1o, kT4o, kC4o};
  for (int i = 0; i < 3; ++i) {
    const int64_t n = h->s[src[i]].numel;
    if (n == 0) continue;
    CTM_TRY(yastn_norm(h->s[src[i]].buf, n, YASTN_DTYPE_F64, h->norms + 2 * i, h->norm_ws, hip_stream));
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_ctm_divide, dim3(g), dim3(256), 0, st, h->s[src[i]].buf, h->s[dst[i]].buf, n,
                       h->norms + 2 * i);
    CTM_HIP(hipGetLastError());
  }
  CTM_HIP(hipEventRecord(h->ev[6], st));
  CTM_HIP(hipEventSynchronize(h->ev[6]));
  for (int i = 0; i < 6; ++i) {
    float t = 0.f;
    CTM_HIP(hipEventElapsedTime(&t, h->ev[i], h->ev[i + 1]));
    h->ms[i] = t;
  }
  // useful flops of the contractions before and after the SVD
  for (int half = 0; half < 2; ++half) {
    h->flops[half] = 0.0;
    for (auto p : half ? h->post : h->pre) {
      int32_t np = 0;
      CTM_TRY(yastn_plan_info(p, nullptr, &np));
      for (int32_t i = 0; i < np; ++i) {
        yastn_stats stt{};
        CTM_TRY(yastn_plan_stats(p, i, &stt));
        h->flops[half] += stt.useful_flops;
      }
    }
  }
  h->have_result = true;
  return YASTN_OK;
}

yastn_status yastn_ctm_tensor(yastn_ctm_t h, int32_t which, yastn_tensor_desc *desc, int64_t *numel,
                              const void **data) {
  if (!h) return set_error(YASTN_ERR_ARG, "null handle");
  static const int map[YASTN_CTM_NTENSORS] = {kQ1,   kQ2,  kQ3,  kQ4,  kRup, kRdn, kM,   kUs,  kVts, kPup, kPdn,
                                              kQ1a,  kC4T3, kZ1, kZ2,  kZ3,  kC1n, kT4n, kC4n, kC1o, kT4o, kC4o};
  if (which < 0 || which >= YASTN_CTM_NTENSORS) return set_error(YASTN_ERR_ARG, "tensor id out of range");
  const int id = map[which];
  if (id >= kUs && !h->have_result) return set_error(YASTN_ERR_STATE, "no CTM move result yet");
  const Slot &s = h->s[id];
  if (desc) *desc = s.d.view();
  if (numel) *numel = s.numel;
  if (data) *data = s.buf;
  return YASTN_OK;
}

yastn_status yastn_ctm_copy(yastn_ctm_t h, int32_t which, void *dst, void *hip_stream) {
  yastn_tensor_desc d{};
  int64_t numel = 0;
  const void *src = nullptr;
  CTM_TRY(yastn_ctm_tensor(h, which, &d, &numel, &src));
  if (numel == 0) return YASTN_OK;
  if (!dst) return set_error(YASTN_ERR_ARG, "null destination");
  CTM_HIP(hipMemcpyAsync(dst, src, size_t(numel) * 8, hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(hip_stream)));
  return YASTN_OK;
}

yastn_status yastn_ctm_info(yastn_ctm_t h, int32_t *kept, int32_t *sweeps, double *ms, double *flops) {
  if (!h) return set_error(YASTN_ERR_ARG, "null handle");
  if (!h->have_result) return set_error(YASTN_ERR_STATE, "no CTM move result yet");
  if (kept) *kept = h->kept_total;
  if (sweeps) *sweeps = h->sweeps;
  if (ms) std::memcpy(ms, h->ms, sizeof(h->ms));
  if (flops) std::memcpy(flops, h->flops, sizeof(h->flops));
  return YASTN_OK;
}

void yastn_ctm_free(yastn_ctm_t h) {
  if (!h) return;
  for (auto p : h->pre) yastn_free(p);
  release_post(*h);
  yastn_svd_free(h->svd);
  if (h->pre_mem) (void)hipFree(h->pre_mem);
  if (h->post_mem) (void)hipFree(h->post_mem);
  if (h->ws) (void)hipFree(h->ws);
  if (h->svd_ws) (void)hipFree(h->svd_ws);
  for (auto ev : h->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete h;
}

}  // extern "C"
