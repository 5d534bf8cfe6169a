// Complex128 block-sparse tensordot and fermionic swap gates.  gfx950.
//
// Complex tensordot (yastn_zplan_*).  A complex contraction C = A.B with
// interleaved (re, im) storage is one real contraction of the library's FP64
// MFMA kernels with K and N doubled:
//   * A is read as a real tensor with one more leg z (charge 0, dim 2,
//     signature +1) holding (re, im): complex element e at real 2e, 2e + 1,
//     which is A's own buffer (no copy);
//   * B is expanded into a real tensor with two more legs s (charge 0, dim 2,
//     signature -1, contracted with z) and t (charge 0, dim 2, signature +1,
//     free): each complex element b = br + i bi becomes the 2 x 2 block
//         [[br,            sb bi],
//          [-sa sb bi,     sa br]]      (sa, sb = -1 for a conjugated A, B)
//     so that sum over z of a_z B[z, t] is the real (t = 0) and imaginary
//     (t = 1) part of a b, conj(a) b, a conj(b) or conj(a) conj(b);
//   * the real output has one more trailing leg t of dim 2: the complex
//     output in interleaved storage, C's own buffer.
// Conjugating an operand (Sec. II.A: the dual leg flips the signature and
// conjugates the values) flips its signatures and total charge on the host
// and changes the signs of the expansion; the flops are those of the complex
// products (8 m k n per matched block pair), nothing is spent on zeros.  The
// expansion is one streaming kernel over B (read 16 B, write 32 B per
// element); B is the small operand in the CTM contractions.
//
// Swap gates (yastn_swap_*).  In the fermionic scheme the paper follows
// (Sec. III, Hubbard example) a swap gate on two groups of legs changes the
// sign of every block whose charges have odd parity on both groups; the
// plan lists those blocks once, and the gate negates them in place (one
// read and one write of the negated blocks only, none of the others).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/yastn.h"
#include "planner.hpp"

#define FER_HIP(call)                                                                                            \
  do {                                                                                                           \
    hipError_t e_ = (call);                                                                                      \
    if (e_ != hipSuccess) return set_error(YASTN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace yastn {
namespace {

// a descriptor with its own arrays
struct OwnDesc {
  std::vector<int32_t> sym_mod, n, charges;
  std::vector<int8_t> sig;
  std::vector<int64_t> shapes, offsets;
  yastn_tensor_desc d{};
  void seal(int rank, int nsym, int64_t nblocks) {
    d.rank = rank;
    d.nsym = nsym;
    d.nblocks = nblocks;
    d.sym_mod = sym_mod.data();
    d.sig = sig.data();
    d.n = n.data();
    d.charges = charges.data();
    d.shapes = shapes.data();
    d.offsets = offsets.data();
  }
};

int32_t negate_charge(int32_t v, int32_t m) {
  if (m == 0) return -v;
  const int64_t r = (-(int64_t)v) % m;
  return int32_t(r < 0 ? r + m : r);
}

// the validated tensor with `extra` trailing legs of charge 0 and dim 2,
// signatures `xsig`, offsets scaled by `scale`; conj flips every original
// signature and the total charge
void augment(const HostTensor &t, bool conj, int extra, const int8_t *xsig, int64_t scale, OwnDesc &o) {
  const int r = t.rank, ns = t.nsym, R = r + extra;
  o.sym_mod.assign(t.sym_mod, t.sym_mod + ns);
  o.n.resize(size_t(ns));
  for (int c = 0; c < ns; ++c) o.n[c] = conj ? negate_charge(t.n[c], t.sym_mod[c]) : t.n[c];
  o.sig.resize(size_t(R));
  for (int i = 0; i < r; ++i) o.sig[i] = int8_t(conj ? -t.sig[i] : t.sig[i]);
  for (int i = 0; i < extra; ++i) o.sig[r + i] = xsig[i];
  const int64_t nb = t.nblocks;
  o.charges.assign(size_t(nb) * R * ns, 0);
  o.shapes.resize(size_t(nb) * R);
  o.offsets.resize(size_t(nb));
  for (int64_t b = 0; b < nb; ++b) {
    std::memcpy(&o.charges[size_t(b) * R * ns], t.q(b, 0), sizeof(int32_t) * size_t(r) * ns);
    for (int i = 0; i < r; ++i) o.shapes[size_t(b) * R + i] = t.dim(b, i);
    for (int i = 0; i < extra; ++i) o.shapes[size_t(b) * R + r + i] = 2;
    o.offsets[b] = t.offsets[b] * scale;
  }
  o.seal(R, ns, nb);
}

int64_t span_of(const HostTensor &t) {
  int64_t s = 0;
  for (int64_t b = 0; b < t.nblocks; ++b) s = std::max(s, t.offsets[b] + t.size(b));
  return s;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// B (n complex elements, interleaved) -> the 2 x 2 real blocks
__global__ void __launch_bounds__(256) k_zexpand(const double2 *__restrict__ b, double2 *__restrict__ out, int64_t n,
                                                 double sa, double sb) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double2 v = b[i];
    out[2 * i] = make_double2(v.x, sb * v.y);
    out[2 * i + 1] = make_double2(-sa * sb * v.y, sa * v.x);
  }
}

// in-place negation of listed segments (element offset, count) of a buffer
struct DevSeg {
  int64_t off;
  int32_t n, pad;
};
constexpr int kSegMax = 4096;

__device__ __forceinline__ double neg(double v) { return -v; }
__device__ __forceinline__ float neg(float v) { return -v; }
__device__ __forceinline__ double2 neg(double2 v) { return make_double2(-v.x, -v.y); }

template <class T>
__global__ void __launch_bounds__(256) k_negate(const DevSeg *__restrict__ segs, int64_t nseg, T *__restrict__ x) {
  for (int64_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const DevSeg g = segs[s];
    for (int e = threadIdx.x; e < g.n; e += 256) x[g.off + e] = neg(x[g.off + e]);
  }
}

}  // namespace
}  // namespace yastn

using namespace yastn;

struct yastn_zplan_s {
  yastn_plan_t real = nullptr;
  int32_t nprob = 0, conj = 0;
  std::vector<OwnDesc> out;       // complex output descriptors
  std::vector<int64_t> out_numel;  // complex elements
  std::vector<int64_t> b_span;     // complex elements spanned by each B
  std::vector<size_t> bexp_off;    // workspace byte offset of each expanded B
  size_t real_ws = 0, ws_bytes = 0;
};

struct yastn_swap_s {
  std::vector<DevSeg> segs;  // in elements of the tensor
  DevSeg *d_segs = nullptr;
  int64_t blocks = 0, elements = 0, span = 0;
};

extern "C" {

yastn_status yastn_zplan(const yastn_problem *probs, int32_t nprob, int32_t conj, void *hip_stream,
                         yastn_zplan_t *out) {
  if (!probs || !out) return set_error(YASTN_ERR_ARG, "null argument");
  *out = nullptr;
  if (nprob < 1) return set_error(YASTN_ERR_ARG, "nprob must be >= 1");
  if (conj & ~(YASTN_CONJ_A | YASTN_CONJ_B)) return set_error(YASTN_ERR_ARG, "unknown conj flags");
  const bool ca = conj & YASTN_CONJ_A, cb = conj & YASTN_CONJ_B;
  const size_t np = static_cast<size_t>(nprob);
  std::vector<OwnDesc> ad(np), bd(np);
  std::vector<std::vector<int32_t>> axa(np), axb(np);
  std::vector<yastn_problem> rp(np);
  yastn_zplan_t h = nullptr;
  try {
    h = new yastn_zplan_s;
  } catch (const std::bad_alloc &) {
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  auto fail = [&](yastn_status s) {
    yastn_zplan_free(h);
    return s;
  };
  h->nprob = nprob;
  h->conj = conj;
  const int8_t zsig[1] = {1}, stsig[2] = {-1, 1};
  for (int32_t p = 0; p < nprob; ++p) {
    HostTensor ta, tb;
    yastn_status s = validate_tensor(probs[p].a, "A", ta);
    if (s == YASTN_OK) s = validate_tensor(probs[p].b, "B", tb);
    if (s != YASTN_OK) return fail(s);
    if (ta.rank + 1 > YASTN_MAX_RANK || tb.rank + 2 > YASTN_MAX_RANK)
      return fail(set_error(YASTN_ERR_ARG, "complex operands: A rank <= " + std::to_string(YASTN_MAX_RANK - 1) +
                                               ", B rank <= " + std::to_string(YASTN_MAX_RANK - 2)));
    const int nc = probs[p].ncontract;
    if (nc < 0 || nc > ta.rank || nc > tb.rank || (nc > 0 && (!probs[p].axes_a || !probs[p].axes_b)))
      return fail(set_error(YASTN_ERR_ARG, "axes"));
    augment(ta, ca, 1, zsig, 2, ad[p]);
    augment(tb, cb, 2, stsig, 4, bd[p]);
    axa[p].assign(probs[p].axes_a, probs[p].axes_a + nc);
    axb[p].assign(probs[p].axes_b, probs[p].axes_b + nc);
    axa[p].push_back(ta.rank);  // z
    axb[p].push_back(tb.rank);  // s
    rp[p].a = ad[p].d;
    rp[p].b = bd[p].d;
    rp[p].ncontract = nc + 1;
    rp[p].axes_a = axa[p].data();
    rp[p].axes_b = axb[p].data();
    h->b_span.push_back(span_of(tb));
  }
  yastn_status s = yastn_plan(rp.data(), nprob, nullptr, hip_stream, &h->real);
  if (s != YASTN_OK) return fail(s);
  if ((s = yastn_plan_workspace(h->real, &h->real_ws)) != YASTN_OK) return fail(s);
  size_t off = al256(std::max<size_t>(256, h->real_ws));
  for (int32_t p = 0; p < nprob; ++p) {
    h->bexp_off.push_back(off);
    off += al256(size_t(std::max<int64_t>(1, h->b_span[p])) * 32);
  }
  h->ws_bytes = off;
  // complex outputs: the real output without its trailing (re, im) leg
  h->out.resize(np);
  for (int32_t p = 0; p < nprob; ++p) {
    yastn_tensor_desc c{};
    int64_t numel = 0;
    if ((s = yastn_plan_output(h->real, p, &c, &numel)) != YASTN_OK) return fail(s);
    OwnDesc &o = h->out[p];
    const int R = c.rank, r = R - 1, ns = c.nsym;
    o.sym_mod.assign(c.sym_mod, c.sym_mod + ns);
    o.n.assign(c.n, c.n + ns);
    o.sig.assign(c.sig, c.sig + r);
    o.charges.resize(size_t(c.nblocks) * r * ns);
    o.shapes.resize(size_t(c.nblocks) * r);
    o.offsets.resize(size_t(c.nblocks));
    for (int64_t b = 0; b < c.nblocks; ++b) {
      std::memcpy(&o.charges[size_t(b) * r * ns], &c.charges[size_t(b) * R * ns], sizeof(int32_t) * size_t(r) * ns);
      std::memcpy(&o.shapes[size_t(b) * r], &c.shapes[size_t(b) * R], sizeof(int64_t) * size_t(r));
      o.offsets[b] = c.offsets[b] / 2;
    }
    o.seal(r, ns, c.nblocks);
    h->out_numel.push_back(numel / 2);
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_zplan_output(yastn_zplan_t h, int32_t prob, yastn_tensor_desc *c, int64_t *c_numel) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (prob < 0 || prob >= h->nprob) return set_error(YASTN_ERR_ARG, "problem index out of range");
  if (c) *c = h->out[prob].d;
  if (c_numel) *c_numel = h->out_numel[prob];
  return YASTN_OK;
}

yastn_status yastn_zplan_workspace(yastn_zplan_t h, size_t *bytes) {
  if (!h || !bytes) return set_error(YASTN_ERR_ARG, "null argument");
  *bytes = h->ws_bytes;
  return YASTN_OK;
}

yastn_status yastn_zplan_real(yastn_zplan_t h, yastn_plan_t *real) {
  if (!h || !real) return set_error(YASTN_ERR_ARG, "null argument");
  *real = h->real;
  return YASTN_OK;
}

namespace {
// B of every problem expanded into the workspace; bx receives their addresses
yastn_status expand_b(yastn_zplan_t h, const void *const *b, void *workspace, hipStream_t st,
                      std::vector<const void *> &bx) {
  if (!workspace) return set_error(YASTN_ERR_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u) return set_error(YASTN_ERR_ARG, "workspace must be 256-byte aligned");
  const double sa = (h->conj & YASTN_CONJ_A) ? -1.0 : 1.0, sb = (h->conj & YASTN_CONJ_B) ? -1.0 : 1.0;
  bx.assign(static_cast<size_t>(h->nprob), nullptr);
  char *ws = reinterpret_cast<char *>(workspace);
  for (int32_t p = 0; p < h->nprob; ++p) {
    const int64_t n = h->b_span[p];
    bx[p] = ws + h->bexp_off[p];
    if (n == 0) continue;
    if (!b[p]) return set_error(YASTN_ERR_ARG, "null B buffer");
    if (reinterpret_cast<uintptr_t>(b[p]) & 15u) return set_error(YASTN_ERR_ARG, "complex buffers must be 16-byte aligned");
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_zexpand, dim3(g), dim3(256), 0, st, reinterpret_cast<const double2 *>(b[p]),
                       reinterpret_cast<double2 *>(ws + h->bexp_off[p]), n, sa, sb);
  }
  FER_HIP(hipGetLastError());
  return YASTN_OK;
}
}  // namespace

yastn_status yastn_zcontract(yastn_zplan_t h, const void *const *a, const void *const *b, void *const *c,
                             void *workspace, void *hip_stream) {
  if (!h || !a || !b || !c) return set_error(YASTN_ERR_ARG, "null argument");
  std::vector<const void *> bx;
  yastn_status s = expand_b(h, b, workspace, reinterpret_cast<hipStream_t>(hip_stream), bx);
  if (s != YASTN_OK) return s;
  return yastn_contract(h->real, a, bx.data(), c, workspace, hip_stream);
}

yastn_status yastn_zplan_autotune(yastn_zplan_t h, const void *const *a, const void *const *b, void *const *c,
                                  void *workspace, void *hip_stream, int32_t reps, int32_t *chosen,
                                  float *times_ms) {
  if (!h || !a || !b || !c) return set_error(YASTN_ERR_ARG, "null argument");
  std::vector<const void *> bx;
  yastn_status s = expand_b(h, b, workspace, reinterpret_cast<hipStream_t>(hip_stream), bx);
  if (s != YASTN_OK) return s;
  return yastn_plan_autotune(h->real, a, bx.data(), c, workspace, hip_stream, reps, chosen, times_ms);
}

void yastn_zplan_free(yastn_zplan_t h) {
  if (!h) return;
  yastn_free(h->real);
  delete h;
}

yastn_status yastn_swap_plan(const yastn_tensor_desc *t, int32_t n1, const int32_t *legs1, int32_t n2,
                             const int32_t *legs2, const int32_t *fermionic, yastn_swap_t *out) {
  if (!t || !out || !fermionic || (n1 > 0 && !legs1) || (n2 > 0 && !legs2))
    return set_error(YASTN_ERR_ARG, "null argument");
  *out = nullptr;
  HostTensor x;
  yastn_status s = validate_tensor(*t, "T", x);
  if (s != YASTN_OK) return s;
  if (n1 < 0 || n2 < 0 || n1 > x.rank || n2 > x.rank) return set_error(YASTN_ERR_ARG, "leg group sizes");
  for (int i = 0; i < n1; ++i)
    if (legs1[i] < 0 || legs1[i] >= x.rank) return set_error(YASTN_ERR_ARG, "leg out of range");
  for (int i = 0; i < n2; ++i)
    if (legs2[i] < 0 || legs2[i] >= x.rank) return set_error(YASTN_ERR_ARG, "leg out of range");
  for (int c = 0; c < x.nsym; ++c)
    if (fermionic[c] != 0 && fermionic[c] != 1) return set_error(YASTN_ERR_ARG, "fermionic entries must be 0 or 1");
  yastn_swap_t h = nullptr;
  try {
    h = new yastn_swap_s;
  } catch (const std::bad_alloc &) {
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  auto par = [&](int64_t b, int leg) {
    const int32_t *q = x.q(b, leg);
    int64_t p = 0;
    for (int c = 0; c < x.nsym; ++c) p += fermionic[c] ? (int64_t)q[c] : 0;
    return int(((p % 2) + 2) % 2);
  };
  for (int64_t b = 0; b < x.nblocks; ++b) {
    int p1 = 0, p2 = 0;
    for (int i = 0; i < n1; ++i) p1 ^= par(b, legs1[i]);
    for (int i = 0; i < n2; ++i) p2 ^= par(b, legs2[i]);
    if (!(p1 & p2)) continue;
    const int64_t sz = x.size(b);
    ++h->blocks;
    h->elements += sz;
    for (int64_t e = 0; e < sz; e += kSegMax)
      h->segs.push_back(DevSeg{x.offsets[b] + e, (int32_t)std::min<int64_t>(kSegMax, sz - e), 0});
  }
  h->span = span_of(x);
  if (!h->segs.empty()) {
    if (hipMalloc(&h->d_segs, h->segs.size() * sizeof(DevSeg)) != hipSuccess) {
      (void)hipGetLastError();
      yastn_swap_free(h);
      return set_error(YASTN_ERR_NOMEM, "swap gate table");
    }
    if (hipMemcpy(h->d_segs, h->segs.data(), h->segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      yastn_swap_free(h);
      return set_error(YASTN_ERR_HIP, "swap gate table upload");
    }
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_swap_info(yastn_swap_t h, int64_t *blocks, int64_t *elements) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (blocks) *blocks = h->blocks;
  if (elements) *elements = h->elements;
  return YASTN_OK;
}

yastn_status yastn_swap_gate(yastn_swap_t h, void *data, yastn_dtype dtype, void *hip_stream) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (h->segs.empty()) return YASTN_OK;
  if (!data) return set_error(YASTN_ERR_ARG, "null buffer");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t ns = (int64_t)h->segs.size();
  const unsigned g = (unsigned)std::min<int64_t>(ns, 65535);
  switch (dtype) {
    case YASTN_DTYPE_F64:
      hipLaunchKernelGGL(k_negate<double>, dim3(g), dim3(256), 0, st, h->d_segs, ns, reinterpret_cast<double *>(data));
      break;
    case YASTN_DTYPE_F32:
      hipLaunchKernelGGL(k_negate<float>, dim3(g), dim3(256), 0, st, h->d_segs, ns, reinterpret_cast<float *>(data));
      break;
    case YASTN_DTYPE_C128:
      hipLaunchKernelGGL(k_negate<double2>, dim3(g), dim3(256), 0, st, h->d_segs, ns,
                         reinterpret_cast<double2 *>(data));
      break;
    default:
      return set_error(YASTN_ERR_ARG, "unknown dtype");
  }
  FER_HIP(hipGetLastError());
  return YASTN_OK;
}

void yastn_swap_free(yastn_swap_t h) {
  if (!h) return;
  if (h->d_segs) (void)hipFree(h->d_segs);
  delete h;
}

}  // extern "C"
