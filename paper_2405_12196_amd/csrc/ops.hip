// Leg permutation (transpose) of a block tensor, and the reverse-mode
// gradient of a tensordot built from one contraction plan and one
// permutation (the C ABI declared in include/yastn.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/yastn.h"
#include "index.hpp"
#include "planner.hpp"

#define OPS_HIP(call)                                                                                            \
  do {                                                                                                           \
    hipError_t e_ = (call);                                                                                      \
    if (e_ != hipSuccess) return set_error(YASTN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace yastn {
namespace {

constexpr int kPermTile = 1024;  // output elements of one block per workgroup tile

// One output block of a permutation: where it reads and writes, its dims in
// output order (with multiply-high constants for dividing by them) and the
// input stride of each output axis.
struct DevPermBlock {
  int64_t in_off, out_off;
  int32_t numel, rank;
  int32_t dim[YASTN_MAX_RANK];
  uint32_t mag[YASTN_MAX_RANK];
  int32_t sh[YASTN_MAX_RANK];
  int64_t istr[YASTN_MAX_RANK];
};
struct DevPermTile {
  int32_t blk, start;
};

// One thread per output element: the element's output index is split into
// its axis indices (last axis fastest) and re-weighted by the input strides.
// Writes are contiguous within a block; reads gather.
template <typename T>
__global__ void __launch_bounds__(256) k_permute(const DevPermBlock *__restrict__ blocks,
                                                 const DevPermTile *__restrict__ tiles, int ntiles,
                                                 const T *__restrict__ x, T *__restrict__ y) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DevPermTile tl = tiles[t];
    const DevPermBlock &b = blocks[tl.blk];
    const int end = min(tl.start + kPermTile, b.numel);
    for (int e = tl.start + (int)threadIdx.x; e < end; e += 256) {
      uint32_t r = (uint32_t)e;
      int64_t src = 0;
      for (int d = b.rank - 1; d >= 0; --d) {
        const uint32_t q = (uint32_t)(((uint64_t)r * b.mag[d]) >> b.sh[d]);
        src += (int64_t)(r - q * (uint32_t)b.dim[d]) * b.istr[d];
        r = q;
      }
      y[b.out_off + e] = x[b.in_off + src];
    }
  }
}

bool lex_less(const int32_t *a, const int32_t *b, int n) { return std::lexicographical_compare(a, a + n, b, b + n); }

}  // namespace

struct PermPlanImpl {
  int rank = 0, nsym = 0;
  int32_t sym_mod[YASTN_MAX_NSYM] = {0};
  int8_t sig[YASTN_MAX_RANK] = {0};
  int32_t n[YASTN_MAX_NSYM] = {0};
  std::vector<int32_t> charges;
  std::vector<int64_t> shapes, offsets;
  int64_t numel = 0, x_span = 0;
  int ntiles = 0;
  void *dev_mem = nullptr;
  DevPermBlock *dblocks = nullptr;
  DevPermTile *dtiles = nullptr;
};

struct GradPlanImpl {
  int wrt = 0;
  yastn_options opts{};
  yastn_plan_t contraction = nullptr;
  yastn_perm_t perm = nullptr;  // null when the contraction already gives the operand's leg order
  size_t ws_contraction = 0, tmp_off = 0, ws_bytes = 0;
};

}  // namespace yastn

struct yastn_perm_s {
  yastn::PermPlanImpl p;
};
struct yastn_grad_s {
  yastn::GradPlanImpl g;
};

using namespace yastn;

extern "C" {

yastn_status yastn_perm_plan(const yastn_tensor_desc *x, const int32_t *perm, void *hip_stream, yastn_perm_t *out) {
  if (!x || !out || (x->rank > 0 && !perm)) return set_error(YASTN_ERR_ARG, "null argument");
  *out = nullptr;
  HostTensor t;
  yastn_status st = validate_tensor(*x, "X", t);
  if (st != YASTN_OK) return st;
  const int r = t.rank, ns = t.nsym;
  bool seen[YASTN_MAX_RANK] = {false};
  for (int i = 0; i < r; ++i) {
    if (perm[i] < 0 || perm[i] >= r || seen[perm[i]]) return set_error(YASTN_ERR_ARG, "perm is not a permutation");
    seen[perm[i]] = true;
  }
  yastn_perm_t h = nullptr;
  try {
    h = new yastn_perm_s;
    PermPlanImpl &p = h->p;
    p.rank = r;
    p.nsym = ns;
    for (int c = 0; c < ns; ++c) {
      p.sym_mod[c] = t.sym_mod[c];
      p.n[c] = t.n[c];
    }
    for (int i = 0; i < r; ++i) p.sig[i] = t.sig[perm[i]];
    // permuted charge tuples, output blocks in ascending order
    const int64_t nb = t.nblocks;
    std::vector<int32_t> pq(size_t(nb) * r * ns);
    for (int64_t b = 0; b < nb; ++b)
      for (int i = 0; i < r; ++i)
        for (int c = 0; c < ns; ++c) pq[(b * r + i) * ns + c] = t.q(b, perm[i])[c];
    std::vector<int64_t> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int64_t a, int64_t b) { return lex_less(&pq[a * r * ns], &pq[b * r * ns], r * ns); });
    std::vector<DevPermBlock> blocks(nb);
    std::vector<DevPermTile> tiles;
    p.charges.resize(pq.size());
    p.shapes.resize(size_t(nb) * r);
    p.offsets.resize(nb);
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t b = order[k];
      std::memcpy(&p.charges[k * r * ns], &pq[b * r * ns], sizeof(int32_t) * r * ns);
      // input strides of X's block b (C order)
      int64_t xstr[YASTN_MAX_RANK];
      int64_t s = 1;
      for (int i = r - 1; i >= 0; --i) {
        xstr[i] = s;
        s *= t.dim(b, i);
      }
      DevPermBlock &db = blocks[k];
      std::memset(&db, 0, sizeof(db));
      db.in_off = t.offsets[b];
      db.out_off = p.numel;
      db.numel = (int32_t)t.size(b);
      db.rank = r;
      for (int i = 0; i < r; ++i) {
        const int64_t d = t.dim(b, perm[i]);
        p.shapes[k * r + i] = d;
        db.dim[i] = (int32_t)d;
        div_magic((uint32_t)d, &db.mag[i], &db.sh[i]);
        db.istr[i] = xstr[perm[i]];
      }
      p.offsets[k] = p.numel;
      for (int32_t e = 0; e < db.numel; e += kPermTile) tiles.push_back(DevPermTile{(int32_t)k, e});
      p.numel += db.numel;
      p.x_span = std::max(p.x_span, t.offsets[b] + db.numel);
    }
    if (tiles.size() > size_t(INT32_MAX)) {
      delete h;
      return set_error(YASTN_ERR_ARG, "tensor too large to permute in one launch");
    }
    p.ntiles = (int)tiles.size();
    if (nb > 0) {
      const size_t bb = blocks.size() * sizeof(DevPermBlock), tb = tiles.size() * sizeof(DevPermTile);
      const size_t to = (bb + 255) / 256 * 256;
      if (hipMalloc(&p.dev_mem, to + tb) != hipSuccess) {
        delete h;
        return set_error(YASTN_ERR_NOMEM, "device tables of the permutation");
      }
      p.dblocks = reinterpret_cast<DevPermBlock *>(p.dev_mem);
      p.dtiles = reinterpret_cast<DevPermTile *>(static_cast<char *>(p.dev_mem) + to);
      hipStream_t sm = reinterpret_cast<hipStream_t>(hip_stream);
      if (hipMemcpyAsync(p.dblocks, blocks.data(), bb, hipMemcpyHostToDevice, sm) != hipSuccess ||
          hipMemcpyAsync(p.dtiles, tiles.data(), tb, hipMemcpyHostToDevice, sm) != hipSuccess ||
          hipStreamSynchronize(sm) != hipSuccess) {
        yastn_perm_free(h);
        return set_error(YASTN_ERR_HIP, "uploading the permutation tables");
      }
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_perm_output(yastn_perm_t h, yastn_tensor_desc *y, int64_t *y_numel) {
  if (!h || !y) return set_error(YASTN_ERR_ARG, "null argument");
  const PermPlanImpl &p = h->p;
  y->rank = p.rank;
  y->nsym = p.nsym;
  y->sym_mod = p.sym_mod;
  y->sig = p.sig;
  y->n = p.n;
  y->nblocks = (int64_t)p.offsets.size();
  y->charges = p.charges.data();
  y->shapes = p.shapes.data();
  y->offsets = p.offsets.data();
  if (y_numel) *y_numel = p.numel;
  return YASTN_OK;
}

yastn_status yastn_permute(yastn_perm_t h, yastn_dtype dtype, const void *x, void *y, void *hip_stream) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  if (dtype != YASTN_DTYPE_F64 && dtype != YASTN_DTYPE_F32) return set_error(YASTN_ERR_ARG, "unknown dtype");
  const PermPlanImpl &p = h->p;
  if (p.ntiles == 0) return YASTN_OK;
  if (!x || !y) return set_error(YASTN_ERR_ARG, "null buffer");
  const size_t es = dtype == YASTN_DTYPE_F64 ? 8 : 4;
  const char *xb = static_cast<const char *>(x), *yb = static_cast<const char *>(y);
  if (xb < yb + p.numel * es && yb < xb + p.x_span * es) return set_error(YASTN_ERR_ARG, "X and Y overlap");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int grid = std::min(p.ntiles, 8192);
  if (dtype == YASTN_DTYPE_F64)
    k_permute<double><<<grid, 256, 0, st>>>(p.dblocks, p.dtiles, p.ntiles, static_cast<const double *>(x),
                                            static_cast<double *>(y));
  else
    k_permute<float><<<grid, 256, 0, st>>>(p.dblocks, p.dtiles, p.ntiles, static_cast<const float *>(x),
                                           static_cast<float *>(y));
  OPS_HIP(hipGetLastError());
  return YASTN_OK;
}

void yastn_perm_free(yastn_perm_t h) {
  if (!h) return;
  if (h->p.dev_mem) (void)hipFree(h->p.dev_mem);
  delete h;
}

yastn_status yastn_grad_plan(const yastn_problem *prob, int32_t wrt, const yastn_options *opts, void *hip_stream,
                             yastn_grad_t *out) {
  if (!prob || !out) return set_error(YASTN_ERR_ARG, "null argument");
  if (wrt != 0 && wrt != 1) return set_error(YASTN_ERR_ARG, "wrt must be 0 (A) or 1 (B)");
  *out = nullptr;
  // C's structure (the structure of dC) from a plan of the forward contraction
  yastn_plan_t fwd = nullptr;
  yastn_status st = yastn_plan(prob, 1, nullptr, hip_stream, &fwd);
  if (st != YASTN_OK) return st;
  yastn_tensor_desc cd{};
  int64_t cn = 0;
  yastn_plan_output(fwd, 0, &cd, &cn);
  std::vector<int8_t> c_sig(cd.sig, cd.sig + cd.rank);
  std::vector<int32_t> c_sym(cd.sym_mod, cd.sym_mod + cd.nsym), c_n(cd.n, cd.n + cd.nsym);
  std::vector<int32_t> c_q(cd.charges, cd.charges + cd.nblocks * cd.rank * cd.nsym);
  std::vector<int64_t> c_sh(cd.shapes, cd.shapes + cd.nblocks * cd.rank), c_off(cd.offsets, cd.offsets + cd.nblocks);
  yastn_free(fwd);
  cd.sig = c_sig.data();
  cd.sym_mod = c_sym.data();
  cd.n = c_n.data();
  cd.charges = c_q.data();
  cd.shapes = c_sh.data();
  cd.offsets = c_off.data();
  // the other operand, conjugated: flipped signatures and total charge
  const yastn_tensor_desc &o = wrt == 0 ? prob->b : prob->a;
  std::vector<int8_t> o_sig(o.rank);
  std::vector<int32_t> o_n(o.nsym);
  for (int i = 0; i < o.rank; ++i) o_sig[i] = (int8_t)-o.sig[i];
  for (int c = 0; c < o.nsym; ++c) o_n[c] = -o.n[c];
  yastn_tensor_desc oc = o;
  oc.sig = o_sig.data();
  oc.n = o_n.data();
  // free legs of A and B in order
  const int ra = prob->a.rank, rb = prob->b.rank, nc = prob->ncontract;
  bool ca[YASTN_MAX_RANK] = {false}, cb[YASTN_MAX_RANK] = {false};
  for (int c = 0; c < nc; ++c) {
    ca[prob->axes_a[c]] = true;
    cb[prob->axes_b[c]] = true;
  }
  std::vector<int32_t> fa, fb;
  for (int i = 0; i < ra; ++i)
    if (!ca[i]) fa.push_back(i);
  for (int i = 0; i < rb; ++i)
    if (!cb[i]) fb.push_back(i);
  const int nfa = (int)fa.size(), nfb = (int)fb.size();
  // backward contraction and the operand leg each of its output legs is
  yastn_problem bw{};
  std::vector<int32_t> ax1, ax2, nat;  // nat[i] = operand leg of output leg i
  if (wrt == 0) {
    bw.a = cd;
    bw.b = oc;
    for (int i = 0; i < nfb; ++i) {
      ax1.push_back(nfa + i);
      ax2.push_back(fb[i]);
    }
    nat = fa;
    for (int l = 0; l < rb; ++l)  // B's contracted legs stay, in B's leg order
      for (int c = 0; c < nc; ++c)
        if (prob->axes_b[c] == l) nat.push_back(prob->axes_a[c]);
  } else {
    bw.a = oc;
    bw.b = cd;
    for (int i = 0; i < nfa; ++i) {
      ax1.push_back(fa[i]);
      ax2.push_back(i);
    }
    for (int l = 0; l < ra; ++l)  // A's contracted legs stay, in A's leg order
      for (int c = 0; c < nc; ++c)
        if (prob->axes_a[c] == l) nat.push_back(prob->axes_b[c]);
    for (int i = 0; i < nfb; ++i) nat.push_back(fb[i]);
  }
  bw.ncontract = (int32_t)ax1.size();
  bw.axes_a = ax1.data();
  bw.axes_b = ax2.data();
  yastn_grad_t h = nullptr;
  try {
    h = new yastn_grad_s;
  } catch (const std::bad_alloc &) {
    return set_error(YASTN_ERR_NOMEM, "host allocation");
  }
  GradPlanImpl &g = h->g;
  g.wrt = wrt;
  if ((st = yastn_plan(&bw, 1, opts, hip_stream, &g.contraction)) != YASTN_OK) {
    yastn_grad_free(h);
    return st;
  }
  yastn_plan_info(g.contraction, &g.opts, nullptr);
  yastn_plan_workspace(g.contraction, &g.ws_contraction);
  // leg order: transpose the contraction output back to the operand's order
  const int r = (int)nat.size();
  std::vector<int32_t> perm(r);
  bool ident = true;
  for (int l = 0; l < r; ++l) {
    perm[l] = (int32_t)(std::find(nat.begin(), nat.end(), l) - nat.begin());
    ident = ident && perm[l] == l;
  }
  g.ws_bytes = g.ws_contraction;
  if (!ident) {
    yastn_tensor_desc nd{};
    int64_t nn = 0;
    yastn_plan_output(g.contraction, 0, &nd, &nn);
    if ((st = yastn_perm_plan(&nd, perm.data(), hip_stream, &g.perm)) != YASTN_OK) {
      yastn_grad_free(h);
      return st;
    }
    const size_t es = g.opts.out_dtype == YASTN_DTYPE_F64 ? 8 : 4;
    g.tmp_off = (g.ws_contraction + 255) / 256 * 256;
    g.ws_bytes = g.tmp_off + std::max<size_t>(1, size_t(nn)) * es;
  }
  *out = h;
  return YASTN_OK;
}

yastn_status yastn_grad_output(yastn_grad_t h, yastn_tensor_desc *d, int64_t *numel) {
  if (!h || !d) return set_error(YASTN_ERR_ARG, "null argument");
  if (h->g.perm) return yastn_perm_output(h->g.perm, d, numel);
  return yastn_plan_output(h->g.contraction, 0, d, numel);
}

yastn_status yastn_grad_workspace(yastn_grad_t h, size_t *bytes) {
  if (!h || !bytes) return set_error(YASTN_ERR_ARG, "null argument");
  *bytes = h->g.ws_bytes;
  return YASTN_OK;
}

yastn_status yastn_grad(yastn_grad_t h, const void *dc, const void *other, void *out, void *workspace,
                        void *hip_stream) {
  if (!h) return set_error(YASTN_ERR_ARG, "null plan");
  const GradPlanImpl &g = h->g;
  const void *a = g.wrt == 0 ? dc : other, *b = g.wrt == 0 ? other : dc;
  if (!g.perm) return yastn_contract(g.contraction, &a, &b, &out, workspace, hip_stream);
  if (!workspace) return set_error(YASTN_ERR_ARG, "null workspace");
  void *tmp = static_cast<char *>(workspace) + g.tmp_off;
  yastn_status st = yastn_contract(g.contraction, &a, &b, &tmp, workspace, hip_stream);
  if (st != YASTN_OK) return st;
  return yastn_permute(g.perm, g.opts.out_dtype, tmp, out, hip_stream);
}

void yastn_grad_free(yastn_grad_t h) {
  if (!h) return;
  yastn_free(h->g.contraction);
  yastn_perm_free(h->g.perm);
  delete h;
}

}  // extern "C"
