// Host side of the plan: descriptor validation, output structure and tiling.
//
// Validation follows the paper's definitions (Sec. II.A): a stored block obeys
// sum_i s_i rho_i = n; a leg carries one dim per charge; blocks are named by
// their charge tuple, so a tuple occurs once.  Contracted legs pair a leg with
// its dual (opposite signature) and must agree on the dim of every charge
// both carry; a charge present on one side only contributes nothing (Sec.
// II.B footnote on contraction partners).
//
// The matching itself (which A block meets which B block) comes from the
// charge-hash join kernel; this file only groups its matches into sectors
// (fused contracted charge X), row/contracted/column tuples, output blocks
// and wave tiles.
#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>

#include "index.hpp"
#include "planner.hpp"

namespace yastn {

namespace {
thread_local std::string g_err;

int64_t norm_charge(int64_t v, int32_t m) {
  if (m == 0) return v;
  int64_t r = v % m;
  return r < 0 ? r + m : r;
}

yastn_status copy_tensor(const yastn_tensor_desc &d, HostTensor &t, const char *name) {
  std::string nm(name);
  if (d.rank < 0 || d.rank > YASTN_MAX_RANK) return set_error(YASTN_ERR_ARG, nm + ": rank out of range");
  if (d.nsym < 1 || d.nsym > YASTN_MAX_NSYM) return set_error(YASTN_ERR_ARG, nm + ": nsym out of range");
  if (!d.sym_mod || !d.n || (d.rank > 0 && !d.sig)) return set_error(YASTN_ERR_ARG, nm + ": null pointer");
  if (d.nblocks < 0) return set_error(YASTN_ERR_ARG, nm + ": negative nblocks");
  if (d.nblocks > 0 && ((d.rank > 0 && (!d.charges || !d.shapes)) || !d.offsets))
    return set_error(YASTN_ERR_ARG, nm + ": null block arrays");
  if (d.nblocks > (int64_t(1) << 30)) return set_error(YASTN_ERR_ARG, nm + ": too many blocks");
  t.rank = d.rank;
  t.nsym = d.nsym;
  for (int c = 0; c < d.nsym; ++c) t.sym_mod[c] = d.sym_mod[c];
  for (int i = 0; i < d.rank; ++i) t.sig[i] = d.sig[i];
  t.nblocks = d.nblocks;
  t.charges.assign(size_t(d.nblocks) * d.rank * d.nsym, 0);
  t.shapes.assign(size_t(d.nblocks) * d.rank, 0);
  t.offsets.assign(size_t(d.nblocks), 0);
  if (d.nblocks) {
    if (d.rank) {
      std::memcpy(t.shapes.data(), d.shapes, t.shapes.size() * sizeof(int64_t));
      for (size_t e = 0; e < t.charges.size(); ++e)
        t.charges[e] = (int32_t)norm_charge(d.charges[e], d.sym_mod[e % d.nsym]);
    }
    std::memcpy(t.offsets.data(), d.offsets, t.offsets.size() * sizeof(int64_t));
  }
  for (int c = 0; c < d.nsym; ++c) t.n[c] = (int32_t)norm_charge(d.n[c], d.sym_mod[c]);
  return YASTN_OK;
}

struct TupleLess {
  const HostTensor *t;
  bool operator()(int64_t x, int64_t y) const {
    const int32_t *a = t->q(x, 0), *b = t->q(y, 0);
    return std::lexicographical_compare(a, a + t->rank * t->nsym, b, b + t->rank * t->nsym);
  }
};

yastn_status check_tensor(HostTensor &t, const char *name) {
  std::string nm(name);
  for (int i = 0; i < t.rank; ++i)
    if (t.sig[i] != 1 && t.sig[i] != -1) return set_error(YASTN_ERR_ARG, nm + ": signature must be +1 or -1");
  for (int64_t b = 0; b < t.nblocks; ++b)
    for (int i = 0; i < t.rank; ++i) {
      if (t.dim(b, i) < 1) return set_error(YASTN_ERR_SHAPE, nm + ": block dims must be >= 1");
      if (t.dim(b, i) > (int64_t(1) << 30)) return set_error(YASTN_ERR_ARG, nm + ": block dim too large");
    }
  for (int64_t b = 0; b < t.nblocks; ++b) {
    int64_t sz = 1;
    for (int i = 0; i < t.rank; ++i) {
      sz *= t.dim(b, i);
      if (sz > (int64_t(1) << 31) - 1) return set_error(YASTN_ERR_ARG, nm + ": block larger than 2^31 elements");
    }
  }
  // the distinct charges of each leg, ascending, and each block's index
  // among them (charges packed into order-preserving 128-bit keys); a charge
  // with two dims is reported after the duplicate and conservation checks
  const int ns = t.nsym;
  t.qid.assign(size_t(t.nblocks) * t.rank, 0);
  t.legq.clear();
  t.legdim.clear();
  bool twodims = false;
  {
    // per leg: an open-addressing table from charge key to first-seen slot,
    // then the (few) distinct keys sorted and the slots renumbered ascending
    typedef unsigned __int128 u128k;
    size_t cap = 16;
    while (cap < 2 * size_t(t.nblocks)) cap <<= 1;
    std::vector<u128k> hkey(cap);
    std::vector<int32_t> hslot(cap), first(size_t(t.nblocks)), tmp(size_t(t.nblocks));
    std::vector<u128k> dkeys;
    for (int i = 0; i < t.rank; ++i) {
      t.legq0[i] = (int64_t)t.legdim.size();
      std::fill(hslot.begin(), hslot.end(), -1);
      dkeys.clear();
      for (int64_t b = 0; b < t.nblocks; ++b) {
        u128k k = 0;
        for (int c = 0; c < ns; ++c) k = (k << 32) | (uint32_t)(t.q(b, i)[c] ^ INT32_MIN);
        uint64_t h = (uint64_t)k * 0x9E3779B97F4A7C15ull ^ (uint64_t)(k >> 64) * 0xC2B2AE3D27D4EB4Full;
        size_t p = (size_t)(h ^ (h >> 29)) & (cap - 1);
        while (hslot[p] >= 0 && hkey[p] != k) p = (p + 1) & (cap - 1);
        if (hslot[p] < 0) {
          hkey[p] = k;
          hslot[p] = (int32_t)dkeys.size();
          first[dkeys.size()] = (int32_t)b;
          dkeys.push_back(k);
        } else if (t.dim(first[hslot[p]], i) != t.dim(b, i)) {
          twodims = true;
        }
        tmp[b] = hslot[p];
      }
      std::vector<int32_t> ord(dkeys.size()), rank(dkeys.size());
      std::iota(ord.begin(), ord.end(), 0);
      std::sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return dkeys[x] < dkeys[y]; });
      for (size_t r = 0; r < ord.size(); ++r) {
        rank[ord[r]] = (int32_t)r;
        const int64_t b = first[ord[r]];
        t.legq.insert(t.legq.end(), t.q(b, i), t.q(b, i) + ns);
        t.legdim.push_back(t.dim(b, i));
      }
      for (int64_t b = 0; b < t.nblocks; ++b) t.qid[b * t.rank + i] = rank[tmp[b]];
      t.nq[i] = (int32_t)dkeys.size();
    }
  }
  t.legq0[t.rank] = (int64_t)t.legdim.size();
  // duplicates (a charge tuple names one block): the tuple of leg indices
  // as one key when it fits 128 bits, else a comparison of charge tuples
  {
    long double span = 1.0L;
    for (int i = 0; i < t.rank; ++i) span *= (long double)std::max(1, t.nq[i]);
    bool dup = false;
    if (span < 1.0e38L) {
      std::vector<unsigned __int128> full(size_t(t.nblocks));
      for (int64_t b = 0; b < t.nblocks; ++b) {
        unsigned __int128 k = 0;
        for (int i = 0; i < t.rank; ++i) k = k * (uint32_t)t.nq[i] + (uint32_t)t.qid[b * t.rank + i];
        full[b] = k;
      }
      std::sort(full.begin(), full.end());
      dup = std::adjacent_find(full.begin(), full.end()) != full.end();
    } else {
      std::vector<int64_t> idx(t.nblocks);
      std::iota(idx.begin(), idx.end(), 0);
      std::sort(idx.begin(), idx.end(), TupleLess{&t});
      for (int64_t k = 1; k < t.nblocks && !dup; ++k)
        dup = !TupleLess{&t}(idx[k - 1], idx[k]) && !TupleLess{&t}(idx[k], idx[k - 1]);
    }
    if (dup) return set_error(YASTN_ERR_DUPLICATE, nm + ": a charge tuple occurs twice");
  }
  // block form of charge conservation
  for (int64_t b = 0; b < t.nblocks; ++b)
    for (int c = 0; c < t.nsym; ++c) {
      int64_t s = 0;
      for (int i = 0; i < t.rank; ++i) s += int64_t(t.sig[i]) * t.q(b, i)[c];
      if (norm_charge(s, t.sym_mod[c]) != t.n[c])
        return set_error(YASTN_ERR_CHARGE, nm + ": a block violates sum_i s_i rho_i = n");
    }
  if (twodims) return set_error(YASTN_ERR_SHAPE, nm + ": one charge has two dims on a leg");
  // offsets: non-negative, blocks disjoint
  std::vector<std::pair<int64_t, int64_t>> spans(t.nblocks);
  for (int64_t b = 0; b < t.nblocks; ++b) {
    if (t.offsets[b] < 0) return set_error(YASTN_ERR_ARG, nm + ": negative block offset");
    spans[b] = {t.offsets[b], t.size(b)};
  }
  std::sort(spans.begin(), spans.end());
  for (int64_t k = 1; k < t.nblocks; ++k)
    if (spans[k - 1].first + spans[k - 1].second > spans[k].first)
      return set_error(YASTN_ERR_ARG, nm + ": blocks overlap in the 1D buffer");
  return YASTN_OK;
}

}  // namespace

int64_t HostTensor::size(int64_t b) const {
  int64_t s = 1;
  for (int i = 0; i < rank; ++i) s *= dim(b, i);
  return s;
}

yastn_status set_error(yastn_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

const char *last_error_cstr() { return g_err.c_str(); }

yastn_status check_options(const yastn_options *o, yastn_options *out) {
  yastn_options d{};
  d.precision = YASTN_F64;
  d.in_dtype = YASTN_DTYPE_F64;
  d.out_dtype = YASTN_DTYPE_F64;
  d.tile_rows = 0;
  d.flags = 0;
  if (o) d = *o;
  if (d.precision < YASTN_F64 || d.precision > YASTN_BF16X6) return set_error(YASTN_ERR_ARG, "unknown precision");
  if (d.in_dtype != YASTN_DTYPE_F64 && d.in_dtype != YASTN_DTYPE_F32) return set_error(YASTN_ERR_ARG, "unknown in_dtype");
  if (d.out_dtype != YASTN_DTYPE_F64 && d.out_dtype != YASTN_DTYPE_F32) return set_error(YASTN_ERR_ARG, "unknown out_dtype");
  if (d.precision == YASTN_F64 && (d.in_dtype != YASTN_DTYPE_F64 || d.out_dtype != YASTN_DTYPE_F64))
    return set_error(YASTN_ERR_ARG, "F64 arithmetic needs F64 input and output buffers");
  if (d.tile_rows != 0 && d.tile_rows != 16 && d.tile_rows != 32 && d.tile_rows != 64 && d.tile_rows != 128 &&
      d.tile_rows != 256 && d.tile_rows != 512)
    return set_error(YASTN_ERR_ARG, "tile_rows must be 0, 16, 32, 64, 128, 256 or 512");
  const int32_t fam = d.flags & ~YASTN_FLAG_NOCACHE;
  if (fam != 0 && fam != YASTN_FLAG_MFMA && fam != YASTN_FLAG_ROWS)
    return set_error(YASTN_ERR_ARG, "flags must be 0, YASTN_FLAG_MFMA or YASTN_FLAG_ROWS, optionally with YASTN_FLAG_NOCACHE");
  *out = d;
  return YASTN_OK;
}

yastn_status validate_tensor(const yastn_tensor_desc &d, const char *name, HostTensor &t) {
  if (d.nsym < 1 || d.nsym > YASTN_MAX_NSYM) return set_error(YASTN_ERR_ARG, std::string(name) + ": nsym out of range");
  if (!d.sym_mod) return set_error(YASTN_ERR_ARG, std::string(name) + ": null sym_mod");
  for (int c = 0; c < d.nsym; ++c)
    if (d.sym_mod[c] < 0 || d.sym_mod[c] == 1) return set_error(YASTN_ERR_SYM, "sym_mod must be 0 (U(1)) or >= 2 (Z_m)");
  yastn_status st = copy_tensor(d, t, name);
  if (st != YASTN_OK) return st;
  return check_tensor(t, name);
}

yastn_status validate_problem(const yastn_problem &p, HostProblem &hp) {
  const yastn_tensor_desc &A = p.a, &B = p.b;
  if (p.ncontract < 0 || p.ncontract > YASTN_MAX_RANK) return set_error(YASTN_ERR_ARG, "ncontract out of range");
  if (p.ncontract > 0 && (!p.axes_a || !p.axes_b)) return set_error(YASTN_ERR_ARG, "null axes");
  if (A.rank < 0 || A.rank > YASTN_MAX_RANK || B.rank < 0 || B.rank > YASTN_MAX_RANK)
    return set_error(YASTN_ERR_ARG, "rank out of range");
  if (p.ncontract > A.rank || p.ncontract > B.rank) return set_error(YASTN_ERR_ARG, "more contracted legs than legs");
  bool used_a[YASTN_MAX_RANK] = {false}, used_b[YASTN_MAX_RANK] = {false};
  for (int c = 0; c < p.ncontract; ++c) {
    int x = p.axes_a[c], y = p.axes_b[c];
    if (x < 0 || x >= A.rank || y < 0 || y >= B.rank || used_a[x] || used_b[y])
      return set_error(YASTN_ERR_ARG, "axes out of range or repeated");
    used_a[x] = used_b[y] = true;
  }
  if (A.nsym != B.nsym) return set_error(YASTN_ERR_SYM, "A and B have different nsym");
  if (A.nsym < 1 || A.nsym > YASTN_MAX_NSYM) return set_error(YASTN_ERR_ARG, "nsym out of range");
  if (!A.sym_mod || !B.sym_mod) return set_error(YASTN_ERR_ARG, "null sym_mod");
  for (int c = 0; c < A.nsym; ++c) {
    if (A.sym_mod[c] != B.sym_mod[c]) return set_error(YASTN_ERR_SYM, "A and B have different symmetry");
    if (A.sym_mod[c] < 0 || A.sym_mod[c] == 1) return set_error(YASTN_ERR_SYM, "sym_mod must be 0 (U(1)) or >= 2 (Z_m)");
  }
  yastn_status st;
  if ((st = copy_tensor(A, hp.a, "A")) != YASTN_OK) return st;
  if ((st = copy_tensor(B, hp.b, "B")) != YASTN_OK) return st;
  if ((st = check_tensor(hp.a, "A")) != YASTN_OK) return st;
  if ((st = check_tensor(hp.b, "B")) != YASTN_OK) return st;
  for (int c = 0; c < p.ncontract; ++c)
    if (hp.a.sig[p.axes_a[c]] == hp.b.sig[p.axes_b[c]])
      return set_error(YASTN_ERR_SIGNATURE, "a contracted leg pair has equal signatures");
  // a charge on both legs of a contracted pair has one dim (merge of the two
  // ascending lists of distinct charges)
  const int ns = hp.a.nsym;
  for (int c = 0; c < p.ncontract; ++c) {
    const int la = p.axes_a[c], lb = p.axes_b[c];
    int64_t x = hp.a.legq0[la], y = hp.b.legq0[lb];
    const int64_t xe = hp.a.legq0[la + 1], ye = hp.b.legq0[lb + 1];
    while (x < xe && y < ye) {
      const int32_t *qa = &hp.a.legq[size_t(x) * ns], *qb = &hp.b.legq[size_t(y) * ns];
      if (std::lexicographical_compare(qa, qa + ns, qb, qb + ns)) {
        ++x;
      } else if (std::lexicographical_compare(qb, qb + ns, qa, qa + ns)) {
        ++y;
      } else {
        if (hp.a.legdim[x] != hp.b.legdim[y])
          return set_error(YASTN_ERR_SHAPE, "a contracted charge has different dims in A and B");
        ++x;
        ++y;
      }
    }
  }
  hp.nc = p.ncontract;
  for (int c = 0; c < p.ncontract; ++c) {
    hp.axes_a[c] = p.axes_a[c];
    hp.axes_b[c] = p.axes_b[c];
  }
  hp.nfa = hp.nfb = 0;
  for (int i = 0; i < A.rank; ++i)
    if (!used_a[i]) hp.fa[hp.nfa++] = i;
  for (int i = 0; i < B.rank; ++i)
    if (!used_b[i]) hp.fb[hp.nfb++] = i;
  for (int64_t b = 0; b < hp.a.nblocks; ++b) hp.a.numel += hp.a.size(b);
  for (int64_t b = 0; b < hp.b.nblocks; ++b) hp.b.numel += hp.b.size(b);
  return YASTN_OK;
}

void contracted_keys(const HostTensor &t, const int *axes, int nc, std::vector<int32_t> &keys) {
  keys.assign(size_t(t.nblocks) * nc * t.nsym, 0);
  for (int64_t b = 0; b < t.nblocks; ++b)
    for (int c = 0; c < nc; ++c)
      for (int s = 0; s < t.nsym; ++s) keys[(b * nc + c) * t.nsym + s] = t.q(b, axes[c])[s];
}

namespace {
// Order-preserving integer keys of charge tuples: the mixed-radix number of
// the legs' charge indices (validation numbers each leg's distinct charges in
// ascending order), first leg most significant, so comparing keys compares
// the tuples lexicographically.  No heap allocation per key.
typedef unsigned __int128 u128;

bool key_fits(const HostTensor &t, const int *legs, int nl) {
  long double p = 1.0L;
  for (int i = 0; i < nl; ++i) p *= (long double)std::max(1, t.nq[legs[i]]);
  return p < 1.0e38L;
}

u128 pack_key(const HostTensor &t, int64_t b, const int *legs, int nl) {
  u128 k = 0;
  for (int i = 0; i < nl; ++i) k = k * (u128)(uint32_t)t.nq[legs[i]] + (u128)(uint32_t)t.qid[b * t.rank + legs[i]];
  return k;
}

// The fused contracted charge X of an A block (nsym components, each
// normalised), as an order-preserving key.
u128 sector_key(const HostTensor &A, int64_t b, const int *axes, int nc) {
  u128 k = 0;
  for (int s = 0; s < A.nsym; ++s) {
    int64_t v = 0;
    for (int c = 0; c < nc; ++c) v += int64_t(A.sig[axes[c]]) * A.q(b, axes[c])[s];
    k = (k << 32) | (u128)(uint32_t)(int32_t)((int32_t)norm_charge(v, A.sym_mod[s]) ^ INT32_MIN);
  }
  return k;
}

template <typename T> int32_t rank_of(const std::vector<T> &sorted, const T &v) {
  return (int32_t)(std::lower_bound(sorted.begin(), sorted.end(), v) - sorted.begin());
}

template <typename T> void sort_unique(std::vector<T> &v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}
}  // namespace

yastn_status build_structure(HostProblem &hp, int prob, const std::vector<std::pair<int32_t, int32_t>> &pairs,
                             int64_t a_base, int64_t b_base, PlanTables &t, bool gather) {
  const HostTensor &A = hp.a, &B = hp.b;
  const int nsym = A.nsym, nc = hp.nc;
  if (!key_fits(A, hp.fa, hp.nfa) || !key_fits(A, hp.axes_a, nc) || !key_fits(B, hp.fb, hp.nfb))
    return set_error(YASTN_ERR_ARG, "too many distinct charges on the legs of one tensor (planner keys are 128-bit)");
  // ---- per block: sector, row tuple, contracted tuple (A) and column tuple (B) keys
  std::vector<u128> ax(size_t(A.nblocks)), ar(size_t(A.nblocks)), ac(size_t(A.nblocks)), bj(size_t(B.nblocks));
  for (int64_t b = 0; b < A.nblocks; ++b) {
    ax[b] = sector_key(A, b, hp.axes_a, nc);
    ar[b] = pack_key(A, b, hp.fa, hp.nfa);
    ac[b] = pack_key(A, b, hp.axes_a, nc);
  }
  for (int64_t b = 0; b < B.nblocks; ++b) bj[b] = pack_key(B, b, hp.fb, hp.nfb);
  // ---- sectors in ascending X; the pairs of each sector in join order
  std::vector<u128> xs;
  xs.reserve(pairs.size());
  for (auto &pr : pairs) xs.push_back(ax[pr.first]);
  sort_unique(xs);
  const int nS = (int)xs.size();
  std::vector<int32_t> psec(pairs.size()), scount(size_t(nS) + 1, 0);
  for (size_t k = 0; k < pairs.size(); ++k) {
    psec[k] = rank_of(xs, ax[pairs[k].first]);
    ++scount[size_t(psec[k]) + 1];
  }
  for (int x = 0; x < nS; ++x) scount[x + 1] += scount[x];
  std::vector<int32_t> sorder(pairs.size());
  {
    std::vector<int32_t> fill(scount.begin(), scount.end() - 1);
    for (size_t k = 0; k < pairs.size(); ++k) sorder[size_t(fill[psec[k]]++)] = (int32_t)k;
  }
  // ---- A storage structure: classes of free legs, contracted positions
  bool isctr[YASTN_MAX_RANK] = {false};
  int cpos[YASTN_MAX_RANK];  // storage leg -> index in axes order
  for (int c = 0; c < nc; ++c) {
    isctr[hp.axes_a[c]] = true;
    cpos[hp.axes_a[c]] = c;
  }
  int act_g[kMaxAct + 1], nact = 0, fcls[YASTN_MAX_RANK];
  for (int q = 0; q < hp.nfa; ++q) {
    int f = hp.fa[q], g = 0;
    for (int l = f + 1; l < A.rank; ++l) g += isctr[l];
    if (nact == 0 || act_g[nact - 1] != g) {
      if (nact == kMaxAct) return set_error(YASTN_ERR_ARG, "leg interleaving of A too deep (more than 4 free-leg groups)");
      act_g[nact++] = g;
    }
    fcls[q] = nact - 1;
  }
  // contracted legs in storage order (for P_a: dims of the last g contracted legs)
  int ctr_storage[YASTN_MAX_RANK], nct = 0;
  for (int l = 0; l < A.rank; ++l)
    if (isctr[l]) ctr_storage[nct++] = cpos[l];
  DevProb dp{};
  dp.nact = nact;
  dp.nc = nc;
  dp.nfb = hp.nfb;
  for (int64_t b = 0; b < A.nblocks; ++b) dp.a_span = std::max<int64_t>(dp.a_span, A.offsets[b] + A.size(b));
  for (int64_t b = 0; b < B.nblocks; ++b) dp.b_span = std::max<int64_t>(dp.b_span, B.offsets[b] + B.size(b));
  const size_t prob_slot = t.probs.size();
  t.probs.push_back(dp);
  // ---- output blocks: (A free tuple, B free tuple) reached by >= 1 pair, ascending order
  struct CKey {
    u128 r, j;      // A free tuple, B free tuple
    int32_t ia, jb; // a pair that reaches the block (its dims and charges)
    bool operator<(const CKey &o) const { return r < o.r || (r == o.r && j < o.j); }
    bool operator==(const CKey &o) const { return r == o.r && j == o.j; }
  };
  std::vector<CKey> ck;
  ck.reserve(pairs.size());
  for (auto &pr : pairs) ck.push_back(CKey{ar[pr.first], bj[pr.second], pr.first, pr.second});
  std::sort(ck.begin(), ck.end());
  ck.erase(std::unique(ck.begin(), ck.end()), ck.end());
  hp.c_rank = hp.nfa + hp.nfb;
  for (int q = 0; q < hp.nfa; ++q) hp.c_sig[q] = A.sig[hp.fa[q]];
  for (int q = 0; q < hp.nfb; ++q) hp.c_sig[hp.nfa + q] = B.sig[hp.fb[q]];
  for (int s = 0; s < nsym; ++s) hp.c_n[s] = (int32_t)norm_charge(int64_t(A.n[s]) + B.n[s], A.sym_mod[s]);
  hp.c_charges.clear();
  hp.c_shapes.clear();
  hp.c_offsets.clear();
  hp.c_charges.reserve(ck.size() * size_t(hp.nfa + hp.nfb) * nsym);
  hp.c_shapes.reserve(ck.size() * size_t(hp.nfa + hp.nfb));
  hp.c_offsets.reserve(ck.size());
  int64_t pos = 0;
  for (const CKey &k : ck) {
    int64_t sz = 1;
    for (int q = 0; q < hp.nfa; ++q) {
      hp.c_charges.insert(hp.c_charges.end(), A.q(k.ia, hp.fa[q]), A.q(k.ia, hp.fa[q]) + nsym);
      hp.c_shapes.push_back(A.dim(k.ia, hp.fa[q]));
      sz *= A.dim(k.ia, hp.fa[q]);
    }
    for (int q = 0; q < hp.nfb; ++q) {
      hp.c_charges.insert(hp.c_charges.end(), B.q(k.jb, hp.fb[q]), B.q(k.jb, hp.fb[q]) + nsym);
      hp.c_shapes.push_back(B.dim(k.jb, hp.fb[q]));
      sz *= B.dim(k.jb, hp.fb[q]);
    }
    hp.c_offsets.push_back(pos);
    pos += sz;
  }
  hp.c_numel = pos;
  t.probs[prob_slot].c_numel = pos;
  // ---- A block offsets and B block strides (plan-global indices)
  for (int64_t b = 0; b < A.nblocks; ++b) t.aoff.push_back(A.offsets[b]);
  for (int64_t b = 0; b < B.nblocks; ++b) {
    DevBBlock bb{};
    bb.off = B.offsets[b];
    int64_t stride[YASTN_MAX_RANK];
    int64_t st = 1;
    for (int l = B.rank - 1; l >= 0; --l) {
      stride[l] = st;
      st *= B.dim(b, l);
    }
    for (int c = 0; c < nc; ++c) bb.sc[c] = (int32_t)stride[hp.axes_b[c]];
    for (int q = 0; q < hp.nfb; ++q) bb.sf[q] = (int32_t)stride[hp.fb[q]];
    t.bblocks.push_back(bb);
  }
  // ---- sectors, tuples, grids, pack items, tiles
  yastn_stats &S = hp.stats;
  S = yastn_stats{};
  S.blocks_a = A.nblocks;
  S.blocks_b = B.nblocks;
  S.pairs = (int64_t)pairs.size();
  S.sectors = (int64_t)nS;
  S.c_blocks = (int64_t)ck.size();
  S.c_numel = hp.c_numel;
  S.numel_a = A.numel;
  S.numel_b = B.numel;
  std::vector<u128> rk, sk, jk;  // the sector's distinct row / contracted / column tuple keys, ascending
  for (int x = 0; x < nS; ++x) {
    const int32_t p0 = scount[x], p1 = scount[x + 1];
    rk.clear();
    sk.clear();
    jk.clear();
    for (int32_t u = p0; u < p1; ++u) {
      const auto &pr = pairs[size_t(sorder[u])];
      rk.push_back(ar[pr.first]);
      sk.push_back(ac[pr.first]);
      jk.push_back(bj[pr.second]);
    }
    sort_unique(rk);
    sort_unique(sk);
    sort_unique(jk);
    const int R = (int)rk.size(), Sn = (int)sk.size(), Q = (int)jk.size();
    DevSector ds{};
    ds.prob = prob;
    ds.S = Sn;
    ds.Q = Q;
    ds.ctr0 = (int32_t)t.ctrs.size();
    ds.col0 = (int32_t)t.cols.size();
    ds.nact = nact;
    // representative blocks for the dims of each tuple
    std::vector<int64_t> row_rep(R, -1), ctr_rep(Sn, -1), col_rep(Q, -1);
    std::vector<int32_t> agrid(size_t(R) * Sn, -1), bgrid(size_t(Sn) * Q, -1);
    for (int32_t u = p0; u < p1; ++u) {
      const auto &pr = pairs[size_t(sorder[u])];
      const int i = rank_of(rk, ar[pr.first]), s = rank_of(sk, ac[pr.first]), j = rank_of(jk, bj[pr.second]);
      row_rep[i] = pr.first;
      ctr_rep[s] = pr.first;
      col_rep[j] = pr.second;
      agrid[size_t(i) * Sn + s] = (int32_t)(a_base + pr.first);
      bgrid[size_t(s) * Q + j] = (int32_t)(b_base + pr.second);
    }
    // contracted tuples (K space, ascending charge order)
    int32_t K = 0;
    for (int s = 0; s < Sn; ++s) {
      DevCtrTuple ct{};
      int64_t ia = ctr_rep[s];
      int64_t k = 1;
      for (int c = 0; c < nc; ++c) {
        ct.dims[c] = (int32_t)A.dim(ia, hp.axes_a[c]);
        k *= ct.dims[c];
      }
      ct.k = (int32_t)k;
      ct.ko = K;
      for (int c = 0; c < nc; ++c) {
        int64_t p = 1;
        for (int l = hp.axes_a[c] + 1; l < A.rank; ++l)
          if (isctr[l]) p *= A.dim(ia, l);
        ct.cac[c] = (int32_t)p;
      }
      for (int a = 0; a < nact; ++a) {
        int64_t p = 1;
        for (int g = 0; g < act_g[a]; ++g) p *= ct.dims[ctr_storage[nct - 1 - g]];
        ct.p[a] = (int32_t)p;
      }
      K += ct.k;
      t.ctrs.push_back(ct);
    }
    ds.K = K;
    // digits of each contracted index k of the sector within its tuple (C
    // order over the contracted legs in axes order)
    std::vector<int32_t> kdig(size_t(K) * std::max(1, nc));
    for (int s = 0; s < Sn; ++s) {
      const DevCtrTuple &ct = t.ctrs[ds.ctr0 + s];
      for (int32_t kd = 0; kd < ct.k; ++kd) {
        int32_t r = kd;
        for (int c = nc - 1; c >= 0; --c) {
          kdig[size_t(ct.ko + kd) * nc + c] = r % ct.dims[c];
          r /= ct.dims[c];
        }
      }
    }
    int32_t N = 0;
    for (int j = 0; j < Q; ++j) {
      DevColTuple ctp{};
      int64_t n = 1;
      for (int q = 0; q < hp.nfb; ++q) {
        ctp.dims[q] = (int32_t)B.dim(col_rep[j], hp.fb[q]);
        n *= ctp.dims[q];
      }
      ctp.n = (int32_t)n;
      ctp.no = N;
      N += ctp.n;
      t.cols.push_back(ctp);
    }
    ds.N = N;
    ds.bpack = t.bpack_elems;
    t.bpack_elems += int64_t(K) * N;
    // P_a of every contracted index, and the column map of C_X / B_X
    ds.kp0 = (int64_t)t.kp.size();
    for (int s = 0; s < Sn; ++s) {
      const DevCtrTuple &ct = t.ctrs[ds.ctr0 + s];
      DevKP kp{};
      for (int a = 0; a < kMaxAct; ++a) kp.p[a] = ct.p[a];
      for (int k = 0; k < ct.k; ++k) t.kp.push_back(kp);
    }
    ds.cm0 = (int64_t)t.colmap.size();
    for (int j = 0; j < Q; ++j) {
      const DevColTuple &cl = t.cols[ds.col0 + j];
      for (int c = 0; c < cl.n; ++c) t.colmap.push_back(DevColMap{j, c, cl.n, 0});
    }
    // element offset in B's buffer of every (k, column) of B_X (-1: sub-block absent)
    ds.bofs0 = (int64_t)t.bofs.size();
    t.bofs.resize(t.bofs.size() + size_t(K) * N, -1);
    bool sec_over = !gather || int64_t(K) * N > INT32_MAX || hp.b.numel == 0;  // gathers read B[0] for absent entries
    for (int s = 0; s < Sn; ++s)
      for (int j = 0; j < Q; ++j) {
        const int32_t blk = bgrid[size_t(s) * Q + j];
        if (blk < 0) continue;
        const DevCtrTuple &ct = t.ctrs[ds.ctr0 + s];
        const DevColTuple &cl = t.cols[ds.col0 + j];
        for (int32_t kd = 0; kd < ct.k; ++kd)
          for (int32_t cb = 0; cb < cl.n; ++cb) {
            const int64_t o = b_offset(t.bblocks[blk], ct, cl, t.probs[prob_slot], kd, cb);
            if (o > INT32_MAX) t.bofs_overflow = sec_over = true;
            t.bofs[ds.bofs0 + int64_t(ct.ko + kd) * N + cl.no + cb] = (int32_t)std::min<int64_t>(o, INT32_MAX);
          }
      }
    const int32_t sec_id = (int32_t)t.sectors.size();
    t.sectors.push_back(ds);
    t.sec_row0.push_back((int32_t)t.rows.size());
    if (!sec_over) {
      // gathers through the offset table: long coalesced runs, one table read each
      const int64_t total = int64_t(K) * N;
      for (int64_t e0 = 0; e0 < total; e0 += kGatherItem)
        t.items.push_back(DevPackItem{sec_id, -1, (int32_t)std::min<int64_t>(kGatherItem, total - e0), -1,
                                      (int32_t)e0, 0});
    } else {
      for (int s = 0; s < Sn; ++s)
        for (int j = 0; j < Q; ++j) {
          const int64_t total = int64_t(t.ctrs[ds.ctr0 + s].k) * t.cols[ds.col0 + j].n;
          for (int64_t e0 = 0; e0 < total; e0 += kPackItem)
            t.items.push_back(DevPackItem{sec_id, s, j, bgrid[size_t(s) * Q + j], (int32_t)e0, 0});
        }
    }
    int64_t M = 0;
    for (int i = 0; i < R; ++i) {
      DevRowTuple rt{};
      rt.sector = sec_id;
      int64_t ia = row_rep[i];
      int64_t m = 1;
      for (int q = 0; q < hp.nfa; ++q) m *= A.dim(ia, hp.fa[q]);
      rt.m = (int32_t)m;
      M += m;
      for (int a = 0; a <= nact; ++a) {
        int64_t p = 1;
        for (int q = 0; q < hp.nfa; ++q)
          if (fcls[q] >= a) p *= A.dim(ia, hp.fa[q]);
        rt.lsuf[a] = (int32_t)p;
        div_magic((uint32_t)p, &rt.lmag[a], &rt.lsh[a]);
      }
      for (int c = 0; c < nc; ++c) {
        int64_t p = 1;
        for (int q = 0; q < hp.nfa; ++q)
          if (hp.fa[q] > hp.axes_a[c]) p *= A.dim(ia, hp.fa[q]);
        rt.fac[c] = (int32_t)p;
      }
      rt.agrid = (int64_t)t.agrid.size();
      t.agrid.insert(t.agrid.end(), agrid.begin() + size_t(i) * Sn, agrid.begin() + size_t(i + 1) * Sn);
      // offset of A(row 0, k) for every contracted index k of the sector (-1: block absent)
      // (the digits of each contracted index are the sector's kdig table)
      rt.kofs = (int64_t)t.kofs.size();
      t.kofs.resize(t.kofs.size() + size_t(K));
      int64_t *ko = t.kofs.data() + rt.kofs;
      for (int s = 0; s < Sn; ++s) {
        const DevCtrTuple &ct = t.ctrs[ds.ctr0 + s];
        const int32_t blk = agrid[size_t(i) * Sn + s];
        if (blk < 0) {
          std::fill(ko + ct.ko, ko + ct.ko + ct.k, int64_t(-1));
          continue;
        }
        int64_t w[YASTN_MAX_RANK];
        for (int c = 0; c < nc; ++c) w[c] = (int64_t)rt.fac[c] * ct.cac[c];
        const int64_t base = t.aoff[blk];
        for (int32_t kd = 0; kd < ct.k; ++kd) {
          const int32_t *dg = &kdig[size_t(ct.ko + kd) * nc];
          int64_t koff = base;
          for (int c = 0; c < nc; ++c) koff += dg[c] * w[c];
          ko[ct.ko + kd] = koff;
        }
      }
      rt.cgrid = (int64_t)t.cgrid.size();
      for (int j = 0; j < Q; ++j) {
        const CKey key{rk[i], jk[j], 0, 0};
        auto it = std::lower_bound(ck.begin(), ck.end(), key);
        t.cgrid.push_back(it != ck.end() && *it == key ? hp.c_offsets[size_t(it - ck.begin())] : -1);
      }
      t.rows.push_back(rt);
    }
    S.max_m = std::max<int64_t>(S.max_m, M);
    S.max_k = std::max<int64_t>(S.max_k, K);
    S.max_n = std::max<int64_t>(S.max_n, N);
    for (int32_t u = p0; u < p1; ++u) {
      const auto &pr = pairs[size_t(sorder[u])];
      double m = 1, k = 1, n = 1;
      for (int q = 0; q < hp.nfa; ++q) m *= double(A.dim(pr.first, hp.fa[q]));
      for (int c = 0; c < nc; ++c) k *= double(A.dim(pr.first, hp.axes_a[c]));
      for (int q = 0; q < hp.nfb; ++q) n *= double(B.dim(pr.second, hp.fb[q]));
      S.useful_flops += 2.0 * m * k * n;
    }
  }
  return YASTN_OK;
}

void build_tiles(Plan &plan, int rb, int cb, int nch, bool ksplit) {
  PlanTables &t = plan.t;
  const int TN = 16 * cb, TM = 16 * rb * nch;
  plan.rb = rb;
  plan.cb = cb;
  plan.nch = nch;
  t.tiles.clear();
  t.red.clear();
  plan.prob_t0.assign(plan.probs.size(), 0);
  for (auto &hp : plan.probs) {
    hp.stats.tiles = 0;
    hp.stats.mfma_flops = 0.0;
  }
  const int nsec = (int)t.sectors.size();
  int prev = -1;
  for (int x = 0; x < nsec; ++x) {
    const DevSector &ds = t.sectors[x];
    const int prob = ds.prob;
    for (int p = prev + 1; p <= prob; ++p) plan.prob_t0[p] = (int32_t)t.tiles.size();
    prev = prob;
    yastn_stats &S = plan.probs[prob].stats;
    const int32_t r0 = t.sec_row0[x], r1 = x + 1 < nsec ? t.sec_row0[x + 1] : (int32_t)t.rows.size();
    const int32_t K = ds.K, N = ds.N;
    // split-K only for sectors with few output tiles (small M_X x N_X, e.g.
    // the gradient with respect to a site tensor): the partial slots cost
    // nslots x the tile's accumulators of workspace and a reduction pass
    int64_t Msec = 0;
    for (int32_t i = r0; i < r1; ++i) Msec += t.rows[i].m;
    const bool split_sec = ksplit && K > kSplitMinK && Msec * int64_t(N) <= kSplitMaxMN;
    // split-K: a sector with a long K (few, long tiles: small M and N) is
    // computed in nslots k ranges by separate tiles (same output tile), each
    // into its own partial slot, summed afterwards in slot order
    int32_t nslots = 1, chunk = K;
    if (split_sec) {
      nslots = (int32_t)std::min<int64_t>(kSplitMaxSlots, (K + kSplitChunk - 1) / kSplitChunk);
      chunk = (int32_t)(((K + nslots - 1) / nslots + 7) / 8 * 8);
      nslots = (int32_t)((K + chunk - 1) / chunk);
    }
    for (int32_t row_id = r0; row_id < r1; ++row_id) {
      const int32_t m = t.rows[row_id].m;
      for (int32_t m0 = 0; m0 < m; m0 += TM)
        for (int32_t n0 = 0; n0 < N; n0 += TN) {
          DevTile tl{};
          tl.rowtuple = row_id;
          tl.sector = x;
          tl.m0 = m0;
          tl.n0 = n0;
          tl.nrows = std::min<int32_t>(TM, m - m0);
          tl.ncols = std::min<int32_t>(TN, N - n0);
          tl.red = -1;
          if (nslots > 1) {
            tl.red = (int32_t)t.red.size();
            t.red.push_back(RedGroup{prob, row_id, x, m0, n0, tl.nrows, tl.ncols, nslots});
          }
          for (int32_t sl = 0; sl < nslots; ++sl) {
            tl.k0 = sl * chunk;
            tl.kn = (int32_t)std::min<int64_t>(chunk, K - tl.k0);
            tl.part = sl;
            t.tiles.push_back(tl);
            S.tiles += 1;
            S.mfma_flops += 2.0 * (16.0 * ((tl.nrows + 15) / 16)) * (4.0 * ((tl.kn + 3) / 4)) *
                            (16.0 * ((tl.ncols + 15) / 16));
          }
        }
    }
  }
  for (int p = prev + 1; p < (int)plan.probs.size(); ++p) plan.prob_t0[p] = (int32_t)t.tiles.size();
}

void finish_tiles(Plan &plan) {
  PlanTables &t = plan.t;
  const size_t in_b = plan.opts.in_dtype == YASTN_DTYPE_F64 ? 8 : 4;
  const size_t out_b = plan.opts.out_dtype == YASTN_DTYPE_F64 ? 8 : 4;
  for (auto &hp : plan.probs)
    hp.stats.alg_bytes = double(hp.a.numel + hp.b.numel) * in_b + double(hp.c_numel) * out_b;
  // longest tiles first within each launch group, so the waves that start
  // last get the short tiles.  (Keeping tiles of one sector side by side, for
  // cache sharing, measured slower: neighbouring waves then stream the same
  // rows of A and C and contend for the same memory channels.)
  const int np = (int)plan.probs.size();
  plan.prob_t0.push_back((int32_t)t.tiles.size());
  plan.prob_i0.push_back((int32_t)t.items.size());
  plan.groups.clear();
  t.ljobs.clear();
  for (int p0 = 0; p0 < np; p0 += kMaxTableProbs) {
    Group g{};
    g.plo = p0;
    g.phi = std::min(np, p0 + kMaxTableProbs);
    g.t0 = plan.prob_t0[g.plo];
    g.t1 = plan.prob_t0[g.phi];
    g.i0 = plan.prob_i0[g.plo];
    g.i1 = plan.prob_i0[g.phi];
    g.r0 = g.r1 = 0;
    while (g.r0 < (int32_t)t.red.size() && t.red[g.r0].prob < g.plo) ++g.r0;
    g.r1 = g.r0;
    while (g.r1 < (int32_t)t.red.size() && t.red[g.r1].prob < g.phi) ++g.r1;
    std::vector<double> cost(size_t(g.t1 - g.t0));
    for (int32_t i = g.t0; i < g.t1; ++i) {
      const DevTile &tl = t.tiles[i];
      double rows = 16.0 * ((tl.nrows + 15) / 16), cols = 16.0 * ((tl.ncols + 15) / 16);
      double k4 = 4.0 * ((tl.kn + 3) / 4);
      cost[i - g.t0] = 2.0 * rows * k4 * cols / 9.8 + 8.0 * tl.nrows * (double(tl.kn) + tl.ncols);
    }
    std::vector<size_t> order(cost.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<DevTile> sorted(order.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = t.tiles[g.t0 + order[i]];
    std::copy(sorted.begin(), sorted.end(), t.tiles.begin() + g.t0);
    // shared-B jobs: the tiles of each (sector, k range, column range) in
    // runs of kLdsJobTiles (costliest first, so wave w's two tiles are the
    // w-th and (w+4)-th costliest of the run); jobs costliest first
    {
      std::vector<double> tcost(order.size());
      for (size_t i = 0; i < order.size(); ++i) tcost[i] = cost[order[i]];
      std::vector<int32_t> byk(order.size());
      std::iota(byk.begin(), byk.end(), 0);
      auto key = [&](int32_t i) {
        const DevTile &tl = t.tiles[g.t0 + i];
        return std::make_tuple(tl.sector, tl.k0, tl.n0);
      };
      std::stable_sort(byk.begin(), byk.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
      std::vector<std::pair<double, DevLdsJob>> jobs;
      for (size_t i = 0; i < byk.size();) {
        size_t e = i;
        while (e < byk.size() && key(byk[e]) == key(byk[i])) ++e;
        for (size_t s0 = i; s0 < e; s0 += kLdsJobTiles) {
          DevLdsJob lj{};
          double wave[4] = {0, 0, 0, 0};
          for (int u = 0; u < kLdsJobTiles; ++u) {
            const bool in = s0 + u < e;
            lj.t[u] = in ? g.t0 + byk[s0 + u] : -1;
            if (in) wave[u % 4] += tcost[byk[s0 + u]];
          }
          jobs.push_back({*std::max_element(wave, wave + 4), lj});
        }
        i = e;
      }
      std::stable_sort(jobs.begin(), jobs.end(),
                       [](const std::pair<double, DevLdsJob> &x, const std::pair<double, DevLdsJob> &y) {
                         return x.first > y.first;
                       });
      g.l0 = (int32_t)t.ljobs.size();
      for (auto &jj : jobs) t.ljobs.push_back(jj.second);
      g.l1 = (int32_t)t.ljobs.size();
    }
    plan.groups.push_back(g);
  }
  const size_t elem = plan.opts.precision == YASTN_F64 ? 8 : 4;
  plan.norm_off = ((size_t(t.bpack_elems) * elem + 255) / 256) * 256;
  plan.ws_bytes = plan.norm_off + ((t.tiles.size() * 2 * sizeof(double) + 255) / 256) * 256;
  // problem pointer table of a group of more than kMaxProbs problems
  plan.ptab_off = plan.ws_bytes;
  if (np > kMaxProbs) plan.ws_bytes += ((size_t(std::min(np, kMaxTableProbs)) * sizeof(ProbPtrs) + 255) / 256) * 256;
  // split-K partial slots (accumulators of the compute type, 64 columns a row)
  for (RedGroup &r : t.red) {
    r.off0 = (int64_t)plan.ws_bytes;
    r.slot_bytes = (int64_t)(((size_t(r.nrows) * 64 * elem + 255) / 256) * 256);
    plan.ws_bytes += size_t(r.slot_bytes) * r.nslots;
  }
}

void build_tile_records(const Plan &plan, const DevPlan &at, std::vector<DevTileRec> &recs) {
  const PlanTables &t = plan.t;
  recs.assign(t.tiles.size(), DevTileRec{});
  for (size_t i = 0; i < t.tiles.size(); ++i) {
    const DevTile &tl = t.tiles[i];
    const DevRowTuple &rt = t.rows[tl.rowtuple];
    const DevSector &sec = t.sectors[tl.sector];
    const DevProb &pr = t.probs[sec.prob];
    DevTileRec &r = recs[i];
    r.kofs = at.kofs + rt.kofs + tl.k0;
    r.kp = at.kp + sec.kp0 + tl.k0;
    r.bofs = at.bofs + sec.bofs0 + int64_t(tl.k0) * sec.N;
    r.cmap = at.colmap + sec.cm0 + tl.n0;
    r.cgrid = at.cgrid + rt.cgrid;
    r.a_span = pr.a_span;
    r.b_span = pr.b_span;
    r.c_numel = pr.c_numel;
    r.m0 = tl.m0;
    r.nrows = tl.nrows;
    r.n0 = tl.n0;
    r.ncols = tl.ncols;
    r.K = tl.kn;
    r.N = sec.N;
    r.nact = sec.nact;
    r.prob = sec.prob;
    r.bpack = sec.bpack + int64_t(tl.k0) * sec.N;
    r.split = tl.red >= 0 ? 1 : 0;
    r.part = tl.red >= 0 ? t.red[tl.red].off0 + int64_t(tl.part) * t.red[tl.red].slot_bytes : 0;
    for (int a = 0; a < kRecAct; ++a) {
      r.lsuf[a] = a + 1 <= sec.nact ? rt.lsuf[a + 1] : 1;
      r.lsh[a] = a + 1 <= sec.nact ? rt.lsh[a + 1] : 31;
      r.lmag[a] = a + 1 <= sec.nact ? rt.lmag[a + 1] : (1u << 31);
    }
  }
}

}  // namespace yastn
