// CPU replay of the library's plan and kernel indexing (test harness).
//
// Builds a plan with the library's own host planner (host.cpp) and address
// helpers (index.hpp), matching blocks with a plain host map instead of the
// device hash join, then replays the pack and grouped-GEMM loops of the HIP
// kernels element by element, with the kernels' guards, checking every read
// and write against its buffer and that every output element is written
// exactly once.  FP64 arithmetic, any summation order.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../paper_2405_12196_amd/csrc/index.hpp"
#include "../../paper_2405_12196_amd/csrc/planner.hpp"

using namespace yastn;

namespace {
std::string g_msg;
bool g_gather = true;  // pack form of the plans built next
struct Emu {
  Plan pl;
  DevPlan dp;
};
int fail(const std::string &m) {
  g_msg = m;
  return -1;
}
}  // namespace

extern "C" {

const char *emu_error() { return g_msg.c_str(); }
void emu_set_pack_gather(int on) { g_gather = on != 0; }

void *emu_plan(const yastn_problem *probs, int nprob, int rb_override, int cb_override) {
  Emu *e = new Emu();
  Plan &pl = e->pl;
  check_options(nullptr, &pl.opts);
  pl.probs.resize(nprob);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> pairs(nprob);
  for (int p = 0; p < nprob; ++p) {
    if (validate_problem(probs[p], pl.probs[p]) != YASTN_OK) {
      g_msg = "validation failed";
      delete e;
      return nullptr;
    }
    HostProblem &hp = pl.probs[p];
    std::vector<int32_t> ka, kb;
    contracted_keys(hp.a, hp.axes_a, hp.nc, ka);
    contracted_keys(hp.b, hp.axes_b, hp.nc, kb);
    const int kl = hp.nc * hp.a.nsym;
    std::map<std::vector<int32_t>, std::vector<int32_t>> byk;
    for (int64_t j = 0; j < hp.b.nblocks; ++j)
      byk[std::vector<int32_t>(kb.begin() + j * kl, kb.begin() + (j + 1) * kl)].push_back((int32_t)j);
    for (int64_t i = 0; i < hp.a.nblocks; ++i) {
      auto it = byk.find(std::vector<int32_t>(ka.begin() + i * kl, ka.begin() + (i + 1) * kl));
      if (it != byk.end())
        for (int32_t j : it->second) pairs[p].push_back({(int32_t)i, j});
    }
  }
  int64_t ab = 0, bb = 0;
  for (int p = 0; p < nprob; ++p) {
    pl.prob_i0.push_back((int32_t)pl.t.items.size());
    if (build_structure(pl.probs[p], p, pairs[p], ab, bb, pl.t, g_gather) != YASTN_OK) {
      g_msg = "build_structure failed";
      delete e;
      return nullptr;
    }
    ab += pl.probs[p].a.nblocks;
    bb += pl.probs[p].b.nblocks;
  }
  // exercise multi-chunk tiles too
  build_tiles(pl, rb_override, cb_override, 1 + (rb_override == 2), false);
  finish_tiles(pl);
  // shared-B jobs (k_gemm_lds): per group, every tile exactly once, the tiles
  // of a job on one (sector, k range, column range), its first slot filled
  for (const Group &g : pl.groups) {
    std::vector<int> seen(size_t(g.t1 - g.t0), 0);
    for (int32_t j = g.l0; j < g.l1; ++j) {
      const DevLdsJob &lj = pl.t.ljobs[j];
      if (lj.t[0] < 0) {
        g_msg = "ljobs: empty first slot";
        delete e;
        return nullptr;
      }
      const DevTile &t0 = pl.t.tiles[lj.t[0]];
      for (int u = 0; u < kLdsJobTiles; ++u) {
        const int32_t ti = lj.t[u];
        if (ti < 0) continue;
        const DevTile &tu = pl.t.tiles[ti];
        if (ti < g.t0 || ti >= g.t1 || seen[ti - g.t0]++ || tu.sector != t0.sector || tu.k0 != t0.k0 ||
            tu.n0 != t0.n0 || tu.ncols != t0.ncols) {
          g_msg = "ljobs: tile outside its group, repeated, or on another B tile";
          delete e;
          return nullptr;
        }
      }
    }
    for (int v : seen)
      if (v != 1) {
        g_msg = "ljobs: a tile of the group is in no job";
        delete e;
        return nullptr;
      }
  }
  DevPlan &d = e->dp;
  d.probs = pl.t.probs.data();
  d.sectors = pl.t.sectors.data();
  d.rows = pl.t.rows.data();
  d.ctrs = pl.t.ctrs.data();
  d.cols = pl.t.cols.data();
  d.agrid = pl.t.agrid.data();
  d.aoff = pl.t.aoff.data();
  d.cgrid = pl.t.cgrid.data();
  d.bblocks = pl.t.bblocks.data();
  d.tiles = pl.t.tiles.data();
  d.items = pl.t.items.data();
  d.kofs = pl.t.kofs.data();
  d.kp = pl.t.kp.data();
  d.colmap = pl.t.colmap.data();
  d.bofs = pl.t.bofs.data();
  d.ntiles = (int32_t)pl.t.tiles.size();
  d.nitems = (int32_t)pl.t.items.size();
  return e;
}

int emu_output(void *h, int p, yastn_tensor_desc *c, int64_t *numel) {
  HostProblem &hp = static_cast<Emu *>(h)->pl.probs[p];
  c->rank = hp.c_rank;
  c->nsym = hp.a.nsym;
  c->sym_mod = hp.a.sym_mod;
  c->sig = hp.c_sig;
  c->n = hp.c_n;
  c->nblocks = (int64_t)hp.c_offsets.size();
  c->charges = hp.c_charges.data();
  c->shapes = hp.c_shapes.data();
  c->offsets = hp.c_offsets.data();
  *numel = hp.c_numel;
  return 0;
}

int emu_contract(void *h, const double *const *a, const int64_t *alen, const double *const *b,
                 const int64_t *blen, double *const *c, const int64_t *clen) {
  Emu *e = static_cast<Emu *>(h);
  const Plan &pl = e->pl;
  const DevPlan &P = e->dp;
  std::vector<double> ws(size_t(pl.t.bpack_elems) + 1, 0.0);
  std::vector<char> packed(size_t(pl.t.bpack_elems) + 1, 0);
  // ---- k_pack_b: a gather item = up to kGatherItem consecutive elements of B_X
  // through the offset table; a sub-block item = up to kPackItem elements of
  // one (s, j) sub-block
  for (int g = 0; g < P.nitems; ++g) {
    const DevPackItem it = P.items[g];
    const DevSector &sec = P.sectors[it.sector];
    if (it.s < 0) {
      const int64_t total = (int64_t)sec.K * sec.N;
      if (it.j < 1 || it.j > kGatherItem || it.e0 < 0 || it.e0 + (int64_t)it.j > total)
        return fail("pack: gather item outside B_X");
      if (blen[sec.prob] < 1) return fail("pack: gather item over an empty B");
      for (int tid = 0; tid < 256; ++tid)
        for (int r = 0; r < kGatherItem / 256; ++r) {
          const int32_t e = tid + 256 * r, ec = std::min(e, it.j - 1);  // the kernel's clamped read
          const int32_t o = P.bofs[sec.bofs0 + it.e0 + ec];
          if (std::max(o, 0) >= blen[sec.prob]) return fail("pack: gather B read out of bounds");
          if (e >= it.j) continue;
          const int64_t d = sec.bpack + it.e0 + e;
          if (packed[d]++) return fail("pack: element written twice");
          ws[d] = o >= 0 ? b[sec.prob][o] : 0.0;
        }
      continue;
    }
    const DevCtrTuple &ct = P.ctrs[sec.ctr0 + it.s];
    const DevColTuple &cl = P.cols[sec.col0 + it.j];
    for (int tid = 0; tid < kPackItem; ++tid) {
      const int32_t e = it.e0 + tid;
      if (e >= ct.k * cl.n) continue;
      const int32_t kd = e / cl.n, cb = e - kd * cl.n;
      const int64_t d = sec.bpack + (int64_t)(ct.ko + kd) * sec.N + cl.no + cb;
      if (d < sec.bpack || d >= sec.bpack + (int64_t)sec.K * sec.N) return fail("pack: write outside B_X");
      if (packed[d]++) return fail("pack: element written twice");
      if (it.bblk < 0) {
        ws[d] = 0.0;
        continue;
      }
      const int64_t o = b_offset(P.bblocks[it.bblk], ct, cl, P.probs[sec.prob], kd, cb);
      if (o < 0 || o >= blen[sec.prob]) return fail("pack: B read out of bounds");
      ws[d] = b[sec.prob][o];
    }
  }
  for (int64_t i = 0; i < pl.t.bpack_elems; ++i)
    if (packed[i] != 1) return fail("pack: packed B element not written");
  // ---- direct B reads (k_gemm_res): the offset table must give the packed values
  if ((int64_t)pl.t.bofs.size() != pl.t.bpack_elems) return fail("bofs: table size differs from packed B");
  for (size_t si = 0; si < pl.t.sectors.size(); ++si) {
    const DevSector &sec = P.sectors[si];
    for (int64_t e = 0; e < (int64_t)sec.K * sec.N; ++e) {
      const int32_t o = P.bofs[sec.bofs0 + e];
      const double want = ws[sec.bpack + e];
      if (o < 0) {
        if (want != 0.0) return fail("bofs: absent entry where packed B is non-zero");
        continue;
      }
      if (o >= blen[sec.prob]) return fail("bofs: B read out of bounds");
      if (b[sec.prob][o] != want) return fail("bofs: offset table disagrees with packed B");
    }
  }
  std::vector<DevTileRec> recs;
  build_tile_records(pl, P, recs);
  // ---- k_gemm4: per tile, the lane's rows / columns / k as the kernel forms them
  std::vector<std::vector<char>> wrote(pl.probs.size());
  for (size_t p = 0; p < pl.probs.size(); ++p) wrote[p].assign(size_t(clen[p]) + 1, 0);
  const int TM = 16 * pl.rb * pl.nch, TN = 16 * pl.cb;
  for (int t = 0; t < P.ntiles; ++t) {
    const DevTile tile = P.tiles[t];
    const DevRowTuple rt = P.rows[tile.rowtuple];
    const DevSector sec = P.sectors[rt.sector];
    const int nact = P.probs[sec.prob].nact;
    if (tile.nrows > TM || tile.ncols > TN) return fail("tile larger than a wave tile");
    const double *Bp = ws.data() + sec.bpack;
    const int64_t *kofs = P.kofs + rt.kofs;
    const DevKP *kp = P.kp + sec.kp0;
    if (rt.kofs + sec.K > (int64_t)pl.t.kofs.size() || sec.kp0 + sec.K > (int64_t)pl.t.kp.size())
      return fail("offset table overflow");
    // the tile record (what k_gemm_res reads) must describe this tile, and the
    // fast row split (multiply-high, from the record) must agree with the modulo form
    const DevTileRec &rec = recs[t];
    if (rec.kofs != P.kofs + rt.kofs || rec.kp != P.kp + sec.kp0 || rec.bofs != P.bofs + sec.bofs0 ||
        rec.cmap != P.colmap + sec.cm0 + tile.n0 || rec.cgrid != P.cgrid + rt.cgrid || rec.m0 != tile.m0 ||
        rec.nrows != tile.nrows || rec.n0 != tile.n0 || rec.ncols != tile.ncols || rec.K != sec.K || rec.N != sec.N ||
        rec.nact != nact || rec.prob != sec.prob || rec.bpack != sec.bpack || rec.a_span != P.probs[sec.prob].a_span ||
        rec.b_span != P.probs[sec.prob].b_span || rec.c_numel != P.probs[sec.prob].c_numel)
      return fail("tile record differs from the tables");
    DevRowTuple fromrec{};
    for (int a = 0; a < kRecAct; ++a) {
      fromrec.lsuf[a + 1] = rec.lsuf[a];
      fromrec.lmag[a + 1] = rec.lmag[a];
      fromrec.lsh[a + 1] = rec.lsh[a];
    }
    for (int lr = 0; lr < tile.nrows; ++lr) {
      int32_t r1[kMaxAct], r2[kMaxAct];
      a_rowparts(rt, nact, tile.m0 + lr, r1);
      a_rowparts_fast<kMaxAct>(fromrec, nact, tile.m0 + lr, r2);
      for (int a = 0; a < kMaxAct; ++a)
        if (r1[a] != r2[a]) return fail("fast row split disagrees with the modulo form");
    }
    std::vector<double> acc(size_t(TM) * TN, 0.0);
    for (int k = 0; k < sec.K; ++k) {
      const int64_t ko = kofs[k];
      const DevKP p = kp[k];
      for (int lr = 0; lr < TM; ++lr) {
        if (lr >= tile.nrows) continue;
        int32_t rg[kMaxAct];
        a_rowparts(rt, nact, tile.m0 + lr, rg);
        double av = 0.0;
        if (ko >= 0) {
          const int64_t o = a_offset(ko, p.p, rg);
          if (o < 0 || o >= alen[sec.prob]) return fail("gemm: A read out of bounds");
          av = a[sec.prob][o];
        }
        for (int lc = 0; lc < TN; ++lc) {
          const int col = tile.n0 + lc;
          if (col >= sec.N) continue;
          acc[size_t(lr) * TN + lc] += av * Bp[(int64_t)k * sec.N + col];
        }
      }
    }
    // k_gemm_res epilogue: 16-row blocks, walked one column tuple piece at a
    // time; every address it forms must be the one the per-element form gives
    for (int r0 = 0; r0 < tile.nrows; r0 += 16) {
      const int rrows = std::min(16, tile.nrows - r0);
      for (int cc0 = 0; cc0 < tile.ncols;) {
        const DevColMap cm = P.colmap[sec.cm0 + tile.n0 + cc0];
        const int w = std::min(cm.nj - cm.cl, tile.ncols - cc0);
        if (w < 1) return fail("res epilogue: empty column piece");
        const int64_t cbase = P.cgrid[rt.cgrid + cm.j];
        const float inv = 1.0f / (float)w;
        for (int e = 0; e < rrows * w && cbase >= 0; ++e) {
          const int r = (int)(((float)e + 0.5f) * inv);
          const int cc = e - r * w;
          if (r != e / w) return fail("res epilogue: float quotient inexact");
          const DevColMap cmx = P.colmap[sec.cm0 + tile.n0 + cc0 + cc];
          const int64_t want = P.cgrid[rt.cgrid + cmx.j] + (int64_t)(tile.m0 + r0 + r) * cmx.nj + cmx.cl;
          const int64_t got = cbase + (int64_t)(tile.m0 + r0) * cm.nj + cm.cl + (int64_t)r * cm.nj + cc;
          if (got != want) return fail("res epilogue: address differs from the per-element form");
        }
        cc0 += w;
      }
    }
    for (int lc = 0; lc < TN; ++lc) {
      if (lc >= tile.ncols) continue;
      if (sec.cm0 + tile.n0 + lc >= (int64_t)pl.t.colmap.size()) return fail("colmap overflow");
      const DevColMap cm = P.colmap[sec.cm0 + tile.n0 + lc];
      const int64_t cbase = P.cgrid[rt.cgrid + cm.j];
      if (cbase < 0) continue;
      for (int lr = 0; lr < tile.nrows; ++lr) {
        const int64_t o = cbase + (int64_t)(tile.m0 + lr) * cm.nj + cm.cl;
        if (o < 0 || o >= clen[sec.prob]) return fail("gemm: C write out of bounds");
        if (wrote[sec.prob][o]++) return fail("gemm: C element written twice");
        c[sec.prob][o] = acc[size_t(lr) * TN + lc];
      }
    }
  }
  for (size_t p = 0; p < pl.probs.size(); ++p)
    for (int64_t i = 0; i < clen[p]; ++i)
      if (wrote[p][i] != 1) return fail("gemm: C element never written");
  return 0;
}

void emu_free(void *h) { delete static_cast<Emu *>(h); }

}  // extern "C"
