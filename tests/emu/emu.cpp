// CPU replay of the library's plan and kernel indexing (test harness).
//
// Builds a plan with the library's own host planner (host.cpp) and address
// helpers (index.hpp), matching blocks with a plain host map instead of the
// device hash join, then replays the pack and grouped-GEMM loops of the HIP
// kernels element by element, with the kernels' guards, checking every read
// and write against its buffer and that every output element is written
// exactly once.  FP64 arithmetic, any summation order.
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

void *emu_plan(const yastn_problem *probs, int nprob, int cb_override) {
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
  pl.cb = cb_override;
  int64_t ab = 0, bb = 0;
  for (int p = 0; p < nprob; ++p) {
    pl.prob_t0.push_back((int32_t)pl.t.tiles.size());
    pl.prob_i0.push_back((int32_t)pl.t.items.size());
    if (build_structure(pl.probs[p], p, pairs[p], ab, bb, pl.t, pl.cb) != YASTN_OK) {
      g_msg = "build_structure failed";
      delete e;
      return nullptr;
    }
    ab += pl.probs[p].a.nblocks;
    bb += pl.probs[p].b.nblocks;
  }
  finish_tiles(pl);
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
  // ---- k_pack_b
  for (int g = 0; g < P.nitems; ++g) {
    const DevPackItem it = P.items[g];
    const DevSector sec = P.sectors[it.sector];
    const DevCtrTuple &ct = P.ctrs[sec.ctr0 + it.s];
    const DevColTuple &cl = P.cols[sec.col0 + it.j];
    const DevProb pr = P.probs[sec.prob];
    const int64_t base = sec.bpack + (int64_t)ct.ko * sec.N + cl.no;
    const int64_t total = (int64_t)ct.k * cl.n;
    for (int64_t el = 0; el < total; ++el) {
      const int64_t kd = el / cl.n, cb = el - kd * cl.n;
      const int64_t d = base + kd * sec.N + cb;
      if (d < sec.bpack || d >= sec.bpack + (int64_t)sec.K * sec.N) return fail("pack: write outside B_X");
      if (packed[d]++) return fail("pack: element written twice");
      if (it.bblk < 0) {
        ws[d] = 0.0;
        continue;
      }
      const int64_t o = b_offset(P.bblocks[it.bblk], ct, cl, pr, kd, cb);
      if (o < 0 || o >= blen[sec.prob]) return fail("pack: B read out of bounds");
      ws[d] = b[sec.prob][o];
    }
  }
  for (int64_t i = 0; i < pl.t.bpack_elems; ++i)
    if (packed[i] != 1) return fail("pack: packed B element not written");
  // ---- k_gemm4 (tile, row, column, k loops with the kernel's guards)
  std::vector<std::vector<char>> wrote(pl.probs.size());
  for (size_t p = 0; p < pl.probs.size(); ++p) wrote[p].assign(size_t(clen[p]) + 1, 0);
  for (int t = 0; t < P.ntiles; ++t) {
    const DevTile tile = P.tiles[t];
    const DevRowTuple rt = P.rows[tile.rowtuple];
    const DevSector sec = P.sectors[rt.sector];
    const DevProb pr = P.probs[sec.prob];
    if (tile.nrows > kWaveRows || tile.ncols > 16 * pl.cb) return fail("tile larger than a wave tile");
    const double *Bp = ws.data() + sec.bpack;
    std::vector<double> acc(size_t(kWaveRows) * 16 * pl.cb, 0.0);
    for (int k0 = 0; k0 < sec.K; k0 += kKChunk) {
      const int kend = std::min(sec.K, k0 + kKChunk);
      if (kend - k0 > kKChunk) return fail("offset table overflow");
      for (int k = k0; k < kend; ++k) {
        int32_t pk[kMaxAct];
        const int64_t koff = a_koffset(P, rt, sec, pr, k, pk);
        for (int lr = 0; lr < tile.nrows; ++lr) {
          int32_t rg[kMaxAct];
          a_rowparts(rt, pr.nact, tile.m0 + lr, rg);
          double av = 0.0;
          if (koff >= 0) {
            const int64_t o = a_offset(koff, pk, rg);
            if (o < 0 || o >= alen[sec.prob]) return fail("gemm: A read out of bounds");
            av = a[sec.prob][o];
          }
          for (int lc = 0; lc < 16 * pl.cb; ++lc) {
            const int col = tile.n0 + lc;
            if (col >= sec.N) continue;
            const int64_t bi = (int64_t)k * sec.N + col;
            if (bi >= (int64_t)sec.K * sec.N) return fail("gemm: packed B read out of bounds");
            acc[size_t(lr) * 16 * pl.cb + lc] += av * Bp[bi];
          }
        }
      }
    }
    const DevColTuple *cols = P.cols + sec.col0;
    for (int lc = 0; lc < 16 * pl.cb; ++lc) {
      const int col = tile.n0 + lc;
      if (col >= sec.N || col >= tile.n0 + tile.ncols) continue;
      const int j = find_col(cols, sec.Q, col);
      const int64_t cbase = P.cgrid[rt.cgrid + j];
      if (cbase < 0) continue;
      const int64_t nj = cols[j].n, cl = col - cols[j].no;
      for (int lr = 0; lr < tile.nrows; ++lr) {
        const int64_t o = cbase + (int64_t)(tile.m0 + lr) * nj + cl;
        if (o < 0 || o >= clen[sec.prob]) return fail("gemm: C write out of bounds");
        if (wrote[sec.prob][o]++) return fail("gemm: C element written twice");
        c[sec.prob][o] = acc[size_t(lr) * 16 * pl.cb + lc];
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
