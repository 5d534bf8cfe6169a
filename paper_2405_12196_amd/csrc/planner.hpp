// Host-side plan structures (validation, structure building, tiling).
#pragma once
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/yastn.h"
#include "plan.hpp"

namespace yastn {

struct HostTensor {
  int rank = 0, nsym = 0;
  int32_t sym_mod[YASTN_MAX_NSYM] = {0};
  int8_t sig[YASTN_MAX_RANK] = {0};
  int32_t n[YASTN_MAX_NSYM] = {0};
  int64_t nblocks = 0;
  std::vector<int32_t> charges;  // [nblocks][rank][nsym], Z_m components reduced into [0, m)
  std::vector<int64_t> shapes;   // [nblocks][rank]
  std::vector<int64_t> offsets;  // [nblocks]
  int64_t numel = 0;             // stored elements (sum of block sizes)
  // distinct charges of each leg in ascending (lexicographic) order, set by
  // validation: qid[b * rank + l] = index of block b's charge on leg l
  // among the nq[l] distinct charges of leg l; legq / legdim hold those
  // charges (nsym ints each) and their dims, leg l from entry legq0[l]
  std::vector<int32_t> qid;
  int32_t nq[YASTN_MAX_RANK] = {0};
  std::vector<int32_t> legq;
  std::vector<int64_t> legdim;
  int64_t legq0[YASTN_MAX_RANK + 1] = {0};
  const int32_t *q(int64_t b, int leg) const { return &charges[(b * rank + leg) * nsym]; }
  int64_t dim(int64_t b, int leg) const { return shapes[b * rank + leg]; }
  int64_t size(int64_t b) const;
};

struct HostProblem {
  HostTensor a, b;
  int nc = 0;
  int axes_a[YASTN_MAX_RANK] = {0}, axes_b[YASTN_MAX_RANK] = {0};
  int nfa = 0, nfb = 0;
  int fa[YASTN_MAX_RANK] = {0}, fb[YASTN_MAX_RANK] = {0};
  // output C (rule: A free legs then B free legs, ascending charge order)
  int c_rank = 0;
  int8_t c_sig[YASTN_MAX_RANK] = {0};
  int32_t c_n[YASTN_MAX_NSYM] = {0};
  std::vector<int32_t> c_charges;
  std::vector<int64_t> c_shapes, c_offsets;
  int64_t c_numel = 0;
  yastn_stats stats{};
};

// A split-K group on the host (see DevRedItem): one output tile whose K range
// is computed by nslots tiles into partial slots.
struct RedGroup {
  int32_t prob, rowtuple, sector, m0, n0, nrows, ncols, nslots;
  int64_t off0 = 0, slot_bytes = 0;  // set when the workspace is laid out
};

// Device tables of a plan, built on the host and uploaded once.
struct PlanTables {
  std::vector<DevProb> probs;
  std::vector<DevSector> sectors;
  std::vector<DevRowTuple> rows;
  std::vector<DevCtrTuple> ctrs;
  std::vector<DevColTuple> cols;
  std::vector<int32_t> agrid;
  std::vector<int64_t> aoff;
  std::vector<int64_t> cgrid;
  std::vector<DevBBlock> bblocks;
  std::vector<DevTile> tiles;
  std::vector<DevPackItem> items;
  std::vector<int64_t> kofs;
  std::vector<DevKP> kp;
  std::vector<DevColMap> colmap;
  std::vector<int32_t> bofs;
  int64_t bpack_elems = 0;  // packed B elements in the workspace
  bool bofs_overflow = false;  // some B offset does not fit in int32 (no direct B reads then)
  std::vector<RedGroup> red;   // split-K groups, in problem order
  std::vector<DevLdsJob> ljobs;  // shared-B workgroup jobs, per group
  std::vector<int32_t> sec_row0;  // first row tuple of each sector (a sector's row tuples are contiguous)
};

// Problems are launched in groups: all of a plan's problems in one group (up
// to kMaxTableProbs); a group of at most kMaxProbs problems takes its device
// pointers as kernel arguments, a larger one from a table in the workspace.
// Tiles are cost-sorted within a group.
struct Group {
  int32_t plo, phi;          // problems [plo, phi)
  int32_t t0, t1;            // plan-local tiles
  int32_t i0, i1;            // plan-local pack items
  int32_t r0, r1;            // split-K groups of these problems
  int32_t l0, l1;            // shared-B jobs of these problems
};

struct Plan {
  std::vector<HostProblem> probs;
  std::vector<int32_t> prob_t0, prob_i0;  // first tile / item of each problem (before sorting)
  std::vector<Group> groups;
  yastn_options opts{};
  PlanTables t;
  int cb = 4;               // column blocks (16 columns each) per wave tile
  int rb = 4;               // row blocks (16 rows each) per chunk of a wave tile
  int nch = 1;              // chunks per wave tile
  bool buf_ok = true;       // every buffer small enough for 32-bit buffer addressing
  bool rows_fit = false;    // every sector has K, N <= 64: the row-per-lane kernel can run
  bool res_fit = false;     // every sector has K <= 80 and B offsets fit int32: k_gemm_res can run
  bool pair_ok = false;     // A's rows run contiguously in even-length runs: paired-row loads can run
  bool ldsk_fit = false;    // B offsets fit int32, rows and block widths below 2^24: the K-chunked shared-B kernel can run
  int nact = 1;             // largest number of A free-leg classes over the plan's problems
  int variant = 0;          // tuned kernel variant (0 = not tuned; set by yastn_plan_autotune)
  uint64_t tkey[2] = {0, 0};  // the request's fingerprint in the tuning store (valid if have_tkey)
  bool have_tkey = false;
  float tuned_ms[YASTN_NUM_VARIANTS] = {0};  // the tuning run's times (ms per launch, -1 = does not fit)
  int kmax = 0;             // largest K_X of the plan
  void *dev_mem = nullptr;  // one device allocation holding every table
  DevPlan *dplan = nullptr; // device copy of the table of pointers
  const DevTileRec *drecs = nullptr;  // device tile records
  const DevRedItem *dred = nullptr;   // device split-K groups (null when none)
  const DevLdsJob *dljobs = nullptr;  // device shared-B jobs
  const DevTileRec *dljrecs = nullptr;  // device records of the shared-B jobs' tiles, in job order
  size_t ws_bytes = 0;
  size_t norm_off = 0;      // workspace offset of the fused norm's per-tile parts
  size_t ptab_off = 0;      // workspace offset of the problem pointer table (groups of > kMaxProbs problems)
  int device = 0;
  double prof_ms[4] = {0, 0, 0, 0};  // planning time: validation, join, host tables, upload
};

// error reporting (thread-local message)
yastn_status set_error(yastn_status s, const std::string &msg);

// host.cpp
yastn_status check_options(const yastn_options *o, yastn_options *out);
yastn_status validate_problem(const yastn_problem &p, HostProblem &hp);
// one tensor alone: symmetry, signatures, dims, duplicates, conservation, offsets
yastn_status validate_tensor(const yastn_tensor_desc &d, const char *name, HostTensor &t);
void contracted_keys(const HostTensor &t, const int *axes, int nc, std::vector<int32_t> &keys);
// ksplit: sectors with K > kSplitMinK and M_X * N_X <= kSplitMaxMN are
// computed in k ranges (split-K); the caller passes ksplit only when the
// pipelined kernel (the one that writes partial slots) can run the plan.
// gather: pack B through the offset table where it fits (else sub-block items)
constexpr int64_t kSplitMinK = 4096, kSplitChunk = 1024, kSplitMaxSlots = 256, kSplitMaxMN = 64 * 64 * 16;
// Tables of one problem (structure, sectors, tuples, offsets, pack items);
// no tiles yet.
yastn_status build_structure(HostProblem &hp, int prob, const std::vector<std::pair<int32_t, int32_t>> &pairs,
                             int64_t a_base, int64_t b_base, PlanTables &t, bool gather = true);
// Wave tiles of every problem (16 * rb * nch rows x 16 * cb columns), the
// split-K groups, prob_t0 and the tile statistics.
void build_tiles(Plan &plan, int rb, int cb, int nch, bool ksplit);
void finish_tiles(Plan &plan);
// Tile records with absolute addresses: `at` gives the address of each table
// (device addresses for the GPU, host vector data for the CPU replay).
void build_tile_records(const Plan &plan, const DevPlan &at, std::vector<DevTileRec> &recs);

}  // namespace yastn
