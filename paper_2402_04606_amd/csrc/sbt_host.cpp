// Host engine behind the sbt_* C ABI: block-forest builder and validator,
// device memory plan, the level schedule of Algorithm 1 (unrolled into a
// static phase list), HIP graph capture, readout, checkpoint and tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "sbt.h"
#include "sbt_internal.h"

using namespace sbt;

namespace {

thread_local std::string g_err;

sbt_status fail(sbt_status code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(SBT_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t storage_bytes(int st) { return st == SBT_F64 ? 8 : (st == SBT_F32 ? 4 : 2); }

// LDS per workgroup on gfx950.
constexpr size_t kLdsBytes = 163840;

uint32_t morton(uint32_t x, uint32_t y) {
  auto spread = [](uint32_t v) {
    v &= 0xffff;
    v = (v | (v << 8)) & 0x00ff00ff;
    v = (v | (v << 4)) & 0x0f0f0f0f;
    v = (v | (v << 2)) & 0x33333333;
    v = (v | (v << 1)) & 0x55555555;
    return v;
  };
  return spread(x) | (spread(y) << 1);
}

const int DCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};  // opposite direction
const int DCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// ---------------------------------------------------------------------------
// Block forest of one case (Sec. 2.3): levels 0..m-1 of 16x16-cell blocks.
// region_l = union of the level-l boxes (level 0: the whole domain);
// own_l = region_l minus the cells covered by region_{l+1}.
// ---------------------------------------------------------------------------
struct Forest {
  int m = 1;
  bool per_x = false, per_y = false;
  int nx[kMaxLevels], ny[kMaxLevels], nbx[kMaxLevels], nby[kMaxLevels];
  std::vector<std::vector<uint8_t>> region;      // [l][by * nbx + bx]
  std::vector<std::vector<int>> own, ghost;      // block ids (by * nbx + bx), Morton order

  bool reg(int l, int bx, int by) const {
    if (l >= m) return false;
    if (bx < 0 || bx >= nbx[l]) {
      if (!per_x) return false;
      bx = ((bx % nbx[l]) + nbx[l]) % nbx[l];
    }
    if (by < 0 || by >= nby[l]) {
      if (!per_y) return false;
      by = ((by % nby[l]) + nby[l]) % nby[l];
    }
    return region[l][(size_t)by * nbx[l] + bx] != 0;
  }
  bool wrapc(int l, int &x, int &y) const {
    if (x < 0 || x >= nx[l]) {
      if (!per_x) return false;
      x = ((x % nx[l]) + nx[l]) % nx[l];
    }
    if (y < 0 || y >= ny[l]) {
      if (!per_y) return false;
      y = ((y % ny[l]) + ny[l]) % ny[l];
    }
    return true;
  }
  bool cell_region(int l, int x, int y) const {
    if (!wrapc(l, x, y)) return false;
    return reg(l, x >> 4, y >> 4);
  }
  bool cell_hidden(int l, int x, int y) const {
    if (!wrapc(l, x, y)) return false;
    return l + 1 < m && reg(l, x >> 4, y >> 4) && reg(l + 1, (2 * x) >> 4, (2 * y) >> 4);
  }
  bool cell_own(int l, int x, int y) const {
    if (!wrapc(l, x, y)) return false;
    return reg(l, x >> 4, y >> 4) && !(l + 1 < m && reg(l + 1, (2 * x) >> 4, (2 * y) >> 4));
  }
  bool block_has_own(int l, int bx, int by) const {
    if (!reg(l, bx, by)) return false;
    if (l + 1 >= m) return true;
    for (int q = 0; q < 4; ++q)
      if (!reg(l + 1, 2 * bx + (q & 1), 2 * by + (q >> 1))) return true;
    return false;
  }
  bool block_has_hidden(int l, int bx, int by) const {
    if (!reg(l, bx, by) || l + 1 >= m) return false;
    for (int q = 0; q < 4; ++q)
      if (reg(l + 1, 2 * bx + (q & 1), 2 * by + (q >> 1))) return true;
    return false;
  }
};

sbt_status build_forest(const sbt_case_desc &d, Forest &F) {
  if (d.block_n != kB) return fail(SBT_ERR_ARG, "block_n must be 16");
  if (d.n_levels < 1 || d.n_levels > kMaxLevels) return fail(SBT_ERR_ARG, "n_levels must be 1..6");
  if (d.nx0 <= 0 || d.ny0 <= 0 || d.nx0 % kB || d.ny0 % kB)
    return fail(SBT_ERR_ARG, "nx0, ny0 must be positive multiples of 16");
  if (!(d.tau0 > 0.5)) return fail(SBT_ERR_ARG, "tau0 must exceed 1/2");
  if (!(d.rho0 > 0.0)) return fail(SBT_ERR_ARG, "rho0 must be positive");
  for (int e = 0; e < 4; ++e)
    if (d.bc[e] < 0 || d.bc[e] > SBT_BC_SYMMETRY) return fail(SBT_ERR_ARG, "bad edge kind");
  if ((d.bc[0] == SBT_BC_PERIODIC) != (d.bc[1] == SBT_BC_PERIODIC) ||
      (d.bc[2] == SBT_BC_PERIODIC) != (d.bc[3] == SBT_BC_PERIODIC))
    return fail(SBT_ERR_ARG, "periodic edges must come in W/E or S/N pairs");
  if (d.storage < SBT_F64 || d.storage > SBT_BF16S) return fail(SBT_ERR_ARG, "bad storage");
  if (d.cf_mode != SBT_CF_HOMOGENEOUS && d.cf_mode != SBT_CF_RESCALE) return fail(SBT_ERR_ARG, "bad cf_mode");
  if (d.collision != SBT_COLL_BGK && d.collision != SBT_COLL_MRT) return fail(SBT_ERR_ARG, "bad collision model");
  if (d.collision == SBT_COLL_MRT)
    for (int k = 0; k < 3; ++k)
      if (!(d.mrt_rates[k] > 0.0 && d.mrt_rates[k] < 2.0)) return fail(SBT_ERR_ARG, "MRT rates must lie in (0, 2)");
  if (d.max_markers < 0 || d.mdf_iters < 0) return fail(SBT_ERR_ARG, "negative marker count or N_F");
  if (d.max_markers > 0 && d.history_cap <= 0) return fail(SBT_ERR_ARG, "history_cap must be positive");
  if (d.max_markers > kMaxMarkers) return fail(SBT_ERR_ARG, "at most 1024 markers per body");
  if (d.n_refine < 0 || (d.n_refine > 0 && !d.refine)) return fail(SBT_ERR_ARG, "bad refine list");
  F.m = d.n_levels;
  F.per_x = d.bc[0] == SBT_BC_PERIODIC;
  F.per_y = d.bc[2] == SBT_BC_PERIODIC;
  F.region.assign(F.m, {});
  for (int l = 0; l < F.m; ++l) {
    F.nx[l] = d.nx0 << l;
    F.ny[l] = d.ny0 << l;
    F.nbx[l] = F.nx[l] / kB;
    F.nby[l] = F.ny[l] / kB;
    if ((size_t)F.nbx[l] * F.nby[l] > (size_t)1 << 28) return fail(SBT_ERR_ARG, "level too large");
    F.region[l].assign((size_t)F.nbx[l] * F.nby[l], l == 0 ? 1 : 0);
  }
  for (int r = 0; r < d.n_refine; ++r) {
    const sbt_box &b = d.refine[r];
    if (b.level < 1 || b.level >= F.m) return fail(SBT_ERR_TOPOLOGY, "refine box level out of range");
    int l = b.level;
    if (b.bx0 < 0 || b.by0 < 0 || b.bx1 > F.nbx[l] || b.by1 > F.nby[l] || b.bx0 >= b.bx1 || b.by0 >= b.by1)
      return fail(SBT_ERR_TOPOLOGY, "refine box outside its level");
    for (int by = b.by0; by < b.by1; ++by)
      for (int bx = b.bx0; bx < b.bx1; ++bx) F.region[l][(size_t)by * F.nbx[l] + bx] = 1;
  }
  // Nesting and 2:1 balance: every level-l block, widened by one cell of
  // level l-1 (its two halo layers), lies inside region_{l-1} and inside the
  // domain unless the axis is periodic.
  for (int l = 1; l < F.m; ++l) {
    bool any = false;
    for (int by = 0; by < F.nby[l]; ++by)
      for (int bx = 0; bx < F.nbx[l]; ++bx) {
        if (!F.region[l][(size_t)by * F.nbx[l] + bx]) continue;
        any = true;
        int cx0 = bx * 8 - 1, cx1 = bx * 8 + 8, cy0 = by * 8 - 1, cy1 = by * 8 + 8;
        for (int cy : {cy0, cy1})
          for (int cx : {cx0, cx1}) {
            int x = cx, y = cy;
            if (!F.wrapc(l - 1, x, y))
              return fail(SBT_ERR_TOPOLOGY, "refined level " + std::to_string(l) + " reaches a non-periodic edge");
            if (!F.reg(l - 1, x >> 4, y >> 4))
              return fail(SBT_ERR_TOPOLOGY, "level " + std::to_string(l) + " block not nested in level " +
                                                std::to_string(l - 1) + " with a one-cell margin");
          }
      }
    if (!any) return fail(SBT_ERR_TOPOLOGY, "level " + std::to_string(l) + " has no block");
  }
  // Blocks with owned cells, then halo blocks, Morton order per level.
  F.own.assign(F.m, {});
  F.ghost.assign(F.m, {});
  for (int l = 0; l < F.m; ++l) {
    std::vector<std::pair<uint32_t, int>> o, g;
    for (int by = 0; by < F.nby[l]; ++by)
      for (int bx = 0; bx < F.nbx[l]; ++bx) {
        int id = by * F.nbx[l] + bx;
        if (F.block_has_own(l, bx, by)) {
          o.push_back({morton(bx, by), id});
        } else if (l > 0 && !F.reg(l, bx, by)) {
          bool adj = false;
          for (int dy = -1; dy <= 1 && !adj; ++dy)
            for (int dx = -1; dx <= 1 && !adj; ++dx)
              if ((dx || dy) && F.block_has_own(l, bx + dx, by + dy)) adj = true;
          if (adj) g.push_back({morton(bx, by), id});
        }
      }
    std::sort(o.begin(), o.end());
    std::sort(g.begin(), g.end());
    for (auto &p : o) F.own[l].push_back(p.second);
    for (auto &p : g) F.ghost[l].push_back(p.second);
  }
  return SBT_OK;
}

// ---------------------------------------------------------------------------
// Device memory plan (bump allocator, 256-byte aligned).
// ---------------------------------------------------------------------------
struct Carver {
  char *base = nullptr;
  size_t off = 0;
  void *take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

struct CaseLevelRange {
  int v = -1;
  int own0 = 0, own1 = 0, ghost0 = 0, ghost1 = 0;
};

struct Pool {
  int n_own = 0, n_ghost = 0;
  std::vector<BlockMeta> meta;
  std::vector<uint16_t> codes;
  std::vector<int32_t> fast, slow, band;   // interior blocks, other owned blocks, halo-band cells
  std::vector<int32_t> solid;              // blocks with solid cells or links (generic kernel)
  std::vector<uint16_t> sbits;             // solid records [record][256]
  std::vector<double> sq;                  // [record][9][256]
  uint16_t *d_sbits = nullptr;
  double *d_sq = nullptr;
  int32_t *d_solid = nullptr;
  BlockMeta *d_meta = nullptr;
  uint16_t *d_codes = nullptr;
  int32_t *d_list = nullptr, *d_band = nullptr;   // d_list = fast blocks, then slow blocks
  void *lat[2] = {nullptr, nullptr};
  int cur = 0;
  int total() const { return n_own + n_ghost; }
};

struct CaseHost {
  sbt_case_desc d;
  std::vector<sbt_box> boxes;
  Forest F;
  int vshift = 0;
  std::vector<CaseLevelRange> lr;  // per true level
  CaseDev dev;                     // host copy (pointers already device)
  std::vector<int32_t> bmap;
  bool has_body = false;
  std::vector<std::vector<uint8_t>> smask;  // per level: dense solid mask (empty = none)
  std::vector<std::vector<double>> sq;      // per level: dense [cell][9] wall fractions
  int n_markers = 0;
  int win_cap = 0;
  size_t hist_cap = 0;
};

enum PhaseType { PH_LEVEL = 0, PH_MDF = 1 };
struct Phase {
  int type, v, p;
};

}  // namespace

// Polls of a persistent-step grid-barrier wait before it gives up (with a
// short sleep each, about a second).
constexpr uint32_t kBarrierSpins = 1u << 21;

struct sbt_ctx {
  int n_cases = 0, V = 1, storage = 0;
  int kvar = 0;  // level-launch variant: storage | (collision model << 2)
  std::vector<CaseHost> cs;
  std::vector<Pool> pools;         // one pool per virtual level: the blocks of every case
  CaseDev *d_cases = nullptr;
  CaseDev *d_bodies = nullptr;     // parameters of the cases with a body (one per forcing workgroup)
  int n_bodies = 0;
  int32_t *d_err = nullptr;
  double *d_stage = nullptr, *d_partial = nullptr, *d_diag = nullptr;
  size_t stage_blocks = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  bool post = false;               // false: lattices hold the initial pre-collision state
  int tile = 0, xcd = 1, use_graph = 1;
  int persistent = 0;              // one persistent launch per step instead of the launch chain
  PPhase *d_ptab = nullptr;        // [2 * plan_bufs][ptab_cap] phase tables of the persistent step
  int ptab_cap = 0;
  std::vector<char> ptab_ready;
  std::vector<int> ptab_n;
  uint32_t *d_bar = nullptr;       // grid-barrier state of the persistent step
  int p_groups = 0;                // its workgroups (0: not sized yet)
  uint32_t p_spins = kBarrierSpins;  // polls of a grid-barrier wait before it gives up
  size_t p_lds = 0;
  std::vector<int> kpw_level;   // interior blocks per workgroup per virtual level (0: automatic)
  int lds_window = 0;           // IBM window cells whose plan-builder counters fit in LDS
  int cell_cap = 0;             // stencil cells per IBM plan (fits the forcing kernel's LDS)
  int plan_bufs = 1;            // IBM plan buffers per body: the finest substeps of a step
  int max_body_markers = 0;     // largest body set so far (LDS table stride)
  int64_t k_host = 0;           // finest substeps issued (every body's forcing-loop counter)

  std::vector<Phase> step_phases;
  std::vector<hipGraphExec_t> graph;   // [level-0 parity + 2 * plan buffer + 2 * plan_bufs * size index]
  hipEvent_t step_event = nullptr;
  bool graph_dirty = true;
  size_t bytes_used = 0;
  int static_dev = -1;             // device whose static array holds the memory (sbt_create_static), or -1
  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_level, ev_fast, ev_mdf;
  double prof_bytes = 0.0, prof_updates = 0.0;
};

namespace {

void build_tables(sbt_ctx &X);
std::vector<Phase> step_phases(int V);
void advance_host(sbt_ctx &X, int steps);

// Copy and validate a case's solid regions (dense per level), applying the
// q = 1/2 rule where a short link has no fluid cell behind it.
sbt_status take_solids(CaseHost &C) {
  const Forest &F = C.F;
  C.smask.assign(F.m, {});
  C.sq.assign(F.m, {});
  if (C.d.n_solids < 0 || (C.d.n_solids > 0 && !C.d.solids)) return fail(SBT_ERR_ARG, "bad solid list");
  for (int k = 0; k < C.d.n_solids; ++k) {
    const sbt_solid &S = C.d.solids[k];
    if (S.level < 0 || S.level >= F.m || !S.mask) return fail(SBT_ERR_ARG, "bad solid level or mask");
    const int l = S.level, nx = F.nx[l], ny = F.ny[l];
    if (!C.smask[l].empty()) return fail(SBT_ERR_ARG, "one solid region per level");
    std::vector<uint8_t> &m = C.smask[l];
    m.assign((size_t)nx * ny, 0);
    bool any = false;
    for (size_t q = 0; q < m.size(); ++q) any |= (m[q] = S.mask[q] ? 1 : 0) != 0;
    if (!any) {
      m.clear();
      continue;
    }
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        if (!m[(size_t)y * nx + x]) continue;
        for (int dy = -2; dy <= 2; ++dy)
          for (int dx = -2; dx <= 2; ++dx)
            if (!F.cell_own(l, x + dx, y + dy))
              return fail(SBT_ERR_TOPOLOGY, "solid cells need two owned, uncovered cells of their level around them");
      }
    std::vector<double> &sq = C.sq[l];
    sq.assign((size_t)nx * ny * kQ, 0.5);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t c = (size_t)y * nx + x;
        if (m[c]) continue;
        for (int i = 1; i < kQ; ++i) {
          int ax = x + DCX[i], ay = y + DCY[i];
          if (!F.wrapc(l, ax, ay) || !m[(size_t)ay * nx + ax]) continue;
          double v = S.q ? S.q[c * kQ + i] : 0.5;
          if (!(v > 0.0 && v <= 1.0)) return fail(SBT_ERR_ARG, "wall fractions must lie in (0, 1]");
          int ux = x - DCX[i], uy = y - DCY[i];
          if (v < 0.5 && (!F.wrapc(l, ux, uy) || m[(size_t)uy * nx + ux])) v = 0.5;
          sq[c * kQ + i] = v;
        }
      }
  }
  return SBT_OK;
}

sbt_status plan_ctx(const sbt_case_desc *cases, int32_t n_cases, sbt_ctx &X, Carver &cv) {
  if (!cases || n_cases <= 0) return fail(SBT_ERR_ARG, "no cases");
  X.n_cases = n_cases;
  X.cs.resize(n_cases);
  X.V = 1;
  X.storage = cases[0].storage;
  X.kvar = X.storage | (cases[0].collision == SBT_COLL_MRT ? 4 : 0);
  for (int c = 0; c < n_cases; ++c) {
    CaseHost &C = X.cs[c];
    C.d = cases[c];
    if (C.d.storage != X.storage) return fail(SBT_ERR_ARG, "all cases of a context share one storage");
    if (C.d.collision != cases[0].collision) return fail(SBT_ERR_ARG, "all cases of a context share one collision model");
    C.boxes.assign(C.d.refine, C.d.refine + std::max(0, C.d.n_refine));
    C.d.refine = C.boxes.data();
    sbt_status st = build_forest(C.d, C.F);
    if (st) return fail(st, "case " + std::to_string(c) + ": " + g_err);
    st = take_solids(C);
    if (st) return fail(st, "case " + std::to_string(c) + ": " + g_err);
    if (C.d.cf_mode == SBT_CF_RESCALE)
      for (int l = 0; l + 1 < C.F.m; ++l) {
        double tau = 0.5 + (double)(1 << l) * (C.d.tau0 - 0.5);
        if (std::fabs(tau - 1.0) < 1e-6) return fail(SBT_ERR_ARG, "RESCALE needs tau != 1 on coarse levels");
      }
    X.V = std::max(X.V, C.F.m);
  }
  // one IBM plan buffer per finest substep of a step
  X.plan_bufs = 1 << (X.V - 1);
  const size_t s = storage_bytes(X.storage);
  // Pools: one per virtual level, the own blocks of every case, then their
  // halo blocks.  Each phase of a step is one launch over a pool.
  X.pools.assign((size_t)X.V, Pool());
  for (int c = 0; c < n_cases; ++c) {
    CaseHost &C = X.cs[c];
    C.vshift = X.V - C.F.m;
    C.lr.assign(C.F.m, CaseLevelRange());
    for (int l = 0; l < C.F.m; ++l) {
      int v = l + C.vshift;
      Pool &P = X.pools[v];
      C.lr[l].v = v;
      C.lr[l].own0 = P.n_own;
      P.n_own += (int)C.F.own[l].size();
      C.lr[l].own1 = P.n_own;
    }
  }
  for (int c = 0; c < n_cases; ++c) {
    CaseHost &C = X.cs[c];
    for (int l = 0; l < C.F.m; ++l) {
      Pool &P = X.pools[C.lr[l].v];
      C.lr[l].ghost0 = P.n_own + P.n_ghost;
      P.n_ghost += (int)C.F.ghost[l].size();
      C.lr[l].ghost1 = P.n_own + P.n_ghost;
    }
  }
  // Per-case IBM dimensions (host).
  for (int c = 0; c < n_cases; ++c) {
    CaseHost &C = X.cs[c];
    CaseDev &D = C.dev;
    std::memset(&D, 0, sizeof(D));
    D.body_kind = -1;
    C.has_body = C.d.max_markers > 0;
    if (!C.has_body) continue;
    const int lf = C.F.m - 1;
    // finest-level block map over the bounding box of region_{m-1}
    int x0 = C.F.nbx[lf], y0 = C.F.nby[lf], x1 = -1, y1 = -1;
    for (int id : C.F.own[lf]) {
      int bx = id % C.F.nbx[lf], by = id / C.F.nbx[lf];
      x0 = std::min(x0, bx); y0 = std::min(y0, by); x1 = std::max(x1, bx); y1 = std::max(y1, by);
    }
    D.bm_x0 = x0; D.bm_y0 = y0; D.bm_w = x1 - x0 + 1; D.bm_h = y1 - y0 + 1;
    size_t area = (size_t)D.bm_w * D.bm_h * kCells;
    size_t side = (size_t)C.d.max_markers + 8;
    C.win_cap = (int)std::min(area, side * side);
    C.hist_cap = (size_t)C.d.history_cap;
  }
  // Stencil cells per IBM plan: what the forcing kernel's LDS holds next to
  // the marker tables of the largest body (160 KB per workgroup on gfx950),
  // at most four per lane.
  {
    int nm = 0;
    for (auto &C : X.cs) nm = std::max(nm, C.has_body ? C.d.max_markers : 0);
    long cap = ((long)kLdsBytes - 2048 - (long)sbt_mdf_lds_bytes(nm, 0)) / (long)sbt_mdf_lds_bytes(0, 1);
    // a multiple of 4 keeps the forcing kernel's LDS list 16-byte aligned
    X.cell_cap = (int)std::max(0L, std::min(4096L, cap)) & ~3;
    if (nm > 0 && X.cell_cap < 64) return fail(SBT_ERR_ARG, "max_markers too large for one workgroup's LDS");
  }
  build_tables(X);
  // Device memory plan.
  size_t max_blocks = 1;
  for (auto &P : X.pools) {
    P.d_meta = (BlockMeta *)cv.take(sizeof(BlockMeta) * P.total());
    P.d_codes = (uint16_t *)cv.take(sizeof(uint16_t) * std::max<size_t>(1, P.codes.size()));
    P.d_list = (int32_t *)cv.take(sizeof(int32_t) * std::max<size_t>(1, P.fast.size() + P.slow.size()));
    P.d_band = (int32_t *)cv.take(sizeof(int32_t) * std::max<size_t>(1, P.band.size()));
    P.d_solid = (int32_t *)cv.take(sizeof(int32_t) * std::max<size_t>(1, P.solid.size()));
    P.d_sbits = (uint16_t *)cv.take(sizeof(uint16_t) * std::max<size_t>(1, P.sbits.size()));
    P.d_sq = (double *)cv.take(sizeof(double) * std::max<size_t>(1, P.sq.size()));
    P.lat[0] = cv.take(s * kQ * kCells * (size_t)P.total());
    P.lat[1] = cv.take(s * kQ * kCells * (size_t)P.total());
  }
  for (int c = 0; c < n_cases; ++c)
    for (int l = 0; l < X.cs[c].F.m; ++l)
      max_blocks = std::max(max_blocks, (size_t)(X.cs[c].lr[l].own1 - X.cs[c].lr[l].own0));
  X.stage_blocks = max_blocks;
  X.d_stage = (double *)cv.take(sizeof(double) * 3 * kCells * max_blocks);
  X.d_partial = (double *)cv.take(sizeof(double) * 3 * max_blocks);
  X.d_diag = (double *)cv.take(sizeof(double) * 16);  // diagnostics [0, 4), force stats [4, 12), E [12, 16)
  X.d_err = (int32_t *)cv.take(sizeof(int32_t) * 4);
  // persistent step: one phase table per (level-0 parity, first plan buffer)
  X.ptab_cap = 1 + (int)step_phases(X.V).size();
  X.d_ptab = (PPhase *)cv.take(sizeof(PPhase) * (size_t)X.ptab_cap * 2 * X.plan_bufs);
  X.ptab_ready.assign((size_t)2 * X.plan_bufs, 0);
  X.ptab_n.assign((size_t)2 * X.plan_bufs, 0);
  X.d_bar = (uint32_t *)cv.take(sizeof(uint32_t) * 4);
  X.d_cases = (CaseDev *)cv.take(sizeof(CaseDev) * n_cases);
  X.d_bodies = (CaseDev *)cv.take(sizeof(CaseDev) * n_cases);
  for (int c = 0; c < n_cases; ++c) {
    CaseHost &C = X.cs[c];
    CaseDev &D = C.dev;
    if (!C.has_body) continue;
    const size_t N = (size_t)C.d.max_markers;
    D.xb = (double *)cv.take(sizeof(double) * N);
    D.yb = (double *)cv.take(sizeof(double) * N);
    D.ds = (double *)cv.take(sizeof(double) * N);
    D.ftot = (double *)cv.take(sizeof(double) * 4 * N);
    D.hist = (double *)cv.take(sizeof(double) * 2 * C.hist_cap);
    D.kcount = (int64_t *)cv.take(sizeof(int64_t));
    D.hud = (double *)cv.take(sizeof(double) * 2 * (size_t)C.d.max_markers);
    const size_t nm = (size_t)C.d.max_markers, cc = (size_t)X.cell_cap;
    const size_t B = (size_t)X.plan_bufs;
    D.win = (IbmWindow *)cv.take(sizeof(IbmWindow) * B);
    D.phdr = (int32_t *)cv.take(sizeof(int32_t) * 4 * B);
    D.wF = (double *)cv.take(sizeof(double) * 2 * B * C.win_cap);
    D.wCnt = (int32_t *)cv.take(sizeof(int32_t) * B * C.win_cap);
    D.wIdx = (int32_t *)cv.take(sizeof(int32_t) * B * C.win_cap);
    D.p_ij = (int32_t *)cv.take(sizeof(int32_t) * 2 * B * nm);
    D.p_w = (double *)cv.take(sizeof(double) * 8 * B * nm);
    D.p_ud = (double *)cv.take(sizeof(double) * 2 * B * nm);
    D.p_tap = (uint16_t *)cv.take(sizeof(uint16_t) * 16 * B * nm);
    D.p_cell = (int32_t *)cv.take(sizeof(int32_t) * 8 * B * cc);
    D.p_list = (uint16_t *)cv.take(sizeof(uint16_t) * 16 * B * nm);
    D.bmap = (const int32_t *)cv.take(sizeof(int32_t) * (size_t)D.bm_w * D.bm_h);
  }
  return SBT_OK;
}

// Fill block metadata, cell codes and case parameters (host side).
void build_tables(sbt_ctx &X) {
  for (auto &P : X.pools) {
    P.meta.assign(P.total(), BlockMeta());
    P.codes.clear();
    P.sbits.clear();
    P.sq.clear();
  }
  for (int c = 0; c < X.n_cases; ++c) {
    CaseHost &C = X.cs[c];
    const Forest &F = C.F;
    // dense maps block id -> pool index, per level
    std::vector<std::vector<int32_t>> map(F.m);
    for (int l = 0; l < F.m; ++l) {
      map[l].assign((size_t)F.nbx[l] * F.nby[l], -1);
      for (size_t k = 0; k < F.own[l].size(); ++k) map[l][F.own[l][k]] = C.lr[l].own0 + (int)k;
      for (size_t k = 0; k < F.ghost[l].size(); ++k) map[l][F.ghost[l][k]] = C.lr[l].ghost0 + (int)k;
    }
    auto lookup = [&](int l, int bx, int by) -> int32_t {
      if (bx < 0 || bx >= F.nbx[l]) {
        if (!F.per_x) return -1;
        bx = ((bx % F.nbx[l]) + F.nbx[l]) % F.nbx[l];
      }
      if (by < 0 || by >= F.nby[l]) {
        if (!F.per_y) return -1;
        by = ((by % F.nby[l]) + F.nby[l]) % F.nby[l];
      }
      return map[l][(size_t)by * F.nbx[l] + bx];
    };
    for (int l = 0; l < F.m; ++l) {
      Pool &P = X.pools[C.lr[l].v];
      for (int pass = 0; pass < 2; ++pass) {
        const std::vector<int> &ids = pass == 0 ? F.own[l] : F.ghost[l];
        int base = pass == 0 ? C.lr[l].own0 : C.lr[l].ghost0;
        for (size_t k = 0; k < ids.size(); ++k) {
          int id = ids[k], bx = id % F.nbx[l], by = id / F.nbx[l];
          BlockMeta &M = P.meta[base + k];
          M.ox = bx * kB;
          M.oy = by * kB;
          for (int d = 1; d < 9; ++d) M.nbr[d - 1] = lookup(l, bx + DCX[d], by + DCY[d]);
          for (int q = 0; q < 4; ++q)
            M.child[q] = (pass == 0 && l + 1 < F.m) ? lookup(l + 1, 2 * bx + (q & 1), 2 * by + (q >> 1)) : -1;
          M.case_id = c;
          M.level = l;
          M.flags = pass == 1 ? BF_GHOST : 0;
          M.code = -1;
          M.solid = -1;
          if (pass == 0 && !C.smask[l].empty()) {  // solid cells and the links into them
            const std::vector<uint8_t> &sm = C.smask[l];
            std::vector<uint16_t> bits(kCells, 0);
            std::vector<double> qv((size_t)kQ * kCells, 0.5);
            bool any = false;
            for (int cell = 0; cell < kCells; ++cell) {
              const int gx = M.ox + (cell & 15), gy = M.oy + (cell >> 4);
              const size_t g = (size_t)gy * F.nx[l] + gx;
              if (sm[g]) {
                bits[cell] = SB_SOLID;
                any = true;
                continue;
              }
              for (int i = 1; i < kQ; ++i) {
                int sx = gx - DCX[i], sy = gy - DCY[i];
                if (!F.wrapc(l, sx, sy) || !sm[(size_t)sy * F.nx[l] + sx]) continue;
                const int o = OPP[i];  // the population sent toward the wall
                bits[cell] |= (uint16_t)(1u << i);
                qv[(size_t)i * kCells + cell] = C.sq[l][g * kQ + o];
                any = true;
              }
            }
            if (any) {
              M.flags |= BF_SOLID;
              M.solid = (int32_t)(P.sbits.size() / kCells);
              P.sbits.insert(P.sbits.end(), bits.begin(), bits.end());
              P.sq.insert(P.sq.end(), qv.begin(), qv.end());
            }
          }
          if (pass == 0 && l == 0) {
            if ((!F.per_x && (bx == 0 || bx == F.nbx[0] - 1)) || (!F.per_y && (by == 0 || by == F.nby[0] - 1)))
              M.flags |= BF_EDGE;
          }
          if (pass == 0 && l == F.m - 1 && C.has_body) M.flags |= BF_IBM;
          // per-cell codes where a hidden cell is within reach, and in halo blocks
          bool need = pass == 1;
          if (pass == 0 && l + 1 < F.m)
            for (int dy = -1; dy <= 1 && !need; ++dy)
              for (int dx = -1; dx <= 1 && !need; ++dx)
                if (F.block_has_hidden(l, bx + dx, by + dy)) need = true;
          if (!need) continue;
          std::vector<uint16_t> code(kCells, 0);
          bool any = false;
          for (int cell = 0; cell < kCells; ++cell) {
            int gx = M.ox + (cell & 15), gy = M.oy + (cell >> 4);
            uint16_t cc = 0;
            if (pass == 0) {
              if (F.cell_hidden(l, gx, gy)) cc |= CC_HIDDEN;
              for (int i = 1; i < 9; ++i)
                if (F.cell_hidden(l, gx - DCX[i], gy - DCY[i])) cc |= (uint16_t)(1u << i);
              if (!(cc & CC_HIDDEN) && (cc & CC_HSRC)) cc |= CC_IFACE;
            } else {
              for (int dy = -2; dy <= 2 && !(cc & CC_BAND); ++dy)
                for (int dx = -2; dx <= 2; ++dx)
                  if (F.cell_own(l, gx + dx, gy + dy)) {
                    cc |= CC_BAND;
                    break;
                  }
            }
            code[cell] = cc;
            any |= cc != 0;
          }
          if (!any && pass == 0) continue;
          M.flags |= BF_CODES;
          M.code = (int32_t)(P.codes.size() / kCells);
          P.codes.insert(P.codes.end(), code.begin(), code.end());
        }
      }
    }
    if (C.has_body) {
      const int lf = F.m - 1;
      C.bmap.assign((size_t)C.dev.bm_w * C.dev.bm_h, -1);
      for (size_t k = 0; k < F.own[lf].size(); ++k) {
        int id = F.own[lf][k], bx = id % F.nbx[lf] - C.dev.bm_x0, by = id / F.nbx[lf] - C.dev.bm_y0;
        C.bmap[(size_t)by * C.dev.bm_w + bx] = C.lr[lf].own0 + (int)k;
      }
    }
    // case parameters (the arithmetic below mirrors the relations stated in
    // the header: tau_l, body force per level, interface factors)
    CaseDev &D = C.dev;
    const sbt_case_desc &d = C.d;
    for (int l = 0; l < F.m; ++l) {
      double tau = 0.5 + (double)(1 << l) * (d.tau0 - 0.5);
      D.tau[l] = tau;
      D.pre[l] = 1.0 - 0.5 / tau;
      D.fx[l] = d.fext[0] / (double)(1 << l);
      D.fy[l] = d.fext[1] / (double)(1 << l);
      D.omega_f[l] = (float)(1.0 / tau);
      D.pre_f[l] = (float)D.pre[l];
      D.fx_f[l] = (float)D.fx[l];
      D.fy_f[l] = (float)D.fy[l];
      D.nx[l] = F.nx[l];
      D.ny[l] = F.ny[l];
    }
    for (int l = 0; l < F.m; ++l) {
      if (l > 0) D.s_cf[l] = (D.tau[l] - 1.0) / (2.0 * (D.tau[l - 1] - 1.0));
      if (l + 1 < F.m) D.s_fc[l] = 2.0 * D.tau[l] / D.tau[l + 1];
      D.s_cf_f[l] = (float)D.s_cf[l];
      D.s_fc_f[l] = (float)D.s_fc[l];
    }
    D.rho0 = d.rho0;
    for (int k = 0; k < 3; ++k) {
      D.mrt_s[k] = d.collision == SBT_COLL_MRT ? d.mrt_rates[k] : 0.0;
      D.mrt_s_f[k] = (float)D.mrt_s[k];
    }
    for (int e = 0; e < 4; ++e) {
      D.bc[e] = d.bc[e];
      D.bcu[e][0] = d.bc_u[e][0];
      D.bcu[e][1] = d.bc_u[e][1];
    }
    D.per_x = F.per_x;
    D.per_y = F.per_y;
    D.cf_mode = d.cf_mode;
    D.n_levels = F.m;
    D.mdf_iters = d.mdf_iters;
    D.hist_cap = (int32_t)C.hist_cap;
    D.win_cap = C.win_cap;
    D.nm_cap = C.d.max_markers;
    D.cell_cap = X.cell_cap;
    D.plan_mask = X.plan_bufs - 1;
  }
  // launch lists: interior blocks take the LDS-staged kernel
  for (auto &P : X.pools) {
    P.fast.clear();
    P.slow.clear();
    P.band.clear();
    P.solid.clear();
    for (int b = 0; b < P.n_own; ++b) {
      const BlockMeta &M = P.meta[b];
      if (M.flags & BF_SOLID) {
        P.solid.push_back(b);
        continue;
      }
      bool all_nbr = true;
      for (int d = 0; d < 8; ++d) all_nbr &= M.nbr[d] >= 0;
      if (!(M.flags & (BF_CODES | BF_EDGE)) && all_nbr) P.fast.push_back(b);
      else P.slow.push_back(b);
    }
    for (int b = P.n_own; b < P.total(); ++b) {
      const BlockMeta &M = P.meta[b];
      if (!(M.flags & BF_CODES)) continue;
      for (int cell = 0; cell < kCells; ++cell)
        if (P.codes[(size_t)M.code * kCells + cell] & CC_BAND) P.band.push_back(b * kCells + cell);
    }
  }
}

// ---------------------------------------------------------------------------
// Schedule: the recursion of Algorithm 1 unrolled over virtual levels.  With
// the pull scheme a level launch streams the previous collision's output and
// performs the next collision, so the launches follow the order in which the
// paper's StreamingStep calls occur: streams(v) = streams(v+1), S_v(first),
// streams(v+1), S_v(second); the finest level's launches are each preceded by
// the IBM (UpdateVelocity) launch.
// ---------------------------------------------------------------------------
void rec_phases(int v, int V, std::vector<Phase> &out) {
  if (v == V - 1) {
    for (int p = 1; p <= 2; ++p) {
      out.push_back({PH_MDF, v, p});
      out.push_back({PH_LEVEL, v, p});
    }
    return;
  }
  rec_phases(v + 1, V, out);
  out.push_back({PH_LEVEL, v, 1});
  rec_phases(v + 1, V, out);
  out.push_back({PH_LEVEL, v, 2});
}

std::vector<Phase> step_phases(int V) {
  std::vector<Phase> out;
  if (V == 1) {
    out.push_back({PH_MDF, 0, 1});
    out.push_back({PH_LEVEL, 0, 1});
    return out;
  }
  rec_phases(1, V, out);
  out.push_back({PH_LEVEL, 0, 1});
  return out;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
};

// Interior blocks per workgroup of a tile launch.  Automatic: for 2-byte
// storage as many as keep about four workgroups per resident slot (256 CUs
// x 8), up to 8, so small launches still fill the chip and large ones
// pipeline their loads; one otherwise.
int blocks_per_wg(const sbt_ctx &X, int v, int n_fast) {
  int k = v < (int)X.kpw_level.size() ? X.kpw_level[v] : 0;
  if (k > 0) return k;
  // 8- and 4-byte storage saturate HBM with one block per workgroup; the
  // 2-byte forms move too few bytes per block to hide latency without runs
  if (storage_bytes(X.storage) > 2) return 1;
  k = 1;
  while (k < 8 && (int64_t)n_fast >= (int64_t)k * 2 * 4 * 2048) k *= 2;
  return k;
}

// Arguments of a level launch of pool v in the current state.
LevelArgs level_args(const sbt_ctx &X, int v, int mode) {
  const Pool &P = X.pools[v];
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.meta = P.d_meta;
  a.codes = P.d_codes;
  a.sbits = P.d_sbits;
  a.sq = P.d_sq;
  a.src = P.lat[P.cur];
  a.dst = P.lat[1 - P.cur];
  if (v + 1 < X.V) {
    const Pool &Q = X.pools[v + 1];
    a.fmeta = Q.d_meta;
    a.fcodes = Q.d_codes;
    a.fprev = Q.lat[1 - Q.cur];
    a.fcur = Q.lat[Q.cur];
  }
  a.cases = X.d_cases;
  a.mode = mode;
  a.xcd_remap = X.xcd;
  // the finest level collides with the force of the forcing loop just run
  a.ibm_parity = (v == X.V - 1 && X.n_bodies > 0 && X.k_host > 0) ? (int)((X.k_host - 1) & (X.plan_bufs - 1)) : -1;
  a.err = X.d_err;
  return a;
}

sbt_status launch_level(sbt_ctx &X, int v, int p, int mode, hipStream_t s) {
  Pool &P = X.pools[v];
  LevelArgs a = level_args(X, v, mode);
  auto timed = [&](bool fast, auto &&launch) -> sbt_status {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (X.profiling) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s));
    }
    HIPCHK(launch());
    if (X.profiling) {
      HIPCHK(hipEventRecord(e1, s));
      (fast ? X.ev_fast : X.ev_level).push_back({e0, e1});
    }
    return SBT_OK;
  };
  sbt_status st = SBT_OK;
  if (mode == 0) {
    LevelArgs t = a;
    t.list = P.d_list;
    t.n_fast = (int)P.fast.size();
    t.n_blocks = (int)(P.fast.size() + P.slow.size());
    t.kpw = blocks_per_wg(X, v, t.n_fast);
    if (p == 1) {
      t.band = P.d_band;
      t.n_band = (int)P.band.size();
    }
    if (t.n_blocks + t.n_band > 0) st = timed(true, [&] { return sbt_launch_level_tile(X.kvar, &t, s); });
    if (!st && !P.solid.empty()) {  // blocks next to solid cells: generic kernel, same substep
      LevelArgs u = a;
      u.list = P.d_solid;
      u.n_blocks = (int)P.solid.size();
      st = timed(false, [&] { return sbt_launch_level(X.kvar, 0, &u, s); });
    }
  } else {
    a.list = nullptr;
    a.b0 = 0;
    a.n_blocks = P.n_own;
    st = timed(false, [&] { return sbt_launch_level(X.kvar, 0, &a, s); });
  }
  if (st) return st;
  P.cur = 1 - P.cur;
  return SBT_OK;
}

// Arguments of the forcing loop of the next finest substep.
MdfArgs mdf_args(const sbt_ctx &X, bool first) {
  const Pool &P = X.pools[X.V - 1];
  MdfArgs a;
  a.meta = P.d_meta;
  a.src = P.lat[P.cur];
  a.cases = X.d_cases;
  a.bodies = X.d_bodies;
  a.first = first ? 1 : 0;
  a.err = X.d_err;
  a.max_markers = X.max_body_markers;
  a.cell_cap = X.cell_cap;
  a.parity = (int)(X.k_host & (X.plan_bufs - 1));
  return a;
}

sbt_status launch_mdf(sbt_ctx &X, bool first, hipStream_t s) {
  if (X.n_bodies == 0) return SBT_OK;
  MdfArgs a = mdf_args(X, first);
  ++X.k_host;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (X.profiling) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
  }
  HIPCHK(sbt_launch_mdf(X.storage, &a, X.n_bodies, s));
  if (X.profiling) {
    HIPCHK(hipEventRecord(e1, s));
    X.ev_mdf.push_back({e0, e1});
  }
  return SBT_OK;
}

int forcing_phases(const sbt_ctx &X) {
  int n = 0;
  for (const Phase &ph : X.step_phases) n += ph.type == PH_MDF;
  return n;
}

// Build the IBM plans of every body for the next n_plans finest
// substeps (those of kcount .. kcount + n_plans - 1), one workgroup per body
// and substep.  The plan of substep k goes to buffer k & (plan_bufs - 1);
// every earlier reader of those buffers precedes this launch in stream order.
IbmArgs prep_args(const sbt_ctx &X, int n_plans) {
  IbmArgs a;
  a.cases = X.d_cases;
  a.bodies = X.d_bodies;
  a.max_markers = X.max_body_markers;
  a.cell_cap = X.cell_cap;
  a.lds_window = X.lds_window;
  a.n_bodies = X.n_bodies;
  a.n_plans = n_plans;
  return a;
}

sbt_status launch_prep(sbt_ctx &X, int n_plans, hipStream_t s) {
  if (X.n_bodies == 0) return SBT_OK;
  if (n_plans > X.plan_bufs) return fail(SBT_ERR_STATE, "more IBM plans than plan buffers");
  IbmArgs a = prep_args(X, n_plans);
  HIPCHK(sbt_launch_ibm_prep(&a, s));
  return SBT_OK;
}

// Collide once on every level from the initial pre-collision state (the
// first CollisionStep of every level), finest first so that each coarse
// level explodes into its finer level's current lattice.
sbt_status run_prologue(sbt_ctx &X, hipStream_t s) {
  sbt_status st = SBT_OK;
  for (int v = X.V - 1; v >= 0; --v) {
    if (v == X.V - 1) {
      st = launch_prep(X, 1, s);
      if (!st) st = launch_mdf(X, true, s);
      if (st) return st;
    }
    st = launch_level(X, v, 1, MODE_LOCAL, s);
    if (st) return st;
  }
  X.post = true;
  return SBT_OK;
}

// One step: the IBM plans of all its finest substeps (they depend on the
// marker positions only), then the phases in order.
sbt_status run_step_eager(sbt_ctx &X, hipStream_t s) {
  sbt_status st = launch_prep(X, forcing_phases(X), s);
  if (st) return st;
  for (const Phase &ph : X.step_phases) {
    st = ph.type == PH_MDF ? launch_mdf(X, false, s) : launch_level(X, ph.v, ph.p, 0, s);
    if (st) return st;
  }
  return SBT_OK;
}

void destroy_graphs(sbt_ctx &X) {
  for (auto &g : X.graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  X.graph_dirty = true;
  X.ptab_ready.assign(X.ptab_ready.size(), 0);
}

// ---- the persistent step ------------------------------------------------------
// The phase table of one step from the current state: the same plan
// builder, forcing loops and level substeps, with the same arguments, as the
// launch chain (run_step_eager), in the same order.
void build_phase_table(sbt_ctx &X, std::vector<PPhase> &out) {
  out.clear();
  std::vector<int> saved(X.pools.size());
  for (size_t i = 0; i < X.pools.size(); ++i) saved[i] = X.pools[i].cur;
  const int64_t saved_k = X.k_host;
  auto blank = [] {
    PPhase q;
    std::memset(&q, 0, sizeof(q));
    return q;
  };
  if (X.n_bodies > 0) {
    PPhase q = blank();
    q.type = PP_PREP;
    q.ibm = prep_args(X, forcing_phases(X));
    q.n_items = X.n_bodies * q.ibm.n_plans;
    out.push_back(q);
  }
  for (const Phase &ph : X.step_phases) {
    PPhase q = blank();
    if (ph.type == PH_MDF) {
      if (X.n_bodies == 0) continue;
      q.type = PP_MDF;
      q.mdf = mdf_args(X, false);
      q.n_items = X.n_bodies;
      ++X.k_host;
    } else {
      Pool &P = X.pools[ph.v];
      q.type = PP_LEVEL;
      q.lv = level_args(X, ph.v, 0);
      q.lv.list = P.d_list;
      q.n_list = (int)(P.fast.size() + P.slow.size());
      q.solid = P.d_solid;
      q.n_solid = (int)P.solid.size();
      if (ph.p == 1) {
        q.lv.band = P.d_band;
        q.lv.n_band = (int)P.band.size();
      }
      q.n_items = q.n_list + q.n_solid;
      P.cur = 1 - P.cur;
    }
    out.push_back(q);
  }
  for (size_t i = 0; i < X.pools.size(); ++i) X.pools[i].cur = saved[i];
  X.k_host = saved_k;
}

// One step as one persistent launch.  The table depends on the state only
// through level 0's lattice parity and the plan buffer of the step's first
// substep (as the captured graphs do); each of those tables is uploaded once.
sbt_status run_step_persistent(sbt_ctx &X, hipStream_t s) {
  if (X.p_groups == 0) {
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    X.p_lds = 0;
    if (X.n_bodies > 0)
      X.p_lds = std::max(sbt_mdf_lds_bytes(X.max_body_markers, X.cell_cap),
                         sbt_prep_lds_bytes(X.max_body_markers, X.cell_cap, X.lds_window));
    const int per_cu = sbt_step_persistent_occupancy(X.kvar, X.p_lds);
    if (per_cu <= 0) return fail(SBT_ERR_DEVICE, "the persistent step kernel cannot launch");
    X.p_groups = per_cu * cus;
  }
  const int slot = X.pools[0].cur + 2 * (int)(X.k_host & (X.plan_bufs - 1));
  PPhase *tab = X.d_ptab + (size_t)slot * X.ptab_cap;
  if (!X.ptab_ready[slot]) {
    std::vector<PPhase> t;
    build_phase_table(X, t);
    if ((int)t.size() > X.ptab_cap) return fail(SBT_ERR_STATE, "phase table larger than planned");
    HIPCHK(hipMemcpyAsync(tab, t.data(), sizeof(PPhase) * t.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // t is released on return
    X.ptab_n[slot] = (int)t.size();
    X.ptab_ready[slot] = 1;
  }
  HIPCHK(sbt_launch_step_persistent(X.kvar, tab, X.ptab_n[slot], X.d_bar, X.d_err, X.p_spins, X.p_groups, X.p_lds, s));
  advance_host(X, 1);
  return SBT_OK;
}

// Steps per graph launch: a call of n steps replays graphs of 4, 2 and 1
// steps, so the launch gap between graphs is paid once per 4 steps.
constexpr int kGraphSteps[3] = {1, 2, 4};

sbt_status ensure_capture_stream(sbt_ctx &X) {
  if (!X.cap_stream) HIPCHK(hipStreamCreateWithFlags(&X.cap_stream, hipStreamNonBlocking));
  if ((int)X.graph.size() != 3 * 2 * X.plan_bufs) X.graph.assign(3 * 2 * X.plan_bufs, nullptr);
  return SBT_OK;
}

// A graph bakes in the lattice parities and the IBM plan buffers of its
// substeps.  Over a step only level 0's parity flips (every finer level
// runs an even number of substeps) and the forcing-loop counter advances by
// the number of plan buffers, so the key is level 0's parity and the plan
// buffer of the step's first substep.
int graph_slot(const sbt_ctx &X, int si) {
  return X.pools[0].cur + 2 * (int)(X.k_host & (X.plan_bufs - 1)) + 2 * X.plan_bufs * si;
}

// The host-side state changes of `steps` graph-replayed steps.
void advance_host(sbt_ctx &X, int steps) {
  for (int t = 0; t < steps; ++t) {
    for (const Phase &ph : X.step_phases)
      if (ph.type == PH_LEVEL) X.pools[ph.v].cur ^= 1;
    if (X.n_bodies > 0) X.k_host += forcing_phases(X);
  }
}

// `steps` steps as one graph: the eager launch list captured on one stream
// (the launches depend on each other in order, so the graph is a chain).
sbt_status capture_graph(sbt_ctx &X, int slot, int steps) {
  sbt_status st = ensure_capture_stream(X);
  if (st) return st;
  std::vector<int> saved(X.pools.size());
  for (size_t i = 0; i < X.pools.size(); ++i) saved[i] = X.pools[i].cur;
  const int64_t saved_k = X.k_host;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(X.cap_stream, hipStreamCaptureModeThreadLocal));
  for (int t = 0; t < steps && !st; ++t)
    st = run_step_eager(X, X.cap_stream);
  hipError_t e = hipStreamEndCapture(X.cap_stream, &g);
  for (size_t i = 0; i < X.pools.size(); ++i) X.pools[i].cur = saved[i];
  X.k_host = saved_k;
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(SBT_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&X.graph[slot], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(SBT_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return SBT_OK;
}

// Every graph size for both parities of level 0 at the current plan buffer,
// so a long call never captures inside its run.
sbt_status capture_all(sbt_ctx &X) {
  for (int flip = 0; flip < 2; ++flip) {
    if (flip)
      X.pools[0].cur ^= 1;
    sbt_status st = SBT_OK;
    for (int si = 0; si < 3 && !st; ++si) {
      const int slot = graph_slot(X, si);
      if (!X.graph[slot]) st = capture_graph(X, slot, kGraphSteps[si]);
    }
    if (flip)
      X.pools[0].cur ^= 1;
    if (st) return st;
  }
  return SBT_OK;
}

sbt_status check_case(sbt_ctx *ctx, int32_t c) {
  if (!ctx) return fail(SBT_ERR_ARG, "null context");
  if (c < 0 || c >= ctx->n_cases) return fail(SBT_ERR_ARG, "case index out of range");
  return SBT_OK;
}

sbt_status check_level(sbt_ctx *ctx, int32_t c, int32_t l) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  if (l < 0 || l >= ctx->cs[c].F.m) return fail(SBT_ERR_ARG, "level out of range");
  return SBT_OK;
}

// Gather a dense level field into per-block order [n][3][256] (host).
void dense_to_blocks(const Forest &F, int l, const double *r, const double *u, const double *v,
                     std::vector<double> &out) {
  const auto &ids = F.own[l];
  out.assign(ids.size() * 3 * kCells, 0.0);
  for (size_t k = 0; k < ids.size(); ++k) {
    int bx = ids[k] % F.nbx[l], by = ids[k] / F.nbx[l];
    for (int cell = 0; cell < kCells; ++cell) {
      size_t g = (size_t)(by * kB + (cell >> 4)) * F.nx[l] + bx * kB + (cell & 15);
      out[(k * 3 + 0) * kCells + cell] = r[g];
      out[(k * 3 + 1) * kCells + cell] = u[g];
      out[(k * 3 + 2) * kCells + cell] = v[g];
    }
  }
}

sbt_status readout_level(sbt_ctx &X, int c, int l, hipStream_t s) {
  CaseHost &C = X.cs[c];
  int v = C.lr[l].v;
  Pool &P = X.pools[v];
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ibm_parity = -1;
  a.kpw = 1;
  a.meta = P.d_meta;
  a.codes = P.d_codes;
  a.sbits = P.d_sbits;
  a.sq = P.d_sq;
  // after a step the state to read is the one the last launch streamed from
  a.src = X.post ? P.lat[1 - P.cur] : P.lat[P.cur];
  if (v + 1 < X.V) {
    Pool &Q = X.pools[v + 1];
    a.fmeta = Q.d_meta;
    a.fcodes = Q.d_codes;
    a.fprev = Q.lat[1 - Q.cur];
    a.fcur = Q.lat[Q.cur];
  }
  a.cases = X.d_cases;
  a.list = nullptr;
  a.b0 = C.lr[l].own0;
  a.n_blocks = C.lr[l].own1 - C.lr[l].own0;
  a.mode = MODE_READOUT | (X.post ? 0 : MODE_LOCAL);
  a.xcd_remap = 0;
  a.out = X.d_stage;
  a.partial = X.d_partial;
  a.err = X.d_err;
  HIPCHK(sbt_launch_level(X.kvar, 0, &a, s));
  return SBT_OK;
}

sbt_status upload_case(sbt_ctx &X, int c) {
  HIPCHK(hipMemcpyAsync(X.d_cases + c, &X.cs[c].dev, sizeof(CaseDev), hipMemcpyHostToDevice, X.stream));
  return SBT_OK;
}

// Reset counters and device IBM state; lattices keep their contents.
sbt_status reset_counters(sbt_ctx &X) {
  for (auto &C : X.cs) {
    if (!C.has_body) continue;
    HIPCHK(hipMemsetAsync(C.dev.kcount, 0, sizeof(int64_t), X.stream));
    HIPCHK(hipMemsetAsync(C.dev.win, 0, X.plan_bufs * sizeof(IbmWindow), X.stream));
  }
  X.post = false;
  X.k_host = 0;
  for (auto &P : X.pools) P.cur = 0;
  destroy_graphs(X);
  return SBT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *sbt_last_error(void) { return g_err.c_str(); }

sbt_status sbt_set_error(sbt_status code, const char *msg) { return fail(code, msg); }

sbt_status sbt_plan(const sbt_case_desc *cases, int32_t n_cases, size_t *device_bytes) {
  if (!device_bytes) return fail(SBT_ERR_ARG, "null output");
  sbt_ctx X;
  Carver cv;
  sbt_status st = plan_ctx(cases, n_cases, X, cv);
  if (st) return st;
  *device_bytes = cv.off + 256;
  return SBT_OK;
}

sbt_status sbt_create(const sbt_case_desc *cases, int32_t n_cases, void *device_buf, size_t bytes,
                      void *hip_stream, sbt_ctx **out) {
  return sbt_create_in(cases, n_cases, device_buf, bytes, hip_stream, -1, out);
}

sbt_status sbt_create_in(const sbt_case_desc *cases, int32_t n_cases, void *device_buf, size_t bytes,
                         void *hip_stream, int32_t static_dev, sbt_ctx **out) {
  if (!out) return fail(SBT_ERR_ARG, "null output");
  *out = nullptr;
  if (!device_buf) return fail(SBT_ERR_ARG, "null device buffer");
  if (((uintptr_t)device_buf) & 255) return fail(SBT_ERR_ARG, "device buffer must be 256-byte aligned");
  sbt_ctx *X = new sbt_ctx();
  Carver cv;
  cv.base = (char *)device_buf;
  sbt_status st = plan_ctx(cases, n_cases, *X, cv);
  if (st) {
    delete X;
    return st;
  }
  if (cv.off > bytes) {
    delete X;
    return fail(SBT_ERR_NOMEM, "device buffer smaller than sbt_plan reported");
  }
  X->bytes_used = cv.off;
  X->stream = (hipStream_t)hip_stream;
  X->static_dev = static_dev;
  auto cleanup_fail = [&](sbt_status s) {
    delete X;
    return s;
  };
  std::vector<int32_t> bodies;
  for (int c = 0; c < X->n_cases; ++c)
    if (X->cs[c].has_body) bodies.push_back(c);
  X->n_bodies = 0;  // bodies become active with sbt_set_body
  hipStream_t s = X->stream;
  for (auto &P : X->pools) {
    if (hipMemcpyAsync(P.d_meta, P.meta.data(), sizeof(BlockMeta) * P.meta.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return cleanup_fail(fail(SBT_ERR_DEVICE, "meta upload"));
    if (!P.codes.empty() &&
        hipMemcpyAsync(P.d_codes, P.codes.data(), sizeof(uint16_t) * P.codes.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess)
      return cleanup_fail(fail(SBT_ERR_DEVICE, "code upload"));
    bool ok = true;
    if (!P.fast.empty())
      ok &= hipMemcpyAsync(P.d_list, P.fast.data(), sizeof(int32_t) * P.fast.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    if (!P.slow.empty())
      ok &= hipMemcpyAsync(P.d_list + P.fast.size(), P.slow.data(), sizeof(int32_t) * P.slow.size(),
                           hipMemcpyHostToDevice, s) == hipSuccess;
    if (!P.band.empty())
      ok &= hipMemcpyAsync(P.d_band, P.band.data(), sizeof(int32_t) * P.band.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    if (!P.solid.empty()) {
      ok &= hipMemcpyAsync(P.d_solid, P.solid.data(), sizeof(int32_t) * P.solid.size(), hipMemcpyHostToDevice, s) ==
            hipSuccess;
      ok &= hipMemcpyAsync(P.d_sbits, P.sbits.data(), sizeof(uint16_t) * P.sbits.size(), hipMemcpyHostToDevice, s) ==
            hipSuccess;
      ok &= hipMemcpyAsync(P.d_sq, P.sq.data(), sizeof(double) * P.sq.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    }
    if (!ok) return cleanup_fail(fail(SBT_ERR_DEVICE, "list upload"));
    size_t n = (size_t)P.total() * kQ * kCells;
    if (sbt_launch_fill_nan(P.lat[0], n, X->storage, s) != hipSuccess ||
        sbt_launch_fill_nan(P.lat[1], n, X->storage, s) != hipSuccess)
      return cleanup_fail(fail(SBT_ERR_DEVICE, "lattice fill"));
  }
  for (int c = 0; c < X->n_cases; ++c) {
    CaseHost &C = X->cs[c];
    if (C.has_body) {
      if (hipMemcpyAsync((void *)C.dev.bmap, C.bmap.data(), sizeof(int32_t) * C.bmap.size(), hipMemcpyHostToDevice,
                         s) != hipSuccess)
        return cleanup_fail(fail(SBT_ERR_DEVICE, "block map upload"));
    }
    if (upload_case(*X, c)) return cleanup_fail(SBT_ERR_DEVICE);
  }
  if (hipMemsetAsync(X->d_err, 0, sizeof(int32_t) * 4, s) != hipSuccess ||
      hipMemsetAsync(X->d_bar, 0, sizeof(uint32_t) * 4, s) != hipSuccess)
    return cleanup_fail(fail(SBT_ERR_DEVICE, "memset"));
  if (reset_counters(*X)) return cleanup_fail(SBT_ERR_DEVICE);
  for (auto &P : X->pools) {
    if (sbt_launch_init(X->storage, P.d_meta, P.d_codes, X->d_cases, P.lat[0], 0, P.n_own, nullptr, nullptr, s) !=
        hipSuccess)
      return cleanup_fail(fail(SBT_ERR_DEVICE, "init"));
  }
  X->step_phases = step_phases(X->V);
  if (hipStreamSynchronize(s) != hipSuccess) return cleanup_fail(fail(SBT_ERR_DEVICE, "create sync"));
  *out = X;
  return SBT_OK;
}

sbt_status sbt_destroy(sbt_ctx *ctx) {
  if (!ctx) return SBT_OK;
  (void)hipStreamSynchronize(ctx->stream);
  destroy_graphs(*ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->step_event) (void)hipEventDestroy(ctx->step_event);
  const int dev = ctx->static_dev;
  delete ctx;
  if (dev >= 0) sbt_static_release(dev);
  return SBT_OK;
}

sbt_status sbt_level_blocks(sbt_ctx *ctx, int32_t c, int32_t level, int32_t *n_blocks, int32_t *ox,
                            int32_t *oy) {
  sbt_status st = check_level(ctx, c, level);
  if (st) return st;
  const Forest &F = ctx->cs[c].F;
  const auto &ids = F.own[level];
  if (n_blocks) *n_blocks = (int32_t)ids.size();
  for (size_t k = 0; k < ids.size(); ++k) {
    if (ox) ox[k] = (ids[k] % F.nbx[level]) * kB;
    if (oy) oy[k] = (ids[k] / F.nbx[level]) * kB;
  }
  return SBT_OK;
}

sbt_status sbt_level_info(sbt_ctx *ctx, int32_t c, int32_t level, int64_t out[4]) {
  sbt_status st = check_level(ctx, c, level);
  if (st) return st;
  const Forest &F = ctx->cs[c].F;
  int64_t owned = 0;
  for (int id : F.own[level]) {
    int bx = id % F.nbx[level], by = id / F.nbx[level];
    owned += kCells;
    if (level + 1 < F.m)
      for (int q = 0; q < 4; ++q)
        if (F.reg(level + 1, 2 * bx + (q & 1), 2 * by + (q >> 1))) owned -= kCells / 4;
  }
  out[0] = owned;
  out[1] = (int64_t)F.own[level].size();
  out[2] = (int64_t)F.ghost[level].size();
  out[3] = (int64_t)1 << (level + ctx->cs[c].vshift);
  return SBT_OK;
}

sbt_status sbt_updates_per_step(sbt_ctx *ctx, int64_t *updates) {
  if (!ctx || !updates) return fail(SBT_ERR_ARG, "null argument");
  int64_t u = 0;
  for (int c = 0; c < ctx->n_cases; ++c)
    for (int l = 0; l < ctx->cs[c].F.m; ++l) {
      int64_t info[4];
      sbt_level_info(ctx, c, l, info);
      u += info[0] * info[3];
    }
  *updates = u;
  return SBT_OK;
}

sbt_status sbt_init_fields(sbt_ctx *ctx, int32_t c, int32_t level, const double *rho, const double *ux,
                           const double *uy) {
  sbt_status st = check_level(ctx, c, level);
  if (st) return st;
  if (!rho || !ux || !uy) return fail(SBT_ERR_ARG, "null field");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  HIPCHK(hipStreamSynchronize(X.stream));
  // Going back to the initial state: the pre-collision populations live in
  // lattice 0 of every pool.  Other levels keep their initial values only if
  // the context has not stepped; after stepping, re-initialise them too.
  if (X.post) {  // back to the initial state: every level at rest, counters cleared
    for (auto &P : X.pools) {
      size_t n = (size_t)P.total() * kQ * kCells;
      HIPCHK(sbt_launch_fill_nan(P.lat[0], n, X.storage, X.stream));
      HIPCHK(sbt_launch_fill_nan(P.lat[1], n, X.storage, X.stream));
      HIPCHK(sbt_launch_init(X.storage, P.d_meta, P.d_codes, X.d_cases, P.lat[0], 0, P.n_own, nullptr, nullptr, X.stream));
    }
    if (reset_counters(X)) return SBT_ERR_DEVICE;
  }
  std::vector<double> host;
  dense_to_blocks(C.F, level, rho, ux, uy, host);
  size_t n = C.F.own[level].size();
  for (size_t k0 = 0; k0 < n; k0 += X.stage_blocks) {
    size_t k1 = std::min(n, k0 + X.stage_blocks);
    HIPCHK(hipMemcpyAsync(X.d_stage, host.data() + k0 * 3 * kCells, sizeof(double) * 3 * kCells * (k1 - k0),
                          hipMemcpyHostToDevice, X.stream));
    Pool &P = X.pools[C.lr[level].v];
    HIPCHK(sbt_launch_init(X.storage, P.d_meta, P.d_codes, X.d_cases, P.lat[0], C.lr[level].own0 + (int)k0,
                           (int)(k1 - k0), X.d_stage, nullptr, X.stream));
    HIPCHK(hipStreamSynchronize(X.stream));
  }
  return SBT_OK;
}

sbt_status sbt_init_uniform(sbt_ctx *ctx, int32_t c, double rho, double ux, double uy) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  if (!(rho > 0.0)) return fail(SBT_ERR_ARG, "rho must be positive");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  HIPCHK(hipStreamSynchronize(X.stream));
  if (X.post) {
    for (auto &P : X.pools) {
      size_t n = (size_t)P.total() * kQ * kCells;
      HIPCHK(sbt_launch_fill_nan(P.lat[0], n, X.storage, X.stream));
      HIPCHK(sbt_launch_fill_nan(P.lat[1], n, X.storage, X.stream));
      HIPCHK(sbt_launch_init(X.storage, P.d_meta, P.d_codes, X.d_cases, P.lat[0], 0, P.n_own, nullptr, nullptr,
                             X.stream));
    }
    if (reset_counters(X)) return SBT_ERR_DEVICE;
  }
  double u0[3] = {rho, ux, uy};
  for (int l = 0; l < C.F.m; ++l) {
    Pool &P = X.pools[C.lr[l].v];
    HIPCHK(sbt_launch_init(X.storage, P.d_meta, P.d_codes, X.d_cases, P.lat[0], C.lr[l].own0,
                           C.lr[l].own1 - C.lr[l].own0, nullptr, u0, X.stream));
  }
  HIPCHK(hipStreamSynchronize(X.stream));
  return SBT_OK;
}

sbt_status sbt_set_body(sbt_ctx *ctx, int32_t c, const sbt_body *body) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  if (X.post) return fail(SBT_ERR_STATE, "bodies can only be set before the first step");
  if (!C.has_body) return fail(SBT_ERR_ARG, "case was created with max_markers = 0");
  if (!body || body->n <= 0 || body->n > C.d.max_markers) return fail(SBT_ERR_ARG, "marker count out of range");
  if (!body->xb || !body->yb || !body->ds) return fail(SBT_ERR_ARG, "null marker arrays");
  if (body->kind < SBT_BODY_FIXED || body->kind > SBT_BODY_TRI) return fail(SBT_ERR_ARG, "bad body kind");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(body->p[i])) return fail(SBT_ERR_ARG, "kinematic parameters must be finite");
  {
    const double *p = body->p;
    const bool moving = body->kind == SBT_BODY_FLAP || body->kind == SBT_BODY_RAMP || body->kind == SBT_BODY_TRI;
    if (moving && (p[8] == 0.0 || p[9] == 0.0)) return fail(SBT_ERR_ARG, "U_ref and chord must be nonzero");
    if (body->kind == SBT_BODY_FLAP && p[6] == 0.0) return fail(SBT_ERR_ARG, "flap period must be nonzero");
    if (body->kind == SBT_BODY_RAMP && !(p[3] > 0.0 && p[4] > 0.0 && p[2] != 0.0))
      return fail(SBT_ERR_ARG, "ramp needs A != 0, a_s > 0 and K > 0");
    if (body->kind == SBT_BODY_TRI &&
        !(p[3] > 0.0 && p[3] < 1.0 && p[4] > 0.0 && p[5] > 0.0 && 2.0 * p[5] <= std::min(p[3], 1.0 - p[3])))
      return fail(SBT_ERR_ARG, "triangular law needs 0 < xi < 1, T > 0 and 0 < ta/T <= min(xi, 1 - xi)/2");
  }
  {
    int dev = 0, lds_max = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int nmax = body->n;
    for (auto &K : X.cs) nmax = std::max(nmax, K.n_markers);
    const size_t mdf = sbt_mdf_lds_bytes(nmax, X.cell_cap), prep = sbt_prep_lds_bytes(nmax, X.cell_cap, 0);
    if (mdf + 1024 > (size_t)lds_max || prep + 1024 > (size_t)lds_max)
      return fail(SBT_ERR_ARG, "too many markers for one workgroup's LDS (" + std::to_string(lds_max) + " bytes)");
    // the plan builder keeps window counters in LDS with what is left
    // (global memory beyond that), within half the CU's LDS when its tables
    // leave room, so that two plan builders share a CU
    const size_t half = (size_t)lds_max / 2 - 1024;
    const size_t budget = prep + 4096 * 4 <= half ? half : (size_t)lds_max - 1024;
    X.lds_window = (int)std::min<size_t>(32768, (budget - prep) / 4 - 1);
    X.max_body_markers = nmax;
  }
  HIPCHK(hipStreamSynchronize(X.stream));
  const size_t N = (size_t)body->n;
  HIPCHK(hipMemcpy((void *)C.dev.xb, body->xb, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)C.dev.yb, body->yb, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)C.dev.ds, body->ds, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(C.dev.hud, 0, sizeof(double) * 2 * (size_t)C.d.max_markers));
  C.dev.body_kind = body->kind;
  C.dev.n_markers = body->n;
  std::memcpy(C.dev.bp, body->p, sizeof(body->p));
  C.n_markers = body->n;
  HIPCHK(hipMemcpy(X.d_cases + c, &C.dev, sizeof(CaseDev), hipMemcpyHostToDevice));
  // the bodies in case order, one forcing workgroup each
  std::vector<CaseDev> bd;
  for (const CaseHost &K : X.cs)
    if (K.has_body && K.n_markers > 0) bd.push_back(K.dev);
  X.n_bodies = (int)bd.size();
  if (!bd.empty()) HIPCHK(hipMemcpy(X.d_bodies, bd.data(), sizeof(CaseDev) * bd.size(), hipMemcpyHostToDevice));
  destroy_graphs(X);
  return SBT_OK;
}

sbt_status sbt_set_markers(sbt_ctx *ctx, int32_t c, int32_t n, const double *x, const double *y,
                           const double *udx, const double *udy, const double *ds) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  if (!C.has_body || C.dev.body_kind != SBT_BODY_HOST) return fail(SBT_ERR_ARG, "case has no caller-placed body");
  if (n != C.n_markers) return fail(SBT_ERR_ARG, "marker count differs from the body's");
  if (!x || !y || !udx || !udy) return fail(SBT_ERR_ARG, "null marker arrays");
  if (ds)
    for (int j = 0; j < n; ++j)
      if (!(ds[j] > 0.0 && std::isfinite(ds[j]))) return fail(SBT_ERR_ARG, "ds must be positive and finite");
  HIPCHK(hipStreamSynchronize(X.stream));
  const size_t N = (size_t)n, nm = (size_t)C.d.max_markers;
  if (ds) HIPCHK(hipMemcpy((void *)C.dev.ds, ds, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)C.dev.xb, x, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)C.dev.yb, y, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(C.dev.hud, udx, sizeof(double) * N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(C.dev.hud + nm, udy, sizeof(double) * N, hipMemcpyHostToDevice));
  return SBT_OK;
}

sbt_status sbt_step(sbt_ctx *ctx, int32_t n) {
  if (!ctx) return fail(SBT_ERR_ARG, "null context");
  if (n < 0) return fail(SBT_ERR_ARG, "negative step count");
  sbt_ctx &X = *ctx;
  if (n == 0) return SBT_OK;
  if (!X.post) {
    sbt_status st = run_prologue(X, X.stream);
    if (st) return st;
  }
  for (int t = 0; t < n;) {
    if (X.persistent && !X.profiling) {
      sbt_status st = run_step_persistent(X, X.stream);
      if (st) return st;
      ++t;
    } else if (X.use_graph && !X.profiling) {
      sbt_status st = ensure_capture_stream(X);
      if (st) return st;
      const int rem = n - t, si = rem >= 4 ? 2 : (rem >= 2 ? 1 : 0);
      const int slot = graph_slot(X, si);
      if (!X.graph[slot]) {
        st = capture_all(X);
        if (st) return st;
      }
      HIPCHK(hipGraphLaunch(X.graph[slot], X.stream));
      // the graph performs the same lattice flips and forcing loops as the
      // eager list
      advance_host(X, kGraphSteps[si]);
      t += kGraphSteps[si];
    } else {
      sbt_status st = run_step_eager(X, X.stream);
      if (st) return st;
      ++t;
    }
  }
  return SBT_OK;
}

sbt_status sbt_synchronize(sbt_ctx *ctx) {
  if (!ctx) return fail(SBT_ERR_ARG, "null context");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  int32_t err[4];
  HIPCHK(hipMemcpy(err, ctx->d_err, sizeof(err), hipMemcpyDeviceToHost));
  if (err[0]) {
    HIPCHK(hipMemset(ctx->d_err, 0, sizeof(err)));
    if (err[0] & ERR_NONFINITE) return fail(SBT_ERR_NONFINITE, "a density became NaN or Inf");
    if (err[0] & ERR_MARKER) return fail(SBT_ERR_MARKER_OUTSIDE, "a marker stencil left the finest owned cells");
    if (err[0] & ERR_CONTRIB)
      return fail(SBT_ERR_MARKER_OUTSIDE, "IBM stencil cells exceed the plan capacity (" + std::to_string(ctx->cell_cap) + ")");
    if (err[0] & ERR_WINDOW) return fail(SBT_ERR_MARKER_OUTSIDE, "IBM window larger than planned");
    if (err[0] & ERR_PLAN) return fail(SBT_ERR_STATE, "IBM plan out of step with the forcing loop");
    if (err[0] & ERR_BARRIER) return fail(SBT_ERR_DEVICE, "persistent step: a grid barrier timed out");
  }
  return SBT_OK;
}

sbt_status sbt_read_fields(sbt_ctx *ctx, int32_t c, int32_t level, double *rho, double *ux, double *uy) {
  sbt_status st = check_level(ctx, c, level);
  if (st) return st;
  if (!rho || !ux || !uy) return fail(SBT_ERR_ARG, "null field");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  const Forest &F = C.F;
  size_t ncell = (size_t)F.nx[level] * F.ny[level];
  for (size_t q = 0; q < ncell; ++q) rho[q] = ux[q] = uy[q] = std::nan("");
  st = readout_level(X, c, level, X.stream);
  if (st) return st;
  size_t n = F.own[level].size();
  std::vector<double> host(n * 3 * kCells);
  HIPCHK(hipMemcpyAsync(host.data(), X.d_stage, sizeof(double) * host.size(), hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  for (size_t k = 0; k < n; ++k) {
    int bx = F.own[level][k] % F.nbx[level], by = F.own[level][k] / F.nbx[level];
    for (int cell = 0; cell < kCells; ++cell) {
      size_t g = (size_t)(by * kB + (cell >> 4)) * F.nx[level] + bx * kB + (cell & 15);
      rho[g] = host[(k * 3 + 0) * kCells + cell];
      ux[g] = host[(k * 3 + 1) * kCells + cell];
      uy[g] = host[(k * 3 + 2) * kCells + cell];
    }
  }
  return SBT_OK;
}

sbt_status sbt_read_fields_blocks(sbt_ctx *ctx, int32_t c, int32_t level, double *out) {
  sbt_status st = check_level(ctx, c, level);
  if (st) return st;
  if (!out) return fail(SBT_ERR_ARG, "null output");
  sbt_ctx &X = *ctx;
  st = readout_level(X, c, level, X.stream);
  if (st) return st;
  size_t n = X.cs[c].F.own[level].size();
  HIPCHK(hipMemcpyAsync(out, X.d_stage, sizeof(double) * n * 3 * kCells, hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  return SBT_OK;
}

sbt_status sbt_diagnostics(sbt_ctx *ctx, int32_t c, double out[3]) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  for (int l = 0; l < C.F.m; ++l) {
    st = readout_level(X, c, l, X.stream);
    if (st) return st;
    HIPCHK(sbt_launch_reduce(X.d_partial, C.lr[l].own1 - C.lr[l].own0, 1.0 / (double)(1 << (2 * l)), X.d_diag,
                             l > 0 ? 1 : 0, X.stream));
  }
  HIPCHK(hipMemcpyAsync(out, X.d_diag, sizeof(double) * 3, hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  return SBT_OK;
}

sbt_status sbt_snapshot_bytes(sbt_ctx *ctx, int32_t c, size_t *bytes) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  if (!bytes) return fail(SBT_ERR_ARG, "null output");
  const CaseHost &C = ctx->cs[c];
  size_t n = 0;
  for (int l = 0; l < C.F.m; ++l) n += (size_t)(C.lr[l].own1 - C.lr[l].own0);
  *bytes = n * 2 * kCells * sizeof(double);
  return SBT_OK;
}

sbt_status sbt_convergence(sbt_ctx *ctx, int32_t c, void *snapshot, size_t bytes, int32_t mode, double out[3]) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  size_t need = 0;
  sbt_snapshot_bytes(ctx, c, &need);
  if (mode < SBT_SNAP_STORE || mode > (SBT_SNAP_STORE | SBT_SNAP_COMPARE)) return fail(SBT_ERR_ARG, "bad mode");
  if (!snapshot || ((uintptr_t)snapshot & 7)) return fail(SBT_ERR_ARG, "snapshot must be an 8-byte aligned device pointer");
  if (bytes < need) return fail(SBT_ERR_BUFSIZE, "snapshot needs " + std::to_string(need) + " bytes");
  if ((mode & SBT_SNAP_COMPARE) && !out) return fail(SBT_ERR_ARG, "null output");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  double *snap = (double *)snapshot;
  double *acc = X.d_diag + 12;
  for (int l = 0; l < C.F.m; ++l) {
    const int n = C.lr[l].own1 - C.lr[l].own0;
    st = readout_level(X, c, l, X.stream);
    if (st) return st;
    const Pool &P = X.pools[C.lr[l].v];
    HIPCHK(sbt_launch_velocity_change(P.d_meta, P.d_codes, P.d_sbits, C.lr[l].own0, n, X.d_stage, snap, mode, X.d_partial,
                                      X.stream));
    if (mode & SBT_SNAP_COMPARE)
      HIPCHK(sbt_launch_reduce(X.d_partial, n, 1.0 / (double)(1 << (2 * l)), acc, l > 0 ? 1 : 0, X.stream));
    snap += (size_t)n * 2 * kCells;
  }
  if (mode & SBT_SNAP_COMPARE) {
    double h[3];
    HIPCHK(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, X.stream));
    HIPCHK(hipStreamSynchronize(X.stream));
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[0] / h[1];
  } else {
    HIPCHK(hipStreamSynchronize(X.stream));
  }
  return SBT_OK;
}

static int64_t read_kcount(sbt_ctx &X, CaseHost &C) {
  int64_t k = 0;
  if (hipMemcpyAsync(&k, C.dev.kcount, sizeof(k), hipMemcpyDeviceToHost, X.stream) != hipSuccess) return -1;
  if (hipStreamSynchronize(X.stream) != hipSuccess) return -1;
  return k;
}

sbt_status sbt_read_marker_forces(sbt_ctx *ctx, int32_t c, double *fx, double *fy) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  if (!C.has_body || C.n_markers == 0) return fail(SBT_ERR_STATE, "case has no body");
  int64_t k = read_kcount(X, C);
  if (k < 0) return fail(SBT_ERR_DEVICE, "kcount read");
  // the last launch computed the IBM of the next substep already
  int64_t done = X.post ? k - 1 : 0;
  if (done <= 0) return fail(SBT_ERR_STATE, "no completed substep yet");
  size_t slot = (size_t)((done - 1) & 1);
  const size_t N = C.n_markers;
  HIPCHK(hipMemcpyAsync(fx, C.dev.ftot + slot * 2 * N, sizeof(double) * N, hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipMemcpyAsync(fy, C.dev.ftot + slot * 2 * N + N, sizeof(double) * N, hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  return SBT_OK;
}

sbt_status sbt_read_force_history(sbt_ctx *ctx, int32_t c, int32_t cap, double *fx, double *fy, int32_t *n_out) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  if (!n_out || cap < 0) return fail(SBT_ERR_ARG, "bad output");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  *n_out = 0;
  if (!C.has_body || C.n_markers == 0) return SBT_OK;
  int64_t k = read_kcount(X, C);
  if (k < 0) return fail(SBT_ERR_DEVICE, "kcount read");
  int64_t done = X.post ? k - 1 : 0;
  int64_t n = std::min<int64_t>({done, (int64_t)cap, (int64_t)C.hist_cap});
  if (n <= 0) return SBT_OK;
  std::vector<double> h(2 * C.hist_cap);
  HIPCHK(hipMemcpyAsync(h.data(), C.dev.hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  for (int64_t t = 0; t < n; ++t) {
    int64_t sub = done - n + t;
    size_t slot = (size_t)(sub % (int64_t)C.hist_cap);
    fx[t] = h[2 * slot];
    fy[t] = h[2 * slot + 1];
  }
  *n_out = (int32_t)n;
  return SBT_OK;
}

sbt_status sbt_force_stats(sbt_ctx *ctx, int32_t c, int32_t n_last, double U, double L, double out[7]) {
  sbt_status st = check_case(ctx, c);
  if (st) return st;
  if (!out || n_last <= 0 || !(U > 0.0) || !(L > 0.0)) return fail(SBT_ERR_ARG, "need n_last > 0, U > 0, L > 0, out");
  sbt_ctx &X = *ctx;
  CaseHost &C = X.cs[c];
  if (!C.has_body || C.n_markers == 0) return fail(SBT_ERR_STATE, "case has no body");
  int64_t k = read_kcount(X, C);
  if (k < 0) return fail(SBT_ERR_DEVICE, "kcount read");
  const int64_t done = X.post ? k - 1 : 0;
  const int64_t n = std::min<int64_t>({done, (int64_t)n_last, (int64_t)C.hist_cap});
  if (n < 2) return fail(SBT_ERR_STATE, "fewer than two recorded substeps");
  const double scale = 1.0 / (0.5 * C.dev.rho0 * U * U * L);
  HIPCHK(sbt_launch_force_stats(C.dev.hist, (int64_t)C.hist_cap, done - n, n, scale, L / U, X.d_diag + 4, X.stream));
  HIPCHK(hipMemcpyAsync(out, X.d_diag + 4, sizeof(double) * 7, hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
  return SBT_OK;
}

// ---- checkpoint -----------------------------------------------------------
struct StateHeader {
  uint64_t magic, bytes;
  int32_t post, V, n_cases, storage, n_pools, pad;
};

sbt_status sbt_state_bytes(sbt_ctx *ctx, size_t *bytes) {
  if (!ctx || !bytes) return fail(SBT_ERR_ARG, "null argument");
  size_t b = sizeof(StateHeader) + sizeof(int32_t) * ctx->pools.size();
  const size_t s = storage_bytes(ctx->storage);
  for (auto &P : ctx->pools) b += 2 * s * kQ * kCells * (size_t)P.total();
  for (auto &C : ctx->cs)
    if (C.has_body) b += sizeof(int64_t) + sizeof(double) * (4 * (size_t)C.d.max_markers + 2 * C.hist_cap);
  *bytes = b;
  return SBT_OK;
}

sbt_status sbt_read_state(sbt_ctx *ctx, void *host, size_t bytes) {
  size_t need = 0;
  sbt_status st = sbt_state_bytes(ctx, &need);
  if (st) return st;
  if (!host || bytes != need) return fail(SBT_ERR_BUFSIZE, "state buffer size mismatch");
  sbt_ctx &X = *ctx;
  HIPCHK(hipStreamSynchronize(X.stream));
  char *p = (char *)host;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = 0x5342545354415445ull;
  h.bytes = need;
  h.post = X.post;
  h.V = X.V;
  h.n_cases = X.n_cases;
  h.storage = X.storage;
  h.n_pools = (int32_t)X.pools.size();
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  for (auto &P : X.pools) {
    int32_t cur = P.cur;
    std::memcpy(p, &cur, sizeof(cur));
    p += sizeof(cur);
  }
  const size_t s = storage_bytes(X.storage);
  for (auto &P : X.pools)
    for (int k = 0; k < 2; ++k) {
      size_t nb = s * kQ * kCells * (size_t)P.total();
      HIPCHK(hipMemcpy(p, P.lat[k], nb, hipMemcpyDeviceToHost));
      p += nb;
    }
  for (auto &C : X.cs) {
    if (!C.has_body) continue;
    HIPCHK(hipMemcpy(p, C.dev.kcount, sizeof(int64_t), hipMemcpyDeviceToHost));
    p += sizeof(int64_t);
    size_t nb = sizeof(double) * 4 * (size_t)C.d.max_markers;
    HIPCHK(hipMemcpy(p, C.dev.ftot, nb, hipMemcpyDeviceToHost));
    p += nb;
    nb = sizeof(double) * 2 * C.hist_cap;
    HIPCHK(hipMemcpy(p, C.dev.hist, nb, hipMemcpyDeviceToHost));
    p += nb;
  }
  return SBT_OK;
}

sbt_status sbt_write_state(sbt_ctx *ctx, const void *host, size_t bytes) {
  size_t need = 0;
  sbt_status st = sbt_state_bytes(ctx, &need);
  if (st) return st;
  if (!host || bytes != need) return fail(SBT_ERR_BUFSIZE, "state buffer size mismatch");
  sbt_ctx &X = *ctx;
  const char *p = (const char *)host;
  StateHeader h;
  std::memcpy(&h, p, sizeof(h));
  if (h.magic != 0x5342545354415445ull || h.V != X.V || h.n_cases != X.n_cases || h.storage != X.storage ||
      h.n_pools != (int32_t)X.pools.size())
    return fail(SBT_ERR_ARG, "state does not match this context");
  p += sizeof(h);
  std::vector<int32_t> curs(X.pools.size());
  std::memcpy(curs.data(), p, sizeof(int32_t) * curs.size());
  p += sizeof(int32_t) * curs.size();
  HIPCHK(hipStreamSynchronize(X.stream));
  const size_t s = storage_bytes(X.storage);
  for (auto &P : X.pools)
    for (int k = 0; k < 2; ++k) {
      size_t nb = s * kQ * kCells * (size_t)P.total();
      HIPCHK(hipMemcpy(P.lat[k], p, nb, hipMemcpyHostToDevice));
      p += nb;
    }
  for (auto &C : X.cs) {
    if (!C.has_body) continue;
    HIPCHK(hipMemcpy(C.dev.kcount, p, sizeof(int64_t), hipMemcpyHostToDevice));
    std::memcpy(&X.k_host, p, sizeof(int64_t));  // every body shares the substep counter
    p += sizeof(int64_t);
    size_t nb = sizeof(double) * 4 * (size_t)C.d.max_markers;
    HIPCHK(hipMemcpy(C.dev.ftot, p, nb, hipMemcpyHostToDevice));
    p += nb;
    nb = sizeof(double) * 2 * C.hist_cap;
    HIPCHK(hipMemcpy(C.dev.hist, p, nb, hipMemcpyHostToDevice));
    p += nb;
  }
  X.post = h.post != 0;
  for (size_t i = 0; i < X.pools.size(); ++i) X.pools[i].cur = curs[i];
  destroy_graphs(X);
  return SBT_OK;
}

// ---- tuning and measurement -------------------------------------------------
sbt_status sbt_set_option(sbt_ctx *ctx, int32_t option, int32_t value) {
  if (!ctx) return fail(SBT_ERR_ARG, "null context");
  switch (option) {
    case SBT_OPT_GRAPH: ctx->use_graph = value != 0; break;
    case SBT_OPT_TILE:
      if (value < 0 || value > 16) return fail(SBT_ERR_ARG, "blocks per workgroup must be 0..16");
      ctx->tile = value;
      ctx->kpw_level.assign(ctx->V, value);
      break;
    case SBT_OPT_XCD_REMAP: ctx->xcd = value != 0; break;
    case SBT_OPT_PERSISTENT: ctx->persistent = value != 0; break;
    case SBT_OPT_BARRIER_SPINS:
      if (value < 0) return fail(SBT_ERR_ARG, "barrier spins must be >= 0");
      ctx->p_spins = value == 0 ? kBarrierSpins : (uint32_t)value;
      break;
    default: return fail(SBT_ERR_ARG, "unknown option");
  }
  destroy_graphs(*ctx);
  return SBT_OK;
}

sbt_status sbt_profile(sbt_ctx *ctx, int32_t n, double out[9]) {
  if (!ctx || !out || n <= 0) return fail(SBT_ERR_ARG, "bad argument");
  sbt_ctx &X = *ctx;
  HIPCHK(hipStreamSynchronize(X.stream));
  X.profiling = true;
  X.ev_level.clear();
  X.ev_fast.clear();
  X.ev_mdf.clear();
  sbt_status st = SBT_OK;
  if (!X.post) st = run_prologue(X, X.stream);
  X.ev_level.clear();
  X.ev_fast.clear();
  X.ev_mdf.clear();
  for (int t = 0; t < n && !st; ++t) st = run_step_eager(X, X.stream);
  X.profiling = false;
  hipError_t e = hipStreamSynchronize(X.stream);
  auto total = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>> &ev) {
    double t = 0;
    for (auto &p : ev) {
      float ms = 0;
      if (!st && e == hipSuccess) (void)hipEventElapsedTime(&ms, p.first, p.second);
      t += ms;
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    double cnt = (double)ev.size();
    ev.clear();
    return std::make_pair(t, cnt);
  };
  auto fl = total(X.ev_fast), gl = total(X.ev_level), md = total(X.ev_mdf);
  if (st) return st;
  if (e != hipSuccess) return fail(SBT_ERR_DEVICE, hipGetErrorString(e));
  int64_t upd = 0;
  sbt_updates_per_step(ctx, &upd);
  const double bpu = 2.0 * kQ * (double)storage_bytes(X.storage);
  out[0] = fl.first + gl.first;
  out[1] = fl.second + gl.second;
  out[2] = md.first;
  out[3] = md.second;
  out[5] = (double)upd * n;
  out[4] = out[5] * bpu;
  out[6] = fl.first;
  out[7] = fl.second;
  out[8] = out[4];  // the tile kernel performs every cell update of a step
  return SBT_OK;
}

static std::string kpw_string(const std::vector<int> &k) {
  std::string r;
  for (size_t i = 0; i < k.size(); ++i) r += (i ? "," : "") + std::to_string(k[i]);
  return r;
}

sbt_status sbt_autotune(sbt_ctx *ctx, int32_t steps, const char *cache_path) {
  if (!ctx || steps <= 0) return fail(SBT_ERR_ARG, "bad argument");
  sbt_ctx &X = *ctx;
  // cache key: storage and the block counts of every pool
  std::ostringstream key;
  key << "st" << X.kvar;
  for (auto &P : X.pools) key << "_" << P.n_own << "/" << P.n_ghost;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      size_t k = line.find("\"" + key.str() + "\"");
      if (k == std::string::npos) continue;
      size_t q0 = line.find('"', line.find(':', k));
      size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
      if (q1 == std::string::npos) continue;
      std::vector<int> got;
      std::stringstream ss(line.substr(q0 + 1, q1 - q0 - 1));
      std::string tok;
      while (std::getline(ss, tok, ',')) got.push_back(std::atoi(tok.c_str()));
      if ((int)got.size() == X.V) {
        X.kpw_level = got;
        destroy_graphs(X);
        return SBT_OK;
      }
    }
  }
  size_t sb = 0;
  sbt_status st = sbt_state_bytes(ctx, &sb);
  if (st) return st;
  std::vector<char> saved(sb);
  st = sbt_read_state(ctx, saved.data(), sb);
  if (st) return st;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // start from the automatic choice, then settle one level at a time,
  // finest first (it carries most of the updates)
  std::vector<int> cur(X.V);
  for (int v = 0; v < X.V; ++v) {
    int nf = 0;
    nf = (int)X.pools[v].fast.size();
    X.kpw_level.assign(X.V, 0);
    cur[v] = blocks_per_wg(X, v, nf);
  }
  auto trial = [&](const std::vector<int> &k, float &ms) -> sbt_status {
    X.kpw_level = k;
    destroy_graphs(X);
    sbt_status r = sbt_step(ctx, 1);  // warm-up (captures the graph)
    if (r) return r;
    HIPCHK(hipEventRecord(e0, X.stream));
    r = sbt_step(ctx, steps);
    if (r) return r;
    HIPCHK(hipEventRecord(e1, X.stream));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return sbt_write_state(ctx, saved.data(), sb);
  };
  float best_ms = 0;
  st = trial(cur, best_ms);
  for (int v = X.V - 1; v >= 0 && !st; --v) {
    for (int k : {1, 2, 3, 4, 6, 8}) {
      if (k == cur[v]) continue;
      std::vector<int> t = cur;
      t[v] = k;
      float ms = 0;
      st = trial(t, ms);
      if (st) break;
      if (ms < best_ms) {
        best_ms = ms;
        cur = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  X.kpw_level = cur;
  destroy_graphs(X);
  if (st) return st;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::stringstream buf;
    buf << in.rdbuf();
    std::string body = buf.str();
    std::vector<std::string> lines;
    std::string line;
    std::istringstream is(body);
    while (std::getline(is, line))
      if (line.find("\":") != std::string::npos && line.find("\"" + key.str() + "\"") == std::string::npos) {
        while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
        lines.push_back(line);
      }
    lines.push_back("  \"" + key.str() + "\": \"" + kpw_string(cur) + "\"");
    std::ofstream out(cache_path);
    out << "{\n";
    for (size_t k = 0; k < lines.size(); ++k) out << lines[k] << (k + 1 < lines.size() ? ",\n" : "\n");
    out << "}\n";
  }
  return SBT_OK;
}

}  // extern "C"
