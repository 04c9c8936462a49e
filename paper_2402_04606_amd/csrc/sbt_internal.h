// Internal structures shared by the host engine and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbt.h"

namespace sbt {

constexpr int kQ = 9;
constexpr int kB = 16;           // block edge in cells
constexpr int kCells = kB * kB;  // cells per block
constexpr int kMaxLevels = 6;
constexpr int kMaxMarkers = 1024; // markers per body (one per lane of the MDF workgroup)

// Block flags.
enum : int32_t {
  BF_GHOST = 1,    // halo block: holds the two halo layers of its level
  BF_CODES = 2,    // block has a per-cell code array (hidden / interface / hidden sources)
  BF_EDGE = 4,     // some source of this block lies outside a non-periodic domain edge
  BF_IBM = 8,      // finest-level block of a case with a body
  BF_SOLID = 16,   // block with solid cells or links into them (interpolated bounce-back)
};

// Per-cell solid bits (blocks with BF_SOLID): bit i = the source x - c_i of
// direction i is solid; SB_SOLID = the cell itself is solid.
enum : uint16_t { SB_SOLID = 0x200 };

// Per-cell code bits (blocks with BF_CODES).
enum : uint16_t {
  CC_HSRC = 0x1FF,    // bit i: source of direction i is hidden (covered by level l+1)
  CC_HIDDEN = 0x200,  // the cell itself is covered by level l+1
  CC_IFACE = 0x400,   // coarse cell next to level l+1: coalesce-on-read and explode
  CC_BAND = 0x800,    // halo block: cell belongs to the two halo layers
};

struct alignas(16) BlockMeta {
  int32_t ox, oy;      // origin, in cells of the block's own level
  int32_t nbr[8];      // same-pool neighbours, directions 1..8 of D2Q9; -1 if none
  int32_t child[4];    // pool v+1 blocks under the quadrants (x>=8) + 2 (y>=8); -1 if none
  int32_t case_id;
  int32_t level;       // true level of the case
  int32_t flags;
  int32_t code;        // index into the cell-code array, or -1
  int32_t solid;       // index into the solid-record arrays, or -1
};
static_assert(sizeof(BlockMeta) == 80, "block table entries stay 80 bytes");

// IBM window of one body for the current finest substep: a dense box of
// finest cells covering every marker stencil.
struct alignas(16) IbmWindow {
  int32_t x0, y0, w, h;
};

struct alignas(16) CaseDev {
  double tau[kMaxLevels];
  double pre[kMaxLevels];      // 1 - 1/(2 tau)
  double fx[kMaxLevels], fy[kMaxLevels];
  double s_cf[kMaxLevels];     // (l-1 -> l) post-collision factor, index l
  double s_fc[kMaxLevels];     // (l+1 -> l) pre-collision factor, index l
  float omega_f[kMaxLevels];   // 1/tau
  float pre_f[kMaxLevels];
  float fx_f[kMaxLevels], fy_f[kMaxLevels];
  float s_cf_f[kMaxLevels], s_fc_f[kMaxLevels];
  double mrt_s[3];             // MRT rates s_e, s_eps, s_q (the shear rate is 1/tau of the level)
  float mrt_s_f[3];
  double rho0;
  double bcu[4][2];
  int32_t bc[4];
  int32_t nx[kMaxLevels], ny[kMaxLevels];
  int32_t per_x, per_y, cf_mode, n_levels;
  // ---- body ----
  int32_t body_kind;           // -1: none
  int32_t n_markers, mdf_iters, hist_cap;
  int32_t win_cap;             // cells of the IBM window buffers
  int32_t bm_x0, bm_y0, bm_w, bm_h;  // finest-level block map: origin and size (blocks)
  double bp[16];
  const double *xb, *yb, *ds;
  double *ftot;                // [2 slots][2][n]: total marker force, slot = substep parity
  double *hist;                // [hist_cap][2]
  int64_t *kcount;             // finest substeps whose forcing loop has run
  double *hud;                 // [2][nm_cap] desired velocity of caller-placed markers
  int32_t nm_cap;              // marker capacity of the plan buffers
  int32_t cell_cap;            // stencil-cell capacity of a plan
  int32_t plan_mask;           // plan buffers - 1 (a power of two >= the finest substeps of a step)
  IbmWindow *win;              // [plan_mask + 1] window of the plan in buffer k & plan_mask
  int32_t *phdr;               // [plan_mask + 1][4] plan header: stamp (low 32 bits of k), stencil cells, status, 0
  double *wF;                  // [plan_mask + 1][2][win_cap] force density in the window, per plan buffer
  int32_t *wCnt, *wIdx;        // [plan_mask + 1][win_cap] plan builder's counters / compact index beyond LDS
  int32_t *p_ij;               // [plan_mask + 1][2][nm_cap] first tap of each marker (x, y)
  double *p_w;                 // [plan_mask + 1][8][nm_cap] Peskin weights of the 4 x and 4 y taps
  double *p_ud;                // [plan_mask + 1][2][nm_cap] desired marker velocity
  uint16_t *p_tap;             // [plan_mask + 1][16][nm_cap] stencil cell of each tap
  int32_t *p_cell;             // [plan_mask + 1][cell_cap][8] window index, 4 source blocks, list start, count, 0
  uint16_t *p_list;            // [plan_mask + 1][16 nm_cap] markers over each stencil cell, ascending
  const int32_t *bmap;         // finest-level block map -> pool index (-1 outside)
};

// Arguments of one level (collide+stream) launch.
struct LevelArgs {
  const BlockMeta *meta;
  const uint16_t *codes;
  const void *src;             // lattice read (post-collision state of the pool)
  void *dst;                   // lattice written
  const BlockMeta *fmeta;      // pool v+1 (finer) or null
  const uint16_t *fcodes;
  const uint16_t *sbits;       // solid records: [record][256] SB_* bits
  const double *sq;            // [record][9][256] wall fraction of the link of each pulled direction
  const void *fprev;           // finer pool lattice read by its last substep
  void *fcur;                  // finer pool current lattice (explosion target)
  const CaseDev *cases;
  const int32_t *list;         // blocks to process, or null for b0 .. b0 + n_blocks - 1
  int32_t b0;
  int32_t n_blocks;            // entries of list (or length of the range)
  int32_t n_fast;              // leading list entries that are interior blocks
  int32_t kpw;                 // interior blocks per workgroup (tile launch, >= 1)
  int32_t ibm_parity;          // IBM plan buffer of the substep (-1: from the forcing-loop counter)
  const int32_t *band;         // halo-band cells (block * 256 + cell), gathered after the blocks
  int32_t n_band;
  int32_t mode;                // MODE_* bits
  int32_t xcd_remap;
  double *out;                 // readout: [block - b0][3][256] rho, ux, uy
  double *partial;             // readout: [block - b0][3] mass, jx, jy partial sums
  int32_t *err;                // device error flags
};

struct MdfArgs {
  const BlockMeta *meta;       // finest pool
  const void *src;             // finest pool lattice the next level launch reads
  const CaseDev *cases;
  const CaseDev *bodies;       // copies of the body cases' parameters, one per body (workgroup)
  int32_t first;               // 1: local read (initial pre-collision state)
  int32_t max_markers;         // LDS marker-table stride (>= every body's markers)
  int32_t cell_cap;            // LDS stencil-cell table size (>= every plan's cells)
  int32_t parity;              // plan buffer of this substep (its index & plan_mask)
  int32_t *err;
};

struct IbmArgs {
  const CaseDev *cases;
  const CaseDev *bodies;       // copies of the body cases' parameters, one per body (workgroup)
  int32_t max_markers;         // LDS list stride (>= every body's markers)
  int32_t cell_cap;            // stencil-cell capacity
  int32_t lds_window;          // window cells whose counters fit in LDS
  int32_t n_bodies;            // bodies per plan: workgroup w builds plan w / n_bodies of body w % n_bodies
  int32_t n_plans;             // plans per body: substeps kcount .. kcount + n_plans - 1
};

// One phase of the persistent step (one launch per step): the plan builder
// of the step's finest substeps, a forcing loop, or a level substep.
enum : int32_t { PP_PREP = 0, PP_MDF = 1, PP_LEVEL = 2 };
struct PPhase {
  int32_t type;
  int32_t n_items;             // PREP: plans (bodies x substeps); MDF: bodies; LEVEL: list + solid blocks
  int32_t n_list;              // LEVEL: entries of lv.list (interior and edge / interface blocks)
  int32_t n_solid;             // LEVEL: entries of `solid`
  const int32_t *solid;
  LevelArgs lv;                // LEVEL (band cells in lv.band / lv.n_band)
  MdfArgs mdf;
  IbmArgs ibm;
};

// Level launch modes: LOCAL = read the cell's own populations (initial
// pre-collision state) instead of streaming; READOUT = moments only, no write.
enum : int32_t { MODE_LOCAL = 1, MODE_READOUT = 2 };

enum : int32_t { ERR_NONFINITE = 1, ERR_MARKER = 2, ERR_CONTRIB = 4, ERR_WINDOW = 8, ERR_PLAN = 16, ERR_BARRIER = 32 };

}  // namespace sbt

// Launchers implemented in sbt_kernels.hip.
extern "C" {
// sbt_create on a given device region; static_dev >= 0 marks a context whose
// region is that device's static array (sbt_destroy releases it).
sbt_status sbt_create_in(const sbt_case_desc *cases, int32_t n_cases, void *device_buf, size_t bytes,
                         void *hip_stream, int32_t static_dev, sbt_ctx **out);
// Mark the static array of device dev free again (sbt_static.hip).
void sbt_static_release(int dev);
// Message for sbt_last_error (the thread's last failure); returns code.
sbt_status sbt_set_error(sbt_status code, const char *msg);
// Generic level kernel: any block (interfaces, domain edges, readout,
// initial collision) and halo-band cells.
// `storage` of the level launches: SBT_F64 .. SBT_BF16S, plus 4 for the MRT collision.
hipError_t sbt_launch_level(int storage, int tile, const sbt::LevelArgs *a, hipStream_t s);
// One LDS-staged stream + collide launch for a level substep: list entries
// [0, n_fast) are interior blocks (no cell codes, no domain edge, all eight
// neighbours present), kpw of them per workgroup; [n_fast, n_blocks) blocks
// next to a finer level or a domain edge; then n_band packed halo-band cells.
hipError_t sbt_launch_level_tile(int storage, const sbt::LevelArgs *a, hipStream_t s);
// One step as a single persistent launch of `groups` 1024-lane workgroups
// (all resident at once) over the phase table `ph` (n_ph entries, device
// memory), phases separated by grid barriers on bar[3] (zero between
// launches).  A barrier wait of `spins` polls that does not pass raises
// ERR_BARRIER in err and every workgroup skips the remaining phases.
hipError_t sbt_launch_step_persistent(int storage, const sbt::PPhase *ph, int n_ph, uint32_t *bar, int32_t *err,
                                      uint32_t spins, int groups, size_t lds_bytes, hipStream_t s);
// Resident 1024-lane workgroups per CU of the persistent step kernel with
// lds_bytes of dynamic LDS (0 if it cannot launch).
int sbt_step_persistent_occupancy(int storage, size_t lds_bytes);
// IBM plan of the next finest substep of every body, one workgroup each.
hipError_t sbt_launch_ibm_prep(const sbt::IbmArgs *a, hipStream_t s);
// Multi-direct forcing loop of the current finest substep on its plan.
hipError_t sbt_launch_mdf(int storage, const sbt::MdfArgs *a, int n_bodies, hipStream_t s);
size_t sbt_mdf_lds_bytes(int max_markers, int cell_cap);
size_t sbt_prep_lds_bytes(int max_markers, int cell_cap, int lds_window);
hipError_t sbt_launch_reduce(const double *partial, int n_blocks, double vol, double *out,
                             int accumulate, hipStream_t s);
// Force statistics of history entries [first, first + n) (ring of cap
// entries) into out[7]; velocity change / snapshot of one level's owned blocks
// (sbt_stats.hip).
hipError_t sbt_launch_force_stats(const double *hist, int64_t cap, int64_t first, int64_t n, double scale,
                                  double l_over_u, double *out, hipStream_t s);
hipError_t sbt_launch_velocity_change(const sbt::BlockMeta *meta, const uint16_t *codes, const uint16_t *sbits, int b0, int n,
                                      const double *fields, double *snap, int mode, double *partial,
                                      hipStream_t s);
hipError_t sbt_launch_fill_nan(void *p, size_t n_elems, int storage, hipStream_t s);
// f = f^eq(rho, u) on the owned cells of blocks [b0, b0+n) from per-block FP64
// fields [n][3][256], or from the constant state u0 = {rho, ux, uy} when
// fields is null (u0 null: rest at rho0).
hipError_t sbt_launch_init(int storage, const sbt::BlockMeta *meta, const uint16_t *codes,
                           const sbt::CaseDev *cases, void *lat, int b0, int n, const double *fields,
                           const double *u0, hipStream_t s);
}
