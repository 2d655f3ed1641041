// Internal declarations shared by the host plan code and the HIP kernels of libkldi.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/kldi.h"

namespace kldi {

constexpr int kG = 128;          // points per grid block
constexpr int kD = 32;           // AOs per tile
constexpr int kChunk = 4;        // AO tiles per workgroup row chunk (one per wave)
constexpr int kMaxTilesPerBlock = 512;

// Device view of the basis in internal (reordered) AO order.
struct BasisDev {
  const double *sh_xyz;    // [n_shells*3] centre of each internal shell
  const int *sh_prim;      // [n_shells*2] primitive range
  const int *sh_l;         // [n_shells]
  const int *sh_ao0;       // [n_shells] first internal AO
  const double *pexp;      // [n_prim]
  const double *pcoef;     // [n_prim]
  const int *ao_shell;     // [n_ao_pad] internal shell of each AO, -1 on padding rows
  const int *ao_comp;      // [n_ao_pad] cartesian powers packed lx | ly<<2 | lz<<4
  const int *tile_sh;      // [n_tiles*2] shells overlapping each tile
  int n_ao;
  int n_tiles;
};

// Device view of the reordered, padded grid.
struct GridDev {
  const double *x, *y, *z, *w;   // [n_pad]
  const int64_t *orig;           // [n_pad] caller index, -1 on padding
  int64_t n_blocks;
};

// Retained block structure (BCS(C) by grid block, plus a dense (block, tile) -> position map).
struct StructDev {
  const int64_t *blk_off;  // [n_blocks+1] first retained tile of each block
  const int *ret_p;        // [n_ret] AO tile of each retained tile
  const int *ret_r;        // [n_ret] grid block of each retained tile
  const int *idx_map;      // [n_blocks*n_tiles] position within S_r or -1
  const double *bphi;      // [n_ret] max |Phi| of the tile
};

struct EvalDev {
  void *Dt;                // [n_tiles^2 * 1024] internal tiled D, working precision
  double *amax;            // [n_tiles^2] max |D_pq|
  void *phi;               // [n_ret * 4096] Phi workspace, working precision
  void *zws;               // [n_ret * 4096] Z workspace
  double *zmax;            // [n_ret]
  double *eblk;            // [n_blocks]
  double *vpart;           // [n_items * 16384]
  double *mfull;           // [(n_chunks*128)^2]
  unsigned long long *counters;  // [4]: pairs X, pairs V, nonfinite flag, spare
};

struct VItem {
  int pc, qc;
  int r0, r1;
};

struct Plan {
  int device = 0;
  kldi_opts opts{};
  bool gga = false;
  int n_ao = 0, n_tiles = 0, n_chunks = 0, n_shells = 0;
  int64_t n_points = 0, n_blocks = 0, n_pad = 0, n_ret = 0, n_cand = 0;
  int max_np = 0;
  int v_segment = 0;
  std::vector<int32_t> ao_perm;       // internal -> caller
  std::vector<int64_t> pt_perm;       // internal -> caller
  std::vector<int64_t> blk_off_h;
  std::vector<int32_t> ret_p_h;
  std::vector<double> bphi_h;
  std::vector<VItem> items_h;
  int n_pairs = 0;
  double plan_ms = 0.0;
  size_t bytes = 0;
  std::vector<void *> allocs;
  // device
  BasisDev basis{};
  GridDev grid{};
  StructDev st{};
  EvalDev ev{};
  VItem *items = nullptr;
  int *pair_ptr = nullptr;   // [n_pairs+1] CSR over pair_items
  int *pair_items = nullptr; // item indices grouped by chunk pair, segment order
  int *pair_pq = nullptr;    // [2*n_pairs] (row chunk, column chunk) of each pair
  int32_t *ao_perm_d = nullptr;
  // optional per-stage timing: events[slot][KLDI_N_STAGES + 1]
  bool timing = false;
  int n_timed = 0;
  std::vector<hipEvent_t> events;
};

constexpr int kTimingSlots = 256;

// error reporting (host.cpp)
void set_error(const std::string &msg);

// launchers (kernels.hip); each returns hipSuccess or the launch error
hipError_t launch_screen(const BasisDev &b, const GridDev &g, const int *cand_p, const int64_t *cand_r,
                         int64_t n_cand, bool gga, double *out_b, double *out_g, hipStream_t s);
hipError_t launch_eval(const Plan &P, const double *D, double *rho, double *exc, double *vxc, hipStream_t s,
                       hipEvent_t *ev /* KLDI_N_STAGES + 1 events, or NULL */);

}  // namespace kldi
