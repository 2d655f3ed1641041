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
constexpr int kMlpWidth = 64;       // hidden width of the functional surrogate
constexpr int kMlpParams = 8707;    // 2-64-64-64-3 weights and biases

// Device view of a trained functional surrogate.
struct MlpDev {
  const unsigned short *theta_b;  // [kMlpParams] BF16 weights (inference)
  const float *bias;              // [kMlpParams] FP32 master parameters (biases read from here)
  double box[4];                  // training range of log rho and log sigma
  double tmean[3], tstd[3];       // target standardisation
  double rho_min;                 // below this density the analytic functional is used
};

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
  void *phi;               // [max chunk retained tiles * 4096] Phi workspace, working precision
  void *zws;               // [max chunk retained tiles * 4096] Z workspace
  double *xpart;           // [max chunk X items * 4 * 128] rho / grad rho partials of each X work item
  double *coef;            // [n_pad * 4] Z coefficients per point
  double *zmax;            // [n_ret]
  double *eblk;            // [n_blocks]
  double *vpart;           // [n_items * 16384]
  int *vflag;              // [n_items] 1 if the item wrote a partial
  unsigned short *vmask;   // [max chunk blocks * n_pairs] executable tile pairs of each chunk pair
  double *mfull;           // [(n_chunks*128)^2]
  unsigned long long *counters;  // [4]: pairs X, pairs V, nonfinite flag, points on the surrogate
  double *escratch;        // [1] E_xc of kldi_eval_grid
};

// A range of grid blocks processed with one filling of the Phi / Z workspaces.
struct GridChunk {
  int64_t blk0, blk1;      // grid blocks
  int64_t ret0, ret1;      // retained tiles (blk_off at the block boundaries)
  int64_t xit0, xit1;      // X work items
  int64_t vit0, vit1;      // Vxc work items (whole segments)
};

struct VItem {
  int pc, qc;
  int r0, r1;
  int pair;      // index of (pc, qc) in the pair table
  int pad;
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
  int64_t n_xitems = 0;
  int *xit_r = nullptr;        // [n_xitems] grid block of each X work item
  int *xit_c = nullptr;        // [n_xitems] chunk index within S_r
  int64_t *blk_item_off = nullptr;  // [n_blocks+1]
  std::vector<int64_t> blk_item_off_h;
  std::vector<GridChunk> chunks_h;
  VItem *items = nullptr;
  int *pair_ptr = nullptr;   // [n_pairs+1] CSR over pair_items
  int *pair_items = nullptr; // item indices grouped by chunk pair, segment order
  int *pair_pq = nullptr;    // [2*n_pairs] (row chunk, column chunk) of each pair
  int *cinfo = nullptr;      // [n_blocks*n_chunks] (first position in S_r) << 4 | retained mask
  int32_t *ao_perm_d = nullptr;
  // functional surrogate attached with kldi_plan_attach_mlp
  bool has_mlp = false;
  MlpDev mlp{};
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
hipError_t launch_eval(const Plan &P, const double *D, double *rho, double *sigma, double *exc, double *vxc,
                       hipStream_t s, hipEvent_t *ev /* KLDI_N_STAGES + 1 events, or NULL */);
hipError_t launch_xc_arrays(int xc, const double *rho, const double *sigma, int64_t n, double rho_cut, double *f,
                            double *vr, double *vs, hipStream_t s);
// functional surrogate (mlp.hip)
hipError_t mlp_launch_grad(const float *theta, const float *x, const float *t, int64_t n, int64_t start, int64_t count,
                           int64_t pa, int64_t pb, float *gpart, double *lpart, hipStream_t s);
hipError_t mlp_launch_adam(float *theta, float *m, float *v, void *theta_b, const float *gpart, int n_wg, float lr,
                           int step, float *grad_out, hipStream_t s);
hipError_t mlp_launch_tobf16(const float *theta, void *theta_b, hipStream_t s);
hipError_t mlp_launch_loss_sum(const double *lpart, int n, double *out, hipStream_t s);
hipError_t mlp_launch_flags(const double *rho, int64_t n, double rho_min, int *flag, int *blk_count, hipStream_t s);
hipError_t mlp_launch_compact(const double *rho, const double *sigma, int64_t n, const int *flag, const int64_t *blk_off,
                              double *rho_c, double *sigma_c, hipStream_t s);
hipError_t mlp_launch_logrange(const double *rho, const double *sigma, int64_t n, double *out, int nblk, hipStream_t s);
hipError_t mlp_launch_data(const double *rho, const double *sigma, int64_t n, int xc, const double *box, float *x,
                           double *traw, double *stat, int nblk, hipStream_t s);
hipError_t mlp_launch_standardise(const double *traw, int64_t n, const double *mean, const double *sd, float *t,
                                  hipStream_t s);
namespace dev {
struct FArgs;
}
hipError_t mlp_launch_xfunc(const dev::FArgs &fa, const MlpDev &m, int64_t nblk, hipStream_t s);
hipError_t mlp_launch_forward(const MlpDev &m, const double *rho, const double *sigma, int64_t n, int xc, double *f,
                              double *vr, double *vs, int *used, hipStream_t s);

}  // namespace kldi

struct kldi_plan {
  kldi::Plan impl;
};
