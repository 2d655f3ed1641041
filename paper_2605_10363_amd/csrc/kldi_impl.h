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
constexpr int kGSeg = 64;        // parts of each row chunk's item sequence in the gradient's final reduction
constexpr int kChunk = 4;        // AO tiles per workgroup row chunk (one per wave)
constexpr int kMaxTilesPerBlock = 512;
// Largest plan (in grid blocks) the queue schedule accepts.  A persistent form of that schedule
// (workgroups pulling items from atomic counters) went silent on the GPU at the sizes of the 200-atom
// chain and of eight batch molecules without a cause being found; the present one-workgroup-per-item
// form has been run only on plans up to the 12-atom workload (413 blocks), so it stays within that class.
constexpr int64_t kQueueMaxBlocks = 1024;
constexpr int kMlpWidth = 64;       // hidden width of the functional surrogate
constexpr int kMlpParams = 8707;    // 2-64-64-64-3 weights and biases

// BF16 pieces per operand of the X product (0: the plan's operands are FP64 or FP32)
inline bool is_mgga_xc(int xc) { return xc == KLDI_XC_MVS || xc == KLDI_XC_MVS_X; }
inline int bf16_pieces(int prec) { return prec == KLDI_PREC_BF16X3 ? 2 : (prec == KLDI_PREC_BF16X6 ? 3 : 0); }

// Device view of a trained functional surrogate.  Every field points into the network's own device
// memory, which training updates in place, so a plan (or a captured graph) holding the view always
// reads the current parameters and statistics.
struct MlpDev {
  const unsigned short *theta_b;  // [kMlpParams] BF16 weights (inference)
  const float *bias;              // [kMlpParams] FP32 master parameters (biases read from here)
  const double *stats;            // [kMlpStats]: box[4] (training range of log rho, log sigma),
                                  // tmean[3], tstd[3] (target standardisation), rho_min (below it
                                  // the analytic functional is used)
};
constexpr int kMlpStats = 11;
constexpr int64_t kMlpStaticMaxPoints = 16384;   // batch limit of the allocation-free training step

// A plan holds one molecule or a batch of independent molecules in one index space: the AO tiles,
// grid blocks, retained tiles and work items of all molecules are numbered consecutively, and every
// tile or block belongs to exactly one molecule.  Per-molecule offsets:
struct MolDev {
  int tile0, nt;          // first AO tile, AO tiles
  int nc;                 // chunks of 4 tiles
  int pair0, npairs;      // Vxc chunk pairs (global index range)
  int n_ao;               // AOs
  int ld;                 // leading dimension of the molecule's M workspace (nc * 128)
  int pad_;
  int64_t row0;           // first row of the molecule in the stacked caller AO index (sum of n_ao)
  int64_t dt0;            // first (p, q) tile pair in Dt / amax (sum of nt^2)
  int64_t d0;             // first element of D and Vxc in the packed caller arrays (sum of n_ao^2)
  int64_t blk0, blk1;     // grid blocks
  int64_t mf0;            // first element of the M workspace
};

// Caller buffers of the running evaluation.  k_begin writes them to device memory at the start of
// each evaluation, so a captured graph of the remaining kernels serves any buffers.
struct IoDev {
  const double *D;        // packed D (molecule m at MolDev::d0, n_ao x n_ao row-major)
  double *rho;            // packed rho in caller point order, or NULL
  double *sigma;          // packed sigma, or NULL
  double *exc;            // [n_mol]
  double *vxc;            // packed Vxc, or NULL
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
  const int *tile_nv;      // [n_tiles] AOs of each tile (32 but on a molecule's last tile)
  // [n_shells * kShRec] the same shell data packed per shell (one 96-byte record, read with wide scalar
  // loads): centre x y z; int32 first internal AO and l | n_prim << 2; int32 first primitive; the first
  // kShPrimIn primitives as (exponent, coefficient); further primitives from pexp / pcoef
  const double *shrec;
};
constexpr int kShRec = 11;      // doubles per shell record
constexpr int kShPrimIn = 3;    // primitives held in a shell record

// Device view of the reordered, padded grid.
struct GridDev {
  const double *x, *y, *z, *w;   // [n_pad]
  const int64_t *orig;           // [n_pad] caller index (packed over molecules), -1 on padding
  int64_t n_blocks;
};

// Retained block structure (BCS(C) by grid block) and the molecule table.
struct StructDev {
  const int64_t *blk_off;  // [n_blocks+1] first retained tile of each block
  const int *ret_p;        // [n_ret] AO tile of each retained tile
  const int *ret_r;        // [n_ret] grid block of each retained tile
  const double *bphi;      // [n_ret] max |Phi| of the tile
  const int *blk_mol;      // [n_blocks] molecule of each block
  const MolDev *mol;       // [n_mol]
  int n_mol;
};

struct EvalDev {
  void *Dt;                // [sum nt^2 * 1024] internal tiled D, working precision (BF16 split plans:
                           // [sum nt^2][piece][1024] BF16 pieces)
  double *amax;            // [sum nt^2] max |D_pq|
  void *phi;               // [max chunk retained tiles * 4096] Phi workspace, working precision
  void *zws;               // [max chunk retained tiles * 4096] Z workspace
  unsigned short *phil;    // FP32 plans: [max chunk retained tiles * 4096] bf16(Phi - fl32(Phi)); else NULL
  unsigned short *phix;    // BF16 split plans: per retained tile the BF16 pieces of Phi, [piece][AO/8][point][8]
  double *xpart;           // [max chunk X items * 4 * 128] rho / grad rho partials of each X work item
  double *coef;            // [n_pad * 4] Z coefficients per point
  double *zmax;            // [n_ret]
  double *eblk;            // [n_blocks]
  double *vpart;           // [n_items * 16384]
  int *vflag;              // [n_items] 1 if the item wrote a partial
  unsigned short *vmask;   // [max chunk mask entries] executable tile pairs of each (block, chunk pair)
  double *mfull;           // [sum (nc*128)^2]
  unsigned long long *counters;  // [8]: pairs X, pairs V, nonfinite flag, points on the surrogate; [4], [5]:
                                 // pairs of the meta-GGA tau products (X, V), kept apart
  double *tdphi;           // meta-GGA: [max chunk retained tiles * 4096] d_a Phi (one component at a time)
  double *tB;              // meta-GGA: [max chunk retained tiles * 4096] (w v_tau / 4) d_a Phi
  double *tpart[3];        // meta-GGA: per component, X-item partials of D d_a Phi (as xpart)
  double *ctau;            // meta-GGA: [n_pad] w v_tau / 4
  double *escratch;        // [n_mol] E_xc of kldi_eval_grid
  IoDev *io;               // [1] caller buffers of the running evaluation
};

// A range of grid blocks processed with one filling of the Phi / Z workspaces.
struct GridChunk {
  int64_t blk0, blk1;      // grid blocks
  int64_t ret0, ret1;      // retained tiles (blk_off at the block boundaries)
  int64_t xit0, xit1;      // X work items
  int64_t vit0, vit1;      // Vxc work items (whole segments)
};

struct VItem {
  int pc, qc;    // row and column chunk (molecule-local)
  int r0, r1;    // grid blocks of the segment
  int pair;      // global index of (pc, qc) in the pair table
  int lpair;     // index of (pc, qc) among the molecule's pairs
};

// Work order of the GEMM kernels: each grid chunk's items in 8 queues, one per XCD; workgroup b runs
// position b / 8 of queue b % 8.  KLDI_SCHED_GRID deals grid blocks / Vxc segments round-robin over the
// queues (Vxc queues in decreasing estimated cost); KLDI_SCHED_QUEUE cuts contiguous ranges of about
// equal estimated cost, each ordered by decreasing cost.
struct Queues {
  int *order = nullptr;          // [n_items] item ids in queue order
  int64_t *qoff = nullptr;       // [n_gchunks * 9] queue boundaries (positions in order)
  std::vector<int64_t> maxlen_h; // [n_gchunks] longest queue of each grid chunk
};

struct Plan {
  int device = 0;
  kldi_opts opts{};
  bool gga = false;
  int n_mol = 0;
  int n_ao = 0, n_tiles = 0, n_shells = 0;   // totals over molecules
  int64_t n_points = 0, n_blocks = 0, n_pad = 0, n_ret = 0, n_cand = 0;
  int64_t n_dt = 0, n_mfull = 0;
  int max_np = 0, max_nao = 0;
  int v_segment = 0;
  int schedule = KLDI_SCHED_GRID;
  std::vector<MolDev> mols_h;
  std::vector<int32_t> ao_perm;       // internal AO (padded, all molecules) -> caller AO within its molecule
  std::vector<int64_t> pt_perm;       // internal point -> caller point (single-molecule plans)
  std::vector<int64_t> pt_off_h;      // [n_mol+1] first caller point of each molecule
  std::vector<int64_t> blk_off_h;
  std::vector<int32_t> ret_p_h;
  std::vector<int32_t> blk_mol_h;
  std::vector<double> bphi_h;
  std::vector<int64_t> cioff_h, vmoff_h;
  std::vector<int> cinfo_h;
  std::vector<VItem> items_h;
  int n_pairs = 0;
  double plan_ms = 0.0;
  size_t bytes = 0;
  std::vector<void *> allocs;         // held for the plan's life
  std::vector<void *> sched_allocs;   // work lists and workspaces of the current schedule
  size_t sched_bytes = 0;
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
  int *pair_info = nullptr;  // [3*n_pairs] (row chunk, column chunk, molecule) of each pair
  int *cinfo = nullptr;      // per (block, chunk of its molecule): (first position in S_r) << 4 | mask
  int64_t *cioff = nullptr;  // [n_blocks+1] first cinfo entry of each block
  int64_t *vmoff = nullptr;  // [n_blocks+1] first vmask entry of each block
  int32_t *ao_perm_d = nullptr;
  Queues xq, vq;
  int *ditems = nullptr;              // Vxc items of diagonal chunk pairs (pc = qc), grouped by grid chunk
  std::vector<int64_t> dchunk_h;      // [n_gchunks + 1] offsets into ditems
  // nuclear gradient (kldi_eval_grad): workspaces of the current schedule, allocated on first use
  struct GradWs {
    double *gA = nullptr;     // [max chunk retained tiles * 4096] operand of the gradient products
    double *gAmax = nullptr;  // [max chunk retained tiles] max |gA| of each tile
    double *gWmax = nullptr;  // [max chunk retained tiles] max |W| of each tile (W in the Z workspace)
    double *gQ = nullptr;     // GGA: [max chunk retained tiles * 4096] Q^a, the second operand of the products
    double *gQmax = nullptr;  // GGA: [max chunk retained tiles] max |Q^a| of each tile
    double *gpart = nullptr;  // [row chunks * kGSeg * 3 * 128] partial per-AO sums of the final reduction
    double *gD = nullptr;     // FP32 plans: D as FP64 32 x 32 tiles for the contraction of the products
    double *gitem = nullptr;  // [n_items][6][128] per-item contracted partials
    double *gao = nullptr;    // [3][nc * 128] per-AO sums
  } grad_ws;
  int *ao_atom = nullptr;             // [n_ao_pad] caller atom of each internal AO (single-molecule plans), -1 on padding
  int n_atoms0 = 0;                   // atoms of the first molecule
  int64_t max_ret = 0;                // largest retained-tile count of a grid chunk in the current schedule
  // functional surrogate attached with kldi_plan_attach_mlp
  bool has_mlp = false;
  MlpDev mlp{};
  // optional per-stage timing: events[slot][KLDI_N_STAGES + 1]
  bool timing = false;
  int n_timed = 0;
  std::vector<hipEvent_t> events;
  // captured launch graphs of one evaluation after k_begin: [0] without Vxc, [1] with Vxc
  bool use_graph = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  // FP32 plans: k_vdiag runs on a side stream forked from the evaluation's stream before k_vgemm_f32 and
  // joined back after it (default priority, non-blocking)
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

constexpr int kTimingSlots = 256;

// error reporting (host.cpp)
void set_error(const std::string &msg);
// drops the captured graphs (after a change of what one evaluation launches)
void invalidate_graphs(Plan &P);

// launchers (kernels.hip); each returns hipSuccess or the launch error
hipError_t launch_screen(const BasisDev &b, const GridDev &g, const int *cand_p, const int64_t *cand_r,
                         int64_t n_cand, bool gga, double *out_b, double *out_g, hipStream_t s);
// k_begin: record the caller buffers of this evaluation and clear its counters and queues
hipError_t launch_begin(const Plan &P, const IoDev &io, hipStream_t s);
// everything after k_begin (captured into a graph when the plan runs in graph mode)
hipError_t launch_body(const Plan &P, bool want_v, hipStream_t s,
                       hipEvent_t *ev /* KLDI_N_STAGES + 1 events, or NULL */);
// nuclear gradient of a single-molecule FP64 plan after k_begin (grad: [n_atoms * 3] device)
hipError_t launch_grad(const Plan &P, double *grad, hipStream_t s);
hipError_t launch_xc_arrays(int xc, const double *rho, const double *sigma, int64_t n, double rho_cut, double *f,
                            double *vr, double *vs, hipStream_t s);
// functional surrogate (mlp.hip)
hipError_t mlp_launch_grad(const float *theta, const float *x, const float *t, int64_t n, int64_t start, int64_t count,
                           int64_t pa, int64_t pb, float *gpart, double *lpart, hipStream_t s);
hipError_t mlp_launch_adam(float *theta, float *m, float *v, void *theta_b, const float *gpart, int n_wg, float lr,
                           int step, float *grad_out, hipStream_t s);
hipError_t mlp_launch_tobf16(const float *theta, void *theta_b, hipStream_t s);
// one Adam step with the partial gradients in the library's static scratch (n <= kMlpStaticMaxPoints)
hipError_t mlp_launch_step_static(float *theta, float *m, float *v, void *theta_b, const float *x, const float *t,
                                  int64_t n, float lr, int step, double *loss, hipStream_t s);
size_t mlp_static_scratch_bytes();
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
