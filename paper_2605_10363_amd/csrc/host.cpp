// Host side of libkldi: the C ABI, argument validation, the per-geometry plan (reordering, tiling,
// shell radii, screening, retained-block lists) for one molecule or a batch of molecules, the work
// schedule (work lists, per-XCD queue orders, workspaces), graph capture and the autotuner.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <tuple>

#include "kldi_impl.h"

namespace kldi {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

struct Error {
  kldi_status code;
  std::string msg;
};

[[noreturn]] void fail(kldi_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(KLDI_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T *dev_alloc(Plan &P, size_t n, bool sched = false) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(KLDI_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  if (sched) {
    P.sched_allocs.push_back(p);
    P.sched_bytes += bytes;
  } else {
    P.allocs.push_back(p);
    P.bytes += bytes;
  }
  return static_cast<T *>(p);
}

template <class T>
T *dev_upload(Plan &P, const std::vector<T> &h, bool sched = false) {
  T *d = dev_alloc<T>(P, h.size(), sched);
  if (!h.empty()) check_hip(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
  return d;
}

void free_list(std::vector<void *> &v) {
  for (void *p : v) (void)hipFree(p);
  v.clear();
}

void free_graphs(Plan &P) {
  for (hipGraphExec_t &g : P.graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

void free_plan(Plan &P) {
  free_graphs(P);
  if (P.cap_stream) (void)hipStreamDestroy(P.cap_stream);
  P.cap_stream = nullptr;
  if (P.side_stream) (void)hipStreamDestroy(P.side_stream);
  P.side_stream = nullptr;
  if (P.fork_ev) (void)hipEventDestroy(P.fork_ev);
  if (P.join_ev) (void)hipEventDestroy(P.join_ev);
  P.fork_ev = P.join_ev = nullptr;
  free_list(P.sched_allocs);
  free_list(P.allocs);
  for (hipEvent_t e : P.events) (void)hipEventDestroy(e);
  P.events.clear();
}

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian powers in lexicographic order (x, y, z; xx, xy, xz, yy, yz, zz).
void cart_powers(int l, int c, int &lx, int &ly, int &lz) {
  static const int P1[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  static const int P2[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
  if (l == 0) {
    lx = ly = lz = 0;
  } else if (l == 1) {
    lx = P1[c][0]; ly = P1[c][1]; lz = P1[c][2];
  } else {
    lx = P2[c][0]; ly = P2[c][1]; lz = P2[c][2];
  }
}

// Morton key of eq. morton_code: bit k of z at 3k, of y at 3k+1, of x at 3k+2 (20 bits per axis).
uint64_t morton(uint64_t ix, uint64_t iy, uint64_t iz) {
  uint64_t m = 0;
  for (int k = 0; k < 20; ++k) {
    m |= ((iz >> k) & 1ull) << (3 * k);
    m |= ((iy >> k) & 1ull) << (3 * k + 1);
    m |= ((ix >> k) & 1ull) << (3 * k + 2);
  }
  return m;
}

uint64_t discretise(double c, double origin) {
  double q = std::floor((c - origin) * 128.0);
  if (q < 0) q = 0;
  if (q > double((1 << 20) - 1)) q = double((1 << 20) - 1);
  return static_cast<uint64_t>(q);
}

// Upper bound of |chi| (and |grad chi| for GGA) of any component of a shell at distance r:
// |dx^a dy^b dz^c| <= r^l and N_rel <= sqrt(3).
double shell_bound(int l, const double *ex, const double *co, int np, bool gga, double r) {
  double s0 = 0, s1 = 0;
  for (int k = 0; k < np; ++k) {
    double e = std::fabs(co[k]) * std::exp(-ex[k] * r * r);
    s0 += e;
    s1 += 2.0 * ex[k] * e;
  }
  double nmax = (l == 2) ? std::sqrt(3.0) : 1.0;
  double v = nmax * std::pow(r, l) * s0;
  if (gga) {
    double g = nmax * ((l > 0 ? l * std::pow(r, l - 1) * s0 : 0.0) + std::pow(r, l + 1) * s1);
    v = std::max(v, g);
  }
  return v;
}

// Radius beyond which the bound stays below t_b (conservative: the bound is decreasing beyond r0).
double shell_radius(int l, const double *ex, const double *co, int np, bool gga, double t_b) {
  if (!(t_b > 0)) return std::numeric_limits<double>::infinity();
  double amin = ex[0];
  for (int k = 1; k < np; ++k) amin = std::min(amin, ex[k]);
  double r0 = std::sqrt((l + 1.0) / (2.0 * amin));
  if (shell_bound(l, ex, co, np, gga, r0) < t_b) return r0 * 1.000001 + 1e-9;
  double lo = r0, hi = 2.0 * r0 + 1.0;
  while (shell_bound(l, ex, co, np, gga, hi) >= t_b) {
    lo = hi;
    hi *= 2.0;
    if (hi > 1e6) return std::numeric_limits<double>::infinity();
  }
  for (int it = 0; it < 100; ++it) {
    double mid = 0.5 * (lo + hi);
    if (shell_bound(l, ex, co, np, gga, mid) >= t_b) lo = mid; else hi = mid;
  }
  return hi * 1.000001 + 1e-9;
}

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void validate_opts(const kldi_opts *o) {
  if (!(o->t_b >= 0) || !(o->t_d >= 0) || !(o->rho_cut >= 0) || !std::isfinite(o->t_b) ||
      !std::isfinite(o->t_d) || !std::isfinite(o->rho_cut))
    fail(KLDI_E_ARG, "t_b, t_d and rho_cut must be finite and >= 0");
  if (o->grid_block <= 0 || o->grid_block % 64 != 0) fail(KLDI_E_ARG, "grid_block must be a positive multiple of 64");
  if (o->grid_block != kG && o->grid_block != 2 * kG) fail(KLDI_E_UNSUPPORTED, "libkldi supports grid_block = 128 or 256");
  if (o->ao_block != kD) fail(KLDI_E_UNSUPPORTED, "libkldi supports ao_block = 32");
  if (o->prec != KLDI_PREC_FP64 && o->prec != KLDI_PREC_FP32 && o->prec != KLDI_PREC_BF16X3 &&
      o->prec != KLDI_PREC_BF16X6)
    fail(KLDI_E_ARG, "unknown prec");
  if (o->xc != KLDI_XC_LDA_X && o->xc != KLDI_XC_PBE && o->xc != KLDI_XC_PBE_X && !is_mgga_xc(o->xc))
    fail(KLDI_E_ARG, "unknown xc");
  if (is_mgga_xc(o->xc) && o->prec != KLDI_PREC_FP64)
    fail(KLDI_E_UNSUPPORTED, "the meta-GGA functionals run on FP64 plans");
  if (o->v_segment < 0) fail(KLDI_E_ARG, "v_segment must be >= 0");
  if (o->chunk_tiles < 0) fail(KLDI_E_ARG, "chunk_tiles must be >= 0");
  if (o->schedule != KLDI_SCHED_GRID && o->schedule != KLDI_SCHED_QUEUE) fail(KLDI_E_ARG, "unknown schedule");
}

void validate(const kldi_basis *b, const kldi_grid *g) {
  if (!b || !g) fail(KLDI_E_ARG, "basis and grid must not be NULL");
  if (b->n_atoms <= 0) fail(KLDI_E_ARG, "n_atoms must be positive");
  if (b->n_shells <= 0) fail(KLDI_E_ARG, "n_shells must be positive");
  if (!b->atom_xyz || !b->shell_atom || !b->shell_l || !b->shell_prim_ptr || !b->prim_exp || !b->prim_coef)
    fail(KLDI_E_ARG, "basis arrays must not be NULL");
  if (!finite_all(b->atom_xyz, int64_t(b->n_atoms) * 3)) fail(KLDI_E_ARG, "atom_xyz not finite");
  if (b->shell_prim_ptr[0] != 0) fail(KLDI_E_ARG, "shell_prim_ptr[0] must be 0");
  for (int s = 0; s < b->n_shells; ++s) {
    if (b->shell_atom[s] < 0 || b->shell_atom[s] >= b->n_atoms) fail(KLDI_E_ARG, "shell_atom out of range");
    if (b->shell_l[s] < 0 || b->shell_l[s] > 2) fail(KLDI_E_ARG, "shell_l must be 0, 1 or 2");
    if (b->shell_prim_ptr[s + 1] <= b->shell_prim_ptr[s]) fail(KLDI_E_ARG, "shell_prim_ptr must increase");
  }
  int np = b->shell_prim_ptr[b->n_shells];
  for (int k = 0; k < np; ++k) {
    if (!(b->prim_exp[k] > 0) || !std::isfinite(b->prim_exp[k])) fail(KLDI_E_ARG, "prim_exp must be positive");
    if (!std::isfinite(b->prim_coef[k])) fail(KLDI_E_ARG, "prim_coef not finite");
  }
  if (g->n_points <= 0) fail(KLDI_E_ARG, "n_points must be positive");
  if (!g->xyz || !g->weight || !g->point_atom) fail(KLDI_E_ARG, "grid arrays must not be NULL");
  if (g->n_points > (int64_t(1) << 31) - 1024) fail(KLDI_E_UNSUPPORTED, "n_points beyond 2^31");
  if (!finite_all(g->xyz, g->n_points * 3) || !finite_all(g->weight, g->n_points))
    fail(KLDI_E_ARG, "grid coordinates/weights not finite");
  for (int64_t i = 0; i < g->n_points; ++i)
    if (g->point_atom[i] < 0 || g->point_atom[i] >= b->n_atoms) fail(KLDI_E_ARG, "point_atom out of range");
}

// ------------------------------------------------------------------------------------------------
// One molecule's reordering, tiling and candidate (tile, block) pairs, in molecule-local indices.
// ------------------------------------------------------------------------------------------------
struct MolPrep {
  int n_ao = 0, n_tiles = 0, n_shells = 0;
  int64_t n_points = 0, n_blocks = 0;
  std::vector<int32_t> ao_perm;        // internal -> caller AO
  std::vector<int64_t> pt_perm;        // internal -> caller point
  std::vector<double> sh_xyz, pexp, pcoef;
  std::vector<int> sh_prim, sh_l, sh_ao0, ao_shell, ao_comp, tile_sh, tile_nv;
  std::vector<int> ao_atom;            // internal AO -> caller atom (-1 on padding)
  std::vector<double> px, py, pz, pw;
  std::vector<int64_t> porig;
  std::vector<int> cand_p;
  std::vector<int64_t> cand_r;
};

void prepare_mol(MolPrep &M, const kldi_basis *b, const kldi_grid *g, bool gga, double t_b, const int32_t *shell_seq,
                 int pair_blocks) {
  const int na = b->n_atoms, ns = b->n_shells;
  const int64_t npt = g->n_points;
  M.n_points = npt;
  M.n_shells = ns;

  // reordering (Sec. III-B.2): atoms by Morton key of their centres, points grouped by associated
  // atom then Morton-sorted, AOs grouped by atom
  double origin[3];
  for (int d = 0; d < 3; ++d) {
    double m = b->atom_xyz[d];
    for (int a = 0; a < na; ++a) m = std::min(m, b->atom_xyz[3 * a + d]);
    for (int64_t i = 0; i < npt; ++i) m = std::min(m, g->xyz[3 * i + d]);
    origin[d] = m;
  }
  std::vector<uint64_t> akey(na);
  for (int a = 0; a < na; ++a)
    akey[a] = morton(discretise(b->atom_xyz[3 * a], origin[0]), discretise(b->atom_xyz[3 * a + 1], origin[1]),
                     discretise(b->atom_xyz[3 * a + 2], origin[2]));
  std::vector<int> aorder(na);
  std::iota(aorder.begin(), aorder.end(), 0);
  std::stable_sort(aorder.begin(), aorder.end(), [&](int x, int y) { return akey[x] < akey[y]; });
  std::vector<int> arank(na);
  for (int i = 0; i < na; ++i) arank[aorder[i]] = i;

  std::vector<int64_t> cao0(ns);  // caller first AO of each shell
  {
    int64_t off = 0;
    for (int s = 0; s < ns; ++s) {
      cao0[s] = off;
      off += ncart(b->shell_l[s]);
    }
    if (off > (1 << 24)) fail(KLDI_E_UNSUPPORTED, "more than 2^24 AOs");
    M.n_ao = int(off);
  }
  std::vector<std::vector<int>> shells_of(na);
  for (int s = 0; s < ns; ++s) shells_of[b->shell_atom[s]].push_back(s);
  std::vector<int> shell_order;  // internal -> caller shell
  if (shell_seq) {
    // a caller shell order (the overlap-signature reordering, kldi_overlap_order): a permutation
    std::vector<char> seen(ns, 0);
    for (int i = 0; i < ns; ++i) {
      const int s = shell_seq[i];
      if (s < 0 || s >= ns || seen[s]) fail(KLDI_E_ARG, "shell_order is not a permutation of the shells");
      seen[s] = 1;
      shell_order.push_back(s);
    }
  } else {
    for (int a : aorder)
      for (int s : shells_of[a]) shell_order.push_back(s);
  }

  M.n_tiles = (M.n_ao + kD - 1) / kD;
  const int nao_pad = M.n_tiles * kD;
  M.sh_xyz.assign(3 * ns, 0.0);
  M.sh_prim.assign(2 * ns, 0);
  M.sh_l.assign(ns, 0);
  M.sh_ao0.assign(ns, 0);
  M.ao_shell.assign(nao_pad, -1);
  M.ao_comp.assign(nao_pad, 0);
  M.ao_perm.assign(M.n_ao, 0);
  M.ao_atom.assign(nao_pad, -1);
  {
    int ao = 0;
    for (int is = 0; is < ns; ++is) {
      int s = shell_order[is];
      int l = b->shell_l[s];
      for (int d = 0; d < 3; ++d) M.sh_xyz[3 * is + d] = b->atom_xyz[3 * b->shell_atom[s] + d];
      M.sh_prim[2 * is] = int(M.pexp.size());
      for (int k = b->shell_prim_ptr[s]; k < b->shell_prim_ptr[s + 1]; ++k) {
        M.pexp.push_back(b->prim_exp[k]);
        M.pcoef.push_back(b->prim_coef[k]);
      }
      M.sh_prim[2 * is + 1] = int(M.pexp.size());
      M.sh_l[is] = l;
      M.sh_ao0[is] = ao;
      for (int c = 0; c < ncart(l); ++c) {
        int lx, ly, lz;
        cart_powers(l, c, lx, ly, lz);
        M.ao_shell[ao] = is;
        M.ao_comp[ao] = lx | (ly << 2) | (lz << 4);
        M.ao_perm[ao] = int32_t(cao0[s] + c);
        M.ao_atom[ao] = b->shell_atom[s];
        ++ao;
      }
    }
  }
  M.tile_sh.assign(2 * M.n_tiles, 0);
  M.tile_nv.assign(M.n_tiles, 0);
  for (int p = 0; p < M.n_tiles; ++p) {
    int a0 = p * kD, a1 = std::min(M.n_ao, a0 + kD) - 1;
    M.tile_sh[2 * p] = M.ao_shell[a0];
    M.tile_sh[2 * p + 1] = M.ao_shell[a1] + 1;
    M.tile_nv[p] = a1 - a0 + 1;
  }

  // points
  std::vector<uint64_t> pkey(npt);
  for (int64_t i = 0; i < npt; ++i)
    pkey[i] = morton(discretise(g->xyz[3 * i], origin[0]), discretise(g->xyz[3 * i + 1], origin[1]),
                     discretise(g->xyz[3 * i + 2], origin[2]));
  M.pt_perm.resize(npt);
  std::iota(M.pt_perm.begin(), M.pt_perm.end(), int64_t(0));
  std::stable_sort(M.pt_perm.begin(), M.pt_perm.end(), [&](int64_t x, int64_t y) {
    int rx = arank[g->point_atom[x]], ry = arank[g->point_atom[y]];
    if (rx != ry) return rx < ry;
    return pkey[x] < pkey[y];
  });
  M.n_blocks = (npt + kG - 1) / kG;
  const int64_t n_pad = M.n_blocks * kG;
  M.px.assign(n_pad, 0.0);
  M.py.assign(n_pad, 0.0);
  M.pz.assign(n_pad, 0.0);
  M.pw.assign(n_pad, 0.0);
  M.porig.assign(n_pad, -1);
  for (int64_t i = 0; i < n_pad; ++i) {
    int64_t c = M.pt_perm[std::min(i, npt - 1)];
    M.px[i] = g->xyz[3 * c];
    M.py[i] = g->xyz[3 * c + 1];
    M.pz[i] = g->xyz[3 * c + 2];
    if (i < npt) {
      M.pw[i] = g->weight[c];
      M.porig[i] = c;
    }
  }

  // shell radii and candidate (tile, block) pairs: a shell of the tile within its radius of the
  // block's bounding box
  std::vector<double> rad(ns);
  for (int is = 0; is < ns; ++is)
    rad[is] = shell_radius(M.sh_l[is], &M.pexp[M.sh_prim[2 * is]], &M.pcoef[M.sh_prim[2 * is]],
                           M.sh_prim[2 * is + 1] - M.sh_prim[2 * is], gga, t_b);
  // 256-point screening blocks (pair_blocks): the two 128-point compute blocks of a pair share the
  // bounding box, hence the candidate list
  for (int64_t r = 0; r < M.n_blocks; ++r) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    const int64_t rb0 = pair_blocks ? (r & ~int64_t(1)) : r, rb1 = pair_blocks ? rb0 + 2 : r + 1;
    for (int64_t i = rb0 * kG; i < std::min(npt, rb1 * kG); ++i) {
      lo[0] = std::min(lo[0], M.px[i]); hi[0] = std::max(hi[0], M.px[i]);
      lo[1] = std::min(lo[1], M.py[i]); hi[1] = std::max(hi[1], M.py[i]);
      lo[2] = std::min(lo[2], M.pz[i]); hi[2] = std::max(hi[2], M.pz[i]);
    }
    for (int p = 0; p < M.n_tiles; ++p) {
      bool near = false;
      for (int is = M.tile_sh[2 * p]; is < M.tile_sh[2 * p + 1] && !near; ++is) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) {
          double c = M.sh_xyz[3 * is + d];
          double e = std::max(0.0, std::max(lo[d] - c, c - hi[d]));
          d2 += e * e;
        }
        near = std::sqrt(d2) <= rad[is];
      }
      if (near) {
        M.cand_p.push_back(p);
        M.cand_r.push_back(r);
      }
    }
  }
}

template <class T, class F>
void append(std::vector<T> &dst, const std::vector<T> &src, F &&map) {
  for (const T &v : src) dst.push_back(map(v));
}

// ------------------------------------------------------------------------------------------------
// Work schedule: X and Vxc work lists for a Vxc segment length, grid chunks, the per-XCD queue
// orders, and the workspaces sized by them.  Rebuilt by the autotuner.
// ------------------------------------------------------------------------------------------------
void visit_v_items(const Plan &P, const std::vector<std::vector<int>> &blk_chunks, int seg,
                   const std::function<void(int m, int lpair, int r0, int r1)> &emit) {
  for (int m = 0; m < P.n_mol; ++m) {
    const MolDev &mo = P.mols_h[m];
    const bool gga = P.gga;
    const int nc = mo.nc;
    std::vector<int> stamp(mo.npairs, -1);
    auto pair_index = [&](int pc, int qc) { return gga ? pc * nc + qc : pc * nc - pc * (pc - 1) / 2 + (qc - pc); };
    const int64_t nseg = (mo.blk1 - mo.blk0 + seg - 1) / seg;
    for (int64_t sg = 0; sg < nseg; ++sg) {
      const int r0 = int(mo.blk0 + sg * seg), r1 = int(std::min<int64_t>(mo.blk1, mo.blk0 + (sg + 1) * seg));
      std::vector<int> act;
      for (int r = r0; r < r1; ++r)
        for (int pc : blk_chunks[r])
          for (int qc : blk_chunks[r]) {
            if (!gga && qc < pc) continue;
            const int pi = pair_index(pc, qc);
            if (stamp[pi] != int(sg)) {
              stamp[pi] = int(sg);
              act.push_back(pi);
            }
          }
      std::sort(act.begin(), act.end());
      for (int pi : act) emit(m, pi, r0, r1);
    }
  }
}

std::vector<std::vector<int>> block_chunks(const Plan &P) {
  std::vector<std::vector<int>> bc(P.n_blocks);
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    const int tile0 = P.mols_h[P.blk_mol_h[r]].tile0;
    for (int64_t k = P.blk_off_h[r]; k < P.blk_off_h[r + 1]; ++k) {
      const int c = (P.ret_p_h[k] - tile0) / kChunk;
      if (bc[r].empty() || bc[r].back() != c) bc[r].push_back(c);
    }
  }
  return bc;
}

int64_t count_v_items(const Plan &P, const std::vector<std::vector<int>> &blk_chunks, int seg) {
  int64_t n = 0;
  visit_v_items(P, blk_chunks, seg, [&](int, int, int, int) { ++n; });
  return n;
}

// Deal groups of consecutive items (group_start; the last ends at i1) round-robin over 8 queues, group g
// to queue g % 8, each queue keeping its groups' items in order, or -- with item costs (indexed by item
// - i0) -- ordered by decreasing cost (stable).  Appends to order and writes 9 boundaries to qoff.
void make_rr_queues(int64_t i0, int64_t i1, const std::vector<int64_t> &group_start, const std::vector<double> *cost,
                    std::vector<int> &order, int64_t *qoff) {
  const size_t ng = group_start.size();
  for (int x = 0; x < 8; ++x) {
    qoff[x] = int64_t(order.size());
    for (size_t g = size_t(x); g < ng; g += 8) {
      const int64_t e = (g + 1 < ng) ? group_start[g + 1] : i1;
      for (int64_t it = group_start[g]; it < e; ++it) order.push_back(int(it));
    }
    if (cost)
      std::stable_sort(order.begin() + qoff[x], order.end(),
                       [&](int a, int b) { return (*cost)[size_t(a - i0)] > (*cost)[size_t(b - i0)]; });
  }
  qoff[8] = int64_t(order.size());
}

// Split items [i0, i1) -- groups of consecutive items given by group_end -- into 8 contiguous ranges
// of about equal cost, then order each range by decreasing group cost (items of a group stay
// together, in their order).  Appends to order and writes 9 boundaries to qoff.
void make_queues(int64_t i0, int64_t i1, const std::vector<int64_t> &group_start, const std::vector<double> &gcost,
                 std::vector<int> &order, int64_t *qoff) {
  const size_t ng = gcost.size();
  double total = 0.0;
  for (double c : gcost) total += c;
  size_t g = 0;
  double acc = 0.0;
  for (int x = 0; x < 8; ++x) {
    qoff[x] = int64_t(order.size());
    const double target = total * (x + 1) / 8.0;
    std::vector<size_t> mine;
    while (g < ng && (acc + 0.5 * gcost[g] <= target || x == 7)) {
      mine.push_back(g);
      acc += gcost[g];
      ++g;
    }
    std::stable_sort(mine.begin(), mine.end(), [&](size_t a, size_t b) { return gcost[a] > gcost[b]; });
    for (size_t k : mine) {
      const int64_t e = (k + 1 < ng) ? group_start[k + 1] : i1;
      for (int64_t it = group_start[k]; it < e; ++it) order.push_back(int(it));
    }
  }
  qoff[8] = int64_t(order.size());
  (void)i0;
}

void build_schedule(Plan &P, int seg, int schedule, int64_t chunk_tiles) {
  if (schedule == KLDI_SCHED_QUEUE && P.n_blocks > kQueueMaxBlocks)
    fail(KLDI_E_UNSUPPORTED, "the queue schedule is limited to plans of at most " + std::to_string(kQueueMaxBlocks) +
                                 " grid blocks");
  free_list(P.sched_allocs);
  P.sched_bytes = 0;
  P.grad_ws = Plan::GradWs{};
  P.items_h.clear();
  P.chunks_h.clear();
  P.blk_item_off_h.clear();
  const auto blk_chunks = block_chunks(P);

  // X work items: (block, chunk of 4 consecutive retained tiles), block-major
  std::vector<int> xr, xc;
  std::vector<int64_t> boff(P.n_blocks + 1, 0);
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    const int np = int(P.blk_off_h[r + 1] - P.blk_off_h[r]);
    for (int c = 0; kChunk * c < np; ++c) {
      xr.push_back(int(r));
      xc.push_back(c);
    }
    boff[r + 1] = int64_t(xr.size());
  }
  P.n_xitems = int64_t(xr.size());
  P.xit_r = dev_upload(P, xr, true);
  P.xit_c = dev_upload(P, xc, true);
  P.blk_item_off = dev_upload(P, boff, true);
  P.blk_item_off_h = boff;

  // Vxc work items: (molecule, row chunk, column chunk, segment of grid blocks)
  size_t fr0 = 0, tot0 = 0;
  check_hip(hipMemGetInfo(&fr0, &tot0), "hipMemGetInfo");
  if (seg <= 0) {
    // shortest segment (better L2 sharing among the items of a segment) whose FP64 partials fit a
    // budget of min(16 GiB, 1/5 of free device memory)
    const size_t budget = std::min<size_t>(size_t(16) << 30, fr0 / 5);
    int64_t maxblk = 1;
    for (const MolDev &mo : P.mols_h) maxblk = std::max<int64_t>(maxblk, mo.blk1 - mo.blk0);
    for (seg = 16;; seg *= 2)
      if (size_t(count_v_items(P, blk_chunks, seg)) * 16384 * 8 <= budget || seg >= maxblk) break;
  }
  // 256-point blocks pair compute blocks 2k, 2k + 1 of a molecule: segments (and so grid chunks) start at
  // even offsets
  if (P.opts.grid_block == 2 * kG && (seg & 1)) ++seg;
  P.v_segment = seg;
  P.schedule = schedule;
  std::vector<std::vector<int>> pair_lists(P.n_pairs);
  std::vector<int> pinfo_pc(P.n_pairs), pinfo_qc(P.n_pairs);
  for (int m = 0; m < P.n_mol; ++m) {
    const MolDev &mo = P.mols_h[m];
    for (int pc = 0; pc < mo.nc; ++pc)
      for (int qc = P.gga ? 0 : pc; qc < mo.nc; ++qc) {
        const int lp = P.gga ? pc * mo.nc + qc : pc * mo.nc - pc * (pc - 1) / 2 + (qc - pc);
        pinfo_pc[mo.pair0 + lp] = pc;
        pinfo_qc[mo.pair0 + lp] = qc;
      }
  }
  visit_v_items(P, blk_chunks, seg, [&](int m, int lp, int r0, int r1) {
    const int gp = P.mols_h[m].pair0 + lp;
    pair_lists[gp].push_back(int(P.items_h.size()));
    VItem it;
    it.pc = pinfo_pc[gp];
    it.qc = pinfo_qc[gp];
    it.r0 = r0;
    it.r1 = r1;
    it.pair = gp;
    it.lpair = lp;
    P.items_h.push_back(it);
  });
  std::vector<int> pair_ptr(P.n_pairs + 1, 0), pair_items;
  for (int i = 0; i < P.n_pairs; ++i) {
    pair_ptr[i + 1] = pair_ptr[i] + int(pair_lists[i].size());
    pair_items.insert(pair_items.end(), pair_lists[i].begin(), pair_lists[i].end());
  }
  P.items = dev_upload(P, P.items_h, true);
  P.pair_ptr = dev_upload(P, pair_ptr, true);
  P.pair_items = dev_upload(P, pair_items, true);

  // all segments of all molecules in block order (they partition the blocks) and their item ranges
  // (items are emitted segment by segment)
  std::vector<int64_t> seg_r0, seg_r1, seg_it0, seg_it1;
  {
    size_t it = 0;
    for (const MolDev &mo : P.mols_h)
      for (int64_t r0 = mo.blk0; r0 < mo.blk1; r0 += seg) {
        const int64_t r1 = std::min<int64_t>(mo.blk1, r0 + seg);
        seg_r0.push_back(r0);
        seg_r1.push_back(r1);
        seg_it0.push_back(int64_t(it));
        while (it < P.items_h.size() && P.items_h[it].r0 == r0) ++it;
        seg_it1.push_back(int64_t(it));
      }
    if (it != P.items_h.size()) fail(KLDI_E_ARG, "internal: Vxc items out of segment order");
  }
  const int64_t n_segs = int64_t(seg_r0.size());

  // grid chunks: whole segments whose retained tiles fit the Phi / Z workspaces
  const size_t esz = (P.opts.prec == KLDI_PREC_FP64) ? 8 : 4;
  // Phi + Z (+ bf16 low part of Phi) (+ the BF16 pieces of Phi for the X product)
  const size_t per_tile = 2 * 4096 * esz + (esz == 4 ? 4096 * 2 : 0) + size_t(4096) * 2 * bf16_pieces(P.opts.prec) +
                          (is_mgga_xc(P.opts.xc) ? size_t(2) * 4096 * 8 : 0);
  const size_t vfixed = P.items_h.size() * (16384 * 8 + 4);
  int64_t cap = chunk_tiles;
  {
    const size_t reserve = size_t(1) << 30;
    if (vfixed + reserve > fr0) fail(KLDI_E_OOM, "Vxc partials need " + std::to_string(vfixed >> 20) + " MiB");
    const int64_t fit = int64_t((fr0 - vfixed - reserve) * 0.8 / (per_tile + 4096));
    if (cap <= 0 || cap > fit) cap = fit;
    if (cap < 1) fail(KLDI_E_OOM, "no room for the Phi / Z workspaces");
  }
  for (int64_t s0 = 0; s0 < n_segs;) {
    int64_t s1 = s0 + 1;
    while (s1 < n_segs && P.blk_off_h[seg_r1[s1]] - P.blk_off_h[seg_r0[s0]] <= cap) ++s1;
    GridChunk C;
    C.blk0 = seg_r0[s0];
    C.blk1 = seg_r1[s1 - 1];
    C.ret0 = P.blk_off_h[C.blk0];
    C.ret1 = P.blk_off_h[C.blk1];
    C.xit0 = P.blk_item_off_h[C.blk0];
    C.xit1 = P.blk_item_off_h[C.blk1];
    C.vit0 = seg_it0[s0];
    C.vit1 = seg_it1[s1 - 1];
    P.chunks_h.push_back(C);
    s0 = s1;
  }
  int64_t max_ret = 1, max_xit = 1, max_vm = 1;
  for (const GridChunk &C : P.chunks_h) {
    max_ret = std::max(max_ret, C.ret1 - C.ret0);
    max_xit = std::max(max_xit, C.xit1 - C.xit0);
    max_vm = std::max(max_vm, P.vmoff_h[C.blk1] - P.vmoff_h[C.blk0]);
  }
  P.max_ret = max_ret;

  // per-XCD item orders of the schedule, per grid chunk
  const size_t nch = P.chunks_h.size();
  {
    // Vxc items of diagonal chunk pairs, per grid chunk (their diagonal tiles run in FP64)
    std::vector<int> di;
    P.dchunk_h.assign(nch + 1, 0);
    for (size_t ci = 0; ci < nch; ++ci) {
      for (int64_t it = P.chunks_h[ci].vit0; it < P.chunks_h[ci].vit1; ++it)
        if (P.items_h[it].pc == P.items_h[it].qc) di.push_back(int(it));
      P.dchunk_h[ci + 1] = int64_t(di.size());
    }
    P.ditems = dev_upload(P, di, true);
  }
  {
    std::vector<int> xorder, vorder;
    std::vector<int64_t> xqoff(9 * nch), vqoff(9 * nch);
    for (size_t ci = 0; ci < nch; ++ci) {
      const GridChunk &C = P.chunks_h[ci];
      // X: groups = blocks, cost ~ retained tiles of the block (the K extent) per item
      std::vector<int64_t> gs;
      std::vector<double> gc;
      for (int64_t r = C.blk0; r < C.blk1; ++r) {
        if (P.blk_item_off_h[r + 1] == P.blk_item_off_h[r]) continue;
        gs.push_back(P.blk_item_off_h[r]);
        const double np = double(P.blk_off_h[r + 1] - P.blk_off_h[r]);
        gc.push_back(double(P.blk_item_off_h[r + 1] - P.blk_item_off_h[r]) * (np + 4.0));
      }
      // V: cost of an item ~ candidate tile pairs over its segment
      std::vector<double> vc;
      for (int64_t it = C.vit0; it < C.vit1; ++it) {
        const VItem &v = P.items_h[it];
        double c = 1.0;
        for (int r = v.r0; r < v.r1; ++r) {
          const int *ci_r = P.cinfo_h.data() + P.cioff_h[r];
          c += double(__builtin_popcount(ci_r[v.pc] & 15) * __builtin_popcount(ci_r[v.qc] & 15));
        }
        vc.push_back(c);
      }
      if (schedule == KLDI_SCHED_GRID) {
        // grid blocks (X) and Vxc segments (V) dealt round-robin over the XCDs: the items of a block or
        // segment share its Phi / Z tiles in one L2, and every XCD gets an interleaved share of the
        // molecule (its cost varies along the molecule).  The V queues are ordered by decreasing cost:
        // the dispatcher hands workgroups to the XCDs in turn, so neighbouring workgroups of similar cost
        // keep every XCD fed (measured: Vxc stage -10% at the 200-atom chain; no effect on X).
        make_rr_queues(C.xit0, C.xit1, gs, nullptr, xorder, &xqoff[9 * ci]);
        std::vector<int64_t> vs;
        for (int64_t it = C.vit0; it < C.vit1; ++it)
          if (it == C.vit0 || P.items_h[it].r0 != P.items_h[it - 1].r0) vs.push_back(it);
        make_rr_queues(C.vit0, C.vit1, vs, &vc, vorder, &vqoff[9 * ci]);
        continue;
      }
      make_queues(C.xit0, C.xit1, gs, gc, xorder, &xqoff[9 * ci]);
      // V: one group per item
      std::vector<int64_t> vs;
      for (int64_t it = C.vit0; it < C.vit1; ++it) vs.push_back(it);
      make_queues(C.vit0, C.vit1, vs, vc, vorder, &vqoff[9 * ci]);
    }
    P.xq.maxlen_h.assign(nch, 0);
    P.vq.maxlen_h.assign(nch, 0);
    for (size_t ci = 0; ci < nch; ++ci)
      for (int x = 0; x < 8; ++x) {
        P.xq.maxlen_h[ci] = std::max(P.xq.maxlen_h[ci], xqoff[9 * ci + x + 1] - xqoff[9 * ci + x]);
        P.vq.maxlen_h[ci] = std::max(P.vq.maxlen_h[ci], vqoff[9 * ci + x + 1] - vqoff[9 * ci + x]);
      }
    P.xq.order = dev_upload(P, xorder, true);
    P.xq.qoff = dev_upload(P, xqoff, true);
    P.vq.order = dev_upload(P, vorder, true);
    P.vq.qoff = dev_upload(P, vqoff, true);
  }

  EvalDev &E = P.ev;
  if (esz == 8) {
    E.phi = dev_alloc<double>(P, size_t(max_ret) * 4096, true);
    E.zws = dev_alloc<double>(P, size_t(max_ret) * 4096, true);
    E.phil = nullptr;
  } else {
    E.phi = dev_alloc<float>(P, size_t(max_ret) * 4096, true);
    E.zws = dev_alloc<float>(P, size_t(max_ret) * 4096, true);
    E.phil = dev_alloc<unsigned short>(P, size_t(max_ret) * 4096, true);
  }
  const int npc = bf16_pieces(P.opts.prec);
  E.phix = npc ? dev_alloc<unsigned short>(P, size_t(max_ret) * 4096 * npc, true) : nullptr;
  E.xpart = dev_alloc<double>(P, size_t(max_xit) * 4 * kG, true);
  if (is_mgga_xc(P.opts.xc)) {
    E.tdphi = dev_alloc<double>(P, size_t(max_ret) * 4096, true);
    E.tB = dev_alloc<double>(P, size_t(max_ret) * 4096, true);
    for (int a = 0; a < 3; ++a) E.tpart[a] = dev_alloc<double>(P, size_t(max_xit) * 4 * kG, true);
  } else {
    E.tdphi = E.tB = nullptr;
    E.tpart[0] = E.tpart[1] = E.tpart[2] = nullptr;
  }
  E.vpart = dev_alloc<double>(P, P.items_h.size() * 16384, true);
  E.vflag = dev_alloc<int>(P, P.items_h.size(), true);
  E.vmask = dev_alloc<unsigned short>(P, size_t(max_vm), true);
}

// ------------------------------------------------------------------------------------------------
// The plan over n_mol molecules
// ------------------------------------------------------------------------------------------------
void build_plan(Plan &P, int n_mol, const kldi_basis *bs, const kldi_grid *gs, const kldi_opts *o,
                hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  check_hip(hipGetDevice(&P.device), "hipGetDevice");
  P.opts = *o;
  P.gga = (o->xc != KLDI_XC_LDA_X);
  P.n_mol = n_mol;

  // per-molecule preparation on host threads
  std::vector<MolPrep> mp(n_mol);
  {
    std::atomic<int> next{0};
    std::vector<std::string> errs(n_mol);
    std::vector<kldi_status> codes(n_mol, KLDI_OK);
    const int nth = std::max(1, std::min<int>(n_mol, int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())))));
    auto work = [&] {
      for (int m = next++; m < n_mol; m = next++) {
        try {
          prepare_mol(mp[m], &bs[m], &gs[m], P.gga, o->t_b, o->shell_order, o->grid_block == 2 * kG);
        } catch (const Error &e) {
          codes[m] = e.code;
          errs[m] = e.msg;
        } catch (const std::bad_alloc &) {
          codes[m] = KLDI_E_OOM;
          errs[m] = "host allocation failed";
        }
      }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    for (int m = 0; m < n_mol; ++m)
      if (codes[m] != KLDI_OK) fail(codes[m], "molecule " + std::to_string(m) + ": " + errs[m]);
  }

  // one index space: offsets of every molecule
  std::vector<int> shell0(n_mol), prim0(n_mol);
  P.mols_h.resize(n_mol);
  int ns = 0, npr = 0, nt = 0, npairs = 0;
  int64_t nblk = 0, row = 0, dt = 0, d0 = 0, mf = 0, pt0 = 0;
  for (int m = 0; m < n_mol; ++m) {
    const MolPrep &M = mp[m];
    MolDev &mo = P.mols_h[m];
    shell0[m] = ns;
    prim0[m] = npr;
    mo.tile0 = nt;
    mo.nt = M.n_tiles;
    mo.nc = (M.n_tiles + kChunk - 1) / kChunk;
    mo.pair0 = npairs;
    mo.npairs = P.gga ? mo.nc * mo.nc : mo.nc * (mo.nc + 1) / 2;
    mo.n_ao = M.n_ao;
    mo.ld = mo.nc * 128;
    mo.pad_ = 0;
    mo.row0 = row;
    mo.dt0 = dt;
    mo.d0 = d0;
    mo.blk0 = nblk;
    mo.blk1 = nblk + M.n_blocks;
    mo.mf0 = mf;
    ns += M.n_shells;
    npr += int(M.pexp.size());
    nt += M.n_tiles;
    npairs += mo.npairs;
    nblk += M.n_blocks;
    row += M.n_ao;
    dt += int64_t(M.n_tiles) * M.n_tiles;
    d0 += int64_t(M.n_ao) * M.n_ao;
    mf += int64_t(mo.ld) * mo.ld;
    pt0 += M.n_points;
    P.max_nao = std::max(P.max_nao, M.n_ao);
  }
  if (int64_t(nt) * kD > (int64_t(1) << 30)) fail(KLDI_E_UNSUPPORTED, "too many AOs in one plan");
  P.n_shells = ns;
  P.n_tiles = nt;
  P.n_ao = int(row);
  P.n_pairs = npairs;
  P.n_blocks = nblk;
  P.n_pad = nblk * kG;
  P.n_points = pt0;
  P.n_dt = dt;
  P.n_mfull = mf;
  if (n_mol == 1) P.pt_perm = mp[0].pt_perm;
  P.pt_off_h.assign(n_mol + 1, 0);
  for (int m = 0; m < n_mol; ++m) P.pt_off_h[m + 1] = P.pt_off_h[m] + mp[m].n_points;

  // concatenated host arrays
  std::vector<double> sh_xyz, pexp, pcoef, px, py, pz, pw;
  std::vector<int> sh_prim, sh_l, sh_ao0, ao_shell, ao_comp, tile_sh, tile_nv, cand_p;
  std::vector<int64_t> porig, cand_r;
  std::vector<int32_t> blk_mol(nblk);
  P.ao_perm.assign(size_t(nt) * kD, 0);
  {
    int64_t ptoff = 0;
    for (int m = 0; m < n_mol; ++m) {
      const MolPrep &M = mp[m];
      const MolDev &mo = P.mols_h[m];
      const int s0 = shell0[m], q0 = prim0[m], a0 = mo.tile0 * kD;
      append(sh_xyz, M.sh_xyz, [](double v) { return v; });
      for (size_t k = 0; k < M.sh_prim.size(); ++k) sh_prim.push_back(M.sh_prim[k] + q0);
      append(sh_l, M.sh_l, [](int v) { return v; });
      append(sh_ao0, M.sh_ao0, [&](int v) { return v + a0; });
      append(pexp, M.pexp, [](double v) { return v; });
      append(pcoef, M.pcoef, [](double v) { return v; });
      append(ao_shell, M.ao_shell, [&](int v) { return v < 0 ? -1 : v + s0; });
      append(ao_comp, M.ao_comp, [](int v) { return v; });
      append(tile_sh, M.tile_sh, [&](int v) { return v + s0; });
      append(tile_nv, M.tile_nv, [](int v) { return v; });
      append(px, M.px, [](double v) { return v; });
      append(py, M.py, [](double v) { return v; });
      append(pz, M.pz, [](double v) { return v; });
      append(pw, M.pw, [](double v) { return v; });
      append(porig, M.porig, [&](int64_t v) { return v < 0 ? int64_t(-1) : v + ptoff; });
      append(cand_p, M.cand_p, [&](int v) { return v + mo.tile0; });
      append(cand_r, M.cand_r, [&](int64_t v) { return v + mo.blk0; });
      for (int i = 0; i < M.n_ao; ++i) P.ao_perm[size_t(a0) + i] = M.ao_perm[i];
      for (int64_t r = mo.blk0; r < mo.blk1; ++r) blk_mol[r] = m;
      ptoff += M.n_points;
    }
  }
  std::vector<int> ao_atom0 = mp[0].ao_atom;   // kept for the gradient (first molecule)
  mp.clear();
  mp.shrink_to_fit();
  P.n_cand = int64_t(cand_p.size());
  P.blk_mol_h = blk_mol;

  // device copies of basis, grid and molecule table
  BasisDev &B = P.basis;
  B.sh_xyz = dev_upload(P, sh_xyz);
  B.sh_prim = dev_upload(P, sh_prim);
  B.sh_l = dev_upload(P, sh_l);
  B.sh_ao0 = dev_upload(P, sh_ao0);
  B.pexp = dev_upload(P, pexp);
  B.pcoef = dev_upload(P, pcoef);
  B.ao_shell = dev_upload(P, ao_shell);
  B.ao_comp = dev_upload(P, ao_comp);
  B.tile_sh = dev_upload(P, tile_sh);
  B.tile_nv = dev_upload(P, tile_nv);
  {
    const size_t ns = sh_l.size();
    std::vector<double> rec(ns * kShRec, 0.0);
    for (size_t s = 0; s < ns; ++s) {
      double *r = rec.data() + s * kShRec;
      r[0] = sh_xyz[3 * s];
      r[1] = sh_xyz[3 * s + 1];
      r[2] = sh_xyz[3 * s + 2];
      const int p0 = sh_prim[2 * s], np = sh_prim[2 * s + 1] - p0;
      const int32_t w[4] = {sh_ao0[s], sh_l[s] | (np << 2), p0, 0};
      std::memcpy(r + 3, w, sizeof(w));
      for (int k = 0; k < std::min(np, kShPrimIn); ++k) {
        r[5 + 2 * k] = pexp[size_t(p0 + k)];
        r[6 + 2 * k] = pcoef[size_t(p0 + k)];
      }
    }
    B.shrec = dev_upload(P, rec);
  }
  GridDev &Gd = P.grid;
  Gd.x = dev_upload(P, px);
  Gd.y = dev_upload(P, py);
  Gd.z = dev_upload(P, pz);
  Gd.w = dev_upload(P, pw);
  Gd.orig = dev_upload(P, porig);
  Gd.n_blocks = P.n_blocks;
  px = py = pz = pw = std::vector<double>();

  // exact block maxima on the device (eq. block_summary_A), retention (eq. block_filter_A)
  std::vector<double> cb(P.n_cand), cg(P.n_cand);
  if (P.n_cand > 0) {
    int *dcp = dev_upload(P, cand_p);
    int64_t *dcr = dev_upload(P, cand_r);
    double *db = dev_alloc<double>(P, P.n_cand), *dg = dev_alloc<double>(P, P.n_cand);
    check_hip(launch_screen(B, Gd, dcp, dcr, P.n_cand, P.gga, db, dg, stream), "screen launch");
    check_hip(hipMemcpyAsync(cb.data(), db, sizeof(double) * P.n_cand, hipMemcpyDeviceToHost, stream), "copy");
    check_hip(hipMemcpyAsync(cg.data(), dg, sizeof(double) * P.n_cand, hipMemcpyDeviceToHost, stream), "copy");
    check_hip(hipStreamSynchronize(stream), "screen sync");
    // the candidate buffers are no longer needed
    for (void *ptr : {(void *)dcp, (void *)dcr, (void *)db, (void *)dg}) {
      auto it = std::find(P.allocs.begin(), P.allocs.end(), ptr);
      if (it != P.allocs.end()) {
        (void)hipFree(*it);
        P.allocs.erase(it);
      }
    }
  }
  if (o->grid_block == 2 * kG && P.n_cand > 0) {
    // 256-point blocks: the summaries of a tile over a pair of compute blocks (molecule-local 2k, 2k + 1)
    // are the maxima over both, so both halves retain the same tiles with the same b_pr
    std::vector<int64_t> coff(P.n_blocks + 1, 0);
    for (int64_t c = 0; c < P.n_cand; ++c) coff[cand_r[c] + 1]++;
    for (int64_t r = 0; r < P.n_blocks; ++r) coff[r + 1] += coff[r];
    for (const MolDev &mo : P.mols_h)
      for (int64_t r = mo.blk0; r + 1 < mo.blk1; r += 2) {
        const int64_t n = coff[r + 1] - coff[r];
        if (coff[r + 2] - coff[r + 1] != n) fail(KLDI_E_ARG, "internal: paired blocks with different candidates");
        for (int64_t k = 0; k < n; ++k) {
          const int64_t c0 = coff[r] + k, c1 = coff[r + 1] + k;
          cb[c0] = cb[c1] = std::max(cb[c0], cb[c1]);
          cg[c0] = cg[c1] = std::max(cg[c0], cg[c1]);
        }
      }
  }
  P.blk_off_h.assign(P.n_blocks + 1, 0);
  std::vector<int> ret_r;
  for (int64_t c = 0; c < P.n_cand; ++c) {
    double s = P.gga ? std::max(cb[c], cg[c]) : cb[c];
    if (s >= o->t_b) {
      int64_t r = cand_r[c];
      P.blk_off_h[r + 1]++;
      P.ret_p_h.push_back(cand_p[c]);
      ret_r.push_back(int(r));
      P.bphi_h.push_back(cb[c]);
    }
  }
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    P.max_np = std::max<int>(P.max_np, int(P.blk_off_h[r + 1]));
    P.blk_off_h[r + 1] += P.blk_off_h[r];
  }
  P.n_ret = P.blk_off_h[P.n_blocks];
  if (P.max_np > kMaxTilesPerBlock) fail(KLDI_E_UNSUPPORTED, "more than 512 retained tiles in one grid block");
  StructDev &S = P.st;
  S.blk_off = dev_upload(P, P.blk_off_h);
  S.ret_p = dev_upload(P, P.ret_p_h);
  S.ret_r = dev_upload(P, ret_r);
  S.bphi = dev_upload(P, P.bphi_h);
  S.blk_mol = dev_upload(P, blk_mol);
  S.mol = dev_upload(P, P.mols_h);
  S.n_mol = n_mol;

  // per (block, chunk of its molecule): position in S_r of the chunk's first retained tile and its
  // 4-bit mask; per block: first cinfo entry and first Vxc-mask entry; the chunk-pair table
  P.cioff_h.assign(P.n_blocks + 1, 0);
  P.vmoff_h.assign(P.n_blocks + 1, 0);
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    const MolDev &mo = P.mols_h[blk_mol[r]];
    P.cioff_h[r + 1] = P.cioff_h[r] + mo.nc;
    P.vmoff_h[r + 1] = P.vmoff_h[r] + mo.npairs;
  }
  P.cinfo_h.assign(size_t(P.cioff_h[P.n_blocks]), 0);
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    const int tile0 = P.mols_h[blk_mol[r]].tile0;
    for (int64_t k = P.blk_off_h[r + 1] - 1; k >= P.blk_off_h[r]; --k) {
      const int p = P.ret_p_h[k] - tile0, c = p / kChunk;
      int &ci = P.cinfo_h[size_t(P.cioff_h[r]) + c];
      ci = (int(k - P.blk_off_h[r]) << 4) | (ci & 15) | (1 << (p % kChunk));
    }
  }
  P.cinfo = dev_upload(P, P.cinfo_h);
  P.cioff = dev_upload(P, P.cioff_h);
  P.vmoff = dev_upload(P, P.vmoff_h);
  {
    std::vector<int> pinfo(3 * size_t(P.n_pairs));
    for (int m = 0; m < n_mol; ++m) {
      const MolDev &mo = P.mols_h[m];
      for (int pc = 0; pc < mo.nc; ++pc)
        for (int qc = P.gga ? 0 : pc; qc < mo.nc; ++qc) {
          const int lp = P.gga ? pc * mo.nc + qc : pc * mo.nc - pc * (pc - 1) / 2 + (qc - pc);
          const size_t g = size_t(mo.pair0 + lp);
          pinfo[3 * g] = pc;
          pinfo[3 * g + 1] = qc;
          pinfo[3 * g + 2] = m;
        }
    }
    P.pair_info = dev_upload(P, pinfo);
  }
  P.ao_perm_d = dev_upload(P, P.ao_perm);
  P.ao_atom = dev_upload(P, ao_atom0);
  P.n_atoms0 = bs[0].n_atoms;

  // fixed workspaces
  const size_t esz = (o->prec == KLDI_PREC_FP64) ? 8 : 4;
  EvalDev &E = P.ev;
  const int npc = bf16_pieces(o->prec);
  if (esz == 8)
    E.Dt = dev_alloc<double>(P, size_t(P.n_dt) * 1024);
  else if (npc)
    E.Dt = dev_alloc<unsigned short>(P, size_t(P.n_dt) * 1024 * npc);
  else
    E.Dt = dev_alloc<float>(P, size_t(P.n_dt) * 1024);
  E.amax = dev_alloc<double>(P, size_t(P.n_dt));
  E.zmax = dev_alloc<double>(P, P.n_ret);
  E.coef = dev_alloc<double>(P, size_t(P.n_pad) * 4);
  E.eblk = dev_alloc<double>(P, P.n_blocks);
  E.mfull = dev_alloc<double>(P, size_t(P.n_mfull));
  E.counters = dev_alloc<unsigned long long>(P, 8);
  E.ctau = is_mgga_xc(o->xc) ? dev_alloc<double>(P, size_t(P.n_pad)) : nullptr;
  E.escratch = dev_alloc<double>(P, n_mol);
  E.io = dev_alloc<IoDev>(P, 1);
  check_hip(hipMemsetAsync(E.counters, 0, 4 * sizeof(unsigned long long), stream), "memset");
  check_hip(hipStreamSynchronize(stream), "plan sync");

  build_schedule(P, o->v_segment, o->schedule, o->chunk_tiles);
  check_hip(hipStreamCreateWithFlags(&P.side_stream, hipStreamNonBlocking), "hipStreamCreate");
  check_hip(hipEventCreateWithFlags(&P.fork_ev, hipEventDisableTiming), "hipEventCreate");
  check_hip(hipEventCreateWithFlags(&P.join_ev, hipEventDisableTiming), "hipEventCreate");
  P.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------------------------------------
// One evaluation: k_begin, then the body launch by launch or as a captured graph
// ------------------------------------------------------------------------------------------------
void run_eval(Plan &P, const IoDev &io, bool want_v, hipStream_t s, hipEvent_t *ev) {
  check_hip(launch_begin(P, io, s), "begin launch");
  if (!P.use_graph) {
    check_hip(launch_body(P, want_v, s, ev), "eval launch");
    return;
  }
  hipGraphExec_t &gx = P.graph[want_v ? 1 : 0];
  if (!gx) {
    if (!P.cap_stream) check_hip(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    hipGraph_t g = nullptr;
    check_hip(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const hipError_t le = launch_body(P, want_v, P.cap_stream, nullptr);
    const hipError_t ce = hipStreamEndCapture(P.cap_stream, &g);
    check_hip(le, "launch during capture");
    check_hip(ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check_hip(ie, "hipGraphInstantiate");
  }
  check_hip(hipGraphLaunch(gx, s), "hipGraphLaunch");
}

hipEvent_t *timing_slot(Plan &P) {
  if (!P.timing || P.use_graph) return nullptr;
  hipEvent_t *ev = &P.events[size_t(P.n_timed % kTimingSlots) * (KLDI_N_STAGES + 1)];
  P.n_timed++;
  return ev;
}

// ------------------------------------------------------------------------------------------------
// Autotuner cache: plan shape -> (v_segment, schedule)
// ------------------------------------------------------------------------------------------------
typedef std::tuple<int, int64_t, int64_t, int64_t, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;

TuneKey tune_key(const Plan &P) {
  return TuneKey(P.n_mol, int64_t(P.n_ao), P.n_blocks, P.n_ret, P.opts.xc, P.opts.prec);
}

template <class F>
kldi_status guarded(F &&f) {
  try {
    f();
    return KLDI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return KLDI_E_OOM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return KLDI_E_ARG;
  } catch (...) {
    set_error("unknown error");
    return KLDI_E_ARG;
  }
}

kldi_status create(int32_t n_mol, const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts,
                   void *stream, kldi_plan **out) {
  set_error("");
  if (!out) {
    set_error("out must not be NULL");
    return KLDI_E_ARG;
  }
  *out = nullptr;
  kldi_plan *plan = nullptr;
  kldi_status st = guarded([&] {
    if (n_mol < 1) fail(KLDI_E_ARG, "n_mol must be >= 1");
    if (!basis || !grid || !opts) fail(KLDI_E_ARG, "basis, grid and opts must not be NULL");
    validate_opts(opts);
    for (int m = 0; m < n_mol; ++m) {
      try {
        validate(&basis[m], &grid[m]);
      } catch (const Error &e) {
        fail(e.code, n_mol > 1 ? "molecule " + std::to_string(m) + ": " + e.msg : e.msg);
      }
    }
    plan = new kldi_plan();
    build_plan(plan->impl, n_mol, basis, grid, opts, static_cast<hipStream_t>(stream));
  });
  if (st != KLDI_OK) {
    if (plan) {
      free_plan(plan->impl);
      delete plan;
    }
    return st;
  }
  *out = plan;
  return KLDI_OK;
}

}  // namespace

void invalidate_graphs(Plan &P) { free_graphs(P); }

}  // namespace kldi

using kldi::Plan;

extern "C" {

void kldi_opts_default(kldi_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->t_b = 1e-10;
  o->t_d = 1e-10;
  o->rho_cut = 1e-14;
  o->grid_block = kldi::kG;
  o->ao_block = kldi::kD;
  o->prec = KLDI_PREC_FP64;
  o->xc = KLDI_XC_LDA_X;
  o->v_segment = 0;
  o->chunk_tiles = 0;
  o->schedule = KLDI_SCHED_GRID;
  o->shell_order = nullptr;
}

kldi_status kldi_plan_create(const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts, void *stream,
                             kldi_plan **out) {
  return kldi::create(1, basis, grid, opts, stream, out);
}

kldi_status kldi_batch_create(int32_t n_mol, const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts,
                              void *stream, kldi_plan **out) {
  if (opts && opts->shell_order && n_mol != 1) {
    kldi::set_error("shell_order applies to single-molecule plans");
    return KLDI_E_UNSUPPORTED;
  }
  return kldi::create(n_mol, basis, grid, opts, stream, out);
}

kldi_status kldi_batch_layout(const kldi_plan *plan, int64_t *ao_off, int64_t *d_off, int64_t *pt_off) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  const Plan &P = plan->impl;
  for (int m = 0; m <= P.n_mol; ++m) {
    if (ao_off) ao_off[m] = (m < P.n_mol) ? P.mols_h[m].row0 : int64_t(P.n_ao);
    if (d_off) {
      const kldi::MolDev &last = P.mols_h.back();
      d_off[m] = (m < P.n_mol) ? P.mols_h[m].d0 : last.d0 + int64_t(last.n_ao) * last.n_ao;
    }
    if (pt_off) pt_off[m] = P.pt_off_h[m];
  }
  return KLDI_OK;
}

kldi_status kldi_plan_destroy(kldi_plan *plan) {
  if (!plan) return KLDI_OK;
  (void)hipSetDevice(plan->impl.device);
  (void)hipDeviceSynchronize();
  kldi::free_plan(plan->impl);
  delete plan;
  return KLDI_OK;
}

kldi_status kldi_plan_info(const kldi_plan *plan, kldi_plan_info_t *out) {
  if (!plan || !out) {
    kldi::set_error("plan and out must not be NULL");
    return KLDI_E_ARG;
  }
  const Plan &P = plan->impl;
  std::memset(out, 0, sizeof(*out));
  out->n_ao = P.n_ao;
  out->n_tiles = P.n_tiles;
  out->n_points = P.n_points;
  out->n_blocks = P.n_blocks;
  out->n_candidate_tiles = P.n_cand;
  out->n_retained_tiles = P.n_ret;
  double all = 0.0;
  for (const kldi::MolDev &mo : P.mols_h) all += double(mo.nt) * double(mo.blk1 - mo.blk0);
  out->retained_fraction = double(P.n_ret) / all;
  out->max_tiles_per_block = P.max_np;
  out->v_segment = P.v_segment;
  out->n_v_items = int64_t(P.items_h.size());
  out->workspace_bytes = int64_t(P.bytes + P.sched_bytes);
  out->n_grid_chunks = int32_t(P.chunks_h.size());
  out->plan_ms = P.plan_ms;
  out->n_mol = P.n_mol;
  out->schedule = P.schedule;
  out->graph = P.use_graph ? 1 : 0;
  out->n_x_items = P.n_xitems;
  return KLDI_OK;
}

kldi_status kldi_plan_structure(const kldi_plan *plan, int32_t *ao_perm, int64_t *pt_perm, uint8_t *retained,
                                double *phi_max) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  const Plan &P = plan->impl;
  if (P.n_mol != 1) {
    kldi::set_error("kldi_plan_structure covers single-molecule plans");
    return KLDI_E_UNSUPPORTED;
  }
  if (ao_perm) std::copy(P.ao_perm.begin(), P.ao_perm.begin() + P.n_ao, ao_perm);
  if (pt_perm) std::copy(P.pt_perm.begin(), P.pt_perm.end(), pt_perm);
  size_t n = size_t(P.n_tiles) * size_t(P.n_blocks);
  if (retained) std::memset(retained, 0, n);
  if (phi_max) std::fill(phi_max, phi_max + n, 0.0);
  for (int64_t r = 0; r < P.n_blocks; ++r)
    for (int64_t k = P.blk_off_h[r]; k < P.blk_off_h[r + 1]; ++k) {
      size_t at = size_t(r) * P.n_tiles + P.ret_p_h[k];
      if (retained) retained[at] = 1;
      if (phi_max) phi_max[at] = P.bphi_h[k];
    }
  return KLDI_OK;
}

kldi_status kldi_eval(kldi_plan *plan, const double *D_dev, double *rho_dev, double *exc_dev, double *vxc_dev,
                      void *stream) {
  if (!plan || !D_dev || !exc_dev) {
    kldi::set_error("plan, D and exc must not be NULL");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    kldi::IoDev io{D_dev, rho_dev, nullptr, exc_dev, vxc_dev};
    kldi::run_eval(P, io, vxc_dev != nullptr, static_cast<hipStream_t>(stream), kldi::timing_slot(P));
  });
}

kldi_status kldi_eval_grad(kldi_plan *plan, const double *D_dev, double *grad_dev, double *exc_dev, void *stream) {
  if (!plan || !D_dev || !grad_dev) {
    kldi::set_error("plan, D and grad must not be NULL");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    if (P.n_mol != 1) kldi::fail(KLDI_E_UNSUPPORTED, "the nuclear gradient is for single-molecule plans");
    if (P.opts.prec != KLDI_PREC_FP64 && P.opts.prec != KLDI_PREC_FP32)
      kldi::fail(KLDI_E_UNSUPPORTED, "the nuclear gradient runs on FP64 and FP32 plans");
    if (P.has_mlp) kldi::fail(KLDI_E_UNSUPPORTED, "the nuclear gradient needs the analytic functional");
    if (kldi::is_mgga_xc(P.opts.xc)) kldi::fail(KLDI_E_UNSUPPORTED, "the nuclear gradient covers LDA and GGA functionals");
    if (P.opts.grid_block != kldi::kG) kldi::fail(KLDI_E_UNSUPPORTED, "the nuclear gradient runs on 128-point blocks");
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    if (!P.grad_ws.gA) {
      P.grad_ws.gA = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.max_ret, 1)) * 4096, true);
      P.grad_ws.gAmax = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.max_ret, 1)), true);
      P.grad_ws.gWmax = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.max_ret, 1)), true);
      P.grad_ws.gitem = kldi::dev_alloc<double>(P, std::max<size_t>(P.items_h.size(), 1) * 6 * 128, true);
      P.grad_ws.gao = kldi::dev_alloc<double>(P, size_t(3) * P.mols_h[0].nc * 128, true);
      P.grad_ws.gpart = kldi::dev_alloc<double>(P, size_t(P.mols_h[0].nc) * kldi::kGSeg * 3 * 128, true);
    }
    if (P.gga && !P.grad_ws.gQ) {
      P.grad_ws.gQ = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.max_ret, 1)) * 4096, true);
      P.grad_ws.gQmax = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.max_ret, 1)), true);
    }
    if (P.opts.prec != KLDI_PREC_FP64 && !P.grad_ws.gD)
      P.grad_ws.gD = kldi::dev_alloc<double>(P, size_t(std::max<int64_t>(P.n_dt, 1)) * 1024, true);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    kldi::IoDev io{D_dev, nullptr, nullptr, exc_dev ? exc_dev : P.ev.escratch, nullptr};
    kldi::check_hip(kldi::launch_begin(P, io, s), "begin launch");
    kldi::check_hip(kldi::launch_grad(P, grad_dev, s), "gradient launch");
  });
}

kldi_status kldi_eval_check(kldi_plan *plan, kldi_eval_stats_t *out, void *stream) {
  if (!plan || !out) {
    kldi::set_error("plan and out must not be NULL");
    return KLDI_E_ARG;
  }
  unsigned long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  kldi_status st = kldi::guarded([&] {
    kldi::check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "sync");
    kldi::check_hip(hipMemcpy(c, plan->impl.ev.counters, sizeof(c), hipMemcpyDeviceToHost), "copy counters");
  });
  if (st != KLDI_OK) return st;
  out->n_pairs_x = int64_t(c[0]);
  out->n_pairs_v = int64_t(c[1]);
  out->gemm_flops = 2.0 * kldi::kD * kldi::kD * kldi::kG * double(c[0] + c[1]);
  out->n_points_mlp = int64_t(c[3]);
  out->n_pairs_v_diag = int64_t(c[6]);
  out->nonfinite_d = c[2] ? 1 : 0;
  if (c[2]) {
    kldi::set_error("D holds a non-finite entry");
    return KLDI_E_NONFINITE;
  }
  return KLDI_OK;
}

kldi_status kldi_plan_timing(kldi_plan *plan, int32_t enable) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    if (enable && P.events.empty()) {
      P.events.resize(size_t(kldi::kTimingSlots) * (KLDI_N_STAGES + 1));
      for (auto &e : P.events) kldi::check_hip(hipEventCreate(&e), "hipEventCreate");
    }
    P.timing = enable != 0;
    P.n_timed = 0;
  });
}

kldi_status kldi_eval_timing(kldi_plan *plan, double *stage_ms, int32_t *n_evals) {
  if (!plan || !stage_ms) {
    kldi::set_error("plan and stage_ms must not be NULL");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    for (int s = 0; s < KLDI_N_STAGES; ++s) stage_ms[s] = 0.0;
    const int n = std::min(P.n_timed, kldi::kTimingSlots);
    if (n_evals) *n_evals = n;
    if (n == 0) return;
    for (int i = 0; i < n; ++i) {
      hipEvent_t *ev = &P.events[size_t(i) * (KLDI_N_STAGES + 1)];
      kldi::check_hip(hipEventSynchronize(ev[KLDI_N_STAGES]), "hipEventSynchronize");
      for (int s = 0; s < KLDI_N_STAGES; ++s) {
        float ms = 0.f;
        kldi::check_hip(hipEventElapsedTime(&ms, ev[s], ev[s + 1]), "hipEventElapsedTime");
        stage_ms[s] += ms;
      }
    }
    for (int s = 0; s < KLDI_N_STAGES; ++s) stage_ms[s] /= n;
  });
}

kldi_status kldi_eval_grid(kldi_plan *plan, const double *D_dev, double *rho_dev, double *sigma_dev, void *stream) {
  if (!plan || !D_dev || (!rho_dev && !sigma_dev)) {
    kldi::set_error("plan and D must not be NULL; one of rho, sigma must be given");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    // E_xc of this call goes to the plan's scratch
    kldi::IoDev io{D_dev, rho_dev, sigma_dev, P.ev.escratch, nullptr};
    kldi::run_eval(P, io, false, static_cast<hipStream_t>(stream), nullptr);
  });
}

kldi_status kldi_plan_graph(kldi_plan *plan, int32_t enable) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  Plan &P = plan->impl;
  P.use_graph = enable != 0;
  if (!P.use_graph) kldi::invalidate_graphs(P);
  return KLDI_OK;
}

kldi_status kldi_plan_autotune(kldi_plan *plan, const double *D_dev, int32_t reps, void *stream, kldi_tune_t *out) {
  if (!plan || !D_dev || reps < 0) {
    kldi::set_error("plan and D must not be NULL; reps >= 0");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    Plan &P = plan->impl;
    hipStream_t s = static_cast<hipStream_t>(stream);
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    kldi::check_hip(hipStreamSynchronize(s), "sync");
    const kldi::TuneKey key = kldi::tune_key(P);
    kldi_tune_t res{P.v_segment, P.schedule, 0.0, 0};
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(kldi::g_tune_mu);
      auto it = kldi::g_tune_cache.find(key);
      if (it != kldi::g_tune_cache.end()) {
        cached = true;
        res.v_segment = it->second.first;
        res.schedule = it->second.second;
      }
    }
    kldi::invalidate_graphs(P);
    if (cached || reps == 0) {
      if (cached && (res.v_segment != P.v_segment || res.schedule != P.schedule))
        kldi::build_schedule(P, res.v_segment, res.schedule, P.opts.chunk_tiles);
      if (out) *out = res;
      return;
    }
    // candidates: Vxc tile depths whose partials fit, each with both schedules
    const auto bc = kldi::block_chunks(P);
    size_t fr = 0, tot = 0;
    kldi::check_hip(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    const size_t budget = (fr + P.sched_bytes) / 3;
    kldi::IoDev io{D_dev, nullptr, nullptr, P.ev.escratch, nullptr};
    std::vector<double> vbuf;
    double *vtmp = nullptr;
    kldi::check_hip(hipMalloc(&vtmp, sizeof(double) * std::max<size_t>(1, size_t(P.mols_h.back().d0) +
                                                                            size_t(P.mols_h.back().n_ao) * P.mols_h.back().n_ao)),
                    "hipMalloc");
    io.vxc = vtmp;
    hipEvent_t e0, e1;
    kldi::check_hip(hipEventCreate(&e0), "hipEventCreate");
    kldi::check_hip(hipEventCreate(&e1), "hipEventCreate");
    double best = 1e300;
    int best_seg = P.v_segment, best_sched = P.schedule, tried = 0;
    const bool was_graph = P.use_graph;
    P.use_graph = false;
    try {
      for (int seg : {8, 16, 32, 64}) {
        if (size_t(kldi::count_v_items(P, bc, seg)) * 16384 * 8 > budget) continue;
        for (int sched : {int(KLDI_SCHED_GRID), int(KLDI_SCHED_QUEUE)}) {
          if (sched == KLDI_SCHED_QUEUE && P.n_blocks > kldi::kQueueMaxBlocks) continue;
          try {
            kldi::build_schedule(P, seg, sched, P.opts.chunk_tiles);
          } catch (const kldi::Error &e) {
            if (e.code == KLDI_E_OOM) continue;
            throw;
          }
          kldi::run_eval(P, io, true, s, nullptr);   // warm-up
          kldi::check_hip(hipEventRecord(e0, s), "hipEventRecord");
          for (int k = 0; k < reps; ++k) kldi::run_eval(P, io, true, s, nullptr);
          kldi::check_hip(hipEventRecord(e1, s), "hipEventRecord");
          kldi::check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
          float ms = 0.f;
          kldi::check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
          ++tried;
          if (ms / reps < best) {
            best = ms / reps;
            best_seg = seg;
            best_sched = sched;
          }
        }
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      (void)hipFree(vtmp);
      P.use_graph = was_graph;
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(vtmp);
    P.use_graph = was_graph;
    kldi::build_schedule(P, best_seg, best_sched, P.opts.chunk_tiles);
    {
      std::lock_guard<std::mutex> lk(kldi::g_tune_mu);
      kldi::g_tune_cache[key] = std::make_pair(best_seg, best_sched);
    }
    res.v_segment = best_seg;
    res.schedule = best_sched;
    res.ms = best;
    res.n_tried = tried;
    if (out) *out = res;
  });
}

kldi_status kldi_xc_eval(int32_t xc, const double *rho_dev, const double *sigma_dev, int64_t n, double rho_cut,
                         double *f_dev, double *vrho_dev, double *vsigma_dev, void *stream) {
  if (n < 0 || !rho_dev || !f_dev || !vrho_dev || (xc != KLDI_XC_LDA_X && (!sigma_dev || !vsigma_dev)) ||
      (xc != KLDI_XC_LDA_X && xc != KLDI_XC_PBE && xc != KLDI_XC_PBE_X) || !(rho_cut >= 0)) {
    kldi::set_error("bad arguments to kldi_xc_eval");
    return KLDI_E_ARG;
  }
  return kldi::guarded([&] {
    kldi::check_hip(kldi::launch_xc_arrays(xc, rho_dev, xc == KLDI_XC_LDA_X ? nullptr : sigma_dev, n, rho_cut, f_dev,
                                           vrho_dev, xc == KLDI_XC_LDA_X ? nullptr : vsigma_dev,
                                           static_cast<hipStream_t>(stream)),
                    "xc launch");
  });
}

const char *kldi_last_error(void) { return kldi::g_last_error.c_str(); }

int32_t kldi_version(void) { return 4; }

}  // extern "C"
