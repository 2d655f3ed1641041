// Host side of libkldi: the C ABI, argument validation and the per-geometry plan
// (reordering, tiling, shell radii, screening, retained-block lists, work lists, workspaces).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <numeric>
#include <stdexcept>

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
T *dev_alloc(Plan &P, size_t n) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(KLDI_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  P.allocs.push_back(p);
  P.bytes += bytes;
  return static_cast<T *>(p);
}

template <class T>
T *dev_upload(Plan &P, const std::vector<T> &h) {
  T *d = dev_alloc<T>(P, h.size());
  if (!h.empty()) check_hip(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
  return d;
}

void free_plan(Plan &P) {
  for (void *p : P.allocs) (void)hipFree(p);
  P.allocs.clear();
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

void validate(const kldi_basis *b, const kldi_grid *g, const kldi_opts *o) {
  if (!b || !g || !o) fail(KLDI_E_ARG, "basis, grid and opts must not be NULL");
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
  if (!(o->t_b >= 0) || !(o->t_d >= 0) || !(o->rho_cut >= 0) || !std::isfinite(o->t_b) ||
      !std::isfinite(o->t_d) || !std::isfinite(o->rho_cut))
    fail(KLDI_E_ARG, "t_b, t_d and rho_cut must be finite and >= 0");
  if (o->grid_block <= 0 || o->grid_block % 64 != 0) fail(KLDI_E_ARG, "grid_block must be a positive multiple of 64");
  if (o->grid_block != kG) fail(KLDI_E_UNSUPPORTED, "this build supports grid_block = 128");
  if (o->ao_block != kD) fail(KLDI_E_UNSUPPORTED, "this build supports ao_block = 32");
  if (o->prec != KLDI_PREC_FP64 && o->prec != KLDI_PREC_FP32) fail(KLDI_E_ARG, "unknown prec");
  if (o->xc != KLDI_XC_LDA_X && o->xc != KLDI_XC_PBE && o->xc != KLDI_XC_PBE_X) fail(KLDI_E_ARG, "unknown xc");
  if (o->v_segment < 0) fail(KLDI_E_ARG, "v_segment must be >= 0");
  if (o->chunk_tiles < 0) fail(KLDI_E_ARG, "chunk_tiles must be >= 0");
}

void build_plan(Plan &P, const kldi_basis *b, const kldi_grid *g, const kldi_opts *o, hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  check_hip(hipGetDevice(&P.device), "hipGetDevice");
  P.opts = *o;
  P.gga = (o->xc != KLDI_XC_LDA_X);
  const int na = b->n_atoms, ns = b->n_shells;
  const int64_t npt = g->n_points;
  P.n_points = npt;
  P.n_shells = ns;

  // ---- reordering (Sec. III-B.2): atoms by Morton key of their centres, points grouped by
  // associated atom then Morton-sorted, AOs grouped by atom
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
    P.n_ao = int(off);
  }
  std::vector<std::vector<int>> shells_of(na);
  for (int s = 0; s < ns; ++s) shells_of[b->shell_atom[s]].push_back(s);
  std::vector<int> shell_order;  // internal -> caller shell
  for (int a : aorder)
    for (int s : shells_of[a]) shell_order.push_back(s);

  P.n_tiles = (P.n_ao + kD - 1) / kD;
  P.n_chunks = (P.n_tiles + kChunk - 1) / kChunk;
  const int nao_pad = P.n_tiles * kD;
  std::vector<double> sh_xyz(3 * ns), pexp, pcoef;
  std::vector<int> sh_prim(2 * ns), sh_l(ns), sh_ao0(ns), ao_shell(nao_pad, -1), ao_comp(nao_pad, 0);
  P.ao_perm.assign(P.n_ao, 0);
  {
    int ao = 0;
    for (int is = 0; is < ns; ++is) {
      int s = shell_order[is];
      int l = b->shell_l[s];
      for (int d = 0; d < 3; ++d) sh_xyz[3 * is + d] = b->atom_xyz[3 * b->shell_atom[s] + d];
      sh_prim[2 * is] = int(pexp.size());
      for (int k = b->shell_prim_ptr[s]; k < b->shell_prim_ptr[s + 1]; ++k) {
        pexp.push_back(b->prim_exp[k]);
        pcoef.push_back(b->prim_coef[k]);
      }
      sh_prim[2 * is + 1] = int(pexp.size());
      sh_l[is] = l;
      sh_ao0[is] = ao;
      for (int c = 0; c < ncart(l); ++c) {
        int lx, ly, lz;
        cart_powers(l, c, lx, ly, lz);
        ao_shell[ao] = is;
        ao_comp[ao] = lx | (ly << 2) | (lz << 4);
        P.ao_perm[ao] = int32_t(cao0[s] + c);
        ++ao;
      }
    }
  }
  std::vector<int> tile_sh(2 * P.n_tiles);
  for (int p = 0; p < P.n_tiles; ++p) {
    int a0 = p * kD, a1 = std::min(P.n_ao, a0 + kD) - 1;
    tile_sh[2 * p] = ao_shell[a0];
    tile_sh[2 * p + 1] = ao_shell[a1] + 1;
  }

  // points
  std::vector<uint64_t> pkey(npt);
  for (int64_t i = 0; i < npt; ++i)
    pkey[i] = morton(discretise(g->xyz[3 * i], origin[0]), discretise(g->xyz[3 * i + 1], origin[1]),
                     discretise(g->xyz[3 * i + 2], origin[2]));
  P.pt_perm.resize(npt);
  std::iota(P.pt_perm.begin(), P.pt_perm.end(), int64_t(0));
  std::stable_sort(P.pt_perm.begin(), P.pt_perm.end(), [&](int64_t x, int64_t y) {
    int rx = arank[g->point_atom[x]], ry = arank[g->point_atom[y]];
    if (rx != ry) return rx < ry;
    return pkey[x] < pkey[y];
  });
  P.n_blocks = (npt + kG - 1) / kG;
  P.n_pad = P.n_blocks * kG;
  std::vector<double> px(P.n_pad), py(P.n_pad), pz(P.n_pad), pw(P.n_pad, 0.0);
  std::vector<int64_t> porig(P.n_pad, -1);
  for (int64_t i = 0; i < P.n_pad; ++i) {
    int64_t c = P.pt_perm[std::min(i, npt - 1)];
    px[i] = g->xyz[3 * c];
    py[i] = g->xyz[3 * c + 1];
    pz[i] = g->xyz[3 * c + 2];
    if (i < npt) {
      pw[i] = g->weight[c];
      porig[i] = c;
    }
  }

  // ---- shell radii and candidate (tile, block) pairs
  std::vector<double> rad(ns);
  for (int is = 0; is < ns; ++is)
    rad[is] = shell_radius(sh_l[is], &pexp[sh_prim[2 * is]], &pcoef[sh_prim[2 * is]],
                           sh_prim[2 * is + 1] - sh_prim[2 * is], P.gga, o->t_b);
  std::vector<int> cand_p;
  std::vector<int64_t> cand_r;
  for (int64_t r = 0; r < P.n_blocks; ++r) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = r * kG; i < std::min(npt, (r + 1) * kG); ++i) {
      lo[0] = std::min(lo[0], px[i]); hi[0] = std::max(hi[0], px[i]);
      lo[1] = std::min(lo[1], py[i]); hi[1] = std::max(hi[1], py[i]);
      lo[2] = std::min(lo[2], pz[i]); hi[2] = std::max(hi[2], pz[i]);
    }
    for (int p = 0; p < P.n_tiles; ++p) {
      bool near = false;
      for (int is = tile_sh[2 * p]; is < tile_sh[2 * p + 1] && !near; ++is) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) {
          double c = sh_xyz[3 * is + d];
          double e = std::max(0.0, std::max(lo[d] - c, c - hi[d]));
          d2 += e * e;
        }
        near = std::sqrt(d2) <= rad[is];
      }
      if (near) {
        cand_p.push_back(p);
        cand_r.push_back(r);
      }
    }
  }
  P.n_cand = int64_t(cand_p.size());

  // ---- device copies of basis and grid
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
  B.n_ao = P.n_ao;
  B.n_tiles = P.n_tiles;
  GridDev &Gd = P.grid;
  Gd.x = dev_upload(P, px);
  Gd.y = dev_upload(P, py);
  Gd.z = dev_upload(P, pz);
  Gd.w = dev_upload(P, pw);
  Gd.orig = dev_upload(P, porig);
  Gd.n_blocks = P.n_blocks;

  // ---- exact block maxima on the device (eq. block_summary_A), retention (eq. block_filter_A)
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
  P.blk_off_h.assign(P.n_blocks + 1, 0);
  std::vector<int> ret_r;
  std::vector<int> idx_map(size_t(P.n_blocks) * P.n_tiles, -1);
  for (int64_t c = 0; c < P.n_cand; ++c) {
    double s = P.gga ? std::max(cb[c], cg[c]) : cb[c];
    if (s >= o->t_b) {
      int64_t r = cand_r[c];
      idx_map[size_t(r) * P.n_tiles + cand_p[c]] = int(P.blk_off_h[r + 1]);
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
  S.idx_map = dev_upload(P, idx_map);
  S.bphi = dev_upload(P, P.bphi_h);
  // X work items: (block, chunk of 4 consecutive retained tiles), block-major
  {
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
    P.xit_r = dev_upload(P, xr);
    P.xit_c = dev_upload(P, xc);
    P.blk_item_off = dev_upload(P, boff);
    P.blk_item_off_h = boff;
  }

  // ---- Vxc work list: (row chunk, column chunk, segment of grid blocks)
  const int nc = P.n_chunks;
  const int npairs = P.gga ? nc * nc : nc * (nc + 1) / 2;
  P.n_pairs = npairs;
  auto pair_index = [&](int pc, int qc) { return P.gga ? pc * nc + qc : pc * nc - pc * (pc - 1) / 2 + (qc - pc); };
  // chunks present at each block
  std::vector<std::vector<int>> blk_chunks(P.n_blocks);
  for (int64_t r = 0; r < P.n_blocks; ++r)
    for (int64_t k = P.blk_off_h[r]; k < P.blk_off_h[r + 1]; ++k) {
      const int c = P.ret_p_h[k] / kChunk;
      if (blk_chunks[r].empty() || blk_chunks[r].back() != c) blk_chunks[r].push_back(c);
    }
  // work items of a segment length: the chunk pairs that co-occur at some block of the segment
  std::vector<int> stamp(npairs, -1);
  auto visit_items = [&](int seg, auto &&emit) {
    const int64_t nseg = (P.n_blocks + seg - 1) / seg;
    for (int64_t sg = 0; sg < nseg; ++sg) {
      const int r0 = int(sg * seg), r1 = int(std::min<int64_t>(P.n_blocks, (sg + 1) * seg));
      std::vector<int> act;
      for (int r = r0; r < r1; ++r)
        for (int pc : blk_chunks[r])
          for (int qc : blk_chunks[r]) {
            if (!P.gga && qc < pc) continue;
            const int pi = pair_index(pc, qc);
            if (stamp[pi] != int(sg)) {
              stamp[pi] = int(sg);
              act.push_back(pi);
            }
          }
      std::sort(act.begin(), act.end());
      for (int pi : act) emit(pi, r0, r1);
    }
    std::fill(stamp.begin(), stamp.end(), -1);
  };
  int seg = o->v_segment;
  if (seg <= 0) {
    // shortest segment (better L2 sharing among the items of a segment) whose FP64 partials fit a
    // budget of min(16 GiB, 1/5 of free device memory)
    size_t fr0 = 0, tot0 = 0;
    check_hip(hipMemGetInfo(&fr0, &tot0), "hipMemGetInfo");
    const size_t budget = std::min<size_t>(size_t(16) << 30, fr0 / 5);
    for (seg = 16;; seg *= 2) {
      int64_t n = 0;
      visit_items(seg, [&](int, int, int) { ++n; });
      if (size_t(n) * 16384 * 8 <= budget || seg >= P.n_blocks) break;
    }
  }
  P.v_segment = seg;
  std::vector<std::vector<int>> pair_lists(npairs);
  std::vector<int> pair_pc(npairs), pair_qc(npairs);
  for (int pc = 0; pc < nc; ++pc)
    for (int qc = P.gga ? 0 : pc; qc < nc; ++qc) {
      pair_pc[pair_index(pc, qc)] = pc;
      pair_qc[pair_index(pc, qc)] = qc;
    }
  const int64_t n_segs = (P.n_blocks + seg - 1) / seg;
  std::vector<int64_t> seg_item_off(n_segs + 1, 0);
  visit_items(seg, [&](int pi, int r0, int r1) {
    pair_lists[pi].push_back(int(P.items_h.size()));
    P.items_h.push_back(VItem{pair_pc[pi], pair_qc[pi], r0, r1, pi, 0});
    seg_item_off[r0 / seg + 1] = int64_t(P.items_h.size());
  });
  for (int64_t sg = 1; sg <= n_segs; ++sg) seg_item_off[sg] = std::max(seg_item_off[sg], seg_item_off[sg - 1]);
  std::vector<int> pair_ptr(npairs + 1, 0), pair_items, pair_pq(2 * npairs);
  for (int i = 0; i < npairs; ++i) {
    pair_pq[2 * i] = pair_pc[i];
    pair_pq[2 * i + 1] = pair_qc[i];
  }
  for (int i = 0; i < npairs; ++i) {
    pair_ptr[i + 1] = pair_ptr[i] + int(pair_lists[i].size());
    pair_items.insert(pair_items.end(), pair_lists[i].begin(), pair_lists[i].end());
  }
  P.items = dev_upload(P, P.items_h);
  P.pair_ptr = dev_upload(P, pair_ptr);
  P.pair_items = dev_upload(P, pair_items);
  P.pair_pq = dev_upload(P, pair_pq);
  {
    // per (block, chunk): position in S_r of the chunk's first retained tile, and its 4-bit mask
    std::vector<int> cinfo(size_t(P.n_blocks) * nc, 0);
    for (int64_t r = 0; r < P.n_blocks; ++r)
      for (int64_t k = P.blk_off_h[r + 1] - 1; k >= P.blk_off_h[r]; --k) {
        const int p = P.ret_p_h[k], c = p / kChunk;
        int &ci = cinfo[size_t(r) * nc + c];
        ci = (int(k - P.blk_off_h[r]) << 4) | (ci & 15) | (1 << (p % kChunk));
      }
    P.cinfo = dev_upload(P, cinfo);
  }
  P.ao_perm_d = dev_upload(P, P.ao_perm);

  // ---- grid chunks: whole Vxc segments whose retained tiles fit the Phi / Z workspaces
  const size_t esz = (o->prec == KLDI_PREC_FP64) ? 8 : 4;
  const size_t fixed = size_t(P.items_h.size()) * 16384 * 8 + size_t(nc * kChunk * kD) * size_t(nc * kChunk * kD) * 8 +
                       size_t(P.n_pad) * 32 + size_t(P.n_ret) * 8 + size_t(P.n_tiles) * P.n_tiles * (1024 * esz + 8);
  const size_t per_tile = 2 * 4096 * esz;       // Phi + Z
  int64_t cap = o->chunk_tiles;
  {
    size_t fr = 0, tot = 0;
    check_hip(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    const size_t reserve = size_t(1) << 30;
    if (fixed + reserve > fr) fail(KLDI_E_OOM, "fixed workspaces need " + std::to_string(fixed >> 20) + " MiB");
    const int64_t fit = int64_t((fr - fixed - reserve) * 0.8 / (per_tile + 4096));
    if (cap <= 0 || cap > fit) cap = fit;
  }
  {
    int64_t s0 = 0;
    while (s0 < n_segs) {
      int64_t s1 = s0 + 1;
      auto ret_of = [&](int64_t a, int64_t b) {
        return P.blk_off_h[std::min<int64_t>(P.n_blocks, b * seg)] - P.blk_off_h[a * seg];
      };
      while (s1 < n_segs && ret_of(s0, s1 + 1) <= cap) ++s1;
      GridChunk C;
      C.blk0 = s0 * seg;
      C.blk1 = std::min<int64_t>(P.n_blocks, s1 * seg);
      C.ret0 = P.blk_off_h[C.blk0];
      C.ret1 = P.blk_off_h[C.blk1];
      C.xit0 = P.blk_item_off_h[C.blk0];
      C.xit1 = P.blk_item_off_h[C.blk1];
      C.vit0 = seg_item_off[s0];
      C.vit1 = seg_item_off[s1];
      P.chunks_h.push_back(C);
      s0 = s1;
    }
  }
  int64_t max_ret = 0, max_xit = 0, max_blk = 0;
  for (const GridChunk &C : P.chunks_h) {
    max_ret = std::max(max_ret, C.ret1 - C.ret0);
    max_xit = std::max(max_xit, C.xit1 - C.xit0);
    max_blk = std::max(max_blk, C.blk1 - C.blk0);
  }
  EvalDev &E = P.ev;
  size_t nt2 = size_t(P.n_tiles) * P.n_tiles;
  E.Dt = (esz == 8) ? (void *)dev_alloc<double>(P, nt2 * 1024) : (void *)dev_alloc<float>(P, nt2 * 1024);
  E.amax = dev_alloc<double>(P, nt2);
  if (esz == 8) {
    E.phi = dev_alloc<double>(P, size_t(max_ret) * 4096);
    E.zws = dev_alloc<double>(P, size_t(max_ret) * 4096);
  } else {
    E.phi = dev_alloc<float>(P, size_t(max_ret) * 4096);
    E.zws = dev_alloc<float>(P, size_t(max_ret) * 4096);
  }
  E.zmax = dev_alloc<double>(P, P.n_ret);
  E.xpart = dev_alloc<double>(P, size_t(max_xit) * 4 * kG);
  E.coef = dev_alloc<double>(P, size_t(P.n_pad) * 4);
  E.eblk = dev_alloc<double>(P, P.n_blocks);
  E.vpart = dev_alloc<double>(P, P.items_h.size() * 16384);
  E.vflag = dev_alloc<int>(P, P.items_h.size());
  E.vmask = dev_alloc<unsigned short>(P, size_t(max_blk) * npairs);
  E.mfull = dev_alloc<double>(P, size_t(nc * kChunk * kD) * size_t(nc * kChunk * kD));
  E.counters = dev_alloc<unsigned long long>(P, 4);
  E.escratch = dev_alloc<double>(P, 1);
  check_hip(hipMemsetAsync(E.counters, 0, 4 * sizeof(unsigned long long), stream), "memset");
  check_hip(hipStreamSynchronize(stream), "plan sync");
  P.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
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

}  // namespace
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
}

kldi_status kldi_plan_create(const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts, void *stream,
                             kldi_plan **out) {
  kldi::set_error("");
  if (!out) {
    kldi::set_error("out must not be NULL");
    return KLDI_E_ARG;
  }
  *out = nullptr;
  kldi_plan *plan = nullptr;
  kldi_status st = kldi::guarded([&] {
    kldi::validate(basis, grid, opts);
    plan = new kldi_plan();
    kldi::build_plan(plan->impl, basis, grid, opts, static_cast<hipStream_t>(stream));
  });
  if (st != KLDI_OK) {
    if (plan) {
      kldi::free_plan(plan->impl);
      delete plan;
    }
    return st;
  }
  *out = plan;
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
  out->retained_fraction = double(P.n_ret) / (double(P.n_tiles) * double(P.n_blocks));
  out->max_tiles_per_block = P.max_np;
  out->v_segment = P.v_segment;
  out->n_v_items = int64_t(P.items_h.size());
  out->workspace_bytes = int64_t(P.bytes);
  out->n_grid_chunks = int32_t(P.chunks_h.size());
  out->plan_ms = P.plan_ms;
  return KLDI_OK;
}

kldi_status kldi_plan_structure(const kldi_plan *plan, int32_t *ao_perm, int64_t *pt_perm, uint8_t *retained,
                                double *phi_max) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  const Plan &P = plan->impl;
  if (ao_perm) std::copy(P.ao_perm.begin(), P.ao_perm.end(), ao_perm);
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
    const Plan &P = plan->impl;
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    hipEvent_t *ev = nullptr;
    if (P.timing) {
      ev = &plan->impl.events[size_t(P.n_timed % kldi::kTimingSlots) * (KLDI_N_STAGES + 1)];
      plan->impl.n_timed++;
    }
    kldi::check_hip(
        kldi::launch_eval(P, D_dev, rho_dev, nullptr, exc_dev, vxc_dev, static_cast<hipStream_t>(stream), ev),
        "eval launch");
  });
}

kldi_status kldi_eval_check(kldi_plan *plan, kldi_eval_stats_t *out, void *stream) {
  if (!plan || !out) {
    kldi::set_error("plan and out must not be NULL");
    return KLDI_E_ARG;
  }
  unsigned long long c[4] = {0, 0, 0, 0};
  kldi_status st = kldi::guarded([&] {
    kldi::check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "sync");
    kldi::check_hip(hipMemcpy(c, plan->impl.ev.counters, sizeof(c), hipMemcpyDeviceToHost), "copy counters");
  });
  if (st != KLDI_OK) return st;
  out->n_pairs_x = int64_t(c[0]);
  out->n_pairs_v = int64_t(c[1]);
  out->gemm_flops = 2.0 * kldi::kD * kldi::kD * kldi::kG * double(c[0] + c[1]);
  out->n_points_mlp = int64_t(c[3]);
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
    const Plan &P = plan->impl;
    kldi::check_hip(hipSetDevice(P.device), "hipSetDevice");
    // E_xc of this call goes to the plan's per-block partials only
    kldi::check_hip(kldi::launch_eval(P, D_dev, rho_dev, sigma_dev, P.ev.escratch, nullptr,
                                      static_cast<hipStream_t>(stream), nullptr),
                    "eval launch");
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

int32_t kldi_version(void) { return 1; }

}  // extern "C"
