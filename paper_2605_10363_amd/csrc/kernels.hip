// HIP kernels of libkldi for gfx950 (MI355X): block-filtered EXC integration.
//
// Per evaluation (one stream, no host synchronisation):
//   k_reset    clear the executed-pair counters
//   k_dprep    D (caller order, FP64) -> internal AO order, 32x32 tiles, working precision; block
//              summaries a_pq = max|D_pq| (eq. block_summary_A); non-finite check
//   k_basis    Phi on the retained (tile, grid block) pairs only (eq. phi_def)
//   k_xtask    one workgroup per grid block r: for each chunk of 4 output tiles p of S_r, the
//              executable q are selected by a_pq * b_qr >= t_d (eq. block_pair_filter) and
//              compacted by prefix sum (Appendix D); X_pr = sum_q D_pq Phi_qr on MFMA with LDS-staged
//              tiles, accumulated in registers before the epilogue (Sec. III-C.2); rho and grad rho
//              epilogue; the functional; Z on all retained tiles of r with their max-abs summaries
//   k_vgemm    one workgroup per (row chunk, column chunk, segment of grid blocks): executable grid
//              blocks selected by b_pr * z_qr >= t_d and compacted; M_pq = sum_r Phi_pr Z_qr^T on MFMA
//   k_vreduce  FP64 sum of the segment partials in fixed order
//   k_vsym     Vxc = M + M^T (GGA) or mirrored 2M (LDA), back to the caller's AO order
//   k_esum     E_xc as a fixed-order FP64 sum of per-block partials
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kldi_impl.h"

namespace kldi {
namespace {

constexpr int NT = 256;          // threads per workgroup (4 waves of 64)
constexpr int LDA_S = 33;        // LDS row stride of 32-wide row tiles
constexpr int LDB_S = 130;       // LDS row stride of 128-wide rows
constexpr int kMaxNp = 512;      // retained tiles per grid block handled by k_xtask

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------------
// MFMA 16x16x4 wrappers.  Lane l supplies A[l%16][l/16] and B[l/16][l%16]; element v of the
// accumulator of lane l is C[row(v,l)][l%16] -- row = 4v + l/16 for FP64, 4(l/16) + v for FP32
// (measured on gfx950).
// ------------------------------------------------------------------------------------------------
template <class T>
struct Mma;
template <>
struct Mma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 4 * v + (l >> 4); }
};
template <>
struct Mma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 4 * (l >> 4) + v; }
};

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n) {
  // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
  // work items so neighbouring items (similar retained supports) share an L2
  int64_t per = (n + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Exclusive prefix sum of a 0/1 flag over the 256 threads of a workgroup (parallel addressing):
// ballot + popcount within each wave, wave totals through LDS.  Returns the thread's slot and the
// total in *total.  Must be called by all threads.
__device__ __forceinline__ int block_scan(int flag, int *s_w, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long bal = __ballot(flag);
  int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) s_w[w] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < 4; ++i) {
    off += (i < w) ? s_w[i] : 0;
    tot += s_w[i];
  }
  __syncthreads();
  *total = tot;
  return off + before;
}

// ------------------------------------------------------------------------------------------------
// Basis functions (contracted cartesian Gaussians, N_rel-normalised components)
// ------------------------------------------------------------------------------------------------
__constant__ int c_pow[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                 {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
__constant__ double c_nrel[10] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.7320508075688772, 1.7320508075688772,
                                  1.0, 1.7320508075688772, 1.0};

__device__ __forceinline__ void pw4(double d, double *p) {
  p[0] = 1.0;
  p[1] = d;
  p[2] = d * d;
  p[3] = p[2] * d;
}

// Calls emit(a, value, gx, gy, gz) for every AO a (local row 0..31) of tile p at (x, y, z).
template <bool GRAD, class F>
__device__ __forceinline__ void for_tile_aos(const BasisDev &B, int p, double x, double y, double z, F &&emit) {
  const int s0 = B.tile_sh[2 * p], s1 = B.tile_sh[2 * p + 1];
  const int a_lo = p * kD, a_hi = a_lo + kD;
  for (int s = s0; s < s1; ++s) {
    const double dx = x - B.sh_xyz[3 * s], dy = y - B.sh_xyz[3 * s + 1], dz = z - B.sh_xyz[3 * s + 2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    double R = 0.0, R1 = 0.0;
    for (int k = B.sh_prim[2 * s]; k < B.sh_prim[2 * s + 1]; ++k) {
      const double e = B.pcoef[k] * exp(-B.pexp[k] * r2);
      R += e;
      if (GRAD) R1 -= 2.0 * B.pexp[k] * e;
    }
    const int l = B.sh_l[s], ao0 = B.sh_ao0[s];
    const int cb = (l == 0) ? 0 : (l == 1 ? 1 : 4), nc = (l + 1) * (l + 2) / 2;
    double px[4], py[4], pz[4];
    pw4(dx, px);
    pw4(dy, py);
    pw4(dz, pz);
    for (int c = 0; c < nc; ++c) {
      const int ao = ao0 + c;
      if (ao < a_lo || ao >= a_hi) continue;
      const int lx = c_pow[cb + c][0], ly = c_pow[cb + c][1], lz = c_pow[cb + c][2];
      const double nr = c_nrel[cb + c];
      const double ang = px[lx] * py[ly] * pz[lz];
      double gx = 0, gy = 0, gz = 0;
      if (GRAD) {
        gx = nr * ((lx ? lx * px[lx - 1] * py[ly] * pz[lz] : 0.0) * R + ang * dx * R1);
        gy = nr * ((ly ? ly * px[lx] * py[ly - 1] * pz[lz] : 0.0) * R + ang * dy * R1);
        gz = nr * ((lz ? lz * px[lx] * py[ly] * pz[lz - 1] : 0.0) * R + ang * dz * R1);
      }
      emit(ao - a_lo, nr * ang * R, gx, gy, gz);
    }
  }
}

// Value and gradient of one internal AO at (x, y, z); zero on padding rows.
__device__ __forceinline__ void eval_ao(const BasisDev &B, int ao, double x, double y, double z, double &v,
                                        double &gx, double &gy, double &gz) {
  v = gx = gy = gz = 0.0;
  const int s = B.ao_shell[ao];
  if (s < 0) return;
  const double dx = x - B.sh_xyz[3 * s], dy = y - B.sh_xyz[3 * s + 1], dz = z - B.sh_xyz[3 * s + 2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  double R = 0.0, R1 = 0.0;
  for (int k = B.sh_prim[2 * s]; k < B.sh_prim[2 * s + 1]; ++k) {
    const double e = B.pcoef[k] * exp(-B.pexp[k] * r2);
    R += e;
    R1 -= 2.0 * B.pexp[k] * e;
  }
  const int cp = B.ao_comp[ao];
  const int lx = cp & 3, ly = (cp >> 2) & 3, lz = (cp >> 4) & 3;
  const double nr = ((lx == 1) + (ly == 1) + (lz == 1) == 2) ? 1.7320508075688772 : 1.0;
  double px[4], py[4], pz[4];
  pw4(dx, px);
  pw4(dy, py);
  pw4(dz, pz);
  const double ang = px[lx] * py[ly] * pz[lz];
  v = nr * ang * R;
  gx = nr * ((lx ? lx * px[lx - 1] * py[ly] * pz[lz] : 0.0) * R + ang * dx * R1);
  gy = nr * ((ly ? ly * px[lx] * py[ly - 1] * pz[lz] : 0.0) * R + ang * dy * R1);
  gz = nr * ((lz ? lz * px[lx] * py[ly] * pz[lz - 1] : 0.0) * R + ang * dz * R1);
}

// ------------------------------------------------------------------------------------------------
// Functionals, FP64 (spin-unpolarised).  LDA: Slater exchange.  PBE: PBE exchange (kappa = 0.804,
// mu = beta pi^2/3), PW92 correlation (unpolarised fit), PBE gradient correction H (phi = 1).
// Returns f (energy per volume), v_rho = df/drho, v_sigma = df/dsigma.
// ------------------------------------------------------------------------------------------------
struct Xc {
  double f, vr, vs;
};

__device__ __forceinline__ Xc xc_lda(double rho) {
  const double cx = 0.73855876638202234;  // (3/4)(3/pi)^(1/3)
  const double r13 = cbrt(rho);
  return Xc{-cx * rho * r13, -(4.0 / 3.0) * cx * r13, 0.0};
}

__device__ __forceinline__ Xc xc_pbe_x(double rho, double sigma) {
  const double cx = 0.73855876638202234, kappa = 0.804, mu = 0.21951497276451709;
  const double r13 = cbrt(rho);
  const double kf = cbrt(29.608813203268074 * rho);  // (3 pi^2 rho)^(1/3)
  const double ds2 = 1.0 / (4.0 * kf * kf * rho * rho);
  const double s2 = sigma * ds2;
  const double den = 1.0 + mu * s2 / kappa;
  const double F = 1.0 + kappa - kappa / den;
  const double dF = mu / (den * den);
  const double el = -cx * rho * r13;
  return Xc{el * F, -cx * r13 * ((4.0 / 3.0) * F - (8.0 / 3.0) * s2 * dF), el * dF * ds2};
}

__device__ __forceinline__ Xc xc_pbe_c(double rho, double sigma) {
  const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double beta = 0.06672455060314922, gamma = 0.031090690869654895;  // (1 - ln 2)/pi^2
  const double rs = cbrt(0.23873241463784300 / rho);                      // (3/(4 pi rho))^(1/3)
  const double srs = sqrt(rs);
  const double q0 = -2.0 * A * (1.0 + a1 * rs);
  const double q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
  const double dq1 = 2.0 * A * (0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs);
  const double lg = log1p(1.0 / q1);
  const double eps = q0 * lg;
  const double deps_drs = -2.0 * A * a1 * lg - q0 * dq1 / (q1 * q1 + q1);
  const double deps = deps_drs * (-rs / (3.0 * rho));
  const double kf = cbrt(29.608813203268074 * rho);
  const double ks2 = 4.0 * kf / 3.14159265358979324;
  const double dt2 = 1.0 / (4.0 * ks2 * rho * rho);
  const double t2 = sigma * dt2;
  const double bg = beta / gamma;
  const double Ac = bg / expm1(-eps / gamma);
  const double dAc = Ac * Ac * exp(-eps / gamma) / beta;
  const double u = Ac * t2;
  const double den = 1.0 + u + u * u;
  const double Q = (1.0 + u) / den;
  const double dQ = -u * (2.0 + u) / (den * den);
  const double y = bg * t2 * Q;
  const double H = gamma * log1p(y);
  const double dHy = gamma / (1.0 + y);
  const double dyt2 = bg * (Q + t2 * dQ * Ac);
  const double dyA = bg * t2 * dQ * t2;
  const double dHr = dHy * (dyA * dAc * deps + dyt2 * (-7.0 / 3.0) * t2 / rho);
  return Xc{rho * (eps + H), eps + H + rho * (deps + dHr), rho * dHy * dyt2 * dt2};
}

__device__ __forceinline__ Xc xc_eval(int xc, double rho, double sigma, double rho_cut) {
  if (!(rho > rho_cut)) return Xc{0.0, 0.0, 0.0};
  if (xc == KLDI_XC_LDA_X) return xc_lda(rho);
  Xc x = xc_pbe_x(rho, sigma);
  if (xc == KLDI_XC_PBE_X) return x;
  Xc c = xc_pbe_c(rho, sigma);
  return Xc{x.f + c.f, x.vr + c.vr, x.vs + c.vs};
}

// ------------------------------------------------------------------------------------------------
// plan-time screening: exact max |Phi| (and max |grad Phi|) of candidate (tile, block) pairs
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kG) void k_screen(BasisDev B, GridDev g, const int *cand_p, const int64_t *cand_r,
                                              int64_t n_cand, int gga, double *out_b, double *out_g) {
  const int64_t c = blockIdx.x;
  if (c >= n_cand) return;
  const int p = cand_p[c];
  const int64_t ip = cand_r[c] * kG + threadIdx.x;
  const double x = g.x[ip], y = g.y[ip], z = g.z[ip];
  double bm = 0.0, gm = 0.0;
  if (gga) {
    for_tile_aos<true>(B, p, x, y, z, [&](int, double v, double gx, double gy, double gz) {
      bm = fmax(bm, fabs(v));
      gm = fmax(gm, fmax(fabs(gx), fmax(fabs(gy), fabs(gz))));
    });
  } else {
    for_tile_aos<false>(B, p, x, y, z, [&](int, double v, double, double, double) { bm = fmax(bm, fabs(v)); });
  }
  __shared__ double s[2][2];
  bm = wave_max(bm);
  gm = wave_max(gm);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[0][w] = bm;
    s[1][w] = gm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out_b[c] = fmax(s[0][0], s[0][1]);
    out_g[c] = fmax(s[1][0], s[1][1]);
  }
}

// ------------------------------------------------------------------------------------------------
// per-evaluation kernels
// ------------------------------------------------------------------------------------------------
__global__ void k_reset(unsigned long long *counters) {
  if (threadIdx.x < 4) counters[threadIdx.x] = 0ull;
}

template <class T>
__global__ __launch_bounds__(NT) void k_dprep(const double *__restrict__ D, const int *__restrict__ perm, int n_ao,
                                             int n_tiles, T *__restrict__ Dt, double *__restrict__ amax,
                                             unsigned long long *counters) {
  const int p = blockIdx.x / n_tiles, q = blockIdx.x % n_tiles;
  double m = 0.0;
  int bad = 0;
  for (int e = threadIdx.x; e < kD * kD; e += NT) {
    const int i = p * kD + e / kD, j = q * kD + e % kD;
    double v = 0.0;
    if (i < n_ao && j < n_ao) v = D[size_t(perm[i]) * n_ao + perm[j]];
    if (!isfinite(v)) bad = 1;
    m = fmax(m, fabs(v));
    Dt[size_t(blockIdx.x) * (kD * kD) + e] = T(v);
  }
  __shared__ double s[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&counters[2], 1ull);
  __syncthreads();
  if (threadIdx.x == 0) amax[blockIdx.x] = fmax(fmax(s[0], s[1]), fmax(s[2], s[3]));
}

template <class T>
__global__ __launch_bounds__(kG) void k_basis(BasisDev B, GridDev g, StructDev st, T *__restrict__ phi) {
  const int64_t k = blockIdx.x;
  const int p = st.ret_p[k];
  const int64_t ip = int64_t(st.ret_r[k]) * kG + threadIdx.x;
  const double x = g.x[ip], y = g.y[ip], z = g.z[ip];
  T *out = phi + size_t(k) * (kD * kG) + threadIdx.x;
  const int nvalid = min(kD, B.n_ao - p * kD);
  for (int a = nvalid; a < kD; ++a) out[a * kG] = T(0);
  for_tile_aos<false>(B, p, x, y, z, [&](int a, double v, double, double, double) { out[a * kG] = T(v); });
}

// 16-byte unit copies between global memory and LDS rows
template <class T>
struct Units {
  static constexpr int E = 16 / sizeof(T);  // elements per 16-byte unit
};

template <class T>
__device__ __forceinline__ void lds_store_unit(T *dst, const uint4 &u) {
  const T *src = reinterpret_cast<const T *>(&u);
#pragma unroll
  for (int m = 0; m < Units<T>::E; ++m) dst[m] = src[m];
}

struct XArgs {
  BasisDev B;
  GridDev g;
  StructDev st;
  const void *Dt;
  const double *amax;
  const void *phi;
  void *zws;
  double *zmax;
  double *eblk;
  double *rho_out;
  unsigned long long *counters;
  double t_b, t_d, rho_cut;
  int xc;
  int want_z;
};

// One workgroup per grid block r (4 waves; wave w owns output tile 4c + w of each chunk c).
template <class T, bool GGA>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? 2 : 1) void k_xtask(XArgs A) {
  typedef Mma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int E = Units<T>::E;
  const int64_t r = xcd_remap(blockIdx.x, A.g.n_blocks);
  if (r >= A.g.n_blocks) return;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int n_tiles = A.B.n_tiles;
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  const T *Dt = static_cast<const T *>(A.Dt);
  const T *phi = static_cast<const T *>(A.phi);

  // LDS: the K loop double-buffers A (128 x 32) and B (32 x 128) tiles; the epilogue reuses the
  // same bytes for two 32 x 128 X tiles at a time
  constexpr int kA = 128 * LDA_S, kB = 32 * LDB_S;
  constexpr int kStageBytes = 2 * (kA + kB) * int(sizeof(T));
  static_assert(kStageBytes >= 2 * kD * kG * int(sizeof(T)), "epilogue X tiles must fit the staging area");
  __shared__ __align__(16) unsigned char s_raw[kStageBytes];
  T *sA = reinterpret_cast<T *>(s_raw);   // [2][kA]
  T *sB = sA + 2 * kA;                     // [2][kB]
  T *Xs = sA;                              // [2][32][kG] in the epilogue
  __shared__ int s_p[kMaxNp];
  __shared__ int s_list[kMaxNp];
  __shared__ int s_w[4];
  __shared__ double s_acc[2][4][kG];  // rho, grad rho partial sums, one copy per half workgroup
  __shared__ double s_red[kG];

  for (int t = tid; t < np; t += NT) s_p[t] = A.st.ret_p[k0 + t];
  for (int e = tid; e < 8 * kG; e += NT) (&s_acc[0][0][0])[e] = 0.0;
  __syncthreads();
  const int half = tid >> 7, j = tid & (kG - 1);
  const int64_t ipj = r * kG + j;
  double px = 0, py = 0, pz = 0;
  if (GGA) {
    px = A.g.x[ipj];
    py = A.g.y[ipj];
    pz = A.g.z[ipj];
  }

  unsigned long long pairs = 0;
  for (int c = 0; 4 * c < np; ++c) {
    // ---- executable pairs for this chunk (eq. block_pair_filter), compacted (Appendix D)
    int n_list = 0;
    for (int base = 0; base < np; base += NT) {
      const int t = base + tid;
      int mask = 0;
      if (t < np) {
        const int q = s_p[t];
        const double bq = A.st.bphi[k0 + t];
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          if (4 * c + ww < np) {
            const double a = A.amax[size_t(s_p[4 * c + ww]) * n_tiles + q];
            if (a >= A.t_b && a * bq >= A.t_d) mask |= 1 << ww;
          }
        }
      }
      int tot;
      const int pos = block_scan(mask != 0, s_w, &tot);
      if (mask) {
        s_list[n_list + pos] = t | (mask << 16);
        pairs += __popc(mask);
      }
      n_list += tot;
    }
    __syncthreads();

    // ---- X = sum over executable q of D_pq Phi_qr (MFMA).  Tiles of step e+1 are fetched into
    // registers while step e multiplies out of LDS; one barrier per step (double-buffered LDS)
    acc_t acc[2][8];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 8; ++tj) acc[ti][tj] = acc_t{};
    const bool has_w = 4 * c + w < np;
    constexpr int UA = (kD * kD) / E;   // 16-byte units per D tile
    constexpr int UB = (kD * kG) / E;   // units per Phi tile
    constexpr int NA = 4 * UA / NT, NB = UB / NT;
    uint4 ra[NA], rb[NB];
    auto fetch = [&](int e) {
      const int t = s_list[e] & 0xffff;
      const int q = s_p[t];
#pragma unroll
      for (int m = 0; m < NA; ++m) {
        const int u = tid + NT * m, ww = u / UA, uu = u % UA;
        ra[m] = make_uint4(0, 0, 0, 0);
        if (4 * c + ww < np)
          ra[m] = reinterpret_cast<const uint4 *>(Dt + (size_t(s_p[4 * c + ww]) * n_tiles + q) * (kD * kD))[uu];
      }
      const uint4 *src = reinterpret_cast<const uint4 *>(phi + size_t(k0 + t) * (kD * kG));
#pragma unroll
      for (int m = 0; m < NB; ++m) rb[m] = src[tid + NT * m];
    };
    auto stash = [&](int buf) {
      T *a = sA + buf * kA;
      T *b = sB + buf * kB;
#pragma unroll
      for (int m = 0; m < NA; ++m) {
        const int u = tid + NT * m, ww = u / UA, e0 = (u % UA) * E;
        lds_store_unit<T>(&a[(32 * ww + e0 / kD) * LDA_S + e0 % kD], ra[m]);
      }
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const int e0 = (tid + NT * m) * E;
        lds_store_unit<T>(&b[(e0 / kG) * LDB_S + e0 % kG], rb[m]);
      }
    };
    if (n_list > 0) {
      fetch(0);
      stash(0);
    }
    __syncthreads();
    for (int e = 0; e < n_list; ++e) {
      const int buf = e & 1;
      const int mask = s_list[e] >> 16;
      if (e + 1 < n_list) fetch(e + 1);
      if ((mask >> w) & 1) {
        const T *a = sA + buf * kA;
        const T *b = sB + buf * kB;
#pragma unroll 2
        for (int kk = 0; kk < 8; ++kk) {
          const int kc = 4 * kk + (l >> 4);
          const T a0 = a[(32 * w + (l & 15)) * LDA_S + kc];
          const T a1 = a[(32 * w + 16 + (l & 15)) * LDA_S + kc];
#pragma unroll
          for (int tj = 0; tj < 8; ++tj) {
            const T bv = b[kc * LDB_S + 16 * tj + (l & 15)];
            acc[0][tj] = M::mma(a0, bv, acc[0][tj]);
            acc[1][tj] = M::mma(a1, bv, acc[1][tj]);
          }
        }
      }
      if (e + 1 < n_list) stash(buf ^ 1);
      __syncthreads();
    }

    // ---- epilogue: rho_i += sum_mu Phi_mu,i X_mu,i and grad rho_i += 2 sum_mu grad Phi_mu,i X_mu,i
    // over the AOs of each output tile; X goes through LDS two tiles at a time, then one thread per
    // (tile, point) evaluates the tile's shells once
    for (int round = 0; round < 2; ++round) {
      if ((w >> 1) == round && has_w) {
        T *Xw = Xs + (w & 1) * (kD * kG);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 8; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v) Xw[(16 * ti + M::row(v, l)) * kG + 16 * tj + (l & 15)] = acc[ti][tj][v];
      }
      __syncthreads();
      const int slot = 4 * c + 2 * round + half;
      if (slot < np) {
        const T *Xw = Xs + half * (kD * kG);
        double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        if (GGA) {
          for_tile_aos<true>(A.B, s_p[slot], px, py, pz, [&](int a, double v, double gx, double gy, double gz) {
            const double X = double(Xw[a * kG + j]);
            s0 += v * X;
            sx += gx * X;
            sy += gy * X;
            sz += gz * X;
          });
        } else {
          const T *ph = phi + size_t(k0 + slot) * (kD * kG) + j;
          for (int a = 0; a < kD; ++a) s0 += double(ph[a * kG]) * double(Xw[a * kG + j]);
        }
        s_acc[half][0][j] += s0;
        s_acc[half][1][j] += 2.0 * sx;
        s_acc[half][2][j] += 2.0 * sy;
        s_acc[half][3][j] += 2.0 * sz;
      }
      __syncthreads();
    }
  }

  // ---- functional, E_xc partial, rho out; then the Z coefficients
  if (tid < kG) {
    const int64_t ip = r * kG + tid;
    const double rho = s_acc[0][0][tid] + s_acc[1][0][tid];
    const double gx = s_acc[0][1][tid] + s_acc[1][1][tid], gy = s_acc[0][2][tid] + s_acc[1][2][tid],
                 gz = s_acc[0][3][tid] + s_acc[1][3][tid];
    const double sigma = gx * gx + gy * gy + gz * gz;
    const Xc f = xc_eval(A.xc, rho, sigma, A.rho_cut);
    const double wgt = A.g.w[ip];
    s_red[tid] = wgt * f.f;
    const int64_t o = A.g.orig[ip];
    if (A.rho_out && o >= 0) A.rho_out[o] = rho;
    s_acc[0][0][tid] = 0.5 * wgt * f.vr;
    s_acc[0][1][tid] = 2.0 * wgt * f.vs * gx;
    s_acc[0][2][tid] = 2.0 * wgt * f.vs * gy;
    s_acc[0][3][tid] = 2.0 * wgt * f.vs * gz;
  }
  __syncthreads();
  for (int s = kG / 2; s > 0; s >>= 1) {
    if (tid < s) s_red[tid] += s_red[tid + s];
    __syncthreads();
  }
  if (tid == 0) A.eblk[r] = s_red[0];
  // executed X pairs of this block (thread-private partial counts)
  {
    double pd = double(pairs);
    pd = wave_sum(pd);
    if (l == 0 && pd > 0) atomicAdd(&A.counters[0], (unsigned long long)(pd + 0.5));
  }
  if (!A.want_z) return;

  // ---- Z_{mu i} = w (v_rho Phi / 2 + 2 v_sigma grad rho . grad Phi) on the retained tiles of r
  T *zws = static_cast<T *>(A.zws);
  __syncthreads();
  const double c0 = s_acc[0][0][j], c1x = s_acc[0][1][j], c1y = s_acc[0][2][j], c1z = s_acc[0][3][j];
  for (int tb = 0; tb < np; tb += 2) {
    const int t = tb + half;
    double zm = 0.0;
    if (t < np) {
      const int64_t k = k0 + t;
      T *out = zws + size_t(k) * (kD * kG) + j;
      if (GGA) {
        const int p = s_p[t];
        const int nvalid = min(kD, A.B.n_ao - p * kD);
        for (int a = nvalid; a < kD; ++a) out[a * kG] = T(0);
        for_tile_aos<true>(A.B, p, px, py, pz, [&](int a, double v, double gx, double gy, double gz) {
          const double zz = c0 * v + c1x * gx + c1y * gy + c1z * gz;
          const T zt = T(zz);
          out[a * kG] = zt;
          zm = fmax(zm, fabs(double(zt)));
        });
      } else {
        const T *in = phi + size_t(k) * (kD * kG) + j;
        for (int a = 0; a < kD; ++a) {
          const T zt = T(c0 * double(in[a * kG]));
          out[a * kG] = zt;
          zm = fmax(zm, fabs(double(zt)));
        }
      }
    }
    zm = wave_max(zm);
    if (l == 0) s_red[w] = zm;
    __syncthreads();
    if (t < np && j == 0) A.zmax[k0 + t] = fmax(s_red[2 * half], s_red[2 * half + 1]);
    __syncthreads();
  }
}

struct VArgs {
  StructDev st;
  const VItem *items;
  int64_t n_items;
  int n_tiles;
  const void *phi;
  const void *zws;
  const double *zmax;
  double *vpart;
  unsigned long long *counters;
  double t_b, t_d;
  int upper_only;   // LDA: only tiles p <= q are formed (Vxc is mirrored)
};

// One workgroup per (row chunk pc, column chunk qc, segment of grid blocks).  Wave w owns AO tile
// 4pc + w (32 rows); columns are the 128 AOs of tiles 4qc .. 4qc+3.
template <class T>
__global__ __launch_bounds__(NT, 1) void k_vgemm(VArgs A) {
  typedef Mma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int E = Units<T>::E;
  const int64_t item = xcd_remap(blockIdx.x, A.n_items);
  if (item >= A.n_items) return;
  const VItem it = A.items[item];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int n_tiles = A.n_tiles;
  const T *phi = static_cast<const T *>(A.phi);
  const T *zws = static_cast<const T *>(A.zws);

  constexpr int kS = 128 * LDA_S;                 // one A or B stage
  __shared__ __align__(16) T sA[2 * kS];
  __shared__ __align__(16) T sB[2 * kS];
  __shared__ int s_r[NT];
  __shared__ int s_m[NT];
  __shared__ int s_k[NT * 8];   // positions within S_r of the 4 row tiles and 4 column tiles
  __shared__ int s_w[4];

  acc_t acc[2][8];
  double dacc[2][8][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) {
      acc[ti][tj] = acc_t{};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] = 0.0;
    }
  unsigned long long pairs = 0;

  for (int base = it.r0; base < it.r1; base += NT) {
    const int r = base + tid;
    int mask = 0;
    int kp[4] = {-1, -1, -1, -1}, kq[4] = {-1, -1, -1, -1};
    if (r < it.r1) {
      const int64_t bo = A.st.blk_off[r];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = 4 * it.pc + u, q = 4 * it.qc + u;
        kp[u] = (p < n_tiles) ? A.st.idx_map[size_t(r) * n_tiles + p] : -1;
        kq[u] = (q < n_tiles) ? A.st.idx_map[size_t(r) * n_tiles + q] : -1;
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (kq[jj] < 0) continue;
        const double zq = A.zmax[bo + kq[jj]];
        if (!(zq >= A.t_b)) continue;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          if (A.upper_only && it.pc == it.qc && ww > jj) continue;
          if (kp[ww] >= 0 && A.st.bphi[bo + kp[ww]] * zq >= A.t_d) mask |= 1 << (4 * ww + jj);
        }
      }
    }
    int tot;
    const int pos = block_scan(mask != 0, s_w, &tot);
    if (mask) {
      s_r[pos] = r;
      s_m[pos] = mask;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s_k[pos * 8 + u] = kp[u];
        s_k[pos * 8 + 4 + u] = kq[u];
      }
      pairs += __popc(mask);
    }
    __syncthreads();
    // stages s = 4 e + sub: entry e of the compacted list, points 32 sub .. 32 sub + 31
    constexpr int UR = kD / E;          // units per 32-element row slice
    constexpr int UT = kD * UR;         // units per 32 x 32 slab
    constexpr int NU = 8 * UT / NT;     // units per thread (4 A slabs + 4 B slabs)
    uint4 rv[NU];
    int rmask = 0;                      // which units of this thread were fetched
    auto fetch = [&](int st) {
      const int e = st >> 2, sub = st & 3;
      const int m = s_m[e];
      const int64_t bo = A.st.blk_off[s_r[e]];
      rmask = 0;
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        const int u = tid + NT * k, which = u / UT, uu = u % UT;
        const int i = uu / UR, j0 = (uu % UR) * E;
        // a row tile is needed if any of its pairs runs, a column tile likewise
        const bool need = (which < 4) ? ((m >> (4 * which)) & 15) != 0 : ((m >> (which - 4)) & 0x1111) != 0;
        const int kk = s_k[e * 8 + which];
        if (need && kk >= 0) {
          const T *src = ((which < 4) ? phi : zws) + size_t(bo + kk) * (kD * kG) + i * kG + 32 * sub + j0;
          rv[k] = *reinterpret_cast<const uint4 *>(src);
          rmask |= 1 << k;
        }
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        if (!((rmask >> k) & 1)) continue;
        const int u = tid + NT * k, which = u / UT, uu = u % UT;
        const int i = uu / UR, j0 = (uu % UR) * E;
        T *dst = (which < 4) ? &sA[buf * kS + (32 * which + i) * LDA_S + j0]
                             : &sB[buf * kS + (32 * (which - 4) + i) * LDA_S + j0];
        lds_store_unit<T>(dst, rv[k]);
      }
    };
    const int nst = 4 * tot;
    if (nst > 0) {
      fetch(0);
      stash(0);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      const int wm = (s_m[st >> 2] >> (4 * w)) & 15;
      if (st + 1 < nst) fetch(st + 1);
      if (wm) {
        const T *a = sA + buf * kS;
        const T *b = sB + buf * kS;
#pragma unroll 2
        for (int kk = 0; kk < 8; ++kk) {
          const int kc = 4 * kk + (l >> 4);
          const T a0 = a[(32 * w + (l & 15)) * LDA_S + kc];
          const T a1 = a[(32 * w + 16 + (l & 15)) * LDA_S + kc];
#pragma unroll
          for (int tj = 0; tj < 8; ++tj) {
            if ((wm >> (tj >> 1)) & 1) {
              const T bv = b[(16 * tj + (l & 15)) * LDA_S + kc];
              acc[0][tj] = M::mma(a0, bv, acc[0][tj]);
              acc[1][tj] = M::mma(a1, bv, acc[1][tj]);
            }
          }
        }
        if (sizeof(T) == 4) {
          // FP32 accumulation spans one 32-point slab; the running sum over slabs and grid blocks
          // is FP64
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 8; ++tj) {
#pragma unroll
              for (int v = 0; v < 4; ++v) dacc[ti][tj][v] += double(acc[ti][tj][v]);
              acc[ti][tj] = acc_t{};
            }
        }
      }
      if (st + 1 < nst) stash(buf ^ 1);
      __syncthreads();
    }
    __syncthreads();
  }
  double *out = A.vpart + size_t(item) * (128 * 128);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * w + 16 * ti + M::row(v, l), col = 16 * tj + (l & 15);
        out[row * 128 + col] = dacc[ti][tj][v] + double(acc[ti][tj][v]);
      }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[1], (unsigned long long)(pd + 0.5));
}

__global__ __launch_bounds__(NT) void k_vreduce(const int *pair_ptr, const int *pair_items, const int *pair_pq,
                                               const double *__restrict__ vpart, double *__restrict__ mfull, int ld) {
  const int pr = blockIdx.x;
  const int e = blockIdx.y * NT + threadIdx.x;  // 0 .. 16383
  const int i = e >> 7, j = e & 127;
  double s = 0.0;
  for (int k = pair_ptr[pr]; k < pair_ptr[pr + 1]; ++k) s += vpart[size_t(pair_items[k]) * 16384 + e];
  const int pc = pair_pq[2 * pr], qc = pair_pq[2 * pr + 1];
  mfull[size_t(128 * pc + i) * ld + 128 * qc + j] = s;
}

__global__ __launch_bounds__(NT) void k_vsym(const double *__restrict__ mfull, int ld, const int *__restrict__ perm,
                                            int n_ao, int gga, double *__restrict__ vxc) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= n_ao) return;
  const double mij = mfull[size_t(i) * ld + j], mji = mfull[size_t(j) * ld + i];
  double v;
  if (gga) {
    v = mij + mji;
  } else {
    const int p = i / kD, q = j / kD;
    v = (p < q) ? 2.0 * mij : (p > q ? 2.0 * mji : mij + mji);
  }
  vxc[size_t(perm[i]) * n_ao + perm[j]] = v;
}

__global__ __launch_bounds__(NT) void k_esum(const double *__restrict__ eblk, int64_t n, double *exc) {
  __shared__ double s[NT];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) a += eblk[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) exc[0] = s[0];
}

template <class T>
hipError_t eval_typed(const Plan &P, const double *D, double *rho, double *exc, double *vxc, hipStream_t s,
                      hipEvent_t *ev) {
  const EvalDev &E = P.ev;
  const int nt = P.n_tiles;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  };
  mark(0);
  k_reset<<<1, 64, 0, s>>>(E.counters);
  k_dprep<T><<<nt * nt, NT, 0, s>>>(D, P.ao_perm_d, P.n_ao, nt, static_cast<T *>(E.Dt), E.amax, E.counters);
  mark(1);
  if (P.n_ret > 0) k_basis<T><<<P.n_ret, kG, 0, s>>>(P.basis, P.grid, P.st, static_cast<T *>(E.phi));
  mark(2);
  XArgs xa;
  xa.B = P.basis;
  xa.g = P.grid;
  xa.st = P.st;
  xa.Dt = E.Dt;
  xa.amax = E.amax;
  xa.phi = E.phi;
  xa.zws = E.zws;
  xa.zmax = E.zmax;
  xa.eblk = E.eblk;
  xa.rho_out = rho;
  xa.counters = E.counters;
  xa.t_b = P.opts.t_b;
  xa.t_d = P.opts.t_d;
  xa.rho_cut = P.opts.rho_cut;
  xa.xc = P.opts.xc;
  xa.want_z = vxc != nullptr;
  const int64_t gx = 8 * ((P.n_blocks + 7) / 8);
  if (P.gga)
    k_xtask<T, true><<<gx, NT, 0, s>>>(xa);
  else
    k_xtask<T, false><<<gx, NT, 0, s>>>(xa);
  mark(3);
  if (!vxc) mark(4);
  if (vxc) {
    VArgs va;
    va.st = P.st;
    va.items = P.items;
    va.n_items = int64_t(P.items_h.size());
    va.n_tiles = nt;
    va.phi = E.phi;
    va.zws = E.zws;
    va.zmax = E.zmax;
    va.vpart = E.vpart;
    va.counters = E.counters;
    va.t_b = P.opts.t_b;
    va.t_d = P.opts.t_d;
    va.upper_only = P.gga ? 0 : 1;
    if (va.n_items > 0) k_vgemm<T><<<8 * ((va.n_items + 7) / 8), NT, 0, s>>>(va);
    mark(4);
    const int ld = P.n_chunks * 128;
    k_vreduce<<<dim3(P.n_pairs, 64), NT, 0, s>>>(P.pair_ptr, P.pair_items, P.pair_pq, E.vpart, E.mfull, ld);
    k_vsym<<<dim3((P.n_ao + NT - 1) / NT, P.n_ao), NT, 0, s>>>(E.mfull, ld, P.ao_perm_d, P.n_ao, P.gga ? 1 : 0, vxc);
  }
  k_esum<<<1, NT, 0, s>>>(E.eblk, P.n_blocks, exc);
  mark(5);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_screen(const BasisDev &b, const GridDev &g, const int *cand_p, const int64_t *cand_r,
                         int64_t n_cand, bool gga, double *out_b, double *out_g, hipStream_t s) {
  if (n_cand <= 0) return hipSuccess;
  k_screen<<<n_cand, kG, 0, s>>>(b, g, cand_p, cand_r, n_cand, gga ? 1 : 0, out_b, out_g);
  return hipGetLastError();
}

hipError_t launch_eval(const Plan &P, const double *D, double *rho, double *exc, double *vxc, hipStream_t s,
                       hipEvent_t *ev) {
  if (P.opts.prec == KLDI_PREC_FP64) return eval_typed<double>(P, D, rho, exc, vxc, s, ev);
  return eval_typed<float>(P, D, rho, exc, vxc, s, ev);
}

}  // namespace kldi
