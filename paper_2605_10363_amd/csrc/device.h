// Device helpers shared by the HIP sources of libkldi: MFMA wrappers, wave reductions, the
// workgroup prefix sum, basis-function evaluation and the exchange-correlation functionals.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kldi_impl.h"

namespace kldi {
namespace dev {

constexpr int NT = 256;          // threads per workgroup (4 waves of 64)
constexpr int kMaxNp = 512;      // retained tiles per grid block handled by the X kernels

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
// Cartesian components in AO order: s; x y z; xx xy xz yy yz zz.  N_rel = sqrt(3) for xy, xz, yz, else 1.
constexpr double kSqrt3 = 1.7320508075688772;

__device__ __forceinline__ void pw4(double d, double *p) {
  p[0] = 1.0;
  p[1] = d;
  p[2] = d * d;
  p[3] = p[2] * d;
}

// The basis tables are never written by a kernel: reading them through the constant address space lets
// a wave-uniform access become a scalar load.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *ro(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// Calls emit(a, value, gx, gy, gz) for every AO a (local row 0..31) of tile p at (x, y, z).
// The shell data come from the packed per-shell records (wide scalar loads, the next shell's issued before
// this shell's arithmetic): the loop waits on memory once per shell instead of once per
// table and primitive.
struct ShRec {
  double v[kShRec];
};
__device__ __forceinline__ ShRec load_shrec(const BasisDev &B, int s) {
  const auto r = ro(B.shrec) + size_t(s) * kShRec;
  ShRec o;
#pragma unroll
  for (int i = 0; i < kShRec; ++i) o.v[i] = r[i];
  return o;
}
// e^(-a r2) of one primitive, or 0 where a r2 >= kExpCut: such a term is below e^-70 (4e-31) of its
// coefficient, under FP64 resolution of every basis value and density the screening and the functional
// act on (the density floor is 1e-14).  The test is per lane, so a point's value does not depend on its
// wave; the exponential is skipped where every lane of the wave is that far from the primitive (tight
// primitives at the distant points of a retained tile).
constexpr double kExpCut = 70.0;
__device__ __forceinline__ double prim_exp(double a, double r2) {
  const double q = a * r2;
  double e = 0.0;
  if (q < kExpCut) e = exp(-q);
  return e;
}
template <bool GRAD, class F>
__device__ __forceinline__ void for_tile_aos(const BasisDev &B, int p, double x, double y, double z, F &&emit) {
  const auto tile_sh = ro(B.tile_sh);
  const auto pexp = ro(B.pexp), pcoef = ro(B.pcoef);
  const int s0 = tile_sh[2 * p], s1 = tile_sh[2 * p + 1];
  const int a_lo = p * kD, a_hi = a_lo + kD;
  ShRec nxt;
  if (s0 < s1) nxt = load_shrec(B, s0);
  for (int s = s0; s < s1; ++s) {
    const ShRec rc = nxt;
    if (s + 1 < s1) nxt = load_shrec(B, s + 1);
    const int32_t *w = reinterpret_cast<const int32_t *>(&rc.v[3]);
    const int l = w[1] & 3, np = w[1] >> 2, ao0 = w[0], pb = w[2];
    const double dx = x - rc.v[0], dy = y - rc.v[1], dz = z - rc.v[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    double R = 0.0, R1 = 0.0;
#pragma unroll
    for (int k = 0; k < kShPrimIn; ++k) {
      if (k >= np) break;
      const double e = rc.v[6 + 2 * k] * prim_exp(rc.v[5 + 2 * k], r2);
      R += e;
      if (GRAD) R1 -= 2.0 * rc.v[5 + 2 * k] * e;
    }
    for (int k = pb + kShPrimIn; k < pb + np; ++k) {
      const double e = pcoef[k] * prim_exp(pexp[k], r2);
      R += e;
      if (GRAD) R1 -= 2.0 * pexp[k] * e;
    }
    // component c of the shell: angular factor A (N_rel included) and its derivatives; value A R,
    // gradient dA R + A (dx, dy, dz) R1, in AO order.
    auto put = [&](int c, double A, double ax, double ay, double az) {
      const int ao = ao0 + c;
      if (ao < a_lo || ao >= a_hi) return;
      double gx = 0, gy = 0, gz = 0;
      if (GRAD) {
        gx = ax * R + A * dx * R1;
        gy = ay * R + A * dy * R1;
        gz = az * R + A * dz * R1;
      }
      emit(ao - a_lo, A * R, gx, gy, gz);
    };
    if (l == 0) {
      put(0, 1.0, 0.0, 0.0, 0.0);
    } else if (l == 1) {
      put(0, dx, 1.0, 0.0, 0.0);
      put(1, dy, 0.0, 1.0, 0.0);
      put(2, dz, 0.0, 0.0, 1.0);
    } else {
      const double r3 = kSqrt3;
      put(0, dx * dx, 2.0 * dx, 0.0, 0.0);
      put(1, r3 * dx * dy, r3 * dy, r3 * dx, 0.0);
      put(2, r3 * dx * dz, r3 * dz, 0.0, r3 * dx);
      put(3, dy * dy, 0.0, 2.0 * dy, 0.0);
      put(4, r3 * dy * dz, 0.0, r3 * dz, r3 * dy);
      put(5, dz * dz, 0.0, 0.0, 2.0 * dz);
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
    const double e = B.pcoef[k] * prim_exp(B.pexp[k], r2);
    R += e;
    R1 -= 2.0 * B.pexp[k] * e;
  }
  const int cp = B.ao_comp[ao];
  const int lx = cp & 3, ly = (cp >> 2) & 3, lz = (cp >> 4) & 3;
  const double nr = ((lx == 1) + (ly == 1) + (lz == 1) == 2) ? kSqrt3 : 1.0;
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

// Value, gradient and second derivatives h = (xx, xy, xz, yy, yz, zz) of one internal AO at (x, y, z);
// zero on padding rows.  With A the monomial (N_rel included), R = sum c e^{-a r^2}, R1 = sum (-2a) c
// e^{-a r^2}, R2 = sum (2a)^2 c e^{-a r^2}:  d_a chi = A_a R + A d_a R1,
// d_a d_b chi = A_ab R + A_a d_b R1 + A_b d_a R1 + A (delta_ab R1 + d_a d_b R2).
// Value, gradient and Hessian (xx xy xz yy yz zz) of the cartesian component with powers cp = lx | ly << 2 |
// lz << 4 (N_rel included) from the shell's radial sums R = sum c e^(-a r2), R1 = sum -2a c e^(-a r2),
// R2 = sum 4a^2 c e^(-a r2) at offset d from its centre.
__device__ __forceinline__ void ao_hess_from_radial(int cp, const double *d, double R, double R1, double R2, double &v,
                                                    double *g, double *h) {
  const int l[3] = {cp & 3, (cp >> 2) & 3, (cp >> 4) & 3};
  const double nr = ((l[0] == 1) + (l[1] == 1) + (l[2] == 1) == 2) ? kSqrt3 : 1.0;
  // t^l and its first two derivatives per axis
  double p0[3], p1[3], p2[3];
  for (int a = 0; a < 3; ++a) {
    const double t = d[a];
    p0[a] = l[a] == 0 ? 1.0 : (l[a] == 1 ? t : t * t);
    p1[a] = l[a] == 0 ? 0.0 : (l[a] == 1 ? 1.0 : 2.0 * t);
    p2[a] = l[a] == 2 ? 2.0 : 0.0;
  }
  const double A = nr * p0[0] * p0[1] * p0[2];
  double Aa[3];
  Aa[0] = nr * p1[0] * p0[1] * p0[2];
  Aa[1] = nr * p0[0] * p1[1] * p0[2];
  Aa[2] = nr * p0[0] * p0[1] * p1[2];
  v = A * R;
  for (int a = 0; a < 3; ++a) g[a] = Aa[a] * R + A * d[a] * R1;
  int k = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b, ++k) {
      double Aab;
      if (a == b)
        Aab = nr * (a == 0 ? p2[0] * p0[1] * p0[2] : (a == 1 ? p0[0] * p2[1] * p0[2] : p0[0] * p0[1] * p2[2]));
      else {
        const double q[3] = {(a == 0 || b == 0) ? p1[0] : p0[0], (a == 1 || b == 1) ? p1[1] : p0[1],
                             (a == 2 || b == 2) ? p1[2] : p0[2]};
        Aab = nr * q[0] * q[1] * q[2];
      }
      h[k] = Aab * R + Aa[a] * d[b] * R1 + Aa[b] * d[a] * R1 + A * ((a == b ? R1 : 0.0) + d[a] * d[b] * R2);
    }
}

__device__ __forceinline__ void eval_ao_hess(const BasisDev &B, int ao, double x, double y, double z, double &v,
                                             double *g, double *h) {
  v = 0.0;
  for (int k = 0; k < 3; ++k) g[k] = 0.0;
  for (int k = 0; k < 6; ++k) h[k] = 0.0;
  const int s = B.ao_shell[ao];
  if (s < 0) return;
  const double d[3] = {x - B.sh_xyz[3 * s], y - B.sh_xyz[3 * s + 1], z - B.sh_xyz[3 * s + 2]};
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double R = 0.0, R1 = 0.0, R2 = 0.0;
  for (int k = B.sh_prim[2 * s]; k < B.sh_prim[2 * s + 1]; ++k) {
    const double a2 = 2.0 * B.pexp[k];
    const double e = B.pcoef[k] * prim_exp(B.pexp[k], r2);
    R += e;
    R1 -= a2 * e;
    R2 += a2 * a2 * e;
  }
  ao_hess_from_radial(B.ao_comp[ao], d, R, R1, R2, v, g, h);
}

// Calls emit(a, value, gradient[3], hessian[6]) for every AO a (local row 0..31) of tile p at (x, y, z),
// as eval_ao_hess computes them (the same arithmetic), with the radial sums formed once per shell from the
// packed shell records.
template <class F>
__device__ __forceinline__ void for_tile_aos_hess(const BasisDev &B, int p, double x, double y, double z, F &&emit) {
  const auto tile_sh = ro(B.tile_sh);
  const auto pexp = ro(B.pexp), pcoef = ro(B.pcoef);
  const auto ao_comp = ro(B.ao_comp);
  const int s0 = tile_sh[2 * p], s1 = tile_sh[2 * p + 1];
  const int a_lo = p * kD, a_hi = a_lo + kD;
  for (int s = s0; s < s1; ++s) {
    const ShRec rc = load_shrec(B, s);
    const int32_t *w = reinterpret_cast<const int32_t *>(&rc.v[3]);
    const int l = w[1] & 3, np = w[1] >> 2, ao0 = w[0], pb = w[2];
    const double d[3] = {x - rc.v[0], y - rc.v[1], z - rc.v[2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double R = 0.0, R1 = 0.0, R2 = 0.0;
#pragma unroll
    for (int k = 0; k < kShPrimIn; ++k) {
      if (k >= np) break;
      const double a2 = 2.0 * rc.v[5 + 2 * k];
      const double e = rc.v[6 + 2 * k] * prim_exp(rc.v[5 + 2 * k], r2);
      R += e;
      R1 -= a2 * e;
      R2 += a2 * a2 * e;
    }
    for (int k = pb + kShPrimIn; k < pb + np; ++k) {
      const double a2 = 2.0 * pexp[k];
      const double e = pcoef[k] * prim_exp(pexp[k], r2);
      R += e;
      R1 -= a2 * e;
      R2 += a2 * a2 * e;
    }
    const int nc = (l + 1) * (l + 2) / 2;
    for (int c = 0; c < nc; ++c) {
      const int ao = ao0 + c;
      if (ao < a_lo || ao >= a_hi) continue;
      double v, g[3], h[6];
      ao_hess_from_radial(ao_comp[ao], d, R, R1, R2, v, g, h);
      emit(ao - a_lo, v, g, h);
    }
  }
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

// Meta-GGA: MVS exchange (Sun, Perdew, Ruzsinszky 2015) with PBE correlation.  alpha = (tau - tau_W) /
// tau_unif, tau_W = sigma / (8 rho), tau_unif = (3/10)(3 pi^2)^(2/3) rho^(5/3);
// F_x = (1 + k0 f(alpha)) / (1 + b s^4)^(1/8), f = (1 - alpha) ((1 + e1 alpha^2)^2 + c1 alpha^4)^(-1/4).
struct Xc4 {
  double f, vr, vs, vt;
};

__device__ __forceinline__ Xc4 xc_mvs_x(double rho, double sigma, double tau) {
  const double cx = 0.73855876638202234, k0 = 0.174, e1 = -1.6665, c1 = 0.7672, b = 0.0233;
  const double ctau = 2.8712340001881915;   // (3/10)(3 pi^2)^(2/3)
  const double r13 = cbrt(rho);
  const double kf = cbrt(29.608813203268074 * rho);
  const double ds2 = 1.0 / (4.0 * kf * kf * rho * rho);
  const double s2 = sigma * ds2;
  const double tu = ctau * rho * r13 * r13;
  const double alpha = (tau - sigma / (8.0 * rho)) / tu;
  const double a2 = alpha * alpha;
  const double g = (1.0 + e1 * a2) * (1.0 + e1 * a2) + c1 * a2 * a2;
  const double dg = 4.0 * e1 * alpha * (1.0 + e1 * a2) + 4.0 * c1 * a2 * alpha;
  const double gq = pow(g, -0.25);
  const double fa = (1.0 - alpha) * gq;
  const double dfa = -gq - 0.25 * (1.0 - alpha) * gq / g * dg;
  const double q = 1.0 + b * s2 * s2;
  const double den = pow(q, 0.125);
  const double num = 1.0 + k0 * fa;
  const double F = num / den;
  const double dF_ds2 = -num * 0.25 * b * s2 / (den * q);
  const double dF_da = k0 * dfa / den;
  const double el = -cx * rho * r13;
  const double da_drho = (sigma / (8.0 * rho * rho)) / tu - (5.0 / 3.0) * alpha / rho;
  const double da_dsigma = -1.0 / (8.0 * rho * tu);
  return Xc4{el * F, -(4.0 / 3.0) * cx * r13 * F + el * (dF_ds2 * (-8.0 / 3.0) * s2 / rho + dF_da * da_drho),
             el * (dF_ds2 * ds2 + dF_da * da_dsigma), el * dF_da / tu};
}

__device__ __forceinline__ Xc4 xc_eval_mgga(int xc, double rho, double sigma, double tau, double rho_cut) {
  if (!(rho > rho_cut)) return Xc4{0.0, 0.0, 0.0, 0.0};
  Xc4 x = xc_mvs_x(rho, sigma, tau);
  if (xc == KLDI_XC_MVS_X) return x;
  const Xc c = xc_pbe_c(rho, sigma);
  return Xc4{x.f + c.f, x.vr + c.vr, x.vs + c.vs, x.vt};
}

__device__ __forceinline__ bool is_mgga(int xc) { return xc == KLDI_XC_MVS || xc == KLDI_XC_MVS_X; }

struct FArgs {
  GridDev g;
  const int64_t *blk_item_off;   // [n_blocks+1] X work items of each block
  int64_t blk0, item0;           // first block of this launch; first X item held by part
  const double *part;
  double *coef;                  // [n_pad][4]: w v_rho / 2, 2 w v_sigma grad rho
  double *eblk;
  const IoDev *io;               // rho / sigma outputs (caller grid order) of the running evaluation
  unsigned long long *counters;  // [3] counts points evaluated by the surrogate
  double rho_cut;
  int xc;
  int gga;
  const double *tpart[3];        // meta-GGA: the X-type partials of D d_a Phi (component 1 + a holds
                                 // 2 sum_mu d_a chi_mu (D d_a Phi)_mu), else NULL
  double *ctau;                  // meta-GGA: [n_pad] w v_tau / 4 per point
};

}  // namespace dev
}  // namespace kldi
