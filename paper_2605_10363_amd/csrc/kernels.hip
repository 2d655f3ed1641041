// HIP kernels of libkldi for gfx950 (MI355X): block-filtered EXC integration.
//
// Per evaluation (one stream, no host synchronisation):
//   k_reset    clear the executed-pair counters
//   k_dprep    D (caller order, FP64) -> internal AO order, 32x32 tiles, working precision; block
//              summaries a_pq = max|D_pq| (eq. block_summary_A); non-finite check
//   k_basis    Phi on the retained (tile, grid block) pairs only (eq. phi_def)
//   k_xgemm    one workgroup per (grid block r, chunk of 4 output tiles p of S_r): the executable q
//              are selected by a_pq * b_qr >= t_d (eq. block_pair_filter) and compacted by prefix
//              sum (Appendix D); X_pr = sum_q D_pq Phi_qr on MFMA with LDS-staged tiles, accumulated
//              in registers before the epilogue (Sec. III-C.2); the chunk's rho / grad rho partials
//   k_xfunc    one workgroup per grid block: fixed-order FP64 rho, the functional, E_xc partial
//   k_zform    Z on every retained tile with its max-abs summary
//   k_vgemm    one workgroup per (row chunk, column chunk, segment of grid blocks): executable grid
//              blocks selected by b_pr * z_qr >= t_d and compacted; M_pq = sum_r Phi_pr Z_qr^T on MFMA
//   k_vreduce  FP64 sum of the segment partials in fixed order
//   k_vsym     Vxc = M + M^T (GGA) or mirrored 2M (LDA), back to the caller's AO order
//   k_esum     E_xc as a fixed-order FP64 sum of per-block partials
#include "device.h"

namespace kldi {
namespace {
using namespace dev;

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
__global__ __launch_bounds__(kG) void k_basis(BasisDev B, GridDev g, StructDev st, int64_t ret0, T *__restrict__ phi) {
  const int64_t k = ret0 + blockIdx.x;     // retained tile; the workspace holds the chunk from ret0
  const int p = st.ret_p[k];
  const int64_t ip = int64_t(st.ret_r[k]) * kG + threadIdx.x;
  const double x = g.x[ip], y = g.y[ip], z = g.z[ip];
  T *out = phi + size_t(blockIdx.x) * (kD * kG) + threadIdx.x;
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
  const int *xit_r;        // [n_items] grid block of each X work item
  const int *xit_c;        // [n_items] chunk (4 consecutive entries of S_r) of each item
  int64_t item0, n_items;  // the items of this launch: item0 .. item0 + n_items - 1
  int64_t ret0;            // first retained tile held by the Phi workspace
  const void *Dt;
  const double *amax;
  const void *phi;
  double *part;            // [n_items][4][kG] rho, grad rho partial sums, indexed from item0
  unsigned long long *counters;
  double t_b, t_d;
};

constexpr int NTX = 512;   // threads per X workgroup: 8 waves, each 32 rows x 64 points

// One workgroup per (grid block r, chunk c of 4 retained output tiles): X_pr = sum_q D_pq Phi_qr for
// the 4 tiles p = S_r[4c .. 4c+3], then the chunk's contribution to rho and grad rho.  Wave w owns
// tile 4c + (w & 3) and points 64 (w >> 2) .. 64 (w >> 2) + 63.  The chunks of one block are
// consecutive work items and run side by side on one XCD, sharing the block's Phi tiles in L2.
// FP32 operands: MFMA accumulation spans one 32-AO K tile, the running sum is FP64.
template <class T, bool GGA>
__global__ __launch_bounds__(NTX, 2) void k_xgemm(XArgs A) {
  typedef Mma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int E = Units<T>::E;
  constexpr int STAGES = (sizeof(T) == 4) ? 2 : 1;   // LDS stages of the K loop
  const int64_t il = xcd_remap(blockIdx.x, A.n_items);
  if (il >= A.n_items) return;
  const int64_t it = A.item0 + il;
  const int64_t r = A.xit_r[it];
  const int c = A.xit_c[it];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int u = w & 3, h = w >> 2;
  const int n_tiles = A.B.n_tiles;
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  const T *Dt = static_cast<const T *>(A.Dt);
  const T *phi = static_cast<const T *>(A.phi) - size_t(A.ret0) * (kD * kG);   // indexed by retained tile

  constexpr int kA = 128 * LDA_S, kB = 32 * LDB_S;
  constexpr int kStageBytes = STAGES * (kA + kB) * int(sizeof(T));
  static_assert(kStageBytes >= 2 * kD * kG * 8, "two FP64 X tiles must fit the staging area");
  __shared__ __align__(16) unsigned char s_raw[kStageBytes];
  T *sA = reinterpret_cast<T *>(s_raw);                 // [STAGES][kA]
  T *sB = sA + STAGES * kA;                              // [STAGES][kB]
  double *Xs = reinterpret_cast<double *>(s_raw);        // [2][32][kG] in the epilogue
  __shared__ int s_p[kMaxNp];
  __shared__ int s_list[kMaxNp];
  __shared__ int s_w[8];
  __shared__ double s_acc[2][4][kG];

  for (int t = tid; t < np; t += NTX) s_p[t] = A.st.ret_p[k0 + t];
  for (int e = tid; e < 8 * kG; e += NTX) (&s_acc[0][0][0])[e] = 0.0;
  __syncthreads();

  // ---- executable pairs of this chunk (eq. block_pair_filter), compacted by an exclusive prefix
  // sum over the workgroup (Appendix D); np <= 512 = one candidate per thread
  unsigned long long pairs = 0;
  int n_list;
  {
    const int t = tid;
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
    const unsigned long long bal = __ballot(mask != 0);
    const int before = __popcll(bal & ((1ull << l) - 1ull));
    if (l == 0) s_w[w] = __popcll(bal);
    __syncthreads();
    int pos = before, tot = 0;
    for (int i = 0; i < 8; ++i) {
      pos += (i < w) ? s_w[i] : 0;
      tot += s_w[i];
    }
    if (mask) {
      s_list[pos] = t | (mask << 16);
      pairs += __popc(mask);
    }
    n_list = tot;
  }
  __syncthreads();

  // ---- X = sum over executable q of D_pq Phi_qr (MFMA).  The tiles of step e+1 are fetched into
  // registers while step e multiplies out of LDS.
  acc_t acc[2][4];
  double dacc[2][4][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      acc[ti][tj] = acc_t{};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] = 0.0;
    }
  const bool has_u = 4 * c + u < np;
  constexpr int UA = (kD * kD) / E;   // 16-byte units per D tile
  constexpr int UB = (kD * kG) / E;   // units per Phi tile
  constexpr int NA = 4 * UA / NTX, NB = UB / NTX;
  uint4 ra[NA], rb[NB];
  auto fetch = [&](int e) {
    const int t = s_list[e] & 0xffff;
    const int q = s_p[t];
#pragma unroll
    for (int m = 0; m < NA; ++m) {
      const int un = tid + NTX * m, ww = un / UA, uu = un % UA;
      ra[m] = make_uint4(0, 0, 0, 0);
      if (4 * c + ww < np)
        ra[m] = reinterpret_cast<const uint4 *>(Dt + (size_t(s_p[4 * c + ww]) * n_tiles + q) * (kD * kD))[uu];
    }
    const uint4 *src = reinterpret_cast<const uint4 *>(phi + size_t(k0 + t) * (kD * kG));
#pragma unroll
    for (int m = 0; m < NB; ++m) rb[m] = src[tid + NTX * m];
  };
  auto stash = [&](int buf) {
    T *a = sA + buf * kA;
    T *b = sB + buf * kB;
#pragma unroll
    for (int m = 0; m < NA; ++m) {
      const int un = tid + NTX * m, ww = un / UA, e0 = (un % UA) * E;
      lds_store_unit<T>(&a[(32 * ww + e0 / kD) * LDA_S + e0 % kD], ra[m]);
    }
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const int e0 = (tid + NTX * m) * E;
      lds_store_unit<T>(&b[(e0 / kG) * LDB_S + e0 % kG], rb[m]);
    }
  };
  if (n_list > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int e = 0; e < n_list; ++e) {
    const int buf = (STAGES == 2) ? (e & 1) : 0;
    const int mask = s_list[e] >> 16;
    if (e + 1 < n_list) fetch(e + 1);
    if ((mask >> u) & 1) {
      const T *a = sA + buf * kA;
      const T *b = sB + buf * kB;
#pragma unroll 2
      for (int kk = 0; kk < 8; ++kk) {
        const int kc = 4 * kk + (l >> 4);
        const T a0 = a[(32 * u + (l & 15)) * LDA_S + kc];
        const T a1 = a[(32 * u + 16 + (l & 15)) * LDA_S + kc];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
          const T bv = b[kc * LDB_S + 64 * h + 16 * tj + (l & 15)];
          acc[0][tj] = M::mma(a0, bv, acc[0][tj]);
          acc[1][tj] = M::mma(a1, bv, acc[1][tj]);
        }
      }
      if (sizeof(T) == 4) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
            for (int v = 0; v < 4; ++v) dacc[ti][tj][v] += double(acc[ti][tj][v]);
            acc[ti][tj] = acc_t{};
          }
      }
    }
    if (STAGES == 1) {
      __syncthreads();
      if (e + 1 < n_list) stash(0);
    } else if (e + 1 < n_list) {
      stash(buf ^ 1);
    }
    __syncthreads();
  }

  // ---- epilogue: rho_i += sum_mu Phi_mu,i X_mu,i and grad rho_i += 2 sum_mu grad Phi_mu,i X_mu,i over
  // the AOs of the chunk's tiles.  X (FP64) goes through LDS two tiles at a time; then one thread per
  // (tile, point) evaluates the tile's shells once.
  const int slot_h = (tid >> 7) & 1, j = tid & (kG - 1);
  const bool worker = tid < 2 * kG;
  double px = 0, py = 0, pz = 0;
  if (GGA && worker) {
    const int64_t ip = r * kG + j;
    px = A.g.x[ip];
    py = A.g.y[ip];
    pz = A.g.z[ip];
  }
  for (int round = 0; round < 2; ++round) {
    if ((u >> 1) == round && has_u) {
      double *Xw = Xs + (u & 1) * (kD * kG);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            Xw[(16 * ti + M::row(v, l)) * kG + 64 * h + 16 * tj + (l & 15)] = dacc[ti][tj][v] + double(acc[ti][tj][v]);
    }
    __syncthreads();
    const int slot = 4 * c + 2 * round + slot_h;
    if (worker && slot < np) {
      const double *Xw = Xs + slot_h * (kD * kG);
      double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
      if (GGA) {
        for_tile_aos<true>(A.B, s_p[slot], px, py, pz, [&](int a, double v, double gx, double gy, double gz) {
          const double X = Xw[a * kG + j];
          s0 += v * X;
          sx += gx * X;
          sy += gy * X;
          sz += gz * X;
        });
      } else {
        const T *ph = phi + size_t(k0 + slot) * (kD * kG) + j;
        for (int a = 0; a < kD; ++a) s0 += double(ph[a * kG]) * Xw[a * kG + j];
      }
      s_acc[slot_h][0][j] += s0;
      s_acc[slot_h][1][j] += 2.0 * sx;
      s_acc[slot_h][2][j] += 2.0 * sy;
      s_acc[slot_h][3][j] += 2.0 * sz;
    }
    __syncthreads();
  }
  if (tid < kG) {
    double *out = A.part + size_t(il) * (4 * kG);
#pragma unroll
    for (int cp = 0; cp < (GGA ? 4 : 1); ++cp) out[cp * kG + tid] = s_acc[0][cp][tid] + s_acc[1][cp][tid];
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[0], (unsigned long long)(pd + 0.5));
}

// One workgroup per grid block: rho and grad rho as fixed-order FP64 sums over the chunk partials,
// the functional, the block's E_xc partial, rho in caller order, and the Z coefficients.
__global__ __launch_bounds__(kG) void k_xfunc(FArgs A) {
  const int64_t r = A.blk0 + blockIdx.x;
  const int j = threadIdx.x;
  const int64_t ip = r * kG + j;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t it = A.blk_item_off[r]; it < A.blk_item_off[r + 1]; ++it) {
    const double *pp = A.part + size_t(it - A.item0) * (4 * kG) + j;
    s[0] += pp[0];
    if (A.gga) {
      s[1] += pp[kG];
      s[2] += pp[2 * kG];
      s[3] += pp[3 * kG];
    }
  }
  const double sigma = s[1] * s[1] + s[2] * s[2] + s[3] * s[3];
  const Xc f = xc_eval(A.xc, s[0], sigma, A.rho_cut);
  const double wgt = A.g.w[ip];
  const int64_t o = A.g.orig[ip];
  if (A.rho_out && o >= 0) A.rho_out[o] = s[0];
  if (A.sigma_out && o >= 0) A.sigma_out[o] = sigma;
  double *cf = A.coef + size_t(ip) * 4;
  cf[0] = 0.5 * wgt * f.vr;
  cf[1] = 2.0 * wgt * f.vs * s[1];
  cf[2] = 2.0 * wgt * f.vs * s[2];
  cf[3] = 2.0 * wgt * f.vs * s[3];
  __shared__ double s_red[kG];
  s_red[j] = wgt * f.f;
  __syncthreads();
  for (int k = kG / 2; k > 0; k >>= 1) {
    if (j < k) s_red[j] += s_red[j + k];
    __syncthreads();
  }
  if (j == 0) A.eblk[r] = s_red[0];
}

// One workgroup per retained tile (q, r): Z_{mu i} = w_i (v_rho Phi / 2 + 2 v_sigma grad rho . grad Phi)
// and its max-abs summary z_qr.
template <class T, bool GGA>
__global__ __launch_bounds__(kG) void k_zform(BasisDev B, GridDev g, StructDev st, int64_t ret0,
                                             const double *__restrict__ coef, const T *__restrict__ phi,
                                             T *__restrict__ zws, double *__restrict__ zmax) {
  const int64_t k = ret0 + blockIdx.x;
  const int j = threadIdx.x;
  const int p = st.ret_p[k];
  const int64_t ip = int64_t(st.ret_r[k]) * kG + j;
  const double *cf = coef + size_t(ip) * 4;
  const double c0 = cf[0];
  T *out = zws + size_t(blockIdx.x) * (kD * kG) + j;
  double zm = 0.0;
  if (GGA) {
    const double c1x = cf[1], c1y = cf[2], c1z = cf[3];
    const int nvalid = min(kD, B.n_ao - p * kD);
    for (int a = nvalid; a < kD; ++a) out[a * kG] = T(0);
    for_tile_aos<true>(B, p, g.x[ip], g.y[ip], g.z[ip], [&](int a, double v, double gx, double gy, double gz) {
      const T zt = T(c0 * v + c1x * gx + c1y * gy + c1z * gz);
      out[a * kG] = zt;
      zm = fmax(zm, fabs(double(zt)));
    });
  } else {
    const T *in = phi + size_t(blockIdx.x) * (kD * kG) + j;
    for (int a = 0; a < kD; ++a) {
      const T zt = T(c0 * double(in[a * kG]));
      out[a * kG] = zt;
      zm = fmax(zm, fabs(double(zt)));
    }
  }
  __shared__ double s[2];
  zm = wave_max(zm);
  if ((j & 63) == 0) s[j >> 6] = zm;
  __syncthreads();
  if (j == 0) zmax[k] = fmax(s[0], s[1]);
}

struct VMaskArgs {
  StructDev st;
  const int *cinfo;        // [n_blocks * n_chunks]: (first position in S_r) << 4 | retained 4-bit mask
  const int *pair_pq;      // [2 * n_pairs]
  int n_pairs, n_chunks;
  const double *zmax;
  int64_t blk0;            // first block of this launch
  unsigned short *vmask;   // [blocks of the launch * n_pairs]
  double t_b, t_d;
  int upper_only;          // LDA: only tiles p <= q are formed (Vxc is mirrored)
};

// Position in S_r of tile 4c + u, from the chunk info (first position, 4-bit retained mask).
__device__ __forceinline__ int tile_pos(int info, int u) { return (info >> 4) + __popc(info & 15 & ((1 << u) - 1)); }

// One workgroup per grid block r: the executable (p, q) tile pairs of the Vxc product at r
// (eq. block_pair_filter for C = Phi Z^T: (p,r), (q,r) retained, z_qr >= t_b, b_pr z_qr >= t_d), as a
// 16-bit mask per (row chunk, column chunk) pair.
__global__ __launch_bounds__(NT) void k_vmask(VMaskArgs A) {
  const int64_t r = A.blk0 + blockIdx.x;
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  __shared__ double s_b[kMaxNp], s_z[kMaxNp];
  for (int t = threadIdx.x; t < np; t += NT) {
    s_b[t] = A.st.bphi[k0 + t];
    s_z[t] = A.zmax[k0 + t];
  }
  __syncthreads();
  const int *ci = A.cinfo + size_t(r) * A.n_chunks;
  for (int pr = threadIdx.x; pr < A.n_pairs; pr += NT) {
    const int pc = A.pair_pq[2 * pr], qc = A.pair_pq[2 * pr + 1];
    const int ip = ci[pc], iq = ci[qc];
    int mask = 0;
    if ((ip & 15) && (iq & 15)) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (!((iq >> jj) & 1)) continue;
        const double zq = s_z[tile_pos(iq, jj)];
        if (!(zq >= A.t_b)) continue;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          if (!((ip >> ww) & 1)) continue;
          if (A.upper_only && pc == qc && ww > jj) continue;
          if (s_b[tile_pos(ip, ww)] * zq >= A.t_d) mask |= 1 << (4 * ww + jj);
        }
      }
    }
    A.vmask[size_t(blockIdx.x) * A.n_pairs + pr] = (unsigned short)mask;
  }
}

struct VArgs {
  StructDev st;
  const VItem *items;
  int64_t item0, n_items;  // the items of this launch
  int64_t blk0, ret0;      // first block of the vmask slice; first retained tile of the workspaces
  const int *cinfo;
  int n_chunks, n_pairs;
  const unsigned short *vmask;
  const void *phi;
  const void *zws;
  double *vpart;
  int *vflag;              // [n_items] 1 if the item wrote a partial
  unsigned long long *counters;
};

constexpr int NTV = 512;   // threads per Vxc workgroup: 8 waves, each 32 rows x 64 columns

// One workgroup per (row chunk pc, column chunk qc, segment of grid blocks): M_pq = sum_r Phi_pr Z_qr^T
// over the executable grid blocks of the segment, compacted by prefix sum.  Wave w owns AO tile
// 4pc + (w & 3) (32 rows) and the two column tiles 4qc + 2(w >> 2) + {0, 1}.
template <class T>
__global__ __launch_bounds__(NTV, 2) void k_vgemm(VArgs A) {
  typedef Mma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int E = Units<T>::E;
  const int64_t il = xcd_remap(blockIdx.x, A.n_items);
  if (il >= A.n_items) return;
  const int64_t item = A.item0 + il;
  const VItem it = A.items[item];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int u = w & 3, h = w >> 2;
  const T *phi = static_cast<const T *>(A.phi) - size_t(A.ret0) * (kD * kG);   // indexed by retained tile
  const T *zws = static_cast<const T *>(A.zws) - size_t(A.ret0) * (kD * kG);
  const int pr = it.pair;

  constexpr int kS = 128 * LDA_S;  // one A or B stage (4 tiles x 32 rows x 32 points)
  __shared__ __align__(16) T sA[2 * kS];
  __shared__ __align__(16) T sB[2 * kS];
  __shared__ int s_m[NTV];
  __shared__ int s_ip[NTV], s_iq[NTV];
  __shared__ long long s_bo[NTV];
  __shared__ int s_w[8];

  acc_t acc[2][4];
  double dacc[2][4][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      acc[ti][tj] = acc_t{};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] = 0.0;
    }
  unsigned long long pairs = 0;
  int any = 0;

  for (int base = it.r0; base < it.r1; base += NTV) {
    const int r = base + tid;
    int mask = 0;
    if (r < it.r1) mask = A.vmask[size_t(r - A.blk0) * A.n_pairs + pr];
    // exclusive prefix sum over the 8 waves (parallel addressing)
    const unsigned long long bal = __ballot(mask != 0);
    const int before = __popcll(bal & ((1ull << l) - 1ull));
    if (l == 0) s_w[w] = __popcll(bal);
    __syncthreads();
    int pos = before, tot = 0;
    for (int i = 0; i < 8; ++i) {
      pos += (i < w) ? s_w[i] : 0;
      tot += s_w[i];
    }
    if (mask) {
      s_m[pos] = mask;
      s_ip[pos] = A.cinfo[size_t(r) * A.n_chunks + it.pc];
      s_iq[pos] = A.cinfo[size_t(r) * A.n_chunks + it.qc];
      s_bo[pos] = A.st.blk_off[r];
      pairs += __popc(mask);
    }
    __syncthreads();
    any |= tot;

    // stages s = 4 e + sub: entry e of the compacted list, points 32 sub .. 32 sub + 31
    constexpr int UR = kD / E;          // units per 32-element row slice
    constexpr int UT = kD * UR;         // units per 32 x 32 slab
    constexpr int NU = 8 * UT / NTV;    // units per thread (4 A slabs + 4 B slabs)
    uint4 rv[NU];
    int rmask = 0;
    auto fetch = [&](int st) {
      const int e = st >> 2, sub = st & 3;
      const int m = s_m[e], ip = s_ip[e], iq = s_iq[e];
      const int64_t bo = s_bo[e];
      rmask = 0;
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        const int un = tid + NTV * k, which = un / UT, uu = un % UT;
        const int i = uu / UR, j0 = (uu % UR) * E;
        const int slot = which & 3;
        // a row tile is needed if any of its pairs runs, a column tile likewise
        const bool need = (which < 4) ? ((m >> (4 * slot)) & 15) != 0 : ((m >> slot) & 0x1111) != 0;
        if (need) {
          const int pos = tile_pos(which < 4 ? ip : iq, slot);
          const T *src = ((which < 4) ? phi : zws) + size_t(bo + pos) * (kD * kG) + i * kG + 32 * sub + j0;
          rv[k] = *reinterpret_cast<const uint4 *>(src);
          rmask |= 1 << k;
        }
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        if (!((rmask >> k) & 1)) continue;
        const int un = tid + NTV * k, which = un / UT, uu = un % UT;
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
      const int wm = (s_m[st >> 2] >> (4 * u + 2 * h)) & 3;   // this wave's two column tiles
      if (st + 1 < nst) fetch(st + 1);
      if (wm) {
        const T *a = sA + buf * kS;
        const T *b = sB + buf * kS;
#pragma unroll 2
        for (int kk = 0; kk < 8; ++kk) {
          const int kc = 4 * kk + (l >> 4);
          const T a0 = a[(32 * u + (l & 15)) * LDA_S + kc];
          const T a1 = a[(32 * u + 16 + (l & 15)) * LDA_S + kc];
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) {
            if ((wm >> (tj >> 1)) & 1) {
              const T bv = b[(64 * h + 16 * tj + (l & 15)) * LDA_S + kc];
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
            for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
              for (int v = 0; v < 4; ++v) dacc[ti][tj][v] += double(acc[ti][tj][v]);
              acc[ti][tj] = acc_t{};
            }
        }
      }
      if (st + 1 < nst) stash(buf ^ 1);
      __syncthreads();
    }
  }
  if (!any) {
    if (tid == 0) A.vflag[item] = 0;
    return;
  }
  double *out = A.vpart + size_t(item) * (128 * 128);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * u + 16 * ti + M::row(v, l), col = 64 * h + 16 * tj + (l & 15);
        out[row * 128 + col] = dacc[ti][tj][v] + double(acc[ti][tj][v]);
      }
  if (tid == 0) A.vflag[item] = 1;
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[1], (unsigned long long)(pd + 0.5));
}

__global__ __launch_bounds__(NT) void k_vreduce(const int *pair_ptr, const int *pair_items, const int *pair_pq,
                                               const int *__restrict__ vflag, const double *__restrict__ vpart,
                                               double *__restrict__ mfull, int ld) {
  const int pr = blockIdx.x;
  const int e = blockIdx.y * NT + threadIdx.x;  // 0 .. 16383
  const int i = e >> 7, j = e & 127;
  double s = 0.0;
  for (int k = pair_ptr[pr]; k < pair_ptr[pr + 1]; ++k) {
    const int itm = pair_items[k];
    if (vflag[itm]) s += vpart[size_t(itm) * 16384 + e];
  }
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
hipError_t eval_typed(const Plan &P, const double *D, double *rho, double *sigma, double *exc, double *vxc,
                      hipStream_t s, hipEvent_t *ev) {
  const EvalDev &E = P.ev;
  const int nt = P.n_tiles;
  // stage events: per stage when the grid is processed in one chunk; with several chunks the
  // stages interleave and everything between the D preparation and the final sums is one stage
  const bool one = P.chunks_h.size() == 1;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  };
  mark(0);
  k_reset<<<1, 64, 0, s>>>(E.counters);
  k_dprep<T><<<nt * nt, NT, 0, s>>>(D, P.ao_perm_d, P.n_ao, nt, static_cast<T *>(E.Dt), E.amax, E.counters);
  mark(1);
  if (!one) {
    mark(2);
    mark(3);
    mark(4);
  }
  for (const GridChunk &C : P.chunks_h) {
    const int64_t nret = C.ret1 - C.ret0, nblk = C.blk1 - C.blk0, nxit = C.xit1 - C.xit0, nvit = C.vit1 - C.vit0;
    if (nret > 0) k_basis<T><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, static_cast<T *>(E.phi));
    if (one) mark(2);
    XArgs xa;
    xa.B = P.basis;
    xa.g = P.grid;
    xa.st = P.st;
    xa.xit_r = P.xit_r;
    xa.xit_c = P.xit_c;
    xa.item0 = C.xit0;
    xa.n_items = nxit;
    xa.ret0 = C.ret0;
    xa.Dt = E.Dt;
    xa.amax = E.amax;
    xa.phi = E.phi;
    xa.part = E.xpart;
    xa.counters = E.counters;
    xa.t_b = P.opts.t_b;
    xa.t_d = P.opts.t_d;
    if (nxit > 0) {
      const int64_t gx = 8 * ((nxit + 7) / 8);
      if (P.gga)
        k_xgemm<T, true><<<gx, NTX, 0, s>>>(xa);
      else
        k_xgemm<T, false><<<gx, NTX, 0, s>>>(xa);
    }
    if (one) mark(3);
    FArgs fa;
    fa.g = P.grid;
    fa.blk_item_off = P.blk_item_off;
    fa.blk0 = C.blk0;
    fa.item0 = C.xit0;
    fa.part = E.xpart;
    fa.coef = E.coef;
    fa.eblk = E.eblk;
    fa.rho_out = rho;
    fa.sigma_out = sigma;
    fa.counters = E.counters;
    fa.rho_cut = P.opts.rho_cut;
    fa.xc = P.opts.xc;
    fa.gga = P.gga ? 1 : 0;
    if (nblk > 0) {
      if (P.has_mlp)
        mlp_launch_xfunc(fa, P.mlp, nblk, s);
      else
        k_xfunc<<<nblk, kG, 0, s>>>(fa);
    }
    if (vxc && nret > 0) {
      if (P.gga)
        k_zform<T, true><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, static_cast<const T *>(E.phi),
                                             static_cast<T *>(E.zws), E.zmax);
      else
        k_zform<T, false><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, static_cast<const T *>(E.phi),
                                              static_cast<T *>(E.zws), E.zmax);
    }
    if (one) mark(4);
    if (vxc && nblk > 0) {
      VMaskArgs ma;
      ma.st = P.st;
      ma.cinfo = P.cinfo;
      ma.pair_pq = P.pair_pq;
      ma.n_pairs = P.n_pairs;
      ma.n_chunks = P.n_chunks;
      ma.zmax = E.zmax;
      ma.blk0 = C.blk0;
      ma.vmask = E.vmask;
      ma.t_b = P.opts.t_b;
      ma.t_d = P.opts.t_d;
      ma.upper_only = P.gga ? 0 : 1;
      k_vmask<<<nblk, NT, 0, s>>>(ma);
      VArgs va;
      va.st = P.st;
      va.items = P.items;
      va.item0 = C.vit0;
      va.n_items = nvit;
      va.blk0 = C.blk0;
      va.ret0 = C.ret0;
      va.cinfo = P.cinfo;
      va.n_chunks = P.n_chunks;
      va.n_pairs = P.n_pairs;
      va.vmask = E.vmask;
      va.phi = E.phi;
      va.zws = E.zws;
      va.vpart = E.vpart;
      va.vflag = E.vflag;
      va.counters = E.counters;
      if (nvit > 0) k_vgemm<T><<<8 * ((nvit + 7) / 8), NTV, 0, s>>>(va);
    }
  }
  mark(5);
  if (vxc) {
    const int ld = P.n_chunks * 128;
    k_vreduce<<<dim3(P.n_pairs, 64), NT, 0, s>>>(P.pair_ptr, P.pair_items, P.pair_pq, E.vflag, E.vpart, E.mfull, ld);
    k_vsym<<<dim3((P.n_ao + NT - 1) / NT, P.n_ao), NT, 0, s>>>(E.mfull, ld, P.ao_perm_d, P.n_ao, P.gga ? 1 : 0, vxc);
  }
  k_esum<<<1, NT, 0, s>>>(E.eblk, P.n_blocks, exc);
  mark(6);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_screen(const BasisDev &b, const GridDev &g, const int *cand_p, const int64_t *cand_r,
                         int64_t n_cand, bool gga, double *out_b, double *out_g, hipStream_t s) {
  if (n_cand <= 0) return hipSuccess;
  k_screen<<<n_cand, kG, 0, s>>>(b, g, cand_p, cand_r, n_cand, gga ? 1 : 0, out_b, out_g);
  return hipGetLastError();
}

hipError_t launch_eval(const Plan &P, const double *D, double *rho, double *sigma, double *exc, double *vxc,
                       hipStream_t s, hipEvent_t *ev) {
  if (P.opts.prec == KLDI_PREC_FP64) return eval_typed<double>(P, D, rho, sigma, exc, vxc, s, ev);
  return eval_typed<float>(P, D, rho, sigma, exc, vxc, s, ev);
}

}  // namespace kldi
