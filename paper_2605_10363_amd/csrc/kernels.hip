// HIP kernels of libkldi for gfx950 (MI355X): block-filtered EXC integration.
//
// A plan holds one molecule or a batch of independent molecules in one index space (tiles, blocks,
// retained tiles and work items numbered consecutively, each belonging to one molecule); every stage
// below is one launch over all molecules.
//
// Per evaluation (one stream, no host synchronisation):
//   k_begin    record the caller buffers of the evaluation, clear the counters and work queues
//   k_dprep    D (caller order, FP64) -> internal AO order, 32x32 tiles, working precision; block
//              summaries a_pq = max|D_pq| (eq. block_summary_A); non-finite check
//   k_basis    Phi on the retained (tile, grid block) pairs only (eq. phi_def)
//   k_xgemm_*  one workgroup per (grid block r, chunk of 4 output tiles p of S_r): the executable q
//              are selected by a_pq * b_qr >= t_d (eq. block_pair_filter) and compacted by prefix
//              sum (Appendix D); X_pr = sum_q D_pq Phi_qr on MFMA with LDS-staged tiles, accumulated
//              in registers before the epilogue (Sec. III-C.2); the chunk's rho / grad rho partials
//              (_f32 / _f64: FP32 / FP64 operands, 4 waves; _bf16: BF16 split operands, 8 waves)
//   k_xfunc    one workgroup per grid block: fixed-order FP64 rho, the functional, E_xc partial
//   k_zform    Z on every retained tile with its max-abs summary
//   k_vgemm_*  one workgroup per (row chunk, column chunk, segment of grid blocks): executable grid
//              blocks selected by b_pr * z_qr >= t_d and compacted; M_pq = sum_r Phi_pr Z_qr^T on MFMA
//              (_f32 / _f64: FP32 / FP64 operands, 4 waves)
//   k_vreduce  FP64 sum of the segment partials in fixed order
//   k_vsym     Vxc = M + M^T (GGA) or mirrored 2M (LDA), back to the caller's AO order
//   k_esum     E_xc of each molecule as a fixed-order FP64 sum of its per-block partials
// The two GEMM kernels run one workgroup per work item, in item order or in per-XCD queue order
// (kldi_schedule).
#include <algorithm>
#include <type_traits>

#include <hip/hip_bf16.h>

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
__global__ __launch_bounds__(NT) void k_begin(IoDev *cell, IoDev io, unsigned long long *counters) {
  if (threadIdx.x == 0) *cell = io;
  if (threadIdx.x < 8) counters[threadIdx.x] = 0ull;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
  __hip_bfloat16 b = __float2bfloat16(x);
  return *reinterpret_cast<unsigned short *>(&b);
}
__device__ __forceinline__ double from_bf16(unsigned short u) {
  return double(__uint_as_float(uint32_t(u) << 16));
}

// Molecule m with off(mol[m]) <= x < off(mol[m + 1]) for an increasing offset field.
template <class F>
__device__ __forceinline__ int find_mol(const MolDev *mol, int n_mol, int64_t x, F &&off) {
  int lo = 0, hi = n_mol - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off(mol[mid]) <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One workgroup per (p, q) tile pair of a molecule.
template <class T>
__global__ __launch_bounds__(NT) void k_dprep(const MolDev *__restrict__ mol, int n_mol, const IoDev *io,
                                             const int *__restrict__ perm, T *__restrict__ Dt,
                                             double *__restrict__ amax, unsigned long long *counters) {
  const int64_t g = blockIdx.x;
  const MolDev mo = mol[find_mol(mol, n_mol, g, [](const MolDev &x) { return x.dt0; })];
  const int loc = int(g - mo.dt0);
  const int p = loc / mo.nt, q = loc % mo.nt, n_ao = mo.n_ao;
  const double *D = io->D + mo.d0;
  const int *pm = perm + size_t(mo.tile0) * kD;
  double m = 0.0;
  int bad = 0;
  for (int e = threadIdx.x; e < kD * kD; e += NT) {
    const int i = p * kD + e / kD, j = q * kD + e % kD;
    double v = 0.0;
    if (i < n_ao && j < n_ao) v = D[size_t(pm[i]) * n_ao + pm[j]];
    if (!isfinite(v)) bad = 1;
    m = fmax(m, fabs(v));
    Dt[size_t(g) * (kD * kD) + e] = T(v);
  }
  __shared__ double s[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&counters[2], 1ull);
  __syncthreads();
  if (threadIdx.x == 0) amax[g] = fmax(fmax(s[0], s[1]), fmax(s[2], s[3]));
}

// BF16 split plans: the NPC BF16 pieces of each D element, v = v_0 + v_1 (+ v_2), piece k the BF16
// rounding of what pieces 0 .. k-1 leave of v; tile g holds [piece][row i][column k].
__device__ __forceinline__ void split_bf16(double v, int npc, unsigned short *out, size_t stride) {
  double r = v;
  for (int k = 0; k < npc; ++k) {
    const unsigned short b = to_bf16(float(r));
    out[k * stride] = b;
    r -= from_bf16(b);
  }
}

template <int NPC>
__global__ __launch_bounds__(NT) void k_dprep_b(const MolDev *__restrict__ mol, int n_mol, const IoDev *io,
                                               const int *__restrict__ perm, unsigned short *__restrict__ Dt,
                                               double *__restrict__ amax, unsigned long long *counters) {
  const int64_t g = blockIdx.x;
  const MolDev mo = mol[find_mol(mol, n_mol, g, [](const MolDev &x) { return x.dt0; })];
  const int loc = int(g - mo.dt0);
  const int p = loc / mo.nt, q = loc % mo.nt, n_ao = mo.n_ao;
  const double *D = io->D + mo.d0;
  const int *pm = perm + size_t(mo.tile0) * kD;
  double m = 0.0;
  int bad = 0;
  for (int e = threadIdx.x; e < kD * kD; e += NT) {
    const int i = p * kD + e / kD, j = q * kD + e % kD;
    double v = 0.0;
    if (i < n_ao && j < n_ao) v = D[size_t(pm[i]) * n_ao + pm[j]];
    if (!isfinite(v)) bad = 1;
    m = fmax(m, fabs(v));
    split_bf16(v, NPC, Dt + size_t(g) * (NPC * kD * kD) + e, kD * kD);
  }
  __shared__ double s[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&counters[2], 1ull);
  __syncthreads();
  if (threadIdx.x == 0) amax[g] = fmax(fmax(s[0], s[1]), fmax(s[2], s[3]));
}

// FP32 operands also get Phi_lo = bf16(Phi - fl32(Phi)) (phil != NULL): the term the split product of
// the Vxc GEMM adds back.  BF16 split plans also get the NPC BF16 pieces of Phi in phix, per tile
// [piece][unit u][point][8 AOs] (AOs 8u .. 8u + 7 of a point in one 16-byte unit: the X product contracts
// over AOs, and consecutive threads store consecutive units).
template <class T, int NPC>
__global__ __launch_bounds__(kG) void k_basis(BasisDev B, GridDev g, StructDev st, int64_t ret0, T *__restrict__ phi,
                                             unsigned short *__restrict__ phil, unsigned short *__restrict__ phix) {
  const int64_t k = ret0 + blockIdx.x;     // retained tile; the workspace holds the chunk from ret0
  const int p = st.ret_p[k];
  const int j = threadIdx.x;
  const int64_t ip = int64_t(st.ret_r[k]) * kG + j;
  const double x = g.x[ip], y = g.y[ip], z = g.z[ip];
  const size_t o = size_t(blockIdx.x) * (kD * kG) + j;
  T *out = phi + o;
  for (int a = B.tile_nv[p]; a < kD; ++a) out[a * kG] = T(0);
  if constexpr (NPC > 0) {
    // this point's row of each piece, 16 bytes (8 AOs) at a time: the AOs of a tile arrive in
    // increasing order (the same order in every thread), so a unit is stored once its last AO is in;
    // units past the tile's AOs are zero
    unsigned short *px = phix + size_t(blockIdx.x) * (NPC * kG * kD) + size_t(j) * 8;
    uint32_t bw[NPC][4];
    int cu = 0;
    auto clear = [&]() {
#pragma unroll
      for (int c = 0; c < NPC; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) bw[c][q] = 0u;
    };
    auto store = [&](int u) {
#pragma unroll
      for (int c = 0; c < NPC; ++c)
        *reinterpret_cast<uint4 *>(px + c * (kG * kD) + u * (kG * 8)) = make_uint4(bw[c][0], bw[c][1], bw[c][2], bw[c][3]);
    };
    clear();
    unsigned short *lo = phil + o;
    for (int a = B.tile_nv[p]; a < kD; ++a) lo[a * kG] = 0;
    for_tile_aos<false>(B, p, x, y, z, [&](int a, double v, double, double, double) {
      while (cu < (a >> 3)) {
        store(cu);
        clear();
        ++cu;
      }
      const T h = T(v);
      out[a * kG] = h;
      lo[a * kG] = to_bf16(float(v - double(h)));
      const int q = (a & 7) >> 1, sh = 16 * (a & 1);
      double rem = v;
#pragma unroll
      for (int c = 0; c < NPC; ++c) {
        const unsigned short b = to_bf16(float(rem));
        rem -= from_bf16(b);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          if (qq == q) bw[c][qq] |= uint32_t(b) << sh;
      }
    });
    for (; cu < 4; ++cu) {
      store(cu);
      clear();
    }
  } else if (sizeof(T) == 4 && phil) {
    unsigned short *lo = phil + o;
    for (int a = B.tile_nv[p]; a < kD; ++a) lo[a * kG] = 0;
    for_tile_aos<false>(B, p, x, y, z, [&](int a, double v, double, double, double) {
      const T h = T(v);
      out[a * kG] = h;
      lo[a * kG] = to_bf16(float(v - double(h)));
    });
  } else {
    for_tile_aos<false>(B, p, x, y, z, [&](int a, double v, double, double, double) { out[a * kG] = T(v); });
  }
}

// 16-byte unit copies between global memory and LDS rows
// Global -> LDS copies that bypass registers (global_load_lds_dwordx4): lane l of the wave writes its
// 16 bytes at lds_wave + 16 l (measured on gfx950); lds_wave must be the same for the whole wave (it
// goes to M0).  The copies count in vmcnt like vector loads, in issue order; the GEMM loops wait for
// them with an explicit s_waitcnt and then meet at a bare s_barrier (a fence would wait for every copy
// in flight).  Issued from inline assembly: the compiler would otherwise wait for all copies in flight
// before every LDS read it cannot prove disjoint from them.  Its own vmcnt waits stay correct (copies
// issued after one of its loads only make such a wait longer).
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void dma16(const void *src, void *lds_wave) {
  const uint32_t lds = __builtin_amdgcn_readfirstlane(
      static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_void *)lds_wave)));
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds)
               : "memory", "m0");
}
// Swizzle of the 16-byte units of a 128-byte LDS row i (32 rows to a tile slab): unit c of the row is
// stored at c ^ swz(i).  The fragment reads take one unit of each of 16 consecutive rows per 16 lanes;
// under this map the 16 units fall in 16 distinct 16-byte bank groups whether the LDS serves 8 lanes
// over 32 banks or 16 lanes over 64 banks per cycle (c ^ (i & 7) left rows i and i + 8 in one group of
// 64 banks, a two-way conflict on every read).  Rows i and i + 16 share a swizzle, so the reads of the
// two 16-row halves of a slab differ by a constant offset.
__device__ __forceinline__ int swz(int i) { return (i ^ ((i >> 3) & 1)) & 7; }
// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
template <int N>
__device__ __forceinline__ void wait_vm_lds() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}
// s_barrier that the compiler may not move memory accesses across
__device__ __forceinline__ void wg_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Work-item schedules: 8 per-XCD queues of items (host-built, see kldi_schedule); workgroup b runs
// position b / 8 of queue b % 8 -- the dispatcher places workgroup b on XCD b % 8 -- or nothing past
// the end of its queue.  Grid: grid blocks / Vxc segments dealt round-robin over the queues, the Vxc
// queues ordered by decreasing cost (measured: contiguous item ranges per XCD leave most XCDs idle while
// the densest region of the molecule finishes).  Queue: contiguous ranges of about equal estimated cost,
// each ordered by decreasing cost.
struct QArgs {
  const int *order;        // item ids in queue order
  const int64_t *qoff;     // [9] queue boundaries of this launch
};

template <class F>
__device__ __forceinline__ void run_items(const QArgs &q, int64_t item0, F &&run) {
  const int qx = blockIdx.x & 7;
  const int64_t pos = q.qoff[qx] + (blockIdx.x >> 3);
  if (pos < q.qoff[qx + 1]) run(int64_t(q.order[pos]) - item0);
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
  const unsigned short *phil;   // FP32 operands: bf16(Phi - fl32(Phi)), else NULL
  const unsigned short *phix;   // BF16 split plans: the BF16 pieces of Phi, [piece][point][AO] per tile
  double *part;            // [n_items][4][kG] rho, grad rho partial sums, indexed from item0
  unsigned long long *counters;
  double t_b, t_d;
  QArgs q;
};

constexpr int NTX = 512;   // threads per BF16 X workgroup: 8 waves, each 32 rows x 64 points


// BF16 split plans: one workgroup per (grid block r, chunk c of 4 retained output tiles): X_pr =
// sum_q D_pq Phi_qr for the 4 tiles p = S_r[4c .. 4c+3], then the chunk's contribution to rho and grad rho.
// Wave w owns tile 4c + (w & 3) and points 64 (w >> 2) .. 64 (w >> 2) + 63.  The operands are NPC BF16
// pieces each, on BF16 MFMA (Dt holds D's pieces, phix Phi's), accumulated in FP32 per K tile and in
// FP64 beyond; the FP32 Phi serves the epilogue.
template <bool GGA, int NPC>
__global__ __launch_bounds__(NTX, 2) void k_xgemm_bf16(XArgs A) {
  typedef Mma<float> M;
  typedef typename M::acc_t acc_t;
  typedef float T;
  constexpr int kXsBytes = 4 * kD * kG * 8;   // the epilogue's X (FP64, 4 tiles) overlays the staging area
  constexpr int kStageBytes = kXsBytes;
  __shared__ __align__(16) unsigned char s_raw[kStageBytes];
  __shared__ int s_p[kMaxNp];
  __shared__ int s_list[kMaxNp];
  __shared__ int s_q[kMaxNp];      // q of each compacted entry
  __shared__ int s_w[8];
  __shared__ double s_acc[4][4][kG];
  run_items(A.q, A.item0, [&](int64_t il) {
  const int64_t it = A.item0 + il;
  const int64_t r = A.xit_r[it];
  const int c = A.xit_c[it];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int u = w & 3, h = w >> 2;
  const MolDev mo = A.st.mol[A.st.blk_mol[r]];
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  const T *phi = static_cast<const T *>(A.phi) - size_t(A.ret0) * (kD * kG);   // indexed by retained tile
  // (p, q) tile pair of the molecule -> its position in Dt / amax
  auto dtile = [&](int p, int q) { return size_t(mo.dt0) + size_t(p - mo.tile0) * mo.nt + (q - mo.tile0); };
  double *Xs = reinterpret_cast<double *>(s_raw);        // [4][32][kG] in the epilogue

  for (int t = tid; t < np; t += NTX) s_p[t] = A.st.ret_p[k0 + t];
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
          const double a = A.amax[dtile(s_p[4 * c + ww], q)];
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
      s_q[pos] = s_p[t];
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
  {
    // ---- BF16 pieces.  Slot e % 2 holds entry e of the compacted list: the NPC pieces of the 4 D
    // tiles (p_u, q), each [row i][k], then the NPC pieces of Phi_q, each [point][k]; a row is 64
    // bytes, 4 units of 16 bytes, unit c of row i stored at c ^ ((i >> 1) & 3) (the 8 rows a
    // 16-byte LDS read serves at once then fall on distinct banks).  Copies global -> LDS directly,
    // one entry ahead, one barrier per entry.  v_mfma_f32_16x16x32_bf16: lane l supplies row (or
    // point) 16 t + l % 16 at k = 8 (l / 16) .. + 7, one 16-byte read per piece and sub-tile; the
    // products of pieces (a, b) with a + b <= NPC - 1 are added smallest first into the FP32
    // accumulator of the K tile, which is then flushed to the FP64 sums.
    constexpr int kTileB = kD * kD, kPhiB = kG * kD;
    constexpr int kEntB = NPC * (4 * kTileB + kPhiB);     // bf16 elements per entry
    constexpr int kPhiRounds = NPC * kPhiB / 8 / 64 / 4;   // 64-unit copies per Phi wave and entry
    static_assert(2 * kEntB * 2 <= kStageBytes, "ring exceeds the staging area");
    unsigned short *ring = reinterpret_cast<unsigned short *>(s_raw);
    const int ws = __builtin_amdgcn_readfirstlane(w), us = ws & 3;
    const int m16 = l & 15, g = l >> 4;
    const unsigned short *Db = static_cast<const unsigned short *>(A.Dt);
    const unsigned short *Pb = A.phix - size_t(A.ret0) * (NPC * kPhiB);   // indexed by retained tile
    // D tile row of this wave's chunk entry (waves 0-3): an entry past the end of S_r uses entry np - 1
    // (valid memory, never multiplied: its wave has no executable pair)
    const int pa = __builtin_amdgcn_readfirstlane(s_p[min(4 * c + us, np - 1)]);
    const unsigned short *Drow = Db + dtile(pa, mo.tile0) * (NPC * kTileB);
    auto issue = [&](int e) {
      unsigned short *dst = ring + (e & 1) * kEntB;
      if (ws < 4) {
        const int q = __builtin_amdgcn_readfirstlane(s_q[e]);
        const unsigned short *src = Drow + size_t(q - mo.tile0) * (NPC * kTileB);
        dst += ws * (NPC * kTileB);
#pragma unroll
        for (int m = 0; m < 2 * NPC; ++m) {
          const int du = 64 * m + l, pc = du >> 7, i = (du >> 2) & 31, cu = (du & 3) ^ ((i >> 1) & 3);
          dma16(src + pc * kTileB + i * kD + 8 * cu, dst + 512 * m);
        }
      } else {
        const int t = __builtin_amdgcn_readfirstlane(s_list[e] & 0xffff);
        const unsigned short *src = Pb + size_t(k0 + t) * (NPC * kPhiB);
        const int u0 = (ws - 4) * (64 * kPhiRounds);
        dst += NPC * 4 * kTileB;
#pragma unroll
        for (int m = 0; m < kPhiRounds; ++m) {
          const int du = u0 + 64 * m + l, pc = du >> 9, i = (du >> 2) & 127, cu = (du & 3) ^ ((i >> 1) & 3);
          dma16(src + pc * kPhiB + cu * (kG * 8) + i * 8, dst + 8 * (u0 + 64 * m));
        }
      }
    };
    auto rd = [&](const unsigned short *base, int i) {
      return *reinterpret_cast<const bf16x8 *>(base + i * kD + 8 * (g ^ ((i >> 1) & 3)));
    };
    if (n_list > 0) issue(0);
    for (int e = 0; e < n_list; ++e) {
      wait_vm_lds<0>();
      wg_barrier();
      if (e + 1 < n_list) issue(e + 1);
      if ((__builtin_amdgcn_readfirstlane(s_list[e] >> 16) >> us) & 1) {
        const unsigned short *se = ring + (e & 1) * kEntB;
        bf16x8 b[4][NPC];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
          for (int pc = 0; pc < NPC; ++pc) b[tj][pc] = rd(se + NPC * 4 * kTileB + pc * kPhiB, 64 * h + 16 * tj + m16);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          bf16x8 a[NPC];
#pragma unroll
          for (int pc = 0; pc < NPC; ++pc) a[pc] = rd(se + us * (NPC * kTileB) + pc * kTileB, 16 * ti + m16);
          // products by decreasing piece order: (2,0) (1,1) (0,2), then (1,0) (0,1), then (0,0)
#pragma unroll
          for (int ord = NPC - 1; ord >= 0; --ord)
#pragma unroll
            for (int pa_ = ord; pa_ >= 0; --pa_)
#pragma unroll
              for (int tj = 0; tj < 4; ++tj)
                acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pa_], b[tj][ord - pa_], acc[ti][tj], 0, 0, 0);
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
            for (int v = 0; v < 4; ++v) dacc[ti][tj][v] += double(acc[ti][tj][v]);
            acc[ti][tj] = acc_t{};
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: rho_i += sum_mu Phi_mu,i X_mu,i and grad rho_i += 2 sum_mu grad Phi_mu,i X_mu,i over
  // the AOs of the chunk's tiles.  X (FP64) of the 4 tiles goes through LDS; then one thread per (tile,
  // point) evaluates the tile's shells once, in FP64 (a wave shares one tile, so the shell data are
  // scalar loads), and the 4 tiles are summed in a fixed order.
  const int slot_w = tid >> 7, j = tid & (kG - 1);
  if (has_u) {
    double *Xw = Xs + u * (kD * kG);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Xw[(16 * ti + M::row(v, l)) * kG + 64 * h + 16 * tj + (l & 15)] =
              dacc[ti][tj][v] + double(acc[ti][tj][v]);
  }
  __syncthreads();
  {
    const int slot = 4 * c + slot_w;
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    if (slot < np) {
      const double *Xw = Xs + slot_w * (kD * kG);
      if (GGA) {
        const int64_t ip = r * kG + j;
        const int pt = __builtin_amdgcn_readfirstlane(s_p[slot]);
        for_tile_aos<true>(A.B, pt, A.g.x[ip], A.g.y[ip], A.g.z[ip], [&](int a, double v, double gx, double gy,
                                                                          double gz) {
          const double X = Xw[a * kG + j];
          s0 += v * X;
          sx += gx * X;
          sy += gy * X;
          sz += gz * X;
        });
      } else {
        const T *ph = phi + size_t(k0 + slot) * (kD * kG) + j;
        if (sizeof(T) == 4 && A.phil) {
          const unsigned short *pl = A.phil + size_t(k0 + slot - A.ret0) * (kD * kG) + j;
          for (int a = 0; a < kD; ++a) s0 += (double(ph[a * kG]) + from_bf16(pl[a * kG])) * Xw[a * kG + j];
        } else {
          for (int a = 0; a < kD; ++a) s0 += double(ph[a * kG]) * Xw[a * kG + j];
        }
      }
    }
    s_acc[slot_w][0][j] = s0;
    s_acc[slot_w][1][j] = 2.0 * sx;
    s_acc[slot_w][2][j] = 2.0 * sy;
    s_acc[slot_w][3][j] = 2.0 * sz;
  }
  __syncthreads();
  if (tid < kG) {
    double *out = A.part + size_t(il) * (4 * kG);
#pragma unroll
    for (int cp = 0; cp < (GGA ? 4 : 1); ++cp)
      out[cp * kG + tid] = (s_acc[0][cp][tid] + s_acc[2][cp][tid]) + (s_acc[1][cp][tid] + s_acc[3][cp][tid]);
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[0], (unsigned long long)(pd + 0.5));
  });
}

constexpr int NTX4 = 256;   // threads per FP32 X workgroup: 4 waves, wave u owns output tile u (32 rows x 128 points)

// FP32 operands: one workgroup of 4 waves per (grid block r, chunk c of 4 retained output tiles p = S_r[4c ..
// 4c+3]): X_pr = sum_q D_pq Phi_qr over the executable q, then the chunk's contribution to rho and grad rho.
// Its LDS (78 KB: a two-slot ring of one compacted entry each,
// 4 D tiles + one Phi tile, which the epilogue's FP64 X of two tiles overlays) lets two workgroups share
// a CU, so one workgroup's copies, barriers and epilogue overlap the other's MFMAs.  Wave u multiplies
// D_(p_u, q) (32 x 32) by Phi_qr (32 x 128) on v_mfma_f32_16x16x4f32: MFMA step kk takes k = 8 (l / 16) + kk,
// output column c of sub-tile tj is point 64 (tj / 4) + 4 c + tj % 4, so a lane reads its 8 values of a
// row of Phi_q with two 16-byte loads and the 16 lanes of a row read 256 contiguous bytes per load (no
// bank conflicts; 8 contiguous points per lane made every Phi read a two-way conflict).  The FP32 accumulators of sub-tile row ti are added to the FP64 sums once per 32
// values of k (row 0 after step 3, row 1 after step 7 of each entry, so the two rows' flushes alternate
// with MFMAs).
template <bool GGA>
__global__ __launch_bounds__(NTX4, 2) void k_xgemm_f32(XArgs A) {
  typedef Mma<float> M;
  constexpr int kEnt = 4 * kD * kD + kD * kG;   // floats per ring slot (32 KB)
  __shared__ __align__(16) float ring[2 * kEnt];
  __shared__ int s_p[kMaxNp];
  __shared__ int s_list[kMaxNp];
  __shared__ int s_q[kMaxNp];
  __shared__ int s_w[4];
  __shared__ double s_acc[2][4][kG];
  static_assert(2 * kD * kG * sizeof(double) <= sizeof(ring), "epilogue X exceeds the ring");
  run_items(A.q, A.item0, [&](int64_t il) {
  const int64_t it = A.item0 + il;
  const int64_t r = A.xit_r[it];
  const int c = A.xit_c[it];
  const int tid = threadIdx.x, l = tid & 63;
  const int ws = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m16 = l & 15, g = l >> 4;
  const MolDev mo = A.st.mol[A.st.blk_mol[r]];
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  const float *Df = static_cast<const float *>(A.Dt);
  const float *phi = static_cast<const float *>(A.phi) - size_t(A.ret0) * (kD * kG);   // by retained tile
  auto dtile = [&](int p, int q) { return size_t(mo.dt0) + size_t(p - mo.tile0) * mo.nt + (q - mo.tile0); };

  for (int t = tid; t < np; t += NTX4) s_p[t] = A.st.ret_p[k0 + t];
  __syncthreads();

  // ---- executable pairs of this chunk (eq. block_pair_filter), compacted by exclusive prefix sums
  // over the workgroup (Appendix D), NTX4 candidates per round
  unsigned long long pairs = 0;
  int n_list = 0;
  for (int base = 0; base < np; base += NTX4) {
    const int t = base + tid;
    int mask = 0;
    if (t < np) {
      const int q = s_p[t];
      const double bq = A.st.bphi[k0 + t];
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        if (4 * c + ww < np) {
          const double a = A.amax[dtile(s_p[4 * c + ww], q)];
          if (a >= A.t_b && a * bq >= A.t_d) mask |= 1 << ww;
        }
      }
    }
    int tot;
    const int pos = n_list + block_scan(mask != 0, s_w, &tot);
    if (mask) {
      s_list[pos] = t | (mask << 16);
      s_q[pos] = s_p[t];
      pairs += __popc(mask);
    }
    n_list += tot;
  }
  __syncthreads();

  // ---- X_(p_u) r = sum over the compacted q of D_(p_u) q Phi_qr
  f4 acc[2][8];
  double dacc[2][8][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) {
      acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] = 0.0;
    }
  // D tile row of this wave's output tile: a slot past the end of S_r uses entry np - 1 (valid memory,
  // never multiplied: its wave has no executable pair)
  const int pa = __builtin_amdgcn_readfirstlane(s_p[min(4 * c + ws, np - 1)]);
  const float *Drow = Df + dtile(pa, mo.tile0) * (kD * kD);
  // entry e goes to slot e % 2: wave w copies D_(p_w, q) as [row i][k] with the 16-byte units of row i
  // XOR-swizzled (unit c at c ^ swz(i)), and quarter w of Phi_q as [k][point], global -> LDS directly
  auto issue = [&](int e) {
    float *dst = ring + (e & 1) * kEnt;
    const int q = __builtin_amdgcn_readfirstlane(s_q[e]);
    const float *src = Drow + size_t(q - mo.tile0) * (kD * kD);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int tu = 64 * m + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
      dma16(src + i * kD + 4 * cu, dst + ws * (kD * kD) + 256 * m);
    }
    const int t = __builtin_amdgcn_readfirstlane(s_list[e] & 0xffff);
    const float *ps = phi + size_t(k0 + t) * (kD * kG) + 1024 * ws;
#pragma unroll
    for (int m = 0; m < 4; ++m) dma16(ps + 4 * (64 * m + l), dst + 4 * kD * kD + 1024 * ws + 256 * m);
  };
  // the FP32 window of row 0 is steps 4-7 of one computed entry and steps 0-3 of the next, that of row 1
  // steps 0-7 of one entry; a window's first MFMA takes a zero accumulator (no register clearing), and the
  // epilogue adds the window still open
  auto flush = [&](int ti) {
#pragma unroll
    for (int tj = 0; tj < 8; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] += double(acc[ti][tj][v]);
  };
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  if (n_list > 0) issue(0);
  // entry e: wait until this wave's copies of e have landed and its reads of e - 1 are done; after the
  // barrier the slot of e - 1 takes e + 1
  for (int e = 0; e < n_list; ++e) {
    wait_vm_lds<0>();
    wg_barrier();
    if (e + 1 < n_list) issue(e + 1);
    if ((__builtin_amdgcn_readfirstlane(s_list[e] >> 16) >> ws) & 1) {
      const float *se = ring + (e & 1) * kEnt;
      f4 a[2][2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
          a[ti][hh] = *reinterpret_cast<const f4 *>(se + ws * (kD * kD) + (16 * ti + m16) * kD +
                                                    4 * ((2 * g + hh) ^ swz(16 * ti + m16)));
      const float *sb = se + 4 * kD * kD + 4 * m16;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const f4 b0 = *reinterpret_cast<const f4 *>(sb + (8 * g + kk) * kG);
        const f4 b1 = *reinterpret_cast<const f4 *>(sb + (8 * g + kk) * kG + 64);
        const float a0 = a[0][kk >> 2][kk & 3], a1 = a[1][kk >> 2][kk & 3];
#pragma unroll
        for (int tj = 0; tj < 8; ++tj) {
          const float bv = tj < 4 ? b0[tj] : b1[tj - 4];
          acc[0][tj] = M::mma(a0, bv, kk == 4 ? zero : acc[0][tj]);
          acc[1][tj] = M::mma(a1, bv, kk == 0 ? zero : acc[1][tj]);
        }
        if (kk == 3) flush(0);
        if (kk == 7) flush(1);
      }
    }
  }
  __syncthreads();

  // ---- epilogue: rho_i += sum_mu Phi_mu,i X_mu,i and grad rho_i += 2 sum_mu grad Phi_mu,i X_mu,i over
  // the AOs of the chunk's tiles, two tiles per round: their X (FP64) goes through LDS, then one thread
  // per (tile, point) evaluates the tile's shells in FP64 (a wave shares one tile, so the shell data are
  // scalar loads); the per-point sums are ((tile 0 + tile 1) + (tile 2 + tile 3)).
  double *Xs = reinterpret_cast<double *>(ring);   // [2][kD][kG]
  const int slot_w = tid >> 7, j = tid & (kG - 1);
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int R = 0; R < 2; ++R) {
    if ((ws >> 1) == R && 4 * c + ws < np) {
      double *Xw = Xs + (ws & 1) * (kD * kG);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 8; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * ti + M::row(v, l);
            Xw[row * kG + 64 * (tj >> 2) + 4 * m16 + (tj & 3)] =
                ti == 0 ? dacc[ti][tj][v] + double(acc[ti][tj][v]) : dacc[ti][tj][v];   // row 1: flushed
          }
    }
    __syncthreads();
    const int slot = 4 * c + 2 * R + slot_w;
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    if (slot < np) {
      const double *Xw = Xs + slot_w * (kD * kG);
      if (GGA) {
        const int64_t ip = r * kG + j;
        const int pt = __builtin_amdgcn_readfirstlane(s_p[slot]);
        for_tile_aos<true>(A.B, pt, A.g.x[ip], A.g.y[ip], A.g.z[ip], [&](int a, double v, double gx, double gy,
                                                                          double gz) {
          const double X = Xw[a * kG + j];
          s0 += v * X;
          sx += gx * X;
          sy += gy * X;
          sz += gz * X;
        });
      } else {
        const float *ph = phi + size_t(k0 + slot) * (kD * kG) + j;
        const unsigned short *pl = A.phil + size_t(k0 + slot - A.ret0) * (kD * kG) + j;
        for (int a = 0; a < kD; ++a)
          s0 += (double(ph[a * kG]) + from_bf16(pl[a * kG])) * Xw[a * kG + j];
      }
    }
    s_acc[slot_w][0][j] = s0;
    s_acc[slot_w][1][j] = 2.0 * sx;
    s_acc[slot_w][2][j] = 2.0 * sy;
    s_acc[slot_w][3][j] = 2.0 * sz;
    __syncthreads();
    if (tid < kG) {
#pragma unroll
      for (int cp = 0; cp < 4; ++cp) tot[cp] += s_acc[0][cp][tid] + s_acc[1][cp][tid];
    }
  }
  if (tid < kG) {
    double *out = A.part + size_t(il) * (4 * kG);
#pragma unroll
    for (int cp = 0; cp < (GGA ? 4 : 1); ++cp) out[cp * kG + tid] = tot[cp];
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[0], (unsigned long long)(pd + 0.5));
  });
}

// FP64 operands: the 4-wave X kernel of k_xgemm_f32 on v_mfma_f64_16x16x4f64 (same items).  An FP64 entry (64 KB) is taken in two K halves of 16 values, each a ring slot of 32 KB
// (4 D half-tiles [row i][k] with the 16-byte units of row i XOR-swizzled, unit c at c ^ swz(i), and
// half of Phi_q as [k][point]); MFMA step kk of a half takes k = 4 (l / 16) + kk, and output column c of
// sub-tile tj is point 32 (tj / 2) + 2 c + tj % 2 (the 16 lanes of a row read 256 contiguous bytes per
// 16-byte load).  The accumulators are FP64, so X needs no flush.
template <bool GGA>
__global__ __launch_bounds__(NTX4, 2) void k_xgemm_f64(XArgs A) {
  typedef Mma<double> M;
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int kHalf = kD / 2;                       // K values per sub-step
  constexpr int kSub = 4 * kD * kHalf + kHalf * kG;   // doubles per ring slot (32 KB)
  __shared__ __align__(16) double ring[2 * kSub];
  __shared__ int s_p[kMaxNp];
  __shared__ int s_list[kMaxNp];
  __shared__ int s_q[kMaxNp];
  __shared__ int s_w[4];
  __shared__ double s_acc[2][4][kG];
  static_assert(2 * kD * kG <= 2 * kSub, "epilogue X exceeds the ring");
  run_items(A.q, A.item0, [&](int64_t il) {
  const int64_t it = A.item0 + il;
  const int64_t r = A.xit_r[it];
  const int c = A.xit_c[it];
  const int tid = threadIdx.x, l = tid & 63;
  const int ws = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m16 = l & 15, g = l >> 4;
  const MolDev mo = A.st.mol[A.st.blk_mol[r]];
  const int64_t k0 = A.st.blk_off[r];
  const int np = int(A.st.blk_off[r + 1] - k0);
  const double *Dd = static_cast<const double *>(A.Dt);
  const double *phi = static_cast<const double *>(A.phi) - size_t(A.ret0) * (kD * kG);   // by retained tile
  auto dtile = [&](int p, int q) { return size_t(mo.dt0) + size_t(p - mo.tile0) * mo.nt + (q - mo.tile0); };

  for (int t = tid; t < np; t += NTX4) s_p[t] = A.st.ret_p[k0 + t];
  __syncthreads();

  unsigned long long pairs = 0;
  int n_list = 0;
  for (int base = 0; base < np; base += NTX4) {
    const int t = base + tid;
    int mask = 0;
    if (t < np) {
      const int q = s_p[t];
      const double bq = A.st.bphi[k0 + t];
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        if (4 * c + ww < np) {
          const double a = A.amax[dtile(s_p[4 * c + ww], q)];
          if (a >= A.t_b && a * bq >= A.t_d) mask |= 1 << ww;
        }
      }
    }
    int tot;
    const int pos = n_list + block_scan(mask != 0, s_w, &tot);
    if (mask) {
      s_list[pos] = t | (mask << 16);
      s_q[pos] = s_p[t];
      pairs += __popc(mask);
    }
    n_list += tot;
  }
  __syncthreads();

  d4 acc[2][8];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
  const int pa = __builtin_amdgcn_readfirstlane(s_p[min(4 * c + ws, np - 1)]);
  const double *Drow = Dd + dtile(pa, mo.tile0) * (kD * kD);
  // sub-step st = 2 e + h: K half h of entry e, into slot st % 2; wave w copies D_(p_w, q) and quarter w
  // of the half of Phi_q, global -> LDS directly
  auto issue = [&](int st) {
    const int e = st >> 1, h = st & 1;
    double *dst = ring + (st & 1) * kSub;
    const int q = __builtin_amdgcn_readfirstlane(s_q[e]);
    const double *src = Drow + size_t(q - mo.tile0) * (kD * kD) + kHalf * h;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int tu = 64 * m + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
      dma16(src + i * kD + 2 * cu, dst + ws * (kD * kHalf) + 128 * m);
    }
    const int t = __builtin_amdgcn_readfirstlane(s_list[e] & 0xffff);
    const double *ps = phi + size_t(k0 + t) * (kD * kG) + (kHalf * kG) * h + 512 * ws;
#pragma unroll
    for (int m = 0; m < 4; ++m) dma16(ps + 2 * (64 * m + l), dst + 4 * kD * kHalf + 512 * ws + 128 * m);
  };
  const int nst = 2 * n_list;
  if (nst > 0) issue(0);
  for (int st = 0; st < nst; ++st) {
    wait_vm_lds<0>();
    wg_barrier();
    if (st + 1 < nst) issue(st + 1);
    if ((__builtin_amdgcn_readfirstlane(s_list[st >> 1] >> 16) >> ws) & 1) {
      const double *se = ring + (st & 1) * kSub;
      d2 a[2][2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
          a[ti][hh] = *reinterpret_cast<const d2 *>(se + ws * (kD * kHalf) + (16 * ti + m16) * kHalf +
                                                    2 * ((2 * g + hh) ^ swz(16 * ti + m16)));
      const double *sb = se + 4 * kD * kHalf + 2 * m16;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        d2 b[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) b[jj] = *reinterpret_cast<const d2 *>(sb + (4 * g + kk) * kG + 32 * jj);
        const double a0 = a[0][kk >> 1][kk & 1], a1 = a[1][kk >> 1][kk & 1];
#pragma unroll
        for (int tj = 0; tj < 8; ++tj) {
          const double bv = b[tj >> 1][tj & 1];
          acc[0][tj] = M::mma(a0, bv, acc[0][tj]);
          acc[1][tj] = M::mma(a1, bv, acc[1][tj]);
        }
      }
    }
  }
  __syncthreads();

  // ---- epilogue as in k_xgemm_f32
  double *Xs = ring;   // [2][kD][kG]
  const int slot_w = tid >> 7, j = tid & (kG - 1);
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int R = 0; R < 2; ++R) {
    if ((ws >> 1) == R && 4 * c + ws < np) {
      double *Xw = Xs + (ws & 1) * (kD * kG);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 8; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * ti + M::row(v, l);
            Xw[row * kG + 32 * (tj >> 1) + 2 * m16 + (tj & 1)] = acc[ti][tj][v];
          }
    }
    __syncthreads();
    const int slot = 4 * c + 2 * R + slot_w;
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    if (slot < np) {
      const double *Xw = Xs + slot_w * (kD * kG);
      if (GGA) {
        const int64_t ip = r * kG + j;
        const int pt = __builtin_amdgcn_readfirstlane(s_p[slot]);
        for_tile_aos<true>(A.B, pt, A.g.x[ip], A.g.y[ip], A.g.z[ip], [&](int a, double v, double gx, double gy,
                                                                          double gz) {
          const double X = Xw[a * kG + j];
          s0 += v * X;
          sx += gx * X;
          sy += gy * X;
          sz += gz * X;
        });
      } else {
        const double *ph = phi + size_t(k0 + slot) * (kD * kG) + j;
        for (int a = 0; a < kD; ++a) s0 += ph[a * kG] * Xw[a * kG + j];
      }
    }
    s_acc[slot_w][0][j] = s0;
    s_acc[slot_w][1][j] = 2.0 * sx;
    s_acc[slot_w][2][j] = 2.0 * sy;
    s_acc[slot_w][3][j] = 2.0 * sz;
    __syncthreads();
    if (tid < kG) {
#pragma unroll
      for (int cp = 0; cp < 4; ++cp) tot[cp] += s_acc[0][cp][tid] + s_acc[1][cp][tid];
    }
  }
  if (tid < kG) {
    double *out = A.part + size_t(il) * (4 * kG);
#pragma unroll
    for (int cp = 0; cp < (GGA ? 4 : 1); ++cp) out[cp * kG + tid] = tot[cp];
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[0], (unsigned long long)(pd + 0.5));
  });
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
  Xc f;
  const double wgt = A.g.w[ip];
  if (A.tpart[0]) {
    // meta-GGA: tau = (1/2) sum_a sum_mu d_a chi_mu (D d_a Phi)_mu, from component 1 + a of the partials
    // of the product with d_a Phi (each 2 sum_mu d_a chi_mu X^a_mu), in item order
    double t = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int64_t it = A.blk_item_off[r]; it < A.blk_item_off[r + 1]; ++it)
        t += A.tpart[a][size_t(it - A.item0) * (4 * kG) + (1 + a) * kG + j];
    const Xc4 m = xc_eval_mgga(A.xc, s[0], sigma, 0.25 * t, A.rho_cut);
    f = Xc{m.f, m.vr, m.vs};
    A.ctau[ip] = 0.25 * wgt * m.vt;
  } else {
    f = xc_eval(A.xc, s[0], sigma, A.rho_cut);
  }
  const int64_t o = A.g.orig[ip];
  double *rho_out = A.io->rho, *sigma_out = A.io->sigma;
  if (rho_out && o >= 0) rho_out[o] = s[0];
  if (sigma_out && o >= 0) sigma_out[o] = sigma;
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
                                             const unsigned short *__restrict__ phil, T *__restrict__ zws,
                                             double *__restrict__ zmax) {
  const int64_t k = ret0 + blockIdx.x;
  const int j = threadIdx.x;
  const int p = st.ret_p[k];
  const int64_t ip = int64_t(st.ret_r[k]) * kG + j;
  const double *cf = coef + size_t(ip) * 4;
  const double c0 = cf[0];
  const size_t o = size_t(blockIdx.x) * (kD * kG) + j;
  T *out = zws + o;
  double zm = 0.0;
  auto put = [&](int a, double zv) {
    const T zt = T(zv);
    out[a * kG] = zt;
    zm = fmax(zm, fabs(double(zt)));
  };
  if (GGA) {
    const double c1x = cf[1], c1y = cf[2], c1z = cf[3];
    for (int a = B.tile_nv[p]; a < kD; ++a) out[a * kG] = T(0);
    for_tile_aos<true>(B, p, g.x[ip], g.y[ip], g.z[ip], [&](int a, double v, double gx, double gy, double gz) {
      put(a, c0 * v + c1x * gx + c1y * gy + c1z * gz);
    });
  } else {
    // Z from the stored Phi, with its low part for FP32 operands (Z then carries no rounding of Phi)
    const T *in = phi + o;
    for (int a = 0; a < kD; ++a) {
      double v = double(in[a * kG]);
      if (sizeof(T) == 4 && phil) v += from_bf16(phil[o + a * kG]);
      put(a, c0 * v);
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
  const int *cinfo;        // per (block, chunk of its molecule): (first position in S_r) << 4 | 4-bit mask
  const int64_t *cioff;    // [n_blocks+1] first cinfo entry of each block
  const int64_t *vmoff;    // [n_blocks+1] first vmask entry of each block
  int64_t vm_base;         // vmoff of the launch's first block (the vmask slice starts there)
  const int *pair_info;    // [3 * n_pairs] (row chunk, column chunk, molecule)
  const double *zmax;
  int64_t blk0;            // first block of this launch
  unsigned short *vmask;   // mask slice of the launch
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
  const MolDev mo = A.st.mol[A.st.blk_mol[r]];
  const int *ci = A.cinfo + A.cioff[r];
  unsigned short *out = A.vmask + (A.vmoff[r] - A.vm_base);
  for (int pr = threadIdx.x; pr < mo.npairs; pr += NT) {
    const int pc = A.pair_info[3 * (mo.pair0 + pr)], qc = A.pair_info[3 * (mo.pair0 + pr) + 1];
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
    out[pr] = (unsigned short)mask;
  }
}

// Gradient products: each item's 128 x 128 partial (rows: AOs of row chunk pc, columns: AOs of column chunk
// qc) times D element by element, summed along each row (mode 0: one sum per row AO) or each column (mode 1:
// one per column AO), into slot `slot` of the item's gradient partial (zeros where nothing executed),
// formed from the Vxc kernels' accumulators instead of a stored partial.
struct GContract {
  const int *pair_info;    // [3 * pairs]: the molecule of each chunk pair in entry 2
  const double *Dt;        // D as FP64 32 x 32 tiles
  double *gitem;           // [items * 6 * 128]
  int mode, slot;
};

struct VArgs {
  StructDev st;
  const VItem *items;
  int64_t item0, n_items;  // the items of this launch
  int64_t ret0;            // first retained tile of the workspaces
  const int *cinfo;
  const int64_t *cioff, *vmoff;
  int64_t vm_base;         // vmoff of the launch's first block
  const unsigned short *vmask;
  const void *phi;
  const void *zws;
  double *vpart;
  int *vflag;              // [n_items] 1 if the item wrote a partial
  unsigned long long *counters;
  QArgs q;
  int accumulate;          // FP64 operands: add to the item's partial when an earlier launch wrote one
  int keep_diag;           // FP32 operands: also the pairs (a, a) of diagonal chunk pairs (no k_vdiag beside it)
  GContract gc;            // contracting kernels (gradient products): where the contractions go
};

// The contraction of GContract from the accumulators of a Vxc kernel: wave w holds tile pair (a, (w - a)
// mod 4) for a = 0..3, val(a, ti, tj, v) at row 32 a + 16 ti + row(v), column 32 b + 16 tj + (lane % 16).
// A wave's 4 pairs cover every row (and every column) of the chunk pair once, so each wave sums its part
// of every row (column) over the 16 lanes (4 lane groups) that hold it, and the 4 waves' parts are added in
// wave order.
template <class Val, class Row>
__device__ __forceinline__ void grad_contract(const VArgs &A, const VItem &it, int64_t item, bool any, int ws,
                                              double (*s_red)[128], Val &&val, Row &&row) {
  const int tid = threadIdx.x, l = tid & 63, m16 = l & 15, g = l >> 4;
  double *gout = A.gc.gitem + (size_t(item) * 6 + A.gc.slot) * 128;
  if (!any) {
    if (tid < 128) gout[tid] = 0.0;
    return;
  }
  const MolDev mo = A.st.mol[A.gc.pair_info[3 * it.pair + 2]];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int b = (ws - a) & 3, p = 4 * it.pc + a, q = 4 * it.qc + b;
    const bool ok = p < mo.nt && q < mo.nt;   // tiles past the molecule's AOs: D = 0
    const double *dt = A.gc.Dt + (size_t(mo.dt0) + size_t(p) * mo.nt + q) * 1024;
    if (A.gc.mode == 0) {
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * ti + row(v);
          double sm = 0.0;
          if (ok) {
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) sm += val(a, ti, tj, v) * dt[r * 32 + 16 * tj + m16];
          }
          sm += __shfl_xor(sm, 1);
          sm += __shfl_xor(sm, 2);
          sm += __shfl_xor(sm, 4);
          sm += __shfl_xor(sm, 8);
          if (m16 == 0) s_red[ws][32 * a + r] = sm;
        }
    } else {
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        double sm = 0.0;
        if (ok) {
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) sm += val(a, ti, tj, v) * dt[(16 * ti + row(v)) * 32 + 16 * tj + m16];
        }
        sm += __shfl_xor(sm, 16);
        sm += __shfl_xor(sm, 32);
        if (g == 0) s_red[ws][32 * b + 16 * tj + m16] = sm;
      }
    }
  }
  __syncthreads();
  if (tid < 128) gout[tid] = (s_red[0][tid] + s_red[1][tid]) + (s_red[2][tid] + s_red[3][tid]);
}


constexpr int NTV4 = 256;   // threads per FP32 Vxc workgroup: 4 waves, wave a owns row tile a (32 x 128)

// FP32 operands: one workgroup of 4 waves per Vxc item (row chunk pc, column chunk qc, segment of grid
// blocks): M_pq = sum_r Phi_pr Z_qr^T over the executable grid
// blocks of the segment, compacted by prefix sum.  Its LDS (69 KB: a two-slot ring of one 32-point
// sub-step each, 4 Phi slabs and 4 Z slabs of 32 x 32) lets two workgroups share a CU, so one
// workgroup's copies, barriers and compaction overlap the other's MFMAs.  Wave w owns the tile pairs
// (a, (w - a) mod 4), a = 0..3: one of every row and every column of the 4 x 4 chunk pair.  A block's
// pair mask is sparse (about 4 of 16 pairs execute at the bench workload) and close to the outer product
// of the retained row and column tiles, which this ownership spreads over the 4 waves (owning a row each
// left the waves of unretained rows idle: 41.8 ms against 35.9 ms for the Vxc stage of the bench
// workload).  MFMA step kk takes point 8 (l / 16) + kk of the sub-step, so a lane reads the 8 values of
// its row of a slab with two 16-byte loads.  The FP32 accumulators of a pair are added to the FP64 sums
// after each sub-step (32 points).  The diagonal pairs (a, a) of a diagonal chunk pair are k_vdiag's
// (FP64) unless keep_diag is set (the nuclear gradient's products, which are not symmetric).  CONTRACT: the
// item's partial goes into its gradient contraction (GContract) instead of vpart.
template <bool CONTRACT>
__global__ __launch_bounds__(NTV4, 2) void k_vgemm_f32(VArgs A) {
  typedef Mma<float> M;
  constexpr int kSP = 32, kNS = kG / kSP, kSlab = kD * kSP, kSlot = 8 * kSlab;
  __shared__ __align__(16) float ring[2 * kSlot];
  __shared__ int s_m[NTV4];
  __shared__ int s_ip[NTV4], s_iq[NTV4];
  __shared__ long long s_bo[NTV4];
  __shared__ int s_w[4];
  run_items(A.q, A.item0, [&](int64_t il) {
  const int64_t item = A.item0 + il;
  const VItem it = A.items[item];
  const int tid = threadIdx.x, l = tid & 63;
  const int ws = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m16 = l & 15, g = l >> 4;
  const float *Pf = static_cast<const float *>(A.phi) - size_t(A.ret0) * (kD * kG);   // by retained tile
  const float *Zf = static_cast<const float *>(A.zws) - size_t(A.ret0) * (kD * kG);
  const bool diag = it.pc == it.qc && !A.keep_diag;   // its pairs (a, a) are k_vdiag's

  f4 acc[2][8];
  double dacc[2][8][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) {
      acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[ti][tj][v] = 0.0;
    }
  unsigned long long pairs = 0;
  int any = 0;
  for (int base = it.r0; base < it.r1; base += NTV4) {
    const int r = base + tid;
    int mask = 0;
    if (r < it.r1) mask = A.vmask[A.vmoff[r] - A.vm_base + it.lpair];
    int tot;
    const int pos = block_scan(mask != 0, s_w, &tot);
    if (mask) {
      s_m[pos] = mask;
      const int64_t cb = A.cioff[r];
      s_ip[pos] = A.cinfo[cb + it.pc];
      s_iq[pos] = A.cinfo[cb + it.qc];
      s_bo[pos] = A.st.blk_off[r];
      pairs += __popc(mask);
    }
    __syncthreads();
    any |= tot;
    // sub-step st = kNS e + sub: entry e of the compacted list, points kSP sub .. kSP sub + kSP - 1.  Slot
    // st % 2: slab a < 4 is Phi_(4pc+a), slab 4 + b is Z_(4qc+b), each [row i][point] with the 16-byte
    // units of row i XOR-swizzled (unit c at c ^ swz(i)); wave w copies slabs w and 4 + w, global -> LDS
    // directly, one sub-step ahead, and only where the slab's tile has an executable pair.
    const int nst = kNS * tot;
    auto issue = [&](int st) {
      const int e = st / kNS, sub = st % kNS;
      const int m = __builtin_amdgcn_readfirstlane(s_m[e]);
      const long long bo = s_bo[e];
      float *dst = ring + (st & 1) * kSlot;
      if ((m >> (4 * ws)) & 15) {
        const int info = __builtin_amdgcn_readfirstlane(s_ip[e]);
        const float *src = Pf + size_t(bo + tile_pos(info, ws)) * (kD * kG) + kSP * sub;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tu = 64 * k + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
          dma16(src + i * kG + 4 * cu, dst + ws * kSlab + 256 * k);
        }
      }
      if ((m >> ws) & 0x1111) {
        const int info = __builtin_amdgcn_readfirstlane(s_iq[e]);
        const float *src = Zf + size_t(bo + tile_pos(info, ws)) * (kD * kG) + kSP * sub;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tu = 64 * k + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
          dma16(src + i * kG + 4 * cu, dst + (4 + ws) * kSlab + 256 * k);
        }
      }
    };
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    if (nst > 0) issue(0);
    for (int st = 0; st < nst; ++st) {
      // this wave's copies of sub-step st have landed and its reads of st - 1 are done; after the
      // barrier the slot of st - 1 takes sub-step st + 1
      wait_vm_lds<0>();
      wg_barrier();
      if (st + 1 < nst) issue(st + 1);
      const int m = __builtin_amdgcn_readfirstlane(s_m[st / kNS]);
      const float *sl = ring + (st & 1) * kSlot;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        // pair a of this wave: row tile a, column tile b = (w - a) mod 4; accumulators 2a, 2a + 1
        const int b = (ws - a) & 3;
        if (!((m >> (4 * a + b)) & 1) || (diag && a == b)) continue;
        f4 fa[2][2], fb[2][2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int off = (16 * t + m16) * kSP + 4 * ((2 * g + hh) ^ swz(16 * t + m16));
            fa[t][hh] = *reinterpret_cast<const f4 *>(sl + a * kSlab + off);
            fb[t][hh] = *reinterpret_cast<const f4 *>(sl + (4 + b) * kSlab + off);
          }
        // FP32 sums of 32 points each (the first MFMA takes a zero accumulator), FP64 beyond
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
              acc[ti][2 * a + tj] = M::mma(fa[ti][kk >> 2][kk & 3], fb[tj][kk >> 2][kk & 3],
                                           kk == 0 ? zero : acc[ti][2 * a + tj]);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v) dacc[ti][2 * a + tj][v] += double(acc[ti][2 * a + tj][v]);
      }
    }
    __syncthreads();
  }
  if constexpr (CONTRACT) {
    // the ring is free after the loop's last barrier
    grad_contract(A, it, item, any != 0, ws, reinterpret_cast<double (*)[128]>(ring),
                  [&](int a, int ti, int tj, int v) { return dacc[ti][2 * a + tj][v]; },
                  [&](int v) { return M::row(v, l); });
  } else {
    if (!any) {
      if (tid == 0 && !A.accumulate) A.vflag[item] = 0;
      return;
    }
    double *out = A.vpart + size_t(item) * (128 * 128);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int b = (ws - a) & 3;
      if (diag && a == b) continue;           // written by k_vdiag
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 32 * a + 16 * ti + M::row(v, l), col = 32 * b + 16 * tj + m16;
            out[row * 128 + col] = dacc[ti][2 * a + tj][v];
          }
    }
    if (tid == 0) A.vflag[item] = 1;
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[1], (unsigned long long)(pd + 0.5));
  });
}

// FP64 operands: the 4-wave Vxc kernel of k_vgemm_f32 on v_mfma_f64_16x16x4f64 (same items and pair
// ownership), with 16-point sub-steps so that a ring slot (4 Phi slabs and 4 Z slabs of 32 x 16) stays
// 32 KB; MFMA step kk takes point 4 (l / 16) + kk of the sub-step.  With `accumulate` set, an item whose
// partial an earlier launch wrote adds to it (the meta-GGA term).  CONTRACT as for k_vgemm_f32.
template <bool CONTRACT>
__global__ __launch_bounds__(NTV4, 2) void k_vgemm_f64(VArgs A) {
  typedef Mma<double> M;
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int kSP = 16, kNS = kG / kSP, kSlab = kD * kSP, kSlot = 8 * kSlab;
  __shared__ __align__(16) double ring[2 * kSlot];
  __shared__ int s_m[NTV4];
  __shared__ int s_ip[NTV4], s_iq[NTV4];
  __shared__ long long s_bo[NTV4];
  __shared__ int s_w[4];
  run_items(A.q, A.item0, [&](int64_t il) {
  const int64_t item = A.item0 + il;
  const VItem it = A.items[item];
  const int tid = threadIdx.x, l = tid & 63;
  const int ws = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m16 = l & 15, g = l >> 4;
  const double *Pd = static_cast<const double *>(A.phi) - size_t(A.ret0) * (kD * kG);   // by retained tile
  const double *Zd = static_cast<const double *>(A.zws) - size_t(A.ret0) * (kD * kG);
  const int prev = A.accumulate ? A.vflag[item] : 0;

  d4 acc[2][8];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 8; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
  unsigned long long pairs = 0;
  int any = 0;
  for (int base = it.r0; base < it.r1; base += NTV4) {
    const int r = base + tid;
    int mask = 0;
    if (r < it.r1) mask = A.vmask[A.vmoff[r] - A.vm_base + it.lpair];
    int tot;
    const int pos = block_scan(mask != 0, s_w, &tot);
    if (mask) {
      s_m[pos] = mask;
      const int64_t cb = A.cioff[r];
      s_ip[pos] = A.cinfo[cb + it.pc];
      s_iq[pos] = A.cinfo[cb + it.qc];
      s_bo[pos] = A.st.blk_off[r];
      pairs += __popc(mask);
    }
    __syncthreads();
    any |= tot;
    const int nst = kNS * tot;
    auto issue = [&](int st) {
      const int e = st / kNS, sub = st % kNS;
      const int m = __builtin_amdgcn_readfirstlane(s_m[e]);
      const long long bo = s_bo[e];
      double *dst = ring + (st & 1) * kSlot;
      if ((m >> (4 * ws)) & 15) {
        const int info = __builtin_amdgcn_readfirstlane(s_ip[e]);
        const double *src = Pd + size_t(bo + tile_pos(info, ws)) * (kD * kG) + kSP * sub;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tu = 64 * k + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
          dma16(src + i * kG + 2 * cu, dst + ws * kSlab + 128 * k);
        }
      }
      if ((m >> ws) & 0x1111) {
        const int info = __builtin_amdgcn_readfirstlane(s_iq[e]);
        const double *src = Zd + size_t(bo + tile_pos(info, ws)) * (kD * kG) + kSP * sub;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tu = 64 * k + l, i = tu >> 3, cu = (tu & 7) ^ swz(i);
          dma16(src + i * kG + 2 * cu, dst + (4 + ws) * kSlab + 128 * k);
        }
      }
    };
    if (nst > 0) issue(0);
    for (int st = 0; st < nst; ++st) {
      wait_vm_lds<0>();
      wg_barrier();
      if (st + 1 < nst) issue(st + 1);
      const int m = __builtin_amdgcn_readfirstlane(s_m[st / kNS]);
      const double *sl = ring + (st & 1) * kSlot;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        // pair a of this wave: row tile a, column tile b = (w - a) mod 4; accumulators 2a, 2a + 1
        const int b = (ws - a) & 3;
        if (!((m >> (4 * a + b)) & 1)) continue;
        d2 fa[2][2], fb[2][2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int off = (16 * t + m16) * kSP + 2 * ((2 * g + hh) ^ swz(16 * t + m16));
            fa[t][hh] = *reinterpret_cast<const d2 *>(sl + a * kSlab + off);
            fb[t][hh] = *reinterpret_cast<const d2 *>(sl + (4 + b) * kSlab + off);
          }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
              acc[ti][2 * a + tj] = M::mma(fa[ti][kk >> 1][kk & 1], fb[tj][kk >> 1][kk & 1], acc[ti][2 * a + tj]);
      }
    }
    __syncthreads();
  }
  if constexpr (CONTRACT) {
    grad_contract(A, it, item, any != 0, ws, reinterpret_cast<double (*)[128]>(ring),
                  [&](int a, int ti, int tj, int v) { return acc[ti][2 * a + tj][v]; },
                  [&](int v) { return M::row(v, l); });
  } else {
    if (!any) {
      if (tid == 0 && !A.accumulate) A.vflag[item] = 0;
      return;
    }
    double *out = A.vpart + size_t(item) * (128 * 128);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int b = (ws - a) & 3;
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 32 * a + 16 * ti + M::row(v, l), col = 32 * b + 16 * tj + m16;
            const double val = acc[ti][2 * a + tj][v];
            out[row * 128 + col] = prev ? out[row * 128 + col] + val : val;
          }
    }
    if (tid == 0) A.vflag[item] = 1;
  }
  double pd = wave_sum(double(pairs));
  if (l == 0 && pd > 0) atomicAdd(&A.counters[1], (unsigned long long)(pd + 0.5));
  });
}

// One workgroup row per chunk pair (all molecules): FP64 sum of its segment partials in segment order.
// FP32 plans: the diagonal tiles M_pp of the Vxc product in FP64.  One workgroup per Vxc item of a
// diagonal chunk pair (pc = qc); wave w owns the tile p = 4 pc + w and walks the segment's blocks whose
// pair mask executes (p, p) (eq. block_pair_filter, as k_vgemm_f32), M_pp += Phi_pr Z_pr^T on FP64 MFMA with
// the operand Phi_hi + Phi_lo; the result goes to the tile's place in the item's partial, whose other
// tiles k_vgemm_f32 writes.  The two kernels share no output, so they run concurrently (an item in which
// nothing executes gets zeros here and is skipped by the reduction).
struct VDArgs {
  StructDev st;
  const VItem *items;
  const int *ditems;       // items of diagonal chunk pairs, this launch
  int64_t n;
  int64_t ret0;
  const int *cinfo;
  const int64_t *cioff, *vmoff;
  int64_t vm_base;
  const unsigned short *vmask;
  const float *phi;
  const unsigned short *phil;
  const float *zws;
  double *vpart;
  unsigned long long *counters;
};

__global__ __launch_bounds__(NT) void k_vdiag(VDArgs A) {
  const int64_t item = A.ditems[blockIdx.x];
  const VItem it = A.items[item];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  d4 dd[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti) dd[ti][0] = dd[ti][1] = d4{0.0, 0.0, 0.0, 0.0};
  int n_exec = 0;
  for (int r = it.r0; r < it.r1; ++r) {
    const int mask = A.vmask[A.vmoff[r] - A.vm_base + it.lpair];
    if (!((mask >> (5 * w)) & 1)) continue;      // bit 4 w + w: the pair (p, p)
    ++n_exec;
    const int ci = A.cinfo[A.cioff[r] + it.pc];
    const size_t t = size_t(A.st.blk_off[r] + tile_pos(ci, w) - A.ret0) * (kD * kG);
    // MFMA step kk of lane group g = l / 16 takes point 32 g + kk, so a lane reads 8 consecutive points
    // of each of its two rows (i0, i0 + 16) with 16-byte loads per 8 steps
    const int i0 = l & 15, g = l >> 4;
    const float *ph = A.phi + t + i0 * kG + 32 * g;
    const unsigned short *pl = A.phil + t + i0 * kG + 32 * g;
    const float *zt = A.zws + t + i0 * kG + 32 * g;
    for (int c8 = 0; c8 < 4; ++c8) {
      f4 h[2][2], z[2][2];
      uint4 lo[2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        const int o = ti * 16 * kG + 8 * c8;
        h[ti][0] = *reinterpret_cast<const f4 *>(ph + o);
        h[ti][1] = *reinterpret_cast<const f4 *>(ph + o + 4);
        z[ti][0] = *reinterpret_cast<const f4 *>(zt + o);
        z[ti][1] = *reinterpret_cast<const f4 *>(zt + o + 4);
        lo[ti] = *reinterpret_cast<const uint4 *>(pl + o);
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        double a[2], bz[2];
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          const unsigned w32 = (&lo[ti].x)[kk >> 1];
          a[ti] = double(h[ti][kk >> 2][kk & 3]) + from_bf16((unsigned short)((kk & 1) ? (w32 >> 16) : (w32 & 0xffff)));
          bz[ti] = double(z[ti][kk >> 2][kk & 3]);
        }
        dd[0][0] = Mma<double>::mma(a[0], bz[0], dd[0][0]);
        dd[0][1] = Mma<double>::mma(a[0], bz[1], dd[0][1]);
        dd[1][0] = Mma<double>::mma(a[1], bz[0], dd[1][0]);
        dd[1][1] = Mma<double>::mma(a[1], bz[1], dd[1][1]);
      }
    }
  }
  double *out = A.vpart + size_t(item) * (128 * 128);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * w + 16 * ti + Mma<double>::row(v, l), col = 32 * w + 16 * tj + (l & 15);
        out[row * 128 + col] = dd[ti][tj][v];
      }
  if (l == 0 && n_exec > 0) atomicAdd(&A.counters[6], (unsigned long long)n_exec);
}

__global__ __launch_bounds__(NT) void k_vreduce(const int *pair_ptr, const int *pair_items, const int *pair_info,
                                               const MolDev *mol, const int *__restrict__ vflag,
                                               const double *__restrict__ vpart, double *__restrict__ mfull) {
  const int pr = blockIdx.x;
  const int e = blockIdx.y * NT + threadIdx.x;  // 0 .. 16383
  const int i = e >> 7, j = e & 127;
  // items in list order; 8 loads in flight per step, added in the same order (an item that wrote no
  // partial adds 0)
  double s = 0.0;
  const int k1 = pair_ptr[pr + 1];
  int k = pair_ptr[pr];
  for (; k + 8 <= k1; k += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int itm = pair_items[k + u];
      v[u] = vflag[itm] ? vpart[size_t(itm) * 16384 + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < k1; ++k) {
    const int itm = pair_items[k];
    if (vflag[itm]) s += vpart[size_t(itm) * 16384 + e];
  }
  const int pc = pair_info[3 * pr], qc = pair_info[3 * pr + 1];
  const MolDev mo = mol[pair_info[3 * pr + 2]];
  mfull[size_t(mo.mf0) + size_t(128 * pc + i) * mo.ld + 128 * qc + j] = s;
}

// Vxc = M + M^T (GGA) or mirrored 2M (LDA), back to the caller's AO order.  One workgroup per
// (stacked AO row, group of NT columns).
__global__ __launch_bounds__(NT) void k_vsym(const MolDev *mol, int n_mol, int ncol, const double *__restrict__ mfull,
                                            const int *__restrict__ perm, int gga, const IoDev *io) {
  const int64_t g = blockIdx.x / ncol;
  const int j = (blockIdx.x % ncol) * NT + threadIdx.x;
  const MolDev mo = mol[find_mol(mol, n_mol, g, [](const MolDev &x) { return x.row0; })];
  const int i = int(g - mo.row0), n_ao = mo.n_ao;
  if (j >= n_ao) return;
  const double *mf = mfull + mo.mf0;
  const int *pm = perm + size_t(mo.tile0) * kD;
  const double mij = mf[size_t(i) * mo.ld + j], mji = mf[size_t(j) * mo.ld + i];
  double v;
  if (gga) {
    v = mij + mji;
  } else {
    const int p = i / kD, q = j / kD;
    v = (p < q) ? 2.0 * mij : (p > q ? 2.0 * mji : mij + mji);
  }
  io->vxc[size_t(mo.d0) + size_t(pm[i]) * n_ao + pm[j]] = v;
}

// One workgroup per molecule: E_xc as a fixed-order FP64 sum of its block partials.
__global__ __launch_bounds__(NT) void k_esum(const MolDev *mol, const double *__restrict__ eblk, const IoDev *io) {
  const MolDev mo = mol[blockIdx.x];
  __shared__ double s[NT];
  double a = 0.0;
  for (int64_t i = mo.blk0 + threadIdx.x; i < mo.blk1; i += NT) a += eblk[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) io->exc[blockIdx.x] = s[0];
}

// One workgroup per retained tile (p, r) of the chunk, from one evaluation of the tile's values, gradients
// and second derivatives: d_a Phi into Aout, Q^a = sum_b c_b d_a d_b Phi into Qout and W = c0 Phi + sum_b
// c_b d_b Phi into Wout (Qout and Wout when not NULL), and, when Amax is not NULL, each tile's max |.| of
// what it wrote for the products' pair filter.
template <class T>
__global__ __launch_bounds__(kG) void k_gterm(BasisDev B, GridDev g, StructDev st, int64_t ret0,
                                             const double *__restrict__ coef, int ax, T *__restrict__ Aout,
                                             T *__restrict__ Qout, T *__restrict__ Wout,
                                             double *__restrict__ Amax, double *__restrict__ Qmax,
                                             double *__restrict__ Wmax) {
  const int64_t k = ret0 + blockIdx.x;
  const int j = threadIdx.x;
  const int p = st.ret_p[k];
  const int64_t ip = int64_t(st.ret_r[k]) * kG + j;
  const double *cf = coef + size_t(ip) * 4;
  const double c0 = 2.0 * cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
  const double x = g.x[ip], y = g.y[ip], z = g.z[ip];
  const size_t o = size_t(blockIdx.x) * (kD * kG) + j;
  // second-derivative slots (xx xy xz yy yz zz) of row ax
  const int h0 = ax == 0 ? 0 : (ax == 1 ? 1 : 2), h1 = ax == 0 ? 1 : (ax == 1 ? 3 : 4), h2 = ax == 0 ? 2 : (ax == 1 ? 4 : 5);
  double am = 0.0, qm = 0.0, wm = 0.0;
  for (int a = B.tile_nv[p]; a < kD; ++a) {   // padding rows
    Aout[o + a * kG] = T(0);
    if (Qout) Qout[o + a * kG] = T(0);
    if (Wout) Wout[o + a * kG] = T(0);
  }
  for_tile_aos_hess(B, p, x, y, z, [&](int a, double v, const double *gr, const double *h) {
    const double av = gr[ax];
    Aout[o + a * kG] = T(av);
    am = fmax(am, fabs(av));
    if (Qout) {
      const double qv = c1 * h[h0] + c2 * h[h1] + c3 * h[h2];
      Qout[o + a * kG] = T(qv);
      qm = fmax(qm, fabs(qv));
    }
    if (Wout) {
      const double wv = c0 * v + c1 * gr[0] + c2 * gr[1] + c3 * gr[2];
      Wout[o + a * kG] = T(wv);
      wm = fmax(wm, fabs(wv));
    }
  });
  // the tile's max |A|, |Q|, |W| for the products' pair filter
  __shared__ double s_m[2][3];
  am = wave_max(am);
  qm = wave_max(qm);
  wm = wave_max(wm);
  if ((j & 63) == 0) {
    s_m[j >> 6][0] = am;
    s_m[j >> 6][1] = qm;
    s_m[j >> 6][2] = wm;
  }
  __syncthreads();
  if (j == 0 && Amax) {
    Amax[blockIdx.x] = fmax(s_m[0][0], s_m[1][0]);
    if (Qout) Qmax[blockIdx.x] = fmax(s_m[0][1], s_m[1][1]);
    if (Wout) Wmax[blockIdx.x] = fmax(s_m[0][2], s_m[1][2]);
  }
}

// 256-point screening blocks: one workgroup per compute block r of the chunk with (r - first block of its
// molecule) even and a partner r + 1: z_qr of both halves becomes the maximum over the two (the retained
// lists of the halves are the same tiles in the same order).
__global__ __launch_bounds__(NT) void k_zpair(StructDev st, int64_t blk0, double *__restrict__ zmax) {
  const int64_t r = blk0 + blockIdx.x;
  const MolDev mo = st.mol[st.blk_mol[r]];
  if (((r - mo.blk0) & 1) || r + 1 >= mo.blk1) return;
  const int64_t k0 = st.blk_off[r], k1 = st.blk_off[r + 1];
  const int64_t n = k1 - k0;
  for (int64_t t = threadIdx.x; t < n; t += NT) {
    const double z = fmax(zmax[k0 + t], zmax[k1 + t]);
    zmax[k0 + t] = z;
    zmax[k1 + t] = z;
  }
}

// One workgroup per retained tile of the chunk: B = (w v_tau / 4) d_a Phi, the column operand of the
// meta-GGA Vxc term.
__global__ __launch_bounds__(kG) void k_tscale(StructDev st, int64_t ret0, const double *__restrict__ ctau,
                                              const double *__restrict__ dphi, double *__restrict__ out) {
  const int64_t k = ret0 + blockIdx.x;
  const int j = threadIdx.x;
  const double c = ctau[int64_t(st.ret_r[k]) * kG + j];
  const size_t o = size_t(blockIdx.x) * (kD * kG) + j;
  for (int a = 0; a < kD; ++a) out[o + a * kG] = c * dphi[o + a * kG];
}

// The X stage of grid chunk ci: Phi on its retained tiles, X = D Phi with the rho / grad rho epilogue,
// then the functional (rho, E_xc partials, Z coefficients).  mark(k) records stage event k when the plan
// runs in one chunk.
template <class T, int NPC, class Mark>
void x_stage(const Plan &P, size_t ci, hipStream_t s, Mark &&mark) {
  const EvalDev &E = P.ev;
  const GridChunk &C = P.chunks_h[ci];
  const int64_t nret = C.ret1 - C.ret0, nblk = C.blk1 - C.blk0, nxit = C.xit1 - C.xit0;
  if (nret > 0)
    k_basis<T, NPC><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, static_cast<T *>(E.phi), E.phil, E.phix);
  mark(2);
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
  xa.phil = E.phil;
  xa.phix = E.phix;
  xa.part = E.xpart;
  xa.counters = E.counters;
  xa.t_b = P.opts.t_b;
  xa.t_d = P.opts.t_d;
  xa.q = QArgs{P.xq.order, P.xq.qoff + 9 * ci};
  const int64_t gx = 8 * P.xq.maxlen_h[ci];
  if (nxit > 0) {
    if constexpr (sizeof(T) == 4 && NPC == 0) {
      if (P.gga)
        k_xgemm_f32<true><<<gx, NTX4, 0, s>>>(xa);
      else
        k_xgemm_f32<false><<<gx, NTX4, 0, s>>>(xa);
    } else if constexpr (sizeof(T) == 8) {
      if (P.gga)
        k_xgemm_f64<true><<<gx, NTX4, 0, s>>>(xa);
      else
        k_xgemm_f64<false><<<gx, NTX4, 0, s>>>(xa);
    } else {
      if (P.gga)
        k_xgemm_bf16<true, NPC><<<gx, NTX, 0, s>>>(xa);
      else
        k_xgemm_bf16<false, NPC><<<gx, NTX, 0, s>>>(xa);
    }
    if constexpr (sizeof(T) == 8 && NPC == 0) {
      if (is_mgga_xc(P.opts.xc)) {
        // meta-GGA: the products D d_a Phi on the same items (operand d_a Phi, every retained operand tile
        // with a retained D block: t_d = 0), their pairs counted apart
        XArgs ta = xa;
        ta.phi = E.tdphi;
        ta.t_d = 0.0;
        ta.counters = E.counters + 4;
        for (int a = 0; a < 3; ++a) {
          k_gterm<double><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, a, E.tdphi, nullptr,
                                              nullptr, nullptr, nullptr, nullptr);
          ta.part = E.tpart[a];
          k_xgemm_f64<true><<<gx, NTX4, 0, s>>>(ta);
        }
      }
    }
  }
  mark(3);
  FArgs fa;
  fa.g = P.grid;
  fa.blk_item_off = P.blk_item_off;
  fa.blk0 = C.blk0;
  fa.item0 = C.xit0;
  fa.part = E.xpart;
  fa.coef = E.coef;
  fa.eblk = E.eblk;
  fa.io = E.io;
  fa.counters = E.counters;
  fa.rho_cut = P.opts.rho_cut;
  fa.xc = P.opts.xc;
  fa.gga = P.gga ? 1 : 0;
  for (int a = 0; a < 3; ++a) fa.tpart[a] = E.tpart[a];
  fa.ctau = E.ctau;
  if (nblk > 0) {
    if (P.has_mlp)
      (void)mlp_launch_xfunc(fa, P.mlp, nblk, s);
    else
      k_xfunc<<<nblk, kG, 0, s>>>(fa);
  }
}

// Arguments of a Vxc GEMM launch over the Vxc items of grid chunk ci with operands A (rows) and B.
VArgs v_args(const Plan &P, size_t ci, const void *A, const void *B) {
  const EvalDev &E = P.ev;
  const GridChunk &C = P.chunks_h[ci];
  VArgs va;
  va.st = P.st;
  va.items = P.items;
  va.item0 = C.vit0;
  va.n_items = C.vit1 - C.vit0;
  va.ret0 = C.ret0;
  va.cinfo = P.cinfo;
  va.cioff = P.cioff;
  va.vmoff = P.vmoff;
  va.vm_base = P.vmoff_h[C.blk0];
  va.vmask = E.vmask;
  va.phi = A;
  va.zws = B;
  va.vpart = E.vpart;
  va.vflag = E.vflag;
  va.counters = E.counters;
  va.q = QArgs{P.vq.order, P.vq.qoff + 9 * ci};
  va.accumulate = 0;
  va.keep_diag = 0;
  return va;
}

VMaskArgs m_args(const Plan &P, size_t ci) {
  const EvalDev &E = P.ev;
  const GridChunk &C = P.chunks_h[ci];
  VMaskArgs ma;
  ma.st = P.st;
  ma.cinfo = P.cinfo;
  ma.cioff = P.cioff;
  ma.vmoff = P.vmoff;
  ma.vm_base = P.vmoff_h[C.blk0];
  ma.pair_info = P.pair_info;
  ma.zmax = E.zmax;
  ma.blk0 = C.blk0;
  ma.vmask = E.vmask;
  ma.t_b = P.opts.t_b;
  ma.t_d = P.opts.t_d;
  ma.upper_only = P.gga ? 0 : 1;
  return ma;
}

template <class T, int NPC>
hipError_t body_typed(const Plan &P, bool want_v, hipStream_t s, hipEvent_t *ev) {
  const EvalDev &E = P.ev;
  // stage events: per stage when the grid is processed in one chunk; with several chunks the
  // stages interleave and everything between the D preparation and the final sums is one stage
  const bool one = P.chunks_h.size() == 1;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  };
  auto mark1 = [&](int i) {
    if (one) mark(i);
  };
  mark(0);
  if constexpr (NPC > 0)
    k_dprep_b<NPC><<<P.n_dt, NT, 0, s>>>(P.st.mol, P.n_mol, E.io, P.ao_perm_d, static_cast<unsigned short *>(E.Dt),
                                         E.amax, E.counters);
  else
    k_dprep<T><<<P.n_dt, NT, 0, s>>>(P.st.mol, P.n_mol, E.io, P.ao_perm_d, static_cast<T *>(E.Dt), E.amax, E.counters);
  mark(1);
  if (!one) {
    mark(2);
    mark(3);
    mark(4);
  }
  for (size_t ci = 0; ci < P.chunks_h.size(); ++ci) {
    const GridChunk &C = P.chunks_h[ci];
    const int64_t nret = C.ret1 - C.ret0, nblk = C.blk1 - C.blk0, nvit = C.vit1 - C.vit0;
    x_stage<T, NPC>(P, ci, s, mark1);
    if (want_v && nret > 0) {
      if (P.gga)
        k_zform<T, true><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, static_cast<const T *>(E.phi),
                                             E.phil, static_cast<T *>(E.zws), E.zmax);
      else
        k_zform<T, false><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, static_cast<const T *>(E.phi),
                                              E.phil, static_cast<T *>(E.zws), E.zmax);
    }
    if (want_v && nblk > 0 && P.opts.grid_block == 2 * kG) k_zpair<<<nblk, NT, 0, s>>>(P.st, C.blk0, E.zmax);
    mark1(4);
    if (want_v && nblk > 0) {
      k_vmask<<<nblk, NT, 0, s>>>(m_args(P, ci));
      VArgs va = v_args(P, ci, E.phi, E.zws);
      const int64_t gv = 8 * P.vq.maxlen_h[ci];
      const int64_t nd = P.dchunk_h[ci + 1] - P.dchunk_h[ci];
      const bool diag = sizeof(T) == 4 && nd > 0;
      // k_vdiag needs what k_vmask and the stages before it wrote and shares no output with k_vgemm_f32: it
      // runs on the side stream beside k_vgemm_f32, which joins back before the next use of the workspaces
      if (diag) {
        hipError_t e = hipEventRecord(P.fork_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(P.side_stream, P.fork_ev, 0);
        if (e != hipSuccess) return e;
      }
      if (nvit > 0) {
        if constexpr (sizeof(T) == 4)
          k_vgemm_f32<false><<<gv, NTV4, 0, s>>>(va);
        else
          k_vgemm_f64<false><<<gv, NTV4, 0, s>>>(va);
      }
      if constexpr (sizeof(T) == 8 && NPC == 0) {
        if (is_mgga_xc(P.opts.xc) && nvit > 0 && nret > 0) {
          // meta-GGA: + sum_a d_a Phi (w v_tau / 4 d_a Phi)^T over every pair of retained tiles of a block
          VMaskArgs ma = m_args(P, ci);
          ma.t_b = 0.0;
          ma.t_d = 0.0;
          k_vmask<<<nblk, NT, 0, s>>>(ma);
          VArgs tv = v_args(P, ci, E.tdphi, E.tB);
          tv.accumulate = 1;
          tv.counters = E.counters + 4;
          for (int a = 0; a < 3; ++a) {
            k_gterm<double><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, a, E.tdphi, nullptr,
                                                nullptr, nullptr, nullptr, nullptr);
            k_tscale<<<nret, kG, 0, s>>>(P.st, C.ret0, E.ctau, E.tdphi, E.tB);
            k_vgemm_f64<false><<<gv, NTV4, 0, s>>>(tv);
          }
        }
      }
      if (diag) {
        VDArgs da;
        da.st = P.st;
        da.items = P.items;
        da.ditems = P.ditems + P.dchunk_h[ci];
        da.n = nd;
        da.ret0 = C.ret0;
        da.cinfo = P.cinfo;
        da.cioff = P.cioff;
        da.vmoff = P.vmoff;
        da.vm_base = P.vmoff_h[C.blk0];
        da.vmask = E.vmask;
        da.phi = static_cast<const float *>(E.phi);
        da.phil = E.phil;
        da.zws = static_cast<const float *>(E.zws);
        da.vpart = E.vpart;
        da.counters = E.counters;
        k_vdiag<<<nd, NT, 0, P.side_stream>>>(da);
        hipError_t e = hipEventRecord(P.join_ev, P.side_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, P.join_ev, 0);
        if (e != hipSuccess) return e;
      }
    }
  }
  mark(5);
  if (want_v) {
    k_vreduce<<<dim3(P.n_pairs, 64), NT, 0, s>>>(P.pair_ptr, P.pair_items, P.pair_info, P.st.mol, E.vflag, E.vpart,
                                                E.mfull);
    const int ncol = (P.max_nao + NT - 1) / NT;
    k_vsym<<<int64_t(P.n_ao) * ncol, NT, 0, s>>>(P.st.mol, P.n_mol, ncol, E.mfull, P.ao_perm_d, P.gga ? 1 : 0, E.io);
  }
  k_esum<<<P.n_mol, NT, 0, s>>>(P.st.mol, E.eblk, E.io);
  mark(6);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Nuclear gradient of E_xc with the grid held fixed (FP64 plans of one molecule):
//   dE/dR_Aa = -2 sum_{mu on A} sum_nu D_{mu nu} K^a_{mu nu},  K^a = (d_a Phi) W^T + Q^a Phi^T,
//   W = c0 Phi + sum_b c_b d_b Phi,  Q^a = sum_b c_b d_a d_b Phi,  c0 = w v_rho,  c_b = 2 w v_sigma d_b rho.
// The products run on k_vgemm_f64 over the Vxc work items, tile pairs (p, q) of a product A B^T executing
// at block r when (p, r), (q, r) are retained, a_pq >= t_b and a_pq max|A_pr| max|B_qr| >= t_d; each
// item's partial is contracted with D at once.
// LDA plans hold the chunk pairs pc <= qc only: there the pairs pc < qc also run the product with
// its operands exchanged, W (d_a Phi)^T = (K^a)^T for the transposed chunk pair, contracted along columns.
// ------------------------------------------------------------------------------------------------

// One workgroup per grid block of the chunk: the executable tile pairs of a gradient product A B^T as
// 16-bit masks per (row chunk, column chunk) pair: (p, r), (q, r) retained, a_pq >= t_b and the bound of
// the triple's D-contracted contribution a_pq max|A_pr| max|B_qr| >= t_d (the pair filter of eq.
// block_pair_filter for the three factors; mA, mB: tile maxima indexed by retained tile - ret0).
// skip_diag: no pair of a diagonal chunk pair (the exchanged-operand pass of LDA plans).
__global__ __launch_bounds__(NT) void k_gmask(VMaskArgs A, const double *__restrict__ amax, int skip_diag,
                                             const double *__restrict__ mA, const double *__restrict__ mB,
                                             int64_t ret0) {
  const int64_t r = A.blk0 + blockIdx.x;
  const MolDev mo = A.st.mol[A.st.blk_mol[r]];
  const int *ci = A.cinfo + A.cioff[r];
  const int64_t k0 = A.st.blk_off[r] - ret0;
  unsigned short *out = A.vmask + (A.vmoff[r] - A.vm_base);
  for (int pr = threadIdx.x; pr < mo.npairs; pr += NT) {
    const int pc = A.pair_info[3 * (mo.pair0 + pr)], qc = A.pair_info[3 * (mo.pair0 + pr) + 1];
    const int ip = ci[pc], iq = ci[qc];
    int mask = 0;
    if (!(skip_diag && pc == qc)) {
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        if (!((ip >> ww) & 1)) continue;
        const double ma = mA[k0 + tile_pos(ip, ww)];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (!((iq >> jj) & 1)) continue;
          const size_t t = size_t(mo.dt0) + size_t(4 * pc + ww) * mo.nt + (4 * qc + jj);
          const double a = amax[t];
          if (a >= A.t_b && a * ma * mB[k0 + tile_pos(iq, jj)] >= A.t_d) mask |= 1 << (4 * ww + jj);
        }
      }
    }
    out[pr] = (unsigned short)mask;
  }
}

// The per-AO gradient sums of the 128 AOs of row chunk c over the items of the chunk's pairs, in a fixed
// order: the pairs of chunk c in pair order -- (pc, c) for pc < c (LDA plans, which hold pc <= qc: its
// columns), then (c, qc) (its rows); pair index pc nc + qc (GGA) or pc nc - pc (pc - 1) / 2 + (qc - pc)
// (LDA) -- and a pair's items in segment order.  Slots per item: 2a and 2a+1 for component a; GGA: both
// are row sums of items with pc = c; LDA: slot 2a row sums of items with pc = c, slot 2a+1 column sums of
// items with qc = c > pc.  That sequence is cut into kGSeg equal parts: k_greduce_part sums part s of
// chunk c (one workgroup per (c, s)), k_greduce the kGSeg partial sums of each AO in order.

// calls f(item, column) for the items of positions [lo, hi) of chunk c's sequence; returns its length
template <class F>
__device__ __forceinline__ int greduce_walk(const MolDev &mo, const int *pair_ptr, int lda, int c, int lo, int hi,
                                            F &&f) {
  const int nc = mo.nc;
  int pos = 0;
  auto pair = [&](int pr, bool col) {
    const int k0 = pair_ptr[pr], n = pair_ptr[pr + 1] - k0;
    const int a = max(lo - pos, 0), b = min(hi - pos, n);
    for (int k = a; k < b; ++k) f(k0 + k, col);
    pos += n;
  };
  if (lda)
    for (int pc = 0; pc < c; ++pc) pair(mo.pair0 + pc * nc - pc * (pc - 1) / 2 + (c - pc), true);
  for (int qc = lda ? c : 0; qc < nc; ++qc) pair(mo.pair0 + (lda ? c * nc - c * (c - 1) / 2 + (qc - c) : c * nc + qc), false);
  return pos;
}

__global__ __launch_bounds__(kG) void k_greduce_part(const MolDev *__restrict__ mol, const int *__restrict__ pair_ptr,
                                                    const int *__restrict__ pair_items,
                                                    const double *__restrict__ gitem, int lda,
                                                    double *__restrict__ gpart) {
  const MolDev mo = mol[0];
  const int c = blockIdx.x / kGSeg, sg = blockIdx.x % kGSeg, i = threadIdx.x;
  const int n = greduce_walk(mo, pair_ptr, lda, c, 0, 0, [](int, bool) {});
  const int lo = int(int64_t(n) * sg / kGSeg), hi = int(int64_t(n) * (sg + 1) / kGSeg);
  double s[3] = {0.0, 0.0, 0.0};
  greduce_walk(mo, pair_ptr, lda, c, lo, hi, [&](int k, bool col) {
    const double *gi = gitem + size_t(pair_items[k]) * 6 * 128 + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (col) {
        s[a] += gi[(2 * a + 1) * 128];
      } else {
        s[a] += gi[(2 * a) * 128];
        if (!lda) s[a] += gi[(2 * a + 1) * 128];
      }
    }
  });
#pragma unroll
  for (int a = 0; a < 3; ++a) gpart[(size_t(blockIdx.x) * 3 + a) * 128 + i] = s[a];
}

__global__ __launch_bounds__(kG) void k_greduce(const double *__restrict__ gpart, double *__restrict__ gao, int ld) {
  const int c = blockIdx.x, i = threadIdx.x;
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int sg = 0; sg < kGSeg; ++sg) s += gpart[((size_t(c) * kGSeg + sg) * 3 + a) * 128 + i];
    gao[size_t(a) * ld + size_t(c) * 128 + i] = s;
  }
}

// One thread per (atom, component): dE/dR_Aa = -2 sum over the atom's AOs (internal order) of the
// per-AO sums.
__global__ __launch_bounds__(NT) void k_gatom(const int *__restrict__ ao_atom, int n_ao, int n_atoms,
                                             const double *__restrict__ gao, int ld, double *__restrict__ grad) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= 3 * n_atoms) return;
  const int A = t / 3, a = t % 3;
  double s = 0.0;
  for (int mu = 0; mu < n_ao; ++mu)
    if (ao_atom[mu] == A) s += gao[size_t(a) * ld + mu];
  grad[t] = -2.0 * s;
}

// The nuclear gradient on an FP64 plan (T = double: FP64 operands) or an FP32 plan (T = float: the X
// product and the gradient products on FP32 MFMA with FP64 running sums, including the products' diagonal
// tile pairs; the contraction with D in FP64).
template <class T>
hipError_t grad_body(const Plan &P, double *grad, hipStream_t s) {
  constexpr bool kF64 = std::is_same<T, double>::value;
  const EvalDev &E = P.ev;
  const MolDev &mo = P.mols_h[0];
  auto none = [](int) {};
  k_dprep<T><<<P.n_dt, NT, 0, s>>>(P.st.mol, P.n_mol, E.io, P.ao_perm_d, static_cast<T *>(E.Dt), E.amax,
                                   E.counters);
  double *Dt = kF64 ? static_cast<double *>(E.Dt) : P.grad_ws.gD;
  if (!kF64) k_dprep<double><<<P.n_dt, NT, 0, s>>>(P.st.mol, P.n_mol, E.io, P.ao_perm_d, Dt, E.amax, E.counters);
  T *A = reinterpret_cast<T *>(P.grad_ws.gA);
  T *Q = reinterpret_cast<T *>(P.grad_ws.gQ);
  T *Z = static_cast<T *>(E.zws);
  for (size_t ci = 0; ci < P.chunks_h.size(); ++ci) {
    const GridChunk &C = P.chunks_h[ci];
    const int64_t nret = C.ret1 - C.ret0, nblk = C.blk1 - C.blk0, nvit = C.vit1 - C.vit0;
    x_stage<T, 0>(P, ci, s, none);
    if (nret == 0 || nvit == 0) continue;
    const int64_t gv = 8 * P.vq.maxlen_h[ci];
    const double *Am = P.grad_ws.gAmax, *Qm = P.grad_ws.gQmax, *Wm = P.grad_ws.gWmax;   // tile maxima
    const double *Pm = P.st.bphi + C.ret0;
    auto product = [&](const void *opA, const void *opB, const double *mA, const double *mB, int skip_diag,
                       int mode, int slot) {
      k_gmask<<<nblk, NT, 0, s>>>(m_args(P, ci), E.amax, skip_diag, mA, mB, C.ret0);
      VArgs va = v_args(P, ci, opA, opB);
      va.gc = GContract{P.pair_info, Dt, P.grad_ws.gitem, mode, slot};
      if (kF64) {
        k_vgemm_f64<true><<<gv, NTV4, 0, s>>>(va);
      } else {
        va.keep_diag = 1;
        k_vgemm_f32<true><<<gv, NTV4, 0, s>>>(va);
      }
    };
    for (int ax = 0; ax < 3; ++ax) {
      k_gterm<T><<<nret, kG, 0, s>>>(P.basis, P.grid, P.st, C.ret0, E.coef, ax, A, P.gga ? Q : nullptr,
                                     ax == 0 ? Z : nullptr, P.grad_ws.gAmax, P.grad_ws.gQmax, P.grad_ws.gWmax);
      product(A, Z, Am, Wm, 0, 0, 2 * ax);                  // (d_a Phi) W^T
      if (P.gga) {
        product(Q, E.phi, Qm, Pm, 0, 0, 2 * ax + 1);        // Q^a Phi^T
      } else {
        product(Z, A, Wm, Am, 1, 1, 2 * ax + 1);            // W (d_a Phi)^T of the pairs pc < qc
      }
    }
  }
  k_esum<<<P.n_mol, NT, 0, s>>>(P.st.mol, E.eblk, E.io);
  const int ld = mo.nc * 128;
  k_greduce_part<<<mo.nc * kGSeg, kG, 0, s>>>(P.st.mol, P.pair_ptr, P.pair_items, P.grad_ws.gitem, P.gga ? 0 : 1,
                                              P.grad_ws.gpart);
  k_greduce<<<mo.nc, kG, 0, s>>>(P.grad_ws.gpart, P.grad_ws.gao, ld);
  k_gatom<<<(3 * P.n_atoms0 + NT - 1) / NT, NT, 0, s>>>(P.ao_atom, mo.n_ao, P.n_atoms0, P.grad_ws.gao, ld,
                                                       grad);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_screen(const BasisDev &b, const GridDev &g, const int *cand_p, const int64_t *cand_r,
                         int64_t n_cand, bool gga, double *out_b, double *out_g, hipStream_t s) {
  if (n_cand <= 0) return hipSuccess;
  k_screen<<<n_cand, kG, 0, s>>>(b, g, cand_p, cand_r, n_cand, gga ? 1 : 0, out_b, out_g);
  return hipGetLastError();
}

hipError_t launch_begin(const Plan &P, const IoDev &io, hipStream_t s) {
  k_begin<<<1, NT, 0, s>>>(P.ev.io, io, P.ev.counters);
  return hipGetLastError();
}

hipError_t launch_grad(const Plan &P, double *grad, hipStream_t s) {
  return P.opts.prec == KLDI_PREC_FP64 ? grad_body<double>(P, grad, s) : grad_body<float>(P, grad, s);
}

hipError_t launch_body(const Plan &P, bool want_v, hipStream_t s, hipEvent_t *ev) {
  switch (P.opts.prec) {
    case KLDI_PREC_FP64: return body_typed<double, 0>(P, want_v, s, ev);
    case KLDI_PREC_BF16X3: return body_typed<float, 2>(P, want_v, s, ev);
    case KLDI_PREC_BF16X6: return body_typed<float, 3>(P, want_v, s, ev);
    default: return body_typed<float, 0>(P, want_v, s, ev);
  }
}

}  // namespace kldi
