// Learned functional surrogate: a 2-64-64-64-3 SiLU network that stands in for the GGA functional
// evaluation.  Training runs here too: forward + back-propagation kernels (FP32) that write
// per-workgroup partial gradients, a fixed-order reduction fused with the Adam update, and BF16
// inference on MFMA (v_mfma_f32_16x16x32_bf16) for the two 64 x 64 layers.
//
// Inputs: x = (n(log rho), n(log sigma)), n(.) the affine map of the training range box onto
// [-1, 1].  Outputs: three standardised heads y; t = y * t_std + t_mean are f / rho^(4/3),
// v_rho / rho^(1/3) and v_sigma * rho^(4/3).  Points with rho < rho_min or features outside the box
// fall back to the analytic functional.
#include <mutex>

#include <hip/hip_bf16.h>

#include "device.h"

namespace kldi {
namespace {
using namespace dev;

constexpr int W = kMlpWidth;     // 64
constexpr int TP = 64;           // points per training workgroup
constexpr int LDH = W + 1;       // LDS row stride of FP32 activation tiles

__device__ __forceinline__ float silu_f(float a) { return a / (1.0f + __expf(-a)); }
__device__ __forceinline__ float dsilu_f(float a) {
  const float s = 1.0f / (1.0f + __expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

// parameter offsets (row-major W[out][in]): W1 b1 W2 b2 W3 b3 W4 b4
constexpr int oW1 = 0, ob1 = oW1 + W * 2, oW2 = ob1 + W, ob2 = oW2 + W * W, oW3 = ob2 + W, ob3 = oW3 + W * W,
              oW4 = ob3 + W, ob4 = oW4 + 3 * W;
static_assert(ob4 + 3 == kMlpParams, "parameter layout");

// ------------------------------------------------------------------------------------------------
// training: one workgroup per TP points of the batch; writes the batch-mean-loss gradient of its
// points (scaled by 1 / (3 B)) and its share of the loss
// ------------------------------------------------------------------------------------------------
struct GradArgs {
  const float *theta;      // [kMlpParams]
  const float *x;          // [n * 2] features
  const float *t;          // [n * 3] standardised targets
  int64_t n;               // points in the data set
  int64_t start, count;    // this batch: permuted positions start .. start + count - 1
  int64_t perm_a, perm_b;  // permutation i -> (perm_a * i + perm_b) mod n
  float *gpart;            // [n_wg * kMlpParams]
  double *lpart;           // [n_wg]
};

__global__ __launch_bounds__(256) void k_mlp_grad(GradArgs A) {
  __shared__ float xs[TP][2], ts[TP][3], gy[TP][3];
  __shared__ float A1[TP][LDH], A2[TP][LDH], A3[TP][LDH], Hs[TP][LDH];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const float *th = A.theta;
  const int64_t p0 = int64_t(blockIdx.x) * TP;
  const int np = int(min<int64_t>(TP, A.count - p0));
  if (tid < TP) {
    float x0 = 0.f, x1 = 0.f, t0 = 0.f, t1 = 0.f, t2 = 0.f;
    if (tid < np) {
      const int64_t pos = A.start + p0 + tid;
      const int64_t i = ((A.perm_a % A.n) * (pos % A.n) + A.perm_b) % A.n;   // n < 2^31
      x0 = A.x[2 * i];
      x1 = A.x[2 * i + 1];
      t0 = A.t[3 * i];
      t1 = A.t[3 * i + 1];
      t2 = A.t[3 * i + 2];
    }
    xs[tid][0] = x0;
    xs[tid][1] = x1;
    ts[tid][0] = t0;
    ts[tid][1] = t1;
    ts[tid][2] = t2;
  }
  __syncthreads();
  // forward
  for (int e = tid; e < TP * W; e += 256) {
    const int p = e / W, n = e % W;
    A1[p][n] = th[oW1 + 2 * n] * xs[p][0] + th[oW1 + 2 * n + 1] * xs[p][1] + th[ob1 + n];
    Hs[p][n] = silu_f(A1[p][n]);
  }
  __syncthreads();
  auto dense = [&](int oW, int ob, float (*out)[LDH]) {
    // out[p][n] = sum_k W[n][k] Hs[p][k] + b[n]
    const int n = tid % W, pg = tid / W;
    float wr[W];
#pragma unroll
    for (int k = 0; k < W; ++k) wr[k] = th[oW + n * W + k];
    for (int p = pg * 16; p < pg * 16 + 16; ++p) {
      float acc = th[ob + n];
#pragma unroll
      for (int k = 0; k < W; ++k) acc += wr[k] * Hs[p][k];
      out[p][n] = acc;
    }
  };
  dense(oW2, ob2, A2);
  __syncthreads();
  for (int e = tid; e < TP * W; e += 256) Hs[e / W][e % W] = silu_f(A2[e / W][e % W]);
  __syncthreads();
  dense(oW3, ob3, A3);
  __syncthreads();
  for (int e = tid; e < TP * W; e += 256) Hs[e / W][e % W] = silu_f(A3[e / W][e % W]);
  __syncthreads();
  const float scale = 2.0f / (3.0f * float(A.count));
  double lsum = 0.0;
  if (tid < 3 * TP) {
    const int p = tid / 3, o = tid % 3;
    float y = th[ob4 + o];
    for (int k = 0; k < W; ++k) y += th[oW4 + o * W + k] * Hs[p][k];
    const float r = (p < np) ? (y - ts[p][o]) : 0.f;
    gy[p][o] = scale * r;
    lsum = double(r) * double(r);
  }
  red[tid] = lsum;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0) A.lpart[blockIdx.x] = red[0];
  float *g = A.gpart + size_t(blockIdx.x) * kMlpParams;
  // output layer: g_W4[o][k] = sum_p gy[p][o] h3[p][k], g_b4
  if (tid < 3 * W) {
    const int o = tid / W, k = tid % W;
    float s = 0.f;
    for (int p = 0; p < TP; ++p) s += gy[p][o] * Hs[p][k];
    g[oW4 + o * W + k] = s;
  }
  if (tid < 3) {
    float s = 0.f;
    for (int p = 0; p < TP; ++p) s += gy[p][tid];
    g[ob4 + tid] = s;
  }
  __syncthreads();
  // D3 = (gy W4) . silu'(A3), stored over A3
  for (int e = tid; e < TP * W; e += 256) {
    const int p = e / W, k = e % W;
    const float e3 = gy[p][0] * th[oW4 + k] + gy[p][1] * th[oW4 + W + k] + gy[p][2] * th[oW4 + 2 * W + k];
    A3[p][k] = e3 * dsilu_f(A3[p][k]);
  }
  __syncthreads();
  // hidden layers: g_W[n][k] = sum_p D[p][n] Hin[p][k], g_b[n] = sum_p D[p][n]; Din = (D W) . silu'(Ain)
  auto back = [&](float (*Dl)[LDH], float (*Ain)[LDH], int oW, int ob) {
    for (int e = tid; e < TP * W; e += 256) Hs[e / W][e % W] = silu_f(Ain[e / W][e % W]);
    __syncthreads();
    for (int e = tid; e < W * W; e += 256) {
      const int n = e / W, k = e % W;
      float s = 0.f;
      for (int p = 0; p < TP; ++p) s += Dl[p][n] * Hs[p][k];
      g[oW + n * W + k] = s;
    }
    if (tid < W) {
      float s = 0.f;
      for (int p = 0; p < TP; ++p) s += Dl[p][tid];
      g[ob + tid] = s;
    }
    __syncthreads();
    // Din[p][k] = (sum_n Dl[p][n] W[n][k]) * silu'(Ain[p][k]) -- written over Ain
    {
      const int k = tid % W, pg = tid / W;
      float wc[W];
#pragma unroll
      for (int n = 0; n < W; ++n) wc[n] = th[oW + n * W + k];
      for (int p = pg * 16; p < pg * 16 + 16; ++p) {
        float acc = 0.f;
#pragma unroll
        for (int n = 0; n < W; ++n) acc += Dl[p][n] * wc[n];
        Ain[p][k] = acc * dsilu_f(Ain[p][k]);
      }
    }
    __syncthreads();
  };
  back(A3, A2, oW3, ob3);   // A2 now holds D2
  back(A2, A1, oW2, ob2);   // A1 now holds D1
  // first layer: g_W1[n][i] = sum_p D1[p][n] x[p][i], g_b1
  if (tid < W) {
    float s0 = 0.f, s1 = 0.f, sb = 0.f;
    for (int p = 0; p < TP; ++p) {
      s0 += A1[p][tid] * xs[p][0];
      s1 += A1[p][tid] * xs[p][1];
      sb += A1[p][tid];
    }
    g[oW1 + 2 * tid] = s0;
    g[oW1 + 2 * tid + 1] = s1;
    g[ob1 + tid] = sb;
  }
}

// Fixed-order FP64 sum of the workgroup partial gradients, then one Adam step (FP32 master
// weights) and the BF16 copy used for inference.
__global__ __launch_bounds__(256) void k_mlp_adam(float *theta, float *m, float *v, __hip_bfloat16 *theta_b,
                                                  const float *gpart, int n_wg, float lr, float c1, float c2,
                                                  float *grad_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kMlpParams) return;
  double s = 0.0;
  for (int w = 0; w < n_wg; ++w) s += double(gpart[size_t(w) * kMlpParams + i]);
  const float gi = float(s);
  if (grad_out) grad_out[i] = gi;
  if (lr <= 0.f) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  theta[i] = th;
  theta_b[i] = __float2bfloat16(th);
}

// the batch-mean loss of n points from the workgroup shares, written (not accumulated) to *out
__global__ __launch_bounds__(256) void k_loss_mean(const double *lpart, int n_wg, int64_t n, double *out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n_wg; i += 256) a += lpart[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] / (3.0 * double(n));
}

__global__ __launch_bounds__(256) void k_mlp_tobf16(const float *theta, __hip_bfloat16 *theta_b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kMlpParams) theta_b[i] = __float2bfloat16(theta[i]);
}

__global__ __launch_bounds__(256) void k_loss_sum(const double *lpart, int n, double *out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += lpart[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out += s[0];
}

// ------------------------------------------------------------------------------------------------
// data preparation: features and standardised targets of the analytic functional
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_flags(const double *rho, int64_t n, double rho_min, int *flag,
                                                   int *blk_count) {
  __shared__ int s[4];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int f = (i < n && rho[i] >= rho_min) ? 1 : 0;
  if (i < n) flag[i] = f;
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) blk_count[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// order-preserving compaction with per-block offsets (parallel addressing)
__global__ __launch_bounds__(256) void k_mlp_compact(const double *rho, const double *sigma, int64_t n, const int *flag,
                                                     const int64_t *blk_off, double *rho_c, double *sigma_c) {
  __shared__ int s_w[4];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int f = (i < n) ? flag[i] : 0;
  int tot;
  const int pos = block_scan(f, s_w, &tot);
  if (f) {
    rho_c[blk_off[blockIdx.x] + pos] = rho[i];
    sigma_c[blk_off[blockIdx.x] + pos] = sigma[i];
  }
}

__global__ __launch_bounds__(256) void k_mlp_logrange(const double *rho, const double *sigma, int64_t n, double *out) {
  // per-block (min, max) of log rho and log sigma -> out[block * 4 + ...]
  __shared__ double s[4][256];
  double a0 = 1e300, a1 = -1e300, b0 = 1e300, b1 = -1e300;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double lr = log(rho[i]), ls = log(fmax(sigma[i], 1e-30));
    a0 = fmin(a0, lr);
    a1 = fmax(a1, lr);
    b0 = fmin(b0, ls);
    b1 = fmax(b1, ls);
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  s[2][threadIdx.x] = b0;
  s[3][threadIdx.x] = b1;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + k]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + k]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + k]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

// features, raw targets t = (f / rho^(4/3), v_rho / rho^(1/3), v_sigma rho^(4/3)), and per-block sums
// of t and t^2 for the standardisation
__global__ __launch_bounds__(256) void k_mlp_data(const double *rho, const double *sigma, int64_t n, int xc,
                                                  double lr0, double lr1, double ls0, double ls1, float *x, double *traw,
                                                  double *stat) {
  __shared__ double s[6][256];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double r = rho[i], sg = sigma[i];
    const double lr = log(r), ls = log(fmax(sg, 1e-30));
    x[2 * i] = float(2.0 * (lr - lr0) / (lr1 - lr0) - 1.0);
    x[2 * i + 1] = float(2.0 * (ls - ls0) / (ls1 - ls0) - 1.0);
    const Xc f = xc_eval(xc, r, sg, 0.0);
    const double r13 = cbrt(r), r43 = r * r13;
    const double t[3] = {f.f / r43, f.vr / r13, f.vs * r43};
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      traw[3 * i + o] = t[o];
      acc[o] += t[o];
      acc[3 + o] += t[o] * t[o];
    }
  }
#pragma unroll
  for (int o = 0; o < 6; ++o) s[o][threadIdx.x] = acc[o];
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k)
#pragma unroll
      for (int o = 0; o < 6; ++o) s[o][threadIdx.x] += s[o][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 6) stat[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_mlp_standardise(const double *traw, int64_t n, double m0, double m1, double m2,
                                                         double s0, double s1, double s2, float *t) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  t[3 * i] = float((traw[3 * i] - m0) / s0);
  t[3 * i + 1] = float((traw[3 * i + 1] - m1) / s1);
  t[3 * i + 2] = float((traw[3 * i + 2] - m2) / s2);
}

// ------------------------------------------------------------------------------------------------
// inference on 128 points per workgroup (4 waves): layers 2 and 3 on BF16 MFMA, FP32 accumulation.
// Lane l of a 16x16x32 BF16 MFMA supplies A[l%16][8(l/16)+j] and B[8(l/16)+j][l%16] (j = 0..7) and
// holds C[4(l/16)+v][l%16].
// ------------------------------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int LDB16 = W + 8;   // bf16 row stride of activation tiles (16-byte aligned rows)

struct __align__(16) MlpShared {
  __hip_bfloat16 h[2][128][LDB16];
};

// x[p][2] (features) of the workgroup's 128 points are in xs; writes y[p][3] (standardised heads)
__device__ void mlp_block(const MlpDev &m, const float (*xs)[2], float (*ys)[3], MlpShared &S) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const __hip_bfloat16 *tb = reinterpret_cast<const __hip_bfloat16 *>(m.theta_b);
  for (int e = tid; e < 128 * W; e += 256) {
    const int p = e / W, n = e % W;
    const float a = __bfloat162float(tb[oW1 + 2 * n]) * xs[p][0] + __bfloat162float(tb[oW1 + 2 * n + 1]) * xs[p][1] +
                    m.bias[ob1 + n];
    S.h[0][p][n] = __float2bfloat16(silu_f(a));
  }
  __syncthreads();
  for (int layer = 0; layer < 2; ++layer) {
    const int oW = layer == 0 ? oW2 : oW3, ob = layer == 0 ? ob2 : ob3;
    const int in = layer, out = layer ^ 1;
    f32x4 acc[2][4];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 a[2], b[4];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
        a[ti] = *reinterpret_cast<const bf16x8 *>(&S.h[in][32 * w + 16 * ti + (l & 15)][32 * ks + 8 * (l >> 4)]);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
        b[tj] = *reinterpret_cast<const bf16x8 *>(tb + oW + (16 * tj + (l & 15)) * W + 32 * ks + 8 * (l >> 4));
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = 32 * w + 16 * ti + 4 * (l >> 4) + v, n = 16 * tj + (l & 15);
          S.h[out][p][n] = __float2bfloat16(silu_f(acc[ti][tj][v] + m.bias[ob + n]));
        }
    __syncthreads();
  }
  if (tid < 128) {
    float y[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      float s = m.bias[ob4 + o];
      for (int k = 0; k < W; ++k) s += __bfloat162float(tb[oW4 + o * W + k]) * __bfloat162float(S.h[0][tid][k]);
      y[o] = s;
    }
    ys[tid][0] = y[0];
    ys[tid][1] = y[1];
    ys[tid][2] = y[2];
  }
  __syncthreads();
}

// features of one point; false when the network does not cover it
__device__ __forceinline__ bool mlp_features(const MlpDev &m, double rho, double sigma, float *x) {
  const double *box = m.stats;
  if (!(rho >= m.stats[10])) return false;
  const double lr = log(rho), ls = log(fmax(sigma, 1e-30));
  const double x0 = 2.0 * (lr - box[0]) / (box[1] - box[0]) - 1.0;
  const double x1 = 2.0 * (ls - box[2]) / (box[3] - box[2]) - 1.0;
  x[0] = float(x0);
  x[1] = float(x1);
  return x0 >= -1.0 && x0 <= 1.0 && x1 >= -1.0 && x1 <= 1.0;
}

__device__ __forceinline__ Xc mlp_output(const MlpDev &m, double rho, const float *y) {
  const double r13 = cbrt(rho), r43 = rho * r13;
  const double *tmean = m.stats + 4, *tstd = m.stats + 7;
  const double t0 = double(y[0]) * tstd[0] + tmean[0];
  const double t1 = double(y[1]) * tstd[1] + tmean[1];
  const double t2 = double(y[2]) * tstd[2] + tmean[2];
  return Xc{t0 * r43, t1 * r13, t2 / r43};
}

// array form: f, v_rho, v_sigma at n points; used[i] = 1 where the network was evaluated
__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const double *rho, const double *sigma, int64_t n, int xc,
                                                     double *f, double *vr, double *vs, int *used) {
  __shared__ float xs[128][2], ys[128][3];
  __shared__ int ok[128];
  __shared__ MlpShared S;
  const int64_t i = int64_t(blockIdx.x) * 128 + (threadIdx.x & 127);
  if (threadIdx.x < 128) {
    float x[2] = {0.f, 0.f};
    ok[threadIdx.x] = (i < n) ? mlp_features(m, rho[i], sigma[i], x) : 0;
    xs[threadIdx.x][0] = x[0];
    xs[threadIdx.x][1] = x[1];
  }
  __syncthreads();
  mlp_block(m, xs, ys, S);
  if (threadIdx.x < 128 && i < n) {
    const Xc r = ok[threadIdx.x] ? mlp_output(m, rho[i], ys[threadIdx.x]) : xc_eval(xc, rho[i], sigma[i], 0.0);
    f[i] = r.f;
    vr[i] = r.vr;
    vs[i] = r.vs;
    if (used) used[i] = ok[threadIdx.x];
  }
}

// The functional stage with the surrogate: one workgroup (4 waves) per grid block; rho and grad rho
// as in k_xfunc, then the network on the covered points and the analytic functional elsewhere.
__global__ __launch_bounds__(256) void k_xfunc_mlp(FArgs A, MlpDev m) {
  __shared__ float xs[128][2], ys[128][3];
  __shared__ int ok[128];
  __shared__ double rs[128], sg[128], gs[3][128], s_red[128];
  __shared__ MlpShared S;
  const int64_t r = A.blk0 + blockIdx.x;
  const int j = threadIdx.x;
  if (j < kG) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t it = A.blk_item_off[r]; it < A.blk_item_off[r + 1]; ++it) {
      const double *pp = A.part + size_t(it - A.item0) * (4 * kG) + j;
      s[0] += pp[0];
      s[1] += pp[kG];
      s[2] += pp[2 * kG];
      s[3] += pp[3 * kG];
    }
    rs[j] = s[0];
    gs[0][j] = s[1];
    gs[1][j] = s[2];
    gs[2][j] = s[3];
    sg[j] = s[1] * s[1] + s[2] * s[2] + s[3] * s[3];
    float x[2] = {0.f, 0.f};
    ok[j] = (s[0] > A.rho_cut) && mlp_features(m, s[0], sg[j], x);
    xs[j][0] = x[0];
    xs[j][1] = x[1];
  }
  __syncthreads();
  mlp_block(m, xs, ys, S);
  if (j < kG) {
    const int64_t ip = r * kG + j;
    const double rho = rs[j], sigma = sg[j];
    const Xc f = ok[j] ? mlp_output(m, rho, ys[j]) : xc_eval(A.xc, rho, sigma, A.rho_cut);
    const double wgt = A.g.w[ip];
    const int64_t o = A.g.orig[ip];
    double *rho_out = A.io->rho, *sigma_out = A.io->sigma;
    if (rho_out && o >= 0) rho_out[o] = rho;
    if (sigma_out && o >= 0) sigma_out[o] = sigma;
    double *cf = A.coef + size_t(ip) * 4;
    cf[0] = 0.5 * wgt * f.vr;
    cf[1] = 2.0 * wgt * f.vs * gs[0][j];
    cf[2] = 2.0 * wgt * f.vs * gs[1][j];
    cf[3] = 2.0 * wgt * f.vs * gs[2][j];
    s_red[j] = wgt * f.f;
  }
  __syncthreads();
  for (int k = kG / 2; k > 0; k >>= 1) {
    if (j < k) s_red[j] += s_red[j + k];
    __syncthreads();
  }
  if (j == 0) A.eblk[r] = s_red[0];
  // points evaluated by the network (real points only)
  if (j < kG) {
    const unsigned long long bal = __ballot(ok[j] && A.g.orig[r * kG + j] >= 0);
    if ((j & 63) == 0 && bal) atomicAdd(&A.counters[3], (unsigned long long)__popcll(bal));
  }
}

// analytic functional on arrays
__global__ __launch_bounds__(256) void k_xc_arrays(int xc, const double *rho, const double *sigma, int64_t n,
                                                   double rho_cut, double *f, double *vr, double *vs) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const Xc r = xc_eval(xc, rho[i], sigma ? sigma[i] : 0.0, rho_cut);
  f[i] = r.f;
  vr[i] = r.vr;
  if (vs) vs[i] = r.vs;
}

}  // namespace

// ---- the allocation-free training step's scratch: the per-workgroup partial gradients and loss
// shares of one batch of at most kMlpStaticMaxPoints points, in a file-scope device array.  Each GPU
// holds its own copy until the process ends; its address on the current device is taken once with
// hipGetSymbolAddress (the array's name is only a host-side stand-in) and kept per device.
constexpr int kStaticWg = int(kMlpStaticMaxPoints / TP);
constexpr size_t kScratchGrad = size_t(kStaticWg) * kMlpParams * sizeof(float);
constexpr size_t kScratchBytes = kScratchGrad + size_t(kStaticWg) * sizeof(double);
static_assert(kMlpStaticMaxPoints % TP == 0 && kScratchGrad % 8 == 0, "scratch layout");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call per device)
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

size_t mlp_static_scratch_bytes() { return kScratchBytes; }

// ---- launchers (declared in kldi_impl.h)
hipError_t mlp_launch_grad(const float *theta, const float *x, const float *t, int64_t n, int64_t start, int64_t count,
                           int64_t pa, int64_t pb, float *gpart, double *lpart, hipStream_t s) {
  GradArgs A{theta, x, t, n, start, count, pa, pb, gpart, lpart};
  const int nwg = int((count + TP - 1) / TP);
  k_mlp_grad<<<nwg, 256, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t mlp_launch_adam(float *theta, float *m, float *v, void *theta_b, const float *gpart, int n_wg, float lr,
                           int step, float *grad_out, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, float(step)), c2 = 1.f - powf(0.999f, float(step));
  k_mlp_adam<<<(kMlpParams + 255) / 256, 256, 0, s>>>(theta, m, v, static_cast<__hip_bfloat16 *>(theta_b), gpart, n_wg,
                                                     lr, c1, c2, grad_out);
  return hipGetLastError();
}

hipError_t mlp_launch_step_static(float *theta, float *m, float *v, void *theta_b, const float *x, const float *t,
                                  int64_t n, float lr, int step, double *loss, hipStream_t s) {
  if (n < 1 || n > kMlpStaticMaxPoints) return hipErrorInvalidValue;
  void *base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  float *gpart = static_cast<float *>(base);
  double *lpart = reinterpret_cast<double *>(static_cast<unsigned char *>(base) + kScratchGrad);
  const int nwg = int((n + TP - 1) / TP);
  e = mlp_launch_grad(theta, x, t, n, 0, n, 1, 0, gpart, lpart, s);
  if (e != hipSuccess) return e;
  e = mlp_launch_adam(theta, m, v, theta_b, gpart, nwg, lr, step, nullptr, s);
  if (e != hipSuccess || !loss) return e;
  k_loss_mean<<<1, 256, 0, s>>>(lpart, nwg, n, loss);
  return hipGetLastError();
}

hipError_t mlp_launch_tobf16(const float *theta, void *theta_b, hipStream_t s) {
  k_mlp_tobf16<<<(kMlpParams + 255) / 256, 256, 0, s>>>(theta, static_cast<__hip_bfloat16 *>(theta_b));
  return hipGetLastError();
}

hipError_t mlp_launch_loss_sum(const double *lpart, int n, double *out, hipStream_t s) {
  k_loss_sum<<<1, 256, 0, s>>>(lpart, n, out);
  return hipGetLastError();
}

hipError_t mlp_launch_flags(const double *rho, int64_t n, double rho_min, int *flag, int *blk_count, hipStream_t s) {
  k_mlp_flags<<<int((n + 255) / 256), 256, 0, s>>>(rho, n, rho_min, flag, blk_count);
  return hipGetLastError();
}

hipError_t mlp_launch_compact(const double *rho, const double *sigma, int64_t n, const int *flag, const int64_t *blk_off,
                              double *rho_c, double *sigma_c, hipStream_t s) {
  k_mlp_compact<<<int((n + 255) / 256), 256, 0, s>>>(rho, sigma, n, flag, blk_off, rho_c, sigma_c);
  return hipGetLastError();
}

hipError_t mlp_launch_logrange(const double *rho, const double *sigma, int64_t n, double *out, int nblk, hipStream_t s) {
  k_mlp_logrange<<<nblk, 256, 0, s>>>(rho, sigma, n, out);
  return hipGetLastError();
}

hipError_t mlp_launch_data(const double *rho, const double *sigma, int64_t n, int xc, const double *box, float *x,
                           double *traw, double *stat, int nblk, hipStream_t s) {
  k_mlp_data<<<nblk, 256, 0, s>>>(rho, sigma, n, xc, box[0], box[1], box[2], box[3], x, traw, stat);
  return hipGetLastError();
}

hipError_t mlp_launch_standardise(const double *traw, int64_t n, const double *mean, const double *sd, float *t,
                                  hipStream_t s) {
  k_mlp_standardise<<<int((n + 255) / 256), 256, 0, s>>>(traw, n, mean[0], mean[1], mean[2], sd[0], sd[1], sd[2], t);
  return hipGetLastError();
}

hipError_t mlp_launch_forward(const MlpDev &m, const double *rho, const double *sigma, int64_t n, int xc, double *f,
                              double *vr, double *vs, int *used, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_mlp_forward<<<int((n + 127) / 128), 256, 0, s>>>(m, rho, sigma, n, xc, f, vr, vs, used);
  return hipGetLastError();
}

hipError_t mlp_launch_xfunc(const dev::FArgs &fa, const MlpDev &m, int64_t nblk, hipStream_t s) {
  k_xfunc_mlp<<<nblk, 256, 0, s>>>(fa, m);
  return hipGetLastError();
}

hipError_t launch_xc_arrays(int xc, const double *rho, const double *sigma, int64_t n, double rho_cut, double *f,
                            double *vr, double *vs, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_xc_arrays<<<int((n + 255) / 256), 256, 0, s>>>(xc, rho, sigma, n, rho_cut, f, vr, vs);
  return hipGetLastError();
}

}  // namespace kldi
