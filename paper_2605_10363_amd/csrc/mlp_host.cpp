// Host side of the functional surrogate: creation, training driver, inference and checks.
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "kldi_impl.h"

struct kldi_mlp {
  int device = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr;  // [kMlpParams] FP32 master, Adam moments
  unsigned short *theta_b = nullptr;                    // [kMlpParams] BF16 copy
  double *stats = nullptr;                              // [kMlpStats] device copy of box, tmean, tstd, rho_min
  double box[4] = {0, 1, 0, 1};
  double tmean[3] = {0, 0, 0}, tstd[3] = {1, 1, 1};
  double rho_min = 1e-8;
  int xc = KLDI_XC_PBE;
  int step = 0;
  bool trained = false;
};

namespace {

struct Err {
  kldi_status code;
  std::string msg;
};

void hipc(hipError_t e, const char *what) {
  if (e != hipSuccess) throw Err{KLDI_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class F>
kldi_status run(F &&f) {
  try {
    f();
    return KLDI_OK;
  } catch (const Err &e) {
    kldi::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    kldi::set_error("host allocation failed");
    return KLDI_E_OOM;
  }
}

template <class T>
T *dalloc(size_t n, std::vector<void *> &keep) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    for (void *q : keep) (void)hipFree(q);
    keep.clear();
    throw Err{KLDI_E_OOM, "hipMalloc failed"};
  }
  keep.push_back(p);
  return static_cast<T *>(p);
}

// splitmix64: a counter-based stream of 64-bit words
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

kldi::MlpDev view(const kldi_mlp &M) {
  kldi::MlpDev d;
  d.theta_b = M.theta_b;
  d.bias = M.theta;
  d.stats = M.stats;
  return d;
}

// the host statistics in the device layout of MlpDev::stats
void stats_to_device(const kldi_mlp &M, hipStream_t s) {
  double h[kldi::kMlpStats];
  for (int i = 0; i < 4; ++i) h[i] = M.box[i];
  for (int i = 0; i < 3; ++i) {
    h[4 + i] = M.tmean[i];
    h[7 + i] = M.tstd[i];
  }
  h[10] = M.rho_min;
  hipc(hipMemcpyAsync(M.stats, h, sizeof(h), hipMemcpyHostToDevice, s), "copy");
  hipc(hipStreamSynchronize(s), "sync");
}

bool require_trained(const kldi_mlp *M) {
  if (M->trained) return true;
  kldi::set_error("the network has not been trained (kldi_mlp_train)");
  return false;
}

}  // namespace

extern "C" {

kldi_status kldi_mlp_create(const kldi_mlp_cfg *cfg, kldi_mlp **out) {
  if (!cfg || !out) {
    kldi::set_error("cfg and out must not be NULL");
    return KLDI_E_ARG;
  }
  *out = nullptr;
  kldi_mlp *M = new kldi_mlp();
  std::vector<void *> keep;
  kldi_status st = run([&] {
    hipc(hipGetDevice(&M->device), "hipGetDevice");
    M->theta = dalloc<float>(kldi::kMlpParams, keep);
    M->m = dalloc<float>(kldi::kMlpParams, keep);
    M->v = dalloc<float>(kldi::kMlpParams, keep);
    M->theta_b = dalloc<unsigned short>(kldi::kMlpParams, keep);
    M->stats = dalloc<double>(kldi::kMlpStats, keep);
    // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, in the documented order
    std::vector<float> th(kldi::kMlpParams, 0.f);
    uint64_t s = cfg->seed;
    const int W = kldi::kMlpWidth;
    const int shapes[4][2] = {{W, 2}, {W, W}, {W, W}, {3, W}};
    int o = 0;
    for (int layer = 0; layer < 4; ++layer) {
      const int rows = shapes[layer][0], cols = shapes[layer][1];
      const double lim = 1.0 / std::sqrt(double(cols));
      for (int i = 0; i < rows * cols; ++i) {
        const double u = double(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
        th[o++] = float((2.0 * u - 1.0) * lim);
      }
      o += rows;  // biases stay zero
    }
    std::vector<float> zero(kldi::kMlpParams, 0.f);
    hipc(hipMemcpy(M->theta, th.data(), th.size() * 4, hipMemcpyHostToDevice), "copy");
    hipc(hipMemcpy(M->m, zero.data(), zero.size() * 4, hipMemcpyHostToDevice), "copy");
    hipc(hipMemcpy(M->v, zero.data(), zero.size() * 4, hipMemcpyHostToDevice), "copy");
    hipc(kldi::mlp_launch_tobf16(M->theta, M->theta_b, nullptr), "bf16");
    hipc(hipDeviceSynchronize(), "sync");
    stats_to_device(*M, nullptr);
  });
  if (st != KLDI_OK) {
    for (void *q : keep) (void)hipFree(q);
    delete M;
    return st;
  }
  *out = M;
  return KLDI_OK;
}

kldi_status kldi_mlp_destroy(kldi_mlp *M) {
  if (!M) return KLDI_OK;
  (void)hipSetDevice(M->device);
  (void)hipDeviceSynchronize();
  for (void *p : {(void *)M->theta, (void *)M->m, (void *)M->v, (void *)M->theta_b, (void *)M->stats})
    (void)hipFree(p);
  delete M;
  return KLDI_OK;
}

kldi_status kldi_mlp_params(kldi_mlp *M, float *get, const float *set, double *box, double *tmean, double *tstd) {
  if (!M) {
    kldi::set_error("mlp must not be NULL");
    return KLDI_E_ARG;
  }
  return run([&] {
    hipc(hipSetDevice(M->device), "hipSetDevice");
    if (set) {
      hipc(hipMemcpy(M->theta, set, kldi::kMlpParams * 4, hipMemcpyHostToDevice), "copy");
      hipc(kldi::mlp_launch_tobf16(M->theta, M->theta_b, nullptr), "bf16");
      hipc(hipDeviceSynchronize(), "sync");
    }
    if (get) hipc(hipMemcpy(get, M->theta, kldi::kMlpParams * 4, hipMemcpyDeviceToHost), "copy");
    if (box) std::memcpy(box, M->box, sizeof(M->box));
    if (tmean) std::memcpy(tmean, M->tmean, sizeof(M->tmean));
    if (tstd) std::memcpy(tstd, M->tstd, sizeof(M->tstd));
  });
}

kldi_status kldi_mlp_loss_grad(kldi_mlp *M, const float *x, const float *t, int64_t n, double *loss, float *grad,
                               void *stream) {
  if (!M || !x || !t || n < 1 || n > (1 << 20) || !loss || !grad) {
    kldi::set_error("bad arguments to kldi_mlp_loss_grad");
    return KLDI_E_ARG;
  }
  std::vector<void *> keep;
  kldi_status st = run([&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipc(hipSetDevice(M->device), "hipSetDevice");
    const int nwg = int((n + 63) / 64);
    float *gpart = dalloc<float>(size_t(nwg) * kldi::kMlpParams, keep);
    double *lpart = dalloc<double>(nwg, keep);
    float *g = dalloc<float>(kldi::kMlpParams, keep);
    double *lsum = dalloc<double>(1, keep);
    hipc(hipMemsetAsync(lsum, 0, 8, s), "memset");
    hipc(kldi::mlp_launch_grad(M->theta, x, t, n, 0, n, 1, 0, gpart, lpart, s), "grad");
    hipc(kldi::mlp_launch_adam(M->theta, M->m, M->v, M->theta_b, gpart, nwg, 0.f, 1, g, s), "reduce");
    hipc(kldi::mlp_launch_loss_sum(lpart, nwg, lsum, s), "loss");
    double l = 0;
    hipc(hipMemcpyAsync(grad, g, kldi::kMlpParams * 4, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipMemcpyAsync(&l, lsum, 8, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    *loss = l / (3.0 * double(n));
  });
  for (void *q : keep) (void)hipFree(q);
  return st;
}

kldi_status kldi_mlp_step(kldi_mlp *M, const float *x, const float *t, int64_t n, double lr, double *loss,
                          void *stream) {
  if (!M || !x || !t || n < 1 || n > (1 << 20) || !(lr > 0)) {
    kldi::set_error("bad arguments to kldi_mlp_step");
    return KLDI_E_ARG;
  }
  std::vector<void *> keep;
  kldi_status st = run([&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipc(hipSetDevice(M->device), "hipSetDevice");
    const int nwg = int((n + 63) / 64);
    float *gpart = dalloc<float>(size_t(nwg) * kldi::kMlpParams, keep);
    double *lpart = dalloc<double>(nwg, keep);
    double *lsum = dalloc<double>(1, keep);
    hipc(hipMemsetAsync(lsum, 0, 8, s), "memset");
    hipc(kldi::mlp_launch_grad(M->theta, x, t, n, 0, n, 1, 0, gpart, lpart, s), "grad");
    ++M->step;
    hipc(kldi::mlp_launch_adam(M->theta, M->m, M->v, M->theta_b, gpart, nwg, float(lr), M->step, nullptr, s), "adam");
    hipc(kldi::mlp_launch_loss_sum(lpart, nwg, lsum, s), "loss");
    double l = 0;
    hipc(hipMemcpyAsync(&l, lsum, 8, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    if (loss) *loss = l / (3.0 * double(n));
  });
  for (void *q : keep) (void)hipFree(q);
  return st;
}

kldi_status kldi_mlp_step_static(kldi_mlp *M, const float *x, const float *t, int64_t n, double lr, double *loss,
                                 void *stream) {
  if (!M || !x || !t || n < 1 || !(lr > 0)) {
    kldi::set_error("bad arguments to kldi_mlp_step_static");
    return KLDI_E_ARG;
  }
  if (n > kldi::kMlpStaticMaxPoints) {
    kldi::set_error("kldi_mlp_step_static takes at most " + std::to_string(kldi::kMlpStaticMaxPoints) +
                    " points per call (the size of its static scratch)");
    return KLDI_E_ARG;
  }
  return run([&] {
    hipc(hipSetDevice(M->device), "hipSetDevice");
    ++M->step;
    hipc(kldi::mlp_launch_step_static(M->theta, M->m, M->v, M->theta_b, x, t, n, float(lr), M->step, loss,
                                      static_cast<hipStream_t>(stream)),
         "step");
  });
}

kldi_status kldi_mlp_train(kldi_mlp *M, const double *rho, const double *sigma, int64_t n, const kldi_train_cfg *cfg,
                           double *loss_host, void *stream) {
  if (!M || !rho || !sigma || n < 1 || !cfg || cfg->epochs < 0 || cfg->batch < 1 || !(cfg->lr > 0) ||
      !(cfg->rho_min > 0) || (cfg->xc != KLDI_XC_PBE && cfg->xc != KLDI_XC_PBE_X) || n > (int64_t(1) << 31)) {
    kldi::set_error("bad arguments to kldi_mlp_train");
    return KLDI_E_ARG;
  }
  std::vector<void *> keep;
  kldi_status st = run([&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipc(hipSetDevice(M->device), "hipSetDevice");
    // 1. keep points with rho >= rho_min (order-preserving compaction)
    const int nb = int((n + 255) / 256);
    int *flag = dalloc<int>(n, keep);
    int *cnt = dalloc<int>(nb, keep);
    hipc(kldi::mlp_launch_flags(rho, n, cfg->rho_min, flag, cnt, s), "flags");
    std::vector<int> hc(nb);
    hipc(hipMemcpyAsync(hc.data(), cnt, size_t(nb) * 4, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    std::vector<int64_t> off(nb + 1, 0);
    for (int i = 0; i < nb; ++i) off[i + 1] = off[i] + hc[i];
    const int64_t nk = off[nb];
    if (nk < 1) throw Err{KLDI_E_ARG, "no training point with rho >= rho_min"};
    int64_t *doff = dalloc<int64_t>(nb + 1, keep);
    hipc(hipMemcpyAsync(doff, off.data(), off.size() * 8, hipMemcpyHostToDevice, s), "copy");
    double *rc = dalloc<double>(nk, keep), *sc = dalloc<double>(nk, keep);
    hipc(kldi::mlp_launch_compact(rho, sigma, n, flag, doff, rc, sc, s), "compact");
    // 2. range box
    const int rb = 1024;
    double *rng = dalloc<double>(size_t(rb) * 4, keep);
    hipc(kldi::mlp_launch_logrange(rc, sc, nk, rng, rb, s), "range");
    std::vector<double> hr(size_t(rb) * 4);
    hipc(hipMemcpyAsync(hr.data(), rng, hr.size() * 8, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    double box[4] = {1e300, -1e300, 1e300, -1e300};
    for (int i = 0; i < rb; ++i) {
      box[0] = std::min(box[0], hr[4 * i]);
      box[1] = std::max(box[1], hr[4 * i + 1]);
      box[2] = std::min(box[2], hr[4 * i + 2]);
      box[3] = std::max(box[3], hr[4 * i + 3]);
    }
    if (!(box[1] > box[0])) box[1] = box[0] + 1.0;
    if (!(box[3] > box[2])) box[3] = box[2] + 1.0;
    // 3. features and targets of the analytic functional, standardised
    float *x = dalloc<float>(size_t(nk) * 2, keep);
    float *t = dalloc<float>(size_t(nk) * 3, keep);
    double *traw = dalloc<double>(size_t(nk) * 3, keep);
    double *stat = dalloc<double>(size_t(rb) * 6, keep);
    hipc(kldi::mlp_launch_data(rc, sc, nk, cfg->xc, box, x, traw, stat, rb, s), "data");
    std::vector<double> hs(size_t(rb) * 6);
    hipc(hipMemcpyAsync(hs.data(), stat, hs.size() * 8, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    double mean[3], sd[3];
    for (int o = 0; o < 3; ++o) {
      double a = 0, b = 0;
      for (int i = 0; i < rb; ++i) {
        a += hs[6 * i + o];
        b += hs[6 * i + 3 + o];
      }
      mean[o] = a / double(nk);
      sd[o] = std::sqrt(std::max(b / double(nk) - mean[o] * mean[o], 0.0));
      if (!(sd[o] > 0)) sd[o] = 1.0;
    }
    hipc(kldi::mlp_launch_standardise(traw, nk, mean, sd, t, s), "standardise");
    // 4. Adam over shuffled batches: epoch order i -> (a i + b) mod nk with gcd(a, nk) = 1
    const int64_t B = std::min<int64_t>(cfg->batch, nk);
    const int nwg = int((B + 63) / 64);
    float *gpart = dalloc<float>(size_t(nwg) * kldi::kMlpParams, keep);
    double *lpart = dalloc<double>(nwg, keep);
    double *lsum = dalloc<double>(cfg->epochs > 0 ? cfg->epochs : 1, keep);
    hipc(hipMemsetAsync(lsum, 0, 8 * size_t(std::max(cfg->epochs, 1)), s), "memset");
    uint64_t rs = cfg->seed;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
      int64_t a = int64_t(splitmix(rs) % uint64_t(nk)) | 1;
      while (std::gcd(a, nk) != 1) a += 2;
      const int64_t b = int64_t(splitmix(rs) % uint64_t(nk));
      for (int64_t start = 0; start < nk; start += B) {
        const int64_t count = std::min(B, nk - start);
        const int w = int((count + 63) / 64);
        hipc(kldi::mlp_launch_grad(M->theta, x, t, nk, start, count, a, b, gpart, lpart, s), "grad");
        ++M->step;
        hipc(kldi::mlp_launch_adam(M->theta, M->m, M->v, M->theta_b, gpart, w, float(cfg->lr), M->step, nullptr, s),
             "adam");
        hipc(kldi::mlp_launch_loss_sum(lpart, w, lsum + ep, s), "loss");
      }
    }
    std::vector<double> hl(std::max(cfg->epochs, 1));
    hipc(hipMemcpyAsync(hl.data(), lsum, hl.size() * 8, hipMemcpyDeviceToHost, s), "copy");
    hipc(hipStreamSynchronize(s), "sync");
    if (loss_host)
      for (int ep = 0; ep < cfg->epochs; ++ep) loss_host[ep] = hl[ep] / (3.0 * double(nk));
    std::memcpy(M->box, box, sizeof(box));
    std::memcpy(M->tmean, mean, sizeof(mean));
    std::memcpy(M->tstd, sd, sizeof(sd));
    M->rho_min = cfg->rho_min;
    M->xc = cfg->xc;
    M->trained = true;
    stats_to_device(*M, s);
  });
  for (void *q : keep) (void)hipFree(q);
  return st;
}

kldi_status kldi_mlp_forward(const kldi_mlp *M, const double *rho, const double *sigma, int64_t n, double *f,
                             double *vr, double *vs, int32_t *used, void *stream) {
  if (!M || !rho || !sigma || n < 0 || !f || !vr || !vs) {
    kldi::set_error("bad arguments to kldi_mlp_forward");
    return KLDI_E_ARG;
  }
  if (!require_trained(M)) return KLDI_E_STATE;
  return run([&] {
    hipc(hipSetDevice(M->device), "hipSetDevice");
    hipc(kldi::mlp_launch_forward(view(*M), rho, sigma, n, M->xc, f, vr, vs, used, static_cast<hipStream_t>(stream)),
         "forward");
  });
}

kldi_status kldi_plan_attach_mlp(kldi_plan *plan, const kldi_mlp *M) {
  if (!plan) {
    kldi::set_error("plan must not be NULL");
    return KLDI_E_ARG;
  }
  if (M && plan->impl.opts.xc == KLDI_XC_LDA_X) {
    kldi::set_error("the surrogate replaces a GGA functional; this plan is LDA");
    return KLDI_E_UNSUPPORTED;
  }
  if (M && !require_trained(M)) return KLDI_E_STATE;
  if (M && M->xc != plan->impl.opts.xc) {
    kldi::set_error("the network was trained on another functional than the plan's");
    return KLDI_E_ARG;
  }
  plan->impl.has_mlp = M != nullptr;
  if (M) plan->impl.mlp = view(*M);
  kldi::invalidate_graphs(plan->impl);
  return KLDI_OK;
}

}  // extern "C"
