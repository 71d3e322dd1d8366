// sched.cpp -- choosing a batch's copy schedule: the autotuner (times every
// class on a batch), the tuned table (nearest autotuned batch by histogram
// feature), and the schedule network (trained on the GPU by the project's own
// HIP kernels; evaluated for each submission on the host, where the batch's
// sizes already are, so the choice costs no extra launch and the copy grid
// can be sized for the chosen class).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp.h"
#include "net_host.h"
#include "runtime.h"

namespace hicr {

struct SchedState {
  float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
  float *d_loss = nullptr;
  int step = 0;
  bool net_loaded = false;
  float *d_act = nullptr;  // activations of up to act_cap samples
  float *d_x = nullptr;    // one feature, for the device inference of a plan's class
  int act_cap = 0;
  MlpBufs bufs{};
  std::vector<std::array<float, kMlpIn>> feats;  // tuned table
  std::vector<uint32_t> cls;
  // search index of the tuned table (rebuilt after the table changes): the
  // entries sorted by their distance to the first of three pivots (ties in
  // table order), with their features, distances to the pivots and table
  // positions in that order
  bool idx_dirty = true;
  std::array<std::array<double, kMlpIn>, 3> piv{};
  std::vector<std::array<float, kMlpIn>> sf;
  std::vector<std::array<double, 3>> spd;
  std::vector<uint32_t> sk;
  // host copy of the network for the per-submission choice (h_params as on
  // the device, h_t transposed for the host forward pass); stale after a
  // device training step until the next learned submission reads it back
  std::vector<float> h_params, h_t;
  bool h_stale = false;
  int last_cls = -1;  // class of the most recent learned submission
};

void batch_features(const uint64_t *sizes, uint64_t n, size_t stride, float *out) {
  uint64_t cnt[kMlpIn] = {0};
  const char *p = reinterpret_cast<const char *>(sizes);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t s;
    std::memcpy(&s, p + i * stride, 8);
    int b = s == 0 ? 0 : 63 - __builtin_clzll(s);
    cnt[b > 31 ? 31 : b]++;
  }
  for (int b = 0; b < kMlpIn; b++) out[b] = std::log2(1.0f + (float)cnt[b]);
}

static int state(hicr_ctx c, SchedState **out) {
  if (!c->sched) {
    SchedState *s = new (std::nothrow) SchedState();
    if (!s) return HICR_ENOMEM;
    const size_t pb = sizeof(float) * kMlpParams;
    bool ok = hipMalloc(&s->d_params, pb) == hipSuccess && hipMalloc(&s->d_m, pb) == hipSuccess &&
              hipMalloc(&s->d_v, pb) == hipSuccess && hipMalloc(&s->d_grad, pb) == hipSuccess &&
              hipMalloc(&s->d_loss, 64) == hipSuccess;
    c->sched = s;
    if (!ok) return fail(c, HICR_ENOMEM, "network state");
  }
  *out = c->sched;
  return HICR_OK;
}

static int ensure_act(hicr_ctx c, SchedState *s, int B) {
  if (B <= s->act_cap) return HICR_OK;
  if (s->d_act) (void)hipFree(s->d_act);
  s->d_act = nullptr;
  s->act_cap = 0;
  const size_t per = 2 * kMlpHidden * 2 + kMlpOut * 2 + kMlpHidden * 2 + 1;  // floats/sample
  if (hipMalloc(&s->d_act, sizeof(float) * per * B) != hipSuccess)
    return fail(c, HICR_ENOMEM, "activations for %d samples", B);
  float *p = s->d_act;
  auto take = [&](int n) { float *q = p; p += (size_t)n * B; return q; };
  s->bufs.a1 = take(kMlpHidden);
  s->bufs.h1 = take(kMlpHidden);
  s->bufs.a2 = take(kMlpHidden);
  s->bufs.h2 = take(kMlpHidden);
  s->bufs.z = take(kMlpOut);
  s->bufs.dz = take(kMlpOut);
  s->bufs.d2 = take(kMlpHidden);
  s->bufs.d1 = take(kMlpHidden);
  s->bufs.loss = take(1);
  s->act_cap = B;
  return HICR_OK;
}

static double pivot_dist(const std::array<double, kMlpIn> &p, const float *f) {
  double d = 0.0;
  for (int b = 0; b < kMlpIn; b++) d += (f[b] - p[b]) * (f[b] - p[b]);
  return std::sqrt(d);
}

// Pivots: the origin, the table's mean feature, and the entry farthest from
// the mean; entries are ordered by their distance to the origin.
static void build_index(SchedState *s) {
  const size_t n = s->feats.size();
  s->piv[0].fill(0.0);
  s->piv[1].fill(0.0);
  for (const auto &g : s->feats)
    for (int b = 0; b < kMlpIn; b++) s->piv[1][b] += g[b] / (double)n;
  size_t far = 0;
  double fd = -1.0;
  for (size_t k = 0; k < n; k++) {
    const double d = pivot_dist(s->piv[1], s->feats[k].data());
    if (d > fd) {
      fd = d;
      far = k;
    }
  }
  for (int b = 0; b < kMlpIn; b++) s->piv[2][b] = s->feats[far][b];
  std::vector<std::array<double, 3>> pd(n);
  for (size_t k = 0; k < n; k++)
    for (int j = 0; j < 3; j++) pd[k][j] = pivot_dist(s->piv[j], s->feats[k].data());
  s->sk.resize(n);
  for (size_t k = 0; k < n; k++) s->sk[k] = (uint32_t)k;
  std::stable_sort(s->sk.begin(), s->sk.end(),
                   [&](uint32_t x, uint32_t y) { return pd[x][0] < pd[y][0]; });
  s->sf.resize(n);
  s->spd.resize(n);
  for (size_t i = 0; i < n; i++) {
    s->sf[i] = s->feats[s->sk[i]];
    s->spd[i] = pd[s->sk[i]];
  }
  s->idx_dirty = false;
}

// Squared distance as the tuned table defines it (fp32, bins in order), or
// any value above `bound` once a partial sum (8 bins at a time) exceeds it:
// partial sums of non-negative terms never decrease, so such an entry cannot
// be nearer than `bound`.
static float feat_dist(const float *g, const float *f, float bound) {
  float d = 0.f;
  for (int b = 0; b < kMlpIn; b += 8) {
    for (int q = b; q < b + 8; q++) {
      const float x = g[q] - f[q];
      d += x * x;
    }
    if (d > bound) return d;
  }
  return d;
}

// The class of the first table entry (in table order) at the smallest fp32
// squared distance from f -- the answer of a full scan.  The scan starts at
// the entries whose distance to the origin is closest to f's and walks
// outward; by the triangle inequality an entry e is no nearer than
// |d(e, p) - d(f, p)| for every pivot p, so a direction stops once that gap
// exceeds the best distance found, and an entry is skipped when another
// pivot's gap does.  Gaps are compared with a relative margin of 1e-4, far
// above the fp32 distance's rounding (~2e-6), so nothing a full scan could
// pick is pruned.
static uint32_t nearest(SchedState *s, const float *f) {
  if (s->idx_dirty) build_index(s);
  const size_t n = s->feats.size();
  double q[3];
  for (int j = 0; j < 3; j++) q[j] = pivot_dist(s->piv[j], f);
  size_t hi = std::lower_bound(s->spd.begin(), s->spd.end(), q[0],
                               [](const std::array<double, 3> &e, double v) { return e[0] < v; }) -
              s->spd.begin();
  size_t lo = hi;  // candidates [lo, hi) visited; next are lo - 1 and hi
  float bd = 3.4e38f;
  uint32_t bk = 0;
  auto pruned = [&](double gap) { return gap * gap > (double)bd * (1.0 + 1e-4); };
  for (;;) {
    const double gl = lo > 0 ? q[0] - s->spd[lo - 1][0] : 1e300;
    const double gh = hi < n ? s->spd[hi][0] - q[0] : 1e300;
    const bool take_lo = gl <= gh;
    const double gap = take_lo ? gl : gh;
    if (gap >= 1e300 || pruned(gap)) break;  // both directions are done
    const size_t i = take_lo ? --lo : hi++;
    if (pruned(std::fabs(s->spd[i][1] - q[1])) || pruned(std::fabs(s->spd[i][2] - q[2]))) continue;
    const float d = feat_dist(s->sf[i].data(), f, bd);
    const uint32_t k = s->sk[i];
    if (d < bd || (d == bd && k < bk)) {
      bd = d;
      bk = k;
    }
  }
  return s->cls[bk];
}

// The network's class for one batch feature: forward pass in fp32 on the
// host's transposed copy of the parameters, argmax with ties to the lowest
// class -- the device forward kernel's arithmetic, bit for bit.  The FMA
// build is taken where the CPU has FMA (std::fmaf is otherwise a library
// call: ~18 us per pass instead of ~0.3 us, measured).
static uint32_t net_class(const float *T, const float *x) {
  static const bool fma = __builtin_cpu_supports("fma");
  return fma ? net_class_fma(T, x) : net_class_axpy(T, x);
}

// The network's class for one feature by the device forward kernel (the
// parameters as they are on the device), read back and argmax-ed with ties to
// the lowest class.
static int device_class(hicr_ctx c, SchedState *s, const float *f, uint32_t *cls) {
  int rc = ensure_act(c, s, 1);
  if (rc != HICR_OK) return rc;
  if (!s->d_x && hipMalloc(&s->d_x, sizeof(float) * kMlpIn) != hipSuccess) {
    s->d_x = nullptr;
    return fail(c, HICR_ENOMEM, "network input");
  }
  static_assert(sizeof(float) * kMlpOut <= 64, "logits fit the read-back buffer");
  float *z = reinterpret_cast<float *>(c->h_read);
  hipError_t e = hipMemcpy(s->d_x, f, sizeof(float) * kMlpIn, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = mlp_forward(s->bufs, s->d_params, s->d_x, 1, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(z, s->bufs.z, sizeof(float) * kMlpOut, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "network forward for a plan");
  uint32_t b = 0;
  for (uint32_t k = 1; k < (uint32_t)kMlpOut; k++)
    if (z[k] > z[b]) b = k;
  *cls = b;
  return HICR_OK;
}

int choose_sched(hicr_ctx c, const hicr_desc *d, uint64_t n, uint32_t mode, hicr_sched *out,
                 bool on_device) {
  SchedState *s = c->sched;
  if (mode == HICR_SCHED_LEARNED && s && s->net_loaded && on_device) {
    float f[kMlpIn];
    batch_features(n ? &d[0].size : nullptr, n, sizeof(hicr_desc), f);
    uint32_t k = 0;
    int rc = device_class(c, s, f, &k);
    if (rc != HICR_OK) return rc;
    s->last_cls = (int)k;
    return hicr_sched_class(k, out);
  }
  if (mode == HICR_SCHED_LEARNED && s && s->net_loaded) {
    if (s->h_stale) {
      // parameters changed by device training steps queued on the context stream
      hipError_t e = hipMemcpyAsync(s->h_params.data(), s->d_params, sizeof(float) * kMlpParams,
                                    hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "reading the network parameters");
      s->h_t.resize(kMlpParams);
      net_transpose(s->h_params.data(), s->h_t.data());
      s->h_stale = false;
    }
    float f[kMlpIn];
    batch_features(n ? &d[0].size : nullptr, n, sizeof(hicr_desc), f);
    const uint32_t k = net_class(s->h_t.data(), f);
    s->last_cls = (int)k;
    return hicr_sched_class(k, out);
  }
  // tuned table, the fallback when no network is loaded; default if empty
  if (s && !s->feats.empty() && n) {
    float f[kMlpIn];
    batch_features(&d[0].size, n, sizeof(hicr_desc), f);
    return hicr_sched_class(nearest(s, f), out);
  }
  *out = c->def_sched;
  return HICR_OK;
}

void destroy_sched(hicr_ctx c) {
  SchedState *s = c->sched;
  if (!s) return;
  for (void *p : {(void *)s->d_params, (void *)s->d_m, (void *)s->d_v, (void *)s->d_grad,
                  (void *)s->d_loss, (void *)s->d_act, (void *)s->d_x})
    if (p) (void)hipFree(p);
  delete s;
  c->sched = nullptr;
}

}  // namespace hicr

using namespace hicr;

extern "C" {

int hicr_sched_features(const hicr_desc *descs, uint64_t n, float *out32) {
  return guarded([&]() -> int {
    if (!out32 || (n && !descs)) return HICR_EINVAL;
    if (n == 0) {
      for (int b = 0; b < kMlpIn; b++) out32[b] = 0.f;
      return HICR_OK;
    }
    batch_features(&descs[0].size, n, sizeof(hicr_desc), out32);
    return HICR_OK;
  });
}

int hicr_mlp_set_params(hicr_ctx c, const float *params) {
  return guarded([&]() -> int {
    if (!c || !params) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    int rc = wait_all(c);
    if (rc != HICR_OK) return rc;
    SchedState *s;
    rc = state(c, &s);
    if (rc != HICR_OK) return rc;
    const size_t pb = sizeof(float) * kMlpParams;
    hipError_t e = hipMemcpy(s->d_params, params, pb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->d_m, 0, pb);
    if (e == hipSuccess) e = hipMemset(s->d_v, 0, pb);
    if (e != hipSuccess) return hip_fail(c, e, "loading network parameters");
    s->step = 0;
    s->net_loaded = true;
    s->h_params.assign(params, params + kMlpParams);
    s->h_t.resize(kMlpParams);
    net_transpose(s->h_params.data(), s->h_t.data());
    s->h_stale = false;
    return HICR_OK;
  });
}

int hicr_mlp_get_params(hicr_ctx c, float *out) {
  return guarded([&]() -> int {
    if (!c || !out) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || !c->sched->net_loaded) return fail(c, HICR_EINVAL, "no network loaded");
    (void)hipSetDevice(c->device);
    int rc = wait_all(c);
    if (rc != HICR_OK) return rc;
    hipError_t e = hipMemcpy(out, c->sched->d_params, sizeof(float) * kMlpParams,
                             hipMemcpyDeviceToHost);
    return e == hipSuccess ? HICR_OK : hip_fail(c, e, "reading network parameters");
  });
}

int hicr_mlp_forward(hicr_ctx c, const float *x_dev, uint32_t batch, float *logits_dev) {
  return guarded([&]() -> int {
    if (!c || !x_dev || !logits_dev || batch == 0) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || !c->sched->net_loaded) return fail(c, HICR_EINVAL, "no network loaded");
    (void)hipSetDevice(c->device);
    SchedState *s = c->sched;
    int rc = ensure_act(c, s, (int)batch);
    if (rc != HICR_OK) return rc;
    hipError_t e = mlp_forward(s->bufs, s->d_params, x_dev, (int)batch, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(logits_dev, s->bufs.z, sizeof(float) * kMlpOut * batch,
                         hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? HICR_OK : hip_fail(c, e, "network forward");
  });
}

int hicr_mlp_grad(hicr_ctx c, const float *x_dev, const int32_t *y_dev, uint32_t batch,
                  float *grad_dev, float *loss_dev) {
  return guarded([&]() -> int {
    if (!c || !x_dev || !y_dev || !grad_dev || batch == 0) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || !c->sched->net_loaded) return fail(c, HICR_EINVAL, "no network loaded");
    (void)hipSetDevice(c->device);
    SchedState *s = c->sched;
    int rc = ensure_act(c, s, (int)batch);
    if (rc != HICR_OK) return rc;
    hipError_t e = mlp_forward(s->bufs, s->d_params, x_dev, (int)batch, c->stream);
    if (e == hipSuccess)
      e = mlp_backward(s->bufs, s->d_params, x_dev, y_dev, (int)batch, grad_dev, loss_dev,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? HICR_OK : hip_fail(c, e, "network gradient");
  });
}

int hicr_mlp_train_step(hicr_ctx c, const float *x_dev, const int32_t *y_dev, uint32_t batch,
                        float lr, float *loss_dev) {
  return guarded([&]() -> int {
    if (!c || !x_dev || !y_dev || batch == 0 || !(lr > 0.f)) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || !c->sched->net_loaded) return fail(c, HICR_EINVAL, "no network loaded");
    (void)hipSetDevice(c->device);
    SchedState *s = c->sched;
    int rc = ensure_act(c, s, (int)batch);
    if (rc != HICR_OK) return rc;
    hipError_t e = mlp_forward(s->bufs, s->d_params, x_dev, (int)batch, c->stream);
    if (e == hipSuccess)
      e = mlp_backward(s->bufs, s->d_params, x_dev, y_dev, (int)batch, s->d_grad, loss_dev,
                       c->stream);
    if (e == hipSuccess) e = mlp_adam(s->d_params, s->d_grad, s->d_m, s->d_v, lr, ++s->step, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->push_ev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "network training step");
    c->push_pending = true;
    s->h_stale = true;
    return HICR_OK;
  });
}

int hicr_last_choice(hicr_ctx c, uint32_t *cls) {
  return guarded([&]() -> int {
    if (!c || !cls) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || c->sched->last_cls < 0) return fail(c, HICR_EINVAL, "no learned submission yet");
    *cls = (uint32_t)c->sched->last_cls;
    return HICR_OK;
  });
}

int hicr_tune_add(hicr_ctx c, const hicr_desc *descs, uint64_t n, uint32_t cls) {
  return guarded([&]() -> int {
    if (!c || (n && !descs) || cls >= HICR_NUM_CLASSES) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    SchedState *s;
    int rc = state(c, &s);
    if (rc != HICR_OK) return rc;
    std::array<float, kMlpIn> f{};
    if (n) batch_features(&descs[0].size, n, sizeof(hicr_desc), f.data());
    s->feats.push_back(f);
    s->cls.push_back(cls);
    s->idx_dirty = true;
    return HICR_OK;
  });
}

int hicr_tune_lookup(hicr_ctx c, const hicr_desc *descs, uint64_t n, uint32_t *cls) {
  return guarded([&]() -> int {
    if (!c || (n && !descs) || !cls) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->sched || c->sched->feats.empty()) return fail(c, HICR_EINVAL, "empty tuned table");
    std::array<float, kMlpIn> f{};
    if (n) batch_features(&descs[0].size, n, sizeof(hicr_desc), f.data());
    *cls = nearest(c->sched, f.data());
    return HICR_OK;
  });
}

int hicr_tune_clear(hicr_ctx c) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (c->sched) {
      c->sched->feats.clear();
      c->sched->cls.clear();
      c->sched->idx_dirty = true;
    }
    return HICR_OK;
  });
}

int hicr_autotune(hicr_ctx c, const hicr_desc *descs, uint64_t n, uint32_t reps, float *times_ms,
                  uint32_t *best) {
  return guarded([&]() -> int {
    if (!c || !descs || n == 0 || reps == 0 || reps > 64 || !times_ms) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    int rc = flush_pending(c);
    if (rc == HICR_OK) rc = wait_all(c);
    if (rc != HICR_OK) return rc;
    hipEvent_t t0[64] = {}, t1[64] = {};
    auto destroy_events = [&]() {
      for (uint32_t r = 0; r < reps; r++) {
        if (t0[r]) (void)hipEventDestroy(t0[r]);
        if (t1[r]) (void)hipEventDestroy(t1[r]);
      }
    };
    for (uint32_t r = 0; r < reps; r++) {
      if (hipEventCreate(&t0[r]) != hipSuccess || hipEventCreate(&t1[r]) != hipSuccess) {
        destroy_events();  // the ones created so far
        return fail(c, HICR_EDEVICE, "timing events");
      }
    }
    uint64_t bad = 0;
    for (uint32_t k = 0; k < (uint32_t)HICR_NUM_CLASSES && rc == HICR_OK; k++) {
      hicr_sched sch;
      hicr_sched_class(k, &sch);
      SubmitOpts warm;
      warm.no_count = true;
      rc = submit(c, descs, n, sch, c->stream, &bad, &warm);
      std::vector<float> ms(reps);
      for (uint32_t r = 0; r < reps && rc == HICR_OK; r++) {
        SubmitOpts o;
        o.no_count = true;
        o.t0 = t0[r];
        o.t1 = t1[r];
        rc = submit(c, descs, n, sch, c->stream, &bad, &o);
      }
      if (rc == HICR_OK) rc = wait_all(c);
      for (uint32_t r = 0; r < reps && rc == HICR_OK; r++)
        if (hipEventElapsedTime(&ms[r], t0[r], t1[r]) != hipSuccess)
          rc = fail(c, HICR_EDEVICE, "reading timing events");
      if (rc == HICR_OK) {
        std::sort(ms.begin(), ms.end());
        times_ms[k] = ms[reps / 2];
      }
    }
    destroy_events();
    if (rc != HICR_OK) return rc;
    if (best) {
      uint32_t b = 0;
      for (uint32_t k = 1; k < (uint32_t)HICR_NUM_CLASSES; k++)
        if (times_ms[k] < times_ms[b]) b = k;  // ties go to the lowest class
      *best = b;
    }
    return HICR_OK;
  });
}

}  // extern "C"
