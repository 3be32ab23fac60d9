// Host runtime and C ABI of libsteps (see include/steps.h): contexts,
// argument validation, launch-shape selection, and the orchestration of one
// KDK step (Racz et al. 2018, Sec. 2.3 Eqs. 9-11 around the pair sum of
// Sec. 2.2 Eq. 8).  Every call validates its arguments completely before it
// enqueues anything, so a failing call writes nothing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "steps.h"
#include "steps_cosmo.h"
#include "steps_internal.h"

#define STEPS_VERSION_STRING "libsteps 0.1.0 (gfx950)"

namespace {

constexpr int64_t kMaxN = int64_t(1) << 30;
// below this size the spatial sort costs more than the culling saves
constexpr int64_t kSortMinN = 32768;

thread_local std::string t_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(STEPS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

struct Buffer {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct steps_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = STEPS_FP64;
  uint32_t flags = 0;
  bool tile_forced = false;
  steps_tile tile = {0, 0, 0, 0};
  Buffer part;     // j-split partial sums
  Buffer shadow;   // FP32 shadow of the inputs
  Buffer arena;    // spatial-sort scratch (keys, permutation, sorted copy)
  int *flag = nullptr;  // device int for the finite check
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms = 0.0;
  int64_t prof_count = 0;
  std::mutex mu;  // one call at a time per context
};

namespace {

std::mutex g_default_mu;
std::vector<steps_ctx *> g_default;  // per device, created on first use

int ensure(steps_ctx *c, Buffer &b, size_t bytes, const char *what) {
  if (b.bytes >= bytes) return STEPS_OK;
  if (b.p) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(STEPS_E_NOMEM, "cannot allocate %zu bytes of %s scratch",
                bytes, what);
  }
  b.bytes = bytes;
  return STEPS_OK;
}

// A caller array must be device (or managed) memory on the context device,
// with at least `bytes` bytes from p to the end of its allocation.
int check_ptr(const steps_ctx *c, const void *p, size_t bytes,
              const char *name) {
  if (!p) return fail(STEPS_E_INVAL, "%s is NULL", name);
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(STEPS_E_INVAL, "%s (%p) is not memory known to HIP", name, p);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged &&
      !at.isManaged) {
    return fail(STEPS_E_INVAL, "%s (%p) is not device memory", name, p);
  }
  if (at.type == hipMemoryTypeDevice && at.device != c->device) {
    return fail(STEPS_E_INVAL, "%s is on device %d, the context on device %d",
                name, at.device, c->device);
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
  if (e == hipSuccess && base) {
    const char *b = (const char *)base, *q = (const char *)p;
    if (q + bytes > b + size) {
      return fail(STEPS_E_INVAL,
                  "%s needs %zu bytes but its allocation ends %zu bytes "
                  "after it",
                  name, bytes, (size_t)(b + size - q));
    }
  } else {
    (void)hipGetLastError();
  }
  return STEPS_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

int check_n(int64_t n) {
  if (n < 0) return fail(STEPS_E_INVAL, "n = %lld < 0", (long long)n);
  if (n > kMaxN) {
    return fail(STEPS_E_INVAL, "n = %lld exceeds the limit 2^30",
                (long long)n);
  }
  return STEPS_OK;
}

int prec_class(int precision) {
  return precision == STEPS_FP64 ? steps::kClassF64 : steps::kClassMixed;
}

// tile size of the first compiled variant with this (class, r), or 0
int variant_tj(int cls, int r) {
  int cnt = 0;
  const steps::ForceVariant *v = steps::force_variants(&cnt);
  for (int k = 0; k < cnt; ++k) {
    if (v[k].cls == cls && v[k].r == r) return v[k].tj;
  }
  return 0;
}

// Launch shape: a forced tile, else the heuristic, tuned on MI355X at
// N = 2^18 and 2^21: FP64 r = 4, mixed r = 2 (fewer registers, more waves
// to pair up FP32 issue); r is lowered for small n so that there are at
// least 256 i-blocks where possible; the j range is then split so that the
// grid holds about 8192 (FP64) or 16384 (mixed) workgroups, keeping every
// split at least two tiles.  Culled (sorted) variants from kSortMinN up; in
// FP64 the r^-3 correction stops at first order there (variant 3).
steps_tile choose_tile(const steps_ctx *c, int64_t n) {
  const int cls = prec_class(c->precision);
  steps_tile t;
  if (c->tile_forced) {
    t = c->tile;
  } else {
    const bool f64 = cls == steps::kClassF64;
    int r = f64 ? 4 : 2;
    while (r > 1 && (n + 256LL * r - 1) / (256LL * r) < 256) r /= 2;
    t.r = r;
    t.tj = variant_tj(cls, r);
    const int64_t nb = std::max<int64_t>(1, (n + 256LL * r - 1) / (256LL * r));
    const int64_t target = f64 ? 8192 : 16384;
    int64_t js = (target + nb - 1) / nb;
    js = std::min<int64_t>(js, std::max<int64_t>(1, n / (2LL * t.tj)));
    t.jsplit = (int)std::max<int64_t>(1, std::min<int64_t>(js, 64));
    t.variant = 0;
    if (n >= kSortMinN) {
      t.variant = steps::kVarCull | (f64 ? steps::kVarNoE2 : 0);
    }
  }
  return t;
}

// chunk of the j range per split: a multiple of the tile size
void split_j(int64_t n, int tj, int jsplit, int *chunk, int *js_eff) {
  int64_t per = (n + jsplit - 1) / jsplit;
  per = ((per + tj - 1) / tj) * tj;
  if (per < tj) per = tj;
  *chunk = (int)per;
  *js_eff = (int)std::max<int64_t>(1, (n + per - 1) / per);
}

int prof_begin(steps_ctx *c, hipEvent_t *ev) {
  if (!(c->flags & STEPS_PROFILE)) return STEPS_OK;
  for (int k = 0; k < 2; ++k) {
    if (!c->prof_pool.empty()) {
      ev[k] = c->prof_pool.back();
      c->prof_pool.pop_back();
    } else {
      hipError_t e = hipEventCreate(&ev[k]);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  }
  hipError_t e = hipEventRecord(ev[0], c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  return STEPS_OK;
}

int prof_end(steps_ctx *c, hipEvent_t *ev) {
  if (!(c->flags & STEPS_PROFILE)) return STEPS_OK;
  hipError_t e = hipEventRecord(ev[1], c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  c->prof_pending.emplace_back(ev[0], ev[1]);
  return STEPS_OK;
}

// Sub-allocation of one scratch buffer.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return at;
  }
};

// Enqueue acc <- S(pos) in the context's precision.  Arguments validated.
int run_forces(steps_ctx *c, const double *pos, const double *mass,
               const double *soft, int n, double *acc) {
  if (n == 0) return STEPS_OK;
  const int cls = prec_class(c->precision);
  const steps_tile t = choose_tile(c, n);
  const steps::ForceVariant *v =
      steps::find_force_variant(cls, t.r, t.tj, t.variant);
  if (!v) {
    return fail(STEPS_E_INVAL,
                "no compiled force kernel with r=%d tj=%d variant=%d", t.r,
                t.tj, t.variant);
  }
  const bool cull = (t.variant & steps::kVarCull) != 0;
  int chunk = 0, js = 1;
  split_j(n, t.tj, std::max(1, t.jsplit), &chunk, &js);
  steps::ForceLaunch L;
  L.n = n;
  L.jchunk = chunk;
  L.jsplit = js;
  L.out = acc;
  L.kahan = c->precision == STEPS_MIXED_KAHAN;
  int rc;
  hipError_t e;
  if (js > 1 || cull) {
    rc = ensure(c, c->part, (size_t)js * 3 * (size_t)n * sizeof(double),
                "partial-sum");
    if (rc) return rc;
    L.out = (double *)c->part.p;
  }
  const int *perm = nullptr;
  if (cull) {
    // Morton order: bbox -> keys -> stable sort -> sorted copy -> tile boxes
    size_t cub_bytes = 0;
    e = steps::sort_pairs(nullptr, &cub_bytes, nullptr, nullptr, nullptr,
                          nullptr, n, c->stream);
    if (e != hipSuccess) return hip_fail(e, "radix sort size query");
    const int ntiles = (n + t.tj - 1) / t.tj;
    Carve cv;
    const size_t o_box = cv.take(6 * sizeof(double));
    const size_t o_bpart = cv.take((size_t)steps::bbox_blocks(n) * 6 * sizeof(double));
    const size_t o_k0 = cv.take((size_t)n * 8), o_k1 = cv.take((size_t)n * 8);
    const size_t o_v0 = cv.take((size_t)n * 4), o_v1 = cv.take((size_t)n * 4);
    const size_t o_cub = cv.take(cub_bytes);
    const size_t o_info = cv.take((size_t)ntiles * 8 * sizeof(double));
    const size_t o_soa = cv.take(cls == steps::kClassF64
                                     ? 5 * (size_t)n * sizeof(double)
                                     : 5 * (size_t)n * sizeof(float));
    if ((rc = ensure(c, c->arena, cv.off, "sort"))) return rc;
    char *base = (char *)c->arena.p;
    double *box = (double *)(base + o_box);
    auto *k0 = (unsigned long long *)(base + o_k0);
    auto *k1 = (unsigned long long *)(base + o_k1);
    int *v0 = (int *)(base + o_v0), *v1 = (int *)(base + o_v1);
    double *info = (double *)(base + o_info);
    if ((e = steps::launch_bbox(pos, n, (double *)(base + o_bpart), box,
                                c->stream)) != hipSuccess ||
        (e = steps::launch_morton(pos, n, box, k0, v0, c->stream)) !=
            hipSuccess) {
      return hip_fail(e, "sort-key kernel launch");
    }
    e = steps::sort_pairs(base + o_cub, &cub_bytes, k0, k1, v0, v1, n,
                          c->stream);
    if (e != hipSuccess) return hip_fail(e, "radix sort");
    perm = v1;
    if (cls == steps::kClassF64) {
      double *sorted = (double *)(base + o_soa);
      e = steps::launch_gather(pos, mass, soft, perm, n, sorted, nullptr,
                               c->stream);
      if (e == hipSuccess) {
        e = steps::launch_tile_info_f64(sorted, n, t.tj, info, c->stream);
      }
      L.pos = sorted;
      L.mass = sorted + 3 * (size_t)n;
      L.soft = sorted + 4 * (size_t)n;
    } else {
      float *shadow = (float *)(base + o_soa);
      e = steps::launch_gather(pos, mass, soft, perm, n, nullptr, shadow,
                               c->stream);
      if (e == hipSuccess) {
        e = steps::launch_tile_info_f32(shadow, n, t.tj, info, c->stream);
      }
      L.shadow = shadow;
    }
    if (e != hipSuccess) return hip_fail(e, "gather kernel launch");
    L.tinfo = info;
  } else if (cls == steps::kClassMixed) {
    rc = ensure(c, c->shadow, 5 * (size_t)n * sizeof(float), "FP32 shadow");
    if (rc) return rc;
    e = steps::launch_shadow(pos, mass, soft, n, (float *)c->shadow.p,
                             c->stream);
    if (e != hipSuccess) return hip_fail(e, "shadow kernel launch");
    L.shadow = (const float *)c->shadow.p;
  } else {
    L.pos = pos;
    L.mass = mass;
    L.soft = soft;
  }
  hipEvent_t ev[2];
  if ((rc = prof_begin(c, ev))) return rc;
  e = v->launch(L, c->stream);
  if (e != hipSuccess) return hip_fail(e, "force kernel launch");
  if ((rc = prof_end(c, ev))) return rc;
  if (cull) {
    e = steps::launch_reduce_scatter(L.out, js, n, perm, acc, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  } else if (js > 1) {
    e = steps::launch_reduce_partials(L.out, js, n, acc, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  }
  return STEPS_OK;
}

int check_finite(steps_ctx *c, std::initializer_list<std::pair<const double *, int64_t>> arrays) {
  if (!(c->flags & STEPS_CHECK_FINITE)) return STEPS_OK;
  hipError_t e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  for (const auto &a : arrays) {
    if (a.second == 0) continue;
    e = steps::launch_check_finite(a.first, a.second, c->flag, c->stream);
    if (e != hipSuccess) return hip_fail(e, "finite-check launch");
  }
  int h = 0;
  e = hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost,
                     c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (h) return fail(STEPS_E_NONFINITE, "non-finite value in the inputs");
  return STEPS_OK;
}

steps_ctx *default_ctx(int *rc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_default_mu);
  if ((int)g_default.size() <= dev) g_default.resize(dev + 1, nullptr);
  if (!g_default[dev]) {
    steps_ctx *c = nullptr;
    *rc = steps_ctx_create(dev, &c);
    if (*rc) return nullptr;
    g_default[dev] = c;
  }
  *rc = STEPS_OK;
  return g_default[dev];
}

int validate_cosmo(const steps_cosmology *k) {
  if (!k) return fail(STEPS_E_INVAL, "cosmology is NULL");
  if (k->reserved != 0) return fail(STEPS_E_INVAL, "cosmology.reserved != 0");
  if (k->mode != STEPS_COMOVING_SPHERICAL && k->mode != STEPS_NEWTONIAN_TEST) {
    return fail(STEPS_E_INVAL, "unknown cosmology mode %d", k->mode);
  }
  if (!std::isfinite(k->G) || k->G < 0.0) {
    return fail(STEPS_E_INVAL, "G must be finite and >= 0 (0 = built-in)");
  }
  if (k->mode == STEPS_COMOVING_SPHERICAL) {
    if (!std::isfinite(k->H0) || k->H0 <= 0.0) {
      return fail(STEPS_E_INVAL, "H0 must be finite and > 0");
    }
    if (!std::isfinite(k->omega_m) || !std::isfinite(k->omega_l) ||
        !std::isfinite(k->omega_r) ||
        !(std::isfinite(k->omega_k) || std::isnan(k->omega_k))) {
      return fail(STEPS_E_INVAL, "density parameters must be finite");
    }
  }
  return STEPS_OK;
}

steps::Background make_background(const steps_cosmology *k) {
  const double ok = std::isnan(k->omega_k)
                        ? 1.0 - k->omega_m - k->omega_l - k->omega_r
                        : k->omega_k;
  return steps::Background(k->H0, k->omega_m, k->omega_l, k->omega_r, ok,
                           k->G, k->mode == STEPS_NEWTONIAN_TEST);
}

int check_force_args(steps_ctx *c, const double *pos, const double *mass,
                     const double *soft, int64_t n, const void *out,
                     size_t out_bytes, const char *out_name) {
  int rc = check_n(n);
  if (rc) return rc;
  if (n == 0) return STEPS_OK;
  const size_t v3 = 3 * (size_t)n * sizeof(double), v1 = (size_t)n * sizeof(double);
  if ((rc = check_ptr(c, pos, v3, "pos"))) return rc;
  if ((rc = check_ptr(c, mass, v1, "mass"))) return rc;
  if ((rc = check_ptr(c, soft, v1, "soft"))) return rc;
  if ((rc = check_ptr(c, out, out_bytes, out_name))) return rc;
  if (overlap(out, out_bytes, pos, v3) || overlap(out, out_bytes, mass, v1) ||
      overlap(out, out_bytes, soft, v1)) {
    return fail(STEPS_E_INVAL, "%s overlaps an input array", out_name);
  }
  return STEPS_OK;
}

}  // namespace

extern "C" {

const char *steps_version(void) { return STEPS_VERSION_STRING; }

const char *steps_last_error(void) { return t_err.c_str(); }

double steps_G(void) { return steps::newton_G(); }

double steps_kms_to_mpc_per_gyr(void) { return steps::kms_to_mpc_per_gyr(); }

int steps_ctx_create(int device, steps_ctx **out) {
  if (!out) return fail(STEPS_E_INVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) {
    return fail(STEPS_E_INVAL, "device %d out of range [0, %d)", device, count);
  }
  DeviceGuard g(device);
  steps_ctx *c = new (std::nothrow) steps_ctx();
  if (!c) return fail(STEPS_E_NOMEM, "out of host memory");
  c->device = device;
  e = hipMalloc((void **)&c->flag, sizeof(int));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(STEPS_E_NOMEM, "cannot allocate the context flag");
  }
  *out = c;
  return STEPS_OK;
}

int steps_ctx_destroy(steps_ctx *c) {
  if (!c) return STEPS_OK;
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    for (auto &d : g_default) {
      if (d == c) d = nullptr;
    }
  }
  DeviceGuard g(c->device);
  int rc = STEPS_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
  for (auto &p : c->prof_pending) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  for (auto ev : c->prof_pool) (void)hipEventDestroy(ev);
  if (c->part.p) (void)hipFree(c->part.p);
  if (c->shadow.p) (void)hipFree(c->shadow.p);
  if (c->arena.p) (void)hipFree(c->arena.p);
  if (c->flag) (void)hipFree(c->flag);
  delete c;
  return rc;
}

int steps_ctx_set_stream(steps_ctx *c, void *stream) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  c->stream = (hipStream_t)stream;
  return STEPS_OK;
}

int steps_ctx_set_precision(steps_ctx *c, int precision) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  if (precision != STEPS_FP64 && precision != STEPS_MIXED_F64ACC &&
      precision != STEPS_MIXED_KAHAN) {
    return fail(STEPS_E_INVAL, "unknown precision %d", precision);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->tile_forced && prec_class(precision) != prec_class(c->precision)) {
    c->tile_forced = false;  // a forced tile belongs to one kernel class
  }
  c->precision = precision;
  return STEPS_OK;
}

int steps_ctx_set_flags(steps_ctx *c, uint32_t flags) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  if (flags & ~(STEPS_CHECK_FINITE | STEPS_PROFILE)) {
    return fail(STEPS_E_INVAL, "unknown flag bits 0x%x", flags);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  c->flags = flags;
  return STEPS_OK;
}

int steps_ctx_set_tile(steps_ctx *c, const steps_tile *t) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if (!t) {
    c->tile_forced = false;
    return STEPS_OK;
  }
  if (!steps::find_force_variant(prec_class(c->precision), t->r, t->tj,
                                 t->variant)) {
    return fail(STEPS_E_INVAL,
                "no compiled force kernel with r=%d tj=%d variant=%d for this "
                "precision",
                t->r, t->tj, t->variant);
  }
  if (t->jsplit < 1 || t->jsplit > 1024) {
    return fail(STEPS_E_INVAL, "jsplit must be in [1, 1024]");
  }
  c->tile = *t;
  c->tile_forced = true;
  return STEPS_OK;
}

int steps_ctx_get_tile(steps_ctx *c, int64_t n, steps_tile *out) {
  if (!c || !out) return fail(STEPS_E_INVAL, "ctx or out is NULL");
  int rc = check_n(n);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  *out = choose_tile(c, std::max<int64_t>(n, 1));
  return STEPS_OK;
}

int steps_sync(steps_ctx *c) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  DeviceGuard g(c->device);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return STEPS_OK;
}

int steps_ctx_force_timing(steps_ctx *c, double *total_ms, int64_t *count,
                           int reset) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  for (auto &p : c->prof_pending) {
    hipError_t e = hipEventSynchronize(p.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    c->prof_ms += ms;
    c->prof_count += 1;
    c->prof_pool.push_back(p.first);
    c->prof_pool.push_back(p.second);
  }
  c->prof_pending.clear();
  if (total_ms) *total_ms = c->prof_ms;
  if (count) *count = c->prof_count;
  if (reset) {
    c->prof_ms = 0.0;
    c->prof_count = 0;
  }
  return STEPS_OK;
}

int steps_forces_ctx(steps_ctx *c, const double *pos, const double *mass,
                     const double *soft, int64_t n, double *acc) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = check_force_args(c, pos, mass, soft, n, acc,
                            3 * (size_t)n * sizeof(double), "acc");
  if (rc || n == 0) return rc;
  if ((rc = check_finite(c, {{pos, 3 * n}, {mass, n}, {soft, n}}))) return rc;
  return run_forces(c, pos, mass, soft, (int)n, acc);
}

int steps_forces(const double *pos, const double *mass, const double *soft,
                 int64_t n, double *acc) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_forces_ctx(c, pos, mass, soft, n, acc);
}

int steps_potential_ctx(steps_ctx *c, const double *pos, const double *mass,
                        const double *soft, int64_t n, double *phi) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = check_force_args(c, pos, mass, soft, n, phi,
                            (size_t)n * sizeof(double), "phi");
  if (rc || n == 0) return rc;
  if ((rc = check_finite(c, {{pos, 3 * n}, {mass, n}, {soft, n}}))) return rc;
  constexpr int R = 2, TJ = 128;
  const int64_t nb = (n + 256LL * R - 1) / (256LL * R);
  int64_t want = std::min<int64_t>((2048 + nb - 1) / nb,
                                   std::max<int64_t>(1, n / (2 * TJ)));
  int chunk = 0, js = 1;
  split_j(n, TJ, (int)std::max<int64_t>(1, std::min<int64_t>(want, 1024)),
          &chunk, &js);
  double *out = phi;
  if (js > 1) {
    rc = ensure(c, c->part, (size_t)js * (size_t)n * sizeof(double),
                "partial-sum");
    if (rc) return rc;
    out = (double *)c->part.p;
  }
  hipError_t e = steps::launch_potential(pos, mass, soft, (int)n, chunk, js,
                                         out, c->stream);
  if (e != hipSuccess) return hip_fail(e, "potential kernel launch");
  if (js > 1) {
    e = steps::launch_reduce_partials1(out, js, (int)n, phi, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  }
  return STEPS_OK;
}

int steps_potential(const double *pos, const double *mass, const double *soft,
                    int64_t n, double *phi) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_potential_ctx(c, pos, mass, soft, n, phi);
}

int steps_step_ctx(steps_ctx *c, double *pos, double *vel, const double *mass,
                   const double *soft, int64_t n, double *acc, double a,
                   double da, const steps_cosmology *cosmo) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if (!std::isfinite(a) || !std::isfinite(da)) {
    return fail(STEPS_E_INVAL, "a and da must be finite");
  }
  const bool newton = cosmo->mode == STEPS_NEWTONIAN_TEST;
  if (!newton && (a <= 0.0 || a + da <= 0.0)) {
    return fail(STEPS_E_INVAL, "need a > 0 and a + da > 0");
  }
  if ((rc = check_n(n))) return rc;
  const steps::Background bg = make_background(cosmo);
  double dt = 0.0;
  if (!bg.step_dt(a, da, &dt) || !std::isfinite(dt)) {
    return fail(STEPS_E_INVAL, "H(a)^2 <= 0 somewhere on [a, a + da]");
  }
  const double a1 = a + da, hdt = 0.5 * dt;
  const double ai3_0 = newton ? 1.0 : 1.0 / (a * a * a);
  const double ai3_1 = newton ? 1.0 : 1.0 / (a1 * a1 * a1);
  const double drag0 = 2.0 * bg.hubble(a), drag1 = 2.0 * bg.hubble(a1);
  const double denom = 1.0 + drag1 * hdt;
  if (!(denom > 0.0)) {
    return fail(STEPS_E_INVAL, "backward step too long: 1 + 2 H dt/2 <= 0");
  }
  if (n == 0) return STEPS_OK;
  const size_t v3 = 3 * (size_t)n * sizeof(double), v1 = (size_t)n * sizeof(double);
  if ((rc = check_ptr(c, pos, v3, "pos"))) return rc;
  if ((rc = check_ptr(c, vel, v3, "vel"))) return rc;
  if ((rc = check_ptr(c, mass, v1, "mass"))) return rc;
  if ((rc = check_ptr(c, soft, v1, "soft"))) return rc;
  if ((rc = check_ptr(c, acc, v3, "acc"))) return rc;
  const void *rw[3] = {pos, vel, acc};
  for (int x = 0; x < 3; ++x) {
    if (overlap(rw[x], v3, mass, v1) || overlap(rw[x], v3, soft, v1)) {
      return fail(STEPS_E_INVAL, "pos/vel/acc overlap mass or soft");
    }
    for (int y = x + 1; y < 3; ++y) {
      if (overlap(rw[x], v3, rw[y], v3)) {
        return fail(STEPS_E_INVAL, "pos, vel and acc must not overlap");
      }
    }
  }
  if ((rc = check_finite(c, {{pos, 3 * n}, {vel, 3 * n}, {mass, n}, {soft, n},
                             {acc, 3 * n}}))) {
    return rc;
  }
  const double G = bg.g, rad = bg.radial();
  hipError_t e = steps::launch_kick_drift(pos, vel, acc, (int)n, hdt,
                                          G * ai3_0, rad * ai3_0, drag0, dt,
                                          c->stream);
  if (e != hipSuccess) return hip_fail(e, "kick-drift kernel launch");
  if ((rc = run_forces(c, pos, mass, soft, (int)n, acc))) return rc;
  e = steps::launch_kick_end(pos, vel, acc, (int)n, hdt, G * ai3_1,
                             rad * ai3_1, 1.0 / denom, c->stream);
  if (e != hipSuccess) return hip_fail(e, "kick kernel launch");
  return STEPS_OK;
}

int steps_step(double *pos, double *vel, const double *mass,
               const double *soft, int64_t n, double *acc, double a,
               double da, const steps_cosmology *cosmo) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_step_ctx(c, pos, vel, mass, soft, n, acc, a, da, cosmo);
}

int steps_hubble(const steps_cosmology *cosmo, double a, double *out) {
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if (!out) return fail(STEPS_E_INVAL, "out is NULL");
  if (!std::isfinite(a) || (cosmo->mode == STEPS_COMOVING_SPHERICAL && a <= 0.0)) {
    return fail(STEPS_E_INVAL, "a must be finite and > 0");
  }
  const steps::Background bg = make_background(cosmo);
  if (!bg.newtonian_test && !(bg.e2(a) > 0.0)) {
    return fail(STEPS_E_INVAL, "H(a)^2 <= 0");
  }
  *out = bg.hubble(a);
  return STEPS_OK;
}

int steps_dt(const steps_cosmology *cosmo, double a, double da, double *out) {
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if (!out) return fail(STEPS_E_INVAL, "out is NULL");
  if (!std::isfinite(a) || !std::isfinite(da)) {
    return fail(STEPS_E_INVAL, "a and da must be finite");
  }
  if (cosmo->mode == STEPS_COMOVING_SPHERICAL && (a <= 0.0 || a + da <= 0.0)) {
    return fail(STEPS_E_INVAL, "need a > 0 and a + da > 0");
  }
  const steps::Background bg = make_background(cosmo);
  if (!bg.step_dt(a, da, out)) {
    return fail(STEPS_E_INVAL, "H(a)^2 <= 0 somewhere on [a, a + da]");
  }
  return STEPS_OK;
}

}  // extern "C"
