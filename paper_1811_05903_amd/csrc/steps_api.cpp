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
constexpr int64_t kMfmaMinN = 131072;
constexpr int64_t kSymMinN = 262144;
// below this many chunks (the memory cap binds from N ~ 2^22 and leaves
// fewer than 64 chunks from N ~ 2^23.5) the units no longer fill the device
// evenly and the one-sided kernel is used
constexpr int kSymMinChunks = 64;
constexpr int64_t kMixedSymR4MinN = 524288;
// from here the FP64 symmetric kernel takes its j-quad layout (variant 30):
// 108.8 against 112.3 ms at 2^19, 1559 against 1696 ms at 2^21, and 30.8
// against 30.4 ms at 2^18
constexpr int64_t kSymQuadMinN = 524288;

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
  Buffer diag;     // energy diagnostic: potential and reduction partials
  steps_tile batch_tile = {0, 0, 0, 0};  // shape of the last ensemble run
  // ensemble kernels chosen by STEPS_BATCH_AUTOTUNE: (kernel class, hash of
  // the active members' sizes) -> index into steps::batch_variants
  std::vector<std::pair<std::pair<int, uint64_t>, int>> batch_tuned;
  // periodic geometry (steps_ctx_set_periodic): images 0 = open sphere
  double box_L = 0.0;
  int images = STEPS_IMAGES_NONE;
  // shapes found by steps_autotune: (kernel class, n) -> tile
  std::vector<std::pair<std::pair<int, int64_t>, steps_tile>> tuned;
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
int check_ptr_dev(int device, const void *p, size_t bytes, const char *name) {
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
  if (at.type == hipMemoryTypeDevice && at.device != device) {
    return fail(STEPS_E_INVAL, "%s is on device %d, the call runs on device %d",
                name, at.device, device);
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

int check_ptr(const steps_ctx *c, const void *p, size_t bytes,
              const char *name) {
  return check_ptr_dev(c->device, p, bytes, name);
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

// Chunk count Q of the symmetric kernel (Q (Q + 1) / 2 units (R, s),
// R <= s, of chunk pairs, one workgroup each).  Units are equal, so the
// last round of workgroups runs part-empty; measured on MI355X, more and
// smaller units win until chunks of about 1024 particles (N = 2^18: 34.9 ms
// at Q = 64, 32.5 ms at Q = 256; N = 2^20: 458 ms from Q = 160 on; N =
// 2^21: 1547 against 1563 ms (FP64) and 751 against 761 ms (mixed) at
// Q = 256 against 174).  So: the largest Q up to 192 (256 from 2^20, where
// the larger reduction no longer outweighs the gain) with chunks of at
// least 1024 particles and the partial sums (24 n Q + 48 C Q (Q - 1) / 2
// bytes, about 48 Q n) under 32 GiB.
int sym_chunks(int64_t n) {
  const double cap = 32.0 * (1ull << 30);
  const int qmax = n >= (int64_t(1) << 20) ? 256 : 192;
  int best = 1;
  for (int want = 1; want <= qmax; ++want) {
    int64_t c = (n + want - 1) / want;
    c = std::max<int64_t>(256, (c + 255) / 256 * 256);
    const int q = (int)((n + c - 1) / c);
    const double bytes = 24.0 * n * q + 48.0 * c * q * (q - 1) / 2.0;
    if (q > 1 && (c < 1024 || bytes > cap)) break;
    best = want;
  }
  return best;
}

// j-split for an (r, tj, variant) shape: enough splits that the grid holds
// about 8192 (FP64 VALU), 16384 (mixed) or 65536 (FP64 matrix-core; its
// blocks are a quarter the size) workgroups, keeping every split at least
// two tiles.
int heuristic_jsplit(int cls, int64_t n, int r, int tj, int variant) {
  if (variant & steps::kVarSym) return sym_chunks(n);
  const int64_t nb = std::max<int64_t>(1, (n + 256LL * r - 1) / (256LL * r));
  const int64_t target = cls != steps::kClassF64 ? 16384
                         : (variant & steps::kVarMfma) ? 65536 : 8192;
  int64_t js = (target + nb - 1) / nb;
  js = std::min<int64_t>(js, std::max<int64_t>(1, n / (2LL * tj)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(js, 1024));
}

// Launch shape: a forced tile, else a shape tuned for (class, n), else the
// heuristic, measured on MI355X at N = 2^15 ... 2^21:
//   * FP64 from kSymMinN up: the symmetric matrix-core kernel (variant 14,
//     15% ahead of the one-sided one at 2^18 and 23-25% at 2^20 and 2^21,
//     1-2% ahead of variant 30 at 2^18), from kSymQuadMinN in its j-quad
//     layout (variant 30, a further 2% at 2^19, 4.6% at 2^20 and 7% at
//     2^21), while its memory cap still allows kSymMinChunks chunks;
//   * mixed from kSymMinN up: the symmetric mixed kernel (variant 10),
//     1.31x the one-sided one at 2^18 and 1.45x at 2^21 (FP64
//     accumulation), under the same chunk cap;
//   * FP64 from kMfmaMinN up: the matrix-core kernel (variant 6, tj 256),
//     5-7% ahead of the VALU kernel there and 7% behind it at 2^15;
//   * otherwise FP64 r = 4, mixed r = 2 (fewer registers, more waves to pair
//     up FP32 issue), r lowered for small n so that there are at least 256
//     i-blocks where possible;
//   * culled (sorted) variants from kSortMinN up; in FP64 the r^-3
//     correction stops at first order there (variant 3).
steps_tile choose_tile(const steps_ctx *c, int64_t n) {
  const int cls = prec_class(c->precision);
  steps_tile t;
  for (const auto &e : c->tuned) {
    if (!c->tile_forced && e.first.first == cls && e.first.second == n) {
      return e.second;
    }
  }
  if (c->tile_forced) {
    t = c->tile;
    if (t.jsplit == 0) t.jsplit = heuristic_jsplit(cls, n, t.r, t.tj, t.variant);
    return t;
  }
  const bool f64 = cls == steps::kClassF64;
  if (!f64 && n >= kSymMinN && sym_chunks(n) >= kSymMinChunks) {
    // symmetric mixed kernel: r = 2 at 2^18 (14.6 ms against 16.4 for
    // r = 4), r = 4 from 2^19 on (2^19: 53.5 ms against 56.4; 2^21: 808
    // against 888)
    t.r = n >= kMixedSymR4MinN ? 4 : 2;
    t.tj = 256;
    t.variant = steps::kVarCull | steps::kVarSym;
  } else if (f64 && n >= kMfmaMinN) {
    t.r = 1;
    t.tj = 256;
    t.variant = steps::kVarCull | steps::kVarMfma;
    if (n >= kSymMinN && sym_chunks(n) >= kSymMinChunks) {
      t.variant |= steps::kVarSym | (n >= kSymQuadMinN ? steps::kVarQuad : 0);
    }
  } else {
    int r = f64 ? 4 : 2;
    while (r > 1 && (n + 256LL * r - 1) / (256LL * r) < 256) r /= 2;
    t.r = r;
    t.tj = variant_tj(cls, r);
    t.variant = 0;
    if (n >= kSortMinN) {
      t.variant = steps::kVarCull | (f64 ? steps::kVarNoE2 : 0);
    }
  }
  t.jsplit = heuristic_jsplit(cls, n, t.r, t.tj, t.variant);
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

// Morton order for the culled kernels: bbox -> keys -> stable sort ->
// sorted copy (FP64 [5][n], or the FP32 shadow in mixed mode) -> boxes of
// tiles of tj particles, all in the context arena, with extra_bytes more
// carved after them.  Allocation comes first, so an error return has
// enqueued nothing; with enqueue false only the arena is sized.
struct SortedState {
  const int *perm = nullptr;  // sorted position -> caller index
  double *sorted = nullptr;   // FP64 x, y, z, m, h (kClassF64)
  float *shadow = nullptr;    // FP32 x, y, z, m, h (kClassMixed)
  double *info = nullptr;     // [ntiles][8] tile boxes
  char *extra = nullptr;
};

int sort_for_culling(steps_ctx *c, const double *pos, const double *mass,
                     const double *soft, int n, int tj, int cls,
                     size_t extra_bytes, SortedState *S, bool enqueue) {
  size_t cub_bytes = 0;
  hipError_t e = steps::sort_pairs(nullptr, &cub_bytes, nullptr, nullptr,
                                   nullptr, nullptr, n, c->stream);
  if (e != hipSuccess) return hip_fail(e, "radix sort size query");
  const int ntiles = (n + tj - 1) / tj;
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
  const size_t o_extra = cv.take(extra_bytes);
  int rc = ensure(c, c->arena, cv.off, "sort");
  if (rc || !enqueue) return rc;
  char *base = (char *)c->arena.p;
  double *box = (double *)(base + o_box);
  auto *k0 = (unsigned long long *)(base + o_k0);
  auto *k1 = (unsigned long long *)(base + o_k1);
  int *v0 = (int *)(base + o_v0), *v1 = (int *)(base + o_v1);
  S->info = (double *)(base + o_info);
  S->extra = extra_bytes ? base + o_extra : nullptr;
  if ((e = steps::launch_bbox(pos, n, (double *)(base + o_bpart), box,
                              c->stream)) != hipSuccess ||
      (e = steps::launch_morton(pos, n, box, k0, v0, c->stream)) !=
          hipSuccess) {
    return hip_fail(e, "sort-key kernel launch");
  }
  e = steps::sort_pairs(base + o_cub, &cub_bytes, k0, k1, v0, v1, n,
                        c->stream);
  if (e != hipSuccess) return hip_fail(e, "radix sort");
  S->perm = v1;
  if (cls == steps::kClassF64) {
    S->sorted = (double *)(base + o_soa);
    e = steps::launch_gather(pos, mass, soft, v1, n, S->sorted, nullptr,
                             c->stream);
    if (e == hipSuccess) {
      e = steps::launch_tile_info_f64(S->sorted, n, tj, S->info, c->stream);
    }
  } else {
    S->shadow = (float *)(base + o_soa);
    e = steps::launch_gather(pos, mass, soft, v1, n, nullptr, S->shadow,
                             c->stream);
    if (e == hipSuccess) {
      e = steps::launch_tile_info_f32(S->shadow, n, tj, S->info, c->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "gather kernel launch");
  return STEPS_OK;
}

// Periodic pair sum: FP64 kernel over Morton-sorted particles, j-split
// partials reduced in fixed order and scattered to the caller's order.
// Arguments validated; with enqueue false only the scratch is allocated.
int run_forces_periodic(steps_ctx *c, const double *pos, const double *mass,
                        const double *soft, int n, double *acc, bool enqueue) {
  if (c->precision != STEPS_FP64) {
    return fail(STEPS_E_UNSUPPORTED,
                "periodic boxes are computed in FP64 only");
  }
  const int tj = steps::periodic_tile();
  const int64_t nb = steps::periodic_iblocks(n);  // one-wave workgroups
  int64_t want = (32768 + nb - 1) / nb;
  want = std::min<int64_t>(want, std::max<int64_t>(1, n / (2LL * tj)));
  int chunk = 0, js = 1;
  split_j(n, tj, (int)std::max<int64_t>(1, std::min<int64_t>(want, 1024)),
          &chunk, &js);
  int rc = ensure(c, c->part, (size_t)js * 3 * (size_t)n * sizeof(double),
                  "partial-sum");
  if (rc) return rc;
  double *out = (double *)c->part.p;
  SortedState S;
  if ((rc = sort_for_culling(c, pos, mass, soft, n, tj, steps::kClassF64, 0,
                             &S, enqueue)) ||
      !enqueue) {
    return rc;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  if ((rc = prof_begin(c, ev))) return rc;
  hipError_t e = steps::launch_force_periodic(
      S.sorted, S.sorted + 3 * (size_t)n, S.sorted + 4 * (size_t)n, n,
      c->box_L, c->images, chunk, js, S.info, out, c->stream);
  if (e != hipSuccess) return hip_fail(e, "periodic force kernel launch");
  if ((rc = prof_end(c, ev))) return rc;
  e = steps::launch_reduce_scatter(out, js, n, S.perm, acc, c->stream);
  if (e != hipSuccess) return hip_fail(e, "partial reduction launch");
  return STEPS_OK;
}

// One force evaluation in launch shape t.  Scratch is allocated before
// anything is enqueued, so an STEPS_E_NOMEM return has enqueued nothing;
// with enqueue false only the scratch is allocated.
int run_forces_tile(steps_ctx *c, const double *pos, const double *mass,
                    const double *soft, int n, double *acc,
                    const steps_tile &t, bool enqueue) {
  const int cls = prec_class(c->precision);
  const steps::ForceVariant *v =
      steps::find_force_variant(cls, t.r, t.tj, t.variant);
  if (!v) {
    return fail(STEPS_E_INVAL,
                "no compiled force kernel with r=%d tj=%d variant=%d", t.r,
                t.tj, t.variant);
  }
  const bool cull = (t.variant & steps::kVarCull) != 0;
  const bool sym = (t.variant & steps::kVarSym) != 0;
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
    // symmetric variant: one (value, error) accumulator per off-diagonal unit
    const size_t jacc_bytes =
        sym ? (size_t)js * (js - 1) / 2 * 6 * (size_t)chunk * sizeof(double)
            : 0;
    SortedState S;
    if ((rc = sort_for_culling(c, pos, mass, soft, n, t.tj, cls, jacc_bytes,
                               &S, enqueue)) ||
        !enqueue) {
      return rc;
    }
    perm = S.perm;
    if (cls == steps::kClassF64) {
      L.pos = S.sorted;
      L.mass = S.sorted + 3 * (size_t)n;
      L.soft = S.sorted + 4 * (size_t)n;
    } else {
      L.shadow = S.shadow;
    }
    L.tinfo = S.info;
    if (sym && js > 1) L.jacc = (double *)S.extra;
  } else if (cls == steps::kClassMixed) {
    rc = ensure(c, c->shadow, 5 * (size_t)n * sizeof(float), "FP32 shadow");
    if (rc || !enqueue) return rc;
    e = steps::launch_shadow(pos, mass, soft, n, (float *)c->shadow.p,
                             c->stream);
    if (e != hipSuccess) return hip_fail(e, "shadow kernel launch");
    L.shadow = (const float *)c->shadow.p;
  } else {
    if (!enqueue) return STEPS_OK;
    L.pos = pos;
    L.mass = mass;
    L.soft = soft;
  }
  hipEvent_t ev[2];
  if ((rc = prof_begin(c, ev))) return rc;
  e = v->launch(L, c->stream);
  if (e != hipSuccess) return hip_fail(e, "force kernel launch");
  if ((rc = prof_end(c, ev))) return rc;
  if (sym) {
    e = steps::launch_reduce_sym(L.out, L.jacc, n, chunk, js, perm, acc,
                                 c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  } else if (cull) {
    e = steps::launch_reduce_scatter(L.out, js, n, perm, acc, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  } else if (js > 1) {
    e = steps::launch_reduce_partials(L.out, js, n, acc, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  }
  return STEPS_OK;
}

// Launch shape of the next force evaluation, with all its scratch
// allocated and nothing enqueued.  An automatically chosen symmetric shape
// whose partial sums (about 48 Q n bytes) do not fit falls back to the
// one-sided matrix-core kernel, which needs far less.
int reserve_forces(steps_ctx *c, int n, steps_tile *t) {
  *t = steps_tile{0, 0, 0, 0};
  if (n == 0) return STEPS_OK;
  if (c->images != STEPS_IMAGES_NONE) {
    return run_forces_periodic(c, nullptr, nullptr, nullptr, n, nullptr, false);
  }
  *t = choose_tile(c, n);
  int rc = run_forces_tile(c, nullptr, nullptr, nullptr, n, nullptr, *t, false);
  if (rc == STEPS_E_NOMEM && (t->variant & steps::kVarSym) && !c->tile_forced) {
    t->variant &= ~(steps::kVarSym | steps::kVarQuad);
    t->jsplit = heuristic_jsplit(prec_class(c->precision), n, t->r, t->tj,
                                 t->variant);
    rc = run_forces_tile(c, nullptr, nullptr, nullptr, n, nullptr, *t, false);
  }
  return rc;
}

// Enqueue acc <- S(pos) in shape t from reserve_forces.  Arguments validated.
int enqueue_forces(steps_ctx *c, const double *pos, const double *mass,
                   const double *soft, int n, double *acc, const steps_tile &t) {
  if (n == 0) return STEPS_OK;
  if (c->images != STEPS_IMAGES_NONE) {
    return run_forces_periodic(c, pos, mass, soft, n, acc, true);
  }
  return run_forces_tile(c, pos, mass, soft, n, acc, t, true);
}

// Enqueue acc <- S(pos) in the context's precision.  Arguments validated;
// an error return has enqueued nothing.
int run_forces(steps_ctx *c, const double *pos, const double *mass,
               const double *soft, int n, double *acc) {
  steps_tile t;
  int rc = reserve_forces(c, n, &t);
  if (rc) return rc;
  return enqueue_forces(c, pos, mass, soft, n, acc, t);
}

// Enqueue phi <- G-free softened potential (FP64, unsorted kernel r=2,
// tj=128, j-split to ~2048 workgroups).  Arguments validated.
int run_potential(steps_ctx *c, const double *pos, const double *mass,
                  const double *soft, int n, double *phi) {
  constexpr int R = 2, TJ = 128;
  const int64_t nb = (n + 256LL * R - 1) / (256LL * R);
  int64_t want = std::min<int64_t>((2048 + nb - 1) / nb,
                                   std::max<int64_t>(1, n / (2 * TJ)));
  int chunk = 0, js = 1;
  split_j(n, TJ, (int)std::max<int64_t>(1, std::min<int64_t>(want, 1024)),
          &chunk, &js);
  double *out = phi;
  if (js > 1) {
    int rc = ensure(c, c->part, (size_t)js * (size_t)n * sizeof(double),
                    "partial-sum");
    if (rc) return rc;
    out = (double *)c->part.p;
  }
  hipError_t e = steps::launch_potential(pos, mass, soft, n, chunk, js, out,
                                         c->stream);
  if (e != hipSuccess) return hip_fail(e, "potential kernel launch");
  if (js > 1) {
    e = steps::launch_reduce_partials1(out, js, n, phi, c->stream);
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
  if (k->flags & ~STEPS_REVERSED_GRAVITY) {
    return fail(STEPS_E_INVAL, "unknown cosmology flag bits 0x%x", k->flags);
  }
  if (k->mode != STEPS_COMOVING_SPHERICAL && k->mode != STEPS_NEWTONIAN_TEST &&
      k->mode != STEPS_COMOVING_PERIODIC) {
    return fail(STEPS_E_INVAL, "unknown cosmology mode %d", k->mode);
  }
  if (!std::isfinite(k->G) || k->G < 0.0) {
    return fail(STEPS_E_INVAL, "G must be finite and >= 0 (0 = built-in)");
  }
  if (k->mode != STEPS_NEWTONIAN_TEST) {
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
                           k->G, k->mode == STEPS_NEWTONIAN_TEST,
                           (k->flags & STEPS_REVERSED_GRAVITY) != 0,
                           k->mode == STEPS_COMOVING_PERIODIC);
}

int check_force_args_dev(int device, const double *pos, const double *mass,
                         const double *soft, int64_t n, const void *out,
                         size_t out_bytes, const char *out_name) {
  int rc = check_n(n);
  if (rc) return rc;
  if (n == 0) return STEPS_OK;
  const size_t v3 = 3 * (size_t)n * sizeof(double), v1 = (size_t)n * sizeof(double);
  if ((rc = check_ptr_dev(device, pos, v3, "pos"))) return rc;
  if ((rc = check_ptr_dev(device, mass, v1, "mass"))) return rc;
  if ((rc = check_ptr_dev(device, soft, v1, "soft"))) return rc;
  if ((rc = check_ptr_dev(device, out, out_bytes, out_name))) return rc;
  if (overlap(out, out_bytes, pos, v3) || overlap(out, out_bytes, mass, v1) ||
      overlap(out, out_bytes, soft, v1)) {
    return fail(STEPS_E_INVAL, "%s overlaps an input array", out_name);
  }
  return STEPS_OK;
}

int check_force_args(steps_ctx *c, const double *pos, const double *mass,
                     const double *soft, int64_t n, const void *out,
                     size_t out_bytes, const char *out_name) {
  return check_force_args_dev(c->device, pos, mass, soft, n, out, out_bytes,
                              out_name);
}

// Allocation-free pair sum (steps_forces_noalloc): largest n, and the plan
// of the fixed scratch for one call.  The launch shape is the one-sided FP64
// choice of choose_tile (the symmetric kernels' partial sums grow as
// n^2 / chunk and do not fit a fixed buffer), with its j-split lowered
// until the partial sums fit beside the sort scratch.
constexpr int64_t kNoAllocMaxN = 262144;

struct NoAllocPlan {
  steps_tile t = {0, 0, 0, 0};
  int chunk = 0, js = 1;
  size_t cub_bytes = 0;
  size_t o_box = 0, o_bpart = 0, o_k0 = 0, o_k1 = 0, o_v0 = 0, o_v1 = 0,
         o_cub = 0, o_info = 0, o_soa = 0, o_part = 0, total = 0;
};

int plan_noalloc(int n, hipStream_t s, NoAllocPlan *P) {
  steps_tile t;
  int r = 4;
  if (n >= kMfmaMinN) {
    t = steps_tile{1, 256, 0, steps::kVarCull | steps::kVarMfma};
  } else {
    while (r > 1 && (n + 256LL * r - 1) / (256LL * r) < 256) r /= 2;
    t = steps_tile{r, variant_tj(steps::kClassF64, r), 0,
                   n >= kSortMinN ? steps::kVarCull | steps::kVarNoE2 : 0};
  }
  const bool cull = (t.variant & steps::kVarCull) != 0;
  hipError_t e = steps::sort_pairs(nullptr, &P->cub_bytes, nullptr, nullptr,
                                   nullptr, nullptr, n, s);
  if (e != hipSuccess) return hip_fail(e, "radix sort size query");
  int want = heuristic_jsplit(steps::kClassF64, n, t.r, t.tj, t.variant);
  for (;;) {
    int chunk = 0, js = 1;
    split_j(n, t.tj, want, &chunk, &js);
    Carve cv;
    if (cull) {
      P->o_box = cv.take(6 * sizeof(double));
      P->o_bpart = cv.take((size_t)steps::bbox_blocks(n) * 6 * sizeof(double));
      P->o_k0 = cv.take((size_t)n * 8);
      P->o_k1 = cv.take((size_t)n * 8);
      P->o_v0 = cv.take((size_t)n * 4);
      P->o_v1 = cv.take((size_t)n * 4);
      P->o_cub = cv.take(P->cub_bytes);
      P->o_info = cv.take((size_t)((n + t.tj - 1) / t.tj) * 8 * sizeof(double));
      P->o_soa = cv.take(5 * (size_t)n * sizeof(double));
    }
    P->o_part = cv.take(cull || js > 1 ? (size_t)js * 3 * (size_t)n * sizeof(double) : 0);
    if (cv.off <= steps::kNoAllocScratchBytes) {
      t.jsplit = js;
      P->t = t;
      P->chunk = chunk;
      P->js = js;
      P->total = cv.off;
      return STEPS_OK;
    }
    if (want == 1) break;
    want = std::max(1, want / 2);
  }
  return fail(STEPS_E_INVAL,
              "n = %d needs more than the %zu bytes of fixed scratch", n,
              (size_t)steps::kNoAllocScratchBytes);
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
  if (c->diag.p) (void)hipFree(c->diag.p);
  if (c->flag) (void)hipFree(c->flag);
  delete c;
  return rc;
}

int steps_ctx_set_stream(steps_ctx *c, void *stream) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if ((hipStream_t)stream != c->stream) {
    // scratch may still be in use by work on the old stream; a later resize
    // frees it after synchronizing the new one only
    DeviceGuard g(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
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
  if (t->jsplit < 0 || t->jsplit > 1024) {
    return fail(STEPS_E_INVAL, "jsplit must be in [0, 1024]");
  }
  c->tile = *t;
  c->tile_forced = true;
  return STEPS_OK;
}

int steps_ctx_set_tuned(steps_ctx *c, int64_t n, const steps_tile *t) {
  if (!c || !t) return fail(STEPS_E_INVAL, "ctx or tile is NULL");
  int rc = check_n(n);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  const int cls = prec_class(c->precision);
  if (!steps::find_force_variant(cls, t->r, t->tj, t->variant)) {
    return fail(STEPS_E_INVAL,
                "no compiled force kernel with r=%d tj=%d variant=%d for this "
                "precision",
                t->r, t->tj, t->variant);
  }
  if (t->jsplit < 1 || t->jsplit > 1024) {
    return fail(STEPS_E_INVAL, "jsplit must be in [1, 1024]");
  }
  for (auto &e : c->tuned) {
    if (e.first.first == cls && e.first.second == n) {
      e.second = *t;
      return STEPS_OK;
    }
  }
  c->tuned.push_back({{cls, n}, *t});
  return STEPS_OK;
}

int steps_ctx_set_periodic(steps_ctx *c, double L, int32_t images) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if (images == STEPS_IMAGES_NONE) {
    c->images = STEPS_IMAGES_NONE;
    c->box_L = 0.0;
    return STEPS_OK;
  }
  if (images != STEPS_IMAGES_NEAREST && images != STEPS_IMAGES_ALL) {
    return fail(STEPS_E_INVAL, "unknown image rule %d", images);
  }
  if (!std::isfinite(L) || !(L > 0.0)) {
    return fail(STEPS_E_INVAL, "box side L must be finite and > 0");
  }
  c->images = images;
  c->box_L = L;
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

int steps_autotune(steps_ctx *c, const double *pos, const double *mass,
                   const double *soft, int64_t n, double *acc,
                   steps_tile *out) {
  if (!c || !out) return fail(STEPS_E_INVAL, "ctx or out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  if (c->images != STEPS_IMAGES_NONE) {
    return fail(STEPS_E_UNSUPPORTED, "the periodic kernel has one launch shape");
  }
  int rc = check_force_args(c, pos, mass, soft, n, acc,
                            3 * (size_t)n * sizeof(double), "acc");
  if (rc) return rc;
  const int cls = prec_class(c->precision);
  c->tuned.erase(std::remove_if(c->tuned.begin(), c->tuned.end(),
                                [&](const auto &e) {
                                  return e.first.first == cls &&
                                         e.first.second == n;
                                }),
                 c->tuned.end());
  const bool was_forced = c->tile_forced;
  const steps_tile was_tile = c->tile;
  c->tile_forced = false;
  const steps_tile h = choose_tile(c, std::max<int64_t>(n, 1));
  if (n == 0) {
    *out = h;
    c->tile_forced = was_forced;
    return STEPS_OK;
  }
  // candidates: every compiled kernel of the class with r in {1, 2, 4}
  // that the heuristic could choose (FP64 variants 0, 3, 6 and, from
  // kMfmaMinN, 14; mixed 0, 2 and, from kMfmaMinN, 10), each at its
  // heuristic j-split times 1/2,
  // 1 and 2 (the symmetric kernel's chunk count only times 1/2 and 1: its
  // heuristic count is already the largest within the memory cap)
  std::vector<steps_tile> cands;
  int nvar = 0;
  const steps::ForceVariant *vt = steps::force_variants(&nvar);
  for (int q = 0; q < nvar; ++q) {
    const steps::ForceVariant &v = vt[q];
    const bool sym = (v.variant & steps::kVarSym) != 0;
    const bool usable =
        cls == steps::kClassF64
            ? (v.variant == 0 || v.variant == 3 || v.variant == 6 ||
               (sym && n >= kMfmaMinN))
            : (v.variant == 0 || v.variant == 2 || (sym && n >= kMfmaMinN));
    if (v.cls != cls || !usable || (v.r != 1 && v.r != 2 && v.r != 4)) continue;
    const int hj = heuristic_jsplit(cls, n, v.r, v.tj, v.variant);
    {
      const int r = v.r, tj = v.tj, var = v.variant;
      for (int js : {std::max(1, hj / 2), hj, sym ? hj : std::min(1024, 2 * hj)}) {
        const steps_tile t = {r, tj, js, var};
        bool dup = false;
        for (const auto &q : cands) {
          dup |= q.r == t.r && q.tj == t.tj && q.jsplit == t.jsplit &&
                 q.variant == t.variant;
        }
        if (!dup) cands.push_back(t);
      }
    }
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  steps_tile best = h;
  float best_ms = -1.0f;
  // the heuristic shape first, also as a warm-up (scratch allocation); a
  // shape whose scratch does not fit is skipped
  c->tile = h;
  c->tile_forced = true;
  if (e == hipSuccess) rc = run_forces(c, pos, mass, soft, (int)n, acc);
  int skipped = rc == STEPS_E_NOMEM ? STEPS_E_NOMEM : STEPS_OK;
  if (skipped) rc = STEPS_OK;
  for (size_t k = 0; e == hipSuccess && rc == STEPS_OK && k < cands.size(); ++k) {
    c->tile = cands[k];
    e = hipEventRecord(t0, c->stream);
    if (e != hipSuccess) break;
    rc = run_forces(c, pos, mass, soft, (int)n, acc);
    if (rc == STEPS_E_NOMEM) {
      skipped = rc;
      rc = STEPS_OK;
      continue;
    }
    if (rc) break;
    e = hipEventRecord(t1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
      best_ms = ms;
      best = cands[k];
    }
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  c->tile_forced = was_forced;
  c->tile = was_tile;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  if (rc) return rc;
  if (best_ms < 0.0f && skipped) {
    return fail(skipped, "no candidate shape fits in device memory");
  }
  c->tuned.push_back({{cls, n}, best});
  *out = best;
  return STEPS_OK;
}

int steps_forces(const double *pos, const double *mass, const double *soft,
                 int64_t n, double *acc) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_forces_ctx(c, pos, mass, soft, n, acc);
}

int steps_forces_noalloc(const double *pos, const double *mass,
                         const double *soft, int64_t n, double *acc,
                         void *stream) {
  int rc = check_n(n);
  if (rc || n == 0) return rc;
  if (n > kNoAllocMaxN) {
    return fail(STEPS_E_INVAL,
                "n = %lld exceeds the allocation-free limit %lld",
                (long long)n, (long long)kNoAllocMaxN);
  }
  if (!pos) return fail(STEPS_E_INVAL, "pos is NULL");
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, pos);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(STEPS_E_INVAL, "pos (%p) is not memory known to HIP", pos);
  }
  int device = at.device;
  if (at.type != hipMemoryTypeDevice && (e = hipGetDevice(&device)) != hipSuccess) {
    return hip_fail(e, "hipGetDevice");
  }
  DeviceGuard g(device);
  if ((rc = check_force_args_dev(device, pos, mass, soft, n, acc,
                                 3 * (size_t)n * sizeof(double), "acc"))) {
    return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  void *scr = nullptr;
  if ((e = steps::noalloc_scratch(device, &scr)) != hipSuccess) {
    return hip_fail(e, "fixed scratch address");
  }
  NoAllocPlan P;
  const int ni = (int)n;
  if ((rc = plan_noalloc(ni, s, &P))) return rc;
  const steps::ForceVariant *v = steps::find_force_variant(
      steps::kClassF64, P.t.r, P.t.tj, P.t.variant);
  if (!v) return fail(STEPS_E_INVAL, "no compiled force kernel for n = %d", ni);
  char *base = (char *)scr;
  const bool cull = (P.t.variant & steps::kVarCull) != 0;
  steps::ForceLaunch L;
  L.n = ni;
  L.jchunk = P.chunk;
  L.jsplit = P.js;
  L.out = cull || P.js > 1 ? (double *)(base + P.o_part) : acc;
  const int *perm = nullptr;
  if (cull) {
    auto *k0 = (unsigned long long *)(base + P.o_k0);
    auto *k1 = (unsigned long long *)(base + P.o_k1);
    int *v0 = (int *)(base + P.o_v0), *v1 = (int *)(base + P.o_v1);
    double *box = (double *)(base + P.o_box);
    double *sorted = (double *)(base + P.o_soa);
    size_t cub_bytes = P.cub_bytes;
    if ((e = steps::launch_bbox(pos, ni, (double *)(base + P.o_bpart), box, s)) != hipSuccess ||
        (e = steps::launch_morton(pos, ni, box, k0, v0, s)) != hipSuccess ||
        (e = steps::sort_pairs(base + P.o_cub, &cub_bytes, k0, k1, v0, v1, ni, s)) !=
            hipSuccess ||
        (e = steps::launch_gather(pos, mass, soft, v1, ni, sorted, nullptr, s)) !=
            hipSuccess ||
        (e = steps::launch_tile_info_f64(sorted, ni, P.t.tj,
                                         (double *)(base + P.o_info), s)) != hipSuccess) {
      return hip_fail(e, "spatial sort launch");
    }
    perm = v1;
    L.pos = sorted;
    L.mass = sorted + 3 * (size_t)ni;
    L.soft = sorted + 4 * (size_t)ni;
    L.tinfo = (const double *)(base + P.o_info);
  } else {
    L.pos = pos;
    L.mass = mass;
    L.soft = soft;
  }
  if ((e = v->launch(L, s)) != hipSuccess) return hip_fail(e, "force kernel launch");
  if (cull) {
    e = steps::launch_reduce_scatter(L.out, P.js, ni, perm, acc, s);
  } else if (P.js > 1) {
    e = steps::launch_reduce_partials(L.out, P.js, ni, acc, s);
  }
  if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  return STEPS_OK;
}

int steps_potential_ctx(steps_ctx *c, const double *pos, const double *mass,
                        const double *soft, int64_t n, double *phi) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = check_force_args(c, pos, mass, soft, n, phi,
                            (size_t)n * sizeof(double), "phi");
  if (rc || n == 0) return rc;
  if (c->images != STEPS_IMAGES_NONE) {
    return fail(STEPS_E_UNSUPPORTED, "no softened potential for periodic boxes");
  }
  if ((rc = check_finite(c, {{pos, 3 * n}, {mass, n}, {soft, n}}))) return rc;
  return run_potential(c, pos, mass, soft, (int)n, phi);
}

int steps_energy_ctx(steps_ctx *c, const double *pos, const double *vel,
                     const double *mass, const double *soft, int64_t n,
                     double a, const steps_cosmology *cosmo, double *out) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  if (!out) return fail(STEPS_E_INVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if (c->images != STEPS_IMAGES_NONE || cosmo->mode == STEPS_COMOVING_PERIODIC) {
    return fail(STEPS_E_UNSUPPORTED, "no energies for periodic boxes");
  }
  const bool newton = cosmo->mode == STEPS_NEWTONIAN_TEST;
  if (newton) a = 1.0;
  if (!std::isfinite(a) || !(a > 0.0)) {
    return fail(STEPS_E_INVAL, "a must be finite and > 0");
  }
  if ((rc = check_force_args(c, pos, mass, soft, n, vel,
                             3 * (size_t)n * sizeof(double), "vel"))) {
    return rc;
  }
  double sums[6] = {0, 0, 0, 0, 0, 0};
  if (n > 0) {
    if ((rc = check_finite(c, {{pos, 3 * n}, {vel, 3 * n}, {mass, n},
                               {soft, n}}))) {
      return rc;
    }
    Carve cv;
    const size_t o_phi = cv.take((size_t)n * sizeof(double));
    const size_t o_part = cv.take((size_t)steps::energy_blocks((int)n) * 6 * sizeof(double));
    const size_t o_out = cv.take(6 * sizeof(double));
    if ((rc = ensure(c, c->diag, cv.off, "energy"))) return rc;
    char *base = (char *)c->diag.p;
    double *phi = (double *)(base + o_phi);
    if ((rc = run_potential(c, pos, mass, soft, (int)n, phi))) return rc;
    hipError_t e = steps::launch_energy(pos, vel, mass, phi, (int)n,
                                        (double *)(base + o_part),
                                        (double *)(base + o_out), c->stream);
    if (e != hipSuccess) return hip_fail(e, "energy kernel launch");
    e = hipMemcpyAsync(sums, base + o_out, sizeof(sums), hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "energy readback");
  }
  const steps::Background bg = make_background(cosmo);
  const double a2 = a * a;
  out[0] = a2 * sums[0];
  out[2] = bg.g * sums[1];
  out[3] = -0.5 * bg.radial() * sums[2];
  out[1] = (out[2] + out[3]) / a;
  out[4] = a2 * sums[3];
  out[5] = a2 * sums[4];
  out[6] = a2 * sums[5];
  return STEPS_OK;
}

int steps_kinetic_ctx(steps_ctx *c, const double *vel, const double *mass,
                      int64_t n, double a, double *out) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  if (!out) return fail(STEPS_E_INVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  if (!std::isfinite(a) || !(a > 0.0)) {
    return fail(STEPS_E_INVAL, "a must be finite and > 0");
  }
  int rc = check_n(n);
  if (rc) return rc;
  double sums[6] = {0, 0, 0, 0, 0, 0};
  if (n > 0) {
    if ((rc = check_ptr(c, vel, 3 * (size_t)n * sizeof(double), "vel"))) return rc;
    if ((rc = check_ptr(c, mass, (size_t)n * sizeof(double), "mass"))) return rc;
    if ((rc = check_finite(c, {{vel, 3 * n}, {mass, n}}))) return rc;
    Carve cv;
    const size_t o_part = cv.take((size_t)steps::energy_blocks((int)n) * 6 * sizeof(double));
    const size_t o_out = cv.take(6 * sizeof(double));
    if ((rc = ensure(c, c->diag, cv.off, "energy"))) return rc;
    char *base = (char *)c->diag.p;
    hipError_t e = steps::launch_energy(nullptr, vel, mass, nullptr, (int)n,
                                        (double *)(base + o_part),
                                        (double *)(base + o_out), c->stream);
    if (e != hipSuccess) return hip_fail(e, "energy kernel launch");
    e = hipMemcpyAsync(sums, base + o_out, sizeof(sums), hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "energy readback");
  }
  const double a2 = a * a;
  out[0] = a2 * sums[0];
  out[1] = a2 * sums[3];
  out[2] = a2 * sums[4];
  out[3] = a2 * sums[5];
  return STEPS_OK;
}

int steps_kinetic(const double *vel, const double *mass, int64_t n, double a,
                  double *out) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_kinetic_ctx(c, vel, mass, n, a, out);
}

int steps_energy(const double *pos, const double *vel, const double *mass,
                 const double *soft, int64_t n, double a,
                 const steps_cosmology *cosmo, double *out) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_energy_ctx(c, pos, vel, mass, soft, n, a, cosmo, out);
}

int steps_potential(const double *pos, const double *mass, const double *soft,
                    int64_t n, double *phi) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_potential_ctx(c, pos, mass, soft, n, phi);
}

// One KDK step; the caller holds the context lock and the device guard.
static int step_impl(steps_ctx *c, double *pos, double *vel, const double *mass,
                     const double *soft, int64_t n, double *acc, double a,
                     double da, const steps_cosmology *cosmo) {
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if (cosmo->mode == STEPS_COMOVING_PERIODIC && c->images == STEPS_IMAGES_NONE) {
    return fail(STEPS_E_INVAL,
                "periodic mode needs a periodic context (steps_ctx_set_periodic)");
  }
  if (cosmo->mode == STEPS_COMOVING_SPHERICAL && c->images != STEPS_IMAGES_NONE) {
    return fail(STEPS_E_INVAL,
                "the spherical equations of motion need an open (non-periodic) "
                "context");
  }
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
  // scratch first: a failing allocation must not leave a half-applied step
  steps_tile shape;
  if ((rc = reserve_forces(c, (int)n, &shape))) return rc;
  const double G = bg.g, rad = bg.radial();
  hipError_t e = steps::launch_kick_drift(pos, vel, acc, (int)n, hdt,
                                          G * ai3_0, rad * ai3_0, drag0, dt,
                                          c->stream);
  if (e != hipSuccess) return hip_fail(e, "kick-drift kernel launch");
  if ((rc = enqueue_forces(c, pos, mass, soft, (int)n, acc, shape))) return rc;
  e = steps::launch_kick_end(pos, vel, acc, (int)n, hdt, G * ai3_1,
                             rad * ai3_1, 1.0 / denom, c->stream);
  if (e != hipSuccess) return hip_fail(e, "kick kernel launch");
  return STEPS_OK;
}

int steps_step_ctx(steps_ctx *c, double *pos, double *vel, const double *mass,
                   const double *soft, int64_t n, double *acc, double a,
                   double da, const steps_cosmology *cosmo) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  return step_impl(c, pos, vel, mass, soft, n, acc, a, da, cosmo);
}

// Adaptive step of Eq. 12 at the current state; the caller holds the lock.
static int adaptive_impl(steps_ctx *c, const double *pos, const double *vel,
                         const double *soft, const double *acc, int64_t n,
                         double a, const steps_cosmology *cosmo, double eps,
                         double dt_max, double *dt_out, double *da_out) {
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  const bool newton = cosmo->mode == STEPS_NEWTONIAN_TEST;
  if (!std::isfinite(a) || (!newton && !(a > 0.0))) {
    return fail(STEPS_E_INVAL, "a must be finite (and > 0 unless Newtonian)");
  }
  if (!std::isfinite(eps) || !(eps > 0.0) || !std::isfinite(dt_max) ||
      !(dt_max > 0.0)) {
    return fail(STEPS_E_INVAL, "eps and dt_max must be finite and > 0");
  }
  if ((rc = check_n(n))) return rc;
  double q = INFINITY;
  if (n > 0) {
    const size_t v3 = 3 * (size_t)n * sizeof(double), v1 = (size_t)n * sizeof(double);
    if ((rc = check_ptr(c, pos, v3, "pos"))) return rc;
    if ((rc = check_ptr(c, vel, v3, "vel"))) return rc;
    if ((rc = check_ptr(c, soft, v1, "soft"))) return rc;
    if ((rc = check_ptr(c, acc, v3, "acc"))) return rc;
    if ((rc = check_finite(c, {{pos, 3 * n}, {vel, 3 * n}, {soft, n},
                               {acc, 3 * n}}))) {
      return rc;
    }
    Carve cv;
    const size_t o_part = cv.take((size_t)steps::dt_blocks((int)n) * sizeof(double));
    const size_t o_out = cv.take(sizeof(double));
    if ((rc = ensure(c, c->diag, cv.off, "adaptive step"))) return rc;
    char *base = (char *)c->diag.p;
    const steps::Background bg = make_background(cosmo);
    const double ai3 = newton ? 1.0 : 1.0 / (a * a * a);
    hipError_t e = steps::launch_dt_min(pos, vel, acc, soft, (int)n,
                                        bg.g * ai3, bg.radial() * ai3,
                                        2.0 * bg.hubble(a),
                                        (double *)(base + o_part),
                                        (double *)(base + o_out), c->stream);
    if (e != hipSuccess) return hip_fail(e, "adaptive step kernel launch");
    e = hipMemcpyAsync(&q, base + o_out, sizeof(double), hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "adaptive step readback");
  }
  double dt = dt_max;
  if (std::isfinite(q)) dt = std::min(dt_max, std::sqrt(2.0 * eps * q));
  if (!(dt > 0.0)) {
    return fail(STEPS_E_INVAL,
                "the step of Eq. 12 is zero: a particle with zero softening "
                "(eta = 2.8 h = 0) has a nonzero acceleration");
  }
  double da = 0.0;
  if (!make_background(cosmo).da_for_dt(a, dt, &da)) {
    return fail(STEPS_E_INVAL, "no scale-factor step reaches dt = %g Gyr", dt);
  }
  *dt_out = dt;
  *da_out = da;
  return STEPS_OK;
}

int steps_adaptive_dt_ctx(steps_ctx *c, const double *pos, const double *vel,
                          const double *soft, const double *acc, int64_t n,
                          double a, const steps_cosmology *cosmo, double eps,
                          double dt_max, double *dt, double *da) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  if (!dt || !da) return fail(STEPS_E_INVAL, "dt or da is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  return adaptive_impl(c, pos, vel, soft, acc, n, a, cosmo, eps, dt_max, dt, da);
}

int steps_adaptive_dt(const double *pos, const double *vel, const double *soft,
                      const double *acc, int64_t n, double a,
                      const steps_cosmology *cosmo, double eps, double dt_max,
                      double *dt, double *da) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_adaptive_dt_ctx(c, pos, vel, soft, acc, n, a, cosmo, eps,
                               dt_max, dt, da);
}

int steps_run_adaptive_ctx(steps_ctx *c, double *pos, double *vel,
                           const double *mass, const double *soft, int64_t n,
                           double *acc, double a0, double a1,
                           const steps_cosmology *cosmo, double eps,
                           double dt_max, int64_t max_steps,
                           int64_t *steps_taken, double *a_reached) {
  if (!c) return fail(STEPS_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  if (!std::isfinite(a0) || !std::isfinite(a1) || !(a1 >= a0)) {
    return fail(STEPS_E_INVAL, "need finite a0 <= a1");
  }
  if (max_steps < 0) return fail(STEPS_E_INVAL, "max_steps < 0");
  int rc = validate_cosmo(cosmo);
  if (rc) return rc;
  if ((rc = check_force_args(c, pos, mass, soft, n, acc,
                             3 * (size_t)n * sizeof(double), "acc"))) {
    return rc;
  }
  if (n > 0 && (rc = run_forces(c, pos, mass, soft, (int)n, acc))) return rc;
  double a = a0;
  int64_t k = 0;
  while (a < a1 && k < max_steps) {
    double dt = 0.0, da = 0.0;
    if ((rc = adaptive_impl(c, pos, vel, soft, acc, n, a, cosmo, eps, dt_max,
                            &dt, &da))) {
      break;
    }
    const bool last = a + da >= a1;
    if (last) da = a1 - a;
    if ((rc = step_impl(c, pos, vel, mass, soft, n, acc, a, da, cosmo))) break;
    a = last ? a1 : a + da;
    ++k;
  }
  if (steps_taken) *steps_taken = k;
  if (a_reached) *a_reached = a;
  return rc;
}

int steps_step(double *pos, double *vel, const double *mass,
               const double *soft, int64_t n, double *acc, double a,
               double da, const steps_cosmology *cosmo) {
  int rc = STEPS_OK;
  steps_ctx *c = default_ctx(&rc);
  if (!c) return rc;
  return steps_step_ctx(c, pos, vel, mass, soft, n, acc, a, da, cosmo);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles
// ---------------------------------------------------------------------------
namespace {

struct BatchLayout {
  std::vector<int> tile_beg, tile_end;   // member-local tiles, slot ranges
  std::vector<int4> items;               // (i0, iend, jbeg, jend)
  std::vector<int> tbase;                // first tile of the item's j-range
  std::vector<int> islot;                // j-chunk (output plane) of the item,
                                         // or the unit's slot (symmetric)
  std::vector<int> kc;                   // j-chunks of each member
  int planes = 1;                        // largest kc
  // symmetric kernels: items are the chunk-pair units of every member
  bool sym = false;
  int chunk = 0;                         // particles per chunk
  std::vector<int> moff, mq, mubase;     // per member: start, chunks, slot base
  int64_t nslots = 0;
};

// Work items the persistent ensemble kernel should have to spread evenly
// over the GPU: a few per resident block.
constexpr int64_t kBatchTargetItems = 8192;

// Chunk size of the symmetric ensemble kernels: the smallest of 1024,
// 2048, ... whose unit slots (72 chunk bytes per unit, Q (Q + 1) / 2 units
// for a member of Q chunks) fit in 8 GiB.
// Steps per replay of the multi-step ensemble graph.
constexpr int kBatchGraphSteps = 10;

int batch_sym_chunk(const std::vector<int> &soff) {
  const double cap = 8.0 * (1ull << 30);
  int c = 1024;
  for (;; c *= 2) {
    double slots = 0.0;
    for (size_t a = 0; a + 1 < soff.size(); ++a) {
      const double q = (double)((soff[a + 1] - soff[a] + c - 1) / c);
      slots += q * (q + 1) / 2;
    }
    if (slots * 72.0 * c <= cap || c >= (1 << 20)) return c;
  }
}

// Tiles of tj slots from each member's start; items of 256 r slots.  When
// the ensemble gives fewer than kBatchTargetItems such blocks, each member's
// j-range is also split into up to K tile-aligned chunks (K = target / items,
// at most 64, never below one tile per chunk); an item then covers one
// (i-block, j-chunk) and writes its own output plane, the planes being
// summed in order afterwards.  Items are ordered by member size (the cost of
// an item), largest first.
//
// Symmetric kernels instead cut each member into chunks of batch_sym_chunk
// particles (multiples of tj from the member's start) and take one item per
// unit (R, s), R <= s, of chunk pairs, members largest first, off-diagonal
// units of a member before its diagonal ones.  Unit (R, s) of member a
// writes slot mubase[a] + s (s + 1) / 2 + R.
BatchLayout batch_layout(const std::vector<int> &soff, int r, int tj,
                         bool sym) {
  BatchLayout L;
  const int A = (int)soff.size() - 1;
  std::vector<int> mtb(A);
  int64_t blocks = 0;
  for (int a = 0; a < A; ++a) {
    mtb[a] = (int)L.tile_beg.size();
    for (int k = soff[a]; k < soff[a + 1]; k += tj) {
      L.tile_beg.push_back(k);
      L.tile_end.push_back(std::min(k + tj, soff[a + 1]));
    }
    blocks += (soff[a + 1] - soff[a] + 256LL * r - 1) / (256LL * r);
  }
  std::vector<int> order(A);
  for (int a = 0; a < A; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return soff[x + 1] - soff[x] > soff[y + 1] - soff[y];
  });
  if (sym) {
    L.sym = true;
    L.chunk = batch_sym_chunk(soff);
    const int C = L.chunk;
    L.kc.assign(A, 1);
    L.moff.assign(soff.begin(), soff.end() - 1);
    L.mq.assign(A, 0);
    L.mubase.assign(A, 0);
    for (int a = 0; a < A; ++a) {
      L.mq[a] = (soff[a + 1] - soff[a] + C - 1) / C;
      L.mubase[a] = (int)L.nslots;
      L.nslots += (int64_t)L.mq[a] * (L.mq[a] + 1) / 2;
    }
    for (int a : order) {
      const int q = L.mq[a], o = soff[a], e = soff[a + 1];
      for (int pass = 0; pass < 2; ++pass) {  // off-diagonal, then diagonal
        for (int cs = 0; cs < q; ++cs) {
          for (int cr = 0; cr <= cs; ++cr) {
            if ((cr == cs) != (pass == 1)) continue;
            L.items.push_back(make_int4(o + cr * C, std::min(e, o + (cr + 1) * C),
                                        o + cs * C, std::min(e, o + (cs + 1) * C)));
            L.tbase.push_back(mtb[a] + cs * (C / tj));
            L.islot.push_back(L.mubase[a] + cs * (cs + 1) / 2 + cr);
          }
        }
      }
    }
    return L;
  }
  const int K = (int)std::min<int64_t>(
      64, std::max<int64_t>(1, (kBatchTargetItems + blocks - 1) / std::max<int64_t>(1, blocks)));
  L.kc.assign(A, 1);
  std::vector<int> per(A, 1);
  for (int a = 0; a < A; ++a) {
    const int ntl = (soff[a + 1] - soff[a] + tj - 1) / tj;
    const int ka = std::max(1, std::min(K, ntl));
    per[a] = (ntl + ka - 1) / ka;                  // tiles per chunk
    L.kc[a] = std::max(1, (ntl + per[a] - 1) / per[a]);  // all non-empty
    L.planes = std::max(L.planes, L.kc[a]);
  }
  for (int a : order) {
    for (int i0 = soff[a]; i0 < soff[a + 1]; i0 += 256 * r) {
      const int iend = std::min(i0 + 256 * r, soff[a + 1]);
      for (int c = 0; c < L.kc[a]; ++c) {
        const int jbeg = soff[a] + c * per[a] * tj;
        const int jend = std::min(soff[a + 1], jbeg + per[a] * tj);
        L.items.push_back(make_int4(i0, iend, jbeg, jend));
        L.tbase.push_back(mtb[a] + c * per[a]);
        L.islot.push_back(c);
      }
    }
  }
  return L;
}

bool batch_is_sym(const steps::BatchVariant *v) {
  return (v->variant & steps::kVarSym) != 0;
}

// Everything one ensemble run keeps on the device (carved from the arena).
struct BatchDev {
  double *pos, *vel, *acc, *mass, *soft;  // sorted state, [.][N]
  double *tpos, *tvel, *tacc, *tmass, *tsoft;  // re-sort staging
  int *orig, *torig, *mid;
  unsigned long long *k0, *k1;
  int *v0, *v1;
  void *cub;
  size_t cub_bytes;
  float *shadow;
  double *info, *table, *bpart, *box;
  int *tile_beg, *tile_end, *tbase, *counter;
  int4 *items;
  int *islot, *kc;
  double *part;  // [planes][3][N] j-chunk partials (planes > 1)
  double *usum;  // symmetric kernels: [slots][9][chunk] unit sums
  int *moff, *mq, *mubase;  // symmetric kernels: per-member layout
};

struct BatchRun {
  steps_ctx *c;
  hipStream_t s;
  int N, A, nsteps, cls, kahan;
  BatchDev d;
  const steps::BatchVariant *v = nullptr;
  int ntiles = 0, nitems = 0, planes = 1;
  bool sym = false;
  int chunk = 0;
};

hipError_t batch_forces(BatchRun &R) {
  hipError_t e;
  if (R.cls == steps::kClassF64) {
    e = steps::launch_batch_tile_info_f64(R.d.pos, R.N, R.d.tile_beg,
                                          R.d.tile_end, R.ntiles, R.d.info,
                                          R.s);
  } else {
    e = steps::launch_batch_tile_info_f32(R.d.shadow, R.N, R.d.tile_beg,
                                          R.d.tile_end, R.ntiles, R.d.info,
                                          R.s);
  }
  if (e != hipSuccess) return e;
  steps::BatchLaunch L;
  L.pos = R.d.pos;
  L.mass = R.d.mass;
  L.soft = R.d.soft;
  L.shadow = R.d.shadow;
  L.stride = R.N;
  L.items = R.d.items;
  L.tbase = R.d.tbase;
  L.islot = R.planes > 1 ? R.d.islot : nullptr;
  L.nitems = R.nitems;
  L.tinfo = R.d.info;
  L.out = R.planes > 1 ? R.d.part : R.d.acc;
  L.counter = R.d.counter + 1;
  L.kahan = R.kahan;
  if (R.sym) {
    L.islot = R.d.islot;
    L.out = nullptr;
    L.usum = R.d.usum;
    L.chunk = R.chunk;
    e = R.v->launch(L, R.s);
    if (e == hipSuccess) {
      e = steps::launch_batch_reduce_sym(R.d.usum, R.N, R.d.mid, R.d.moff,
                                         R.d.mq, R.d.mubase, R.chunk, R.d.acc,
                                         R.s);
    }
    return e;
  }
  e = R.v->launch(L, R.s);
  if (e == hipSuccess && R.planes > 1) {
    e = steps::launch_batch_reduce(R.d.part, R.N, R.d.mid, R.d.kc, R.d.acc, R.s);
  }
  return e;
}

// One KDK step; only kernel launches (capturable).
hipError_t batch_step(BatchRun &R) {
  hipError_t e = steps::launch_batch_kick_drift(
      R.d.pos, R.d.vel, R.d.acc, R.cls == steps::kClassMixed ? R.d.shadow : nullptr,
      R.d.mid, R.N, R.d.table, R.A, R.nsteps, R.d.counter, R.s);
  if (e == hipSuccess) e = batch_forces(R);
  if (e == hipSuccess) {
    e = steps::launch_batch_kick_end(R.d.pos, R.d.vel, R.d.acc, R.d.mid, R.N,
                                     R.d.table, R.A, R.nsteps, R.d.counter, R.s);
  }
  if (e == hipSuccess) e = steps::launch_batch_advance(R.d.counter, R.s);
  return e;
}

// Morton order within each member (member index in the key's high bits).
hipError_t batch_resort(BatchRun &R) {
  int mbits = 1;
  while ((1 << mbits) < R.A) ++mbits;
  const int qbits = std::min(21, (63 - mbits) / 3);
  hipError_t e = steps::launch_bbox(R.d.pos, R.N, R.d.bpart, R.d.box, R.s);
  if (e == hipSuccess) {
    e = steps::launch_batch_morton(R.d.pos, R.N, R.d.box, R.d.mid, qbits,
                                   R.d.k0, R.d.v0, R.s);
  }
  if (e == hipSuccess) {
    e = steps::sort_pairs(R.d.cub, &R.d.cub_bytes, R.d.k0, R.d.k1, R.d.v0,
                          R.d.v1, R.N, R.s);
  }
  const int *perm = R.d.v1;
  struct {
    double *a, *t;
    int comps;
  } cols[5] = {{R.d.pos, R.d.tpos, 3}, {R.d.vel, R.d.tvel, 3},
               {R.d.acc, R.d.tacc, 3}, {R.d.mass, R.d.tmass, 1},
               {R.d.soft, R.d.tsoft, 1}};
  for (auto &c : cols) {
    if (e != hipSuccess) break;
    e = steps::launch_gather_cols(c.a, R.N, perm, R.N, c.t, R.N, c.comps, R.s);
    if (e == hipSuccess) {
      e = hipMemcpyAsync(c.a, c.t, (size_t)c.comps * R.N * sizeof(double),
                         hipMemcpyDeviceToDevice, R.s);
    }
  }
  if (e == hipSuccess) e = steps::launch_gather_int(R.d.orig, perm, R.N, R.d.torig, R.s);
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.orig, R.d.torig, (size_t)R.N * sizeof(int),
                       hipMemcpyDeviceToDevice, R.s);
  }
  if (e == hipSuccess && R.cls == steps::kClassMixed) {
    e = steps::launch_shadow(R.d.pos, R.d.mass, R.d.soft, R.N, R.d.shadow, R.s);
  }
  return e;
}

hipError_t upload_layout(BatchRun &R, const BatchLayout &L) {
  R.ntiles = (int)L.tile_beg.size();
  R.nitems = (int)L.items.size();
  hipError_t e = hipMemcpyAsync(R.d.tile_beg, L.tile_beg.data(),
                                L.tile_beg.size() * sizeof(int),
                                hipMemcpyHostToDevice, R.s);
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.tile_end, L.tile_end.data(),
                       L.tile_end.size() * sizeof(int), hipMemcpyHostToDevice,
                       R.s);
  }
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.items, L.items.data(), L.items.size() * sizeof(int4),
                       hipMemcpyHostToDevice, R.s);
  }
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.tbase, L.tbase.data(), L.tbase.size() * sizeof(int),
                       hipMemcpyHostToDevice, R.s);
  }
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.islot, L.islot.data(), L.islot.size() * sizeof(int),
                       hipMemcpyHostToDevice, R.s);
  }
  if (e == hipSuccess) {
    e = hipMemcpyAsync(R.d.kc, L.kc.data(), L.kc.size() * sizeof(int),
                       hipMemcpyHostToDevice, R.s);
  }
  if (e == hipSuccess && L.sym) {
    const std::vector<int> *src[3] = {&L.moff, &L.mq, &L.mubase};
    int *dst[3] = {R.d.moff, R.d.mq, R.d.mubase};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      e = hipMemcpyAsync(dst[k], src[k]->data(), src[k]->size() * sizeof(int),
                         hipMemcpyHostToDevice, R.s);
    }
  }
  R.planes = L.planes;
  R.sym = L.sym;
  R.chunk = L.chunk;
  // the host vectors must outlive the copies
  if (e == hipSuccess) e = hipStreamSynchronize(R.s);
  return e;
}

// Validate one member and fill its rows of the step table; returns a
// STEPS_E_* code (the member is then skipped) or STEPS_OK.
int batch_member(const steps_cosmology *k, double a0, double a1, int nsteps,
                 int A, int a, std::vector<double> &table) {
  if (validate_cosmo(k) != STEPS_OK) return STEPS_E_INVAL;
  if (k->mode == STEPS_COMOVING_PERIODIC) return STEPS_E_UNSUPPORTED;
  const bool newton = k->mode == STEPS_NEWTONIAN_TEST;
  // the log-uniform grid needs a0, a1 > 0 in both modes
  if (!std::isfinite(a0) || !std::isfinite(a1) || a0 <= 0.0 || a1 <= 0.0) {
    return STEPS_E_INVAL;
  }
  const steps::Background bg = make_background(k);
  const double lr = std::log(a1 / a0);
  double ak = a0;
  for (int s = 0; s < nsteps; ++s) {
    const double an = s + 1 == nsteps ? a1 : a0 * std::exp(lr * (s + 1) / nsteps);
    double dt = 0.0;
    if (!bg.step_dt(ak, an - ak, &dt) || !std::isfinite(dt)) return STEPS_E_INVAL;
    const double hdt = 0.5 * dt;
    const double i0 = newton ? 1.0 : 1.0 / (ak * ak * ak);
    const double i1 = newton ? 1.0 : 1.0 / (an * an * an);
    const double den = 1.0 + 2.0 * bg.hubble(an) * hdt;
    if (!(den > 0.0)) return STEPS_E_INVAL;
    double *t = &table[((size_t)s * A + a) * steps::kBatchScalars];
    t[0] = hdt;
    t[1] = bg.g * i0;
    t[2] = bg.radial() * i0;
    t[3] = 2.0 * bg.hubble(ak);
    t[4] = dt;
    t[5] = bg.g * i1;
    t[6] = bg.radial() * i1;
    t[7] = 1.0 / den;
    ak = an;
  }
  return STEPS_OK;
}

// Captured step graphs of one ensemble run: [0] one step, [1] kBatchGraphSteps
// steps in a row.
struct BatchGraphs {
  hipGraph_t g[2] = {nullptr, nullptr};
  hipGraphExec_t x[2] = {nullptr, nullptr};
};

int batch_fail_cleanup(int rc, hipStream_t s, BatchGraphs &gr) {
  for (int k = 0; k < 2; ++k) {
    if (gr.x[k]) (void)hipGraphExecDestroy(gr.x[k]);
    if (gr.g[k]) (void)hipGraphDestroy(gr.g[k]);
    gr.x[k] = nullptr;
    gr.g[k] = nullptr;
  }
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  return rc;
}

}  // namespace

extern "C" {

int steps_batch_tile(steps_ctx *c, steps_tile *out) {
  if (!c || !out) return fail(STEPS_E_INVAL, "ctx or out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  *out = c->batch_tile;
  return STEPS_OK;
}

int steps_batch_run(steps_ctx *c, const steps_batch *b, int32_t *status) {
  if (!c || !b) return fail(STEPS_E_INVAL, "ctx or batch is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  if (c->images != STEPS_IMAGES_NONE) {
    return fail(STEPS_E_UNSUPPORTED, "ensembles run the spherical equations only");
  }
  const int B = b->members;
  if (B < 1) return fail(STEPS_E_INVAL, "members must be >= 1");
  if (b->nsteps < 1) return fail(STEPS_E_INVAL, "nsteps must be >= 1");
  if (!b->offsets || !b->cosmo || !b->a0 || !b->a1) {
    return fail(STEPS_E_INVAL, "offsets, cosmo, a0 and a1 must be host arrays");
  }
  if (b->flags & ~(STEPS_BATCH_GRAPH | STEPS_BATCH_AUTOTUNE)) {
    return fail(STEPS_E_INVAL, "unknown batch flag bits 0x%x", b->flags);
  }
  if (b->resort_every < 0) return fail(STEPS_E_INVAL, "resort_every < 0");
  if (b->offsets[0] != 0) return fail(STEPS_E_INVAL, "offsets[0] != 0");
  for (int m = 0; m < B; ++m) {
    if (b->offsets[m + 1] < b->offsets[m]) {
      return fail(STEPS_E_INVAL, "offsets decrease at member %d", m);
    }
  }
  const int64_t Nc = b->offsets[B];
  int rc = check_n(Nc);
  if (rc) return rc;
  const int nsteps = b->nsteps;

  // per-member validation and step tables (active members only)
  std::vector<int32_t> st(B, STEPS_OK);
  std::vector<int> active;
  std::vector<double> table_all((size_t)nsteps * B * steps::kBatchScalars, 0.0);
  for (int m = 0; m < B; ++m) {
    st[m] = batch_member(&b->cosmo[m], b->a0[m], b->a1[m], nsteps, B, m,
                         table_all);
    if (st[m] == STEPS_OK && b->offsets[m + 1] > b->offsets[m]) active.push_back(m);
  }
  auto write_status = [&]() {
    if (status) {
      for (int m = 0; m < B; ++m) status[m] = st[m];
    }
  };
  if (active.empty()) {
    write_status();
    return STEPS_OK;
  }
  const size_t v3 = 3 * (size_t)Nc * sizeof(double), v1 = (size_t)Nc * sizeof(double);
  if ((rc = check_ptr(c, b->pos, v3, "batch.pos"))) return rc;
  if ((rc = check_ptr(c, b->vel, v3, "batch.vel"))) return rc;
  if ((rc = check_ptr(c, b->acc, v3, "batch.acc"))) return rc;
  if ((rc = check_ptr(c, b->mass, v1, "batch.mass"))) return rc;
  if ((rc = check_ptr(c, b->soft, v1, "batch.soft"))) return rc;
  const void *rw[3] = {b->pos, b->vel, b->acc};
  for (int x = 0; x < 3; ++x) {
    if (overlap(rw[x], v3, b->mass, v1) || overlap(rw[x], v3, b->soft, v1)) {
      return fail(STEPS_E_INVAL, "batch pos/vel/acc overlap mass or soft");
    }
    for (int y = x + 1; y < 3; ++y) {
      if (overlap(rw[x], v3, rw[y], v3)) {
        return fail(STEPS_E_INVAL, "batch pos, vel and acc must not overlap");
      }
    }
  }

  // slot layout of the active members
  const int A = (int)active.size();
  std::vector<int> soff(A + 1, 0), orig, mid;
  for (int a = 0; a < A; ++a) {
    const int m = active[a];
    soff[a + 1] = soff[a] + (int)(b->offsets[m + 1] - b->offsets[m]);
    for (int64_t i = b->offsets[m]; i < b->offsets[m + 1]; ++i) {
      orig.push_back((int)i);
      mid.push_back(a);
    }
  }
  const int N = soff[A];
  std::vector<double> table((size_t)nsteps * A * steps::kBatchScalars);
  for (int s = 0; s < nsteps; ++s) {
    for (int a = 0; a < A; ++a) {
      std::copy_n(&table_all[((size_t)s * B + active[a]) * steps::kBatchScalars],
                  steps::kBatchScalars,
                  &table[((size_t)s * A + a) * steps::kBatchScalars]);
    }
  }

  // kernel candidates of this precision
  BatchRun R;
  R.c = c;
  R.N = N;
  R.A = A;
  R.nsteps = nsteps;
  R.cls = prec_class(c->precision);
  R.kahan = c->precision == STEPS_MIXED_KAHAN;
  std::vector<const steps::BatchVariant *> cands;
  {
    int cnt = 0;
    const steps::BatchVariant *bv = steps::batch_variants(&cnt);
    for (int k = 0; k < cnt; ++k) {
      if (bv[k].cls == R.cls) cands.push_back(&bv[k]);
    }
  }
  if (c->tile_forced) {
    // a shape forced on the context must name an ensemble kernel
    for (const auto *v : cands) {
      if (v->r == c->tile.r && v->tj == c->tile.tj &&
          v->variant == c->tile.variant) {
        R.v = v;
      }
    }
    if (!R.v) {
      return fail(STEPS_E_INVAL,
                  "the forced tile (r=%d tj=%d variant=%d) names no ensemble "
                  "kernel for this precision",
                  c->tile.r, c->tile.tj, c->tile.variant);
    }
    cands.assign(1, R.v);  // nothing for STEPS_BATCH_AUTOTUNE to choose
  } else {
    // default: FP64 r=4 without the e^2 term; mixed: the symmetric kernel
    // with r = 4 (the fastest at the size of workload 4)
    for (const auto *v : cands) {
      const bool want = R.cls == steps::kClassF64
                            ? (v->r == 4 && v->variant == 3)
                            : (v->r == 4 && batch_is_sym(v));
      if (want) R.v = v;
    }
    if (!R.v) R.v = cands.front();
    // without the autotuner only the default runs: size scratch for it alone
    if (!(b->flags & STEPS_BATCH_AUTOTUNE)) cands.assign(1, R.v);
  }
  // a choice the autotuner made before for this precision class and list of
  // member sizes on this context is reused without timing
  uint64_t sizes_hash = 1469598103934665603ull;  // FNV-1a over the sizes
  for (int a = 0; a < A; ++a) {
    sizes_hash = (sizes_hash ^ (uint64_t)(soff[a + 1] - soff[a])) * 1099511628211ull;
  }
  const std::pair<int, uint64_t> tune_key{R.cls, sizes_hash};
  int bcount = 0;
  const steps::BatchVariant *btable = steps::batch_variants(&bcount);
  if ((b->flags & STEPS_BATCH_AUTOTUNE) && cands.size() > 1) {
    for (const auto &e : c->batch_tuned) {
      if (e.first == tune_key) {
        R.v = &btable[e.second];
        cands.assign(1, R.v);
      }
    }
  }

  // device memory
  size_t cub_bytes = 0;
  hipError_t e = steps::sort_pairs(nullptr, &cub_bytes, nullptr, nullptr,
                                   nullptr, nullptr, N, c->stream);
  if (e != hipSuccess) return hip_fail(e, "radix sort size query");
  const size_t max_tiles = (size_t)N / 128 + A + 1;
  size_t max_items = 1, max_planes = 1, max_usum = 0;
  for (const auto *v : cands) {  // every layout the run may use
    const BatchLayout L = batch_layout(soff, v->r, v->tj, batch_is_sym(v));
    max_items = std::max(max_items, L.items.size());
    max_planes = std::max(max_planes, (size_t)L.planes);
    if (L.sym) {
      max_usum = std::max(max_usum, (size_t)L.nslots * 9 * (size_t)L.chunk);
    }
  }
  const size_t n = (size_t)N, d8 = sizeof(double);
  Carve cv;
  const size_t o_pos = cv.take(3 * n * d8), o_vel = cv.take(3 * n * d8),
               o_acc = cv.take(3 * n * d8), o_mass = cv.take(n * d8),
               o_soft = cv.take(n * d8), o_tpos = cv.take(3 * n * d8),
               o_tvel = cv.take(3 * n * d8), o_tacc = cv.take(3 * n * d8),
               o_tmass = cv.take(n * d8), o_tsoft = cv.take(n * d8),
               o_orig = cv.take(n * 4), o_torig = cv.take(n * 4),
               o_mid = cv.take(n * 4), o_k0 = cv.take(n * 8),
               o_k1 = cv.take(n * 8), o_v0 = cv.take(n * 4),
               o_v1 = cv.take(n * 4), o_cub = cv.take(cub_bytes),
               o_shadow = cv.take(R.cls == steps::kClassMixed ? 5 * n * 4 : 0),
               o_info = cv.take(max_tiles * 8 * d8),
               o_table = cv.take(table.size() * d8),
               o_bpart = cv.take((size_t)steps::bbox_blocks(N) * 6 * d8),
               o_box = cv.take(6 * d8), o_tb = cv.take(max_tiles * 4),
               o_te = cv.take(max_tiles * 4), o_tbase = cv.take(max_items * 4),
               o_items = cv.take(max_items * sizeof(int4)),
               o_islot = cv.take(max_items * 4), o_kc = cv.take((size_t)A * 4),
               o_part = cv.take(max_planes > 1 ? max_planes * 3 * n * d8 : 0),
               o_usum = cv.take(max_usum * d8),
               o_moff = cv.take((size_t)A * 4), o_mq = cv.take((size_t)A * 4),
               o_mub = cv.take((size_t)A * 4),
               o_cnt = cv.take(2 * 4);
  if ((rc = ensure(c, c->arena, cv.off, "ensemble"))) return rc;
  char *base = (char *)c->arena.p;
  BatchDev &d = R.d;
  d.pos = (double *)(base + o_pos);
  d.vel = (double *)(base + o_vel);
  d.acc = (double *)(base + o_acc);
  d.mass = (double *)(base + o_mass);
  d.soft = (double *)(base + o_soft);
  d.tpos = (double *)(base + o_tpos);
  d.tvel = (double *)(base + o_tvel);
  d.tacc = (double *)(base + o_tacc);
  d.tmass = (double *)(base + o_tmass);
  d.tsoft = (double *)(base + o_tsoft);
  d.orig = (int *)(base + o_orig);
  d.torig = (int *)(base + o_torig);
  d.mid = (int *)(base + o_mid);
  d.k0 = (unsigned long long *)(base + o_k0);
  d.k1 = (unsigned long long *)(base + o_k1);
  d.v0 = (int *)(base + o_v0);
  d.v1 = (int *)(base + o_v1);
  d.cub = base + o_cub;
  d.cub_bytes = cub_bytes;
  d.shadow = R.cls == steps::kClassMixed ? (float *)(base + o_shadow) : nullptr;
  d.info = (double *)(base + o_info);
  d.table = (double *)(base + o_table);
  d.bpart = (double *)(base + o_bpart);
  d.box = (double *)(base + o_box);
  d.tile_beg = (int *)(base + o_tb);
  d.tile_end = (int *)(base + o_te);
  d.tbase = (int *)(base + o_tbase);
  d.items = (int4 *)(base + o_items);
  d.islot = (int *)(base + o_islot);
  d.kc = (int *)(base + o_kc);
  d.part = max_planes > 1 ? (double *)(base + o_part) : nullptr;
  d.usum = max_usum ? (double *)(base + o_usum) : nullptr;
  d.moff = (int *)(base + o_moff);
  d.mq = (int *)(base + o_mq);
  d.mubase = (int *)(base + o_mub);
  d.counter = (int *)(base + o_cnt);

  // the run uses its own stream (graph capture needs one), ordered after
  // the context's earlier work
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  R.s = s;
  BatchGraphs gr;
#define BATCH_TRY(expr, what)                                              \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      return batch_fail_cleanup(hip_fail(e_, what), s, gr);                \
    }                                                                      \
  } while (0)

  BATCH_TRY(hipMemcpyAsync(d.orig, orig.data(), n * sizeof(int),
                           hipMemcpyHostToDevice, s), "upload");
  BATCH_TRY(hipMemcpyAsync(d.mid, mid.data(), n * sizeof(int),
                           hipMemcpyHostToDevice, s), "upload");
  BATCH_TRY(hipMemcpyAsync(d.table, table.data(), table.size() * d8,
                           hipMemcpyHostToDevice, s), "upload");
  BATCH_TRY(steps::launch_gather_cols(b->pos, (int)Nc, d.orig, N, d.pos, N, 3, s), "gather");
  BATCH_TRY(steps::launch_gather_cols(b->vel, (int)Nc, d.orig, N, d.vel, N, 3, s), "gather");
  BATCH_TRY(steps::launch_gather_cols(b->mass, (int)Nc, d.orig, N, d.mass, N, 1, s), "gather");
  BATCH_TRY(steps::launch_gather_cols(b->soft, (int)Nc, d.orig, N, d.soft, N, 1, s), "gather");
  BATCH_TRY(hipStreamSynchronize(s), "upload");  // host vectors outlive the copies
  BATCH_TRY(batch_resort(R), "ensemble sort");

  // first forces, optionally timing every candidate kernel (once per
  // precision class and list of member sizes on this context: see above)
  if ((b->flags & STEPS_BATCH_AUTOTUNE) && cands.size() > 1) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    BATCH_TRY(hipEventCreate(&t0), "hipEventCreate");
    BATCH_TRY(hipEventCreate(&t1), "hipEventCreate");
    float best = 0.0f;
    const steps::BatchVariant *win = nullptr;
    for (const auto *v : cands) {
      R.v = v;
      BATCH_TRY(upload_layout(R, batch_layout(soff, v->r, v->tj, batch_is_sym(v))),
                "layout");
      BATCH_TRY(steps::launch_batch_init(d.counter, s), "init");
      BATCH_TRY(hipEventRecord(t0, s), "hipEventRecord");
      BATCH_TRY(batch_forces(R), "ensemble force");
      BATCH_TRY(hipEventRecord(t1, s), "hipEventRecord");
      BATCH_TRY(hipEventSynchronize(t1), "hipEventSynchronize");
      float ms = 0.0f;
      BATCH_TRY(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
      if (!win || ms < best) {
        best = ms;
        win = v;
      }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    R.v = win;
    c->batch_tuned.push_back({tune_key, (int)(win - btable)});
  }
  BATCH_TRY(upload_layout(R, batch_layout(soff, R.v->r, R.v->tj, batch_is_sym(R.v))),
            "layout");
  BATCH_TRY(steps::launch_batch_init(d.counter, s), "init");
  BATCH_TRY(batch_forces(R), "ensemble force");
  c->batch_tile = steps_tile{R.v->r, R.v->tj, R.planes, R.v->variant};

  // steps; with graphs, runs of kBatchGraphSteps steps replay one graph
  // that holds them all (the step counter and the scalar table live on the
  // device, so consecutive steps capture as the same kernels), and the
  // steps left before a re-sort or the end replay a one-step graph
  const bool use_graph = (b->flags & STEPS_BATCH_GRAPH) != 0;
  auto capture = [&](int which, int steps) -> hipError_t {
    hipError_t e1 = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e1 != hipSuccess) return e1;
    hipError_t ce = hipSuccess;
    for (int k = 0; k < steps && ce == hipSuccess; ++k) ce = batch_step(R);
    hipError_t ee = hipStreamEndCapture(s, &gr.g[which]);
    if (ce != hipSuccess) return ce;
    if (ee != hipSuccess) return ee;
    return hipGraphInstantiate(&gr.x[which], gr.g[which], nullptr, nullptr, 0);
  };
  for (int k = 0; k < nsteps;) {
    if (b->resort_every > 0 && k > 0 && k % b->resort_every == 0) {
      BATCH_TRY(batch_resort(R), "ensemble sort");
    }
    if (!use_graph) {
      BATCH_TRY(batch_step(R), "ensemble step");
      ++k;
      continue;
    }
    // steps before the next re-sort or the end
    int left = nsteps - k;
    if (b->resort_every > 0) {
      left = std::min(left, b->resort_every - k % b->resort_every);
    }
    const int which = left >= kBatchGraphSteps ? 1 : 0;
    if (!gr.x[which]) {
      BATCH_TRY(capture(which, which ? kBatchGraphSteps : 1), "ensemble step capture");
    }
    BATCH_TRY(hipGraphLaunch(gr.x[which], s), "hipGraphLaunch");
    k += which ? kBatchGraphSteps : 1;
  }

  // back to the caller's order and arrays
  BATCH_TRY(steps::launch_scatter_cols(d.pos, N, d.orig, N, b->pos, (int)Nc, 3, s), "scatter");
  BATCH_TRY(steps::launch_scatter_cols(d.vel, N, d.orig, N, b->vel, (int)Nc, 3, s), "scatter");
  BATCH_TRY(steps::launch_scatter_cols(d.acc, N, d.orig, N, b->acc, (int)Nc, 3, s), "scatter");
  BATCH_TRY(hipStreamSynchronize(s), "ensemble run");
#undef BATCH_TRY
  batch_fail_cleanup(STEPS_OK, s, gr);
  write_status();
  return STEPS_OK;
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
