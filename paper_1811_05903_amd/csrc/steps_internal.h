// Internal interface between the host runtime and the gfx950 kernels of
// libsteps.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace steps {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)

enum PrecClass { kClassF64 = 0, kClassMixed = 1 };

// Arguments of one force-kernel launch.  pos/mass/soft point at double
// arrays (kClassF64) or at the FP32 shadow (kClassMixed): x,y,z,m,h as
// five [n] float arrays starting at `shadow`.
struct ForceLaunch {
  const double *pos = nullptr;
  const double *mass = nullptr;
  const double *soft = nullptr;
  const float *shadow = nullptr;
  int n = 0;
  int jchunk = 0;   // j-range per grid row (multiple of the tile size)
  int jsplit = 1;   // grid rows; > 1 writes partials
  double *out = nullptr;       // [jsplit][3][n] (or acc when jsplit == 1)
  int kahan = 0;               // mixed only: Kahan FP32 accumulation
  const double *tinfo = nullptr;  // culled variants: [n/tj][8] tile boxes
  double *jacc = nullptr;  // symmetric variant: [Q(Q-1)/2][6][jchunk]
};

// variant bits of a force kernel
constexpr int kVarNoE2 = 1;  // FP64: r^-3 correction to first order only
constexpr int kVarCull = 2;  // sorted input, (wave, tile) softening culling
constexpr int kVarMfma = 4;  // FP64 far field on the matrix cores (with kVarCull)
constexpr int kVarSym = 8;   // each pair once, both sides kept (with kVarMfma)
constexpr int kVarQuad = 16; // symmetric FP64: j-quad layout of the far blocks;
                             // symmetric mixed: Newton step on the FP32 r^-3

struct ForceVariant {
  int cls;   // PrecClass
  int r;     // i-particles per lane
  int tj;    // j-particles per LDS tile
  int variant;  // kernel-specific option (FP64: 0 with e^2 term, 1 without)
  hipError_t (*launch)(const ForceLaunch &, hipStream_t);
};

// Arguments of one persistent ensemble force launch (sorted state, culled).
struct BatchLaunch {
  const double *pos = nullptr, *mass = nullptr, *soft = nullptr;  // FP64 [.][stride]
  const float *shadow = nullptr;  // mixed: [5][stride]
  int stride = 0;                 // total particles of the ensemble
  const int4 *items = nullptr;    // (i0, iend, jbeg, jend) per work item
  const int *tbase = nullptr;     // first tile of the item's j-range
  const int *islot = nullptr;     // output plane of each item (NULL: all 0)
  int nitems = 0;
  const double *tinfo = nullptr;  // [tiles][8]
  double *out = nullptr;          // [planes][3][stride]
  int *counter = nullptr;         // work counter, 0 before the launch
  int kahan = 0;
  // symmetric variants: items are chunk-pair units, islot their slots of
  // usum ([slots][9][chunk]: i-side [3][chunk], j-side (value, error)
  // [6][chunk])
  double *usum = nullptr;
  int chunk = 0;
};

struct BatchVariant {
  int cls, r, tj, variant;
  hipError_t (*launch)(const BatchLaunch &, hipStream_t);
};
const BatchVariant *batch_variants(int *count);

// ---- ensemble O(N) kernels (steps_batch.hip) ----------------------------
// per (step, member) scalars: hdt, G/a0^3, radial/a0^3, 2H(a0), dt,
// G/a1^3, radial/a1^3, 1/(1 + 2H(a1) hdt)
constexpr int kBatchScalars = 8;
hipError_t launch_batch_init(int *counter, hipStream_t s);
hipError_t launch_batch_kick_drift(double *pos, double *vel, const double *S,
                                   float *shadow, const int *mid, int n,
                                   const double *table, int members,
                                   int nsteps, int *counter, hipStream_t s);
hipError_t launch_batch_kick_end(const double *pos, double *vel,
                                 const double *S, const int *mid, int n,
                                 const double *table, int members, int nsteps,
                                 const int *counter, hipStream_t s);
// acc <- sum of the j-chunk planes of part ([planes][3][n]), kc[member]
// planes for the particles of each member, in plane order
hipError_t launch_batch_reduce(const double *part, int n, const int *mid,
                               const int *kc, double *acc, hipStream_t s);
hipError_t launch_batch_advance(int *counter, hipStream_t s);
// symmetric ensemble: acc [3][n] (sorted arena) from the unit slots of
// usum; member a starts at slot moff[a] of the arena, has mq[a] chunks and
// its unit (R, s) in slot mubase[a] + s (s + 1) / 2 + R
hipError_t launch_batch_reduce_sym(const double *usum, int n, const int *mid,
                                   const int *moff, const int *mq,
                                   const int *mubase, int chunk, double *acc,
                                   hipStream_t s);
hipError_t launch_batch_tile_info_f64(const double *soa, int stride,
                                      const int *beg, const int *end,
                                      int ntiles, double *info, hipStream_t s);
hipError_t launch_batch_tile_info_f32(const float *soa, int stride,
                                      const int *beg, const int *end,
                                      int ntiles, double *info, hipStream_t s);
hipError_t launch_batch_morton(const double *pos, int n, const double *box,
                               const int *mid, int qbits,
                               unsigned long long *keys, int *vals,
                               hipStream_t s);
hipError_t launch_gather_cols(const double *src, int ss, const int *idx, int n,
                              double *dst, int ds, int comps, hipStream_t s);
hipError_t launch_gather_int(const int *src, const int *idx, int n, int *dst,
                             hipStream_t s);
hipError_t launch_scatter_cols(const double *src, int ss, const int *idx,
                               int n, double *dst, int ds, int comps,
                               hipStream_t s);

// All compiled force-kernel variants.
const ForceVariant *force_variants(int *count);
const ForceVariant *find_force_variant(int cls, int r, int tj, int variant);

// ---- spatial sort for the culled variants (steps_sort.hip) -------------
int bbox_blocks(int n);
// box[6] = (lo xyz, hi xyz) of pos; part holds bbox_blocks(n) * 6 doubles
hipError_t launch_bbox(const double *pos, int n, double *part, double *box,
                       hipStream_t s);
hipError_t launch_morton(const double *pos, int n, const double *box,
                         unsigned long long *keys, int *vals, hipStream_t s);
// stable radix sort of (key, index); tmp == nullptr queries *tmp_bytes
hipError_t sort_pairs(void *tmp, size_t *tmp_bytes,
                      const unsigned long long *kin, unsigned long long *kout,
                      const int *vin, int *vout, int n, hipStream_t s);
// sorted [5][n] FP64 copy (x, y, z, m, h) and/or FP32 shadow (may be null)
hipError_t launch_gather(const double *pos, const double *mass,
                         const double *soft, const int *perm, int n,
                         double *sorted, float *shadow, hipStream_t s);
// per tile of tj sorted particles: (lo xyz, hi xyz, hmax, 0)
hipError_t launch_tile_info_f64(const double *sorted, int n, int tj,
                                double *info, hipStream_t s);
hipError_t launch_tile_info_f32(const float *shadow, int n, int tj,
                                double *info, hipStream_t s);
// acc[d][perm[k]] = sum over the jsplit partials [jsplit][3][n]
hipError_t launch_reduce_scatter(const double *part, int jsplit, int n,
                                 const int *perm, double *acc, hipStream_t s);

// Symmetric variant: acc[d][perm[p]] = planes k..Q-1 of iplane ([Q][3][n])
// plus the accumulators of units (R, k), R < k, of jacc, k = p / chunk.
hipError_t launch_reduce_sym(const double *iplane, const double *jacc, int n,
                             int chunk, int nchunks, const int *perm,
                             double *acc, hipStream_t s);

// Sum jsplit partials [jsplit][3][n] into acc [3][n] in fixed order.
hipError_t launch_reduce_partials(const double *part, int jsplit, int n,
                                  double *acc, hipStream_t s);

// Softened potential (FP64), same partial layout with 1 component.
hipError_t launch_potential(const double *pos, const double *mass,
                            const double *soft, int n, int jchunk, int jsplit,
                            double *out, hipStream_t s);
hipError_t launch_reduce_partials1(const double *part, int jsplit, int n,
                                   double *phi, hipStream_t s);

// Energy sums out[6] = (sum 1/2 m|v|^2, sum 1/2 m phi, sum m|x|^2,
// sum m v_x, sum m v_y, sum m v_z); part holds energy_blocks(n) * 6 doubles.
// periodic pair sum (Eqs. 2 and 5): images 1 = nearest image, 2 = every
// image within 2.6 L; out as the force kernels ([jsplit][3][n] partials)
int periodic_tile();
int periodic_iblocks(int n);
// over Morton-sorted particles with the boxes of their tiles of
// periodic_tile() particles in tinfo
hipError_t launch_force_periodic(const double *pos, const double *mass,
                                 const double *soft, int n, double L,
                                 int images, int jchunk, int jsplit,
                                 const double *tinfo, double *out,
                                 hipStream_t s);
// adaptive step: out[0] <- min_i 2.8 h_i / |g S_i + rad x_i - drag v_i|
int dt_blocks(int n);
hipError_t launch_dt_min(const double *pos, const double *vel,
                         const double *acc, const double *soft, int n,
                         double g, double rad, double drag, double *part,
                         double *out, hipStream_t s);
int energy_blocks(int n);
hipError_t launch_energy(const double *pos, const double *vel,
                         const double *mass, const double *phi, int n,
                         double *part, double *out, hipStream_t s);

// ---- fixed scratch of steps_forces_noalloc (steps_noalloc.hip) ---------
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// This device's copy of the fixed scratch array (kNoAllocScratchBytes),
// its address looked up once per device.
hipError_t noalloc_scratch(int device, void **out);

// FP32 shadow [5][n] (x, y, z, m, h) from the FP64 inputs.
hipError_t launch_shadow(const double *pos, const double *mass,
                         const double *soft, int n, float *shadow,
                         hipStream_t s);

// First half-kick then drift, Eqs. 9-10:
//   v <- v + hdt (gA S + radA x - drag v);  x <- x + dt v
hipError_t launch_kick_drift(double *pos, double *vel, const double *S, int n,
                             double hdt, double gA, double radA, double drag,
                             double dt, hipStream_t s);
// Second half-kick with the drag at the end-of-step velocity:
//   v <- (v + hdt (gA S + radA x)) * inv,  inv = 1 / (1 + drag hdt)
hipError_t launch_kick_end(const double *pos, double *vel, const double *S,
                           int n, double hdt, double gA, double radA,
                           double inv, hipStream_t s);

// Sets *flag (device int, must start at 0) to 1 if any of the count doubles
// at p is NaN or Inf.
hipError_t launch_check_finite(const double *p, int64_t count, int *flag,
                               hipStream_t s);

}  // namespace steps
