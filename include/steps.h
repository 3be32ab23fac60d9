/*
 * steps.h -- C ABI of libsteps, an MI355X (gfx950) implementation of the
 * direct-summation hot path of StePS (Racz, Szapudi, Dobos, Csabai, Szalay
 * 2018, "StePS: A Multi-GPU Cosmological N-body Code for Compactified
 * Simulations"): the O(N^2) spline-softened pair sum over a compactified
 * spherical particle set with per-particle mass and softening, and the
 * comoving kick-drift-kick leapfrog that consumes it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: Mpc, Gyr, solar masses; velocities in Mpc/Gyr; H0 in km/s/Mpc.
 *
 * Pointers: every array argument is a DEVICE pointer on the context's
 * device (hipMalloc'd memory, or a torch tensor's data_ptr()).  Arrays are
 * structure-of-arrays, 8-byte (double) elements, contiguous:
 *   pos, vel, acc : [3][n]  (all x, then all y, then all z)
 *   mass, soft    : [n]
 * Output arrays must not overlap any input array.
 *
 * Ownership: the caller owns every array.  The library never frees a caller
 * pointer and keeps none of them past the call.  The context owns only its
 * scratch memory (partial sums, FP32 shadow copies), allocated on demand and
 * freed by steps_ctx_destroy.
 *
 * Asynchrony: compute calls enqueue work on the context's stream and return
 * without waiting.  Argument errors are reported by the return code before
 * anything is enqueued, and then nothing has been written.  Errors raised by
 * the device while the work runs surface at steps_sync (or at the next call
 * on that context).
 *
 * Return codes: STEPS_OK, or one of the negative STEPS_E_* values below.
 * steps_last_error() returns a message for the last failure on the calling
 * thread.  No C++ exception and no abort crosses this interface.
 *
 * The pair sum S returned by the force calls is G-free:
 *   S_i = sum_{j != i, r_ij > 0} m_j F(r_ij, h_i + h_j) (x_j - x_i) / r_ij
 * with F the spline-softened kernel of Sec. 2.2 Eq. 4 (support radius
 * h = h_i + h_j, Eqs. 2 and 8; F = 1/r^2 for r >= h).  The comoving pair
 * acceleration of Eq. 8 is G S_i / a^3; pass G*m as mass to get physical
 * units directly.  Pairs at zero separation contribute nothing.
 */
#ifndef STEPS_H
#define STEPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ----------------------------------------------------- */
#define STEPS_OK 0
#define STEPS_E_INVAL (-1)       /* bad argument (null pointer, n < 0, ...) */
#define STEPS_E_NOMEM (-2)       /* device scratch allocation failed (an
                                    automatically chosen symmetric shape
                                    first falls back to the one-sided
                                    kernel, which needs far less) */
#define STEPS_E_HIP (-3)         /* HIP runtime error; message has the text */
#define STEPS_E_NONFINITE (-4)   /* non-finite input (STEPS_CHECK_FINITE) */
#define STEPS_E_UNSUPPORTED (-5) /* option not supported by this mode/call */

/* ---- precision modes (steps_ctx_set_precision) ------------------------ */
/* FP64 throughout; deterministic (fixed summation order, no atomics). */
#define STEPS_FP64 0
/* Pair arithmetic in FP32 on an FP32 copy of the inputs; each j-tile's FP32
 * partial sum is added into an FP64 accumulator. */
#define STEPS_MIXED_F64ACC 1
/* As STEPS_MIXED_F64ACC, but tile partials are added into a Kahan-
 * compensated FP32 (sum, compensation) pair. */
#define STEPS_MIXED_KAHAN 2

/* ---- context flags (steps_ctx_set_flags) ------------------------------ */
/* Check pos/vel/mass/soft for NaN/Inf on every compute call (O(N), waits
 * for the device); a non-finite value gives STEPS_E_NONFINITE and nothing
 * else runs. */
#define STEPS_CHECK_FINITE 1u
/* Time every force-kernel launch with HIP events on the context stream;
 * read the totals with steps_ctx_force_timing. */
#define STEPS_PROFILE 2u

/* ---- cosmology modes -------------------------------------------------- */
/* Comoving spherical equations of motion, Sec. 2.2 Eq. 8. */
#define STEPS_COMOVING_SPHERICAL 0
/* Plain Newtonian test mode: a == 1, H == 0, no radial term, the step
 * variable is time itself (dt = da).  For integrator tests only. */
#define STEPS_NEWTONIAN_TEST 1
/* Comoving equations of motion in a periodic box, Sec. 2.2 Eq. 2: the pair
 * term and the Hubble drag, no radial term.  Needs a context made periodic
 * with steps_ctx_set_periodic (and the spherical mode needs one that is
 * not). */
#define STEPS_COMOVING_PERIODIC 2
/* steps_cosmology.flags: reversed gravity, G -> -G in both the pair term
 * and the mean-density (radial) term of Eq. 8, the Hubble drag unchanged.
 * Integrating with it relaxes a particle set into a glass, the way the
 * paper prepares its initial particle loads (Sec. 3): the particles repel
 * each other, the reversed radial term holds the sphere together, the drag
 * damps the motion.  Energies follow the reversed potential. */
#define STEPS_REVERSED_GRAVITY 1

/* Background cosmology (Sec. 2.2 Eq. 1). */
typedef struct steps_cosmology {
  double H0;      /* Hubble constant, km/s/Mpc (> 0 in comoving mode) */
  double omega_m; /* matter density parameter */
  double omega_l; /* dark-energy density parameter */
  double omega_r; /* radiation density parameter */
  double omega_k; /* curvature; NaN means 1 - omega_m - omega_l - omega_r */
  double G;       /* Newton's constant in Mpc^3/(Msun Gyr^2); 0 = built-in */
  int32_t mode;   /* STEPS_COMOVING_SPHERICAL, STEPS_NEWTONIAN_TEST or
                     STEPS_COMOVING_PERIODIC */
  int32_t flags;  /* 0 or STEPS_REVERSED_GRAVITY */
} steps_cosmology;

/* Launch shape of the force kernels.  r: i-particles held per lane;
 * tj: j-particles per LDS tile; jsplit: number of j-ranges the sum is split
 * into (partials reduced in fixed order; 0 in a forced shape = the built-in
 * choice for each n); variant: kernel option bits --
 *   1  STEPS_FP64 only: r^-3 from v_rsq_f64 with a first-order correction
 *      instead of a second-order one (one instruction less per pair, ~1e-15
 *      typical extra relative error);
 *   2  particles sorted along a space-filling curve inside the call, and the
 *      softening test skipped for (wave, tile) blocks whose boxes are
 *      farther apart than their largest combined softening;
 *   4  STEPS_FP64, with 2: well-separated blocks on the matrix cores
 *      (r = 1; tj 128 or 256);
 *   8  each pair between two different chunks of the sorted set evaluated
 *      once and applied to both particles (Newton's third law); jsplit is
 *      then the number of chunks.  STEPS_FP64: with 2 and 4 (r = 1,
 *      tj = 256).  Mixed modes: with 2 (r 2 or 4, tj = 256).
 * Compiled combinations: FP64 0, 1, 2, 3 (r 1, 2, 4, 8; tj 128), 6 (tj 128
 * and 256), 14 (tj 256); mixed modes 0 and 2, and 10 (r 2 and 4,
 * tj 256).  Defaults from N = 2^18 (while the chunk cap allows 64 chunks):
 * FP64 variant 14; mixed modes variant 10, r = 2 below 2^19 and r = 4
 * from there. */
typedef struct steps_tile {
  int32_t r;
  int32_t tj;
  int32_t jsplit;
  int32_t variant;
} steps_tile;

typedef struct steps_ctx steps_ctx;

/* ---- version and errors ----------------------------------------------- */
const char *steps_version(void);
/* Message for the last failing call on this thread ("" if none).  The
 * pointer stays valid until the next call on this thread. */
const char *steps_last_error(void);

/* ---- context ---------------------------------------------------------- */
/* Create a context on HIP device `device`: null stream, STEPS_FP64, no
 * flags, tile chosen by the built-in heuristic.  *out receives the handle. */
int steps_ctx_create(int device, steps_ctx **out);
/* Wait for the context's work, free its scratch and the handle.  NULL is a
 * no-op. */
int steps_ctx_destroy(steps_ctx *ctx);
/* Enqueue subsequent work on `stream` (a hipStream_t on the context's
 * device; NULL = the null stream).  The caller keeps the stream alive.
 * Switching to another stream first waits for the work already enqueued on
 * the old one, whose scratch the new stream's work may reuse. */
int steps_ctx_set_stream(steps_ctx *ctx, void *stream);
int steps_ctx_set_precision(steps_ctx *ctx, int precision);
int steps_ctx_set_flags(steps_ctx *ctx, uint32_t flags);
/* Force a launch shape (validated against the compiled variants; r and tj
 * must name one of them, 0 <= jsplit <= 1024).  Passing NULL returns to
 * automatic selection (tuned table, else heuristic). */
int steps_ctx_set_tile(steps_ctx *ctx, const steps_tile *tile);
/* Periodic box (Sec. 2.2, Eqs. 2 and 5).  With images != NONE every pair
 * sum on this context (steps_forces_ctx, steps_step_ctx, the adaptive step)
 * is taken in a box of side L:
 *   STEPS_IMAGES_ALL:     the softened force summed over every image x_j + n L
 *                         with |x_j + n L - x_i| < 2.6 L -- the formula of
 *                         Eq. 5 as printed, a direct image sum with no
 *                         Fourier-space part;
 *   STEPS_IMAGES_NEAREST: the leading term only, the nearest image (the
 *                         quasi-periodic option; ties at exactly L/2 go to
 *                         the even image);
 *   STEPS_IMAGES_NONE:    back to the open sphere (the default).
 * A particle's own images cancel in pairs and are left out.  Positions may
 * lie anywhere (the sums depend on them modulo L) and are not wrapped.
 * FP64 only (STEPS_E_UNSUPPORTED in the mixed modes); no potential, energy,
 * autotune or ensemble (STEPS_E_UNSUPPORTED).  The full image sum has
 * about 74 terms per pair (about 100 evaluated against the cut for
 * uniformly spread particles).  L finite and > 0. */
#define STEPS_IMAGES_NONE 0
#define STEPS_IMAGES_NEAREST 1
#define STEPS_IMAGES_ALL 2
int steps_ctx_set_periodic(steps_ctx *ctx, double L, int32_t images);
/* Record `tile` as the tuned shape for n particles in the context's current
 * precision, as steps_autotune would (validated like steps_ctx_set_tile;
 * replaces an earlier entry for the same precision and n).  For restoring a
 * shape found by an earlier steps_autotune, e.g. from a file cache. */
int steps_ctx_set_tuned(steps_ctx *ctx, int64_t n, const steps_tile *tile);
/* The shape the context would use for n particles in its precision. */
int steps_ctx_get_tile(steps_ctx *ctx, int64_t n, steps_tile *out);
/* Wait until all work enqueued on the context has finished; reports device
 * errors raised by that work. */
int steps_sync(steps_ctx *ctx);
/* With STEPS_PROFILE: total milliseconds and number of force-kernel
 * launches timed since the last reset (waits for the stream).  reset != 0
 * clears the totals after reading. */
int steps_ctx_force_timing(steps_ctx *ctx, double *total_ms, int64_t *count,
                           int reset);

/* ---- forces: Sec. 2.2 Eq. 8 (pair term) with Eqs. 3-4 ------------------ */
/* acc <- S (G-free pair sum, see top of file) for all n particles.
 * pos [3][n], mass [n], soft [n] (softening lengths h_i >= 0, the support
 * radius of particle i's share of the kernel), acc [3][n] output.
 * n == 0 is a no-op; n == 1 gives acc = 0.  n must be <= 2^30.
 * Scratch is sized before anything is enqueued: STEPS_E_NOMEM (after the
 * symmetric-to-one-sided fallback) leaves acc untouched. */
int steps_forces_ctx(steps_ctx *ctx, const double *pos, const double *mass,
                     const double *soft, int64_t n, double *acc);
/* Same on the default context of the calling thread's current device
 * (null stream, STEPS_FP64). */
int steps_forces(const double *pos, const double *mass, const double *soft,
                 int64_t n, double *acc);
/* Allocation-free steps_forces, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  FP64, same result as steps_forces up to summation
 * order (the one-sided kernels; <= 1e-12 relative to the exact sum), on the
 * device that holds pos, enqueued on `stream` (a hipStream_t; NULL = the
 * null stream) and not waited for.  Arguments as steps_forces, validated
 * before anything is enqueued; n above 262144 is STEPS_E_INVAL.  It calls no
 * allocating routine: its scratch (spatial sort, tile boxes, j-split
 * partial sums) is one fixed 64 MiB device array per GPU, held from the
 * library's load until the process ends.  Every call on a GPU shares that
 * array, so calls that overlap on one GPU (different streams not ordered by
 * the caller, or threads) race; calls ordered on one stream are safe.
 * Nothing in the array needs to start at zero: each call writes every word
 * it reads. */
int steps_forces_noalloc(const double *pos, const double *mass,
                         const double *soft, int64_t n, double *acc,
                         void *stream);

/* Autotuner: time the compiled force kernels of the context's precision on
 * these arrays -- i-particles per lane r in {1, 2, 4}, both the culled
 * (spatially sorted) and the plain variant, and three j-splits around the
 * heuristic's -- one force evaluation each, and keep the fastest for this n:
 * later calls with the same n and precision use it unless a tile is forced.
 * acc [3][n] is scratch output (holds S on return).  Synchronous.  *out
 * receives the chosen shape.  Shapes whose scratch does not fit are
 * skipped; STEPS_E_NOMEM only when none fits. */
int steps_autotune(steps_ctx *ctx, const double *pos, const double *mass,
                   const double *soft, int64_t n, double *acc,
                   steps_tile *out);

/* ---- softened potential (diagnostic) ---------------------------------- */
/* phi_i <- sum_{j != i, r_ij > 0} m_j phi(r_ij, h_i + h_j), G-free, with
 * phi the potential of the Eq. 4 kernel (phi = -1/r for r >= h,
 * d phi/dr = F).  Always FP64.  phi [n] output. */
int steps_potential_ctx(steps_ctx *ctx, const double *pos, const double *mass,
                        const double *soft, int64_t n, double *phi);
int steps_potential(const double *pos, const double *mass, const double *soft,
                    int64_t n, double *phi);

/* ---- comoving energies (diagnostic) ----------------------------------- */
/* The paper gives no energy diagnostic; this one follows from Eq. 8.  With
 * p = m a^2 dx/dt, Eq. 8 is dp/dt = -grad U_c / a for
 *   U_c = (G/2) sum_{i != j} m_i m_j phi(r_ij, h_i + h_j)
 *         - (Omega_m H0^2 / 4) sum_i m_i |x_i|^2,
 * so K = (1/2) sum m a^2 |v|^2 and W = U_c / a obey the cosmic energy
 * equation d(K + W)/dt = -H (2K + W) (Layzer-Irvine).
 * out[7] (HOST): K, W, the pair part of U_c, the radial part, and
 * sum m a^2 v (3 components).  vel [3][n] device.  FP64, O(N^2) (computes
 * the softened potential), waits for the result.  In STEPS_NEWTONIAN_TEST
 * mode a is taken as 1 and there is no radial part. */
int steps_energy_ctx(steps_ctx *ctx, const double *pos, const double *vel,
                     const double *mass, const double *soft, int64_t n,
                     double a, const steps_cosmology *cosmo, double *out);
int steps_energy(const double *pos, const double *vel, const double *mass,
                 const double *soft, int64_t n, double a,
                 const steps_cosmology *cosmo, double *out);
/* Kinetic part alone, O(N), no potential: out[4] (HOST) receives
 * K = (1/2) sum m a^2 |v|^2 and sum m a^2 v.  vel [3][n], mass [n] device.
 * Waits for the result.  With K at every step and the full energy at the
 * two ends, the cosmic energy equation in the form
 * d[a (K + W)]/da = -K can be checked without an O(N^2) potential per
 * step. */
int steps_kinetic_ctx(steps_ctx *ctx, const double *vel, const double *mass,
                      int64_t n, double a, double *out);
int steps_kinetic(const double *vel, const double *mass, int64_t n, double a,
                  double *out);

/* ---- one KDK step: Sec. 2.3 Eqs. 9-11 with the acceleration of Eq. 8 --- */
/* Advance pos, vel from scale factor a to a + da (in STEPS_NEWTONIAN_TEST
 * mode: from time a to a + da) with U = K(dt/2) D(dt) K(dt/2), where
 *   dt = integral_a^{a+da} da' / (a' H(a'))   (exact; Eq. 1)
 *   A  = G S / a^3 + (Omega_m H0^2 / 2) x / a^3 - 2 H(a) v     (Eq. 8)
 * The radial term uses the physical mean density Omega_m rho_crit / a^3.
 * The first half-kick evaluates A at (x_n, v_n, a_n); the second at
 * (x_{n+1}, v_{n+1}, a_{n+1}), solved in closed form since A is linear in v
 * (this keeps the step second order and time reversible).
 * On entry acc must hold S(pos) (call steps_forces once before the first
 * step); on exit pos, vel and acc = S(new pos) are updated.  Exactly one
 * O(N^2) evaluation per step, in the context's precision; kick and drift
 * are always FP64.  da may be negative if a + da > 0.
 * Errors (nothing written): STEPS_E_INVAL for null pointers, n < 0,
 * non-finite a or da, a <= 0 or a + da <= 0 in comoving mode, H0 <= 0,
 * G < 0, unknown flag bits, an unknown mode, or H(a)^2 <= 0 anywhere on
 * [a, a + da]; STEPS_E_NOMEM if the force scratch cannot be allocated
 * (checked before the first kick is enqueued). */
int steps_step_ctx(steps_ctx *ctx, double *pos, double *vel,
                   const double *mass, const double *soft, int64_t n,
                   double *acc, double a, double da,
                   const steps_cosmology *cosmo);
int steps_step(double *pos, double *vel, const double *mass,
               const double *soft, int64_t n, double *acc, double a,
               double da, const steps_cosmology *cosmo);

/* ---- adaptive step (Sec. 2.3, Eq. 12) --------------------------------- */
/* The global step of Eq. 12 at the current state: particle i proposes
 * sqrt(2 eta_i eps / |A_i|), eta_i = 2.8 h_i, with A_i the kick's
 * acceleration of Eq. 8 at the start of the step,
 *   A_i = G S_i / a^3 + (Omega_m H0^2 / 2) x_i / a^3 - 2 H(a) v_i
 * (G S_i in the Newtonian test mode; a particle with A_i = 0 proposes no
 * limit); *dt (HOST, Gyr) is the smallest proposal capped at dt_max, and
 * *da (HOST) the scale-factor step whose cosmic-time interval is *dt (= dt
 * in the Newtonian test mode).  pos, vel, acc [3][n] and soft [n] device;
 * acc must hold S(pos), as steps_step leaves it.  eps and dt_max finite and
 * > 0.  A particle with zero softening and a nonzero acceleration makes the
 * step zero: STEPS_E_INVAL.  Waits for the result (one device
 * min-reduction). */
int steps_adaptive_dt_ctx(steps_ctx *ctx, const double *pos, const double *vel,
                          const double *soft, const double *acc, int64_t n,
                          double a, const steps_cosmology *cosmo, double eps,
                          double dt_max, double *dt, double *da);
int steps_adaptive_dt(const double *pos, const double *vel, const double *soft,
                      const double *acc, int64_t n, double a,
                      const steps_cosmology *cosmo, double eps, double dt_max,
                      double *dt, double *da);
/* Integrate from a0 to a1 (>= a0) with the step of Eq. 12 chosen before
 * every KDK step, the last one shortened to end exactly at a1 (a is the time
 * in the Newtonian test mode).  acc is output: S(pos) is computed first and
 * S of the final positions is left in it.  At most max_steps steps;
 * *steps_taken and *a_reached (HOST, may be NULL) report how far it got.
 * Errors as steps_step and steps_adaptive_dt; on an error the state is that
 * after the last completed step. */
int steps_run_adaptive_ctx(steps_ctx *ctx, double *pos, double *vel,
                           const double *mass, const double *soft, int64_t n,
                           double *acc, double a0, double a1,
                           const steps_cosmology *cosmo, double eps,
                           double dt_max, int64_t max_steps,
                           int64_t *steps_taken, double *a_reached);

/* ---- ensembles of independent simulations ------------------------------ */
/* The paper motivates fast simulations for fitting cosmological parameters
 * (abstract); an ensemble runs many small, independent StePS simulations of
 * uneven size and cosmology together.  Pairs interact only within their
 * own member. */

/* Capture one step (kick+drift, pair sum, kick) as a hipGraph and replay
 * it; without the flag the same kernels are launched one by one (the two
 * give bitwise identical results). */
#define STEPS_BATCH_GRAPH 1u
/* Before stepping, time each compiled ensemble kernel on the first force
 * evaluation and keep the fastest (steps_batch_tile reports it).  The choice
 * is kept in the context for its precision and list of member sizes: a
 * later run with the same sizes uses it without timing again. */
#define STEPS_BATCH_AUTOTUNE 2u

typedef struct steps_batch {
  int32_t members;          /* B >= 1 */
  int32_t nsteps;           /* KDK steps per member, >= 1 */
  const int64_t *offsets;   /* HOST [B + 1]: offsets[0] = 0, nondecreasing;
                               member b owns columns [offsets[b],
                               offsets[b+1]) of the arena */
  double *pos;              /* device [3][N], N = offsets[B]; in/out */
  double *vel;              /* device [3][N]; in/out */
  const double *mass;       /* device [N] */
  const double *soft;       /* device [N] */
  double *acc;              /* device [3][N]; out: S(final pos) per member */
  const steps_cosmology *cosmo; /* HOST [B] */
  const double *a0;         /* HOST [B]: start scale factor (> 0) */
  const double *a1;         /* HOST [B]: end scale factor (> 0) */
  uint32_t flags;           /* STEPS_BATCH_GRAPH | STEPS_BATCH_AUTOTUNE */
  int32_t resort_every;     /* refresh the internal spatial order every k
                               steps; 0 = order once at the start */
} steps_batch;

/* Run every member nsteps KDK steps (as steps_step) on the log-uniform grid
 * a_k = a0 (a1/a0)^(k/nsteps), k = 0..nsteps, in the context's precision.
 * The forces of the initial positions are computed first (acc is output
 * only).  Internally the ensemble is held in one arena in spatial (Morton)
 * order within each member; one persistent kernel launch per step sums all
 * members, its blocks pulling (member, i-block) items longest first from an
 * atomic counter.  Synchronous: returns when the run is complete.
 * member_status (HOST [B], may be NULL) receives per member STEPS_OK or the
 * reason it was skipped (bad cosmology, a0/a1, or H^2 <= 0 on its grid);
 * skipped members' columns are left untouched and do not stop the others.
 * Errors for the whole call: null or invalid pointers, B < 1, nsteps < 1,
 * non-monotone offsets, N > 2^30, overlapping arrays, unknown flags. */
int steps_batch_run(steps_ctx *ctx, const steps_batch *batch,
                    int32_t *member_status);
/* The ensemble kernel is the context's forced tile (steps_ctx_set_tile;
 * its r, tj and variant must name an ensemble kernel of the precision, else
 * STEPS_E_INVAL, and STEPS_BATCH_AUTOTUNE then has no choice to make), or
 * the fastest one under STEPS_BATCH_AUTOTUNE, or a default.
 * Launch shape of the last steps_batch_run on this context (r, tj and
 * variant of its kernel; jsplit = the largest number of parts a member's
 * j-range was cut into, 1 when every work item covers its member's whole
 * j-range): */
int steps_batch_tile(steps_ctx *ctx, steps_tile *out);

/* ---- background helpers (host only, no device work) ------------------- */
/* H(a) in 1/Gyr (Eq. 1). */
int steps_hubble(const steps_cosmology *cosmo, double a, double *out);
/* dt (Gyr) for the scale factor to go from a to a + da. */
int steps_dt(const steps_cosmology *cosmo, double a, double da, double *out);
/* Built-in G in Mpc^3/(Msun Gyr^2) and km/s in Mpc/Gyr. */
double steps_G(void);
double steps_kms_to_mpc_per_gyr(void);

#ifdef __cplusplus
}
#endif

#endif /* STEPS_H */
