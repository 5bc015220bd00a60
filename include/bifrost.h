/*
 * bifrost.h -- C ABI of the MI355X (gfx950) direct-summation pass of the
 * hierarchical fourth-order forward symplectic integrator HHS-FSI
 * (Rantala et al. 2022, BIFROST, arXiv 2210.02472).
 *
 * Library: libbifrost_hip.so (hand-written HIP kernels for gfx950).
 *
 * General conventions (apply to every entry point unless stated otherwise):
 *  - Every array argument is a DEVICE pointer owned by the caller; the library
 *    only owns context-internal scratch (grown on demand, reused afterwards).
 *  - Calls are stream-ordered and asynchronous on the context's stream unless
 *    marked "synchronising".  Inputs must stay valid until the work completes.
 *  - Particle data is structure-of-arrays FP64, particle-indexed, length n.
 *  - Per-particle outputs are particle-indexed (length n); only entries whose
 *    particle is listed in `targets` are written, all others are left untouched.
 *  - Outputs must not alias inputs (bf_fsi_step's in/out state excepted).
 *  - A source equal to the target (same particle index) is skipped.
 *  - Index lists hold int32 particle indices (n < 2^31).  Kernels clamp an
 *    out-of-range list entry to particle 0 (so they never read out of bounds)
 *    and raise BF_FLAG_BADINDEX; bf_validate_set checks a list synchronously.
 *  - Errors are return codes (bf_status); nothing is thrown across the ABI.
 *    Argument checks happen before any launch.  Conditions found on the device
 *    raise bits in a per-context flag word read by bf_read_flags.
 *  - One context per host thread.
 *  - Separations: r_ji = x_j - x_i, s^2 = |r_ji|^2 + eps2 (Plummer softening;
 *    eps2 = 0 is the paper's unsoftened form).
 */
#ifndef BIFROST_H
#define BIFROST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BF_API __attribute__((visibility("default")))

typedef enum {
    BF_OK = 0,
    BF_ERR_ARG = -1,         /* invalid argument (NULL pointer, bad size, bad range, bad enum) */
    BF_ERR_HIP = -2,         /* a HIP runtime call failed (message in bf_last_error) */
    BF_ERR_NONFINITE = -3,   /* reserved for callers that turn BF_FLAG_NONFINITE into an error */
    BF_ERR_UNSUPPORTED = -4, /* no kernel variant for this request */
    BF_ERR_NOMEM = -5        /* scratch allocation failed, or a caller buffer is too small */
} bf_status;

typedef enum {
    BF_PREC_FP64 = 0,  /* all pair arithmetic in FP64 */
    BF_PREC_MIXED = 1  /* FP32 pair arithmetic, per-tile FP32 partial sums merged into FP64
                          accumulators, FP64 re-evaluation of every tile that holds a pair
                          closer than r_fb (see bf_forces) */
} bf_prec;

/* device flag bits (bf_read_flags) */
#define BF_FLAG_NONFINITE  0x1u  /* an output was NaN or infinite */
#define BF_FLAG_COINCIDENT 0x2u  /* two distinct particles at zero separation with eps2 == 0 */
#define BF_FLAG_BADINDEX   0x4u  /* an index list held an entry outside [0, n) */

/* Read-only FP64 particle arrays (x, y, z, vx, vy, vz, m), each of length n.
 * Entry points that do not need velocities accept vx = vy = vz = NULL. */
typedef struct bf_particles {
    const double *x, *y, *z, *vx, *vy, *vz, *m;
    int64_t n;
} bf_particles;

/* Mutable FP64 state for bf_fsi_step (positions and velocities updated in place). */
typedef struct bf_state {
    double *x, *y, *z, *vx, *vy, *vz;
    const double *m;
    int64_t n;
} bf_state;

/* A particle set: if idx != NULL it is the device list idx[0..count) of particle
 * indices; otherwise it is the contiguous range [begin, begin + count).  Sets used
 * as sources of a sum must not repeat a particle. */
typedef struct bf_set {
    const int32_t *idx;
    int32_t count;
    int32_t begin;
} bf_set;

typedef struct bf_ctx bf_ctx;

/* ---- context ------------------------------------------------------------------------ */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  Ownership of *ctx passes to the
 * caller (free with bf_destroy).  BF_ERR_ARG if ctx is NULL or device is invalid. */
BF_API int bf_create(bf_ctx **ctx, int device, void *hip_stream);
/* Destroy a context (synchronising) and free its scratch.  NULL is accepted. */
BF_API int bf_destroy(bf_ctx *ctx);
/* Synchronising.  Free the context's scratch buffers (they grow to the largest pass run; the
 * pair-symmetric sweep's partials take 8.6 GB at n = 2^20) and report the bytes freed in
 * *freed (may be NULL).  Later calls allocate again as needed.  Captured graphs keep their own
 * buffers. */
BF_API int bf_release_scratch(bf_ctx *ctx, size_t *freed);
/* Rebind the context to another stream of the same device. */
BF_API int bf_set_stream(bf_ctx *ctx, void *hip_stream);
/* Static string for a bf_status value. */
BF_API const char *bf_status_string(int status);
/* Thread-local text of the last error raised by a bf_* call on this thread ("" if none). */
BF_API const char *bf_last_error(void);
/* Synchronising: wait for the context's stream, return the device flag word in *flags,
 * and clear it if `clear` != 0. */
BF_API int bf_read_flags(bf_ctx *ctx, uint32_t *flags, int clear);
/* Synchronising: check that every entry of a list set lies in [0, n).  Returns BF_OK or
 * BF_ERR_ARG.  Range sets are checked on the host. */
BF_API int bf_validate_set(bf_ctx *ctx, const bf_set *set, int64_t n);
/* Library version string. */
BF_API const char *bf_version(void);

/* ---- the direct-summation pass ------------------------------------------------------ */

/* Newtonian accelerations (Sec. 2.1, Eq. new-newton-acc; inter-level sums of Sec. 2.2):
 *     a_i = sum_{j in sources, j != i} G m_j r_ji / s^3        for i in targets.
 * Writes ax/ay/az[i] (FP64, particle-indexed) for every target i.
 * prec = BF_PREC_MIXED: every LDS tile of sources is first summed in FP32; a tile in which
 * some pair has s^2 < r_fb^2 (FP32 estimate) is re-evaluated for that wavefront entirely in
 * FP64 from the FP64 masters (this also removes the self pair).  r_fb >= 0 is a length
 * (ignored for BF_PREC_FP64).  Distinct particles at zero separation with eps2 == 0
 * contribute nothing (mixed: BF_FLAG_COINCIDENT is raised).
 * Errors: BF_ERR_ARG for NULL pointers, n <= 0, negative eps2 or r_fb, bad prec, a range
 * outside [0, n), count < 0.  count == 0 for targets or sources is a no-op (targets: nothing
 * written; sources: zeros written). */
BF_API int bf_forces(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                     double G, double eps2, int prec, double r_fb,
                     double *ax, double *ay, double *az);

/* The accelerations of bf_forces (same arguments, same meaning, same results to the mixed or
 * FP64 tolerance), for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine): the pass takes the unsorted directed
 * sweep (no spatial sort, no pair-symmetric sweep) and carves its packed sources, source-chunk
 * partials, fix-up queue and fix-up partials from a static device array of 64 MiB that each
 * device holds until the process ends; it lowers the source split until the partials fit, and
 * records no timing events.  Limit: 256 + 4 n_t (rounded up to 256) + pack + fix-up bytes must
 * fit in 64 MiB, where pack = 32 n_s bytes (rounded up to 256) and fix-up = 3 MiB in mixed
 * precision (0 in FP64): n_t + 8 n_s up to about 15.9 million in mixed precision and 16.7
 * million in FP64.  Larger sets return
 * BF_ERR_ARG before any launch; other errors as bf_forces, and BF_ERR_HIP if the array's device
 * address could not be resolved when the context was created.  Every call on one device uses
 * the same array, which keeps the last call's contents (each pass clears what must start at
 * zero): calls that overlap on one device, from several streams or contexts, race. */
BF_API int bf_forces_noalloc(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                             double G, double eps2, int prec, double r_fb, double *ax, double *ay, double *az);

/* Force-gradient sum (Sec. 2.1, Eq. new-grad-acc; inter-level form Sec. 2.2):
 *     Gsum_i = sum_{j in sources, j != i} G m_j / s^5 (s^2 a_ji - 3 (a_ji . r_ji) r_ji),
 *     a_ji = a_j - a_i,
 * with a given by ax/ay/az (FP64, particle-indexed, the accelerations of the same
 * potential term that is being kicked).  The gradient acceleration of a kick of length
 * eps is a + eps^2/24 Gsum, and g' of the gradient time-step criteria is Gsum/24.
 * Writes gx/gy/gz[i] for every target i.  prec and r_fb as in bf_forces. */
BF_API int bf_force_gradient(bf_ctx *ctx, const bf_particles *P, const bf_set *targets,
                             const bf_set *sources, const double *ax, const double *ay,
                             const double *az, double G, double eps2, int prec, double r_fb,
                             double *gx, double *gy, double *gz);

/* Both inter-set sums at once (Sec. 2.2: the inter-level terms of the hierarchy, S <- F and
 * F <- S, are the same pairs seen from either side).  For every particle i of set a it writes
 * ax/ay/az[i] = the acceleration of i due to the particles of b, and for every particle j of b
 * the acceleration of j due to a; entries outside a and b are not written.  a and b must be
 * disjoint: overlapping ranges and a shared index array fail with BF_ERR_ARG; for other index
 * lists disjointness is the caller's promise (a particle in both gets one of its two sums).
 * Mixed precision with r_fb = 0 and both sets large enough for the spatially sorted mode
 * (bf_set_spatial_sort; here from 2^29 pairs, since the sweep replaces two passes) evaluates
 * every pair once (two-set symmetric sweep, scratch
 * (n_a / 1024 + 1) * 16 bytes per particle of b plus O(n_a)); otherwise it runs as the two
 * passes bf_forces(a <- b) and bf_forces(b <- a).  Results, errors and flags as bf_forces. */
BF_API int bf_forces_between(bf_ctx *ctx, const bf_particles *P, const bf_set *a, const bf_set *b, double G,
                             double eps2, int prec, double r_fb, double *ax, double *ay, double *az);
/* The force-gradient sums between two disjoint sets, as bf_forces_between: a's particles get
 * Gsum over b, b's over a, with a_ji from the given accelerations (particle-indexed). */
BF_API int bf_force_gradient_between(bf_ctx *ctx, const bf_particles *P, const bf_set *a, const bf_set *b,
                                     const double *ax, const double *ay, const double *az, double G, double eps2,
                                     int prec, double r_fb, double *gx, double *gy, double *gz);

/* Pairwise time-steps (Sec. 3.5.3, Eqs. dt-freefall and dt-flyby), unsoftened:
 *     dt_ff,i = eta_ff min_j (|r_ij|^3 / (G (m_i + m_j)))^(1/2)
 *     dt_fb,i = eta_fb min_j |r_ij| / |v_ij|
 * over sources j != i.  A pair with v_ij = 0 gives no fly-by bound; a target without a
 * valid source gets +inf.  Needs velocities.  prec as in bf_forces (the mixed path takes
 * the maxima of G(m_i+m_j)/r^3 and |v_ij|^2/r^2 in FP32 and finishes in FP64; tiles with a
 * pair closer than max(r_fb, tiny) or a rate beyond the FP32 range are re-evaluated in FP64).
 * Writes dt_ff[i], dt_fb[i] for every target i. */
BF_API int bf_dt_min(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                     double G, double eta_ff, double eta_fb, int prec, double r_fb,
                     double *dt_ff, double *dt_fb);

/* Global PN1.0 acceleration (Sec. 3.8, Eqs. subsyspn and subsyspn-mass), FP64: the pairwise
 * first post-Newtonian acceleration summed over sources j != i for which i or j is in
 * bh_idx[0..n_bh) (device list of distinct particle indices).  The two-body term (not
 * printed in the paper) is the harmonic-gauge form; with n = (x_i - x_j)/r, v_ij = v_i - v_j:
 *   a_i += G m_j/(c^2 r^2) {[G(5 m_i + 4 m_j)/r + 3/2 (n.v_j)^2 - v_i^2 + 4 v_i.v_j - 2 v_j^2] n
 *                           + [4 n.v_i - 3 n.v_j] v_ij}.
 * Writes apx/apy/apz[i] for every target i (zero for targets with no such pair).
 * BF_ERR_ARG for c <= 0, n_bh < 0, n_bh > 0 with bh_idx NULL. */
BF_API int bf_pn1_bh(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                     const int32_t *bh_idx, int32_t n_bh, double G, double c,
                     double *apx, double *apy, double *apz);

/* Synchronising.  Kinetic and potential energy of a set (Sec. 2.1, the N-body
 * Hamiltonian) in FP64: T = sum 1/2 m v^2, U = -sum_{i<j} G m_i m_j / s_ij, written to the
 * host scalars *kinetic and *potential.  Each unordered pair is evaluated once (1/s from the
 * hardware reciprocal square root refined to about 2^-69); sums of 64 terms are folded into
 * compensated (Neumaier) sums in a fixed order, so the result is deterministic for a given set
 * and device.  A coincident pair at eps2 = 0 adds nothing.  At most 2^24 particles
 * (BF_ERR_UNSUPPORTED beyond). */
BF_API int bf_energy(bf_ctx *ctx, const bf_particles *P, const bf_set *set, double G, double eps2,
                     double *kinetic, double *potential);

/* ---- integrator step ---------------------------------------------------------------- */

typedef struct bf_fsi_params {
    double G, eps2;
    int prec;          /* bf_prec for the force and gradient passes */
    double r_fb;       /* close-pair radius of the mixed path */
    const int32_t *bh_idx; int32_t n_bh; double c;  /* n_bh == 0: no PN1.0 half-kicks */
} bf_fsi_params;

#define BF_A_VALID 0x1  /* ax/ay/az already hold the accelerations of the current state */

/* One FSI cycle of length dt (Sec. 2.1, Eq. fsi-cycle) over the particles of `set`, which
 * act as both targets and sources (the sub-Hamiltonian of that set):
 *   v += dt/6 a; x += dt/2 v; v += 2dt/3 (a + dt^2/24 Gsum); x += dt/2 v; v += dt/6 a,
 * each a evaluated at the current positions.  With n_bh > 0 the cycle is wrapped in two PN1.0
 * half-kicks v += dt/2 a_PN (Sec. 3.8, composition e^{eps/2 U_PN} e^{eps H_FSI} e^{eps/2 U_PN}).
 * ax/ay/az (particle-indexed, caller-owned) hold the accelerations of the final state on
 * return; with flags & BF_A_VALID their input values are reused for the first kick.
 * All updates are FP64.  Errors as in bf_forces. */
BF_API int bf_fsi_step(bf_ctx *ctx, const bf_state *S, const bf_set *set, double dt,
                       const bf_fsi_params *prm, double *ax, double *ay, double *az, int flags);

/* ---- time-step assignment and the HHS-FSI interval ----------------------------------- */

/* Jerk (Sec. 3.5.5): j_i = sum_{j != i} G m_j / s^5 (s^2 v_ji - 3 (r_ji . v_ji) r_ji),
 * v_ji = v_j - v_i; the same tidal contraction as bf_force_gradient with velocities in place of
 * accelerations.  Writes jx/jy/jz[i] for every target i.  prec as in bf_forces. */
BF_API int bf_jerk(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                   double G, double eps2, int prec, double *jx, double *jy, double *jz);

/* Per-particle time-step of the set: the minimum of
 *   dt_ff, dt_fb                                  (bf_dt_min, Sec. 3.5.3),
 *   eta_grad (|v| / |g'|)^(1/3), eta_grad (|a| / |g'|)^(1/2), g' = Gsum / 24
 *                                                 (Sec. 3.5.4, Eqs. dt-nabla1, dt-nabla2),
 *   eta_jerk |a| / |j|                            (Sec. 3.5.5),
 * where a criterion is skipped if its arrays are NULL (gx/gy/gz or jx/jy/jz), its eta <= 0 or its
 * denominator is zero.  With level != NULL also writes the time-step level: the smallest k in
 * [0, kmax] with dt >= tau / 2^k (slow on level k, Sec. 2.2), kmax if none.  All arrays are
 * particle-indexed; only entries of the set are written. */
BF_API int bf_timestep_assign(bf_ctx *ctx, const bf_particles *P, const bf_set *set,
                              const double *dt_ff, const double *dt_fb,
                              const double *ax, const double *ay, const double *az,
                              const double *gx, const double *gy, const double *gz,
                              const double *jx, const double *jy, const double *jz,
                              double eta_grad, double eta_jerk, double tau, int kmax,
                              double *dt, int32_t *level);

/* Synchronising.  Stable partition of the particles of `set` by level (level: device int32,
 * particle-indexed, values in [0, kmax]): order[0 .. set.count) receives the particle indices
 * sorted by level (ties keep the set's order), counts[0 .. kmax] (host) the number per level.
 * The fast set "level > k" is then the contiguous suffix of order after level k. */
BF_API int bf_level_partition(bf_ctx *ctx, const bf_set *set, int64_t n, const int32_t *level, int kmax,
                              int32_t *order, int64_t *counts);

/* One HHS-FSI interval of length tau over `set` (Sec. 2.2, Eq. hhsfsi-cycle) with fixed
 * per-particle levels (device int32, particle-indexed, in [0, kmax]).  On level k the slow set
 * S holds the particles at level k and the fast set F those deeper:
 *   kick tau/6 with the inter-level accelerations (S <- F, F <- S); FSI(S, tau/2);
 *   HHS(F, tau/2); gradient kick 2 tau/3 with the inter-level accelerations and gradient sums;
 *   HHS(F, tau/2); FSI(S, tau/2); kick tau/6.
 * An empty F ends the recursion with one FSI cycle of S over tau; an empty S gives two half
 * intervals of F.  Positions and velocities of S are updated in place (FP64).  The partition
 * synchronises once; everything else is stream-ordered.  With prm->n_bh > 0 (PN1.0, Sec. 3.8,
 * FP64) every FSI cycle is wrapped in PN half-kicks over its own pairs (as bf_fsi_step) and
 * every level's cycle in PN half-kicks of tau/2 over its inter-level pairs with a listed
 * particle; the paper does not place the PN terms in the hierarchy, this is a reading.
 * Between two visits of a level no particle of that level or deeper moves, so the driver keeps
 * the level's own accelerations after each FSI cycle and its inter-level accelerations after
 * each visit, and the next visit starts from them instead of recomputing them (the result is
 * the same bit for bit; the context holds 3n doubles per level that has both S and F). */
BF_API int bf_hhs_interval(bf_ctx *ctx, const bf_state *S, const bf_set *set, const int32_t *level,
                           int kmax, double tau, const bf_fsi_params *prm);

/* Capture one fixed-level HHS-FSI interval (the recursion of bf_hhs_interval, Sec. 2.2) into a
 * HIP graph: *graph_exec receives a handle for bf_graph_launch / bf_graph_destroy.  Each launch
 * advances the state in S by one interval with the level structure given here (the partition
 * is taken once, at capture; recapture when levels change).  Synchronising; the graph owns its
 * scratch buffers, so later calls on the context never invalidate it.  The passes inside the
 * graph are the eager ones, the spatially sorted mode included; there its Morton order comes
 * from a merge sort, which launches kernels only (the eager radix sort clears its counters with
 * memset operations, which a graph must not hold): both sorts are stable, so a replay equals an
 * eager bf_hhs_interval bit for bit.  With prm->n_bh > 0 the graph holds the PN1.0 half-kicks
 * at the same places as the eager interval (their kernels take the black-hole list captured
 * here).  Kernel timing is off while capturing.  Errors as bf_hhs_interval; an empty set is
 * BF_ERR_ARG. */
BF_API int bf_graph_capture_hhs_interval(bf_ctx *ctx, const bf_state *S, const bf_set *set, const int32_t *level,
                                         int kmax, double tau, const bf_fsi_params *prm, void **graph_exec);

/* One HHS-FSI interval of length tau over `set` with time-steps assigned on every hierarchy
 * level (Sec. 2.2: each level starts by assigning time-steps and splitting its particles at the
 * pivot; Sec. 3.5.1: a time-step cannot grow within the interval).  dt0 (device FP64,
 * particle-indexed) holds the time-steps assigned at the start of the interval from all
 * particles (e.g. bf_timestep_assign); it splits level 0.  On a deeper level k with particle set
 * P and pivot tau / 2^k, every criterion is evaluated again over P alone: the pairwise free-fall
 * and fly-by time-steps (Sec. 3.5.3; eta_ff, eta_fb > 0; unsoftened), both gradient criteria
 * (Sec. 3.5.4, Eqs. dt-nabla1, dt-nabla2; eta_grad, with the acceleration and the gradient sum
 * over P) and the jerk criterion (Sec. 3.5.5; eta_jerk, the jerk over P), as bf_timestep_assign
 * combines them; eta_grad = 0 or eta_jerk = 0 leaves that criterion out.  A particle's time-step
 * is the minimum of these and dt0; particles with time-step >= pivot are slow, the others fast;
 * on level kmax all are slow.  The passes run in precision prm->prec, softened with prm->eps2
 * except the pairwise criteria.  The cycle on each level is the one of bf_hhs_interval.
 * Synchronises once per visited level (the split sizes); max_level / n_levels (host, may be NULL)
 * receive the deepest level reached and the number of levels visited.  PN1.0 as in
 * bf_hhs_interval.  A visit whose slow set (and fast set) equals the previous visit's of the same
 * level starts from that visit's own (and inter-level) accelerations, as bf_hhs_interval does,
 * unless a shallower level changed its split or ran with an empty fast set since (then its
 * particles may have drifted); the context holds 3n doubles per level for that.  Errors:
 * BF_ERR_ARG for a NULL dt0, kmax outside [0, 63], tau not finite and > 0, eta_ff or eta_fb not
 * finite and > 0, eta_grad or eta_jerk negative or not finite; otherwise as bf_hhs_interval. */
BF_API int bf_hhs_interval_adaptive(bf_ctx *ctx, const bf_state *S, const bf_set *set, const double *dt0,
                                    int kmax, double tau, double eta_ff, double eta_fb, double eta_grad,
                                    double eta_jerk, const bf_fsi_params *prm, int *max_level,
                                    int64_t *n_levels);

/* Whether the HHS drivers (bf_hhs_interval, bf_hhs_interval_adaptive, captured intervals) keep a
 * level's own and inter-level accelerations between its visits (on = 1, the default) or
 * recompute every one of them (on = 0).  Kernels are deterministic, so both give the same
 * result bit for bit; the switch exists to check exactly that.  Errors: BF_ERR_ARG for a NULL
 * context. */
BF_API int bf_set_hhs_reuse(bf_ctx *ctx, int on);

/* Elementwise kicks and drifts used by integrator drivers (FP64, over the set):
 *   bf_kick:  v_i += h (a_i + h2 g_i)   (g may be NULL, then h2 is ignored)
 *   bf_drift: x_i += h v_i                                              (Sec. 2.1) */
BF_API int bf_kick(bf_ctx *ctx, const bf_state *S, const bf_set *set, double h, const double *ax,
                   const double *ay, const double *az, double h2, const double *gx, const double *gy,
                   const double *gz);
BF_API int bf_drift(bf_ctx *ctx, const bf_state *S, const bf_set *set, double h);

/* ---- batched ensembles -------------------------------------------------------------- */

/* Accelerations for an ensemble of independent clusters stored back to back in P
 * (cluster c owns particles [cluster_off[c], cluster_off[c+1])), each summing only over its
 * own cluster, for the active particles active_idx[active_off[c] .. active_off[c+1]) of each
 * cluster (global particle indices inside the cluster's range).  cluster_off and active_off
 * are DEVICE arrays of n_clusters + 1 int64 entries; their contents may change between calls
 * (and between replays of a captured graph) as long as max_active_total and max_cluster_n
 * bound them.  One persistent launch covers all clusters (Sec. 2.2's uneven level sizes).
 * Results as bf_forces for each cluster. */
BF_API int bf_forces_batched(bf_ctx *ctx, const bf_particles *P, int32_t n_clusters,
                             const int64_t *cluster_off, const int32_t *active_idx,
                             const int64_t *active_off, int64_t max_active_total, int64_t max_cluster_n,
                             double G, double eps2, int prec, double r_fb,
                             double *ax, double *ay, double *az);

/* Force-gradient sums for the same ensemble layout (Gsum of the active particles of every
 * cluster from all particles of that cluster; ax/ay/az particle-indexed as in
 * bf_force_gradient). */
BF_API int bf_force_gradient_batched(bf_ctx *ctx, const bf_particles *P, int32_t n_clusters,
                                     const int64_t *cluster_off, const int32_t *active_idx,
                                     const int64_t *active_off, int64_t max_active_total,
                                     int64_t max_cluster_n, const double *ax, const double *ay,
                                     const double *az, double G, double eps2, int prec, double r_fb,
                                     double *gx, double *gy, double *gz);

/* One FSI cycle of length dt (Sec. 2.1, Eq. fsi-cycle) of the active particles of every cluster,
 * with every particle of the cluster as a source (inactive particles stay frozen): kick dt/6,
 * drift dt/2, batched forces, batched gradient, kick 2dt/3 with a + dt^2/24 Gsum, drift dt/2,
 * batched forces, kick dt/6.  ax/ay/az must hold the accelerations of the current state of the
 * active particles on entry and hold those of the new state on return.  Stream-ordered. */
BF_API int bf_fsi_step_batched(bf_ctx *ctx, const bf_state *S, int32_t n_clusters,
                               const int64_t *cluster_off, const int32_t *active_idx,
                               const int64_t *active_off, int64_t max_active_total,
                               int64_t max_cluster_n, double G, double eps2, int prec, double r_fb,
                               double dt, double *ax, double *ay, double *az);

/* Capture into a HIP graph the same FSI cycle as bf_fsi_step_batched.  ax/ay/az must hold the
 * accelerations of the current state when the graph is launched and hold those of the new state
 * afterwards.  Scratch is sized here for the given bounds; replays read the device arrays'
 * current contents (offsets, lists) and allocate nothing.  *graph_exec receives an opaque handle
 * (free with bf_graph_destroy). */
BF_API int bf_graph_capture_batched_fsi(bf_ctx *ctx, const bf_state *S, int32_t n_clusters,
                                        const int64_t *cluster_off, const int32_t *active_idx,
                                        const int64_t *active_off, int64_t max_active_total,
                                        int64_t max_cluster_n, double G, double eps2, int prec,
                                        double r_fb, double dt, double *ax, double *ay, double *az,
                                        void **graph_exec);
/* Launch a captured graph on the context's stream. */
BF_API int bf_graph_launch(bf_ctx *ctx, void *graph_exec);
/* Free a captured graph (NULL accepted). */
BF_API int bf_graph_destroy(void *graph_exec);

/* ---- subsystems (Sec. 3.3) ------------------------------------------------------------ */

/* Synchronising.  Neighbour pairs of the subsystem search (Sec. 3.3, Eqs. ngb-bound and
 * ngb-unbound), FP64.  For every target i and source j != i closer than r_max, with
 * mu = G (m_i + m_j), relative separation r, relative velocity v, E = v^2/2 - mu/r and
 * h = |r x v|: a bound pair (E < 0, a = -mu / (2E)) is a neighbour if a < r_ngb or r < r_ngb;
 * an unbound pair if r < r_ngb, or if its periapsis h^2 / (mu (1 + e)),
 * e = sqrt(1 + 2 E h^2 / mu^2), lies below r_ngb and C r / |v| < tau (tau: the pivot time-step
 * of the level, C < 1 a safety factor).  edges (device int32, 2 * cap entries, caller-owned)
 * receives the pairs as rows (i, j), sorted by i then j; *n_edges (host) the number found.
 * With targets = sources every pair appears in both orders.  If more than cap pairs are found,
 * returns BF_ERR_NOMEM with *n_edges set to the number needed (edges then undefined).
 * Distinct particles at zero separation are skipped and raise BF_FLAG_COINCIDENT. */
BF_API int bf_neighbours(bf_ctx *ctx, const bf_particles *P, const bf_set *targets, const bf_set *sources,
                         double G, double r_ngb, double r_max, double C, double tau,
                         int32_t *edges, int64_t cap, int64_t *n_edges);

/* Synchronising.  Subsystems as the connected components of a neighbour graph (Sec. 3.3):
 * label (device int32, n entries, caller-owned) receives for every particle the smallest
 * particle index of its component, so a particle without neighbours carries its own index.
 * edges: device int32 rows (i, j), m rows, indices in [0, n) (others raise BF_FLAG_BADINDEX
 * and are ignored).  *n_subsystems (host, may be NULL): components with two or more members. */
BF_API int bf_subsystems(bf_ctx *ctx, int64_t n, const int32_t *edges, int64_t m, int32_t *label,
                         int64_t *n_subsystems);

/* Exclude intra-subsystem pairs (Sec. 3.3, Alg. 1: accelerations ignore intra-subsystem
 * contributions; time-steps of subsystem members ignore their own subsystem).  label: device
 * int32, particle-indexed (n entries), e.g. from bf_subsystems; a pair (i, j) is skipped in the
 * acceleration, force-gradient and time-step passes (and everything built on them: jerk, FSI,
 * HHS) when label[i] == label[j].  The array is read by later calls and must stay valid until
 * cleared with label = NULL.  Passes on a particle set of another size fail with BF_ERR_ARG;
 * the batched ensemble calls fail with BF_ERR_UNSUPPORTED while labels are set.  bf_pn1_bh and
 * bf_energy do not apply the exclusion.  The subsystems' own integration is outside this
 * library. */
BF_API int bf_set_subsystems(bf_ctx *ctx, const int32_t *label, int64_t n);

/* ---- tuning ------------------------------------------------------------------------- */

typedef enum { BF_OP_FORCES = 0, BF_OP_GRADIENT = 1, BF_OP_DTMIN = 2 } bf_op;
#define BF_SORT_ANY_SIZE 0x100  /* bf_set_spatial_sort: sort passes of any size */
#define BF_SORT_DIRECTED 0x200  /* bf_set_spatial_sort: no pair-symmetric sweep */

/* The tuning table maps (op, prec, sweep kind, log2 bucket of the two sizes) to a launch shape;
 * passes look it up for their own sizes (a forced shape, bf_set_config and the two setters
 * below, wins).  Sweep kinds: directed passes (targets per lane, waves per workgroup, source
 * split), pair-symmetric sweeps (row tiles per wavefront, waves, rounds of resident workgroups
 * that the distance shares aim at) and batched ensembles (targets per lane, waves, sources per
 * work item; buckets of max_active_total and max_cluster_n).  The shapes are the launch
 * parameters of the O(N_active x N) pass (Sec. 2.2's uneven level sizes decide which is
 * fastest); results do not depend on them beyond the FP32 summation order.
 *
 * Synchronising; allocates its own temporaries.  Directed passes on n_targets x n_sources
 * synthetic pairs (uniform cube): every targets-per-lane x waves variant, each with the
 * automatic source split and 1/4, 1/2 and 2 times it; large target sets are timed on a leading
 * sample of 131,072 targets.  The fastest is stored for that size bucket.  If cache_path is not
 * NULL the table is merged into that JSON file (read first if it exists). */
BF_API int bf_autotune(bf_ctx *ctx, int op, int prec, int64_t n_targets, int64_t n_sources,
                       const char *cache_path);
/* Synchronising; allocates its own temporaries.  Tune the pass `op` that the caller is about to
 * run, on the caller's own particles and sets (the near / far tile mix of a clustered set is
 * what decides the spatially sorted kernels' speed).  If the pass takes the pair-symmetric
 * sweep (mixed, spatially sorted, targets and sources one set), the shapes (16 waves of 1 row
 * tile, 8 of 2, 4 of 4) x rounds (4, 8, 16, 32, 64) are timed on the whole set; otherwise the directed
 * variants as in bf_autotune, on a leading sample of at most 131,072 of the targets.  ax/ay/az:
 * the accelerations the gradient pass contracts (required for BF_OP_GRADIENT, else ignored);
 * velocities are required for BF_OP_DTMIN.  Outputs of the timed passes are discarded.  Errors:
 * BF_ERR_ARG (bad arguments, empty sets), BF_ERR_NOMEM. */
BF_API int bf_autotune_pass(bf_ctx *ctx, int op, int prec, const bf_particles *P, const bf_set *targets,
                            const bf_set *sources, const double *ax, const double *ay, const double *az,
                            const char *cache_path);
/* Synchronising; allocates its own temporaries.  Tune the batched pass `op` (BF_OP_FORCES or
 * BF_OP_GRADIENT) on the caller's ensemble (arguments as bf_forces_batched /
 * bf_force_gradient_batched, ax/ay/az required for the gradient): targets per lane {1, 2, 4} x
 * waves {4, 8} x sources per work item {2048, 4096, 8192}; the fastest is stored for the buckets
 * of (max_active_total, max_cluster_n) and used by every batched call and capture of that
 * shape. */
BF_API int bf_autotune_batched(bf_ctx *ctx, int op, int prec, const bf_particles *P, int32_t n_clusters,
                               const int64_t *cluster_off, const int32_t *active_idx,
                               const int64_t *active_off, int64_t max_active_total, int64_t max_cluster_n,
                               const double *ax, const double *ay, const double *az, const char *cache_path);
/* Not synchronising.  The shape a batched pass of op / prec with these bounds would run:
 * targets per lane, waves per workgroup, sources per work item (forced, tuned or default).  Any
 * output pointer may be NULL. */
BF_API int bf_query_batched_config(bf_ctx *ctx, int op, int prec, int64_t max_active_total,
                                   int64_t max_cluster_n, int *k_per_lane, int *waves, int *chunk);
/* Load a tuning table written by the autotuners (tables without the sweep field hold directed
 * entries). */
BF_API int bf_autotune_load(bf_ctx *ctx, const char *cache_path);
/* Force the shape of the pair-symmetric sweep of op (BF_OP_FORCES / BF_OP_GRADIENT / BF_OP_DTMIN):
 * rows x waves in {1 x 16, 2 x 8, 4 x 4} (BF_ERR_UNSUPPORTED otherwise), rounds of resident
 * workgroups in [0, 64] (0: 64).  rows = 0 restores the tuned or default choice. */
BF_API int bf_set_symmetric_config(bf_ctx *ctx, int op, int rows, int waves, int rounds);
/* Scratch limit of a pass that takes a pair-symmetric sweep over one set (its row sums, column
 * partials and running sums; bytes, 0: the default 32 GiB).  A sweep whose partials exceed it
 * runs its distance shares in several passes, each adding its partials onto FP64 running sums
 * per particle (FP32 for the time-step maxima) in the order a single pass uses: the results are
 * bitwise those of one pass with the same shares.  If one share does not fit, the share count
 * grows until it does (the smallest pass is one block distance, 16 bytes per particle for the
 * mixed passes); the row sums are then grouped differently, and the sums may differ from the
 * unlimited pass's in the last bits (the time-step maxima do not).  Results stay bitwise
 * repeatable for a given limit. */
BF_API int bf_set_symmetric_scratch_limit(bf_ctx *ctx, size_t bytes);
/* Sweeps (passes over the distance shares) of the most recent
 * pass; 1 when it did not take a pair-symmetric sweep or ran in one. */
BF_API int bf_last_symmetric_passes(bf_ctx *ctx, int *passes);
/* Force the shape of the batched pass op at precision prec: targets per lane {1, 2, 4}, waves
 * {4, 8}, sources per work item a positive multiple of 64 * waves up to 2^20.  k = 0 restores the
 * tuned or default choice (2, 4, 4096). */
BF_API int bf_set_batched_config(bf_ctx *ctx, int op, int prec, int k_per_lane, int waves, int chunk);

/* Spatially sorted mode of the mixed acceleration and gradient passes.  ops_mask selects the
 * passes that use it: bit (1 << BF_OP_FORCES) and/or bit (1 << BF_OP_GRADIENT); the default is
 * both.  When selected, and r_fb == 0, with at least 16384 targets and 16384 sources and
 * 2^31 pairs (below that the sort costs more than it saves; bit BF_SORT_ANY_SIZE in ops_mask
 * lifts these limits), and without subsystem labels, targets and sources
 * are ordered along a Morton curve and the sources packed into tiles; a tile whose gap to a
 * workgroup's target box is at least kappa times its half-extent
 * is summed from FP32 offsets to the tile centre (pair separation rounding error at most
 * u (1 + 2 sqrt(3) / kappa) relative), nearer tiles from FP64 differences.  kappa = 0 keeps the
 * current value (default 1); otherwise it must lie in [0.5, 64] (BF_ERR_ARG).  Outputs stay
 * particle-indexed; results keep the accuracy of the unsorted mixed path.
 *
 * When the targets and the sources are one set (the same index array, or the same range), the
 * sorted pass evaluates every unordered pair once and applies its two equal and opposite terms
 * (Sec. 2.1: the acceleration term of j on i is -m_j/m_i times that of i on j, and so is the
 * force-gradient term): about 0.6 of the arithmetic.  It needs (n / 2048 + 1) * 16 bytes of
 * scratch per particle (8.6 GB at n = 2^20); above the limit of bf_set_symmetric_scratch_limit
 * (32 GiB) it runs in several passes over its distance shares.  The column sums go through
 * fixed-order partials, so results stay bitwise repeatable.
 * Bit BF_SORT_DIRECTED in ops_mask keeps the directed sweep for such passes.
 *
 * Bit (1 << BF_OP_DTMIN) (on by default) does the same for the mixed time-step pass over one set
 * with r_fb = 0, in the set's own order (no sort): a pair's free-fall and fly-by rates are the
 * same number for both particles, so each unordered pair is evaluated once for the two maxima.
 * From 24,576 particles (BF_SORT_ANY_SIZE: any size; the FP64 acceleration and gradient passes
 * over one set, swept the same way in their own order, from 32,768); (n / 2048 + 1) * 8 + 16
 * bytes of scratch per particle.
 * Results as the directed pass (a maximum is exact in any order), bitwise repeatable. */
BF_API int bf_set_spatial_sort(bf_ctx *ctx, int ops_mask, double kappa);

/* Synchronising.  Counters of the most recent acceleration / gradient / time-step pass: targets
 * re-evaluated in FP64 by the cancellation fix-up, and (spatially sorted mode) tile visits that
 * took the near (FP64-difference) and far (FP32 tile-offset) paths. */
BF_API int bf_last_pass_stats(bf_ctx *ctx, int64_t *fixups, int64_t *near_tiles, int64_t *far_tiles);

/* Not synchronising.  Pair interactions credited by the passes of op (bf_op) since the context
 * was created or last reset (reset != 0 clears the count after reading it): an acceleration,
 * gradient or time-step pass credits n_targets x n_sources directed pairs, less the self-pairs
 * (n_targets x (n_sources - 1)) when its targets and sources are one set (the same index array or
 * range); the two-set sums of bf_forces_between / bf_force_gradient_between credit 2 |a| |b|;
 * passes inside the HHS drivers credit alike.  Batched ensembles are not counted. */
BF_API int bf_pair_credit(bf_ctx *ctx, int op, int64_t *pairs, int reset);

/* Not synchronising.  How the most recent acceleration / gradient / time-step pass ran:
 * kind BF_PASS_UNSORTED, BF_PASS_SORTED (spatially sorted, directed sweep), BF_PASS_SYMMETRIC
 * (spatially sorted, each unordered pair once) or BF_PASS_BETWEEN (the two-set symmetric sweep
 * of bf_forces_between / bf_force_gradient_between); k_per_lane = targets per lane (row tiles per
 * wavefront for the symmetric sweeps), waves = wavefronts per workgroup, split = source chunks
 * (shares of the column range for the symmetric sweeps).  A mixed unsorted acceleration or
 * gradient pass of at most 6,144 targets and sources, with no subsystem labels, r_fb = 0 and no
 * forced or tuned configuration, runs as one launch of the small kernel (16 wavefronts splitting
 * the sources of 16 targets per workgroup) and reports k_per_lane 1, waves 16, split 1.  Any
 * pointer may be NULL.  Before the first pass all are 0. */
#define BF_PASS_UNSORTED 0
#define BF_PASS_SORTED 1
#define BF_PASS_SYMMETRIC 2
#define BF_PASS_BETWEEN 3
BF_API int bf_last_pass_config(bf_ctx *ctx, int *kind, int *k_per_lane, int *waves, int *split);

/* Kernel configuration the context would use for a directed pass of these sizes (for
 * reporting): targets per lane, waves per workgroup, source split.  A pass whose targets and
 * sources are one set may run the pair-symmetric sweep instead, and a small mixed pass the
 * one-launch small kernel; bf_last_pass_config tells. */
BF_API int bf_query_config(bf_ctx *ctx, int op, int prec, int64_t n_targets, int64_t n_sources,
                           int *k_per_lane, int *waves, int *split);
/* Force the kernel configuration for subsequent calls of op/prec (0 restores the default
 * choice; split 0 means automatic). */
BF_API int bf_set_config(bf_ctx *ctx, int op, int prec, int k_per_lane, int waves, int split);

/* ---- kernel timing ------------------------------------------------------------------ */

/* When on != 0 the context records a pair of HIP events on its stream around every launch
 * of the main pair kernel of bf_forces / bf_force_gradient / bf_dt_min, of the two-set sums and
 * of the persistent kernel of the batched passes (pack and reduction kernels excluded; nothing
 * inside a graph capture).  Turning timing on or off discards earlier records. */
BF_API int bf_enable_timing(bf_ctx *ctx, int on);
/* Synchronising.  Copy the durations (milliseconds) of the recorded launches of op
 * (bf_op) into ms[0 .. min(count, cap)), set *count to the number recorded, and discard
 * them. */
BF_API int bf_kernel_times(bf_ctx *ctx, int op, float *ms, int cap, int *count);

#ifdef __cplusplus
}
#endif

#endif /* BIFROST_H */
