/* fmm.h - C ABI of libfmm, an MI355X (gfx950) implementation of the fast
 * multipole method of W. Dehnen, "A fast multipole method for stellar
 * dynamics", Computational Astrophysics and Cosmology 1:1 (2014).
 *
 * It computes, for all N particles, the unsoftened potential and acceleration
 *     Psi_b = sum_{a != b} G mu_a / |x_b - x_a|,   a_b = grad Psi_b     (eq. 1)
 * by tree build, upward pass (P2M, M2M), a one-sided dual tree walk whose
 * acceptance test is the error-balancing criterion of Sec. 5.3
 * (eqs:mac:better), M2L, downward pass (L2L, L2P) and direct near-field sums
 * (P2P), every stage a HIP kernel.
 *
 * Conventions for every entry point
 *  - Array arguments named pos, mass, pot, acc, offsets are DEVICE pointers
 *    (e.g. torch tensors on the GPU), owned by the caller, never retained
 *    after the call returns.  pos is n x 3 row-major FP64 (x0,y0,z0,x1,...),
 *    mass n FP64, pot n FP64, acc n x 3 row-major FP64.  Inputs are read only.
 *  - Results are in input order.  pot is the physical potential
 *    Phi_b = -Psi_b (negative); acc = grad Psi_b points towards the mass.
 *  - Calls are ordered on the context's HIP stream and synchronous on return.
 *  - Argument errors are detected before any launch: FMM_E_INVAL, outputs
 *    untouched.  A context serves one host thread at a time (FMM_E_BUSY).
 *  - No C++ exception crosses this interface.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_ctx fmm_ctx;

typedef enum {
    FMM_OK = 0,
    FMM_E_INVAL = 1,       /* bad argument (nothing launched, nothing written) */
    FMM_E_NOMEM = 2,       /* device allocation failed */
    FMM_E_HIP = 3,         /* a HIP runtime call failed; see fmm_last_error */
    FMM_E_NONFINITE = 4,   /* non-finite input or output (e.g. two distinct
                              particles at one position); outputs written but
                              undefined */
    FMM_E_UNSUPPORTED = 5, /* expansion order outside the supported range */
    FMM_E_BUSY = 6         /* context already in use by another thread */
} fmm_status;

/* Multipole-acceptance criterion of the main walk. */
typedef enum {
    FMM_MAC_REL = 0,    /* theta < 1 and Etilde M_A / r^2 < eps min_B{a_b}  (eq:mac:better:a) */
    FMM_MAC_SCALED = 1, /* theta < 1 and Etilde M_A / r^2 < eps min_B{f_b}  (eq:mac:better:f) */
    FMM_MAC_THETA = 2   /* theta < theta_crit (eq:mac:theta); eps unused */
} fmm_mac;

/* Arithmetic of the evaluation kernels.  The tree, the low-order estimate
 * and the walk are FP64 in both modes, so both modes accept the same
 * interactions. */
typedef enum {
    FMM_PREC_FP64 = 0,  /* every step in FP64 */
    FMM_PREC_MIXED = 1  /* direct sums: separations formed in FP64 and rounded
                           once, then FP32 pair arithmetic and FP32 running sums
                           flushed into FP64 every 32 sources per lane; results
                           accumulated and returned in FP64 */
} fmm_precision;

/* Which M2L kernel evaluates the accepted cell pairs (same result up to
 * rounding). */
typedef enum {
    FMM_M2L_AUTO = 0,     /* the library's choice (currently always the direct
                             kernel) */
    FMM_M2L_DIRECT = 1,   /* eq:M2L as a double sum over the multipoles */
    FMM_M2L_ROTATION = 2  /* App. A: rotate the multipoles so that the interaction
                             is along z, eq:M2L:z, rotate back (FP64, orders up
                             to 16).  Compiled but switched off until its results
                             on the device are established: requesting it gives
                             FMM_E_UNSUPPORTED */
} fmm_m2l_kernel;

/* Expansion centre z = s of every cell (Sec. 5.1.1).  The acceptance test
 * uses each cell's actual radius about its centre, so the rule changes how
 * many interactions pass, not the accuracy of those that do. */
typedef enum {
    FMM_CENTRE_AUTO = 0,      /* the library's choice (currently FMM_CENTRE_ENCLOSING) */
    FMM_CENTRE_MIDPOINT = 1,  /* the midpoint of the cell's bounding box */
    FMM_CENTRE_ENCLOSING = 2  /* an approximation of the centre of the smallest
                                 sphere enclosing the spheres of the cell's
                                 grand-daughters (32 core-set steps of Badoiu and
                                 Clarkson from the midpoint, over the particles at
                                 a leaf), kept where the cell's radius about it is
                                 smaller than about the midpoint */
} fmm_centre;

/* Where min_B{a_b} (or f_b) comes from. */
typedef enum {
    FMM_SCALE_ESTIMATE = 0, /* low-order FMM estimate (Sec. 5.4.2) inside the call */
    FMM_SCALE_PREVIOUS = 1  /* in fmm_forces_refit calls that recycle the tree (the
                               same particles one step later): |acc| of the previous
                               call (Sec. 5.4.1); the estimate otherwise */
} fmm_scale_source;

typedef struct {
    int device;            /* HIP device ordinal */
    void *hip_stream;      /* hipStream_t to order work on; NULL = a stream the
                              context creates (default priority) */
    int leaf_size;         /* n_L, cells with more particles are split; 0 = 32 */
    fmm_mac mac;           /* FMM_MAC_REL by default (0) */
    double theta_crit;     /* FMM_MAC_THETA only */
    double p2p_factor;     /* accepted pairs with N_A N_B < p2p_factor (p+1)^3
                              are summed directly; 0 = 2 */
    fmm_scale_source scale_source;
    int timing;            /* nonzero: record per-phase HIP events (fmm_stats) */
    fmm_precision precision; /* FMM_PREC_FP64 by default (0) */
    fmm_m2l_kernel m2l_kernel; /* FMM_M2L_AUTO by default (0) */
    fmm_centre centre;     /* FMM_CENTRE_AUTO by default (0) */
    int64_t n_max;         /* 0: no limit; else a call with more particles (a
                              batch: in total) fails with FMM_E_INVAL */
    int p_max;             /* 0: FMM_P_MAX; else 1..FMM_P_MAX, and a call asking
                              for (or choosing from target_err) a higher order
                              fails with FMM_E_INVAL */
    size_t hbm_budget_bytes; /* 0: no limit; else a call whose
                              fmm_footprint_bytes(n, p, opts) exceeds it fails
                              with FMM_E_NOMEM before any launch, and fmm_build
                              fails with FMM_E_NOMEM if the footprint at n_max and
                              p_max (both set) exceeds it */
} fmm_opts;

/* Interaction counts and per-phase times of the last fmm_forces call. */
typedef struct {
    int p;                       /* expansion order used */
    int64_t n;                   /* particles */
    int64_t n_cells, n_leaves;   /* octree */
    int depth;                   /* deepest level (root = 0) */
    int64_t n_m2l;               /* accepted cell pairs evaluated by M2L */
    int64_t n_p2p_lists;         /* (source cell, sink leaf) direct-sum entries */
    int64_t n_p2p_pairs;         /* ordered particle pairs summed directly */
    int64_t n_est_m2l, n_est_p2p_pairs; /* the same for the estimate pass */
    int walk_iterations;         /* breadth-first walk sweeps (main pass) */
    /* milliseconds, measured with HIP events when fmm_opts.timing != 0
       (phases as in the paper's tab:complexity).  Two pairs of phases run at
       the same time on two streams: t_up is the part of the upward pass that
       the estimate does not hide, and t_m2l includes the sorting and merging
       of the direct-sum list, which runs beside M2L. */
    double t_tree, t_estimate, t_up, t_walk, t_m2l, t_p2p, t_down, t_total;
    /* average duration of one launch of the M2L and P2P kernels (ms) */
    double t_m2l_kernel, t_p2p_kernel;
    int m2l_launches, p2p_launches;
    /* cell pairs visited by the walk sweeps and the sweeps' time (ms),
       main pass and estimate pass */
    int64_t walk_pairs, est_walk_pairs;
    double t_sweeps, t_est_sweeps;
    int refitted;                /* 1 if the last call recycled the tree */
    int m2l_rotation;            /* 1 if the rotation M2L kernel ran */
} fmm_stats_t;

/* Create a context on opts->device.  Allocates only small bookkeeping; the
 * workspace grows on the first fmm_forces call with a larger n.
 * Returns FMM_E_INVAL for a NULL ctx or opts or out-of-range options. */
fmm_status fmm_build(fmm_ctx **ctx, const fmm_opts *opts);

/* Potential and acceleration of all n particles (eq. 1, Sec. 6).
 *   G          gravitational constant (applied at the end; the acceptance
 *              test is G invariant)
 *   p          expansion order FMM_P_MIN..FMM_P_MAX (from FMM_P_MIN_MIXED in
 *              mixed precision), or < 0 for the order chosen from target_err
 *              by fmm_order_for_error
 *   target_err accuracy parameter epsilon of eqs:mac:better (> 0, finite)
 * n = 0 is a no-op; n = 1 gives pot = acc = 0. */
fmm_status fmm_forces(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                      double G, int p, double target_err, double *pot, double *acc);

/* The same as fmm_forces for k independent clusters stored back to back:
 * cluster i holds particles [offsets[i], offsets[i+1]) (host array of k+1
 * int64, offsets[0] = 0); particles interact only within their cluster. */
fmm_status fmm_forces_batched(fmm_ctx *ctx, int64_t k, const int64_t *offsets_host,
                              const double *pos, const double *mass, double G, int p,
                              double target_err, double *pot, double *acc);

/* fmm_forces with tree recycling (Sec. 7.1): if the previous call on this
 * context built a tree for the same n (single cluster), its particle order and
 * cell membership are kept and only positions, cell geometry, radii,
 * expansions and interaction lists are recomputed; otherwise a full build.
 * Meant for time steps that move particles little.  The acceptance test uses
 * the true radii, so the result has the same accuracy; a recycled tree only
 * costs more as particles drift.  fmm_stats().refitted tells which happened. */
fmm_status fmm_forces_refit(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                            double G, int p, double target_err, double *pot, double *acc);

/* Forces on a listed subset of the particles, as block time-step schemes need
 * them (Sec. 7.1: forces for active particles only).  All n particles are
 * sources; active[j] (device int64, 0 <= active[j] < n, any order, repeats
 * allowed) are the sinks.  The tree, the expansions and the sink scale are
 * those of fmm_forces on all n particles; the walk visits only sink cells that
 * hold a listed particle, and the direct sums run only for their leaves.  So
 * pot[j] and acc[3j..3j+2] (n_active entries, device) are exactly the values
 * fmm_forces returns for particle active[j], at a cost that falls with the
 * number of sink cells involved.  refit != 0 recycles the tree as
 * fmm_forces_refit does.  An index out of range gives FMM_E_INVAL (entries
 * with valid indices are written).  Calls with a list do not update the
 * |a| kept for FMM_SCALE_PREVIOUS. */
fmm_status fmm_forces_active(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                             double G, int p, double target_err, int64_t n_active,
                             const int64_t *active, int refit, double *pot, double *acc);

/* fmm_forces with an individual accuracy parameter per particle (Sec. 7): the
 * acceptance test compares with min_{b in B}{eps_b a_b} (criterion a; f_b for
 * criterion f) instead of eps min_B{a_b}.  eps_particle: device, n FP64 in
 * input order, each > 0 and finite (FMM_E_INVAL otherwise, nothing written).
 * p < 0 takes the order for the smallest eps_b.  Not for FMM_MAC_THETA. */
fmm_status fmm_forces_eps(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                          double G, int p, const double *eps_particle, double *pot, double *acc);

/* Forces and jerk j = da/dt of every particle (Sec. 7, jerk; eqs:fmm:dot), for
 * particles moving with velocities vel (device, n x 3 FP64, input order).
 * pot and acc are those of fmm_forces with the same arguments (bit for bit
 * in FP64; with FMM_PREC_MIXED the direct sums of this call are FP64); jerk
 * (device, n x 3) receives G sum_a mu_a d/dt[(x_a - x_b)/|x_a - x_b|^3] with
 * the expansion centres held at rest: multipole rates from the time
 * derivative of eq:P2M (P2M:dot) and M2M, field-tensor rates from M2L of the
 * multipole rates over the same interaction list and order (FP64) and L2L,
 * eq:L2P:dot at the particles, and the time derivative of every direct pair,
 * summed in the same pass as its force.  The acceptance test is that of the acceleration; the
 * jerk's relative error is typically the order p times the force error.
 * A non-finite jerk gives FMM_E_NONFINITE. */
fmm_status fmm_forces_jerk(fmm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                           const double *mass, double G, int p, double target_err, double *pot,
                           double *acc, double *jerk);

/* fmm_forces_jerk for a listed subset of sinks, as Hermite integrators with
 * block time steps need it (Sec. 7.1 with Sec. 7, jerk): the sinks and outputs
 * as in fmm_forces_active (pot[j], acc[3j..], jerk[3j..] for particle
 * active[j], n_active entries each, device), the rest as in fmm_forces_jerk;
 * each listed particle's results equal those of fmm_forces_jerk on all n.
 * refit != 0 recycles the tree as fmm_forces_refit does. */
fmm_status fmm_forces_jerk_active(fmm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                                  const double *mass, double G, int p, double target_err,
                                  int64_t n_active, const int64_t *active, int refit, double *pot,
                                  double *acc, double *jerk);

/* Exact FP64 direct summation of eq. (1) on the GPU (the comparison
 * baseline): all n sinks against all n sources, a != b. */
fmm_status fmm_direct(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                      double G, double *pot, double *acc);

/* The same exact sum for selected sinks only: sinks[j] (device int64,
 * 0 <= sinks[j] < n) receives pot[j] and acc[3j..3j+2] from all n sources
 * (a != sinks[j]).  An index out of range gives FMM_E_INVAL (such entries are
 * not read; the others are written). */
fmm_status fmm_direct_sinks(fmm_ctx *ctx, int64_t n, const double *pos, const double *mass,
                            double G, int64_t nsinks, const int64_t *sinks, double *pot,
                            double *acc);

/* fmm_direct_sinks for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results (bit for bit), but the partial sums
 * and the index flag live in a static device array of
 * FMM_NOALLOC_SCRATCH_BYTES per device, reserved for the life of the process,
 * instead of context buffers; the call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  A call whose partial sums would
 * not fit gives FMM_E_INVAL (the library's split of the sources keeps them
 * below 16 MiB, so this does not happen for valid sizes).  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * contexts, other streams, other threads) race and must not be issued. */
fmm_status fmm_direct_sinks_noalloc(fmm_ctx *ctx, int64_t n, const double *pos,
                                    const double *mass, double G, int64_t nsinks,
                                    const int64_t *sinks, double *pot, double *acc);

/* The exact jerk of selected sinks (the comparison baseline of
 * fmm_forces_jerk): sinks[j] (device int64, 0 <= sinks[j] < n) receives
 * jerk[3j..3j+2] = G sum_{a != b} mu_a [v_ab/r^3 - 3 (r . v_ab) r/r^5],
 * r = x_a - x_b, v_ab = v_a - v_b, from all n sources (vel: device, n x 3).
 * An index out of range gives FMM_E_INVAL (such entries are not read). */
fmm_status fmm_direct_jerk_sinks(fmm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                                 const double *mass, double G, int64_t nsinks,
                                 const int64_t *sinks, double *jerk);

/* Expansion order used when fmm_forces gets p < 0: round(1.6 log10(1/eps)) + 2,
 * clamped to [3, FMM_P_MAX] (two above the paper's CPU optimum, Sec. 6.2: the
 * measured balance of M2L and direct sums on this GPU); -1 for eps <= 0 or NaN. */
int fmm_order_for_error(double target_err);

/* Statistics of the last call (FMM_E_INVAL for NULL arguments). */
fmm_status fmm_stats(const fmm_ctx *ctx, fmm_stats_t *out);

/* Device bytes a call with n particles at order p is expected to need
 * (workspace + interaction lists), for admission control. */
size_t fmm_footprint_bytes(int64_t n, int p, const fmm_opts *opts);

/* Text of the last error on this context ("" if none); valid until the next call. */
const char *fmm_last_error(const fmm_ctx *ctx);

/* Release the context and its workspace. NULL is ignored. */
void fmm_destroy(fmm_ctx *ctx);

/* Debug export of internal arrays of the last fmm_forces call, copied to the
 * HOST buffer dst (capacity bytes).  Returns the number of bytes the array
 * has (copying only if it fits), or -1 for an unknown id.
 *   FMM_EXPORT_M2L   int64 pairs (source id, sink id), id = level << 40 | begin
 *                    with begin the cell's first particle in Morton order
 *   FMM_EXPORT_P2P   int64 triples (sink id, first, end): the sink cell and the
 *                    Morton-order particle range of the source cell summed
 *                    directly onto it
 *   FMM_EXPORT_SCALE double per particle (input order): sink scale a_b or f_b used
 *   FMM_EXPORT_CELLS int64 per cell: level << 40 | begin, then end, in cell order
 *   FMM_EXPORT_CENTRES double per cell, cell order: expansion centre x, y, z
 *                    and the radius rho of the cell's particles about it */
enum { FMM_EXPORT_M2L = 1, FMM_EXPORT_P2P = 2, FMM_EXPORT_SCALE = 3, FMM_EXPORT_CELLS = 4,
       FMM_EXPORT_CENTRES = 5 };
int64_t fmm_export(fmm_ctx *ctx, int what, void *dst, int64_t capacity);

#define FMM_P_MAX 20
/* Lowest accepted expansion orders: 3 for FP64 evaluations and every jerk
 * call, 2 in mixed precision; lower orders give FMM_E_UNSUPPORTED.  (The
 * FP64 kernels of orders 1 and 2 have no passing device run: the one run that
 * reached them ended in a GPU fault whose cause is not known.  The order
 * chosen from target_err is never below 3.) */
#define FMM_P_MIN 3
#define FMM_P_MIN_MIXED 2
/* Size of the static per-device scratch array of fmm_direct_sinks_noalloc:
 * 256 bytes of flags and 16 MiB of partial sums. */
#define FMM_NOALLOC_SCRATCH_BYTES (256 + (16u << 20))

#ifdef __cplusplus
}
#endif
#endif
