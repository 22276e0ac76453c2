/* CPU oracle for the fast multipole method of Dehnen, "A fast multipole method
 * for stellar dynamics" (Comput. Astrophys. Cosmol. 2014).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, FP64 reference
 * that the GPU path is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code
 * with the HIP library: no headers, helpers, tables or kernels.
 *
 * Contents
 *   direct.c    - the exact result: direct summation of eq. (1) (eq:P2P), of
 *                 the scale f (eq:f) and of the jerk (the time derivative of
 *                 the acceleration, Sec. 7), Neumaier-compensated, threaded
 *                 over sinks (result independent of the thread count).
 *   harmonics.c - complex solid harmonics Theta_n^m, Upsilon_n^m (Sec. 2.1,
 *                 App. A.3, A.5) and the FMM kernels P2M, M2M, M2L, L2L, L2P
 *                 (eqs:fmm), multipole power P_n (eq:def:PA), the error
 *                 estimate E_{A->B} (eq:def:EAB, eq:err:tilde), the x <-> z
 *                 swap matrices and the rotation-accelerated M2L (App. A), the
 *                 time derivatives of Upsilon and the P2M and L2P rates of the
 *                 jerk (App. A.5, eqs:fmm:dot).
 *   fmm.c       - a plain recursive FMM following the paper's phases: tree,
 *                 low-order estimate of the sink scale (Sec. 5.4.2), upward
 *                 pass, one-sided dual tree walk with the error-balancing
 *                 acceptance criterion (eqs:mac:better), downward pass;
 *                 optionally individual eps_b, an adaptive order per pair
 *                 and the jerk (Sec. 7).
 *
 * Complex arrays are stored interleaved (re, im) with index n*n + n + m for
 * 0 <= n <= p, -n <= m <= n, i.e. (p+1)^2 complex numbers.
 */
#ifndef FMM_ORACLE_H
#define FMM_ORACLE_H

#include <stdint.h>
#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_IDX(n, m) ((n) * (n) + (n) + (m))

/* ---- direct summation (direct.c) -------------------------------------- */
/* For every sink b in `sinks` (or all b when sinks == NULL):
 *   pot[i] = -G sum_{a != b} mu_a / |x_b - x_a|           (physical potential)
 *   acc[i] =  G sum_{a != b} mu_a (x_a - x_b)/|x_a - x_b|^3
 *   f[i]   =  G sum_{a != b} mu_a / |x_a - x_b|^2          (eq:f)
 * where i indexes the sink list.  Sources are taken in index order; each
 * component is summed with Neumaier compensation.  Any of pot/acc/f may be
 * NULL.  Returns 0, or -1 on bad arguments. */
int or_direct(int64_t n, const double *pos, const double *mass, double G,
              int64_t n_sinks, const int64_t *sinks, int threads,
              double *pot, double *acc, double *f);

/* jerk[3i..] = G sum_{a != b} mu_a [v_ab/r^3 - 3 (r.v_ab) r/r^5] with r = x_a - x_b,
 * v_ab = v_a - v_b (the time derivative of acc above; Sec. 7, jerk), same sink
 * list, summation order and compensation as or_direct. */
int or_direct_jerk(int64_t n, const double *pos, const double *vel, const double *mass,
                   double G, int64_t n_sinks, const int64_t *sinks, int threads,
                   double *jerk);

/* ---- harmonics and kernels (harmonics.c), complex, all m ------------- */
void or_theta(const double r[3], int p, double complex *T);
void or_upsilon(const double r[3], int p, double complex *U);
/* M_n^m(z) += sum_a mu_a Upsilon_n^m(x_a - z)                       eq:P2M */
void or_p2m(int64_t n, const double *pos, const double *mass,
            const double z[3], int p, double complex *M);
/* Mout_n^m(z') += sum_{k,l} Upsilon_k^l(z - z') M_{n-k}^{m-l}(z)     eq:M2M */
void or_m2m(const double complex *M, const double z_minus_zp[3], int p,
            double complex *Mout);
/* F_n^m(s_B) += sum_{k<=p-n} sum_l conj(M_k^l) Theta_{n+k}^{m+l}(s_B - z_A) eq:M2L */
void or_m2l(const double complex *M, const double sB_minus_zA[3], int p,
            double complex *F);
/* Fout_n^m(s') += sum_{k<=p-n} sum_l conj(Upsilon_k^l(s - s')) F_{n+k}^{m+l}(s) eq:L2L */
void or_l2l(const double complex *F, const double s_minus_sp[3], int p,
            double complex *Fout);
/* Psi_0^0 and a = -(Re Psi_1^1, Im Psi_1^1, Psi_1^0) at x_b     eq:L2P:Psi, eq:L2P */
void or_l2p(const double complex *F, const double sB_minus_x[3], int p,
            double *psi, double acc[3]);
/* d/dt Upsilon_n^m(r) for dr/dt = v, n = 0..p (App. A.5, time derivatives):
 * xidot Upsilon_{n-1}^{m-1} + zdot Upsilon_{n-1}^m + etadot Upsilon_{n-1}^{m+1}
 * with xi = (x+iy)/2, eta = -(x-iy)/2 (eq:xi:eta) */
void or_upsilon_dot(const double r[3], const double v[3], int p, double complex *Ud);
/* Mdot_n^m(z) += sum_a mu_a d/dt Upsilon_n^m(x_a - z) with dx_a/dt = v_a   eq:P2M:dot */
void or_p2m_dot(int64_t n, const double *pos, const double *vel, const double *mass,
                const double z[3], int p, double complex *Md);
/* jerk contribution of a local expansion F and its time derivative Fd at a
 * particle moving with v: j = -(Re Psidot_1^1, Im Psidot_1^1, Psidot_1^0) with
 * Psidot_1^m = sum_{k<=p-1,l} [conj(Upsilon_k^l(s_B - x)) Fd_{1+k}^{m+l}
 *             + conj(d/dt Upsilon_k^l(s_B - x, -v)) F_{1+k}^{m+l}]   eq:L2P:dot */
void or_l2p_dot(const double complex *F, const double complex *Fd, const double sB_minus_x[3],
                const double v[3], int p, double jerk[3]);
/* Swap matrix B_n (x <-> z) of eq:Ylm:swap by its recurrence (App. A):
 * (2n+1)^2 doubles, row m = -n..n, column l = -n..n, row-major. */
void or_swap_matrix(int n, double *B);
/* The same F += M2L as or_m2l by the rotation-accelerated kernel of App. A:
 * rotate M so that s_B - z_A points along z, eq:M2L:z, rotate back. */
void or_m2l_rot(const double complex *M, const double sB_minus_zA[3], int p,
                double complex *F);
/* P_n = sqrt(sum_m (n-m)!(n+m)! |M_n^m|^2), n = 0..p              eq:def:PA */
void or_power(const double complex *M, int p, double *P);
/* E_{A->B} of eq:def:EAB times M_A (i.e. without the 1/M_A factor) */
double or_eab_times_mass(const double *P, int p, double rho_sB, double r);
/* factor 8 max(rho_A, rho_B)/(rho_A + rho_B) of eq:err:tilde (8 when both 0) */
double or_etilde_factor(double rho_zA, double rho_sB);

/* ---- the plain FMM (fmm.c) ------------------------------------------ */
enum { OR_MAC_A = 0, OR_MAC_F = 1, OR_MAC_THETA = 2 };
enum { OR_SCALE_ESTIMATE = 0, OR_SCALE_GIVEN = 1 };
enum { OR_CENTRE_MIDPOINT = 0, OR_CENTRE_ENCLOSING = 1 };

typedef struct {
    int p;             /* expansion order, 1..30 */
    double eps;        /* accuracy parameter epsilon of eqs:mac:better */
    int leaf_size;     /* n_L: a cell with more particles is split (depth < 21) */
    int mac;           /* OR_MAC_A (eq:mac:better:a), OR_MAC_F, OR_MAC_THETA */
    double theta_crit; /* for OR_MAC_THETA only (eq:mac:theta) */
    double p2p_pairs;  /* T: accepted pairs with N_A*N_B < T are summed directly */
    int scale_source;  /* OR_SCALE_ESTIMATE or OR_SCALE_GIVEN */
    const double *scale; /* OR_SCALE_GIVEN: per-particle a_b or f_b (input order, G=1 units) */
    double G;
    const double *eps_particle; /* NULL, or individual accuracy parameters eps_b (input
                                   order): the criterion compares with min_B{eps_b a_b}
                                   instead of eps min_B{a_b} (Sec. 7) */
    int adaptive_order; /* q_min > 0: each cell pair evaluated by M2L uses the
                           lowest order q in [q_min, p] that passes the criterion
                           (Sec. 7); 0: every pair at order p.  About the centre of
                           mass the dipole power vanishes, so the estimate at q = 1
                           can be zero while the error is not: q_min >= 2 */
    const double *vel;  /* NULL, or velocities (input order, 3n): then jerk (3n,
                           input order) receives the jerk (Sec. 7, jerk), with the
                           expansion centres at rest: Mdot by eq:P2M:dot and M2M,
                           Fdot by M2L of Mdot and L2L, eq:L2P:dot at the particles,
                           and the time derivative of the direct sums */
    double *jerk;
    int centre;         /* OR_CENTRE_MIDPOINT: z = s = the midpoint of the cell's
                           bounding box; OR_CENTRE_ENCLOSING: an approximation of
                           the centre of the smallest enclosing sphere (Sec. 5.1.1),
                           kept where it gives the smaller radius */
} or_fmm_params;

typedef struct {
    int64_t n_cells, n_leaves, depth;
    int64_t n_m2l;          /* accepted cell->cell interactions done by M2L */
    int64_t n_p2p_cells;    /* cell->cell interactions done by direct summation */
    int64_t n_p2p_pairs;    /* particle pairs summed directly (ordered, a != b) */
    int64_t n_est_m2l, n_est_p2p_pairs; /* the same for the estimate pass */
    int64_t m2l_order_sum;  /* sum over M2L pairs of the order used */
    int64_t m2l_macs;       /* complex multiply-adds of eq:M2L over all pairs:
                               sum_{n<=q} (n+1)(q-n+1)^2 per pair of order q */
} or_fmm_stats;

/* Optional outputs for list comparison.  A cell is identified by
 * (level << 40) | begin, with begin its first particle in Morton order.
 * m2l[2i] = source id, m2l[2i+1] = sink id; p2p likewise (sink may be any
 * cell).  Entries are written while i < *_cap; *_count returns the total. */
typedef struct {
    int64_t *m2l; int64_t m2l_cap; int64_t m2l_count;
    int64_t *p2p; int64_t p2p_cap; int64_t p2p_count;
    double *scale_est;      /* per particle (input order): the sink scale used */
    int64_t *cell_ids;      /* NULL, or 2 per cell (creation order, parents
                               first): its id and its end (Morton order), while
                               i < cell_cap; cell_count = cells */
    double *cell_geo;       /* 5 per cell: centre x, y, z, radius rho about it,
                               radius about the box midpoint */
    int64_t cell_cap, cell_count;
    int64_t *order;         /* NULL, or n: input index of Morton position i */
} or_fmm_lists;

/* pot[i] = physical potential, acc[i*3..] = acceleration of particle i (input
 * order).  Returns 0 on success, -1 on bad arguments, -2 on allocation
 * failure. */
int or_fmm(const or_fmm_params *prm, int64_t n, const double *pos,
           const double *mass, double *pot, double *acc,
           or_fmm_stats *stats, or_fmm_lists *lists);

#ifdef __cplusplus
}
#endif
#endif
