/* Oracle: exact direct summation (test infrastructure only).
 *
 * The exact result the multipole method approximates: the (negative)
 * potential Psi_b = sum_{a != b} G mu_a / |x_b - x_a| of eq. (1) (eq:P2P),
 * its gradient a_b = grad Psi_b, and the scale f_b = sum_{a != b} G mu_a /
 * |x_a - x_b|^2 of eq:f (Sec. 3.1).  FP64, 1/sqrt with correctly rounded sqrt
 * and division, sources in index order, every sum Neumaier-compensated.
 * Threads split the sink list; each sink's sums are independent of the
 * split, so the result is bitwise the same for any thread count.
 *
 * The jerk j_b = d a_b / dt (Sec. 7, jerk) is the time derivative of the same
 * sum for particles moving with velocities v:
 *   j_b = G sum_{a != b} mu_a [ v_ab / r^3 - 3 (r . v_ab) r / r^5 ],
 *   r = x_a - x_b, v_ab = v_a - v_b.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>

typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else                       k->c += (v - t) + k->s;
    k->s = t;
}
static inline double ks_val(const ksum *k) { return k->s + k->c; }

typedef struct {
    int64_t n; const double *pos, *mass; double G;
    const int64_t *sinks; int64_t lo, hi;
    double *pot, *acc, *f;
    const double *vel; double *jerk;   /* jerk jobs: vel in, jerk out */
} job;

static void one_sink(const job *j, int64_t i) {
    const int64_t b = j->sinks ? j->sinks[i] : i;
    const double xb = j->pos[3 * b], yb = j->pos[3 * b + 1], zb = j->pos[3 * b + 2];
    ksum sp = {0, 0}, sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sf = {0, 0};
    for (int64_t a = 0; a < j->n; ++a) {
        if (a == b) continue;
        const double dx = j->pos[3 * a] - xb;
        const double dy = j->pos[3 * a + 1] - yb;
        const double dz = j->pos[3 * a + 2] - zb;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double r = sqrt(r2);
        const double mu = j->mass[a];
        const double q = mu / r;                 /* mu/r      */
        const double q3 = q / r2;                /* mu/r^3    */
        ks_add(&sp, q);
        ks_add(&sx, q3 * dx);
        ks_add(&sy, q3 * dy);
        ks_add(&sz, q3 * dz);
        ks_add(&sf, mu / r2);
    }
    if (j->pot) j->pot[i] = -j->G * ks_val(&sp);
    if (j->acc) {
        j->acc[3 * i]     = j->G * ks_val(&sx);
        j->acc[3 * i + 1] = j->G * ks_val(&sy);
        j->acc[3 * i + 2] = j->G * ks_val(&sz);
    }
    if (j->f) j->f[i] = j->G * ks_val(&sf);
}

static void one_sink_jerk(const job *j, int64_t i) {
    const int64_t b = j->sinks ? j->sinks[i] : i;
    const double *xb = &j->pos[3 * b], *vb = &j->vel[3 * b];
    ksum s[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t a = 0; a < j->n; ++a) {
        if (a == b) continue;
        double r[3], v[3];
        for (int d = 0; d < 3; ++d) {
            r[d] = j->pos[3 * a + d] - xb[d];
            v[d] = j->vel[3 * a + d] - vb[d];
        }
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double rr = sqrt(r2);
        const double q3 = j->mass[a] / (r2 * rr);            /* mu/r^3 */
        const double rv = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) / r2;
        for (int d = 0; d < 3; ++d) ks_add(&s[d], q3 * (v[d] - 3.0 * rv * r[d]));
    }
    for (int d = 0; d < 3; ++d) j->jerk[3 * i + d] = j->G * ks_val(&s[d]);
}

static void *worker(void *arg) {
    const job *j = (const job *)arg;
    for (int64_t i = j->lo; i < j->hi; ++i) {
        if (j->jerk) one_sink_jerk(j, i);
        else one_sink(j, i);
    }
    return NULL;
}

static int run_jobs(int64_t n, const double *pos, const double *mass, double G,
                    int64_t n_sinks, const int64_t *sinks, int threads,
                    double *pot, double *acc, double *f, const double *vel, double *jerk);

int or_direct(int64_t n, const double *pos, const double *mass, double G,
              int64_t n_sinks, const int64_t *sinks, int threads,
              double *pot, double *acc, double *f) {
    return run_jobs(n, pos, mass, G, n_sinks, sinks, threads, pot, acc, f, NULL, NULL);
}

int or_direct_jerk(int64_t n, const double *pos, const double *vel, const double *mass,
                   double G, int64_t n_sinks, const int64_t *sinks, int threads,
                   double *jerk) {
    if (!jerk || (n > 0 && !vel)) return -1;
    return run_jobs(n, pos, mass, G, n_sinks, sinks, threads, NULL, NULL, NULL, vel, jerk);
}

static int run_jobs(int64_t n, const double *pos, const double *mass, double G,
                    int64_t n_sinks, const int64_t *sinks, int threads,
                    double *pot, double *acc, double *f, const double *vel, double *jerk) {
    if (n < 0 || (n > 0 && (!pos || !mass))) return -1;
    if (!sinks) n_sinks = n;
    if (n_sinks < 0) return -1;
    for (int64_t i = 0; sinks && i < n_sinks; ++i)
        if (sinks[i] < 0 || sinks[i] >= n) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((int64_t)threads > n_sinks) threads = n_sinks > 0 ? (int)n_sinks : 1;
    job jobs[256];
    pthread_t tid[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (job){n, pos, mass, G, sinks, n_sinks * t / threads,
                        n_sinks * (t + 1) / threads, pot, acc, f, vel, jerk};
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) break;
        started = t;
    }
    worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    /* any job whose thread failed to start runs here */
    for (int t = started + 1; t < threads; ++t) worker(&jobs[t]);
    return 0;
}
