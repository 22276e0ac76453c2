/* Oracle: a plain recursive FMM (test infrastructure only).
 *
 * Follows the phases of the paper's solver (Sec. 6.4, tab:complexity):
 *   1. tree:     octree of cubic cells (Sec. 2.2.1); a cell holding more than
 *                n_L particles is split into its non-empty octants.  Octants
 *                come from 21-bit-per-axis quantised coordinates inside the
 *                cube around the bounding box (the tree's definition, shared
 *                with the GPU path by specification, not by code).  A cell
 *                at level 21 that still holds more than n_L particles (a
 *                dense cusp inside a very wide halo) is refined further with
 *                the next 21 bits of the same quantisation: its particles
 *                are re-sorted by those bits (ties by input index) and the
 *                split continues down to level 42, where leaves may be
 *                overfull.  The paper's tree has no depth limit.
 *   2. estimate: low-order FMM for the sink scale (Sec. 5.4.2): centres
 *                z = s = z_com, acceptance theta < 1 with radii about z_com,
 *                p = 1 for the acceleration a_b (criterion a) or the p = 0
 *                monopole of the 1/r^2 Green's function for f_b (criterion f),
 *                exact near field.  Walk one-sided (the paper's estimate pass
 *                walks mutually; the estimate only needs ~15% accuracy).
 *   3. up:       centres and radii, P2M at leaves, M2M upward (eq:P2M,
 *                eq:M2M), multipole power P_n (eq:def:PA), minimum sink scale.
 *   4. walk:     one-sided dual tree walk from (root, root) (Sec. 2.2.2,
 *                Sec. 6.1): accepted interactions by M2L (eq:M2L) - or by
 *                direct summation when N_A N_B is below a threshold - and
 *                the rest split at the larger cell, leaf-leaf by P2P.
 *                Acceptance: theta < 1 and Etilde M_A / r^2 < eps min_B{a_b}
 *                (eq:mac:better:a) or min_B{f_b} (eq:mac:better:f).
 *   5. down:     L2L (eq:L2L) top down, L2P (eq:L2P) at leaf particles.
 * With velocities the same passes also carry the time derivatives for the
 * jerk (Sec. 7, eqs:fmm:dot): centres at rest, Mdot by eq:P2M:dot and M2M,
 * Fdot by M2L of Mdot (same pairs, same order) and L2L, eq:L2P:dot at the
 * particles, and the time derivative of every direct pair.
 *
 * Expansion centre of every cell (z = s): the midpoint of the bounding box of
 * its particles, or (OR_CENTRE_ENCLOSING) an approximation of the paper's
 * centre of the smallest sphere enclosing the spheres of the cell's
 * grand-daughters (Sec. 5.1.1), kept where it gives the smaller radius; rho =
 * max distance of its particles from that centre (Sec. 4: rho_z, rho_s
 * definitions).  The choice changes the cost of the walk, not its accuracy,
 * because the acceptance test uses the actual radius.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KEYLEVELS 21              /* levels resolved by one 63-bit key */
#define MAXLEVEL (2 * KEYLEVELS)  /* levels 22..42 use the second key word */

typedef struct {
    int64_t begin, end;
    int level, nchild;
    int64_t child[8];
    int64_t parent;
    double mass, com[3], rho_com;
    double c[3], rho;
    double rho_mid;          /* radius about the box midpoint (the default centre) */
    double bc[3], bR;        /* enclosing-sphere candidate centre and cover radius */
    double smin;
    double complex *M, *F;   /* order p at c */
    double complex *Md, *Fd; /* their time derivatives (jerk only) */
    double complex Me[4], Fe[4]; /* order 1 at com (estimate of a) */
    double fe;               /* 1/r^2 monopole sum (estimate of f) */
    double *P;
} cell_t;

typedef struct {
    const or_fmm_params *prm;
    int64_t n;
    int p, ncoef;
    /* particles in Morton order */
    double *x;      /* 3n */
    double *m;
    double *v;      /* 3n velocities (jerk only) */
    int64_t *orig;  /* Morton position -> input index */
    uint64_t *key;  /* levels 1..21 */
    uint64_t *key2; /* levels 22..42 (only inside overfull level-21 cells) */
    double lo[3], kscale;     /* key cube: lower corner, 2^21 / side */
    cell_t *cells; int64_t ncells, cap;
    /* accumulators, Morton order */
    double *pot, *acc;      /* near + far */
    double *jerk;           /* 3n (jerk only) */
    double *est_acc, *est_f;
    double *scale;          /* per particle sink scale, Morton order */
    or_fmm_stats *st;
    or_fmm_lists *lists;
    int64_t nm2l_rec, np2p_rec;
    int oom;
} fmm_t;

/* ---------------------------------------------------------------- tree */

typedef struct { uint64_t key; int64_t idx; } keyidx;

static int cmp_keyidx(const void *a, const void *b) {
    const keyidx *u = (const keyidx *)a, *v = (const keyidx *)b;
    if (u->key != v->key) return u->key < v->key ? -1 : 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

/* bit i of the x, y, z cell index goes to key bit 3i, 3i+1, 3i+2 */
static uint64_t morton(uint32_t qx, uint32_t qy, uint32_t qz) {
    uint64_t k = 0;
    for (int i = 0; i < KEYLEVELS; ++i) {
        k |= (uint64_t)((qx >> i) & 1u) << (3 * i);
        k |= (uint64_t)((qy >> i) & 1u) << (3 * i + 1);
        k |= (uint64_t)((qz >> i) & 1u) << (3 * i + 2);
    }
    return k;
}

static int64_t new_cell(fmm_t *t) {
    if (t->ncells == t->cap) {
        int64_t cap = t->cap ? 2 * t->cap : 1024;
        cell_t *c = (cell_t *)realloc(t->cells, sizeof(cell_t) * (size_t)cap);
        if (!c) { t->oom = 1; return -1; }
        t->cells = c; t->cap = cap;
    }
    memset(&t->cells[t->ncells], 0, sizeof(cell_t));
    return t->ncells++;
}

/* The second key word of particle i (Morton order): bits 22..42 of the
 * quantised coordinates, u * 2^21 with u the same product as for the first
 * word (so both words describe one 42-bit cell index per axis). */
static uint64_t deep_key(const fmm_t *t, int64_t i) {
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        const double u = (t->x[3 * i + d] - t->lo[d]) * t->kscale;
        const double u42 = u * 2097152.0;
        const uint64_t v = u42 >= 4398046511103.0 ? 4398046511103ull : (uint64_t)u42;
        q[d] = (uint32_t)(v & 2097151u);
    }
    return morton(q[0], q[1], q[2]);
}

/* sort particles [b, e) by (second key word, input index); the range is one
 * level-21 cell, whose particles are in input-index order */
static int refine(fmm_t *t, int64_t b, int64_t e) {
    const int64_t k = e - b;
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * (size_t)k);
    double *x = (double *)malloc(sizeof(double) * 3 * (size_t)k);
    double *m = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t *o = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!ki || !x || !m || !o) { free(ki); free(x); free(m); free(o); return -1; }
    for (int64_t i = 0; i < k; ++i) { ki[i].key = deep_key(t, b + i); ki[i].idx = i; }
    qsort(ki, (size_t)k, sizeof(keyidx), cmp_keyidx);
    memcpy(x, t->x + 3 * b, sizeof(double) * 3 * (size_t)k);
    memcpy(m, t->m + b, sizeof(double) * (size_t)k);
    memcpy(o, t->orig + b, sizeof(int64_t) * (size_t)k);
    for (int64_t i = 0; i < k; ++i) {
        const int64_t j = ki[i].idx;
        t->orig[b + i] = o[j];
        t->m[b + i] = m[j];
        for (int d = 0; d < 3; ++d) t->x[3 * (b + i) + d] = x[3 * j + d];
        t->key2[b + i] = ki[i].key;
    }
    free(ki); free(x); free(m); free(o);
    return 0;
}

static int64_t build(fmm_t *t, int64_t b, int64_t e, int level, int64_t parent) {
    const int64_t id = new_cell(t);
    if (id < 0) return -1;
    cell_t *C = &t->cells[id];
    C->begin = b; C->end = e; C->level = level; C->parent = parent;
    if (e - b > t->prm->leaf_size && level < MAXLEVEL) {
        if (level == KEYLEVELS && refine(t, b, e) < 0) { t->oom = 1; return -1; }
        const uint64_t *key = level < KEYLEVELS ? t->key : t->key2;
        const int shift = 3 * ((level < KEYLEVELS ? KEYLEVELS : MAXLEVEL) - (level + 1));
        int64_t s = b;
        for (int oct = 0; oct < 8; ++oct) {
            int64_t q = s;
            while (q < e && (int)((key[q] >> shift) & 7u) == oct) ++q;
            if (q > s) {
                const int64_t ch = build(t, s, q, level + 1, id);
                if (ch < 0) return -1;
                C = &t->cells[id]; /* realloc may have moved it */
                C->child[C->nchild++] = ch;
            }
            s = q;
        }
    }
    return id;
}

static int is_leaf(const cell_t *C) { return C->nchild == 0; }

static int64_t cell_id(const cell_t *C) { return ((int64_t)C->level << 40) | C->begin; }

/* mass, centre of mass, bounding-box centre and the radii, straight from the
 * cell's particles */
static void cell_geometry(fmm_t *t, cell_t *C) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double M = 0, mx = 0, my = 0, mz = 0;
    for (int64_t i = C->begin; i < C->end; ++i) {
        const double *x = &t->x[3 * i];
        for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], x[d]); hi[d] = fmax(hi[d], x[d]); }
        M += t->m[i]; mx += t->m[i] * x[0]; my += t->m[i] * x[1]; mz += t->m[i] * x[2];
    }
    C->mass = M;
    C->com[0] = mx / M; C->com[1] = my / M; C->com[2] = mz / M;
    for (int d = 0; d < 3; ++d) C->c[d] = (lo[d] + hi[d]) * 0.5;
    double r2max = 0, r2com = 0;
    for (int64_t i = C->begin; i < C->end; ++i) {
        const double *x = &t->x[3 * i];
        const double dx = x[0] - C->c[0], dy = x[1] - C->c[1], dz = x[2] - C->c[2];
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 > r2max) r2max = r2;
        const double ex = x[0] - C->com[0], ey = x[1] - C->com[1], ez = x[2] - C->com[2];
        const double e2 = (ex * ex + ey * ey) + ez * ez;
        if (e2 > r2com) r2com = e2;
    }
    C->rho = sqrt(r2max);
    C->rho_mid = C->rho;
    C->rho_com = sqrt(r2com);
}

/* ------------------------------------------------- enclosing-sphere centre */

/* Sec. 5.1.1 takes s = z as the centre of the smallest sphere enclosing the
 * spheres of a cell's grand-daughter cells.  Here that centre is approximated
 * by the Frank-Wolfe iteration with exact line search for the minimum
 * enclosing ball (Yildirim 2008, SIAM J. Optim. 19, 1368, Algorithm 1):
 *   start: a = the point of the set farthest from the box midpoint, b = the
 *          point farthest from a; c = (a + b)/2, gamma = |a - b|^2/4;
 *   step:  q = the point farthest from c, D2 = |q - c|^2; stop if gamma <= 0
 *          or delta = D2/gamma - 1 <= OR_FW_TOL (then the radius about c is
 *          within sqrt(1 + OR_FW_TOL), 0.1%, of the optimum), else with
 *          lambda = delta / (2 (1 + delta)) move c += lambda (q - c) and set
 *          gamma = (1 - lambda) gamma + lambda (1 - lambda) D2;
 * at most OR_FW_ITERS steps.  gamma is the dual objective, a lower bound of
 * the squared optimal radius.  The set is, for a leaf, its particles, and for
 * an internal cell the spheres (b, R) of its grand-daughters, a daughter that
 * is a leaf standing in for its own daughters.  Particles are compared by
 * squared distance; "the point farthest from c" of a sphere (x, R) at
 * distance d = |x - c| is x + (x - c) R/d, at distance d + R (x + (R, 0, 0)
 * when d = 0), with D2 = (d + R)^2.  Each cell hands its ancestors the sphere
 * (b, R): b the final c, R the largest distance (d + R) over its set.  Ties in
 * "farthest" go to the first entry in Morton order, and every operation is a
 * single rounding in the order written, so the same specification evaluated
 * elsewhere gives the same bits.  The cell then keeps b if its particles'
 * radius about b is below that about the midpoint (squared radii compared),
 * else the midpoint. */
#ifndef OR_FW_ITERS
#define OR_FW_ITERS 16
#endif
#ifndef OR_FW_TOL
#define OR_FW_TOL 2e-3
#endif

typedef struct { double x[3], R; } sphere_t;

static double dist2(const double *a, const double *b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* the point q of the set farthest from c (first on ties) and D2 = |q - c|^2.
 * Particles (R = 0 throughout) are compared by squared distance and q is the
 * particle itself; spheres by d + R, with D2 = (d + R)^2. */
static void farthest(const sphere_t *S, int64_t n, int points, const double *c, double *q,
                     double *D2) {
    int64_t jmax = 0;
    if (points) {
        double best = -1.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d2 = dist2(S[j].x, c);
            if (d2 > best) { best = d2; jmax = j; }
        }
        for (int d = 0; d < 3; ++d) q[d] = S[jmax].x[d];
        *D2 = best;
        return;
    }
    double emax = -1.0, dmax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double d = sqrt(dist2(S[j].x, c));
        const double e = d + S[j].R;
        if (e > emax) { emax = e; dmax = d; jmax = j; }
    }
    const sphere_t *s = &S[jmax];
    if (dmax > 0.0) {
        const double u = s->R / dmax;
        for (int d = 0; d < 3; ++d) q[d] = s->x[d] + (s->x[d] - c[d]) * u;
    } else {
        q[0] = s->x[0] + s->R; q[1] = s->x[1]; q[2] = s->x[2];
    }
    *D2 = emax * emax;
}

/* the iteration over n >= 1 particles or spheres from the midpoint mid;
 * returns R (the largest distance, or d + R, from the final c), c set */
static double fw_enclosing(const sphere_t *S, int64_t n, int points, const double *mid,
                           double *c) {
    double a[3], b[3], q[3], D2;
    farthest(S, n, points, mid, a, &D2);
    farthest(S, n, points, a, b, &D2);
    for (int d = 0; d < 3; ++d) c[d] = (a[d] + b[d]) * 0.5;
    double gamma = dist2(a, b) * 0.25;
    for (int k = 0; k < OR_FW_ITERS; ++k) {
        farthest(S, n, points, c, q, &D2);
        if (!(gamma > 0.0)) break;
        const double delta = D2 / gamma - 1.0;
        if (!(delta > OR_FW_TOL)) break;
        const double lambda = delta / (2.0 * (1.0 + delta));
        for (int d = 0; d < 3; ++d) c[d] = c[d] + lambda * (q[d] - c[d]);
        const double om = 1.0 - lambda;
        gamma = om * gamma + (lambda * om) * D2;
    }
    if (points) {
        double m2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d2 = dist2(S[j].x, c);
            if (d2 > m2) m2 = d2;
        }
        return sqrt(m2);
    }
    double R = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double e = sqrt(dist2(S[j].x, c)) + S[j].R;
        if (e > R) R = e;
    }
    return R;
}

/* candidate (b, R) of cell C from its particles or grand-daughters, then the
 * choice between b and the midpoint; cells must be visited children first */
static int cell_enclosing(fmm_t *t, cell_t *C) {
    int64_t n = 0;
    sphere_t *S;
    if (is_leaf(C)) {
        n = C->end - C->begin;
        S = (sphere_t *)malloc(sizeof(sphere_t) * (size_t)n);
        if (!S) return -1;
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) S[i].x[d] = t->x[3 * (C->begin + i) + d];
            S[i].R = 0.0;
        }
    } else {
        S = (sphere_t *)malloc(sizeof(sphere_t) * 64);
        if (!S) return -1;
        for (int i = 0; i < C->nchild; ++i) {
            const cell_t *D = &t->cells[C->child[i]];
            const int nd = is_leaf(D) ? 1 : D->nchild;
            for (int j = 0; j < nd; ++j) {
                const cell_t *E = is_leaf(D) ? D : &t->cells[D->child[j]];
                for (int d = 0; d < 3; ++d) S[n].x[d] = E->bc[d];
                S[n].R = E->bR;
                ++n;
            }
        }
    }
    double c[3];
    C->bR = fw_enclosing(S, n, is_leaf(C), C->c, c);
    free(S);
    for (int d = 0; d < 3; ++d) C->bc[d] = c[d];
    double r2b = 0.0, r2m = 0.0;
    for (int64_t i = C->begin; i < C->end; ++i) {
        const double *x = &t->x[3 * i];
        const double eb = dist2(x, c), em = dist2(x, C->c);
        if (eb > r2b) r2b = eb;
        if (em > r2m) r2m = em;
    }
    if (r2b < r2m) {
        for (int d = 0; d < 3; ++d) C->c[d] = c[d];
        C->rho = sqrt(r2b);
    }
    return 0;
}

/* ------------------------------------------------------------ direct sums */

/* jerk (not NULL): also the time derivative of each pair's acceleration */
static void p2p(fmm_t *t, const cell_t *A, const cell_t *B, double *pot, double *acc,
                double *jerk, int64_t *count) {
    for (int64_t b = B->begin; b < B->end; ++b) {
        const double *xb = &t->x[3 * b];
        for (int64_t a = A->begin; a < A->end; ++a) {
            if (a == b) continue;
            const double dx = t->x[3 * a] - xb[0], dy = t->x[3 * a + 1] - xb[1],
                         dz = t->x[3 * a + 2] - xb[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = 1.0 / sqrt(r2);
            const double q = t->m[a] * ir, q3 = q * ir * ir;
            if (pot) pot[b] += q;
            acc[3 * b] += q3 * dx; acc[3 * b + 1] += q3 * dy; acc[3 * b + 2] += q3 * dz;
            if (jerk) {
                const double *va = &t->v[3 * a], *vb = &t->v[3 * b];
                const double vx = va[0] - vb[0], vy = va[1] - vb[1], vz = va[2] - vb[2];
                const double rv = (dx * vx + dy * vy + dz * vz) * ir * ir;
                jerk[3 * b] += q3 * (vx - 3.0 * rv * dx);
                jerk[3 * b + 1] += q3 * (vy - 3.0 * rv * dy);
                jerk[3 * b + 2] += q3 * (vz - 3.0 * rv * dz);
            }
            ++*count;
        }
    }
}

static void p2p_f(fmm_t *t, const cell_t *A, const cell_t *B, double *f, int64_t *count) {
    for (int64_t b = B->begin; b < B->end; ++b)
        for (int64_t a = A->begin; a < A->end; ++a) {
            if (a == b) continue;
            const double dx = t->x[3 * a] - t->x[3 * b], dy = t->x[3 * a + 1] - t->x[3 * b + 1],
                         dz = t->x[3 * a + 2] - t->x[3 * b + 2];
            f[b] += t->m[a] / (dx * dx + dy * dy + dz * dz);
            ++*count;
        }
}

/* ------------------------------------------- estimate of the sink scale */

static int64_t split_choice(const cell_t *A, const cell_t *B, double rA, double rB) {
    /* returns 0 to split A, 1 to split B: the larger cell, B on a tie, never a leaf */
    if (is_leaf(A)) return 1;
    if (is_leaf(B)) return 0;
    return rA > rB ? 0 : 1;
}

static void est_walk(fmm_t *t, int64_t ia, int64_t ib) {
    const cell_t *A = &t->cells[ia], *B = &t->cells[ib];
    const int want_f = t->prm->mac == OR_MAC_F;
    if (ia == ib) {
        if (is_leaf(A)) {
            if (want_f) p2p_f(t, A, A, t->est_f, &t->st->n_est_p2p_pairs);
            else p2p(t, A, A, NULL, t->est_acc, NULL, &t->st->n_est_p2p_pairs);
        } else {
            for (int i = 0; i < A->nchild; ++i)
                for (int j = 0; j < A->nchild; ++j) est_walk(t, A->child[i], A->child[j]);
        }
        return;
    }
    const double d[3] = {B->com[0] - A->com[0], B->com[1] - A->com[1], B->com[2] - A->com[2]};
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (A->rho_com + B->rho_com < r) {
        ++t->st->n_est_m2l;
        if (want_f) t->cells[ib].fe += A->mass / (r * r);
        else or_m2l(A->Me, d, 1, t->cells[ib].Fe);
        return;
    }
    if (is_leaf(A) && is_leaf(B)) {
        if (want_f) p2p_f(t, A, B, t->est_f, &t->st->n_est_p2p_pairs);
        else p2p(t, A, B, NULL, t->est_acc, NULL, &t->st->n_est_p2p_pairs);
        return;
    }
    if (split_choice(A, B, A->rho_com, B->rho_com) == 0) {
        for (int i = 0; i < A->nchild; ++i) est_walk(t, t->cells[ia].child[i], ib);
    } else {
        for (int j = 0; j < B->nchild; ++j) est_walk(t, ia, t->cells[ib].child[j]);
    }
}

static void est_up(fmm_t *t, int64_t ic) {
    cell_t *C = &t->cells[ic];
    if (is_leaf(C)) {
        or_p2m(C->end - C->begin, &t->x[3 * C->begin], &t->m[C->begin], C->com, 1, C->Me);
        return;
    }
    for (int i = 0; i < C->nchild; ++i) {
        est_up(t, C->child[i]);
        const cell_t *D = &t->cells[C->child[i]];
        const double d[3] = {D->com[0] - C->com[0], D->com[1] - C->com[1], D->com[2] - C->com[2]};
        or_m2m(D->Me, d, 1, C->Me);
    }
}

static void est_down(fmm_t *t, int64_t ic) {
    cell_t *C = &t->cells[ic];
    const int want_f = t->prm->mac == OR_MAC_F;
    if (is_leaf(C)) {
        for (int64_t b = C->begin; b < C->end; ++b) {
            if (want_f) { t->est_f[b] += C->fe; continue; }
            const double d[3] = {C->com[0] - t->x[3 * b], C->com[1] - t->x[3 * b + 1],
                                 C->com[2] - t->x[3 * b + 2]};
            double psi, a[3];
            or_l2p(C->Fe, d, 1, &psi, a);
            for (int k = 0; k < 3; ++k) t->est_acc[3 * b + k] += a[k];
        }
        return;
    }
    for (int i = 0; i < C->nchild; ++i) {
        cell_t *D = &t->cells[C->child[i]];
        if (want_f) {
            D->fe += C->fe;
        } else {
            const double d[3] = {C->com[0] - D->com[0], C->com[1] - D->com[1], C->com[2] - D->com[2]};
            or_l2l(C->Fe, d, 1, D->Fe);
        }
        est_down(t, C->child[i]);
    }
}

/* ----------------------------------------------------------- main pass */

static void up(fmm_t *t, int64_t ic) {
    cell_t *C = &t->cells[ic];
    if (is_leaf(C)) {
        or_p2m(C->end - C->begin, &t->x[3 * C->begin], &t->m[C->begin], C->c, t->p, C->M);
        if (t->v)   /* eq:P2M:dot */
            or_p2m_dot(C->end - C->begin, &t->x[3 * C->begin], &t->v[3 * C->begin],
                       &t->m[C->begin], C->c, t->p, C->Md);
    } else {
        for (int i = 0; i < C->nchild; ++i) {
            up(t, C->child[i]);
            const cell_t *D = &t->cells[C->child[i]];
            const double d[3] = {D->c[0] - C->c[0], D->c[1] - C->c[1], D->c[2] - C->c[2]};
            or_m2m(D->M, d, t->p, C->M);
            if (t->v) or_m2m(D->Md, d, t->p, C->Md);   /* centres at rest */
        }
    }
    or_power(C->M, t->p, C->P);
}

static void record(int64_t *buf, int64_t cap, int64_t *cnt, const cell_t *A, const cell_t *B) {
    if (buf && *cnt < cap) { buf[2 * *cnt] = cell_id(A); buf[2 * *cnt + 1] = cell_id(B); }
    ++*cnt;
}

/* the criterion for an expansion of order `order` (E_{A->B} of eq:def:EAB at
 * that order) */
static int accept_order(fmm_t *t, const cell_t *A, const cell_t *B, const double d[3], int order) {
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const or_fmm_params *q = t->prm;
    if (q->mac == OR_MAC_THETA) return A->rho + B->rho < q->theta_crit * r;
    if (!(A->rho + B->rho < r)) return 0;                        /* theta < 1 */
    const double err = or_etilde_factor(A->rho, B->rho) * or_eab_times_mass(A->P, order, B->rho, r)
                       / (r * r);                                /* Etilde M_A / r^2 */
    /* individual eps_b are already folded into smin = min_B{eps_b a_b} (Sec. 7) */
    return err < (q->eps_particle ? 1.0 : q->eps) * B->smin;
}

static int accept(fmm_t *t, const cell_t *A, const cell_t *B, const double d[3]) {
    return accept_order(t, A, B, d, t->p);
}

static void walk(fmm_t *t, int64_t ia, int64_t ib) {
    const cell_t *A = &t->cells[ia], *B = &t->cells[ib];
    if (ia == ib) {
        if (is_leaf(A)) {
            p2p(t, A, A, t->pot, t->acc, t->jerk, &t->st->n_p2p_pairs);
            ++t->st->n_p2p_cells;
            record(t->lists ? t->lists->p2p : NULL, t->lists ? t->lists->p2p_cap : 0,
                   &t->np2p_rec, A, A);
        } else {
            for (int i = 0; i < A->nchild; ++i)
                for (int j = 0; j < A->nchild; ++j) walk(t, A->child[i], A->child[j]);
        }
        return;
    }
    const double d[3] = {B->c[0] - A->c[0], B->c[1] - A->c[1], B->c[2] - A->c[2]};
    const int ok = accept(t, A, B, d);
    if (ok && (double)(A->end - A->begin) * (double)(B->end - B->begin) >= t->prm->p2p_pairs) {
        /* adaptive order (Sec. 7): the lowest order in [q_min, p] that passes the
         * criterion, q_min = adaptive_order */
        int q = t->p;
        if (t->prm->adaptive_order > 0 && t->prm->mac != OR_MAC_THETA)
            for (q = t->prm->adaptive_order; q < t->p; ++q)
                if (accept_order(t, A, B, d, q)) break;
        or_m2l(A->M, d, q, t->cells[ib].F);
        if (t->v) or_m2l(A->Md, d, q, t->cells[ib].Fd);   /* eq:M2L:dot */
        ++t->st->n_m2l;
        t->st->m2l_order_sum += q;
        for (int n = 0; n <= q; ++n)
            t->st->m2l_macs += (int64_t)(n + 1) * (q - n + 1) * (q - n + 1);
        record(t->lists ? t->lists->m2l : NULL, t->lists ? t->lists->m2l_cap : 0,
               &t->nm2l_rec, A, B);
        return;
    }
    if (ok || (is_leaf(A) && is_leaf(B))) {
        p2p(t, A, B, t->pot, t->acc, t->jerk, &t->st->n_p2p_pairs);
        ++t->st->n_p2p_cells;
        record(t->lists ? t->lists->p2p : NULL, t->lists ? t->lists->p2p_cap : 0,
               &t->np2p_rec, A, B);
        return;
    }
    if (split_choice(A, B, A->rho, B->rho) == 0) {
        for (int i = 0; i < A->nchild; ++i) walk(t, t->cells[ia].child[i], ib);
    } else {
        for (int j = 0; j < B->nchild; ++j) walk(t, ia, t->cells[ib].child[j]);
    }
}

static void down(fmm_t *t, int64_t ic) {
    cell_t *C = &t->cells[ic];
    if (is_leaf(C)) {
        for (int64_t b = C->begin; b < C->end; ++b) {
            const double d[3] = {C->c[0] - t->x[3 * b], C->c[1] - t->x[3 * b + 1],
                                 C->c[2] - t->x[3 * b + 2]};
            double psi, a[3];
            or_l2p(C->F, d, t->p, &psi, a);
            t->pot[b] += psi;
            for (int k = 0; k < 3; ++k) t->acc[3 * b + k] += a[k];
            if (t->v) {   /* eq:L2P:dot */
                double j[3];
                or_l2p_dot(C->F, C->Fd, d, &t->v[3 * b], t->p, j);
                for (int k = 0; k < 3; ++k) t->jerk[3 * b + k] += j[k];
            }
        }
        return;
    }
    for (int i = 0; i < C->nchild; ++i) {
        cell_t *D = &t->cells[C->child[i]];
        const double d[3] = {C->c[0] - D->c[0], C->c[1] - D->c[1], C->c[2] - D->c[2]};
        or_l2l(C->F, d, t->p, D->F);
        if (t->v) or_l2l(C->Fd, d, t->p, D->Fd);   /* centres at rest */
        down(t, C->child[i]);
    }
}

static double subtree_min(fmm_t *t, int64_t ic) {
    cell_t *C = &t->cells[ic];
    double s = INFINITY;
    for (int64_t b = C->begin; b < C->end; ++b) s = fmin(s, t->scale[b]);
    C->smin = s;
    for (int i = 0; i < C->nchild; ++i) subtree_min(t, C->child[i]);
    return s;
}

/* ---------------------------------------------------------------- driver */

static void release(fmm_t *t) {
    for (int64_t i = 0; i < t->ncells; ++i) {
        free(t->cells[i].M); free(t->cells[i].F); free(t->cells[i].P);
        free(t->cells[i].Md); free(t->cells[i].Fd);
    }
    free(t->v); free(t->jerk);
    free(t->cells); free(t->x); free(t->m); free(t->orig); free(t->key); free(t->key2);
    free(t->pot); free(t->acc); free(t->est_acc); free(t->est_f); free(t->scale);
}

int or_fmm(const or_fmm_params *prm, int64_t n, const double *pos,
           const double *mass, double *pot, double *acc,
           or_fmm_stats *stats, or_fmm_lists *lists) {
    or_fmm_stats dummy;
    if (!stats) stats = &dummy;
    memset(stats, 0, sizeof(*stats));
    if (!prm || n < 0 || prm->p < 1 || prm->p > 30 || prm->leaf_size < 1) return -1;
    if (n == 0) return 0;
    if (!pos || !mass || !pot || !acc) return -1;
    if (prm->scale_source == OR_SCALE_GIVEN && prm->mac != OR_MAC_THETA && !prm->scale) return -1;
    if (prm->vel && !prm->jerk) return -1;

    fmm_t T; memset(&T, 0, sizeof(T));
    fmm_t *t = &T;
    t->prm = prm; t->n = n; t->p = prm->p; t->ncoef = (prm->p + 1) * (prm->p + 1);
    t->st = stats; t->lists = lists;

    /* 1. keys in the cube around the bounding box, sort, permute */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], pos[3 * i + d]); hi[d] = fmax(hi[d], pos[3 * i + d]); }
    double L = 0;
    for (int d = 0; d < 3; ++d) L = fmax(L, hi[d] - lo[d]);
    const double scale = L > 0 ? 2097152.0 / L : 0.0;   /* 2^21 cells per axis */
    for (int d = 0; d < 3; ++d) t->lo[d] = lo[d];
    t->kscale = scale;
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * (size_t)n);
    t->x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    t->m = (double *)malloc(sizeof(double) * (size_t)n);
    t->orig = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    t->key2 = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    t->pot = (double *)calloc((size_t)n, sizeof(double));
    t->acc = (double *)calloc(3 * (size_t)n, sizeof(double));
    t->est_acc = (double *)calloc(3 * (size_t)n, sizeof(double));
    t->est_f = (double *)calloc((size_t)n, sizeof(double));
    t->scale = (double *)malloc(sizeof(double) * (size_t)n);
    if (!ki || !t->x || !t->m || !t->orig || !t->key || !t->key2 || !t->pot || !t->acc || !t->est_acc ||
        !t->est_f || !t->scale) { free(ki); release(t); return -2; }
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            const double u = (pos[3 * i + d] - lo[d]) * scale;
            q[d] = u >= 2097151.0 ? 2097151u : (uint32_t)u;
        }
        ki[i].key = morton(q[0], q[1], q[2]);
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = ki[i].idx;
        t->orig[i] = j; t->key[i] = ki[i].key; t->m[i] = mass[j];
        for (int d = 0; d < 3; ++d) t->x[3 * i + d] = pos[3 * j + d];
    }
    free(ki);

    /* octree */
    if (build(t, 0, n, 0, -1) < 0 || t->oom) { release(t); return -2; }
    for (int64_t i = 0; i < t->ncells; ++i) {
        cell_t *C = &t->cells[i];
        cell_geometry(t, C);
        C->M = (double complex *)calloc((size_t)t->ncoef, sizeof(double complex));
        C->F = (double complex *)calloc((size_t)t->ncoef, sizeof(double complex));
        C->P = (double *)calloc((size_t)t->p + 1, sizeof(double));
        if (!C->M || !C->F || !C->P) { release(t); return -2; }
        if (prm->vel) {
            C->Md = (double complex *)calloc((size_t)t->ncoef, sizeof(double complex));
            C->Fd = (double complex *)calloc((size_t)t->ncoef, sizeof(double complex));
            if (!C->Md || !C->Fd) { release(t); return -2; }
        }
        if (is_leaf(C)) ++stats->n_leaves;
        if (C->level > stats->depth) stats->depth = C->level;
    }
    stats->n_cells = t->ncells;
    if (prm->centre == OR_CENTRE_ENCLOSING)   /* children have larger indices */
        for (int64_t i = t->ncells - 1; i >= 0; --i)
            if (cell_enclosing(t, &t->cells[i]) < 0) { release(t); return -2; }
    if (lists && lists->order)
        for (int64_t i = 0; i < n; ++i) lists->order[i] = t->orig[i];
    if (lists && lists->cell_ids) {
        lists->cell_count = t->ncells;
        for (int64_t i = 0; i < t->ncells && i < lists->cell_cap; ++i) {
            const cell_t *C = &t->cells[i];
            lists->cell_ids[2 * i] = cell_id(C);
            lists->cell_ids[2 * i + 1] = C->end;
            double *g = &lists->cell_geo[5 * i];
            g[0] = C->c[0]; g[1] = C->c[1]; g[2] = C->c[2]; g[3] = C->rho; g[4] = C->rho_mid;
        }
    }
    if (prm->vel) {   /* velocities in the final particle order */
        t->v = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        t->jerk = (double *)calloc(3 * (size_t)n, sizeof(double));
        if (!t->v || !t->jerk) { release(t); return -2; }
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) t->v[3 * i + d] = prm->vel[3 * t->orig[i] + d];
    }

    /* 2. sink scale */
    if (prm->mac != OR_MAC_THETA) {
        if (prm->scale_source == OR_SCALE_GIVEN) {
            for (int64_t i = 0; i < n; ++i) t->scale[i] = prm->scale[t->orig[i]];
        } else {
            est_up(t, 0);
            est_walk(t, 0, 0);
            est_down(t, 0);
            for (int64_t i = 0; i < n; ++i) {
                const double *a = &t->est_acc[3 * i];
                t->scale[i] = prm->mac == OR_MAC_F ? t->est_f[i]
                                                   : sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            }
        }
        if (prm->eps_particle)               /* min_B{eps_b a_b} (Sec. 7) */
            for (int64_t i = 0; i < n; ++i) t->scale[i] *= prm->eps_particle[t->orig[i]];
        if (lists && lists->scale_est)
            for (int64_t i = 0; i < n; ++i) lists->scale_est[t->orig[i]] = t->scale[i];
        subtree_min(t, 0);
    }

    /* 3-5. upward pass, walk, downward pass */
    up(t, 0);
    walk(t, 0, 0);
    down(t, 0);
    if (lists) { lists->m2l_count = t->nm2l_rec; lists->p2p_count = t->np2p_rec; }

    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = t->orig[i];
        pot[j] = -prm->G * t->pot[i];
        for (int d = 0; d < 3; ++d) acc[3 * j + d] = prm->G * t->acc[3 * i + d];
        if (t->v)
            for (int d = 0; d < 3; ++d) prm->jerk[3 * j + d] = prm->G * t->jerk[3 * i + d];
    }
    release(t);
    return 0;
}
