/* Oracle: complex solid harmonics and the FMM kernels (test infrastructure).
 *
 * Written in the paper's complex notation with every m from -n to n stored,
 * so each kernel is its equation typed out as nested sums: no symmetry
 * folding, no real-valued basis, no blocking.
 *
 * Harmonics (Sec. 2.1 eqs:Ups:The; App. A.3 eq:The:def, eq:Ups:def; App. A.5):
 *   Theta_0^0 = 1/r,   Theta_n^n = (2n-1) (x+iy)/r^2 Theta_{n-1}^{n-1}   (eq:The:nn)
 *   r^2 Theta_n^m = (2n-1) z Theta_{n-1}^m - ((n-1)^2 - m^2) Theta_{n-2}^m
 *   Upsilon_0^0 = 1,   Upsilon_n^n = (x+iy)/(2n) Upsilon_{n-1}^{n-1}
 *   (n^2 - m^2) Upsilon_n^m = (2n-1) z Upsilon_{n-1}^m - r^2 Upsilon_{n-2}^m (eq:Ups:rec)
 *   negative m from the symmetry X_n^{-m} = (-1)^m conj(X_n^m)        (eq:sym)
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>

static double complex get(const double complex *X, int n, int m) {
    if (n < 0 || m > n || m < -n) return 0.0;
    return X[OR_IDX(n, m)];
}

static void fill_negative_m(double complex *X, int p) {
    for (int n = 1; n <= p; ++n)
        for (int m = 1; m <= n; ++m)
            X[OR_IDX(n, -m)] = ((m & 1) ? -1.0 : 1.0) * conj(X[OR_IDX(n, m)]);
}

void or_theta(const double r[3], int p, double complex *T) {
    const double x = r[0], y = r[1], z = r[2];
    const double r2 = x * x + y * y + z * z;
    const double complex w = x + I * y;
    T[OR_IDX(0, 0)] = 1.0 / sqrt(r2);
    for (int n = 1; n <= p; ++n)
        T[OR_IDX(n, n)] = (2.0 * n - 1.0) * w / r2 * T[OR_IDX(n - 1, n - 1)];
    for (int m = 0; m <= p; ++m)
        for (int n = m + 1; n <= p; ++n)
            T[OR_IDX(n, m)] = ((2.0 * n - 1.0) * z * get(T, n - 1, m)
                               - ((double)(n - 1) * (n - 1) - (double)m * m) * get(T, n - 2, m))
                              / r2;
    fill_negative_m(T, p);
}

void or_upsilon(const double r[3], int p, double complex *U) {
    const double x = r[0], y = r[1], z = r[2];
    const double r2 = x * x + y * y + z * z;
    const double complex w = x + I * y;
    U[OR_IDX(0, 0)] = 1.0;
    for (int n = 1; n <= p; ++n)
        U[OR_IDX(n, n)] = w / (2.0 * n) * U[OR_IDX(n - 1, n - 1)];
    for (int m = 0; m <= p; ++m)
        for (int n = m + 1; n <= p; ++n)
            U[OR_IDX(n, m)] = ((2.0 * n - 1.0) * z * get(U, n - 1, m) - r2 * get(U, n - 2, m))
                              / ((double)n * n - (double)m * m);
    fill_negative_m(U, p);
}

static double complex *scratch(int p) {
    return (double complex *)malloc(sizeof(double complex) * (size_t)(p + 1) * (p + 1));
}

/* eq:P2M */
void or_p2m(int64_t n, const double *pos, const double *mass,
            const double z[3], int p, double complex *M) {
    double complex *U = scratch(p);
    for (int64_t a = 0; a < n; ++a) {
        const double d[3] = {pos[3 * a] - z[0], pos[3 * a + 1] - z[1], pos[3 * a + 2] - z[2]};
        or_upsilon(d, p, U);
        for (int k = 0; k < (p + 1) * (p + 1); ++k) M[k] += mass[a] * U[k];
    }
    free(U);
}

/* eq:M2M: M_n^m(z') = sum_{k=0}^{n} sum_{l=-k}^{k} Upsilon_k^l(z - z') M_{n-k}^{m-l}(z) */
void or_m2m(const double complex *M, const double z_minus_zp[3], int p,
            double complex *Mout) {
    double complex *U = scratch(p);
    or_upsilon(z_minus_zp, p, U);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
            double complex s = 0.0;
            for (int k = 0; k <= n; ++k)
                for (int l = -k; l <= k; ++l)
                    s += get(U, k, l) * get(M, n - k, m - l);
            Mout[OR_IDX(n, m)] += s;
        }
    free(U);
}

/* eq:M2L: F_n^m(s_B) = sum_{k=0}^{p-n} sum_{l=-k}^{k} conj(M_k^l(z_A)) Theta_{n+k}^{m+l}(s_B - z_A) */
void or_m2l(const double complex *M, const double sB_minus_zA[3], int p,
            double complex *F) {
    double complex *T = scratch(p);
    or_theta(sB_minus_zA, p, T);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
            double complex s = 0.0;
            for (int k = 0; k <= p - n; ++k)
                for (int l = -k; l <= k; ++l)
                    s += conj(get(M, k, l)) * get(T, n + k, m + l);
            F[OR_IDX(n, m)] += s;
        }
    free(T);
}

/* eq:L2L: F_n^m(s') = sum_{k=0}^{p-n} sum_{l=-k}^{k} conj(Upsilon_k^l(s - s')) F_{n+k}^{m+l}(s) */
void or_l2l(const double complex *F, const double s_minus_sp[3], int p,
            double complex *Fout) {
    double complex *U = scratch(p);
    or_upsilon(s_minus_sp, p, U);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
            double complex s = 0.0;
            for (int k = 0; k <= p - n; ++k)
                for (int l = -k; l <= k; ++l)
                    s += conj(get(U, k, l)) * get(F, n + k, m + l);
            Fout[OR_IDX(n, m)] += s;
        }
    free(U);
}

/* eq:L2P with n = 0, 1; a = grad Psi_0^0 = -(Re Psi_1^1, Im Psi_1^1, Psi_1^0) */
void or_l2p(const double complex *F, const double sB_minus_x[3], int p,
            double *psi, double acc[3]) {
    double complex *U = scratch(p);
    or_upsilon(sB_minus_x, p, U);
    double complex Psi[2][3] = {{0}};
    for (int n = 0; n <= 1 && n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            double complex s = 0.0;
            for (int k = 0; k <= p - n; ++k)
                for (int l = -k; l <= k; ++l)
                    s += conj(get(U, k, l)) * get(F, n + k, m + l);
            Psi[n][m] = s;
        }
    free(U);
    *psi = creal(Psi[0][0]);
    acc[0] = -creal(Psi[1][1]);
    acc[1] = -cimag(Psi[1][1]);
    acc[2] = -creal(Psi[1][0]);
}

/* Time derivatives (App. A.5).  In xi = (x+iy)/2, eta = -(x-iy)/2 and z
 * (eq:xi:eta) the first derivatives of the regular harmonics follow from
 * eq:dUnm with the first-order operators d/dxi (Delta_1^{-1}), d/deta
 * (Delta_1^1) and -d/dz (Delta_1^0):
 *   d/dxi Upsilon_n^m = Upsilon_{n-1}^{m-1},  d/deta Upsilon_n^m = Upsilon_{n-1}^{m+1},
 *   d/dz Upsilon_n^m = Upsilon_{n-1}^m,
 * and the chain rule gives d/dt = xidot d/dxi + etadot d/deta + zdot d/dz.
 * Upsilon_1^1 = xi, whose derivative is xidot, fixes this pairing of xidot
 * with m-1 (the relation as printed pairs xidot with m+1). */
void or_upsilon_dot(const double r[3], const double v[3], int p, double complex *Ud) {
    double complex *U = scratch(p);
    or_upsilon(r, p, U);
    const double complex xid = 0.5 * (v[0] + I * v[1]);
    const double complex etad = -0.5 * (v[0] - I * v[1]);
    Ud[OR_IDX(0, 0)] = 0.0;
    for (int n = 1; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            Ud[OR_IDX(n, m)] = xid * get(U, n - 1, m - 1) + v[2] * get(U, n - 1, m)
                               + etad * get(U, n - 1, m + 1);
    free(U);
}

/* eq:P2M:dot */
void or_p2m_dot(int64_t n, const double *pos, const double *vel, const double *mass,
                const double z[3], int p, double complex *Md) {
    double complex *Ud = scratch(p);
    for (int64_t a = 0; a < n; ++a) {
        const double d[3] = {pos[3 * a] - z[0], pos[3 * a + 1] - z[1], pos[3 * a + 2] - z[2]};
        or_upsilon_dot(d, &vel[3 * a], p, Ud);
        for (int k = 0; k < (p + 1) * (p + 1); ++k) Md[k] += mass[a] * Ud[k];
    }
    free(Ud);
}

/* eq:L2P:dot with n = 1: s_B is at rest, so d/dt (s_B - x) = -v */
void or_l2p_dot(const double complex *F, const double complex *Fd, const double sB_minus_x[3],
                const double v[3], int p, double jerk[3]) {
    double complex *U = scratch(p), *Ud = scratch(p);
    const double mv[3] = {-v[0], -v[1], -v[2]};
    or_upsilon(sB_minus_x, p, U);
    or_upsilon_dot(sB_minus_x, mv, p, Ud);
    double complex Psid[2] = {0.0, 0.0};
    for (int m = 0; m <= 1; ++m) {
        double complex s = 0.0;
        for (int k = 0; k <= p - 1; ++k)
            for (int l = -k; l <= k; ++l)
                s += conj(get(U, k, l)) * get(Fd, 1 + k, m + l)
                     + conj(get(Ud, k, l)) * get(F, 1 + k, m + l);
        Psid[m] = s;
    }
    free(U);
    free(Ud);
    jerk[0] = -creal(Psid[1]);
    jerk[1] = -cimag(Psid[1]);
    jerk[2] = -creal(Psid[0]);
}

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* eq:def:PA */
void or_power(const double complex *M, int p, double *P) {
    for (int n = 0; n <= p; ++n) {
        double s = 0.0;
        for (int m = -n; m <= n; ++m) {
            const double complex v = M[OR_IDX(n, m)];
            s += factorial(n - m) * factorial(n + m) * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
        P[n] = sqrt(s);
    }
}

static double binom(int p, int k) {
    return factorial(p) / (factorial(k) * factorial(p - k));
}

/* eq:def:EAB multiplied by M_A:  sum_{k=0}^{p} C(p,k) P_{k,A} rho_{s,B}^{p-k} / r^p */
double or_eab_times_mass(const double *P, int p, double rho_sB, double r) {
    double s = 0.0;
    for (int k = 0; k <= p; ++k) s += binom(p, k) * P[k] * pow(rho_sB, p - k);
    return s / pow(r, p);
}

/* eq:err:tilde prefactor; when both radii vanish the ratio is taken at its
 * largest value, 8 (the limit as one radius goes to zero). */
double or_etilde_factor(double rho_zA, double rho_sB) {
    const double sum = rho_zA + rho_sB;
    if (!(sum > 0.0)) return 8.0;
    return 8.0 * fmax(rho_zA, rho_sB) / sum;
}

/* Swap matrix B_n for exchanging the x and z axes (App. A, fast rotations,
 * eq:Ylm:swap): Theta_n^m(z, y, x) = sum_l B_n^{ml} Theta_n^l(x, y, z).
 * Built from B_0 = 1 by the recurrences given there, read as: rows |m| <= n-1
 * of B_n from 2 B_n^{ml} = B_{n-1}^{m,l-1} - B_{n-1}^{m,l+1}, and the two new
 * rows m = +-n from 2 B_n^{+-n,l} = B_{n-1}^{+-(n-1),l-1} + B_{n-1}^{+-(n-1),l+1}
 * +- 2 B_{n-1}^{+-(n-1),l}; entries with |l| > n-1 of B_{n-1} are zero.
 * Output: (2n+1)^2 doubles, row m = -n..n, column l = -n..n, row-major. */
void or_swap_matrix(int n, double *B) {
    double *prev = (double *)malloc(sizeof(double) * (size_t)(2 * n + 1) * (2 * n + 1));
    double *cur = (double *)malloc(sizeof(double) * (size_t)(2 * n + 1) * (2 * n + 1));
    cur[0] = 1.0;                                  /* B_0 */
    for (int k = 0; k < n; ++k) {                  /* B_k (in cur) -> B_{k+1} */
        const int w = 2 * k + 1, W = 2 * k + 3;
        for (int i = 0; i < w * w; ++i) prev[i] = cur[i];
#define PB(m, l) (((m) < -k || (m) > k || (l) < -k || (l) > k) ? 0.0 : prev[((m) + k) * w + (l) + k])
        for (int m = -(k + 1); m <= k + 1; ++m)
            for (int l = -(k + 1); l <= k + 1; ++l) {
                double v;
                if (m >= -k && m <= k)
                    v = 0.5 * (PB(m, l - 1) - PB(m, l + 1));
                else if (m == k + 1)
                    v = 0.5 * (PB(k, l - 1) + PB(k, l + 1) + 2.0 * PB(k, l));
                else
                    v = 0.5 * (PB(-k, l - 1) + PB(-k, l + 1) - 2.0 * PB(-k, l));
                cur[(m + k + 1) * W + l + k + 1] = v;
            }
#undef PB
    }
    for (int i = 0; i < (2 * n + 1) * (2 * n + 1); ++i) B[i] = cur[i];
    free(prev);
    free(cur);
}

/* X_n^m *= w^{-m} for every n <= p (a rotation of the frame about z by the
 * angle of the unit complex number w, eq:Ylm:rot:z) */
static void rot_z(double complex *X, int p, double complex w) {
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) X[OR_IDX(n, m)] *= cpow(w, -m);
}

/* X_n <- B_n X_n (Theta-type coefficients) or B_n^T X_n (Upsilon-type: the
 * swap matrices of Upsilon_n^m are the transposes), every degree n <= p */
static void swap_xz(double complex *X, int p, int transpose) {
    double complex *y = (double complex *)malloc(sizeof(double complex) * (size_t)(2 * p + 1));
    double *B = (double *)malloc(sizeof(double) * (size_t)(2 * p + 1) * (2 * p + 1));
    for (int n = 0; n <= p; ++n) {
        const int w = 2 * n + 1;
        or_swap_matrix(n, B);
        for (int m = -n; m <= n; ++m) {
            double complex s = 0.0;
            for (int l = -n; l <= n; ++l)
                s += (transpose ? B[(l + n) * w + m + n] : B[(m + n) * w + l + n]) *
                     X[OR_IDX(n, l)];
            y[m + n] = s;
        }
        for (int m = -n; m <= n; ++m) X[OR_IDX(n, m)] = y[m + n];
    }
    free(y);
    free(B);
}

/* The rotation-accelerated M2L of App. A (a fast M2L kernel), same result as
 * or_m2l up to rounding.  With r = (x, y, z) = s_B - z_A, rho = |(x, y)|:
 * rotate the multipoles about z so that r lies in the y-z plane (angle
 * phi - pi/2, phi the azimuth of r), swap x and z, rotate about the new z axis
 * by atan2(rho, z) so that r lies on the (swapped) x axis, swap back: r is now
 * along +z.  Apply the z-axis kernel eq:M2L:z
 *     Ft_n^m = sum_{k=|m|}^{p-n} (-1)^m Mt_k^m (n+k)! / r^{n+k+1},
 * then undo the rotations in reverse order and add to F. */
void or_m2l_rot(const double complex *M, const double r3[3], int p, double complex *F) {
    const int nc = (p + 1) * (p + 1);
    double complex *X = (double complex *)malloc(sizeof(double complex) * (size_t)nc);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nc);
    const double x = r3[0], y = r3[1], z = r3[2];
    const double rho = sqrt(x * x + y * y), r = sqrt(x * x + y * y + z * z);
    /* e^{i alpha} with alpha = phi - pi/2; any angle when r is on the z axis */
    const double complex wa = rho > 0.0 ? (x + I * y) / rho * (-I) : 1.0;
    const double complex wb = (z + I * rho) / r;   /* e^{i beta}, beta = atan2(rho, z) */
    for (int i = 0; i < nc; ++i) X[i] = M[i];
    rot_z(X, p, wa);
    swap_xz(X, p, 1);
    rot_z(X, p, wb);
    swap_xz(X, p, 1);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
            double complex s = 0.0;
            if (abs(m) <= p - n)
                for (int k = abs(m); k <= p - n; ++k)
                    s += ((m & 1) ? -1.0 : 1.0) * X[OR_IDX(k, m)] * factorial(n + k) /
                         pow(r, n + k + 1);
            Y[OR_IDX(n, m)] = s;
        }
    swap_xz(Y, p, 0);
    rot_z(Y, p, 1.0 / wb);
    swap_xz(Y, p, 0);
    rot_z(Y, p, 1.0 / wa);
    for (int i = 0; i < nc; ++i) F[i] += Y[i];
    free(X);
    free(Y);
}
