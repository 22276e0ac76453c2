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
