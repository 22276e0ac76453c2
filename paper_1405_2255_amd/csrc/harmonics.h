// Solid harmonics on the device, generated one degree ("row") at a time.
//
// Theta_n^m (irregular) and Upsilon_n^m (regular) of Sec. 2.1 are produced by
// the recurrences of App. A.5 (eq:The:nn, eq:Ups:rec and the companion
// recurrence for Theta) for 0 <= m <= n; the m < 0 half follows from
// X_n^{-m} = (-1)^m conj(X_n^m) (eq:sym) and is never stored.  A row n only
// needs rows n-1 and n-2, so a generator keeps two rows of P+1 complex
// numbers in registers: row n overwrites row n-2 in place (entry m of row n
// reads entry m of rows n-1 and n-2 only).
#pragma once

#include "dev.h"

namespace fmm {

__host__ __device__ constexpr int tri(int n, int m) { return n * (n + 1) / 2 + m; }

// rows[2][P+1]: row n lives in rows[n & 1].
template <int P>
struct RowGen {
    cplx rows[2][P + 1];
    double x, y, z, r2, ir2;

    // Theta: start with Theta_0^0 = 1/r.
    __device__ __forceinline__ void theta_start(double dx, double dy, double dz) {
        x = dx; y = dy; z = dz;
        r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double rinv = rsqrt_nr(r2);
        ir2 = rinv * rinv;
        rows[0][0] = {rinv, 0.0};
    }
    // Theta row n >= 1 from rows n-1, n-2:
    //   Theta_n^n = (2n-1) (x+iy)/r^2 Theta_{n-1}^{n-1}
    //   r^2 Theta_n^m = (2n-1) z Theta_{n-1}^m - ((n-1)^2 - m^2) Theta_{n-2}^m
    template <int N>
    __device__ __forceinline__ void theta_row() {
        cplx *cur = rows[N & 1];
        const cplx *prv = rows[(N - 1) & 1];
        const double a = (2.0 * N - 1.0);
#pragma unroll
        for (int m = 0; m <= N - 2; ++m) {
            const double b = (double)((N - 1) * (N - 1) - m * m);
            const double s = a * z;
            cur[m].re = (s * prv[m].re - b * cur[m].re) * ir2;
            cur[m].im = (m == 0) ? 0.0 : (s * prv[m].im - b * cur[m].im) * ir2;
        }
        const cplx t = prv[N - 1];
        cur[N - 1].re = a * z * t.re * ir2;
        cur[N - 1].im = (N - 1 == 0) ? 0.0 : a * z * t.im * ir2;
        const double f = a * ir2;
        cur[N] = {f * (x * t.re - y * t.im), f * (x * t.im + y * t.re)};
    }

    // Upsilon: start with Upsilon_0^0 = 1.
    __device__ __forceinline__ void upsilon_start(double dx, double dy, double dz) {
        x = dx; y = dy; z = dz;
        r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        rows[0][0] = {1.0, 0.0};
    }
    // Upsilon row n >= 1:
    //   Upsilon_n^n = (x+iy)/(2n) Upsilon_{n-1}^{n-1}
    //   (n^2 - m^2) Upsilon_n^m = (2n-1) z Upsilon_{n-1}^m - r^2 Upsilon_{n-2}^m
    template <int N>
    __device__ __forceinline__ void upsilon_row() {
        cplx *cur = rows[N & 1];
        const cplx *prv = rows[(N - 1) & 1];
        const double a = (2.0 * N - 1.0);
#pragma unroll
        for (int m = 0; m <= N - 2; ++m) {
            const double inv = 1.0 / (double)(N * N - m * m);
            const double s = a * z;
            cur[m].re = (s * prv[m].re - r2 * cur[m].re) * inv;
            cur[m].im = (m == 0) ? 0.0 : (s * prv[m].im - r2 * cur[m].im) * inv;
        }
        const cplx t = prv[N - 1];          // Upsilon_n^{n-1} = z Upsilon_{n-1}^{n-1}
        cur[N - 1].re = z * t.re;
        cur[N - 1].im = (N - 1 == 0) ? 0.0 : z * t.im;
        const double h = 1.0 / (2.0 * N);
        cur[N] = {h * (x * t.re - y * t.im), h * (x * t.im + y * t.re)};
    }

    template <int N>
    __device__ __forceinline__ const cplx *row() const { return rows[N & 1]; }
};

// Signed access to the m < 0 half of a stored row: value of X_n^{q} for any
// q with |q| <= n, from the stored entry X_n^{|q|}.
__device__ __forceinline__ cplx sym(cplx v, int q) {
    if (q >= 0) return v;
    return (q & 1) ? cplx{-v.re, v.im} : cplx{v.re, -v.im};
}

// Compile-time loop helper: calls f(std::integral_constant-like) for I in [B, E].
template <int B, int E>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F &&f) {
        if constexpr (B <= E) {
            f.template operator()<B>();
            Unroll<B + 1, E>::run(f);
        }
    }
};

}  // namespace fmm
