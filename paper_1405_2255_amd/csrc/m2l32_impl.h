// Mixed-precision M2L (FP32 arithmetic on scaled quantities), included by the
// per-order translation units next to the FP64 kernel.
//
// Scaling.  With r = |s_B - z_A| and r^ = (s_B - z_A)/r, homogeneity of the
// irregular harmonics (Theta_j(r) = Theta_j(r^) / r^{j+1}) turns eq:M2L into
//   F_n = sum_A r^{-(n+1)} sum_k Theta_{n+k}(r^) (s_A/r)^k Mh_k,
// with Mh_k = M_k / s_A^k (s_A = rho_A, or 1 for a point cell).  A chunk of
// one sink accumulates Fh_n = sigma^{n+1} F_n with sigma = the smallest r of
// the chunk, so each source enters with the factors (s_A/r)^k (sigma/r)^{n+1},
// both at most 1: nothing overflows in FP32 at any tree extent, and what
// underflows is far below the FP32 rounding of the leading terms.  The chunk
// reduction restores F_n = Fh_n sigma^{-(n+1)} in FP64.
//
// Split by degree.  The terms of the lowest degrees j = n + k <= M2L32_JLO
// (monopole to octupole: the large terms, whose rounding would dominate
// where the far field of many cells nearly cancels) are evaluated in FP64
// without scaling, in a short separate pass; the FP32 passes add only the
// terms with j > M2L32_JLO, which are smaller by at least
// max(rho_A, rho_B)/r to the power M2L32_JLO + 1.
#pragma once

#include "m2l_impl.h"

namespace fmm {
namespace m2l32_detail {

struct cplxf {
    float re, im;
};

constexpr int FBUDGET32 = 48;   // complex FP32 accumulators per pass
constexpr int M2L32_JLO = FMM_M2L32_JLO;   // degrees evaluated in FP64

__host__ __device__ constexpr int pass_end32(int p, int n0) {
    int n = n0;
    while (n + 1 <= p && tri(n + 2, 0) - tri(n0, 0) <= FBUDGET32) ++n;
    return n;
}

// Theta at a unit vector, one degree at a time in FP32 (the recurrences of
// App. A.5 with r = 1).
template <int P>
struct UnitTheta32 {
    cplxf rows[2][P + 1];
    float x, y, z;
    __device__ __forceinline__ void start(float ux, float uy, float uz) {
        x = ux; y = uy; z = uz;
        rows[0][0] = {1.0f, 0.0f};
    }
    template <int N>
    __device__ __forceinline__ void next() {
        cplxf *cur = rows[N & 1];
        const cplxf *prv = rows[(N - 1) & 1];
        const float a = 2.0f * N - 1.0f;
#pragma unroll
        for (int m = 0; m <= N - 2; ++m) {
            const float b = (float)((N - 1) * (N - 1) - m * m);
            const float s = a * z;
            cur[m].re = s * prv[m].re - b * cur[m].re;
            cur[m].im = (m == 0) ? 0.0f : s * prv[m].im - b * cur[m].im;
        }
        const cplxf t = prv[N - 1];
        cur[N - 1].re = a * z * t.re;
        cur[N - 1].im = (N - 1 == 0) ? 0.0f : a * z * t.im;
        cur[N] = {a * (x * t.re - y * t.im), a * (x * t.im + y * t.re)};
    }
    template <int N>
    __device__ __forceinline__ const cplxf *row() const { return rows[N & 1]; }
};

template <int P, int N0, int N1, int J>
__device__ __forceinline__ void contract_row32(cplxf *acc, const cplxf *th, const cplxf *Ma,
                                               const float *pa, const float *pb) {
#pragma unroll
    for (int n = N0; n <= (N1 < J ? N1 : J); ++n) {
        const int k = J - n;
        const float sc = pa[k] * pb[n];
        cplxf mk[P + 1];
#pragma unroll
        for (int l = 0; l <= k; ++l) {
            const cplxf v = Ma[tri(k, l)];
            mk[l] = {v.re * sc, v.im * sc};
        }
#pragma unroll
        for (int m = 0; m <= n; ++m) {
            cplxf &a = acc[tri(n, m) - tri(N0, 0)];
#pragma unroll
            for (int l = -k; l <= k; ++l) {
                const int q = m + l;
                if (q > J || q < -J) continue;
                const cplxf mv = mk[l < 0 ? -l : l];
                const float sl = (l < 0 && (l & 1)) ? -1.0f : 1.0f;
                const float cr = sl * mv.re;
                const float ci = (l < 0) ? sl * mv.im : -mv.im;   // conj(M_k^l)
                const cplxf tv = th[q < 0 ? -q : q];
                const float sq = (q < 0 && (q & 1)) ? -1.0f : 1.0f;
                const float tr = sq * tv.re;
                const float ti = (q < 0) ? -sq * tv.im : tv.im;  // Theta_J^q
                a.re = fmaf(cr, tr, fmaf(-ci, ti, a.re));
                if (m != 0) a.im = fmaf(cr, ti, fmaf(ci, tr, a.im));
            }
        }
    }
}

template <int P, int N0, int N1>
__device__ __forceinline__ void m2l32_pass(int B, int e0, int e1, double sigma,
                                           const uint64_t *list, uint64_t mask,
                                           const TreeArrays &t, const cplxf *M, cplxf *out) {
    constexpr int NACC = tri(N1 + 1, 0) - tri(N0, 0);
    cplxf acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = {0.0f, 0.0f};
    const double4 cb = t.cen[B];
    for (int e = e0; e < e1; ++e) {
        const int A = (int)(list[e] & mask);
        const double4 ca = t.cen[A];
        const double dx = cb.x - ca.x, dy = cb.y - ca.y, dz = cb.z - ca.z;
        const double r = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
        const double ir = 1.0 / r;
        const double sa = ca.w > 0.0 ? ca.w : 1.0;
        float pa[P + 1], pb[P + 1];
        const float qa = (float)(sa * ir), qs = (float)(sigma * ir);
        pa[0] = 1.0f;
        pb[0] = qs;
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            pa[k] = pa[k - 1] * qa;
            pb[k] = pb[k - 1] * qs;
        }
        const cplxf *Ma = M + (size_t)A * tri(P + 1, 0);
        UnitTheta32<P> g;
        g.start((float)(dx * ir), (float)(dy * ir), (float)(dz * ir));
        auto row = [&]<int J>() {
            if constexpr (J > 0) g.template next<J>();
            if constexpr (J >= N0 && J > M2L32_JLO)
                contract_row32<P, N0, N1, J>(acc, g.template row<J>(), Ma, pa, pb);
            __asm__ volatile("" ::: "memory");
        };
        Unroll<0, P>::run(row);
    }
#pragma unroll
    for (int i = 0; i < NACC; ++i) out[tri(N0, 0) + i] = acc[i];
}

// FP64 terms of degree j <= JL (unscaled F_n, n <= JL)
template <int P, int JL>
__device__ __forceinline__ void m2l_low(int B, int e0, int e1, const uint64_t *list,
                                        uint64_t mask, const TreeArrays &t, const cplx *M,
                                        cplx *out) {
    constexpr int NACC = tri(JL + 1, 0);
    cplx acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = {0.0, 0.0};
    const double4 cb = t.cen[B];
    for (int e = e0; e < e1; ++e) {
        const int A = (int)(list[e] & mask);
        const double4 ca = t.cen[A];
        const cplx *Ma = M + (size_t)A * tri(P + 1, 0);
        RowGen<JL> g;
        g.theta_start(cb.x - ca.x, cb.y - ca.y, cb.z - ca.z);
        auto row = [&]<int J>() {
            if constexpr (J > 0) g.template theta_row<J>();
            m2l_detail::contract_row<P, 0, JL, J>(acc, g.template row<J>(), Ma);
        };
        Unroll<0, JL>::run(row);
    }
#pragma unroll
    for (int i = 0; i < NACC; ++i) out[i] = acc[i];
}

template <int P, int N0>
__device__ __forceinline__ void m2l32_passes(int B, int e0, int e1, double sigma,
                                             const uint64_t *list, uint64_t mask,
                                             const TreeArrays &t, const cplxf *M, cplxf *out) {
    constexpr int N1 = pass_end32(P, N0);
    m2l32_pass<P, N0, N1>(B, e0, e1, sigma, list, mask, t, M, out);
    if constexpr (N1 < P) m2l32_passes<P, N1 + 1>(B, e0, e1, sigma, list, mask, t, M, out);
}

template <int P>
__global__ void __launch_bounds__(64)
k_m2l32(int nchunks, const int4 *chunks, const uint64_t *list, uint64_t mask, TreeArrays t,
        const double *M, const float *M32, float *Fpart, double *Flow, double *sig) {
    const int ch = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (ch >= nchunks) return;
    const int4 c = chunks[ch];
    // sigma: the smallest separation of the chunk
    const double4 cb = t.cen[c.x];
    double sigma = INFINITY;
    for (int e = c.y; e < c.z; ++e) {
        const double4 ca = t.cen[(int)(list[e] & mask)];
        const double dx = cb.x - ca.x, dy = cb.y - ca.y, dz = cb.z - ca.z;
        sigma = fmin(sigma, sqrt(fma(dx, dx, fma(dy, dy, dz * dz))));
    }
    sig[ch] = sigma;
    constexpr int JL = P < M2L32_JLO ? P : M2L32_JLO;
    m2l_low<P, JL>(c.x, c.y, c.z, list, mask, t, reinterpret_cast<const cplx *>(M),
                   reinterpret_cast<cplx *>(Flow) + (size_t)ch * tri(M2L32_JLO + 1, 0));
    cplxf *out = reinterpret_cast<cplxf *>(Fpart) + (size_t)ch * tri(P + 1, 0);
    m2l32_passes<P, 0>(c.x, c.y, c.z, sigma, list, mask, t,
                       reinterpret_cast<const cplxf *>(M32), out);
}

}  // namespace m2l32_detail
}  // namespace fmm

#define FMM_M2L32_FIXED_DEFINE(P)                                                            \
    namespace fmm {                                                                          \
    hipError_t launch_m2l32_fixed_##P(int nchunks, const int4 *chunks, const uint64_t *list, \
                                      uint64_t mask, const TreeArrays &t, const double *M,   \
                                      const float *M32, float *Fpart, double *Flow,          \
                                      double *sig, hipStream_t s) {                          \
        hipLaunchKernelGGL(m2l32_detail::k_m2l32<P>, dim3((unsigned)((nchunks + 63) / 64)), \
                           dim3(64), 0, s, nchunks, chunks, list, mask, t, M, M32, Fpart,    \
                           Flow, sig);                                                       \
        return hipGetLastError();                                                            \
    }                                                                                        \
    }
