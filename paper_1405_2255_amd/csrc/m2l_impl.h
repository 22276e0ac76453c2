// Register-resident M2L kernel template (see m2l.hip for the algorithm).
// Included by the translation units that instantiate it for a range of
// expansion orders, so that the orders compile in parallel.
#pragma once

#include "internal.h"
#include "harmonics.h"

namespace fmm {
namespace m2l_detail {

constexpr int FBUDGET = 48;   // complex accumulators per pass

__host__ __device__ constexpr int pass_end(int p, int n0) {
    int n = n0;
    while (n + 1 <= p && tri(n + 2, 0) - tri(n0, 0) <= FBUDGET) ++n;
    return n;
}

// first output degree a row of the pass handles: the highest one, whose
// multipoles (degree k = J - n, the fewest) are loaded one row ahead
__host__ __device__ constexpr int first_n(int J, int N1) { return J < N1 ? J : N1; }

template <int P, int N0, int J, int n>
__device__ __forceinline__ void contract_one(cplx *acc, const cplx *th, const cplx *mk) {
    constexpr int k = J - n;
#pragma unroll
    for (int m = 0; m <= n; ++m) {
        cplx &a = acc[tri(n, m) - tri(N0, 0)];
#pragma unroll
        for (int l = -k; l <= k; ++l) {
            const int q = m + l;
            if (q > J || q < -J) continue;
            // conj(M_k^l): for l < 0, M_k^l = (-1)^l conj(M_k^{-l})
            const cplx mv = mk[l < 0 ? -l : l];
            const double sl = (l < 0 && (l & 1)) ? -1.0 : 1.0;
            const double cr = sl * mv.re;
            const double ci = (l < 0) ? sl * mv.im : -mv.im;   // conj(M_k^l) = cr + i ci
            const cplx tv = th[q < 0 ? -q : q];
            const double sq = (q < 0 && (q & 1)) ? -1.0 : 1.0;
            const double tr = sq * tv.re;
            const double ti = (q < 0) ? -sq * tv.im : tv.im;    // Theta_J^q = tr + i ti
            a.re = fma(cr, tr, fma(-ci, ti, a.re));
            if (m != 0) a.im = fma(cr, ti, fma(ci, tr, a.im));
        }
    }
}

// row J, output degrees n = n1 .. N0 (descending): loads M_k (k = J - n) of
// the source and adds the terms; degree first_n is done by the caller from
// the multipoles it loaded one row ahead
template <int P, int N0, int N1, int J, int n>
__device__ __forceinline__ void contract_rest(cplx *acc, const cplx *th, const cplx *Ma) {
    if constexpr (n >= N0) {
        constexpr int k = J - n;
        cplx mk[P + 1];
#pragma unroll
        for (int l = 0; l <= k; ++l) mk[l] = Ma[tri(k, l)];
        contract_one<P, N0, J, n>(acc, th, mk);
        contract_rest<P, N0, N1, J, n - 1>(acc, th, Ma);
    }
}

// every term of row J for the output degrees N0..N1, multipoles loaded here
template <int P, int N0, int N1, int J>
__device__ __forceinline__ void contract_row(cplx *acc, const cplx *th, const cplx *Ma) {
    contract_rest<P, N0, N1, J, first_n(J, N1)>(acc, th, Ma);
}

template <int P, int N0, int N1>
__device__ __forceinline__ void m2l_pass(int B, int e0, int e1, const uint64_t *list,
                                         uint64_t mask, const TreeArrays &t, const cplx *M,
                                         cplx *out) {
    constexpr int NACC = tri(N1 + 1, 0) - tri(N0, 0);
    cplx acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = {0.0, 0.0};
    const double4 cb = t.cen[B];
    int A = (int)(list[e0] & mask);
    double4 ca = t.cen[A];
    for (int e = e0; e < e1; ++e) {
        // the next source's index now, its centre a few rows into this one, so
        // that neither load stalls the start of the next source
        const int An = (int)(list[e + 1 < e1 ? e + 1 : e] & mask);
        double4 can;
        const cplx *Ma = M + (size_t)A * tri(P + 1, 0);
        RowGen<P> g;
        g.theta_start(cb.x - ca.x, cb.y - ca.y, cb.z - ca.z);
        // multipoles of the first output degree of each row, loaded during
        // the row before (a row's loads otherwise stall its first terms)
        cplx pre[P + 1];
        if constexpr (N0 == 0) pre[0] = Ma[0];
        auto row = [&]<int J>() {
            if constexpr (J > 0) g.template theta_row<J>();
            constexpr int k1 = (J + 1) - first_n(J + 1, N1);
            cplx nxt[P + 1];
            if constexpr (J + 1 <= P && J + 1 >= N0) {
#pragma unroll
                for (int l = 0; l <= k1; ++l) nxt[l] = Ma[tri(k1, l)];
            }
            if constexpr (J == (P < 4 ? P : 4)) can = t.cen[An];
            if constexpr (J >= N0) {
                constexpr int n1 = first_n(J, N1);
                contract_rest<P, N0, N1, J, n1 - 1>(acc, g.template row<J>(), Ma);
                contract_one<P, N0, J, n1>(acc, g.template row<J>(), pre);
            }
            // reload the multipoles for every degree instead of keeping them live
            __asm__ volatile("" ::: "memory");
            if constexpr (J + 1 <= P && J + 1 >= N0) {
#pragma unroll
                for (int l = 0; l <= k1; ++l) pre[l] = nxt[l];
            }
        };
        Unroll<0, P>::run(row);
        A = An;
        ca = can;
    }
#pragma unroll
    for (int i = 0; i < NACC; ++i) out[tri(N0, 0) + i] = acc[i];
}

template <int P, int N0>
__device__ __forceinline__ void m2l_passes(int B, int e0, int e1, const uint64_t *list,
                                           uint64_t mask, const TreeArrays &t, const cplx *M,
                                           cplx *out) {
    constexpr int N1 = pass_end(P, N0);
    m2l_pass<P, N0, N1>(B, e0, e1, list, mask, t, M, out);
    if constexpr (N1 < P) m2l_passes<P, N1 + 1>(B, e0, e1, list, mask, t, M, out);
}

template <int P>
__global__ void __launch_bounds__(64)
k_m2l(int nchunks, const int4 *chunks, const uint64_t *list, uint64_t mask, TreeArrays t,
      const double *M, double *Fpart) {
    const int ch = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (ch >= nchunks) return;
    const int4 c = chunks[ch];
    cplx *out = reinterpret_cast<cplx *>(Fpart) + (size_t)ch * tri(P + 1, 0);
    m2l_passes<P, 0>(c.x, c.y, c.z, list, mask, t, reinterpret_cast<const cplx *>(M), out);
}

}  // namespace m2l_detail
}  // namespace fmm

// launcher of the order-P register kernel (defined in the m2l_p*.hip units)
#define FMM_M2L_FIXED_DEFINE(P)                                                              \
    namespace fmm {                                                                          \
    hipError_t launch_m2l_fixed_##P(int nchunks, const int4 *chunks, const uint64_t *list,   \
                                    uint64_t mask, const TreeArrays &t, const double *M,     \
                                    double *Fpart, hipStream_t s) {                          \
        hipLaunchKernelGGL(m2l_detail::k_m2l<P>, dim3((unsigned)((nchunks + 63) / 64)),     \
                           dim3(64), 0, s, nchunks, chunks, list, mask, t, M, Fpart);       \
        return hipGetLastError();                                                            \
    }                                                                                        \
    }
