// M2L (eq:M2L): F_n^m(s_B) += sum_{k=0}^{p-n} sum_{l=-k}^{k} conj(M_k^l(z_A))
//                                Theta_{n+k}^{m+l}(s_B - z_A)
// for every accepted cell pair A -> B.
//
// The (sink-sorted) interaction list is cut into chunks of at most 16 sources
// of one sink.  For orders up to FMM_M2L_FIXED_MAX one lane owns one chunk
// (m2l_impl.h): for each source it generates Theta(s_B - z_A) one degree j at
// a time (two rows of registers) and immediately adds every term with
// n + k = j into its accumulators, reading the needed M_k of the source from
// memory (the multipoles of each row's first output degree, and the next
// source's index and centre, one step ahead, since at one wavefront per SIMD
// nothing else hides a load's latency); when the accumulators of all (p+1)(p+2)/2 outputs would not fit in
// registers, the outputs are split by degree n into passes over the chunk,
// each regenerating Theta.  Higher orders use the generic kernel below.
// Each chunk writes its partial F; a second kernel adds the partial sums of
// each sink in chunk order, so the result is deterministic.
#include <algorithm>

#include "internal.h"
#include "harmonics.h"

namespace fmm {
#define FMM_M2L_FIXED_DECL(P)                                                                  \
    hipError_t launch_m2l_fixed_##P(int, const int4 *, const uint64_t *, uint64_t, const TreeArrays &, \
                                    const double *, double *, hipStream_t);
FMM_M2L_FIXED_DECL(1) FMM_M2L_FIXED_DECL(2) FMM_M2L_FIXED_DECL(3) FMM_M2L_FIXED_DECL(4)
FMM_M2L_FIXED_DECL(5) FMM_M2L_FIXED_DECL(6) FMM_M2L_FIXED_DECL(7) FMM_M2L_FIXED_DECL(8)
FMM_M2L_FIXED_DECL(9) FMM_M2L_FIXED_DECL(10) FMM_M2L_FIXED_DECL(11) FMM_M2L_FIXED_DECL(12)
FMM_M2L_FIXED_DECL(13) FMM_M2L_FIXED_DECL(14) FMM_M2L_FIXED_DECL(15) FMM_M2L_FIXED_DECL(16)
#define FMM_M2L32_FIXED_DECL(P)                                                                \
    hipError_t launch_m2l32_fixed_##P(int, const int4 *, const uint64_t *, uint64_t,            \
                                      const TreeArrays &, const double *, const float *, float *, \
                                      double *, double *, hipStream_t);
FMM_M2L32_FIXED_DECL(1) FMM_M2L32_FIXED_DECL(2) FMM_M2L32_FIXED_DECL(3) FMM_M2L32_FIXED_DECL(4)
FMM_M2L32_FIXED_DECL(5) FMM_M2L32_FIXED_DECL(6) FMM_M2L32_FIXED_DECL(7) FMM_M2L32_FIXED_DECL(8)
FMM_M2L32_FIXED_DECL(9) FMM_M2L32_FIXED_DECL(10) FMM_M2L32_FIXED_DECL(11) FMM_M2L32_FIXED_DECL(12)
FMM_M2L32_FIXED_DECL(13) FMM_M2L32_FIXED_DECL(14) FMM_M2L32_FIXED_DECL(15) FMM_M2L32_FIXED_DECL(16)
}  // namespace fmm

namespace fmm {

namespace {

// Generic order: one workgroup per chunk.  For each source, threads 0..p
// generate one column m of Theta each (Theta_m^m by eq:The:nn, then up in n
// by the recurrence in App. A.5) into LDS while the others stage M_A; then
// thread o accumulates output coefficient o = tri(n, m) from LDS.
__global__ void __launch_bounds__(256)
k_m2l_generic(int p, int nchunks, const int4 *chunks, const uint64_t *list, uint64_t mask,
              TreeArrays t, const double *M, double *Fpart) {
    __shared__ cplx th[tri(FMM_PMAX + 1, 0)];
    __shared__ cplx ma[tri(FMM_PMAX + 1, 0)];
    const int ch = blockIdx.x;
    if (ch >= nchunks) return;
    const int4 c = chunks[ch];
    const int nc = tri(p + 1, 0);
    const int o = threadIdx.x;
    int n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    const int m = o - tri(n, 0);
    const double4 cb = t.cen[c.x];
    cplx acc = {0.0, 0.0};
    for (int e = c.y; e < c.z; ++e) {
        const int A = (int)(list[e] & mask);
        const double4 ca = t.cen[A];
        const cplx *Ma = reinterpret_cast<const cplx *>(M) + (size_t)A * nc;
        if (o <= p) {
            const double x = cb.x - ca.x, y = cb.y - ca.y, z = cb.z - ca.z;
            const double r2 = fma(x, x, fma(y, y, z * z));
            const double ri = rsqrt_nr(r2), ir2 = ri * ri;
            cplx d = {ri, 0.0};                       // Theta_0^0
            for (int i = 1; i <= o; ++i) {            // Theta_i^i
                const double f = (2.0 * i - 1.0) * ir2;
                d = {f * (x * d.re - y * d.im), f * (x * d.im + y * d.re)};
            }
            cplx a2 = {0.0, 0.0}, a1 = d;
            th[tri(o, o)] = d;
            for (int j = o + 1; j <= p; ++j) {
                const double s = (2.0 * j - 1.0) * z, b = (double)((j - 1) * (j - 1) - o * o);
                const cplx v = {(s * a1.re - b * a2.re) * ir2, (s * a1.im - b * a2.im) * ir2};
                th[tri(j, o)] = v;
                a2 = a1;
                a1 = v;
            }
        }
        for (int i = o; i < nc; i += blockDim.x) ma[i] = Ma[i];
        __syncthreads();
        if (o < nc) {
            for (int k = 0; k <= p - n; ++k) {
                for (int l = -k; l <= k; ++l) {
                    const int q = m + l;
                    if (q > n + k || q < -(n + k)) continue;
                    const cplx mv = sym(ma[tri(k, l < 0 ? -l : l)], l);
                    const cplx tv = sym(th[tri(n + k, q < 0 ? -q : q)], q);
                    // conj(M_k^l) Theta_{n+k}^{m+l}
                    acc.re = fma(mv.re, tv.re, fma(mv.im, tv.im, acc.re));
                    acc.im = fma(mv.re, tv.im, fma(-mv.im, tv.re, acc.im));
                }
            }
        }
        __syncthreads();
    }
    if (o < nc) {
        if (m == 0) acc.im = 0.0;
        reinterpret_cast<cplx *>(Fpart)[(size_t)ch * nc + o] = acc;
    }
}

__global__ void k_chunk_count(int ncells, const int64_t *off, int chunk, int *cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    if (c == ncells) {
        cnt[c] = 0;
        return;
    }
    const int64_t len = off[c + 1] - off[c];
    cnt[c] = (int)((len + chunk - 1) / chunk);
}

__global__ void k_chunk_fill(int ncells, const int64_t *off, int chunk, const int *coff,
                             int4 *chunks) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int64_t e0 = off[c], e1 = off[c + 1];
    int k = coff[c];
    for (int64_t e = e0; e < e1; e += chunk, ++k)
        chunks[k] = make_int4(c, (int)e, (int)(e + chunk < e1 ? e + chunk : e1), 0);
}

__global__ void k_m2l_reduce(int ncells, int nc, const int *coff, const double *Fpart,
                             double *F) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(gid / nc), o = (int)(gid % nc);
    if (c >= ncells) return;
    const cplx *src = reinterpret_cast<const cplx *>(Fpart);
    cplx s = {0.0, 0.0};
    for (int k = coff[c]; k < coff[c + 1]; ++k) {
        const cplx v = src[(size_t)k * nc + o];
        s.re += v.re;
        s.im += v.im;
    }
    reinterpret_cast<cplx *>(F)[(size_t)c * nc + o] = s;
}

// FP32 copy of the multipoles, scaled per cell: Mh_n^m = M_n^m / s^n with
// s = rho of the cell (1 for a point cell)
__global__ void k_m2l32_multipoles(int ncells, int p, TreeArrays t, const double *M, float *M32) {
    const int nc = tri(p + 1, 0);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(gid / nc), o = (int)(gid % nc);
    if (c >= ncells) return;
    int n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    const double rho = t.cen[c].w;
    const double is = rho > 0.0 ? 1.0 / rho : 1.0;
    double f = 1.0;
    for (int i = 0; i < n; ++i) f *= is;
    const cplx v = reinterpret_cast<const cplx *>(M)[(size_t)c * nc + o];
    M32[2 * ((size_t)c * nc + o)] = (float)(v.re * f);
    M32[2 * ((size_t)c * nc + o) + 1] = (float)(v.im * f);
}

// F_n^m of each sink = sum over its chunks (in order) of Fh_n^m sigma^{-(n+1)}
// plus, for n <= nlo, the chunk's FP64 low-degree part
// (Flow rows have tri(FMM_M2L32_JLO + 1, 0) entries, of which the first nclo
// are used)
__global__ void k_m2l32_reduce(int ncells, int nc, int nclo, const int *coff, const float *Fpart,
                               const double *Flow, const double *sig, double *F) {
    constexpr int LSTRIDE = tri(FMM_M2L32_JLO + 1, 0);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(gid / nc), o = (int)(gid % nc);
    if (c >= ncells) return;
    int n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    cplx s = {0.0, 0.0};
    for (int k = coff[c]; k < coff[c + 1]; ++k) {
        const double is = 1.0 / sig[k];
        double f = is;
        for (int i = 0; i < n; ++i) f *= is;
        s.re += (double)Fpart[2 * ((size_t)k * nc + o)] * f;
        s.im += (double)Fpart[2 * ((size_t)k * nc + o) + 1] * f;
        if (o < nclo) {
            s.re += Flow[2 * ((size_t)k * LSTRIDE + o)];
            s.im += Flow[2 * ((size_t)k * LSTRIDE + o) + 1];
        }
    }
    reinterpret_cast<cplx *>(F)[(size_t)c * nc + o] = s;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_chunks(int ncells, const int64_t *off, int chunk, int *cnt, int *coff,
                         int *tmp, int *total, int4 *chunks, bool fill, hipStream_t s) {
    if (!fill) {
        hipLaunchKernelGGL(k_chunk_count, dim3(blocks(ncells + 1, 256)), dim3(256), 0, s, ncells,
                           off, chunk, cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // coff has ncells + 1 entries: cnt[ncells] must be 0
        return exclusive_scan(cnt, coff, ncells + 1, tmp, total, s);
    }
    hipLaunchKernelGGL(k_chunk_fill, dim3(blocks(ncells, 256)), dim3(256), 0, s, ncells, off,
                       chunk, coff, chunks);
    return hipGetLastError();
}

hipError_t launch_m2l(int p, int nchunks, const int4 *chunks, const uint64_t *list, int sh,
                      const TreeArrays &t, const double *M, double *Fpart, hipStream_t s,
                      bool generic) {
    if (nchunks <= 0) return hipSuccess;
    if (p < 1 || p > FMM_PMAX) return hipErrorInvalidValue;
    const uint64_t mask = (1ull << sh) - 1;
    if (generic || p > FMM_M2L_FIXED_MAX) {
        hipLaunchKernelGGL(k_m2l_generic, dim3(nchunks), dim3(256), 0, s, p, nchunks, chunks, list,
                           mask, t, M, Fpart);
        return hipGetLastError();
    }
#define CALL(P) return launch_m2l_fixed_##P(nchunks, chunks, list, mask, t, M, Fpart, s)
    switch (p) {
    case 1: CALL(1);   case 2: CALL(2);   case 3: CALL(3);   case 4: CALL(4);
    case 5: CALL(5);   case 6: CALL(6);   case 7: CALL(7);   case 8: CALL(8);
    case 9: CALL(9);   case 10: CALL(10); case 11: CALL(11); case 12: CALL(12);
    case 13: CALL(13); case 14: CALL(14); case 15: CALL(15); case 16: CALL(16);
    default: return hipErrorInvalidValue;
    }
#undef CALL
}

hipError_t launch_m2l_reduce(int p, int ncells, const int *coff, const double *Fpart, double *F,
                             hipStream_t s) {
    const int nc = tri(p + 1, 0);
    hipLaunchKernelGGL(k_m2l_reduce, dim3(blocks((int64_t)ncells * nc, 256)), dim3(256), 0, s,
                       ncells, nc, coff, Fpart, F);
    return hipGetLastError();
}

}  // namespace fmm

namespace fmm {

hipError_t launch_m2l32_multipoles(int p, int ncells, const TreeArrays &t, const double *M,
                                   float *M32, hipStream_t s) {
    const int nc = tri(p + 1, 0);
    hipLaunchKernelGGL(k_m2l32_multipoles, dim3(blocks((int64_t)ncells * nc, 256)), dim3(256), 0,
                       s, ncells, p, t, M, M32);
    return hipGetLastError();
}

hipError_t launch_m2l32(int p, int nchunks, const int4 *chunks, const uint64_t *list, int sh,
                        const TreeArrays &t, const double *M, const float *M32, float *Fpart,
                        double *Flow, double *sig, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    const uint64_t mask = (1ull << sh) - 1;
#define CALL(P)                                                                                \
    return launch_m2l32_fixed_##P(nchunks, chunks, list, mask, t, M, M32, Fpart, Flow, sig, s)
    switch (p) {
    case 1: CALL(1);   case 2: CALL(2);   case 3: CALL(3);   case 4: CALL(4);
    case 5: CALL(5);   case 6: CALL(6);   case 7: CALL(7);   case 8: CALL(8);
    case 9: CALL(9);   case 10: CALL(10); case 11: CALL(11); case 12: CALL(12);
    case 13: CALL(13); case 14: CALL(14); case 15: CALL(15); case 16: CALL(16);
    default: return hipErrorInvalidValue;
    }
#undef CALL
}

hipError_t launch_m2l32_reduce(int p, int ncells, const int *coff, const float *Fpart,
                               const double *Flow, const double *sig, double *F, hipStream_t s) {
    const int nc = tri(p + 1, 0);
    const int nclo = tri(std::min(p, FMM_M2L32_JLO) + 1, 0);
    hipLaunchKernelGGL(k_m2l32_reduce, dim3(blocks((int64_t)ncells * nc, 256)), dim3(256), 0, s,
                       ncells, nc, nclo, coff, Fpart, Flow, sig, F);
    return hipGetLastError();
}

}  // namespace fmm
