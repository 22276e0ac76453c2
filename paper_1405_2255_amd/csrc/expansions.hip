// Upward and downward passes: P2M (eq:P2M), M2M (eq:M2M), multipole power
// P_n (eq:def:PA), L2L (eq:L2L), L2P (eq:L2P:Psi, eq:L2P), and the low-order
// estimate of the sink scale (Sec. 5.4.2).
//
// Storage: per cell the complex X_n^m for 0 <= m <= n <= p at complex index
// tri(n, m) = n(n+1)/2 + m, (Re, Im) adjacent, Im = 0 for m = 0.
#include "internal.h"
#include "harmonics.h"

namespace fmm {

namespace {

// ---- P2M: one wavefront per leaf, lanes over particles ----------------------
// M_n^m(z) = sum_a mu_a Upsilon_n^m(x_a - z): each lane generates the rows of
// its particle, the wavefront sums every coefficient, lane 0 stores it.
template <int P>
__global__ void __launch_bounds__(256)
k_p2m(TreeArrays t, const int *leaf_cell, int nleaves, const double *x, const double *y,
      const double *z, const double *m, double *M) {
    const int leaf = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (leaf >= nleaves) return;
    const int lane = lane_id();
    const int c = leaf_cell[leaf];
    const int beg = t.beg[c], end = t.end[c];
    const double4 cen = t.cen[c];
    cplx *Mc = reinterpret_cast<cplx *>(M) + (size_t)c * tri(P + 1, 0);
    for (int ch = beg; ch < end; ch += FMM_WAVE) {
        const int i = ch + lane;
        const bool valid = i < end;
        const double mu = valid ? m[i] : 0.0;
        RowGen<P> g;
        g.upsilon_start(valid ? x[i] - cen.x : 0.0, valid ? y[i] - cen.y : 0.0,
                        valid ? z[i] - cen.z : 0.0);
        const bool first = ch == beg;
        auto emit = [&]<int N>() {
            if constexpr (N > 0) g.template upsilon_row<N>();
            const cplx *row = g.template row<N>();
#pragma unroll
            for (int mm = 0; mm <= N; ++mm) {
                const double re = wave_sum(mu * row[mm].re);
                const double im = mm == 0 ? 0.0 : wave_sum(mu * row[mm].im);
                if (lane == 0) {
                    cplx &dst = Mc[tri(N, mm)];
                    if (first) dst = {re, im};
                    else dst = {dst.re + re, dst.im + im};
                }
            }
        };
        Unroll<0, P>::run(emit);
    }
}

// ---- Upsilon of each cell's offset from its parent's centre -----------------
template <int P>
__global__ void k_shift_upsilon(TreeArrays t, int c0, int c1, double *U) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    const int pc = t.parent[c];
    if (pc < 0) return;
    const double4 a = t.cen[c], b = t.cen[pc];
    cplx *Uc = reinterpret_cast<cplx *>(U) + (size_t)c * tri(P + 1, 0);
    RowGen<P> g;
    g.upsilon_start(a.x - b.x, a.y - b.y, a.z - b.z);
    auto emit = [&]<int N>() {
        if constexpr (N > 0) g.template upsilon_row<N>();
        const cplx *row = g.template row<N>();
#pragma unroll
        for (int mm = 0; mm <= N; ++mm) Uc[tri(N, mm)] = row[mm];
    };
    Unroll<0, P>::run(emit);
}

__device__ __forceinline__ cplx ld(const cplx *X, int n, int q) {
    return sym(X[tri(n, q < 0 ? -q : q)], q);
}

// ---- M2M: one thread per (parent, coefficient) ------------------------------
// M_n^m(z') = sum_{k=0}^{n} sum_{l=-k}^{k} Upsilon_k^l(z - z') M_{n-k}^{m-l}(z)
__global__ void k_m2m_level(int p, TreeArrays t, int c0, int c1, const double *U, double *M) {
    const int nc = tri(p + 1, 0);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = c0 + (int)(gid / nc);
    const int o = (int)(gid % nc);
    if (c >= c1) return;
    const int nch = t.nchild[c];
    if (nch == 0) return;
    int n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    const int m = o - tri(n, 0);
    const cplx *Ub = reinterpret_cast<const cplx *>(U);
    const cplx *Mb = reinterpret_cast<const cplx *>(M);
    cplx acc = {0.0, 0.0};
    const int k0 = t.child0[c];
    for (int ch = k0; ch < k0 + nch; ++ch) {
        const cplx *Uc = Ub + (size_t)ch * nc;
        const cplx *Mc = Mb + (size_t)ch * nc;
        for (int k = 0; k <= n; ++k) {
            const int nn = n - k;
            const int lmin = max(-k, m - nn), lmax = min(k, m + nn);
            for (int l = lmin; l <= lmax; ++l) {
                const cplx u = ld(Uc, k, l), v = ld(Mc, nn, m - l);
                acc.re = fma(u.re, v.re, fma(-u.im, v.im, acc.re));
                acc.im = fma(u.re, v.im, fma(u.im, v.re, acc.im));
            }
        }
    }
    if (m == 0) acc.im = 0.0;
    reinterpret_cast<cplx *>(M)[(size_t)c * nc + o] = acc;
}

// ---- multipole power P_n^2 = sum_m (n-m)!(n+m)! |M_n^m|^2 ----------------------
__global__ void k_power(int p, int ncells, const double *M, double *P) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int nc = tri(p + 1, 0);
    const cplx *Mc = reinterpret_cast<const cplx *>(M) + (size_t)c * nc;
    double fact[2 * FMM_PMAX + 1];
    fact[0] = 1.0;
    for (int i = 1; i <= 2 * p; ++i) fact[i] = fact[i - 1] * i;
    for (int n = 0; n <= p; ++n) {
        const cplx v0 = Mc[tri(n, 0)];
        double s = fact[n] * fact[n] * v0.re * v0.re;
        for (int m = 1; m <= n; ++m) {
            const cplx v = Mc[tri(n, m)];
            s += 2.0 * fact[n - m] * fact[n + m] * (v.re * v.re + v.im * v.im);
        }
        P[(size_t)c * (p + 1) + n] = sqrt(s);
    }
}

// ---- L2L: one thread per (child, coefficient) -------------------------------
// F_n^m(s') += sum_{k=0}^{p-n} sum_l conj(Upsilon_k^l(s - s')) F_{n+k}^{m+l}(s),
// with Upsilon_k^l(s - s') = (-1)^k Upsilon_k^l(s' - s) from the stored shift.
__global__ void k_l2l_level(int p, TreeArrays t, int c0, int c1, const double *U, double *F) {
    const int nc = tri(p + 1, 0);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = c0 + (int)(gid / nc);
    const int o = (int)(gid % nc);
    if (c >= c1) return;
    const int pc = t.parent[c];
    if (pc < 0) return;
    int n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    const int m = o - tri(n, 0);
    const cplx *Uc = reinterpret_cast<const cplx *>(U) + (size_t)c * nc;
    const cplx *Fp = reinterpret_cast<const cplx *>(F) + (size_t)pc * nc;
    cplx acc = {0.0, 0.0};
    for (int k = 0; k <= p - n; ++k) {
        const double sg = (k & 1) ? -1.0 : 1.0;
        for (int l = -k; l <= k; ++l) {
            const cplx u = ld(Uc, k, l), f = ld(Fp, n + k, m + l);
            // conj(sg u) * f
            const double ur = sg * u.re, ui = -sg * u.im;
            acc.re = fma(ur, f.re, fma(-ui, f.im, acc.re));
            acc.im = fma(ur, f.im, fma(ui, f.re, acc.im));
        }
    }
    cplx &dst = reinterpret_cast<cplx *>(F)[(size_t)c * nc + o];
    dst.re += acc.re;
    if (m != 0) dst.im += acc.im;
}

// ---- L2P: one thread per particle ------------------------------------------
// Psi_0^0 = sum_{k,l} conj(Upsilon_k^l(s - x)) F_k^l and
// Psi_1^m = sum_{k<=p-1,l} conj(Upsilon_k^l(s - x)) F_{k+1}^{m+l};
// a = grad Psi_0^0 = -(Re Psi_1^1, Im Psi_1^1, Psi_1^0).
template <int P>
__global__ void __launch_bounds__(256)
k_l2p(TreeArrays t, const int *leaf_of, const int *leaf_cell, int64_t n, const double *x,
      const double *y, const double *z, const double *F, double4 *out4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = leaf_cell[leaf_of[i]];
    const double4 cen = t.cen[c];
    const cplx *Fc = reinterpret_cast<const cplx *>(F) + (size_t)c * tri(P + 1, 0);
    RowGen<P> g;
    g.upsilon_start(cen.x - x[i], cen.y - y[i], cen.z - z[i]);
    double psi = 0.0;
    cplx p10 = {0.0, 0.0}, p11 = {0.0, 0.0};
    auto emit = [&]<int K>() {
        if constexpr (K > 0) g.template upsilon_row<K>();
        const cplx *u = g.template row<K>();
        // potential: Upsilon_k^0 F_k^0 + 2 sum_{l>0} Re(conj(U) F)
        {
            double s = u[0].re * Fc[tri(K, 0)].re;
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                const cplx f = Fc[tri(K, l)];
                s += 2.0 * (u[l].re * f.re + u[l].im * f.im);
            }
            psi += s;
        }
        if constexpr (K < P) {
#pragma unroll
            for (int l = -K; l <= K; ++l) {
                const cplx ul = sym(u[l < 0 ? -l : l], l);
                const cplx cu = {ul.re, -ul.im};
                const cplx f0 = ld(Fc, K + 1, l), f1 = ld(Fc, K + 1, l + 1);
                p10 = cadd(p10, cmul(cu, f0));
                p11 = cadd(p11, cmul(cu, f1));
            }
        }
    };
    Unroll<0, P>::run(emit);
    out4[i] = make_double4(psi, -p11.re, -p11.im, -p10.re);
}

// ---- low-order estimate (p = 1 at the centre of mass, or the 1/r^2 monopole) --
// Fe = (Psi, F_1^0, Re F_1^1, Im F_1^1); for f only .x is used.
__global__ void k_est_m2l(int want_f, TreeArrays t, int nsinks, const int64_t *off,
                          const uint64_t *list, int sh, double4 *Fe) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nsinks) return;
    const int64_t e0 = off[b], e1 = off[b + 1];
    const double4 sb = t.com[b];
    const uint64_t mask = (1ull << sh) - 1;
    double f0 = 0.0, f10 = 0.0, f11r = 0.0, f11i = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
        const int a = (int)(list[e] & mask);
        const double4 za = t.com[a];
        const double M = t.mass[a];
        const double dx = sb.x - za.x, dy = sb.y - za.y, dz = sb.z - za.z;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (want_f) {
            f0 += M / r2;
        } else {
            const double ri = rsqrt_nr(r2);
            const double q = M * ri, q3 = q * ri * ri;
            f0 += q;                       // M Theta_0^0
            f10 = fma(q3, dz, f10);        // M Theta_1^0 = M z / r^3
            f11r = fma(q3, dx, f11r);      // M Theta_1^1 = M (x + i y) / r^3
            f11i = fma(q3, dy, f11i);
        }
    }
    Fe[b] = make_double4(f0, f10, f11r, f11i);
}

// p = 1 shift: F_1^m is unchanged and F_0^0 is not needed for |a|; so the
// children inherit the parent's coefficients.
__global__ void k_est_l2l_level(int want_f, TreeArrays t, int c0, int c1, double4 *Fe) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    const int pc = t.parent[c];
    if (pc < 0) return;
    const double4 a = Fe[pc];
    double4 v = Fe[c];
    v.x += a.x;
    if (!want_f) {
        v.y += a.y;
        v.z += a.z;
        v.w += a.w;
    }
    Fe[c] = v;
}

__global__ void k_est_l2p(int want_f, TreeArrays t, const int *leaf_of, const int *leaf_cell,
                          int64_t n, const double4 *Fe, double4 *out4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 f = Fe[leaf_cell[leaf_of[i]]];
    out4[i] = want_f ? make_double4(f.x, 0.0, 0.0, 0.0) : make_double4(0.0, -f.z, -f.w, -f.y);
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define FMM_DISPATCH_P(p, CALL)                                                        \
    switch (p) {                                                                       \
    case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;         \
    case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;         \
    case 7: CALL(7); break;   case 8: CALL(8); break;   case 9: CALL(9); break;         \
    case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break;       \
    case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break;       \
    case 16: CALL(16); break; case 17: CALL(17); break; case 18: CALL(18); break;       \
    case 19: CALL(19); break; case 20: CALL(20); break;                                 \
    default: return hipErrorInvalidValue;                                              \
    }

}  // namespace

hipError_t launch_p2m(int p, const TreeArrays &t, const int *leaf_cell, int nleaves,
                      const double *x, const double *y, const double *z, const double *m,
                      double *M, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
#define CALL(P) hipLaunchKernelGGL(k_p2m<P>, dim3(blocks(nleaves, 4)), dim3(256), 0, s, t, \
                                   leaf_cell, nleaves, x, y, z, m, M)
    FMM_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_shift_upsilon(int p, const TreeArrays &t, int c0, int c1, double *U,
                                hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
#define CALL(P) hipLaunchKernelGGL(k_shift_upsilon<P>, dim3(blocks(c1 - c0, 128)), dim3(128), 0, \
                                   s, t, c0, c1, U)
    FMM_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_m2m_level(int p, const TreeArrays &t, int c0, int c1, const double *U,
                            double *M, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    const int64_t work = (int64_t)(c1 - c0) * tri(p + 1, 0);
    hipLaunchKernelGGL(k_m2m_level, dim3(blocks(work, 128)), dim3(128), 0, s, p, t, c0, c1, U, M);
    return hipGetLastError();
}

hipError_t launch_power(int p, int ncells, const double *M, double *P, hipStream_t s) {
    hipLaunchKernelGGL(k_power, dim3(blocks(ncells, 128)), dim3(128), 0, s, p, ncells, M, P);
    return hipGetLastError();
}

hipError_t launch_l2l_level(int p, const TreeArrays &t, int c0, int c1, const double *U,
                            double *F, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    const int64_t work = (int64_t)(c1 - c0) * tri(p + 1, 0);
    hipLaunchKernelGGL(k_l2l_level, dim3(blocks(work, 128)), dim3(128), 0, s, p, t, c0, c1, U, F);
    return hipGetLastError();
}

hipError_t launch_l2p(int p, const TreeArrays &t, const int *leaf_of, const int *leaf_cell,
                      int64_t n, const double *x, const double *y, const double *z,
                      const double *F, double4 *out4, hipStream_t s) {
#define CALL(P) hipLaunchKernelGGL(k_l2p<P>, dim3(blocks(n, 256)), dim3(256), 0, s, t, leaf_of, \
                                   leaf_cell, n, x, y, z, F, out4)
    FMM_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_est_m2l(int want_f, const TreeArrays &t, int nsinks, const int64_t *off,
                          const uint64_t *list, int sh, double4 *Fe, hipStream_t s) {
    hipLaunchKernelGGL(k_est_m2l, dim3(blocks(nsinks, 128)), dim3(128), 0, s, want_f, t, nsinks,
                       off, list, sh, Fe);
    return hipGetLastError();
}

hipError_t launch_est_l2l_level(int want_f, const TreeArrays &t, int c0, int c1, double4 *Fe,
                                hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_est_l2l_level, dim3(blocks(c1 - c0, 128)), dim3(128), 0, s, want_f, t,
                       c0, c1, Fe);
    return hipGetLastError();
}

hipError_t launch_est_l2p(int want_f, const TreeArrays &t, const int *leaf_of,
                          const int *leaf_cell, int64_t n, const double4 *Fe, double4 *out4,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_est_l2p, dim3(blocks(n, 256)), dim3(256), 0, s, want_f, t, leaf_of,
                       leaf_cell, n, Fe, out4);
    return hipGetLastError();
}

}  // namespace fmm
