// Rotation-accelerated M2L (App. A: fast rotations, a fast M2L kernel).
//
// For an accepted pair A -> B with r = s_B - z_A the multipoles of A are
// turned into a frame whose z axis points along r, the interaction is then
// the z-axis kernel eq:M2L:z (one sum over the degree per coefficient), and
// the result is turned back:
//   forward, per degree k:  rotate about z by alpha, swap x<->z, rotate about
//     z by beta, swap x<->z  (alpha = phi - pi/2 puts r into the y-z plane,
//     beta = atan2(rho, z) then brings it onto the z axis; phi is the azimuth
//     of r and rho = |(x, y)|);
//   z-axis kernel: Ft_n^m += (-1)^m Mt_k^m (n+k)!/r^{n+k+1}, m <= min(k, n);
//   backward, per degree n: swap, rotate by -beta, swap, rotate by -alpha.
// A rotation about z by t multiplies X_n^m by e^{-imt}.  The swap matrix of
// the Theta-type local coefficients is B_n (eq:Ylm:swap), that of the
// Upsilon-type multipoles its transpose.  In the real basis (Re and Im of the
// m >= 0 coefficients) each swap splits into a Re block and an Im block, and
// within a block entry (m, l) vanishes unless m + l + n is even (Re) or odd
// (Im): about a quarter of the entries of the complex B_n are nonzero.  Only
// multipoles with m <= min(k, p-k) are needed after the last forward swap and
// only Ft_n^m with m <= min(n, p-n) are nonzero before the first backward
// one, so those swaps run over the reduced rows or columns.
//
// Work decomposition: one wavefront per window of 64 consecutive entries of
// the sink-sorted M2L list, one lane per pair.  The Ft accumulators live in
// registers.  The swap coefficients are the same for every lane and known at
// compile time: nearly all are short dyadic rationals that the FP64
// multiply-add takes as an immediate operand.  After the back rotation of a
// group of degrees, each lane writes its coefficients to its row in LDS and
// lane j adds column j over the window's lanes in list order, writing one
// partial sum per run of equal sinks ("piece") to Fpart; pieces are summed
// per sink in order by the reduce kernel, so the result is deterministic.
#pragma once

#include "internal.h"
#include "harmonics.h"

namespace fmm {
namespace m2lr {

constexpr int WIN = 64;              // list entries per wavefront
constexpr int LDS_STRIDE = WIN + 1;  // doubles per lane row (padding)

// ---- layout of the swap-coefficient table ----------------------------------
// Per degree n: the Upsilon-type block (type 0), then the Theta-type block
// (type 1); each block holds the Re rows m = 0..n (columns l = 0..n with
// m + l + n even) then the Im rows m = 1..n (columns l = 1..n, m + l + n odd),
// columns ascending.
__host__ __device__ constexpr int first_re(int n, int m) { return (m + n) & 1; }
__host__ __device__ constexpr int first_im(int n, int m) { return ((m + n) & 1) ? 2 : 1; }
__host__ __device__ constexpr int count_from(int first, int n) {
    return first > n ? 0 : (n - first) / 2 + 1;
}
__host__ __device__ constexpr int re_rows_before(int n, int m) {
    int s = 0;
    for (int j = 0; j < m; ++j) s += count_from(first_re(n, j), n);
    return s;
}
__host__ __device__ constexpr int im_rows_before(int n, int m) {
    int s = 0;
    for (int j = 1; j < m; ++j) s += count_from(first_im(n, j), n);
    return s;
}
__host__ __device__ constexpr int block_size(int n) {
    return re_rows_before(n, n + 1) + im_rows_before(n, n + 1);
}
__host__ __device__ constexpr int degree_base(int n) {
    int s = 0;
    for (int j = 0; j < n; ++j) s += 2 * block_size(j);
    return s;
}
__host__ __device__ constexpr int re_index(int type, int n, int m, int l) {
    return degree_base(n) + type * block_size(n) + re_rows_before(n, m) +
           (l - first_re(n, m)) / 2;
}
__host__ __device__ constexpr int im_index(int type, int n, int m, int l) {
    return degree_base(n) + type * block_size(n) + re_rows_before(n, n + 1) +
           im_rows_before(n, m) + (l - first_im(n, m)) / 2;
}
__host__ __device__ constexpr int table_size(int pmax) { return degree_base(pmax + 1); }

// The table itself, computed at compile time (every entry becomes an
// immediate operand of the kernel code).  Complex x<->z swap matrices B_n
// (eq:Ylm:swap) by the recurrence of App. A: rows |m| < n of B_n from
// 2 B_n^{ml} = B_{n-1}^{m,l-1} - B_{n-1}^{m,l+1}, rows m = +-n from
// 2 B_n^{+-n,l} = B_{n-1}^{+-(n-1),l-1} + B_{n-1}^{+-(n-1),l+1} +- 2 B_{n-1}^{+-(n-1),l}
// (entries of B_{n-1} with |l| > n-1 are zero); every entry is a dyadic
// rational, exact in FP64.  Real basis, for output m >= 0 and input l > 0
// (X^{-l} = (-1)^l conj(X^l), eq:sym): Re uses B^{ml} + (-1)^l B^{m,-l}, Im
// uses B^{ml} - (-1)^l B^{m,-l}; the Upsilon-type block uses the transpose.
template <int PMAX>
struct SwapTable {
    static constexpr int W = 2 * PMAX + 1;
    double v[table_size(PMAX)];
    bool ok;     // false if an entry the layout leaves out is not zero
    constexpr SwapTable() : v{}, ok(true) {
        int pos = 0;
        double prev[W * W] = {}, cur[W * W] = {};
        cur[0] = 1.0;
        for (int n = 0; n <= PMAX; ++n) {
            const int w = 2 * n - 1, Wn = 2 * n + 1;
            if (n > 0) {
                for (int i = 0; i < w * w; ++i) prev[i] = cur[i];
                auto at = [&](int m, int l) {
                    return (m >= 1 - n && m <= n - 1 && l >= 1 - n && l <= n - 1)
                               ? prev[(m + n - 1) * w + l + n - 1]
                               : 0.0;
                };
                for (int m = -n; m <= n; ++m)
                    for (int l = -n; l <= n; ++l) {
                        double x;
                        if (m == n)
                            x = 0.5 * (at(n - 1, l - 1) + at(n - 1, l + 1) + 2.0 * at(n - 1, l));
                        else if (m == -n)
                            x = 0.5 * (at(1 - n, l - 1) + at(1 - n, l + 1) - 2.0 * at(1 - n, l));
                        else
                            x = 0.5 * (at(m, l - 1) - at(m, l + 1));
                        cur[(m + n) * Wn + l + n] = x;
                    }
            }
            // entries in layout order (re_index / im_index enumerate the same order)
            for (int type = 0; type < 2; ++type) {
                // coefficient of input l in output m: B^{lm} (type 0) or B^{ml}
                auto bt = [&](int mm, int ll) {
                    return type == 0 ? cur[(ll + n) * Wn + mm + n] : cur[(mm + n) * Wn + ll + n];
                };
                auto re = [&](int m, int l) {
                    return l == 0 ? bt(m, 0) : bt(m, l) + ((l & 1) ? -1.0 : 1.0) * bt(m, -l);
                };
                auto im = [&](int m, int l) {
                    return bt(m, l) - ((l & 1) ? -1.0 : 1.0) * bt(m, -l);
                };
                for (int m = 0; m <= n; ++m)
                    for (int l = 0; l <= n; ++l) {
                        if (((m + l + n) & 1) == 0) v[pos++] = re(m, l);
                        else if (re(m, l) != 0.0) ok = false;
                    }
                for (int m = 1; m <= n; ++m)
                    for (int l = 1; l <= n; ++l) {
                        if ((m + l + n) & 1) v[pos++] = im(m, l);
                        else if (im(m, l) != 0.0) ok = false;
                    }
            }
        }
        if (pos != table_size(PMAX)) ok = false;
    }
};
inline constexpr SwapTable<16> kSwap{};
static_assert(kSwap.ok, "real-basis swap matrices do not have the expected sparsity");

// ---- per-lane pieces --------------------------------------------------------
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
// index of Ft_n^m (m <= min(n, P-n)) in the accumulator arrays
template <int P>
__host__ __device__ constexpr int ft(int n, int m) {
    int s = 0;
    for (int j = 0; j < n; ++j) s += cmin(j, P - j) + 1;
    return s + m;
}
// degree groups for the reduction: consecutive degrees [n0, end) with at
// most WIN doubles (Re, Im of m = 0..n per degree)
__host__ __device__ constexpr int group_end(int P, int n0) {
    int n = n0 + 1;
    while (n <= P && 2 * (tri(n + 1, 0) - tri(n0, 0)) <= WIN) ++n;
    return n;
}

// y = R x for one degree N in the real basis: R the type-T swap, rows
// m = 0..MR, input columns l = 0..LC (the others are zero)
// A zero the compiler cannot see through: every product of a swap row is then
// an accumulate into a register, which takes the coefficient as an immediate
// operand (the coefficients are short dyadic rationals) instead of a pair of
// scalar registers loaded per use.
__device__ __forceinline__ double opaque_zero() {
    double z = 0.0;
    __asm__ volatile("" : "+v"(z));
    return z;
}

template <int T, int N, int MR, int LC>
__device__ __forceinline__ void swap_xz(const double (&xa)[N + 1],
                                        const double (&xb)[N + 1], double (&ya)[N + 1],
                                        double (&yb)[N + 1]) {
    Unroll<0, MR>::run([&]<int M>() {
        double s = opaque_zero();
        Unroll<0, LC>::run([&]<int L>() {
            if constexpr (((M + L + N) & 1) == 0) {
                constexpr double c = kSwap.v[re_index(T, N, M, L)];
                s = fma(c, xa[L], s);
            }
        });
        ya[M] = s;
        if constexpr (M >= 1) {
            double u = opaque_zero();
            Unroll<1, LC>::run([&]<int L>() {
                if constexpr (((M + L + N) & 1) == 1) {
                    constexpr double c = kSwap.v[im_index(T, N, M, L)];
                    u = fma(c, xb[L], u);
                }
            });
            yb[M] = u;
        }
    });
}

// X^m *= e^{SIGN i m t} for m = 1..N, e^{it} = c1 + i s1 (powers by recurrence)
template <int N, int SIGN>
__device__ __forceinline__ void rot_z(double (&a)[N + 1], double (&b)[N + 1], double c1,
                                      double s1) {
    double c = c1, s = s1;
    Unroll<1, N>::run([&]<int M>() {
        if constexpr (M > 1) {
            const double cn = fma(c, c1, -s * s1);
            s = fma(s, c1, c * s1);
            c = cn;
        }
        const double ar = a[M], bi = b[M];
        if constexpr (SIGN < 0) {        // (a + ib)(c - is)
            a[M] = fma(ar, c, bi * s);
            b[M] = fma(bi, c, -ar * s);
        } else {                         // (a + ib)(c + is)
            a[M] = fma(ar, c, -bi * s);
            b[M] = fma(bi, c, ar * s);
        }
    });
}

template <int P>
struct Pair {
    static constexpr int NF = ft<P>(P + 1, 0);
    double fr[NF], fi[NF];    // Ft_n^m, real and imaginary parts
    double g[P + 1];          // g_j = j! / r^{j+1}
    double ca, sa, cb, sb;    // e^{i alpha}, e^{i beta}

    __device__ __forceinline__ void setup(double x, double y, double z) {
        const double rho2 = fma(x, x, y * y);
        const double r2 = rho2 + z * z;
        const double ir = rsqrt_nr(r2);
        if (rho2 > 1e-200 * r2) {
            const double irho = rsqrt_nr(rho2);
            ca = y * irho;                // e^{i alpha} = (x + iy)/rho * (-i)
            sa = -x * irho;
            cb = z * ir;                  // e^{i beta} = (z + i rho)/r
            sb = rho2 * irho * ir;
        } else {                          // on the z axis: alpha arbitrary
            ca = 1.0;
            sa = 0.0;
            cb = z > 0.0 ? 1.0 : -1.0;
            sb = 0.0;
        }
        g[0] = ir;
#pragma unroll
        for (int j = 1; j <= P; ++j) g[j] = g[j - 1] * (double)j * ir;
#pragma unroll
        for (int i = 0; i < NF; ++i) fr[i] = fi[i] = 0.0;
    }

    // multipoles of degree K (already loaded into cur): rotate into the
    // interaction frame, then the z-axis kernel into the accumulators
    template <int K>
    __device__ __forceinline__ void forward(const cplx (&cur)[K + 1]) {
        constexpr int MR = cmin(K, P - K);
        double a[K + 1], b[K + 1], a2[K + 1], b2[K + 1];
        Unroll<0, K>::run([&]<int m>() {
            a[m] = cur[m].re;
            b[m] = cur[m].im;
        });
        rot_z<K, -1>(a, b, ca, sa);
        swap_xz<0, K, K, K>(a, b, a2, b2);
        rot_z<K, -1>(a2, b2, cb, sb);
        swap_xz<0, K, MR, K>(a2, b2, a, b);
        Unroll<0, P - K>::run([&]<int N>() {
            const double gk = g[N + K];
            Unroll<0, cmin(K, N)>::run([&]<int M>() {
                constexpr int i = ft<P>(N, M);
                if constexpr (M & 1) {
                    fr[i] = fma(-a[M], gk, fr[i]);
                    fi[i] = fma(-b[M], gk, fi[i]);
                } else {
                    fr[i] = fma(a[M], gk, fr[i]);
                    if constexpr (M > 0) fi[i] = fma(b[M], gk, fi[i]);
                }
            });
        });
    }

    // degrees K..P: the loads of degree K + 1 are issued before degree K is
    // processed, and the memory fence keeps the compiler from hoisting the
    // loads of all degrees to the start (which would hold the whole multipole
    // expansion in registers)
    template <int K>
    __device__ __forceinline__ void forward_from(const cplx *__restrict__ Ma,
                                                 const cplx (&cur)[K + 1]) {
        if constexpr (K < P) {
            cplx nxt[K + 2];
            Unroll<0, K + 1>::run([&]<int m>() { nxt[m] = Ma[tri(K + 1, m)]; });
            forward<K>(cur);
            __asm__ volatile("" ::: "memory");
            forward_from<K + 1>(Ma, nxt);
        } else {
            forward<K>(cur);
        }
    }

    // local coefficients of degree N back in the original frame, written to
    // this lane's LDS row at column `col` (Re, Im of m = 0..N)
    template <int N>
    __device__ __forceinline__ void backward(double *row, int col) {
        constexpr int MC = cmin(N, P - N);
        double a[N + 1], b[N + 1], a2[N + 1], b2[N + 1];
        Unroll<0, N>::run([&]<int m>() {
            if constexpr (m <= MC) {
                constexpr int i = ft<P>(N, m);
                a[m] = fr[i];
                b[m] = m >= 1 ? fi[i] : 0.0;
            } else {
                a[m] = b[m] = 0.0;
            }
        });
        swap_xz<1, N, N, MC>(a, b, a2, b2);
        rot_z<N, +1>(a2, b2, cb, sb);
        swap_xz<1, N, N, N>(a2, b2, a, b);
        rot_z<N, +1>(a, b, ca, sa);
        Unroll<0, N>::run([&]<int m>() {
            row[col + 2 * m] = a[m];
            row[col + 2 * m + 1] = m ? b[m] : 0.0;
        });
    }
};

// degrees [N0, N1) back-rotated into LDS, then the segmented column sums of
// the window written per piece
template <int P, int N0>
__device__ __forceinline__ void backward_groups(Pair<P> &pr, double *lds, int lane,
                                                uint64_t endmask,
                                                int piece, double *__restrict__ Fpart) {
    constexpr int N1 = group_end(P, N0);
    constexpr int GV = 2 * (tri(N1, 0) - tri(N0, 0));
    constexpr int NC = tri(P + 1, 0);
    double *row = lds + lane * LDS_STRIDE;
    Unroll<N0, N1 - 1>::run([&]<int N>() {
        pr.template backward<N>(row, 2 * (tri(N, 0) - tri(N0, 0)));
    });
    __syncthreads();
    if (lane < GV) {
        double acc = 0.0;
        for (int src = 0; src < WIN; ++src) {
            acc += lds[src * LDS_STRIDE + lane];
            if ((endmask >> src) & 1) {
                const int pc = __builtin_amdgcn_readlane(piece, src);
                Fpart[(size_t)pc * 2 * NC + 2 * tri(N0, 0) + lane] = acc;
                acc = 0.0;
            }
        }
    }
    __syncthreads();
    if constexpr (N1 <= P) backward_groups<P, N1>(pr, lds, lane, endmask, piece, Fpart);
}

template <int P>
__global__ void __launch_bounds__(WIN)
k_m2l_rot(int64_t nlist, const uint64_t *__restrict__ list, int sh,
          const int64_t *__restrict__ off, const int *__restrict__ coff, TreeArrays t,
          const double *__restrict__ M, double *__restrict__ Fpart) {
    __shared__ double lds[WIN * LDS_STRIDE];
    const int w = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int64_t e = (int64_t)w * WIN + lane;
    const bool active = e < nlist;
    const uint64_t key = list[active ? e : nlist - 1];
    const int B = (int)(key >> sh);
    const int A = (int)(key & ((1ull << sh) - 1));
    // runs of equal sinks inside the window end where the next entry has
    // another sink (or at the window's or the list's end)
    const int nextB = __shfl_down(B, 1);
    const bool end = active && (lane == WIN - 1 || e + 1 >= nlist || nextB != B);
    const uint64_t endmask = __ballot(end);
    const int piece = coff[B] + (int)((int64_t)w - off[B] / WIN);
    const double4 cb = t.cen[B], ca = t.cen[A];
    Pair<P> pr;
    pr.setup(cb.x - ca.x, cb.y - ca.y, cb.z - ca.z);
    const cplx *Ma = reinterpret_cast<const cplx *>(M) + (size_t)A * tri(P + 1, 0);
    const cplx m0[1] = {Ma[0]};
    pr.template forward_from<0>(Ma, m0);
    backward_groups<P, 0>(pr, lds, lane, endmask, piece, Fpart);
}

}  // namespace m2lr
}  // namespace fmm

// launcher of the order-P rotation kernel (defined in the m2lr_p*.hip units)
#define FMM_M2L_ROT_DEFINE(P)                                                                \
    namespace fmm {                                                                          \
    hipError_t launch_m2l_rot_##P(int64_t nlist, const uint64_t *list, int sh,               \
                                  const int64_t *off, const int *coff, const TreeArrays &t,  \
                                  const double *M, double *Fpart, hipStream_t s) {           \
        const unsigned nwin = (unsigned)((nlist + m2lr::WIN - 1) / m2lr::WIN);               \
        hipLaunchKernelGGL(m2lr::k_m2l_rot<P>, dim3(nwin), dim3(m2lr::WIN), 0, s, nlist,     \
                           list, sh, off, coff, t, M, Fpart);                                \
        return hipGetLastError();                                                            \
    }                                                                                        \
    }
