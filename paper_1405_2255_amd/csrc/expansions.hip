// Upward and downward passes: P2M (eq:P2M), M2M (eq:M2M), multipole power
// P_n (eq:def:PA), L2L (eq:L2L), L2P (eq:L2P:Psi, eq:L2P), and the low-order
// estimate of the sink scale (Sec. 5.4.2).
//
// Storage: per cell the complex X_n^m for 0 <= m <= n <= p at complex index
// tri(n, m) = n(n+1)/2 + m, (Re, Im) adjacent, Im = 0 for m = 0.
#include <algorithm>
#include <stdexcept>
#include <vector>

#include "internal.h"
#include "harmonics.h"

namespace fmm {

namespace {

// 1 / (n^2 - m^2) for 0 <= m < n <= FMM_PMAX (the Upsilon column recurrence)
struct InvTable {
    double v[FMM_PMAX + 1][FMM_PMAX + 1];
};
constexpr InvTable make_inv_table() {
    InvTable tb{};
    for (int n = 0; n <= FMM_PMAX; ++n)
        for (int m = 0; m <= FMM_PMAX; ++m)
            tb.v[n][m] = n > m ? 1.0 / (double)(n * n - m * m) : 0.0;
    return tb;
}
__constant__ InvTable kInvN2M2 = make_inv_table();

// ---- P2M: one wavefront per leaf, a lane per (particle, pair of columns) -----
// M_n^m(z) = sum_a mu_a Upsilon_n^m(x_a - z).  Lanes are (particle slot, j):
// CP lanes per particle, lane j generates columns m = j and m = P - j of its
// particle's Upsilon (P + 2 coefficients in all, the same number on every
// lane, where a lane per column would leave the upper triangle n < m idle):
// the diagonal Upsilon_m^m = prod_{i<=m} (x+iy)/(2i), then
// Upsilon_{m+1}^m = z Upsilon_m^m and
// (n^2 - m^2) Upsilon_n^m = (2n-1) z Upsilon_{n-1}^m - r^2 Upsilon_{n-2}^m,
// step t of the lane's sequence being (n, m) = (j + t, j) for t <= P - j and
// (t - 1, P - j) after that.  Each lane keeps the running sums of its
// sequence; the particle slots are added with cross-lane steps at the end.
// For even P the middle column (j = P / 2) is generated once.
template <int P>
__global__ void __launch_bounds__(256)
k_p2m(TreeArrays t, const int *leaf_cell, int nleaves, const double *x, const double *y,
      const double *z, const double *m, double *M) {
    constexpr int NJ = P / 2 + 1;                              // column pairs (j <= P / 2)
    constexpr int CP = NJ <= 2 ? 2 : NJ <= 4 ? 4 : NJ <= 8 ? 8 : NJ <= 16 ? 16 : 32;
    constexpr int SL = FMM_WAVE / CP;                          // particles per step
    constexpr int T = P + 2;                                   // steps per lane
    const int leaf = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (leaf >= nleaves) return;
    const int lane = lane_id(), j = lane % CP, slot = lane / CP;
    const bool on = j < NJ;
    const int c1 = on ? j : 0, c2 = P - c1;
    const int L1 = P + 1 - c1;             // steps of the first column
    const bool two = c2 > c1;              // a second column (not the middle one)
    const int c = leaf_cell[leaf];
    const int beg = t.beg[c], end = t.end[c];
    const double4 cen = t.cen[c];
    cplx acc[T];
#pragma unroll
    for (int q = 0; q < T; ++q) acc[q] = {0.0, 0.0};
    for (int i0 = beg; i0 < end; i0 += SL) {
        const int i = i0 + slot;
        const bool valid = i < end && on;
        const double mu = valid ? m[i] : 0.0;
        const double dx = valid ? x[i] - cen.x : 0.0, dy = valid ? y[i] - cen.y : 0.0,
                     dz = valid ? z[i] - cen.z : 0.0;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        // the diagonals of both columns from one running product
        cplx d = {1.0, 0.0}, d1 = {1.0, 0.0};
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            if (k <= c2) {
                const double h = 1.0 / (2.0 * k);
                d = {h * (dx * d.re - dy * d.im), h * (dx * d.im + dy * d.re)};
            }
            if (k == c1) d1 = d;
        }
        cplx u1 = {0.0, 0.0}, u2 = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < T; ++q) {
            const bool first = q < L1;
            const int col = first ? c1 : c2;
            const int n = first ? c1 + q : q - 1;
            cplx u;
            if (q == 0 || q == L1) {
                u = first ? d1 : d;
            } else if (n == col + 1) {
                u = {dz * u1.re, dz * u1.im};
            } else {
                const double inv = kInvN2M2.v[n][col];
                const double sc = (2.0 * n - 1.0) * dz;
                u = {(sc * u1.re - r2 * u2.re) * inv, (sc * u1.im - r2 * u2.im) * inv};
            }
            if (first || two) {
                acc[q].re = fma(mu, u.re, acc[q].re);
                acc[q].im = fma(mu, u.im, acc[q].im);
            }
            u2 = u1;
            u1 = u;
        }
    }
#pragma unroll
    for (int off = CP; off < FMM_WAVE; off <<= 1)
#pragma unroll
        for (int q = 0; q < T; ++q) {
            acc[q].re += __shfl_xor(acc[q].re, off, FMM_WAVE);
            acc[q].im += __shfl_xor(acc[q].im, off, FMM_WAVE);
        }
    if (slot != 0 || !on) return;
    cplx *Mc = reinterpret_cast<cplx *>(M) + (size_t)c * tri(P + 1, 0);
#pragma unroll
    for (int q = 0; q < T; ++q) {
        const bool first = q < L1;
        if (!first && !two) continue;
        const int col = first ? c1 : c2;
        const int n = first ? c1 + q : q - 1;
        Mc[tri(n, col)] = {acc[q].re, col == 0 ? 0.0 : acc[q].im};
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

constexpr int NFULL = (FMM_PMAX + 1) * (FMM_PMAX + 1);   // all orders -n..n
// degree and order of coefficient index o (o = tri(n, m))
__device__ __forceinline__ void nm_of(int o, int &n, int &m) {
    n = 0;
    while (tri(n + 1, 0) <= o) ++n;
    m = o - tri(n, 0);
}

// ---- M2M: one block per cell, threads over (output, rows of k) items ---------
// Level by level from the bottom.  The block of cell c first completes M(c):
// for an internal cell the sum, in child order, of the children's shifted
// expansions T(child) written by the previous level's launch (a leaf keeps
// its P2M result); then, unless c is a root, it shifts M(c) to the parent's
// centre,
//   T_n^m(c) = sum_{k=0}^{n} sum_{l=-k}^{k} Upsilon_k^l(z_c - z_parent) M_{n-k}^{m-l}(c),
// with M(c) and the shift Upsilon staged (all orders) in LDS.  The sum of
// each output is cut into items of consecutive k (the plan); each thread
// adds its items' terms, and each output then adds its items in order, so
// that no thread's chain of multiply-adds is longer than about 1/256 of the
// cell's work (the upper levels hold few cells, and there the chain sets the
// time of the launch).
__device__ __forceinline__ int isqrt_full(int f) {
    int n = (int)sqrtf((float)f);
    while (n * n > f) --n;
    while ((n + 1) * (n + 1) <= f) ++n;
    return n;
}

__global__ void __launch_bounds__(XF_THREADS)
k_m2m_level(int p, TreeArrays t, int c0, const double *U, double *M, double *T,
            const short *plan) {
    __shared__ cplx sU[NFULL], sM[NFULL], part[XF_ITEMS];
    const int c = c0 + blockIdx.x, tid = threadIdx.x;
    const int nc = tri(p + 1, 0);
    const int nch = t.nchild[c];
    const bool shift = t.parent[c] >= 0;
    cplx *Mc = reinterpret_cast<cplx *>(M) + (size_t)c * nc;
    const cplx *Tb = reinterpret_cast<const cplx *>(T);
    // complete M(c) (threads over stored coefficients) and stage it
    for (int e = tid; e < nc; e += XF_THREADS) {
        int n, m;
        nm_of(e, n, m);
        cplx v;
        if (nch > 0) {
            // the (at most 8) children's terms loaded together, added in order
            v = {0.0, 0.0};
            const int k0 = t.child0[c];
            cplx xs[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) xs[j] = Tb[(size_t)(k0 + (j < nch ? j : 0)) * nc + e];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (j < nch) {
                    v.re += xs[j].re;
                    v.im += xs[j].im;
                }
            }
            if (m == 0) v.im = 0.0;
            Mc[e] = v;
        } else {
            v = Mc[e];
        }
        sM[n * n + n + m] = v;
        if (m > 0) sM[n * n + n - m] = sym(v, -m);
    }
    if (!shift) return;
    const cplx *Uc = reinterpret_cast<const cplx *>(U) + (size_t)c * nc;
    for (int f = tid; f < (p + 1) * (p + 1); f += XF_THREADS) {
        const int n = isqrt_full(f), q = f - n * n - n;
        sU[f] = ld(Uc, n, q);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < XF_IT; ++r) {
        const int it = plan[XP_LANE + r * XF_THREADS + tid];
        if (it < 0) continue;
        const int n = plan[XP_N + it], m = plan[XP_M + it];
        const int k0 = plan[XP_K0 + it], k1 = plan[XP_K1 + it];
        // four partial sums over consecutive terms: independent chains
        cplx a[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int k = k0; k <= k1; ++k) {
            const int nn = n - k;
            const int lmin = max(-k, m - nn), lmax = min(k, m + nn);
            const int bu = k * k + k, bv = nn * nn + nn + m;
            int l = lmin;
            for (; l + 3 <= lmax; l += 4) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const cplx u = sU[bu + l + j], v = sM[bv - l - j];
                    a[j].re = fma(u.re, v.re, fma(-u.im, v.im, a[j].re));
                    a[j].im = fma(u.re, v.im, fma(u.im, v.re, a[j].im));
                }
            }
            for (; l <= lmax; ++l) {
                const cplx u = sU[bu + l], v = sM[bv - l];
                a[0].re = fma(u.re, v.re, fma(-u.im, v.im, a[0].re));
                a[0].im = fma(u.re, v.im, fma(u.im, v.re, a[0].im));
            }
        }
        part[it] = {(a[0].re + a[1].re) + (a[2].re + a[3].re),
                    (a[0].im + a[1].im) + (a[2].im + a[3].im)};
    }
    __syncthreads();
    cplx *Tc = reinterpret_cast<cplx *>(T) + (size_t)c * nc;
    for (int e = tid; e < nc; e += XF_THREADS) {
        cplx v = {0.0, 0.0};
        for (int i = plan[XP_OUT + e]; i < plan[XP_OUT + e + 1]; ++i) {
            v.re += part[i].re;
            v.im += part[i].im;
        }
        int n, m;
        nm_of(e, n, m);
        Tc[e] = {v.re, m == 0 ? 0.0 : v.im};
    }
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

// ---- L2L: one block per child, threads over (output, rows of k) items --------
// F_n^m(s') += sum_{k=0}^{p-n} sum_l conj(Upsilon_k^l(s - s')) F_{n+k}^{m+l}(s),
// with Upsilon_k^l(s - s') = (-1)^k Upsilon_k^l(s' - s) from the stored shift;
// the parent's F and the child's shift are staged (all orders) in LDS; items
// and their order as for M2M.
__global__ void __launch_bounds__(XF_THREADS)
k_l2l_level(int p, TreeArrays t, int c0, const double *U, double *F, const short *plan,
            const uint8_t *active) {
    __shared__ cplx sU[NFULL], sF[NFULL], part[XF_ITEMS];
    const int c = c0 + blockIdx.x, tid = threadIdx.x;
    if (active && !active[c]) return;      // no listed sink below c
    const int pc = t.parent[c];
    if (pc < 0) return;
    const int nc = tri(p + 1, 0);
    const cplx *Uc = reinterpret_cast<const cplx *>(U) + (size_t)c * nc;
    const cplx *Fp = reinterpret_cast<const cplx *>(F) + (size_t)pc * nc;
    for (int f = tid; f < (p + 1) * (p + 1); f += XF_THREADS) {
        const int n = isqrt_full(f), q = f - n * n - n;
        sU[f] = ld(Uc, n, q);
        sF[f] = ld(Fp, n, q);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < XF_IT; ++r) {
        const int it = plan[XP_LANE + r * XF_THREADS + tid];
        if (it < 0) continue;
        const int n = plan[XP_N + it], m = plan[XP_M + it];
        const int k0 = plan[XP_K0 + it], k1 = plan[XP_K1 + it];
        // four partial sums over consecutive terms (independent chains)
        cplx acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int k = k0; k <= k1; ++k) {
            const double sg = (k & 1) ? -1.0 : 1.0;
            const int nk = n + k;
            const int bu = k * k + k, bf = nk * nk + nk + m;
            int l = -k;
            for (; l + 3 <= k; l += 4) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const cplx u = sU[bu + l + j], f = sF[bf + l + j];
                    // conj(sg u) * f
                    const double ur = sg * u.re, ui = -sg * u.im;
                    acc[j].re = fma(ur, f.re, fma(-ui, f.im, acc[j].re));
                    acc[j].im = fma(ur, f.im, fma(ui, f.re, acc[j].im));
                }
            }
            for (; l <= k; ++l) {
                const cplx u = sU[bu + l], f = sF[bf + l];
                const double ur = sg * u.re, ui = -sg * u.im;
                acc[0].re = fma(ur, f.re, fma(-ui, f.im, acc[0].re));
                acc[0].im = fma(ur, f.im, fma(ui, f.re, acc[0].im));
            }
        }
        part[it] = {(acc[0].re + acc[1].re) + (acc[2].re + acc[3].re),
                    (acc[0].im + acc[1].im) + (acc[2].im + acc[3].im)};
    }
    __syncthreads();
    cplx *Fc = reinterpret_cast<cplx *>(F) + (size_t)c * nc;
    for (int e = tid; e < nc; e += XF_THREADS) {
        cplx v = {0.0, 0.0};
        for (int i = plan[XP_OUT + e]; i < plan[XP_OUT + e + 1]; ++i) {
            v.re += part[i].re;
            v.im += part[i].im;
        }
        int n, m;
        nm_of(e, n, m);
        cplx &dst = Fc[e];
        dst.re += v.re;
        if (m != 0) dst.im += v.im;
    }
}

// ---- L2P: one thread per particle ------------------------------------------
// Psi_0^0 = sum_{k,l} conj(Upsilon_k^l(s - x)) F_k^l and
// Psi_1^m = sum_{k<=p-1,l} conj(Upsilon_k^l(s - x)) F_{k+1}^{m+l};
// a = grad Psi_0^0 = -(Re Psi_1^1, Im Psi_1^1, Psi_1^0).
template <int P>
__global__ void __launch_bounds__(256)
k_l2p(TreeArrays t, const int *leaf_of, const int *leaf_cell, int64_t n, const double *x,
      const double *y, const double *z, const double *F, double4 *out4, const uint8_t *active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = leaf_cell[leaf_of[i]];
    if (active && !active[c]) return;      // a leaf without listed sinks
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
// Fe = (Psi, F_1^0, Re F_1^1, Im F_1^1); for f only .x is used.  One wavefront
// per sink cell: lane j adds entries j, j + 64, ... of the cell's list, then
// the lanes are added in a fixed butterfly order (deterministic).
__global__ void __launch_bounds__(256)
k_est_m2l(int want_f, TreeArrays t, int nsinks, const int64_t *off, const uint64_t *list, int sh,
          double4 *Fe) {
    const int b = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (b >= nsinks) return;
    const int lane = lane_id();
    const int64_t e0 = off[b], e1 = off[b + 1];
    const double4 sb = t.com[b];
    const uint64_t mask = (1ull << sh) - 1;
    double f0 = 0.0, f10 = 0.0, f11r = 0.0, f11i = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += FMM_WAVE) {
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
    f0 = wave_sum(f0);
    f10 = wave_sum(f10);
    f11r = wave_sum(f11r);
    f11i = wave_sum(f11i);
    if (lane == 0) Fe[b] = make_double4(f0, f10, f11r, f11i);
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

// The items of one translation: each output's rows of k are cut, in order,
// into items of at most T terms (T = the larger of the cell's terms / 256
// and the longest row).  The lanes of a wavefront run their items' loops in
// lockstep (rows of k, then the terms of each row), so a wavefront costs the
// longest of its lanes at every step: items are therefore ordered by shape
// (number of rows, first row, then longest first) and dealt in runs of 64
// consecutive ones, one run per wavefront and round; runs go, costliest
// first, to the wavefront with the least work so far (at most XF_IT each).
// A run's cost models its lockstep loops: per row a fixed set-up, per four
// terms of the row's longest lane one unrolled step, per leftover term one
// single step.  Deterministic.
static void item_plan(int p, bool m2m, short *plan) {
    const int nc = tri(p + 1, 0);
    auto row = [&](int n, int m, int k) -> int {
        if (!m2m) return 2 * k + 1;
        const int nn = n - k;
        const int lo = std::max(-k, m - nn), hi = std::min(k, m + nn);
        return hi >= lo ? hi - lo + 1 : 0;
    };
    long total = 0;
    int longest = 0;
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m)
            for (int k = 0; k <= (m2m ? n : p - n); ++k) {
                total += row(n, m, k);
                longest = std::max(longest, row(n, m, k));
            }
    const long T = std::max<long>((total + XF_THREADS - 1) / XF_THREADS, longest);
    struct Item { int n, m, k0, k1; long cost; };
    std::vector<Item> items;
    std::vector<int> first(nc + 1);
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            first[tri(n, m)] = (int)items.size();
            const int kmax = m2m ? n : p - n;
            long cur = 0;
            int k0 = 0;
            for (int k = 0; k <= kmax; ++k) {
                const int r = row(n, m, k);
                if (cur > 0 && cur + r > T) {
                    items.push_back({n, m, k0, k - 1, cur});
                    cur = 0;
                    k0 = k;
                }
                cur += r;
            }
            items.push_back({n, m, k0, kmax, cur});
        }
    first[nc] = (int)items.size();
    if ((int)items.size() > XF_ITEMS) throw std::runtime_error("translation plan: too many items");
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const Item &x = items[a], &y = items[b];
        if (x.k1 - x.k0 != y.k1 - y.k0) return x.k1 - x.k0 < y.k1 - y.k0;
        if (x.k0 != y.k0) return x.k0 < y.k0;
        return x.cost > y.cost;
    });
    constexpr int W = 64;                        // lanes per wavefront
    constexpr int NW = XF_THREADS / W;
    struct Run { int begin, end; long cost; };
    std::vector<Run> runs;
    for (int j = 0; j < (int)order.size(); j += W) {
        Run r{j, std::min(j + W, (int)order.size()), 10};
        for (int row_i = 0;; ++row_i) {
            int longest_q = -1, longest_r = 0;
            for (int t = r.begin; t < r.end; ++t) {
                const Item &it = items[order[t]];
                if (it.k0 + row_i > it.k1) continue;
                const int len = row(it.n, it.m, it.k0 + row_i);
                longest_q = std::max(longest_q, len / 4);
                longest_r = std::max(longest_r, len % 4);
            }
            if (longest_q < 0) break;
            r.cost += 20 + 20 * longest_q + 8 * longest_r;
        }
        runs.push_back(r);
    }
    std::vector<int> by_cost(runs.size());
    for (size_t i = 0; i < by_cost.size(); ++i) by_cost[i] = (int)i;
    std::stable_sort(by_cost.begin(), by_cost.end(),
                     [&](int a, int b) { return runs[a].cost > runs[b].cost; });
    std::vector<long> load(NW, 0);
    std::vector<int> rounds(NW, 0);
    for (int i = 0; i < XP_SIZE; ++i) plan[i] = -1;
    for (int ri : by_cost) {
        int best = -1;
        for (int w = 0; w < NW; ++w)
            if (rounds[w] < XF_IT && (best < 0 || load[w] < load[best])) best = w;
        if (best < 0) throw std::runtime_error("translation plan: too few threads");
        for (int t = runs[ri].begin; t < runs[ri].end; ++t)
            plan[XP_LANE + rounds[best] * XF_THREADS + best * W + (t - runs[ri].begin)] =
                (short)order[t];
        ++rounds[best];
        load[best] += runs[ri].cost;
    }
    for (size_t i = 0; i < items.size(); ++i) {
        plan[XP_N + i] = (short)items[i].n;
        plan[XP_M + i] = (short)items[i].m;
        plan[XP_K0 + i] = (short)items[i].k0;
        plan[XP_K1 + i] = (short)items[i].k1;
    }
    for (int e = 0; e <= nc; ++e) plan[XP_OUT + e] = (short)first[e];
}

void translation_plans(int p, short *m2m, short *l2l) {
    item_plan(p, true, m2m);
    item_plan(p, false, l2l);
}

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
                            double *M, double *T, const short *plan, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_m2m_level, dim3((unsigned)(c1 - c0)), dim3(XF_THREADS), 0, s, p, t, c0, U,
                       M, T, plan);
    return hipGetLastError();
}

hipError_t launch_power(int p, int ncells, const double *M, double *P, hipStream_t s) {
    hipLaunchKernelGGL(k_power, dim3(blocks(ncells, 128)), dim3(128), 0, s, p, ncells, M, P);
    return hipGetLastError();
}

hipError_t launch_l2l_level(int p, const TreeArrays &t, int c0, int c1, const double *U,
                            double *F, const short *plan, hipStream_t s, const uint8_t *active) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_l2l_level, dim3((unsigned)(c1 - c0)), dim3(XF_THREADS), 0, s, p, t, c0, U,
                       F, plan, active);
    return hipGetLastError();
}

hipError_t launch_l2p(int p, const TreeArrays &t, const int *leaf_of, const int *leaf_cell,
                      int64_t n, const double *x, const double *y, const double *z,
                      const double *F, double4 *out4, hipStream_t s, const uint8_t *active) {
#define CALL(P) hipLaunchKernelGGL(k_l2p<P>, dim3(blocks(n, 256)), dim3(256), 0, s, t, leaf_of, \
                                   leaf_cell, n, x, y, z, F, out4, active)
    FMM_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_est_m2l(int want_f, const TreeArrays &t, int nsinks, const int64_t *off,
                          const uint64_t *list, int sh, double4 *Fe, hipStream_t s) {
    hipLaunchKernelGGL(k_est_m2l, dim3(blocks(nsinks, 4)), dim3(256), 0, s, want_f, t, nsinks,
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
