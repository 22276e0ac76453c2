// Jerk kernels (Sec. 7, jerk; eqs:fmm:dot).
//
// Rates of the regular harmonics for dr/dt = v (App. A.5): in the variables
// xi = (x+iy)/2, eta = -(x-iy)/2 (eq:xi:eta) and z, eq:dUnm gives
// d/dxi Upsilon_n^m = Upsilon_{n-1}^{m-1}, d/deta Upsilon_n^m = Upsilon_{n-1}^{m+1}
// and d/dz Upsilon_n^m = Upsilon_{n-1}^m, so
//   d/dt Upsilon_n^m = xidot Upsilon_{n-1}^{m-1} + vz Upsilon_{n-1}^m
//                      + etadot Upsilon_{n-1}^{m+1},
// xidot = (vx + i vy)/2, etadot = -(vx - i vy)/2 (Upsilon_1^1 = xi has rate
// xidot, which fixes the pairing of xidot with m-1).  Every rate of degree n
// is a combination of degree n-1 harmonics, so the P2M and L2P kernels form
// the rates from the row or column they already generate.
#include "jerk.h"
#include "harmonics.h"
#include "range_loads.h"

namespace fmm {

namespace {

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// 1 / (n^2 - m^2) for 0 <= m < n <= FMM_PMAX: the divisor of the column
// recurrence eq:Ups:rec, read per lane instead of divided
struct RecipTable {
    double v[FMM_PMAX + 1][FMM_PMAX + 1];
};
constexpr RecipTable make_recip_table() {
    RecipTable r{};
    for (int n = 0; n <= FMM_PMAX; ++n)
        for (int m = 0; m <= FMM_PMAX; ++m) r.v[n][m] = n > m ? 1.0 / (double)(n * n - m * m) : 0.0;
    return r;
}
__constant__ RecipTable kRecip = make_recip_table();

// xidot X + etadot Y for the velocity (vx, vy)
__device__ __forceinline__ cplx rate_xy(double vx, double vy, cplx X, cplx Y) {
    // (vx + i vy)/2 X - (vx - i vy)/2 Y
    return {0.5 * (vx * (X.re - Y.re) - vy * (X.im + Y.im)),
            0.5 * (vx * (X.im - Y.im) + vy * (X.re + Y.re))};
}

// ---- gather -----------------------------------------------------------------
__global__ void k_gather_vel(int64_t n, const uint32_t *perm, const double *vel, double4 *v4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    v4[i] = make_double4(vel[3 * j], vel[3 * j + 1], vel[3 * j + 2], 0.0);
}

// ---- P2M rates: one wavefront per leaf, a lane per (particle, column m) ------
// Lane `col` of a particle slot generates column m = col of Upsilon_n^m(x_a - z)
// degree by degree (diagonal, then the column recurrence eq:Ups:rec); the rate
// of degree n needs columns col-1, col, col+1 of degree n-1, and the two
// neighbours are read from the adjacent lanes of the same slot.  Column -1 is
// Upsilon_{n-1}^{-1} = -conj(Upsilon_{n-1}^1) (eq:sym).  Slots are added with
// two cross-lane steps at the end.
template <int P>
__global__ void __launch_bounds__(256)
k_p2m_dot(TreeArrays t, const int *leaf_cell, int nleaves, const double *x, const double *y,
          const double *z, const double *m, const double4 *v4, double *Md) {
    constexpr int C = P < 16 ? 16 : 32;       // lanes per particle (columns 0..P)
    constexpr int SL = FMM_WAVE / C;          // particles per step
    const int leaf = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (leaf >= nleaves) return;               // whole wavefronts leave together
    const int lane = lane_id(), col = lane % C, slot = lane / C;
    const int c = leaf_cell[leaf];
    const int beg = t.beg[c], end = t.end[c];
    const double4 cen = t.cen[c];
    cplx acc[P + 1];
#pragma unroll
    for (int n = 0; n <= P; ++n) acc[n] = {0.0, 0.0};
    for (int i0 = beg; i0 < end; i0 += SL) {
        const int i = i0 + slot;
        const bool valid = i < end;
        const double mu = valid && col <= P ? m[i] : 0.0;
        const double dx = valid ? x[i] - cen.x : 0.0, dy = valid ? y[i] - cen.y : 0.0,
                     dz = valid ? z[i] - cen.z : 0.0;
        const double4 v = valid ? v4[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        cplx d = {1.0, 0.0};
#pragma unroll
        for (int j = 1; j <= P; ++j) {
            if (j <= col) {
                const double h = 1.0 / (2.0 * j);
                d = {h * (dx * d.re - dy * d.im), h * (dx * d.im + dy * d.re)};
            }
        }
        cplx u1 = {0.0, 0.0}, u2 = {0.0, 0.0};   // degrees n-1, n-2 of this column
#pragma unroll
        for (int n = 0; n <= P; ++n) {
            // rate of degree n from degree n-1 (u1) of columns col-1, col, col+1
            const int ln = (lane + FMM_WAVE - 1) & (FMM_WAVE - 1), rn = (lane + 1) & (FMM_WAVE - 1);
            const double lre = __shfl(u1.re, ln, FMM_WAVE);
            const double lim = __shfl(u1.im, ln, FMM_WAVE);
            const double rre = __shfl(u1.re, rn, FMM_WAVE);
            const double rim = __shfl(u1.im, rn, FMM_WAVE);
            const cplx right = col + 1 < C ? cplx{rre, rim} : cplx{0.0, 0.0};
            const cplx left = col > 0 ? cplx{lre, lim} : cplx{-right.re, right.im};
            const cplx r = rate_xy(v.x, v.y, left, right);
            acc[n].re = fma(mu, fma(v.z, u1.re, r.re), acc[n].re);
            acc[n].im = fma(mu, fma(v.z, u1.im, r.im), acc[n].im);
            cplx u;
            if (n < col) {
                u = {0.0, 0.0};
            } else if (n == col) {
                u = d;
            } else if (n == col + 1) {
                u = {dz * u1.re, dz * u1.im};
            } else {
                const double inv = kRecip.v[n][col < FMM_PMAX ? col : FMM_PMAX];
                const double s = (2.0 * n - 1.0) * dz;
                u = {(s * u1.re - r2 * u2.re) * inv, (s * u1.im - r2 * u2.im) * inv};
            }
            u2 = u1;
            u1 = u;
        }
    }
#pragma unroll
    for (int off = C; off < FMM_WAVE; off <<= 1)
#pragma unroll
        for (int n = 0; n <= P; ++n) {
            acc[n].re += __shfl_xor(acc[n].re, off, FMM_WAVE);
            acc[n].im += __shfl_xor(acc[n].im, off, FMM_WAVE);
        }
    if (slot != 0 || col > P) return;
    cplx *Mc = reinterpret_cast<cplx *>(Md) + (size_t)c * tri(P + 1, 0);
#pragma unroll
    for (int n = 0; n <= P; ++n)
        if (n >= col) Mc[tri(n, col)] = {acc[n].re, col == 0 ? 0.0 : acc[n].im};
}

// ---- L2P rates: one thread per particle --------------------------------------
// Psidot_1^m = sum_{k <= p-1, l} [conj(Upsilon_k^l(s - x)) Fdot_{k+1}^{m+l}
//              + conj(d/dt Upsilon_k^l(s - x)) F_{k+1}^{m+l}], d(s - x)/dt = -v,
// jerk = -(Re Psidot_1^1, Im Psidot_1^1, Psidot_1^0).  Rows of Upsilon come
// one degree at a time; row k's rates use row k-1, which the generator still
// holds.
__device__ __forceinline__ cplx ldc(const cplx *X, int n, int q) {
    return sym(X[tri(n, q < 0 ? -q : q)], q);
}

template <int P>
__global__ void __launch_bounds__(256)
k_l2p_dot(TreeArrays t, const int *leaf_of, const int *leaf_cell, int64_t n, const double *x,
          const double *y, const double *z, const double4 *v4, const double *F,
          const double *Fd, double4 *jo4, const uint8_t *active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = leaf_cell[leaf_of[i]];
    if (active && !active[c]) return;      // a leaf without listed sinks
    const double4 cen = t.cen[c];
    const cplx *Fc = reinterpret_cast<const cplx *>(F) + (size_t)c * tri(P + 1, 0);
    const cplx *Gc = reinterpret_cast<const cplx *>(Fd) + (size_t)c * tri(P + 1, 0);
    const double4 v = v4[i];
    const double wx = -v.x, wy = -v.y, wz = -v.z;   // rate of s - x
    RowGen<P> g;
    g.upsilon_start(cen.x - x[i], cen.y - y[i], cen.z - z[i]);
    cplx p10 = {0.0, 0.0}, p11 = {0.0, 0.0};
    auto emit = [&]<int K>() {
        if constexpr (K > 0) g.template upsilon_row<K>();
        const cplx *u = g.template row<K>();
#pragma unroll
        for (int l = -K; l <= K; ++l) {
            const cplx ul = sym(u[l < 0 ? -l : l], l);
            const cplx cu = {ul.re, -ul.im};
            p10 = cadd(p10, cmul(cu, ldc(Gc, K + 1, l)));
            p11 = cadd(p11, cmul(cu, ldc(Gc, K + 1, l + 1)));
        }
        if constexpr (K > 0) {
            const cplx *w = g.template row<K - 1>();
#pragma unroll
            for (int l = -K; l <= K; ++l) {
                const int a = l - 1, b = l + 1;     // columns of degree K-1
                const cplx X = (a >= -(K - 1) && a <= K - 1) ? sym(w[a < 0 ? -a : a], a)
                                                             : cplx{0.0, 0.0};
                const cplx Y = (b >= -(K - 1) && b <= K - 1) ? sym(w[b < 0 ? -b : b], b)
                                                             : cplx{0.0, 0.0};
                const cplx Z = (l >= -(K - 1) && l <= K - 1) ? sym(w[l < 0 ? -l : l], l)
                                                             : cplx{0.0, 0.0};
                const cplx r = rate_xy(wx, wy, X, Y);
                const cplx ud = {fma(wz, Z.re, r.re), fma(wz, Z.im, r.im)};
                const cplx cud = {ud.re, -ud.im};
                p10 = cadd(p10, cmul(cud, ldc(Fc, K + 1, l)));
                p11 = cadd(p11, cmul(cud, ldc(Fc, K + 1, l + 1)));
            }
        }
    };
    Unroll<0, P - 1>::run(emit);
    jo4[i] = make_double4(0.0, -p11.re, -p11.im, -p10.re);
}

// ---- near field: potential, acceleration and jerk in one pass ---------------
// d/dt [mu (x_a - x_b)/r^3] = mu [v_ab/r^3 - 3 (r . v_ab) r/r^5],
// r = x_a - x_b, v_ab = v_a - v_b.  Same tasks, lane layout and summation
// order as the force-only direct-sum kernel (a task is up to 64 sinks of a
// leaf against one slice of P2P_TASK sources of the leaf's list; two sinks per
// lane, lanes are (sink group, phase) pairs, phases added through LDS), so
// the potential and acceleration are bit for bit those of the force-only
// call; the jerk reuses each pair's separation and 1/r^3.
constexpr int JR = 2;   // sinks per lane

__device__ __forceinline__ int first_ranges(int c, const int *up, const int64_t *off) {
    return off[c + 1] > off[c] ? c : up[c];
}

struct Sink {
    double4 x, v;            // position (w: mass, unused), velocity
    double4 f;               // (pot, ax, ay, az)
    double jx, jy, jz;
};

// Summed with 2/|r| in place of 1/|r|, as the force-only direct sums are
// (the same operations, so potential and acceleration equal theirs bit for
// bit): potential times 2, acceleration and jerk times 8, scaled back once per
// sink.
constexpr double JERK_POT_BACK = 0.5, JERK_ACC_BACK = 0.125;

__device__ __forceinline__ void pair_jerk(const double4 s, const double4 va, bool skip, Sink &k) {
    const double dx = s.x - k.x.x, dy = s.y - k.x.y, dz = s.z - k.x.z;
    const double r2 = skip ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
    const double mu = skip ? 0.0 : s.w;
    const double ri = rsqrt2_nr(r2);            // 2/|r|
    const double q = mu * ri;
    const double q3 = q * ri * ri;
    k.f.x += q;
    k.f.y = fma(q3, dx, k.f.y);
    k.f.z = fma(q3, dy, k.f.z);
    k.f.w = fma(q3, dz, k.f.w);
    const double ux = va.x - k.v.x, uy = va.y - k.v.y, uz = va.z - k.v.z;
    // 3 (r.u)/r^2 = 0.75 (r.u) (2/|r|)^2
    const double rv = 0.75 * fma(dx, ux, fma(dy, uy, dz * uz)) * (ri * ri);
    k.jx = fma(q3, fma(-rv, dx, ux), k.jx);
    k.jy = fma(q3, fma(-rv, dy, uy), k.jy);
    k.jz = fma(q3, fma(-rv, dz, uz), k.jz);
}

// one lane's share of a source range that overlaps its sinks' own leaf:
// sources a, a + stride, ... below e (the sinks themselves skipped by index),
// the next source loaded before the current one is summed
__device__ __forceinline__ void sum_own_jerk(const double4 *xyzm, const double4 *v4, int a,
                                             int e, int stride, const int (&self)[JR],
                                             Sink (&k)[JR]) {
    if (a >= e) return;
    double4 s = xyzm[a], va = v4[a];
    for (;;) {
        const int b = a + stride;
        const bool more = b < e;
        const double4 s2 = xyzm[more ? b : a], vb = v4[more ? b : a];
#pragma unroll
        for (int r = 0; r < JR; ++r) pair_jerk(s, va, a == self[r], k[r]);
        if (!more) break;
        a = b;
        s = s2;
        va = vb;
    }
}

// The same for a range that holds none of the sinks, read from its start in
// scalar registers: sources xs[i], xs[i + stride], ... below xs[n] with their
// velocities vs[...] (n <= P2P_TASK).
__device__ __forceinline__ void sum_far_jerk(const double4 *xs, const double4 *vs, uint32_t i,
                                             uint32_t n, uint32_t stride, Sink (&k)[JR]) {
    gchar *bx = uniform_base(xs), *bv = uniform_base(vs);
    const uint32_t oe = n * 32u, st = stride * 32u;
    for (uint32_t o = i * 32u; o < oe; o += st) {
        const double4 s = load_source(bx + o), va = load_source(bv + o);
#pragma unroll
        for (int r = 0; r < JR; ++r) pair_jerk(s, va, false, k[r]);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_p2p_jerk(int ntasks, const int2 *tasks, const int *leaf_cell, const int *nsrc_tasks,
           const int *moff, const int64_t *off, const int2 *range, const int *up, TreeArrays t,
           const double4 *xyzm, const double4 *v4, double4 *out4, double4 *jo4,
           double4 *partial, double4 *jpartial) {
    __shared__ double4 red[4][JR * FMM_WAVE];
    __shared__ double4 jred[4][JR * FMM_WAVE];
    const int task = xcd_block(blockIdx.x, gridDim.x) * 4 + threadIdx.x / FMM_WAVE;
    if (task >= ntasks) return;                // whole wavefronts leave together
    const int lane = lane_id(), w = threadIdx.x / FMM_WAVE;
    const int2 tk = tasks[task];
    const int leaf = tk.x;
    const int c = leaf_cell[leaf];
    const int nts = nsrc_tasks[leaf];
    const int sc = tk.y / nts, ts = tk.y % nts;
    const int sb = t.beg[c] + sc * FMM_WAVE;
    const int nb = min(t.end[c] - sb, FMM_WAVE);
    const int ng = (nb + JR - 1) / JR;
    const int S = FMM_WAVE / ng;               // phases per lane group
    const int g = lane % ng, phase = lane / ng;
    const bool active = phase < S;
    Sink k[JR];
    int self[JR];
#pragma unroll
    for (int r = 0; r < JR; ++r) {
        const int slot = g + r * ng < nb ? g + r * ng : g;
        self[r] = sb + slot;
        k[r].x = xyzm[self[r]];
        k[r].v = v4[self[r]];
        k[r].f = make_double4(0.0, 0.0, 0.0, 0.0);
        k[r].jx = k[r].jy = k[r].jz = 0.0;
    }
    int64_t skip = (int64_t)ts * P2P_TASK, left = P2P_TASK;
    for (int anc = first_ranges(c, up, off); anc >= 0 && left > 0; anc = up[anc]) {
        const int64_t r1 = off[anc + 1];
        for (int64_t rb = off[anc]; rb < r1 && left > 0; rb += FMM_WAVE) {
            const int2 mine = rb + lane < r1 ? range[rb + lane] : make_int2(0, 0);
            const int nbat = (int)min((int64_t)FMM_WAVE, r1 - rb);
            for (int j = 0; j < nbat && left > 0; ++j) {
                int2 rg = make_int2(__builtin_amdgcn_readlane(mine.x, j),
                                    __builtin_amdgcn_readlane(mine.y, j));
                const int len = rg.y - rg.x;
                if (skip >= len) {
                    skip -= len;
                    continue;
                }
                rg.x += (int)skip;
                skip = 0;
                if (rg.y - rg.x > left) rg.y = rg.x + (int)left;
                left -= rg.y - rg.x;
                if (!active) continue;
                const bool own = rg.x < sb + nb && rg.y > sb;   // overlaps the task's sinks
                if (own) sum_own_jerk(xyzm, v4, rg.x + phase, rg.y, S, self, k);
                else sum_far_jerk(xyzm + rg.x, v4 + rg.x, phase, (uint32_t)(rg.y - rg.x), S, k);
            }
        }
    }
    // phases of slot q sit at red[w][q + phase * JR * ng]; active lanes cover
    // every index below JR * ng * S <= JR * 64 exactly once
    if (active) {
#pragma unroll
        for (int r = 0; r < JR; ++r) {
            red[w][g + r * ng + phase * JR * ng] = k[r].f;
            jred[w][g + r * ng + phase * JR * ng] = make_double4(0.0, k[r].jx, k[r].jy, k[r].jz);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane >= nb) return;
    double4 v = red[w][lane], jv = jred[w][lane];
    for (int ph = 1; ph < S; ++ph) {
        const double4 q = red[w][lane + ph * JR * ng], qj = jred[w][lane + ph * JR * ng];
        v.x += q.x; v.y += q.y; v.z += q.z; v.w += q.w;
        jv.y += qj.y; jv.z += qj.z; jv.w += qj.w;
    }
    v.x *= JERK_POT_BACK;
    v.y *= JERK_ACC_BACK;
    v.z *= JERK_ACC_BACK;
    v.w *= JERK_ACC_BACK;
    jv.y *= JERK_ACC_BACK;
    jv.z *= JERK_ACC_BACK;
    jv.w *= JERK_ACC_BACK;
    const int bo = sb + lane;
    if (moff[leaf + 1] == moff[leaf]) {        // the leaf's only task
        double4 o = out4[bo];
        o.x += v.x; o.y += v.y; o.z += v.z; o.w += v.w;
        out4[bo] = o;
        double4 oj = jo4[bo];
        oj.y += jv.y; oj.z += jv.z; oj.w += jv.w;
        jo4[bo] = oj;
    } else {
        const int64_t row = ((int64_t)moff[leaf] + tk.y) * FMM_WAVE + lane;
        partial[row] = v;
        jpartial[row] = jv;
    }
}

// listed sinks: jerk[3 j + d] = G jo4[inv[act[j]]].(y, z, w) (indices out of
// range are skipped; the caller reports them)
__global__ void k_output_jerk_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                     const double4 *jo4, double G, double *jerk, int *nonfinite) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nact) return;
    const int64_t idx = act[j];
    if (idx < 0 || idx >= n) return;
    const double4 v = jo4[inv[idx]];
    const double a = G * v.y, b = G * v.z, c = G * v.w;
    jerk[3 * j] = a;
    jerk[3 * j + 1] = b;
    jerk[3 * j + 2] = c;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(nonfinite, 1);
}

__global__ void k_output_jerk(int64_t n, const uint32_t *perm, const double4 *jo4, double G,
                              double *jerk, int *nonfinite) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 v = jo4[i];
    const int64_t j = perm[i];
    const double a = G * v.y, b = G * v.z, c = G * v.w;
    jerk[3 * j] = a;
    jerk[3 * j + 1] = b;
    jerk[3 * j + 2] = c;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(nonfinite, 1);
}

// exact jerk of listed sinks against all n sources, one thread per sink;
// *bad = 1 for an index outside [0, n)
__global__ void __launch_bounds__(256)
k_direct_jerk_sinks(int64_t n, const double *pos, const double *vel, const double *mass,
                    double G, int64_t nsinks, const int64_t *sinks, double *jerk, int *bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ii = t < nsinks ? sinks[t] : 0;
    const bool valid = t < nsinks && ii >= 0 && ii < n;
    if (t < nsinks && !valid) atomicOr(bad, 1);
    if (!valid) ii = 0;
    const double xb = pos[3 * ii], yb = pos[3 * ii + 1], zb = pos[3 * ii + 2];
    const double ub = vel[3 * ii], vb = vel[3 * ii + 1], wb = vel[3 * ii + 2];
    double jx = 0.0, jy = 0.0, jz = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        const double dx = pos[3 * a] - xb, dy = pos[3 * a + 1] - yb, dz = pos[3 * a + 2] - zb;
        const double ux = vel[3 * a] - ub, uy = vel[3 * a + 1] - vb, uz = vel[3 * a + 2] - wb;
        const bool self = a == ii;
        const double r2 = self ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
        const double mu = self ? 0.0 : mass[a];
        const double ri = rsqrt_nr(r2);
        const double ri2 = ri * ri;
        const double q3 = mu * ri * ri2;
        const double rv = 3.0 * fma(dx, ux, fma(dy, uy, dz * uz)) * ri2;
        jx = fma(q3, fma(-rv, dx, ux), jx);
        jy = fma(q3, fma(-rv, dy, uy), jy);
        jz = fma(q3, fma(-rv, dz, uz), jz);
    }
    if (!valid) return;
    jerk[3 * t] = G * jx;
    jerk[3 * t + 1] = G * jy;
    jerk[3 * t + 2] = G * jz;
}

#define FMM_JERK_DISPATCH_P(p, CALL)                                                   \
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

hipError_t launch_gather_vel(int64_t n, const uint32_t *perm, const double *vel, double4 *v4,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_vel, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, vel, v4);
    return hipGetLastError();
}

hipError_t launch_p2m_dot(int p, const TreeArrays &t, const int *leaf_cell, int nleaves,
                          const double *x, const double *y, const double *z, const double *m,
                          const double4 *v4, double *Md, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
#define CALL(P) hipLaunchKernelGGL(k_p2m_dot<P>, dim3(blocks(nleaves, 4)), dim3(256), 0, s, t, \
                                   leaf_cell, nleaves, x, y, z, m, v4, Md)
    FMM_JERK_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_l2p_dot(int p, const TreeArrays &t, const int *leaf_of, const int *leaf_cell,
                          int64_t n, const double *x, const double *y, const double *z,
                          const double4 *v4, const double *F, const double *Fd, double4 *jo4,
                          hipStream_t s, const uint8_t *active) {
    if (n <= 0) return hipSuccess;
#define CALL(P) hipLaunchKernelGGL(k_l2p_dot<P>, dim3(blocks(n, 256)), dim3(256), 0, s, t,   \
                                   leaf_of, leaf_cell, n, x, y, z, v4, F, Fd, jo4, active)
    FMM_JERK_DISPATCH_P(p, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_p2p_jerk(int ntasks, const int2 *tasks, const int *leaf_cell,
                           const int *nsrc_tasks, const int *moff, const int64_t *off,
                           const int2 *range, const int *up, const TreeArrays &t,
                           const double4 *xyzm, const double4 *v4, double4 *out4, double4 *jo4,
                           double4 *partial, double4 *jpartial, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_p2p_jerk, dim3(blocks(ntasks, 4)), dim3(256), 0, s, ntasks, tasks,
                       leaf_cell, nsrc_tasks, moff, off, range, up, t, xyzm, v4, out4, jo4,
                       partial, jpartial);
    return hipGetLastError();
}

hipError_t launch_direct_jerk_sinks(int64_t n, const double *pos, const double *vel,
                                   const double *mass, double G, int64_t nsinks,
                                   const int64_t *sinks, double *jerk, int *bad, hipStream_t s) {
    if (nsinks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_direct_jerk_sinks, dim3(blocks(nsinks, 256)), dim3(256), 0, s, n, pos,
                       vel, mass, G, nsinks, sinks, jerk, bad);
    return hipGetLastError();
}

hipError_t launch_output_jerk_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                     const double4 *jo4, double G, double *jerk, int *nonfinite,
                                     hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_output_jerk_listed, dim3(blocks(nact, 256)), dim3(256), 0, s, n, nact, act,
                       inv, jo4, G, jerk, nonfinite);
    return hipGetLastError();
}

hipError_t launch_output_jerk(int64_t n, const uint32_t *perm, const double4 *jo4, double G,
                              double *jerk, int *nonfinite, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_output_jerk, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, jo4, G,
                       jerk, nonfinite);
    return hipGetLastError();
}

}  // namespace fmm
