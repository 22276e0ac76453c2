// One-sided dual tree walk (Sec. 2.2.2, Sec. 6.1), breadth first.
//
// Each sweep takes a frontier of cell pairs (A -> B: A source, B sink) and
// for every pair decides, as the recursive walk would:
//   A == B:  a leaf interacts with itself directly; otherwise all ordered
//            pairs of its daughters (including each with itself) are next.
//   accepted (criterion below): direct sum if N_A N_B < T, else M2L.
//   not accepted, both leaves: direct sum.
//   otherwise split the larger cell (by radius; B on a tie; never a leaf).
// Acceptance, main pass:   theta < 1 and Etilde M_A / r^2 < eps min_B{a_b}
//                          (eq:mac:better:a, eq:err:tilde, eq:def:EAB; or f_b)
//              theta mode: rho_A + rho_B < theta_crit r          (eq:mac:theta)
//              estimate:   rho_A + rho_B < r about the centres of mass
// The set of decisions depends only on the pair, never on the visiting
// order, so the lists equal those of a depth-first recursion.
//
// The lists are sorted by sink afterwards.  One
// shortcut (marked below) emits, for a sink leaf that no cell below A can
// ever pass the radius test against, the direct sum with all of A at once:
// the same particle pairs as the recursion, without descending A.  An M2L entry
// is (sink cell, source cell); a direct-sum entry is (sink cell, source
// particle range), the sink being any cell: its particles are reached from
// each leaf below it through the leaf's ancestor chain.
#include "internal.h"
#include "dev.h"

namespace fmm {

namespace {

// distance from the unfused squared distance (the same number as the
// definition) by the correctly rounded square root
__device__ __forceinline__ double dist_rn(double4 a, double4 b) {
    return __dsqrt_rn(dist2_exact(b.x, b.y, b.z, a.x, a.y, a.z));
}

// The decision for one cell pair (as the recursive walk would take it).
struct Decision {
    int kind;      // 0 none, 1 self-split, 2 split A, 3 split B, 4 direct, 5 M2L
    int nf;        // frontier pairs emitted
    double pairs;  // particle pairs summed directly
};

__device__ __forceinline__ Decision decide(const WalkParams &wp, const TreeArrays &t,
                                           const double *P, int A, int B) {
    if (wp.active && !wp.active[B]) return {0, 0, 0.0};   // no listed sink below B
    const int nchA = t.nchild[A], nchB = t.nchild[B];
    if (A == B) {
        if (nchA == 0) {
            const double na = (double)(t.end[A] - t.beg[A]);
            return {4, 0, na * (na - 1.0)};
        }
        return {1, nchA * nchA, 0.0};
    }
    const bool est = wp.mode == 2;
    const double4 ca = est ? t.com[A] : t.cen[A];
    const double4 cb = est ? t.com[B] : t.cen[B];
    const double r = dist_rn(ca, cb);
    const double rA = ca.w, rB = cb.w;
    const double tc = wp.mode == 1 ? wp.theta_crit : 1.0;
    bool acc = rA + rB < tc * r;
    if (acc && wp.mode == 0) {
        // Etilde M_A = 8 max/(sum) * sum_k C(p,k) P_k rho_B^{p-k} / r^p, by Horner
        // in q = rho_B / r
        const int p = wp.p;
        const double *Pa = P + (size_t)A * (p + 1);
        const double u = 1.0 / r, q = rB * u;
        double S = Pa[0], up = 1.0;
        for (int k = 1; k <= p; ++k) {
            up *= u;
            S = fma(S, q, wp.binom[k] * Pa[k] * up);
        }
        const double sum = rA + rB;
        const double fac = sum > 0.0 ? 8.0 * fmax(rA, rB) / sum : 8.0;
        acc = fac * S * u * u < wp.eps * t.smin[B];
    }
    const double na = (double)(t.end[A] - t.beg[A]);
    const double nb = (double)(t.end[B] - t.beg[B]);
    if (acc) {
        if (wp.mode != 2 && na * nb < wp.p2p_pairs) return {4, 0, na * nb};
        return {5, 0, 0.0};
    }
    if (nchA == 0 && nchB == 0) return {4, 0, na * nb};
    if (nchB == 0 && rB >= tc * (r + rA) * (1.0 + 1e-12)) {
        // B cannot be split, and no cell below A can pass the radius test
        // against it: every centre below A lies in A's sphere, so its distance
        // to B is at most r + rho_A.  The recursion would end in direct sums
        // with all of A's leaves.
        return {4, 0, na * nb};
    }
    const bool splitA = nchA > 0 && (nchB == 0 || rA > rB);
    return {splitA ? 2 : 3, splitA ? nchA : nchB, 0.0};
}

// Sweeps run without host round trips: sweep i reads its frontier size from
// counters[4 + i - 1].  Each sweep is two launches over a fixed grid of
// WALK_BLOCKS blocks, block b owning a contiguous chunk of the frontier:
// count (per-block totals) and write (each block sums the totals of the
// blocks before it for its offsets, block 0 the sweep's totals; then the
// outputs at their offsets, in frontier order).  No atomics; the output order
// is deterministic.
constexpr int WALK_BLOCKS = 1024;
constexpr int WALK_THREADS = 256;
constexpr int WALK_WBATCH = 4;  // rounds whose loads the write kernel issues together

__device__ __forceinline__ int64_t sweep_input(const WalkParams &wp,
                                               const unsigned long long *cnt, int sweep) {
    return sweep == 0 ? wp.nroots : (int64_t)cnt[4 + sweep - 1];
}

// block-wide inclusive scan of three ints (256 threads = 4 waves)
__device__ __forceinline__ void block_scan3(int &a, int &b, int &c, int *tot) {
    __shared__ int ws[WALK_THREADS / FMM_WAVE][3];
    const int lane = lane_id(), w = threadIdx.x / FMM_WAVE;
    a = wave_incl_scan(a);
    b = wave_incl_scan(b);
    c = wave_incl_scan(c);
    if (lane == FMM_WAVE - 1) {
        ws[w][0] = a;
        ws[w][1] = b;
        ws[w][2] = c;
    }
    __syncthreads();
    int oa = 0, ob = 0, oc = 0, ta = 0, tb = 0, tcn = 0;
#pragma unroll
    for (int i = 0; i < WALK_THREADS / FMM_WAVE; ++i) {
        if (i < w) {
            oa += ws[i][0];
            ob += ws[i][1];
            oc += ws[i][2];
        }
        ta += ws[i][0];
        tb += ws[i][1];
        tcn += ws[i][2];
    }
    __syncthreads();
    a += oa;
    b += ob;
    c += oc;
    tot[0] = ta;
    tot[1] = tb;
    tot[2] = tcn;
}

__global__ void __launch_bounds__(WALK_THREADS)
k_walk_count(WalkParams wp, TreeArrays t, const double *P, WalkBuffers wb, int sweep,
             unsigned long long *btot) {
    const unsigned long long *cnt = wb.counters;
    const int64_t n_in = sweep_input(wp, cnt, sweep);
    unsigned long long f = 0, m = 0, q = 0;
    double pairs = 0.0;
    if (n_in <= wb.cap_out) {
        const int64_t chunk = (n_in + WALK_BLOCKS - 1) / WALK_BLOCKS;
        const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n_in, lo + chunk);
        for (int64_t i = lo + threadIdx.x; i < hi; i += WALK_THREADS) {
            const uint2 pr = wb.in[i];
            const Decision d = decide(wp, t, P, (int)pr.x, (int)pr.y);
            wb.code[i] = (uint16_t)(d.kind | (d.nf << 3));   // kind < 8, nf <= 64
            f += d.nf;
            m += d.kind == 5;
            q += d.kind == 4;
            pairs += d.pairs;
        }
    }
    // block reduction
    double fv = (double)f, mv = (double)m, qv = (double)q;
#pragma unroll
    for (int off = FMM_WAVE / 2; off > 0; off >>= 1) {
        fv += __shfl_xor(fv, off, FMM_WAVE);
        mv += __shfl_xor(mv, off, FMM_WAVE);
        qv += __shfl_xor(qv, off, FMM_WAVE);
        pairs += __shfl_xor(pairs, off, FMM_WAVE);
    }
    __shared__ double red[WALK_THREADS / FMM_WAVE][4];
    const int w = threadIdx.x / FMM_WAVE;
    if (lane_id() == 0) {
        red[w][0] = fv;
        red[w][1] = mv;
        red[w][2] = qv;
        red[w][3] = pairs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int i = 0; i < WALK_THREADS / FMM_WAVE; ++i) {
            s0 += red[i][0];
            s1 += red[i][1];
            s2 += red[i][2];
            s3 += red[i][3];
        }
        unsigned long long *o = btot + 4 * (size_t)blockIdx.x;
        o[0] = (unsigned long long)s0;
        o[1] = (unsigned long long)s1;
        o[2] = (unsigned long long)s2;
        o[3] = (unsigned long long)s3;
    }
}

// Offsets of this block's outputs (the sum of the count pass's totals of the
// blocks before it) and, in block 0, the sweep's totals: the frontier size
// for the next sweep and the running list sizes, kept per sweep in
// counters[WALK_CUM + 3 i + k] so that no block reads a value another block of
// this launch writes.
__device__ __forceinline__ void walk_offsets(const unsigned long long *btot, bool need_prefix,
                                             unsigned long long (&pre)[3],
                                             unsigned long long (&tot)[4]) {
    const int b = blockIdx.x;
    const bool want_tot = b == 0;
    unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};   // pre[0..2], tot[0..3]
    const int jend = want_tot ? WALK_BLOCKS : (need_prefix ? b : 0);
    for (int j = threadIdx.x; j < jend; j += WALK_THREADS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned long long x = btot[4 * j + k];
            if (k < 3 && j < b) v[k] += x;
            v[3 + k] += x;
        }
    }
#pragma unroll
    for (int k = 0; k < 7; ++k)
#pragma unroll
        for (int o = FMM_WAVE / 2; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, FMM_WAVE);
    __shared__ unsigned long long red[WALK_THREADS / FMM_WAVE][7];
    const int w = threadIdx.x / FMM_WAVE;
    if (lane_id() == 0)
#pragma unroll
        for (int k = 0; k < 7; ++k) red[w][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        unsigned long long a = 0;
#pragma unroll
        for (int i = 0; i < WALK_THREADS / FMM_WAVE; ++i) a += red[i][k];
        if (k < 3) pre[k] = a;
        else tot[k - 3] = a;
    }
}

__global__ void __launch_bounds__(WALK_THREADS)
k_walk_write(WalkParams wp, TreeArrays t, const double *P, WalkBuffers wb, int sweep,
             const unsigned long long *btot) {
    unsigned long long *cnt = wb.counters;
    const int64_t n_in = sweep_input(wp, cnt, sweep);
    const int64_t chunk = (n_in + WALK_BLOCKS - 1) / WALK_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n_in, lo + chunk);
    const bool fits = n_in <= wb.cap_out;
    if (blockIdx.x != 0 && (!fits || lo >= hi)) return;   // nothing to write
    unsigned long long pre[3], tot[4];
    walk_offsets(btot, fits && lo < hi, pre, tot);
    unsigned long long *cum = cnt + WALK_CUM + 3 * sweep;   // totals before this sweep
    const unsigned long long m0 = cum[0], p0 = cum[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!fits) cnt[3] = 1ull;
        cnt[4 + sweep] = tot[0];
        cum[3] = cnt[0] = m0 + tot[1];
        cum[4] = cnt[1] = p0 + tot[2];
        cum[5] = cnt[2] = cum[2] + tot[3];
    }
    if (!fits) return;
    int64_t of = (int64_t)pre[0];
    int64_t om = (int64_t)(m0 + pre[1]);
    int64_t op = (int64_t)(p0 + pre[2]);
    // WALK_WBATCH rounds of WALK_THREADS pairs at a time: the pairs, their
    // decisions and the cell data their outputs need are loaded for all rounds
    // first, then the rounds are scanned and written in frontier order
    for (int64_t base0 = lo; base0 < hi; base0 += (int64_t)WALK_THREADS * WALK_WBATCH) {
        int A[WALK_WBATCH], B[WALK_WBATCH], kind[WALK_WBATCH], nf[WALK_WBATCH];
#pragma unroll
        for (int r = 0; r < WALK_WBATCH; ++r) {
            const int64_t i = base0 + (int64_t)r * WALK_THREADS + threadIdx.x;
            const bool v = i < hi;    // the decision the count pass took for this pair
            const uint2 pr = v ? wb.in[i] : make_uint2(0u, 0u);
            const unsigned code = v ? wb.code[i] : 0u;
            A[r] = (int)pr.x;
            B[r] = (int)pr.y;
            kind[r] = (int)(code & 7u);
            nf[r] = (int)(code >> 3);
        }
        int kA[WALK_WBATCH], kB[WALK_WBATCH], nchA[WALK_WBATCH], begA[WALK_WBATCH],
            endA[WALK_WBATCH];
#pragma unroll
        for (int r = 0; r < WALK_WBATCH; ++r) {
            kA[r] = t.child0[A[r]];
            kB[r] = t.child0[B[r]];
            nchA[r] = t.nchild[A[r]];
            begA[r] = t.beg[A[r]];
            endA[r] = t.end[A[r]];
        }
#pragma unroll
        for (int r = 0; r < WALK_WBATCH; ++r) {
            if (base0 + (int64_t)r * WALK_THREADS >= hi) break;   // uniform over the block
            const int k = kind[r], n = nf[r];
            int sf = n, sm = k == 5, sp = k == 4;
            int tot[3];
            block_scan3(sf, sm, sp, tot);
            const int64_t pf = of + sf - n, pm = om + sm - (k == 5), pp = op + sp - (k == 4);
            const int a0 = A[r], b0 = B[r];
            switch (k) {
            case 1: {   // all ordered daughter pairs of A
                const int k0 = kA[r], nch = nchA[r];
                if (pf + n <= wb.cap_out)
                    for (int a = 0; a < nch; ++a)
                        for (int b = 0; b < nch; ++b)
                            wb.out[pf + a * nch + b] = make_uint2(k0 + a, k0 + b);
                break;
            }
            case 2: {
                const int k0 = kA[r];
                if (pf + n <= wb.cap_out)
                    for (int a = 0; a < n; ++a) wb.out[pf + a] = make_uint2(k0 + a, b0);
                break;
            }
            case 3: {
                const int k0 = kB[r];
                if (pf + n <= wb.cap_out)
                    for (int b = 0; b < n; ++b) wb.out[pf + b] = make_uint2(a0, k0 + b);
                break;
            }
            case 4:     // direct sum of A's particles onto B's (B may be any cell)
                if (pp + 1 <= wb.cap_p2p) {
                    if (wp.pack) {
                        wb.p2p[pp] = ((uint64_t)b0 << (2 * wp.pb)) |
                                     ((uint64_t)begA[r] << wp.pb) | (uint64_t)endA[r];
                    } else {
                        wb.p2p[pp] = ((uint64_t)b0 << wp.pb) | (uint64_t)begA[r];
                        wb.p2p_end[pp] = (uint32_t)endA[r];
                    }
                }
                break;
            case 5:
                if (pm + 1 <= wb.cap_m2l) wb.m2l[pm] = ((uint64_t)b0 << wp.sh) | (uint64_t)a0;
                break;
            default:
                break;
            }
            of += tot[0];
            om += tot[1];
            op += tot[2];
        }
    }
}

__global__ void k_list_offsets(const uint64_t *list, int64_t nlist, int nsinks, int sh,
                               int64_t *off) {
    // list sorted by key; the sink is key >> sh
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nsinks) return;
    // first entry whose sink is >= s
    int64_t lo = 0, hi = nlist;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(list[mid] >> sh) < (int64_t)s) lo = mid + 1;
        else hi = mid;
    }
    off[s] = lo;
}

// A direct-sum entry: sink cell, first and end source particle (packed keys
// carry the end; otherwise it is in the separate array)
struct Entry {
    uint64_t sink;
    uint32_t first, end;
};
__device__ __forceinline__ Entry entry(const uint64_t *key, const uint32_t *end, int64_t e,
                                       int pb, int packed) {
    const uint64_t mask = (1ull << pb) - 1, k = key[e];
    if (packed) return {k >> (2 * pb), (uint32_t)((k >> pb) & mask), (uint32_t)(k & mask)};
    return {k >> pb, (uint32_t)(k & mask), end[e]};
}

// Direct-sum entries sorted by (sink, source begin): an entry starts a new
// range unless it continues the previous one (same sink, adjacent particles).
__global__ void k_range_flags(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int packed, int *flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > n) return;
    if (e == n) {
        flag[e] = 0;
        return;
    }
    bool start = e == 0;
    if (!start) {
        const Entry a = entry(key, end, e, pb, packed), b = entry(key, end, e - 1, pb, packed);
        start = a.sink != b.sink || a.first != b.end;
    }
    flag[e] = start ? 1 : 0;
}

// run r = [first entry's begin, last entry's end) with its key (sink << pb) | begin
__global__ void k_range_write(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int packed, const int *scan, int2 *range, uint64_t *rkey) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const Entry a = entry(key, end, e, pb, packed);
    const int starts_here = scan[e + 1] - scan[e];
    const int run = scan[e + 1] - 1;
    if (starts_here) {
        range[run].x = (int)a.first;
        rkey[run] = (a.sink << pb) | (uint64_t)a.first;
    }
    if (e == n - 1 || scan[e + 2] - scan[e + 1]) range[run].y = (int)a.end;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_range_merge(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int packed, int *flag, int *tmp, int *total, int2 *range,
                              uint64_t *rkey, bool write, hipStream_t s) {
    if (!write) {
        hipLaunchKernelGGL(k_range_flags, dim3(blocks(n + 1, 256)), dim3(256), 0, s, key, end, n,
                           pb, packed, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // flag -> exclusive scan of n + 1 entries; flag[n] = 0 so scan[n] = runs
        e = exclusive_scan(flag, flag, n + 1, tmp, total, s);
        if (e != hipSuccess) return e;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_range_write, dim3(blocks(n, 256)), dim3(256), 0, s, key, end, n, pb,
                       packed, flag, range, rkey);
    return hipGetLastError();
}

size_t walk_tmp_u64() { return 4 * (size_t)WALK_BLOCKS; }

__global__ void k_root_pairs(uint2 *f, int nroots) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nroots) f[r] = make_uint2(r, r);
}

hipError_t launch_root_pairs(uint2 *f, int nroots, hipStream_t s) {
    hipLaunchKernelGGL(k_root_pairs, dim3((nroots + 255) / 256), dim3(256), 0, s, f, nroots);
    return hipGetLastError();
}

hipError_t launch_walk(const WalkParams &wp, const TreeArrays &t, const double *P,
                       const WalkBuffers &wb, int sweep, unsigned long long *btmp, hipStream_t s) {
    hipLaunchKernelGGL(k_walk_count, dim3(WALK_BLOCKS), dim3(WALK_THREADS), 0, s, wp, t, P, wb,
                       sweep, btmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_walk_write, dim3(WALK_BLOCKS), dim3(WALK_THREADS), 0, s, wp, t, P, wb,
                       sweep, (const unsigned long long *)btmp);
    return hipGetLastError();
}

hipError_t launch_list_offsets(const uint64_t *list, int64_t nlist, int nsinks, int sh,
                               int64_t *off, hipStream_t s) {
    hipLaunchKernelGGL(k_list_offsets, dim3(blocks(nsinks + 1, 256)), dim3(256), 0, s, list, nlist,
                       nsinks, sh, off);
    return hipGetLastError();
}

}  // namespace fmm
