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
// Outputs are appended with one atomic per wavefront per list; the lists are
// sorted afterwards, which also makes their order deterministic.  An M2L entry
// is (sink cell, source cell); a direct-sum entry is (sink cell, source
// particle range), the sink being any cell: its particles are reached from
// each leaf below it through the leaf's ancestor chain.
#include "internal.h"
#include "dev.h"

namespace fmm {

namespace {

// squared distance without fused multiply-adds (the same number as the
// definition), and its correctly rounded square root
__device__ __forceinline__ double dist_rn(double4 a, double4 b) {
    const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    return __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                __dmul_rn(dz, dz)));
}

__global__ void __launch_bounds__(256)
k_walk(WalkParams wp, TreeArrays t, const double *P, WalkBuffers wb) {
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const bool valid = gi < wb.n_in;
    int nf = 0, nm = 0, np = 0;      // outputs: frontier pairs, M2L entries, P2P entries
    int kind = 0;                    // 1 self-split, 2 split A, 3 split B, 4 P2P range, 5 M2L
    int A = 0, B = 0;
    double npairs = 0.0;
    if (valid) {
        const uint2 pr = wb.in[gi];
        A = (int)pr.x;
        B = (int)pr.y;
        const int nchA = t.nchild[A], nchB = t.nchild[B];
        if (A == B) {
            if (nchA == 0) {
                kind = 4; np = 1;
                const double na = (double)(t.end[A] - t.beg[A]);
                npairs = na * (na - 1.0);
            } else {
                kind = 1; nf = nchA * nchA;
            }
        } else {
            const bool est = wp.mode == 2;
            const double4 ca = est ? t.com[A] : t.cen[A];
            const double4 cb = est ? t.com[B] : t.cen[B];
            const double r = dist_rn(ca, cb);
            const double rA = ca.w, rB = cb.w;
            bool acc;
            if (wp.mode == 1) {
                acc = rA + rB < wp.theta_crit * r;
            } else {
                acc = rA + rB < r;
                if (acc && wp.mode == 0) {
                    // Etilde M_A = 8 max/(sum) * sum_k C(p,k) P_k rho_B^{p-k} / r^p,
                    // by Horner in q = rho_B / r
                    const int p = wp.p;
                    const double *Pa = P + (size_t)A * (p + 1);
                    const double u = 1.0 / r, q = rB * u;
                    double S = Pa[0], up = 1.0, bin = 1.0;
                    for (int k = 1; k <= p; ++k) {
                        up *= u;
                        bin = bin * (double)(p - k + 1) / (double)k;
                        S = fma(S, q, bin * Pa[k] * up);
                    }
                    const double sum = rA + rB;
                    const double fac = sum > 0.0 ? 8.0 * fmax(rA, rB) / sum : 8.0;
                    acc = fac * S * u * u < wp.eps * t.smin[B];
                }
            }
            const double na = (double)(t.end[A] - t.beg[A]), nb = (double)(t.end[B] - t.beg[B]);
            if (acc) {
                if (wp.mode != 2 && na * nb < wp.p2p_pairs) {
                    kind = 4; np = 1; npairs = na * nb;
                } else {
                    kind = 5; nm = 1;
                }
            } else if (nchA == 0 && nchB == 0) {
                kind = 4; np = 1; npairs = na * nb;
            } else {
                const bool splitA = nchA > 0 && (nchB == 0 || rA > rB);
                kind = splitA ? 2 : 3;
                nf = splitA ? nchA : nchB;
            }
        }
    }
    // wavefront-aggregated reservation in the three output lists
    const int sf = wave_incl_scan(nf), sm = wave_incl_scan(nm), sp = wave_incl_scan(np);
    __shared__ unsigned long long base_s[4][3];
    const int w = threadIdx.x / FMM_WAVE;
    if (lane == FMM_WAVE - 1) {
        base_s[w][0] = sf ? atomicAdd(&wb.counters[0], (unsigned long long)sf) : 0ull;
        base_s[w][1] = sm ? atomicAdd(&wb.counters[1], (unsigned long long)sm) : 0ull;
        base_s[w][2] = sp ? atomicAdd(&wb.counters[2], (unsigned long long)sp) : 0ull;
    }
    // pair count of the direct sums, for the statistics
    double tot = npairs;
#pragma unroll
    for (int off = FMM_WAVE / 2; off > 0; off >>= 1) tot += __shfl_xor(tot, off, FMM_WAVE);
    if (lane == 0 && tot > 0.0) atomicAdd(&wb.counters[3], (unsigned long long)tot);
    __syncthreads();
    if (!valid) return;
    const int64_t of = (int64_t)base_s[w][0] + sf - nf;
    const int64_t om = (int64_t)base_s[w][1] + sm - nm;
    const int64_t op = (int64_t)base_s[w][2] + sp - np;
    const int sh = wp.sh;
    switch (kind) {
    case 1: {   // all ordered daughter pairs of A
        const int k0 = t.child0[A], nch = t.nchild[A];
        if (of + nf <= wb.cap_out)
            for (int i = 0; i < nch; ++i)
                for (int j = 0; j < nch; ++j) wb.out[of + i * nch + j] = make_uint2(k0 + i, k0 + j);
        break;
    }
    case 2: {
        const int k0 = t.child0[A];
        if (of + nf <= wb.cap_out)
            for (int i = 0; i < nf; ++i) wb.out[of + i] = make_uint2(k0 + i, B);
        break;
    }
    case 3: {
        const int k0 = t.child0[B];
        if (of + nf <= wb.cap_out)
            for (int i = 0; i < nf; ++i) wb.out[of + i] = make_uint2(A, k0 + i);
        break;
    }
    case 4:     // direct sum of A's particles onto B's (B may be any cell)
        if (op + 1 <= wb.cap_p2p) {
            wb.p2p[op] = ((uint64_t)B << wp.pb) | (uint64_t)t.beg[A];
            wb.p2p_end[op] = (uint32_t)t.end[A];
        }
        break;
    case 5:
        if (om + 1 <= wb.cap_m2l) wb.m2l[om] = ((uint64_t)B << sh) | (uint64_t)A;
        break;
    default:
        break;
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

// Direct-sum entries sorted by (sink, source begin): an entry starts a new
// range unless it continues the previous one (same sink, adjacent particles).
__global__ void k_range_flags(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int *flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > n) return;
    if (e == n) {
        flag[e] = 0;
        return;
    }
    const uint64_t mask = (1ull << pb) - 1;
    bool start = e == 0;
    if (!start) {
        const uint64_t k = key[e], q = key[e - 1];
        start = (k >> pb) != (q >> pb) || (uint32_t)(k & mask) != end[e - 1];
    }
    flag[e] = start ? 1 : 0;
}

// run r = [first entry's begin, last entry's end) with its sink
__global__ void k_range_write(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              const int *scan, int2 *range, uint64_t *rkey) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t mask = (1ull << pb) - 1;
    const int starts_here = scan[e + 1] - scan[e];
    const int run = scan[e + 1] - 1;
    if (starts_here) {
        range[run].x = (int)(key[e] & mask);
        rkey[run] = key[e];
    }
    if (e == n - 1 || scan[e + 2] - scan[e + 1]) range[run].y = (int)end[e];
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_range_merge(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int *flag, int *tmp, int *total, int2 *range, uint64_t *rkey,
                              bool write, hipStream_t s) {
    if (!write) {
        hipLaunchKernelGGL(k_range_flags, dim3(blocks(n + 1, 256)), dim3(256), 0, s, key, end, n,
                           pb, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // flag -> exclusive scan of n + 1 entries; flag[n] = 0 so scan[n] = runs
        e = exclusive_scan(flag, flag, n + 1, tmp, total, s);
        if (e != hipSuccess) return e;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_range_write, dim3(blocks(n, 256)), dim3(256), 0, s, key, end, n, pb, flag,
                       range, rkey);
    return hipGetLastError();
}

hipError_t launch_walk(const WalkParams &wp, const TreeArrays &t, const double *P,
                       const WalkBuffers &wb, hipStream_t s) {
    if (wb.n_in <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk, dim3(blocks(wb.n_in, 256)), dim3(256), 0, s, wp, t, P, wb);
    return hipGetLastError();
}

hipError_t launch_list_offsets(const uint64_t *list, int64_t nlist, int nsinks, int sh,
                               int64_t *off, hipStream_t s) {
    hipLaunchKernelGGL(k_list_offsets, dim3(blocks(nsinks + 1, 256)), dim3(256), 0, s, list, nlist,
                       nsinks, sh, off);
    return hipGetLastError();
}

}  // namespace fmm
