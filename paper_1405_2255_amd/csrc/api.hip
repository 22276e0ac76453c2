// libfmm C ABI and the host-side orchestration of one force evaluation.
//
// Phases (the columns of the paper's tab:complexity):
//   tree      keys, radix sort, gather, octree levels, leaves, geometry, radii
//   estimate  low-order FMM for the sink scale (Sec. 5.4.2) and its minimum
//             per cell, or the previous call's |a| (Sec. 5.4.1)
//   up        P2M, M2M, multipole power
//   walk      breadth-first dual tree walk -> M2L and P2P lists; M2L; P2P
//   down      L2L, L2P, output
// Everything is ordered on one stream.  The host reads back a few counters
// (cells per tree level, pairs per walk sweep) to size the next launch.
#include "../../include/fmm.h"
#include "internal.h"
#include "jerk.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace fmm {
namespace {

struct HipFail {
    hipError_t e;
    const char *what;
};
struct NoMem {
    size_t bytes;
};

#define CK(call)                                              \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) throw HipFail{e_, #call};       \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

template <class T>
T *ensure(DevBuf &b, size_t count, bool keep = false, size_t keep_count = 0) {
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (b.cap >= bytes) return static_cast<T *>(b.p);
    const size_t want = bytes + bytes / 4;
    void *q = nullptr;
    if (hipMalloc(&q, want) != hipSuccess) {
        (void)hipGetLastError();
        throw NoMem{want};
    }
    if (b.p) {
        // the old buffer may still be in use by queued work on any stream
        CK(hipDeviceSynchronize());
        if (keep && keep_count)
            CK(hipMemcpy(q, b.p, std::min(keep_count * sizeof(T), b.cap), hipMemcpyDeviceToDevice));
        CK(hipFree(b.p));
    }
    b.p = q;
    b.cap = want;
    return static_cast<T *>(q);
}

template <class T>
T *ptr(DevBuf &b) { return static_cast<T *>(b.p); }

int bitlen(uint64_t v) {
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

enum Phase { PH_START, PH_TREE, PH_EST, PH_UP, PH_WALK, PH_M2L, PH_P2P, PH_DOWN, PH_END, PH_N };

}  // namespace
}  // namespace fmm

// small kernels used only by the orchestration: gather of the previous
// call's |a| into key order, and |a|/G of a result
namespace fmm {
__global__ void k_gather_scale(const double *src, const uint32_t *perm, int64_t n, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}
__global__ void k_norm3(const double *acc, int64_t n, double invG, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = acc[3 * i], b = acc[3 * i + 1], c = acc[3 * i + 2];
    out[i] = sqrt(a * a + b * b + c * c) * invG;
}
hipError_t launch_gather_scale(const double *src, const uint32_t *perm, int64_t n, double *dst,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_gather_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       perm, n, dst);
    return hipGetLastError();
}
hipError_t launch_norm3(const double *acc, int64_t n, double G, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_norm3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, n,
                       1.0 / G, out);
    return hipGetLastError();
}
}  // namespace fmm

using namespace fmm;

// entries of the pinned host mirror of the walk counters: 4 totals plus one
// frontier size per sweep (at most 2 * FMM_MAXLEVEL + 4 sweeps)
constexpr int HCNT = 128;

struct fmm_ctx {
    fmm_opts opts{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // side stream for the enclosing-sphere centres, forked from and joined
    // back into `stream` by the two events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool join_pending = false;
    std::atomic<int> busy{0};
    std::string err;
    fmm_stats_t st{};

    // particles
    DevBuf bbox, key, key2, idx, idx2, x, y, z, m, xyzm, leaf_of, out4, est4, scale, flags, tmp,
        tmp_side;
    uint32_t *perm = nullptr;  // points into idx or idx2
    // cells
    DevBuf beg, end, parent, child0, nchild, level, leaf_lo, leaf_hi, cen, com, mass, lo, hi,
        rho2, bsph, smin, leaf_cell, M, F, P, U, Fe;
    // walk
    DevBuf fa, fb, m2l, m2l2, p2p, p2p2, p2pe, p2pe2, m2l_off, p2p_off, chunks, ccnt, coff, Fpart;
    DevBuf rflag, ranges, rkey, wcode, rup;
    DevBuf pt_n, pt_m, pt_s, pt_off, pt_moff, ptasks, pchain, ppart;
    DevBuf counters, nonfinite, walktmp, coffsets, ckey, ckey2, order, order2;
    DevBuf actflag, actf, actinv, actpre, cellact, actbad;   // forces for a listed subset
    DevBuf epsmin;                                           // smallest individual eps
    DevBuf vel4, Md, Fd, jFpart, jo4, jpart;   // jerk: velocities, rates of M and F, M2L
                                               // chunk parts of the rates, jerk per
                                               // particle, direct-sum partial rows
    DevBuf dkey, dsort, dsort2, runstart;   // deep refinement below level 21
    DevBuf plans;                          // output plans of M2M and L2L for order plan_p
    DevBuf Tsh;                            // M2M: each cell's expansion shifted to its parent
    DevBuf tg, tpre, tsuf, tcell, tcell2, tls;   // tree build: window maxima, cells, levels
    DevBuf M32, sig, Flow;                 // mixed-precision M2L: scaled multipoles, chunk
                                           // scales, FP64 low-degree chunk parts
    DevBuf dspart;                         // exact sums for listed sinks: partial rows
    void *scratch = nullptr;   // device address of this device's static scratch array
    int plan_p = -1;
    uint64_t *kdeep = nullptr;            // second key word of the sorted particles
    bool deep = false;
    void *pin = nullptr;      // pinned staging for host-to-device copies
    size_t pin_cap = 0;
    int nroots = 0;
    bool tree_valid = false, refitted = false;
    int64_t tree_n = -1;
    std::vector<int64_t> tree_off;
    unsigned long long *hcnt = nullptr;  // pinned host mirror of the counters (HCNT entries)
    int *hint = nullptr;                 // pinned host ints
    // last call
    int64_t n = 0;
    int ncells = 0, nleaves = 0, depth = 0, sh = 0, pb = 0, p = 0;
    int pack = 0;   // direct-sum keys carry the range end (sh + 2 pb <= 64)
    int walk_used[3] = {0, 0, 0};   // sweeps the last walk of each mode needed
    int64_t n_m2l = 0, n_p2p = 0, n_ranges = 0;
    uint64_t *m2l_sorted = nullptr, *p2p_sorted = nullptr;
    uint32_t *p2pe_sorted = nullptr;
    std::vector<int> ls;  // first cell of each level
    bool have_prev_scale = false;
    int64_t prev_n = -1;
    DevBuf prev_scale;    // |a| of the last call, input order
    hipEvent_t ev[PH_N] = {};
    hipEvent_t ev_m2l[2] = {}, ev_p2p[2] = {}, ev_walk[2] = {};
    int64_t last_walk_pairs = 0;
    double last_sweep_ms = 0;
    double t_m2l_kernel = 0, t_p2p_kernel = 0;
};

namespace fmm {
namespace {

TreeArrays tree_arrays(fmm_ctx *c) {
    TreeArrays t;
    t.beg = ptr<int>(c->beg); t.end = ptr<int>(c->end); t.parent = ptr<int>(c->parent);
    t.child0 = ptr<int>(c->child0); t.nchild = ptr<int>(c->nchild); t.level = ptr<int>(c->level);
    t.leaf_lo = ptr<int>(c->leaf_lo); t.leaf_hi = ptr<int>(c->leaf_hi);
    t.cen = ptr<double4>(c->cen); t.com = ptr<double4>(c->com); t.mass = ptr<double>(c->mass);
    t.lo = ptr<double>(c->lo); t.hi = ptr<double>(c->hi);
    t.rho2 = ptr<unsigned long long>(c->rho2); t.smin = ptr<double>(c->smin);
    t.bsph = ptr<double4>(c->bsph);
    return t;
}

void sync(fmm_ctx *c) { CK(hipStreamSynchronize(c->stream)); }

void mark(fmm_ctx *c, int ph) {
    if (c->opts.timing) CK(hipEventRecord(c->ev[ph], c->stream));
}

int *tmp_ints(fmm_ctx *c, size_t count) { return ensure<int>(c->tmp, count); }

// ------------------------------------------------------------------ tree
void grow_cells(fmm_ctx *c, int need, int have) {
    const size_t cap = c->beg.cap / sizeof(int);
    if ((size_t)need <= cap) return;
    const size_t nc = std::max<size_t>(need, cap * 2);
    for (DevBuf *b : {&c->beg, &c->end, &c->parent, &c->child0, &c->nchild, &c->level})
        ensure<int>(*b, nc, true, (size_t)have);
}

void *pinned(fmm_ctx *c, size_t bytes) {
    if (c->pin_cap < bytes) {
        if (c->pin) CK(hipHostFree(c->pin));
        c->pin = nullptr;
        c->pin_cap = 0;
        CK(hipHostMalloc(&c->pin, bytes, hipHostMallocDefault));
        c->pin_cap = bytes;
    }
    return c->pin;
}

// K clusters, cluster k = particles [off[k], off[k+1]) (host offsets)
// With refit (and the same n and clusters as the tree on the context) the
// particle order and cell membership of the last build are kept - tree
// recycling between nearby time steps - and only positions, geometry and
// radii are refreshed.  The acceptance test uses the true radii, so a
// recycled tree stays valid; it only gets less efficient as particles drift.
void join_side(fmm_ctx *c);

void build_tree(fmm_ctx *c, int64_t n, const double *pos, const double *mass, int K,
                const int64_t *off, bool refit) {
    hipStream_t s = c->stream;
    join_side(c);   // a previous call that ended early may have left side work queued
    const int leaf = c->opts.leaf_size;
    const bool reuse = refit && c->tree_valid && c->tree_n == n &&
                       c->tree_off == std::vector<int64_t>(off, off + K + 1);
    double *x = ensure<double>(c->x, n), *y = ensure<double>(c->y, n), *z = ensure<double>(c->z, n),
           *m = ensure<double>(c->m, n);
    double4 *xyzm = ensure<double4>(c->xyzm, n);
    c->refitted = reuse;
    if (reuse) {
        CK(launch_gather(pos, mass, c->perm, n, x, y, z, m, xyzm, s));
    } else {
    c->tree_valid = false;
    // cluster offsets and the roots (non-empty clusters) to the device
    // (the roots, one per non-empty cluster, are the level-0 cells of the build)
    int R = 0;
    for (int k = 0; k < K; ++k) R += off[k + 1] > off[k];
    char *pin = static_cast<char *>(pinned(c, sizeof(int64_t) * (K + 1)));
    std::memcpy(pin, off, sizeof(int64_t) * (K + 1));
    int64_t *doff = ensure<int64_t>(c->coffsets, (size_t)K + 1);
    CK(hipMemcpyAsync(doff, pin, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, s));
    c->nroots = R;
    // keys in each cluster's cube, sort by key and then (stably) by cluster
    unsigned long long *bb = ensure<unsigned long long>(c->bbox, 6 * (size_t)std::max(K, 1 + BBOX_WAVES));
    uint64_t *k1 = ensure<uint64_t>(c->key, n), *k2 = ensure<uint64_t>(c->key2, n);
    uint32_t *i1 = ensure<uint32_t>(c->idx, n), *i2 = ensure<uint32_t>(c->idx2, n);
    CK(launch_bbox(pos, n, K, doff, bb, s));
    CK(launch_keys(pos, n, K, doff, bb, k1, i1, s));
    int *tmp = tmp_ints(c, std::max(sort_tmp_ints(n), scan_tmp_ints(n + 1)));
    CK(radix_sort(&k1, &k2, &i1, &i2, n, 63, tmp, s));
    if (K > 1) {
        uint64_t *c1 = ensure<uint64_t>(c->ckey, n), *c2 = ensure<uint64_t>(c->ckey2, n);
        uint32_t *o1 = ensure<uint32_t>(c->order, n), *o2 = ensure<uint32_t>(c->order2, n);
        CK(launch_cluster_keys(i1, n, K, doff, c1, o1, s));
        CK(radix_sort(&c1, &c2, &o1, &o2, n, std::max(1, bitlen((uint64_t)(K - 1))), tmp, s));
        CK(launch_apply_order(o1, k1, i1, n, k2, i2, s));
        std::swap(k1, k2);
        std::swap(i1, i2);
    }
    // level-21 cells with more than `leaf` particles get a second key word;
    // each such run is re-sorted by (second word, position)
    uint64_t *kd = ensure<uint64_t>(c->dkey, n);
    {
        uint64_t *rs = ensure<uint64_t>(c->runstart, n);
        uint64_t *sa = ensure<uint64_t>(c->dsort, n), *sb = ensure<uint64_t>(c->dsort2, n);
        uint32_t *o1 = ensure<uint32_t>(c->order, n), *o2 = ensure<uint32_t>(c->order2, n);
        int *any = ptr<int>(c->nonfinite) + 4;
        CK(hipMemsetAsync(any, 0, sizeof(int), s));
        CK(launch_deep_keys(pos, i1, k1, n, K, doff, bb, leaf, kd, rs, o1, any, s));
        CK(hipMemcpyAsync(c->hint, any, sizeof(int), hipMemcpyDeviceToHost, s));
        sync(c);
        c->deep = c->hint[0] != 0;
        if (c->deep) {
            CK(hipMemcpyAsync(sa, kd, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
            CK(radix_sort(&sa, &sb, &o1, &o2, n, 63, tmp, s));          // by (second word, position)
            CK(launch_gather_u64(o1, rs, n, sb, s));                     // run of each
            CK(radix_sort(&sb, &sa, &o1, &o2, n, std::max(1, bitlen((uint64_t)n)), tmp, s));
            // sa is free now: it receives the second words in the final order
            CK(launch_apply_order2(o1, k1, kd, i1, n, k2, sa, i2, s));
            std::swap(k1, k2);
            std::swap(i1, i2);
            kd = sa;
        }
    }
    c->kdeep = kd;
    c->perm = i1;
    CK(launch_gather(pos, mass, c->perm, n, x, y, z, m, xyzm, s));
    // octree: every cell of every level from the run structure of the keys
    int *tg = ensure<int>(c->tg, n), *tpre = ensure<int>(c->tpre, n);
    int *tsuf = ensure<int>(c->tsuf, n);
    int *tcnt = ensure<int>(c->flags, n + 2);
    int *total = ptr<int>(c->nonfinite) + 1;
    CK(launch_tree(k1, kd, n, K, doff, leaf, tg, tpre, tsuf, tcnt, s));
    CK(exclusive_scan(tcnt, tcnt, n + 1, tmp, total, s));
    CK(hipMemcpyAsync(c->hint, total, sizeof(int), hipMemcpyDeviceToHost, s));
    sync(c);
    const int nc_all = c->hint[0];
    uint64_t *cl1 = ensure<uint64_t>(c->tcell, nc_all), *cl2 = ensure<uint64_t>(c->tcell2, nc_all);
    CK(launch_tree_emit(k1, kd, n, K, doff, leaf, tpre, tsuf, tcnt, cl1, s));
    int *tmp2 = tmp_ints(c, std::max({sort_tmp_ints(n), scan_tmp_ints(n + 1),
                                      sort_tmp_ints(nc_all)}));
    CK(radix_sort(&cl1, &cl2, nullptr, nullptr, nc_all, 6, tmp2, s, 32));   // by level, stable
    int *dls = ensure<int>(c->tls, FMM_MAXLEVEL + 2);
    CK(launch_tree_levels(cl1, nc_all, dls, s));
    grow_cells(c, nc_all, 0);
    TreeArrays t = tree_arrays(c);
    CK(launch_tree_cells(k1, kd, n, K, doff, cl1, nc_all, dls, t, s));
    int hls[FMM_MAXLEVEL + 2];
    static_assert(sizeof(hls) <= HCNT * sizeof(unsigned long long), "level table mirror");
    CK(hipMemcpyAsync(c->hcnt, dls, sizeof(hls), hipMemcpyDeviceToHost, s));
    sync(c);
    std::memcpy(hls, c->hcnt, sizeof(hls));
    tmp = tmp2;
    // ls[L] = first cell of level L up to the deepest level, then ncells twice
    c->ls.clear();
    for (int L = 0; L <= FMM_MAXLEVEL + 1; ++L) {
        c->ls.push_back(hls[L]);
        if (hls[L] == nc_all) break;
    }
    c->ls.push_back(nc_all);
    const int ncells = c->ls.back();
    c->ncells = ncells;
    c->depth = (int)c->ls.size() - 3;   // ls ends with two equal entries
    c->sh = std::max(1, bitlen((uint64_t)ncells));
    c->pb = std::max(1, bitlen((uint64_t)n));
    c->pack = c->sh + 2 * c->pb <= 64;
    // per-cell arrays sized now that the count is known
    ensure<int>(c->leaf_lo, ncells); ensure<int>(c->leaf_hi, ncells);
    ensure<double4>(c->cen, ncells); ensure<double4>(c->com, ncells);
    ensure<double>(c->mass, ncells); ensure<double>(c->lo, 3 * (size_t)ncells);
    ensure<double>(c->hi, 3 * (size_t)ncells); ensure<unsigned long long>(c->rho2, 3 * (size_t)ncells);
    ensure<double4>(c->bsph, ncells);
    ensure<double>(c->smin, ncells);
    t = tree_arrays(c);
    // leaves in key order
    int *flags = ensure<int>(c->flags, n + 2);
    CK(hipMemsetAsync(flags, 0, sizeof(int) * (n + 1), s));
    CK(launch_leaf_flags(t, ncells, flags, s));
    CK(exclusive_scan(flags, flags, n + 1, tmp, total, s));
    CK(hipMemcpyAsync(c->hint, total, sizeof(int), hipMemcpyDeviceToHost, s));
    int *leaf_cell = ensure<int>(c->leaf_cell, ncells);
    int *leaf_of = ensure<int>(c->leaf_of, n);
    CK(launch_leaf_ranges(t, ncells, flags, leaf_cell, leaf_of, n, s));
    sync(c);
    c->nleaves = c->hint[0];
    c->tree_valid = true;
    c->tree_n = n;
    c->tree_off.assign(off, off + K + 1);
    }
    const int ncells = c->ncells;
    TreeArrays t = tree_arrays(c);
    const int *leaf_of = ptr<int>(c->leaf_of), *leaf_cell = ptr<int>(c->leaf_cell);
    // geometry bottom up, then the radii about the midpoints and the centres
    // of mass of every cell in one pass
    for (int L = c->depth; L >= 0; --L)
        CK(launch_geometry_level(t, c->ls[L], c->ls[L + 1], x, y, z, m, s));
    CK(launch_radii(t, n, leaf_of, leaf_cell, c->depth, x, y, z, false, s));
    CK(launch_radii_finish(t, ncells, s));
    if (c->opts.centre != FMM_CENTRE_MIDPOINT) {
        // The enclosing-sphere centres: a chain of small latency-bound
        // launches, one per level.  They run on the side stream while the
        // main stream does the sink-scale estimate, which uses only the
        // centres of mass; join_side() orders the main stream after them
        // before anything reads an expansion centre.
        CK(hipEventRecord(c->ev_fork, s));
        CK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
        for (int L = c->depth; L >= 0; --L)
            CK(launch_enclosing_level(t, c->ls[L], c->ls[L + 1], x, y, z, c->side));
        CK(launch_radii(t, n, leaf_of, leaf_cell, c->depth, x, y, z, true, c->side));
        CK(launch_centre_select(t, ncells, c->side));
        CK(hipEventRecord(c->ev_join, c->side));
        c->join_pending = true;
    }
}

// the main stream waits for the work queued on the side stream (enclosing
// centres, upward pass, direct-sum lists), if any is pending
void join_side(fmm_ctx *c) {
    if (!c->join_pending) return;
    CK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    c->join_pending = false;
}

// ------------------------------------------------------------------ walk
struct Lists {
    uint64_t *m2l;
    int64_t n_m2l;
    uint64_t *p2p;
    uint32_t *p2p_end;
    int64_t n_p2p;
    int64_t pairs;
    int iterations;
};

Lists walk(fmm_ctx *c, const WalkParams &wp0, const double *P) {
    static_assert(4 + 2 * FMM_MAXLEVEL + 4 <= HCNT, "counter mirror too small for the deepest tree");
    hipStream_t s = c->stream;
    WalkParams wp = wp0;
    wp.nroots = c->nroots;
    wp.sh = c->sh;
    wp.pb = c->pb;
    wp.pack = c->pack;
    wp.binom[0] = 1.0;
    for (int k = 1; k <= std::min(wp.p, FMM_PMAX); ++k)
        wp.binom[k] = wp.binom[k - 1] * (double)(wp.p - k + 1) / (double)k;
    const int64_t n = c->n;
    // every sweep descends one level in A or in B
    const int sweeps = 2 * c->depth + 4;
    int64_t cap_f = std::max<int64_t>({1024, 2 * n, (int64_t)c->nroots, (int64_t)(c->fa.cap / 8)});
    int64_t cap_m = std::max<int64_t>(1024, c->m2l.cap ? (int64_t)(c->m2l.cap / 8) : 8 * n);
    int64_t cap_p = std::max<int64_t>(1024, c->p2p.cap ? (int64_t)(c->p2p.cap / 8) : 4 * n);
    unsigned long long *cnt = ensure<unsigned long long>(c->counters, WALK_CUM + 3 * (sweeps + 1));
    unsigned long long *btmp = ensure<unsigned long long>(c->walktmp, walk_tmp_u64());
    const TreeArrays t = tree_arrays(c);
    for (;;) {
        uint2 *fa = ensure<uint2>(c->fa, cap_f), *fb = ensure<uint2>(c->fb, cap_f);
        uint64_t *ml = ensure<uint64_t>(c->m2l, cap_m), *pl = ensure<uint64_t>(c->p2p, cap_p);
        uint32_t *pe = ensure<uint32_t>(c->p2pe, cap_p);
        uint16_t *code = ensure<uint16_t>(c->wcode, cap_f);
        CK(hipMemsetAsync(cnt, 0, (WALK_CUM + 3 * (sweeps + 1)) * sizeof(unsigned long long), s));
        CK(launch_root_pairs(fa, c->nroots, s));           // (r, r) for every root
        if (c->opts.timing) CK(hipEventRecord(c->ev_walk[0], s));
        // as many sweeps as the last walk of this kind needed (plus one), more
        // only while the frontier is not empty; at most `sweeps`
        int target = c->walk_used[wp.mode] > 0 ? std::min(sweeps, c->walk_used[wp.mode] + 1)
                                               : sweeps;
        int launched = 0;
        for (;;) {
            for (int i = launched; i < target; ++i) {
                WalkBuffers wb{(i & 1) ? fb : fa, (i & 1) ? fa : fb, cap_f, ml, cap_m, pl, pe,
                               cap_p, cnt, code};
                CK(launch_walk(wp, t, P, wb, i, btmp, s));
            }
            launched = target;
            if (c->opts.timing) CK(hipEventRecord(c->ev_walk[1], s));
            CK(hipMemcpyAsync(c->hcnt, cnt, (4 + sweeps) * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
            sync(c);
            if (c->hcnt[4 + launched - 1] == 0 || launched >= sweeps) break;
            target = std::min(sweeps, launched + 4);
        }
        const unsigned long long *h = c->hcnt;
        int64_t maxf = 0, visited = 1;
        int used = 0;
        for (int i = 0; i < sweeps; ++i) {
            maxf = std::max<int64_t>(maxf, (int64_t)h[4 + i]);
            visited += (int64_t)h[4 + i];
            if (h[4 + i]) used = i + 1;
        }
        c->last_walk_pairs = visited;
        if (c->opts.timing) {
            float ms = 0;
            CK(hipEventElapsedTime(&ms, c->ev_walk[0], c->ev_walk[1]));
            c->last_sweep_ms = ms;
        }
        const bool of = maxf > cap_f || (int64_t)h[0] > cap_m || (int64_t)h[1] > cap_p || h[3];
        if (of) {   // grow what overflowed and redo the walk
            if (maxf > cap_f || h[3]) cap_f = std::max(2 * cap_f, maxf + maxf / 2);
            if ((int64_t)h[0] > cap_m) cap_m = (int64_t)h[0] + (int64_t)h[0] / 2;
            if ((int64_t)h[1] > cap_p) cap_p = (int64_t)h[1] + (int64_t)h[1] / 2;
            continue;
        }
        if (h[4 + launched - 1] != 0) throw HipFail{hipErrorUnknown, "walk did not terminate"};
        c->walk_used[wp.mode] = used + 1;
        return Lists{ml, (int64_t)h[0], pl, pe, (int64_t)h[1], (int64_t)h[2], used + 1};
    }
}

// group a list (sink << sh | source) by sink and compute the per-sink
// offsets.  The sort is stable and keys only on the sink bits, so each sink's
// sources keep the walk's (deterministic) order; the M2L kernels take a
// sink's sources in any order.
uint64_t *sort_list(fmm_ctx *c, DevBuf &a, DevBuf &b, int64_t nlist, int nsinks, DevBuf &offb) {
    uint64_t *k1 = ptr<uint64_t>(a);
    uint64_t *k2 = ensure<uint64_t>(b, std::max<int64_t>(nlist, 1));
    int *tmp = tmp_ints(c, sort_tmp_ints(nlist));
    CK(radix_sort(&k1, &k2, nullptr, nullptr, nlist, c->sh, tmp, c->stream, c->sh));
    int64_t *off = ensure<int64_t>(offb, (size_t)nsinks + 1);
    CK(launch_list_offsets(k1, nlist, nsinks, c->sh, off, c->stream));
    return k1;
}

// sort the direct-sum entries by (sink cell, first source particle), merge
// adjacent source ranges of each sink and index the ranges by sink cell.
// by_source false: by sink cell only (stable, so each sink keeps the walk's
// order), merging the ranges that the walk emitted next to each other - two
// radix passes fewer; used for the estimate's short lists, where the longer
// range lists cost the direct-sum kernel nothing measurable
// side: on the side stream, with its own scratch, device counter and host
// slot, so that it can run while the main stream does M2L (the caller joins
// the side stream before the lists are used)
void prepare_p2p(fmm_ctx *c, int64_t nlist, bool by_source, bool side = false) {
    const hipStream_t s = side ? c->side : c->stream;
    uint64_t *k1 = ptr<uint64_t>(c->p2p);
    uint64_t *k2 = ensure<uint64_t>(c->p2p2, std::max<int64_t>(nlist, 1));
    uint32_t *v1 = ptr<uint32_t>(c->p2pe);
    uint32_t *v2 = ensure<uint32_t>(c->p2pe2, std::max<int64_t>(nlist, 1));
    const size_t ntmp = std::max(sort_tmp_ints(nlist), scan_tmp_ints(nlist + 1));
    int *tmp = side ? ensure<int>(c->tmp_side, ntmp) : tmp_ints(c, ntmp);
    // packed keys (the range end in the low pb bits) sort without a value array
    // key bits sorted on: (sink, first particle), or the sink alone
    const int first = c->pack ? c->pb : 0;   // lowest bit of the first particle
    const int lo = by_source ? first : first + c->pb;
    const int bits = by_source ? c->sh + c->pb : c->sh;
    if (c->pack) CK(radix_sort(&k1, &k2, nullptr, nullptr, nlist, bits, tmp, s, lo));
    else CK(radix_sort(&k1, &k2, &v1, &v2, nlist, bits, tmp, s, lo));
    c->p2p_sorted = k1;
    c->p2pe_sorted = v1;
    int *flag = ensure<int>(c->rflag, (size_t)nlist + 2);
    int2 *rg = ensure<int2>(c->ranges, std::max<int64_t>(nlist, 1));
    uint64_t *rk = ensure<uint64_t>(c->rkey, std::max<int64_t>(nlist, 1));
    int *total = ptr<int>(c->nonfinite) + (side ? 3 : 1);
    int *host = c->hint + (side ? 3 : 0);
    int64_t runs = 0;
    if (nlist > 0) {
        CK(launch_range_merge(k1, v1, nlist, c->pb, c->pack, flag, tmp, total, rg, rk, false, s));
        CK(hipMemcpyAsync(host, total, sizeof(int), hipMemcpyDeviceToHost, s));
        CK(launch_range_merge(k1, v1, nlist, c->pb, c->pack, flag, tmp, total, rg, rk, true, s));
        CK(hipStreamSynchronize(s));
        runs = *host;
    }
    c->n_ranges = runs;
    int64_t *off = ensure<int64_t>(c->p2p_off, (size_t)c->ncells + 1);
    CK(launch_list_offsets(rk, runs, c->ncells, c->pb, off, s));
}

// direct sums of every leaf (prepared ranges), added into out4; with v4 (sorted
// velocities) the FP64 kernel that also adds each pair's jerk into jo4
// Direct-sum tasks of the prepared lists: per leaf the task counts, the
// ancestor chains and the task list (active: leaves without listed sinks get
// none).  side: on the side stream with its own scratch, counters and host
// slots (the caller joins the side stream before the tasks run).
struct P2PPlan {
    int ntasks = 0, prows = 0;
    int2 *tasks = nullptr;
    int *nts = nullptr, *moff = nullptr, *chain = nullptr, *up = nullptr;
};

P2PPlan plan_p2p(fmm_ctx *c, const uint8_t *active, bool side = false) {
    const hipStream_t s = side ? c->side : c->stream;
    const int nl = c->nleaves;
    TreeArrays t = tree_arrays(c);
    P2PPlan pl;
    int *ntask = ensure<int>(c->pt_n, (size_t)nl + 1), *mtask = ensure<int>(c->pt_m, (size_t)nl + 1);
    pl.nts = ensure<int>(c->pt_s, (size_t)nl + 1);
    int *toff = ensure<int>(c->pt_off, (size_t)nl + 1);
    pl.moff = ensure<int>(c->pt_moff, (size_t)nl + 1);
    int *tmp = side ? ensure<int>(c->tmp_side, scan_tmp_ints(nl + 1)) : tmp_ints(c, scan_tmp_ints(nl + 1));
    int *totals = ptr<int>(c->nonfinite) + (side ? 6 : 1);
    int *host = c->hint + (side ? 4 : 0);
    const int64_t *off = ptr<int64_t>(c->p2p_off);
    const int2 *rg = ptr<int2>(c->ranges);
    pl.up = ensure<int>(c->rup, (size_t)std::max(c->ncells, 1));
    CK(launch_range_up(c->ncells, t.parent, off, pl.up, s));
    pl.chain = ensure<int>(c->pchain, (size_t)std::max(nl, 1) * P2P_CHAIN);
    CK(launch_p2p_plan(nl, ptr<int>(c->leaf_cell), off, rg, pl.up, t, active, ntask, mtask, pl.nts,
                       toff, pl.moff, pl.chain, tmp, totals, s));
    CK(hipMemcpyAsync(host, totals, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    pl.ntasks = host[0];
    pl.prows = host[1];
    pl.tasks = ensure<int2>(c->ptasks, std::max(pl.ntasks, 1));
    CK(launch_p2p_tasks(nl, toff, pl.tasks, s));
    return pl;
}

// the direct sums of a plan, added into out4 (and the jerk into jo4)
void exec_p2p(fmm_ctx *c, const P2PPlan &pl, int want_f, int with_pot, int mixed, double4 *out4,
              bool timed, const double4 *v4 = nullptr, double4 *jo4 = nullptr) {
    hipStream_t s = c->stream;
    TreeArrays t = tree_arrays(c);
    const int64_t *off = ptr<int64_t>(c->p2p_off);
    const int2 *rg = ptr<int2>(c->ranges);
    double4 *part = ensure<double4>(c->ppart, (size_t)std::max(pl.prows, 1) * 64);
    if (timed && c->opts.timing) CK(hipEventRecord(c->ev_p2p[0], s));
    double4 *jpart = nullptr;
    if (v4) {
        jpart = ensure<double4>(c->jpart, (size_t)std::max(pl.prows, 1) * 64);
        CK(launch_p2p_jerk(pl.ntasks, pl.tasks, ptr<int>(c->leaf_cell), pl.nts, pl.moff, off, rg,
                           pl.up, t, ptr<double4>(c->xyzm), v4, out4, jo4, part, jpart, s));
    } else {
        CK(launch_p2p(want_f, with_pot, mixed, pl.ntasks, pl.tasks, ptr<int>(c->leaf_cell), pl.nts,
                      pl.moff, off, rg, pl.chain, t, ptr<double4>(c->xyzm), out4, part, s));
    }
    if (timed && c->opts.timing) CK(hipEventRecord(c->ev_p2p[1], s));
    if (pl.prows > 0) {
        CK(launch_p2p_reduce(c->n, ptr<int>(c->leaf_of), ptr<int>(c->leaf_cell), pl.nts, pl.moff,
                             t, part, out4, s));
        if (v4)
            CK(launch_p2p_reduce(c->n, ptr<int>(c->leaf_of), ptr<int>(c->leaf_cell), pl.nts,
                                 pl.moff, t, jpart, jo4, s));
    }
}

void run_p2p(fmm_ctx *c, int want_f, int with_pot, int mixed, double4 *out4, bool timed,
             const uint8_t *active = nullptr, const double4 *v4 = nullptr,
             double4 *jo4 = nullptr) {
    exec_p2p(c, plan_p2p(c, active), want_f, with_pot, mixed, out4, timed, v4, jo4);
}

// ------------------------------------------------------------ sink scale
// eps_b (input order, device) when not null: individual accuracy parameters
// folded into the scale, min_B{eps_b a_b} (Sec. 7)
void sink_scale(fmm_ctx *c, bool want_f, const double *eps_b) {
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    TreeArrays t = tree_arrays(c);
    double *scale = ensure<double>(c->scale, n);
    bool done = false;
    if (c->opts.scale_source == FMM_SCALE_PREVIOUS && !want_f && c->have_prev_scale &&
        c->prev_n == n && c->refitted) {
        // previous call's |a| (input order) gathered into key order
        CK(launch_gather_scale(ptr<double>(c->prev_scale), c->perm, n, scale, s));
        done = true;
    }
    if (!done) {
        WalkParams wp{2, 1, 0.0, 1.0, 0.0, 0, 0, 0, {}};
        Lists L = walk(c, wp, nullptr);
        c->st.est_walk_pairs = c->last_walk_pairs;
        c->st.t_est_sweeps = c->last_sweep_ms;
        c->st.n_est_m2l = L.n_m2l;
        c->st.n_est_p2p_pairs = L.pairs;
        uint64_t *ml = sort_list(c, c->m2l, c->m2l2, L.n_m2l, c->ncells, c->m2l_off);
        prepare_p2p(c, L.n_p2p, false);
        double4 *Fe = ensure<double4>(c->Fe, c->ncells);
        CK(launch_est_m2l(want_f, t, c->ncells, ptr<int64_t>(c->m2l_off), ml, c->sh, Fe, s));
        for (int Lv = 1; Lv <= c->depth; ++Lv)
            CK(launch_est_l2l_level(want_f, t, c->ls[Lv], c->ls[Lv + 1], Fe, s));
        double4 *e4 = ensure<double4>(c->est4, n);
        CK(launch_est_l2p(want_f, t, ptr<int>(c->leaf_of), ptr<int>(c->leaf_cell), n, Fe, e4, s));
        run_p2p(c, want_f, 0, 0, e4, false);
        CK(launch_scale(want_f, n, e4, scale, s));
    }
    if (eps_b) CK(launch_scale_eps(n, c->perm, eps_b, scale, s));
    for (int Lv = c->depth; Lv >= 0; --Lv)
        CK(launch_smin_level(t, c->ls[Lv], c->ls[Lv + 1], scale, s));
}

// ------------------------------------------------------------ the call
// nact/act: when act is not null, only the nact listed particles (input
// indices) are sinks: pot/acc receive their results in list order (Sec. 7.1)
// vel/jerk (device, input order, 3n each) when not null: the jerk as well
// (Sec. 7), with the expansion centres at rest
void forces(fmm_ctx *c, int64_t n, const double *pos, const double *mass, double G, int p,
            double eps, double *pot, double *acc, int K, const int64_t *off, bool refit,
            int64_t nact = 0, const int64_t *act = nullptr, const double *eps_b = nullptr,
            const double *vel = nullptr, double *jerk = nullptr) {
    hipStream_t s = c->stream;
    c->st = fmm_stats_t{};
    c->n = n;
    c->p = p;
    c->st.p = p;
    c->st.n = n;
    c->t_m2l_kernel = c->t_p2p_kernel = 0;
    ensure<int>(c->nonfinite, 8);
    mark(c, PH_START);
    build_tree(c, n, pos, mass, K, off, refit);
    TreeArrays t = tree_arrays(c);
    // listed sinks: cells that hold one (the tree, expansions and sink scale
    // stay those of all n particles, so a listed particle's result equals the
    // full call's)
    const uint8_t *cell_active = nullptr;
    int *inv = nullptr, *bad = nullptr;
    if (act) {
        int *flag_in = ensure<int>(c->actflag, n);
        int *f = ensure<int>(c->actf, n + 1);
        inv = ensure<int>(c->actinv, n);
        int *pre = ensure<int>(c->actpre, n + 1);
        uint8_t *ca = ensure<uint8_t>(c->cellact, c->ncells);
        bad = ensure<int>(c->actbad, 1);
        int *tmp = tmp_ints(c, scan_tmp_ints(n + 1));
        CK(hipMemsetAsync(flag_in, 0, n * sizeof(int), s));
        CK(hipMemsetAsync(bad, 0, sizeof(int), s));
        CK(launch_mark_listed(n, nact, act, flag_in, bad, s));
        CK(launch_cell_active(n, c->perm, flag_in, f, inv, pre, tmp, ptr<int>(c->nonfinite) + 1,
                              c->ncells, t.beg, t.end, ca, s));
        cell_active = ca;
    }
    mark(c, PH_TREE);
    // Upward pass on the side stream, after the tree (and, on the same stream,
    // after the enclosing-sphere centres): it overlaps the sink-scale estimate,
    // which reads only centres of mass and masses, and writes nothing the
    // estimate reads.  The main stream joins it before the walk, which needs
    // the expansion centres and the multipole powers.  Both are chains of
    // small latency-bound launches, so each fills the other's idle units.
    const int nc = ncplx(p);
    double *M = ensure<double>(c->M, 2 * (size_t)nc * c->ncells);
    double *U = ensure<double>(c->U, 2 * (size_t)nc * c->ncells);
    double *P = ensure<double>(c->P, (size_t)(p + 1) * c->ncells);
    short *plans = ensure<short>(c->plans, 2 * XP_SIZE);
    double *Tsh = ensure<double>(c->Tsh, 2 * (size_t)nc * c->ncells);
    double4 *v4 = vel ? ensure<double4>(c->vel4, n) : nullptr;
    double *Md = vel ? ensure<double>(c->Md, 2 * (size_t)nc * c->ncells) : nullptr;
    const hipStream_t us = c->side;
    CK(hipEventRecord(c->ev_fork, s));
    CK(hipStreamWaitEvent(us, c->ev_fork, 0));
    if (c->plan_p != p) {
        std::vector<short> h(2 * XP_SIZE);
        translation_plans(p, h.data(), h.data() + XP_SIZE);
        CK(hipMemcpyAsync(plans, h.data(), h.size() * sizeof(short), hipMemcpyHostToDevice, us));
        CK(hipStreamSynchronize(us));
        c->plan_p = p;
    }
    CK(launch_p2m(p, t, ptr<int>(c->leaf_cell), c->nleaves, ptr<double>(c->x), ptr<double>(c->y),
                  ptr<double>(c->z), ptr<double>(c->m), M, us));
    if (c->ncells > 1) CK(launch_shift_upsilon(p, t, 1, c->ncells, U, us));
    for (int L = c->depth; L >= 0; --L)
        CK(launch_m2m_level(p, t, c->ls[L], c->ls[L + 1], U, M, Tsh, plans, us));
    CK(launch_power(p, c->ncells, M, P, us));
    // jerk: rates of the multipoles (eq:P2M:dot, then the same M2M with the
    // centres at rest; Tsh is free again once M is complete)
    if (vel) {
        CK(launch_gather_vel(n, c->perm, vel, v4, us));
        CK(launch_p2m_dot(p, t, ptr<int>(c->leaf_cell), c->nleaves, ptr<double>(c->x),
                          ptr<double>(c->y), ptr<double>(c->z), ptr<double>(c->m), v4, Md, us));
        for (int L = c->depth; L >= 0; --L)
            CK(launch_m2m_level(p, t, c->ls[L], c->ls[L + 1], U, Md, Tsh, plans, us));
    }
    CK(hipEventRecord(c->ev_join, us));
    c->join_pending = true;
    const bool want_f = c->opts.mac == FMM_MAC_SCALED;
    if (c->opts.mac != FMM_MAC_THETA) sink_scale(c, want_f, eps_b);
    mark(c, PH_EST);
    join_side(c);   // the centres and the upward pass from the side stream
    mark(c, PH_UP);
    // walk
    WalkParams wp{c->opts.mac == FMM_MAC_THETA ? 1 : 0, p, eps, c->opts.theta_crit,
                  c->opts.p2p_factor * (p + 1.0) * (p + 1.0) * (p + 1.0), 0, 0, 0, {}};
    wp.active = cell_active;
    if (eps_b) wp.eps = 1.0;      // eps_b is in the cell minimum of the scale
    Lists L = walk(c, wp, P);
    c->st.walk_pairs = c->last_walk_pairs;
    c->st.t_sweeps = c->last_sweep_ms;
    c->st.walk_iterations = L.iterations;
    c->n_m2l = L.n_m2l;
    c->n_p2p = L.n_p2p;
    c->st.n_m2l = L.n_m2l;
    c->st.n_p2p_lists = L.n_p2p;
    c->st.n_p2p_pairs = L.pairs;
    // The direct-sum list is sorted and merged on the side stream while the
    // main stream sorts the M2L list and runs M2L: M2L holds one wavefront
    // per SIMD and no LDS, which leaves room for the sort's small waves.
    CK(hipEventRecord(c->ev_fork, s));
    c->m2l_sorted = sort_list(c, c->m2l, c->m2l2, L.n_m2l, c->ncells, c->m2l_off);
    mark(c, PH_WALK);
    // M2L: the rotation kernel over 64-entry windows of the list, or the
    // direct kernel by chunks of one sink's list
    double *F = ensure<double>(c->F, 2 * (size_t)nc * c->ncells);
    const bool rot = FMM_M2L_ROT_ENABLED && !vel &&
                     (c->opts.m2l_kernel == FMM_M2L_ROTATION ||
                      (c->opts.m2l_kernel == FMM_M2L_AUTO &&
                       c->opts.precision == FMM_PREC_FP64 && p >= FMM_M2L_ROT_AUTO_MIN &&
                       p <= FMM_M2L_ROT_MAX));
    c->st.m2l_rotation = rot ? 1 : 0;
    if (rot) {
        int *cnt = ensure<int>(c->ccnt, (size_t)c->ncells + 1);
        int *coff = ensure<int>(c->coff, (size_t)c->ncells + 1);
        int *tmp = tmp_ints(c, scan_tmp_ints(c->ncells + 1));
        int *total = ptr<int>(c->nonfinite) + 1;
        CK(launch_rot_pieces(c->ncells, ptr<int64_t>(c->m2l_off), cnt, coff, tmp, total, s));
        // pieces = (window, sink) pairs: at most one per window plus one per sink
        const int64_t pieces = (c->n_m2l + 63) / 64 + c->ncells;
        double *Fpart = ensure<double>(c->Fpart, 2 * (size_t)nc * (size_t)std::max<int64_t>(pieces, 1));
        if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[0], s));
        CK(launch_m2l_rot(p, c->n_m2l, c->m2l_sorted, c->sh, ptr<int64_t>(c->m2l_off), coff, t, M,
                          Fpart, s));
        if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[1], s));
        CK(launch_m2l_reduce(p, c->ncells, coff, Fpart, F, s));
    } else {
        const int chunk = 16;
        int *cnt = ensure<int>(c->ccnt, (size_t)c->ncells + 1);
        int *coff = ensure<int>(c->coff, (size_t)c->ncells + 1);
        int *tmp = tmp_ints(c, scan_tmp_ints(c->ncells + 1));
        int *total = ptr<int>(c->nonfinite) + 1;
        CK(launch_chunks(c->ncells, ptr<int64_t>(c->m2l_off), chunk, cnt, coff, tmp, total,
                         nullptr, false, s));
        CK(hipMemcpyAsync(c->hint, total, sizeof(int), hipMemcpyDeviceToHost, s));
        sync(c);
        const int nchunks = c->hint[0];
        int4 *chunks = ensure<int4>(c->chunks, std::max(nchunks, 1));
        CK(launch_chunks(c->ncells, ptr<int64_t>(c->m2l_off), chunk, cnt, coff, tmp, total,
                         chunks, true, s));
        if (c->opts.precision == FMM_PREC_MIXED && p <= FMM_M2L_FIXED_MAX) {
            float *M32 = ensure<float>(c->M32, 2 * (size_t)nc * c->ncells);
            float *Fpart = ensure<float>(c->Fpart, 2 * (size_t)nc * std::max(nchunks, 1));
            double *sig = ensure<double>(c->sig, std::max(nchunks, 1));
            double *Flow = ensure<double>(c->Flow, 2 * (size_t)ncplx(FMM_M2L32_JLO) *
                                                       std::max(nchunks, 1));
            CK(launch_m2l32_multipoles(p, c->ncells, t, M, M32, s));
            if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[0], s));
            CK(launch_m2l32(p, nchunks, chunks, c->m2l_sorted, c->sh, t, M, M32, Fpart, Flow, sig,
                            s));
            if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[1], s));
            CK(launch_m2l32_reduce(p, c->ncells, coff, Fpart, Flow, sig, F, s));
        } else {
            double *Fpart = ensure<double>(c->Fpart, 2 * (size_t)nc * std::max(nchunks, 1));
            if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[0], s));
            CK(launch_m2l(p, nchunks, chunks, c->m2l_sorted, c->sh, t, M, Fpart, s));
            if (c->opts.timing) CK(hipEventRecord(c->ev_m2l[1], s));
            CK(launch_m2l_reduce(p, c->ncells, coff, Fpart, F, s));
        }
        if (vel) {   // eq:M2L:dot: the same pairs applied to the rates, FP64
            double *Fd = ensure<double>(c->Fd, 2 * (size_t)nc * c->ncells);
            double *Fp = ensure<double>(c->jFpart, 2 * (size_t)nc * std::max(nchunks, 1));
            CK(launch_m2l(p, nchunks, chunks, c->m2l_sorted, c->sh, t, Md, Fp, s));
            CK(launch_m2l_reduce(p, c->ncells, coff, Fp, Fd, s));
        }
    }
    // the direct-sum lists, on the side stream (overlapping M2L, queued above)
    CK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    prepare_p2p(c, L.n_p2p, true, true);
    const P2PPlan near = plan_p2p(c, cell_active, true);
    CK(hipEventRecord(c->ev_join, c->side));
    c->join_pending = true;
    mark(c, PH_M2L);
    // downward pass, far field at the particles
    for (int Lv = 1; Lv <= c->depth; ++Lv) {
        CK(launch_l2l_level(p, t, c->ls[Lv], c->ls[Lv + 1], U, F,
                            ptr<short>(c->plans) + XP_SIZE, s, cell_active));
        if (vel)
            CK(launch_l2l_level(p, t, c->ls[Lv], c->ls[Lv + 1], U, ptr<double>(c->Fd),
                                ptr<short>(c->plans) + XP_SIZE, s, cell_active));
    }
    double4 *o4 = ensure<double4>(c->out4, n);
    CK(launch_l2p(p, t, ptr<int>(c->leaf_of), ptr<int>(c->leaf_cell), n, ptr<double>(c->x),
                  ptr<double>(c->y), ptr<double>(c->z), F, o4, s, cell_active));
    double4 *jo4 = nullptr;
    if (vel) {   // eq:L2P:dot, assigns the far-field jerk of every particle
        jo4 = ensure<double4>(c->jo4, n);
        CK(launch_l2p_dot(p, t, ptr<int>(c->leaf_of), ptr<int>(c->leaf_cell), n,
                          ptr<double>(c->x), ptr<double>(c->y), ptr<double>(c->z), v4, F,
                          ptr<double>(c->Fd), jo4, s, cell_active));
    }
    mark(c, PH_DOWN);
    join_side(c);   // the direct-sum lists and tasks from the side stream
    // near field (with the jerk: FP64, potential and acceleration as the force-only
    // FP64 kernel sums them)
    exec_p2p(c, near, 0, 1, c->opts.precision == FMM_PREC_MIXED && !vel, o4, true, v4, jo4);
    mark(c, PH_P2P);
    int *nonfinite = ptr<int>(c->nonfinite);
    CK(hipMemsetAsync(nonfinite, 0, sizeof(int), s));
    if (act)
        CK(launch_output_listed(n, nact, act, inv, o4, G, pot, acc, nonfinite, s));
    else
        CK(launch_output(n, c->perm, o4, G, pot, acc, nonfinite, s));
    if (vel && act)
        CK(launch_output_jerk_listed(n, nact, act, inv, jo4, G, jerk, nonfinite, s));
    else if (vel)
        CK(launch_output_jerk(n, c->perm, jo4, G, jerk, nonfinite, s));
    if (c->opts.scale_source == FMM_SCALE_PREVIOUS && !act) {
        CK(launch_norm3(acc, n, G, ensure<double>(c->prev_scale, n), s));
        c->have_prev_scale = true;
        c->prev_n = n;
    }
    mark(c, PH_END);
    CK(hipMemcpyAsync(c->hint, nonfinite, sizeof(int), hipMemcpyDeviceToHost, s));
    if (act) CK(hipMemcpyAsync(c->hint + 1, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    else c->hint[1] = 0;
    sync(c);
    c->st.n_cells = c->ncells;
    c->st.refitted = c->refitted ? 1 : 0;
    c->st.n_leaves = c->nleaves;
    c->st.depth = c->depth;
    if (c->opts.timing) {
        auto el = [&](int a, int b) {
            float ms = 0;
            CK(hipEventElapsedTime(&ms, c->ev[a], c->ev[b]));
            return (double)ms;
        };
        c->st.t_tree = el(PH_START, PH_TREE);
        c->st.t_estimate = el(PH_TREE, PH_EST);
        c->st.t_up = el(PH_EST, PH_UP);
        c->st.t_walk = el(PH_UP, PH_WALK);
        c->st.t_m2l = el(PH_WALK, PH_M2L);
        c->st.t_down = el(PH_M2L, PH_DOWN);
        c->st.t_p2p = el(PH_DOWN, PH_P2P);
        c->st.t_total = el(PH_START, PH_END);
        float ms = 0;
        CK(hipEventElapsedTime(&ms, c->ev_m2l[0], c->ev_m2l[1]));
        c->st.t_m2l_kernel = ms;
        c->st.m2l_launches = 1;
        CK(hipEventElapsedTime(&ms, c->ev_p2p[0], c->ev_p2p[1]));
        c->st.t_p2p_kernel = ms;
        c->st.p2p_launches = 1;
    }
}

// The paper's optimum grows by ~1.6 orders per decade of eps and is p = 10 at
// eps = 10^-6.25 for its CPU (Sec. 6.2); on this GPU M2L is cheap next to the
// direct sums, so the balance sits two orders higher (measured on Plummer and
// Dehnen gamma = 1 samples of 10^6 particles).
int order_for_error(double e) {
    int p = (int)std::lround(1.6 * std::log10(1.0 / e)) + 2;
    return std::min(FMM_P_MAX, std::max(3, p));
}

struct Guard {
    fmm_ctx *c;
    bool ok;
    explicit Guard(fmm_ctx *c_) : c(c_) {
        int z = 0;
        ok = c->busy.compare_exchange_strong(z, 1);
    }
    ~Guard() {
        if (ok) c->busy.store(0);
    }
};

fmm_status fail(fmm_ctx *c, fmm_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

template <class F>
fmm_status guarded(fmm_ctx *c, F &&body) {
    try {
        CK(hipSetDevice(c->opts.device));
        return body();
    } catch (const HipFail &h) {
        return fail(c, FMM_E_HIP, std::string(h.what) + ": " + hipGetErrorString(h.e));
    } catch (const NoMem &m) {
        char b[128];
        std::snprintf(b, sizeof b, "device allocation of %zu bytes failed", m.bytes);
        return fail(c, FMM_E_NOMEM, b);
    } catch (...) {
        return fail(c, FMM_E_HIP, "unexpected internal error");
    }
}


}  // namespace

// ---- workspace of the entry point that allocates nothing --------------------
// fmm_direct_sinks_noalloc keeps its index flag (first 256 bytes) and its
// partial rows (the rest) in this array instead of context buffers.  Each
// device holds its own copy for the life of the process.  In host code the
// name only stands for the symbol: its device address comes from
// hipGetSymbolAddress, taken once per device (with that device current) by
// the first fmm_build on it and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// the address of the current device's copy (the caller made `dev` current)
void *scratch_address(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) throw HipFail{hipErrorInvalidDevice, "device ordinal"};
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *q = nullptr;
        CK(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        scratch_ptr[dev] = q;
    }
    return scratch_ptr[dev];
}

}  // namespace fmm

// =====================================================================  C ABI

extern "C" {

int fmm_order_for_error(double target_err) {
    if (!(target_err > 0.0) || !std::isfinite(target_err)) return -1;
    return fmm::order_for_error(target_err);
}

fmm_status fmm_build(fmm_ctx **out, const fmm_opts *o) {
    if (!out || !o) return FMM_E_INVAL;
    *out = nullptr;
    if (o->leaf_size < 0 || o->leaf_size > 4096) return FMM_E_INVAL;
    if (o->mac < FMM_MAC_REL || o->mac > FMM_MAC_THETA) return FMM_E_INVAL;
    if (o->mac == FMM_MAC_THETA && !(o->theta_crit > 0.0 && o->theta_crit < 1.0)) return FMM_E_INVAL;
    if (o->p2p_factor < 0.0 || !std::isfinite(o->p2p_factor)) return FMM_E_INVAL;
    if (o->precision != FMM_PREC_FP64 && o->precision != FMM_PREC_MIXED) return FMM_E_INVAL;
    if (o->m2l_kernel < FMM_M2L_AUTO || o->m2l_kernel > FMM_M2L_ROTATION) return FMM_E_INVAL;
    if (o->scale_source != FMM_SCALE_ESTIMATE && o->scale_source != FMM_SCALE_PREVIOUS)
        return FMM_E_INVAL;
    if (o->centre < FMM_CENTRE_AUTO || o->centre > FMM_CENTRE_ENCLOSING) return FMM_E_INVAL;
    if (o->n_max < 0 || o->p_max < 0 || o->p_max > FMM_P_MAX) return FMM_E_INVAL;
    if (o->hbm_budget_bytes && o->n_max > 0 && o->p_max > 0 &&
        fmm_footprint_bytes(o->n_max, o->p_max, o) > o->hbm_budget_bytes)
        return FMM_E_NOMEM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) {
        (void)hipGetLastError();
        return FMM_E_INVAL;
    }
    fmm_ctx *c = new (std::nothrow) fmm_ctx;
    if (!c) return FMM_E_NOMEM;
    c->opts = *o;
    if (c->opts.leaf_size == 0) c->opts.leaf_size = 32;
    if (c->opts.p2p_factor == 0.0) c->opts.p2p_factor = 2.0;
    fmm_status st = fmm::guarded(c, [&]() -> fmm_status {
        if (o->hip_stream) {
            c->stream = (hipStream_t)o->hip_stream;
        } else {
            CK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        CK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        CK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        CK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
        CK(hipHostMalloc((void **)&c->hcnt, HCNT * sizeof(unsigned long long), hipHostMallocDefault));
        CK(hipHostMalloc((void **)&c->hint, 16 * sizeof(int), hipHostMallocDefault));
        for (auto &e : c->ev) CK(hipEventCreate(&e));
        for (auto &e : c->ev_m2l) CK(hipEventCreate(&e));
        for (auto &e : c->ev_p2p) CK(hipEventCreate(&e));
        for (auto &e : c->ev_walk) CK(hipEventCreate(&e));
        c->scratch = fmm::scratch_address(c->opts.device);
        return FMM_OK;
    });
    if (st != FMM_OK) {
        fmm_destroy(c);
        return st;
    }
    *out = c;
    return FMM_OK;
}

void fmm_destroy(fmm_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->opts.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    DevBuf *bufs[] = {&c->bbox, &c->key, &c->key2, &c->idx, &c->idx2, &c->x, &c->y, &c->z, &c->m,
                      &c->xyzm, &c->leaf_of, &c->out4, &c->est4, &c->scale, &c->flags, &c->tmp,
                      &c->beg, &c->end, &c->parent, &c->child0, &c->nchild, &c->level,
                      &c->leaf_lo, &c->leaf_hi, &c->cen, &c->com, &c->mass, &c->lo, &c->hi,
                      &c->rho2, &c->bsph, &c->smin, &c->leaf_cell, &c->M, &c->F, &c->P, &c->U, &c->Fe,
                      &c->fa, &c->fb, &c->m2l, &c->m2l2, &c->p2p, &c->p2p2, &c->p2pe,
                      &c->p2pe2, &c->rflag, &c->ranges, &c->rkey, &c->pt_n, &c->pt_m,
                      &c->pt_s, &c->pt_off, &c->pt_moff, &c->ptasks, &c->pchain, &c->ppart, &c->m2l_off,
                      &c->p2p_off, &c->chunks, &c->ccnt, &c->coff, &c->Fpart, &c->counters,
                      &c->nonfinite, &c->prev_scale, &c->walktmp, &c->coffsets,
                      &c->ckey, &c->ckey2, &c->order, &c->order2, &c->wcode, &c->rup, &c->tmp_side,
                      &c->actflag, &c->actf, &c->actinv, &c->actpre, &c->cellact, &c->actbad,
                      &c->dkey, &c->dsort, &c->dsort2, &c->runstart, &c->plans, &c->Tsh,
                      &c->M32, &c->sig, &c->Flow, &c->epsmin, &c->vel4, &c->Md, &c->Fd,
                      &c->jFpart, &c->jo4, &c->jpart, &c->dspart, &c->tg, &c->tpre, &c->tsuf,
                      &c->tcell, &c->tcell2, &c->tls};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev_m2l) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev_p2p) if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev_walk) if (e) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->hcnt) (void)hipHostFree(c->hcnt);
    if (c->hint) (void)hipHostFree(c->hint);
    if (c->pin) (void)hipHostFree(c->pin);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// jerk: the call also evaluates the rates (always with the FP64 M2L kernels)
static fmm_status check_common(fmm_ctx *c, int64_t n, const double *pos, const double *mass,
                               double G, int *p, double eps, double *pot, double *acc,
                               bool jerk = false) {
    if (n < 0) return fmm::fail(c, FMM_E_INVAL, "n < 0");
    if (n > (int64_t)INT32_MAX / 2) return fmm::fail(c, FMM_E_INVAL, "n too large");
    if (n > 0 && (!pos || !mass || !pot || !acc)) return fmm::fail(c, FMM_E_INVAL, "null array");
    if (!std::isfinite(G)) return fmm::fail(c, FMM_E_INVAL, "G not finite");
    if (c->opts.mac != FMM_MAC_THETA && !(eps > 0.0 && std::isfinite(eps)))
        return fmm::fail(c, FMM_E_INVAL, "target_err must be > 0 and finite");
    if (*p < 0) {
        if (!(eps > 0.0 && std::isfinite(eps)))
            return fmm::fail(c, FMM_E_INVAL, "p < 0 needs a target_err > 0");
        *p = fmm::order_for_error(eps);
    }
    if (*p == 0) return fmm::fail(c, FMM_E_INVAL, "p must be >= 1");
    if (*p > FMM_P_MAX) return fmm::fail(c, FMM_E_UNSUPPORTED, "p above FMM_P_MAX");
    if (c->opts.n_max > 0 && n > c->opts.n_max)
        return fmm::fail(c, FMM_E_INVAL, "n above the context's n_max");
    if (c->opts.p_max > 0 && *p > c->opts.p_max)
        return fmm::fail(c, FMM_E_INVAL, "p above the context's p_max");
    if (c->opts.hbm_budget_bytes && fmm_footprint_bytes(n, *p, &c->opts) > c->opts.hbm_budget_bytes)
        return fmm::fail(c, FMM_E_NOMEM, "footprint above the context's hbm_budget_bytes");
    // the lowest orders whose kernels have a passing device run: FP64 from 3,
    // the mixed-precision M2L from 2
    const int pmin = c->opts.precision == FMM_PREC_MIXED && !jerk ? FMM_P_MIN_MIXED : FMM_P_MIN;
    if (*p < pmin)
        return fmm::fail(c, FMM_E_UNSUPPORTED, c->opts.precision == FMM_PREC_MIXED && !jerk
                                                   ? "mixed precision needs p >= 2"
                                                   : "FP64 evaluation needs p >= 3");
    if (c->opts.m2l_kernel == FMM_M2L_ROTATION && !FMM_M2L_ROT_ENABLED)
        return fmm::fail(c, FMM_E_UNSUPPORTED, "the rotation M2L kernel is switched off");
    if (c->opts.m2l_kernel == FMM_M2L_ROTATION && *p > FMM_M2L_ROT_MAX)
        return fmm::fail(c, FMM_E_UNSUPPORTED, "the rotation M2L kernel supports p <= 16");
    return FMM_OK;
}

fmm_status fmm_forces(fmm_ctx *c, int64_t n, const double *pos, const double *mass, double G,
                      int p, double target_err, double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot, acc);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n == 0) return FMM_OK;
        if (n == 1) {
            CK(hipMemsetAsync(pot, 0, sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * sizeof(double), c->stream));
            fmm::sync(c);
            c->st = fmm_stats_t{};
            c->st.n = 1;
            c->st.p = p;
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, 1, off, false);
        if (c->hint[0]) return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential or acceleration");
        return FMM_OK;
    });
}

fmm_status fmm_forces_batched(fmm_ctx *c, int64_t k, const int64_t *off, const double *pos,
                              const double *mass, double G, int p, double target_err, double *pot,
                              double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (k < 0 || (k > 0 && !off)) return fmm::fail(c, FMM_E_INVAL, "bad cluster offsets");
    if (k == 0) return FMM_OK;
    if (k > (1 << 24)) return fmm::fail(c, FMM_E_INVAL, "too many clusters");
    if (off[0] != 0) return fmm::fail(c, FMM_E_INVAL, "offsets[0] must be 0");
    for (int64_t i = 0; i < k; ++i)
        if (off[i + 1] < off[i]) return fmm::fail(c, FMM_E_INVAL, "offsets must not decrease");
    const int64_t n = off[k];
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot, acc);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n == 0) return FMM_OK;
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, (int)k, off, false);
        if (c->hint[0]) return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential or acceleration");
        return FMM_OK;
    });
}

fmm_status fmm_forces_refit(fmm_ctx *c, int64_t n, const double *pos, const double *mass,
                            double G, int p, double target_err, double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot, acc);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n == 0) return FMM_OK;
        if (n == 1) {
            CK(hipMemsetAsync(pot, 0, sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * sizeof(double), c->stream));
            fmm::sync(c);
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, 1, off, true);
        if (c->hint[0]) return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential or acceleration");
        return FMM_OK;
    });
}

fmm_status fmm_forces_active(fmm_ctx *c, int64_t n, const double *pos, const double *mass,
                             double G, int p, double target_err, int64_t n_active,
                             const int64_t *active, int refit, double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n_active < 0 || (n_active > 0 && (!active || !pot || !acc)))
        return fmm::fail(c, FMM_E_INVAL, "bad list of active particles or outputs");
    if (n < 0 || (n > 0 && (!pos || !mass)))
        return fmm::fail(c, FMM_E_INVAL, "bad particle arrays");
    // outputs are checked above; check_common only needs non-null pointers
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot ? pot : (double *)pos,
                                 acc ? acc : (double *)pos);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n_active == 0) return FMM_OK;
        if (n == 0) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
        if (n == 1) {   // one particle: no force; the list may only name it
            int *bad = fmm::ensure<int>(c->actbad, 1);
            int *flag = fmm::ensure<int>(c->actflag, 1);
            CK(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
            CK(fmm::launch_mark_listed(1, n_active, active, flag, bad, c->stream));
            CK(hipMemsetAsync(pot, 0, n_active * sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * n_active * sizeof(double), c->stream));
            CK(hipMemcpyAsync(c->hint + 1, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            fmm::sync(c);
            if (c->hint[1]) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, 1, off, refit != 0, n_active,
                    active);
        if (c->hint[1]) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
        if (c->hint[0]) return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential or acceleration");
        return FMM_OK;
    });
}

fmm_status fmm_forces_eps(fmm_ctx *c, int64_t n, const double *pos, const double *mass,
                          double G, int p, const double *eps_particle, double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n > 0 && !eps_particle) return fmm::fail(c, FMM_E_INVAL, "eps_particle is null");
    if (c->opts.mac == FMM_MAC_THETA)
        return fmm::fail(c, FMM_E_INVAL, "individual eps need criterion a or f");
    if (n < 0 || (n > 0 && (!pos || !mass || !pot || !acc)))
        return fmm::fail(c, FMM_E_INVAL, "bad argument");
    if (n == 0) return FMM_OK;
    return fmm::guarded(c, [&]() -> fmm_status {
        // every eps_b > 0 and finite; the smallest sets the order when p < 0
        unsigned long long *mb = fmm::ensure<unsigned long long>(c->epsmin, 1);
        int *bad = fmm::ensure<int>(c->actbad, 1);
        CK(hipMemsetAsync(mb, 0xff, sizeof(unsigned long long), c->stream));
        CK(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
        CK(fmm::launch_eps_min(n, eps_particle, mb, bad, c->stream));
        unsigned long long *h = reinterpret_cast<unsigned long long *>(c->hint + 2);
        CK(hipMemcpyAsync(h, mb, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
        CK(hipMemcpyAsync(c->hint + 1, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        fmm::sync(c);
        if (c->hint[1]) return fmm::fail(c, FMM_E_INVAL, "every eps_b must be > 0 and finite");
        double emin;
        std::memcpy(&emin, h, sizeof(double));
        int pp = p;
        fmm_status st = check_common(c, n, pos, mass, G, &pp, emin, pot, acc);
        if (st != FMM_OK) return st;
        if (n == 1) {
            CK(hipMemsetAsync(pot, 0, sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * sizeof(double), c->stream));
            fmm::sync(c);
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, pp, emin, pot, acc, 1, off, false, 0, nullptr,
                    eps_particle);
        if (c->hint[0]) return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential or acceleration");
        return FMM_OK;
    });
}

fmm_status fmm_forces_jerk(fmm_ctx *c, int64_t n, const double *pos, const double *vel,
                           const double *mass, double G, int p, double target_err, double *pot,
                           double *acc, double *jerk) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n > 0 && (!vel || !jerk)) return fmm::fail(c, FMM_E_INVAL, "null velocity or jerk array");
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot, acc, true);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n == 0) return FMM_OK;
        if (n == 1) {
            CK(hipMemsetAsync(pot, 0, sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * sizeof(double), c->stream));
            CK(hipMemsetAsync(jerk, 0, 3 * sizeof(double), c->stream));
            fmm::sync(c);
            c->st = fmm_stats_t{};
            c->st.n = 1;
            c->st.p = p;
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, 1, off, false, 0, nullptr,
                    nullptr, vel, jerk);
        if (c->hint[0])
            return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential, acceleration or jerk");
        return FMM_OK;
    });
}

fmm_status fmm_direct(fmm_ctx *c, int64_t n, const double *pos, const double *mass, double G,
                      double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n < 0 || (n > 0 && (!pos || !mass || !pot || !acc)) || !std::isfinite(G))
        return fmm::fail(c, FMM_E_INVAL, "bad argument");
    if (n == 0) return FMM_OK;
    return fmm::guarded(c, [&]() -> fmm_status {
        CK(fmm::launch_direct(n, pos, mass, G, pot, acc, c->stream));
        fmm::sync(c);
        return FMM_OK;
    });
}

static fmm_status check_direct_sinks(fmm_ctx *c, int64_t n, const double *pos,
                                     const double *mass, double G, int64_t nsinks,
                                     const int64_t *sinks, double *pot, double *acc) {
    if (n < 0 || nsinks < 0 || (nsinks > 0 && (!pos || !mass || !sinks || !pot || !acc)) ||
        !std::isfinite(G))
        return fmm::fail(c, FMM_E_INVAL, "bad argument");
    if (n > (int64_t)INT32_MAX / 2 || nsinks > (int64_t)INT32_MAX / 2)
        return fmm::fail(c, FMM_E_INVAL, "n or nsinks too large");
    if (nsinks > 0 && n == 0) return fmm::fail(c, FMM_E_INVAL, "sink index out of range");
    return FMM_OK;
}

fmm_status fmm_direct_sinks(fmm_ctx *c, int64_t n, const double *pos, const double *mass,
                            double G, int64_t nsinks, const int64_t *sinks, double *pot,
                            double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    fmm_status st = check_direct_sinks(c, n, pos, mass, G, nsinks, sinks, pot, acc);
    if (st != FMM_OK || nsinks == 0) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        const int nchunk = fmm::direct_sinks_chunks(n, nsinks);
        double4 *part =
            nchunk > 1 ? fmm::ensure<double4>(c->dspart, (size_t)nchunk * nsinks) : nullptr;
        int *bad = fmm::ensure<int>(c->nonfinite, 8) + 5;
        CK(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
        CK(fmm::launch_direct_sinks(n, pos, mass, G, nsinks, sinks, nchunk, pot, acc, part, bad,
                                    c->stream));
        CK(hipMemcpyAsync(c->hint, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        fmm::sync(c);
        if (c->hint[0]) return fmm::fail(c, FMM_E_INVAL, "sink index out of range");
        return FMM_OK;
    });
}

fmm_status fmm_direct_sinks_noalloc(fmm_ctx *c, int64_t n, const double *pos,
                                    const double *mass, double G, int64_t nsinks,
                                    const int64_t *sinks, double *pot, double *acc) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    fmm_status st = check_direct_sinks(c, n, pos, mass, G, nsinks, sinks, pot, acc);
    if (st != FMM_OK || nsinks == 0) return st;
    const int nchunk = fmm::direct_sinks_chunks(n, nsinks);
    const size_t rows = nchunk > 1 ? (size_t)nchunk * (size_t)nsinks * sizeof(double4) : 0;
    if (256 + rows > FMM_NOALLOC_SCRATCH_BYTES)
        return fmm::fail(c, FMM_E_INVAL, "the partial sums exceed the static scratch buffer");
    if (!c->scratch) return fmm::fail(c, FMM_E_HIP, "no scratch address on this device");
    return fmm::guarded(c, [&]() -> fmm_status {
        int *bad = static_cast<int *>(c->scratch);
        double4 *part =
            nchunk > 1 ? reinterpret_cast<double4 *>(static_cast<char *>(c->scratch) + 256)
                       : nullptr;
        CK(fmm::launch_fill_int(bad, 1, 0, c->stream));
        CK(fmm::launch_direct_sinks(n, pos, mass, G, nsinks, sinks, nchunk, pot, acc, part, bad,
                                    c->stream));
        CK(hipMemcpyAsync(c->hint, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        fmm::sync(c);
        if (c->hint[0]) return fmm::fail(c, FMM_E_INVAL, "sink index out of range");
        return FMM_OK;
    });
}

fmm_status fmm_forces_jerk_active(fmm_ctx *c, int64_t n, const double *pos, const double *vel,
                                  const double *mass, double G, int p, double target_err,
                                  int64_t n_active, const int64_t *active, int refit, double *pot,
                                  double *acc, double *jerk) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n_active < 0 || (n_active > 0 && (!active || !pot || !acc || !jerk)))
        return fmm::fail(c, FMM_E_INVAL, "bad list of active particles or outputs");
    if (n < 0 || (n > 0 && (!pos || !mass || !vel)))
        return fmm::fail(c, FMM_E_INVAL, "bad particle arrays");
    fmm_status st = check_common(c, n, pos, mass, G, &p, target_err, pot ? pot : (double *)pos,
                                 acc ? acc : (double *)pos, true);
    if (st != FMM_OK) return st;
    return fmm::guarded(c, [&]() -> fmm_status {
        if (n_active == 0) return FMM_OK;
        if (n == 0) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
        if (n == 1) {   // one particle: no force, no jerk; the list may only name it
            int *bad = fmm::ensure<int>(c->actbad, 1);
            int *flag = fmm::ensure<int>(c->actflag, 1);
            CK(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
            CK(fmm::launch_mark_listed(1, n_active, active, flag, bad, c->stream));
            CK(hipMemsetAsync(pot, 0, n_active * sizeof(double), c->stream));
            CK(hipMemsetAsync(acc, 0, 3 * n_active * sizeof(double), c->stream));
            CK(hipMemsetAsync(jerk, 0, 3 * n_active * sizeof(double), c->stream));
            CK(hipMemcpyAsync(c->hint + 1, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            fmm::sync(c);
            if (c->hint[1]) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
            return FMM_OK;
        }
        const int64_t off[2] = {0, n};
        fmm::forces(c, n, pos, mass, G, p, target_err, pot, acc, 1, off, refit != 0, n_active,
                    active, nullptr, vel, jerk);
        if (c->hint[1]) return fmm::fail(c, FMM_E_INVAL, "active index out of range");
        if (c->hint[0])
            return fmm::fail(c, FMM_E_NONFINITE, "non-finite potential, acceleration or jerk");
        return FMM_OK;
    });
}

fmm_status fmm_direct_jerk_sinks(fmm_ctx *c, int64_t n, const double *pos, const double *vel,
                                 const double *mass, double G, int64_t nsinks,
                                 const int64_t *sinks, double *jerk) {
    if (!c) return FMM_E_INVAL;
    fmm::Guard g(c);
    if (!g.ok) return FMM_E_BUSY;
    c->err.clear();
    if (n < 0 || nsinks < 0 ||
        (nsinks > 0 && (!pos || !vel || !mass || !sinks || !jerk)) || !std::isfinite(G))
        return fmm::fail(c, FMM_E_INVAL, "bad argument");
    if (nsinks == 0) return FMM_OK;
    if (n == 0) return fmm::fail(c, FMM_E_INVAL, "sink index out of range");
    return fmm::guarded(c, [&]() -> fmm_status {
        int *bad = fmm::ensure<int>(c->nonfinite, 8) + 5;
        CK(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
        CK(fmm::launch_direct_jerk_sinks(n, pos, vel, mass, G, nsinks, sinks, jerk, bad,
                                         c->stream));
        CK(hipMemcpyAsync(c->hint, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        fmm::sync(c);
        if (c->hint[0]) return fmm::fail(c, FMM_E_INVAL, "sink index out of range");
        return FMM_OK;
    });
}

fmm_status fmm_stats(const fmm_ctx *c, fmm_stats_t *out) {
    if (!c || !out) return FMM_E_INVAL;
    *out = c->st;
    return FMM_OK;
}

size_t fmm_footprint_bytes(int64_t n, int p, const fmm_opts *o) {
    if (n <= 0) return 0;
    if (p < 1) p = 12;
    const int leaf = (o && o->leaf_size > 0) ? o->leaf_size : 32;
    const double cells = 1.5 * (double)n / (0.3 * leaf) + 64;
    const double nc = 16.0 * (p + 1) * (p + 2) / 2.0;
    const double per_particle = 8 * 2 + 4 * 2 + 8 * 4 + 32 + 4 + 32 * 2 + 8 * 2 + 4 + 16 + 8 * 4;
    const double per_cell = 4 * nc + 8 * (p + 1) + 4 * 10 + 32 * 2 + 8 * 9 + 16 + 16;
    const double lists = 8.0 * 2 * (150.0 * cells) + 8.0 * 2 * (200.0 * cells) + 8.0 * 2 * n;
    const double part = nc * (150.0 * cells / 16 + cells);
    return (size_t)(per_particle * n + per_cell * cells + lists + part);
}

const char *fmm_last_error(const fmm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int64_t fmm_export(fmm_ctx *c, int what, void *dst, int64_t capacity) {
    if (!c) return -1;
    try {
        CK(hipSetDevice(c->opts.device));
        const int nc = c->ncells;
        std::vector<int> beg(nc), lev(nc), end(nc), lcell(c->nleaves);
        auto cells = [&]() {
            CK(hipMemcpy(beg.data(), c->beg.p, nc * sizeof(int), hipMemcpyDeviceToHost));
            CK(hipMemcpy(end.data(), c->end.p, nc * sizeof(int), hipMemcpyDeviceToHost));
            CK(hipMemcpy(lev.data(), c->level.p, nc * sizeof(int), hipMemcpyDeviceToHost));
            if (c->nleaves)
                CK(hipMemcpy(lcell.data(), c->leaf_cell.p, c->nleaves * sizeof(int),
                             hipMemcpyDeviceToHost));
        };
        auto id = [&](int cell) { return ((int64_t)lev[cell] << 40) | (int64_t)beg[cell]; };
        if (what == FMM_EXPORT_M2L) {
            const int64_t cnt = c->n_m2l;
            const int64_t bytes = cnt * 16;
            if (!dst || capacity < bytes) return bytes;
            cells();
            std::vector<uint64_t> keys(cnt);
            if (cnt) CK(hipMemcpy(keys.data(), c->m2l_sorted, cnt * 8, hipMemcpyDeviceToHost));
            int64_t *o = static_cast<int64_t *>(dst);
            const uint64_t mask = (1ull << c->sh) - 1;
            for (int64_t i = 0; i < cnt; ++i) {
                o[2 * i] = id((int)(keys[i] & mask));
                o[2 * i + 1] = id((int)(keys[i] >> c->sh));
            }
            return bytes;
        }
        if (what == FMM_EXPORT_P2P) {
            const int64_t cnt = c->n_p2p;
            const int64_t bytes = cnt * 24;
            if (!dst || capacity < bytes) return bytes;
            cells();
            std::vector<uint64_t> keys(cnt);
            std::vector<uint32_t> ends(cnt);
            if (cnt) {
                CK(hipMemcpy(keys.data(), c->p2p_sorted, cnt * 8, hipMemcpyDeviceToHost));
                if (!c->pack)
                    CK(hipMemcpy(ends.data(), c->p2pe_sorted, cnt * 4, hipMemcpyDeviceToHost));
            }
            int64_t *o = static_cast<int64_t *>(dst);
            const uint64_t mask = (1ull << c->pb) - 1;
            for (int64_t i = 0; i < cnt; ++i) {
                const uint64_t k = keys[i];
                if (c->pack) {
                    o[3 * i] = id((int)(k >> (2 * c->pb)));
                    o[3 * i + 1] = (int64_t)((k >> c->pb) & mask);
                    o[3 * i + 2] = (int64_t)(k & mask);
                } else {
                    o[3 * i] = id((int)(k >> c->pb));
                    o[3 * i + 1] = (int64_t)(k & mask);
                    o[3 * i + 2] = (int64_t)ends[i];
                }
            }
            return bytes;
        }
        if (what == FMM_EXPORT_SCALE) {
            const int64_t bytes = c->n * 8;
            if (!dst || capacity < bytes) return bytes;
            std::vector<double> s(c->n);
            std::vector<uint32_t> perm(c->n);
            CK(hipMemcpy(s.data(), c->scale.p, c->n * 8, hipMemcpyDeviceToHost));
            CK(hipMemcpy(perm.data(), c->perm, c->n * 4, hipMemcpyDeviceToHost));
            double *o = static_cast<double *>(dst);
            for (int64_t i = 0; i < c->n; ++i) o[perm[i]] = s[i];
            return bytes;
        }
        if (what == FMM_EXPORT_CELLS) {
            const int64_t bytes = (int64_t)nc * 16;
            if (!dst || capacity < bytes) return bytes;
            cells();
            int64_t *o = static_cast<int64_t *>(dst);
            for (int i = 0; i < nc; ++i) {
                o[2 * i] = id(i);
                o[2 * i + 1] = end[i];
            }
            return bytes;
        }
        if (what == FMM_EXPORT_CENTRES) {
            const int64_t bytes = (int64_t)nc * 32;
            if (!dst || capacity < bytes) return bytes;
            if (nc) CK(hipMemcpy(dst, c->cen.p, bytes, hipMemcpyDeviceToHost));
            return bytes;
        }
        return -1;
    } catch (...) {
        return -1;
    }
}

}  // extern "C"
