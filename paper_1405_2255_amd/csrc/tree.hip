// Tree stage: bounding box, Morton keys, gather into sorted SoA, octree
// levels, leaves, cell geometry (bounding box, mass, centre of mass,
// expansion centre and radii) and the per-cell minimum sink scale.
//
// A batch of K independent clusters (particles of cluster k back to back) is
// one forest: each cluster gets its own cube and keys, the sort groups
// clusters and orders keys inside each, and every non-empty cluster has a
// root at level 0.  All later kernels serve all clusters in the same launch.
//
// The octree (Sec. 2.2.1): cubic cells, a cell holding more than n_L
// particles is split into its non-empty octants, up to depth 21.  Octants
// come from 21-bit quantised coordinates in the cube around the bounding box
// (bit i of the x, y, z cell index at key bit 3i, 3i+1, 3i+2), so every cell
// is a contiguous range of the key-sorted particles.  Cells are numbered
// level by level, and inside a level in key order.
//
// Expansion centre z = s of a cell: the midpoint of its particles' bounding
// box, or with the enclosing-sphere rule an approximate centre of the
// smallest enclosing sphere (Sec. 5.1.1) where that gives the smaller radius;
// rho = the largest distance of its particles from it (the definitions of
// rho_z and rho_s in Sec. 4).  rho_com likewise about the centre of mass (the
// centre of the low-order estimate, Sec. 5.4.2).
#include <climits>

#include "internal.h"
#include "dev.h"

namespace fmm {

namespace {

// cluster of particle i: offsets off[0..K] (off[0] = 0), clusters back to back
__device__ __forceinline__ int cluster_of(const int64_t *off, int K, int64_t i) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// bounding box of every cluster: bb[6k..6k+5] = min x, y, z, max x, y, z as
// order-preserving keys.  Each lane keeps the box of the wavefront's current
// cluster over the chunks of its grid-stride loop; the wavefront reduces the
// lanes' boxes and commits them (6 atomics) only when its cluster changes and
// at the end.  A chunk that spans clusters commits per lane.
__device__ __forceinline__ void commit_box(unsigned long long *bb, int c, const double *lo,
                                           const double *hi) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        atomicMin(&bb[6 * c + d], ordered_key(lo[d]));
        atomicMax(&bb[6 * c + 3 + d], ordered_key(hi[d]));
    }
}

__device__ __forceinline__ void commit_run(unsigned long long *bb, int run, double *lo,
                                           double *hi) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int o = FMM_WAVE / 2; o > 0; o >>= 1) {
            lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, FMM_WAVE));
            hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, FMM_WAVE));
        }
    }
    if (lane_id() == 0) commit_box(bb, run, lo, hi);
}

// part (one cluster only): each wavefront writes its box to its own six
// slots instead of committing atomics (a thousand wavefronts' atomics on the
// same six addresses serialize), and k_bbox_parts reduces the slots.
__global__ void k_bbox(const double *pos, int64_t n, int K, const int64_t *off,
                       unsigned long long *bb, unsigned long long *part) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int run = -1;   // the wavefront's current cluster
    double rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(FMM_WAVE - 1));
         base < n; base += stride) {
        const int64_t i = base + lane;
        const bool valid = i < n;
        const int cl = valid ? cluster_of(off, K, i) : -1;
        double v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = valid ? pos[3 * i + d] : 0.0;
        const int c0 = __shfl(cl, 0, FMM_WAVE);
        const bool uniform = __ballot(valid && cl != c0) == 0ull;
        if (uniform) {
            if (c0 != run) {
                if (run >= 0) commit_run(bb, run, rlo, rhi);
                run = c0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rlo[d] = INFINITY;
                    rhi[d] = -INFINITY;
                }
            }
            if (valid) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rlo[d] = fmin(rlo[d], v[d]);
                    rhi[d] = fmax(rhi[d], v[d]);
                }
            }
        } else if (valid) {
            commit_box(bb, cl, v, v);
        }
    }
    if (part) {
        const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FMM_WAVE;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int o = FMM_WAVE / 2; o > 0; o >>= 1) {
                rlo[d] = fmin(rlo[d], __shfl_xor(rlo[d], o, FMM_WAVE));
                rhi[d] = fmax(rhi[d], __shfl_xor(rhi[d], o, FMM_WAVE));
            }
            if (lane == 0) {
                part[6 * wave + d] = ordered_key(rlo[d]);
                part[6 * wave + 3 + d] = ordered_key(rhi[d]);
            }
        }
        return;
    }
    if (run >= 0) commit_run(bb, run, rlo, rhi);
}

// the box of the single cluster from the wavefronts' slots (one block)
__global__ void __launch_bounds__(256) k_bbox_parts(const unsigned long long *part, int nwaves,
                                                    unsigned long long *bb) {
    __shared__ unsigned long long red[4][6];
    unsigned long long v[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
    for (int w = threadIdx.x; w < nwaves; w += blockDim.x)
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const unsigned long long x = part[6 * w + d];
            v[d] = d < 3 ? (x < v[d] ? x : v[d]) : (x > v[d] ? x : v[d]);
        }
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
        for (int o = FMM_WAVE / 2; o > 0; o >>= 1) {
            const unsigned long long x = __shfl_xor(v[d], o, FMM_WAVE);
            v[d] = d < 3 ? (x < v[d] ? x : v[d]) : (x > v[d] ? x : v[d]);
        }
    if (lane_id() == 0)
#pragma unroll
        for (int d = 0; d < 6; ++d) red[threadIdx.x / FMM_WAVE][d] = v[d];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        unsigned long long r = red[0][d];
        for (int w = 1; w < 4; ++w) r = d < 3 ? (red[w][d] < r ? red[w][d] : r) : (red[w][d] > r ? red[w][d] : r);
        bb[d] = r;
    }
}

__global__ void k_bbox_init(int K, unsigned long long *bb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * K) bb[i] = (i % 6) < 3 ? ~0ull : 0ull;
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_keys(const double *pos, int64_t n, int K, const int64_t *off,
                       const unsigned long long *bb, uint64_t *key, uint32_t *idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long *b = bb + 6 * cluster_of(off, K, i);
    double lo[3], L = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = ordered_val(b[d]);
        L = fmax(L, ordered_val(b[3 + d]) - lo[d]);
    }
    const double scale = L > 0.0 ? 2097152.0 / L : 0.0;   // 2^21 cells per axis
    uint32_t q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = __dmul_rn(pos[3 * i + d] - lo[d], scale);
        q[d] = u >= 2097151.0 ? 2097151u : (uint32_t)u;
    }
    key[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    idx[i] = (uint32_t)i;
}

// second sort of a batch: by cluster, carrying the position in key order
__global__ void k_cluster_keys(const uint32_t *idx, int64_t n, int K, const int64_t *off,
                               uint64_t *ckey, uint32_t *pos_in_key_order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ckey[i] = (uint64_t)cluster_of(off, K, idx[i]);
    pos_in_key_order[i] = (uint32_t)i;
}

__global__ void k_apply_order(const uint32_t *order, const uint64_t *key, const uint32_t *idx,
                              int64_t n, uint64_t *key_out, uint32_t *idx_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = order[i];
    key_out[i] = key[j];
    idx_out[i] = idx[j];
}

__global__ void k_gather(const double *pos, const double *mass, const uint32_t *perm, int64_t n,
                         double *x, double *y, double *z, double *m, double4 *xyzm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    const double a = pos[3 * j], b = pos[3 * j + 1], c = pos[3 * j + 2], w = mass[j];
    x[i] = a; y[i] = b; z[i] = c; m[i] = w;
    xyzm[i] = make_double4(a, b, c, w);
}

// Deep refinement.  A level-21 cell that holds more than leaf_size particles
// (a dense cusp inside a very wide halo) is split further by the next 21 bits
// of the same quantisation, u * 2^21 with u the product of the first word
// (exact: a power-of-two scale), so both words describe one 42-bit cell index
// per axis.  Only the particles of such cells get a second word; the sort then
// orders each overfull run by (second word, position), and positions inside a
// run follow the input order.
__global__ void k_deep_keys(const double *pos, const uint32_t *perm, const uint64_t *key,
                            int64_t n, int K, const int64_t *off, const unsigned long long *bb,
                            int leaf_size, uint64_t *key2, uint64_t *runstart, uint32_t *iota,
                            int *any) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // sorted positions keep the cluster ranges [off[c], off[c+1])
    const int c = cluster_of(off, K, i);
    const int64_t c0 = K > 1 ? off[c] : 0, c1 = K > 1 ? off[c + 1] : n;
    const uint64_t k = key[i];
    int64_t lo = c0, hi = i;            // first position with key == k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    const int64_t a = lo;
    lo = i + 1;
    hi = c1;                            // first position with key > k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] <= k) lo = mid + 1;
        else hi = mid;
    }
    const int64_t b = lo;
    runstart[i] = (uint64_t)a;
    iota[i] = (uint32_t)i;
    uint64_t k2 = 0;
    if (b - a > leaf_size) {
        const unsigned long long *box = bb + 6 * c;
        double l[3], L = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            l[d] = ordered_val(box[d]);
            L = fmax(L, ordered_val(box[3 + d]) - l[d]);
        }
        const double scale = L > 0.0 ? 2097152.0 / L : 0.0;
        const uint32_t j = perm[i];
        uint32_t q[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double u = __dmul_rn(pos[3 * (int64_t)j + d] - l[d], scale);
            const double u42 = u * 2097152.0;
            const uint64_t v = u42 >= 4398046511103.0 ? 4398046511103ull : (uint64_t)u42;
            q[d] = (uint32_t)(v & 2097151u);
        }
        k2 = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
        if (i == a) atomicOr(any, 1);
    }
    key2[i] = k2;
}

__global__ void k_gather_u64(const uint32_t *order, const uint64_t *in, int64_t n,
                             uint64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[order[i]];
}

__global__ void k_apply_order2(const uint32_t *order, const uint64_t *key, const uint64_t *key2,
                               const uint32_t *idx, int64_t n, uint64_t *key_out,
                               uint64_t *key2_out, uint32_t *idx_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = order[i];
    key_out[i] = key[j];
    key2_out[i] = key2[j];
    idx_out[i] = idx[j];
}

// ---- the octree from the run structure of the sorted keys -----------------
// The particles are sorted by (cluster, first key word, second key word), so
// every cell of the octree is a run of particles with one key prefix: at
// level L in 1..21 the top L octal digits of the first word, at L in 22..42
// also the top L - 21 digits of the second word (zero outside level-21 cells
// holding more than n_L particles, which are the only ones refined further),
// at level 0 the cluster.  A cell is split when it holds more than n_L
// particles, so the cell at level L holding particle i exists iff L = 0 or the
// run at level L - 1 holding i has more than n_L particles.  That run has more
// than n_L particles iff some window of n_L + 1 consecutive particles
// containing i shares the prefix of level L - 1, i.e. iff
//   F(i) = max over j in [i - n_L, i] of g(j) >= L - 1,
//   g(j) = levels shared by particles j and j + n_L.
// So particle i lies in cells at levels 0 .. D(i) = min(F(i) + 1, 42) (0 if
// no window fits), and the cells whose first particle is b are those at the
// levels from h(b) + 1 to D(b), h(b) = levels shared by b - 1 and b (-1 at the
// start of a cluster).  Every cell of every level is thus found in one pass
// over the particles; sorting the cells by level (stable, so key order within
// a level) numbers them as the level-by-level definition does.

// levels 0..42 on which the cells of particles i and j agree (-1: different
// clusters); cl holds the cluster of each particle or is null for one cluster
__device__ __forceinline__ int shared_levels(const uint64_t *key, const uint64_t *key2,
                                             const int64_t *off, int K, int64_t i, int64_t j) {
    if (K > 1 && cluster_of(off, K, i) != cluster_of(off, K, j)) return -1;
    const uint64_t x = key[i] ^ key[j];
    if (x) return 20 - (63 - __clzll((long long)x)) / 3;
    const uint64_t x2 = key2[i] ^ key2[j];
    if (x2) return 41 - (63 - __clzll((long long)x2)) / 3;
    return FMM_MAXLEVEL;
}

__global__ void k_tree_window_g(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                                const int64_t *off, int leaf_size, int *g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g[i] = i + leaf_size < n ? shared_levels(key, key2, off, K, i, i + leaf_size) : -1;
}

// running maxima of g inside consecutive chunks of w = n_L + 1 entries, from
// the left (pre) and from the right (suf); the maximum over a window of w
// entries starting at a is max(suf[a], pre[a + w - 1]) (van Herk / Gil-Werman)
__global__ void k_tree_window_scan(const int *g, int64_t n, int w, int *pre, int *suf) {
    const int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t a = ch * w;
    if (a >= n) return;
    const int64_t b = min(n, a + w);
    int m = -1;
    for (int64_t i = a; i < b; ++i) {
        m = max(m, g[i]);
        pre[i] = m;
    }
    m = -1;
    for (int64_t i = b - 1; i >= a; --i) {
        m = max(m, g[i]);
        suf[i] = m;
    }
}

// deepest level of particle i's cells, and the levels it shares with i - 1
__device__ __forceinline__ void cell_levels(const uint64_t *key, const uint64_t *key2, int64_t n,
                                            int K, const int64_t *off, int leaf_size,
                                            const int *pre, const int *suf, int64_t i, int &h,
                                            int &D) {
    const int64_t a = i - leaf_size;
    const int F = a < 0 ? pre[i] : max(suf[a], pre[i]);
    D = F < 0 ? 0 : min(F + 1, FMM_MAXLEVEL);
    h = i > 0 ? shared_levels(key, key2, off, K, i - 1, i) : -1;
}

// cnt[i] = number of cells whose first particle is i; cnt[n] = 0
__global__ void k_tree_count(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                             const int64_t *off, int leaf_size, const int *pre, const int *suf,
                             int *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        cnt[n] = 0;
        return;
    }
    int h, D;
    cell_levels(key, key2, n, K, off, leaf_size, pre, suf, i, h, D);
    cnt[i] = max(0, D - h);
}

// cells in particle order: key (level << 32) | first particle, at the
// particle's offset from the exclusive scan of the counts
__global__ void k_tree_emit(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                            const int64_t *off, int leaf_size, const int *pre, const int *suf,
                            const int *base, uint64_t *cell) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c0 = base[i], c1 = base[i + 1];
    if (c1 == c0) return;
    int h, D;
    cell_levels(key, key2, n, K, off, leaf_size, pre, suf, i, h, D);
    for (int L = h + 1; L <= D; ++L) cell[c0 + (L - h - 1)] = ((uint64_t)L << 32) | (uint64_t)i;
}

// first cell of each level in the level-sorted cells: ls[L] for L = 0..43
__global__ void k_tree_levels(const uint64_t *cell, int ncells, int *ls) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    const int L = c < ncells ? (int)(cell[c] >> 32) : FMM_MAXLEVEL + 1;
    const int Lp = c > 0 ? (int)(cell[c - 1] >> 32) : -1;
    for (int l = Lp + 1; l <= L; ++l) ls[l] = c;     // levels without cells start here too
}

// every cell: range, level, parent; links cleared
__global__ void k_tree_cells(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                             const int64_t *off, const uint64_t *cell, int ncells, const int *ls,
                             TreeArrays t) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int L = (int)(cell[c] >> 32);
    const int64_t b = (int64_t)(cell[c] & 0xffffffffull);
    // end: first particle after b that leaves the level-L prefix (the number of
    // shared levels only falls along the sorted keys)
    int64_t lo = b + 1, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (shared_levels(key, key2, off, K, b, mid) >= L) lo = mid + 1;
        else hi = mid;
    }
    int parent = -1;
    if (L > 0) {                      // the last cell of level L - 1 starting at or before b
        int plo = ls[L - 1], phi = ls[L] - 1;
        while (plo < phi) {
            const int mid = (plo + phi + 1) >> 1;
            if ((int64_t)(cell[mid] & 0xffffffffull) <= b) plo = mid;
            else phi = mid - 1;
        }
        parent = plo;
    }
    t.beg[c] = (int)b;
    t.end[c] = (int)lo;
    t.level[c] = L;
    t.parent[c] = parent;
    t.nchild[c] = 0;
    t.child0[c] = -1;
}

// children counted at their parent; the child sharing its parent's first
// particle is the first child (children are consecutive within their level)
__global__ void k_tree_links(int ncells, TreeArrays t) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int pc = t.parent[c];
    if (pc < 0) return;
    atomicAdd(&t.nchild[pc], 1);
    if (t.beg[pc] == t.beg[c]) t.child0[pc] = c;
}

__global__ void k_leaf_flags(TreeArrays t, int ncells, int *flags) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    if (t.nchild[c] == 0) flags[t.beg[c]] = 1;
}

__global__ void k_leaf_ranges(TreeArrays t, int ncells, const int *scan, int *leaf_cell) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int lo = scan[t.beg[c]], hi = scan[t.end[c]];
    t.leaf_lo[c] = lo;
    t.leaf_hi[c] = hi;
    if (t.nchild[c] == 0) leaf_cell[lo] = c;
}

__global__ void k_leaf_of(const int *scan, int64_t n, int *leaf_of) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) leaf_of[i] = scan[i + 1] - 1;
}

__global__ void k_geometry_level(TreeArrays t, int c0, int c1, const double *x, const double *y,
                                 const double *z, const double *m) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    const int nch = t.nchild[c];
    if (nch == 0) {
        const int e = t.end[c];
#pragma unroll 8
        for (int i = t.beg[c]; i < e; ++i) {
            const double a = x[i], b = y[i], d = z[i], w = m[i];
            lo[0] = fmin(lo[0], a); hi[0] = fmax(hi[0], a);
            lo[1] = fmin(lo[1], b); hi[1] = fmax(hi[1], b);
            lo[2] = fmin(lo[2], d); hi[2] = fmax(hi[2], d);
            M += w; sx = fma(w, a, sx); sy = fma(w, b, sy); sz = fma(w, d, sz);
        }
    } else {
        // the loads of all (at most 8) children first, so that they are in
        // flight together; a missing child reads the first one and is skipped
        const int k0 = t.child0[c];
        double clo[8][3], chi[8][3], cw[8];
        double4 cq[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + (j < nch ? j : 0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                clo[j][d] = t.lo[3 * k + d];
                chi[j][d] = t.hi[3 * k + d];
            }
            cw[j] = t.mass[k];
            cq[j] = t.com[k];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < nch) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    lo[d] = fmin(lo[d], clo[j][d]);
                    hi[d] = fmax(hi[d], chi[j][d]);
                }
                const double w = cw[j];
                M += w; sx = fma(w, cq[j].x, sx); sy = fma(w, cq[j].y, sy); sz = fma(w, cq[j].z, sz);
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t.lo[3 * c + d] = lo[d];
        t.hi[3 * c + d] = hi[d];
    }
    t.mass[c] = M;
    t.com[c] = make_double4(sx / M, sy / M, sz / M, 0.0);
    t.cen[c] = make_double4((lo[0] + hi[0]) * 0.5, (lo[1] + hi[1]) * 0.5, (lo[2] + hi[2]) * 0.5, 0.0);
    t.rho2[3 * c] = 0ull;
    t.rho2[3 * c + 1] = 0ull;
    t.rho2[3 * c + 2] = 0ull;
}

// Squared distance without fused multiply-adds, so that the radius of a cell
// is the same number the definition gives on any machine.
__device__ __forceinline__ double dist2_rn(double ax, double ay, double az, double bx, double by,
                                           double bz) {
    return dist2_exact(ax, ay, az, bx, by, bz);
}

constexpr int RADII_ROWS = 4;   // rows of 64 consecutive particles per wavefront

// atomicMax that first reads the current value and skips the atomic when it
// cannot raise it: the top cells get one commit per wavefront, and most of
// those atomics on a few addresses are needless once the maximum is in place.
// A stale read is never above the current value, so nothing needed is
// skipped.
__device__ __forceinline__ void max_commit(unsigned long long *a, double v) {
    const unsigned long long b = dbits(v);
    if (b > __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(a, b);
}

// Radii of every cell at every level in one pass over the particles.  Each
// wavefront owns 64 * RADII_ROWS consecutive particles, holds their positions
// and their current ancestors (with the ancestors' levels: a parent is one
// level up), and goes up the tree level by level (deepest first): the centre
// loads of all rows are issued together, then per row the squared distances
// are reduced per cell across the 64 lanes (cells are contiguous particle
// ranges, so equal cells are adjacent lanes), the cell that spills into the
// next row is carried, and each cell's maximum is committed with one atomic
// per wavefront.  CAND = false: squared distances to the box midpoint and the
// centre of mass, into rho2[3c] and rho2[3c + 1]; CAND = true: to the
// enclosing-sphere candidate, into rho2[3c + 2].
template <bool CAND>
__global__ void __launch_bounds__(256)
k_radii(TreeArrays t, int64_t n, const int *leaf_of, const int *leaf_cell, int maxlevel,
        const double *x, const double *y, const double *z) {
    constexpr int NV = CAND ? 1 : 2;
    constexpr int SLOT = CAND ? 2 : 0;
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FMM_WAVE;
    const int64_t base = wave * (FMM_WAVE * RADII_ROWS);
    if (base >= n) return;
    int anc[RADII_ROWS], alev[RADII_ROWS];
    double px[RADII_ROWS], py[RADII_ROWS], pz[RADII_ROWS];
#pragma unroll
    for (int j = 0; j < RADII_ROWS; ++j) {
        const int64_t i = base + j * FMM_WAVE + lane;
        anc[j] = i < n ? leaf_cell[leaf_of[i]] : -1;
        px[j] = i < n ? x[i] : 0.0;
        py[j] = i < n ? y[i] : 0.0;
        pz[j] = i < n ? z[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < RADII_ROWS; ++j) alev[j] = anc[j] >= 0 ? t.level[anc[j]] : -1;
    for (int L = maxlevel; L >= 0; --L) {
        // this level's cell of every row, its squared distances, the next
        // ancestor; the loads are unconditional (cell 0 stands in for a row
        // with no cell at this level) so that all rows' loads are in flight
        // together
        int key[RADII_ROWS], par[RADII_ROWS];
        double4 ca[RADII_ROWS], cb[RADII_ROWS];
#pragma unroll
        for (int j = 0; j < RADII_ROWS; ++j) {
            key[j] = alev[j] == L ? anc[j] : -1;
            const int kk = key[j] >= 0 ? key[j] : 0;
            par[j] = t.parent[kk];
            if constexpr (CAND) {
                ca[j] = t.bsph[kk];
            } else {
                ca[j] = t.cen[kk];
                cb[j] = t.com[kk];
            }
        }
        double v[RADII_ROWS][NV];
#pragma unroll
        for (int j = 0; j < RADII_ROWS; ++j) {
            const bool has = key[j] >= 0;
            v[j][0] = has ? dist2_rn(px[j], py[j], pz[j], ca[j].x, ca[j].y, ca[j].z) : 0.0;
            if constexpr (!CAND)
                v[j][1] = has ? dist2_rn(px[j], py[j], pz[j], cb[j].x, cb[j].y, cb[j].z) : 0.0;
            anc[j] = has ? par[j] : anc[j];
            alev[j] = has ? L - 1 : alev[j];
        }
        int ckey = -1;
        double cv[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) cv[u] = 0.0;
#pragma unroll
        for (int j = 0; j < RADII_ROWS; ++j) {
            const int kj = key[j];
            // segmented maximum towards the first lane of each run of equal keys
#pragma unroll
            for (int off = 1; off < FMM_WAVE; off <<= 1) {
                const int ok = __shfl_down(kj, off, FMM_WAVE);
                double o[NV];
#pragma unroll
                for (int u = 0; u < NV; ++u) o[u] = __shfl_down(v[j][u], off, FMM_WAVE);
                if (lane + off < FMM_WAVE && ok == kj) {
#pragma unroll
                    for (int u = 0; u < NV; ++u) v[j][u] = fmax(v[j][u], o[u]);
                }
            }
            const int prev = __shfl_up(kj, 1, FMM_WAVE);
            const bool head = kj >= 0 && (lane == 0 || prev != kj);
            const int last = __shfl(kj, FMM_WAVE - 1, FMM_WAVE);
            const int first = __shfl(kj, 0, FMM_WAVE);
            // merge or flush the carried run
            if (lane == 0 && ckey >= 0) {
                if (first == ckey) {
#pragma unroll
                    for (int u = 0; u < NV; ++u) v[j][u] = fmax(v[j][u], cv[u]);
                } else {
#pragma unroll
                    for (int u = 0; u < NV; ++u) max_commit(&t.rho2[3 * ckey + SLOT + u], cv[u]);
                }
            }
            // the run containing lane 63 may continue into the next row
            const bool open = head && kj == last;
            if (head && !open) {
#pragma unroll
                for (int u = 0; u < NV; ++u) max_commit(&t.rho2[3 * kj + SLOT + u], v[j][u]);
            }
            // hand the open run to lane 0 as the new carry
            const unsigned long long om = __ballot(open);
            if (om) {
                const int src = __ffsll((long long)om) - 1;
#pragma unroll
                for (int u = 0; u < NV; ++u) cv[u] = __shfl(v[j][u], src, FMM_WAVE);
                ckey = last;
            } else {
                ckey = -1;
            }
        }
        if (lane == 0 && ckey >= 0) {
#pragma unroll
            for (int u = 0; u < NV; ++u) max_commit(&t.rho2[3 * ckey + SLOT + u], cv[u]);
        }
    }
}

// Radii about the midpoint and the centre of mass from the squared maxima.
__global__ void k_radii_finish(TreeArrays t, int ncells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    t.cen[c].w = __dsqrt_rn(bitsd(t.rho2[3 * c]));
    t.com[c].w = __dsqrt_rn(bitsd(t.rho2[3 * c + 1]));
}

// Each cell takes its enclosing-sphere candidate where the radius about it
// is strictly smaller than about the midpoint.
__global__ void k_centre_select(TreeArrays t, int ncells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const double r2b = bitsd(t.rho2[3 * c + 2]);
    if (r2b < bitsd(t.rho2[3 * c])) {
        const double4 b = t.bsph[c];
        t.cen[c] = make_double4(b.x, b.y, b.z, __dsqrt_rn(r2b));
    }
}

// ------------------------------------------------- enclosing-sphere centre
//
// Sec. 5.1.1 expands about the centre of the smallest sphere enclosing the
// spheres of a cell's grand-daughters.  That centre is approximated here by
// the Frank-Wolfe iteration with exact line search for the minimum enclosing
// ball (Yildirim 2008, SIAM J. Optim. 19, 1368, Algorithm 1): start at the
// midpoint of a and b, a the point of the set farthest from the box midpoint
// and b the point farthest from a, with gamma = |a - b|^2 / 4; each step takes
// the farthest point q (D2 = |q - c|^2), stops when gamma <= 0 or
// delta = D2 / gamma - 1 <= FW_TOL (the radius about c is then within 0.1% of
// the optimum, gamma being a lower bound of its square), else moves c by
// lambda = delta / (2 (1 + delta))
// of the way to q and sets gamma = (1 - lambda) gamma + lambda (1 - lambda) D2;
// at most FW_ITERS steps.  The set of a leaf is its particles, compared by
// squared distance; that of an internal cell the spheres (b, R) of its
// grand-daughters, where a daughter that is a leaf stands in for its own
// daughters, compared by d + R (the farthest point of a sphere at distance d
// from c), with D2 = (d + R)^2.  A cell's sphere is its final c and R, the
// largest such distance over its set.  Ties in "farthest" go to the first
// entry in Morton order, and each operation is a single correctly rounded one
// in a fixed order (contraction into fused multiply-adds is switched off), so
// the centre is a deterministic function of the particle positions.
//
// ENC_G lanes per cell hold the set in registers, ENC_SLOTS entries to a
// lane (entry i in slot i / ENC_G of lane i % ENC_G), so that a step is
// arithmetic and lane exchanges only; a leaf with more particles than that
// reads them from memory at every step.
constexpr int FW_ITERS = 16;
constexpr double FW_TOL = 2e-3;   // stop once D2 <= (1 + FW_TOL) gamma
constexpr int ENC_G = 16;         // one DPP row
constexpr int ENC_SLOTS = 8;
constexpr int ENC_REG = ENC_G * ENC_SLOTS;

// Lane exchanges inside a row of 16 lanes by DPP: swap neighbours, swap pairs
// of a quad, mirror each half-row, mirror the row.  After the four steps of a
// commutative, associative combine every lane of the row holds the result.
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
    return __hiloint2double(dpp_int<CTRL>(__double2hiint(v)), dpp_int<CTRL>(__double2loint(v)));
}

template <int CTRL>
__device__ __forceinline__ void argmax_step(double &e, int &j) {
    const double oe = dpp_double<CTRL>(e);
    const int oj = dpp_int<CTRL>(j);
    if (oe > e || (oe == e && oj < j)) {
        e = oe;
        j = oj;
    }
}

// largest e over the lane group, ties to the smallest j; every lane ends with it
__device__ __forceinline__ void group_argmax_first(double &e, int &j) {
    static_assert(ENC_G == 16, "the DPP steps span one row of 16 lanes");
    argmax_step<DPP_XOR1>(e, j);
    argmax_step<DPP_XOR2>(e, j);
    argmax_step<DPP_HALF_MIRROR>(e, j);
    argmax_step<DPP_MIRROR>(e, j);
}

__device__ __forceinline__ double group_max(double v) {
    v = fmax(v, dpp_double<DPP_XOR1>(v));
    v = fmax(v, dpp_double<DPP_XOR2>(v));
    v = fmax(v, dpp_double<DPP_HALF_MIRROR>(v));
    return fmax(v, dpp_double<DPP_MIRROR>(v));
}

// cell of entry `item` of the grand-daughter list of internal cell c
__device__ __forceinline__ int granddaughter(const TreeArrays &t, int c, int item) {
    const int k0 = t.child0[c], nch = t.nchild[c];
    for (int k = k0; k < k0 + nch; ++k) {
        const int nk = t.nchild[k];
        const int cnt = nk == 0 ? 1 : nk;
        if (item < cnt) return nk == 0 ? k : t.child0[k] + item;
        item -= cnt;
    }
    return -1;
}

// One Frank-Wolfe step from (cx, cy, cz) towards q; false if converged.
__device__ __forceinline__ bool fw_step(double &cx, double &cy, double &cz, double &gamma,
                                        double qx, double qy, double qz, double D2) {
#pragma clang fp contract(off)
    if (!(gamma > 0.0)) return false;
    const double delta = D2 / gamma - 1.0;
    if (!(delta > FW_TOL)) return false;
    const double lambda = delta / (2.0 * (1.0 + delta));
    cx = cx + lambda * (qx - cx);
    cy = cy + lambda * (qy - cy);
    cz = cz + lambda * (qz - cz);
    const double om = 1.0 - lambda;
    gamma = om * gamma + (lambda * om) * D2;
    return true;
}

// The farthest point q from (px, py, pz) of the set of one cell, held by the
// lanes of its group, and D2 = |q - p|^2.  points: particles (a leaf),
// compared by squared distance; else spheres (x, y, z, R), compared by d + R.
// regs: the entries are in X, Y, Z, R (entry i in slot i / ENC_G of lane
// i % ENC_G); else a leaf's particles [b, b + n) are read from memory.
__device__ __forceinline__ double enc_farthest(bool points, bool regs, int n, int sub, int b,
                                               const double *x, const double *y,
                                               const double *z, const double (&X)[ENC_SLOTS],
                                               const double (&Y)[ENC_SLOTS],
                                               const double (&Z)[ENC_SLOTS],
                                               const double (&R)[ENC_SLOTS], double px,
                                               double py, double pz, double &qx, double &qy,
                                               double &qz) {
#pragma clang fp contract(off)
    // each lane's own best entry (the first in its slot order) and its data;
    // the group's winner is the best of these, sent by the lane that has it
    double best = -1.0, sx = 0.0, sy = 0.0, sz = 0.0, sr = 0.0;
    int j = INT_MAX;
    if (regs) {
#pragma unroll
        for (int s = 0; s < ENC_SLOTS; ++s) {
            const int item = sub + ENC_G * s;
            if (item < n) {
                const double d2 = dist2_rn(X[s], Y[s], Z[s], px, py, pz);
                const double key = points ? d2 : __dsqrt_rn(d2) + R[s];
                if (key > best) {
                    best = key;
                    j = item;
                    sx = X[s];
                    sy = Y[s];
                    sz = Z[s];
                    sr = R[s];
                }
            }
        }
    } else {
        for (int i = sub; i < n; i += ENC_G) {
            const double d2 = dist2_rn(x[b + i], y[b + i], z[b + i], px, py, pz);
            if (d2 > best) {
                best = d2;
                j = i;
            }
        }
        if (j != INT_MAX) {
            sx = x[b + j];
            sy = y[b + j];
            sz = z[b + j];
        }
    }
    group_argmax_first(best, j);
    if (j == INT_MAX) j = 0;   // no comparison held (non-finite input): entry 0
    const int owner = j % ENC_G;
    if (j == 0 && best < 0.0) {
        // entry 0 sits in slot 0 of lane 0 (registers) or at b (memory)
        sx = regs ? X[0] : x[b];
        sy = regs ? Y[0] : y[b];
        sz = regs ? Z[0] : z[b];
        sr = R[0];
    }
    sx = __shfl(sx, owner, ENC_G);
    sy = __shfl(sy, owner, ENC_G);
    sz = __shfl(sz, owner, ENC_G);
    if (!points) sr = __shfl(sr, owner, ENC_G);
    if (points) {
        qx = sx;
        qy = sy;
        qz = sz;
        return best;
    }
    const double d = __dsqrt_rn(dist2_rn(sx, sy, sz, px, py, pz));
    if (d > 0.0) {
        const double u = sr / d;
        qx = sx + (sx - px) * u;
        qy = sy + (sy - py) * u;
        qz = sz + (sz - pz) * u;
    } else {
        qx = sx + sr;
        qy = sy;
        qz = sz;
    }
    return best * best;
}

__global__ void __launch_bounds__(256)
k_enclosing_level(TreeArrays t, int c0, int c1, const double *x, const double *y,
                  const double *z) {
#pragma clang fp contract(off)
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = c0 + (int)(gt / ENC_G);
    if (c >= c1) return;   // whole lane groups leave together
    const int sub = (int)(gt % ENC_G);
    const int nch = t.nchild[c];
    const bool points = nch == 0;
    const int b = t.beg[c];
    int n = 0;
    if (points) {
        n = t.end[c] - b;
    } else {
        const int k0 = t.child0[c];
        for (int k = k0; k < k0 + nch; ++k) {
            const int nk = t.nchild[k];
            n += nk == 0 ? 1 : nk;
        }
    }
    const bool regs = n <= ENC_REG;
    double X[ENC_SLOTS], Y[ENC_SLOTS], Z[ENC_SLOTS], R[ENC_SLOTS];
#pragma unroll
    for (int s = 0; s < ENC_SLOTS; ++s) {
        const int item = sub + ENC_G * s;
        double vx = 0.0, vy = 0.0, vz = 0.0, vr = 0.0;
        if (regs && item < n) {
            if (points) {
                vx = x[b + item];
                vy = y[b + item];
                vz = z[b + item];
            } else {
                const double4 v = t.bsph[granddaughter(t, c, item)];
                vx = v.x;
                vy = v.y;
                vz = v.z;
                vr = v.w;
            }
        }
        X[s] = vx;
        Y[s] = vy;
        Z[s] = vz;
        R[s] = vr;
    }
    const double4 mid = t.cen[c];
    double ax, ay, az, bx, by, bz, qx, qy, qz;
    enc_farthest(points, regs, n, sub, b, x, y, z, X, Y, Z, R, mid.x, mid.y, mid.z, ax, ay, az);
    enc_farthest(points, regs, n, sub, b, x, y, z, X, Y, Z, R, ax, ay, az, bx, by, bz);
    double cx = (ax + bx) * 0.5, cy = (ay + by) * 0.5, cz = (az + bz) * 0.5;
    double gamma = dist2_rn(ax, ay, az, bx, by, bz) * 0.25;
    for (int k = 0; k < FW_ITERS; ++k) {
        const double D2 =
            enc_farthest(points, regs, n, sub, b, x, y, z, X, Y, Z, R, cx, cy, cz, qx, qy, qz);
        if (!fw_step(cx, cy, cz, gamma, qx, qy, qz, D2)) break;
    }
    // the cover radius: largest distance (particles) or d + R (spheres)
    double m = 0.0;
    if (regs) {
#pragma unroll
        for (int s = 0; s < ENC_SLOTS; ++s)
            if (sub + ENC_G * s < n) {
                const double d2 = dist2_rn(X[s], Y[s], Z[s], cx, cy, cz);
                m = fmax(m, points ? d2 : __dsqrt_rn(d2) + R[s]);
            }
    } else {
        for (int i = sub; i < n; i += ENC_G)
            m = fmax(m, dist2_rn(x[b + i], y[b + i], z[b + i], cx, cy, cz));
    }
    m = group_max(m);
    const double Rc = points ? __dsqrt_rn(m) : m;
    if (sub == 0) t.bsph[c] = make_double4(cx, cy, cz, Rc);
}

__global__ void k_smin_level(TreeArrays t, int c0, int c1, const double *scale) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    double s = INFINITY;
    const int nch = t.nchild[c];
    if (nch == 0) {
        const int e = t.end[c];
#pragma unroll 8
        for (int i = t.beg[c]; i < e; ++i) s = fmin(s, scale[i]);
    } else {
        // all children's loads in flight together (a missing child re-reads the first)
        const int k0 = t.child0[c];
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = t.smin[k0 + (j < nch ? j : 0)];
#pragma unroll
        for (int j = 0; j < 8; ++j) s = fmin(s, v[j]);
    }
    t.smin[c] = s;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_bbox(const double *pos, int64_t n, int K, const int64_t *off,
                       unsigned long long *bb, hipStream_t s) {
    unsigned g = blocks(n, 256);
    if (g > 256) g = 256;
    if (K == 1) {
        unsigned long long *part = bb + 6;   // 6 keys per wavefront of the launch
        hipLaunchKernelGGL(k_bbox, dim3(g), dim3(256), 0, s, pos, n, K, off, bb, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bbox_parts, dim3(1), dim3(256), 0, s, part, (int)(g * 4), bb);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bbox_init, dim3(blocks(6 * (int64_t)K, 256)), dim3(256), 0, s, K, bb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbox, dim3(g), dim3(256), 0, s, pos, n, K, off, bb,
                       (unsigned long long *)nullptr);
    return hipGetLastError();
}

hipError_t launch_keys(const double *pos, int64_t n, int K, const int64_t *off,
                       const unsigned long long *bb, uint64_t *key, uint32_t *idx,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_keys, dim3(blocks(n, 256)), dim3(256), 0, s, pos, n, K, off, bb, key, idx);
    return hipGetLastError();
}

hipError_t launch_cluster_keys(const uint32_t *idx, int64_t n, int K, const int64_t *off,
                               uint64_t *ckey, uint32_t *order, hipStream_t s) {
    hipLaunchKernelGGL(k_cluster_keys, dim3(blocks(n, 256)), dim3(256), 0, s, idx, n, K, off, ckey,
                       order);
    return hipGetLastError();
}

hipError_t launch_apply_order(const uint32_t *order, const uint64_t *key, const uint32_t *idx,
                              int64_t n, uint64_t *key_out, uint32_t *idx_out, hipStream_t s) {
    hipLaunchKernelGGL(k_apply_order, dim3(blocks(n, 256)), dim3(256), 0, s, order, key, idx, n,
                       key_out, idx_out);
    return hipGetLastError();
}

hipError_t launch_gather(const double *pos, const double *mass, const uint32_t *perm, int64_t n,
                         double *x, double *y, double *z, double *m, double4 *xyzm,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(blocks(n, 256)), dim3(256), 0, s, pos, mass, perm, n, x, y,
                       z, m, xyzm);
    return hipGetLastError();
}

hipError_t launch_tree(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                       const int64_t *off, int leaf_size, int *g, int *pre, int *suf, int *cnt,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_tree_window_g, dim3(blocks(n, 256)), dim3(256), 0, s, key, key2, n, K,
                       off, leaf_size, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int w = leaf_size + 1;
    hipLaunchKernelGGL(k_tree_window_scan, dim3(blocks((n + w - 1) / w, 64)), dim3(64), 0, s, g, n,
                       w, pre, suf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tree_count, dim3(blocks(n + 1, 256)), dim3(256), 0, s, key, key2, n, K,
                       off, leaf_size, pre, suf, cnt);
    return hipGetLastError();
}

hipError_t launch_tree_emit(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                            const int64_t *off, int leaf_size, const int *pre, const int *suf,
                            const int *base, uint64_t *cell, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_emit, dim3(blocks(n, 256)), dim3(256), 0, s, key, key2, n, K, off,
                       leaf_size, pre, suf, base, cell);
    return hipGetLastError();
}

hipError_t launch_tree_levels(const uint64_t *cell, int ncells, int *ls, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_levels, dim3(blocks((int64_t)ncells + 1, 256)), dim3(256), 0, s,
                       cell, ncells, ls);
    return hipGetLastError();
}

hipError_t launch_tree_cells(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                             const int64_t *off, const uint64_t *cell, int ncells, const int *ls,
                             const TreeArrays &t, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_cells, dim3(blocks(ncells, 256)), dim3(256), 0, s, key, key2, n, K,
                       off, cell, ncells, ls, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tree_links, dim3(blocks(ncells, 256)), dim3(256), 0, s, ncells, t);
    return hipGetLastError();
}

hipError_t launch_deep_keys(const double *pos, const uint32_t *perm, const uint64_t *key,
                            int64_t n, int K, const int64_t *off, const unsigned long long *bb,
                            int leaf_size, uint64_t *key2, uint64_t *runstart, uint32_t *iota,
                            int *any, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_deep_keys, dim3(blocks(n, 256)), dim3(256), 0, s, pos, perm, key, n, K,
                       off, bb, leaf_size, key2, runstart, iota, any);
    return hipGetLastError();
}

hipError_t launch_gather_u64(const uint32_t *order, const uint64_t *in, int64_t n, uint64_t *out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u64, dim3(blocks(n, 256)), dim3(256), 0, s, order, in, n, out);
    return hipGetLastError();
}

hipError_t launch_apply_order2(const uint32_t *order, const uint64_t *key, const uint64_t *key2,
                               const uint32_t *idx, int64_t n, uint64_t *key_out,
                               uint64_t *key2_out, uint32_t *idx_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_order2, dim3(blocks(n, 256)), dim3(256), 0, s, order, key, key2,
                       idx, n, key_out, key2_out, idx_out);
    return hipGetLastError();
}

hipError_t launch_leaf_flags(const TreeArrays &t, int ncells, int *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_flags, dim3(blocks(ncells, 256)), dim3(256), 0, s, t, ncells, flags);
    return hipGetLastError();
}

hipError_t launch_leaf_ranges(const TreeArrays &t, int ncells, const int *leafscan,
                              int *leaf_cell, int *leaf_of, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_ranges, dim3(blocks(ncells, 256)), dim3(256), 0, s, t, ncells,
                       leafscan, leaf_cell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_of, dim3(blocks(n, 256)), dim3(256), 0, s, leafscan, n, leaf_of);
    return hipGetLastError();
}

hipError_t launch_geometry_level(const TreeArrays &t, int c0, int c1, const double *x,
                                 const double *y, const double *z, const double *m,
                                 hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_geometry_level, dim3(blocks(c1 - c0, 128)), dim3(128), 0, s, t, c0, c1,
                       x, y, z, m);
    return hipGetLastError();
}

hipError_t launch_enclosing_level(const TreeArrays &t, int c0, int c1, const double *x,
                                  const double *y, const double *z, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_enclosing_level, dim3(blocks((int64_t)(c1 - c0) * ENC_G, 256)),
                       dim3(256), 0, s, t, c0, c1, x, y, z);
    return hipGetLastError();
}

hipError_t launch_radii(const TreeArrays &t, int64_t n, const int *leaf_of, const int *leaf_cell,
                        int maxlevel, const double *x, const double *y, const double *z,
                        bool candidate, hipStream_t s) {
    const int64_t waves = (n + FMM_WAVE * RADII_ROWS - 1) / (FMM_WAVE * RADII_ROWS);
    if (candidate)
        hipLaunchKernelGGL(k_radii<true>, dim3(blocks(waves * FMM_WAVE, 256)), dim3(256), 0, s, t,
                           n, leaf_of, leaf_cell, maxlevel, x, y, z);
    else
        hipLaunchKernelGGL(k_radii<false>, dim3(blocks(waves * FMM_WAVE, 256)), dim3(256), 0, s,
                           t, n, leaf_of, leaf_cell, maxlevel, x, y, z);
    return hipGetLastError();
}

hipError_t launch_radii_finish(const TreeArrays &t, int ncells, hipStream_t s) {
    hipLaunchKernelGGL(k_radii_finish, dim3(blocks(ncells, 256)), dim3(256), 0, s, t, ncells);
    return hipGetLastError();
}

hipError_t launch_centre_select(const TreeArrays &t, int ncells, hipStream_t s) {
    hipLaunchKernelGGL(k_centre_select, dim3(blocks(ncells, 256)), dim3(256), 0, s, t, ncells);
    return hipGetLastError();
}

hipError_t launch_smin_level(const TreeArrays &t, int c0, int c1, const double *scale,
                             hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_smin_level, dim3(blocks(c1 - c0, 128)), dim3(128), 0, s, t, c0, c1,
                       scale);
    return hipGetLastError();
}

}  // namespace fmm
