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
// box; rho = the largest distance of its particles from it (the definitions
// of rho_z and rho_s in Sec. 4).  rho_com likewise about the centre of mass
// (the centre of the low-order estimate, Sec. 5.4.2).
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
// order-preserving keys.  A wavefront keeps the box of its current cluster
// over its chunks of the grid-stride loop and commits it (6 atomics) only when
// the cluster changes and at the end; a chunk that spans clusters commits
// per lane.
__device__ __forceinline__ void commit_box(unsigned long long *bb, int c, const double *lo,
                                           const double *hi) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        atomicMin(&bb[6 * c + d], ordered_key(lo[d]));
        atomicMax(&bb[6 * c + 3 + d], ordered_key(hi[d]));
    }
}

__global__ void k_bbox(const double *pos, int64_t n, int K, const int64_t *off,
                       unsigned long long *bb) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int run = -1;
    double rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(FMM_WAVE - 1));
         base < n; base += stride) {
        const int64_t i = base + lane;
        const bool valid = i < n;
        const int cl = valid ? cluster_of(off, K, i) : -1;
        double lo[3], hi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = valid ? pos[3 * i + d] : 0.0;
            lo[d] = valid ? v : INFINITY;
            hi[d] = valid ? v : -INFINITY;
        }
        const int c0 = __shfl(cl, 0, FMM_WAVE);
        const bool uniform = __ballot(valid && cl != c0) == 0ull;
        if (uniform) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int o = FMM_WAVE / 2; o > 0; o >>= 1) {
                    lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, FMM_WAVE));
                    hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, FMM_WAVE));
                }
            }
            if (c0 != run) {
                if (run >= 0 && lane == 0) commit_box(bb, run, rlo, rhi);
                run = c0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rlo[d] = lo[d];
                    rhi[d] = hi[d];
                }
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rlo[d] = fmin(rlo[d], lo[d]);
                    rhi[d] = fmax(rhi[d], hi[d]);
                }
            }
        } else if (valid) {
            commit_box(bb, cl, lo, hi);
        }
    }
    if (run >= 0 && lane == 0) commit_box(bb, run, rlo, rhi);
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
        for (int i = t.beg[c]; i < t.end[c]; ++i) {
            const double a = x[i], b = y[i], d = z[i], w = m[i];
            lo[0] = fmin(lo[0], a); hi[0] = fmax(hi[0], a);
            lo[1] = fmin(lo[1], b); hi[1] = fmax(hi[1], b);
            lo[2] = fmin(lo[2], d); hi[2] = fmax(hi[2], d);
            M += w; sx = fma(w, a, sx); sy = fma(w, b, sy); sz = fma(w, d, sz);
        }
    } else {
        const int c0_ = t.child0[c];
        for (int k = c0_; k < c0_ + nch; ++k) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[d] = fmin(lo[d], t.lo[3 * k + d]);
                hi[d] = fmax(hi[d], t.hi[3 * k + d]);
            }
            const double w = t.mass[k];
            const double4 q = t.com[k];
            M += w; sx = fma(w, q.x, sx); sy = fma(w, q.y, sy); sz = fma(w, q.z, sz);
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
    t.rho2[2 * c] = 0ull;
    t.rho2[2 * c + 1] = 0ull;
}

// Squared distance without contraction into fused multiply-adds, so that the
// radius of a cell is the same number the definition gives on any machine.
__device__ __forceinline__ double dist2_rn(double ax, double ay, double az, double bx, double by,
                                           double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

constexpr int RADII_ROWS = 16;   // rows of 64 consecutive particles per wavefront

// Radii of every cell at every level in one pass over the particles.  Each
// wavefront owns 64*16 consecutive particles; it walks each particle's
// ancestor chain level by level (deepest first), reduces the squared
// distances per cell across the row of 64 lanes (cells are contiguous
// particle ranges, so equal cells are adjacent lanes), carries the cell that
// spills into the next row, and commits each cell's maximum with one atomic
// per wavefront.
__global__ void __launch_bounds__(256)
k_radii(TreeArrays t, int64_t n, const int *leaf_of, const int *leaf_cell, int maxlevel,
        const double *x, const double *y, const double *z) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FMM_WAVE;
    const int64_t base = wave * (FMM_WAVE * RADII_ROWS);
    if (base >= n) return;
    int anc[RADII_ROWS];
#pragma unroll
    for (int j = 0; j < RADII_ROWS; ++j) {
        const int64_t i = base + j * FMM_WAVE + lane;
        anc[j] = i < n ? leaf_cell[leaf_of[i]] : -1;
    }
    for (int L = maxlevel; L >= 0; --L) {
        int ckey = -1;
        double cv0 = 0.0, cv1 = 0.0;
#pragma unroll
        for (int j = 0; j < RADII_ROWS; ++j) {
            const int64_t i = base + j * FMM_WAVE + lane;
            int key = -1;
            double v0 = 0.0, v1 = 0.0;
            if (anc[j] >= 0 && t.level[anc[j]] == L) {
                key = anc[j];
                const double px = x[i], py = y[i], pz = z[i];
                const double4 c = t.cen[key], q = t.com[key];
                v0 = dist2_rn(px, py, pz, c.x, c.y, c.z);
                v1 = dist2_rn(px, py, pz, q.x, q.y, q.z);
                anc[j] = t.parent[key];
            }
            // segmented maximum towards the first lane of each run of equal keys
#pragma unroll
            for (int off = 1; off < FMM_WAVE; off <<= 1) {
                const int ok = __shfl_down(key, off, FMM_WAVE);
                const double o0 = __shfl_down(v0, off, FMM_WAVE);
                const double o1 = __shfl_down(v1, off, FMM_WAVE);
                if (lane + off < FMM_WAVE && ok == key) {
                    v0 = fmax(v0, o0);
                    v1 = fmax(v1, o1);
                }
            }
            const int prev = __shfl_up(key, 1, FMM_WAVE);
            const bool head = key >= 0 && (lane == 0 || prev != key);
            const int last = __shfl(key, FMM_WAVE - 1, FMM_WAVE);
            const int first = __shfl(key, 0, FMM_WAVE);
            // merge or flush the carried run
            if (lane == 0 && ckey >= 0) {
                if (first == ckey) {
                    v0 = fmax(v0, cv0);
                    v1 = fmax(v1, cv1);
                } else {
                    atomicMax(&t.rho2[2 * ckey], dbits(cv0));
                    atomicMax(&t.rho2[2 * ckey + 1], dbits(cv1));
                }
            }
            // the run containing lane 63 may continue into the next row
            const bool open = head && key == last;
            if (head && !open) {
                atomicMax(&t.rho2[2 * key], dbits(v0));
                atomicMax(&t.rho2[2 * key + 1], dbits(v1));
            }
            // hand the open run to lane 0 as the new carry
            const unsigned long long om = __ballot(open);
            if (om) {
                const int src = __ffsll((long long)om) - 1;
                const double s0 = __shfl(v0, src, FMM_WAVE), s1 = __shfl(v1, src, FMM_WAVE);
                ckey = last;
                cv0 = s0;
                cv1 = s1;
            } else {
                ckey = -1;
            }
        }
        if (lane == 0 && ckey >= 0) {
            atomicMax(&t.rho2[2 * ckey], dbits(cv0));
            atomicMax(&t.rho2[2 * ckey + 1], dbits(cv1));
        }
    }
}

__global__ void k_radii_finish(TreeArrays t, int ncells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    t.cen[c].w = __dsqrt_rn(bitsd(t.rho2[2 * c]));
    t.com[c].w = __dsqrt_rn(bitsd(t.rho2[2 * c + 1]));
}

__global__ void k_smin_level(TreeArrays t, int c0, int c1, const double *scale) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    double s = INFINITY;
    const int nch = t.nchild[c];
    if (nch == 0) {
        for (int i = t.beg[c]; i < t.end[c]; ++i) s = fmin(s, scale[i]);
    } else {
        const int k0 = t.child0[c];
        for (int k = k0; k < k0 + nch; ++k) s = fmin(s, t.smin[k]);
    }
    t.smin[c] = s;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_bbox(const double *pos, int64_t n, int K, const int64_t *off,
                       unsigned long long *bb, hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_init, dim3(blocks(6 * (int64_t)K, 256)), dim3(256), 0, s, K, bb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned g = blocks(n, 256);
    if (g > 256) g = 256;
    hipLaunchKernelGGL(k_bbox, dim3(g), dim3(256), 0, s, pos, n, K, off, bb);
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

hipError_t launch_radii(const TreeArrays &t, int64_t n, const int *leaf_of, const int *leaf_cell,
                        int maxlevel, const double *x, const double *y, const double *z,
                        hipStream_t s) {
    const int64_t waves = (n + FMM_WAVE * RADII_ROWS - 1) / (FMM_WAVE * RADII_ROWS);
    hipLaunchKernelGGL(k_radii, dim3(blocks(waves * FMM_WAVE, 256)), dim3(256), 0, s, t, n,
                       leaf_of, leaf_cell, maxlevel, x, y, z);
    return hipGetLastError();
}

hipError_t launch_radii_finish(const TreeArrays &t, int ncells, hipStream_t s) {
    hipLaunchKernelGGL(k_radii_finish, dim3(blocks(ncells, 256)), dim3(256), 0, s, t, ncells);
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
