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

// boundaries of the 8 octants at `level + 1` inside the cell's key range
__device__ void octant_bounds(const uint64_t *key1, const uint64_t *key2, int beg, int end,
                              int level, int b[9]) {
    const bool deep = level >= FMM_KEYLEVELS;
    const uint64_t *key = deep ? key2 : key1;
    const int shift = 3 * ((deep ? FMM_MAXLEVEL : FMM_KEYLEVELS) - (level + 1));
    b[0] = beg;
    b[8] = end;
#pragma unroll
    for (int o = 1; o < 8; ++o) {
        int lo = b[o - 1], hi = end;       // first index with digit >= o
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)((key[mid] >> shift) & 7u) < o) lo = mid + 1;
            else hi = mid;
        }
        b[o] = lo;
    }
}

__global__ void k_count_children(const uint64_t *key, const uint64_t *key2, TreeArrays t, int c0,
                                 int c1, int level, int leaf_size, int *nch) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    const int beg = t.beg[c], end = t.end[c];
    int k = 0;
    if (end - beg > leaf_size && level < FMM_MAXLEVEL) {
        int b[9];
        octant_bounds(key, key2, beg, end, level, b);
#pragma unroll
        for (int o = 0; o < 8; ++o) k += b[o + 1] > b[o];
    }
    nch[c - c0] = k;
    t.nchild[c] = k;
}

__global__ void k_make_children(const uint64_t *key, const uint64_t *key2, TreeArrays t, int c0,
                                int c1, int level, const int *child_off, int next0) {
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    if (t.nchild[c] == 0) {
        t.child0[c] = -1;
        return;
    }
    const int first = next0 + child_off[c - c0];
    t.child0[c] = first;
    int b[9];
    octant_bounds(key, key2, t.beg[c], t.end[c], level, b);
    int k = first;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        if (b[o + 1] > b[o]) {
            t.beg[k] = b[o];
            t.end[k] = b[o + 1];
            t.parent[k] = c;
            t.level[k] = level + 1;
            t.nchild[k] = 0;
            t.child0[k] = -1;
            ++k;
        }
    }
}

// one root per non-empty cluster: particles [rb[r], re[r])
__global__ void k_init_roots(TreeArrays t, int nroots, const int2 *roots) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nroots) return;
    t.beg[r] = roots[r].x;
    t.end[r] = roots[r].y;
    t.parent[r] = -1;
    t.level[r] = 0;
    t.nchild[r] = 0;
    t.child0[r] = -1;
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

hipError_t launch_init_roots(const TreeArrays &t, int nroots, const int2 *roots, hipStream_t s) {
    hipLaunchKernelGGL(k_init_roots, dim3(blocks(nroots, 256)), dim3(256), 0, s, t, nroots, roots);
    return hipGetLastError();
}

hipError_t launch_count_children(const uint64_t *key, const uint64_t *key2, const TreeArrays &t,
                                 int c0, int c1, int level, int leaf_size, int *nch,
                                 hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_count_children, dim3(blocks(c1 - c0, 256)), dim3(256), 0, s, key, key2,
                       t, c0, c1, level, leaf_size, nch);
    return hipGetLastError();
}

hipError_t launch_make_children(const uint64_t *key, const uint64_t *key2, const TreeArrays &t,
                                int c0, int c1, int level, const int *child_off, int next0,
                                hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    hipLaunchKernelGGL(k_make_children, dim3(blocks(c1 - c0, 256)), dim3(256), 0, s, key, key2,
                       t, c0, c1, level, child_off, next0);
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
