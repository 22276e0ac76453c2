// Direct sums: the near field (P2P, eq. 1 restricted to the walk's direct
// pairs), the all-pairs GPU direct summation used as a comparison baseline,
// and the final un-permute / scale / finiteness check.
//
// P2P: the sources of a sink leaf are the merged particle ranges listed for
// the leaf and for each of its ancestors (a direct sum accepted for a cell
// applies to all particles below it).  A leaf's work is cut into tasks of at
// most 64 sinks x P2P_TASK sources - a sparse leaf far out in an untruncated
// halo can be summed against every particle, and as one wavefront's serial
// loop it would set the kernel time; short tasks also even out the load of
// the compute units at the end of a launch.  One wavefront per task: every lane holds
// two sinks, lanes are (sink group, phase) pairs, the phases stride through
// each range and are summed through LDS at the end, so small leaves still fill
// the wavefront and every source load serves two pairs.  A leaf with one task
// adds into the output directly; otherwise each task writes a row of partial
// sums that a second kernel adds in task order (deterministic).
// Source particles are read as (x, y, z, m) double4 from the key-sorted copy.
#include <algorithm>

#include "internal.h"
#include "dev.h"
#include "range_loads.h"

namespace fmm {

namespace {

// sinks per lane of the P2P kernel (two halves the source loads per pair;
// more costs occupancy)
constexpr int P2P_R = 2;

// up[c] = the nearest proper ancestor of c that has direct-sum ranges (or -1),
// so that a leaf visits only the cells of its chain that hold work instead of
// every ancestor (each step is a dependent load).
__global__ void k_range_up(int ncells, const int *parent, const int64_t *off, int *up) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int a = parent[c];
    while (a >= 0 && off[a + 1] == off[a]) a = parent[a];
    up[c] = a;
}

__device__ __forceinline__ int first_with_ranges(int c, const int *up, const int64_t *off) {
    return off[c + 1] > off[c] ? c : up[c];
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Work of one sink leaf: the number of source particles in its direct-sum
// ranges and those of its ancestors (one concatenated list); every lane of
// the wavefront ends with it.  Lanes take the range entries in turn.
__device__ __forceinline__ int64_t leaf_sources(int c, const int *up, const int64_t *off,
                                                const int2 *range) {
    int64_t s = 0;
    for (int anc = first_with_ranges(c, up, off); anc >= 0; anc = up[anc])
        for (int64_t r = off[anc] + lane_id(); r < off[anc + 1]; r += FMM_WAVE)
            s += range[r].y - range[r].x;
#pragma unroll
    for (int o = FMM_WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, FMM_WAVE);
    return s;
}

// per leaf (one wavefront each): tasks = sink chunks of 64 x source chunks of
// P2P_TASK sources; mtask = tasks that need a partial-sum row (leaves with
// more than one task) (active: when not null, leaves whose cell holds no
// listed sink get no task); entry nleaves is zeroed for the scans.  Also the
// leaf's chain of ancestors with ranges, so that the direct-sum tasks load it
// at once instead of following it one dependent load at a time.
__global__ void k_p2p_count(int nleaves, const int *leaf_cell, const int64_t *off,
                            const int2 *range, const int *up, TreeArrays t,
                            const uint8_t *active, int *ntask, int *mtask, int *nsrc_tasks,
                            int *chain) {
    const int leaf = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FMM_WAVE);
    if (leaf > nleaves) return;
    const bool head = lane_id() == 0;
    if (leaf == nleaves) {
        if (head) {
            ntask[leaf] = 0;
            mtask[leaf] = 0;
        }
        return;
    }
    const int c = leaf_cell[leaf];
    int *ch = chain + (size_t)leaf * P2P_CHAIN;
    if (active && !active[c]) {
        if (head) {
            nsrc_tasks[leaf] = 1;
            ntask[leaf] = 0;
            mtask[leaf] = 0;
            ch[0] = 0;
        }
        return;
    }
    if (head) {
        int k = 0;
        for (int anc = first_with_ranges(c, up, off); anc >= 0; anc = up[anc]) ch[1 + k++] = anc;
        ch[0] = k;
    }
    const int64_t S = leaf_sources(c, up, off, range);
    if (!head) return;
    const int nsc = (t.end[c] - t.beg[c] + FMM_WAVE - 1) / FMM_WAVE;
    const int nts = (int)max((int64_t)1, (S + P2P_TASK - 1) / P2P_TASK);
    nsrc_tasks[leaf] = nts;
    ntask[leaf] = nsc * nts;
    mtask[leaf] = nsc * nts > 1 ? nsc * nts : 0;
}

// the task list: (leaf, index within the leaf), one wavefront per leaf
__global__ void k_p2p_tasks(int nleaves, const int *task_off, int2 *tasks) {
    const int leaf = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FMM_WAVE);
    if (leaf >= nleaves) return;
    const int k0 = task_off[leaf], k1 = task_off[leaf + 1];
    for (int k = k0 + lane_id(); k < k1; k += FMM_WAVE) tasks[k] = make_int2(leaf, k - k0);
}

// Potentials and accelerations are summed with 2/|r| in place of 1/|r|
// (rsqrt2_nr), that is times 2 and times 8; the sums of a sink are scaled back
// once, before they leave the kernel (exact: powers of two).
constexpr double P2P_POT_BACK = 0.5, P2P_ACC_BACK = 0.125;

template <int WANT_F, int WITH_POT>
__device__ __forceinline__ void pair(const double4 s, const double4 xb, bool skip, double &pot,
                                     double &ax, double &ay, double &az) {
    const double dx = s.x - xb.x, dy = s.y - xb.y, dz = s.z - xb.z;
    const double r2 = skip ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
    const double mu = skip ? 0.0 : s.w;
    if (WANT_F) {
        pot += mu / r2;
    } else {
        const double ri = rsqrt2_nr(r2);        // 2/|r|
        const double q = mu * ri;
        const double q3 = q * ri * ri;
        if (WITH_POT) pot += q;
        ax = fma(q3, dx, ax);
        ay = fma(q3, dy, ay);
        az = fma(q3, dz, az);
    }
}

// Mixed precision: the separation is formed in FP64 and rounded once; the
// squared distance, reciprocal square root, products and the running sums
// are FP32 (every pair's contribution carries a relative error of a few
// FP32 units).  Only ranges without the sinks themselves come here: no
// self-pair test.
template <int WANT_F, int WITH_POT>
__device__ __forceinline__ void pair32(const double4 s, const double4 xb, float &pot, float &ax,
                                       float &ay, float &az) {
    const float dx = (float)(s.x - xb.x), dy = (float)(s.y - xb.y), dz = (float)(s.z - xb.z);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float mu = (float)s.w;
    if (WANT_F) {
        pot += mu * __builtin_amdgcn_rcpf(r2);
    } else {
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float q = mu * ri;
        const float q3 = q * ri * ri;
        if (WITH_POT) pot += q;
        ax = fmaf(q3, dx, ax);
        ay = fmaf(q3, dy, ay);
        az = fmaf(q3, dz, az);
    }
}

// FP32 partial sums run over at most this many sources per lane before they
// are added into the FP64 sums
constexpr int P2P_CHUNK32 = 32;

// One lane's share of a source range that overlaps its R sinks' own leaf:
// sources p[0], p[stride], ... below pe (the sinks themselves skipped by
// address), the next source loaded before the current one is summed.  Always
// FP64.
template <int R, int WANT_F, int WITH_POT>
__device__ __forceinline__ void sum_own(const double4 *p, const double4 *pe, int stride,
                                        const double4 (&xb)[R], const double4 *const (&self)[R],
                                        double4 (&f)[R]) {
    if (p >= pe) return;
    double4 a = p[0];
    for (;;) {
        const double4 *q = p + stride;
        const bool more = q < pe;
        const double4 b = (more ? q : p)[0];
#pragma unroll
        for (int k = 0; k < R; ++k)
            pair<WANT_F, WITH_POT>(a, xb[k], p == self[k], f[k].x, f[k].y, f[k].z, f[k].w);
        if (!more) break;
        p = q;
        a = b;
    }
}

static_assert((int64_t)P2P_TASK * sizeof(double4) < (int64_t(1) << 32),
              "byte offsets within a task's source range fit 32 bits");

// One lane's share of a source range that holds none of its sinks: sources
// base[i], base[i + stride], ... below base[n] (n <= P2P_TASK).
template <int R, int WANT_F, int WITH_POT>
__device__ __forceinline__ void sum_far(const double4 *base, uint32_t i, uint32_t n,
                                        uint32_t stride, const double4 (&xb)[R],
                                        double4 (&f)[R]) {
    gchar *b = uniform_base(base);
    const uint32_t oe = n * 32u, st = stride * 32u;
    for (uint32_t o = i * 32u; o < oe; o += st) {
        const double4 a = load_source(b + o);
#pragma unroll
        for (int k = 0; k < R; ++k)
            pair<WANT_F, WITH_POT>(a, xb[k], false, f[k].x, f[k].y, f[k].z, f[k].w);
    }
}

// The same in mixed precision: FP32 partial sums over at most P2P_CHUNK32
// sources per lane, then added into the FP64 sums.
template <int R, int WANT_F, int WITH_POT>
__device__ __forceinline__ void sum_far32(const double4 *base, uint32_t i, uint32_t n,
                                          uint32_t stride, const double4 (&xb)[R],
                                          double4 (&f)[R]) {
    gchar *b = uniform_base(base);
    const uint32_t oe = n * 32u, st = stride * 32u;
    uint32_t o = i * 32u;
    while (o < oe) {
        float4 g[R];
#pragma unroll
        for (int k = 0; k < R; ++k) g[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int it = 0; it < P2P_CHUNK32 && o < oe; ++it, o += st) {
            const double4 a = load_source(b + o);
#pragma unroll
            for (int k = 0; k < R; ++k)
                pair32<WANT_F, WITH_POT>(a, xb[k], g[k].x, g[k].y, g[k].z, g[k].w);
        }
        constexpr double sp = WANT_F ? 1.0 : 1.0 / P2P_POT_BACK;
        constexpr double sa = WANT_F ? 1.0 : 1.0 / P2P_ACC_BACK;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            f[k].x = fma((double)g[k].x, sp, f[k].x);
            f[k].y = fma((double)g[k].y, sa, f[k].y);
            f[k].z = fma((double)g[k].z, sa, f[k].z);
            f[k].w = fma((double)g[k].w, sa, f[k].w);
        }
    }
}

// R sinks per lane: ng = ceil(nb / R) lane groups, group g holds sink slots
// g, g + ng, g + 2 ng, ... (a slot past the leaf repeats slot g and is
// discarded); lanes [0, ng * S) are (group, phase) with S = floor(64 / ng).
template <int R, int WANT_F, int WITH_POT, int MIXED>
__global__ void __launch_bounds__(256)
k_p2p(int ntasks, const int2 *tasks, const int *leaf_cell, const int *nsrc_tasks,
      const int *moff, const int64_t *off, const int2 *range, const int *chain, TreeArrays t,
      const double4 *xyzm, double4 *out4, double4 *partial) {
    __shared__ double4 red[4][R * FMM_WAVE];
    // blocks in task order: the hardware deals them to the XCDs in turn, which
    // spreads the uneven task lengths evenly (a contiguous eighth of the tasks
    // per XCD left the shorter launches unbalanced)
    const int task = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (task >= ntasks) return;
    const int lane = lane_id(), w = threadIdx.x / FMM_WAVE;
    const int2 tk = tasks[task];
    const int leaf = tk.x;
    const int c = leaf_cell[leaf];
    const int nts = nsrc_tasks[leaf];
    const int sc = tk.y / nts, ts = tk.y % nts;
    const int beg = t.beg[c], end = t.end[c];
    const int sb = beg + sc * FMM_WAVE;
    const int nb = min(end - sb, FMM_WAVE);
    const int ng = (nb + R - 1) / R;
    const int S = FMM_WAVE / ng;
    const int g = lane % ng, phase = lane / ng;
    const bool active = phase < S;
    double4 xb[R], f[R];
    const double4 *self[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int slot = g + k * ng < nb ? g + k * ng : g;
        self[k] = xyzm + sb + slot;
        xb[k] = *self[k];
        f[k] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
    // the chain of ancestors with ranges and their list offsets, one per lane
    const int *ch = chain + (size_t)leaf * P2P_CHAIN;
    const int nchain = ch[0];
    const int myanc = lane < nchain ? ch[1 + lane] : 0;
    const int64_t mr0 = lane < nchain ? off[myanc] : 0, mr1 = lane < nchain ? off[myanc + 1] : 0;
    // sources [ts * P2P_TASK, (ts + 1) * P2P_TASK) of the leaf's list; the range
    // descriptors are read 64 at a time (one per lane) and broadcast in turn
    int64_t skip = (int64_t)ts * P2P_TASK, left = P2P_TASK;
    for (int ci = 0; ci < nchain && left > 0; ++ci) {
        const int64_t r0 = readlane64(mr0, ci), r1 = readlane64(mr1, ci);
        for (int64_t rb = r0; rb < r1 && left > 0; rb += FMM_WAVE) {
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
            // the sinks' own leaf holds their nearest neighbours, the largest
            // terms: summed in FP64 also in mixed precision
            const uint32_t nr = (uint32_t)(rg.y - rg.x);
            if (own)
                sum_own<R, WANT_F, WITH_POT>(xyzm + rg.x + phase, xyzm + rg.y, S, xb, self, f);
            else if (MIXED) sum_far32<R, WANT_F, WITH_POT>(xyzm + rg.x, phase, nr, S, xb, f);
            else sum_far<R, WANT_F, WITH_POT>(xyzm + rg.x, phase, nr, S, xb, f);
          }
        }
    }
    // sum the phases of each sink through LDS: red[w][slot + phase * R * ng];
    // active lanes cover every index below R * ng * S <= R * 64 exactly once
    if (active) {
#pragma unroll
        for (int k = 0; k < R; ++k) red[w][g + k * ng + phase * R * ng] = f[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane >= nb) return;
    double4 v = red[w][lane];
    for (int ph = 1; ph < S; ++ph) {
        const double4 q = red[w][lane + ph * R * ng];
        v.x += q.x; v.y += q.y; v.z += q.z; v.w += q.w;
    }
    if (!WANT_F) {
        v.x *= P2P_POT_BACK;
        v.y *= P2P_ACC_BACK;
        v.z *= P2P_ACC_BACK;
        v.w *= P2P_ACC_BACK;
    }
    const int bi = sb + lane;
    if (moff[leaf + 1] == moff[leaf]) {          // the leaf's only task
        double4 o = out4[bi];
        o.x += v.x; o.y += v.y; o.z += v.z; o.w += v.w;
        out4[bi] = o;
    } else {
        partial[((int64_t)moff[leaf] + tk.y) * FMM_WAVE + lane] = v;
    }
}

// add the partial sums of multi-task leaves, in task order
__global__ void k_p2p_reduce(int64_t n, const int *leaf_of, const int *leaf_cell,
                             const int *nsrc_tasks, const int *moff, TreeArrays t,
                             const double4 *partial, double4 *out4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int leaf = leaf_of[i];
    if (moff[leaf + 1] == moff[leaf]) return;
    const int c = leaf_cell[leaf];
    const int k = (int)(i - t.beg[c]);
    const int sc = k / FMM_WAVE, slot = k % FMM_WAVE, nts = nsrc_tasks[leaf];
    double4 v = out4[i];
    const double4 *row = partial + ((int64_t)moff[leaf] + sc * nts) * FMM_WAVE + slot;
    // eight rows' loads in flight at a time, added in task order
    for (int t0 = 0; t0 < nts; t0 += 8) {
        double4 q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = row[(int64_t)min(t0 + j, nts - 1) * FMM_WAVE];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (t0 + j < nts) {
                v.x += q[j].x; v.y += q[j].y; v.z += q[j].z; v.w += q[j].w;
            }
        }
    }
    out4[i] = v;
}

// all-pairs direct sum: one sink per thread, sources in order, read as
// wavefront-uniform values
__global__ void __launch_bounds__(256)
k_direct(int64_t n, const double *pos, const double *mass, double G, double *pot, double *acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const int64_t ii = active ? i : 0;
    const double xb = pos[3 * ii], yb = pos[3 * ii + 1], zb = pos[3 * ii + 2];
    double p = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double dx = pos[3 * j] - xb, dy = pos[3 * j + 1] - yb, dz = pos[3 * j + 2] - zb;
        const bool self = j == ii;
        const double r2 = self ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
        const double mu = self ? 0.0 : mass[j];
        const double ri = rsqrt_nr(r2);
        const double q = mu * ri, q3 = q * ri * ri;
        p += q;
        ax = fma(q3, dx, ax);
        ay = fma(q3, dy, ay);
        az = fma(q3, dz, az);
    }
    if (!active) return;
    pot[i] = -G * p;
    acc[3 * i] = G * ax;
    acc[3 * i + 1] = G * ay;
    acc[3 * i + 2] = G * az;
}

// The same sum for listed sinks, with the sources split over the grid's y
// dimension: block (x, k) takes sinks [256 x, 256 x + 256) against sources
// [k chunk, min(n, (k + 1) chunk)), one sink per thread, the sources read as
// wavefront-uniform values.  A few thousand sinks thus still fill the chip.
// With one chunk the block writes the results; otherwise it writes row k of
// part (nsinks double4 per row: Psi, a without G) and k_direct_sinks_reduce
// adds the rows of each sink in chunk order, so the result does not depend on
// the order in which blocks run.  An index outside [0, n) sets *bad (by the
// blocks of chunk 0) and its outputs are not written.
__global__ void __launch_bounds__(256)
k_direct_sinks(int64_t n, const double *pos, const double *mass, double G, int64_t nsinks,
               const int64_t *sinks, int64_t chunk, double *pot, double *acc, double4 *part,
               int *bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    int64_t ii = t < nsinks ? sinks[t] : 0;
    const bool valid = t < nsinks && ii >= 0 && ii < n;
    if (k == 0 && t < nsinks && !valid) atomicOr(bad, 1);
    if (!valid) ii = 0;
    const double xb = pos[3 * ii], yb = pos[3 * ii + 1], zb = pos[3 * ii + 2];
    const int64_t j0 = (int64_t)k * chunk, j1 = min(n, j0 + chunk);
    double p = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double dx = pos[3 * j] - xb, dy = pos[3 * j + 1] - yb, dz = pos[3 * j + 2] - zb;
        const bool self = j == ii;
        const double r2 = self ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
        const double mu = self ? 0.0 : mass[j];
        const double ri = rsqrt_nr(r2);
        const double q = mu * ri, q3 = q * ri * ri;
        p += q;
        ax = fma(q3, dx, ax);
        ay = fma(q3, dy, ay);
        az = fma(q3, dz, az);
    }
    if (!valid) return;
    if (part) {
        part[(int64_t)k * nsinks + t] = make_double4(p, ax, ay, az);
        return;
    }
    pot[t] = -G * p;
    acc[3 * t] = G * ax;
    acc[3 * t + 1] = G * ay;
    acc[3 * t + 2] = G * az;
}

__global__ void k_direct_sinks_reduce(int64_t n, double G, int64_t nsinks, const int64_t *sinks,
                                      int nchunk, const double4 *part, double *pot, double *acc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsinks) return;
    const int64_t ii = sinks[t];
    if (ii < 0 || ii >= n) return;
    double4 v = part[t];
    for (int k = 1; k < nchunk; ++k) {
        const double4 q = part[(int64_t)k * nsinks + t];
        v.x += q.x; v.y += q.y; v.z += q.z; v.w += q.w;
    }
    pot[t] = -G * v.x;
    acc[3 * t] = G * v.y;
    acc[3 * t + 1] = G * v.z;
    acc[3 * t + 2] = G * v.w;
}

__global__ void k_fill_int(int *p, int64_t count, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_output(int64_t n, const uint32_t *perm, const double4 *out4, double G,
                         double *pot, double *acc, int *nonfinite) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 v = out4[i];
    const int64_t j = perm[i];
    const double p = -G * v.x, a = G * v.y, b = G * v.z, c = G * v.w;
    pot[j] = p;
    acc[3 * j] = a;
    acc[3 * j + 1] = b;
    acc[3 * j + 2] = c;
    if (!(isfinite(p) && isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(nonfinite, 1);
}

// ---- forces for a listed subset of sinks (Sec. 7.1) ------------------------
// flag_in[act[j]] = 1 (input order, zeroed by the caller); *bad = 1 for an
// index outside [0, n)
__global__ void k_mark_listed(int64_t n, int64_t nact, const int64_t *act, int *flag_in,
                              int *bad) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nact) return;
    const int64_t i = act[j];
    if (i < 0 || i >= n) atomicOr(bad, 1);
    else flag_in[i] = 1;
}

// key order: f[i] = flag of the particle at sorted position i, inv[input] = i
__global__ void k_sorted_flags(int64_t n, const uint32_t *perm, const int *flag_in, int *f,
                               int *inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        f[n] = 0;
        return;
    }
    const uint32_t j = perm[i];
    f[i] = flag_in[j];
    inv[j] = (int)i;
}

// a cell is active if it holds a listed particle: pre is the exclusive scan of f
__global__ void k_cell_active(int ncells, const int *beg, const int *end, const int *pre,
                              uint8_t *active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    active[c] = pre[end[c]] > pre[beg[c]] ? 1 : 0;
}

// results of the listed particles, in list order (indices out of range are skipped)
__global__ void k_output_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                const double4 *out4, double G, double *pot, double *acc,
                                int *nonfinite) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nact) return;
    const int64_t idx = act[j];
    if (idx < 0 || idx >= n) return;
    const double4 v = out4[inv[idx]];
    const double p = -G * v.x, a = G * v.y, b = G * v.z, c = G * v.w;
    pot[j] = p;
    acc[3 * j] = a;
    acc[3 * j + 1] = b;
    acc[3 * j + 2] = c;
    if (!(isfinite(p) && isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(nonfinite, 1);
}

// ---- individual accuracy parameters (Sec. 7) ------------------------------
// every eps_b must be > 0 and finite (*bad = 1 otherwise); the smallest one as
// the bit pattern of a positive double (which orders like the value)
__global__ void __launch_bounds__(256)
k_eps_min(int64_t n, const double *eps_b, unsigned long long *minbits, int *bad) {
    __shared__ unsigned long long red[256 / FMM_WAVE];
    unsigned long long mine = ~0ull;
    int fail = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = eps_b[i];
        if (!(v > 0.0 && isfinite(v))) fail = 1;
        else mine = min(mine, (unsigned long long)__double_as_longlong(v));
    }
    if (__any(fail) && lane_id() == 0) atomicOr(bad, 1);
#pragma unroll
    for (int off = FMM_WAVE / 2; off > 0; off >>= 1) mine = min(mine, __shfl_xor(mine, off));
    if (lane_id() == 0) red[threadIdx.x / FMM_WAVE] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = red[0];
        for (int w = 1; w < 256 / FMM_WAVE; ++w) b = min(b, red[w]);
        atomicMin(minbits, b);
    }
}

// scale[i] *= eps_b of the particle at sorted position i: the cell minimum
// then is min_B{eps_b a_b} (or f_b) and the criterion compares with it alone
__global__ void k_scale_eps(int64_t n, const uint32_t *perm, const double *eps_b, double *scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    scale[i] *= eps_b[perm[i]];
}

// sink scale of the acceptance test from the estimate: |a| (criterion a) or f
__global__ void k_scale(int want_f, int64_t n, const double4 *est4, double *scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 v = est4[i];
    scale[i] = want_f ? v.x : sqrt(fma(v.y, v.y, fma(v.z, v.z, v.w * v.w)));
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_range_up(int ncells, const int *parent, const int64_t *off, int *up,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_range_up, dim3(blocks(ncells, 256)), dim3(256), 0, s, ncells, parent,
                       off, up);
    return hipGetLastError();
}

hipError_t launch_p2p_plan(int nleaves, const int *leaf_cell, const int64_t *off,
                           const int2 *range, const int *up, const TreeArrays &t,
                           const uint8_t *active, int *ntask, int *mtask, int *nsrc_tasks,
                           int *task_off, int *moff, int *chain, int *tmp, int *totals,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_p2p_count, dim3(blocks((int64_t)(nleaves + 1) * FMM_WAVE, 256)),
                       dim3(256), 0, s, nleaves, leaf_cell, off, range, up, t, active, ntask,
                       mtask, nsrc_tasks, chain);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan(ntask, task_off, nleaves + 1, tmp, totals, s);
    if (e != hipSuccess) return e;
    return exclusive_scan(mtask, moff, nleaves + 1, tmp, totals + 1, s);
}

hipError_t launch_p2p_tasks(int nleaves, const int *task_off, int2 *tasks, hipStream_t s) {
    hipLaunchKernelGGL(k_p2p_tasks, dim3(blocks((int64_t)nleaves * FMM_WAVE, 256)), dim3(256), 0,
                       s, nleaves, task_off, tasks);
    return hipGetLastError();
}

hipError_t launch_p2p(int want_f, int with_pot, int mixed, int ntasks, const int2 *tasks,
                      const int *leaf_cell, const int *nsrc_tasks, const int *moff,
                      const int64_t *off, const int2 *range, const int *chain,
                      const TreeArrays &t, const double4 *xyzm, double4 *out4, double4 *partial,
                      hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    const dim3 g(blocks(ntasks, 4)), b(256);
#define FMM_P2P_LAUNCH(F, P, X)                                                                  \
    hipLaunchKernelGGL((k_p2p<P2P_R, F, P, X>), g, b, 0, s, ntasks, tasks, leaf_cell, nsrc_tasks, \
                       moff, off, range, chain, t, xyzm, out4, partial)
    if (mixed) {
        if (want_f) FMM_P2P_LAUNCH(1, 0, 1);
        else if (with_pot) FMM_P2P_LAUNCH(0, 1, 1);
        else FMM_P2P_LAUNCH(0, 0, 1);
    } else {
        if (want_f) FMM_P2P_LAUNCH(1, 0, 0);
        else if (with_pot) FMM_P2P_LAUNCH(0, 1, 0);
        else FMM_P2P_LAUNCH(0, 0, 0);
    }
#undef FMM_P2P_LAUNCH
    return hipGetLastError();
}

hipError_t launch_p2p_reduce(int64_t n, const int *leaf_of, const int *leaf_cell,
                             const int *nsrc_tasks, const int *moff, const TreeArrays &t,
                             const double4 *partial, double4 *out4, hipStream_t s) {
    hipLaunchKernelGGL(k_p2p_reduce, dim3(blocks(n, 256)), dim3(256), 0, s, n, leaf_of, leaf_cell,
                       nsrc_tasks, moff, t, partial, out4);
    return hipGetLastError();
}

hipError_t launch_output(int64_t n, const uint32_t *perm, const double4 *out4, double G,
                         double *pot, double *acc, int *nonfinite, hipStream_t s) {
    hipLaunchKernelGGL(k_output, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, out4, G, pot, acc,
                       nonfinite);
    return hipGetLastError();
}

hipError_t launch_mark_listed(int64_t n, int64_t nact, const int64_t *act, int *flag_in, int *bad,
                             hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_listed, dim3(blocks(nact, 256)), dim3(256), 0, s, n, nact, act,
                       flag_in, bad);
    return hipGetLastError();
}

hipError_t launch_cell_active(int64_t n, const uint32_t *perm, const int *flag_in, int *f,
                              int *inv, int *pre, int *tmp, int *total, int ncells, const int *beg,
                              const int *end, uint8_t *active, hipStream_t s) {
    hipLaunchKernelGGL(k_sorted_flags, dim3(blocks(n + 1, 256)), dim3(256), 0, s, n, perm,
                       flag_in, f, inv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan(f, pre, n + 1, tmp, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_active, dim3(blocks(ncells, 256)), dim3(256), 0, s, ncells, beg, end,
                       pre, active);
    return hipGetLastError();
}

hipError_t launch_output_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                const double4 *out4, double G, double *pot, double *acc,
                                int *nonfinite, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_output_listed, dim3(blocks(nact, 256)), dim3(256), 0, s, n, nact, act, inv,
                       out4, G, pot, acc, nonfinite);
    return hipGetLastError();
}

hipError_t launch_eps_min(int64_t n, const double *eps_b, unsigned long long *minbits, int *bad,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<int64_t>(256, (n + 255) / 256);
    hipLaunchKernelGGL(k_eps_min, dim3(nb), dim3(256), 0, s, n, eps_b, minbits, bad);
    return hipGetLastError();
}

hipError_t launch_scale_eps(int64_t n, const uint32_t *perm, const double *eps_b, double *scale,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_scale_eps, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, eps_b, scale);
    return hipGetLastError();
}

hipError_t launch_scale(int want_f, int64_t n, const double4 *est4, double *scale,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(blocks(n, 256)), dim3(256), 0, s, want_f, n, est4, scale);
    return hipGetLastError();
}

int direct_sinks_chunks(int64_t n, int64_t nsinks) {
    // about DIRECT_SINKS_BLOCKS blocks, at least 2048 sources per chunk
    const int64_t sb = (nsinks + 255) / 256;
    const int64_t want = (DIRECT_SINKS_BLOCKS + sb - 1) / sb;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, n / 2048));
}

hipError_t launch_direct_sinks(int64_t n, const double *pos, const double *mass, double G,
                               int64_t nsinks, const int64_t *sinks, int nchunk, double *pot,
                               double *acc, double4 *part, int *bad, hipStream_t s) {
    if (nsinks <= 0) return hipSuccess;
    if (nchunk < 1 || (nchunk > 1 && !part)) return hipErrorInvalidValue;
    const int64_t chunk = (n + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_direct_sinks, dim3(blocks(nsinks, 256), (unsigned)nchunk), dim3(256), 0,
                       s, n, pos, mass, G, nsinks, sinks, chunk, pot, acc,
                       nchunk > 1 ? part : nullptr, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nchunk == 1) return e;
    hipLaunchKernelGGL(k_direct_sinks_reduce, dim3(blocks(nsinks, 256)), dim3(256), 0, s, n, G,
                       nsinks, sinks, nchunk, (const double4 *)part, pot, acc);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int64_t count, int v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3(blocks(count, 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_direct(int64_t n, const double *pos, const double *mass, double G,
                         double *pot, double *acc, hipStream_t s) {
    hipLaunchKernelGGL(k_direct, dim3(blocks(n, 256)), dim3(256), 0, s, n, pos, mass, G, pot, acc);
    return hipGetLastError();
}

}  // namespace fmm
