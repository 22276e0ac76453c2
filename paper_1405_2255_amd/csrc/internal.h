// Host-side declarations shared by the libfmm translation units: launchers
// for each kernel group and the error-checking macro.  Every launcher takes
// the stream it is ordered on and returns hipSuccess or the launch error.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FMM_KEYLEVELS 21                  // levels resolved by one 63-bit key
#define FMM_MAXLEVEL (2 * FMM_KEYLEVELS)  // levels 22..42 use the second key word
#define FMM_PMAX 20

namespace fmm {

// ---- sort.hip ---------------------------------------------------------
// Exclusive prefix sum of n int32 values (in may equal out).  tmp must hold
// scan_tmp_ints(n) ints.  *total (device, optional) receives the sum.
size_t scan_tmp_ints(int64_t n);
hipError_t exclusive_scan(const int *in, int *out, int64_t n, int *tmp, int *total,
                          hipStream_t s);
// Stable LSD radix sort of (key, value) by key bits [0, bits), 8 per pass.
// Buffers are ping-ponged; on return *keys/*vals point at the sorted data
// (one of the two given buffers).  vals may be null (key-only sort).
size_t sort_tmp_ints(int64_t n);
// (Only key bits [lo_bit, lo_bit + bits) are sorted.)
hipError_t radix_sort(uint64_t **keys, uint64_t **keys_alt, uint32_t **vals,
                      uint32_t **vals_alt, int64_t n, int bits, int *tmp, hipStream_t s,
                      int lo_bit = 0);

// ---- tree.hip ---------------------------------------------------------
struct TreeArrays {
    int *beg, *end, *parent, *child0, *nchild, *level;
    int *leaf_lo, *leaf_hi;     // leaves [leaf_lo, leaf_hi) in Morton leaf order
    double4 *cen;               // (x, y, z, rho): expansion centre z = s, radius
    double4 *com;               // (x, y, z, rho_com): centre of mass, radius about it
    double *mass;
    double *lo, *hi;            // 3 per cell: bounding box of the cell's particles
    unsigned long long *rho2;   // 3 per cell: atomics scratch for squared radii
    double4 *bsph;              // (x, y, z, R): enclosing-sphere candidate and cover radius
    double *smin;               // min over the cell's particles of the sink scale
};

// K clusters: particles [off[k], off[k+1]) (device int64 offsets); bb holds
// 6 max(K, 1 + BBOX_WAVES) keys (the box of cluster k in bb[6k..6k+5]; with
// K = 1 the rest is per-wavefront scratch)
#define BBOX_WAVES 1024
hipError_t launch_bbox(const double *pos, int64_t n, int K, const int64_t *off,
                       unsigned long long *bb, hipStream_t s);
hipError_t launch_keys(const double *pos, int64_t n, int K, const int64_t *off,
                       const unsigned long long *bb, uint64_t *key, uint32_t *idx,
                       hipStream_t s);
hipError_t launch_cluster_keys(const uint32_t *idx, int64_t n, int K, const int64_t *off,
                               uint64_t *ckey, uint32_t *order, hipStream_t s);
hipError_t launch_apply_order(const uint32_t *order, const uint64_t *key, const uint32_t *idx,
                              int64_t n, uint64_t *key_out, uint32_t *idx_out, hipStream_t s);
// Second key word (levels 22..42) of sorted position i, for particles whose
// level-21 cell (a run of equal first keys inside one cluster) holds more
// than leaf_size particles, else 0; runstart[i] = first position of that run;
// *any (device int, zeroed by the caller) set to 1 if some run is overfull.
hipError_t launch_deep_keys(const double *pos, const uint32_t *perm, const uint64_t *key,
                            int64_t n, int K, const int64_t *off, const unsigned long long *bb,
                            int leaf_size, uint64_t *key2, uint64_t *runstart, uint32_t *iota,
                            int *any, hipStream_t s);
// out[i] = in[order[i]]
hipError_t launch_gather_u64(const uint32_t *order, const uint64_t *in, int64_t n, uint64_t *out,
                             hipStream_t s);
// key_out[i] = key[order[i]], key2_out[i] = key2[order[i]], idx_out[i] = idx[order[i]]
hipError_t launch_apply_order2(const uint32_t *order, const uint64_t *key, const uint64_t *key2,
                               const uint32_t *idx, int64_t n, uint64_t *key_out,
                               uint64_t *key2_out, uint32_t *idx_out, hipStream_t s);
hipError_t launch_gather(const double *pos, const double *mass, const uint32_t *perm,
                         int64_t n, double *x, double *y, double *z, double *m,
                         double4 *xyzm, hipStream_t s);
// The octree in one pass over the key-sorted particles (key: levels 1..21,
// key2: levels 22..42, zero outside refined level-21 cells): g, pre, suf hold
// n ints of scratch; cnt (n + 1 ints) receives the number of cells whose first
// particle is each particle (cnt[n] = 0).  After an exclusive scan of cnt,
// launch_tree_emit writes the cells as (level << 32) | first particle in
// particle order; stably sorted by level (key bits 32..37) they are numbered
// level by level and in key order within a level.  launch_tree_levels writes
// ls[L], L = 0..43, the first cell of each level (ncells past the last), and
// launch_tree_cells fills begin, end, level, parent, first child and child
// count of every cell (t sized for ncells).
hipError_t launch_tree(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                       const int64_t *off, int leaf_size, int *g, int *pre, int *suf, int *cnt,
                       hipStream_t s);
hipError_t launch_tree_emit(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                            const int64_t *off, int leaf_size, const int *pre, const int *suf,
                            const int *base, uint64_t *cell, hipStream_t s);
hipError_t launch_tree_levels(const uint64_t *cell, int ncells, int *ls, hipStream_t s);
hipError_t launch_tree_cells(const uint64_t *key, const uint64_t *key2, int64_t n, int K,
                             const int64_t *off, const uint64_t *cell, int ncells, const int *ls,
                             const TreeArrays &t, hipStream_t s);
hipError_t launch_leaf_flags(const TreeArrays &t, int ncells, int *flags, hipStream_t s);
hipError_t launch_leaf_ranges(const TreeArrays &t, int ncells, const int *leafscan,
                              int *leaf_cell, int *leaf_of, int64_t n, hipStream_t s);
hipError_t launch_geometry_level(const TreeArrays &t, int c0, int c1, const double *x,
                                 const double *y, const double *z, const double *m,
                                 hipStream_t s);
// enclosing-sphere candidates of the cells [c0, c1) of one level (children done)
hipError_t launch_enclosing_level(const TreeArrays &t, int c0, int c1, const double *x,
                                  const double *y, const double *z, hipStream_t s);
// squared radii of every cell: candidate = false about the box midpoint and
// the centre of mass (rho2 slots 0, 1), true about the enclosing-sphere
// candidate (slot 2)
hipError_t launch_radii(const TreeArrays &t, int64_t n, const int *leaf_of,
                        const int *leaf_cell, int maxlevel, const double *x, const double *y,
                        const double *z, bool candidate, hipStream_t s);
// cen.w and com.w from slots 0, 1
hipError_t launch_radii_finish(const TreeArrays &t, int ncells, hipStream_t s);
// the candidate replaces the midpoint where its radius (slot 2) is smaller
hipError_t launch_centre_select(const TreeArrays &t, int ncells, hipStream_t s);
hipError_t launch_smin_level(const TreeArrays &t, int c0, int c1, const double *scale,
                             hipStream_t s);

// ---- expansions.hip ---------------------------------------------------
// Internal expansion layout: for each cell, the complex coefficients X_n^m,
// 0 <= m <= n <= p, at complex index n(n+1)/2 + m (Re, Im adjacent); the
// m < 0 half follows from X_n^{-m} = (-1)^m conj(X_n^m).
inline int ncplx(int p) { return (p + 1) * (p + 2) / 2; }
hipError_t launch_p2m(int p, const TreeArrays &t, const int *leaf_cell, int nleaves,
                      const double *x, const double *y, const double *z, const double *m,
                      double *M, hipStream_t s);
hipError_t launch_shift_upsilon(int p, const TreeArrays &t, int c0, int c1, double *U,
                                hipStream_t s);
// Work plans of the translation kernels (M2M, L2L), one block of XF_THREADS
// threads per cell.  Each output coefficient's sum over k is cut into items
// of consecutive k with about equal numbers of terms, the items are dealt to
// the threads (at most XF_IT each, in runs of 64 items of one shape per
// wavefront), and each output adds its items' partial sums in item order.
// Layout (short):
// item i has degree n, order m and rows k0..k1 at XP_N/XP_M/XP_K0/XP_K1 + i;
// thread t's r-th item (or -1) at XP_LANE + r * XF_THREADS + t; the items of
// output e (stored index tri(n, m)) are [XP_OUT + e], [XP_OUT + e + 1]).
// A plan for m2m and one for l2l, XP_SIZE shorts each.
#define XF_THREADS 256
#define XF_ITEMS 512
#define XF_IT 3
#define XP_N 0
#define XP_M XF_ITEMS
#define XP_K0 (2 * XF_ITEMS)
#define XP_K1 (3 * XF_ITEMS)
#define XP_LANE (4 * XF_ITEMS)
#define XP_OUT (XP_LANE + XF_IT * XF_THREADS)
#define XP_SIZE (XP_OUT + (FMM_PMAX + 1) * (FMM_PMAX + 2) / 2 + 1)
void translation_plans(int p, short *m2m, short *l2l);
// Cells [c0, c1) of one level: complete M (internal cells: sum of the
// children's T) and write T = M shifted to the parent's centre (not for
// roots).  Run from the deepest level up to level 0.
hipError_t launch_m2m_level(int p, const TreeArrays &t, int c0, int c1, const double *U,
                            double *M, double *T, const short *plan, hipStream_t s);
hipError_t launch_power(int p, int ncells, const double *M, double *P, hipStream_t s);
// (active: when not null, cells / leaves without listed sinks are skipped)
hipError_t launch_l2l_level(int p, const TreeArrays &t, int c0, int c1, const double *U,
                            double *F, const short *plan, hipStream_t s,
                            const uint8_t *active = nullptr);
// far field at every particle of every leaf: out4[i] = (Psi, ax, ay, az)
hipError_t launch_l2p(int p, const TreeArrays &t, const int *leaf_of, const int *leaf_cell,
                      int64_t n, const double *x, const double *y, const double *z,
                      const double *F, double4 *out4, hipStream_t s,
                      const uint8_t *active = nullptr);
// low-order estimate: monopole M2L into per-cell (Psi, a) at com (gravity)
// or the 1/r^2 sum (f); L2L of the same; evaluation at particles.
hipError_t launch_est_m2l(int want_f, const TreeArrays &t, int nsinks, const int64_t *off,
                          const uint64_t *list, int sh, double4 *Fe, hipStream_t s);
hipError_t launch_est_l2l_level(int want_f, const TreeArrays &t, int c0, int c1, double4 *Fe,
                                hipStream_t s);
hipError_t launch_est_l2p(int want_f, const TreeArrays &t, const int *leaf_of,
                          const int *leaf_cell, int64_t n, const double4 *Fe, double4 *out4,
                          hipStream_t s);

// ---- walk.hip -----------------------------------------------------------
struct WalkParams {
    int mode;          // 0 main (criterion a/f), 1 main (theta), 2 estimate (theta<1 on com)
    int p;
    double eps;
    double theta_crit;
    double p2p_pairs;  // accepted with N_A N_B < p2p_pairs -> direct
    int nroots;        // the walk starts from (r, r) for every root r < nroots
    int sh;            // M2L keys are (sink << sh) | source cell
    int pb;            // direct-sum keys are (sink << pb) | first source particle
    double binom[FMM_PMAX + 1];   // C(p, k)
    int pack;          // nonzero: direct-sum keys carry the range end too,
                       // (sink << 2pb) | (first << pb) | end (needs sh + 2 pb <= 64)
    const uint8_t *active;   // not null: pairs whose sink cell holds no listed
                             // particle are dropped (forces for a subset, Sec. 7.1)
};
struct WalkBuffers {
    const uint2 *in;
    uint2 *out; int64_t cap_out;     // both frontier buffers hold cap_out pairs
    uint64_t *m2l; int64_t cap_m2l;
    uint64_t *p2p; uint32_t *p2p_end; int64_t cap_p2p;   // key, end of the source range
    unsigned long long *counters;   // [0] m2l, [1] direct entries, [2] direct particle
                                    // pairs, [3] overflow, [4 + i] frontier after sweep i,
                                    // [WALK_CUM + 3 i + k] those three totals before sweep i
    uint16_t *code;                 // cap_out: each input pair's decision (count -> write)
};
// sweep i reads the frontier size from counters[4 + i - 1] (1 for sweep 0);
// btmp holds walk_tmp_u64() entries of per-block scratch
size_t walk_tmp_u64();
// first of the per-sweep running totals in WalkBuffers::counters, which hold
// WALK_CUM + 3 (sweeps + 1) entries
constexpr int WALK_CUM = 4 + 2 * FMM_MAXLEVEL + 4;
hipError_t launch_root_pairs(uint2 *f, int nroots, hipStream_t s);
hipError_t launch_walk(const WalkParams &wp, const TreeArrays &t, const double *P,
                       const WalkBuffers &wb, int sweep, unsigned long long *btmp, hipStream_t s);
// offsets of the sorted (sink << sh | source) list per sink: off[c] for c in [0, nsinks]
hipError_t launch_list_offsets(const uint64_t *list, int64_t nlist, int nsinks, int sh,
                               int64_t *off, hipStream_t s);
// merge key-sorted direct-sum entries into maximal particle ranges per sink:
// first call (write = false) flags and scans (flag: n + 1 ints, *total = runs);
// second call writes range[run] = (begin, end) and rkey[run] = (sink << pb) |
// begin.  packed: the keys carry the ends (WalkParams::pack), end is unused.
hipError_t launch_range_merge(const uint64_t *key, const uint32_t *end, int64_t n, int pb,
                              int packed, int *flag, int *tmp, int *total, int2 *range,
                              uint64_t *rkey, bool write, hipStream_t s);

// ---- m2l.hip ------------------------------------------------------------
// chunk table of the sink-sorted M2L list: first call (fill = false) counts the
// chunks per cell into cnt and scans them into coff (ncells + 1 entries,
// *total = chunks); second call (fill = true) writes chunks[] = (sink, e0, e1).
hipError_t launch_chunks(int ncells, const int64_t *off, int chunk, int *cnt, int *coff,
                         int *tmp, int *total, int4 *chunks, bool fill, hipStream_t s);
// orders up to FMM_M2L_FIXED_MAX use register-resident kernels compiled per
// order; higher orders (or generic = true) use the LDS-staged generic kernel
#define FMM_M2L_FIXED_MAX 16
hipError_t launch_m2l(int p, int nchunks, const int4 *chunks, const uint64_t *list, int sh,
                      const TreeArrays &t, const double *M, double *Fpart, hipStream_t s,
                      bool generic = false);
// Mixed precision (orders up to FMM_M2L_FIXED_MAX): scaled FP32 multipoles,
// FP32 chunk sums Fh with their scale sigma, the FP64 terms of degree
// n + k <= FMM_M2L32_JLO per chunk (Flow: tri(min(p, JLO) + 1, 0) complex
// each), reduction to FP64 F.
#define FMM_M2L32_JLO 3
hipError_t launch_m2l32_multipoles(int p, int ncells, const TreeArrays &t, const double *M,
                                   float *M32, hipStream_t s);
hipError_t launch_m2l32(int p, int nchunks, const int4 *chunks, const uint64_t *list, int sh,
                        const TreeArrays &t, const double *M, const float *M32, float *Fpart,
                        double *Flow, double *sig, hipStream_t s);
hipError_t launch_m2l32_reduce(int p, int ncells, const int *coff, const float *Fpart,
                               const double *Flow, const double *sig, double *F, hipStream_t s);
hipError_t launch_m2l_reduce(int p, int ncells, const int *coff, const double *Fpart, double *F,
                             hipStream_t s);

// ---- m2l_rot.hip ---------------------------------------------------------
// Rotation-accelerated M2L (App. A), orders 1..FMM_M2L_ROT_MAX: one wavefront
// per 64 consecutive entries of the sink-sorted list; partial sums per piece
// (a run of one sink's entries inside one window) go to Fpart (2 tri(p+1, 0)
// doubles each) and launch_m2l_reduce adds them per sink.  Pieces: at most
// ceil(nlist / 64) + ncells; launch_rot_pieces counts them per cell into cnt
// and scans into coff (ncells + 1 entries, *total = pieces).
#define FMM_M2L_ROT_MAX 16
// The rotation kernel is switched off until its results on the device are
// established: FMM_M2L_AUTO never selects it (FMM_M2L_ROT_AUTO_MIN above
// FMM_M2L_ROT_MAX) and an explicit request fails with FMM_E_UNSUPPORTED.
#define FMM_M2L_ROT_ENABLED 0
#define FMM_M2L_ROT_AUTO_MIN (FMM_M2L_ROT_MAX + 1)
hipError_t launch_rot_pieces(int ncells, const int64_t *off, int *cnt, int *coff, int *tmp,
                             int *total, hipStream_t s);
hipError_t launch_m2l_rot(int p, int64_t nlist, const uint64_t *list, int sh, const int64_t *off,
                          const int *coff, const TreeArrays &t, const double *M, double *Fpart,
                          hipStream_t s);

// ---- p2p.hip ------------------------------------------------------------
// near field of each sink leaf over its list, added to out4 (sorted order)
// off: ncells + 1 offsets into range (per sink cell).  Planning: per leaf
// the task counts (ntask, mtask, nsrc_tasks: nleaves + 1 ints each) and their
// scans task_off, moff; totals[0] = tasks, totals[1] = partial rows.
#define P2P_TASK 2048
// up[c]: nearest proper ancestor of c with direct-sum ranges (or -1)
hipError_t launch_range_up(int ncells, const int *parent, const int64_t *off, int *up,
                           hipStream_t s);
// chain: P2P_CHAIN ints per leaf, [0] = the number of cells on the leaf's
// chain of ancestors that hold direct-sum ranges (the leaf first), then their
// indices; written by the plan, read by the direct-sum kernel
#define P2P_CHAIN (FMM_MAXLEVEL + 2)
hipError_t launch_p2p_plan(int nleaves, const int *leaf_cell, const int64_t *off,
                           const int2 *range, const int *up, const TreeArrays &t,
                           const uint8_t *active, int *ntask, int *mtask, int *nsrc_tasks,
                           int *task_off, int *moff, int *chain, int *tmp, int *totals,
                           hipStream_t s);
hipError_t launch_p2p_tasks(int nleaves, const int *task_off, int2 *tasks, hipStream_t s);
// mixed != 0: FP32 pair arithmetic (separations in FP64, sums flushed to FP64)
hipError_t launch_p2p(int want_f, int with_pot, int mixed, int ntasks, const int2 *tasks,
                      const int *leaf_cell, const int *nsrc_tasks, const int *moff,
                      const int64_t *off, const int2 *range, const int *chain,
                      const TreeArrays &t, const double4 *xyzm, double4 *out4, double4 *partial,
                      hipStream_t s);
hipError_t launch_p2p_reduce(int64_t n, const int *leaf_of, const int *leaf_cell,
                             const int *nsrc_tasks, const int *moff, const TreeArrays &t,
                             const double4 *partial, double4 *out4, hipStream_t s);
hipError_t launch_output(int64_t n, const uint32_t *perm, const double4 *out4, double G,
                         double *pot, double *acc, int *nonfinite, hipStream_t s);
// forces for a listed subset of sinks (Sec. 7.1): flag_in (n ints, zeroed by the
// caller) marks the listed input indices, *bad = 1 if one is outside [0, n);
// then per sorted position f (n + 1), inv (input -> sorted, n), the exclusive
// scan pre (n + 1, scratch tmp/total) and active[c] = 1 for cells holding a
// listed particle; the output kernel writes the listed particles in list order
hipError_t launch_mark_listed(int64_t n, int64_t nact, const int64_t *act, int *flag_in, int *bad,
                             hipStream_t s);
hipError_t launch_cell_active(int64_t n, const uint32_t *perm, const int *flag_in, int *f,
                              int *inv, int *pre, int *tmp, int *total, int ncells, const int *beg,
                              const int *end, uint8_t *active, hipStream_t s);
// individual accuracy parameters (Sec. 7): *bad = 1 unless every eps_b is
// > 0 and finite; *minbits (set to all ones by the caller) = bit pattern of the
// smallest; launch_scale_eps multiplies the key-ordered sink scale by eps_b
hipError_t launch_eps_min(int64_t n, const double *eps_b, unsigned long long *minbits, int *bad,
                         hipStream_t s);
hipError_t launch_scale_eps(int64_t n, const uint32_t *perm, const double *eps_b, double *scale,
                           hipStream_t s);
hipError_t launch_output_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                const double4 *out4, double G, double *pot, double *acc,
                                int *nonfinite, hipStream_t s);
hipError_t launch_scale(int want_f, int64_t n, const double4 *est4, double *scale,
                        hipStream_t s);
// Exact sums for listed sinks (an index outside [0, n) sets *bad and its
// outputs are left alone).  The sources are cut into nchunk chunks of
// ceil(n / nchunk), one per grid row; with nchunk > 1 the partial sums go to
// part (nchunk * nsinks double4) and are added per sink in chunk order.
// direct_sinks_chunks gives the library's choice: about DIRECT_SINKS_BLOCKS
// blocks of 256 sinks, chunks of at least 2048 sources.  When nchunk > 1,
// nchunk * nsinks < 2 * DIRECT_SINKS_BLOCKS * 256.
#define DIRECT_SINKS_BLOCKS 1024
int direct_sinks_chunks(int64_t n, int64_t nsinks);
hipError_t launch_direct_sinks(int64_t n, const double *pos, const double *mass, double G,
                               int64_t nsinks, const int64_t *sinks, int nchunk, double *pot,
                               double *acc, double4 *part, int *bad, hipStream_t s);
// p[0 .. count) = v (a kernel, so that no memset node enters a captured graph)
hipError_t launch_fill_int(int *p, int64_t count, int v, hipStream_t s);
hipError_t launch_direct(int64_t n, const double *pos, const double *mass, double G,
                         double *pot, double *acc, hipStream_t s);

}  // namespace fmm
