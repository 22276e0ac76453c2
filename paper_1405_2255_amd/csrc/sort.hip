// Device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Scan: reduce-then-scan over tiles of 2048 ints (256 threads x 8), the tile
// sums scanned recursively.  Radix sort: 8-bit digits; per pass a tile
// histogram (digit-major layout), an exclusive scan of all histograms, and a
// stable scatter in which each key's rank inside its tile comes from 64-wide
// ballot matching of equal digits.
#include "internal.h"
#include "dev.h"

namespace fmm {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ int block_excl_scan(int v, int *total) {
    // 256 threads = 4 waves
    __shared__ int wsum[SCAN_THREADS / FMM_WAVE];
    const int lane = lane_id(), w = threadIdx.x / FMM_WAVE;
    const int inc = wave_incl_scan(v);
    if (lane == FMM_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / FMM_WAVE; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    if (total) *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const int *in, int64_t n, int *sums) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (j < n) s += in[j];
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_tile_scan(const int *in, int *out, int64_t n, const int *offs, int *total) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + i;
        v[i] = j < n ? in[j] : 0;
        s += v[i];
    }
    int tot;
    int run = block_excl_scan(s, &tot) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t j = base + i;
        if (j < n) out[j] = run;
        run += v[i];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) *total = run;
}

// One block scans an array of up to SCAN1_MAX ints in a single launch (the
// radix sort's digit counts, for instance), instead of the three launches of
// the tiled scan: each thread sums a contiguous chunk, the block scans the
// chunk sums, and each thread writes its chunk's prefixes.  in and out may be
// the same array (each thread reads its chunk before it writes it).
constexpr int SCAN1_THREADS = 1024;
constexpr int64_t SCAN1_MAX = 1 << 14;

__global__ void __launch_bounds__(SCAN1_THREADS)
k_scan_single(const int *in, int *out, int64_t n, int *total) {
    __shared__ int wsum[SCAN1_THREADS / FMM_WAVE];
    const int t = threadIdx.x, lane = lane_id(), w = t / FMM_WAVE;
    const int64_t chunk = (n + SCAN1_THREADS - 1) / SCAN1_THREADS;
    const int64_t lo = min(n, (int64_t)t * chunk), hi = min(n, lo + chunk);
    int s = 0;
#pragma unroll 8
    for (int64_t i = lo; i < hi; ++i) s += in[i];
    const int inc = wave_incl_scan(s);
    if (lane == FMM_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int run = inc - s;
    for (int i = 0; i < w; ++i) run += wsum[i];
    if (total && t == SCAN1_THREADS - 1) *total = run + s;
#pragma unroll 8
    for (int64_t i = lo; i < hi; ++i) {
        const int v = in[i];
        out[i] = run;
        run += v;
    }
}

// ---- radix sort -------------------------------------------------------
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;              // rounds of 256 keys per tile
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / FMM_WAVE;

__global__ void __launch_bounds__(RS_THREADS)
k_rs_hist(const uint64_t *keys, int64_t n, int shift, int *hist, int ntiles) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t j = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (j < n) atomicAdd(&h[(int)((keys[j] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <bool HAS_VAL>
__global__ void __launch_bounds__(RS_THREADS)
k_rs_scatter(const uint64_t *keys, const uint32_t *vals, uint64_t *okeys, uint32_t *ovals,
             int64_t n, int shift, const int *hist_scan, int ntiles) {
    __shared__ int base_d[256];                 // running output position per digit
    __shared__ int wcount[RS_WAVES][256];       // per-wave digit counts of this round
    const int lane = lane_id(), w = threadIdx.x / FMM_WAVE;
    base_d[threadIdx.x] = hist_scan[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) wcount[i][threadIdx.x] = 0;
        __syncthreads();
        const int64_t j = tbase + (int64_t)r * RS_THREADS + threadIdx.x;
        const bool valid = j < n;
        uint64_t k = valid ? keys[j] : 0;
        const int d = (int)((k >> shift) & 255u);
        // lanes holding the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcount[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = base_d[d] + rank;
            for (int i = 0; i < w; ++i) pos += wcount[i][d];
            okeys[pos] = k;
            if (HAS_VAL) ovals[pos] = vals[j];
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) add += wcount[i][threadIdx.x];
        base_d[threadIdx.x] += add;
        __syncthreads();
    }
}

}  // namespace

size_t scan_tmp_ints(int64_t n) {
    size_t total = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        total += (size_t)m;
    }
    return total + 1;
}

hipError_t exclusive_scan(const int *in, int *out, int64_t n, int *tmp, int *total,
                          hipStream_t s) {
    if (n <= 0) {
        if (total) return hipMemsetAsync(total, 0, sizeof(int), s);
        return hipSuccess;
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles > 1 && n <= SCAN1_MAX) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN1_THREADS), 0, s, in, out, n, total);
        return hipGetLastError();
    }
    if (tiles == 1) {
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n,
                           (const int *)nullptr, total);
        return hipGetLastError();
    }
    int *sums = tmp;
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan(sums, sums, tiles, tmp + tiles, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, in, out, n,
                       (const int *)sums, (int *)nullptr);
    return hipGetLastError();
}

size_t sort_tmp_ints(int64_t n) {
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * tiles) + scan_tmp_ints(256 * tiles) + 4;
}

hipError_t radix_sort(uint64_t **keys, uint64_t **keys_alt, uint32_t **vals,
                      uint32_t **vals_alt, int64_t n, int bits, int *tmp, hipStream_t s,
                      int lo_bit) {
    if (n <= 1) return hipSuccess;
    const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    int *hist = tmp;
    int *stmp = tmp + (size_t)256 * ntiles;
    for (int shift = lo_bit; shift < lo_bit + bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(RS_THREADS), 0, s, *keys, n, shift, hist,
                           ntiles);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan(hist, hist, (int64_t)256 * ntiles, stmp, nullptr, s);
        if (e != hipSuccess) return e;
        if (vals) {
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(ntiles), dim3(RS_THREADS), 0, s, *keys,
                               *vals, *keys_alt, *vals_alt, n, shift, hist, ntiles);
            uint32_t *tv = *vals; *vals = *vals_alt; *vals_alt = tv;
        } else {
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(ntiles), dim3(RS_THREADS), 0, s, *keys,
                               (const uint32_t *)nullptr, *keys_alt, (uint32_t *)nullptr, n, shift,
                               hist, ntiles);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = *keys; *keys = *keys_alt; *keys_alt = tk;
    }
    return hipSuccess;
}

}  // namespace fmm
