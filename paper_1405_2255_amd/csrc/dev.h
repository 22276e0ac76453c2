// Device-side helpers shared by the libfmm kernels: complex arithmetic,
// wavefront reductions and order-preserving encodings for atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FMM_WAVE 64

namespace fmm {

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }

// acc += s * conj?(a) * b with the conjugation of a chosen at compile time.
template <bool CONJ_A>
__device__ __forceinline__ void cmac(cplx &acc, cplx a, cplx b, double s) {
    const double ar = a.re * s, ai = (CONJ_A ? -a.im : a.im) * s;
    acc.re = fma(ar, b.re, fma(-ai, b.im, acc.re));
    acc.im = fma(ar, b.im, fma(ai, b.re, acc.im));
}

// Non-negative doubles order like their bit patterns: max/min of them can be
// taken with integer atomics.
__device__ __forceinline__ unsigned long long dbits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
    return __longlong_as_double((long long)b);
}
// Any double to an unsigned key with the same order (for min/max atomics).
__device__ __forceinline__ unsigned long long ordered_key(double x) {
    unsigned long long b = dbits(x);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ordered_val(unsigned long long k) {
    return bitsd((k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ((ax-bx)^2 + (ay-by)^2) + (az-bz)^2 with every operation rounded on its
// own.  HIP contracts a*b + c into a fused multiply-add by default (and the
// __dmul_rn / __dadd_rn helpers are plain operators that it contracts too),
// so contraction is switched off here: the value is the one IEEE double
// arithmetic gives for this expression on any machine.
__device__ __forceinline__ double dist2_exact(double ax, double ay, double az, double bx,
                                              double by, double bz) {
#pragma clang fp contract(off)
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

// Inclusive prefix sum over the wavefront (all 64 lanes active).
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < FMM_WAVE; off <<= 1) {
        const int o = __shfl_up(v, off, FMM_WAVE);
        if (lane >= off) v += o;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = FMM_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, FMM_WAVE);
    return v;
}

// 1/sqrt(x) to double precision: the hardware estimate refined by one
// Newton-Raphson step (y <- y (3 - x y^2)/2), which doubles its number of
// correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    return fma(y * 0.5, e, y);
}

// 2/sqrt(x): the same Newton step without its factor 1/2, one multiply fewer
// (y (3 - x y^2)).  The direct-sum kernels sum with it and undo the powers of
// two once per sink (exact).
__device__ __forceinline__ double rsqrt2_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-(x * y), y, 3.0);
}

// XCD-aware block order.  Workgroups are handed to the 8 XCDs of the chip in
// turn (block b to XCD b % 8), and each XCD has its own L2.  Work items in
// Morton order that are close share their inputs (neighbouring sinks read
// mostly the same sources), so block b is given logical index
// start(x) + b / 8 with x = b % 8: XCD x then processes one contiguous eighth
// of the work.  A bijection of [0, nb) for any nb.
constexpr int FMM_NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % FMM_NXCD, j = b / FMM_NXCD;
    const int q = nb / FMM_NXCD, r = nb % FMM_NXCD;
    return x * q + (x < r ? x : r) + j;
}

}  // namespace fmm
