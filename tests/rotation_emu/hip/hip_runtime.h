// host-only stand-in for the HIP runtime header: just enough for the kernel
// headers' per-lane code to compile as plain C++ on the CPU
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__ static
struct double4 { double x, y, z, w; };
struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
struct uint2 { unsigned x, y; };
struct float4 { float x, y, z, w; };
struct dim3 { unsigned x, y, z; };
typedef int hipError_t;
typedef void *hipStream_t;
static dim3 threadIdx, blockIdx, gridDim, blockDim;
inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
inline long long __double_as_longlong(double x) { long long b; std::memcpy(&b, &x, 8); return b; }
inline double __longlong_as_double(long long b) { double x; std::memcpy(&x, &b, 8); return x; }
int __lane_id();
template <class T> T __shfl_up(T, int, int = 64);
template <class T> T __shfl_down(T, int, int = 64);
template <class T> T __shfl_xor(T, int, int = 64);
unsigned long long __ballot(int);
int __builtin_amdgcn_readlane(int, int);
void __syncthreads();
