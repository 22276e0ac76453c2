// Direct sums: the near field (P2P, eq. 1 restricted to the walk's direct
// pairs), the all-pairs GPU direct summation used as a comparison baseline,
// and the final un-permute / scale / finiteness check.
//
// P2P: one wavefront per sink leaf.  For a leaf of nb <= 64 particles the
// 64 lanes are (sink, phase) with nbp = next power of two >= nb sinks and
// 64/nbp phases; the phases stride through each source cell's particles and
// are summed with shuffles at the end, so small leaves still fill the
// wavefront.  Source particles are read as (x, y, z, m) double4 from the
// Morton-sorted copy, contiguous per source cell.
#include "internal.h"
#include "dev.h"

namespace fmm {

namespace {

template <int WANT_F, int WITH_POT>
__global__ void __launch_bounds__(256)
k_p2p(int nleaves, const int *leaf_cell, const int64_t *off, const uint64_t *list, uint64_t mask,
      TreeArrays t, const double4 *xyzm, double4 *out4) {
    const int leaf = blockIdx.x * 4 + threadIdx.x / FMM_WAVE;
    if (leaf >= nleaves) return;
    const int lane = lane_id();
    const int c = leaf_cell[leaf];
    const int beg = t.beg[c], end = t.end[c];
    const int64_t e0 = off[leaf], e1 = off[leaf + 1];
    for (int sb = beg; sb < end; sb += FMM_WAVE) {
        const int nb = min(end - sb, FMM_WAVE);
        int nbp = 1;
        while (nbp < nb) nbp <<= 1;
        const int S = FMM_WAVE / nbp;
        const int slot = lane & (nbp - 1), phase = lane / nbp;
        const int bi = sb + slot;
        const bool active = slot < nb;
        const double4 xb = xyzm[active ? bi : sb];
        double pot = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int A = (int)(list[e] & mask);
            const int a0 = t.beg[A], a1 = t.end[A];
            for (int j = a0 + phase; j < a1; j += S) {
                const double4 s = xyzm[j];
                const double dx = s.x - xb.x, dy = s.y - xb.y, dz = s.z - xb.z;
                const bool self = j == bi;
                const double r2 = self ? 1.0 : fma(dx, dx, fma(dy, dy, dz * dz));
                const double mu = self ? 0.0 : s.w;
                if (WANT_F) {
                    pot += mu / r2;
                } else {
                    const double ri = rsqrt_nr(r2);
                    const double q = mu * ri;
                    const double q3 = q * ri * ri;
                    if (WITH_POT) pot += q;
                    ax = fma(q3, dx, ax);
                    ay = fma(q3, dy, ay);
                    az = fma(q3, dz, az);
                }
            }
        }
        // sum the phases of each sink
        for (int o = nbp; o < FMM_WAVE; o <<= 1) {
            pot += __shfl_xor(pot, o, FMM_WAVE);
            if (!WANT_F) {
                ax += __shfl_xor(ax, o, FMM_WAVE);
                ay += __shfl_xor(ay, o, FMM_WAVE);
                az += __shfl_xor(az, o, FMM_WAVE);
            }
        }
        if (active && phase == 0) {
            double4 v = out4[bi];
            v.x += pot;
            v.y += ax;
            v.z += ay;
            v.w += az;
            out4[bi] = v;
        }
        (void)S;
    }
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

// sink scale of the acceptance test from the estimate: |a| (criterion a) or f
__global__ void k_scale(int want_f, int64_t n, const double4 *est4, double *scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 v = est4[i];
    scale[i] = want_f ? v.x : sqrt(fma(v.y, v.y, fma(v.z, v.z, v.w * v.w)));
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_p2p(int want_f, int with_pot, int nleaves, const int *leaf_cell,
                      const int64_t *off, const uint64_t *list, int sh, const TreeArrays &t,
                      const double4 *xyzm, double4 *out4, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    const uint64_t mask = (1ull << sh) - 1;
    const dim3 g(blocks(nleaves, 4)), b(256);
    if (want_f)
        hipLaunchKernelGGL((k_p2p<1, 0>), g, b, 0, s, nleaves, leaf_cell, off, list, mask, t, xyzm,
                           out4);
    else if (with_pot)
        hipLaunchKernelGGL((k_p2p<0, 1>), g, b, 0, s, nleaves, leaf_cell, off, list, mask, t, xyzm,
                           out4);
    else
        hipLaunchKernelGGL((k_p2p<0, 0>), g, b, 0, s, nleaves, leaf_cell, off, list, mask, t, xyzm,
                           out4);
    return hipGetLastError();
}

hipError_t launch_output(int64_t n, const uint32_t *perm, const double4 *out4, double G,
                         double *pot, double *acc, int *nonfinite, hipStream_t s) {
    hipLaunchKernelGGL(k_output, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, out4, G, pot, acc,
                       nonfinite);
    return hipGetLastError();
}

hipError_t launch_scale(int want_f, int64_t n, const double4 *est4, double *scale,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(blocks(n, 256)), dim3(256), 0, s, want_f, n, est4, scale);
    return hipGetLastError();
}

hipError_t launch_direct(int64_t n, const double *pos, const double *mass, double G,
                         double *pot, double *acc, hipStream_t s) {
    hipLaunchKernelGGL(k_direct, dim3(blocks(n, 256)), dim3(256), 0, s, n, pos, mass, G, pot, acc);
    return hipGetLastError();
}

}  // namespace fmm
