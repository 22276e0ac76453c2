// Launchers of the jerk kernels (Sec. 7, jerk; eqs:fmm:dot): with the
// expansion centres at rest, the rates Mdot come from eq:P2M:dot and the
// ordinary M2M, the rates Fdot from the ordinary M2L of Mdot (same list, same
// order) and L2L, and eq:L2P:dot evaluates the far-field jerk at each particle;
// the near field adds the time derivative of every direct pair.
#pragma once

#include "internal.h"

namespace fmm {

// v4[i] = (v_x, v_y, v_z, 0) of sorted particle i: vel (input order, 3n doubles)
// gathered through perm
hipError_t launch_gather_vel(int64_t n, const uint32_t *perm, const double *vel, double4 *v4,
                             hipStream_t s);
// Mdot_n^m of every leaf (same layout as M): sum_a mu_a d/dt Upsilon_n^m(x_a - z)
hipError_t launch_p2m_dot(int p, const TreeArrays &t, const int *leaf_cell, int nleaves,
                          const double *x, const double *y, const double *z, const double *m,
                          const double4 *v4, double *Md, hipStream_t s);
// far-field jerk of every particle: jo4[i] = (0, j_x, j_y, j_z) (G = 1), from
// the leaf's F and Fdot (assigned, not added); with active, only particles of
// leaves that hold a listed sink
hipError_t launch_l2p_dot(int p, const TreeArrays &t, const int *leaf_of, const int *leaf_cell,
                          int64_t n, const double *x, const double *y, const double *z,
                          const double4 *v4, const double *F, const double *Fd, double4 *jo4,
                          hipStream_t s, const uint8_t *active = nullptr);
// near field with jerk, FP64, in place of launch_p2p (same prepared tasks,
// ranges and partial-row layout, same summation order, so out4 receives the
// same values launch_p2p would add): (pot, a) added into out4, the jerk into
// jo4; rows of multi-task leaves go to partial / jpartial and
// launch_p2p_reduce adds each into its output
hipError_t launch_p2p_jerk(int ntasks, const int2 *tasks, const int *leaf_cell,
                           const int *nsrc_tasks, const int *moff, const int64_t *off,
                           const int2 *range, const int *up, const TreeArrays &t,
                           const double4 *xyzm, const double4 *v4, double4 *out4, double4 *jo4,
                           double4 *partial, double4 *jpartial, hipStream_t s);
// exact jerk of listed sinks (input indices) against all n sources, written in
// list order; *bad (zeroed by the caller) = 1 for an index outside [0, n)
hipError_t launch_direct_jerk_sinks(int64_t n, const double *pos, const double *vel,
                                   const double *mass, double G, int64_t nsinks,
                                   const int64_t *sinks, double *jerk, int *bad, hipStream_t s);
// listed sinks (input indices act[j], inverse permutation inv): jerk in list order
hipError_t launch_output_jerk_listed(int64_t n, int64_t nact, const int64_t *act, const int *inv,
                                     const double4 *jo4, double G, double *jerk, int *nonfinite,
                                     hipStream_t s);
// jerk[3 perm[i] + d] = G jo4[i].(y, z, w); *nonfinite = 1 on a non-finite value
hipError_t launch_output_jerk(int64_t n, const uint32_t *perm, const double4 *jo4, double G,
                              double *jerk, int *nonfinite, hipStream_t s);

}  // namespace fmm
