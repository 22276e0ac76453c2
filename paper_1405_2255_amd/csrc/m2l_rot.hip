// Rotation-accelerated M2L (App. A): the piece bookkeeping of the windowed
// kernel and the dispatch over orders.  The kernel template and its
// compile-time table of swap coefficients are in m2l_rot_impl.h.
#include "m2l_rot_impl.h"

namespace fmm {

// pieces of sink c: the 64-entry windows its list [off[c], off[c+1]) touches
__global__ void k_rot_piece_count(int ncells, const int64_t *off, int *cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    if (c == ncells) {
        cnt[c] = 0;
        return;
    }
    const int64_t e0 = off[c], e1 = off[c + 1];
    cnt[c] = e1 > e0 ? (int)((e1 - 1) / m2lr::WIN - e0 / m2lr::WIN + 1) : 0;
}

hipError_t launch_rot_pieces(int ncells, const int64_t *off, int *cnt, int *coff, int *tmp,
                             int *total, hipStream_t s) {
    hipLaunchKernelGGL(k_rot_piece_count, dim3((unsigned)((ncells + 256) / 256)), dim3(256), 0, s,
                       ncells, off, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return exclusive_scan(cnt, coff, ncells + 1, tmp, total, s);
}

#define FMM_M2L_ROT_DECLARE(P)                                                               \
    hipError_t launch_m2l_rot_##P(int64_t nlist, const uint64_t *list, int sh,               \
                                  const int64_t *off, const int *coff, const TreeArrays &t,  \
                                  const double *M, double *Fpart, hipStream_t s);
FMM_M2L_ROT_DECLARE(1) FMM_M2L_ROT_DECLARE(2) FMM_M2L_ROT_DECLARE(3) FMM_M2L_ROT_DECLARE(4)
FMM_M2L_ROT_DECLARE(5) FMM_M2L_ROT_DECLARE(6) FMM_M2L_ROT_DECLARE(7) FMM_M2L_ROT_DECLARE(8)
FMM_M2L_ROT_DECLARE(9) FMM_M2L_ROT_DECLARE(10) FMM_M2L_ROT_DECLARE(11)
FMM_M2L_ROT_DECLARE(12) FMM_M2L_ROT_DECLARE(13) FMM_M2L_ROT_DECLARE(14)
FMM_M2L_ROT_DECLARE(15) FMM_M2L_ROT_DECLARE(16)
#undef FMM_M2L_ROT_DECLARE

hipError_t launch_m2l_rot(int p, int64_t nlist, const uint64_t *list, int sh, const int64_t *off,
                          const int *coff, const TreeArrays &t, const double *M, double *Fpart,
                          hipStream_t s) {
    if (nlist <= 0) return hipSuccess;
#define CALL(P) return launch_m2l_rot_##P(nlist, list, sh, off, coff, t, M, Fpart, s)
    switch (p) {
    case 1: CALL(1);   case 2: CALL(2);   case 3: CALL(3);   case 4: CALL(4);
    case 5: CALL(5);   case 6: CALL(6);   case 7: CALL(7);   case 8: CALL(8);
    case 9: CALL(9);   case 10: CALL(10); case 11: CALL(11); case 12: CALL(12);
    case 13: CALL(13); case 14: CALL(14); case 15: CALL(15); case 16: CALL(16);
    default: return hipErrorInvalidValue;
    }
#undef CALL
}

}  // namespace fmm
