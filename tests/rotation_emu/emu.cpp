// CPU emulation of the rotation M2L kernel k_m2l_rot<P> (test infrastructure).
// The kernel's own per-lane code (Pair<P>, swap_xz, rot_z, the table and index
// functions) is compiled for the host from a copy of m2l_rot_impl.h in which
// only the register constraint of the inline asm barrier names an x86 register
// class; the lane-collective steps (shfl_down, ballot, readlane, the LDS column
// sums) are stepped lane by lane here, and every LDS row and Fpart index is
// checked.  Input and output go through files (see main).
#include "m2l_rot_impl_host.h"

#include <cstdio>
#include <cstdlib>
#include <vector>
#include <cstdio>

using namespace fmm;
using namespace fmm::m2lr;

static int g_fail = 0;
#define CHECK(c, ...)                                                     \
    do {                                                                  \
        if (!(c)) {                                                       \
            if (g_fail < 20) {                                            \
                std::fprintf(stderr, "CHECK failed %s:%d: %s: ", __FILE__, __LINE__, #c); \
                std::fprintf(stderr, __VA_ARGS__);                        \
                std::fprintf(stderr, "\n");                               \
            }                                                             \
            ++g_fail;                                                     \
        }                                                                 \
    } while (0)

struct Lds {
    // one separately allocated row per lane, so that a write past a row is an
    // out-of-bounds access (AddressSanitizer) and not a write into the next row
    std::vector<double *> rows;
    Lds() {
        for (int l = 0; l < WIN; ++l) rows.push_back(new double[LDS_STRIDE]);
    }
    ~Lds() {
        for (auto r : rows) delete[] r;
    }
};

template <int P, int N0>
static void groups(Pair<P> *pr, Lds &lds, uint64_t endmask, const int *piece, double *Fpart,
                   int64_t fpart_len, std::vector<int> &written) {
    constexpr int N1 = group_end(P, N0);
    constexpr int GV = 2 * (tri(N1, 0) - tri(N0, 0));
    constexpr int NC = tri(P + 1, 0);
    static_assert(GV <= WIN && GV <= LDS_STRIDE, "group wider than a row");
    for (int lane = 0; lane < WIN; ++lane) {
        double *row = lds.rows[lane];
        for (int i = 0; i < LDS_STRIDE; ++i) row[i] = NAN;   // stale values show up
        Unroll<N0, N1 - 1>::run([&]<int N>() {
            const int col = 2 * (tri(N, 0) - tri(N0, 0));
            CHECK(col + 2 * N + 1 < LDS_STRIDE, "row col %d N %d", col, N);
            pr[lane].template backward<N>(row, col);
        });
    }
    for (int lane = 0; lane < GV; ++lane) {
        double acc = 0.0;
        for (int src = 0; src < WIN; ++src) {
            CHECK(lane < LDS_STRIDE, "lane %d", lane);
            acc += lds.rows[src][lane];
            if ((endmask >> src) & 1) {
                const int pc = piece[src];
                const int64_t idx = (int64_t)pc * 2 * NC + 2 * tri(N0, 0) + lane;
                CHECK(pc >= 0 && idx >= 0 && idx < fpart_len, "piece %d idx %lld len %lld", pc,
                      (long long)idx, (long long)fpart_len);
                if (idx >= 0 && idx < fpart_len) {
                    Fpart[idx] = acc;
                    written[idx] += 1;
                }
                acc = 0.0;
            }
        }
    }
    if constexpr (N1 <= P) groups<P, N1>(pr, lds, endmask, piece, Fpart, fpart_len, written);
}

// nlist keys (sink << sh | source), sink-sorted; off: ncells + 1 list offsets;
// coff: ncells + 1 piece offsets; cen: 4 doubles per cell; M: tri(P+1,0)
// complex per cell; F out: tri(P+1,0) complex per cell.  Returns the number of
// failed checks.
template <int P>
static int run(int64_t nlist, const uint64_t *list, int sh, int ncells, const int64_t *off,
               const int *coff, const double *cen, const double *M, double *F) {
    constexpr int NC = tri(P + 1, 0);
    const int64_t npieces = coff[ncells];
    const int64_t bound = (nlist + 63) / 64 + ncells;
    CHECK(npieces <= bound, "pieces %lld above bound %lld", (long long)npieces, (long long)bound);
    const int64_t fpart_len = 2 * (int64_t)NC * std::max<int64_t>(bound, 1);
    std::vector<double> Fpart(fpart_len, NAN);
    std::vector<int> written(fpart_len, 0);
    const int64_t nwin = (nlist + WIN - 1) / WIN;
    // the kernel's block -> window map is a bijection
    {
        std::vector<int> seen(nwin, 0);
        for (int64_t b = 0; b < nwin; ++b) {
            const int w = xcd_block((int)b, (int)nwin);
            CHECK(w >= 0 && w < nwin, "xcd_block %d of %lld", w, (long long)nwin);
            if (w >= 0 && w < nwin) seen[w]++;
        }
        for (int64_t w = 0; w < nwin; ++w) CHECK(seen[w] == 1, "window %lld seen %d", (long long)w, seen[w]);
    }
    std::vector<Pair<P>> pr(WIN);
    Lds lds;
    for (int64_t w = 0; w < nwin; ++w) {
        int Bv[WIN], Av[WIN], piece[WIN];
        bool act[WIN];
        for (int lane = 0; lane < WIN; ++lane) {
            const int64_t e = w * WIN + lane;
            act[lane] = e < nlist;
            const uint64_t key = list[act[lane] ? e : nlist - 1];
            Bv[lane] = (int)(key >> sh);
            Av[lane] = (int)(key & ((1ull << sh) - 1));
            CHECK(Bv[lane] >= 0 && Bv[lane] < ncells && Av[lane] >= 0 && Av[lane] < ncells,
                  "cells %d %d", Bv[lane], Av[lane]);
        }
        uint64_t endmask = 0;
        for (int lane = 0; lane < WIN; ++lane) {
            const int64_t e = w * WIN + lane;
            const int nextB = lane + 1 < WIN ? Bv[lane + 1] : Bv[lane];   // __shfl_down(B, 1)
            const bool end = act[lane] && (lane == WIN - 1 || e + 1 >= nlist || nextB != Bv[lane]);
            if (end) endmask |= 1ull << lane;
            const int B = Bv[lane];
            piece[lane] = coff[B] + (int)((int64_t)w - off[B] / WIN);
            if (act[lane]) {
                CHECK(off[B] <= e && e < off[B + 1], "entry %lld outside its sink's range", (long long)e);
                CHECK(piece[lane] >= coff[B] && piece[lane] < coff[B + 1], "piece %d of sink %d [%d, %d)",
                      piece[lane], B, coff[B], coff[B + 1]);
            }
            const double *cb = cen + 4 * (size_t)B, *ca = cen + 4 * (size_t)Av[lane];
            pr[lane].setup(cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2]);
            const cplx *Ma = reinterpret_cast<const cplx *>(M) + (size_t)Av[lane] * NC;
            const cplx m0[1] = {Ma[0]};
            pr[lane].template forward_from<0>(Ma, m0);
        }
        groups<P, 0>(pr.data(), lds, endmask, piece, Fpart.data(), fpart_len, written);
    }
    // every piece written exactly once, nothing else
    for (int64_t pc = 0; pc < bound; ++pc)
        for (int i = 0; i < 2 * NC; ++i) {
            const int wv = written[pc * 2 * NC + i];
            CHECK(wv == (pc < npieces ? 1 : 0), "piece %lld coef %d written %d times", (long long)pc, i, wv);
        }
    // the reduce: pieces of each sink in order
    for (int c = 0; c < ncells; ++c)
        for (int i = 0; i < 2 * NC; ++i) {
            double s = 0.0;
            for (int pc = coff[c]; pc < coff[c + 1]; ++pc) s += Fpart[(size_t)pc * 2 * NC + i];
            F[(size_t)c * 2 * NC + i] = s;
        }
    return g_fail;
}

static int dispatch(int p, int64_t nlist, const uint64_t *list, int sh, int ncells,
                    const int64_t *off, const int *coff, const double *cen, const double *M,
                    double *F) {
    switch (p) {
#define C(P) case P: return run<P>(nlist, list, sh, ncells, off, coff, cen, M, F);
    EMU_ORDERS
#undef C
    default: return -1;
    }
}

// in:  int64 p, nlist, sh, ncells; then keys u64[nlist], off i64[ncells+1],
//      coff i32[ncells+1], cen f64[4 ncells], M f64[2 tri(p+1,0) ncells]
// out: int64 failed checks, then F f64[2 tri(p+1,0) ncells]
int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t h[4];
    if (std::fread(h, 8, 4, f) != 4) return 2;
    const int p = (int)h[0], sh = (int)h[2], ncells = (int)h[3];
    const int64_t nlist = h[1];
    const size_t nc = (size_t)(p + 1) * (p + 2) / 2;
    std::vector<uint64_t> keys(nlist);
    std::vector<int64_t> off(ncells + 1);
    std::vector<int> coff(ncells + 1);
    std::vector<double> cen(4 * (size_t)ncells), M(2 * nc * ncells), F(2 * nc * ncells, 0.0);
    bool ok = std::fread(keys.data(), 8, nlist, f) == (size_t)nlist &&
              std::fread(off.data(), 8, ncells + 1, f) == (size_t)ncells + 1 &&
              std::fread(coff.data(), 4, ncells + 1, f) == (size_t)ncells + 1 &&
              std::fread(cen.data(), 8, cen.size(), f) == cen.size() &&
              std::fread(M.data(), 8, M.size(), f) == M.size();
    std::fclose(f);
    if (!ok) return 2;
    g_fail = 0;
    const int64_t fails = dispatch(p, nlist, keys.data(), sh, ncells, off.data(), coff.data(),
                                   cen.data(), M.data(), F.data());
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    std::fwrite(&fails, 8, 1, o);
    std::fwrite(F.data(), 8, F.size(), o);
    std::fclose(o);
    return 0;
}
