// grid.hpp -- output-tile order of the persistent update kernels.
//
// A region of C is cut into tiles, the tiles grouped into square super-tiles;
// workgroups are dealt to the 8 XCDs round-robin, and each XCD works through
// whole super-tiles so the operand blocks they read stay in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

namespace ff {

constexpr int GRID_MAXSUP = 640;   // super-tiles the balanced order can describe

struct Grid {
    int tm, tn;        // output tile rows, columns
    int gm, gn;        // tiles per super-tile along M and N
    int nbm, nbn;      // tiles along M and N
    int nsm, nsn;      // super-tiles along M and N
    int flat;          // 1: slot = bi + bj * nbm, no super-tiles (small regions)
    int tri;           // 1: square lower region enumerated as a triangle of super-tiles
    int shift;         // LOWER: write only i - j >= shift
    int nslots;        // flat slots covering every super-tile
    // Balanced order: the region's tiles listed super-tile by super-tile; XCD x
    // (workgroups b with b % 8 == x) takes the x-th eighth of the list and its
    // workgroups stride through it, so shares differ by at most one tile.
    int balanced;
    int nsup;
    int ntiles;
    int tfirst, tlast;          // the launch covers tiles [tfirst, tlast) of the balanced order
    int pre[GRID_MAXSUP + 1];   // tiles in super-tiles [0, u)
};

// Super-tile u of the slot order.
__host__ __device__ __forceinline__ void super_of(const Grid& g, int u, int& SI, int& SJ) {
    if (g.tri) {
        SJ = 0;
        while (u >= g.nsm - SJ) { u -= g.nsm - SJ; ++SJ; }
        SI = SJ + u;
    } else {
        SI = u % g.nsm;
        SJ = u / g.nsm;
    }
}

__host__ __device__ __forceinline__ bool tile_in_region(const Grid& g, bool lower, int bi, int bj) {
    return bi < g.nbm && bj < g.nbn && !(lower && (bi * g.tm + g.tm - 1) - bj * g.tn < g.shift);
}

// The t-th tile of the balanced order (column-major inside a super-tile).
__host__ __device__ __forceinline__ void tile_of_index(const Grid& g, bool lower, int t, int& bi, int& bj) {
    int lo = 0, hi = g.nsup - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    int local = t - g.pre[lo];
    int SI, SJ;
    super_of(g, lo, SI, SJ);
    bi = SI * g.gm;
    bj = SJ * g.gn;
    if (g.pre[lo + 1] - g.pre[lo] == g.gm * g.gn) {     // a whole super-tile
        bi += local % g.gm;
        bj += local / g.gm;
        return;
    }
    for (int c = 0; c < g.gn; ++c)
        for (int r = 0; r < g.gm; ++r)
            if (tile_in_region(g, lower, SI * g.gm + r, SJ * g.gn + c)) {
                if (local == 0) { bi = SI * g.gm + r; bj = SJ * g.gn + c; return; }
                --local;
            }
}

// This workgroup's walk over the tile order: a balanced grid's range [tfirst,
// tlast) is cut into 8 contiguous XCD shares (workgroup b runs on XCD b % 8),
// each walked grid-stride by that XCD's workgroups; a flat grid walks its slots.
__device__ __forceinline__ void tile_walk(const Grid& g, int& it0, int& it1, int& itd) {
    if (g.balanced) {
        const int xg = blockIdx.x % N_XCD;
        const int64_t nt = g.tlast - g.tfirst;
        it0 = g.tfirst + (int)(nt * xg / N_XCD) + (int)blockIdx.x / N_XCD;
        it1 = g.tfirst + (int)(nt * (xg + 1) / N_XCD);
        itd = (int)gridDim.x / N_XCD;
    } else {
        it0 = (int)blockIdx.x;
        it1 = g.nslots;
        itd = (int)gridDim.x;
    }
}

// Map a flat slot to an output tile (bi, bj).  Returns false when the slot is
// empty.  Workgroups are dealt to the 8 XCDs round-robin, so slot % 8 is the XCD;
// each XCD works through whole super-tiles and the operand blocks of a
// super-tile stay in that XCD's L2.
__device__ __forceinline__ bool tile_of_slot(const Grid& g, int slot, bool lower, int& bi, int& bj) {
    if (g.flat) {
        bi = slot % g.nbm;
        bj = slot / g.nbm;
        if (bj >= g.nbn) return false;
        return !(lower && (bi * g.tm + g.tm - 1) - bj * g.tn < g.shift);
    }
    const int per = g.gm * g.gn;
    const int xcd = slot % N_XCD;
    const int k = slot / N_XCD;
    const int u = (k / per) * N_XCD + xcd;
    const int within = k % per;
    if (u >= (g.tri ? g.nsm * (g.nsm + 1) / 2 : g.nsm * g.nsn)) return false;
    int SI, SJ;
    super_of(g, u, SI, SJ);
    bi = SI * g.gm + (within % g.gm);
    bj = SJ * g.gn + (within / g.gm);
    if (bi >= g.nbm || bj >= g.nbn) return false;
    if (lower && (bi * g.tm + g.tm - 1) - bj * g.tn < g.shift) return false;   // wholly above the line
    return true;
}
// Super-tiles are square (gm * tm == gn * tn) so that a square lower region can be
// enumerated as a triangle of them.
inline Grid make_grid(int tm, int tn, int gm, int gn, int M, int N, bool lower, int shift) {
    Grid g;
    g.tm = tm;
    g.tn = tn;
    g.gm = gm;
    g.gn = gn;
    g.nbm = (M + tm - 1) / tm;
    g.nbn = (N + tn - 1) / tn;
    g.nsm = (g.nbm + gm - 1) / gm;
    g.nsn = (g.nbn + gn - 1) / gn;
    g.tri = (lower && M == N && shift == 0 && gm * tm == gn * tn) ? 1 : 0;
    g.shift = shift;
    const int nsup = g.tri ? g.nsm * (g.nsm + 1) / 2 : g.nsm * g.nsn;
    g.nslots = ((nsup + N_XCD - 1) / N_XCD) * N_XCD * gm * gn;
    // Regions of fewer tiles than the chip has CUs gain nothing from the L2
    // grouping, and the rounding up to whole super-tiles per XCD would launch
    // mostly empty workgroups.
    g.flat = (int64_t)g.nbm * g.nbn < 256 ? 1 : 0;
    if (g.flat) g.nslots = g.nbm * g.nbn;
    g.balanced = 0;
    g.nsup = nsup;
    g.ntiles = 0;
    g.tfirst = g.tlast = 0;
    if (!g.flat && nsup <= GRID_MAXSUP) {
        g.pre[0] = 0;
        for (int u = 0; u < nsup; ++u) {
            int SI, SJ, c = 0;
            super_of(g, u, SI, SJ);
            for (int jj = 0; jj < gn; ++jj)
                for (int ii = 0; ii < gm; ++ii) c += tile_in_region(g, lower, SI * gm + ii, SJ * gn + jj);
            g.pre[u + 1] = g.pre[u] + c;
        }
        g.ntiles = g.pre[nsup];
        g.balanced = 1;
        g.tlast = g.ntiles;
    }
    return g;
}
// Grid size of a persistent launch: at most max_wg, a multiple of the XCD count,
// and no more than the tiles (the balanced order needs whole XCD groups).
inline int persistent_grid(Grid& g, int max_wg) {
    if (!g.balanced) return max_wg < g.nslots ? max_wg : g.nslots;
    const int nt = g.tlast - g.tfirst;
    int nwg = max_wg < nt ? max_wg : nt;
    nwg = (nwg + N_XCD - 1) / N_XCD * N_XCD;
    return nwg > N_XCD ? nwg : N_XCD;
}
// Restrict a balanced grid to the tiles [f0 * ntiles, f1 * ntiles) of its order
// (0 <= f0 <= f1 <= 1).  Returns false for a flat grid, whose order is not split.
inline bool grid_set_range(Grid& g, double f0, double f1) {
    if (!g.balanced) return false;
    g.tfirst = (int)(f0 * g.ntiles + 0.5);
    g.tlast = (int)(f1 * g.ntiles + 0.5);
    if (g.tlast > g.ntiles) g.tlast = g.ntiles;
    if (g.tfirst > g.tlast) g.tfirst = g.tlast;
    return true;
}
inline Grid make_grid(int tile, int M, int N, bool lower, int shift) {
    return make_grid(tile, tile, UPD_GROUP, UPD_GROUP, M, N, lower, shift);
}

// Offsets of a 128 x 128 tile of a matrix with leading dimension ld stay below
// BUF_RECORDS.
inline bool ld_fits(int64_t ld, size_t sz) { return (128 + 128 * ld) * (int64_t)sz < (int64_t)BUF_RECORDS; }

// Compute units of the current device (cached per device).
inline int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

}  // namespace ff
