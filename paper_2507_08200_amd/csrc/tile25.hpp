// Geometry of the 2.5D tiled passes (k_st25, k_rb32): which tile a
// workgroup owns and which elements each of its threads loads and stores.
// The same functions run in the kernels and on the host, where
// vd_check_tiles25 walks every access of a launch and checks it against the
// array bounds (the kernels load from wrapped or clamped addresses without
// branches, so an index mistake would not show as a wrong value first).
#pragma once

#include <hip/hip_runtime.h>

namespace vd {

// tile of 32 units (cells, or half-row positions) x 16 rows x kz planes
constexpr int kT25X = 32, kT25Y = 16, kT25W = kT25X + 2;

// wrapped (periodic) or clamped index of position p along a direction of n
// cells; ok tells whether the position stands for a cell (inside the
// domain, or one wrap across a periodic face).  The index is always valid.
__host__ __device__ __forceinline__ int wrap_idx(int p, int n, bool per, bool &ok) {
    const bool in = p >= 0 && p < n;
    const int w = p < 0 ? p + n : p - n;
    const bool wrapped = per && !in && w >= 0 && w < n;
    ok = in || wrapped;
    const int c = p < 0 ? 0 : (p >= n ? n - 1 : p);
    return in ? p : (wrapped ? w : c);
}

__host__ __device__ __forceinline__ int tiles25(int nu, int ny, int nz, int kz) {
    return ((nu + kT25X - 1) / kT25X) * ((ny + kT25Y - 1) / kT25Y) * ((nz + kz - 1) / kz);
}

// origin of tile lt of a level with nu units per row: first unit u0, row
// j0, planes [k0, k1)
struct Tile25 {
    int u0, j0, k0, k1;
};

__host__ __device__ __forceinline__ Tile25 tile25(int lt, int nu, int ny, int nz, int kz) {
    const int ntx = (nu + kT25X - 1) / kT25X, nty = (ny + kT25Y - 1) / kT25Y;
    Tile25 T;
    T.u0 = (lt % ntx) * kT25X;
    lt /= ntx;
    T.j0 = (lt % nty) * kT25Y;
    T.k0 = (lt / nty) * kz;
    T.k1 = T.k0 + kz < nz ? T.k0 + kz : nz;
    return T;
}

// Thread tid of a tile: units (ua, ua + 1) of row j, and the element
// offsets within a plane of everything it loads.  Rows are nx elements
// apart; the pair being read lies other_ofs into its row, the right-hand
// side pair upd_ofs (0 for lexicographic levels; the colour halves of a
// parity-split row otherwise).  Loads never depend on a branch: a position
// that is not a cell is loaded from a clamped address and zeroed (ok
// flags false).
struct Thr25 {
    int ua, j;
    bool own;          // the pair is inside the level (it updates or sums)
    bool halo;         // the thread also loads one halo element per plane
    bool okp, okh;     // the loaded pair / halo element stands for cells
    long pair_off;     // first element of the pair read from x
    long b_off;        // first element of the right-hand side pair
    long h_off;        // halo element
};

__host__ __device__ __forceinline__ Thr25 thr25(const Tile25 &T, int tid, int nu, int nx, int ny, bool px, bool py,
                                                long other_ofs, long upd_ofs) {
    Thr25 H;
    const int tp = tid & 15, r = tid >> 4;
    H.ua = T.u0 + 2 * tp;
    H.j = T.j0 + r;
    H.own = H.ua < nu && H.j < ny;
    H.halo = tid < 2 * kT25Y + 2 * kT25X;
    bool oku, oky;
    int uw = wrap_idx(H.ua, nu, px, oku);
    uw = uw < nu - 2 ? uw : nu - 2;
    const int jw = wrap_idx(H.j, ny, py, oky);
    H.okp = oku && oky;
    H.pair_off = other_ofs + uw + (long)nx * jw;
    H.b_off = upd_ofs + (H.ua < nu - 2 ? H.ua : nu - 2) + (long)nx * (H.j < ny - 1 ? H.j : ny - 1);
    int hu, hj;
    if (tid < 2 * kT25Y) {
        hu = (tid / kT25Y) ? T.u0 + kT25X : T.u0 - 1;
        hj = T.j0 + (tid & (kT25Y - 1));
    } else {
        const int q = tid - 2 * kT25Y;
        hu = T.u0 + (q & (kT25X - 1));
        hj = (q / kT25X) ? T.j0 + kT25Y : T.j0 - 1;
    }
    bool okhu, okhj;
    H.h_off = other_ofs + wrap_idx(hu, nu, px, okhu) + (long)nx * wrap_idx(hj, ny, py, okhj);
    H.okh = H.halo && okhu && okhj;
    return H;
}

// LDS slot of the halo element of thread tid (< 96) in a (kT25Y + 2) x
// kT25W tile
__host__ __device__ __forceinline__ int halo_slot(int tid) {
    if (tid < 2 * kT25Y) {
        const int rr = tid & (kT25Y - 1), side = tid / kT25Y;
        return (rr + 1) * kT25W + (side ? kT25X + 1 : 0);
    }
    const int q = tid - 2 * kT25Y, cc = q & (kT25X - 1), side = q / kT25X;
    return (side ? kT25Y + 1 : 0) * kT25W + cc + 1;
}

// first of the four consecutive FP64 cells 2 ua .. 2 ua + 3 of row j that
// a parity-split pass of unit pair ua updates (clamped like b_off)
__host__ __device__ __forceinline__ long quad_off25(int ua, int j, int nh, int nx, int ny) {
    return 2 * (long)(ua < nh - 2 ? ua : nh - 2) + (long)nx * (j < ny - 1 ? j : ny - 1);
}

}  // namespace vd
