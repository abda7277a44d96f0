// Host-side walk over every memory access of the 2.5D tiled passes
// (k_st25 in all its modes, which also covers the residual checks of
// k_res25u, k_rb32 in all its modes, and the direct residual checks k_resd
// with their coefficient arrays) for one level shape and tile depth, using
// the kernels' own geometry functions (tile25.hpp).  Nothing here touches
// the GPU.
#include "vd_internal.hpp"
#include "tile25.hpp"

namespace vd {
namespace {

struct Walk {
    long n;              // elements of the array being addressed
    int64_t accesses = 0, violations = 0;
    void elem(long off, long n_arr) {
        accesses++;
        if (off < 0 || off >= n_arr) violations++;
    }
    // a vector access of w consecutive elements, aligned to w elements
    void vec(long off, int w, long n_arr) {
        accesses++;
        if (off < 0 || off + w > n_arr || off % w) violations++;
    }
    void lds(int slot) {
        accesses++;
        if (slot < 0 || slot >= (kT25Y + 2) * kT25W) violations++;
    }
};

// xcd_tile(): workgroup b of a launch of 8 * ceil(nt / 8) takes tile
// (b & 7) * chunk + (b >> 3); every tile must be taken exactly once
bool xcd_mapping_ok(int nt) {
    const int chunk = (nt + 7) >> 3, grid = 8 * ((nt + 7) / 8);
    std::vector<int> seen(nt > 0 ? nt : 1, 0);
    for (int b = 0; b < grid; b++) {
        const int t = (b & 7) * chunk + (b >> 3);
        if (t < nt) seen[t]++;
    }
    for (int t = 0; t < nt; t++)
        if (seen[t] != 1) return false;
    return true;
}

void walk_st25(Walk &W, int nx, int ny, int nz, bool px, bool py, bool pz, int kz) {
    const long n = (long)nx * ny * nz, nxy = (long)nx * ny;
    const int nt = tiles25(nx, ny, nz, kz);
    for (int lt = 0; lt < nt; lt++) {
        const Tile25 T = tile25(lt, nx, ny, nz, kz);
        for (int tid = 0; tid < kBlock; tid++) {
            const Thr25 H = thr25(T, tid, nx, nx, ny, px, py, 0, 0);
            const int tp = tid & 15, r = tid >> 4;
            auto pair = [&](int kk) {   // ld_pair: x (FP64 or FP32), wide
                bool ok;
                W.vec(H.pair_off + nxy * wrap_idx(kk, nz, pz, ok), 2, n);
            };
            auto halo = [&](int kk) {   // ld_h
                bool ok;
                W.elem(H.h_off + nxy * wrap_idx(kk, nz, pz, ok), n);
            };
            auto rhs = [&](int kk) {    // ld_b
                W.vec(H.b_off + nxy * (kk < nz - 1 ? kk : nz - 1), 2, n);
            };
            pair(T.k0 - 1);
            pair(T.k0);
            pair(T.k0 + 1);
            halo(T.k0);
            rhs(T.k0);
            for (int k = T.k0; k < T.k1; k++) {
                W.lds((r + 1) * kT25W + 2 * tp + 1);
                W.lds((r + 1) * kT25W + 2 * tp + 2);
                if (H.halo) W.lds(halo_slot(tid));
                pair(k + 2);
                halo(k + 1);
                rhs(k + 1);
                W.vec(H.b_off + nxy * k, 2, n);                 // MODE 5: FP64 unknown pair
                if (!H.own) continue;
                W.lds((r + 1) * kT25W + 2 * tp);                 // x- of cell ia
                W.lds((r + 1) * kT25W + 2 * tp + 3);             // x+ of cell ia + 1
                for (int q = 0; q < 2; q++) {
                    W.lds(r * kT25W + 2 * tp + 1 + q);
                    W.lds((r + 2) * kT25W + 2 * tp + 1 + q);
                    // MODE 2: FP32 residual and unknown, lexicographic or
                    // parity-split by row
                    LevDesc D;
                    memset(&D, 0, sizeof D);
                    D.nx = nx; D.ny = ny; D.nz = nz; D.nxy = (int)nxy;
                    for (int rb = 0; rb < 2; rb++) {
                        if (rb && nx % 4) continue;
                        D.rb = rb;
                        W.elem(cell_pos(D, H.ua + q, H.j, k), n);
                    }
                }
                W.vec(H.ua + (long)nx * H.j + nxy * k, 2, n);  // MODE 0/4 store, MODE 5 FP64 store
            }
        }
    }
}

void walk_rb32(Walk &W, int nx, int ny, int nz, bool px, bool py, bool pz, int kz) {
    const long n = (long)nx * ny * nz, nxy = (long)nx * ny;
    const int nh = nx >> 1;
    const int nt = tiles25(nh, ny, nz, kz);
    for (int colour = 0; colour < 2; colour++) {
        const int oofs = (1 - colour) * nh, uofs = colour * nh;
        for (int lt = 0; lt < nt; lt++) {
            const Tile25 T = tile25(lt, nh, ny, nz, kz);
            for (int tid = 0; tid < kBlock; tid++) {
                const Thr25 H = thr25(T, tid, nh, nx, ny, px, py, oofs, uofs);
                const int tp = tid & 15, r = tid >> 4;
                const long q_off = quad_off25(H.ua, H.j, nh, nx, ny);
                auto pair = [&](int kk) {
                    bool ok;
                    W.vec(H.pair_off + nxy * wrap_idx(kk, nz, pz, ok), 2, n);
                };
                auto halo = [&](int kk) {
                    bool ok;
                    W.elem(H.h_off + nxy * wrap_idx(kk, nz, pz, ok), n);
                };
                auto rhs = [&](int kk) { W.vec(H.b_off + nxy * (kk < nz - 1 ? kk : nz - 1), 2, n); };
                pair(T.k0 - 1);
                pair(T.k0);
                pair(T.k0 + 1);
                halo(T.k0);
                rhs(T.k0);
                for (int k = T.k0; k < T.k1; k++) {
                    W.lds((r + 1) * kT25W + 2 * tp + 1);
                    W.lds((r + 1) * kT25W + 2 * tp + 2);
                    if (H.halo) W.lds(halo_slot(tid));
                    pair(k + 2);
                    halo(k + 1);
                    rhs(k + 1);
                    W.vec(q_off + nxy * k, 2, n);          // PM 5: FP64 cells 2ma, 2ma + 1
                    W.vec(q_off + 2 + nxy * k, 2, n);      //        and 2ma + 2, 2ma + 3
                    if (!H.own) continue;
                    for (int q = 0; q < 2; q++) {
                        const int lc = (r + 1) * kT25W + 2 * tp + 1 + q;
                        W.lds(lc - 1);
                        W.lds(lc + 1);
                        W.lds(lc - kT25W);
                        W.lds(lc + kT25W);
                    }
                    W.vec(uofs + H.ua + (long)nx * H.j + nxy * k, 2, n);   // PM 0/4 store
                }
            }
        }
    }
}

// k_resd: a thread owns the pair (ia, ia + 1) of row j and reads its x-y
// neighbours, its z window, the right-hand side, the face arrays and the
// cell coefficient directly; it stores the FP32 residual in either layout
void walk_resd(Walk &W, int nx, int ny, int nz, bool px, bool py, bool pz, int kz) {
    const long n = (long)nx * ny * nz, nxy = (long)nx * ny;
    const long nbx = (long)(nx + 1) * ny * nz, nby = (long)nx * (ny + 1) * nz, nbz = nxy * (nz + 1);
    const int nt = tiles25(nx, ny, nz, kz);
    for (int lt = 0; lt < nt; lt++) {
        const Tile25 T = tile25(lt, nx, ny, nz, kz);
        for (int tid = 0; tid < kBlock; tid++) {
            const int ia = T.u0 + 2 * (tid & 15), j = T.j0 + (tid >> 4);
            if (!(ia < nx && j < ny)) continue;
            bool okl, okr, oks, okn;
            const long il = wrap_idx(ia - 1, nx, px, okl), ir = wrap_idx(ia + 2, nx, px, okr);
            const long js = wrap_idx(j - 1, ny, py, oks), jn = wrap_idx(j + 1, ny, py, okn);
            const long oc = ia + (long)nx * j;
            auto zpair = [&](int kk) {
                bool ok;
                W.vec(oc + nxy * wrap_idx(kk, nz, pz, ok), 2, n);
            };
            zpair(T.k0 - 1);
            zpair(T.k0);
            for (int k = T.k0; k < T.k1; k++) {
                const long pk = nxy * k;
                zpair(k + 1);
                W.elem(il + (long)nx * j + pk, n);
                W.elem(ir + (long)nx * j + pk, n);
                W.vec(ia + (long)nx * js + pk, 2, n);
                W.vec(ia + (long)nx * jn + pk, 2, n);
                W.vec(oc + pk, 2, n);                                        // b
                const long fxrow = (long)(nx + 1) * (j + (long)ny * k), fyrow = (long)nx * (j + (long)(ny + 1) * k);
                for (int q = 0; q < 3; q++) W.elem(fxrow + ia + q, nbx);      // x faces
                W.vec(fyrow + ia, 2, nby);                                   // y faces
                W.vec(fyrow + nx + ia, 2, nby);
                W.vec(oc + pk, 2, nbz);                                      // z faces
                W.vec(oc + pk + nxy, 2, nbz);
                W.vec(oc + pk, 2, n);                                        // cell coefficient
                LevDesc D;
                memset(&D, 0, sizeof D);
                D.nx = nx; D.ny = ny; D.nz = nz; D.nxy = (int)nxy;
                for (int q = 0; q < 2; q++)
                    for (int rb = 0; rb < 2; rb++) {
                        if (rb && nx % 4) continue;
                        D.rb = rb;
                        W.elem(cell_pos(D, ia + q, j, k), n);                // FP32 residual / unknown
                    }
                W.vec(oc + pk, 2, n);                                        // lexicographic pair store
            }
        }
    }
}

}  // namespace
}  // namespace vd

extern "C" vd_status vd_check_tiles25(int32_t nx, int32_t ny, int32_t nz, int32_t periodic, int32_t kz, int32_t kernel,
                                      int64_t *accesses, int64_t *violations) {
    using namespace vd;
    if (nx < 2 || ny < 1 || nz < 1 || kz < 1 || !accesses || !violations) return VD_EINVAL;
    if (kernel == 0 && nx % 2) return VD_EINVAL;
    if (kernel == 1 && nx % 4) return VD_EINVAL;
    if (kernel == 2 && nx % 2) return VD_EINVAL;
    if (kernel < 0 || kernel > 2) return VD_EINVAL;
    const bool px = periodic & 1, py = periodic & 2, pz = periodic & 4;
    Walk W;
    if (kernel == 0) walk_st25(W, nx, ny, nz, px, py, pz, kz);
    else if (kernel == 1) walk_rb32(W, nx, ny, nz, px, py, pz, kz);
    else walk_resd(W, nx, ny, nz, px, py, pz, kz);
    const int nt = kernel == 1 ? tiles25(nx >> 1, ny, nz, kz) : tiles25(nx, ny, nz, kz);
    W.accesses++;
    if (!xcd_mapping_ok(nt)) W.violations++;
    *accesses = W.accesses;
    *violations = W.violations;
    return VD_OK;
}
