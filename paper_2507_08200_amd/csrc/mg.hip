// Geometric multigrid for batches of Helmholtz problems (alpha - div beta grad) x = b
// on uniform Cartesian grids, FP64 or FP32 inside FP64 iterative refinement.
//
// Each implicit equation of the scheme is cast in Helmholtz form and solved
// by multigrid (Sec. 4 of the paper); several right-hand sides go through
// one solve (Sec. 7).  The cycle itself is this library's design: V(nu1,nu2)
// with red-black Gauss-Seidel, mean-of-8 restriction, piecewise-constant
// prolongation, coarse operators rediscretised from averaged coefficients
// and FP64 Jacobi-PCG on the coarsest level.
//
// Launch structure on gfx950:
//   * fine levels: one launch per colour / transfer covers that level of
//     every problem in the batch (block -> (problem, tile) via a prefix
//     table; blocks are spread so each XCD gets a contiguous tile range);
//   * coarse levels (<= kCoarseMax cells) and the bottom solve of every
//     problem run in ONE fused launch, one workgroup per problem;
//   * residual norms are deterministic two-stage reductions, and the
//     convergence decisions are taken on the device (per-problem active
//     flags), so the host reads back one small state array per chunk.
#include "vd_internal.hpp"
#include "tile25.hpp"

#include <type_traits>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace vd {

constexpr int kCoarseMax = 4096;     // levels at or below this size run in the fused kernel
constexpr int kBottomMaxIt = 500;
constexpr double kBottomTol = 1e-14;

// ------------------------------------------------------------ cell bodies
template <typename T>
__device__ __forceinline__ T load_b(const LevDesc &L, int c, int i, int j, int k) {
    T b = gld((const T *)L.b, c);
    if (L.lift) b = (T)((double)b + lift_term(L, i, j, k));
    return b;
}

template <typename T>
__device__ __forceinline__ void gs_update(const LevDesc &L, int c, int i, int j, int k) {
    if (L.has_mask && !gld(L.mask, c)) return;
    T *x = (T *)L.x;
    T dg, of;
    row_terms<T, T>(L, x, i, j, k, c, dg, of);
    T b = load_b<T>(L, c, i, j, k);
    gst(x, c, (b + of) / dg);
}

template <typename T>
__device__ __forceinline__ T residual_at(const LevDesc &L, int c, int i, int j, int k) {
    if (L.has_mask && !gld(L.mask, c)) return (T)0;
    const T *x = (const T *)L.x;
    T dg, of;
    row_terms<T, T>(L, x, i, j, k, c, dg, of);
    T b = load_b<T>(L, c, i, j, k);
    return b - (dg * gld(x, c) - of);
}

// coarse cell (I,J,K): mean of the 8 children's residuals (k, j, i order)
template <typename T>
__device__ __forceinline__ void restrict_cell(const LevDesc &F, const LevDesc &C, int cc, int I, int J, int K) {
    T s = 0;
    for (int kk = 0; kk < 2; kk++)
        for (int jj = 0; jj < 2; jj++)
            for (int ii = 0; ii < 2; ii++) {
                int i = 2 * I + ii, j = 2 * J + jj, k = 2 * K + kk;
                int c = i + F.nx * j + F.nxy * k;
                s += residual_at<T>(F, c, i, j, k);
            }
    T v = (C.has_mask && !gld(C.mask, cc)) ? (T)0 : (T)0.125 * s;
    gst((T *)C.b, cc, v);
    gst((T *)C.x, cc, (T)0);
}

// residual of a uniform-coefficient level (no mask) at (i, j, k): the six
// neighbours are loaded from wrapped or clamped indices without branches
// (an out-of-domain neighbour is ignored by the row), so all loads of a
// coarse cell's eight children can be in flight together
template <typename T>
__device__ __forceinline__ T residual_uni(const LevDesc &F, const T *__restrict__ x, int i, int j, int k) {
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const long nxy = F.nxy;
    auto w = [](int p, int n, bool per) { return p < 0 ? (per ? p + n : 0) : (p >= n ? (per ? p - n : n - 1) : p); };
    const bool px = F.kind[0] == VD_BC_PERIODIC, py = F.kind[2] == VD_BC_PERIODIC, pz = F.kind[4] == VD_BC_PERIODIC;
    (void)nxy;
    T nb[6];
    nb[0] = gld(x, cell_pos(F, w(i - 1, nx, px), j, k));
    nb[1] = gld(x, cell_pos(F, w(i + 1, nx, px), j, k));
    nb[2] = gld(x, cell_pos(F, i, w(j - 1, ny, py), k));
    nb[3] = gld(x, cell_pos(F, i, w(j + 1, ny, py), k));
    nb[4] = gld(x, cell_pos(F, i, j, w(k - 1, nz, pz)));
    nb[5] = gld(x, cell_pos(F, i, j, w(k + 1, nz, pz)));
    const long cp = cell_pos(F, i, j, k);
    const T xc = gld(x, cp);
    T bv = gld((const T *)F.b, cp);
    T dg, of;
    row_terms_uni<T>(F, i, j, k, nb, dg, of);
    if (F.lift) bv = (T)((double)bv + lift_term_uni(F, i, j, k));
    return bv - (dg * xc - of);
}

template <typename T>
__device__ __forceinline__ void restrict_cell_uni(const LevDesc &F, const LevDesc &C, int cc, int I, int J, int K) {
    const T *x = (const T *)F.x;
    T r[8];
#pragma unroll
    for (int q = 0; q < 8; q++) r[q] = residual_uni<T>(F, x, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2));
    T s = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) s += r[q];
    gst((T *)C.b, cc, (T)0.125 * s);
    gst((T *)C.x, cc, (T)0);
}

// residual of a level with face and/or cell coefficient arrays and no mask
// at (i, j, k): the six neighbours, the six face coefficients, the cell
// coefficient and b are loaded from valid (wrapped or clamped) addresses
// without branches, and the row is row_terms_fc's (the arithmetic of
// residual_at: same faces, order and lifting), so all loads of a coarse
// cell's eight children can be in flight together
template <typename T>
__device__ __forceinline__ T residual_fc(const LevDesc &F, const T *__restrict__ x, int i, int j, int k) {
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const long nxy = F.nxy;
    auto w = [](int p, int n, bool per) { return p < 0 ? (per ? p + n : 0) : (p >= n ? (per ? p - n : n - 1) : p); };
    const bool px = F.kind[0] == VD_BC_PERIODIC, py = F.kind[2] == VD_BC_PERIODIC, pz = F.kind[4] == VD_BC_PERIODIC;
    const long c = i + (long)nx * j + nxy * k;
    T nb[6], fc[6];
    nb[0] = gld(x, w(i - 1, nx, px) + (long)nx * j + nxy * k);
    nb[1] = gld(x, w(i + 1, nx, px) + (long)nx * j + nxy * k);
    nb[2] = gld(x, i + (long)nx * w(j - 1, ny, py) + nxy * k);
    nb[3] = gld(x, i + (long)nx * w(j + 1, ny, py) + nxy * k);
    nb[4] = gld(x, i + (long)nx * j + nxy * w(k - 1, nz, pz));
    nb[5] = gld(x, i + (long)nx * j + nxy * w(k + 1, nz, pz));
    const T xc = gld(x, c);
    T bv = gld((const T *)F.b, c);
    const bool fb = F.var_beta;
    const T *__restrict__ BX = fb ? (const T *)Coef<T>::bx(F) : x;
    const T *__restrict__ BY = fb ? (const T *)Coef<T>::by(F) : x;
    const T *__restrict__ BZ = fb ? (const T *)Coef<T>::bz(F) : x;
    const T *__restrict__ AL = F.var_alpha ? (const T *)Coef<T>::al(F) : x;
    const long fxrow = (long)(nx + 1) * (j + (long)ny * k), fyrow = (long)nx * (j + (long)(ny + 1) * k);
    fc[0] = gld(BX, fb ? fxrow + i : c);
    fc[1] = gld(BX, fb ? fxrow + i + 1 : c);
    fc[2] = gld(BY, fb ? fyrow + i : c);
    fc[3] = gld(BY, fb ? fyrow + i + nx : c);
    fc[4] = gld(BZ, fb ? i + (long)nx * j + nxy * k : c);
    fc[5] = gld(BZ, fb ? i + (long)nx * j + nxy * (k + 1) : c);
    const T alv = gld(AL, c);
    if (!fb)
        for (int f = 0; f < 6; f++) fc[f] = (T)F.beta_c;
    const T al = F.var_alpha ? alv : (T)F.alpha_c;
    T dg, of;
    double lf;
    row_terms_fc<T>(F, i, j, k, nb, fc, al, dg, of, lf);
    if (F.lift) bv = (T)((double)bv + lf);
    return bv - (dg * xc - of);
}

template <typename T>
__device__ __forceinline__ void restrict_cell_fc(const LevDesc &F, const LevDesc &C, int cc, int I, int J, int K) {
    const T *x = (const T *)F.x;
    T r[8];
#pragma unroll
    for (int q = 0; q < 8; q++) r[q] = residual_fc<T>(F, x, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2));
    T s = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) s += r[q];
    gst((T *)C.b, cc, (T)0.125 * s);
    gst((T *)C.x, cc, (T)0);
}

template <typename T>
__device__ __forceinline__ void prolong_cell(const LevDesc &F, const LevDesc &C, int c, int i, int j, int k) {
    if (F.has_mask && !gld(F.mask, c)) return;
    int cc = (i >> 1) + C.nx * (j >> 1) + C.nxy * (k >> 1);
    const long fp = F.rb ? cell_pos(F, i, j, k) : (long)c;
    gst((T *)F.x, fp, gld((T *)F.x, fp) + gld((const T *)C.x, cc));
}

// ------------------------------------------------------------ grid kernels
// Cells (or row pairs) per thread in each tile of the persistent loops.
constexpr int kGsrbU = 1;       // GSRB: 256 row pairs (512 cells) per tile
constexpr int kRestrictU = 1;   // restriction: 256 coarse cells per tile
constexpr int kProlongU = 2;    // prolongation: 512 fine cells per tile
constexpr int kNormU = 4;       // norms, prep, refinement update: 1024 cells per tile

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gsrb(const LevDesc *__restrict__ descs, Plan pl, int colour,
                                                 const ProbState *__restrict__ st) {
    for_tiles(pl, [&](int d, int lt, int) {
        const LevDesc L = descs[pl.ids[d]];
        if (!gld(&st[L.prob].active, 0)) return;
        if ((L.nx & 1) == 0) {
            // one thread per pair (2m, 2m+1) of a row; exactly one has the colour
            for (int u = 0; u < kGsrbU; u++) {
                int c0 = 2 * ((lt * kGsrbU + u) * kBlock + (int)threadIdx.x);
                if (c0 >= L.ncell) break;
                int i, j, k;
                cell_ijk(L, c0, i, j, k);
                int off = ((i + j + k) & 1) != colour;
                gs_update<T>(L, c0 + off, i + off, j, k);
            }
        } else {
            for (int u = 0; u < kGsrbU; u++) {
                int c = (lt * kGsrbU + u) * kBlock + threadIdx.x;
                if (c >= L.ncell) break;
                int i, j, k;
                cell_ijk(L, c, i, j, k);
                if (((i + j + k) & 1) == colour) gs_update<T>(L, c, i, j, k);
            }
        }
    });
}

// plan over COARSE descriptors; fine = descs[id - 1]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(const LevDesc *__restrict__ descs, Plan pl,
                                                     const ProbState *__restrict__ st, int flip) {
    for_tiles(pl, [&](int d, int lt, int) {
        int id = pl.ids[d];
        const LevDesc C = descs[id];
        if (!gld(&st[C.prob].active, 0)) return;
        LevDesc F = descs[id - 1];
        if (flip) F.x = F.x2;      // the fine iterate is in the alternate buffer
        const bool uni = !F.var_beta && !F.var_alpha && !F.has_mask;
        for (int u = 0; u < kRestrictU; u++) {
            int cc = (lt * kRestrictU + u) * kBlock + threadIdx.x;
            if (cc >= C.ncell) break;
            int I, J, K;
            cell_ijk(C, cc, I, J, K);
            if (uni) restrict_cell_uni<T>(F, C, cc, I, J, K);
            else if (!F.has_mask && !F.rb && !C.has_mask) restrict_cell_fc<T>(F, C, cc, I, J, K);
            else restrict_cell<T>(F, C, cc, I, J, K);
        }
    });
}

// plan over FINE descriptors; coarse = descs[id + 1]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(const LevDesc *__restrict__ descs, Plan pl,
                                                    const ProbState *__restrict__ st, int flip) {
    for_tiles(pl, [&](int d, int lt, int) {
        int id = pl.ids[d];
        LevDesc F = descs[id];
        if (flip) F.x = F.x2;
        if (!gld(&st[F.prob].active, 0)) return;
        const LevDesc C = descs[id + 1];
        for (int u = 0; u < kProlongU; u++) {
            int c = (lt * kProlongU + u) * kBlock + threadIdx.x;
            if (c >= F.ncell) break;
            int i, j, k;
            cell_ijk(F, c, i, j, k);
            prolong_cell<T>(F, C, c, i, j, k);
        }
    });
}

// Sum of squares of the lifted right-hand side (mode 0) or of the FP64
// residual (mode 1) per tile of the finest level; mode 2 additionally
// stores the residual rounded to FP32 into the FP32 hierarchy's finest
// right-hand side and clears its unknown (iterative refinement).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_norm(const LevDesc *__restrict__ d64, const LevDesc *__restrict__ d32,
                                                 Plan pl, double *__restrict__ partials,
                                                 const ProbState *__restrict__ st, int check_active,
                                                 double *__restrict__ partials_b) {
    __shared__ double lds[kBlock / 64];
    for_tiles(pl, [&](int d, int lt, int t) {
        int id = pl.ids[d];
        const LevDesc L = d64[id];
        if (check_active && !gld(&st[L.prob].active, 0)) return;
        double v = 0.0, vb = 0.0;
        for (int u = 0; u < kNormU; u++) {
            int c = (lt * kNormU + u) * kBlock + threadIdx.x;
            if (c >= L.ncell) break;
            int i, j, k;
            cell_ijk(L, c, i, j, k);
            bool valid = !(L.has_mask && !gld(L.mask, c));
            double r;
            if (MODE == 0) r = valid ? load_b<double>(L, c, i, j, k) : 0.0;
            else r = residual_at<double>(L, c, i, j, k);
            v += r * r;
            if (MODE != 0 && partials_b) {
                const double bv = valid ? load_b<double>(L, c, i, j, k) : 0.0;
                vb += bv * bv;
            }
            if (MODE == 2) {
                const LevDesc &E = d32[id];
                gst((float *)E.b, c, (float)r);
                gst((float *)E.x, c, 0.0f);
            }
        }
        double s = block_sum(v, lds);
        if (threadIdx.x == 0) gst(partials, t, s);
        if (MODE != 0 && partials_b) {
            const double sb = block_sum(vb, lds);
            if (threadIdx.x == 0) gst(partials_b, t, sb);
        }
    });
}

// x = 0 on covered cells, on problems whose right-hand side vanishes, and
// everywhere for a zero initial guess.  when = 0: before ||b|| is known
// (zero guess and covered cells only); 1: after it, on the problems whose
// ||b|| is 0 only.
__global__ void __launch_bounds__(kBlock) k_prep(const LevDesc *__restrict__ d64, Plan pl,
                                                 const ProbState *__restrict__ st, int zero_guess, int when) {
    for_tiles(pl, [&](int d, int lt, int) {
        const LevDesc &L = d64[pl.ids[d]];
        const bool b0 = gld(&st[L.prob].bnorm, 0) == 0.0;
        if (when == 1 && !b0) return;
        const bool all = when == 1 || zero_guess;
        if (!all && !L.has_mask) return;
        for (int u = 0; u < kNormU; u++) {
            int c = (lt * kNormU + u) * kBlock + threadIdx.x;
            if (c >= L.ncell) break;
            if (all || !gld(L.mask, c)) gst((double *)L.x, c, 0.0);
        }
    });
}

// x = 0 on the problems whose ||b|| is 0, once ||b|| is known: one
// workgroup per problem, which returns at once in the common case
__global__ void __launch_bounds__(kBlock) k_zero_b0(const LevDesc *__restrict__ d64, Plan pl, const ProbState *__restrict__ st) {
    const LevDesc &L = d64[pl.ids[blockIdx.x]];
    if (gld(&st[L.prob].bnorm, 0) != 0.0) return;
    for (long c = threadIdx.x; c < L.ncell; c += blockDim.x) gst((double *)L.x, c, 0.0);
}

// x64 += e32 after the inner FP32 cycles of an outer refinement step.
__global__ void __launch_bounds__(kBlock) k_ir_update(const LevDesc *__restrict__ d64, const LevDesc *__restrict__ d32,
                                                      Plan pl, const ProbState *__restrict__ st) {
    for_tiles(pl, [&](int d, int lt, int) {
        int id = pl.ids[d];
        const LevDesc &L = d64[id];
        if (!gld(&st[L.prob].active, 0)) return;
        const float *e = (const float *)d32[id].x;
        double *x = (double *)L.x;
        for (int u = 0; u < kNormU; u++) {
            int c = (lt * kNormU + u) * kBlock + threadIdx.x;
            if (c >= L.ncell) break;
            gst(x, c, gld(x, c) + (double)gld(e, c));
        }
    });
}

// ------------------------------------------------ 2.5D LDS-tiled stencils
// A workgroup owns a 32 x 16 tile of x-y planes and marches kz planes in z.
// Each thread holds one row pair (i, i+1) in registers for planes k-1, k,
// k+1 (wide loads); the x-y neighbours of plane k come from an LDS copy of
// the tile with a one-cell halo.  Every element is fetched from memory once
// per pass (plus the halo).  Needs an even nx (row pairs).

typedef double PairD __attribute__((ext_vector_type(2)));
typedef float PairF __attribute__((ext_vector_type(2)));
template <typename T> struct Pair;
template <> struct Pair<double> { using V = PairD; };
template <> struct Pair<float> { using V = PairF; };

// value at (i, j, k) with periodic wrap; 0 across a non-periodic face
template <typename T>
__device__ __forceinline__ T ld_wrap(const LevDesc &L, const T *__restrict__ X, int i, int j, int k) {
    if (i < 0 || i >= L.nx) { if (L.kind[0] != VD_BC_PERIODIC) return (T)0; i = i < 0 ? i + L.nx : i - L.nx; }
    if (j < 0 || j >= L.ny) { if (L.kind[2] != VD_BC_PERIODIC) return (T)0; j = j < 0 ? j + L.ny : j - L.ny; }
    if (k < 0 || k >= L.nz) { if (L.kind[4] != VD_BC_PERIODIC) return (T)0; k = k < 0 ? k + L.nz : k - L.nz; }
    return gld(X, i + (long)L.nx * j + (long)L.nxy * k);
}

// the two values of row pair (ia, ia+1) of row j in plane k: a wide load
// for pairs inside the domain, wrapped (or zero) values otherwise
template <typename T>
__device__ __forceinline__ void ld_slot(const LevDesc &L, const T *__restrict__ X, int ia, int j, int k, bool own, T &a,
                                        T &b) {
    if (!own) {
        a = ld_wrap<T>(L, X, ia, j, k);
        b = ld_wrap<T>(L, X, ia + 1, j, k);
        return;
    }
    if (k < 0 || k >= L.nz) {
        if (L.kind[4] != VD_BC_PERIODIC) { a = b = (T)0; return; }
        k = k < 0 ? k + L.nz : k - L.nz;
    }
    typename Pair<T>::V v = *(const VD_GAS typename Pair<T>::V *)(X + ia + (long)L.nx * j + (long)L.nxy * k);
    a = v.x;
    b = v.y;
}

// halo value of plane k loaded by thread tid (< 96): x-halo columns for
// tid < 32, y-halo rows otherwise
template <typename T>
__device__ __forceinline__ T ld_halo(const LevDesc &L, const T *__restrict__ X, int tid, int i0, int j0, int k) {
    if (tid < 2 * kT25Y) {
        const int rr = tid & (kT25Y - 1), side = tid / kT25Y;
        return ld_wrap<T>(L, X, side ? i0 + kT25X : i0 - 1, j0 + rr, k);
    }
    const int q = tid - 2 * kT25Y, cc = q & (kT25X - 1), side = q / kT25X;
    return ld_wrap<T>(L, X, i0 + cc, side ? j0 + kT25Y : j0 - 1, k);
}



// Zeros read in place of positions that are not cells: a load whose
// position lies outside a non-periodic face (or past the tile) takes its
// address here, so the loaded value needs no masking afterwards.
__device__ double g_zero4[4];

// MODE 0: one Gauss-Seidel colour pass (in place); MODE 1: FP64 residual
// norm partials; MODE 2: same, also storing the FP32 residual and, unless
// colour is 1, clearing the FP32 unknown (iterative refinement).  MODE 4:
// the first colour pass of a correction solve, from a zero iterate (no
// loads of x; the pair is stored with the other colour 0).  MODE 5: the
// last colour pass of a correction solve, which adds the final correction
// pair to the FP64 unknown (d32 then holds the FP64 descriptors) instead of
// storing it.  Software-pipelined: while plane k is computed, plane k+2's
// pair, plane k+1's halo and b (and in MODE 5 its FP64 pair) are in flight;
// the LDS tile is double-buffered so one barrier per plane suffices.  The
// plane loop is unrolled by four, one named register set per plane of the
// z window, so no register is copied while its load is in flight, and
// positions that are not cells read from g_zero4 (no masking after the
// load); the face coefficients of a plane are issued before its barrier.
// one tile t of the pass (the body of k_st25 and of its persistent form)
template <typename T, int MODE, bool UNIONLY>
__device__ __forceinline__ void st25_tile(int t, T (*xs)[(kT25Y + 2) * kT25W], double *red, const LevDesc *__restrict__ descs,
                                          const LevDesc *__restrict__ d32, const Plan &pl, int kz, int colour,
                                          double *__restrict__ partials, const ProbState *__restrict__ st,
                                          int check_active, double *__restrict__ partials_b) {
    const int d = plan_find(pl, t);
    const int id = pl.ids[d];
    const LevDesc L = descs[id];
    constexpr bool PASS = MODE == 0 || MODE == 4 || MODE == 5;
    if ((PASS || check_active) && !gld(&st[L.prob].active, 0)) return;
    const int lt = t - pl.prefix[d];
    const int slot = pl.gbase ? pl.gbase[d] + lt : t;    // partial slot of this tile
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const Tile25 T25 = tile25(lt, nx, ny, nz, kz);
    const int k0 = T25.k0, k1 = T25.k1;
    const int tid = threadIdx.x;
    const int tp = tid & 15, r = tid >> 4;
    float *__restrict__ Eb = MODE == 2 ? (float *)d32[id].b : nullptr;
    float *__restrict__ Ex = MODE == 2 ? (float *)d32[id].x : nullptr;
    const bool rbE = MODE == 2 && d32[id].rb;
    const int hslot = halo_slot(tid);
    T *__restrict__ X = (T *)L.x;
    const T *__restrict__ B = (const T *)L.b;
    // Branch-free loads: every thread issues the same loads on every plane
    // (wrapped or clamped addresses, zeroed where the position is not a
    // cell), so the compiler can count outstanding loads and the look-ahead
    // really overlaps with the computation.  x / y parts are fixed per thread.
    const bool px = L.kind[0] == VD_BC_PERIODIC, py = L.kind[2] == VD_BC_PERIODIC, pz = L.kind[4] == VD_BC_PERIODIC;
    const Thr25 H = thr25(T25, tid, nx, nx, ny, px, py, 0, 0);
    const int ia = H.ua, j = H.j;
    const bool own = H.own, halo_thread = H.halo;
    const bool okxy = H.okp, okh = H.okh;
    const long pair_off = H.pair_off, b_off = H.b_off, h_off = H.h_off;
    const long nxy = L.nxy;
    const T *zero = (const T *)g_zero4;
    using PV = typename Pair<T>::V;
    struct PT {
        T a, b;
    };
    auto ld_pair = [&](int kk) -> PT {
        if constexpr (MODE == 4) return PT{(T)0, (T)0};
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const T *p = (okxy && okz) ? X + (pair_off + nxy * kw) : zero;
        const PV v = *(const VD_GAS PV *)p;
        return PT{v.x, v.y};
    };
    auto ld_h = [&](int kk) -> T {
        if constexpr (MODE == 4) return (T)0;
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const T *p = (okh && okz) ? X + (h_off + nxy * kw) : zero;
        return *(const VD_GAS T *)p;
    };
    auto ld_b = [&](int kk) -> PT {
        const T *p = (own && kk < k1) ? B + (b_off + nxy * kk) : zero;
        const PV v = *(const VD_GAS PV *)p;
        return PT{v.x, v.y};
    };
    // MODE 5: the FP64 unknown pair of plane kk
    auto ld_x64 = [&](int kk) -> PairD {
        if constexpr (MODE != 5) return PairD{};
        const double *p = (own && kk < k1) ? (const double *)d32[id].x + (b_off + nxy * kk) : g_zero4;
        return *(const VD_GAS PairD *)p;
    };
    const long rowoff = (long)nx * j;
    double v = 0.0, vb = 0.0;
    // the plane loop, instantiated per level kind:
    // variant 1: uniform coefficients, no mask (nothing loaded inside the
    // pipeline); 2: coefficient arrays, no mask (faces and alpha of the pair
    // loaded together, from clamped addresses); 0: general
    auto march = [&](auto var_tag) {
    constexpr int VAR = decltype(var_tag)::value;
    constexpr bool UNI = VAR == 1;
    const long jc = min(j, ny - 1);
    const int ic = min(ia, nx - 2);
    const T *__restrict__ BX = VAR == 2 && L.var_beta ? (const T *)Coef<T>::bx(L) : X;
    const T *__restrict__ BY = VAR == 2 && L.var_beta ? (const T *)Coef<T>::by(L) : X;
    const T *__restrict__ BZ = VAR == 2 && L.var_beta ? (const T *)Coef<T>::bz(L) : X;
    const T *__restrict__ AL = VAR == 2 && L.var_alpha ? (const T *)Coef<T>::al(L) : X;
    // plane k: xm, xc, xp the pairs of planes k-1, k, k+1, xq receives
    // plane k+2; hc / bcur / qc plane k's halo element, right-hand side and
    // (MODE 5) FP64 pair, hn / bn / qn receive plane k+1's
    auto plane = [&](int k, const PT &xm, const PT &xc, const PT &xp, PT &xq, const T &hc, T &hn, const PT &bcur,
                     PT &bn, const PairD &qc, PairD &qn) {
        // coefficient arrays of this plane for the pair (variant 2): all
        // issued together from clamped addresses, before the barrier
        T fx0 = 0, fx1 = 0, fx2 = 0;
        PV fyl{}, fyh{}, fzl{}, fzh{}, alp{};
        if constexpr (VAR == 2) {
            const long fxrow = (long)(nx + 1) * (jc + (long)ny * k);
            const long fyrow = (long)nx * (jc + (long)(ny + 1) * k);
            const long fz = (long)nx * jc + ic;
            const bool fb = L.var_beta;
            fx0 = gld(BX, fb ? fxrow + ic : pair_off);
            fx1 = gld(BX, fb ? fxrow + ic + 1 : pair_off);
            fx2 = gld(BX, fb ? fxrow + ic + 2 : pair_off);
            fyl = *(const VD_GAS PV *)(BY + (fb ? fyrow + ic : pair_off));
            fyh = *(const VD_GAS PV *)(BY + (fb ? fyrow + nx + ic : pair_off));
            fzl = *(const VD_GAS PV *)(BZ + (fb ? fz + nxy * k : pair_off));
            fzh = *(const VD_GAS PV *)(BZ + (fb ? fz + nxy * (k + 1) : pair_off));
            alp = *(const VD_GAS PV *)(AL + (L.var_alpha ? ic + (long)nx * jc + nxy * k : pair_off));
        }
        T *buf = xs[k & 1];
        buf[(r + 1) * kT25W + 2 * tp + 1] = xc.a;
        buf[(r + 1) * kT25W + 2 * tp + 2] = xc.b;
        if (halo_thread) buf[hslot] = hc;
        // look-ahead for the next planes
        xq = ld_pair(k + 2);
        hn = ld_h(k + 1);
        bn = ld_b(k + 1);
        qn = ld_x64(k + 1);
        __syncthreads();
        if (!own) return;
        // colour pass: the pair is stored whole (the other cell with its
        // unchanged value, which no other thread writes in this pass), so
        // every cache line is written in full
        T out0 = xc.a, out1 = xc.b;
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const int i = ia + q;
            if (PASS && ((i + j + k) & 1) != colour) continue;
            const int c = i + nx * j + L.nxy * k;
            const bool valid = VAR != 0 || !(L.has_mask && !gld(L.mask, c));
            if (PASS && !valid) continue;
            T nbv[6];
            nbv[0] = q == 0 ? buf[(r + 1) * kT25W + 2 * tp] : xc.a;
            nbv[1] = q == 0 ? xc.b : buf[(r + 1) * kT25W + 2 * tp + 3];
            nbv[2] = buf[r * kT25W + 2 * tp + 1 + q];
            nbv[3] = buf[(r + 2) * kT25W + 2 * tp + 1 + q];
            nbv[4] = q == 0 ? xm.a : xm.b;
            nbv[5] = q == 0 ? xp.a : xp.b;
            T dg, of;
            T b = q == 0 ? bcur.a : bcur.b;
            if constexpr (VAR == 2) {
                T fc[6];
                fc[0] = q == 0 ? fx0 : fx1;
                fc[1] = q == 0 ? fx1 : fx2;
                fc[2] = q == 0 ? fyl.x : fyl.y;
                fc[3] = q == 0 ? fyh.x : fyh.y;
                fc[4] = q == 0 ? fzl.x : fzl.y;
                fc[5] = q == 0 ? fzh.x : fzh.y;
                if (!L.var_beta) for (int f = 0; f < 6; f++) fc[f] = (T)L.beta_c;
                const T al = L.var_alpha ? (q == 0 ? alp.x : alp.y) : (T)L.alpha_c;
                double lf;
                row_terms_fc<T>(L, i, j, k, nbv, fc, al, dg, of, lf);
                if (L.lift) b = (T)((double)b + lf);
            } else {
                if constexpr (UNI) row_terms_uni<T>(L, i, j, k, nbv, dg, of);
                else row_terms_nb<T>(L, i, j, k, c, nbv, dg, of);
                if (L.lift) b = (T)((double)b + (UNI ? lift_term_uni(L, i, j, k) : lift_term(L, i, j, k)));
            }
            if (PASS) {
                if (q == 0) out0 = (b + of) / dg;
                else out1 = (b + of) / dg;
            } else {
                const T xv = q == 0 ? xc.a : xc.b;
                const double rv = valid ? (double)(b - (dg * xv - of)) : 0.0;
                v += rv * rv;
                if (partials_b && valid) vb += (double)b * (double)b;
                if (MODE == 2) {
                    const long ce = rbE ? cell_pos(d32[id], i, j, k) : (long)c;
                    gst(Eb, ce, (float)rv);
                    if (colour != 1) gst(Ex, ce, 0.0f);
                }
            }
        }
        if (MODE == 0 || MODE == 4) {
            PV pv;
            pv.x = out0;
            pv.y = out1;
            *(VD_GAS PV *)(X + ia + rowoff + (long)L.nxy * k) = pv;
        } else if (MODE == 5) {
            PairD x64v = qc;
            x64v.x = x64v.x + (double)out0;
            x64v.y = x64v.y + (double)out1;
            *(VD_GAS PairD *)((double *)d32[id].x + ia + rowoff + (long)L.nxy * k) = x64v;
        }
    };
    PT P0 = ld_pair(k0 - 1), P1 = ld_pair(k0), P2 = ld_pair(k0 + 1), P3;
    T H0 = ld_h(k0), H1;
    PT B0 = ld_b(k0), B1;
    PairD Q0 = ld_x64(k0), Q1;
    for (int k = k0; k < k1; k += 4) {
        plane(k, P0, P1, P2, P3, H0, H1, B0, B1, Q0, Q1);
        if (k + 1 >= k1) break;
        plane(k + 1, P1, P2, P3, P0, H1, H0, B1, B0, Q1, Q0);
        if (k + 2 >= k1) break;
        plane(k + 2, P2, P3, P0, P1, H0, H1, B0, B1, Q0, Q1);
        if (k + 3 >= k1) break;
        plane(k + 3, P3, P0, P1, P2, H1, H0, B1, B0, Q1, Q0);
    }
    };
    if constexpr (UNIONLY) {
        march(std::integral_constant<int, 1>{});   // every problem of the plan has uniform coefficients
    } else {
        if (!L.var_beta && !L.var_alpha && !L.has_mask) march(std::integral_constant<int, 1>{});
        else if (!L.has_mask) march(std::integral_constant<int, 2>{});
        else march(std::integral_constant<int, 0>{});
    }
    if (!PASS) {
        const double sum = block_sum(v, red);
        if (tid == 0) gst(partials, slot, sum);
        if (partials_b) {
            const double sb = block_sum(vb, red);
            if (tid == 0) gst(partials_b, slot, sb);
        }
    }
}

template <typename T, int MODE, bool UNIONLY = false>
__global__ void __launch_bounds__(kBlock) k_st25(const LevDesc *__restrict__ descs, const LevDesc *__restrict__ d32, Plan pl,
                                                 int kz, int colour, double *__restrict__ partials,
                                                 const ProbState *__restrict__ st, int check_active,
                                                 double *__restrict__ partials_b) {
    __shared__ T xs[2][(kT25Y + 2) * kT25W];
    __shared__ double red[kBlock / 64];
    const int t = xcd_tile(pl.ntiles);
    if (t >= pl.ntiles) return;
    st25_tile<T, MODE, UNIONLY>(t, xs, red, descs, d32, pl, kz, colour, partials, st, check_active, partials_b);
}

// Persistent colour pass (VD_MG_PERSISTENT): a grid of resident workgroups
// (a multiple of 8) walks the plan's (problem, tile) items; workgroup b
// works in XCD b % 8's contiguous eighth of the tiles, striding by the
// workgroups of its XCD; a barrier separates consecutive tiles (they reuse
// the LDS buffers).  Every workgroup exits after its last item.
template <typename T, bool UNIONLY>
__global__ void __launch_bounds__(kBlock) k_st25p(const LevDesc *__restrict__ descs, Plan pl, int kz, int colour,
                                                  const ProbState *__restrict__ st) {
    __shared__ T xs[2][(kT25Y + 2) * kT25W];
    __shared__ double red[kBlock / 64];
    const int chunk = (pl.ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, per_xcd = gridDim.x >> 3;
    const int end = min(pl.ntiles, (x + 1) * chunk);
    for (int t = x * chunk + (int)(blockIdx.x >> 3); t < end; t += per_xcd) {
        __syncthreads();
        st25_tile<T, 0, UNIONLY>(t, xs, red, descs, nullptr, pl, kz, colour, nullptr, st, 1, nullptr);
    }
}

// --------------------------------- FP64 residual check, uniform levels (LDS)
// The residual checks of k_st25 (modes 1 and 2) for levels with uniform
// coefficients and no mask, with the plane loop unrolled by four: one named
// register set per plane of the z window (k-1 .. k+2), so no register is
// copied while its load is in flight, and positions that are not cells read
// from g_zero4 (address select) instead of being masked after the load.
// The x-y part of each cell's diagonal and Dirichlet lifting is summed once
// per thread (the same additions in the same order as row_terms_uni /
// lift_term_uni, completed per plane by the z faces), and neighbours outside
// a non-periodic face, which read as zero, enter the off-diagonal sum with
// their weight (a zero term leaves the sum's bits unchanged).  Residuals,
// partial sums and the stored FP32 residual are bit-identical to k_st25's.
// MODE 1: partial sums of r^2 (and of b^2 when partials_b is given); MODE 2:
// also r rounded to FP32 into the FP32 hierarchy's finest right-hand side
// (either row layout) and, unless keep_e, its unknown cleared.
struct Pr {
    double a, b;
};

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_res25u(const LevDesc *__restrict__ descs, const LevDesc *__restrict__ d32,
                                                   Plan pl, int kz, int keep_e, double *__restrict__ partials,
                                                   const ProbState *__restrict__ st, int check_active,
                                                   double *__restrict__ partials_b) {
    __shared__ double xs[2][(kT25Y + 2) * kT25W];
    __shared__ double red[kBlock / 64];
    const int t = xcd_tile(pl.ntiles);
    if (t >= pl.ntiles) return;
    const int d = plan_find(pl, t);
    const int id = pl.ids[d];
    const LevDesc L = descs[id];
    if (check_active && !gld(&st[L.prob].active, 0)) return;
    const int lt = t - pl.prefix[d];
    const int slot = pl.gbase ? pl.gbase[d] + lt : t;
    const int nx = L.nx, ny = L.ny, nz = L.nz, nxy = L.nxy;
    const Tile25 T25 = tile25(lt, nx, ny, nz, kz);
    const int k0 = T25.k0, k1 = T25.k1;
    const int tid = threadIdx.x;
    const int tp = tid & 15, r = tid >> 4;
    const bool px = L.kind[0] == VD_BC_PERIODIC, py = L.kind[2] == VD_BC_PERIODIC, pz = L.kind[4] == VD_BC_PERIODIC;
    const Thr25 H = thr25(T25, tid, nx, nx, ny, px, py, 0, 0);
    const int ia = H.ua, j = H.j;
    const bool own = H.own, halo_thread = H.halo, okxy = H.okp, okh = H.okh;
    const int pair_off = (int)H.pair_off, b_off = (int)H.b_off, h_off = (int)H.h_off;
    const int hslot = halo_slot(tid);
    const double *__restrict__ X = (const double *)L.x;
    const double *__restrict__ B = (const double *)L.b;
    const double *zero = g_zero4;
    const double bc = L.beta_c;
    const double cfx = bc * L.idx2, cfy = bc * L.idy2, cfz = bc * L.idz2;
    // x-y prefixes of the diagonal and of the lifting, per cell of the pair
    double dgxy[2], lfxy[2];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int i = ia + q;
        const bool in[4] = {i > 0, i < nx - 1, j > 0, j < ny - 1};
        double dg = L.alpha_c, lf = 0.0;
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const double cf = f < 2 ? cfx : cfy;
            const int kd = L.kind[f];
            if (in[f] || kd == VD_BC_PERIODIC) dg += cf;
            else if (kd == VD_BC_DIRICHLET) dg += 2.0 * cf;
        }
        if (i == 0 && L.kind[0] == VD_BC_DIRICHLET) lf += 2.0 * bc * L.gval[0] * L.idx2;
        if (i == nx - 1 && L.kind[1] == VD_BC_DIRICHLET) lf += 2.0 * bc * L.gval[1] * L.idx2;
        if (j == 0 && L.kind[2] == VD_BC_DIRICHLET) lf += 2.0 * bc * L.gval[2] * L.idy2;
        if (j == ny - 1 && L.kind[3] == VD_BC_DIRICHLET) lf += 2.0 * bc * L.gval[3] * L.idy2;
        dgxy[q] = dg;
        lfxy[q] = lf;
    }
    const bool lift = L.lift;
    const double lz0 = 2.0 * bc * L.gval[4] * L.idz2, lz1 = 2.0 * bc * L.gval[5] * L.idz2;
    const bool dz0 = L.kind[4] == VD_BC_DIRICHLET, dz1 = L.kind[5] == VD_BC_DIRICHLET;
    float *__restrict__ Eb = MODE == 2 ? (float *)d32[id].b : nullptr;
    float *__restrict__ Ex = MODE == 2 ? (float *)d32[id].x : nullptr;
    const bool rbE = MODE == 2 && d32[id].rb;
    const int nh = nx >> 1;
    auto ld_pair = [&](int kk) -> Pr {
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const double *p = (okxy && okz) ? X + (pair_off + nxy * kw) : zero;
        const PairD v = *(const VD_GAS PairD *)p;
        return Pr{v.x, v.y};
    };
    auto ld_h = [&](int kk) -> double {
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const double *p = (okh && okz) ? X + (h_off + nxy * kw) : zero;
        return *(const VD_GAS double *)p;
    };
    auto ld_b = [&](int kk) -> Pr {
        const double *p = (own && kk < k1) ? B + (b_off + nxy * kk) : zero;
        const PairD v = *(const VD_GAS PairD *)p;
        return Pr{v.x, v.y};
    };
    double v = 0.0, vb = 0.0;
    const int lc = (r + 1) * kT25W + 2 * tp + 1;
    // plane k: xm, xc, xp the pairs of planes k-1, k, k+1 (loaded), xq
    // receives plane k+2; hc / bcur plane k's halo element and right-hand
    // side, hn / bn receive plane k+1's
    auto plane = [&](int k, const Pr &xm, const Pr &xc, const Pr &xp, Pr &xq, const double &hc, double &hn,
                     const Pr &bcur, Pr &bn) {
        double *buf = xs[k & 1];
        buf[lc] = xc.a;
        buf[lc + 1] = xc.b;
        if (halo_thread) buf[hslot] = hc;
        xq = ld_pair(k + 2);
        hn = ld_h(k + 1);
        bn = ld_b(k + 1);
        __syncthreads();
        if (!own) return;
        // z faces of this plane: diagonal and lifting terms
        const double az0 = (k > 0 || pz) ? cfz : (dz0 ? 2.0 * cfz : 0.0);
        const double az1 = (k < nz - 1 || pz) ? cfz : (dz1 ? 2.0 * cfz : 0.0);
        const double lzk0 = (k == 0 && dz0) ? lz0 : 0.0, lzk1 = (k == nz - 1 && dz1) ? lz1 : 0.0;
        const double wl = buf[lc - 1], wr = buf[lc + 2];
        double rv[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double xv = q == 0 ? xc.a : xc.b;
            double of = 0.0;
            of += cfx * (q == 0 ? wl : xc.a);
            of += cfx * (q == 0 ? xc.b : wr);
            of += cfy * buf[lc + q - kT25W];
            of += cfy * buf[lc + q + kT25W];
            of += cfz * (q == 0 ? xm.a : xm.b);
            of += cfz * (q == 0 ? xp.a : xp.b);
            double dg = dgxy[q];
            dg += az0;
            dg += az1;
            double b = q == 0 ? bcur.a : bcur.b;
            if (lift) {
                double lf = lfxy[q];
                lf += lzk0;
                lf += lzk1;
                b = b + lf;
            }
            rv[q] = b - (dg * xv - of);
            v += rv[q] * rv[q];
            if (partials_b) vb += b * b;
        }
        if (MODE == 2) {
            const int row = nx * j + nxy * k;
            if (rbE) {
                // cell ia is red ((i+j+k) even) when j + k is even; the
                // pair's cells sit at position ia/2 of the two halves
                const int h0 = ((j + k) & 1) ? nh : 0;
                gst(Eb, row + h0 + (ia >> 1), (float)rv[0]);
                gst(Eb, row + (nh - h0) + (ia >> 1), (float)rv[1]);
                if (!keep_e) {
                    gst(Ex, row + h0 + (ia >> 1), 0.0f);
                    gst(Ex, row + (nh - h0) + (ia >> 1), 0.0f);
                }
            } else {
                PairF rp;
                rp.x = (float)rv[0];
                rp.y = (float)rv[1];
                *(VD_GAS PairF *)(Eb + row + ia) = rp;
                if (!keep_e) *(VD_GAS PairF *)(Ex + row + ia) = PairF{0.0f, 0.0f};
            }
        }
    };
    Pr P0 = ld_pair(k0 - 1), P1 = ld_pair(k0), P2 = ld_pair(k0 + 1), P3;
    double H0 = ld_h(k0), H1;
    Pr B0 = ld_b(k0), B1;
    for (int k = k0; k < k1; k += 4) {
        plane(k, P0, P1, P2, P3, H0, H1, B0, B1);
        if (k + 1 >= k1) break;
        plane(k + 1, P1, P2, P3, P0, H1, H0, B1, B0);
        if (k + 2 >= k1) break;
        plane(k + 2, P2, P3, P0, P1, H0, H1, B0, B1);
        if (k + 3 >= k1) break;
        plane(k + 3, P3, P0, P1, P2, H1, H0, B1, B0);
    }
    const double sum = block_sum(v, red);
    if (tid == 0) gst(partials, slot, sum);
    if (partials_b) {
        const double sb = block_sum(vb, red);
        if (tid == 0) gst(partials_b, slot, sb);
    }
}

// ---------------------------------------- FP64 residual checks, direct form
// The residual checks of k_st25 (modes 1 and 2) for levels with face and/or
// cell coefficient arrays and no mask (the electrons' variable diffusion, a
// variable permittivity), with no LDS and no barrier: a thread owns the row
// pair (i, i+1) of row j
// in a 32 x 16 tile and marches the tile's KZ planes (fully unrolled, so no
// register is copied while its load is in flight); the pair's x-y
// neighbours are loaded straight from memory (the cache serves the re-reads
// of the neighbouring threads and tiles) and its z neighbours are carried in
// registers.  With no barrier each wavefront runs ahead on its own loads,
// which keeps far more bytes in flight than the LDS-staged march.  Tiles and
// partial slots are those of the 2.5D plans.
//
// Each row is row_terms_fc's from the loaded faces (the arithmetic of
// k_st25's face-coefficient march), so residuals, partial sums and the
// stored FP32 residual are bit-identical to k_st25's.  This form carries 88
// VGPRs against the march's 113 (five wavefronts per SIMD instead of four).  MODE 1: partial sums of
// r^2 (and of b^2 when partials_b is given); MODE 2: also r rounded to FP32
// into the FP32 hierarchy's finest right-hand side (either row layout) and,
// unless keep_e, its unknown cleared.
struct MaskPair {
    unsigned char x, y;   // validity of the cells of a pair (1 valid, 0 covered)
};

template <int MODE, int KZ, bool MASK = false>
__global__ void __launch_bounds__(kBlock) k_resd(const LevDesc *__restrict__ descs, const LevDesc *__restrict__ d32,
                                                 Plan pl, int keep_e, double *__restrict__ partials,
                                                 const ProbState *__restrict__ st, int check_active,
                                                 double *__restrict__ partials_b) {
    __shared__ double red[kBlock / 64];
    const int t = xcd_tile(pl.ntiles);
    if (t >= pl.ntiles) return;
    const int d = plan_find(pl, t);
    const int id = pl.ids[d];
    const LevDesc L = descs[id];
    if (check_active && !gld(&st[L.prob].active, 0)) return;
    const int lt = t - pl.prefix[d];
    const int slot = pl.gbase ? pl.gbase[d] + lt : t;
    const int nx = L.nx, ny = L.ny, nz = L.nz, nxy = L.nxy;
    const Tile25 T25 = tile25(lt, nx, ny, nz, KZ);
    const int k0 = T25.k0, k1 = T25.k1;
    const int tid = threadIdx.x;
    const int ia = T25.u0 + 2 * (tid & 15), j = T25.j0 + (tid >> 4);
    double v = 0.0, vb = 0.0;
    if (ia < nx && j < ny) {
        const bool px = L.kind[0] == VD_BC_PERIODIC, py = L.kind[2] == VD_BC_PERIODIC, pz = L.kind[4] == VD_BC_PERIODIC;
        bool okl, okr, oks, okn;
        const int il = wrap_idx(ia - 1, nx, px, okl), ir = wrap_idx(ia + 2, nx, px, okr);
        const int js = wrap_idx(j - 1, ny, py, oks), jn = wrap_idx(j + 1, ny, py, okn);
        const int oc = ia + nx * j, ol = il + nx * j, orr = ir + nx * j, os = ia + nx * js, on = ia + nx * jn;
        const double *__restrict__ X = (const double *)L.x;
        const double *__restrict__ B = (const double *)L.b;
        auto ldp = [&](int off) -> PairD { return *(const VD_GAS PairD *)(X + off); };
        // pair of plane kk (zero where the plane is not one of cells)
        auto zpair = [&](int kk) -> PairD {
            bool okz;
            const int kw = wrap_idx(kk, nz, pz, okz);
            const PairD q = ldp(oc + nxy * kw);
            return okz ? q : PairD{0.0, 0.0};
        };
        const double bc = L.beta_c;
        const bool lift = L.lift;
        // coefficient arrays: faces of the pair and its cell
        // coefficient, read from x's own addresses when absent
        const double *__restrict__ BX = L.var_beta ? L.bx : X;
        const double *__restrict__ BY = L.var_beta ? L.by : X;
        const double *__restrict__ BZ = L.var_beta ? L.bz : X;
        const double *__restrict__ AL = L.var_alpha ? L.alpha : X;
        float *__restrict__ Eb = MODE == 2 ? (float *)d32[id].b : nullptr;
        float *__restrict__ Ex = MODE == 2 ? (float *)d32[id].x : nullptr;
        const bool rbE = MODE == 2 && d32[id].rb;
        const int nh = nx >> 1;
        PairD xm = zpair(k0 - 1), xc = zpair(k0);
        // masked levels: validity of the pair's cells and of their six
        // neighbours (a covered neighbour is a homogeneous Dirichlet face:
        // its value reads as 0 and the diagonal gains the face coefficient
        // once more; a covered cell has no residual)
        // (a plan may mix masked and unmasked problems: only a problem
        // with a mask has a mask array)
        const bool mk = MASK && L.has_mask;
        const uint8_t *__restrict__ MK = mk ? L.mask : nullptr;
        auto mpair = [&](int off) -> MaskPair {
            const uint16_t v = *(const VD_GAS uint16_t *)(MK + off);
            return MaskPair{(unsigned char)(v & 0xFFu), (unsigned char)(v >> 8)};
        };
#pragma unroll
        for (int q = 0; q < KZ; q++) {
            const int k = k0 + q;
            if (k >= k1) break;
            const PairD xp = zpair(k + 1);
            const int pk = nxy * k;
            const double wl0 = gld(X, ol + pk), wr0 = gld(X, orr + pk);
            const PairD ys0 = ldp(os + pk), yn0 = ldp(on + pk);
            const PairD bv = __builtin_nontemporal_load((const VD_GAS PairD *)(B + oc + pk));
            MaskPair mo{1, 1}, ms{1, 1}, mn{1, 1}, mzm{1, 1}, mzp{1, 1};
            unsigned char ml = 1, mr = 1;
            bool okzm = true, okzp = true;
            if (MASK && mk) {
                mo = mpair(oc + pk);
                ml = okl ? MK[ol + pk] : (unsigned char)1;
                mr = okr ? MK[orr + pk] : (unsigned char)1;
                if (oks) ms = mpair(os + pk);
                if (okn) mn = mpair(on + pk);
                const int kwm = wrap_idx(k - 1, nz, pz, okzm), kwp = wrap_idx(k + 1, nz, pz, okzp);
                if (okzm) mzm = mpair(oc + nxy * kwm);
                if (okzp) mzp = mpair(oc + nxy * kwp);
            }
            const double wl = okl ? wl0 : 0.0, wr = okr ? wr0 : 0.0;
            const PairD ys = oks ? ys0 : PairD{0.0, 0.0}, yn = okn ? yn0 : PairD{0.0, 0.0};
            double rv[2];
            {
                const bool fb = L.var_beta;
                const int fxrow = (nx + 1) * (j + ny * k), fyrow = nx * (j + (ny + 1) * k);
                const double fx0 = gld(BX, fb ? fxrow + ia : oc), fx1 = gld(BX, fb ? fxrow + ia + 1 : oc),
                             fx2 = gld(BX, fb ? fxrow + ia + 2 : oc);
                const PairD fyl = *(const VD_GAS PairD *)(BY + (fb ? fyrow + ia : oc));
                const PairD fyh = *(const VD_GAS PairD *)(BY + (fb ? fyrow + nx + ia : oc));
                const PairD fzl = *(const VD_GAS PairD *)(BZ + (fb ? oc + pk : oc));
                const PairD fzh = *(const VD_GAS PairD *)(BZ + (fb ? oc + pk + nxy : oc));
                const PairD alp = *(const VD_GAS PairD *)(AL + (L.var_alpha ? oc + pk : oc));
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const int i = ia + c;
                    double nbv[6], fc[6];
                    nbv[0] = c == 0 ? wl : xc.x;
                    nbv[1] = c == 0 ? xc.y : wr;
                    nbv[2] = c == 0 ? ys.x : ys.y;
                    nbv[3] = c == 0 ? yn.x : yn.y;
                    nbv[4] = c == 0 ? xm.x : xm.y;
                    nbv[5] = c == 0 ? xp.x : xp.y;
                    fc[0] = c == 0 ? fx0 : fx1;
                    fc[1] = c == 0 ? fx1 : fx2;
                    fc[2] = c == 0 ? fyl.x : fyl.y;
                    fc[3] = c == 0 ? fyh.x : fyh.y;
                    fc[4] = c == 0 ? fzl.x : fzl.y;
                    fc[5] = c == 0 ? fzh.x : fzh.y;
                    if (!fb) for (int f = 0; f < 6; f++) fc[f] = bc;
                    const double al = L.var_alpha ? (c == 0 ? alp.x : alp.y) : L.alpha_c;
                    bool cov[6] = {false, false, false, false, false, false}, own_valid = true;
                    if (MASK && mk) {
                        own_valid = (c == 0 ? mo.x : mo.y) != 0;
                        cov[0] = (c == 0 ? (okl && !ml) : !mo.x);
                        cov[1] = (c == 0 ? !mo.y : (okr && !mr));
                        cov[2] = oks && !(c == 0 ? ms.x : ms.y);
                        cov[3] = okn && !(c == 0 ? mn.x : mn.y);
                        cov[4] = okzm && !(c == 0 ? mzm.x : mzm.y);
                        cov[5] = okzp && !(c == 0 ? mzp.x : mzp.y);
                        for (int f = 0; f < 6; f++)
                            if (cov[f]) nbv[f] = 0.0;
                    }
                    double dg, of, lf;
                    row_terms_fc<double>(L, i, j, k, nbv, fc, al, dg, of, lf);
                    if (MASK && mk) {
                        const double ih2[3] = {L.idx2, L.idy2, L.idz2};
                        for (int f = 0; f < 6; f++)
                            if (cov[f]) dg += fc[f] * ih2[f >> 1];
                    }
                    double b = c == 0 ? bv.x : bv.y;
                    if (lift) b = b + lf;
                    rv[c] = b - (dg * (c == 0 ? xc.x : xc.y) - of);
                    if (MASK && !own_valid) rv[c] = 0.0;
                    v += rv[c] * rv[c];
                    if (partials_b && own_valid) vb += b * b;
                }
            }
            if (MODE == 2) {
                const int row = nx * j + pk;
                if (rbE) {
                    // cell ia is red ((i+j+k) even) when j + k is even; the
                    // pair's cells sit at position ia/2 of the two halves
                    const int h0 = ((j + k) & 1) ? nh : 0;
                    __builtin_nontemporal_store((float)rv[0], (VD_GAS float *)(Eb + row + h0 + (ia >> 1)));
                    __builtin_nontemporal_store((float)rv[1], (VD_GAS float *)(Eb + row + (nh - h0) + (ia >> 1)));
                    if (!keep_e) {
                        __builtin_nontemporal_store(0.0f, (VD_GAS float *)(Ex + row + h0 + (ia >> 1)));
                        __builtin_nontemporal_store(0.0f, (VD_GAS float *)(Ex + row + (nh - h0) + (ia >> 1)));
                    }
                } else {
                    PairF rp;
                    rp.x = (float)rv[0];
                    rp.y = (float)rv[1];
                    __builtin_nontemporal_store(rp, (VD_GAS PairF *)(Eb + row + ia));
                    if (!keep_e) __builtin_nontemporal_store(PairF{0.0f, 0.0f}, (VD_GAS PairF *)(Ex + row + ia));
                }
            }
            xm = xc;
            xc = xp;
        }
    }
    const double sum = block_sum(v, red);
    if (tid == 0) gst(partials, slot, sum);
    if (partials_b) {
        const double sb = block_sum(vb, red);
        if (tid == 0) gst(partials_b, slot, sb);
    }
}

// ------------------------- parity-split colour pass (refinement corrections)
// The FP32 corrections of the finest level of uniform-coefficient problems
// are held parity-split by row (cell_pos): a colour pass then reads only
// the other colour's values and the right-hand side of the updated colour,
// and writes only the updated colour, half the bytes of a pass over the
// lexicographic layout.  A workgroup owns 32 half-row positions x 16 rows
// and marches kz planes; a thread updates two cells of its row (half-row
// positions m, m+1), and holds the other colour's values at those positions
// for planes k-1..k+1 in registers; the other colour's x-y neighbours of
// plane k come from LDS.  In a row whose updated cells sit at i = 2m + s,
// the x-neighbours of cell m are the other colour's positions m-1+s and
// m+s, the y- and z-neighbours its position m in the adjacent rows.  Each
// update is the same expression as in the lexicographic colour pass.
// PM 4: the first (red) pass from a zero correction (nothing of the other
// colour is read); 0: a colour pass; 5: the last (black) pass, which adds
// the final correction of the thread's four consecutive cells to the FP64
// unknown (d64) instead of storing it.  Needs nx % 4 == 0.
struct Pf {
    float a, b;
};
struct Q4 {
    PairD lo, hi;
};

template <int PM>
__global__ void __launch_bounds__(kBlock) k_rb32(const LevDesc *__restrict__ descs, const LevDesc *__restrict__ d64, Plan pl,
                                                 int kz, int colour, const ProbState *__restrict__ st) {
    __shared__ float xs[2][(kT25Y + 2) * kT25W];
    const int t = xcd_tile(pl.ntiles);
    if (t >= pl.ntiles) return;
    const int d = plan_find(pl, t);
    const int id = pl.ids[d];
    const LevDesc L = descs[id];
    if (!gld(&st[L.prob].active, 0)) return;
    const int lt = t - pl.prefix[d];
    const int nx = L.nx, ny = L.ny, nz = L.nz, nh = nx >> 1, nxy = L.nxy;
    const Tile25 T25 = tile25(lt, nh, ny, nz, kz);
    const int k0 = T25.k0, k1 = T25.k1;
    const int tid = threadIdx.x;
    const int tp = tid & 15, r = tid >> 4;
    const int hslot = halo_slot(tid);
    float *__restrict__ X = (float *)L.x;
    const float *__restrict__ B = (const float *)L.b;
    const float *zero = (const float *)g_zero4;
    const int oofs = (1 - colour) * nh, uofs = colour * nh;   // half-row offsets: other / updated colour
    const bool px = L.kind[0] == VD_BC_PERIODIC, py = L.kind[2] == VD_BC_PERIODIC, pz = L.kind[4] == VD_BC_PERIODIC;
    // the thread's pair of the other colour: wrapped (a partial tile's
    // positions past the row end hold the row's first ones when periodic)
    // or zeroed; a halo position wraps with the row (position -1 of the
    // other colour is its last one, position nh its first)
    const Thr25 H = thr25(T25, tid, nh, nx, ny, px, py, oofs, uofs);
    const int ma = H.ua, j = H.j;
    const bool own = H.own;      // nh is even, so the pair (ma, ma + 1) is whole
    const bool halo_thread = H.halo;
    const bool okp = H.okp, okh = H.okh;
    const int pair_off = (int)H.pair_off, b_off = (int)H.b_off, h_off = (int)H.h_off;
    // loads from the address of a cell, or of zeros where the position is
    // not one (no masking after the load)
    auto ld_pair = [&](int kk) -> Pf {
        if constexpr (PM == 4) return Pf{0.0f, 0.0f};
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const float *p = (okp && okz) ? X + (pair_off + nxy * kw) : zero;
        const PairF v = *(const VD_GAS PairF *)p;
        return Pf{v.x, v.y};
    };
    auto ld_h = [&](int kk) -> float {
        if constexpr (PM == 4) return 0.0f;
        bool okz;
        const int kw = wrap_idx(kk, nz, pz, okz);
        const float *p = (okh && okz) ? X + (h_off + nxy * kw) : zero;
        return *(const VD_GAS float *)p;
    };
    auto ld_b = [&](int kk) -> Pf {
        const float *p = (own && kk < k1) ? B + (b_off + nxy * kk) : zero;
        const PairF v = *(const VD_GAS PairF *)p;
        return Pf{v.x, v.y};
    };
    const int q_off = (int)quad_off25(ma, j, nh, nx, ny);   // first of the four cells (FP64)
    double *__restrict__ X64 = PM == 5 ? (double *)d64[id].x : nullptr;
    auto ld_q = [&](int kk) -> Q4 {
        if constexpr (PM != 5) return Q4{};
        const double *p = (own && kk < k1) ? X64 + (q_off + nxy * kk) : g_zero4;
        return Q4{*(const VD_GAS PairD *)p, *(const VD_GAS PairD *)(p + 2)};
    };
    const int lc0 = (r + 1) * kT25W + 2 * tp + 1;    // LDS slot of position ma
    // plane k: xm, xc, xp the other colour's pairs of planes k-1, k, k+1,
    // xq receives plane k+2; hc / bcur / qc plane k's halo element,
    // right-hand side pair and (PM 5) FP64 quad, hn / bn / qn receive plane
    // k+1's
    auto plane = [&](int k, const Pf &xm, const Pf &xc, const Pf &xp, Pf &xq, const float &hc, float &hn,
                     const Pf &bcur, Pf &bn, const Q4 &qc, Q4 &qn) {
        float *buf = xs[k & 1];
        buf[lc0] = xc.a;
        buf[lc0 + 1] = xc.b;
        if (halo_thread) buf[hslot] = hc;
        xq = ld_pair(k + 2);
        hn = ld_h(k + 1);
        bn = ld_b(k + 1);
        qn = ld_q(k + 1);
        __syncthreads();
        if (!own) return;
        const int s = (j + k + colour) & 1;      // updated cells at i = 2m + s
        float out[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const int i = 2 * (ma + q) + s;
            float nbv[6];
            const int lc = lc0 + q;               // LDS slot of position ma + q
            nbv[0] = s ? buf[lc] : buf[lc - 1];
            nbv[1] = s ? buf[lc + 1] : buf[lc];
            nbv[2] = buf[lc - kT25W];
            nbv[3] = buf[lc + kT25W];
            nbv[4] = q == 0 ? xm.a : xm.b;
            nbv[5] = q == 0 ? xp.a : xp.b;
            float dg, of;
            row_terms_uni<float>(L, i, j, k, nbv, dg, of);
            out[q] = ((q == 0 ? bcur.a : bcur.b) + of) / dg;
        }
        if constexpr (PM == 5) {
            // cells 2ma .. 2ma+3: updated at offsets s and s+2, the other
            // colour (this plane's values xc) at 1-s and 3-s
            PairD xa = qc.lo, xb = qc.hi;
            xa.x = xa.x + (double)(s ? xc.a : out[0]);
            xa.y = xa.y + (double)(s ? out[0] : xc.a);
            xb.x = xb.x + (double)(s ? xc.b : out[1]);
            xb.y = xb.y + (double)(s ? out[1] : xc.b);
            double *x64 = X64 + (q_off + nxy * k);
            *(VD_GAS PairD *)x64 = xa;
            *(VD_GAS PairD *)(x64 + 2) = xb;
        } else {
            PairF pv;
            pv.x = out[0];
            pv.y = out[1];
            *(VD_GAS PairF *)(X + uofs + ma + nx * j + nxy * k) = pv;
        }
    };
    Pf P0 = ld_pair(k0 - 1), P1 = ld_pair(k0), P2 = ld_pair(k0 + 1), P3;
    float H0 = ld_h(k0), H1;
    Pf B0 = ld_b(k0), B1;
    Q4 Q0 = ld_q(k0), Q1;
    for (int k = k0; k < k1; k += 4) {
        plane(k, P0, P1, P2, P3, H0, H1, B0, B1, Q0, Q1);
        if (k + 1 >= k1) break;
        plane(k + 1, P1, P2, P3, P0, H1, H0, B1, B0, Q1, Q0);
        if (k + 2 >= k1) break;
        plane(k + 2, P2, P3, P0, P1, H0, H1, B0, B1, Q0, Q1);
        if (k + 3 >= k1) break;
        plane(k + 3, P3, P0, P1, P2, H1, H0, B1, B0, Q1, Q0);
    }
}

// ------------------------------------------- fused red-black sweep (2.5D)
// One launch = one full Gauss-Seidel sweep (all red cells, then all black
// cells), out of place: the old iterate is read from one buffer and the new
// one written to the other, so no workgroup ever reads a value another
// workgroup has already overwritten.  A workgroup owns a 32 x 16 tile and
// marches its kz planes in z.  Red is computed on the tile plus a one-cell
// ring (the ring's red values are also computed by the neighbouring tiles;
// they are identical), from the old iterate held in LDS with a two-cell
// ring; black is computed on the tile from the new red values in LDS.  The
// red plane runs one plane ahead of the black plane.  Each cell's update is
// the same expression as in the colour passes, so the result equals a red
// pass followed by a black pass.
constexpr int kSwOX = kT25X + 4, kSwOY = kT25Y + 4;   // old iterate, 2-cell ring
constexpr int kSwRX = kT25X + 2, kSwRY = kT25Y + 2;   // new red values, 1-cell ring

// wrapped coordinate of position p along a direction of n cells; false if
// the position is not a cell (outside a non-periodic face, or further out
// than the two-cell ring)
__device__ __forceinline__ bool wrap_pos(int p, int n, bool periodic, int &w) {
    if (p >= 0 && p < n) { w = p; return true; }
    if (!periodic || p < -2 || p >= n + 2) return false;
    w = p < 0 ? p + n : p - n;
    return w >= 0 && w < n;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sweep25(const LevDesc *__restrict__ descs, Plan pl, int kz, int flip,
                                                    const ProbState *__restrict__ st) {
    __shared__ T xo[4][kSwOY * kSwOX];
    __shared__ T xr[3][kSwRY * kSwRX];
    const int t = xcd_tile(pl.ntiles);
    if (t >= pl.ntiles) return;
    const int d = plan_find(pl, t);
    const LevDesc L = descs[pl.ids[d]];
    if (!gld(&st[L.prob].active, 0)) return;
    int lt = t - pl.prefix[d];
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int ntx = (nx + kT25X - 1) / kT25X, nty = (ny + kT25Y - 1) / kT25Y;
    const int tx = lt % ntx;
    lt /= ntx;
    const int ty = lt % nty;
    const int zc = lt / nty;
    const int i0 = tx * kT25X, j0 = ty * kT25Y, k0 = zc * kz;
    const int k1 = min(k0 + kz, nz);
    const int tid = threadIdx.x;
    const bool px = L.kind[0] == VD_BC_PERIODIC, py = L.kind[2] == VD_BC_PERIODIC, pz = L.kind[4] == VD_BC_PERIODIC;
    const T *__restrict__ X = (const T *)(flip ? L.x2 : L.x);
    T *__restrict__ Y = (T *)(flip ? L.x : L.x2);
    const T *__restrict__ B = (const T *)L.b;
    const long nxy = L.nxy;
    constexpr int kOld = kSwOY * kSwOX;                 // 720 old values per plane
    constexpr int kOldPer = (kOld + kBlock - 1) / kBlock;
    constexpr int kRed = kSwRY * (kSwRX / 2);           // 306 red cells per ring plane
    constexpr int kRedPer = (kRed + kBlock - 1) / kBlock;

    // per-thread x-y parts of every load (plane-invariant); a position that
    // is not a cell reads a clamped valid address and is zeroed
    long o_off[kOldPer];
    bool o_ok[kOldPer];
#pragma unroll
    for (int m = 0; m < kOldPer; m++) {
        const int e = tid + m * kBlock;
        const int ri = e % kSwOX, rj = e / kSwOX;
        bool oi, oj;
        const int wi = wrap_idx(i0 - 2 + ri, nx, px, oi), wj = wrap_idx(j0 - 2 + rj, ny, py, oj);
        o_off[m] = wi + (long)nx * wj;
        o_ok[m] = e < kOld && oi && oj && (i0 - 2 + ri) >= -2 && (i0 - 2 + ri) < nx + 2 && (j0 - 2 + rj) >= -2 &&
                  (j0 - 2 + rj) < ny + 2;
    }
    // red cells of the ring: position depends on the plane's parity
    int r_ri[2][kRedPer], r_rj[kRedPer];
    long r_off[2][kRedPer];
    bool r_ok[2][kRedPer], r_own[2][kRedPer];
    int r_wi[2][kRedPer], r_wj[kRedPer];
#pragma unroll
    for (int m = 0; m < kRedPer; m++) {
        const int mm = tid + m * kBlock;
        const int rj = mm / (kSwRX / 2), h = mm - rj * (kSwRX / 2);
        const int gj = j0 - 1 + rj;
        bool oj;
        const int wj = wrap_idx(gj, ny, py, oj);
        r_rj[m] = rj;
        r_wj[m] = wj;
#pragma unroll
        for (int par = 0; par < 2; par++) {
            const int ri = 2 * h + ((i0 - 1 + gj + par) & 1);
            const int gi = i0 - 1 + ri;
            bool oi;
            const int wi = wrap_idx(gi, nx, px, oi);
            r_ri[par][m] = ri;
            r_wi[par][m] = wi;
            r_off[par][m] = wi + (long)nx * wj;
            r_ok[par][m] = mm < kRed && oi && oj;
            r_own[par][m] = r_ok[par][m] && ri >= 1 && ri <= kT25X && rj >= 1 && rj <= kT25Y && gi < nx && gj < ny;
        }
    }
    // the black cell of the tile owned by this thread, per plane parity
    const int b_r = tid >> 4, b_h = tid & 15;
    const int b_gj = j0 + b_r;
    int b_gi[2];
    long b_off[2];
    bool b_ok[2];
#pragma unroll
    for (int par = 0; par < 2; par++) {
        b_gi[par] = i0 + 2 * b_h + (((i0 + b_gj + par) & 1) ^ 1);
        b_ok[par] = b_gi[par] < nx && b_gj < ny;
        b_off[par] = min(b_gi[par], nx - 1) + (long)nx * min(b_gj, ny - 1);
    }

    auto plane_of = [&](int q, bool &ok) { return wrap_idx(q, nz, pz, ok); };
    auto ld_old = [&](int q, T v[kOldPer]) {
        bool okz;
        const long pz_off = nxy * plane_of(q, okz);
#pragma unroll
        for (int m = 0; m < kOldPer; m++) {
            const T g = gld(X, o_off[m] + pz_off);
            v[m] = (okz && o_ok[m]) ? g : (T)0;
        }
    };
    auto st_old = [&](int q, const T v[kOldPer]) {
        T *s = xo[(q + 4) & 3];
#pragma unroll
        for (int m = 0; m < kOldPer; m++) {
            const int e = tid + m * kBlock;
            if (e < kOld) lst(s, e, v[m]);
        }
    };
    auto ld_bred = [&](int p, T v[kRedPer]) {
        bool okz;
        const long pz_off = nxy * plane_of(p, okz);
        const int par = p & 1;
#pragma unroll
        for (int m = 0; m < kRedPer; m++) v[m] = gld(B, r_off[par][m] + pz_off);
    };
    auto ld_bblk = [&](int p) -> T {
        const int pc = min(max(p, 0), nz - 1);
        return gld(B, b_off[p & 1] + nxy * pc);
    };

    auto march = [&](auto uni_tag) {
        constexpr bool UNI = decltype(uni_tag)::value;
        T rowv[6];
        auto cell_row = [&](int i, int j, int k, int c, T &dg, T &of) {
            if constexpr (UNI) row_terms_uni<T>(L, i, j, k, rowv, dg, of);
            else row_terms_nb<T>(L, i, j, k, c, rowv, dg, of);
        };
        auto lift = [&](int i, int j, int k) -> double {
            if constexpr (UNI) return lift_term_uni(L, i, j, k);
            else return lift_term(L, i, j, k);
        };
        // red values of plane p on the tile and its ring (own cells stored)
        auto red_plane = [&](int p, const T bred[kRedPer]) {
            T *rs = xr[(p + 3) % 3];
            const T *om = xo[(p + 3) & 3], *oc = xo[(p + 4) & 3], *op = xo[(p + 5) & 3];
            bool okz;
            const int wk = plane_of(p, okz);
            const bool own_plane = p >= k0 && p < k1;
            const int par = p & 1;
#pragma unroll
            for (int m = 0; m < kRedPer; m++) {
                if (tid + m * kBlock >= kRed) break;
                const int ri = r_ri[par][m], rj = r_rj[m];
                T val = (T)0;
                if (okz && r_ok[par][m]) {
                    const int wi = r_wi[par][m], wj = r_wj[m];
                    const int c = wi + nx * wj + (int)nxy * wk;
                    const int o = (rj + 1) * kSwOX + ri + 1;
                    if (!UNI && L.has_mask && !gld(L.mask, c)) {
                        val = lld(oc, o);
                    } else {
                        rowv[0] = lld(oc, o - 1);
                        rowv[1] = lld(oc, o + 1);
                        rowv[2] = lld(oc, o - kSwOX);
                        rowv[3] = lld(oc, o + kSwOX);
                        rowv[4] = lld(om, o);
                        rowv[5] = lld(op, o);
                        T dg, of;
                        cell_row(wi, wj, wk, c, dg, of);
                        T bv = bred[m];
                        if (L.lift) bv = (T)((double)bv + lift(wi, wj, wk));
                        val = (bv + of) / dg;
                    }
                    if (own_plane && r_own[par][m]) gst(Y, c, val);
                }
                lst(rs, rj * kSwRX + ri, val);
            }
        };
        // black value of the thread's tile cell on plane p
        auto black_plane = [&](int p, T bv) {
            const int par = p & 1;
            if (!b_ok[par]) return;
            const T *rm = xr[(p + 2) % 3], *rc = xr[(p + 3) % 3], *rp = xr[(p + 4) % 3];
            const int gi = b_gi[par];
            const int c = gi + nx * b_gj + (int)nxy * p;
            const int ri = gi - i0 + 1, rj = b_r + 1;
            T val;
            if (!UNI && L.has_mask && !gld(L.mask, c)) {
                val = lld(xo[(p + 4) & 3], (rj + 1) * kSwOX + ri + 1);
            } else {
                const int o = rj * kSwRX + ri;
                rowv[0] = lld(rc, o - 1);
                rowv[1] = lld(rc, o + 1);
                rowv[2] = lld(rc, o - kSwRX);
                rowv[3] = lld(rc, o + kSwRX);
                rowv[4] = lld(rm, o);
                rowv[5] = lld(rp, o);
                T dg, of;
                cell_row(gi, b_gj, p, c, dg, of);
                if (L.lift) bv = (T)((double)bv + lift(gi, b_gj, p));
                val = (bv + of) / dg;
            }
            gst(Y, c, val);
        };

        // prologue: old planes k0-2 .. k0 in LDS, plane k0+1 and the
        // right-hand sides of the first red plane in registers
        T ov[kOldPer], bred[kRedPer], bblk = (T)0, bblk_next;
        ld_old(k0 - 2, ov);
        st_old(k0 - 2, ov);
        ld_old(k0 - 1, ov);
        st_old(k0 - 1, ov);
        ld_old(k0, ov);
        st_old(k0, ov);
        ld_old(k0 + 1, ov);
        ld_bred(k0 - 1, bred);
        __syncthreads();
        for (int p = k0 - 1; p <= k1; p++) {
            red_plane(p, bred);
            // plane p+2 goes to the slot of plane p-2; then the look-ahead
            // loads for the next plane are issued
            if (p + 2 <= k1 + 1) st_old(p + 2, ov);
            if (p + 3 <= k1 + 1) ld_old(p + 3, ov);
            ld_bred(p + 1, bred);
            bblk_next = ld_bblk(p);
            __syncthreads();
            if (p - 1 >= k0) black_plane(p - 1, bblk);
            bblk = bblk_next;
            __syncthreads();
        }
    };
    if (!L.var_beta && !L.var_alpha && !L.has_mask) march(std::true_type{});
    else march(std::false_type{});
}

// x <- x2 on every level of the plan (after an odd number of fused sweeps)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy_x2(const LevDesc *__restrict__ descs, Plan pl,
                                                    const ProbState *__restrict__ st) {
    for_tiles(pl, [&](int d, int lt, int) {
        const LevDesc L = descs[pl.ids[d]];
        if (!gld(&st[L.prob].active, 0)) return;
        for (int u = 0; u < 2 * kGsrbU; u++) {
            const int c = (lt * 2 * kGsrbU + u) * kBlock + threadIdx.x;
            if (c >= L.ncell) break;
            gst((T *)L.x, c, gld((const T *)L.x2, c));
        }
    });
}

__global__ void k_state_init(ProbState *st, int n) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    ProbState s;
    s.active = 1; s.cycles = 0; s.outer = 0; s.status = VD_OK;
    s.bnorm = 0.0; s.rel0 = 0.0; s.rel = 0.0;
    st[p] = s;
}

// One workgroup per problem: sum its partials in a fixed order and take the
// stopping decision.  mode 0: ||b||; mode 1: residual check before a cycle.
__global__ void __launch_bounds__(kBlock) k_finalize(Plan pl, const int *__restrict__ prob_of, const double *__restrict__ partials,
                                                     ProbState *__restrict__ st, int mode, double rtol, int max_cycles,
                                                     int fixed, int inner, const double *__restrict__ partials_b) {
    __shared__ double lds[kBlock / 64];
    int d = blockIdx.x;
    int p = prob_of[d];
    ProbState s = st[p];
    if ((mode == 1 || mode == 3) && !s.active) return;
    double v = 0.0, vb = 0.0;
    for (int q = pl.prefix[d] + threadIdx.x; q < pl.prefix[d + 1]; q += blockDim.x) {
        v += gld(partials, q);
        if (mode == 3) vb += gld(partials_b, q);
    }
    double tot = block_sum(v, lds);
    double totb = mode == 3 ? block_sum(vb, lds) : 0.0;
    if (threadIdx.x != 0) return;
    if (mode == 3) {             // first check: ||b|| from the same pass
        s.bnorm = sqrt(totb);
        if (s.bnorm == 0.0) { s.active = 0; s.rel = 0.0; st[p] = s; return; }
        mode = 1;
    }
    if (mode == 0) {
        s.bnorm = sqrt(tot);
        if (s.bnorm == 0.0) { s.active = 0; s.rel = 0.0; }
        st[p] = s;
        return;
    }
    double rel = sqrt(tot) / s.bnorm;
    if (mode == 2) {             // report only (residual of an initial guess)
        s.rel = rel;
        st[p] = s;
        return;
    }
    if (s.outer == 0) s.rel0 = rel;
    s.rel = rel;
    s.outer += 1;
    int done_iters = s.outer - 1;   // cycles (FP64) or outer steps (IR) already run
    if (!isfinite(rel)) { s.status = VD_ENOCONV; s.active = 0; }
    else if (fixed > 0) { if (done_iters == fixed) s.active = 0; }
    else if (rel <= rtol) s.active = 0;
    else if (done_iters == max_cycles) { s.status = VD_ENOCONV; s.active = 0; }
    if (s.active) s.cycles += inner;
    st[p] = s;
}

// ---------------------------------------------------- fused coarse kernel
struct FusedDesc {
    int prob, lc, L, base;     // base = index of level 0 in the descriptor arrays
    double *pcg;               // FP64 scratch: 6 * bottom cells (used when not in LDS)
};

constexpr int kFusedThreads = 256;
constexpr int kPcgLdsCells = 768;    // bottom levels up to this size keep the CG vectors in LDS

template <typename T>
__device__ __forceinline__ void block_sweep(const LevDesc L, int colour) {
    for (int c = threadIdx.x; c < L.ncell; c += blockDim.x) {
        int i, j, k;
        cell_ijk(L, c, i, j, k);
        if (((i + j + k) & 1) == colour) gs_update<T>(L, c, i, j, k);
    }
    __syncthreads();
}

// two deterministic block sums with one pair of barriers
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds) {
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_xor(a, o, 64); b += __shfl_xor(b, o, 64); }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { lds[2 * w] = a; lds[2 * w + 1] = b; }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; q++) { sa += lds[2 * q]; sb += lds[2 * q + 1]; }
    __syncthreads();
    a = sa;
    b = sb;
}

// Jacobi-preconditioned CG in FP64 on the coarsest level, from a zero guess,
// to ||r|| <= 1e-14 ||b|| or 500 iterations.  vec: 6 n doubles (LDS or global).
template <typename T>
__device__ void block_pcg(const LevDesc &A64, const LevDesc &AT, double *vec, double *red) {
    const int n = A64.ncell;
    double *r = vec, *z = vec + n, *p = vec + 2 * n, *q = vec + 3 * n, *dg = vec + 4 * n, *xb = vec + 5 * n;
    const T *bT = (const T *)AT.b;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        bool valid = !(A64.has_mask && !gld(A64.mask, c));
        gst(r, c, valid ? (double)gld(bT, c) : 0.0);
        gst(xb, c, 0.0);
    }
    __syncthreads();
    double rr = 0.0, rz = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int i, j, k;
        cell_ijk(A64, c, i, j, k);
        double d, of;
        row_terms<double, double>(A64, xb, i, j, k, c, d, of);   // xb is zero: only the diagonal is used
        gst(dg, c, d);
        bool valid = !(A64.has_mask && !gld(A64.mask, c));
        const double rc = gld(r, c);
        double zz = valid ? rc / d : 0.0;
        gst(z, c, zz);
        gst(p, c, zz);
        rr += rc * rc;
        rz += rc * zz;
    }
    block_sum2(rr, rz, red);
    const double bn = sqrt(rr);
    for (int it = 0; it < kBottomMaxIt; it++) {
        if (!(sqrt(rr) > kBottomTol * bn)) break;
        double v = 0.0;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            double qq = 0.0;
            const double pc = gld(p, c);
            if (!(A64.has_mask && !gld(A64.mask, c))) {
                int i, j, k;
                cell_ijk(A64, c, i, j, k);
                double d, of;
                row_terms<double, double>(A64, p, i, j, k, c, d, of);
                qq = d * pc - of;
            }
            gst(q, c, qq);
            v += pc * qq;
        }
        double pq = block_sum(v, red);
        if (pq == 0.0) break;
        const double a = rz / pq;
        double rz_new = 0.0, rr_new = 0.0;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const double pc = gld(p, c);
            gst(xb, c, gld(xb, c) + a * pc);
            double rc = gld(r, c) - a * gld(q, c);
            gst(r, c, rc);
            bool valid = !(A64.has_mask && !gld(A64.mask, c));
            double zz = valid ? rc / gld(dg, c) : 0.0;
            gst(z, c, zz);
            rz_new += rc * zz;
            rr_new += rc * rc;
        }
        block_sum2(rz_new, rr_new, red);
        const double bcoef = rz_new / rz;
        rz = rz_new;
        rr = rr_new;
        for (int c = threadIdx.x; c < n; c += blockDim.x) gst(p, c, gld(z, c) + bcoef * gld(p, c));
        __syncthreads();
    }
    T *xT = (T *)AT.x;
    for (int c = threadIdx.x; c < n; c += blockDim.x) gst(xT, c, (T)gld(xb, c));
    __syncthreads();
}

// Same CG on a single wavefront (lanes 0..63, vectors in LDS): the
// reductions are shuffle trees and the only synchronisation is the
// wavefront's own, so a small bottom level costs no workgroup barriers.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sum over the 64 lanes of a wavefront (all lanes active), in every lane:
// quad and row steps with DPP lane moves, then the four row sums read as
// scalars.  No LDS round trips, unlike a shuffle tree.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x124>(v);   // row_ror 4
    v += dpp_move<0x128>(v);   // row_ror 8: every lane holds its row's sum
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

template <typename T, int BAS>
__device__ void wave_pcg(const LevDesc &A64, const T *bT, T *xT, double *vec) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int n = A64.ncell;
        double *r = vec, *z = vec + n, *p = vec + 2 * n, *q = vec + 3 * n, *dg = vec + 4 * n, *xb = vec + 5 * n;
        for (int c = lane; c < n; c += 64) {
            const bool valid = !(A64.has_mask && !gld(A64.mask, c));
            lst(r, c, valid ? (double)mld<BAS>(bT, c) : 0.0);
            lst(xb, c, 0.0);
        }
        wave_sync();
        double rr = 0.0, rz = 0.0;
        for (int c = lane; c < n; c += 64) {
            int i, j, k;
            cell_ijk(A64, c, i, j, k);
            double d, of;
            row_terms<double, double, 3>(A64, xb, i, j, k, c, d, of);   // xb is zero: only the diagonal is used
            lst(dg, c, d);
            const bool valid = !(A64.has_mask && !gld(A64.mask, c));
            const double rc = lld(r, c);
            const double zz = valid ? rc / d : 0.0;
            lst(z, c, zz);
            lst(p, c, zz);
            rr += rc * rc;
            rz += rc * zz;
        }
        rr = wave_sum(rr);
        rz = wave_sum(rz);
        wave_sync();
        const double bn = sqrt(rr);
        for (int it = 0; it < kBottomMaxIt; it++) {
            if (!(sqrt(rr) > kBottomTol * bn)) break;
            double v = 0.0;
            for (int c = lane; c < n; c += 64) {
                double qq = 0.0;
                const double pc = lld(p, c);
                if (!(A64.has_mask && !gld(A64.mask, c))) {
                    int i, j, k;
                    cell_ijk(A64, c, i, j, k);
                    double d, of;
                    row_terms<double, double, 3>(A64, p, i, j, k, c, d, of);
                    qq = d * pc - of;
                }
                lst(q, c, qq);
                v += pc * qq;
            }
            const double pq = wave_sum(v);
            if (pq == 0.0) break;
            const double a = rz / pq;
            double rz_new = 0.0, rr_new = 0.0;
            for (int c = lane; c < n; c += 64) {
                const double pc = lld(p, c);
                lst(xb, c, lld(xb, c) + a * pc);
                const double rc = lld(r, c) - a * lld(q, c);
                lst(r, c, rc);
                const bool valid = !(A64.has_mask && !gld(A64.mask, c));
                const double zz = valid ? rc / lld(dg, c) : 0.0;
                lst(z, c, zz);
                rz_new += rc * zz;
                rr_new += rc * rc;
            }
            rz_new = wave_sum(rz_new);
            rr_new = wave_sum(rr_new);
            const double bcoef = rz_new / rz;
            rz = rz_new;
            rr = rr_new;
            for (int c = lane; c < n; c += 64) lst(p, c, lld(z, c) + bcoef * lld(p, c));
            wave_sync();
        }
        for (int c = lane; c < n; c += 64) mst<BAS>(xT, c, (T)lld(xb, c));
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kFusedThreads) k_coarse(const LevDesc *__restrict__ dT, const LevDesc *__restrict__ d64,
                                                          const FusedDesc *__restrict__ fd, const ProbState *__restrict__ st,
                                                          int nu_pre, int nu_post, int pcg_in_lds) {
    __shared__ double red[2 * (kFusedThreads / 64)];
    extern __shared__ double pcg_lds[];
    const FusedDesc f = fd[blockIdx.x];
    if (!gld(&st[f.prob].active, 0)) return;
    const int base = f.base, lc = f.lc, L = f.L;
    if (L == 1) {
        const LevDesc &A = dT[base];
        for (int s = 0; s < nu_pre + nu_post; s++) { block_sweep<T>(A, 0); block_sweep<T>(A, 1); }
        return;
    }
    for (int l = lc; l < L - 1; l++) {
        const LevDesc &A = dT[base + l];
        for (int s = 0; s < nu_pre; s++) { block_sweep<T>(A, 0); block_sweep<T>(A, 1); }
        const LevDesc &C = dT[base + l + 1];
        for (int cc = threadIdx.x; cc < C.ncell; cc += blockDim.x) {
            int I, J, K;
            cell_ijk(C, cc, I, J, K);
            restrict_cell<T>(A, C, cc, I, J, K);
        }
        __syncthreads();
    }
    if (pcg_in_lds) wave_pcg<T, 1>(d64[base + L - 1], (const T *)dT[base + L - 1].b, (T *)dT[base + L - 1].x, pcg_lds);
    else block_pcg<T>(d64[base + L - 1], dT[base + L - 1], f.pcg, red);
    for (int l = L - 2; l >= lc; l--) {
        const LevDesc &A = dT[base + l];
        const LevDesc &C = dT[base + l + 1];
        for (int c = threadIdx.x; c < A.ncell; c += blockDim.x) {
            int i, j, k;
            cell_ijk(A, c, i, j, k);
            prolong_cell<T>(A, C, c, i, j, k);
        }
        __syncthreads();
        for (int s = 0; s < nu_post; s++) { block_sweep<T>(A, 0); block_sweep<T>(A, 1); }
    }
}

// ------------------------------------------- LDS-resident coarse V-cycle
// One workgroup per problem runs every level from lc down to the bottom
// entirely out of LDS, then writes level lc's unknown back.  A resident
// level holds x and b; a level with variable coefficients or a mask also
// holds its assembled seven-point row (diagonal and six neighbour weights,
// zero where the neighbour is absent), assembled once per solve by
// k_stencils from the same face logic as row_terms, in the hierarchy's
// precision (the bottom CG also gets an FP64 copy in FP32 hierarchies).  A
// level with uniform coefficients and no mask forms its row on the fly from
// the level descriptor (row_terms_uni), which leaves room for one more
// level in LDS.  Neighbour indices always wrap; an absent neighbour has
// weight 0.
constexpr int kLdsThreads = 1024;
constexpr int kPcgSlots = 2;     // register-resident bottom CG: up to 64 * kPcgSlots cells

__host__ __device__ __forceinline__ size_t lds_al16(size_t b) { return (b + 15) & ~(size_t)15; }
// bytes of one resident level: x (with a zero slot after the n cells), b,
// then either the assembled row (diagonal then 6 weight planes, contiguous
// as assembled) or the 64-entry diagonal and inverse-diagonal tables of a
// uniform row, then the optional mask
constexpr int kUniTab = 64;
__host__ __device__ __forceinline__ size_t lds_level_bytes(long n, size_t sT, bool mask, bool rows) {
    return lds_al16((size_t)(n + 1) * sT) + lds_al16((size_t)n * sT) +
           (rows ? lds_al16((size_t)7 * n * sT) : lds_al16((size_t)2 * kUniTab * sT)) + (mask ? lds_al16((size_t)n) : 0);
}
// bytes of the bottom CG: r, z, p, q, x (+ FP64 row copy in FP32 hierarchies
// with assembled rows)
__host__ __device__ __forceinline__ size_t lds_pcg_bytes(long nb, bool fp32_rows) {
    return 5 * lds_al16((size_t)nb * sizeof(double)) + (fp32_rows ? lds_al16((size_t)7 * nb * sizeof(double)) : 0);
}

template <typename T>
struct LLev {
    T *x, *b, *dg, *w;        // w: 6 weight planes of n values; dg null: uniform row
    T *tab;                   // uniform row: diagonal, then its inverse, by the faces that join the sum
    const uint8_t *m;         // covered-cell mask in LDS (null: all valid)
    int nx, ny, nz, nxy, n;
    int half;                 // n / 2 when held split by the parity of i (even nx), else 0
    float inx, inxy;
    T a0, cx, cy, cz;         // uniform row: alpha and beta / h^2 per direction
    int per, dir;             // uniform row: bit f set when face f is periodic / Dirichlet
};

// LDS slot of cell c.  A level with an even nx is held as two halves, the
// cells of even i then those of odd i, so the unit-stride pair walks of the
// colour passes touch consecutive slots (no bank conflicts).
template <typename T>
__device__ __forceinline__ int lslot(const LLev<T> &v, int c) {
    return v.half ? (c >> 1) + (c & 1) * v.half : c;
}

template <typename T>
__device__ __forceinline__ LLev<T> lds_lev(char *raw, const LevDesc *dT, int base, int lc, int l) {
    size_t off = 0;
    for (int m = lc; m < l; m++)
        off += lds_level_bytes(dT[base + m].ncell, sizeof(T), dT[base + m].has_mask, dT[base + m].sten != nullptr);
    const LevDesc &D = dT[base + l];
    LLev<T> v;
    const size_t ax = lds_al16((size_t)(D.ncell + 1) * sizeof(T)), a = lds_al16((size_t)D.ncell * sizeof(T));
    const bool rows = D.sten != nullptr;
    v.x = (T *)(raw + off);
    v.b = (T *)(raw + off + ax);
    v.dg = rows ? (T *)(raw + off + ax + a) : nullptr;
    v.w = rows ? v.dg + D.ncell : nullptr;
    v.tab = rows ? nullptr : (T *)(raw + off + ax + a);
    const size_t rb = rows ? lds_al16((size_t)7 * D.ncell * sizeof(T)) : lds_al16((size_t)2 * kUniTab * sizeof(T));
    v.m = D.has_mask ? (const uint8_t *)(raw + off + ax + a + rb) : nullptr;
    v.nx = D.nx; v.ny = D.ny; v.nz = D.nz; v.nxy = D.nxy; v.n = D.ncell;
    v.half = (D.nx & 1) ? 0 : D.ncell >> 1;
    v.inx = 1.0f / (float)D.nx;
    v.inxy = 1.0f / (float)D.nxy;
    v.a0 = (T)D.alpha_c;
    v.cx = (T)D.beta_c * (T)D.idx2;
    v.cy = (T)D.beta_c * (T)D.idy2;
    v.cz = (T)D.beta_c * (T)D.idz2;
    v.per = 0;
    v.dir = 0;
    for (int f = 0; f < 6; f++) {
        v.per |= D.kind[f] == VD_BC_PERIODIC ? 1 << f : 0;
        v.dir |= D.kind[f] == VD_BC_DIRICHLET ? 1 << f : 0;
    }
    return v;
}

// (i, j, k) of cell c; (c + 0.5) / d rounded in FP32 stays within the
// open unit interval of the true quotient for c < 2^22
template <typename T>
__device__ __forceinline__ void llev_ijk(const LLev<T> &v, int c, int &i, int &j, int &k) {
    k = (int)(((float)c + 0.5f) * v.inxy);
    const int r = c - k * v.nxy;
    j = (int)(((float)r + 0.5f) * v.inx);
    i = r - j * v.nx;
}

// the six neighbour slots of cell c (indices wrap; an absent neighbour has
// weight 0) and the faces that join the sum of a uniform row
template <typename T>
__device__ __forceinline__ int llev_nbrs(const LLev<T> &v, int c, int i, int j, int k, int nb[6]) {
    nb[0] = lslot(v, i > 0 ? c - 1 : c + v.nx - 1);
    nb[1] = lslot(v, i < v.nx - 1 ? c + 1 : c - (v.nx - 1));
    nb[2] = lslot(v, j > 0 ? c - v.nx : c + v.nx * (v.ny - 1));
    nb[3] = lslot(v, j < v.ny - 1 ? c + v.nx : c - v.nx * (v.ny - 1));
    nb[4] = lslot(v, k > 0 ? c - v.nxy : c + v.nxy * (v.nz - 1));
    nb[5] = lslot(v, k < v.nz - 1 ? c + v.nxy : c - v.nxy * (v.nz - 1));
    return v.per | (i > 0 ? 1 : 0) | (i < v.nx - 1 ? 2 : 0) | (j > 0 ? 4 : 0) | (j < v.ny - 1 ? 8 : 0) |
           (k > 0 ? 16 : 0) | (k < v.nz - 1 ? 32 : 0);
}

// diagonal of a uniform row from the faces that join the sum (a Dirichlet
// domain face adds 2 beta / h^2, a Neumann one nothing)
template <typename T>
__device__ __forceinline__ T llev_diag_uni(const LLev<T> &v, int use) {
    T m[6];
#pragma unroll
    for (int f = 0; f < 6; f++) m[f] = (use >> f) & 1 ? (T)1 : ((v.dir >> f) & 1 ? (T)2 : (T)0);
    return v.a0 + v.cx * (m[0] + m[1]) + v.cy * (m[2] + m[3]) + v.cz * (m[4] + m[5]);
}

// diagonal and neighbour sum of cell c's row applied to x (slot-indexed)
template <typename T>
__device__ __forceinline__ void llev_row(const LLev<T> &v, const T *x, int c, int i, int j, int k, T &dg, T &of) {
    int nb[6];
    const int use = llev_nbrs(v, c, i, j, k, nb);
    T e[6];
#pragma unroll
    for (int f = 0; f < 6; f++) e[f] = lld(x, nb[f]);
    if (v.dg) {
        const int sc = lslot(v, c), n = v.n;
        T s = 0;
#pragma unroll
        for (int f = 0; f < 6; f++) s += lld(v.w, f * n + sc) * e[f];
        dg = lld(v.dg, sc);
        of = s;
    } else {
#pragma unroll
        for (int f = 0; f < 6; f++) e[f] = (use >> f) & 1 ? e[f] : (T)0;
        dg = llev_diag_uni(v, use);
        of = v.cx * (e[0] + e[1]) + v.cy * (e[2] + e[3]) + v.cz * (e[4] + e[5]);
    }
}

// the row of cell c applied to the level's own iterate: an absent
// non-periodic neighbour of a uniform row reads the zero slot, and the
// diagonal and its inverse come from the level's tables
template <typename T>
__device__ __forceinline__ void llev_row_x(const LLev<T> &v, int c, int i, int j, int k, T &dg, T &idg, T &of) {
    if (v.dg) {
        llev_row(v, v.x, c, i, j, k, dg, of);
        idg = (T)0;
        return;
    }
    const int z = v.n;
    const bool u0 = i > 0 || (v.per & 1), u1 = i < v.nx - 1 || (v.per & 2);
    const bool u2 = j > 0 || (v.per & 4), u3 = j < v.ny - 1 || (v.per & 8);
    const bool u4 = k > 0 || (v.per & 16), u5 = k < v.nz - 1 || (v.per & 32);
    const int s0 = u0 ? lslot(v, i > 0 ? c - 1 : c + v.nx - 1) : z;
    const int s1 = u1 ? lslot(v, i < v.nx - 1 ? c + 1 : c - (v.nx - 1)) : z;
    const int s2 = u2 ? lslot(v, j > 0 ? c - v.nx : c + v.nx * (v.ny - 1)) : z;
    const int s3 = u3 ? lslot(v, j < v.ny - 1 ? c + v.nx : c - v.nx * (v.ny - 1)) : z;
    const int s4 = u4 ? lslot(v, k > 0 ? c - v.nxy : c + v.nxy * (v.nz - 1)) : z;
    const int s5 = u5 ? lslot(v, k < v.nz - 1 ? c + v.nxy : c - v.nxy * (v.nz - 1)) : z;
    const int use = (u0 ? 1 : 0) | (u1 ? 2 : 0) | (u2 ? 4 : 0) | (u3 ? 8 : 0) | (u4 ? 16 : 0) | (u5 ? 32 : 0);
    const T *x = v.x;
    of = v.cx * (lld(x, s0) + lld(x, s1)) + v.cy * (lld(x, s2) + lld(x, s3)) + v.cz * (lld(x, s4) + lld(x, s5));
    dg = lld(v.tab, use);
    idg = lld(v.tab, kUniTab + use);
}

template <typename T>
__device__ __forceinline__ bool llev_valid(const LLev<T> &v, int c) {
    return !v.m || lld(v.m, lslot(v, c)) != 0;
}

// one colour pass; with an even nx the two cells of a pair are one of each
// colour, so every thread updates a cell
template <typename T>
__device__ __forceinline__ void llev_sweep(const LLev<T> &v, int colour) {
    if (v.half) {
        const int np = v.half;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            int i, j, k;
            llev_ijk(v, 2 * p, i, j, k);
            const int s = (i + j + k + colour) & 1;
            const int c = 2 * p + s;
            i += s;
            if (!llev_valid(v, c)) continue;
            T dg, idg, of;
            llev_row_x(v, c, i, j, k, dg, idg, of);
            const int sc = p + s * np;
            lst(v.x, sc, v.dg ? (lld(v.b, sc) + of) / dg : (lld(v.b, sc) + of) * idg);
        }
    } else {
        for (int c = threadIdx.x; c < v.n; c += blockDim.x) {
            int i, j, k;
            llev_ijk(v, c, i, j, k);
            if (((i + j + k) & 1) != colour || !llev_valid(v, c)) continue;
            T dg, idg, of;
            llev_row_x(v, c, i, j, k, dg, idg, of);
            lst(v.x, c, v.dg ? (lld(v.b, c) + of) / dg : (lld(v.b, c) + of) * idg);
        }
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ T llev_resid(const LLev<T> &v, int c) {
    if (!llev_valid(v, c)) return (T)0;
    int i, j, k;
    llev_ijk(v, c, i, j, k);
    T dg, idg, of;
    llev_row_x(v, c, i, j, k, dg, idg, of);
    const int sc = lslot(v, c);
    return lld(v.b, sc) - (dg * lld(v.x, sc) - of);
}

// Jacobi-preconditioned CG on the bottom level, one wavefront, FP64; vd
// gives the FP64 row (assembled in LDS or uniform), b and x are the level's
// LDS arrays, vec holds the CG vectors (slot-indexed like the level).
// Bottom levels of up to 64 * kPcgSlots cells keep r, z, p, x and their
// rows in registers (lane l owns cells l, l + 64, ...) and publish only p
// to LDS for the product; larger ones keep every vector in LDS.  The
// stopping test ||r|| <= tol ||b|| is taken on the squares.
template <typename T>
__device__ __forceinline__ void llev_pcg(const LLev<T> &v, const LLev<double> &vd, double *vec) {
    const int lane = threadIdx.x, n = v.n;
    const double tol2 = kBottomTol * kBottomTol;
    if (lane >= 64) {
        // the other wavefronts wait at the closing barrier
    } else if (n <= 64 * kPcgSlots) {
        double *pl = vec;
        double r[kPcgSlots], z[kPcgSlots], p[kPcgSlots], x[kPcgSlots], dg[kPcgSlots], idg[kPcgSlots], w[kPcgSlots][6];
        int nb[kPcgSlots][6], sl[kPcgSlots];
        double rr = 0.0, rz = 0.0;
#pragma unroll
        for (int s = 0; s < kPcgSlots; s++) {
            const int c0 = lane + 64 * s;
            const bool ok = c0 < n && llev_valid(v, c0);
            const int c = c0 < n ? c0 : 0;
            int i, j, k;
            llev_ijk(vd, c, i, j, k);
            const int use = llev_nbrs(vd, c, i, j, k, nb[s]);
            sl[s] = lslot(vd, c);
            if (vd.dg) {
#pragma unroll
                for (int f = 0; f < 6; f++) w[s][f] = lld(vd.w, f * n + sl[s]);
                dg[s] = lld(vd.dg, sl[s]);
            } else {
                const double cf[3] = {vd.cx, vd.cy, vd.cz};
#pragma unroll
                for (int f = 0; f < 6; f++) w[s][f] = (use >> f) & 1 ? cf[f >> 1] : 0.0;
                dg[s] = llev_diag_uni(vd, use);
            }
            // a masked or absent cell: no row, zero residual
            if (!ok) {
#pragma unroll
                for (int f = 0; f < 6; f++) w[s][f] = 0.0;
                dg[s] = 0.0;
            }
            idg[s] = ok ? 1.0 / dg[s] : 0.0;
            r[s] = ok ? (double)lld(v.b, sl[s]) : 0.0;
            z[s] = r[s] * idg[s];
            p[s] = z[s];
            x[s] = 0.0;
            rr += r[s] * r[s];
            rz += r[s] * z[s];
        }
        rr = wave_sum(rr);
        rz = wave_sum(rz);
        const double lim = tol2 * rr;
        for (int it = 0; it < kBottomMaxIt; it++) {
            if (!(rr > lim)) break;
#pragma unroll
            for (int s = 0; s < kPcgSlots; s++)
                if (lane + 64 * s < n) lst(pl, sl[s], p[s]);
            wave_sync();
            double q[kPcgSlots], pq = 0.0;
#pragma unroll
            for (int s = 0; s < kPcgSlots; s++) {
                double of = 0.0;
#pragma unroll
                for (int f = 0; f < 6; f++) of += w[s][f] * lld(pl, nb[s][f]);
                q[s] = dg[s] * p[s] - of;
                pq += p[s] * q[s];
            }
            pq = wave_sum(pq);
            if (pq == 0.0) break;
            const double al = rz / pq;
            double rz_new = 0.0, rr_new = 0.0;
#pragma unroll
            for (int s = 0; s < kPcgSlots; s++) {
                x[s] = x[s] + al * p[s];
                r[s] = r[s] - al * q[s];
                z[s] = r[s] * idg[s];
                rz_new += r[s] * z[s];
                rr_new += r[s] * r[s];
            }
            rz_new = wave_sum(rz_new);
            rr_new = wave_sum(rr_new);
            const double bcoef = rz_new / rz;
            rz = rz_new;
            rr = rr_new;
#pragma unroll
            for (int s = 0; s < kPcgSlots; s++) p[s] = z[s] + bcoef * p[s];
            wave_sync();
        }
#pragma unroll
        for (int s = 0; s < kPcgSlots; s++)
            if (lane + 64 * s < n) lst(v.x, sl[s], (T)x[s]);
    } else {
        const size_t a = lds_al16((size_t)n * sizeof(double)) / sizeof(double);
        double *r = vec, *z = vec + a, *p = vec + 2 * a, *q = vec + 3 * a, *xb = vec + 4 * a;
        double rr = 0.0, rz = 0.0;
        for (int c = lane; c < n; c += 64) lst(p, lslot(vd, c), 0.0);
        wave_sync();
        // q holds 1 / diagonal (0 for a masked cell) throughout
        for (int c = lane; c < n; c += 64) {
            const bool valid = llev_valid(v, c);
            const int sc = lslot(vd, c);
            int i, j, k;
            llev_ijk(vd, c, i, j, k);
            double d, of;
            llev_row(vd, (const double *)p, c, i, j, k, d, of);
            const double id = valid ? 1.0 / d : 0.0;
            const double rc = valid ? (double)lld(v.b, sc) : 0.0;
            lst(r, sc, rc);
            lst(z, sc, id);
            lst(xb, sc, 0.0);
            rr += rc * rc;
            rz += rc * rc * id;
        }
        wave_sync();
        for (int c = lane; c < n; c += 64) {
            const int sc = lslot(vd, c);
            lst(q, sc, lld(z, sc));
            lst(p, sc, lld(r, sc) * lld(z, sc));
        }
        rr = wave_sum(rr);
        rz = wave_sum(rz);
        wave_sync();
        const double lim = tol2 * rr;
        double *Ap = z;   // z is recomputed from r and q each iteration
        for (int it = 0; it < kBottomMaxIt; it++) {
            if (!(rr > lim)) break;
            double pq = 0.0;
            for (int c = lane; c < n; c += 64) {
                const int sc = lslot(vd, c);
                const double pc = lld(p, sc);
                double aq = 0.0;
                if (llev_valid(v, c)) {
                    int i, j, k;
                    llev_ijk(vd, c, i, j, k);
                    double d, of;
                    llev_row(vd, (const double *)p, c, i, j, k, d, of);
                    aq = d * pc - of;
                }
                lst(Ap, sc, aq);
                pq += pc * aq;
            }
            pq = wave_sum(pq);
            if (pq == 0.0) break;
            const double al = rz / pq;
            double rz_new = 0.0, rr_new = 0.0;
            wave_sync();
            for (int c = lane; c < n; c += 64) {
                const int sc = lslot(vd, c);
                lst(xb, sc, lld(xb, sc) + al * lld(p, sc));
                const double rc = lld(r, sc) - al * lld(Ap, sc);
                lst(r, sc, rc);
                const double zz = rc * lld(q, sc);
                rz_new += rc * zz;
                rr_new += rc * rc;
            }
            rz_new = wave_sum(rz_new);
            rr_new = wave_sum(rr_new);
            const double bcoef = rz_new / rz;
            rz = rz_new;
            rr = rr_new;
            wave_sync();
            for (int c = lane; c < n; c += 64) {
                const int sc = lslot(vd, c);
                lst(p, sc, lld(r, sc) * lld(q, sc) + bcoef * lld(p, sc));
            }
            wave_sync();
        }
        for (int c = lane; c < n; c += 64) lst(v.x, lslot(v, c), (T)lld(xb, lslot(vd, c)));
    }
    __syncthreads();
}

// global (cell order) -> LDS (slot order), four loads in flight per thread
template <typename T>
__device__ __forceinline__ void lds_copy_in(const LLev<T> &v, T *dst, const T *src, int planes) {
    const int n = v.n, tot = planes * n, step = blockDim.x;
    auto slot = [&](int e) {
        const int pl = e / n, c = e - pl * n;
        return pl * n + lslot(v, c);
    };
    int e = threadIdx.x;
    for (; e + 3 * step < tot; e += 4 * step) {
        const T v0 = gld(src, e), v1 = gld(src, e + step), v2 = gld(src, e + 2 * step), v3 = gld(src, e + 3 * step);
        lst(dst, slot(e), v0);
        lst(dst, slot(e + step), v1);
        lst(dst, slot(e + 2 * step), v2);
        lst(dst, slot(e + 3 * step), v3);
    }
    for (; e < tot; e += step) lst(dst, slot(e), gld(src, e));
}

template <typename T>
__global__ void __launch_bounds__(kLdsThreads) k_coarse_lds(const LevDesc *__restrict__ dT, const LevDesc *__restrict__ d64,
                                                            const FusedDesc *__restrict__ fd, const ProbState *__restrict__ st,
                                                            int nu_pre, int nu_post) {
    extern __shared__ double lds_raw[];
    char *raw = (char *)lds_raw;
    const FusedDesc f = fd[blockIdx.x];
    if (!gld(&st[f.prob].active, 0)) return;
    const int base = f.base, lc = f.lc, L = f.L;
    // load: level lc's x and b (b + Dirichlet lifting on a finest level), every
    // resident level's assembled row and mask
    for (int l = lc; l < L; l++) {
        const LevDesc &D = dT[base + l];
        const LLev<T> v = lds_lev<T>(raw, dT, base, lc, l);
        if (v.dg) lds_copy_in(v, v.dg, (const T *)D.sten, 7);   // dg and the weight planes are contiguous
        if (v.tab && threadIdx.x < kUniTab) {
            const T d = llev_diag_uni(v, (int)threadIdx.x);
            lst(v.tab, threadIdx.x, d);
            lst(v.tab, kUniTab + threadIdx.x, (T)1 / d);
        }
        if (threadIdx.x == 0) lst(v.x, v.n, (T)0);
        if (v.m)
            for (int c = threadIdx.x; c < v.n; c += blockDim.x) lst(const_cast<uint8_t *>(v.m), lslot(v, c), gld(D.mask, c));
        if (l == lc) {
            // a coarse level enters with the zero iterate the restriction wrote
            if (lc == 0) lds_copy_in(v, v.x, (const T *)D.x, 1);
            else for (int c = threadIdx.x; c < v.n; c += blockDim.x) lst(v.x, c, (T)0);
            if (D.lift) {
                for (int c = threadIdx.x; c < v.n; c += blockDim.x) {
                    int i, j, k;
                    cell_ijk(D, c, i, j, k);
                    lst(v.b, lslot(v, c), (T)((double)gld((const T *)D.b, c) + lift_term(D, i, j, k)));
                }
            } else {
                lds_copy_in(v, v.b, (const T *)D.b, 1);
            }
        }
    }
    size_t used = 0;
    for (int m = lc; m < L; m++)
        used += lds_level_bytes(dT[base + m].ncell, sizeof(T), dT[base + m].has_mask, dT[base + m].sten != nullptr);
    double *pcg = (double *)(raw + used);
    const LevDesc &B64 = d64[base + L - 1];
    const size_t ab = lds_al16((size_t)B64.ncell * sizeof(double)) / sizeof(double);
    LLev<double> vd = lds_lev<double>(raw, d64, base, L - 1, L - 1);   // FP64 view of the bottom row
    if constexpr (sizeof(T) == 4) {
        vd.dg = nullptr;
        vd.w = nullptr;
        if (L >= 2 && B64.sten) {
            vd.dg = pcg + 5 * ab;
            vd.w = vd.dg + B64.ncell;
            lds_copy_in(vd, vd.dg, (const double *)B64.sten, 7);
        }
    }
    __syncthreads();
    if (L == 1) {
        const LLev<T> v = lds_lev<T>(raw, dT, base, 0, 0);
        for (int s = 0; s < nu_pre + nu_post; s++) { llev_sweep(v, 0); llev_sweep(v, 1); }
    } else {
        for (int l = lc; l < L - 1; l++) {
            const LLev<T> v = lds_lev<T>(raw, dT, base, lc, l);
            for (int s = 0; s < nu_pre; s++) { llev_sweep(v, 0); llev_sweep(v, 1); }
            const LLev<T> cv = lds_lev<T>(raw, dT, base, lc, l + 1);
            for (int cc = threadIdx.x; cc < cv.n; cc += blockDim.x) {
                int I, J, K;
                llev_ijk(cv, cc, I, J, K);
                const int c0 = 2 * I + v.nx * 2 * J + v.nxy * 2 * K;
                T sum = 0;
                sum += llev_resid(v, c0);
                sum += llev_resid(v, c0 + 1);
                sum += llev_resid(v, c0 + v.nx);
                sum += llev_resid(v, c0 + v.nx + 1);
                sum += llev_resid(v, c0 + v.nxy);
                sum += llev_resid(v, c0 + v.nxy + 1);
                sum += llev_resid(v, c0 + v.nxy + v.nx);
                sum += llev_resid(v, c0 + v.nxy + v.nx + 1);
                const int sc = lslot(cv, cc);
                lst(cv.b, sc, llev_valid(cv, cc) ? (T)0.125 * sum : (T)0);
                lst(cv.x, sc, (T)0);
            }
            __syncthreads();
        }
        {
            const LLev<T> v = lds_lev<T>(raw, dT, base, lc, L - 1);
            if constexpr (sizeof(T) == 4) llev_pcg(v, vd, pcg);
            else llev_pcg(v, v, pcg);
        }
        for (int l = L - 2; l >= lc; l--) {
            const LLev<T> v = lds_lev<T>(raw, dT, base, lc, l);
            const LLev<T> cv = lds_lev<T>(raw, dT, base, lc, l + 1);
            for (int c = threadIdx.x; c < v.n; c += blockDim.x) {
                if (!llev_valid(v, c)) continue;
                int i, j, k;
                llev_ijk(v, c, i, j, k);
                const int sc = lslot(v, c);
                lst(v.x, sc, lld(v.x, sc) + lld(cv.x, lslot(cv, (i >> 1) + cv.nx * (j >> 1) + cv.nxy * (k >> 1))));
            }
            __syncthreads();
            for (int s = 0; s < nu_post; s++) { llev_sweep(v, 0); llev_sweep(v, 1); }
        }
    }
    {
        const LLev<T> v = lds_lev<T>(raw, dT, base, lc, lc);
        T *gx = (T *)dT[base + lc].x;
        for (int c = threadIdx.x; c < v.n; c += blockDim.x) gst(gx, c, lld(v.x, lslot(v, c)));
    }
}

// Assembled rows of every LDS-resident level (one workgroup per problem):
// the diagonal, then the six neighbour weights in the order x-, x+, y-, y+,
// z-, z+, by the same rules as row_terms.  FP32 hierarchies also get the
// bottom level's FP64 row for the bottom CG.
template <typename T>
__device__ void stencil_rows(const LevDesc &L, T *out) {
    const int n = L.ncell;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int i, j, k;
        cell_ijk(L, c, i, j, k);
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        T dg = L.var_alpha ? gld(Coef<T>::al(L), c) : (T)L.alpha_c;
        const T bc = (T)L.beta_c;
        const long fxrow = (long)(nx + 1) * (j + (long)ny * k);
        const long fyrow = (long)nx * (j + (long)(ny + 1) * k);
        const long fzpl = (long)nx * j;
        const bool inside[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1};
        const int nbi[6] = {i > 0 ? c - 1 : c + nx - 1, i < nx - 1 ? c + 1 : c - (nx - 1),
                            j > 0 ? c - nx : c + nx * (ny - 1), j < ny - 1 ? c + nx : c - nx * (ny - 1),
                            k > 0 ? c - L.nxy : c + L.nxy * (nz - 1), k < nz - 1 ? c + L.nxy : c - L.nxy * (nz - 1)};
#pragma unroll
        for (int f = 0; f < 6; f++) {
            T beta;
            if (!L.var_beta) beta = bc;
            else if (f == 0) beta = gld(Coef<T>::bx(L), fxrow + i);
            else if (f == 1) beta = gld(Coef<T>::bx(L), fxrow + i + 1);
            else if (f == 2) beta = gld(Coef<T>::by(L), fyrow + i);
            else if (f == 3) beta = gld(Coef<T>::by(L), fyrow + i + nx);
            else if (f == 4) beta = gld(Coef<T>::bz(L), fzpl + i + (long)L.nxy * k);
            else beta = gld(Coef<T>::bz(L), fzpl + i + (long)L.nxy * (k + 1));
            const T cf = beta * (T)(f < 2 ? L.idx2 : (f < 4 ? L.idy2 : L.idz2));
            T wv = 0;
            if (inside[f] || L.kind[f] == VD_BC_PERIODIC) {
                if (L.has_mask && !gld(L.mask, nbi[f])) dg += (T)2 * cf;
                else { dg += cf; wv = cf; }
            } else if (L.kind[f] == VD_BC_DIRICHLET) {
                dg += (T)2 * cf;
            }
            gst(out, (long)(f + 1) * n + c, wv);
        }
        gst(out, (long)c, dg);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_stencils(const LevDesc *__restrict__ dT, const LevDesc *__restrict__ d64,
                                                  const FusedDesc *__restrict__ fd) {
    const FusedDesc f = fd[blockIdx.x];
    for (int l = f.lc; l < f.L; l++)
        if (dT[f.base + l].sten) stencil_rows<T>(dT[f.base + l], (T *)dT[f.base + l].sten);
    if constexpr (sizeof(T) == 4)
        if (f.L >= 2 && d64[f.base + f.L - 1].sten)
            stencil_rows<double>(d64[f.base + f.L - 1], (double *)d64[f.base + f.L - 1].sten);
}

// -------------------------------------------------------- setup kernels
__device__ __forceinline__ double harmonic(double a, double b) { return (a + b == 0.0) ? 0.0 : 2.0 * a * b / (a + b); }

// finest-level face coefficients from the cell coefficient (harmonic mean;
// a non-periodic domain face takes the boundary cell's value)
__global__ void __launch_bounds__(kBlock) k_faces0(const double *__restrict__ beta, int nx, int ny, int nz, int perx,
                                                   int pery, int perz, double *bx, double *by, double *bz, float *bx32,
                                                   float *by32, float *bz32) {
    long nfx = (long)(nx + 1) * ny * nz, nfy = (long)nx * (ny + 1) * nz, nfz = (long)nx * ny * (nz + 1);
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nxy = (long)nx * ny;
    if (q < nfx) {
        int i = (int)(q % (nx + 1));
        long r = q / (nx + 1);
        int j = (int)(r % ny), k = (int)(r / ny);
        long row = nx * (j + (long)ny * k);
        double v;
        if (i > 0 && i < nx) v = harmonic(beta[row + i - 1], beta[row + i]);
        else if (perx) v = harmonic(beta[row + nx - 1], beta[row]);
        else v = beta[row + (i == 0 ? 0 : nx - 1)];
        bx[q] = v;
        if (bx32) bx32[q] = (float)v;
        return;
    }
    q -= nfx;
    if (q < nfy) {
        int i = (int)(q % nx);
        long r = q / nx;
        int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
        long pl = nxy * k + i;
        double v;
        if (j > 0 && j < ny) v = harmonic(beta[pl + (long)nx * (j - 1)], beta[pl + (long)nx * j]);
        else if (pery) v = harmonic(beta[pl + (long)nx * (ny - 1)], beta[pl]);
        else v = beta[pl + (long)nx * (j == 0 ? 0 : ny - 1)];
        by[q] = v;
        if (by32) by32[q] = (float)v;
        return;
    }
    q -= nfy;
    if (q < nfz) {
        long col = q % nxy;
        int k = (int)(q / nxy);
        double v;
        if (k > 0 && k < nz) v = harmonic(beta[col + nxy * (k - 1)], beta[col + nxy * k]);
        else if (perz) v = harmonic(beta[col + nxy * (nz - 1)], beta[col]);
        else v = beta[col + nxy * (k == 0 ? 0 : nz - 1)];
        bz[q] = v;
        if (bz32) bz32[q] = (float)v;
    }
}

// coarse faces (mean of 4 coincident fine faces), alpha (mean of 8 children),
// mask (valid iff all 8 children are); FP64 plus optional FP32 copies
__global__ void __launch_bounds__(kBlock) k_coarsen(LevDesc F, LevDesc C, double *bx, double *by, double *bz, double *al,
                                                    uint8_t *mk, float *bx32, float *by32, float *bz32, float *al32) {
    const int nx = C.nx, ny = C.ny, nz = C.nz, fx = F.nx, fy = F.ny;
    long nfx = C.var_beta ? (long)(nx + 1) * ny * nz : 0;
    long nfy = C.var_beta ? (long)nx * (ny + 1) * nz : 0;
    long nfz = C.var_beta ? (long)nx * ny * (nz + 1) : 0;
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nfx) {
        int i = (int)(q % (nx + 1));
        long r = q / (nx + 1);
        int j = (int)(r % ny), k = (int)(r / ny);
        double s = 0.0;
        for (int kk = 0; kk < 2; kk++)
            for (int jj = 0; jj < 2; jj++) s += gld(F.bx, (long)(2 * i) + (long)(fx + 1) * ((2 * j + jj) + (long)fy * (2 * k + kk)));
        bx[q] = 0.25 * s;
        if (bx32) bx32[q] = (float)(0.25 * s);
        return;
    }
    q -= nfx;
    if (q < nfy) {
        int i = (int)(q % nx);
        long r = q / nx;
        int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
        double s = 0.0;
        for (int kk = 0; kk < 2; kk++)
            for (int ii = 0; ii < 2; ii++) s += gld(F.by, (long)(2 * i + ii) + (long)fx * ((2 * j) + (long)(fy + 1) * (2 * k + kk)));
        by[q] = 0.25 * s;
        if (by32) by32[q] = (float)(0.25 * s);
        return;
    }
    q -= nfy;
    if (q < nfz) {
        int i = (int)(q % nx);
        long r = q / nx;
        int j = (int)(r % ny), k = (int)(r / ny);
        double s = 0.0;
        for (int jj = 0; jj < 2; jj++)
            for (int ii = 0; ii < 2; ii++) s += gld(F.bz, (long)(2 * i + ii) + (long)fx * ((2 * j + jj) + (long)fy * (2 * k)));
        bz[q] = 0.25 * s;
        if (bz32) bz32[q] = (float)(0.25 * s);
        return;
    }
    q -= nfz;
    if (q < (long)C.ncell) {
        int c = (int)q;
        int i, j, k;
        cell_ijk(C, c, i, j, k);
        double s = 0.0;
        int valid = 1;
        for (int kk = 0; kk < 2; kk++)
            for (int jj = 0; jj < 2; jj++)
                for (int ii = 0; ii < 2; ii++) {
                    long f = (long)(2 * i + ii) + (long)fx * ((2 * j + jj) + (long)fy * (2 * k + kk));
                    if (C.var_alpha) s += gld(F.alpha, f);
                    if (C.has_mask) valid = valid && gld(F.mask, f);
                }
        if (C.var_alpha) { al[c] = 0.125 * s; if (al32) al32[c] = (float)(0.125 * s); }
        if (C.has_mask) mk[c] = (uint8_t)valid;
    }
}

__global__ void __launch_bounds__(kBlock) k_to_f32(const double *__restrict__ a, float *__restrict__ b, long n) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (float)a[q];
}

// ---------------------------------------------------------- host engine
struct HLevel {
    int nx, ny, nz;
    DevBuf<double> bx, by, bz, alpha, x, b;
    DevBuf<float> bx32, by32, bz32, alpha32, x32, b32;
    DevBuf<uint8_t> mask;
    DevBuf<double> st64;     // assembled rows (LDS-resident levels; FP64 bottom of FP32 hierarchies)
    DevBuf<float> st32;
    DevBuf<double> x2;       // alternate iterate of the fused sweeps (levels smoothed by k_sweep25)
    DevBuf<float> x2_32;
};

struct HProblem {
    int L = 1, lc = 0;
    int lds_lc = -1;            // first LDS-resident coarse level (-1: none fits)
    size_t lds_bytes = 0;
    bool var_beta = false, var_alpha = false, has_mask = false;
    std::vector<HLevel> lv;
    DevBuf<double> pcg;
};

struct HPlan {
    DevBuf<int> ids, prefix;
    int nd = 0, ntiles = 0;
    int kz = 0;                  // 2.5D tiled plans: planes per workgroup
    bool uni = false;            // every problem in the plan has uniform coefficients and no mask
    std::vector<int> h_ids, h_prefix;
    DevBuf<int> gbase;           // split norm plans: first partial slot of each descriptor in the full plan
    Plan dev() const { return Plan{ids.p, prefix.p, nd, ntiles, gbase.p}; }
};

struct Solver {
    int nprob = 0, Lmax = 0, prec = VD_FP64;
    std::vector<HProblem> probs;
    DevBuf<LevDesc> d64, d32;
    std::vector<LevDesc> h64, h32;
    LevDesc *pin64 = nullptr, *pin32 = nullptr;   // host staging of the descriptors
    DevBuf<ProbState> st;
    ProbState *pin_st = nullptr;
    bool pinned = true;           // staging in pinned memory (ordinary host memory without allocation)
    DevBuf<double> partials, partials_b;
    DevBuf<FusedDesc> fused;
    int nfused = 0;
    size_t pcg_lds_bytes = 0;     // dynamic LDS of the fused kernel (0: CG vectors in global memory)
    bool lds_mode = false;        // coarse levels held in LDS (k_coarse_lds)
    HPlan rb0;                    // finest levels of the uniform problems, parity-split FP32 corrections (k_rb32)
    bool rb_on = false;           // those corrections are currently held parity-split
    size_t lds_bytes = 0;         // its dynamic LDS
    DevBuf<int> prob_of;
    HPlan all0;                                  // finest level, every problem
    std::vector<HPlan> pre, restr, prolong;      // per level
    HPlan all0_25;                               // finest level as 2.5D tiles (residual norms), if usable
    std::vector<HPlan> pre25;                    // smoother levels as 2.5D tiles, if usable
    HPlan norm25u, norm25g;                      // all0_25 split the same way (partials keep the full plan's slots)
    std::vector<HPlan> pre25u, pre25g;           // the same split into uniform-coefficient and other problems
                                                 // (built only when a level mixes both)
    std::vector<char> key;                       // problem bytes the descriptors were built from
    bool rows_valid = false;                     // assembled LDS rows match the descriptors
    hipGraphExec_t gexec = nullptr;              // one captured cycle (VD_MG_GRAPH)
    std::string gkey;                            // options the graph was captured with
    bool tuned = false;                          // smoother tiles autotuned (VD_MG_AUTOTUNE)
    int nu_pre = -1, nu_post = -1;               // smoothing schedule chosen by VD_MG_TUNE_NU (-1: not tuned)
    bool persistent = false;                     // colour passes in persistent launches (VD_MG_PERSISTENT)
    int last_iters = 2;                          // cycles (refinement steps) the previous solve needed
    std::vector<int> use_fused;                  // per level: fused out-of-place sweeps instead of colour passes
    // timed launches of the current solve, credited with the algorithmic
    // bytes of the problems still active at that point once the solve ends
    struct LaunchRec { const char *family; const HPlan *plan; bool fp32; int kind; double factor; int it, phase; };
    std::vector<LaunchRec> recs;
    int cur_it = 0, cur_phase = 2;     // phase 0: residual check of iteration it, 1: its cycle(s), 2: set-up
    bool aligned = true;                         // finest-level unknowns 16-byte aligned (row-pair loads)
    ~Solver() {
        stage_free(pin64, pinned);
        stage_free(pin32, pinned);
        stage_free(pin_st, pinned);
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

template <typename T>
__global__ void k_coarse_lds(const LevDesc *__restrict__ dT, const LevDesc *__restrict__ d64,
                             const struct FusedDesc *__restrict__ fd, const ProbState *__restrict__ st, int nu_pre, int nu_post);

// LDS a workgroup may allocate on this device; the LDS-resident coarse
// kernel is allowed to use all of it
static size_t lds_limit_bytes() {
    static size_t cached = 0;
    if (cached) return cached;
    int dev = 0, v = 0;
    VD_HIP(hipGetDevice(&dev));
    VD_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    size_t lim = v > 0 ? (size_t)v : 65536;
    if (lim > 65536) {
        if (hipFuncSetAttribute((const void *)k_coarse_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim - 1024) !=
                hipSuccess ||
            hipFuncSetAttribute((const void *)k_coarse_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim - 1024) !=
                hipSuccess) {
            (void)hipGetLastError();
            lim = 65536;
        }
    }
    cached = lim;
    return cached;
}

static void upload_plan(HPlan &pl, hipStream_t s) {
    pl.nd = (int)pl.h_ids.size();
    pl.ntiles = pl.h_prefix.empty() ? 0 : pl.h_prefix.back();
    if (pl.nd == 0) return;
    pl.ids.alloc(pl.nd);
    pl.prefix.alloc(pl.nd + 1);
    VD_HIP(hipMemcpyAsync(pl.ids.p, pl.h_ids.data(), sizeof(int) * pl.nd, hipMemcpyHostToDevice, s));
    VD_HIP(hipMemcpyAsync(pl.prefix.p, pl.h_prefix.data(), sizeof(int) * (pl.nd + 1), hipMemcpyHostToDevice, s));
    VD_HIP(hipStreamSynchronize(s));
}

static void plan_add(HPlan &pl, int id, long units, int per_tile) {
    if (pl.h_prefix.empty()) pl.h_prefix.push_back(0);
    pl.h_ids.push_back(id);
    pl.h_prefix.push_back(pl.h_prefix.back() + ceil_div(units, per_tile));
}

static int count_levels(const vd_grid &g, int requested) {
    if (requested > 0) {
        int nx = g.nx, ny = g.ny, nz = g.nz;
        for (int l = 1; l < requested; l++) {
            if (nx % 2 || ny % 2 || nz % 2) return -1;
            nx /= 2; ny /= 2; nz /= 2;
        }
        return requested;
    }
    int nl = 1, nx = g.nx, ny = g.ny, nz = g.nz;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx > 4 && ny > 4 && nz > 4) {
        nx /= 2; ny /= 2; nz /= 2; nl++;
    }
    return nl;
}

static void validate(int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    VD_CHECK(nprob >= 1, "nprob must be >= 1");
    VD_CHECK(probs != nullptr && o != nullptr, "null problems or options");
    VD_CHECK(o->precision == VD_FP64 || o->precision == VD_FP32_IR, "unknown precision");
    VD_CHECK(o->nu_pre >= 0 && o->nu_post >= 0 && o->nu_pre + o->nu_post >= 1, "need at least one smoothing sweep");
    VD_CHECK(o->max_cycles >= 0 && o->fixed_cycles >= 0, "negative cycle counts");
    VD_CHECK(o->guess == VD_GUESS_GIVEN || o->guess == VD_GUESS_ZERO, "guess must be GIVEN or ZERO here");
    VD_CHECK(o->precision == VD_FP64 || o->ir_inner >= 1, "ir_inner must be >= 1");
    for (int p = 0; p < nprob; p++) {
        const vd_problem &P = probs[p];
        const vd_grid &g = P.grid;
        VD_CHECK(g.nx >= 1 && g.ny >= 1 && g.nz >= 1, "grid dimensions must be positive");
        VD_CHECK((long)g.nx * g.ny * g.nz < (1L << 31) / 2, "grid too large");
        VD_CHECK(g.dx > 0 && g.dy > 0 && g.dz > 0, "mesh spacing must be positive");
        for (int d = 0; d < 3; d++) {
            int a = P.bc.kind[2 * d], b = P.bc.kind[2 * d + 1];
            VD_CHECK(a >= 0 && a <= 3 && b >= 0 && b <= 3, "unknown boundary kind");
            VD_CHECK((a == VD_BC_PERIODIC) == (b == VD_BC_PERIODIC), "periodic must be set on both faces of a direction");
        }
        VD_CHECK(P.rhs != nullptr && P.x != nullptr, "rhs and x are required");
        const int L = count_levels(g, o->n_levels);
        VD_CHECK(L >= 1 && L <= 16, "n_levels not compatible with the grid (dimensions must stay even, at most 16 levels)");
        // red-black ordering is only a valid parallel colouring if a periodic
        // direction has an even number of cells on every smoothed level
        const int nd[3] = {g.nx, g.ny, g.nz};
        for (int d = 0; d < 3; d++) {
            if (P.bc.kind[2 * d] != VD_BC_PERIODIC) continue;
            for (int l = 0; l <= std::max(L - 2, 0); l++)
                VD_CHECK(((nd[d] >> l) % 2) == 0, "periodic direction needs an even cell count on every smoothed level");
        }
        bool dir = false;
        for (int f = 0; f < 6; f++) dir = dir || P.bc.kind[f] == VD_BC_DIRICHLET;
        if (!P.alpha && P.alpha_c == 0.0 && !P.mask && !dir)
            throw Error{VD_ESINGULAR, "singular operator: alpha = 0, no Dirichlet face and no mask (problem " +
                                          std::to_string(p) + ")"};
    }
}

static std::vector<char> problem_key(int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    std::vector<char> k(sizeof(vd_problem) * nprob + sizeof(int) * 3);
    memcpy(k.data(), probs, sizeof(vd_problem) * nprob);
    int extra[3] = {o->precision, o->n_levels, nprob};
    memcpy(k.data() + sizeof(vd_problem) * nprob, extra, sizeof(extra));
    return k;
}

static std::string shape_key(int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    std::string s = "mg:" + std::to_string(o->precision) + ":" + std::to_string(o->n_levels) + ":";
    for (int p = 0; p < nprob; p++) {
        const vd_problem &P = probs[p];
        char buf[160];
        snprintf(buf, sizeof buf, "%d,%d,%d,%d%d%d;", P.grid.nx, P.grid.ny, P.grid.nz, P.beta != nullptr,
                 P.alpha != nullptr, P.mask != nullptr);
        s += buf;
        for (int f = 0; f < 6; f++) s += std::to_string(P.bc.kind[f]);
    }
    return s;
}

static LevDesc make_desc(const HProblem &H, const vd_problem &P, int l, int prob, bool fp32) {
    const HLevel &V = H.lv[l];
    LevDesc D;
    memset(&D, 0, sizeof(D));
    D.nx = V.nx; D.ny = V.ny; D.nz = V.nz;
    D.nxy = V.nx * V.ny;
    D.ncell = V.nx * V.ny * V.nz;
    for (int f = 0; f < 6; f++) { D.kind[f] = P.bc.kind[f]; D.gval[f] = P.bc.value[f]; }
    D.var_beta = H.var_beta; D.var_alpha = H.var_alpha; D.has_mask = H.has_mask;
    D.lift = (l == 0 && !fp32) ? 1 : 0;
    D.prob = prob;
    // spacing from the problem of this call (a cached hierarchy is shared by
    // every problem of the same shape, whatever its mesh spacing)
    const double dx = P.grid.dx * (double)(1 << l), dy = P.grid.dy * (double)(1 << l), dz = P.grid.dz * (double)(1 << l);
    D.idx2 = 1.0 / (dx * dx); D.idy2 = 1.0 / (dy * dy); D.idz2 = 1.0 / (dz * dz);
    D.beta_c = P.beta_c; D.alpha_c = P.alpha_c;
    D.bx = V.bx.p; D.by = V.by.p; D.bz = V.bz.p;
    D.alpha = (l == 0) ? P.alpha : V.alpha.p;
    D.bx32 = V.bx32.p; D.by32 = V.by32.p; D.bz32 = V.bz32.p; D.alpha32 = V.alpha32.p;
    D.mask = (l == 0) ? P.mask : V.mask.p;
    if (fp32) { D.x = V.x32.p; D.b = V.b32.p; }
    else if (l == 0) { D.x = P.x; D.b = P.rhs; }
    else { D.x = V.x.p; D.b = V.b.p; }
    D.sten = fp32 ? (void *)V.st32.p : (void *)V.st64.p;
    D.x2 = fp32 ? (void *)V.x2_32.p : (void *)V.x2.p;
    return D;
}

// 2.5D tiled plan over (descriptor id, level) items: usable when every
// level has an even nx.  kz = planes per workgroup; 0 picks the deepest
// tile that still gives a launch >= 2048 workgroups.
static void build_plan25(vd_ctx *ctx, HPlan &out, const std::vector<std::pair<int, const HLevel *>> &items, int force_kz,
                         int max_kz = 8) {
    out = HPlan{};
    if (items.empty()) return;
    for (auto &it : items) if (it.second->nx % 2) return;
    int kz = force_kz;
    if (kz <= 0) {
        // the deepest of 8, 4, 2 planes (at most max_kz) that still gives
        // 2048 tiles (16 planes measured slower for the FP64 residual checks)
        kz = 2;
        for (int cand : {8, 4, 2}) {
            if (cand > max_kz) continue;
            long tot = 0;
            for (auto &it : items)
                tot += (long)ceil_div(it.second->nx, kT25X) * ceil_div(it.second->ny, kT25Y) * ceil_div(it.second->nz, cand);
            if (tot >= 2048 || cand == 2) { kz = cand; break; }
        }
    }
    out.kz = kz;
    for (auto &it : items)
        plan_add(out, it.first, (long)ceil_div(it.second->nx, kT25X) * ceil_div(it.second->ny, kT25Y) *
                                    ceil_div(it.second->nz, kz), 1);
    upload_plan(out, ctx->stream);
}

// A level whose tiled plan mixes uniform-coefficient problems with others
// is also planned as two halves, so the uniform ones run in the leaner
// kernel (the colour pass is launched once per half).  Each half picks its
// own tile depth, so a half of few problems still fills the device.
static void split25(vd_ctx *ctx, Solver &S, int l) {
    HPlan &P = S.pre25[l];
    S.pre25u[l] = HPlan{};
    S.pre25g[l] = HPlan{};
    if (!P.nd || P.uni) return;
    std::vector<std::pair<int, const HLevel *>> u, g;
    for (int id : S.pre[l].h_ids) {
        const HProblem &H = S.probs[id / S.Lmax];
        (!H.var_beta && !H.var_alpha && !H.has_mask ? u : g).push_back({id, &H.lv[id % S.Lmax]});
    }
    if (u.empty() || g.empty()) return;
    build_plan25(ctx, S.pre25u[l], u, 0);
    S.pre25u[l].uni = true;
    build_plan25(ctx, S.pre25g[l], g, 0);
}

static std::shared_ptr<Solver> build_solver(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    auto S = std::make_shared<Solver>();
    S->nprob = nprob;
    S->prec = o->precision;
    bool ir = o->precision == VD_FP32_IR;
    size_t lds_limit = lds_limit_bytes() - 1024;   // leave room for the static reduction buffer
    S->probs.resize(nprob);
    for (int p = 0; p < nprob; p++) {
        HProblem &H = S->probs[p];
        const vd_problem &P = probs[p];
        H.L = count_levels(P.grid, o->n_levels);
        H.var_beta = P.beta != nullptr;
        H.var_alpha = P.alpha != nullptr;
        H.has_mask = P.mask != nullptr;
        H.lv.resize(H.L);
        for (int l = 0; l < H.L; l++) {
            HLevel &V = H.lv[l];
            V.nx = P.grid.nx >> l; V.ny = P.grid.ny >> l; V.nz = P.grid.nz >> l;
            long n = (long)V.nx * V.ny * V.nz;
            if (H.var_beta) {
                V.bx.alloc((size_t)(V.nx + 1) * V.ny * V.nz);
                V.by.alloc((size_t)V.nx * (V.ny + 1) * V.nz);
                V.bz.alloc((size_t)V.nx * V.ny * (V.nz + 1));
                if (ir) { V.bx32.alloc(V.bx.n); V.by32.alloc(V.by.n); V.bz32.alloc(V.bz.n); }
            }
            if (H.var_alpha) {
                if (l > 0) V.alpha.alloc(n);
                if (ir) V.alpha32.alloc(n);
            }
            if (H.has_mask && l > 0) V.mask.alloc(n);
            if (l > 0) { V.x.alloc(n); V.b.alloc(n); }
            if (ir) { V.x32.alloc(n); V.b32.alloc(n); }
        }
        H.lc = H.L == 1 ? (((long)H.lv[0].nx * H.lv[0].ny * H.lv[0].nz <= kCoarseMax) ? 0 : 1) : H.L - 1;
        for (int l = 0; l < H.L - 1; l++)
            if ((long)H.lv[l].nx * H.lv[l].ny * H.lv[l].nz <= kCoarseMax) { H.lc = l; break; }
        // LDS-resident coarse levels: the largest set of coarse levels whose
        // unknowns, right-hand sides, assembled rows and CG vectors fit in one
        // workgroup's LDS
        {
            const size_t sT = ir ? sizeof(float) : sizeof(double);
            const long nb = H.L >= 2 ? (long)H.lv[H.L - 1].nx * H.lv[H.L - 1].ny * H.lv[H.L - 1].nz : 0;
            int best = -1;
            size_t best_bytes = 0;
            const bool rows = H.var_beta || H.var_alpha || H.has_mask;
            for (int l = H.L - 1; l >= 0; l--) {
                size_t need = H.L >= 2 ? lds_pcg_bytes(nb, ir && rows) : 0;
                for (int m = l; m < H.L; m++)
                    need += lds_level_bytes((long)H.lv[m].nx * H.lv[m].ny * H.lv[m].nz, sT, H.has_mask, rows);
                if (need > lds_limit) break;
                best = l;
                best_bytes = need;
            }
            // a single large level is smoothed by the grid kernels, not fused
            H.lds_lc = (H.L == 1 && best < 0) ? -2 : best;
            H.lds_bytes = best_bytes;
        }
        if (H.L >= 2) {
            const HLevel &B = H.lv[H.L - 1];
            H.pcg.alloc((size_t)6 * B.nx * B.ny * B.nz);
        }
        S->Lmax = std::max(S->Lmax, H.L);
    }
    // use the LDS-resident coarse kernel when every problem's bottom fits;
    // its coarse boundary then replaces the global-memory one
    {
        bool all = true;
        for (auto &H : S->probs) all = all && (H.lds_lc >= 0 || H.lds_lc == -2);
        if (all) {
            S->lds_mode = true;
            for (auto &H : S->probs) {
                H.lc = H.lds_lc >= 0 ? H.lds_lc : 1;
                if (H.lds_lc >= 0) S->lds_bytes = std::max(S->lds_bytes, H.lds_bytes);
                // uniform-coefficient problems form their rows on the fly
                if (!(H.var_beta || H.var_alpha || H.has_mask)) continue;
                for (int l = H.lc; l < H.L; l++) {
                    HLevel &V = H.lv[l];
                    const size_t n7 = (size_t)7 * V.nx * V.ny * V.nz;
                    if (ir) V.st32.alloc(n7);
                    else V.st64.alloc(n7);
                    if (ir && l == H.L - 1 && H.L >= 2) V.st64.alloc(n7);
                }
            }
        }
    }
    int Lmax = S->Lmax;
    S->h64.assign((size_t)nprob * Lmax, LevDesc{});
    S->h32.assign((size_t)nprob * Lmax, LevDesc{});
    S->d64.alloc(S->h64.size());
    if (ir) S->d32.alloc(S->h32.size());
    S->pin64 = (LevDesc *)stage_alloc(sizeof(LevDesc) * S->h64.size(), &S->pinned);
    if (ir) S->pin32 = (LevDesc *)stage_alloc(sizeof(LevDesc) * S->h32.size(), &S->pinned);
    S->st.alloc(nprob);
    S->pin_st = (ProbState *)stage_alloc(sizeof(ProbState) * nprob, &S->pinned);
    // plans
    S->pre.resize(Lmax);
    S->restr.resize(Lmax);
    S->prolong.resize(Lmax);
    std::vector<FusedDesc> fds;
    std::vector<int> prob_of;
    long max_bottom = 0;
    for (int p = 0; p < nprob; p++) {
        HProblem &H = S->probs[p];
        int base = p * Lmax;
        long n0 = (long)H.lv[0].nx * H.lv[0].ny * H.lv[0].nz;
        plan_add(S->all0, base, n0, kNormU * kBlock);
        prob_of.push_back(p);
        for (int l = 0; l < H.lc; l++) {
            long n = (long)H.lv[l].nx * H.lv[l].ny * H.lv[l].nz;
            plan_add(S->pre[l], base + l, (H.lv[l].nx % 2 == 0) ? (n + 1) / 2 : n, kGsrbU * kBlock);
            if (H.L >= 2) {
                long nc = (long)H.lv[l + 1].nx * H.lv[l + 1].ny * H.lv[l + 1].nz;
                plan_add(S->restr[l], base + l + 1, nc, kRestrictU * kBlock);
                plan_add(S->prolong[l], base + l, n, kProlongU * kBlock);
            }
        }
        if (H.lc < H.L) fds.push_back(FusedDesc{p, H.lc, H.L, base, H.pcg.p});
        if (H.L >= 2) {
            const HLevel &Bt = H.lv[H.L - 1];
            max_bottom = std::max(max_bottom, (long)Bt.nx * Bt.ny * Bt.nz);
        }
    }
    auto build25 = [&](HPlan &out, const std::vector<std::pair<int, const HLevel *>> &items) {
        build_plan25(ctx, out, items, 0);
    };
    {
        std::vector<std::pair<int, const HLevel *>> items;
        for (int p = 0; p < nprob; p++) items.push_back({p * Lmax, &S->probs[p].lv[0]});
        build25(S->all0_25, items);
    }
    S->pre25.resize(Lmax);
    S->use_fused.assign(Lmax, 0);
    for (int l = 0; l < Lmax; l++) {
        std::vector<std::pair<int, const HLevel *>> items;
        for (int id : S->pre[l].h_ids) items.push_back({id, &S->probs[id / Lmax].lv[id % Lmax]});
        build25(S->pre25[l], items);
    }
    auto mark_uni = [&](HPlan &pl) {
        pl.uni = pl.nd > 0;
        for (int id : pl.h_ids) {
            const HProblem &H = S->probs[id / Lmax];
            pl.uni = pl.uni && !H.var_beta && !H.var_alpha && !H.has_mask;
        }
    };
    mark_uni(S->all0_25);
    for (int l = 0; l < Lmax; l++) mark_uni(S->pre25[l]);
    S->pre25u.resize(Lmax);
    S->pre25g.resize(Lmax);
    for (int l = 0; l < Lmax; l++) split25(ctx, *S, l);
    // refinement corrections of the uniform problems' finest levels held
    // parity-split: every such problem smoothed by the tiled passes needs
    // nx % 4 == 0 (whole position pairs per half-row)
    if (ir && Lmax > 0) {
        std::vector<std::pair<int, const HLevel *>> items;
        bool ok = true;
        for (int id : S->pre[0].h_ids) {
            const HProblem &H = S->probs[id / Lmax];
            if (H.var_beta || H.var_alpha || H.has_mask) continue;
            const HLevel &V = H.lv[0];
            ok = ok && V.nx % 4 == 0;
            items.push_back({id, &V});
        }
        if (ok && !items.empty()) {
            int kz = 2;
            for (int cand : {16, 8, 4, 2}) {
                long tot = 0;
                for (auto &it : items)
                    tot += (long)ceil_div(it.second->nx / 2, kT25X) * ceil_div(it.second->ny, kT25Y) * ceil_div(it.second->nz, cand);
                if (tot >= 1024 || cand == 2) { kz = cand; break; }
            }
            S->rb0.kz = kz;
            for (auto &it : items)
                plan_add(S->rb0, it.first, (long)ceil_div(it.second->nx / 2, kT25X) * ceil_div(it.second->ny, kT25Y) *
                                               ceil_div(it.second->nz, kz), 1);
            upload_plan(S->rb0, ctx->stream);
            S->rb0.uni = true;
        }
    }
    if (S->all0_25.nd && !S->all0_25.uni) {
        // finest-level residual norms split like the smoother; item p of
        // the full plan is problem p
        std::vector<std::pair<int, const HLevel *>> u, g;
        std::vector<int> gu, gg;
        for (int p = 0; p < nprob; p++) {
            const HProblem &H = S->probs[p];
            const bool uni = !H.var_beta && !H.var_alpha && !H.has_mask;
            (uni ? u : g).push_back({p * Lmax, &H.lv[0]});
            (uni ? gu : gg).push_back(S->all0_25.h_prefix[p]);
        }
        if (!u.empty() && !g.empty()) {
            build_plan25(ctx, S->norm25u, u, S->all0_25.kz);
            build_plan25(ctx, S->norm25g, g, S->all0_25.kz);
            S->norm25u.uni = true;
            for (auto *pr : {&S->norm25u, &S->norm25g}) {
                const std::vector<int> &gb = pr == &S->norm25u ? gu : gg;
                pr->gbase.alloc(gb.size());
                VD_HIP(hipMemcpyAsync(pr->gbase.p, gb.data(), sizeof(int) * gb.size(), hipMemcpyHostToDevice, ctx->stream));
            }
            VD_HIP(hipStreamSynchronize(ctx->stream));   // gu, gg are read by the copies
        }
    }
    upload_plan(S->all0, ctx->stream);
    for (int l = 0; l < Lmax; l++) {
        upload_plan(S->pre[l], ctx->stream);
        upload_plan(S->restr[l], ctx->stream);
        upload_plan(S->prolong[l], ctx->stream);
    }
    S->partials.alloc(std::max(1, std::max(S->all0.ntiles, S->all0_25.ntiles)));
    S->partials_b.alloc(std::max(1, std::max(S->all0.ntiles, S->all0_25.ntiles)));
    S->nfused = (int)fds.size();
    S->pcg_lds_bytes = (max_bottom > 0 && max_bottom <= kPcgLdsCells) ? (size_t)6 * max_bottom * sizeof(double) : 0;
    if (S->nfused) {
        S->fused.alloc(fds.size());
        VD_HIP(hipMemcpyAsync(S->fused.p, fds.data(), sizeof(FusedDesc) * fds.size(), hipMemcpyHostToDevice, ctx->stream));
    }
    S->prob_of.alloc(nprob);
    VD_HIP(hipMemcpyAsync(S->prob_of.p, prob_of.data(), sizeof(int) * nprob, hipMemcpyHostToDevice, ctx->stream));
    VD_HIP(hipStreamSynchronize(ctx->stream));
    return S;
}

static void refresh_descs(vd_ctx *ctx, Solver &S, int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    auto key = problem_key(nprob, probs, o);
    if (key == S.key) return;
    bool ir = S.prec == VD_FP32_IR;
    for (int p = 0; p < nprob; p++)
        for (int l = 0; l < S.probs[p].L; l++) {
            S.h64[(size_t)p * S.Lmax + l] = make_desc(S.probs[p], probs[p], l, p, false);
            if (ir) S.h32[(size_t)p * S.Lmax + l] = make_desc(S.probs[p], probs[p], l, p, true);
        }
    // the stream may still read the pinned staging of a previous call
    VD_HIP(hipStreamSynchronize(ctx->stream));
    memcpy(S.pin64, S.h64.data(), sizeof(LevDesc) * S.h64.size());
    VD_HIP(hipMemcpyAsync(S.d64.p, S.pin64, sizeof(LevDesc) * S.h64.size(), hipMemcpyHostToDevice, ctx->stream));
    if (ir) {
        memcpy(S.pin32, S.h32.data(), sizeof(LevDesc) * S.h32.size());
        VD_HIP(hipMemcpyAsync(S.d32.p, S.pin32, sizeof(LevDesc) * S.h32.size(), hipMemcpyHostToDevice, ctx->stream));
    }
    S.aligned = true;
    for (int p = 0; p < nprob; p++)
        S.aligned = S.aligned && ((uintptr_t)probs[p].x % 16 == 0) && ((uintptr_t)probs[p].rhs % 16 == 0);
    S.key = std::move(key);
    S.rows_valid = false;
    S.rb_on = false;     // rebuilt descriptors are lexicographic
}

// Coefficients of every level from the user's arrays (values may change
// between calls with the same pointers, so this runs on every solve).
static void setup_coefficients(vd_ctx *ctx, Solver &S, const vd_problem *probs) {
    bool ir = S.prec == VD_FP32_IR;
    hipStream_t s = ctx->stream;
    for (int p = 0; p < S.nprob; p++) {
        HProblem &H = S.probs[p];
        const vd_problem &P = probs[p];
        HLevel &V0 = H.lv[0];
        long n0 = (long)V0.nx * V0.ny * V0.nz;
        if (H.var_beta) {
            long nf = (long)(V0.nx + 1) * V0.ny * V0.nz + (long)V0.nx * (V0.ny + 1) * V0.nz + (long)V0.nx * V0.ny * (V0.nz + 1);
            timed(ctx, "setup", 0.0, [&] {
                k_faces0<<<ceil_div(nf, kBlock), kBlock, 0, s>>>(P.beta, V0.nx, V0.ny, V0.nz, P.bc.kind[0] == VD_BC_PERIODIC,
                                                                  P.bc.kind[2] == VD_BC_PERIODIC, P.bc.kind[4] == VD_BC_PERIODIC,
                                                                  V0.bx.p, V0.by.p, V0.bz.p, V0.bx32.p, V0.by32.p, V0.bz32.p);
            });
        }
        if (H.var_alpha && ir)
            timed(ctx, "setup", 0.0, [&] { k_to_f32<<<ceil_div(n0, kBlock), kBlock, 0, s>>>(P.alpha, V0.alpha32.p, n0); });
        if (!(H.var_beta || H.var_alpha || H.has_mask)) continue;
        for (int l = 1; l < H.L; l++) {
            HLevel &V = H.lv[l];
            const LevDesc &F = S.h64[(size_t)p * S.Lmax + l - 1];
            const LevDesc &C = S.h64[(size_t)p * S.Lmax + l];
            long nf = H.var_beta ? ((long)(V.nx + 1) * V.ny * V.nz + (long)V.nx * (V.ny + 1) * V.nz + (long)V.nx * V.ny * (V.nz + 1)) : 0;
            long tot = nf + (long)V.nx * V.ny * V.nz;
            timed(ctx, "setup", 0.0, [&] {
                k_coarsen<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(F, C, V.bx.p, V.by.p, V.bz.p, V.alpha.p, V.mask.p, V.bx32.p,
                                                                    V.by32.p, V.bz32.p, V.alpha32.p);
            });
        }
    }
    // assembled rows of the LDS-resident levels (constant-coefficient rows
    // depend only on the descriptors, so they are kept until those change)
    bool var_any = false;
    for (auto &H : S.probs) var_any = var_any || H.var_beta || H.var_alpha || H.has_mask;
    if (S.lds_mode && S.nfused && (var_any || !S.rows_valid)) {
        timed(ctx, "setup", 0.0, [&] {
            if (ir) k_stencils<float><<<S.nfused, 256, 0, s>>>(S.d32.p, S.d64.p, S.fused.p);
            else k_stencils<double><<<S.nfused, 256, 0, s>>>(S.d64.p, S.d64.p, S.fused.p);
        });
        S.rows_valid = true;
    }
}

// Algorithmic bytes of one launch over a plan (inputs read once, outputs
// written once).  kind 0: one colour pass of GSRB (half the cells updated:
// their b read and x written, the other colour's x read; every face
// coefficient touches one updated cell); 1: residual + restriction into the
// coarse level; 2: prolongation + correction; 3: norm of b; 4: residual
// norm; 5: residual norm + FP32 copy; 6: one fused out-of-place sweep (x
// and b read, the alternate iterate written, every coefficient read once);
// 7: copy of the alternate iterate back.
static double plan_bytes(const Solver &S, const HPlan &pl, bool fp32, int kind, const std::vector<char> *active = nullptr) {
    double total = 0.0;
    const double sT = fp32 ? 4.0 : 8.0;
    for (int id : pl.h_ids) {
        if (active && !(*active)[id / S.Lmax]) continue;
        const LevDesc &D = fp32 ? S.h32[id] : S.h64[id];
        double N = (double)D.ncell;
        double coef = (D.var_beta ? 3.0 * N * sT : 0.0) + (D.var_alpha ? N * sT : 0.0) + (D.has_mask ? N : 0.0);
        switch (kind) {
        case 0: total += 1.5 * N * sT + (D.var_beta ? 3.0 * N * sT : 0.0) + (D.var_alpha ? 0.5 * N * sT : 0.0) + (D.has_mask ? N : 0.0); break;
        case 1: { const LevDesc &F = fp32 ? S.h32[id - 1] : S.h64[id - 1];
                  double NF = (double)F.ncell;
                  total += 2.0 * NF * sT + 2.0 * N * sT + (F.var_beta ? 3.0 * NF * sT : 0.0) + (F.var_alpha ? NF * sT : 0.0) + (F.has_mask ? NF : 0.0);
                  break; }
        case 2: total += 2.0 * N * sT + N / 8.0 * sT; break;
        case 6: total += 3.0 * N * sT + coef; break;          // full out-of-place sweep: x, b read, x2 written
        case 7: total += 2.0 * N * sT; break;                 // copy
        case 3: total += N * 8.0; break;
        // FP64 residual checks (FP64 descriptors: coef counts the FP64
        // coefficient arrays once): x and b read; 10 also stores the FP32
        // residual, the default also clears the FP32 correction
        case 4: total += 2.0 * N * 8.0 + coef; break;
        case 8: total += 1.0 * N * sT + (D.var_beta ? 3.0 * N * sT : 0.0) + (D.var_alpha ? 0.5 * N * sT : 0.0) + (D.has_mask ? N : 0.0); break;
        // last pass of a refinement step: the other colour and the updated
        // colour's b read, the FP64 unknown read and written (the FP32
        // correction of the updated colour is not stored)
        case 9: total += 1.0 * N * sT + 16.0 * N + (D.var_beta ? 3.0 * N * sT : 0.0) + (D.var_alpha ? 0.5 * N * sT : 0.0) + (D.has_mask ? N : 0.0); break;
        case 10: total += 2.0 * N * 8.0 + coef + N * 4.0; break;
        default: total += 2.0 * N * 8.0 + coef + 2.0 * N * 4.0; break;
        }
    }
    return total;
}

template <typename F>
static void timed_mg(vd_ctx *ctx, Solver &S, const char *family, const HPlan &pl, bool fp32, int kind, double factor,
                     F &&launch) {
    timed(ctx, family, 0.0, launch);
    if (!ctx->timing.families.empty()) S.recs.push_back({family, &pl, fp32, kind, factor, S.cur_it, S.cur_phase});
}

// Credit the recorded launches of a finished solve: a problem contributes
// to a residual check of iteration it if it was checked then (it < outer
// checks; every problem at it = 0), to the cycle launches of iteration it
// if it was cycled then (it < cycles / inner), to set-up launches always.
static void credit_launches(vd_ctx *ctx, Solver &S, int inner) {
    if (S.recs.empty()) return;
    std::vector<char> act(S.nprob);
    for (auto &r : S.recs) {
        for (int p = 0; p < S.nprob; p++) {
            const ProbState &q = S.pin_st[p];
            if (r.phase == 2) act[p] = 1;
            else if (r.phase == 0) act[p] = r.it == 0 || q.outer > r.it;
            else act[p] = q.cycles / inner > r.it;
        }
        timing_add_units(ctx, r.family, plan_bytes(S, *r.plan, r.fp32, r.kind, &act) * r.factor);
    }
    S.recs.clear();
}

// one Gauss-Seidel colour pass over level l of every problem in the plan
template <typename T>
static void gs_pass(vd_ctx *ctx, Solver &S, int l, const LevDesc *dT, int col, int pmode = 0) {
    const HPlan &pp = S.pre[l];
    const HPlan &p25 = S.pre25[l];
    hipStream_t s = ctx->stream;
    const HPlan &pu = S.pre25u[l], &pg = S.pre25g[l];
    // pmode 4 / 5 (FP32 corrections of the refinement, level 0 only): the
    // zero-start first pass and the last pass that updates the FP64 unknown
    const LevDesc *alt = pmode == 5 ? S.d64.p : nullptr;
    const int kind = pmode == 4 ? 8 : (pmode == 5 ? 9 : 0);
    auto st25 = [&](const HPlan &q, bool uni) {
        if (pmode == 0 && S.persistent) {
            const int g = std::min(xcd_grid(q.ntiles), kMaxGrid);
            if (uni) k_st25p<T, true><<<g, kBlock, 0, s>>>(dT, q.dev(), q.kz, col, S.st.p);
            else k_st25p<T, false><<<g, kBlock, 0, s>>>(dT, q.dev(), q.kz, col, S.st.p);
            return;
        }
        if (uni) {
            if (pmode == 4)
                k_st25<T, 4, true><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
            else if (pmode == 5)
                k_st25<T, 5, true><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
            else
                k_st25<T, 0, true><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
        } else {
            if (pmode == 4)
                k_st25<T, 4><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
            else if (pmode == 5)
                k_st25<T, 5><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
            else
                k_st25<T, 0><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(dT, alt, q.dev(), q.kz, col, nullptr, S.st.p, 1, nullptr);
        }
    };
    if constexpr (sizeof(T) == 4) {
        if (l == 0 && S.rb_on) {
            // parity-split corrections of the uniform problems; the others
            // (if any) in the general kernel
            const HPlan &rb = S.rb0;
            timed_mg(ctx, S, "gsrb_fine", rb, true, kind, 1.0, [&] {
                if (pmode == 4)
                    k_rb32<4><<<xcd_grid(rb.ntiles), kBlock, 0, s>>>(dT, S.d64.p, rb.dev(), rb.kz, col, S.st.p);
                else if (pmode == 5)
                    k_rb32<5><<<xcd_grid(rb.ntiles), kBlock, 0, s>>>(dT, S.d64.p, rb.dev(), rb.kz, col, S.st.p);
                else
                    k_rb32<0><<<xcd_grid(rb.ntiles), kBlock, 0, s>>>(dT, S.d64.p, rb.dev(), rb.kz, col, S.st.p);
            });
            if (pg.nd && pu.nd) timed_mg(ctx, S, "gsrb", pg, true, kind, 1.0, [&] { st25(pg, false); });
            return;
        }
    }
    if (S.aligned && pu.nd && pg.nd) {
        // mixed level: the uniform problems in the lean kernel, the rest in
        // the general one
        timed_mg(ctx, S, l == 0 ? "gsrb_fine" : "gsrb_uniform", pu, sizeof(T) == 4, kind, 1.0, [&] { st25(pu, true); });
        timed_mg(ctx, S, "gsrb", pg, sizeof(T) == 4, kind, 1.0, [&] { st25(pg, false); });
        return;
    }
    // one timing family per kernel instantiation: the uniform-coefficient
    // colour pass and the general one
    timed_mg(ctx, S, (p25.nd && S.aligned && p25.uni) ? (l == 0 ? "gsrb_fine" : "gsrb_uniform") : "gsrb", pp, sizeof(T) == 4, kind,
             1.0, [&] {
        if (p25.nd && S.aligned) st25(p25, p25.uni);
        else k_gsrb<T><<<xcd_grid(pp.ntiles), kBlock, 0, s>>>(dT, pp.dev(), col, S.st.p);
    });
}

// one full fused sweep of level l (every problem of the plan), reading the
// iterate from x (flip 0) or x2 (flip 1) and writing the other
template <typename T>
static void sweep_pass(vd_ctx *ctx, Solver &S, int l, const LevDesc *dT, int flip) {
    const HPlan &p25 = S.pre25[l];
    timed_mg(ctx, S, "sweep", S.pre[l], sizeof(T) == 4, 6, 1.0, [&] {
        k_sweep25<T><<<xcd_grid(p25.ntiles), kBlock, 0, ctx->stream>>>(dT, p25.dev(), p25.kz, flip, S.st.p);
    });
}

// nu smoothing sweeps of level l; par tracks which buffer holds the iterate
template <typename T>
static void smooth_level(vd_ctx *ctx, Solver &S, int l, const LevDesc *dT, int nu, int &par, bool zero_first = false,
                         bool update_last = false) {
    const HPlan &p25 = S.pre25[l];
    if (p25.nd && S.use_fused[l]) {
        timing_group_begin(ctx, "sweep");
        for (int q = 0; q < nu; q++) {
            sweep_pass<T>(ctx, S, l, dT, par);
            par ^= 1;
        }
        timing_group_end(ctx);
    } else {
        // the colour passes of one level are back-to-back launches of one
        // kernel (unless the level is split): one event pair around them
        const bool split = S.aligned && S.pre25u[l].nd && S.pre25g[l].nd;
        // timing families: uniform-coefficient colour passes of the finest
        // level (bandwidth-bound) and of the coarser ones (latency-bound),
        // and the general passes
        if (!split)
            timing_group_begin(ctx, (p25.nd && S.aligned && p25.uni) ? (l == 0 ? "gsrb_fine" : "gsrb_uniform") : "gsrb");
        for (int q = 0; q < nu; q++)
            for (int col = 0; col < 2; col++) {
                const int pm = (zero_first && q == 0 && col == 0) ? 4 : ((update_last && q == nu - 1 && col == 1) ? 5 : 0);
                gs_pass<T>(ctx, S, l, dT, col, pm);
            }
        if (!split) timing_group_end(ctx);
    }
}

template <typename T>
static void vcycle(vd_ctx *ctx, Solver &S, const LevDesc *dT, const vd_mg_opts *o, bool zero_start = false,
                   bool final_update = false) {
    hipStream_t s = ctx->stream;
    const ProbState *st = S.st.p;
    std::vector<int> par(S.Lmax, 0);
    for (int l = 0; l < S.Lmax; l++) {
        if (S.pre[l].nd)
            smooth_level<T>(ctx, S, l, dT, o->nu_pre, par[l], l == 0 && zero_start,
                            l == 0 && final_update && o->nu_post == 0 && S.Lmax == 1);
        const HPlan &pr = S.restr[l];
        if (pr.nd)
            timed_mg(ctx, S, "resid_restrict", pr, sizeof(T) == 4, 1, 1.0, [&] {
                k_restrict<T><<<xcd_grid(pr.ntiles), kBlock, 0, s>>>(dT, pr.dev(), st, par[l]);
            });
    }
    if (S.nfused && S.lds_mode)
        timed(ctx, "coarse", 0.0, [&] {
            k_coarse_lds<T><<<S.nfused, kLdsThreads, S.lds_bytes, s>>>(dT, S.d64.p, S.fused.p, st, o->nu_pre, o->nu_post);
        });
    else if (S.nfused)
        timed(ctx, "coarse", 0.0, [&] {
            k_coarse<T><<<S.nfused, kFusedThreads, S.pcg_lds_bytes, s>>>(dT, S.d64.p, S.fused.p, st, o->nu_pre, o->nu_post,
                                                                          S.pcg_lds_bytes > 0);
        });
    for (int l = S.Lmax - 1; l >= 0; l--) {
        const HPlan &pp = S.prolong[l];
        if (pp.nd)
            timed_mg(ctx, S, "prolong", pp, sizeof(T) == 4, 2, 1.0, [&] {
                k_prolong<T><<<xcd_grid(pp.ntiles), kBlock, 0, s>>>(dT, pp.dev(), st, par[l]);
            });
        const HPlan &ps = S.pre[l];
        if (ps.nd) {
            smooth_level<T>(ctx, S, l, dT, o->nu_post, par[l], false, l == 0 && final_update);
            if (par[l]) {
                // an odd number of sweeps: the iterate goes back to x
                timed_mg(ctx, S, "copy", ps, sizeof(T) == 4, 7, 1.0, [&] {
                    k_copy_x2<T><<<xcd_grid(ps.ntiles), kBlock, 0, s>>>(dT, ps.dev(), st);
                });
                par[l] = 0;
            }
        }
    }
}

static const HPlan &norm_plan(const Solver &S, int mode) {
    return (mode != 0 && S.all0_25.nd && S.aligned) ? S.all0_25 : S.all0;
}

// keep_e (mode 2): leave the FP32 correction as it is, for a correction
// solve that starts from zero without reading it
static void launch_norm(vd_ctx *ctx, Solver &S, int mode, int check_active, bool with_b = false, bool keep_e = false) {
    double *pb = with_b ? S.partials_b.p : nullptr;
    const int ksel = (mode == 2 && keep_e) ? 1 : 0;
    const int kind = (mode == 2 && keep_e) ? 10 : 3 + mode;
    const HPlan &pl = S.all0;
    hipStream_t s = ctx->stream;
    // the direct (barrier-free) residual kernels for tiles of 2, 4 or 8 planes
    auto direct = [&](const HPlan &q, auto mode_tag, auto mask_tag) -> bool {
        constexpr int M = decltype(mode_tag)::value;
        constexpr bool MK = decltype(mask_tag)::value;
        const dim3 g = xcd_grid(q.ntiles);
        const Plan P = q.dev();
        if (q.kz == 8)
            k_resd<M, 8, MK><<<g, kBlock, 0, s>>>(S.d64.p, S.d32.p, P, ksel, S.partials.p, S.st.p, check_active, pb);
        else if (q.kz == 4)
            k_resd<M, 4, MK><<<g, kBlock, 0, s>>>(S.d64.p, S.d32.p, P, ksel, S.partials.p, S.st.p, check_active, pb);
        else if (q.kz == 2)
            k_resd<M, 2, MK><<<g, kBlock, 0, s>>>(S.d64.p, S.d32.p, P, ksel, S.partials.p, S.st.p, check_active, pb);
        else
            return false;
        return true;
    };
    auto launch25 = [&](const HPlan &q, bool uni) {
        // uniform levels: the LDS march; levels with coefficient arrays or a
        // mask: the direct kernel (the general march for other tile depths)
        bool masked = false;
        for (int id : q.h_ids) masked = masked || S.probs[id / S.Lmax].has_mask;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using NoMask = std::false_type;
        using Masked = std::true_type;
        if (!masked && !uni) {
            if (mode == 1 && direct(q, I1{}, NoMask{})) return;
            if (mode == 2 && direct(q, I2{}, NoMask{})) return;
        }
        // masked levels (uniform coefficients or arrays): the direct kernel
        // with the mask (covered neighbours as homogeneous Dirichlet faces)
        if (masked) {
            if (mode == 1 && direct(q, I1{}, Masked{})) return;
            if (mode == 2 && direct(q, I2{}, Masked{})) return;
        }
        if (mode == 1 && uni)
            k_res25u<1><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, q.dev(), q.kz, 0, S.partials.p, S.st.p,
                                                              check_active, pb);
        else if (mode == 1)
            k_st25<double, 1><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, q.dev(), q.kz, 0, S.partials.p, S.st.p,
                                                                    check_active, pb);
        else if (uni)
            k_res25u<2><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, q.dev(), q.kz, ksel, S.partials.p, S.st.p,
                                                              check_active, pb);
        else
            k_st25<double, 2><<<xcd_grid(q.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, q.dev(), q.kz, ksel, S.partials.p, S.st.p,
                                                                    check_active, pb);
    };
    if (mode != 0 && S.aligned && S.norm25u.nd && S.norm25g.nd) {
        // mixed batch: uniform problems in the lean kernel; partial slots
        // stay those of the full plan
        timed_mg(ctx, S, "norm", S.norm25u, false, kind, 1.0, [&] { launch25(S.norm25u, true); });
        timed_mg(ctx, S, "norm", S.norm25g, false, kind, 1.0, [&] { launch25(S.norm25g, false); });
        return;
    }
    if (mode != 0 && S.all0_25.nd && S.aligned) {
        timed_mg(ctx, S, "norm", pl, false, kind, 1.0, [&] { launch25(S.all0_25, S.all0_25.uni); });
        return;
    }
    timed_mg(ctx, S, "norm", pl, false, 3 + mode, 1.0, [&] {
        if (mode == 0)
            k_norm<0><<<xcd_grid(pl.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, pl.dev(), S.partials.p, S.st.p, check_active,
                                                             nullptr);
        else if (mode == 1)
            k_norm<1><<<xcd_grid(pl.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, pl.dev(), S.partials.p, S.st.p, check_active, pb);
        else
            k_norm<2><<<xcd_grid(pl.ntiles), kBlock, 0, s>>>(S.d64.p, S.d32.p, pl.dev(), S.partials.p, S.st.p, check_active, pb);
    });
}

static void launch_finalize(vd_ctx *ctx, Solver &S, int mode, const vd_mg_opts *o, int inner) {
    const HPlan &pl = norm_plan(S, mode);
    timed(ctx, "finalize", 0.0, [&] {
        k_finalize<<<S.nprob, kBlock, 0, ctx->stream>>>(pl.dev(), S.prob_of.p, S.partials.p, S.st.p, mode, o->rtol,
                                                        o->max_cycles, o->fixed_cycles, inner, S.partials_b.p);
    });
}

static int read_active(vd_ctx *ctx, Solver &S) {
    VD_HIP(hipMemcpyAsync(S.pin_st, S.st.p, sizeof(ProbState) * S.nprob, hipMemcpyDeviceToHost, ctx->stream));
    VD_HIP(hipStreamSynchronize(ctx->stream));
    int n = 0;
    for (int p = 0; p < S.nprob; p++) n += S.pin_st[p].active;
    return n;
}

// The FP32 corrections of a refinement step can start from zero without
// clearing them and add themselves to the FP64 unknown in their last colour
// pass when every problem's finest level is smoothed by the tiled colour
// passes before and after the coarse correction.
static bool ir_fusable(const Solver &S, const vd_mg_opts *o) {
    if (S.prec != VD_FP32_IR || !S.aligned || !S.pre25[0].nd || S.use_fused[0]) return false;
    // the correction's first pass is a pre-smoothing pass; its last pass is
    // the last post-smoothing pass, or without post-smoothing the last
    // pre-smoothing pass of a single-level solve (no coarse correction
    // follows it)
    if (o->nu_pre < 1 || (o->nu_post < 1 && S.Lmax > 1) || S.pre[0].nd != S.nprob) return false;
    for (const HProblem &H : S.probs)
        if (H.lc < 1) return false;
    return true;
}

// Hold the uniform problems' finest FP32 corrections parity-split while the
// fused refinement path is in use (and lexicographic otherwise).
static void set_rb(vd_ctx *ctx, Solver &S, const vd_mg_opts *o) {
    const bool on = S.rb0.nd > 0 && ir_fusable(S, o);
    if (on == S.rb_on) return;
    for (int id : S.rb0.h_ids) S.h32[id].rb = on ? 1 : 0;
    VD_HIP(hipStreamSynchronize(ctx->stream));
    memcpy(S.pin32, S.h32.data(), sizeof(LevDesc) * S.h32.size());
    VD_HIP(hipMemcpyAsync(S.d32.p, S.pin32, sizeof(LevDesc) * S.h32.size(), hipMemcpyHostToDevice, ctx->stream));
    S.rb_on = on;
}

// One refinement step's corrections: ir_inner FP32 cycles, then the FP64
// update (inside the last cycle's last pass when fusable).
static void ir_corrections(vd_ctx *ctx, Solver &S, const vd_mg_opts *o, bool fused) {
    for (int q = 0; q < o->ir_inner; q++) vcycle<float>(ctx, S, S.d32.p, o, fused && q == 0, fused && q == o->ir_inner - 1);
    if (!fused)
        timed_mg(ctx, S, "ir_update", S.all0, false, 3, 2.5, [&] {
            k_ir_update<<<xcd_grid(S.all0.ntiles), kBlock, 0, ctx->stream>>>(S.d64.p, S.d32.p, S.all0.dev(), S.st.p);
        });
}

// One tolerance-mode iteration: residual check (which retires converged
// problems on the device), then a V-cycle, or in IR mode ir_inner FP32
// cycles and the FP64 update.
static void one_cycle(vd_ctx *ctx, Solver &S, const vd_mg_opts *o) {
    if (S.prec != VD_FP32_IR) {
        launch_norm(ctx, S, 1, 1);
        launch_finalize(ctx, S, 1, o, 1);
        vcycle<double>(ctx, S, S.d64.p, o);
    } else {
        const bool fz = ir_fusable(S, o);
        launch_norm(ctx, S, 2, 1, false, fz);
        launch_finalize(ctx, S, 1, o, o->ir_inner);
        ir_corrections(ctx, S, o, fz);
    }
}

// The iteration above captured once into a HIP graph (on a private
// non-blocking stream, since the caller's stream may be the null stream)
// and replayed on the caller's stream.  Kernel arguments are device
// descriptor tables whose contents are refreshed outside the graph, so the
// graph stays valid until the options, the tiling or the alignment change.
static hipGraphExec_t cycle_graph(vd_ctx *ctx, Solver &S, const vd_mg_opts *o) {
    char kb[160];
    snprintf(kb, sizeof(kb), "%d,%d,%d,%d,%.17g,%d,%d,%d,%d", o->nu_pre, o->nu_post, o->ir_inner, o->max_cycles, o->rtol,
             o->fixed_cycles, (int)S.aligned, (int)S.tuned, (int)S.persistent);
    std::string gk = kb;
    for (int l = 0; l < S.Lmax; l++) gk += "," + std::to_string(S.pre25[l].kz) + (S.use_fused[l] ? "f" : "c");
    if (S.gexec && S.gkey == gk) return S.gexec;
    if (S.gexec) { (void)hipGraphExecDestroy(S.gexec); S.gexec = nullptr; }
    if (!ctx->cap_stream) VD_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // the descriptor uploads above must land before the replay, which is
    // ordered on the caller's stream; capture itself runs nothing
    hipStream_t saved = ctx->stream;
    hipGraph_t g = nullptr;
    VD_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->stream = ctx->cap_stream;
    try {
        one_cycle(ctx, S, o);
    } catch (...) {
        ctx->stream = saved;
        (void)hipStreamEndCapture(ctx->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    ctx->stream = saved;
    VD_HIP(hipStreamEndCapture(ctx->cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&S.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { S.gexec = nullptr; throw Error{VD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)}; }
    S.gkey = gk;
    return S.gexec;
}

// alternate iterates of level l (fused out-of-place sweeps), in the
// precision of the hierarchy that is smoothed; the descriptors are rebuilt
// by the next refresh
static void alloc_x2(Solver &S, int l) {
    for (int id : S.pre[l].h_ids) {
        HLevel &Vl = S.probs[id / S.Lmax].lv[id % S.Lmax];
        const size_t n = (size_t)Vl.nx * Vl.ny * Vl.nz;
        if (S.prec == VD_FP32_IR) Vl.x2_32.alloc(n);
        else Vl.x2.alloc(n);
    }
    S.key.clear();
}

// Smoother autotuning: for each level with a tiled plan, time one sweep
// as two in-place colour passes and as one fused out-of-place sweep, each
// for kz in {2, 4, 8, 16}, and keep the fastest (all variants compute the
// same values).  Every level's unknowns are saved first and restored after,
// so the solve that follows starts from the caller's iterate.
template <typename T, typename R>
static void autotune_t(vd_ctx *ctx, Solver &S, const LevDesc *dT, const std::vector<LevDesc> &hT, R &&refresh) {
    hipStream_t s = ctx->stream;
    std::vector<std::pair<void *, size_t>> xs;
    size_t total = 0;
    for (int l = 0; l < S.Lmax; l++)
        for (int id : S.pre[l].h_ids) { xs.push_back({hT[id].x, (size_t)hT[id].ncell * sizeof(T)}); total += xs.back().second; }
    DevBuf<char> save;
    save.alloc(total);
    size_t off = 0;
    for (auto &x : xs) { VD_HIP(hipMemcpyAsync(save.p + off, x.first, x.second, hipMemcpyDeviceToDevice, s)); off += x.second; }
    hipEvent_t e0, e1;
    VD_HIP(hipEventCreate(&e0));
    VD_HIP(hipEventCreate(&e1));
    for (int l = 0; l < S.Lmax; l++) {
        if (!S.pre25[l].nd) continue;
        std::vector<std::pair<int, const HLevel *>> items;
        for (int id : S.pre[l].h_ids) items.push_back({id, &S.probs[id / S.Lmax].lv[id % S.Lmax]});
        float best = 1e30f;
        int best_kz = S.pre25[l].kz, best_fused = 0;
        for (int fused = 0; fused < 2; fused++)
            for (int kz : {2, 4, 8, 16}) {
                if (fused && kz == 2) {
                    // the fused sweep writes the alternate iterate: allocate
                    // it and point this level's descriptors at it
                    alloc_x2(S, l);
                    refresh(ctx);
                }
                HPlan cand;
                build_plan25(ctx, cand, items, kz);
                auto pass = [&] {
                    if (fused)
                        k_sweep25<T><<<xcd_grid(cand.ntiles), kBlock, 0, s>>>(dT, cand.dev(), cand.kz, 0, S.st.p);
                    else
                        for (int col = 0; col < 2; col++) {
                            if (S.pre25[l].uni)
                                k_st25<T, 0, true><<<xcd_grid(cand.ntiles), kBlock, 0, s>>>(dT, nullptr, cand.dev(), cand.kz,
                                                                                         col, nullptr, S.st.p, 1, nullptr);
                            else
                                k_st25<T, 0><<<xcd_grid(cand.ntiles), kBlock, 0, s>>>(dT, nullptr, cand.dev(), cand.kz, col,
                                                                                   nullptr, S.st.p, 1, nullptr);
                        }
                };
                pass();   // warm
                VD_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 3; r++) pass();
                VD_HIP(hipEventRecord(e1, s));
                VD_HIP(hipGetLastError());
                VD_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                VD_HIP(hipEventElapsedTime(&ms, e0, e1));
                // the fused sweep is taken only when clearly faster: timed
                // alone it gains from a warm cache that it does not keep
                // inside a cycle
                if (ms < best * (fused ? 0.85f : 0.97f)) { best = ms; best_kz = kz; best_fused = fused; }
            }
        if (best_kz != S.pre25[l].kz) {
            const bool uni = S.pre25[l].uni;
            build_plan25(ctx, S.pre25[l], items, best_kz);
            S.pre25[l].uni = uni;
            split25(ctx, S, l);
        }
        S.use_fused[l] = best_fused;
        if (!best_fused) {
            VD_HIP(hipStreamSynchronize(s));
            for (int id : S.pre[l].h_ids) {
                HLevel &Vl = S.probs[id / S.Lmax].lv[id % S.Lmax];
                Vl.x2.release();
                Vl.x2_32.release();
            }
            S.key.clear();
        }
    }
    refresh(ctx);
    off = 0;
    for (auto &x : xs) { VD_HIP(hipMemcpyAsync(x.first, save.p + off, x.second, hipMemcpyDeviceToDevice, s)); off += x.second; }
    VD_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

static void autotune(vd_ctx *ctx, Solver &S, int nprob, const vd_problem *probs, const vd_mg_opts *o) {
    auto refresh = [&](vd_ctx *c) { refresh_descs(c, S, nprob, probs, o); };
    // the smoother kernels skip problems whose flag is clear; the state is
    // re-initialised by the solve that follows
    k_state_init<<<ceil_div(S.nprob, 64), 64, 0, ctx->stream>>>(S.st.p, S.nprob);
    VD_HIP(hipGetLastError());
    if (S.aligned) {
        if (S.prec == VD_FP32_IR) autotune_t<float>(ctx, S, S.d32.p, S.h32, refresh);
        else autotune_t<double>(ctx, S, S.d64.p, S.h64, refresh);
    }
    S.tuned = true;
}

// FNV-1a hash of a string, as the key of a persisted tuning result
static uint64_t fnv1a(const std::string &k) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : k) { h ^= c; h *= 1099511628211ull; }
    return h;
}

static vd_status mg_solve_impl(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                               const char *cache_tag, bool check_guess, bool noalloc);

// VD_MG_TUNE_NU: the smoothing schedule that reaches the tolerance fastest
// from the caller's starting iterates (which are restored), looked up in
// and appended to the file named by VD_TUNE_CACHE when it is set.
static void tune_nu(vd_ctx *ctx, Solver &S, int nprob, const vd_problem *probs, const vd_mg_opts *o, const char *tag) {
    char kbuf[96];
    snprintf(kbuf, sizeof kbuf, ":%s:%.6e:%d", tag ? tag : "", o->rtol, o->ir_inner);
    const std::string key = shape_key(nprob, probs, o) + kbuf;
    char hkey[24];
    snprintf(hkey, sizeof hkey, "%016llx", (unsigned long long)fnv1a(key));
    const char *path = getenv("VD_TUNE_CACHE");
    if (path && *path) {
        if (FILE *f = fopen(path, "r")) {
            char line[128], h[32];
            int a, b;
            while (fgets(line, sizeof line, f))
                if (sscanf(line, "vdnu %31s %d %d", h, &a, &b) == 3 && !strcmp(h, hkey) && a >= 0 && b >= 0 && a + b > 0) {
                    S.nu_pre = a;
                    S.nu_post = b;
                }
            fclose(f);
            if (S.nu_pre >= 0) return;
        }
    }
    hipStream_t s = ctx->stream;
    long total = 0;
    for (int p = 0; p < nprob; p++) total += (long)probs[p].grid.nx * probs[p].grid.ny * probs[p].grid.nz;
    DevBuf<double> save;
    save.alloc(total);
    auto copy_x = [&](bool to_save) {
        long off = 0;
        for (int p = 0; p < nprob; p++) {
            const long n = (long)probs[p].grid.nx * probs[p].grid.ny * probs[p].grid.nz;
            if (to_save) VD_HIP(hipMemcpyAsync(save.p + off, probs[p].x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            else VD_HIP(hipMemcpyAsync(probs[p].x, save.p + off, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            off += n;
        }
    };
    copy_x(true);
    hipEvent_t e0, e1;
    VD_HIP(hipEventCreate(&e0));
    VD_HIP(hipEventCreate(&e1));
    // the faster of two solves with schedule (a, b) from the saved start;
    // a negative time if it does not reach the tolerance within max_cycles
    auto time_schedule = [&](int a, int b) -> float {
        vd_mg_opts oc = *o;
        oc.nu_pre = a;
        oc.nu_post = b;
        oc.flags &= ~VD_MG_TUNE_NU;
        float best_ms = -1.0f;
        for (int rep = 0; rep < 2; rep++) {
            copy_x(false);
            VD_HIP(hipEventRecord(e0, s));
            try {
                mg_solve_impl(ctx, nprob, probs, &oc, nullptr, tag, false, false);
            } catch (const Error &) {
                return -1.0f;
            }
            VD_HIP(hipEventRecord(e1, s));
            VD_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            VD_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (best_ms < 0.0f || ms < best_ms) best_ms = ms;
        }
        return best_ms;
    };
    // the caller's schedule is the baseline; another replaces it only when
    // it is more than 3 % faster
    int bp = o->nu_pre, bq = o->nu_post;
    const float base = time_schedule(bp, bq);
    float best = base;
    static const int cand[][2] = {{1, 1}, {2, 1}, {1, 2}, {2, 2}, {3, 3}};
    for (const auto &c : cand) {
        if (c[0] == o->nu_pre && c[1] == o->nu_post) continue;
        const float ms = time_schedule(c[0], c[1]);
        if (ms < 0.0f) continue;
        if (best < 0.0f || (ms < best && (base < 0.0f || ms < 0.97f * base))) { best = ms; bp = c[0]; bq = c[1]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    copy_x(false);
    VD_HIP(hipStreamSynchronize(s));
    S.nu_pre = bp;
    S.nu_post = bq;
    if (path && *path)
        if (FILE *f = fopen(path, "a")) {
            fprintf(f, "vdnu %s %d %d\n", hkey, bp, bq);
            fclose(f);
        }
}

// Full solve of a batch (the engine behind vd_poisson_solve,
// vd_helmholtz_solve_batched and the implicit solves of vd_step).
static vd_status mg_solve_impl(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                               const char *cache_tag, bool check_guess, bool noalloc = false);

vd_status mg_solve_batch(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                         const char *cache_tag) {
    return mg_solve_impl(ctx, nprob, probs, o, infos, cache_tag, false);
}

// As mg_solve_batch, starting from the guess already in x (a learned
// prediction): if its relative residual is not below 1 (or not finite) the
// guess is replaced by zero and infos[p].fallback is set.
vd_status mg_solve_batch_guess(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                               const char *cache_tag) {
    vd_mg_opts og = *o;
    og.guess = VD_GUESS_GIVEN;
    return mg_solve_impl(ctx, nprob, probs, &og, infos, cache_tag, true);
}

// The same solve without allocating: the hierarchy, plans, descriptor
// tables and convergence words are carved from the arena's device region on
// every call (nothing carries over between calls, so nothing there needs to
// start at zero: each array is written by the call before it is read), the
// host staging is ordinary memory, and the options that allocate (graph
// capture, autotuning) are refused.
vd_status mg_solve_noalloc(vd_ctx *ctx, Arena *arena, int nprob, const vd_problem *probs, const vd_mg_opts *o,
                           vd_solve_info *infos) {
    VD_CHECK(o, "null options");
    VD_CHECK(!(o->flags & (VD_MG_GRAPH | VD_MG_AUTOTUNE)), "graph replay and autotuning allocate: not available without allocation");
    VD_CHECK(o->guess == VD_GUESS_GIVEN || o->guess == VD_GUESS_ZERO, "only given or zero initial guesses without allocation");
    struct Bind {
        explicit Bind(Arena *a) { a->used = 0; tl_arena = a; }
        ~Bind() { tl_arena = nullptr; }
    } bind(arena);
    return mg_solve_impl(ctx, nprob, probs, o, infos, nullptr, false, true);
}

static vd_status mg_solve_impl(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                               const char *cache_tag, bool check_guess, bool noalloc) {
    validate(nprob, probs, o);
    std::shared_ptr<Solver> S;
    if (noalloc) {
        // built afresh in the arena; kept until the next such call so that
        // its host staging outlives the copies enqueued from it (building
        // the next one synchronises the stream before this one is dropped)
        S = build_solver(ctx, nprob, probs, o);
        ctx->cache["noalloc:solver"] = S;
    } else {
        std::string key = std::string(cache_tag ? cache_tag : "") + shape_key(nprob, probs, o);
        auto it = ctx->cache.find(key);
        if (it != ctx->cache.end()) S = std::static_pointer_cast<Solver>(it->second);
        else {
            S = build_solver(ctx, nprob, probs, o);
            ctx->cache[key] = S;
        }
    }
    refresh_descs(ctx, *S, nprob, probs, o);
    setup_coefficients(ctx, *S, probs);
    // tuning runs smoother passes on the caller's iterate (restored after),
    // before the convergence state of this solve is initialised
    if ((o->flags & VD_MG_AUTOTUNE) && !S->tuned) autotune(ctx, *S, nprob, probs, o);
    // the tuned smoothing schedule replaces the caller's for this shape
    vd_mg_opts onu;
    if ((o->flags & VD_MG_TUNE_NU) && o->fixed_cycles == 0 && !noalloc) {
        if (S->nu_pre < 0) tune_nu(ctx, *S, nprob, probs, o, cache_tag);
        onu = *o;
        onu.nu_pre = S->nu_pre;
        onu.nu_post = S->nu_post;
        onu.flags &= ~VD_MG_TUNE_NU;
        o = &onu;
    }
    if ((o->flags & VD_MG_FUSED_SWEEP) && !S->tuned) {
        bool any = false;
        for (int l = 0; l < S->Lmax; l++)
            if (S->pre25[l].nd && !S->use_fused[l]) { alloc_x2(*S, l); S->use_fused[l] = 1; any = true; }
        if (any) refresh_descs(ctx, *S, nprob, probs, o);
    }
    if (S->prec == VD_FP32_IR) set_rb(ctx, *S, o);
    S->persistent = (o->flags & VD_MG_PERSISTENT) != 0;
    hipStream_t s = ctx->stream;
    S->recs.clear();
    S->cur_it = 0;
    S->cur_phase = 2;
    k_state_init<<<ceil_div(nprob, 64), 64, 0, s>>>(S->st.p, nprob);
    VD_HIP(hipGetLastError());
    // ||b|| comes from the first residual pass, except on the guess-checking
    // path, which needs it before that pass
    const bool fuse_b = !check_guess;
    if (!fuse_b) {
        launch_norm(ctx, *S, 0, 0);
        launch_finalize(ctx, *S, 0, o, 0);
    }
    // zero guess, or covered cells of a given guess set to 0 (nothing to do
    // for a given guess without masks)
    bool any_mask = false;
    for (const HProblem &H : S->probs) any_mask = any_mask || H.has_mask;
    if (o->guess == VD_GUESS_ZERO || any_mask)
        timed(ctx, "prep", 0.0, [&] {
            k_prep<<<xcd_grid(S->all0.ntiles), kBlock, 0, s>>>(S->d64.p, S->all0.dev(), S->st.p, o->guess == VD_GUESS_ZERO, 0);
        });
    if (!fuse_b)
        timed(ctx, "prep", 0.0, [&] {
            k_prep<<<xcd_grid(S->all0.ntiles), kBlock, 0, s>>>(S->d64.p, S->all0.dev(), S->st.p, 0, 1);
        });
    std::vector<int> fell_back(nprob, 0);
    if (check_guess) {
        launch_norm(ctx, *S, 1, 1);
        launch_finalize(ctx, *S, 2, o, 0);
        read_active(ctx, *S);
        bool any = false;
        for (int p = 0; p < nprob; p++)
            if (S->pin_st[p].active && !(S->pin_st[p].rel < 1.0)) { fell_back[p] = 1; any = true; }
        if (any) {
            // zero every rejected guess (one problem per call on this path)
            VD_CHECK(nprob == 1, "internal: guess fallback expects one problem");
            timed(ctx, "prep", 0.0, [&] {
                k_prep<<<xcd_grid(S->all0.ntiles), kBlock, 0, s>>>(S->d64.p, S->all0.dev(), S->st.p, 1, 0);
            });
        }
    }
    const bool ir = S->prec == VD_FP32_IR;
    const bool async_fixed = o->fixed_cycles > 0 && infos == nullptr;
    const bool use_graph = (o->flags & VD_MG_GRAPH) && !async_fixed && ctx->timing.families.empty();
    hipGraphExec_t gexec = use_graph ? cycle_graph(ctx, *S, o) : nullptr;
    int iters = 0;
    const int chunk = async_fixed ? (o->fixed_cycles + 1) : 2;
    // the first check of a fused solve also finalises ||b||, then clears x
    // of the problems whose right-hand side vanishes
    const bool ir_fz = ir && ir_fusable(*S, o);
    auto check = [&](int nmode, int inner) {
        const bool first = fuse_b && iters == 0;
        S->cur_it = iters;
        S->cur_phase = 0;
        launch_norm(ctx, *S, nmode, 1, first, nmode == 2 && ir_fz);
        launch_finalize(ctx, *S, first ? 3 : 1, o, inner);
        if (first)
            timed(ctx, "prep", 0.0, [&] {
                k_zero_b0<<<S->all0.nd, kBlock, 0, s>>>(S->d64.p, S->all0.dev(), S->st.p);
            });
    };
    if (gexec) {
        while (true) {
            for (int c = 0; c < chunk; c++) {
                if (!(fuse_b && iters == 0)) {
                    VD_HIP(hipGraphLaunch(gexec, s));
                } else if (!ir) {
                    check(1, 1);
                    S->cur_phase = 1;
                    vcycle<double>(ctx, *S, S->d64.p, o);
                } else {
                    check(2, o->ir_inner);
                    S->cur_phase = 1;
                    ir_corrections(ctx, *S, o, ir_fz);
                }
                iters++;
            }
            if (read_active(ctx, *S) == 0) break;
            if (iters > 4 * (o->max_cycles + 2) + 8) throw Error{VD_ENOCONV, "internal: convergence loop did not terminate"};
        }
    } else {
        // the cycles the previous solve of this hierarchy needed (or the
        // fixed count) are issued without a host synchronisation, ending
        // with a check; then one cycle per check until every problem has
        // retired
        const int pred = async_fixed ? o->fixed_cycles : std::max(1, S->last_iters);
        auto do_check = [&] {
            if (!ir) check(1, 1);
            else check(2, o->ir_inner);
        };
        auto do_cycle = [&] {
            S->cur_phase = 1;
            if (!ir) vcycle<double>(ctx, *S, S->d64.p, o);
            else ir_corrections(ctx, *S, o, ir_fz);
            iters++;
        };
        for (int c = 0; c <= pred; c++) {
            do_check();
            if (c == pred) break;
            do_cycle();
        }
        if (async_fixed) {
            iters++;
        } else {
            while (read_active(ctx, *S) != 0) {
                do_cycle();
                do_check();
                if (iters > 4 * (o->max_cycles + 2) + 8) throw Error{VD_ENOCONV, "internal: convergence loop did not terminate"};
            }
            int need = 0;
            for (int p = 0; p < nprob; p++) need = std::max(need, S->pin_st[p].outer - 1);
            S->last_iters = need;
        }
    }
    if (!S->recs.empty()) {
        if (async_fixed) read_active(ctx, *S);
        credit_launches(ctx, *S, ir ? o->ir_inner : 1);
    }
    vd_status worst = VD_OK;
    if (infos) {
        for (int p = 0; p < nprob; p++) {
            const ProbState &q = S->pin_st[p];
            vd_solve_info &I = infos[p];
            memset(&I, 0, sizeof(I));
            I.cycles = q.cycles;
            I.outer_iters = q.outer;
            I.levels = S->probs[p].L;
            I.status = q.status;
            I.rel_res = q.rel;
            I.rel_res0 = q.rel0;
            I.bnorm = q.bnorm;
            I.fallback = fell_back[p];
            I.nu_pre = o->nu_pre;
            I.nu_post = o->nu_post;
            if (q.status != VD_OK) worst = (vd_status)q.status;
        }
    } else if (!async_fixed) {
        for (int p = 0; p < nprob; p++)
            if (S->pin_st[p].status != VD_OK) worst = (vd_status)S->pin_st[p].status;
    }
    if (worst != VD_OK) throw Error{worst, "multigrid did not converge (non-finite residual or max_cycles reached)"};
    return VD_OK;
}

// ------------------------------------------------ inspection entry points
__global__ void __launch_bounds__(kBlock) k_flags(const LevDesc *__restrict__ descs, int id, uint8_t *out) {
    const LevDesc &L = descs[id];
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= L.ncell) return;
    int i, j, k;
    cell_ijk(L, c, i, j, k);
    uint8_t fl = (uint8_t)((i + j + k) & 1);
    if (!(L.has_mask && !L.mask[c])) {
        fl |= 2;
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        int pos[6] = {i, i, j, j, k, k};
        int lim[6] = {0, nx - 1, 0, ny - 1, 0, nz - 1};
        int step[6] = {-1, 1, -nx, nx, -L.nxy, L.nxy};
        int wrap[6] = {nx - 1, -(nx - 1), nx * (ny - 1), -nx * (ny - 1), L.nxy * (nz - 1), -L.nxy * (nz - 1)};
        for (int f = 0; f < 6; f++) {
            bool inside = pos[f] != lim[f];
            bool closed;
            if (inside || L.kind[f] == VD_BC_PERIODIC) {
                int nb = c + (inside ? step[f] : wrap[f]);
                closed = L.has_mask && !L.mask[nb];
            } else {
                closed = true;
            }
            if (closed) fl |= (uint8_t)(1 << (2 + f));
        }
    }
    out[c] = fl;
}

__global__ void __launch_bounds__(kBlock) k_smooth_colour(const LevDesc *__restrict__ descs, int id, int colour) {
    const LevDesc &L = descs[id];
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= L.ncell) return;
    int i, j, k;
    cell_ijk(L, c, i, j, k);
    if (((i + j + k) & 1) != colour) return;
    gs_update<double>(L, c, i, j, k);
}

vd_status mg_cell_flags(vd_ctx *ctx, const vd_problem *prob, int n_levels, int level, uint8_t *out) {
    VD_CHECK(prob && out, "null argument");
    vd_mg_opts o{};
    o.rtol = 1e-10; o.max_cycles = 1; o.nu_pre = 1; o.n_levels = n_levels; o.precision = VD_FP64;
    vd_problem P = *prob;
    double dummy_ptr = 0;  // rhs/x are not touched by the flag kernel
    if (!P.rhs) P.rhs = &dummy_ptr;
    if (!P.x) P.x = &dummy_ptr;
    validate(1, &P, &o);
    int L = count_levels(P.grid, n_levels);
    VD_CHECK(level >= 0 && level < L, "level out of range");
    std::string key = "flags" + shape_key(1, &P, &o);
    auto S = build_solver(ctx, 1, &P, &o);
    refresh_descs(ctx, *S, 1, &P, &o);
    setup_coefficients(ctx, *S, &P);
    const LevDesc &D = S->h64[level];
    k_flags<<<ceil_div(D.ncell, kBlock), kBlock, 0, ctx->stream>>>(S->d64.p, level, out);
    VD_HIP(hipGetLastError());
    VD_HIP(hipStreamSynchronize(ctx->stream));
    return VD_OK;
}

vd_status mg_smooth(vd_ctx *ctx, const vd_problem *prob, int ncolour) {
    VD_CHECK(prob && ncolour >= 0, "bad argument");
    vd_mg_opts o{};
    o.rtol = 1e-10; o.max_cycles = 1; o.nu_pre = 1; o.n_levels = 1; o.precision = VD_FP64;
    validate(1, prob, &o);
    auto S = build_solver(ctx, 1, prob, &o);
    refresh_descs(ctx, *S, 1, prob, &o);
    setup_coefficients(ctx, *S, prob);
    const LevDesc &D = S->h64[0];
    for (int q = 0; q < ncolour; q++) {
        k_smooth_colour<<<ceil_div(D.ncell, kBlock), kBlock, 0, ctx->stream>>>(S->d64.p, 0, q & 1);
        VD_HIP(hipGetLastError());
    }
    VD_HIP(hipStreamSynchronize(ctx->stream));
    return VD_OK;
}

}  // namespace vd
