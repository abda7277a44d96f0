// Internal declarations of libvd (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/vd.h"

namespace vd {

// ---------------------------------------------------------------- errors
struct Error {
    vd_status code;
    std::string msg;
};

#define VD_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::vd::Error{VD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define VD_CHECK(cond, msg)                                           \
    do {                                                              \
        if (!(cond)) throw ::vd::Error{VD_EINVAL, std::string(msg)}; \
    } while (0)

// ------------------------------------------------------- device buffers
// A fixed device region handed out front to back (256-byte aligned) while
// an allocation-free call runs on this host thread: buffers created then
// take their memory from it instead of hipMalloc and never free it.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void *carve(size_t bytes) {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > cap || bytes > cap - off)
            throw Error{VD_EINVAL, "the problem needs more than the " + std::to_string(cap >> 20) +
                                       " MiB of device scratch memory of the allocation-free entry point"};
        used = off + bytes;
        return base + off;
    }
};
inline thread_local Arena *tl_arena = nullptr;

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    bool owned = false;     // hipMalloc'd (freed on release) rather than carved from an arena
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), owned(o.owned) { o.p = nullptr; o.n = 0; o.owned = false; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; owned = o.owned;
            o.p = nullptr; o.n = 0; o.owned = false;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        n = 0;
        owned = false;
    }
    void alloc(size_t count) {
        if (count <= n && p) return;
        release();
        if (count == 0) return;
        if (tl_arena) {
            p = (T *)tl_arena->carve(count * sizeof(T));
            n = count;
            return;
        }
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{VD_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
        }
        n = count;
        owned = true;
    }
};

// Host staging buffers of the solvers: pinned, or ordinary host memory
// while an allocation-free call runs (no hipHostMalloc then).
inline void *stage_alloc(size_t bytes, bool *pinned) {
    void *p = nullptr;
    *pinned = tl_arena == nullptr;
    if (*pinned) {
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess)
            throw Error{VD_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed"};
    } else {
        p = ::operator new(bytes);
    }
    return p;
}
inline void stage_free(void *p, bool pinned) {
    if (!p) return;
    if (pinned) (void)hipHostFree(p);
    else ::operator delete(p);
}

// ---------------------------------------------------- level descriptor
// One multigrid level of one problem, as the kernels see it.  Coefficient
// pointers are null for uniform coefficients (beta_c / alpha_c used).
struct LevDesc {
    int nx, ny, nz, ncell;
    int kind[6];
    int var_beta, var_alpha, has_mask, lift;
    int prob, nxy;
    double idx2, idy2, idz2;     // 1/h^2 per direction
    double beta_c, alpha_c;
    double gval[6];              // Dirichlet face values (used when lift)
    const double *bx, *by, *bz, *alpha;
    const float *bx32, *by32, *bz32, *alpha32;
    const uint8_t *mask;
    void *x;                     // unknown (double or float by hierarchy)
    const void *b;               // right-hand side
    void *sten;                  // assembled rows of an LDS-resident level (diagonal + 6 weight planes), else null
    void *x2;                    // alternate iterate of the out-of-place fused sweeps, else null
    int rb;                      // x and b held parity-split by row (FP32 refinement corrections, finest level)
    int pad_;
};

// Position of cell (i, j, k) in a level's x / b: lexicographic, or, when the
// level is held parity-split by row, the row's red cells ((i+j+k) even, in
// order of i) followed by its black cells.
__host__ __device__ __forceinline__ long cell_pos(const LevDesc &L, int i, int j, int k) {
    const long row = (long)L.nx * j + (long)L.nxy * k;
    return L.rb ? row + (((i + j + k) & 1) ? (L.nx >> 1) : 0) + (i >> 1) : row + i;
}

// Per-problem convergence state, device resident.
struct ProbState {
    int active;      // 1 while more cycles are needed
    int cycles;      // V-cycles run (inner cycles in IR mode)
    int outer;       // FP64 residual checks
    int status;
    double bnorm, rel0, rel;
};

// A launch plan: a list of level descriptors and the prefix sum of their
// tile counts; block -> (descriptor, tile) by search.
struct Plan {
    const int *ids;
    const int *prefix;
    int nd;
    int ntiles;
    const int *gbase;   // nullable: per descriptor, the first partial slot in the full plan (split norm launches)
};

constexpr int kBlock = 256;

// Address-space qualified access.  Pointers that reach a kernel through a
// descriptor struct are generic to the compiler, which then emits FLAT
// instructions; FLAT loads also count against the LDS counter, so every LDS
// wait would wait for them as well.  Casting to the global (1) or LDS (3)
// address space gives global_load / ds_read instead.
#define VD_GAS __attribute__((address_space(1)))
#define VD_LAS __attribute__((address_space(3)))

template <typename T>
__device__ __forceinline__ T gld(const T *p, long i) { return ((const VD_GAS T *)p)[i]; }
template <typename T>
__device__ __forceinline__ void gst(T *p, long i, T v) { ((VD_GAS T *)p)[i] = v; }
template <typename T>
__device__ __forceinline__ T lld(const T *p, long i) { return ((const VD_LAS T *)p)[i]; }
template <typename T>
__device__ __forceinline__ void lst(T *p, long i, T v) { ((VD_LAS T *)p)[i] = v; }

// memory-space tagged access: AS 1 = global, 3 = LDS
template <int AS, typename T>
__device__ __forceinline__ T mld(const T *p, long i) {
    if constexpr (AS == 3) return lld(p, i);
    else return gld(p, i);
}
template <int AS, typename T>
__device__ __forceinline__ void mst(T *p, long i, T v) {
    if constexpr (AS == 3) lst(p, i, v);
    else gst(p, i, v);
}

// ------------------------------------------------------- kernel timing
struct TimingAcc {
    int64_t launches = 0;
    double total_ms = 0.0;
    double units = 0.0;      // algorithmic bytes (or cells) summed over launches
};
struct TimingPending {
    std::string family;
    hipEvent_t a, b;
};
struct Timing {
    std::vector<std::string> families;          // selected kernel families
    std::map<std::string, TimingAcc> acc;
    std::vector<TimingPending> pending;
    std::vector<hipEvent_t> pool;
    // an open group: consecutive launches of one family bracketed by a
    // single event pair (fewer events between back-to-back kernels)
    std::string group;
    int group_n = 0;
    hipEvent_t ga = nullptr, gb = nullptr;
};

}  // namespace vd

struct vd_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;    // private stream for HIP graph capture
    std::string last_error;
    vd::Timing timing;
    std::map<std::string, std::shared_ptr<void>> cache;   // solver hierarchies by key
    vd::DevBuf<double> scratch64;
    vd::DevBuf<char> scratch_bytes;
};

namespace vd {

// Small host blobs (kernel descriptor tables) mirrored in device memory.
// The device copy is refreshed only when the bytes change, so repeated calls
// with the same arguments enqueue no host-to-device copy.
struct DevBlob {
    DevBuf<char> d;
    std::vector<char> last;
    char *pinned = nullptr;
    size_t cap = 0;
    ~DevBlob() { if (pinned) (void)hipHostFree(pinned); }
};

inline const void *upload_blob(vd_ctx *ctx, const std::string &key, const void *data, size_t bytes) {
    std::shared_ptr<DevBlob> B;
    auto it = ctx->cache.find("blob:" + key);
    if (it != ctx->cache.end()) B = std::static_pointer_cast<DevBlob>(it->second);
    else { B = std::make_shared<DevBlob>(); ctx->cache["blob:" + key] = B; }
    if (B->last.size() == bytes && memcmp(B->last.data(), data, bytes) == 0) return B->d.p;
    VD_HIP(hipStreamSynchronize(ctx->stream));   // the previous staging may still be in flight
    if (B->cap < bytes) {
        if (B->pinned) (void)hipHostFree(B->pinned);
        B->pinned = nullptr;
        VD_HIP(hipHostMalloc((void **)&B->pinned, bytes, hipHostMallocDefault));
        B->cap = bytes;
    }
    B->d.alloc(bytes);
    memcpy(B->pinned, data, bytes);
    VD_HIP(hipMemcpyAsync(B->d.p, B->pinned, bytes, hipMemcpyHostToDevice, ctx->stream));
    B->last.assign((const char *)data, (const char *)data + bytes);
    return B->d.p;
}

// Kernel timing hooks (host).  begin() returns true when the family matches.
bool timing_begin(vd_ctx *ctx, const char *family, hipEvent_t *ev0, hipEvent_t *ev1);
void timing_flush(vd_ctx *ctx);

void timing_end(vd_ctx *ctx, const char *family, hipEvent_t ev0, hipEvent_t ev1, double units, int nlaunch = 1);
// algorithmic bytes credited to a family after the launches (work that is
// known only once the device-side convergence state has been read)
void timing_add_units(vd_ctx *ctx, const char *family, double units);

template <typename F>
inline void timed(vd_ctx *ctx, const char *family, double units, F &&launch) {
    Timing &T = ctx->timing;
    if (!T.group.empty() && T.group == family) {     // inside an open group of this family
        launch();
        VD_HIP(hipGetLastError());
        T.group_n += 1;
        return;
    }
    hipEvent_t a = nullptr, b = nullptr;
    bool on = !ctx->timing.families.empty() && timing_begin(ctx, family, &a, &b);
    if (on) VD_HIP(hipEventRecord(a, ctx->stream));
    launch();
    VD_HIP(hipGetLastError());
    if (on) {
        VD_HIP(hipEventRecord(b, ctx->stream));
        timing_end(ctx, family, a, b, units);
    }
}

// open / close a group of consecutive launches of one selected family
inline void timing_group_begin(vd_ctx *ctx, const char *family) {
    Timing &T = ctx->timing;
    if (T.families.empty() || !T.group.empty()) return;
    hipEvent_t a, b;
    if (!timing_begin(ctx, family, &a, &b)) return;
    VD_HIP(hipEventRecord(a, ctx->stream));
    T.group = family;
    T.group_n = 0;
    T.ga = a;
    T.gb = b;
}

inline void timing_group_end(vd_ctx *ctx) {
    Timing &T = ctx->timing;
    if (T.group.empty()) return;
    VD_HIP(hipEventRecord(T.gb, ctx->stream));
    const std::string f = T.group;
    T.group.clear();
    timing_end(ctx, f.c_str(), T.ga, T.gb, 0.0, T.group_n);
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Grid of 8*ceil(n/8) blocks; the kernel maps block -> tile so that each
// of the 8 XCDs (blocks are dealt round-robin) gets a contiguous range of
// tiles, keeping stencil neighbours in the same L2.
inline int xcd_grid(int ntiles) { return 8 * ceil_div(ntiles, 8); }

__device__ __forceinline__ int xcd_tile(int ntiles) {
    int chunk = (ntiles + 7) >> 3;
    int b = blockIdx.x;
    return (b & 7) * chunk + (b >> 3);
}

__device__ __forceinline__ int plan_find(const Plan &pl, int tile) {
    int lo = 0, hi = pl.nd - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pl.prefix[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Upper bound of resident workgroups for the persistent grid kernels
// (256 CUs x 8 workgroups of 256 threads).
constexpr int kMaxGrid = 2048;

inline int persistent_grid(int ntiles) {
    int g = 8 * ceil_div(ntiles, 8);
    return g < kMaxGrid ? g : kMaxGrid;
}

// Persistent, XCD-aware tile loop: workgroups are dealt round-robin to the 8
// XCDs, so XCD x (= blockIdx.x mod 8) takes the contiguous tile range
// [x*chunk, (x+1)*chunk) and its workgroups stride through it.  Neighbouring
// tiles of a stencil therefore share that XCD's L2.  fn(d, local_tile) is
// called with the plan entry d and the tile index within that entry.
template <typename F>
__device__ __forceinline__ void for_tiles(const Plan &pl, F &&fn) {
    const int chunk = (pl.ntiles + 7) >> 3;
    const int xcd = blockIdx.x & 7;
    const int per_xcd = gridDim.x >> 3;
    const int t0 = xcd * chunk;
    const int t1 = min(t0 + chunk, pl.ntiles);
    int d = -1, lo = 0, hi = 0;
    for (int t = t0 + (int)(blockIdx.x >> 3); t < t1; t += per_xcd) {
        if (t < lo || t >= hi) { d = plan_find(pl, t); lo = pl.prefix[d]; hi = pl.prefix[d + 1]; }
        fn(d, t - lo, t);
    }
}

// ------------------------------------------------ the 7-point operator
template <typename T> struct Coef;
template <> struct Coef<double> {
    static __device__ __forceinline__ const double *bx(const LevDesc &L) { return L.bx; }
    static __device__ __forceinline__ const double *by(const LevDesc &L) { return L.by; }
    static __device__ __forceinline__ const double *bz(const LevDesc &L) { return L.bz; }
    static __device__ __forceinline__ const double *al(const LevDesc &L) { return L.alpha; }
};
template <> struct Coef<float> {
    static __device__ __forceinline__ const float *bx(const LevDesc &L) { return L.bx32; }
    static __device__ __forceinline__ const float *by(const LevDesc &L) { return L.by32; }
    static __device__ __forceinline__ const float *bz(const LevDesc &L) { return L.bz32; }
    static __device__ __forceinline__ const float *al(const LevDesc &L) { return L.alpha32; }
};

// diag and off-diagonal sum of row c = (i,j,k): (A x)_c = diag x_c - off.
// Faces in the order x-, x+, y-, y+, z-, z+.  A Dirichlet domain face or a
// covered neighbour adds twice the face coefficient to the diagonal;
// Neumann and wall faces add nothing; periodic faces wrap.
template <typename T, typename XT, int AS = 1>
__device__ __forceinline__ void row_terms(const LevDesc &L, const XT *__restrict__ x, int i, int j, int k, int c,
                                          T &diag, T &off) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    T dg = L.var_alpha ? gld(Coef<T>::al(L), c) : (T)L.alpha_c;
    T of = 0;
    const T bc = (T)L.beta_c;
#define VD_FACE(NBCOND, NBIDX, BETA_ARR, BETA_IDX, IH2, FACE)            \
    {                                                                    \
        T cf = (L.var_beta ? gld(BETA_ARR, BETA_IDX) : bc) * (T)(IH2);   \
        int nb;                                                          \
        bool inside = (NBCOND);                                          \
        int kd = L.kind[FACE];                                           \
        if (inside || kd == VD_BC_PERIODIC) {                            \
            nb = (NBIDX);                                                \
            if (L.has_mask && !gld(L.mask, nb)) dg += (T)2 * cf;         \
            else { dg += cf; of += cf * (T)mld<AS>(x, nb); }             \
        } else if (kd == VD_BC_DIRICHLET) {                              \
            dg += (T)2 * cf;                                             \
        }                                                                \
    }
    const long fxrow = (long)(nx + 1) * (j + (long)ny * k);
    const long fyrow = (long)nx * (j + (long)(ny + 1) * k);
    const long fzpl = (long)nx * j;
    VD_FACE(i > 0, (i > 0 ? c - 1 : c + nx - 1), Coef<T>::bx(L), fxrow + i, L.idx2, 0)
    VD_FACE(i < nx - 1, (i < nx - 1 ? c + 1 : c - (nx - 1)), Coef<T>::bx(L), fxrow + i + 1, L.idx2, 1)
    VD_FACE(j > 0, (j > 0 ? c - nx : c + nx * (ny - 1)), Coef<T>::by(L), fyrow + i, L.idy2, 2)
    VD_FACE(j < ny - 1, (j < ny - 1 ? c + nx : c - nx * (ny - 1)), Coef<T>::by(L), fyrow + i + nx, L.idy2, 3)
    VD_FACE(k > 0, (k > 0 ? c - L.nxy : c + L.nxy * (nz - 1)), Coef<T>::bz(L), fzpl + i + (long)L.nxy * k, L.idz2, 4)
    VD_FACE(k < nz - 1, (k < nz - 1 ? c + L.nxy : c - L.nxy * (nz - 1)), Coef<T>::bz(L), fzpl + i + (long)L.nxy * (k + 1), L.idz2, 5)
#undef VD_FACE
    diag = dg;
    off = of;
}

// Same row as row_terms, with the six neighbour values already gathered
// (order x-, x+, y-, y+, z-, z+; a value across a non-periodic domain face
// is ignored).  Covered neighbours are still read from the mask.
template <typename T>
__device__ __forceinline__ void row_terms_nb(const LevDesc &L, int i, int j, int k, int c, const T nbv[6], T &diag,
                                             T &off) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    T dg = L.var_alpha ? gld(Coef<T>::al(L), c) : (T)L.alpha_c;
    T of = 0;
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
        const T ih2 = (T)(f < 2 ? L.idx2 : (f < 4 ? L.idy2 : L.idz2));
        const T cf = beta * ih2;
        const int kd = L.kind[f];
        if (inside[f] || kd == VD_BC_PERIODIC) {
            if (L.has_mask && !gld(L.mask, nbi[f])) dg += (T)2 * cf;
            else { dg += cf; of += cf * nbv[f]; }
        } else if (kd == VD_BC_DIRICHLET) {
            dg += (T)2 * cf;
        }
    }
    diag = dg;
    off = of;
}

// Same row for a uniform-coefficient level (no coefficient arrays, no
// mask): nothing is loaded, so it can sit inside a software pipeline.
template <typename T>
__device__ __forceinline__ void row_terms_uni(const LevDesc &L, int i, int j, int k, const T nbv[6], T &diag, T &off) {
    T dg = (T)L.alpha_c;
    T of = 0;
    const T bc = (T)L.beta_c;
    const bool inside[6] = {i > 0, i < L.nx - 1, j > 0, j < L.ny - 1, k > 0, k < L.nz - 1};
#pragma unroll
    for (int f = 0; f < 6; f++) {
        const T cf = bc * (T)(f < 2 ? L.idx2 : (f < 4 ? L.idy2 : L.idz2));
        const int kd = f == 0 ? L.kind[0] : f == 1 ? L.kind[1] : f == 2 ? L.kind[2] : f == 3 ? L.kind[3] : f == 4 ? L.kind[4] : L.kind[5];
        if (inside[f] || kd == VD_BC_PERIODIC) { dg += cf; of += cf * nbv[f]; }
        else if (kd == VD_BC_DIRICHLET) dg += (T)2 * cf;
    }
    diag = dg;
    off = of;
}

// Same row with the six face coefficients and the diagonal coefficient
// already loaded (no mask): cf_f = fc[f] / h^2; lift (finest level) from the
// same faces.
template <typename T>
__device__ __forceinline__ void row_terms_fc(const LevDesc &L, int i, int j, int k, const T nbv[6], const T fc[6], T alpha,
                                             T &diag, T &off, double &lift) {
    T dg = alpha;
    T of = 0;
    double lf = 0.0;
    const bool inside[6] = {i > 0, i < L.nx - 1, j > 0, j < L.ny - 1, k > 0, k < L.nz - 1};
#pragma unroll
    for (int f = 0; f < 6; f++) {
        const double ih2 = f < 2 ? L.idx2 : (f < 4 ? L.idy2 : L.idz2);
        const T cf = fc[f] * (T)ih2;
        const int kd = f == 0 ? L.kind[0] : f == 1 ? L.kind[1] : f == 2 ? L.kind[2] : f == 3 ? L.kind[3] : f == 4 ? L.kind[4] : L.kind[5];
        const double g = f == 0 ? L.gval[0] : f == 1 ? L.gval[1] : f == 2 ? L.gval[2] : f == 3 ? L.gval[3] : f == 4 ? L.gval[4] : L.gval[5];
        if (inside[f] || kd == VD_BC_PERIODIC) { dg += cf; of += cf * nbv[f]; }
        else if (kd == VD_BC_DIRICHLET) { dg += (T)2 * cf; lf += 2.0 * (double)fc[f] * g * ih2; }
    }
    diag = dg;
    off = of;
    lift = lf;
}

// Dirichlet lifting of a uniform-coefficient finest level (no loads)
__device__ __forceinline__ double lift_term_uni(const LevDesc &L, int i, int j, int k) {
    double v = 0.0;
    const double bc = L.beta_c;
    if (i == 0 && L.kind[0] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[0] * L.idx2;
    if (i == L.nx - 1 && L.kind[1] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[1] * L.idx2;
    if (j == 0 && L.kind[2] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[2] * L.idy2;
    if (j == L.ny - 1 && L.kind[3] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[3] * L.idy2;
    if (k == 0 && L.kind[4] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[4] * L.idz2;
    if (k == L.nz - 1 && L.kind[5] == VD_BC_DIRICHLET) v += 2.0 * bc * L.gval[5] * L.idz2;
    return v;
}

// Dirichlet lifting of the finest level: 2 beta_f g / h^2 per Dirichlet
// face of a boundary cell, added to the right-hand side.
__device__ __forceinline__ double lift_term(const LevDesc &L, int i, int j, int k) {
    double v = 0.0;
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    if (i == 0 && L.kind[0] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.bx, (long)(nx + 1) * (j + (long)ny * k)) : L.beta_c) * L.gval[0] * L.idx2;
    if (i == nx - 1 && L.kind[1] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.bx, (long)(nx + 1) * (j + (long)ny * k) + nx) : L.beta_c) * L.gval[1] * L.idx2;
    if (j == 0 && L.kind[2] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.by, i + (long)nx * ((long)(ny + 1) * k)) : L.beta_c) * L.gval[2] * L.idy2;
    if (j == ny - 1 && L.kind[3] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.by, i + (long)nx * (ny + (long)(ny + 1) * k)) : L.beta_c) * L.gval[3] * L.idy2;
    if (k == 0 && L.kind[4] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.bz, i + (long)nx * j) : L.beta_c) * L.gval[4] * L.idz2;
    if (k == nz - 1 && L.kind[5] == VD_BC_DIRICHLET)
        v += 2.0 * (L.var_beta ? gld(L.bz, i + (long)nx * (j + (long)ny * nz)) : L.beta_c) * L.gval[5] * L.idz2;
    return v;
}

__device__ __forceinline__ void cell_ijk(const LevDesc &L, int c, int &i, int &j, int &k) {
    k = c / L.nxy;
    int r = c - k * L.nxy;
    j = r / L.nx;
    i = r - j * L.nx;
}

// Deterministic block sum (fixed shuffle tree, then fixed LDS order).
__device__ __forceinline__ double block_sum(double v, double *lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; q++) s += lds[q];
    __syncthreads();
    return s;
}

}  // namespace vd
