// extern "C" entry points of libvd: argument checks, error capture and
// dispatch to the internal engines.  No exception crosses this boundary.
#include <mutex>

#include "physics.hpp"

namespace vd {
vd_status step(vd_ctx *ctx, const vd_step_params *P, const vd_state *st, vd_step_info *info);
vd_status step_reset(vd_ctx *ctx);
vd_status species_flux(vd_ctx *ctx, const vd_grid *g, const vd_bc *phi_bc, const vd_bc *sp_bc, int S, const vd_species *sp,
                       const double *n, const double *phi, const double *mu, const double *D, const double *Te, double Tg,
                       const vd_consts *c, double *div, int flux_species, double *face_flux);
vd_status reaction_source(vd_ctx *ctx, int mech, long ncell, int S, const double *n, const double *Te, const double *bg,
                          double qe, double *G, double *S_inel);

bool timing_begin(vd_ctx *ctx, const char *family, hipEvent_t *ev0, hipEvent_t *ev1) {
    Timing &T = ctx->timing;
    bool sel = false;
    for (auto &f : T.families) sel = sel || f == family;
    if (!sel) return false;
    if (T.pool.size() < 2) {
        // timing-only events: no system-scope fence (no cache writeback and
        // invalidation around the timed kernels); read after a stream sync
        for (int q = 0; q < 1024; q++) {
            hipEvent_t e;
            VD_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            T.pool.push_back(e);
        }
    }
    *ev0 = T.pool.back(); T.pool.pop_back();
    *ev1 = T.pool.back(); T.pool.pop_back();
    return true;
}

void timing_end(vd_ctx *ctx, const char *family, hipEvent_t ev0, hipEvent_t ev1, double units, int nlaunch) {
    Timing &T = ctx->timing;
    T.pending.push_back(TimingPending{family, ev0, ev1});
    TimingAcc &A = T.acc[family];
    A.units += units;
    A.launches += nlaunch;
    if (T.pending.size() >= 8192) timing_flush(ctx);
}

void timing_add_units(vd_ctx *ctx, const char *family, double units) {
    Timing &T = ctx->timing;
    for (auto &f : T.families)
        if (f == family) { T.acc[family].units += units; return; }
}

void timing_flush(vd_ctx *ctx) {
    Timing &T = ctx->timing;
    for (auto &pr : T.pending) {
        VD_HIP(hipEventSynchronize(pr.b));
        float ms = 0.0f;
        VD_HIP(hipEventElapsedTime(&ms, pr.a, pr.b));
        T.acc[pr.family].total_ms += ms;
        T.pool.push_back(pr.a);
        T.pool.push_back(pr.b);
    }
    T.pending.clear();
}

vd_status nn_create(vd_ctx *ctx, const vd_nn_config *cfg, const float *params);
int64_t nn_param_count(const vd_nn_config *cfg);
vd_status nn_params(vd_ctx *ctx, int which, float *host, int set);
vd_status nn_forward(vd_ctx *ctx, const vd_grid *g, const uint16_t *in, float *out);
vd_status nn_train_step(vd_ctx *ctx, const vd_grid *g, const uint16_t *in, const float *target, float lr, int update,
                        double *loss);
vd_status nn_features(vd_ctx *ctx, const vd_grid *g, const vd_bc *bc, const double *rho, double eps, uint16_t *out,
                      double *vref);
vd_status nn_guess(vd_ctx *ctx, const vd_grid *g, const vd_bc *bc, const double *rho, double eps, double *x);
vd_status nn_save(vd_ctx *ctx, const char *path);
vd_status nn_load(vd_ctx *ctx, const char *path);
vd_status nn_conv3d(vd_ctx *ctx, const vd_grid *g, const uint16_t *x, int ci, const float *w, const float *b, int co, int relu,
                    float *y, const float *dy, float *dx, float *dw, float *db);
vd_status mg_solve_batch_guess(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                               const char *cache_tag);
}  // namespace vd

// ---------------------------------------------- allocation-free solves
// Device scratch of vd_poisson_solve_noalloc: a static array that every GPU
// the library runs on holds until the process ends.  In host code the
// array's name only identifies the symbol; kernels get the device address
// that hipGetSymbolAddress returns for the current device, resolved once
// per device (at context creation, or on the first such call on a device).
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

vd_status resolve_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VD_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return VD_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return VD_OK;
}
}  // namespace

namespace vd {
template <typename F>
static vd_status guarded(vd_ctx *ctx, F &&fn) {
    if (!ctx) return VD_EINVAL;
    try {
        vd_status s = fn();
        if (s == VD_OK) ctx->last_error.clear();
        return s;
    } catch (const vd::Error &e) {
        ctx->last_error = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return VD_EHIP;
    }
}
}  // namespace vd
using vd::guarded;

extern "C" {

const char *vd_version(void) { return "libvd 0.1 gfx950"; }

vd_status vd_ctx_create(vd_ctx **out, void *stream) {
    if (!out) return VD_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return VD_EHIP;
    void *scratch_ptr = nullptr;
    if (resolve_scratch(&scratch_ptr) != VD_OK) return VD_EHIP;
    vd_ctx *c = new (std::nothrow) vd_ctx();
    if (!c) return VD_ENOMEM;
    c->stream = (hipStream_t)stream;
    *out = c;
    return VD_OK;
}

void vd_ctx_destroy(vd_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    try { vd::timing_flush(ctx); } catch (...) {}
    for (auto &e : ctx->timing.pool) (void)hipEventDestroy(e);
    ctx->cache.clear();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

vd_status vd_ctx_set_stream(vd_ctx *ctx, void *stream) {
    return guarded(ctx, [&] {
        VD_HIP(hipStreamSynchronize(ctx->stream));
        ctx->stream = (hipStream_t)stream;
        return VD_OK;
    });
}

const char *vd_last_error(const vd_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

vd_status vd_poisson_solve(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const uint8_t *mask, const double *beta_cell,
                           double beta_c, const double *rho, double *phi, const vd_mg_opts *opts, vd_solve_info *info) {
    return guarded(ctx, [&] {
        VD_CHECK(grid && phi_bc && rho && phi && opts, "null argument");
        VD_CHECK(beta_cell || beta_c > 0.0, "permittivity must be positive");
        vd_problem p;
        memset(&p, 0, sizeof(p));
        p.grid = *grid; p.bc = *phi_bc; p.mask = mask; p.beta = beta_cell; p.beta_c = beta_c;
        p.rhs = rho; p.x = phi;
        if (opts->guess == VD_GUESS_LEARNED) {
            vd::nn_guess(ctx, grid, phi_bc, rho, beta_c > 0.0 ? beta_c : 8.8541878128e-12, phi);
            return vd::mg_solve_batch_guess(ctx, 1, &p, opts, info, "poisson:");
        }
        return vd::mg_solve_batch(ctx, 1, &p, opts, info, "poisson:");
    });
}

vd_status vd_poisson_solve_noalloc(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const uint8_t *mask,
                                   const double *beta_cell, double beta_c, const double *rho, double *phi,
                                   const vd_mg_opts *opts, vd_solve_info *info) {
    return guarded(ctx, [&] {
        VD_CHECK(grid && phi_bc && rho && phi && opts, "null argument");
        VD_CHECK(beta_cell || beta_c > 0.0, "permittivity must be positive");
        void *ptr = nullptr;
        if (resolve_scratch(&ptr) != VD_OK) throw vd::Error{VD_EHIP, "no device address for the scratch array"};
        vd_problem p;
        memset(&p, 0, sizeof(p));
        p.grid = *grid; p.bc = *phi_bc; p.mask = mask; p.beta = beta_cell; p.beta_c = beta_c;
        p.rhs = rho; p.x = phi;
        vd::Arena arena;
        arena.base = (char *)ptr;
        arena.cap = kScratchBytes;
        return vd::mg_solve_noalloc(ctx, &arena, 1, &p, opts, info);
    });
}

vd_status vd_helmholtz_solve_batched(vd_ctx *ctx, int32_t nprob, const vd_problem *probs, const vd_mg_opts *opts,
                                     vd_solve_info *infos) {
    return guarded(ctx, [&] { return vd::mg_solve_batch(ctx, nprob, probs, opts, infos, "batch:"); });
}

vd_status vd_species_flux(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const vd_bc *species_bc, int32_t S,
                          const vd_species *species, const double *n, const double *phi, const double *mu, const double *D,
                          const double *Te_K, double Tg, const vd_consts *consts, double *div_drift, int32_t flux_species,
                          double *face_flux) {
    return guarded(ctx, [&] {
        return vd::species_flux(ctx, grid, phi_bc, species_bc, S, species, n, phi, mu, D, Te_K, Tg, consts, div_drift,
                                flux_species, face_flux);
    });
}

vd_status vd_reaction_source(vd_ctx *ctx, int32_t mech, int64_t ncells, int32_t S, const double *n, const double *Te_K,
                             const double *bg, double qe, double *G, double *S_inel) {
    return guarded(ctx, [&] { return vd::reaction_source(ctx, mech, (long)ncells, S, n, Te_K, bg, qe, G, S_inel); });
}

vd_status vd_step(vd_ctx *ctx, const vd_step_params *params, const vd_state *state, vd_step_info *info) {
    return guarded(ctx, [&] { return vd::step(ctx, params, state, info); });
}

vd_status vd_step_reset(vd_ctx *ctx) {
    return guarded(ctx, [&] { return vd::step_reset(ctx); });
}

vd_status vd_cell_flags(vd_ctx *ctx, const vd_problem *prob, int32_t n_levels, int32_t level, uint8_t *out) {
    return guarded(ctx, [&] { return vd::mg_cell_flags(ctx, prob, n_levels, level, out); });
}

vd_status vd_smooth(vd_ctx *ctx, const vd_problem *prob, int32_t ncolour) {
    return guarded(ctx, [&] { return vd::mg_smooth(ctx, prob, ncolour); });
}

int64_t vd_nn_param_count(const vd_nn_config *cfg) {
    try { return vd::nn_param_count(cfg); } catch (...) { return -1; }
}

vd_status vd_nn_create(vd_ctx *ctx, const vd_nn_config *cfg, const float *params) {
    return guarded(ctx, [&] { return vd::nn_create(ctx, cfg, params); });
}

vd_status vd_nn_get(vd_ctx *ctx, int32_t which, float *host) {
    return guarded(ctx, [&] { return vd::nn_params(ctx, which, host, 0); });
}

vd_status vd_nn_set(vd_ctx *ctx, int32_t which, const float *host) {
    return guarded(ctx, [&] { return vd::nn_params(ctx, which, const_cast<float *>(host), 1); });
}

vd_status vd_nn_forward(vd_ctx *ctx, const vd_grid *grid, const uint16_t *in_bf16, float *out) {
    return guarded(ctx, [&] { return vd::nn_forward(ctx, grid, in_bf16, out); });
}

vd_status vd_nn_train_step(vd_ctx *ctx, const vd_grid *grid, const uint16_t *in_bf16, const float *target, float lr,
                           int32_t update, double *loss) {
    return guarded(ctx, [&] { return vd::nn_train_step(ctx, grid, in_bf16, target, lr, update, loss); });
}

vd_status vd_nn_features(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const double *rho, double eps,
                         uint16_t *out_bf16, double *vref) {
    return guarded(ctx, [&] { return vd::nn_features(ctx, grid, phi_bc, rho, eps, out_bf16, vref); });
}

vd_status vd_nn_save(vd_ctx *ctx, const char *path) {
    return guarded(ctx, [&] { return vd::nn_save(ctx, path); });
}

vd_status vd_nn_load(vd_ctx *ctx, const char *path) {
    return guarded(ctx, [&] { return vd::nn_load(ctx, path); });
}

vd_status vd_nn_conv3d(vd_ctx *ctx, const vd_grid *grid, const uint16_t *x_bf16, int32_t ci, const float *w, const float *b,
                       int32_t co, int32_t relu, float *y, const float *dy, float *dx, float *dw, float *db) {
    return guarded(ctx, [&] { return vd::nn_conv3d(ctx, grid, x_bf16, ci, w, b, co, relu, y, dy, dx, dw, db); });
}

vd_status vd_timing_select(vd_ctx *ctx, const char *kernels) {
    return guarded(ctx, [&] {
        vd::timing_flush(ctx);
        ctx->timing.families.clear();
        ctx->timing.acc.clear();
        std::string s = kernels ? kernels : "";
        size_t pos = 0;
        while (pos < s.size()) {
            size_t e = s.find(',', pos);
            if (e == std::string::npos) e = s.size();
            if (e > pos) ctx->timing.families.push_back(s.substr(pos, e - pos));
            pos = e + 1;
        }
        return VD_OK;
    });
}

vd_status vd_timing_read(vd_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms, double *units) {
    return guarded(ctx, [&] {
        VD_CHECK(kernel, "kernel family required");
        vd::timing_flush(ctx);
        vd::TimingAcc A;
        auto it = ctx->timing.acc.find(kernel);
        if (it != ctx->timing.acc.end()) A = it->second;
        if (launches) *launches = A.launches;
        if (total_ms) *total_ms = A.total_ms;
        if (units) *units = A.units;
        return VD_OK;
    });
}

}  // extern "C"
