// Argument blocks of the explicit-term kernels (internal).
#pragma once
#include "vd_internal.hpp"

namespace vd {

struct GridDev {
    int n[3];
    int nxy, ncell;
    long stride[3];
    double ih[3];       // 1/h for the field
    double ihl[3];      // 1/h for the divergence
    int phi_kind[6];
    double phi_val[6];
};

// One field whose drift divergence is taken: u with signed mobility mu
// (array, or constant mu_c when mu is null), boundary kinds of the field,
// wall model; for the electron energy ne_wall is the electron density whose
// wall flux times 2 kB Te is the energy wall flux.
struct FieldDesc {
    const double *u;
    const double *mu;
    double mu_c;
    double mu_scale;       // velocity = mu_scale * mu * E (5/3 for the electron energy)
    int kind[6];
    double gval[6];
    int wall;
    double mass;
    const double *ne_wall;
    double *out;
    const double *u0;      // time level n (right-hand side mode)
    const double *src;     // chemical source (right-hand side mode)
    const double *extra;   // extra source (right-hand side mode)
};

constexpr int kMaxFields = 33;

struct DriftArgs {
    GridDev g;
    const double *phi;
    const double *Te;
    double Tg, kB, me, inv_dt;
    int mode;
    const FieldDesc *f;    // device table, one entry per field (blockIdx.y)
};

struct TransportArgs {
    GridDev g;
    const double *phi;
    double *Te;
    const double *ne, *Ee;
    int te_mode;
    const double *lfa;
    double lfa_ln_min, lfa_ln_max;
    int lfa_n;
    double N_gas, Tg, kB, qe, Te_max;
    int nvar;
    double var_sign[4];
    double *mu, *D;        // [nvar][cells]
    double *beta_e;        // 5/3 D of the variable species e_var (electron energy), or null
    int e_var;
};

struct ReactArgs {
    long ncell;
    int mech, S;
    const double *n, *Te;
    double bg0, qe;
    double *G, *S_inel;
};

struct RhoArgs {
    long ncell;
    int S;
    double qe;
    double Z[32];
    const double *n;
    double *rho;
};

struct EnergyArgs {
    GridDev g;
    const double *phi, *Te;
    double Tg, kB, me, qe, m_bg, inv_dt;
    FieldDesc fE;            // electron energy at u* (drift with 5/3 mu_e)
    FieldDesc fe;            // electron density at u* (mobility, kinds)
    const double *De;        // electron diffusion per cell (or De_c)
    double De_c;
    const double *S_inel, *extra, *Ee0;
    double *out;
};

GridDev make_grid(const vd_grid &g, const vd_bc &phi_bc);
void launch_transport(vd_ctx *ctx, const TransportArgs &a);
void launch_drift(vd_ctx *ctx, DriftArgs a, const FieldDesc *fields, int nfields, const char *tag);
// total face flux (drift + central diffusion with cell diffusion D) of one field
void launch_face_flux(vd_ctx *ctx, DriftArgs a, const FieldDesc &field, const double *D, double *out);
void launch_react(vd_ctx *ctx, const ReactArgs &a);
void launch_rho(vd_ctx *ctx, const RhoArgs &a);
void launch_energy(vd_ctx *ctx, const EnergyArgs &a);
void launch_mid(vd_ctx *ctx, const double *u0, const double *u, double *out, long n);
// Poisson guess extrapolated from earlier steps' potentials (order 0..2)
void launch_extrap(vd_ctx *ctx, double *phi, const double *h1, double *hdst, int order, long n);
// species guesses extrapolated in time (order 0..2) from FP32 histories:
// x[q] the species array, h1[q] the previous step's, hd[q] the one before
// (overwritten with x[q]), for q < count
struct ExtrapSet {
    double *x[32];
    const float *h1[32];
    float *hd[32];
};
void launch_extrap_species(vd_ctx *ctx, const ExtrapSet &e, int count, int order, long n);

vd_status mg_solve_batch(vd_ctx *ctx, int nprob, const vd_problem *probs, const vd_mg_opts *o, vd_solve_info *infos,
                         const char *cache_tag);
vd_status mg_solve_noalloc(vd_ctx *ctx, Arena *arena, int nprob, const vd_problem *probs, const vd_mg_opts *o,
                           vd_solve_info *infos);
vd_status mg_cell_flags(vd_ctx *ctx, const vd_problem *prob, int n_levels, int level, uint8_t *out);
vd_status mg_smooth(vd_ctx *ctx, const vd_problem *prob, int ncolour);

}  // namespace vd
