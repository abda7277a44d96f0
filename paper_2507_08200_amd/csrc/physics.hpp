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
    const uint8_t *mask;   // cell mask of a masked step (1 valid, 0 covered), or null
};

constexpr int kMaxSee = 8;   // ion species returning secondary electrons

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
    // right-hand side already formed by k_react (a field without drift): the
    // drift kernels leave its output alone, the wall fluxes are still added
    int rhs_done;
    // wall variants (Sec. 2.2): the sticking coefficient of a neutral wall
    // flux; secondary emission: gamma and the ion species whose wall fluxes
    // at the same face it returns (densities, signed mobilities per cell or
    // constant)
    double stick;
    double see_gamma;
    int nion;
    const double *ion_n[kMaxSee];
    const double *ion_mu[kMaxSee];
    double ion_mu_c[kMaxSee];
};

constexpr int kMaxFields = 33;

struct DriftArgs {
    GridDev g;
    const double *phi;
    const double *Te;
    double Tg, kB, me, inv_dt;
    int mode;
    const FieldDesc *f;    // device table, one entry per field (blockIdx.y)
    const uint8_t *near;   // masked step: cells whose stencils reach a covered cell (or null)
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
    double *ion;           // rate of R2 (direct ionization of Ar), or null
    // species (bit k) whose implicit right-hand side u0/dt + G (+ extra) is
    // written to rhs in place of G: fields without drift, whose right-hand
    // side needs nothing else; rhs, u0, extra: [S][cells] bases
    unsigned rhs_mask;
    double *rhs;
    const double *u0, *extra;
    double inv_dt;
};

// Photoionization terms (Sec. 2.1, Eqs. (9)-(12)): right-hand sides coef_q
// * S_i of the Helmholtz terms, then S_ph = sum_q S_q added to the sources
// of the electrons (Ge) and of an ion (Gi)
struct PhotoArgs {
    long ncell;
    int nterm;
    double coef[3];
    // each term is solved for S_q / scale[q] (a power of two near its
    // right-hand side's largest magnitude): exact in FP64, and the FP32
    // corrections of a refinement stay in range; ratio[q] = the previous
    // scale / this one rescales the stored terms, the next starting iterates
    double scale[3], inv_scale[3], ratio[3];
    const double *ion;     // S_i per cell
    double *rhs;           // [nterm][cells]
    double *S;             // [nterm][cells], scaled terms
    double *Ge, *Gi;
};

// Surface charge of one dielectric face (Sec. 2.1, Eq. (13))
struct SigmaArgs {
    GridDev g;
    const double *phi, *Te;
    const FieldDesc *f;    // device table, every species (u at the mid-point)
    int S;
    double Z[32];
    double Tg, kB, me, qe, dt, h;
    int face, na, nb, mid;
    long off;              // offset of the face's values in the packed arrays
    double *sigma;
    const double *sig0;
    double *rho;
};

// Adaptive time step (Sec. 3, Eq. (20)): per-workgroup minima
struct DtArgs {
    GridDev g;
    const double *phi, *Te, *ne;
    double N_gas, kB, qe, eps0;
    int fit;               // electron mobility from the E/N fit (else constant)
    double mu_c, D_c;
    double c_adv, c_diff, c_diel, dxmin, dt_max;
    double *partial;
};

struct RhoArgs {
    long ncell;
    int S;                 // charged species only (neutrals add nothing)
    double qe;
    double Z[32];          // their charge numbers, in species order
    int idx[32];           // and their species indices
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
bool drift25_path(const GridDev &g);
// total face flux (drift + central diffusion with cell diffusion D) of one field
void launch_face_flux(vd_ctx *ctx, DriftArgs a, const FieldDesc &field, const double *D, double *out);
void launch_react(vd_ctx *ctx, const ReactArgs &a);
void launch_rho(vd_ctx *ctx, const RhoArgs &a);
// masked step: lifting of the covered cells' potentials into the Poisson
// right-hand side of their valid neighbours, and their restore after a solve
void launch_mask_lift(vd_ctx *ctx, const GridDev &G, const double *phi_cov, const double *eps, double eps0, double *rho);
void launch_mask_restore(vd_ctx *ctx, const GridDev &G, const double *phi_cov, double *phi);
// masked step: flag the cells that are covered or have a covered cell
// within three cells along x, y or z (their drift stencils reach one)
void launch_mask_near(vd_ctx *ctx, const GridDev &G, uint8_t *near);
void launch_energy(vd_ctx *ctx, const EnergyArgs &a);
void launch_mid(vd_ctx *ctx, const double *u0, const double *u, double *out, long n);
void launch_photo_rhs(vd_ctx *ctx, const PhotoArgs &a);
// per-workgroup maxima of |S_i| (partial), returns the number of workgroups
int launch_photo_max(vd_ctx *ctx, const double *ion, long ncell, double *partial);
// out[q] = S[q] * scale[q] (the terms in physical units)
void launch_photo_unscale(vd_ctx *ctx, const PhotoArgs &a, double *out);
void launch_photo_add(vd_ctx *ctx, const PhotoArgs &a);
void launch_sigma(vd_ctx *ctx, const SigmaArgs &a, int update);
// per-workgroup minima of the time-step limits into a.partial; returns the
// number of workgroups
int launch_dt_limit(vd_ctx *ctx, const DtArgs &a);
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
