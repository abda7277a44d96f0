// One semi-implicit step of the plasma-fluid model (Sec. 3 of the paper):
// segregated Poisson -> electron energy -> species, explicit WENO5 drift and
// chemistry at the mid-point state u*, implicit central diffusion, with the
// mid-point corrector iteration of Eqs. (18)-(19).
#include "physics.hpp"

#include <chrono>

namespace vd {

struct StepBuffers {
    long ncell = 0;
    int S = 0;
    DevBuf<double> rho, G, b, S_inel, mu, D, n0, nstar, Ee0, Eestar, Erhs, beta_e;
    DevBuf<double> ion, photo, prhs, sig0, dtpart, phic, pmax;
    double photo_scale[3] = {1.0, 1.0, 1.0};   // scales of the stored photoionization terms
    DevBuf<uint8_t> near;
    bool photo_zeroed = false;
};

// phi arrays passed in by the previous steps with an extrapolated Poisson
// guess, except the first call after a restart (its phi is the caller's
// initial guess, not a step result): slot[newest] the last one,
// slot[1 - newest] the one before (valid when count is 2); count -1 right
// after a restart.  Keyed by the phi pointer, the grid and dt.
struct PhiHistory {
    DevBuf<double> slot[2];
    int count = -1, newest = 0;
    const double *phi = nullptr;
    int nx = 0, ny = 0, nz = 0;
    double dt = 0.0;
};

// species arrays passed in by the previous steps with extrapolated species
// guesses, rounded to FP32 (same restart rule as PhiHistory): per species,
// slot[newest] the last one, slot[1 - newest] the one before (valid when
// count is 2); count -1 right after a restart.  Keyed by the n pointer, the
// grid, S, dt and the transported species.
struct SpeciesHistory {
    DevBuf<float> slot[2];
    int count = -1, newest = 0;
    const double *n = nullptr;
    int nx = 0, ny = 0, nz = 0, S = 0;
    double dt = 0.0;
    uint32_t transported = 0;
};

static void validate_step(const vd_step_params *P, const vd_state *st) {
    VD_CHECK(P && st, "null params or state");
    const vd_grid &g = P->grid;
    VD_CHECK(g.nx >= 3 && g.ny >= 3 && g.nz >= 3 && g.dx > 0 && g.dy > 0 && g.dz > 0,
             "bad grid (WENO5 ghosts need at least 3 cells per direction)");
    VD_CHECK(P->S >= 1 && P->S <= 32, "S must be in 1..32");
    VD_CHECK(P->dt > 0 && P->n_t >= 1, "dt must be positive and n_t >= 1");
    VD_CHECK(P->species && P->species_bc, "species and species_bc are required");
    if (P->mask) {
        bool diel = false;
        for (int f = 0; f < 6; f++) diel = diel || P->diel[f];
        VD_CHECK(P->photo_n == 0 && !diel, "a masked step takes neither photoionization nor dielectric faces");
        for (int f = 0; f < 6; f++) {
            VD_CHECK(P->phi_bc.kind[f] != VD_BC_PERIODIC && P->energy_bc.kind[f] != VD_BC_PERIODIC,
                     "a masked step takes no periodic face");
            for (int k = 0; k < P->S; k++) VD_CHECK(P->species_bc[k].kind[f] != VD_BC_PERIODIC, "a masked step takes no periodic face");
        }
    }
    VD_CHECK(st->n && st->phi && st->Te, "state n, phi and Te are required");
    VD_CHECK(P->te_mode >= VD_TE_FIXED && P->te_mode <= VD_TE_ENERGY, "unknown te_mode");
    VD_CHECK(P->poisson.guess == VD_GUESS_GIVEN || P->poisson.guess == VD_GUESS_ZERO || P->poisson.guess == VD_GUESS_EXTRAP,
             "the step's Poisson guess must be GIVEN, ZERO or EXTRAP");
    VD_CHECK(P->species_mg.guess == VD_GUESS_GIVEN || P->species_mg.guess == VD_GUESS_ZERO ||
                 P->species_mg.guess == VD_GUESS_EXTRAP,
             "the step's species guess must be GIVEN, ZERO or EXTRAP");
    VD_CHECK(P->energy_mg.guess == VD_GUESS_GIVEN || P->energy_mg.guess == VD_GUESS_ZERO,
             "the step's energy guess must be GIVEN or ZERO");
    if (P->te_mode == VD_TE_LFA) VD_CHECK(P->lfa_te && P->lfa_n >= 2 && P->lfa_ln_max > P->lfa_ln_min, "LFA table required");
    if (P->te_mode == VD_TE_ENERGY) {
        VD_CHECK(st->Ee, "Ee required in energy mode");
        VD_CHECK(P->electron >= 0 && P->electron < P->S, "electron index required in energy mode");
        VD_CHECK(P->m_bg > 0, "background mass required in energy mode");
    }
    if (P->mech == VD_MECH_ARH2_15) VD_CHECK(P->S == 15, "Ar-H2 mechanism needs S = 15");
    if (P->mech == VD_MECH_AR3) VD_CHECK(P->S == 3, "argon subset needs S = 3");
    VD_CHECK(P->mech >= VD_MECH_NONE && P->mech <= VD_MECH_ARH2_15, "unknown mechanism");
    int nvar = 0;
    for (int k = 0; k < P->S; k++) {
        const vd_species &s = P->species[k];
        VD_CHECK(s.mob_kind >= 0 && s.mob_kind <= 3 && s.wall_kind >= 0 && s.wall_kind <= 3, "bad species model");
        if (s.mob_kind == VD_MOB_ELECTRON_FIT) nvar++;
        VD_CHECK(s.mob_kind == VD_MOB_CONST || P->N_gas > 0, "N_gas required for fitted mobilities");
        for (int d = 0; d < 3; d++) {
            int a = P->species_bc[k].kind[2 * d], b = P->species_bc[k].kind[2 * d + 1];
            VD_CHECK(a >= 0 && a <= 3 && b >= 0 && b <= 3 && ((a == 3) == (b == 3)), "bad species boundary kinds");
        }
    }
    VD_CHECK(nvar <= 4, "at most 4 species with field-dependent mobility");
    VD_CHECK(P->photo_n >= 0 && P->photo_n <= 3, "photo_n must be in 0..3");
    if (P->photo_n > 0) {
        VD_CHECK(P->photo_e >= 0 && P->photo_e < P->S && P->photo_ion >= 0 && P->photo_ion < P->S,
                 "photoionization species indices out of range");
        VD_CHECK(P->photo_mg.guess == VD_GUESS_GIVEN || P->photo_mg.guess == VD_GUESS_ZERO,
                 "the photoionization guess must be GIVEN or ZERO");
        for (int q = 0; q < P->photo_n; q++)
            VD_CHECK(P->photo_lambda[q] * P->photo_pO2 != 0.0, "photoionization terms need lambda_j p_O2 != 0");
    }
    VD_CHECK(P->dt_mode == 0 || P->dt_mode == 1, "dt_mode must be 0 or 1");
    if (P->dt_mode == 1) VD_CHECK(P->electron >= 0 && P->electron < P->S, "the adaptive time step needs the electron index");
    bool any_diel = false;
    for (int f = 0; f < 6; f++) any_diel = any_diel || P->diel[f];
    VD_CHECK(!any_diel || P->sigma, "dielectric faces need the sigma array");
    if (P->see_gamma != 0.0) {
        int nion = 0;
        for (int k = 0; k < P->S; k++) nion += P->species[k].wall_kind == VD_WALL_ION;
        VD_CHECK(nion <= kMaxSee, "secondary emission takes at most 8 species with the ion wall model");
    }
}

// number of values of dielectric face f's surface-charge array
static long diel_size(const vd_grid &g, int f) {
    return f < 2 ? (long)g.ny * g.nz : (f < 4 ? (long)g.nx * g.nz : (long)g.nx * g.ny);
}

static inline double sgn(double z) { return z > 0.0 ? 1.0 : (z < 0.0 ? -1.0 : 0.0); }

// constant (cell-independent) mobility and diffusion of a species
static void const_transport(const vd_species &s, const vd_step_params *P, double *mu, double *D) {
    const double N0 = 2.68e25;
    const vd_consts &c = P->consts;
    if (s.mob_kind == VD_MOB_ION_N0) {
        double m = s.mob_coef * N0 / P->N_gas;
        *mu = sgn(s.Z) * m;
        *D = m * c.kB * P->Tg / c.qe;
    } else if (s.mob_kind == VD_MOB_NEUTRAL_N0) {
        *mu = 0.0;
        *D = s.mob_coef * N0 / P->N_gas * c.kB * P->Tg / c.qe;
    } else {
        *mu = s.mu_const;
        *D = s.D_const;
    }
}

static vd_bc implicit_bc(const vd_bc &b) {
    vd_bc o = b;
    for (int f = 0; f < 6; f++)
        if (o.kind[f] == VD_BC_WALLFLUX) o.kind[f] = VD_BC_NEUMANN;
    return o;
}

vd_status step(vd_ctx *ctx, const vd_step_params *P, const vd_state *st, vd_step_info *info) {
    validate_step(P, st);
    const vd_grid &g = P->grid;
    const long N = (long)g.nx * g.ny * g.nz;
    const int S = P->S;
    const bool energy = P->te_mode == VD_TE_ENERGY;
    const bool corr = P->n_t > 1;
    hipStream_t s = ctx->stream;
    auto t_start = std::chrono::steady_clock::now();

    // buffers cached on the context for this shape
    std::string key = "step:" + std::to_string(g.nx) + "," + std::to_string(g.ny) + "," + std::to_string(g.nz) + ":" +
                      std::to_string(S);
    std::shared_ptr<StepBuffers> B;
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) B = std::static_pointer_cast<StepBuffers>(it->second);
    else { B = std::make_shared<StepBuffers>(); ctx->cache[key] = B; }
    int var_idx[32];
    int nvar = 0;
    for (int k = 0; k < S; k++) var_idx[k] = (P->species[k].mob_kind == VD_MOB_ELECTRON_FIT) ? nvar++ : -1;
    B->rho.alloc(N);
    B->G.alloc(N * S);
    B->b.alloc(N * S);
    B->S_inel.alloc(N);
    if (nvar) { B->mu.alloc(N * nvar); B->D.alloc(N * nvar); }
    if (corr) { B->n0.alloc(N * S); B->nstar.alloc(N * S); }
    if (energy) {
        B->Erhs.alloc(N);
        B->beta_e.alloc(N);
        if (corr) { B->Ee0.alloc(N); B->Eestar.alloc(N); }
    }
    if (corr) {
        VD_HIP(hipMemcpyAsync(B->n0.p, st->n, sizeof(double) * N * S, hipMemcpyDeviceToDevice, s));
        if (energy) VD_HIP(hipMemcpyAsync(B->Ee0.p, st->Ee, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    }
    const double *n_old = corr ? B->n0.p : st->n;          // u^n
    const double *Ee_old = energy ? (corr ? B->Ee0.p : st->Ee) : nullptr;

    // constant transport per species, on the host
    double mu_c[32], D_c[32];
    for (int k = 0; k < S; k++) const_transport(P->species[k], P, &mu_c[k], &D_c[k]);

    GridDev G = make_grid(g, P->phi_bc);
    G.mask = P->mask;
    // masked step: the covered cells' potentials (the Dirichlet values of
    // their faces with valid cells), before anything writes phi
    if (P->mask) {
        B->phic.alloc(N);
        VD_HIP(hipMemcpyAsync(B->phic.p, st->phi, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        B->near.alloc(N);
        launch_mask_near(ctx, G, B->near.p);
    }
    vd_step_info I;
    memset(&I, 0, sizeof(I));
    // time step: fixed, or the least of the limits of Eq. (20) over the
    // state passed in (one host synchronisation)
    double dt = P->dt;
    if (P->dt_mode == 1) {
        DtArgs da;
        memset(&da, 0, sizeof(da));
        da.g = G; da.phi = st->phi; da.Te = st->Te; da.ne = st->n + (long)P->electron * N;
        da.N_gas = P->N_gas > 0 ? P->N_gas : 1.0; da.kB = P->consts.kB; da.qe = P->consts.qe; da.eps0 = P->consts.eps0;
        da.fit = P->species[P->electron].mob_kind == VD_MOB_ELECTRON_FIT;
        da.mu_c = mu_c[P->electron]; da.D_c = D_c[P->electron];
        da.c_adv = P->c_adv; da.c_diff = P->c_diff; da.c_diel = P->c_diel;
        da.dxmin = std::min(g.dx, std::min(g.dy, g.dz));
        da.dt_max = P->dt;
        B->dtpart.alloc(ceil_div(N, kBlock));
        da.partial = B->dtpart.p;
        const int nb = launch_dt_limit(ctx, da);
        std::vector<double> part(nb);
        VD_HIP(hipMemcpyAsync(part.data(), B->dtpart.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        VD_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < nb; q++) dt = part[q] < dt ? part[q] : dt;
    }
    I.dt_used = dt;
    // surface charge of the dielectric faces at time level n
    long nsig = 0;
    long sig_off[6];
    for (int f = 0; f < 6; f++) {
        sig_off[f] = nsig;
        if (P->diel[f]) nsig += diel_size(g, f);
    }
    if (nsig) {
        B->sig0.alloc(nsig);
        VD_HIP(hipMemcpyAsync(B->sig0.p, P->sigma, sizeof(double) * nsig, hipMemcpyDeviceToDevice, s));
    }
    // photoionization: ionization rate, right-hand sides and the terms'
    // solutions (kept from call to call as the next starting iterates)
    if (P->photo_n > 0) {
        B->ion.alloc(N);
        B->prhs.alloc(N * 3);
        if (B->photo.n < (size_t)N * 3 || !B->photo.p) B->photo_zeroed = false;
        B->photo.alloc(N * 3);
        if (!B->photo_zeroed) {
            VD_HIP(hipMemsetAsync(B->photo.p, 0, sizeof(double) * N * 3, s));
            B->photo_zeroed = true;
            for (int q = 0; q < 3; q++) B->photo_scale[q] = 1.0;
        }
        B->pmax.alloc(ceil_div(N, kBlock));
    }
    // wall variants of a species' field: sticking and secondary emission
    auto wall_variants = [&](FieldDesc &F, int k, const double *nbase) {
        F.stick = P->stick ? P->stick[k] : 1.0;
        F.see_gamma = 0.0;
        F.nion = 0;
        if (P->species[k].wall_kind != VD_WALL_ELECTRON || P->see_gamma == 0.0) return;
        F.see_gamma = P->see_gamma;
        for (int q = 0; q < S; q++) {
            if (P->species[q].wall_kind != VD_WALL_ION) continue;
            F.ion_n[F.nion] = nbase + (long)q * N;
            F.ion_mu[F.nion] = var_idx[q] >= 0 ? B->mu.p + (long)var_idx[q] * N : nullptr;
            F.ion_mu_c[F.nion] = mu_c[q];
            F.nion++;
        }
    };
    const bool want_info = info != nullptr;
    hipEvent_t ev[6];
    if (want_info) for (auto &e : ev) VD_HIP(hipEventCreate(&e));
    double ms_poisson = 0, ms_transport = 0, ms_energy = 0, ms_species = 0;

    // Poisson guess of the first corrector extrapolated in time from the
    // phi arrays of the previous steps (history restarted on a new array,
    // grid or dt)
    vd_mg_opts popt = P->poisson;
    if (popt.guess == VD_GUESS_EXTRAP) {
        std::shared_ptr<PhiHistory> H;
        auto ih = ctx->cache.find("phi_history");
        if (ih != ctx->cache.end()) H = std::static_pointer_cast<PhiHistory>(ih->second);
        else { H = std::make_shared<PhiHistory>(); ctx->cache["phi_history"] = H; }
        if (H->phi != st->phi || H->nx != g.nx || H->ny != g.ny || H->nz != g.nz || H->dt != dt) {
            H->count = -1;
            H->newest = 0;
            H->phi = st->phi;
            H->nx = g.nx; H->ny = g.ny; H->nz = g.nz;
            H->dt = dt;
        }
        if (H->count < 0) {
            H->count = 0;
        } else {
            H->slot[0].alloc(N);
            H->slot[1].alloc(N);
            launch_extrap(ctx, st->phi, H->slot[H->newest].p, H->slot[1 - H->newest].p, H->count, N);
            H->newest = 1 - H->newest;
            H->count = H->count < 2 ? H->count + 1 : 2;
        }
        popt.guess = VD_GUESS_GIVEN;
    }
    // species guesses of the first corrector: history kept the same way
    vd_mg_opts sopt = P->species_mg;
    std::shared_ptr<SpeciesHistory> SH;
    if (sopt.guess == VD_GUESS_EXTRAP) {
        auto ih = ctx->cache.find("species_history");
        if (ih != ctx->cache.end()) SH = std::static_pointer_cast<SpeciesHistory>(ih->second);
        else { SH = std::make_shared<SpeciesHistory>(); ctx->cache["species_history"] = SH; }
        uint32_t tmask = 0;
        for (int k = 0; k < S; k++) if (P->species[k].transported) tmask |= 1u << k;
        if (SH->n != st->n || SH->nx != g.nx || SH->ny != g.ny || SH->nz != g.nz || SH->S != S || SH->dt != dt ||
            SH->transported != tmask) {
            SH->count = -1;
            SH->newest = 0;
            SH->n = st->n;
            SH->nx = g.nx; SH->ny = g.ny; SH->nz = g.nz; SH->S = S;
            SH->dt = dt;
            SH->transported = tmask;
        }
        sopt.guess = VD_GUESS_GIVEN;
    }

    for (int m = 0; m < P->n_t; m++) {
        // ---- u* = (u^n + u^m)/2
        const double *nst = st->n;
        const double *Est = energy ? st->Ee : nullptr;
        if (corr && m > 0) {
            launch_mid(ctx, n_old, st->n, B->nstar.p, N * S);
            nst = B->nstar.p;
            if (energy) { launch_mid(ctx, Ee_old, st->Ee, B->Eestar.p, N); Est = B->Eestar.p; }
        }
        if (want_info) VD_HIP(hipEventRecord(ev[0], s));
        // ---- Poisson at u*: -div(eps grad phi) = e sum Z n*
        RhoArgs ra;
        memset(&ra, 0, sizeof(ra));
        ra.ncell = N; ra.qe = P->consts.qe; ra.n = nst; ra.rho = B->rho.p;
        ra.S = 0;
        for (int k = 0; k < S; k++)
            if (P->species[k].Z != 0.0) { ra.Z[ra.S] = P->species[k].Z; ra.idx[ra.S] = k; ra.S++; }
        launch_rho(ctx, ra);
        // surface charge over the adjacent cells' width (mid-point value)
        auto sigma_args = [&](int f, const double *nbase) {
            SigmaArgs sa;
            memset(&sa, 0, sizeof(sa));
            sa.g = G; sa.phi = st->phi; sa.Te = st->Te; sa.S = S;
            for (int k = 0; k < S; k++) sa.Z[k] = P->species[k].Z;
            sa.Tg = P->Tg; sa.kB = P->consts.kB; sa.me = P->consts.me; sa.qe = P->consts.qe; sa.dt = dt;
            sa.h = f < 2 ? g.dx : (f < 4 ? g.dy : g.dz);
            sa.face = f;
            sa.na = f < 2 ? g.ny : g.nx;
            sa.nb = f < 4 ? g.nz : g.ny;
            sa.mid = m > 0;
            sa.off = sig_off[f];
            sa.sigma = P->sigma; sa.sig0 = B->sig0.p; sa.rho = B->rho.p;
            (void)nbase;
            return sa;
        };
        for (int f = 0; f < 6; f++)
            if (P->diel[f]) launch_sigma(ctx, sigma_args(f, nst), 0);
        if (P->mask) launch_mask_lift(ctx, G, B->phic.p, P->eps_cell, P->consts.eps0, B->rho.p);
        vd_problem pp;
        memset(&pp, 0, sizeof(pp));
        pp.grid = g; pp.bc = P->phi_bc; pp.beta = P->eps_cell; pp.beta_c = P->consts.eps0;
        pp.mask = P->mask;
        pp.rhs = B->rho.p; pp.x = st->phi;
        vd_solve_info pinfo;
        mg_solve_batch(ctx, 1, &pp, &popt, &pinfo, "poisson:");
        if (P->mask) launch_mask_restore(ctx, G, B->phic.p, st->phi);
        I.poisson_cycles += pinfo.cycles;
        I.poisson_rel = pinfo.rel_res;
        if (want_info) VD_HIP(hipEventRecord(ev[1], s));

        // ---- E/N, Te, field-dependent mobilities at u*
        TransportArgs ta;
        memset(&ta, 0, sizeof(ta));
        ta.g = G; ta.phi = st->phi; ta.Te = st->Te; ta.te_mode = P->te_mode;
        ta.ne = energy ? nst + (long)P->electron * N : nullptr;
        ta.Ee = Est;
        ta.lfa = P->lfa_te; ta.lfa_ln_min = P->lfa_ln_min; ta.lfa_ln_max = P->lfa_ln_max; ta.lfa_n = P->lfa_n;
        ta.N_gas = P->N_gas > 0 ? P->N_gas : 1.0; ta.Tg = P->Tg; ta.kB = P->consts.kB; ta.qe = P->consts.qe;
        ta.Te_max = 1e6;
        ta.nvar = nvar; ta.mu = B->mu.p; ta.D = B->D.p;
        for (int k = 0; k < S; k++) if (var_idx[k] >= 0) ta.var_sign[var_idx[k]] = sgn(P->species[k].Z);
        ta.beta_e = nullptr; ta.e_var = -1;
        if (energy && var_idx[P->electron] >= 0) { ta.beta_e = B->beta_e.p; ta.e_var = var_idx[P->electron]; }
        launch_transport(ctx, ta);

        // ---- chemistry at u*
        ReactArgs rc;
        memset(&rc, 0, sizeof(rc));
        rc.ncell = N; rc.mech = P->mech; rc.S = S; rc.n = nst; rc.Te = st->Te;
        rc.bg0 = P->mech == VD_MECH_DECAY ? P->k_decay : P->bg[0];
        rc.qe = P->consts.qe; rc.G = B->G.p; rc.S_inel = B->S_inel.p;
        rc.ion = P->photo_n > 0 ? B->ion.p : nullptr;
        // transported fields without drift: their right-hand side is
        // u^n/dt + G (+ extra), formed here in place of G, where the drift
        // kernel adds the wall-face fluxes in a pass of their own
        unsigned nodrift = 0;
        for (int k = 0; k < S && drift25_path(G); k++) {
            const bool photo_target = P->photo_n > 0 && (k == P->photo_e || k == P->photo_ion);
            if (P->species[k].transported && var_idx[k] < 0 && mu_c[k] == 0.0 && !photo_target) nodrift |= 1u << k;
        }
        rc.rhs_mask = nodrift; rc.rhs = B->b.p; rc.u0 = n_old; rc.extra = P->extra_source; rc.inv_dt = 1.0 / dt;
        launch_react(ctx, rc);
        // photoionization (Sec. 2.1, Eqs. (9)-(12)) into the sources
        if (P->photo_n > 0) {
            PhotoArgs pa;
            memset(&pa, 0, sizeof(pa));
            pa.ncell = N; pa.nterm = P->photo_n; pa.ion = B->ion.p; pa.rhs = B->prhs.p; pa.S = B->photo.p;
            pa.Ge = B->G.p + (long)P->photo_e * N; pa.Gi = B->G.p + (long)P->photo_ion * N;
            const double cem = P->photo_pq / (P->photo_p + P->photo_pq) * P->photo_xi * P->photo_nu_ratio;
            vd_problem pr[3];
            memset(pr, 0, sizeof(pr));
            // each term's scale: the power of two at or above its
            // right-hand side's largest magnitude (one host synchronisation)
            const int nbm = launch_photo_max(ctx, B->ion.p, N, B->pmax.p);
            std::vector<double> pm(nbm);
            VD_HIP(hipMemcpyAsync(pm.data(), B->pmax.p, sizeof(double) * nbm, hipMemcpyDeviceToHost, s));
            VD_HIP(hipStreamSynchronize(s));
            double mion = 0.0;
            for (double v : pm) mion = v > mion ? v : mion;
            for (int q = 0; q < P->photo_n; q++) {
                pa.coef[q] = P->photo_A[q] * P->photo_pg * P->photo_pg * cem;
                const double m = std::fabs(pa.coef[q]) * mion;
                int e = 0;
                double sc = 1.0;
                if (m > 0.0 && std::isfinite(m)) (void)std::frexp(m, &e);
                // a power of two whose inverse is finite and normal (a
                // right-hand side below 2^-1000 keeps the scale 1)
                if (e > -1000 && e < 1000) sc = std::ldexp(1.0, e);
                pa.scale[q] = sc;
                pa.inv_scale[q] = 1.0 / sc;
                // the stored terms, rescaled exactly (both scales are powers
                // of two); a ratio beyond the normal range restarts from zero
                pa.ratio[q] = B->photo_scale[q] / sc;
                if (!std::isnormal(pa.ratio[q])) pa.ratio[q] = 0.0;
                B->photo_scale[q] = sc;
                const double kl = P->photo_lambda[q] * P->photo_pO2;
                pr[q].grid = g; pr[q].bc = P->photo_bc; pr[q].alpha_c = kl * kl; pr[q].beta_c = 1.0;
                for (int f = 0; f < 6; f++) pr[q].bc.value[f] = P->photo_bc.value[f] * pa.inv_scale[q];
                pr[q].rhs = B->prhs.p + (long)q * N; pr[q].x = B->photo.p + (long)q * N;
            }
            launch_photo_rhs(ctx, pa);
            mg_solve_batch(ctx, P->photo_n, pr, &P->photo_mg, nullptr, "photo:");
            launch_photo_add(ctx, pa);
        }
        if (want_info) VD_HIP(hipEventRecord(ev[2], s));

        // ---- electron energy
        if (energy) {
            const int e = P->electron;
            EnergyArgs ea;
            memset(&ea, 0, sizeof(ea));
            ea.g = G; ea.phi = st->phi; ea.Te = st->Te; ea.Tg = P->Tg; ea.kB = P->consts.kB; ea.me = P->consts.me;
            ea.qe = P->consts.qe; ea.m_bg = P->m_bg; ea.inv_dt = 1.0 / dt;
            FieldDesc fe;
            memset(&fe, 0, sizeof(fe));
            fe.u = nst + (long)e * N;
            fe.mu = var_idx[e] >= 0 ? B->mu.p + (long)var_idx[e] * N : nullptr;
            fe.mu_c = mu_c[e];
            fe.mu_scale = 1.0;
            for (int f = 0; f < 6; f++) { fe.kind[f] = P->species_bc[e].kind[f]; fe.gval[f] = P->species_bc[e].value[f]; }
            fe.wall = VD_WALL_ELECTRON; fe.mass = P->consts.me;
            wall_variants(fe, e, nst);
            FieldDesc fE = fe;
            fE.u = Est;
            fE.mu_scale = 5.0 / 3.0;
            for (int f = 0; f < 6; f++) { fE.kind[f] = P->energy_bc.kind[f]; fE.gval[f] = P->energy_bc.value[f]; }
            fE.ne_wall = nst + (long)e * N;
            ea.fE = fE; ea.fe = fe;
            ea.De = var_idx[e] >= 0 ? B->D.p + (long)var_idx[e] * N : nullptr;
            ea.De_c = D_c[e];
            ea.S_inel = B->S_inel.p; ea.extra = P->extra_energy; ea.Ee0 = Ee_old; ea.out = B->Erhs.p;
            launch_energy(ctx, ea);
            vd_problem ep;
            memset(&ep, 0, sizeof(ep));
            ep.grid = g; ep.bc = implicit_bc(P->energy_bc); ep.alpha_c = 1.0 / dt;
            ep.mask = P->mask;
            ep.beta = var_idx[e] >= 0 ? B->beta_e.p : nullptr;
            ep.beta_c = 5.0 / 3.0 * D_c[e];
            ep.rhs = B->Erhs.p; ep.x = st->Ee;
            vd_solve_info einfo;
            mg_solve_batch(ctx, 1, &ep, &P->energy_mg, &einfo, "energy:");
            I.energy_cycles = std::max(I.energy_cycles, einfo.cycles);
        }
        if (want_info) VD_HIP(hipEventRecord(ev[3], s));

        // ---- species right-hand sides: n^n/dt - div(mu n* E)_WENO + G(u*) + extra
        DriftArgs da;
        memset(&da, 0, sizeof(da));
        da.g = G; da.phi = st->phi; da.Te = st->Te; da.Tg = P->Tg; da.kB = P->consts.kB; da.me = P->consts.me;
        da.inv_dt = 1.0 / dt; da.mode = 1;
        da.near = P->mask ? B->near.p : nullptr;
        vd_problem sp[32];
        FieldDesc fds[32];
        memset(fds, 0, sizeof(fds));
        int nf = 0;
        for (int k = 0; k < S; k++) {
            if (!P->species[k].transported) continue;
            FieldDesc &F = fds[nf];
            F.u = nst + (long)k * N;
            F.mu = var_idx[k] >= 0 ? B->mu.p + (long)var_idx[k] * N : nullptr;
            F.mu_c = mu_c[k];
            F.mu_scale = 1.0;
            for (int f = 0; f < 6; f++) { F.kind[f] = P->species_bc[k].kind[f]; F.gval[f] = P->species_bc[k].value[f]; }
            F.wall = P->species[k].wall_kind;
            F.mass = P->species[k].mass_kg;
            F.ne_wall = nullptr;
            F.out = B->b.p + (long)k * N;
            F.u0 = n_old + (long)k * N;
            F.src = B->G.p + (long)k * N;
            F.extra = P->extra_source ? P->extra_source + (long)k * N : nullptr;
            F.rhs_done = (nodrift >> k) & 1u;
            wall_variants(F, k, nst);
            vd_problem &q = sp[nf];
            memset(&q, 0, sizeof(q));
            q.grid = g; q.bc = implicit_bc(P->species_bc[k]); q.alpha_c = 1.0 / dt;
            q.mask = P->mask;
            q.beta = var_idx[k] >= 0 ? B->D.p + (long)var_idx[k] * N : nullptr;
            q.beta_c = D_c[k];
            q.rhs = F.out; q.x = st->n + (long)k * N;
            nf++;
        }
        launch_drift(ctx, da, fds, nf, "step");
        // surface charge (Sec. 2.1, Eq. (13)) from the wall fluxes of this
        // mid-point state, before the species arrays are overwritten
        if (nsig) {
            FieldDesc all[32];
            memset(all, 0, sizeof(all));
            for (int k = 0; k < S; k++) {
                FieldDesc &F = all[k];
                F.u = nst + (long)k * N;
                F.mu = var_idx[k] >= 0 ? B->mu.p + (long)var_idx[k] * N : nullptr;
                F.mu_c = mu_c[k];
                F.mu_scale = 1.0;
                for (int f = 0; f < 6; f++) { F.kind[f] = P->species_bc[k].kind[f]; F.gval[f] = P->species_bc[k].value[f]; }
                F.wall = P->species[k].wall_kind;
                F.mass = P->species[k].mass_kg;
                wall_variants(F, k, nst);
            }
            const FieldDesc *dall = (const FieldDesc *)upload_blob(ctx, "fields:sigma", all, sizeof(FieldDesc) * S);
            for (int f = 0; f < 6; f++) {
                if (!P->diel[f]) continue;
                SigmaArgs sa = sigma_args(f, nst);
                sa.f = dall;
                launch_sigma(ctx, sa, 1);
            }
        }
        // the right-hand sides hold u^n now: the first corrector's species
        // iterates may start from the extrapolated guesses
        if (SH && m == 0) {
            if (SH->count < 0) {
                SH->count = 0;
            } else {
                SH->slot[0].alloc((size_t)N * S);
                SH->slot[1].alloc((size_t)N * S);
                ExtrapSet e;
                memset(&e, 0, sizeof(e));
                int q = 0;
                for (int k = 0; k < S; k++) {
                    if (!P->species[k].transported) continue;
                    e.x[q] = st->n + (long)k * N;
                    e.h1[q] = SH->slot[SH->newest].p + (long)k * N;
                    e.hd[q] = SH->slot[1 - SH->newest].p + (long)k * N;
                    q++;
                }
                launch_extrap_species(ctx, e, q, SH->count, N);
                SH->newest = 1 - SH->newest;
                SH->count = SH->count < 2 ? SH->count + 1 : 2;
            }
        }
        if (want_info) VD_HIP(hipEventRecord(ev[4], s));
        if (nf) {
            vd_solve_info sinfo[32];
            mg_solve_batch(ctx, nf, sp, &sopt, want_info ? sinfo : nullptr, "species:");
            if (want_info)
                for (int q = 0; q < nf; q++) I.species_cycles = std::max(I.species_cycles, sinfo[q].cycles);
        }
        if (want_info) {
            VD_HIP(hipEventRecord(ev[5], s));
            VD_HIP(hipEventSynchronize(ev[5]));
            float a;
            VD_HIP(hipEventElapsedTime(&a, ev[0], ev[1])); ms_poisson += a;
            VD_HIP(hipEventElapsedTime(&a, ev[1], ev[2])); ms_transport += a;
            VD_HIP(hipEventElapsedTime(&a, ev[2], ev[3])); ms_energy += a;
            VD_HIP(hipEventElapsedTime(&a, ev[3], ev[5])); ms_species += a;
        }
    }
    if (P->photo_n > 0 && P->photo_out) {
        PhotoArgs pu;
        memset(&pu, 0, sizeof(pu));
        pu.ncell = N; pu.nterm = P->photo_n; pu.S = B->photo.p;
        for (int q = 0; q < P->photo_n; q++) pu.scale[q] = B->photo_scale[q];
        launch_photo_unscale(ctx, pu, P->photo_out);
    }
    if (energy) {
        // Te from the new electron energy and density
        TransportArgs ta;
        memset(&ta, 0, sizeof(ta));
        ta.g = G; ta.phi = st->phi; ta.Te = st->Te; ta.te_mode = VD_TE_ENERGY;
        ta.ne = st->n + (long)P->electron * N; ta.Ee = st->Ee;
        ta.N_gas = P->N_gas > 0 ? P->N_gas : 1.0; ta.Tg = P->Tg; ta.kB = P->consts.kB; ta.qe = P->consts.qe;
        ta.Te_max = 1e6; ta.nvar = 0;
        launch_transport(ctx, ta);
    }
    if (want_info) {
        VD_HIP(hipStreamSynchronize(s));
        for (auto &e : ev) (void)hipEventDestroy(e);
        I.ms_poisson = ms_poisson; I.ms_transport = ms_transport; I.ms_energy = ms_energy; I.ms_species = ms_species;
        I.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        I.status = VD_OK;
        *info = I;
    }
    return VD_OK;
}

// Forget both histories of extrapolated guesses: the next vd_step with
// VD_GUESS_EXTRAP starts as after a restart.
vd_status step_reset(vd_ctx *ctx) {
    auto ih = ctx->cache.find("phi_history");
    if (ih != ctx->cache.end()) {
        auto H = std::static_pointer_cast<PhiHistory>(ih->second);
        H->count = -1; H->newest = 0; H->phi = nullptr;
    }
    auto is = ctx->cache.find("species_history");
    if (is != ctx->cache.end()) {
        auto H = std::static_pointer_cast<SpeciesHistory>(is->second);
        H->count = -1; H->newest = 0; H->n = nullptr;
    }
    return VD_OK;
}

// Standalone drift divergence (vd_species_flux), and the total face flux
// of one species when asked for.
vd_status species_flux(vd_ctx *ctx, const vd_grid *g, const vd_bc *phi_bc, const vd_bc *sp_bc, int S, const vd_species *sp,
                       const double *n, const double *phi, const double *mu, const double *D, const double *Te, double Tg,
                       const vd_consts *c, double *div, int flux_species, double *face_flux) {
    VD_CHECK(g && phi_bc && sp_bc && sp && n && phi && mu && Te && c && div, "null argument");
    VD_CHECK(S >= 1 && S <= kMaxFields, "S out of range");
    VD_CHECK(g->nx >= 3 && g->ny >= 3 && g->nz >= 3, "WENO5 ghosts need at least 3 cells per direction");
    VD_CHECK(!face_flux || (flux_species >= 0 && flux_species < S && D),
             "face fluxes need a species index in 0..S-1 and the diffusion coefficients");
    const long N = (long)g->nx * g->ny * g->nz;
    DriftArgs da;
    memset(&da, 0, sizeof(da));
    da.g = make_grid(*g, *phi_bc);
    da.phi = phi; da.Te = Te; da.Tg = Tg; da.kB = c->kB; da.me = c->me; da.mode = 0;
    FieldDesc fds[kMaxFields];
    memset(fds, 0, sizeof(fds));
    for (int k = 0; k < S; k++) {
        FieldDesc &F = fds[k];
        F.u = n + (long)k * N;
        F.mu = mu + (long)k * N;
        F.mu_scale = 1.0;
        for (int f = 0; f < 6; f++) { F.kind[f] = sp_bc[k].kind[f]; F.gval[f] = sp_bc[k].value[f]; }
        F.wall = sp[k].wall_kind;
        F.mass = sp[k].mass_kg;
        F.stick = 1.0;
        F.out = div + (long)k * N;
    }
    launch_drift(ctx, da, fds, S, "flux");
    if (face_flux) launch_face_flux(ctx, da, fds[flux_species], D + (long)flux_species * N, face_flux);
    return VD_OK;
}

vd_status reaction_source(vd_ctx *ctx, int mech, long ncell, int S, const double *n, const double *Te, const double *bg,
                          double qe, double *G, double *S_inel) {
    VD_CHECK(n && Te && G && ncell > 0, "null argument");
    VD_CHECK(mech >= VD_MECH_NONE && mech <= VD_MECH_ARH2_15, "unknown mechanism");
    VD_CHECK(mech != VD_MECH_ARH2_15 || S == 15, "Ar-H2 mechanism needs S = 15");
    VD_CHECK(mech != VD_MECH_AR3 || S == 3, "argon subset needs S = 3");
    VD_CHECK(S >= 1 && S <= 32, "S out of range");
    ReactArgs rc;
    memset(&rc, 0, sizeof(rc));
    rc.ncell = ncell; rc.mech = mech; rc.S = S; rc.n = n; rc.Te = Te;
    rc.bg0 = bg ? bg[0] : 0.0; rc.qe = qe; rc.G = G; rc.S_inel = S_inel;
    launch_react(ctx, rc);
    return VD_OK;
}

}  // namespace vd
