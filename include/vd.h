/*
 * vd.h -- C ABI of libvd, an MI355X (gfx950) implementation of the hot path
 * of one semi-implicit non-equilibrium plasma-fluid time step on a uniform
 * 3D Cartesian grid (Vidyut3d, arXiv 2507.08200).
 *
 * Conventions for every entry point:
 *   - Array arguments documented "device" are device pointers owned by the
 *     caller (allocated in HBM, e.g. by PyTorch); the library never frees
 *     them.  Arrays documented "host" are ordinary host memory.
 *   - Cell arrays are contiguous [nz][ny][nx] (x fastest); multi-field
 *     arrays are [S][nz][ny][nx].  FP64 unless noted.  SI units; electron
 *     temperature in kelvin.
 *   - Boundary faces are indexed x-, x+, y-, y+, z-, z+.
 *   - Work is enqueued on the context's stream in order.  A function that
 *     fills a host info struct synchronises that stream before returning.
 *   - Errors are status codes; no exception crosses the ABI.  The message of
 *     the last failure is available from vd_last_error().  Arguments are
 *     validated on the host before anything is launched; on VD_EINVAL no
 *     device memory has been touched.
 *   - One context per host thread.  Calls on one context must not overlap.
 */
#ifndef VD_H
#define VD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vd_ctx vd_ctx;

typedef enum {
    VD_OK = 0,
    VD_EINVAL = -1,      /* bad argument (shape, kind, pointer, option) */
    VD_ENOMEM = -2,      /* device allocation failed */
    VD_EHIP = -3,        /* HIP runtime error */
    VD_ENOCONV = -4,     /* solver did not reach the tolerance, or produced a non-finite residual */
    VD_ESINGULAR = -5    /* operator is singular (alpha = 0, no Dirichlet face, no mask) */
} vd_status;

/* Boundary kinds (per domain face).  DIRICHLET imposes a face value
 * (ghost 2g - x_c); NEUMANN a zero normal gradient; WALLFLUX (species and
 * electron energy) a zero diffusive flux in the implicit operator with the
 * wall flux of Sec. 2.2 entering through the drift divergence; PERIODIC
 * wraps (both faces of a direction or neither). */
enum { VD_BC_DIRICHLET = 0, VD_BC_NEUMANN = 1, VD_BC_WALLFLUX = 2, VD_BC_PERIODIC = 3 };

enum { VD_FP64 = 0, VD_FP32_IR = 1 };                               /* vd_mg_opts.precision */
/* vd_mg_opts.guess.  VD_GUESS_EXTRAP (vd_step's Poisson and species solves
 * only; not in the paper): the solve starts from a polynomial extrapolation
 * in time of the arrays passed in by this context's earlier vd_step calls,
 * see vd_step. */
enum { VD_GUESS_GIVEN = 0, VD_GUESS_ZERO = 1, VD_GUESS_LEARNED = 2, VD_GUESS_EXTRAP = 3 };
/* vd_mg_opts.flags.  VD_MG_GRAPH: in tolerance mode each cycle (residual
 * check + V-cycle, or the IR outer step) is replayed from a HIP graph
 * captured on the first call for this problem shape and options, instead of
 * being launched kernel by kernel (ignored while kernel timing is on).
 * VD_MG_AUTOTUNE: on the first solve of a problem shape, time each level's
 * smoother for the candidate tile depths and keep the fastest,
 * and choose between two in-place colour passes and one out-of-place sweep
 * (both colours in one launch, recomputing the red values of a one-cell
 * ring around each tile) for each level (the iterate is restored
 * afterwards; every variant computes the same values).  VD_MG_FUSED_SWEEP:
 * use the out-of-place sweep on every tiled level without timing.  Tuning
 * results and the forced choice stay with the context's cached hierarchy of
 * that problem shape.  VD_MG_TUNE_NU (tolerance mode only): on the first
 * solve of a problem shape, time solves (the faster of two) with the
 * caller's schedule and with each V(nu_pre, nu_post) of (1,1), (2,1), (1,2),
 * (2,2), (3,3) from the caller's starting iterates (restored after each),
 * and keep the fastest to reach the tolerance, another than the caller's
 * only if more than 3 % faster, for this and later solves of the shape
 * (reported in
 * vd_solve_info.nu_pre / nu_post; the iterates change, the stopping test
 * does not).  When the environment variable VD_TUNE_CACHE names a file,
 * the choice is looked up there first (key: a hash of the problem shapes,
 * precision, levels, rtol and the solve's role) and appended after tuning,
 * so later processes skip it.  Not with vd_poisson_solve_noalloc.
 * VD_MG_PERSISTENT: the tiled colour passes run as persistent launches (a
 * fixed grid of resident workgroups walking the level's (problem, tile)
 * items) instead of one workgroup per tile; same values. */
enum { VD_MG_GRAPH = 1, VD_MG_AUTOTUNE = 2, VD_MG_FUSED_SWEEP = 4, VD_MG_TUNE_NU = 8, VD_MG_PERSISTENT = 16 };
enum { VD_TE_FIXED = 0, VD_TE_LFA = 1, VD_TE_ENERGY = 2 };          /* electron temperature */
enum { VD_MECH_NONE = 0, VD_MECH_DECAY = 1, VD_MECH_AR3 = 2, VD_MECH_ARH2_15 = 3 };
/* mobility models (Table A.4 with the Einstein relation):
 *   CONST:        mu = mu_const (signed), D = D_const
 *   ELECTRON_FIT: |mu| = exp(0.05481 - 2.911 tanh(0.289 ln(E/N) + 0.543)) 1.1296e25/N,
 *                 mu = sign(Z)|mu|, D = |mu| kB Te / e
 *   ION_N0:       |mu| = mob_coef N0/N, mu = sign(Z)|mu|, D = |mu| kB Tg / e
 *   NEUTRAL_N0:   mu = 0, D = mob_coef (N0/N) kB Tg / e (the ionic counterpart's) */
enum { VD_MOB_CONST = 0, VD_MOB_ELECTRON_FIT = 1, VD_MOB_ION_N0 = 2, VD_MOB_NEUTRAL_N0 = 3 };
/* wall-flux models at WALLFLUX faces (Sec. 2.2, Eqs. (14) and (16), and the
 * neutral variant stated after them):
 *   ELECTRON: n/4 sqrt(8 kB Te/(pi m_e)); ION: max(mu n E.n, 0);
 *   NEUTRAL: n/4 sqrt(8 kB Tg/(pi m)); NONE: no flux (background gas). */
enum { VD_WALL_NONE = 0, VD_WALL_ELECTRON = 1, VD_WALL_ION = 2, VD_WALL_NEUTRAL = 3 };

typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } vd_grid;
typedef struct { int32_t kind[6]; double value[6]; } vd_bc;

/* Multigrid options.  Cycles: V(nu_pre, nu_post) with red-black Gauss-Seidel,
 * mean-of-8 restriction, piecewise-constant prolongation, FP64
 * Jacobi-preconditioned CG on the coarsest level (to 1e-14 or 500
 * iterations).  Levels: n_levels if > 0 (each coarsening needs every
 * dimension even), otherwise coarsen while every dimension is even and
 * larger than 4.  With one level a cycle is nu_pre + nu_post sweeps.
 * Stopping: before each cycle ||b - A x||_2 / ||b||_2 over valid cells (b
 * including the Dirichlet lifting) is compared with rtol; fixed_cycles > 0
 * runs exactly that many cycles instead.  precision = VD_FP32_IR runs the
 * cycles in FP32 on the FP64 residual and adds the FP32 correction to the
 * FP64 iterate (iterative refinement; ir_inner cycles per outer step; the
 * outer residual, face coefficients and bottom solve stay FP64). */
typedef struct {
    double rtol;
    int32_t max_cycles;
    int32_t fixed_cycles;
    int32_t nu_pre, nu_post;
    int32_t n_levels;
    int32_t precision;
    int32_t guess;
    int32_t ir_inner;
    int32_t flags;          /* VD_MG_* bits */
} vd_mg_opts;

/* cycles: V-cycles run (FP32 cycles in IR mode); outer_iters: FP64
 * residual evaluations in IR mode; rel_res0 / rel_res: relative residual
 * before the first and after the last cycle; bnorm = ||b||_2; status as the
 * return code for this problem; fallback = 1 if a learned guess was
 * rejected; nu_pre / nu_post: the smoothing schedule the solve used. */
typedef struct {
    int32_t cycles, outer_iters, fallback, levels, status, pad;
    double rel_res, rel_res0, bnorm;
    int32_t nu_pre, nu_post;
} vd_solve_info;

/* One Helmholtz problem (alpha - div(beta grad)) x = rhs (Sec. 3, the
 * Helmholtz casting of each implicit equation; Sec. 4).  Cell-centred
 * alpha and beta; face coefficients are harmonic means of the two cells
 * (the boundary cell's value on a domain face).  NULL alpha / beta mean
 * uniform alpha_c / beta_c.  mask (uint8, nullable): 1 valid, 0 covered;
 * covered cells hold 0 and act as a homogeneous Dirichlet face for their
 * valid neighbours (cell masking of Sec. 3).  rhs, x: device cell arrays; x
 * holds the initial guess on entry and the solution on exit. */
typedef struct {
    vd_grid grid;
    vd_bc bc;
    const uint8_t *mask;
    const double *alpha;
    double alpha_c;
    const double *beta;
    double beta_c;
    const double *rhs;
    double *x;
} vd_problem;

typedef struct {
    double Z;               /* charge number */
    double mass_kg;
    int32_t transported;    /* 0: density held fixed in the step */
    int32_t mob_kind;       /* VD_MOB_* */
    int32_t wall_kind;      /* VD_WALL_* */
    int32_t pad;
    double mob_coef, mu_const, D_const;
} vd_species;

typedef struct { double qe, eps0, kB, me; } vd_consts;

/* ------------------------------------------------------------------ */
vd_status vd_ctx_create(vd_ctx **out, void *hip_stream /* hipStream_t, NULL = default stream */);
void vd_ctx_destroy(vd_ctx *ctx);
vd_status vd_ctx_set_stream(vd_ctx *ctx, void *hip_stream);
const char *vd_last_error(const vd_ctx *ctx);
const char *vd_version(void);

/* Electrostatic Poisson (Sec. 2.1, Eqs. (3)-(4)) in Helmholtz form:
 *   -div(beta grad phi) = rho,  beta = eps (beta_cell, NULL = beta_c everywhere),
 *   rho = e sum_k Z_k n_k (C/m^3; device cell array).
 * phi: device cell array, initial guess in (ignored for VD_GUESS_ZERO),
 * solution out.  Electrodes are Dirichlet faces of phi_bc.
 * VD_ESINGULAR when no face is Dirichlet and no mask is given. */
vd_status vd_poisson_solve(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const uint8_t *mask,
                           const double *beta_cell, double beta_c, const double *rho, double *phi,
                           const vd_mg_opts *opts, vd_solve_info *info /* host, nullable */);

/* vd_poisson_solve without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, arithmetic and results
 * as vd_poisson_solve, bit for bit.  Every multigrid array, plan and
 * descriptor table of the solve is carved from one static device array of
 * 64 MiB per GPU, which the library holds from the first context created on
 * that GPU until the process ends; the call makes no hipMalloc, hipFree or
 * hipHostMalloc and no allocating library call.  The hierarchy is rebuilt
 * on every call (nothing is cached between calls), so the call costs
 * set-up time that vd_poisson_solve spends only once per shape.  Fits, for
 * example, a 160^3 uniform-permittivity solve in FP64 or in FP32
 * refinement; a problem whose hierarchy needs more than 64 MiB returns
 * VD_EINVAL with the caller's arrays untouched.  opts.flags must not ask for
 * VD_MG_GRAPH or VD_MG_AUTOTUNE (they allocate) and opts.guess must be
 * VD_GUESS_GIVEN or VD_GUESS_ZERO; otherwise VD_EINVAL.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (other
 * streams, other contexts, other host threads) race and give undefined
 * results; calls ordered on one stream are safe.  The current device must
 * be the one the context's stream runs on. */
vd_status vd_poisson_solve_noalloc(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const uint8_t *mask,
                                   const double *beta_cell, double beta_c, const double *rho, double *phi,
                                   const vd_mg_opts *opts, vd_solve_info *info /* host, nullable */);

/* nprob independent Helmholtz problems of possibly different sizes solved
 * together (Sec. 7: several components per multigrid solve): one launch per
 * smoother colour covers every problem's level, coarse levels of all
 * problems run in one fused launch, and per-problem convergence flags live
 * on the device.  probs, infos: host arrays [nprob]. */
vd_status vd_helmholtz_solve_batched(vd_ctx *ctx, int32_t nprob, const vd_problem *probs,
                                     const vd_mg_opts *opts, vd_solve_info *infos /* host, nullable */);

/* Divergence of the drift flux mu_k n_k E of every species (Sec. 2.1,
 * Eq. (2); WENO5 upwind reconstruction of Sec. 3): face velocity
 * v = mu_f E_f with E_f = -(phi_R - phi_L)/h (Dirichlet faces of phi_bc:
 * over half a cell; Neumann: 0) and mu_f the mean of the two cells' signed
 * mobilities; flux = v times the upwind WENO5 value (ghosts: mirror at
 * Neumann/wall faces, odd reflection at Dirichlet faces, wrap at periodic).
 * WALLFLUX faces of species_bc[k] carry the wall flux of species[k].wall_kind
 * at the boundary cell instead (Sec. 2.2: electron and ion wall fluxes,
 * Eqs. (14) and (16), and the neutral variant with Tg).
 *   n, mu: device [S][cells]; phi, Te_K: device cells; Tg: gas temperature.
 *   div_drift: device [S][cells] output.
 * Optional total face flux of species flux_species (face_flux non-NULL;
 * then D, device [S][cells] cell diffusion coefficients, is required and
 * 0 <= flux_species < S): Gamma . e_d = drift part as above (the wall flux,
 * with the outward normal's sign, at a WALLFLUX face; 0 at a Neumann face)
 * plus the central diffusive part -D_f (n_R - n_L)/h of Sec. 3 (D_f the
 * harmonic mean of the two cells' D; a Dirichlet face over half a cell with
 * the boundary cell's D; 0 at Neumann and WALLFLUX faces), the flux Gamma_e
 * whose cell mean enters the Joule term of Eq. (8).  face_flux: device FP64
 * x faces [nz][ny][nx+1], then y faces [nz][ny+1][nx], then z faces
 * [nz+1][ny][nx].  D may be NULL and flux_species anything when face_flux
 * is NULL. */
vd_status vd_species_flux(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const vd_bc *species_bc /* host[S] */,
                          int32_t S, const vd_species *species /* host[S] */, const double *n, const double *phi,
                          const double *mu, const double *D, const double *Te_K, double Tg, const vd_consts *consts,
                          double *div_drift, int32_t flux_species, double *face_flux);

/* Chemical production rates G_k = sum_i nu_ik r_i, r_i = k_i(Te) prod n
 * (#/m^3/s) and electron inelastic loss sum_i dE_i e r_i (J/m^3/s) of the
 * mechanism of Appendix A (Tables A.1-A.3).  mech VD_MECH_ARH2_15: S = 15
 * in the order e, Ar+, Ar2+, H+, H2+, H3+, ArH+, Ar*, Ar2*, H2(v1), H2(v2),
 * H2(v3), H, Ar, H2.  VD_MECH_AR3: S = 3 (e, Ar+, Ar*) with background Ar
 * density bg[0] and reactions R1-R5, R12, R13.  VD_MECH_DECAY: G = -k n for
 * every species (k = bg[0]).  n: device [S][ncells]; Te_K: device cells;
 * G: device [S][ncells]; S_inel: device cells or NULL. */
vd_status vd_reaction_source(vd_ctx *ctx, int32_t mech, int64_t ncells, int32_t S, const double *n,
                             const double *Te_K, const double *bg /* host[4] */, double qe, double *G,
                             double *S_inel);

/* Parameters of one semi-implicit step (Sec. 3). */
typedef struct {
    vd_grid grid;
    double dt;
    int32_t n_t;            /* mid-point corrector iterations, Eqs. (18)-(19) (1 = Backward Euler) */
    int32_t mech;           /* VD_MECH_* */
    int32_t S;              /* species count, 1..32 */
    int32_t te_mode;        /* VD_TE_* */
    int32_t electron;       /* index of the electron species, -1 if none */
    int32_t pad0;
    double Tg;              /* gas temperature, K */
    double N_gas;           /* gas number density for E/N and ion mobilities, m^-3 */
    double m_bg;            /* background neutral mass for the elastic loss, kg */
    double k_decay;         /* VD_MECH_DECAY rate */
    double bg[4];           /* background densities used by the mechanism */
    vd_consts consts;
    vd_bc phi_bc;
    vd_bc energy_bc;
    const vd_bc *species_bc;        /* host [S] */
    const vd_species *species;      /* host [S] */
    const double *lfa_te;           /* device [lfa_n], Te (K) on uniform ln(E/N[Td]) nodes */
    double lfa_ln_min, lfa_ln_max;
    int32_t lfa_n, pad1;
    const double *extra_source;     /* device [S][cells] or NULL */
    const double *extra_energy;     /* device cells or NULL */
    const double *eps_cell;         /* device cells or NULL (eps0) */
    vd_mg_opts poisson, species_mg, energy_mg;
    /* Photoionization (Sec. 2.1, Eqs. (9)-(12)): photo_n terms (0 = off,
     * at most 3), each (lambda_j p_O2)^2 S_j - lap S_j = A_j p_g^2 I under
     * photo_bc, solved after the chemistry of every corrector; S_ph = sum_j
     * S_j is added to the sources of species photo_e (electrons) and
     * photo_ion.  Emission function I = p_q / (p + p_q) * xi * nu_ratio *
     * S_i with S_i the rate of R2 (e + Ar -> Ar+ + 2e, direct ionization of
     * the background gas; 0 for mechanisms without it); nu_ratio = 1 gives
     * Eq. (11), the ratio nu_u / nu_i Eq. (12).  Units are the caller's:
     * lambda_j p_O2 in 1/m, A_j p_g^2 in 1/m^2.  photo_mg.guess: VD_GUESS_GIVEN
     * starts each term from its solution of the previous call (zero at
     * first), VD_GUESS_ZERO from zero.  photo_out: device [3][cells] or NULL,
     * receives the S_j of the last corrector.  Each term is solved for S_j /
     * 2^e, 2^e the power of two at or above its right-hand side's largest
     * magnitude (exact in FP64; keeps VD_FP32_IR corrections in range; one
     * host synchronisation per corrector). */
    int32_t photo_n, photo_e, photo_ion;
    int32_t dt_mode;                /* 0: dt; 1: adaptive time step (Sec. 3, Eq. (20)) */
    double photo_A[3], photo_lambda[3];
    double photo_pO2, photo_pg, photo_xi, photo_pq, photo_p, photo_nu_ratio;
    vd_bc photo_bc;
    vd_mg_opts photo_mg;
    double *photo_out;
    /* Adaptive time step (dt_mode 1): the least over cells of c_adv dx_min /
     * (|mu_e| |E|), c_diff / 3 dx_min^2 / (2 D_e) and c_diel eps0 / (e |mu_e|
     * n_e) for the electron species `electron`, from the phi, Te and n
     * passed in; dt is the largest step taken; the step taken is returned in
     * vd_step_info.dt_used.  Synchronises the stream once per step. */
    double c_adv, c_diff, c_diel;
    /* Dielectric walls (Sec. 2.1, Eq. (13)): diel[f] != 0 marks domain face
     * f (x-, x+, y-, y+, z-, z+) as dielectric.  sigma: device, the surface
     * charge (C/m^2) of the marked faces back to back in face order (x faces
     * ny*nz values at j + ny*k, y faces nx*nz at i + nx*k, z faces nx*ny at
     * i + nx*j), read and advanced in place: sigma / h_d of the corrector's
     * mid-point is added to the Poisson source of the adjacent cells, and
     * sigma = sigma^n + dt sum_s q_s Gamma_s . n_hat with the outward wall
     * fluxes of the corrector's mid-point state.  see_gamma (Sec. 2.2):
     * secondary electron emission coefficient of every wall face (the
     * electron wall flux less gamma times the ion wall fluxes of the face;
     * at most 8 species with the ion wall model).  stick: host [S] sticking
     * coefficients that multiply the neutral wall fluxes, NULL = 1. */
    int32_t diel[6];
    double *sigma;
    double see_gamma;
    const double *stick;
    /* Cell mask (Sec. 3, masking paragraph): device uint8 [cells], 1 valid,
     * 0 covered, NULL = every cell valid.  Every solve of the step is
     * masked (covered cells take no part and are Dirichlet faces for their
     * valid neighbours).  The potential stored in a covered cell is the
     * Dirichlet value of its faces with valid cells: it is lifted into the
     * Poisson right-hand side (2 beta_f g / h^2, beta_f the operator's face
     * coefficient) and kept; the field at such a face is the one-sided
     * difference over half a cell.  The densities take the homogeneous
     * Dirichlet value there (covered cells hold 0 after the step), and the
     * WENO5 drift stencils close the valid runs like Dirichlet domain faces
     * (positions past the closing face take minus the value mirrored
     * across it, 0 when the mirror leaves the run); the drift at a
     * covered-valid face uses the valid cell's mobility; the diffusive
     * electron flux of the Joule term is the homogeneous Dirichlet face
     * flux there; the adaptive step takes its limits over the valid cells.
     * Not with periodic faces, photoionization or dielectric faces
     * (VD_EINVAL). */
    const uint8_t *mask;
} vd_step_params;

/* State updated in place (device arrays). */
typedef struct {
    double *n;      /* [S][cells] */
    double *phi;    /* [cells]; in: guess, out: potential at the last corrector's u* */
    double *Te;     /* [cells], K; input in VD_TE_FIXED, output otherwise */
    double *Ee;     /* [cells], electron energy density (J/m^3); VD_TE_ENERGY only */
} vd_state;

typedef struct {
    int32_t poisson_cycles, species_cycles, energy_cycles, status;
    double poisson_rel, dt_used;
    double ms_poisson, ms_transport, ms_energy, ms_species, ms_total;
} vd_step_info;

/* One step of the segregated semi-implicit scheme (Sec. 3):
 *   for m = 0..n_t-1:  u* = (u^n + u^m)/2;  Poisson at u*;  E, E/N, Te,
 *   mobilities at u*;  [electron energy: (1/dt - div(5/3 D_e grad)) Ee^{m+1} =
 *   Ee^n/dt - div(5/3 mu_e Ee* E) + Joule - elastic - inelastic];  species:
 *   (1/dt - div(D_k grad)) n_k^{m+1} = n_k^n/dt - div(mu_k n*_k E) + G_k(u*)
 *   (+ extra_source);  u^{n+1} = u^{n_t}.
 * The species solves of each corrector go through one batched multigrid
 * solve.  No host copies happen inside the step besides the per-solve
 * convergence words.
 * poisson.guess = VD_GUESS_EXTRAP (not in the paper): the context keeps the
 * phi arrays passed in by its last two such calls (h1 the previous, h2 the
 * one before) for the same phi pointer, grid and dt; a change of any of
 * these restarts the history, and the phi of the first call after a restart
 * (the caller's initial guess rather than a step result) is not kept.  The
 * first corrector's Poisson solve then starts from 2 phi - h1 (one array
 * kept) or 3 phi - 3 h1 + h2 (two; each product and sum rounded on its
 * own, in that order) instead of phi, and still stops on the same residual
 * test, so the result differs from a VD_GUESS_GIVEN step only within the
 * solver tolerance.  The history holds the arrays as passed in: the phi a
 * step returns, unless the caller changed it between calls.  Costs two cell
 * arrays of device memory.
 * species_mg.guess = VD_GUESS_EXTRAP: the same for the transported species:
 * the context keeps n of the last two calls rounded to FP32 (for the same n
 * pointer, grid, S, dt and set of transported species; restarted and
 * skipped as above), and once the first corrector's right-hand sides are
 * built (they hold n^n), its species solves start from 2 n - h1 or
 * 3 n - 3 h1 + h2 (h widened to FP64; rounded as for phi) instead of n.
 * Costs S cell arrays of device memory.  energy_mg.guess must be GIVEN or
 * ZERO. */
vd_status vd_step(vd_ctx *ctx, const vd_step_params *params, const vd_state *state,
                  vd_step_info *info /* host, nullable */);

/* Forget the potentials and densities this context keeps for
 * VD_GUESS_EXTRAP: the next vd_step starts its histories afresh, as after
 * a change of array, grid or dt.  A caller that writes an unrelated state
 * into the arrays it passed before (or whose allocator may hand a freed
 * array's address to a new state) calls this first, or the next step would
 * extrapolate across two trajectories.  Enqueues nothing. */
vd_status vd_step_reset(vd_ctx *ctx);

/* ---- learned initial guess for the Poisson solve ----
 * Not in the paper: a small 3D U-Net (bfloat16 storage, FP32 accumulation
 * on the matrix cores) predicts phi from the charge density; the multigrid
 * solve of vd_poisson_solve then runs from that guess (opts.guess =
 * VD_GUESS_LEARNED) and still decides convergence.  Architecture: per level
 * l < levels two 3x3x3 convolutions with ReLU (c_l channels; level l+1 on
 * the 2x2x2 mean of level l); decoder per level l from levels-2 to 0: a
 * 3x3x3 convolution c_{l+1} -> c_l with ReLU at level l+1, nearest
 * upsampling, plus the encoder output of level l, a 3x3x3 convolution with
 * ReLU; a final 3x3x3 convolution c_0 -> 1.  Zero padding, biases.
 * Parameters: one FP32 vector, per convolution in that order (encoder a, b
 * per level; then up, dec from level levels-2 down to 0; then the output)
 * the weights [co][dz][dy][dx][ci] followed by the biases [co].
 * Tensors: [cell][channel], cells in the [nz][ny][nx] order, device. */
typedef struct {
    int32_t levels;     /* 1..4 */
    int32_t ch[4];      /* channels per level, 1..64 */
    int32_t cin;        /* input channels (2 for the warm start) */
} vd_nn_config;

/* parameter count of a configuration, -1 if it is invalid */
int64_t vd_nn_param_count(const vd_nn_config *cfg);

/* create (or replace) the context's network; params: host FP32
 * [param_count], NULL = zeros.  Adam moments start at zero. */
vd_status vd_nn_create(vd_ctx *ctx, const vd_nn_config *cfg, const float *params);

/* copy a host FP32 vector from (get) or into (set) the network: which = 0
 * parameters, 1 gradients of the last train step, 2 / 3 Adam first / second
 * moments */
vd_status vd_nn_get(vd_ctx *ctx, int32_t which, float *host);
vd_status vd_nn_set(vd_ctx *ctx, int32_t which, const float *host);

/* inference: in [cells][cin] bfloat16 bits, out [cells] FP32 (device);
 * every grid dimension divisible by 2^(levels-1) */
vd_status vd_nn_forward(vd_ctx *ctx, const vd_grid *grid, const uint16_t *in_bf16, float *out);

/* one training step on one sample: loss = mean((net(in) - target)^2),
 * gradients by backpropagation, then (update != 0) one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8) with learning rate lr.  loss: host, nullable. */
vd_status vd_nn_train_step(vd_ctx *ctx, const vd_grid *grid, const uint16_t *in_bf16, const float *target, float lr,
                           int32_t update, double *loss);

/* network input of the warm start for a potential problem: channel 0 =
 * rho Lx^2 / (eps V), channel 1 = (linear ramp between the Dirichlet values
 * of the two x faces, 0 unless both are Dirichlet) / V, with V the largest
 * |Dirichlet value| of phi_bc (1 if none); out [cells][2] bfloat16 (device);
 * vref (host, nullable) receives V.  The guess is phi = V * net output. */
vd_status vd_nn_features(vd_ctx *ctx, const vd_grid *grid, const vd_bc *phi_bc, const double *rho, double eps,
                         uint16_t *out_bf16, double *vref);

/* network file: 8-byte tag, vd_nn_config, int64 parameter count, FP32
 * parameters; load creates the network */
vd_status vd_nn_save(vd_ctx *ctx, const char *path);
vd_status vd_nn_load(vd_ctx *ctx, const char *path);

/* one 3x3x3 convolution (zero padding) and, if dy is given, its gradients:
 * x [cells][ci] bfloat16 bits, w [co][27][ci] and b [co] FP32 (the weights
 * are rounded to bfloat16, accumulation FP32), y [cells][co] FP32 (nullable;
 * ReLU if relu), dy [cells][co] FP32 -> dx [cells][ci], dw [co][27][ci],
 * db [co] FP32.  All device pointers; synchronises. */
vd_status vd_nn_conv3d(vd_ctx *ctx, const vd_grid *grid, const uint16_t *x_bf16, int32_t ci, const float *w, const float *b,
                       int32_t co, int32_t relu, float *y, const float *dy, float *dx, float *dw, float *db);

/* ---- inspection entry points (tests and tuning) ---- */

/* Per-cell flags of multigrid level `level` of a problem: bit 0 colour
 * (i+j+k)&1, bit 1 valid (a coarse cell is valid iff its 8 children are),
 * bit 2+f face f does not couple to a valid neighbour.  out: device uint8
 * cells of that level. */
vd_status vd_cell_flags(vd_ctx *ctx, const vd_problem *prob, int32_t n_levels, int32_t level, uint8_t *out);

/* ncolour Gauss-Seidel half-sweeps (red first) on the finest level of one
 * problem, with the Dirichlet lifting; x updated in place. */
vd_status vd_smooth(vd_ctx *ctx, const vd_problem *prob, int32_t ncolour);

/* Host-side check of the memory accesses of the 2.5D tiled passes (no GPU
 * call): for a level of nx x ny x nz cells (periodic: bit d set when
 * direction d wraps) and tiles of kz planes, walks every load and store
 * that every thread of every tile issues in the lexicographic colour /
 * residual pass in all its modes (kernel 0: x and b pairs with their look-
 * ahead planes, halo elements, FP64 unknown pairs of the fused last colour
 * pass, FP32 residual stores in both row layouts, LDS slots) or in the
 * parity-split FP32 colour pass (kernel 1, both colours: other-colour
 * pairs, halo, b, the four FP64 cells of the fused last pass, stores) or in
 * the direct residual check of levels with coefficient arrays (kernel 2: x
 * window and x-y neighbours, b, the three face arrays, the cell
 * coefficient, FP32 residual stores in both row layouts), with the kernels'
 * own index functions, and counts the accesses (accesses) and those outside
 * the level's arrays or the LDS tile, or misaligned for a vector access
 * (violations; also 1 if the workgroup-to-tile mapping does not take every
 * tile once).  VD_EINVAL for nx odd (kernels 0 and 2) or not a multiple of
 * 4 (kernel 1), another kernel number, kz < 1, or null outputs. */
vd_status vd_check_tiles25(int32_t nx, int32_t ny, int32_t nz, int32_t periodic, int32_t kz, int32_t kernel,
                           int64_t *accesses, int64_t *violations);

/* Kernel timing: bracket every launch of the selected kernel families
 * (comma-separated, e.g. "gsrb,weno,coarse"; NULL or "" turns timing off)
 * with HIP events on the context stream, and read back per family the
 * launch count, the summed device milliseconds and the summed algorithmic
 * bytes of those launches (the bytes a launch must move at minimum: its
 * inputs read once and its outputs written once).  Selecting resets the
 * accumulators. */
vd_status vd_timing_select(vd_ctx *ctx, const char *kernels);
vd_status vd_timing_read(vd_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* VD_H */
