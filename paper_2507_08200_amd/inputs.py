"""Seeded synthetic workloads shared by the GPU path and the FP64 oracle.

This module only draws random numbers and lays out initial states, boundary
descriptors and time-step parameters.  It contains none of the method's
arithmetic (no operator, flux, rate or solver code), so both the HIP library
and the oracle can consume its arrays without sharing any numerical code.

Workloads (all SI units unless stated):

* ``cfg1``: 32^3 cube of 1 cm, three species (e, Ar+, Ar*) over a background
  of Ar at 1 atm / 300 K; Gaussian blob (peak 1e17 m^-3, sigma 2 mm) at the
  centre on a 1e13 m^-3 background with 1 % seeded uniform noise; Te = 2 eV
  fixed; phi = 1 kV at x = 0 and 0 at x = L, Neumann elsewhere; dt = 1e-12 s.
* ``cfg3``: 160^3 cube of 12.5 mm, 15-species Ar-H2 (95/5 by volume at
  101325 Pa, 300 K); electron/Ar+ Gaussian seed (peak 1e19 m^-3, sigma
  0.5 mm) centred 1 mm from the x = 0 electrode at 15 kV; background 1e13
  m^-3 with 1 % noise; Te from the reduced-field table; dt = 1e-12 s.
* ``cfg2``: manufactured solution on the unit cube (the method of Sec. 5.1 in
  3D): 8 species with signed constant mobilities and constant diffusion, a
  charge pair that sustains an analytic potential, nondimensional constants;
  the exact source that makes the analytic fields steady is passed to the
  step as its extra species source.
* ``cfg4``: 64 independent Helmholtz problems of uneven size (edges drawn
  from {32, 48, ..., 160}), log-uniform beta with a sheath-like slab jump,
  random Dirichlet/Neumann faces, N(0,1) right-hand sides.
* Random small Helmholtz / Poisson problems and the manufactured-solution
  fields used by the tests.

The electron temperature table used in local-field mode is a stand-in for
the Boltzmann-solver output the paper uses (Sec. 2.3 and the streamer
benchmark in Sec. 5.4): Te[eV] = 0.02585 + 5.47 (E/N / 300 Td)^0.6, sampled on
256 log-spaced points between 1e-2 and 1e3 Td.  Only its shape (about 5.5 eV
at 300 Td, the pairing the paper reports at 3D streamer heads in Sec. 6.1)
is taken from the paper.
"""
from __future__ import annotations

import numpy as np

# Boundary kinds, per domain face in the order x-, x+, y-, y+, z-, z+.
BC_DIRICHLET, BC_NEUMANN, BC_WALLFLUX, BC_PERIODIC = 0, 1, 2, 3

# Electron-temperature modes of the time step.
TE_FIXED, TE_LFA, TE_ENERGY = 0, 1, 2

# Mechanism identifiers.
MECH_NONE, MECH_DECAY, MECH_AR3, MECH_ARH2_15 = 0, 1, 2, 3

# Unit-conversion and gas-state constants used to *describe* the inputs.
EV_IN_K = 11604.518
ATM = 101325.0
KB = 1.380649e-23
N_1ATM_300K = ATM / (KB * 300.0)          # 2.4463e25 m^-3

LFA_NPTS = 256
LFA_EN_MIN_TD = 1e-2
LFA_EN_MAX_TD = 1e3


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 generator; every workload names its own seed."""
    return np.random.default_rng(seed)


def lfa_table() -> dict:
    """Stand-in Te(E/N) table (K) on log-spaced reduced fields (Td)."""
    ln_en = np.linspace(np.log(LFA_EN_MIN_TD), np.log(LFA_EN_MAX_TD), LFA_NPTS)
    en = np.exp(ln_en)
    te_ev = 0.02585 + 5.47 * (en / 300.0) ** 0.6
    return {
        "te_K": np.ascontiguousarray(te_ev * EV_IN_K, dtype=np.float64),
        "ln_en_min": float(ln_en[0]),
        "ln_en_max": float(ln_en[-1]),
        "npts": LFA_NPTS,
    }


def bc(kinds, values=(0.0,) * 6) -> dict:
    return {"kind": [int(k) for k in kinds], "value": [float(v) for v in values]}


def cell_centres(nx, ny, nz, dx, dy, dz):
    """Cell-centre coordinates, each array shaped [nz][ny][nx]."""
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    z = (np.arange(nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _blob(X, Y, Z, c, sigma):
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


def cfg1(seed: int = 1, n: int = 32) -> dict:
    """Three-species argon step on an n^3 grid over a 1 cm cube."""
    L = 0.01
    h = L / n
    g = rng(seed)
    X, Y, Z = cell_centres(n, n, n, h, h, h)
    shape = _blob(X, Y, Z, (L / 2, L / 2, L / 2), 2e-3)
    base = 1e13 + 1e17 * shape
    S = 3
    dens = np.empty((S, n, n, n))
    dens[0] = base * (1.0 + 0.01 * g.uniform(-1, 1, base.shape))   # e
    dens[1] = base * (1.0 + 0.01 * g.uniform(-1, 1, base.shape))   # Ar+
    dens[2] = 1e13 * (1.0 + 0.01 * g.uniform(-1, 1, base.shape))   # Ar*
    te = np.full((n, n, n), 2.0 * EV_IN_K)
    wall = [BC_WALLFLUX, BC_WALLFLUX, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN]
    return {
        "name": "cfg1-ar3-%d" % n,
        "grid": (n, n, n, h, h, h),
        "mech": MECH_AR3,
        "n": dens,
        "phi": np.zeros((n, n, n)),
        "Te": te,
        "te_mode": TE_FIXED,
        "phi_bc": bc([BC_DIRICHLET, BC_DIRICHLET] + [BC_NEUMANN] * 4, [1000.0, 0, 0, 0, 0, 0]),
        "species_bc": [bc(wall)] * S,
        "energy_bc": bc(wall),
        "dt": 1e-12,
        "n_t": 1,
        "Tg": 300.0,
        "N_gas": N_1ATM_300K,
        "bg": [N_1ATM_300K],
        # Constant electron mobility 0.03 m^2/Vs with Einstein diffusion at
        # 2 eV: D = mu * (kB Te / e) = 0.03 * 2 V.
        "electron_const": (-0.03, 0.06),
    }


def cfg3(seed: int = 3, n: int = 160, L: float = 0.0125, voltage: float = 15e3,
         seed_centre=None, ny: int = 0, nz: int = 0) -> dict:
    """15-species Ar-H2 streamer-shaped state on an n^3 grid (n x ny x nz
    cells of edge L/n when ny, nz are given; the seed sits 1 mm from the
    x = 0 electrode on the transverse axis)."""
    h = L / n
    ny = ny or n
    nz = nz or n
    g = rng(seed)
    X, Y, Z = cell_centres(n, ny, nz, h, h, h)
    c = seed_centre if seed_centre is not None else (1.0e-3, ny * h / 2, nz * h / 2)
    shape = _blob(X, Y, Z, c, 0.5e-3)
    base = 1e13 + 1e19 * shape
    S = 15
    N = N_1ATM_300K
    dens = np.zeros((S, nz, ny, n))
    dens[0] = base * (1.0 + 0.01 * g.uniform(-1, 1, base.shape))    # e
    dens[1] = base * (1.0 + 0.01 * g.uniform(-1, 1, base.shape))    # Ar+
    dens[13] = 0.95 * N                                               # Ar
    dens[14] = 0.05 * N                                               # H2
    wall = [BC_WALLFLUX, BC_WALLFLUX, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN]
    return {
        "name": "cfg3-arh2-%d" % n if ny == n and nz == n else "cfg3-arh2-%dx%dx%d" % (n, ny, nz),
        "grid": (n, ny, nz, h, h, h),
        "mech": MECH_ARH2_15,
        "n": dens,
        "phi": np.zeros((nz, ny, n)),
        "Te": np.full((nz, ny, n), 300.0),
        "te_mode": TE_LFA,
        "phi_bc": bc([BC_DIRICHLET, BC_DIRICHLET] + [BC_NEUMANN] * 4, [voltage, 0, 0, 0, 0, 0]),
        "species_bc": [bc(wall)] * S,
        "energy_bc": bc(wall),
        "dt": 1e-12,
        "n_t": 1,
        "Tg": 300.0,
        "N_gas": N,
        "bg": [],
        "lfa": lfa_table(),
    }


UNIT_CONSTS = {"qe": 1.0, "eps0": 1.0, "kB": 1.0, "me": 1.0}


def cfg2(seed: int = 2, n: int = 128, S: int = 8, levels: int = 4) -> dict:
    """Manufactured steady solution on the unit cube with n^3 cells.

    With s(x) = sin 2 pi x sin 2 pi y sin 2 pi z the species densities are
    n_k = a_k (1 + c_k s / 2) (a_k ~ U[1, 2], c_k ~ U[0.5, 1]), the
    potential phi = B s and Te = 1 + s / 10; species 0 and 1 carry charge
    +1 and -1 with a_0 = a_1, the others none, so that with e = eps0 = 1
    Poisson's equation -lap phi = sum_k Z_k n_k holds exactly for
    B = a_0 (c_0 - c_1) / (24 pi^2) (lap s = -12 pi^2 s).  Mobilities are
    signed constants, |mu_k| ~ U[0.1, 1] with a random sign, D_k ~
    U[0.05, 0.5].  x faces are Dirichlet with the exact values (s = 0 there:
    phi = 0, n_k = a_k), y and z periodic.  The exact source is the
    continuous drift-diffusion divergence of the analytic fields,
    div(mu_k n_k E) - D_k lap n_k with E = -grad phi (Eqs. (1)-(2); no
    chemistry), evaluated in closed form at the cell centres, so that the
    analytic fields are a steady solution of the continuous problem.
    Returned "exact" holds the analytic n and phi at the cell centres."""
    g = rng(seed)
    h = 1.0 / n
    X, Y, Z = cell_centres(n, n, n, h, h, h)
    tp = 2.0 * np.pi
    sx, sy, sz = np.sin(tp * X), np.sin(tp * Y), np.sin(tp * Z)
    cx, cy, cz = np.cos(tp * X), np.cos(tp * Y), np.cos(tp * Z)
    s = sx * sy * sz
    grad_s = (tp * cx * sy * sz, tp * sx * cy * sz, tp * sx * sy * cz)
    grad_s2 = grad_s[0] ** 2 + grad_s[1] ** 2 + grad_s[2] ** 2
    lap_s = -3.0 * tp * tp * s
    a = g.uniform(1.0, 2.0, S)
    a[1] = a[0]
    c = g.uniform(0.5, 1.0, S)
    mu = g.uniform(0.1, 1.0, S) * np.where(g.uniform(0, 1, S) < 0.5, -1.0, 1.0)
    D = g.uniform(0.05, 0.5, S)
    Zc = np.zeros(S)
    Zc[0], Zc[1] = 1.0, -1.0
    B = a[0] * (c[0] - c[1]) / (24.0 * np.pi ** 2)
    phi = B * s
    dens = np.empty((S, n, n, n))
    src = np.empty((S, n, n, n))
    for k in range(S):
        dens[k] = a[k] * (1.0 + 0.5 * c[k] * s)
        # grad n . E = -(a c / 2) B |grad s|^2 ;  div E = -B lap s
        gradn_dot_E = -0.5 * a[k] * c[k] * B * grad_s2
        div_E = -B * lap_s
        lap_n = 0.5 * a[k] * c[k] * lap_s
        src[k] = mu[k] * (gradn_dot_E + dens[k] * div_E) - D[k] * lap_n
    species = [{"Z": float(Zc[k]), "mass": 1.0, "mob_kind": 0, "wall_kind": 0, "mu_const": float(mu[k]),
                "D_const": float(D[k]), "transported": 1} for k in range(S)]
    sbc = [bc([BC_DIRICHLET, BC_DIRICHLET, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC],
              [a[k], a[k], 0, 0, 0, 0]) for k in range(S)]
    per_x_dir = [BC_DIRICHLET, BC_DIRICHLET, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC]
    return {
        "name": "cfg2-mms-%d" % n,
        "grid": (n, n, n, h, h, h),
        "mech": MECH_NONE,
        "n": dens.copy(),
        "phi": phi.copy(),
        "Te": 1.0 + 0.1 * s,
        "te_mode": TE_FIXED,
        "phi_bc": bc(per_x_dir),
        "species_bc": sbc,
        "energy_bc": bc(per_x_dir),
        "dt": 0.05,
        "n_t": 1,
        "Tg": 1.0,
        "N_gas": 1.0,
        "bg": [],
        "levels": levels,
        "species": species,
        "extra_source": src,
        "exact": {"n": dens, "phi": phi},
    }


def random_helmholtz(seed: int, shape, *, alpha_kind="array", beta_kind="array",
                     kinds=None, mask_holes=0, beta_jump=False, h=None) -> dict:
    """A random (alpha - div beta grad) x = b problem for solver tests.

    shape = (nx, ny, nz).  alpha_kind / beta_kind in {"array", "const",
    "zero" (alpha only)}.  kinds: six boundary kinds (random if None).
    mask_holes: number of covered boxes cut into the mask.
    """
    g = rng(seed)
    nx, ny, nz = shape
    if h is None:
        h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    if kinds is None:
        kinds = []
        for d in range(3):
            if g.uniform() < 0.2:
                kinds += [BC_PERIODIC, BC_PERIODIC]
            else:
                kinds += [int(g.choice([BC_DIRICHLET, BC_NEUMANN])) for _ in range(2)]
        if BC_DIRICHLET not in kinds:
            kinds[0] = BC_DIRICHLET
    values = g.uniform(-1, 1, 6)
    prob = {"grid": (nx, ny, nz) + tuple(h), "bc": bc(kinds, values)}
    if alpha_kind == "array":
        prob["alpha"], prob["alpha_c"] = g.uniform(0.5, 2.0, (nz, ny, nx)), 0.0
    elif alpha_kind == "const":
        prob["alpha"], prob["alpha_c"] = None, float(g.uniform(0.5, 2.0))
    else:
        prob["alpha"], prob["alpha_c"] = None, 0.0
    if beta_kind == "array":
        beta = np.exp(g.uniform(np.log(1e-3), 0.0, (nz, ny, nx)))
        if beta_jump:
            beta = np.full((nz, ny, nx), np.exp(g.uniform(np.log(1e-3), 0.0)))
            w = int(g.integers(2, 7))
            beta[:, :, :w] = np.exp(g.uniform(np.log(1e-3), 0.0))
        prob["beta"], prob["beta_c"] = beta, 0.0
    else:
        prob["beta"], prob["beta_c"] = None, float(np.exp(g.uniform(np.log(1e-3), 0.0)))
    mask = None
    if mask_holes:
        mask = np.ones((nz, ny, nx), dtype=np.uint8)
        for _ in range(mask_holes):
            lo = [int(g.integers(0, s - 1)) for s in (nz, ny, nx)]
            ext = [int(g.integers(1, max(2, s // 3))) for s in (nz, ny, nx)]
            mask[lo[0]:lo[0] + ext[0], lo[1]:lo[1] + ext[1], lo[2]:lo[2] + ext[2]] = 0
    prob["mask"] = mask
    prob["rhs"] = g.standard_normal((nz, ny, nx))
    prob["x0"] = g.standard_normal((nz, ny, nx))
    return prob


def cfg4(seed: int = 4, count: int = 64, sizes=tuple(range(32, 161, 16))) -> list:
    """64 uneven Helmholtz problems with a sheath-like beta jump each."""
    g = rng(seed)
    probs = []
    for p in range(count):
        n = int(g.choice(sizes))
        h = 1.0 / n
        kinds = [int(g.choice([BC_DIRICHLET, BC_NEUMANN])) for _ in range(6)]
        values = g.uniform(-1, 1, 6)
        bulk = np.exp(g.uniform(np.log(1e-3), 0.0))
        sheath = np.exp(g.uniform(np.log(1e-3), 0.0))
        width = int(g.integers(2, 7))
        face = int(g.integers(0, 6))
        beta = np.full((n, n, n), bulk)
        axis, side = 2 - face // 2, face % 2
        sl = [slice(None)] * 3
        sl[axis] = slice(0, width) if side == 0 else slice(n - width, n)
        beta[tuple(sl)] = sheath
        probs.append({
            "grid": (n, n, n, h, h, h),
            "bc": bc(kinds, values),
            "alpha": None, "alpha_c": 1.0,
            "beta": beta, "beta_c": 0.0,
            "mask": None,
            "rhs": g.standard_normal((n, n, n)),
            "x0": np.zeros((n, n, n)),
        })
    return probs


# ------------------------------------------------ warm-start network inputs
NN_CFG = {"levels": 4, "ch": [16, 32, 64, 64], "cin": 2}


def nn_init(seed: int, cfg: dict = NN_CFG) -> np.ndarray:
    """Seeded initial parameters of the warm-start U-Net as one FP32 vector:
    per convolution (encoder a/b per level, then up/dec from the second
    coarsest level to the finest, then the 1-channel output) He-normal
    weights of shape (co, 3, 3, 3, ci) followed by zero biases."""
    g = rng(seed)
    L, ch, cin = cfg["levels"], list(cfg["ch"]), cfg.get("cin", 2)
    shapes = []
    for l in range(L):
        shapes += [(cin if l == 0 else ch[l - 1], ch[l]), (ch[l], ch[l])]
    for l in range(L - 2, -1, -1):
        shapes += [(ch[l + 1], ch[l]), (ch[l], ch[l])]
    shapes.append((ch[0], 1))
    out = []
    for ci, co in shapes:
        out.append(g.standard_normal(co * 27 * ci) * np.sqrt(2.0 / (27 * ci)))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def warmstart_runs(seed: int, count: int, L: float = 0.0125) -> list:
    """Seeded variations of the streamer state for the warm-start data:
    electrode voltage U[5, 20] kV, seed centre x in U[0.5, 2] mm and y, z
    within 2 mm of the axis, and a noise seed per run."""
    g = rng(seed)
    out = []
    for r in range(count):
        V = float(g.uniform(5e3, 20e3))
        c = (float(g.uniform(0.5e-3, 2.0e-3)), float(L / 2 + g.uniform(-2e-3, 2e-3)),
             float(L / 2 + g.uniform(-2e-3, 2e-3)))
        out.append({"voltage": V, "centre": c, "seed": int(g.integers(1, 2 ** 31 - 1))})
    return out
