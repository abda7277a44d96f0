"""ctypes wrapper of the FP64 CPU oracle (vd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  It holds
no numerical method code itself: every function marshals numpy arrays into
the C oracle and back.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# timing build for the all-cores CPU baseline: the same source with OpenMP
# on its independent per-cell loops (sums stay sequential: same results)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, EINVAL, ENOMEM, ENOCONV, ESINGULAR = 0, -1, -2, -4, -5
MOB_CONST, MOB_ELECTRON_FIT, MOB_ION_N0, MOB_NEUTRAL_N0 = 0, 1, 2, 3
WALL_NONE, WALL_ELECTRON, WALL_ION, WALL_NEUTRAL = 0, 1, 2, 3


def build(force: bool = False, parallel: bool = False) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction);
    parallel=True builds the OpenMP timing variant."""
    out = _LIB_OMP if parallel else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall"] +
                              (["-fopenmp"] if parallel else []) + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 6), ("value", C.c_double * 6)]


class Problem(C.Structure):
    _fields_ = [("grid", Grid), ("bc", BC), ("mask", C.c_void_p),
                ("alpha", C.c_void_p), ("alpha_c", C.c_double),
                ("beta", C.c_void_p), ("beta_c", C.c_double)]


class MGOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_cycles", C.c_int32), ("fixed_cycles", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("n_levels", C.c_int32)]


class MGInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("levels", C.c_int32), ("status", C.c_int32),
                ("bottom_iters", C.c_int32), ("rel_res", C.c_double), ("rel_res0", C.c_double),
                ("bnorm", C.c_double)]


class Species(C.Structure):
    _fields_ = [("Z", C.c_double), ("mass", C.c_double), ("transported", C.c_int32),
                ("mob_kind", C.c_int32), ("wall_kind", C.c_int32), ("pad", C.c_int32),
                ("mob_coef", C.c_double), ("mu_const", C.c_double), ("D_const", C.c_double)]


class Consts(C.Structure):
    _fields_ = [("qe", C.c_double), ("eps0", C.c_double), ("kB", C.c_double), ("me", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("grid", Grid), ("dt", C.c_double),
                ("n_t", C.c_int32), ("mech", C.c_int32), ("S", C.c_int32), ("te_mode", C.c_int32),
                ("electron", C.c_int32), ("dt_mode", C.c_int32),
                ("Tg", C.c_double), ("N_gas", C.c_double), ("m_bg", C.c_double), ("k_decay", C.c_double),
                ("bg", C.c_double * 4),
                ("c_adv", C.c_double), ("c_diff", C.c_double), ("c_diel", C.c_double), ("pad0", C.c_double),
                ("c", Consts), ("phi_bc", BC), ("energy_bc", BC),
                ("species_bc", C.c_void_p), ("species", C.c_void_p),
                ("lfa_te", C.c_void_p), ("lfa_ln_min", C.c_double), ("lfa_ln_max", C.c_double),
                ("lfa_n", C.c_int32), ("pad1", C.c_int32),
                ("extra_source", C.c_void_p), ("extra_energy", C.c_void_p), ("eps_cell", C.c_void_p),
                ("poisson", MGOpts), ("species_mg", MGOpts), ("energy_mg", MGOpts),
                ("species_guess", C.c_void_p), ("phi_fixed", C.c_int32), ("pad2", C.c_int32),
                ("check_n", C.c_void_p), ("check_Ee", C.c_void_p), ("check_res", C.c_void_p),
                ("photo_n", C.c_int32), ("photo_e", C.c_int32), ("photo_ion", C.c_int32), ("pad3", C.c_int32),
                ("photo_A", C.c_double * 3), ("photo_lambda", C.c_double * 3),
                ("photo_pO2", C.c_double), ("photo_pg", C.c_double), ("photo_xi", C.c_double),
                ("photo_pq", C.c_double), ("photo_p", C.c_double), ("photo_nu_ratio", C.c_double),
                ("photo_bc", BC), ("photo_mg", MGOpts), ("photo_out", C.c_void_p),
                ("diel", C.c_int32 * 6), ("sigma", C.c_void_p), ("see_gamma", C.c_double), ("stick", C.c_void_p),
                ("mask", C.c_void_p)]


class StepInfo(C.Structure):
    _fields_ = [("poisson_cycles", C.c_int32), ("species_cycles", C.c_int32),
                ("energy_cycles", C.c_int32), ("status", C.c_int32),
                ("poisson_rel", C.c_double), ("dt_used", C.c_double)]


_libs = {}


def lib(parallel: bool = False):
    """The oracle library (parallel: the OpenMP timing build, whose threads
    follow OMP_NUM_THREADS)."""
    _lib = _libs.get(parallel)
    if _lib is None:
        _lib = C.CDLL(build(parallel=parallel))
        _libs[parallel] = _lib
        d = C.c_double
        P = C.c_void_p
        _lib.or_mu_electron.restype = d
        _lib.or_mu_electron.argtypes = [d, d]
        _lib.or_te_lfa.restype = d
        _lib.or_te_lfa.argtypes = [P, C.c_int, d, d, d]
        _lib.or_weno5.restype = d
        _lib.or_weno5.argtypes = [P]
        _lib.or_rates_arh2.restype = None
        _lib.or_rates_arh2.argtypes = [d, P]
        _lib.or_reaction_source.argtypes = [C.c_int, C.c_size_t, C.c_int, P, P, P, d, d, P, P]
        _lib.or_species_flux.argtypes = [P, P, P, C.c_int, P, P, P, P, P, d, P, P]
        _lib.or_efield.argtypes = [P, P, P, P, P, P, P]
        _lib.or_mg_solve.argtypes = [P, P, P, P, P]
        _lib.or_apply_op.argtypes = [P, P, P]
        _lib.or_residual.argtypes = [P, P, P, P]
        _lib.or_smooth.argtypes = [P, P, P, C.c_int]
        _lib.or_cell_flags.argtypes = [P, C.c_int, C.c_int, P]
        _lib.or_arh2_stoich.argtypes = [C.c_int, P]
        _lib.or_step.argtypes = [P, P, P, P, P, P]
        _lib.or_face_flux.argtypes = [P, P, P, P, P, P, P, P, P, d, P, P, P, P]
        _lib.or_transport.argtypes = [P, P, d, d, d, d, P, P]
        _lib.or_transport.restype = None
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def grid(g):
    nx, ny, nz, dx, dy, dz = g
    return Grid(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz))


def bc(b):
    out = BC()
    for f in range(6):
        out.kind[f] = int(b["kind"][f])
        out.value[f] = float(b["value"][f])
    return out


def mg_opts(rtol=1e-10, max_cycles=100, fixed_cycles=0, nu_pre=2, nu_post=2, n_levels=0):
    return MGOpts(float(rtol), int(max_cycles), int(fixed_cycles), int(nu_pre), int(nu_post), int(n_levels))


def _problem(prob, keep):
    mask = prob.get("mask")
    alpha = prob.get("alpha")
    beta = prob.get("beta")
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
    if alpha is not None:
        alpha = _f64(alpha)
    if beta is not None:
        beta = _f64(beta)
    keep += [mask, alpha, beta]
    return Problem(grid(prob["grid"]), bc(prob["bc"]), _ptr(mask), _ptr(alpha),
                   float(prob.get("alpha_c", 0.0)), _ptr(beta), float(prob.get("beta_c", 0.0)))


def mg_solve(prob, rhs, x0, parallel=False, **opts):
    """(alpha - div beta grad) x = rhs; returns (x, info dict, status)."""
    keep = []
    P = _problem(prob, keep)
    x = _f64(x0).copy()
    r = _f64(rhs)
    o = mg_opts(**opts)
    info = MGInfo()
    st = lib(parallel).or_mg_solve(C.byref(P), _ptr(r), _ptr(x), C.byref(o), C.byref(info))
    d = {k: getattr(info, k) for k, _ in MGInfo._fields_}
    return x, d, st


def apply_op(prob, x):
    keep = []
    P = _problem(prob, keep)
    x = _f64(x)
    y = np.empty_like(x)
    st = lib().or_apply_op(C.byref(P), _ptr(x), _ptr(y))
    assert st == OK
    return y


def residual(prob, rhs, x):
    keep = []
    P = _problem(prob, keep)
    x = _f64(x)
    rhs = _f64(rhs)
    r = np.empty_like(x)
    st = lib().or_residual(C.byref(P), _ptr(rhs), _ptr(x), _ptr(r))
    assert st == OK
    return r


def smooth(prob, rhs, x0, ncolour):
    keep = []
    P = _problem(prob, keep)
    x = _f64(x0).copy()
    rhs = _f64(rhs)
    st = lib().or_smooth(C.byref(P), _ptr(rhs), _ptr(x), int(ncolour))
    assert st == OK
    return x


def cell_flags(prob, level, n_levels=0):
    keep = []
    P = _problem(prob, keep)
    nx, ny, nz = prob["grid"][:3]
    out = np.zeros(((nz >> level), (ny >> level), (nx >> level)), dtype=np.uint8)
    st = lib().or_cell_flags(C.byref(P), int(n_levels), int(level), _ptr(out))
    assert st == OK, st
    return out


def efield(g, phi_bc, phi):
    nx, ny, nz = g[:3]
    phi = _f64(phi)
    ex = np.empty((nz, ny, nx + 1))
    ey = np.empty((nz, ny + 1, nx))
    ez = np.empty((nz + 1, ny, nx))
    ec = np.empty((nz, ny, nx, 3))
    G, B = grid(g), bc(phi_bc)
    lib().or_efield(C.byref(G), C.byref(B), _ptr(phi), _ptr(ex), _ptr(ey), _ptr(ez), _ptr(ec))
    return ex, ey, ez, ec


def weno5(v):
    v = _f64(v)
    assert v.shape == (5,)
    return lib().or_weno5(_ptr(v))


def rates_arh2(te_K):
    k = np.empty(33)
    lib().or_rates_arh2(float(te_K), _ptr(k))
    return k


def mu_electron(en_td, N):
    return lib().or_mu_electron(float(en_td), float(N))


def te_lfa(table, en_td):
    t = _f64(table["te_K"])
    return lib().or_te_lfa(_ptr(t), int(table["npts"]), float(table["ln_en_min"]),
                           float(table["ln_en_max"]), float(en_td))


def stoich(q):
    out = np.zeros(15, dtype=np.int32)
    lib().or_arh2_stoich(int(q), _ptr(out))
    return out


def reaction_source(mech, n, Te, bg=(), k_decay=0.0, qe=1.602176634e-19):
    n = _f64(n)
    S = n.shape[0]
    nc = n[0].size
    Te = _f64(Te)
    bga = _f64(list(bg) + [0.0] * (4 - len(bg)))
    G = np.empty_like(n)
    Sin = np.empty(Te.shape)
    st = lib().or_reaction_source(int(mech), nc, S, _ptr(n), _ptr(Te), _ptr(bga), float(k_decay),
                                  float(qe), _ptr(G), _ptr(Sin))
    assert st == OK, st
    return G, Sin


def species_array(species):
    arr = (Species * len(species))()
    for s, sp in enumerate(species):
        arr[s] = Species(float(sp["Z"]), float(sp["mass"]), int(sp.get("transported", 1)),
                         int(sp["mob_kind"]), int(sp["wall_kind"]), 0, float(sp.get("mob_coef", 0.0)),
                         float(sp.get("mu_const", 0.0)), float(sp.get("D_const", 0.0)))
    return arr


PHYS = {"qe": 1.602176634e-19, "eps0": 8.8541878128e-12, "kB": 1.380649e-23, "me": 9.1093837015e-31}


def transport(sp, en_td, Te, Tg, N, consts=PHYS):
    """(signed mobility, diffusion) of one species dict at E/N (Td), Te, Tg (K), N."""
    arr = species_array([sp])
    cs = Consts(**consts)
    mu, D = C.c_double(), C.c_double()
    lib().or_transport(arr, C.byref(cs), float(en_td), float(Te), float(Tg), float(N), C.byref(mu), C.byref(D))
    return mu.value, D.value


def species_flux(g, phi_bc, sp_bcs, species, n, phi, mu, Te, Tg, consts=PHYS):
    n = _f64(n)
    S = n.shape[0]
    G, PB = grid(g), bc(phi_bc)
    SB = (BC * S)(*[bc(b) for b in sp_bcs])
    SP = species_array(species)
    cs = Consts(**consts)
    phi, mu, Te = _f64(phi), _f64(mu), _f64(Te)
    div = np.empty_like(n)
    st = lib().or_species_flux(C.byref(G), C.byref(PB), SB, S, SP, _ptr(n), _ptr(phi), _ptr(mu),
                               _ptr(Te), float(Tg), C.byref(cs), _ptr(div))
    assert st == OK
    return div


def face_flux(g, phi_bc, sp_bc, sp, u, phi, mu, D, Te, Tg, consts=PHYS):
    """Total face flux (drift + diffusion) of one species: (fx, fy, fz)
    shaped (nz, ny, nx+1), (nz, ny+1, nx), (nz+1, ny, nx)."""
    nx, ny, nz = g[:3]
    G, PB, UB = grid(g), bc(phi_bc), bc(sp_bc)
    SP = species_array([sp])
    cs = Consts(**consts)
    u, phi, mu, D, Te = _f64(u), _f64(phi), _f64(mu), _f64(D), _f64(Te)
    fx = np.empty((nz, ny, nx + 1))
    fy = np.empty((nz, ny + 1, nx))
    fz = np.empty((nz + 1, ny, nx))
    st = lib().or_face_flux(C.byref(G), C.byref(PB), C.byref(UB), SP, _ptr(u), _ptr(phi), _ptr(mu), _ptr(D),
                            _ptr(Te), float(Tg), C.byref(cs), _ptr(fx), _ptr(fy), _ptr(fz))
    assert st == OK
    return fx, fy, fz


def step(cfg, species, *, n=None, phi=None, Te=None, Ee=None, consts=PHYS, poisson=None, species_mg=None,
         energy_mg=None, extra_source=None, extra_energy=None, eps_cell=None, electron=0, m_bg=0.0,
         k_decay=0.0, species_guess=None, phi_fixed=False, check_n=None, check_Ee=None, parallel=False,
         photo=None, adaptive_dt=None, diel=None, sigma=None, see_gamma=0.0, stick=None, mask=None):
    """One step of the semi-implicit scheme on a workload dict (see inputs).
    species_guess ([S][cells], optional): starting iterate of the first
    corrector's species solves in place of n^n.
    photo (optional dict): photoionization terms -- "A", "lam" (lists of up
    to 3), "pO2", "pg", "xi", "pq", "p", "nu_ratio" (default 1), "e", "ion"
    (species indices), "bc" (boundary dict, default homogeneous Dirichlet),
    "mg" (solver options); the S_j of the last corrector come back as
    "photo_S" ([3][cells]).  adaptive_dt (optional dict "c_adv", "c_diff",
    "c_diel"): time step of Eq. (20) with cfg["dt"] as its largest value
    (the electron species index is `electron`).  diel (six flags) with
    sigma (packed surface charge of the marked faces, see the C header):
    dielectric faces, sigma advanced and returned as "sigma".  see_gamma:
    secondary emission coefficient; stick ([S]): sticking coefficients.
    mask ([cells] uint8, 1 valid / 0 covered): a masked step (the covered
    cells' potentials are Dirichlet values of the Poisson solve, see the C
    header).
    Checking a step computed elsewhere (n_t = 1): phi_fixed takes phi as the
    Poisson result (its relative residual in info["poisson_rel"]); check_n /
    check_Ee replace the species / energy solves by the relative residuals
    of those iterates, returned as "check_res" ([S] species, then energy)."""
    n = _f64(cfg["n"] if n is None else n).copy()
    phi = _f64(cfg["phi"] if phi is None else phi).copy()
    Te = _f64(cfg["Te"] if Te is None else Te).copy()
    Ee = None if Ee is None else _f64(Ee).copy()
    S = n.shape[0]
    P = StepParams()
    P.grid = grid(cfg["grid"])
    P.dt = float(cfg["dt"])
    P.n_t = int(cfg.get("n_t", 1))
    P.mech = int(cfg["mech"])
    P.S = S
    P.te_mode = int(cfg["te_mode"])
    P.electron = int(electron)
    P.Tg = float(cfg["Tg"])
    P.N_gas = float(cfg["N_gas"])
    P.m_bg = float(m_bg)
    P.k_decay = float(k_decay)
    bg = list(cfg.get("bg", []))
    for i in range(4):
        P.bg[i] = bg[i] if i < len(bg) else 0.0
    P.c = Consts(**consts)
    P.phi_bc = bc(cfg["phi_bc"])
    P.energy_bc = bc(cfg["energy_bc"])
    SB = (BC * S)(*[bc(b) for b in cfg["species_bc"]])
    SP = species_array(species)
    P.species_bc = C.addressof(SB)
    P.species = C.addressof(SP)
    keep = [SB, SP]
    if "lfa" in cfg:
        t = _f64(cfg["lfa"]["te_K"])
        keep.append(t)
        P.lfa_te = _ptr(t)
        P.lfa_ln_min = cfg["lfa"]["ln_en_min"]
        P.lfa_ln_max = cfg["lfa"]["ln_en_max"]
        P.lfa_n = cfg["lfa"]["npts"]
    for name, arr in (("extra_source", extra_source), ("extra_energy", extra_energy), ("eps_cell", eps_cell),
                      ("species_guess", species_guess)):
        if arr is not None:
            a = _f64(arr)
            keep.append(a)
            setattr(P, name, _ptr(a))
    P.phi_fixed = 1 if phi_fixed else 0
    res = np.zeros(S + 1)
    for name, arr in (("check_n", check_n), ("check_Ee", check_Ee)):
        if arr is not None:
            a = _f64(arr)
            keep.append(a)
            setattr(P, name, _ptr(a))
    P.check_res = _ptr(res)
    P.poisson = poisson or mg_opts()
    P.species_mg = species_mg or mg_opts()
    P.energy_mg = energy_mg or mg_opts()
    nc = int(np.prod(n.shape[1:]))
    photo_S = None
    if photo is not None:
        A, lam = list(photo["A"]), list(photo["lam"])
        if not 1 <= len(A) <= 3 or len(lam) != len(A):
            raise ValueError("photoionization takes one to three terms")
        P.photo_n = len(A)
        for q in range(len(A)):
            P.photo_A[q], P.photo_lambda[q] = float(A[q]), float(lam[q])
        P.photo_pO2, P.photo_pg = float(photo["pO2"]), float(photo["pg"])
        P.photo_xi, P.photo_pq, P.photo_p = float(photo["xi"]), float(photo["pq"]), float(photo["p"])
        P.photo_nu_ratio = float(photo.get("nu_ratio", 1.0))
        P.photo_e, P.photo_ion = int(photo["e"]), int(photo["ion"])
        P.photo_bc = bc(photo.get("bc", {"kind": [0] * 6, "value": [0.0] * 6}))
        P.photo_mg = photo.get("mg") or mg_opts()
        photo_S = np.zeros((3,) + tuple(n.shape[1:]))
        P.photo_out = _ptr(photo_S)
    if adaptive_dt is not None:
        P.dt_mode = 1
        P.c_adv, P.c_diff, P.c_diel = (float(adaptive_dt[k]) for k in ("c_adv", "c_diff", "c_diel"))
    sig = None
    if diel is not None:
        for f in range(6):
            P.diel[f] = int(bool(diel[f]))
        sig = _f64(sigma).copy()
        P.sigma = _ptr(sig)
    P.see_gamma = float(see_gamma)
    if stick is not None:
        a = _f64(stick)
        keep.append(a)
        P.stick = _ptr(a)
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        if mk.size != nc:
            raise ValueError("mask has %d cells, the grid %d" % (mk.size, nc))
        keep.append(mk)
        P.mask = mk.ctypes.data
    info = StepInfo()
    st = lib(parallel).or_step(C.byref(P), _ptr(n), _ptr(phi), _ptr(Te), _ptr(Ee), C.byref(info))
    d = {k: getattr(info, k) for k, _ in StepInfo._fields_}
    return {"n": n, "phi": phi, "Te": Te, "Ee": Ee, "info": d, "status": st, "check_res": res, "photo_S": photo_S,
            "sigma": sig}


def trajectory(cfg, species, steps, *, poisson=None, species_mg=None, extrapolate=True, parallel=False, **kw):
    """`steps` oracle steps from the workload's initial state.  With
    extrapolate, each step's Poisson and species solves start from the
    polynomial extrapolation in time of the oracle's own earlier results
    (2u - h1 after one kept result, 3u - 3h1 + h2 after two; the initial
    state's potential, a guess rather than a result, is not kept), else from
    the previous values.  Harness code: the guesses are starting iterates
    and the solves still stop on their residual tests.  Returns the final
    state, the wall time of every step, the cycle counts and the inputs of
    the last step (to time that same step again)."""
    import time
    n, phi, Te = (_f64(cfg[k]).copy() for k in ("n", "phi", "Te"))
    hphi, hn = [], []          # kept results, newest last
    times, infos = [], []
    for t in range(steps):
        pg, sg = phi, None
        if extrapolate and len(hphi) == 1:
            pg = 2.0 * phi - hphi[-1]
        elif extrapolate and len(hphi) >= 2:
            pg = 3.0 * phi - 3.0 * hphi[-1] + hphi[-2]
        if extrapolate and len(hn) == 1:
            sg = 2.0 * n - hn[-1]
        elif extrapolate and len(hn) >= 2:
            sg = 3.0 * n - 3.0 * hn[-1] + hn[-2]
        last = {"n": n, "phi": pg, "Te": Te, "species_guess": sg}
        t0 = time.perf_counter()
        r = step(cfg, species, n=n, phi=pg, Te=Te, poisson=poisson, species_mg=species_mg, species_guess=sg,
                 parallel=parallel, **kw)
        times.append(time.perf_counter() - t0)
        if r["status"] != OK:
            raise RuntimeError("oracle step %d failed with status %d" % (t, r["status"]))
        if t > 0:
            hphi = (hphi + [phi])[-2:]
            hn = (hn + [n])[-2:]
        n, phi, Te = r["n"], r["phi"], r["Te"]
        infos.append(r["info"])
    return {"n": n, "phi": phi, "Te": Te, "times": times, "infos": infos, "last_step_inputs": last}


# ---------------------------------------------------------------------------
# The oracle's own transcription of the mechanism species (Appendix A,
# Table A.4 mobilities; neutral diffusion equal to the ionic counterpart's;
# background gases carry no wall flux).  Written independently of the
# product's tables.
# ---------------------------------------------------------------------------
AMU = 1.66053906660e-27
ME = 9.1093837015e-31


def _sp(Z, mass_u, mob_kind, wall, coef=0.0, transported=1, mass_kg=None):
    return {"Z": Z, "mass": mass_kg if mass_kg is not None else mass_u * AMU, "mob_kind": mob_kind,
            "wall_kind": wall, "mob_coef": coef, "transported": transported}


def species_arh2_15():
    """e, Ar+, Ar2+, H+, H2+, H3+, ArH+, Ar*, Ar2*, H2(v1), H2(v2), H2(v3), H, Ar, H2."""
    return [
        _sp(-1, 0, MOB_ELECTRON_FIT, WALL_ELECTRON, mass_kg=ME),
        _sp(+1, 39.948, MOB_ION_N0, WALL_ION, 1.85e-4),
        _sp(+1, 79.896, MOB_ION_N0, WALL_ION, 1.835e-4),
        _sp(+1, 1.008, MOB_ION_N0, WALL_ION, 30e-4),
        _sp(+1, 2.016, MOB_ION_N0, WALL_ION, 25.0e-4),
        _sp(+1, 3.024, MOB_ION_N0, WALL_ION, 32.0e-4),
        _sp(+1, 40.956, MOB_ION_N0, WALL_ION, 19.0e-4),
        _sp(0, 39.948, MOB_NEUTRAL_N0, WALL_NEUTRAL, 1.85e-4),
        _sp(0, 79.896, MOB_NEUTRAL_N0, WALL_NEUTRAL, 1.835e-4),
        _sp(0, 2.016, MOB_NEUTRAL_N0, WALL_NEUTRAL, 25.0e-4),
        _sp(0, 2.016, MOB_NEUTRAL_N0, WALL_NEUTRAL, 25.0e-4),
        _sp(0, 2.016, MOB_NEUTRAL_N0, WALL_NEUTRAL, 25.0e-4),
        _sp(0, 1.008, MOB_NEUTRAL_N0, WALL_NEUTRAL, 30e-4),
        _sp(0, 39.948, MOB_NEUTRAL_N0, WALL_NONE, 1.85e-4),
        _sp(0, 2.016, MOB_NEUTRAL_N0, WALL_NONE, 25.0e-4),
    ]


def species_ar3(mu_e=-0.03, D_e=0.06):
    """e (constant mobility/diffusion), Ar+, Ar*."""
    e = _sp(-1, 0, MOB_CONST, WALL_ELECTRON, mass_kg=ME)
    e["mu_const"], e["D_const"] = mu_e, D_e
    return [e, _sp(+1, 39.948, MOB_ION_N0, WALL_ION, 1.85e-4),
            _sp(0, 39.948, MOB_NEUTRAL_N0, WALL_NEUTRAL, 1.85e-4)]
