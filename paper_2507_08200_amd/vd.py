"""Python binding of libvd (ctypes).  Argument marshalling only.

Every computation runs in the HIP kernels of libvd.so; this module only
checks tensors (FP64, contiguous, on the GPU, right shape), packs the C
structs of include/vd.h and calls the C ABI with the same names.  PyTorch
provides device memory and the stream.  If libvd.so has not been built the
import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvd.so")

VD_OK, VD_EINVAL, VD_ENOMEM, VD_EHIP, VD_ENOCONV, VD_ESINGULAR = 0, -1, -2, -3, -4, -5
BC_DIRICHLET, BC_NEUMANN, BC_WALLFLUX, BC_PERIODIC = 0, 1, 2, 3
FP64, FP32_IR = 0, 1
GUESS_GIVEN, GUESS_ZERO, GUESS_LEARNED, GUESS_EXTRAP = 0, 1, 2, 3
MG_GRAPH, MG_AUTOTUNE, MG_FUSED_SWEEP, MG_TUNE_NU, MG_PERSISTENT = 1, 2, 4, 8, 16
TE_FIXED, TE_LFA, TE_ENERGY = 0, 1, 2
MECH_NONE, MECH_DECAY, MECH_AR3, MECH_ARH2_15 = 0, 1, 2, 3
MOB_CONST, MOB_ELECTRON_FIT, MOB_ION_N0, MOB_NEUTRAL_N0 = 0, 1, 2, 3
WALL_NONE, WALL_ELECTRON, WALL_ION, WALL_NEUTRAL = 0, 1, 2, 3

EXPORTS = ["vd_ctx_create", "vd_ctx_destroy", "vd_ctx_set_stream", "vd_last_error", "vd_version",
           "vd_poisson_solve", "vd_poisson_solve_noalloc", "vd_helmholtz_solve_batched", "vd_species_flux",
           "vd_reaction_source",
           "vd_step", "vd_cell_flags", "vd_smooth", "vd_timing_select", "vd_timing_read",
           "vd_nn_param_count", "vd_nn_create", "vd_nn_get", "vd_nn_set", "vd_nn_forward", "vd_nn_train_step",
           "vd_nn_features", "vd_nn_save", "vd_nn_load", "vd_nn_conv3d", "vd_check_tiles25", "vd_step_reset"]


class VDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libvd status %d: %s" % (status, msg))
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 6), ("value", C.c_double * 6)]


class MGOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_cycles", C.c_int32), ("fixed_cycles", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("n_levels", C.c_int32),
                ("precision", C.c_int32), ("guess", C.c_int32), ("ir_inner", C.c_int32),
                ("flags", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("outer_iters", C.c_int32), ("fallback", C.c_int32),
                ("levels", C.c_int32), ("status", C.c_int32), ("pad", C.c_int32),
                ("rel_res", C.c_double), ("rel_res0", C.c_double), ("bnorm", C.c_double),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("grid", Grid), ("bc", BC), ("mask", C.c_void_p), ("alpha", C.c_void_p),
                ("alpha_c", C.c_double), ("beta", C.c_void_p), ("beta_c", C.c_double),
                ("rhs", C.c_void_p), ("x", C.c_void_p)]


class Species(C.Structure):
    _fields_ = [("Z", C.c_double), ("mass_kg", C.c_double), ("transported", C.c_int32),
                ("mob_kind", C.c_int32), ("wall_kind", C.c_int32), ("pad", C.c_int32),
                ("mob_coef", C.c_double), ("mu_const", C.c_double), ("D_const", C.c_double)]


class Consts(C.Structure):
    _fields_ = [("qe", C.c_double), ("eps0", C.c_double), ("kB", C.c_double), ("me", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("grid", Grid), ("dt", C.c_double), ("n_t", C.c_int32), ("mech", C.c_int32),
                ("S", C.c_int32), ("te_mode", C.c_int32), ("electron", C.c_int32), ("pad0", C.c_int32),
                ("Tg", C.c_double), ("N_gas", C.c_double), ("m_bg", C.c_double), ("k_decay", C.c_double),
                ("bg", C.c_double * 4), ("consts", Consts), ("phi_bc", BC), ("energy_bc", BC),
                ("species_bc", C.c_void_p), ("species", C.c_void_p), ("lfa_te", C.c_void_p),
                ("lfa_ln_min", C.c_double), ("lfa_ln_max", C.c_double), ("lfa_n", C.c_int32),
                ("pad1", C.c_int32), ("extra_source", C.c_void_p), ("extra_energy", C.c_void_p),
                ("eps_cell", C.c_void_p), ("poisson", MGOpts), ("species_mg", MGOpts), ("energy_mg", MGOpts),
                ("photo_n", C.c_int32), ("photo_e", C.c_int32), ("photo_ion", C.c_int32), ("dt_mode", C.c_int32),
                ("photo_A", C.c_double * 3), ("photo_lambda", C.c_double * 3),
                ("photo_pO2", C.c_double), ("photo_pg", C.c_double), ("photo_xi", C.c_double),
                ("photo_pq", C.c_double), ("photo_p", C.c_double), ("photo_nu_ratio", C.c_double),
                ("photo_bc", BC), ("photo_mg", MGOpts), ("photo_out", C.c_void_p),
                ("c_adv", C.c_double), ("c_diff", C.c_double), ("c_diel", C.c_double),
                ("diel", C.c_int32 * 6), ("sigma", C.c_void_p), ("see_gamma", C.c_double), ("stick", C.c_void_p),
                ("mask", C.c_void_p)]


class NNConfig(C.Structure):
    _fields_ = [("levels", C.c_int32), ("ch", C.c_int32 * 4), ("cin", C.c_int32)]


def nn_config(cfg):
    ch = list(cfg["ch"]) + [0] * (4 - len(cfg["ch"]))
    return NNConfig(int(cfg["levels"]), (C.c_int32 * 4)(*ch), int(cfg.get("cin", 2)))


class State(C.Structure):
    _fields_ = [("n", C.c_void_p), ("phi", C.c_void_p), ("Te", C.c_void_p), ("Ee", C.c_void_p)]


class StepInfo(C.Structure):
    _fields_ = [("poisson_cycles", C.c_int32), ("species_cycles", C.c_int32), ("energy_cycles", C.c_int32),
                ("status", C.c_int32), ("poisson_rel", C.c_double), ("dt_used", C.c_double),
                ("ms_poisson", C.c_double), ("ms_transport", C.c_double), ("ms_energy", C.c_double),
                ("ms_species", C.c_double), ("ms_total", C.c_double)]


_lib = None


def load():
    """Load libvd.so (built in-tree by build.py); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvd.so not found at %s: build it with paper_2507_08200_amd.build.build()" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    P, i32, d = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "vd_ctx_create": ([C.POINTER(P), P], i32),
        "vd_ctx_destroy": ([P], None),
        "vd_ctx_set_stream": ([P, P], i32),
        "vd_last_error": ([P], C.c_char_p),
        "vd_version": ([], C.c_char_p),
        "vd_poisson_solve": ([P, P, P, P, P, d, P, P, P, P], i32),
        "vd_poisson_solve_noalloc": ([P, P, P, P, P, d, P, P, P, P], i32),
        "vd_helmholtz_solve_batched": ([P, i32, P, P, P], i32),
        "vd_species_flux": ([P, P, P, P, i32, P, P, P, P, P, P, d, P, P, i32, P], i32),
        "vd_reaction_source": ([P, i32, C.c_int64, i32, P, P, P, d, P, P], i32),
        "vd_step": ([P, P, P, P], i32),
        "vd_step_reset": ([P], i32),
        "vd_cell_flags": ([P, P, i32, i32, P], i32),
        "vd_smooth": ([P, P, i32], i32),
        "vd_nn_param_count": ([P], C.c_int64),
        "vd_nn_create": ([P, P, P], i32),
        "vd_nn_get": ([P, i32, P], i32),
        "vd_nn_set": ([P, i32, P], i32),
        "vd_nn_forward": ([P, P, P, P], i32),
        "vd_nn_train_step": ([P, P, P, P, C.c_float, i32, C.POINTER(C.c_double)], i32),
        "vd_nn_features": ([P, P, P, P, d, P, C.POINTER(C.c_double)], i32),
        "vd_nn_save": ([P, C.c_char_p], i32),
        "vd_nn_load": ([P, C.c_char_p], i32),
        "vd_nn_conv3d": ([P, P, P, i32, P, P, i32, i32, P, P, P, P, P], i32),
        "vd_timing_select": ([P, C.c_char_p], i32),
        "vd_check_tiles25": ([i32, i32, i32, i32, i32, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], i32),
        "vd_timing_read": ([P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


# ------------------------------------------------------------- marshalling
def _dptr(t, shape=None, dtype=torch.float64, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


def _bf16_ptr(t, numel):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.bfloat16 or not t.is_contiguous():
        raise ValueError("expected a contiguous bfloat16 tensor on the GPU")
    if t.numel() < numel:
        raise ValueError("bfloat16 tensor too small: %d < %d" % (t.numel(), numel))
    return t.data_ptr()


def grid(g):
    nx, ny, nz, dx, dy, dz = g
    return Grid(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz))


def bc(b):
    out = BC()
    for f in range(6):
        out.kind[f] = int(b["kind"][f])
        out.value[f] = float(b["value"][f])
    return out


def mg_opts(rtol=1e-10, max_cycles=100, fixed_cycles=0, nu_pre=2, nu_post=2, n_levels=0, precision=FP64,
            guess=GUESS_GIVEN, ir_inner=4, graph=False, autotune=False, fused_sweep=False, tune_nu=False,
            persistent=False):
    return MGOpts(float(rtol), int(max_cycles), int(fixed_cycles), int(nu_pre), int(nu_post), int(n_levels),
                  int(precision), int(guess), int(ir_inner),
                  (MG_GRAPH if graph else 0) | (MG_AUTOTUNE if autotune else 0) |
                  (MG_FUSED_SWEEP if fused_sweep else 0) | (MG_TUNE_NU if tune_nu else 0) |
                  (MG_PERSISTENT if persistent else 0))


def _info(si):
    return {k: getattr(si, k) for k, _ in si._fields_ if k != "pad"}


class Context:
    """A libvd context bound to a HIP stream (torch's current stream)."""

    def __init__(self, stream=None):
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        st = self.lib.vd_ctx_create(C.byref(h), C.c_void_p(stream.cuda_stream))
        if st != VD_OK:
            raise VDError(st, "vd_ctx_create failed (is a GPU visible?)")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.vd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != VD_OK and st not in allow:
            msg = self.lib.vd_last_error(self.h)
            raise VDError(st, msg.decode() if msg else "")
        return st

    # ---------------------------------------------------------- solvers
    def vd_poisson_solve(self, g, phi_bc, rho, phi, *, mask=None, beta=None, beta_c=8.8541878128e-12,
                         opts=None, allow_fail=False, want_info=True):
        return self._poisson(self.lib.vd_poisson_solve, g, phi_bc, rho, phi, mask, beta, beta_c, opts, allow_fail,
                             want_info)

    def vd_poisson_solve_noalloc(self, g, phi_bc, rho, phi, *, mask=None, beta=None, beta_c=8.8541878128e-12,
                                 opts=None, allow_fail=False, want_info=True):
        """vd_poisson_solve with every work array in the library's static
        device scratch (no device allocation)."""
        return self._poisson(self.lib.vd_poisson_solve_noalloc, g, phi_bc, rho, phi, mask, beta, beta_c, opts,
                             allow_fail, want_info)

    def _poisson(self, fn, g, phi_bc, rho, phi, mask, beta, beta_c, opts, allow_fail, want_info):
        nx, ny, nz = g[:3]
        shp = (nz, ny, nx)
        info = SolveInfo()
        st = fn(self.h, C.byref(grid(g)), C.byref(bc(phi_bc)), _dptr(mask, shp, torch.uint8, "mask"),
                _dptr(beta, shp, name="beta"), float(beta_c), _dptr(rho, shp, name="rho"), _dptr(phi, shp, name="phi"),
                C.byref(opts or mg_opts()), C.byref(info) if want_info else None)
        self._check(st, (VD_ENOCONV,) if allow_fail else ())
        if not want_info:
            return {"return": st}
        d = _info(info)
        d["return"] = st
        return d

    def vd_helmholtz_solve_batched(self, problems, opts=None, allow_fail=False):
        """problems: list of dicts with keys grid, bc, rhs, x and optional
        mask, alpha / alpha_c, beta / beta_c (tensors on the GPU)."""
        n = len(problems)
        arr = (Problem * n)()
        for p, pr in enumerate(problems):
            nx, ny, nz = pr["grid"][:3]
            shp = (nz, ny, nx)
            arr[p] = Problem(grid(pr["grid"]), bc(pr["bc"]), _dptr(pr.get("mask"), shp, torch.uint8, "mask"),
                             _dptr(pr.get("alpha"), shp, name="alpha"), float(pr.get("alpha_c", 0.0)),
                             _dptr(pr.get("beta"), shp, name="beta"), float(pr.get("beta_c", 0.0)),
                             _dptr(pr["rhs"], shp, name="rhs"), _dptr(pr["x"], shp, name="x"))
        infos = (SolveInfo * n)()
        st = self.lib.vd_helmholtz_solve_batched(self.h, n, arr, C.byref(opts or mg_opts()), infos)
        self._check(st, (VD_ENOCONV,) if allow_fail else ())
        return [_info(infos[p]) for p in range(n)], st

    # ------------------------------------------------- warm-start network
    def vd_nn_create(self, cfg, params=None):
        """cfg: {"levels", "ch", "cin"}; params: numpy FP32 vector or None."""
        c = nn_config(cfg)
        n = self.lib.vd_nn_param_count(C.byref(c))
        if n < 0:
            raise ValueError("invalid network configuration %r" % (cfg,))
        buf = None
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            if params.size != n:
                raise ValueError("expected %d parameters, got %d" % (n, params.size))
            buf = params.ctypes.data
        self._check(self.lib.vd_nn_create(self.h, C.byref(c), buf))
        self._nn_n = int(n)
        return int(n)

    def vd_nn_get(self, which=0):
        out = np.empty(self._nn_n, dtype=np.float32)
        self._check(self.lib.vd_nn_get(self.h, int(which), out.ctypes.data))
        return out

    def vd_nn_set(self, params, which=0):
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.size != self._nn_n:
            raise ValueError("expected %d values" % self._nn_n)
        self._check(self.lib.vd_nn_set(self.h, int(which), params.ctypes.data))

    def vd_nn_forward(self, g, x_bf16):
        nx, ny, nz = g[:3]
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=x_bf16.device)
        self._check(self.lib.vd_nn_forward(self.h, C.byref(grid(g)), _bf16_ptr(x_bf16, nx * ny * nz),
                                           _dptr(out, dtype=torch.float32, name="out")))
        return out

    def vd_nn_train_step(self, g, x_bf16, target, lr, update=True):
        nx, ny, nz = g[:3]
        loss = C.c_double(0.0)
        self._check(self.lib.vd_nn_train_step(self.h, C.byref(grid(g)), _bf16_ptr(x_bf16, nx * ny * nz),
                                              _dptr(target, (nz, ny, nx), torch.float32, "target"), float(lr),
                                              int(bool(update)), C.byref(loss)))
        return loss.value

    def vd_nn_features(self, g, phi_bc, rho, eps=8.8541878128e-12):
        nx, ny, nz = g[:3]
        out = torch.empty((nz, ny, nx, 2), dtype=torch.bfloat16, device=rho.device)
        vref = C.c_double(0.0)
        self._check(self.lib.vd_nn_features(self.h, C.byref(grid(g)), C.byref(bc(phi_bc)),
                                            _dptr(rho, (nz, ny, nx), name="rho"), float(eps), out.data_ptr(),
                                            C.byref(vref)))
        return out, vref.value

    def vd_nn_save(self, path):
        self._check(self.lib.vd_nn_save(self.h, str(path).encode()))

    def vd_nn_load(self, path):
        self._check(self.lib.vd_nn_load(self.h, str(path).encode()))
        with open(path, "rb") as f:
            head = f.read(8 + 6 * 4 + 8)
        self._nn_n = int(np.frombuffer(head[32:40], dtype=np.int64)[0])
        return self._nn_n

    def vd_nn_conv3d(self, g, x_bf16, w, b, relu=False, dy=None):
        """One convolution: x [cells][ci] bf16, w [co][27][ci], b [co] FP32.
        Returns y [cells][co] and, with dy, (dx, dw, db)."""
        nx, ny, nz = g[:3]
        n = nx * ny * nz
        co, ci = int(w.shape[0]), int(w.shape[-1])
        y = torch.empty((n, co), dtype=torch.float32, device=x_bf16.device)
        dx = dw = db = None
        if dy is not None:
            dx = torch.empty((n, ci), dtype=torch.float32, device=x_bf16.device)
            dw = torch.empty_like(w)
            db = torch.empty_like(b)
        self._check(self.lib.vd_nn_conv3d(
            self.h, C.byref(grid(g)), _bf16_ptr(x_bf16, n * ci), ci, _dptr(w, dtype=torch.float32, name="w"),
            _dptr(b, dtype=torch.float32, name="b"), co, int(bool(relu)), y.data_ptr(),
            None if dy is None else _dptr(dy, (n, co), torch.float32, "dy"),
            None if dx is None else dx.data_ptr(), None if dw is None else dw.data_ptr(),
            None if db is None else db.data_ptr()))
        return y if dy is None else (y, dx, dw, db)

    def vd_species_flux(self, g, phi_bc, species_bc, species, n, phi, mu, Te, Tg, consts, D=None, flux_species=-1):
        """Drift divergence [S][cells]; with flux_species >= 0 (and D) also
        the total face flux of that species as (fx, fy, fz)."""
        nx, ny, nz = g[:3]
        S = len(species)
        shp = (nz, ny, nx)
        out = torch.empty((S,) + shp, dtype=torch.float64, device=n.device)
        faces = None
        if flux_species >= 0:
            nf = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
            faces = torch.empty(nf, dtype=torch.float64, device=n.device)
        SB = (BC * S)(*[bc(b) for b in species_bc])
        SP = species_array(species)
        st = self.lib.vd_species_flux(self.h, C.byref(grid(g)), C.byref(bc(phi_bc)), SB, S, SP,
                                      _dptr(n, (S,) + shp, name="n"), _dptr(phi, shp, name="phi"),
                                      _dptr(mu, (S,) + shp, name="mu"),
                                      None if D is None else _dptr(D, (S,) + shp, name="D"),
                                      _dptr(Te, shp, name="Te"), float(Tg),
                                      C.byref(Consts(**consts)), _dptr(out, name="div"), int(flux_species),
                                      None if faces is None else faces.data_ptr())
        self._check(st)
        if faces is None:
            return out
        a, b = (nx + 1) * ny * nz, nx * (ny + 1) * nz
        return out, (faces[:a].view(nz, ny, nx + 1), faces[a:a + b].view(nz, ny + 1, nx),
                     faces[a + b:].view(nz + 1, ny, nx))

    def vd_reaction_source(self, mech, n, Te, bg=(), qe=1.602176634e-19):
        S = n.shape[0]
        nc = n[0].numel()
        G = torch.empty_like(n)
        Sin = torch.empty_like(Te)
        bga = (C.c_double * 4)(*(list(bg) + [0.0] * (4 - len(bg))))
        st = self.lib.vd_reaction_source(self.h, int(mech), nc, S, _dptr(n, name="n"), _dptr(Te, name="Te"), bga,
                                         float(qe), _dptr(G), _dptr(Sin))
        self._check(st)
        return G, Sin

    def vd_step(self, params, state, want_info=True):
        """params: StepParams built by step_params(); state: dict of tensors."""
        S = params.S
        nx, ny, nz = params.grid.nx, params.grid.ny, params.grid.nz
        shp = (nz, ny, nx)
        s = State(_dptr(state["n"], (S,) + shp, name="n"), _dptr(state["phi"], shp, name="phi"),
                  _dptr(state["Te"], shp, name="Te"), _dptr(state.get("Ee"), shp, name="Ee"))
        info = StepInfo()
        st = self.lib.vd_step(self.h, C.byref(params), C.byref(s), C.byref(info) if want_info else None)
        self._check(st)
        return _info(info) if want_info else None

    # ------------------------------------------------------- inspection
    def vd_step_reset(self):
        self._check(self.lib.vd_step_reset(self.h))

    def vd_cell_flags(self, problem, level, n_levels=0):
        nx, ny, nz = problem["grid"][:3]
        shp = (nz, ny, nx)
        p = Problem(grid(problem["grid"]), bc(problem["bc"]), _dptr(problem.get("mask"), shp, torch.uint8, "mask"),
                    _dptr(problem.get("alpha"), shp), float(problem.get("alpha_c", 0.0)), _dptr(problem.get("beta"), shp),
                    float(problem.get("beta_c", 0.0)), None, None)
        out = torch.empty((nz >> level, ny >> level, nx >> level), dtype=torch.uint8, device="cuda")
        self._check(self.lib.vd_cell_flags(self.h, C.byref(p), int(n_levels), int(level), _dptr(out, dtype=torch.uint8)))
        return out

    def vd_smooth(self, problem, ncolour):
        nx, ny, nz = problem["grid"][:3]
        shp = (nz, ny, nx)
        p = Problem(grid(problem["grid"]), bc(problem["bc"]), _dptr(problem.get("mask"), shp, torch.uint8, "mask"),
                    _dptr(problem.get("alpha"), shp), float(problem.get("alpha_c", 0.0)), _dptr(problem.get("beta"), shp),
                    float(problem.get("beta_c", 0.0)), _dptr(problem["rhs"], shp), _dptr(problem["x"], shp))
        self._check(self.lib.vd_smooth(self.h, C.byref(p), int(ncolour)))

    def vd_timing_select(self, kernels):
        """kernels: comma-separated kernel families, or None to stop timing."""
        self._check(self.lib.vd_timing_select(self.h, kernels.encode() if kernels else None))

    def vd_timing_read(self, kernel):
        """(launches, total device ms, algorithmic bytes) of one family."""
        n, ms, u = C.c_int64(), C.c_double(), C.c_double()
        self._check(self.lib.vd_timing_read(self.h, kernel.encode(), C.byref(n), C.byref(ms), C.byref(u)))
        return n.value, ms.value, u.value


def check_tiles25(nx, ny, nz, periodic, kz, kernel):
    """(accesses, violations) of the host-side walk over a 2.5D tiled pass
    (vd_check_tiles25; no GPU needed)."""
    a, v = C.c_int64(), C.c_int64()
    st = load().vd_check_tiles25(int(nx), int(ny), int(nz), int(periodic), int(kz), int(kernel), C.byref(a), C.byref(v))
    if st != VD_OK:
        raise VDError(st, "vd_check_tiles25 rejected the shape")
    return a.value, v.value


def species_array(species):
    arr = (Species * len(species))()
    for s, sp in enumerate(species):
        arr[s] = Species(float(sp["Z"]), float(sp["mass"]), int(sp.get("transported", 1)), int(sp["mob_kind"]),
                         int(sp["wall_kind"]), 0, float(sp.get("mob_coef", 0.0)), float(sp.get("mu_const", 0.0)),
                         float(sp.get("D_const", 0.0)))
    return arr


PHYS = {"qe": 1.602176634e-19, "eps0": 8.8541878128e-12, "kB": 1.380649e-23, "me": 9.1093837015e-31}


def step_params(cfg, species, *, consts=PHYS, lfa=None, poisson=None, species_mg=None, energy_mg=None,
                extra_source=None, extra_energy=None, eps_cell=None, electron=0, m_bg=0.0, k_decay=0.0,
                photo=None, adaptive_dt=None, diel=None, sigma=None, see_gamma=0.0, stick=None, mask=None):
    """Pack a workload dict (see inputs) into vd_step_params.  Device arrays
    (lfa table, sources, sigma, photo["out"]) must be torch tensors; the
    returned object keeps references to everything it points at.
    photo: dict with "A", "lam" (one to three terms), "pO2", "pg", "xi",
    "pq", "p", "nu_ratio" (default 1), "e", "ion", "bc" (default
    homogeneous Dirichlet), "mg" (mg_opts), "out" (optional [3][cells]).
    adaptive_dt: dict with "c_adv", "c_diff", "c_diel".  diel: six flags with
    sigma the packed surface charge (advanced in place).  stick: [S].
    mask: uint8 tensor [cells] (1 valid, 0 covered)."""
    P = StepParams()
    P.grid = grid(cfg["grid"])
    P.dt = float(cfg["dt"])
    P.n_t = int(cfg.get("n_t", 1))
    P.mech = int(cfg["mech"])
    P.S = len(species)
    P.te_mode = int(cfg["te_mode"])
    P.electron = int(electron)
    P.Tg = float(cfg["Tg"])
    P.N_gas = float(cfg["N_gas"])
    P.m_bg = float(m_bg)
    P.k_decay = float(k_decay)
    bg = list(cfg.get("bg", []))
    for i in range(4):
        P.bg[i] = bg[i] if i < len(bg) else 0.0
    P.consts = Consts(**consts)
    P.phi_bc = bc(cfg["phi_bc"])
    P.energy_bc = bc(cfg["energy_bc"])
    SB = (BC * P.S)(*[bc(b) for b in cfg["species_bc"]])
    SP = species_array(species)
    P.species_bc = C.addressof(SB)
    P.species = C.addressof(SP)
    keep = [SB, SP]
    if lfa is not None:
        P.lfa_te = _dptr(lfa["te_K"], name="lfa")
        P.lfa_ln_min = float(lfa["ln_en_min"])
        P.lfa_ln_max = float(lfa["ln_en_max"])
        P.lfa_n = int(lfa["npts"])
        keep.append(lfa["te_K"])
    for name, arr in (("extra_source", extra_source), ("extra_energy", extra_energy), ("eps_cell", eps_cell)):
        if arr is not None:
            setattr(P, name, _dptr(arr, name=name))
            keep.append(arr)
    P.poisson = poisson or mg_opts()
    P.species_mg = species_mg or mg_opts()
    P.energy_mg = energy_mg or mg_opts()
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
        if photo.get("out") is not None:
            P.photo_out = _dptr(photo["out"], name="photo out")
            keep.append(photo["out"])
    if adaptive_dt is not None:
        P.dt_mode = 1
        P.c_adv, P.c_diff, P.c_diel = (float(adaptive_dt[k]) for k in ("c_adv", "c_diff", "c_diel"))
    if diel is not None:
        for f in range(6):
            P.diel[f] = int(bool(diel[f]))
        P.sigma = _dptr(sigma, name="sigma")
        keep.append(sigma)
    P.see_gamma = float(see_gamma)
    if stick is not None:
        st = (C.c_double * P.S)(*[float(v) for v in stick])
        keep.append(st)
        P.stick = C.addressof(st)
    if mask is not None:
        nx, ny, nz = cfg["grid"][:3]
        P.mask = _dptr(mask, (nz, ny, nx), torch.uint8, "mask")
        keep.append(mask)
    P._keep = keep
    return P
