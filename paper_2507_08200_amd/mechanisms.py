"""Species descriptors of the mechanisms the library carries (Appendix A).

Mobilities follow Table A.4 (electron fit in E/N; ions c_i N0/N); every
diffusion coefficient comes from the Einstein relation; a neutral diffuses
like its ionic counterpart of the same molecular structure.  The background
gases (Ar, H2) carry no wall flux.  Order matches the reaction kernels:
e, Ar+, Ar2+, H+, H2+, H3+, ArH+, Ar*, Ar2*, H2(v1), H2(v2), H2(v3), H, Ar, H2.
"""
from __future__ import annotations

from . import vd

DALTON = 1.66053906660e-27
M_E = 9.1093837015e-31

# (name, charge, mass in Da, mobility model, wall model, Table A.4 coefficient)
_ARH2 = [
    ("e", -1, None, vd.MOB_ELECTRON_FIT, vd.WALL_ELECTRON, 0.0),
    ("Ar+", 1, 39.948, vd.MOB_ION_N0, vd.WALL_ION, 1.85e-4),
    ("Ar2+", 1, 2 * 39.948, vd.MOB_ION_N0, vd.WALL_ION, 1.835e-4),
    ("H+", 1, 1.008, vd.MOB_ION_N0, vd.WALL_ION, 30e-4),
    ("H2+", 1, 2 * 1.008, vd.MOB_ION_N0, vd.WALL_ION, 25.0e-4),
    ("H3+", 1, 3 * 1.008, vd.MOB_ION_N0, vd.WALL_ION, 32.0e-4),
    ("ArH+", 1, 39.948 + 1.008, vd.MOB_ION_N0, vd.WALL_ION, 19.0e-4),
    ("Ar*", 0, 39.948, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 1.85e-4),       # like Ar+
    ("Ar2*", 0, 2 * 39.948, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 1.835e-4),  # like Ar2+
    ("H2(v1)", 0, 2 * 1.008, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 25.0e-4),  # like H2+
    ("H2(v2)", 0, 2 * 1.008, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 25.0e-4),
    ("H2(v3)", 0, 2 * 1.008, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 25.0e-4),
    ("H", 0, 1.008, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 30e-4),              # like H+
    ("Ar", 0, 39.948, vd.MOB_NEUTRAL_N0, vd.WALL_NONE, 1.85e-4),
    ("H2", 0, 2 * 1.008, vd.MOB_NEUTRAL_N0, vd.WALL_NONE, 25.0e-4),
]

ARH2_NAMES = [s[0] for s in _ARH2]


def _desc(Z, mass_da, mob, wall, coef, mass_kg=None):
    return {"Z": Z, "mass": mass_kg if mass_kg is not None else mass_da * DALTON, "mob_kind": mob,
            "wall_kind": wall, "mob_coef": coef, "transported": 1}


def arh2_15(transport_background: bool = True):
    """The 15-species Ar-H2 mechanism.  transport_background=False holds
    the background Ar and H2 densities fixed."""
    out = []
    for name, Z, mda, mob, wall, coef in _ARH2:
        d = _desc(Z, mda, mob, wall, coef, mass_kg=M_E if name == "e" else None)
        if name in ("Ar", "H2") and not transport_background:
            d["transported"] = 0
        out.append(d)
    return out


def ar3(mu_e: float = -0.03, D_e: float = 0.06):
    """e (constant mobility and diffusion), Ar+, Ar* over background Ar."""
    e = _desc(-1, 0.0, vd.MOB_CONST, vd.WALL_ELECTRON, 0.0, mass_kg=M_E)
    e["mu_const"], e["D_const"] = mu_e, D_e
    return [e, _desc(1, 39.948, vd.MOB_ION_N0, vd.WALL_ION, 1.85e-4),
            _desc(0, 39.948, vd.MOB_NEUTRAL_N0, vd.WALL_NEUTRAL, 1.85e-4)]
