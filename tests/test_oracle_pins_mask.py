"""Pins of the oracle's masked step (covered regions inside the domain).

Expected results come from other code paths of the oracle, not from the
masked formulas themselves: an all-valid mask is the unmasked step; covered
planes at the x+ end hold the potential g and must reproduce, cell for cell,
the unmasked step on the smaller grid whose x+ face is a Dirichlet face
(potential g, densities 0) -- the half-cell field, the lifting, the WENO5
ghosts mirrored across the face, the mobility at the face and the
homogeneous Dirichlet rows of the implicit solves all have their domain-face
counterparts there; and a covered box centred in y and z with data that are
mirror-symmetric in y and z gives a mirror-symmetric step.  A wrong sign or
factor in the lifting or the face field, a mirror index off by one, a
stencil that reads a covered cell or a missing restore of the covered
potentials fails one of these.
"""
import numpy as np
import pytest

from paper_2507_08200_amd import inputs as I

D, N, W, P = I.BC_DIRICHLET, I.BC_NEUMANN, I.BC_WALLFLUX, I.BC_PERIODIC
TOL_MG = dict(rtol=1e-13, max_cycles=400)


def _fields(r):
    return {"n": r["n"], "phi": r["phi"], "Te": r["Te"]}


def test_all_valid_mask_is_the_unmasked_step(oracle):
    cfg = I.cfg1(n=16)
    sp = oracle.species_ar3()
    kw = dict(poisson=oracle.mg_opts(fixed_cycles=6), species_mg=oracle.mg_opts(fixed_cycles=2))
    a = oracle.step(cfg, sp, **kw)
    b = oracle.step(cfg, sp, mask=np.ones(16 ** 3, np.uint8), **kw)
    assert a["status"] == 0 and b["status"] == 0
    for k in ("n", "phi", "Te"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("ncov", [2, 4])
def test_covered_x_planes_equal_a_dirichlet_face(oracle, ncov):
    """16 valid x-planes plus ncov covered ones holding phi = g equal the
    16-plane step with a Dirichlet x+ face (phi = g, densities 0), to the
    solver tolerance (the two grids have different multigrid hierarchies)."""
    small = I.cfg1(n=16)
    g = 250.0
    nx, h = 16, small["grid"][3]
    small["phi_bc"] = I.bc([D, D, N, N, N, N], [1000.0, g, 0, 0, 0, 0])
    small["species_bc"] = [I.bc([W, D, N, N, N, N], [0, 0, 0, 0, 0, 0])] * 3
    big = dict(small)
    nb = nx + ncov
    big["grid"] = (nb, 16, 16, h, h, h)
    rng = np.random.default_rng(5)
    nbig = rng.uniform(1e14, 1e16, (3, 16, 16, nb))     # covered values must not matter
    nbig[:, :, :, :nx] = small["n"]
    pbig = np.zeros((16, 16, nb))
    pbig[:, :, nx:] = g
    big["n"], big["phi"] = nbig, pbig
    big["Te"] = np.full((16, 16, nb), small["Te"][0, 0, 0])
    big["phi_bc"] = I.bc([D, N, N, N, N, N], [1000.0, 0, 0, 0, 0, 0])   # beyond the covered planes: unused
    big["species_bc"] = [I.bc([W, W, N, N, N, N])] * 3
    mask = np.ones((16, 16, nb), np.uint8)
    mask[:, :, nx:] = 0
    sp = oracle.species_ar3()
    kw = dict(poisson=oracle.mg_opts(**TOL_MG), species_mg=oracle.mg_opts(**TOL_MG))
    rs = oracle.step(small, sp, **kw)
    rb = oracle.step(big, sp, mask=mask, **kw)
    assert rs["status"] == 0 and rb["status"] == 0
    for k in range(3):
        a, b = rb["n"][k][:, :, :nx], rs["n"][k]
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max(), k
        assert np.all(rb["n"][k][:, :, nx:] == 0.0)
    assert np.abs(rb["phi"][:, :, :nx] - rs["phi"]).max() <= 1e-10 * np.abs(rs["phi"]).max()
    assert np.all(rb["phi"][:, :, nx:] == g)


def test_mirror_symmetric_electrode(oracle):
    """A covered box centred in y and z (an electrode at 400 V inside the
    gas) with y- and z-symmetric data: the step is y- and z-symmetric."""
    n = 16
    cfg = I.cfg1(n=n)
    dens = cfg["n"]
    dens = 0.25 * (dens + dens[:, :, ::-1, :] + dens[:, ::-1, :, :] + dens[:, ::-1, ::-1, :])
    cfg["n"] = dens
    cfg["species_bc"] = [I.bc([W, W, W, W, W, W])] * 3
    mask = np.ones((n, n, n), np.uint8)
    mask[6:10, 6:10, 9:12] = 0
    phi = np.zeros((n, n, n))
    phi[mask == 0] = 400.0
    cfg["phi"] = phi
    sp = oracle.species_ar3()
    r = oracle.step(cfg, sp, mask=mask.ravel(), poisson=oracle.mg_opts(**TOL_MG), species_mg=oracle.mg_opts(**TOL_MG))
    assert r["status"] == 0
    assert np.all(r["phi"][mask == 0] == 400.0)
    assert np.all(r["n"][:, mask == 0] == 0.0)
    for f in (r["phi"], r["n"][0], r["n"][1]):
        s = np.abs(f).max()
        assert np.abs(f - f[::-1, :, :]).max() <= 1e-9 * s
        assert np.abs(f - f[:, ::-1, :]).max() <= 1e-9 * s
    # next to the electrode the potential moves toward its 400 V
    u = oracle.step(cfg, sp, poisson=oracle.mg_opts(**TOL_MG), species_mg=oracle.mg_opts(**TOL_MG))
    for c in ((8, 8, 8), (8, 8, 12)):
        assert abs(r["phi"][c] - 400.0) < abs(u["phi"][c] - 400.0), c


def test_mask_rejects_unsupported_combinations(oracle):
    cfg = I.cfg1(n=8)
    sp = oracle.species_ar3()
    m = np.ones(8 ** 3, np.uint8)
    m[0] = 0
    c2 = dict(cfg, phi_bc=I.bc([D, D, P, P, N, N], [1000.0, 0, 0, 0, 0, 0]))
    assert oracle.step(c2, sp, mask=m)["status"] != 0
    ph = {"A": [1e3], "lam": [20.0], "pO2": 150.0, "pg": 760.0, "xi": 0.06, "pq": 30.0, "p": 760.0, "e": 0, "ion": 1}
    assert oracle.step(cfg, sp, mask=m, photo=ph)["status"] != 0
    assert oracle.step(cfg, sp, mask=m, diel=[1, 0, 0, 0, 0, 0], sigma=np.zeros(64))["status"] != 0


def test_masked_adaptive_dt_equals_the_dirichlet_face_grid(oracle):
    """Eq. (20) over the valid cells: the covered planes' grid takes the same
    step as the grid with the Dirichlet x+ face (the field next to the face
    is the half-cell difference on both, and the advection limit there is
    the least); the covered cells' density of 1e18, whose dielectric limit
    (~9e-10 s) would be the least, does not enter the minimum."""
    small = I.cfg1(n=16)
    g = -2000.0                      # a steep drop at the face: the advection limit sits there
    nx, h = 16, small["grid"][3]
    small["dt"] = 1e-8
    small["phi_bc"] = I.bc([D, D, N, N, N, N], [1000.0, g, 0, 0, 0, 0])
    small["species_bc"] = [I.bc([W, D, N, N, N, N], [0, 0, 0, 0, 0, 0])] * 3
    big = dict(small)
    nb = nx + 2
    big["grid"] = (nb, 16, 16, h, h, h)
    nbig = np.full((3, 16, 16, nb), 1e18)
    nbig[:, :, :, :nx] = small["n"]
    pbig = np.zeros((16, 16, nb))
    pbig[:, :, nx:] = g
    pbig[:, :, nx + 1:] = 5e5            # a huge field between the covered planes: must not count
    big["n"], big["phi"] = nbig, pbig
    big["Te"] = np.full((16, 16, nb), small["Te"][0, 0, 0])
    big["phi_bc"] = I.bc([D, N, N, N, N, N], [1000.0, 0, 0, 0, 0, 0])
    big["species_bc"] = [I.bc([W, W, N, N, N, N])] * 3
    mask = np.ones((16, 16, nb), np.uint8)
    mask[:, :, nx:] = 0
    sp = oracle.species_ar3()
    ad = {"c_adv": 0.3, "c_diff": 10.0, "c_diel": 0.5}
    kw = dict(poisson=oracle.mg_opts(**TOL_MG), species_mg=oracle.mg_opts(**TOL_MG), adaptive_dt=ad, electron=0)
    small["phi"] = pbig[:, :, :nx].copy()
    rs = oracle.step(small, sp, **kw)
    rb = oracle.step(big, sp, mask=mask, **kw)
    assert rs["status"] == 0 and rb["status"] == 0
    ds, db = rs["info"]["dt_used"], rb["info"]["dt_used"]
    assert ds < small["dt"]
    assert abs(db - ds) <= 1e-14 * ds


def test_masked_energy_equation_equals_the_dirichlet_face_grid(oracle):
    """Electron energy (Eqs. (5)-(8)) in a masked step: the covered planes'
    grid equals the grid with a Dirichlet x+ face (potential g, densities
    and energy 0), Joule heating with the drift and diffusive electron face
    fluxes included, to the solver tolerance."""
    small = I.cfg1(n=16)
    g = 250.0
    nx, h = 16, small["grid"][3]
    small["te_mode"] = I.TE_ENERGY
    small["phi_bc"] = I.bc([D, D, N, N, N, N], [1000.0, g, 0, 0, 0, 0])
    small["species_bc"] = [I.bc([W, D, N, N, N, N], [0, 0, 0, 0, 0, 0])] * 3
    small["energy_bc"] = I.bc([W, D, N, N, N, N], [0, 0, 0, 0, 0, 0])
    kB = 1.380649e-23
    Ee_s = 1.5 * small["n"][0] * kB * small["Te"]
    big = dict(small)
    nb = nx + 2
    big["grid"] = (nb, 16, 16, h, h, h)
    nbig = np.full((3, 16, 16, nb), 2e15)
    nbig[:, :, :, :nx] = small["n"]
    pbig = np.zeros((16, 16, nb))
    pbig[:, :, nx:] = g
    big["n"], big["phi"] = nbig, pbig
    big["Te"] = np.full((16, 16, nb), small["Te"][0, 0, 0])
    big["phi_bc"] = I.bc([D, N, N, N, N, N], [1000.0, 0, 0, 0, 0, 0])
    big["species_bc"] = [I.bc([W, W, N, N, N, N])] * 3
    big["energy_bc"] = I.bc([W, W, N, N, N, N])
    Ee_b = np.full((16, 16, nb), 7e-3)
    Ee_b[:, :, :nx] = Ee_s
    mask = np.ones((16, 16, nb), np.uint8)
    mask[:, :, nx:] = 0
    sp = oracle.species_ar3()
    kw = dict(poisson=oracle.mg_opts(**TOL_MG), species_mg=oracle.mg_opts(**TOL_MG), energy_mg=oracle.mg_opts(**TOL_MG),
              electron=0, m_bg=39.948 * 1.66053906660e-27)
    rs = oracle.step(small, sp, Ee=Ee_s, **kw)
    rb = oracle.step(big, sp, Ee=Ee_b, mask=mask, **kw)
    assert rs["status"] == 0 and rb["status"] == 0
    for a, b in ((rb["Ee"][:, :, :nx], rs["Ee"]), (rb["Te"][:, :, :nx], rs["Te"]), (rb["n"][0][:, :, :nx], rs["n"][0])):
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    assert np.all(rb["Ee"][:, :, nx:] == 0.0)
    assert np.abs(rs["Ee"] - Ee_s).max() > 1e-6 * np.abs(Ee_s).max()     # the energy really moved
