"""Pins of the oracle's transport, chemistry and electron-energy terms.

Every expected value here comes from outside the oracle: the rate and
mobility expressions of Appendix A evaluated at stated conditions and
stored as numbers (tests/golden/), or closed-form solutions of reduced
cases of the step (uniform states, linear profiles) in which the electron
energy equation (Sec. 2.1, Eqs. (5)-(8)) collapses to an algebraic update.
A transcription mistake in a rate coefficient, a mobility, the reduced
field, the Joule, elastic or wall terms changes one of these numbers.
"""
import os

import numpy as np
import pytest

from paper_2507_08200_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
PHYS = {"qe": 1.602176634e-19, "eps0": 8.8541878128e-12, "kB": 1.380649e-23, "me": 9.1093837015e-31}
AMU = 1.66053906660e-27
N_GAS = 2.4463e25       # 1 atm, 300 K
M_AR = 39.948 * AMU


def _golden_rows(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


# --------------------------------------------------------------------------
# Appendix A, Tables A.1-A.3: all 33 rate expressions at 2, 5 and 30 eV
# --------------------------------------------------------------------------
RATE_ROWS = _golden_rows("arh2_rates.txt")


@pytest.mark.parametrize("row", RATE_ROWS, ids=["%s@%seV" % (r[0], r[1]) for r in RATE_ROWS])
def test_rate_table_value(oracle, row):
    q = int(row[0][1:])
    te_ev = float(row[1])
    want = float(row[2])
    got = oracle.rates_arh2(te_ev * I.EV_IN_K)[q - 1]
    # the stored values have 10 significant digits; the largest exponent
    # (R2 at 2 eV, -299) amplifies a last-bit difference of the argument
    # to ~1e-13 relative
    assert abs(got - want) <= 2e-9 * abs(want), (row, got)


def test_rate_table_covers_every_reaction():
    seen = {(r[0], r[1]) for r in RATE_ROWS}
    assert len(seen) == 33 * 3
    assert {r[0] for r in RATE_ROWS} == {"R%d" % q for q in range(1, 34)}


# --------------------------------------------------------------------------
# Table A.4: the species list and its transport
# --------------------------------------------------------------------------
SPECIES_ROWS = _golden_rows("table_a4_species.txt")
_KIND = {"electron": 1, "ion": 2, "neutral": 3}
_WALL = {"none": 0, "electron": 1, "ion": 2, "neutral": 3}


def test_species_table_matches_table_a4(oracle):
    sp = oracle.species_arh2_15()
    assert len(sp) == len(SPECIES_ROWS) == 15
    for s, row in zip(sp, SPECIES_ROWS):
        name, Z, kind, c, _partner, mass_u, wall = row
        assert s["Z"] == float(Z), name
        assert s["mob_kind"] == _KIND[kind], name
        assert s["wall_kind"] == _WALL[wall], name
        if kind == "electron":
            assert s["mass"] == PHYS["me"]
        else:
            assert s["mob_coef"] == float(c), name
            assert abs(s["mass"] - float(mass_u) * AMU) <= 1e-15 * s["mass"], name


# Hand values at N = 2.4463e25 m^-3, Tg = 300 K, Te = 2 eV (23209.036 K),
# E/N = 100 Td: |mu| = c N0/N with N0/N = 2.68/2.4463 = 1.0955320; D from
# the Einstein relation with kB Tg/e = 0.025851999 V (ions and, through the
# counterpart, neutrals) or kB Te/e = 1.9999999790 V (electrons).
# Electron fit at 100 Td: ln 100 = 4.6051702; tanh(0.289*4.6051702 + 0.543)
# = tanh(1.8738942) = 0.95394586; exp(0.05481 - 2.911*0.95394586)
# = 0.06573510; * 1.1296e25/2.4463e25 = 0.030353620.
TRANSPORT_HAND = {
    1.85e-4: (2.026734252e-04, 5.239513344e-06),
    1.835e-4: (2.010301271e-04, 5.197030804e-06),
    30e-4: (3.286596084e-03, 8.496508126e-05),
    25.0e-4: (2.738830070e-03, 7.080423438e-05),
    32.0e-4: (3.505702489e-03, 9.062942001e-05),
    19.0e-4: (2.081510853e-03, 5.381121813e-05),
}
MU_E_100TD = 3.035362050e-02
D_E_100TD_2EV = 6.070724036e-02


def test_transport_hand_values(oracle):
    te = 2.0 * I.EV_IN_K
    for s, row in zip(oracle.species_arh2_15(), SPECIES_ROWS):
        mu, D = oracle.transport(s, 100.0, te, 300.0, N_GAS)
        if row[2] == "electron":
            assert abs(mu + MU_E_100TD) <= 1e-9 * MU_E_100TD
            assert abs(D - D_E_100TD_2EV) <= 1e-9 * D_E_100TD_2EV
            continue
        m_want, d_want = TRANSPORT_HAND[float(row[3])]
        if row[2] == "ion":
            assert abs(mu - m_want) <= 1e-9 * m_want, row
        else:
            assert mu == 0.0, row
        assert abs(D - d_want) <= 1e-9 * d_want, row


def test_transport_constant_model(oracle):
    s = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": -0.03, "D_const": 0.06}
    assert oracle.transport(s, 250.0, 5e4, 300.0, N_GAS) == (-0.03, 0.06)


def test_electron_fit_reduced_field_floor(oracle):
    """E/N below 1e-3 Td is floored there before the log (a reading)."""
    assert oracle.mu_electron(0.0, N_GAS) == oracle.mu_electron(1e-3, N_GAS)
    assert oracle.mu_electron(1e-5, N_GAS) == oracle.mu_electron(1e-3, N_GAS)


# --------------------------------------------------------------------------
# Reduced field, Joule heating and elastic loss in a uniform field
# --------------------------------------------------------------------------
def _plates_cfg(n, h, V, te_mode, *, species_x, energy_x, ne, Ee=None, Te_K=2.0 * I.EV_IN_K,
                sp_values=(0,) * 6, en_values=(0,) * 6):
    """Two plates at x = 0 (V) and x = L (0), periodic in y and z; an
    electron and an ion species of equal density (no space charge)."""
    nz = ny = 4
    return {"grid": (n, ny, nz, h, h, h), "mech": 0, "n": np.stack([ne, ne]),
            "phi": np.zeros((nz, ny, n)), "Te": np.full((nz, ny, n), Te_K), "te_mode": te_mode,
            "phi_bc": I.bc([0, 0, 3, 3, 3, 3], (V, 0, 0, 0, 0, 0)),
            "species_bc": [I.bc(species_x + [3, 3, 3, 3], sp_values)] * 2,
            "energy_bc": I.bc(energy_x + [3, 3, 3, 3], en_values),
            "dt": 1e-12, "n_t": 1, "Tg": 300.0, "N_gas": N_GAS, "bg": []}


def _fit_electron():
    return {"Z": -1, "mass": PHYS["me"], "mob_kind": 1, "wall_kind": 1}


def _still_ion():
    return {"Z": 1, "mass": M_AR, "mob_kind": 0, "wall_kind": 0, "mu_const": 0.0, "D_const": 0.0}


def test_uniform_field_energy_closed_form(oracle):
    """Uniform plasma between plates, periodic species and energy: the
    potential is the linear plate solution, E = V/L, E/N = 100 Td, so the
    electron mobility is the fit's hand value; every flux divergence is zero
    and one step of the energy equation is the algebraic update
    Ee1 = Ee0 + dt (e |mu_e| n E^2 - 1.5 n kB (Te - Tg) (2 me / mb) e / (me |mu_e|))
    (Joule heating by the drift flux, elastic loss; Eq. (8), no chemistry)."""
    n, h = 8, 1e-4
    L = n * h
    E = 100.0 * 1e-21 * N_GAS
    V = E * L
    ne0, Te0 = 1e18, 2.0 * I.EV_IN_K
    Ee0 = 1.5 * ne0 * PHYS["kB"] * Te0
    cfg = _plates_cfg(n, h, V, I.TE_ENERGY, species_x=[3, 3], energy_x=[3, 3], ne=np.full((4, 4, n), ne0))
    cfg["dt"] = dt = 2e-11
    tight = oracle.mg_opts(rtol=1e-14, max_cycles=2000)
    r = oracle.step(cfg, [_fit_electron(), _still_ion()], Ee=np.full((4, 4, n), Ee0), m_bg=M_AR,
                    poisson=tight, energy_mg=tight, species_mg=tight)
    assert r["status"] == 0
    mu = MU_E_100TD
    joule = PHYS["qe"] * mu * ne0 * E * E
    nu = PHYS["qe"] / (PHYS["me"] * mu)
    elastic = 1.5 * ne0 * PHYS["kB"] * (Te0 - 300.0) * (2 * PHYS["me"] / M_AR) * nu
    Ee1 = Ee0 + dt * (joule - elastic)
    assert 0.2 < (Ee1 - Ee0) / Ee0 < 2.0         # the source is resolved, not buried in Ee0
    np.testing.assert_allclose(r["Ee"], Ee1, rtol=1e-9)
    np.testing.assert_allclose(r["Te"], Ee1 / (1.5 * ne0 * PHYS["kB"]), rtol=1e-9)
    np.testing.assert_allclose(r["n"], ne0, rtol=1e-13)


def test_uniform_field_local_field_temperature(oracle):
    """Same plates in local-field mode: Te is the table at E/N = 100 Td in
    every cell.  The stand-in table 0.02585 + 5.47 (E/N / 300 Td)^0.6 eV
    gives 2.8559 eV at 100 Td (linear interpolation in ln(E/N) between its
    nodes changes that by < 1e-4)."""
    n, h = 8, 1e-4
    E = 100.0 * 1e-21 * N_GAS
    cfg = _plates_cfg(n, h, E * n * h, I.TE_LFA, species_x=[3, 3], energy_x=[3, 3],
                      ne=np.full((4, 4, n), 1e16))
    cfg["lfa"] = I.lfa_table()
    tight = oracle.mg_opts(rtol=1e-14, max_cycles=2000)
    r = oracle.step(cfg, [_fit_electron(), _still_ion()], poisson=tight, species_mg=tight)
    assert r["status"] == 0
    hand_ev = 0.02585 + 5.47 * (1.0 / 3.0) ** 0.6
    np.testing.assert_allclose(r["Te"] / I.EV_IN_K, hand_ev, rtol=1e-4)
    np.testing.assert_allclose(r["Te"], oracle.te_lfa(cfg["lfa"], 100.0), rtol=1e-12)


def test_energy_wall_flux_closed_form(oracle):
    """No field, no energy diffusion, walls at x = 0 and L: each wall cell
    loses dt/h times the energy wall flux 2 kB Te n/4 sqrt(8 kB Te/(pi me))
    (Eq. (15)) besides the elastic loss every cell has; interior cells lose
    only the elastic part."""
    n, h = 8, 1e-4
    ne0, Te0 = 1e18, 3.0 * I.EV_IN_K
    Ee0 = 1.5 * ne0 * PHYS["kB"] * Te0
    cfg = _plates_cfg(n, h, 0.0, I.TE_ENERGY, species_x=[2, 2], energy_x=[2, 2], ne=np.full((4, 4, n), ne0))
    e = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": -0.03, "D_const": 0.0}
    tight = oracle.mg_opts(rtol=1e-14, max_cycles=2000)
    r = oracle.step(cfg, [e, _still_ion()], Ee=np.full((4, 4, n), Ee0), m_bg=M_AR,
                    poisson=tight, energy_mg=tight, species_mg=tight)
    assert r["status"] == 0
    nu = PHYS["qe"] / (PHYS["me"] * 0.03)
    elastic = 1.5 * ne0 * PHYS["kB"] * (Te0 - 300.0) * (2 * PHYS["me"] / M_AR) * nu
    wall = 2 * PHYS["kB"] * Te0 * ne0 / 4 * np.sqrt(8 * PHYS["kB"] * Te0 / (np.pi * PHYS["me"]))
    interior = Ee0 - 1e-12 * elastic
    edge = interior - 1e-12 * wall / h
    assert (Ee0 - edge) > 3 * (Ee0 - interior)  # the wall term dominates at the wall
    np.testing.assert_allclose(r["Ee"][:, :, 1:-1], interior, rtol=1e-13)
    np.testing.assert_allclose(r["Ee"][:, :, 0], edge, rtol=1e-13)
    np.testing.assert_allclose(r["Ee"][:, :, -1], edge, rtol=1e-13)


def test_joule_with_diffusive_flux_linear_density(oracle):
    """Electron density linear in x between Dirichlet values, uniform field:
    WENO5 reproduces linear data exactly and the central difference gives
    the exact gradient, so the cell electron flux is mu n_c E - D s (s the
    density slope) and the Joule term is -e (mu n_c E - D s) E.  With a
    uniform Ee held at its value on Dirichlet faces the energy drift has no
    divergence, and the step's Ee must satisfy the implicit energy equation
    (1/dt - div(5/3 D grad)) Ee1 = Ee0/dt + Joule - elastic exactly; checked
    through the (eigenmode-pinned) discrete operator."""
    n, h = 16, 5e-5
    L = n * h
    V = 400.0
    E = V / L
    mu, D = -0.03, 0.08
    g0, g1 = 2e17, 6e17
    X, _, _ = I.cell_centres(n, 4, 4, h, h, h)
    s = (g1 - g0) / L
    ne = g0 + s * X
    Ee0 = 1.5 * 4e17 * PHYS["kB"] * 2.0 * I.EV_IN_K
    cfg = _plates_cfg(n, h, V, I.TE_ENERGY, species_x=[0, 0], energy_x=[0, 0], ne=ne,
                      sp_values=(g0, g1, 0, 0, 0, 0), en_values=(Ee0, Ee0, 0, 0, 0, 0))
    e = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": mu, "D_const": D}
    tight = oracle.mg_opts(rtol=1e-14, max_cycles=2000)
    Ee_in = np.full(ne.shape, Ee0)
    r = oracle.step(cfg, [e, dict(e, Z=1, wall_kind=2)], Ee=Ee_in, m_bg=M_AR,
                    poisson=tight, energy_mg=tight, species_mg=tight)
    assert r["status"] == 0
    joule = -PHYS["qe"] * (mu * ne * E - D * s) * E
    nu = PHYS["qe"] / (PHYS["me"] * abs(mu))
    Te = Ee0 / (1.5 * ne * PHYS["kB"])
    elastic = 1.5 * ne * PHYS["kB"] * (Te - 300.0) * (2 * PHYS["me"] / M_AR) * nu
    rhs = Ee0 / 1e-12 + joule - elastic
    # the diffusive part of the flux is visible in the source
    assert np.abs(PHYS["qe"] * D * s * E).min() > 1e-3 * np.abs(joule).max()
    prob = {"grid": cfg["grid"], "bc": cfg["energy_bc"], "alpha_c": 1e12, "beta_c": 5.0 / 3.0 * D}
    res = oracle.residual(prob, rhs, r["Ee"])
    assert np.abs(res).max() <= 1e-12 * np.abs(rhs).max()
    # and the field really moved the energy by the Joule term
    assert np.abs(r["Ee"] - Ee0).max() > 1e-3 * Ee0


# --------------------------------------------------------------------------
# Reaction source: rates of progress and electron energy loss of isolated
# reaction groups (Tables A.1-A.3; the loss uses the energy column)
# --------------------------------------------------------------------------
E_, ARP, AR2P, HP, H2P, H3P, ARHP, ARS, AR2S, V1, V2, V3, H_, AR, H2 = range(15)


# at 5 eV every energetic reaction's term is within a few decades of the
# others of its group (at 2 eV R2 is 1e-101 of R1 and its energy would not
# show)
def _k5ev():
    return {int(r[0][1:]): float(r[2]) for r in RATE_ROWS if r[1] == "5.0"}


def _source_of(oracle, present):
    n = np.zeros((15, 1))
    for s, v in present.items():
        n[s, 0] = v
    G, Sin = oracle.reaction_source(I.MECH_ARH2_15, n, np.array([5.0 * I.EV_IN_K]))
    return G[:, 0], Sin[0]


def _close(got, want, what):
    # the stored rates carry 10 significant digits
    assert abs(got - want) <= 1e-9 * abs(want), (what, got, want)


def test_isolated_electron_argon(oracle):
    """Only e and Ar: R1 (excitation, 11.6 eV) and R2 (ionization, 15.759 eV)."""
    k = _k5ev()
    ne, nar = 1e18, 2.3e25
    G, S = _source_of(oracle, {E_: ne, AR: nar})
    qe = PHYS["qe"]
    _close(S, qe * ne * nar * (11.6 * k[1] + 15.759 * k[2]), "S_inel")
    _close(G[ARS], k[1] * ne * nar, "Ar*")
    _close(G[ARP], k[2] * ne * nar, "Ar+")
    _close(G[E_], k[2] * ne * nar, "e")
    _close(G[AR], -(k[1] + k[2]) * ne * nar, "Ar")


def test_isolated_three_body_ion_conversion(oracle):
    """Only Ar+ and Ar: R9, Ar+ + 2Ar -> Ar2+ + Ar, rate k9 n_Ar+ n_Ar^2."""
    k = _k5ev()
    ni, nar = 1e18, 2.3e25
    G, S = _source_of(oracle, {ARP: ni, AR: nar})
    r = k[9] * ni * nar * nar
    _close(G[AR2P], r, "Ar2+")
    _close(G[ARP], -r, "Ar+")
    _close(G[AR], -r, "Ar")
    assert S == 0.0


def test_isolated_excimer(oracle):
    """Only Ar2*: R10 (Ar2* -> 2Ar, 1/s) and R11 (2 Ar2* -> Ar2+ + 2Ar + e)."""
    k = _k5ev()
    n = 3e19
    G, S = _source_of(oracle, {AR2S: n})
    _close(G[AR2S], -k[10] * n - 2 * k[11] * n * n, "Ar2*")
    _close(G[AR2P], k[11] * n * n, "Ar2+")
    _close(G[E_], k[11] * n * n, "e")
    _close(G[AR], 2 * k[10] * n + 2 * k[11] * n * n, "Ar")
    assert S == 0.0


def test_isolated_electron_hydrogen(oracle):
    """Only e and H2: R15 (14.68 eV), R17 (15.4 eV), R18 (28.08 eV) and the
    vibrational excitations R24-R26 (no energy printed)."""
    k = _k5ev()
    ne, nh2 = 1e18, 1.2e24
    G, S = _source_of(oracle, {E_: ne, H2: nh2})
    p = ne * nh2
    _close(S, PHYS["qe"] * p * (14.68 * k[15] + 15.4 * k[17] + 28.08 * k[18]), "S_inel")
    _close(G[H_], p * (2 * k[15] + k[18]), "H")
    _close(G[HP], p * k[18], "H+")
    _close(G[H2P], p * k[17], "H2+")
    _close(G[E_], p * (k[17] + k[18]), "e")
    _close(G[V1], p * k[24], "H2(v1)")
    _close(G[V2], p * k[25], "H2(v2)")
    _close(G[V3], p * k[26], "H2(v3)")
    _close(G[H2], -p * (k[15] + k[17] + k[18] + k[24] + k[25] + k[26]), "H2")


def test_isolated_electron_metastable(oracle):
    """Only e and Ar*: R3 (step ionization, 4.159 eV), R4 (pooling), R5
    (quenching)."""
    k = _k5ev()
    ne, ns = 1e18, 5e19
    G, S = _source_of(oracle, {E_: ne, ARS: ns})
    _close(S, PHYS["qe"] * 4.159 * k[3] * ne * ns, "S_inel")
    _close(G[ARP], k[3] * ne * ns + k[4] * ns * ns, "Ar+")
    _close(G[ARS], -k[3] * ne * ns - 2 * k[4] * ns * ns - k[5] * ns * ne, "Ar*")
    _close(G[AR], k[4] * ns * ns + k[5] * ns * ne, "Ar")


def test_isolated_recombination(oracle):
    """Only e and Ar+: R12 (radiative, k12 n+ ne) and R13 (three-body,
    k13 n+ ne^2)."""
    k = _k5ev()
    ne, ni = 1e19, 2e19
    G, S = _source_of(oracle, {E_: ne, ARP: ni})
    _close(G[ARS], k[12] * ni * ne + k[13] * ni * ne * ne, "Ar*")
    _close(G[E_], -k[12] * ni * ne - k[13] * ni * ne * ne, "e")
    assert S == 0.0


@pytest.mark.parametrize("partner,rxn,dE", [(H_, 16, 13.6), (AR2S, 6, 4.2)])
def test_isolated_single_ionization_energy(oracle, partner, rxn, dE):
    """e + H (R16, 13.6 eV) and e + Ar2* (R6 read as Ar2+ + 2e, 4.2 eV;
    R7 dissociates without an energy)."""
    k = _k5ev()
    ne, nn = 1e18, 4e19
    G, S = _source_of(oracle, {E_: ne, partner: nn})
    _close(S, PHYS["qe"] * dE * k[rxn] * ne * nn, "S_inel")


def test_isolated_molecular_ion_dissociation(oracle):
    """Only e and H2+: R19 (H+ + H + e, 12.68 eV) and R22 (2H)."""
    k = _k5ev()
    ne, ni = 1e18, 3e18
    G, S = _source_of(oracle, {E_: ne, H2P: ni})
    _close(S, PHYS["qe"] * 12.68 * k[19] * ne * ni, "S_inel")
    _close(G[H_], ne * ni * (k[19] + 2 * k[22]), "H")
    _close(G[H2P], -ne * ni * (k[19] + k[22]), "H2+")


def test_energy_temperature_clamped_at_gas_temperature(oracle):
    """Te = Ee / (1.5 ne kB) is clamped below at Tg (a reading)."""
    n, h = 8, 1e-4
    ne0 = 1e16
    Ee0 = 1.5 * ne0 * PHYS["kB"] * 100.0       # 100 K < Tg
    cfg = _plates_cfg(n, h, 0.0, I.TE_ENERGY, species_x=[3, 3], energy_x=[3, 3], ne=np.full((4, 4, n), ne0))
    e = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": -0.03, "D_const": 0.0}
    r = oracle.step(cfg, [e, _still_ion()], Ee=np.full((4, 4, n), Ee0), m_bg=M_AR,
                    poisson=oracle.mg_opts(rtol=1e-14, max_cycles=2000))
    assert r["status"] == 0
    assert np.all(r["Te"] == 300.0)


# --------------------------------------------------------------------------
# Face flux Gamma = mu n E - D grad n (Eq. (2)) on every face
# --------------------------------------------------------------------------
def test_face_flux_linear_density_closed_form(oracle):
    """Linear density between Dirichlet values in a uniform field: WENO5 is
    exact on linear data (its ghosts continue the line), the central
    difference gives the exact slope, so every x face carries
    mu E n(x_f) - D s and the y, z faces nothing."""
    nx, ny, nz, h = 12, 4, 6, 1e-4
    L = nx * h
    V, mu, D = 30.0, -0.03, 0.07
    g0, g1 = 1e17, 5e17
    X, _, _ = I.cell_centres(nx, ny, nz, h, h, h)
    s = (g1 - g0) / L
    u = g0 + s * X
    phi = V * (1 - X / L)
    pbc = I.bc([0, 0, 3, 3, 3, 3], (V, 0, 0, 0, 0, 0))
    ubc = I.bc([0, 0, 3, 3, 1, 1], (g0, g1, 0, 0, 0, 0))
    sp = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": mu}
    fx, fy, fz = oracle.face_flux((nx, ny, nz, h, h, h), pbc, ubc, sp, u, phi, np.full(u.shape, mu),
                                  np.full(u.shape, D), np.full(u.shape, 2e4), 300.0)
    xf = np.arange(nx + 1) * h
    want = mu * (V / L) * (g0 + s * xf) - D * s
    scale = np.abs(want).max()
    assert np.abs(fx - want[None, None, :]).max() <= 1e-12 * scale
    assert np.abs(fy).max() <= 1e-12 * scale
    assert np.abs(fz).max() <= 1e-12 * scale


def test_face_flux_wall_faces(oracle):
    """Uniform density, no field: interior faces carry nothing; a WALLFLUX
    face carries the Maxwellian electron flux outwards (negative along +x
    at x = 0, positive at x = L) and no diffusion."""
    nx, ny, nz, h = 8, 4, 4, 1e-4
    n0, Te = 3e16, 3.0 * I.EV_IN_K
    u = np.full((nz, ny, nx), n0)
    ubc = I.bc([2, 2, 3, 3, 3, 3])
    sp = {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1, "mu_const": -0.03}
    fx, fy, fz = oracle.face_flux((nx, ny, nz, h, h, h), I.bc([0, 0, 3, 3, 3, 3]), ubc, sp, u, np.zeros(u.shape),
                                  np.full(u.shape, -0.03), np.full(u.shape, 0.1), np.full(u.shape, Te), 300.0)
    fl = n0 / 4 * np.sqrt(8 * PHYS["kB"] * Te / (np.pi * PHYS["me"]))
    np.testing.assert_allclose(fx[:, :, 0], -fl, rtol=1e-14)
    np.testing.assert_allclose(fx[:, :, -1], fl, rtol=1e-14)
    assert np.all(fx[:, :, 1:-1] == 0) and np.all(fy == 0) and np.all(fz == 0)


def test_step_check_mode_reproduces_the_solver_residuals(oracle):
    """The check mode (potential given, species iterates given) recomputes
    the relative residuals the solves stopped on: a converged oracle step
    checks below its tolerance, a perturbed density does not."""
    cfg = I.cfg1(n=16)
    sp = oracle.species_ar3()
    opts = oracle.mg_opts(rtol=1e-10)
    r = oracle.step(cfg, sp, poisson=opts, species_mg=opts)
    assert r["status"] == 0
    c = oracle.step(cfg, sp, phi=r["phi"], phi_fixed=True, check_n=r["n"], poisson=opts, species_mg=opts)
    assert c["status"] == 0
    assert abs(c["info"]["poisson_rel"] - r["info"]["poisson_rel"]) <= 1e-3 * r["info"]["poisson_rel"]
    assert np.all(c["check_res"][:3] <= 1e-10 * 1.001)
    np.testing.assert_array_equal(c["n"], r["n"])
    bad = r["n"].copy()
    bad[1, 8, 8, 8] *= 1.0 + 1e-6
    c2 = oracle.step(cfg, sp, phi=r["phi"], phi_fixed=True, check_n=bad, poisson=opts, species_mg=opts)
    assert c2["check_res"][1] > 1e-9 and c2["check_res"][0] <= 1.001e-10
