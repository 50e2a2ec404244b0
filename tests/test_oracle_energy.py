"""Pins of the oracle's particle energy equation (eqs. e3-8..e3-13,
e3-18..e3-23, e3-41, e3-49, e3-50, e4-4, e4-5; Tables C1, C3) against
textbook thermochemistry, closed forms and conservation (no GPU)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_03908_amd import workloads as W
from tests.util import box_workload

H2, H2O, N2, FE2O3, FE3O4, FEO, FE = range(7)
MOLAR = {H2: 2.016e-3, H2O: 18.015e-3, N2: 28.013e-3}


def test_formation_enthalpies_at_298():
    """H(298.15 K) of eq. e3-22 is the standard enthalpy of formation
    (NIST-JANAF, kJ/mol): 0 for the elements, -241.83 H2O(g), -824.2 Fe2O3,
    -1118.4 Fe3O4, -272.0 FeO."""
    ref = {H2: 0.0, H2O: -241.83, N2: 0.0, FE2O3: -824.2, FE3O4: -1118.4, FEO: -272.0, FE: 0.0}
    for sp, h in ref.items():
        assert O.h_mol(sp, 298.15) / 1e3 == pytest.approx(h, abs=1.0), sp


def test_heat_capacities_at_298():
    """C_p(298.15 K) of eq. e3-23 against NIST-JANAF (J/(mol K))."""
    ref = {H2: 28.84, H2O: 33.58, N2: 29.12, FE2O3: 103.9, FE3O4: 150.7, FEO: 49.9, FE: 25.1}
    for sp, c in ref.items():
        assert O.cp_mol(sp, 298.15) == pytest.approx(c, rel=0.015), sp
    # per unit mass for the gases (eq. e3-57 with one species): 14.3 kJ/(kg K) H2, 1.04 N2
    assert O.cp_g(298.15, 1.0, 0.0, 0.0) == pytest.approx(14300.0, rel=0.005)
    assert O.cp_g(298.15, 0.0, 0.0, 1.0) == pytest.approx(1040.0, rel=0.005)


@pytest.mark.parametrize("sp", range(7))
def test_enthalpy_is_continuous_and_integrates_cp(sp):
    """dH/dT = C_p everywhere (central differences), H continuous across the
    range bounds, C_p positive from 300 K to 1600 K."""
    for T in np.linspace(400.5, 1600.5, 121):  # off the range bounds, where C_p steps
        d = 1e-3
        dh = (O.h_mol(sp, T + d) - O.h_mol(sp, T - d)) / (2 * d)
        assert dh == pytest.approx(O.cp_mol(sp, T), rel=1e-5, abs=1e-4), (sp, T)
        assert O.cp_mol(sp, T) > 0.0
    for Tb in (850.0, 960.0, 1000.0, 1042.0, 1184.0):
        assert abs(O.h_mol(sp, Tb + 1e-7) - O.h_mol(sp, Tb - 1e-7)) < 1e-3, (sp, Tb)


def _dH(r, T):
    h = lambda sp: O.h_mol(sp, T)
    if r == 0:
        return 2 * h(FE3O4) + h(H2O) - 3 * h(FE2O3) - h(H2)
    if r == 1:
        return 3 * h(FEO) + h(H2O) - h(FE3O4) - h(H2)
    return h(FE) + h(H2O) - h(FEO) - h(H2)


def test_reaction_enthalpies_follow_table1():
    """Table 1: R1 exothermic, R2 and R3 endothermic, at the temperatures the
    beds of Table 3 run (hematite 973-1073 K, magnetite 903-943 K), with the
    textbook magnitudes (R2 about +30..+75, R3 about +15..+30 kJ/mol)."""
    for T in (973.0, 1023.0, 1073.0):
        assert _dH(0, T) < 0.0, T
    for T in (903.0, 923.0, 943.0, 973.0, 1023.0, 1073.0):
        assert 25e3 < _dH(1, T) < 75e3, T
        assert 15e3 < _dH(2, T) < 30e3, T
    # at 298.15 K the values follow from the formation enthalpies alone
    assert _dH(2, 298.15) / 1e3 == pytest.approx(-241.83 + 272.0, abs=1.0)


def test_gas_conductivity_values():
    """Table C3 at 1000 K against textbook conductivities (W/(m K)): H2
    about 0.45, N2 about 0.065; the mixture is mass-weighted (eq. e3-59)."""
    assert O.lambda_g(1000.0, 1.0, 0.0, 0.0) == pytest.approx(0.45, rel=0.05)
    assert O.lambda_g(1000.0, 0.0, 0.0, 1.0) == pytest.approx(0.065, rel=0.05)
    lh, ln = O.lambda_g(1000.0, 1.0, 0.0, 0.0), O.lambda_g(1000.0, 0.0, 0.0, 1.0)
    Yh = 0.5 * 2.016 / (0.5 * 2.016 + 0.5 * 28.013)
    assert O.lambda_g(1000.0, 0.5, 0.0, 0.5) == pytest.approx(Yh * lh + (1 - Yh) * ln, rel=1e-12)


def test_nusselt_limits():
    """eq. e3-12: a lone sphere in still gas (eps = 1, Re = 0) conducts with
    Nu = 2; convection raises it."""
    assert O.nusselt(1.0, 0.0, 0.7) == pytest.approx(2.0, rel=1e-14)
    assert O.nusselt(0.5, 0.0, 0.7) == pytest.approx(7 - 5 + 1.25, rel=1e-14)
    assert O.nusselt(0.9, 10.0, 0.7) > O.nusselt(0.9, 1.0, 0.7) > O.nusselt(0.9, 0.0, 0.7)


def _lone(Tp_offset, species, k=2.0, dp=1e-4, T=1073.0, dt=1e-5):
    ore = W.Ore(xi0=1.0 - 4500.0 / W.RHO_TRUE[0], d_pore_cm=3.3e-6)
    w = box_workload([(0.011, 0.011, 0.011)], k * dp, k=k, ore=ore, u=(0.0, 0.0, 0.0), T=T,
                     dt=dt, energy_on=1)
    for key, v in zip(("nh", "nm", "nw", "nfe"), species):
        w.parcels[key] = np.array([v])
    return W.with_energy(w, dT=Tp_offset)


def test_lone_parcel_relaxes_to_gas_temperature():
    """A parcel of iron (no reaction) at rest in still gas: m C_p dT/dt =
    k^3 Nu lambda_g pi d_p (T_g - T_p) with Nu = 7 - 10 eps + 5 eps^2, whose
    explicit-Euler steps shrink T_g - T_p by (1 - dt/tau) each."""
    k, dp, T, dt = 2.0, 1e-4, 1073.0, 1e-5
    w = _lone(-5.0, (0.0, 0.0, 0.0, 1e-9), k=k, dp=dp, T=T, dt=dt)
    ora = O.Oracle(w, g=(0.0, 0.0, 0.0))
    st = ora.state()
    d = float(w.parcels["d"][0])
    dpr = d / k
    eps = 1.0 - math.pi / 6 * d ** 3 / 2e-3 ** 3
    Nu = 7 - 10 * eps + 5 * eps ** 2
    hA = k ** 3 * Nu * O.lambda_g(T, 1.0, 0.0, 0.0) / dpr * math.pi * dpr ** 2
    mcp = k ** 3 * 1e-9 * O.cp_mol(FE, T - 5.0)
    assert st["mcp"][0] == pytest.approx(mcp, rel=1e-14)
    n = 50
    ora.step(n)
    expect = T - 5.0 * (1 - dt * hA / mcp) ** n
    assert ora.state()["Tp"][0] == pytest.approx(expect, rel=1e-13)
    # the deposit of eqs. e4-4 / e4-5 (times V_cell) sees the same k^3 h A
    out = ora.react(1e-4)
    c = np.flatnonzero(out["hA"])
    assert c.size == 1
    assert out["hA"][c[0]] == pytest.approx(hA, rel=1e-13)
    assert out["hAT"][c[0]] == pytest.approx(hA * ora.state()["Tp"][0], rel=1e-13)
    assert out["Qrm"][c[0]] == 0.0 and out["Hr"][c[0]] == 0.0


def test_reaction_heat_is_reaction_enthalpy():
    """A wustite parcel (R3 only): k^3 (Q_r + Q_rm) = -k^3 dH_R3(T_p) xi3 / dt
    with xi3 the iron formed; R3 is endothermic, so the parcel cools; at
    T_p = T_g the gas-side terms of eqs. e3-38 and e3-39 cancel."""
    k, T, dt = 2.0, 1073.0, 1e-3
    w = _lone(0.0, (0.0, 0.0, 2e-10, 0.0), k=k, T=T)
    ora = O.Oracle(w, g=(0.0, 0.0, 0.0))
    out = ora.react(dt)
    st = ora.state()
    xi3 = st["nfe"][0]
    assert xi3 > 0
    q = -k ** 3 * _dH(2, T) * xi3 / dt
    assert st["qrx"][0] == pytest.approx(q, rel=1e-12)
    assert st["qrx"][0] < 0.0
    c = np.flatnonzero(out["Hr"])[0]
    assert out["Qrm"][c] == pytest.approx(-out["Hr"][c], rel=1e-14)
    # and the next steps apply it: dT = dt_DEM (k^3 h A (T_g - T_p) + q) / (m C_p)
    T0 = st["Tp"][0]
    ora.step(1)
    expect = T0 + w.params["dt"] * q / st["mcp"][0]
    assert ora.state()["Tp"][0] == pytest.approx(expect, rel=1e-14)


def test_isothermal_parcels_react_as_without_energy():
    """With T_p = T_g the reaction update is the isothermal one, bit for bit."""
    w0 = W.with_velocities(W.cfg1(n=400, seed=5), 5)
    w1 = W.with_energy(w0, 0.0)
    a, b = O.Oracle(w0), O.Oracle(w1)
    ra, rb = a.react(1e-3), b.react(1e-3)
    assert np.array_equal(ra["fov"], rb["fov"])
    for k in ("mdotH2", "mdotH2O", "sumEQ", "sumES"):
        assert np.array_equal(ra[k], rb[k]), k


def test_hotter_parcels_reduce_faster():
    """Kinetics at the particle temperature: the same bed 30 K hotter than
    its gas reduces faster; 30 K colder, slower."""
    w = W.cfg1(n=400, seed=6)
    f = [O.Oracle(W.with_energy(w, dT)).react(1e-2)["fov"].mean() for dT in (-30.0, 0.0, 30.0)]
    assert f[0] < f[1] < f[2]


def test_energy_sums_conserve_deposits():
    """Every parcel's k^3 h A lands in its cell: sum over cells of hA equals the
    per-parcel sum, and with uniform T_p the H1 deposit is T_p times H0."""
    w = W.with_energy(W.with_velocities(W.cfg1(n=600, seed=8), 8), 0.0)
    w.gas["T"][:] = 1073.0
    w.parcels["Tp"][:] = 1050.0
    ora = O.Oracle(w)
    out = ora.react(1e-4)
    assert np.allclose(out["hAT"], 1050.0 * out["hA"], rtol=1e-14, atol=0)
    assert np.all(out["hA"][out["hA"] != 0] > 0)
    occ = np.zeros(ora.n_cells, bool)
    occ[np.flatnonzero(ora.couple()["np"])] = True
    assert np.array_equal(out["hA"] > 0, occ)
