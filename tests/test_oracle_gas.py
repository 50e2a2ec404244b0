"""Pins of the oracle's gas-species step of the two-way coupling (eq. e3-40
with the semi-implicit sources of eqs. e4-9..e4-11; no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_03908_amd import workloads as W
from tests.util import box_workload


def _bed(u=(0.0, 0.0, 0.0), xh2=0.6, xh2o=0.1):
    w = box_workload([(0.005, 0.005, 0.003), (0.015, 0.015, 0.017)], 5e-4, u=u, xh2=xh2, xh2o=xh2o,
                     L=(0.02, 0.02, 0.02), h=2e-3)
    return w, O.Oracle(w)


def test_inlet_composition_is_steady_without_sources():
    w, ora = _bed(u=(0.0, 0.0, 0.4))
    z = np.zeros(ora.n_cells)
    out = ora.gas_species(1e-4, z, z, (0.6, 0.1))
    for k in ("xH2", "xH2O", "xN2"):
        assert np.allclose(out[k], w.gas[k], rtol=1e-13, atol=0), k


def test_upwind_carries_inlet_composition_up_one_cell_per_courant_unit():
    """A new inlet composition enters the bottom cells at the Courant number
    c = w dt / h: after one step the bottom layer holds the mix c x_in +
    (1 - c) x_old (uniform voidage), the layer above is unchanged."""
    w, ora = _bed(u=(0.0, 0.0, 0.4))
    ora.couple()
    eps = ora.state()["eps"]
    nx, ny, nz = w.beds[0].n
    z = np.zeros(ora.n_cells)
    dt, h = 1e-3, w.beds[0].h
    out = ora.gas_species(dt, z, z, (0.2, 0.3))
    c = 0.4 * dt / h
    x = out["xH2"].reshape(nz, ny, nx)
    e = eps.reshape(nz, ny, nx)
    # bottom cells whose voidage equals that of the gas entering (1 everywhere empty)
    sel = (e[0] == 1.0)
    # mole fractions of the mixed cell: moles from old and inlet gas in proportion (1 - c) : c
    assert np.allclose(x[0][sel], (1 - c) * 0.6 + c * 0.2, rtol=1e-12)
    assert np.allclose(x[2], 0.6, rtol=1e-13)


def test_closed_cell_relaxes_to_network_equilibrium():
    """Without flow the semi-implicit H2 balance of eq. e4-9 has the fixed point
    x_H2 / (x_H2 + x_H2O) = sum(E S) / sum(E Q): the N2-free fraction at which
    the resistance network's net flux vanishes; H atoms are conserved."""
    w, ora = _bed()
    n = ora.n_cells
    eq = np.full(n, -2e-9)
    es = np.full(n, -0.35 * 2e-9)
    g = dict(w.gas)
    V = w.beds[0].h ** 3
    for _ in range(400):
        out = ora.gas_species(5e-3, eq, es, (0.6, 0.1))
        for k in ("xH2", "xH2O", "xN2"):
            g[k] = out[k]
        ora.set_gas(g)
    X = out["xH2"] + out["xH2O"]
    assert np.allclose(out["xH2"] / X, 0.35, rtol=1e-6)
    assert np.allclose(X, 0.7, rtol=1e-12)      # H2 -> H2O one to one in moles
    assert np.allclose(out["xN2"], 0.3, rtol=1e-12)


def test_h2_taken_matches_the_particle_rate_for_a_small_step():
    """For a short step the H2 removed from a closed cell equals dt times the
    particle-side rate of eq. e4-8, -sum(E (Q x - S)) M_H2 p / R per cell."""
    w, ora = _bed()
    n = ora.n_cells
    eq = np.full(n, -3e-10)
    es = np.full(n, -0.5 * 3e-10)
    dt = 1e-7
    ora.couple()
    eps = ora.state()["eps"]
    out = ora.gas_species(dt, eq, es, (0.6, 0.1))
    T, p = w.gas["T"][0], w.gas["p"][0]
    V = w.beds[0].h ** 3
    x, X = 0.6, 0.7
    rate = -(eq[0] * x / X - es[0]) * 2.016e-3 * p / 8.314  # kg/s per cell, H2 taken
    # H2 moles before and after, per unit cell volume (ideal gas, frozen T, p)
    c_tot = p / (8.314 * T)
    taken = eps * c_tot * (0.6 - out["xH2"]) * 2.016e-3 * V  # kg; total moles unchanged (1:1)
    assert np.allclose(taken, rate * dt, rtol=1e-4)


# ------------------------------------------------------------- momentum
def _momentum_bed(v_scale=0.05, u=(0.0, 0.0, 0.5), grad_p=(0.0, 0.0, 0.0)):
    """Parcels without contacts spread over a few gas cells, in random motion."""
    rng = np.random.Generator(np.random.PCG64(12))
    pos = [(0.003 + 0.004 * i, 0.005 + 0.002 * (j % 2), 0.007 + 0.003 * j) for i in range(3) for j in range(3)]
    v = rng.uniform(-v_scale, v_scale, (len(pos), 3))
    w = box_workload(pos, 2.5e-4, k=2.0, u=u, v=v, L=(0.012, 0.012, 0.016), h=2e-3, grad_p=grad_p)
    return w


def _cell_of(w, st):
    b = w.beds[0]
    q = [np.clip(np.floor((st[a] - b.origin[k]) / b.h), 0, b.n[k] - 1).astype(int)
         for k, a in enumerate(("x", "y", "z"))]
    return q[0] + b.n[0] * (q[1] + b.n[1] * q[2])


def test_gas_momentum_balances_the_particle_drag():
    """Newton's third law across the phases: over a short step the gas of
    each cell loses, per unit time, the drag that the particle side's force
    routine applies to the cell's parcels (gravity and pressure gradient
    off, no contacts)."""
    w = _momentum_bed()
    ora = O.Oracle(w, g=(0.0, 0.0, 0.0))
    F, _ = ora.forces()
    st = ora.state()
    cells = _cell_of(w, st)
    sums = ora.couple()
    dt = 1e-10
    new = ora.gas_momentum(dt, sums)
    rho, _ = O.gas_props(1073.0, 101325.0, 1.0, 0.0, 0.0)
    V = w.beds[0].h ** 3
    eps = st["eps"]
    for c in np.unique(cells):
        for a, k in enumerate(("ug", "vg", "wg")):
            gain = eps[c] * rho * V * (new[k][c] - w.gas[k][c]) / dt
            drag = F[cells == c, a].sum()
            assert gain == pytest.approx(-drag, rel=1e-6, abs=1e-12 * np.abs(F).max())
    assert np.abs(F).max() > 0


def test_gas_momentum_relaxes_exponentially_to_the_parcels_velocity():
    """A cell holding parcels, pressure gradient hydrostatic (it cancels the
    gas weight): the exact solution of eps rho du/dt = -(sum K / V)(u - u*)
    relaxes u to u* = sum K v / sum K at the rate r = sum K / (eps rho V).
    Repeated implicit steps converge to it at first order."""
    rho, _ = O.gas_props(1073.0, 101325.0, 1.0, 0.0, 0.0)
    w = _momentum_bed(u=(0.02, -0.01, 0.5), grad_p=(0.0, 0.0, -9.81 * rho))
    ora = O.Oracle(w)
    st = ora.state()
    sums = ora.couple()
    c = int(np.bincount(_cell_of(w, st)).argmax())
    V = w.beds[0].h ** 3
    r = sums["sumK"][c] / (st["eps"][c] * rho * V)
    T = 2.0 / r
    errs = []
    for nsub in (50, 100, 200):
        gas = dict(w.gas)
        ora.set_gas(gas)
        for _ in range(nsub):
            out = ora.gas_momentum(T / nsub, sums)
            gas = {**gas, **out}
            ora.set_gas(gas)
        e = []
        for k, s in (("ug", "sumKu"), ("vg", "sumKv"), ("wg", "sumKw")):
            ustar = sums[s][c] / sums["sumK"][c]
            exact = ustar + (w.gas[k][c] - ustar) * np.exp(-r * T)
            e.append(abs(gas[k][c] - exact) / abs(w.gas[k][c] - ustar))
        errs.append(max(e))
    assert errs[0] < 0.02
    assert errs[1] == pytest.approx(errs[0] / 2, rel=0.05)
    assert errs[2] == pytest.approx(errs[1] / 2, rel=0.05)


def test_gas_momentum_without_parcels():
    """An empty cell accelerates freely, du/dt = g - grad p / rho; with a
    hydrostatic pressure gradient the gas stays at rest."""
    rho, _ = O.gas_props(1073.0, 101325.0, 1.0, 0.0, 0.0)
    w = _momentum_bed(u=(0.0, 0.1, 0.3))
    ora = O.Oracle(w)
    st = ora.state()
    empty = np.setdiff1d(np.arange(ora.n_cells), _cell_of(w, st))
    z = np.zeros(ora.n_cells)
    sums = {"sumK": z, "sumKu": z, "sumKv": z, "sumKw": z}
    dt = 1e-4
    out = ora.gas_momentum(dt, sums)
    assert np.allclose(out["wg"][empty], 0.3 - 9.81 * dt, rtol=1e-13)
    assert np.allclose(out["vg"][empty], 0.1, rtol=1e-13)
    ws = _momentum_bed(u=(0.0, 0.0, 0.0), grad_p=(0.0, 0.0, -9.81 * rho))
    out = O.Oracle(ws).gas_momentum(dt, sums)
    assert np.max(np.abs(out["wg"][empty])) < 1e-15
