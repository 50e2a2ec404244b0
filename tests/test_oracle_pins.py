"""Pins of the oracle's drag law, gas viscosity and reduction degree against
results fixed outside the paper's own formulas (no GPU):

- the dense branch of the drag (eq. e3-5-1, eps < 0.8) reproduces Ergun's
  packed-bed pressure drop through the fixed-bed force balance;
- the dilute branch reproduces the Richardson-Zaki expansion law of a
  homogeneous bed in the viscous limit (which fixes its voidage exponent)
  and the standard drag curve of a single sphere (which fixes its C_D);
- the viscosity correlation of Table C2 (eqs. e3-55, e3-56) gives the
  textbook viscosities of the pure gases;
- the overall reduction degree of eqs. e2-18 / e2-19 is the fraction of
  the ore's oxygen removed.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.util import golden

TB = golden("textbook_values.json")
G = 9.81


# ------------------------------------------------------------- dense branch: Ergun
def _ergun_dp_per_l(eps, U, rho, mu, d):
    """Ergun (1952): pressure drop per bed length at superficial velocity U."""
    e = TB["ergun_packed_bed"]
    return (e["A"] * mu * U * (1 - eps) ** 2 / (eps ** 3 * d ** 2)
            + e["B"] * rho * U ** 2 * (1 - eps) / (eps ** 3 * d))


def _model_dp_per_l(eps, U, rho, mu, d, printed=0):
    """The same fixed bed in the two-fluid model: the steady gas momentum
    balance 0 = -eps grad p - beta (u_g - v) with v = 0 and the interstitial
    gas velocity u_g = U / eps gives -grad p = beta U / eps^2."""
    beta = O.beta_over_epsp(eps, rho, mu, U / eps, d, printed) * (1.0 - eps)
    return beta * U / eps ** 2


@pytest.mark.parametrize("eps", [0.4, 0.7])
@pytest.mark.parametrize("U", [0.05, 2.0])
def test_dense_drag_reproduces_ergun_pressure_drop(eps, U):
    """Viscous and inertial terms both matter at U = 2 m/s (their ratio is
    about 1.5 for 1 mm spheres in air); the viscous term dominates at 0.05."""
    rho, mu, d = 1.2, 1.8e-5, 1e-3
    assert _model_dp_per_l(eps, U, rho, mu, d) == pytest.approx(_ergun_dp_per_l(eps, U, rho, mu, d), rel=1e-12)


def test_printed_inertial_term_misses_ergun():
    """The inertial term as printed in eq. e3-5-1 (eps_g instead of eps_p)
    does not give Ergun's pressure drop; Gidaspow's form (the reading used)
    does, so the pin decides between the two."""
    eps, U, rho, mu, d = 0.4, 2.0, 1.2, 1.8e-5, 1e-3
    ref = _ergun_dp_per_l(eps, U, rho, mu, d)
    assert abs(_model_dp_per_l(eps, U, rho, mu, d, printed=1) / ref - 1.0) > 0.1


# ------------------------------------------------------------- dilute branch
def _drag_force(eps, slip, rho, mu, d):
    """Drag on one sphere of diameter d at interstitial slip (eq. e3-5)."""
    return O.beta_over_epsp(eps, rho, mu, slip, d) * (math.pi / 6 * d ** 3) * slip


def _slip_for_force(eps, F, rho, mu, d):
    lo, hi = 0.0, 1.0
    while _drag_force(eps, hi, rho, mu, d) < F:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _drag_force(eps, mid, rho, mu, d) < F:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("eps", [0.85, 0.9, 0.95])
def test_dilute_drag_reproduces_richardson_zaki(eps):
    """Homogeneous fluidization of uniform spheres in the viscous limit.  The
    pressure gradient carries the mixture, -grad p = (eps rho_g + eps_p
    rho_p) g, so the drag on a particle balances eps (rho_p - rho_g) V g; at
    eps = 1 that is the terminal velocity u_t.  With the superficial gas
    velocity U = eps s (s the interstitial slip), U / u_t must follow
    Richardson and Zaki's eps^4.65."""
    rho_p, rho, mu, d = 4000.0, 0.2, 4e-5, 3e-6
    W = (rho_p - rho) * math.pi / 6 * d ** 3 * G
    u_t = _slip_for_force(1.0, W, rho, mu, d)
    assert rho * u_t * d / mu < 1e-5  # viscous limit (the finite-Re correction of C_D is below 1e-4)
    U = eps * _slip_for_force(eps, eps * W, rho, mu, d)
    n = TB["richardson_zaki_low_re_exponent"]["n"]
    assert U / u_t == pytest.approx(eps ** n, rel=1e-4)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_dilute_drag_follows_standard_sphere_curve(q):
    """A single sphere (eps = 1): C_D = F / (rho s^2 / 2 * pi d^2 / 4) at
    Re = rho d s / mu of 1, 10 and 100 against the standard drag curve."""
    ref = TB["sphere_standard_drag_curve"]
    Re, cd_ref = ref["Re"][q], ref["C_D"][q]
    rho, mu, d = 1.2, 1.8e-5, 1e-4
    s = Re * mu / (rho * d)
    cd = _drag_force(1.0, s, rho, mu, d) / (0.5 * rho * s * s * math.pi * d * d / 4)
    assert cd == pytest.approx(cd_ref, rel=ref["rel_tol"])


def test_dilute_drag_newton_regime():
    """Above Re = 1000 the sphere drag coefficient is the Newton value 0.44."""
    rho, mu, d = 1.2, 1.8e-5, 1e-3
    for Re in (2000.0, 1e5):
        s = Re * mu / (rho * d)
        cd = _drag_force(1.0, s, rho, mu, d) / (0.5 * rho * s * s * math.pi * d * d / 4)
        assert cd == pytest.approx(0.44, rel=1e-12)


# ------------------------------------------------------------- viscosity
@pytest.mark.parametrize("gas,T", [("H2", 300), ("H2", 1000), ("N2", 300), ("N2", 1000), ("H2O", 1000)])
def test_pure_gas_viscosity_textbook(gas, T):
    ref = TB["pure_gas_viscosity_Pa_s"]
    x = {"H2": (1.0, 0.0, 0.0), "H2O": (0.0, 1.0, 0.0), "N2": (0.0, 0.0, 1.0)}[gas]
    _, mu = O.gas_props(float(T), 101325.0, *x)
    tol = ref["rel_tol"].get(f"{gas}_{T}", ref["rel_tol"]["default"])
    assert mu == pytest.approx(ref[gas][str(T)], rel=tol)


def test_viscosity_rises_with_temperature_and_mixes_by_mass():
    """Gas viscosity grows with T; the mixture rule of eq. e3-56 weights the
    pure-gas values by mass fraction (a mixture of equal mass fractions sits
    midway between its pure gases, far from the mole-weighted value)."""
    for x in ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)):
        mus = [O.gas_props(T, 101325.0, *x)[1] for T in (700.0, 900.0, 1100.0, 1300.0)]
        assert all(a < b for a, b in zip(mus, mus[1:]))
    M = (2.016, 28.013)
    xh = (0.5 / M[0]) / (0.5 / M[0] + 0.5 / M[1])
    mu_h = O.gas_props(1000.0, 101325.0, 1.0, 0.0, 0.0)[1]
    mu_n = O.gas_props(1000.0, 101325.0, 0.0, 0.0, 1.0)[1]
    mu_mix = O.gas_props(1000.0, 101325.0, xh, 0.0, 1.0 - xh)[1]
    assert mu_mix == pytest.approx(0.5 * (mu_h + mu_n), rel=1e-12)
    assert abs(mu_mix - (xh * mu_h + (1 - xh) * mu_n)) > 0.2 * mu_mix


# ------------------------------------------------------------- reduction degree
def test_reduction_degree_of_pure_phases():
    """Hematite ore (eq. e2-18): Fe3O4 carries 8/9 of Fe2O3's oxygen per Fe,
    FeO 6/9, Fe none; magnetite ore (eq. e2-19): FeO carries 3/4 of Fe3O4's."""
    N = 6.0  # Fe atoms
    hem = {"Fe2O3": ((N / 2, 0, 0, 0), 0.0), "Fe3O4": ((0, N / 3, 0, 0), 1 / 9), "FeO": ((0, 0, N, 0), 1 / 3),
           "Fe": ((0, 0, 0, N), 1.0)}
    for name, (sp, f) in hem.items():
        assert O.fov(sp, 0) == pytest.approx(f, abs=1e-15), name
    mag = {"Fe3O4": ((0, N / 3, 0, 0), 0.0), "FeO": ((0, 0, N, 0), 0.25), "Fe": ((0, 0, 0, N), 1.0)}
    for name, (sp, f) in mag.items():
        assert O.fov(sp, 1) == pytest.approx(f, abs=1e-15), name


def test_reduction_degree_is_oxygen_removed():
    """Any mixture: f_ov = 1 - O / O_ref, O = 3 n_h + 4 n_m + n_w, with
    O_ref = 3/2 N_Fe for hematite ore and 4/3 N_Fe for magnetite ore (no
    Fe2O3 in it)."""
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(200):
        sp = rng.uniform(0.0, 1.0, 4) * (rng.uniform(size=4) > 0.2)
        if sp.sum() == 0:
            continue
        nfe = 2 * sp[0] + 3 * sp[1] + sp[2] + sp[3]
        o = 3 * sp[0] + 4 * sp[1] + sp[2]
        assert O.fov(sp, 0) == pytest.approx(1.0 - o / (1.5 * nfe), abs=1e-14)
        sm = sp.copy()
        sm[0] = 0.0
        if sm.sum() == 0:
            continue
        nfe = 3 * sm[1] + sm[2] + sm[3]
        o = 4 * sm[1] + sm[2]
        assert O.fov(sm, 1) == pytest.approx(1.0 - o / (4.0 / 3.0 * nfe), abs=1e-14)
