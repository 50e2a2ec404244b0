"""Input generators: shapes and invariants of the seeded workloads (no GPU)."""
import numpy as np
import pytest

from paper_2311_03908_amd import workloads as W


def test_split_bed_partitions_parcels_and_cells():
    w = W.cfg5(n_beds=7, n_scale=0.03, seed=3)
    parts = [W.split_bed(w, b) for b in range(len(w.beds))]
    assert sum(p.n for p in parts) == w.n
    assert sum(p.n_cells for p in parts) == w.n_cells
    for b, p in enumerate(parts):
        sel = np.flatnonzero(w.parcels["bed"] == b)
        assert np.array_equal(p.parcels["x"], w.parcels["x"][sel])
        assert np.all(p.parcels["bed"] == 0)
        c0 = int(w.cell_offset[b])
        assert np.array_equal(p.gas["T"], w.gas["T"][c0:c0 + w.beds[b].n_cells])


def test_cfg3_is_a_fixed_bed_without_overlaps_at_start():
    w = W.cfg3(n=20_000)
    assert w.params["kn"] == 200.0
    assert np.allclose(w.gas["wg"][w.gas["wg"] != 0], 0.01, rtol=0.11)
    d = w.parcels["d"]
    # radii FP32-representable (the exact contact test uses them unchanged)
    assert np.array_equal(d.astype(np.float32).astype(np.float64), d)


def test_sweep_beds_follow_table3():
    """Bed I / Bed II shapes of Table 3 at a small scale: real particle counts
    over k^3, ore kinds and sphericities, initial mass fractions, gas
    composition and pressure, and the per-bed kinetic sets."""
    n_scale = 0.002
    w = W.sweep(n_scale=n_scale)
    assert len(w.beds) == len(W.SWEEP_BEDS)
    mag, hem = w.ores
    assert (mag.kind, mag.psi, hem.kind, hem.psi) == (W.ORE_MAGNETITE, 0.85, W.ORE_HEMATITE, 0.86)
    for b, (kind, T, u, theta) in enumerate(W.SWEEP_BEDS):
        sel = w.parcels["bed"] == b
        k = 2.8 if kind == "I" else 3.0
        real = 5_140_800 if kind == "I" else 5_095_837
        assert sel.sum() == round(real / k ** 3 * n_scale)
        assert np.all(w.parcels["ore"][sel] == (0 if kind == "I" else 1))
        assert np.allclose(w.parcels["k"][sel], k)
        dp = w.parcels["d"][sel].astype(np.float64) / k
        assert dp.mean() == pytest.approx(1e-4 if kind == "I" else 3.5e-4, rel=0.02)
        assert w.beds[b].theta == tuple(theta)
        c0 = int(w.cell_offset[b])
        c1 = c0 + w.beds[b].n_cells
        assert np.all(w.gas["T"][c0:c1] == T)
        assert np.all(w.gas["xH2"][c0:c1] == (0.7 if kind == "I" else 0.65))
        assert np.all(w.gas["p"][c0:c1] == (101325.0 if kind == "I" else 110000.0))
        # mass fractions of the ore (Table 3) from the initial moles
        nh, nm, nw = (w.parcels[q][sel] for q in ("nh", "nm", "nw"))
        m = nh * 159.687 + nm * 231.531 + nw * 71.844
        if kind == "I":
            assert np.allclose(nm * 231.531 / m, 0.6994) and np.all(nh == 0)
        else:
            assert np.allclose(nh * 159.687 / m, 0.9628) and np.all(nm == 0)
    assert np.exp(W.THETA_MAGNETITE_FIT[2]) == pytest.approx(8.0)
    assert np.exp(W.THETA_MAGNETITE_FIT[4]) == pytest.approx(6000.0)
