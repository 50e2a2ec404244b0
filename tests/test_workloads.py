"""Input generators: shapes and invariants of the seeded workloads (no GPU)."""
import numpy as np

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
