"""Particle energy equation on the GPU (through the C-ABI) against the FP64
oracle: reaction heats, heat capacities and heat sums at identical state,
particle temperatures over coupled intervals (eager and graph-replayed), and
batched beds against single-bed contexts.

Gates: heat sums and reduction at identical state within 1e-12 relative (FP64
on both sides); particle temperatures after 60 DEM steps and 3 reaction
updates within 1e-8 K (FP64 path) and 1e-4 K (mixed path, FP32 velocities and
heat-transfer coefficients)."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2311_03908_amd import workloads as W
from paper_2311_03908_amd.capi import DemError

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_03908_amd.bed import Bed


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


CASES = {
    "cfg1_fp64": lambda: W.with_energy(W.with_velocities(W.squeeze(W.cfg1(), 0.995, 0), 31, vscale=0.05,
                                                         wscale=20.0), -40.0, seed=31, spread=15.0),
    "cfg2_mixed": lambda: W.with_energy(W.with_velocities(W.squeeze(W.cfg2(n=3000, seed=32), 0.995, 0), 32,
                                                          vscale=0.03, wscale=20.0), -40.0, seed=32, spread=15.0),
}


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", list(CASES))
def test_reaction_heat_and_sums_at_identical_state(case):
    w = CASES[case]()
    _say(f"[energy/react] {case} n={w.n}")
    bed = Bed(w)
    ora = O.Oracle(w)
    bed.couple()
    ora.couple()
    dt = 20 * w.params["dt"]
    for it in range(2):
        rg = bed.react(dt)
        ro = ora.react(dt)
        assert np.max(np.abs(_np(rg["fov"]) - ro["fov"])) <= 1e-11, it
        for k in ("mdotH2", "mdotH2O", "sumEQ", "sumES", "hA", "hAT", "Qrm", "Hr"):
            e = _rel(_np(rg[k]), ro[k])
            _say(f"  {k}: {e:.2e}")
            assert e <= 1e-12, (it, k, e)
    assert np.max(np.abs(ro["Hr"])) > 0 and np.max(ro["hA"]) > 0


@pytest.mark.parametrize("case", list(CASES))
def test_temperatures_over_coupled_intervals(case):
    """Three intervals of 20 DEM steps and a reaction update: each parcel's
    T_p against the oracle's."""
    w = CASES[case]()
    mixed = w.precision == "mixed"
    _say(f"[energy/trajectory] {case} n={w.n}")
    bed = Bed(w)
    ora = O.Oracle(w)
    dt = 20 * w.params["dt"]
    T0 = w.parcels["Tp"].copy()
    for _ in range(3):
        bed.step(20)
        ora.step(20)
        bed.couple()
        ora.couple()
        bed.react(dt)
        ora.react(dt)
    sg, so = bed.state(), ora.state()
    err = np.abs(_np(sg["Tp"]) - so["Tp"])
    moved = np.abs(so["Tp"] - T0)
    _say(f"  max |dT| {moved.max():.3f} K, max err {err.max():.2e} K")
    assert moved.max() > 0.02  # the parcels heat up measurably
    assert err.max() <= (1e-4 if mixed else 1e-8)


def test_graph_replay_matches_eager_with_energy():
    w = CASES["cfg2_mixed"]()
    a, b = Bed(w), Bed(w)
    oa = a.run(4, 20, sources=True, bed_fov=True)
    for _ in range(4):
        b.step(20)
        b.couple()
        ob = b.react(20 * w.params["dt"], keys=("mdotH2", "mdotH2O", "sumEQ", "sumES", "hA", "hAT", "Qrm", "Hr"))
    sa, sb = a.state(), b.state()
    assert torch.equal(sa["Tp"], sb["Tp"])
    for k in ("hA", "hAT", "Qrm", "Hr"):
        assert torch.equal(oa[k], ob[k]), k
    assert oa["bed_fov"][0] == ob["bed_fov"][0]


def test_batched_beds_with_energy_equal_single_beds():
    w = W.with_energy(W.with_velocities(W.cfg5(n_beds=4, n_scale=0.05, seed=93), 93), -30.0, seed=93, spread=10.0)
    bed = Bed(w)
    ob = bed.run(3, 20, sources=True, bed_fov=True)
    sb = bed.state()
    ids = w.parcels["bed"]
    for b in range(len(w.beds)):
        one = Bed(W.split_bed(w, b))
        o1 = one.run(3, 20, sources=True, bed_fov=True)
        s1 = one.state()
        sel = torch.as_tensor(np.flatnonzero(ids == b), device=sb["x"].device)
        assert torch.equal(s1["Tp"], sb["Tp"][sel]), b
        c0 = int(w.cell_offset[b])
        c1 = c0 + w.beds[b].n_cells
        for k in ("hA", "hAT", "Qrm", "Hr"):
            assert torch.equal(o1[k], ob[k][c0:c1]), (b, k)


def test_set_state_temperature_and_isothermal_gradient_only():
    w = CASES["cfg2_mixed"]()
    bed = Bed(w)
    st = {k: _np(v) for k, v in bed.state().items()}
    st["Tp"] = st["Tp"] + 7.0
    bed.set_state(st)
    assert np.array_equal(_np(bed.state()["Tp"]), st["Tp"])
    with pytest.raises(DemError) as e:
        bed.grad(10, 0.1, 10, 10, W.THETA_HEMATITE_FIT)
    assert e.value.code == -1


def test_energy_full_size_cylinder_bed():
    """The 200,000-parcel cylinder bed with the energy equation on, in the
    autotuned launch shapes: heat sums at identical state within 1e-12
    relative, then T_p after three intervals of 20 steps and a reaction
    update within the mixed-path bar (1e-4 K)."""
    w = W.with_energy(W.with_velocities(W.squeeze(W.cfg2(), 0.985, 0), 33, vscale=0.03, wscale=20.0),
                      -40.0, seed=33, spread=15.0)
    _say(f"[energy] full size n={w.n}")
    bed = Bed(w)
    bed.autotune()
    ora = O.Oracle(w)
    dt = 20 * w.params["dt"]
    bed.couple()
    ora.couple()
    rg, ro = bed.react(dt), ora.react(dt)
    for k in ("hA", "hAT", "Qrm", "Hr"):
        assert _rel(_np(rg[k]), ro[k]) <= 1e-12, k
    T0 = w.parcels["Tp"].copy()
    for _ in range(3):
        bed.step(20)
        ora.step(20)
        bed.couple()
        ora.couple()
        bed.react(dt)
        ora.react(dt)
    err = np.abs(_np(bed.state()["Tp"]) - ora.state()["Tp"])
    moved = np.abs(ora.state()["Tp"] - T0)
    _say(f"  max |dT| {moved.max():.3f} K, max err {err.max():.2e} K")
    assert moved.max() > 0.02
    assert err.max() <= 1e-4
    bed.close()
