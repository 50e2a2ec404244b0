"""Batched execution: beds of uneven size and temperature in one context give,
bit for bit, what each bed gives in a context of its own (per-parcel state,
per-cell sources, bed-mean reduction degree), through the graph-replayed
coupling intervals."""
import sys

import numpy as np
import pytest
import torch

from paper_2311_03908_amd import workloads as W

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_03908_amd.bed import Bed


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def test_batched_equals_per_bed_contexts():
    w = W.with_velocities(W.cfg5(n_beds=5, n_scale=0.05, seed=91), 91)
    _say(f"[batched] {len(w.beds)} beds, {w.n} parcels")
    bed = Bed(w)
    ob = bed.run(3, 20, sources=True, bed_fov=True)
    sb = bed.state()
    bed.close()
    ids = w.parcels["bed"]
    for b in range(len(w.beds)):
        wb = W.split_bed(w, b)
        one = Bed(wb)
        o1 = one.run(3, 20, sources=True, bed_fov=True)
        s1 = one.state()
        one.close()
        sel = torch.as_tensor(np.flatnonzero(ids == b), device=sb["x"].device)
        for k in s1:
            assert torch.equal(s1[k], sb[k][sel]), (b, k)
        c0 = int(w.cell_offset[b])
        c1 = c0 + w.beds[b].n_cells
        for k in o1:
            if k == "bed_fov":
                assert o1[k][0] == ob[k][b], b
            else:
                assert torch.equal(o1[k], ob[k][c0:c1]), (b, k)


def test_empty_bed_in_a_batch():
    """A bed without parcels in a batched context: its cells stay at voidage 1
    with no sources and its bed-mean reduction degree is 0 (the oracle's
    convention); the other beds step exactly as in their own contexts."""
    w = W.with_velocities(W.cfg5(n_beds=3, n_scale=0.05, seed=97), 97)
    keep = w.parcels["bed"] != 1
    p = {k: np.ascontiguousarray(v[keep]) for k, v in w.parcels.items()}
    w = W.dataclasses.replace(w, parcels=p)
    _say(f"[batched] empty middle bed, {w.n} parcels")
    bed = Bed(w)
    ob = bed.run(2, 20, sources=True, bed_fov=True)
    assert ob["bed_fov"][1] == 0.0 and ob["bed_fov"][0] > 0.0 and ob["bed_fov"][2] > 0.0
    c0 = int(w.cell_offset[1])
    c1 = c0 + w.beds[1].n_cells
    eps = bed.couple()["eps"]
    assert torch.all(eps[c0:c1] == 1.0)
    for k in ("mdotH2", "sumK", "np"):
        assert torch.all(ob[k][c0:c1] == 0.0), k
    sb = bed.state()
    ids = w.parcels["bed"]
    for b in (0, 2):
        one = Bed(W.split_bed(w, b))
        one.run(2, 20, sources=True, bed_fov=True)
        s1 = one.state()
        sel = torch.as_tensor(np.flatnonzero(ids == b), device=sb["x"].device)
        for k in ("x", "z", "vz", "nh", "nfe"):
            assert torch.equal(s1[k], sb[k][sel]), (b, k)


@pytest.mark.parametrize("case", ["mixed_batch", "fp64_box"])
def test_results_do_not_depend_on_launch_shapes(case):
    """Two contexts on the same beds, one in the smallest and one in the
    largest launch shapes (dem_set_launch), step bit-identically through
    graph-replayed coupling intervals with neighbour rebuilds; out-of-range
    shapes are rejected and leave the context usable."""
    if case == "mixed_batch":
        w = W.with_velocities(W.squeeze(W.cfg5(n_beds=4, n_scale=0.05, seed=93), 0.97, 0), 93)
    else:
        w = W.with_velocities(W.squeeze(W.cfg1(), 0.995, 0), 94, vscale=0.05, wscale=20.0)
    _say(f"[launch] {case}: {len(w.beds)} beds, {w.n} parcels")
    out = []
    for shape in ((64, 1, 1), (512, 64, 2048)):
        bed = Bed(w)
        bed.set_launch(*shape)
        o = bed.run(3, 20, sources=True, bed_fov=True)
        out.append((bed.state(), o, bed.pairs()))
        bed.close()
    (s0, o0, p0), (s1, o1, p1) = out
    assert np.array_equal(p0, p1) and len(p0) > 0
    for k in s0:
        assert torch.equal(s0[k], s1[k]), k
    for k in o0:
        if k == "bed_fov":
            assert np.array_equal(o0[k], o1[k])
        else:
            assert torch.equal(o0[k], o1[k]), k
    bed = Bed(w)
    for bad in ((96, 1, 1), (64, 0, 1), (64, 65, 1), (64, 1, 0)):
        with pytest.raises(Exception):
            bed.set_launch(*bad)
    bed.run(1, 20)
    bed.close()
