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
