"""Batched execution: beds of uneven size and temperature in one context give,
bit for bit, what each bed gives in a context of its own (per-parcel state,
per-cell sources, bed-mean reduction degree), through the graph-replayed
coupling intervals."""
import json
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
    """Contexts on the same beds in different launch shapes (dem_set_launch:
    step block, XCD chunk, build grid; dem_set_build: build block size, LDS
    tile, work-item width) step bit-identically through graph-replayed
    coupling intervals with neighbour rebuilds; out-of-range shapes are
    rejected and leave the context usable."""
    if case == "mixed_batch":
        w = W.with_velocities(W.squeeze(W.cfg5(n_beds=4, n_scale=0.05, seed=93), 0.97, 0), 93)
    else:
        w = W.with_velocities(W.squeeze(W.cfg1(), 0.995, 0), 94, vscale=0.05, wscale=20.0)
    _say(f"[launch] {case}: {len(w.beds)} beds, {w.n} parcels")
    out = []
    shapes = (((64, 1, 1), (256, 1024, 8)), ((512, 64, 2048), (1024, 4096, 32)), ((128, 4, 0), (512, 2048, 16)),
              ((256, 16, 0), (256, 2048, 32)))
    for launch, build in shapes:
        bed = Bed(w)
        bed.set_launch(*launch)
        bed.set_build(*build)
        o = bed.run(3, 20, sources=True, bed_fov=True)
        st = bed.stats()
        assert (st["build_threads"], st["build_tile"], st["build_item_x"]) == build
        out.append((bed.state(), o, bed.pairs()))
        bed.close()
    s0, o0, p0 = out[0]
    assert len(p0) > 0
    for s1, o1, p1 in out[1:]:
        assert np.array_equal(p0, p1)
        for k in s0:
            assert torch.equal(s0[k], s1[k]), k
        for k in o0:
            if k == "bed_fov":
                assert np.array_equal(o0[k], o1[k])
            else:
                assert torch.equal(o0[k], o1[k]), k
    bed = Bed(w)
    for bad in ((96, 1, 1), (64, 0, 1), (64, 65, 1), (64, 1, -1)):
        with pytest.raises(Exception):
            bed.set_launch(*bad)
    for bad in ((512, 1024, 16), (512, 2048, 12), (128, 2048, 16)):
        with pytest.raises(Exception):
            bed.set_build(*bad)
    bed.run(1, 20)
    bed.close()


def test_autotune_leaves_state_and_springs_unchanged():
    """dem_autotune times step candidates (full steps whose springs and
    contact masks go to spare buffers) and whole forced rebuild chains on the
    context's own data: the state and the contact springs it leaves are the
    ones it found, bit for bit."""
    w = W.with_velocities(W.squeeze(W.cfg3(n=20000, seed=23), 0.98, 0), 95, vscale=0.03, wscale=20.0)
    _say(f"[autotune] state and springs, n={w.n}")
    bed = Bed(w)
    bed.step(40)
    s0, c0 = bed.state(), bed.contacts()
    assert len(c0["ids"]) > 100
    bed.autotune()
    s1, c1 = bed.state(), bed.contacts()
    for k in s0:
        assert torch.equal(s0[k], s1[k]), k
    o0, o1 = np.lexsort(c0["ids"].T[::-1]), np.lexsort(c1["ids"].T[::-1])
    assert np.array_equal(c0["ids"][o0], c1["ids"][o1])
    assert np.array_equal(c0["xi"][o0], c1["xi"][o1])
    assert np.array_equal(c0["wall_on"], c1["wall_on"])
    assert np.array_equal(c0["wall_xi"], c1["wall_xi"])
    bed.close()


def test_autotuner_cache_keyed_by_arch_and_config(tmp_path, monkeypatch):
    """dem_autotune with DEMRX_TUNE_CACHE: the first context times the
    candidates and stores its choice under the key of the device architecture
    and configuration; a second context of the same configuration applies the
    stored shapes without timing; another configuration is tuned anew."""
    path = tmp_path / "tune.json"
    monkeypatch.setenv("DEMRX_TUNE_CACHE", str(path))
    shape_keys = ("step_block", "step_xcd", "build_threads", "build_tile", "build_item_x")
    w = W.with_velocities(W.squeeze(W.cfg1(), 0.995, 0), 95)
    _say(f"[tune] {w.n} parcels")
    a = Bed(w)
    a.autotune()
    sa = a.stats()
    a.close()
    assert sa["tune_cached"] == 0
    doc = json.loads(path.read_text())
    assert len(doc) == 1
    (key, val), = doc.items()
    assert key.startswith("gfx") and f"|n={w.n}|" in key
    assert (val["step_block"], val["step_xcd"], val["build_threads"], val["build_tile"], val["item_x"]) == \
        tuple(sa[k] for k in shape_keys)
    b = Bed(w)
    b.autotune()
    sb = b.stats()
    b.run(2, 20)
    b.close()
    assert sb["tune_cached"] == 1
    assert all(sb[k] == sa[k] for k in shape_keys)
    w2 = W.with_velocities(W.cfg5(n_beds=2, n_scale=0.05, seed=96), 96)
    c = Bed(w2)
    c.autotune()
    assert c.stats()["tune_cached"] == 0
    c.close()
    assert len(json.loads(path.read_text())) == 2
