"""Kinetic gradient of the bed-mean reduction degree (adjoint, dem_grad)
against the oracle's forward-mode dual numbers and against central finite
differences of the HIP forward.

Protocol: n_substeps reaction updates of dt_react, one DEM step and a voidage
deposit before every dyn_every updates, masses frozen.  Gates: FP64 state
J within 1e-11 and each gradient component within 1e-7 of the largest
component of its kind (ln k0 or E_a); FP32 state within 1e-3 (the north-star
gradient bar); finite differences within 1e-3.
"""
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

TH = np.array(W.THETA_HEMATITE_FIT)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _w(name, n, precision="fp64", seed=None):
    kw = {"n": n} if seed is None else {"n": n, "seed": seed}
    w = W.make(name, **kw)
    return W.dataclasses.replace(w, precision=precision)


def _grad_err(g, ref):
    """Per-component error relative to the largest component of its kind."""
    g = np.asarray(g)
    ref = np.asarray(ref)
    s_k = max(np.max(np.abs(ref[0::2])), 1e-300)
    s_e = max(np.max(np.abs(ref[1::2])), 1e-300)
    scale = np.array([s_k, s_e, s_k, s_e, s_k, s_e])
    return float(np.max(np.abs(g - ref) / scale))


# (workload, n, n_substeps, dt_react, dyn_every, ckpt_every): ragged intervals
# and segments, a checkpoint longer than the run, one substep
PROTOCOLS = {
    "cfg2_ragged": ("cfg2", 2000, 205, 0.1, 10, 50),
    "cfg2_deep": ("cfg2", 2000, 205, 0.5, 7, 64),
    "cfg4_onesegment": ("cfg4", 3000, 120, 0.1, 10, 1000),
    "cfg2_single": ("cfg2", 1500, 1, 0.3, 10, 1),
}


@pytest.mark.parametrize("case", list(PROTOCOLS))
def test_grad_fp64_matches_oracle(case):
    name, n, ns, dt, de, ck = PROTOCOLS[case]
    w = _w(name, n)
    _say(f"[adjoint] {case} n={w.n} substeps={ns} dt={dt} dyn_every={de} ckpt={ck}")
    bed = Bed(w)
    J, g = bed.grad(ns, dt, de, ck, TH, state_fp32=False)
    Jo, go = O.Oracle(w).grad(ns, dt, de, TH)
    _say(f"  J {J:.15f} oracle {Jo:.15f}  grad err {_grad_err(g, go):.3e}")
    assert abs(J - Jo) <= 1e-11
    assert _grad_err(g, go) <= 1e-7
    bed.close()


def test_grad_fp32_state_and_mixed_dem():
    """FP32 reaction state with the FP64 adjoint, on a mixed-precision DEM."""
    w = _w("cfg4", 4000, precision="mixed")
    bed = Bed(w)
    J, g = bed.grad(300, 0.1, 10, 100, TH, state_fp32=True)
    Jo, go = O.Oracle(w).grad(300, 0.1, 10, TH)
    _say(f"[adjoint] fp32 state: J {J:.9f} oracle {Jo:.9f} grad err {_grad_err(g, go):.3e}")
    assert abs(J - Jo) <= 1e-5
    assert _grad_err(g, go) <= 1e-3
    bed.close()


def test_grad_vs_finite_differences():
    w = _w("cfg2", 2000, seed=7)
    bed = Bed(w)
    ns, dt, de, ck = 150, 0.2, 10, 40
    J, g = bed.grad(ns, dt, de, ck, TH, state_fp32=False)
    steps = np.array([1e-4, 1.0, 1e-4, 1.0, 1e-4, 1.0])
    fd = np.zeros(6)
    for q in range(6):
        tp = TH.copy()
        tm = TH.copy()
        tp[q] += steps[q]
        tm[q] -= steps[q]
        Jp, _ = bed.grad(ns, dt, de, ck, tp, state_fp32=False, with_grad=False)
        Jm, _ = bed.grad(ns, dt, de, ck, tm, state_fp32=False, with_grad=False)
        fd[q] = (Jp - Jm) / (2 * steps[q])
    _say(f"[adjoint] fd {fd}\n  adj {g}\n  err {_grad_err(g, fd):.3e}")
    assert _grad_err(g, fd) <= 1e-3
    bed.close()


def test_grad_full_size_vs_finite_differences():
    """The 500,000-parcel gradient workload over its whole protocol (20,000
    substeps of 1e-4 s, one DEM step per 10, checkpoints every 500) as the
    benchmark runs it: the FP32-state adjoint against central differences
    (h = 1e-4 relative) of FP64-state forward runs, each component within
    1e-3 of the largest of its kind; J of the FP32 state within 1e-5 of the
    FP64 state's."""
    w = W.cfg4()
    spec = W.grad_spec_cfg4()
    args = (spec["n_substeps"], spec["dt_react"], spec["dyn_every"], spec["ckpt_every"])
    _say(f"[adjoint] full size: n={w.n} substeps={args[0]}")
    bed = Bed(w)
    J, g = bed.grad(*args, TH, state_fp32=True)
    J64, _ = bed.grad(*args, TH, state_fp32=False, with_grad=False)
    fd = np.zeros(6)
    for q in range(6):
        h = 1e-4 * abs(TH[q])
        Jq = []
        for sgn in (1.0, -1.0):
            tq = TH.copy()
            tq[q] += sgn * h
            Jq.append(bed.grad(*args, tq, state_fp32=False, with_grad=False)[0])
        fd[q] = (Jq[0] - Jq[1]) / (2 * h)
    bed.close()
    _say(f"  J {J:.9f} (FP64 state {J64:.9f}); grad err vs FP64 differences {_grad_err(g, fd):.3e}")
    assert abs(J - J64) <= 1e-5
    assert _grad_err(g, fd) <= 1e-3


def test_grad_leaves_state_and_repeats():
    """dem_grad restores the DEM state; a plain forward gives the same J; a
    second call gives the same result bit for bit."""
    w = _w("cfg2", 2000, precision="mixed")
    bed = Bed(w)
    s0 = bed.state()
    J1, g1 = bed.grad(100, 0.2, 10, 30, TH)
    s1 = bed.state()
    for k in ("x", "y", "z", "vx", "vy", "vz", "nh", "nm", "nw", "nfe"):
        assert torch.equal(s0[k], s1[k]), k
    J2, g2 = bed.grad(100, 0.2, 10, 30, TH)
    Jf, _ = bed.grad(100, 0.2, 10, 30, TH, with_grad=False)
    assert J1 == J2 and np.array_equal(g1, g2)
    assert abs(Jf - J1) <= 1e-12
    # the state stays usable: a coupling interval after the gradient runs
    bed.run(2, 20)
    bed.sync()
    bed.close()


def test_grad_bad_spec():
    w = _w("cfg2", 1000)
    bed = Bed(w)
    for args in ((0, 0.1, 10, 10), (10, 0.0, 10, 10), (10, 0.1, 0, 10), (10, 0.1, 10, 0)):
        with pytest.raises(DemError) as e:
            bed.grad(*args, TH)
        assert e.value.code == -1
    with pytest.raises(DemError):
        bed.grad(10, 0.1, 10, 10, [float("nan")] + list(TH[1:]))
    bed.close()


def test_reduction_degree_autograd_function():
    """torch.autograd.Function over dem_grad: J and dJ/dtheta through
    backward() equal a direct dem_grad call; a few gradient steps on ln k0 of
    R3 move J towards a target value."""
    from paper_2311_03908_amd.bed import ReductionDegree

    w = _w("cfg2", 1500, precision="mixed")
    bed = Bed(w)
    spec = dict(n_substeps=60, dt_react=0.2, dyn_every=10, ckpt_every=20, state_fp32=False)
    theta = torch.tensor(TH, dtype=torch.float64, requires_grad=True)
    J = ReductionDegree.apply(theta, bed, spec)
    J.backward()
    Jd, gd = bed.grad(60, 0.2, 10, 20, TH, state_fp32=False)
    assert float(J.detach()) == Jd
    assert np.array_equal(theta.grad.numpy(), gd)
    # calibration as in Section 5.1.1, as gradient descent on (J - target)^2
    target = Jd + 0.02
    th = torch.tensor(TH, dtype=torch.float64, requires_grad=True)
    mask = torch.zeros(6, dtype=torch.float64)
    mask[4] = 1.0  # ln k0 of FeO -> Fe
    loss0 = None
    for _ in range(4):
        Jt = ReductionDegree.apply(th, bed, spec)
        loss = (Jt - target) ** 2
        if loss0 is None:
            loss0 = float(loss.detach())
        th.grad = None
        loss.backward()
        with torch.no_grad():
            th -= 0.5 * mask * th.grad / max(float(th.grad[4] ** 2), 1e-300) * float(loss.detach())
    assert float(loss.detach()) < 0.5 * loss0
    bed.close()
