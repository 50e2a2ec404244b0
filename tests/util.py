"""Small hand-built workloads for the pins and parity tests (inputs only)."""
import dataclasses
import json
import math
import os

import numpy as np

from paper_2311_03908_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def box_workload(pos, d_p, k=1.0, rho=4500.0, L=(0.02, 0.02, 0.02), h=2e-3, v=None, w=None,
                 precision="fp64", ore=None, gas=None, wall=W.WALL_BOX, R=0.0, theta=W.THETA_HEMATITE_FIT,
                 mu_override=4e-5, T=1073.0, xh2=1.0, xh2o=0.0, u=(0.0, 0.0, 0.5), grad_p=(0, 0, 0),
                 wt=None, **params):
    """A single bed holding the given parcels (positions in m, real diameters d_p)."""
    pos = np.asarray(pos, float).reshape(-1, 3)
    n = pos.shape[0]
    d_p = np.broadcast_to(np.asarray(d_p, float), (n,)).astype(np.float32).astype(np.float64)
    nx = [max(1, int(round(L[i] / h))) for i in range(3)]
    Lr = [nx[i] * h for i in range(3)]
    hi = (Lr[0], Lr[1], L[2] if wall == W.WALL_CYL else Lr[2])
    bed = W.Bed(wall, (0.0, 0.0, 0.0), hi, R, (0.0, 0.0, 0.0), h, tuple(nx), 1, tuple(theta),
                mu_override=mu_override)
    ore = ore or W.Ore(xi0=1.0 - rho / W.RHO_TRUE[0], d_pore_cm=3.3e-6)
    rho_eff = (1.0 - ore.xi0) * ore.rho_true[0]
    wt = wt or (W.HEMATITE_WT if ore.kind == W.ORE_HEMATITE else W.MAGNETITE_WT)
    parcels = W._parcels(pos, d_p, k, np.zeros(n), np.zeros(n), {0: rho_eff}, {0: wt})
    if precision == "mixed":
        pass
    if v is not None:
        v = np.asarray(v, float).reshape(-1, 3)
        parcels["vx"], parcels["vy"], parcels["vz"] = [np.ascontiguousarray(v[:, i]) for i in range(3)]
    if w is not None:
        w = np.asarray(w, float).reshape(-1, 3)
        parcels["wx"], parcels["wy"], parcels["wz"] = [np.ascontiguousarray(w[:, i]) for i in range(3)]
    rng = np.random.Generator(np.random.PCG64(0))
    g = gas or W._gas(rng, [bed], T, xh2, xh2o, u, 0.0, False, grad_p=grad_p)
    prm = W.base_params(**params)
    return W.Workload("custom", precision, prm, [bed], [ore], parcels, g, np.array([0]), 0, 10)


def rel_err(a, b, floor):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)) if a.size else 0.0
