"""Seeded synthetic inputs shaped like the paper's fluidized-bed workloads.

This module only *constructs inputs*: parcel positions, sizes, ore labels,
initial composition, per-cell frozen gas fields and the physical/numerical
parameters of each workload.  It performs none of the method's arithmetic
(no contact law, drag, diffusion, kinetics or network solve) and is shared by
the test-suite, the oracle driver and the GPU driver alike.

Workloads (all seeded with ``numpy.random.Generator(PCG64(seed))``):

* ``cfg1`` -- 2,048 hematite parcels, d = 1 mm +-5 %, k = 1, rho = 4500 kg/m3,
  random sequential addition in a closed 16x16x64 mm box, pure H2 at 1073 K,
  uniform 0.5 m/s upflow on an 8x8x32 grid, fixed viscosity 4e-5 Pa s,
  dt = 1e-5 s, coupling every 10 steps, FP64 everywhere.
* ``cfg2`` -- 200,000 parcels, d_p = 150 um +-20 %, k = 3 (Bed II ore of the
  paper's Table 3: xi0 = 0.34, rho = 3500), cylinder 40 mm x 200 mm, grid
  32x32x160 (1.25 mm) with a seeded +-10 % perturbation on 0.3 m/s upflow,
  90 % H2 + N2 at 973 K, dt = 5e-6 s, mixed precision.
* ``cfg3`` -- 2,000,000 parcels, lognormal d_p (median 100 um, sigma 0.3,
  truncated at 3 sigma), k = 5, two hematite ore types 50/50 (xi0 0.05 / 0.25,
  pore diameter 3.3e-6 / 9.5e-6 cm), cylinder 100 mm x 600 mm on a 64x64x384
  grid, pure H2 at 1073 K with 0.01 m/s upflow (a fixed bed), kn = 200 N/m,
  dt = 5e-6 s, mixed precision.
* ``cfg4`` -- 500,000 parcels with cfg2 statistics at 1073 K (adjoint bed).
* ``cfg5`` -- 64 beds, N_b log-uniform in [5000, 80000], cfg1 parcels in boxes
  scaled to hold them, an 8x8 factorial over T (973-1173 K) and H2 fraction
  (0.6-1.0, N2 balance), dt = 5e-6 s, mixed precision.

Any workload can be shrunk with ``n=...``: the container is scaled by
``(n/N)^(1/3)`` at fixed cell size so the packing density is unchanged.

Placement: the dilute box beds (cfg1, cfg5) use random sequential addition
without overlap over the whole box.  The cylindrical beds (cfg2-4) start as a
packed bed, as the paper's bubbling beds do before fluidization: parcels are
split into size classes and stacked from the floor up in horizontal layers
that cycle through the classes; each layer is a square lattice whose pitch is
the largest parcel of its class plus a 2 % gap, with each parcel jittered
inside its own lattice cube (so no two parcels overlap and neighbours are
nearly touching); original ids are then shuffled so id order carries no
spatial information.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Any

import numpy as np

# Molar masses (kg/mol), used here only to express an initial ore composition
# given in mass fractions as moles per real particle.
_MOLAR_MASS = {"Fe2O3": 159.687e-3, "Fe3O4": 231.531e-3, "FeO": 71.844e-3, "Fe": 55.845e-3}

RHO_TRUE = (5300.0, 5180.0, 5390.0, 7900.0)  # Fe2O3, Fe3O4, FeO, Fe (Table 3)
HEMATITE_WT = {"Fe2O3": 0.9628, "FeO": 0.0372}  # Bed II ore (Table 3)
MAGNETITE_WT = {"Fe3O4": 0.6994, "FeO": 0.3006}  # Bed I ore (Table 3)

# Fitted hematite kinetics of the paper's Section 5.2: k0 = 10, 7e-4, 0.022 m/s,
# Ea = 42.4, 19.3, 33.88 kJ/mol.  Parameter vector (ln k0_i, Ea_i), i = R1..R3.
THETA_HEMATITE_FIT = (math.log(10.0), 42400.0, math.log(7e-4), 19300.0, math.log(0.022), 33880.0)
# Takenaka constants of Table 2 (used by magnetite-ore tests).
THETA_TABLE2 = (math.log(29.17), 66974.0, math.log(15.56), 75345.0, math.log(2858.0), 117204.0)

WALL_BOX = 0
WALL_CYL = 1
ORE_HEMATITE = 0
ORE_MAGNETITE = 1


@dataclasses.dataclass
class Bed:
    wall: int                  # WALL_BOX or WALL_CYL
    lo: tuple                  # box corner (m); for a cylinder the bounding box
    hi: tuple
    R: float                   # cylinder radius (m), axis at the xy centre of lo/hi
    origin: tuple              # gas grid origin (m)
    h: float                   # gas cell edge (m)
    n: tuple                   # gas cells per axis
    refine: int                # DEM cells per gas-cell edge (1 or 2)
    theta: tuple               # (ln k0_i, Ea_i) for R1..R3
    mu_override: float = 0.0   # >0: gas viscosity fixed to this value (Pa s)

    @property
    def n_cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


@dataclasses.dataclass
class Ore:
    xi0: float                 # initial particle porosity
    d_pore_cm: float           # pore diameter d_a (cm)
    tau: float = 2.0           # tortuosity
    kind: int = ORE_HEMATITE
    rho_true: tuple = RHO_TRUE
    psi: float = 0.0           # sphericity: 0 spheres, (0, 1] Gidaspow-Ganser drag (Table 3: 0.85 / 0.86)


@dataclasses.dataclass
class Workload:
    name: str
    precision: str             # "fp64" or "mixed"
    params: dict               # scalar physics / numerics
    beds: list
    ores: list
    parcels: dict              # name -> np.ndarray, original id order
    gas: dict                  # name -> np.ndarray over all gas cells (beds concatenated)
    cell_offset: np.ndarray    # first gas cell of each bed
    steps: int
    couple_every: int

    @property
    def n(self) -> int:
        return int(self.parcels["x"].shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.gas["T"].shape[0])


# Neighbour lists: checked every check_every steps (and at every coupling)
# and rebuilt on the device when the largest displacement since the last
# build plus 2 check_every dt times the largest speed could reach skin/2.
def base_params(**kw) -> dict:
    p = dict(kn=1000.0, e_p=0.9, mu_s=0.3, mu_r=0.0, kt_over_kn=2.0 / 7.0, gt_over_gn=0.0,
             eps_min=0.35, skin=5e-5, g=(0.0, 0.0, -9.81), dt=1e-5, check_every=10,
             max_nbr=48, ergun_printed=0, energy_on=0)
    p.update(kw)
    return p


# ---------------------------------------------------------------- placement

def _grid_lin(ci, nc):
    return ci[:, 0] + nc[0] * (ci[:, 1] + nc[1] * ci[:, 2])


def _grid_insert(grid, fill, lin, ids):
    srt = np.argsort(lin, kind="stable")
    lin_s = lin[srt]
    ids_s = ids[srt]
    _, first = np.unique(lin_s, return_index=True)
    rank = np.arange(lin_s.size) - np.repeat(first, np.diff(np.append(first, lin_s.size)))
    slot = fill[lin_s] + rank
    if np.any(slot >= grid.shape[1]):
        raise RuntimeError("placement grid capacity exceeded")
    grid[lin_s, slot] = ids_s
    np.add.at(fill, lin_s, 1)


_OFFS27 = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)])


def _grid_hits(grid, nc, ci, p, r, cpos, crad, later_than=None):
    """For each query (p, r) in cell ci, True if it overlaps an entry of
    ``grid`` (entries index cpos/crad).  With ``later_than`` (query ranks),
    only entries with a smaller rank count."""
    hit = np.zeros(p.shape[0], bool)
    for o in _OFFS27:
        cj = ci + o
        inb = np.all((cj >= 0) & (cj < nc), axis=1)
        lin = np.where(inb, _grid_lin(cj, nc), 0)
        nb = grid[lin]
        valid = (nb >= 0) & inb[:, None]
        nbs = np.where(valid, nb, 0)
        if later_than is not None:
            valid &= nbs < later_than[:, None]
        dd = p[:, None, :] - cpos[nbs]
        dist2 = np.einsum("ijk,ijk->ij", dd, dd)
        hit |= np.any(valid & (dist2 <= (r[:, None] + crad[nbs]) ** 2), axis=1)
    return hit


def _rsa_box(rng, d, lo, hi, max_rounds=20000):
    """Random sequential addition of spheres of diameters ``d`` (largest
    first, in batches) uniformly inside the box [lo, hi] without overlap with
    each other or the walls.  Returns centres (n, 3)."""
    n = d.shape[0]
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    order = np.argsort(-d, kind="stable")
    nc = np.maximum(1, np.floor((hi - lo) / float(d.max())).astype(np.int64))
    cell_sz = (hi - lo) / nc
    ncell = int(nc.prod())
    cap = int(math.ceil(0.74 * float(np.prod(cell_sz)) / (math.pi / 6.0 * float(d.min()) ** 3))) + 2
    grid = -np.ones((ncell, cap), np.int64)
    fill = np.zeros(ncell, np.int64)
    pos = np.zeros((n, 3))
    rad = 0.5 * d
    pending = order.copy()
    for _ in range(max_rounds):
        if pending.size == 0:
            break
        bsz = max(256, min(pending.size, max(2048, ncell // 8)))
        batch = pending[:bsz]
        rest = pending[bsz:]
        r = rad[batch]
        p = lo + r[:, None] + rng.random((batch.size, 3)) * ((hi - lo) - 2 * r[:, None])
        ci = np.minimum(np.floor((p - lo) / cell_sz).astype(np.int64), nc - 1)
        ok = ~_grid_hits(grid, nc, ci, p, r, pos, rad)
        idx = np.nonzero(ok)[0]
        if idx.size > 1:
            # conflicts inside the batch: candidates may still overlap each
            # other, so their grid is sized by the fullest cell of this batch
            tlin = _grid_lin(ci[idx], nc)
            tgrid = -np.ones((ncell, int(np.bincount(tlin).max())), np.int64)
            _grid_insert(tgrid, np.zeros(ncell, np.int64), tlin, np.arange(idx.size))
            clash = _grid_hits(tgrid, nc, ci[idx], p[idx], r[idx], p[idx], r[idx],
                               later_than=np.arange(idx.size))
            idx = idx[~clash]
        acc = np.zeros(batch.size, bool)
        acc[idx] = True
        ids = batch[acc]
        pos[ids] = p[acc]
        _grid_insert(grid, fill, _grid_lin(ci[acc], nc), ids)
        pending = np.concatenate([rest, batch[~acc]])
    if pending.size:
        raise RuntimeError(f"RSA could not place {pending.size} parcels")
    return pos


def _layer_pack(rng, d, R, cx, cy, z0, gap_frac=0.02, jitter=0.5, classes=1):
    """Layered lattice packing inside a cylinder of radius R (axis at cx, cy)
    from height z0 up.  Parcels are split into ``classes`` size classes (by
    quantile); horizontal layers cycle through the classes, each layer a
    square lattice of pitch a = d_max(class)*(1+gap_frac) filled with parcels
    of its class at random sites, each parcel jittered inside its own a^3 cube
    by up to jitter*(a-d)/2 per axis (so no two parcels overlap).  Cycling the
    classes keeps sizes mixed along the bed height.  Returns (n, 3) centres."""
    n = d.shape[0]
    order = np.argsort(-d, kind="stable")
    groups = [g for g in np.array_split(order, classes) if g.size]
    pos = np.zeros((n, 3))
    taken = [0] * len(groups)
    z = z0
    c = 0
    left = n
    while left > 0:
        g = groups[c]
        if taken[c] < g.size:
            a = float(d[g[taken[c]:]].max()) * (1.0 + gap_frac)
            m = int(math.floor(2 * R / a))
            lat = (np.arange(m) - (m - 1) / 2.0) * a
            gx, gy = np.meshgrid(lat, lat, indexing="ij")
            gx = gx.ravel()
            gy = gy.ravel()
            inside = np.sqrt(gx ** 2 + gy ** 2) + 0.5 * a * math.sqrt(2.0) <= R
            sx = gx[inside] + cx
            sy = gy[inside] + cy
            if sx.size == 0:
                raise RuntimeError("container too small for one lattice layer")
            take = g[taken[c]:taken[c] + sx.size]
            sel = rng.permutation(sx.size)[: take.size]
            r = 0.5 * d[take]
            amp = jitter * (0.5 * a - r)
            pos[take, 0] = sx[sel] + amp * (2 * rng.random(take.size) - 1)
            pos[take, 1] = sy[sel] + amp * (2 * rng.random(take.size) - 1)
            pos[take, 2] = z + 0.5 * a + amp * (2 * rng.random(take.size) - 1)
            z += a
            taken[c] += take.size
            left -= take.size
        c = (c + 1) % len(groups)
    return pos


def _moles(rng, d_p, rho_eff, wt):
    """Initial moles per real particle of Fe2O3, Fe3O4, FeO, Fe from mass fractions."""
    m_p = rho_eff * math.pi / 6.0 * d_p.astype(np.float64) ** 3
    out = {}
    for key, name in (("nh", "Fe2O3"), ("nm", "Fe3O4"), ("nw", "FeO"), ("nfe", "Fe")):
        out[key] = m_p * wt.get(name, 0.0) / _MOLAR_MASS[name]
    return out


def _gas(rng, beds, T, xh2, xh2o, u, perturb, mask_cyl, grad_p=(0.0, 0.0, 0.0), p=101325.0):
    """Frozen gas fields per cell (beds concatenated).  T, xh2, xh2o may be
    per-bed sequences."""
    fields = {k: [] for k in ("ug", "vg", "wg", "p", "dpdx", "dpdy", "dpdz", "T", "xH2", "xH2O", "xN2")}
    for b, bed in enumerate(beds):
        nx, ny, nz = bed.n
        nc = nx * ny * nz
        Tb = T[b] if np.ndim(T) else T
        xb = xh2[b] if np.ndim(xh2) else xh2
        wb = xh2o[b] if np.ndim(xh2o) else xh2o
        uvec = np.tile(np.asarray(u, float), (nc, 1))
        if perturb > 0:
            uvec = uvec + perturb * (2 * rng.random((nc, 3)) - 1)
        if mask_cyl and bed.wall == WALL_CYL:
            ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
            xc = bed.origin[0] + (ii + 0.5) * bed.h
            yc = bed.origin[1] + (jj + 0.5) * bed.h
            cx = 0.5 * (bed.lo[0] + bed.hi[0])
            cy = 0.5 * (bed.lo[1] + bed.hi[1])
            inside2d = (xc - cx) ** 2 + (yc - cy) ** 2 <= bed.R ** 2
            inside = np.broadcast_to(inside2d.T[None, :, :], (nz, ny, nx)).reshape(-1)
            uvec[~inside] = 0.0
        fields["ug"].append(uvec[:, 0])
        fields["vg"].append(uvec[:, 1])
        fields["wg"].append(uvec[:, 2])
        fields["p"].append(np.full(nc, p))
        fields["dpdx"].append(np.full(nc, grad_p[0]))
        fields["dpdy"].append(np.full(nc, grad_p[1]))
        fields["dpdz"].append(np.full(nc, grad_p[2]))
        fields["T"].append(np.full(nc, float(Tb)))
        fields["xH2"].append(np.full(nc, float(xb)))
        fields["xH2O"].append(np.full(nc, float(wb)))
        fields["xN2"].append(np.full(nc, 1.0 - float(xb) - float(wb)))
    return {k: np.ascontiguousarray(np.concatenate(v)) for k, v in fields.items()}


def _parcels(pos, d_p, k, ore, bed, rho_eff_of_ore, wt_of_ore):
    n = pos.shape[0]
    d = (k * d_p).astype(np.float32)  # parcel diameter, FP32-representable
    out = dict(x=np.ascontiguousarray(pos[:, 0]), y=np.ascontiguousarray(pos[:, 1]),
               z=np.ascontiguousarray(pos[:, 2]))
    for key in ("vx", "vy", "vz", "wx", "wy", "wz"):
        out[key] = np.zeros(n)
    out["d"] = d
    out["k"] = np.full(n, k, np.float32) if np.ndim(k) == 0 else k.astype(np.float32)
    out["ore"] = ore.astype(np.int32)
    out["bed"] = bed.astype(np.int32)
    dp64 = d.astype(np.float64) / out["k"].astype(np.float64)
    sp = {key: np.zeros(n) for key in ("nh", "nm", "nw", "nfe")}
    for o in np.unique(ore):
        sel = ore == o
        mo = _moles(None, dp64[sel], rho_eff_of_ore[int(o)], wt_of_ore[int(o)])
        for key in sp:
            sp[key][sel] = mo[key]
    out.update(sp)
    return out


def _shuffle_ids(rng, parcels):
    n = parcels["x"].shape[0]
    perm = rng.permutation(n)
    return {k: np.ascontiguousarray(v[perm]) for k, v in parcels.items()}


def _cyl_bed(R, H, h, refine, theta, pad=0.0):
    nxy = int(math.ceil(2 * R / h))
    nz = int(math.ceil(H / h))
    side = nxy * h
    lo = (0.0, 0.0, 0.0)
    hi = (side, side, nz * h)
    return Bed(wall=WALL_CYL, lo=lo, hi=(side, side, H), R=R, origin=lo, h=h, n=(nxy, nxy, nz),
               refine=refine, theta=tuple(theta))


# ---------------------------------------------------------------- workloads

def cfg1(n=2048, seed=1, steps=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = (n / 2048.0) ** (1.0 / 3.0)
    h = 2e-3
    nx = max(2, int(round(8 * s)))
    nz = max(4, int(round(32 * s)))
    L, Hz = nx * h, nz * h
    bed = Bed(WALL_BOX, (0.0, 0.0, 0.0), (L, L, Hz), 0.0, (0.0, 0.0, 0.0), h, (nx, nx, nz), 1,
              THETA_HEMATITE_FIT, mu_override=4e-5)
    d_p = rng.uniform(0.95e-3, 1.05e-3, n).astype(np.float32).astype(np.float64)
    pos = _rsa_box(rng, d_p, bed.lo, bed.hi)
    rho = 4500.0
    ore = Ore(xi0=1.0 - rho / RHO_TRUE[0], d_pore_cm=3.3e-6)
    parcels = _parcels(pos, d_p, 1.0, np.zeros(n), np.zeros(n), {0: rho}, {0: HEMATITE_WT})
    gas = _gas(rng, [bed], 1073.0, 1.0, 0.0, (0.0, 0.0, 0.5), 0.0, False)
    params = base_params(dt=1e-5, skin=1e-4, check_every=10)
    return Workload("cfg1", "fp64", params, [bed], [ore], parcels, gas, np.array([0]), steps, 10)


def _cfg_cyl(name, n, N0, R0, H0, h, refine, d_sampler, k, ores, ore_split, T, xh2, seed, steps,
             dt=5e-6, couple=20, precision="mixed", skin=6e-5, u=0.3, classes=8, check=10, kn=1000.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = (n / float(N0)) ** (1.0 / 3.0)
    R = R0 * s
    H = H0 * s
    bed = _cyl_bed(R, H, h, refine, THETA_HEMATITE_FIT)
    d_p = d_sampler(rng, n).astype(np.float32).astype(np.float64)
    if np.max(k * d_p) * (1 + 0.02) > h / refine - skin:
        raise ValueError("DEM cell smaller than the largest parcel plus skin")
    ore_idx = ore_split(rng, n)
    cx = 0.5 * (bed.lo[0] + bed.hi[0])
    cy = 0.5 * (bed.lo[1] + bed.hi[1])
    pos = _layer_pack(rng, (k * d_p), R, cx, cy, 0.0, classes=classes)
    if pos[:, 2].max() + 0.5 * k * d_p.max() > H:
        raise RuntimeError("packed bed higher than the container")
    rho_of = {i: (1.0 - o.xi0) * o.rho_true[0] for i, o in enumerate(ores)}
    wt_of = {i: (HEMATITE_WT if o.kind == ORE_HEMATITE else MAGNETITE_WT) for i, o in enumerate(ores)}
    parcels = _parcels(pos, d_p, k, ore_idx, np.zeros(n), rho_of, wt_of)
    parcels = _shuffle_ids(rng, parcels)
    gas = _gas(rng, [bed], T, xh2, 0.0, (0.0, 0.0, u), 0.1 * u, True)
    params = base_params(dt=dt, skin=skin, check_every=check, kn=kn)
    return Workload(name, precision, params, [bed], ores, parcels, gas, np.array([0]), steps, couple)


def cfg2(n=200_000, seed=2, steps=2000):
    return _cfg_cyl("cfg2", n, 200_000, 20e-3, 200e-3, 1.25e-3, 2,
                    lambda rng, m: rng.uniform(120e-6, 180e-6, m), 3.0,
                    [Ore(xi0=0.34, d_pore_cm=3.3e-6)], lambda rng, m: np.zeros(m, np.int32),
                    973.0, 0.9, seed, steps)


def _lognormal_dp(rng, m):
    z = rng.standard_normal(m)
    bad = np.abs(z) > 3.0
    while bad.any():
        z[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(z) > 3.0
    return 100e-6 * np.exp(0.3 * z)


def cfg3(n=2_000_000, seed=3, steps=500, u=0.01, kn=200.0, xh2=1.0):
    """The 2M-parcel bed.  By default gas upflow 0.01 m/s of pure H2, below the
    minimum fluidization velocity of the median real particle (about
    0.014 m/s for 100 um ore in H2 at 1073 K), so the bed is a fixed bed, the
    regime the paper's hematite bed starts in; fluidized() gives the
    described 0.3 m/s of 90 % H2.  kn = 200 N/m: a linear stiffness of the
    size a Hertzian contact with the paper's Y = 1e7 Pa at u_c = 1 m/s gives
    for these parcels, and one that keeps the contact of the smallest parcels
    (d = 0.2 mm, 3 sigma below the median) resolved at dt = 5 us (kn = 1000
    N/m would make it unstable).  Skin 0.1 mm, lists checked at every coupling
    (20 steps); the voidage and source deposits re-sort by cell at every
    coupling on their own."""
    ores = [Ore(xi0=0.05, d_pore_cm=3.3e-6), Ore(xi0=0.25, d_pore_cm=9.5e-6)]
    return _cfg_cyl("cfg3", n, 2_000_000, 50e-3, 600e-3, 1.5625e-3, 1, _lognormal_dp, 5.0, ores,
                    lambda rng, m: (rng.random(m) < 0.5).astype(np.int32), 1073.0, xh2, seed, steps,
                    skin=1e-4, check=20, u=u, kn=kn)


def fluidized(w):
    """The same bed (same parcels and state) under the 2M-parcel bed's
    described gas: 0.3 m/s upflow with a seeded +-10 % perturbation per cell,
    90 % H2 and N2 at 1073 K."""
    rng = np.random.Generator(np.random.PCG64(33))
    gas = _gas(rng, w.beds, 1073.0, 0.9, 0.0, (0.0, 0.0, 0.3), 0.03, True)
    return dataclasses.replace(w, gas=gas)


def cfg4(n=500_000, seed=4, steps=20_000):
    R = 20e-3 * (2.5 ** (1.0 / 3.0))
    H = 200e-3 * (2.5 ** (1.0 / 3.0))
    w = _cfg_cyl("cfg4", n, 500_000, R, H, 1.25e-3, 2,
                 lambda rng, m: rng.uniform(120e-6, 180e-6, m), 3.0,
                 [Ore(xi0=0.34, d_pore_cm=3.3e-6)], lambda rng, m: np.zeros(m, np.int32),
                 1073.0, 0.9, seed, steps)
    w.params.update(dt=5e-6)
    return w


def grad_spec_cfg4(n_substeps=20_000):
    """Adjoint protocol of the kinetic-gradient workload."""
    return dict(n_substeps=n_substeps, dt_react=1e-4, dyn_every=10, ckpt_every=500)


def cfg5(n_beds=64, seed=5, steps=1000, n_scale=1.0):
    ss = np.random.SeedSequence(seed)
    rng0 = np.random.Generator(np.random.PCG64(ss))
    Nb = np.floor(np.exp(rng0.uniform(math.log(5000), math.log(80000), n_beds))).astype(np.int64)
    Nb = np.maximum(16, (Nb * n_scale).astype(np.int64))
    kids = ss.spawn(n_beds)
    beds, parts, Ts, xs = [], [], [], []
    h = 2e-3
    for b in range(n_beds):
        rng = np.random.Generator(np.random.PCG64(kids[b]))
        s = (Nb[b] / 2048.0) ** (1.0 / 3.0)
        nx = max(2, int(math.ceil(8 * s)))
        nz = max(4, int(math.ceil(32 * s)))
        i, j = divmod(b % 64, 8)
        Ts.append(973.0 + 200.0 * i / 7.0)
        xs.append(0.6 + 0.4 * j / 7.0)
        bed = Bed(WALL_BOX, (0.0, 0.0, 0.0), (nx * h, nx * h, nz * h), 0.0, (0.0, 0.0, 0.0), h,
                  (nx, nx, nz), 1, THETA_HEMATITE_FIT)
        d_p = rng.uniform(0.95e-3, 1.05e-3, int(Nb[b])).astype(np.float32).astype(np.float64)
        pos = _rsa_box(rng, d_p, bed.lo, bed.hi)
        pc = _parcels(pos, d_p, 1.0, np.zeros(Nb[b]), np.full(Nb[b], b), {0: 4500.0}, {0: HEMATITE_WT})
        beds.append(bed)
        parts.append(pc)
    ore = Ore(xi0=1.0 - 4500.0 / RHO_TRUE[0], d_pore_cm=3.3e-6)
    parcels = {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts])) for k in parts[0]}
    rng = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    gas = _gas(rng, beds, Ts, xs, 0.0, (0.0, 0.0, 0.5), 0.0, False)
    offs = np.concatenate([[0], np.cumsum([bd.n_cells for bd in beds])[:-1]])
    params = base_params(dt=5e-6, skin=2e-4, check_every=20)
    return Workload("cfg5", "mixed", params, beds, [ore], parcels, gas, offs, steps, 20)


# Magnetite kinetics: Table 2 (Takenaka) for R1, and for R2 / R3 the
# activation energies of Section 5.1 with the fitted pre-exponential factors
# 8 and 6000 m/s (the starting guess 8 and 5000 in THETA_MAGNETITE_START).
THETA_MAGNETITE_FIT = (math.log(29.17), 66974.0, math.log(8.0), 75345.0, math.log(6000.0), 117204.0)
THETA_MAGNETITE_START = (math.log(29.17), 66974.0, math.log(8.0), 75345.0, math.log(5000.0), 117204.0)

# (bed, T (K), superficial gas velocity (m/s), kinetic set) of the sweep: the
# Bed I magnetite temperatures of Fig. 12 with the fitted set, the starting
# set of Fig. 7 at 943 K, and the Bed II hematite temperatures of Fig. 13
SWEEP_BEDS = (("I", 943.0, 0.183, THETA_MAGNETITE_FIT), ("I", 923.0, 0.179, THETA_MAGNETITE_FIT),
              ("I", 903.0, 0.175, THETA_MAGNETITE_FIT), ("I", 943.0, 0.183, THETA_MAGNETITE_START),
              ("II", 1073.0, 0.43, THETA_HEMATITE_FIT), ("II", 1023.0, 0.41, THETA_HEMATITE_FIT),
              ("II", 973.0, 0.39, THETA_HEMATITE_FIT))


def sweep(n_scale=1.0, seed=6, steps=500, beds=SWEEP_BEDS):
    """Kinetic sweep over Bed I / Bed II shaped beds in one batched context
    (Table 3).  Bed I: magnetite ore (69.94 % Fe3O4, 30.06 % FeO, rho_p0 3720,
    porosity 0.29, pore 9.5e-6 cm, sphericity 0.85), real d_p 0.1 mm (+-10 %),
    k = 2.8, 5,140,800 real particles in a 20 x 60 mm cylinder, 1.25 mm gas
    cells, 70 % H2 in N2 at 101325 Pa.  Bed II: hematite ore (96.28 % Fe2O3,
    3.72 % FeO, rho_p0 3500, porosity 0.34, pore 3.3e-6 cm, sphericity 0.86),
    d_p 0.35 mm (+-10 %), k = 3, 5,095,837 real particles in a 68 x 200 mm
    cylinder, 4.25 mm gas cells, 65 % H2 in N2 at 110000 Pa.  n_scale scales
    the parcel counts (and the cylinders by its cube root).  One DEM step of
    5 us for all beds (Bed I's), coupling every 20 steps, lists rebuilt every
    40; kn = 100 N/m, the linear stiffness a Hertzian contact with Y = 1e7 Pa
    gives the Bed I parcels at 1 % overlap."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(len(beds) + 1)
    ores = [Ore(xi0=0.29, d_pore_cm=9.5e-6, kind=ORE_MAGNETITE, psi=0.85),
            Ore(xi0=0.34, d_pore_cm=3.3e-6, kind=ORE_HEMATITE, psi=0.86)]
    shape = {"I": dict(R=10e-3, H=60e-3, h=1.25e-3, dp=0.1e-3, k=2.8, real=5_140_800, ore=0, rho=3720.0,
                       wt=MAGNETITE_WT, xh2=0.7, p=101325.0),
             "II": dict(R=34e-3, H=200e-3, h=4.25e-3, dp=0.35e-3, k=3.0, real=5_095_837, ore=1, rho=3500.0,
                        wt=HEMATITE_WT, xh2=0.65, p=110000.0)}
    s = n_scale ** (1.0 / 3.0)
    bl, parts, gases = [], [], []
    for b, (kind, T, u, theta) in enumerate(beds):
        sh = shape[kind]
        rng = np.random.Generator(np.random.PCG64(kids[b]))
        n = max(16, int(round(sh["real"] / sh["k"] ** 3 * n_scale)))
        bed = _cyl_bed(sh["R"] * s, sh["H"] * s, sh["h"], 3, theta)
        d_p = rng.uniform(0.9 * sh["dp"], 1.1 * sh["dp"], n).astype(np.float32).astype(np.float64)
        cx = 0.5 * (bed.lo[0] + bed.hi[0])
        cy = 0.5 * (bed.lo[1] + bed.hi[1])
        pos = _layer_pack(rng, sh["k"] * d_p, bed.R, cx, cy, 0.0, classes=4)
        if pos[:, 2].max() + 0.5 * sh["k"] * d_p.max() > bed.hi[2]:
            raise RuntimeError("packed bed higher than the container")
        pc = _parcels(pos, d_p, sh["k"], np.full(n, sh["ore"]), np.full(n, b), {sh["ore"]: sh["rho"]},
                      {sh["ore"]: sh["wt"]})
        bl.append(bed)
        parts.append(_shuffle_ids(rng, pc))
        gases.append(_gas(rng, [bed], T, sh["xh2"], 0.0, (0.0, 0.0, u), 0.1 * u, True, p=sh["p"]))
    parcels = {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts])) for k in parts[0]}
    gas = {k: np.ascontiguousarray(np.concatenate([g[k] for g in gases])) for k in gases[0]}
    offs = np.concatenate([[0], np.cumsum([bd.n_cells for bd in bl])[:-1]])
    params = base_params(dt=5e-6, skin=1e-4, check_every=20, kn=100.0)
    return Workload("sweep", "mixed", params, bl, ores, parcels, gas, offs, steps, 20)


def make(name: str, **kw) -> Workload:
    return {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4, "cfg5": cfg5, "sweep": sweep}[name](**kw)


def with_velocities(w: Workload, seed: int, vscale=0.05, wscale=50.0) -> Workload:
    """Copy of ``w`` with seeded random translational and angular velocities
    (used by tests to exercise damping, friction and rolling terms)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = dict(w.parcels)
    n = w.n
    for key in ("vx", "vy", "vz"):
        p[key] = vscale * (2 * rng.random(n) - 1)
    for key in ("wx", "wy", "wz"):
        p[key] = wscale * (2 * rng.random(n) - 1)
    if w.precision == "mixed":
        for key in ("vx", "vy", "vz", "wx", "wy", "wz"):
            p[key] = p[key].astype(np.float32).astype(np.float64)
    return dataclasses.replace(w, parcels=p)


def with_energy(w: Workload, dT: float = 0.0, seed: int = None, spread: float = 0.0) -> Workload:
    """Copy of ``w`` with the particle energy equation on: every parcel starts
    at the gas temperature of its cell plus ``dT`` (K), plus a seeded uniform
    offset in [-spread, spread] when ``seed`` is given."""
    p = dict(w.parcels)
    Tp = np.zeros(w.n)
    for b, bed in enumerate(w.beds):
        sel = np.flatnonzero(p["bed"] == b)
        q = [np.clip(np.floor((p[a][sel] - bed.origin[i]) / bed.h), 0, bed.n[i] - 1).astype(np.int64)
             for i, a in enumerate(("x", "y", "z"))]
        c = int(w.cell_offset[b]) + q[0] + bed.n[0] * (q[1] + bed.n[1] * q[2])
        Tp[sel] = w.gas["T"][c]
    Tp += dT
    if seed is not None:
        rng = np.random.Generator(np.random.PCG64(seed))
        Tp += spread * (2 * rng.random(w.n) - 1)
    p["Tp"] = Tp
    prm = dict(w.params)
    prm["energy_on"] = 1
    return dataclasses.replace(w, parcels=p, params=prm)


def squeeze(w: Workload, factor: float, seed: int) -> Workload:
    """Copy of ``w`` with parcel centres pulled towards each bed's lower centre
    by ``factor`` (<1), which creates overlapping contacts for force tests.
    Positions stay FP64; nothing else changes."""
    p = dict(w.parcels)
    x, y, z = p["x"].copy(), p["y"].copy(), p["z"].copy()
    for b, bed in enumerate(w.beds):
        sel = p["bed"] == b
        cx = 0.5 * (bed.lo[0] + bed.hi[0])
        cy = 0.5 * (bed.lo[1] + bed.hi[1])
        x[sel] = cx + (x[sel] - cx) * factor
        y[sel] = cy + (y[sel] - cy) * factor
        z[sel] = bed.lo[2] + (z[sel] - bed.lo[2]) * factor
    p["x"], p["y"], p["z"] = x, y, z
    return dataclasses.replace(w, parcels=p)


def split_bed(w: Workload, b: int) -> Workload:
    """Bed b of a multi-bed workload as a workload of its own (its parcels in
    original order, its gas cells), for running beds one at a time."""
    sel = np.flatnonzero(w.parcels["bed"] == b)
    p = {k: np.ascontiguousarray(v[sel]) for k, v in w.parcels.items()}
    p["bed"] = np.zeros(sel.size, dtype=w.parcels["bed"].dtype)
    c0 = int(w.cell_offset[b])
    c1 = c0 + w.beds[b].n_cells
    gas = {k: np.ascontiguousarray(v[c0:c1]) for k, v in w.gas.items()}
    return dataclasses.replace(w, name=f"{w.name}_bed{b}", beds=[w.beds[b]], parcels=p, gas=gas,
                               cell_offset=np.array([0]))
