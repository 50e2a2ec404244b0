"""Thin Python binding over the demrx C-ABI with PyTorch device memory.

``Bed`` owns one demrx context: it uploads a workload's parcels and gas fields
into torch CUDA tensors, passes their device pointers to the library and
returns results as tensors.  No numerics happen here.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import capi
from .capi import DemError


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Bed:
    def __init__(self, w, device="cuda:0", drag_on=True, g=None, stream=None, theta=None, max_nbr=None,
                 check_every=None):
        self.L = capi.load()
        self.w = w
        self.device = torch.device(device)
        self.mixed = w.precision == "mixed"
        self.vdtype = torch.float32 if self.mixed else torch.float64
        self.n = w.n
        self.n_beds = len(w.beds)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        prm = w.params
        beds = (capi.DemBed * len(w.beds))()
        for b, bd in enumerate(w.beds):
            s = beds[b]
            s.wall_kind = bd.wall
            for i in range(3):
                s.lo[i], s.hi[i], s.origin[i], s.n[i] = bd.lo[i], bd.hi[i], bd.origin[i], bd.n[i]
            s.R, s.h, s.refine, s.mu_override = bd.R, bd.h, bd.refine, bd.mu_override
            th = bd.theta if theta is None else theta
            for i in range(6):
                s.theta[i] = th[i]
        ores = (capi.DemOre * len(w.ores))()
        for o, od in enumerate(w.ores):
            s = ores[o]
            s.xi0, s.d_pore_cm, s.tau, s.kind = od.xi0, od.d_pore_cm, od.tau, od.kind
            s.psi = getattr(od, "psi", 0.0)
            for i in range(4):
                s.rho_true[i] = od.rho_true[i]
        P = capi.DemParams()
        P.precision = capi.DEM_MIXED if self.mixed else capi.DEM_FP64
        P.n_beds, P.beds, P.n_ores, P.ores = len(w.beds), beds, len(w.ores), ores
        P.kn, P.e_p, P.mu_s, P.mu_r = prm["kn"], prm["e_p"], prm["mu_s"], prm["mu_r"]
        P.kt_over_kn, P.gt_over_gn, P.eps_min = prm["kt_over_kn"], prm["gt_over_gn"], prm["eps_min"]
        P.skin, P.dt = prm["skin"], prm["dt"]
        gg = prm["g"] if g is None else g
        for i in range(3):
            P.g[i] = gg[i]
        P.max_nbr = prm["max_nbr"] if max_nbr is None else max_nbr
        P.check_every = prm["check_every"] if check_every is None else check_every
        P.ergun_printed = int(prm.get("ergun_printed", 0))
        P.drag_on = int(drag_on)
        P.energy_on = int(prm.get("energy_on", 0))
        self.energy = bool(P.energy_on)
        self._P, self._beds, self._ores = P, beds, ores
        dev = self.device
        p = w.parcels
        self.inp = {}
        for k in ("x", "y", "z", "nh", "nm", "nw", "nfe"):
            self.inp[k] = torch.as_tensor(np.ascontiguousarray(p[k], dtype=np.float64), device=dev)
        for k in ("vx", "vy", "vz", "wx", "wy", "wz"):
            self.inp[k] = torch.as_tensor(np.asarray(p[k], dtype=np.float64), device=dev).to(self.vdtype)
        self.inp["d"] = torch.as_tensor(np.ascontiguousarray(p["d"], dtype=np.float32), device=dev)
        self.inp["k"] = torch.as_tensor(np.ascontiguousarray(p["k"], dtype=np.float32), device=dev)
        self.inp["ore"] = torch.as_tensor(np.ascontiguousarray(p["ore"], dtype=np.int32), device=dev)
        self.inp["bed"] = torch.as_tensor(np.ascontiguousarray(p["bed"], dtype=np.int32), device=dev)
        if self.energy:
            self.inp["Tp"] = torch.as_tensor(np.ascontiguousarray(p["Tp"], dtype=np.float64), device=dev)
        self.set_gas(w.gas)
        self.n_cells = int(self.gas_t["T"].shape[0])
        pc = capi.DemParcels(*[_ptr(self.inp.get(f)) for f in capi.PARCEL_FIELDS])
        h = C.c_void_p()
        with torch.cuda.device(dev):
            torch.cuda.synchronize(dev)
            r = self.L.dem_init(C.byref(P), C.byref(pc), self.n, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if r != 0:
            raise DemError(r, self.L.dem_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------ helpers
    def _check(self, r):
        if r != 0:
            raise DemError(r, self.L.dem_last_error(self.h).decode())

    def set_gas(self, gas):
        self.gas_t = {k: torch.as_tensor(np.ascontiguousarray(gas[k], dtype=np.float64), device=self.device)
                      for k in capi.GAS_FIELDS}
        self._gas = capi.DemGas(*[_ptr(self.gas_t[f]) for f in capi.GAS_FIELDS])

    def _sources(self, keys):
        out = {k: torch.zeros(self.n_cells, dtype=torch.float64, device=self.device) for k in keys}
        s = capi.DemSources(*[_ptr(out.get(f)) for f in capi.SOURCE_FIELDS])
        return out, s

    def close(self):
        if getattr(self, "h", None):
            self.L.dem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ API
    def step(self, n=1):
        self._check(self.L.dem_step(self.h, int(n), C.byref(self._gas)))

    def couple(self, keys=("eps", "np", "sumK", "sumKu", "sumKv", "sumKw", "sumKs")):
        out, s = self._sources(keys)
        self._check(self.L.dem_couple(self.h, C.byref(self._gas), C.byref(s)))
        self.sync()
        return out

    def react(self, dt, keys=None, fov=True):
        if keys is None:
            keys = ("mdotH2", "mdotH2O", "sumEQ", "sumES") + (("hA", "hAT", "Qrm", "Hr") if self.energy else ())
        out, s = self._sources(keys)
        bf = (C.c_double * self.n_beds)()
        fv = torch.zeros(self.n, dtype=torch.float64, device=self.device) if fov else None
        self._check(self.L.dem_react(self.h, float(dt), C.byref(self._gas), C.byref(s), bf, _ptr(fv)))
        out["bed_fov"] = np.array(bf[:])
        if fov:
            out["fov"] = fv
        return out

    def gas_species(self, dt, sources, xin, update=True):
        """One gas-side species step (dem_gas_species) from the sumEQ / sumES of
        a previous react(); returns the new mole fractions and, with update,
        copies them into this bed's gas fields."""
        out = {k: torch.zeros(self.n_cells, dtype=torch.float64, device=self.device) for k in ("xH2", "xH2O", "xN2")}
        xi = (C.c_double * 2)(float(xin[0]), float(xin[1]))
        self._check(self.L.dem_gas_species(self.h, float(dt), C.byref(self._gas), _ptr(sources["sumEQ"]),
                                           _ptr(sources["sumES"]), xi, _ptr(out["xH2"]), _ptr(out["xH2O"]),
                                           _ptr(out["xN2"])))
        if update:
            for k in out:
                self.gas_t[k].copy_(out[k])
        return out

    def gas_momentum(self, dt, sums, update=True):
        """One gas-side momentum step (dem_gas_momentum) from the drag sums of
        a previous couple(); returns the new (ug, vg, wg) and, with update,
        copies them into this bed's gas fields."""
        out = {k: torch.zeros(self.n_cells, dtype=torch.float64, device=self.device) for k in ("ug", "vg", "wg")}
        self._check(self.L.dem_gas_momentum(self.h, float(dt), C.byref(self._gas),
                                            *[_ptr(sums[k]) for k in ("sumK", "sumKu", "sumKv", "sumKw")],
                                            *[_ptr(out[k]) for k in ("ug", "vg", "wg")]))
        if update:
            for k in out:
                self.gas_t[k].copy_(out[k])
        return out

    def forces(self):
        F = torch.zeros(3 * self.n, dtype=torch.float64, device=self.device)
        T = torch.zeros(3 * self.n, dtype=torch.float64, device=self.device)
        self._check(self.L.dem_forces(self.h, C.byref(self._gas), _ptr(F), _ptr(T)))
        self.sync()
        return F.view(-1, 3), T.view(-1, 3)

    def state(self):
        out = {k: torch.zeros(self.n, dtype=torch.float64, device=self.device) for k in
               ("x", "y", "z", "nh", "nm", "nw", "nfe")}
        for k in ("vx", "vy", "vz", "wx", "wy", "wz"):
            out[k] = torch.zeros(self.n, dtype=self.vdtype, device=self.device)
        if self.energy:
            out["Tp"] = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        pc = capi.DemParcels(*[_ptr(out.get(f)) for f in capi.PARCEL_FIELDS])
        self._check(self.L.dem_get_state(self.h, C.byref(pc)))
        return out

    def set_state(self, st):
        t = {}
        for k in ("x", "y", "z", "nh", "nm", "nw", "nfe"):
            t[k] = torch.as_tensor(np.asarray(st[k], dtype=np.float64), device=self.device)
        for k in ("vx", "vy", "vz", "wx", "wy", "wz"):
            t[k] = torch.as_tensor(np.asarray(st[k], dtype=np.float64), device=self.device).to(self.vdtype)
        if self.energy and "Tp" in st:
            t["Tp"] = torch.as_tensor(np.asarray(st["Tp"], dtype=np.float64), device=self.device)
        pc = capi.DemParcels(*[_ptr(t.get(f)) for f in capi.PARCEL_FIELDS])
        self._check(self.L.dem_set_state(self.h, C.byref(pc)))

    def pairs(self):
        cap = max(16, 8 * self.n)
        while True:
            buf = (C.c_uint32 * (2 * cap))()
            npairs = C.c_int64()
            self._check(self.L.dem_pairs(self.h, buf, cap, C.byref(npairs)))
            if npairs.value <= cap:
                return np.frombuffer(buf, dtype=np.uint32, count=2 * npairs.value).reshape(-1, 2).astype(np.int64)
            cap = npairs.value

    def contacts(self):
        """Springs of the pairs and walls in contact (dem_get_contacts): ids
        (P, 2) with a < b, xi (P, 3), wall_on (n, 6), wall_xi (n, 6, 3)."""
        cap = max(16, 4 * self.n)
        while True:
            ids = np.zeros((cap, 2), dtype=np.uint32)
            xi = np.zeros((cap, 3), dtype=np.float64)
            won = np.zeros((self.n, 6), dtype=np.uint8)
            wxi = np.zeros((self.n, 6, 3), dtype=np.float64)
            c = capi.DemContacts(cap, 0, ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                                 xi.ctypes.data_as(C.POINTER(C.c_double)), won.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 wxi.ctypes.data_as(C.POINTER(C.c_double)))
            self._check(self.L.dem_get_contacts(self.h, C.byref(c)))
            if c.count <= cap:
                k = int(c.count)
                return {"ids": ids[:k].copy(), "xi": xi[:k].copy(), "wall_on": won, "wall_xi": wxi}
            cap = int(c.count)

    def set_contacts(self, ct):
        ids = np.ascontiguousarray(ct["ids"], dtype=np.uint32).reshape(-1, 2)
        xi = np.ascontiguousarray(ct["xi"], dtype=np.float64).reshape(-1, 3)
        won = np.ascontiguousarray(ct["wall_on"], dtype=np.uint8).reshape(self.n, 6)
        wxi = np.ascontiguousarray(ct["wall_xi"], dtype=np.float64).reshape(self.n, 6, 3)
        if len(ids) != len(xi):
            raise ValueError("ids and xi differ in length")
        c = capi.DemContacts(len(ids), len(ids), ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                             xi.ctypes.data_as(C.POINTER(C.c_double)), won.ctypes.data_as(C.POINTER(C.c_uint8)),
                             wxi.ctypes.data_as(C.POINTER(C.c_double)))
        self._check(self.L.dem_set_contacts(self.h, C.byref(c)))

    def save_checkpoint(self, path):
        """Parcel state and contact springs in one .npz file."""
        st = {k: v.cpu().numpy() for k, v in self.state().items()}
        ct = self.contacts()
        np.savez(path, **{"state_" + k: v for k, v in st.items()}, **{"contacts_" + k: v for k, v in ct.items()})

    def load_checkpoint(self, path):
        """Resume from save_checkpoint: state first, then the springs."""
        with np.load(path, allow_pickle=False) as z:
            self.set_state({k[6:]: z[k] for k in z.files if k.startswith("state_")})
            self.set_contacts({k[9:]: z[k] for k in z.files if k.startswith("contacts_")})

    def stats(self):
        s = capi.DemStats()
        self._check(self.L.dem_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in capi.DemStats._fields_}

    def run(self, n_intervals, couple_every, sources=False, bed_fov=False):
        keys = capi.SOURCE_FIELDS if sources else ()
        out, s = self._sources(keys)
        bf = (C.c_double * self.n_beds)() if bed_fov else None
        self._check(self.L.dem_run(self.h, int(n_intervals), int(couple_every), C.byref(self._gas),
                                   C.byref(s) if sources else None, bf))
        if bed_fov:
            out["bed_fov"] = np.array(bf[:])
        return out

    def profile(self, enable=True):
        self._check(self.L.dem_profile(self.h, int(enable)))

    def autotune(self):
        self._check(self.L.dem_autotune(self.h, C.byref(self._gas)))

    def set_launch(self, step_block, step_xcd_chunk, build_grid):
        self._check(self.L.dem_set_launch(self.h, int(step_block), int(step_xcd_chunk), int(build_grid)))

    def set_build(self, threads, tile, item_x):
        self._check(self.L.dem_set_build(self.h, int(threads), int(tile), int(item_x)))

    def grad(self, n_substeps, dt_react, dyn_every, ckpt_every, theta, state_fp32=True, with_grad=True):
        spec = capi.DemGradSpec(int(n_substeps), float(dt_react), int(dyn_every), int(ckpt_every), int(state_fp32))
        th = (C.c_double * 6)(*[float(v) for v in theta])
        J = C.c_double()
        g = (C.c_double * 6)()
        self._check(self.L.dem_grad(self.h, C.byref(spec), C.byref(self._gas), th, C.byref(J),
                                    g if with_grad else None))
        return J.value, (np.array(g[:]) if with_grad else None)

    def sync(self):
        self._check(self.L.dem_sync(self.h))


class ReductionDegree(torch.autograd.Function):
    """J(theta), the bed-mean reduction degree after the gradient protocol of
    ``spec`` (n_substeps, dt_react, dyn_every, ckpt_every[, state_fp32]), as a
    differentiable function of the six kinetic parameters theta = (ln k0_i,
    E_a,i): forward runs dem_grad (forward sweep with checkpoints and the
    adjoint sweep) and keeps the gradient; backward returns gJ * dJ/dtheta.
    theta is a float64 tensor of 6 values; J is returned on its device."""

    @staticmethod
    def forward(ctx, theta, bed, spec):
        th = theta.detach().to("cpu", torch.float64).numpy()
        J, g = bed.grad(spec["n_substeps"], spec["dt_react"], spec["dyn_every"], spec["ckpt_every"], th,
                        state_fp32=spec.get("state_fp32", True))
        ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return gJ * g, None, None
