"""ctypes driver for the FP64 CPU oracle (ora.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libora.so")
SRC = os.path.join(HERE, "ora.c")


FLAGS = ["-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = False) -> str:
    """Compile the oracle (plain C, -O2 -ffp-contract=off, no FMA, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "ora.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", *FLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_native(path: str) -> str:
    """The same source built -O3 -march=native for the host it runs on (the
    CPU-baseline timing); contraction stays off, so results are unchanged."""
    tmp = path + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", *FLAGS, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, path)
    return path


class OraBed(C.Structure):
    _fields_ = [("wall_kind", C.c_int), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("R", C.c_double), ("origin", C.c_double * 3), ("h", C.c_double),
                ("n", C.c_int * 3), ("cell_off", C.c_int), ("theta", C.c_double * 6),
                ("mu_override", C.c_double)]


class OraOre(C.Structure):
    _fields_ = [("xi0", C.c_double), ("d_pore_cm", C.c_double), ("tau", C.c_double),
                ("rho_true", C.c_double * 4), ("kind", C.c_int), ("psi", C.c_double)]


class OraParams(C.Structure):
    _fields_ = [("kn", C.c_double), ("e_p", C.c_double), ("mu_s", C.c_double), ("mu_r", C.c_double),
                ("kt_over_kn", C.c_double), ("gt_over_gn", C.c_double), ("eps_min", C.c_double),
                ("dt", C.c_double), ("g", C.c_double * 3), ("ergun_printed", C.c_int),
                ("drag_on", C.c_int), ("n_beds", C.c_int), ("n_ores", C.c_int), ("energy_on", C.c_int)]


_GAS_KEYS = ("ug", "vg", "wg", "p", "dpdx", "dpdy", "dpdz", "T", "xH2", "xH2O", "xN2")


class OraGas(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in _GAS_KEYS]


_lib = None
_lib_path = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (before first use)."""
    global _lib_path
    if _lib is not None:
        raise RuntimeError("oracle library already loaded")
    _lib_path = path


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().ora_set_threads(int(n))


def threads() -> int:
    return int(lib().ora_threads())


def host_threads() -> int:
    """Threads this host gives the process: OMP_NUM_THREADS if set, else the
    cores in its affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "").split(",")[0].strip()
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = C.CDLL(_lib_path or LIB)
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_set_threads.restype = None
        L.ora_threads.restype = C.c_int
        L.ora_set_threads(1)  # one thread unless set_threads() asks for more
        L.ora_new.restype = C.c_void_p
        L.ora_new.argtypes = [C.POINTER(OraParams), C.POINTER(OraBed), C.POINTER(OraOre), C.c_int] + \
            [_dp] * 9 + [_dp, _dp, _ip, _ip] + [_dp] * 4
        L.ora_free.argtypes = [C.c_void_p]
        L.ora_n_cells.argtypes = [C.c_void_p]
        L.ora_pairs.restype = C.c_long
        L.ora_pairs.argtypes = [C.c_void_p, C.c_int, _ip, C.c_long]
        L.ora_forces.argtypes = [C.c_void_p, C.POINTER(OraGas), _dp, _dp]
        L.ora_force_scale.argtypes = [C.c_void_p, C.POINTER(OraGas), _dp, _dp]
        L.ora_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(OraGas)]
        L.ora_step_perturbed.argtypes = [C.c_void_p, C.c_int, C.POINTER(OraGas), C.c_double, C.c_ulonglong,
                                         C.c_int]
        L.ora_couple.argtypes = [C.c_void_p, C.POINTER(OraGas)] + [_dp] * 7
        L.ora_react.restype = C.c_long
        L.ora_react.argtypes = [C.c_void_p, C.c_double, C.POINTER(OraGas), C.c_int] + [_dp] * 10
        L.ora_set_temperature.argtypes = [C.c_void_p, _dp]
        L.ora_get_energy.argtypes = [C.c_void_p, _dp, _dp, _dp]
        for name in ("ora_h_mol", "ora_cp_mol"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_int, C.c_double]
        for name in ("ora_lambda_g", "ora_cp_g"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 4
        L.ora_gas_species.argtypes = [C.c_void_p, C.POINTER(OraGas), C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.ora_gas_momentum.argtypes = [C.c_void_p, C.POINTER(OraGas), C.c_double] + [_dp] * 7
        L.ora_nusselt.restype = C.c_double
        L.ora_nusselt.argtypes = [C.c_double] * 3
        L.ora_get.argtypes = [C.c_void_p] + [_dp] * 15
        L.ora_contacts.restype = C.c_long
        L.ora_contacts.argtypes = [C.c_void_p, _ip, _dp, C.c_long, C.POINTER(C.c_ubyte), _dp]
        L.ora_set_contacts.restype = C.c_int
        L.ora_set_contacts.argtypes = [C.c_void_p, _ip, _dp, C.c_long, C.POINTER(C.c_ubyte), _dp]
        L.ora_grad.argtypes = [C.c_void_p, C.POINTER(OraGas), C.c_int, C.c_double, C.c_int, _dp, _dp, _dp]
        for name in ("ora_e_cgp", "ora_zeta", "ora_knudsen_h2", "ora_keq"):
            getattr(L, name).restype = C.c_double
        L.ora_e_cgp.argtypes = [C.c_double, C.c_double]
        L.ora_zeta.argtypes = [C.c_double]
        L.ora_knudsen_h2.argtypes = [C.c_double, C.c_double]
        L.ora_keq.argtypes = [C.c_int, C.c_double]
        L.ora_gas_props.argtypes = [C.c_double] * 6 + [_dp, _dp]
        L.ora_fuller.restype = C.c_double
        L.ora_fuller.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
        L.ora_wilke_h2.restype = C.c_double
        L.ora_wilke_h2.argtypes = [C.c_double] * 5
        L.ora_pore_diff.restype = C.c_double
        L.ora_pore_diff.argtypes = [C.c_double] * 6
        L.ora_layer_porosity.argtypes = [C.POINTER(OraOre), _dp]
        L.ora_sherwood.restype = C.c_double
        L.ora_sherwood.argtypes = [C.c_double] * 3
        L.ora_film.restype = C.c_double
        L.ora_film.argtypes = [C.c_double] * 9
        L.ora_beta_over_epsp.restype = C.c_double
        L.ora_beta_over_epsp.argtypes = [C.c_double] * 5 + [C.c_int]
        L.ora_beta_ganser_over_epsp.restype = C.c_double
        L.ora_beta_ganser_over_epsp.argtypes = [C.c_double] * 7 + [C.c_int]
        L.ora_ladder.argtypes = [_ip, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.ora_react_point.restype = C.c_int
        L.ora_react_point.argtypes = [_dp, _dp]
        L.ora_fov.restype = C.c_double
        L.ora_fov.argtypes = [_dp, C.c_int]
        _lib = L
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def ore_struct(o) -> OraOre:
    s = OraOre()
    s.xi0, s.d_pore_cm, s.tau, s.kind = o.xi0, o.d_pore_cm, o.tau, o.kind
    s.psi = getattr(o, "psi", 0.0)
    for i in range(4):
        s.rho_true[i] = o.rho_true[i]
    return s


class Oracle:
    """One oracle system built from a workload (see paper_2311_03908_amd.workloads)."""

    def __init__(self, w, drag_on=True, g=None, theta=None):
        L = lib()
        prm = w.params
        P = OraParams()
        P.kn, P.e_p, P.mu_s, P.mu_r = prm["kn"], prm["e_p"], prm["mu_s"], prm["mu_r"]
        P.kt_over_kn, P.gt_over_gn, P.eps_min, P.dt = prm["kt_over_kn"], prm["gt_over_gn"], prm["eps_min"], prm["dt"]
        gg = prm["g"] if g is None else g
        for i in range(3):
            P.g[i] = gg[i]
        P.ergun_printed = int(prm.get("ergun_printed", 0))
        P.drag_on = int(drag_on)
        P.n_beds, P.n_ores = len(w.beds), len(w.ores)
        P.energy_on = int(prm.get("energy_on", 0))
        beds = (OraBed * len(w.beds))()
        for b, bd in enumerate(w.beds):
            s = beds[b]
            s.wall_kind = bd.wall
            for i in range(3):
                s.lo[i], s.hi[i], s.origin[i], s.n[i] = bd.lo[i], bd.hi[i], bd.origin[i], bd.n[i]
            s.R, s.h, s.cell_off, s.mu_override = bd.R, bd.h, int(w.cell_offset[b]), bd.mu_override
            th = bd.theta if theta is None else theta
            for i in range(6):
                s.theta[i] = th[i]
        ores = (OraOre * len(w.ores))(*[ore_struct(o) for o in w.ores])
        p = w.parcels
        self._keep = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in
                      ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "d", "k", "nh", "nm", "nw", "nfe")}
        self._keep["ore"] = np.ascontiguousarray(p["ore"], dtype=np.int32)
        self._keep["bed"] = np.ascontiguousarray(p["bed"], dtype=np.int32)
        kp = self._keep
        self.n = w.n
        self.h = L.ora_new(C.byref(P), beds, ores, self.n,
                           *[_p(kp[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "d", "k")],
                           _p(kp["ore"], C.c_int), _p(kp["bed"], C.c_int),
                           *[_p(kp[k]) for k in ("nh", "nm", "nw", "nfe")])
        self.n_cells = L.ora_n_cells(self.h)
        self.energy = bool(P.energy_on)
        if self.energy:
            self._keep["Tp"] = np.ascontiguousarray(p["Tp"], dtype=np.float64)
            L.ora_set_temperature(self.h, _p(self._keep["Tp"]))
        self.set_gas(w.gas)

    def set_gas(self, gas):
        self._gas = {k: np.ascontiguousarray(gas[k], dtype=np.float64) for k in _GAS_KEYS}
        self._gs = OraGas(*[_p(self._gas[k]) for k in _GAS_KEYS])

    def __del__(self):
        if getattr(self, "h", None):
            lib().ora_free(self.h)
            self.h = None

    def pairs(self, brute=False):
        L = lib()
        cap = max(16, 8 * self.n)
        while True:
            buf = np.zeros(2 * cap, np.int32)
            n = L.ora_pairs(self.h, int(brute), _p(buf, C.c_int), cap)
            if n <= cap:
                return buf[: 2 * n].reshape(-1, 2)
            cap = int(n)

    def forces(self):
        F = np.zeros(3 * self.n)
        T = np.zeros(3 * self.n)
        lib().ora_forces(self.h, C.byref(self._gs), _p(F), _p(T))
        return F.reshape(-1, 3), T.reshape(-1, 3)

    def force_scale(self):
        """Per parcel, the sums of the magnitudes of the products that
        forces() builds F and T from (ora_force_scale): F and T evaluated in
        a lower precision carry a rounding error proportional to these
        scales, not to |F| and |T|."""
        Fs = np.zeros(self.n)
        Ts = np.zeros(self.n)
        lib().ora_force_scale(self.h, C.byref(self._gs), _p(Fs), _p(Ts))
        return Fs, Ts

    def step(self, n=1):
        lib().ora_step(self.h, int(n), C.byref(self._gs))

    def step_perturbed(self, n, rel, seed=1, round32=False):
        """Test harness: steps with every force and torque component biased by
        rel of the parcel's force-term scale, with a sign fixed per parcel,
        component and seed, and with round32 the velocities, spins and
        springs rounded to FP32 after every step (ora_step_perturbed)."""
        lib().ora_step_perturbed(self.h, int(n), C.byref(self._gs), float(rel), int(seed), int(round32))

    def couple(self):
        out = {k: np.zeros(self.n_cells) for k in ("eps", "np", "sumK", "sumKu", "sumKv", "sumKw", "sumKs")}
        lib().ora_couple(self.h, C.byref(self._gs), *[_p(out[k]) for k in
                         ("eps", "np", "sumK", "sumKu", "sumKv", "sumKw", "sumKs")])
        return out

    def react(self, dt, update_mass=True, n_beds=1):
        keys = ("mdotH2", "mdotH2O", "sumEQ", "sumES")
        heat = ("hA", "hAT", "Qrm", "Hr")
        out = {k: np.zeros(self.n_cells) for k in keys + heat}
        fov = np.zeros(self.n)
        bf = np.zeros(n_beds)
        cl = lib().ora_react(self.h, float(dt), C.byref(self._gs), int(update_mass),
                             *[_p(out[k]) for k in keys], _p(fov), _p(bf), *[_p(out[k]) for k in heat])
        if not self.energy:
            for k in heat:
                del out[k]
        out["fov"] = fov
        out["bed_fov"] = bf
        out["clamps"] = int(cl)
        return out

    def gas_species(self, dt, sumEQ, sumES, xin):
        """New (xH2, xH2O, xN2) per cell after one transport step (see ora_gas_species)."""
        out = [np.zeros(self.n_cells) for _ in range(3)]
        eq = np.ascontiguousarray(sumEQ, dtype=np.float64)
        es = np.ascontiguousarray(sumES, dtype=np.float64)
        xi = np.ascontiguousarray(xin, dtype=np.float64)
        lib().ora_gas_species(self.h, C.byref(self._gs), float(dt), _p(eq), _p(es), _p(xi), *[_p(o) for o in out])
        return {"xH2": out[0], "xH2O": out[1], "xN2": out[2]}

    def gas_momentum(self, dt, sums):
        """New gas velocity (ug, vg, wg) per cell after one step dt of the
        interphase momentum exchange with the drag sums of a deposit
        (sumK, sumKu, sumKv, sumKw; see ora_gas_momentum)."""
        out = [np.zeros(self.n_cells) for _ in range(3)]
        ins = [np.ascontiguousarray(sums[k], dtype=np.float64) for k in ("sumK", "sumKu", "sumKv", "sumKw")]
        lib().ora_gas_momentum(self.h, C.byref(self._gs), float(dt), *[_p(a) for a in ins], *[_p(o) for o in out])
        return {"ug": out[0], "vg": out[1], "wg": out[2]}

    def grad(self, n_sub, dt_react, dyn_every, theta):
        if self.energy:
            raise ValueError("the gradient protocol is isothermal")
        th = np.ascontiguousarray(theta, dtype=np.float64)
        J = np.zeros(1)
        g = np.zeros(6)
        lib().ora_grad(self.h, C.byref(self._gs), int(n_sub), float(dt_react), int(dyn_every), _p(th), _p(J), _p(g))
        return float(J[0]), g

    def contacts(self):
        """Tangential springs held: ids (P, 2) with i < j, xi (P, 3) in i's
        orientation, wall_on (n, 6), wall_xi (n, 6, 3) (ora_contacts)."""
        cap = max(16, 4 * self.n)
        while True:
            ij = np.zeros(2 * cap, np.int32)
            xi = np.zeros(3 * cap)
            won = np.zeros(6 * self.n, np.uint8)
            wxi = np.zeros(18 * self.n)
            m = lib().ora_contacts(self.h, _p(ij, C.c_int), _p(xi), cap, _p(won, C.c_ubyte), _p(wxi))
            if m <= cap:
                return {"ids": ij[: 2 * m].reshape(-1, 2).astype(np.uint32), "xi": xi[: 3 * m].reshape(-1, 3),
                        "wall_on": won.reshape(self.n, 6), "wall_xi": wxi.reshape(self.n, 6, 3)}
            cap = int(m)

    def set_contacts(self, ct):
        ij = np.ascontiguousarray(ct["ids"], dtype=np.int32).reshape(-1)
        xi = np.ascontiguousarray(ct["xi"], dtype=np.float64).reshape(-1)
        won = np.ascontiguousarray(ct["wall_on"], dtype=np.uint8).reshape(-1)
        wxi = np.ascontiguousarray(ct["wall_xi"], dtype=np.float64).reshape(-1)
        if lib().ora_set_contacts(self.h, _p(ij, C.c_int), _p(xi), len(ij) // 2, _p(won, C.c_ubyte), _p(wxi)) != 0:
            raise ValueError("bad contact pairs")

    def state(self):
        keys = ("x", "y", "z", "vx", "vy", "vz", "wx", "wy", "wz", "nh", "nm", "nw", "nfe", "mass")
        out = {k: np.zeros(self.n) for k in keys}
        out["eps"] = np.zeros(self.n_cells)
        lib().ora_get(self.h, *[_p(out[k]) for k in keys], _p(out["eps"]))
        if self.energy:
            for k in ("Tp", "qrx", "mcp"):
                out[k] = np.zeros(self.n)
            lib().ora_get_energy(self.h, _p(out["Tp"]), _p(out["qrx"]), _p(out["mcp"]))
        return out


# ---------------------------------------------------------------- point functions
def e_cgp(e_p, k):
    return lib().ora_e_cgp(e_p, k)


def zeta(e):
    return lib().ora_zeta(e)


def keq(i, T):
    return lib().ora_keq(i, T)


def gas_props(T, p, xh2, xh2o, xn2, mu_override=0.0):
    r, m = C.c_double(), C.c_double()
    lib().ora_gas_props(T, p, xh2, xh2o, xn2, mu_override, C.byref(r), C.byref(m))
    return r.value, m.value


def fuller(T, p, i, j):
    return lib().ora_fuller(T, p, i, j)


def wilke_h2(T, p, xh2, xh2o, xn2):
    return lib().ora_wilke_h2(T, p, xh2, xh2o, xn2)


def knudsen_h2(T, d_pore_cm):
    return lib().ora_knudsen_h2(T, d_pore_cm)


def pore_diff(T, p, xh2, xh2o, xn2, d_pore_cm):
    return lib().ora_pore_diff(T, p, xh2, xh2o, xn2, d_pore_cm)


def layer_porosity(ore):
    xi = np.zeros(4)
    s = ore_struct(ore)
    lib().ora_layer_porosity(C.byref(s), _p(xi))
    return xi


def sherwood(eps, Re, Sc):
    return lib().ora_sherwood(eps, Re, Sc)


def film(T, p, xh2, xh2o, xn2, mu_override, eps, slip, dp):
    return lib().ora_film(T, p, xh2, xh2o, xn2, mu_override, eps, slip, dp)


def beta_over_epsp(eps, rho, mu, slip, dp, printed=0):
    return lib().ora_beta_over_epsp(eps, rho, mu, slip, dp, int(printed))


def beta_ganser_over_epsp(eps, rho, mu, slip, dp, psi, Dbed, printed=False):
    return lib().ora_beta_ganser_over_epsp(eps, rho, mu, slip, dp, psi, Dbed, int(printed))


def ladder(active, A, B, F, x, xeq):
    act = np.ascontiguousarray(active, dtype=np.int32)
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    xe = np.ascontiguousarray(xeq, dtype=np.float64)
    r = np.zeros(3)
    Q, S = C.c_double(), C.c_double()
    lib().ora_ladder(_p(act, C.c_int), _p(A), _p(B), float(F), float(x), _p(xe), _p(r), C.byref(Q), C.byref(S))
    return r, Q.value, S.value


def react_point(env, sp):
    e = np.ascontiguousarray(env, dtype=np.float64)
    assert e.shape == (18,)
    s = np.ascontiguousarray(sp, dtype=np.float64).copy()
    c = lib().ora_react_point(_p(e), _p(s))
    return s, c


def fov(sp, kind):
    """Overall reduction degree of one state (nh, nm, nw, nfe), eq. e2-18 / e2-19."""
    s = np.ascontiguousarray(sp, dtype=np.float64)
    assert s.shape == (4,)
    return lib().ora_fov(_p(s), int(kind))


# species: 0 H2, 1 H2O, 2 N2, 3 Fe2O3, 4 Fe3O4, 5 FeO, 6 Fe (Table C1)
def h_mol(sp, T):
    return lib().ora_h_mol(int(sp), float(T))


def cp_mol(sp, T):
    return lib().ora_cp_mol(int(sp), float(T))


def lambda_g(T, xh2, xh2o, xn2):
    return lib().ora_lambda_g(T, xh2, xh2o, xn2)


def cp_g(T, xh2, xh2o, xn2):
    return lib().ora_cp_g(T, xh2, xh2o, xn2)


def nusselt(eps, Re, Pr):
    return lib().ora_nusselt(eps, Re, Pr)
