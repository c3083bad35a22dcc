"""CPU oracle (test infrastructure only).

ctypes front end of `oracle.c`.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the HIP product
path never does.  Every function works on one periodic cubic box in the
caller's (original) atom order; multi-box helpers loop over boxes, each box
independent of the others (the paper's multiple-box scheme keeps boxes
independent, Section 4.4).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")

KAPPA = 1.602176634e-19 / 1.66053906660e-27 * 1e-10
KB_EV = 8.617333262e-5


def build(force: bool = True, out: str = None, tuned: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP, no FP contraction).

    tuned: -O3 -march=native for the host that runs the build (the timed
    CPU-baseline copy, built where it runs, into `out`); otherwise -O2 for
    any x86-64 host.  The arithmetic is the same either way: contraction
    stays off and no fast-math option is given."""
    dst = out or _LIB
    if force or not os.path.exists(dst):
        opt = ["-O3", "-march=native"] if tuned else ["-O2"]
        cmd = ["gcc", *opt, "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp", "-shared",
               "-fPIC", _SRC, "-o", dst + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(dst + ".tmp", dst)
    return dst


def use_tuned(directory: str) -> str:
    """Build the -O3 -march=native copy into `directory` and load it in place
    of the default library (for timing the oracle on the host it runs on)."""
    global _lib, _LIB
    path = build(out=os.path.join(directory, "liboracle_native.so"), tuned=True)
    _LIB, _lib = path, None
    return path


def set_threads(n: int) -> None:
    """OpenMP threads used by later calls."""
    lib().orc_set_threads(int(n))


class _Pot(C.Structure):
    _fields_ = [("kind", C.c_int), ("rc", C.c_double), ("par", C.c_void_p),
                ("tab", C.c_void_p * 3), ("ntab", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER(_Pot)
        i64, dbl, i32 = C.c_int64, C.c_double, C.c_int
        L.orc_pot_eval.argtypes = [P, i32, dbl, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)]
        L.orc_wrap.argtypes = [i64, _f64p, _f64p, _f64p, dbl]
        for fn in (L.orc_list_cells, L.orc_list_brute):
            fn.argtypes = [i64, _f64p, _f64p, _f64p, dbl, dbl, i32, _i32p, _i32p]
            fn.restype = i32
        L.orc_density.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, _i32p, _i32p, i32, _f64p]
        L.orc_embed.argtypes = [i64, P, _f64p, _f64p, _f64p, _f64p]
        L.orc_forces.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, _i32p, _i32p, i32, _f64p,
                                 _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_energy_direct.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P]
        L.orc_energy_direct.restype = dbl
        L.orc_forces_direct.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, _f64p, _f64p, _f64p,
                                        _f64p, _f64p]
        L.orc_sample_forces.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, i64, _i64p, _f64p,
                                        _f64p, _f64p, _f64p, _f64p]
        L.orc_sample_list.argtypes = [i64, _f64p, _f64p, _f64p, dbl, dbl, i64, _i64p, i32,
                                      _i32p, _i32p]
        L.orc_rlist.argtypes = [dbl, dbl, dbl]
        L.orc_rlist.restype = dbl
        L.orc_vv.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, dbl, P, dbl, dbl,
                             dbl, i32, i32, C.c_void_p, C.c_void_p]
        L.orc_vv.restype = i32
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_adjoint.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, _i32p, _i32p, i32, _f64p,
                                  _f64p, _f64p, dbl, _f64p]
        L.orc_virial.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P, _i32p, _i32p, i32, _f64p]
        L.orc_virial.restype = dbl
        L.orc_virial_direct.argtypes = [i64, _f64p, _f64p, _f64p, dbl, P]
        L.orc_virial_direct.restype = dbl
        L.orc_vv_baro.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                  C.POINTER(dbl), P, dbl, dbl, dbl, i32, i32, dbl, dbl, dbl,
                                  dbl, dbl, C.c_void_p]
        L.orc_vv_baro.restype = i32
        L.orc_vv_thermo.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, dbl, P, dbl,
                                    dbl, dbl, i32, i32, dbl, dbl, C.c_void_p, C.c_void_p]
        L.orc_vv_thermo.restype = i32
        _lib = L
    return _lib


class Pot:
    """Holds a potential (from workloads.Potential) in oracle form."""

    def __init__(self, pot):
        self.pot = pot
        self._par = np.ascontiguousarray(np.asarray(pot.params, dtype=np.float64).ravel())
        if self._par.size == 0:
            self._par = np.zeros(1)
        self._tabs = [np.ascontiguousarray(np.asarray(t, dtype=np.float64)) for t in pot.tables]
        s = _Pot()
        s.kind = int(pot.kind)
        s.rc = float(pot.rc)
        s.par = self._par.ctypes.data
        for k, t in enumerate(self._tabs):
            s.tab[k] = t.ctypes.data
            s.ntab[k] = t.shape[0]
        for k in range(3):
            s.lo[k] = float(pot.lo[k])
            s.hi[k] = float(pot.hi[k])
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)

    @property
    def rc(self):
        return float(self.pot.rc)

    def eval(self, which: int, x: float):
        v, d1, d2 = C.c_double(), C.c_double(), C.c_double()
        lib().orc_pot_eval(self.ref, which, float(x), C.byref(v), C.byref(d1), C.byref(d2))
        return v.value, d1.value, d2.value


def _xyz(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return (np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
            np.ascontiguousarray(pos[:, 2]))


def rlist(rc: float, skin: float, L: float) -> float:
    return lib().orc_rlist(rc, skin, L)


def wrap(pos, L):
    x, y, z = _xyz(pos)
    lib().orc_wrap(x.size, x, y, z, float(L))
    return np.stack([x, y, z], axis=1)


def neighbor_list(pos, L, r_list, maxn=256, brute=False):
    """Full neighbour list (ascending ids per row).  Returns (count, ids[n, maxn])."""
    x, y, z = _xyz(pos)
    n = x.size
    count = np.zeros(n, dtype=np.int32)
    ids = np.full((n, maxn), -1, dtype=np.int32)
    fn = lib().orc_list_brute if brute else lib().orc_list_cells
    worst = fn(n, x, y, z, float(L), float(r_list), maxn, count, ids)
    if worst > maxn:
        raise ValueError(f"neighbour row overflow: {worst} > {maxn}")
    return count, ids


def forces(pos, L, pot: Pot, count=None, ids=None, skin=0.3):
    """Density, embedding and force passes over a (fresh) list.
    Returns dict rho, F, Fp, Fpp, f[n,3], e_atom, E."""
    x, y, z = _xyz(pos)
    n = x.size
    if count is None:
        count, ids = neighbor_list(pos, L, rlist(pot.rc, skin, L))
    maxn = ids.shape[1]
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    rho = np.zeros(n)
    lib().orc_density(n, x, y, z, float(L), pot.ref, count, ids, maxn, rho)
    F, Fp, Fpp = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_embed(n, pot.ref, rho, F, Fp, Fpp)
    fx, fy, fz, e = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_forces(n, x, y, z, float(L), pot.ref, count, ids, maxn, F, Fp, fx, fy, fz, e)
    return {"rho": rho, "F": F, "Fp": Fp, "Fpp": Fpp, "f": np.stack([fx, fy, fz], axis=1),
            "e_atom": e, "E": float(e.sum())}


def forces_direct(pos, L, pot: Pot):
    x, y, z = _xyz(pos)
    n = x.size
    rho, fx, fy, fz, e = (np.zeros(n) for _ in range(5))
    lib().orc_forces_direct(n, x, y, z, float(L), pot.ref, rho, fx, fy, fz, e)
    return {"rho": rho, "f": np.stack([fx, fy, fz], axis=1), "e_atom": e, "E": float(e.sum())}


def energy_direct(pos, L, pot: Pot) -> float:
    x, y, z = _xyz(pos)
    return lib().orc_energy_direct(x.size, x, y, z, float(L), pot.ref)


def sample_forces(pos, L, pot: Pot, idx):
    x, y, z = _xyz(pos)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.size
    rho, fx, fy, fz, e = (np.zeros(m) for _ in range(5))
    lib().orc_sample_forces(x.size, x, y, z, float(L), pot.ref, m, idx, rho, fx, fy, fz, e)
    return {"rho": rho, "f": np.stack([fx, fy, fz], axis=1), "e_atom": e}


def sample_list(pos, L, r_list, idx, maxn=256):
    x, y, z = _xyz(pos)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    count = np.zeros(idx.size, dtype=np.int32)
    ids = np.full((idx.size, maxn), -1, dtype=np.int32)
    lib().orc_sample_list(x.size, x, y, z, float(L), float(r_list), idx.size, idx, maxn,
                          count, ids)
    return count, ids


def vv(pos, vel, L, pot: Pot, mass, dt, skin, nsteps, maxn=256, energies=True):
    """Velocity-Verlet trajectory of one box.  Returns (pos, vel, epot, ekin, rebuilds)."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    ep = np.zeros(nsteps + 1)
    ek = np.zeros(nsteps + 1)
    nreb = lib().orc_vv(x.size, x, y, z, vx, vy, vz, float(L), pot.ref, float(mass),
                        float(dt), float(skin), int(nsteps), int(maxn),
                        ep.ctypes.data if energies else None,
                        ek.ctypes.data if energies else None)
    if nreb < 0:
        raise ValueError("neighbour row overflow in orc_vv")
    return (np.stack([x, y, z], axis=1), np.stack([vx, vy, vz], axis=1), ep, ek, nreb)


def adjoint(pos, L, pot: Pot, g, e, skin=0.3, gtheta=None):
    """VJP of (forces, box energy) w.r.t. the B-spline coefficients of one box."""
    x, y, z = _xyz(pos)
    count, ids = neighbor_list(pos, L, rlist(pot.rc, skin, L))
    gx, gy, gz = _xyz(g)
    K = pot.s.ntab[0]
    if gtheta is None:
        gtheta = np.zeros(3 * K)
    lib().orc_adjoint(x.size, x, y, z, float(L), pot.ref, count, ids, ids.shape[1], gx, gy, gz,
                      float(e), gtheta)
    return gtheta


# ------------------------------------------------------------------ multi-box

def boxes(W):
    """Yield (b, slice, L) for the boxes of a workload."""
    for b in range(W.n_boxes):
        s = slice(int(W.box_offset[b]), int(W.box_offset[b + 1]))
        yield b, s, float(W.box_len[b, 0])


def forces_multi(W, pos=None, pot=None):
    pos = W.pos if pos is None else pos
    pot = pot or Pot(W.pot)
    n = pos.shape[0]
    out = {"rho": np.zeros(n), "f": np.zeros((n, 3)), "e_atom": np.zeros(n),
           "Fp": np.zeros(n), "E_box": np.zeros(W.n_boxes)}
    for b, s, L in boxes(W):
        r = forces(wrap(pos[s], L), L, pot, skin=W.skin)
        out["rho"][s] = r["rho"]
        out["f"][s] = r["f"]
        out["e_atom"][s] = r["e_atom"]
        out["Fp"][s] = r["Fp"]
        out["E_box"][b] = r["E"]
    return out


def virial(pos, L, pot: Pot, skin=0.3):
    """Pair virial W = sum_{i<j} r_ij . f_ij (eq. 6 for a periodic box) over a
    fresh list."""
    x, y, z = _xyz(pos)
    count, ids = neighbor_list(pos, L, rlist(pot.rc, skin, L))
    r = forces(pos, L, pot, count, ids)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    return float(lib().orc_virial(x.size, x, y, z, float(L), pot.ref, count, ids, ids.shape[1],
                                  r["Fp"]))


def virial_direct(pos, L, pot: Pot):
    x, y, z = _xyz(pos)
    return float(lib().orc_virial_direct(x.size, x, y, z, float(L), pot.ref))


def pressure(pos, vel, L, pot: Pot, mass, skin=0.3):
    """Instantaneous pressure of eq. (6), P = (2 E_kin + W) / (3 V), in eV/Angstrom^3."""
    return (2.0 * kinetic(vel, mass) + virial(pos, L, pot, skin)) / (3.0 * float(L) ** 3)


def vv_baro(pos, vel, L, pot: Pot, mass, dt, skin, nsteps, p0, tau, beta, maxn=256,
            te=0.0, tau_t=0.0):
    """Velocity Verlet with the Berendsen barostat of eq. (5), and the
    electron-gas friction of eq. (4) when tau_t > 0.
    Returns (pos, vel, L, pressures[nsteps + 1], rebuilds)."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    Lc = C.c_double(float(L))
    pr = np.zeros(nsteps + 1)
    nreb = lib().orc_vv_baro(x.size, x, y, z, vx, vy, vz, C.byref(Lc), pot.ref, float(mass),
                             float(dt), float(skin), int(nsteps), int(maxn), float(p0),
                             float(tau), float(beta), float(te), float(tau_t),
                             pr.ctypes.data)
    if nreb < 0:
        raise ValueError("neighbour row overflow in orc_vv_baro")
    return (np.stack([x, y, z], axis=1), np.stack([vx, vy, vz], axis=1), Lc.value, pr, nreb)


def vv_frozen(pos, vel, L, pot: Pot, mass, dt, skin, nsteps, frozen, maxn=256, energies=True):
    """Velocity Verlet with frozen atoms (atom states, Section 3.1): frozen
    atoms keep zero velocity and stay in place.  Returns (pos, vel, epot,
    ekin, rebuilds)."""
    L_ = lib()
    if not hasattr(L_, "_frozen_ready"):
        i32, i64, dbl = C.c_int, C.c_int64, C.c_double
        L_.orc_vv_frozen.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, dbl,
                                     C.c_void_p, dbl, dbl, dbl, i32, i32, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
        L_.orc_vv_frozen.restype = i32
        L_._frozen_ready = True
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    fr = np.ascontiguousarray(frozen, dtype=np.uint8)
    ep = np.zeros(nsteps + 1)
    ek = np.zeros(nsteps + 1)
    nreb = L_.orc_vv_frozen(x.size, x, y, z, vx, vy, vz, float(L), pot.ref, float(mass),
                            float(dt), float(skin), int(nsteps), int(maxn), fr.ctypes.data,
                            ep.ctypes.data if energies else None,
                            ek.ctypes.data if energies else None)
    if nreb < 0:
        raise ValueError("neighbour row overflow in orc_vv_frozen")
    return (np.stack([x, y, z], axis=1), np.stack([vx, vy, vz], axis=1), ep, ek, nreb)


def vv_thermo(pos, vel, L, pot: Pot, mass, dt, skin, nsteps, te, tau, maxn=256, energies=True):
    """Velocity Verlet with the electron-gas friction of eq. (4) (tau <= 0: none).
    Returns (pos, vel, epot, ekin, rebuilds)."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    ep = np.zeros(nsteps + 1)
    ek = np.zeros(nsteps + 1)
    nreb = lib().orc_vv_thermo(x.size, x, y, z, vx, vy, vz, float(L), pot.ref, float(mass),
                               float(dt), float(skin), int(nsteps), int(maxn), float(te),
                               float(tau), ep.ctypes.data if energies else None,
                               ek.ctypes.data if energies else None)
    if nreb < 0:
        raise ValueError("neighbour row overflow in orc_vv_thermo")
    return (np.stack([x, y, z], axis=1), np.stack([vx, vy, vz], axis=1), ep, ek, nreb)


class _Alloy(C.Structure):
    _fields_ = [("ntypes", C.c_int), ("rc", C.c_double), ("V", C.c_void_p), ("rho", C.c_void_p),
                ("F", C.c_void_p), ("nint", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("rcp", C.c_void_p)]


class Alloy:
    """Several-species tables (workloads.Potential with n_types > 1) in oracle form."""

    def __init__(self, pot):
        self.pot = pot
        T = int(pot.n_types)
        self._t = [np.ascontiguousarray(np.asarray(t, dtype=np.float64)) for t in pot.tables]
        assert self._t[0].shape[0] == T * T and self._t[1].shape[0] == T * T
        assert self._t[2].shape[0] == T
        s = _Alloy()
        s.ntypes = T
        s.rc = float(pot.rc)
        s.V, s.rho, s.F = (t.ctypes.data for t in self._t)
        for k in range(3):
            s.nint[k] = self._t[k].shape[1]
            s.lo[k] = float(pot.lo[k])
            s.hi[k] = float(pot.hi[k])
        rcp = getattr(pot, "rc_pair", None)
        self._rcp = None if rcp is None else np.ascontiguousarray(rcp, dtype=np.float64).ravel()
        s.rcp = None if self._rcp is None else self._rcp.ctypes.data
        self._s = s

    @property
    def ref(self):
        return C.byref(self._s)


def _alloy_lib():
    L = lib()
    if not hasattr(L, "_alloy_ready"):
        i32, i64, dbl = C.c_int, C.c_int64, C.c_double
        L.orc_alloy_eval.argtypes = [i64, _f64p, _f64p, _f64p, dbl, C.c_void_p, _i32p,
                                     C.c_void_p, C.c_void_p, i32, C.c_void_p, C.c_void_p, _f64p,
                                     _f64p, _f64p, _f64p, _f64p]
        L.orc_alloy_eval.restype = dbl
        L.orc_alloy_vv.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, dbl,
                                   C.c_void_p, _i32p, _f64p, dbl, dbl, i32, i32, dbl, dbl,
                                   C.c_void_p, C.c_void_p]
        L.orc_alloy_vv.restype = i32
        L.orc_alloy_list.argtypes = [i64, _f64p, _f64p, _f64p, dbl, C.c_void_p, _i32p, dbl, i32,
                                     _i32p, _i32p]
        L.orc_alloy_list.restype = i32
        L._alloy_ready = True
    return L


def alloy_eval(pos, L, pot: Alloy, types, count=None, ids=None):
    """Densities, embedding values, forces, per-atom energies, total energy and
    pair virial of one box with several species (eqs. 1-3 and 6), by the list
    (count, ids) or, when it is None, over all pairs."""
    x, y, z = (np.ascontiguousarray(pos[:, k], dtype=np.float64) for k in range(3))
    n = x.size
    t = np.ascontiguousarray(types, dtype=np.int32)
    out = {k: np.zeros(n) for k in ("rho", "F", "Fp", "fx", "fy", "fz", "e_atom")}
    if count is not None:
        count = np.ascontiguousarray(count, dtype=np.int32)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        cp, ip, maxn = count.ctypes.data, ids.ctypes.data, ids.shape[1]
    else:
        cp, ip, maxn = None, None, 0
    W = _alloy_lib().orc_alloy_eval(n, x, y, z, float(L), pot.ref, t, cp, ip, int(maxn),
                                    out["rho"].ctypes.data, out["F"].ctypes.data, out["Fp"],
                                    out["fx"], out["fy"], out["fz"], out["e_atom"])
    f = np.stack([out.pop("fx"), out.pop("fy"), out.pop("fz")], axis=1)
    out["f"] = f
    out["E"] = float(out["e_atom"].sum())
    out["W"] = float(W)
    return out


def alloy_list(pos, L, pot: Alloy, types, skin, maxn=256):
    """Neighbour list of one box with the list radius taken per pair of types
    (RCUT(a, b) + skin, clamped below L/2): (count, ids[n, maxn]), rows ascending."""
    x, y, z = _xyz(pos)
    n = x.size
    count = np.zeros(n, dtype=np.int32)
    ids = np.full((n, maxn), -1, dtype=np.int32)
    t = np.ascontiguousarray(types, dtype=np.int32)
    worst = _alloy_lib().orc_alloy_list(n, x, y, z, float(L), pot.ref, t, float(skin),
                                        int(maxn), count, ids)
    if worst > maxn:
        raise ValueError(f"neighbour row overflow: {worst} > {maxn}")
    ids[np.arange(maxn)[None, :] >= count[:, None]] = -1
    return count, ids


def alloy_vv(pos, vel, L, pot: Alloy, types, type_mass, dt, skin, nsteps, te=0.0, tau=0.0,
             maxn=256, energies=True):
    """Velocity Verlet for several species (per-type masses; the friction of
    eq. (4) when tau > 0).  Returns (pos, vel, epot, ekin, rebuilds)."""
    x, y, z = _xyz(pos)
    vx, vy, vz = _xyz(vel)
    ep = np.zeros(nsteps + 1)
    ek = np.zeros(nsteps + 1)
    t = np.ascontiguousarray(types, dtype=np.int32)
    m = np.ascontiguousarray(type_mass, dtype=np.float64)
    nreb = _alloy_lib().orc_alloy_vv(x.size, x, y, z, vx, vy, vz, float(L), pot.ref, t, m,
                                     float(dt), float(skin), int(nsteps), int(maxn), float(te),
                                     float(tau), ep.ctypes.data if energies else None,
                                     ek.ctypes.data if energies else None)
    if nreb < 0:
        raise ValueError("neighbour row overflow in orc_alloy_vv")
    return (np.stack([x, y, z], axis=1), np.stack([vx, vy, vz], axis=1), ep, ek, nreb)


def threads() -> int:
    return int(lib().orc_threads())


def kinetic(vel, mass):
    return 0.5 * mass * float((np.asarray(vel) ** 2).sum()) / KAPPA
