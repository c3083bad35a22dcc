"""Thin ctypes binding of libmd.so (C ABI in include/md.h).

Argument marshalling only: every step of the force path runs in the HIP
kernels of libmd.so.  PyTorch supplies device memory (float64 CUDA tensors)
and the current stream.  There is no CPU fallback: if the library or a GPU
is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import functools
import os

import numpy as np
import torch  # imported first: libmd.so then binds to the HIP runtime torch loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd.so")

MD_OK = 0
MD_ERR_ARG, MD_ERR_BOX, MD_ERR_NLIST_OVERFLOW, MD_ERR_TABLE_RANGE = -1, -2, -3, -4
MD_ERR_NONFINITE, MD_ERR_DEVICE, MD_ERR_STATE, MD_ERR_NOMEM, MD_ERR_SCRATCH = -5, -6, -7, -8, -9
(MD_FLAG_NLIST_OVERFLOW, MD_FLAG_TABLE_RANGE, MD_FLAG_NONFINITE, MD_FLAG_TILE_OVERFLOW,
 MD_FLAG_BOX_RANGE) = 1, 2, 4, 8, 16
MD_POT_FS, MD_POT_SMTB, MD_POT_SPLINE, MD_POT_BSPLINE = 1, 2, 3, 4
MD_OPT_BATCHED, MD_OPT_BATCH_BLOCK, MD_OPT_USE_GRAPH, MD_OPT_GRAPH_STEPS, MD_OPT_TILED = 1, 2, 3, 4, 5
(MD_OPT_BATCH_PACK, MD_OPT_BATCH_ORDER, MD_OPT_TILE_SHAPE, MD_OPT_TILE_SHAPES,
 MD_OPT_TILE_DIMS) = 6, 7, 8, 9, 10
(MD_PASS_BUILD, MD_PASS_DENSITY, MD_PASS_FORCE, MD_PASS_KICK_DRIFT, MD_PASS_FORCE_STEP,
 MD_PASS_PRESSURE) = 0, 1, 2, 3, 4, 5


class MDError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().md_strerror(code).decode()} ({code})")


class md_potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_params", C.c_int32), ("rc", C.c_double),
                ("params", C.c_void_p), ("tab", C.c_void_p * 3), ("n_tab", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("n_types", C.c_int32), ("rc_pair", C.c_void_p)]


class md_system(C.Structure):
    _fields_ = [("n_boxes", C.c_int32), ("max_neighbors", C.c_int32),
                ("box_offset", C.c_void_p), ("box_len", C.c_void_p), ("mass", C.c_double),
                ("dt", C.c_double), ("skin", C.c_double)]


_lib = None
_SIGS = {
    "md_create": ([C.POINTER(md_system), C.POINTER(md_potential), C.POINTER(C.c_void_p)], C.c_int),
    "md_destroy": ([C.c_void_p], None),
    "md_strerror": ([C.c_int], C.c_char_p),
    "md_set_potential": ([C.c_void_p, C.POINTER(md_potential), C.c_void_p], C.c_int),
    "md_set_theta": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_set_state": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_get_state": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_bind": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_build_neighbors": ([C.c_void_p, C.c_void_p], C.c_int),
    "md_density": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_embed": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_forces": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_step": ([C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "md_kinetic": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_get_neighbors": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "md_max_neighbors": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "md_set_max_neighbors": ([C.c_void_p, C.c_int32], C.c_int),
    "md_status": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_int64)], C.c_int),
    "md_adjoint": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_set_option": ([C.c_void_p, C.c_int32, C.c_int64], C.c_int),
    "md_get_option": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int64)], C.c_int),
    "md_time_pass": ([C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_double)],
                     C.c_int),
    "md_pressure": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_set_barostat": ([C.c_void_p, C.c_double, C.c_double, C.c_double], C.c_int),
    "md_get_box": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_set_thermostat": ([C.c_void_p, C.c_double, C.c_double], C.c_int),
    "md_set_types": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "md_set_frozen": ([C.c_void_p, C.c_void_p], C.c_int),
    "md_workspace_size": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "md_autotune": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "md_create_in": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "md_forces_static": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                          C.c_void_p], C.c_int),
    "md_static_bytes": ([], C.c_size_t),
}


def lib():
    """Load libmd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1212_6332_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code, where):
    if code != MD_OK:
        raise MDError(code, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(a, device):
    t = torch.as_tensor(a, dtype=torch.float64, device=device)
    return t.contiguous()


class _PotHolder:
    """Keeps the host arrays referenced by an md_potential alive."""

    def __init__(self, pot):
        self.params = np.ascontiguousarray(np.asarray(pot.params, dtype=np.float64).ravel())
        self.tabs = [np.ascontiguousarray(np.asarray(t, dtype=np.float64)) for t in pot.tables]
        T = int(getattr(pot, "n_types", 1) or 1)
        s = md_potential()
        s.n_types = T
        s.kind = int(pot.kind)
        s.n_params = int(self.params.size)
        s.rc = float(pot.rc)
        s.params = self.params.ctypes.data if self.params.size else None
        for k, t in enumerate(self.tabs):
            s.tab[k] = t.ctypes.data
            # several species: [tables, intervals, 4] -> intervals per table
            s.n_tab[k] = int(t.shape[1] if T > 1 else t.shape[0])
        for k in range(3):
            s.lo[k] = float(pot.lo[k])
            s.hi[k] = float(pot.hi[k])
        rcp = getattr(pot, "rc_pair", None)
        self.rcp = None if rcp is None else np.ascontiguousarray(rcp, dtype=np.float64).ravel()
        s.rc_pair = None if self.rcp is None else self.rcp.ctypes.data
        self.s = s


def _mutates(fn):
    """Methods that change the state, the list or the settings of a context
    count up `System.epoch`: work captured in a graph before them no longer
    describes the context."""
    @functools.wraps(fn)
    def wrap(self, *a, **k):
        self.epoch = getattr(self, "epoch", 0) + 1
        return fn(self, *a, **k)
    return wrap


def forces_static(box_offset, box_len, pot, mass, pos, dt=1.0, skin=0.3, max_neighbors=0):
    """md_forces_static: forces [N, 3], per-atom energies [N] and per-box
    energies [B] of `pos`, with every device buffer in the library's static
    device array (no allocation by the library; torch allocates the outputs
    here).  Synchronises the current stream."""
    lib()
    dev = torch.device("cuda", torch.cuda.current_device())
    off = np.ascontiguousarray(np.asarray(box_offset, dtype=np.int64))
    bl = np.asarray(box_len, dtype=np.float64)
    bl = np.ascontiguousarray(bl[:, 0] if bl.ndim == 2 else bl)
    holder = _PotHolder(pot)
    sysd = md_system(n_boxes=int(bl.size), max_neighbors=int(max_neighbors),
                     box_offset=off.ctypes.data, box_len=bl.ctypes.data, mass=float(mass),
                     dt=float(dt), skin=float(skin))
    n = int(off[-1])
    p = _dev_f64(pos, dev)
    f = torch.empty(n, 3, dtype=torch.float64, device=dev)
    e = torch.empty(n, dtype=torch.float64, device=dev)
    eb = torch.empty(int(bl.size), dtype=torch.float64, device=dev)
    _check(lib().md_forces_static(C.byref(sysd), C.byref(holder.s), _ptr(p), _ptr(f), _ptr(e),
                                  _ptr(eb), _stream()), "md_forces_static")
    return f, e, eb


def static_bytes():
    """Size of the static device array md_forces_static works in."""
    return int(lib().md_static_bytes())


class System:
    """One md_ctx: B periodic cubic boxes sharing a potential.

    box_offset [B+1] (int), box_len [B] or [B, 3] (cubic: first column used),
    pot: a workloads.Potential (or any object with kind, rc, params, tables,
    lo, hi).  All per-atom tensors are float64 on the current CUDA device, in
    original atom order, shaped [N, 3] for vectors.
    """

    def __init__(self, box_offset, box_len, pot, mass, dt=1.0, skin=0.3, max_neighbors=0,
                 workspace=None):
        lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.box_offset = np.ascontiguousarray(np.asarray(box_offset, dtype=np.int64))
        bl = np.asarray(box_len, dtype=np.float64)
        self.box_len = np.ascontiguousarray(bl[:, 0] if bl.ndim == 2 else bl)
        self.n_boxes = int(self.box_len.size)
        self.n_atoms = int(self.box_offset[-1])
        self._pot = _PotHolder(pot)
        self.pot = pot
        sysd = md_system()
        sysd.n_boxes = self.n_boxes
        sysd.max_neighbors = int(max_neighbors)
        sysd.box_offset = self.box_offset.ctypes.data
        sysd.box_len = self.box_len.ctypes.data
        sysd.mass, sysd.dt, sysd.skin = float(mass), float(dt), float(skin)
        self._sysd = sysd
        h = C.c_void_p()
        if workspace is None:
            _check(lib().md_create(C.byref(sysd), C.byref(self._pot.s), C.byref(h)), "md_create")
        else:
            # every device buffer of the context comes from this tensor
            nbytes = workspace.numel() * workspace.element_size()
            _check(lib().md_create_in(C.byref(sysd), C.byref(self._pot.s),
                                      C.c_void_p(workspace.data_ptr()), nbytes, C.byref(h)),
                   "md_create_in")
        self._workspace = workspace
        self._h = h
        self.epoch = 0

    @staticmethod
    def workspace_size(box_offset, box_len, pot, mass, dt=1.0, skin=0.3, max_neighbors=0):
        """Device bytes a context for these arguments needs (md_workspace_size)."""
        lib()
        off = np.ascontiguousarray(np.asarray(box_offset, dtype=np.int64))
        bl = np.asarray(box_len, dtype=np.float64)
        bl = np.ascontiguousarray(bl[:, 0] if bl.ndim == 2 else bl)
        holder = _PotHolder(pot)
        sysd = md_system(n_boxes=int(bl.size), max_neighbors=int(max_neighbors),
                         box_offset=off.ctypes.data, box_len=bl.ctypes.data, mass=float(mass),
                         dt=float(dt), skin=float(skin))
        n = C.c_size_t()
        _check(lib().md_workspace_size(C.byref(sysd), C.byref(holder.s), C.byref(n)),
               "md_workspace_size")
        return int(n.value)

    @classmethod
    def workload_workspace_size(cls, W, pot=None, **kw):
        return cls.workspace_size(W.box_offset, W.box_len, pot or W.pot, W.mass, W.dt, W.skin,
                                  **kw)

    @classmethod
    def from_workload(cls, W, pot=None, **kw):
        s = cls(W.box_offset, W.box_len, pot or W.pot, W.mass, W.dt, W.skin, **kw)
        if getattr(W, "types", None) is not None and int(getattr(s.pot, "n_types", 1)) > 1:
            s.set_types(W.types, W.type_mass)
        return s

    @_mutates
    def autotune(self):
        """md_autotune: the fastest block shape of the persistent multi-box
        stepper (workgroup size, box packing, visiting order), or elsewhere the
        per-atom passes or the tiled passes with one of the candidate tile
        shapes (a shape whose halo overflows a tile's LDS on the current state
        is passed over); returns the stepper's workgroup size."""
        b = C.c_int32()
        _check(lib().md_autotune(self._h, _stream(), C.byref(b)), "md_autotune")
        return int(b.value)

    @_mutates
    def set_frozen(self, frozen):
        """Atom states: a nonzero entry (host array, original order) freezes that atom;
        None frees every atom."""
        if frozen is None:
            _check(lib().md_set_frozen(self._h, None), "md_set_frozen")
            return
        f = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))
        if f.size != self.n_atoms:
            raise ValueError("one flag per atom")
        _check(lib().md_set_frozen(self._h, f.ctypes.data_as(C.c_void_p)), "md_set_frozen")

    @_mutates
    def set_types(self, types, type_mass=None):
        """Species of every atom (host array, original order) and per-species masses."""
        t = np.ascontiguousarray(np.asarray(types, dtype=np.int32))
        if t.size != self.n_atoms:
            raise ValueError("one type per atom")
        m = None if type_mass is None else np.ascontiguousarray(np.asarray(type_mass,
                                                                             dtype=np.float64))
        _check(lib().md_set_types(self._h, t.ctypes.data_as(C.c_void_p),
                                  None if m is None else m.ctypes.data_as(C.c_void_p)),
               "md_set_types")

    @_mutates
    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize()
            lib().md_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def _f64(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    @_mutates
    def set_state(self, pos, vel=None):
        p = _dev_f64(pos, self.device)
        v = None if vel is None else _dev_f64(vel, self.device)
        _check(lib().md_set_state(self._h, _ptr(p), _ptr(v), _stream()), "md_set_state")
        torch.cuda.current_stream().synchronize()

    @_mutates
    def bind(self, pos, vel=None):
        """md_bind: float64 CUDA tensors [N, 3] (contiguous) become the state
        of record; md_step writes back into them.  bind(None) unbinds."""
        if pos is None:
            _check(lib().md_bind(self._h, None, None, _stream()), "md_bind")
            self._bound = None
            return
        for t in (pos, vel):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                                      and tuple(t.shape) == (self.n_atoms, 3)):
                raise ValueError("bound buffers: contiguous float64 CUDA tensors [N, 3]")
        _check(lib().md_bind(self._h, _ptr(pos), _ptr(vel), _stream()), "md_bind")
        self._bound = (pos, vel)   # keeps the memory alive while bound

    def get_state(self):
        p, v = self._f64(self.n_atoms, 3), self._f64(self.n_atoms, 3)
        _check(lib().md_get_state(self._h, _ptr(p), _ptr(v), _stream()), "md_get_state")
        return p, v

    @_mutates
    def set_potential(self, pot):
        holder = _PotHolder(pot)
        _check(lib().md_set_potential(self._h, C.byref(holder.s), _stream()), "md_set_potential")
        self._pot, self.pot = holder, pot

    def set_theta(self, theta):
        t = _dev_f64(theta, self.device).reshape(-1)
        # the same memory at the same version as the last upload (e.g. the
        # backward pass of the forward that set them): nothing to do.  Views
        # share the version counter, so an in-place change through any of
        # them is seen; the held tensor keeps the memory from being reused.
        last = getattr(self, "_theta", None)
        if (last is not None and t.data_ptr() == last[0].data_ptr()
                and t.numel() == last[0].numel() and t._version == last[1]):
            return
        _check(lib().md_set_theta(self._h, _ptr(t), _stream()), "md_set_theta")
        # the copy is stream ordered; holding t keeps its memory until the next upload
        self._theta = (t, t._version)

    @_mutates
    def build_neighbors(self):
        _check(lib().md_build_neighbors(self._h, _stream()), "md_build_neighbors")

    def density(self):
        rho = self._f64(self.n_atoms)
        _check(lib().md_density(self._h, _ptr(rho), _stream()), "md_density")
        return rho

    def embed(self):
        F, Fp = self._f64(self.n_atoms), self._f64(self.n_atoms)
        _check(lib().md_embed(self._h, _ptr(F), _ptr(Fp), _stream()), "md_embed")
        return F, Fp

    def forces(self, energy=True, atom_energy=True):
        """Forces [N, 3]; with `energy` also per-atom energies (None unless
        `atom_energy`) and per-box energies."""
        f = self._f64(self.n_atoms, 3)
        e = self._f64(self.n_atoms) if energy and atom_energy else None
        eb = self._f64(self.n_boxes) if energy else None
        _check(lib().md_forces(self._h, _ptr(f), _ptr(e), _ptr(eb), _stream()), "md_forces")
        return (f, e, eb) if energy else f

    @_mutates
    def step(self, nsteps):
        _check(lib().md_step(self._h, int(nsteps), _stream()), "md_step")

    def kinetic(self):
        ke = self._f64(self.n_boxes)
        _check(lib().md_kinetic(self._h, _ptr(ke), _stream()), "md_kinetic")
        return ke

    def neighbors(self, max_cols=None):
        cols = int(max_cols or self.max_neighbors)
        counts = torch.zeros(self.n_atoms, dtype=torch.int32, device=self.device)
        ids = torch.full((self.n_atoms, cols), -1, dtype=torch.int32, device=self.device)
        _check(lib().md_get_neighbors(self._h, _ptr(counts), _ptr(ids), cols, _stream()),
               "md_get_neighbors")
        return counts, ids

    @property
    def max_neighbors(self):
        v = C.c_int32()
        _check(lib().md_max_neighbors(self._h, C.byref(v)), "md_max_neighbors")
        return v.value

    @_mutates
    def set_max_neighbors(self, mn):
        _check(lib().md_set_max_neighbors(self._h, int(mn)), "md_set_max_neighbors")

    def status(self):
        """(flags, builds, steps); synchronises and clears the status bits."""
        fl = C.c_uint32()
        cnt = (C.c_int64 * 2)()
        _check(lib().md_status(self._h, _stream(), C.byref(fl), cnt), "md_status")
        return fl.value, cnt[0], cnt[1]

    def adjoint(self, g, e):
        g = _dev_f64(g, self.device)
        e = _dev_f64(e, self.device)
        K = int(self._pot.s.n_tab[0])
        out = self._f64(3 * K)
        _check(lib().md_adjoint(self._h, _ptr(g), _ptr(e), _ptr(out), _stream()), "md_adjoint")
        return out

    def pressure(self):
        """Per-box pressure of eq. (6) (eV/Angstrom^3) and pair virial W (eV)."""
        p = torch.empty(self.n_boxes, dtype=torch.float64, device=self.device)
        w = torch.empty(self.n_boxes, dtype=torch.float64, device=self.device)
        _check(lib().md_pressure(self._h, _ptr(p), _ptr(w), _stream()), "md_pressure")
        return p, w

    @_mutates
    def set_barostat(self, p0, tau, beta):
        """Berendsen barostat of eq. (5) in md_step; tau <= 0 switches it off."""
        _check(lib().md_set_barostat(self._h, float(p0), float(tau), float(beta)),
               "md_set_barostat")

    @_mutates
    def set_thermostat(self, t_e, tau_t):
        """Electron-gas friction of eq. (4) in md_step; tau_t <= 0 switches it off."""
        _check(lib().md_set_thermostat(self._h, float(t_e), float(tau_t)), "md_set_thermostat")

    def box(self):
        """Current box edges (numpy, length B)."""
        out = np.zeros(self.n_boxes)
        _check(lib().md_get_box(self._h, out.ctypes.data_as(C.c_void_p), _stream()), "md_get_box")
        return out

    @_mutates
    def time_pass(self, which, reps):
        """Mean duration (ms) of one launch of a pass, from HIP events on the stream."""
        ms = C.c_double()
        _check(lib().md_time_pass(self._h, int(which), int(reps), _stream(), C.byref(ms)),
               "md_time_pass")
        return ms.value

    @_mutates
    def set_option(self, key, value):
        _check(lib().md_set_option(self._h, int(key), int(value)), "md_set_option")

    def get_option(self, key):
        v = C.c_int64()
        _check(lib().md_get_option(self._h, int(key), C.byref(v)), "md_get_option")
        return v.value
