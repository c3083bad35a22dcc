"""Seeded synthetic inputs for the many-body MD force path.

This module only *generates inputs*: lattices, Gaussian displacements, Maxwell
velocities, potential parameters and the lookup tables that the method reads
(Hou et al., Section 3.3: the density and pair tables are built once on the host
and copied to the device).  It evaluates none of the method's steps (binning,
neighbour lists, density, embedding, forces, integration, adjoint).  Both the
HIP path and the CPU oracle consume exactly the arrays produced here.

Units: Angstrom, eV, fs, amu.  Arrays are float64 unless stated.

The five workloads
  fs256      FCC 4x4x4 (256 atoms), analytic Finnis-Sinclair, 100 NVE steps
  bcc128k    BCC 40^3 (128,000 atoms), 5,000-knot cubic spline tables
  fcc4m      FCC 100^3 (4,000,000 atoms), analytic second-moment tight binding
  batch2048  2,048 uneven FCC boxes n^3, n in {3..8}, spline tables of bcc128k
  adjoint64  64 BCC 5^3 boxes (250 atoms each), B-spline potential parameters
  alloy      binary FCC 100^3 (4,000,000 atoms), two species, per-type-pair tables
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

# Physical constants (CODATA 2018 exact/recommended values).
EV = 1.602176634e-19          # J
AMU = 1.66053906660e-27       # kg
KB_EV = 8.617333262e-5        # eV/K
# Acceleration unit: (eV/Angstrom)/amu in Angstrom/fs^2 (eV/Angstrom = e*1e10 N,
# 1 m/s^2 = 1e-20 Angstrom/fs^2), about 9.6485e-3.
KAPPA = EV / AMU * 1e-10

MASS_CU = 63.546
MASS_FE = 55.845

SEED_BASE = 12126332
ESCALE = 0.1

# Potential kinds (mirrors the C ABI enum values).
POT_FS = 1
POT_SMTB = 2
POT_SPLINE = 3
POT_BSPLINE = 4

FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


@dataclass
class Potential:
    """Potential description shared by both implementations.

    kind     one of POT_FS, POT_SMTB, POT_SPLINE, POT_BSPLINE
    rc       force cutoff (Angstrom)
    params   analytic parameters
               FS:   [c, d, c0, c1, c2, A]
                     phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2) (r < c), f(r) = (r-d)^2 (r < d),
                     F(rho) = -A sqrt(rho)
               SMTB: [A, xi, p, q, r0]
                     V(r) = 2A exp(-p(r/r0-1)), rho(r) = xi^2 exp(-2q(r/r0-1)), F = -sqrt(rho)
    tables   SPLINE: three arrays [n_int, 4] of per-interval cubic coefficients
                     (a, b, c, d) with S = a + b t + c t^2 + d t^3, t in [0, 1),
                     for phi(r), f(r), F(rho), each on a uniform grid [lo, hi].
             BSPLINE: three arrays [64] of uniform cubic B-spline coefficients
                     (61 intervals on [lo, hi]) for phi(r), f(r), F(rho).
    lo, hi   grid ranges of the three tables (phi, f, F)
    """
    kind: int
    rc: float
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    tables: tuple = ()
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (0.0, 0.0, 0.0)
    n_types: int = 1         # SPLINE with T > 1 species: tables[0] V^(ab) [T*T, n, 4],
                             # tables[1] rho^(ab) [T*T, n, 4] (density at an a atom from
                             # a b atom), tables[2] F^(a) [T, n, 4]; index a*T + b
    rc_pair: np.ndarray = None  # [T, T] cutoff of each pair of types, symmetric, at most
                                # rc (None: rc for every pair)


@dataclass
class Workload:
    name: str
    box_offset: np.ndarray      # int64 [B+1]
    box_len: np.ndarray         # float64 [B, 3] (cubic boxes: all three equal)
    pos: np.ndarray             # float64 [N, 3]
    vel: np.ndarray             # float64 [N, 3]
    mass: float
    dt: float
    skin: float
    pot: Potential
    steps: int
    lattice_const: float = 0.0
    structure: str = ""
    extra: dict = field(default_factory=dict)
    types: np.ndarray = None     # int32 [N] species of each atom (several species only)
    type_mass: np.ndarray = None  # float64 [T] mass of each species (amu)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_boxes(self) -> int:
        return int(self.box_len.shape[0])


# ----------------------------------------------------------------------------- geometry

def lattice(structure: str, ncell: int, a: float) -> np.ndarray:
    """Sites of an ncell^3 cubic supercell, ordered by (ix, iy, iz, basis)."""
    basis = FCC_BASIS if structure == "fcc" else BCC_BASIS
    g = np.arange(ncell, dtype=np.float64)
    ix, iy, iz = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return sites * a


def shells(structure: str, a: float, rmax: float):
    """Neighbour shells (distance, count) of the infinite lattice up to rmax.

    Pure enumeration of lattice vectors; used only to choose potential
    parameters (zero-pressure condition) and as test geometry.
    """
    basis = FCC_BASIS if structure == "fcc" else BCC_BASIS
    m = int(np.ceil(rmax / a)) + 1
    g = np.arange(-m, m + 1, dtype=np.float64)
    ix, iy, iz = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    pts = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    d = np.sqrt((pts ** 2).sum(axis=1))
    d = d[(d > 1e-9) & (d < rmax)]
    key = np.round(d, 9)
    r, cnt = np.unique(key, return_counts=True)
    return r, cnt


# ----------------------------------------------------------------------------- initial state

def maxwell_velocities(rng: np.random.Generator, n: int, mass: float, temp: float) -> np.ndarray:
    """Gaussian velocities at temperature temp, zero centre-of-mass velocity,
    rescaled to exactly temp with 3n-3 degrees of freedom."""
    sigma = np.sqrt(KB_EV * temp * KAPPA / mass)
    v = rng.normal(0.0, sigma, size=(n, 3))
    v -= v.mean(axis=0)
    ekin = 0.5 * mass * (v ** 2).sum() / KAPPA
    t_now = 2.0 * ekin / ((3 * n - 3) * KB_EV)
    v *= np.sqrt(temp / t_now)
    return v


def _displace(rng, sites, sigma):
    return sites + rng.normal(0.0, sigma, size=sites.shape)


# ----------------------------------------------------------------------------- potentials

def _fs_derivs(r, c, c0, c1, c2):
    """phi'(r) and f'(r) of the FS forms; used only for parameter selection."""
    poly = c0 + c1 * r + c2 * r * r
    dphi = 2.0 * (r - c) * poly + (r - c) ** 2 * (c1 + 2.0 * c2 * r)
    df = 2.0 * (r - c)
    return dphi, df


def draw_fs(rng: np.random.Generator, structure: str, a: float, cut: float) -> np.ndarray:
    """Seeded Finnis-Sinclair parameters [c, d, c0, c1, c2, A] with c = d = cut.

    c0 ~ U[0.5, 1.5], c1 ~ U[-0.5, 0], c2 ~ U[-0.05, 0.05], all then multiplied
    by the energy scale ESCALE; A follows from the zero-pressure condition of the
    perfect lattice at the stated lattice constant,
    A = sqrt(rho0) * sum_s n_s phi'(r_s) r_s / sum_s n_s f'(r_s) r_s.
    Draws are repeated (same stream) until A > 0 and phi(r_1) > 0.
    With cutoffs near 5 Angstrom the unscaled forms are about ten times stiffer
    than a real metal; ESCALE = 0.1 brings the lattice stiffness to the usual
    range, so that thermal displacements stay near the stated temperature.
    """
    r, n = shells(structure, a, cut)
    for _ in range(1000):
        c0 = rng.uniform(0.5, 1.5) * ESCALE
        c1 = rng.uniform(-0.5, 0.0) * ESCALE
        c2 = rng.uniform(-0.05, 0.05) * ESCALE
        rho0 = float((n * (r - cut) ** 2).sum())
        dphi, df = _fs_derivs(r, cut, c0, c1, c2)
        num = float((n * dphi * r).sum())
        den = float((n * df * r).sum())
        A = np.sqrt(rho0) * num / den
        phi1 = (r[0] - cut) ** 2 * (c0 + c1 * r[0] + c2 * r[0] ** 2)
        if A > 0.0 and phi1 > 0.0:
            return np.array([cut, cut, c0, c1, c2, A])
    raise RuntimeError("no admissible FS parameters")


def _cubic_table(x, y, bc):
    """Per-interval cubic coefficients (a, b, c, d) in the local variable
    t = (x - x_m)/h of the interpolating cubic spline through (x, y)."""
    from scipy.interpolate import CubicSpline
    cs = CubicSpline(x, y, bc_type=bc)
    h = x[1] - x[0]
    c = cs.c  # [4, n_int], powers (x-x_m)^3, ^2, ^1, ^0
    tab = np.empty((x.size - 1, 4))
    tab[:, 0] = c[3]
    tab[:, 1] = c[2] * h
    tab[:, 2] = c[1] * h * h
    tab[:, 3] = c[0] * h * h * h
    return np.ascontiguousarray(tab)


def spline_tables_from_fs(par: np.ndarray, rho_hi: float, knots: int = 5000,
                          r_hi: float = None) -> Potential:
    """Tabulated EAM: clamped cubic interpolating splines through `knots`
    uniform samples of the FS forms (phi and f on [0, r_hi], r_hi = c unless
    given, the forms zero beyond c; F on [0, rho_hi]; F has a natural end at 0
    and a clamped end at rho_hi)."""
    c, d, c0, c1, c2, A = par
    r_hi = float(c) if r_hi is None else float(r_hi)
    r = np.linspace(0.0, r_hi, knots)
    phi = np.where(r < c, (r - c) ** 2 * (c0 + c1 * r + c2 * r * r), 0.0)
    f = np.where(r < d, (r - d) ** 2, 0.0)
    dphi0, _ = _fs_derivs(0.0, c, c0, c1, c2)
    t_phi = _cubic_table(r, phi, ((1, dphi0), (1, 0.0)))
    t_f = _cubic_table(r, f, ((1, -2.0 * d), (1, 0.0)))
    rho = np.linspace(0.0, rho_hi, knots)
    F = -A * np.sqrt(rho)
    t_F = _cubic_table(rho, F, ((2, 0.0), (1, -A / (2.0 * np.sqrt(rho_hi)))))
    return Potential(kind=POT_SPLINE, rc=r_hi, tables=(t_phi, t_f, t_F),
                     lo=(0.0, 0.0, 0.0), hi=(r_hi, r_hi, float(rho_hi)),
                     params=np.asarray(par, dtype=np.float64))


def bspline_from_fs(par: np.ndarray, r_lo: float, r_hi: float, rho_hi: float,
                    ncoef: int = 64) -> Potential:
    """Uniform cubic B-spline coefficients (ncoef per function, ncoef-3
    intervals) taken as samples of the FS forms at the B-spline centres
    (Schoenberg's variation-diminishing choice), clamped into the grid range."""
    c, d, c0, c1, c2, A = par
    nint = ncoef - 3

    def centres(lo, hi):
        h = (hi - lo) / nint
        return np.clip(lo + (np.arange(ncoef) - 1.0) * h, lo, hi)

    rr = centres(r_lo, r_hi)
    th_phi = np.where(rr < c, (rr - c) ** 2 * (c0 + c1 * rr + c2 * rr * rr), 0.0)
    th_f = np.where(rr < d, (rr - d) ** 2, 0.0)
    pp = centres(0.0, rho_hi)
    th_F = -A * np.sqrt(pp)
    return Potential(kind=POT_BSPLINE, rc=float(r_hi), tables=(th_phi, th_f, th_F),
                     lo=(r_lo, r_lo, 0.0), hi=(r_hi, r_hi, rho_hi))


def smtb_cu(rc: float = 5.85) -> Potential:
    """Second-moment tight-binding parameters of the fcc4m workload."""
    return Potential(kind=POT_SMTB, rc=rc,
                     params=np.array([0.0855, 1.224, 10.96, 2.278, 2.556]))


# ----------------------------------------------------------------------------- workloads

def _single_box(name, structure, ncell, a, sigma, temp, mass, pot, steps, seed,
                dt=1.0, skin=0.3, rng=None):
    rng = rng or np.random.Generator(np.random.PCG64(seed))
    sites = lattice(structure, ncell, a)
    pos = _displace(rng, sites, sigma)
    vel = maxwell_velocities(rng, sites.shape[0], mass, temp)
    L = ncell * a
    return Workload(name=name, box_offset=np.array([0, sites.shape[0]], dtype=np.int64),
                    box_len=np.full((1, 3), L), pos=pos, vel=vel, mass=mass, dt=dt,
                    skin=skin, pot=pot, steps=steps, lattice_const=a, structure=structure)


def fs256(ncell: int = 4) -> Workload:
    """FCC 4x4x4 (256 atoms), a = 3.615, analytic FS with c = d = 4.95,
    sigma 0.05, 300 K, dt 1 fs, 100 NVE steps, skin 0.3."""
    ss = np.random.SeedSequence(SEED_BASE + 0)
    rng = np.random.Generator(np.random.PCG64(ss))
    par = draw_fs(rng, "fcc", 3.615, 4.95)
    pot = Potential(kind=POT_FS, rc=4.95, params=par)
    return _single_box("fs256", "fcc", ncell, 3.615, 0.05, 300.0, MASS_CU, pot, 100,
                       None, rng=rng)


def _c2_potential():
    ss = np.random.SeedSequence(SEED_BASE + 1)
    rng = np.random.Generator(np.random.PCG64(ss))
    par = draw_fs(rng, "bcc", 2.8665, 5.3)
    r, n = shells("bcc", 2.8665, 5.3)
    rho0 = float((n * (r - 5.3) ** 2).sum())
    return spline_tables_from_fs(par, rho_hi=2.0 * rho0), rng


def bcc128k(ncell: int = 40) -> Workload:
    """BCC 40^3 (128,000 atoms), a = 2.8665, 5,000-knot cubic spline tables
    sampled from a seeded FS (cutoff 5.3), sigma 0.05, 600 K, 1,000 steps."""
    pot, rng = _c2_potential()
    return _single_box("bcc128k", "bcc", ncell, 2.8665, 0.05, 600.0, MASS_FE, pot, 1000,
                       None, rng=rng)


def fcc4m(ncell: int = 100) -> Workload:
    """FCC 100^3 (4,000,000 atoms), a = 3.615, SMTB (A 0.0855 eV, xi 1.224 eV,
    p 10.96, q 2.278, r0 2.556), cutoff 5.85 (five shells, 78 neighbours),
    sigma 0.05, 300 K, 200 steps.  Smaller ncell gives the same material in a
    smaller box (used for tests)."""
    ss = np.random.SeedSequence(SEED_BASE + 2)
    rng = np.random.Generator(np.random.PCG64(ss))
    return _single_box("fcc4m", "fcc", ncell, 3.615, 0.05, 300.0, MASS_CU, smtb_cu(), 200,
                       None, rng=rng)


def batch2048(n_boxes: int = 2048, nmin: int = 3, nmax: int = 8) -> Workload:
    """2,048 independent periodic FCC boxes n^3 (n uniform in {3..8}),
    a = 3.615, per-box temperature U[300, 1200] K, sigma 0.05, the spline
    tables of bcc128k, 1,000 steps."""
    pot, _ = _c2_potential()
    ss = np.random.SeedSequence(SEED_BASE + 3)
    kids = ss.spawn(n_boxes + 1)
    g = np.random.Generator(np.random.PCG64(kids[0]))
    ns = g.integers(nmin, nmax + 1, size=n_boxes)
    temps = g.uniform(300.0, 1200.0, size=n_boxes)
    a = 3.615
    pos, vel, lens, off = [], [], [], [0]
    for b in range(n_boxes):
        rng = np.random.Generator(np.random.PCG64(kids[b + 1]))
        sites = lattice("fcc", int(ns[b]), a)
        pos.append(_displace(rng, sites, 0.05))
        vel.append(maxwell_velocities(rng, sites.shape[0], MASS_FE, float(temps[b])))
        lens.append(ns[b] * a)
        off.append(off[-1] + sites.shape[0])
    return Workload(name="batch2048", box_offset=np.array(off, dtype=np.int64),
                    box_len=np.repeat(np.array(lens)[:, None], 3, axis=1),
                    pos=np.concatenate(pos), vel=np.concatenate(vel), mass=MASS_FE, dt=1.0,
                    skin=0.3, pot=pot, steps=1000, lattice_const=a, structure="fcc",
                    extra={"ncell": ns, "temps": temps})


MASS_AG = 107.8682


def alloy_tables(pars, chis, rho_hi: float, knots: int = 5000) -> Potential:
    """Tabulated EAM for several species from per-species FS forms (each with
    its own cutoff c_a = d_a) and density strengths chi: V^(aa) the species'
    own pair term, V^(ab) = (V^(aa) + V^(bb))/2 for a != b, rho^(ab)(r) =
    chi_b f_b(r) (an atom's density is the sum of the functions of its
    neighbours' species), F^(a) = -(A_a / sqrt(chi_a)) sqrt(rho), so that each
    pure species is its FS form.  Clamped cubic interpolating splines through
    `knots` samples on the grid [0, max c_a] shared by all tables, as in
    spline_tables_from_fs.  Cutoffs per pair of types: RCUT(a, b) =
    max(c_a, c_b), beyond which every table of the pair vanishes."""
    T = len(pars)
    cs = [float(p[0]) for p in pars]
    assert all(float(p[1]) == float(p[0]) for p in pars)
    c = max(cs)
    single = []
    for p, chi in zip(pars, chis):
        q = np.array(p, dtype=np.float64)
        q[5] /= np.sqrt(chi)
        single.append(spline_tables_from_fs(q, rho_hi, knots, r_hi=c))
    V = np.empty((T * T,) + single[0].tables[0].shape)
    R = np.empty((T * T,) + single[0].tables[1].shape)
    F = np.empty((T,) + single[0].tables[2].shape)
    for a in range(T):
        F[a] = single[a].tables[2]
        for b in range(T):
            V[a * T + b] = 0.5 * (single[a].tables[0] + single[b].tables[0])
            R[a * T + b] = chis[b] * single[b].tables[1]
    rcp = np.array([[max(ca, cb) for cb in cs] for ca in cs])
    return Potential(kind=POT_SPLINE, rc=c, tables=(V, R, F), lo=single[0].lo,
                     hi=single[0].hi, n_types=T, rc_pair=None if (rcp == c).all() else rcp)


def alloy(ncell: int = 100, frac: float = 0.3, cuts=(5.3, 5.0)) -> Workload:
    """Random substitutional binary FCC alloy: 100^3 cells (4,000,000 atoms),
    a = 3.615, a fraction `frac` of the sites species 1 (mass 107.8682), the
    rest species 0 (mass 63.546); two seeded FS species with cutoffs `cuts`
    (5.3 and 5.0 Angstrom: species 1 reaches its third shell only), each with
    A from its own zero-pressure condition at a, density strengths 1 and 1.6,
    tabulated on 5,000 knots with alloy_tables (so RCUT(a, b) = 5.3 except
    RCUT(1, 1) = 5.0); sigma 0.05, 300 K.  Smaller ncell gives the same
    material in a smaller box."""
    ss = np.random.SeedSequence(SEED_BASE + 5)
    kids = ss.spawn(3)
    a = 3.615
    pars = [draw_fs(np.random.Generator(np.random.PCG64(kids[k])), "fcc", a, cuts[k])
            for k in range(2)]
    r, n = shells("fcc", a, max(cuts))
    rho0 = float((n * (r - max(cuts)) ** 2).sum())
    chis = (1.0, 1.6)
    pot = alloy_tables(pars, chis, rho_hi=2.0 * max(chis) * rho0)
    rng = np.random.Generator(np.random.PCG64(kids[2]))
    sites = lattice("fcc", ncell, a)
    types = (rng.random(sites.shape[0]) < frac).astype(np.int32)
    mass_t = np.array([MASS_CU, MASS_AG])
    pos = _displace(rng, sites, 0.05)
    # Maxwell velocities per species, then the whole box's momentum removed and
    # the kinetic energy set to 300 K with 3N - 3 degrees of freedom
    vel = np.zeros_like(pos)
    for t in range(2):
        sel = types == t
        vel[sel] = rng.normal(0.0, np.sqrt(KB_EV * 300.0 * KAPPA / mass_t[t]),
                              size=(int(sel.sum()), 3))
    m = mass_t[types][:, None]
    vel -= (m * vel).sum(axis=0) / m.sum()
    ekin = 0.5 * float((m * vel * vel).sum()) / KAPPA
    vel *= np.sqrt(1.5 * (sites.shape[0] - 1) * KB_EV * 300.0 / ekin)
    L = ncell * a
    return Workload(name="alloy", box_offset=np.array([0, sites.shape[0]], dtype=np.int64),
                    box_len=np.full((1, 3), L), pos=pos, vel=vel, mass=MASS_CU, dt=1.0,
                    skin=0.3, pot=pot, steps=200, lattice_const=a, structure="fcc",
                    types=types, type_mass=mass_t)


def adjoint64(n_boxes: int = 64, ncell: int = 5) -> Workload:
    """64 BCC 5^3 boxes (250 atoms each), a = 2.8665, sigma 0.1.

    extra["target_pot"]: the seeded reference FS (stream 0) whose forces and
    energies are the fitting targets; pot: the B-spline starting point theta0
    (64 coefficients per function) sampled from a second seeded FS (stream 1);
    extra["w"] = 0.1 is the energy weight of the loss."""
    ss = np.random.SeedSequence(SEED_BASE + 4)
    kids = ss.spawn(n_boxes + 2)
    par_t = draw_fs(np.random.Generator(np.random.PCG64(kids[0])), "bcc", 2.8665, 5.3)
    par_0 = draw_fs(np.random.Generator(np.random.PCG64(kids[1])), "bcc", 2.8665, 5.3)
    r, n = shells("bcc", 2.8665, 5.3)
    rho0 = float((n * (r - 5.3) ** 2).sum())
    pot0 = bspline_from_fs(par_0, 1.5, 5.3, 2.0 * rho0)
    target = Potential(kind=POT_FS, rc=5.3, params=par_t)
    a = 2.8665
    pos, off = [], [0]
    for b in range(n_boxes):
        rng = np.random.Generator(np.random.PCG64(kids[b + 2]))
        sites = lattice("bcc", ncell, a)
        pos.append(_displace(rng, sites, 0.1))
        off.append(off[-1] + sites.shape[0])
    P = np.concatenate(pos)
    L = ncell * a
    return Workload(name="adjoint64", box_offset=np.array(off, dtype=np.int64),
                    box_len=np.full((n_boxes, 3), L), pos=P, vel=np.zeros_like(P),
                    mass=MASS_FE, dt=1.0, skin=0.3, pot=pot0, steps=0, lattice_const=a,
                    structure="bcc", extra={"target_pot": target, "w": 0.1})


WORKLOADS = {"fs256": fs256, "bcc128k": bcc128k, "fcc4m": fcc4m,
             "batch2048": batch2048, "adjoint64": adjoint64, "alloy": alloy}
