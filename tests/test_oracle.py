"""Pins of the CPU oracle against facts fixed by the mathematics, not by the oracle.

Each test names the plausible mistakes it would catch.  All run on the CPU.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1212_6332_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SHELLS = json.load(open(os.path.join(HERE, "golden", "lattice_shells.json")))


def golden_shells(structure, a, rmax):
    g = SHELLS[structure]
    r = np.sqrt(np.array(g["r_over_a_squared"])) * a
    n = np.array(g["count"])
    keep = r < rmax
    return r[keep], n[keep]


# --------------------------------------------------------------------------- lists

def py_brute_list(pos, L, r_list):
    """Independent pure-Python O(N^2) neighbour sets with the same rounding:
    minimum image per component, r^2 = (dx*dx + dy*dy) + dz*dz, strict <."""
    n = len(pos)
    out = []
    r2max = r_list * r_list
    for i in range(n):
        row = []
        for j in range(n):
            if j == i:
                continue
            d = []
            for k in range(3):
                t = float(pos[j][k]) - float(pos[i][k])
                if t > 0.5 * L:
                    t -= L
                elif t < -0.5 * L:
                    t += L
                d.append(t)
            r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            if r2 < r2max:
                row.append(j)
        out.append(row)
    return out


@pytest.mark.parametrize("structure,ncell,a,r_list", [
    ("fcc", 2, 3.615, 3.5),     # one cell per dimension (L/r_list < 3)
    ("bcc", 3, 2.8665, 4.2),    # two cells per dimension
    ("fcc", 3, 3.615, 3.0),     # three cells per dimension
])
def test_list_tiny_matches_python_brute_force(orc, structure, ncell, a, r_list):
    """Catches: wrong minimum image, self in the list, duplicated stencil cells
    for fewer than three cells per dimension, a non-strict cutoff test."""
    rng = np.random.default_rng(1)
    L = ncell * a
    pos = orc.wrap(W.lattice(structure, ncell, a) + rng.normal(0, 0.15, (ncell ** 3 * (4 if structure == "fcc" else 2), 3)), L)
    count, ids = orc.neighbor_list(pos, L, r_list)
    ref = py_brute_list(pos.tolist(), L, r_list)
    for i, row in enumerate(ref):
        assert count[i] == len(row)
        assert list(ids[i, :count[i]]) == row


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_list_cells_equals_brute_force(orc, seed):
    """Linked cells (Section 3.2) against the all-pairs list on displaced boxes."""
    rng = np.random.default_rng(seed)
    ncell = 6 + seed
    a = 3.615
    L = ncell * a
    pos = orc.wrap(W.lattice("fcc", ncell, a) + rng.normal(0, 0.2, (4 * ncell ** 3, 3)), L)
    c1, i1 = orc.neighbor_list(pos, L, 6.15)
    c2, i2 = orc.neighbor_list(pos, L, 6.15, brute=True)
    assert np.array_equal(c1, c2)
    assert np.array_equal(i1, i2)


@pytest.mark.parametrize("structure,a,r_list,expect", [
    ("fcc", 3.615, 6.15, 78),   # five shells
    ("fcc", 3.615, 5.25, 54),   # four shells
    ("fcc", 3.615, 5.6, 54),
    ("bcc", 2.8665, 5.6, 58),   # five shells
])
def test_perfect_lattice_neighbour_counts(orc, structure, a, r_list, expect):
    r, n = golden_shells(structure, a, r_list)
    assert int(n.sum()) == expect
    ncell = 6
    pos = W.lattice(structure, ncell, a)
    count, _ = orc.neighbor_list(pos, ncell * a, r_list)
    assert np.all(count == expect)


def test_generator_shells_agree_with_golden():
    for structure, a in (("fcc", 3.615), ("bcc", 2.8665)):
        r, n = W.shells(structure, a, 6.3)
        gr, gn = golden_shells(structure, a, 6.3)
        assert np.allclose(r, gr) and np.array_equal(n, gn)


def test_wrap_into_box(orc):
    rng = np.random.default_rng(3)
    L = 10.0
    pos = rng.uniform(-25.0, 35.0, (500, 3))
    pos[0] = [-1e-300, -0.0, L]
    w = orc.wrap(pos, L)
    assert np.all(w >= 0.0) and np.all(w < L)
    k = (pos - w) / L
    assert np.allclose(k, np.round(k), atol=1e-12)


# --------------------------------------------------------------------------- potentials

def smtb_closed_form(a, rc):
    A, xi, p, q, r0 = 0.0855, 1.224, 10.96, 2.278, 2.556
    r, n = golden_shells("fcc", a, rc)
    rho = float((n * xi * xi * np.exp(-2 * q * (r / r0 - 1))).sum())
    rep = float((n * A * np.exp(-p * (r / r0 - 1))).sum())
    return rho, rep - math.sqrt(rho)


def test_smtb_perfect_lattice_closed_form(orc):
    """Cohesive energy and density of perfect FCC under the five-shell SMTB
    (eqs. 1-2 with F = -sqrt(rho)).  Catches: missing 1/2 on the pair sum, a
    wrong exponent, a density summed over the wrong shells."""
    a, ncell = 3.615, 7
    pot = orc.Pot(W.smtb_cu())
    pos = W.lattice("fcc", ncell, a)
    r = orc.forces(pos, ncell * a, pot)
    rho, ecoh = smtb_closed_form(a, 5.85)
    assert np.allclose(r["rho"], rho, rtol=1e-13, atol=0)
    assert abs(r["E"] / len(pos) - ecoh) <= 1e-12 * abs(ecoh)
    assert abs(ecoh - (-3.543628)) < 5e-7   # five-shell Cu value
    assert np.abs(r["f"]).max() <= 1e-12


def test_fs_perfect_lattice_closed_form(orc):
    wl = W.fs256()
    c, d, c0, c1, c2, A = wl.pot.params
    r, n = golden_shells("fcc", 3.615, 4.95)
    rho = float((n * (r - d) ** 2).sum())
    pair = float((n * (r - c) ** 2 * (c0 + c1 * r + c2 * r * r)).sum())
    ecoh = -A * math.sqrt(rho) + 0.5 * pair
    pos = W.lattice("fcc", 4, 3.615)
    out = orc.forces(pos, 4 * 3.615, orc.Pot(wl.pot))
    assert np.allclose(out["rho"], rho, rtol=1e-13, atol=0)
    assert abs(out["E"] / 256 - ecoh) <= 1e-12 * abs(ecoh)
    assert np.abs(out["f"]).max() <= 1e-12
    # zero pressure at the stated lattice constant: dE/da = 0 (FD in a)
    def e_of(s):
        return orc.forces(W.lattice("fcc", 4, 3.615 * s), 4 * 3.615 * s, orc.Pot(wl.pot))["E"]
    h = 1e-5
    assert abs((e_of(1 + h) - e_of(1 - h)) / (2 * h)) < 1e-6 * 256


def test_spline_table_interpolates_and_reproduces_quadratic(orc):
    """The 5,000-knot table of bcc128k: values at knots equal the samples, and
    f(r) = (r-d)^2 (a quadratic) is reproduced exactly by the clamped cubic."""
    wl = W.bcc128k(ncell=2)
    pot = orc.Pot(wl.pot)
    c, d, c0, c1, c2, A = wl.pot.params
    h = c / 4999
    for k in (0, 1, 17, 2500, 4998):
        r = k * h
        v, dv, _ = pot.eval(1, r)
        assert abs(v - (r - d) ** 2) < 1e-12
        assert abs(dv - 2 * (r - d)) < 1e-9
        v, dv, _ = pot.eval(0, r)
        assert abs(v - (r - c) ** 2 * (c0 + c1 * r + c2 * r * r)) < 1e-12
    for r in np.linspace(2.0, 5.2, 57):
        v, dv, _ = pot.eval(1, r)
        assert abs(v - (r - d) ** 2) < 1e-11
        # phi is quartic: cubic-spline error <= (5/384) h^4 max|phi''''|
        v, dv, _ = pot.eval(0, r)
        exact = (r - c) ** 2 * (c0 + c1 * r + c2 * r * r)
        assert abs(v - exact) <= 5 / 384 * h ** 4 * 24 * abs(c2) + 1e-13
    rho = 120.0
    v, dv, ddv = pot.eval(2, rho)
    assert abs(v + A * math.sqrt(rho)) < 1e-9
    assert abs(dv + A / (2 * math.sqrt(rho))) < 1e-7


def test_bspline_basis_identities(orc):
    """Uniform cubic B-spline evaluation: partition of unity (all theta = 1 gives
    1 with zero derivative) and linear reproduction (theta_k = x at the centres
    gives S(x) = x), plus exact linearity in theta."""
    K, lo, hi = 64, 1.5, 5.3
    h = (hi - lo) / (K - 3)
    centres = lo + (np.arange(K) - 1.0) * h
    ones = W.Potential(kind=W.POT_BSPLINE, rc=hi, tables=(np.ones(K), centres.copy(), np.zeros(K)),
                       lo=(lo, lo, 0.0), hi=(hi, hi, 1.0))
    pot = orc.Pot(ones)
    for x in np.linspace(lo, hi - 1e-9, 41):
        v, dv, _ = pot.eval(0, x)
        assert abs(v - 1.0) < 1e-14 and abs(dv) < 1e-12
        v, dv, _ = pot.eval(1, x)
        assert abs(v - x) < 1e-13 and abs(dv - 1.0) < 1e-12
    rng = np.random.default_rng(5)
    th1, th2 = rng.normal(size=K), rng.normal(size=K)
    p1 = orc.Pot(W.Potential(W.POT_BSPLINE, hi, tables=(th1, th1, th1), lo=(lo, lo, lo), hi=(hi, hi, hi)))
    p2 = orc.Pot(W.Potential(W.POT_BSPLINE, hi, tables=(th2, th2, th2), lo=(lo, lo, lo), hi=(hi, hi, hi)))
    p3 = orc.Pot(W.Potential(W.POT_BSPLINE, hi, tables=(2 * th1 - th2,) * 3, lo=(lo,) * 3, hi=(hi,) * 3))
    for x in (1.7, 2.9, 4.123, 5.2):
        assert abs(p3.eval(0, x)[0] - (2 * p1.eval(0, x)[0] - p2.eval(0, x)[0])) < 1e-12
        # derivative against central differences
        e = 1e-6
        fd = (p1.eval(2, x + e)[0] - p1.eval(2, x - e)[0]) / (2 * e)
        assert abs(fd - p1.eval(2, x)[1]) < 1e-6
        fd2 = (p1.eval(2, x + e)[1] - p1.eval(2, x - e)[1]) / (2 * e)
        assert abs(fd2 - p1.eval(2, x)[2]) < 1e-4


def test_embedding_derivatives(orc):
    wl = W.fs256()
    pot = orc.Pot(wl.pot)
    A = wl.pot.params[5]
    for rho in (0.5, 20.0, 86.0):
        F, dF, ddF = pot.eval(2, rho)
        assert abs(F + A * math.sqrt(rho)) < 1e-13 * A * math.sqrt(rho) + 1e-15
        assert abs(dF + A / (2 * math.sqrt(rho))) < 1e-14
        assert abs(ddF - A / (4 * rho * math.sqrt(rho))) < 1e-14
    assert pot.eval(2, 0.0) == (0.0, 0.0, 0.0)


# --------------------------------------------------------------------------- forces

def _fd_check(orc, pos, L, pot, atoms, h=1e-5):
    out = orc.forces(pos, L, pot)
    E = abs(out["E"])
    fmax = np.abs(out["f"]).max()
    eps = np.finfo(float).eps
    for i in atoms:
        for k in range(3):
            p1 = pos.copy(); p1[i, k] += h
            p2 = pos.copy(); p2[i, k] -= h
            fd = -(orc.energy_direct(p1, L, pot) - orc.energy_direct(p2, L, pot)) / (2 * h)
            tol = 1e-7 * fmax + 20 * eps * E / h
            assert abs(fd - out["f"][i, k]) <= tol, (i, k, fd, out["f"][i, k])


def test_forces_are_minus_energy_gradient_fs(orc):
    """f = -dE/dx (eq. 3 from eq. 2).  Catches: a dropped F'(rho_j) term,
    a wrong sign of r_ij, a missing factor on the pair derivative."""
    wl = W.fs256()
    L = wl.box_len[0, 0]
    _fd_check(orc, orc.wrap(wl.pos, L), L, orc.Pot(wl.pot), atoms=[0, 77, 255])


def test_forces_are_minus_energy_gradient_smtb(orc):
    wl = W.fcc4m(ncell=4)
    L = wl.box_len[0, 0]
    pos = orc.wrap(wl.pos, L)
    _fd_check(orc, pos, L, orc.Pot(wl.pot), atoms=[3, 100])


def test_forces_are_minus_energy_gradient_spline(orc):
    wl = W.bcc128k(ncell=4)
    L = wl.box_len[0, 0]
    _fd_check(orc, orc.wrap(wl.pos, L), L, orc.Pot(wl.pot), atoms=[5, 64])


def test_list_passes_equal_direct_sums(orc):
    """Density/force passes over a fresh list with r_list > rc give the
    all-pairs result of eqs. (2)-(3)."""
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pos = orc.wrap(wl.pos, L)
    pot = orc.Pot(wl.pot)
    a = orc.forces(pos, L, pot)
    b = orc.forces_direct(pos, L, pot)
    assert np.allclose(a["rho"], b["rho"], rtol=1e-14, atol=0)
    assert np.abs(a["f"] - b["f"]).max() <= 1e-13 * np.abs(b["f"]).max()
    assert abs(a["E"] - b["E"]) <= 1e-13 * abs(b["E"])


def test_total_force_vanishes(orc):
    """Newton's third law holds pairwise, so the forces sum to zero."""
    for wl in (W.fs256(), W.fcc4m(ncell=5)):
        L = wl.box_len[0, 0]
        out = orc.forces(orc.wrap(wl.pos, L), L, orc.Pot(wl.pot))
        assert np.abs(out["f"].sum(axis=0)).max() <= 1e-12 * np.abs(out["f"]).sum()


def test_sampled_forces_match_full_pass(orc):
    wl = W.fcc4m(ncell=6)
    L = wl.box_len[0, 0]
    pos = orc.wrap(wl.pos, L)
    pot = orc.Pot(wl.pot)
    full = orc.forces(pos, L, pot)
    idx = np.array([0, 1, 13, 400, len(pos) - 1])
    s = orc.sample_forces(pos, L, pot, idx)
    assert np.allclose(s["rho"], full["rho"][idx], rtol=1e-13, atol=0)
    assert np.abs(s["f"] - full["f"][idx]).max() <= 1e-12 * np.abs(full["f"]).max()
    assert np.allclose(s["e_atom"], full["e_atom"][idx], rtol=1e-13, atol=0)
    c, ids = orc.sample_list(pos, L, 6.15, idx)
    c2, ids2 = orc.neighbor_list(pos, L, 6.15)
    assert np.array_equal(c, c2[idx]) and np.array_equal(ids, ids2[idx])


# --------------------------------------------------------------------------- dynamics

def test_nve_conservation_and_dt_squared(orc):
    """Velocity Verlet is second order: the energy error shrinks ~4x per halving
    of dt, and stays below 1e-4 eV/atom over 100 fs (FS forms vanish with zero
    slope at the cutoff)."""
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pot = orc.Pot(wl.pot)
    errs = []
    for dt in (1.0, 0.5, 0.25):
        _, v, ep, ek, _ = orc.vv(wl.pos, wl.vel, L, pot, wl.mass, dt, wl.skin, int(round(100 / dt)))
        E = ep + ek
        errs.append(np.abs(E - E[0]).max() / wl.n_atoms)
        assert np.abs(v.sum(axis=0)).max() <= 1e-10 * np.abs(v).sum()
    assert errs[0] < 1e-4
    assert 2.5 < errs[0] / errs[1] < 6.5 and 2.5 < errs[1] / errs[2] < 6.5


def test_time_reversibility(orc):
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pot = orc.Pot(wl.pot)
    x0 = orc.wrap(wl.pos, L)
    x1, v1, *_ = orc.vv(x0, wl.vel, L, pot, wl.mass, 1.0, wl.skin, 50)
    x2, v2, *_ = orc.vv(x1, -v1, L, pot, wl.mass, 1.0, wl.skin, 50)
    d = x2 - x0
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + wl.vel).max() < 1e-9


def test_box_independence(orc):
    """Multi-box evaluation: perturbing one box leaves the others unchanged."""
    wl = W.adjoint64(n_boxes=3)
    wl.pot = wl.extra["target_pot"]
    a = orc.forces_multi(wl)
    pos = wl.pos.copy()
    pos[260] += 0.05
    b = orc.forces_multi(wl, pos=pos)
    assert np.array_equal(a["f"][:250], b["f"][:250])
    assert np.array_equal(a["f"][500:], b["f"][500:])
    assert not np.array_equal(a["f"][250:500], b["f"][250:500])


# --------------------------------------------------------------------------- adjoint

def _loss_and_parts(orc, wl, pot, targets, w):
    out = orc.forces_multi(wl, pot=pot)
    dF = out["f"] - targets["f"]
    dE = out["E_box"] - targets["E_box"]
    return float((dF ** 2).sum() + w * (dE ** 2).sum()), out


def test_adjoint_matches_finite_differences(orc):
    """Gradient of the force/energy-matching loss with respect to the 3x64
    B-spline coefficients, against central differences (h = 1e-6).  The loss
    is exactly quadratic in the phi and F coefficients, so only rounding
    limits those blocks; the f block carries O(h^2) truncation."""
    wl = W.adjoint64(n_boxes=2)
    w = wl.extra["w"]
    targets = orc.forces_multi(wl, pot=orc.Pot(wl.extra["target_pot"]))
    pot = orc.Pot(wl.pot)
    L0, out = _loss_and_parts(orc, wl, pot, targets, w)
    g = 2.0 * (out["f"] - targets["f"])
    e = 2.0 * w * (out["E_box"] - targets["E_box"])
    grad = np.zeros(192)
    for b, s, L in orc.boxes(wl):
        orc.adjoint(orc.wrap(wl.pos[s], L), L, pot, g[s], e[b], gtheta=grad)
    th = [np.array(t, dtype=float) for t in wl.pot.tables]
    h = 1e-6
    rng = np.random.default_rng(0)
    picks = sorted(set(list(rng.choice(192, 40, replace=False)) + [10, 70, 140]))
    eps = np.finfo(float).eps
    for k in picks:
        fn, kk = divmod(k, 64)
        vals = []
        for sgn in (+1, -1):
            t2 = [t.copy() for t in th]
            t2[fn][kk] += sgn * h
            p2 = W.Potential(W.POT_BSPLINE, wl.pot.rc, tables=tuple(t2), lo=wl.pot.lo, hi=wl.pot.hi)
            vals.append(_loss_and_parts(orc, wl, orc.Pot(p2), targets, w)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        tol = 1e-6 * np.abs(grad).max() + 50 * eps * abs(L0) / h
        assert abs(fd - grad[k]) <= tol, (k, fd, grad[k], tol)
