"""Pins of the oracle's pressure (eq. 6) and Berendsen barostat (eq. 5).

The virial is taken in its pair form W = sum_{i<j} r_ij . f_ij (the periodic
form of sum_i f_i . r_i), and P = (2 E_kin + W) / (3 V).  Pins:
  * W from the neighbour list equals W summed directly over all pairs;
  * W = -dE/dlambda for a uniform scaling x -> lambda x, L -> lambda L of the
    whole box (the static part of P is -dE/dV), by central differences;
  * W of a perfect FCC lattice under SMTB from the closed form of the
    cohesive energy's derivative with respect to the lattice constant;
  * the barostat with an infinite coupling time reproduces velocity Verlet
    bit for bit, and a compressed box relaxes towards the target pressure.
"""
import json
import math
import os

import numpy as np

from paper_1212_6332_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SHELLS = json.load(open(os.path.join(HERE, "golden", "lattice_shells.json")))


def squeezed(wl, s):
    """The workload's box and positions scaled by s (a uniformly strained state)."""
    L = wl.box_len[0, 0]
    return wl.pos * s, L * s


def min_gap_to_cutoff(pos, L, rc):
    """Smallest |r_ij - rc| over all pairs (minimum image), numpy brute force."""
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    return float(np.abs(r - rc).min())


def test_virial_list_equals_direct_sum(orc):
    for wl in (W.fs256(), W.fcc4m(ncell=4), W.bcc128k(ncell=5)):
        L = wl.box_len[0, 0]
        pos = orc.wrap(wl.pos, L)
        pot = orc.Pot(wl.pot)
        w1, w2 = orc.virial(pos, L, pot), orc.virial_direct(pos, L, pot)
        assert abs(w1 - w2) <= 1e-12 * max(1.0, abs(w2)), (w1, w2)


def _check_dE_dlambda(orc, wl, s, h):
    pos, L = squeezed(wl, s)
    pos = orc.wrap(pos, L)
    pot = orc.Pot(wl.pot)
    # the central difference must not move a pair across the cutoff (the
    # SMTB functions are not zero there)
    assert min_gap_to_cutoff(pos, L, wl.pot.rc) > 4 * h * wl.pot.rc
    E = lambda lam: orc.energy_direct(pos * lam, L * lam, pot)
    fd = -(E(1 + h) - E(1 - h)) / (2 * h)
    w = orc.virial(pos, L, pot)
    eps = np.finfo(float).eps
    tol = 1e-8 * abs(w) + 50 * eps * abs(E(1.0)) / h
    assert abs(fd - w) <= tol, (fd, w)
    return w


def test_virial_is_minus_energy_derivative_under_box_scaling(orc):
    """Static pressure -dE/dV = W / (3V).  Catches: a missing 1/2 (full lists
    count each pair twice), r_ij taken as r_j - r_i, a dropped F'(rho_j)."""
    ws = [_check_dE_dlambda(orc, W.fs256(), 0.97, 1e-6),
          _check_dE_dlambda(orc, W.fcc4m(ncell=4), 0.98, 1e-7),
          _check_dE_dlambda(orc, W.bcc128k(ncell=5), 0.98, 1e-6)]
    assert all(w > 0 for w in ws)   # compressed boxes push outwards


def test_virial_perfect_fcc_smtb_closed_form(orc):
    """W = -dE/dlambda = -N a de_coh/da with the five-shell SMTB cohesive
    energy e(a) = sum_s n_s A e^{-p(r_s/r0-1)} - sqrt(sum_s n_s xi^2 e^{-2q(r_s/r0-1)}),
    r_s = a c_s, differentiated by hand."""
    A, xi, p, q, r0 = 0.0855, 1.224, 10.96, 2.278, 2.556
    for a in (3.55, 3.615):
        g = SHELLS["fcc"]
        c = np.sqrt(np.array(g["r_over_a_squared"]))
        n = np.array(g["count"])
        keep = c * a < 5.85
        c, n = c[keep], n[keep]
        ef = np.exp(-2 * q * (a * c / r0 - 1))
        ev = np.exp(-p * (a * c / r0 - 1))
        rho = float((n * xi * xi * ef).sum())
        drho = float((n * xi * xi * ef * (-2 * q * c / r0)).sum())
        drep = float((n * A * ev * (-p * c / r0)).sum())
        de_da = drep - drho / (2 * math.sqrt(rho))
        ncell = 4
        pos = W.lattice("fcc", ncell, a)
        N = len(pos)
        w = orc.virial(pos, ncell * a, orc.Pot(W.smtb_cu()))
        assert abs(w - (-N * a * de_da)) <= 1e-12 * abs(N * a * de_da), (a, w, -N * a * de_da)


def test_barostat_initial_pressure_and_infinite_coupling_time(orc):
    """With tau -> infinity the scale factor rounds to exactly 1, so the
    barostat trajectory must equal the plain velocity-Verlet one bit for bit;
    its first pressure must equal the standalone pressure of the initial
    state."""
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pot = orc.Pot(wl.pot)
    pos0 = orc.wrap(wl.pos, L)
    x1, v1, L1, pr, nb1 = orc.vv_baro(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30,
                                      p0=0.0, tau=1e300, beta=1.0)
    x2, v2, ep, ek, nb2 = orc.vv(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30)
    assert L1 == L and nb1 == nb2
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    p_init = orc.pressure(pos0, wl.vel, L, pot, wl.mass)
    assert abs(pr[0] - p_init) <= 1e-14 * abs(p_init)


def test_barostat_relaxes_compressed_box(orc):
    """A Cu box compressed by 2 % (SMTB; positive pressure) under P0 = 0
    expands and its pressure falls to a small fraction of the initial value;
    the first step's box edge follows eq. (5) exactly."""
    wl = W.fcc4m(ncell=4)
    pos, L = squeezed(wl, 0.98)
    pot = orc.Pot(wl.pot)
    pos = orc.wrap(pos, L)
    p_init = orc.pressure(pos, wl.vel, L, pot, wl.mass)
    assert p_init > 0
    tau, beta, dt = 100.0, 1.0, wl.dt
    _, _, L1, pr1, _ = orc.vv_baro(pos, wl.vel, L, pot, wl.mass, dt, wl.skin, 1, 0.0, tau, beta)
    assert L1 == L * np.cbrt(1.0 - beta * (dt / tau) * (0.0 - p_init))
    _, _, Ln, pr, _ = orc.vv_baro(pos, wl.vel, L, pot, wl.mass, dt, wl.skin, 400, 0.0, tau, beta)
    assert Ln > L
    assert abs(pr[-100:].mean()) < 0.1 * p_init
