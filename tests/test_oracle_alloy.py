"""Pins of the oracle for several species (eqs. 1-3 with atom types).

Reading: rho_i = sum_j rho^(ab)(r_ij) (density at an a atom contributed by a b
atom), E_i = F^(a)(rho_i) + 1/2 sum_j V^(ab), and the force takes the
derivative of rho_j from rho^(ba).  Pins:
  * one species, and two identical species, reproduce the single-species
    oracle (itself pinned in test_oracle.py);
  * a dimer with linear tables, by hand: which table feeds which density and
    which term of the force;
  * forces are minus the gradient of the energy (central differences) with
    rho^(ab) != rho^(ba), and sum to zero; the pair virial is -dE/dlambda;
  * the list result equals the all-pairs result;
  * velocity Verlet with per-species masses conserves energy and momentum;
  * the friction of eq. (4) drives each species to its own v_e^2 = 3 k_B T_e / m.
"""
import numpy as np

from paper_1212_6332_amd import workloads as W


def one_species(pot1):
    """A single-species spline potential as a one-type table set."""
    V, R, F = (np.asarray(t)[None] for t in pot1.tables)
    return W.Potential(kind=W.POT_SPLINE, rc=pot1.rc, tables=(V, R, F), lo=pot1.lo,
                       hi=pot1.hi, n_types=1)


def small_alloy(ncell=3, frac=0.4, seed=1):
    wl = W.alloy(ncell=ncell, frac=frac)
    return wl, wl.box_len[0, 0]


def test_one_species_equals_spline_oracle(orc):
    wl = W.bcc128k(ncell=5)
    L = wl.box_len[0, 0]
    pos = orc.wrap(wl.pos, L)
    ref = orc.forces_direct(pos, L, orc.Pot(wl.pot))
    got = orc.alloy_eval(pos, L, orc.Alloy(one_species(wl.pot)), np.zeros(wl.n_atoms))
    s = np.abs(ref["f"]).max()
    assert np.abs(got["f"] - ref["f"]).max() <= 1e-14 * s
    assert np.abs(got["rho"] - ref["rho"]).max() <= 1e-14 * np.abs(ref["rho"]).max()
    assert abs(got["E"] - ref["E"]) <= 1e-14 * abs(ref["E"])
    w = orc.virial_direct(pos, L, orc.Pot(wl.pot))
    assert abs(got["W"] - w) <= 1e-12 * max(abs(w), 1.0)


def test_identical_species_equal_one_species(orc):
    wl = W.bcc128k(ncell=5)
    L = wl.box_len[0, 0]
    pos = orc.wrap(wl.pos, L)
    V, R, F = wl.pot.tables
    two = W.Potential(kind=W.POT_SPLINE, rc=wl.pot.rc, tables=(np.stack([V] * 4),
                      np.stack([R] * 4), np.stack([F] * 2)), lo=wl.pot.lo, hi=wl.pot.hi,
                      n_types=2)
    types = np.random.default_rng(0).integers(0, 2, wl.n_atoms)
    a = orc.alloy_eval(pos, L, orc.Alloy(two), types)
    b = orc.alloy_eval(pos, L, orc.Alloy(one_species(wl.pot)), np.zeros(wl.n_atoms))
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["e_atom"], b["e_atom"])


def linear_table(slope, lo, hi, n=8):
    """Per-interval cubic coefficients of S(x) = slope * x on [lo, hi]."""
    h = (hi - lo) / n
    m = np.arange(n)
    return np.stack([slope * (lo + h * m), np.full(n, slope * h), np.zeros(n), np.zeros(n)], 1)


def test_dimer_by_hand(orc):
    """Atom 0 (type 0) and atom 1 (type 1) at distance r, alone in a large
    box, with rho^(ab)(r) = g_ab r, V^(ab)(r) = w r, F^(a)(rho) = s_a rho:
      rho_0 = g01 r, rho_1 = g10 r, E = s0 g01 r + s1 g10 r + w r,
      f_0 = -(s0 g01 + s1 g10 + w) (x_0 - x_1) / r."""
    g = np.array([[0.3, 0.7], [1.9, 1.1]])     # g[a, b]: at an a atom from a b atom
    s = np.array([-0.5, -2.0])
    w = 0.25
    rc = 5.0
    V = np.stack([linear_table(w, 0.0, rc)] * 4)
    R = np.stack([linear_table(g[a, b], 0.0, rc) for a in range(2) for b in range(2)])
    F = np.stack([linear_table(s[a], 0.0, 20.0) for a in range(2)])
    pot = W.Potential(kind=W.POT_SPLINE, rc=rc, tables=(V, R, F), lo=(0.0, 0.0, 0.0),
                      hi=(rc, rc, 20.0), n_types=2)
    d = np.array([1.2, -2.0, 1.5])
    r = np.linalg.norm(d)
    pos = np.array([[10.0, 10.0, 10.0], 10.0 + d])
    out = orc.alloy_eval(pos, 30.0, orc.Alloy(pot), np.array([0, 1]))
    assert np.allclose(out["rho"], [g[0, 1] * r, g[1, 0] * r], rtol=1e-14, atol=0)
    assert np.allclose(out["e_atom"], [s[0] * g[0, 1] * r + 0.5 * w * r,
                                       s[1] * g[1, 0] * r + 0.5 * w * r], rtol=1e-14, atol=0)
    k = s[0] * g[0, 1] + s[1] * g[1, 0] + w
    f0 = -k * (pos[0] - pos[1]) / r
    assert np.allclose(out["f"][0], f0, rtol=1e-13, atol=0)
    assert np.allclose(out["f"][1], -f0, rtol=1e-13, atol=0)
    # pair virial of eq. (6): W = -k r
    assert abs(out["W"] - (-k * r)) <= 1e-13 * abs(k * r)


def test_forces_are_minus_energy_gradient(orc):
    wl, L = small_alloy()
    pot = orc.Alloy(wl.pot)
    pos = orc.wrap(wl.pos, L)
    out = orc.alloy_eval(pos, L, pot, wl.types)
    assert np.abs(out["f"].sum(axis=0)).max() <= 1e-12 * np.abs(out["f"]).sum()
    rng = np.random.default_rng(3)
    h = 1e-5
    for i in rng.choice(wl.n_atoms, 6, replace=False):
        for k in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, k] += h
            p2[i, k] -= h
            fd = -(orc.alloy_eval(p1, L, pot, wl.types)["E"]
                   - orc.alloy_eval(p2, L, pot, wl.types)["E"]) / (2 * h)
            assert abs(fd - out["f"][i, k]) <= 1e-7 * np.abs(out["f"]).max(), (i, k)
    # both species present, and the two density functions differ
    assert 0 < wl.types.sum() < wl.n_atoms
    assert not np.array_equal(wl.pot.tables[1][1], wl.pot.tables[1][2])


def test_virial_is_minus_energy_derivative(orc):
    wl, L = small_alloy()
    pot = orc.Alloy(wl.pot)
    pos = orc.wrap(wl.pos * 0.98, L * 0.98)
    Ls = L * 0.98
    h = 1e-6
    E = lambda lam: orc.alloy_eval(pos * lam, Ls * lam, pot, wl.types)["E"]
    fd = -(E(1 + h) - E(1 - h)) / (2 * h)
    w = orc.alloy_eval(pos, Ls, pot, wl.types)["W"]
    assert abs(fd - w) <= 1e-8 * abs(w) + 50 * np.finfo(float).eps * abs(E(1.0)) / h


def test_list_equals_all_pairs(orc):
    wl, L = small_alloy(ncell=4)
    pot = orc.Alloy(wl.pot)
    pos = orc.wrap(wl.pos, L)
    cnt, ids = orc.neighbor_list(pos, L, orc.rlist(wl.pot.rc, wl.skin, L))
    a = orc.alloy_eval(pos, L, pot, wl.types, cnt, ids)
    b = orc.alloy_eval(pos, L, pot, wl.types)
    assert np.abs(a["f"] - b["f"]).max() <= 1e-13 * np.abs(b["f"]).max()
    assert abs(a["E"] - b["E"]) <= 1e-13 * abs(b["E"])


def test_vv_conserves_energy_and_momentum(orc):
    wl, L = small_alloy(ncell=4)
    pot = orc.Alloy(wl.pot)
    x, v, ep, ek, nreb = orc.alloy_vv(wl.pos, wl.vel, L, pot, wl.types, wl.type_mass, wl.dt,
                                      wl.skin, 400)
    e = ep + ek
    assert np.abs(e - e[0]).max() / wl.n_atoms < 1e-4
    m = wl.type_mass[wl.types][:, None]
    p0, p1 = (m * wl.vel).sum(axis=0), (m * v).sum(axis=0)
    assert np.abs(p1 - p0).max() <= 1e-10 * (m * np.abs(wl.vel)).sum()
    assert nreb >= 1


def test_friction_per_species(orc):
    """Atoms too far apart to interact, two species of different mass: each
    relaxes to its own v_e^2 = 3 k_B T_e / m_a as eq. (4) integrated by RK4."""
    te, tau, dt, nsteps = 500.0, 30.0, 1.0, 50
    mass_t = np.array([W.MASS_CU, W.MASS_AG])
    rng = np.random.default_rng(5)
    g = np.arange(2) * 14.0
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 3.0
    types = np.array([0, 1, 0, 1, 1, 0, 1, 0])
    vel = rng.normal(size=(8, 3)) * 0.02
    pot = orc.Alloy(W.alloy(ncell=2).pot)
    x, v, ep, ek, _ = orc.alloy_vv(pos, vel, 28.0, pot, types, mass_t, dt, 0.3, nsteps, te, tau)
    assert np.all(ep == 0.0)
    for i in range(8):
        m = mass_t[types[i]]
        u = vel[i].copy()
        h = 0.01
        acc = lambda q: -(1.0 - te / (m * (q @ q) / (3 * W.KB_EV * W.KAPPA))) * q / tau
        for _ in range(int(nsteps * dt / h)):
            k1 = acc(u)
            k2 = acc(u + 0.5 * h * k1)
            k3 = acc(u + 0.5 * h * k2)
            k4 = acc(u + h * k3)
            u = u + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        assert np.allclose(v[i], u, rtol=1e-9, atol=0), (i, v[i], u)


# ------------------------------------------------------------------ RCUT(a, b)

def test_pair_cutoffs_dimer_by_hand(orc):
    """Cutoffs per pair of types (Sections 3.2 and 3.3, RCUT(ity, jty)) with
    linear tables that do not vanish at the cutoffs: a dimer of types (a, b)
    just inside RCUT(a, b) has the hand-computed density, energy and force;
    just outside it, the two atoms do not interact at all."""
    g = np.array([[1.0, 0.7], [1.3, 0.9]])
    s = np.array([-0.8, -1.1])
    w = 0.25
    rmax = 5.0
    rcp = np.array([[5.0, 4.6], [4.6, 4.2]])
    V = np.stack([linear_table(w, 0.0, rmax)] * 4)
    R = np.stack([linear_table(g[a, b], 0.0, rmax) for a in range(2) for b in range(2)])
    F = np.stack([linear_table(s[a], 0.0, 20.0) for a in range(2)])
    pot = W.Potential(kind=W.POT_SPLINE, rc=rmax, tables=(V, R, F), lo=(0.0, 0.0, 0.0),
                      hi=(rmax, rmax, 20.0), n_types=2, rc_pair=rcp)
    u = np.array([0.6, -0.48, 0.64])           # unit vector
    for a in range(2):
        for b in range(2):
            rc = rcp[a, b]
            for r, inside in ((rc * (1 - 1e-12), True), (rc * (1 + 1e-12), False)):
                pos = np.array([[10.0, 10.0, 10.0], 10.0 + r * u])
                out = orc.alloy_eval(pos, 30.0, orc.Alloy(pot), np.array([a, b]))
                rr = np.linalg.norm(pos[1] - pos[0])
                if inside:
                    assert np.allclose(out["rho"], [g[a, b] * rr, g[b, a] * rr], rtol=1e-12)
                    e = [s[a] * g[a, b] * rr + 0.5 * w * rr, s[b] * g[b, a] * rr + 0.5 * w * rr]
                    assert np.allclose(out["e_atom"], e, rtol=1e-12)
                    k = s[a] * g[a, b] + s[b] * g[b, a] + w
                    assert np.allclose(out["f"][0], k * u, rtol=1e-12)
                else:
                    assert np.all(out["rho"] == 0.0) and np.all(out["f"] == 0.0)
                    assert np.all(out["e_atom"] == 0.0)


def brute_pair_list(pos, L, types, rcp, skin):
    """O(N^2) list with the list radius per pair of types, min(RCUT + skin,
    L/2 - 1e-9), on the squared separation rounded term by term."""
    n = pos.shape[0]
    rows = []
    for i in range(n):
        d = pos - pos[i]
        d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        rl = np.minimum(rcp[types[i], types] + skin, 0.5 * L - 1e-9)
        ok = r2 < rl * rl
        ok[i] = False
        rows.append(np.nonzero(ok)[0].tolist())
    return rows


def test_pair_list_radius_is_per_pair(orc):
    wl, L = small_alloy(ncell=4)
    pos = orc.wrap(wl.pos, L)
    rcp = wl.pot.rc_pair
    assert rcp is not None and rcp[1, 1] < rcp[0, 0]
    count, ids = orc.alloy_list(pos, L, orc.Alloy(wl.pot), wl.types, wl.skin)
    ref = brute_pair_list(pos, L, wl.types, rcp, wl.skin)
    for i in range(wl.n_atoms):
        assert ids[i, :count[i]].tolist() == ref[i], i
    # rows of two species-1 atoms end at 5.3 Angstrom instead of 5.6
    one = np.nonzero(wl.types == 1)[0]
    full = orc.neighbor_list(pos, L, orc.rlist(wl.pot.rc, wl.skin, L))
    assert (count[one] < full[0][one]).any()


def test_equal_pair_cutoffs_change_nothing(orc):
    wl, L = small_alloy(ncell=3)
    pos = orc.wrap(wl.pos, L)
    a = orc.alloy_eval(pos, L, orc.Alloy(wl.pot), wl.types)
    same = W.Potential(wl.pot.kind, wl.pot.rc, wl.pot.params, wl.pot.tables, wl.pot.lo,
                       wl.pot.hi, n_types=2, rc_pair=np.full((2, 2), wl.pot.rc))
    none = W.Potential(wl.pot.kind, wl.pot.rc, wl.pot.params, wl.pot.tables, wl.pot.lo,
                       wl.pot.hi, n_types=2)
    b = orc.alloy_eval(pos, L, orc.Alloy(same), wl.types)
    c = orc.alloy_eval(pos, L, orc.Alloy(none), wl.types)
    assert np.array_equal(b["f"], c["f"]) and np.array_equal(b["e_atom"], c["e_atom"])
    # the workload's own RCUT(1, 1) = 5.0 cuts only where its tables vanish, up
    # to the ripple an interpolating spline through samples of a form whose
    # second derivative jumps at c carries past c (a few parts in 1e9 here)
    assert np.abs(a["f"] - c["f"]).max() <= 1e-8 * np.abs(c["f"]).max()
