"""Pins of the oracle's electron-gas thermostat (eq. 4).

Reading: the friction on atom i is -(m/tau)((T_i - T_e)/T_i) v_i with
T_i = m v_i^2 / (3 k_B), taken as an exact flow over each half step around the
force half kicks.  Pins, none of which uses the oracle's update formula:
  * tau -> infinity reproduces plain velocity Verlet bit for bit (also under
    the barostat);
  * atoms too far apart to interact follow eq. (4) as integrated here by a
    fine-step Runge-Kutta method (heating, cooling, T_e = 0 pure damping), and
    keep their directions; an atom at rest stays at rest;
  * an interacting SMTB Cu crystal, started cold or hot, settles at the
    electron temperature.
"""
import numpy as np

from paper_1212_6332_amd import workloads as W


def free_gas(rng, n_side, spacing, speeds):
    """Atoms on a simple cubic grid of the given spacing, random directions."""
    g = np.arange(n_side) * spacing
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 0.25 * spacing
    d = rng.normal(size=pos.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return pos, d * speeds[:, None], n_side * spacing


def rk4_eq4(v0, m, tau, te, t_end, h):
    """Integrate m dv/dt = -(m/tau)(1 - T_e/T_i) v for one atom, classic RK4."""
    def acc(v):
        ti = m * (v @ v) / (3 * W.KB_EV * W.KAPPA)   # (1/2) m v^2 / kappa = (3/2) k_B T_i
        return -(1.0 - te / ti) * v / tau
    v = np.array(v0, dtype=float)
    for _ in range(int(round(t_end / h))):
        k1 = acc(v)
        k2 = acc(v + 0.5 * h * k1)
        k3 = acc(v + 0.5 * h * k2)
        k4 = acc(v + h * k3)
        v = v + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return v


def test_infinite_coupling_time_is_plain_vv(orc):
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pot = orc.Pot(wl.pot)
    pos0 = orc.wrap(wl.pos, L)
    a = orc.vv(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30)
    for tau in (1e300, 0.0, -1.0):
        b = orc.vv_thermo(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30, 300.0, tau)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[4] == b[4]
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    c = orc.vv_baro(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 20, 0.0, 500.0, 1.0)
    d = orc.vv_baro(pos0, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 20, 0.0, 500.0, 1.0,
                    te=300.0, tau_t=1e300)
    assert np.array_equal(c[0], d[0]) and np.array_equal(c[1], d[1]) and c[2] == d[2]


def test_free_atoms_follow_eq4(orc):
    """No atom is within the cutoff of another (energy identically zero), so
    each velocity obeys eq. (4) alone."""
    rng = np.random.default_rng(4)
    mass, dt, tau, te = W.MASS_CU, 1.0, 40.0, 300.0
    ve = np.sqrt(3 * W.KB_EV * te * W.KAPPA / mass)
    # cold and hot atoms, one at exactly the electron temperature, one at rest
    speeds = ve * np.array([0.05, 0.3, 0.9, 1.0, 1.7, 3.0, 0.0, 2.2])
    pos, vel, L = free_gas(rng, 2, 14.0, speeds)
    pot = orc.Pot(W.smtb_cu())
    nsteps = 60
    x, v, ep, ek, _ = orc.vv_thermo(pos, vel, L, pot, mass, dt, 0.3, nsteps, te, tau)
    assert np.all(ep == 0.0)
    for i in range(len(speeds)):
        if speeds[i] == 0.0:
            assert np.all(v[i] == 0.0)
            continue
        ref = rk4_eq4(vel[i], mass, tau, te, nsteps * dt, 0.01)
        assert np.allclose(v[i], ref, rtol=1e-9, atol=0), (i, v[i], ref)
        assert abs(v[i] @ vel[i] / (np.linalg.norm(v[i]) * speeds[i]) - 1) < 1e-14
    # the atom at T_i = T_e feels no friction
    assert abs(np.linalg.norm(v[3]) - ve) <= 1e-14 * ve
    # electrons at 0 K: pure damping v(t) = v(0) exp(-t / tau)
    x, v0, ep, ek, _ = orc.vv_thermo(pos, vel, L, pot, mass, dt, 0.3, nsteps, 0.0, tau)
    assert np.allclose(v0, vel * np.exp(-nsteps * dt / tau), rtol=1e-13, atol=0)


def _temperature(ek, n):
    return 2.0 * ek / (3 * n * W.KB_EV)


def test_crystal_settles_at_electron_temperature(orc):
    """SMTB Cu (256 atoms, 4x4x4 FCC) started at 5 K and at 900 K relaxes to
    T_e = 300 K: the time-averaged kinetic temperature of the last 400 fs is
    within 5 % of T_e from either side."""
    te, tau = 300.0, 50.0
    for t0 in (5.0, 900.0):
        rng = np.random.default_rng(7)
        pos = W.lattice("fcc", 4, 3.615)
        vel = W.maxwell_velocities(rng, len(pos), W.MASS_CU, t0)
        L = 4 * 3.615
        _, _, ep, ek, _ = orc.vv_thermo(pos, vel, L, orc.Pot(W.smtb_cu()), W.MASS_CU, 1.0, 0.3,
                                        1200, te, tau)
        t = _temperature(ek, len(pos))
        assert abs(t[-400:].mean() - te) < 0.05 * te, (t0, t[-400:].mean())
