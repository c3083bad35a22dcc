"""Pins of the oracle's frozen atoms (atom states, Section 3.1).

Frozen atoms keep zero velocity and stay in place; they still exert forces.
Pins: nothing frozen is plain velocity Verlet bit for bit; everything frozen
leaves positions and energy unchanged; with a frozen slab the free atoms move
in the fixed field of the slab, so their kinetic energy plus the total
potential energy is conserved (a slab that exerted no force would break it).
"""
import numpy as np

from paper_1212_6332_amd import workloads as W


def slab(wl, frac=0.25):
    """Atoms in the bottom quarter of the box (by z) frozen."""
    L = wl.box_len[0, 0]
    return (np.mod(wl.pos[:, 2], L) < frac * L).astype(np.uint8)


def test_nothing_frozen_is_plain_vv(orc):
    wl = W.fs256()
    L = wl.box_len[0, 0]
    pot = orc.Pot(wl.pot)
    a = orc.vv(wl.pos, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30)
    b = orc.vv_frozen(wl.pos, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 30,
                      np.zeros(wl.n_atoms, dtype=np.uint8))
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    assert a[4] == b[4]


def test_everything_frozen_stays(orc):
    wl = W.fs256()
    L = wl.box_len[0, 0]
    x0 = orc.wrap(wl.pos, L)
    x, v, ep, ek, _ = orc.vv_frozen(x0, wl.vel, L, orc.Pot(wl.pot), wl.mass, wl.dt, wl.skin, 20,
                                    np.ones(wl.n_atoms, dtype=np.uint8))
    assert np.array_equal(x, x0) and np.all(v == 0.0)
    assert np.all(ep == ep[0]) and np.all(ek == 0.0)


def test_frozen_slab_conserves_energy_of_free_atoms(orc):
    wl = W.fs256(ncell=5)
    L = wl.box_len[0, 0]
    fr = slab(wl)
    assert 0 < fr.sum() < wl.n_atoms
    x0 = orc.wrap(wl.pos, L)
    x, v, ep, ek, nreb = orc.vv_frozen(x0, wl.vel, L, orc.Pot(wl.pot), wl.mass, wl.dt, wl.skin,
                                       300, fr)
    f = fr.astype(bool)
    assert np.array_equal(x[f], x0[f]) and np.all(v[f] == 0.0)
    assert np.abs(x[~f] - x0[~f]).max() > 1e-3
    e = ep + ek
    assert np.abs(e - e[0]).max() / wl.n_atoms < 1e-4
    # the free atoms' momentum is not conserved: the slab pushes on them
    m = wl.mass
    assert np.abs((m * v[~f]).sum(axis=0) - (m * wl.vel[~f]).sum(axis=0)).max() > 1e-6
