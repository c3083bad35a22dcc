"""Edge cases of the HIP path against the oracle, through the C ABI:
isolated atoms (empty rows), coordinates several box lengths outside the
box, list overflow and recovery in a tiled context, and a box of the
smallest admissible size (two atoms, edge just above twice the cutoff)
next to an ordinary one."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_isolated_atoms_have_empty_rows_and_fly_free():
    """A simple cubic gas of spacing 7 A (beyond the list radius 6.15 A of
    the SMTB Cu potential): every row is empty, rho = F = f = E = 0, and 20
    steps are free flight (the oracle's trajectory)."""
    g = np.arange(8) * 7.0
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 1.0
    n, L = pos.shape[0], 56.0
    vel = np.random.default_rng(2).normal(0.0, 0.004, size=(n, 3))
    wl = W.Workload(name="gas", box_offset=np.array([0, n], dtype=np.int64),
                    box_len=np.full((1, 3), L), pos=pos, vel=vel, mass=W.MASS_CU, dt=1.0,
                    skin=0.3, pot=W.smtb_cu(), steps=0)
    S = md.System.from_workload(wl)
    S.set_state(pos, vel)
    counts, _ = S.neighbors()
    rho = S.density()
    f, e, eb = S.forces()
    assert int(counts.max()) == 0
    assert float(rho.abs().max()) == 0.0 and float(f.abs().max()) == 0.0
    assert float(e.abs().max()) == 0.0 and float(eb[0]) == 0.0
    S.step(20)
    p, v = S.get_state()
    assert S.status()[0] == 0
    S.close()
    x, vo, *_ = O.vv(pos, vel, L, O.Pot(wl.pot), wl.mass, wl.dt, wl.skin, 20)
    d = p.cpu().numpy() - x
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-12
    assert np.array_equal(v.cpu().numpy(), vo)


def test_far_outside_coordinates_are_wrapped():
    """Atoms moved by whole multiples of the box edge (up to +-3 L) give the
    forces of the wrapped configuration."""
    wl = W.fcc4m(ncell=7)
    L = wl.box_len[0, 0]
    k = np.random.default_rng(4).integers(-3, 4, size=wl.pos.shape)
    shifted = wl.pos + k * L
    S = md.System.from_workload(wl)
    S.set_state(shifted, wl.vel)
    f, e, eb = S.forces()
    assert S.status()[0] == 0
    p, _ = S.get_state()
    S.close()
    ref = O.forces(O.wrap(wl.pos, L), L, O.Pot(wl.pot))
    assert rel(f.cpu().numpy(), ref["f"]) <= TOL
    assert abs(float(eb[0]) - ref["E"]) <= TOL * abs(ref["E"])
    p = p.cpu().numpy()
    assert p.min() >= 0.0 and p.max() < L


def test_overflow_and_recovery_in_tiles():
    """A capacity below the row lengths of a tiled box (halo mode A) raises
    MD_FLAG_NLIST_OVERFLOW; after md_set_max_neighbors the forces match the
    oracle."""
    wl = W.fcc4m(ncell=11)
    L = wl.box_len[0, 0]
    S = md.System.from_workload(wl, max_neighbors=40)
    assert S.get_option(md.MD_OPT_TILED) == 1
    S.set_state(wl.pos, wl.vel)
    S.build_neighbors()
    assert S.status()[0] & md.MD_FLAG_NLIST_OVERFLOW
    S.set_max_neighbors(128)
    S.set_state(wl.pos, wl.vel)
    f, e, eb = S.forces()
    assert S.status()[0] == 0
    S.close()
    ref = O.forces(O.wrap(wl.pos, L), L, O.Pot(wl.pot))
    assert rel(f.cpu().numpy(), ref["f"]) <= TOL


def test_smallest_box_next_to_ordinary_box():
    """Box 0: two atoms 3 A apart in a box of edge 2 rc + 0.01 (list radius
    clamped to just under half the edge); box 1: an ordinary FCC box.  Both
    against the oracle; the pair of box 0 feels no image of itself."""
    rc = 5.85
    L0 = 2 * rc + 0.01
    a = W.fcc4m(ncell=4)
    p0 = np.array([[1.0, 2.0, 3.0], [3.4, 3.1, 4.4]])
    v0 = np.array([[0.001, -0.002, 0.0005], [-0.001, 0.002, -0.0005]])
    wl = W.Workload(name="tiny+fcc", box_offset=np.array([0, 2, 2 + a.n_atoms], dtype=np.int64),
                    box_len=np.array([[L0] * 3, a.box_len[0]]),
                    pos=np.concatenate([p0, a.pos]), vel=np.concatenate([v0, a.vel]),
                    mass=a.mass, dt=1.0, skin=0.3, pot=a.pot, steps=0)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    f, e, eb = S.forces()
    counts, _ = S.neighbors()
    assert S.status()[0] == 0
    S.step(15)
    p, v = S.get_state()
    assert S.status()[0] == 0
    S.close()
    f, p, v = f.cpu().numpy(), p.cpu().numpy(), v.cpu().numpy()
    assert counts[0] == 1 and counts[1] == 1
    pot = O.Pot(wl.pot)
    for b, s, L in O.boxes(wl):
        ref = O.forces(O.wrap(wl.pos[s], L), L, pot, skin=wl.skin)
        assert rel(f[s], ref["f"]) <= TOL
        assert abs(float(eb[b]) - ref["E"]) <= TOL * abs(ref["E"])
        x, vo, *_ = O.vv(O.wrap(wl.pos[s], L), wl.vel[s], L, pot, wl.mass, wl.dt, wl.skin, 15)
        d = p[s] - x
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-10
        assert np.abs(v[s] - vo).max() <= 1e-9 * np.abs(vo).max()
