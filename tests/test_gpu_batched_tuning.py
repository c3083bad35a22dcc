"""Block shapes of the persistent multi-box stepper (form (2)) and several
species in it.

Workgroup size, packs of several small boxes per workgroup and the order in
which threads visit a pack's atoms leave each atom's arithmetic unchanged, so
every shape and the autotuner's pick give bitwise the trajectory of the
default shape (over more than one captured 100-step launch).  With several
species (per-type-pair tables, cutoffs RCUT(a, b) and masses, Sections
3.2-3.3) the stepper's own forces match the oracle at 1e-11 per box, before
and after a step in which every box rebuilds, and its trajectories match the
oracle's velocity Verlet per box.
"""
import numpy as np
import pytest

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11
RCP = np.array([[5.3, 5.1], [5.1, 4.9]])


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def boxes_of(wls):
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    w0 = wls[0]
    types = None if w0.types is None else np.concatenate([w.types for w in wls])
    return W.Workload(name="boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.concatenate([w.vel for w in wls]), mass=w0.mass, dt=w0.dt,
                      skin=w0.skin, pot=w0.pot, steps=0, types=types, type_mass=w0.type_mass)


def alloy_boxes(cutoffs):
    wls = [W.alloy(ncell=n, frac=f) for n, f in ((3, 0.3), (4, 0.5), (5, 0.2), (3, 0.7),
                                                  (6, 0.4), (4, 0.3), (3, 0.5))]
    wl = boxes_of(wls)
    if cutoffs:
        t = wl.pot
        wl.pot = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, t.hi, n_types=2,
                             rc_pair=RCP.copy())
    return wl


SHAPES = [(256, 0, 0), (512, 512, 0), (1024, 2048, 1), (256, 256, 1), (512, 1024, 1),
          (1024, 0, 1)]


def run(wl, nsteps, shape=None, tune=False, te=0.0, tau=0.0):
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_BATCHED) == 1
    if shape is not None:
        S.set_option(md.MD_OPT_BATCH_BLOCK, shape[0])
        S.set_option(md.MD_OPT_BATCH_PACK, shape[1])
        S.set_option(md.MD_OPT_BATCH_ORDER, shape[2])
    S.set_state(wl.pos, wl.vel)
    if tau > 0:
        S.set_thermostat(te, tau)
    picked = None
    if tune:
        S.autotune()
        picked = tuple(S.get_option(k) for k in (md.MD_OPT_BATCH_BLOCK, md.MD_OPT_BATCH_PACK,
                                                 md.MD_OPT_BATCH_ORDER))
    S.step(nsteps)
    p, v = (t.cpu().numpy() for t in S.get_state())
    st = S.status()
    S.close()
    return p, v, st, picked


@pytest.mark.parametrize("name", ["spline", "alloy"])
def test_block_shapes_change_nothing(name):
    wl = W.batch2048(n_boxes=96) if name == "spline" else alloy_boxes(True)
    nsteps = 130
    ref = run(wl, nsteps, SHAPES[0])
    assert ref[2][0] == 0 and ref[2][2] == nsteps
    for sh in SHAPES[1:]:
        p, v, st, _ = run(wl, nsteps, sh)
        assert st[0] == 0
        assert np.array_equal(p, ref[0]) and np.array_equal(v, ref[1]), sh


def test_shapes_with_frozen_atoms_and_friction():
    """Packs, visiting order and workgroup size with a frozen slab and the
    electron-gas friction of eq. (4): bitwise the default shape, frozen atoms
    in place."""
    wl = alloy_boxes(True)
    L = np.repeat(wl.box_len[:, 0], np.diff(wl.box_offset))
    frozen = (np.mod(wl.pos[:, 2], L) < 0.25 * L).astype(np.uint8)

    def go(shape):
        S = md.System.from_workload(wl)
        S.set_option(md.MD_OPT_BATCH_BLOCK, shape[0])
        S.set_option(md.MD_OPT_BATCH_PACK, shape[1])
        S.set_option(md.MD_OPT_BATCH_ORDER, shape[2])
        S.set_frozen(frozen)
        S.set_state(wl.pos, wl.vel)
        S.set_thermostat(900.0, 20.0)
        S.step(60)
        p, v = (t.cpu().numpy() for t in S.get_state())
        assert S.status()[0] == 0
        S.close()
        return p, v

    p0, v0 = go(SHAPES[0])
    f = frozen.astype(bool)
    assert not v0[f].any()
    for b, s, L in O.boxes(wl):       # frozen atoms stay where the first build wrapped them
        assert np.array_equal(p0[s][f[s]], O.wrap(wl.pos[s], L)[f[s]]), b
    for sh in SHAPES[1:4]:
        p, v = go(sh)
        assert np.array_equal(p, p0) and np.array_equal(v, v0), sh


def test_pack_option_checks():
    wl = W.batch2048(n_boxes=8)
    S = md.System.from_workload(wl)
    for key, bad in ((md.MD_OPT_BATCH_PACK, -1), (md.MD_OPT_BATCH_PACK, 65536),
                     (md.MD_OPT_BATCH_ORDER, 2)):
        with pytest.raises(md.MDError):
            S.set_option(key, bad)
    S.set_option(md.MD_OPT_BATCH_PACK, 100000 // 2)   # larger than every pack: all boxes in few packs
    S.set_state(wl.pos, wl.vel)
    S.step(3)
    p = S.get_state()[0].cpu().numpy()
    S.close()
    q = run(wl, 3, SHAPES[0])[0]
    assert np.array_equal(p, q)


def test_autotune_picks_a_shape_and_changes_nothing():
    wl = W.batch2048(n_boxes=64)
    p, v, st, picked = run(wl, 40, tune=True)
    assert picked[0] in (256, 512, 1024) and picked[2] in (0, 1)
    assert picked[1] in (0, picked[0], 2 * picked[0])
    q, u, _, _ = run(wl, 40)
    assert np.array_equal(p, q) and np.array_equal(v, u)


@pytest.mark.parametrize("cutoffs", [False, True])
def test_species_stepper_forces_match_oracle(cutoffs):
    """md_step(ctx, 0) brings the stepper's list and forces up to date and
    md_forces without energies returns those forces as computed."""
    wl = alloy_boxes(cutoffs)
    pot = O.Alloy(wl.pot)
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_BATCHED) == 1
    S.set_option(md.MD_OPT_BATCH_PACK, 512)
    vel = np.zeros_like(wl.vel)
    first = wl.box_offset[:-1]
    vel[first, 0] = 0.4            # past half the skin in one step: every box rebuilds
    S.set_state(wl.pos, vel)
    S.step(0)
    f0 = S.forces(energy=False).cpu().numpy()
    S.step(1)
    f1 = S.forces(energy=False).cpu().numpy()
    p1 = S.get_state()[0].cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    for pos, f in ((wl.pos, f0), (p1, f1)):
        for b, s, L in O.boxes(wl):
            p = O.wrap(pos[s], L)
            cnt, ids = O.alloy_list(p, L, pot, wl.types[s], wl.skin)
            r = O.alloy_eval(p, L, pot, wl.types[s], cnt, ids)
            assert rel(f[s], r["f"]) <= TOL, (b, rel(f[s], r["f"]))


@pytest.mark.parametrize("cutoffs,thermo", [(False, False), (True, False), (True, True)])
def test_species_stepper_trajectory_matches_oracle(cutoffs, thermo):
    wl = alloy_boxes(cutoffs)
    te, tau = (800.0, 30.0) if thermo else (0.0, 0.0)
    nsteps = 40
    p, v, st, _ = run(wl, nsteps, (512, 1024, 1), te=te, tau=tau)
    assert st[0] == 0 and st[2] == nsteps
    pot = O.Alloy(wl.pot)
    for b, s, L in O.boxes(wl):
        x, vo, *_ = O.alloy_vv(O.wrap(wl.pos[s], L), wl.vel[s], L, pot, wl.types[s],
                               wl.type_mass, wl.dt, wl.skin, nsteps, te, tau, energies=False)
        d = p[s] - x
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-10, b
        assert np.abs(v[s] - vo).max() <= 1e-9 * np.abs(vo).max(), b
    # the merged-box kernels give the same trajectory within the same bars
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_BATCHED, 0)
    S.set_state(wl.pos, wl.vel)
    if tau > 0:
        S.set_thermostat(te, tau)
    S.step(nsteps)
    q = S.get_state()[0].cpu().numpy()
    S.close()
    for b, s, L in O.boxes(wl):
        d = p[s] - q[s]
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-10, b


def test_many_small_boxes_in_large_packs():
    """3,000 boxes of 108 atoms: packs limited by the 64 boxes a pack holds
    and by LDS, bitwise the trajectory of one box per workgroup."""
    wl = W.batch2048(n_boxes=3000, nmin=3, nmax=3)
    assert (np.diff(wl.box_offset) == 108).all()
    a = run(wl, 30, (256, 0, 0))
    b = run(wl, 30, (1024, 65535, 1))
    assert a[2][0] == 0 and b[2][0] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
