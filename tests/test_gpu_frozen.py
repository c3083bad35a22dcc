"""Frozen atoms (atom states, Section 3.1) on the HIP path against the
oracle, through the C ABI.

Bars as for velocity Verlet: 1e-10 Angstrom in positions and 1e-9 relative
in velocities, same device-decided rebuilds; frozen atoms bitwise in place
with exactly zero velocity.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu


def slab(wl, frac=0.25):
    """Atoms in the bottom quarter of each box (by z) frozen."""
    L = np.repeat(wl.box_len[:, 0], np.diff(wl.box_offset))
    return (np.mod(wl.pos[:, 2], L) < frac * L).astype(np.uint8)


def boxes(make, ncells):
    wls = [make(n) for n in ncells]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    return W.Workload(name="boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.concatenate([w.vel for w in wls]), mass=wls[0].mass, dt=1.0,
                      skin=0.3, pot=wls[0].pot, steps=0)


CASES = {
    "fs500": (lambda: W.fs256(ncell=5), {}),
    "smtb5324_tiled": (lambda: W.fcc4m(ncell=11), {}),       # tiles, mode A, fused graph
    "smtb5324_per_atom": (lambda: W.fcc4m(ncell=11), {"tiled": 0}),
    "fs_boxes_batched": (lambda: boxes(lambda n: W.fs256(ncell=n), (3, 4, 5, 4)), {}),
    "fs_boxes_merged": (lambda: boxes(lambda n: W.fs256(ncell=n), (3, 4, 5, 4)), {"batched": 0}),
}


def run(wl, nsteps, frozen, tiled=None, batched=None, use_graph=1):
    S = md.System.from_workload(wl)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    if batched is not None:
        S.set_option(md.MD_OPT_BATCHED, batched)
    S.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    S.set_frozen(frozen)
    S.set_state(wl.pos, wl.vel)
    S.step(nsteps)
    p, v = S.get_state()
    st = S.status()
    S.close()
    return p.cpu().numpy(), v.cpu().numpy(), st


@pytest.mark.parametrize("name", list(CASES))
def test_frozen_trajectory_matches_oracle(name):
    make, kw = CASES[name]
    wl = make()
    fr = slab(wl)
    nsteps = 40
    p, v, (flags, builds, steps) = run(wl, nsteps, fr, **kw)
    assert flags == 0 and steps == nsteps
    f = fr.astype(bool)
    assert np.all(v[f] == 0.0)
    for b, s, L in O.boxes(wl):
        x0 = O.wrap(wl.pos[s], L)
        x, vo, _, _, nreb = O.vv_frozen(x0, wl.vel[s], L, O.Pot(wl.pot), wl.mass, wl.dt,
                                        wl.skin, nsteps, fr[s], energies=False)
        d = p[s] - x
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-10
        assert np.abs(v[s] - vo).max() <= 1e-9 * np.abs(vo).max()
        fb = f[s]
        assert np.array_equal(p[s][fb], x0[fb])     # frozen atoms did not move at all
        if wl.n_boxes == 1:
            assert builds == 1 + nreb


def test_frozen_graph_equals_direct_launches():
    wl = W.fcc4m(ncell=11)
    fr = slab(wl)
    a = run(wl, 37, fr, use_graph=1)
    b = run(wl, 37, fr, use_graph=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_freeze_midway_and_release():
    """Freezing after the state is set stops those atoms at once; releasing
    them lets them move again; the barostat refuses frozen atoms, and
    freezing refuses a running barostat."""
    wl = W.fcc4m(ncell=7)
    fr = slab(wl)
    f = fr.astype(bool)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(5)
    S.set_frozen(fr)
    p0, v0 = S.get_state()
    assert float(v0.cpu()[torch.from_numpy(f)].abs().max()) == 0.0
    S.step(12)
    p1, v1 = S.get_state()
    assert np.array_equal(p1.cpu().numpy()[f], p0.cpu().numpy()[f])
    with pytest.raises(md.MDError):
        S.set_barostat(0.0, 100.0, 1.0)
    S.set_frozen(None)
    S.step(12)
    p2, _ = S.get_state()
    assert np.abs(p2.cpu().numpy()[f] - p1.cpu().numpy()[f]).max() > 1e-4
    S.set_barostat(0.0, 100.0, 1.0)
    with pytest.raises(md.MDError):
        S.set_frozen(fr)
    assert S.status()[0] == 0
    S.close()
