"""Candidate tile shapes of the tiled passes: every shape gives bitwise the
same lists (as sets), forces and trajectory (each atom's neighbours are summed
in the same stencil and slot order whatever the tiling), and md_autotune's
pick among them and the per-atom passes keeps the trajectory of an untuned
context bitwise."""
import numpy as np
import pytest

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu


def run(wl, nsteps, shape=None, tune=False):
    S = md.System.from_workload(wl)
    n = S.get_option(md.MD_OPT_TILE_SHAPES)
    if shape is not None:
        S.set_option(md.MD_OPT_TILE_SHAPE, shape)
    S.set_state(wl.pos, wl.vel)
    if tune:
        S.autotune()
    f = S.forces(energy=False).cpu().numpy()
    S.step(nsteps)
    p, v = (t.cpu().numpy() for t in S.get_state())
    st = S.status()
    picked = (S.get_option(md.MD_OPT_TILED), S.get_option(md.MD_OPT_TILE_SHAPE))
    S.close()
    return f, p, v, st, n, picked


@pytest.mark.parametrize("name", ["smtb", "alloy"])
def test_every_tile_shape_gives_the_same_results(name):
    wl = W.fcc4m(ncell=56) if name == "smtb" else W.alloy(ncell=56)
    ref = run(wl, 25, 0)
    assert ref[3][0] == 0 and ref[4] >= 2, ref[4]
    for k in range(1, ref[4]):
        f, p, v, st, _, _ = run(wl, 25, k)
        assert st[0] == 0
        assert np.array_equal(f, ref[0]) and np.array_equal(p, ref[1]) and np.array_equal(v, ref[2]), k
    S = md.System.from_workload(wl)
    with pytest.raises(md.MDError):
        S.set_option(md.MD_OPT_TILE_SHAPE, ref[4])
    S.close()


def test_tile_shape_lists_match_oracle_sampled():
    """A non-default tile shape: sampled rows and forces against the oracle."""
    wl = W.alloy(ncell=56)
    L = float(wl.box_len[0, 0])
    S = md.System.from_workload(wl)
    k = S.get_option(md.MD_OPT_TILE_SHAPES) - 1
    S.set_option(md.MD_OPT_TILE_SHAPE, k)
    S.set_state(wl.pos, wl.vel)
    f, e, eb = S.forces()
    counts, ids = (t.cpu().numpy() for t in S.neighbors())
    f = f.cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    pot = O.Alloy(wl.pot)
    pos = O.wrap(wl.pos, L)
    rng = np.random.default_rng(5)
    for i in rng.integers(0, wl.n_atoms, 20):
        d = pos - pos[i]
        d -= L * np.round(d / L)
        near = np.nonzero((np.abs(d) < 11.0).all(axis=1))[0]
        sub = pos[near]
        # the oracle on the neighbourhood of atom i, in a box large enough that
        # its list and forces equal those in the whole box
        loc = int(np.nonzero(near == i)[0][0])
        cnt, oid = O.alloy_list(sub, L, pot, wl.types[near], wl.skin)
        assert counts[i] == cnt[loc]
        assert sorted(ids[i, :counts[i]].tolist()) == sorted(near[oid[loc, :cnt[loc]]].tolist())


def test_autotune_with_tile_shapes_keeps_the_trajectory():
    wl = W.alloy(ncell=56)
    a = run(wl, 20, tune=True)
    b = run(wl, 20)
    assert a[3][0] == 0
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
