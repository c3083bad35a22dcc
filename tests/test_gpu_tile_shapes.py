"""Candidate tile shapes of the tiled passes.  Every shape gives the same
lists; each atom's neighbours are visited in the same stencil and slot order
whatever the tiling, but the atoms of a tile beyond one per thread of its
1024-thread workgroup have their rows summed by several lanes (tiles of 1025
to 1088 atoms; with spline tables up to 1536), so shapes agree in rounding
only.  Such tiles are checked against the oracle, and md_autotune's pick
among the shapes and the per-atom passes keeps the trajectory of an untuned
context with the same settings bitwise.  The SMTB box of 500,000 atoms has
about a hundred tiles of 1025 to 1088 atoms in the planner's 4 x 4 x 3 cells;
the 702,464-atom alloy about 300, and as many more with up to 1,187 atoms, in
its 6 x 4 x 3."""
import numpy as np
import pytest

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def tile_sizes(wl, dims):
    """Atoms per tile of a one-box workload for tiles of dims = (tx, ty, tz)
    cells, on the host (cells at least the list radius wide)."""
    L = float(wl.box_len[0, 0])
    nc = int(np.floor(L / (wl.pot.rc + wl.skin)))
    c = np.minimum((O.wrap(wl.pos, L) * (nc / L)).astype(np.int64), nc - 1)
    nt = [-(-nc // d) for d in dims]
    t = c // np.asarray(dims)
    return np.bincount((t[:, 2] * nt[1] + t[:, 1]) * nt[0] + t[:, 0])


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
def test_tile_shapes_agree(name):
    """Forces of every shape within 1e-13 of the default's, and 25-step
    trajectories within 1e-11 Angstrom; each run is bitwise reproducible."""
    wl = W.fcc4m(ncell=50) if name == "smtb" else W.alloy(ncell=56)
    L = float(wl.box_len[0, 0])
    ref = run(wl, 25, 0)
    assert ref[3][0] == 0 and ref[4] >= 2, ref[4]
    for k in range(1, ref[4]):
        f, p, v, st, _, _ = run(wl, 25, k)
        assert st[0] == 0
        assert rel(f, ref[0]) <= 1e-13, k
        d = p - ref[1]
        assert np.abs(d - L * np.round(d / L)).max() <= 1e-11, k
        assert rel(v, ref[2]) <= 1e-10, k
        again = run(wl, 25, k)
        assert np.array_equal(f, again[0]) and np.array_equal(p, again[1]), k
    S = md.System.from_workload(wl)
    with pytest.raises(md.MDError):
        S.set_option(md.MD_OPT_TILE_SHAPE, ref[4])
    S.close()


@pytest.mark.parametrize("name", ["smtb", "alloy"])
def test_tiles_with_surplus_atoms_match_oracle(name):
    """Every tile shape, including those whose tiles hold a few more atoms
    than the workgroup has threads: densities, forces and energies against
    the oracle at 1e-11."""
    wl = W.fcc4m(ncell=50) if name == "smtb" else W.alloy(ncell=56)
    L = float(wl.box_len[0, 0])
    p = O.wrap(wl.pos, L)
    most = 1088 if name == "smtb" else 1536   # tiles whose surplus shares rows
    if name == "smtb":
        cnt, ids = O.neighbor_list(p, L, O.rlist(wl.pot.rc, wl.skin, L))
        ref = O.forces(p, L, O.Pot(wl.pot), cnt, ids)
    else:
        cnt, ids = O.alloy_list(p, L, O.Alloy(wl.pot), wl.types, wl.skin, maxn=96)
        ref = O.alloy_eval(p, L, O.Alloy(wl.pot), wl.types, cnt, ids)
    S = md.System.from_workload(wl)
    n = S.get_option(md.MD_OPT_TILE_SHAPES)
    surplus = 0
    for k in range(n):
        S.set_option(md.MD_OPT_TILE_SHAPE, k)
        dims = S.get_option(md.MD_OPT_TILE_DIMS)
        sizes = tile_sizes(wl, (dims & 255, (dims >> 8) & 255, dims >> 16))
        surplus += int(((sizes > 1024) & (sizes <= most)).sum())
        S.set_state(wl.pos, wl.vel)
        f, e, eb = S.forces()
        rho = S.density()
        assert S.status()[0] == 0
        assert rel(f.cpu().numpy(), ref["f"]) <= 1e-11, k
        assert rel(rho.cpu().numpy(), ref["rho"]) <= 1e-11, k
        assert rel(e.cpu().numpy(), ref["e_atom"]) <= 1e-11, k
        assert abs(float(eb[0]) - ref["E"]) <= 1e-11 * abs(ref["E"]), k
    S.close()
    assert surplus > 0   # some shape has tiles with surplus atoms


def test_tile_dims_option():
    """MD_OPT_TILE_DIMS reads each candidate's cells per tile (the planner's
    first); a B-spline context, which runs the per-atom passes only, reads 0."""
    wl = W.fcc4m(ncell=50)
    S = md.System.from_workload(wl)
    seen = set()
    for k in range(S.get_option(md.MD_OPT_TILE_SHAPES)):
        S.set_option(md.MD_OPT_TILE_SHAPE, k)
        d = S.get_option(md.MD_OPT_TILE_DIMS)
        dims = (d & 255, (d >> 8) & 255, d >> 16)
        assert all(1 <= v <= 6 for v in dims), dims
        seen.add(dims)
    assert len(seen) == S.get_option(md.MD_OPT_TILE_SHAPES)
    with pytest.raises(md.MDError):
        S.set_option(md.MD_OPT_TILE_DIMS, 0)        # read only
    S.close()
    B = md.System.from_workload(W.adjoint64())
    assert B.get_option(md.MD_OPT_TILED) == 0 and B.get_option(md.MD_OPT_TILE_DIMS) == 0
    B.close()


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
    """The tuned context's trajectory is bitwise that of an untuned context
    set to the pick (tiled or per-atom passes, tile shape)."""
    wl = W.alloy(ncell=56)
    a = run(wl, 20, tune=True)
    tiled, shape = a[5]
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_TILE_SHAPE, shape)
    S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    S.forces(energy=False)
    S.step(20)
    p, v = (t.cpu().numpy() for t in S.get_state())
    S.close()
    assert a[3][0] == 0
    assert np.array_equal(a[1], p) and np.array_equal(a[2], v)
