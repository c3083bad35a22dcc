"""Device conditions through the C ABI: list and tile overflow are handled by
the library (capacity raised, list built again) before any pass reads a
truncated list, inside md_step too; table-range and non-finite conditions
are returned by md_step; md_bind keeps caller buffers as the state of
record."""
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


def squeeze(ncell=10, centre=None):
    """SMTB box whose atoms within 7 Angstrom of the centre move inward at
    0.012 fs^-1 times their distance: within ten steps the longest row grows
    from 82 to about 134 (far beyond a capacity fitted to the start)."""
    wl = W.fcc4m(ncell=ncell)
    L = float(wl.box_len[0, 0])
    wl.pos = O.wrap(wl.pos, L)
    c = np.full(3, L / 2) if centre is None else centre
    d = wl.pos - c
    sel = np.linalg.norm(d, axis=1) < 7.0
    wl.vel = wl.vel.copy()
    wl.vel[sel] = -0.012 * d[sel]
    return wl


def run(wl, nsteps, tiled=None, **kw):
    S = md.System.from_workload(wl, **kw)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    S.step(nsteps)
    p, v = (t.cpu().numpy() for t in S.get_state())
    mn = S.max_neighbors
    flags, builds, steps = S.status()
    S.close()
    return p, v, mn, flags, steps


def test_host_build_raises_the_capacity():
    """A capacity of 8: the first pass after md_set_state builds, finds the
    rows too long, raises the capacity and builds again; the forces are the
    oracle's."""
    wl = W.fcc4m(ncell=11)
    L = float(wl.box_len[0, 0])
    ref = O.forces(O.wrap(wl.pos, L), L, O.Pot(wl.pot))
    for tiled in (1, 0):
        S = md.System.from_workload(wl, max_neighbors=8)
        S.set_option(md.MD_OPT_TILED, tiled)
        S.set_state(wl.pos, wl.vel)
        f, e, eb = S.forces()
        assert S.max_neighbors >= 80
        assert S.status()[0] == md.MD_FLAG_NLIST_OVERFLOW
        S.close()
        assert rel(f.cpu().numpy(), ref["f"]) <= TOL
        assert abs(float(eb[0]) - ref["E"]) <= TOL * abs(ref["E"])


@pytest.mark.parametrize("tiled", [1, 0])
def test_overflow_inside_md_step_resumes(tiled):
    """The capacity fits the start; a list rebuilt inside the steps outgrows
    it.  md_step halts there, raises the capacity, completes the halted step
    and takes the rest: the trajectory is bitwise that of a context with
    enough capacity from the start."""
    wl = squeeze(ncell=14)                  # 8 cells per axis: tiles (halo mode A) fit
    nsteps = 20
    p_ref, v_ref, mn_ref, fl_ref, st_ref = run(wl, nsteps, tiled, max_neighbors=200)
    assert fl_ref == 0 and st_ref == nsteps
    S = md.System.from_workload(wl, max_neighbors=88)
    S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    S.build_neighbors()                     # the start fits the capacity
    assert S.status()[0] == 0 and S.max_neighbors == 88
    S.step(nsteps)
    p, v = (t.cpu().numpy() for t in S.get_state())
    assert S.max_neighbors > 120
    flags, builds, steps = S.status()
    S.close()
    assert flags == md.MD_FLAG_NLIST_OVERFLOW and steps == nsteps
    assert np.array_equal(p, p_ref) and np.array_equal(v, v_ref)


def test_overflow_with_the_barostat():
    wl = squeeze()
    nsteps = 16

    def go(mn):
        S = md.System.from_workload(wl, max_neighbors=mn)
        S.set_barostat(0.0, 500.0, 1.0)
        S.set_state(wl.pos, wl.vel)
        S.step(nsteps)
        p, v = (t.cpu().numpy() for t in S.get_state())
        out = (p, v, S.box(), S.max_neighbors, S.status())
        S.close()
        return out

    a, b = go(88), go(200)
    assert a[3] > 120 and a[4][0] == md.MD_FLAG_NLIST_OVERFLOW and a[4][2] == nsteps
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_batched_overflow_takes_the_call_again():
    """Several boxes in the persistent stepper, one of them squeezed: the
    call is taken again from its start state with a larger capacity, and
    ends bitwise where a context with enough capacity ends."""
    boxes = [squeeze(ncell=6)] + [W.fcc4m(ncell=n) for n in (5, 6, 7)]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in boxes])]).astype(np.int64)
    wl = W.Workload(name="b", box_offset=off, box_len=np.concatenate([w.box_len for w in boxes]),
                    pos=np.concatenate([w.pos for w in boxes]),
                    vel=np.concatenate([w.vel for w in boxes]), mass=boxes[0].mass, dt=1.0,
                    skin=0.3, pot=boxes[0].pot, steps=0)
    nsteps = 20
    a = run(wl, nsteps, max_neighbors=96)
    b = run(wl, nsteps, max_neighbors=200)
    assert a[2] > 96 and a[3] & md.MD_FLAG_NLIST_OVERFLOW and a[4] == nsteps
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def cube():
    """3,400 atoms moved into a 2x2x2-cell cube of a tiled box (8 cells per
    axis): the halo of every tile around it exceeds the LDS of a workgroup,
    and rows in the cube hold about 1,700 neighbours."""
    wl = W.fcc4m(ncell=14)
    L = float(wl.box_len[0, 0])
    pos = O.wrap(wl.pos, L)
    w = L / 8
    rng = np.random.default_rng(21)
    far = np.nonzero(pos[:, 0] > 5 * w)[0][:3400]
    assert far.size == 3400
    pos[far] = 2 * w + rng.uniform(0.0, 2 * w, size=(far.size, 3))
    wl.pos = pos
    count, ids = O.neighbor_list(pos, L, O.rlist(wl.pot.rc, wl.skin, L), maxn=4096)
    return wl, O.forces(pos, L, O.Pot(wl.pot), count, ids)


def test_tile_overflow_moves_to_per_atom_passes():
    """The cube: the context moves to the per-atom passes and raises the row
    capacity, and the forces are the oracle's."""
    wl, ref = cube()
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_TILED) == 1
    S.set_state(wl.pos)
    f, e, eb = S.forces()
    assert S.get_option(md.MD_OPT_TILED) == 0
    assert S.max_neighbors > 1500
    S.close()
    assert rel(f.cpu().numpy(), ref["f"]) <= TOL
    assert abs(float(eb[0]) - ref["E"]) <= TOL * abs(ref["E"])


def test_autotune_passes_over_tile_shapes_that_overflow():
    """The cube timed by md_autotune before any pass: the build of every
    candidate tile shape overflows and is passed over, the per-atom passes
    are kept, no overflow condition is left behind, and the forces are the
    oracle's."""
    wl, ref = cube()
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_TILE_SHAPES) >= 1
    S.set_state(wl.pos)
    S.autotune()
    assert S.get_option(md.MD_OPT_TILED) == 0
    assert S.status()[0] & md.MD_FLAG_TILE_OVERFLOW == 0
    f, e, eb = S.forces()
    assert S.status()[0] & md.MD_FLAG_TILE_OVERFLOW == 0
    assert S.max_neighbors > 1500
    S.close()
    assert rel(f.cpu().numpy(), ref["f"]) <= TOL
    assert abs(float(eb[0]) - ref["E"]) <= TOL * abs(ref["E"])


def test_step_returns_table_range_once():
    ws = W.bcc128k(ncell=6)
    t = ws.pot
    small = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, (t.hi[0], t.hi[1], 50.0))
    S = md.System.from_workload(ws, small)
    S.set_state(ws.pos, ws.vel)
    with pytest.raises(md.MDError) as e:
        S.step(3)
    assert e.value.code == md.MD_ERR_TABLE_RANGE
    assert S.status()[0] & md.MD_FLAG_TABLE_RANGE == 0   # reported once
    S.close()


def test_bind_writes_the_state_back():
    wl = W.fcc4m(ncell=8)
    pos = torch.tensor(wl.pos, device="cuda")
    vel = torch.tensor(wl.vel, device="cuda")
    S = md.System.from_workload(wl)
    S.bind(pos, vel)
    S.step(12)
    torch.cuda.synchronize()
    T = md.System.from_workload(wl)
    T.set_state(wl.pos, wl.vel)
    T.step(12)
    p, v = T.get_state()
    assert torch.equal(pos, p) and torch.equal(vel, v)
    # the caller changes the bound buffers, binds again, steps on
    pos += 0.01
    start = (pos.clone(), vel.clone())
    S.bind(pos, vel)
    S.step(5)
    T.set_state(*start)
    T.step(5)
    p, v = T.get_state()
    assert torch.equal(pos, p) and torch.equal(vel, v)
    S.bind(None)
    S.step(2)                 # unbound: the buffers keep the last written state
    assert torch.equal(pos, p)
    S.close()
    T.close()
