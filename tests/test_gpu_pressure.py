"""Pressure (eq. 6) and the Berendsen barostat (eq. 5) of the HIP path against
the oracle, through the C ABI.

Bars: per-box virial and pressure within 1e-11 relative (the virial with a
floor of 1 eV, since for boxes near zero pressure it is a small difference of
large pair sums); barostat trajectories of 40 steps within 1e-10 Angstrom in
positions and 1e-9 relative in velocities, box edges within 1e-13 relative.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu


def squeezed(wl, s):
    wl.pos = wl.pos * s
    wl.box_len = wl.box_len * s
    return wl


def oracle_pressure(wl, pot=None):
    pot = O.Pot(pot or wl.pot)
    out = []
    for b, sl, L in O.boxes(wl):
        pos = O.wrap(wl.pos[sl], L)
        w = O.virial(pos, L, pot, wl.skin)
        k = O.kinetic(wl.vel[sl], wl.mass)
        out.append(((2 * k + w) / (3 * L ** 3), w))
    return np.array(out)


def gpu_pressure(wl, tiled=None):
    S = md.System.from_workload(wl)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    p, w = S.pressure()
    flags, _, _ = S.status()
    S.close()
    assert flags == 0
    return np.stack([p.cpu().numpy(), w.cpu().numpy()], axis=1)


CASES = {
    "fs256": (lambda: W.fs256(), None),
    "smtb1372": (lambda: W.fcc4m(ncell=7), None),
    "smtb1372_per_atom": (lambda: W.fcc4m(ncell=7), 0),
    "smtb5324_compressed": (lambda: squeezed(W.fcc4m(ncell=11), 0.98), None),  # tiles, mode A
    "spline2662": (lambda: W.bcc128k(ncell=11), None),
    "merged_boxes": (lambda: W.batch2048(n_boxes=6), None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pressure_matches_oracle(name):
    make, tiled = CASES[name]
    wl = make()
    g, o = gpu_pressure(wl, tiled), oracle_pressure(wl)
    assert np.all(np.abs(g[:, 1] - o[:, 1]) <= 1e-11 * np.maximum(np.abs(o[:, 1]), 1.0))
    assert np.all(np.abs(g[:, 0] - o[:, 0]) <= 1e-11 * np.maximum(np.abs(o[:, 0]), 1e-6))


def run_barostat(wl, nsteps, p0, tau, beta, use_graph=1):
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    S.set_state(wl.pos, wl.vel)
    S.set_barostat(p0, tau, beta)
    S.step(nsteps)
    p, v = S.get_state()
    L = S.box()
    flags, builds, steps = S.status()
    pr, _ = S.pressure()
    S.close()
    return p.cpu().numpy(), v.cpu().numpy(), L, (flags, builds, steps), pr.cpu().numpy()


@pytest.mark.parametrize("name,nsteps", [("smtb256", 40), ("smtb5324", 20)])
def test_barostat_trajectory_matches_oracle(name, nsteps):
    """A Cu box compressed by 2 % relaxes under P0 = 0: positions, velocities,
    box edge and the final pressure against the oracle's Berendsen steps
    (device-decided rebuilds included)."""
    wl = squeezed(W.fcc4m(ncell=4 if name == "smtb256" else 11), 0.98)
    L0 = wl.box_len[0, 0]
    tau, beta = 100.0, 1.0
    x, v, L, (flags, builds, steps), pr = run_barostat(wl, nsteps, 0.0, tau, beta)
    assert flags == 0 and steps == nsteps
    xo, vo, Lo, pro, nreb = O.vv_baro(O.wrap(wl.pos, L0), wl.vel, L0, O.Pot(wl.pot), wl.mass,
                                      wl.dt, wl.skin, nsteps, 0.0, tau, beta)
    assert abs(L[0] - Lo) <= 1e-13 * Lo and L[0] > L0
    d = x - xo
    d -= Lo * np.round(d / Lo)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v - vo).max() <= 1e-9 * np.abs(vo).max()
    assert abs(pr[0] - pro[-1]) <= 1e-10 * abs(pro[-1])
    assert builds == 1 + nreb


def test_barostat_several_boxes_match_oracle():
    """Three boxes, compressed by different amounts, each scaled by its own
    pressure (eq. 5 per box) in the merged-box kernels: box edges, positions
    and velocities against the oracle box by box."""
    parts = [squeezed(W.fcc4m(ncell=n), s) for n, s in ((4, 0.98), (5, 0.99), (4, 1.01))]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in parts])]).astype(np.int64)
    wl = W.Workload(name="baro_boxes", box_offset=off,
                    box_len=np.concatenate([w.box_len for w in parts]),
                    pos=np.concatenate([w.pos for w in parts]),
                    vel=np.concatenate([w.vel for w in parts]), mass=parts[0].mass, dt=1.0,
                    skin=0.3, pot=parts[0].pot, steps=0)
    nsteps, tau, beta = 30, 100.0, 1.0
    x, v, L, (flags, builds, steps), pr = run_barostat(wl, nsteps, 0.0, tau, beta)
    assert flags == 0 and steps == nsteps
    for b, s, L0 in O.boxes(wl):
        xo, vo, Lo, pro, nreb = O.vv_baro(O.wrap(wl.pos[s], L0), wl.vel[s], L0, O.Pot(wl.pot),
                                          wl.mass, wl.dt, wl.skin, nsteps, 0.0, tau, beta)
        assert abs(L[b] - Lo) <= 1e-13 * Lo
        d = x[s] - xo
        d -= Lo * np.round(d / Lo)
        assert np.abs(d).max() < 1e-10
        assert np.abs(v[s] - vo).max() <= 1e-9 * np.abs(vo).max()
        assert abs(pr[b] - pro[-1]) <= 1e-10 * abs(pro[-1])
    # compressed boxes expand, the stretched one shrinks
    assert L[0] > wl.box_len[0, 0] and L[2] < wl.box_len[2, 0]


def test_boxes_after_barostat_step_with_their_new_edges():
    """Several boxes scaled by the barostat, which is then switched off: the
    persistent multi-box stepper steps with the new box edges (it agrees with
    the merged-box kernels, which read them on the device), and a caller's
    choice of the merged kernels survives the switch."""
    parts = [squeezed(W.fcc4m(ncell=n), s) for n, s in ((4, 0.98), (5, 0.985))]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in parts])]).astype(np.int64)
    wl = W.Workload(name="baro_boxes", box_offset=off,
                    box_len=np.concatenate([w.box_len for w in parts]),
                    pos=np.concatenate([w.pos for w in parts]),
                    vel=np.concatenate([w.vel for w in parts]), mass=parts[0].mass, dt=1.0,
                    skin=0.3, pot=parts[0].pot, steps=0)
    out = []
    for batched in (1, 0):
        S = md.System.from_workload(wl)
        S.set_option(md.MD_OPT_BATCHED, batched)
        S.set_state(wl.pos, wl.vel)
        S.set_barostat(0.0, 50.0, 1.0)
        S.step(30)
        S.set_barostat(0.0, 0.0, 1.0)
        assert S.get_option(md.MD_OPT_BATCHED) == batched
        L = S.box()
        S.step(30)
        p, v = S.get_state()
        assert S.status()[0] == 0
        out.append((p.cpu().numpy(), v.cpu().numpy(), L))
        S.close()
    assert np.array_equal(out[0][2], out[1][2]) and np.all(out[0][2] > wl.box_len[:, 0])
    d = out[0][0] - out[1][0]
    Lr = np.repeat(out[0][2], np.diff(wl.box_offset))[:, None]
    d -= Lr * np.round(d / Lr)
    assert np.abs(d).max() < 1e-10
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-9 * np.abs(out[1][1]).max()


def test_barostat_graph_equals_direct_launches():
    wl = squeezed(W.fcc4m(ncell=4), 0.98)
    a = run_barostat(wl, 31, 0.0, 100.0, 1.0, use_graph=1)
    b = run_barostat(wl, 31, 0.0, 100.0, 1.0, use_graph=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2]) and a[3] == b[3]


def test_barostat_off_and_box_range_guard():
    """Switching the barostat off keeps the scaled box; a target that would
    shrink a box below its cell grid leaves that box unscaled and raises
    MD_FLAG_BOX_RANGE (no kernel ever sees a box narrower than its cells)."""
    wl = squeezed(W.fcc4m(ncell=4), 0.98)
    L0 = wl.box_len[0, 0]
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.set_barostat(0.0, 100.0, 1.0)
    S.step(10)
    L1 = S.box()[0]
    assert L1 > L0
    S.set_barostat(0.0, 0.0, 1.0)
    S.step(10)
    assert S.box()[0] == L1
    assert S.status()[0] == 0
    # a huge target pressure asks for a shrink far past the cell grid
    S.set_barostat(1e3, 1.0, 1.0)
    S.step(3)
    flags, _, _ = S.status()
    assert flags & md.MD_FLAG_BOX_RANGE
    assert S.box()[0] == L1
    S.close()


def test_pressure_full_size():
    """The 4,000,000-atom box of the benchmark's pressure leg: virial and
    pressure against the oracle's list pass over every atom."""
    wl = W.fcc4m()
    g = gpu_pressure(wl)
    o = oracle_pressure(wl)
    assert abs(g[0, 1] - o[0, 1]) <= 1e-11 * abs(o[0, 1])
    assert abs(g[0, 0] - o[0, 0]) <= 1e-11 * abs(o[0, 0])
