"""Electron-gas thermostat (eq. 4) of the HIP path against the oracle, through
the C ABI.

Bars as for plain velocity Verlet: trajectories within 1e-10 Angstrom in
positions and 1e-9 relative in velocities, with the same device-decided
rebuilds; captured and direct launches bitwise equal.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TE, TAU = 600.0, 25.0   # strong coupling, so the friction changes every trajectory


def run(wl, nsteps, te=TE, tau=TAU, tiled=None, batched=None, use_graph=1, graph_steps=None):
    S = md.System.from_workload(wl)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    if batched is not None:
        S.set_option(md.MD_OPT_BATCHED, batched)
    S.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    if graph_steps is not None:
        S.set_option(md.MD_OPT_GRAPH_STEPS, graph_steps)
    S.set_state(wl.pos, wl.vel)
    S.set_thermostat(te, tau)
    S.step(nsteps)
    p, v = S.get_state()
    st = S.status()
    S.close()
    return p.cpu().numpy(), v.cpu().numpy(), st


def oracle_run(wl, nsteps, te=TE, tau=TAU):
    pot = O.Pot(wl.pot)
    P, V, nreb = np.zeros_like(wl.pos), np.zeros_like(wl.vel), []
    for b, s, L in O.boxes(wl):
        x, v, _, _, n = O.vv_thermo(O.wrap(wl.pos[s], L), wl.vel[s], L, pot, wl.mass, wl.dt,
                                    wl.skin, nsteps, te, tau, maxn=160, energies=False)
        P[s], V[s] = x, v
        nreb.append(n)
    return P, V, nreb


def check(wl, g, o, nsteps):
    p, v, (flags, builds, steps) = g
    P, V, nreb = o
    assert flags == 0 and steps == nsteps
    d = p - P
    L = np.repeat(wl.box_len[:, 0], np.diff(wl.box_offset))[:, None]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10, np.abs(d).max()
    assert np.abs(v - V).max() <= 1e-9 * np.abs(V).max()
    if wl.n_boxes == 1:
        assert builds == 1 + nreb[0]


CASES = {
    "fs256": (lambda: W.fs256(), {}),
    "smtb256": (lambda: W.fcc4m(ncell=4), {}),
    "smtb5324_tiled": (lambda: W.fcc4m(ncell=11), {}),          # tiles, mode A, fused passes
    "smtb5324_per_atom": (lambda: W.fcc4m(ncell=11), {"tiled": 0}),
    "spline2662": (lambda: W.bcc128k(ncell=11), {}),
    "batched6": (lambda: W.batch2048(n_boxes=6), {}),            # persistent stepper
    "merged6": (lambda: W.batch2048(n_boxes=6), {"batched": 0}),  # merged-box kernels
}


@pytest.mark.parametrize("name", list(CASES))
def test_thermostat_trajectory_matches_oracle(name):
    make, kw = CASES[name]
    wl = make()
    nsteps = 40
    check(wl, run(wl, nsteps, **kw), oracle_run(wl, nsteps), nsteps)


@pytest.mark.parametrize("graph_steps", [9, 8])
def test_thermostat_graph_equals_direct_launches(graph_steps):
    wl = W.fcc4m(ncell=11)
    a = run(wl, 37, use_graph=1, graph_steps=graph_steps)
    b = run(wl, 37, use_graph=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert a[2][1] >= 2


def test_thermostat_off_is_plain_vv_bitwise():
    """Switching the thermostat on and off again, or an infinite coupling time
    (friction factor exactly 1), leaves the plain velocity-Verlet trajectory."""
    wl = W.fcc4m(ncell=11)
    ref = run(wl, 20, te=0.0, tau=0.0)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.set_thermostat(300.0, 50.0)
    S.set_thermostat(300.0, 0.0)
    S.step(20)
    p, v = S.get_state()
    assert np.array_equal(p.cpu().numpy(), ref[0]) and np.array_equal(v.cpu().numpy(), ref[1])
    S.close()
    inf = run(wl, 20, te=300.0, tau=1e300)
    assert np.array_equal(inf[0], ref[0]) and np.array_equal(inf[1], ref[1])


def test_thermostat_arguments():
    S = md.System.from_workload(W.fs256())
    for te, tau in ((300.0, float("nan")), (300.0, float("inf")), (-1.0, 10.0),
                    (float("nan"), 10.0), (float("inf"), 10.0)):
        with pytest.raises(md.MDError):
            S.set_thermostat(te, tau)
    S.set_thermostat(-1.0, 0.0)   # off: T_e is not used
    S.close()


def test_thermostat_with_barostat_matches_oracle():
    """Both couplings at once on a Cu box compressed by 2 %: box edge,
    positions and velocities against the oracle's Berendsen steps with the
    friction flow around the kicks."""
    wl = W.fcc4m(ncell=4)
    wl.pos, wl.box_len = wl.pos * 0.98, wl.box_len * 0.98
    L0 = wl.box_len[0, 0]
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.set_barostat(0.0, 100.0, 1.0)
    S.set_thermostat(TE, TAU)
    S.step(40)
    p, v = S.get_state()
    L = S.box()[0]
    flags, builds, steps = S.status()
    pr, _ = S.pressure()
    S.close()
    assert flags == 0 and steps == 40
    x, vo, Lo, pro, nreb = O.vv_baro(O.wrap(wl.pos, L0), wl.vel, L0, O.Pot(wl.pot), wl.mass,
                                     wl.dt, wl.skin, 40, 0.0, 100.0, 1.0, te=TE, tau_t=TAU)
    assert abs(L - Lo) <= 1e-13 * Lo
    d = p.cpu().numpy() - x
    d -= Lo * np.round(d / Lo)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v.cpu().numpy() - vo).max() <= 1e-9 * np.abs(vo).max()
    assert abs(float(pr[0]) - pro[-1]) <= 1e-10 * abs(pro[-1])
    assert builds == 1 + nreb


def test_thermostat_heats_crystal_to_electron_temperature():
    """Property at any size: SMTB Cu (5,324 atoms, from 300 K) coupled to
    electrons at 900 K settles there: mean kinetic temperature of the last
    400 steps within 5 % of T_e."""
    wl = W.fcc4m(ncell=11)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.set_thermostat(900.0, 50.0)
    S.step(800)
    t = []
    for _ in range(40):
        S.step(10)
        t.append(2 * float(S.kinetic()[0]) / (3 * wl.n_atoms * W.KB_EV))
    assert S.status()[0] == 0
    S.close()
    assert abs(np.mean(t) - 900.0) < 0.05 * 900.0, np.mean(t)


def test_thermostat_full_size_matches_oracle():
    """The 4,000,000-atom SMTB Cu box in the configuration the benchmark
    times (tiles, one captured graph of nine steps with fused force passes),
    thermostat on: the whole state after nine steps against the oracle."""
    wl = W.fcc4m()
    nsteps = 9
    check(wl, run(wl, nsteps), oracle_run(wl, nsteps), nsteps)
