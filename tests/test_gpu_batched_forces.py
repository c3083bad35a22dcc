"""The persistent multi-box stepper's own force evaluation against the oracle.

md_step(ctx, 0) brings the list and forces up to date with the kernels that
would take the steps, and md_forces without energies then returns those
forces as computed, so the stepper's density and force code (which is not
the merged-box kernels') is compared with the oracle force by force, at
1e-11 per box, on the state it was given and again after one step in which
every box rebuilds its list.
"""
import numpy as np
import pytest

import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def boxes_of(make, ncells):
    wls = [make(n) for n in ncells]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    return W.Workload(name="boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.concatenate([w.vel for w in wls]), mass=wls[0].mass, dt=1.0,
                      skin=0.3, pot=wls[0].pot, steps=0)


CASES = {
    # spline tables; n = 3 boxes (108 atoms) have the list radius clamped to L/2
    "spline": lambda: W.batch2048(n_boxes=40),
    "smtb": lambda: boxes_of(lambda n: W.fcc4m(ncell=n), (4, 5, 6, 4, 7)),
    "fs": lambda: boxes_of(lambda n: W.fs256(ncell=n), (3, 4, 5, 3, 6)),
}


def oracle_box_forces(wl, pos):
    pot = O.Pot(wl.pot)
    out = np.zeros_like(pos)
    for b, s, L in O.boxes(wl):
        out[s] = O.forces(O.wrap(pos[s], L), L, pot, skin=wl.skin)["f"]
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_stepper_forces_match_oracle(name):
    wl = CASES[name]()
    if name == "spline":
        assert (np.diff(wl.box_offset) == 108).any()
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_BATCHED) == 1
    vel = np.zeros_like(wl.vel)
    # one atom per box fast enough to move past half the skin in one step
    first = wl.box_offset[:-1]
    vel[first, 0] = 0.4
    S.set_state(wl.pos, vel)
    S.step(0)
    f0 = S.forces(energy=False).cpu().numpy()
    ref0 = oracle_box_forces(wl, wl.pos)
    S.step(1)
    f1 = S.forces(energy=False).cpu().numpy()
    p1, _ = S.get_state()
    p1 = p1.cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    ref1 = oracle_box_forces(wl, p1)
    for b, s, L in O.boxes(wl):
        assert rel(f0[s], ref0[s]) <= TOL, (b, rel(f0[s], ref0[s]))
        assert rel(f1[s], ref1[s]) <= TOL, (b, rel(f1[s], ref1[s]))
    # the fast atoms did move past half the skin (so each box rebuilt)
    d = p1[first] - wl.pos[first]
    L = wl.box_len[:, 0]
    d[:, 0] -= L * np.round(d[:, 0] / L)
    assert (np.abs(d[:, 0]) > 0.15).all()


def test_set_state_again_on_a_batched_context():
    """set_state, steps, a merged-box force pass (which re-sorts the slots),
    steps, then set_state with another state: the trajectory from there is
    bitwise that of a fresh context given that state."""
    wl = W.batch2048(n_boxes=24)
    rng = np.random.default_rng(3)
    pos_b = wl.pos + rng.normal(scale=0.02, size=wl.pos.shape)
    vel_b = wl.vel[::-1].copy()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(7)
    S.forces()
    S.step(5)
    S.set_state(pos_b, vel_b)
    S.step(9)
    p, v = (t.cpu().numpy() for t in S.get_state())
    S.close()
    T = md.System.from_workload(wl)
    T.set_state(pos_b, vel_b)
    T.step(9)
    q, u = (t.cpu().numpy() for t in T.get_state())
    T.close()
    assert np.array_equal(p, q) and np.array_equal(v, u)
