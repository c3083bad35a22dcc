"""Pairs one rounding step inside or outside the force cutoff and the list
radius, inside the box and across a periodic face, through every path that
evaluates pairs: tiled passes (halo modes A and B), per-atom passes, the
persistent multi-box stepper and the adjoint.  Each path must decide these
pairs exactly as the oracle does (separation, then the periodic shift, then
(dx dx + dy dy) + dz dz rounded term by term, strict <): rows bit-exact and
densities, F', forces and energies within 1e-11 (the adjoint within 1e-10,
its bar elsewhere).  tests/test_edge_fixture.py checks on the CPU that every
such pair would be decided the other way by a fused sum of squares or by a
shift added before the difference.
"""
import numpy as np
import pytest
import torch

import edge_pairs as E
import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def smtb_edge(ncell, seed):
    wl = W.fcc4m(ncell=ncell)
    L = float(wl.box_len[0, 0])
    rc = wl.pot.rc
    rl = O.rlist(rc, wl.skin, L)
    radii = [(rc, True, False), (rc, False, False), (rc, True, True), (rc, False, True),
             (rl, True, False), (rl, False, True)]
    pos, pairs = E.edge_state(O.wrap(wl.pos, L), L, radii, np.random.default_rng(seed))
    wl.pos = pos
    return wl, pairs


def multi(wls):
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    return W.Workload(name="edge_boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.zeros((int(off[-1]), 3)), mass=wls[0].mass, dt=1.0,
                      skin=wls[0].skin, pot=wls[0].pot, steps=0)


@pytest.mark.parametrize("ncell,seed,tiled", [(14, 5, 1), (14, 5, 0), (4, 7, 1), (4, 7, 0),
                                              (6, 9, 1)])
def test_single_box_edge_pairs(ncell, seed, tiled):
    """ncell 14: 8 cells per axis, tiles with halo mode A; ncell 4 and 6: one
    tile per box (mode B).  tiled = 0: the per-atom kernels."""
    wl, pairs = smtb_edge(ncell, seed)
    L = float(wl.box_len[0, 0])
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos)
    rho = S.density().cpu().numpy()
    F, Fp = (t.cpu().numpy() for t in S.embed())
    f, e, eb = (t.cpu().numpy() for t in S.forces())
    counts, ids = (t.cpu().numpy() for t in S.neighbors())
    flags = S.status()[0]
    S.close()
    assert flags == 0
    rl = O.rlist(wl.pot.rc, wl.skin, L)
    count, oid = O.neighbor_list(wl.pos, L, rl)
    for i in range(wl.n_atoms):
        assert counts[i] == count[i], i
        assert sorted(ids[i, :counts[i]].tolist()) == oid[i, :count[i]].tolist(), i
    o = O.forces(wl.pos, L, O.Pot(wl.pot), count, oid)
    for k, g in (("rho", rho), ("F", F), ("Fp", Fp), ("e_atom", e)):
        assert rel(g, o[k]) <= TOL, (k, rel(g, o[k]))
    assert rel(f, o["f"]) <= TOL, rel(f, o["f"])
    assert abs(eb[0] - o["E"]) <= TOL * abs(o["E"])
    # the edge atoms themselves, elementwise
    for i, j, r, inside, cross in pairs:
        for a in (i, j):
            assert abs(rho[a] - o["rho"][a]) <= TOL * o["rho"][a]


def test_batched_stepper_edge_pairs():
    """The persistent multi-box stepper's own density and force evaluation
    (md_step with no step, then md_forces returns its forces) on SMTB boxes
    with edge pairs in each box."""
    boxes = [smtb_edge(n, s)[0] for n, s in ((4, 3), (5, 4), (6, 5), (4, 6))]
    wl = multi(boxes)
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_BATCHED) == 1
    S.set_state(wl.pos)
    S.step(0)
    f = S.forces(energy=False).cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    pot = O.Pot(wl.pot)
    for b, s, L in O.boxes(wl):
        o = O.forces(wl.pos[s], L, pot, skin=wl.skin)
        assert rel(f[s], o["f"]) <= TOL, (b, rel(f[s], o["f"]))


def test_adjoint_edge_pairs():
    """B-spline boxes with pairs one step inside and outside rc: forces and
    the coefficient gradient against the oracle."""
    wl = W.adjoint64(n_boxes=3)
    rc = wl.pot.rc
    pos = wl.pos.copy()
    for b, s, L in O.boxes(wl):
        radii = [(rc, True, False), (rc, False, False), (rc, True, True), (rc, False, True)]
        p, _ = E.edge_state(O.wrap(pos[s], L), L, radii, np.random.default_rng(40 + b))
        pos[s] = p
    wl.pos = pos
    rng = np.random.default_rng(12)
    g = rng.normal(size=(wl.n_atoms, 3))
    e = rng.normal(size=wl.n_boxes)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos)
    f = S.forces(energy=False).cpu().numpy()
    gt = S.adjoint(torch.tensor(g, device="cuda"), torch.tensor(e, device="cuda")).cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    pot = O.Pot(wl.pot)
    ref = np.zeros(gt.size)
    for b, s, L in O.boxes(wl):
        o = O.forces(wl.pos[s], L, pot, skin=wl.skin)
        assert rel(f[s], o["f"]) <= TOL, (b, rel(f[s], o["f"]))
        O.adjoint(wl.pos[s], L, pot, g[s], e[b], skin=wl.skin, gtheta=ref)
    K = gt.size // 3
    for blk in range(3):
        sl = slice(K * blk, K * blk + K)
        assert rel(gt[sl], ref[sl]) < 1e-10, (blk, rel(gt[sl], ref[sl]))
