"""Cutoffs per pair of types, RCUT(a, b) (Sections 3.2-3.3), on the GPU
against the oracle, with tables that do not vanish at those cutoffs (so the
cutoffs change the result) and with pairs of the chosen types placed one
rounding step inside or outside RCUT(a, b) and RCUT(a, b) + skin, in the box
and across a periodic face: rows bit-exact (the list radius is taken per
pair), densities, F', forces and energies within 1e-11; tiled passes (halo
mode A) and per-atom passes."""
import numpy as np
import pytest

import edge_pairs as E
import oracle as O
from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11
RCP = np.array([[5.3, 5.1], [5.1, 4.9]])


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def case(ncell, seed):
    wl = W.alloy(ncell=ncell)
    t = wl.pot
    wl.pot = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, t.hi, n_types=2,
                         rc_pair=RCP.copy())
    L = float(wl.box_len[0, 0])
    rl = lambda r: O.rlist(r, wl.skin, L)
    want = [(4.9, True, False, 1, 1), (4.9, False, True, 1, 1), (5.1, True, True, 0, 1),
            (5.1, False, False, 1, 0), (rl(4.9), True, False, 1, 1),
            (rl(5.1), False, True, 0, 1), (rl(4.9), False, True, 1, 1)]
    pos, pairs = E.edge_state(O.wrap(wl.pos, L), L, [w[:3] for w in want],
                              np.random.default_rng(seed))
    types = wl.types.copy()
    for (i, j, r, inside, cross), w in zip(pairs, want):
        types[i], types[j] = w[3], w[4]
    wl.pos, wl.types = pos, types
    return wl, L


@pytest.mark.parametrize("tiled", [1, 0])
def test_pair_cutoffs_match_oracle(tiled):
    wl, L = case(14, 31)
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    rho = S.density().cpu().numpy()
    F, Fp = (t.cpu().numpy() for t in S.embed())
    f, e, eb = (t.cpu().numpy() for t in S.forces())
    counts, ids = (t.cpu().numpy() for t in S.neighbors())
    flags = S.status()[0]
    S.close()
    assert flags == 0
    pot = O.Alloy(wl.pot)
    cnt, oid = O.alloy_list(wl.pos, L, pot, wl.types, wl.skin)
    for i in range(wl.n_atoms):
        assert counts[i] == cnt[i], i
        assert sorted(ids[i, :counts[i]].tolist()) == oid[i, :cnt[i]].tolist(), i
    o = O.alloy_eval(wl.pos, L, pot, wl.types, cnt, oid)
    for k, g in (("rho", rho), ("F", F), ("Fp", Fp), ("e_atom", e)):
        assert rel(g, o[k]) <= TOL, (k, rel(g, o[k]))
    assert rel(f, o["f"]) <= TOL
    assert abs(eb[0] - o["E"]) <= TOL * abs(o["E"])
    # the per-pair cutoffs matter here: one cutoff for all pairs differs
    one = W.Potential(wl.pot.kind, wl.pot.rc, wl.pot.params, wl.pot.tables, wl.pot.lo,
                      wl.pot.hi, n_types=2)
    c2, i2 = O.alloy_list(wl.pos, L, O.Alloy(one), wl.types, wl.skin)
    assert rel(O.alloy_eval(wl.pos, L, O.Alloy(one), wl.types, c2, i2)["f"], o["f"]) > 1e-6


def test_pair_cutoff_descriptor_checks():
    wl = W.alloy(ncell=4)
    t = wl.pot
    for bad in (np.array([[5.3, 5.1], [5.0, 4.9]]),      # not symmetric
                np.array([[5.4, 5.1], [5.1, 4.9]]),      # above rc
                np.array([[5.3, 0.0], [0.0, 4.9]])):     # not positive
        p = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, t.hi, n_types=2, rc_pair=bad)
        with pytest.raises(md.MDError) as e:
            md.System.from_workload(wl, p)
        assert e.value.code == md.MD_ERR_ARG


def test_pair_cutoff_trajectory_matches_oracle():
    wl = W.alloy(ncell=6)
    t = wl.pot
    wl.pot = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, t.hi, n_types=2,
                         rc_pair=RCP.copy())
    L = float(wl.box_len[0, 0])
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(30)
    p, v = (t.cpu().numpy() for t in S.get_state())
    S.close()
    x, vo, *_ = O.alloy_vv(wl.pos, wl.vel, L, O.Alloy(wl.pot), wl.types, wl.type_mass, wl.dt,
                           wl.skin, 30, energies=False)
    d = p - x
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10
    assert rel(v, vo) < 1e-9


@pytest.mark.parametrize("tiled", [1, 0])
def test_set_potential_changes_pair_cutoffs(tiled):
    """md_set_potential with other cutoffs per pair: the lists are built again
    and the forces are the oracle's for the new cutoffs; another rc is refused."""
    wl, L = case(14, 37)
    t = wl.pot
    S = md.System.from_workload(wl)
    S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    S.forces()
    other = W.Potential(t.kind, t.rc, t.params, t.tables, t.lo, t.hi, n_types=2,
                        rc_pair=np.array([[5.2, 5.0], [5.0, 4.8]]))
    S.set_potential(other)
    f, e, eb = (x.cpu().numpy() for x in S.forces())
    assert S.status()[0] == 0
    bad_rc = W.Potential(t.kind, 5.2, t.params, t.tables, t.lo, t.hi, n_types=2)
    with pytest.raises(md.MDError) as err:
        S.set_potential(bad_rc)
    assert err.value.code == md.MD_ERR_ARG
    S.close()
    pot = O.Alloy(other)
    cnt, oid = O.alloy_list(wl.pos, L, pot, wl.types, wl.skin)
    o = O.alloy_eval(wl.pos, L, pot, wl.types, cnt, oid)
    assert rel(f, o["f"]) <= TOL
    assert abs(eb[0] - o["E"]) <= TOL * abs(o["E"])
