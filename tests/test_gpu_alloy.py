"""Several species (eqs. 1-3 with per-type-pair tables) on the HIP path
against the oracle, through the C ABI.

Bars as for one species: neighbour rows bit-exact; densities, embedding
values, forces, per-atom and per-box energies within 1e-11 normwise;
trajectories with per-species masses within 1e-10 Angstrom and 1e-9 relative
in velocities; pressures within 1e-11.
"""
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


def merged(*wls):
    """Several alloy boxes in one workload (types and masses carried along)."""
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    w0 = wls[0]
    return W.Workload(name="alloy_boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.concatenate([w.vel for w in wls]), mass=w0.mass, dt=w0.dt,
                      skin=w0.skin, pot=w0.pot, steps=0, types=np.concatenate(
                          [w.types for w in wls]), type_mass=w0.type_mass)


CASES = {
    "alloy256": (lambda: W.alloy(ncell=4), None),           # one tile (halo mode B)
    "alloy6912_tiled": (lambda: W.alloy(ncell=12), None),   # 7 cells per axis: tiles, mode A
    "alloy6912_per_atom": (lambda: W.alloy(ncell=12), 0),
    "alloy_boxes": (lambda: merged(W.alloy(ncell=4), W.alloy(ncell=5, frac=0.6)), None),
}


def oracle_eval(wl):
    pot = O.Alloy(wl.pot)
    n = wl.n_atoms
    res = {k: np.zeros(n) for k in ("rho", "F", "Fp", "e_atom")}
    res["f"] = np.zeros((n, 3))
    res["E_box"] = np.zeros(wl.n_boxes)
    res["W"] = np.zeros(wl.n_boxes)
    res["rows"] = [None] * n
    for b, s, L in O.boxes(wl):
        p = O.wrap(wl.pos[s], L)
        cnt, ids = O.alloy_list(p, L, pot, wl.types[s], wl.skin)
        r = O.alloy_eval(p, L, pot, wl.types[s], cnt, ids)
        for k in ("rho", "F", "Fp", "e_atom", "f"):
            res[k][s] = r[k]
        res["E_box"][b] = r["E"]
        res["W"][b] = r["W"]
        for i in range(s.stop - s.start):
            res["rows"][s.start + i] = (ids[i, :cnt[i]] + s.start).tolist()
    return res


def gpu_eval(wl, tiled=None):
    S = md.System.from_workload(wl)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    S.set_state(wl.pos, wl.vel)
    S.build_neighbors()
    rho = S.density()
    F, Fp = S.embed()
    f, e, eb = S.forces()
    counts, ids = S.neighbors()
    p, w = S.pressure()
    flags, _, _ = S.status()
    out = {k: v.cpu().numpy() for k, v in dict(rho=rho, F=F, Fp=Fp, f=f, e_atom=e, E_box=eb,
                                                 counts=counts, ids=ids, P=p, W=w).items()}
    out["flags"] = flags
    S.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_alloy_passes_match_oracle(name):
    make, tiled = CASES[name]
    wl = make()
    g, o = gpu_eval(wl, tiled), oracle_eval(wl)
    assert g["flags"] == 0
    for i, row in enumerate(o["rows"]):
        assert g["counts"][i] == len(row), i
        assert sorted(g["ids"][i, :g["counts"][i]].tolist()) == row, i
    for k in ("rho", "F", "Fp", "e_atom", "E_box", "f"):
        assert rel(g[k], o[k]) <= TOL, (k, rel(g[k], o[k]))
    assert np.all(np.abs(g["W"] - o["W"]) <= TOL * np.maximum(np.abs(o["W"]), 1.0))
    # pressure of eq. (6) with per-species masses in the kinetic term
    for b, s, L in O.boxes(wl):
        m = wl.type_mass[wl.types[s]][:, None]
        K = 0.5 * float((m * wl.vel[s] ** 2).sum()) / W.KAPPA
        P = (2 * K + o["W"][b]) / (3 * L ** 3)
        assert abs(g["P"][b] - P) <= TOL * max(abs(P), 1e-6)


def run(wl, nsteps, tiled=None, use_graph=1, te=0.0, tau=0.0):
    S = md.System.from_workload(wl)
    if tiled is not None:
        S.set_option(md.MD_OPT_TILED, tiled)
    S.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    S.set_state(wl.pos, wl.vel)
    if tau > 0:
        S.set_thermostat(te, tau)
    S.step(nsteps)
    p, v = S.get_state()
    st = S.status()
    S.close()
    return p.cpu().numpy(), v.cpu().numpy(), st


@pytest.mark.parametrize("name,tiled,thermo", [("alloy6912", None, False),
                                               ("alloy6912", 0, False),
                                               ("alloy6912", None, True),
                                               ("alloy256", None, True)])
def test_alloy_trajectory_matches_oracle(name, tiled, thermo):
    """Velocity Verlet with per-species masses (and the friction of eq. (4)
    per species), device-decided rebuilds, against the oracle."""
    wl = W.alloy(ncell=12 if name == "alloy6912" else 4)
    L = wl.box_len[0, 0]
    te, tau = (700.0, 25.0) if thermo else (0.0, 0.0)
    nsteps = 40
    p, v, (flags, builds, steps) = run(wl, nsteps, tiled, te=te, tau=tau)
    assert flags == 0 and steps == nsteps
    x, vo, _, _, nreb = O.alloy_vv(O.wrap(wl.pos, L), wl.vel, L, O.Alloy(wl.pot), wl.types,
                                   wl.type_mass, wl.dt, wl.skin, nsteps, te, tau,
                                   energies=False)
    d = p - x
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v - vo).max() <= 1e-9 * np.abs(vo).max()
    assert builds == 1 + nreb


def test_alloy_graph_equals_direct_launches():
    wl = W.alloy(ncell=12)
    a = run(wl, 37, use_graph=1, te=500.0, tau=40.0)
    b = run(wl, 37, use_graph=0, te=500.0, tau=40.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert a[2][1] >= 2


def test_set_types_checks_and_changes():
    """Types out of range, non-positive masses, a single-species context and
    the persistent multi-box stepper on one box are refused; new types after
    the state is set take effect at once (rows carry the neighbours' species)."""
    wl = W.alloy(ncell=12)
    S = md.System.from_workload(wl)
    assert S.get_option(md.MD_OPT_BATCHED) == 0
    with pytest.raises(md.MDError):
        S.set_option(md.MD_OPT_BATCHED, 1)
    bad = wl.types.copy()
    bad[5] = 2
    with pytest.raises(md.MDError):
        S.set_types(bad, wl.type_mass)
    with pytest.raises(md.MDError):
        S.set_types(wl.types, np.array([63.5, 0.0]))
    S.set_state(wl.pos, wl.vel)
    S.forces()
    flipped = (1 - wl.types).astype(np.int32)
    S.set_types(flipped, wl.type_mass)
    f, e, eb = S.forces()
    assert S.status()[0] == 0
    S.close()
    L = wl.box_len[0, 0]
    p = O.wrap(wl.pos, L)
    cnt, ids = O.alloy_list(p, L, O.Alloy(wl.pot), flipped, wl.skin)
    r = O.alloy_eval(p, L, O.Alloy(wl.pot), flipped, cnt, ids)
    assert rel(f.cpu().numpy(), r["f"]) <= TOL
    assert abs(float(eb[0]) - r["E"]) <= TOL * abs(r["E"])
    one = md.System.from_workload(W.fs256())
    with pytest.raises(md.MDError):
        one.set_types(np.zeros(256, dtype=np.int32))
    one.close()


def test_alloy_full_size_matches_oracle():
    """The 4,000,000-atom binary alloy in the configuration the benchmark
    times: every force, density and energy against the oracle's list pass."""
    wl = W.alloy()
    L = wl.box_len[0, 0]
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    f, e, eb = S.forces()
    rho = S.density()
    flags, _, _ = S.status()
    f, e, rho = f.cpu().numpy(), e.cpu().numpy(), rho.cpu().numpy()
    S.close()
    assert flags == 0
    p = O.wrap(wl.pos, L)
    cnt, ids = O.alloy_list(p, L, O.Alloy(wl.pot), wl.types, wl.skin, maxn=96)
    r = O.alloy_eval(p, L, O.Alloy(wl.pot), wl.types, cnt, ids)
    assert rel(f, r["f"]) <= TOL
    assert rel(rho, r["rho"]) <= TOL
    assert rel(e, r["e_atom"]) <= TOL
    assert abs(float(eb[0]) - r["E"]) <= TOL * abs(r["E"])
