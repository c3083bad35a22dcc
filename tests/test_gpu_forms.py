"""Forms (2) and (3) on the GPU against the oracle: the persistent batched
stepper for many uneven boxes, and the adjoint with respect to B-spline
coefficients."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1212_6332_amd import md, workloads as W
from paper_1212_6332_amd.autograd import SplineEAMFunction, force_matching_loss

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run_batch(wl, nsteps, batched=True, block=256):
    S = md.System.from_workload(wl)
    if batched:
        assert S.get_option(md.MD_OPT_BATCHED) == 1
        S.set_option(md.MD_OPT_BATCH_BLOCK, block)
    else:
        S.set_option(md.MD_OPT_BATCHED, 0)
    S.set_state(wl.pos, wl.vel)
    S.step(nsteps)
    p, v = S.get_state()
    flags, builds, steps = S.status()
    out = (p.cpu().numpy(), v.cpu().numpy(), flags, steps)
    S.close()
    return out


def oracle_batch(wl, nsteps):
    pot = O.Pot(wl.pot)
    P, V = np.zeros_like(wl.pos), np.zeros_like(wl.vel)
    for b, s, L in O.boxes(wl):
        x, v, *_ = O.vv(wl.pos[s], wl.vel[s], L, pot, wl.mass, wl.dt, wl.skin, nsteps,
                        energies=False)
        P[s], V[s] = x, v
    return P, V


def wrapped_diff(p, q, wl):
    d = p - q
    L = np.repeat(wl.box_len[:, 0], np.diff(wl.box_offset))[:, None]
    return d - L * np.round(d / L)


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_batched_matches_oracle(block):
    wl = W.batch2048(n_boxes=40)
    nsteps = 25
    p, v, flags, steps = run_batch(wl, nsteps, block=block)
    assert flags == 0 and steps == nsteps
    P, V = oracle_batch(wl, nsteps)
    assert np.abs(wrapped_diff(p, P, wl)).max() < 1e-10
    assert rel(v, V) < 1e-9


def analytic_boxes(make, ncells):
    """Several boxes of one analytic potential, of different sizes."""
    wls = [make(n) for n in ncells]
    off = np.concatenate([[0], np.cumsum([w.n_atoms for w in wls])]).astype(np.int64)
    return W.Workload(name="analytic_boxes", box_offset=off,
                      box_len=np.concatenate([w.box_len for w in wls]),
                      pos=np.concatenate([w.pos for w in wls]),
                      vel=np.concatenate([w.vel for w in wls]), mass=wls[0].mass, dt=1.0,
                      skin=0.3, pot=wls[0].pot, steps=0)


BOXES = {"smtb": (lambda n: W.fcc4m(ncell=n), (4, 5, 6, 4, 7)),
         "fs": (lambda n: W.fs256(ncell=n), (3, 4, 5, 3, 6))}


@pytest.mark.parametrize("kind", list(BOXES))
@pytest.mark.parametrize("batched", [True, False])
def test_analytic_boxes_match_oracle(kind, batched):
    """The analytic potentials (SMTB, FS) in the persistent stepper (which
    evaluates them itself) and in the merged-box kernels, per box against the
    oracle."""
    make, ncells = BOXES[kind]
    wl = analytic_boxes(make, ncells)
    nsteps = 25
    p, v, flags, steps = run_batch(wl, nsteps, batched=batched)
    assert flags == 0 and steps == nsteps
    P, V = oracle_batch(wl, nsteps)
    assert np.abs(wrapped_diff(p, P, wl)).max() < 1e-10
    assert rel(v, V) < 1e-9


def test_batched_equals_merged_box_path():
    wl = W.batch2048(n_boxes=32)
    a = run_batch(wl, 30, batched=True)
    b = run_batch(wl, 30, batched=False)
    assert np.abs(wrapped_diff(a[0], b[0], wl)).max() < 1e-10
    assert rel(a[1], b[1]) < 1e-9


def test_batched_box_independence_and_determinism():
    wl = W.batch2048(n_boxes=24)
    a = run_batch(wl, 20)
    a2 = run_batch(wl, 20)
    assert np.array_equal(a[0], a2[0]) and np.array_equal(a[1], a2[1])
    s = slice(int(wl.box_offset[5]), int(wl.box_offset[6]))
    wl.pos[s] += 0.01
    b = run_batch(wl, 20)
    other = np.ones(wl.n_atoms, bool)
    other[s] = False
    assert np.array_equal(a[0][other], b[0][other])
    assert not np.array_equal(a[0][s], b[0][s])


def test_batched_forces_then_generic():
    """After batched steps, md_forces (merged-box list) sees the new state."""
    wl = W.batch2048(n_boxes=16)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(15)
    f, e, eb = S.forces()
    p, v = S.get_state()
    S.close()
    p = p.cpu().numpy()
    ref = O.forces_multi(wl, pos=p)
    assert rel(f.cpu().numpy(), ref["f"]) < 1e-11
    assert rel(eb.cpu().numpy(), ref["E_box"]) < 1e-11


# ------------------------------------------------------------------ adjoint

def adjoint_setup(n_boxes):
    wl = W.adjoint64(n_boxes=n_boxes)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos)
    return wl, S


@pytest.mark.parametrize("n_boxes", [3, 64])
def test_adjoint_vjp_matches_oracle(n_boxes):
    wl, S = adjoint_setup(n_boxes)
    rng = np.random.default_rng(11)
    g = rng.normal(size=(wl.n_atoms, 3))
    e = rng.normal(size=wl.n_boxes)
    gt = S.adjoint(torch.tensor(g, device="cuda"), torch.tensor(e, device="cuda")).cpu().numpy()
    gt2 = S.adjoint(torch.tensor(g, device="cuda"), torch.tensor(e, device="cuda")).cpu().numpy()
    assert np.array_equal(gt, gt2)
    assert S.status()[0] == 0
    S.close()
    pot = O.Pot(wl.pot)
    ref = np.zeros(192)
    for b, s, L in O.boxes(wl):
        O.adjoint(O.wrap(wl.pos[s], L), L, pot, g[s], e[b], gtheta=ref)
    for blk in range(3):
        sl = slice(64 * blk, 64 * blk + 64)
        assert rel(gt[sl], ref[sl]) < 1e-10, (blk, rel(gt[sl], ref[sl]))


@pytest.mark.parametrize("ncoef", [200, 700, 2730])
def test_adjoint_many_coefficients_matches_oracle(ncoef):
    """Coefficient counts whose LDS columns leave room for fewer atoms per
    workgroup (more lanes per atom: 16 lanes at 200, 64 at 700 and at the
    largest count a context accepts, 2,730)."""
    wl = W.adjoint64(n_boxes=3)
    par = W.draw_fs(np.random.default_rng(21), "bcc", 2.8665, 5.3)
    r, n = W.shells("bcc", 2.8665, 5.3)
    rho0 = float((n * (r - 5.3) ** 2).sum())
    pot = W.bspline_from_fs(par, 1.5, 5.3, 2.0 * rho0, ncoef=ncoef)
    S = md.System.from_workload(wl, pot)
    S.set_state(wl.pos)
    rng = np.random.default_rng(12)
    g = rng.normal(size=(wl.n_atoms, 3))
    e = rng.normal(size=wl.n_boxes)
    gt = S.adjoint(torch.tensor(g, device="cuda"), torch.tensor(e, device="cuda")).cpu().numpy()
    assert S.status()[0] == 0
    S.close()
    opot = O.Pot(pot)
    ref = np.zeros(3 * ncoef)
    for b, s, L in O.boxes(wl):
        O.adjoint(O.wrap(wl.pos[s], L), L, opot, g[s], e[b], gtheta=ref)
    for blk in range(3):
        sl = slice(ncoef * blk, ncoef * (blk + 1))
        assert rel(gt[sl], ref[sl]) < 1e-10, (blk, rel(gt[sl], ref[sl]))


def test_autograd_loss_gradient_matches_oracle():
    wl, S = adjoint_setup(4)
    w = wl.extra["w"]
    tgt = O.forces_multi(wl, pot=O.Pot(wl.extra["target_pot"]))
    th = [torch.tensor(t, device="cuda", requires_grad=True) for t in wl.pot.tables]
    ft = torch.tensor(tgt["f"], device="cuda")
    et = torch.tensor(tgt["E_box"], device="cuda")
    loss = force_matching_loss(S, th[0], th[1], th[2], ft, et, w)
    loss.backward()
    grad = torch.cat([t.grad for t in th]).cpu().numpy()
    S.close()
    # oracle: forward, loss derivatives, adjoint
    pot = O.Pot(wl.pot)
    out = O.forces_multi(wl, pot=pot)
    L0 = float(((out["f"] - tgt["f"]) ** 2).sum() + w * ((out["E_box"] - tgt["E_box"]) ** 2).sum())
    assert abs(float(loss) - L0) <= 1e-11 * L0
    g = 2.0 * (out["f"] - tgt["f"])
    e = 2.0 * w * (out["E_box"] - tgt["E_box"])
    ref = np.zeros(192)
    for b, s, L in O.boxes(wl):
        O.adjoint(O.wrap(wl.pos[s], L), L, pot, g[s], e[b], gtheta=ref)
    assert rel(grad, ref) < 1e-9


def test_set_theta_sees_in_place_changes():
    """A second upload of the same coefficient tensor is skipped only while
    its contents are unchanged: an in-place update (as an optimiser makes)
    reaches the device, and so does a view of the updated memory."""
    import dataclasses
    wl, S = adjoint_setup(2)
    theta = torch.tensor(np.concatenate(wl.pot.tables), device="cuda")
    S.set_theta(theta)
    S.forces()
    with torch.no_grad():
        theta[64:128] *= 1.01  # rho(r)
        theta[:64] -= 0.002    # V(r)
    S.set_theta(theta)
    f1, _, e1 = S.forces(energy=True)
    S.set_theta(theta.view(3, 64))  # same memory and version: no upload needed
    f2, _, e2 = S.forces(energy=True)
    S.close()
    tabs = theta.view(3, 64).cpu().numpy()
    pot = O.Pot(dataclasses.replace(wl.pot, tables=tuple(np.array(t) for t in tabs)))
    ref = O.forces_multi(wl, pot=pot)
    assert rel(f1.cpu().numpy(), ref["f"]) < 1e-11
    assert rel(e1.cpu().numpy(), ref["E_box"]) < 1e-11
    assert torch.equal(f1, f2) and torch.equal(e1, e2)


def test_graphed_loss_replays_match_eager_and_oracle():
    """The loss and its backward pass captured in a graph and replayed with
    new coefficients (eager evaluations between the replays) give the eager
    loss and gradient bit for bit every time, and the last one matches the
    oracle; once the system moves on, replay is refused."""
    import dataclasses
    from paper_1212_6332_amd.autograd import GraphedLoss
    wl, S = adjoint_setup(4)
    w = wl.extra["w"]
    tgt = O.forces_multi(wl, pot=O.Pot(wl.extra["target_pot"]))
    ft = torch.tensor(tgt["f"], device="cuda")
    et = torch.tensor(tgt["E_box"], device="cuda")
    th = [torch.tensor(t, device="cuda", requires_grad=True) for t in wl.pot.tables]
    G = GraphedLoss(S, th, lambda: force_matching_loss(S, *th, ft, et, w))
    rng = np.random.default_rng(5)
    for rep in range(4):
        vals = [np.asarray(t) * (1 + 0.01 * rng.normal(size=np.shape(t))) for t in wl.pot.tables]
        with torch.no_grad():
            for t, v in zip(th, vals):
                t.copy_(torch.tensor(v, device="cuda"))
        loss, grads = G.replay()
        lg, gg = float(loss), torch.cat(grads).cpu().numpy()
        ts = [torch.tensor(v, device="cuda", requires_grad=True) for v in vals]
        le = force_matching_loss(S, *ts, ft, et, w)
        le.backward()
        assert lg == float(le), rep
        assert np.array_equal(gg, torch.cat([t.grad for t in ts]).cpu().numpy()), rep
    pot = O.Pot(dataclasses.replace(wl.pot, tables=tuple(vals)))
    out = O.forces_multi(wl, pot=pot)
    L0 = float(((out["f"] - tgt["f"]) ** 2).sum() + w * ((out["E_box"] - tgt["E_box"]) ** 2).sum())
    assert abs(lg - L0) <= 1e-11 * L0
    g = 2.0 * (out["f"] - tgt["f"])
    e = 2.0 * w * (out["E_box"] - tgt["E_box"])
    ref = np.zeros(192)
    for b, s, L in O.boxes(wl):
        O.adjoint(O.wrap(wl.pos[s], L), L, pot, g[s], e[b], gtheta=ref)
    assert rel(gg, ref) < 1e-9
    S.step(1)
    with pytest.raises(RuntimeError):
        G.replay()
    S.close()


def test_autograd_matches_finite_differences():
    wl, S = adjoint_setup(2)
    w = wl.extra["w"]
    tgt = O.forces_multi(wl, pot=O.Pot(wl.extra["target_pot"]))
    ft = torch.tensor(tgt["f"], device="cuda")
    et = torch.tensor(tgt["E_box"], device="cuda")
    base = [torch.tensor(t, device="cuda") for t in wl.pot.tables]
    th = [t.clone().requires_grad_(True) for t in base]
    loss = force_matching_loss(S, *th, ft, et, w)
    loss.backward()
    grad = torch.cat([t.grad for t in th]).cpu().numpy()
    h = 1e-6
    eps = np.finfo(float).eps
    for k in (3, 40, 64 + 10, 64 + 55, 128 + 20, 128 + 33):
        vals = []
        for sgn in (1, -1):
            t2 = [t.clone() for t in base]
            t2[k // 64][k % 64] += sgn * h
            with torch.no_grad():
                vals.append(float(force_matching_loss(S, *t2, ft, et, w)))
        fd = (vals[0] - vals[1]) / (2 * h)
        tol = 1e-6 * np.abs(grad).max() + 50 * eps * float(loss) / h
        assert abs(fd - grad[k]) <= tol, (k, fd, grad[k])
    S.close()


def test_batched_full_size_sampled_boxes():
    """All 2,048 boxes in the configuration the benchmark times (persistent
    stepper), 10 steps; 16 boxes drawn at random, and the largest and the
    smallest, against the oracle box by box."""
    wl = W.batch2048()
    nsteps = 10
    p, v, flags, steps = run_batch(wl, nsteps)
    assert flags == 0 and steps == nsteps
    sizes = np.diff(wl.box_offset)
    pick = set(np.random.default_rng(11).choice(wl.n_boxes, 16, replace=False).tolist())
    pick |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
    pot = O.Pot(wl.pot)
    for b in sorted(pick):
        s = slice(int(wl.box_offset[b]), int(wl.box_offset[b + 1]))
        L = float(wl.box_len[b, 0])
        x, vo, *_ = O.vv(wl.pos[s], wl.vel[s], L, pot, wl.mass, wl.dt, wl.skin, nsteps,
                         energies=False)
        d = p[s] - x
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-10, b
        assert np.abs(v[s] - vo).max() <= 1e-9 * np.abs(vo).max(), b


def test_autotune_and_graph_replay_keep_the_trajectory():
    """md_autotune between md_set_state and md_step picks a workgroup size and
    leaves the trajectory bitwise that of an untuned context with that size;
    250 steps (one launch that rebuilds, one replayed graph of 100 steps, a
    tail) equal direct launches bitwise; a one-box context has nothing to
    tune."""
    wl = W.batch2048(n_boxes=40)

    def run(tune, block=None, use_graph=1):
        S = md.System.from_workload(wl)
        S.set_option(md.MD_OPT_USE_GRAPH, use_graph)
        if block is not None:
            S.set_option(md.MD_OPT_BATCH_BLOCK, block)
        S.set_state(wl.pos, wl.vel)
        chosen = S.autotune() if tune else S.get_option(md.MD_OPT_BATCH_BLOCK)
        S.step(250)
        p, v = S.get_state()
        st = S.status()
        S.close()
        return chosen, p.cpu().numpy(), v.cpu().numpy(), st

    t, p1, v1, st1 = run(True)
    assert t in (256, 512, 1024) and st1[0] == 0 and st1[2] == 250
    _, p2, v2, st2 = run(False, t)
    _, p3, v3, st3 = run(False, t, use_graph=0)
    assert np.array_equal(p1, p2) and np.array_equal(v1, v2)
    assert np.array_equal(p2, p3) and np.array_equal(v2, v3) and st2 == st3
    one = md.System.from_workload(W.fs256())
    one.set_state(W.fs256().pos, W.fs256().vel)
    assert one.autotune() == one.get_option(md.MD_OPT_BATCH_BLOCK)
    one.close()


@pytest.mark.parametrize("name", ["bcc128k", "smtb5324"])
def test_autotune_single_box_keeps_the_trajectory(name):
    """For one box md_autotune chooses between the tiled and the per-atom
    passes by timing them; the trajectory afterwards is bitwise that of an
    untuned context with the chosen setting, and matches the oracle."""
    wl = W.bcc128k() if name == "bcc128k" else W.fcc4m(ncell=11)
    nsteps = 30

    def run(tune, tiled=None):
        S = md.System.from_workload(wl)
        if tiled is not None:
            S.set_option(md.MD_OPT_TILED, tiled)
        S.set_state(wl.pos, wl.vel)
        if tune:
            S.autotune()
        chosen = S.get_option(md.MD_OPT_TILED)
        S.step(nsteps)
        p, v = S.get_state()
        st = S.status()
        S.close()
        return chosen, p.cpu().numpy(), v.cpu().numpy(), st

    t, p1, v1, st1 = run(True)
    assert t in (0, 1) and st1[0] == 0
    other = 1 - t
    _, p2, v2, _ = run(False, t)
    assert np.array_equal(p1, p2) and np.array_equal(v1, v2)
    _, p3, v3, _ = run(False, other)
    L = wl.box_len[0, 0]
    d = p1 - p3
    assert np.abs(d - L * np.round(d / L)).max() < 1e-9
    if name == "smtb5324":
        x, v, *_ = O.vv(wl.pos, wl.vel, L, O.Pot(wl.pot), wl.mass, wl.dt, wl.skin, nsteps,
                        energies=False)
        d = p1 - x
        assert np.abs(d - L * np.round(d / L)).max() < 1e-10
        assert rel(v1, v) < 1e-9
