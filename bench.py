#!/usr/bin/env python3
"""Throughput of the FP64 many-body MD step on one MI355X.

Headline: atom-steps/s of velocity-Verlet steps (list rebuilds decided on the
device, density + embedding, force + kick) for the 4,000,000-atom FCC
second-moment tight-binding workload, inputs resident in HBM.  Also reported:
the roofline position of the dominant kernel (the force pass), the batched
many-box stepper (box-steps/s), the adjoint (gradient evaluations/s), the
128,000-atom spline workload, and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                    # MI355X HBM3E
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # FP64 VALU lane-operations: 256 CUs x 64 lanes x 2.4 GHz
METRIC = "atom-steps/s FP64 EAM step at 4M atoms; HBM GB/s fraction; batched box-steps/s"
COUNTERS = os.path.join(ROOT, "profiles", "step_force_fcc4m_counters.txt")
CSRC = os.path.join(ROOT, "paper_1212_6332_amd", "csrc")
# the sources the force kernel is compiled from
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("md_tiled.hip", "md_device.h", "md_internal.h")]
FORCE_KERNEL = "k_tile_force<2, false, 2, 1>"

# Algorithmic FP64 work, in lane-operations (one VALU operation on one lane):
# every list entry costs the separation (3 differences), r^2 (3 multiplies
# and 2 additions, each rounded on its own, so that every kernel and the
# oracle decide a pair at the cutoff alike) and the cutoff compare; every
# pair inside the cutoff costs 1/r and r
# (estimate, one third-order correction, one multiply: 7) and, per
# exponential 2^t, its argument (1), reduction (3), degree-10 polynomial (10,
# the lowest degree within a few units in the last place) and scaling (1);
# the force pass takes two exponentials and assembles (F'_i + F'_j) rho' + V'
# and the three force components (6), the density pass takes one exponential
# and one accumulation.
OPS_ENTRY = 9
OPS_FORCE_PAIR = 7 + 2 * 15 + 6
OPS_DENSITY_PAIR = 7 + 15 + 1
# the step's force kernel also takes, per atom, two half kicks (6), the drift
# (3) and the displacement test against the list's reference positions (6)
OPS_STEP_ATOM = 15


def force_pass_bytes(n_atoms, mean_list):
    """Algorithmic HBM bytes of one force pass with the fused half kick:
    per atom x,y,z (24) + F' (8) + count (4) + list (4 per entry) + force
    out (24) + velocity in/out (48); neighbour records counted once."""
    return n_atoms * (108.0 + 4.0 * mean_list)


def step_force_bytes(n_atoms, mean_list):
    """The force kernel as the step runs it (this step's second half kick,
    the next step's first half kick and drift fused): the force pass's bytes
    without the force out (it goes into the velocities only) plus the list's
    reference positions in (24) and the drifted positions out (24)."""
    return n_atoms * (132.0 + 4.0 * mean_list)


def density_pass_bytes(n_atoms, mean_list):
    """x,y,z (24) + count (4) + list (4 per entry) + rho, F, F' out (24)."""
    return n_atoms * (52.0 + 4.0 * mean_list)


def kernel_source_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def read_counters():
    """HBM bytes per force-pass launch from the committed rocprofv3 counter
    summary, or None if it is missing or was taken from other kernel sources."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def list_stats(S, rc):
    """Entries of the neighbour list and pairs inside the cutoff, counted on
    the device from the list the passes use (measurement only)."""
    import torch
    counts, ids = S.neighbors()
    pos, _ = S.get_state()
    L = float(S.box_len[0])
    entries = int(counts.sum())
    pairs = 0
    for a in range(0, ids.shape[0], 1 << 19):
        blk = ids[a:a + (1 << 19)].long()
        ok = blk >= 0
        d = pos[blk.clamp(min=0)] - pos[a:a + blk.shape[0], None, :]
        d -= L * torch.round(d / L)
        r2 = (d * d).sum(-1)
        pairs += int(((r2 < rc * rc) & ok).sum())
    return entries, pairs


def log(msg):
    """Progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def median_pass(S, which, reps, n=5):
    return float(sorted(S.time_pass(which, reps) for _ in range(n))[n // 2])


def timed_steps(S, steps, warmup):
    import torch
    S.step(warmup)
    torch.cuda.synchronize()
    _, b0, _ = S.status()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    S.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags, b1, _ = S.status()
    if flags:
        raise RuntimeError(f"device status flags {flags} after the timed steps")
    return t1 - t0, ev0.elapsed_time(ev1) / 1e3, b1 - b0


def copy_gbs(nbytes=1 << 31, reps=5):
    """HBM bandwidth of a plain device-to-device copy (bytes read plus
    written per second), the practical ceiling beside the nominal 8 TB/s."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / 1e3 / reps
    del src, dst
    return 2 * nbytes / t / 1e9


def bench_main(steps, warmup, reps):
    import torch
    from paper_1212_6332_amd import md, workloads as W

    wl = W.fcc4m()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.autotune()                  # tiled or per-atom passes and the tile shape, by timing
    dims = int(S.get_option(md.MD_OPT_TILE_DIMS))
    tuned = {"tiled": int(S.get_option(md.MD_OPT_TILED)),
             "tile_shape": int(S.get_option(md.MD_OPT_TILE_SHAPE)),
             "tile_shapes": int(S.get_option(md.MD_OPT_TILE_SHAPES)),
             "tile_cells": [dims & 255, (dims >> 8) & 255, dims >> 16],
             "graph_steps": int(S.get_option(md.MD_OPT_GRAPH_STEPS))}
    S.forces(energy=False)
    entries, pairs = list_stats(S, wl.pot.rc)
    n = wl.n_atoms
    mean_list = entries / n
    wall, gpu_s, rebuilds = timed_steps(S, steps, warmup)
    # four more windows of the same length (the headline stays the first)
    windows = [wall / steps * 1e3] + [timed_steps(S, steps, 0)[0] / steps * 1e3 for _ in range(4)]
    # each pass: the median of 5 timings, each the mean of `reps` launches
    # bracketed by HIP events on the library's stream
    ms = {name: median_pass(S, p, reps) for name, p in (
        ("force_step", md.MD_PASS_FORCE_STEP), ("force", md.MD_PASS_FORCE),
        ("density", md.MD_PASS_DENSITY), ("kick_drift", md.MD_PASS_KICK_DRIFT),
        ("build", md.MD_PASS_BUILD))}
    f_ops = OPS_ENTRY * entries + OPS_FORCE_PAIR * pairs + OPS_STEP_ATOM * n
    d_ops = OPS_ENTRY * entries + OPS_DENSITY_PAIR * pairs
    t_f = ms["force_step"]
    achieved = f_ops / (t_f * 1e-3) / 1e12
    fbytes = step_force_bytes(n, mean_list)
    traffic = read_counters()
    res = {
        "value": n * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "gpu_ms_per_step": gpu_s / steps * 1e3,
        "ms_per_step_5_windows": windows,
        "ms_per_step_median_of_5": sorted(windows)[2],
        "rebuilds": int(rebuilds),
        "mean_list_len": mean_list,
        "pairs_per_atom": pairs / n,
        "pass_ms": ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "T FP64 lane-ops/s", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": traffic,
                     "kernel": f"{FORCE_KERNEL}: the step's force kernel (half kick, next "
                               f"half kick and drift fused)",
                     "ops_per_launch": f_ops, "ms_per_launch": t_f,
                     "ms_per_launch_from": "median of 5 x mean of %d launches" % reps,
                     "hbm": {"algorithmic_bytes_per_launch": fbytes,
                             "algorithmic_gbs": fbytes / (t_f * 1e-3) / 1e9,
                             "measured_gbs": (traffic / (t_f * 1e-3) / 1e9
                                              if traffic else None),
                             "peak_gbs": HBM_PEAK_GBS,
                             "copy_kernel_gbs": copy_gbs()},
                     "density_pass": {"ops_per_launch": d_ops,
                                      "achieved": d_ops / (ms["density"] * 1e-3) / 1e12,
                                      "algorithmic_gbs": density_pass_bytes(n, mean_list)
                                      / (ms["density"] * 1e-3) / 1e9}},
        "n_atoms": n,
        "tuned": tuned,
    }
    S.close()
    return res


# Spline potentials (one species): per pair inside the cutoff, r and 1/r (7),
# the interval and local coordinate (5), then for the density one cubic (3)
# and the accumulation (1); for the force V, V' and rho' on the interleaved
# interval (9), the coefficient (2) and the three force components (3).
OPS_SPLINE_DENSITY_PAIR = 7 + 5 + 3 + 1
OPS_SPLINE_FORCE_PAIR = 7 + 5 + 9 + 2 + 3


def multibox_pair_stats(S, wl, rc):
    """Entries of the multi-box neighbour list and pairs inside the cutoff
    (measurement only), each box with its own edge."""
    import numpy as np
    import torch
    counts, ids = S.neighbors()
    pos, _ = S.get_state()
    nb = np.diff(wl.box_offset)
    Lat = torch.repeat_interleave(torch.tensor(wl.box_len[:, 0], device=pos.device),
                                  torch.tensor(nb, device=pos.device))
    blk = ids.long()
    ok = blk >= 0
    d = pos[blk.clamp(min=0)] - pos[:, None, :]
    L = Lat[:, None, None]
    d -= L * torch.round(d / L)
    pairs = int((((d * d).sum(-1) < rc * rc) & ok).sum())
    return int(counts.sum()), pairs


def bench_batched(steps=200, warmup=5):
    from paper_1212_6332_amd import md, workloads as W

    wl = W.batch2048()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.forces(energy=False)
    entries, pairs = multibox_pair_stats(S, wl, wl.pot.rc)
    S.set_state(wl.pos, wl.vel)
    wall_d, _, _ = timed_steps(S, steps, warmup)     # default shape: one box per 256-thread workgroup
    S.set_state(wl.pos, wl.vel)
    S.autotune()                  # block shape picked by timing (md_autotune)
    shape = {k: int(S.get_option(o)) for k, o in (("workgroup", md.MD_OPT_BATCH_BLOCK),
                                                  ("pack_atoms", md.MD_OPT_BATCH_PACK),
                                                  ("cell_order", md.MD_OPT_BATCH_ORDER))}
    wall, gpu_s, _ = timed_steps(S, steps, warmup)
    S.close()
    # the same boxes through the merged-box kernels (the paper's scheme of Section 4.4)
    M = md.System.from_workload(wl)
    M.set_option(md.MD_OPT_BATCHED, 0)
    M.set_state(wl.pos, wl.vel)
    wall_m, _, _ = timed_steps(M, steps, warmup)
    M.close()
    ops = 2 * OPS_ENTRY * entries + (OPS_SPLINE_DENSITY_PAIR + OPS_SPLINE_FORCE_PAIR) * pairs
    ms = gpu_s / steps * 1e3
    achieved = ops / (ms * 1e-3) / 1e12
    return {"workload": "batch2048: 2,048 FCC boxes n^3, n in {3..8}, 5,000-knot splines",
            "n_boxes": wl.n_boxes, "n_atoms": wl.n_atoms, "steps": steps,
            "box_steps_per_s": wl.n_boxes * steps / wall,
            "atom_steps_per_s": wl.n_atoms * steps / wall,
            "ms_per_step": wall / steps * 1e3, "shape": shape, "shape_from": "md_autotune",
            "default_shape_box_steps_per_s": wl.n_boxes * steps / wall_d,
            "merged_kernels_box_steps_per_s": wl.n_boxes * steps / wall_m,
            "roofline": {"bound": "alu", "kernel": "k_batched<3, %d>" % shape["workgroup"],
                         "achieved": achieved, "peak": VALU_PEAK_TOPS,
                         "unit": "T FP64 lane-ops/s", "frac": achieved / VALU_PEAK_TOPS,
                         "ops_per_step": ops, "ms_per_step": ms, "entries": entries,
                         "pairs": pairs,
                         "binding": "vector L1 gathers of the spline intervals (one per pair "
                                    "and table, each lane its own line): about 0.8 L1 "
                                    "accesses per CU per cycle in the rocprofv3 counters"}}


def bench_adjoint(evals=50, steps=100):
    import torch
    from paper_1212_6332_amd import md, workloads as W
    from paper_1212_6332_amd.autograd import GraphedLoss, force_matching_loss

    wl = W.adjoint64()
    T = md.System.from_workload(wl, wl.extra["target_pot"])
    T.set_state(wl.pos)
    ft, _, et = T.forces()
    T.close()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos)
    th = [torch.tensor(t, device="cuda", requires_grad=True) for t in wl.pot.tables]
    w = wl.extra["w"]

    def one():
        for t in th:
            t.grad = None
        loss = force_matching_loss(S, th[0], th[1], th[2], ft, et, w)
        loss.backward()

    for _ in range(3):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(evals):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / evals
    # the same evaluation captured once and replayed from a HIP graph
    G = GraphedLoss(S, th, lambda: force_matching_loss(S, th[0], th[1], th[2], ft, et, w))
    for _ in range(3):
        G.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4 * evals):
        G.replay()
    torch.cuda.synchronize()
    dtg = (time.perf_counter() - t0) / (4 * evals)
    # the plain step on the same boxes and potential, for comparison
    S.set_state(wl.pos, None)
    wall, _, _ = timed_steps(S, steps, 5)
    S.close()
    return {"workload": "adjoint64: 64 BCC 5^3 boxes (16,000 atoms), 3x64 B-spline coefficients",
            "grad_evals_per_s": 1.0 / dt, "ms_per_grad_eval": dt * 1e3,
            "graph_grad_evals_per_s": 1.0 / dtg, "graph_ms_per_grad_eval": dtg * 1e3,
            "atom_grads_per_s": wl.n_atoms / dt,
            "plain_step_atom_steps_per_s": wl.n_atoms * steps / wall}


def bench_pressure(steps=100, warmup=10, reps=10):
    """The 4M-atom box with the pressure of eq. (6): force pass with energies
    and the pair virial (plus the per-box reductions) against the plain force
    pass, and steps with the Berendsen barostat of eq. (5) switched on."""
    from paper_1212_6332_amd import md, workloads as W

    wl = W.fcc4m()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    p0, _ = S.pressure()
    ms_plain = median_pass(S, md.MD_PASS_FORCE, reps)
    ms_virial = median_pass(S, md.MD_PASS_PRESSURE, reps)
    S.set_barostat(0.0, 1000.0, 1.0)
    wall, _, reb = timed_steps(S, steps, warmup)
    L = float(S.box()[0])
    p1, _ = S.pressure()
    S.close()
    return {"workload": "fcc4m with the Berendsen barostat (P0 = 0, tau = 1000 fs, beta = 1 A^3/eV)",
            "force_pass_ms": ms_plain, "force_pass_with_virial_ms": ms_virial,
            "barostat_atom_steps_per_s": wl.n_atoms * steps / wall,
            "barostat_ms_per_step": wall / steps * 1e3, "rebuilds": int(reb),
            "pressure_start_eV_A3": float(p0[0]), "pressure_end_eV_A3": float(p1[0]),
            "box_start_A": float(wl.box_len[0, 0]), "box_end_A": L}


def bench_thermostat(steps=100, warmup=10, reps=10):
    """The 4M-atom box with the electron-gas friction of eq. (4) in every
    half kick: steps with the thermostat on, and the fused force pass with and
    without the friction."""
    from paper_1212_6332_amd import md, workloads as W

    wl = W.fcc4m()
    te, tau = 600.0, 100.0
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(1)
    ms_plain = median_pass(S, md.MD_PASS_FORCE_STEP, reps)
    S.set_thermostat(te, tau)
    ms_fric = median_pass(S, md.MD_PASS_FORCE_STEP, reps)
    t_of = lambda: 2 * float(S.kinetic()[0]) / (3 * wl.n_atoms * W.KB_EV)
    t0 = t_of()
    wall, _, reb = timed_steps(S, steps, warmup)
    t1 = t_of()
    S.close()
    return {"workload": f"fcc4m with the electron-gas thermostat (T_e = {te:g} K, "
                        f"tau_T = {tau:g} fs)",
            "thermostat_atom_steps_per_s": wl.n_atoms * steps / wall,
            "thermostat_ms_per_step": wall / steps * 1e3, "rebuilds": int(reb),
            "force_step_pass_ms": ms_plain, "force_step_pass_with_friction_ms": ms_fric,
            "kinetic_T_start_K": t0, "kinetic_T_end_K": t1}


def bench_frozen(steps=100, warmup=10, reps=10):
    """The 4M-atom box with a frozen slab (the atoms in the tenth of the box
    with the smallest x keep zero velocity and their positions): steps, and the
    fused force pass with and without the atom states."""
    import numpy as np
    import torch
    from paper_1212_6332_amd import md, workloads as W

    wl = W.fcc4m()
    L = float(wl.box_len[0, 0])
    x = wl.pos[:, 0] - L * np.floor(wl.pos[:, 0] / L)
    frozen = x < 0.1 * L
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.step(1)
    ms_plain = median_pass(S, md.MD_PASS_FORCE_STEP, reps)
    S.set_frozen(frozen.astype(np.uint8))
    ms_frozen = median_pass(S, md.MD_PASS_FORCE_STEP, reps)
    idx = torch.as_tensor(np.nonzero(frozen)[0], device="cuda")
    p0 = S.get_state()[0][idx].clone()
    wall, _, reb = timed_steps(S, steps, warmup)
    d = S.get_state()[0][idx] - p0
    # a frozen atom keeps its position up to the periodic wrap of the list builds
    # (one rounding of the added box edge)
    still = bool((d - L * torch.round(d / L)).abs().max() <= 1e-12 * L)
    S.close()
    return {"workload": "fcc4m with a frozen slab (x < L / 10, "
                        f"{int(frozen.sum()):,} of {wl.n_atoms:,} atoms)",
            "frozen_atom_steps_per_s": wl.n_atoms * steps / wall,
            "frozen_ms_per_step": wall / steps * 1e3, "rebuilds": int(reb),
            "force_step_pass_ms": ms_plain, "force_step_pass_with_frozen_ms": ms_frozen,
            "frozen_atoms_in_place": still}


def bench_alloy(steps=100, warmup=10, reps=10):
    """The 4M-atom binary FCC alloy (per-type-pair spline tables, two masses):
    steps, and the force, density and list-build passes."""
    from paper_1212_6332_amd import md, workloads as W

    wl = W.alloy()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.autotune()                  # tiled or per-atom passes and the tile shape, by timing
    shape = int(S.get_option(md.MD_OPT_TILE_SHAPE))
    wall, _, reb = timed_steps(S, steps, warmup)
    ms = {"force_step": median_pass(S, md.MD_PASS_FORCE_STEP, reps),
          "density": median_pass(S, md.MD_PASS_DENSITY, reps),
          "build": median_pass(S, md.MD_PASS_BUILD, reps)}
    S.close()
    return {"workload": "alloy: binary FCC 100^3 cells (4,000,000 atoms, 30 % species 1), "
                        "per-type-pair 5,000-knot splines, rc 5.3 A, skin 0.3 A, 300 K",
            "atom_steps_per_s": wl.n_atoms * steps / wall, "ms_per_step": wall / steps * 1e3,
            "rebuilds": int(reb), "steps": steps, "pass_ms": ms,
            "tile_shape": shape, "tile_shape_from": "md_autotune"}


def bench_32m(steps=50, warmup=5):
    """One 32,000,000-atom box (FCC 200^3 cells of the same SMTB material)
    on the one GPU: the headline step at eight times the atoms."""
    from paper_1212_6332_amd import md, workloads as W

    wl = W.fcc4m(ncell=200)
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    wall, _, reb = timed_steps(S, steps, warmup)
    S.close()
    return {"workload": "fcc32m: FCC 200^3 cells (32,000,000 atoms), the fcc4m material",
            "atom_steps_per_s": wl.n_atoms * steps / wall, "ms_per_step": wall / steps * 1e3,
            "rebuilds": int(reb), "steps": steps}


def bench_c2(steps=1000, warmup=20):
    from paper_1212_6332_amd import md, workloads as W

    wl = W.bcc128k()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.autotune()                  # tiled or per-atom passes, picked by timing
    tiled = S.get_option(md.MD_OPT_TILED)
    wall, _, reb = timed_steps(S, steps, warmup)
    S.close()
    return {"workload": "bcc128k: BCC 40^3 (128,000 atoms), 5,000-knot splines",
            "atom_steps_per_s": wl.n_atoms * steps / wall, "ms_per_step": wall / steps * 1e3,
            "rebuilds": int(reb), "steps": steps,
            "passes": ("tiled" if tiled else "per-atom") + " (md_autotune)"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_vv_rate(O, wl, steps):
    """Seconds of setup (list build + first forces) and atom-steps/s of the
    steps after it, for the oracle's velocity Verlet on one box."""
    L = float(wl.box_len[0, 0])
    pot = O.Pot(wl.pot)
    t = time.perf_counter()
    O.vv(wl.pos, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 0, energies=False)
    setup = time.perf_counter() - t
    t = time.perf_counter()
    _, _, _, _, reb = O.vv(wl.pos, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, steps,
                           energies=False)
    run = time.perf_counter() - t
    return setup, wl.n_atoms * steps / max(run - setup, 1e-9), run + setup, int(reb)


def cpu_baseline(steps=10, ncell_1t=50, steps_1t=3):
    """The CPU oracle, built -O3 -march=native on this host, on the headline
    workload itself (the 4,000,000-atom FCC SMTB box, 10 velocity-Verlet
    steps, list build and first forces timed separately and excluded) with
    every OpenMP thread, and on a 500,000-atom box of the same material
    (3 steps) with one thread."""
    import tempfile

    import oracle as O
    from paper_1212_6332_amd import workloads as W

    O.use_tuned(tempfile.mkdtemp(prefix="oracle_native_"))
    threads = O.threads()
    wl = W.fcc4m()
    setup, rate, secs, reb = _oracle_vv_rate(O, wl, steps)
    O.set_threads(1)
    w1 = W.fcc4m(ncell=ncell_1t)
    setup1, rate1, secs1, _ = _oracle_vv_rate(O, w1, steps_1t)
    O.set_threads(threads)
    # the other step workloads: bcc128k (100 steps after the setup) and
    # batch2048 (10 steps per box, each box's first list build included)
    wc2 = W.bcc128k()
    setup2, rate2, secs2, _ = _oracle_vv_rate(O, wc2, 100)
    wc4 = W.batch2048()
    pot4 = O.Pot(wc4.pot)
    t = time.perf_counter()
    for b, sl, L in O.boxes(wc4):
        O.vv(wc4.pos[sl], wc4.vel[sl], L, pot4, wc4.mass, wc4.dt, wc4.skin, 10, energies=False)
    secs4 = time.perf_counter() - t
    return {"value": rate, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the 4,000,000-atom FCC SMTB box, {steps} velocity-Verlet steps "
                      f"({reb} list rebuilds inside them); setup (list build + first forces, "
                      f"{setup:.1f} s) excluded; oracle built -O3 -march=native "
                      f"-ffp-contract=off -fopenmp",
            "host_cpu": _cpu_model(), "seconds": secs,
            "one_thread": {"value": rate1, "unit": "atom-steps/s", "cores": 1,
                           "sample": f"FCC SMTB {ncell_1t}^3 cells ({w1.n_atoms} atoms, the "
                                     f"same material), {steps_1t} steps; setup "
                                     f"({setup1:.1f} s) excluded",
                           "seconds": secs1},
            "bcc128k": {"value": rate2, "unit": "atom-steps/s", "cores": threads,
                        "sample": f"bcc128k, 100 steps; setup ({setup2:.1f} s) excluded",
                        "seconds": secs2},
            "batch2048": {"value": wc4.n_boxes * 10 / secs4, "unit": "box-steps/s",
                          "atom_steps_per_s": wc4.n_atoms * 10 / secs4, "cores": threads,
                          "sample": "batch2048, 10 steps of every box, each box's first "
                                    "list build included", "seconds": secs4}}


def pmc_probe(reps, workload="fcc4m"):
    """Short run for hardware-counter collection: force (plain and as run in
    the step), density and list-build passes of the 4M-atom workload (or of
    the 4M-atom alloy), or 100 steps of the persistent multi-box stepper on
    batch2048 in its default shape; then one plain 2 GiB device copy used to
    scale the counters."""
    import torch
    from paper_1212_6332_amd import md, workloads as W

    if workload == "batch2048":
        wl = W.batch2048()
        S = md.System.from_workload(wl)
        S.set_state(wl.pos, wl.vel)
        S.step(100)
        torch.cuda.synchronize()
        S.close()
        src = torch.ones(2 ** 28, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}))
        return
    wl = W.alloy() if workload == "alloy" else W.fcc4m()
    S = md.System.from_workload(wl)
    S.set_state(wl.pos, wl.vel)
    S.forces(energy=False)
    counts, _ = S.neighbors(1)
    print(json.dumps({"mean_list_len": float(counts.double().mean()), "n_atoms": wl.n_atoms,
                      "force_bytes": force_pass_bytes(wl.n_atoms, float(counts.double().mean()))}))
    S.time_pass(md.MD_PASS_FORCE, reps)
    S.time_pass(md.MD_PASS_FORCE_STEP, reps)
    S.time_pass(md.MD_PASS_DENSITY, reps)
    S.time_pass(md.MD_PASS_BUILD, reps)
    torch.cuda.synchronize()
    src = torch.ones(2 ** 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8}))
    S.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--reps", type=int, default=20, help="launches per timed pass")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true", help="counter-collection run only")
    ap.add_argument("--pmc-workload", default="fcc4m", choices=["fcc4m", "alloy", "batch2048"],
                    help="workload of the counter-collection run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the whole box fits in one MI355X's HBM); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.pmc_probe:
        pmc_probe(args.reps, args.pmc_workload)
        return
    t0 = time.perf_counter()
    r = bench_main(args.steps, args.warmup, args.reps)
    log(f"headline workload done ({time.perf_counter() - t0:.1f} s)")
    out = {
        "metric": METRIC, "value": r["value"], "unit": "atom-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fcc4m: FCC 100^3 cells (4,000,000 atoms), second-moment "
                               "tight binding (Cu), rc 5.85 A, skin 0.3 A, 300 K, dt 1 fs",
                   "n_atoms": r["n_atoms"], "rebuilds_in_timed_steps": r["rebuilds"],
                   "mean_list_len": r["mean_list_len"], "pairs_per_atom": r["pairs_per_atom"],
                   "gpu_ms_per_step": r["gpu_ms_per_step"],
                   "ms_per_step_5_windows": r["ms_per_step_5_windows"],
                   "ms_per_step_median_of_5": r["ms_per_step_median_of_5"],
                   "pass_ms": r["pass_ms"], "tuned": r["tuned"]},
        "roofline": r["roofline"],
    }
    if not args.no_extras:
        for key, leg in (("batched", bench_batched), ("adjoint", bench_adjoint),
                         ("bcc128k", bench_c2), ("pressure", bench_pressure),
                         ("thermostat", bench_thermostat), ("frozen", bench_frozen),
                         ("alloy", bench_alloy),
                         ("fcc32m", bench_32m)):
            out[key] = leg()
            log(f"{key} done ({time.perf_counter() - t0:.1f} s)")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        log(f"cpu baseline done ({time.perf_counter() - t0:.1f} s)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
