"""The C ABI from a C++ caller with no Python and no torch
(tests/c_abi/forces_from_c.cpp, compiled by build()): hipMalloc'd buffers,
md_create, md_set_state, md_build_neighbors, md_density, md_forces, ten
md_step steps, md_get_state, md_status, md_destroy.  Forces and the box energy
within 1e-11 of the oracle, the positions after ten steps within 1e-10
Angstrom of the oracle's velocity Verlet."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1212_6332_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_abi", "forces_from_c")


def test_c_caller_matches_oracle(tmp_path):
    assert os.path.exists(BIN), "the C caller is compiled by __graft_entry__.build()"
    wl = W.fs256(ncell=5)
    L = float(wl.box_len[0, 0])
    n = wl.n_atoms
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as fh:
        np.array([n], dtype=np.int64).tofile(fh)
        np.array([L, wl.mass, wl.dt, wl.skin, wl.pot.rc], dtype=np.float64).tofile(fh)
        np.asarray(wl.pot.params, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(wl.pos, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(wl.vel, dtype=np.float64).tofile(fh)
    r = subprocess.run([BIN, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr + r.stdout
    raw = np.fromfile(dst, dtype=np.uint8)
    f = raw[:24 * n].view(np.float64).reshape(n, 3)
    e_box = raw[24 * n:24 * n + 8].view(np.float64)[0]
    after = raw[24 * n + 8:48 * n + 8].view(np.float64).reshape(n, 3)
    flags = raw[48 * n + 8:48 * n + 12].view(np.uint32)[0]
    assert flags == 0
    pot = O.Pot(wl.pot)
    ref = O.forces(O.wrap(wl.pos, L), L, pot)
    assert np.abs(f - ref["f"]).max() <= 1e-11 * np.abs(ref["f"]).max()
    assert abs(e_box - ref["E"]) <= 1e-11 * abs(ref["E"])
    x, *_ = O.vv(wl.pos, wl.vel, L, pot, wl.mass, wl.dt, wl.skin, 10, energies=False)
    d = after - x
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10
