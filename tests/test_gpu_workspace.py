"""Contexts in a caller's workspace (md_workspace_size, md_create_in): the
library allocates no device memory for them, and they compute exactly what
a context with its own memory computes."""
import numpy as np
import pytest
import torch

from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "smtb108k_tiled": lambda: W.fcc4m(ncell=30),
    "spline_boxes": lambda: W.batch2048(n_boxes=12),       # persistent stepper buffers too
    "alloy6912": lambda: W.alloy(ncell=12),                # species arrays and tables
}


def trajectory(S, wl, nsteps):
    S.set_state(wl.pos, wl.vel)
    S.step(nsteps)
    p, v = S.get_state()
    f, e, eb = S.forces()
    out = (p.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy(), eb.cpu().numpy(), S.status())
    S.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_workspace_context_allocates_nothing_and_matches(name):
    wl = CASES[name]()
    size = md.System.workload_workspace_size(wl)
    assert size > 0
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    S = md.System.from_workload(wl, workspace=ws)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # the context's buffers all live in ws (the runtime may take a little for its stream)
    assert free0 - free1 < min(16 << 20, size // 4), (free0 - free1, size)
    a = trajectory(S, wl, 25)
    b = trajectory(md.System.from_workload(wl), wl, 25)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    assert a[4] == b[4] and a[4][0] == 0


def test_workspace_too_small_and_capacity_growth():
    wl = W.fcc4m(ncell=11)
    size = md.System.workload_workspace_size(wl)
    small = torch.empty(size - 4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(md.MDError):
        md.System.from_workload(wl, workspace=small)
    exact = torch.empty(size, dtype=torch.uint8, device="cuda")
    S = md.System.from_workload(wl, workspace=exact)
    S.set_state(wl.pos, wl.vel)
    with pytest.raises(md.MDError):          # no room left for a bigger list
        S.set_max_neighbors(200)
    f, e, eb = S.forces()                    # the context is as it was
    assert S.status()[0] == 0 and float(f.abs().max()) > 0.0
    S.close()
    mn = md.System.from_workload(wl)
    list_bytes = 4 * wl.n_atoms * 200 + 4096
    mn.close()
    roomy = torch.empty(size + list_bytes, dtype=torch.uint8, device="cuda")
    S = md.System.from_workload(wl, workspace=roomy)
    S.set_max_neighbors(200)
    a = trajectory(S, wl, 15)
    ref = md.System.from_workload(wl)
    ref.set_max_neighbors(200)
    b = trajectory(ref, wl, 15)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)


def test_size_query_allocates_nothing():
    """md_workspace_size only counts: it answers for a system whose workspace
    exceeds the whole device memory, and the free memory does not move."""
    wl = W.fcc4m(ncell=72)                   # 1,492,992 atoms
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    size = md.System.workspace_size(wl.box_offset, wl.box_len, wl.pot, wl.mass, wl.dt,
                                    wl.skin, max_neighbors=65528)
    free1, _ = torch.cuda.mem_get_info()
    assert size > total
    assert free1 == free0
    # and the count is the one md_create_in consumes (the smaller system above
    # needs exactly its measured size: see test_workspace_too_small_...)
    assert size >= 4 * 65528 * wl.n_atoms
