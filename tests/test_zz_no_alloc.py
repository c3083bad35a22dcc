"""md_forces_static (every device buffer in the library's static array)
against md_forces of an ordinary context, through the C ABI: two calls in a
row, the second with a smaller system, each to the parity bar (here bitwise:
the same kernels run on the same inputs)."""
import numpy as np
import pytest
import torch

from paper_1212_6332_amd import md, workloads as W

pytestmark = pytest.mark.gpu


def reference(wl):
    S = md.System.from_workload(wl)
    S.set_state(wl.pos)
    f, e, eb = (t.cpu().numpy() for t in S.forces())
    assert S.status()[0] == 0
    S.close()
    return f, e, eb


def static(wl):
    f, e, eb = md.forces_static(wl.box_offset, wl.box_len, wl.pot, wl.mass, wl.pos, wl.dt,
                                wl.skin)
    return f.cpu().numpy(), e.cpu().numpy(), eb.cpu().numpy()


def check(wl):
    a, b = static(wl), reference(wl)
    for u, v in zip(a, b):
        assert np.abs(u - v).max() <= 1e-11 * np.abs(v).max()
        assert np.array_equal(u, v)


def test_static_twice_second_smaller():
    big = W.fcc4m(ncell=20)          # 32,000 atoms, tiled (halo mode A)
    small = W.fcc4m(ncell=6)         # 864 atoms, one tile
    assert md.System.workload_workspace_size(big) <= md.static_bytes()
    check(big)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    check(small)
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0 or abs(free1 - free0) < (8 << 20)


def test_static_several_boxes_and_spline():
    wl = W.batch2048(n_boxes=20)
    check(wl)
    check(W.bcc128k(ncell=8))


def test_static_refuses_too_large():
    wl = W.fcc4m(ncell=60)           # 864,000 atoms: buffers beyond 64 MiB
    assert md.System.workload_workspace_size(wl) > md.static_bytes()
    with pytest.raises(md.MDError) as e:
        md.forces_static(wl.box_offset, wl.box_len, wl.pot, wl.mass, wl.pos, wl.dt, wl.skin)
    assert e.value.code == md.MD_ERR_SCRATCH
