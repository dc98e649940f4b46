"""The allocation-free reduction against hdg_reduce: two calls in a row on one
GPU (the second on a smaller mesh, so the shared scratch array holds the first
call's larger partial set when it starts), and a non-finite entry."""
import sys

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _compare(torch, m, r):
    ref = hdg.hdg_reduce(m, r, allow_nonfinite=True)
    out = torch.full((13,), -7.0, dtype=torch.float64, device="cuda")
    hdg.hdg_reduce_noalloc(m, r, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    # the same kernels and workgroup count: bitwise the same results
    assert np.array_equal(o[0:4], ref["sum"], equal_nan=True)
    assert np.array_equal(np.sqrt(o[4:8]), ref["l2"], equal_nan=True)
    assert np.array_equal(o[8:12], ref["max"], equal_nan=True)
    assert o[12] == (0.0 if ref["finite"] else 1.0)
    return o


def test_noalloc_reduce_equals_reduce(torch_cuda):
    torch = torch_cuda
    ctx = hdg.hdg_init(0)
    rng = np.random.default_rng(3)
    big = W.periodic_box(6, Pg=2, curve_amp=0.3)
    small = W.periodic_box(3, Pg=1)
    mb = hdg.hdg_mesh_create(ctx, big, 4, W.bernoulli_mask(big.n_elem, 0.5, 1), hdg.make_params())
    ms = hdg.hdg_mesh_create(ctx, small, 2, W.bernoulli_mask(small.n_elem, 0.5, 2), hdg.make_params())
    rb = torch.from_numpy(rng.uniform(-1, 1, mb.state_shape)).cuda()
    rs = torch.from_numpy(rng.uniform(-1, 1, ms.state_shape)).cuda()
    _say(f"reduce_noalloc: {big.n_elem} elements P=4, then {small.n_elem} elements P=2")
    o1 = _compare(torch, mb, rb)
    o2 = _compare(torch, ms, rs)
    assert o1[12] == 0.0 and o2[12] == 0.0
    # a mesh of several orders (the mixed-order reduction kernel)
    mesh = W.periodic_box(3, Pg=1, curve_amp=0.25)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, 4)
    mm = hdg.hdg_mesh_create(ctx, mesh, W.mixed_orders(flag, 4), flag, hdg.make_params())
    rm = torch.from_numpy(rng.uniform(-1, 1, mm.state_shape)).cuda()
    _compare(torch, mm, rm)
    # a non-finite entry sets the flag (hdg_reduce reports HDG_ENONFINITE)
    rs[5] = float("nan")
    o3 = _compare(torch, ms, rs)
    assert o3[12] == 1.0
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_reduce_noalloc(ms, rs, torch.empty(4, dtype=torch.float64, device="cuda"))
    assert ex.value.status == hdg.HDG_EINVAL
