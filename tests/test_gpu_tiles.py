"""Launch shapes and the autotuner: every (workgroup size, persistent) pair a
kernel supports gives bitwise-identical results, since it changes only which
workgroup takes which tile of elements."""
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


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    return hdg.hdg_init(0)


def _shapes(N):
    out = []
    for B in (128, 256, 384, 512):
        lanes = N ** 3 if N ** 3 < 64 else (N ** 3 + 63) // 64 * 64
        if lanes <= B and (B != 384 or N == 7):       # 384-lane kernels exist for order 7 only
            out += [(B, True), (B, False)]
    return out


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 7])
def test_launch_shapes_bitwise(torch_cuda, ctx, P):
    torch = torch_cuda
    m0, _ = W.reorient(W.periodic_box(4, Pg=2, curve_amp=0.25), seed=P)
    flag = W.bernoulli_mask(m0.n_elem, 0.5, P)
    prm = hdg.make_params(c0sq=25.0, nu=5e-3, les_model=1 + P % 2, C_les=0.1)
    m = hdg.hdg_mesh_create(ctx, m0, P, flag, prm)
    N = P + 1
    q0 = W.taylor_green_state(hdg.hdg_mesh_node_coords(m), 0.05, seed=P)
    _say(f"launch shapes, curved box 4^3 P={P}: {_shapes(N)}")
    ref = {}
    for prec in (hdg.HDG_F64, hdg.HDG_F32):
        for B, pers in _shapes(N):
            for k in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL):
                hdg.hdg_mesh_set_launch(m, k, prec, N, B, pers)
            q = torch.from_numpy(q0).cuda()
            r = torch.empty(q.shape, dtype=torch.float32 if prec == hdg.HDG_F32 else torch.float64, device="cuda")
            hdg.hdg_residual(m, q, r, prec=prec)
            dq = torch.empty_like(q)
            hdg.hdg_rk3_steps(m, q, dq, 1e-4, 2, prec=prec)
            torch.cuda.synchronize()
            out = (r.cpu().numpy(), q.cpu().numpy())
            if prec not in ref:
                ref[prec] = out
            else:
                assert np.array_equal(out[0], ref[prec][0]), f"residual differs for block {B} persistent {pers}"
                assert np.array_equal(out[1], ref[prec][1]), f"RK state differs for block {B} persistent {pers}"


def test_autotune_picks_a_supported_shape(torch_cuda, ctx):
    torch = torch_cuda
    w = W.tgv_box_small()
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q0 = W.taylor_green_state(hdg.hdg_mesh_node_coords(m), 0.01, seed=0)
    q = torch.from_numpy(q0).cuda()
    r_before = torch.empty_like(q)
    hdg.hdg_residual(m, q, r_before)
    _say("autotune on the small TGV box")
    hdg.hdg_mesh_autotune(m, q, reps=2)
    N = w.P + 1
    for prec in (hdg.HDG_F64, hdg.HDG_F32):
        for k in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL):
            c = hdg.hdg_mesh_get_launch(m, k, prec, N)
            _say(f"prec {prec} kernel {k}: {c}")
            assert (c["block"], c["persistent"]) in _shapes(N)
            assert c["us_per_launch"] > 0.0
    assert np.array_equal(q.cpu().numpy(), q0)        # the state is not modified
    r_after = torch.empty_like(q)
    hdg.hdg_residual(m, q, r_after)
    assert torch.equal(r_before, r_after)
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_set_launch(m, 0, hdg.HDG_F64, 8, 256, True)
    assert ex.value.status == hdg.HDG_EUNSUPPORTED


def test_rk_graph_replays_match_eager(torch_cuda, ctx):
    """Graph-captured RK steps, replayed several times with eager work and
    synchronisations in between, equal eager launches bitwise every time."""
    torch = torch_cuda
    w = W.tgv_box_small()
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q0 = W.taylor_green_state(hdg.hdg_mesh_node_coords(m), 0.01, seed=3)
    _say("RK graph replays vs eager on the small TGV box")
    for prec in (hdg.HDG_F64, hdg.HDG_F32):
        hdg.hdg_mesh_set_graphs(m, False)
        qe = torch.from_numpy(q0).cuda()
        dqe = torch.empty_like(qe)
        eager = []
        for _ in range(3):
            hdg.hdg_rk3_steps(m, qe, dqe, 1e-3, 4, prec=prec)
            eager.append(qe.cpu().numpy())
        hdg.hdg_mesh_set_graphs(m, True)
        qg = torch.from_numpy(q0).cuda()
        dqg = torch.empty_like(qg)
        for k in range(3):
            hdg.hdg_rk3_steps(m, qg, dqg, 1e-3, 4, prec=prec)      # two replays of the two-step graph
            torch.cuda.synchronize()
            scratch = torch.empty_like(qg)
            hdg.hdg_residual(m, qg, scratch)                       # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(qg.cpu().numpy(), eager[k]), f"replay {k} prec {prec}"
        # odd step count: graph replays plus one eager step
        qo = torch.from_numpy(q0).cuda()
        hdg.hdg_rk3_steps(m, qo, dqg, 1e-3, 5, prec=prec)
        hdg.hdg_mesh_set_graphs(m, False)
        qp = torch.from_numpy(q0).cuda()
        hdg.hdg_rk3_steps(m, qp, dqe, 1e-3, 5, prec=prec)
        assert torch.equal(qo, qp)
