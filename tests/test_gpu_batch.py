"""Batches of independent meshes: every member's result is bitwise the result
of the same mesh advanced on its own, whatever else is in the batch and when
members join or leave."""
import sys

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, workloads as W
from parity import TOL_F32, TOL_F64, flat_errors, flat_mass, increment_errors, oracle_mass

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


def _requests(k, seed):
    """k small periodic-box solves with seeded size, order, mask fraction and viscosity."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(rng.integers(3, 6))
        P = int(rng.integers(1, 8))
        frac = float(rng.uniform(0.2, 0.8))
        nu = float(10 ** rng.uniform(-4, -2))
        out.append(dict(n=n, P=P, frac=frac, nu=nu, seed=1000 * seed + i))
    return out


def _make(ctx, r):
    mesh = W.periodic_box(r["n"], Pg=1)
    flag = W.bernoulli_mask(mesh.n_elem, r["frac"], r["seed"])
    m = hdg.hdg_mesh_create(ctx, mesh, r["P"], flag,
                            hdg.make_params(c0sq=25.0, nu=r["nu"], les_model=1, C_les=0.1))
    q0 = W.taylor_green_state(hdg.hdg_mesh_node_coords(m), 0.01, seed=r["seed"])
    dt = 0.5 * W.cfl_dt(mesh, r["P"], q0, 25.0)
    return m, q0, dt


def _alone(torch, m, q0, dt, steps, prec):
    q = torch.from_numpy(q0).cuda()
    dq = torch.empty_like(q)
    hdg.hdg_rk3_steps(m, q, dq, dt, steps, prec=prec)
    torch.cuda.synchronize()
    return q.cpu().numpy()


@pytest.mark.parametrize("prec", [hdg.HDG_F64, hdg.HDG_F32])
@pytest.mark.parametrize("graphs", [True, False])
def test_batch_members_equal_alone(torch_cuda, ctx, prec, graphs):
    torch = torch_cuda
    reqs = _requests(6, seed=7 + prec)
    made = [_make(ctx, r) for r in reqs]
    _say(f"batch of {len(reqs)} boxes (n, P) = {[(r['n'], r['P']) for r in reqs]}, prec {prec}, graphs {graphs}")
    alone = [_alone(torch, m, q0, dt, 5, prec) for (m, q0, dt) in made]
    b = hdg.hdg_batch_create(ctx, 8)
    hdg.hdg_batch_set_graphs(b, graphs)
    qs = []
    for (m, q0, dt) in made:
        q = torch.from_numpy(q0).cuda()
        dq = torch.empty_like(q)
        hdg.hdg_batch_add(b, m, q, dq, dt)
        qs.append(q)
    info = hdg.hdg_batch_info(b)
    assert info["n_members"] == len(reqs)
    # the first call after members joined runs eagerly, the next at the same
    # membership replays a captured graph (when graphs are on)
    hdg.hdg_batch_rk3_steps(b, 1, prec=prec)
    hdg.hdg_batch_rk3_steps(b, 4, prec=prec)
    torch.cuda.synchronize()
    for i, q in enumerate(qs):
        assert np.array_equal(q.cpu().numpy(), alone[i]), f"member {i} differs from its solve alone"


def _mixed_mesh(seed):
    """A curved (quadratic) periodic box whose elements carry orders 2..6
    (faces between orders through mortars)."""
    mesh = W.periodic_box(3, Pg=2, curve_amp=0.2)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, seed)
    return mesh, flag, W.mixed_orders(flag, seed)


def _mixed_member(ctx, seed):
    """The mixed-order box with a TGV state per element."""
    mesh, flag, Pe = _mixed_mesh(seed)
    m = hdg.hdg_mesh_create(ctx, mesh, Pe, flag, hdg.make_params(c0sq=25.0, nu=5e-3, les_model=1, C_les=0.1))
    x = hdg.hdg_mesh_node_coords(m)
    n3 = (Pe.astype(np.int64) + 1) ** 3
    off = np.concatenate([[0], np.cumsum(n3)])
    q0 = np.empty(4 * off[-1])
    for e in range(len(Pe)):
        X = x[3 * off[e]:3 * off[e + 1]].reshape(3, n3[e])
        q0[4 * off[e]:4 * off[e + 1]] = W.taylor_green_state(X[None], 0.05, seed + e)[0].ravel()
    return m, q0, 2e-3, np.bincount(Pe)[2:]


@pytest.mark.parametrize("prec", [hdg.HDG_F64, hdg.HDG_F32])
@pytest.mark.parametrize("graphs", [True, False])
def test_batch_with_mixed_order_member(torch_cuda, ctx, prec, graphs):
    """A member of several orders (its own mortar launches in every stage)
    among one-order members: every member equals its solve alone, bitwise."""
    torch = torch_cuda
    reqs = _requests(3, seed=51 + prec)
    made = [_make(ctx, r) for r in reqs]
    mm, mq0, mdt, counts = _mixed_member(ctx, 4)
    made.insert(1, (mm, mq0, mdt))
    _say(f"batch with a mixed-order member (orders 2..6: {counts}) and boxes "
         f"{[(r['n'], r['P']) for r in reqs]}, prec {prec}, graphs {graphs}")
    alone = [_alone(torch, m, q0, dt, 5, prec) for (m, q0, dt) in made]
    b = hdg.hdg_batch_create(ctx, 6)
    hdg.hdg_batch_set_graphs(b, graphs)
    qs = []
    for (m, q0, dt) in made:
        q = torch.from_numpy(q0).cuda()
        hdg.hdg_batch_add(b, m, q, torch.empty_like(q), dt)
        qs.append(q)
    hdg.hdg_batch_rk3_steps(b, 1, prec=prec)
    hdg.hdg_batch_rk3_steps(b, 4, prec=prec)
    torch.cuda.synchronize()
    for i, q in enumerate(qs):
        out = q.cpu().numpy()
        assert np.isfinite(out).all()
        assert np.array_equal(out, alone[i]), f"member {i} differs from its solve alone"
    assert np.abs(alone[1] - mq0).max() > 1e-6                 # the mixed member did move


def test_batch_join_and_leave(torch_cuda, ctx):
    """Members join and leave between calls (continuous batching); each one's
    state equals its own solve advanced by the steps it was in the batch."""
    torch = torch_cuda
    prec = hdg.HDG_F32
    reqs = _requests(5, seed=21)
    made = [_make(ctx, r) for r in reqs]
    _say(f"join/leave on boxes (n, P) = {[(r['n'], r['P']) for r in reqs]}")
    b = hdg.hdg_batch_create(ctx, 3)
    state = {}
    slot_of = {}

    def join(i):
        m, q0, dt = made[i]
        q = torch.from_numpy(q0).cuda()
        dq = torch.empty_like(q)
        slot_of[i] = hdg.hdg_batch_add(b, m, q, dq, dt)
        state[i] = [q, 0]

    def run(k):
        hdg.hdg_batch_rk3_steps(b, k, prec=prec)
        for i in slot_of:
            state[i][1] += k

    def leave(i):
        torch.cuda.synchronize()
        hdg.hdg_batch_remove(b, slot_of.pop(i))

    join(0); join(1); join(2)
    with pytest.raises(hdg.HdgError) as ex:          # three slots: the fourth waits
        m, q0, dt = made[3]
        qq = torch.from_numpy(q0).cuda()
        hdg.hdg_batch_add(b, m, qq, torch.empty_like(qq), dt)
    assert ex.value.status == hdg.HDG_ENOMEM
    run(3)
    leave(1)
    join(3)
    run(2)
    leave(0)
    join(4)
    run(3)
    torch.cuda.synchronize()
    for i, (q, steps) in state.items():
        m, q0, dt = made[i]
        ref = _alone(torch, m, q0, dt, steps, prec)
        assert np.array_equal(q.cpu().numpy(), ref), f"request {i} after {steps} steps"
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_batch_remove(b, 7)
    assert ex.value.status == hdg.HDG_EINVAL


def test_batch_autotune_keeps_results(torch_cuda, ctx):
    torch = torch_cuda
    reqs = _requests(4, seed=33)
    made = [_make(ctx, r) for r in reqs]
    b = hdg.hdg_batch_create(ctx, 4)
    qs = []
    for (m, q0, dt) in made:
        q = torch.from_numpy(q0).cuda()
        qs.append(q)
        hdg.hdg_batch_add(b, m, q, torch.empty_like(q), dt)
    hdg.hdg_batch_autotune(b, reps=2)
    for (m, q0, dt), q in zip(made, qs):
        assert np.array_equal(q.cpu().numpy(), q0)      # the states are not modified
    hdg.hdg_batch_rk3_steps(b, 2, prec=hdg.HDG_F64)
    torch.cuda.synchronize()
    for i, (m, q0, dt) in enumerate(made):
        assert np.array_equal(qs[i].cpu().numpy(), _alone(torch, m, q0, dt, 2, hdg.HDG_F64))
    c = hdg.hdg_batch_get_launch(b, hdg.HDG_KERNEL_RESIDUAL, hdg.HDG_F64, reqs[0]["P"] + 1)
    assert c["us_per_launch"] > 0


def test_batch_precision_switch_and_two_streams(torch_cuda, ctx):
    """One batch stepped in FP64, then FP32 (the captured graph is dropped and
    recaptured), then on a second stream and back: each member equals its
    solve alone stepped through the same sequence, bitwise.  The batch's calls
    are chained, so a call on another stream starts after the previous one."""
    torch = torch_cuda
    reqs = _requests(3, seed=61)
    made = [_make(ctx, r) for r in reqs]
    _say(f"precision switch and two streams, boxes {[(r['n'], r['P']) for r in reqs]}")
    seq = [(hdg.HDG_F64, 1, 0), (hdg.HDG_F64, 2, 0), (hdg.HDG_F32, 2, 0), (hdg.HDG_F32, 4, 1),
           (hdg.HDG_F64, 2, 1), (hdg.HDG_F64, 3, 0)]
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    alone = []
    for (m, q0, dt) in made:
        q = torch.from_numpy(q0).cuda()
        dq = torch.empty_like(q)
        for prec, k, _ in seq:
            hdg.hdg_rk3_steps(m, q, dq, dt, k, prec=prec)
        torch.cuda.synchronize()
        alone.append(q.cpu().numpy())
    b = hdg.hdg_batch_create(ctx, 4)
    qs = []
    for (m, q0, dt) in made:
        q = torch.from_numpy(q0).cuda()
        hdg.hdg_batch_add(b, m, q, torch.empty_like(q), dt)
        qs.append(q)
    torch.cuda.synchronize()
    for prec, k, on_side in seq:
        hdg.hdg_batch_rk3_steps(b, k, prec=prec, stream=side if on_side else main)
    torch.cuda.synchronize()
    for i, q in enumerate(qs):
        assert np.array_equal(q.cpu().numpy(), alone[i]), f"member {i} differs from its solve alone"


def _oracle_case(orc, r):
    mesh = W.periodic_box(r["n"], Pg=1)
    flag = W.bernoulli_mask(mesh.n_elem, r["frac"], r["seed"])
    prm = dict(c0sq=25.0, nu=r["nu"], les_model=1, C_les=0.1, mixed_face=0, q_inf=(0, 0, 0, 0))
    return orc.OracleMesh(mesh, r["P"], flag), orc.make_params(**prm)


@pytest.mark.parametrize("prec", [hdg.HDG_F64, hdg.HDG_F32])
def test_batch_members_match_oracle(orc, torch_cuda, ctx, prec):
    """Members of one batch (three one-order boxes of different orders and a
    member of orders 2..6 with mortars) against the FP64 oracle's RK3, per
    field on the increments q - q0: FP64 within 1e-12 (or the states'
    rounding floor), FP32 residual arithmetic within 1e-5 on the velocity rows
    (the pressure row's floored error is reported)."""
    torch = torch_cuda
    reqs = [dict(n=3, P=2, frac=0.5, nu=3e-3, seed=71), dict(n=3, P=4, frac=0.3, nu=1e-3, seed=72),
            dict(n=3, P=5, frac=0.7, nu=5e-3, seed=73)]
    made = [_make(ctx, r) for r in reqs]
    mm, mq0, mdt, counts = _mixed_member(ctx, 8)
    steps = 4
    _say(f"batch vs oracle, prec {prec}: boxes {[(r['n'], r['P']) for r in reqs]} and orders 2..6 {counts}")
    b = hdg.hdg_batch_create(ctx, 4)
    qs = []
    for (m, q0, dt) in made + [(mm, mq0, mdt)]:
        q = torch.from_numpy(np.ascontiguousarray(q0)).cuda()
        hdg.hdg_batch_add(b, m, q, torch.empty_like(q), dt)
        qs.append(q)
    hdg.hdg_batch_rk3_steps(b, 1, prec=prec)
    hdg.hdg_batch_rk3_steps(b, steps - 1, prec=prec)
    torch.cuda.synchronize()
    for i, (r, (m, q0, dt)) in enumerate(zip(reqs, made)):
        om, po = _oracle_case(orc, r)
        ref = om.rk3(po, q0, dt, steps)
        out = qs[i].cpu().numpy().reshape(ref.shape)
        e = increment_errors(out, ref, q0, oracle_mass(orc, om, r["P"]))
        _say(f"member {i} (P={r['P']}): increment errors L2 {e['l2']}, max {e['max']}")
        if prec == hdg.HDG_F64:
            assert np.all(e["l2"] <= np.maximum(TOL_F64, e["floor_l2"]))
            assert np.all(e["max"] <= np.maximum(TOL_F64, e["floor_max"]))
        else:
            assert e["l2"][1:].max() <= TOL_F32 and e["max"][1:].max() <= 10 * TOL_F32
            assert e["l2"][1:].max() > 1e-12          # the FP32 path ran
    # the member of several orders
    mesh, flag, Pe = _mixed_mesh(8)
    om = orc.OracleMesh(mesh, Pe, flag)
    po = orc.make_params(c0sq=25.0, nu=5e-3, les_model=1, C_les=0.1)
    ref = om.rk3(po, mq0, mdt, steps)
    out = qs[3].cpu().numpy()
    l2, mx = flat_errors(om, flat_mass(orc, om), out - mq0, ref - mq0)
    _say(f"mixed-order member: increment errors L2 {l2}, max {mx}")
    if prec == hdg.HDG_F64:
        assert max(l2.max(), mx.max()) <= TOL_F64
    else:
        assert l2[1:].max() <= TOL_F32 and mx[1:].max() <= 10 * TOL_F32
