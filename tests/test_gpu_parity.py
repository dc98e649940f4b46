"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Every case prints its name, shape and seed before touching the GPU.
"""
import math
import sys

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, workloads as W
from parity import TOL_F64, assert_increment_parity, assert_parity, field_errors, oracle_mass

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


def _params(**kw):
    base = dict(c0sq=25.0, nu=1e-3, les_model=1, C_les=0.1, mixed_face=0, q_inf=(0, 0, 0, 0))
    base.update(kw)
    return base


def _run_pair(orc, torch, ctx, mesh, P, flag, prm, q, rk=None):
    """Residual (or rk=(dt, nsteps)) on the GPU and in the oracle."""
    om = orc.OracleMesh(mesh, P, flag)
    m = hdg.hdg_mesh_create(ctx, mesh, P, flag, hdg.make_params(**prm))
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    if rk is None:
        rd = torch.empty_like(qd)
        hdg.hdg_residual(m, qd, rd)
        torch.cuda.synchronize()
        out = rd.cpu().numpy()
        ref = om.residual(orc.make_params(**prm), q)
    else:
        dt, n = rk
        dq = torch.empty_like(qd)
        hdg.hdg_rk3_steps(m, qd, dq, dt, n)
        torch.cuda.synchronize()
        out = qd.cpu().numpy()
        ref = om.rk3(orc.make_params(**prm), q, dt, n)
    return out, ref, oracle_mass(orc, om, P), m


def test_residual_parity_tgv_box(orc, torch_cuda, ctx):
    w = W.tgv_box_small()
    _say(f"{w.name} residual, mask seed 1, noise seed 0")
    om = orc.OracleMesh(w.mesh, w.P, w.flag)
    q = W.initial_state(w, om.node_coords())
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, w.mesh, w.P, w.flag, w.params, q)
    e = assert_parity(out, ref, mass, what=w.name)
    _say(f"errors l2={e['l2']} max={e['max']}")


def test_rk3_parity_tgv_box(orc, torch_cuda, ctx):
    w = W.tgv_box_small()
    _say(f"{w.name} {w.nsteps} RK3 steps dt={w.dt}")
    om = orc.OracleMesh(w.mesh, w.P, w.flag)
    q = W.initial_state(w, om.node_coords())
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, w.mesh, w.P, w.flag, w.params, q, rk=(w.dt, w.nsteps))
    assert_parity(out, ref, mass, what=w.name + " rk3")
    e = assert_increment_parity(out, ref, q, mass, what=w.name + " rk3 increments")
    _say(f"increment errors l2={e['l2']} max={e['max']} (rounding floor max {e['floor_max']})")
    assert np.abs(out - q).max() > 1e-4          # the state did move


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("mask", ["mixed", "euler", "viscous"])
def test_residual_parity_orders_and_masks(orc, torch_cuda, ctx, P, mask):
    """Curved, randomly re-oriented periodic box: every order (N^3 = 8 .. 512 nodes,
    ragged against 64-lane waves), all-Euler (no viscous launch), all-viscous."""
    base = W.periodic_box(3, Pg=2, curve_amp=0.3)
    mesh, _ = W.reorient(base, seed=P)
    flag = {"mixed": W.bernoulli_mask(mesh.n_elem, 0.5, P), "euler": np.zeros(mesh.n_elem, np.uint8),
            "viscous": np.ones(mesh.n_elem, np.uint8)}[mask]
    _say(f"reoriented curved box 3^3 P={P} mask={mask} seed={P}")
    om = orc.OracleMesh(mesh, P, flag)
    q = W.taylor_green_state(om.node_coords(), 0.05, seed=P)
    prm = _params(nu=5e-3, les_model=1 + (P % 2), C_les=0.1 if P % 2 == 0 else 0.07)
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, mesh, P, flag, prm, q)
    assert_parity(out, ref, mass, what=f"P={P} {mask}")


@pytest.mark.parametrize("P", [2, 4, 6])
def test_residual_parity_rusanov(orc, torch_cuda, ctx, P):
    """The Rusanov flux switch: residual (FP64 and FP32) and two RK steps on a
    curved re-oriented box with a mixed mask."""
    torch = torch_cuda
    mesh, _ = W.reorient(W.periodic_box(3, Pg=2, curve_amp=0.3), seed=20 + P)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, 20 + P)
    _say(f"Rusanov flux, reoriented curved box 3^3 P={P}")
    om = orc.OracleMesh(mesh, P, flag)
    q = W.taylor_green_state(om.node_coords(), 0.05, seed=P)
    prm = _params(nu=5e-3, riemann=hdg.HDG_RUSANOV)
    out, ref, mass, m = _run_pair(orc, torch, ctx, mesh, P, flag, prm, q)
    assert_parity(out, ref, mass, what=f"Rusanov P={P}")
    roe = om.residual(orc.make_params(**_params(nu=5e-3)), q)
    assert np.abs(roe - ref).max() > 1e-6 * np.abs(ref).max()       # the switch changes the result
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    r32 = torch.empty(qd.shape, dtype=torch.float32, device="cuda")
    hdg.hdg_residual(m, qd, r32, prec=hdg.HDG_F32)
    torch.cuda.synchronize()
    e = field_errors(r32.cpu().numpy().astype(np.float64), ref, mass)
    _say(f"Rusanov FP32 P={P}: per-field L2 {e['l2']}")
    assert e["l2"][1:].max() <= 1e-5                 # velocity rows (pressure row: see the FP32 tests)
    out, ref, mass, _ = _run_pair(orc, torch, ctx, mesh, P, flag, prm, q, rk=(1e-3, 2))
    assert_parity(out, ref, mass, what=f"Rusanov RK P={P}")


@pytest.mark.parametrize("mixed_face,riemann", [(0, 0), (1, 0), (0, 1)])
def test_residual_parity_ogrid_small(orc, torch_cuda, ctx, mixed_face, riemann):
    """Walls and far field (ghost states), both mixed-face readings, both fluxes."""
    mesh = W.naca_ogrid(48, 16, 4, Pg=2)
    flag = W.naca_mask(mesh)
    P = 4
    _say(f"O-grid 48x16x4 P=4 mixed_face={mixed_face} riemann={riemann}")
    q = W.uniform_inflow_state(mesh.n_elem, 125, 20.0, 1.0, 0.01, seed=3)
    prm = _params(nu=1e-4, q_inf=W.free_stream(20.0), mixed_face=mixed_face, riemann=riemann)
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, mesh, P, flag, prm, q)
    assert_parity(out, ref, mass, what="ogrid small")


@pytest.mark.parametrize("flagged", [0, 1])
def test_single_element_all_boundary(orc, torch_cuda, ctx, flagged):
    """One element whose six faces are far-field boundaries (no interior face,
    one tile of one element): residual and RK against the oracle; zero RK
    steps leave the state as it was."""
    torch = torch_cuda
    mesh = W.box((1, 1, 1), periodic=(False, False, False))
    flag = np.array([flagged], np.uint8)
    P = 3
    _say(f"single element, far field on all faces, flagged={flagged}")
    om = orc.OracleMesh(mesh, P, flag)
    q = W.taylor_green_state(om.node_coords(), 0.05, seed=2)
    prm = _params(nu=5e-3, q_inf=(0.0, 0.5, 0.0, 0.0))
    out, ref, mass, m = _run_pair(orc, torch_cuda, ctx, mesh, P, flag, prm, q)
    assert_parity(out, ref, mass, what="single element")
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, mesh, P, flag, prm, q, rk=(1e-3, 3))
    assert_parity(out, ref, mass, what="single element rk3")
    assert_increment_parity(out, ref, q, mass, what="single element rk3 increments")
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    hdg.hdg_rk3_steps(m, qd, torch.empty_like(qd), 1e-3, 0)
    torch.cuda.synchronize()
    assert np.array_equal(qd.cpu().numpy(), q)


def test_residual_parity_naca_working_size(orc, torch_cuda, ctx):
    """The benchmark workload at full size (96x48x8, P=4, 4.6M nodes), all outputs."""
    w = W.naca_working()
    _say(f"{w.name} residual at full size")
    q = W.initial_state(w, None)
    out, ref, mass, m = _run_pair(orc, torch_cuda, ctx, w.mesh, w.P, w.flag, w.params, q)
    e = assert_parity(out, ref, mass, what=w.name)
    _say(f"errors l2={e['l2']} max={e['max']} raw_max={e['max_raw']}")


def test_rk3_parity_naca_working_size(orc, torch_cuda, ctx):
    """Two fused RK steps on the full benchmark mesh, compared on the
    increments q - q0 per field.  At the workload's dt = 2e-8 two steps move
    the state by about 1e-4 of itself, so a comparison of states (or of
    increments, whose rounding floor is then ~1e-12) would pin the RK update
    only loosely: the steps are taken at 100 dt, where the increment is large
    enough for the 1e-12 bound to bite (two steps stay finite there)."""
    w = W.naca_working()
    q = W.initial_state(w, None)
    dt = 100 * w.dt
    _say(f"{w.name} 2 RK3 steps dt={dt:.3e}")
    out, ref, mass, _ = _run_pair(orc, torch_cuda, ctx, w.mesh, w.P, w.flag, w.params, q, rk=(dt, 2))
    assert_parity(out, ref, mass, what=w.name + " rk3")
    e = assert_increment_parity(out, ref, q, mass, what=w.name + " rk3 increments")
    _say(f"increment errors l2={e['l2']} max={e['max']} (rounding floor max {e['floor_max']})")
    assert e["floor_max"].max() < 1e-13          # the comparison is not rounding-limited


def test_naca_working_size_stays_bounded(torch_cuda, ctx):
    """100 RK steps of the benchmark workload at its stated dt: finite and bounded."""
    torch = torch_cuda
    w = W.naca_working()
    _say(f"{w.name} {w.nsteps} RK3 steps dt={w.dt:.1e}: finiteness")
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q = torch.from_numpy(W.initial_state(w, None)).cuda()
    dq = torch.empty_like(q)
    hdg.hdg_rk3_steps(m, q, dq, w.dt, w.nsteps)
    red = hdg.hdg_reduce(m, q)
    assert red["finite"] and red["max"][1:].max() < 3.0


def test_deterministic_bitwise(orc, torch_cuda, ctx):
    torch = torch_cuda
    w = W.naca_working(48, 16, 4)
    _say("determinism: residual and RK twice on O-grid 48x16x4")
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q = torch.from_numpy(W.initial_state(w, None)).cuda()
    r1, r2 = torch.empty_like(q), torch.empty_like(q)
    hdg.hdg_residual(m, q, r1)
    hdg.hdg_residual(m, q, r2)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    qa, qb = q.clone(), q.clone()
    dq = torch.empty_like(q)
    hdg.hdg_rk3_steps(m, qa, dq, 1e-7, 3)
    hdg.hdg_rk3_steps(m, qb, dq, 1e-7, 3)
    torch.cuda.synchronize()
    assert torch.equal(qa, qb)


def test_rk_split_equals_whole(orc, torch_cuda, ctx):
    """5 + 5 steps equal 10 steps bitwise (the register is dead between steps)."""
    torch = torch_cuda
    w = W.tgv_box_small()
    _say("rk 5+5 vs 10 on the small box")
    om = orc.OracleMesh(w.mesh, w.P, w.flag)
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q0 = torch.from_numpy(W.initial_state(w, om.node_coords())).cuda()
    qa, qb, dq = q0.clone(), q0.clone(), torch.empty_like(q0)
    hdg.hdg_rk3_steps(m, qa, dq, w.dt, 10)
    dq.fill_(float("nan"))           # the first stage must not read the register
    hdg.hdg_rk3_steps(m, qb, dq, w.dt, 5)
    hdg.hdg_rk3_steps(m, qb, dq, w.dt, 5)
    torch.cuda.synchronize()
    assert torch.equal(qa, qb)


def test_gpu_conservation_and_freestream(orc, torch_cuda, ctx):
    torch = torch_cuda
    P = 4
    mesh, _ = W.reorient(W.periodic_box(3, Pg=2, curve_amp=0.3), seed=9)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, 4)
    _say("conservation + freestream on reoriented curved box P=4")
    m = hdg.hdg_mesh_create(ctx, mesh, P, flag, hdg.make_params(**_params(les_model=2, C_les=0.07)))
    rng = np.random.default_rng(5)
    q = torch.from_numpy(rng.uniform(-1, 1, size=(mesh.n_elem, 4, 125))).cuda()
    r = torch.empty_like(q)
    hdg.hdg_residual(m, q, r)
    red = hdg.hdg_reduce(m, r)
    absr = hdg.hdg_reduce(m, r.abs())
    assert np.all(np.abs(red["sum"]) < 1e-13 * absr["sum"])
    qc = torch.zeros_like(q)
    qc[:, 0], qc[:, 1], qc[:, 2], qc[:, 3] = 0.2, 0.9, -0.4, 0.3
    hdg.hdg_residual(m, qc, r)
    red = hdg.hdg_reduce(m, r)
    assert red["max"].max() < 1e-10 * 25.0


def test_set_flags_and_params(orc, torch_cuda, ctx):
    torch = torch_cuda
    w = W.tgv_box_small()
    _say("re-flag + new params on the small box")
    om = orc.OracleMesh(w.mesh, w.P, w.flag)
    q = W.initial_state(w, om.node_coords())
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    flag2 = W.bernoulli_mask(w.mesh.n_elem, 0.3, 77)
    prm2 = dict(w.params, les_model=2, C_les=0.07, mixed_face=1)
    hdg.hdg_mesh_set_flags(m, flag2)
    hdg.hdg_mesh_set_params(m, hdg.make_params(**prm2))
    qd = torch.from_numpy(q).cuda()
    rd = torch.empty_like(qd)
    hdg.hdg_residual(m, qd, rd)
    torch.cuda.synchronize()
    om.set_flags(flag2)
    ref = om.residual(orc.make_params(**prm2), q)
    assert_parity(rd.cpu().numpy(), ref, oracle_mass(orc, om, w.P), what="reflagged")
    assert hdg.hdg_mesh_info(m)["n_viscous"] == int(flag2.sum())


def test_error_paths(torch_cuda, ctx):
    torch = torch_cuda
    w = W.tgv_box_small()
    _say("error paths")
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q = torch.zeros(m.state_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_residual(m, q, q)
    assert ex.value.status == hdg.HDG_EINVAL
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_residual(m, q, torch.empty_like(q), prec=7)
    assert ex.value.status == hdg.HDG_EINVAL
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_rk3_steps(m, q, torch.empty_like(q), -1.0, 1)
    assert ex.value.status == hdg.HDG_EINVAL
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_set_params(m, hdg.make_params(c0sq=-1.0))
    assert ex.value.status == hdg.HDG_EINVAL
    bad = W.HexMesh(Pg=1, xyz_geom=w.mesh.xyz_geom, corners=w.mesh.corners, nbr=w.mesh.nbr.copy(),
                    nbr_face=w.mesh.nbr_face, orient=w.mesh.orient, centroid=w.mesh.centroid)
    bad.nbr[3, 2] = 0
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_create(ctx, bad, 3, w.flag, hdg.make_params(**w.params))
    assert ex.value.status == hdg.HDG_EMESH
    r = torch.full_like(q, float("nan"))
    out = hdg.hdg_reduce(m, r, allow_nonfinite=True)
    assert not out["finite"]
    with pytest.raises(hdg.HdgError) as ex:                        # no such kernel class
        hdg.hdg_timing_samples(m, hdg.HDG_KERNEL_COUNT)
    assert ex.value.status == hdg.HDG_EINVAL
    assert hdg.hdg_timing_samples(m, hdg.HDG_KERNEL_RESIDUAL) == []  # timing never enabled


def test_timing_and_copy_probe(torch_cuda, ctx):
    torch = torch_cuda
    w = W.naca_working(48, 16, 4)
    _say("kernel timing events + copy probe")
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q = torch.from_numpy(W.initial_state(w, None)).cuda()
    dq = torch.empty_like(q)
    hdg.hdg_timing_enable(m, True)
    hdg.hdg_rk3_steps(m, q, dq, 1e-7, 2)
    for k in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL):
        ms, n = hdg.hdg_timing_read(m, k)
        # one viscous launch per stage; the residual tiles of Euler elements
        # with no flagged neighbour are a launch of their own
        assert (n == 6 if k == hdg.HDG_KERNEL_VISCOUS else n == 12) and ms > 0
        us = hdg.hdg_timing_samples(m, k)                           # the same launches, one by one
        assert len(us) == n and min(us) > 0
        assert abs(sum(us) / 1e3 - ms) <= 1e-3 * ms
    assert hdg.hdg_timing_read(m, hdg.HDG_KERNEL_MORTAR)[1] == 0     # one order: no mortar faces
    assert hdg.hdg_timing_samples(m, hdg.HDG_KERNEL_MORTAR) == []
    hdg.hdg_timing_enable(m, False)
    # the timer's events are recorded by each dispatch: the launches run one
    # after another, so their durations add up to less than the span of the
    # steps on the stream
    hdg.hdg_timing_enable(m, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hdg.hdg_rk3_steps(m, q, dq, 1e-7, 2)
    e1.record()
    torch.cuda.synchronize()
    span = e0.elapsed_time(e1)
    total = sum(hdg.hdg_timing_read(m, k)[0] for k in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL))
    _say(f"kernel time {total:.4f} ms of a {span:.4f} ms span")
    assert 0 < total < span
    hdg.hdg_timing_enable(m, False)
    # a scattered mask (periodic 4^3 box, Bernoulli(0.5)): 2 of the 28 Euler
    # elements have no flagged neighbour, too few for a launch of their own,
    # so each stage takes one residual launch
    box = W.periodic_box(4, Pg=1)
    fb = W.bernoulli_mask(box.n_elem, 0.5, 1)
    mb = hdg.hdg_mesh_create(ctx, box, 3, fb, hdg.make_params(**w.params))
    qb = torch.zeros(mb.nodes * 4, dtype=torch.float64, device="cuda")
    hdg.hdg_timing_enable(mb, True)
    hdg.hdg_rk3_steps(mb, qb, torch.empty_like(qb), 1e-3, 2)
    assert hdg.hdg_timing_read(mb, hdg.HDG_KERNEL_VISCOUS)[1] == 6
    assert hdg.hdg_timing_read(mb, hdg.HDG_KERNEL_RESIDUAL)[1] == 6
    hdg.hdg_timing_enable(mb, False)
    a = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    hdg.hdg_stream_copy(ctx, b, a, a.numel() * 8)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_handles_released_in_any_order(orc, torch_cuda):
    """The context is released first (as a garbage collector may do with a
    cycle): the mesh made from it still computes the same residual, and its
    and a batch's destruction afterwards leave no HIP error behind for the
    next torch launch."""
    torch = torch_cuda
    mesh, _ = W.reorient(W.periodic_box(3, Pg=2, curve_amp=0.2), seed=3)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, 3)
    _say("handles released in any order: box 3^3 P=3")
    c2 = hdg.hdg_init(0)
    m = hdg.hdg_mesh_create(c2, mesh, 3, flag, hdg.make_params(**_params()))
    b = hdg.hdg_batch_create(c2, 2)
    q = W.taylor_green_state(orc.OracleMesh(mesh, 3, flag).node_coords(), 0.05, seed=3)
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    r0 = torch.empty_like(qd)
    hdg.hdg_residual(m, qd, r0)
    torch.cuda.synchronize()
    hdg.lib().hdg_finalize(c2.handle)
    c2.handle = None
    r1 = torch.empty_like(qd)
    hdg.hdg_residual(m, qd, r1)
    torch.cuda.synchronize()
    assert torch.equal(r0, r1)
    del b, m
    x = torch.cos(torch.ones(1000, dtype=torch.float64, device="cuda")).sum()
    torch.cuda.synchronize()
    assert abs(x.item() - 1000 * math.cos(1.0)) < 1e-9


def test_translated_elements_share_metric_blocks(orc, torch_cuda, ctx):
    """Elements that are translates of one another read one metric block: one
    block for a uniform periodic box, one per span column of the extruded
    O-grid, one per element where the curved displacement makes every element
    different.  The residual with shared blocks stays within 1e-12 of the
    oracle (which builds every element's own terms)."""
    torch = torch_cuda
    box = W.periodic_box(4, Pg=1)
    og = W.naca_ogrid(24, 8, 4, Pg=2)
    curved = W.periodic_box(3, Pg=2, curve_amp=0.3)
    _say("metric blocks: uniform box, extruded O-grid 24x8x4, curved box")
    for mesh, P, want in ((box, 3, 1), (og, 4, og.n_elem // 4), (curved, 4, curved.n_elem)):
        flag = W.bernoulli_mask(mesh.n_elem, 0.5, 3)
        m = hdg.hdg_mesh_create(ctx, mesh, P, flag, hdg.make_params(**_params(q_inf=W.free_stream(20.0))))
        assert hdg.hdg_mesh_metric_blocks(m) == want
    flag = W.naca_mask(og)
    prm = _params(nu=1e-3, q_inf=W.free_stream(20.0))
    om = orc.OracleMesh(og, 4, flag)
    q = W.uniform_inflow_state(og.n_elem, 125, 20.0, 1.0, 0.05, seed=4)
    out, ref, mass, _ = _run_pair(orc, torch, ctx, og, 4, flag, prm, q)
    e = assert_parity(out, ref, mass, what="extruded O-grid with shared metric blocks")
    _say(f"errors l2={e['l2']} max={e['max']}")


def _rows(q, P):
    """(nodes, 4) rows p, u, v, w of a flat state, element after element."""
    out, o = [], 0
    for p in P:
        n3 = (int(p) + 1) ** 3
        out.append(q[4 * o:4 * (o + n3)].reshape(4, n3).T)
        o += n3
    return np.concatenate(out)


def test_max_wave_speed_matches_oracle(orc, torch_cuda, ctx):
    torch = torch_cuda
    rng = np.random.default_rng(21)
    mesh = W.periodic_box(3, Pg=1, curve_amp=0.2)
    flag = W.bernoulli_mask(mesh.n_elem, 0.5, 3)
    for label, P in (("one order P = 4", np.full(mesh.n_elem, 4, np.int32)),
                     ("orders 2..6", W.mixed_orders(flag, 5).astype(np.int32))):
        _say(f"max wave speed, warped box 3^3, {label}")
        m = hdg.hdg_mesh_create(ctx, mesh, P, flag, hdg.make_params(**_params(c0sq=16.0)))
        q = rng.normal(size=4 * int(((P + 1) ** 3).sum()))
        got = hdg.hdg_max_wave_speed(m, torch.from_numpy(q).cuda())
        ref = orc.max_wave_speed(_rows(q, P), 16.0)
        assert abs(got - ref) <= 1e-14 * ref, (label, got, ref)
    qn = torch.from_numpy(q).cuda()
    qn[2] = float("nan")                       # a pressure: not part of the wave speed
    assert hdg.hdg_max_wave_speed(m, qn) == got
    n3 = (int(P[0]) + 1) ** 3
    qn[2 * n3 + 2] = float("inf")              # a velocity (v) of the first element
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_max_wave_speed(m, qn)
    assert ex.value.status == hdg.HDG_ENONFINITE
