"""Clustering on the GPU (node features, Gaussian mixture, element regions)
against the FP64 oracle, and the flags it produces applied to the residual."""
import sys

import numpy as np
import pytest

from oracle import cluster as CL
from paper_2403_05463_amd import hdg, workloads as W
from parity import TOL_F64

pytestmark = pytest.mark.gpu

ITERS = 40
REG = 1e-6
# EM carries the features' rounding through its iterations: parameters and
# memberships are compared at 1e-8, the features themselves at 1e-11 of
# their largest magnitude.
TOL_FEAT = 1e-11
TOL_FIT = 1e-8


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


def _jet(X, d=0.5):
    """A jet along x with a spanwise-modulated core in a periodic [0, 2 pi]^3 box."""
    y, z = X[..., 1, :], X[..., 2, :]
    return np.exp(-((y - np.pi) / d) ** 2) * (1.0 + 0.3 * np.sin(z)), 0.1 * np.sin(y) * np.cos(z)


def _cases():
    m = W.periodic_box(4, Pg=1, curve_amp=0.25)
    yield "warped periodic box 4^3, P=3, jet", m, 3, W.bernoulli_mask(m.n_elem, 0.5, 1), dict(nu=5e-3)
    m2, _ = W.reorient(W.periodic_box(3, Pg=1, curve_amp=0.2), seed=4)
    f2 = W.bernoulli_mask(m2.n_elem, 0.5, 3)
    yield "reoriented warped box 3^3, P 2..6 (mortars), jet", m2, W.mixed_orders(f2, 5), f2, dict(nu=5e-3)
    g = W.naca_ogrid(48, 16, 4, Pg=2)
    yield "O-grid 48x16x4 quadratic geometry, P=3, developed airfoil flow", g, 3, W.naca_mask(g), \
        dict(nu=1e-3, q_inf=W.free_stream(20.0))


def _params(kw):
    base = dict(c0sq=25.0, nu=5e-3, les_model=1, C_les=0.1, mixed_face=0, q_inf=(0, 0, 0, 0))
    base.update(kw)
    return base


def _state(name, om):
    X = om.node_coords()
    if "airfoil" in name:
        return W.developed_airfoil_state(X)
    q = np.zeros(4 * om.nodes) if not om.uniform else np.zeros((om.n_elem, 4, om.N3))
    for e in range(om.n_elem):
        blk = om.element(X, e, 3)
        u, w = _jet(blk)
        qe = om.element(q, e, 4)
        qe[1], qe[3] = u, w
        qe[0] = 0.1 * np.cos(blk[0])
    return q


def _setup(orc, torch, ctx, case):
    name, mesh, P, flag, kw = list(_cases())[case]
    prm = _params(kw)
    om = orc.OracleMesh(mesh, P, flag)
    q = _state(name, om)
    m = hdg.hdg_mesh_create(ctx, mesh, P, flag, hdg.make_params(**prm))
    return name, om, orc.make_params(**prm), q, m


def _near_tie(pv, tol):
    return np.abs(pv - 0.5) < tol


@pytest.mark.parametrize("case", [0, 1, 2])
def test_features_and_fit_parity(orc, torch_cuda, ctx, case):
    torch = torch_cuda
    name, om, oprm, q, m = _setup(orc, torch, ctx, case)
    _say(f"clustering: {name}")
    Xo = CL.node_features(om, oprm, q)
    qd = torch.from_numpy(np.ascontiguousarray(q).ravel()).cuda()
    Xg = torch.empty(3 * om.nodes, dtype=torch.float64, device="cuda")
    hdg.hdg_cluster_features(m, qd, Xg)
    torch.cuda.synchronize()
    Xgn = Xg.cpu().numpy().reshape(3, -1)
    scale = np.abs(Xo).max(axis=1)
    err = np.abs(Xgn - Xo).max(axis=1) / scale
    _say(f"{name}: feature errors (Q_S, R_S, Q_Omega) relative to max {err}")
    assert err.max() <= TOL_FEAT

    fo = CL.fit_gmm(Xo, ITERS, REG)
    pvo = CL.element_means(fo.p_visc, om.offsets, om.Ps)
    flo = CL.element_flags(pvo)
    pv = torch.empty(om.nodes, dtype=torch.float64, device="cuda")
    epv = torch.empty(om.n_elem, dtype=torch.float64, device="cuda")
    res, flags = hdg.hdg_cluster_fit(m, Xg, ITERS, REG, p_visc=pv, elem_pv=epv)
    assert not res["degenerate"] and res["iterations"] == ITERS
    assert np.all(np.abs(res["feat_mean"] - fo.feat_mean) <= 1e-10 * np.abs(fo.feat_mean) + 1e-12 * scale)
    np.testing.assert_allclose(res["feat_std"], fo.feat_std, rtol=1e-10)
    np.testing.assert_allclose(res["weight"], fo.mixture.weight, rtol=TOL_FIT, atol=TOL_FIT)
    np.testing.assert_allclose(res["mean"], fo.mixture.mean, rtol=TOL_FIT, atol=TOL_FIT)
    np.testing.assert_allclose(res["cov"], fo.mixture.cov, rtol=TOL_FIT, atol=TOL_FIT)
    assert abs(res["log_likelihood"] - fo.log_likelihood) <= TOL_FIT * max(1.0, abs(fo.log_likelihood))
    np.testing.assert_allclose(pv.cpu().numpy(), fo.p_visc, atol=TOL_FIT)
    epvn = epv.cpu().numpy()
    np.testing.assert_allclose(epvn, pvo, atol=TOL_FIT)
    clear = ~_near_tie(pvo, 1e-6)
    assert np.array_equal(flags[clear], flo[clear])
    assert res["n_viscous"] == int(flags.sum())
    _say(f"{name}: {flags.sum()} of {om.n_elem} elements viscous, weights {res['weight']}, "
         f"log-likelihood {res['log_likelihood']:.6f}")
    assert 0 < flags.sum() < om.n_elem


def test_fit_of_oracle_features_and_determinism(orc, torch_cuda, ctx):
    """The fit alone, on the oracle's own features: tighter agreement; two
    fits give identical results."""
    torch = torch_cuda
    name, om, oprm, q, m = _setup(orc, torch, ctx, 2)
    Xo = CL.node_features(om, oprm, q)
    X = torch.from_numpy(Xo.ravel().copy()).cuda()
    fo = CL.fit_gmm(Xo, 60, REG)
    out = []
    for _ in range(2):
        pv = torch.empty(om.nodes, dtype=torch.float64, device="cuda")
        res, flags = hdg.hdg_cluster_fit(m, X, 60, REG, p_visc=pv)
        out.append((res, flags, pv.cpu().numpy()))
    (r0, f0, p0), (r1, f1, p1) = out
    assert np.array_equal(p0, p1) and np.array_equal(f0, f1)
    assert np.array_equal(r0["cov"], r1["cov"])
    np.testing.assert_allclose(r0["mean"], fo.mixture.mean, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(r0["cov"], fo.mixture.cov, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(p0, fo.p_visc, atol=1e-9)
    assert not r0["converged"]
    # a tolerance ends the fit on the device at the oracle's iteration, unless
    # the deciding change sits within rounding of the tolerance
    for tol in (1e-4, 1e-8):
        ft = CL.fit_gmm(Xo, 500, REG, tol)
        steps = np.abs(np.diff(ft.history))
        if np.any(np.abs(steps - tol) < 1e-12):
            continue
        rt, _ = hdg.hdg_cluster_fit(m, X, 500, REG, tol=tol)
        assert rt["converged"] and rt["iterations"] == len(ft.history) < 500
        np.testing.assert_allclose(rt["mean"], ft.mixture.mean, rtol=1e-9, atol=1e-10)


def test_fluid_at_rest_is_degenerate(orc, torch_cuda, ctx):
    torch = torch_cuda
    m = W.periodic_box(3, Pg=1, curve_amp=0.2)
    flag = np.zeros(m.n_elem, np.uint8)
    mesh = hdg.hdg_mesh_create(ctx, m, 3, flag, hdg.make_params(**_params({})))
    q = np.zeros((m.n_elem, 4, 64))
    q[:, 0] = np.linspace(0.0, 1.0, m.n_elem)[:, None]
    qd = torch.from_numpy(q).cuda()
    X = torch.empty(3 * mesh.nodes, dtype=torch.float64, device="cuda")
    hdg.hdg_cluster_features(mesh, qd, X)
    pv = torch.full((mesh.nodes,), 7.0, dtype=torch.float64, device="cuda")
    res, flags = hdg.hdg_cluster_fit(mesh, X, 10, REG, p_visc=pv)
    assert torch.all(X == 0.0)
    assert res["degenerate"] and res["n_viscous"] == 0 and not flags.any()
    assert torch.all(pv == 0.0)


def test_reflag_then_residual_parity(orc, torch_cuda, ctx):
    """A clustering step of a dynamic run: the flags found are applied to the
    mesh, and the residual with them matches the oracle's with the same flags."""
    torch = torch_cuda
    name, om, oprm, q, m = _setup(orc, torch, ctx, 1)
    qd = torch.from_numpy(np.ascontiguousarray(q).ravel()).cuda()
    X = torch.empty(3 * om.nodes, dtype=torch.float64, device="cuda")
    hdg.hdg_cluster_features(m, qd, X)
    res, flags = hdg.hdg_cluster_fit(m, X, ITERS, REG)
    hdg.hdg_mesh_set_flags(m, flags)
    om.set_flags(flags)
    ref = om.residual(oprm, q)
    r = torch.empty_like(qd)
    hdg.hdg_residual(m, qd, r)
    torch.cuda.synchronize()
    got = r.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"residual after re-flagging ({flags.sum()} viscous): max error {err:.3e}")
    assert err <= 10 * TOL_F64
    assert hdg.hdg_mesh_info(m)["n_viscous"] == int(flags.sum())


def test_full_size_airfoil(orc, torch_cuda, ctx):
    """The benchmark's airfoil mesh (96 x 48 x 8, quadratic geometry, P = 4,
    4.6M nodes) with the developed-flow stand-in, in the configuration the
    benchmark times: every node's features and a 10-iteration fit against
    the oracle."""
    torch = torch_cuda
    w = W.naca_working()
    _say(f"full-size clustering: {w.name}")
    om = orc.OracleMesh(w.mesh, w.P, w.flag)
    q = W.developed_airfoil_state(om.node_coords())
    oprm = orc.make_params(**w.params)
    m = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    qd = torch.from_numpy(q).cuda()
    X = torch.empty(3 * om.nodes, dtype=torch.float64, device="cuda")
    hdg.hdg_cluster_features(m, qd, X)
    torch.cuda.synchronize()
    Xo = CL.node_features(om, oprm, q)
    Xg = X.cpu().numpy().reshape(3, -1)
    err = np.abs(Xg - Xo).max(axis=1) / np.abs(Xo).max(axis=1)
    _say(f"feature errors {err}")
    assert err.max() <= TOL_FEAT
    fo = CL.fit_gmm(Xo, 10, REG)
    pvo = CL.element_means(fo.p_visc, om.offsets, om.Ps)
    res, flags = hdg.hdg_cluster_fit(m, X, 10, REG)
    np.testing.assert_allclose(res["mean"], fo.mixture.mean, rtol=TOL_FIT, atol=TOL_FIT)
    np.testing.assert_allclose(res["cov"], fo.mixture.cov, rtol=TOL_FIT, atol=TOL_FIT)
    clear = ~_near_tie(pvo, 1e-6)
    assert np.array_equal(flags[clear], CL.element_flags(pvo)[clear])
    frac = flags.mean()
    _say(f"viscous fraction {frac:.3f} (geometric mask {w.flag.mean():.3f})")
    assert 0.02 < frac < 0.6
