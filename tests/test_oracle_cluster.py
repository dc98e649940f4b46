"""Pins for the clustering oracle (Sec. 2.1: velocity-gradient invariants,
two-component Gaussian mixture, element means of the memberships).

Each pin uses what the mathematics or an independent implementation fixes:
closed forms of the invariants, their rotation invariance and the identity
Q_S + Q_W = Q of the full gradient, exactness on a linear velocity field,
the library implementation of EM for the same model from the same start,
the EM monotonicity of the likelihood, recovery of well separated clusters,
brute force for the element rule and its tie, and the degenerate case."""
import warnings

import numpy as np
import pytest

from oracle import cluster as CL
from paper_2403_05463_amd import workloads as W
from test_oracle_pins import _interior_box, _params


def test_invariants_closed_forms():
    w = 1.7
    rot = np.array([[0.0, -w, 0.0], [w, 0.0, 0.0], [0.0, 0.0, 0.0]])
    np.testing.assert_allclose(CL.invariants(rot), [0.0, 0.0, w * w], atol=1e-15)
    a, b, c = 0.3, -1.1, 0.5
    np.testing.assert_allclose(CL.invariants(np.diag([a, b, c])), [a * b + b * c + c * a, -a * b * c / 3, 0.0],
                               atol=1e-15)
    # simple shear du/dy = g: S has eigenvalues +-g/2, 0; W rotation rate g/2
    g = 2.0
    sh = np.array([[0.0, g, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    np.testing.assert_allclose(CL.invariants(sh), [-g * g / 4, 0.0, g * g / 4], atol=1e-15)


def test_invariants_identities_random():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((200, 3, 3))
    F = CL.invariants(G)
    # Q of the full gradient splits into the strain and rotation parts
    trG = np.trace(G, axis1=1, axis2=2)
    trG2 = np.einsum("nij,nji->n", G, G)
    np.testing.assert_allclose(F[:, 0] + F[:, 2], 0.5 * (trG ** 2 - trG2), rtol=1e-12, atol=1e-12)
    # R_S from the eigenvalues of the symmetric part
    lam = np.linalg.eigvalsh(0.5 * (G + G.transpose(0, 2, 1)))
    np.testing.assert_allclose(F[:, 1], -lam.prod(axis=1) / 3, rtol=1e-11, atol=1e-12)
    # Q_W = |omega|^2 / 4 with the vorticity omega = curl u
    om = np.stack([G[:, 2, 1] - G[:, 1, 2], G[:, 0, 2] - G[:, 2, 0], G[:, 1, 0] - G[:, 0, 1]], axis=1)
    np.testing.assert_allclose(F[:, 2], (om ** 2).sum(axis=1) / 4, rtol=1e-12)
    # invariance under a change of frame G -> Q G Q^T
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    np.testing.assert_allclose(CL.invariants(Q @ G @ Q.T), F, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("P", [3, 4])
def test_node_features_exact_on_linear_field(orc, P):
    """u = u0 + G x: the BR1 gradient is G on interior elements, so the node
    features are the invariants of G there."""
    m, ec = _interior_box(P)
    flag = np.zeros(m.n_elem, np.uint8)      # the features do not depend on the flags
    om = orc.OracleMesh(m, P, flag)
    X = om.node_coords()
    rng = np.random.default_rng(40 + P)
    u0, G = rng.standard_normal(3), rng.standard_normal((3, 3))
    x = X.transpose(0, 2, 1)
    q = np.empty((m.n_elem, 4, (P + 1) ** 3))
    q[:, 0] = rng.standard_normal()
    q[:, 1:] = (u0[None, None] + x @ G.T).transpose(0, 2, 1)
    F = CL.node_features(om, _params(orc, nu=0.01), q)
    n3 = (P + 1) ** 3
    expect = CL.invariants(G)
    np.testing.assert_allclose(F[:, ec * n3:(ec + 1) * n3].T, np.broadcast_to(expect, (n3, 3)), atol=1e-11)
    assert np.array_equal(om.flag, flag)


def _two_blobs(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    B = rng.standard_normal((3, 3)) * 0.3
    x0 = rng.standard_normal((int(0.7 * n), 3)) @ A.T
    x1 = rng.standard_normal((n - len(x0), 3)) @ B.T + np.array([1.0, -2.0, 4.0])
    return np.concatenate([x0, x1]).T.copy(), A @ A.T, B @ B.T


def test_em_matches_library_implementation():
    from sklearn.mixture import GaussianMixture
    X, _, _ = _two_blobs(3000, 5)
    m, v = X.mean(axis=1), X.var(axis=1)
    sq = np.sqrt((v[0] + v[2]) / 2)
    s = np.array([sq, sq ** 1.5, sq])
    Xs = ((X - m[:, None]) / s[:, None]).T
    R0 = np.zeros((Xs.shape[0], 2))
    R0[:, 1] = Xs[:, 2] > 0.0
    R0[:, 0] = 1.0 - R0[:, 1]
    nk = R0.sum(axis=0)
    mu0 = R0.T @ Xs / nk[:, None]
    cov0 = np.stack([(R0[:, k, None] * (Xs - mu0[k])).T @ (Xs - mu0[k]) / nk[k] + 1e-6 * np.eye(3) for k in range(2)])
    for iters in (1, 7, 40):
        f = CL.fit_gmm(X, iters, 1e-6)
        gm = GaussianMixture(2, covariance_type="full", reg_covar=1e-6, max_iter=iters, tol=0.0,
                             weights_init=nk / nk.sum(), means_init=mu0, precisions_init=np.linalg.inv(cov0))
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            gm.fit(Xs)
        v = 0 if gm.means_[0, 2] > gm.means_[1, 2] else 1
        order = [1 - v, v]
        np.testing.assert_allclose(f.mixture.weight, gm.weights_[order], rtol=1e-9)
        np.testing.assert_allclose(f.mixture.mean, gm.means_[order], rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(f.mixture.cov, gm.covariances_[order], rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(f.p_visc, gm.predict_proba(Xs)[:, v], atol=1e-9)
        np.testing.assert_allclose(f.feat_mean, m, rtol=1e-14)
        np.testing.assert_allclose(f.feat_std, s, rtol=1e-14)


def test_scaling_is_unit_free_and_keeps_vanishing_features_small():
    """Velocity gradients scaled by c: Q invariants by c^2, R_S by c^3; the
    fit is the same.  A planar flow has R_S = 0 identically: its round-off
    must not be scaled up to unit spread."""
    X, _, _ = _two_blobs(3000, 8)
    X[0] = -np.abs(X[0])
    c = 37.0
    Xc = X * np.array([c * c, c ** 3, c * c])[:, None]
    a, b = CL.fit_gmm(X, 20, 1e-6), CL.fit_gmm(Xc, 20, 1e-6)
    np.testing.assert_allclose(a.p_visc, b.p_visc, atol=1e-9)
    np.testing.assert_allclose(a.mixture.cov, b.mixture.cov, rtol=1e-8, atol=1e-10)
    X[1] = 1e-28 * np.random.default_rng(0).standard_normal(X.shape[1])
    f = CL.fit_gmm(X, 5, 1e-6)
    assert np.abs((X[1] - f.feat_mean[1]) / f.feat_std[1]).max() < 1e-20


def test_em_tolerance_stop_matches_library():
    """With a tolerance, the fit stops at the same iteration as the library's
    EM with the same convergence test."""
    from sklearn.mixture import GaussianMixture
    X, _, _ = _two_blobs(2500, 9)
    X[2] += 0.3 * X[0] ** 2
    f0 = CL.fit_gmm(X, 0, 1e-6)
    Xs = ((X - f0.feat_mean[:, None]) / f0.feat_std[:, None]).T
    R0 = np.zeros((Xs.shape[0], 2))
    R0[:, 1] = Xs[:, 2] > 0.0
    R0[:, 0] = 1.0 - R0[:, 1]
    nk = R0.sum(axis=0)
    mu0 = R0.T @ Xs / nk[:, None]
    cov0 = np.stack([(R0[:, k, None] * (Xs - mu0[k])).T @ (Xs - mu0[k]) / nk[k] + 1e-6 * np.eye(3) for k in range(2)])
    for tol in (1e-2, 1e-5):
        f = CL.fit_gmm(X, 500, 1e-6, tol)
        gm = GaussianMixture(2, covariance_type="full", reg_covar=1e-6, max_iter=500, tol=tol,
                             weights_init=nk / nk.sum(), means_init=mu0, precisions_init=np.linalg.inv(cov0))
        gm.fit(Xs)
        assert gm.converged_ and gm.n_iter_ == len(f.history) < 500
        v = 0 if gm.means_[0, 2] > gm.means_[1, 2] else 1
        np.testing.assert_allclose(f.mixture.mean, gm.means_[[1 - v, v]], rtol=1e-9, atol=1e-10)


def test_em_likelihood_never_decreases():
    X, _, _ = _two_blobs(2000, 11)
    X[2] += 0.5 * X[0] ** 2           # not Gaussian: EM still climbs
    f = CL.fit_gmm(X, 60, 1e-6)
    h = np.array(f.history)
    assert np.all(np.diff(h) >= -1e-12 * np.abs(h[1:]))
    assert h[-1] > h[0]


def test_recovers_well_separated_clusters():
    X, CA, CB = _two_blobs(40000, 21)
    f = CL.fit_gmm(X, 100, 1e-9)
    s = f.feat_std
    # the second blob has the larger third feature: the "viscous" component
    mean_v = f.mixture.mean[1] * s + f.feat_mean
    np.testing.assert_allclose(mean_v, [1.0, -2.0, 4.0], atol=0.03)
    cov_v = f.mixture.cov[1] * np.outer(s, s)
    np.testing.assert_allclose(cov_v, CB, atol=0.05 * np.abs(CB).max())
    np.testing.assert_allclose(f.mixture.weight, [0.7, 0.3], atol=0.01)
    truth = np.r_[np.zeros(28000), np.ones(12000)]
    assert np.mean((f.p_visc > 0.5) == truth) > 0.99


def test_element_means_and_tie_rule():
    Ps = np.array([1, 1, 2, 1])
    n3 = (Ps + 1) ** 3
    off = np.r_[0, np.cumsum(n3)[:-1]]
    p = np.zeros(n3.sum())
    p[0:8] = 0.9                       # viscous
    p[8:16] = [0.5] * 8                # tie -> viscous
    p[16:16 + 27] = np.r_[np.ones(13), np.zeros(14)]   # 13/27 < 1/2 -> inviscid
    p[43:51] = [1, 1, 1, 1, 0, 0, 0, 0.01]             # 4.01/8 > 1/2 -> viscous
    pm = CL.element_means(p, off, Ps)
    np.testing.assert_allclose(pm, [0.9, 0.5, 13 / 27, 4.01 / 8])
    assert CL.element_flags(pm).tolist() == [1, 1, 0, 1]


def test_fluid_at_rest_has_no_viscous_region(orc):
    """Zero velocity: every gradient and feature is exactly zero, Q_W is
    constant and there is no second region."""
    m = W.periodic_box(3, Pg=1, curve_amp=0.2)
    om = orc.OracleMesh(m, 3, np.zeros(m.n_elem, np.uint8))
    q = np.zeros((m.n_elem, 4, 64))
    q[:, 0] = np.linspace(0.0, 1.0, m.n_elem)[:, None]
    X, f, pv, flags = CL.cluster(om, _params(orc, nu=0.01), q, 20)
    assert np.all(X == 0.0)
    assert f.degenerate and not flags.any() and np.all(pv == 0.0)


def test_shear_layer_is_found(orc):
    """A jet u = exp(-((y - pi)/d)^2) in a periodic box: elements in the
    shear layers go viscous, elements far from the jet stay inviscid."""
    n, P, d = 8, 3, 0.5
    m = W.periodic_box(n, Pg=1)
    om = orc.OracleMesh(m, P, np.zeros(m.n_elem, np.uint8))
    X = om.node_coords()
    q = np.zeros((m.n_elem, 4, (P + 1) ** 3))
    y = X[:, 1]
    q[:, 1] = np.exp(-((y - np.pi) / d) ** 2)
    _, f, pv, flags = CL.cluster(om, _params(orc, nu=0.01), q, 50)
    yc = y.mean(axis=1)
    near = np.abs(np.abs(yc - np.pi) - d / np.sqrt(2)) < 0.4     # the shear is largest there
    far = np.abs(yc - np.pi) > 2.2
    assert flags[near].all()
    assert not flags[far].any()
