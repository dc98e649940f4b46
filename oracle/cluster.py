"""FP64 oracle of the clustering that produces the equation flag (Sec. 2.1).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product package never imports it and it
shares no code with the HIP library.

Steps, in the order the method takes them:

1. node features (Sec. 2.1): from the velocity gradient J = grad U at every
   node, the strain rate S = (J + J^T)/2 and rotation rate W = (J - J^T)/2,
   and their invariants
       Q_S = (tr(S)^2 - tr(S^2)) / 2,  R_S = -det(S) / 3,  Q_W = -tr(W^2) / 2;
   J is the BR1 lifted gradient of the discretisation (the one the viscous
   operator uses), evaluated on every element;
2. a two-component Gaussian mixture over the node features gives each node a
   membership p_v of the viscous/rotational region and p_i = 1 - p_v of the
   inviscid one;
3. element means of p_v and p_i over the element's (P + 1)^3 nodes; the
   element takes the region of the larger mean.

Readings where the paper is silent (its text names the model and the
features but not how the mixture is fitted):
  * full covariance matrices, fitted by expectation-maximisation with at
    most a given number of iterations, optionally ending early once the mean
    log-likelihood moves by less than ``tol`` between two E-steps (after
    that iteration's M-step), a ridge ``reg_covar`` added to each covariance
    diagonal, and the component counts guarded by 10 machine epsilons, as in
    the common library implementation of the same model;
  * the features are centred (global means) and scaled by the gradient
    scale of the flow: Q_S and Q_W (units of a squared velocity gradient)
    by s_Q, the pooled population standard deviation of Q_S and Q_W, and R_S
    (a cubed gradient) by s_Q^(3/2); s_Q = 0 (no gradient anywhere) leaves
    them unscaled.  The fit then does not depend on the flow's units, and a
    feature that vanishes identically (R_S in a planar flow) stays at its
    round-off level instead of being blown up to unit spread;
  * initial split: nodes whose Q_W exceeds its mean start in the second
    component, the others in the first (responsibilities 0/1), followed by
    one M-step; without such nodes (a constant Q_W) there is no second
    region and every node gets p_v = 0;
  * the viscous/rotational component is the one with the larger mean Q_W
    after fitting (ties: the second component);
  * an element exactly at p_v mean = p_i mean goes to the viscous region.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

EPS_COUNT = 10.0 * np.finfo(np.float64).eps


def invariants(G):
    """(Q_S, R_S, Q_W) of velocity gradients G[..., r, d] = du_r/dx_d (Sec. 2.1)."""
    G = np.asarray(G, dtype=np.float64)
    Gt = np.swapaxes(G, -1, -2)
    S = 0.5 * (G + Gt)
    W = 0.5 * (G - Gt)
    trS = np.trace(S, axis1=-2, axis2=-1)
    trS2 = np.einsum("...ij,...ji->...", S, S)
    trW2 = np.einsum("...ij,...ji->...", W, W)
    QS = 0.5 * (trS * trS - trS2)
    with np.errstate(divide="ignore", invalid="ignore"):   # singular S (no strain) has det 0
        RS = -np.linalg.det(S) / 3.0
    QW = -0.5 * trW2
    return np.stack([QS, RS, QW], axis=-1)


def node_gradients(om, params, q):
    """BR1 gradient at every node, element after element: array [nodes][3][3].
    The oracle mesh computes it on flagged elements, so every element is
    flagged for the call (the gradient does not depend on the flags)."""
    keep = om.flag
    om.set_flags(np.ones(om.n_elem, dtype=np.uint8))
    try:
        G = om.gradient(params, q)
    finally:
        om.set_flags(keep)
    out = np.empty((om.nodes, 3, 3))
    for e in range(om.n_elem):
        n3 = (int(om.Ps[e]) + 1) ** 3
        o = int(om.offsets[e])
        blk = G[e] if om.uniform else G[9 * o:9 * (o + n3)].reshape(3, 3, n3)
        out[o:o + n3] = np.moveaxis(blk, -1, 0)
    return out


def node_features(om, params, q):
    """Features [3][nodes]: Q_S, R_S, Q_W of the BR1 gradient at every node."""
    return np.ascontiguousarray(invariants(node_gradients(om, params, q)).T)


def standardize(X):
    """Feature means and scales of X[3][n] = (Q_S, R_S, Q_W): s_Q for the two
    Q invariants, s_Q^(3/2) for R_S (module notes)."""
    m = X.mean(axis=1)
    v = ((X - m[:, None]) ** 2).mean(axis=1)
    sq = np.sqrt(0.5 * (v[0] + v[2]))
    if not sq > 0.0:
        return m, np.ones(3)
    return m, np.array([sq, sq ** 1.5, sq])


@dataclass
class Mixture:
    weight: np.ndarray        # [2]
    mean: np.ndarray          # [2][3]
    cov: np.ndarray           # [2][3][3]


def m_step(Xs, R, reg_covar):
    """Weights, means and covariances from responsibilities R[n][2] over
    standardised features Xs[n][3]."""
    nk = R.sum(axis=0) + EPS_COUNT
    mean = (R.T @ Xs) / nk[:, None]
    cov = np.empty((2, 3, 3))
    for k in range(2):
        d = Xs - mean[k]
        cov[k] = (R[:, k, None] * d).T @ d / nk[k] + reg_covar * np.eye(3)
    return Mixture(nk / Xs.shape[0], mean, cov)


def log_gauss(Xs, mean, cov):
    """log N(x | mean, cov) per row, through the Cholesky factor of cov."""
    L = np.linalg.cholesky(cov)
    z = np.linalg.solve(L, (Xs - mean).T)
    return -0.5 * (3 * np.log(2.0 * np.pi) + (z * z).sum(axis=0)) - np.log(np.diag(L)).sum()


def e_step(Xs, mix: Mixture):
    """Responsibilities R[n][2] and the mean log-likelihood per node."""
    lw = np.stack([np.log(mix.weight[k]) + log_gauss(Xs, mix.mean[k], mix.cov[k]) for k in range(2)], axis=1)
    top = lw.max(axis=1, keepdims=True)
    lse = top[:, 0] + np.log(np.exp(lw - top).sum(axis=1))
    return np.exp(lw - lse[:, None]), float(lse.mean())


@dataclass
class Fit:
    feat_mean: np.ndarray     # [3]
    feat_std: np.ndarray      # [3]
    mixture: Mixture          # ordered: [0] inviscid, [1] viscous
    p_visc: np.ndarray        # [nodes]
    log_likelihood: float     # mean per node, E-step of the last iteration (nan if none)
    history: list             # mean log-likelihood of every E-step
    degenerate: bool          # no second region


def fit_gmm(X, iterations: int, reg_covar: float = 1e-6, tol: float = 0.0) -> Fit:
    """Two-component mixture over X[3][nodes] (step 2 of the module notes):
    at most ``iterations`` EM iterations, ending after the M-step of one whose
    mean log-likelihood moved by less than ``tol`` from the previous one."""
    X = np.asarray(X, dtype=np.float64)
    m, s = standardize(X)
    Xs = ((X - m[:, None]) / s[:, None]).T
    R = np.zeros((Xs.shape[0], 2))
    R[:, 1] = Xs[:, 2] > 0.0
    R[:, 0] = 1.0 - R[:, 1]
    if R[:, 1].sum() == 0.0 or R[:, 0].sum() == 0.0:
        mix = Mixture(np.array([1.0, 0.0]), np.zeros((2, 3)), np.stack([np.eye(3)] * 2))
        return Fit(m, s, mix, np.zeros(Xs.shape[0]), float("nan"), [], True)
    mix = m_step(Xs, R, reg_covar)
    hist = []
    for _ in range(iterations):
        R, ll = e_step(Xs, mix)
        hist.append(ll)
        mix = m_step(Xs, R, reg_covar)
        if len(hist) > 1 and abs(hist[-1] - hist[-2]) < tol:
            break
    R, _ = e_step(Xs, mix)
    v = 0 if mix.mean[0, 2] > mix.mean[1, 2] else 1
    order = [1 - v, v]
    mix = Mixture(mix.weight[order], mix.mean[order], mix.cov[order])
    return Fit(m, s, mix, R[:, v].copy(), hist[-1] if hist else float("nan"), hist, False)


def element_means(p_visc, offsets, Ps):
    """Mean of p_v over each element's nodes (the element-wise representation of Sec. 2.1)."""
    out = np.empty(len(Ps))
    for e in range(len(Ps)):
        n3 = (int(Ps[e]) + 1) ** 3
        o = int(offsets[e])
        out[e] = p_visc[o:o + n3].mean()
    return out


def element_flags(pv_mean):
    """Region with the larger mean membership, p_i = 1 - p_v; ties go viscous."""
    pv_mean = np.asarray(pv_mean)
    return (pv_mean >= 1.0 - pv_mean).astype(np.uint8)


def cluster(om, params, q, iterations: int, reg_covar: float = 1e-6):
    """Features, fit, element means and flags of state q on oracle mesh om."""
    X = node_features(om, params, q)
    f = fit_gmm(X, iterations, reg_covar)
    pv = element_means(f.p_visc, om.offsets, om.Ps)
    return X, f, pv, element_flags(pv)
