"""Pins of the oracle's coupling of elements of different order (mortar
faces): free stream, discrete conservation, polynomial exactness across the
mortar from both sides, and orientation invariance; on curved (quadratic and
cubic) geometry, one face normal on both sides of every such face."""
import math

import numpy as np
import pytest

from paper_2403_05463_amd import workloads as W

C0SQ = 25.0


def _params(orc, **kw):
    base = dict(c0sq=C0SQ, nu=1e-2, les_model=1, C_les=0.1, mixed_face=0, q_inf=(0, 0, 0, 0))
    base.update(kw)
    return orc.make_params(**base)


def _flat(om, fields, fn):
    """Flat array element after element: fn(e, n3) -> (fields, n3)."""
    out = np.empty(fields * om.nodes)
    for e in range(om.n_elem):
        n3 = (int(om.Ps[e]) + 1) ** 3
        o = fields * int(om.offsets[e])
        out[o:o + fields * n3] = np.asarray(fn(e, n3)).reshape(-1)
    return out


def _mass(orc, om):
    J, _ = om.metrics()
    out = np.empty(om.nodes)
    for e in range(om.n_elem):
        P = int(om.Ps[e])
        _, w, _ = orc.lgl(P)
        n3 = (P + 1) ** 3
        o = int(om.offsets[e])
        out[o:o + n3] = J[o:o + n3] * np.einsum("k,j,i->kji", w, w, w).ravel()
    return out


def _warped_box(seed):
    m = W.periodic_box(3, Pg=1, curve_amp=0.25)
    flag = W.bernoulli_mask(m.n_elem, 0.5, seed)
    P = W.mixed_orders(flag, seed)
    return m, flag, P


def test_mixed_orders_really_mix(orc):
    m, flag, P = _warped_box(1)
    nonconf = sum(1 for e in range(m.n_elem) for f in range(6)
                  if m.nbr[e, f] >= 0 and P[m.nbr[e, f]] != P[e])
    assert nonconf > m.n_elem            # most elements have a mortar face
    assert P[flag == 1].mean() > P[flag == 0].mean()


def test_mortar_rejects_orders_below_the_geometry(orc):
    m = W.periodic_box(3, Pg=3, curve_amp=0.15)
    P = np.full(m.n_elem, 2, dtype=np.int32)
    P[0] = 4
    with pytest.raises(ValueError):
        orc.OracleMesh(m, P, np.zeros(m.n_elem, np.uint8))
    m1 = W.periodic_box(3, Pg=1, curve_amp=0.2)
    P1 = np.full(m1.n_elem, 1, dtype=np.int32)
    P1[0] = 3
    with pytest.raises(ValueError):
        orc.OracleMesh(m1, P1, np.zeros(m1.n_elem, np.uint8))


@pytest.mark.parametrize("les", [1, 2])
@pytest.mark.parametrize("seed", [1, 2])
def test_mortar_freestream(orc, les, seed):
    m, flag, P = _warped_box(seed)
    om = orc.OracleMesh(m, P, flag)
    qc = np.array([0.3, 1.0, -0.5, 0.2])
    q = _flat(om, 4, lambda e, n3: np.repeat(qc[:, None], n3, axis=1))
    R = om.residual(_params(orc, les_model=les, C_les=0.1 if les == 1 else 0.07), q)
    scale = C0SQ * 1.2 / (2 * math.pi / 3)
    assert np.abs(R).max() < 1e-10 * scale


@pytest.mark.parametrize("riemann", [0, 1])
@pytest.mark.parametrize("mixed_face", [0, 1])
def test_mortar_discrete_conservation(orc, mixed_face, riemann):
    m, flag, P = _warped_box(3)
    om = orc.OracleMesh(m, P, flag)
    rng = np.random.default_rng(4)
    q = rng.uniform(-1, 1, size=4 * om.nodes)
    R = om.residual(_params(orc, mixed_face=mixed_face, riemann=riemann), q)
    WJ = _mass(orc, om)
    for f in range(4):
        Rf = np.concatenate([om.element(R, e, 4)[f] for e in range(om.n_elem)])
        tot = (WJ * Rf).sum()
        mag = np.abs(WJ * Rf).sum()
        assert abs(tot) < 1e-13 * mag, (f, tot, mag)


def _interior_orders(center, seed, lo, hi):
    rng = np.random.default_rng(seed)
    P = rng.integers(lo, hi + 1, size=27).astype(np.int32)
    P[13] = center
    # make sure the centre has both higher- and lower-order face neighbours
    P[12], P[14] = center + 1, center - 1
    return P


@pytest.mark.parametrize("center", [4, 5])
def test_mortar_polynomial_exactness_euler_linear_state(orc, center):
    """Linear state (quadratic flux): the centre element of a 3^3 box with
    neighbours of higher and lower order gets the exact -div f at its nodes
    (a flux of degree d < P is reproduced through the mortar from both sides)."""
    m = W.box((3, 3, 3), lo=(-1.2, -0.9, -1.0), hi=(1.3, 1.0, 0.8), Pg=1, skew=0.3)
    P = _interior_orders(center, center, 3, 6)
    om = orc.OracleMesh(m, P, np.zeros(m.n_elem, np.uint8))
    X = om.node_coords()
    rng = np.random.default_rng(center)
    p0, gp = rng.standard_normal(), rng.standard_normal(3)
    u0, G = rng.standard_normal(3), rng.standard_normal((3, 3))

    def state(e, n3):
        x = om.element(X, e, 3).T
        return np.vstack([p0 + x @ gp, (u0[None] + x @ G.T).T])
    q = _flat(om, 4, state)
    R = om.residual(_params(orc, q_inf=(0.2, 0.1, 0.0, 0.3)), q)
    xe = om.element(X, 13, 3).T
    u = u0[None] + xe @ G.T
    tr = np.trace(G)
    Re = om.element(R, 13, 4)
    np.testing.assert_allclose(Re[0], -C0SQ * tr * np.ones(xe.shape[0]), atol=1e-11 * C0SQ)
    np.testing.assert_allclose(Re[1:].T, -(u @ G.T) - u * tr - gp[None], atol=1e-11 * C0SQ)


def test_mortar_polynomial_exactness_viscous_quadratic_state(orc):
    """All-viscous, quadratic velocity, LES off: the centre element gets
    -div f_c + nu (lap u + grad div u) exactly through mortars on both sides
    (BR1 lift and viscous traces extended and integrated on the mortar)."""
    m = W.box((3, 3, 3), lo=(-1.2, -0.9, -1.0), hi=(1.3, 1.0, 0.8), Pg=1, skew=0.3)
    P = _interior_orders(6, 2, 5, 7)
    om = orc.OracleMesh(m, P, np.ones(m.n_elem, np.uint8))
    X = om.node_coords()
    rng = np.random.default_rng(12)
    p0, gp = rng.standard_normal(), rng.standard_normal(3)
    u0, G = rng.standard_normal(3), rng.standard_normal((3, 3))
    H = rng.standard_normal((3, 3, 3))
    H = 0.5 * (H + H.transpose(0, 2, 1))

    def vel(x):
        return u0[None] + x @ G.T + 0.5 * np.einsum("ni,rij,nj->nr", x, H, x)

    def state(e, n3):
        x = om.element(X, e, 3).T
        return np.vstack([p0 + x @ gp, vel(x).T])
    q = _flat(om, 4, state)
    nu = 0.05
    R = om.residual(_params(orc, nu=nu, les_model=0, C_les=0.0), q)
    xe = om.element(X, 13, 3).T
    ue = vel(xe)
    grad = G[None] + np.einsum("rij,nj->nri", H, xe)
    div = np.einsum("nrr->n", grad)
    conv = np.einsum("nrd,nd->nr", grad, ue) + ue * div[:, None]
    lap = np.einsum("rii->r", H)
    graddiv = np.einsum("ddr->r", H)
    Re = om.element(R, 13, 4)
    np.testing.assert_allclose(Re[0], -C0SQ * div, atol=1e-10 * C0SQ)
    np.testing.assert_allclose(Re[1:].T, -conv - gp[None] + nu * (lap + graddiv)[None], atol=1e-10 * C0SQ)


def test_mortar_orientation_invariance(orc):
    base, flag, P = _warped_box(5)
    om0 = orc.OracleMesh(base, P, flag)
    X0 = om0.node_coords()
    q0 = _flat(om0, 4, lambda e, n3: W.taylor_green_state(om0.element(X0, e, 3)[None], 0.05, e)[0])
    prm = _params(orc, les_model=2, C_les=0.07)
    R0 = om0.residual(prm, q0)
    m1, frames = W.reorient(base, seed=23)
    om1 = orc.OracleMesh(m1, P, flag)
    maps = [W.index_map(perm, flips, int(P[e])) for e, (perm, flips) in enumerate(frames)]
    q1 = np.empty_like(q0)
    for e, mp in enumerate(maps):
        om1.element(q1, e, 4)[:, mp] = om0.element(q0, e, 4)
    R1 = om1.residual(prm, q1)
    err = 0.0
    for e, mp in enumerate(maps):
        err = max(err, np.abs(om1.element(R1, e, 4)[:, mp] - om0.element(R0, e, 4)).max())
    assert err < 1e-12 * np.abs(R0).max()


def _lagrange_matrix(x_from, x_to):
    """L[i, k] = l_k(x_to[i]) for the Lagrange basis on x_from (product formula)."""
    L = np.ones((len(x_to), len(x_from)))
    for k, xk in enumerate(x_from):
        for j, xj in enumerate(x_from):
            if j != k:
                L[:, k] *= (x_to - xj) / (xk - xj)
    return L


@pytest.mark.parametrize("viscous", [False, True])
def test_mortar_equals_conforming_face_after_raising_the_order(orc, viscous):
    """A degree-3 neighbour raised exactly to degree 5 (its field interpolated
    to the order-5 nodes) turns the mortar into a conforming face; the
    order-5 element on the other side must then see the same numerical flux
    and the same BR1 mean u*, so its residual (Euler) and its gradient
    (viscous) do not change."""
    m = W.periodic_box(3, Pg=1, curve_amp=0.25)
    A = 13
    B = int(m.nbr[A, 1])
    Pm = np.full(m.n_elem, 5, dtype=np.int32)
    Pm[B] = 3
    flag = np.full(m.n_elem, 1 if viscous else 0, dtype=np.uint8)
    om_m = orc.OracleMesh(m, Pm, flag)
    om_c = orc.OracleMesh(m, 5, flag)
    Xm = om_m.node_coords()
    rng = np.random.default_rng(8)
    # a different smooth field per element: traces jump across every face
    q_m = _flat(om_m, 4, lambda e, n3: W.taylor_green_state(om_m.element(Xm, e, 3)[None], 0.0, 0)[0]
                * (1.0 + 0.3 * rng.standard_normal()) + 0.1 * rng.standard_normal((4, 1)))
    q_c = np.empty((m.n_elem, 4, 216))
    x3, _, _ = orc.lgl(3)
    x5, _, _ = orc.lgl(5)
    I = _lagrange_matrix(x3, x5)
    for e in range(m.n_elem):
        blk = om_m.element(q_m, e, 4)
        if e == B:
            b3 = blk.reshape(4, 4, 4, 4)                         # [f][k][j][i]
            q_c[e] = np.einsum("ai,bj,ck,fkji->fcba", I, I, I, b3).reshape(4, 216)
        else:
            q_c[e] = blk
    prm = _params(orc, nu=0.02, les_model=0, C_les=0.0)
    if viscous:
        Gm = om_m.gradient(prm, q_m)
        Gc = om_c.gradient(prm, q_c)
        ga, gb = om_m.element(Gm, A, 9), Gc[A].reshape(9, -1)
        assert np.abs(ga - gb).max() < 1e-12 * np.abs(gb).max()
    else:
        Rm = om_m.residual(prm, q_m)
        Rc = om_c.residual(prm, q_c)
        ra, rb = om_m.element(Rm, A, 4), Rc[A]
        assert np.abs(ra - rb).max() < 1e-12 * np.abs(rb).max()


# --- curved faces between orders -------------------------------------------
#
# Curl-form metric terms of a degree-Pg map have degree 2 Pg - 1 per face
# direction, more than a low-order side represents.  The oracle restricts the
# curl-form product field on faces and edges where orders meet so that both
# sides carry one face normal of degree <= P_lo - 1 per direction (reading in
# the oracle's header of that code).  These pins check that reading's purpose
# directly (one normal, of that degree) and its consequences (free stream and
# conservation through curved mortars).


def _curved_mixed_box(Pg, seed):
    m = W.periodic_box(3, Pg=Pg, curve_amp=0.2 if Pg == 2 else 0.15)
    flag = W.bernoulli_mask(m.n_elem, 0.5, seed)
    P = np.maximum(W.mixed_orders(flag, seed), Pg).astype(np.int32)
    return m, flag, P


@pytest.mark.parametrize("Pg", [2, 3])
@pytest.mark.parametrize("les", [0, 1, 2])
def test_curved_mortar_freestream(orc, Pg, les):
    m, flag, P = _curved_mixed_box(Pg, 1 + les)
    assert len(set(P.tolist())) >= 3
    om = orc.OracleMesh(m, P, flag)
    qc = np.array([0.3, 1.0, -0.5, 0.2])
    q = _flat(om, 4, lambda e, n3: np.repeat(qc[:, None], n3, axis=1))
    R = om.residual(_params(orc, les_model=les, C_les=0.07 if les == 2 else 0.1), q)
    scale = C0SQ * 1.2 / (2 * math.pi / 3)
    assert np.abs(R).max() < 1e-11 * scale
    G = om.gradient(_params(orc), q)
    assert np.abs(np.concatenate([om.element(G, e, 9).ravel() for e in range(m.n_elem) if flag[e]])).max() < 1e-11


@pytest.mark.parametrize("Pg", [2, 3])
@pytest.mark.parametrize("mixed_face", [0, 1])
def test_curved_mortar_discrete_conservation(orc, Pg, mixed_face):
    m, flag, P = _curved_mixed_box(Pg, 7)
    om = orc.OracleMesh(m, P, flag)
    rng = np.random.default_rng(9)
    q = rng.uniform(-1, 1, size=4 * om.nodes)
    R = om.residual(_params(orc, mixed_face=mixed_face), q)
    WJ = _mass(orc, om)
    for f in range(4):
        Rf = np.concatenate([om.element(R, e, 4)[f] for e in range(om.n_elem)])
        tot = (WJ * Rf).sum()
        mag = np.abs(WJ * Rf).sum()
        assert abs(tot) < 1e-13 * mag, (f, tot, mag)


def _face_normals(om, Ja, e, f):
    """Element e's outward s n at the nodes of its local face f: [a][b][3],
    (a, b) the face-local indices (the two other reference directions in
    increasing order)."""
    N = int(om.Ps[e]) + 1
    A = om.element(Ja, e, 9).reshape(3, 3, N, N, N)[f // 2]      # [d][c][b][a]
    s = (f & 1) * (N - 1)
    d = f // 2
    F = A[:, :, :, s] if d == 0 else A[:, :, s, :] if d == 1 else A[:, s]
    return (1.0 if f & 1 else -1.0) * np.transpose(F, (2, 1, 0))


def _orient_map(o, M, a, b):
    s, t = (b, a) if o & 1 else (a, b)
    return (M - s if o & 2 else s), (M - t if o & 4 else t)


@pytest.mark.parametrize("Pg", [2, 3])
def test_curved_mortar_one_face_normal(orc, Pg):
    """On every face between orders the lower side's s n is a polynomial of
    degree <= P_lo - 1 per face direction, and the higher side's s n at its
    own face nodes is the same polynomial, with the opposite sign."""
    m, flag, P = _curved_mixed_box(Pg, 11)
    om = orc.OracleMesh(m, P, flag)
    _, Ja = om.metrics()
    checked = 0
    worst_deg = worst_match = 0.0
    for e in range(m.n_elem):
        for f in range(6):
            e2 = int(m.nbr[e, f])
            if e2 < 0 or P[e2] >= P[e]:
                continue
            f2 = int(m.nbr_face[e, f])
            M, Nl = int(P[e]) + 1, int(P[e2]) + 1
            xh, _, _ = orc.lgl(M - 1)
            xl, _, _ = orc.lgl(Nl - 1)
            xd, _, _ = orc.lgl(Nl - 2)
            nh = _face_normals(om, Ja, e, f)
            nl = _face_normals(om, Ja, e2, f2)
            scale = np.abs(nl).max()
            # degree <= P_lo - 1: the values at P_lo points reproduce all nodes
            Ld = _lagrange_matrix(xd, xl)
            Ld_back = _lagrange_matrix(xl, xd)
            fit = np.einsum("ai,bj,ijc->abc", Ld, Ld, np.einsum("ia,jb,abc->ijc", Ld_back, Ld_back, nl))
            worst_deg = max(worst_deg, np.abs(fit - nl).max() / scale)
            # the same polynomial seen from the higher side
            L = _lagrange_matrix(xl, xh)
            for j in range(M):
                for i in range(M):
                    il, jl = _orient_map(int(m.orient[e, f]), M - 1, i, j)
                    val = np.einsum("a,b,abc->c", L[il], L[jl], nl)
                    worst_match = max(worst_match, np.abs(nh[i, j] + val).max() / scale)
            checked += 1
    assert checked > m.n_elem
    assert worst_deg < 1e-13, worst_deg
    assert worst_match < 1e-13, worst_match


@pytest.mark.parametrize("Pg", [2, 3])
def test_curved_mortar_metric_identities(orc, Pg):
    """sum_i d(Ja^i)/dxi^i = 0 at every node of every element."""
    m, flag, P = _curved_mixed_box(Pg, 13)
    om = orc.OracleMesh(m, P, flag)
    _, Ja = om.metrics()
    worst = 0.0
    for e in range(m.n_elem):
        N = int(P[e]) + 1
        _, _, D = orc.lgl(N - 1)
        A = om.element(Ja, e, 9).reshape(3, 3, N, N, N)             # [i][d][c][b][a]
        div = (np.einsum("ak,dcbk->dcba", D, A[0]) + np.einsum("bk,dcka->dcba", D, A[1])
               + np.einsum("ck,dkba->dcba", D, A[2]))
        worst = max(worst, np.abs(div).max() / np.abs(A).max())
    assert worst < 1e-13, worst


def test_uniform_order_metrics_are_not_restricted(orc):
    """On a mesh of one order the restriction changes nothing: a single
    element of another order far away leaves every element that shares no
    edge or face with it bitwise as on the uniform mesh."""
    m = W.periodic_box(4, Pg=2, curve_amp=0.2)
    P0 = np.full(m.n_elem, 3, dtype=np.int32)
    P1 = P0.copy()
    P1[0] = 5
    om0 = orc.OracleMesh(m, P0, np.zeros(m.n_elem, np.uint8))
    om1 = orc.OracleMesh(m, P1, np.zeros(m.n_elem, np.uint8))
    _, Ja0 = om0.metrics()
    _, Ja1 = om1.metrics()
    near = set(int(v) for v in np.where(np.isin(m.corners, m.corners[0]).any(axis=1))[0])
    same = changed = 0
    for e in range(1, m.n_elem):
        a, b = om0.element(Ja0, e, 9).ravel(), om1.element(Ja1, e, 9).ravel()
        if e in near:
            changed += int(not np.array_equal(a, b))
        else:
            assert np.array_equal(a, b), e
            same += 1
    assert same > 0 and changed > 0
