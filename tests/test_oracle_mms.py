"""Order of accuracy of the whole oracle scheme on manufactured solutions.

The semi-discrete hybrid DGSEM (App. B: collocated Gauss-Lobatto spectral
elements, Roe + BR1 face fluxes; Sec. 2.3: low-storage RK3 in time) should
converge at the design order P + 1 for smooth solutions.  Each case takes a
smooth periodic field q_ex(x, t), derives the source term
S = dq_ex/dt + div F(q_ex) symbolically (sympy), integrates
dq/dt = R_oracle(q) + S(x, t) from the interpolant of q_ex(0) with the
three-stage low-storage RK (stage times 0, 1/3, 3/4) to T, and measures the
mass-weighted L2 error against q_ex(T) on two meshes, n^3 and (2n)^3
elements.  The time step comes from the finer mesh and is used on both, so
the time error is far below the space error (halving it changes no digit).

Asserted: the observed slope log2(e_n / e_2n) >= P + 1/2 (design order P + 1).
A mistake in any term of the scheme (a dropped or doubled flux term, a wrong
sign, the eddy viscosity entering as nu + nu_t instead of 2 (nu + nu_t) in the
stress) leaves an O(1) or O(h^2) inconsistency, and the slope collapses.

Regimes.  The fields have amplitude 0.01 (0.05 with the eddy viscosity), so
convection is weakly nonlinear: with amplitude 0.5 the collocated quadratic
flux (aliasing, App. B's collocated quadrature) holds the slope near P + 0.3 on
these meshes, and only the linear regime reaches the asymptotic order with
meshes a CPU test can afford.  The convective terms themselves are pinned
exactly by the polynomial-exactness tests.  Viscosity 0.002 keeps the cases
convection dominated (BR1's diffusion-dominated order is about P + 1/2).
The eddy-viscosity case uses an ABC (Beltrami) velocity with coefficients
(1, 1, 2): its strain rate S never vanishes (|A^2 - C^2| > B^2), so the
Smagorinsky viscosity (C_s Delta)^2 sqrt(2 S:S) is smooth.
"""
import math

import numpy as np
import pytest

sp = pytest.importorskip("sympy")

from paper_2403_05463_amd import workloads as W

X3 = sp.symbols("x y z", real=True)


def _fields(kind, amp):
    x, y, z = X3
    if kind == "abc":
        U = [amp * (sp.sin(z) + 2 * sp.cos(y)), amp * (sp.sin(x) + sp.cos(z)), amp * (2 * sp.sin(y) + sp.cos(x))]
    else:   # a general field with div U != 0, every velocity gradient entry non-zero
        U = [amp * (sp.sin(y) + sp.cos(z) / 2 + sp.sin(x) / 4),
             amp * (sp.cos(x) + sp.sin(z) / 2 + sp.cos(y) / 3),
             amp * (sp.sin(x) / 2 + sp.cos(y) / 3 + sp.cos(z) / 5)]
    Pa = amp * sp.cos(x) * sp.sin(y) / 2
    Pb = amp * sp.sin(z) / 3
    return U, Pa, Pb


# q_ex(x, t) = (Pa(x) + h(t) Pb(x), g(t) U(x)), g > 0
def _g(t): return 1.0 + 0.1 * math.sin(t)
def _gp(t): return 0.1 * math.cos(t)
def _h(t): return math.sin(t)
def _hp(t): return math.cos(t)


def _source_terms(U, Pa, Pb, c0sq, nu, C_les, delta):
    """S = dq/dt + div(f_c - f_v) for q_ex, split by time factor:
    S = S_1 + g S_g + g^2 S_gg + g' S_g' + h S_h + h' S_h'.  The viscous flux
    2 (nu + nu_t) sym(grad u) with the Smagorinsky nu_t = (C Delta)^2 sqrt(2 S:S)
    scales as g (nu part) and g^2 (nu_t part, since g > 0)."""
    G = [[sp.diff(U[r], X3[d]) for d in range(3)] for r in range(3)]
    S = [[(G[r][d] + G[d][r]) / 2 for d in range(3)] for r in range(3)]
    nut = 0
    if C_les:
        nut = (C_les * delta) ** 2 * sp.sqrt(2 * sum(S[r][d] ** 2 for r in range(3) for d in range(3)))
    T = {k: [sp.Integer(0)] * 4 for k in ("1", "g", "gg", "gp", "h", "hp")}
    T["g"][0] = c0sq * sum(G[d][d] for d in range(3))
    T["hp"][0] = Pb
    for r in range(3):
        T["gp"][1 + r] = U[r]
        T["1"][1 + r] = sp.diff(Pa, X3[r])
        T["h"][1 + r] = sp.diff(Pb, X3[r])
        conv = visc = les = 0
        for d in range(3):
            conv += sp.diff(U[r] * U[d], X3[d])
            visc += sp.diff(2 * nu * S[r][d], X3[d])
            les += sp.diff(2 * nut * S[r][d], X3[d])
        T["g"][1 + r] = -visc
        T["gg"][1 + r] = conv - les
    return T


def _on_nodes(exprs, X):
    f = sp.lambdify(X3, exprs, "numpy")
    vals = f(X[:, 0], X[:, 1], X[:, 2])
    return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), X[:, 0].shape) for v in vals], axis=1)


def _mms_error(orc, *, kind, viscous, P, n, T, dt, c0sq, nu, amp, curved, C_les=0.0):
    m = W.periodic_box(n, Pg=2 if curved else 1, curve_amp=0.25 if curved else 0.0)
    om = orc.OracleMesh(m, P, np.full(m.n_elem, 1 if viscous else 0, np.uint8))
    X = om.node_coords()
    U, Pa, Pb = _fields(kind, amp)
    delta = om.filter_width(0) if C_les else None
    if C_les:
        # the source uses one filter width: every element of the box has it
        assert all(abs(om.filter_width(e) - delta) < 1e-14 for e in range(m.n_elem))
    terms = {k: _on_nodes(v, X) for k, v in _source_terms(U, Pa, Pb, c0sq, nu if viscous else 0.0,
                                                           C_les, delta).items()}
    Ux = _on_nodes(U, X)
    Pax, Pbx = _on_nodes([Pa], X)[:, 0], _on_nodes([Pb], X)[:, 0]

    def q_ex(t):
        q = np.empty((m.n_elem, 4, X.shape[2]))
        q[:, 0] = Pax + _h(t) * Pbx
        q[:, 1:] = _g(t) * Ux
        return q

    def src(t):
        g = _g(t)
        return (terms["1"] + g * terms["g"] + g * g * terms["gg"] + _gp(t) * terms["gp"]
                + _h(t) * terms["h"] + _hp(t) * terms["hp"])

    prm = orc.make_params(c0sq=c0sq, nu=nu if viscous else 0.0, les_model=1 if C_les else 0, C_les=C_les)
    nsteps = int(math.ceil(T / dt - 1e-9))
    dt = T / nsteps
    # Williamson's low-storage RK3 (Sec. 2.3), with the source at the stage times
    A, B, c = (0.0, -5.0 / 9.0, -153.0 / 128.0), (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0), (0.0, 1.0 / 3.0, 0.75)
    q, dq, t = q_ex(0.0), None, 0.0
    for _ in range(nsteps):
        for s in range(3):
            rhs = om.residual(prm, q) + src(t + c[s] * dt)
            dq = dt * rhs if s == 0 else A[s] * dq + dt * rhs
            q = q + B[s] * dq
        t += dt
    J, _ = om.metrics()
    _, w, _ = orc.lgl(P)
    mass = J * np.einsum("k,j,i->kji", w, w, w).ravel()[None]
    e = q - q_ex(T)
    return math.sqrt((mass[:, None] * e * e).sum() / mass.sum())


def _slope(orc, P, n, amp, **kw):
    c0sq = 1.0
    lam = 3.5 * amp + math.sqrt((3.5 * amp) ** 2 + c0sq)       # bound on |u_n| + sqrt(u_n^2 + c0^2)
    dt = 0.5 * (2 * math.pi / (2 * n)) / ((P + 1) ** 2 * lam)
    e1 = _mms_error(orc, P=P, n=n, T=0.5, dt=dt, c0sq=c0sq, amp=amp, **kw)
    e2 = _mms_error(orc, P=P, n=2 * n, T=0.5, dt=dt, c0sq=c0sq, amp=amp, **kw)
    return e1, e2, math.log2(e1 / e2)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("viscous", [False, True], ids=["euler", "navier_stokes"])
@pytest.mark.parametrize("curved", [False, True], ids=["cartesian", "curved"])
def test_design_order_on_manufactured_solution(orc, P, viscous, curved):
    e1, e2, rate = _slope(orc, P, 6, 0.01, kind="gen", viscous=viscous, nu=0.002, curved=curved)
    print(f"P={P} viscous={viscous} curved={curved}: L2 errors {e1:.3e} (6^3), {e2:.3e} (12^3), slope {rate:.2f}")
    assert rate >= P + 0.5, (e1, e2, rate)


def test_design_order_with_smagorinsky_eddy_viscosity(orc):
    """Pure LES (nu = 0, C_s = 0.5): the eddy viscosity is the only viscous
    term, and it is exact in the source per mesh (filter width of that mesh)."""
    e1, e2, rate = _slope(orc, 3, 6, 0.05, kind="abc", viscous=True, nu=0.0, curved=False, C_les=0.5)
    print(f"LES P=3: L2 errors {e1:.3e} (6^3), {e2:.3e} (12^3), slope {rate:.2f}")
    assert rate >= 3.5, (e1, e2, rate)


def test_abc_strain_rate_never_vanishes():
    """The premise of the eddy-viscosity case: for ABC coefficients (A, B, C) =
    (1, 1, 2), S:S > 0 everywhere (on a fine grid, min S:S well above zero)."""
    U, _, _ = _fields("abc", 1.0)
    G = [[sp.diff(U[r], X3[d]) for d in range(3)] for r in range(3)]
    ss = sum(((G[r][d] + G[d][r]) / 2) ** 2 for r in range(3) for d in range(3))
    f = sp.lambdify(X3, ss, "numpy")
    s = np.linspace(0, 2 * np.pi, 61)
    x, y, z = np.meshgrid(s, s, s, indexing="ij")
    assert f(x, y, z).min() > 0.1
