/*
 * FP64 CPU oracle for the hybrid NS-LES / Euler DGSEM residual.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, by the smoke check and by
 * the benchmark's CPU-baseline leg; never by the product path.  Plain loops,
 * double precision, the discretisation written in the weak form the paper
 * states (App. B, the integrated-by-parts element equations with a numerical
 * flux on the element boundary and collocated quadrature).  OpenMP only
 * splits independent elements across threads; every element's arithmetic is
 * the same sequential loop whatever the thread count.
 *
 * Method (paper: Sec. 2.3 and App. A-B), as read here:
 *  - unknowns (p, u, v, w) of the incompressible equations in artificial
 *    compressibility form, dp/dt + c0^2 div u = 0 (unit density);
 *  - every element gets the convective flux (Sec. 2.3); elements flagged
 *    viscous/turbulent also get the viscous + LES flux 2 (nu + nu_t) S
 *    (App. A stress tensor, incompressible, no trace term);
 *  - element coupling through a Roe flux on every face and the BR1
 *    (Bassi-Rebay 1) average of viscous fluxes on faces with a viscous side,
 *    single valued per face (Sec. 2.3 face cases, Sec. 4 remark on a
 *    single-valued viscous flux);
 *  - LES eddy viscosity: Smagorinsky or Vreman (App. A, Vreman equation);
 *  - Gauss-Lobatto-Legendre collocation, curvilinear hexahedra with metric
 *    terms in curl (conservative) form (App. B transformed equation);
 *  - three-stage low-storage RK (Sec. 2.3 time marching), Williamson's
 *    2N-storage coefficients.
 */
#include "hdg_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 9

static char g_err[512];
const char *orc_last_error(void) { return g_err; }

struct orc_mesh {
    int ne;
    int *P;         /* [e] polynomial order */
    size_t *off;    /* [e] first node of element e; element e holds (P_e+1)^3 nodes */
    size_t nodes;   /* total nodes */
    /* GLL rule of every order in use, indexed by N = P + 1 */
    double xi[MAXN + 1][MAXN], w[MAXN + 1][MAXN], D[MAXN + 1][MAXN * MAXN];
    double *x;      /* [e][3][N_e^3] node coordinates */
    double *J;      /* [e][N_e^3] Jacobian */
    double *Ja;     /* [e][3 (i)][3 (d)][N_e^3] contravariant metric Ja^i_d */
    double *delta;  /* [e] LES filter width */
    int *nbr;
    signed char *nbr_face, *orient;
    unsigned char *flag;
};

static int NE(const orc_mesh *m, int e) { return m->P[e] + 1; }
static int N3E(const orc_mesh *m, int e) { int n = m->P[e] + 1; return n * n * n; }

static int g_threads = 0;
void orc_set_threads(int n) { g_threads = n; }
int orc_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Quadrature: Gauss-Lobatto-Legendre nodes/weights, Lagrange derivative.    */
/*                                                                          */
/* The quadrature rule and the element geometry are set-up quantities, not  */
/* part of the residual arithmetic: they are evaluated in x87 extended      */
/* precision and rounded once to double, so that they are the correctly     */
/* rounded values of the quantities they define.                            */
/* ------------------------------------------------------------------------ */

typedef long double xreal;

/* Legendre polynomial L_n and its derivative at x by the three-term recurrence. */
static void legendre(int n, xreal x, xreal *L, xreal *dL)
{
    xreal l0 = 1.0L, l1 = x, d0 = 0.0L, d1 = 1.0L;
    if (n == 0) { *L = 1.0L; *dL = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
        xreal l2 = ((2.0L * k + 1.0L) * x * l1 - k * l0) / (k + 1.0L);
        xreal d2 = d0 + (2.0L * k + 1.0L) * l1;
        l0 = l1; l1 = l2; d0 = d1; d1 = d2;
    }
    *L = l1; *dL = d1;
}

/* l_j'(x_i) for the Lagrange basis on nodes x[0..N-1], from its definition
 * l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m). */
static void lagrange_derivative_matrix(int N, const xreal *x, xreal *D)
{
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            xreal s = 0.0L;
            for (int k = 0; k < N; ++k) {
                if (k == j) continue;
                xreal t = 1.0L / (x[j] - x[k]);
                for (int m = 0; m < N; ++m) {
                    if (m == j || m == k) continue;
                    t *= (x[i] - x[m]) / (x[j] - x[m]);
                }
                s += t;
            }
            D[i * N + j] = s;
        }
}

static xreal lagrange_value(int M1, const xreal *nodes, int k, xreal x)
{
    xreal v = 1.0L;
    for (int m = 0; m < M1; ++m)
        if (m != k) v *= (x - nodes[m]) / (nodes[k] - nodes[m]);
    return v;
}

/* d l_k / dx at x: sum over m != k of 1/(x_k - x_m) times the product of
 * the remaining factors of l_k */
static xreal lagrange_deriv(int M1, const xreal *nodes, int k, xreal x)
{
    xreal s = 0.0L;
    for (int m = 0; m < M1; ++m) {
        if (m == k) continue;
        xreal t = 1.0L / (nodes[k] - nodes[m]);
        for (int j = 0; j < M1; ++j)
            if (j != k && j != m) t *= (x - nodes[j]) / (nodes[k] - nodes[j]);
        s += t;
    }
    return s;
}

static void lgl_rule_x(int P, xreal *xi, xreal *w, xreal *D)
{
    int N = P + 1;
    xi[0] = -1.0L;
    xi[P] = 1.0L;
    /* interior nodes: roots of L_P', Newton from Chebyshev-Lobatto guesses */
    for (int k = 1; k < P; ++k) {
        xreal x = -cosl(3.14159265358979323846264338327950288L * k / P);
        for (int it = 0; it < 100; ++it) {
            xreal L, dL;
            legendre(P, x, &L, &dL);
            xreal d2L = (2.0L * x * dL - P * (P + 1.0L) * L) / (1.0L - x * x);
            xreal dx = dL / d2L;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        xi[k] = x;
    }
    for (int k = 0; k < N; ++k) {
        xreal L, dL;
        legendre(P, xi[k], &L, &dL);
        w[k] = 2.0L / (P * (P + 1.0L) * L * L);
    }
    lagrange_derivative_matrix(N, xi, D);
}

void orc_lgl(int P, double *xi, double *w, double *D)
{
    int N = P + 1;
    xreal x[MAXN], wx[MAXN], Dx[MAXN * MAXN];
    lgl_rule_x(P, x, wx, Dx);
    for (int k = 0; k < N; ++k) { xi[k] = (double)x[k]; w[k] = (double)wx[k]; }
    for (int k = 0; k < N * N; ++k) D[k] = (double)Dx[k];
}

/* ------------------------------------------------------------------------ */
/* Mesh topology helpers                                                     */
/* ------------------------------------------------------------------------ */

/* volume node of face-local point (a, b) on local face f */
static int face_node(int N, int f, int a, int b)
{
    int d = f / 2, s = (f & 1) ? N - 1 : 0;
    if (d == 0) return s + N * a + N * N * b;
    if (d == 1) return a + N * s + N * N * b;
    return a + N * b + N * N * s;
}

static void orient_map(int o, int M, int a, int b, int *a2, int *b2)
{
    int s = (o & 1) ? b : a, t = (o & 1) ? a : b;
    *a2 = (o & 2) ? M - s : s;
    *b2 = (o & 4) ? M - t : t;
}

static int is_owner(const orc_mesh *m, int e, int f)
{
    int e2 = m->nbr[e * 6 + f];
    if (e2 < 0) return 1;
    int f2 = m->nbr_face[e * 6 + f];
    return (e < e2) || (e == e2 && f < f2);
}

/* This element's own outward s*n at face f, node n: +-Ja^{f/2}. */
static void own_outward(const orc_mesh *m, int e, int f, int node, double v[3])
{
    int i = f / 2;
    double sg = (f & 1) ? 1.0 : -1.0;
    size_t n3 = N3E(m, e);
    for (int d = 0; d < 3; ++d)
        v[d] = sg * m->Ja[9 * m->off[e] + (size_t)(i * 3 + d) * n3 + node];
}

typedef struct {
    int interior;      /* 1 if a neighbour element, else boundary */
    int bc;            /* -1 wall, -2 far field (boundary only) */
    int e2, f2, node2; /* partner element, face and its volume node */
} partner_t;

/* Partner of a face point on a conforming face (both sides of one order). */
static partner_t partner(const orc_mesh *m, int e, int f, int a, int b)
{
    partner_t p;
    int N = NE(m, e);
    int e2 = m->nbr[e * 6 + f];
    if (e2 < 0) {
        p.interior = 0; p.bc = e2; p.e2 = e; p.f2 = f; p.node2 = face_node(N, f, a, b);
        return p;
    }
    int a2, b2;
    orient_map(m->orient[e * 6 + f], N - 1, a, b, &a2, &b2);
    p.interior = 1; p.bc = 0; p.e2 = e2; p.f2 = m->nbr_face[e * 6 + f];
    p.node2 = face_node(N, p.f2, a2, b2);
    return p;
}

/* A face between elements of different order (p-nonconforming) is coupled
 * through a mortar (the paper's solver supports such faces, Sec. 2.2):
 *  - the mortar carries the higher order M and the higher-order side's face
 *    nodes, frame and outward normal;
 *  - the lower-order side's trace is extended to the mortar nodes by its own
 *    Lagrange interpolant;
 *  - the numerical flux is evaluated once per mortar node;
 *  - the higher-order side takes it at its nodes; the lower-order side's
 *    surface integral of (flux x test function) is evaluated exactly on the
 *    mortar (the M-node Gauss-Lobatto rule integrates a degree M + P_low <=
 *    2M - 1 integrand exactly).
 * Returns 1 if face f of e is such a face. */
static int is_mortar(const orc_mesh *m, int e, int f)
{
    int e2 = m->nbr[e * 6 + f];
    return e2 >= 0 && m->P[e2] != m->P[e];
}

/* value of the order-P Lagrange basis function k at the M-node GLL point i */
static double interp_coef(const orc_mesh *m, int Nlo, int Nhi, int i, int k)
{
    xreal xl[MAXN];
    for (int a = 0; a < Nlo; ++a) xl[a] = m->xi[Nlo][a];
    return (double)lagrange_value(Nlo, xl, k, (xreal)m->xi[Nhi][i]);
}

/* ------------------------------------------------------------------------ */
/* Mesh construction: geometry at the nodes, curl-form metrics               */
/* ------------------------------------------------------------------------ */

/* Metric terms where orders meet.
 *
 * Reading (the paper's solver couples elements of different order, Sec. 2.2,
 * with curl-form metrics, App. B; how the two are made compatible on curved
 * faces is not stated): on a mesh of mixed order the curl-form product field
 * V = X_l grad_xi X_m is restricted on the element boundary before its curl is
 * taken, so that both sides of a face carry one polynomial normal s n:
 *  - edge rule: on an edge around which the orders differ, the component of V
 *    along the edge is replaced by its interpolant at the GLL points of degree
 *    P_E - 1, P_E the lowest order around the edge;
 *  - face rule: on a face between orders P_lo < P_hi, both sides replace each
 *    of the two tangential components by its interpolant of degree P_lo - 1
 *    along its own direction and P_lo across it, whose values on the face's
 *    edges along that direction come from the edge rule.
 * The face-normal metric (the tangential curl of these two components) then
 * has degree <= P_lo - 1 in each face direction on both sides, which the
 * mortar's exact integration against the lower side's basis reproduces.  The
 * discrete metric identities hold for any nodal V (difference operators of a
 * tensor grid commute).  A face or edge whose elements all have one order is
 * left alone, so a mesh of one order is unchanged.
 *
 * Local edge k runs along reference direction k / 4; bit 0 (bit 1) of k gives
 * the end, 0 or 1, of the lower (higher) of the two other directions. */
static void other_dirs(int dir, int *p, int *q)
{
    *p = dir == 0 ? 1 : 0;
    *q = dir == 2 ? 1 : 2;
}

static int edge_between(const int c0[3], const int c1[3])
{
    int dir = c0[0] != c1[0] ? 0 : c0[1] != c1[1] ? 1 : 2, p, q;
    other_dirs(dir, &p, &q);
    return 4 * dir + c0[p] + 2 * c0[q];
}

/* element corner of face-local corner (a, b) of local face f */
static void face_corner(int f, int a, int b, int c[3])
{
    int d = f / 2, p, q;
    other_dirs(d, &p, &q);
    c[d] = f & 1;
    c[p] = a;
    c[q] = b;
}

/* fdeg[e][6]: P_lo of a face between orders, else 0.  edeg[e][12]: lowest order
 * around an edge where orders differ, else 0.  The lowest and highest order
 * around each edge are propagated across faces until nothing changes. */
static void boundary_orders(int ne, const int *P, const int *nbr, const signed char *nbr_face,
                            const signed char *orient, int *fdeg, int *edeg)
{
    static const int corners[4][4] = {{0, 0, 1, 0}, {0, 1, 1, 1}, {0, 0, 0, 1}, {1, 0, 1, 1}};
    int *lo = malloc(sizeof(int) * 12 * (size_t)ne), *hi = malloc(sizeof(int) * 12 * (size_t)ne);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 12; ++k) lo[e * 12 + k] = hi[e * 12 + k] = P[e];
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int e = 0; e < ne; ++e)
            for (int f = 0; f < 6; ++f) {
                int e2 = nbr[e * 6 + f];
                if (e2 < 0) continue;
                int f2 = nbr_face[e * 6 + f];
                for (int s = 0; s < 4; ++s) {
                    int c0[3], c1[3], d0[3], d1[3], a2, b2;
                    face_corner(f, corners[s][0], corners[s][1], c0);
                    face_corner(f, corners[s][2], corners[s][3], c1);
                    orient_map(orient[e * 6 + f], 1, corners[s][0], corners[s][1], &a2, &b2);
                    face_corner(f2, a2, b2, d0);
                    orient_map(orient[e * 6 + f], 1, corners[s][2], corners[s][3], &a2, &b2);
                    face_corner(f2, a2, b2, d1);
                    int k = e * 12 + edge_between(c0, c1), k2 = e2 * 12 + edge_between(d0, d1);
                    int l = lo[k] < lo[k2] ? lo[k] : lo[k2], h = hi[k] > hi[k2] ? hi[k] : hi[k2];
                    if (l != lo[k] || l != lo[k2] || h != hi[k] || h != hi[k2]) {
                        lo[k] = lo[k2] = l;
                        hi[k] = hi[k2] = h;
                        changed = 1;
                    }
                }
            }
    }
    for (int e = 0; e < ne; ++e) {
        for (int k = 0; k < 12; ++k) edeg[e * 12 + k] = lo[e * 12 + k] < hi[e * 12 + k] ? lo[e * 12 + k] : 0;
        for (int f = 0; f < 6; ++f) {
            int e2 = nbr[e * 6 + f];
            fdeg[e * 6 + f] = (e2 >= 0 && P[e2] != P[e]) ? (P[e] < P[e2] ? P[e] : P[e2]) : 0;
        }
    }
    free(lo);
    free(hi);
}

/* V_k of physical row nn, (X_l - X_l(first control point)) dX_m/dxi_k with
 * (nn, m, l) cyclic, at reference point xi, from the degree-Pg map. */
static xreal map_V(int Pg, const xreal *gn, const double *X, int nn, int k, const xreal xi[3])
{
    int G1 = Pg + 1, G3 = G1 * G1 * G1, mm = (nn + 1) % 3, ll = (nn + 2) % 3;
    xreal lv[3][MAXN], ld[3][MAXN];
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < G1; ++j) {
            lv[d][j] = lagrange_value(G1, gn, j, xi[d]);
            ld[d][j] = lagrange_deriv(G1, gn, j, xi[d]);
        }
    const double *Xl = X + (size_t)ll * G3, *Xm = X + (size_t)mm * G3;
    xreal xl = 0.0L, dxm = 0.0L;
    for (int k3 = 0; k3 < G1; ++k3)
        for (int k2 = 0; k2 < G1; ++k2)
            for (int k1 = 0; k1 < G1; ++k1) {
                int i = k1 + G1 * k2 + G1 * G1 * k3;
                xl += ((xreal)Xl[i] - (xreal)Xl[0]) * lv[0][k1] * lv[1][k2] * lv[2][k3];
                xreal b = (k == 0 ? ld[0][k1] : lv[0][k1]) * (k == 1 ? ld[1][k2] : lv[1][k2])
                          * (k == 2 ? ld[2][k3] : lv[2][k3]);
                dxm += ((xreal)Xm[i] - (xreal)Xm[0]) * b;
            }
    return xl * dxm;
}

/* the edge rule's polynomial on local edge k (degree pe - 1) at coordinate t
 * along the edge */
static xreal edge_poly(int Pg, const xreal *gn, const double *X, int nn, int k, int pe, xreal t)
{
    xreal xs[MAXN], ws[MAXN], Ds[MAXN * MAXN];
    lgl_rule_x(pe - 1, xs, ws, Ds);
    int dir = k / 4, p, q;
    other_dirs(dir, &p, &q);
    xreal s = 0.0L;
    for (int j = 0; j < pe; ++j) {
        xreal pt[3];
        pt[dir] = xs[j];
        pt[p] = (k & 1) ? 1.0L : -1.0L;
        pt[q] = (k & 2) ? 1.0L : -1.0L;
        s += lagrange_value(pe, xs, j, t) * map_V(Pg, gn, X, nn, dir, pt);
    }
    return s;
}

/* Applies the edge and face rules to the nodal V[3][N^3] of row nn. */
static void restrict_boundary(int N, const xreal *xq, int Pg, const xreal *gn, const double *X, int nn,
                              const int *fdeg, const int *edeg, xreal *V)
{
    int N3 = N * N * N;
    for (int k = 0; k < 12; ++k) {
        if (!edeg[k]) continue;
        int dir = k / 4, p, q;
        other_dirs(dir, &p, &q);
        for (int a = 0; a < N; ++a) {
            int idx[3];
            idx[dir] = a;
            idx[p] = (k & 1) ? N - 1 : 0;
            idx[q] = (k & 2) ? N - 1 : 0;
            V[dir * N3 + idx[0] + N * idx[1] + N * N * idx[2]] = edge_poly(Pg, gn, X, nn, k, edeg[k], xq[a]);
        }
    }
    for (int f = 0; f < 6; ++f) {
        int pf = fdeg[f];
        if (!pf) continue;
        int d = f / 2, t[2];
        other_dirs(d, &t[0], &t[1]);
        xreal xa[MAXN], xb[MAXN], wx[MAXN], Dx[MAXN * MAXN];
        lgl_rule_x(pf - 1, xa, wx, Dx);   /* pf points along the component's own direction */
        lgl_rule_x(pf, xb, wx, Dx);       /* pf + 1 points across it */
        for (int ci = 0; ci < 2; ++ci) {
            int c = t[ci], o = t[1 - ci];
            xreal S[MAXN][MAXN];
            for (int i = 0; i < pf; ++i)
                for (int j = 0; j <= pf; ++j) {
                    if (j == 0 || j == pf) {
                        /* on the face's edge along c, at the end j of direction o */
                        int cc[3], p, q;
                        cc[d] = f & 1;
                        cc[o] = j == pf;
                        cc[c] = 0;
                        other_dirs(c, &p, &q);
                        int k = 4 * c + cc[p] + 2 * cc[q];
                        if (edeg[k]) { S[i][j] = edge_poly(Pg, gn, X, nn, k, edeg[k], xa[i]); continue; }
                    }
                    xreal pt[3];
                    pt[d] = (f & 1) ? 1.0L : -1.0L;
                    pt[c] = xa[i];
                    pt[o] = xb[j];
                    S[i][j] = map_V(Pg, gn, X, nn, c, pt);
                }
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    xreal v = 0.0L;
                    for (int i = 0; i < pf; ++i)
                        for (int j = 0; j <= pf; ++j)
                            v += lagrange_value(pf, xa, i, xq[a]) * lagrange_value(pf + 1, xb, j, xq[b]) * S[i][j];
                    int idx[3];
                    idx[d] = (f & 1) ? N - 1 : 0;
                    idx[c] = a;
                    idx[o] = b;
                    V[c * N3 + idx[0] + N * idx[1] + N * N * idx[2]] = v;
                }
        }
    }
}

static void element_metrics(orc_mesh *m, int e, int Pg, const double *X, const int *fdeg, const int *edeg)
{
    int N = NE(m, e), N3 = N3E(m, e), G1 = Pg + 1;
    xreal xq[MAXN], wq[MAXN], Dq[MAXN * MAXN];
    lgl_rule_x(m->P[e], xq, wq, Dq);
    xreal gn[MAXN];
    for (int k = 0; k < G1; ++k) gn[k] = -1.0L + 2.0L * k / Pg;
    xreal lg[MAXN][MAXN]; /* lg[a][k] = l_k^geom(xi_a) */
    for (int a = 0; a < N; ++a)
        for (int k = 0; k < G1; ++k) lg[a][k] = lagrange_value(G1, gn, k, xq[a]);

    /* The metric terms are invariant under a translation of the element, so
     * the geometry is interpolated and differentiated in coordinates relative
     * to the element's first control point: round-off then stays relative to
     * the element size rather than to its distance from the origin. */
    double *x = m->x + 3 * m->off[e];
    xreal *xl = malloc(sizeof(xreal) * 3 * N3);
    for (int c = 0; c < 3; ++c) {
        const double *Xc = X + (size_t)c * G1 * G1 * G1;
        for (int n = 0; n < N3; ++n) {
            int a = n % N, b = (n / N) % N, cc = n / (N * N);
            xreal s = 0.0L;
            for (int k3 = 0; k3 < G1; ++k3)
                for (int k2 = 0; k2 < G1; ++k2)
                    for (int k1 = 0; k1 < G1; ++k1)
                        s += ((xreal)Xc[k1 + G1 * k2 + G1 * G1 * k3] - (xreal)Xc[0])
                             * lg[a][k1] * lg[b][k2] * lg[cc][k3];
            xl[c * N3 + n] = s;
            x[c * N3 + n] = (double)((xreal)Xc[0] + s);
        }
    }

    /* derivative of a nodal field along reference direction k at node n */
#define DREF(field, k, n, out)                                                  \
    do {                                                                        \
        int a_ = (n) % N, b_ = ((n) / N) % N, c_ = (n) / (N * N);               \
        xreal s_ = 0.0L;                                                        \
        for (int q_ = 0; q_ < N; ++q_) {                                        \
            int idx_ = (k) == 0 ? q_ + N * b_ + N * N * c_                      \
                     : (k) == 1 ? a_ + N * q_ + N * N * c_                      \
                                : a_ + N * b_ + N * N * q_;                     \
            int row_ = (k) == 0 ? a_ : (k) == 1 ? b_ : c_;                      \
            s_ += Dq[row_ * N + q_] * (field)[idx_];                            \
        }                                                                       \
        (out) = s_;                                                             \
    } while (0)

    xreal *dX = malloc(sizeof(xreal) * 9 * N3);   /* dX[c][k][n] = dX_c/dxi_k */
    for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 3; ++k)
            for (int n = 0; n < N3; ++n) DREF(xl + c * N3, k, n, dX[(c * 3 + k) * N3 + n]);

    double *J = m->J + m->off[e];
    xreal vol = 0.0L;
    for (int n = 0; n < N3; ++n) {
        xreal a11 = dX[(0 * 3 + 0) * N3 + n], a12 = dX[(0 * 3 + 1) * N3 + n], a13 = dX[(0 * 3 + 2) * N3 + n];
        xreal a21 = dX[(1 * 3 + 0) * N3 + n], a22 = dX[(1 * 3 + 1) * N3 + n], a23 = dX[(1 * 3 + 2) * N3 + n];
        xreal a31 = dX[(2 * 3 + 0) * N3 + n], a32 = dX[(2 * 3 + 1) * N3 + n], a33 = dX[(2 * 3 + 2) * N3 + n];
        xreal Jx = a11 * (a22 * a33 - a23 * a32) - a12 * (a21 * a33 - a23 * a31) + a13 * (a21 * a32 - a22 * a31);
        J[n] = (double)Jx;
        int a = n % N, b = (n / N) % N, c = n / (N * N);
        vol += wq[a] * wq[b] * wq[c] * Jx;
    }

    /* Ja^i_n = -[curl_xi (X_l grad_xi X_m)]_i with (n, m, l) cyclic */
    xreal *V = malloc(sizeof(xreal) * 3 * N3);
    for (int nn = 0; nn < 3; ++nn) {
        int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
        for (int k = 0; k < 3; ++k)
            for (int n = 0; n < N3; ++n)
                V[k * N3 + n] = xl[ll * N3 + n] * dX[(mm * 3 + k) * N3 + n];
        restrict_boundary(N, xq, Pg, gn, X, nn, fdeg, edeg, V);
        for (int n = 0; n < N3; ++n) {
            xreal d1V2, d2V1, d2V0, d0V2, d0V1, d1V0;
            DREF(V + 2 * N3, 1, n, d1V2);
            DREF(V + 1 * N3, 2, n, d2V1);
            DREF(V + 0 * N3, 2, n, d2V0);
            DREF(V + 2 * N3, 0, n, d0V2);
            DREF(V + 1 * N3, 0, n, d0V1);
            DREF(V + 0 * N3, 1, n, d1V0);
            xreal curl[3] = {d1V2 - d2V1, d2V0 - d0V2, d0V1 - d1V0};
            for (int i = 0; i < 3; ++i)
                m->Ja[9 * m->off[e] + (size_t)(i * 3 + nn) * N3 + n] = (double)(-curl[i]);
        }
    }
#undef DREF
    free(V);
    free(xl);
    free(dX);
    m->delta[e] = (double)(cbrtl(vol) / N);
}

orc_mesh *orc_mesh_new_mixed(int ne, const int *P, int Pg, const double *xyz_geom, const int *nbr,
                             const signed char *nbr_face, const signed char *orient,
                             const unsigned char *flag)
{
    g_err[0] = 0;
    if (ne <= 0 || Pg < 1 || Pg > MAXN - 1) {
        snprintf(g_err, sizeof g_err, "bad sizes: n_elem=%d Pg=%d", ne, Pg);
        return NULL;
    }
    for (int e = 0; e < ne; ++e)
        if (P[e] < 1 || P[e] > MAXN - 1) {
            snprintf(g_err, sizeof g_err, "element %d: order %d outside 1..%d", e, P[e], MAXN - 1);
            return NULL;
        }
    /* connectivity must be symmetric with mutually inverse orientation maps */
    for (int e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            int e2 = nbr[e * 6 + f];
            if (e2 < 0) {
                if (e2 != -1 && e2 != -2) {
                    snprintf(g_err, sizeof g_err, "element %d face %d: bad boundary code %d", e, f, e2);
                    return NULL;
                }
                continue;
            }
            int f2 = nbr_face[e * 6 + f];
            if (e2 >= ne || f2 < 0 || f2 > 5 || nbr[e2 * 6 + f2] != e || nbr_face[e2 * 6 + f2] != f) {
                snprintf(g_err, sizeof g_err, "element %d face %d: asymmetric connectivity", e, f);
                return NULL;
            }
            int o = orient[e * 6 + f], o2 = orient[e2 * 6 + f2];
            if (o < 0 || o > 7 || o2 < 0 || o2 > 7) {
                snprintf(g_err, sizeof g_err, "element %d face %d: bad orientation", e, f);
                return NULL;
            }
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int a2, b2, a3, b3;
                    orient_map(o, 1, a, b, &a2, &b2);
                    orient_map(o2, 1, a2, b2, &a3, &b3);
                    if (a3 != a || b3 != b) {
                        snprintf(g_err, sizeof g_err, "element %d face %d: orientation codes not inverse", e, f);
                        return NULL;
                    }
                }
        }

    /* a face between orders: the face rule needs P_lo >= 2 (degree P_lo - 1
     * >= 1 along each direction), and P_lo >= Pg so that the restricted
     * product field of both sides differs only by a translation term whose
     * curl vanishes exactly */
    for (int e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            int e2 = nbr[e * 6 + f];
            if (e2 >= 0 && P[e2] != P[e]) {
                int plo = P[e] < P[e2] ? P[e] : P[e2];
                if (plo < 2 || plo < Pg) {
                    snprintf(g_err, sizeof g_err,
                             "element %d face %d: orders %d/%d need a lower order >= 2 and >= the geometry order %d",
                             e, f, P[e], P[e2], Pg);
                    return NULL;
                }
            }
        }

    orc_mesh *m = calloc(1, sizeof *m);
    m->ne = ne;
    m->P = malloc(sizeof(int) * ne);
    m->off = malloc(sizeof(size_t) * ne);
    memcpy(m->P, P, sizeof(int) * ne);
    size_t tot = 0;
    for (int e = 0; e < ne; ++e) { m->off[e] = tot; tot += (size_t)N3E(m, e); }
    m->nodes = tot;
    for (int n = 2; n <= MAXN; ++n) orc_lgl(n - 1, m->xi[n], m->w[n], m->D[n]);
    m->x = malloc(sizeof(double) * tot * 3);
    m->J = malloc(sizeof(double) * tot);
    m->Ja = malloc(sizeof(double) * tot * 9);
    m->delta = malloc(sizeof(double) * ne);
    m->nbr = malloc(sizeof(int) * ne * 6);
    m->nbr_face = malloc(ne * 6);
    m->orient = malloc(ne * 6);
    m->flag = malloc(ne);
    memcpy(m->nbr, nbr, sizeof(int) * ne * 6);
    memcpy(m->nbr_face, nbr_face, ne * 6);
    memcpy(m->orient, orient, ne * 6);
    memcpy(m->flag, flag, ne);
    size_t G3 = (size_t)(Pg + 1) * (Pg + 1) * (Pg + 1);
    int *fdeg = malloc(sizeof(int) * 6 * (size_t)ne), *edeg = malloc(sizeof(int) * 12 * (size_t)ne);
    boundary_orders(ne, P, nbr, nbr_face, orient, fdeg, edeg);
#pragma omp parallel for schedule(static) num_threads(orc_get_threads())
    for (int e = 0; e < ne; ++e)
        element_metrics(m, e, Pg, xyz_geom + (size_t)e * 3 * G3, fdeg + 6 * (size_t)e, edeg + 12 * (size_t)e);
    free(fdeg);
    free(edeg);
    for (int e = 0; e < ne; ++e)
        for (size_t i = 0; i < (size_t)N3E(m, e); ++i)
            if (!(m->J[m->off[e] + i] > 0.0)) {
                snprintf(g_err, sizeof g_err, "non-positive Jacobian in element %d", e);
                orc_mesh_free(m);
                return NULL;
            }
    return m;
}

orc_mesh *orc_mesh_new(int ne, int P, int Pg, const double *xyz_geom, const int *nbr,
                       const signed char *nbr_face, const signed char *orient,
                       const unsigned char *flag)
{
    if (ne <= 0) {
        snprintf(g_err, sizeof g_err, "bad sizes: n_elem=%d", ne);
        return NULL;
    }
    int *Pe = malloc(sizeof(int) * ne);
    for (int e = 0; e < ne; ++e) Pe[e] = P;
    orc_mesh *m = orc_mesh_new_mixed(ne, Pe, Pg, xyz_geom, nbr, nbr_face, orient, flag);
    free(Pe);
    return m;
}

size_t orc_mesh_nodes(const orc_mesh *m) { return m->nodes; }

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->x); free(m->J); free(m->Ja); free(m->delta); free(m->P); free(m->off);
    free(m->nbr); free(m->nbr_face); free(m->orient); free(m->flag);
    free(m);
}

void orc_set_flags(orc_mesh *m, const unsigned char *flag) { memcpy(m->flag, flag, m->ne); }

void orc_node_coords(const orc_mesh *m, double *xyz)
{
    memcpy(xyz, m->x, sizeof(double) * m->nodes * 3);
}

void orc_metrics(const orc_mesh *m, double *J, double *Ja)
{
    if (J) memcpy(J, m->J, sizeof(double) * m->nodes);
    if (Ja) memcpy(Ja, m->Ja, sizeof(double) * m->nodes * 9);
}

double orc_filter_width(const orc_mesh *m, int e) { return m->delta[e]; }

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

/* normal convective flux F.n of (p, u): (c0^2 u.n, u (u.n) + p n) */
static void normal_flux(double c0sq, const double *q, const double *n, double *F)
{
    double un = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    F[0] = c0sq * un;
    for (int r = 0; r < 3; ++r) F[1 + r] = q[1 + r] * un + q[0] * n[r];
}

/* Invert a 4x4 matrix by Gauss-Jordan elimination with partial pivoting. */
static void invert4(const double A_in[4][4], double inv[4][4])
{
    double A[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = j < 4 ? A_in[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 8; ++j) { double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
        double d = A[c][c];
        for (int j = 0; j < 8; ++j) A[c][j] /= d;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            double fct = A[r][c];
            for (int j = 0; j < 8; ++j) A[r][j] -= fct * A[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) inv[i][j] = A[i][j + 4];
}

/* Roe flux for the artificial-compressibility system along the unit normal n:
 * F = (F(qL) + F(qR))/2 - |A(qbar)| (qR - qL) / 2, with |A| = R |Lambda| R^-1
 * built from the eigen-decomposition of the flux Jacobian at the mean state.
 * Since the flux is quadratic, A(qbar) (qR - qL) = F(qR) - F(qL) exactly. */
void orc_roe_flux(double c0sq, const double *qL, const double *qR, const double *n, double *F)
{
    double FL[4], FR[4];
    normal_flux(c0sq, qL, n, FL);
    normal_flux(c0sq, qR, n, FR);
    double ub[3] = {0.5 * (qL[1] + qR[1]), 0.5 * (qL[2] + qR[2]), 0.5 * (qL[3] + qR[3])};
    double un = ub[0] * n[0] + ub[1] * n[1] + ub[2] * n[2];
    double a = sqrt(un * un + c0sq);
    /* acoustic eigenpairs: lambda = un +- a, vector (pi, v) with pi = -un +- a,
     * v = +-(pi n + ubar)/a; tangential pair: lambda = un, vector (0, t), t.n = 0 */
    double pip = -un + a, pim = -un - a;
    double R[4][4], lam[4];
    R[0][0] = pip;
    R[0][1] = pim;
    for (int d = 0; d < 3; ++d) {
        R[1 + d][0] = (pip * n[d] + ub[d]) / a;
        R[1 + d][1] = -(pim * n[d] + ub[d]) / a;
    }
    lam[0] = un + a;
    lam[1] = un - a;
    double h[3] = {1.0, 0.0, 0.0};
    if (fabs(n[0]) > 0.9) { h[0] = 0.0; h[1] = 1.0; }
    double hn = h[0] * n[0] + h[1] * n[1] + h[2] * n[2];
    double t1[3] = {h[0] - hn * n[0], h[1] - hn * n[1], h[2] - hn * n[2]};
    double t1n = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int d = 0; d < 3; ++d) t1[d] /= t1n;
    double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    R[0][2] = 0.0; R[0][3] = 0.0;
    for (int d = 0; d < 3; ++d) { R[1 + d][2] = t1[d]; R[1 + d][3] = t2[d]; }
    lam[2] = un; lam[3] = un;
    double Ri[4][4];
    invert4(R, Ri);
    double dq[4], alpha[4];
    for (int k = 0; k < 4; ++k) dq[k] = qR[k] - qL[k];
    for (int k = 0; k < 4; ++k) {
        alpha[k] = 0.0;
        for (int j = 0; j < 4; ++j) alpha[k] += Ri[k][j] * dq[j];
    }
    for (int r = 0; r < 4; ++r) {
        double diss = 0.0;
        for (int k = 0; k < 4; ++k) diss += R[r][k] * fabs(lam[k]) * alpha[k];
        F[r] = 0.5 * (FL[r] + FR[r]) - 0.5 * diss;
    }
}

/* Rusanov (local Lax-Friedrichs) flux, the alternative to Roe offered by the
 * scheme parameters: F = (F(qL) + F(qR))/2 - lambda (qR - qL)/2 with lambda
 * the larger spectral radius |u_n| + sqrt(u_n^2 + c0^2) of the two states'
 * normal flux Jacobians. */
void orc_rusanov_flux(double c0sq, const double *qL, const double *qR, const double *n, double *F)
{
    double FL[4], FR[4];
    normal_flux(c0sq, qL, n, FL);
    normal_flux(c0sq, qR, n, FR);
    double uL = qL[1] * n[0] + qL[2] * n[1] + qL[3] * n[2];
    double uR = qR[1] * n[0] + qR[2] * n[1] + qR[3] * n[2];
    double lL = fabs(uL) + sqrt(uL * uL + c0sq), lR = fabs(uR) + sqrt(uR * uR + c0sq);
    double lam = lL > lR ? lL : lR;
    for (int r = 0; r < 4; ++r) F[r] = 0.5 * (FL[r] + FR[r]) - 0.5 * lam * (qR[r] - qL[r]);
}

static void numerical_flux(const orc_params *p, const double *qL, const double *qR, const double *n, double *F)
{
    if (p->riemann == 1)
        orc_rusanov_flux(p->c0sq, qL, qR, n, F);
    else
        orc_roe_flux(p->c0sq, qL, qR, n, F);
}

/* LES eddy viscosity from the velocity gradient G[r*3+d] = du_r/dx_d. */
double orc_les_nut(int model, double C, double delta, const double *G)
{
    if (model == 1) {          /* Smagorinsky: (Cs Delta)^2 sqrt(2 S:S) */
        double SS = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int d = 0; d < 3; ++d) {
                double s = 0.5 * (G[r * 3 + d] + G[d * 3 + r]);
                SS += s * s;
            }
        return (C * delta) * (C * delta) * sqrt(2.0 * SS);
    }
    if (model == 2) {          /* Vreman: Cv sqrt(B_beta / alpha:alpha), unit density */
        double al[3][3], be[3][3], aa = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) { al[i][j] = G[j * 3 + i]; aa += al[i][j] * al[i][j]; }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int mm = 0; mm < 3; ++mm) s += al[mm][i] * al[mm][j];
                be[i][j] = delta * delta * s;
            }
        double B = be[0][0] * be[1][1] - be[0][1] * be[0][1] + be[0][0] * be[2][2] - be[0][2] * be[0][2]
                 + be[1][1] * be[2][2] - be[1][2] * be[1][2];
        if (aa == 0.0) return 0.0;
        if (B < 0.0) B = 0.0;
        return C * sqrt(B / aa);
    }
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Traces                                                                    */
/* ------------------------------------------------------------------------ */

static void trace_outside(const orc_mesh *m, const orc_params *p, const double *q, int e,
                          int node, partner_t pt, double out[4])
{
    if (pt.interior) {
        size_t n3 = N3E(m, pt.e2);
        for (int k = 0; k < 4; ++k) out[k] = q[4 * m->off[pt.e2] + (size_t)k * n3 + pt.node2];
    } else if (pt.bc == -1) {   /* no-slip wall: mirrored velocity, same pressure */
        size_t n3 = N3E(m, e);
        out[0] = q[4 * m->off[e] + node];
        for (int k = 1; k < 4; ++k) out[k] = -q[4 * m->off[e] + (size_t)k * n3 + node];
    } else {                    /* far field: prescribed state */
        for (int k = 0; k < 4; ++k) out[k] = p->q_inf[k];
    }
}

/* The outward s*n of the face's owner at this face point (single valued per face). */
static void owner_normal(const orc_mesh *m, int e, int f, int node, partner_t pt, double v[3])
{
    if (is_owner(m, e, f)) own_outward(m, e, f, node, v);
    else own_outward(m, pt.e2, pt.f2, pt.node2, v);
}

/* A mortar face seen from its higher-order side (eh, fh): the lower-order
 * side (el, fl), the mortar size M = N_eh, and for mortar node (i, j) of the
 * higher side the index (i', j') of the same point in the lower side's face
 * frame on an M-node grid. */
typedef struct {
    int eh, fh, el, fl, M, Nl;
} mortar_t;

static mortar_t mortar_of(const orc_mesh *m, int e, int f)
{
    mortar_t mt;
    int e2 = m->nbr[e * 6 + f], f2 = m->nbr_face[e * 6 + f];
    if (m->P[e] > m->P[e2]) { mt.eh = e; mt.fh = f; mt.el = e2; mt.fl = f2; }
    else { mt.eh = e2; mt.fh = f2; mt.el = e; mt.fl = f; }
    mt.M = NE(m, mt.eh);
    mt.Nl = NE(m, mt.el);
    return mt;
}

static void mortar_lowframe(const orc_mesh *m, const mortar_t *mt, int i, int j, int *il, int *jl)
{
    orient_map(m->orient[mt->eh * 6 + mt->fh], mt->M - 1, i, j, il, jl);
}

/* lower side's nodal field g[a + Nl b] (face-local) extended to mortar node (i, j) */
static double mortar_extend(const orc_mesh *m, const mortar_t *mt, const double *g, int i, int j)
{
    int il, jl;
    mortar_lowframe(m, mt, i, j, &il, &jl);
    double s = 0.0;
    for (int b = 0; b < mt->Nl; ++b)
        for (int a = 0; a < mt->Nl; ++a)
            s += interp_coef(m, mt->Nl, mt->M, il, a) * interp_coef(m, mt->Nl, mt->M, jl, b) * g[a + mt->Nl * b];
    return s;
}

/* exact surface integral of a mortar field G(i, j) against the lower side's
 * basis function of face node (a, b): sum_ij w_i w_j l_a l_b G */
static double mortar_project(const orc_mesh *m, const mortar_t *mt, const double *G, int a, int b)
{
    double s = 0.0;
    for (int j = 0; j < mt->M; ++j)
        for (int i = 0; i < mt->M; ++i) {
            int il, jl;
            mortar_lowframe(m, mt, i, j, &il, &jl);
            s += m->w[mt->M][i] * m->w[mt->M][j] * interp_coef(m, mt->Nl, mt->M, il, a)
                 * interp_coef(m, mt->Nl, mt->M, jl, b) * G[i + mt->M * j];
        }
    return s;
}

/* ------------------------------------------------------------------------ */
/* BR1 gradient (weak form) on viscous elements                              */
/* ------------------------------------------------------------------------ */

/* Mortar u* (s n) of the higher side at every mortar node: us[3 (r)][3 (d)][M^2] */
static void mortar_ustar_sn(const orc_mesh *m, const double *q, const mortar_t *mt, double *us)
{
    int M = mt->M, Nl = mt->Nl;
    size_t n3h = N3E(m, mt->eh), n3l = N3E(m, mt->el);
    double *gl = malloc(sizeof(double) * Nl * Nl);
    for (int r = 0; r < 3; ++r) {
        for (int b = 0; b < Nl; ++b)
            for (int a = 0; a < Nl; ++a)
                gl[a + Nl * b] = q[4 * m->off[mt->el] + (size_t)(1 + r) * n3l + face_node(Nl, mt->fl, a, b)];
        for (int j = 0; j < M; ++j)
            for (int i = 0; i < M; ++i) {
                int node = face_node(M, mt->fh, i, j);
                double uh = q[4 * m->off[mt->eh] + (size_t)(1 + r) * n3h + node];
                double ul = mortar_extend(m, mt, gl, i, j);
                double nv[3];
                own_outward(m, mt->eh, mt->fh, node, nv);
                for (int d = 0; d < 3; ++d) us[(r * 3 + d) * M * M + i + M * j] = 0.5 * (uh + ul) * nv[d];
            }
    }
    free(gl);
}

static void element_gradient(const orc_mesh *m, const orc_params *p, const double *q, int e, double *G)
{
    int N = NE(m, e), N3 = N3E(m, e);
    const double *w = m->w[N], *D = m->D[N];
    const double *qe = q + 4 * m->off[e];
    const double *Ja = m->Ja + 9 * m->off[e];
    const double *J = m->J + m->off[e];
    /* mortar faces: u* (s n) integrated against each face node's basis function */
    double *msurf[6] = {0};
    for (int f = 0; f < 6; ++f) {
        if (!is_mortar(m, e, f)) continue;
        mortar_t mt = mortar_of(m, e, f);
        int MM = mt.M * mt.M;
        double *us = malloc(sizeof(double) * 9 * MM);
        mortar_ustar_sn(m, q, &mt, us);
        msurf[f] = malloc(sizeof(double) * 9 * N * N);
        for (int b = 0; b < N; ++b)
            for (int a = 0; a < N; ++a)
                for (int k = 0; k < 9; ++k) {
                    double v;
                    if (mt.eh == e) v = w[a] * w[b] * us[k * MM + a + mt.M * b];
                    else v = -mortar_project(m, &mt, us + k * MM, a, b);   /* lower side: inward normal */
                    msurf[f][k * N * N + a + N * b] = v;
                }
        free(us);
    }
    for (int j = 0; j < N3; ++j) {
        int ijk[3] = {j % N, (j / N) % N, j / (N * N)};
        double acc[3][3] = {{0}};
        /* - sum over quadrature nodes of W (Ja^i_d u_r) d(phi_j)/dxi^i */
        for (int i = 0; i < 3; ++i) {
            double wother = 1.0;
            for (int k = 0; k < 3; ++k) if (k != i) wother *= w[ijk[k]];
            for (int mq = 0; mq < N; ++mq) {
                int mijk[3] = {ijk[0], ijk[1], ijk[2]};
                mijk[i] = mq;
                int mn = mijk[0] + N * mijk[1] + N * N * mijk[2];
                double coef = w[mq] * wother * D[mq * N + ijk[i]];
                for (int r = 0; r < 3; ++r)
                    for (int d = 0; d < 3; ++d)
                        acc[r][d] -= coef * qe[(1 + r) * N3 + mn] * Ja[(i * 3 + d) * N3 + mn];
            }
        }
        /* + surface integral of u* (s n)_out phi_j, u* = mean of the two traces */
        for (int f = 0; f < 6; ++f) {
            int d = f / 2, s = (f & 1) ? N - 1 : 0;
            if (ijk[d] != s) continue;
            int a = d == 0 ? ijk[1] : ijk[0];
            int b = d == 2 ? ijk[1] : ijk[2];
            if (msurf[f]) {
                for (int r = 0; r < 3; ++r)
                    for (int dd = 0; dd < 3; ++dd) acc[r][dd] += msurf[f][(r * 3 + dd) * N * N + a + N * b];
                continue;
            }
            partner_t pt = partner(m, e, f, a, b);
            double qo[4], nv[3];
            trace_outside(m, p, q, e, j, pt, qo);
            owner_normal(m, e, f, j, pt, nv);
            double sg = is_owner(m, e, f) ? 1.0 : -1.0;
            double wf = w[a] * w[b];
            for (int r = 0; r < 3; ++r) {
                double ustar = 0.5 * (qe[(1 + r) * N3 + j] + qo[1 + r]);
                for (int dd = 0; dd < 3; ++dd) acc[r][dd] += wf * ustar * sg * nv[dd];
            }
        }
        double mass = w[ijk[0]] * w[ijk[1]] * w[ijk[2]] * J[j];
        for (int r = 0; r < 3; ++r)
            for (int d = 0; d < 3; ++d) G[((size_t)(r * 3 + d)) * N3 + j] = acc[r][d] / mass;
    }
    for (int f = 0; f < 6; ++f) free(msurf[f]);
}

void orc_gradient(const orc_mesh *m, const orc_params *p, const double *q, double *G)
{
#pragma omp parallel for schedule(dynamic, 8) num_threads(orc_get_threads())
    for (int e = 0; e < m->ne; ++e)
        if (m->flag[e]) element_gradient(m, p, q, e, G + 9 * m->off[e]);
}

/* ------------------------------------------------------------------------ */
/* Residual                                                                  */
/* ------------------------------------------------------------------------ */

/* viscous flux 2 (nu + nu_t) S at every node of a viscous element: fv[r][d][N3] */
static void element_viscous_flux(const orc_mesh *m, const orc_params *p, const double *G, int e, double *fv)
{
    int N3 = N3E(m, e);
    for (int n = 0; n < N3; ++n) {
        double g[9];
        for (int k = 0; k < 9; ++k) g[k] = G[(size_t)k * N3 + n];
        double nut = orc_les_nut(p->les_model, p->C_les, m->delta[e], g);
        for (int r = 0; r < 3; ++r)
            for (int d = 0; d < 3; ++d)
                fv[(size_t)(r * 3 + d) * N3 + n] = 2.0 * (p->nu + nut) * 0.5 * (g[r * 3 + d] + g[d * 3 + r]);
    }
}

/* fv . v at a node (momentum rows), zero for an Euler element */
static void fv_dot(const orc_mesh *m, const double *fv, int e, int node, const double v[3], double out[3])
{
    if (!m->flag[e]) { out[0] = out[1] = out[2] = 0.0; return; }
    size_t N3 = N3E(m, e);
    const double *fe = fv + 9 * m->off[e];
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += fe[(size_t)(r * 3 + d) * N3 + node] * v[d];
        out[r] = s;
    }
}

/* Numerical flux through face f of element e at face point (a, b), outward for e,
 * already multiplied by the surface scaling s (conforming and boundary faces). */
static void face_flux(const orc_mesh *m, const orc_params *p, const double *q, const double *fv,
                      int e, int f, int a, int b, double Fout[4])
{
    size_t N3 = N3E(m, e);
    int node = face_node(NE(m, e), f, a, b);
    partner_t pt = partner(m, e, f, a, b);
    int own = is_owner(m, e, f);
    double qm[4], qp[4], nv[3];
    for (int k = 0; k < 4; ++k) qm[k] = q[4 * m->off[e] + (size_t)k * N3 + node];
    trace_outside(m, p, q, e, node, pt, qp);
    owner_normal(m, e, f, node, pt, nv);
    double s = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double nh[3] = {nv[0] / s, nv[1] / s, nv[2] / s};
    const double *qL = own ? qm : qp;
    const double *qR = own ? qp : qm;
    double F[4];
    numerical_flux(p, qL, qR, nh, F);
    for (int k = 0; k < 4; ++k) F[k] *= s;

    /* BR1 viscous flux: mean of the two sides' viscous fluxes along s n */
    double fvo[3] = {0, 0, 0};
    if (!pt.interior) {
        fv_dot(m, fv, e, node, nv, fvo);              /* boundary: interior viscous flux */
    } else {
        int eo = own ? e : pt.e2, no = own ? node : pt.node2;     /* owner side */
        int en = own ? pt.e2 : e, nn = own ? pt.node2 : node;     /* other side */
        double fL[3], fR[3];
        fv_dot(m, fv, eo, no, nv, fL);
        fv_dot(m, fv, en, nn, nv, fR);
        int both = m->flag[eo] && m->flag[en];
        if (p->mixed_face == 0 || both)
            for (int r = 0; r < 3; ++r) fvo[r] = 0.5 * (fL[r] + fR[r]);
    }
    for (int r = 0; r < 3; ++r) F[1 + r] -= fvo[r];
    double sg = own ? 1.0 : -1.0;
    for (int k = 0; k < 4; ++k) Fout[k] = sg * F[k];
}

/* Numerical flux at every mortar node, outward for the higher side and
 * multiplied by s: Roe on (higher trace, extended lower trace) with the
 * higher side's normal, minus the BR1 mean of the higher side's viscous
 * trace and the extended lower side's viscous trace (each side's viscous
 * flux dotted with the mortar's s n direction at its own nodes).
 * F[row][M^2]. */
static void mortar_flux(const orc_mesh *m, const orc_params *p, const double *q, const double *fv,
                        const mortar_t *mt, double *F)
{
    int M = mt->M, Nl = mt->Nl, MM = M * M;
    size_t n3h = N3E(m, mt->eh), n3l = N3E(m, mt->el);
    int vh = m->flag[mt->eh], vl = m->flag[mt->el];
    int keep = p->mixed_face == 0 || (vh && vl);
    double *gl = malloc(sizeof(double) * 7 * Nl * Nl);   /* lower side: 4 state fields + 3 viscous trace rows */
    for (int b = 0; b < Nl; ++b)
        for (int a = 0; a < Nl; ++a) {
            int node = face_node(Nl, mt->fl, a, b);
            for (int k = 0; k < 4; ++k) gl[k * Nl * Nl + a + Nl * b] = q[4 * m->off[mt->el] + (size_t)k * n3l + node];
            double nv[3], t[3];
            own_outward(m, mt->el, mt->fl, node, nv);
            for (int d = 0; d < 3; ++d) nv[d] = -nv[d];      /* the mortar's direction */
            fv_dot(m, fv, mt->el, node, nv, t);
            for (int r = 0; r < 3; ++r) gl[(4 + r) * Nl * Nl + a + Nl * b] = t[r];
        }
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
            int node = face_node(M, mt->fh, i, j);
            double qh[4], ql[4], nv[3], th[3], tl[3];
            for (int k = 0; k < 4; ++k) {
                qh[k] = q[4 * m->off[mt->eh] + (size_t)k * n3h + node];
                ql[k] = mortar_extend(m, mt, gl + k * Nl * Nl, i, j);
            }
            own_outward(m, mt->eh, mt->fh, node, nv);
            double s = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            double nh[3] = {nv[0] / s, nv[1] / s, nv[2] / s};
            double Fr[4];
            numerical_flux(p, qh, ql, nh, Fr);
            fv_dot(m, fv, mt->eh, node, nv, th);
            for (int r = 0; r < 3; ++r) tl[r] = vl ? mortar_extend(m, mt, gl + (4 + r) * Nl * Nl, i, j) : 0.0;
            for (int k = 0; k < 4; ++k) F[k * MM + i + M * j] = s * Fr[k];
            if (vh || vl)
                for (int r = 0; r < 3; ++r) F[(1 + r) * MM + i + M * j] -= keep ? 0.5 * (th[r] + tl[r]) : 0.0;
        }
    free(gl);
}

static void element_residual(const orc_mesh *m, const orc_params *p, const double *q, const double *fv,
                             int e, double *Re)
{
    int N = NE(m, e), N3 = N3E(m, e);
    const double *w = m->w[N], *D = m->D[N];
    const double *qe = q + 4 * m->off[e];
    const double *Ja = m->Ja + 9 * m->off[e];
    const double *J = m->J + m->off[e];
    const double *fve = fv + 9 * m->off[e];
    double *Ft = malloc(sizeof(double) * 12 * N3);     /* Ft[i][row][n] */
    for (int n = 0; n < N3; ++n) {
        double pr = qe[n], u[3] = {qe[N3 + n], qe[2 * N3 + n], qe[3 * N3 + n]};
        double f[4][3];
        for (int d = 0; d < 3; ++d) {
            f[0][d] = p->c0sq * u[d];
            for (int r = 0; r < 3; ++r) f[1 + r][d] = u[r] * u[d] + (r == d ? pr : 0.0);
        }
        if (m->flag[e])
            for (int r = 0; r < 3; ++r)
                for (int d = 0; d < 3; ++d) f[1 + r][d] -= fve[(size_t)(r * 3 + d) * N3 + n];
        for (int i = 0; i < 3; ++i)
            for (int row = 0; row < 4; ++row) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d) s += Ja[(i * 3 + d) * N3 + n] * f[row][d];
                Ft[(i * 4 + row) * N3 + n] = s;
            }
    }
    /* mortar faces: the flux integrated against each face node's basis function */
    double *msurf[6] = {0};
    for (int f = 0; f < 6; ++f) {
        if (!is_mortar(m, e, f)) continue;
        mortar_t mt = mortar_of(m, e, f);
        int MM = mt.M * mt.M;
        double *Fm = malloc(sizeof(double) * 4 * MM);
        mortar_flux(m, p, q, fv, &mt, Fm);
        msurf[f] = malloc(sizeof(double) * 4 * N * N);
        for (int b = 0; b < N; ++b)
            for (int a = 0; a < N; ++a)
                for (int row = 0; row < 4; ++row) {
                    double v;
                    if (mt.eh == e) v = w[a] * w[b] * Fm[row * MM + a + mt.M * b];
                    else v = -mortar_project(m, &mt, Fm + row * MM, a, b);   /* outward for the lower side */
                    msurf[f][row * N * N + a + N * b] = v;
                }
        free(Fm);
    }
    for (int j = 0; j < N3; ++j) {
        int ijk[3] = {j % N, (j / N) % N, j / (N * N)};
        double vol[4] = {0, 0, 0, 0}, surf[4] = {0, 0, 0, 0};
        /* + sum over quadrature nodes of W Ft^i d(phi_j)/dxi^i */
        for (int i = 0; i < 3; ++i) {
            double wother = 1.0;
            for (int k = 0; k < 3; ++k) if (k != i) wother *= w[ijk[k]];
            for (int mq = 0; mq < N; ++mq) {
                int mijk[3] = {ijk[0], ijk[1], ijk[2]};
                mijk[i] = mq;
                int mn = mijk[0] + N * mijk[1] + N * N * mijk[2];
                double coef = w[mq] * wother * D[mq * N + ijk[i]];
                for (int row = 0; row < 4; ++row) vol[row] += coef * Ft[(i * 4 + row) * N3 + mn];
            }
        }
        /* surface integral of the numerical flux times phi_j */
        for (int f = 0; f < 6; ++f) {
            int d = f / 2, s = (f & 1) ? N - 1 : 0;
            if (ijk[d] != s) continue;
            int a = d == 0 ? ijk[1] : ijk[0];
            int b = d == 2 ? ijk[1] : ijk[2];
            if (msurf[f]) {
                for (int row = 0; row < 4; ++row) surf[row] += msurf[f][row * N * N + a + N * b];
                continue;
            }
            double Fo[4];
            face_flux(m, p, q, fv, e, f, a, b, Fo);
            double wf = w[a] * w[b];
            for (int row = 0; row < 4; ++row) surf[row] += wf * Fo[row];
        }
        double mass = w[ijk[0]] * w[ijk[1]] * w[ijk[2]] * J[j];
        for (int row = 0; row < 4; ++row) Re[(size_t)row * N3 + j] = (vol[row] - surf[row]) / mass;
    }
    for (int f = 0; f < 6; ++f) free(msurf[f]);
    free(Ft);
}

void orc_residual(const orc_mesh *m, const orc_params *p, const double *q, double *R)
{
    double *fv = malloc(sizeof(double) * m->nodes * 9);
#pragma omp parallel num_threads(orc_get_threads())
    {
        double *G = malloc(sizeof(double) * 9 * MAXN * MAXN * MAXN);
#pragma omp for schedule(dynamic, 8)
        for (int e = 0; e < m->ne; ++e) {
            if (!m->flag[e]) continue;
            element_gradient(m, p, q, e, G);
            element_viscous_flux(m, p, G, e, fv + 9 * m->off[e]);
        }
        free(G);
#pragma omp for schedule(dynamic, 8)
        for (int e = 0; e < m->ne; ++e) element_residual(m, p, q, fv, e, R + 4 * m->off[e]);
    }
    free(fv);
}

/* ------------------------------------------------------------------------ */
/* Low-storage three-stage RK (Williamson 2N coefficients)                   */
/* ------------------------------------------------------------------------ */

typedef void (*rhs_fn)(void *ctx, const double *y, double *r);

static void rk3_drive(size_t n, double *y, double dt, int nsteps, rhs_fn f, void *ctx)
{
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    double *dq = calloc(n, sizeof(double));
    double *r = malloc(n * sizeof(double));
    for (int step = 0; step < nsteps; ++step)
        for (int s = 0; s < 3; ++s) {
            f(ctx, y, r);
            for (size_t i = 0; i < n; ++i) {
                dq[i] = A[s] * dq[i] + dt * r[i];
                y[i] += B[s] * dq[i];
            }
        }
    free(r);
    free(dq);
}

typedef struct { const orc_mesh *m; const orc_params *p; } mesh_ctx;
static void mesh_rhs(void *ctx, const double *y, double *r)
{
    mesh_ctx *c = ctx;
    orc_residual(c->m, c->p, y, r);
}

void orc_rk3_steps(const orc_mesh *m, const orc_params *p, double *q, double dt, int nsteps)
{
    mesh_ctx c = {m, p};
    rk3_drive(4 * m->nodes, q, dt, nsteps, mesh_rhs, &c);
}

typedef struct { double re, im; } lin_ctx;
static void linear_rhs(void *ctx, const double *y, double *r)
{
    lin_ctx *c = ctx;
    r[0] = c->re * y[0] - c->im * y[1];
    r[1] = c->re * y[1] + c->im * y[0];
}

void orc_rk3_linear(double lam_re, double lam_im, double dt, int nsteps, double *y_re, double *y_im)
{
    lin_ctx c = {lam_re, lam_im};
    double y[2] = {*y_re, *y_im};
    rk3_drive(2, y, dt, nsteps, linear_rhs, &c);
    *y_re = y[0];
    *y_im = y[1];
}

static void riccati_rhs(void *ctx, const double *y, double *r)
{
    (void)ctx;
    r[0] = -y[0] * y[0];
}

double orc_rk3_riccati(double y0, double dt, int nsteps)
{
    double y = y0;
    rk3_drive(1, &y, dt, nsteps, riccati_rhs, NULL);
    return y;
}
