// Host-side set-up: Gauss-Lobatto-Legendre rule, node geometry and metric
// terms, processing order.  Runs once per mesh (App. B: the mapping of every
// curvilinear hexahedron onto the reference cube, its Jacobian and the
// contravariant metric terms that turn physical fluxes into reference ones).
//
// These set-up quantities are evaluated in x87 extended precision and rounded
// once to double, so the stored rule and metric terms are the correctly
// rounded values of what they define; the residual itself is all FP64.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>

#include "hdg_internal.h"

namespace hdg {

namespace {

using xreal = long double;

// Legendre L_n(x) and L_n'(x).
void legendre_pair(int n, xreal x, xreal &L, xreal &dL)
{
    xreal lm1 = 1.0L, l = x, dlm1 = 0.0L, dl = 1.0L;
    if (n == 0) { L = 1.0L; dL = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        xreal lk = ((2 * k - 1) * x * l - (k - 1) * lm1) / k;
        xreal dlk = dlm1 + (2 * k - 1) * l;
        lm1 = l; l = lk; dlm1 = dl; dl = dlk;
    }
    L = l; dL = dl;
}

// Extended-precision GLL rule: nodes, weights, derivative matrix.
void gll_rule_x(int P, std::vector<xreal> &xi, std::vector<xreal> &w, std::vector<xreal> &D)
{
    const int N = P + 1;
    const xreal pi = 3.14159265358979323846264338327950288L;
    xi.assign(N, 0.0L);
    w.assign(N, 0.0L);
    D.assign(N * N, 0.0L);
    xi[0] = -1.0L;
    xi[P] = 1.0L;
    for (int j = 1; 2 * j <= P; ++j) {
        xreal x = -std::cos(pi * (j + 0.25L) / P - 3.0L / (8.0L * P * pi * (j + 0.25L)));
        for (int it = 0; it < 200; ++it) {
            xreal La, dLa, Lb, dLb;
            legendre_pair(P + 1, x, La, dLa);
            legendre_pair(P - 1, x, Lb, dLb);
            xreal step = (La - Lb) / (dLa - dLb);
            x -= step;
            if (std::fabs(step) <= 1e-19L) break;
        }
        xi[j] = x;
        xi[P - j] = -x;
    }
    if (P % 2 == 0) xi[P / 2] = 0.0L;
    for (int j = 0; j < N; ++j) {
        xreal L, dL;
        legendre_pair(P, xi[j], L, dL);
        w[j] = 2.0L / (P * (P + 1.0L) * L * L);
    }
    std::vector<xreal> lam(N, 1.0L);
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k)
            if (k != j) lam[j] /= (xi[j] - xi[k]);
    for (int i = 0; i < N; ++i) {
        xreal diag = 0.0L;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            xreal v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[i * N + j] = v;
            diag -= v;
        }
        D[i * N + i] = diag;
    }
}

}  // namespace

// GLL nodes are the zeros of q(x) = L_{P+1}(x) - L_{P-1}(x) (which contains
// the end points): Newton on q with q' = L'_{P+1} - L'_{P-1}.  The derivative
// matrix uses barycentric weights; its diagonal is the negative row sum, so
// it maps constants to zero.
void gll_rule(int P, std::vector<double> &xi, std::vector<double> &w, std::vector<double> &D)
{
    std::vector<xreal> x, wx, Dx;
    gll_rule_x(P, x, wx, Dx);
    xi.assign(x.begin(), x.end());
    w.assign(wx.begin(), wx.end());
    D.assign(Dx.begin(), Dx.end());
}

namespace {

// Lagrange interpolation matrix from nodes src (m points) to points dst.
std::vector<xreal> interp_matrix(const std::vector<xreal> &src, const std::vector<xreal> &dst)
{
    const int m = (int)src.size(), n = (int)dst.size();
    std::vector<xreal> bw(m, 1.0L);
    for (int j = 0; j < m; ++j)
        for (int k = 0; k < m; ++k)
            if (k != j) bw[j] /= (src[j] - src[k]);
    std::vector<xreal> I(n * m, 0.0L);
    for (int i = 0; i < n; ++i) {
        int hit = -1;
        for (int j = 0; j < m; ++j)
            if (dst[i] == src[j]) hit = j;
        if (hit >= 0) { I[i * m + hit] = 1.0L; continue; }
        xreal den = 0.0L;
        for (int j = 0; j < m; ++j) den += bw[j] / (dst[i] - src[j]);
        for (int j = 0; j < m; ++j) I[i * m + j] = (bw[j] / (dst[i] - src[j])) / den;
    }
    return I;
}

// out[n] = sum_k M[idx(n,dir)][k] in[... k along dir ...] on an (nx, ny, nz) lattice,
// producing an (ox, oy, oz) lattice where only dir changes size.
void apply_dir(const std::vector<xreal> &M, int rows, int cols, int dir, const xreal *in,
               int nx, int ny, int nz, xreal *out)
{
    int dims_in[3] = {nx, ny, nz};
    int dims_out[3] = {nx, ny, nz};
    dims_out[dir] = rows;
    (void)cols;
    for (int c = 0; c < dims_out[2]; ++c)
        for (int b = 0; b < dims_out[1]; ++b)
            for (int a = 0; a < dims_out[0]; ++a) {
                int o[3] = {a, b, c};
                xreal s = 0.0L;
                for (int k = 0; k < dims_in[dir]; ++k) {
                    int ii[3] = {a, b, c};
                    ii[dir] = k;
                    s += M[o[dir] * dims_in[dir] + k] * in[ii[0] + dims_in[0] * (ii[1] + dims_in[1] * ii[2])];
                }
                out[a + dims_out[0] * (b + dims_out[1] * c)] = s;
            }
}

}  // namespace

void gll_interp(int Plo, int Phi, std::vector<double> &I)
{
    std::vector<xreal> xl, wl, Dl, xh, wh, Dh;
    gll_rule_x(Plo, xl, wl, Dl);
    gll_rule_x(Phi, xh, wh, Dh);
    const std::vector<xreal> Ix = interp_matrix(xl, xh);
    I.assign(Ix.begin(), Ix.end());
}

namespace {

// Reference-cube corner (bits along xi1, xi2, xi3) of corner (a, b) of local
// face f; the face's own coordinates are the two other directions in
// increasing order, as for its nodes.
void face_corner_bits(int f, int a, int b, int c[3])
{
    const int d = f / 2;
    c[d] = f & 1;
    c[d == 0 ? 1 : 0] = a;
    c[d == 2 ? 1 : 2] = b;
}

// Local edge through two corners: 4 * direction + end of the lower other
// direction + 2 * end of the higher one.
int edge_through(const int u[3], const int v[3])
{
    int dir = 0;
    while (u[dir] == v[dir]) ++dir;
    return 4 * dir + u[dir == 0 ? 1 : 0] + 2 * u[dir == 2 ? 1 : 2];
}

int64_t root_of(std::vector<int64_t> &par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

}  // namespace

// The element edges meeting at one mesh edge are joined through the faces
// that share it (union-find over element-edge slots); each mesh edge then
// knows the lowest and highest order around it.  A rule whose interpolation
// is exact is skipped: the product field has degree 2 Pg - 1 along an edge
// and (2 Pg - 1, 2 Pg) on a face, so an edge with 2 Pg <= P_E and a face with
// 2 Pg <= P_lo none of whose edges is restricted keep their values.
void boundary_orders(const hdg_mesh_desc &d, BoundaryOrders &b)
{
    const int64_t ne = d.n_elem;
    b.face.assign(ne * 6, 0);
    b.edge.assign(ne * 12, 0);
    b.any = false;
    for (int64_t e = 1; e < ne && !b.any; ++e) b.any = d.P[e] != d.P[0];
    if (!b.any) return;
    static const int sides[4][4] = {{0, 0, 1, 0}, {0, 1, 1, 1}, {0, 0, 0, 1}, {1, 0, 1, 1}};
    std::vector<int64_t> par(ne * 12);
    std::iota(par.begin(), par.end(), 0);
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t e2 = d.nbr[e * 6 + f];
            if (e2 < 0) continue;
            if (d.P[e2] != d.P[e]) b.face[e * 6 + f] = (int8_t)std::min(d.P[e], d.P[e2]);
            const int f2 = d.nbr_face[e * 6 + f], o = d.orient[e * 6 + f];
            for (const auto &sd : sides) {
                int u[3], v[3], u2[3], v2[3];
                face_corner_bits(f, sd[0], sd[1], u);
                face_corner_bits(f, sd[2], sd[3], v);
                // the same two corners in the neighbour's face coordinates
                auto across = [&](int a, int bb, int out[3]) {
                    const int s = (o & 1) ? bb : a, t = (o & 1) ? a : bb;
                    face_corner_bits(f2, (o & 2) ? 1 - s : s, (o & 4) ? 1 - t : t, out);
                };
                across(sd[0], sd[1], u2);
                across(sd[2], sd[3], v2);
                const int64_t x = root_of(par, e * 12 + edge_through(u, v));
                const int64_t y = root_of(par, (int64_t)e2 * 12 + edge_through(u2, v2));
                if (x != y) par[std::max(x, y)] = std::min(x, y);
            }
        }
    std::vector<int8_t> lo(ne * 12, 127), hi(ne * 12, 0);
    for (int64_t slot = 0; slot < ne * 12; ++slot) {
        const int64_t r = root_of(par, slot);
        const int8_t P = (int8_t)d.P[slot / 12];
        lo[r] = std::min(lo[r], P);
        hi[r] = std::max(hi[r], P);
    }
    const int twice_pg = 2 * d.geom_order;
    for (int64_t slot = 0; slot < ne * 12; ++slot) {
        const int64_t r = root_of(par, slot);
        if (lo[r] < hi[r] && lo[r] < twice_pg) b.edge[slot] = lo[r];
    }
    // edges of each local face: along a (bit of b) and along b (bit of a)
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            if (!b.face[e * 6 + f] || b.face[e * 6 + f] < twice_pg) continue;
            bool edges = false;
            for (const auto &sd : sides) {
                int u[3], v[3];
                face_corner_bits(f, sd[0], sd[1], u);
                face_corner_bits(f, sd[2], sd[3], v);
                edges = edges || b.edge[e * 12 + edge_through(u, v)] != 0;
            }
            if (!edges) b.face[e * 6 + f] = 0;
        }
    b.any = false;
    for (int8_t c : b.face) b.any = b.any || c;
    for (int8_t c : b.edge) b.any = b.any || c;
}

namespace {

// One overwritten entry of the curl-form product field: component k at node
// p, its value for each physical row n.
struct BoundaryValue {
    int k;
    int p;
    xreal v[3];
};

// The edge and face rules on element e (see BoundaryOrders): the values
// they give to the element's boundary entries of V_k = (x_l - x_l0) dx_m/dxi_k,
// (n, m, l) cyclic, x_l0 the first control point.  Edges come first, faces
// after (a face rule's edge values are the edge rule's).
void boundary_values(const double *Xe, int Pg, const std::vector<xreal> &gnodes, const std::vector<xreal> &Dg,
                     int N, const std::vector<xreal> &xq, const int8_t *fo, const int8_t *eo,
                     std::vector<BoundaryValue> &out)
{
    const int G1 = Pg + 1, G3 = G1 * G1 * G1;
    out.clear();
    auto ctrl = [&](int c, const int i[3]) {
        return (xreal)Xe[c * G3 + i[0] + G1 * (i[1] + G1 * i[2])] - (xreal)Xe[c * G3];
    };
    // the edge rule's samples: V along edge k at its pe GLL points (degree pe - 1)
    auto edge_samples = [&](int k, int pe, std::vector<xreal> &xs, std::vector<xreal> &vals) {
        std::vector<xreal> ww, DD;
        gll_rule_x(pe - 1, xs, ww, DD);
        const int dir = k / 4, p = dir == 0 ? 1 : 0, q = dir == 2 ? 1 : 2;
        xreal line[3][13], dline[3][13];
        for (int c = 0; c < 3; ++c)
            for (int g = 0; g < G1; ++g) {
                int i[3];
                i[dir] = g;
                i[p] = (k & 1) * Pg;
                i[q] = ((k >> 1) & 1) * Pg;
                line[c][g] = ctrl(c, i);
            }
        for (int c = 0; c < 3; ++c)
            for (int g = 0; g < G1; ++g) {
                xreal s = 0.0L;
                for (int h = 0; h < G1; ++h) s += Dg[g * G1 + h] * line[c][h];
                dline[c][g] = s;
            }
        const std::vector<xreal> L = interp_matrix(gnodes, xs);
        vals.assign(3 * pe, 0.0L);
        for (int j = 0; j < pe; ++j) {
            xreal X[3] = {0, 0, 0}, dX[3] = {0, 0, 0};
            for (int c = 0; c < 3; ++c)
                for (int g = 0; g < G1; ++g) {
                    X[c] += L[j * G1 + g] * line[c][g];
                    dX[c] += L[j * G1 + g] * dline[c][g];
                }
            for (int n = 0; n < 3; ++n) vals[n * pe + j] = X[(n + 2) % 3] * dX[(n + 1) % 3];
        }
    };
    for (int k = 0; k < 12; ++k) {
        const int pe = eo[k];
        if (!pe) continue;
        std::vector<xreal> xs, vals;
        edge_samples(k, pe, xs, vals);
        const std::vector<xreal> Ie = interp_matrix(xs, xq);
        const int dir = k / 4, p = dir == 0 ? 1 : 0, q = dir == 2 ? 1 : 2;
        for (int a = 0; a < N; ++a) {
            int i[3];
            i[dir] = a;
            i[p] = (k & 1) * (N - 1);
            i[q] = ((k >> 1) & 1) * (N - 1);
            BoundaryValue bv{dir, i[0] + N * (i[1] + N * i[2]), {0, 0, 0}};
            for (int n = 0; n < 3; ++n)
                for (int j = 0; j < pe; ++j) bv.v[n] += Ie[a * pe + j] * vals[n * pe + j];
            out.push_back(bv);
        }
    }
    for (int f = 0; f < 6; ++f) {
        const int pf = fo[f];
        if (!pf) continue;
        const int d = f / 2, side = f & 1, t[2] = {d == 0 ? 1 : 0, d == 2 ? 1 : 2};
        std::vector<xreal> xa, xb, ww, DD;
        gll_rule_x(pf - 1, xa, ww, DD);      // pf points along the component's own direction
        gll_rule_x(pf, xb, ww, DD);          // pf + 1 points across it
        const std::vector<xreal> La = interp_matrix(gnodes, xa), Lb = interp_matrix(gnodes, xb);
        const std::vector<xreal> Ia = interp_matrix(xa, xq), Ib = interp_matrix(xb, xq);
        for (int ci = 0; ci < 2; ++ci) {
            const int c = t[ci], o = t[1 - ci];
            // control net of the face as [g along c][g along o], and its derivative along c
            std::vector<xreal> net(3 * G1 * G1), dnet(3 * G1 * G1, 0.0L);
            for (int cc = 0; cc < 3; ++cc)
                for (int gc = 0; gc < G1; ++gc)
                    for (int go = 0; go < G1; ++go) {
                        int i[3];
                        i[d] = side * Pg;
                        i[c] = gc;
                        i[o] = go;
                        net[(cc * G1 + gc) * G1 + go] = ctrl(cc, i);
                    }
            for (int cc = 0; cc < 3; ++cc)
                for (int gc = 0; gc < G1; ++gc)
                    for (int go = 0; go < G1; ++go)
                        for (int h = 0; h < G1; ++h)
                            dnet[(cc * G1 + gc) * G1 + go] += Dg[gc * G1 + h] * net[(cc * G1 + h) * G1 + go];
            std::vector<xreal> S(3 * pf * (pf + 1));
            for (int i = 0; i < pf; ++i)
                for (int j = 0; j <= pf; ++j) {
                    xreal X[3] = {0, 0, 0}, dX[3] = {0, 0, 0};
                    for (int cc = 0; cc < 3; ++cc)
                        for (int gc = 0; gc < G1; ++gc)
                            for (int go = 0; go < G1; ++go) {
                                const xreal wgt = La[i * G1 + gc] * Lb[j * G1 + go];
                                X[cc] += wgt * net[(cc * G1 + gc) * G1 + go];
                                dX[cc] += wgt * dnet[(cc * G1 + gc) * G1 + go];
                            }
                    for (int n = 0; n < 3; ++n) S[(n * pf + i) * (pf + 1) + j] = X[(n + 2) % 3] * dX[(n + 1) % 3];
                }
            // the two edges of the face along c take the edge rule's polynomial
            for (int end = 0; end < 2; ++end) {
                int bits[3] = {0, 0, 0};
                bits[d] = side;
                bits[o] = end;
                const int k = 4 * c + bits[c == 0 ? 1 : 0] + 2 * bits[c == 2 ? 1 : 2];
                if (!eo[k]) continue;
                std::vector<xreal> xs, vals;
                edge_samples(k, eo[k], xs, vals);
                const std::vector<xreal> Ie = interp_matrix(xs, xa);
                const int j = end ? pf : 0, pe = eo[k];
                for (int i = 0; i < pf; ++i)
                    for (int n = 0; n < 3; ++n) {
                        xreal v = 0.0L;
                        for (int m = 0; m < pe; ++m) v += Ie[i * pe + m] * vals[n * pe + m];
                        S[(n * pf + i) * (pf + 1) + j] = v;
                    }
            }
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) {
                    int i3[3];
                    i3[d] = side * (N - 1);
                    i3[c] = a;
                    i3[o] = b;
                    BoundaryValue bv{c, i3[0] + N * (i3[1] + N * i3[2]), {0, 0, 0}};
                    for (int n = 0; n < 3; ++n)
                        for (int i = 0; i < pf; ++i)
                            for (int j = 0; j <= pf; ++j)
                                bv.v[n] += Ia[a * pf + i] * Ib[b * (pf + 1) + j] * S[(n * pf + i) * (pf + 1) + j];
                    out.push_back(bv);
                }
        }
    }
}

}  // namespace

bool build_geometry(const hdg_mesh_desc &d, HostGeometry &g, std::string &msg, const std::vector<int32_t> *rep,
                    const BoundaryOrders *bo)
{
    const int Pg = d.geom_order, G1 = Pg + 1, G3 = G1 * G1 * G1;
    const int64_t ne = d.n_elem;
    // rules of every order in use, in extended precision
    std::vector<xreal> xqs[kMaxN + 1], wqs[kMaxN + 1], Dqs[kMaxN + 1], Is[kMaxN + 1];
    std::vector<xreal> gnodes(G1);
    for (int k = 0; k < G1; ++k) gnodes[k] = -1.0L + 2.0L * k / Pg;
    // derivative matrix on the geometry's equispaced nodes (barycentric weights)
    std::vector<xreal> Dg(G1 * G1, 0.0L), bwg(G1, 1.0L);
    for (int j = 0; j < G1; ++j)
        for (int k = 0; k < G1; ++k)
            if (k != j) bwg[j] /= (gnodes[j] - gnodes[k]);
    for (int i = 0; i < G1; ++i)
        for (int j = 0; j < G1; ++j)
            if (j != i) {
                Dg[i * G1 + j] = (bwg[j] / bwg[i]) / (gnodes[i] - gnodes[j]);
                Dg[i * G1 + i] -= Dg[i * G1 + j];
            }
    BoundaryOrders own_bo;
    if (!bo) {
        boundary_orders(d, own_bo);
        bo = &own_bo;
    }
    g.Ne.resize(ne);
    g.off.resize(ne);
    int64_t tot = 0;
    for (int64_t e = 0; e < ne; ++e) {
        const int N = d.P[e] + 1;
        g.Ne[e] = N;
        g.off[e] = tot;
        tot += (int64_t)N * N * N;
        if (xqs[N].empty()) {
            gll_rule_x(N - 1, xqs[N], wqs[N], Dqs[N]);
            Is[N] = interp_matrix(gnodes, xqs[N]);
        }
    }
    g.nodes = tot;
    g.N = g.Ne[0];
    g.N3 = g.N * g.N * g.N;
    for (int N = 2; N <= kMaxN; ++N) {
        if (xqs[N].empty()) continue;
        g.xis[N].assign(xqs[N].begin(), xqs[N].end());
        g.ws[N].assign(wqs[N].begin(), wqs[N].end());
        g.Ds[N].assign(Dqs[N].begin(), Dqs[N].end());
    }
    g.xi = g.xis[g.N];
    g.w = g.ws[g.N];
    g.D = g.Ds[g.N];
    // metric terms once per group of translates: slots for the groups'
    // first elements only (every element's own slot without groups)
    g.moff.assign(ne, 0);
    int64_t mtot = tot;
    if (rep) {
        mtot = 0;
        for (int64_t e = 0; e < ne; ++e)
            if ((*rep)[e] == e) {
                g.moff[e] = mtot;
                mtot += (int64_t)g.Ne[e] * g.Ne[e] * g.Ne[e];
            }
        for (int64_t e = 0; e < ne; ++e) g.moff[e] = g.moff[(*rep)[e]];
    } else {
        g.moff = g.off;
    }
    g.x.assign(tot * 3, 0.0);
    g.J.assign(mtot, 0.0);
    g.Ja.assign(mtot * 9, 0.0);
    g.delta.assign(ne, 0.0);
    std::atomic<int64_t> bad{-1};

    auto body = [&](int64_t e) {
        const int N = g.Ne[e], N3 = N * N * N;
        const std::vector<xreal> &wq = wqs[N], &Dq = Dqs[N], &I = Is[N];
        const int64_t o = g.off[e];
        std::vector<xreal> t1(N * G1 * G1), t2(N * N * G1), loc(3 * N3), dX(9 * N3), V(3 * N3), dV(9 * N3);
        std::vector<xreal> rel(G3);
        std::vector<BoundaryValue> bvals;
        const double *Xe = d.xyz_geom + e * 3 * G3;
        // geometry at the nodes, relative to the element's first control point
        // (the metric terms do not depend on a translation; this keeps their
        // round-off relative to the element size)
        for (int c = 0; c < 3; ++c) {
            for (int k = 0; k < G3; ++k) rel[k] = (xreal)Xe[c * G3 + k] - (xreal)Xe[c * G3];
            apply_dir(I, N, G1, 0, rel.data(), G1, G1, G1, t1.data());
            apply_dir(I, N, G1, 1, t1.data(), N, G1, G1, t2.data());
            apply_dir(I, N, G1, 2, t2.data(), N, N, G1, &loc[c * N3]);
            for (int n = 0; n < N3; ++n) g.x[3 * o + c * N3 + n] = (double)((xreal)Xe[c * G3] + loc[c * N3 + n]);
        }
        // a translate of another element shares its slot (and takes its filter
        // width in a second pass)
        if (rep && (*rep)[e] != e) return;
        const int64_t mo = g.moff[e];
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) apply_dir(Dq, N, N, k, &loc[c * N3], N, N, N, &dX[(c * 3 + k) * N3]);
        xreal vol = 0.0L;
        for (int n = 0; n < N3; ++n) {
            auto m = [&](int c, int k) { return dX[(c * 3 + k) * N3 + n]; };
            const xreal J = m(0, 0) * (m(1, 1) * m(2, 2) - m(1, 2) * m(2, 1))
                          - m(0, 1) * (m(1, 0) * m(2, 2) - m(1, 2) * m(2, 0))
                          + m(0, 2) * (m(1, 0) * m(2, 1) - m(1, 1) * m(2, 0));
            g.J[mo + n] = (double)J;
            const int a = n % N, b = (n / N) % N, c = n / (N * N);
            vol += wq[a] * wq[b] * wq[c] * J;
            if (!(J > 0.0L)) bad.store(e);
        }
        g.delta[e] = (double)(std::cbrt(vol) / N);
        // curl form: Ja^i_n = -(curl_xi (x_l grad_xi x_m))_i, (n, m, l) cyclic,
        // with the product field restricted where orders meet
        if (bo->any)
            boundary_values(Xe, Pg, gnodes, Dg, N, xqs[N], &bo->face[e * 6], &bo->edge[e * 12], bvals);
        for (int n = 0; n < 3; ++n) {
            const int mm = (n + 1) % 3, ll = (n + 2) % 3;
            for (int k = 0; k < 3; ++k)
                for (int p = 0; p < N3; ++p) V[k * N3 + p] = loc[ll * N3 + p] * dX[(mm * 3 + k) * N3 + p];
            for (const BoundaryValue &bv : bvals) V[bv.k * N3 + bv.p] = bv.v[n];
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j)
                    if (j != k) apply_dir(Dq, N, N, j, &V[k * N3], N, N, N, &dV[(k * 3 + j) * N3]);
            for (int p = 0; p < N3; ++p) {
                auto dv = [&](int k, int j) { return dV[(k * 3 + j) * N3 + p]; };
                g.Ja[9 * mo + (0 * 3 + n) * N3 + p] = (double)(-(dv(2, 1) - dv(1, 2)));
                g.Ja[9 * mo + (1 * 3 + n) * N3 + p] = (double)(-(dv(0, 2) - dv(2, 0)));
                g.Ja[9 * mo + (2 * 3 + n) * N3 + p] = (double)(-(dv(1, 0) - dv(0, 1)));
            }
        }
    };
    const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int64_t e = t; e < ne; e += nt) body(e);
        });
    for (auto &th : pool) th.join();
    if (rep)
        for (int64_t e = 0; e < ne; ++e) g.delta[e] = g.delta[(*rep)[e]];
    if (bad.load() >= 0) {
        msg = "non-positive Jacobian in element " + std::to_string(bad.load());
        return false;
    }
    return true;
}

namespace {

void bisect(std::vector<int32_t> &ids, size_t lo, size_t hi, const std::vector<double> &cen, int depth)
{
    if (hi - lo <= 32 || depth > 40) return;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (size_t i = lo; i < hi; ++i)
        for (int c = 0; c < 3; ++c) {
            mn[c] = std::min(mn[c], cen[3 * ids[i] + c]);
            mx[c] = std::max(mx[c], cen[3 * ids[i] + c]);
        }
    int ax = 0;
    for (int c = 1; c < 3; ++c)
        if (mx[c] - mn[c] > mx[ax] - mn[ax]) ax = c;
    size_t mid = lo + (hi - lo) / 2;
    std::nth_element(ids.begin() + lo, ids.begin() + mid, ids.begin() + hi, [&](int32_t a, int32_t b) {
        double va = cen[3 * a + ax], vb = cen[3 * b + ax];
        return va < vb || (va == vb && a < b);
    });
    bisect(ids, lo, mid, cen, depth + 1);
    bisect(ids, mid, hi, cen, depth + 1);
}

}  // namespace

std::vector<int32_t> locality_order(const hdg_mesh_desc &d, const std::vector<int32_t> *rep)
{
    const int G1 = d.geom_order + 1, G3 = G1 * G1 * G1;
    std::vector<double> cen(3 * (size_t)d.n_elem);
    for (int64_t e = 0; e < d.n_elem; ++e)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < G3; ++k) s += d.xyz_geom[(e * 3 + c) * G3 + k];
            cen[3 * e + c] = s / G3;
        }
    if (!rep) {
        std::vector<int32_t> ids(d.n_elem);
        std::iota(ids.begin(), ids.end(), 0);
        bisect(ids, 0, ids.size(), cen, 0);
        return ids;
    }
    // groups in bisection order of their mean centroids, members in id order
    std::vector<int32_t> gid(d.n_elem, -1), heads;
    std::vector<std::vector<int32_t>> members;
    for (int32_t e = 0; e < d.n_elem; ++e) {
        const int32_t r = (*rep)[e];
        if (gid[r] < 0) {
            gid[r] = (int32_t)heads.size();
            heads.push_back(r);
            members.emplace_back();
        }
        members[gid[r]].push_back(e);
    }
    std::vector<double> gc(3 * heads.size(), 0.0);
    for (size_t g = 0; g < heads.size(); ++g) {
        for (int32_t e : members[g])
            for (int c = 0; c < 3; ++c) gc[3 * g + c] += cen[3 * e + c];
        for (int c = 0; c < 3; ++c) gc[3 * g + c] /= (double)members[g].size();
    }
    std::vector<int32_t> gids(heads.size());
    std::iota(gids.begin(), gids.end(), 0);
    bisect(gids, 0, gids.size(), gc, 0);
    std::vector<int32_t> ids;
    ids.reserve(d.n_elem);
    for (int32_t g : gids)
        for (int32_t e : members[g]) ids.push_back(e);
    return ids;
}

int64_t metric_groups(const hdg_mesh_desc &d, std::vector<int32_t> &rep, const BoundaryOrders *bo)
{
    const int G1 = d.geom_order + 1, G3 = G1 * G1 * G1;
    rep.resize(d.n_elem);
    // key: the order and the relative control points rounded to 1e-10 of the
    // element's size; a hit is confirmed to 1e-12 of that size
    std::unordered_map<std::string, std::vector<int32_t>> buckets;
    std::vector<double> rel(3 * G3);
    std::string key;
    int64_t groups = 0;
    for (int32_t e = 0; e < d.n_elem; ++e) {
        double size = 0.0;
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < G3; ++k) {
                const double v = d.xyz_geom[((int64_t)e * 3 + c) * G3 + k] - d.xyz_geom[((int64_t)e * 3 + c) * G3];
                rel[c * G3 + k] = v;
                size = std::max(size, std::fabs(v));
            }
        key.assign((const char *)&d.P[e], sizeof(int32_t));
        if (bo && bo->any) {     // restricted boundaries are part of the metric terms
            key.append((const char *)&bo->face[e * 6], 6);
            key.append((const char *)&bo->edge[e * 12], 12);
        }
        for (double v : rel) {
            const int64_t q = (int64_t)std::llround(v / (1e-10 * size));
            key.append((const char *)&q, sizeof q);
        }
        auto &cand = buckets[key];
        int32_t found = -1;
        for (int32_t r : cand) {
            double dev = 0.0;
            for (int c = 0; c < 3; ++c)
                for (int k = 0; k < G3; ++k) {
                    const double vr = d.xyz_geom[((int64_t)r * 3 + c) * G3 + k] - d.xyz_geom[((int64_t)r * 3 + c) * G3];
                    dev = std::max(dev, std::fabs(vr - rel[c * G3 + k]));
                }
            if (dev <= 1e-12 * size) {
                found = r;
                break;
            }
        }
        if (found < 0) {
            cand.push_back(e);
            found = e;
            ++groups;
        }
        rep[e] = found;
    }
    return groups;
}

}  // namespace hdg
