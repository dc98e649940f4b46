// gfx950 kernels of the hybrid Navier-Stokes-LES / Euler DGSEM residual.
//
// One workgroup per element, one lane per collocation node (N^3 nodes rounded
// up to whole 64-lane waves).  Work is split by equation flag (Sec. 2.3):
//
//  k_viscous   (flagged elements only) lifts the velocity gradient (BR1:
//              volume derivative of Ja^i u plus a face correction towards the
//              mean of the two traces), evaluates the eddy viscosity and the
//              viscous stress 2 (nu + nu_t) S, and writes
//                - the viscous part of the element's reference divergence,
//                  -D F_v + (own-face flux)/w_end, 3 momentum rows per node,
//                - the viscous face traces tau . (s n) of its six faces, per
//                  face side, for the single-valued BR1 face flux;
//  k_residual  (every element) forms the contravariant convective fluxes in
//              LDS, takes their reference divergence, adds on face nodes the
//              jump between the single-valued numerical flux (Roe + BR1 mean
//              of the stored viscous traces) and its own flux over the end
//              weight, adds the viscous part on flagged elements, scales by
//              -1/J and writes R or applies a low-storage RK stage.
// This is the strong (summation-by-parts) equivalent of the weak form in
// App. B: on Gauss-Lobatto nodes the two agree to round-off.  Euler elements
// run no gradient, LES or viscous-flux arithmetic at all.
#include "hdg_internal.h"

namespace hdg {
namespace {

template <int N>
struct Shape {
    static constexpr int N2 = N * N;
    static constexpr int N3 = N * N * N;
    static constexpr int NT = ((N3 + 63) / 64) * 64;
};

// Workgroups are dealt to the XCDs round-robin; give every XCD a contiguous
// run of the (spatially ordered) element list so neighbour traces hit its L2.
__device__ __forceinline__ int xcd_slot(int per_xcd)
{
    const int b = blockIdx.x;
    return (b % kXcd) * per_xcd + b / kXcd;
}

template <int N>
__device__ __forceinline__ int face_node(int f, int a, int b)
{
    const int s = (f & 1) ? N - 1 : 0;
    const int d = f >> 1;
    return d == 0 ? s + N * (a + N * b) : d == 1 ? a + N * (s + N * b) : a + N * (b + N * s);
}

template <int N>
__device__ __forceinline__ void orient_map(int o, int a, int b, int &a2, int &b2)
{
    const int s = (o & 1) ? b : a, t = (o & 1) ? a : b;
    a2 = (o & 2) ? N - 1 - s : s;
    b2 = (o & 4) ? N - 1 - t : t;
}

// Roe flux of the artificial-compressibility system along the unit normal n
// (Sec. 2.3: Roe Riemann solver).  The mean-state Jacobian has eigenvalues
// u_n (twice, tangential) and u_n +- a, a = sqrt(u_n^2 + c0^2); the jump is
// projected on its eigenvectors in closed form.
__device__ __forceinline__ void roe_flux(double c0sq, const double (&qL)[4], const double (&qR)[4],
                                         const double (&n)[3], double (&F)[4])
{
    const double unL = qL[1] * n[0] + qL[2] * n[1] + qL[3] * n[2];
    const double unR = qR[1] * n[0] + qR[2] * n[1] + qR[3] * n[2];
    const double ub[3] = {0.5 * (qL[1] + qR[1]), 0.5 * (qL[2] + qR[2]), 0.5 * (qL[3] + qR[3])};
    const double un = ub[0] * n[0] + ub[1] * n[1] + ub[2] * n[2];
    const double a = sqrt(un * un + c0sq);
    const double ia = 1.0 / a;
    const double dp = qR[0] - qL[0];
    const double du[3] = {qR[1] - qL[1], qR[2] - qL[2], qR[3] - qL[3]};
    const double s = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    const double pip = a - un, pim = -a - un;
    const double alp = 0.5 * ia * (dp - pim * s);     // acoustic wave un + a
    const double alm = 0.5 * ia * (pip * s - dp);     // acoustic wave un - a
    const double lp = (un + a) * alp, lm = (a - un) * alm, l0 = fabs(un);
    F[0] = 0.5 * (c0sq * (unL + unR) - (lp * pip + lm * pim));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double vp = (pip * n[d] + ub[d]) * ia;
        const double vm = -(pim * n[d] + ub[d]) * ia;
        const double tang = du[d] - alp * vp - alm * vm;
        const double flux = qL[1 + d] * unL + qR[1 + d] * unR + (qL[0] + qR[0]) * n[d];
        F[1 + d] = 0.5 * (flux - (lp * vp + lm * vm + l0 * tang));
    }
}

// LES eddy viscosity from the velocity gradient G[r][d] = du_r/dx_d
// (App. A: Vreman, unit density; Smagorinsky as the alternative closure).
__device__ __forceinline__ double les_nut(int model, double C, double delta, const double (&G)[3][3])
{
    if (model == HDG_LES_SMAGORINSKY) {
        double ss = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double sd = 0.5 * (G[r][d] + G[d][r]);
                ss += sd * sd;
            }
        const double cd = C * delta;
        return cd * cd * sqrt(2.0 * ss);
    }
    if (model == HDG_LES_VREMAN) {
        // alpha_ij = du_j/dx_i = G[j][i]; beta_ij = Delta^2 sum_m G[i][m] G[j][m]
        double b[3][3], aa = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) aa += G[r][d] * G[r][d];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                b[i][j] = delta * delta * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
        double B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2]
                 + b[1][1] * b[2][2] - b[1][2] * b[1][2];
        B = B > 0.0 ? B : 0.0;
        return aa > 0.0 ? C * sqrt(B / aa) : 0.0;
    }
    return 0.0;
}

// Outside state at a face node: neighbour's trace or boundary ghost.
// Returns the coordinates of the node in the face owner's ordering.
template <int N, int NF>
__device__ __forceinline__ void outside_state(const ElemArgs &A, const FaceRef &fr, int fa, int fb,
                                              const double (&q)[4], double (&qo)[NF], int &oa, int &ob)
{
    constexpr int N3 = Shape<N>::N3;
    const bool own = fr.code & kOwnerBit;
    oa = fa;
    ob = fb;
    if (fr.nbr >= 0) {
        int a2, b2;
        orient_map<N>(fr.code & 7, fa, fb, a2, b2);
        if (!own) { oa = a2; ob = b2; }
        const double *qn = A.q + (size_t)fr.nbr * 4 * N3 + face_node<N>((fr.code >> 3) & 7, a2, b2);
#pragma unroll
        for (int c = 0; c < NF; ++c) qo[c] = qn[(4 - NF + c) * N3];
    } else if (fr.nbr == HDG_WALL) {
#pragma unroll
        for (int c = 0; c < NF; ++c) qo[c] = (4 - NF + c == 0) ? q[0] : -q[4 - NF + c];
    } else {
#pragma unroll
        for (int c = 0; c < NF; ++c) qo[c] = A.qinf[4 - NF + c];
    }
}

template <int N>
struct ElemCtx {
    int e, tid, t, i, j, k;
    bool act;
    double q[4];
    double invJ;
    double Ja[3][3];
    double Dx[N], Dy[N], Dz[N];
};

// Common prologue: element id, own state and metric terms, derivative matrix in LDS.
// Returns false for workgroups past the end of the list (uniform per block).
template <int N>
__device__ __forceinline__ bool load_element(const ElemArgs &A, double *sD, ElemCtx<N> &c)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    const int slot = xcd_slot(A.per_xcd);
    if (slot >= A.count) return false;
    c.e = A.list[slot];
    c.tid = threadIdx.x;
    c.act = c.tid < N3;
    c.t = c.act ? c.tid : N3 - 1;
    c.i = c.t % N;
    c.j = (c.t / N) % N;
    c.k = c.t / N2;
    for (int x = c.tid; x < N2; x += blockDim.x) sD[x] = A.Dmat[x];
    const double *qe = A.q + (size_t)c.e * 4 * N3;
#pragma unroll
    for (int f = 0; f < 4; ++f) c.q[f] = qe[f * N3 + c.t];
    const double *me = A.metric + (size_t)c.e * 10 * N3;
    c.invJ = me[c.t];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int d = 0; d < 3; ++d) c.Ja[ii][d] = me[(1 + 3 * ii + d) * N3 + c.t];
    __syncthreads();
    return true;
}

// Rows of the derivative matrix for this lane's node (after load_element).
template <int N>
__device__ __forceinline__ void load_drows(const double *sD, ElemCtx<N> &c)
{
#pragma unroll
    for (int m = 0; m < N; ++m) {
        c.Dx[m] = sD[c.i * N + m];
        c.Dy[m] = sD[c.j * N + m];
        c.Dz[m] = sD[c.k * N + m];
    }
}

template <int N>
__device__ __forceinline__ FaceRef select_face(const FaceRef (&frs)[6], int f)
{
    FaceRef fr = frs[0];
    if (f == 1) fr = frs[1];
    if (f == 2) fr = frs[2];
    if (f == 3) fr = frs[3];
    if (f == 4) fr = frs[4];
    if (f == 5) fr = frs[5];
    return fr;
}

// Viscous operator of a flagged element.
//  1. face-node tasks gather the neighbours' velocity traces and this
//     element's outward s n (the face owner's normal, signed) into LDS;
//  2. BR1 lifted gradient: J G = sum_i D_i (Ja^i u) + on face nodes
//     (u* (s n) - u (+-Ja^dir)) / w_end, u* the mean of the two traces
//     (no-slip wall: ghost -u; far field: ghost u_inf);
//  3. eddy viscosity and stress tau = 2 (nu + nu_t) S;
//  4. viscous part of the reference divergence, -D F_v + (+-F_v^dir)/w_end on
//     face nodes, and the face traces tau . (s n) with the owner's normal.
template <int N>
__global__ __launch_bounds__(Shape<N>::NT) void k_viscous(ElemArgs A)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3, NT = Shape<N>::NT;
    constexpr int NFT = 6 * N2;
    constexpr int TPT = (NFT + NT - 1) / NT;
    __shared__ double lds[12 * N3];        // u, v, w and Ja; later the viscous contravariant fluxes
    __shared__ double sfu[3 * NFT];        // neighbour velocity trace per face node (interior faces), [r][task]
    __shared__ double sfn[3 * NFT];        // outward s n per face node, [d][task]
    __shared__ double sD[N2];
    ElemCtx<N> c;
    if (!load_element<N>(A, sD, c)) return;
    FaceRef frs[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) frs[f] = A.conn[(size_t)c.e * 6 + f];
    if (c.act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) lds[r * N3 + c.tid] = c.q[1 + r];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int d = 0; d < 3; ++d) lds[(3 + 3 * ii + d) * N3 + c.tid] = c.Ja[ii][d];
    }
#pragma unroll 1
    for (int kk = 0; kk < TPT; ++kk) {
        const int task = c.tid + kk * NT;
        if (task < NFT) {
            const int f = task / N2, fn = task % N2, fa = fn % N, fb = fn / N;
            const FaceRef fr = select_face<N>(frs, f);
            const bool own = fr.code & kOwnerBit;
            int oa = fa, ob = fb;
            if (fr.nbr >= 0) {
                int a2, b2;
                orient_map<N>(fr.code & 7, fa, fb, a2, b2);
                if (!own) { oa = a2; ob = b2; }
                const double *qn = A.q + (size_t)fr.nbr * 4 * N3 + face_node<N>((fr.code >> 3) & 7, a2, b2);
#pragma unroll
                for (int r = 0; r < 3; ++r) sfu[r * NFT + task] = qn[(1 + r) * N3];
            }
            const double *g = A.fgeo + ((size_t)fr.face * N2 + oa + N * ob) * 4;
            const double so = own ? g[3] : -g[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) sfn[d * NFT + task] = g[d] * so;
        }
    }
    __syncthreads();

    double G[3][3];
    {
        double JG[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) JG[r][d] = 0.0;
#pragma unroll 1
        for (int m = 0; m < N; ++m) {
            const int n0 = m + N * c.j + N2 * c.k, n1 = c.i + N * m + N2 * c.k, n2 = c.i + N * c.j + N2 * m;
            double u0[3], u1[3], u2[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                u0[r] = lds[r * N3 + n0];
                u1[r] = lds[r * N3 + n1];
                u2[r] = lds[r * N3 + n2];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double g0 = sD[c.i * N + m] * lds[(3 + d) * N3 + n0];
                const double g1 = sD[c.j * N + m] * lds[(6 + d) * N3 + n1];
                const double g2 = sD[c.k * N + m] * lds[(9 + d) * N3 + n2];
#pragma unroll
                for (int r = 0; r < 3; ++r) JG[r][d] += g0 * u0[r] + g1 * u1[r] + g2 * u2[r];
            }
        }
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
            if (c.act && (idx == 0 || idx == N - 1)) {
                const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
                const int task = f * N2 + (dir == 0 ? c.j : c.i) + N * (dir == 2 ? c.j : c.k);
                const FaceRef fr = select_face<N>(frs, f);
                double uo[3];
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    uo[r] = fr.nbr >= 0 ? sfu[r * NFT + task] : fr.nbr == HDG_WALL ? -c.q[1 + r] : A.qinf[1 + r];
                const double sf = (f & 1) ? 1.0 : -1.0;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const double ustar = 0.5 * (c.q[1 + r] + uo[r]);
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        JG[r][d] += (ustar * sfn[d * NFT + task] - c.q[1 + r] * sf * c.Ja[dir][d]) * A.inv_wend;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) G[r][d] = JG[r][d] * c.invJ;
    }
    double fv[3][3];
    {
        const double mu = A.nu + les_nut(A.les_model, A.C_les, A.delta[c.e], G);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) fv[r][d] = mu * (G[r][d] + G[d][r]);
    }
    __syncthreads();     // every lane is done reading u and Ja from lds
    if (c.act) {
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                lds[(ii * 3 + r) * N3 + c.tid] = c.Ja[ii][0] * fv[r][0] + c.Ja[ii][1] * fv[r][1] + c.Ja[ii][2] * fv[r][2];
    }
    __syncthreads();
    double W[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int m = 0; m < N; ++m) {
        const int n0 = m + N * c.j + N2 * c.k, n1 = c.i + N * m + N2 * c.k, n2 = c.i + N * c.j + N2 * m;
#pragma unroll
        for (int r = 0; r < 3; ++r)
            W[r] -= sD[c.i * N + m] * lds[r * N3 + n0] + sD[c.j * N + m] * lds[(3 + r) * N3 + n1] + sD[c.k * N + m] * lds[(6 + r) * N3 + n2];
    }
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
        if (c.act && (idx == 0 || idx == N - 1)) {
            const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
            const double sf = (f & 1) ? 1.0 : -1.0;
#pragma unroll
            for (int r = 0; r < 3; ++r) W[r] += sf * lds[(dir * 3 + r) * N3 + c.tid] * A.inv_wend;
            // face trace tau . (s n) with the face owner's outward normal
            const int fa = dir == 0 ? c.j : c.i;
            const int fb = dir == 2 ? c.j : c.k;
            const int task = f * N2 + fa + N * fb;
            const FaceRef fr = select_face<N>(frs, f);
            const bool own = fr.code & kOwnerBit;
            int oa = fa, ob = fb;
            if (!own) orient_map<N>(fr.code & 7, fa, fb, oa, ob);
            const double so = own ? 1.0 : -1.0;
            const double sn[3] = {sfn[task] * so, sfn[NFT + task] * so, sfn[2 * NFT + task] * so};
            double *out = A.fvt + ((size_t)fr.face * 2 + (own ? 0 : 1)) * 3 * N2 + oa + N * ob;
#pragma unroll
            for (int r = 0; r < 3; ++r) out[r * N2] = fv[r][0] * sn[0] + fv[r][1] * sn[1] + fv[r][2] * sn[2];
        }
    }
    if (c.act) {
        double *wv = A.wvis + (size_t)c.e * 3 * N3 + c.tid;
#pragma unroll
        for (int r = 0; r < 3; ++r) wv[r * N3] = W[r];
    }
}

// Single-valued numerical flux through one face node of element e, outward for
// e and multiplied by the surface scale: Roe on the two traces, minus the BR1
// mean of the stored viscous traces when a side is flagged.  Both elements of
// a face evaluate it with the owner's trace on the left and the owner's
// normal, so the two results are exact negatives of each other.
template <int N>
__device__ __forceinline__ void face_flux(const ElemArgs &A, int e, bool visc, int f, int fa, int fb,
                                          double (&F)[4], const FaceRef (&frs)[6])
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    FaceRef fr = frs[0];
    if (f == 1) fr = frs[1];
    if (f == 2) fr = frs[2];
    if (f == 3) fr = frs[3];
    if (f == 4) fr = frs[4];
    if (f == 5) fr = frs[5];
    const bool own = fr.code & kOwnerBit;
    const double *qe = A.q + (size_t)e * 4 * N3 + face_node<N>(f, fa, fb);
    double qm[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) qm[x] = qe[x * N3];
    double qo[4];
    int oa, ob;
    outside_state<N, 4>(A, fr, fa, fb, qm, qo, oa, ob);
    const int fnode = oa + N * ob;
    const double *g = A.fgeo + ((size_t)fr.face * N2 + fnode) * 4;
    const double nh[3] = {g[0], g[1], g[2]};
    const double s = g[3];
    const bool nb_visc = fr.nbr >= 0 && A.flag[fr.nbr];
    const bool visL = own ? visc : nb_visc;
    const bool visR = own ? nb_visc : visc;
    double tvL[3] = {0.0, 0.0, 0.0}, tvR[3] = {0.0, 0.0, 0.0};
    const double *tv = A.fvt + (size_t)fr.face * 6 * N2 + fnode;
    if (visL) {
#pragma unroll
        for (int r = 0; r < 3; ++r) tvL[r] = tv[r * N2];
    }
    if (visR && fr.nbr >= 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r) tvR[r] = tv[(3 + r) * N2];
    }
    double qL[4], qR[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        qL[x] = own ? qm[x] : qo[x];
        qR[x] = own ? qo[x] : qm[x];
    }
    roe_flux(A.c0sq, qL, qR, nh, F);
#pragma unroll
    for (int x = 0; x < 4; ++x) F[x] *= s;
    if (visL || visR) {
        // BR1: mean of the two sides' viscous traces (an Euler side contributes
        // zero); a boundary face takes the interior trace
        const bool keep = fr.nbr < 0 || A.mixed_face == 0 || (visL && visR);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double fvn = fr.nbr < 0 ? tvL[r] : 0.5 * (tvL[r] + tvR[r]);
            F[1 + r] -= keep ? fvn : 0.0;
        }
    }
    if (!own) {
#pragma unroll
        for (int x = 0; x < 4; ++x) F[x] = -F[x];
    }
}

template <int N, int EPI>
__global__ __launch_bounds__(Shape<N>::NT) void k_residual(ElemArgs A)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3, NT = Shape<N>::NT;
    constexpr int NFT = 6 * N2;                        // face-node tasks per element
    constexpr int TPT = (NFT + NT - 1) / NT;           // tasks per lane
    __shared__ double lds[12 * N3];                    // contravariant fluxes
    __shared__ double sface[4 * NFT];                  // numerical fluxes, outward, [row][face node]
    __shared__ double sD[N2];
    ElemCtx<N> c;
    if (!load_element<N>(A, sD, c)) return;
    const bool visc = A.flag[c.e] != 0;

    // contravariant convective fluxes F^i_row = sum_d Ja^i_d f_{row,d}
    {
        double f[4][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[0][d] = A.c0sq * c.q[1 + d];
#pragma unroll
            for (int r = 0; r < 3; ++r) f[1 + r][d] = c.q[1 + r] * c.q[1 + d] + (r == d ? c.q[0] : 0.0);
        }
        if (c.act) {
#pragma unroll
            for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                for (int row = 0; row < 4; ++row)
                    lds[(ii * 4 + row) * N3 + c.tid] =
                        c.Ja[ii][0] * f[row][0] + c.Ja[ii][1] * f[row][1] + c.Ja[ii][2] * f[row][2];
        }
    }

    FaceRef frs[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) frs[f] = A.conn[(size_t)c.e * 6 + f];
    // face-node tasks, spread evenly over the workgroup
#pragma unroll 1
    for (int k = 0; k < TPT; ++k) {
        const int task = c.tid + k * NT;
        if (task < NFT) {
            const int f = task / N2, fn = task % N2;
            double F[4];
            face_flux<N>(A, c.e, visc, f, fn % N, fn / N, F, frs);
#pragma unroll
            for (int row = 0; row < 4; ++row) sface[row * NFT + task] = F[row];
        }
    }
    double dq_old[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (EPI == (int)Epi::RkStage) {
        if (!A.first_stage) {
            const double *dqe = A.dq + (size_t)c.e * 4 * N3 + c.t;
#pragma unroll
            for (int row = 0; row < 4; ++row) dq_old[row] = dqe[row * N3];
        }
    }
    __syncthreads();
    load_drows<N>(sD, c);

    // reference divergence
    double V[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int n0 = m + N * c.j + N2 * c.k, n1 = c.i + N * m + N2 * c.k, n2 = c.i + N * c.j + N2 * m;
#pragma unroll
        for (int row = 0; row < 4; ++row)
            V[row] += c.Dx[m] * lds[row * N3 + n0] + c.Dy[m] * lds[(4 + row) * N3 + n1]
                    + c.Dz[m] * lds[(8 + row) * N3 + n2];
    }

    // face nodes: numerical flux minus own flux, over w_end
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
        if (c.act && (idx == 0 || idx == N - 1)) {
            const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
            const int fa = dir == 0 ? c.j : c.i;
            const int fb = dir == 2 ? c.j : c.k;
            const double sf = (f & 1) ? 1.0 : -1.0;
            const double *Fs = sface + f * N2 + fa + N * fb;
#pragma unroll
            for (int row = 0; row < 4; ++row)
                V[row] += (Fs[row * NFT] - sf * lds[(dir * 4 + row) * N3 + c.tid]) * A.inv_wend;
        }
    }

    if (!c.act) return;
    if (visc) {
        const double *wv = A.wvis + (size_t)c.e * 3 * N3 + c.tid;
#pragma unroll
        for (int r = 0; r < 3; ++r) V[1 + r] += wv[r * N3];
    }
    const size_t base = (size_t)c.e * 4 * N3 + c.tid;
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const double R = -V[row] * c.invJ;
        const size_t idx = base + (size_t)row * N3;
        if constexpr (EPI == (int)Epi::Residual) {
            A.out[idx] = R;
        } else {
            const double d = A.first_stage ? A.dt * R : A.rkA * dq_old[row] + A.dt * R;
            A.dq[idx] = d;
            A.out[idx] = c.q[row] + A.rkB * d;
        }
    }
}

// Per-block partial reductions over whole elements: sum(m r), sum(m r^2),
// max |r| per field, and a non-finite flag.  Fixed order, no atomics.
template <int N>
__global__ __launch_bounds__(256) void k_reduce_partial(const double *r, const double *mass, int64_t ne,
                                                        double *partials)
{
    constexpr int N3 = Shape<N>::N3;
    __shared__ double red[13][256];
    double acc[13];
#pragma unroll
    for (int x = 0; x < 13; ++x) acc[x] = 0.0;
    const int64_t total = ne * N3;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = p / N3, n = p % N3;
        const double m = mass[p];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double v = r[(e * 4 + f) * N3 + n];
            acc[f] += m * v;
            acc[4 + f] += m * v * v;
            const double av = fabs(v);
            acc[8 + f] = av > acc[8 + f] ? av : acc[8 + f];
            if (!isfinite(v)) acc[12] = 1.0;
        }
    }
#pragma unroll
    for (int x = 0; x < 13; ++x) red[x][threadIdx.x] = acc[x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int x = 0; x < 8; ++x) red[x][threadIdx.x] += red[x][threadIdx.x + w];
#pragma unroll
            for (int x = 8; x < 13; ++x) red[x][threadIdx.x] = fmax(red[x][threadIdx.x], red[x][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 13) partials[(size_t)blockIdx.x * 13 + threadIdx.x] = red[threadIdx.x][0];
}

// Final reduction of the per-block partials: 256 lanes, fixed order (lane x
// takes blocks x, x + 256, ...; then a tree), so results are deterministic.
__global__ __launch_bounds__(256) void k_reduce_final(const double *partials, int nblocks, double *out)
{
    __shared__ double red[13][256];
    double acc[13];
#pragma unroll
    for (int x = 0; x < 13; ++x) acc[x] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int x = 0; x < 13; ++x) {
            const double p = partials[(size_t)b * 13 + x];
            acc[x] = x < 8 ? acc[x] + p : fmax(acc[x], p);
        }
    }
#pragma unroll
    for (int x = 0; x < 13; ++x) red[x][threadIdx.x] = acc[x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int x = 0; x < 8; ++x) red[x][threadIdx.x] += red[x][threadIdx.x + w];
#pragma unroll
            for (int x = 8; x < 13; ++x) red[x][threadIdx.x] = fmax(red[x][threadIdx.x], red[x][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 13) out[threadIdx.x] = red[threadIdx.x][0];
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 2;
constexpr int kCopyBlock = 512;

// Streaming copy: every lane moves kCopyUnroll 16-byte chunks, both loads in
// flight before the first store (the fastest of the tile shapes measured on
// MI355X; 8 chunks x 256 lanes hits a pathological access pattern).
__global__ __launch_bounds__(kCopyBlock) void k_copy(u32x4 *dst, const u32x4 *src, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * (kCopyUnroll * kCopyBlock) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kCopyBlock;
        if (i < n16) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kCopyBlock;
        if (i < n16) dst[i] = v[u];
    }
}

template <int N>
hipError_t launch_viscous_n(const ElemArgs &a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_viscous<N>, dim3(kXcd * a.per_xcd), dim3(Shape<N>::NT), 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t launch_residual_n(Epi epi, const ElemArgs &a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    const dim3 grid(kXcd * a.per_xcd), block(Shape<N>::NT);
    if (epi == Epi::Residual) hipLaunchKernelGGL((k_residual<N, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_residual<N, 1>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t launch_reduce_n(const double *r, const double *mass, int64_t ne, double *partials, int nblocks,
                           double *final13, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partial<N>, dim3(nblocks), dim3(256), 0, s, r, mass, ne, partials);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partials, nblocks, final13);
    return hipGetLastError();
}

}  // namespace

#define HDG_DISPATCH_N(N, CALL)                                                       \
    switch (N) {                                                                       \
    case 2: return CALL(2);                                                            \
    case 3: return CALL(3);                                                            \
    case 4: return CALL(4);                                                            \
    case 5: return CALL(5);                                                            \
    case 6: return CALL(6);                                                            \
    case 7: return CALL(7);                                                            \
    case 8: return CALL(8);                                                            \
    default: return hipErrorInvalidValue;                                              \
    }

hipError_t launch_viscous(int N, const ElemArgs &a, hipStream_t s)
{
#define C_(n) launch_viscous_n<n>(a, s)
    HDG_DISPATCH_N(N, C_)
#undef C_
}

hipError_t launch_residual(int N, Epi epi, const ElemArgs &a, hipStream_t s)
{
#define C_(n) launch_residual_n<n>(epi, a, s)
    HDG_DISPATCH_N(N, C_)
#undef C_
}

hipError_t launch_reduce(int N, const double *r, const double *mass, int64_t n_elem, double *partials,
                         int nblocks, double *final13, hipStream_t s)
{
#define C_(n) launch_reduce_n<n>(r, mass, n_elem, partials, nblocks, final13, s)
    HDG_DISPATCH_N(N, C_)
#undef C_
}

hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t s)
{
    const int64_t n16 = nbytes / 16;
    if (n16 == 0) return hipSuccess;
    const int64_t blocks = (n16 + kCopyUnroll * kCopyBlock - 1) / (kCopyUnroll * kCopyBlock);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kCopyBlock), 0, s, (u32x4 *)dst, (const u32x4 *)src,
                       n16);
    return hipGetLastError();
}

}  // namespace hdg
