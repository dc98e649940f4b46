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
//              difference between the single-valued numerical flux (Roe +
//              BR1 mean of the stored viscous traces, Sec. 2.3) and its own
//              flux over the end weight, adds the viscous part on flagged
//              elements, scales by -1/J and writes R or applies a low-storage
//              RK stage.
// Derivatives act on deviations from a per-element reference state and the
// surface terms are formed from the trace jumps, so rounding errors scale
// with variations of the solution, not with its size; this is what keeps the
// FP32 instantiation accurate.
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

// LES eddy viscosity from the velocity gradient G[r][d] = du_r/dx_d
// (App. A: Vreman, unit density; Smagorinsky as the alternative closure).
template <class T>
__device__ __forceinline__ T les_nut(int model, T C, T delta, const T (&G)[3][3])
{
    if (model == HDG_LES_SMAGORINSKY) {
        T ss = T(0);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T sd = T(0.5) * (G[r][d] + G[d][r]);
                ss += sd * sd;
            }
        const T cd = C * delta;
        return cd * cd * sqrt(T(2) * ss);
    }
    if (model == HDG_LES_VREMAN) {
        // alpha_ij = du_j/dx_i = G[j][i]; beta_ij = Delta^2 sum_m G[i][m] G[j][m]
        T b[3][3], aa = T(0);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) aa += G[r][d] * G[r][d];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                b[i][j] = delta * delta * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
        T B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2]
            + b[1][1] * b[2][2] - b[1][2] * b[1][2];
        B = B > T(0) ? B : T(0);
        return aa > T(0) ? C * sqrt(B / aa) : T(0);
    }
    return T(0);
}

// Per-launch constants converted to the compute type.
template <class T>
struct Consts {
    T c0sq, nu, C_les, inv_wend, qinf[4];
    __device__ explicit Consts(const ElemArgs &A)
        : c0sq((T)A.c0sq), nu((T)A.nu), C_les((T)A.C_les), inv_wend((T)A.inv_wend),
          qinf{(T)A.qinf[0], (T)A.qinf[1], (T)A.qinf[2], (T)A.qinf[3]} {}
};

template <int N, class T>
struct ElemCtx {
    int e, tid, t, i, j, k;
    bool act;
    double qd[4];   // own state, FP64 (the RK stage accumulates in FP64)
    T q[4];         // own state in the compute type
    T qr[4];        // the element's reference state (its centre node) ...
    T qt[4];        // ... and this node's deviation from it, formed in FP64
    T invJ;
    T Ja[3][3];
};

// Common prologue: element id, own state and metric terms, derivative matrix in LDS.
// Returns false for workgroups past the end of the list (uniform per block).
//
// Volume derivatives act on deviations from a per-element reference state
// q_r: the flux of a constant state has zero discrete divergence (the curl-form
// metric terms satisfy the discrete metric identities), so subtracting it
// changes nothing in exact arithmetic, while the rounding error of the
// contraction scales with the deviation instead of the state.  The deviation
// is formed in FP64 before conversion to the compute type.
template <int N, class T>
__device__ __forceinline__ bool load_element(const ElemArgs &A, T *sD, ElemCtx<N, T> &c)
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
    const T *Dm = (const T *)A.Dmat;
    for (int x = c.tid; x < N2; x += blockDim.x) sD[x] = Dm[x];
    const double *qe = A.q + (size_t)c.e * 4 * N3;
    constexpr int cref = (N / 2) * (1 + N + N2);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const double ref = qe[f * N3 + cref];
        c.qd[f] = qe[f * N3 + c.t];
        c.q[f] = (T)c.qd[f];
        c.qr[f] = (T)ref;
        c.qt[f] = (T)(c.qd[f] - ref);
    }
    const T *me = (const T *)A.metric + (size_t)c.e * 10 * N3;
    c.invJ = me[c.t];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int d = 0; d < 3; ++d) c.Ja[ii][d] = me[(1 + 3 * ii + d) * N3 + c.t];
    __syncthreads();
    return true;
}

// The six face records of an element, loaded once per workgroup (uniform, so
// scalar loads) and kept in named fields: a private array indexed by a lane's
// face number would be placed in scratch memory.
struct Faces6 {
    FaceRef f0, f1, f2, f3, f4, f5;
    __device__ explicit Faces6(const FaceRef *c)
        : f0(c[0]), f1(c[1]), f2(c[2]), f3(c[3]), f4(c[4]), f5(c[5]) {}
    // field-wise selects on plain integers (a select of whole structs would
    // again go through memory)
    __device__ __forceinline__ FaceRef operator[](int f) const
    {
        FaceRef r;
        r.face = f == 0 ? f0.face : f == 1 ? f1.face : f == 2 ? f2.face : f == 3 ? f3.face : f == 4 ? f4.face : f5.face;
        r.nbr = f == 0 ? f0.nbr : f == 1 ? f1.nbr : f == 2 ? f2.nbr : f == 3 ? f3.nbr : f == 4 ? f4.nbr : f5.nbr;
        r.code = f == 0 ? f0.code : f == 1 ? f1.code : f == 2 ? f2.code : f == 3 ? f3.code : f == 4 ? f4.code : f5.code;
        r.pad = 0;
        return r;
    }
};

// Viscous operator of a flagged element.
//  1. face-node tasks form u* - u, half the jump to the other side's velocity
//     trace, in FP64 and stage it in LDS;
//  2. BR1 lifted gradient: J G = sum_i D_i (Ja^i (u - u_r)) + on face nodes
//     (u* - u) (+-Ja^dir) / w_end, u* the mean of the two traces (no-slip
//     wall: ghost -u; far field: ghost u_inf); +-Ja^dir is this element's
//     outward s n, the same face geometry as the face owner's normal;
//  3. eddy viscosity and stress tau = 2 (nu + nu_t) S;
//  4. viscous part of the reference divergence, -D F_v + (+-F_v^dir)/w_end on
//     face nodes, and the face traces tau . (s n) oriented by the face
//     owner's outward normal, staged in LDS and stored by face-node lanes so
//     that consecutive lanes write consecutive words.
template <int N, class T>
__global__ __launch_bounds__(Shape<N>::NT) void k_viscous(ElemArgs A)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3, NT = Shape<N>::NT;
    constexpr int NFT = 6 * N2;
    constexpr int TPT = (NFT + NT - 1) / NT;
    __shared__ T lds[12 * N3];        // u, v, w and Ja; later the viscous contravariant fluxes
    __shared__ T sfu[3 * NFT];        // [r][face node]: neighbour velocity trace, later tau . (s n)
    __shared__ T sD[N2];
    ElemCtx<N, T> c;
    if (!load_element<N, T>(A, sD, c)) return;
    const Consts<T> K(A);
    const Faces6 frs(A.conn + (size_t)c.e * 6);
    if (c.act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) lds[r * N3 + c.tid] = c.qt[1 + r];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int d = 0; d < 3; ++d) lds[(3 + 3 * ii + d) * N3 + c.tid] = c.Ja[ii][d];
    }
#pragma unroll 1
    for (int kk = 0; kk < TPT; ++kk) {
        const int task = c.tid + kk * NT;
        if (task < NFT) {
            // u* - u = (u_other - u) / 2, formed in FP64
            const int f = task / N2, fn = task % N2;
            const FaceRef fr = frs[f];
            const double *qm = A.q + (size_t)c.e * 4 * N3 + face_node<N>(f, fn % N, fn / N);
            double uo[3];
            if (fr.nbr >= 0) {
                int a2, b2;
                orient_map<N>(fr.code & 7, fn % N, fn / N, a2, b2);
                const double *qn = A.q + (size_t)fr.nbr * 4 * N3 + face_node<N>((fr.code >> 3) & 7, a2, b2);
#pragma unroll
                for (int r = 0; r < 3; ++r) uo[r] = qn[(1 + r) * N3];
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r) uo[r] = fr.nbr == HDG_WALL ? -qm[(1 + r) * N3] : A.qinf[1 + r];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) sfu[r * NFT + task] = (T)(0.5 * (uo[r] - qm[(1 + r) * N3]));
        }
    }
    __syncthreads();

    T G[3][3];
    {
        T JG[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) JG[r][d] = T(0);
#pragma unroll 1
        for (int m = 0; m < N; ++m) {
            const int n0 = m + N * c.j + N2 * c.k, n1 = c.i + N * m + N2 * c.k, n2 = c.i + N * c.j + N2 * m;
            T u0[3], u1[3], u2[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                u0[r] = lds[r * N3 + n0];
                u1[r] = lds[r * N3 + n1];
                u2[r] = lds[r * N3 + n2];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T g0 = sD[c.i * N + m] * lds[(3 + d) * N3 + n0];
                const T g1 = sD[c.j * N + m] * lds[(6 + d) * N3 + n1];
                const T g2 = sD[c.k * N + m] * lds[(9 + d) * N3 + n2];
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
                const T sf = (f & 1) ? T(1) : T(-1);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const T jump = sfu[r * NFT + task] * sf * K.inv_wend;
#pragma unroll
                    for (int d = 0; d < 3; ++d) JG[r][d] += jump * c.Ja[dir][d];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) G[r][d] = JG[r][d] * c.invJ;
    }
    T fv[3][3];
    {
        const T mu = K.nu + les_nut<T>(A.les_model, K.C_les, (T)A.delta[c.e], G);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) fv[r][d] = mu * (G[r][d] + G[d][r]);
    }
    __syncthreads();     // every lane is done reading u, Ja and the neighbour traces from lds
    if (c.act) {
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                lds[(ii * 3 + r) * N3 + c.tid] = c.Ja[ii][0] * fv[r][0] + c.Ja[ii][1] * fv[r][1] + c.Ja[ii][2] * fv[r][2];
    }
    __syncthreads();
    T W[3] = {T(0), T(0), T(0)};
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
            const T sf = (f & 1) ? T(1) : T(-1);
#pragma unroll
            for (int r = 0; r < 3; ++r) W[r] += sf * lds[(dir * 3 + r) * N3 + c.tid] * K.inv_wend;
            // tau . (s n) with the owner's outward normal: +-(this element's outward)
            const int task = f * N2 + (dir == 0 ? c.j : c.i) + N * (dir == 2 ? c.j : c.k);
            const FaceRef fr = frs[f];
            const T so = (fr.code & kOwnerBit) ? sf : -sf;
            const T sn[3] = {so * c.Ja[dir][0], so * c.Ja[dir][1], so * c.Ja[dir][2]};
#pragma unroll
            for (int r = 0; r < 3; ++r) sfu[r * NFT + task] = fv[r][0] * sn[0] + fv[r][1] * sn[1] + fv[r][2] * sn[2];
        }
    }
    if (c.act) {
        T *wv = (T *)A.wvis + (size_t)c.e * 3 * N3 + c.tid;
#pragma unroll
        for (int r = 0; r < 3; ++r) wv[r * N3] = W[r];
    }
    __syncthreads();
    T *fvt = (T *)A.fvt;
#pragma unroll 1
    for (int kk = 0; kk < TPT; ++kk) {
        const int task = c.tid + kk * NT;
        if (task < NFT) {
            const int f = task / N2, fn = task % N2;
            const FaceRef fr = frs[f];
            const bool own = fr.code & kOwnerBit;
            int oa = fn % N, ob = fn / N;
            if (!own) orient_map<N>(fr.code & 7, fn % N, fn / N, oa, ob);
            T *out = fvt + ((size_t)fr.face * 2 + (own ? 0 : 1)) * 3 * N2 + oa + N * ob;
#pragma unroll
            for (int r = 0; r < 3; ++r) out[r * N2] = sfu[r * NFT + task];
        }
    }
}

// Surface term of one face node of element e: the single-valued numerical flux
// minus e's own flux, both outward for e and multiplied by the surface scale.
// Both elements of a face work with the owner's trace on the left (q_L), the
// jump dq = q_R - q_L formed in FP64, and the owner's unit normal n:
//   Roe:  F* = (F_n(q_L) + F_n(q_R))/2 - |A(q_mean)| dq / 2,
//   so    F* - F_n(q_L) = (dF - |A| dq)/2  and  F_n(q_R) - F* = (dF + |A| dq)/2,
// with dF = F_n(q_R) - F_n(q_L) = [c0^2 du_n ; u_L du_n + du u_R,n + dp n]
// exact for the quadratic artificial-compressibility flux, so every term is
// proportional to the jump.  The BR1 viscous flux is the mean of the stored
// viscous traces when a side is flagged.  The non-owner sees -F*, and the two
// sides' implied fluxes are exact negatives in exact arithmetic.
template <int N, class T>
__device__ __forceinline__ void face_jump(const ElemArgs &A, const Consts<T> &K, int e, bool visc, int f, int fa,
                                          int fb, T (&F)[4], const Faces6 &frs)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    const FaceRef fr = frs[f];
    const bool own = fr.code & kOwnerBit;
    const double *qe = A.q + (size_t)e * 4 * N3 + face_node<N>(f, fa, fb);
    double qm[4], qo[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) qm[x] = qe[x * N3];
    int oa = fa, ob = fb;
    if (fr.nbr >= 0) {
        int a2, b2;
        orient_map<N>(fr.code & 7, fa, fb, a2, b2);
        if (!own) { oa = a2; ob = b2; }
        const double *qn = A.q + (size_t)fr.nbr * 4 * N3 + face_node<N>((fr.code >> 3) & 7, a2, b2);
#pragma unroll
        for (int x = 0; x < 4; ++x) qo[x] = qn[x * N3];
    } else if (fr.nbr == HDG_WALL) {
        qo[0] = qm[0];
#pragma unroll
        for (int x = 1; x < 4; ++x) qo[x] = -qm[x];
    } else {
#pragma unroll
        for (int x = 0; x < 4; ++x) qo[x] = A.qinf[x];
    }
    const int fnode = oa + N * ob;
    const T *g = (const T *)A.fgeo + ((size_t)fr.face * N2 + fnode) * 4;
    const T n[3] = {g[0], g[1], g[2]};
    const T sc = g[3];
    T uL[3], du[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        uL[d] = (T)(own ? qm[1 + d] : qo[1 + d]);
        du[d] = (T)(own ? qo[1 + d] - qm[1 + d] : qm[1 + d] - qo[1 + d]);
    }
    const T dp = (T)(own ? qo[0] - qm[0] : qm[0] - qo[0]);
    const T h = T(0.5);
    const T uLn = uL[0] * n[0] + uL[1] * n[1] + uL[2] * n[2];
    const T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    const T uRn = uLn + dun;
    // mean-state eigen-decomposition of |A| dq (eigenvalues u_n, u_n, u_n +- a)
    const T un = uLn + h * dun;
    const T a = sqrt(un * un + K.c0sq);
    const T ia = T(1) / a;
    const T pip = a - un, pim = -a - un;
    const T alp = h * ia * (dp - pim * dun);   // acoustic wave u_n + a
    const T alm = h * ia * (pip * dun - dp);   // acoustic wave u_n - a
    const T lp = (un + a) * alp, lm = (a - un) * alm, l0 = fabs(un);
    const T sg = own ? T(-1) : T(1);           // -|A| dq for the owner, + for the other side
    F[0] = h * sc * (K.c0sq * dun + sg * (lp * pip + lm * pim));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T ub = uL[d] + h * du[d];
        const T vp = (pip * n[d] + ub) * ia;
        const T vm = -(pim * n[d] + ub) * ia;
        const T tang = du[d] - alp * vp - alm * vm;
        const T dF = uL[d] * dun + du[d] * uRn + dp * n[d];
        F[1 + d] = h * sc * (dF + sg * (lp * vp + lm * vm + l0 * tang));
    }
    const bool nb_visc = fr.nbr >= 0 && A.flag[fr.nbr];
    const bool visL = own ? visc : nb_visc;
    const bool visR = own ? nb_visc : visc;
    if (visL || visR) {
        // BR1: mean of the two sides' viscous traces (an Euler side contributes
        // zero); a boundary face takes the interior trace.  F* carries -F_v*.
        const bool keep = fr.nbr < 0 || A.mixed_face == 0 || (visL && visR);
        const T *tv = (const T *)A.fvt + (size_t)fr.face * 6 * N2 + fnode;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const T tL = visL ? tv[r * N2] : T(0);
            const T tR = (visR && fr.nbr >= 0) ? tv[(3 + r) * N2] : T(0);
            const T fvn = fr.nbr < 0 ? tL : h * (tL + tR);
            F[1 + r] += keep ? sg * fvn : T(0);
        }
    }
}

template <int N, int EPI, class T>
__global__ __launch_bounds__(Shape<N>::NT) void k_residual(ElemArgs A)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3, NT = Shape<N>::NT;
    constexpr int NFT = 6 * N2;                        // face-node tasks per element
    constexpr int TPT = (NFT + NT - 1) / NT;           // tasks per lane
    __shared__ T lds[12 * N3];                         // contravariant fluxes
    __shared__ T sface[4 * NFT];                       // surface terms F* - F_own, [row][face node]
    __shared__ T sD[N2];
    ElemCtx<N, T> c;
    if (!load_element<N, T>(A, sD, c)) return;
    const Consts<T> K(A);
    const bool visc = A.flag[c.e] != 0;

    // contravariant convective fluxes F^i_row = sum_d Ja^i_d f_{row,d} of the
    // deviation f(q) - f(q_r): c0^2 (u - u_r) and
    // u u^T - u_r u_r^T + (p - p_r) I = u (u - u_r)^T + (u - u_r) u_r^T + (p - p_r) I
    {
        T f[4][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[0][d] = K.c0sq * c.qt[1 + d];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                f[1 + r][d] = c.q[1 + r] * c.qt[1 + d] + c.qt[1 + r] * c.qr[1 + d] + (r == d ? c.qt[0] : T(0));
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

    const Faces6 frs(A.conn + (size_t)c.e * 6);
    // face-node tasks, spread evenly over the workgroup
#pragma unroll 1
    for (int k = 0; k < TPT; ++k) {
        const int task = c.tid + k * NT;
        if (task < NFT) {
            const int f = task / N2, fn = task % N2;
            T F[4];
            face_jump<N, T>(A, K, c.e, visc, f, fn % N, fn / N, F, frs);
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
    T Dx[N], Dy[N], Dz[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        Dx[m] = sD[c.i * N + m];
        Dy[m] = sD[c.j * N + m];
        Dz[m] = sD[c.k * N + m];
    }

    // reference divergence
    T V[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int n0 = m + N * c.j + N2 * c.k, n1 = c.i + N * m + N2 * c.k, n2 = c.i + N * c.j + N2 * m;
#pragma unroll
        for (int row = 0; row < 4; ++row)
            V[row] += Dx[m] * lds[row * N3 + n0] + Dy[m] * lds[(4 + row) * N3 + n1] + Dz[m] * lds[(8 + row) * N3 + n2];
    }

    // face nodes: numerical flux minus own flux, over w_end
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
        if (c.act && (idx == 0 || idx == N - 1)) {
            const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
            const int fa = dir == 0 ? c.j : c.i;
            const int fb = dir == 2 ? c.j : c.k;
            const T *Fs = sface + f * N2 + fa + N * fb;
#pragma unroll
            for (int row = 0; row < 4; ++row) V[row] += Fs[row * NFT] * K.inv_wend;
        }
    }

    if (!c.act) return;
    if (visc) {
        const T *wv = (const T *)A.wvis + (size_t)c.e * 3 * N3 + c.tid;
#pragma unroll
        for (int r = 0; r < 3; ++r) V[1 + r] += wv[r * N3];
    }
    const size_t base = (size_t)c.e * 4 * N3 + c.tid;
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const T R = -V[row] * c.invJ;
        const size_t idx = base + (size_t)row * N3;
        if constexpr (EPI == (int)Epi::Residual) {
            ((T *)A.out)[idx] = R;
        } else {
            // FP64 stage accumulation into the state
            const double Rd = (double)R;
            const double d = A.first_stage ? A.dt * Rd : A.rkA * dq_old[row] + A.dt * Rd;
            A.dq[idx] = d;
            ((double *)A.out)[idx] = c.qd[row] + A.rkB * d;
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
hipError_t launch_viscous_n(bool f32, const ElemArgs &a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    const dim3 grid(kXcd * a.per_xcd), block(Shape<N>::NT);
    if (f32) hipLaunchKernelGGL((k_viscous<N, float>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_viscous<N, double>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t launch_residual_n(Epi epi, bool f32, const ElemArgs &a, hipStream_t s)
{
    if (a.count == 0) return hipSuccess;
    const dim3 grid(kXcd * a.per_xcd), block(Shape<N>::NT);
    if (f32) {
        if (epi == Epi::Residual) hipLaunchKernelGGL((k_residual<N, 0, float>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_residual<N, 1, float>), grid, block, 0, s, a);
    } else {
        if (epi == Epi::Residual) hipLaunchKernelGGL((k_residual<N, 0, double>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_residual<N, 1, double>), grid, block, 0, s, a);
    }
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

hipError_t launch_viscous(int N, bool f32, const ElemArgs &a, hipStream_t s)
{
#define C_(n) launch_viscous_n<n>(f32, a, s)
    HDG_DISPATCH_N(N, C_)
#undef C_
}

hipError_t launch_residual(int N, Epi epi, bool f32, const ElemArgs &a, hipStream_t s)
{
#define C_(n) launch_residual_n<n>(epi, f32, a, s)
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
