// gfx950 kernels of the hybrid Navier-Stokes-LES / Euler DGSEM residual.
//
// Work comes as a list of tiles.  A tile holds up to tile_ept() elements of
// one order N and one equation class from one member mesh; one workgroup of B
// lanes takes it, one lane per collocation node (element s of the tile owns
// lanes [s N^3, (s+1) N^3)).  Each launch is persistent: a fixed grid walks
// the whole tile list, every order and every member mesh of the batch, in one
// dispatch.  Work is split by equation flag (Sec. 2.3):
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
//
// This is the strong (summation-by-parts) equivalent of the weak form in
// App. B: on Gauss-Lobatto nodes the two agree to round-off.  Euler elements
// run no gradient, LES or viscous-flux arithmetic at all.
#include "hdg_internal.h"

#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>

// Scratch of the allocation-free reduction (hdg_reduce_noalloc): the
// per-workgroup partial sums, kReduceScratchBlocks x 13 doubles (104 KiB).
// Each GPU the library runs on holds one copy until the process ends.  Host
// code never passes this name to a kernel (on the host it is a stand-in, not a
// device address): it uses the address scratch_address() obtained with
// hipGetSymbolAddress on that device.
static __device__ __align__(256) double scratch[hdg::kReduceScratchBlocks * 13];

namespace hdg {
namespace {

template <int N>
struct Shape {
    static constexpr int N2 = N * N;
    static constexpr int N3 = N * N * N;
};

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

// Pointers read from the member table are generic pointers to the compiler;
// casting them through the global address space lets it emit global (not
// flat) memory instructions with scalar bases.
template <class T>
using gmem = __attribute__((address_space(1))) T;

template <class P>
__device__ __forceinline__ gmem<P> *gp(P *p)
{
    return (gmem<P> *)p;
}

// First node of element e: a table on a mesh of mixed order, a plain
// product when every element has order N (the table is then absent).  On
// the hot paths the tile-list entry (eoe) and the face records carry these
// offsets, so no table lookup sits between a record and the loads it
// addresses; the table serves the batch and clustering paths.
template <int N>
__device__ __forceinline__ int64_t elem_off(const Member &M, int e)
{
    return M.eoff ? gp(M.eoff)[e] : (int64_t)e * (N * N * N);
}

// A conforming face's first face node: on a mesh of mixed order the record
// holds it (no lookup), on a one-order mesh it is f N^2.
template <int N>
__device__ __forceinline__ int64_t face_first(bool mixed, const FaceRef &r)
{
    return mixed ? (int64_t)r.face : (int64_t)r.face * (N * N);
}

// The neighbour's first node across a conforming face (record on a mesh of
// mixed order, nbr N^3 otherwise).
template <int N>
__device__ __forceinline__ int64_t nbr_first(bool mixed, const FaceRef &r)
{
    return mixed ? (int64_t)r.nbr_off : (int64_t)r.nbr * (N * N * N);
}

// A mortar face's slab and the two sides' orders, from the element's own
// order and its face record (no load of the mortar's record).
struct MortarSide {
    int64_t slab;
    int Nh, Nl;
    bool hi;
};

template <int N>
__device__ __forceinline__ MortarSide mortar_side(const FaceRef &r)
{
    MortarSide m;
    const int other = r.code & 15;
    m.hi = (r.code & kOwnerBit) != 0;
    m.slab = (int64_t)(uint32_t)r.nbr_off;
    m.Nh = m.hi ? N : other;
    m.Nl = m.hi ? other : N;
    return m;
}

__device__ __forceinline__ FaceRef load_face(const FaceRef *conn, size_t i)
{
    typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
    const i32x4 v = *(gp((const i32x4 *)conn) + i);      // one 16-byte load
    FaceRef r;
    r.face = v.x;
    r.nbr = v.y;
    r.code = v.z;
    r.nbr_off = v.w;
    return r;
}

template <class T> __device__ __forceinline__ const T *dtable(const StageArgs &A);
template <> __device__ __forceinline__ const double *dtable<double>(const StageArgs &A) { return A.D64; }
template <> __device__ __forceinline__ const float *dtable<float>(const StageArgs &A) { return A.D32; }
template <class T> constexpr int prec_index() { return sizeof(T) == 4 ? 1 : 0; }
template <class T> __device__ __forceinline__ const T *itable(const StageArgs &A);
template <> __device__ __forceinline__ const double *itable<double>(const StageArgs &A) { return A.I64; }
template <> __device__ __forceinline__ const float *itable<float>(const StageArgs &A) { return A.I32; }
template <class T> __device__ __forceinline__ const T *wtable(const StageArgs &A);
template <> __device__ __forceinline__ const double *wtable<double>(const StageArgs &A) { return A.W64; }
template <> __device__ __forceinline__ const float *wtable<float>(const StageArgs &A) { return A.W32; }

__device__ __forceinline__ MortarRef load_mortar(const MortarRef *mr, int m)
{
    const gmem<const int32_t> *p = gp((const int32_t *)(mr + m));
    MortarRef r;
    r.eh = p[0]; r.fh = p[1]; r.el = p[2]; r.fl = p[3];
    r.Nh = p[4]; r.Nl = p[5]; r.code_h = p[6]; r.flags = p[7];
    const gmem<const int64_t> *p64 = gp((const int64_t *)(mr + m)) + 4;
    r.slab = p64[0];
    r.geo = p64[1];
    r.oh = p64[2];
    r.ol = p64[3];
    return r;
}

// One lane's view of its element and node within a tile.
template <int N, class T>
struct TileCtx {
    int tid, s, t, i, j, k;
    int g;            // s N^3 + t: node index in the tile's LDS arrays
    bool act;         // the lane holds a node of a real element
    int e;            // member-local element id
    int64_t eo;       // first node of the element
    double qd[4];     // own state, FP64 (the RK stage accumulates in FP64)
    T q[4];           // own state in the compute type
    T qr[4];          // the element's reference state (its centre node) ...
    T qt[4];          // ... and this node's deviation from it, formed in FP64
    T invJ;
    T Ja[3][3];
    T c0sq, nu, C_les, inv_wend;
    const gmem<double> *qin;
};

// Common prologue: element and node of this lane, own state and metric terms,
// derivative matrix in LDS.  Lanes past an element's nodes or the tile's
// elements take the last node of an element of the tile (reads only).
//
// Volume derivatives act on deviations from a per-element reference state
// q_r: the flux of a constant state has zero discrete divergence (the curl-form
// metric terms satisfy the discrete metric identities), so subtracting it
// changes nothing in exact arithmetic, while the rounding error of the
// contraction scales with the deviation instead of the state.  The deviation
// is formed in FP64 before conversion to the compute type.
// Element ids and face records of a tile's elements, staged in LDS once per
// tile so that face tasks and face-node lanes read them without a dependent
// global load.
template <int EPT>
struct TileFaces {
    int32_t e[EPT];
    int64_t eo[EPT];          // the elements' first nodes
    FaceRef f[6 * EPT];
};

// With STAGE_Q the own state is also staged in LDS, FP64 [4][EPT N^3] at
// the start of smem, for face tasks to read instead of gathering it again.
// With sjf, each face node's Ja^dir is staged there too, [3][EPT 6 N^2] in
// face-task order, for the face tasks' normals.
template <int N, int EPT, class T, bool STAGE_Q = false>
__device__ __forceinline__ void load_tile(const StageArgs &A, const Member &M, const Tile &tl, T *sD,
                                          TileFaces<EPT> &tf, TileCtx<N, T> &c, double *sq = nullptr,
                                          T *sjf = nullptr)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3, NL = tile_lanes(N);
    c.tid = threadIdx.x;
    const int raw = c.tid / NL, within = c.tid - raw * NL;
    c.act = raw < tl.count && within < N3;
    c.s = raw < tl.count ? raw : tl.count - 1;
    // from N = 4 on an element spans whole waves: its slot is wave-uniform
    if constexpr (NL % 64 == 0) c.s = __builtin_amdgcn_readfirstlane(c.s);
    c.t = c.act ? within : N3 - 1;
    c.g = c.s * N3 + c.t;
    c.i = c.t % N;
    c.j = (c.t / N) % N;
    c.k = c.t / N2;
    c.e = A.elems[tl.first + c.s];
    c.eo = A.eoe ? A.eoe[tl.first + c.s] : elem_off<N>(M, c.e);
    // Loads are issued before any LDS write that needs one of them: the load
    // counter is in order, so the metric terms, issued last and needed last,
    // stay in flight across the barrier while face tasks start.  The first
    // pass of the derivative-matrix and face-record copies goes through
    // registers for that reason (N^2 <= 64 and 7 EPT < EPT N^3 never exceed a
    // workgroup, whose size is at least 128), with unconditional loads at clamped indices: a branch that
    // wrote the destination registers instead would have to wait for them.
    const T *Dm = dtable<T>(A) + d_offset(N);
    const T dval = Dm[c.tid < N2 ? c.tid : N2 - 1];
    const int rs = c.tid < EPT ? c.tid : (c.tid - EPT) / 6;            // element slot of the record
    // one element per tile: its id is the lane's own (a scalar load), so the
    // record load does not wait on a vector load
    const int32_t rel = EPT == 1 ? c.e : A.elems[tl.first + (rs < tl.count ? rs : tl.count - 1)];
    // the record lanes' element's first node, for face tasks (EPT > 1)
    const int64_t reo = EPT == 1 ? c.eo
                        : A.eoe ? A.eoe[tl.first + (rs < tl.count ? rs : tl.count - 1)] : elem_off<N>(M, rel);
    const FaceRef rrec = load_face(M.conn, (size_t)rel * 6 + (c.tid < EPT ? 0 : (c.tid - EPT) - 6 * rs));
    c.qin = gp((const double *)(A.q_in ? A.q_in : (A.parity ? M.qB : M.qA)));
    const gmem<double> *qe = c.qin + 4 * c.eo;
    constexpr int cref = (N / 2) * (1 + N + N2);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const double ref = qe[f * N3 + cref];
        c.qd[f] = qe[f * N3 + c.t];
        c.q[f] = (T)c.qd[f];
        c.qr[f] = (T)ref;
        c.qt[f] = (T)(c.qd[f] - ref);
    }
    // translates of one element share its metric block; the tile plan holds
    // the block of each entry beside its element id (one dependent load fewer)
    const int64_t mo = A.emo ? A.emo[tl.first + c.s] : M.moff ? gp(M.moff)[c.e] : c.eo;
    const gmem<const T> *me = gp((const T *)M.metric[prec_index<T>()]) + 10 * mo;
    c.invJ = me[c.t];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int d = 0; d < 3; ++d) c.Ja[ii][d] = me[(1 + 3 * ii + d) * N3 + c.t];
    c.c0sq = (T)M.c0sq;
    c.nu = (T)M.nu;
    c.C_les = (T)M.C_les;
    c.inv_wend = T(N * (N - 1) / 2);   // 1 / w_0 = P (P + 1) / 2
    if (c.tid < N2) sD[c.tid] = dval;
    if (c.tid < EPT) {
        tf.e[c.tid] = c.tid < tl.count ? rel : 0;
        tf.eo[c.tid] = c.tid < tl.count ? reo : 0;
    }
    else if (c.tid < 7 * EPT) tf.f[c.tid - EPT] = rs < tl.count ? rrec : FaceRef{0, HDG_WALL, 0, 0};
    if constexpr (STAGE_Q) {
        if (c.act) {
#pragma unroll
            for (int f = 0; f < 4; ++f) sq[f * (EPT * N3) + c.g] = c.qd[f];
        }
    }
    if (sjf && c.act) {
        constexpr int NTASK = EPT * 6 * N2;
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
            if (idx == 0 || idx == N - 1) {
                const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
                const int task = c.s * 6 * N2 + f * N2 + (dir == 0 ? c.j : c.i) + N * (dir == 2 ? c.j : c.k);
#pragma unroll
                for (int d = 0; d < 3; ++d) sjf[d * NTASK + task] = c.Ja[dir][d];
            }
        }
    }
    __syncthreads();
}

// Face-node task of a tile: element slot, element id, face, face coordinates.
template <int N>
struct FaceTask {
    int s, e, f, fa, fb;
};

template <int N, int EPT>
__device__ __forceinline__ FaceTask<N> face_task(const TileFaces<EPT> &tf, const Tile &tl, int task)
{
    constexpr int N2 = Shape<N>::N2, NFT = 6 * N2;
    FaceTask<N> ft;
    ft.s = EPT == 1 ? 0 : task / NFT;       // one element: its id stays uniform
    const int r = task - ft.s * NFT;
    ft.f = r / N2;
    const int fn = r - ft.f * N2;
    ft.fa = fn % N;
    ft.fb = fn / N;
    ft.e = tf.e[ft.s];
    return ft;
}

// Viscous operator of the flagged elements of one tile.
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
template <int N, int EPT, class T, bool FEAT = false>
__device__ __forceinline__ void viscous_tile(const StageArgs &A, const Tile &tl, char *smem)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    constexpr int NFT = 6 * N2, NN = EPT * N3, NTASK = EPT * NFT;
    T *lds = (T *)smem;               // [12][NN]: u - u_r, v - v_r, w - w_r and Ja; later F_v
    T *sfu = lds + 12 * NN;           // [3][NTASK]: half jumps, later tau . (s n)
    T *sD = sfu + 3 * NTASK;          // [N2]
    const Member &M = A.mem[tl.member];
    TileCtx<N, T> c;
    __shared__ TileFaces<EPT> tf;
    load_tile<N, EPT, T>(A, M, tl, sD, tf, c);
    const T delta = (T)gp(M.delta)[c.e];   // LES filter width, loaded here to be ready after the gradient
    if (c.act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) lds[r * NN + c.g] = c.qt[1 + r];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int d = 0; d < 3; ++d) lds[(3 + 3 * ii + d) * NN + c.g] = c.Ja[ii][d];
    }
#pragma unroll 1
    for (int task = c.tid; task < NTASK; task += blockDim.x) {
        const FaceTask<N> ft = face_task<N, EPT>(tf, tl, task);
        const FaceRef fr = tf.f[ft.s * 6 + ft.f];
        if (ft.s < tl.count && !(fr.code & kMortarBit)) {
            // u* - u = (u_other - u) / 2, formed in FP64
            const gmem<const double> *qm = c.qin + 4 * tf.eo[ft.s] + face_node<N>(ft.f, ft.fa, ft.fb);
            double uo[3];
            if (fr.nbr >= 0) {
                int a2, b2;
                orient_map<N>(fr.code & 7, ft.fa, ft.fb, a2, b2);
                const gmem<const double> *qn = c.qin + 4 * nbr_first<N>(M.eoff != nullptr, fr) +
                                               face_node<N>((fr.code >> 3) & 7, a2, b2);
#pragma unroll
                for (int r = 0; r < 3; ++r) uo[r] = qn[(1 + r) * N3];
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r) uo[r] = fr.nbr == HDG_WALL ? -qm[(1 + r) * N3] : M.qinf[1 + r];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) sfu[r * NTASK + task] = (T)(0.5 * (uo[r] - qm[(1 + r) * N3]));
        }
    }
    __syncthreads();

    const int base = c.s * N3;
    const int tbase = c.s * NFT;
    T G[3][3];
    {
        T JG[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) JG[r][d] = T(0);
#pragma unroll 1
        for (int m = 0; m < N; ++m) {
            const int n0 = base + m + N * c.j + N2 * c.k, n1 = base + c.i + N * m + N2 * c.k,
                      n2 = base + c.i + N * c.j + N2 * m;
            T u0[3], u1[3], u2[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                u0[r] = lds[r * NN + n0];
                u1[r] = lds[r * NN + n1];
                u2[r] = lds[r * NN + n2];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T g0 = sD[c.i * N + m] * lds[(3 + d) * NN + n0];
                const T g1 = sD[c.j * N + m] * lds[(6 + d) * NN + n1];
                const T g2 = sD[c.k * N + m] * lds[(9 + d) * NN + n2];
#pragma unroll
                for (int r = 0; r < 3; ++r) JG[r][d] += g0 * u0[r] + g1 * u1[r] + g2 * u2[r];
            }
        }
        // the lane's metric terms, read back from LDS rather than kept in
        // registers through the contraction
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int d = 0; d < 3; ++d) c.Ja[ii][d] = lds[(3 + 3 * ii + d) * NN + c.g];
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
            if (c.act && (idx == 0 || idx == N - 1)) {
                const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
                const int fidx = (dir == 0 ? c.j : c.i) + N * (dir == 2 ? c.j : c.k);
                const int task = tbase + f * N2 + fidx;
                const T sf = (f & 1) ? T(1) : T(-1);
                const FaceRef fr = tf.f[c.s * 6 + f];
                if (fr.code & kMortarBit) {
                    const MortarSide mr = mortar_side<N>(fr);
                    const bool hi = mr.hi;
                    const gmem<const T> *lf = gp((const T *)M.mslab) + mr.slab + mslab_lift(mr.Nh, mr.Nl, hi) + fidx;
                    if (hi) {
                        // higher side: the mortar is its own face, (u* - u) (s n)_own
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const T jump = (lf[r * N2] - c.qt[1 + r]) * sf * c.inv_wend;
#pragma unroll
                            for (int d = 0; d < 3; ++d) JG[r][d] += jump * c.Ja[dir][d];
                        }
                    } else {
                        // lower side: (u* - u_r) (s n) integrated on the mortar, minus (u - u_r) (s n)_own;
                        // one row at a time (scheduling barriers), so that the nine loads do not
                        // all hold registers at once at the kernel's register peak
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
#pragma unroll
                            for (int d = 0; d < 3; ++d)
                                JG[r][d] += (lf[(r * 3 + d) * N2] - c.qt[1 + r] * sf * c.Ja[dir][d]) * c.inv_wend;
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const T jump = sfu[r * NTASK + task] * sf * c.inv_wend;
#pragma unroll
                        for (int d = 0; d < 3; ++d) JG[r][d] += jump * c.Ja[dir][d];
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) G[r][d] = JG[r][d] * c.invJ;
    }
    if constexpr (FEAT) {
        // node features of the clustering (Sec. 2.1): invariants of the
        // strain rate S = (G + G^T)/2 and rotation rate W = (G - G^T)/2
        if (c.act) {
            T S[3][3], w2 = T(0);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    S[r][d] = T(0.5) * (G[r][d] + G[d][r]);
                    const T wr = T(0.5) * (G[r][d] - G[d][r]);
                    w2 += wr * wr;
                }
            const T trS = S[0][0] + S[1][1] + S[2][2];
            T trS2 = T(0);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int d = 0; d < 3; ++d) trS2 += S[r][d] * S[d][r];
            const T det = S[0][0] * (S[1][1] * S[2][2] - S[1][2] * S[2][1]) -
                          S[0][1] * (S[1][0] * S[2][2] - S[1][2] * S[2][0]) +
                          S[0][2] * (S[1][0] * S[2][1] - S[1][1] * S[2][0]);
            gmem<T> *out = gp((T *)A.r) + c.eo + c.t;
            out[0] = T(0.5) * (trS * trS - trS2);        // Q_S
            out[A.nodes] = -det / T(3);                   // R_S
            out[2 * A.nodes] = T(0.5) * w2;               // Q_Omega = -tr(W^2)/2 = |W|^2/2
        }
        return;
    }
    T fv[3][3];
    {
        const T mu = c.nu + les_nut<T>(M.les_model, c.C_les, delta, G);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) fv[r][d] = mu * (G[r][d] + G[d][r]);
    }
    __syncthreads();     // every lane is done reading u, Ja and the half jumps from LDS
    if (c.act) {
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                lds[(ii * 3 + r) * NN + c.g] = c.Ja[ii][0] * fv[r][0] + c.Ja[ii][1] * fv[r][1] + c.Ja[ii][2] * fv[r][2];
    }
    __syncthreads();
    T W[3] = {T(0), T(0), T(0)};
#pragma unroll 1
    for (int m = 0; m < N; ++m) {
        const int n0 = base + m + N * c.j + N2 * c.k, n1 = base + c.i + N * m + N2 * c.k,
                  n2 = base + c.i + N * c.j + N2 * m;
#pragma unroll
        for (int r = 0; r < 3; ++r)
            W[r] -= sD[c.i * N + m] * lds[r * NN + n0] + sD[c.j * N + m] * lds[(3 + r) * NN + n1] +
                    sD[c.k * N + m] * lds[(6 + r) * NN + n2];
    }
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
        if (c.act && (idx == 0 || idx == N - 1)) {
            const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
            const T sf = (f & 1) ? T(1) : T(-1);
#pragma unroll
            for (int r = 0; r < 3; ++r) W[r] += sf * lds[(dir * 3 + r) * NN + c.g] * c.inv_wend;
            // tau . (s n) with the owner's outward normal (mortar: the higher
            // side's outward normal): +-(this element's outward)
            const int fidx = (dir == 0 ? c.j : c.i) + N * (dir == 2 ? c.j : c.k);
            const int task = tbase + f * N2 + fidx;
            const FaceRef fr = tf.f[c.s * 6 + f];
            const T so = (fr.code & kOwnerBit) ? sf : -sf;
            const T sn[3] = {so * c.Ja[dir][0], so * c.Ja[dir][1], so * c.Ja[dir][2]};
            if (fr.code & kMortarBit) {
                const MortarSide mr = mortar_side<N>(fr);
                gmem<T> *tr = gp((T *)M.mslab) + mr.slab + mslab_tr(mr.Nh, mr.Nl, mr.hi) + fidx;
#pragma unroll
                for (int r = 0; r < 3; ++r) tr[r * N2] = fv[r][0] * sn[0] + fv[r][1] * sn[1] + fv[r][2] * sn[2];
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    sfu[r * NTASK + task] = fv[r][0] * sn[0] + fv[r][1] * sn[1] + fv[r][2] * sn[2];
            }
        }
    }
    if (c.act) {
        gmem<T> *wv = gp((T *)M.wvis) + 3 * c.eo + c.t;
#pragma unroll
        for (int r = 0; r < 3; ++r) wv[r * N3] = W[r];
    }
    __syncthreads();
    gmem<T> *fvt = gp((T *)M.fvt);
#pragma unroll 1
    for (int task = c.tid; task < NTASK; task += blockDim.x) {
        const FaceTask<N> ft = face_task<N, EPT>(tf, tl, task);
        const FaceRef fr = tf.f[ft.s * 6 + ft.f];
        if (ft.s < tl.count && !(fr.code & kMortarBit)) {
            const bool own = fr.code & kOwnerBit;
            int oa = ft.fa, ob = ft.fb;
            if (!own) orient_map<N>(fr.code & 7, ft.fa, ft.fb, oa, ob);
            gmem<T> *out = fvt + 6 * face_first<N>(M.foff != nullptr, fr) + (own ? 0 : 3 * N2) + oa + N * ob;
#pragma unroll
            for (int r = 0; r < 3; ++r) out[r * N2] = sfu[r * NTASK + task];
        }
    }
}

// 1/sqrt(x) for a normal x > 0: the hardware estimate refined by Newton's
// method for x^(-1/2), y <- y + y (1 - x y^2) / 2, which squares the relative
// error (times 3/2) per step; two steps in FP64, one in FP32.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}
__device__ __forceinline__ float rsqrt_refined(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}

// Upwind dissipation D dq of a jump dq = (dp, du) between two traces along a
// unit normal n, for the artificial-compressibility flux (Sec. 2.3).  The
// normal Jacobian at the mean state (normal velocity u_n = uLn + dun/2) has
// the eigenvalues u_n +- a, a = sqrt(u_n^2 + c0^2), and u_n twice; dq splits
// into the two acoustic waves, amplitudes
//   alpha_+ = (dp - pi_- du_n) / (2a),  alpha_- = (pi_+ du_n - dp) / (2a),
//   pi_+- = +-a - u_n, eigenvectors (pi_+-, v_+-) with v_+ = (pi_+ n + u)/a,
//   v_- = -(pi_- n + u)/a, and the rest, du - alpha_+ v_+ - alpha_- v_-.
// Roe weights each part by its |eigenvalue|; Rusanov weights all by lambda,
// the larger spectral radius |u_n| + sqrt(u_n^2 + c0^2) of the two traces
// (the sum is then lambda dq).  Collecting terms, with s_+-, s_0 the weights:
//   (D dq)_p = s_+ alpha_+ pi_+ + s_- alpha_- pi_-,
//   (D dq)_u = X n + Y u + s_0 du,  u = uL + du/2 the mean velocity,
//   X = P pi_+ - Q pi_-,  Y = P - Q,  P = alpha_+ (s_+ - s_0)/a,  Q = alpha_- (s_- - s_0)/a.
template <class T>
struct Dissipation {
    T p, X, Y, s0;
};

template <class T>
__device__ __forceinline__ Dissipation<T> dissipation(int riemann, T c0sq, T uLn, T dun, T dp)
{
    const T h = T(0.5);
    const T un = uLn + h * dun;
    const T a2 = un * un + c0sq;
    const T ia = rsqrt_refined(a2);
    const T a = a2 * ia;
    const T pip = a - un, pim = -a - un;
    const T alp = h * ia * (dp - pim * dun);
    const T alm = h * ia * (pip * dun - dp);
    T sp = un + a, sm = a - un, s0 = fabs(un);
    if (riemann == HDG_RUSANOV) {
        const T uRn = uLn + dun;
        const T xL = uLn * uLn + c0sq, xR = uRn * uRn + c0sq;
        const T lL = fabs(uLn) + xL * rsqrt_refined(xL), lR = fabs(uRn) + xR * rsqrt_refined(xR);
        sp = sm = s0 = lL > lR ? lL : lR;
    }
    const T P = alp * (sp - s0) * ia, Q = alm * (sm - s0) * ia;
    Dissipation<T> D;
    D.p = sp * alp * pip + sm * alm * pim;
    D.X = P * pip - Q * pim;
    D.Y = P - Q;
    D.s0 = s0;
    return D;
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
// Member fields that face tasks read, taken once per tile: read through the
// member record inside the task loop, they are reloaded on every iteration.
template <class T>
struct FaceData {
    const T *geo;             // face geometry in the compute type
    const T *fvt;             // viscous face traces
    const int64_t *eoff, *foff;
    const double *qinf;
    int32_t riemann, mixed_face;
};

template <class T>
__device__ __forceinline__ FaceData<T> face_data(const Member &M)
{
    FaceData<T> d;
    d.geo = (const T *)M.fgeo[prec_index<T>()];
    d.fvt = (const T *)M.fvt;
    d.eoff = M.eoff;
    d.foff = M.foff;
    d.qinf = M.qinf;
    d.riemann = M.riemann;
    d.mixed_face = M.mixed_face;
    return d;
}

// The other side's trace at a face node of element e, in FP64: the
// neighbour's node (its face frame mapped by the orientation code), the wall
// ghost (p, -u) or the far-field state.  The load is issued for every lane,
// at this element's own node where there is no conforming neighbour (a
// boundary or a mortar face), so that callers may gather several tasks'
// traces before using any of them.
template <int N, class T>
__device__ __forceinline__ void face_other(const FaceData<T> &M, const gmem<const double> *qin,
                                           const gmem<const double> *qself, int fa, int fb, const FaceRef &fr,
                                           double (&qo)[4])
{
    constexpr int N3 = Shape<N>::N3;
    const gmem<const double> *qn = qself;
    if (fr.nbr >= 0 && !(fr.code & kMortarBit)) {
        int a2, b2;
        orient_map<N>(fr.code & 7, fa, fb, a2, b2);
        qn = qin + 4 * nbr_first<N>(M.eoff != nullptr, fr) + face_node<N>((fr.code >> 3) & 7, a2, b2);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) qo[x] = qn[x * N3];
}

// Boundary ghosts replace the gathered value where there is no neighbour.
template <class T>
__device__ __forceinline__ void face_ghost(const FaceData<T> &M, const FaceRef &fr, const double (&qm)[4],
                                           double (&qo)[4])
{
    if (fr.nbr == HDG_WALL) {
        qo[0] = qm[0];
#pragma unroll
        for (int x = 1; x < 4; ++x) qo[x] = -qm[x];
    } else if (fr.nbr < 0) {
#pragma unroll
        for (int x = 0; x < 4; ++x) qo[x] = gp(M.qinf)[x];
    }
}

// jf, when given, points at this element's Ja^dir at the face node (three
// values NTASK apart) and sf is the face's side (-1 for a minus face, +1 for
// a plus face): sf Ja^dir is this element's outward s n, the owner's is its
// negative on the other side (the two elements' metric terms agree at a
// shared face node to round-off).  Without jf the owner's stored unit normal
// and scale are read.  qo is the other side's trace (face_other, face_ghost).
template <int N, class T, int NTASK = 0>
__device__ __forceinline__ void face_flux(const FaceData<T> &M, T c0sq, bool visc, int fa, int fb,
                                          const FaceRef &fr, const double (&qm)[4], const double (&qo)[4],
                                          T (&F)[4], const T *jf = nullptr, T sf = T(1))
{
    constexpr int N2 = Shape<N>::N2;
    const bool own = fr.code & kOwnerBit;
    int oa = fa, ob = fb;
    if (fr.nbr >= 0 && !own) orient_map<N>(fr.code & 7, fa, fb, oa, ob);
    const int fnode = oa + N * ob;
    const int64_t fo = face_first<N>(M.foff != nullptr, fr);
    T n[3], sc;
    if constexpr (NTASK > 0) {
        // the owner's outward s n from this element's own metric terms
        const T so = own ? sf : -sf;
        const T v[3] = {so * jf[0], so * jf[NTASK], so * jf[2 * NTASK]};
        const T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const T iv = rsqrt_refined(v2);
        sc = v2 * iv;
#pragma unroll
        for (int d = 0; d < 3; ++d) n[d] = v[d] * iv;
    } else {
        const gmem<const T> *g = gp(M.geo) + 4 * (fo + fnode);
        n[0] = g[0];
        n[1] = g[1];
        n[2] = g[2];
        sc = g[3];
    }
    T uL[3], du[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double dd = qo[1 + d] - qm[1 + d];
        uL[d] = (T)(own ? qm[1 + d] : qo[1 + d]);
        du[d] = (T)(own ? dd : -dd);
    }
    const double dpd = qo[0] - qm[0];
    const T dp = (T)(own ? dpd : -dpd);
    const T h = T(0.5);
    const T uLn = uL[0] * n[0] + uL[1] * n[1] + uL[2] * n[2];
    const T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    const T uRn = uLn + dun;
    const T sg = own ? T(-1) : T(1);           // -dissipation for the owner, + for the other side
    const Dissipation<T> D = dissipation<T>(M.riemann, c0sq, uLn, dun, dp);
    // F_{1+d} = (dF_d + sg (D dq)_d) sc/2 with dF_d = uL_d du_n + du_d uR_n + dp n_d,
    // the terms collected per vector
    const T hs = h * sc;
    const T cU = dun + sg * D.Y, cD = uRn + sg * (h * D.Y + D.s0), cN = dp + sg * D.X;
    F[0] = hs * (c0sq * dun + sg * D.p);
#pragma unroll
    for (int d = 0; d < 3; ++d) F[1 + d] = hs * (uL[d] * cU + du[d] * cD + n[d] * cN);
    const bool nb_visc = (fr.code & kNbrViscBit) != 0;
    const bool visL = own ? visc : nb_visc;
    const bool visR = own ? nb_visc : visc;
    if (visL || visR) {
        // BR1: mean of the two sides' viscous traces (an Euler side contributes
        // zero); a boundary face takes the interior trace.  F* carries -F_v*.
        const bool keep = fr.nbr < 0 || M.mixed_face == 0 || (visL && visR);
        const gmem<const T> *tv = gp(M.fvt) + 6 * fo + fnode;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const T tL = visL ? tv[r * N2] : T(0);
            const T tR = (visR && fr.nbr >= 0) ? tv[(3 + r) * N2] : T(0);
            const T fvn = fr.nbr < 0 ? tL : h * (tL + tR);
            F[1 + r] += keep ? sg * fvn : T(0);
        }
    }
}

// Surface terms of a face-node lane: the numerical flux minus its own flux,
// over w_end.  Conforming faces take F* - F_own from the face tasks (sface);
// a mortar face takes the mortar's surface term relative to the reference
// flux minus this element's outward deviation flux (own flux from the flux
// area, so only once the fluxes are there).  CONF and MORT select which.
template <int N, int EPT, class T, bool CONF, bool MORT>
__device__ __forceinline__ void surface_terms(const Member &M, const TileFaces<EPT> &tf, const TileCtx<N, T> &c,
                                              const T *sface, const T *lds, T (&V)[4])
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    constexpr int NFT = 6 * N2, NN = EPT * N3, NTASK = EPT * NFT;
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const int idx = dir == 0 ? c.i : dir == 1 ? c.j : c.k;
        if (c.act && (idx == 0 || idx == N - 1)) {
            const int f = 2 * dir + (idx == N - 1 ? 1 : 0);
            const int fa = dir == 0 ? c.j : c.i;
            const int fb = dir == 2 ? c.j : c.k;
            const FaceRef fr = tf.f[c.s * 6 + f];
            if (fr.code & kMortarBit) {
                if (MORT) {
                    const MortarSide mr = mortar_side<N>(fr);
                    const T sf = (f & 1) ? T(1) : T(-1);
                    const gmem<const T> *sm = gp((const T *)M.mslab) + mr.slab + mslab_surf(mr.Nh, mr.Nl, mr.hi) +
                                              fa + N * fb;
#pragma unroll
                    for (int row = 0; row < 4; ++row)
                        V[row] += (sm[row * N2] - sf * lds[(dir * 4 + row) * NN + c.g]) * c.inv_wend;
                }
            } else if (CONF) {
                const T *Fs = sface + c.s * NFT + f * N2 + fa + N * fb;
#pragma unroll
                for (int row = 0; row < 4; ++row) V[row] += Fs[row * NTASK] * c.inv_wend;
            }
        }
    }
}

// FP64 tiles that stage the state (orders 3 to 5) keep the surface terms in
// the flux area too, behind the staged state (4 EPT N^3 + 4 EPT 6 N^2 doubles
// fit in 12 EPT N^3 from N = 3 on): the workgroup's LDS then drops by a
// quarter, which is what limits occupancy at those orders.
template <int N, class T>
constexpr bool residual_sface_in_flux() { return N <= 5 && N >= 3 && sizeof(T) == 8; }

// Order-5 tiles take the face normals from the element's own metric terms,
// staged per face node in LDS ([3][EPT 6 N^2] after the derivative matrix),
// instead of loading the stored face geometry.
template <int N>
constexpr bool residual_face_ja() { return N == 5; }

template <int N, int EPT, class T>
constexpr int residual_lds_words()
{
    return 12 * EPT * N * N * N + (residual_sface_in_flux<N, T>() ? 0 : 4 * EPT * 6 * N * N) + N * N +
           (residual_face_ja<N>() ? 3 * EPT * 6 * N * N : 0);
}

template <int N, int EPT, int EPI, class T>
__device__ __forceinline__ void residual_tile(const StageArgs &A, const Tile &tl, char *smem)
{
    constexpr int N2 = Shape<N>::N2, N3 = Shape<N>::N3;
    constexpr int NFT = 6 * N2, NN = EPT * N3, NTASK = EPT * NFT;
    constexpr bool SF_IN_FLUX = residual_sface_in_flux<N, T>();
    T *lds = (T *)smem;               // [12][NN] contravariant fluxes
    // [4][NTASK] surface terms F* - F_own: after the staged state in the flux
    // area, or after the flux area
    T *sface = SF_IN_FLUX ? (T *)((double *)smem + 4 * NN) : lds + 12 * NN;
    T *sD = SF_IN_FLUX ? lds + 12 * NN : sface + 4 * NTASK;   // [N2]
    constexpr bool FACE_JA = residual_face_ja<N>();
    T *sjf = sD + N2;                 // [3][NTASK] Ja^dir at the face nodes (FACE_JA)
    const Member &M = A.mem[tl.member];
    TileCtx<N, T> c;
    __shared__ TileFaces<EPT> tf;
    // Face tasks read the element's own trace from its state staged in LDS
    // up to N = 5; above that, keeping the element's context live across the
    // face tasks costs more registers (and occupancy) than the gathers it
    // saves, and the trace is gathered from global memory after the fluxes.
    constexpr bool STAGE = N <= 5;
    double *sq = (double *)smem;      // [4][NN] own state, FP64, until the fluxes replace it
    // the face nodes' Ja^dir are staged with the rest, behind the same barrier
    load_tile<N, EPT, T, STAGE>(A, M, tl, sD, tf, c, sq, FACE_JA ? sjf : nullptr);
    const bool visc = tl.flag != 0;   // a tile's elements share one equation flag
    const FaceData<T> fd = face_data<T>(M);
    if constexpr (STAGE) {
        // face-node tasks, spread evenly over the workgroup; a tile's elements
        // share one equation class.  A task's own trace comes from the staged
        // state, the other side's from global memory.
#pragma unroll 1
        for (int task = c.tid; task < NTASK; task += blockDim.x) {
            const FaceTask<N> ft = face_task<N, EPT>(tf, tl, task);
            const FaceRef fr = tf.f[ft.s * 6 + ft.f];
            if (ft.s < tl.count && !(fr.code & kMortarBit)) {
                const int fnode = face_node<N>(ft.f, ft.fa, ft.fb), node = ft.s * N3 + fnode;
                const double qm[4] = {sq[node], sq[NN + node], sq[2 * NN + node], sq[3 * NN + node]};
                double qo[4];
                face_other<N, T>(fd, c.qin, c.qin + 4 * tf.eo[ft.s] + fnode, ft.fa, ft.fb, fr, qo);
                face_ghost<T>(fd, fr, qm, qo);
                T F[4];
                if constexpr (FACE_JA)
                    face_flux<N, T, NTASK>(fd, c.c0sq, visc, ft.fa, ft.fb, fr, qm, qo, F, sjf + task,
                                           (ft.f & 1) ? T(1) : T(-1));
                else
                    face_flux<N, T>(fd, c.c0sq, visc, ft.fa, ft.fb, fr, qm, qo, F);
#pragma unroll
                for (int row = 0; row < 4; ++row) sface[row * NTASK + task] = F[row];
            }
        }
        __syncthreads();     // the staged state is read; the fluxes take its place
        if constexpr (sizeof(T) == 8) {
            // the own state and its deviation from the reference, taken again
            // from the lane's own staged slots (which only this lane's fluxes
            // overwrite) rather than held in registers through the face tasks
            // (FP64: 16 registers fewer at the kernel's register peak)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                c.qd[f] = sq[f * NN + c.g];
                c.q[f] = (T)c.qd[f];
                c.qt[f] = (T)(c.qd[f] - (double)c.qr[f]);
            }
        }
    }
    T V[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (SF_IN_FLUX) {
        // conforming faces' surface terms now, before the fluxes overwrite them
        surface_terms<N, EPT, T, true, false>(M, tf, c, sface, lds, V);
        __syncthreads();
    }

    // contravariant convective fluxes F^i_row = sum_d Ja^i_d f_{row,d} of the
    // deviation f(q) - f(q_r): c0^2 (u - u_r) and
    // u u^T - u_r u_r^T + (p - p_r) I = u (u - u_r)^T + (u - u_r) u_r^T + (p - p_r) I
    {
        T f[4][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[0][d] = c.c0sq * c.qt[1 + d];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                f[1 + r][d] = c.q[1 + r] * c.qt[1 + d] + c.qt[1 + r] * c.qr[1 + d] + (r == d ? c.qt[0] : T(0));
        }
        if (c.act) {
#pragma unroll
            for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                for (int row = 0; row < 4; ++row)
                    lds[(ii * 4 + row) * NN + c.g] =
                        c.Ja[ii][0] * f[row][0] + c.Ja[ii][1] * f[row][1] + c.Ja[ii][2] * f[row][2];
        }
    }

    if constexpr (!STAGE) {
#pragma unroll 1
        for (int task = c.tid; task < NTASK; task += blockDim.x) {
            const FaceTask<N> ft = face_task<N, EPT>(tf, tl, task);
            const FaceRef fr = tf.f[ft.s * 6 + ft.f];
            if (ft.s < tl.count && !(fr.code & kMortarBit)) {
                const gmem<const double> *qe = c.qin + 4 * tf.eo[ft.s] + face_node<N>(ft.f, ft.fa, ft.fb);
                const double qm[4] = {qe[0], qe[N3], qe[2 * N3], qe[3 * N3]};
                double qo[4];
                face_other<N, T>(fd, c.qin, qe, ft.fa, ft.fb, fr, qo);
                face_ghost<T>(fd, fr, qm, qo);
                T F[4];
                face_flux<N, T>(fd, c.c0sq, visc, ft.fa, ft.fb, fr, qm, qo, F);
#pragma unroll
                for (int row = 0; row < 4; ++row) sface[row * NTASK + task] = F[row];
            }
        }
    }
    gmem<double> *dqp = gp(A.q_in ? A.dq : M.dq);
    double dq_old[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (EPI == (int)Epi::RkStage) {
        if (!A.first_stage) {
            const gmem<double> *dqe = dqp + 4 * c.eo + c.t;
#pragma unroll
            for (int row = 0; row < 4; ++row) dq_old[row] = __builtin_nontemporal_load(dqe + row * N3);
        }
    }
    // the viscous operator's volume part, loaded before the contraction so
    // that its latency is hidden behind it
    T wvol[3] = {T(0), T(0), T(0)};
    if (c.act && visc) {
        const gmem<const T> *wv = gp((const T *)M.wvis) + 3 * c.eo + c.t;
#pragma unroll
        for (int r = 0; r < 3; ++r) wvol[r] = wv[r * N3];
    }
    __syncthreads();

    // reference divergence, with the contraction loop rolled: unrolled, the
    // scheduler hoists all 12 N LDS reads and needs about twice the
    // registers (measured: occupancy falls and both launch forms slow down)
    const int base = c.s * N3;
#pragma unroll 1
    for (int m = 0; m < N; ++m) {
        const int n0 = base + m + N * c.j + N2 * c.k, n1 = base + c.i + N * m + N2 * c.k,
                  n2 = base + c.i + N * c.j + N2 * m;
        const T dx = sD[c.i * N + m], dy = sD[c.j * N + m], dz = sD[c.k * N + m];
#pragma unroll
        for (int row = 0; row < 4; ++row)
            V[row] += dx * lds[row * NN + n0] + dy * lds[(4 + row) * NN + n1] + dz * lds[(8 + row) * NN + n2];
    }

    // face nodes: numerical flux minus own flux, over w_end (mortar faces
    // only if the conforming ones were added before the fluxes)
    surface_terms<N, EPT, T, !SF_IN_FLUX, true>(M, tf, c, sface, lds, V);

    if (c.act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) V[1 + r] += wvol[r];
        const size_t base_o = 4 * c.eo + c.t;
        // read from the member record before the first store: a store could
        // alias it, and a reload after each one would wait for that store
        const double dt = EPI == (int)Epi::RkStage ? (A.q_in ? A.dt : M.dt) : 0.0;
        gmem<double> *qout = EPI == (int)Epi::RkStage ? gp(A.q_in ? A.q_out : (A.parity ? M.qA : M.qB)) : nullptr;
#pragma unroll
        for (int row = 0; row < 4; ++row) {
            const T R = -V[row] * c.invJ;
            const size_t idx = base_o + (size_t)row * N3;
            if constexpr (EPI == (int)Epi::Residual) {
                gp((T *)A.r)[idx] = R;
            } else {
                // FP64 stage accumulation into the state
                const double Rd = (double)R;
                const double d = A.first_stage ? dt * Rd : A.rkA * dq_old[row] + dt * Rd;
                // streaming stores: the next state and the register are not
                // read again in this stage, and left out of the L2 they leave
                // room for the states that neighbouring tiles gather
                if (A.store_dq) __builtin_nontemporal_store(d, dqp + idx);
                __builtin_nontemporal_store(c.qd[row] + A.rkB * d, qout + idx);
            }
        }
    }
}

// Tile assignment: the grid is a multiple of kXcd; workgroup b runs on XCD
// b mod kXcd (round-robin dispatch) and takes tiles from that XCD's
// contiguous chunk of the (spatially ordered) tile list, so neighbour traces
// hit its L2.  Persistent launches walk the chunk; otherwise the grid is
// kXcd * chunk and every workgroup takes exactly one tile.
#define HDG_TILE_LOOP(A, tl)                                                                   \
    const int xcd_ = blockIdx.x % kXcd, loc_ = blockIdx.x / kXcd, nloc_ = gridDim.x / kXcd;   \
    for (int i_ = loc_; i_ < (A).chunk; i_ += nloc_)                                           \
        if (const int ti_ = xcd_ * (A).chunk + i_; ti_ < (A).ntiles)                            \
            if (const Tile tl = (A).tiles[ti_]; true)

#define HDG_ONE_TILE(A, tl)                                                                    \
    const int xcd_ = blockIdx.x % kXcd, loc_ = blockIdx.x / kXcd;                              \
    if (const int ti_ = xcd_ * (A).chunk + loc_; loc_ < (A).chunk && ti_ < (A).ntiles)          \
        if (const Tile tl = (A).tiles[ti_]; true)

// One kernel per (kind, order, workgroup size, persistence): a single kernel
// over every order would carry the register demand of all of them at once
// (measured: about 1.7x the largest single order), halving occupancy.  Only
// persistent launches loop over tiles; the others take one tile each.
template <class T, int N, int B, bool PERS>
__global__ __launch_bounds__(B) void k_viscous(StageArgs A)
{
    constexpr int EPT = tile_ept(N, B, kTileViscous);
    static_assert(EPT > 0, "tile does not fit the workgroup");
    constexpr int N2 = N * N, NN = EPT * N * N2, NTASK = EPT * 6 * N2;
    __shared__ __attribute__((aligned(16))) char smem[(12 * NN + 3 * NTASK + N2) * sizeof(T)];
    if constexpr (PERS) {
        HDG_TILE_LOOP(A, tl) {
            viscous_tile<N, EPT, T>(A, tl, smem);
            __syncthreads();
        }
    } else {
        HDG_ONE_TILE(A, tl) viscous_tile<N, EPT, T>(A, tl, smem);
    }
}

// Node features of the clustering: the viscous operator's BR1 gradient on
// every element of the tile list, then its invariants (FP64).
template <int N, int B>
__global__ __launch_bounds__(B) void k_features(StageArgs A)
{
    constexpr int EPT = tile_ept(N, B, kTileViscous);
    static_assert(EPT > 0, "tile does not fit the workgroup");
    constexpr int N2 = N * N, NN = EPT * N * N2, NTASK = EPT * 6 * N2;
    __shared__ __attribute__((aligned(16))) char smem[(12 * NN + 3 * NTASK + N2) * sizeof(double)];
    HDG_ONE_TILE(A, tl) viscous_tile<N, EPT, double, true>(A, tl, smem);
}

// FP64 order-5 tiles launched one per workgroup fit five waves per SIMD
// (at most 96 registers) without spilling; the persistent form's tile loop
// would spill there and keeps the compiler's choice, and 512-lane
// workgroups are held to four waves by their LDS.
template <class T, int N, int B, bool PERS>
constexpr int residual_min_waves() { return sizeof(T) == 8 && N == 5 && B <= 256 && !PERS ? 5 : 1; }

template <class T, int EPI, int N, int B, bool PERS>
__global__ __launch_bounds__(B, (residual_min_waves<T, N, B, PERS>())) void k_residual(StageArgs A)
{
    constexpr int EPT = tile_ept(N, B, kTileResidual);
    static_assert(EPT > 0, "tile does not fit the workgroup");
    __shared__ __attribute__((aligned(16))) char smem[residual_lds_words<N, EPT, T>() * sizeof(T)];
    if constexpr (PERS) {
        HDG_TILE_LOOP(A, tl) {
            residual_tile<N, EPT, EPI, T>(A, tl, smem);
            __syncthreads();
        }
    } else {
        HDG_ONE_TILE(A, tl) residual_tile<N, EPT, EPI, T>(A, tl, smem);
    }
}

// ---------------------------------------------------------------------------
// Mortars: faces between elements of different order.  The mortar carries
// the higher order NH in the higher side's face frame; the lower side's
// traces are extended to it by their own interpolants, the numerical flux is
// evaluated once per mortar node with the higher side's normal, and the
// lower side's share is its exact surface integral on the mortar against
// each of its face basis functions (GLL weights of the mortar, interpolation
// coefficients as test functions), divided by its own face weights.  Values
// are formed relative to each side's reference state q_r (its centre node),
// as in the element kernels, so that only deviations enter the compute type.
//
// Launch shape: one kernel per (NL, NH) pair, 256 lanes per workgroup; a
// mortar takes NH^2 consecutive lanes (256 / NH^2 mortars per workgroup, a
// mortar may straddle two waves: every phase ends at a workgroup barrier).  The
// lower side's face trace is staged once per mortar in LDS; extension and
// projection are separable contractions with the interpolation rows held in
// registers.  The lower side's quantities on the mortar are stored in LDS in
// its own face frame, where the projection factorises; the mortar weights
// are symmetric under every face orientation, so w_i w_j of a node is the
// same in either frame.
// ---------------------------------------------------------------------------

template <int NL, int NH>
struct MortarShape {
    static constexpr int M2 = NH * NH, L2 = NL * NL;
    static constexpr int N3H = NH * NH * NH, N3L = NL * NL * NL;
    static constexpr int SLOTS = 256 / M2;       // mortars per workgroup
};

// One lane's mortar and node; `valid` is false for lanes past the last mortar
// or past the workgroup's last whole mortar.
template <int NL, int NH>
struct MortarLane {
    int slot, node, i, j, il, jl;
    bool valid;
    MortarRef mr;
    const gmem<const double> *qh, *ql;
};

template <int NL, int NH>
__device__ __forceinline__ MortarLane<NL, NH> mortar_lane(const StageArgs &A, const Member &M)
{
    using S = MortarShape<NL, NH>;
    MortarLane<NL, NH> L;
    L.slot = threadIdx.x / S::M2;
    L.node = threadIdx.x - L.slot * S::M2;
    const int mi = blockIdx.x * S::SLOTS + L.slot;
    L.valid = L.slot < S::SLOTS && mi < A.mcount;
    L.i = L.node % NH;
    L.j = L.node / NH;
    L.il = L.jl = 0;
    L.qh = L.ql = nullptr;
    if (L.valid) {
        L.mr = load_mortar(A.mlist, mi);
        orient_map<NH>(L.mr.code_h & 7, L.i, L.j, L.il, L.jl);
        // the stage's input state: given, or the member's ping-pong buffer
        const gmem<const double> *q = gp((const double *)(A.q_in ? A.q_in : (A.parity ? M.qB : M.qA)));
        L.qh = q + 4 * L.mr.oh;
        L.ql = q + 4 * L.mr.ol;
    }
    return L;
}

// Extension of a lower-side face field f[a + NL b] (LDS) to mortar node
// (il, jl): sum_b I[jl][b] sum_a I[il][a] f[a, b], in FP64.
template <int NL>
__device__ __forceinline__ double extend_face(const double (&Ia)[NL], const double (&Ib)[NL], const double *f)
{
    double s = 0.0;
#pragma unroll 1
    for (int b = 0; b < NL; ++b) {
        double sb = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a) sb += Ia[a] * f[a + NL * b];
        s += Ib[b] * sb;
    }
    return s;
}

// Projection onto the lower side's face basis function (a, b): G holds the
// integrand times the mortar weights at mortar node (il, jl) of the lower
// frame, Wa / Wb the interpolation columns I[.][a], I[.][b].
template <int NL, int NH, class T>
__device__ __forceinline__ T project_face(const T (&Wa)[NH], const T (&Wb)[NH], const T *G)
{
    T s = T(0);
#pragma unroll 1
    for (int jl = 0; jl < NH; ++jl) {
        T sj = T(0);
#pragma unroll
        for (int il = 0; il < NH; ++il) sj += Wa[il] * G[il + NH * jl];
        s += Wb[jl] * sj;
    }
    return s;
}

template <int NL, int NH, class T>
__global__ __launch_bounds__(256) void k_mortar_lift(StageArgs A)
{
    using S = MortarShape<NL, NH>;
    constexpr int M2 = S::M2, L2 = S::L2;
    __shared__ double sq[S::SLOTS][3 * L2];     // lower side's velocity face trace
    __shared__ T G[S::SLOTS][9 * M2];           // lower side's lift integrand, lower frame
    const Member &M = A.mem[0];
    const MortarLane<NL, NH> L = mortar_lane<NL, NH>(A, M);
    constexpr int crefh = (NH / 2) * (1 + NH + NH * NH), crefl = (NL / 2) * (1 + NL + NL * NL);
    // the lane's own loads are issued together with the staging loads (one
    // memory latency before the barrier, not one per dependent step)
    double uh[3] = {0.0, 0.0, 0.0}, rfh[3] = {0.0, 0.0, 0.0}, rfl[3] = {0.0, 0.0, 0.0};
    T gv[4] = {T(0), T(0), T(0), T(0)};
    if (L.valid) {
        const gmem<const T> *g = gp((const T *)M.mgeo[prec_index<T>()]) + 4 * (L.mr.geo + L.node);
        const int nodeh = face_node<NH>(L.mr.fh, L.i, L.j);
#pragma unroll
        for (int x = 0; x < 4; ++x) gv[x] = g[x];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            uh[r] = L.qh[(1 + r) * S::N3H + nodeh];
            rfh[r] = L.qh[(1 + r) * S::N3H + crefh];
            rfl[r] = L.ql[(1 + r) * S::N3L + crefl];
        }
        constexpr int K = (3 * L2 + M2 - 1) / M2;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int v = L.node + k * M2;
            if (v < 3 * L2) {
                const int r = v / L2, ab = v - r * L2;
                sq[L.slot][v] = L.ql[(1 + r) * S::N3L + face_node<NL>(L.mr.fl, ab % NL, ab / NL)];
            }
        }
    }
    __syncthreads();
    if (L.valid) {
        const double *I = A.I64 + i_offset(NL, NH);
        const T *wh = wtable<T>(A) + w_offset(NH);
        double Ia[NL], Ib[NL];
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            Ia[a] = I[L.il * NL + a];
            Ib[a] = I[L.jl * NL + a];
        }
        const T w2 = wh[L.i] * wh[L.j];
        const T sn[3] = {gv[0] * gv[3] * w2, gv[1] * gv[3] * w2, gv[2] * gv[3] * w2};
        gmem<T> *lh = gp((T *)M.mslab) + L.mr.slab + mslab_lift(NH, NL, true) + L.node;
        const int gl = L.il + NH * L.jl;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double ul = extend_face<NL>(Ia, Ib, &sq[L.slot][r * L2]);
            const double us = 0.5 * (uh[r] + ul);
            // higher side: u* - u_r; its own s n is applied by the element kernel
            lh[r * M2] = (T)(us - rfh[r]);
            const T dl = (T)(us - rfl[r]);
#pragma unroll
            for (int d = 0; d < 3; ++d) G[L.slot][(r * 3 + d) * M2 + gl] = -dl * sn[d];
        }
    }
    __syncthreads();
    if (L.valid && L.node < L2) {
        const int a = L.node % NL, b = L.node / NL;
        const T *I = itable<T>(A) + i_offset(NL, NH);
        const T *wl = wtable<T>(A) + w_offset(NL);
        T Wa[NH], Wb[NH];
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            Wa[k] = I[k * NL + a];
            Wb[k] = I[k * NL + b];
        }
        const T iw = T(1) / (wl[a] * wl[b]);
        gmem<T> *ll = gp((T *)M.mslab) + L.mr.slab + mslab_lift(NH, NL, false) + L.node;
#pragma unroll
        for (int k = 0; k < 9; ++k) ll[k * L2] = project_face<NL, NH, T>(Wa, Wb, &G[L.slot][k * M2]) * iw;
    }
}

template <int NL, int NH, class T>
__global__ __launch_bounds__(256) void k_mortar_flux(StageArgs A)
{
    using S = MortarShape<NL, NH>;
    constexpr int M2 = S::M2, L2 = S::L2;
    __shared__ double sq[S::SLOTS][4 * L2];     // lower side's state face trace
    __shared__ T st[S::SLOTS][3 * L2];          // lower side's viscous traces
    __shared__ T G[S::SLOTS][4 * M2];           // lower side's surface integrand, lower frame
    const Member &M = A.mem[0];
    const MortarLane<NL, NH> L = mortar_lane<NL, NH>(A, M);
    // the sides' flags travel in the record; the lane's own loads are issued
    // together with the staging loads (one memory latency before the barrier)
    const bool vh = L.valid && (L.mr.flags & 1), vl = L.valid && (L.mr.flags & 2);
    const bool visc = (vh || vl) && (M.mixed_face == 0 || (vh && vl));
    constexpr int crefh = (NH / 2) * (1 + NH + NH * NH), crefl = (NL / 2) * (1 + NL + NL * NL);
    double qa[4] = {0.0, 0.0, 0.0, 0.0}, rh[4] = {0.0, 0.0, 0.0, 0.0}, rl[4] = {0.0, 0.0, 0.0, 0.0};
    T gv[4] = {T(0), T(0), T(0), T(0)}, thv[3] = {T(0), T(0), T(0)};
    if (L.valid) {
        const gmem<const T> *g = gp((const T *)M.mgeo[prec_index<T>()]) + 4 * (L.mr.geo + L.node);
        const int nodeh = face_node<NH>(L.mr.fh, L.i, L.j);
        if (visc && vh) {
            const gmem<const T> *th = gp((const T *)M.mslab) + L.mr.slab + mslab_tr(NH, NL, true) + L.node;
#pragma unroll
            for (int r = 0; r < 3; ++r) thv[r] = th[r * M2];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            gv[x] = g[x];
            qa[x] = L.qh[x * S::N3H + nodeh];
            rh[x] = L.qh[x * S::N3H + crefh];
            rl[x] = L.ql[x * S::N3L + crefl];
        }
        constexpr int KQ = (4 * L2 + M2 - 1) / M2;
#pragma unroll
        for (int k = 0; k < KQ; ++k) {
            const int v = L.node + k * M2;
            if (v < 4 * L2) {
                const int x = v / L2, ab = v - x * L2;
                sq[L.slot][v] = L.ql[x * S::N3L + face_node<NL>(L.mr.fl, ab % NL, ab / NL)];
            }
        }
        if (visc && vl) {
            const gmem<const T> *tl = gp((const T *)M.mslab) + L.mr.slab + mslab_tr(NH, NL, false);
            constexpr int KT = (3 * L2 + M2 - 1) / M2;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                const int v = L.node + k * M2;
                if (v < 3 * L2) st[L.slot][v] = tl[v];
            }
        }
    }
    __syncthreads();
    if (L.valid) {
        const double *I = A.I64 + i_offset(NL, NH);
        const T *wh = wtable<T>(A) + w_offset(NH);
        double Ia[NL], Ib[NL];
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            Ia[a] = I[L.il * NL + a];
            Ib[a] = I[L.jl * NL + a];
        }
        const T n[3] = {gv[0], gv[1], gv[2]};
        const T sc = gv[3];
        const T c0sq = (T)M.c0sq, h = T(0.5);
        double qb[4];                            // extended lower trace
#pragma unroll
        for (int x = 0; x < 4; ++x) qb[x] = extend_face<NL>(Ia, Ib, &sq[L.slot][x * L2]);
        // dissipation with L = higher side, R = lower side
        T uL[3], du[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            uL[d] = (T)qa[1 + d];
            du[d] = (T)(qb[1 + d] - qa[1 + d]);
        }
        const T dp = (T)(qb[0] - qa[0]);
        const T uLn = uL[0] * n[0] + uL[1] * n[1] + uL[2] * n[2];
        const T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
        const Dissipation<T> D = dissipation<T>(M.riemann, c0sq, uLn, dun, dp);
        T Ad[4];
        Ad[0] = D.p;
#pragma unroll
        for (int d = 0; d < 3; ++d) Ad[1 + d] = D.X * n[d] + D.Y * (uL[d] + h * du[d]) + D.s0 * du[d];
        // BR1: mean of the two sides' viscous traces along the higher side's s n
        T fvn[3] = {T(0), T(0), T(0)};
        if (visc) {
            T Ta[NL], Tb[NL];
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                Ta[k] = (T)Ia[k];
                Tb[k] = (T)Ib[k];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                T b_ = T(0);
                if (vl) {
#pragma unroll 1
                    for (int bb = 0; bb < NL; ++bb) {
                        T sb = T(0);
#pragma unroll
                        for (int aa = 0; aa < NL; ++aa) sb += Ta[aa] * st[L.slot][r * L2 + aa + NL * bb];
                        b_ += Tb[bb] * sb;
                    }
                }
                fvn[r] = h * (thv[r] + b_);
            }
        }
        // flux relative to each side's reference flux F_n(q_r):
        //   F* - F_n(q_r) = ((F_n(qa) - F_n(q_r)) + (F_n(qb) - F_n(q_r)))/2 - |A| dq / 2,
        //   F_n(q) - F_n(q_r) = [c0^2 du_n ; u du_n + du u_r,n + dp n], du = u - u_r
        const T w2 = wh[L.i] * wh[L.j];
        gmem<T> *sh = gp((T *)M.mslab) + L.mr.slab + mslab_surf(NH, NL, true) + L.node;
        const int gl = L.il + NH * L.jl;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double *qr = side == 0 ? rh : rl;
            const T urn = (T)qr[1] * n[0] + (T)qr[2] * n[1] + (T)qr[3] * n[2];
            T F[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int lr = 0; lr < 2; ++lr) {
                const double *qs = lr == 0 ? qa : qb;
                const T dpp = (T)(qs[0] - qr[0]);
                const T dv[3] = {(T)(qs[1] - qr[1]), (T)(qs[2] - qr[2]), (T)(qs[3] - qr[3])};
                const T dvn = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
                F[0] += c0sq * dvn;
#pragma unroll
                for (int d = 0; d < 3; ++d) F[1 + d] += (T)qs[1 + d] * dvn + dv[d] * urn + dpp * n[d];
            }
            T out[4];
            out[0] = sc * h * (F[0] - Ad[0]);
#pragma unroll
            for (int d = 0; d < 3; ++d) out[1 + d] = sc * h * (F[1 + d] - Ad[1 + d]) - fvn[d];
            if (side == 0) {
#pragma unroll
                for (int row = 0; row < 4; ++row) sh[row * M2] = out[row];
            } else {
#pragma unroll
                for (int row = 0; row < 4; ++row) G[L.slot][row * M2 + gl] = -out[row] * w2;   // outward for the lower side
            }
        }
    }
    __syncthreads();
    if (L.valid && L.node < L2) {
        const int a = L.node % NL, b = L.node / NL;
        const T *I = itable<T>(A) + i_offset(NL, NH);
        const T *wl = wtable<T>(A) + w_offset(NL);
        T Wa[NH], Wb[NH];
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            Wa[k] = I[k * NL + a];
            Wb[k] = I[k * NL + b];
        }
        const T iw = T(1) / (wl[a] * wl[b]);
        gmem<T> *sl = gp((T *)M.mslab) + L.mr.slab + mslab_surf(NH, NL, false) + L.node;
#pragma unroll
        for (int row = 0; row < 4; ++row) sl[row * L2] = project_face<NL, NH, T>(Wa, Wb, &G[L.slot][row * M2]) * iw;
    }
}

// ---------------------------------------------------------------------------
// Clustering (Sec. 2.1): a two-component Gaussian mixture over the node
// features (Q_S, R_S, Q_Omega), fitted by expectation-maximisation.  Every
// pass streams the three feature arrays once, standardising on the fly, and
// leaves per-workgroup partial sums (fixed order, no atomics); a one-lane
// update turns them into the next state in device memory, so a whole fit
// runs on the stream without the host.
// ---------------------------------------------------------------------------

constexpr int kGmmBlock = 256;

// E-step of one node: log(w_k N(x | mu_k, cov_k)) for both components,
// their log-sum-exp and the responsibilities.
__device__ __forceinline__ void gmm_estep(const gmem<const GmmState> *S, const double (&x)[3], double (&r)[2],
                                          double &lse)
{
    double a[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const gmem<const double> *Li = S->Li[k];
        const double d0 = x[0] - S->mu[k][0], d1 = x[1] - S->mu[k][1], d2 = x[2] - S->mu[k][2];
        const double z0 = Li[0] * d0;
        const double z1 = Li[1] * d0 + Li[2] * d1;
        const double z2 = Li[3] * d0 + Li[4] * d1 + Li[5] * d2;
        a[k] = S->logw[k] - S->cst[k] - 0.5 * (z0 * z0 + z1 * z1 + z2 * z2);
    }
    const double top = a[0] > a[1] ? a[0] : a[1];
    lse = top + log(exp(a[0] - top) + exp(a[1] - top));
    r[0] = exp(a[0] - lse);
    r[1] = exp(a[1] - lse);
}

template <int NV>
__device__ __forceinline__ void block_sums(double (&acc)[NV], double *partials)
{
    __shared__ double red[kGmmBlock / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double t = acc[v];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        acc[v] = t;
    }
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wv][v] = acc[v];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kGmmBlock / 64; ++w) t += red[w][threadIdx.x];
        gp(partials)[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;    // [value][workgroup]
    }
}

// MODE 0: sums of x; 1: sums of (x - mean)^2; 2: statistics of the initial
// split (Q_Omega above its mean: second component); 3: E-step statistics
// about the current means, plus the log-likelihood.
template <int MODE>
__global__ __launch_bounds__(kGmmBlock) void k_gmm_accum(const double *X, int64_t n, const GmmState *st,
                                                         double *partials)
{
    constexpr int NV = MODE < 2 ? 3 : kGmmStats;
    const gmem<const GmmState> *S = gp(st);
    const gmem<const double> *Xg = gp(X);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const bool skip = MODE == 3 && (S->degenerate || S->converged);
    for (int64_t i = (int64_t)blockIdx.x * kGmmBlock + threadIdx.x; !skip && i < n;
         i += (int64_t)gridDim.x * kGmmBlock) {
        double x[3] = {Xg[i], Xg[n + i], Xg[2 * n + i]};
        if constexpr (MODE == 0) {
#pragma unroll
            for (int f = 0; f < 3; ++f) acc[f] += x[f];
        } else if constexpr (MODE == 1) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double d = x[f] - S->fm[f];
                acc[f] += d * d;
            }
        } else {
#pragma unroll
            for (int f = 0; f < 3; ++f) x[f] = (x[f] - S->fm[f]) * S->fsi[f];
            double r[2], c[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
            if constexpr (MODE == 2) {
                r[1] = x[2] > 0.0 ? 1.0 : 0.0;
                r[0] = 1.0 - r[1];
            } else {
                double lse;
                gmm_estep(S, x, r, lse);
                acc[20] += lse;
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int f = 0; f < 3; ++f) c[k][f] = S->mu[k][f];
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double d0 = x[0] - c[k][0], d1 = x[1] - c[k][1], d2 = x[2] - c[k][2];
                double *a = acc + 10 * k;
                a[0] += r[k];
                a[1] += r[k] * d0;
                a[2] += r[k] * d1;
                a[3] += r[k] * d2;
                a[4] += r[k] * d0 * d0;
                a[5] += r[k] * d0 * d1;
                a[6] += r[k] * d0 * d2;
                a[7] += r[k] * d1 * d1;
                a[8] += r[k] * d1 * d2;
                a[9] += r[k] * d2 * d2;
            }
        }
    }
    block_sums<NV>(acc, partials);
}

// Sum the partials in a fixed order and write the next state (one lane).
// Lane t of the kGmmUpdate-lane workgroup adds workgroups t, t + kGmmUpdate,
// ... of every value with all its loads independent, then shuffle trees and
// one pass over the waves reduce them.
constexpr int kGmmUpdate = kMaxGmmBlocks / 2;

template <int MODE>
__global__ __launch_bounds__(kGmmUpdate) void k_gmm_update(const double *partials, int nblocks, int64_t n,
                                                           double reg, double tol, GmmState *st)
{
    constexpr int NV = MODE < 2 ? 3 : kGmmStats;
    constexpr int NW = kGmmUpdate / 64;
    __shared__ double red[NW][NV];
    __shared__ double tot[NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const gmem<const double> *p = gp(partials) + (size_t)v * nblocks;
        const int b0 = threadIdx.x, b1 = threadIdx.x + kGmmUpdate;
        acc[v] = (b0 < nblocks ? p[b0] : 0.0) + (b1 < nblocks ? p[b1] : 0.0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
    }
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wv][v] = acc[v];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += red[w][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    gmem<GmmState> *S = gp(st);
    const double dn = (double)n;
    if constexpr (MODE == 0) {
        for (int f = 0; f < 3; ++f) S->fm[f] = tot[f] / dn;
        S->degenerate = 0;
        S->converged = 0;
        S->iter = 0;
        S->ll = __builtin_nan("");
    } else if constexpr (MODE == 1) {
        // gradient scale: pooled deviation s_Q of the two Q invariants; R_S,
        // a cubed gradient, scales with s_Q^(3/2)
        const double sq = sqrt(0.5 * (tot[0] / dn + tot[2] / dn));
        const bool ok = sq > 0.0;
        S->fs[0] = ok ? sq : 1.0;
        S->fs[1] = ok ? sq * sqrt(sq) : 1.0;
        S->fs[2] = ok ? sq : 1.0;
        for (int f = 0; f < 3; ++f) S->fsi[f] = 1.0 / S->fs[f];
    } else {
        if (MODE == 2 && (tot[0] == 0.0 || tot[10] == 0.0)) {
            S->degenerate = 1;
            return;
        }
        if (MODE == 3) {
            if (S->degenerate || S->converged) return;
            const double ll = tot[20] / dn;
            // the M-step below still applies; later passes skip
            if (S->iter > 0 && fabs(ll - S->ll) < tol) S->converged = 1;
            S->ll = ll;
            S->iter = S->iter + 1;
        }
        for (int k = 0; k < 2; ++k) {
            const double *a = tot + 10 * k;
            const double nk = a[0] + 10.0 * __DBL_EPSILON__;
            const double c0 = MODE == 3 ? S->mu[k][0] : 0.0, c1 = MODE == 3 ? S->mu[k][1] : 0.0,
                         c2 = MODE == 3 ? S->mu[k][2] : 0.0;
            const double e0 = a[1] / nk, e1 = a[2] / nk, e2 = a[3] / nk;
            const double C00 = a[4] / nk - e0 * e0 + reg, C01 = a[5] / nk - e0 * e1, C02 = a[6] / nk - e0 * e2,
                         C11 = a[7] / nk - e1 * e1 + reg, C12 = a[8] / nk - e1 * e2, C22 = a[9] / nk - e2 * e2 + reg;
            S->mu[k][0] = c0 + e0;
            S->mu[k][1] = c1 + e1;
            S->mu[k][2] = c2 + e2;
            S->w[k] = nk / dn;
            S->logw[k] = log(nk / dn);
            S->cov[k][0] = C00; S->cov[k][1] = C01; S->cov[k][2] = C02;
            S->cov[k][3] = C11; S->cov[k][4] = C12; S->cov[k][5] = C22;
            // lower Cholesky factor L of the covariance and its inverse
            const double L00 = sqrt(C00), L10 = C01 / L00, L20 = C02 / L00;
            const double L11 = sqrt(C11 - L10 * L10), L21 = (C12 - L20 * L10) / L11;
            const double L22 = sqrt(C22 - L20 * L20 - L21 * L21);
            const double i00 = 1.0 / L00, i11 = 1.0 / L11, i22 = 1.0 / L22;
            const double i10 = -L10 * i00 * i11, i21 = -L21 * i11 * i22, i20 = -(L20 * i00 + L21 * i10) * i22;
            S->Li[k][0] = i00; S->Li[k][1] = i10; S->Li[k][2] = i11;
            S->Li[k][3] = i20; S->Li[k][4] = i21; S->Li[k][5] = i22;
            S->cst[k] = 1.5 * log(2.0 * M_PI) + log(L00) + log(L11) + log(L22);
        }
    }
}

// One wave per element: p_v of each node from the fitted mixture (the
// component with the larger mean Q_Omega is the viscous one), the element
// mean and the region (mean p_v >= mean p_i = 1 - mean p_v: viscous).
__global__ __launch_bounds__(kGmmBlock) void k_gmm_assign(const double *X, int64_t n, const GmmState *st,
                                                          const int64_t *eoff, const int8_t *Ne, int N3, int64_t ne,
                                                          double *p_visc, double *elem_pv, uint8_t *flags)
{
    const int64_t e = (int64_t)blockIdx.x * (kGmmBlock / 64) + (threadIdx.x >> 6);
    if (e >= ne) return;                       // wave-uniform; no workgroup barrier follows
    const int lane = threadIdx.x & 63;
    const gmem<const GmmState> *S = gp(st);
    const int64_t o = eoff ? gp(eoff)[e] : e * N3;
    const int n3 = eoff ? (int)gp(Ne)[e] * gp(Ne)[e] * gp(Ne)[e] : N3;
    const bool deg = S->degenerate != 0;
    const int vis = S->mu[0][2] > S->mu[1][2] ? 0 : 1;
    const gmem<const double> *Xg = gp(X);
    double sum = 0.0;
    for (int t = lane; t < n3; t += 64) {
        double p = 0.0;
        if (!deg) {
            double x[3], r[2], lse;
#pragma unroll
            for (int f = 0; f < 3; ++f) x[f] = (Xg[f * n + o + t] - S->fm[f]) * S->fsi[f];
            gmm_estep(S, x, r, lse);
            p = r[vis];
        }
        if (p_visc) gp(p_visc)[o + t] = p;
        sum += p;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (lane == 0) {
        const double pm = sum / n3;
        if (elem_pv) gp(elem_pv)[e] = pm;
        gp(flags)[e] = pm >= 1.0 - pm ? 1 : 0;
    }
}

// Partial reductions over the elements of a mesh of mixed order: workgroup
// b takes a contiguous range of elements, its lanes stride over each
// element's nodes.  Fixed order, no atomics.
__global__ __launch_bounds__(256) void k_reduce_partial_mixed(const double *r, const double *mass, const int64_t *eoff,
                                                              const int8_t *Ne, int64_t ne, double *partials)
{
    __shared__ double red[13][256];
    double acc[13];
#pragma unroll
    for (int x = 0; x < 13; ++x) acc[x] = 0.0;
    const int64_t per = (ne + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = e0 + per < ne ? e0 + per : ne;
    for (int64_t e = e0; e < e1; ++e) {
        const int N = Ne[e];
        const int N3 = N * N * N;
        const int64_t o = eoff[e];
        for (int n = threadIdx.x; n < N3; n += blockDim.x) {
            const double m = mass[o + n];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const double v = r[4 * o + (int64_t)f * N3 + n];
                acc[f] += m * v;
                acc[4 + f] += m * v * v;
                const double av = fabs(v);
                acc[8 + f] = av > acc[8 + f] ? av : acc[8 + f];
                if (!isfinite(v)) acc[12] = 1.0;
            }
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

// Largest wave speed of the artificial-compressibility flux over the state:
// the flux Jacobian along a unit normal n has eigenvalues u.n and
// u.n +- sqrt((u.n)^2 + c0^2), whose largest magnitude over all n is
// |u| + sqrt(|u|^2 + c0^2).  Per-block maxima over whole elements (the
// reduction's element ranges), with a non-finite flag; element e has N^3
// nodes from e N^3, or Ne[e]^3 from eoff[e] when eoff is set.
__global__ __launch_bounds__(256) void k_wave_speed_partial(const double *q, const int64_t *eoff, const int8_t *Ne,
                                                            int Nu, int64_t ne, double c0sq, double *partials)
{
    __shared__ double red[2][256];
    double lam = 0.0, bad = 0.0;
    const int64_t per = (ne + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = e0 + per < ne ? e0 + per : ne;
    for (int64_t e = e0; e < e1; ++e) {
        const int N = eoff ? Ne[e] : Nu;
        const int N3 = N * N * N;
        const int64_t o = eoff ? eoff[e] : e * (int64_t)N3;
        for (int n = threadIdx.x; n < N3; n += blockDim.x) {
            const double *qe = q + 4 * o + n;
            const double u = qe[N3], v = qe[2 * N3], w = qe[3 * N3];
            const double a = sqrt(u * u + v * v + w * w);
            const double l = a + sqrt(a * a + c0sq);
            if (!isfinite(l)) bad = 1.0;
            else lam = l > lam ? l : lam;
        }
    }
    red[0][threadIdx.x] = lam;
    red[1][threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) partials[(size_t)blockIdx.x * 2 + threadIdx.x] = red[threadIdx.x][0];
}

// Maxima of the per-block pairs into out[2].
__global__ __launch_bounds__(256) void k_max2_final(const double *partials, int nblocks, double *out)
{
    __shared__ double red[2][256];
    double acc[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        acc[0] = fmax(acc[0], partials[(size_t)b * 2]);
        acc[1] = fmax(acc[1], partials[(size_t)b * 2 + 1]);
    }
    red[0][threadIdx.x] = acc[0];
    red[1][threadIdx.x] = acc[1];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) out[threadIdx.x] = red[threadIdx.x][0];
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

// Calls f(integral_constant<N>, integral_constant<B>) for a supported pair.
template <class F>
hipError_t by_shape(int N, int B, F f)
{
#define SH_(n, b)                                                                          \
    if (N == n && B == b) return f(std::integral_constant<int, n>{}, std::integral_constant<int, b>{});
    SH_(2, 128) SH_(3, 128) SH_(4, 128) SH_(5, 128)
    SH_(2, 256) SH_(3, 256) SH_(4, 256) SH_(5, 256) SH_(6, 256)
    SH_(7, 384)
    SH_(2, 512) SH_(3, 512) SH_(4, 512) SH_(5, 512) SH_(6, 512) SH_(7, 512) SH_(8, 512)
#undef SH_
    return hipErrorInvalidValue;
}

// Grid check: a non-persistent launch must cover every tile with one workgroup.
bool grid_ok(const StageArgs &a, int grid, bool pers)
{
    if (grid <= 0 || grid % kXcd) return false;
    return pers || grid / kXcd >= a.chunk;
}

// One launch of a stage kernel (argument: the StageArgs by value), with the
// dispatch recording the timer's events when they are given.
template <class K>
static void launch_stage_kernel(K kernel, int grid, int block, hipStream_t s, const LaunchEvents &ev,
                                const StageArgs &a)
{
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, ev.start, ev.stop, 0, a);
    else
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, a);
}

hipError_t launch_viscous(int N, int B, bool f32, bool pers, const StageArgs &a, int grid, hipStream_t s,
                          const LaunchEvents &ev)
{
    if (a.ntiles == 0) return hipSuccess;
    if (!grid_ok(a, grid, pers)) return hipErrorInvalidValue;
    return by_shape(N, B, [&](auto nc, auto bc) {
        constexpr int NN = decltype(nc)::value, BB = decltype(bc)::value;
        if (f32) {
            if (pers) launch_stage_kernel(k_viscous<float, NN, BB, true>, grid, BB, s, ev, a);
            else launch_stage_kernel(k_viscous<float, NN, BB, false>, grid, BB, s, ev, a);
        } else {
            if (pers) launch_stage_kernel(k_viscous<double, NN, BB, true>, grid, BB, s, ev, a);
            else launch_stage_kernel(k_viscous<double, NN, BB, false>, grid, BB, s, ev, a);
        }
        return hipGetLastError();
    });
}

template <class T, int NN, int BB>
void launch_residual_t(Epi epi, bool pers, const StageArgs &a, int grid, hipStream_t s, const LaunchEvents &ev)
{
    if (epi == Epi::Residual) {
        if (pers) launch_stage_kernel(k_residual<T, 0, NN, BB, true>, grid, BB, s, ev, a);
        else launch_stage_kernel(k_residual<T, 0, NN, BB, false>, grid, BB, s, ev, a);
    } else {
        if (pers) launch_stage_kernel(k_residual<T, 1, NN, BB, true>, grid, BB, s, ev, a);
        else launch_stage_kernel(k_residual<T, 1, NN, BB, false>, grid, BB, s, ev, a);
    }
}

hipError_t launch_residual(int N, int B, Epi epi, bool f32, bool pers, const StageArgs &a, int grid, hipStream_t s,
                           const LaunchEvents &ev)
{
    if (a.ntiles == 0) return hipSuccess;
    if (!grid_ok(a, grid, pers)) return hipErrorInvalidValue;
    return by_shape(N, B, [&](auto nc, auto bc) {
        constexpr int NN = decltype(nc)::value, BB = decltype(bc)::value;
        if (f32) launch_residual_t<float, NN, BB>(epi, pers, a, grid, s, ev);
        else launch_residual_t<double, NN, BB>(epi, pers, a, grid, s, ev);
        return hipGetLastError();
    });
}

int resident_blocks_per_cu(int kind, int N, int B, Epi epi, bool f32)
{
    // occupancy of the persistent kernels; it does not change at run time:
    // query each configuration once
    static int cache[2][kMaxN + 1][3][2][2] = {};
    int &slot = cache[kind & 1][N][B <= 128 ? 0 : B <= 256 ? 1 : 2][(int)epi & 1][f32];
    if (slot > 0) return slot;
    int n = 0;
    hipError_t e = by_shape(N, B, [&](auto nc, auto bc) {
        constexpr int NN = decltype(nc)::value, BB = decltype(bc)::value;
        const void *fn = nullptr;
        if (kind == kTileViscous)
            fn = f32 ? (const void *)k_viscous<float, NN, BB, true> : (const void *)k_viscous<double, NN, BB, true>;
        else if (f32)
            fn = epi == Epi::Residual ? (const void *)k_residual<float, 0, NN, BB, true>
                                      : (const void *)k_residual<float, 1, NN, BB, true>;
        else
            fn = epi == Epi::Residual ? (const void *)k_residual<double, 0, NN, BB, true>
                                      : (const void *)k_residual<double, 1, NN, BB, true>;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, BB, 0);
    });
    slot = e == hipSuccess && n > 0 ? n : 1;
    return slot;
}

// Every (lower, higher) pair of orders a mortar can join: the lower side has
// P >= 2 (its geometry must be resolved, 2 Pg <= P, Pg >= 1).
#define HDG_MORTAR_PAIRS(X) \
    X(3, 4) X(3, 5) X(4, 5) X(3, 6) X(4, 6) X(5, 6) X(3, 7) X(4, 7) X(5, 7) X(6, 7) X(3, 8) X(4, 8) X(5, 8) X(6, 8) X(7, 8)

bool mortar_pair_supported(int Nl, int Nh)
{
#define P_(l, h) if (Nl == l && Nh == h) return true;
    HDG_MORTAR_PAIRS(P_)
#undef P_
    return false;
}

template <int NL, int NH, class T>
static hipError_t launch_mortar_kernel(bool lift, const StageArgs &a, hipStream_t s, const LaunchEvents &ev)
{
    const int grid = (a.mcount + MortarShape<NL, NH>::SLOTS - 1) / MortarShape<NL, NH>::SLOTS;
    if (lift) launch_stage_kernel(k_mortar_lift<NL, NH, T>, grid, 256, s, ev, a);
    else launch_stage_kernel(k_mortar_flux<NL, NH, T>, grid, 256, s, ev, a);
    return hipGetLastError();
}

hipError_t launch_mortar(bool lift, int Nl, int Nh, bool f32, const StageArgs &a, hipStream_t s,
                         const LaunchEvents &ev)
{
    if (a.mcount == 0) return hipSuccess;
#define P_(l, h)                                                                          \
    if (Nl == l && Nh == h)                                                               \
        return f32 ? launch_mortar_kernel<l, h, float>(lift, a, s, ev) : launch_mortar_kernel<l, h, double>(lift, a, s, ev);
    HDG_MORTAR_PAIRS(P_)
#undef P_
    return hipErrorInvalidValue;
}

int feature_block(int N) { return N <= 5 ? 128 : N == 6 ? 256 : N == 7 ? 384 : 512; }

hipError_t launch_features(int N, const StageArgs &a, int grid, hipStream_t s)
{
#define F_(n, b)                                                                             \
    case n:                                                                                  \
        static_assert(tile_ept(n, b, kTileViscous) > 0, "feature tile does not fit");       \
        hipLaunchKernelGGL((k_features<n, b>), dim3(grid), dim3(b), 0, s, a);                \
        break;
    switch (N) {
        F_(2, 128) F_(3, 128) F_(4, 128) F_(5, 128) F_(6, 256) F_(7, 384) F_(8, 512)
    default: return hipErrorInvalidValue;
    }
#undef F_
    return hipGetLastError();
}

hipError_t launch_gmm_pass(int mode, const double *X, int64_t n, GmmState *st, double *partials, int nblocks,
                           double reg, double tol, hipStream_t s)
{
    if (nblocks < 1 || nblocks > kMaxGmmBlocks) return hipErrorInvalidValue;
#define G_(m)                                                                                          \
    case m:                                                                                            \
        hipLaunchKernelGGL(k_gmm_accum<m>, dim3(nblocks), dim3(kGmmBlock), 0, s, X, n, st, partials);  \
        hipLaunchKernelGGL(k_gmm_update<m>, dim3(1), dim3(kGmmUpdate), 0, s, partials, nblocks, n, reg, tol,  \
                           st);                                                                         \
        break;
    switch (mode) {
        G_(0) G_(1) G_(2) G_(3)
    default: return hipErrorInvalidValue;
    }
#undef G_
    return hipGetLastError();
}

hipError_t launch_gmm_assign(const double *X, int64_t n, const GmmState *st, const int64_t *eoff, const int8_t *Ne,
                             int N3, int64_t ne, double *p_visc, double *elem_pv, uint8_t *flags, hipStream_t s)
{
    const int64_t grid = (ne + kGmmBlock / 64 - 1) / (kGmmBlock / 64);
    hipLaunchKernelGGL(k_gmm_assign, dim3((unsigned)grid), dim3(kGmmBlock), 0, s, X, n, st, eoff, Ne, N3, ne, p_visc,
                       elem_pv, flags);
    return hipGetLastError();
}

hipError_t launch_reduce_mixed(const double *r, const double *mass, const int64_t *eoff, const int8_t *Ne,
                               int64_t n_elem, double *partials, int nblocks, double *final13, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partial_mixed, dim3(nblocks), dim3(256), 0, s, r, mass, eoff, Ne, n_elem, partials);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partials, nblocks, final13);
    return hipGetLastError();
}

hipError_t launch_wave_speed(const double *q, const int64_t *eoff, const int8_t *Ne, int N, int64_t n_elem,
                             double c0sq, double *partials, int nblocks, double *final2, hipStream_t s)
{
    if (nblocks < 1 || n_elem < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wave_speed_partial, dim3(nblocks), dim3(256), 0, s, q, eoff, Ne, N, n_elem, c0sq, partials);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_max2_final, dim3(1), dim3(256), 0, s, partials, nblocks, final2);
    return hipGetLastError();
}

bool shape_supported(int N, int B)
{
    return by_shape(N, B, [](auto, auto) { return hipSuccess; }) == hipSuccess;
}

hipError_t launch_reduce(int N, const double *r, const double *mass, int64_t n_elem, double *partials,
                         int nblocks, double *final13, hipStream_t s)
{
#define C_(n) launch_reduce_n<n>(r, mass, n_elem, partials, nblocks, final13, s)
    HDG_DISPATCH_N(N, C_)
#undef C_
}

hipError_t scratch_address(int device, double **ptr)
{
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // called with `device` current: each GPU holds its own copy of the
        // array at its own address
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *ptr = addr[device];
    return hipSuccess;
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
