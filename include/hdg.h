/*
 * hdg.h -- C ABI of the hybrid Navier-Stokes-LES / Euler DGSEM residual library
 * for AMD Instinct MI355X (gfx950).
 *
 * The operation is the spatial residual of a discontinuous Galerkin spectral
 * element method (DGSEM) on curvilinear hexahedra, in which every element
 * carries an equation flag: flagged (viscous/turbulent) elements solve the
 * Navier-Stokes equations with an LES eddy viscosity, the others the Euler
 * equations, and neighbours of either kind couple through numerical face
 * fluxes.  Paper: Otmani, Mateo-Gabin, Rubio, Ferrer, "Accelerating high order
 * discontinuous Galerkin solvers through a clustering-based
 * viscous/turbulent-inviscid domain decomposition" (arXiv 2403.05463):
 *   - the per-element choice of equations and the three kinds of face
 *     coupling: Sec. 2.3;
 *   - the element region ID that the flag stands for: Sec. 2.1 (element
 *     means of node memberships);
 *   - the equations (convective flux, viscous + turbulent stress, Vreman
 *     model): App. A;
 *   - the DGSEM discretisation (mapped element, contravariant fluxes, weak
 *     form with a numerical flux, BR1 viscous treatment, collocated
 *     quadrature): App. B;
 *   - the low-storage third-order explicit Runge-Kutta time marching: Sec. 2.3.
 * Equation system used here: incompressible flow in artificial-compressibility
 * form with unknowns (p, u, v, w) and unit density,
 *     dp/dt + c0^2 div u = 0,   du/dt + div(u u + p I) = div(2 (nu + nu_t) S),
 * with the viscous right-hand side present only on flagged elements.
 *
 * Conventions
 *   N = P + 1 Gauss-Lobatto-Legendre nodes per direction, N^3 per element.
 *   State / residual layout: element-major, then field (p, u, v, w), then node
 *   a + N b + N^2 c (a along xi).  Element e starts at offset 4 N^3 e.
 *   Geometry: (Pg+1)^3 control points per element at equispaced reference
 *   positions -1 + 2k/Pg, stored [e][3][(Pg+1)^3], x index fastest.
 *   Local faces: 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+.  Face
 *   coordinates (a, b): (eta, zeta) on faces 0/1, (xi, zeta) on 2/3, (xi, eta)
 *   on 4/5.  orient[e][f] maps my face coordinates to the neighbour's:
 *   (s, t) = bit0 ? (b, a) : (a, b); a' = bit1 ? N-1-s : s; b' = bit2 ? N-1-t : t.
 *   nbr[e][f] >= 0 is the neighbouring element; HDG_WALL (no-slip wall, ghost
 *   state (p, -u)) or HDG_FARFIELD (ghost state q_inf) marks a boundary face.
 *
 * Ownership
 *   The caller owns every state, residual and RK buffer (device pointers,
 *   e.g. from torch tensors).  The library owns geometry, metric terms,
 *   connectivity, element lists and its scratch (face viscous-flux traces, the
 *   RK ping-pong state, reduction partials) from hdg_mesh_create to
 *   hdg_mesh_destroy.  hdg_residual, hdg_rk3_steps, hdg_reduce and
 *   hdg_max_wave_speed allocate no device memory.  These calls do: hdg_mesh_set_flags (new tile lists),
 *   hdg_mesh_autotune (a trial buffer, freed before it returns), the first
 *   hdg_cluster_features / hdg_cluster_fit on a mesh (feature tile lists, EM
 *   partials; kept until hdg_mesh_destroy) and the first RK call after graphs
 *   are enabled (graph instantiation).
 *
 * Errors
 *   Every call returns an hdg_status and never throws across the ABI;
 *   hdg_last_error() gives a thread-local message for the last failure.
 *   hdg_mesh_create validates the mesh (symmetric connectivity, mutually
 *   inverse orientation codes, positive Jacobian).  Kernel launch failures
 *   map to HDG_EHIP.  Calls taking a stream are asynchronous on it, except
 *   hdg_reduce, hdg_max_wave_speed, hdg_mesh_autotune, hdg_batch_autotune
 *   and hdg_cluster_fit, which synchronise it.  hdg_mesh_set_flags and hdg_mesh_set_params wait
 *   for the device; hdg_timing_read and hdg_timing_samples wait for the
 *   launches they report.
 */
#ifndef HDG_H
#define HDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx hdg_ctx;
typedef struct hdg_mesh hdg_mesh;

typedef enum {
    HDG_OK = 0,
    HDG_EINVAL = -1,        /* bad argument (null pointer, size, code) */
    HDG_ENOMEM = -2,        /* device or host allocation failed */
    HDG_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    HDG_EUNSUPPORTED = -4,  /* valid request the library does not implement */
    HDG_EMESH = -5,         /* inconsistent mesh description */
    HDG_ENONFINITE = -6     /* hdg_reduce found a NaN or Inf */
} hdg_status;

typedef enum { HDG_F64 = 0, HDG_F32 = 1 } hdg_prec;

enum { HDG_WALL = -1, HDG_FARFIELD = -2 };
enum { HDG_LES_NONE = 0, HDG_LES_SMAGORINSKY = 1, HDG_LES_VREMAN = 2 };
enum { HDG_ROE = 0, HDG_RUSANOV = 1 };

/* Kernel classes reported by hdg_timing_read. */
enum {
    HDG_KERNEL_VISCOUS = 0,   /* flagged elements: BR1 gradient, LES, viscous divergence and face traces */
    HDG_KERNEL_RESIDUAL = 1,  /* every element: convective divergence, face fluxes, -1/J (or fused RK stage) */
    HDG_KERNEL_MORTAR = 2,    /* faces between elements of different order (BR1 lift, numerical flux) */
    HDG_KERNEL_COUNT = 3
};

/* Mesh description (Sec. 2.1: per-element region ID; App. B: curvilinear
 * hexahedra mapped from the reference cube by a polynomial map).  All
 * pointers are host pointers read during hdg_mesh_create only. */
typedef struct {
    int32_t n_elem;
    const int32_t *P;          /* [n_elem] polynomial order, 1..7, per element (Sec. 2.2: the
                                  order set per element from the regions, p-nonconforming
                                  faces between them).  A face between
                                  orders is coupled through a mortar of the higher order: the
                                  lower side's traces are extended by their own interpolants,
                                  the Roe + BR1 flux is evaluated on the mortar with the higher
                                  side's normal, and the lower side's surface integral is exact
                                  on the mortar.  Where orders meet, the curl-form metric
                                  terms are built from a product field x_l grad x_m whose
                                  boundary values are restricted (on such a face to degree
                                  P_lo - 1 along each tangential component's own direction
                                  and P_lo across it; on an edge where orders differ to the
                                  lowest order around it minus one along the edge), so that
                                  both sides of the face share one polynomial normal and a
                                  constant state stays constant on curved meshes.  Such
                                  faces need a lower order >= 2 and >= geom_order
                                  (HDG_EUNSUPPORTED otherwise). */
    int32_t geom_order;        /* Pg >= 1: geometry control points per direction minus one */
    const double *xyz_geom;    /* [n_elem][3][(Pg+1)^3] */
    const uint8_t *flag;       /* [n_elem] 1: Navier-Stokes + LES, 0: Euler (Sec. 2.3) */
    const int32_t *nbr;        /* [n_elem][6] */
    const int8_t *nbr_face;    /* [n_elem][6] the neighbour's local face, -1 on boundaries */
    const int8_t *orient;      /* [n_elem][6] orientation code 0..7 */
} hdg_mesh_desc;

/* Physical and scheme parameters. */
typedef struct {
    double c0sq;         /* artificial sound speed squared, > 0 */
    double nu;           /* kinematic viscosity on flagged elements, >= 0 */
    int32_t les_model;   /* HDG_LES_* (App. A: Vreman; Smagorinsky also offered) */
    double C_les;        /* Cs (Smagorinsky) or Cv (Vreman), >= 0 */
    int32_t mixed_face;  /* viscous flux on a face with one Euler side: 0 = BR1 mean with
                            a zero Euler-side flux, 1 = no viscous flux */
    double q_inf[4];     /* far-field state (p, u, v, w) */
    int32_t riemann;     /* numerical flux of the convective terms: HDG_ROE (Sec. 2.3) or
                            HDG_RUSANOV (mean flux minus the larger spectral radius
                            |u_n| + sqrt(u_n^2 + c0^2) of the two traces times the jump) */
} hdg_params;

/* Bind a context to HIP device `device`.  hdg_finalize releases the
 * caller's hold on it; the context (its operator tables on the device) lives
 * on until the last mesh and batch made from it are destroyed as well, so the
 * handles may be released in any order.  Each handle is released once. */
hdg_status hdg_init(hdg_ctx **ctx, int32_t device);
void hdg_finalize(hdg_ctx *ctx);

/* Set-up of the discretisation of App. B on the mesh: validate it, build
 * the Gauss-Lobatto-Legendre rules, node geometry, metric terms J and Ja
 * (curl form; translated elements share one block), face normals, the
 * mortars between elements of different order (Sec. 2.2), element lists,
 * and upload them.  The equation flag of each element (Sec. 2.1 regions)
 * comes with the description.  Synchronous.  HDG_EMESH on inconsistent
 * connectivity or J <= 0, HDG_EUNSUPPORTED on a face between orders whose
 * lower order is below 2 or below geom_order.
 * State layout: element after element, [4][(P_e+1)^3] each. */
hdg_status hdg_mesh_create(hdg_ctx *ctx, const hdg_mesh_desc *desc, const hdg_params *params,
                           hdg_mesh **out);
void hdg_mesh_destroy(hdg_mesh *mesh);

/* Replace the equation flags (a new clustering, Sec. 2.3 static/dynamic
 * clustering).  Host array [n_elem].  Synchronous. */
hdg_status hdg_mesh_set_flags(hdg_mesh *mesh, const uint8_t *flag_host);
hdg_status hdg_mesh_set_params(hdg_mesh *mesh, const hdg_params *params);

/* Sizes: nodes = n_elem N^3, state_len = 4 nodes (doubles), bytes of device
 * memory the mesh holds, number of flagged elements.  Any pointer may be NULL. */
hdg_status hdg_mesh_info(const hdg_mesh *mesh, int64_t *n_nodes, int64_t *state_len,
                         int64_t *device_bytes, int32_t *n_viscous);

/* Distinct metric blocks the kernels read.  Elements whose control points,
 * relative to their first one, agree to 1e-12 of the element's size (and
 * whose orders agree) are translates of one another with the same metric
 * terms (App. B: J and Ja depend only on derivatives of the map); each reads
 * the block of the first of them, and the processing order keeps such
 * elements together.  An extruded mesh of k identical layers has n_elem / k
 * blocks; a mesh without repeated elements has n_elem. */
hdg_status hdg_mesh_metric_blocks(const hdg_mesh *mesh, int64_t *blocks);

/* Physical coordinates of the collocation nodes, host array [n_elem][3][N^3]. */
hdg_status hdg_mesh_node_coords(const hdg_mesh *mesh, double *xyz_host);

/* Host-only (no device needed): the geometry hdg_mesh_create would build for
 * this description (App. B mapping): node coordinates xyz [n_elem][3][N^3],
 * Jacobian J [n_elem][N^3], contravariant metric terms Ja [n_elem][3 (i)][3 (d)][N^3]
 * in curl form, and the GLL rule xi[N], w[N], D[N*N] (D[i*N+j] = l_j'(xi_i)).
 * Any output may be NULL.  Validates the description like hdg_mesh_create. */
hdg_status hdg_mesh_geometry(const hdg_mesh_desc *desc, double *xyz, double *J, double *Ja,
                             double *xi, double *w, double *D);

/* R = dq/dt of the semi-discrete hybrid DGSEM (App. B with the Sec. 2.3
 * coupling), for device state q_dev (double, [e][4][N^3]) into device r_dev
 * (same layout, must not alias q_dev).
 *   HDG_F64: all arithmetic in double, r_dev is double.
 *   HDG_F32: contractions, fluxes and their accumulation in float, from one
 *            float rounding of the metric terms, face geometry and derivative
 *            matrix; r_dev is float. */
hdg_status hdg_residual(hdg_mesh *mesh, const void *q_dev, void *r_dev, hdg_prec prec, void *stream);

/* nsteps steps of the three-stage low-storage RK (Sec. 2.3; Williamson 2N
 * coefficients A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15)) on the device
 * state q_dev in place.  dq_dev is the caller's second register (same length);
 * its content on entry is ignored and on return unspecified: a step's first
 * stage does not read the register (A = 0), so its last stage does not store
 * it.  dt > 0 fixed.  prec selects the residual arithmetic (as in
 * hdg_residual); the stage accumulation dq = A dq + dt R, q += B dq and both
 * registers are double in either case. */
hdg_status hdg_rk3_steps(hdg_mesh *mesh, double *q_dev, double *dq_dev, double dt, int32_t nsteps,
                         hdg_prec prec, void *stream);

/* With graphs enabled (the default) and kernel timing off, hdg_rk3_steps
 * captures two RK steps (six stages) once per (q, dq, dt, prec) into a HIP
 * graph on a private stream and replays it on the caller's stream; an odd
 * last step runs eagerly.  Results are bitwise identical to eager launches.
 * Re-flagging, new parameters or launch shapes drop the captured graph. */
hdg_status hdg_mesh_set_graphs(hdg_mesh *mesh, int32_t enable);

/* Per-field reductions of a device array in state layout, with the
 * quadrature of App. B (GLL weights times J at each node): mass-weighted sum
 * sum w_a w_b w_c J r (the discrete conservation statement of the scheme's
 * single-valued face fluxes, Sec. 2.3), mass-weighted L2 norm and max
 * |r|.  Host outputs, any may be NULL.  Synchronises the stream.
 * HDG_ENONFINITE if any entry is NaN or Inf (outputs still written). */
hdg_status hdg_reduce(hdg_mesh *mesh, const double *r_dev, double out_sum[4], double out_l2[4],
                      double out_max[4], void *stream);

/* Allocation-free variant of hdg_reduce, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same reductions of the device array r_dev
 * (state layout) with the same kernels and workgroup count, so the results
 * are bitwise those of hdg_reduce; the partial sums live in a fixed device
 * array of the library (1024 workgroups x 13 doubles, 104 KiB per GPU, held
 * until the process ends) and the results go to the caller's device buffer
 * out_dev[13]: out_dev[f] = sum w_a w_b w_c J r_f, out_dev[4 + f] = the same
 * of r_f^2 (the square of hdg_reduce's L2 norm), out_dev[8 + f] = max |r_f|,
 * out_dev[12] = 1.0 if any entry is NaN or Inf, else 0.0 (f = p, u, v, w).
 * Asynchronous on `stream`: no host wait, no allocation, no library routine
 * that allocates.  The scratch array is shared by every call on one GPU, so
 * calls that overlap on a GPU (concurrent streams, other threads) race; it
 * needs no clearing (every partial a call reads, it has written).
 * HDG_EINVAL on a NULL argument; HDG_EUNSUPPORTED if the mesh needed more
 * partial sums than the array holds (not the case for any mesh hdg_mesh_create
 * builds: it uses at most 1024 workgroups). */
hdg_status hdg_reduce_noalloc(hdg_mesh *mesh, const double *r_dev, double *out_dev, void *stream);

/* Largest wave speed of the state q_dev (device, state layout), for the time
 * step of the explicit RK (Sec. 2.3): the flux Jacobian of the
 * artificial-compressibility system along a unit normal n has eigenvalues
 * u.n and u.n +- sqrt((u.n)^2 + c0^2), so the largest magnitude over all n
 * at a node is |u| + sqrt(|u|^2 + c0^2); *out_host receives its maximum over
 * every node.  Uses the mesh's reduction buffers (one such call or
 * hdg_reduce at a time per mesh), allocates nothing, synchronises the
 * stream.  HDG_EINVAL on a NULL argument; HDG_ENONFINITE if a velocity is
 * NaN or Inf (*out_host is then the maximum over the finite nodes). */
hdg_status hdg_max_wave_speed(hdg_mesh *mesh, const double *q_dev, double *out_host, void *stream);

/* Kernel timing: while enabled, every launch the mesh makes is serialised on
 * its stream and carries a pair of HIP events that the dispatch itself
 * records at the kernel's start and end (hipExtLaunchKernelGGL), so that a
 * launch's time is the kernel's own duration (up to 65536 launches are
 * kept).  hdg_timing_read
 * synchronises on the last event, then returns the summed duration and count
 * of the launches of one kernel class (HDG_KERNEL_*) since enabling. */
hdg_status hdg_timing_enable(hdg_mesh *mesh, int32_t enable);
hdg_status hdg_timing_read(hdg_mesh *mesh, int32_t kernel_class, double *total_ms, int64_t *launches);

/* Per-launch durations (microseconds, launch order) of one kernel class
 * since timing was enabled: us[0 .. min(*count, capacity)) is filled and
 * *count receives the number of launches recorded.  us may be NULL when
 * capacity is 0 (a size query).  Synchronises with the recorded events.
 * HDG_EINVAL on a NULL mesh or count or a bad class. */
hdg_status hdg_timing_samples(hdg_mesh *mesh, int32_t kernel_class, float *us, int64_t capacity, int64_t *count);

/* Launch configuration of one kernel class for one precision and one order N
 * = P + 1.  Work is cut into tiles of same-order, same-class elements, one
 * tile per workgroup of `block` lanes (128, 256 or 512, and 384 for N = 7; an
 * element takes N^3 lanes from P = 3 on rounded to whole 64-lane waves, fewer
 * elements share a wave below); `persistent` launches only as many workgroups as stay
 * resident, each walking its XCD's share of the tiles, else one workgroup per
 * tile.  The configuration changes launch shape only: results are bitwise
 * identical for every choice. */
typedef struct {
    int32_t block;
    int32_t persistent;
    double us_per_launch;   /* the autotuner's timing with this choice: a whole fused RK stage
                               (hdg_mesh_autotune) or this kernel's launch (hdg_batch_autotune);
                               0 when not tuned */
} hdg_launch_cfg;

/* Autotuner: for each precision, kernel class and order present (residual
 * kernels first, then viscous ones), times every supported (block,
 * persistent) pair on this mesh with reps whole fused RK stages reading q_dev
 * (device state, not modified), launched as the RK driver launches them
 * (every launch of the stage, with its concurrent branches), three times,
 * and keeps the pair with the least time.  Allocates a scratch register for the duration of the call,
 * writes the mesh's internal ping-pong state, drops any captured graph and
 * synchronises the stream.
 * Default without tuning: the smallest block that fits an element, one
 * workgroup per tile. */
hdg_status hdg_mesh_autotune(hdg_mesh *mesh, const double *q_dev, int32_t reps, void *stream);
/* kernel_class: HDG_KERNEL_VISCOUS or HDG_KERNEL_RESIDUAL (else HDG_EINVAL). */
hdg_status hdg_mesh_get_launch(const hdg_mesh *mesh, int32_t kernel_class, hdg_prec prec, int32_t N,
                               hdg_launch_cfg *out);
/* HDG_EUNSUPPORTED if no kernel exists for (N, block); us_per_launch ignored. */
hdg_status hdg_mesh_set_launch(hdg_mesh *mesh, int32_t kernel_class, hdg_prec prec, int32_t N,
                               const hdg_launch_cfg *cfg);

/* ---- Batches of independent meshes (continuous batching) ----
 *
 * A batch advances many independent solves together: each member is a mesh
 * created as above with its own device state q, RK register dq (both
 * caller-owned, double, state layout), time step dt and parameters (copied
 * from the mesh at add).  Every RK stage of the whole batch is one persistent
 * launch per (kernel kind, order present) over the union of the members'
 * element tiles, so small meshes share launches.  Each element is computed
 * exactly as for its mesh alone: a member's result is bitwise independent of
 * the rest of the batch.  Members can be added and removed between calls
 * (at RK step boundaries).  A mesh in a batch uses its internal ping-pong and
 * viscous scratch for the batch: do not step it on its own, re-flag it or
 * change its parameters while it is a member, and remove it before
 * destroying it.  All batch launches of one batch go to one stream. */
typedef struct hdg_batch hdg_batch;

hdg_status hdg_batch_create(hdg_ctx *ctx, int32_t max_members, hdg_batch **out);
void hdg_batch_destroy(hdg_batch *batch);
/* Adds `mesh` with its state q_dev, register dq_dev (distinct device arrays of
 * the mesh's state length) and dt > 0; returns the slot.  A mesh of several
 * orders joins the order-N launches with its order-N elements and adds its
 * own mortar launches to each stage.  HDG_ENOMEM when every slot is taken,
 * HDG_EINVAL if the mesh is already a member. */
hdg_status hdg_batch_add(hdg_batch *batch, hdg_mesh *mesh, double *q_dev, double *dq_dev, double dt,
                         int32_t *slot);
hdg_status hdg_batch_remove(hdg_batch *batch, int32_t slot);
hdg_status hdg_batch_info(const hdg_batch *batch, int32_t *n_members, int64_t *n_elements, int64_t *n_nodes);
/* nsteps RK steps of every member with its own dt (as hdg_rk3_steps; prec
 * selects the residual arithmetic).  After a membership change the first call
 * waits for the stream and rebuilds the tile lists; with graphs enabled (the
 * default) two steps at a time replay a captured HIP graph. */
hdg_status hdg_batch_rk3_steps(hdg_batch *batch, int32_t nsteps, hdg_prec prec, void *stream);
hdg_status hdg_batch_set_graphs(hdg_batch *batch, int32_t enable);
/* Autotuner over the batch's tiles (as hdg_mesh_autotune); writes every
 * member's RK register and ping-pong buffer, not its state. */
hdg_status hdg_batch_autotune(hdg_batch *batch, int32_t reps, void *stream);
hdg_status hdg_batch_get_launch(const hdg_batch *batch, int32_t kernel_class, hdg_prec prec, int32_t N,
                                hdg_launch_cfg *out);

/* ---- Clustering that produces the equation flags (Sec. 2.1) ----
 *
 * Node features: at every node of every element (the flags do not enter),
 * the invariants of the strain rate S = (J + J^T)/2 and rotation rate
 * W = (J - J^T)/2 of the velocity gradient J,
 *   Q_S = (tr(S)^2 - tr(S^2))/2,  R_S = -det(S)/3,  Q_Omega = -tr(W^2)/2,
 * with J the BR1 lifted gradient the viscous operator uses.
 * q: device FP64 state of the mesh (state layout).  features: device,
 * 3 * nodes doubles, [3][nodes] (Q_S, R_S, Q_Omega), node t of element e at
 * position eoff(e) + t, eoff(e) the element's first node (its state starts at
 * 4 eoff(e)).  Caller-owned buffers.  Asynchronous on `stream`. */
hdg_status hdg_cluster_features(hdg_mesh *mesh, const double *q, double *features, void *stream);

typedef struct {
    int32_t iterations;   /* most EM iterations after the initial split, 0..100000 */
    int32_t pad;
    double reg_covar;     /* ridge added to each covariance diagonal (scaled units), >= 0 */
    double tol;           /* stop after the M-step of an iteration whose mean log-likelihood
                             changed by less than tol from the previous one; 0: run them all */
} hdg_gmm_opts;

typedef struct {
    double feat_mean[3], feat_std[3];  /* centring and scales of (Q_S, R_S, Q_Omega): s_Q, s_Q^(3/2), s_Q */
    double weight[2];                  /* mixture weights, [0] inviscid, [1] viscous/rotational */
    double mean[2][3];                 /* component means, standardised units */
    double cov[2][3][3];               /* component covariances, standardised units */
    double log_likelihood;             /* mean per node of the last E-step; NaN without iterations */
    int32_t iterations;                /* E-steps taken */
    int32_t degenerate;                /* 1: Q_Omega constant, no second region, every p_v = 0 */
    int32_t converged;                 /* 1: stopped by tol before the iteration limit */
    int32_t pad;
    int64_t n_viscous;                 /* elements assigned to the viscous/rotational region */
} hdg_gmm_result;

/* Two-component Gaussian mixture over the node features and the element
 * regions (Sec. 2.1: memberships p_v, p_i = 1 - p_v per node; element means;
 * an element takes the region of the larger mean, a tie going viscous).
 * The features are centred and scaled by the flow's gradient scale: s_Q, the
 * pooled population standard deviation of Q_S and Q_Omega, for those two and
 * s_Q^(3/2) for R_S (1 if s_Q = 0); nodes with Q_Omega above its mean start in
 * the second component; EM runs up to opts->iterations times (fewer with
 * opts->tol > 0) with full covariances and a ridge on their diagonals; the
 * component with the larger mean Q_Omega is the viscous one.
 * features: device [3][nodes] as written by hdg_cluster_features.
 * p_visc (device [nodes]) and elem_pv (device [n_elem]) receive the node
 * memberships and element means when not NULL; flags (host [n_elem]) the
 * regions, 1 viscous.  Results are deterministic (fixed-order reductions).
 * Synchronises `stream`.  Apply the flags with hdg_mesh_set_flags. */
hdg_status hdg_cluster_fit(hdg_mesh *mesh, const double *features, const hdg_gmm_opts *opts,
                           hdg_gmm_result *result, double *p_visc, double *elem_pv, uint8_t *flags,
                           void *stream);

/* Plain device-to-device copy kernel (nbytes a multiple of 16, 16-byte aligned
 * pointers): the HBM bandwidth probe that calibrates traffic counters. */
hdg_status hdg_stream_copy(hdg_ctx *ctx, void *dst_dev, const void *src_dev, int64_t nbytes,
                           void *stream);

/* Message describing the last error on this thread ("" if none). */
const char *hdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
