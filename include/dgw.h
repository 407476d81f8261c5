/*
 * dgw.h -- C ABI of libdgw.so, the MI355X (gfx950) nodal discontinuous
 * Galerkin Maxwell solver hot path.
 *
 * What it computes (Kloeckner, Warburton, Hesthaven, "Solving Wave Equations
 * on Unstructured Geometries"):
 *   - the initial boundary value problem of the section "A Precise
 *     Mathematical Problem Statement": 2D transverse-magnetic Maxwell
 *     (eq. tm-maxwells, with +dEz/dx in the Hy equation) or 3D Maxwell
 *     (section "Adding Generality", three dimensions) on a polyhedral domain
 *     meshed by straight-sided, face-conforming simplices, with a perfectly
 *     electrically conducting (PEC) wall, no source, initial fields at t = 0;
 *   - the semi-discrete DG operator of eq. dg-strong-explicit: element-local
 *     differentiation by the reference matrices Dr/Ds(/Dt) with per-element
 *     geometric factors (eq. dg-diff-local-to-global), the face gather with
 *     the upwind flux of eq. max2d-numflux (factor 1/2, jumps
 *     [q] = q^- - q^+), and the LIFT = M^{-1} M^{dI} apply of eq. dg-lift;
 *   - an explicit Runge-Kutta method in time (section "Implementation
 *     Aspects"): five-stage, fourth-order, 2N-storage LSRK (Carpenter and
 *     Kennedy 1994), fused with the right-hand side into one kernel per stage.
 *
 * Conventions
 *   - Every call returns DGW_OK (0) or a negative DGW_E* code; the text of
 *     the last error on the calling thread is available from dgw_last_error().
 *     No exception crosses the ABI.
 *   - Pointers passed in are caller-owned and read (or written) only during
 *     the call.  Handles are library-owned until the matching destroy call.
 *   - A solver handle must not be used from two threads at once; the server
 *     calls are thread-safe.
 *   - Element order in every array is the caller's order given at creation,
 *     whatever the internal renumbering.  Node order inside an element is the
 *     lattice order of the equispaced set the warp & blend node map starts
 *     from: 2D for j in 0..N, for i in 0..N-j (node (i, j)); 3D for k in 0..N,
 *     for j in 0..N-k, for i in 0..N-j-k.  Reference simplex vertices:
 *     2D (-1,-1), (1,-1), (-1,1); 3D (-1,-1,-1), (1,-1,-1), (-1,1,-1),
 *     (-1,-1,1); element vertex v_i of elem_verts maps to reference vertex i.
 *   - Field arrays are [n_fields][K][Np], FP64 on the host.  n_fields = 3 in
 *     2D (Hx, Hy, Ez) and 6 in 3D (Hx, Hy, Hz, Ex, Ey, Ez).
 */
#ifndef DGW_H
#define DGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define DGW_OK           0
#define DGW_EINVAL      -1   /* bad argument (NULL, size, enum)              */
#define DGW_EMESH       -2   /* J <= 0, non-conforming face, bad vertex id   */
#define DGW_EORDER      -3   /* order outside 1..8 (2D) / 1..4 (3D solver)   */
#define DGW_ENOMEM      -4   /* host or device allocation failed             */
#define DGW_ETOOBIG     -5   /* footprint exceeds a size limit or budget     */
#define DGW_EDEVICE     -6   /* HIP runtime error (text in dgw_last_error)   */
#define DGW_ENONFINITE  -7   /* a field became NaN/Inf                       */
#define DGW_ECANCELLED  -8   /* request cancelled                            */
#define DGW_ENOTFOUND   -9   /* unknown ticket                               */
#define DGW_ENODEVICE  -10   /* call needs a device, handle is host-only     */

/* Static text for a code. */
const char *dgw_strerror(int code);
/* Text of the last error raised on the calling thread ("" if none). */
const char *dgw_last_error(void);

/* ------------------------------------------------------------------ inputs */
/* Mesh of straight-sided simplices (section "Construction of the Method":
 * straight-sided, face-conforming triangles; tetrahedra in 3D).
 * vx, vy (and vz in 3D): n_verts coordinates.  elem_verts: n_elems x (dim+1)
 * vertex ids, each element positively oriented (J > 0, counter-clockwise in
 * 2D); a face is shared by at most two elements and faces shared by none are
 * the PEC wall.  eps, mu: per-element relative permittivity/permeability
 * (NULL means 1); the 3D path supports eps = mu = 1 only. */
typedef struct {
    int32_t dim;                 /* 2 or 3 */
    int64_t n_verts;
    const double *vx, *vy, *vz;  /* vz NULL in 2D */
    int64_t n_elems;
    const int32_t *elem_verts;
    const double *eps, *mu;
} dgw_mesh;

/* Arithmetic of the stage.  Fields are FP32 in the first three variants.
 * The split variants evaluate each Op*B product (Op = [Dr | Ds | LIFT]) as
 * Op_hi*B_hi + Op_hi*B_lo + Op_lo*B_hi in 16-bit parts with FP32
 * accumulation on the matrix cores, and keep the geometric factors, normals
 * and surface Jacobians in FP64 on the device (split-FP16: 2D only; both
 * run on their own kernels: kernel 1 or 3 is DGW_EINVAL).  DGW_FP64
 * (section "Adding Generality", item "Double Precision": the method run
 * with double-precision fields) keeps the fields, the RK residual, the
 * operators, the factors and every operation of the stage in FP64 (kernel
 * 0, 2 or 3: the derivative-first kernel on the FP64 matrix cores; 1: the
 * scalar-operand kernel); 2D only, and the FP32 device-pointer calls
 * (dgw_set_fields_dev, dgw_get_fields_dev) return DGW_EINVAL for it.
 * Measured accuracy is stated beside every result (relative L2 against
 * the FP64 reference). */
typedef enum {
    DGW_FP32 = 0,        /* all contractions in FP32                              */
    DGW_SPLIT_BF16 = 1,  /* Dr/Ds/LIFT as BF16 hi+lo split products, FP32 accum.  */
    DGW_SPLIT_FP16 = 2,  /* same with FP16 hi+lo split products                   */
    DGW_FP64 = 3         /* FP64 fields and arithmetic throughout (2D)            */
} dgw_precision;

typedef struct {
    double alpha;        /* flux parameter: 1 upwind (default), 0 central          */
    double cfl;          /* multiplier on the CFL step rule (default 1)           */
    int32_t prec;        /* dgw_precision                                         */
    int32_t renumber;    /* 1 (default): space-filling-curve element order on GPU */
    int32_t device;      /* HIP device ordinal; -1 = host-only handle (setup only)*/
    int32_t kernel;      /* 2D stage kernel: 0 auto (FP32: 3 up to order 6, else 2;
                            FP64: 3), 1 scalar-operand VALU, 2 fused-operand
                            MFMA, 3 derivative-first MFMA (FP32, FP64), 4
                            element-major MFMA (FP32; fields stored element by
                            element, limited to 2 GiB field arrays).  3D has one
                            kernel per arithmetic (3, 4 are DGW_EINVAL there)   */
    void *hip_stream;    /* hipStream_t to launch on; NULL = library's own stream */
    /* Work partition of the stage (section "Rethinking the Work Partition"):
     * elements per lane of the 2D derivative-first FP32 kernel (0 or 1: one,
     * 2: two, i.e. 32 elements per wave); wave_private = 1: in 3D each wave
     * reads partner traces only from its own 16 elements' LDS copy and the
     * tile loop runs without work-group barriers (0: the work-group's pair of
     * tiles is shared through LDS).  dgw_autotune searches both. */
    int32_t lane_elems;
    int32_t wave_private;
} dgw_opts;

/* Fill *o with the defaults (alpha 1, cfl 1, FP32, renumber 1, device 0). */
int dgw_opts_default(dgw_opts *o);

/* ------------------------------------------------------------------ reference element (host only) */
/* Nodal reference element of the given dim and order (section
 * "Implementation Aspects": Lagrange basis on warp & blend nodes, operators
 * from orthonormal simplex polynomials).  Any output pointer may be NULL.
 *   r, s, t : Np node coordinates (t only in 3D)
 *   Dr, Ds, Dt : Np x Np row-major differentiation matrices
 *   M : Np x Np mass matrix;  LIFT : Np x (Nfaces*Nfp) row-major, columns
 *   ordered face by face, each face's nodes in the order of dgw_face_nodes.
 *   face_nodes : Nfaces x Nfp volume-node indices of each face. */
int dgw_reference_element(int32_t dim, int32_t order, int32_t *Np, int32_t *Nfp,
                          double *r, double *s, double *t, double *Dr, double *Ds,
                          double *Dt, double *M, double *LIFT, int32_t *face_nodes);

/* ------------------------------------------------------------------ solver */
typedef struct dgw_solver dgw_solver;

typedef struct {
    int64_t steps;            /* steps taken by the last advance              */
    double dt;                /* step used                                    */
    double t;                 /* simulated time reached since set_fields      */
    double setup_s;           /* host setup + upload of dgw_create            */
    double solve_ms;          /* device time of the last advance (HIP events) */
    double dof_updates_per_s; /* n_fields*K*Np*steps / solve time             */
    int32_t kernel;           /* stage kernel in use (dgw_opts.kernel numbering, resolved) */
    int32_t groups_per_cu;    /* persistent work-groups per CU (0: not persistent)     */
    int32_t lane_elems;       /* elements per lane of the derivative-first FP32 kernel */
    int32_t wave_private;     /* 3D work partition in use (dgw_opts.wave_private)      */
} dgw_info;

/* Set up the discretisation of order `order` on `mesh` (host FP64), upload
 * operators and geometry, allocate the fields (zero).  The inputs are those of
 * the section "A Precise Mathematical Problem Statement": the domain meshed by
 * straight-sided simplices, the material eps, mu per element (eq.
 * tm-maxwells), the PEC wall on every face without a neighbour; the order N
 * fixes the local polynomial space of "Construction of the Method", and the
 * operators Dr, Ds(, Dt), M, LIFT and the affine factors are built as in
 * "Implementation Aspects" (eqs. dg-diff-local-to-global, dg-lift).  The
 * caller's arrays are read during the call only; the handle is library-owned
 * until dgw_destroy.  Errors: EINVAL,
 * EMESH, EORDER, ENOMEM, EDEVICE; ETOOBIG for 2^26 elements or more, for a
 * 2D field array of 2^32 values or more (n_fields * Np * K rounded up to 64
 * elements; partner traces are addressed by 32-bit element indices) and for
 * a 3D field array of 2 GiB or more (32-bit byte offsets). */
int dgw_create(const dgw_mesh *mesh, int32_t order, const dgw_opts *opts, dgw_solver **out);
void dgw_destroy(dgw_solver *s);

int dgw_sizes(const dgw_solver *s, int64_t *K, int32_t *Np, int32_t *n_fields);
/* Physical node coordinates, [K][Np] each, caller order (z NULL in 2D). */
int dgw_node_coords(const dgw_solver *s, double *x, double *y, double *z);
/* Time step of the CFL rule: cfl * (1/2) * min LGL spacing(N) *
 * min_k inradius_k sqrt(eps_k mu_k). */
int dgw_cfl_dt(const dgw_solver *s, double *dt);

/* Fields in/out, FP64 host arrays [n_fields][K][Np] (converted to the device
 * precision).  set_fields gives the initial value at t = 0 of the problem
 * statement ("A Precise Mathematical Problem Statement") as nodal values;
 * get_fields returns the fields at the time reached (t_final after
 * dgw_advance).  set_fields zeroes the RK residual and the time.  Both copy
 * through host memory synchronously; EINVAL for NULL, ENODEVICE for a
 * host-only handle. */
int dgw_set_fields(dgw_solver *s, const double *q);
int dgw_get_fields(dgw_solver *s, double *q);
/* Initial value at t = 0 (problem statement) computed on the device in FP64:
 * the closed-form PEC cavity mode of the 2D TM system (eq. tm-maxwells) or of
 * the 3D system, sampled at the nodes:
 * 2D Ez = sin(m pi x) sin(n pi y), H = 0 (mode = {m, n, -});
 * 3D E = (n cos(m pi x) sin(n pi y) sin(l pi z), -m sin cos sin, 0), H = 0. */
int dgw_set_cavity_mode(dgw_solver *s, const int32_t mode[3]);

/* Time integration by the explicit Runge-Kutta method of "Implementation
 * Aspects" (read as the five-stage fourth-order 2N-storage scheme of
 * Carpenter and Kennedy): take `nsteps` steps of size dt (dt <= 0: the CFL
 * step), each stage res <- a_s res + dt L(q), q <- q + b_s res with L the
 * operator of eq. dg-strong-explicit, fused into one kernel launch per stage
 * on the solver's stream, no host sync inside the loop; returns after the
 * stream has drained.  EDEVICE on a launch failure. */
int dgw_advance_steps(dgw_solver *s, int64_t nsteps, double dt);
/* Advance to t_final: with dt <= 0 the step is the CFL step shortened to
 * t_final / ceil(t_final / dt_cfl). */
int dgw_advance(dgw_solver *s, double t_final, double dt, int64_t *steps_taken);

/* One evaluation of the semi-discrete right-hand side L(q) of eq.
 * dg-strong-explicit: local differentiation with the chain rule (eq.
 * dg-diff-local-to-global), the face jumps and upwind flux of eq.
 * max2d-numflux (factor 1/2) with the PEC mirror state, and LIFT (eq.
 * dg-lift) -- the operation of the CPU right-hand side and of the GPU volume
 * and surface kernels of "A Minimal Implementation" -- evaluated by the same
 * fused stage kernel (RK coefficients a = 0, dt = 1, b = 0).  q and rhs are
 * caller-owned FP64 host arrays [n_fields][K][Np].  Leaves the solver's
 * fields and residual overwritten with q and L(q).  EINVAL for NULL. */
int dgw_rhs(dgw_solver *s, const double *q, double *rhs);

/* FP64 device reduction of the discrete energy
 * 0.5 * sum_k J_k sum_f w_f q_f^T M q_f (w = mu for H, eps for E): the
 * M-norm (mass matrix of "Implementation Aspects", |A_k| M on element k) that
 * the upwind flux of eq. max2d-numflux keeps non-increasing.  ENONFINITE
 * when the result is not finite. */
int dgw_energy(dgw_solver *s, double *energy);
/* Allocation-free form of dgw_energy, for callers that cannot allocate or
 * synchronise (code under HIP graph capture, tight serving loops): the same
 * FP64 reduction, bitwise the same value, written asynchronously on `stream`
 * (a hipStream_t; NULL = the solver's stream) to energy_dev, a caller-owned
 * device pointer to one double on the solver's device.  Calls no hipMalloc,
 * hipFree, host synchronisation or allocating library routine: the per-block
 * partial sums live in a static device array of the library (1024 doubles
 * per device, set up by dgw_create; the reduction uses 512 of them and
 * overwrites each one, so nothing needs clearing), shared by every call on
 * that device: calls that overlap in time on one device race and must be
 * ordered by the caller (one stream, or events).  No finiteness check (the
 * value is not read back): the caller tests it.  Errors: EINVAL (NULL
 * output), ENODEVICE, EDEVICE; ETOOBIG if the reduction needed more partials
 * than the static array holds. */
int dgw_energy_noalloc(dgw_solver *s, double *energy_dev, void *stream);
/* FP64 device reduction of the relative L2 error (mass-matrix norm, unit field
 * weights) of the current fields against the closed-form cavity mode at time
 * t (2D: uniform eps, mu of element 0; 3D: eps = mu = 1). */
int dgw_cavity_error(dgw_solver *s, const int32_t mode[3], double t, double *rel_l2);

int dgw_last_info(const dgw_solver *s, dgw_info *info);

/* Device-pointer plumbing for callers holding FP32 device buffers (e.g. torch
 * tensors): q_dev is [n_fields][K][Np] FP32 in caller order on the solver's
 * device, stream a hipStream_t (NULL = solver stream).  Asynchronous on that
 * stream.  DGW_EINVAL for a DGW_FP64 solver. */
int dgw_set_fields_dev(dgw_solver *s, const float *q_dev, void *stream);
int dgw_get_fields_dev(dgw_solver *s, float *q_dev, void *stream);
/* Launch `nsteps` steps on `stream` without waiting (for timing by the
 * caller); dt must be > 0. */
int dgw_launch_steps(dgw_solver *s, int64_t nsteps, double dt, void *stream);
/* Automated tuning over kernel variants (sections "Rethinking the Work
 * Partition" and "Using Run-Time Code Generation": time each variant of the
 * work partition and keep the fastest): time `stages` fused stages (<= 0: 10, after 2 untimed ones)
 * of every candidate on this solver's own mesh and buffers, and keep the
 * fastest for all later launches.  Candidates: each 2D kernel that serves the
 * solver's arithmetic (FP32: fused-operand MFMA, derivative-first MFMA with
 * one or two elements per lane, scalar-operand VALU, element-major MFMA;
 * FP64: derivative-first MFMA, VALU; split: its kernel), in 3D the shared
 * pair window and the wave-private partition, each persistent kernel at
 * 1 .. min(occupancy, 4) work-groups per CU.  All candidates compute the same arithmetic per element, so results
 * do not depend on the choice beyond the rounding differences between
 * kernels.  The fields, the residual and the time are restored bitwise
 * afterwards.  Allocates two state-sized device buffers for the duration of
 * the call; the solver must not be in use on another thread.  out may be
 * NULL.  Errors: ENODEVICE, ENOMEM, EDEVICE. */
#define DGW_TUNE_MAX 24
typedef struct {
    int32_t kernel;          /* chosen variant (dgw_opts.kernel numbering)           */
    int32_t groups_per_cu;   /* chosen persistent work-groups per CU (0: not persistent) */
    int32_t lane_elems;      /* chosen elements per lane (dgw_opts.lane_elems)       */
    int32_t wave_private;    /* chosen 3D partition (dgw_opts.wave_private)          */
    double best_us;          /* its mean stage time                                  */
    int32_t n_tried;
    int32_t tried_kernel[DGW_TUNE_MAX];
    int32_t tried_groups_per_cu[DGW_TUNE_MAX];
    int32_t tried_lane_elems[DGW_TUNE_MAX];
    int32_t tried_wave_private[DGW_TUNE_MAX];
    double tried_us[DGW_TUNE_MAX];
} dgw_tune_info;
int dgw_autotune(dgw_solver *s, int32_t stages, dgw_tune_info *out);

/* Kernel name and per-launch algorithmic HBM bytes and flops of one fused
 * stage (the units behind the roofline figures). */
int dgw_stage_cost(const dgw_solver *s, double *bytes, double *flops);

/* Device bytes dgw_create would allocate for this mesh, order and options
 * (fields, factors, tables, node coordinates); the request server admits by
 * this figure.  Host-only, no device call.  Errors: EINVAL, EORDER. */
int dgw_footprint(const dgw_mesh *mesh, int32_t order, const dgw_opts *opts, int64_t *bytes);

/* ------------------------------------------------------------------ request server */
/* Continuous batching of many independent cavity solves on one device.
 * Requests are admitted in arrival order while a slot is free and their
 * footprint fits the HBM budget; admitted requests are set up on host worker
 * threads (FP64 geometry, upload, field initialisation) while the device
 * keeps stepping the running ones.  All running requests of one order and
 * material class advance together: one batched launch per stage covers the
 * tiles of every such request (each with its own dt), launches of different
 * classes run on their own streams and overlap.  Steps are issued in chunks
 * that end where the next request finishes (or after max_chunk_steps), at
 * which point finished requests leave, their memory is released and newly
 * set-up requests join.  Per-element arithmetic does not depend on what else
 * runs, so a request's result is bitwise the same alone and in any mix.
 * The server calls are thread-safe; handles are library-owned. */
typedef struct dgw_server dgw_server;

typedef struct {
    int64_t hbm_budget_bytes;  /* admission limit on summed footprints (<= 0: 80% of free device memory) */
    int32_t max_slots;         /* maximum admitted requests (<= 0: 64)                                 */
    int32_t device;            /* HIP device ordinal                                                    */
    int32_t setup_threads;     /* host set-up / finalisation workers (<= 0: 4)                         */
    int32_t max_chunk_steps;   /* steps between admission points (<= 0: 64)                             */
} dgw_server_opts;

/* One solve: the mesh arrays (and q0) are copied by dgw_submit. */
typedef struct {
    dgw_mesh mesh;        /* 2D meshes; eps/mu per element or NULL                          */
    int32_t order;        /* 1..8                                                            */
    int32_t mode[3];      /* initial fields: the closed-form cavity mode (m, n) at t = 0    */
    const double *q0;     /* or explicit initial fields [3][K][Np] (caller order); NULL: mode */
    double t_final;       /* > 0; reached with ceil(t_final / dt_cfl) equal steps              */
    double alpha;         /* flux parameter in [0, 1]                                          */
    int32_t prec;         /* DGW_FP32                                                          */
    int32_t keep_fields;  /* 1: keep the final fields for dgw_wait                             */
} dgw_request;

typedef struct {
    int32_t status;        /* DGW_OK, DGW_ECANCELLED, or the error of a failed set-up          */
    int32_t order;
    int64_t K;
    int64_t steps;
    double dt;
    double energy;         /* FP64 device reduction of the final fields                         */
    double rel_l2_mode;    /* relative L2 vs the closed-form mode at t_final when the request
                              started from a mode with uniform eps, mu; else NaN                 */
    int64_t footprint_bytes;
    double t_arrival, t_admit, t_start, t_finish;  /* seconds since dgw_server_create          */
} dgw_result;

/* Errors: EINVAL, EDEVICE, ENOMEM. */
int dgw_server_create(const dgw_server_opts *opts, dgw_server **out);
/* Queue a request; non-blocking.  Errors: EINVAL, EORDER, ETOOBIG (footprint
 * above the budget: could never be admitted), ECANCELLED (server closing). */
int dgw_submit(dgw_server *srv, const dgw_request *req, uint64_t *ticket);
/* *done = 1 once the request has finished, failed or been cancelled.
 * Errors: ENOTFOUND (unknown or already collected ticket). */
int dgw_poll(dgw_server *srv, uint64_t ticket, int32_t *done);
/* Block until the request ends; fill *res (nullable) and, if q_out is not
 * NULL, the final fields [3][K][Np] in caller order (needs keep_fields).
 * Collects the ticket.  Returns the request's status (DGW_OK,
 * DGW_ECANCELLED, ...) or ENOTFOUND / EINVAL. */
int dgw_wait(dgw_server *srv, uint64_t ticket, double *q_out, dgw_result *res);
/* Cancel a request that has not finished; a running request leaves at the
 * next chunk boundary.  Errors: ENOTFOUND. */
int dgw_cancel(dgw_server *srv, uint64_t ticket);
/* Server-wide counters: requests completed, DOF-updates issued and the
 * device-busy seconds they took (summed chunk times). */
int dgw_server_stats(dgw_server *srv, int64_t *completed, double *dof_updates, double *busy_s);
/* Cancel everything not finished, wait for the workers, free the device
 * memory.  Uncollected results are discarded.  No other call on this server
 * may be in progress, or made afterwards. */
void dgw_server_destroy(dgw_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* DGW_H */
