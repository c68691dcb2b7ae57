/*
 * afe.h -- C ABI of libafe: the ADER-AFE-DG hot path on one AMD Instinct GPU.
 *
 * The method (Michel, Diazzi, Boscheri: "Continuous 3D finite element subgrid
 * basis functions for discontinuous Galerkin methods on polyhedral meshes"):
 * each polyhedral cell P_i carries continuous P_N Lagrange functions on a
 * sub-tetrahedral grid (Sec. 4.1, eq:interp_u); one time step is a cell-local
 * space-time Galerkin predictor (Sec. 4.3, eq:ADER-localCauchy, eq:ader4)
 * followed by a quadrature-free corrector with Rusanov face fluxes (Sec. 4.4)
 * and a flattener-driven artificial viscosity (Sec. 4.5); the time step obeys
 * eqn.timestep (Sec. 4.2).
 *
 * Conventions for every call:
 *   - Pointers are host pointers unless the argument says "device".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that return host values synchronise it.
 *   - Errors are reported by the returned afe_status; nothing is thrown across
 *     the ABI.  afe_last_error() gives a message for the calling thread.
 *   - The state u is caller-owned device memory, FP64, SoA u[5][ndof] with the
 *     conserved variables (rho, rho u, rho v, rho w, rho E) and the DOFs in
 *     cell-major order (cell c owns [cell_dof_ptr[c], cell_dof_ptr[c+1]) ).
 *   - Everything reached from an afe_cell_data is owned by the library and
 *     released by afe_free.  A cell-data object may be used from one host
 *     thread at a time; calls on one object on different streams race.
 */
#ifndef AFE_H
#define AFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AFE_OK = 0,
    AFE_E_ARG = -1,               /* invalid argument                               */
    AFE_E_BAD_MESH = -2,          /* open cell, unmatched face, vertex seen twice   */
    AFE_E_DEGENERATE_SUBTET = -3, /* a sub-tetrahedron with |det J| <= 0            */
    AFE_E_NO_CONVERGENCE = -4,    /* predictor did not reach tol within max_iter    */
    AFE_E_POSITIVITY = -5,        /* rho <= 0 or p <= 0 at a DOF after the update   */
    AFE_E_HBM_BUDGET = -6,        /* device memory needed exceeds params.hbm_budget */
    AFE_E_HIP = -7,               /* a HIP runtime call failed                      */
    AFE_E_NONFINITE = -8          /* NaN or Inf in the state after the update       */
} afe_status;

/* Polyhedral mesh of a periodic cube [0, box)^3 or of a bounded domain (host
 * arrays, copied).  Each vertex is stored once; a face is a polygon listed
 * once, oriented outward from its owner by the right-hand rule; a corner's
 * position in the owner's frame is xyz[v] + face_vshift[corner] * box, and the
 * neighbour's seed in the owner's frame is shifted by nbr_shift * box, so the
 * neighbour sees the corner at xyz[v] + (face_vshift - nbr_shift) * box.
 * A face whose neighbour is -1 lies on the boundary of a bounded mesh (its
 * shifts are 0); the solution there is given by Dirichlet data, see
 * afe_set_boundary_states. */
typedef struct {
    int32_t n_vertices;
    const double *xyz;          /* [n_vertices][3]                              */
    int32_t n_faces;
    const int32_t *face_ptr;    /* [n_faces + 1] CSR offsets into face_vtx      */
    const int32_t *face_vtx;    /* [face_ptr[n_faces]] corner vertex ids         */
    const int8_t *face_vshift;  /* [face_ptr[n_faces]][3] corner image shifts    */
    const int32_t *face_cell;   /* [n_faces][2] owner, neighbour (-1: boundary)  */
    const int8_t *nbr_shift;    /* [n_faces][3] neighbour image shift            */
    int32_t n_cells;
    double box;                 /* edge of the periodic cube                    */
} afe_mesh;

enum { AFE_FP64 = 0, AFE_MIXED = 1 };

/* Physics and solver parameters (Sec. 2, Sec. 4.3, Sec. 4.5). */
typedef struct {
    double gamma;        /* ratio of specific heats (1.4 in the paper)              */
    double mu;           /* physical dynamic viscosity (0 = Euler)                  */
    double m1;           /* flattener constant m1 (0.1, Sec. 4.5)                   */
    int32_t av;          /* 1: artificial viscosity from the flattener              */
    int32_t max_iter;    /* predictor iteration cap                                 */
    double tol;          /* predictor stop: max|G(q)-q| <= tol * max(1, max|G(q)|); */
                         /* tol = 0: every cell takes exactly max_iter applications */
                         /* of the map (a fixed-sweep mode), which is not a failure */
    int32_t accel_depth; /* Anderson depth m of the predictor iteration (0 = plain)  */
    int32_t precision;   /* AFE_FP64; AFE_MIXED: the predictor iterates with an FP32  */
                         /* Jacobi-scaled copy of M_i^{-1} as preconditioner of the   */
                         /* FP64 residual of eq:ADER-localCauchy (same fixed point)   */
    size_t hbm_budget;   /* bytes of device memory the object may use (0 = no cap)  */
    int32_t predictor_guess; /* 0: every step starts the predictor iteration from    */
                         /* q = u^n at all time nodes; 1: from the previous step's    */
                         /* converged predictor of this object extrapolated in time   */
                         /* (Lagrange on the time nodes, shifted to u^n), when that   */
                         /* step succeeded on the same state and the cell is not      */
                         /* troubled.  The fixed point, hence the result up to the    */
                         /* stop test, is the same; fewer iterations are needed.      */
    int32_t history_cells; /* 0: every cell stores its whole Anderson history          */
                         /* (accel_depth difference pairs of its space-time block);   */
                         /* > 0: every cell stores 8 pairs in place and at most this   */
                         /* many cells at once take the other accel_depth - 8 from a   */
                         /* shared pool (memory for large meshes).  The results are   */
                         /* the same bits; a step in which more cells need the pool   */
                         /* fails with AFE_E_HBM_BUDGET.                               */
    double kappa;        /* heat conduction coefficient: the energy flux carries      */
                         /* -kappa grad T (Sec. 2); 0 = none, as in the paper's tests */
    double cv;           /* specific heat at constant volume: T = p / (rho R) with    */
                         /* R = (gamma - 1) cv (2.5 in the paper's viscous test)      */
} afe_params;

typedef struct {
    int64_t ndof;          /* total cell DOFs (per conserved variable)  */
    int32_t n_cells;
    int64_t n_subtets;
    int32_t N;             /* polynomial degree                         */
    int32_t max_cell_dofs; /* largest N_i                               */
    int32_t max_cell_subtets;
    size_t device_bytes;   /* device memory held by the object          */
    double h_min;          /* smallest cell diameter                    */
} afe_info;

typedef struct {
    int32_t iters_min, iters_max; /* predictor iterations over cells           */
    double iters_mean;
    int32_t n_troubled;           /* cells with flattener beta > 0             */
    int32_t status_cell;          /* first failing cell, -1 if none            */
} afe_step_report;

typedef struct afe_cell_data afe_cell_data;

/* Build the sub-tetrahedral grid and all per-cell data of `mesh` for degree N
 * (Sec. 4.1): every polygon is fanned about its vertex-mean centroid and coned
 * to the cell's vertex-mean centroid; the cell DOFs are the sub-tet nodes
 * without repetition; sub-tet Jacobians, boundary sub-triangles and their
 * pairing with the neighbour's, and the inverse cell mass matrices M_i^{-1}
 * (Sec. 4.4, M_i; Sec. 4.3, the stored inverse of K_1,i) are computed.
 * 1 <= N <= 3.  On success *out owns all device memory of the object.
 * Errors: AFE_E_ARG, AFE_E_BAD_MESH, AFE_E_DEGENERATE_SUBTET,
 * AFE_E_HBM_BUDGET, AFE_E_HIP. */
afe_status build_afe_cell_data(const afe_mesh *mesh, int32_t N, const afe_params *params,
                               void *stream, afe_cell_data **out);

/* Sizes of a built object. */
afe_status afe_query(const afe_cell_data *cd, afe_info *out);

/* Cell DOF offsets: cell_dof_ptr [n_cells + 1] (host, int64). */
afe_status afe_cell_dof_ptr(const afe_cell_data *cd, int64_t *cell_dof_ptr);

/* DOF coordinates in each cell's frame: xyz device [3][ndof]. */
afe_status afe_dof_coords(const afe_cell_data *cd, double *xyz, void *stream);

/* Sub-grid connectivity for inspection (host copies):
 *   subtet_ptr [n_cells + 1] int64, conn [n_subtets][np] int32 cell-local DOF of
 *   each sub-tet node (np = (N+1)(N+2)(N+3)/6, App. A node order),
 *   nbr_subtet [n_subtets] int32 global index of the neighbour's sub-tet on the
 *   same boundary triangle (-1 - b on boundary triangle b of a bounded mesh,
 *   b counting those triangles in ascending sub-tet order), nbr_perm
 *   [n_subtets][nf] int32 matching face node (j itself on a boundary triangle).
 * Any output pointer may be NULL. */
afe_status afe_connectivity(const afe_cell_data *cd, int64_t *subtet_ptr, int32_t *conn,
                            int32_t *nbr_subtet, int32_t *nbr_perm);

/* Dirichlet data of a bounded mesh (Sec. 5.1-5.2: the exact solution imposed
 * on all sides).  A boundary triangle's outside state in the Rusanov flux of
 * Sec. 4.4 is the given solution at its face nodes at the predictor's time
 * nodes t^n + tau_a dt: qbar = dt sum_a w_a q_a and Fbar = dt sum_a w_a F(q_a)
 * (Euler flux, or Navier-Stokes flux with the given gradient, below); the
 * detector of Sec. 4.5 counts no velocity jump across it.
 * afe_boundary_nodes writes *count = (boundary triangles) * nf, the boundary
 * face nodes (triangle b's face node j is node b * nf + j, triangles in
 * ascending sub-tet order), and, when not NULL, their coordinates xyz host
 * [count][3] and the N+1 time nodes tau host [N+1] in (0, 1).
 * afe_set_boundary_states registers prim, device [count][N+1][5]: the
 * primitive state (rho, u, v, w, p) at each boundary node and time node of the
 * next step; caller-owned, read by every following ader_step, ader_correct
 * and ader_step_noalloc, so the caller refills it (for the new t^n and dt)
 * before each step; NULL unregisters.  A step of a bounded object without
 * registered states fails with AFE_E_ARG.  With viscosity, heat conduction
 * or artificial viscosity the outside flux is the Navier-Stokes flux of the
 * given state with its gradient and the inside cell's viscosity:
 * afe_set_boundary_gradients registers grad, device [count][N+1][3][5], the
 * gradient d prim_k / d x_d of the primitive state at each boundary node and
 * time node (same ownership and refill rule); a viscous step of a bounded
 * object without it fails with AFE_E_ARG.  Bounded objects are stepped alone
 * with the caller's dt (afe_batch_attach fails with AFE_E_ARG).
 * Errors: AFE_E_ARG. */
afe_status afe_boundary_nodes(const afe_cell_data *cd, int64_t *count, double *xyz, double *tau);
afe_status afe_set_boundary_states(afe_cell_data *cd, const double *prim);
afe_status afe_set_boundary_gradients(afe_cell_data *cd, const double *grad);

/* Host-only construction of the same sub-grid (no device memory, no GPU):
 * afe_subgrid_sizes returns sizes[0] = number of sub-tets, sizes[1] = number
 * of DOFs; afe_subgrid_host fills caller-allocated host arrays:
 *   subtet_ptr, dof_ptr [n_cells + 1] int64; conn [nsub][np] int32;
 *   nbr_subtet [nsub] int32; nbr_perm [nsub][nf] int32;
 *   geo [nsub][10] (J^{-1} row-major, |det J|); tri [nsub][4] (2 * area of the
 *   boundary triangle, unit outward normal).  Any output may be NULL.
 * Errors as for build_afe_cell_data (no AFE_E_HIP). */
afe_status afe_subgrid_sizes(const afe_mesh *mesh, int32_t N, int64_t *sizes);
afe_status afe_subgrid_host(const afe_mesh *mesh, int32_t N, int64_t *subtet_ptr, int64_t *dof_ptr,
                            int32_t *conn, int32_t *nbr_subtet, int32_t *nbr_perm, double *geo, double *tri);

/* Convert primitive (rho, u, v, w, p) to conserved variables (Sec. 2, EOS):
 * prim and u are device [5][ndof]; they may alias. */
afe_status afe_prim_to_cons(afe_cell_data *cd, const double *prim, double *u, void *stream);

/* Time step of eqn.timestep for state u (device): runs the detector of
 * Sec. 4.5 (for mu_i) and returns dt = cfl * h_min / ((2N+1) max(|lambda| +
 * 2 |lambda^v| (2N+1)/h_i)) in *dt_host.  Synchronises `stream`. */
afe_status ader_cfl_dt(afe_cell_data *cd, const double *u, double cfl, double *dt_host, void *stream);

/* Detector + space-time predictor of Sec. 4.3 for every cell from state u
 * (device), time step dt.  Leaves in library buffers the time-integrated
 * volume term and the face traces used by ader_correct.  Non-convergence is
 * latched in the object's device status word (reported by ader_step). */
afe_status ader_predict(afe_cell_data *cd, const double *u, double dt, void *stream);

/* Corrector of Sec. 4.4 after ader_predict on the same u and dt: Rusanov
 * fluxes on all boundary sub-triangles, u <- u + M_i^{-1}(volume - faces)
 * in place, then the positivity check (latched in the status word). */
afe_status ader_correct(afe_cell_data *cd, double *u, double dt, void *stream);

/* One full ADER step u^n -> u^{n+1} in place (device u): predict + correct,
 * then one synchronisation to read the status word.  Fills *rep when not NULL.
 * Returns AFE_E_NO_CONVERGENCE, AFE_E_POSITIVITY or AFE_E_NONFINITE when the
 * step failed (u then holds the failed update). */
afe_status ader_step(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, void *stream);

/* ader_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step, the same kernels and the same result, but nothing is allocated
 * (no hipMalloc, hipFree or host-pinned allocation; ader_step allocates its
 * predictor lists on first use and again whenever it is handed another
 * state).  The lists, their lengths and the slot table live in a fixed
 * 16 MiB device array of the library, one per device, found once per device
 * with hipGetSymbolAddress; no side stream is used (the corrector runs after
 * the last predictor iteration on `stream`).  Limits: at most 2,097,120 cells
 * (AFE_E_ARG beyond), the current device must be the one cd was built on
 * (AFE_E_ARG), cd must not be attached to a batch (AFE_E_ARG).  Every call
 * on a device shares that device's array: calls that overlap on one device
 * (two host threads, or two streams without ordering) race.  Other errors
 * and the report as for ader_step. */
afe_status ader_step_noalloc(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, void *stream);

/* Copy the last predictor solution (the space-time nodal values q of
 * eq:ader4) to device memory q [ndof][(N+1)*5]: DOF-major, then time node,
 * then conserved variable. */
afe_status afe_predictor_state(const afe_cell_data *cd, double *q, void *stream);

/* Per-cell predictor iteration counts and viscosities of the last step
 * (host arrays [n_cells]); either may be NULL.  Synchronises `stream`. */
afe_status afe_cell_diagnostics(const afe_cell_data *cd, int32_t *iters, double *mu, void *stream);

/* Timing of the dominant kernel (the M_i^{-1} application of the predictor
 * iteration, Sec. 4.3 eq:ader4): when enabled, HIP events bracket each of its
 * launches on the object's stream and the kernel counts the bytes it moves.
 * afe_profile_read returns the sums since the last enable: *bytes the
 * algorithmic bytes, per cell and iteration the packed symmetric M_i^{-1}
 * (N_i (N_i + 1) / 2 entries: 8 bytes each in FP64, 4 in the mixed-precision
 * FP32 copy) plus the space-time block read and the result written once
 * (16 N_i 5(N+1) in FP64; 12 N_i 5(N+1) in mixed precision, FP32 in and FP64
 * out); *bytes_stored the bytes of the layout as stored and streamed.  Any
 * output pointer may be NULL. */
afe_status afe_profile_enable(afe_cell_data *cd, int32_t enable);
afe_status afe_profile_read(afe_cell_data *cd, double *kernel_ms, int64_t *launches, double *bytes,
                            double *bytes_stored);

/* Error norm of Sec. 5: ||e||_2 = (sum over cells of int_cell |u_h - u_e|^2)^(1/2)
 * for one conserved variable (var 0..4), each cell integral taken over its
 * sub-tets with a conical product of (N+3)-point Gauss-Legendre rules
 * (nq = (N+3)^3 points per sub-tet, exact for polynomials of degree 2N+3).
 * afe_l2_points writes *nq (host) and, when xq is not NULL, the points' physical
 * coordinates in each cell's frame, xq device [n_subtets * nq][3] (sub-tet
 * major), from the DOF coordinates dof_xyz device [3][ndof] of afe_dof_coords;
 * the caller evaluates u_e there (points may lie outside [0, box): a periodic
 * u_e wraps them).  afe_l2_error takes those values, ref device
 * [n_subtets * nq] (a NaN leaves its point out of the sum: the norm over a
 * part of the domain), and the state u device [5][ndof], and returns the norm in
 * *err (host); the sum is in a fixed order (bit-reproducible).  It uses the
 * object's work buffers: not concurrently with a step of the same object.
 * Synchronises `stream`.  Errors: AFE_E_ARG, AFE_E_HIP. */
afe_status afe_l2_points(afe_cell_data *cd, const double *dof_xyz, double *xq, int32_t *nq, void *stream);
afe_status afe_l2_error(afe_cell_data *cd, const double *u, int32_t var, const double *ref, double *err,
                        void *stream);

void afe_free(afe_cell_data *cd);
const char *afe_last_error(void);

/* Device memory build_afe_cell_data(mesh, N, params) would allocate, from
 * the mesh's per-cell vertex, face and polygon-edge counts and the closed
 * form of the sub-grid DOF count (Sec. 4.1); host only, no device memory.
 * Used to admit work against a device-memory budget.  Errors: AFE_E_ARG,
 * AFE_E_BAD_MESH (a cell without faces). */
afe_status afe_estimate_bytes(const afe_mesh *mesh, int32_t N, const afe_params *params, size_t *bytes);

/* ---------------------------------------------------------------- batches
 *
 * A batch steps several simulations (cell-data objects, each with its own
 * mesh, degree, parameters and state) together: one ADER step of every
 * attached simulation per afe_batch_step.  The predictor iterations of all
 * simulations with the same degree, precision and viscosity (physical or
 * artificial, or none) share each kernel launch
 * (their cells are packed into one list of (simulation, cell) entries, cells
 * of uneven size included); the time step of each simulation comes from its
 * own CFL number and state (eqn.timestep) and stays on the device.  Results
 * are bit-identical to stepping each simulation alone in a batch of one,
 * whatever else is attached and whatever launch shape is used.
 *
 * Ownership: the batch references, and does not own, the attached objects
 * and states; both must stay valid until detached or the batch is freed.
 * An object belongs to at most one batch.  Calls on one batch must come from
 * one host thread at a time.  The batch runs its work on a stream of its own,
 * ordered after the work already enqueued on `stream`, and `stream` is made
 * to wait for it before afe_batch_step returns. */
#define AFE_BATCH_SLOTS 64

typedef struct afe_batch afe_batch;

/* Launch shape of the predictor iteration.  Each kernel (sub-tet fluxes and
 * assembly, M_i^{-1} application, Anderson update) runs as a persistent grid
 * of `x` times the number of its workgroups that fit on the device at once
 * (x = 0: one workgroup per work item, sized from the current list length).
 * `rounds` iterations are enqueued between two reads of the number of cells
 * still iterating; with graph = 1 (every x > 0 required) the step's phases
 * and each group of rounds are captured once as HIP graphs and replayed.
 * Default {1, 0, 0, 2, 0}. */
typedef struct {
    double sub, minv, anderson;
    int32_t rounds; /* 1 .. 16 */
    int32_t graph;
} afe_launch_shape;

typedef struct {
    int32_t status;      /* afe_status of this simulation's step            */
    int32_t iters_min, iters_max;
    double iters_mean;   /* predictor iterations over its cells             */
    int32_t n_troubled;  /* cells with flattener beta > 0                   */
    int32_t status_cell; /* first failing cell, -1 if none                  */
    double dt;           /* time step taken                                 */
} afe_batch_report;

afe_status afe_batch_create(afe_batch **out);
void afe_batch_free(afe_batch *b);

/* Attach cd with device state u (SoA [5][ndof]) and CFL number cfl > 0;
 * *slot (may be NULL) receives its slot index in [0, AFE_BATCH_SLOTS).
 * Errors: AFE_E_ARG (full batch, object already in a batch, bad cfl). */
afe_status afe_batch_attach(afe_batch *b, afe_cell_data *cd, double *u, double cfl, int32_t *slot);
afe_status afe_batch_detach(afe_batch *b, afe_cell_data *cd);

/* One step of every attached simulation; reps (host, may be NULL) has
 * n_reps entries indexed by slot.  Returns the first failing simulation's
 * status (its state then holds the failed update), AFE_OK if none failed.
 * When the call fails before the step completes (AFE_E_ARG, AFE_E_HIP from a
 * launch, graph capture or allocation), every attached slot's report carries
 * that status, with zero iteration counts and dt. */
afe_status afe_batch_step(afe_batch *b, afe_batch_report *reps, int32_t n_reps, void *stream);

afe_status afe_batch_set_shape(afe_batch *b, const afe_launch_shape *shape);
afe_status afe_batch_get_shape(const afe_batch *b, afe_launch_shape *shape);

/* Autotuner: times one step of the attached simulations for each candidate
 * launch shape (coordinate search over the three grid multiples, the rounds
 * between reads and graph replay) on copies of their states, keeps the
 * fastest and returns it in *chosen (may be NULL).  The attached states are
 * not modified.  Allocates temporary device memory for the copies. */
afe_status afe_batch_tune(afe_batch *b, void *stream, afe_launch_shape *chosen);

/* As afe_profile_enable / afe_profile_read for the batch's M_i^{-1} launches
 * of its first group of simulations (graph replay is off while enabled). */
afe_status afe_batch_profile_enable(afe_batch *b, int32_t enable);
afe_status afe_batch_profile_read(afe_batch *b, double *kernel_ms, int64_t *launches, double *bytes,
                                  double *bytes_stored);

#ifdef __cplusplus
}
#endif
#endif /* AFE_H */
