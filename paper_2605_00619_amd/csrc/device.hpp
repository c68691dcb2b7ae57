// Device-side layout of an afe_cell_data object and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace afe {

// Reference data in device memory (one copy per object), sized for N <= 4;
// entries are indexed with the object's own np, nf, nt, nq.
constexpr int kRefNp = 35;                      // (N+1)(N+2)(N+3)/6 at N = 4
constexpr int kRefNf = 15;                      // (N+1)(N+2)/2
constexpr int kRefNt = 5;                       // N + 1 time nodes
constexpr int kRefNq = 343;                     // (N+3)^3 error-norm points
constexpr int kRefTiles = (kRefNp + 15) / 16;   // row tiles of the contraction
constexpr int kRefSteps = (3 * kRefNp + 3) / 4; // its k-steps of 4
struct DevRef {
    double M[kRefNp * kRefNp];       // M^[m][p] = int phi_m phi_p
    double K[3 * kRefNp * kRefNp];   // K^_d[m][p] = int phi_m d_d phi_p
    double D[3 * kRefNp * kRefNp];   // D^_d[m][p] = d_d phi_p (x_m)
    double Z[kRefNf * kRefNf];       // face mass on the reference triangle
    double zsum[kRefNf];             // int_tri phi_j = sum_i Z[i][j]
    double w[kRefNt];                // Gauss-Legendre weights on [0, 1]
    double tau[kRefNt];              // Gauss-Legendre nodes on [0, 1]
    double Ktau_inv[kRefNt * kRefNt];  // inverse of the upwind time operator
    double Ktau[kRefNt * kRefNt];      // upwind time operator psi_a(1) psi_b(1) - int psi_a' psi_b
    int fn[kRefNf];                  // face node -> reference node
    // K^ as the A operand of the sub-tet contraction on the matrix cores:
    // tile (row tile t, k-step j) of the 16 x 4 blocks of A[m][d np + p] =
    // K^_d[m][p], zero-padded, one double per lane of v_mfma_f64_16x16x4f64
    // (A[i][k] in lane i + 16 k), at (t * steps + j) * 64 + lane with
    // steps = (3 np + 3) / 4
    double Kfrag[kRefTiles * kRefSteps * 64];
    // The same for the mixed-precision contraction, whose inner index has a
    // fourth block: A[m][3 np + p] = M^[m][p], steps = np
    double KMfrag[kRefTiles * kRefNp * 64];
    // V^ = K^ transposed for the volume term of the corrector, the same
    // layout: A[m][d np + p] = K^_d[p][m]
    double Vfrag[kRefTiles * kRefSteps * 64];
    // volume quadrature of the error norms: points, weights (sum 1/6) and
    // basis values phi_m(xi_q) at [q * np + m]
    int nq;
    double qxi[kRefNq * 3];
    double qw[kRefNq];
    double qphi[kRefNq * kRefNp];
};

struct DevGrid {
    int N, np, nf, nt, nc;   // nc = 5 * nt columns of the space-time blocks
    int n_cells;
    int64_t ndof, nsub;
    int max_cell_dofs, max_cell_subtets;
    double gamma, mu, m1;
    double kappa, cv;         // heat conduction: energy flux - kappa grad T, T = p / (rho (gamma - 1) cv)
    int av;
    int mixed;                // 1: FP32 preconditioner for the predictor iteration
    int guess;                // 1: predictor start extrapolated from the previous step
    // Anderson history: slots 0..hist_small-1 of a cell in place (DOF-major, as
    // the cell's block), slots hist_small..depth-1 in the cell's pool slot
    // (hist_small = depth: no pool)
    int hist_small, pool_cap;
    int64_t pool_stride;      // doubles per pool slot: (depth - hist_small) * max_cell_dofs * nc
    // connectivity and geometry
    const int64_t *dof_ptr;   // [n_cells + 1]
    const int64_t *sub_ptr;   // [n_cells + 1]
    const int64_t *minv_ptr;  // [n_cells + 1] offsets of the dense M_i^{-1}
    const int32_t *conn;      // [nsub][np]
    const int32_t *sub_cell;  // [nsub]
    const double *geo;        // [nsub][10]
    const double *tri;        // [nsub][4]
    const int32_t *nbr_sub;   // [nsub]; -1 - b on boundary triangle b of a bounded mesh
    const int32_t *perm;      // [nsub][nf]
    // Dirichlet data of a bounded mesh: primitive states (rho, u, v, w, p) at
    // boundary face node b * nf + j and time node a, [n_btri * nf][nt][5]
    // (caller-owned; null when none are registered)
    const double *bstate;
    // their gradients d prim_k / d x_d, [n_btri * nf][nt][3][5] (caller-owned;
    // needed with viscosity or heat conduction)
    const double *bgrad;
    int64_t n_btri;
    const double *h, *vol;    // [n_cells]
    const double *mrow;       // [ndof]
    const int32_t *dof_cell;  // [ndof]
    const int32_t *inc_ptr, *inc_idx;
    const int32_t *finc_ptr, *finc_idx;
    const DevRef *ref;
    double *minv;             // dense M_i^{-1}, row-major, symmetric, rows padded to 16
    double *dscale;           // [ndof] Jacobi scales diag(M_i)^{-1/2}
    float *minv32;            // mixed: FP32 scaled inverse, rows padded to 32
    const int64_t *minv32_ptr;
};

// Work buffers of the predictor / corrector.
struct DevWork {
    double *x;       // [ndof][nc] current predictor iterate (final: the solution)
    double *R;       // [ndof][nc] assembled stiffness term (FP64 path)
    float *R32;      // [ndof][nc] mixed: scaled FP32 residual
    double *un5;     // [ndof][5] mixed: u^n DOF-major (written at the start of each predictor)
    double *S;       // [ndof][nc] M^{-1} R
    double *Sp;      // [4][ndof][nc] FP64: partial products of a split M^{-1} (tail iterations)
    double *rk;      // [nsub][np][nc] per-sub-tet contributions
    double *fprev;   // [ndof][nc] residual G(x) - x of the current iterate
    double *gprev;   // [ndof][nc] G(x) of the current iterate
    double *part;    // [n_cells][tiles of 64 DOFs][2 * 64 + 2] partial dots and norms
    double *dF;      // per cell: hist_small columns of n_c * nc
    double *dG;
    double *dFp, *dGp;   // history pool: pool_cap slots of pool_stride doubles
    int32_t *pool_slot;  // [n_cells] pool slot of the cell in this step, -1: none
    int32_t *pool_count; // [1] pool slots handed out in this step
    double *gram;    // [n_cells][63][63] Cholesky rows, [n_cells][63][63] Gram, [n_cells][63] scales
    int32_t *hist;   // [n_cells][2]: stored difference pairs
    double *trace;   // [nsub][nf][20]: qbar (5), Fbar (15) at face nodes
    double *vk;      // [nsub][np][5] volume-term contributions
    double *fc;      // [nsub][nf][5] face-term contributions
    double *rhs;     // [ndof][5]
    double *mu_cell; // [n_cells]
    double *beta;    // [n_cells]
    double *cflterm; // [n_cells]
    int32_t *iters;  // [n_cells] predictor iterations done in this step
    int32_t *status; // [8]: flags, first bad cell, -, troubled count, iterations min, max, sum (64 bit)
    double *gamma;   // [n_cells][63] Anderson coefficients
    int32_t *kuse;   // [n_cells] history columns used by the update
    int32_t *late;   // [n_cells] pass of the cell's time integrals: 0 early, 1 middle, 2 final
    int32_t *late2;  // [n_cells] pass of the cell's corrector: 0 early, 1 final
    double *dt;      // [1] time step of the current step
    double *dt_prev; // [1] time step of the last successful step
    int32_t *guess_ok; // [1] 1: x holds the converged predictor of that step
    const double *u; // state u^n of the current step, SoA [5][ndof] (caller-owned)
    double tol;      // predictor stop: max|G(q)-q| <= tol * max(1, max|G(q)|)
    int max_iter;
    int depth;
};

// One simulation as seen by the batched predictor kernels.
struct DevSlot {
    DevGrid g;
    DevWork w;
};

// Entries of the active lists: slot << kSlotShift | cell.
constexpr int kSlotShift = 24;
constexpr int kMaxSlots = 64;
constexpr int kMaxCellsPerSlot = 1 << kSlotShift;

enum : int { kStatusNoConv = 1, kStatusPositivity = 2, kStatusNonfinite = 4, kStatusHistoryPool = 8 };

// Grid sizes of one predictor iteration's kernels: workgroups of a
// persistent grid, 0 = one workgroup per work item.
struct IterShape {
    int g_sub = 0, g_gather = 0, g_minv = 0, g_dots = 0, g_solve = 0, g_update = 0;
};

// Events bracketing each launch of the predictor's M^{-1} kernel, and its
// byte counters: [0] algorithmic bytes (the packed triangle of M_i^{-1},
// n_i (n_i + 1) / 2 entries, plus the right-hand side read and the result
// written once, per cell and iteration), [1] bytes as stored and streamed.
constexpr int kMaxRounds = 16;
struct ProfileHooks {
    hipEvent_t start[kMaxRounds], stop[kMaxRounds];
    unsigned long long *bytes;
};

hipError_t launch_reset_status(const DevGrid &g, const DevWork &w, hipStream_t s);
hipError_t launch_mass_assemble(const DevGrid &g, hipStream_t s);
hipError_t launch_mass_invert(const DevGrid &g, hipStream_t s);
hipError_t launch_prim_to_cons(const DevGrid &g, const double *prim, double *u, hipStream_t s);
hipError_t launch_detect(const DevGrid &g, const DevWork &w, const double *u, hipStream_t s);
// Time step of eqn.timestep into *w.dt (cfl > 0) from the detector's cell
// terms; the largest term is also written to *smax.
hipError_t launch_cfl_dt(const DevGrid &g, const DevWork &w, double cfl, double h_min, double *smax, hipStream_t s);
hipError_t launch_set_dt(const DevWork &w, double dt, hipStream_t s);
// Predictor start for one slot: q = u^n at every time node, counters cleared,
// the slot's cells written to list[base ...].
hipError_t launch_pred_init(const DevGrid &g, const DevWork &w, int slot, int32_t *list, int64_t base, hipStream_t s);
hipError_t launch_set_count(int32_t *count, int value, hipStream_t s);
// One predictor iteration over the listed (slot, cell) entries of one group
// of slots with the same degree and precision.  n_upper bounds the list
// length (grids are sized from it, persistent ones capped by it; -1 when
// unknown, which needs persistent grids); max_cell_dofs and
// max_cell_subtets are maxima over the group.
// The predictor's M^-1 product of an FP64 cell splits its inner index over
// kMinvSplitK workgroups per row tile from iteration kMinvSplitAfter on.
constexpr int kMinvSplitK = 4;
constexpr int kMinvSplitAfter = 3;
// The update kernel takes items of 256 values, one per thread, when the list
// has at most kUpdFineTiles tiles of 64 DOFs (the last iterations: few cells,
// long histories), else one tile per item.
constexpr int kUpdFineTiles = 1024;

struct RoundArgs {
    int N, mixed, visc;  // visc: 0 inviscid, 1 viscosity, 2 viscosity and heat conduction
    const DevSlot *tab;
    const int32_t *list, *count;
    int32_t *next, *next_count;
    int n_upper, max_cell_dofs, max_cell_subtets;
    int split;  // M^-1 item split factor: 4 if a listed cell may split its product (tail, or unknown), else 1
    int upd_fine;    // update items of 256 values (1) or of one 64-DOF tile (0)
    IterShape shape;
    hipEvent_t ev0, ev1;
    unsigned long long *bytes;  // [2] algorithmic, as stored (see ProfileHooks); null: not counted
};
hipError_t launch_pred_round(const RoundArgs &a, hipStream_t s);
// Early passes over cells whose predictor is final while others still
// iterate (the lists' lengths, count, are known on the host):
//   clear_late:   late[] = 0 for one slot;
//   relabel_late: late[] 2 -> 1 for one slot (final pass -> middle pass);
//   mark_listed:  late[] = value for the cells of the listed entries;
//   clear_late2:  late2[] = 0 for one slot;
//   mark_late2:   late2[] = 1 for the listed cells and their face neighbours.
hipError_t launch_clear_late(const DevGrid &g, const DevWork &w, hipStream_t s);
hipError_t launch_relabel_late(const DevGrid &g, const DevWork &w, hipStream_t s);
hipError_t launch_mark_listed(const DevSlot *tab, const int32_t *list, int count, int value, hipStream_t s);
hipError_t launch_clear_late2(const DevGrid &g, const DevWork &w, hipStream_t s);
hipError_t launch_mark_late2(const DevSlot *tab, const int32_t *list, int count, hipStream_t s);
// Time integrals of the converged predictor for the sub-tets of cells with
// late[c] == which.
hipError_t launch_pred_post(const DevGrid &g, const DevWork &w, int which, hipStream_t s);
// Corrector (faces, right-hand side, M^-1 update of u, positivity) for the
// cells with late2[c] == which.
// max_blocks > 0 caps the grid of the M^-1 update (its items are then strided).
hipError_t launch_correct(const DevGrid &g, const DevWork &w, double *u, int which, hipStream_t s,
                          int max_blocks = 0);
// Predictor iteration counts of the step into status[4..7].
hipError_t launch_step_stats(const DevGrid &g, const DevWork &w, hipStream_t s);
// Physical coordinates of the error-norm quadrature points of every sub-tet,
// xq [nsub * nq][3], from the DOF coordinates dof_xyz [3][ndof].
hipError_t launch_l2_points(const DevGrid &g, const double *dof_xyz, double *xq, hipStream_t s);
// sum over sub-tets and points of w_q |det J| (u_h[var](x_q) - ref_q)^2 into
// *out (device), deterministic; partial [blocks] is scratch.
hipError_t launch_l2_error(const DevGrid &g, const double *u, int var, const double *ref, double *partial,
                           double *out, hipStream_t s);
int64_t l2_blocks(const DevGrid &g);
// Occupancy-derived persistent grid sizes for degree N, precision and
// viscosity (workgroups that fit on the device at once, per kernel).
IterShape resident_shape(int N, int mixed, int visc);

}  // namespace afe
