// HIP kernels of the ADER-AFE-DG step for gfx950 (FP64 path).
//
// Layout: state u is SoA [5][ndof]; space-time blocks (predictor iterate,
// assembled stiffness term, M^{-1} applied) are DOF-major [ndof][nc] with
// nc = 5 (N+1) columns (time node major, conserved variable minor), so one
// DOF's space-time values are contiguous.  Every per-DOF accumulation is a
// gather over a fixed, ascending incidence list: no floating-point atomics,
// results are bit-reproducible.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <algorithm>
#include <cmath>

#include "device.hpp"

namespace afe {
namespace {

constexpr int kWave = 64;
constexpr int kMaxDepth = 63;  // Anderson history columns (a wave holds one per lane)

template <int N>
struct Dim {
    static constexpr int np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int nf = (N + 1) * (N + 2) / 2;
    static constexpr int nt = N + 1;
    static constexpr int nc = 5 * nt;
    static constexpr int npt = nt * np;                     // threads per sub-tet
    static constexpr int spb = (256 / npt) > 0 ? 256 / npt : 1;  // sub-tets per block
    static constexpr int threads = spb * npt;
};

// v of lane i (i the same in every lane), in every lane
__device__ inline double lane_bcast(double v, int i) {
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(unsigned(b)), i);
    const int hi = __builtin_amdgcn_readlane(int(unsigned(b >> 32)), i);
    return __hiloint2double(hi, lo);
}

// v of another lane of the same row of 16, chosen by a DPP control word
template <int kCtrl>
__device__ inline double dpp_f64(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Reduction over the 64 lanes of a wave (every lane active), the same bits in
// every lane: within each row of 16 by DPP (partner lane xor 1, xor 2, then
// the mirrored half-row and row, so each step combines two equal-sized
// disjoint sets and both partners compute the same value), then the four row
// results taken with readlane and combined in row order.
template <class Op>
__device__ inline double wave_reduce(double v, Op op) {
    v = op(v, dpp_f64<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    v = op(v, dpp_f64<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    v = op(v, dpp_f64<0x141>(v));  // row_half_mirror
    v = op(v, dpp_f64<0x140>(v));  // row_mirror
    return op(op(op(lane_bcast(v, 0), lane_bcast(v, 16)), lane_bcast(v, 32)), lane_bcast(v, 48));
}
__device__ inline double wave_sum(double v) {
    return wave_reduce(v, [](double a, double b) { return a + b; });
}
__device__ inline double wave_max(double v) {
    return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}
__device__ inline double wave_min(double v) {
    return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}

// Triangular solves of one wave, column by column, with the factor rows in
// LDS (L[j][i] = Ls[j][i], j > i): unknown i is acc_i / L[i][i] (rinv of lane
// i holds 1 / L[i][i]), broadcast from lane i, and lane j > i subtracts
// L[j][i] (lower) or L[i][j] (upper, the transposed factor) times it from its
// running residual acc_j.  Steps go in blocks of kSubBlock whose LDS reads are
// issued together.  n is the same in every lane; the result is in lane i.
constexpr int kSubBlock = 4;
template <bool kUpper>
__device__ inline double tri_solve(const double (*Ls)[kMaxDepth], double acc, double rinv, int n) {
    const int lane = threadIdx.x % kWave, lr = min(lane, kMaxDepth - 1);
    double x = 0.0;
    for (int b = 0; b < n; b += kSubBlock) {
        double l[kSubBlock];
#pragma unroll
        for (int u = 0; u < kSubBlock; ++u) {
            const int i = max(min(kUpper ? n - 1 - (b + u) : b + u, kMaxDepth - 1), 0);
            l[u] = kUpper ? Ls[i][lr] : Ls[lr][i];
        }
        // no branches inside the block, so that its reads stay ahead of it
#pragma unroll
        for (int u = 0; u < kSubBlock; ++u) {
            const bool step = b + u < n;
            const int i = max(min(kUpper ? n - 1 - (b + u) : b + u, kWave - 1), 0);
            const double xi = lane_bcast(acc * rinv, i);
            x = (step && lane == i) ? xi : x;
            const bool upd = step && (kUpper ? lane < i : (lane > i && lane < n));
            acc = upd ? fma(-l[u], xi, acc) : acc;
        }
    }
    return x;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// The per-cell kernels use several blocks per cell that share the cell's
// operands; this bijection gives every XCD a contiguous range of logical block
// ids, so the blocks of one cell run on one XCD and share its L2.
__device__ inline int xcd_block() {
    constexpr int kXcd = 8;
    const int bid = blockIdx.x, nb = gridDim.x;
    const int q = nb / kXcd, r = nb % kXcd;
    const int x = bid % kXcd, local = bid / kXcd;
    return x * q + min(x, r) + local;
}

// Leading dimension of the stored M_i^{-1}: rows padded to 128 bytes.
__device__ __host__ inline int64_t minv_ld(int64_t n) { return (n + 15) & ~int64_t(15); }

// Physical flux F[x][v] of the compressible Navier-Stokes equations (Sec. 2)
// at one point.  gq[x][v] = d q_v / d x_x feeds the viscous stress when
// mu != 0 and, with HEAT, the heat flux -kappa grad T when kappa != 0.
template <bool HEAT>
__device__ inline void ns_flux(const double q[5], const double gq[3][5], double gamma, double mu, double kappa,
                               double cv, double F[3][5]) {
    const double rho = q[0];
    const double ir = 1.0 / rho;
    const double v[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * v[0] + q[2] * v[1] + q[3] * v[2]));
    double sig[3][3] = {{p, 0, 0}, {0, p, 0}, {0, 0, p}};
    if (mu != 0.0) {
        double gv[3][3];  // gv[i][j] = d v_j / d x_i
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gv[i][j] = (gq[i][1 + j] - v[j] * gq[i][0]) * ir;
        const double dv = gv[0][0] + gv[1][1] + gv[2][2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                sig[i][j] += (i == j ? (2.0 / 3.0) * mu * dv : 0.0) - mu * (gv[i][j] + gv[j][i]);
    }
    for (int x = 0; x < 3; ++x) {
        F[x][0] = q[1 + x];
        for (int j = 0; j < 3; ++j) F[x][1 + j] = rho * v[x] * v[j] + sig[x][j];
        F[x][4] = v[x] * q[4] + (sig[0][x] * v[0] + sig[1][x] * v[1] + sig[2][x] * v[2]);
    }
    if (HEAT && kappa != 0.0) {
        // - kappa grad T, grad T = (grad e - v . grad v) / cv with e = rho E / rho
        const double e = q[4] * ir;
        for (int x = 0; x < 3; ++x) {
            const double ge = (gq[x][4] - e * gq[x][0]) * ir;
            double vgv = 0.0;
            for (int j = 0; j < 3; ++j) vgv += v[j] * ((gq[x][1 + j] - v[j] * gq[x][0]) * ir);
            F[x][4] -= kappa * ((ge - vgv) / cv);
        }
    }
}

// Largest viscous eigenvalue max(4 mu / (3 rho), kappa / (cv rho)): the second
// is gamma mu / (Pr rho) with Pr = mu gamma cv / kappa.
__device__ inline double visc_eig(double mu, double kappa, double cv, double rho) {
    return fmax(4.0 * mu / (3.0 * rho), kappa / (cv * rho));
}

__device__ inline double pressure5(const double q[5], double gamma) {
    return (gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// ------------------------------------------------------------------ set-up

// M_i = sum_k |J_k| P_k^T M^ P_k, written densely into the M^{-1} slot.
// Sub-tets are added one after the other; the nodes of one sub-tet map to
// distinct DOFs, so the threads of one addition never collide.
template <int N>
__global__ void __launch_bounds__(256) k_mass_assemble(DevGrid g) {
    constexpr int np = Dim<N>::np;
    const int c = blockIdx.x;
    const int64_t n = g.dof_ptr[c + 1] - g.dof_ptr[c];
    const int64_t ld = minv_ld(n);
    double *M = g.minv + g.minv_ptr[c];
    for (int64_t e = threadIdx.x; e < n * ld; e += blockDim.x) M[e] = 0.0;
    __syncthreads();
    for (int64_t k = g.sub_ptr[c]; k < g.sub_ptr[c + 1]; ++k) {
        const double dj = g.geo[k * 10 + 9];
        for (int t = threadIdx.x; t < np * np; t += blockDim.x) {
            const int m = t / np, p = t % np;
            const int64_t i = g.conn[k * np + m], j = g.conn[k * np + p];
            M[i * ld + j] += dj * g.ref->M[m * np + p];
        }
        __syncthreads();
    }
}

// In-place inverse of M_i: Jacobi scaling to unit diagonal, blocked
// Gauss-Jordan elimination without pivoting (the scaled matrix is symmetric
// positive definite), unscaling, symmetrisation.  Pivots are taken kPanel at
// a time: with K the panel's rows/columns and O the others, one panel step is
//   A_KK <- A_KK^{-1},  A_KO <- A_KK^{-1} A_KO,
//   A_OK <- -A_OK A_KK^{-1},  A_OO <- A_OO - A_OK A_KK^{-1} A_KO,
// which equals kPanel single-pivot Gauss-Jordan steps.  The pivot block is
// inverted in LDS; each thread owns matrix columns, holds the column's new
// panel entries in registers and applies the rank-kPanel update to the other
// rows, whose panel entries are staged through LDS 64 rows at a time.
constexpr int kPanel = 32;
constexpr int kRowChunk = 64;
constexpr int kInvThreads = 512;

__global__ void __launch_bounds__(kInvThreads) k_mass_invert(DevGrid g) {
    __shared__ double P[kPanel][kPanel + 1];
    __shared__ double Rs[kRowChunk][kPanel];
    extern __shared__ double dsc[];
    const int c = blockIdx.x;
    const int n = int(g.dof_ptr[c + 1] - g.dof_ptr[c]);
    double *A = g.minv + g.minv_ptr[c];
    const int64_t ld = minv_ld(n);
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int i = tid; i < n; i += nth) {
        dsc[i] = 1.0 / sqrt(A[int64_t(i) * ld + i]);
        g.dscale[g.dof_ptr[c] + i] = dsc[i];
    }
    __syncthreads();
    for (int64_t e = tid; e < int64_t(n) * n; e += nth) {
        const int i = int(e / n), j = int(e % n);
        A[int64_t(i) * ld + j] *= dsc[i] * dsc[j];
    }
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int b = min(kPanel, n - k0);
        // pivot block inverse (single-pivot Gauss-Jordan in LDS); thread tid
        // owns entries tid + q * nth of the kPanel x kPanel block
        constexpr int kPer = (kPanel * kPanel + kInvThreads - 1) / kInvThreads;
        for (int q = 0; q < kPer; ++q) {
            const int t = tid + q * nth, pi = t / kPanel, pj = t % kPanel;
            if (t < kPanel * kPanel && pi < b && pj < b) P[pi][pj] = A[int64_t(k0 + pi) * ld + k0 + pj];
        }
        __syncthreads();
        for (int p = 0; p < b; ++p) {
            const double ip = 1.0 / P[p][p];
            double nv[kPer];
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int t = tid + q * nth, pi = t / kPanel, pj = t % kPanel;
                nv[q] = 0.0;
                if (t < kPanel * kPanel && pi < b && pj < b) {
                    const double rowp = (pj == p ? 1.0 : P[p][pj]) * ip;
                    nv[q] = pi == p ? rowp : (pj == p ? 0.0 : P[pi][pj]) - P[pi][p] * rowp;
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int t = tid + q * nth, pi = t / kPanel, pj = t % kPanel;
                if (t < kPanel * kPanel && pi < b && pj < b) P[pi][pj] = nv[q];
            }
            __syncthreads();
        }
        // columns owned by this thread: new panel entries T[:, j].  With more
        // columns than threads, the group holding the panel columns goes last:
        // the other groups' updates read the panel columns' old entries.
        const int ngroups = (n + nth - 1) / nth, gK = k0 / nth;
        for (int q = 0; q < ngroups; ++q) {
            const int j0 = ((gK + 1 + q) % ngroups) * nth;
            const int j = j0 + tid;
            const bool own = j < n;
            const bool inK = j >= k0 && j < k0 + b;
            double T[kPanel];
#pragma unroll
            for (int k = 0; k < kPanel; ++k) T[k] = 0.0;
            if (own) {
                if (inK) {
#pragma unroll
                    for (int k = 0; k < kPanel; ++k) T[k] = k < b ? P[k][j - k0] : 0.0;
                } else {
                    for (int m = 0; m < b; ++m) {
                        const double am = A[int64_t(k0 + m) * ld + j];
#pragma unroll
                        for (int k = 0; k < kPanel; ++k) T[k] = fma(k < b ? P[k][m] : 0.0, am, T[k]);
                    }
                }
            }
            // rank-b update of the other rows, 64 rows at a time
            for (int r0 = 0; r0 < n; r0 += kRowChunk) {
                const int rn = min(kRowChunk, n - r0);
                __syncthreads();
                for (int t = tid; t < rn * kPanel; t += nth) {
                    const int r = t / kPanel, k = t % kPanel;
                    Rs[r][k] = k < b ? A[int64_t(r0 + r) * ld + k0 + k] : 0.0;
                }
                __syncthreads();
                if (own) {
                    for (int r = 0; r < rn; ++r) {
                        const int i = r0 + r;
                        if (i >= k0 && i < k0 + b) continue;
                        double acc = inK ? 0.0 : A[int64_t(i) * ld + j];
#pragma unroll
                        for (int k = 0; k < kPanel; ++k) acc = fma(-Rs[r][k], T[k], acc);
                        A[int64_t(i) * ld + j] = acc;
                    }
                }
            }
            __syncthreads();
            // the panel rows take their new entries last (the update read their old ones)
            if (own) {
#pragma unroll
                for (int k = 0; k < kPanel; ++k)
                    if (k < b) A[int64_t(k0 + k) * ld + j] = T[k];
            }
            __syncthreads();
        }
    }
    for (int64_t e = tid; e < int64_t(n) * n; e += nth) {
        const int i = int(e / n), j = int(e % n);
        if (j < i) continue;
        const double v = 0.5 * (A[int64_t(i) * ld + j] + A[int64_t(j) * ld + i]) * dsc[i] * dsc[j];
        A[int64_t(i) * ld + j] = v;
        A[int64_t(j) * ld + i] = v;
    }
}

// FP32 copy of the Jacobi-scaled inverse: M_i^{-1} = D A D with D = diag(M_i)^{-1/2};
// A (entries O(1), condition ~17) is stored in FP32, D stays FP64.
__device__ __host__ inline int64_t minv32_ld(int64_t n) { return (n + 31) & ~int64_t(31); }

__global__ void __launch_bounds__(256) k_minv_to_f32(DevGrid g) {
    const int c = blockIdx.x;
    const int64_t d0 = g.dof_ptr[c];
    const int64_t n = g.dof_ptr[c + 1] - d0;
    const int64_t ld = minv_ld(n), ld32 = minv32_ld(n);
    const double *A = g.minv + g.minv_ptr[c];
    float *B = g.minv32 + g.minv32_ptr[c];
    for (int64_t e = threadIdx.x; e < n * ld32; e += blockDim.x) {
        const int64_t i = e / ld32, j = e % ld32;
        B[e] = j < n ? float(A[i * ld + j] / (g.dscale[d0 + i] * g.dscale[d0 + j])) : 0.0f;
    }
}

__global__ void k_prim_to_cons(int64_t ndof, double gamma, const double *prim, double *u) {
    const int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (l >= ndof) return;
    const double r = prim[l], a = prim[ndof + l], b = prim[2 * ndof + l], c = prim[3 * ndof + l],
                 p = prim[4 * ndof + l];
    u[l] = r;
    u[ndof + l] = r * a;
    u[2 * ndof + l] = r * b;
    u[3 * ndof + l] = r * c;
    u[4 * ndof + l] = p / (gamma - 1.0) + 0.5 * r * (a * a + b * b + c * c);
}

// ------------------------------------------------------- detector and CFL

// One wave per cell (Sec. 4.5): velocity-jump divergence over the boundary
// sub-triangles, minimum sound speed over their nodes on both sides, the
// flattener beta_i and the cell viscosity mu_i; then the cell's contribution
// max(|v| + c + 2 (4 mu_i / (3 rho)) (2N+1) / h_i) to the time step.
template <int N>
__global__ void __launch_bounds__(256) k_detect(DevGrid g, DevWork w, const double *__restrict__ u) {
    constexpr int np = Dim<N>::np, nf = Dim<N>::nf;
    const int lane = threadIdx.x % kWave;
    const int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= g.n_cells) return;
    const int64_t nd = g.ndof;
    const int64_t s0 = g.sub_ptr[c], s1 = g.sub_ptr[c + 1], d0 = g.dof_ptr[c];
    const int64_t n = g.dof_ptr[c + 1] - d0;
    const double gam = g.gamma;
    double jsum = 0.0, cmin = DBL_MAX;
    for (int64_t e = lane; e < (s1 - s0) * nf; e += kWave) {
        const int64_t k = s0 + e / nf;
        const int j = int(e % nf);
        const int64_t li = d0 + g.conn[k * np + g.ref->fn[j]];
        const int64_t kn = g.nbr_sub[k];
        double qi[5], qo[5];
        for (int v = 0; v < 5; ++v) qi[v] = u[v * nd + li];
        if (kn < 0) {
            // boundary triangle of a bounded mesh: no jump, inside sound speed only
            cmin = fmin(cmin, sqrt(gam * pressure5(qi, gam) / qi[0]));
            continue;
        }
        const int jn = g.perm[k * nf + j];
        const int64_t lo = g.dof_ptr[g.sub_cell[kn]] + g.conn[kn * np + g.ref->fn[jn]];
        for (int v = 0; v < 5; ++v) qo[v] = u[v * nd + lo];
        const double *T = g.tri + k * 4;
        const double jn_ = (qo[1] / qo[0] - qi[1] / qi[0]) * T[1] + (qo[2] / qo[0] - qi[2] / qi[0]) * T[2] +
                           (qo[3] / qo[0] - qi[3] / qi[0]) * T[3];
        jsum += T[0] * g.ref->zsum[j] * jn_;
        cmin = fmin(cmin, fmin(sqrt(gam * pressure5(qi, gam) / qi[0]), sqrt(gam * pressure5(qo, gam) / qo[0])));
    }
    double lam = 0.0, rsum = 0.0;
    for (int64_t l = lane; l < n; l += kWave) {
        double q[5];
        for (int v = 0; v < 5; ++v) q[v] = u[v * nd + d0 + l];
        const double vv = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
        lam = fmax(lam, vv + sqrt(gam * pressure5(q, gam) / q[0]));
        rsum += g.mrow[d0 + l] * q[0];
    }
    jsum = wave_sum(jsum);
    cmin = wave_min(cmin);
    lam = wave_max(lam);
    rsum = wave_sum(rsum);
    const double h = g.h[c], vol = g.vol[c], m1 = g.m1;
    const double div = jsum / vol;
    const double beta = fmin(1.0, fmax(0.0, -(h * div + m1 * cmin) / (m1 * cmin)));
    const double mu_c = g.av ? g.mu + beta * (rsum / vol) * lam * h / double(2 * N + 1) : g.mu;
    double ct = 0.0;
    for (int64_t l = lane; l < n; l += kWave) {
        double q[5];
        for (int v = 0; v < 5; ++v) q[v] = u[v * nd + d0 + l];
        const double vv = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
        const double lv = visc_eig(mu_c, g.kappa, g.cv, q[0]);
        ct = fmax(ct, vv + sqrt(gam * pressure5(q, gam) / q[0]) + 2.0 * lv * double(2 * N + 1) / h);
    }
    ct = wave_max(ct);
    if (lane == 0) {
        w.mu_cell[c] = mu_c;
        w.beta[c] = g.av ? beta : 0.0;
        w.cflterm[c] = ct;
        if (g.av && beta > 0.0) atomicAdd(&w.status[3], 1);
    }
}

// Largest cell term s_max into *smax and, for cfl > 0, the time step
// dt = cfl h_min / ((2N+1) s_max) into *w.dt; a non-finite or non-positive
// s_max gives dt = 0 and the non-finite status.  NaN terms propagate.
__global__ void __launch_bounds__(1024) k_cfl_dt(int n, DevWork w, double *smax, double cfl, double h_min, int n21) {
    __shared__ double red[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double t = w.cflterm[i];
        m = (t != t || m != m) ? t + m : fmax(m, t);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o, kWave);
        m = (t != t || m != m) ? t + m : fmax(m, t);
    }
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < int(blockDim.x) / kWave; ++i) v = (red[i] != red[i] || v != v) ? red[i] + v : fmax(v, red[i]);
        smax[0] = v;
        if (cfl > 0.0) {
            const bool ok = v > 0.0 && isfinite(v);
            w.dt[0] = ok ? cfl * h_min / (double(n21) * v) : 0.0;
            if (!ok) atomicOr(&w.status[0], kStatusNonfinite);
        }
    }
}

// ------------------------------------------------------------- predictor
//
// The iteration kernels run over a list of (slot, cell) entries that may mix
// cells of several simulations of one degree and precision (a slot is one
// simulation's DevGrid and DevWork in a device table).  Each kernel is a
// grid-stride loop over work items, so one launch shape serves every list
// length: a persistent grid of a fixed number of workgroups, or one
// workgroup per item.  Logical block L (xcd_block) takes items L, L + G, ...,
// so the consecutive items of one cell run on one XCD and share its L2.

// Pointers read from the slot table are generic; the M^{-1} kernels restate
// them in the global address space (the streamed matrix) and in the constant
// address space (the right-hand side, read-only during the kernel and
// wave-uniform, so it is fetched with scalar loads).
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

// Wave-uniform copies (the value of lane 0) of values that are uniform but
// that the compiler cannot prove so.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32))));
    return int64_t((uint64_t(hi) << 32) | lo);
}
template <typename T>
__device__ inline T *uni_ptr(T *p) {
    return reinterpret_cast<T *>(uni64(reinterpret_cast<int64_t>(p)));
}

__device__ inline void decode(int32_t e, int &slot, int &c) {
    slot = e >> kSlotShift;
    c = e & (kMaxCellsPerSlot - 1);
}

// Lagrange basis on the nt time nodes at t.
template <int NT>
__device__ inline void time_lagrange(const double *tau, double t, double L[NT]) {
    for (int a = 0; a < NT; ++a) {
        double v = 1.0;
        for (int c = 0; c < NT; ++c)
            if (c != a) v *= (t - tau[c]) / (tau[a] - tau[c]);
        L[a] = v;
    }
}

// Start of the predictor iteration.  From u^n: one thread per element of the
// DOF-major iterate (consecutive threads write consecutive elements).  From
// the previous step's converged predictor q' (still in x): one thread per
// (DOF, variable), q(tau_b) = u^n + sum_a (L_a(1 + r tau_b) - L_a(1)) q'(tau_a)
// with r = dt / dt', the polynomial continued past the old step and shifted
// to the new initial data; cells with a troubled flag start from u^n.  The
// first n_cells threads also reset the cell's counters and list entry.
template <int N>
__global__ void k_pred_init(DevGrid g, DevWork w, int slot, int32_t *list, int64_t base) {
    constexpr int nc = Dim<N>::nc, nt = Dim<N>::nt;
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const bool guess = g.guess && *w.guess_ok != 0;
    if (!guess) {
        if (t < g.ndof * nc) {
            const int64_t l = t / nc;
            w.x[t] = w.u[(t % nc) % 5 * g.ndof + l];
        }
    } else if (t < g.ndof * 5) {
        const int64_t l = t / 5;
        const int v = int(t % 5);
        const double un = w.u[v * g.ndof + l];
        double *xl = w.x + l * nc + v;
        if (w.beta[g.dof_cell[l]] > 0.0) {
            for (int b = 0; b < nt; ++b) xl[b * 5] = un;
        } else {
            const double r = *w.dt / *w.dt_prev;
            double L1[nt], qp[nt];
            time_lagrange<nt>(g.ref->tau, 1.0, L1);
            for (int a = 0; a < nt; ++a) qp[a] = xl[a * 5];
            for (int b = 0; b < nt; ++b) {
                double Lb[nt];
                time_lagrange<nt>(g.ref->tau, 1.0 + r * g.ref->tau[b], Lb);
                double acc = un;
                for (int a = 0; a < nt; ++a) acc += (Lb[a] - L1[a]) * qp[a];
                xl[b * 5] = acc;
            }
        }
    }
    if (g.mixed && t < g.ndof * 5) w.un5[t] = w.u[(t % 5) * g.ndof + t / 5];  // u^n DOF-major
    const int64_t l = t;
    if (l < g.n_cells) {
        list[base + l] = (slot << kSlotShift) | int32_t(l);
        w.iters[l] = 0;
        w.late[l] = 2;
        w.late2[l] = 1;
        w.pool_slot[l] = -1;
        w.hist[2 * l] = 0;
        w.hist[2 * l + 1] = 0;
    }
}

__global__ void k_clear_late(DevGrid g, DevWork w) {
    const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (c < g.n_cells) w.late[c] = 0;
}

__global__ void k_relabel_late(DevGrid g, DevWork w) {
    const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (c < g.n_cells && w.late[c] == 2) w.late[c] = 1;
}

__global__ void k_mark_listed(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list, int count,
                              int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int slot, c;
    decode(list[i], slot, c);
    tab[slot].w.late[c] = value;
}

__global__ void k_clear_late2(DevGrid g, DevWork w) {
    const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (c < g.n_cells) w.late2[c] = 0;
}

// One block per listed entry: the cell and, across each of its sub-tets'
// boundary triangles, the neighbouring cell (stores of the same value).
__global__ void __launch_bounds__(256) k_mark_late2(const DevSlot *__restrict__ tab,
                                                    const int32_t *__restrict__ list, int count) {
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        int slot, c;
        decode(list[i], slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        if (threadIdx.x == 0) w.late2[c] = 1;
        for (int64_t k = g.sub_ptr[c] + threadIdx.x; k < g.sub_ptr[c + 1]; k += blockDim.x)
            if (g.nbr_sub[k] >= 0) w.late2[g.sub_cell[g.nbr_sub[k]]] = 1;
    }
}

__global__ void k_set_int(int32_t *p, int v) {
    if (threadIdx.x == 0) p[0] = v;
}

__global__ void k_set_double(double *p, double v) {
    if (threadIdx.x == 0) p[0] = v;
}

// Nodal flux of the Navier-Stokes equations at node m of a sub-tet for one
// time node (gradient from the reference derivatives when mu_c != 0) and its
// contravariant form f*_d = dt sum_x G[d][x] F_x (eq:modified_fluxes).  Dt
// holds D^ transposed, D^_d[m][p] at Dt[(d np + p) np + m], so that the lanes
// of one sub-tet (consecutive m) read consecutive LDS words.
template <int N, int VISC>
__device__ inline void node_flux(const double *Dt, const double (*qn)[5], int m, const double G[9], const double q[5],
                                 double gamma, double mu_c, double kappa, double cv, double dt, double *fstar,
                                 double F[3][5]) {
    constexpr int np = Dim<N>::np;
    double gq[3][5] = {};
    if (VISC == 0) mu_c = 0.0;  // inviscid group: no cell viscosity
    if (VISC < 2) kappa = 0.0;  // no heat conduction below level 2
    if (VISC > 0 && (mu_c != 0.0 || kappa != 0.0)) {
        double rg[3][5] = {};
        for (int d = 0; d < 3; ++d)
            for (int p = 0; p < np; ++p) {
                const double dd = Dt[(d * np + p) * np + m];
                for (int v = 0; v < 5; ++v) rg[d][v] += dd * qn[p][v];
            }
        for (int x = 0; x < 3; ++x)
            for (int v = 0; v < 5; ++v) gq[x][v] = G[0 * 3 + x] * rg[0][v] + G[1 * 3 + x] * rg[1][v] + G[2 * 3 + x] * rg[2][v];
    }
    ns_flux<VISC == 2>(q, gq, gamma, mu_c, kappa, cv, F);
    for (int d = 0; d < 3; ++d)
        for (int v = 0; v < 5; ++v)
            fstar[d * 5 + v] = dt * (G[d * 3 + 0] * F[0][v] + G[d * 3 + 1] * F[1][v] + G[d * 3 + 2] * F[2][v]);
}

// Operand layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16x4, B 4x16, D
// 16x16, one double of A and of B and four of D per lane): A[i][k] in lane
// i + 16 k (the host writes DevRef::Kfrag in this order), B[k][j] in lane
// j + 16 k, D[i][j] in lane j + 16 (i % 4), item i / 4.
__device__ inline int mf_b_k(int l) { return l / 16; }
__device__ inline int mf_b_col(int l) { return l % 16; }
__device__ inline int mf_d_row(int l, int r) { return l / 16 + 4 * r; }
__device__ inline int mf_d_col(int l, int) { return l % 16; }
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Column of element (row, col) of an LDS B operand: the low 4 bits of the
// column are XORed with the row's, and (PAIR, rows of 32 k doubles) odd rows
// swap neighbouring 16-column tiles.  Writes down a column (one row per
// lane) then fall in distinct banks, and with PAIR the MFMA read of 4 rows x
// 16 columns spreads over both halves of the banks.
template <bool PAIR>
__device__ inline int lds_swz(int row, int col) { return col ^ (row & 15) ^ (PAIR ? ((row & 1) << 4) : 0); }
// B-operand row length for ct column tiles: whole tile pairs when there are two or more
__host__ __device__ constexpr int lds_ld(int ct) { return ct >= 2 ? 32 * ((ct + 1) / 2) : 16 * ct; }

// Shape of the chunk's stiffness contraction as one matrix product:
// rows = node m, inner index = (d, p), columns = (sub-tet, time node, variable);
// in mixed precision a fourth inner block d = 3 carries the mass term.
template <int N, bool MIXED = false>
struct Contraction {
    static constexpr int np = Dim<N>::np;
    static constexpr int inner = (MIXED ? 4 : 3) * np;
    static constexpr int ks = (inner + 3) / 4;  // k-steps of 4
    static constexpr int cols = Dim<N>::spb * Dim<N>::nt * 5;
    static constexpr int ct = (cols + 15) / 16;  // column tiles
    static constexpr int mt = (np + 15) / 16;    // row tiles
    static constexpr int ld = lds_ld(ct);        // row stride of the B operand in LDS
    static constexpr bool pair = ct >= 2;        // lds_swz variant
};

// Work item = (entry, chunk of spb sub-tets of the cell), 256 threads.  Per
// sub-tet and time node (one thread each): the nodal flux f*; then the
// reference stiffness contraction rk[a][m] = w_a |J| sum_d sum_p K^_d[m][p]
// f*_d[a][p] (eq:ader4) of the whole chunk as one product on the matrix
// cores, K^ (rows m, inner (d, p)) times f* (inner (d, p), columns (sub-tet,
// a, v)), wave w taking column tiles w, w + 4, ...  In mixed precision the
// sub-tet's part of (K_tau (x) M_i)(q - 1 (x) u^n) is added, which makes rk
// the unpreconditioned residual of eq:ADER-localCauchy: it enters the same
// product as a fourth inner block, M^ (rows m, inner p) times
// g_a[p][v] = (1 / w_a) sum_b K_tau[a][b] (q_b - u^n)[p][v].  Block 0 clears
// the next list's length.  VISC: 0 inviscid group, 1 some simulation of the
// group has a physical or artificial viscosity, 2 some has heat conduction as
// well (the temperature gradient enters the energy flux); MIXED: the group's
// precision.
template <int N, int VISC, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_round_subtet(const DevSlot *__restrict__ tab,
                                                                   const int32_t *__restrict__ list,
                                                                   const int32_t *__restrict__ count, int chunks,
                                                                   int32_t *next_count) {
    using C = Contraction<N, MIXED>;
    constexpr int np = Dim<N>::np, nt = Dim<N>::nt, nc = Dim<N>::nc, npt = Dim<N>::npt, spb = Dim<N>::spb;
    constexpr bool QS = VISC;  // nodal states shared through LDS (the viscous gradient)
    constexpr int nd = VISC ? 3 * np * np : 1;
    constexpr int qsp = QS ? spb : 1, qnt = QS ? nt : 1, qnp = QS ? np : 1;
    __shared__ double fT[4 * C::ks][C::ld];  // B operand: f*_d[s][a][p][v] at (d np + p, (s nt + a) 5 + v); g at d = 3
    __shared__ double Dt[nd];                // D^ transposed, as node_flux reads it
    __shared__ double qs[qsp][qnt][qnp][5];  // nodal states
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int s = tid / npt, a = (tid / np) % nt, m = tid % np;
    const bool node = s < spb;
    const int n_items = *count * chunks;
    bool loaded = false;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(list[item / chunks], slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        const int64_t s0 = g.sub_ptr[c], s1 = g.sub_ptr[c + 1];
        const int nchunk = int((s1 - s0 + spb - 1) / spb);
        const int chunk = item % chunks;
        if (chunk >= nchunk) continue;
        if (!loaded) {
            // the same for every item of the block: the padding of the
            // operands stays zero, the inner index beyond 3 np included
            for (int t = tid; t < 4 * C::ks * C::ld; t += blockDim.x) fT[t / C::ld][t % C::ld] = 0.0;
            if (VISC)
                for (int t = tid; t < 3 * np * np; t += blockDim.x) {
                    const int d = t / (np * np), mm = (t / np) % np, p = t % np;
                    Dt[VISC ? (d * np + p) * np + mm : 0] = g.ref->D[t];
                }
            loaded = true;
            __syncthreads();
        }
        const int64_t k = s0 + int64_t(chunk) * spb + s;
        const bool valid = node && (k < s1);
        const double dt = *w.dt;
        double G[9], mu_c = 0.0;
        double q[5] = {1, 0, 0, 0, 1};
        int64_t l = 0;
        if (valid) {
            // every load of the item is issued here, through global-address
            // pointers: generic loads after the LDS writes below would each
            // wait for those writes and for one another
            const gptr<double> geo = (gptr<double>)(g.geo + k * 10);
            for (int i = 0; i < 9; ++i) G[i] = geo[i];
            mu_c = w.mu_cell[c];
            l = g.dof_ptr[c] + g.conn[k * np + m];
            if (MIXED) {
                // g_a at node m: the mass term's inner block, from the node's
                // row of the iterate (all time nodes) and the DOF-major u^n
                double xr[nt * 5], ur[5], kt[nt];
                const gptr<double> xg = (gptr<double>)(w.x + l * nc);
                const gptr<double> ug = (gptr<double>)(w.un5 + l * 5);
                const gptr<double> kg = (gptr<double>)(g.ref->Ktau + a * nt);
                for (int i = 0; i < nt * 5; ++i) xr[i] = xg[i];
                for (int v = 0; v < 5; ++v) ur[v] = ug[v];
                for (int b = 0; b < nt; ++b) kt[b] = kg[b];
                const double rw = 1.0 / ((gptr<double>)g.ref->w)[a];
                for (int v = 0; v < 5; ++v) q[v] = xg[a * 5 + v];  // not xr[]: a is per thread
                for (int v = 0; v < 5; ++v) {
                    const double un = ur[v];
                    double acc = 0.0;
                    for (int b = 0; b < nt; ++b) acc += kt[b] * (xr[b * 5 + v] - un);
                    fT[3 * np + m][lds_swz<C::pair>(3 * np + m, (s * nt + a) * 5 + v)] = rw * acc;
                }
            } else {
                const gptr<double> xg = (gptr<double>)(w.x + l * nc + a * 5);
                for (int v = 0; v < 5; ++v) q[v] = xg[v];
            }
            if (QS)
                for (int v = 0; v < 5; ++v) qs[QS ? s : 0][QS ? a : 0][QS ? m : 0][v] = q[v];
        }
        if (QS) __syncthreads();
        if (valid) {
            double F[3][5], fst[15];
            node_flux<N, VISC>(Dt, qs[QS ? s : 0][QS ? a : 0], m, G, q, g.gamma, mu_c, g.kappa, g.cv, dt, fst, F);
            for (int d = 0; d < 3; ++d)
                for (int v = 0; v < 5; ++v) fT[d * np + m][lds_swz<C::pair>(d * np + m, (s * nt + a) * 5 + v)] = fst[d * 5 + v];
        }
        __syncthreads();
        const gptr<double> Kf = (gptr<double>)uni_ptr(MIXED ? g.ref->KMfrag : g.ref->Kfrag) + lane;
        for (int ctile = wv; ctile < C::ct; ctile += 4) {
            // a lane's D column is the same for all its outputs: one factor
            // w_a |J| per lane, loaded before the products
            const int col = 16 * ctile + mf_d_col(lane, 0);
            const int ss = col / (nt * 5), aa = (col / 5) % nt, vv = col % 5;
            const int64_t kk = s0 + int64_t(chunk) * spb + ss;
            const bool colok = col < C::cols && kk < s1;
            const double fac = colok ? ((gptr<double>)g.ref->w)[aa] * ((gptr<double>)g.geo)[kk * 10 + 9] : 0.0;
            dbl4 acc[C::mt];
#pragma unroll
            for (int mtile = 0; mtile < C::mt; ++mtile) acc[mtile] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kst = 0; kst < C::ks; ++kst) {
                const int br = 4 * kst + mf_b_k(lane);
                const double bv = fT[br][lds_swz<C::pair>(br, 16 * ctile + mf_b_col(lane))];
#pragma unroll
                for (int mtile = 0; mtile < C::mt; ++mtile)
                    acc[mtile] = __builtin_amdgcn_mfma_f64_16x16x4f64(Kf[(mtile * C::ks + kst) * kWave], bv, acc[mtile], 0,
                                                                      0, 0);
            }
            if (colok) {
                double *out = w.rk + kk * np * nc + aa * 5 + vv;
#pragma unroll
                for (int mtile = 0; mtile < C::mt; ++mtile)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * mtile + mf_d_row(lane, r);
                        if (row < np) out[row * nc] = fac * acc[mtile][r];
                    }
            }
        }
        __syncthreads();  // LDS is rewritten by the next item
    }
}

// Sum of p[idx[q] * stride + col] over q in [q0, q1), added in ascending q
// (the order fixes the rounding); index and value loads are issued kGatherBatch
// at a time, so a long incidence list costs few dependent round trips.
constexpr int kGatherBatch = 16;
__device__ inline double ordered_gather_sum(const double *__restrict__ p, const int32_t *__restrict__ idx, int q0,
                                            int q1, int stride, int col) {
    const gptr<double> pg = (gptr<double>)p;
    const gptr<int32_t> ig = (gptr<int32_t>)idx;
    double acc = 0.0;
    for (int q = q0; q < q1; q += kGatherBatch) {
        // index loads without a branch each (past the end the last entry is
        // read again), so that they are in flight together
        int32_t ix[kGatherBatch];
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) ix[u] = ig[min(q + u, q1 - 1)];
        double v[kGatherBatch];
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) v[u] = q + u < q1 ? pg[int64_t(ix[u]) * stride + col] : 0.0;
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u)
            if (q + u < q1) acc += v[u];
    }
    return acc;
}

// Assembly R[l][col] = sum over the DOF's ascending incidence list of the
// sub-tet contributions rk (mixed: the FP32 scaled residual D R); work item
// = (entry, 256 consecutive elements of the cell's DOF-major block).
template <int N>
__global__ void __launch_bounds__(256) k_round_gather(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ count, int per) {
    constexpr int nc = Dim<N>::nc;
    const int n_items = *count * per;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(list[item / per], slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        const int64_t d0 = g.dof_ptr[c];
        const int64_t e = int64_t(item % per) * blockDim.x + threadIdx.x;
        if (e >= (g.dof_ptr[c + 1] - d0) * nc) continue;
        const int64_t t = d0 * nc + e;
        const int64_t l = t / nc;
        const int col = int(t % nc);
        const double acc = ordered_gather_sum(w.rk, g.inc_idx, g.inc_ptr[l], g.inc_ptr[l + 1], nc, col);
        if (g.mixed)
            w.R32[t] = float(acc * g.dscale[l]);
        else
            w.R[t] = acc;
    }
}

// Time integrals of the converged predictor, all sub-tets of one simulation:
// the volume term |J| sum_d V^_d F*bar_d (Sec. 4.4) and the face traces
// (qbar, Fbar) at the boundary-triangle nodes.
template <int N, int VISC>
__global__ void __launch_bounds__(Dim<N>::threads) k_subtet_post(DevGrid g, DevWork w, int which) {
    constexpr int np = Dim<N>::np, nt = Dim<N>::nt, nc = Dim<N>::nc, npt = Dim<N>::npt, spb = Dim<N>::spb;
    constexpr int nf = Dim<N>::nf;
    // the volume term as one product on the matrix cores: rows m, inner
    // (d, p), columns (sub-tet, variable)
    constexpr int inner = 3 * np, ks = (inner + 3) / 4, cols = spb * 5, ct = (cols + 15) / 16;
    constexpr int ld = lds_ld(ct);
    constexpr bool pair = ct >= 2;
    constexpr int mt = (np + 15) / 16;
    static_assert(kWave * (ct < 4 ? ct : 4) <= Dim<N>::threads, "every wave that takes a column tile is full");
    __shared__ double Dt[VISC ? 3 * np * np : 1];  // D^ transposed, as node_flux reads it
    __shared__ double qs[spb][nt][np][5];
    __shared__ double fs[spb][nt][np][15];  // f*, then (once fbar is formed) the physical fluxes F
    __shared__ double fbT[4 * ks][ld];      // B operand: Fbar*_d[s][p][v] at (d np + p, s 5 + v)
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int s = tid / npt, a = (tid / np) % nt, m = tid % np;
    const int64_t k = int64_t(blockIdx.x) * spb + s;
    const int c = (s < spb) && (k < g.nsub) ? g.sub_cell[k] : -1;
    const bool valid = c >= 0 && w.late[c] == which;
    // the later passes have few cells: blocks without one leave before loading anything
    if (!__syncthreads_or(valid)) return;
    for (int t = tid; t < 4 * ks * ld; t += blockDim.x) fbT[t / ld][t % ld] = 0.0;  // padding stays zero
    if (VISC)
        for (int t = tid; t < 3 * np * np; t += blockDim.x) {
            const int d = t / (np * np), mm = (t / np) % np, p = t % np;
            Dt[VISC ? (d * np + p) * np + mm : 0] = g.ref->D[t];
        }
    const double dt = *w.dt;
    double G[9], dj = 0.0, mu_c = 0.0;
    double q[5] = {1, 0, 0, 0, 1};
    if (valid) {
        for (int i = 0; i < 9; ++i) G[i] = g.geo[k * 10 + i];
        dj = g.geo[k * 10 + 9];
        mu_c = w.mu_cell[c];
        const int64_t l = g.dof_ptr[c] + g.conn[k * np + m];
        for (int v = 0; v < 5; ++v) {
            q[v] = w.x[l * nc + a * 5 + v];
            qs[s][a][m][v] = q[v];
        }
    }
    __syncthreads();
    double F[3][5];
    if (valid) node_flux<N, VISC>(Dt, qs[s][a], m, G, q, g.gamma, mu_c, g.kappa, g.cv, dt, fs[s][a][m], F);
    __syncthreads();
    // time averages Fbar*_{d}[m][v] = sum_b w_b f*_d[b][m][v], the 15 entries
    // of a node split over its nt threads
    if (valid)
        for (int i = a; i < 15; i += nt) {
            double acc = 0.0;
            for (int b = 0; b < nt; ++b) acc += g.ref->w[b] * fs[s][b][m][i];
            fbT[(i / 5) * np + m][lds_swz<pair>((i / 5) * np + m, s * 5 + i % 5)] = acc;
        }
    __syncthreads();
    if (valid)
        for (int x = 0; x < 3; ++x)
            for (int v = 0; v < 5; ++v) fs[s][a][m][x * 5 + v] = F[x][v];
    __syncthreads();
    // volume term vk[k][m][v] = |J_k| sum_d sum_p V^_d[m][p] Fbar*_d[p][v], V^_d[m][p] = K^_d[p][m]
    const int64_t k0 = int64_t(blockIdx.x) * spb;
    const gptr<double> Vf = (gptr<double>)uni_ptr(g.ref->Vfrag) + lane;
    for (int ctile = wv; ctile < ct; ctile += 4) {
        // a lane's D column (sub-tet, variable) is the same for all its
        // outputs: whether it is written, and its factor |J|, loaded before
        // the products
        const int col = 16 * ctile + mf_d_col(lane, 0);
        const int ss = col / 5, vv = col % 5;
        const int64_t kk = k0 + ss;
        bool colok = col < cols && kk < g.nsub;
        if (colok) colok = w.late[g.sub_cell[kk]] == which;
        const double fac = colok ? ((gptr<double>)g.geo)[kk * 10 + 9] : 0.0;
        dbl4 acc[mt];
#pragma unroll
        for (int mtile = 0; mtile < mt; ++mtile) acc[mtile] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kst = 0; kst < ks; ++kst) {
            const int br = 4 * kst + mf_b_k(lane);
            const double bv = fbT[br][lds_swz<pair>(br, 16 * ctile + mf_b_col(lane))];
#pragma unroll
            for (int mtile = 0; mtile < mt; ++mtile)
                acc[mtile] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vf[(mtile * ks + kst) * kWave], bv, acc[mtile], 0, 0, 0);
        }
        if (colok) {
            double *out = w.vk + kk * np * 5 + vv;
#pragma unroll
            for (int mtile = 0; mtile < mt; ++mtile)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mtile + mf_d_row(lane, r);
                    if (row < np) out[row * 5] = fac * acc[mtile][r];
                }
        }
    }
    if (!valid) return;
    if (a == 1 || nt == 1) {
        // traces at face nodes (the weights in registers: the stores below
        // could otherwise alias them and force a reload after each)
        if (m < nf) {
            const int j = m, mm = g.ref->fn[j];
            double wb[nt];
            for (int b = 0; b < nt; ++b) wb[b] = ((gptr<double>)g.ref->w)[b];
            double *out = w.trace + (k * nf + j) * 20;
            for (int v = 0; v < 5; ++v) {
                double acc = 0.0;
                for (int b = 0; b < nt; ++b) acc += wb[b] * qs[s][b][mm][v];
                out[v] = dt * acc;
            }
            for (int i = 0; i < 15; ++i) {
                double acc = 0.0;
                for (int b = 0; b < nt; ++b) acc += wb[b] * fs[s][b][mm][i];
                out[5 + i] = dt * acc;
            }
        }
    }
}

constexpr int kMinvUnroll = 8;

// Splits of the predictor's M^-1 product for cell c in its current iteration.
__device__ inline int minv_splits(const DevGrid &g, const DevWork &w, int c) {
    return (!g.mixed && w.iters[c] >= kMinvSplitAfter) ? kMinvSplitK : 1;
}

// Y = M_i^{-1} X for rows [64 tile, 64 tile + 64) of cell c; X and Y DOF-major
// with NC columns.  The 4 waves of the block split the inner index j into 4
// contiguous ranges; their partial sums are added in a fixed wave order
// through LDS (deterministic).  M_i^{-1} is symmetric, so row j of the stored
// matrix supplies column j: one j is a coalesced 512-byte load across the
// wave, and X[j][:] is wave-uniform.
// MODE 0: Y = S (predictor);  MODE 1: add Y into the SoA state u (corrector).
// Inner index range [jb, je) (the whole row, 0..n, except in a split of the
// predictor's tail iterations); the 4 waves take contiguous quarters of it.
template <int NC, int MODE>
__device__ inline void minv_tile(const DevGrid &g, int c, int tile, int jb, int je, const double *__restrict__ X,
                                 double *__restrict__ Y, unsigned long long *bytes, double (*part)[kWave]) {
    const int lane = threadIdx.x % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t d0 = uni64(g.dof_ptr[c]);
    const int n = uni(int(g.dof_ptr[c + 1] - d0));
    const int64_t ld = minv_ld(n);
    const int r0 = tile * kWave;
    if (r0 >= n) return;
    if (bytes != nullptr && threadIdx.x == 0) {
        // as stored: matrix and right-hand side once over the splits, the result once per row
        const unsigned long long rows = unsigned(min(kWave, n - r0)), w = unsigned(je - jb);
        atomicAdd(bytes + 1, 8ull * (rows * w + (jb == 0 ? rows * NC : 0u) + (tile == 0 ? w * NC : 0u)));
        // algorithmic, once per cell: the packed triangle, the right-hand side and the result
        if (tile == 0 && jb == 0) {
            const unsigned long long nn = unsigned(n);
            atomicAdd(bytes, 4ull * nn * (nn + 1) + 16ull * nn * NC);
        }
    }
    const int row = r0 + lane;
    const bool ok = row < n;
    const int rowc = ok ? row : n - 1;  // clamped: out-of-range lanes read a valid address
    const gptr<double> A = (gptr<double>)(uni_ptr(g.minv + g.minv_ptr[c]) + rowc);
    const cptr<double> B = (cptr<double>)uni_ptr(X + d0 * NC);
    const int span = uni((je - jb + 3) / 4);
    const int j0 = uni(min(je, jb + wv * span)), j1 = uni(min(je, j0 + span));
    double acc[NC];
#pragma unroll
    for (int col = 0; col < NC; ++col) acc[col] = 0.0;
    int j = j0;
    for (; j + kMinvUnroll <= j1; j += kMinvUnroll) {  // kMinvUnroll loads in flight per wave
        double m[kMinvUnroll];
#pragma unroll
        for (int u = 0; u < kMinvUnroll; ++u) m[u] = A[int64_t(j + u) * ld];
        const cptr<double> b = B + int64_t(j) * NC;
#pragma unroll
        for (int u = 0; u < kMinvUnroll; ++u)
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fma(m[u], b[u * NC + col], acc[col]);
    }
    for (; j < j1; ++j) {
        const double m0 = A[int64_t(j) * ld];
        const cptr<double> b = B + int64_t(j) * NC;
#pragma unroll
        for (int col = 0; col < NC; ++col) acc[col] = fma(m0, b[col], acc[col]);
    }
    // partial sums added wave 3, 2, 1, 0 through one LDS buffer (10 KB at
    // NC = 20, so LDS does not cap the number of resident blocks)
    for (int s = 3; s >= 1; --s) {
        if (wv == s) {
#pragma unroll
            for (int col = 0; col < NC; ++col) part[col][lane] = s == 3 ? acc[col] : part[col][lane] + acc[col];
        }
        __syncthreads();
    }
    if (wv == 0 && ok) {
#pragma unroll
        for (int col = 0; col < NC; ++col) {
            const double v = part[col][lane] + acc[col];
            if (MODE == 0)
                Y[(d0 + row) * NC + col] = v;
            else
                Y[col * g.ndof + d0 + row] += v;
        }
    }
}

// Predictor: S = M_i^{-1} R for the listed cells, work item = (entry, tile,
// split).  From iteration kMinvSplitAfter on (few cells are left, and a tile's
// time is one wave's chain of dependent loads) the inner index of an FP64
// cell is split kMinvSplitK ways over workgroups, each writing its partial
// product to Sp[split]; the Anderson kernel adds them in split order.  The
// split depends only on the cell's iteration count, so a cell's bits do not
// depend on what it is batched with.  spl = the item split factor of this
// launch, kMinvSplitK whenever some listed cell may split.
template <int NC>
__global__ void __launch_bounds__(256) k_round_minv(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ count, int tpc, int spl,
                                                    unsigned long long *bytes) {
    __shared__ double part[NC][kWave];
    const int per_entry = tpc * spl;
    const int n_items = *count * per_entry;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(uni(list[item / per_entry]), slot, c);
        const DevSlot &sl = tab[slot];
        const int rem = item % per_entry, tile = rem / spl, split = rem % spl;
        const int sk = uni(minv_splits(sl.g, sl.w, c));
        if (split >= sk) continue;
        const int n = uni(int(sl.g.dof_ptr[c + 1] - sl.g.dof_ptr[c]));
        const int per = (n + sk - 1) / sk, jb = min(n, split * per), je = min(n, jb + per);
        double *Y = sk == 1 ? sl.w.S : sl.w.Sp + int64_t(split) * sl.g.ndof * NC;
        minv_tile<NC, 0>(sl.g, c, tile, jb, je, sl.w.R, uni_ptr(Y), bytes, part);
        __syncthreads();
    }
}

// Corrector: u += M_i^{-1} rhs for every cell of one simulation, work item =
// (cell, 64-row tile); a grid smaller than the item count strides over them.
template <int NC>
__global__ void __launch_bounds__(256) k_minv_update(DevGrid g, const double *__restrict__ X, double *__restrict__ Y,
                                                     int tpc, const int32_t *__restrict__ late2, int which) {
    __shared__ double part[NC][kWave];
    const int n_items = g.n_cells * tpc;
    for (int lb = xcd_block(); lb < n_items; lb += gridDim.x) {
        const int c = lb / tpc;
        if (late2[c] != which) continue;
        minv_tile<NC, 1>(g, c, lb % tpc, 0, int(g.dof_ptr[c + 1] - g.dof_ptr[c]), X, Y, nullptr, part);
        __syncthreads();  // part is rewritten by the next item
    }
}

// Mixed precision: S = D (A32 (D R)) with the FP32 scaled inverse A32 and the
// FP32 right-hand side X32 = D R (written by the assembly); FP32
// accumulation, result scaled back to FP64.  Same tiling as minv_tile.
template <int NC>
__global__ void __launch_bounds__(256) k_round_minv32(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ count, int tpc,
                                                      unsigned long long *bytes) {
    __shared__ float part[NC][kWave];
    const int lane = threadIdx.x % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int n_items = *count * tpc;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(uni(list[item / tpc]), slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        const int tile = item % tpc;
        const int64_t d0 = uni64(g.dof_ptr[c]);
        const int n = uni(int(g.dof_ptr[c + 1] - d0));
        const int64_t ld = minv32_ld(n);
        const int r0 = tile * kWave;
        if (r0 >= n) continue;
        if (bytes != nullptr && threadIdx.x == 0) {
            // as stored: FP32 rows, FP64 result, FP32 right-hand side once
            const unsigned long long rows = unsigned(min(kWave, n - r0));
            atomicAdd(bytes + 1, 4ull * rows * unsigned(n) + 8ull * rows * NC + (tile == 0 ? 4ull * unsigned(n) * NC : 0ull));
            // algorithmic, once per cell: the packed FP32 triangle, FP32 right-hand side, FP64 result
            if (tile == 0) {
                const unsigned long long nn = unsigned(n);
                atomicAdd(bytes, 2ull * nn * (nn + 1) + 12ull * nn * NC);
            }
        }
        const int row = r0 + lane;
        const bool ok = row < n;
        const int rowc = ok ? row : n - 1;
        const gptr<float> A = (gptr<float>)(uni_ptr(g.minv32 + g.minv32_ptr[c]) + rowc);
        const cptr<float> B = (cptr<float>)uni_ptr(w.R32 + d0 * NC);
        const int span = (n + 3) / 4;
        const int j0 = min(n, wv * span), j1 = min(n, j0 + span);
        float acc[NC];
#pragma unroll
        for (int col = 0; col < NC; ++col) acc[col] = 0.0f;
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
            const float m0 = A[int64_t(j) * ld], m1 = A[int64_t(j + 1) * ld];
            const float m2 = A[int64_t(j + 2) * ld], m3 = A[int64_t(j + 3) * ld];
            const cptr<float> b = B + int64_t(j) * NC;
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fmaf(m0, b[col], acc[col]);
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fmaf(m1, b[NC + col], acc[col]);
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fmaf(m2, b[2 * NC + col], acc[col]);
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fmaf(m3, b[3 * NC + col], acc[col]);
        }
        for (; j < j1; ++j) {
            const float m0 = A[int64_t(j) * ld];
            const cptr<float> b = B + int64_t(j) * NC;
#pragma unroll
            for (int col = 0; col < NC; ++col) acc[col] = fmaf(m0, b[col], acc[col]);
        }
        for (int s = 3; s >= 1; --s) {
            if (wv == s) {
#pragma unroll
                for (int col = 0; col < NC; ++col) part[col][lane] = s == 3 ? acc[col] : part[col][lane] + acc[col];
            }
            __syncthreads();
        }
        if (wv == 0 && ok) {
            const double sc = g.dscale[d0 + row];
#pragma unroll
            for (int col = 0; col < NC; ++col) {
                const float v = part[col][lane] + acc[col];
                w.S[(d0 + row) * NC + col] = sc * double(v);
            }
        }
        __syncthreads();
    }
}

// Anderson acceleration of the predictor map (eq:ader4 after
// K_1^{-1} = K_tau^{-1} (x) M_i^{-1}): G(x) = u - (K_tau^{-1} (x) I) S with
// S = M_i^{-1} R(x), residual f = G(x) - x, and x <- G(x) - dG gamma with
// gamma = argmin |f - dF gamma|.  Three kernels per iteration:
//   k_round_dots   (item = entry, tile of 64 DOFs): G, f, the new difference
//                  pair into the ring, partial dot products of the history
//                  with the new column and with f, partial max norms;
//   k_round_solve  (one wave per entry): reduces the partials in tile order,
//                  tests convergence, extends (or rebuilds after dropping the
//                  oldest pairs) the Jacobi-scaled Cholesky factor of the
//                  Gram matrix of dF, solves for gamma, builds the next list;
//   k_round_update (item = entry, tile or chunk of 256 values):
//                  x <- G(x) - sum_j gamma_j dG_j.
// Difference pairs live in a ring of `depth` slots, logical order oldest
// first; a column adding no new direction is not appended; when the ring is
// full the 8 oldest pairs are dropped.  Depth 0 is the plain fixed-point map.
// The iteration count of a cell is w.iters[c] (iterations done so far).
constexpr int kDrop = 8;
constexpr int kPartStride = 2 * (kMaxDepth + 1) + 2;

// Column of ring slot s of cell c in a history area (dF or dG): in place for
// s < hist_small, else in the cell's pool slot.  HT is the element type of
// the history: double, or float in mixed precision (the same areas, read as
// floats).
template <typename HT>
__device__ inline HT *hist_col(const DevGrid &g, const DevWork &w, double *in_place, double *pool, int c,
                               int64_t base, int64_t len, int s) {
    HT *ip = reinterpret_cast<HT *>(in_place), *pl = reinterpret_cast<HT *>(pool);
    if (s < g.hist_small) return ip + base * g.hist_small + int64_t(s) * len;
    return pl + int64_t(w.pool_slot[c]) * g.pool_stride + int64_t(s - g.hist_small) * len;
}

// The same, with the cell's history layout read once (the pool slot of a
// cell does not change while its columns are read), so that a column's
// address is arithmetic and many columns' loads can be in flight together.
struct HistLayout {
    int small;
    int64_t ip_off, pool_off, len;
    __device__ HistLayout(const DevGrid &g, const DevWork &w, int c, int64_t base, int64_t len_)
        : small(g.hist_small), ip_off(base * g.hist_small), pool_off(int64_t(w.pool_slot[c]) * g.pool_stride),
          len(len_) {}
    template <typename HT>
    __device__ const HT *col(const double *in_place, const double *pool, int s) const {
        const HT *ip = reinterpret_cast<const HT *>(in_place), *pl = reinterpret_cast<const HT *>(pool);
        return s < small ? ip + ip_off + int64_t(s) * len : pl + pool_off + int64_t(s - small) * len;
    }
};

// history bookkeeping: (count kept, head slot) after the drop this iteration makes
__device__ inline void ring_state(const DevWork &w, int c, int &k, int &head, bool &dropped) {
    k = w.hist[2 * c];
    head = k == 0 ? 0 : w.hist[2 * c + 1];
    dropped = false;
    if (k >= w.depth && w.depth > 0) {
        const int drop = min(kDrop, k);
        head = (head + drop) % w.depth;
        k -= drop;
        dropped = true;
    }
}

// Tiles of 64 DOFs per cell in the partials buffer of a simulation.
__device__ inline int part_tiles(const DevGrid &g) { return (g.max_cell_dofs + 63) / 64; }

// History columns per pass of the dot products: kDotCols, or in the instance
// launched on short lists kDotColsWide (FP32 history) / kDotColsWide64 (FP64
// history): fewer passes, each a round trip to memory, for more registers,
// which only the short lists can afford (16 FP64 columns would take 208
// VGPRs).  Each column's sum is the same either way.
constexpr int kDotCols = 4;
constexpr int kDotColsWide = 16;
constexpr int kDotColsWide64 = 8;

template <int N, int DC, typename HT>
__device__ inline void and_dots_tile(const DevGrid &g, const DevWork &w, int c, int tile, double (*accs)[4]) {
    constexpr int nc = Dim<N>::nc, nt = Dim<N>::nt;
    constexpr int kPer = (64 * nc + 255) / 256;  // elements per thread
    const int64_t d0 = g.dof_ptr[c];
    const int n = int(g.dof_ptr[c + 1] - d0);
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int depth = w.depth;
    const bool hist_on = depth > 0 && w.iters[c] > 0;
    const int sk = minv_splits(g, w, c);
    int k = 0, head = 0;
    bool dropped = false;
    if (hist_on) ring_state(w, c, k, head, dropped);
    const int snew = hist_on ? (head + k) % depth : 0;
    const int64_t len = int64_t(n) * nc;
    const int64_t base = d0 * nc;

    const int64_t e0 = int64_t(tile) * 64 * nc;
    const int64_t e1 = min(len, e0 + int64_t(64) * nc);
    double fe[kPer], dfe[kPer];
    int64_t ie[kPer];
    double fmx = 0.0, gmx = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        ie[q] = e0 + int64_t(q) * 256 + tid;
        fe[q] = dfe[q] = 0.0;
        if (ie[q] < e1) {
            const int64_t e = ie[q];
            const int l = int(e / nc);
            const int col = int(e % nc);
            const int b = col / 5, v = col % 5;
            double sv[nt];
            if (sk == 1) {
                const double *sr = w.S + base + int64_t(l) * nc + v;
#pragma unroll
                for (int a = 0; a < nt; ++a) sv[a] = sr[a * 5];
            } else {  // split M^-1 product: its partials added in split order (all loads first)
                const double *pr = w.Sp + base + int64_t(l) * nc + v;
                const int64_t ps = g.ndof * nc;
                double pv[kMinvSplitK][nt];
#pragma unroll
                for (int q = 0; q < kMinvSplitK; ++q)
#pragma unroll
                    for (int a = 0; a < nt; ++a) pv[q][a] = pr[q * ps + a * 5];
#pragma unroll
                for (int a = 0; a < nt; ++a) {
                    double t = pv[0][a];
#pragma unroll
                    for (int q = 1; q < kMinvSplitK; ++q) t += pv[q][a];
                    sv[a] = t;
                }
            }
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < nt; ++a) acc += g.ref->Ktau_inv[b * nt + a] * sv[a];
            const double xv = w.x[base + e];
            // FP64: G = u^n - ..., mixed: G = x - ... with S from the residual
            const double gv = (g.mixed ? xv : w.u[v * g.ndof + d0 + l]) - acc;
            const double fv = gv - xv;
            fmx = fmax(fmx, fabs(fv));
            gmx = fmax(gmx, fabs(gv));
            if (hist_on) {
                // the column as stored (rounded to HT) enters the dot products too
                const HT dfn = HT(fv - w.fprev[base + e]);
                hist_col<HT>(g, w, w.dF, w.dFp, c, base, len, snew)[e] = dfn;
                hist_col<HT>(g, w, w.dG, w.dGp, c, base, len, snew)[e] = HT(gv - w.gprev[base + e]);
                dfe[q] = double(dfn);
            }
            fe[q] = fv;
            w.fprev[base + e] = fv;
            w.gprev[base + e] = gv;
        }
    }
    double *part = w.part + (int64_t(c) * part_tiles(g) + tile) * kPartStride;
    fmx = wave_max(fmx);
    gmx = wave_max(gmx);
    if (lane == 0) {
        accs[0][wv] = fmx;
        accs[1][wv] = gmx;
    }
    if (hist_on) {
        // DC history columns per pass, so that their loads are in flight together
        // Column addresses from the layout read once, and loads without a
        // branch each: past the last column, in-place slot 0 is read and its
        // value not used; past the tile's last element, its first is read and
        // d = dfe = fe = 0 adds +0 (the sums start at +0 and cannot become -0,
        // so they keep their bits).
        const HistLayout hl(g, w, c, base, len);
        const gptr<double> dFa = (gptr<double>)w.dF, dFpa = (gptr<double>)w.dFp;
        for (int j0 = 0; j0 <= k; j0 += DC) {
            double ph[DC], pb[DC];
            const HT *cols[DC];
#pragma unroll
            for (int u = 0; u < DC; ++u) {
                ph[u] = pb[u] = 0.0;
                cols[u] = uni_ptr(hl.col<HT>((const double *)dFa, (const double *)dFpa, j0 + u < k ? (head + j0 + u) % depth : 0));
            }
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const bool in = ie[q] < e1;
                const int64_t e = in ? ie[q] : e0;
                double d[DC];
#pragma unroll
                for (int u = 0; u < DC; ++u) {
                    const double h = double(((const __attribute__((address_space(1))) HT *)cols[u])[e]);
                    d[u] = (in && j0 + u < k) ? h : dfe[q];
                }
#pragma unroll
                for (int u = 0; u < DC; ++u) {
                    ph[u] = fma(d[u], dfe[q], ph[u]);
                    pb[u] = fma(d[u], fe[q], pb[u]);
                }
                // FP64 history: one element's columns in flight at a time (all of
                // them would cost the short-list instance an occupancy step)
                if (sizeof(HT) == 8) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int u = 0; u < DC; ++u) {
                const int j = j0 + u;
                if (j <= k) {
                    const double sh = wave_sum(ph[u]), sb = wave_sum(pb[u]);
                    if (lane == 0) {
                        accs[2 + j][wv] = sh;
                        accs[2 + kMaxDepth + 1 + j][wv] = sb;
                    }
                }
            }
        }
    }
    __syncthreads();
    const int nv = hist_on ? 2 * (kMaxDepth + 1) + 2 : 2;
    for (int t = tid; t < nv; t += blockDim.x) {
        const bool used = t < 2 || (t >= 2 && t < 2 + k + 1) || (t >= 2 + kMaxDepth + 1 && t < 2 + kMaxDepth + 1 + k + 1);
        if (!used) continue;
        double r = accs[t][0];
        if (t < 2) {
            r = fmax(fmax(r, accs[t][1]), fmax(accs[t][2], accs[t][3]));
        } else {
            r = ((r + accs[t][1]) + accs[t][2]) + accs[t][3];
        }
        part[t] = r;
    }
}

// One wave: w.gamma[c][0..kuse) receives the coefficients, w.kuse[c] = kuse
// and w.hist[2c + 1] the head slot of the history.  The scaled Cholesky
// factor is worked on in LDS (Ls, logical rows): loaded with independent
// loads, updated there, and its changed rows written back.  Triangular
// solves go column by column: unknown i is broadcast from lane i and every
// lane j updates its own running residual with L[j][i] (or L[i][j] for the
// transposed factor), so a step is a broadcast and a fused multiply-add
// rather than a reduction over the wave; lane i keeps 1 / L[i][i].
constexpr int kSolveBatch = 16;

__device__ inline void and_solve_cell(const DevGrid &g, const DevWork &w, int c, int32_t entry, int32_t *next,
                                      int32_t *next_count, double (*Ls)[kMaxDepth]) {
    const int lane = threadIdx.x;
    const int n = int(g.dof_ptr[c + 1] - g.dof_ptr[c]);
    const int ntile = (n + 63) / 64;
    const double *part = w.part + int64_t(c) * part_tiles(g) * kPartStride;
    const int depth = w.depth;
    const int it = w.iters[c];
    const bool hist_on = depth > 0 && it > 0;
    // reduce the per-tile partials in tile order (loads batched by kSolveBatch)
    double res = 0.0, gm = 0.0;
    for (int t0 = 0; t0 < ntile; t0 += kSolveBatch) {
        double a[kSolveBatch], b[kSolveBatch];
#pragma unroll
        for (int u = 0; u < kSolveBatch; ++u) {
            const bool in = t0 + u < ntile;
            a[u] = in ? part[(t0 + u) * kPartStride + 0] : 0.0;
            b[u] = in ? part[(t0 + u) * kPartStride + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSolveBatch; ++u) {
            res = fmax(res, a[u]);
            gm = fmax(gm, b[u]);
        }
    }
    const int it1 = it + 1;
    const bool conv = res <= w.tol * fmax(1.0, gm);
    const bool last = it1 >= w.max_iter;
    double *gam = w.gamma + int64_t(c) * kMaxDepth;
    if (lane == 0) {
        w.iters[c] = it1;
        if (!(conv || last)) next[atomicAdd(next_count, 1)] = entry;
        if (last && !conv && w.tol > 0.0) {  // tol = 0: exactly max_iter sweeps, not a failure
            atomicOr(&w.status[0], kStatusNoConv);
            atomicMin(&w.status[1], c);
        }
    }
    if (conv || last || !hist_on) {
        if (lane == 0) {
            w.hist[2 * c] = 0;
            w.hist[2 * c + 1] = 0;
            w.kuse[c] = 0;
        }
        return;
    }
    int k, head;
    bool dropped;
    ring_state(w, c, k, head, dropped);
    const int64_t cells_sq = int64_t(g.n_cells) * kMaxDepth * kMaxDepth;
    double *Lc = w.gram + int64_t(c) * kMaxDepth * kMaxDepth;             // scaled Cholesky, logical rows
    double *Hc = w.gram + cells_sq + int64_t(c) * kMaxDepth * kMaxDepth;  // Gram of dF, by slot
    double *dsc = w.gram + 2 * cells_sq + int64_t(c) * kMaxDepth;         // column scales, by slot
    const int lr = min(lane, kMaxDepth - 1);  // this lane's row of the factor
    double rinv = 0.0;                         // lane i: 1 / L[i][i]
    k = uni(k);  // the same in every lane
    head = uni(head);
    if (dropped) {
        for (int i = 0; i < k; ++i) {
            // row i of the rebuilt factor: L[0:i, 0:i] y = scaled H[i][0:i]
            const int si = (head + i) % depth;
            const int sl = (head + lane) % depth;
            const double rhs = (lane < i) ? Hc[si * kMaxDepth + sl] * dsc[si] * dsc[sl] : 0.0;
            const double y = tri_solve<false>(Ls, rhs, rinv, i);
            const double ysq = wave_sum(lane < i ? y * y : 0.0);
            const double lii = sqrt(fmax(1.0 + 1e-12 - ysq, 1e-10));
            if (lane < i) Ls[i][lane] = y;
            if (lane == 0) Ls[i][i] = lii;
            if (lane == i) rinv = 1.0 / lii;
            __syncthreads();
        }
    } else {
        for (int i0 = 0; i0 < k; i0 += kSolveBatch) {
            double r[kSolveBatch];
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u) r[u] = (i0 + u < k && lane <= i0 + u) ? Lc[(i0 + u) * kMaxDepth + lane] : 0.0;
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u)
                if (i0 + u < k && lane <= i0 + u) Ls[i0 + u][lane] = r[u];
        }
        __syncthreads();
        if (lane < k) rinv = 1.0 / Ls[lr][lr];
    }
    // reduced dots: h_j = <dF_j, dF_new>, b_j = <dF_j, f>, j = 0..k (k = new column)
    double hj = 0.0, bj_raw = 0.0;
    if (lane <= k) {
        for (int t0 = 0; t0 < ntile; t0 += kSolveBatch) {
            double a[kSolveBatch], b[kSolveBatch];
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u) {
                const bool in = t0 + u < ntile;
                a[u] = in ? part[(t0 + u) * kPartStride + 2 + lane] : 0.0;
                b[u] = in ? part[(t0 + u) * kPartStride + 2 + kMaxDepth + 1 + lane] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSolveBatch; ++u)
                if (t0 + u < ntile) {
                    hj += a[u];
                    bj_raw += b[u];
                }
        }
    }
    const int snew = (head + k) % depth;
    const double hkk = __shfl(hj, k, kWave);
    const double dk = hkk > 0.0 ? 1.0 / sqrt(hkk) : 0.0;
    const int sl = (head + (lane < k ? lane : 0)) % depth;
    const double dj = (lane < k) ? dsc[sl] : 0.0;
    // new row of the factor: L y = scaled h
    const double y = tri_solve<false>(Ls, (lane < k) ? hj * dj * dk : 0.0, rinv, k);
    const double ysq = wave_sum(lane < k ? y * y : 0.0);
    const double diag = 1.0 + 1e-12 - ysq;
    const bool add = (hkk > 0.0) && (diag > 1e-10);
    const int kuse = uni(add ? k + 1 : k);
    const double lkk = add ? sqrt(diag) : 1.0;
    if (add) {
        if (lane < k) {
            Hc[snew * kMaxDepth + sl] = hj;
            Hc[sl * kMaxDepth + snew] = hj;
            Ls[k][lane] = y;
        }
        if (lane == 0) {
            Hc[snew * kMaxDepth + snew] = hkk;
            dsc[snew] = dk;
        }
        if (lane == k) {
            Ls[k][k] = lkk;
            rinv = 1.0 / lkk;
        }
    }
    __syncthreads();
    const double scl = (lane < k) ? dj : ((lane == k) ? dk : 0.0);
    // L z = scaled b, then L^T x = z
    const double z = tri_solve<false>(Ls, (lane < kuse) ? bj_raw * scl : 0.0, rinv, kuse);
    const double xs = tri_solve<true>(Ls, z, rinv, kuse);
    if (lane < kuse) gam[lane] = xs * scl;
    // write back the rows that changed: all after a rebuild, else the new one
    if (dropped)
        for (int i = 0; i < k; ++i)
            if (lane <= i) Lc[i * kMaxDepth + lane] = Ls[i][lane];
    if (add) {
        if (lane < k) Lc[k * kMaxDepth + lane] = y;
        if (lane == 0) Lc[k * kMaxDepth + k] = lkk;
    }
    if (lane == 0) {
        w.kuse[c] = kuse;
        w.hist[2 * c] = kuse;
        w.hist[2 * c + 1] = head;
        if (g.hist_small < depth) {
            // the slot the next iteration appends to: a pool slot is taken the
            // first time it lies beyond the in-place columns
            int k2 = kuse, h2 = kuse == 0 ? 0 : head;  // as ring_state reads it back
            if (k2 >= depth) {
                const int drop = min(kDrop, k2);
                h2 = (h2 + drop) % depth;
                k2 -= drop;
            }
            if ((h2 + k2) % depth >= g.hist_small && w.pool_slot[c] < 0) {
                const int p = atomicAdd(w.pool_count, 1);
                if (p < g.pool_cap) {
                    w.pool_slot[c] = p;
                } else {  // pool exhausted: the step fails; the cell restarts its history in place
                    atomicOr(&w.status[0], kStatusHistoryPool);
                    atomicMin(&w.status[1], c);
                    w.hist[2 * c] = 0;
                    w.hist[2 * c + 1] = 0;
                }
            }
        }
    }
    __syncthreads();  // Ls is reused by the next item
}

template <int N, int DC, typename HT>
__global__ void __launch_bounds__(256) k_round_dots(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ count, int tpc) {
    __shared__ double accs[kPartStride][4];
    const int n_items = *count * tpc;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(list[item / tpc], slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        const int tile = item % tpc;
        if (tile * 64 >= int(g.dof_ptr[c + 1] - g.dof_ptr[c])) continue;
        and_dots_tile<N, DC, HT>(g, w, c, tile, accs);
        __syncthreads();  // accs is rewritten by the next item
    }
}

__global__ void __launch_bounds__(64) k_round_solve(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ count, int32_t *next,
                                                    int32_t *next_count) {
    __shared__ double Ls[kMaxDepth][kMaxDepth];
    const int n_items = *count;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int32_t entry = list[item];
        int slot, c;
        decode(entry, slot, c);
        and_solve_cell(tab[slot].g, tab[slot].w, c, entry, next, next_count, Ls);
    }
}

constexpr int kUpdBatch = 8;

// Work item = (entry, span of the cell's space-time values): one 64-DOF tile
// (64 nc values), or with `fine` 256 values, one per thread, so that in the
// last iterations, with few cells left and long histories, a cell's history
// columns are read by five times as many waves.  Each value's arithmetic is
// the same either way.
template <int N, typename HT>
__global__ void __launch_bounds__(256) k_round_update(const DevSlot *__restrict__ tab, const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ count, int per, int fine) {
    constexpr int nc = Dim<N>::nc;
    const int span = fine ? 256 : 64 * nc;
    const int n_items = *count * per;
    for (int item = xcd_block(); item < n_items; item += gridDim.x) {
        int slot, c;
        decode(list[item / per], slot, c);
        const DevGrid &g = tab[slot].g;
        const DevWork &w = tab[slot].w;
        const int64_t d0 = g.dof_ptr[c];
        const int64_t len = (g.dof_ptr[c + 1] - d0) * nc;
        const int64_t e0 = int64_t(item % per) * span;
        if (e0 >= len) continue;
        const int64_t e1 = min(len, e0 + span);
        const int64_t base = d0 * nc;
        const int kuse = w.kuse[c];
        const int depth = w.depth;
        const int head = w.hist[2 * c + 1];
        const cptr<double> gam = (cptr<double>)uni_ptr(w.gamma + int64_t(c) * kMaxDepth);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            double xv = w.gprev[base + e];
            int j = 0;
            for (; j + kUpdBatch <= kuse; j += kUpdBatch) {
                double d[kUpdBatch];
#pragma unroll
                for (int u = 0; u < kUpdBatch; ++u)
                    d[u] = double(hist_col<HT>(g, w, w.dG, w.dGp, c, base, len, (head + j + u) % depth)[e]);
#pragma unroll
                for (int u = 0; u < kUpdBatch; ++u) xv -= gam[j + u] * d[u];
            }
            for (; j < kuse; ++j) xv -= gam[j] * double(hist_col<HT>(g, w, w.dG, w.dGp, c, base, len, (head + j) % depth)[e]);
            w.x[base + e] = xv;
        }
    }
}

// ------------------------------------------------------------- corrector

// Outside trace of a boundary face node of a bounded mesh from the Dirichlet
// data: the exact state q_a at the predictor's time nodes (primitive, from
// g.bstate), qbar = dt sum_a w_a q_a and Fbar_x = dt sum_a w_a F_x(q_a, grad
// q_a), laid out as a trace entry: qbar (5), Fbar (3 x 5).  With viscosity
// mu (the inside cell's) or heat conduction the flux is the Navier-Stokes one
// with the exact gradient (g.bgrad, primitive, turned into the conserved
// variables' here); else the Euler flux.
template <int N>
__device__ inline void boundary_trace(const DevGrid &g, int64_t node, double dt, double mu, double tb[20]) {
    constexpr int nt = N + 1;
#pragma unroll
    for (int e = 0; e < 20; ++e) tb[e] = 0.0;
    const double *s = g.bstate + node * nt * 5;
    const double gam = g.gamma;
    const bool viscous = (mu != 0.0 || g.kappa != 0.0) && g.bgrad != nullptr;
#pragma unroll
    for (int a = 0; a < nt; ++a) {
        const double r = s[a * 5], vx = s[a * 5 + 1], vy = s[a * 5 + 2], vz = s[a * 5 + 3], p = s[a * 5 + 4];
        const double q[5] = {r, r * vx, r * vy, r * vz, p / (gam - 1.0) + 0.5 * r * (vx * vx + vy * vy + vz * vz)};
        double F[3][5];
        double gq[3][5] = {};
        if (viscous) {
            const double *gw = g.bgrad + (node * nt + a) * 15;  // [d][k]
            for (int d = 0; d < 3; ++d) {
                const double gr = gw[d * 5], gu = gw[d * 5 + 1], gv = gw[d * 5 + 2], gz = gw[d * 5 + 3], gp = gw[d * 5 + 4];
                gq[d][0] = gr;
                gq[d][1] = vx * gr + r * gu;
                gq[d][2] = vy * gr + r * gv;
                gq[d][3] = vz * gr + r * gz;
                gq[d][4] = gp / (gam - 1.0) + 0.5 * (vx * vx + vy * vy + vz * vz) * gr + r * (vx * gu + vy * gv + vz * gz);
            }
        }
        ns_flux<true>(q, gq, gam, viscous ? mu : 0.0, viscous ? g.kappa : 0.0, g.cv, F);
        const double wa = g.ref->w[a];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            tb[v] += wa * q[v];
#pragma unroll
            for (int x = 0; x < 3; ++x) tb[5 + 5 * x + v] += wa * F[x][v];
        }
    }
#pragma unroll
    for (int e = 0; e < 20; ++e) tb[e] *= dt;
}

// Rusanov flux with viscous penalty (eq. 3.33) at the face nodes of every
// boundary sub-triangle, contracted with the face mass: fc[k][j'] =
// 2 A_k sum_j Z^[j'][j] G_j.  One value of the dissipation coefficient per
// sub-triangle: the maximum over its nodes and both sides.
template <int N>
__global__ void __launch_bounds__(256) k_face(DevGrid g, DevWork w, int which) {
    constexpr int nf = Dim<N>::nf;
    const double dt = *w.dt;
    constexpr int tpb = 256 / nf;
    __shared__ double lam_s[tpb][nf], lamv_s[tpb][nf];
    __shared__ double G_s[tpb][nf][5];
    const int t = threadIdx.x / nf, j = threadIdx.x % nf;
    const int64_t k = int64_t(blockIdx.x) * tpb + t;
    const bool valid = t < tpb && k < g.nsub && w.late2[g.sub_cell[k]] == which;
    double Gv[5] = {0, 0, 0, 0, 0};
    double nrm[3] = {0, 0, 0}, a2 = 0.0;
    double eps = 0.0;
    if (valid) {
        const int64_t kn = g.nbr_sub[k];
        const double *ti = w.trace + (k * nf + j) * 20;
        double to[20];  // outside trace, in registers (constant indices only)
        if (kn >= 0) {
            const double *tr = w.trace + (kn * nf + g.perm[k * nf + j]) * 20;
#pragma unroll
            for (int e = 0; e < 20; ++e) to[e] = tr[e];
        } else {
            boundary_trace<N>(g, (-1 - kn) * nf + j, dt, w.mu_cell[g.sub_cell[k]], to);
        }
        const double *T = g.tri + k * 4;
        a2 = T[0];
        nrm[0] = T[1];
        nrm[1] = T[2];
        nrm[2] = T[3];
        // outside viscosity and length scale: the cell's own at a boundary (mu = 0 there)
        const int ci = g.sub_cell[k], co = kn >= 0 ? g.sub_cell[kn] : ci;
        double qi[5], qo[5];
        const double idt = 1.0 / dt;
        for (int v = 0; v < 5; ++v) {
            qi[v] = ti[v] * idt;
            qo[v] = to[v] * idt;
        }
        const double gam = g.gamma;
        const double vni = (qi[1] * nrm[0] + qi[2] * nrm[1] + qi[3] * nrm[2]) / qi[0];
        const double vno = (qo[1] * nrm[0] + qo[2] * nrm[1] + qo[3] * nrm[2]) / qo[0];
        const double li = fabs(vni) + sqrt(gam * pressure5(qi, gam) / qi[0]);
        const double lo = fabs(vno) + sqrt(gam * pressure5(qo, gam) / qo[0]);
        lam_s[t][j] = fmax(li, lo);
        lamv_s[t][j] = fmax(visc_eig(w.mu_cell[ci], g.kappa, g.cv, qi[0]), visc_eig(w.mu_cell[co], g.kappa, g.cv, qo[0]));
        eps = double(2 * N + 1) / ((g.h[ci] + g.h[co]) * sqrt(M_PI / 2.0));
        for (int v = 0; v < 5; ++v) {
            const double fsum0 = to[5 + v] + ti[5 + v];
            const double fsum1 = to[10 + v] + ti[10 + v];
            const double fsum2 = to[15 + v] + ti[15 + v];
            Gv[v] = fsum0 * nrm[0] + fsum1 * nrm[1] + fsum2 * nrm[2];
        }
        for (int v = 0; v < 5; ++v) G_s[t][j][v] = to[v] - ti[v];  // qbar jump, scaled below
    }
    __syncthreads();
    if (valid) {
        double lam = 0.0, lamv = 0.0;
        for (int i = 0; i < nf; ++i) {
            lam = fmax(lam, lam_s[t][i]);
            lamv = fmax(lamv, lamv_s[t][i]);
        }
        const double sdiss = lam + 2.0 * eps * lamv;
        for (int v = 0; v < 5; ++v) Gv[v] = 0.5 * Gv[v] - 0.5 * sdiss * G_s[t][j][v];
    }
    __syncthreads();
    if (valid)
        for (int v = 0; v < 5; ++v) G_s[t][j][v] = Gv[v];
    __syncthreads();
    if (valid) {
        double out[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < nf; ++i) {
            const double z = g.ref->Z[j * nf + i];
            for (int v = 0; v < 5; ++v) out[v] += z * G_s[t][i][v];
        }
        double *o = w.fc + (k * nf + j) * 5;
        for (int v = 0; v < 5; ++v) o[v] = a2 * out[v];
    }
}

// rhs[l][v] = volume term - face term, gathered over the incidence lists.
template <int N>
__global__ void __launch_bounds__(256) k_rhs(DevGrid g, DevWork w, int which) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= g.ndof * 5) return;
    const int64_t l = t / 5;
    if (w.late2[g.dof_cell[l]] != which) return;
    const int v = int(t % 5);
    const double acc = ordered_gather_sum(w.vk, g.inc_idx, g.inc_ptr[l], g.inc_ptr[l + 1], 5, v);
    const double fac = ordered_gather_sum(w.fc, g.finc_idx, g.finc_ptr[l], g.finc_ptr[l + 1], 5, v);
    w.rhs[t] = acc - fac;
}

__global__ void k_reset_status(DevWork w, int n_cells) {
    if (threadIdx.x == 0) {
        w.status[0] = 0;
        w.status[1] = INT_MAX;
        w.status[2] = n_cells;
        w.status[3] = 0;
        w.status[4] = 0;
        w.status[5] = 0;
        w.status[6] = 0;
        w.status[7] = 0;
        *w.pool_count = 0;
    }
}

// Predictor iteration counts over the cells of one simulation: status[4] =
// min, status[5] = max, status[6..7] = 64-bit sum.
__global__ void __launch_bounds__(1024) k_step_stats(DevWork w, int n_cells) {
    if (threadIdx.x == 0) {
        // a successful step leaves its converged predictor in x for the next start
        *w.guess_ok = w.status[0] == 0 ? 1 : 0;
        *w.dt_prev = *w.dt;
    }
    __shared__ int smin[16], smax[16];
    __shared__ unsigned long long ssum[16];
    int mn = INT_MAX, mx = 0;
    unsigned long long sum = 0;
    for (int i = threadIdx.x; i < n_cells; i += blockDim.x) {
        const int v = w.iters[i];
        mn = min(mn, v);
        mx = max(mx, v);
        sum += unsigned(v);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, kWave));
        mx = max(mx, __shfl_xor(mx, o, kWave));
        sum += __shfl_xor(sum, o, kWave);
    }
    const int wv = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        smin[wv] = mn;
        smax[wv] = mx;
        ssum[wv] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < int(blockDim.x) / kWave; ++i) {
            mn = min(mn, smin[i]);
            mx = max(mx, smax[i]);
            sum += ssum[i];
        }
        w.status[4] = n_cells > 0 ? mn : 0;
        w.status[5] = mx;
        *reinterpret_cast<unsigned long long *>(w.status + 6) = sum;
    }
}

__global__ void k_positivity(DevGrid g, DevWork w, const double *__restrict__ u, int which) {
    const int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (l >= g.ndof || w.late2[g.dof_cell[l]] != which) return;
    double q[5];
    bool finite = true;
    for (int v = 0; v < 5; ++v) {
        q[v] = u[v * g.ndof + l];
        finite = finite && isfinite(q[v]);
    }
    int flag = 0;
    if (!finite)
        flag = kStatusNonfinite;
    else if (!(q[0] > 0.0) || !(pressure5(q, g.gamma) > 0.0))
        flag = kStatusPositivity;
    if (flag) {
        atomicOr(&w.status[0], flag);
        atomicMin(&w.status[1], g.dof_cell[l]);
    }
}

// ------------------------------------------------------- error norms
//
// The L2 norm of Sec. 5, (sum over cells of int |u_h - u_e|^2)^(1/2), with
// each cell's integral taken over its sub-tets by the conical product rule of
// the reference data: thread = (sub-tet k, point q).  The vertices of sub-tet
// k are its reference nodes 0..3 (the App. A order), so the point is
// X0 + sum_d xi_d (X_d - X0) with X the DOF coordinates of those nodes.

constexpr int kL2Threads = 256;

__global__ void __launch_bounds__(kL2Threads) k_l2_points(DevGrid g, const double *__restrict__ dof_xyz,
                                                         double *__restrict__ xq) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int nq = g.ref->nq;
    if (t >= g.nsub * nq) return;
    const int64_t k = t / nq;
    const int q = int(t % nq);
    const int64_t d0 = g.dof_ptr[g.sub_cell[k]];
    double X[4][3];
    for (int v = 0; v < 4; ++v) {
        const int64_t l = d0 + g.conn[k * g.np + v];
        for (int x = 0; x < 3; ++x) X[v][x] = dof_xyz[x * g.ndof + l];
    }
    const double *xi = g.ref->qxi + 3 * q;
    for (int x = 0; x < 3; ++x)
        xq[t * 3 + x] = X[0][x] + xi[0] * (X[1][x] - X[0][x]) + xi[1] * (X[2][x] - X[0][x]) + xi[2] * (X[3][x] - X[0][x]);
}

// Block b sums its 256 terms in a fixed tree order into partial[b].
__global__ void __launch_bounds__(kL2Threads) k_l2_terms(DevGrid g, const double *__restrict__ u, int var,
                                                        const double *__restrict__ ref, double *__restrict__ partial) {
    __shared__ double red[kL2Threads];
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int nq = g.ref->nq, np = g.np;
    double e = 0.0;
    if (t < g.nsub * nq) {
        const int64_t k = t / nq;
        const int q = int(t % nq);
        const int64_t d0 = g.dof_ptr[g.sub_cell[k]];
        const double *ph = g.ref->qphi + q * np;
        double uh = 0.0;
        for (int m = 0; m < np; ++m) uh += ph[m] * u[var * g.ndof + d0 + g.conn[k * np + m]];
        const double r = ref[t];
        const double d = uh - r;
        e = r == r ? g.ref->qw[q] * g.geo[k * 10 + 9] * d * d : 0.0;  // NaN: point left out
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int h = kL2Threads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block: the partials in a fixed order (each thread a strided sum, then a tree).
__global__ void __launch_bounds__(kL2Threads) k_l2_sum(const double *__restrict__ partial, int64_t n, double *out) {
    __shared__ double red[kL2Threads];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a += partial[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = kL2Threads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <typename F>
hipError_t dispatch(int N, F &&f) {
    switch (N) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        default: return hipErrorInvalidValue;
    }
}

inline unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

}  // namespace

hipError_t launch_reset_status(const DevGrid &g, const DevWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, w, g.n_cells);
    return hipGetLastError();
}

hipError_t launch_mass_assemble(const DevGrid &g, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        hipLaunchKernelGGL(k_mass_assemble<decltype(n)::value>, dim3(g.n_cells), dim3(256), 0, s, g);
        return hipGetLastError();
    });
}

hipError_t launch_mass_invert(const DevGrid &g, hipStream_t s) {
    size_t shmem = size_t(g.max_cell_dofs) * sizeof(double);
    hipLaunchKernelGGL(k_mass_invert, dim3(g.n_cells), dim3(kInvThreads), shmem, s, g);
    if (g.mixed) hipLaunchKernelGGL(k_minv_to_f32, dim3(g.n_cells), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_prim_to_cons(const DevGrid &g, const double *prim, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_prim_to_cons, dim3(blocks_for(g.ndof, 256)), dim3(256), 0, s, g.ndof, g.gamma, prim, u);
    return hipGetLastError();
}

hipError_t launch_detect(const DevGrid &g, const DevWork &w, const double *u, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        hipLaunchKernelGGL(k_detect<decltype(n)::value>, dim3(blocks_for(g.n_cells, 4)), dim3(256), 0, s, g, w, u);
        return hipGetLastError();
    });
}

hipError_t launch_cfl_dt(const DevGrid &g, const DevWork &w, double cfl, double h_min, double *smax, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl_dt, dim3(1), dim3(1024), 0, s, g.n_cells, w, smax, cfl, h_min, 2 * g.N + 1);
    return hipGetLastError();
}

hipError_t launch_set_dt(const DevWork &w, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, s, w.dt, dt);
    return hipGetLastError();
}

hipError_t launch_pred_init(const DevGrid &g, const DevWork &w, int slot, int32_t *list, int64_t base, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        const int64_t elems = g.ndof * Dim<decltype(n)::value>::nc;
        const int64_t m = elems > g.n_cells ? elems : g.n_cells;
        hipLaunchKernelGGL(k_pred_init<decltype(n)::value>, dim3(blocks_for(m, 256)), dim3(256), 0, s, g, w, slot,
                           list, base);
        return hipGetLastError();
    });
}

hipError_t launch_set_count(int32_t *count, int value, hipStream_t s) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, count, value);
    return hipGetLastError();
}

hipError_t launch_pred_round(const RoundArgs &a, hipStream_t s) {
    return dispatch(a.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        const int chunks = (a.max_cell_subtets + D::spb - 1) / D::spb;
        const int tpc = (a.max_cell_dofs + 63) / 64;
        // one workgroup per item of the longest possible list, at most the
        // persistent grid (n_upper < 0: length unknown, graph capture)
        auto grid = [&](int persistent, int per) {
            if (a.n_upper < 0) return dim3(unsigned(persistent));
            const int items = std::max(1, a.n_upper * per);
            return dim3(unsigned(persistent > 0 ? std::min(persistent, items) : items));
        };
        const int per = int((int64_t(a.max_cell_dofs) * D::nc + 255) / 256);
        auto sub = a.visc == 2 ? (a.mixed ? k_round_subtet<NN, 2, true> : k_round_subtet<NN, 2, false>)
                   : a.visc == 1 ? (a.mixed ? k_round_subtet<NN, 1, true> : k_round_subtet<NN, 1, false>)
                                 : (a.mixed ? k_round_subtet<NN, 0, true> : k_round_subtet<NN, 0, false>);
        hipLaunchKernelGGL(sub, grid(a.shape.g_sub, chunks), dim3(256), 0, s, a.tab, a.list, a.count, chunks,
                           a.next_count);
        hipLaunchKernelGGL(k_round_gather<NN>, grid(a.shape.g_gather, per), dim3(256), 0, s, a.tab, a.list, a.count,
                           per);
        if (a.ev0) (void)hipEventRecord(a.ev0, s);
        if (a.mixed)
            hipLaunchKernelGGL(k_round_minv32<D::nc>, grid(a.shape.g_minv, tpc), dim3(256), 0, s, a.tab, a.list,
                               a.count, tpc, a.bytes);
        else
            hipLaunchKernelGGL(k_round_minv<D::nc>, grid(a.shape.g_minv, tpc * a.split), dim3(256), 0, s, a.tab,
                               a.list, a.count, tpc, a.split, a.bytes);
        if (a.ev1) (void)hipEventRecord(a.ev1, s);
        auto dots = a.mixed ? (a.upd_fine && a.n_upper >= 0 ? k_round_dots<NN, kDotColsWide, float>
                                                           : k_round_dots<NN, kDotCols, float>)
                            : (a.upd_fine && a.n_upper >= 0 ? k_round_dots<NN, kDotColsWide64, double>
                                                           : k_round_dots<NN, kDotCols, double>);
        hipLaunchKernelGGL(dots, grid(a.shape.g_dots, tpc), dim3(256), 0, s, a.tab, a.list, a.count, tpc);
        hipLaunchKernelGGL(k_round_solve, grid(a.shape.g_solve, 1), dim3(kWave), 0, s, a.tab, a.list, a.count, a.next,
                           a.next_count);
        const int upd_per = a.upd_fine ? per : tpc;
        auto upd = a.mixed ? k_round_update<NN, float> : k_round_update<NN, double>;
        hipLaunchKernelGGL(upd, grid(a.shape.g_update, upd_per), dim3(256), 0, s, a.tab, a.list, a.count, upd_per,
                           a.upd_fine);
        return hipGetLastError();
    });
}

hipError_t launch_clear_late(const DevGrid &g, const DevWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_late, dim3(blocks_for(g.n_cells, 256)), dim3(256), 0, s, g, w);
    return hipGetLastError();
}

hipError_t launch_relabel_late(const DevGrid &g, const DevWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_relabel_late, dim3(blocks_for(g.n_cells, 256)), dim3(256), 0, s, g, w);
    return hipGetLastError();
}

hipError_t launch_mark_listed(const DevSlot *tab, const int32_t *list, int count, int value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_listed, dim3(blocks_for(count, 256)), dim3(256), 0, s, tab, list, count, value);
    return hipGetLastError();
}

hipError_t launch_clear_late2(const DevGrid &g, const DevWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_late2, dim3(blocks_for(g.n_cells, 256)), dim3(256), 0, s, g, w);
    return hipGetLastError();
}

hipError_t launch_mark_late2(const DevSlot *tab, const int32_t *list, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_late2, dim3(unsigned(std::min(count, 4096))), dim3(256), 0, s, tab, list, count);
    return hipGetLastError();
}

hipError_t launch_pred_post(const DevGrid &g, const DevWork &w, int which, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        auto post = g.kappa != 0.0              ? k_subtet_post<NN, 2>
                    : (g.mu != 0.0 || g.av) ? k_subtet_post<NN, 1>
                                            : k_subtet_post<NN, 0>;
        hipLaunchKernelGGL(post, dim3(blocks_for(g.nsub, D::spb)), dim3(D::threads), 0, s, g, w, which);
        return hipGetLastError();
    });
}

hipError_t launch_correct(const DevGrid &g, const DevWork &w, double *u, int which, hipStream_t s, int max_blocks) {
    return dispatch(g.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        hipLaunchKernelGGL(k_face<NN>, dim3(blocks_for(g.nsub, 256 / D::nf)), dim3(256), 0, s, g, w, which);
        hipLaunchKernelGGL(k_rhs<NN>, dim3(blocks_for(g.ndof * 5, 256)), dim3(256), 0, s, g, w, which);
        const int tpc = (g.max_cell_dofs + 63) / 64;
        unsigned blocks = unsigned(g.n_cells) * tpc;
        if (max_blocks > 0) blocks = std::min(blocks, unsigned(max_blocks));
        hipLaunchKernelGGL(k_minv_update<5>, dim3(blocks), dim3(256), 0, s, g, w.rhs, u, tpc, w.late2, which);
        hipLaunchKernelGGL(k_positivity, dim3(blocks_for(g.ndof, 256)), dim3(256), 0, s, g, w, u, which);
        return hipGetLastError();
    });
}

hipError_t launch_step_stats(const DevGrid &g, const DevWork &w, hipStream_t s) {
    hipLaunchKernelGGL(k_step_stats, dim3(1), dim3(1024), 0, s, w, g.n_cells);
    return hipGetLastError();
}

int64_t l2_blocks(const DevGrid &g) { return (g.nsub * int64_t((g.N + 3) * (g.N + 3) * (g.N + 3)) + kL2Threads - 1) / kL2Threads; }

hipError_t launch_l2_points(const DevGrid &g, const double *dof_xyz, double *xq, hipStream_t s) {
    hipLaunchKernelGGL(k_l2_points, dim3(unsigned(l2_blocks(g))), dim3(kL2Threads), 0, s, g, dof_xyz, xq);
    return hipGetLastError();
}

hipError_t launch_l2_error(const DevGrid &g, const double *u, int var, const double *ref, double *partial,
                           double *out, hipStream_t s) {
    const int64_t nb = l2_blocks(g);
    hipLaunchKernelGGL(k_l2_terms, dim3(unsigned(nb)), dim3(kL2Threads), 0, s, g, u, var, ref, partial);
    hipLaunchKernelGGL(k_l2_sum, dim3(1), dim3(kL2Threads), 0, s, partial, nb, out);
    return hipGetLastError();
}

IterShape resident_shape(int N, int mixed, int visc) {
    IterShape sh;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    auto fit = [&](const void *f, int threads) {
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, 0) != hipSuccess || per < 1) per = 1;
        return per * cus;
    };
    (void)dispatch(N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        const void *subs[3][2] = {{reinterpret_cast<const void *>(&k_round_subtet<NN, 0, false>),
                                   reinterpret_cast<const void *>(&k_round_subtet<NN, 0, true>)},
                                  {reinterpret_cast<const void *>(&k_round_subtet<NN, 1, false>),
                                   reinterpret_cast<const void *>(&k_round_subtet<NN, 1, true>)},
                                  {reinterpret_cast<const void *>(&k_round_subtet<NN, 2, false>),
                                   reinterpret_cast<const void *>(&k_round_subtet<NN, 2, true>)}};
        sh.g_sub = fit(subs[visc < 0 ? 0 : visc > 2 ? 2 : visc][mixed ? 1 : 0],
                       256);
        sh.g_gather = fit(reinterpret_cast<const void *>(&k_round_gather<NN>), 256);
        sh.g_minv = mixed ? fit(reinterpret_cast<const void *>(&k_round_minv32<D::nc>), 256)
                          : fit(reinterpret_cast<const void *>(&k_round_minv<D::nc>), 256);
        sh.g_dots = mixed ? fit(reinterpret_cast<const void *>(&k_round_dots<NN, kDotCols, float>), 256)
                          : fit(reinterpret_cast<const void *>(&k_round_dots<NN, kDotCols, double>), 256);
        sh.g_solve = fit(reinterpret_cast<const void *>(&k_round_solve), kWave);
        sh.g_update = mixed ? fit(reinterpret_cast<const void *>(&k_round_update<NN, float>), 256)
                            : fit(reinterpret_cast<const void *>(&k_round_update<NN, double>), 256);
        return hipSuccess;
    });
    return sh;
}

}  // namespace afe
