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

__device__ inline double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline double wave_min(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// Physical flux F[x][v] of the compressible Navier-Stokes equations (Sec. 2)
// at one point.  gq[x][v] = d q_v / d x_x is used only when mu != 0; heat
// conduction is zero.
__device__ inline void ns_flux(const double q[5], const double gq[3][5], double gamma, double mu, double F[3][5]) {
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
    double *M = g.minv + g.minv_ptr[c];
    for (int64_t e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = 0.0;
    __syncthreads();
    for (int64_t k = g.sub_ptr[c]; k < g.sub_ptr[c + 1]; ++k) {
        const double dj = g.geo[k * 10 + 9];
        for (int t = threadIdx.x; t < np * np; t += blockDim.x) {
            const int m = t / np, p = t % np;
            const int64_t i = g.conn[k * np + m], j = g.conn[k * np + p];
            M[i * n + j] += dj * g.ref->M[m * np + p];
        }
        __syncthreads();
    }
}

// In-place inverse of M_i: Jacobi scaling to unit diagonal, Gauss-Jordan
// elimination without pivoting (the scaled matrix is symmetric positive
// definite), unscaling, symmetrisation.
__global__ void __launch_bounds__(1024) k_mass_invert(DevGrid g) {
    extern __shared__ double sh[];
    const int c = blockIdx.x;
    const int n = int(g.dof_ptr[c + 1] - g.dof_ptr[c]);
    double *A = g.minv + g.minv_ptr[c];
    double *dsc = sh;
    double *rowk = sh + n;
    double *colk = sh + 2 * n;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int tx = tid % 64, ty = tid / 64, ny = nth / 64;
    for (int i = tid; i < n; i += nth) dsc[i] = 1.0 / sqrt(A[int64_t(i) * n + i]);
    __syncthreads();
    for (int i = ty; i < n; i += ny)
        for (int j = tx; j < n; j += 64) A[int64_t(i) * n + j] *= dsc[i] * dsc[j];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = A[int64_t(k) * n + k];
        const double ip = 1.0 / piv;
        for (int j = tid; j < n; j += nth) {
            rowk[j] = (j == k ? 1.0 : A[int64_t(k) * n + j]) * ip;
            colk[j] = (j == k ? 0.0 : A[int64_t(j) * n + k]);
        }
        __syncthreads();
        for (int i = ty; i < n; i += ny) {
            const double ci = colk[i];
            double *Ai = A + int64_t(i) * n;
            if (i == k) {
                for (int j = tx; j < n; j += 64) Ai[j] = rowk[j];
            } else {
                for (int j = tx; j < n; j += 64) Ai[j] = (j == k ? 0.0 : Ai[j]) - ci * rowk[j];
            }
        }
        __syncthreads();
    }
    for (int i = ty; i < n; i += ny)
        for (int j = tx; j < n; j += 64) {
            if (j < i) continue;
            const double v = 0.5 * (A[int64_t(i) * n + j] + A[int64_t(j) * n + i]) * dsc[i] * dsc[j];
            A[int64_t(i) * n + j] = v;
            A[int64_t(j) * n + i] = v;
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
        const int jn = g.perm[k * nf + j];
        const int64_t lo = g.dof_ptr[g.sub_cell[kn]] + g.conn[kn * np + g.ref->fn[jn]];
        double qi[5], qo[5];
        for (int v = 0; v < 5; ++v) {
            qi[v] = u[v * nd + li];
            qo[v] = u[v * nd + lo];
        }
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
        const double lv = 4.0 * mu_c / (3.0 * q[0]);
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

__global__ void __launch_bounds__(1024) k_cfl_max(int n, const double *__restrict__ term, double *out) {
    __shared__ double red[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, term[i]);
    m = wave_max(m);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x < kWave) {
        double v = threadIdx.x < blockDim.x / kWave ? red[threadIdx.x] : 0.0;
        v = wave_max(v);
        if (threadIdx.x == 0) out[0] = v;
    }
}

// ------------------------------------------------------------- predictor

template <int N>
__global__ void k_pred_init(DevGrid g, DevWork w, const double *__restrict__ u) {
    constexpr int nc = Dim<N>::nc, nt = Dim<N>::nt;
    const int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (l < g.ndof)
        for (int a = 0; a < nt; ++a)
            for (int v = 0; v < 5; ++v) w.x[l * nc + a * 5 + v] = u[v * g.ndof + l];
    if (l < g.n_cells) {
        w.active[l] = 1;
        w.iters[l] = 0;
        w.hist[2 * l] = 0;
        w.hist[2 * l + 1] = 0;
    }
}

// Per sub-tet and time node: nodal flux, contravariant transform
// f*_d = dt sum_x G[d][x] F_x (eq:modified_fluxes), and the reference stiffness
// contraction r[a][m] = w_a |J| sum_d sum_p K^_d[m][p] f*_d[a][p] (eq:ader4).
// POST = true instead forms the time integrals of the converged predictor:
// the volume term |J| sum_d V^_d F*bar_d (Sec. 4.4) and the face traces
// (qbar, Fbar) at the boundary-triangle nodes.
template <int N, bool POST>
__global__ void __launch_bounds__(Dim<N>::threads) k_subtet(DevGrid g, DevWork w, double dt) {
    constexpr int np = Dim<N>::np, nt = Dim<N>::nt, nc = Dim<N>::nc, npt = Dim<N>::npt, spb = Dim<N>::spb;
    constexpr int nf = Dim<N>::nf;
    __shared__ double Ks[3 * np * np];
    __shared__ double Ds[3 * np * np];
    __shared__ double qs[spb][nt][np][5];
    __shared__ double fs[spb][nt][np][15];
    __shared__ double Fs[POST ? spb : 1][POST ? nt : 1][POST ? np : 1][15];
    __shared__ double fbar[POST ? spb : 1][POST ? np : 1][15];
    const int tid = threadIdx.x;
    for (int t = tid; t < 3 * np * np; t += blockDim.x) {
        Ks[t] = g.ref->K[t];
        Ds[t] = g.ref->D[t];
    }
    const int s = tid / npt, a = (tid / np) % nt, m = tid % np;
    const int64_t k = int64_t(blockIdx.x) * spb + s;
    bool valid = (s < spb) && (k < g.nsub);
    int c = 0;
    if (valid) {
        c = g.sub_cell[k];
        if (!POST) valid = w.active[c] != 0;
    }
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
    if (valid) {
        double gq[3][5] = {};
        if (mu_c != 0.0) {
            double rg[3][5] = {};
            for (int d = 0; d < 3; ++d)
                for (int p = 0; p < np; ++p) {
                    const double dd = Ds[(d * np + m) * np + p];
                    for (int v = 0; v < 5; ++v) rg[d][v] += dd * qs[s][a][p][v];
                }
            for (int x = 0; x < 3; ++x)
                for (int v = 0; v < 5; ++v) gq[x][v] = G[0 * 3 + x] * rg[0][v] + G[1 * 3 + x] * rg[1][v] + G[2 * 3 + x] * rg[2][v];
        }
        double F[3][5];
        ns_flux(q, gq, g.gamma, mu_c, F);
        for (int d = 0; d < 3; ++d)
            for (int v = 0; v < 5; ++v)
                fs[s][a][m][d * 5 + v] = dt * (G[d * 3 + 0] * F[0][v] + G[d * 3 + 1] * F[1][v] + G[d * 3 + 2] * F[2][v]);
        if (POST)
            for (int x = 0; x < 3; ++x)
                for (int v = 0; v < 5; ++v) Fs[POST ? s : 0][POST ? a : 0][POST ? m : 0][x * 5 + v] = F[x][v];
    }
    __syncthreads();
    if (!POST) {
        if (!valid) return;
        double r[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; ++d)
            for (int p = 0; p < np; ++p) {
                const double kk = Ks[(d * np + m) * np + p];
                for (int v = 0; v < 5; ++v) r[v] += kk * fs[s][a][p][d * 5 + v];
            }
        const double sc = g.ref->w[a] * dj;
        double *out = w.rk + (k * np + m) * nc + a * 5;
        for (int v = 0; v < 5; ++v) out[v] = sc * r[v];
        return;
    }
    // POST: time integrals
    if (valid && a == 0) {
        for (int i = 0; i < 15; ++i) {
            double acc = 0.0;
            for (int b = 0; b < nt; ++b) acc += g.ref->w[b] * fs[s][b][m][i];
            fbar[POST ? s : 0][POST ? m : 0][i] = acc;
        }
    }
    __syncthreads();
    if (!valid) return;
    if (a == 0) {
        // volume term: V^_d[m][p] = K^_d[p][m]
        double r[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; ++d)
            for (int p = 0; p < np; ++p) {
                const double kk = Ks[(d * np + p) * np + m];
                for (int v = 0; v < 5; ++v) r[v] += kk * fbar[POST ? s : 0][p][d * 5 + v];
            }
        double *out = w.vk + (k * np + m) * 5;
        for (int v = 0; v < 5; ++v) out[v] = dj * r[v];
    } else if (a == 1 || nt == 1) {
        // traces at face nodes (threads of time node 1 are free here)
        if (m < nf) {
            const int j = m, mm = g.ref->fn[j];
            double *out = w.trace + (k * nf + j) * 20;
            for (int v = 0; v < 5; ++v) {
                double acc = 0.0;
                for (int b = 0; b < nt; ++b) acc += g.ref->w[b] * qs[s][b][mm][v];
                out[v] = dt * acc;
            }
            for (int i = 0; i < 15; ++i) {
                double acc = 0.0;
                for (int b = 0; b < nt; ++b) acc += g.ref->w[b] * Fs[POST ? s : 0][POST ? b : 0][POST ? mm : 0][i];
                out[5 + i] = dt * acc;
            }
        }
    }
}

// R[l][col] = sum over the DOF's incidence list of the sub-tet contributions.
template <int N>
__global__ void __launch_bounds__(256) k_gather(DevGrid g, DevWork w) {
    constexpr int nc = Dim<N>::nc;
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= g.ndof * nc) return;
    const int64_t l = t / nc;
    const int col = int(t % nc);
    if (!w.active[g.dof_cell[l]]) return;
    double acc = 0.0;
    for (int e = g.inc_ptr[l]; e < g.inc_ptr[l + 1]; ++e) acc += w.rk[int64_t(g.inc_idx[e]) * nc + col];
    w.R[t] = acc;
}

// Y = M_i^{-1} X for every (active) cell, X and Y DOF-major with NC columns.
// One wave owns up to 256 rows of one cell (4 groups of 64 rows, lane-strided);
// M_i^{-1} is symmetric, so row j of the stored matrix supplies column j and
// the loads of one j are coalesced across the wave.  X[j][:] is uniform over
// the wave.  MODE 0: Y = S (predictor, active cells only);  MODE 1: add Y
// into the SoA state u (corrector, all cells).
template <int NC, int MODE>
__global__ void __launch_bounds__(256) k_minv(DevGrid g, const int32_t *__restrict__ active,
                                               const double *__restrict__ X, double *__restrict__ Y, int tpc) {
    const int lane = threadIdx.x % kWave;
    const int64_t id = int64_t(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int c = int(id / tpc);
    const int tile = int(id % tpc);
    if (c >= g.n_cells) return;
    if (MODE == 0 && !active[c]) return;
    const int64_t d0 = g.dof_ptr[c];
    const int n = int(g.dof_ptr[c + 1] - d0);
    const int r0 = tile * 256;
    if (r0 >= n) return;
    const int ng = min(4, (n - r0 + 63) / 64);
    const double *__restrict__ A = g.minv + g.minv_ptr[c];
    const double *__restrict__ B = X + d0 * NC;
    double acc[4][NC];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int col = 0; col < NC; ++col) acc[i][col] = 0.0;
    int row[4];
    bool ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        row[i] = r0 + 64 * i + lane;
        ok[i] = row[i] < n;
    }
    for (int j = 0; j < n; ++j) {
        double b[NC];
#pragma unroll
        for (int col = 0; col < NC; ++col) b[col] = B[int64_t(j) * NC + col];
        const double *Aj = A + int64_t(j) * n;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i < ng) {
                const double mij = ok[i] ? Aj[row[i]] : 0.0;
#pragma unroll
                for (int col = 0; col < NC; ++col) acc[i][col] = fma(mij, b[col], acc[i][col]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < ng && ok[i]) {
            if (MODE == 0) {
#pragma unroll
                for (int col = 0; col < NC; ++col) Y[(d0 + row[i]) * NC + col] = acc[i][col];
            } else {
#pragma unroll
                for (int col = 0; col < NC; ++col) Y[col * g.ndof + d0 + row[i]] += acc[i][col];
            }
        }
    }
}

// One block per active cell: G(x) = u - (K_tau^{-1} (x) I) S  (eq:ader4 after
// K_1^{-1} = K_tau^{-1} (x) M_i^{-1}), the residual test, and the Anderson
// update x <- G(x) - dG gamma, gamma = argmin |f - dF gamma|.  The history of
// difference pairs is append-only (restarted when full), so the Gram matrix of
// dF only gains a row per iteration; its Jacobi-scaled Cholesky factor is
// extended by one row, a column that adds no new direction is not appended.
// Depth 0 is the plain fixed-point map.
template <int N>
__global__ void __launch_bounds__(256) k_anderson(DevGrid g, DevWork w, const double *__restrict__ u, int it,
                                                   int max_iter, double tol) {
    constexpr int nc = Dim<N>::nc, nt = Dim<N>::nt;
    constexpr int kChunk = 4;  // elements per thread per chunk of the dot products
    __shared__ double red[2][4];
    __shared__ double accH[kMaxDepth + 1][4], accB[kMaxDepth + 1][4];
    __shared__ double gam_s[kMaxDepth];
    __shared__ int kuse_s;
    const int c = blockIdx.x;
    if (!w.active[c]) return;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid % kWave, wv = tid / kWave;
    const int nw = nth / kWave;
    const int64_t d0 = g.dof_ptr[c];
    const int n = int(g.dof_ptr[c + 1] - d0);
    const int64_t len = int64_t(n) * nc;
    const int64_t base = d0 * nc;
    const int64_t nd = g.ndof;
    double Ki[nt * nt];
    for (int i = 0; i < nt * nt; ++i) Ki[i] = g.ref->Ktau_inv[i];
    double fmx = 0.0, gmx = 0.0;
    for (int l = tid; l < n; l += nth) {
        double s[nc];
        for (int i = 0; i < nc; ++i) s[i] = w.S[base + int64_t(l) * nc + i];
        for (int b = 0; b < nt; ++b)
            for (int v = 0; v < 5; ++v) {
                double acc = 0.0;
                for (int a2 = 0; a2 < nt; ++a2) acc += Ki[b * nt + a2] * s[a2 * 5 + v];
                const double gv = u[v * nd + d0 + l] - acc;
                const int64_t idx = base + int64_t(l) * nc + b * 5 + v;
                const double fv = gv - w.x[idx];
                w.gcur[idx] = gv;
                w.fcur[idx] = fv;
                fmx = fmax(fmx, fabs(fv));
                gmx = fmax(gmx, fabs(gv));
            }
    }
    fmx = wave_max(fmx);
    gmx = wave_max(gmx);
    if (lane == 0) {
        red[0][wv] = fmx;
        red[1][wv] = gmx;
    }
    __syncthreads();
    double res = 0.0, gm = 0.0;
    for (int i = 0; i < nw; ++i) {
        res = fmax(res, red[0][i]);
        gm = fmax(gm, red[1][i]);
    }
    const int it1 = it + 1;
    const bool conv = res <= tol * fmax(1.0, gm);
    const bool last = it1 >= max_iter;
    const int depth = w.depth;
    if (conv || last || depth == 0 || it == 0) {
        for (int64_t i = tid; i < len; i += nth) {
            const double gv = w.gcur[base + i];
            w.x[base + i] = gv;
            if (!(conv || last)) {
                w.fprev[base + i] = w.fcur[base + i];
                w.gprev[base + i] = gv;
            }
        }
        if (tid == 0) {
            w.iters[c] = it1;
            w.hist[2 * c] = 0;
            if (conv || last) {
                w.active[c] = 0;
                atomicSub(&w.status[2], 1);
                if (!conv) {
                    atomicOr(&w.status[0], kStatusNoConv);
                    atomicMin(&w.status[1], c);
                }
            }
        }
        return;
    }
    int k = w.hist[2 * c];
    if (k >= depth) k = 0;  // restart with the newest pair only
    const int64_t hoff = base * depth;
    double *dF = w.dF + hoff;
    double *dG = w.dG + hoff;
    double *Lc = w.gram + int64_t(c) * kMaxDepth * kMaxDepth;  // Cholesky rows, row-major
    double *dsc = w.gram + int64_t(g.n_cells) * kMaxDepth * kMaxDepth + int64_t(c) * kMaxDepth;
    for (int j = tid; j <= k; j += nth) {
        accH[j][0] = accH[j][1] = accH[j][2] = accH[j][3] = 0.0;
        accB[j][0] = accB[j][1] = accB[j][2] = accB[j][3] = 0.0;
    }
    __syncthreads();
    // new difference pair (slot k) and the dots <dF_j, dF_new>, <dF_j, f>
    for (int64_t c0 = 0; c0 < len; c0 += int64_t(nth) * kChunk) {
        double fe[kChunk], dfe[kChunk];
        int64_t ie[kChunk];
#pragma unroll
        for (int e = 0; e < kChunk; ++e) {
            ie[e] = c0 + int64_t(e) * nth + tid;
            fe[e] = dfe[e] = 0.0;
            if (ie[e] < len) {
                const double f = w.fcur[base + ie[e]];
                const double dfn = f - w.fprev[base + ie[e]];
                fe[e] = f;
                dfe[e] = dfn;
                dF[int64_t(k) * len + ie[e]] = dfn;
                dG[int64_t(k) * len + ie[e]] = w.gcur[base + ie[e]] - w.gprev[base + ie[e]];
            }
        }
        for (int j = 0; j <= k; ++j) {
            double ph = 0.0, pb = 0.0;
#pragma unroll
            for (int e = 0; e < kChunk; ++e) {
                const double d = (j == k) ? dfe[e] : (ie[e] < len ? dF[int64_t(j) * len + ie[e]] : 0.0);
                ph = fma(d, dfe[e], ph);
                pb = fma(d, fe[e], pb);
            }
            ph = wave_sum(ph);
            pb = wave_sum(pb);
            if (lane == 0) {
                accH[j][wv] += ph;
                accB[j][wv] += pb;
            }
        }
    }
    __syncthreads();
    if (wv == 0) {
        // one wave: extend the scaled Cholesky factor by row k, solve for gamma
        const double hkk = accH[k][0] + accH[k][1] + accH[k][2] + accH[k][3];
        const double dk = hkk > 0.0 ? 1.0 / sqrt(hkk) : 0.0;
        // lane j holds entries of index j (k <= kMaxDepth - 1 < 64)
        const double hj = (lane < k) ? (accH[lane][0] + accH[lane][1] + accH[lane][2] + accH[lane][3]) : 0.0;
        const double dj = (lane < k) ? dsc[lane] : 0.0;
        const double rhs = hj * dj * dk;  // scaled Gram row
        double y = 0.0;                   // solve L[0:k,0:k] y = rhs by forward substitution
        for (int i = 0; i < k; ++i) {
            const double lij = (lane < i) ? Lc[i * kMaxDepth + lane] : 0.0;
            const double s = wave_sum(lij * y);
            const double yi = (__shfl(rhs, i, kWave) - s) / Lc[i * kMaxDepth + i];
            if (lane == i) y = yi;
        }
        const double ysq = wave_sum(lane < k ? y * y : 0.0);
        const double diag = 1.0 + 1e-12 - ysq;
        const bool add = (hkk > 0.0) && (diag > 1e-10);
        const int kuse = add ? k + 1 : k;
        if (add) {
            if (lane < k) Lc[k * kMaxDepth + lane] = y;
            if (lane == 0) {
                Lc[k * kMaxDepth + k] = sqrt(diag);
                dsc[k] = dk;
            }
        }
        __threadfence_block();
        // gamma: (D H D + reg) z = D b, gamma = D z
        const double bj = (lane < kuse) ? (accB[lane][0] + accB[lane][1] + accB[lane][2] + accB[lane][3]) *
                                              ((lane == k) ? dk : dsc[lane < k ? lane : 0])
                                        : 0.0;
        double z = 0.0;
        for (int i = 0; i < kuse; ++i) {
            const double lij = (lane < i) ? ((i == k && add) ? y : Lc[i * kMaxDepth + lane]) : 0.0;
            const double s = wave_sum(lij * z);
            const double lii = (i == k && add) ? sqrt(diag) : Lc[i * kMaxDepth + i];
            const double zi = (__shfl(bj, i, kWave) - s) / lii;
            if (lane == i) z = zi;
        }
        double x = 0.0;
        for (int i = kuse - 1; i >= 0; --i) {
            // L^T x = z: x_i = (z_i - sum_{j > i} L[j][i] x_j) / L[i][i]
            const double yi_new = __shfl(y, i, kWave);  // L[k][i] of the new row
            const double lji = (lane > i && lane < kuse) ? ((lane == k && add) ? yi_new : Lc[lane * kMaxDepth + i]) : 0.0;
            const double s = wave_sum(lji * x);
            const double lii = (i == k && add) ? sqrt(diag) : Lc[i * kMaxDepth + i];
            const double xi = (__shfl(z, i, kWave) - s) / lii;
            if (lane == i) x = xi;
        }
        if (lane < kuse) gam_s[lane] = x * ((lane == k) ? dk : dsc[lane < k ? lane : 0]);
        if (lane == 0) {
            kuse_s = kuse;
            w.hist[2 * c] = kuse;
            w.iters[c] = it1;
        }
    }
    __syncthreads();
    const int kuse = kuse_s;
    for (int64_t i = tid; i < len; i += nth) {
        double xv = w.gcur[base + i];
        for (int j = 0; j < kuse; ++j) xv -= gam_s[j] * dG[int64_t(j) * len + i];
        w.x[base + i] = xv;
        w.fprev[base + i] = w.fcur[base + i];
        w.gprev[base + i] = w.gcur[base + i];
    }
}

// ------------------------------------------------------------- corrector

// Rusanov flux with viscous penalty (eq. 3.33) at the face nodes of every
// boundary sub-triangle, contracted with the face mass: fc[k][j'] =
// 2 A_k sum_j Z^[j'][j] G_j.  One value of the dissipation coefficient per
// sub-triangle: the maximum over its nodes and both sides.
template <int N>
__global__ void __launch_bounds__(256) k_face(DevGrid g, DevWork w, double dt) {
    constexpr int nf = Dim<N>::nf;
    constexpr int tpb = 256 / nf;
    __shared__ double lam_s[tpb][nf], lamv_s[tpb][nf];
    __shared__ double G_s[tpb][nf][5];
    const int t = threadIdx.x / nf, j = threadIdx.x % nf;
    const int64_t k = int64_t(blockIdx.x) * tpb + t;
    const bool valid = t < tpb && k < g.nsub;
    double Gv[5] = {0, 0, 0, 0, 0};
    double nrm[3] = {0, 0, 0}, a2 = 0.0;
    double eps = 0.0;
    if (valid) {
        const int64_t kn = g.nbr_sub[k];
        const int jn = g.perm[k * nf + j];
        const double *ti = w.trace + (k * nf + j) * 20;
        const double *to = w.trace + (kn * nf + jn) * 20;
        const double *T = g.tri + k * 4;
        a2 = T[0];
        nrm[0] = T[1];
        nrm[1] = T[2];
        nrm[2] = T[3];
        const int ci = g.sub_cell[k], co = g.sub_cell[kn];
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
        lamv_s[t][j] = fmax(4.0 * w.mu_cell[ci] / (3.0 * qi[0]), 4.0 * w.mu_cell[co] / (3.0 * qo[0]));
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
__global__ void __launch_bounds__(256) k_rhs(DevGrid g, DevWork w) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= g.ndof * 5) return;
    const int64_t l = t / 5;
    const int v = int(t % 5);
    double acc = 0.0;
    for (int e = g.inc_ptr[l]; e < g.inc_ptr[l + 1]; ++e) acc += w.vk[int64_t(g.inc_idx[e]) * 5 + v];
    double fac = 0.0;
    for (int e = g.finc_ptr[l]; e < g.finc_ptr[l + 1]; ++e) fac += w.fc[int64_t(g.finc_idx[e]) * 5 + v];
    w.rhs[t] = acc - fac;
}

__global__ void k_reset_status(DevWork w, int n_cells) {
    if (threadIdx.x == 0) {
        w.status[0] = 0;
        w.status[1] = INT_MAX;
        w.status[2] = n_cells;
        w.status[3] = 0;
    }
}

__global__ void k_positivity(DevGrid g, DevWork w, const double *__restrict__ u) {
    const int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (l >= g.ndof) return;
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

template <typename F>
hipError_t dispatch(int N, F &&f) {
    switch (N) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
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
    size_t shmem = size_t(3) * g.max_cell_dofs * sizeof(double);
    hipLaunchKernelGGL(k_mass_invert, dim3(g.n_cells), dim3(1024), shmem, s, g);
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

hipError_t launch_cfl_max(const DevGrid &g, const DevWork &w, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl_max, dim3(1), dim3(1024), 0, s, g.n_cells, w.cflterm, out);
    return hipGetLastError();
}

hipError_t launch_pred_init(const DevGrid &g, const DevWork &w, const double *u, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        int64_t m = g.ndof > g.n_cells ? g.ndof : g.n_cells;
        hipLaunchKernelGGL(k_pred_init<decltype(n)::value>, dim3(blocks_for(m, 256)), dim3(256), 0, s, g, w, u);
        return hipGetLastError();
    });
}

hipError_t launch_pred_iteration(const DevGrid &g, const DevWork &w, const double *u, double dt, int it,
                                 int max_iter, double tol, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        hipLaunchKernelGGL((k_subtet<NN, false>), dim3(blocks_for(g.nsub, D::spb)), dim3(D::threads), 0, s, g, w, dt);
        hipLaunchKernelGGL(k_gather<NN>, dim3(blocks_for(g.ndof * D::nc, 256)), dim3(256), 0, s, g, w);
        const int tpc = (g.max_cell_dofs + 255) / 256;
        hipLaunchKernelGGL((k_minv<D::nc, 0>), dim3(blocks_for(int64_t(g.n_cells) * tpc, 4)), dim3(256), 0, s, g,
                           w.active, w.R, w.S, tpc);
        hipLaunchKernelGGL(k_anderson<NN>, dim3(g.n_cells), dim3(256), 0, s, g, w, u, it, max_iter, tol);
        return hipGetLastError();
    });
}

hipError_t launch_pred_post(const DevGrid &g, const DevWork &w, double dt, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        hipLaunchKernelGGL((k_subtet<NN, true>), dim3(blocks_for(g.nsub, D::spb)), dim3(D::threads), 0, s, g, w, dt);
        return hipGetLastError();
    });
}

hipError_t launch_correct(const DevGrid &g, const DevWork &w, double *u, double dt, hipStream_t s) {
    return dispatch(g.N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        using D = Dim<NN>;
        hipLaunchKernelGGL(k_face<NN>, dim3(blocks_for(g.nsub, 256 / D::nf)), dim3(256), 0, s, g, w, dt);
        hipLaunchKernelGGL(k_rhs<NN>, dim3(blocks_for(g.ndof * 5, 256)), dim3(256), 0, s, g, w);
        const int tpc = (g.max_cell_dofs + 255) / 256;
        hipLaunchKernelGGL((k_minv<5, 1>), dim3(blocks_for(int64_t(g.n_cells) * tpc, 4)), dim3(256), 0, s, g,
                           w.active, w.rhs, u, tpc);
        hipLaunchKernelGGL(k_positivity, dim3(blocks_for(g.ndof, 256)), dim3(256), 0, s, g, w, u);
        return hipGetLastError();
    });
}

}  // namespace afe
