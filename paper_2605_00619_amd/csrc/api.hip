// C ABI of libafe (see include/afe.h): object life cycle, buffers, and the
// host-side sequencing of the step kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/afe.h"
#include "device.hpp"
#include "refelem.hpp"
#include "subgrid.hpp"

namespace {

thread_local std::string g_err;

afe_status fail(afe_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(AFE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct afe_cell_data {
    afe::HostGrid host;
    afe::DevGrid g{};
    afe::DevWork w{};
    afe_params params{};
    std::vector<void *> allocs;
    size_t bytes = 0;
    double *d_scalar = nullptr;  // device scratch scalar (CFL max)
    int32_t *h_status = nullptr; // pinned host copy of the status word
    double *h_scalar = nullptr;
    // profiling of the predictor's M^{-1} kernel
    bool prof_on = false;
    afe::ProfileHooks hooks{};
    unsigned long long *h_bytes = nullptr;
    double prof_ms = 0.0;
    int64_t prof_launches = 0;

    template <typename T>
    hipError_t alloc(T *&p, size_t count) {
        void *v = nullptr;
        size_t b = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc(&v, b);
        if (e == hipSuccess) {
            allocs.push_back(v);
            bytes += b;
            p = static_cast<T *>(v);
        }
        return e;
    }
    template <typename T>
    hipError_t upload(const T *&dst, const std::vector<T> &src, hipStream_t s) {
        T *p = nullptr;
        hipError_t e = alloc(p, src.size());
        if (e != hipSuccess) return e;
        dst = p;
        if (!src.empty()) e = hipMemcpyAsync(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
        return e;
    }
    ~afe_cell_data() {
        for (int i = 0; i < afe::kSyncEvery; ++i) {
            if (hooks.start[i]) (void)hipEventDestroy(hooks.start[i]);
            if (hooks.stop[i]) (void)hipEventDestroy(hooks.stop[i]);
        }
        if (h_bytes) (void)hipHostFree(h_bytes);
        for (void *p : allocs) (void)hipFree(p);
        if (h_status) (void)hipHostFree(h_status);
        if (h_scalar) (void)hipHostFree(h_scalar);
    }
};

namespace {

size_t estimate_bytes(const afe::HostGrid &h, int depth, bool mixed) {
    const size_t nc = size_t(5) * (h.N + 1);
    size_t b = 0;
    for (int c = 0; c < h.n_cells; ++c) {
        size_t n = size_t(h.dof_ptr[c + 1] - h.dof_ptr[c]);
        b += n * ((n + 15) & ~size_t(15)) * sizeof(double);
        if (mixed) b += n * ((n + 31) & ~size_t(31)) * sizeof(float);
    }
    b += size_t(h.ndof) * nc * sizeof(double) * (5 + 2 * size_t(std::max(depth, 1)));
    b += size_t(h.n_cells) * ((h.max_cell_dofs + 63) / 64) * 130 * sizeof(double);
    b += size_t(h.nsub) * h.np * nc * sizeof(double);
    b += size_t(h.nsub) * h.nf * 25 * sizeof(double) + size_t(h.nsub) * h.np * 5 * sizeof(double);
    b += size_t(h.ndof) * (5 * 8 + 3 * 8 + 8 + 4 + 8);
    b += size_t(h.nsub) * (h.np * 4 + 10 * 8 + 4 * 8 + 4 + 4 + h.nf * 4);
    b += size_t(h.n_cells) * ((2 * 63 * 63 + 63) * 8 + 64);
    return b;
}

}  // namespace

extern "C" {

const char *afe_last_error(void) { return g_err.c_str(); }

void afe_free(afe_cell_data *cd) { delete cd; }

afe_status build_afe_cell_data(const afe_mesh *mesh, int32_t N, const afe_params *params, void *stream,
                               afe_cell_data **out) {
    if (!mesh || !params || !out) return fail(AFE_E_ARG, "null argument");
    *out = nullptr;
    if (params->precision != AFE_FP64 && params->precision != AFE_MIXED) return fail(AFE_E_ARG, "unknown precision");
    if (params->accel_depth < 0 || params->accel_depth > 63) return fail(AFE_E_ARG, "accel_depth must be in [0, 63]");
    if (params->max_iter < 1) return fail(AFE_E_ARG, "max_iter must be >= 1");
    if (!(params->gamma > 1.0) || params->mu < 0.0 || !(params->tol >= 0.0))
        return fail(AFE_E_ARG, "invalid physics or tolerance parameter");
    hipStream_t s = static_cast<hipStream_t>(stream);
    afe_cell_data *cd = new (std::nothrow) afe_cell_data();
    if (!cd) return fail(AFE_E_ARG, "out of host memory");
    std::string err;
    afe_status st = afe::build_host_grid(*mesh, N, cd->host, err);
    if (st != AFE_OK) {
        delete cd;
        return fail(st, err);
    }
    cd->params = *params;
    const afe::HostGrid &h = cd->host;
    const int depth = params->accel_depth;
    size_t need = estimate_bytes(h, depth, params->precision == AFE_MIXED);
    if (params->hbm_budget > 0 && need > params->hbm_budget) {
        delete cd;
        return fail(AFE_E_HBM_BUDGET, "needs " + std::to_string(need) + " bytes, budget " +
                                          std::to_string(params->hbm_budget));
    }
    auto &g = cd->g;
    auto &w = cd->w;
    g.N = N;
    g.np = h.np;
    g.nf = h.nf;
    g.nt = N + 1;
    g.nc = 5 * (N + 1);
    g.n_cells = h.n_cells;
    g.ndof = h.ndof;
    g.nsub = h.nsub;
    g.max_cell_dofs = h.max_cell_dofs;
    g.max_cell_subtets = h.max_cell_subtets;
    g.gamma = params->gamma;
    g.mu = params->mu;
    g.m1 = params->m1;
    g.av = params->av;
    g.mixed = params->precision == AFE_MIXED ? 1 : 0;
    std::vector<int64_t> minv_ptr(h.n_cells + 1, 0), minv32_ptr(h.n_cells + 1, 0);
    for (int c = 0; c < h.n_cells; ++c) {
        int64_t n = h.dof_ptr[c + 1] - h.dof_ptr[c];
        minv_ptr[c + 1] = minv_ptr[c] + n * ((n + 15) & ~int64_t(15));  // rows padded to 128 bytes
        minv32_ptr[c + 1] = minv32_ptr[c] + (g.mixed ? n * ((n + 31) & ~int64_t(31)) : 0);
    }
    hipError_t e;
    if ((e = cd->upload(g.dof_ptr, h.dof_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.sub_ptr, h.sub_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.minv_ptr, minv_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.minv32_ptr, minv32_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.conn, h.conn, s)) != hipSuccess ||
        (e = cd->upload(g.sub_cell, h.sub_cell, s)) != hipSuccess ||
        (e = cd->upload(g.geo, h.geo, s)) != hipSuccess ||
        (e = cd->upload(g.tri, h.tri, s)) != hipSuccess ||
        (e = cd->upload(g.nbr_sub, h.nbr_sub, s)) != hipSuccess ||
        (e = cd->upload(g.perm, h.perm, s)) != hipSuccess ||
        (e = cd->upload(g.h, h.h, s)) != hipSuccess ||
        (e = cd->upload(g.vol, h.vol, s)) != hipSuccess ||
        (e = cd->upload(g.mrow, h.mrow, s)) != hipSuccess ||
        (e = cd->upload(g.dof_cell, h.dof_cell, s)) != hipSuccess ||
        (e = cd->upload(g.inc_ptr, h.inc_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.inc_idx, h.inc_idx, s)) != hipSuccess ||
        (e = cd->upload(g.finc_ptr, h.finc_ptr, s)) != hipSuccess ||
        (e = cd->upload(g.finc_idx, h.finc_idx, s)) != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete cd;
        return fail(AFE_E_HIP, "upload: " + m);
    }
    // reference data
    const afe::RefData &R = afe::ref_data(N);
    afe::DevRef ref{};
    for (int i = 0; i < R.np * R.np; ++i) ref.M[i] = R.M[i];
    for (int i = 0; i < 3 * R.np * R.np; ++i) {
        ref.K[i] = R.K[i];
        ref.D[i] = R.D[i];
    }
    for (int i = 0; i < R.nf * R.nf; ++i) ref.Z[i] = R.Z[i];
    for (int j = 0; j < R.nf; ++j) {
        double sacc = 0.0;
        for (int i = 0; i < R.nf; ++i) sacc += R.Z[i * R.nf + j];
        ref.zsum[j] = sacc;
        ref.fn[j] = R.face_nodes[j];
    }
    for (int a = 0; a < R.nt; ++a) ref.w[a] = R.w[a];
    for (int i = 0; i < R.nt * R.nt; ++i) {
        ref.Ktau_inv[i] = R.Ktau_inv[i];
        ref.Ktau[i] = R.Ktau[i];
    }
    afe::DevRef *dref = nullptr;
    if ((e = cd->alloc(dref, 1)) != hipSuccess || (e = hipMemcpyAsync(dref, &ref, sizeof(ref), hipMemcpyHostToDevice, s)) != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete cd;
        return fail(AFE_E_HIP, "reference upload: " + m);
    }
    g.ref = dref;
    const size_t nc = size_t(g.nc);
    const size_t nd = size_t(h.ndof);
    const int dslots = std::max(depth, 1);
    w.depth = depth;
    if ((e = cd->alloc(g.minv, size_t(minv_ptr[h.n_cells]))) != hipSuccess ||
        (e = cd->alloc(g.dscale, nd)) != hipSuccess ||
        (e = cd->alloc(g.minv32, size_t(minv32_ptr[h.n_cells]))) != hipSuccess ||
        (e = cd->alloc(w.R32, g.mixed ? nd * nc : 1)) != hipSuccess ||
        (e = cd->alloc(w.x, nd * nc)) != hipSuccess || (e = cd->alloc(w.R, nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.S, nd * nc)) != hipSuccess || (e = cd->alloc(w.fprev, nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.gprev, nd * nc)) != hipSuccess || 
        (e = cd->alloc(w.part, size_t(h.n_cells) * ((h.max_cell_dofs + 63) / 64) * 130)) != hipSuccess ||
        (e = cd->alloc(w.gamma, size_t(h.n_cells) * 63)) != hipSuccess ||
        (e = cd->alloc(w.kuse, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.dF, nd * nc * dslots)) != hipSuccess ||
        (e = cd->alloc(w.dG, nd * nc * dslots)) != hipSuccess ||
        (e = cd->alloc(w.gram, size_t(h.n_cells) * (2 * 63 * 63 + 63))) != hipSuccess ||
        (e = cd->alloc(w.hist, size_t(h.n_cells) * 2)) != hipSuccess ||
        (e = cd->alloc(w.rk, size_t(h.nsub) * h.np * nc)) != hipSuccess ||
        (e = cd->alloc(w.trace, size_t(h.nsub) * h.nf * 20)) != hipSuccess ||
        (e = cd->alloc(w.vk, size_t(h.nsub) * h.np * 5)) != hipSuccess ||
        (e = cd->alloc(w.fc, size_t(h.nsub) * h.nf * 5)) != hipSuccess ||
        (e = cd->alloc(w.rhs, nd * 5)) != hipSuccess ||
        (e = cd->alloc(w.mu_cell, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.beta, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.cflterm, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.alist, size_t(h.n_cells) * 2)) != hipSuccess ||
        (e = cd->alloc(w.acount, 2)) != hipSuccess ||
        (e = cd->alloc(w.iters, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.status, 4)) != hipSuccess || (e = cd->alloc(cd->d_scalar, 1)) != hipSuccess ||
        (e = hipHostMalloc(&cd->h_status, 4 * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(&cd->h_scalar, sizeof(double), hipHostMallocDefault)) != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete cd;
        return fail(e == hipErrorOutOfMemory ? AFE_E_HBM_BUDGET : AFE_E_HIP, "allocation: " + m);
    }
    // zero the per-cell viscosity so a predictor without a prior detector is Euler
    if ((e = hipMemsetAsync(w.mu_cell, 0, sizeof(double) * h.n_cells, s)) != hipSuccess ||
        (e = afe::launch_reset_status(g, w, s)) != hipSuccess || (e = afe::launch_mass_assemble(g, s)) != hipSuccess ||
        (e = afe::launch_mass_invert(g, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete cd;
        return fail(AFE_E_HIP, "mass matrices: " + m);
    }
    *out = cd;
    return AFE_OK;
}

afe_status afe_query(const afe_cell_data *cd, afe_info *out) {
    if (!cd || !out) return fail(AFE_E_ARG, "null argument");
    out->ndof = cd->host.ndof;
    out->n_cells = cd->host.n_cells;
    out->n_subtets = cd->host.nsub;
    out->N = cd->host.N;
    out->max_cell_dofs = cd->host.max_cell_dofs;
    out->max_cell_subtets = cd->host.max_cell_subtets;
    out->device_bytes = cd->bytes;
    out->h_min = cd->host.h_min;
    return AFE_OK;
}

afe_status afe_cell_dof_ptr(const afe_cell_data *cd, int64_t *p) {
    if (!cd || !p) return fail(AFE_E_ARG, "null argument");
    std::memcpy(p, cd->host.dof_ptr.data(), cd->host.dof_ptr.size() * sizeof(int64_t));
    return AFE_OK;
}

afe_status afe_dof_coords(const afe_cell_data *cd, double *xyz, void *stream) {
    if (!cd || !xyz) return fail(AFE_E_ARG, "null argument");
    HIP_TRY(hipMemcpyAsync(xyz, cd->host.dof_x.data(), cd->host.dof_x.size() * sizeof(double), hipMemcpyHostToDevice,
                           static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return AFE_OK;
}

afe_status afe_connectivity(const afe_cell_data *cd, int64_t *subtet_ptr, int32_t *conn, int32_t *nbr_subtet,
                            int32_t *nbr_perm) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    const auto &h = cd->host;
    if (subtet_ptr) std::memcpy(subtet_ptr, h.sub_ptr.data(), h.sub_ptr.size() * sizeof(int64_t));
    if (conn) std::memcpy(conn, h.conn.data(), h.conn.size() * sizeof(int32_t));
    if (nbr_subtet) std::memcpy(nbr_subtet, h.nbr_sub.data(), h.nbr_sub.size() * sizeof(int32_t));
    if (nbr_perm) std::memcpy(nbr_perm, h.perm.data(), h.perm.size() * sizeof(int32_t));
    return AFE_OK;
}

afe_status afe_subgrid_sizes(const afe_mesh *mesh, int32_t N, int64_t *sizes) {
    if (!mesh || !sizes) return fail(AFE_E_ARG, "null argument");
    afe::HostGrid h;
    std::string err;
    afe_status st = afe::build_host_grid(*mesh, N, h, err);
    if (st != AFE_OK) return fail(st, err);
    sizes[0] = h.nsub;
    sizes[1] = h.ndof;
    return AFE_OK;
}

afe_status afe_subgrid_host(const afe_mesh *mesh, int32_t N, int64_t *subtet_ptr, int64_t *dof_ptr, int32_t *conn,
                            int32_t *nbr_subtet, int32_t *nbr_perm, double *geo, double *tri) {
    if (!mesh) return fail(AFE_E_ARG, "null argument");
    afe::HostGrid h;
    std::string err;
    afe_status st = afe::build_host_grid(*mesh, N, h, err);
    if (st != AFE_OK) return fail(st, err);
    if (subtet_ptr) std::memcpy(subtet_ptr, h.sub_ptr.data(), h.sub_ptr.size() * sizeof(int64_t));
    if (dof_ptr) std::memcpy(dof_ptr, h.dof_ptr.data(), h.dof_ptr.size() * sizeof(int64_t));
    if (conn) std::memcpy(conn, h.conn.data(), h.conn.size() * sizeof(int32_t));
    if (nbr_subtet) std::memcpy(nbr_subtet, h.nbr_sub.data(), h.nbr_sub.size() * sizeof(int32_t));
    if (nbr_perm) std::memcpy(nbr_perm, h.perm.data(), h.perm.size() * sizeof(int32_t));
    if (geo) std::memcpy(geo, h.geo.data(), h.geo.size() * sizeof(double));
    if (tri) std::memcpy(tri, h.tri.data(), h.tri.size() * sizeof(double));
    return AFE_OK;
}

afe_status afe_prim_to_cons(afe_cell_data *cd, const double *prim, double *u, void *stream) {
    if (!cd || !prim || !u) return fail(AFE_E_ARG, "null argument");
    HIP_TRY(afe::launch_prim_to_cons(cd->g, prim, u, static_cast<hipStream_t>(stream)));
    return AFE_OK;
}

afe_status ader_cfl_dt(afe_cell_data *cd, const double *u, double cfl, double *dt_host, void *stream) {
    if (!cd || !u || !dt_host || !(cfl > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(afe::launch_reset_status(cd->g, cd->w, s));
    HIP_TRY(afe::launch_detect(cd->g, cd->w, u, s));
    HIP_TRY(afe::launch_cfl_max(cd->g, cd->w, cd->d_scalar, s));
    HIP_TRY(hipMemcpyAsync(cd->h_scalar, cd->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double smax = *cd->h_scalar;
    if (!(smax > 0.0) || !std::isfinite(smax)) return fail(AFE_E_NONFINITE, "non-finite wave speed");
    *dt_host = cfl * cd->host.h_min / ((2 * cd->host.N + 1) * smax);
    return AFE_OK;
}

afe_status ader_predict(afe_cell_data *cd, const double *u, double dt, void *stream) {
    if (!cd || !u || !(dt > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto &p = cd->params;
    HIP_TRY(afe::launch_reset_status(cd->g, cd->w, s));
    HIP_TRY(afe::launch_detect(cd->g, cd->w, u, s));
    HIP_TRY(afe::launch_pred_init(cd->g, cd->w, u, s));
    // Iterations are launched in batches of kSyncEvery without waiting: the
    // kernels read the current list length on the device and idle blocks exit,
    // the host only needs an upper bound, refreshed at each synchronisation.
    int n_upper = cd->host.n_cells;
    for (int it = 0; it < p.max_iter && n_upper > 0;) {
        // large lists shrink fast: synchronise every iteration until few cells remain
        const int batch_len = n_upper > 256 ? 1 : afe::kSyncEvery;
        int batch = 0;
        for (; batch < batch_len && it < p.max_iter; ++batch, ++it) {
            const int cur = it % 2, nxt = 1 - cur;
            int32_t *list = cd->w.alist + size_t(cur) * cd->host.n_cells;
            int32_t *next = cd->w.alist + size_t(nxt) * cd->host.n_cells;
            HIP_TRY(afe::launch_pred_iteration(cd->g, cd->w, u, dt, it, p.max_iter, p.tol, list, cd->w.acount + cur,
                                               n_upper, next, cd->w.acount + nxt, s,
                                               cd->prof_on ? cd->hooks.start[batch] : nullptr,
                                               cd->prof_on ? cd->hooks.stop[batch] : nullptr,
                                               cd->prof_on ? cd->hooks.bytes : nullptr));
        }
        HIP_TRY(hipMemcpyAsync(cd->h_status + 2, cd->w.acount + (it % 2), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        n_upper = cd->h_status[2];
        if (cd->prof_on) {
            for (int b = 0; b < batch; ++b) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, cd->hooks.start[b], cd->hooks.stop[b]));
                cd->prof_ms += ms;
                cd->prof_launches += 1;
            }
        }
    }
    HIP_TRY(afe::launch_pred_post(cd->g, cd->w, dt, s));
    return AFE_OK;
}

afe_status ader_correct(afe_cell_data *cd, double *u, double dt, void *stream) {
    if (!cd || !u || !(dt > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    HIP_TRY(afe::launch_correct(cd->g, cd->w, u, dt, static_cast<hipStream_t>(stream)));
    return AFE_OK;
}

afe_status ader_step(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, void *stream) {
    afe_status st = ader_predict(cd, u, dt, stream);
    if (st != AFE_OK) return st;
    st = ader_correct(cd, u, dt, stream);
    if (st != AFE_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(cd->h_status, cd->w.status, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int flags = cd->h_status[0];
    if (rep) {
        std::vector<int32_t> it(cd->host.n_cells);
        HIP_TRY(hipMemcpy(it.data(), cd->w.iters, it.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        int mn = INT_MAX, mx = 0;
        double sum = 0.0;
        for (int v : it) {
            mn = std::min(mn, v);
            mx = std::max(mx, v);
            sum += v;
        }
        rep->iters_min = it.empty() ? 0 : mn;
        rep->iters_max = mx;
        rep->iters_mean = it.empty() ? 0.0 : sum / double(it.size());
        rep->n_troubled = cd->h_status[3];
        rep->status_cell = flags ? cd->h_status[1] : -1;
    }
    if (flags & afe::kStatusNonfinite) return fail(AFE_E_NONFINITE, "non-finite state after the update");
    if (flags & afe::kStatusNoConv) return fail(AFE_E_NO_CONVERGENCE, "predictor did not converge");
    if (flags & afe::kStatusPositivity) return fail(AFE_E_POSITIVITY, "density or pressure not positive");
    return AFE_OK;
}

afe_status afe_profile_enable(afe_cell_data *cd, int32_t enable) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    if (enable && !cd->hooks.bytes) {
        for (int i = 0; i < afe::kSyncEvery; ++i) {
            HIP_TRY(hipEventCreate(&cd->hooks.start[i]));
            HIP_TRY(hipEventCreate(&cd->hooks.stop[i]));
        }
        HIP_TRY(cd->alloc(cd->hooks.bytes, 1));
    }
    cd->prof_on = enable != 0;
    cd->prof_ms = 0.0;
    cd->prof_launches = 0;
    if (cd->hooks.bytes) HIP_TRY(hipMemset(cd->hooks.bytes, 0, sizeof(unsigned long long)));
    return AFE_OK;
}

afe_status afe_profile_read(afe_cell_data *cd, double *kernel_ms, int64_t *launches, double *bytes) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    unsigned long long b = 0;
    if (cd->hooks.bytes) HIP_TRY(hipMemcpy(&b, cd->hooks.bytes, sizeof(b), hipMemcpyDeviceToHost));
    if (kernel_ms) *kernel_ms = cd->prof_ms;
    if (launches) *launches = cd->prof_launches;
    if (bytes) *bytes = double(b);
    return AFE_OK;
}

afe_status afe_predictor_state(const afe_cell_data *cd, double *q, void *stream) {
    if (!cd || !q) return fail(AFE_E_ARG, "null argument");
    HIP_TRY(hipMemcpyAsync(q, cd->w.x, size_t(cd->host.ndof) * cd->g.nc * sizeof(double), hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    return AFE_OK;
}

afe_status afe_cell_diagnostics(const afe_cell_data *cd, int32_t *iters, double *mu, void *stream) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s));
    if (iters) HIP_TRY(hipMemcpy(iters, cd->w.iters, sizeof(int32_t) * cd->host.n_cells, hipMemcpyDeviceToHost));
    if (mu) HIP_TRY(hipMemcpy(mu, cd->w.mu_cell, sizeof(double) * cd->host.n_cells, hipMemcpyDeviceToHost));
    return AFE_OK;
}

}  // extern "C"
