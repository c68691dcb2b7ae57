// C ABI of libafe (see include/afe.h): object life cycle, buffers, and the
// host-side sequencing of the step kernels for one simulation or a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
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

#define AFE_TRY(expr)                \
    do {                             \
        afe_status s_ = (expr);      \
        if (s_ != AFE_OK) return s_; \
    } while (0)

constexpr int kStatusWords = 8;

// One group of slots with the same degree, precision and viscosity (physical
// or artificial, or none): they share the predictor's launches through one
// list of (slot, cell) entries.  A simulation always runs the same kernel
// instances, whatever it is batched with, so its results do not depend on
// its batch-mates.
struct Group {
    int N = 0, mixed = 0;
    int visc = 0;
    std::vector<int> slots;
    std::vector<int64_t> base;  // list offset of each slot's cells
    int64_t cells = 0;
    int max_cell_dofs = 0, max_cell_subtets = 0;
    int32_t *lists = nullptr;   // device [2][cells] (ping-pong)
    int32_t *counts = nullptr;  // device [2]
    afe::IterShape resident;    // workgroups that fit at once, per kernel
    afe::IterShape shape;       // grids in use
};

// Sequencing of the step kernels over a set of slots.  A cell-data object
// owns an engine with itself as its only slot; a batch owns one with many.
struct Engine {
    afe::DevSlot *d_tab = nullptr;     // device table [kMaxSlots]
    std::vector<afe::DevSlot> tab;     // host image of the table
    std::vector<afe_cell_data *> cds;  // slot -> object (nullptr: free)
    std::vector<double *> u;           // slot -> state
    std::vector<double> cfl;           // slot -> CFL number (batch steps)
    std::vector<Group> groups;
    bool dirty = true;                 // table or grouping changed since the last upload
    afe_launch_shape shape{1.0, 0.0, 0.0, 2, 0};  // the tuner's usual choice
    int32_t *h_counts = nullptr;       // pinned [kMaxSlots]
    hipStream_t own = nullptr;         // private stream (graph capture needs a non-null stream)
    hipEvent_t join[2] = {nullptr, nullptr};
    // early time-integral pass: once few cells still iterate, the time
    // integrals of the converged ones run on a side stream under the tail
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_early = nullptr;
    bool forked = false;
    // early corrector: the caller steps u in full (not a predictor-only call)
    bool allow_correct = false;
    // batch_step_on reached the per-slot reports of this call
    bool reported = false;
    // early passes on a side stream allowed (off for the allocation-free step)
    bool side_ok = true;
    bool forked2 = false;
    hipGraphExec_t g_pre = nullptr, g_post = nullptr, g_chunk[2] = {nullptr, nullptr};
    // profiling of the first group's M^{-1} launches
    bool prof_on = false;
    afe::ProfileHooks hooks{};
    unsigned long long *d_bytes = nullptr;
    double prof_ms = 0.0;
    int64_t prof_launches = 0;

    Engine() : tab(afe::kMaxSlots), cds(afe::kMaxSlots, nullptr), u(afe::kMaxSlots, nullptr), cfl(afe::kMaxSlots, 0.0) {}
    ~Engine() {
        drop_graphs();
        drop_groups();
        for (int i = 0; i < afe::kMaxRounds; ++i) {
            if (hooks.start[i]) (void)hipEventDestroy(hooks.start[i]);
            if (hooks.stop[i]) (void)hipEventDestroy(hooks.stop[i]);
        }
        if (d_bytes) (void)hipFree(d_bytes);
        if (d_tab) (void)hipFree(d_tab);
        if (h_counts) (void)hipHostFree(h_counts);
        for (auto &e : join)
            if (e) (void)hipEventDestroy(e);
        if (own) (void)hipStreamDestroy(own);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_early) (void)hipEventDestroy(ev_early);
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
    }
    void drop_graphs() {
        for (hipGraphExec_t *g : {&g_pre, &g_post, &g_chunk[0], &g_chunk[1]})
            if (*g) {
                (void)hipGraphExecDestroy(*g);
                *g = nullptr;
            }
    }
    void drop_groups() {
        for (auto &gr : groups) {
            if (gr.lists) (void)hipFree(gr.lists);
            if (gr.counts) (void)hipFree(gr.counts);
        }
        groups.clear();
    }
    int n_slots() const {
        int n = 0;
        for (auto *c : cds) n += c != nullptr;
        return n;
    }
};

}  // namespace

struct afe_cell_data {
    afe::HostGrid host;
    afe::DevGrid g{};
    afe::DevWork w{};
    afe_params params{};
    std::vector<void *> allocs;
    size_t bytes = 0;
    double *d_scalar = nullptr;  // device scratch scalar (largest CFL term)
    int32_t *h_status = nullptr; // pinned host copy of the status words
    double *h_scalar = nullptr;  // pinned host scalars [2]: largest CFL term, dt
    int32_t *h_counts = nullptr; // pinned host list lengths of the allocation-free step
    int device = 0;              // device the object's memory lives on
    Engine solo;                 // this object as the only slot
    afe_batch *batch = nullptr;  // batch it is attached to, if any

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
        for (void *p : allocs) (void)hipFree(p);
        if (h_status) (void)hipHostFree(h_status);
        if (h_scalar) (void)hipHostFree(h_scalar);
        if (h_counts) (void)hipHostFree(h_counts);
    }
};

struct afe_batch {
    Engine eng;
};

namespace {

// Device bytes of one simulation (the allocations of build_afe_cell_data).
// In-place history slots per cell and pool slots for accel_depth `depth` and
// afe_params.history_cells.
int hist_small_of(int depth, int history_cells) { return history_cells > 0 ? std::min(depth, 8) : depth; }

// Doubles to allocate for `values` history entries: FP64, or FP32 in mixed
// precision (two per double).
size_t hist_doubles(size_t values, bool mixed) { return mixed ? (values + 1) / 2 : values; }

size_t estimate_bytes(int N, const std::vector<int64_t> &cell_dofs, int64_t nsub, int max_cell_dofs, int depth,
                      bool mixed, int history_cells) {
    const size_t nc = size_t(5) * (N + 1);
    const size_t np = size_t(N + 1) * (N + 2) * (N + 3) / 6, nf = size_t(N + 1) * (N + 2) / 2;
    const size_t n_cells = cell_dofs.size();
    size_t b = 0, ndof = 0;
    for (int64_t n : cell_dofs) {
        b += size_t(n) * size_t((n + 15) & ~int64_t(15)) * sizeof(double);
        if (mixed) b += size_t(n) * size_t((n + 31) & ~int64_t(31)) * sizeof(float);
        ndof += size_t(n);
    }
    const int hs = hist_small_of(depth, history_cells);
    b += ndof * nc * sizeof(double) * 5;  // x, R, S, f, G(x)
    b += 2 * hist_doubles(ndof * nc * size_t(std::max(hs, 1)), mixed) * sizeof(double);  // in-place history
    b += 2 * hist_doubles(hs < depth ? size_t(history_cells) * size_t(depth - hs) * size_t(max_cell_dofs) * nc : 1,
                          mixed) * sizeof(double);  // pooled history
    if (mixed) b += ndof * nc * sizeof(float) + ndof * 5 * sizeof(double);  // FP32 residual, u^n DOF-major
    else b += size_t(afe::kMinvSplitK) * ndof * nc * sizeof(double);  // split M^-1 partials
    b += n_cells * size_t((max_cell_dofs + 63) / 64) * 130 * sizeof(double);
    b += size_t(nsub) * np * nc * sizeof(double);
    b += size_t(nsub) * nf * 25 * sizeof(double) + size_t(nsub) * np * 5 * sizeof(double);  // traces, faces, volume
    b += ndof * (5 * 8 + 8 + 4 + 8 + 4 + 4);  // rhs, column sums, DOF cell, scales, incidence offsets
    b += size_t(nsub) * (2 * np * 4 + 10 * 8 + 4 * 8 + 4 + 4 + 2 * nf * 4);  // connectivity, geometry, incidences
    b += n_cells * ((2 * 63 * 63 + 2 * 63) * 8 + 96);  // Gram / Cholesky, coefficients, per-cell scalars and offsets
    b += 2 * n_cells * sizeof(int32_t);           // predictor list of a batch of one
    return b;
}

afe_status check_params(const afe_params *p) {
    if (p->precision != AFE_FP64 && p->precision != AFE_MIXED) return fail(AFE_E_ARG, "unknown precision");
    if (p->predictor_guess != 0 && p->predictor_guess != 1) return fail(AFE_E_ARG, "predictor_guess must be 0 or 1");
    if (p->history_cells < 0) return fail(AFE_E_ARG, "history_cells must be >= 0");
    if (p->accel_depth < 0 || p->accel_depth > 63) return fail(AFE_E_ARG, "accel_depth must be in [0, 63]");
    if (p->max_iter < 1) return fail(AFE_E_ARG, "max_iter must be >= 1");
    if (!(p->gamma > 1.0) || p->mu < 0.0 || !(p->tol >= 0.0) || !(p->kappa >= 0.0) || !(p->cv > 0.0))
        return fail(AFE_E_ARG, "invalid physics or tolerance parameter");
    return AFE_OK;
}

// A bounded mesh's corrector reads the caller's boundary states.
afe_status check_boundary(const afe_cell_data *cd) {
    if (cd->host.n_btri > 0 && !cd->g.bstate)
        return fail(AFE_E_ARG, "bounded mesh: no boundary states registered (afe_set_boundary_states)");
    const afe_params &p = cd->params;
    if (cd->host.n_btri > 0 && (p.mu != 0.0 || p.kappa != 0.0 || p.av) && !cd->g.bgrad)
        return fail(AFE_E_ARG, "bounded viscous mesh: no boundary gradients registered (afe_set_boundary_gradients)");
    return AFE_OK;
}

// ----------------------------------------------------------------- engine

afe_status ensure_stream(Engine &E) {
    if (!E.own) {
        HIP_TRY(hipStreamCreateWithFlags(&E.own, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&E.join[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&E.join[1], hipEventDisableTiming));
    }
    return AFE_OK;
}

// Regroup the slots and upload the table when attachments changed.
afe_status sync_layout(Engine &E, hipStream_t s) {
    if (!E.d_tab) {
        HIP_TRY(hipMalloc(&E.d_tab, sizeof(afe::DevSlot) * afe::kMaxSlots));
        HIP_TRY(hipHostMalloc(&E.h_counts, sizeof(int32_t) * afe::kMaxSlots, hipHostMallocDefault));
    }
    if (!E.dirty) return AFE_OK;
    HIP_TRY(hipStreamSynchronize(s));
    E.drop_graphs();
    E.drop_groups();
    std::map<std::tuple<int, int, int>, int> gid;
    for (int sl = 0; sl < afe::kMaxSlots; ++sl) {
        afe_cell_data *cd = E.cds[sl];
        if (!cd) continue;
        E.tab[sl].g = cd->g;
        E.tab[sl].w = cd->w;
        E.tab[sl].w.u = E.u[sl];
        // 0: inviscid, 1: viscosity, 2: viscosity and heat conduction
        const int visc = cd->g.kappa != 0.0 ? 2 : (cd->g.mu != 0.0 || cd->g.av) ? 1 : 0;
        const auto key = std::make_tuple(cd->g.N, cd->g.mixed, visc);
        auto it = gid.find(key);
        if (it == gid.end()) {
            it = gid.emplace(key, int(E.groups.size())).first;
            Group gr;
            gr.N = cd->g.N;
            gr.mixed = cd->g.mixed;
            gr.visc = visc;
            E.groups.push_back(gr);
        }
        Group &gr = E.groups[it->second];
        gr.slots.push_back(sl);
        gr.base.push_back(gr.cells);
        gr.cells += cd->host.n_cells;
        gr.max_cell_dofs = std::max(gr.max_cell_dofs, cd->host.max_cell_dofs);
        gr.max_cell_subtets = std::max(gr.max_cell_subtets, cd->host.max_cell_subtets);
    }
    for (auto &gr : E.groups) {
        gr.resident = afe::resident_shape(gr.N, gr.mixed, gr.visc);
        if (gr.cells > INT_MAX / 64) return fail(AFE_E_ARG, "too many cells in one group");
        HIP_TRY(hipMalloc(&gr.lists, sizeof(int32_t) * 2 * size_t(gr.cells)));
        HIP_TRY(hipMalloc(&gr.counts, sizeof(int32_t) * 2));
    }
    HIP_TRY(hipMemcpy(E.d_tab, E.tab.data(), sizeof(afe::DevSlot) * afe::kMaxSlots, hipMemcpyHostToDevice));
    E.dirty = false;
    return AFE_OK;
}

void apply_shape(Engine &E) {
    auto scale = [](double x, int res) { return x > 0.0 ? std::max(1, int(std::lround(x * res))) : 0; };
    for (auto &gr : E.groups) {
        gr.shape.g_sub = scale(E.shape.sub, gr.resident.g_sub);
        gr.shape.g_gather = scale(E.shape.sub, gr.resident.g_gather);
        gr.shape.g_minv = scale(E.shape.minv, gr.resident.g_minv);
        gr.shape.g_dots = scale(E.shape.anderson, gr.resident.g_dots);
        gr.shape.g_solve = scale(E.shape.anderson, gr.resident.g_solve);
        gr.shape.g_update = scale(E.shape.anderson, gr.resident.g_update);
    }
}

bool persistent(const Engine &E) { return E.shape.sub > 0.0 && E.shape.minv > 0.0 && E.shape.anderson > 0.0; }

// Start of a step for every slot: status cleared, detector (Sec. 4.5), the
// time step (batch: from the CFL number, on the device) and the predictor's
// initial iterate and lists.
afe_status launch_pre(Engine &E, bool cfl_dt, hipStream_t s) {
    for (auto &gr : E.groups) {
        for (size_t i = 0; i < gr.slots.size(); ++i) {
            const int sl = gr.slots[i];
            afe_cell_data *cd = E.cds[sl];
            const afe::DevWork &w = E.tab[sl].w;
            HIP_TRY(afe::launch_reset_status(cd->g, w, s));
            HIP_TRY(afe::launch_detect(cd->g, w, E.u[sl], s));
            if (cfl_dt) HIP_TRY(afe::launch_cfl_dt(cd->g, w, E.cfl[sl], cd->host.h_min, cd->d_scalar, s));
            HIP_TRY(afe::launch_pred_init(cd->g, w, sl, gr.lists, gr.base[i], s));
            // the start is consumed: only a completed step (k_step_stats) re-arms it
            HIP_TRY(afe::launch_set_count(w.guess_ok, 0, s));
        }
        HIP_TRY(afe::launch_set_count(gr.counts, int(gr.cells), s));
    }
    return AFE_OK;
}

// One predictor iteration of every group, iteration index it (list parity).
afe_status launch_round(Engine &E, int it, const std::vector<int> &upper, int prof_slot, hipStream_t s) {
    for (size_t gi = 0; gi < E.groups.size(); ++gi) {
        Group &gr = E.groups[gi];
        const int cur = it % 2, nxt = 1 - cur;
        afe::RoundArgs a{};
        a.N = gr.N;
        a.mixed = gr.mixed;
        a.visc = gr.visc;
        a.tab = E.d_tab;
        a.list = gr.lists + size_t(cur) * gr.cells;
        a.count = gr.counts + cur;
        a.next = gr.lists + size_t(nxt) * gr.cells;
        a.next_count = gr.counts + nxt;
        a.n_upper = upper.empty() ? -1 : upper[gi];
        // every listed cell is at iteration it; graph chunks replay at any it
        a.split = (!gr.mixed && (upper.empty() || it >= afe::kMinvSplitAfter)) ? afe::kMinvSplitK : 1;
        // short lists (or unknown length): more workgroups per cell in the update
        a.upd_fine = upper.empty() || int64_t(upper[gi]) * ((gr.max_cell_dofs + 63) / 64) <= afe::kUpdFineTiles;
        a.max_cell_dofs = gr.max_cell_dofs;
        a.max_cell_subtets = gr.max_cell_subtets;
        a.shape = gr.shape;
        const bool prof = gi == 0 && prof_slot >= 0;
        a.ev0 = prof ? E.hooks.start[prof_slot] : nullptr;
        a.ev1 = prof ? E.hooks.stop[prof_slot] : nullptr;
        a.bytes = prof ? E.d_bytes : nullptr;
        HIP_TRY(afe::launch_pred_round(a, s));
    }
    return AFE_OK;
}

afe_status capture(Engine &E, hipGraphExec_t *out, hipStream_t s, afe_status (*body)(Engine &, int, hipStream_t),
                   int arg) {
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    afe_status st = body(E, arg, s);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != AFE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(AFE_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(AFE_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
    return AFE_OK;
}

afe_status chunk_body(Engine &E, int parity, hipStream_t s) {
    static const std::vector<int> none;
    for (int r = 0; r < E.shape.rounds; ++r) AFE_TRY(launch_round(E, parity + r, none, -1, s));
    return AFE_OK;
}

afe_status ensure_side(Engine &E) {
    if (E.side) return AFE_OK;
    HIP_TRY(hipStreamCreateWithFlags(&E.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&E.ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&E.ev_early, hipEventDisableTiming));
    return AFE_OK;
}

// A cell's predictor is final once it has left the lists.  When at most
// 1/kEarlyFraction of the cells still iterate, the cells of the lists for
// iteration `it` are marked late and the time integrals of all other cells
// are computed on the side stream, overlapping the remaining iterations;
// finish_post joins it and computes the late cells' integrals.  The pass a
// sub-tet falls in does not change its result.
constexpr int64_t kEarlyFraction = 16;

afe_status launch_early_post(Engine &E, int it, const std::vector<int> &upper, hipStream_t s) {
    AFE_TRY(ensure_side(E));
    for (auto &gr : E.groups)
        for (int sl : gr.slots) HIP_TRY(afe::launch_clear_late(E.cds[sl]->g, E.tab[sl].w, s));
    for (size_t gi = 0; gi < E.groups.size(); ++gi) {
        const Group &gr = E.groups[gi];
        HIP_TRY(afe::launch_mark_listed(E.d_tab, gr.lists + size_t(it % 2) * gr.cells, upper[gi], 2, s));
    }
    HIP_TRY(hipEventRecord(E.ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(E.side, E.ev_fork, 0));
    for (auto &gr : E.groups)
        for (int sl : gr.slots) HIP_TRY(afe::launch_pred_post(E.cds[sl]->g, E.tab[sl].w, 0, E.side));
    HIP_TRY(hipEventRecord(E.ev_early, E.side));
    E.forked = true;
    return AFE_OK;
}

// Later, when at most 1/kLateCorrectFraction of the cells still iterate: the
// time integrals of the cells that converged since the early pass (middle
// pass), then the corrector of every cell neither listed nor next to a listed
// cell, whose own and neighbours' time integrals are then all final, on the
// side stream after the early pass.  The final pass corrects the rest.  The
// predictor kernels read u^n of listed cells only, which this pass leaves
// alone; the pass a cell falls in does not change its bits.
constexpr int64_t kLateCorrectFraction = 256;
// Grid of that pass's M^-1 update, in workgroups (two per CU): a full grid
// would fill every CU ahead of the few-cell launches of the iteration tail it
// overlaps.  Measured against 256 and 1024 and the full grid.
constexpr int kSideMinvBlocks = 512;

afe_status launch_early_correct(Engine &E, int it, const std::vector<int> &upper, hipStream_t s) {
    for (auto &gr : E.groups)
        for (int sl : gr.slots) {
            HIP_TRY(afe::launch_relabel_late(E.cds[sl]->g, E.tab[sl].w, s));
            HIP_TRY(afe::launch_clear_late2(E.cds[sl]->g, E.tab[sl].w, s));
        }
    for (size_t gi = 0; gi < E.groups.size(); ++gi) {
        const Group &gr = E.groups[gi];
        const int32_t *list = gr.lists + size_t(it % 2) * gr.cells;
        HIP_TRY(afe::launch_mark_listed(E.d_tab, list, upper[gi], 2, s));
        HIP_TRY(afe::launch_mark_late2(E.d_tab, list, upper[gi], s));
    }
    HIP_TRY(hipEventRecord(E.ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(E.side, E.ev_fork, 0));
    for (auto &gr : E.groups)
        for (int sl : gr.slots) {
            afe_cell_data *cd = E.cds[sl];
            HIP_TRY(afe::launch_pred_post(cd->g, E.tab[sl].w, 1, E.side));
            HIP_TRY(afe::launch_correct(cd->g, E.tab[sl].w, E.u[sl], 0, E.side, kSideMinvBlocks));
        }
    HIP_TRY(hipEventRecord(E.ev_early, E.side));
    E.forked2 = true;
    return AFE_OK;
}

// Orders s after the early pass, if one ran in this step.
afe_status join_early(Engine &E, hipStream_t s) {
    if (E.forked) HIP_TRY(hipStreamWaitEvent(s, E.ev_early, 0));
    return AFE_OK;
}

// Predictor iterations until every list is empty: `rounds` iterations are
// enqueued between two reads of the list lengths (with grids sized from the
// lengths: one per read while lists are long).  Cells leave the lists when
// converged or at their max_iter.
afe_status iterate(Engine &E, hipStream_t s) {
    int max_it = 0;
    for (auto &gr : E.groups)
        for (int sl : gr.slots) max_it = std::max(max_it, E.cds[sl]->params.max_iter);
    const bool pers = persistent(E);
    const bool graph = E.shape.graph && pers && !E.prof_on;
    std::vector<int> upper(E.groups.size());
    int64_t total = 0;
    for (size_t gi = 0; gi < E.groups.size(); ++gi) total += upper[gi] = int(E.groups[gi].cells);
    const int64_t all_cells = total;
    E.forked = false;
    E.forked2 = false;
    int it = 0;
    while (total > 0 && it < max_it) {
        int R = E.shape.rounds;
        if (graph) {
            const int p = it % 2;
            if (!E.g_chunk[p]) AFE_TRY(capture(E, &E.g_chunk[p], s, chunk_body, p));
            HIP_TRY(hipGraphLaunch(E.g_chunk[p], s));
        } else {
            int64_t longest = 0;
            for (int v : upper) longest = std::max<int64_t>(longest, v);
            if (!pers && longest > 256) R = 1;  // long lists shrink fast: resize the grids every iteration
            for (int r = 0; r < R; ++r)
                AFE_TRY(launch_round(E, it + r, upper, E.prof_on && r < afe::kMaxRounds ? r : -1, s));
        }
        it += R;
        for (size_t gi = 0; gi < E.groups.size(); ++gi)
            HIP_TRY(hipMemcpyAsync(E.h_counts + gi, E.groups[gi].counts + (it % 2), sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        total = 0;
        for (size_t gi = 0; gi < E.groups.size(); ++gi) total += upper[gi] = E.h_counts[gi];
        if (E.side_ok && !E.forked && total > 0 && total * kEarlyFraction <= all_cells)
            AFE_TRY(launch_early_post(E, it, upper, s));
        if (E.allow_correct && E.forked && !E.forked2 && total > 0 && total * kLateCorrectFraction <= all_cells)
            AFE_TRY(launch_early_correct(E, it, upper, s));
        if (E.prof_on && !graph) {
            for (int r = 0; r < std::min(R, afe::kMaxRounds); ++r) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, E.hooks.start[r], E.hooks.stop[r]));
                E.prof_ms += ms;
                E.prof_launches += 1;
            }
        }
    }
    return AFE_OK;
}

// End of a step for every slot: time integrals of the predictor, corrector
// (Sec. 4.4) with the positivity check, iteration statistics.
afe_status launch_post(Engine &E, hipStream_t s) {
    for (auto &gr : E.groups)
        for (int sl : gr.slots) {
            afe_cell_data *cd = E.cds[sl];
            const afe::DevWork &w = E.tab[sl].w;
            HIP_TRY(afe::launch_pred_post(cd->g, w, 2, s));
            HIP_TRY(afe::launch_correct(cd->g, w, E.u[sl], 1, s));
            HIP_TRY(afe::launch_step_stats(cd->g, w, s));
        }
    return AFE_OK;
}

afe_status pre_body(Engine &E, int, hipStream_t s) { return launch_pre(E, true, s); }
afe_status post_body(Engine &E, int, hipStream_t s) { return launch_post(E, s); }

afe_status profile_enable(Engine &E, int32_t enable) {
    if (enable && !E.d_bytes) {
        for (int i = 0; i < afe::kMaxRounds; ++i) {
            HIP_TRY(hipEventCreate(&E.hooks.start[i]));
            HIP_TRY(hipEventCreate(&E.hooks.stop[i]));
        }
        HIP_TRY(hipMalloc(&E.d_bytes, 2 * sizeof(unsigned long long)));
    }
    E.prof_on = enable != 0;
    E.prof_ms = 0.0;
    E.prof_launches = 0;
    if (E.d_bytes) HIP_TRY(hipMemset(E.d_bytes, 0, 2 * sizeof(unsigned long long)));
    return AFE_OK;
}

afe_status profile_read(Engine &E, double *kernel_ms, int64_t *launches, double *bytes, double *bytes_stored) {
    unsigned long long b[2] = {0, 0};
    if (E.d_bytes) HIP_TRY(hipMemcpy(b, E.d_bytes, sizeof(b), hipMemcpyDeviceToHost));
    if (kernel_ms) *kernel_ms = E.prof_ms;
    if (launches) *launches = E.prof_launches;
    if (bytes) *bytes = double(b[0]);
    if (bytes_stored) *bytes_stored = double(b[1]);
    return AFE_OK;
}

afe_status status_of(int flags) {
    if (flags & afe::kStatusHistoryPool) return AFE_E_HBM_BUDGET;  // the root cause of anything after it
    if (flags & afe::kStatusNonfinite) return AFE_E_NONFINITE;
    if (flags & afe::kStatusNoConv) return AFE_E_NO_CONVERGENCE;
    if (flags & afe::kStatusPositivity) return AFE_E_POSITIVITY;
    return AFE_OK;
}

const char *status_text(afe_status st) {
    switch (st) {
        case AFE_E_NONFINITE: return "non-finite state after the update";
        case AFE_E_NO_CONVERGENCE: return "predictor did not converge";
        case AFE_E_POSITIVITY: return "density or pressure not positive";
        case AFE_E_HBM_BUDGET: return "more cells needed the Anderson history pool than history_cells";
        default: return "";
    }
}

// One step of every slot of a batch on stream s (the engine's own stream).
afe_status batch_step_on(Engine &E, afe_batch_report *reps, int32_t n_reps, hipStream_t s) {
    apply_shape(E);
    const bool graph = E.shape.graph && persistent(E) && !E.prof_on;
    if (graph) {
        if (!E.g_pre) AFE_TRY(capture(E, &E.g_pre, s, pre_body, 0));
        HIP_TRY(hipGraphLaunch(E.g_pre, s));
    } else {
        AFE_TRY(launch_pre(E, true, s));
    }
    E.allow_correct = true;
    const afe_status it_st = iterate(E, s);
    E.allow_correct = false;
    AFE_TRY(it_st);
    AFE_TRY(join_early(E, s));
    if (graph) {
        if (!E.g_post) AFE_TRY(capture(E, &E.g_post, s, post_body, 0));
        HIP_TRY(hipGraphLaunch(E.g_post, s));
    } else {
        AFE_TRY(launch_post(E, s));
    }
    for (int sl = 0; sl < afe::kMaxSlots; ++sl) {
        afe_cell_data *cd = E.cds[sl];
        if (!cd) continue;
        HIP_TRY(hipMemcpyAsync(cd->h_status, cd->w.status, kStatusWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(cd->h_scalar + 1, cd->w.dt, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    E.reported = true;
    afe_status first = AFE_OK;
    for (int sl = 0; sl < afe::kMaxSlots; ++sl) {
        afe_cell_data *cd = E.cds[sl];
        if (!cd) continue;
        const int32_t *h = cd->h_status;
        const afe_status st = status_of(h[0]);
        if (first == AFE_OK && st != AFE_OK) first = st;
        if (reps && sl < n_reps) {
            afe_batch_report &r = reps[sl];
            r.status = st;
            r.iters_min = h[4];
            r.iters_max = h[5];
            unsigned long long sum = 0;
            std::memcpy(&sum, h + 6, sizeof(sum));
            r.iters_mean = cd->host.n_cells ? double(sum) / double(cd->host.n_cells) : 0.0;
            r.n_troubled = h[3];
            r.status_cell = h[0] ? h[1] : -1;
            r.dt = cd->h_scalar[1];
        }
    }
    if (first != AFE_OK) return fail(first, status_text(first));
    return AFE_OK;
}

// Run `fn` on the engine's stream, ordered after the work on `user`, and
// order the later work on `user` after it.
template <typename F>
afe_status on_own_stream(Engine &E, hipStream_t user, F &&fn) {
    AFE_TRY(ensure_stream(E));
    HIP_TRY(hipEventRecord(E.join[0], user));
    HIP_TRY(hipStreamWaitEvent(E.own, E.join[0], 0));
    afe_status st = fn(E.own);
    HIP_TRY(hipEventRecord(E.join[1], E.own));
    HIP_TRY(hipStreamWaitEvent(user, E.join[1], 0));
    return st;
}

}  // namespace

extern "C" {

const char *afe_last_error(void) { return g_err.c_str(); }

void afe_free(afe_cell_data *cd) {
    if (cd && cd->batch) (void)afe_batch_detach(cd->batch, cd);
    delete cd;
}

afe_status build_afe_cell_data(const afe_mesh *mesh, int32_t N, const afe_params *params, void *stream,
                               afe_cell_data **out) {
    if (!mesh || !params || !out) return fail(AFE_E_ARG, "null argument");
    *out = nullptr;
    AFE_TRY(check_params(params));
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
    if (h.n_cells >= afe::kMaxCellsPerSlot) {
        delete cd;
        return fail(AFE_E_ARG, "too many cells");
    }
    std::vector<int64_t> cell_dofs(h.n_cells);
    for (int c = 0; c < h.n_cells; ++c) cell_dofs[c] = h.dof_ptr[c + 1] - h.dof_ptr[c];
    size_t need = estimate_bytes(N, cell_dofs, h.nsub, h.max_cell_dofs, depth, params->precision == AFE_MIXED,
                                 params->history_cells);
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
    g.kappa = params->kappa;
    g.cv = params->cv;
    g.av = params->av;
    g.mixed = params->precision == AFE_MIXED ? 1 : 0;
    g.guess = params->predictor_guess;
    g.bstate = nullptr;
    g.bgrad = nullptr;
    g.n_btri = h.n_btri;
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
    static_assert(afe::kRefNp >= afe::kMaxNp && afe::kRefNf >= afe::kMaxNf && afe::kRefNt >= afe::kMaxNt &&
                      afe::kRefNq >= afe::kMaxNq,
                  "device reference arrays smaller than the largest degree");
    std::unique_ptr<afe::DevRef> ref_box(new (std::nothrow) afe::DevRef{});
    if (!ref_box) {
        delete cd;
        return fail(AFE_E_ARG, "out of host memory");
    }
    afe::DevRef &ref = *ref_box;
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
    {
        const int inner = 3 * R.np, steps = (inner + 3) / 4, tiles = (R.np + 15) / 16;
        for (int t = 0; t < tiles; ++t)
            for (int j = 0; j < steps; ++j)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * t + l % 16, kk = 4 * j + l / 16;
                    ref.Kfrag[(t * steps + j) * 64 + l] =
                        row < R.np && kk < inner ? R.K[((kk / R.np) * R.np + row) * R.np + kk % R.np] : 0.0;
                    ref.Vfrag[(t * steps + j) * 64 + l] =
                        row < R.np && kk < inner ? R.K[((kk / R.np) * R.np + kk % R.np) * R.np + row] : 0.0;
                }
        const int inner4 = 4 * R.np, steps4 = (inner4 + 3) / 4;
        for (int t = 0; t < tiles; ++t)
            for (int j = 0; j < steps4; ++j)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * t + l % 16, kk = 4 * j + l / 16;
                    double v = 0.0;
                    if (row < R.np && kk < inner)
                        v = R.K[((kk / R.np) * R.np + row) * R.np + kk % R.np];
                    else if (row < R.np && kk < inner4)
                        v = R.M[row * R.np + kk - inner];
                    ref.KMfrag[(t * steps4 + j) * 64 + l] = v;
                }
    }
    for (int a = 0; a < R.nt; ++a) {
        ref.w[a] = R.w[a];
        ref.tau[a] = R.tau[a];
    }
    ref.nq = R.nq;
    for (int q = 0; q < R.nq; ++q) {
        for (int x = 0; x < 3; ++x) ref.qxi[3 * q + x] = R.qxi[3 * q + x];
        ref.qw[q] = R.qw[q];
        for (int m = 0; m < R.np; ++m) ref.qphi[q * R.np + m] = R.qphi[q * R.np + m];
    }
    for (int i = 0; i < R.nt * R.nt; ++i) {
        ref.Ktau_inv[i] = R.Ktau_inv[i];
        ref.Ktau[i] = R.Ktau[i];
    }
    afe::DevRef *dref = nullptr;
    if ((e = cd->alloc(dref, 1)) != hipSuccess || (e = hipMemcpy(dref, &ref, sizeof(ref), hipMemcpyHostToDevice)) != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete cd;
        return fail(AFE_E_HIP, "reference upload: " + m);
    }
    g.ref = dref;
    const size_t nc = size_t(g.nc);
    const size_t nd = size_t(h.ndof);
    g.hist_small = hist_small_of(depth, params->history_cells);
    g.pool_cap = g.hist_small < depth ? params->history_cells : 0;
    g.pool_stride = int64_t(depth - g.hist_small) * h.max_cell_dofs * int64_t(g.nc);
    const int dslots = std::max(g.hist_small, 1);
    const size_t pool = g.pool_cap > 0 ? size_t(g.pool_cap) * size_t(g.pool_stride) : 1;
    w.depth = depth;
    w.tol = params->tol;
    w.max_iter = params->max_iter;
    if ((e = cd->alloc(g.minv, size_t(minv_ptr[h.n_cells]))) != hipSuccess ||
        (e = cd->alloc(g.dscale, nd)) != hipSuccess ||
        (e = cd->alloc(g.minv32, size_t(minv32_ptr[h.n_cells]))) != hipSuccess ||
        (e = cd->alloc(w.R32, g.mixed ? nd * nc : 1)) != hipSuccess ||
        (e = cd->alloc(w.un5, g.mixed ? nd * 5 : 1)) != hipSuccess ||
        (e = cd->alloc(w.x, nd * nc)) != hipSuccess || (e = cd->alloc(w.R, nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.S, nd * nc)) != hipSuccess || (e = cd->alloc(w.fprev, nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.Sp, g.mixed ? 1 : size_t(afe::kMinvSplitK) * nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.gprev, nd * nc)) != hipSuccess ||
        (e = cd->alloc(w.part, size_t(h.n_cells) * ((h.max_cell_dofs + 63) / 64) * 130)) != hipSuccess ||
        (e = cd->alloc(w.dF, hist_doubles(nd * nc * dslots, g.mixed))) != hipSuccess ||
        (e = cd->alloc(w.dG, hist_doubles(nd * nc * dslots, g.mixed))) != hipSuccess ||
        (e = cd->alloc(w.dFp, hist_doubles(pool, g.mixed))) != hipSuccess ||
        (e = cd->alloc(w.dGp, hist_doubles(pool, g.mixed))) != hipSuccess ||
        (e = cd->alloc(w.pool_slot, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.pool_count, 1)) != hipSuccess ||
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
        (e = cd->alloc(w.iters, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.gamma, size_t(h.n_cells) * 63)) != hipSuccess ||
        (e = cd->alloc(w.kuse, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.late, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.late2, size_t(h.n_cells))) != hipSuccess ||
        (e = cd->alloc(w.dt, 1)) != hipSuccess || (e = cd->alloc(w.dt_prev, 1)) != hipSuccess ||
        (e = cd->alloc(w.guess_ok, 1)) != hipSuccess || (e = hipMemsetAsync(w.guess_ok, 0, sizeof(int32_t), s)) != hipSuccess ||
        (e = cd->alloc(w.status, kStatusWords)) != hipSuccess || (e = cd->alloc(cd->d_scalar, 1)) != hipSuccess ||
        (e = hipHostMalloc(&cd->h_status, kStatusWords * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(&cd->h_scalar, 2 * sizeof(double), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc(&cd->h_counts, sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (e = hipGetDevice(&cd->device)) != hipSuccess) {
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
    cd->solo.cds[0] = cd;
    *out = cd;
    return AFE_OK;
}

afe_status afe_estimate_bytes(const afe_mesh *mesh, int32_t N, const afe_params *params, size_t *bytes) {
    if (!mesh || !params || !bytes) return fail(AFE_E_ARG, "null argument");
    if (N < 1 || N > afe::kMaxN) return fail(AFE_E_ARG, "N must be 1, 2, 3 or 4");
    if (mesh->n_cells < 1 || mesh->n_faces < 1 || !mesh->face_ptr || !mesh->face_vtx || !mesh->face_cell)
        return fail(AFE_E_ARG, "empty mesh");
    // per cell: V vertices, F faces, E polygon edges; its sub-grid has
    // V + F + 1 vertices, 3E + V + F edges, 5E triangles and 2E sub-tets
    const int nc = mesh->n_cells;
    std::vector<int64_t> F(nc, 0), E(nc, 0);
    std::vector<std::vector<int32_t>> verts(nc);
    for (int f = 0; f < mesh->n_faces; ++f) {
        const int k = mesh->face_ptr[f + 1] - mesh->face_ptr[f];
        for (int side = 0; side < 2; ++side) {
            const int c = mesh->face_cell[2 * f + side];
            if (side == 1 && c == -1) continue;  // boundary face of a bounded mesh
            if (c < 0 || c >= nc) return fail(AFE_E_BAD_MESH, "face cell out of range");
            F[c] += 1;
            E[c] += k;
            for (int i = mesh->face_ptr[f]; i < mesh->face_ptr[f + 1]; ++i) verts[c].push_back(mesh->face_vtx[i]);
        }
    }
    const int64_t a = N - 1;
    std::vector<int64_t> dofs(nc);
    int64_t nsub = 0;
    int max_dofs = 0;
    for (int c = 0; c < nc; ++c) {
        if (F[c] == 0) return fail(AFE_E_BAD_MESH, "cell without faces");
        std::sort(verts[c].begin(), verts[c].end());
        const int64_t V = std::unique(verts[c].begin(), verts[c].end()) - verts[c].begin();
        const int64_t Ec = E[c] / 2;
        dofs[c] = (V + F[c] + 1) + a * (3 * Ec + V + F[c]) + (a * (a - 1) / 2) * 5 * Ec +
                  (a * (a - 1) * (a - 2) / 6) * 2 * Ec;
        nsub += 2 * Ec;
        max_dofs = std::max<int>(max_dofs, int(dofs[c]));
    }
    *bytes = estimate_bytes(N, dofs, nsub, max_dofs, params->accel_depth, params->precision == AFE_MIXED,
                            params->history_cells);
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

afe_status afe_boundary_nodes(const afe_cell_data *cd, int64_t *count, double *xyz, double *tau) {
    if (!cd || !count) return fail(AFE_E_ARG, "null argument");
    const afe::HostGrid &h = cd->host;
    *count = h.n_btri * h.nf;
    if (xyz && !h.bnode_x.empty()) std::memcpy(xyz, h.bnode_x.data(), h.bnode_x.size() * sizeof(double));
    if (tau) {
        const afe::RefData &R = afe::ref_data(h.N);
        for (int a = 0; a <= h.N; ++a) tau[a] = R.tau[a];
    }
    return AFE_OK;
}

afe_status afe_set_boundary_states(afe_cell_data *cd, const double *prim) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    if (prim && cd->host.n_btri == 0) return fail(AFE_E_ARG, "the mesh has no boundary faces");
    cd->g.bstate = prim;
    return AFE_OK;
}

afe_status afe_set_boundary_gradients(afe_cell_data *cd, const double *grad) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    if (grad && cd->host.n_btri == 0) return fail(AFE_E_ARG, "the mesh has no boundary faces");
    cd->g.bgrad = grad;
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
    HIP_TRY(afe::launch_cfl_dt(cd->g, cd->w, 0.0, cd->host.h_min, cd->d_scalar, s));
    HIP_TRY(hipMemcpyAsync(cd->h_scalar, cd->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double smax = *cd->h_scalar;
    if (!(smax > 0.0) || !std::isfinite(smax)) return fail(AFE_E_NONFINITE, "non-finite wave speed");
    *dt_host = cfl * cd->host.h_min / ((2 * cd->host.N + 1) * smax);
    return AFE_OK;
}

}  // extern "C"

namespace {
// Predictor of one object; with `full`, the caller goes on to correct u in
// the same step, so the corrector may start early for cells that allow it.
afe_status predict_impl(afe_cell_data *cd, const double *u, double dt, void *stream, bool full) {
    if (!cd || !u || !(dt > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    if (full) AFE_TRY(check_boundary(cd));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Engine &E = cd->solo;
    if (E.u[0] != u) {
        E.u[0] = const_cast<double *>(u);
        E.dirty = true;
        HIP_TRY(afe::launch_set_count(cd->w.guess_ok, 0, s));  // another state: start from u^n
    }
    AFE_TRY(sync_layout(E, s));
    apply_shape(E);
    HIP_TRY(afe::launch_set_dt(cd->w, dt, s));
    AFE_TRY(launch_pre(E, false, s));
    E.allow_correct = full;
    const afe_status it_st = iterate(E, s);
    E.allow_correct = false;
    AFE_TRY(it_st);
    AFE_TRY(join_early(E, s));
    HIP_TRY(afe::launch_pred_post(cd->g, E.tab[0].w, 2, s));
    return AFE_OK;
}
}  // namespace

extern "C" {

afe_status ader_predict(afe_cell_data *cd, const double *u, double dt, void *stream) {
    return predict_impl(cd, u, dt, stream, false);
}

afe_status ader_correct(afe_cell_data *cd, double *u, double dt, void *stream) {
    if (!cd || !u || !(dt > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    AFE_TRY(check_boundary(cd));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(afe::launch_set_dt(cd->w, dt, s));
    HIP_TRY(afe::launch_correct(cd->g, cd->w, u, 1, s));
    HIP_TRY(afe::launch_step_stats(cd->g, cd->w, s));
    return AFE_OK;
}

afe_status ader_step(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, void *stream) {
    AFE_TRY(predict_impl(cd, u, dt, stream, true));
    AFE_TRY(ader_correct(cd, u, dt, stream));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(cd->h_status, cd->w.status, kStatusWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int32_t *h = cd->h_status;
    if (rep) {
        unsigned long long sum = 0;
        std::memcpy(&sum, h + 6, sizeof(sum));
        rep->iters_min = h[4];
        rep->iters_max = h[5];
        rep->iters_mean = cd->host.n_cells ? double(sum) / double(cd->host.n_cells) : 0.0;
        rep->n_troubled = h[3];
        rep->status_cell = h[0] ? h[1] : -1;
    }
    const afe_status st = status_of(h[0]);
    if (st != AFE_OK) return fail(st, status_text(st));
    return AFE_OK;
}

}  // extern "C"

namespace {

// ------------------------------------------------ allocation-free step
//
// The step's only device memory beyond the object's own buffers (built once
// by build_afe_cell_data) is the engine's slot table, its two list lengths
// and its two predictor lists; ader_step allocates them lazily, and again
// whenever it is handed another state.  The allocation-free step keeps them
// in this file-scope array instead, one copy per device (each device that
// runs the library holds it until the process ends), laid out as
//   [0, kScratchTable)                          slot table (one DevSlot)
//   [kScratchTable, kScratchTable + 256)        list lengths (2 int32)
//   [kScratchTable + 256, kScratchBytes)        lists (2 x n_cells int32)
// Every call on a device shares that device's array and overwrites it; calls
// that overlap on one device race.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr size_t kScratchTable = (sizeof(afe::DevSlot) + 255) & ~size_t(255);
constexpr size_t kScratchLists = kScratchTable + 256;
constexpr int64_t kScratchMaxCells = int64_t((kScratchBytes - kScratchLists) / (2 * sizeof(int32_t)));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (the array's name is a host-side stand-in, not a device address).
afe_status scratch_address(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(AFE_E_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(AFE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_dev[dev]);
    return AFE_OK;
}

// An engine over one object whose table, lists and list lengths point into
// the scratch array; it owns nothing (its destructor frees nothing).
struct ScratchEngine {
    Engine E;
    ~ScratchEngine() {
        E.d_tab = nullptr;
        E.h_counts = nullptr;
        for (auto &gr : E.groups) gr.lists = gr.counts = nullptr;
        E.groups.clear();
    }
};

afe_status step_noalloc(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, hipStream_t s) {
    AFE_TRY(check_boundary(cd));
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != cd->device) return fail(AFE_E_ARG, "the current device is not the object's device");
    if (int64_t(cd->host.n_cells) > kScratchMaxCells)
        return fail(AFE_E_ARG, "mesh has " + std::to_string(cd->host.n_cells) + " cells; the allocation-free step takes at most " +
                                   std::to_string(kScratchMaxCells));
    unsigned char *base = nullptr;
    AFE_TRY(scratch_address(dev, &base));
    if (cd->solo.u[0] != u) {  // another state: the predictor starts from u^n
        cd->solo.u[0] = u;
        cd->solo.dirty = true;
        HIP_TRY(afe::launch_set_count(cd->w.guess_ok, 0, s));
    }
    ScratchEngine se;
    Engine &E = se.E;
    E.side_ok = false;
    E.cds[0] = cd;
    E.u[0] = u;
    E.tab[0].g = cd->g;
    E.tab[0].w = cd->w;
    E.tab[0].w.u = u;
    Group gr;
    gr.N = cd->g.N;
    gr.mixed = cd->g.mixed;
    gr.visc = cd->g.kappa != 0.0 ? 2 : (cd->g.mu != 0.0 || cd->g.av) ? 1 : 0;
    gr.slots.push_back(0);
    gr.base.push_back(0);
    gr.cells = cd->host.n_cells;
    gr.max_cell_dofs = cd->host.max_cell_dofs;
    gr.max_cell_subtets = cd->host.max_cell_subtets;
    gr.resident = afe::resident_shape(gr.N, gr.mixed, gr.visc);
    gr.counts = reinterpret_cast<int32_t *>(base + kScratchTable);
    gr.lists = reinterpret_cast<int32_t *>(base + kScratchLists);
    E.groups.push_back(gr);
    E.d_tab = reinterpret_cast<afe::DevSlot *>(base);
    E.h_counts = cd->h_counts;
    E.dirty = false;
    E.shape = cd->solo.shape;
    E.shape.graph = 0;
    // the table lives in host memory of this call until the final synchronisation
    HIP_TRY(hipMemcpyAsync(E.d_tab, E.tab.data(), sizeof(afe::DevSlot), hipMemcpyHostToDevice, s));
    apply_shape(E);
    HIP_TRY(afe::launch_set_dt(cd->w, dt, s));
    AFE_TRY(launch_pre(E, false, s));  // list lengths and lists are written here
    AFE_TRY(iterate(E, s));
    HIP_TRY(afe::launch_pred_post(cd->g, E.tab[0].w, 2, s));
    HIP_TRY(afe::launch_correct(cd->g, cd->w, u, 1, s));
    HIP_TRY(afe::launch_step_stats(cd->g, cd->w, s));
    HIP_TRY(hipMemcpyAsync(cd->h_status, cd->w.status, kStatusWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int32_t *h = cd->h_status;
    if (rep) {
        unsigned long long sum = 0;
        std::memcpy(&sum, h + 6, sizeof(sum));
        rep->iters_min = h[4];
        rep->iters_max = h[5];
        rep->iters_mean = cd->host.n_cells ? double(sum) / double(cd->host.n_cells) : 0.0;
        rep->n_troubled = h[3];
        rep->status_cell = h[0] ? h[1] : -1;
    }
    const afe_status st = status_of(h[0]);
    if (st != AFE_OK) return fail(st, status_text(st));
    return AFE_OK;
}

}  // namespace

extern "C" {

afe_status ader_step_noalloc(afe_cell_data *cd, double *u, double dt, afe_step_report *rep, void *stream) {
    if (!cd || !u || !(dt > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    if (cd->batch) return fail(AFE_E_ARG, "object is attached to a batch");
    return step_noalloc(cd, u, dt, rep, static_cast<hipStream_t>(stream));
}

afe_status afe_l2_points(afe_cell_data *cd, const double *dof_xyz, double *xq, int32_t *nq, void *stream) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    const afe::RefData &R = afe::ref_data(cd->host.N);
    if (nq) *nq = R.nq;
    if (!xq) return AFE_OK;
    if (!dof_xyz) return fail(AFE_E_ARG, "null DOF coordinates");
    HIP_TRY(afe::launch_l2_points(cd->g, dof_xyz, xq, static_cast<hipStream_t>(stream)));
    return AFE_OK;
}

afe_status afe_l2_error(afe_cell_data *cd, const double *u, int32_t var, const double *ref, double *err,
                        void *stream) {
    if (!cd || !u || !ref || !err) return fail(AFE_E_ARG, "null argument");
    if (var < 0 || var > 4) return fail(AFE_E_ARG, "var must be in [0, 4]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the partial sums use the object's Anderson partials buffer (free between steps)
    const int64_t cap = int64_t(cd->host.n_cells) * ((cd->host.max_cell_dofs + 63) / 64) * 130;
    if (afe::l2_blocks(cd->g) > cap) return fail(AFE_E_ARG, "error-norm partials exceed the work buffer");
    HIP_TRY(afe::launch_l2_error(cd->g, u, var, ref, cd->w.part, cd->d_scalar, s));
    HIP_TRY(hipMemcpyAsync(cd->h_scalar, cd->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *err = std::sqrt(cd->h_scalar[0]);
    return AFE_OK;
}

afe_status afe_profile_enable(afe_cell_data *cd, int32_t enable) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    return profile_enable(cd->solo, enable);
}

afe_status afe_profile_read(afe_cell_data *cd, double *kernel_ms, int64_t *launches, double *bytes,
                            double *bytes_stored) {
    if (!cd) return fail(AFE_E_ARG, "null argument");
    return profile_read(cd->solo, kernel_ms, launches, bytes, bytes_stored);
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

// ----------------------------------------------------------------- batches

afe_status afe_batch_create(afe_batch **out) {
    if (!out) return fail(AFE_E_ARG, "null argument");
    *out = new (std::nothrow) afe_batch();
    if (!*out) return fail(AFE_E_ARG, "out of host memory");
    return AFE_OK;
}

void afe_batch_free(afe_batch *b) {
    if (!b) return;
    for (afe_cell_data *cd : b->eng.cds)
        if (cd) cd->batch = nullptr;
    delete b;
}

afe_status afe_batch_attach(afe_batch *b, afe_cell_data *cd, double *u, double cfl, int32_t *slot) {
    if (!b || !cd || !u || !(cfl > 0.0)) return fail(AFE_E_ARG, "invalid argument");
    if (cd->batch) return fail(AFE_E_ARG, "object already attached to a batch");
    if (cd->host.n_btri > 0)
        return fail(AFE_E_ARG, "a bounded mesh is stepped alone: its caller fills the boundary states for each time step");
    Engine &E = b->eng;
    int sl = 0;
    while (sl < afe::kMaxSlots && E.cds[sl]) ++sl;
    if (sl == afe::kMaxSlots) return fail(AFE_E_ARG, "batch full");
    HIP_TRY(hipMemset(cd->w.guess_ok, 0, sizeof(int32_t)));  // the batch's state may be another one
    E.cds[sl] = cd;
    E.u[sl] = u;
    E.cfl[sl] = cfl;
    E.dirty = true;
    cd->batch = b;
    if (slot) *slot = sl;
    return AFE_OK;
}

afe_status afe_batch_detach(afe_batch *b, afe_cell_data *cd) {
    if (!b || !cd || cd->batch != b) return fail(AFE_E_ARG, "object not in this batch");
    Engine &E = b->eng;
    for (int sl = 0; sl < afe::kMaxSlots; ++sl)
        if (E.cds[sl] == cd) {
            E.cds[sl] = nullptr;
            E.u[sl] = nullptr;
        }
    E.dirty = true;
    cd->batch = nullptr;
    return AFE_OK;
}

afe_status afe_batch_step(afe_batch *b, afe_batch_report *reps, int32_t n_reps, void *stream) {
    if (!b || (reps && n_reps < 0)) return fail(AFE_E_ARG, "invalid argument");
    Engine &E = b->eng;
    if (E.n_slots() == 0) return AFE_OK;
    E.reported = false;
    const afe_status st = on_own_stream(E, static_cast<hipStream_t>(stream), [&](hipStream_t s) -> afe_status {
        AFE_TRY(sync_layout(E, s));
        return batch_step_on(E, reps, n_reps, s);
    });
    if (st != AFE_OK && reps && !E.reported) {
        // the call failed before its per-simulation reports: every attached
        // simulation carries the call's status (its step did not complete)
        for (int sl = 0; sl < afe::kMaxSlots && sl < n_reps; ++sl)
            if (E.cds[sl]) {
                reps[sl] = afe_batch_report{};
                reps[sl].status = st;
                reps[sl].status_cell = -1;
            }
    }
    return st;
}

afe_status afe_batch_set_shape(afe_batch *b, const afe_launch_shape *shape) {
    if (!b || !shape) return fail(AFE_E_ARG, "null argument");
    if (shape->rounds < 1 || shape->rounds > afe::kMaxRounds || !(shape->sub >= 0.0) || !(shape->minv >= 0.0) ||
        !(shape->anderson >= 0.0) || shape->sub > 64.0 || shape->minv > 64.0 || shape->anderson > 64.0)
        return fail(AFE_E_ARG, "launch shape out of range");
    if (shape->graph && !(shape->sub > 0.0 && shape->minv > 0.0 && shape->anderson > 0.0))
        return fail(AFE_E_ARG, "graph replay needs persistent grids");
    Engine &E = b->eng;
    E.shape = *shape;
    E.drop_graphs();
    return AFE_OK;
}

afe_status afe_batch_get_shape(const afe_batch *b, afe_launch_shape *shape) {
    if (!b || !shape) return fail(AFE_E_ARG, "null argument");
    *shape = b->eng.shape;
    return AFE_OK;
}

afe_status afe_batch_tune(afe_batch *b, void *stream, afe_launch_shape *chosen) {
    if (!b) return fail(AFE_E_ARG, "null argument");
    Engine &E = b->eng;
    if (E.n_slots() == 0) {
        if (chosen) *chosen = E.shape;
        return AFE_OK;
    }
    if (E.prof_on) return fail(AFE_E_ARG, "profiling is enabled");
    return on_own_stream(E, static_cast<hipStream_t>(stream), [&](hipStream_t s) -> afe_status {
        // every candidate steps a working copy of the states, refreshed from a saved copy
        std::vector<double *> orig(E.u);
        std::vector<double *> work(afe::kMaxSlots, nullptr), saved(afe::kMaxSlots, nullptr);
        size_t total = 0;
        for (int sl = 0; sl < afe::kMaxSlots; ++sl)
            if (E.cds[sl]) total += size_t(5) * E.cds[sl]->host.ndof;
        double *scratch = nullptr;
        HIP_TRY(hipMalloc(&scratch, 2 * total * sizeof(double)));
        size_t off = 0;
        for (int sl = 0; sl < afe::kMaxSlots; ++sl)
            if (E.cds[sl]) {
                const size_t n = size_t(5) * E.cds[sl]->host.ndof;
                saved[sl] = scratch + off;
                work[sl] = scratch + total + off;
                off += n;
            }
        afe_status st = AFE_OK;
        for (int sl = 0; sl < afe::kMaxSlots && st == AFE_OK; ++sl)
            if (E.cds[sl] && hipMemcpyAsync(saved[sl], orig[sl], size_t(5) * E.cds[sl]->host.ndof * sizeof(double),
                                            hipMemcpyDeviceToDevice, s) != hipSuccess)
                st = fail(AFE_E_HIP, "state copy");
        for (int sl = 0; sl < afe::kMaxSlots; ++sl)
            if (E.cds[sl]) E.u[sl] = work[sl];
        E.dirty = true;
        auto time_shape = [&](const afe_launch_shape &sh, double &ms) -> afe_status {
            E.shape = sh;
            E.drop_graphs();
            for (int rep = 0; rep < 2; ++rep) {  // the first run captures graphs and warms caches
                for (int sl = 0; sl < afe::kMaxSlots; ++sl)
                    if (E.cds[sl]) {
                        HIP_TRY(hipMemcpyAsync(work[sl], saved[sl], size_t(5) * E.cds[sl]->host.ndof * sizeof(double),
                                               hipMemcpyDeviceToDevice, s));
                        HIP_TRY(afe::launch_set_count(E.cds[sl]->w.guess_ok, 0, s));  // every trial starts from u^n
                    }
                AFE_TRY(sync_layout(E, s));
                HIP_TRY(hipStreamSynchronize(s));
                const auto t0 = std::chrono::steady_clock::now();
                const afe_status r = batch_step_on(E, nullptr, 0, s);
                if (r != AFE_OK && r != AFE_E_NO_CONVERGENCE && r != AFE_E_POSITIVITY && r != AFE_E_NONFINITE) return r;
                ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            return AFE_OK;
        };
        afe_launch_shape best{1.0, 1.0, 1.0, 4, 0};  // start: all grids persistent
        double best_ms = 0.0;
        if (st == AFE_OK) st = time_shape(best, best_ms);
        auto trial = [&](afe_launch_shape cand) -> afe_status {
            if (cand.graph && !(cand.sub > 0.0 && cand.minv > 0.0 && cand.anderson > 0.0)) return AFE_OK;
            double ms = 0.0;
            AFE_TRY(time_shape(cand, ms));
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
            return AFE_OK;
        };
        const double mults[] = {0.0, 1.0, 2.0, 4.0};
        for (double m : mults)
            if (st == AFE_OK && m != best.minv) {
                afe_launch_shape c = best;
                c.minv = m;
                st = trial(c);
            }
        for (double m : mults)
            if (st == AFE_OK && m != best.sub) {
                afe_launch_shape c = best;
                c.sub = m;
                st = trial(c);
            }
        for (double m : mults)
            if (st == AFE_OK && m != best.anderson) {
                afe_launch_shape c = best;
                c.anderson = m;
                st = trial(c);
            }
        const int rounds[] = {2, 4, 8, 16};
        for (int gflag = 0; gflag < 2; ++gflag)
            for (int r : rounds)
                if (st == AFE_OK && !(r == best.rounds && gflag == best.graph)) {
                    afe_launch_shape c = best;
                    c.rounds = r;
                    c.graph = gflag;
                    st = trial(c);
                }
        for (int sl = 0; sl < afe::kMaxSlots; ++sl) {
            E.u[sl] = orig[sl];
            // the predictors left by the trials belong to the working copies
            if (E.cds[sl] && afe::launch_set_count(E.cds[sl]->w.guess_ok, 0, s) != hipSuccess && st == AFE_OK)
                st = fail(AFE_E_HIP, "predictor start reset");
        }
        E.dirty = true;
        E.shape = best;
        E.drop_graphs();
        (void)hipStreamSynchronize(s);
        (void)hipFree(scratch);
        if (st != AFE_OK) return st;
        if (chosen) *chosen = best;
        return AFE_OK;
    });
}

afe_status afe_batch_profile_enable(afe_batch *b, int32_t enable) {
    if (!b) return fail(AFE_E_ARG, "null argument");
    return profile_enable(b->eng, enable);
}

afe_status afe_batch_profile_read(afe_batch *b, double *kernel_ms, int64_t *launches, double *bytes,
                                  double *bytes_stored) {
    if (!b) return fail(AFE_E_ARG, "null argument");
    return profile_read(b->eng, kernel_ms, launches, bytes, bytes_stored);
}

}  // extern "C"
