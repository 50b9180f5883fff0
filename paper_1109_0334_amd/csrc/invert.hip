// invert.hip -- whole PSO inversions as one HIP graph (IP, paper Sec. 2.3 and 3.4).
//
// The paper keeps host-device traffic to a minimum (Sec. 3.1): here a complete inversion --
// swarm initialisation, then for every generation the misfit of all particles followed by the
// swarm update, then the gather of the best positions -- is captured once on the plan's private
// stream and replayed with a single graph launch.  Generation numbers are baked into the
// captured kernel arguments, so a replay needs no host round-trip at all.
#include <algorithm>
#include <numeric>
#include <vector>

#include "afm_internal.hpp"

namespace afm {

struct GraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t S = 0, P = 0, T = 0, lb_steps = 0, lb_k = 0;
    uint64_t seed = 0;
    double cutoff = 0;
    const double *targets = nullptr;
    const int32_t *ncyc = nullptr;
    const double *sparams = nullptr;
    void *ws = nullptr;
};

void release_graph(afm_plan *plan) {
    if (!plan->graph) return;
    if (plan->graph->exec) (void)hipGraphExecDestroy(plan->graph->exec);
    if (plan->graph->graph) (void)hipGraphDestroy(plan->graph->graph);
    delete plan->graph;
    plan->graph = nullptr;
}

namespace {

struct WsLayout {
    size_t bytes;
    size_t z, v, pbest_z, theta, pbest_J, J, gbest_z, gbest_J, gen, status;
    size_t taken, zsel, tsel, nsel, Jsel, bsel, polish;  // polish of the top-k (if requested)
    size_t items, head;                                  // persistent queue (uneven periods)
    size_t order, keys;                                  // lane order within each swarm
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout layout(const afm_plan *plan, int32_t D, int32_t S, int32_t P, int32_t k) {
    const size_t n = (size_t)S * P;
    WsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.z = take(sizeof(double) * D * n);
    L.v = take(sizeof(double) * D * n);
    L.pbest_z = take(sizeof(double) * D * n);
    L.theta = take(sizeof(double) * D * n);
    L.pbest_J = take(sizeof(double) * n);
    L.J = take(sizeof(double) * n);
    L.gbest_z = take(sizeof(double) * D * S);
    L.gbest_J = take(sizeof(double) * S);
    L.gen = take(sizeof(int32_t) * S);
    L.status = take(sizeof(int32_t) * n);
    L.items = take(sizeof(int32_t) * (size_t)S * ((P + 63) / 64));
    L.head = take(sizeof(int32_t));
    L.order = take(sizeof(int32_t) * n);
    L.keys = take(sizeof(double) * n);
    if (k > 0) {
        const size_t m = (size_t)S * k;
        L.taken = take(sizeof(int32_t) * n);
        L.zsel = take(sizeof(double) * D * m);
        L.tsel = take(sizeof(int32_t) * m);
        L.nsel = take(sizeof(int32_t) * m);
        L.Jsel = take(sizeof(double) * m);
        L.bsel = take(sizeof(double) * kMaxParams * m);
        L.polish = take(polish_total_bytes(plan, (int64_t)m, kPolishStride));
    }
    L.bytes = off;
    return L;
}

afm_status ensure_workspace(afm_plan *plan, size_t bytes) {
    if (plan->ws_bytes >= bytes) return AFM_OK;
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "afm_invert workspace sync");
    release_graph(plan);  // captured graphs point into the old workspace
    if (plan->ws) (void)hipFree(plan->ws);
    plan->ws = nullptr;
    plan->ws_bytes = 0;
    e = hipMalloc(&plan->ws, bytes);
    if (e != hipSuccess) return fail(AFM_ERR_NOMEM, "afm_invert: workspace allocation failed");
    plan->ws_bytes = bytes;
    return AFM_OK;
}

}  // namespace

}  // namespace afm

using namespace afm;

extern "C" afm_status afm_invert(afm_plan *plan, int32_t n_swarms, const double *targets,
                                 const int32_t *n_cycles, const double *swarm_params,
                                 int32_t particles, int32_t iters,
                                 uint64_t seed, double cutoff, int32_t lbfgs_steps,
                                 int32_t lbfgs_topk, double *best_theta, double *best_J,
                                 int32_t *gen_to_cutoff, afm_stream_t stream) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    const int32_t D = plan->prob.n_free;
    if (D < 1) return fail(AFM_ERR_INVALID, "the problem has no free parameters");
    if (n_swarms < 1 || particles < 1 || iters < 1)
        return fail(AFM_ERR_INVALID, "n_swarms, particles and iters must be >= 1");
    if ((int64_t)n_swarms * particles > INT32_MAX) return fail(AFM_ERR_INVALID, "swarm too large");
    if (!targets || !best_theta || !best_J || !gen_to_cutoff)
        return fail(AFM_ERR_INVALID, "targets and outputs are required");
    if (lbfgs_steps < 0 || lbfgs_topk < 0 || lbfgs_topk > particles)
        return fail(AFM_ERR_INVALID, "need 0 <= lbfgs_steps and 0 <= lbfgs_topk <= particles");
    if (lbfgs_steps > 0 && lbfgs_topk > 0 && plan->kc.steady_rtol > 0.0)
        return fail(AFM_ERR_UNSUPPORTED, "the adjoint of the adaptive steady-state exit is not built");
    const int32_t kpol = lbfgs_steps > 0 ? lbfgs_topk : 0;
    const WsLayout L = layout(plan, D, n_swarms, particles, kpol);
    afm_status st = ensure_workspace(plan, L.bytes);
    if (st != AFM_OK) return st;
    char *ws = (char *)plan->ws;
    afm_swarm sw{};
    sw.n_dim = D;
    sw.particles = particles;
    sw.swarms = n_swarms;
    sw.z = (double *)(ws + L.z);
    sw.v = (double *)(ws + L.v);
    sw.pbest_z = (double *)(ws + L.pbest_z);
    sw.theta = (double *)(ws + L.theta);
    sw.pbest_J = (double *)(ws + L.pbest_J);
    sw.gbest_z = (double *)(ws + L.gbest_z);
    sw.gbest_J = (double *)(ws + L.gbest_J);
    sw.gen_to_cutoff = (int32_t *)(ws + L.gen);
    double *J = (double *)(ws + L.J);
    int32_t *status = (int32_t *)(ws + L.status);

    GraphCache *g = plan->graph;
    const bool hit = g && g->S == n_swarms && g->P == particles && g->T == iters && g->seed == seed &&
                     g->cutoff == cutoff && g->targets == targets && g->ncyc == n_cycles &&
                     g->ws == plan->ws && g->lb_steps == lbfgs_steps && g->lb_k == kpol &&
                     g->sparams == swarm_params;
    hipError_t e;
    const int32_t chunks = (particles + 63) / 64;
    const int32_t n_items = n_swarms * chunks;
    if (!hit) {
        // a new graph rewrites the plan's workspace (queue order, tuning launches): let earlier
        // replays on the plan's stream finish first
        e = hipStreamSynchronize(plan->stream);
        if (e != hipSuccess) return hip_fail(e, "afm_invert waiting for earlier replays");
    }
    if (!hit && n_cycles) {
        // work queue: the groups' 64-lane chunks, longest period count first (read once, when
        // the graph is built; the order only affects load balance, never the results).  The
        // counts are read on the caller's stream, after the caller's earlier work.
        std::vector<int32_t> nc(n_swarms), items(n_items);
        e = hipMemcpyAsync(nc.data(), n_cycles, sizeof(int32_t) * n_swarms, hipMemcpyDeviceToHost,
                           (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "afm_invert reading n_cycles");
        std::iota(items.begin(), items.end(), 0);
        std::stable_sort(items.begin(), items.end(),
                         [&](int32_t a, int32_t b) { return nc[a / chunks] > nc[b / chunks]; });
        e = hipMemcpy(ws + L.items, items.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "afm_invert queue upload");
    }
    if (!hit) {
        FwdArgs a{};
        a.n = (int64_t)n_swarms * particles;
        a.ld = a.n;
        a.theta = sw.theta;
        a.n_cycles = n_cycles;
        a.targets = targets;
        a.n_targets = n_swarms;
        a.group = particles;
        a.row_by_group = 1;
        a.base = swarm_params;
        a.base_ld = n_swarms;
        if (n_cycles) {
            a.items = (const int32_t *)(ws + L.items);
            a.n_items = n_items;
            a.chunks = chunks;
            a.head = (int32_t *)(ws + L.head);
            a.order_buf = (int32_t *)(ws + L.order);
            a.key_buf = (double *)(ws + L.keys);
        }
        a.J = J;
        a.status = status;
        if (!n_cycles && !forward_shape_known(plan, plan->precision, a)) {
            // the captured forward launches take whatever launch shape the plan holds for this
            // batch size, so let it be tuned first: an eager swarm init and forward, ordered
            // after the caller's earlier work (the graph repeats both)
            e = hipEventRecord(plan->ev_in, (hipStream_t)stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(plan->stream, plan->ev_in, 0);
            if (e == hipSuccess) e = launch_swarm_init(plan, sw, seed, plan->stream);
            if (e == hipSuccess) e = launch_forward(plan, a, plan->stream);
            if (e != hipSuccess) return hip_fail(e, "afm_invert launch-shape tuning");
        }
        release_graph(plan);
        g = new GraphCache();
        plan->graph = g;
        e = hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "afm_invert capture begin");
        e = launch_swarm_init(plan, sw, seed, plan->stream);
        for (int32_t t = 0; t < iters && e == hipSuccess; ++t) {
            e = launch_forward(plan, a, plan->stream);
            if (e == hipSuccess)
                e = launch_pso_step(plan, sw, J, seed, t, t == iters - 1, cutoff, plan->stream);
        }
        if (e == hipSuccess && kpol > 0) {
            const int64_t m = (int64_t)n_swarms * kpol;
            double *zsel = (double *)(ws + L.zsel), *Jsel = (double *)(ws + L.Jsel);
            double *bsel = (double *)(ws + L.bsel);
            int32_t *tsel = (int32_t *)(ws + L.tsel), *nsel = (int32_t *)(ws + L.nsel);
            e = enqueue_topk(plan, sw, kpol, (int32_t *)(ws + L.taken), zsel, tsel, n_cycles, nsel,
                             swarm_params, bsel, plan->stream);
            if (e == hipSuccess)
                e = enqueue_polish(plan, ws + L.polish, m, zsel, tsel, targets, n_swarms,
                                   n_cycles ? nsel : nullptr, swarm_params ? bsel : nullptr,
                                   lbfgs_steps, kPolishStride, Jsel, plan->stream);
            if (e == hipSuccess) e = enqueue_merge(sw, kpol, zsel, Jsel, plan->stream);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(plan->stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            release_graph(plan);
            return hip_fail(e != hipSuccess ? e : e2, "afm_invert capture");
        }
        g->graph = graph;
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            release_graph(plan);
            return hip_fail(e, "afm_invert graph instantiate");
        }
        g->S = n_swarms;
        g->P = particles;
        g->T = iters;
        g->seed = seed;
        g->cutoff = cutoff;
        g->targets = targets;
        g->ncyc = n_cycles;
        g->ws = plan->ws;
        g->lb_steps = lbfgs_steps;
        g->lb_k = kpol;
        g->sparams = swarm_params;
    }
    // order the replay after the caller's earlier work and the caller's later work after it
    e = hipEventRecord(plan->ev_in, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->stream, plan->ev_in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, plan->stream);
    // the results go to the caller's buffers outside the graph, so that a graph is replayed
    // whatever output buffers each call brings
    if (e == hipSuccess)
        e = launch_gather_best(plan, sw, best_theta, best_J, gen_to_cutoff, plan->stream);
    if (e == hipSuccess) e = hipEventRecord(plan->ev_out, plan->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)stream, plan->ev_out, 0);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_invert launch");
}

// One generation's forward solves of afm_invert without the swarm: the misfits of S swarms of P
// points, each swarm against its own target row, period count and parameter vector, through the
// same launch (the persistent work queue, longest period count first, when period counts are
// given; the tuned plain grid otherwise).
extern "C" afm_status afm_misfit_swarms(afm_plan *plan, int32_t n_swarms, int32_t particles,
                                        const double *theta, const int32_t *n_cycles,
                                        const double *swarm_params, const double *targets,
                                        double *J, int32_t *status, afm_stream_t stream) {
    if (!plan) return fail(AFM_ERR_INVALID, "plan is NULL");
    if (n_swarms < 0 || particles < 1) return fail(AFM_ERR_INVALID, "need n_swarms >= 0 and particles >= 1");
    if ((int64_t)n_swarms * particles > INT32_MAX) return fail(AFM_ERR_INVALID, "batch too large");
    if (n_swarms == 0) return AFM_OK;
    if ((plan->prob.n_free > 0 && !theta) || !targets || !J || !status)
        return fail(AFM_ERR_INVALID, "theta, targets, J and status are required");
    const int32_t chunks = (particles + 63) / 64;
    const int32_t n_items = n_swarms * chunks;
    FwdArgs a{};
    a.n = (int64_t)n_swarms * particles;
    a.ld = a.n;
    a.theta = theta;
    a.n_cycles = n_cycles;
    a.targets = targets;
    a.n_targets = n_swarms;
    a.group = particles;
    a.row_by_group = 1;
    a.base = swarm_params;
    a.base_ld = n_swarms;
    a.J = J;
    a.status = status;
    hipError_t e;
    if (n_cycles) {
        // [items, padded to 64][head, 64][lane order, n][keys, n doubles]
        const size_t n = (size_t)n_swarms * particles;
        const size_t off_head = ((size_t)n_items + 63) / 64 * 64;
        const size_t off_order = off_head + 64;
        const size_t off_keys = (off_order + n + 1) / 2 * 2;  // 8-byte aligned, in int32 units
        const size_t bytes = sizeof(int32_t) * (off_keys + 2 * n);
        const bool hit = plan->q_ncyc == n_cycles && plan->q_S == n_swarms &&
                         plan->q_P == particles && plan->qws_bytes >= bytes;
        if (!hit) {
            if (plan->qws_bytes < bytes) {
                if (plan->qws) (void)hipFree(plan->qws);  // waits for work still using it
                plan->qws = nullptr;
                plan->qws_bytes = 0;
                if (hipMalloc(&plan->qws, bytes) != hipSuccess)
                    return fail(AFM_ERR_NOMEM, "afm_misfit_swarms: workspace allocation failed");
                plan->qws_bytes = bytes;
            }
            // longest period count first (the order only balances the load; results do not
            // depend on it); read on the caller's stream after its earlier work
            std::vector<int32_t> nc(n_swarms), items(n_items);
            e = hipMemcpyAsync(nc.data(), n_cycles, sizeof(int32_t) * n_swarms,
                               hipMemcpyDeviceToHost, (hipStream_t)stream);
            if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "afm_misfit_swarms reading n_cycles");
            std::iota(items.begin(), items.end(), 0);
            std::stable_sort(items.begin(), items.end(),
                             [&](int32_t x, int32_t y) { return nc[x / chunks] > nc[y / chunks]; });
            e = hipMemcpy(plan->qws, items.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "afm_misfit_swarms queue upload");
            plan->q_ncyc = n_cycles;
            plan->q_S = n_swarms;
            plan->q_P = particles;
        }
        a.items = (const int32_t *)plan->qws;
        a.n_items = n_items;
        a.chunks = chunks;
        a.head = (int32_t *)plan->qws + off_head;
        a.order_buf = (int32_t *)plan->qws + off_order;
        a.key_buf = reinterpret_cast<double *>((int32_t *)plan->qws + off_keys);
    }
    e = launch_forward(plan, a, (hipStream_t)stream);
    return e == hipSuccess ? AFM_OK : hip_fail(e, "afm_misfit_swarms launch");
}
