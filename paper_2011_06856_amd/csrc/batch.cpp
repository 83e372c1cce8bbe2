// batch.cpp -- the batched form of the C ABI: many independent problems of
// uneven size advance together in one launch per step (a persistent
// work-queue launch or a flat launch of every (problem, tile) item), replayed
// from a captured HIP graph, with the launch mode and work-group shape chosen
// by an autotuner.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>

#include "rlbm_internal.h"

struct rlbm_batch_s {
    std::vector<rlbm_ctx> ctx;   // one context per problem (own buffers and tables)
    // problems stepped by the tile kernel (persistent or flat launch) and by
    // the push kernel (one flat launch of 4-row work-groups), by the same
    // automatic choice as a single problem
    std::vector<int> tile_ix, push_ix;
    void* d_pdesc = nullptr;     // push descriptors
    int push_wgs = 0;
    int push_bands = 0;          // bands of 4 rows per work-group group of the push part (0: default)
    int desc_bands = -1;         // band grouping the push descriptors were built for
    int graph_bands = -1;        // band grouping the graph was captured for
    std::string err;
    int prec = RLBM_F32, nmax = 3, max_np = 1, waves = 0, grid = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;     // created here: graphs cannot capture the null stream
    BatchDesc* d_desc = nullptr;
    int* d_counters = nullptr;   // 8 range counters and the exit count, 64 bytes apart
    int* d_bounds = nullptr;     // 9 range bounds of the item list
    int parity = 0;              // buffer holding the current populations
    int total_items = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int mode = RLBM_BATCH_PERSISTENT;
    int graph_waves = -1;        // shape the graph was captured for
    int graph_mode = -1;         // launch mode the graph was captured for
    int desc_waves = -1;         // shape the descriptors were built for
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

int bfail(rlbm_batch b, int code, const std::string& msg)
{
    if (b) b->err = msg;
    return code;
}

int bhip(rlbm_batch b, hipError_t e, const char* where)
{
    return bfail(b, RLBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_graph(rlbm_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_waves = -1;
    b->graph_mode = -1;
    b->graph_bands = -1;
}

int effective_waves(rlbm_batch b)
{
    if (b->waves) return b->waves;
    int nv = 0;   // the largest velocity set of the tile-kernel problems decides the default shape
    for (int i : b->tile_ix) nv = std::max(nv, b->ctx[i]->q.nvel);
    if (!nv) nv = 64;
    return default_waves(b->prec, b->nmax, nv);
}

int effective_bands(rlbm_batch b) { return b->push_bands ? b->push_bands : RLBM_PUSH_BANDS; }

// Upload the descriptors for a work-group shape (chunk sizes depend on it),
// once no launch on the batch's stream reads them any more.
int upload_descs(rlbm_batch b, int waves)
{
    hipError_t se = hipStreamSynchronize(b->st);
    if (se != hipSuccess) return bhip(b, se, "sync");
    std::vector<BatchDesc> d(b->tile_ix.size());
    int item = 0;
    for (size_t i = 0; i < b->tile_ix.size(); ++i) {
        rlbm_ctx c = b->ctx[b->tile_ix[i]];
        d[i].f[0] = c->f[0];
        d[i].f[1] = c->f[1];
        d[i].P = make_params(c, waves);
        d[i].tiles = ((c->nx + 63) / 64) * c->ny;
        d[i].item0 = item;
        item += d[i].tiles;
    }
    b->total_items = item;
    if (d.empty()) {
        b->grid = 0;
        return RLBM_OK;
    }
    std::vector<int> bounds(9);
    for (int k = 0; k <= 8; ++k) bounds[k] = (int)((long long)item * k / 8);
    hipError_t e = hipMemcpy(b->d_desc, d.data(), d.size() * sizeof(BatchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_bounds, bounds.data(), 9 * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(b, e, "descriptor upload");
    b->grid = batch_grid(b->prec, b->nmax, waves, b->max_np);
    if (b->grid < 1) return bfail(b, RLBM_EDEVICE, "no resident work-group for this shape");
    b->grid = std::min(b->grid, std::max(item, 1));
    return RLBM_OK;
}

// One step.  Persistent mode: the persistent step (its work counters are zero
// on entry and left at zero).  Flat mode: one work-group per item.
// Then the push-kernel problems in one flat launch.
hipError_t enqueue_step(rlbm_batch b, int waves, int parity)
{
    hipError_t e = hipSuccess;
    const int nt = (int)b->tile_ix.size();
    if (nt > 0) {
        if (b->mode == RLBM_BATCH_FLAT) {
            e = launch_batch_flat(b->prec, b->nmax, waves, b->total_items, b->d_desc, nt, parity, b->ctx[0]->d_Pc,
                                  b->max_np, b->st);
        } else {
            e = launch_batch_step(b->prec, b->nmax, waves, b->grid, b->d_desc, nt, b->d_counters, b->d_bounds,
                                  parity, b->ctx[0]->d_Pc, b->max_np, b->st);
        }
    }
    if (e == hipSuccess && !b->push_ix.empty())
        e = launch_push_batch(b->prec, b->nmax, b->d_pdesc, (int)b->push_ix.size(), b->push_wgs, parity, b->st);
    return e;
}

// Push-kernel problems: tables, partial-sum buffers and the partial sums of
// the current populations (outside any graph capture), then descriptors for
// the current band grouping.
int prepare_push(rlbm_batch b)
{
    if (b->push_ix.empty()) return RLBM_OK;
    std::vector<rlbm_ctx> cs;
    for (int i : b->push_ix) {
        rlbm_ctx c = b->ctx[i];
        std::string err;
        const int rc = push_prepare(c, err);
        if (rc != RLBM_OK) return bfail(b, rc, "push kernel setup: " + err);
        cs.push_back(c);
    }
    const int bands = effective_bands(b);
    if (!b->d_pdesc || b->desc_bands != bands) {
        drop_graph(b);
        hipError_t e = hipStreamSynchronize(b->st);   // no step in flight reads the old descriptors
        if (e != hipSuccess) return bhip(b, e, "sync");
        b->desc_bands = -1;
        const int rc = push_batch_descs(cs, bands, &b->d_pdesc, &b->push_wgs);
        if (rc != RLBM_OK) return bfail(b, rc, "push descriptors");
        b->desc_bands = bands;
    }
    return RLBM_OK;
}

// Capture two steps (parity 0 then 1) into a graph for the current shape.
int build_graph(rlbm_batch b, int waves)
{
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "begin capture");
    hipError_t e1 = enqueue_step(b, waves, 0);
    hipError_t e2 = e1 == hipSuccess ? enqueue_step(b, waves, 1) : e1;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->st, &g);
    if (e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bhip(b, e2, "captured launch");
    }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return bhip(b, e, "graph instantiate");
    }
    b->graph_waves = waves;
    b->graph_mode = b->mode;
    b->graph_bands = b->desc_bands;
    return RLBM_OK;
}

void set_parity(rlbm_batch b, int parity)
{
    b->parity = parity;
    for (rlbm_ctx c : b->ctx) c->cur = parity;
    for (int i : b->push_ix) b->ctx[i]->pcur = parity;   // partial sums follow the populations
}

int step_impl(rlbm_batch b, int nsteps, int use_graph)
{
    {   // also for nsteps = 0: a graph captured now must hold the push launch
        const int rc = prepare_push(b);
        if (rc != RLBM_OK) return rc;
    }
    const int waves = effective_waves(b);
    if (b->desc_waves != waves) {
        drop_graph(b);
        const int rc = upload_descs(b, waves);
        if (rc != RLBM_OK) return rc;
        b->desc_waves = waves;
    }
    if (use_graph && (b->graph_waves != waves || b->graph_mode != b->mode || b->graph_bands != b->desc_bands)) {
        const int rc = build_graph(b, waves);
        if (rc != RLBM_OK) return rc;
    }
    int s = 0;
    if (b->parity == 1 && nsteps > 0) {   // the graph starts from parity 0
        hipError_t e = enqueue_step(b, waves, 1);
        if (e != hipSuccess) return bhip(b, e, "batch step");
        set_parity(b, 0);
        s = 1;
    }
    if (use_graph && b->exec) {
        for (; s + 2 <= nsteps; s += 2) {
            hipError_t e = hipGraphLaunch(b->exec, b->st);
            if (e != hipSuccess) return bhip(b, e, "graph launch");
        }
    }
    for (; s < nsteps; ++s) {
        hipError_t e = enqueue_step(b, waves, b->parity);
        if (e != hipSuccess) return bhip(b, e, "batch step");
        set_parity(b, b->parity ^ 1);
    }
    for (rlbm_ctx c : b->ctx) c->steps += nsteps;
    return RLBM_OK;
}

}  // namespace

extern "C" {

int rlbm_batch_create(rlbm_batch* out, const rlbm_problem* probs, int count, int precision, void* hip_stream)
{
    if (!out || !probs || count < 1 || count > 65536) return RLBM_EINVAL;
    if (precision != RLBM_F32 && precision != RLBM_F64) return RLBM_EINVAL;
    *out = nullptr;
    rlbm_batch b = new (std::nothrow) rlbm_batch_s();
    if (!b) return RLBM_ENOMEM;
    b->prec = precision;
    b->st = static_cast<hipStream_t>(hip_stream);
    if (!b->st) {
        if (hipStreamCreate(&b->st) != hipSuccess) {
            delete b;
            return RLBM_EDEVICE;
        }
        b->own_stream = true;
    }
    int nmax = -1;
    for (int i = 0; i < count; ++i) {
        const rlbm_problem& p = probs[i];
        if (special_bc(p.bc_x, p.bc_y)) {   // the batch kernels carry no boundary loads
            rlbm_batch_destroy(b);
            return RLBM_EINVAL;
        }
        rlbm_ctx c = nullptr;
        int rc = rlbm_init_quadrature(&c, p.n_radial, p.n_angle, p.order, p.rotate);
        if (rc == RLBM_OK) {
            b->ctx.push_back(c);
            rc = rlbm_init_fields(c, p.nx, p.ny, p.n, p.T, p.ux, p.uy, p.tau, p.dt, p.bc_x, p.bc_y, precision,
                                  nullptr, b->st);
        }
        const int nm = c ? nmax_of(c->q.N) : -1;
        if (rc == RLBM_OK && nmax >= 0 && nm != nmax) rc = RLBM_EINVAL;   // one kernel instance per launch
        if (rc != RLBM_OK) {
            rlbm_batch_destroy(b);
            return rc;
        }
        nmax = nm;
        b->max_np = std::max(b->max_np, c->q.Np);
    }
    b->nmax = nmax;
    for (int i = 0; i < count; ++i)
        (resolve_kernel(b->ctx[i]) == RLBM_KERNEL_PUSH ? b->push_ix : b->tile_ix).push_back(i);
    hipError_t e = hipMalloc(&b->d_desc, sizeof(BatchDesc) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_counters, 9 * 16 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&b->d_bounds, 16 * sizeof(int));
    if (e == hipSuccess) e = hipMemset(b->d_counters, 0, 9 * 16 * sizeof(int));
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e != hipSuccess) {
        rlbm_batch_destroy(b);
        return RLBM_ENOMEM;
    }
    *out = b;
    return RLBM_OK;
}

int rlbm_batch_count(rlbm_batch b) { return b ? (int)b->ctx.size() : RLBM_EINVAL; }

int rlbm_batch_problem(rlbm_batch b, int i, rlbm_ctx* ctx)
{
    if (!b || !ctx || i < 0 || i >= (int)b->ctx.size()) return RLBM_EINVAL;
    *ctx = b->ctx[i];
    return RLBM_OK;
}

int rlbm_batch_set_waves(rlbm_batch b, int waves)
{
    if (!b) return RLBM_EINVAL;
    if (waves < 0 || waves > 16) return bfail(b, RLBM_EINVAL, "waves must be in [0, 16]");
    b->waves = waves;
    return RLBM_OK;
}

int rlbm_batch_get_waves(rlbm_batch b, int* waves)
{
    if (!b || !waves) return RLBM_EINVAL;
    *waves = effective_waves(b);
    return RLBM_OK;
}

int rlbm_batch_step(rlbm_batch b, int nsteps)
{
    if (!b) return RLBM_EINVAL;
    if (nsteps < 0) return bfail(b, RLBM_EINVAL, "nsteps < 0");
    return step_impl(b, nsteps, 1);
}

int rlbm_batch_step_eager(rlbm_batch b, int nsteps)
{
    if (!b) return RLBM_EINVAL;
    if (nsteps < 0) return bfail(b, RLBM_EINVAL, "nsteps < 0");
    return step_impl(b, nsteps, 0);
}

int rlbm_batch_step_timed(rlbm_batch b, int nsteps, double* ms)
{
    if (!b || !ms) return RLBM_EINVAL;
    // shape, descriptors and graph are set up outside the timed region
    int rc = step_impl(b, 0, 1);
    if (rc != RLBM_OK) return rc;
    hipError_t e = hipEventRecord(b->ev0, b->st);
    if (e != hipSuccess) return bhip(b, e, "event");
    if ((rc = step_impl(b, nsteps, 1)) != RLBM_OK) return rc;
    if ((e = hipEventRecord(b->ev1, b->st)) != hipSuccess) return bhip(b, e, "event");
    if ((e = hipEventSynchronize(b->ev1)) != hipSuccess) return bhip(b, e, "event sync");
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, b->ev0, b->ev1)) != hipSuccess) return bhip(b, e, "elapsed");
    *ms = t;
    return RLBM_OK;
}

int rlbm_batch_autotune(rlbm_batch b, const int* candidates, int ncand, int steps, int* best_waves, double* best_ms)
{
    if (!b || !candidates || ncand < 1 || steps < 1) return RLBM_EINVAL;
    hipError_t e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) return bhip(b, e, "sync");
    // the tuning steps change the state: save every problem's populations
    std::vector<void*> saved(b->ctx.size(), nullptr);
    const int parity0 = b->parity;
    int rc = RLBM_OK;
    for (size_t i = 0; i < b->ctx.size() && rc == RLBM_OK; ++i) {
        size_t bytes = 0;
        rlbm_populations_bytes(b->ctx[i], &bytes);
        if (hipMalloc(&saved[i], bytes) != hipSuccess) rc = bfail(b, RLBM_ENOMEM, "autotune backup");
        else if (hipMemcpy(saved[i], b->ctx[i]->f[parity0], bytes, hipMemcpyDeviceToDevice) != hipSuccess)
            rc = bfail(b, RLBM_EDEVICE, "autotune backup copy");
    }
    const int keep = b->waves, keep_mode = b->mode, keep_bands = b->push_bands;
    int bw = 0, bm = keep_mode, bb = keep_bands;
    double bms = 1e300;
    auto trial = [&](double* ms) {
        return step_impl(b, 2, 1) == RLBM_OK &&   // warm-up, graph build
               rlbm_batch_step_timed(b, steps, ms) == RLBM_OK;
    };
    // the tile-kernel part: work-group shape and launch mode
    for (int k = 0; k < ncand && rc == RLBM_OK; ++k)
        for (int mode = RLBM_BATCH_PERSISTENT; mode <= RLBM_BATCH_FLAT; ++mode) {
            const int w = candidates[k];
            if (w < 1 || w > 16) continue;
            b->waves = w;
            b->mode = mode;
            double ms = 0.0;
            if (!trial(&ms)) continue;
            if (ms < bms) {
                bms = ms;
                bw = w;
                bm = mode;
            }
        }
    // the push part, with that shape: bands of 4 rows per work-group group
    if (bw && !b->push_ix.empty() && rc == RLBM_OK) {
        b->waves = bw;
        b->mode = bm;
        for (int sb : {1, 2, 4, 8}) {
            b->push_bands = sb;
            double ms = 0.0;
            if (!trial(&ms)) continue;
            if (ms < bms) {
                bms = ms;
                bb = sb;
            }
        }
    }
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        if (saved[i]) {
            size_t bytes = 0;
            rlbm_populations_bytes(b->ctx[i], &bytes);
            if (rc == RLBM_OK && hipMemcpy(b->ctx[i]->f[parity0], saved[i], bytes, hipMemcpyDeviceToDevice) != hipSuccess)
                rc = bfail(b, RLBM_EDEVICE, "autotune restore");
            (void)hipFree(saved[i]);
        }
    }
    set_parity(b, parity0);
    for (int i : b->push_ix) b->ctx[i]->pvalid = 0;   // populations restored: rebuild their partial sums
    if (rc != RLBM_OK || !bw) {
        b->waves = keep;
        b->mode = keep_mode;
        b->push_bands = keep_bands;
        return rc != RLBM_OK ? rc : bfail(b, RLBM_EDEVICE, "no candidate shape ran");
    }
    b->waves = bw;
    b->mode = bm;
    b->push_bands = bb;
    if (best_waves) *best_waves = bw;
    if (best_ms) *best_ms = bms;
    return RLBM_OK;
}

int rlbm_batch_set_push_bands(rlbm_batch b, int bands)
{
    if (!b) return RLBM_EINVAL;
    if (bands < 0 || bands > 64) return bfail(b, RLBM_EINVAL, "bands must be in [0, 64]");
    b->push_bands = bands;
    return RLBM_OK;
}

int rlbm_batch_get_push_bands(rlbm_batch b, int* bands)
{
    if (!b || !bands) return RLBM_EINVAL;
    *bands = effective_bands(b);
    return RLBM_OK;
}

int rlbm_batch_set_mode(rlbm_batch b, int mode)
{
    if (!b) return RLBM_EINVAL;
    if (mode != RLBM_BATCH_PERSISTENT && mode != RLBM_BATCH_FLAT) return bfail(b, RLBM_EINVAL, "unknown launch mode");
    b->mode = mode;
    return RLBM_OK;
}

int rlbm_batch_get_mode(rlbm_batch b, int* mode)
{
    if (!b || !mode) return RLBM_EINVAL;
    *mode = b->mode;
    return RLBM_OK;
}

int rlbm_batch_info(rlbm_batch b, int* grid, int* items)
{
    if (!b) return RLBM_EINVAL;
    const int waves = effective_waves(b);
    if (b->desc_waves != waves) {
        drop_graph(b);
        const int rc = upload_descs(b, waves);
        if (rc != RLBM_OK) return rc;
        b->desc_waves = waves;
    }
    if (grid) *grid = b->grid;
    if (items) *items = b->total_items;
    return RLBM_OK;
}

const char* rlbm_batch_last_error(rlbm_batch b) { return b ? b->err.c_str() : "null batch"; }

int rlbm_batch_destroy(rlbm_batch b)
{
    if (!b) return RLBM_EINVAL;
    if (b->st) (void)hipStreamSynchronize(b->st);
    drop_graph(b);
    for (rlbm_ctx c : b->ctx) rlbm_destroy(c);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_pdesc) (void)hipFree(b->d_pdesc);
    if (b->d_counters) (void)hipFree(b->d_counters);
    if (b->d_bounds) (void)hipFree(b->d_bounds);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return RLBM_OK;
}

}  // extern "C"
