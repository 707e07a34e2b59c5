// Batched form: many independent periodic D2Q37 runs of uneven sizes and
// parameters advanced together.  All runs live in one workspace; a device
// run table holds each run's grid, offsets and parameters, and a work list
// splits every run into fixed-size items.  One persistent launch per pass
// walks the work list with a grid stride, and the step loop is captured once
// into a HIP graph that is replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <vector>

#include "holb_cell.h"
#include "holb_host.h"
#include "holb_internal.h"

using namespace holb;

namespace holb {

struct RunDesc {
    int nx, ny, N;
    unsigned flags;
    long long off;     // element offset of the run's Q planes in a population buffer
    long long tab;     // float offset of the run's per-plane frames and shifts in the table region
    long long pitch;   // elements per population plane of this run
    long long cell0;   // offset of the run's cells in the theta field
    float omega, kappa, g0, g1, hfac;
    float rho_ref, thb_ref;
    FastDiv div_nx, div_ny;
    int pad;
};

constexpr int BATCH_ITEM = 256;

__device__ __forceinline__ KParams run_params(const RunDesc& r, unsigned* err, const float* tab)
{
    KParams p = {};
    p.nx = r.nx; p.ny = r.ny; p.nz = 1;
    p.walls = 0;
    p.N = r.N;
    p.nlayer = r.nx;
    p.div_nx = r.div_nx;
    p.div_ny = r.div_ny;
    p.div_layer = r.div_nx;
    p.pitch = r.pitch;
    p.flags = r.flags;
    p.omega = r.omega; p.kappa = r.kappa;
    p.g[0] = r.g0; p.g[1] = r.g1; p.g[2] = 0.f;
    p.hfac = r.hfac;
    p.rho_ref = r.rho_ref;
    p.thb_ref = r.thb_ref;
    p.err = err;
    p.plane_frame = tab + r.tab;
    p.plane_shift = tab + r.tab + 2 * r.ny;
    return p;
}

template <int FAM>
__global__ void __launch_bounds__(BATCH_ITEM)
k_batch_aux(const RunDesc* __restrict__ runs, const int2* __restrict__ items, int nitems, int tile,
            const float* __restrict__ fin, float* __restrict__ aux, const double* __restrict__ tgi, unsigned* err,
            const float* __restrict__ tab)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 t = items[it];
        for (int c0 = t.y;; c0 += BATCH_ITEM) {
            asm volatile("" ::: "memory");
            const RunDesc r = runs[t.x];
            const int end = min(t.y + tile, r.N);
            if (c0 >= end) break;
            const KParams p = run_params(r, err, tab);
            const int cell = c0 + threadIdx.x;
            if (cell < end)
                aux_cell<D2Q37, ST_F32, FAM, false, FM_PLANE>(p, fin + r.off, tgi, aux + r.cell0, nullptr, cell);
        }
    }
}

template <int FAM>
__global__ void __launch_bounds__(BATCH_ITEM)
k_batch_step(const RunDesc* __restrict__ runs, const int2* __restrict__ items, int nitems, int tile,
             const float* __restrict__ fin, float* __restrict__ fout, const float* __restrict__ aux,
             const double* __restrict__ auxd, const double* __restrict__ tgi, double* __restrict__ tgo, unsigned* err,
             const float* __restrict__ tab, float* __restrict__ theta_out)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 t = items[it];
        for (int c0 = t.y;; c0 += BATCH_ITEM) {
            // the run's parameters are re-read per chunk: held across the
            // chunks of an item they would cost a wave of occupancy
            asm volatile("" ::: "memory");
            const RunDesc r = runs[t.x];
            const int end = min(t.y + tile, r.N);
            if (c0 >= end) break;
            const KParams p = run_params(r, err, tab);
            const int cell = c0 + threadIdx.x;
            if (cell < end)
                step_cell<D2Q37, ST_F32, FAM, false, FM_PLANE>(p, fin + r.off, fout + r.off, aux + r.cell0, auxd, tgi,
                                                               tgo, cell, theta_out ? theta_out + r.cell0 : nullptr);
        }
    }
}

}  // namespace holb

struct holb_batch {
    std::vector<holb_config> cfgs;
    std::vector<RunDesc> runs;
    std::vector<int2> items;
    int n = 0;
    int fam = FAM_LOCAL;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    size_t pop_off[2] = {0, 0}, pop_elems = 0, aux_off = 0, aux2_off = 0, desc_off = 0, items_off = 0;
    // grad_lag: the collision reads the theta field of the last step and
    // writes its own into the other one (one launch per step)
    bool lag = false;
    size_t part_off = 0, out_off = 0, err_off = 0, total = 0;
    size_t tab_off = 0;
    int max_partials = 0;
    int cur = 0;
    bool initialized = false;
    int variant = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};

    void drop_graphs()
    {
        for (int k = 0; k < 2; ++k)
            if (graph[k]) {
                (void)hipGraphExecDestroy(graph[k]);
                graph[k] = nullptr;
            }
    }
    ~holb_batch()
    {
        drop_timing();
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }

    const RunDesc* d_runs() const { return (const RunDesc*)(ws + desc_off); }
    const int2* d_items() const { return (const int2*)(ws + items_off); }
    float* pop(int k) const { return (float*)(ws + pop_off[k]); }
    float* aux() const { return (float*)(ws + aux_off); }
    // the theta field of the state in buffer k (grad_lag)
    float* lag_field(int k) const { return (float*)(ws + (k ? aux2_off : aux_off)); }
    float* tab() const { return (float*)(ws + tab_off); }
    unsigned* err() const { return (unsigned*)(ws + err_off); }

    // Launch shape of a variant v in [0, BATCH_VARIANTS): work items of
    // 256 << (v / 3) consecutive cells of one run (a block takes them 256 at a
    // time), and a persistent grid of 4, 8 or 2 blocks per compute unit
    // (v % 3) walking the work list.  Every cell is computed by the same code
    // whichever block takes it, so the variants agree bitwise.
    static int tile_of(int v) { return BATCH_ITEM << (v / 3); }
    static int per_cu_of(int v)
    {
        static const int k[3] = {4, 8, 2};
        return k[v % 3];
    }
    int tile = BATCH_ITEM;  // cells per work item of the uploaded list
    int grid() const { return std::max(1, std::min((int)items.size(), 256 * per_cu_of(variant))); }

    // Work list for items of `t` cells: (run, first cell) of each item.
    void build_items(int t)
    {
        items.clear();
        for (int r = 0; r < n; ++r)
            for (int c0 = 0; c0 < runs[r].N; c0 += t) items.push_back(make_int2(r, c0));
        tile = t;
    }

    // The temperature pass over the state in buffer `from` into `field`.
    hipError_t theta_pass(hipStream_t s, int from, float* field) const
    {
        hipLaunchKernelGGL(k_batch_aux<FAM_THERMAL>, dim3(grid()), dim3(BATCH_ITEM), 0, s, d_runs(), d_items(),
                           (int)items.size(), tile, (const float*)pop(from), field, (const double*)nullptr, err(),
                           (const float*)tab());
        return hipGetLastError();
    }

    // One step: the temperature pass (thermal family, same-step gradient),
    // then the collision kernel, optionally between the two timing events.
    // With grad_lag the collision reads the last step's field and writes
    // this step's: one launch per step.
    hipError_t step_once(hipStream_t s, int from, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) const
    {
        const int nit = (int)items.size();
        const float* fin = pop(from);
        float* fout = pop(1 - from);
        if (lag) {
            if (ev0) {
                hipError_t e = hipEventRecord(ev0, s);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(k_batch_step<FAM_THERMAL>, dim3(grid()), dim3(BATCH_ITEM), 0, s, d_runs(),
                               d_items(), nit, tile, fin, fout, (const float*)lag_field(from), (const double*)nullptr,
                               (const double*)nullptr, (double*)nullptr, err(), (const float*)tab(),
                               lag_field(1 - from));
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
            return e;
        }
        if (fam == FAM_THERMAL) {
            hipLaunchKernelGGL(k_batch_aux<FAM_THERMAL>, dim3(grid()), dim3(BATCH_ITEM), 0, s, d_runs(), d_items(),
                               nit, tile, fin, aux(), (const double*)nullptr, err(), (const float*)tab());
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (ev0) {
            hipError_t e = hipEventRecord(ev0, s);
            if (e != hipSuccess) return e;
        }
        if (fam == FAM_THERMAL)
            hipLaunchKernelGGL(k_batch_step<FAM_THERMAL>, dim3(grid()), dim3(BATCH_ITEM), 0, s, d_runs(),
                               d_items(), nit, tile, fin, fout, (const float*)aux(), (const double*)nullptr,
                               (const double*)nullptr, (double*)nullptr, err(), (const float*)tab(),
                               (float*)nullptr);
        else
            hipLaunchKernelGGL(k_batch_step<FAM_LOCAL>, dim3(grid()), dim3(BATCH_ITEM), 0, s, d_runs(), d_items(),
                               nit, tile, fin, fout, (const float*)aux(), (const double*)nullptr, (const double*)nullptr,
                               (double*)nullptr, err(), (const float*)tab(), (float*)nullptr);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
        return e;
    }

    std::vector<hipEvent_t> timing;  // event pairs of the timed steps
    size_t timed = 0;
    void drop_timing()
    {
        for (hipEvent_t ev : timing) (void)hipEventDestroy(ev);
        timing.clear();
        timed = 0;
    }

    LaunchCtx run_ctx(int r) const
    {
        LaunchCtx c;
        memset(&c, 0, sizeof c);
        c.lattice = HOLB_D2Q37;
        c.storage = ST_F32;
        c.family = fam;
        c.frames = FM_PLANE;
        c.kp = params_of(&cfgs[r]);
        c.kp.pitch = runs[r].pitch;
        c.kp.err = err();
        c.kp.plane_frame = tab() + runs[r].tab;
        c.kp.plane_shift = tab() + runs[r].tab + 2 * runs[r].ny;
        c.pop_in = pop(cur) + runs[r].off;
        c.pop_out = pop(1 - cur) + runs[r].off;
        c.aux_f = aux() + runs[r].cell0;
        c.partials = (double*)(ws + part_off);
        c.max_partials = max_partials;
        c.stream = stream;
        return c;
    }
};

namespace {

holb_status validate_batch(const holb_config* cfgs, int32_t n)
{
    if (!cfgs || n < 1) return fail(HOLB_EINVAL, "need at least one run");
    for (int r = 0; r < n; ++r) {
        holb_status s = validate(&cfgs[r]);
        if (s) return fail(s, "run %d: %s", r, g_last_error.c_str());
        const holb_config& c = cfgs[r];
        if (c.lattice != HOLB_D2Q37 || c.storage != HOLB_STORE_F32 || c.isothermal || c.walls)
            return fail(HOLB_EUNSUPPORTED, "run %d: batches hold periodic, non-isothermal D2Q37 FP32 runs", r);
        if (c.grad_lag != cfgs[0].grad_lag)
            return fail(HOLB_EUNSUPPORTED, "run %d: all runs must share grad_lag", r);
        if (c.frames == HOLB_FRAMES_CELL)
            return fail(HOLB_EUNSUPPORTED, "run %d: batched runs use per-plane frames", r);
        if (c.sources & HOLB_SRC_PTENSOR) return fail(HOLB_EUNSUPPORTED, "run %d: no pressure tensor in batches", r);
        if (family_of(c.sources) != family_of(cfgs[0].sources))
            return fail(HOLB_EUNSUPPORTED, "run %d: all runs must share the thermal source on/off", r);
    }
    return HOLB_OK;
}

void plan(holb_batch* b, const holb_config* cfgs, int n)
{
    b->n = n;
    b->cfgs.assign(cfgs, cfgs + n);
    b->fam = family_of(cfgs[0].sources);
    b->lag = cfgs[0].grad_lag != 0;
    b->runs.resize(n);
    b->items.clear();
    size_t elems = 0, cells = 0, tabf = 0;
    int maxblk = 0;
    for (int r = 0; r < n; ++r) {
        const holb_config& c = cfgs[r];
        RunDesc& d = b->runs[r];
        memset(&d, 0, sizeof d);
        d.nx = c.nx; d.ny = c.ny; d.N = c.nx * c.ny;
        d.div_nx = make_fastdiv((unsigned)c.nx);
        d.div_ny = make_fastdiv((unsigned)c.ny);
        const KParams p = params_of(&c);
        d.flags = p.flags;
        d.omega = p.omega; d.kappa = p.kappa; d.g0 = p.g[0]; d.g1 = p.g[1]; d.hfac = p.hfac;
        d.rho_ref = p.rho_ref;
        d.thb_ref = p.thb_ref;
        d.pitch = (long long)align_up((size_t)d.N, 64);
        d.off = (long long)elems;
        d.cell0 = (long long)cells;
        elems += (size_t)D2Q37::Q * d.pitch;
        d.tab = (long long)tabf;
        tabf += (size_t)(2 + 7 * D2Q37::NS) * c.ny;
        cells += align_up((size_t)d.N, 64);
        maxblk = std::max(maxblk, (d.N + 255) / 256);
    }
    // the list of the smallest items is the longest: the workspace holds it
    b->build_items(BATCH_ITEM);
    b->pop_elems = elems;
    size_t off = 0;
    b->pop_off[0] = off; off = align_up(off + elems * 4);
    b->pop_off[1] = off; off = align_up(off + elems * 4);
    b->aux_off = off; off = align_up(off + cells * 4);
    if (b->lag) {
        b->aux2_off = off;
        off = align_up(off + cells * 4);
    }
    b->tab_off = off; off = align_up(off + tabf * 4);
    b->desc_off = off; off = align_up(off + (size_t)n * sizeof(RunDesc));
    b->items_off = off; off = align_up(off + b->items.size() * sizeof(int2));
    b->max_partials = maxblk;
    b->part_off = off; off = align_up(off + (size_t)maxblk * 5 * sizeof(double));
    b->out_off = off; off = align_up(off + 8 * sizeof(double));
    b->err_off = off; off = align_up(off + sizeof(unsigned));
    b->total = off;
}

holb_status batch_check_flags(holb_batch* b)
{
    unsigned flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, b->err(), sizeof flags, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the error flags");
    if (flags) return fail(HOLB_ENUMERIC, "device numeric error flags 0x%x", flags);
    return HOLB_OK;
}

}  // namespace

extern "C" {

holb_status holb_batch_workspace_size(const holb_config* cfgs, int32_t n_runs, size_t* bytes)
{
    holb_status s = validate_batch(cfgs, n_runs);
    if (s) return s;
    if (!bytes) return fail(HOLB_EINVAL, "bytes is NULL");
    holb_batch tmp;
    plan(&tmp, cfgs, n_runs);
    *bytes = tmp.total;
    return HOLB_OK;
}

holb_status holb_batch_create(const holb_config* cfgs, int32_t n_runs, void* dev_workspace, size_t bytes,
                              void* hip_stream, holb_batch** out)
{
    if (!out) return fail(HOLB_EINVAL, "out is NULL");
    *out = nullptr;
    holb_status s = validate_batch(cfgs, n_runs);
    if (s) return s;
    if (!dev_workspace) return fail(HOLB_EINVAL, "workspace is NULL");
    if ((uintptr_t)dev_workspace % ALIGN) return fail(HOLB_ESIZE, "workspace must be 256-byte aligned");
    holb_batch* b = new (std::nothrow) holb_batch();
    if (!b) return fail(HOLB_EINVAL, "out of host memory");
    plan(b, cfgs, n_runs);
    if (bytes < b->total) {
        size_t need = b->total;
        delete b;
        return fail(HOLB_ESIZE, "workspace has %zu bytes, needs %zu", bytes, need);
    }
    b->ws = (char*)dev_workspace;
    b->stream = (hipStream_t)hip_stream;
    // Upload the run table and work list (host copies live in the handle).
    hipError_t e = hipMemcpyAsync(b->ws + b->desc_off, b->runs.data(), b->runs.size() * sizeof(RunDesc),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->items_off, b->items.data(), b->items.size() * sizeof(int2),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->err(), 0, sizeof(unsigned), b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "uploading the run table");
    }
    *out = b;
    return HOLB_OK;
}

holb_status holb_batch_init(holb_batch* b, const float* const* rho, const float* const* u,
                            const float* const* theta)
{
    if (!b || !rho || !u || !theta) return fail(HOLB_EINVAL, "NULL argument");
    for (int r = 0; r < b->n; ++r) {
        if (!rho[r] || !u[r] || !theta[r]) return fail(HOLB_EINVAL, "run %d: NULL field", r);
        LaunchCtx c = b->run_ctx(r);
        c.pop_out = b->pop(b->cur) + b->runs[r].off;
        hipError_t e = launch_init(c, rho[r], u[r], theta[r]);
        if (e != hipSuccess) return hip_fail(e, "batched init");
    }
    if (b->lag) {
        // the theta field of the initial state, which the first step reads
        hipError_t e = b->theta_pass(b->stream, b->cur, b->lag_field(b->cur));
        if (e != hipSuccess) return hip_fail(e, "initial theta field");
    }
    b->initialized = true;
    return HOLB_OK;
}

// Steps per captured graph (even: a replay ends in the buffer it started from).
static const int BATCH_GRAPH_STEPS = 16;

static holb_status ensure_graph(holb_batch* b, int from)
{
    if (b->graph[from]) return HOLB_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t e2 = hipSuccess;
    for (int k = 0; k < BATCH_GRAPH_STEPS && e2 == hipSuccess; ++k) e2 = b->step_once(b->cap, (from + k) % 2);
    e = hipStreamEndCapture(b->cap, &g);
    if (e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e2, "capturing the step loop");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph[from] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return HOLB_OK;
}

holb_status holb_batch_step(holb_batch* b, int64_t n)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    if (n < 0) return fail(HOLB_EINVAL, "n must be >= 0");
    if (!b->initialized) return fail(HOLB_ESTATE, "holb_batch_step before holb_batch_init");
    if (!b->timing.empty()) {
        // timed steps run eagerly, each collision launch between two events
        for (int64_t k = 0; k < n; ++k) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (2 * (b->timed + 1) <= b->timing.size()) {
                e0 = b->timing[2 * b->timed];
                e1 = b->timing[2 * b->timed + 1];
                ++b->timed;
            }
            hipError_t e = b->step_once(b->stream, b->cur, e0, e1);
            if (e != hipSuccess) return hip_fail(e, "batched step");
            b->cur = 1 - b->cur;
        }
        return HOLB_OK;
    }
    if (n >= BATCH_GRAPH_STEPS) {
        holb_status s = ensure_graph(b, b->cur);
        if (s) return s;
        for (; n >= BATCH_GRAPH_STEPS; n -= BATCH_GRAPH_STEPS) {
            hipError_t e = hipGraphLaunch(b->graph[b->cur], b->stream);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
    }
    for (; n > 0; --n) {
        hipError_t e = b->step_once(b->stream, b->cur);
        if (e != hipSuccess) return hip_fail(e, "batched step");
        b->cur = 1 - b->cur;
    }
    return HOLB_OK;
}

holb_status holb_batch_fields(holb_batch* b, int32_t run, float* rho, float* u, float* theta)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    if (run < 0 || run >= b->n) return fail(HOLB_EINVAL, "run %d out of range", run);
    if (!b->initialized) return fail(HOLB_ESTATE, "fields before init");
    hipError_t e = launch_fields(b->run_ctx(run), rho, u, theta);
    if (e != hipSuccess) return hip_fail(e, "batched fields");
    return batch_check_flags(b);
}

holb_status holb_batch_reduce(holb_batch* b, int32_t run, double out[5])
{
    if (!b || !out) return fail(HOLB_EINVAL, "NULL argument");
    if (run < 0 || run >= b->n) return fail(HOLB_EINVAL, "run %d out of range", run);
    if (!b->initialized) return fail(HOLB_ESTATE, "reduce before init");
    double* dout = (double*)(b->ws + b->out_off);
    hipError_t e = launch_reduce(b->run_ctx(run), dout);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 5 * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batched reduce");
    return batch_check_flags(b);
}

// launch shapes: work items of 256, 512, 1024 or 2048 cells x 4, 8 or 2
// blocks per compute unit (holb_batch::tile_of, per_cu_of)
static const int BATCH_VARIANTS = 12;

holb_status holb_batch_set_variant(holb_batch* b, int32_t variant)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    if (variant < 0 || variant >= BATCH_VARIANTS) return fail(HOLB_EUNSUPPORTED, "variant %d not available", variant);
    if (variant == b->variant) return HOLB_OK;
    b->drop_graphs();
    const int t = holb_batch::tile_of(variant);
    if (t != b->tile) {
        // a new work list (never longer than the one the workspace was sized for)
        b->build_items(t);
        hipError_t e = hipMemcpyAsync(b->ws + b->items_off, b->items.data(), b->items.size() * sizeof(int2),
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, "uploading the work list");
    }
    b->variant = variant;
    return HOLB_OK;
}

holb_status holb_batch_timing_start(holb_batch* b, int32_t max_steps)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    if (max_steps < 1 || max_steps > 100000) return fail(HOLB_EINVAL, "max_steps must be in [1, 100000]");
    b->drop_timing();
    b->timing.resize(2 * (size_t)max_steps, nullptr);
    for (auto& ev : b->timing) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            ev = nullptr;
            b->drop_timing();
            return hip_fail(e, "hipEventCreate");
        }
    }
    return HOLB_OK;
}

holb_status holb_batch_timing_stop(holb_batch* b, double* kernel_ms, int64_t* launches, int64_t* cells_per_launch,
                                   char* kernel, size_t kernel_len)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    double total = 0.0;
    hipError_t e = hipSuccess;
    if (b->timed) e = hipEventSynchronize(b->timing[2 * b->timed - 1]);
    for (size_t k = 0; k < b->timed && e == hipSuccess; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, b->timing[2 * k], b->timing[2 * k + 1]);
        total += ms;
    }
    const int64_t n = (int64_t)b->timed;
    b->drop_timing();
    if (e != hipSuccess) return hip_fail(e, "reading the timing events");
    long long cells = 0;
    for (const RunDesc& r : b->runs) cells += r.N;
    if (kernel && kernel_len)
        snprintf(kernel, kernel_len, "k_batch_step<%d>", b->fam);
    if (kernel_ms) *kernel_ms = total;
    if (launches) *launches = n;
    if (cells_per_launch) *cells_per_launch = cells;
    return HOLB_OK;
}

holb_status holb_batch_tune(holb_batch* b, int32_t* variant_out)
{
    if (!b) return fail(HOLB_EINVAL, "handle is NULL");
    if (!b->initialized) return fail(HOLB_ESTATE, "tune before init");
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    // per shape the fastest of three timings of 4 steps, in round-robin passes
    float vms[BATCH_VARIANTS];
    for (int v = 0; v < BATCH_VARIANTS; ++v) vms[v] = 1e30f;
    for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
        for (int v = 0; v < BATCH_VARIANTS && e == hipSuccess; ++v) {
            holb_status st = holb_batch_set_variant(b, v);
            if (st != HOLB_OK) {
                (void)hipEventDestroy(t0);
                (void)hipEventDestroy(t1);
                return st;
            }
            // trial steps read the current buffer and write the other one
            e = b->step_once(b->stream, b->cur);
            if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
            for (int r = 0; r < 4 && e == hipSuccess; ++r) e = b->step_once(b->stream, b->cur);
            if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess) vms[v] = std::min(vms[v], ms);
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "batched tuning");
    int best = 0;
    for (int v = 1; v < BATCH_VARIANTS; ++v)
        if (vms[v] < vms[best]) best = v;
    holb_status st = holb_batch_set_variant(b, best);
    if (st != HOLB_OK) return st;
    if (variant_out) *variant_out = best;
    return HOLB_OK;
}

holb_status holb_batch_destroy(holb_batch* b)
{
    delete b;
    return HOLB_OK;
}

}  // extern "C"
