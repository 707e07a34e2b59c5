// C ABI of the library: configuration checks, workspace layout, state
// bookkeeping and dispatch to the kernel launchers.  No device memory is
// allocated here; the caller owns the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/holb.h"
#include "holb_host.h"
#include "holb_internal.h"

using namespace holb;

namespace holb {
thread_local std::string g_last_error;
}

namespace {

struct Layout {
    size_t elem = 4;          // bytes per stored population
    size_t pitch = 0;         // elements per population plane
    size_t pop_bytes = 0;     // one population buffer
    size_t tab_off = 0, tab_bytes = 0;  // per-plane frames and shifts (FP32 storage)
    int nm = 0;               // planes along the last axis
    size_t pop_off[2] = {0, 0};
    size_t aux_off = 0, aux_bytes = 0, aux2_off = 0;
    size_t tgt_off[2] = {0, 0};
    size_t tgt_bytes = 0;
    size_t wall_off = 0, wall_bytes = 0;  // solved wall-node targets and fluid-layer masses (FP64)
    size_t part_off = 0;
    int max_partials = 0;
    size_t out_off = 0;
    size_t err_off = 0;
    size_t total = 0;
};

Layout layout_of(const holb_config* c)
{
    Layout L;
    const int Q = lattice_Q(c->lattice), D = lattice_D(c->lattice);
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    L.elem = c->storage == HOLB_STORE_F32 ? 4 : 2;
    L.pitch = align_up(N, ALIGN / L.elem);
    // Q population planes; with per-cell frames, then one binary16 pair (rho,
    // theta - 1) per cell: the frame the cell's populations are stored in
    // (with momentum, a second such plane of packed momentum words).
    // Per-plane frames are kept in a table of (2 + 7 NS) floats per plane.
    const int fm = frames_of(c);
    const bool per_cell = fm != FM_PLANE;
    L.pop_bytes = (size_t)Q * L.pitch * L.elem + (per_cell ? align_up(N * 4) * (fm == FM_CELLU ? 2 : 1) : 0);
    L.nm = D == 3 ? c->nz : c->ny;
    L.tab_bytes = per_cell ? 0 : (size_t)(2 + 7 * lattice_NS(c->lattice)) * L.nm * sizeof(float);
    size_t off = 0;
    L.pop_off[0] = off; off = align_up(off + L.pop_bytes);
    L.pop_off[1] = off; off = align_up(off + L.pop_bytes);
    L.tab_off = off; off = align_up(off + L.tab_bytes);
    const int fam = family_of(c->sources);
    L.aux_bytes = fam == FAM_PTENSOR ? N * 8 : (fam == FAM_THERMAL ? N * 4 : 0);
    L.aux_off = off; off = align_up(off + L.aux_bytes);
    // with the previous step's gradient: a second theta field (the two swap
    // roles every step, like the population buffers)
    L.aux2_off = off; off = align_up(off + (c->grad_lag ? L.aux_bytes : 0));
    if (c->walls) {
        const size_t nlayer = D == 2 ? (size_t)c->nx : (size_t)c->nx * c->ny;
        L.tgt_bytes = (TGT_SLOTS * (size_t)(D + 2) + 2 * 16) * nlayer * sizeof(double);
        L.wall_bytes = (2 * WSOL_COMPS + 2 * 2) * nlayer * sizeof(double) + 2 * WCLOSED_SLOTS * nlayer * sizeof(float);
    }
    L.tgt_off[0] = off; off = align_up(off + L.tgt_bytes);
    L.tgt_off[1] = off; off = align_up(off + L.tgt_bytes);
    L.wall_off = off; off = align_up(off + L.wall_bytes);
    L.max_partials = (int)((N + 255) / 256);
    L.part_off = off; off = align_up(off + (size_t)L.max_partials * 5 * sizeof(double));
    L.out_off = off; off = align_up(off + 8 * sizeof(double));
    L.err_off = off; off = align_up(off + sizeof(unsigned));
    L.total = off;
    return L;
}

}  // namespace

struct holb_sim {
    holb_config cfg;
    Layout lay;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;            // buffer holding the current state
    bool initialized = false;
    int variant = 0;
    LaunchCtx base;
    std::vector<hipEvent_t> timing;  // event pairs of the timed steps
    size_t timed = 0;                // pairs recorded so far
    // Step loop as HIP graphs of GRAPH_STEPS steps, one per starting buffer
    // (captured on a private stream when first needed, replayed on the
    // caller's stream).
    hipStream_t cap = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // Walled domains: the stream and events of the wall work of a step
    // (created with the first step).
    hipStream_t side = nullptr;
    hipEvent_t side_ev[3] = {nullptr, nullptr, nullptr};

    void drop_timing()
    {
        for (hipEvent_t e : timing) (void)hipEventDestroy(e);
        timing.clear();
        timed = 0;
    }
    void drop_graphs()
    {
        for (int k = 0; k < 2; ++k)
            if (graph[k]) {
                (void)hipGraphExecDestroy(graph[k]);
                graph[k] = nullptr;
            }
    }
    ~holb_sim()
    {
        drop_timing();
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (hipEvent_t e : side_ev)
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }

    LaunchCtx ctx(bool advance) const
    {
        LaunchCtx c = base;
        const int nxt = 1 - cur;
        c.pop_in = ws + lay.pop_off[cur];
        c.pop_out = ws + lay.pop_off[nxt];
        c.tgt_in = (const double*)(ws + lay.tgt_off[cur]);
        c.tgt_out = (double*)(ws + lay.tgt_off[advance ? nxt : cur]);
        if (cfg.grad_lag) {
            // a step reads the last step's theta and writes its own; passes
            // that do not step (fields, totals) get the other field as
            // scratch for the wall closure's theta output, which the next
            // step overwrites whole
            float* th[2] = {(float*)(ws + lay.aux_off), (float*)(ws + lay.aux2_off)};
            c.aux_f = advance ? th[cur] : th[nxt];
            c.theta_out = advance ? th[nxt] : nullptr;
        }
        c.variant = variant;
        if (side) {
            c.side = side;
            c.ev_fork = side_ev[0];
            c.ev_wall = side_ev[1];
            c.ev_join = side_ev[2];
        }
        return c;
    }
};

// The second stream of a walled simulation and its events.
static holb_status ensure_side(holb_sim* s)
{
    if (!s->cfg.walls || s->side) return HOLB_OK;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        if (!s->side_ev[k]) e = hipEventCreateWithFlags(&s->side_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "creating the wall-stream events");
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "creating the wall stream");
    s->side = st;
    return HOLB_OK;
}

// With the previous step's gradient: the theta field the next step reads is
// part of the state.
static size_t lag_bytes(const holb_sim* s) { return s->cfg.grad_lag ? s->lay.aux_bytes : 0; }
static char* lag_field(const holb_sim* s) { return s->ws + (s->cur ? s->lay.aux2_off : s->lay.aux_off); }

extern "C" {

const char* holb_last_error(void) { return g_last_error.c_str(); }

holb_status holb_lattice_info(int32_t lattice, int32_t* Q, int32_t* D, int32_t* c, double* w, double* c0sq)
{
    if (lattice != HOLB_D2Q37 && lattice != HOLB_D3Q39) return fail(HOLB_EINVAL, "unknown lattice %d", lattice);
    if (Q) *Q = lattice_Q(lattice);
    if (D) *D = lattice_D(lattice);
    std::vector<int> cc(3 * 39);
    lattice_table(lattice, cc.data(), w, c0sq);
    if (c)
        for (int k = 0; k < 3 * lattice_Q(lattice); ++k) c[k] = cc[k];
    return HOLB_OK;
}

holb_status holb_workspace_size(const holb_config* cfg, size_t* bytes)
{
    holb_status s = validate(cfg);
    if (s) return s;
    if (!bytes) return fail(HOLB_EINVAL, "bytes is NULL");
    *bytes = layout_of(cfg).total;
    return HOLB_OK;
}

holb_status holb_create(const holb_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                        holb_sim** out)
{
    if (!out) return fail(HOLB_EINVAL, "out is NULL");
    *out = nullptr;
    holb_status s = validate(cfg);
    if (s) return s;
    Layout L = layout_of(cfg);
    if (!dev_workspace) return fail(HOLB_EINVAL, "workspace is NULL");
    if ((uintptr_t)dev_workspace % ALIGN) return fail(HOLB_ESIZE, "workspace must be 256-byte aligned");
    if (bytes < L.total) return fail(HOLB_ESIZE, "workspace has %zu bytes, needs %zu", bytes, L.total);
    holb_sim* h = new (std::nothrow) holb_sim();
    if (!h) return fail(HOLB_EINVAL, "out of host memory");
    h->cfg = *cfg;
    h->lay = L;
    h->ws = (char*)dev_workspace;
    h->stream = (hipStream_t)hip_stream;
    LaunchCtx& c = h->base;
    memset(&c, 0, sizeof c);
    c.lattice = cfg->lattice;
    c.storage = cfg->storage;
    c.family = family_of(cfg->sources);
    c.frames = frames_of(cfg);
    c.kp = params_of(cfg);
    c.kp.err = (unsigned*)(h->ws + L.err_off);
    c.kp.pitch = (long long)L.pitch;
    if (L.tab_bytes) {
        c.kp.plane_frame = (const float*)(h->ws + L.tab_off);
        c.kp.plane_shift = c.kp.plane_frame + 2 * L.nm;
    }
    if (L.wall_bytes) {
        const size_t nlayer = c.kp.nlayer;
        c.kp.wsol = (double*)(h->ws + L.wall_off);
        c.kp.mflu = c.kp.wsol + 2 * WSOL_COMPS * nlayer;
        c.kp.wclosed = (float*)(c.kp.mflu + 2 * 2 * nlayer);
    }
    c.aux_f = L.aux_bytes ? (float*)(h->ws + L.aux_off) : nullptr;
    c.aux_d = L.aux_bytes ? (double*)(h->ws + L.aux_off) : nullptr;
    c.partials = (double*)(h->ws + L.part_off);
    c.max_partials = L.max_partials;
    c.stream = h->stream;
    *out = h;
    return HOLB_OK;
}

static holb_status check_flags(holb_sim* s)
{
    unsigned flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, s->ws + s->lay.err_off, sizeof flags, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the error flags");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (flags) return fail(HOLB_ENUMERIC, "device numeric error flags 0x%x (1 density, 2 theta, 4 EOS, 8 wall closure)", flags);
    return HOLB_OK;
}

holb_status holb_init(holb_sim* s, const float* rho, const float* u, const float* theta)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (!rho || !u || (!theta && !s->cfg.isothermal)) return fail(HOLB_EINVAL, "field pointer is NULL");
    if (((uintptr_t)rho | (uintptr_t)u | (uintptr_t)theta) % 4) return fail(HOLB_ESIZE, "fields must be 4-byte aligned");
    hipError_t e = hipMemsetAsync(s->ws + s->lay.err_off, 0, sizeof(unsigned), s->stream);
    if (e != hipSuccess) return hip_fail(e, "clearing the error flags");
    // The init kernel writes the pre-streamed equilibrium into the current
    // buffer and the initial fields as the wall targets of the first step.
    LaunchCtx c = s->ctx(false);
    c.pop_out = s->ws + s->lay.pop_off[s->cur];
    c.tgt_out = (double*)(s->ws + s->lay.tgt_off[s->cur]);
    e = launch_init(c, rho, u, theta ? theta : rho);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    if (s->cfg.grad_lag) {
        // the theta field of the initial state, which the first step's
        // gradient reads
        LaunchCtx ca = s->ctx(false);
        ca.aux_f = (float*)lag_field(s);
        e = launch_aux(ca);
        if (e != hipSuccess) return hip_fail(e, "initial theta field");
    }
    s->initialized = true;
    return HOLB_OK;
}

// Steps per captured graph (even: a replay leaves the state in the buffer it
// started from).
static const int GRAPH_STEPS = 16;

static holb_status ensure_graph(holb_sim* s, int from)
{
    if (s->graph[from]) return HOLB_OK;
    hipError_t e = hipSuccess;
    if (!s->cap) e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "creating the capture stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t el = hipSuccess;
    int cur = from;
    for (int k = 0; k < GRAPH_STEPS && el == hipSuccess; ++k) {
        LaunchCtx c = s->ctx(true);
        // the context of the step k of the replay, on the capture stream
        const int nxt = 1 - cur;
        c.pop_in = s->ws + s->lay.pop_off[cur];
        c.pop_out = s->ws + s->lay.pop_off[nxt];
        c.tgt_in = (const double*)(s->ws + s->lay.tgt_off[cur]);
        c.tgt_out = (double*)(s->ws + s->lay.tgt_off[nxt]);
        if (s->cfg.grad_lag) {
            float* th[2] = {(float*)(s->ws + s->lay.aux_off), (float*)(s->ws + s->lay.aux2_off)};
            c.aux_f = th[cur];
            c.theta_out = th[nxt];
        }
        c.stream = s->cap;
        el = launch_step(c);
        cur = nxt;
    }
    e = hipStreamEndCapture(s->cap, &g);
    if (el != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(el, "capturing the step loop");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->graph[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph[from] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return HOLB_OK;
}

holb_status holb_step(holb_sim* s, int64_t n)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (n < 0) return fail(HOLB_EINVAL, "n must be >= 0");
    if (!s->initialized) return fail(HOLB_ESTATE, "holb_step before holb_init");
    if (n == 0) return HOLB_OK;
    holb_status ss = ensure_side(s);
    if (ss) return ss;
    if (s->timing.empty() && n >= GRAPH_STEPS) {
        // untimed: whole graphs of GRAPH_STEPS steps, the rest eagerly
        holb_status st = ensure_graph(s, s->cur);
        if (st) return st;
        for (; n >= GRAPH_STEPS; n -= GRAPH_STEPS) {
            hipError_t e = hipGraphLaunch(s->graph[s->cur], s->stream);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        LaunchCtx c = s->ctx(true);
        if (2 * (s->timed + 1) <= s->timing.size()) {
            c.ev_begin = s->timing[2 * s->timed];
            c.ev_end = s->timing[2 * s->timed + 1];
            ++s->timed;
        }
        hipError_t e = launch_step(c);
        if (e != hipSuccess) return hip_fail(e, "step kernel");
        s->cur = 1 - s->cur;
    }
    return HOLB_OK;
}

holb_status holb_fields(holb_sim* s, float* rho, float* u, float* theta)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (!s->initialized) return fail(HOLB_ESTATE, "holb_fields before holb_init");
    if (((uintptr_t)rho | (uintptr_t)u | (uintptr_t)theta) % 4) return fail(HOLB_ESIZE, "fields must be 4-byte aligned");
    hipError_t e = launch_fields(s->ctx(false), rho, u, theta);
    if (e != hipSuccess) return hip_fail(e, "fields kernel");
    return check_flags(s);
}

holb_status holb_reduce(holb_sim* s, double out[5])
{
    if (!s || !out) return fail(HOLB_EINVAL, "NULL argument");
    if (!s->initialized) return fail(HOLB_ESTATE, "holb_reduce before holb_init");
    double* dout = (double*)(s->ws + s->lay.out_off);
    hipError_t e = launch_reduce(s->ctx(false), dout);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel");
    e = hipMemcpyAsync(out, dout, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "copying the totals");
    return check_flags(s);
}

// holb_reduce_noalloc: the block partials (5 doubles per 256-cell block) and
// the 5 totals in a file-scope device array.  Host code never uses the
// array's name as an address: its device address is looked up once per
// device (hipGetSymbolAddress) and kept.
namespace {
constexpr int NOALLOC_BLOCKS = HOLB_NOALLOC_MAX_CELLS / 256;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) double scratch[(size_t)NOALLOC_BLOCKS * 5 + 8];

static holb_status scratch_of_current_device(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HOLB_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch array");
        g_scratch_dev[dev] = (double*)ptr;
    }
    *out = g_scratch_dev[dev];
    return HOLB_OK;
}

holb_status holb_reduce_noalloc(holb_sim* s, double out[5])
{
    if (!s || !out) return fail(HOLB_EINVAL, "NULL argument");
    const int nb = reduce_blocks(s->base);
    if (nb > NOALLOC_BLOCKS)
        return fail(HOLB_ESIZE, "holb_reduce_noalloc takes at most %d cells, the grid has %d", HOLB_NOALLOC_MAX_CELLS,
                    s->base.kp.N);
    if (!s->initialized) return fail(HOLB_ESTATE, "holb_reduce_noalloc before holb_init");
    double* sp = nullptr;
    holb_status st = scratch_of_current_device(&sp);
    if (st) return st;
    LaunchCtx c = s->ctx(false);
    c.partials = sp;
    c.max_partials = NOALLOC_BLOCKS;
    double* dout = sp + (size_t)NOALLOC_BLOCKS * 5;
    hipError_t e = launch_reduce(c, dout);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel");
    e = hipMemcpyAsync(out, dout, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "copying the totals");
    return check_flags(s);
}

holb_status holb_error_flags(holb_sim* s, uint32_t* flags)
{
    if (!s || !flags) return fail(HOLB_EINVAL, "NULL argument");
    unsigned f = 0;
    hipError_t e = hipMemcpyAsync(&f, s->ws + s->lay.err_off, sizeof f, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the error flags");
    *flags = f;
    return HOLB_OK;
}

// State blob: the current population buffer, then the per-plane table (if
// any), then the wall targets of the next step (walled domains: the last
// step's rho, u, theta on the three layers next to each wall).

holb_status holb_state_bytes(holb_sim* s, size_t* bytes)
{
    if (!s || !bytes) return fail(HOLB_EINVAL, "NULL argument");
    *bytes = s->lay.pop_bytes + s->lay.tab_bytes + s->lay.tgt_bytes + lag_bytes(s);
    return HOLB_OK;
}

holb_status holb_get_state(holb_sim* s, void* dst, size_t bytes)
{
    if (!s || !dst) return fail(HOLB_EINVAL, "NULL argument");
    const size_t pb = s->lay.pop_bytes, tb = s->lay.tab_bytes, gb = s->lay.tgt_bytes, lb = lag_bytes(s);
    if (bytes != pb + tb + gb + lb)
        return fail(HOLB_ESIZE, "state is %zu bytes, got %zu", pb + tb + gb + lb, bytes);
    hipError_t e = hipMemcpyAsync(dst, s->ws + s->lay.pop_off[s->cur], pb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && lb)
        e = hipMemcpyAsync((char*)dst + pb + tb + gb, lag_field(s), lb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && tb)
        e = hipMemcpyAsync((char*)dst + pb, s->ws + s->lay.tab_off, tb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && gb)
        e = hipMemcpyAsync((char*)dst + pb + tb, s->ws + s->lay.tgt_off[s->cur], gb, hipMemcpyDeviceToDevice,
                           s->stream);
    if (e != hipSuccess) return hip_fail(e, "copying the state out");
    return HOLB_OK;
}

holb_status holb_set_state(holb_sim* s, const void* src, size_t bytes)
{
    if (!s || !src) return fail(HOLB_EINVAL, "NULL argument");
    const size_t pb = s->lay.pop_bytes, tb = s->lay.tab_bytes, gb = s->lay.tgt_bytes, lb = lag_bytes(s);
    if (bytes != pb + tb + gb + lb)
        return fail(HOLB_ESIZE, "state is %zu bytes, got %zu", pb + tb + gb + lb, bytes);
    // a fresh simulation may take a state without holb_init: clear its flags
    hipError_t e = hipMemsetAsync(s->ws + s->lay.err_off, 0, sizeof(unsigned), s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->ws + s->lay.pop_off[s->cur], src, pb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && tb)
        e = hipMemcpyAsync(s->ws + s->lay.tab_off, (const char*)src + pb, tb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && gb)
        e = hipMemcpyAsync(s->ws + s->lay.tgt_off[s->cur], (const char*)src + pb + tb, gb, hipMemcpyDeviceToDevice,
                           s->stream);
    if (e == hipSuccess && lb)
        e = hipMemcpyAsync(lag_field(s), (const char*)src + pb + tb + gb, lb, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "copying the state in");
    s->initialized = true;
    return HOLB_OK;
}

holb_status holb_num_variants(holb_sim* s, int32_t* n)
{
    if (!s || !n) return fail(HOLB_EINVAL, "NULL argument");
    *n = num_variants(s->base);
    return HOLB_OK;
}

holb_status holb_set_variant(holb_sim* s, int32_t variant)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (variant < 0 || variant >= num_variants(s->base) || !variant_supported(s->base, variant))
        return fail(HOLB_EUNSUPPORTED, "variant %d does not apply to this configuration", variant);
    if (variant != s->variant) s->drop_graphs();  // captured with the old variant
    s->variant = variant;
    return HOLB_OK;
}

holb_status holb_tune(holb_sim* s, int32_t* variant_out)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (!s->initialized) return fail(HOLB_ESTATE, "holb_tune before holb_init");
    holb_status ss = ensure_side(s);
    if (ss) return ss;
    // Trial steps read the current buffer and write the other one (and the
    // other wall-target buffer); the current state is left untouched.
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    // Per variant the fastest of three timings of 4 steps, taken in
    // round-robin passes so that a slow phase of the device favours none.
    const int nv = num_variants(s->base);
    std::vector<float> vms((size_t)nv, 1e30f);
    for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
        for (int v = 0; v < nv && e == hipSuccess; ++v) {
            if (!variant_supported(s->base, v)) continue;
            LaunchCtx c = s->ctx(true);
            c.variant = v;
            e = launch_step(c);  // warm-up
            if (e != hipSuccess) break;
            e = hipEventRecord(t0, s->stream);
            for (int r = 0; r < 4 && e == hipSuccess; ++r) e = launch_step(c);
            if (e == hipSuccess) e = hipEventRecord(t1, s->stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess) vms[(size_t)v] = std::min(vms[(size_t)v], ms);
        }
    }
    int best = s->variant;
    for (int v = 0; v < nv; ++v)
        if (vms[(size_t)v] < vms[(size_t)best]) best = v;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "tuning");
    if (best != s->variant) s->drop_graphs();
    s->variant = best;
    if (variant_out) *variant_out = best;
    return HOLB_OK;
}

holb_status holb_timing_start(holb_sim* s, int32_t max_steps)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    if (max_steps < 1 || max_steps > 100000) return fail(HOLB_EINVAL, "max_steps must be in [1, 100000]");
    s->drop_timing();
    s->timing.resize(2 * (size_t)max_steps, nullptr);
    for (auto& ev : s->timing) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            ev = nullptr;
            s->drop_timing();
            return hip_fail(e, "hipEventCreate");
        }
    }
    return HOLB_OK;
}

holb_status holb_timing_stop(holb_sim* s, double* kernel_ms, int64_t* launches, int64_t* cells_per_launch,
                             char* kernel, size_t kernel_len)
{
    if (!s) return fail(HOLB_EINVAL, "handle is NULL");
    double total = 0.0;
    hipError_t e = hipSuccess;
    if (s->timed) e = hipEventSynchronize(s->timing[2 * s->timed - 1]);
    for (size_t k = 0; k < s->timed && e == hipSuccess; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, s->timing[2 * k], s->timing[2 * k + 1]);
        total += ms;
    }
    const int64_t n = (int64_t)s->timed;
    s->drop_timing();
    if (e != hipSuccess) return hip_fail(e, "reading the timing events");
    long long cells = 0;
    LaunchCtx c = s->ctx(true);
    dominant_kernel(c, kernel, kernel_len, &cells);
    if (kernel_ms) *kernel_ms = total;
    if (launches) *launches = n;
    if (cells_per_launch) *cells_per_launch = cells;
    return HOLB_OK;
}

holb_status holb_destroy(holb_sim* s)
{
    delete s;
    return HOLB_OK;
}

}  // extern "C"
