// Context management and the exported C ABI of libmbh (see include/mbh.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mbh.h"
#include "mbh_internal.h"

using namespace mbh;

// Workspace of mbh_loglike_batch_noalloc, for callers that cannot allocate
// device memory: one fixed array per GPU, held until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (in host
// code the name 'scratch' is not a device address) and only that address is
// passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct mbh_ctx {
    mbh_ctx_desc desc;
    Modes md;
    GridDesc g;
    int max_batch;
    int max_items;
    int precision;
    // resident data
    double2 *d = nullptr;
    double *w = nullptr;
    double *pre = nullptr;
    float2 *dhi32 = nullptr;      // FP32 dense stage only
    float2 *dlo32 = nullptr;
    float *sw32 = nullptr;
    // workspace
    Work wk;
    double *params = nullptr;     // [max_batch][11] staging for graph launches
    double *logL = nullptr;       // [max_batch]
    std::vector<void *> allocs;
    // one captured likelihood graph per batch size; the nodes of its first
    // kernel (reads the walker parameters) and last kernel (writes ln L) are
    // pointed at the caller's buffers before each launch
    struct GraphEntry {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t src = nullptr, red = nullptr;
        int src_nargs = 0;                // arguments of the kernel in node src (the parameters are argument 0)
        const double *params = nullptr;   // buffers the exec's nodes use now
        double *logL = nullptr;
    };
    std::map<int, GraphEntry> graphs;
    hipGraph_t graph_tmp = nullptr;
    std::string err;
    // stage order of the staged calls: the last completed stage over the
    // workspace (0 none, 1 waveform_gen, 2 response or a full evaluation) and
    // the batch size it covered
    int stage = 0;
    int stage_B = 0;
    bool timing = false;
    Schedule sch;                 // dense launch shape (mbh_set_schedule / mbh_autotune)
    int device = 0;               // device the context was created on
    unsigned char *scratch_dev = nullptr;   // that device's copy of 'scratch' (null if unavailable)
    std::string scratch_err;      // why scratch_dev is null
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};

namespace {

const char *kNoCtx = "mbh: null context";

mbh_status fail(mbh_ctx *c, mbh_status st, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

mbh_status hip_fail(mbh_ctx *c, hipError_t e, const char *where)
{
    return fail(c, MBH_EHIP, "mbh: %s failed: %s", where, hipGetErrorString(e));
}

template <typename T>
mbh_status dalloc(mbh_ctx *c, T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    const char *inj = getenv("MBH_FAULT_INJECT");
    if (inj && strcmp(inj, "alloc") == 0) return fail(c, MBH_ENOMEM, "mbh: injected allocation failure");
    void *raw = nullptr;
    hipError_t e = hipMalloc(&raw, count * sizeof(T));
    if (e != hipSuccess || raw == nullptr) {
        (void)hipGetLastError();
        return fail(c, MBH_ENOMEM, "mbh: hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    c->allocs.push_back(raw);
    *p = static_cast<T *>(raw);
    return MBH_OK;
}

void drop_events(mbh_ctx *c)
{
    for (auto &ev : c->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    c->events.clear();
}

void drop_graphs(mbh_ctx *c)
{
    for (auto &kv : c->graphs) {
        (void)hipGraphExecDestroy(kv.second.exec);
        (void)hipGraphDestroy(kv.second.graph);
    }
    c->graphs.clear();
}

void release(mbh_ctx *c)
{
    drop_events(c);
    drop_graphs(c);
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

bool mode_ok(int l, int m)
{
    return (l == 2 && m == 2) || (l == 3 && m == 3) || (l == 4 && m == 4) || (l == 2 && m == 1) ||
           (l == 3 && m == 2) || (l == 4 && m == 3);
}

Data data_of(const mbh_ctx *c) { return Data{c->d, c->w, c->pre, c->dhi32, c->dlo32, c->sw32}; }

// The workspace must hold stage 'need' (or later) for exactly B walkers.
mbh_status check_stage(mbh_ctx *c, int need, int B, const char *call)
{
    if (B == 0) return MBH_OK;
    if (c->stage < need || c->stage_B != B)
        return fail(c, MBH_EINVAL, "mbh: %s needs a preceding %s with the same B (workspace holds stage %d for B = %d)",
                    call, need == 1 ? "mbh_waveform_gen" : "mbh_response", c->stage, c->stage_B);
    return MBH_OK;
}

void set_stage(mbh_ctx *c, int stage, int B)
{
    c->stage = stage;
    c->stage_B = B;
}

mbh_status check_B(mbh_ctx *c, int B)
{
    if (B < 0) return fail(c, MBH_EINVAL, "mbh: negative batch %d", B);
    if (B > c->max_batch) return fail(c, MBH_EBATCH, "mbh: batch %d exceeds max_batch %d", B, c->max_batch);
    return MBH_OK;
}

// The three stages, enqueued on st.
mbh_status enqueue_all(mbh_ctx *c, const double *params, int B, double *out7, double *logL, hipStream_t st,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    hipError_t e;
    // small batches: the sparse stage as one kernel; larger ones: one kernel
    // per step.  One walker (tickets) needs no item list: the sparse kernel
    // zeroes the counter and the dense kernel takes the walker's tiles.
    const bool fused = B <= kFusedSparseMaxBatch;
    const bool one = fused && B == 1 && !c->sch.one_per_walker;
    if (fused) {
        if ((e = launch_sparse(params, B, c->md, c->g, c->wk, one, st)) != hipSuccess)
            return hip_fail(c, e, "sparse");
    } else {
        if ((e = launch_waveform(params, B, c->md, c->g, c->wk, st)) != hipSuccess) return hip_fail(c, e, "waveform");
        if ((e = launch_response(B, c->md, c->g, c->wk, st)) != hipSuccess) return hip_fail(c, e, "response");
        if ((e = launch_spline(B, c->md, c->g, c->wk, st)) != hipSuccess) return hip_fail(c, e, "spline");
    }
    if ((e = launch_coef32(B, c->md, c->g, c->wk, st)) != hipSuccess) return hip_fail(c, e, "coef32");
    if ((e = launch_walker_bands(B, c->md, c->g, c->wk, st)) != hipSuccess) return hip_fail(c, e, "bands");
    if ((e = launch_dense(B, c->md, c->g, c->wk, data_of(c), c->max_items, c->sch, false, st, ev0, ev1, one)) !=
        hipSuccess)
        return hip_fail(c, e, "dense");
    if ((e = launch_reduce(B, c->g, c->wk, data_of(c), out7, logL, st)) != hipSuccess) return hip_fail(c, e, "reduce");
    return MBH_OK;
}

// The kernel node of 'fn' in a captured graph (nullptr if absent).
hipGraphNode_t find_kernel_node(hipGraph_t graph, const void *fn)
{
    size_t nn = 0;
    if (hipGraphGetNodes(graph, nullptr, &nn) != hipSuccess || nn == 0) return nullptr;
    std::vector<hipGraphNode_t> nodes(nn);
    if (hipGraphGetNodes(graph, nodes.data(), &nn) != hipSuccess) return nullptr;
    for (hipGraphNode_t n : nodes) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(n, &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if (hipGraphKernelNodeGetParams(n, &kp) != hipSuccess) continue;
        if (kp.func == fn && kp.kernelParams != nullptr) return n;
    }
    return nullptr;
}

// Point argument 'arg' (a device pointer) of kernel node 'node' of 'exec' at p;
// the other arguments keep their captured values.
hipError_t retarget(hipGraphExec_t exec, hipGraphNode_t node, int arg, int nargs, const void *p)
{
    hipKernelNodeParams kp;
    hipError_t e = hipGraphKernelNodeGetParams(node, &kp);
    if (e != hipSuccess) return e;
    std::vector<void *> args(kp.kernelParams, kp.kernelParams + nargs);
    args[arg] = &p;
    kp.kernelParams = args.data();
    return hipGraphExecKernelNodeSetParams(exec, node, &kp);
}

// Device address of 'scratch' on each device, taken once per device with
// that device current.
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;

// Sets c->scratch_dev for the current device (c->scratch_err on failure).
void bind_scratch(mbh_ctx *c)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        c->scratch_err = std::string("hipGetDevice failed: ") + hipGetErrorString(e);
        return;
    }
    auto it = g_scratch_addr.find(c->device);
    if (it == g_scratch_addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            c->scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return;
        }
        it = g_scratch_addr.emplace(c->device, static_cast<unsigned char *>(p)).first;
    }
    c->scratch_dev = it->second;
}

// Per-call workspace of B walkers carved from base (256-byte aligned
// pieces); returns the bytes it needs.  base == nullptr only measures.
// The read-only sin/cos tables stay the context's.
size_t carve_workspace(const mbh_ctx *c, int B, unsigned char *base, Work *wk, int *max_items)
{
    const int nm = c->md.nm, ns = c->g.ns;
    const long long ntile_max = (c->g.n + c->g.tile_bins - 1) / c->g.tile_bins + 1;
    const long long items = (long long)B * ntile_max;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? static_cast<void *>(base + off) : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        return p;
    };
    Work w = {};
    w.src = static_cast<Source *>(take(sizeof(Source) * B));
    w.band = static_cast<ModeBand *>(take(sizeof(ModeBand) * B * nm));
    w.wband = static_cast<WalkerBand *>(take(sizeof(WalkerBand) * B));
    w.kf = static_cast<double *>(take(sizeof(double) * B * nm * ns));
    w.kt = static_cast<double *>(take(sizeof(double) * B * nm * ns));
    w.fn = static_cast<double *>(take(sizeof(double) * B * nm * kNumFn * ns));
    w.coef = static_cast<double *>(take(sizeof(double) * B * nm * (ns - 1) * kCoefPerIv));
    w.kbin = static_cast<int *>(take(sizeof(int) * B * nm * ns));
    w.item_w = static_cast<int *>(take(sizeof(int) * items));
    w.item_t = static_cast<int *>(take(sizeof(int) * items));
    w.tile_off = static_cast<int *>(take(sizeof(int) * (ntile_max + 1)));
    w.ticket = static_cast<int *>(take(sizeof(int) * 64));
    w.wbase = static_cast<int *>(take(sizeof(int) * (B + 1)));
    w.partial = static_cast<double *>(take(sizeof(double) * items * kPartials));
    w.out7 = nullptr;
    if (c->precision == MBH_FP32C) w.coef32 = static_cast<float *>(take(sizeof(float) * B * nm * (ns - 1) * kCoefPerIv));
    w.cis_tab = c->wk.cis_tab;
    w.cis32 = c->wk.cis32;
    if (wk) *wk = w;
    if (max_items) *max_items = (int)std::min<long long>(items, 0x7fffffffLL);
    return off;
}

}  // namespace

extern "C" {

int mbh_version(void) { return 100; }

const char *mbh_last_error(const mbh_ctx *ctx) { return ctx ? ctx->err.c_str() : kNoCtx; }

mbh_status mbh_ctx_create(const mbh_ctx_desc *desc, mbh_ctx **out)
{
    if (!out) return MBH_EINVAL;
    *out = nullptr;
    if (!desc || !desc->data || !desc->psd) return MBH_EINVAL;
    if (!(desc->df > 0.0) || !std::isfinite(desc->df) || desc->k0 < 1 || desc->n < 4 ||
        desc->k0 + desc->n > (int64_t)0x7fffffff)
        return MBH_EINVAL;
    if (desc->n_modes < 1 || desc->n_modes > kMaxModes) return MBH_EINVAL;
    if (desc->n_sparse < 8 || desc->n_sparse > 1024) return MBH_EINVAL;
    if (desc->max_batch < 1 || desc->max_batch > (1 << 16)) return MBH_EINVAL;
    if (desc->precision != MBH_FP64 && desc->precision != MBH_FP32C) return MBH_EINVAL;
    if (!std::isfinite(desc->t0)) return MBH_EINVAL;
    for (int i = 0; i < desc->n_modes; ++i) {
        if (!mode_ok(desc->modes[i][0], desc->modes[i][1])) return MBH_EINVAL;
        for (int j = 0; j < i; ++j)
            if (desc->modes[i][0] == desc->modes[j][0] && desc->modes[i][1] == desc->modes[j][1]) return MBH_EINVAL;
    }
    const int64_t n = desc->n;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!(desc->psd[i] > 0.0) || !std::isfinite(desc->psd[i])) return MBH_EINVAL;

    mbh_ctx *c = new (std::nothrow) mbh_ctx();
    if (!c) return MBH_ENOMEM;
    c->desc = *desc;
    c->desc.data = nullptr;
    c->desc.psd = nullptr;
    c->md.nm = desc->n_modes;
    for (int i = 0; i < kMaxModes; ++i) {
        c->md.l[i] = i < desc->n_modes ? desc->modes[i][0] : 0;
        c->md.m[i] = i < desc->n_modes ? desc->modes[i][1] : 0;
    }
    c->g.df = desc->df;
    c->g.t0 = desc->t0;
    c->g.k0 = (int)desc->k0;
    c->g.n = (int)n;
    c->g.ns = desc->n_sparse;
    c->g.precision = desc->precision;
    c->max_batch = desc->max_batch;
    c->precision = desc->precision;
    c->g.steps = dense_steps(n, desc->max_batch);
    c->g.tile_bins = kDenseThreads * c->g.steps;
    const long long ntile_max = (n + c->g.tile_bins - 1) / c->g.tile_bins + 1;
    const long long items = (long long)desc->max_batch * ntile_max;
    if (items > 0x7fffffffLL) { delete c; return MBH_EINVAL; }
    c->max_items = (int)items;

    const int B = desc->max_batch, nm = desc->n_modes, ns = desc->n_sparse;
    mbh_status st = MBH_OK;
    double *psd_dev = nullptr, *scratch = nullptr;
    const size_t nchunks = (size_t)((n + 2047) / 2048);
#define TRY(x)                       \
    do {                             \
        if ((st = (x)) != MBH_OK) {  \
            release(c);              \
            delete c;                \
            return st;               \
        }                            \
    } while (0)
    const size_t n_pad = (size_t)data_padded(n);
    double2 *d_in = nullptr;      // the data as uploaded, [3][n]; freed after set-up
    TRY(dalloc(c, &c->d, 3 * n_pad));
    TRY(dalloc(c, &c->w, 3 * n_pad));
    TRY(dalloc(c, &d_in, (size_t)3 * n));
    TRY(dalloc(c, &c->pre, (size_t)3 * (n + 1)));
    TRY(dalloc(c, &psd_dev, (size_t)3 * n));
    TRY(dalloc(c, &scratch, (size_t)3 * n + 3 * nchunks));
    TRY(dalloc(c, &c->wk.src, (size_t)B));
    TRY(dalloc(c, &c->wk.band, (size_t)B * nm));
    TRY(dalloc(c, &c->wk.wband, (size_t)B));
    TRY(dalloc(c, &c->wk.kf, (size_t)B * nm * ns));
    TRY(dalloc(c, &c->wk.kt, (size_t)B * nm * ns));
    TRY(dalloc(c, &c->wk.fn, (size_t)B * nm * kNumFn * ns));
    TRY(dalloc(c, &c->wk.coef, (size_t)B * nm * (ns - 1) * kCoefPerIv));
    TRY(dalloc(c, &c->wk.kbin, (size_t)B * nm * ns));
    TRY(dalloc(c, &c->wk.item_w, (size_t)c->max_items));
    TRY(dalloc(c, &c->wk.item_t, (size_t)c->max_items));
    TRY(dalloc(c, &c->wk.tile_off, (size_t)ntile_max + 1));
    TRY(dalloc(c, &c->wk.ticket, (size_t)64));
    TRY(dalloc(c, &c->wk.wbase, (size_t)B + 1));
    TRY(dalloc(c, &c->wk.partial, (size_t)c->max_items * kPartials));
    TRY(dalloc(c, &c->wk.out7, (size_t)B * 7));
    TRY(dalloc(c, &c->wk.cis_tab, (size_t)kCisTabDoubles));
    TRY(dalloc(c, &c->wk.cis32, (size_t)32));
    if (desc->precision == MBH_FP32C) {
        TRY(dalloc(c, &c->dhi32, (size_t)3 * n));
        TRY(dalloc(c, &c->dlo32, (size_t)3 * n));
        TRY(dalloc(c, &c->sw32, (size_t)3 * n));
        TRY(dalloc(c, &c->wk.coef32, (size_t)B * nm * (ns - 1) * kCoefPerIv));
    }
    TRY(dalloc(c, &c->params, (size_t)B * 11));
    TRY(dalloc(c, &c->logL, (size_t)B));
#undef TRY
    hipError_t e;
    int ncis = 0, ncis32 = 0;
    const double *cis_host = cis_table_host(&ncis);
    const float *cis32_host = cis32_table_host(&ncis32);
    if ((e = hipMemcpy(c->wk.cis_tab, cis_host, sizeof(double) * ncis, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->wk.cis32, cis32_host, sizeof(float) * ncis32, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_in, desc->data, sizeof(double) * 6 * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(c->wk.src, 0, sizeof(Source) * B)) != hipSuccess ||
        (e = hipMemset(c->wk.band, 0, sizeof(ModeBand) * B * nm)) != hipSuccess ||
        (e = hipMemcpy(psd_dev, desc->psd, sizeof(double) * 3 * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = launch_setup_data(psd_dev, d_in, c->d, c->w, c->pre, scratch, c->dhi32, c->dlo32, c->sw32, c->g,
                               4.0 * desc->df, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        release(c);
        delete c;
        return MBH_EHIP;
    }
    // the uploaded data, the PSD copy and the setup scratch are no longer needed
    for (auto it = c->allocs.begin(); it != c->allocs.end();) {
        if (*it == psd_dev || *it == scratch || *it == d_in) {
            (void)hipFree(*it);
            it = c->allocs.erase(it);
        } else {
            ++it;
        }
    }
    bind_scratch(c);
    *out = c;
    return MBH_OK;
}

void mbh_ctx_destroy(mbh_ctx *ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    release(ctx);
    delete ctx;
}

mbh_status mbh_waveform_gen(mbh_ctx *ctx, const double *params_dev, int B, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (B > 0 && !params_dev) return fail(ctx, MBH_EINVAL, "mbh: null params");
    set_stage(ctx, 0, 0);
    hipError_t e = launch_waveform(params_dev, B, ctx->md, ctx->g, ctx->wk, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "waveform_gen");
    set_stage(ctx, 1, B);
    return MBH_OK;
}

mbh_status mbh_response(mbh_ctx *ctx, int B, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if ((st = check_stage(ctx, 1, B, "mbh_response"))) return st;
    hipError_t e = launch_response(B, ctx->md, ctx->g, ctx->wk, (hipStream_t)stream);
    if (e == hipSuccess) e = launch_spline(B, ctx->md, ctx->g, ctx->wk, (hipStream_t)stream);
    if (e == hipSuccess) e = launch_coef32(B, ctx->md, ctx->g, ctx->wk, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "response");
    if (B > 0) set_stage(ctx, 2, B);
    return MBH_OK;
}

mbh_status mbh_interp_and_inner(mbh_ctx *ctx, int B, double *out7_dev, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (B > 0 && !out7_dev) return fail(ctx, MBH_EINVAL, "mbh: null out7");
    if ((st = check_stage(ctx, 2, B, "mbh_interp_and_inner"))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_walker_bands(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_dense(B, ctx->md, ctx->g, ctx->wk, data_of(ctx), ctx->max_items, ctx->sch, true, s);
    if (e == hipSuccess) e = launch_reduce(B, ctx->g, ctx->wk, data_of(ctx), out7_dev, nullptr, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "interp_and_inner");
    return MBH_OK;
}

mbh_status mbh_loglike_batch(mbh_ctx *ctx, const double *params_dev, int B, double *logL_dev, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (B == 0) return MBH_OK;
    if (!params_dev || !logL_dev) return fail(ctx, MBH_EINVAL, "mbh: null params or logL");
    set_stage(ctx, 0, 0);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (ctx->timing) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(ctx, e, "event create");
        if ((e = hipEventCreate(&e1)) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return hip_fail(ctx, e, "event create");
        }
        ctx->events.emplace_back(e0, e1);
        st = enqueue_all(ctx, params_dev, B, ctx->wk.out7, logL_dev, s, e0, e1);
        if (st != MBH_OK) return st;
        set_stage(ctx, 2, B);
        return MBH_OK;
    }
    auto it = ctx->graphs.find(B);
    if (it == ctx->graphs.end()) {
        // capture the fixed sequence of kernels for this batch size on a
        // private stream (with the context's staging buffers), then
        // instantiate it and find the two nodes that touch caller memory
        hipStream_t cap;
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return hip_fail(ctx, e, "stream");
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = enqueue_all(ctx, ctx->params, B, ctx->wk.out7, ctx->logL, cap);
            hipError_t e2 = hipStreamEndCapture(cap, &graph);
            if (st == MBH_OK && e2 != hipSuccess) st = hip_fail(ctx, e2, "end capture");
        } else {
            st = hip_fail(ctx, e, "begin capture");
        }
        (void)hipStreamDestroy(cap);
        if (st != MBH_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        mbh_ctx::GraphEntry ge;
        ge.graph = graph;
        ge.src = find_kernel_node(graph, source_kernel());
        ge.src_nargs = 4;
        if (!ge.src) {
            ge.src = find_kernel_node(graph, sparse_kernel(ctx->g.ns));
            ge.src_nargs = 5;
        }
        ge.red = find_kernel_node(graph, reduce_kernel());
        ge.params = ctx->params;
        ge.logL = ctx->logL;
        e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(ctx, e, "graph instantiate");
        }
        it = ctx->graphs.emplace(B, ge).first;
    }
    mbh_ctx::GraphEntry &ge = it->second;
    // the first kernel reads params (argument 0 of 4 in k_source, of 5 in
    // k_sparse), the last writes ln L (argument 8 of 9); where a node was not
    // found, the parameters and ln L go through the context's staging
    // buffers instead
    const bool direct_in = ge.src != nullptr, direct_out = ge.red != nullptr;
    if (direct_in && ge.params != params_dev) {
        if ((e = retarget(ge.exec, ge.src, 0, ge.src_nargs, params_dev)) != hipSuccess)
            return hip_fail(ctx, e, "graph node update");
        ge.params = params_dev;
    }
    if (direct_out && ge.logL != logL_dev) {
        if ((e = retarget(ge.exec, ge.red, 8, 9, logL_dev)) != hipSuccess) return hip_fail(ctx, e, "graph node update");
        ge.logL = logL_dev;
    }
    if (!direct_in &&
        (e = hipMemcpyAsync(ctx->params, params_dev, sizeof(double) * 11 * B, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(ctx, e, "params copy");
    if ((e = hipGraphLaunch(ge.exec, s)) != hipSuccess) return hip_fail(ctx, e, "graph launch");
    if (!direct_out &&
        (e = hipMemcpyAsync(logL_dev, ctx->logL, sizeof(double) * B, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(ctx, e, "logL copy");
    set_stage(ctx, 2, B);
    return MBH_OK;
}

mbh_status mbh_loglike_batch_noalloc(mbh_ctx *ctx, const double *params_dev, int B, double *logL_dev, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (B == 0) return MBH_OK;
    if (!params_dev || !logL_dev) return fail(ctx, MBH_EINVAL, "mbh: null params or logL");
    if (!ctx->scratch_dev) return fail(ctx, MBH_EHIP, "mbh: no static workspace on this device (%s)", ctx->scratch_err.c_str());
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
    if (dev != ctx->device)
        return fail(ctx, MBH_EINVAL, "mbh: context belongs to device %d but device %d is current", ctx->device, dev);
    const size_t need = carve_workspace(ctx, B, nullptr, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(ctx, MBH_EBATCH,
                    "mbh: B = %d needs %zu bytes of workspace, more than the %zu-byte static workspace of "
                    "mbh_loglike_batch_noalloc (use a smaller batch or mbh_loglike_batch)",
                    B, need, kScratchBytes);
    Work wk;
    int max_items = 0;
    carve_workspace(ctx, B, ctx->scratch_dev, &wk, &max_items);
    // the same kernels in the same order as the graph of mbh_loglike_batch;
    // every scratch value is written before it is read (the tile list
    // kernels reset the work-item counter), so nothing is cleared here
    hipStream_t s = (hipStream_t)stream;
    const Data dt = data_of(ctx);
    if ((e = launch_waveform(params_dev, B, ctx->md, ctx->g, wk, s)) != hipSuccess) return hip_fail(ctx, e, "waveform");
    if ((e = launch_response(B, ctx->md, ctx->g, wk, s)) != hipSuccess) return hip_fail(ctx, e, "response");
    if ((e = launch_spline(B, ctx->md, ctx->g, wk, s)) != hipSuccess) return hip_fail(ctx, e, "spline");
    if ((e = launch_coef32(B, ctx->md, ctx->g, wk, s)) != hipSuccess) return hip_fail(ctx, e, "coef32");
    if ((e = launch_walker_bands(B, ctx->md, ctx->g, wk, s)) != hipSuccess) return hip_fail(ctx, e, "bands");
    if ((e = launch_dense(B, ctx->md, ctx->g, wk, dt, max_items, ctx->sch, false, s)) != hipSuccess)
        return hip_fail(ctx, e, "dense");
    if ((e = launch_reduce(B, ctx->g, wk, dt, nullptr, logL_dev, s)) != hipSuccess) return hip_fail(ctx, e, "reduce");
    return MBH_OK;
}

mbh_status mbh_set_timing(mbh_ctx *ctx, int on)
{
    if (!ctx) return MBH_EINVAL;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "sync");
    drop_events(ctx);
    ctx->timing = on != 0;
    return MBH_OK;
}

mbh_status mbh_get_timing(mbh_ctx *ctx, double *dense_ms_total, int64_t *count)
{
    if (!ctx) return MBH_EINVAL;
    double total = 0.0;
    for (auto &ev : ctx->events) {
        hipError_t e = hipEventSynchronize(ev.second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
        if (e != hipSuccess) return hip_fail(ctx, e, "event timing");
        total += ms;
    }
    if (dense_ms_total) *dense_ms_total = total;
    if (count) *count = (int64_t)ctx->events.size();
    return MBH_OK;
}

mbh_status mbh_set_schedule(mbh_ctx *ctx, int blocks_per_cu, int one_per_walker)
{
    if (!ctx) return MBH_EINVAL;
    if (blocks_per_cu < 1 || blocks_per_cu > 32)
        return fail(ctx, MBH_EINVAL, "mbh: blocks_per_cu %d outside [1, 32]", blocks_per_cu);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "sync");
    drop_graphs(ctx);
    ctx->sch.blocks_per_cu = blocks_per_cu;
    ctx->sch.one_per_walker = one_per_walker != 0;
    return MBH_OK;
}

mbh_status mbh_get_schedule(const mbh_ctx *ctx, int *blocks_per_cu, int *one_per_walker)
{
    if (!ctx) return MBH_EINVAL;
    if (blocks_per_cu) *blocks_per_cu = ctx->sch.blocks_per_cu;
    if (one_per_walker) *one_per_walker = ctx->sch.one_per_walker;
    return MBH_OK;
}

mbh_status mbh_autotune(mbh_ctx *ctx, const double *params_dev, int B, int reps, int *best_bpc_host,
                        double *best_ms_host, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    if (B < 1) return fail(ctx, MBH_EINVAL, "mbh: autotune needs B >= 1");
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (!params_dev) return fail(ctx, MBH_EINVAL, "mbh: null params");
    if (reps < 1 || reps > 100) return fail(ctx, MBH_EINVAL, "mbh: reps %d outside [1, 100]", reps);
    set_stage(ctx, 0, 0);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_waveform(params_dev, B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_response(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_spline(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_coef32(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_walker_bands(B, ctx->md, ctx->g, ctx->wk, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune stages");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(ctx, e, "event create");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(ctx, e, "event create");
    }
    static const int kCand[] = {2, 3, 4, 6, 8, 9, 12, 16, 24, 32};
    int best = ctx->sch.blocks_per_cu;
    double best_ms = 1e300;
    for (int c : kCand) {
        Schedule sch;
        sch.blocks_per_cu = c;
        std::vector<float> ms;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = launch_dense(B, ctx->md, ctx->g, ctx->wk, data_of(ctx), ctx->max_items, sch, false, s, e0, e1);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            ms.push_back(t);
        }
        if (e != hipSuccess) break;
        std::sort(ms.begin(), ms.end());
        const double med = ms[ms.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    drop_graphs(ctx);
    ctx->sch.blocks_per_cu = best;
    ctx->sch.one_per_walker = 0;
    set_stage(ctx, 2, B);
    if (best_bpc_host) *best_bpc_host = best;
    if (best_ms_host) *best_ms_host = best_ms;
    return MBH_OK;
}

mbh_status mbh_template(mbh_ctx *ctx, const double *params_dev, double *h_dev, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    if (!params_dev || !h_dev) return fail(ctx, MBH_EINVAL, "mbh: null params or h");
    set_stage(ctx, 0, 0);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_waveform(params_dev, 1, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_response(1, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_spline(1, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_walker_bands(1, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_template(ctx->md, ctx->g, ctx->wk, reinterpret_cast<double2 *>(h_dev), s);
    if (e != hipSuccess) return hip_fail(ctx, e, "template");
    set_stage(ctx, 2, 1);
    return MBH_OK;
}

mbh_status mbh_get_sparse(mbh_ctx *ctx, int w, int64_t *band_host, double *fband_host, double *f_host,
                          double *fn_host, double *coef_host, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    if (w < 0 || w >= ctx->max_batch) return fail(ctx, MBH_EINVAL, "mbh: walker index %d out of range", w);
    const int nm = ctx->md.nm, ns = ctx->g.ns;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "sync");
    if (band_host || fband_host) {
        std::vector<ModeBand> b(nm);
        if ((e = hipMemcpy(b.data(), ctx->wk.band + (size_t)w * nm, sizeof(ModeBand) * nm, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(ctx, e, "copy band");
        for (int i = 0; i < nm; ++i) {
            if (band_host) {
                band_host[4 * i] = b[i].active;
                band_host[4 * i + 1] = b[i].klo;
                band_host[4 * i + 2] = b[i].khi;
                band_host[4 * i + 3] = 0;
            }
            if (fband_host) {
                fband_host[2 * i] = b[i].fs;
                fband_host[2 * i + 1] = b[i].fe;
            }
        }
    }
    if (f_host && (e = hipMemcpy(f_host, ctx->wk.kf + (size_t)w * nm * ns, sizeof(double) * nm * ns, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(ctx, e, "copy knots");
    if (fn_host && (e = hipMemcpy(fn_host, ctx->wk.fn + (size_t)w * nm * kNumFn * ns, sizeof(double) * nm * kNumFn * ns,
                                  hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(ctx, e, "copy values");
    if (coef_host) {
        // device layout [nm][ns-1][8][4], each cubic centred on the first dense
        // bin of the next interval (fc = kbin[i+1] df); host layout
        // [nm][8][ns-1][4] in powers of f - f_i: a Taylor shift by f_i - fc
        std::vector<double> tmp((size_t)nm * (ns - 1) * kCoefPerIv), kf((size_t)nm * ns);
        std::vector<int> kb((size_t)nm * ns);
        if ((e = hipMemcpy(tmp.data(), ctx->wk.coef + (size_t)w * nm * (ns - 1) * kCoefPerIv, sizeof(double) * tmp.size(),
                           hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(kf.data(), ctx->wk.kf + (size_t)w * nm * ns, sizeof(double) * kf.size(),
                           hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(kb.data(), ctx->wk.kbin + (size_t)w * nm * ns, sizeof(int) * kb.size(),
                           hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(ctx, e, "copy coefficients");
        for (int im = 0; im < nm; ++im)
            for (int i = 0; i < ns - 1; ++i) {
                const double sh = kf[(size_t)im * ns + i] - (double)kb[(size_t)im * ns + i + 1] * ctx->g.df;
                for (int q = 0; q < kNumFn; ++q) {
                    const double *c = &tmp[(((size_t)im * (ns - 1) + i) * kNumFn + q) * 4];
                    double *o = &coef_host[(((size_t)im * kNumFn + q) * (ns - 1) + i) * 4];
                    o[0] = c[0] + sh * (c[1] + sh * (c[2] + sh * c[3]));
                    o[1] = c[1] + sh * (2.0 * c[2] + 3.0 * sh * c[3]);
                    o[2] = c[2] + 3.0 * sh * c[3];
                    o[3] = c[3];
                }
            }
    }
    return MBH_OK;
}

mbh_status mbh_set_sparse(mbh_ctx *ctx, int B, const int64_t *band_host, const double *fband_host,
                          const double *f_host, const double *fn_host, void *stream)
{
    if (!ctx) return MBH_EINVAL;
    mbh_status st = check_B(ctx, B);
    if (st) return st;
    if (B > 0 && (!band_host || !fband_host || !f_host || !fn_host)) return fail(ctx, MBH_EINVAL, "mbh: null input");
    const int nm = ctx->md.nm, ns = ctx->g.ns;
    hipStream_t s = (hipStream_t)stream;
    std::vector<ModeBand> b((size_t)B * nm);
    std::vector<Source> src(B);
    for (int w = 0; w < B; ++w) {
        std::memset(&src[w], 0, sizeof(Source));
        src[w].valid = 1;
        for (int i = 0; i < nm; ++i) {
            ModeBand &mb = b[(size_t)w * nm + i];
            std::memset(&mb, 0, sizeof(ModeBand));
            const int64_t *bh = band_host + ((size_t)w * nm + i) * 4;
            if (bh[0] && (bh[1] < ctx->g.k0 || bh[2] >= (int64_t)ctx->g.k0 + ctx->g.n || bh[2] < bh[1] + 3))
                return fail(ctx, MBH_EINVAL, "mbh: band of walker %d mode %d outside the grid", w, i);
            const double *fk = f_host + ((size_t)w * nm + i) * ns;
            if (bh[0]) {
                for (int j = 0; j + 1 < ns; ++j)
                    if (!(fk[j + 1] > fk[j])) return fail(ctx, MBH_EINVAL, "mbh: knots not increasing");
                if (fk[0] > (double)bh[1] * ctx->g.df || fk[ns - 1] < (double)bh[2] * ctx->g.df)
                    return fail(ctx, MBH_EINVAL, "mbh: knots do not cover the band");
            }
            mb.active = (int)bh[0];
            mb.klo = (int)bh[1];
            mb.khi = (int)bh[2];
            mb.fs = fband_host[((size_t)w * nm + i) * 2];
            mb.fe = fband_host[((size_t)w * nm + i) * 2 + 1];
        }
    }
    set_stage(ctx, 0, 0);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(ctx->wk.src, src.data(), sizeof(Source) * B, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->wk.band, b.data(), sizeof(ModeBand) * b.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->wk.kf, f_host, sizeof(double) * B * nm * ns, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ctx->wk.fn, fn_host, sizeof(double) * B * nm * kNumFn * ns, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_spline(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = launch_coef32(B, ctx->md, ctx->g, ctx->wk, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "set_sparse");
    if (B > 0) set_stage(ctx, 2, B);
    return MBH_OK;
}

}  // extern "C"
