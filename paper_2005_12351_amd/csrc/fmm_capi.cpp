// C ABI of libfmm.so: argument checking, device memory, and the order in
// which the kernels of the Cartesian FMM / Barnes-Hut method are queued
// (Pepper & Fangohr, arXiv 2005.12351, Section 3.2).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "fmm_internal.h"

static thread_local char g_err[1024];

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

extern "C" const char *fmm_last_error(void) { return g_err; }

#define FAIL(code, ...)          \
    do {                         \
        set_error(__VA_ARGS__);  \
        return code;             \
    } while (0)

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            FAIL(FMM_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

hipError_t launch_prep_positions(fmm_tree *t, const double *pos, hipStream_t s);

// ------------------------------------------------------------------ profiling
// events come from a per-context pool so that bracketing every launch costs
// two hipEventRecord calls and no allocation
static hipEvent_t pool_event(fmm_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(fmm_ctx *c, hipStream_t st, const char *nm) : ctx(c), s(st), name(nm)
{
    if (!ctx->profile) return;
    b = pool_event(ctx);
    if (b) hipEventRecord(b, s);
}

ProfScope::~ProfScope()
{
    if (!ctx->profile || !b) return;
    hipEvent_t e = pool_event(ctx);
    if (!e) return;
    hipEventRecord(e, s);
    ctx->prof.push_back(ProfEntry{name, b, e, 0.0});
}

static void drop_graphs(fmm_tree *t)
{
    for (auto &g : t->graphs) (void)hipGraphExecDestroy(g.exec);
    t->graphs.clear();
}

extern "C" int fmm_ctx_set_overlap(fmm_ctx *ctx, int on)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    if (on < 0 || on > FMM_OVERLAP_TAIL) FAIL(FMM_EINVAL, "overlap mode %d (0, 1, 2 or 3)", on);
    // the auxiliary stream exists only once some overlap asks for it: every
    // stream takes one of the process's few hardware queues, which contexts
    // without overlap (the serving slots) would otherwise share
    if (on != FMM_OVERLAP_OFF && !ctx->aux && !ctx->fake) {
        HIPCHK(hipSetDevice(ctx->device));
        if (hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) != hipSuccess) {
            ctx->aux = nullptr;
            FAIL(FMM_EDEVICE, "stream creation failed");
        }
    }
    ctx->overlap = on;
    for (fmm_tree *t : ctx->trees) drop_graphs(t);
    return FMM_OK;
}

extern "C" int fmm_ctx_set_m2l_basis(fmm_ctx *ctx, int basis)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    if (basis != FMM_M2L_FULL && basis != FMM_M2L_HARMONIC) FAIL(FMM_EINVAL, "unknown M2L basis %d", basis);
    ctx->m2l_basis = basis;   // trees pick it up at their next upward pass
    return FMM_OK;
}

extern "C" int fmm_ctx_set_m2l_schedule(fmm_ctx *ctx, int where)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    if (where != FMM_SCHEDULE_DEVICE && where != FMM_SCHEDULE_HOST && where != FMM_SCHEDULE_AUTO)
        FAIL(FMM_EINVAL, "unknown M2L schedule %d", where);
    ctx->m2l_schedule = where;   // trees built from now on
    return FMM_OK;
}

extern "C" int fmm_ctx_set_m2l_engine(fmm_ctx *ctx, int engine)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    if (engine != FMM_M2L_ENGINE_VALU && engine != FMM_M2L_ENGINE_MFMA && engine != FMM_M2L_ENGINE_AUTO)
        FAIL(FMM_EINVAL, "unknown M2L engine %d", engine);
    ctx->m2l_engine = engine;   // trees pick it up at their next upward pass
    return FMM_OK;
}

extern "C" int fmm_ctx_set_graphs(fmm_ctx *ctx, int on)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    ctx->graphs = on != 0;
    return FMM_OK;
}

// Runs `body` (which queues kernels on stream s) either directly or through a
// cached HIP graph of the same launch sequence.  Graphs are not used while
// profiling, because the per-kernel events must bracket real launches.
template <typename F>
static int run_cached(fmm_ctx *ctx, fmm_tree *t, const int64_t *key, hipStream_t s, F &&body)
{
    if (!ctx->graphs || ctx->profile) return body();
    for (auto &g : t->graphs)
        if (memcmp(g.key, key, sizeof(g.key)) == 0) {
            HIPCHK(hipGraphLaunch(g.exec, s));
            return FMM_OK;
        }
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = body();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc != FMM_OK) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) FAIL(FMM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    fmm_tree::GraphEntry ge;
    memcpy(ge.key, key, sizeof(ge.key));
    e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) FAIL(FMM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    t->graphs.push_back(ge);
    HIPCHK(hipGraphLaunch(ge.exec, s));
    return FMM_OK;
}

extern "C" int fmm_profile_enable(fmm_ctx *ctx, int on)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    ctx->profile = on != 0;
    return FMM_OK;
}

extern "C" int fmm_profile_reset(fmm_ctx *ctx)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    if (ctx->fake) FAIL(FMM_EINVAL, "context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    for (auto &e : ctx->prof) {
        if (!e.a) continue;   // a host phase holds no events
        ctx->ev_pool.push_back(e.a);
        ctx->ev_pool.push_back(e.b);
    }
    ctx->prof.clear();
    return FMM_OK;
}

extern "C" int fmm_profile_read(fmm_ctx *ctx, const char **names, double *ms, int64_t *launches, int cap)
{
    if (!ctx || cap < 0) FAIL(FMM_EINVAL, "bad arguments");
    if (ctx->fake) FAIL(FMM_EINVAL, "context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    std::vector<const char *> nm;
    std::vector<double> tot;
    std::vector<int64_t> cnt;
    for (auto &e : ctx->prof) {
        float t = (float)e.host_ms;
        if (e.a) HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
        size_t k = 0;
        while (k < nm.size() && strcmp(nm[k], e.name) != 0) ++k;
        if (k == nm.size()) {
            nm.push_back(e.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[k] += t;
        cnt[k] += 1;
    }
    const int nk = (int)std::min<size_t>(nm.size(), (size_t)cap);
    for (int k = 0; k < nk; ++k) {
        if (names) names[k] = nm[k];
        if (ms) ms[k] = tot[k];
        if (launches) launches[k] = cnt[k];
    }
    return (int)nm.size();
}

// ------------------------------------------------------------------ context
extern "C" int fmm_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, fmm_ctx **out)
{
    if (!out) FAIL(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) FAIL(FMM_EINVAL, "device %d out of range (have %d)", device, ndev);
    HIPCHK(hipSetDevice(device));
    fmm_ctx *c = new fmm_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            FAIL(FMM_EDEVICE, "stream creation failed");
        }
        c->own_stream = true;
    }
    if (hipEventCreateWithFlags(&c->ev_up, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_near, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_m2l, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_near2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_upload, hipEventDisableTiming) != hipSuccess) {
        delete c;
        FAIL(FMM_EDEVICE, "stream/event creation failed");
    }
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) c->ncu = 256;
    // Memory freed to the device's stream-ordered pool stays mapped for the
    // next allocation instead of going back to the driver at each stream
    // wait: growing a build arena or a tree block cache then costs no new
    // mapping (a first build on a fresh context took about 10 ms before).
    {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
    }
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)fr);
    // the device address of the allocation-free call's static scratch on
    // this device (resolved once per device, with the device current)
    if (const hipError_t e = noalloc_scratch(device, &c->noalloc_scratch); e != hipSuccess) {
        fmm_ctx_destroy(c);
        FAIL(FMM_EDEVICE, "scratch address: %s", hipGetErrorString(e));
    }
    *out = c;
    return FMM_OK;
}

// Size classes of tree blocks: 256 B, then four per power of two (at most
// 25 % above the request), so that released blocks fit later requests.
static size_t size_class(size_t b)
{
    if (b <= 256) return 256;
    const int e = 63 - __builtin_clzll((unsigned long long)(b - 1));   // 2^e < b <= 2^(e+1)
    const size_t step = (size_t)1 << (e - 2);
    return (b + step - 1) / step * step;
}

size_t ctx_cache_limit(const fmm_ctx *ctx) { return std::min(ctx->budget / 8, (size_t)4 << 30); }

// A released block goes to the context's cache (or back to the allocator
// when the cache is full).  Work on the context stream queued after this
// point, and on the auxiliary stream forked from it, is ordered after every
// earlier use of the block, so handing it to a later tree_alloc is safe.
static void ctx_dev_free(fmm_ctx *c, void *p, size_t bytes)
{
    const size_t cls = size_class(bytes);
    if (c->dev_cache_bytes + cls <= ctx_cache_limit(c)) {
        c->dev_cache.emplace(cls, p);
        c->dev_cache_bytes += cls;
    } else {
        (void)hipFreeAsync(p, c->stream);
    }
}

static void ctx_cache_drop(fmm_ctx *c)
{
    for (auto &kv : c->dev_cache) (void)hipFreeAsync(kv.second, c->stream);
    c->dev_cache.clear();
    c->dev_cache_bytes = 0;
}

static void tree_release_device(fmm_tree *t)
{
    drop_graphs(t);
    // the near field may still run on the auxiliary stream
    if (t->ctx->aux) (void)hipStreamSynchronize(t->ctx->aux);
    for (auto &a : t->allocs) ctx_dev_free(t->ctx, a.first, a.second);
    t->allocs.clear();
    t->dev_bytes = 0;
}

extern "C" int fmm_ctx_destroy(fmm_ctx *c)
{
    if (!c) return FMM_OK;
    serve_destroy(c);
    if (c->fake) {
        delete c;
        return FMM_OK;
    }
    (void)hipSetDevice(c->device);
    hipDeviceSynchronize();
    // trees still alive lose their device memory and become orphans that
    // only fmm_tree_destroy accepts
    for (fmm_tree *t : c->trees) {
        tree_release_device(t);
        t->ctx = nullptr;
    }
    c->trees.clear();
    ctx_cache_drop(c);
    if (c->arena) (void)hipFreeAsync(c->arena, c->stream);
    c->arena = nullptr;
    c->arena_cap = 0;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->prof) {
        if (!e.a) continue;   // a host phase holds no events
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->pin_small) (void)hipHostFree(c->pin_small);
    if (c->sig) (void)hipHostFree(c->sig);
    hipEventDestroy(c->ev_up);
    hipEventDestroy(c->ev_near);
    hipEventDestroy(c->ev_fork);
    hipEventDestroy(c->ev_m2l);
    hipEventDestroy(c->ev_near2);
    hipEventDestroy(c->ev_upload);
    if (c->aux) hipStreamDestroy(c->aux);
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return FMM_OK;
}

// ------------------------------------------------------------------ tree
// Device memory comes from the context's cache of released blocks of the
// same size class, else from the stream-ordered allocator on the context's
// stream: neither synchronises the device, so requests served on other
// streams keep running while a tree is built or freed.  A tree's size
// (dev_bytes, the tree limit) counts the requested bytes.
int tree_alloc(fmm_tree *t, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (t->ctx->tree_limit && t->dev_bytes + bytes > t->ctx->tree_limit)
        FAIL(FMM_ENOMEM, "device allocation of %zu bytes would exceed the tree limit of %zu bytes (%zu held)", bytes,
             t->ctx->tree_limit, t->dev_bytes);
    fmm_ctx *c = t->ctx;
    const size_t cls = size_class(bytes);
    auto hit = c->dev_cache.find(cls);
    if (hit != c->dev_cache.end()) {
        *p = hit->second;
        c->dev_cache.erase(hit);
        c->dev_cache_bytes -= cls;
    } else if (hipMallocAsync(p, cls, c->stream) != hipSuccess) {
        // the cached blocks back to the allocator, then once more
        (void)hipGetLastError();
        ctx_cache_drop(c);
        if (hipMallocAsync(p, cls, c->stream) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            FAIL(FMM_ENOMEM, "device allocation of %zu bytes failed", bytes);
        }
    }
    t->allocs.emplace_back(*p, bytes);
    t->dev_bytes += bytes;
    return FMM_OK;
}

static void tree_free_block(fmm_tree *t, void *p)
{
    if (!p) return;
    auto it = std::find_if(t->allocs.begin(), t->allocs.end(), [p](const auto &a) { return a.first == p; });
    if (it != t->allocs.end()) {
        t->dev_bytes -= it->second;
        ctx_dev_free(t->ctx, p, it->second);
        t->allocs.erase(it);
    } else {
        (void)hipFreeAsync(p, t->ctx->stream);
    }
}

extern "C" int fmm_ctx_set_tree_limit(fmm_ctx *ctx, size_t bytes)
{
    if (!ctx) FAIL(FMM_EINVAL, "null context");
    ctx->tree_limit = bytes;
    return FMM_OK;
}

hipError_t ctx_pinned(fmm_ctx *ctx, size_t bytes, char **base)
{
    // the copies of the last flush of uploads read the buffer until they end
    if (ctx->upload_pending) {
        const hipError_t e = hipEventSynchronize(ctx->ev_upload);
        ctx->upload_pending = false;
        if (e != hipSuccess) return e;
    }
    if (ctx->pinned_bytes < bytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        const size_t want = std::max(bytes + bytes / 4, (size_t)1 << 20);
        hipError_t e = hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        ctx->pinned_bytes = want;
    }
    *base = (char *)ctx->pinned;
    return hipSuccess;
}

// Uploads of host vectors into new tree allocations: add() allocates and
// records the vector's data pointer, flush() packs the data into the
// context's pinned buffer, queues the copies and records ev_upload after
// them (the next use of the pinned buffer waits for that event).  Every
// vector passed to add() must live, unchanged, until flush() returns.
struct Uploads {
    fmm_tree *t;
    struct Item {
        void *dst;
        const void *src;
        size_t bytes;
    };
    std::vector<Item> items;
    size_t total = 0;
    template <typename T>
    int add(T **dst, const std::vector<T> &src)
    {
        int rc = tree_alloc(t, (void **)dst, src.size() * sizeof(T));
        if (rc) return rc;
        if (!src.empty()) {
            items.push_back(Item{*dst, src.data(), src.size() * sizeof(T)});
            total += (src.size() * sizeof(T) + 255) / 256 * 256;
        }
        return FMM_OK;
    }
    int flush(hipStream_t s)
    {
        if (items.empty()) return FMM_OK;
        char *base;
        HIPCHK(ctx_pinned(t->ctx, total, &base));
        size_t o = 0;
        for (const Item &it : items) {
            memcpy(base + o, it.src, it.bytes);
            HIPCHK(hipMemcpyAsync(it.dst, base + o, it.bytes, hipMemcpyHostToDevice, s));
            o += (it.bytes + 255) / 256 * 256;
        }
        HIPCHK(hipEventRecord(t->ctx->ev_upload, s));
        t->ctx->upload_pending = true;
        items.clear();
        total = 0;
        return FMM_OK;
    }
};

extern "C" int fmm_tree_destroy(fmm_tree *t)
{
    if (!t) return FMM_OK;
    if (fmm_ctx *c = t->ctx) {
        (void)hipSetDevice(c->device);
        tree_release_device(t);
        c->trees.erase(std::remove(c->trees.begin(), c->trees.end(), t), c->trees.end());
    }
    delete t;
    return FMM_OK;
}


extern "C" int fmm_build_tree(fmm_ctx *ctx, const double *pos, int64_t n, int ncrit, double theta, int method,
                              fmm_tree **out)
{
    if (!ctx || !out) FAIL(FMM_EINVAL, "null context or output");
    if (ctx->fake) FAIL(FMM_EINVAL, "context has no device");
    *out = nullptr;
    if (!pos) FAIL(FMM_EINVAL, "positions are NULL");
    if (n < 1 || n > (int64_t)INT32_MAX / 4) FAIL(FMM_EINVAL, "n = %lld out of range", (long long)n);
    if (ncrit < 1) FAIL(FMM_EINVAL, "ncrit = %d must be >= 1", ncrit);
    if (!(theta > 0.0 && theta < 1.0)) FAIL(FMM_EINVAL, "theta = %g must lie in (0, 1)", theta);
    if (method != FMM_METHOD_FMM && method != FMM_METHOD_BH) FAIL(FMM_EINVAL, "unknown method %d", method);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    fmm_tree *t = new fmm_tree();
    t->ctx = ctx;
    t->method = method;
    t->ncrit = ncrit;
    t->theta = theta;
    HostScope hs_all(ctx, "host:build_tree");
    DevKeep dt;
    dt.keep = [t](void **p, size_t bytes) { return tree_alloc(t, p, bytes) == FMM_OK ? hipSuccess : hipErrorOutOfMemory; };
    dt.tl = &t->tiling;
    // automatic: the device, measured faster than the host threads for
    // every tree from 3·10^3 list entries on (builds of 10^3 to 10^4
    // particles: 0.60-1.21 ms against 0.63-2.71 ms)
    dt.tiling = method == FMM_METHOD_FMM && ctx->m2l_schedule != FMM_SCHEDULE_HOST;
    dt.min_pairs = 0;
    {
        HostScope hs_gpu(ctx, "host:tree_device_build");   // the marked phases plus the release of the build's scratch
        const hipError_t e = gpu_build_tree(pos, n, ncrit, theta, method == FMM_METHOD_FMM, s, t->ht, ctx, &dt);
        if (e != hipSuccess) {
            fmm_tree_destroy(t);
            if (e == hipErrorInvalidValue) FAIL(FMM_EINVAL, "non-finite position");
            if (e == hipErrorOutOfMemory) FAIL(FMM_ENOMEM, "tree construction: out of device memory");
            FAIL(FMM_EDEVICE, "tree construction: %s", hipGetErrorString(e));
        }
    }
    HostTree &h = t->ht;
    const int64_t nc = h.ncells();
    t->d_cells = dt.cells;
    t->d_perm = dt.perm;
    t->d_key = dt.key;
    if (method == FMM_METHOD_FMM) {
        if (dt.done) {
            t->d_ucls = dt.ucls;
            t->d_usrc = dt.usrc;
            t->d_cell_slot = dt.cell_slot;
            t->d_cls_geom = dt.cls_geom;
            t->d_m2l_ptr = dt.m2l_ptr;
            t->d_m2l_src = dt.m2l_src;
        } else {
            HostScope hs(ctx, "host:m2l_tiling");
            build_m2l_tiling(h, t->tiling);
        }
    } else {
        h.m2l_ptr.assign(nc + 1, 0);
        h.p2p_ptr.assign(nc + 1, 0);
    }
    // leaves, per-particle leaf, non-leaf cells per level, P2P CSR per leaf
    HostScope hs_sched(ctx, "host:tree_near_schedule");
    std::vector<int32_t> level_cells(nc);
    for (int64_t c = 0; c < nc; ++c) {
        level_cells[c] = (int32_t)c;
        if (h.nchild[c] == 0) {
            t->leaves.push_back((int32_t)c);
        }
    }
    t->nleaves = (int64_t)t->leaves.size();
    const int nlev = (int)h.level_ptr.size() - 1;
    t->level_nonleaf_ptr.assign(nlev + 1, 0);
    for (int l = 0; l < nlev; ++l) {
        for (int64_t c = h.level_ptr[l]; c < h.level_ptr[l + 1]; ++c)
            if (h.nchild[c]) t->level_nonleaf.push_back((int32_t)c);
        t->level_nonleaf_ptr[l + 1] = (int32_t)t->level_nonleaf.size();
    }
    // M2M is needed only into parents at or below the shallowest M2L source
    // level, L2L only below the shallowest M2L target level: above them the
    // multipoles are never read and the locals are zero.  Barnes-Hut may
    // accept a cell at any level.
    // (a list is sorted by source index and cells are level-major, so its
    // first source is its shallowest)
    int src_top = nlev, tgt_top = nlev;
    if (t->tiling.on_device && dt.tgt_top >= 0) {
        tgt_top = dt.tgt_top;
        src_top = dt.src_top;
    } else if ((int64_t)h.m2l_ptr.size() == nc + 1)
        for (int64_t c = 0; c < nc; ++c)
            if (h.m2l_ptr[c + 1] > h.m2l_ptr[c]) {
                tgt_top = std::min(tgt_top, h.level[c]);
                src_top = std::min(src_top, h.level[h.m2l_src[h.m2l_ptr[c]]]);
            }
    t->m2m_top = method == FMM_METHOD_BH ? 0 : src_top;
    t->l2l_from = tgt_top + 1;
    // P2P CSR per leaf, each leaf's pairs and its cost (a workgroup's time
    // grows with its pairs); the sums are of integers below 2^53, exact in
    // any order, so the leaves are done in parallel
    const int64_t nlv_ = t->nleaves;
    std::vector<int32_t> pptr(nlv_ + 1, 0);
    for (int64_t k = 0; k < nlv_; ++k) {
        const int64_t b = t->leaves[k];
        pptr[k + 1] = pptr[k] + (int32_t)(h.p2p_ptr[b + 1] - h.p2p_ptr[b]);
    }
    // With the sources kept on the device (dt.p2p_src, a build with lists)
    // the costs come from the device and the per-leaf CSR is the device's
    // list as it is; otherwise (no lists: every leaf's list is empty) it is
    // built here.
    const bool dev_src = dt.p2p_src != nullptr;
    std::vector<int32_t> psrc(dev_src ? 0 : pptr[nlv_]);
    std::vector<double> leaf_cost(nlv_, 0.0), leaf_pairs(nlv_, 0.0);
    // (the host threads pay from about a thousand leaves on)
    constexpr int64_t kSerialLeaves = 1024;
    host_parallel_for(nlv_, [&](int64_t k) {
        const int64_t b = t->leaves[k];
        if (dev_src) {
            leaf_cost[k] = (double)h.p2p_cost[b];
        } else {
            int32_t *o = psrc.data() + pptr[k];
            double srcs = 0.0;
            for (int64_t e = h.p2p_ptr[b]; e < h.p2p_ptr[b + 1]; ++e) {
                const int64_t A = h.p2p_src[e];
                *o++ = (int32_t)A;
                srcs += (double)h.count[A];
            }
            leaf_cost[k] = srcs * (double)h.count[b];
        }
        // the pairs, without the self pair of each particle
        leaf_pairs[k] = leaf_cost[k] - (h.p2p_ptr[b + 1] > h.p2p_ptr[b] ? (double)h.count[b] : 0.0);
    }, dev_src ? INT64_MAX : kSerialLeaves);
    double p2p_pairs = 0.0;
    for (double v : leaf_pairs) p2p_pairs += v;
    t->work[2] = p2p_pairs;
    // Near-field dispatch order.  Workgroups go to the eight XCDs in turn
    // (workgroup g to XCD g % 8) and each XCD has its own L2, so the leaves,
    // in Morton order (the order of their first particle), are cut into
    // eight ranges of equal cost and workgroup g takes the (g / 8)-th leaf of
    // range g % 8: the leaves one XCD works on are neighbours and share most
    // of their source leaves in its L2.  Within a range the heaviest leaves
    // go first (to within a bucket of cost), so that the light ones fill the
    // end of the launch.
    constexpr int kXcd = 8;
    std::vector<int32_t> p2p_order;
    {
        // the leaves in the order of their first particle: a depth-first
        // walk with the children in octant order (each child's particles
        // follow its elder sibling's)
        std::vector<int32_t> leaf_index(nc, -1), mort;
        mort.reserve(t->nleaves);
        for (int64_t k = 0; k < t->nleaves; ++k) leaf_index[t->leaves[k]] = (int32_t)k;
        {
            std::vector<int32_t> stack{0};
            while (!stack.empty()) {
                const int32_t c = stack.back();
                stack.pop_back();
                if (h.nchild[c] == 0) {
                    mort.push_back(leaf_index[c]);
                    continue;
                }
                for (int k = h.nchild[c] - 1; k >= 0; --k) stack.push_back((int32_t)(h.child0[c] + k));
            }
        }
        double tot = 0.0;
        for (double c : leaf_cost) tot += c;
        std::vector<std::vector<int32_t>> range(kXcd);
        double acc = 0.0;
        for (int32_t k : mort) {
            const int r = std::min(kXcd - 1, tot > 0.0 ? (int)(acc * kXcd / tot) : 0);
            range[r].push_back(k);
            acc += leaf_cost[k];
        }
        // heaviest first within a range: a stable counting sort on the cost's
        // octave and its next three bits (eight buckets an octave, about 9 %
        // wide), so leaves of nearly equal cost keep their Morton order; one
        // pass, no comparison sort and no host threads to wake
        // (the bucket is read off the double: its biased exponent and the top
        // three bits of its mantissa, counted from 1.0 up)
        constexpr int kBuckets = 512;
        std::vector<int16_t> slot(nlv_);
        for (int64_t k = 0; k < nlv_; ++k) {
            const double c = leaf_cost[k];
            uint64_t bits;
            memcpy(&bits, &c, sizeof bits);
            const int64_t b = c >= 1.0 ? (int64_t)(bits >> 49) - (int64_t)(1023 << 3) + 1 : 0;
            slot[k] = (int16_t)(kBuckets - 1 - std::min<int64_t>(kBuckets - 1, b));   // heaviest first
        }
        std::vector<int32_t> cnt(kBuckets), tmp;
        for (auto &rg : range) {
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int32_t k : rg) ++cnt[slot[k]];
            int32_t acc = 0;
            for (int b = 0; b < kBuckets; ++b) {
                const int32_t c = cnt[b];
                cnt[b] = acc;
                acc += c;
            }
            tmp.resize(rg.size());
            for (int32_t k : rg) tmp[cnt[slot[k]]++] = k;
            rg.swap(tmp);
        }
        size_t longest = 0;
        for (auto &rg : range) longest = std::max(longest, rg.size());
        for (size_t i = 0; i < longest; ++i)
            for (auto &rg : range)
                if (i < rg.size()) p2p_order.push_back(rg[i]);
    }
    {
        // split point of the near field for FMM_OVERLAP_SPLIT: half the cost
        double tot = 0.0, acc = 0.0;
        for (double c : leaf_cost) tot += c;
        int k = 0;
        while (k < (int)t->nleaves && acc < 0.5 * tot) acc += leaf_cost[p2p_order[k++]];
        t->p2p_split = k;
    }

    hs_sched.end();
    HostScope hs_up(ctx, "host:tree_upload");
    int rc = FMM_OK;
    Uploads up{t};
#define UP(dst, vec)                                   \
    if ((rc = up.add(&(dst), vec)) != FMM_OK) {        \
        fmm_tree_destroy(t);                           \
        return rc;                                     \
    }
    UP(t->d_leaves, t->leaves);
    UP(t->d_nonleaf, t->level_nonleaf);
    UP(t->d_level_cells, level_cells);
    UP(t->d_p2p_ptr, pptr);
    if (dev_src) t->d_p2p_src = dt.p2p_src;
    else UP(t->d_p2p_src, psrc);
    UP(t->d_p2p_order, p2p_order);
    std::vector<int32_t> cell_slot;   // lives until the flush below
    if (method == FMM_METHOD_FMM && !t->tiling.on_device) {
        const M2LTiling &tl = t->tiling;
        UP(t->d_ucls, tl.ucls);
        UP(t->d_usrc, tl.usrc);
        cell_slot.assign(nc, -1);
        for (size_t k = 0; k < tl.tile_cell.size(); ++k)
            if (tl.tile_cell[k] >= 0) cell_slot[tl.tile_cell[k]] = (int32_t)k;
        UP(t->d_cell_slot, cell_slot);
        UP(t->d_cls_geom, tl.cls_geom);
    }
    if (method == FMM_METHOD_FMM) t->work[0] = (double)t->tiling.pairs;
#undef UP
    if ((rc = up.flush(s)) || (rc = tree_alloc(t, (void **)&t->d_x, sizeof(double) * 3 * n))) {
        fmm_tree_destroy(t);
        return rc;
    }
    hipError_t e = launch_prep_positions(t, pos, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fmm_tree_destroy(t);
        FAIL(FMM_EDEVICE, "tree upload failed: %s", hipGetErrorString(e));
    }
    ctx->trees.push_back(t);
    *out = t;
    return FMM_OK;
}

// ------------------------------------------------------------------ upward
static int ensure_expansions(fmm_tree *t, int code, int p, int prec)
{
    HostScope hs(t->ctx, "host:expansions");
    const int smask = code_mask(code), order = mask_min_order(smask);
    const bool fmm = t->method == FMM_METHOD_FMM;
    const int basis = t->ctx->m2l_basis;
    const bool harm = basis == FMM_M2L_HARMONIC;
    // matrix cores: measured faster from p = 8 on (the contraction per list
    // entry grows as p^3, the operand traffic as p^2)
    const int eng = t->ctx->m2l_engine;
    const bool mfma = fmm && harm && prec == FMM_PREC_MIXED &&
                      (eng == FMM_M2L_ENGINE_MFMA || (eng == FMM_M2L_ENGINE_AUTO && p >= 8));
    if (t->d_mom && t->order == order && t->smask == smask && t->p == p && t->prec == prec && t->basis == basis &&
        t->mfma == mfma)
        return FMM_OK;
    drop_graphs(t);
    // the tree holds no valid expansion set from here until every buffer
    // below exists: a failure on the way leaves it marked so, and the next
    // call sets it up again whatever its parameters
    t->p = -1;
    // the host-built tables go up in one flush at the end (their vectors
    // live until then)
    Uploads up{t};
    std::vector<int4> work;
    std::vector<int32_t> pack;
    for (void **pp : {(void **)&t->d_mom, (void **)&t->d_mom32, (void **)&t->d_M64, (void **)&t->d_M32, &t->d_Mh,
                      (void **)&t->d_Mf64, (void **)&t->d_part, (void **)&t->d_L64, (void **)&t->d_near, (void **)&t->d_near_g,
                      (void **)&t->d_D64,
                      (void **)&t->d_D32, (void **)&t->d_sc64, (void **)&t->d_sc32, (void **)&t->d_work,
                      (void **)&t->d_tile_chunk0, (void **)&t->d_tile_nchunk, (void **)&t->d_wave_ptr}) {
        tree_free_block(t, *pp);
        *pp = nullptr;
    }
    t->dtab_p = -1;
    const int64_t n = t->ht.n, nc = t->ht.ncells();
    const int nm = nterms(p) - nterms(order - 1), nmp = (nm + 3) / 4 * 4, nl = nterms(p - order);
    int rc;
    if ((rc = tree_alloc(t, (void **)&t->d_mom, sizeof(double) * mask_width(smask) * n)) ||
        (rc = tree_alloc(t, (void **)&t->d_mom32, sizeof(float) * m32_width(smask) * n)) ||
        (rc = tree_alloc(t, (void **)&t->d_near, sizeof(double) * 4 * n)))
        return rc;
    // full rows are the upward state of the full basis only; the harmonic
    // basis keeps folded rows (below)
    if (!harm && (rc = tree_alloc(t, (void **)&t->d_M64, sizeof(double) * (nc + 1) * nmp))) return rc;
    // the FP64 folded rows of the harmonic basis in MIXED (in FP64 the M2L's
    // own rows are the state), row stride nhp
    auto alloc_state = [&](int nhp) -> int {
        if (!harm || prec != FMM_PREC_MIXED) return FMM_OK;
        int r = tree_alloc(t, (void **)&t->d_Mf64, sizeof(double) * (size_t)(nc + 1) * nhp);
        if (r) return r;
        hipError_t e = launch_fill(t->d_Mf64, (size_t)(nc + 1) * nhp, t->ctx->stream);
        if (e != hipSuccess) FAIL(FMM_EDEVICE, "fill failed: %s", hipGetErrorString(e));
        return FMM_OK;
    };
    // the full FP32 copy feeds the full-basis M2L and the Barnes-Hut M2P
    if (prec == FMM_PREC_MIXED && !harm && (rc = tree_alloc(t, (void **)&t->d_M32, sizeof(float) * (nc + 1) * nmp)))
        return rc;
    if (t->method == FMM_METHOD_BH && !t->d_bhcount &&
        (rc = tree_alloc(t, (void **)&t->d_bhcount, 2 * sizeof(unsigned long long))))
        return rc;
    if (!fmm && harm) {
        // folded rows the Barnes-Hut M2P reads (FMM trees size them from the M2L variant below)
        const size_t es = prec == FMM_PREC_MIXED ? sizeof(float) : sizeof(double);
        const int nhp = (hterms(p) - hterms(order - 1) + 3) / 4 * 4;
        t->nhp = nhp;
        if ((rc = tree_alloc(t, &t->d_Mh, es * (size_t)(nc + 1) * nhp))) return rc;
        hipError_t e = launch_fill((double *)t->d_Mh, es * (size_t)(nc + 1) * nhp / 8, t->ctx->stream);
        if (e != hipSuccess) FAIL(FMM_EDEVICE, "fill failed: %s", hipGetErrorString(e));
        if ((rc = alloc_state(nhp))) return rc;
    }
    if (fmm) {
        M2LVariant v;
        if (!m2l_lookup(p, order, prec == FMM_PREC_MIXED, harm, &v, mfma))
            FAIL(FMM_EINVAL, "no M2L kernel for p=%d s=%d", p, order);
        const size_t es = prec == FMM_PREC_MIXED ? sizeof(float) : sizeof(double);
        const int nc_ = std::max(1, t->tiling.nclasses);
        const int scw = (p + 1 + 3) / 4 * 4;
        // one wave per resident slot of the device
        const int ncu = t->ctx->ncu;
        // one M2L workgroup per resident workgroup slot; each writes its own
        // partial rows where its piece of the work ends
        build_m2l_work(t->tiling, v, ncu * v.occupancy(), t->m2lwork);
        work.resize(t->m2lwork.work.size() / 4);
        for (size_t k = 0; k < work.size(); ++k)
            work[k] = make_int4(t->m2lwork.work[4 * k], t->m2lwork.work[4 * k + 1], t->m2lwork.work[4 * k + 2],
                                t->m2lwork.work[4 * k + 3]);
        if ((rc = up.add(&t->d_work, work)) || (rc = up.add(&t->d_tile_chunk0, t->m2lwork.chunk0)) ||
            (rc = up.add(&t->d_tile_nchunk, t->m2lwork.nchunk)) || (rc = up.add(&t->d_wave_ptr, t->m2lwork.wave_ptr)))
            return rc;
        if ((rc = tree_alloc(t, &t->d_part, es * (size_t)std::max<int64_t>(1, t->m2lwork.nrows) * v.nl_pad)) ||
            (rc = tree_alloc(t, (void **)&t->d_L64, sizeof(double) * nc * (harm ? hterms(p - order) : nl))) ||
            (rc = tree_alloc(t, (void **)&t->d_D64, sizeof(double) * nc_ * v.nd)) ||
            (rc = tree_alloc(t, (void **)&t->d_D32, sizeof(float) * nc_ * v.nd)) ||
            (rc = tree_alloc(t, (void **)&t->d_sc64, sizeof(double) * nc_ * scw)) ||
            (rc = tree_alloc(t, (void **)&t->d_sc32, sizeof(float) * nc_ * scw)))
            return rc;
        // reduced multipole rows, plus the zero row that padded slots read
        // (the M2L variant fixes the row stride: the matrix-core kernels
        // align every row to a 128-byte cache line)
        t->nhp = v.nm_pad;
        if (harm && (rc = tree_alloc(t, &t->d_Mh, es * (size_t)(nc + 1) * v.nm_pad))) return rc;
        if (harm) {
            hipError_t e = launch_fill((double *)t->d_Mh, es * (size_t)(nc + 1) * v.nm_pad / 8, t->ctx->stream);
            if (e != hipSuccess) FAIL(FMM_EDEVICE, "fill failed: %s", hipGetErrorString(e));
            if ((rc = alloc_state(v.nm_pad))) return rc;
        }
    }
    if (t->method == FMM_METHOD_FMM && t->l2p_pack_q != p - order) {
        // L2P waves: consecutive leaves while they hold at most 64 particles
        // together and fit the layout's budget (a larger leaf gets a wave of
        // its own)
        auto packing = [&](int kmax) {
            std::vector<int32_t> pk(1, 0);
            int64_t cnt = 0;
            for (int64_t k = 0; k < t->nleaves; ++k) {
                const int64_t c = t->ht.count[t->leaves[k]];
                const int in_pack = (int)(k - pk.back());
                if (in_pack > 0 && (cnt + c > 64 || in_pack >= kmax)) {
                    pk.push_back((int32_t)k);
                    cnt = 0;
                }
                cnt += c;
            }
            pk.push_back((int32_t)t->nleaves);
            return pk;
        };
        const int q = p - order;
        pack = packing(l2p_pack_limit(q, false));
        const int ncu = t->ctx->ncu;
        std::vector<int32_t> pack_cols = packing(l2p_pack_limit(q, true));
        t->l2p_columns = pack_cols.size() < pack.size() || l2p_columns_pay(q, (int)pack.size() - 1, ncu);
        if (t->l2p_columns) pack.swap(pack_cols);
        if (t->d_l2p_pack) tree_free_block(t, t->d_l2p_pack);
        t->d_l2p_pack = nullptr;
        t->l2p_pack_q = -1;
        if ((rc = up.add(&t->d_l2p_pack, pack))) return rc;
        t->l2p_npacks = (int)pack.size() - 1;
        t->l2p_pack_q = p - order;
    }
    if ((rc = up.flush(t->ctx->stream))) return rc;
    hipError_t e = t->d_M64 ? launch_fill(t->d_M64, (size_t)(nc + 1) * nmp, t->ctx->stream) : hipSuccess;
    // P2M and M2M write the FP32 copy too; the rest (the zero row the padded
    // M2L slots read, unused levels) stays zero (nmp is a multiple of 4)
    if (e == hipSuccess && t->d_M32)
        e = launch_fill((double *)t->d_M32, (size_t)(nc + 1) * nmp / 2, t->ctx->stream);
    if (e != hipSuccess) FAIL(FMM_EDEVICE, "fill failed: %s", hipGetErrorString(e));
    t->order = order;
    t->smask = smask;
    t->p = p;
    t->prec = prec;
    t->basis = basis;
    t->mfma = mfma;
    if (fmm) {
        // derivative tensors of the translation classes depend on p only
        e = launch_dtable(t, t->ctx->stream);
        if (e != hipSuccess) {
            t->p = -1;
            FAIL(FMM_EDEVICE, "dtable failed: %s", hipGetErrorString(e));
        }
        t->dtab_p = p;
    }
    return FMM_OK;
}

#define KCHK(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) FAIL(FMM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

static int check_upward_args(fmm_ctx *ctx, fmm_tree *t, int order, const double *moments, int p, int precision)
{
    if (!ctx || !t || t->ctx != ctx) FAIL(FMM_EINVAL, "null or foreign context/tree");
    if (!((order >= 0 && order <= 3) || (order > FMM_MIXED && order < FMM_MIXED + 16)))
        FAIL(FMM_EINVAL, "source order code %d is neither 0, 1, 2, 3 nor FMM_MIXED | mask", order);
    if (!moments) FAIL(FMM_EINVAL, "moments are NULL");
    if (precision != FMM_PREC_FP64 && precision != FMM_PREC_MIXED) FAIL(FMM_EINVAL, "unknown precision %d", precision);
    const int s = mask_min_order(code_mask(order));
    const int pmin = t->method == FMM_METHOD_FMM ? s + 1 : std::max(s, 1);
    if (p < pmin || p > FMM_P_MAX) FAIL(FMM_EINVAL, "p = %d must lie in [%d, %d]", p, pmin, FMM_P_MAX);
    return FMM_OK;
}

static int check_eval_args(fmm_ctx *ctx, fmm_tree *t, int outputs, const double *phi, const double *field)
{
    if (!ctx || !t || t->ctx != ctx) FAIL(FMM_EINVAL, "null or foreign context/tree");
    if (outputs <= 0 || (outputs & ~(FMM_POT | FMM_FIELD))) FAIL(FMM_EINVAL, "bad output mask %d", outputs);
    if ((outputs & FMM_POT) && !phi) FAIL(FMM_EINVAL, "potential requested but phi is NULL");
    if ((outputs & FMM_FIELD) && !field) FAIL(FMM_EINVAL, "field requested but field is NULL");
    return FMM_OK;
}

// Queues the upward pass on the context stream: P2M (which also writes the
// sorted FP64 and FP32 moments), M2M by level (both also write the
// harmonic-basis or FP32 copy the M2L reads).  For FMM trees the near field
// (which needs only the sorted moments) is forked after P2M onto the
// auxiliary stream; with join it is joined back at the end, otherwise the
// caller joins it (ev_near).
static int queue_upward(fmm_ctx *ctx, fmm_tree *t, bool join)
{
    hipStream_t s = ctx->stream;
    const bool fmm = t->method == FMM_METHOD_FMM;
    // tail overlap: inside fmm_run the near field follows the M2L
    // (queue_evaluate); alone, fmm_upward runs it on its own stream
    const bool tail = ctx->overlap == FMM_OVERLAP_TAIL;
    hipStream_t a = ctx->overlap && !tail && fmm ? ctx->aux : s;
    {
        ProfScope ps(ctx, s, "p2m");
        KCHK(launch_p2m(t, s));
    }
    if (fmm && !(tail && !join)) {
        if (a != s) {
            KCHK(hipEventRecord(ctx->ev_fork, s));
            KCHK(hipStreamWaitEvent(a, ctx->ev_fork, 0));
        }
        {
            ProfScope ps(ctx, a, "p2p");
            // split overlap inside fmm_run: the first half here (beside M2M),
            // the second after the M2L (queue_evaluate)
            if (ctx->overlap == FMM_OVERLAP_SPLIT && !join) KCHK(launch_p2p_part(t, a, 0, t->p2p_split));
            else KCHK(launch_p2p(t, a));
        }
        if (a != s) KCHK(hipEventRecord(ctx->ev_near, a));
    }
    const int nlev = (int)t->ht.level_ptr.size() - 1;
    for (int l = nlev - 2; l >= t->m2m_top; --l) {
        ProfScope ps(ctx, s, "m2m");
        KCHK(launch_m2m_level(t, l, s));
    }
    if (join && a != s) KCHK(hipStreamWaitEvent(s, ctx->ev_near, 0));
    return FMM_OK;
}

// Queues the far field and the final combination (FMM) or the Barnes-Hut
// traversal; wait_near: join the near field forked by queue_upward right
// before the final L2P.  outputs & FMM_GRAD: for FMM the near-field gradient
// pass runs before the L2P, which then writes grad too; for BH the traversal
// kernel's gradient variant writes it.
static int queue_evaluate(fmm_ctx *ctx, fmm_tree *t, int outputs, double *phi, double *field, bool wait_near,
                          double *grad = nullptr, double *near_g = nullptr)
{
    hipStream_t s = ctx->stream;
    if (t->method == FMM_METHOD_BH) {
        ProfScope ps(ctx, s, "bh");
        KCHK(launch_bh(t, outputs, phi, field, grad, s));
        return FMM_OK;
    }
    const bool split = wait_near && ctx->overlap == FMM_OVERLAP_SPLIT;
    const bool tail = wait_near && ctx->overlap == FMM_OVERLAP_TAIL;
    if (split) KCHK(hipStreamWaitEvent(s, ctx->ev_near, 0));   // the first near-field half
    {
        ProfScope ps(ctx, s, "m2l");
        KCHK(launch_m2l(t, s));
    }
    if (split || tail) {
        // the near field (split: its second half) beside the combine and L2L
        KCHK(hipEventRecord(ctx->ev_m2l, s));
        KCHK(hipStreamWaitEvent(ctx->aux, ctx->ev_m2l, 0));
        {
            ProfScope ps(ctx, ctx->aux, "p2p");
            if (split) KCHK(launch_p2p_part(t, ctx->aux, t->p2p_split, -1));
            else KCHK(launch_p2p(t, ctx->aux));
        }
        KCHK(hipEventRecord(ctx->ev_near2, ctx->aux));
    }
    {
        ProfScope ps(ctx, s, "m2l_combine");
        KCHK(launch_m2l_combine(t, s));
    }
    const int nlev = (int)t->ht.level_ptr.size() - 1;
    for (int l = std::max(1, t->l2l_from); l < nlev; ++l) {
        ProfScope ps(ctx, s, "l2l");
        KCHK(launch_l2l_level(t, l, s));
    }
    if (split || tail) KCHK(hipStreamWaitEvent(s, ctx->ev_near2, 0));
    else if (wait_near && ctx->overlap) KCHK(hipStreamWaitEvent(s, ctx->ev_near, 0));
    if (outputs & FMM_GRAD) {
        ProfScope ps(ctx, s, "p2p_grad");
        KCHK(launch_p2p(t, s, true, near_g));
    }
    {
        ProfScope ps(ctx, s, "l2p");
        KCHK(launch_l2p_final(t, outputs, phi, field, grad, s, near_g));
    }
    return FMM_OK;
}

// FLOPs per P2P pair as counted in the FP32 kernel (multiply-add = 2,
// reciprocal square root = 1), potential and field
static double p2p_flops_mask(int m)
{
    return (m & 1 ? 20.0 : 0.0) + (m & 2 ? 32.0 : 0.0) + (m & 4 ? 58.0 : 0.0) + (m & 8 ? 100.0 : 0.0);
}

// algorithmic work of an evaluation (see fmm_work_counts)
static void set_work_counts(fmm_tree *t)
{
    if (t->method != FMM_METHOD_FMM) return;
    const int s_ = t->order, p = t->p;
    const int64_t nc = t->ht.ncells();
    const int nl = nterms(p - s_);
    const bool harm = t->basis == FMM_M2L_HARMONIC;
    // multiply-adds per list entry: outputs of order k times inputs of
    // orders s..p-k, all components or (harmonic basis) 2l+1 per order l
    double fc = 0;
    for (int k = 0; k <= p - s_; ++k)
        fc += harm ? (double)(2 * k + 1) * (hterms(p - k) - hterms(s_ - 1))
                   : (double)((k + 1) * (k + 2) / 2) * (nterms(p - k) - nterms(s_ - 1));
    const size_t es = t->prec == FMM_PREC_MIXED ? 4 : 8;
    t->work[1] = 2.0 * fc * t->work[0];
    t->work[3] = p2p_flops_mask(t->smask) * t->work[2];
    t->work[6] = harm ? (double)nc * (double)(hterms(p) - hterms(s_ - 1) + hterms(p - s_)) * es
                      : (double)nc * (double)(nterms(p) - nterms(s_ - 1) + nl) * es;
    t->work[7] = (double)t->ht.n * (es * (4 + 8) + 32);
}

extern "C" int fmm_upward(fmm_ctx *ctx, fmm_tree *t, int order, const double *moments, int p, int precision)
{
    int rc = check_upward_args(ctx, t, order, moments, p, precision);
    if (rc) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    t->have_up = 0;
    if ((rc = ensure_expansions(t, order, p, precision))) return rc;
    t->mom_user = moments;
    const int64_t key[kGraphKey] = {1, order, p, precision, (int64_t)(uintptr_t)moments, ctx->overlap, 0, 0, 0, 0};
    rc = run_cached(ctx, t, key, ctx->stream, [&]() { return queue_upward(ctx, t, true); });
    if (rc) return rc;
    t->have_up = 1;
    return FMM_OK;
}

extern "C" int fmm_evaluate(fmm_ctx *ctx, fmm_tree *t, int outputs, double *phi, double *field)
{
    int rc = check_eval_args(ctx, t, outputs, phi, field);
    if (rc) return rc;
    if (!t->have_up) FAIL(FMM_ESTATE, "fmm_upward has not run on this tree");
    HIPCHK(hipSetDevice(ctx->device));
    if (t->method == FMM_METHOD_BH) return queue_evaluate(ctx, t, outputs, phi, field, false);
    const int64_t key[kGraphKey] = {2, outputs, (int64_t)(uintptr_t)phi, (int64_t)(uintptr_t)field, 0, 0, 0, 0, 0, 0};
    rc = run_cached(ctx, t, key, ctx->stream, [&]() { return queue_evaluate(ctx, t, outputs, phi, field, false); });
    if (rc) return rc;
    set_work_counts(t);
    return FMM_OK;
}

extern "C" int fmm_evaluate_grad(fmm_ctx *ctx, fmm_tree *t, int outputs, double *phi, double *field, double *grad)
{
    if (!ctx || !t || t->ctx != ctx) FAIL(FMM_EINVAL, "null or foreign context/tree");
    if (outputs <= 0 || (outputs & ~(FMM_POT | FMM_FIELD | FMM_GRAD))) FAIL(FMM_EINVAL, "bad output mask %d", outputs);
    if ((outputs & FMM_POT) && !phi) FAIL(FMM_EINVAL, "potential requested but phi is NULL");
    if ((outputs & FMM_FIELD) && !field) FAIL(FMM_EINVAL, "field requested but field is NULL");
    if ((outputs & FMM_GRAD) && !grad) FAIL(FMM_EINVAL, "field gradient requested but grad is NULL");
    if (!t->have_up) FAIL(FMM_ESTATE, "fmm_upward has not run on this tree");
    if (t->method == FMM_METHOD_BH) {
        HIPCHK(hipSetDevice(ctx->device));
        return queue_evaluate(ctx, t, outputs, phi, field, false, grad);
    }
    if ((outputs & FMM_GRAD) && t->p - t->order < 2)
        FAIL(FMM_EINVAL, "field gradient needs p - s >= 2 (p = %d, lowest source order %d): below that the "
                         "truncated local expansion has no second derivative", t->p, t->order);
    HIPCHK(hipSetDevice(ctx->device));
    int rc;
    if ((outputs & FMM_GRAD) && !t->d_near_g &&
        (rc = tree_alloc(t, (void **)&t->d_near_g, sizeof(double) * 6 * (size_t)std::max<int64_t>(1, t->ht.n))))
        return rc;
    const int64_t key[kGraphKey] = {4, outputs, (int64_t)(uintptr_t)phi, (int64_t)(uintptr_t)field,
                                    (int64_t)(uintptr_t)grad, 0, 0, 0, 0, 0};
    rc = run_cached(ctx, t, key, ctx->stream,
                    [&]() { return queue_evaluate(ctx, t, outputs, phi, field, false, grad); });
    if (rc) return rc;
    set_work_counts(t);
    return FMM_OK;
}

extern "C" int fmm_evaluate_grad_noalloc(fmm_ctx *ctx, fmm_tree *t, int outputs, double *phi, double *field,
                                         double *grad)
{
    if (!ctx || !t || t->ctx != ctx) FAIL(FMM_EINVAL, "null or foreign context/tree");
    if (outputs <= 0 || (outputs & ~(FMM_POT | FMM_FIELD | FMM_GRAD))) FAIL(FMM_EINVAL, "bad output mask %d", outputs);
    if ((outputs & FMM_POT) && !phi) FAIL(FMM_EINVAL, "potential requested but phi is NULL");
    if ((outputs & FMM_FIELD) && !field) FAIL(FMM_EINVAL, "field requested but field is NULL");
    if ((outputs & FMM_GRAD) && !grad) FAIL(FMM_EINVAL, "field gradient requested but grad is NULL");
    if (!t->have_up) FAIL(FMM_ESTATE, "fmm_upward has not run on this tree");
    HIPCHK(hipSetDevice(ctx->device));
    // kernels launched one by one (a graph would be instantiated on the
    // first call); Barnes-Hut trees write the gradient from the traversal
    // kernel and use no scratch
    if (t->method == FMM_METHOD_BH) return queue_evaluate(ctx, t, outputs, phi, field, false, grad);
    if ((outputs & FMM_GRAD) && t->p - t->order < 2)
        FAIL(FMM_EINVAL, "field gradient needs p - s >= 2 (p = %d, lowest source order %d)", t->p, t->order);
    double *near_g = nullptr;
    if (outputs & FMM_GRAD) {
        if (t->ht.n > kNoAllocMaxN)
            FAIL(FMM_EINVAL, "n = %lld exceeds the %lld particles the allocation-free scratch holds; use "
                             "fmm_evaluate_grad", (long long)t->ht.n, (long long)kNoAllocMaxN);
        if (!ctx->noalloc_scratch) FAIL(FMM_ESTATE, "context has no scratch address");
        near_g = ctx->noalloc_scratch;
    }
    const int rc = queue_evaluate(ctx, t, outputs, phi, field, false, grad, near_g);
    if (rc) return rc;
    set_work_counts(t);
    return FMM_OK;
}

extern "C" int fmm_evaluate_derivs(fmm_ctx *ctx, fmm_tree *t, int K, double *out)
{
    if (!ctx || !t || t->ctx != ctx) FAIL(FMM_EINVAL, "null or foreign context/tree");
    if (!out) FAIL(FMM_EINVAL, "out is NULL");
    if (K < 1 || K > 3) FAIL(FMM_EINVAL, "derivative order %d (1, 2 or 3)", K);
    if (!t->have_up) FAIL(FMM_ESTATE, "fmm_upward has not run on this tree");
    if (t->method == FMM_METHOD_BH) {
        // Eq. 6 differentiated K times on the Eq. 12 traversal: no truncation
        // limit beyond the multipole order itself
        HIPCHK(hipSetDevice(ctx->device));
        ProfScope ps(ctx, ctx->stream, "bh_derivs");
        KCHK(launch_bh_derivs(t, K, out, ctx->stream));
        return FMM_OK;
    }
    if (K > t->p - t->order)
        FAIL(FMM_EINVAL, "derivative order %d exceeds p - s = %d: the truncated local expansion has no "
                         "derivative of that order", K, t->p - t->order);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // the locals of the leaves (as fmm_evaluate forms them), then Eq. 10 and
    // the pairs' derivatives in one pass
    {
        ProfScope ps(ctx, s, "m2l");
        KCHK(launch_m2l(t, s));
    }
    {
        ProfScope ps(ctx, s, "m2l_combine");
        KCHK(launch_m2l_combine(t, s));
    }
    const int nlev = (int)t->ht.level_ptr.size() - 1;
    for (int l = std::max(1, t->l2l_from); l < nlev; ++l) {
        ProfScope ps(ctx, s, "l2l");
        KCHK(launch_l2l_level(t, l, s));
    }
    {
        ProfScope ps(ctx, s, "derivs");
        KCHK(launch_derivs(t, K, out, s));
    }
    return FMM_OK;
}

extern "C" int fmm_run(fmm_ctx *ctx, fmm_tree *t, int order, const double *moments, int p, int precision, int outputs,
                       double *phi, double *field)
{
    int rc = check_upward_args(ctx, t, order, moments, p, precision);
    if (rc || (rc = check_eval_args(ctx, t, outputs, phi, field))) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    t->have_up = 0;
    if ((rc = ensure_expansions(t, order, p, precision))) return rc;
    t->mom_user = moments;
    // one launch sequence: the near field overlaps the whole far field and is
    // joined before the final L2P
    const int64_t key[kGraphKey] = {3, order, p, precision, (int64_t)(uintptr_t)moments, ctx->overlap,
                                    outputs, (int64_t)(uintptr_t)phi, (int64_t)(uintptr_t)field, 0};
    rc = run_cached(ctx, t, key, ctx->stream, [&]() {
        const int r = queue_upward(ctx, t, false);
        return r ? r : queue_evaluate(ctx, t, outputs, phi, field, true);
    });
    if (rc) return rc;
    t->have_up = 1;
    set_work_counts(t);
    return FMM_OK;
}

extern "C" int fmm_work_counts(const fmm_tree *t, double *w)
{
    if (!t || !w) FAIL(FMM_EINVAL, "null argument");
    for (int k = 0; k < 8; ++k) w[k] = t->work[k];
    if (t->method == FMM_METHOD_BH && t->d_bhcount && t->have_up) {
        // counted by the traversal kernel itself (synchronises the stream)
        unsigned long long c[2] = {0, 0};
        HIPCHK(hipSetDevice(t->ctx->device));
        HIPCHK(hipMemcpyAsync(c, t->d_bhcount, sizeof(c), hipMemcpyDeviceToHost, t->ctx->stream));
        HIPCHK(hipStreamSynchronize(t->ctx->stream));
        const int p = t->p, s_ = t->order;
        // contraction terms and derivative-tensor components up to p + 1
        // (harmonic basis: the components with m_z <= 1, k_z <= 2)
        double nm = (double)(nterms(p) - nterms(s_ - 1));
        double np4 = (double)(p + 4) * (p + 3) * (p + 2) / 6.0;   // C(p+4, 3)
        if (t->basis == FMM_M2L_HARMONIC) {
            nm = (double)(hterms(p) - hterms(s_ - 1));
            np4 = 0.0;
            for (int l = 0; l <= p + 1; ++l)
                for (int kz = 0; kz <= std::min(2, l); ++kz) np4 += (double)(l - kz + 1);
        }
        w[2] = (double)c[1];
        w[3] = p2p_flops_mask(t->smask) * w[2];
        w[4] = (double)c[0];
        w[5] = (8.0 * nm + 12.0 * np4) * w[4];
    }
    return FMM_OK;
}

extern "C" int fmm_tree_info(const fmm_tree *t, int64_t *info)
{
    if (!t || !info) FAIL(FMM_EINVAL, "null argument");
    const HostTree &h = t->ht;
    info[0] = h.n;
    info[1] = h.ncells();
    info[2] = (int64_t)h.level_ptr.size() - 1;
    info[3] = t->nleaves;
    info[4] = t->tiling.on_device ? t->tiling.pairs : h.m2l_ptr.empty() ? 0 : h.m2l_ptr.back();
    info[5] = h.p2p_ptr.empty() ? 0 : h.p2p_ptr.back();
    info[6] = t->tiling.nclasses;
    info[7] = t->tiling.ntiles;
    info[8] = t->tiling.nentries * kTileW;
    info[9] = (int64_t)t->dev_bytes;
    return FMM_OK;
}

extern "C" int fmm_tree_m2l_schedule(const fmm_tree *t, int32_t *tile_cell, int32_t *tile_uoff, int32_t *ucls,
                                     int32_t *usrc, double *cls_geom, int *where)
{
    if (!t) FAIL(FMM_EINVAL, "null tree");
    if (t->method != FMM_METHOD_FMM) FAIL(FMM_EINVAL, "a Barnes-Hut tree has no M2L schedule");
    if (!t->ctx) FAIL(FMM_EINVAL, "the tree's context was destroyed");
    const M2LTiling &tl = t->tiling;
    if (where) *where = tl.on_device ? FMM_SCHEDULE_DEVICE : FMM_SCHEDULE_HOST;
    auto cp = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(tile_cell, tl.tile_cell);
    cp(tile_uoff, tl.tile_uoff);
    HIPCHK(hipSetDevice(t->ctx->device));
    hipStream_t s = t->ctx->stream;
    // the tables as the M2L reads them (device copies of either schedule)
    if (ucls && tl.nentries)
        HIPCHK(hipMemcpyAsync(ucls, t->d_ucls, sizeof(int32_t) * tl.nentries, hipMemcpyDeviceToHost, s));
    if (usrc && tl.nentries)
        HIPCHK(hipMemcpyAsync(usrc, t->d_usrc, sizeof(int32_t) * tl.nentries * kTileW, hipMemcpyDeviceToHost, s));
    if (cls_geom && tl.nclasses)
        HIPCHK(hipMemcpyAsync(cls_geom, t->d_cls_geom, sizeof(double) * 4 * tl.nclasses, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FMM_OK;
}

extern "C" int fmm_tree_export(const fmm_tree *t, double *geom, uint64_t *key, int64_t *perm, int32_t *level,
                               int32_t *ix, int64_t *first, int64_t *count, int64_t *parent, int64_t *child0,
                               int32_t *nchild, int64_t *m2l_ptr, int64_t *m2l_src, int64_t *p2p_ptr, int64_t *p2p_src)
{
    if (!t) FAIL(FMM_EINVAL, "null tree");
    const HostTree &h = t->ht;
    auto cp = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    if (geom) {
        geom[0] = h.lo[0];
        geom[1] = h.lo[1];
        geom[2] = h.lo[2];
        geom[3] = h.W;
    }
    if (key || perm) {
        // the order and the keys stayed on the device
        if (!t->ctx) FAIL(FMM_EINVAL, "the tree's context was destroyed");
        HIPCHK(hipSetDevice(t->ctx->device));
        hipStream_t s = t->ctx->stream;
        std::vector<int32_t> p32(perm ? h.n : 0);
        if (key) HIPCHK(hipMemcpyAsync(key, t->d_key, sizeof(uint64_t) * h.n, hipMemcpyDeviceToHost, s));
        if (perm) HIPCHK(hipMemcpyAsync(p32.data(), t->d_perm, sizeof(int32_t) * h.n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (perm) std::copy(p32.begin(), p32.end(), perm);
    }
    cp(level, h.level);
    cp(ix, h.ix);
    cp(first, h.first);
    cp(count, h.count);
    cp(parent, h.parent);
    cp(child0, h.child0);
    cp(nchild, h.nchild);
    if (t->tiling.on_device && (m2l_ptr || m2l_src)) {
        // the lists stayed on the device
        if (!t->ctx) FAIL(FMM_EINVAL, "the tree's context was destroyed");
        HIPCHK(hipSetDevice(t->ctx->device));
        hipStream_t s = t->ctx->stream;
        const int64_t nc = h.ncells(), m = t->tiling.pairs;
        std::vector<int32_t> p32(nc + 1), s32(m);
        HIPCHK(hipMemcpyAsync(p32.data(), t->d_m2l_ptr, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost, s));
        if (m) HIPCHK(hipMemcpyAsync(s32.data(), t->d_m2l_src, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (m2l_ptr) std::copy(p32.begin(), p32.end(), m2l_ptr);
        if (m2l_src) std::copy(s32.begin(), s32.end(), m2l_src);
    } else {
        cp(m2l_ptr, h.m2l_ptr);
        cp(m2l_src, h.m2l_src);
    }
    cp(p2p_ptr, h.p2p_ptr);
    const int64_t np2p = h.p2p_ptr.empty() ? 0 : h.p2p_ptr.back();
    if (p2p_src && np2p > 0 && h.p2p_src.empty()) {
        // the sources stayed on the device, in the same CSR order
        if (!t->ctx) FAIL(FMM_EINVAL, "the tree's context was destroyed");
        HIPCHK(hipSetDevice(t->ctx->device));
        hipStream_t s = t->ctx->stream;
        std::vector<int32_t> s32(np2p);
        HIPCHK(hipMemcpyAsync(s32.data(), t->d_p2p_src, sizeof(int32_t) * np2p, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::copy(s32.begin(), s32.end(), p2p_src);
    } else {
        cp(p2p_src, h.p2p_src);
    }
    return FMM_OK;
}
