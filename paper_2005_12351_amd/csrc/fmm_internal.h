// Internal declarations of libfmm.so (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <chrono>
#include <functional>
#include <map>
#include <vector>

#include "../../include/fmm.h"

// ------------------------------------------------------------------ indexing
// Coefficients are ordered by total order k, then n_x descending, then n_y
// descending (the default lexicographic mapping of Section 3.1).
__host__ __device__ constexpr int nterms(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int mindex(int nx, int ny, int nz)
{
    return nterms(nx + ny + nz - 1) + (ny + nz) * (ny + nz + 1) / 2 + nz;
}

constexpr int kMaxLevel = 21;        // 21 bits per axis, 63-bit keys
constexpr int kTileW = 64;           // targets per M2L tile = wavefront width
constexpr int kPTable = 12;
constexpr int kGraphKey = 10;        // arguments a captured launch sequence is keyed by          // multi-index tables cover orders <= 12

struct MultiIndex { int8_t x, y, z, k; };

// Source order codes: 0, 1, 2, 3 for one order (charge, dipole, quadrupole,
// octupole), or FMM_MIXED + a bit mask of the orders present in one system
// (bit k: order k); moment rows hold the present orders' physical moments in
// ascending order, (k+1)(k+2)/2 values for order k.
__host__ __device__ constexpr int code_mask(int code) { return code >= FMM_MIXED ? code - FMM_MIXED : 1 << code; }
__host__ __device__ constexpr int mask_width(int m)
{
    return (m & 1 ? 1 : 0) + (m & 2 ? 3 : 0) + (m & 4 ? 6 : 0) + (m & 8 ? 10 : 0);
}
__host__ __device__ constexpr int mask_min_order(int m) { return m & 1 ? 0 : (m & 2 ? 1 : (m & 4 ? 2 : 3)); }
__host__ __device__ constexpr bool mask_single(int m) { return m == 1 || m == 2 || m == 4 || m == 8; }
// FP32 moments per particle, in float4 groups: one order of 0..2: 8 floats
// (q | mu | six Q and the trace); octupoles alone: 16 ([O xxx xxy xxz xyy]
// [xyz xzz yyy yyz] [yzz zzz t_x t_y] [t_z 0 0 0], t the trace vector
// t_k = sum_i O_iik); several orders: 12 ([q mu] [xx xy xz yy] [yz zz tr 0],
// absent parts 0), followed by the 16 of the octupole block when that order
// is present
__host__ __device__ constexpr int m32_width(int m)
{
    return mask_single(m) ? (m == 8 ? 16 : 8) : ((m & 8) ? 28 : 12);
}

// Harmonic (reduced) basis: the components with n_z <= 1 of every order, in
// storage order; order l holds 2l+1 of them and starts at index l^2.
__host__ __device__ constexpr int hindex(int nx, int ny, int nz)
{
    return (nx + ny + nz) * (nx + ny + nz) + (ny + nz == 0 ? 0 : 2 * (ny + nz) - 1 + nz);
}
__host__ __device__ constexpr int hterms(int p) { return p < 0 ? 0 : (p + 1) * (p + 1); }
// the multi-index of harmonic component h (the inverse of hindex)
__host__ __device__ inline void hmulti(int h, int &nx, int &ny, int &nz)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= h) ++l;
    const int off = h - l * l, t = (off + 1) / 2;
    nz = off == 0 ? 0 : off - (2 * t - 1);
    ny = t - nz;
    nx = l - t;
}

// Folding onto the harmonic basis.  Component h = (a, b, r), r <= 1, of a
// folded multipole row is
//   sum_j (-1)^j sum_i C(j,i) row[(a - 2i, b - 2(j - i), r + 2j)],
// which carries the row's contraction with any harmonic tensor D (such as
// the derivatives of 1/r, D_{k+2e_x} + D_{k+2e_y} + D_{k+2e_z} = 0) onto the
// components with m_z <= 1 without changing it; the order is kept.  The
// terms are tabulated once: for h, entries [start[h], start[h+1]) hold the
// row index and the signed binomial weight.
constexpr int kFoldTerms = 1036;   // terms of all components up to order kPTable
struct FoldTable {
    int16_t start[hterms(kPTable) + 1];
    int16_t idx[kFoldTerms];
    float w[kFoldTerms];
};
constexpr FoldTable make_fold()
{
    FoldTable f{};
    int e = 0, h = 0;
    for (int l = 0; l <= kPTable; ++l)
        for (int t = 0; t <= l; ++t)
            for (int r = 0; r <= (t == 0 ? 0 : 1); ++r) {
                f.start[h++] = (int16_t)e;
                const int a = l - t, b = t - r;
                for (int j = 0; 2 * j <= a + b; ++j) {
                    int c = 1;   // C(j, i)
                    for (int i = 0; i <= j; ++i) {
                        if (a - 2 * i >= 0 && b - 2 * (j - i) >= 0) {
                            f.idx[e] = (int16_t)mindex(a - 2 * i, b - 2 * (j - i), r + 2 * j);
                            f.w[e] = (float)((j & 1) ? -c : c);
                            ++e;
                        }
                        c = c * (j - i) / (i + 1);
                    }
                }
            }
    f.start[h] = (int16_t)e;
    return f;
}

// multi-indices in storage order (total order ascending; within an order
// n_x descending, then n_y descending), up to order kPTable
struct MITable {
    MultiIndex v[nterms(kPTable)];
};
constexpr MITable make_mi()
{
    MITable t{};
    int i = 0;
    for (int k = 0; k <= kPTable; ++k)
        for (int nx = k; nx >= 0; --nx)
            for (int ny = k - nx; ny >= 0; --ny) t.v[i++] = MultiIndex{(int8_t)nx, (int8_t)ny, (int8_t)(k - nx - ny), (int8_t)k};
    return t;
}

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
#define FMM_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return FMM_EDEVICE;                                                    \
        }                                                                          \
    } while (0)

// ------------------------------------------------------------------ tree
struct DevCell {       // 48 bytes, canonical order
    int32_t level, ix, iy, iz;
    int32_t first, count, parent, child0;
    int32_t nchild, pad0, pad1, pad2;
};

struct HostTree {      // canonical tree, host copy
    int64_t n = 0;
    double lo[3] = {0, 0, 0}, W = 1.0, h = 0.0;
    std::vector<uint64_t> key;
    std::vector<int64_t> perm;
    std::vector<int32_t> level, ix;        // ix: 3 per cell
    std::vector<int64_t> first, count, parent, child0;
    std::vector<int32_t> nchild;
    std::vector<int64_t> level_ptr;        // nlevels + 1
    std::vector<int64_t> m2l_ptr, m2l_src, p2p_ptr, p2p_src;
    // per cell: its particle count times the particles of its P2P sources
    // (filled when the P2P sources stay on the device; p2p_src is empty then)
    std::vector<int64_t> p2p_cost;
    int64_t ncells() const { return (int64_t)level.size(); }
};

// canonical tree and (if lists) the dual-tree interaction lists of n device
// positions, built on the GPU on stream s and returned in host form
// (tree_gpu.hip).  hipErrorInvalidValue: a position is not finite;
// hipErrorOutOfMemory: a list or frontier exceeds 2^31 entries or the device
// is out of memory.
// The context's pinned staging buffer, grown to at least `bytes` (its
// earlier contents are lost then); no copy through it may be in flight.
// Copies from pageable memory go through one staging buffer of the runtime
// and serialise the host threads of all contexts; these do not.
hipError_t ctx_pinned(fmm_ctx *ctx, size_t bytes, char **base);
// most bytes a context keeps cached in released tree blocks, and in its
// build arena
size_t ctx_cache_limit(const fmm_ctx *ctx);
// the context's build arena grown to at least `bytes` (at most the cache
// limit), allocated on its stream and waited for (tree_gpu.hip)
hipError_t ctx_arena_reserve(fmm_ctx *ctx, size_t bytes);

// stable sort of n (key, value) pairs on the low `bits` key bits into
// kout/vout (sort.hip); with tmp null only sets tmp_bytes
hipError_t dev_sort_pairs(void *tmp, size_t &tmp_bytes, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                          int32_t *vout, int n, int bits, hipStream_t s);

struct DevKeep;
hipError_t gpu_build_tree(const double *pos, int64_t n, int ncrit, double theta, bool lists, hipStream_t s,
                          HostTree &t, fmm_ctx *ctx = nullptr, DevKeep *dt = nullptr);

// M2L tiling (tree_host.cpp)
struct M2LTiling {
    int ntiles = 0, nclasses = 0;
    int64_t nentries = 0;                  // union entries over all tiles
    std::vector<int32_t> tile_cell;        // ntiles*64: target cell or -1
    std::vector<int32_t> tile_uoff;        // ntiles+1: entry range of each tile
    std::vector<int32_t> ucls;             // nentries: class id
    std::vector<int32_t> usrc;             // nentries*64: source cell (or zero row)
    std::vector<double> cls_geom;          // nclasses*4: (z_B - z_A)/r_B, r_A/r_B
    int64_t pairs = 0;                     // real list entries
    bool on_device = false;                // ucls, usrc, cls_geom exist on the device only
};
void build_m2l_tiling(const HostTree &t, M2LTiling &out);
// f(i) for i in [0, n) on the host threads of the scheduling passes
// (tree_host.cpp); each i must write its own results only.  Below
// serial_below items the calling thread does them all: waking the pool
// costs tens of microseconds, more than small loops take.
void host_parallel_for(int64_t n, const std::function<void(int64_t)> &f, int64_t serial_below = 0);

// Device buffers of a tree that gpu_build_tree (tree_gpu.hip) leaves on
// the device: `keep` allocates them (the tree's own allocations).  Always:
// cells (DevCell per cell), perm (input index of sorted particle i, int32)
// and key (sorted Morton keys); the host tree then holds neither perm nor
// key.  With `tiling`, also the M2L tiling of build_m2l_tiling made on the
// device: on return `done` says whether it is complete (false: a packed key
// would overflow, or a tile has more distinct pair geometries than the
// device table holds, and the host code must build it from the host lists).
// `tl` receives its host parts (sizes, tile_cell, tile_uoff, pairs).  When
// done, the M2L lists stay on the device (m2l_ptr over ncells + 1, m2l_src)
// and the host tree holds none; tgt_top / src_top are the shallowest target
// and source levels of the lists (-1: no list).
struct DevKeep {
    std::function<hipError_t(void **, size_t)> keep;
    DevCell *cells = nullptr;
    int32_t *perm = nullptr;
    uint64_t *key = nullptr;
    bool tiling = false;
    int64_t min_pairs = 0;   // the device tiling only for at least this many M2L pairs
    int32_t *ucls = nullptr, *usrc = nullptr, *cell_slot = nullptr;
    int32_t *m2l_ptr = nullptr, *m2l_src = nullptr;
    // With lists: the P2P sources stay on the device (CSR over the cells by
    // the host's p2p_ptr; only leaves have entries, so it is also the
    // per-leaf CSR in leaf order), and the host gets per-cell costs instead.
    int32_t *p2p_src = nullptr;
    double *cls_geom = nullptr;
    M2LTiling *tl = nullptr;
    int tgt_top = -1, src_top = -1;
    bool done = false;
};

// M2L work for one kernel variant: the (tile, output block, entry) units,
// concatenated, are cut into nwaves pieces of equal cost, one per resident
// M2L workgroup (whose waves split it); a piece that
// crosses a (tile, block) boundary becomes several items, each with its own
// 64 partial-result rows
struct M2LWork {
    std::vector<int32_t> work;             // nitems*4: tile | block << 24, u0, u1, first row
    std::vector<int32_t> wave_ptr;         // nwaves+1: items of each piece
    std::vector<int32_t> chunk0, nchunk;   // per (tile, block): first row set, row-set count
    int64_t nrows = 0;
    int nwaves = 0;
};

// ------------------------------------------------------------------ M2L kernels
struct M2LArgs {
    const int4 *work;          // x = tile | block << 24, y/z = entry range, w = first output row
    const int32_t *ucls, *usrc;
    const void *D, *sc, *M;
    void *part;
    const int32_t *wave_ptr;   // items of workgroup w's piece: work[wave_ptr[w] .. wave_ptr[w+1])
    int zero;                  // always 0; offsets the table pointer per chunk so
                               // that the compiler reloads instead of keeping it live
};
// generated dispatch (m2l_generated_*.hip)
typedef hipError_t (*m2l_launch_fn)(const M2LArgs &, int nwaves, hipStream_t);
struct M2LVariant {
    m2l_launch_fn launch;
    int (*occupancy)();        // resident workgroups per CU
    int nl_pad, nm_pad, nd, nblocks;
    int blo[17];               // output blocks: coefficients [blo[b], blo[b+1])
    int bfma[16];              // multiply-adds per list entry in each block
};
// mfma: the matrix-core kernels (FP32 harmonic basis only)
bool m2l_lookup(int p, int s, bool fp32, bool harmonic, M2LVariant *out, bool mfma = false);
void build_m2l_work(const M2LTiling &tl, const M2LVariant &v, int nwaves, M2LWork &out);

// ------------------------------------------------------------------ context
// a kernel range between two events, or (a null) a host phase of host_ms
struct ProfEntry { const char *name; hipEvent_t a, b; double host_ms; };

struct fmm_ctx {
    int device = 0;
    hipStream_t stream = nullptr, aux = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    bool profile = false;
    int overlap = 0;                      // P2P on the auxiliary stream: 0 off, 1 whole, 2 split (FMM_OVERLAP_*)
    bool graphs = true;                   // replay captured HIP graphs
    int m2l_basis = FMM_M2L_HARMONIC;     // basis of the M2L contraction (FMM trees)
    int m2l_engine = FMM_M2L_ENGINE_AUTO; // units of the FP32 harmonic-basis M2L
    int m2l_schedule = FMM_SCHEDULE_AUTO;     // where tree builds make the M2L schedule
    bool fake = false;                    // no device: serving-logic tests only
    double fake_ns = 0.0;                 // simulated cost per particle (fake)
    size_t tree_limit = 0;                // device bytes one tree may hold (0: no limit)
    double *noalloc_scratch = nullptr;    // device address of the static gradient scratch on `device`
    void *pinned = nullptr;               // pinned host staging of tree construction's copies
    size_t pinned_bytes = 0;
    int64_t *pin_small = nullptr;         // pinned words for the totals a tree build reads back
    // coherent host words a tree build's read-backs arrive in: a one-thread
    // kernel writes the words, then the sequence number sig_seq, which the
    // host polls (tree_gpu.hip, read_words)
    int64_t *sig = nullptr, *sig_dev = nullptr;
    int64_t sig_seq = 0;
    int ncu = 256;                        // compute units of the device
    // Device blocks released by this context's trees, by size class, reused
    // in the order of the context stream (tree_alloc); and the scratch
    // arena of its tree builds (gpu_build_tree).  The stream-ordered
    // allocator serialises the host threads of all contexts, so a context
    // that serves one request after another calls it only to grow these.
    std::multimap<size_t, void *> dev_cache;
    size_t dev_cache_bytes = 0;
    char *arena = nullptr;
    size_t arena_cap = 0;
    hipEvent_t ev_fork = nullptr;
    std::vector<ProfEntry> prof;
    std::vector<hipEvent_t> ev_pool;
    hipEvent_t ev_up = nullptr, ev_near = nullptr;
    hipEvent_t ev_m2l = nullptr, ev_near2 = nullptr;   // split overlap: M2L queued, second P2P part done
    hipEvent_t ev_upload = nullptr;       // after the copies of the last flush of uploads from `pinned`
    bool upload_pending = false;          // ev_upload recorded and not yet waited for
    struct Server *server = nullptr;
    std::vector<struct fmm_tree *> trees;  // live trees; released with the context
};

struct fmm_tree {
    fmm_ctx *ctx = nullptr;
    int method = FMM_METHOD_FMM, ncrit = 0;
    double theta = 0.5;
    HostTree ht;
    int64_t nleaves = 0;
    std::vector<int32_t> leaves;           // cell index of every leaf
    std::vector<int32_t> level_nonleaf_ptr, level_nonleaf;  // M2M work per level
    int m2m_top = 0;                       // shallowest parent level M2M runs into
    int l2l_from = 1;                      // shallowest child level L2L runs into
    M2LTiling tiling;
    // device copies
    DevCell *d_cells = nullptr;
    int32_t *d_perm = nullptr, *d_leaves = nullptr;
    int32_t *d_nonleaf = nullptr, *d_level_cells = nullptr;
    double *d_x = nullptr;                 // sorted positions, SoA x[n] y[n] z[n]
    int32_t *d_p2p_ptr = nullptr, *d_p2p_src = nullptr;   // per leaf, sources as cell ids
    int4 *d_work = nullptr;                // per expansion configuration
    int32_t *d_ucls = nullptr, *d_usrc = nullptr, *d_cell_slot = nullptr;   // cell -> tile slot or -1
    int32_t *d_m2l_ptr = nullptr, *d_m2l_src = nullptr;   // M2L lists, kept when the host holds none
    uint64_t *d_key = nullptr;                            // sorted Morton keys (the host holds none)
    int32_t *d_tile_chunk0 = nullptr, *d_tile_nchunk = nullptr;
    int32_t *d_p2p_order = nullptr;        // leaf ordinals by decreasing near-field cost
    int p2p_split = 0;                     // first position of p2p_order past half the near-field cost
    int32_t *d_l2p_pack = nullptr;         // L2P: leaf-ordinal range of every wave
    int l2p_npacks = 0, l2p_pack_q = -1;
    bool l2p_columns = false;              // L2P keeps the locals as packed columns (see l2p_columns_pay)
    int32_t *d_wave_ptr = nullptr;
    M2LWork m2lwork;
    double *d_cls_geom = nullptr;
    unsigned long long *d_bhcount = nullptr;   // Barnes-Hut interaction counters (2)
    // per expansion state
    int have_up = 0, order = 0, p = 0, prec = 0, dtab_p = -1;   // order: the lowest source order s
    int smask = 1;                         // source orders present (bit mask)
    int basis = FMM_M2L_FULL;              // M2L basis the expansions were set up for
    bool mfma = false;                     // the M2L runs on the matrix cores (FP32 harmonic basis)
    int nhp = 0;                           // row stride of the folded multipoles d_Mh (harmonic basis)
    const double *mom_user = nullptr;
    double *d_mom = nullptr;               // sorted moments FP64 (w per particle)
    float *d_mom32 = nullptr;              // sorted moments FP32 (8 per particle)
    // Expansion storage.  Full basis: every component, d_M64 (FP64, the
    // upward state; d_M32 its FP32 copy in MIXED) and d_L64 (nterms(p - s)
    // per cell).  Harmonic basis, O(p^2) per cell: the multipoles only as
    // rows folded onto their m_z <= 1 components (d_Mh in the M2L precision,
    // plus the FP64 state d_Mf64 in MIXED; in FP64 d_Mh is the state), the
    // locals only as their n_z <= 1 components (d_L64, hterms(p - s) per
    // cell), the rest of a local row rebuilt where it is read.
    double *d_M64 = nullptr;
    float *d_M32 = nullptr;
    void *d_Mh = nullptr;                  // harmonic basis: reduced multipole rows (M2L precision)
    double *d_Mf64 = nullptr;              // harmonic basis, MIXED: FP64 folded rows (stride nhp)
    void *d_part = nullptr;
    double *d_L64 = nullptr;
    double *d_near = nullptr;              // 4 per particle
    double *d_near_g = nullptr;            // 6 per particle: near-field gradient (allocated on first use)
    double *d_D64 = nullptr, *d_sc64 = nullptr;
    float *d_D32 = nullptr, *d_sc32 = nullptr;
    size_t dev_bytes = 0;
    std::vector<std::pair<void *, size_t>> allocs;   // every device block the tree holds, with its size
    // captured launch sequences, keyed by the arguments they bake in
    struct GraphEntry {
        int64_t key[kGraphKey];
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    double work[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

// allocation helper that records the block on the tree
int tree_alloc(fmm_tree *t, void **p, size_t bytes);

// profiling helper: launch wrapper
struct ProfScope {
    fmm_ctx *ctx;
    hipStream_t s;
    const char *name;
    hipEvent_t b = nullptr;
    ProfScope(fmm_ctx *c, hipStream_t st, const char *nm);
    ~ProfScope();
};

// wall-clock time of a host phase (tree construction, set-up), recorded
// with the kernel ranges while profiling is on
struct HostScope {
    fmm_ctx *ctx;
    const char *name;
    std::chrono::steady_clock::time_point t0;
    bool done = false;
    HostScope(fmm_ctx *c, const char *nm) : ctx(c), name(nm), t0(std::chrono::steady_clock::now()) {}
    // records the phase now (once; the destructor then records nothing)
    void end()
    {
        if (done) return;
        done = true;
        if (!ctx || !ctx->profile) return;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ctx->prof.push_back(ProfEntry{name, nullptr, nullptr, ms});
    }
    ~HostScope() { end(); }
};

// kernels entry points (host launchers), return hipError_t
hipError_t launch_prep_positions(fmm_tree *t, const double *pos, hipStream_t s);
hipError_t launch_p2m(fmm_tree *t, hipStream_t s);
hipError_t launch_m2m_level(fmm_tree *t, int level, hipStream_t s);
hipError_t launch_dtable(fmm_tree *t, hipStream_t s);
hipError_t launch_fill(double *p, size_t count, hipStream_t s);
hipError_t launch_m2l(fmm_tree *t, hipStream_t s);
hipError_t launch_m2l_combine(fmm_tree *t, hipStream_t s);
hipError_t launch_l2l_level(fmm_tree *t, int level, hipStream_t s);
// grad: field gradient to near_g (NULL: the tree's d_near_g)
hipError_t launch_p2p(fmm_tree *t, hipStream_t s, bool grad = false, double *near_g = nullptr);
hipError_t launch_l2p_final(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s,
                            const double *near_g = nullptr);
// largest particle count of the allocation-free gradient call, and the
// device address of its static scratch (6 doubles per particle) on the
// current device, resolved once per device
constexpr int64_t kNoAllocMaxN = 1 << 18;
hipError_t noalloc_scratch(int device, double **ptr);
int l2p_pack_limit(int q, bool cols);   // leaves one L2P wave may take at expansion order q, per layout
bool l2p_columns_pay(int q, int npacks, int ncu);   // L2P layout choice for a launch of npacks waves
hipError_t launch_bh(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s);
// P2P over the leaves p2p_order[first .. first + count) (count < 0: to the end)
hipError_t launch_p2p_part(fmm_tree *t, hipStream_t s, int first, int count);
// derivatives of order K (1..3) of the potential at every particle, out in
// caller order, (K+1)(K+2)/2 per particle; needs the locals (M2L, L2L) queued
hipError_t launch_derivs(fmm_tree *t, int K, double *out, hipStream_t s);
hipError_t launch_bh_derivs(fmm_tree *t, int K, double *out, hipStream_t s);

// serving (serve.cpp)
int serve_destroy(fmm_ctx *ctx);
