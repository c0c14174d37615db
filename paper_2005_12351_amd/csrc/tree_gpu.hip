// Octree construction and dual-tree interaction lists on the GPU (Pepper &
// Fangohr, arXiv 2005.12351, Section 3.2): root box, 21-bit quantisation,
// Morton keys, stable sort, adaptive octree (split while a cell holds more
// than ncrit particles, depth cap 21), and the dual traversal with the FMM
// acceptance criterion (Eq. 13), which yields the M2L and P2P lists.
//
// Canonical definitions (the same as the test oracle's, shared by
// specification only): root cube of side W = largest extent at the
// componentwise minimum; q = floor((x - lo) * 2^21 / W) clamped to 2^21 - 1;
// key = bit interleave with x most significant in every octal digit; stable
// sort by key; cells level-major in ascending key order, children in octant
// order, empty children not created; geometry in units of h = W 2^-22 with
// centre (2i+1) 2^(21-l) and radius (half side) 2^(21-l); acceptance
// (rA + rB)^2 < theta^2 d^2 evaluated in FP64 on exact integers; when a pair
// is neither accepted nor a leaf pair the larger cell is split (both on a
// tie; a leaf is never split).  Each target's lists are sorted by source.
//
// Layout of the work: stable sorts (a bitonic sort in LDS on (key, position)
// for small inputs, the library's LSD radix sort with 8-bit digits for the
// rest), eight lanes per cell and one pass per level for the tree, and a
// breadth-first traversal over a frontier of cell pairs with prefix sums for
// the output positions, so that every pass is deterministic.  The host reads
// back only totals (sizes of the next level or frontier).  After the lists,
// the M2L schedule is made here too (see launch_tiling).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <vector>

#include "fmm_internal.h"

namespace {

constexpr int kScanT = 256;           // threads per scan block
constexpr int kScanI = 4;             // items per thread
constexpr int kScanTile = kScanT * kScanI;

// ---------------------------------------------------------------- scans
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive prefix over the threads of a block of NT threads; returns the
// block total through *tot
template <int NT>
__device__ int block_excl_scan(int v, int *sh, int *tot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int base = 0, all = 0;
    for (int k = 0; k < NT / 64; ++k) {
        if (k < w) base += sh[k];
        all += sh[k];
    }
    __syncthreads();
    *tot = all;
    return base + inc - v;
}

// one block of 1024 threads: exclusive scan of up to kSmallScan values,
// 64-bit total to *total
constexpr int kSmallT = 1024;
constexpr int kSmallScan = 1 << 16;
__device__ __forceinline__ void scan_small_body(const int32_t *__restrict__ in, int32_t *__restrict__ out, int n,
                                                int64_t *__restrict__ total);
__global__ __launch_bounds__(kSmallT) void scan_small_kernel(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                             int n, int64_t *__restrict__ total)
{
    scan_small_body(in, out, n, total);
}

// three independent small scans in one launch, one block each
struct Scan3 {
    const int32_t *in[3];
    int32_t *out[3];
    int64_t *total[3];
};
__global__ __launch_bounds__(kSmallT) void scan_small3_kernel(Scan3 a, int n)
{
    scan_small_body(a.in[blockIdx.x], a.out[blockIdx.x], n, a.total[blockIdx.x]);
}

__device__ __forceinline__ void scan_small_body(const int32_t *__restrict__ in, int32_t *__restrict__ out, int n,
                                                int64_t *__restrict__ total)
{
    __shared__ int sh[kSmallT / 64];
    __shared__ long long t64[kSmallT / 64];
    const int per = (n + kSmallT - 1) / kSmallT;
    const int b0 = threadIdx.x * per, b1 = min(n, b0 + per);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += in[b];
    int tot;
    int run = block_excl_scan<kSmallT>(s, sh, &tot);
    for (int b = b0; b < b1; ++b) {
        const int v = in[b];
        out[b] = run;
        run += v;
    }
    // 64-bit total: per-wave sums of the per-thread sums
    long long w64 = s;
    for (int o = 32; o > 0; o >>= 1) w64 += __shfl_down(w64, o, 64);
    if ((threadIdx.x & 63) == 0) t64[threadIdx.x >> 6] = w64;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0;
        for (int k = 0; k < kSmallT / 64; ++k) a += t64[k];
        *total = a;
    }
}

// per block: exclusive scan of its tile, block total to sums[b]
__global__ __launch_bounds__(kScanT) void scan_tile_kernel(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                           int n, int32_t *__restrict__ sums)
{
    __shared__ int sh[kScanT / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
    int v[kScanI], s = 0;
#pragma unroll
    for (int j = 0; j < kScanI; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    int tot;
    int run = block_excl_scan<kScanT>(s, sh, &tot);
#pragma unroll
    for (int j = 0; j < kScanI; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums in place; grand total (64-bit)
// to *total
__global__ __launch_bounds__(kScanT) void scan_sums_kernel(int32_t *__restrict__ sums, int nb, int64_t *__restrict__ total)
{
    __shared__ int sh[kScanT / 64];
    const int per = (nb + kScanT - 1) / kScanT;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    int s = 0;
    long long s64 = 0;
    for (int b = b0; b < b1; ++b) {
        s += sums[b];
        s64 += sums[b];
    }
    int tot;
    int run = block_excl_scan<kScanT>(s, sh, &tot);
    for (int b = b0; b < b1; ++b) {
        const int v = sums[b];
        sums[b] = run;
        run += v;
    }
    // 64-bit total, in case the 32-bit prefix overflowed (checked by the host)
    __shared__ long long t64[kScanT];
    t64[threadIdx.x] = s64;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0;
        for (int k = 0; k < kScanT; ++k) a += t64[k];
        *total = a;
    }
}

__global__ __launch_bounds__(kScanT) void scan_add_kernel(int32_t *__restrict__ out, int n, const int32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
    const int add = sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanI; ++j)
        if (base + j < n) out[base + j] += add;
}

// ---------------------------------------------------------------- small sort
// one workgroup, in place: the order of the stable sort on (key & mask) for
// n <= kSmallSort items, as a bitonic sort of (masked key, position) in LDS;
// keys and values are then gathered by position
constexpr int kSmallSort = 2048;
constexpr int kSmallSortT = 1024;
__global__ __launch_bounds__(kSmallSortT) void small_sort_kernel(uint64_t *__restrict__ k, int32_t *__restrict__ v, int n,
                                                                 uint64_t mask)
{
    __shared__ uint64_t sk[kSmallSort];
    __shared__ uint16_t sp[kSmallSort];
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += kSmallSortT) {
        sk[i] = i < n ? (k[i] & mask) : mask;   // padding sorts last: its position is >= n
        sp[i] = (uint16_t)i;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
        for (int j = size >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += kSmallSortT) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = sk[i], b = sk[l];
                    const uint16_t pa = sp[i], pb = sp[l];
                    const bool gt = a > b || (a == b && pa > pb);
                    if (gt == ((i & size) == 0)) {
                        sk[i] = b;
                        sk[l] = a;
                        sp[i] = pb;
                        sp[l] = pa;
                    }
                }
            }
            __syncthreads();
        }
    constexpr int kPer = kSmallSort / kSmallSortT;
    uint64_t kk[kPer];
    int32_t vv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kSmallSortT;
        if (i < n) {
            kk[q] = k[sp[i]];
            vv[q] = v[sp[i]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kSmallSortT;
        if (i < n) {
            k[i] = kk[q];
            v[i] = vv[q];
        }
    }
}

// ---------------------------------------------------------------- keys
// per block: componentwise min and max, and 1 if any coordinate is not finite
__global__ void bbox_partial_kernel(const double *__restrict__ pos, int64_t n, double *__restrict__ part)
{
    __shared__ double sh[7][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int d = 0; d < 3; ++d) {
            const double x = pos[3 * i + d];
            if (!isfinite(x)) bad = 1.0;
            lo[d] = fmin(lo[d], x);
            hi[d] = fmax(hi[d], x);
        }
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + s]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + s]);
            }
            sh[6][threadIdx.x] = fmax(sh[6][threadIdx.x], sh[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[7 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// one block of 256: the 7 components (3 minima, 3 maxima, the non-finite
// flag) over the nb partial results, strided over the threads, then an LDS
// tree; min and max are exact, so the order does not matter
__global__ __launch_bounds__(256) void bbox_final_kernel(const double *__restrict__ part, int nb,
                                                         double *__restrict__ out)
{
    __shared__ double sh[7][256];
    double v[7];
    for (int k = 0; k < 7; ++k) v[k] = k < 3 ? INFINITY : -INFINITY;
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 7; ++k) v[k] = k < 3 ? fmin(v[k], part[7 * b + k]) : fmax(v[k], part[7 * b + k]);
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 7; ++k)
                sh[k][threadIdx.x] = k < 3 ? fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + w])
                                           : fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 7) out[threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 0) {   // out[7]: the key scale 2^21 / W, W the largest extent (1 if all coincide)
        const double e0 = sh[3][0] - sh[0][0], e1 = sh[4][0] - sh[1][0], e2 = sh[5][0] - sh[2][0];
        const double m12 = e1 < e2 ? e2 : e1;
        double W = e0 < m12 ? m12 : e0;
        if (W == 0.0) W = 1.0;
        out[7] = ldexp(1.0, kMaxLevel) / W;
    }
}

__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// box: the componentwise minima, maxima, the non-finite flag and the key
// scale (bbox_final_kernel); with a non-finite position every key is 0 (the
// host rejects the build at its first read-back)
__global__ void keys_kernel(const double *__restrict__ pos, int n, const double *__restrict__ box,
                            uint64_t *__restrict__ key, int32_t *__restrict__ idx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    idx[i] = i;
    if (box[6] != 0.0) {
        key[i] = 0;
        return;
    }
    const double scale = box[7];
    const int64_t qmax = (int64_t(1) << kMaxLevel) - 1;
    uint64_t q[3];
    for (int d = 0; d < 3; ++d) {
        const double v = __dmul_rn(__dsub_rn(pos[3 * (size_t)i + d], box[d]), scale);
        const int64_t qi = (int64_t)floor(v);
        q[d] = (uint64_t)min(max(qi, (int64_t)0), qmax);
    }
    key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

// ---------------------------------------------------------------- tree
// The levels are built without the host: each level's first cell is kept in
// LevelState::lev, which the kernels read.  Grids are sized by a bound on the
// number of cells of the level (cells past the level's end exit); a level
// whose children would exceed the cell capacity sets `flag` and writes
// nothing, and every later kernel of the batch then does nothing, so the
// host can grow the array and run the batch again.
struct LevelState {
    double box[8];                 // minima, maxima, non-finite flag, key scale
    int32_t flag;                  // 1: cell capacity exceeded, 2: a level above its bound
    int32_t pad;
    int32_t lev[kMaxLevel + 3];    // first cell of every level (lev[l + 1]: end of level l)
};

__global__ void level_init_kernel(LevelState *ls)
{
    if (threadIdx.x < kMaxLevel + 3) ls->lev[threadIdx.x] = threadIdx.x == 1 ? 1 : 0;
    if (threadIdx.x == 0) ls->flag = 0;
}

__global__ void level_flag_clear_kernel(LevelState *ls)
{
    if (threadIdx.x == 0) ls->flag = 0;
}

// eight lanes per cell, lane `dig` finding the end of the run of child
// digit dig (the first index in the cell's range whose digit exceeds dig;
// the keys are sorted, so the runs are consecutive), all eight at once
__global__ __launch_bounds__(256) void tree_split_kernel(const DevCell *__restrict__ cells, const LevelState *ls,
                                                         int level, const uint64_t *__restrict__ key, int ncrit,
                                                         int32_t *__restrict__ nch, int2 *__restrict__ runs)
{
    if (ls->flag) return;
    const int lb = ls->lev[level], le = ls->lev[level + 1];
    if (lb >= le) return;   // an empty level (past the deepest)
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = lb + (g >> 3), dig = g & 7;
    const bool live = c < le;
    const DevCell cell = cells[live ? c : lb];
    const bool split = live && cell.count > ncrit && level < kMaxLevel;
    const int e = cell.first + cell.count;
    int lo = cell.first;
    if (split) {
        const int shift = 3 * (kMaxLevel - level - 1);
        int hi = e;
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if ((int)((key[m] >> shift) & 7) <= dig) lo = m + 1;
            else hi = m;
        }
    }
    // the run of digit dig starts where digit dig - 1 ends (eight lanes of
    // one cell are consecutive lanes of one wave)
    const int prev = __shfl_up(lo, 1, 8);
    const int a = dig == 0 ? cell.first : prev;
    const int nonempty = split && lo > a ? 1 : 0;
    int cntc = nonempty;
    for (int w = 1; w < 8; w <<= 1) cntc += __shfl_xor(cntc, w, 8);
    if (!live) return;
    if (split) runs[(size_t)(c - lb) * 8 + dig] = make_int2(a, lo - a);
    if (dig == 0) nch[c - lb] = split ? cntc : 0;
}

// one block: the children's offsets within the next level, and its end
__global__ __launch_bounds__(kSmallT) void level_scan_kernel(const int32_t *__restrict__ nch, int32_t *__restrict__ off,
                                                             LevelState *ls, int level, int bound, int64_t *tot)
{
    int m = ls->flag ? 0 : ls->lev[level + 1] - ls->lev[level];
    if (m > bound) {   // never expected: the bound is a theorem; read nothing past the buffers
        if (threadIdx.x == 0) ls->flag = 2;
        m = 0;
    }
    scan_small_body(nch, off, m, tot);
    if (threadIdx.x == 0) ls->lev[level + 2] = ls->lev[level + 1] + (int)*tot;
}

__global__ void tree_emit_kernel(DevCell *__restrict__ cells, LevelState *ls, int level, int cap,
                                 const int32_t *__restrict__ nch, const int32_t *__restrict__ off,
                                 const int2 *__restrict__ runs)
{
    if (ls->flag) return;
    const int lb = ls->lev[level], le = ls->lev[level + 1];
    if (ls->lev[level + 2] > cap) {   // the children do not fit: nothing is written
        if (threadIdx.x == 0) ls->flag = 1;
        return;
    }
    const int c = lb + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= le) return;
    const int k = nch[c - lb];
    DevCell cell = cells[c];
    cell.child0 = k ? le + off[c - lb] : -1;
    cell.nchild = k;
    cells[c] = cell;
    int o = cell.child0;
    for (int dig = 0; dig < 8 && k; ++dig) {
        const int2 r = runs[(size_t)(c - lb) * 8 + dig];
        if (r.y == 0) continue;
        DevCell ch{};
        ch.level = cell.level + 1;
        ch.ix = 2 * cell.ix + (dig >> 2);
        ch.iy = 2 * cell.iy + ((dig >> 1) & 1);
        ch.iz = 2 * cell.iz + (dig & 1);
        ch.first = r.x;
        ch.count = r.y;
        ch.parent = c;
        ch.child0 = -1;
        ch.nchild = 0;
        cells[o++] = ch;
    }
}

// ---------------------------------------------------------------- traversal
struct PairAct {
    int m2l, p2p, nkids, mode;   // mode: 0 none, 1 children of A, 2 of B, 3 both
};

__device__ __forceinline__ PairAct pair_action(const DevCell &a, const DevCell &b, double th2)
{
    const int64_t ra = int64_t(1) << (kMaxLevel - a.level), rb = int64_t(1) << (kMaxLevel - b.level);
    const int64_t dx = (2 * (int64_t)b.ix + 1) * rb - (2 * (int64_t)a.ix + 1) * ra;
    const int64_t dy = (2 * (int64_t)b.iy + 1) * rb - (2 * (int64_t)a.iy + 1) * ra;
    const int64_t dz = (2 * (int64_t)b.iz + 1) * rb - (2 * (int64_t)a.iz + 1) * ra;
    const int64_t d2 = dx * dx + dy * dy + dz * dz;
    const double s = (double)(ra + rb);
    const bool leafA = a.nchild == 0, leafB = b.nchild == 0;
    PairAct r{0, 0, 0, 0};
    if (__dmul_rn(s, s) < __dmul_rn(th2, (double)d2)) {
        r.m2l = 1;
    } else if (leafA && leafB) {
        r.p2p = 1;
    } else if (leafB || (!leafA && ra > rb)) {
        r.mode = 1;
        r.nkids = a.nchild;
    } else if (leafA || rb > ra) {
        r.mode = 2;
        r.nkids = b.nchild;
    } else {
        r.mode = 3;
        r.nkids = a.nchild * b.nchild;
    }
    return r;
}

__global__ void trav_count_kernel(const int2 *__restrict__ fr, int nf, const DevCell *__restrict__ cells, double th2,
                                  int32_t *__restrict__ nk, int32_t *__restrict__ m2l, int32_t *__restrict__ p2p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int2 ab = fr[i];
    const PairAct r = pair_action(cells[ab.x], cells[ab.y], th2);
    nk[i] = r.nkids;
    m2l[i] = r.m2l;
    p2p[i] = r.p2p;
}

__global__ void trav_emit_kernel(const int2 *__restrict__ fr, int nf, const DevCell *__restrict__ cells, double th2,
                                 const int32_t *__restrict__ ok, const int32_t *__restrict__ om,
                                 const int32_t *__restrict__ op, int kb, int2 *__restrict__ next,
                                 uint64_t *__restrict__ m2l_key, int64_t m2l_base, uint64_t *__restrict__ p2p_key,
                                 int64_t p2p_base)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int2 ab = fr[i];
    const DevCell a = cells[ab.x], b = cells[ab.y];
    const PairAct r = pair_action(a, b, th2);
    // list entries keyed (target, source) so that one sort gives the CSR
    if (r.m2l) m2l_key[m2l_base + om[i]] = ((uint64_t)ab.y << kb) | (uint64_t)ab.x;
    if (r.p2p) p2p_key[p2p_base + op[i]] = ((uint64_t)ab.y << kb) | (uint64_t)ab.x;
    int o = ok[i];
    if (r.mode == 1) {
        for (int k = 0; k < a.nchild; ++k) next[o++] = make_int2(a.child0 + k, ab.y);
    } else if (r.mode == 2) {
        for (int k = 0; k < b.nchild; ++k) next[o++] = make_int2(ab.x, b.child0 + k);
    } else if (r.mode == 3) {
        for (int ka = 0; ka < a.nchild; ++ka)
            for (int kb2 = 0; kb2 < b.nchild; ++kb2) next[o++] = make_int2(a.child0 + ka, b.child0 + kb2);
    }
}

// keys sorted by target: each wave adds the length of each of its runs of
// one target with one atomic (instead of one per key)
__global__ void list_count_kernel(const uint64_t *__restrict__ key, int64_t m, int kb, int32_t *__restrict__ cnt)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int t = i < m ? (int)(key[i] >> kb) : -1;
    const int prev = __shfl_up(t, 1, 64);
    const bool head = lane == 0 || prev != t;
    const unsigned long long heads = __ballot(head);
    if (head && t >= 0) {
        const unsigned long long later = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
        const int next = later ? __ffsll((long long)later) - 1 : 64;
        atomicAdd(&cnt[t], next - lane);
    }
}

__global__ void list_src_kernel(const uint64_t *__restrict__ key, int64_t m, int kb, int32_t *__restrict__ src)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    src[i] = (int32_t)(key[i] & ((1ull << kb) - 1));
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------- host side
// Scratch memory of one build.  With a context, blocks come first from its
// arena by bumping a pointer (a released arena block is reused only by the
// next build on the same stream, after this one's work); what does not fit
// comes from the stream-ordered allocator, and the arena grows to this
// build's total (up to the context's cache limit) for the next build.
struct Dev {
    hipStream_t s;
    int64_t *pin = nullptr;   // 8 pinned words for read-backs (or none)
    fmm_ctx *ctx = nullptr;
    size_t used = 0, need = 0;
    std::vector<void *> blocks;
    hipError_t err = hipSuccess;
    template <typename T>
    T *alloc(size_t count)
    {
        void *p = nullptr;
        if (err != hipSuccess) return nullptr;
        const size_t b = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
        need += b;
        if (ctx && ctx->arena && used + b <= ctx->arena_cap) {
            p = ctx->arena + used;
            used += b;
            return (T *)p;
        }
        err = hipMallocAsync(&p, b, s);
        if (err != hipSuccess) return nullptr;
        blocks.push_back(p);
        return (T *)p;
    }
    void release(void *p)
    {
        auto it = std::find(blocks.begin(), blocks.end(), p);
        if (it != blocks.end()) {
            hipFreeAsync(p, s);
            blocks.erase(it);
        }
    }
    ~Dev()
    {
        for (void *p : blocks) hipFreeAsync(p, s);
        if (ctx && need > ctx->arena_cap && err == hipSuccess) {
            // twice this build's need (at least 32 MB), so that builds up to
            // twice as large grow it no further
            const size_t want = std::min(std::max(2 * need, (size_t)32 << 20), ctx_cache_limit(ctx));
            if (want > ctx->arena_cap) {
                if (ctx->arena) hipFreeAsync(ctx->arena, s);
                ctx->arena = nullptr;
                ctx->arena_cap = 0;
                void *p = nullptr;
                if (hipMallocAsync(&p, want, s) == hipSuccess) {
                    ctx->arena = (char *)p;
                    ctx->arena_cap = want;
                } else {
                    (void)hipGetLastError();
                }
            }
        }
    }
};

#define GCHK(expr)                              \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// exclusive scan of n int32 values into out (in place allowed); the 64-bit
// total goes to the device word *total.  No host synchronisation.
hipError_t scan_i32(Dev &dv, const int32_t *in, int32_t *out, int n, int64_t *total)
{
    if (n <= kSmallScan) {
        hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(kSmallT), 0, dv.s, in, out, n, total);
        return hipGetLastError();
    }
    const int nb = (int)nblk(n, kScanTile);
    int32_t *sums = dv.alloc<int32_t>(nb);
    GCHK(dv.err);
    hipLaunchKernelGGL(scan_tile_kernel, dim3(nb), dim3(kScanT), 0, dv.s, in, out, n, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanT), 0, dv.s, sums, nb, total);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanT), 0, dv.s, out, n, sums);
    GCHK(hipGetLastError());
    dv.release(sums);
    return hipSuccess;
}

// Read-backs of a few device words through the context's coherent host
// words: one thread copies them with system-scope stores, then stores the
// read-back's sequence number with release order, and the host polls that
// number (about 6 us from the kernel's launch to the words on the host,
// against about 14 us for a copy and a stream wait).  After kSigSpin of
// polling the host waits for the stream instead, which also reports a
// failed kernel.
constexpr int kSigWords = 64;                  // words one read-back carries; the sequence number follows
constexpr double kSigSpinUs = 1000.0;
__global__ void publish_kernel(const int64_t *__restrict__ src, int n, int64_t *host, int64_t seq)
{
    if (threadIdx.x != 0) return;
    for (int i = 0; i < n; ++i) __hip_atomic_store(&host[i], src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host[kSigWords], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// the first k device words (8-byte aligned), read on the host; this waits
// for the stream's work up to them
hipError_t read_words(Dev &dv, const void *dev, int k, void *host)
{
    if (dv.ctx && dv.ctx->sig && k <= kSigWords) {
        fmm_ctx *c = dv.ctx;
        const int64_t seq = ++c->sig_seq;
        hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(64), 0, dv.s, (const int64_t *)dev, k, c->sig_dev, seq);
        GCHK(hipGetLastError());
        const auto t0 = std::chrono::steady_clock::now();
        while (__atomic_load_n(&c->sig[kSigWords], __ATOMIC_ACQUIRE) != seq) {
            if (std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() > kSigSpinUs) {
                GCHK(hipStreamSynchronize(dv.s));
                if (__atomic_load_n(&c->sig[kSigWords], __ATOMIC_ACQUIRE) != seq) return hipErrorUnknown;
                break;
            }
        }
        memcpy(host, c->sig, sizeof(int64_t) * k);
        return hipSuccess;
    }
    void *dst = dv.pin ? (void *)dv.pin : host;
    GCHK(hipMemcpyAsync(dst, dev, sizeof(int64_t) * k, hipMemcpyDeviceToHost, dv.s));
    GCHK(hipStreamSynchronize(dv.s));
    if (dst != host) memcpy(host, dst, sizeof(int64_t) * k);
    return hipSuccess;
}

// the first k (<= 8) device words, read on the host (synchronises the
// stream)
hipError_t read_totals(Dev &dv, const void *dev, int k, void *host)
{
    return read_words(dv, dev, k, host);
}

// stable sort of (key, val) on the low `bits` bits of the key: one workgroup
// for at most kSmallSort items, else the library radix sort (8-bit digits);
// the result ends in k/v (the buffers are swapped as needed)
hipError_t radix_sort(Dev &dv, uint64_t *&k, int32_t *&v, int n, int bits)
{
    if (n <= 1) return hipSuccess;
    if (n <= kSmallSort) {
        const uint64_t mask = bits >= 64 ? ~0ull : (1ull << bits) - 1;
        hipLaunchKernelGGL(small_sort_kernel, dim3(1), dim3(kSmallSortT), 0, dv.s, k, v, n, mask);
        return hipGetLastError();
    }
    size_t tb = 0;
    GCHK(dev_sort_pairs(nullptr, tb, k, nullptr, v, nullptr, n, std::min(bits, 64), dv.s));
    uint64_t *k2 = dv.alloc<uint64_t>(n);
    int32_t *v2 = dv.alloc<int32_t>(n);
    char *tmp = dv.alloc<char>(tb);
    GCHK(dv.err);
    GCHK(dev_sort_pairs(tmp, tb, k, k2, v, v2, n, std::min(bits, 64), dv.s));
    std::swap(k, k2);
    std::swap(v, v2);
    return hipSuccess;
}

int bits_for(int64_t m)
{
    int b = 1;
    while ((int64_t(1) << b) <= m) ++b;
    return b;
}

// CSR (ptr over ncells + 1, src) of the (target << kb | source) keys
// The CSR lists of m (target, source) keys: sorted on the device, then per
// target counts and the sources as int32 (copied to the host with the rest
// of the tree, see csr_finish)
hipError_t csr_launch(Dev &dv, uint64_t *key, int64_t m, int kb, int nc, int32_t **cnt, int32_t **s32)
{
    *cnt = dv.alloc<int32_t>(nc);
    *s32 = dv.alloc<int32_t>(m);
    GCHK(dv.err);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(nc, 256)), dim3(256), 0, dv.s, *cnt, (int64_t)nc);
    if (m == 0) return hipGetLastError();
    int32_t *val = dv.alloc<int32_t>(m);
    GCHK(dv.err);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(m, 256)), dim3(256), 0, dv.s, val, m);
    GCHK(radix_sort(dv, key, val, (int)m, 2 * kb));
    hipLaunchKernelGGL(list_count_kernel, dim3(nblk(m, 256)), dim3(256), 0, dv.s, key, m, kb, *cnt);
    hipLaunchKernelGGL(list_src_kernel, dim3(nblk(m, 256)), dim3(256), 0, dv.s, key, m, kb, *s32);
    return hipGetLastError();
}

void csr_finish(const int32_t *c, const int32_t *s, int64_t m, int nc, std::vector<int64_t> &ptr,
                std::vector<int64_t> &src)
{
    ptr.assign(nc + 1, 0);
    src.resize(m);
    for (int i = 0; i < nc; ++i) ptr[i + 1] = ptr[i] + c[i];
    for (int64_t i = 0; i < m; ++i) src[i] = s[i];
}

// host staging of the device-to-host copies: the context's pinned buffer
// (fast, asynchronous copies), grown on demand, or plain host memory
struct Staging {
    fmm_ctx *ctx;
    std::vector<char> plain;
    char *base = nullptr;
    hipError_t reserve(size_t bytes)
    {
        if (ctx) {
            GCHK(ctx_pinned(ctx, bytes, &base));
        } else {
            plain.resize(bytes);
            base = plain.data();
        }
        return hipSuccess;
    }
};

// ------------------------------------------------------------------ M2L scheduling
// The tiling of build_m2l_tiling (tree_host.cpp) on the device, with the same
// result: targets in (level, octant, same-level signature, list length
// descending, cell) order, 64 to a tile; per tile the sorted distinct pair
// geometries; class ids the ranks in the sorted union; per entry and lane
// the source (or the zero row).  Keys are packed into 64 bits in the order
// of the host comparators; a key that does not fit (or a tile with more
// distinct geometries than its hash table holds) sends the tree back to the
// host code.

constexpr int kTileHashBits = 13;
constexpr int kTileHash = 1 << kTileHashBits;   // open-addressing slots per tile (LDS)
constexpr int kTileMaxU = kTileHash / 2;        // distinct geometries a tile may have here
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int64_t kClsR = 1 << 18;         // offset range of a packed pair geometry

// first probe of a key in the tile table (Fibonacci hashing)
__device__ __forceinline__ int tile_slot(uint64_t k) { return (int)((k * 0x9E3779B97F4A7C15ull) >> (64 - kTileHashBits)); }

// (dl + 32) << 57 | (d0 + R) << 38 | (d1 + R) << 19 | (d2 + R): the order
// of (dl, d0, d1, d2)
__device__ __forceinline__ bool pack_class(const DevCell &A, const DevCell &B, uint64_t &key)
{
    const int la = A.level, lb = B.level, lm = max(la, lb);
    const int64_t d0 = ((2 * (int64_t)B.ix + 1) << (lm - lb)) - ((2 * (int64_t)A.ix + 1) << (lm - la));
    const int64_t d1 = ((2 * (int64_t)B.iy + 1) << (lm - lb)) - ((2 * (int64_t)A.iy + 1) << (lm - la));
    const int64_t d2 = ((2 * (int64_t)B.iz + 1) << (lm - lb)) - ((2 * (int64_t)A.iz + 1) << (lm - la));
    const bool ok = d0 >= -kClsR && d0 < kClsR && d1 >= -kClsR && d1 < kClsR && d2 >= -kClsR && d2 < kClsR;
    key = ((uint64_t)(lb - la + 32) << 57) | ((uint64_t)(d0 + kClsR) << 38) | ((uint64_t)(d1 + kClsR) << 19) |
          (uint64_t)(d2 + kClsR);
    return ok;
}

__device__ __forceinline__ void unpack_class(uint64_t k, int &dl, int64_t &d0, int64_t &d1, int64_t &d2)
{
    const uint64_t m = (1ull << 19) - 1;
    dl = (int)(k >> 57) - 32;
    d0 = (int64_t)((k >> 38) & m) - kClsR;
    d1 = (int64_t)((k >> 19) & m) - kClsR;
    d2 = (int64_t)(k & m) - kClsR;
}

// target keys: level (5 bits) | octant (3) | lo0 hi0 lo1 hi1 lo2 hi2 (7 each,
// + 64) | 8191 - length (13); cells without an M2L list sort last
// one wave per cell: its lanes stride over the list, then reduce; the
// block's targets, shallowest levels and overflow flag go to `info` with one
// atomic each per block
constexpr int kKeyT = 1024;
__global__ __launch_bounds__(kKeyT) void tile_key_kernel(const DevCell *__restrict__ cells, int nc,
                                                         const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
                                                         uint64_t *__restrict__ key, int32_t *__restrict__ val,
                                                         unsigned long long *__restrict__ info)
{
    __shared__ int s_cnt, s_bad, s_tl, s_sl;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_bad = 0;
        s_tl = INT_MAX;
        s_sl = INT_MAX;
    }
    __syncthreads();
    const int c = blockIdx.x * (kKeyT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c < nc) {   // whole waves
        const int e0 = ptr[c], e1 = ptr[c + 1];
        const DevCell B = cells[c];
        int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
        for (int e = e0 + lane; e < e1; e += 64) {
            const DevCell A = cells[src[e]];
            if (A.level != B.level) continue;
            const int o[3] = {A.ix - B.ix, A.iy - B.iy, A.iz - B.iz};
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], o[d]);
                hi[d] = max(hi[d], o[d]);
            }
        }
        for (int d = 0; d < 3; ++d)
            for (int w = 32; w > 0; w >>= 1) {
                lo[d] = min(lo[d], __shfl_xor(lo[d], w, 64));
                hi[d] = max(hi[d], __shfl_xor(hi[d], w, 64));
            }
        if (lane == 0) {
            val[c] = c;
            if (e1 == e0) {
                key[c] = kEmptyKey;
            } else {
                if (lo[0] > hi[0])   // no same-level source
                    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = 0;
                const int len = e1 - e0;
                bool ok = len <= 8191 && B.level < 32;
                uint64_t k = ((uint64_t)B.level << 58) |
                             ((uint64_t)(((B.ix & 1) << 2) | ((B.iy & 1) << 1) | (B.iz & 1)) << 55);
                for (int d = 0; d < 3; ++d) {
                    ok = ok && lo[d] >= -64 && lo[d] < 64 && hi[d] >= -64 && hi[d] < 64;
                    k |= (uint64_t)((lo[d] + 64) & 127) << (48 - 14 * d);
                    k |= (uint64_t)((hi[d] + 64) & 127) << (41 - 14 * d);
                }
                k |= (uint64_t)(8191 - min(len, 8191));
                key[c] = k;
                atomicAdd(&s_cnt, 1);
                if (!ok) s_bad = 1;
                atomicMin(&s_tl, B.level);
                atomicMin(&s_sl, (int)cells[src[e0]].level);   // lists sorted by source, cells level-major
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt > 0) {
        atomicAdd(&info[0], (unsigned long long)s_cnt);        // targets
        if (s_bad) atomicOr(&info[1], 1ull);                   // a key field overflows
        atomicMin(&info[4], (unsigned long long)s_tl);         // shallowest target
        atomicMin(&info[5], (unsigned long long)s_sl);         // shallowest source
    }
}

__global__ void tile_info_init_kernel(unsigned long long *info)
{
    if (threadIdx.x < 6) info[threadIdx.x] = threadIdx.x < 4 ? 0ull : ~0ull;
}

// one workgroup per tile: the tile's distinct pair geometries in an LDS hash
// table.  EMIT = false: their number; EMIT = true: sorted into U, written
// at the tile's entry offset, and every (entry, lane) source placed in usrc
constexpr int kClsT = 1024;   // threads per tile: kClsT / 64 per lane
template <bool EMIT>
__global__ __launch_bounds__(kClsT) void tile_classes_kernel(const DevCell *__restrict__ cells,
                                                           const int32_t *__restrict__ tcell,
                                                           const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ src,
                                                           unsigned long long *__restrict__ info,
                                                           int32_t *__restrict__ tcnt, const int32_t *__restrict__ uoff,
                                                           uint64_t *__restrict__ ukey, int32_t *__restrict__ usrc)
{
    __shared__ uint64_t tab[kTileHash];
    __shared__ uint64_t U[EMIT ? kTileMaxU : 1];
    __shared__ int16_t pos[EMIT ? kTileHash : 1];
    __shared__ int cnt, bad;
    const int tile = blockIdx.x, ntg = (int)info[0];
    if (tile * kTileW >= ntg) {   // the grid is sized by all cells
        if (!EMIT && threadIdx.x == 0) tcnt[tile] = 0;
        return;
    }
    for (int h = threadIdx.x; h < kTileHash; h += blockDim.x) tab[h] = kEmptyKey;
    if (threadIdx.x == 0) {
        cnt = 0;
        bad = 0;
    }
    __syncthreads();
    // kClsT / 64 threads per lane, each taking every (kClsT / 64)-th entry of the lane's list
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int slot = tile * kTileW + lane;
    const int B = slot < ntg ? tcell[slot] : -1;
    const int e0 = B >= 0 ? ptr[B] : 0, e1 = B >= 0 ? ptr[B + 1] : 0;
    const DevCell cb = cells[B >= 0 ? B : 0];
    auto probe = [&](uint64_t k) {   // the slot of k, inserting it
        int h = tile_slot(k);
        for (int n = 0; n < kTileHash; ++n) {
            const uint64_t old = atomicCAS((unsigned long long *)&tab[h], (unsigned long long)kEmptyKey,
                                           (unsigned long long)k);
            if (old == kEmptyKey) {
                if (atomicAdd(&cnt, 1) >= kTileMaxU) bad = 1;
                return h;
            }
            if (old == k) return h;
            h = (h + 1) & (kTileHash - 1);
        }
        bad = 1;
        return -1;
    };
    for (int e = e0 + part; e < e1; e += kClsT / 64) {
        uint64_t k;
        if (!pack_class(cells[src[e]], cb, k)) bad = 1;
        probe(k);
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) {
            atomicOr(&info[1], 2ull);
            if (!EMIT) tcnt[tile] = 0;
        }
        return;
    }
    const int nu = cnt;
    if constexpr (!EMIT) {
        if (threadIdx.x == 0) tcnt[tile] = nu;
        return;
    } else {
        // compact, then a bitonic sort of the next power of two
        __shared__ int fill;
        if (threadIdx.x == 0) fill = 0;
        __syncthreads();
        for (int h = threadIdx.x; h < kTileHash; h += blockDim.x)
            if (tab[h] != kEmptyKey) U[atomicAdd(&fill, 1)] = tab[h];
        int np = 1;
        while (np < nu) np <<= 1;
        __syncthreads();
        for (int j = nu + threadIdx.x; j < np; j += blockDim.x) U[j] = kEmptyKey;
        __syncthreads();
        for (int k = 2; k <= np; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < np; i += blockDim.x) {
                    const int l = i ^ j;
                    if (l > i) {
                        const uint64_t a = U[i], b = U[l];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            U[i] = b;
                            U[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        // sorted position of every slot's key
        const int base = uoff[tile];
        for (int j = threadIdx.x; j < nu; j += blockDim.x) {
            const uint64_t k = U[j];
            int h = tile_slot(k);
            while (tab[h] != k) h = (h + 1) & (kTileHash - 1);
            pos[h] = (int16_t)j;
            ukey[base + j] = k;
        }
        __syncthreads();
        for (int e = e0 + part; e < e1; e += kClsT / 64) {
            const int A = src[e];
            uint64_t k;
            pack_class(cells[A], cb, k);
            int h = tile_slot(k);
            while (tab[h] != k) h = (h + 1) & (kTileHash - 1);
            usrc[(size_t)(base + pos[h]) * kTileW + lane] = A;
        }
    }
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// cell -> tile slot, for the targets of the tiles
__global__ void tile_slots_kernel(const int32_t *__restrict__ tcell, int ntg, int32_t *__restrict__ cell_slot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntg) cell_slot[tcell[i]] = i;
}

// after the sort of all tiles' geometries: first-of-a-kind flags
__global__ void class_flags_kernel(const uint64_t *__restrict__ k, int n, int32_t *__restrict__ f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}

// class id of every tile entry (the rank of its geometry) and the class
// geometry ((z_B - z_A) / r_B, r_A / r_B), as the host computes it
__global__ void class_ids_kernel(const uint64_t *__restrict__ k, const int32_t *__restrict__ idx,
                                 const int32_t *__restrict__ rank_excl, const int32_t *__restrict__ f, int n,
                                 int32_t *__restrict__ ucls, double *__restrict__ geom)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = rank_excl[i] + f[i] - 1;
    ucls[idx[i]] = r;
    if (f[i]) {
        int dl;
        int64_t d0, d1, d2;
        unpack_class(k[i], dl, d0, d1, d2);
        const double unit = ldexp(1.0, min(0, dl));
        geom[4 * r] = (double)d0 * unit;
        geom[4 * r + 1] = (double)d1 * unit;
        geom[4 * r + 2] = (double)d2 * unit;
        geom[4 * r + 3] = ldexp(1.0, dl);
    }
}

__global__ void last_of_scan_kernel(int32_t *ptr, int n, const int64_t *total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ptr[n] = (int32_t)*total;
}

// per cell: its particle count times the particles of its P2P sources (the
// direct-sum work of a target leaf), one wave per cell; integers, exact
constexpr int kCostT = 256;
__global__ __launch_bounds__(kCostT) void p2p_cost_kernel(const DevCell *__restrict__ cells, int nc,
                                                          const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ src, int64_t *__restrict__ cost)
{
    const int c = blockIdx.x * (kCostT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= nc) return;   // whole waves
    int64_t s = 0;
    for (int e = ptr[c] + lane; e < ptr[c + 1]; e += 64) s += cells[src[e]].count;
    for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
    if (lane == 0) cost[c] = s * (int64_t)cells[c].count;
}

__global__ void root_cell_kernel(DevCell *c, int32_t n)
{
    if (threadIdx.x == 0) {
        DevCell r{};
        r.level = 0;
        r.first = 0;
        r.count = n;
        r.parent = -1;
        r.child0 = -1;
        c[0] = r;
    }
}

__global__ void iota_i32_kernel(int32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

// Device M2L tiling, first part: the M2L CSR offsets, the target order, the
// per-tile geometry counts and their offsets, then one wait for the sizes.
// On success with dt.done the kept buffers hold the per-entry tables and
// *tcell / *uoff / *nclasses_dev the parts the host copies back with the
// tree (finish_tiling).  `done` false: fall back to the host code.
struct TileState {
    int32_t *tcell = nullptr, *uoff = nullptr;
    double *geom = nullptr;
    unsigned long long *info = nullptr;   // ntargets, overflow flags, nentries, nclasses, top levels
    int ntg = 0, ntiles = 0;
    int64_t nentries = 0;
};

hipError_t launch_tiling(Dev &dv, const DevCell *cells, int nc, const int32_t *cnt, const int32_t *src, int64_t nsrc,
                         DevKeep &dt, TileState &ts)
{
    dt.done = false;
    hipStream_t s = dv.s;
    int32_t *ptr = dv.alloc<int32_t>((size_t)nc + 1);
    uint64_t *key = dv.alloc<uint64_t>(nc);
    int32_t *val = dv.alloc<int32_t>(nc);
    ts.info = dv.alloc<unsigned long long>(6);
    GCHK(dv.err);
    hipLaunchKernelGGL(tile_info_init_kernel, dim3(1), dim3(64), 0, s, ts.info);
    int64_t *itot = (int64_t *)(ts.info + 2);
    GCHK(scan_i32(dv, cnt, ptr, nc, itot));
    hipLaunchKernelGGL(last_of_scan_kernel, dim3(1), dim3(64), 0, s, ptr, nc, itot);
    hipLaunchKernelGGL(tile_key_kernel, dim3(nblk(nc, kKeyT / 64)), dim3(kKeyT), 0, s, cells, nc, ptr, src, key, val,
                       ts.info);
    GCHK(hipGetLastError());
    GCHK(radix_sort(dv, key, val, nc, 64));
    const int ntmax = (int)nblk(nc, kTileW);
    int32_t *tcnt = dv.alloc<int32_t>(ntmax);
    ts.uoff = dv.alloc<int32_t>((size_t)ntmax + 1);
    GCHK(dv.err);
    hipLaunchKernelGGL(tile_classes_kernel<false>, dim3(ntmax), dim3(kClsT), 0, s, cells, val, ptr, src, ts.info, tcnt,
                       (const int32_t *)nullptr, (uint64_t *)nullptr, (int32_t *)nullptr);
    GCHK(hipGetLastError());
    GCHK(scan_i32(dv, tcnt, ts.uoff, ntmax, itot));
    hipLaunchKernelGGL(last_of_scan_kernel, dim3(1), dim3(64), 0, s, ts.uoff, ntmax, itot);
    GCHK(hipGetLastError());
    unsigned long long hi[4];
    GCHK(read_totals(dv, ts.info, 4, hi));
    if (hi[1] != 0 || hi[2] * (unsigned long long)kTileW > (unsigned long long)INT32_MAX) return hipSuccess;
    ts.ntg = (int)hi[0];
    ts.ntiles = (ts.ntg + kTileW - 1) / kTileW;
    ts.nentries = (int64_t)hi[2];
    ts.tcell = val;
    const int64_t ne = ts.nentries;
    // the tables the tree keeps, and its M2L lists (they stay on the device)
    GCHK(dt.keep((void **)&dt.m2l_ptr, sizeof(int32_t) * ((size_t)nc + 1)));
    GCHK(dt.keep((void **)&dt.m2l_src, sizeof(int32_t) * (size_t)std::max<int64_t>(1, nsrc)));
    GCHK(hipMemcpyAsync(dt.m2l_ptr, ptr, sizeof(int32_t) * ((size_t)nc + 1), hipMemcpyDeviceToDevice, s));
    if (nsrc) GCHK(hipMemcpyAsync(dt.m2l_src, src, sizeof(int32_t) * nsrc, hipMemcpyDeviceToDevice, s));
    GCHK(dt.keep((void **)&dt.ucls, sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne)));
    GCHK(dt.keep((void **)&dt.usrc, sizeof(int32_t) * (size_t)std::max<int64_t>(1, ne * kTileW)));
    GCHK(dt.keep((void **)&dt.cell_slot, sizeof(int32_t) * (size_t)nc));
    hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(nc, 256)), dim3(256), 0, s, dt.cell_slot, (int64_t)nc, -1);
    hipLaunchKernelGGL(tile_slots_kernel, dim3(nblk(ts.ntg, 256)), dim3(256), 0, s, val, ts.ntg, dt.cell_slot);
    GCHK(hipGetLastError());
    if (ne == 0) {
        hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t *)(ts.info + 3), (int64_t)2);
        dt.done = true;
        return hipGetLastError();
    }
    // zero rows where a lane lacks the class, then every tile's sorted
    // geometries and (entry, lane) sources
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)std::min<int64_t>(4096, nblk(ne * kTileW, 256))), dim3(256), 0, s,
                       dt.usrc, ne * kTileW, (int32_t)nc);
    uint64_t *ukey = dv.alloc<uint64_t>(ne);
    int32_t *uidx = dv.alloc<int32_t>(ne), *flag = dv.alloc<int32_t>(ne), *rank = dv.alloc<int32_t>(ne);
    ts.geom = dv.alloc<double>(4 * (size_t)ne);
    GCHK(dv.err);
    hipLaunchKernelGGL(tile_classes_kernel<true>, dim3(ts.ntiles), dim3(kClsT), 0, s, cells, val, ptr, src, ts.info,
                       (int32_t *)nullptr, (const int32_t *)ts.uoff, ukey, dt.usrc);
    hipLaunchKernelGGL(iota_i32_kernel, dim3(nblk(ne, 256)), dim3(256), 0, s, uidx, (int)ne);
    GCHK(hipGetLastError());
    // class ids: ranks in the sorted union of all tiles' geometries
    GCHK(radix_sort(dv, ukey, uidx, (int)ne, 64));
    hipLaunchKernelGGL(class_flags_kernel, dim3(nblk(ne, 256)), dim3(256), 0, s, ukey, (int)ne, flag);
    GCHK(hipGetLastError());
    GCHK(scan_i32(dv, flag, rank, (int)ne, (int64_t *)(ts.info + 3)));
    hipLaunchKernelGGL(class_ids_kernel, dim3(nblk(ne, 256)), dim3(256), 0, s, ukey, uidx, rank, flag, (int)ne, dt.ucls,
                       ts.geom);
    GCHK(hipGetLastError());
    dt.done = true;
    return hipSuccess;
}

}  // namespace

hipError_t ctx_arena_reserve(fmm_ctx *ctx, size_t bytes)
{
    bytes = std::min(bytes, ctx_cache_limit(ctx));
    if (ctx->arena_cap >= bytes) return hipSuccess;
    if (ctx->arena) (void)hipFreeAsync(ctx->arena, ctx->stream);
    ctx->arena = nullptr;
    ctx->arena_cap = 0;
    void *p = nullptr;
    const hipError_t e = hipMallocAsync(&p, bytes, ctx->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    ctx->arena = (char *)p;
    ctx->arena_cap = bytes;
    return hipStreamSynchronize(ctx->stream);
}

// Builds the canonical tree (and, when theta > 0, the interaction lists) of
// the n device positions on stream s, and returns it in host form.  ctx (may
// be null): its pinned staging buffer and, while profiling, the wall-clock
// phases.
hipError_t gpu_build_tree(const double *pos, int64_t n, int ncrit, double theta, bool lists, hipStream_t s,
                          HostTree &t, fmm_ctx *ctx, DevKeep *dt)
{
    t = HostTree();
    t.n = n;
    Dev dv{s};
    if (ctx) {
        if (!ctx->pin_small) GCHK(hipHostMalloc((void **)&ctx->pin_small, 4096, hipHostMallocDefault));
        if (!ctx->sig) {
            GCHK(hipHostMalloc((void **)&ctx->sig, sizeof(int64_t) * (kSigWords + 1),
                               hipHostMallocCoherent | hipHostMallocMapped));
            ctx->sig[kSigWords] = ctx->sig_seq;
            const hipError_t e = hipHostGetDevicePointer((void **)&ctx->sig_dev, ctx->sig, 0);
            if (e != hipSuccess) {
                (void)hipHostFree(ctx->sig);
                ctx->sig = nullptr;
                return e;
            }
        }
        dv.pin = ctx->pin_small;
        dv.ctx = ctx;
    }
    // wall-clock phases for the context's profile (the device work of a
    // phase is counted where the host next waits for it)
    auto t_last = std::chrono::steady_clock::now();
    auto mark = [&](const char *nm) {
        if (!ctx || !ctx->profile) return;
        const auto now = std::chrono::steady_clock::now();
        ctx->prof.push_back(ProfEntry{nm, nullptr, nullptr, std::chrono::duration<double, std::milli>(now - t_last).count()});
        t_last = now;
    };
    // root box (read back with the first batch of levels)
    LevelState *ls = dv.alloc<LevelState>(1);
    const int nbb = (int)std::min<int64_t>(1024, nblk(n, 256));
    double *part = dv.alloc<double>(7 * (size_t)nbb);
    GCHK(dv.err);
    hipLaunchKernelGGL(level_init_kernel, dim3(1), dim3(64), 0, s, ls);
    hipLaunchKernelGGL(bbox_partial_kernel, dim3(nbb), dim3(256), 0, s, pos, n, part);
    hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(256), 0, s, part, nbb, ls->box);
    GCHK(hipGetLastError());

    // keys and stable sort
    uint64_t *key = dv.alloc<uint64_t>(n);
    int32_t *idx = dv.alloc<int32_t>(n);
    GCHK(dv.err);
    hipLaunchKernelGGL(keys_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, pos, (int)n, (const double *)ls->box, key, idx);
    GCHK(hipGetLastError());
    GCHK(radix_sort(dv, key, idx, (int)n, 3 * kMaxLevel));
    mark("host:tree_box");

    int64_t *dtot = dv.alloc<int64_t>(4);
    GCHK(dv.err);
    // Cells level by level, in batches of levels between read-backs.  A
    // level holds at most 8^l cells, and at most 8 children of each cell
    // that splits, a split cell holds more than ncrit particles and the
    // cells of one level are disjoint, and at most n non-empty cells: that
    // bound sizes the grids and the per-level buffers (shared by the levels).
    // The cell array starts at 10 n / ncrit cells (at most 4 n): a uniform
    // tree just past a split of a whole level holds about 9 n / ncrit, and a
    // tree that needs more grows the array and runs its batch again.
    size_t cap = std::max<size_t>(64, (size_t)std::min<int64_t>(10 * n / std::max(1, ncrit), 4 * n) + 64);
    DevCell *cells = dv.alloc<DevCell>(cap);
    const int64_t split_max = n / ((int64_t)ncrit + 1);
    const int64_t umax = std::max<int64_t>(1, std::min<int64_t>(n, 8 * split_max));
    int32_t *nch = dv.alloc<int32_t>(umax), *off = dv.alloc<int32_t>(umax);
    int2 *runs = dv.alloc<int2>((size_t)umax * 8);
    GCHK(dv.err);
    hipLaunchKernelGGL(root_cell_kernel, dim3(1), dim3(64), 0, s, cells, (int32_t)n);
    GCHK(hipGetLastError());
    std::vector<int64_t> ub(kMaxLevel + 2, 1);   // ub[l]: bound on the cells of level l
    for (int l = 0; l + 1 <= kMaxLevel + 1; ++l) ub[l + 1] = std::min<int64_t>(umax, std::min<int64_t>(8 * ub[l], n));
    LevelState hs;
    int l0 = 0, nlev = -1;
    bool first = true;
    // the first batch: the levels of a uniform tree of n particles (each
    // split leaves about an eighth of a cell's particles per child) and the
    // one below it, whose cells do not split; deeper trees take batches of
    // four more (a level past the tree's end launches kernels that only
    // find nothing to do)
    int first_batch = 2;
    for (double m = (double)n / std::max(1, ncrit); m > 1.0 && first_batch < kMaxLevel + 1; m /= 8.0) ++first_batch;
    while (nlev < 0) {
        const int l1 = std::min(l0 + (first ? first_batch : 4), kMaxLevel + 1);
        for (int l = l0; l < l1; ++l) {
            const int64_t m = ub[l];
            hipLaunchKernelGGL(tree_split_kernel, dim3(nblk(m * 8, 256)), dim3(256), 0, s, cells, (const LevelState *)ls,
                               l, key, ncrit, nch, runs);
            hipLaunchKernelGGL(level_scan_kernel, dim3(1), dim3(kSmallT), 0, s, nch, off, ls, l, (int)m, dtot);
            hipLaunchKernelGGL(tree_emit_kernel, dim3(nblk(m, 256)), dim3(256), 0, s, cells, ls, l, (int)cap, nch, off,
                               runs);
            GCHK(hipGetLastError());
        }
        static_assert(sizeof(LevelState) % 8 == 0 && sizeof(LevelState) <= 8 * kSigWords,
                      "the level state is read back as whole words");
        GCHK(read_words(dv, ls, (int)(sizeof(LevelState) / 8), &hs));
        if (first) {
            if (hs.box[6] != 0.0) return hipErrorInvalidValue;   // a position is not finite
            double W = std::max(hs.box[3] - hs.box[0], std::max(hs.box[4] - hs.box[1], hs.box[5] - hs.box[2]));
            if (W == 0.0) W = 1.0;
            for (int d = 0; d < 3; ++d) t.lo[d] = hs.box[d];
            t.W = W;
            t.h = std::ldexp(W, -22);
            first = false;
        }
        if (hs.flag == 2) return hipErrorUnknown;   // a level above its bound (not expected)
        if (hs.flag == 1) {
            // grow the cell array past the largest level end seen and run the batch again
            size_t need = cap;
            for (int l = l0; l < l1; ++l) need = std::max(need, (size_t)hs.lev[l + 2]);
            const size_t ncap = std::max(2 * cap, need + need / 4);
            if (ncap > (size_t)INT32_MAX) return hipErrorOutOfMemory;
            DevCell *c2 = dv.alloc<DevCell>(ncap);
            GCHK(dv.err);
            GCHK(hipMemcpyAsync(c2, cells, sizeof(DevCell) * cap, hipMemcpyDeviceToDevice, s));
            dv.release(cells);
            cells = c2;
            cap = ncap;
            hipLaunchKernelGGL(level_flag_clear_kernel, dim3(1), dim3(64), 0, s, ls);
            GCHK(hipGetLastError());
            continue;
        }
        // the first level of the batch without children is the deepest
        for (int l = l0; l < l1 && nlev < 0; ++l)
            if (hs.lev[l + 2] == hs.lev[l + 1]) nlev = l + 1;
        l0 = l1;
    }
    t.level_ptr.assign(hs.lev, hs.lev + nlev + 1);
    const int le = hs.lev[nlev];
    const int nc = le;
    mark("host:tree_sort_levels");

    // interaction lists: breadth-first over cell pairs
    int32_t *m2l_cnt = nullptr, *m2l_s32 = nullptr, *p2p_cnt = nullptr, *p2p_s32 = nullptr;
    int64_t n_m2l = 0, n_p2p = 0;
    if (lists) {
        const double th2 = theta * theta;
        const int kb = bits_for(nc);
        // The list keys of all steps go to one buffer per list at running
        // offsets.  Capacities from the usual list lengths at this theta
        // (about 170 M2L entries per cell and 30 P2P entries per leaf at
        // theta 0.5, growing as theta^-2.6 and theta^-3), with a margin; a
        // step that would not fit grows its buffer first (a copy of what
        // the earlier steps wrote).
        const double rth = 0.5 / theta;
        auto capped = [](double v) { return (int64_t)std::min(v, (double)INT32_MAX); };
        int64_t mcap = capped(1.3 * 170.0 * std::pow(rth, 2.6) * nc + 4096);
        int64_t pcap = capped(1.3 * 30.0 * rth * rth * rth * nc + 4096);
        int64_t moff = 0, poff = 0;
        uint64_t *mall = dv.alloc<uint64_t>(mcap), *pall = dv.alloc<uint64_t>(pcap);
        auto ensure = [&](uint64_t *&buf, int64_t &cap, int64_t off, int64_t need) -> hipError_t {
            if (off + need <= cap) return hipSuccess;
            const int64_t ncap = std::max(2 * cap, off + need + (off + need) / 4);
            uint64_t *b2 = dv.alloc<uint64_t>(ncap);
            GCHK(dv.err);
            if (off) GCHK(hipMemcpyAsync(b2, buf, sizeof(uint64_t) * off, hipMemcpyDeviceToDevice, s));
            dv.release(buf);
            buf = b2;
            cap = ncap;
            return hipSuccess;
        };
        int2 *fr = dv.alloc<int2>(1);
        GCHK(dv.err);
        hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t *)fr, (int64_t)2);   // (root, root)
        GCHK(hipGetLastError());
        int64_t nf = 1;
        while (nf > 0) {
            if (nf > INT32_MAX) return hipErrorOutOfMemory;
            int32_t *nk = dv.alloc<int32_t>(nf), *fm = dv.alloc<int32_t>(nf), *fp = dv.alloc<int32_t>(nf);
            GCHK(dv.err);
            hipLaunchKernelGGL(trav_count_kernel, dim3(nblk(nf, 256)), dim3(256), 0, s, fr, (int)nf, cells, th2, nk, fm, fp);
            GCHK(hipGetLastError());
            if (nf <= kSmallScan) {   // the three scans in one launch
                Scan3 a{{nk, fm, fp}, {nk, fm, fp}, {dtot, dtot + 1, dtot + 2}};
                hipLaunchKernelGGL(scan_small3_kernel, dim3(3), dim3(kSmallT), 0, s, a, (int)nf);
                GCHK(hipGetLastError());
            } else {
                GCHK(scan_i32(dv, nk, nk, (int)nf, dtot));
                GCHK(scan_i32(dv, fm, fm, (int)nf, dtot + 1));
                GCHK(scan_i32(dv, fp, fp, (int)nf, dtot + 2));
            }
            int64_t tt[3];
            GCHK(read_totals(dv, dtot, 3, tt));
            const int64_t tk = tt[0], tm = tt[1], tp = tt[2];
            if (tk > INT32_MAX) return hipErrorOutOfMemory;
            int2 *next = dv.alloc<int2>(tk);
            GCHK(dv.err);
            if (moff + tm > INT32_MAX || poff + tp > INT32_MAX) return hipErrorOutOfMemory;
            GCHK(ensure(mall, mcap, moff, tm));
            GCHK(ensure(pall, pcap, poff, tp));
            hipLaunchKernelGGL(trav_emit_kernel, dim3(nblk(nf, 256)), dim3(256), 0, s, fr, (int)nf, cells, th2, nk, fm, fp,
                               kb, next, mall, moff, pall, poff);
            GCHK(hipGetLastError());
            dv.release(nk);
            dv.release(fm);
            dv.release(fp);
            dv.release(fr);
            fr = next;
            nf = tk;
            moff += tm;
            poff += tp;
        }
        mark("host:tree_traverse");
        // sort by (target, source)
        const int64_t mm = moff, pm = poff;
        GCHK(csr_launch(dv, mall, mm, kb, nc, &m2l_cnt, &m2l_s32));
        GCHK(csr_launch(dv, pall, pm, kb, nc, &p2p_cnt, &p2p_s32));
        n_m2l = mm;
        n_p2p = pm;
    }
    // the P2P sources stay on the device with the tree; the host gets the
    // per-cell costs that order the near-field dispatch
    int64_t *p2p_cost = nullptr;
    const bool keep_p2p = lists && dt;
    if (keep_p2p) {
        int32_t *pptr = dv.alloc<int32_t>((size_t)nc + 1);
        p2p_cost = dv.alloc<int64_t>(nc);
        GCHK(dv.err);
        GCHK(scan_i32(dv, p2p_cnt, pptr, nc, dtot + 3));
        hipLaunchKernelGGL(last_of_scan_kernel, dim3(1), dim3(64), 0, s, pptr, nc, (const int64_t *)(dtot + 3));
        hipLaunchKernelGGL(p2p_cost_kernel, dim3(nblk(nc, kCostT / 64)), dim3(kCostT), 0, s, (const DevCell *)cells, nc,
                           (const int32_t *)pptr, (const int32_t *)p2p_s32, p2p_cost);
        GCHK(hipGetLastError());
        GCHK(dt->keep((void **)&dt->p2p_src, sizeof(int32_t) * (size_t)std::max<int64_t>(1, n_p2p)));
        if (n_p2p)
            GCHK(hipMemcpyAsync(dt->p2p_src, p2p_s32, sizeof(int32_t) * n_p2p, hipMemcpyDeviceToDevice, s));
    }
    mark("host:tree_lists");
    TileState ts;
    if (lists && dt && dt->tiling && n_m2l >= dt->min_pairs) {
        GCHK(launch_tiling(dv, cells, nc, m2l_cnt, m2l_s32, n_m2l, *dt, ts));
        mark("host:tree_tiling");
    }
    const bool dtile = lists && dt && dt->tiling && dt->done;
    if (dt) {
        // cells, order and keys stay on the device for the tree
        GCHK(dt->keep((void **)&dt->cells, sizeof(DevCell) * nc));
        GCHK(dt->keep((void **)&dt->perm, sizeof(int32_t) * n));
        GCHK(dt->keep((void **)&dt->key, sizeof(uint64_t) * n));
        GCHK(hipMemcpyAsync(dt->cells, cells, sizeof(DevCell) * nc, hipMemcpyDeviceToDevice, s));
        GCHK(hipMemcpyAsync(dt->perm, idx, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        GCHK(hipMemcpyAsync(dt->key, key, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    }
    const int64_t n_host = dt ? 0 : n;   // particles whose order and key the host copies

    // host copies of the cells, the order, the keys and the lists, in one
    // staging buffer and one wait
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_cells = 0, o_perm = o_cells + al(sizeof(DevCell) * nc),
                 o_key = o_perm + al(sizeof(int32_t) * n_host), o_mc = o_key + al(sizeof(uint64_t) * n_host),
                 o_ms = o_mc + al(sizeof(int32_t) * nc),
                 o_pc = o_ms + al(sizeof(int32_t) * (dtile ? 0 : n_m2l)), o_ps = o_pc + al(sizeof(int32_t) * nc),
                 o_pk = o_ps + al(sizeof(int32_t) * (keep_p2p ? 0 : n_p2p)),
                 o_tc = o_pk + al(sizeof(int64_t) * (keep_p2p ? nc : 0)), o_tu = o_tc + al(sizeof(int32_t) * ts.ntg),
                 o_ti = o_tu + al(sizeof(int32_t) * (ts.ntiles + 1)), o_end = o_ti + al(sizeof(int64_t) * 4);
    Staging st{ctx};
    GCHK(st.reserve(o_end));
    GCHK(hipMemcpyAsync(st.base + o_cells, cells, sizeof(DevCell) * nc, hipMemcpyDeviceToHost, s));
    if (n_host) {
        GCHK(hipMemcpyAsync(st.base + o_perm, idx, sizeof(int32_t) * n_host, hipMemcpyDeviceToHost, s));
        GCHK(hipMemcpyAsync(st.base + o_key, key, sizeof(uint64_t) * n_host, hipMemcpyDeviceToHost, s));
    }
    if (lists) {
        // with the schedule made on the device the host needs no M2L list
        if (!dtile) {
            GCHK(hipMemcpyAsync(st.base + o_mc, m2l_cnt, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
            if (n_m2l)
                GCHK(hipMemcpyAsync(st.base + o_ms, m2l_s32, sizeof(int32_t) * n_m2l, hipMemcpyDeviceToHost, s));
        }
        GCHK(hipMemcpyAsync(st.base + o_pc, p2p_cnt, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
        if (keep_p2p) GCHK(hipMemcpyAsync(st.base + o_pk, p2p_cost, sizeof(int64_t) * nc, hipMemcpyDeviceToHost, s));
        else if (n_p2p)
            GCHK(hipMemcpyAsync(st.base + o_ps, p2p_s32, sizeof(int32_t) * n_p2p, hipMemcpyDeviceToHost, s));
    }
    if (dtile) {
        if (ts.ntg) GCHK(hipMemcpyAsync(st.base + o_tc, ts.tcell, sizeof(int32_t) * ts.ntg, hipMemcpyDeviceToHost, s));
        GCHK(hipMemcpyAsync(st.base + o_tu, ts.uoff, sizeof(int32_t) * (ts.ntiles + 1), hipMemcpyDeviceToHost, s));
        GCHK(hipMemcpyAsync(st.base + o_ti, ts.info + 2, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
    }
    GCHK(hipStreamSynchronize(s));
    mark("host:tree_copy");
    if (lists) {
        if (!dtile)
            csr_finish((const int32_t *)(st.base + o_mc), (const int32_t *)(st.base + o_ms), n_m2l, nc, t.m2l_ptr,
                       t.m2l_src);
        if (keep_p2p) {
            const int32_t *c = (const int32_t *)(st.base + o_pc);
            t.p2p_ptr.assign(nc + 1, 0);
            for (int i = 0; i < nc; ++i) t.p2p_ptr[i + 1] = t.p2p_ptr[i] + c[i];
            t.p2p_src.clear();
            const int64_t *k = (const int64_t *)(st.base + o_pk);
            t.p2p_cost.assign(k, k + nc);
        } else {
            csr_finish((const int32_t *)(st.base + o_pc), (const int32_t *)(st.base + o_ps), n_p2p, nc, t.p2p_ptr,
                       t.p2p_src);
        }
    }
    const DevCell *hc = (const DevCell *)(st.base + o_cells);
    const int32_t *perm = (const int32_t *)(st.base + o_perm);
    t.key.assign((const uint64_t *)(st.base + o_key), (const uint64_t *)(st.base + o_key) + n_host);
    t.perm.assign(perm, perm + n_host);
    t.level.resize(nc);
    t.ix.resize(3 * (size_t)nc);
    t.first.resize(nc);
    t.count.resize(nc);
    t.parent.resize(nc);
    t.child0.resize(nc);
    t.nchild.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const DevCell &d = hc[c];
        t.level[c] = d.level;
        t.ix[3 * c] = d.ix;
        t.ix[3 * c + 1] = d.iy;
        t.ix[3 * c + 2] = d.iz;
        t.first[c] = d.first;
        t.count[c] = d.count;
        t.parent[c] = d.parent;
        t.child0[c] = d.child0;
        t.nchild[c] = d.nchild;
    }
    if (dtile) {
        M2LTiling &tl = *dt->tl;
        tl = M2LTiling();
        tl.on_device = true;
        tl.ntiles = ts.ntiles;
        tl.nentries = ts.nentries;
        const int64_t *ti = (const int64_t *)(st.base + o_ti);
        tl.nclasses = ts.nentries ? (int)ti[1] : 0;
        dt->tgt_top = ts.ntg ? (int)ti[2] : -1;
        dt->src_top = ts.ntg ? (int)ti[3] : -1;
        tl.pairs = n_m2l;
        tl.tile_cell.assign((size_t)ts.ntiles * kTileW, -1);
        std::copy((const int32_t *)(st.base + o_tc), (const int32_t *)(st.base + o_tc) + ts.ntg, tl.tile_cell.begin());
        tl.tile_uoff.assign((const int32_t *)(st.base + o_tu), (const int32_t *)(st.base + o_tu) + ts.ntiles + 1);
        GCHK(dt->keep((void **)&dt->cls_geom, sizeof(double) * 4 * (size_t)std::max(1, tl.nclasses)));
        if (tl.nclasses)
            GCHK(hipMemcpyAsync(dt->cls_geom, ts.geom, sizeof(double) * 4 * tl.nclasses, hipMemcpyDeviceToDevice, s));
    } else if (dt) {
        dt->done = false;
    }
    mark("host:tree_copyback");
    return hipSuccess;
}
