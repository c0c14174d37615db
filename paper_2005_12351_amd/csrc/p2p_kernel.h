// Near-field kernels of libfmm.so (the direct sums over the P2P lists,
// Section 3.2 of Pepper & Fangohr, arXiv 2005.12351), shared by the two
// translation units that instantiate them per source-order mask
// (p2p_lo.hip: masks 1-7, p2p_oct.hip: masks with octupoles, 8-15), which
// build in parallel.
#pragma once
#include <type_traits>

#include "fmm_internal.h"
#include "pair_kernels.h"

// ------------------------------------------------------------------ P2P
// Direct interaction over the near-field lists (Section 3.2).  One workgroup
// of 256 threads per target leaf (heaviest leaves first).  The sources of the
// leaf's list are staged in LDS in chunks, in list order; the threads form a
// (target, slice) grid with floor(256 / targets) slices, each slice taking a
// contiguous share of every chunk, so nearly all lanes work for any leaf size.
// The slices' sums are added per target in a fixed order (deterministic).
// MIXED: positions relative to the target leaf centre in units of its radius
// (FP32 stays well scaled for any box), FP32 pair terms summed per chunk and
// added into Kahan-compensated accumulators, scaled back in FP64.  FP64:
// physical positions, reciprocal square root refined to full precision.
__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

struct P2PArgs {
    const int32_t *leaves, *ptr, *src, *order;
    const DevCell *cells;
    const float *m32;       // m32_width(mask) per particle
    const double *xs;       // SoA
    const double *m64;
    double *near;           // 4 per particle (phi, E)
    double *near_g;         // 6 per particle (field gradient), gradient kernels only
    int n;
    double h, lo[3];
};

// One staged source: its position relative to the target leaf (FP64, in
// units of the leaf radius) and its FP32 moment blocks in one record, so the
// pair loop walks all of them with a single LDS address.
template <int NV>
struct alignas(16) P2PStaged {
    double x, y, z, unused;
    float4 m[NV];
};

constexpr int kPT = 256;        // threads per target leaf
constexpr int kPList = 256;     // list entries per window
constexpr int kPChunk32 = 512;  // staged sources per chunk (FP32)
constexpr int kPChunk64 = 256;  // staged sources per chunk (FP64)

// exclusive prefix over the 256 threads of the block; block total to *tot
__device__ __forceinline__ int p2p_block_scan(int v, int *sh, int *tot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int base = 0, all = 0;
    for (int k = 0; k < kPT / 64; ++k) {
        if (k < w) base += sh[k];
        all += sh[k];
    }
    __syncthreads();
    *tot = all;
    return base + inc - v;
}

// Window of up to kPList list entries: start offset of each entry's particles
// within the window, first particle, source geometry relative to the target
// leaf (centre difference in units of r_b, and r_A / r_b), and the window
// offset of the target leaf's own entry (-1 if absent).  The slots of
// wstart past the window's entries hold INT_MAX (see p2p_entry).  Returns
// the number of staged sources of the window.
static __device__ int p2p_window(const P2PArgs &a, const DevCell &cb, int b, int w0, int nw, int *wstart, int *wfirst,
                          float4 *wgeo, int *wself, int *sh)
{
    const int q = threadIdx.x;
    int cnt = 0;
    if (q < nw) {
        const int A = a.src[w0 + q];
        const DevCell c = a.cells[A];
        cnt = c.count;
        wfirst[q] = c.first;
        const double rho = ldexp(1.0, cb.level - c.level);
        wgeo[q] = make_float4((float)((double)(2 * c.ix + 1) * rho - (double)(2 * cb.ix + 1)),
                              (float)((double)(2 * c.iy + 1) * rho - (double)(2 * cb.iy + 1)),
                              (float)((double)(2 * c.iz + 1) * rho - (double)(2 * cb.iz + 1)), (float)rho);
        if (A == b) *wself = -2 - q;   // marks the entry; replaced by its start below
    }
    int tot;
    const int st = p2p_block_scan(cnt, sh, &tot);
    static_assert(kPT == kPList, "one thread per window slot");
    wstart[q] = q < nw ? st : INT_MAX;
    __syncthreads();
    if (q < nw && *wself == -2 - q) *wself = st;
    __syncthreads();
    return tot;
}

// entry of window source j: the last q with wstart[q] <= j.  Steps of
// powers of two from the largest below nw: the index stays below twice that
// step, so within the kPList slots, and the slots past the window hold
// INT_MAX, so no bound test is needed; the step count is the same for the
// whole wave (a scalar loop)
__device__ __forceinline__ int p2p_entry(const int *wstart, int nw, int j)
{
    int q = 0;
    for (int step = nw > 1 ? 1 << (31 - __clz(nw - 1)) : 0; step > 0; step >>= 1)
        if (wstart[q + step] <= j) q += step;
    return q;
}

// the pair terms of one source of several orders: each order's terms go to
// its own sums (the orders scale differently with the leaf radius); mv is the
// particle's staged FP32 block (m32_width)
template <int MASK, int NV>
__device__ __forceinline__ void p2p_pair_mixed(float rx, float ry, float rz, float inv, const float4 (&mv)[NV],
                                               float (&bp)[4], float (&bx)[4], float (&by)[4], float (&bz)[4])
{
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (MASK & 1) p2p_pair_f32<0>(rx, ry, rz, inv, mv[0], z4, bp[0], bx[0], by[0], bz[0]);
    if constexpr (MASK & 2)
        p2p_pair_f32<1>(rx, ry, rz, inv, make_float4(mv[0].y, mv[0].z, mv[0].w, 0.f), z4, bp[1], bx[1], by[1], bz[1]);
    if constexpr (MASK & 4) p2p_pair_f32<2>(rx, ry, rz, inv, mv[1], mv[2], bp[2], bx[2], by[2], bz[2]);
    if constexpr (MASK & 8) p2p_pair_oct_f32(rx, ry, rz, inv, mv[3], mv[4], mv[5], mv[6], bp[3], bx[3], by[3], bz[3]);
}

template <int MASK, int NV>
__device__ __forceinline__ void p2p_pair_grad_mixed(float rx, float ry, float rz, float inv, const float4 (&mv)[NV],
                                                    float (&g)[6][4])
{
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float t[6];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!(MASK & (1 << k))) continue;
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = g[c][k];
        if constexpr (MASK & 1)
            if (k == 0) p2p_pair_grad_f32<0>(rx, ry, rz, inv, mv[0], z4, t);
        if constexpr (MASK & 2)
            if (k == 1) p2p_pair_grad_f32<1>(rx, ry, rz, inv, make_float4(mv[0].y, mv[0].z, mv[0].w, 0.f), z4, t);
        if constexpr (MASK & 4)
            if (k == 2) p2p_pair_grad_f32<2>(rx, ry, rz, inv, mv[1], mv[2], t);
        if constexpr (MASK & 8)
            if (k == 3) p2p_pair_grad_oct_f32(rx, ry, rz, inv, mv[3], mv[4], mv[5], mv[6], t);
#pragma unroll
        for (int c = 0; c < 6; ++c) g[c][k] = t[c];
    }
}

// GRAD: the six field-gradient components instead of phi and E (sums of
// order k scaled by r_b^-(k+3)), written to near_g.  The launch bound asks
// for five resident workgroups per CU, which fits the dipole kernel in 82
// VGPRs without spills (114 unbounded).
template <int MASK, bool GRAD>
__global__ __launch_bounds__(kPT, 5) void p2p_f32_kernel(P2PArgs a)
{
    constexpr int NO = GRAD ? 6 : 4;                 // output components
    constexpr bool ONE = mask_single(MASK);
    constexpr int S = mask_min_order(MASK);
    // float4 of moments per staged source (the parts the pair terms read) and
    // per particle in the sorted FP32 moments
    constexpr int NV = ONE ? (S == 3 ? 4 : (S == 2 ? 2 : 1)) : ((MASK & 8) ? 7 : 3);
    constexpr int MW = m32_width(MASK) / 4;
    // sources per chunk: half as many for the wide octupole blocks
    constexpr int CH = NV > 3 ? kPChunk32 / 2 : kPChunk32;
    // the staging area doubles as the reduction buffer at the end of a pass
    // (8 KB less LDS per workgroup, one more workgroup per CU)
    __shared__ P2PStaged<NV> sst[CH];
    static_assert(NO * kPT * sizeof(double) <= sizeof(P2PStaged<NV>) * CH, "reduction buffer exceeds the staging area");
    double (*const red)[kPT] = reinterpret_cast<double (*)[kPT]>(sst);
    __shared__ int wstart[kPList], wfirst[kPList];
    __shared__ float4 wgeo[kPList];
    __shared__ int sh[kPT / 64];
    __shared__ int wself;
    const int tid = threadIdx.x;
    const int lk = a.order[blockIdx.x];
    const int b = a.leaves[lk];
    const DevCell cb = a.cells[b];
    const double rb = ldexp(1.0, kMaxLevel - cb.level) * a.h;
    const double irb = 1.0 / rb;
    // physical scale of the order-k sums: potential r_b^-(k+1), field r_b^-(k+2)
    double sphi[4], sfld[4];
    sphi[0] = irb;
    sphi[1] = irb * irb;
    sphi[2] = sphi[1] * irb;
    sphi[3] = sphi[2] * irb;
    sfld[0] = sphi[1];
    sfld[1] = sphi[2];
    sfld[2] = sphi[3];
    sfld[3] = sphi[3] * irb;
    // scale of output component c of the order-k sums
    auto scale = [&](int c, int k) { return GRAD ? sfld[k] * irb : (c == 0 ? sphi[k] : sfld[k]); };
    double zb[3];
    {
        const double r = ldexp(1.0, kMaxLevel - cb.level);
        zb[0] = a.lo[0] + (double)(2 * cb.ix + 1) * r * a.h;
        zb[1] = a.lo[1] + (double)(2 * cb.iy + 1) * r * a.h;
        zb[2] = a.lo[2] + (double)(2 * cb.iz + 1) * r * a.h;
    }
    const size_t n = a.n;
    const int e0 = a.ptr[lk], e1 = a.ptr[lk + 1];
    const float4 *m4 = reinterpret_cast<const float4 *>(a.m32);
    for (int tg0 = 0; tg0 < cb.count; tg0 += kPT) {
        const int cs = min(kPT, cb.count - tg0);
        const int ns = kPT / cs;                 // slices
        const int t = tid % cs, sl = tid / cs;
        const bool act = sl < ns;
        const int i = cb.first + tg0 + t;
        // positions relative to the target leaf centre in units of its radius,
        // FP64: the pair separation is formed before rounding to FP32, so
        // close pairs keep their relative accuracy
        const double tx = (a.xs[i] - zb[0]) * irb, ty = (a.xs[n + i] - zb[1]) * irb,
                     tz = (a.xs[2 * n + i] - zb[2]) * irb;
        // Kahan-compensated sums per output component and source order
        float ks[NO][4], kc[NO][4];
#pragma unroll
        for (int c = 0; c < NO; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) ks[c][k] = kc[c][k] = 0.f;
        for (int w0 = e0; w0 < e1; w0 += kPList) {
            const int nw = min(kPList, e1 - w0);
            __syncthreads();
            if (tid == 0) wself = -1;
            __syncthreads();
            const int nsw = p2p_window(a, cb, b, w0, nw, wstart, wfirst, wgeo, &wself, sh);
            // chunks are a multiple of the slice count long, and the last one
            // is padded with zero sources far away (their terms are exactly
            // zero), so every slice takes the same number of sources and the
            // pair loop runs on a counter common to the whole workgroup
            // The slices of one wave read records per * 48 bytes apart (for
            // dipoles); with per a multiple of 8 slices two apart hit the same
            // LDS banks, so per is kept off those multiples (one more padding
            // source per slice where needed, within the chunk).
            // (per is the same for the whole workgroup; read through the first
            // lane so that the compiler keeps the pair loop's counter scalar)
            const int pmax = CH / ns - ((CH / ns > 1 && (CH / ns) % 8 == 0) ? 1 : 0);
            const int cstep = pmax * ns;
            for (int c0 = 0; c0 < nsw; c0 += cstep) {
                const int nc = min(cstep, nsw - c0);
                const int per0 = (nc + ns - 1) / ns;   // sources per slice
                const int per = __builtin_amdgcn_readfirstlane(per0 + ((per0 % 8 == 0 && per0 < pmax) ? 1 : 0));
                __syncthreads();
                for (int j = tid; j < per * ns; j += kPT) {
                    if (j < nc) {
                        const int q = p2p_entry(wstart, nw, c0 + j);
                        const size_t pj = (size_t)wfirst[q] + (c0 + j - wstart[q]);
                        sst[j].x = (a.xs[pj] - zb[0]) * irb;
                        sst[j].y = (a.xs[n + pj] - zb[1]) * irb;
                        sst[j].z = (a.xs[2 * n + pj] - zb[2]) * irb;
#pragma unroll
                        for (int v = 0; v < NV; ++v) sst[j].m[v] = m4[MW * pj + v];
                    } else {
                        sst[j].x = sst[j].y = sst[j].z = 1.0e4;
#pragma unroll
                        for (int v = 0; v < NV; ++v) sst[j].m[v] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
                __syncthreads();
                if (act) {
                    const int ja = sl * per;
                    // the target itself, if it is staged in this chunk; only a
                    // chunk holding part of the target leaf's own entry needs
                    // the per-pair test (the same for the whole workgroup)
                    const int jself = wself >= 0 ? wself + tg0 + t - c0 : -1;
                    const bool own = wself >= 0 && wself < c0 + nc && wself + cb.count > c0;
                    float bs[NO][4];
#pragma unroll
                    for (int c = 0; c < NO; ++c)
#pragma unroll
                        for (int k = 0; k < 4; ++k) bs[c][k] = 0.f;
                    auto pairs = [&](auto check) {
                    for (int jj = 0; jj < per; ++jj) {
                        const int j = ja + jj;
                        const float rx = (float)(tx - sst[j].x), ry = (float)(ty - sst[j].y), rz = (float)(tz - sst[j].z);
                        const float r2 = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, rz * rz));
                        const float inv = (decltype(check)::value && j == jself) ? 0.f : __builtin_amdgcn_rsqf(r2);
                        float4 mv[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) mv[v] = sst[j].m[v];
                        if constexpr (GRAD) {
                            if constexpr (ONE) {
                                float t6[6];
#pragma unroll
                                for (int c = 0; c < 6; ++c) t6[c] = bs[c][S];
                                if constexpr (S == 3) p2p_pair_grad_oct_f32(rx, ry, rz, inv, mv[0], mv[1], mv[2], mv[3], t6);
                                else p2p_pair_grad_f32<S>(rx, ry, rz, inv, mv[0], mv[NV > 1 ? 1 : 0], t6);
#pragma unroll
                                for (int c = 0; c < 6; ++c) bs[c][S] = t6[c];
                            } else {
                                p2p_pair_grad_mixed<MASK, NV>(rx, ry, rz, inv, mv, bs);
                            }
                        } else if constexpr (ONE) {
                            if constexpr (S == 3)
                                p2p_pair_oct_f32(rx, ry, rz, inv, mv[0], mv[1], mv[2], mv[3], bs[0][3], bs[1][3], bs[2][3],
                                                 bs[3][3]);
                            else p2p_pair_f32<S>(rx, ry, rz, inv, mv[0], mv[NV > 1 ? 1 : 0], bs[0][S], bs[1][S], bs[2][S],
                                                 bs[3][S]);
                        } else {
                            p2p_pair_mixed<MASK, NV>(rx, ry, rz, inv, mv, bs[0], bs[1], bs[2], bs[3]);
                        }
                    }
                    };
                    if (own) pairs(std::true_type{});
                    else pairs(std::false_type{});
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (!(MASK & (1 << k))) continue;
#pragma unroll
                        for (int c = 0; c < NO; ++c) kahan_add(ks[c][k], kc[c][k], bs[c][k]);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NO; ++c) {
            double q = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!(MASK & (1 << k))) continue;
                q += ((double)ks[c][k] - (double)kc[c][k]) * scale(c, k);
            }
            red[c][tid] = act ? q : 0.0;
        }
        __syncthreads();
        if (tid < cs) {
            double v[NO];
#pragma unroll
            for (int c = 0; c < NO; ++c) v[c] = 0.0;
            for (int k = 0; k < ns; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) v[c] += red[c][tid + k * cs];
            double *o = GRAD ? a.near_g + 6 * (size_t)i : a.near + 4 * (size_t)i;
#pragma unroll
            for (int c = 0; c < NO; ++c) o[c] = v[c];
        }
    }
}

// (five resident workgroups per CU, as the FP32 kernel)
template <int MASK, bool GRAD>
__global__ __launch_bounds__(kPT, 5) void p2p_f64_kernel(P2PArgs a)
{
    constexpr int W = mask_width(MASK);
    constexpr int NO = GRAD ? 6 : 4;
    __shared__ double sx[kPChunk64], sy[kPChunk64], sz[kPChunk64], sm[W][kPChunk64];
    __shared__ int wstart[kPList], wfirst[kPList];
    __shared__ float4 wgeo[kPList];
    __shared__ double red[NO][kPT];
    __shared__ int sh[kPT / 64];
    __shared__ int wself;
    const int tid = threadIdx.x;
    const int lk = a.order[blockIdx.x];
    const int b = a.leaves[lk];
    const DevCell cb = a.cells[b];
    const size_t n = a.n;
    const int e0 = a.ptr[lk], e1 = a.ptr[lk + 1];
    // position of the padding sources: 10^4 leaf radii beyond the leaf
    // centre (finite; with zero moments their terms are exactly zero)
    double far[3];
    {
        const double r = ldexp(1.0, kMaxLevel - cb.level) * a.h;
        far[0] = a.lo[0] + (double)(2 * cb.ix + 1) * r + 1.0e4 * r;
        far[1] = a.lo[1] + (double)(2 * cb.iy + 1) * r + 1.0e4 * r;
        far[2] = a.lo[2] + (double)(2 * cb.iz + 1) * r + 1.0e4 * r;
    }
    for (int tg0 = 0; tg0 < cb.count; tg0 += kPT) {
        const int cs = min(kPT, cb.count - tg0);
        const int ns = kPT / cs;
        const int t = tid % cs, sl = tid / cs;
        const bool act = sl < ns;
        const int i = cb.first + tg0 + t;
        const double xi = a.xs[i], yi = a.xs[n + i], zi = a.xs[2 * n + i];
        double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int w0 = e0; w0 < e1; w0 += kPList) {
            const int nw = min(kPList, e1 - w0);
            __syncthreads();
            if (tid == 0) wself = -1;
            __syncthreads();
            const int nsw = p2p_window(a, cb, b, w0, nw, wstart, wfirst, wgeo, &wself, sh);
            // as in the FP32 kernel: chunks a multiple of the slice count long,
            // the last padded with zero sources 10^4 leaf radii away, so all
            // slices take the same number of sources
            const int cstep = (kPChunk64 / ns) * ns;
            for (int c0 = 0; c0 < nsw; c0 += cstep) {
                const int nc = min(cstep, nsw - c0);
                const int per = (nc + ns - 1) / ns;
                __syncthreads();
                for (int j = tid; j < per * ns; j += kPT) {
                    if (j < nc) {
                        const int q = p2p_entry(wstart, nw, c0 + j);
                        const size_t pj = (size_t)wfirst[q] + (c0 + j - wstart[q]);
                        sx[j] = a.xs[pj];
                        sy[j] = a.xs[n + pj];
                        sz[j] = a.xs[2 * n + pj];
#pragma unroll
                        for (int c = 0; c < W; ++c) sm[c][j] = a.m64[pj * W + c];
                    } else {
                        sx[j] = far[0];
                        sy[j] = far[1];
                        sz[j] = far[2];
#pragma unroll
                        for (int c = 0; c < W; ++c) sm[c][j] = 0.0;
                    }
                }
                __syncthreads();
                if (act) {
                    const int ja = sl * per;
                    const int jself = wself >= 0 ? wself + tg0 + t - c0 : -1;
                    // only a chunk holding part of the target leaf's own entry
                    // needs the self test (the same for the whole workgroup)
                    const bool own = wself >= 0 && wself < c0 + nc && wself + cb.count > c0;
                    auto pairs = [&](auto check) {
                    for (int jj = 0; jj < per; ++jj) {
                        const int j = ja + jj;
                        if (decltype(check)::value && j == jself) continue;
                        const double rx = xi - sx[j], ry = yi - sy[j], rz = zi - sz[j];
                        double m[W];
#pragma unroll
                        for (int c = 0; c < W; ++c) m[c] = sm[c][j];
                        // a source of several orders adds each order's terms
                        if constexpr (GRAD) {
                            if constexpr (MASK & 1) p2p_pair_grad_f64<0>(rx, ry, rz, m, g);
                            if constexpr (MASK & 2) p2p_pair_grad_f64<1>(rx, ry, rz, m + (MASK & 1), g);
                            if constexpr (MASK & 4) p2p_pair_grad_f64<2>(rx, ry, rz, m + mask_width(MASK & 3), g);
                            if constexpr (MASK & 8) p2p_pair_grad_oct_f64(rx, ry, rz, m + mask_width(MASK & 7), g);
                        } else {
                            if constexpr (MASK & 1) p2p_pair_f64<0>(rx, ry, rz, m, ph, ex, ey, ez);
                            if constexpr (MASK & 2) p2p_pair_f64<1>(rx, ry, rz, m + (MASK & 1), ph, ex, ey, ez);
                            if constexpr (MASK & 4) p2p_pair_f64<2>(rx, ry, rz, m + mask_width(MASK & 3), ph, ex, ey, ez);
                            if constexpr (MASK & 8) p2p_pair_oct_f64(rx, ry, rz, m + mask_width(MASK & 7), ph, ex, ey, ez);
                        }
                    }
                    };
                    if (own) pairs(std::true_type{});
                    else pairs(std::false_type{});
                }
            }
        }
        __syncthreads();
        const double mine[4] = {ph, ex, ey, ez};
#pragma unroll
        for (int c = 0; c < NO; ++c) red[c][tid] = act ? (GRAD ? g[c] : mine[c % 4]) : 0.0;
        __syncthreads();
        if (tid < cs) {
            double v[NO];
#pragma unroll
            for (int c = 0; c < NO; ++c) v[c] = 0.0;
            for (int k = 0; k < ns; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) v[c] += red[c][tid + k * cs];
            double *o = GRAD ? a.near_g + 6 * (size_t)i : a.near + 4 * (size_t)i;
#pragma unroll
            for (int c = 0; c < NO; ++c) o[c] = v[c];
        }
    }
}


// launches the P2P kernel of mask M in the precision and variant asked for
template <int M>
inline void p2p_launch_mask(bool f32, bool grad, unsigned nblocks, hipStream_t s, const P2PArgs &a)
{
    const dim3 g(nblocks), bl(kPT);
    if (f32 && grad) hipLaunchKernelGGL((p2p_f32_kernel<M, true>), g, bl, 0, s, a);
    else if (f32) hipLaunchKernelGGL((p2p_f32_kernel<M, false>), g, bl, 0, s, a);
    else if (grad) hipLaunchKernelGGL((p2p_f64_kernel<M, true>), g, bl, 0, s, a);
    else hipLaunchKernelGGL((p2p_f64_kernel<M, false>), g, bl, 0, s, a);
}

// per translation unit: false when the mask is not one of its own
bool p2p_dispatch_lo(int mask, bool f32, bool grad, unsigned nblocks, hipStream_t s, const P2PArgs &a);
bool p2p_dispatch_oct(int mask, bool f32, bool grad, unsigned nblocks, hipStream_t s, const P2PArgs &a);
