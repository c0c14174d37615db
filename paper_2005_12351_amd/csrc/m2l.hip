// M2L support kernels of libfmm.so (Pepper & Fangohr, arXiv 2005.12351,
// Eq. 7-8): the derivative tensor of every translation class, the launch of
// the generated contraction kernels, and the FP64 combination of their
// partial rows into the local expansions.
#include <cmath>

#include "fmm_internal.h"

static __constant__ MITable k_mi = make_mi();

// ------------------------------------------------------------------ D table
// Derivatives D_k = d^k (1/r) at every M2L class geometry, |k| <= p, by the
// Hermite-type recursion on R^(j)_n = d^n f^(j)(u), f(u) = (2u)^-1/2,
// u = r^2/2:  R^(j)_0 = (-1)^j (2j-1)!! r^-(2j+1),
//             R^(j)_{m+e_d} = x_d R^(j+1)_m + m_d R^(j+1)_{m-e_d},
// and D_k = R^(0)_k.  FP64; an FP32 copy feeds the mixed-precision M2L.
// Also writes the scale row rho^k, k = 0..p.
__global__ __launch_bounds__(64) void dtable_kernel(int p, int nd, int scw, const double *__restrict__ geom,
                                                    double *__restrict__ D64, float *__restrict__ D32,
                                                    double *__restrict__ S64, float *__restrict__ S32)
{
    __shared__ double Rall[1820];   // all R^(j) blocks: sum_j nterms(p - j) = C(p+4,4) <= 1820 for p <= 12
    const int c = blockIdx.x;
    const double x[3] = {geom[4 * c], geom[4 * c + 1], geom[4 * c + 2]};
    const double rho = geom[4 * c + 3];
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    // offsets of the R^(j) blocks
    auto off = [&](int j) {
        int o = 0;
        for (int q = 0; q < j; ++q) o += nterms(p - q);
        return o;
    };
    if ((int)threadIdx.x <= p) {
        const int j = threadIdx.x;
        double v = 1.0 / sqrt(r2);
        const double ir2 = 1.0 / r2;
        for (int q = 1; q <= j; ++q) v *= -(2.0 * q - 1.0) * ir2;
        Rall[off(j)] = v;
    }
    __syncthreads();
    for (int t = 1; t <= p; ++t) {
        const int per = (t + 1) * (t + 2) / 2;
        const int items = per * (p - t + 1);
        for (int it = threadIdx.x; it < items; it += blockDim.x) {
            const int j = it / per;
            const MultiIndex nn = k_mi.v[nterms(t - 1) + it % per];
            int m[3] = {nn.x, nn.y, nn.z};
            const int d = nn.x > 0 ? 0 : (nn.y > 0 ? 1 : 2);
            m[d] -= 1;
            const double *Rn = Rall + off(j + 1);
            double v = x[d] * Rn[mindex(m[0], m[1], m[2])];
            if (m[d] > 0) {
                int q[3] = {m[0], m[1], m[2]};
                q[d] -= 1;
                v = fma((double)m[d], Rn[mindex(q[0], q[1], q[2])], v);
            }
            Rall[off(j) + mindex(nn.x, nn.y, nn.z)] = v;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
        const double v = k < nterms(p) ? Rall[k] : 0.0;
        D64[(size_t)c * nd + k] = v;
        D32[(size_t)c * nd + k] = (float)v;
    }
    for (int k = threadIdx.x; k < scw; k += blockDim.x) {
        const double v = k <= p ? ldexp(1.0, ilogb(rho) * k) : 0.0;   // rho is a power of two
        S64[(size_t)c * scw + k] = v;
        S32[(size_t)c * scw + k] = (float)v;
    }
}

hipError_t launch_dtable(fmm_tree *t, hipStream_t s)
{
    if (t->tiling.nclasses == 0) return hipSuccess;
    M2LVariant v;
    m2l_lookup(t->p, t->order, true, false, &v);   // nd is the same in both bases
    const int scw = (t->p + 1 + 3) / 4 * 4;
    hipLaunchKernelGGL(dtable_kernel, dim3(t->tiling.nclasses), dim3(64), 0, s, t->p, v.nd, scw, t->d_cls_geom,
                       t->d_D64, t->d_D32, t->d_sc64, t->d_sc32);
    return hipGetLastError();
}

// ------------------------------------------------------------------ M2L
hipError_t launch_m2l(fmm_tree *t, hipStream_t s)
{
    const M2LWork &wk = t->m2lwork;
    if (wk.work.empty()) return hipSuccess;
    const bool f32 = t->prec == FMM_PREC_MIXED, harm = t->basis == FMM_M2L_HARMONIC;
    M2LVariant v;
    if (!m2l_lookup(t->p, t->order, f32, harm, &v, t->mfma)) return hipErrorInvalidValue;
    M2LArgs a;
    a.work = t->d_work;
    a.ucls = t->d_ucls;
    a.usrc = t->d_usrc;
    a.D = f32 ? (const void *)t->d_D32 : (const void *)t->d_D64;
    a.sc = f32 ? (const void *)t->d_sc32 : (const void *)t->d_sc64;
    a.M = harm ? (const void *)t->d_Mh : (f32 ? (const void *)t->d_M32 : (const void *)t->d_M64);
    a.part = t->d_part;
    a.wave_ptr = t->d_wave_ptr;
    a.zero = 0;
    return v.launch(a, wk.nwaves, s);
}

// L~ of every cell (FP64): the sum, in chunk order, of the partial rows of the
// cell's tile slot (each output block of a tile has its own chunks), or zero
// for a cell without M2L sources; so the locals need no separate clearing.
// The loads of eight chunks are issued before their fixed-order sum.
// Harmonic basis: the rows hold the components with n_z <= 1; another
// component (a, b, 2j + r) is (-1)^j sum_i C(j,i) of the summed components
// (a + 2i, b + 2(j - i), r), the identity the locals inherit from D (their
// truncation |m| <= p - |n| is the same for every component of one order).
struct BlockBounds {
    int lo[17];
    int nb;
};

template <typename T>
__device__ __forceinline__ double sum_partials(int n, int tile, int lane, int nlp, const BlockBounds &bb,
                                               const int32_t *__restrict__ chunk0,
                                               const int32_t *__restrict__ nchunk, const T *__restrict__ part)
{
    int b = 0;
    while (b + 1 < bb.nb && n >= bb.lo[b + 1]) ++b;
    const int c0 = chunk0[tile * bb.nb + b], nc = nchunk[tile * bb.nb + b];
    const T *p = part + ((size_t)c0 * kTileW + lane) * nlp + n;
    const size_t stride = (size_t)kTileW * nlp;
    double acc = 0.0;
    int k = 0;
    for (; k + 8 <= nc; k += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = p[(size_t)(k + q) * stride];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += (double)v[q];
    }
    for (; k < nc; ++k) acc += (double)p[(size_t)k * stride];
    return acc;
}

template <typename T>
__global__ void m2l_combine_kernel(int ncells, int nl, int nlp, BlockBounds bb, const int32_t *__restrict__ cell_slot,
                                   const int32_t *__restrict__ chunk0, const int32_t *__restrict__ nchunk,
                                   const T *__restrict__ part, double *__restrict__ L)
{
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)ncells * nl) return;
    const int cell = (int)(id / nl), n = (int)(id % nl);
    const int slot = cell_slot[cell];
    double acc = 0.0;
    if (slot >= 0) acc = sum_partials(n, slot / kTileW, slot % kTileW, nlp, bb, chunk0, nchunk, part);
    L[(size_t)cell * nl + n] = acc;
}

// Harmonic basis, kHarmCells cells per workgroup: the summed components with
// n_z <= 1 go to LDS, then every component of the cells' rows is written
// (full rows, nl per cell) or, when the locals are kept reduced (nl == 0),
// just those components (nlh per cell).
constexpr int kHarmCells = 4;
template <typename T>
__global__ __launch_bounds__(256) void m2l_combine_h_kernel(int ncells, int nl, int nlh, int nlp, BlockBounds bb,
                                                            const int32_t *__restrict__ cell_slot,
                                                            const int32_t *__restrict__ chunk0,
                                                            const int32_t *__restrict__ nchunk,
                                                            const T *__restrict__ part, double *__restrict__ L)
{
    __shared__ double red[kHarmCells][hterms(FMM_P_MAX)];
    const int c0 = blockIdx.x * kHarmCells;
    for (int it = threadIdx.x; it < kHarmCells * nlh; it += blockDim.x) {
        const int cc = it / nlh, h = it % nlh, cell = c0 + cc;
        double v = 0.0;
        const int slot = cell < ncells ? cell_slot[cell] : -1;
        if (slot >= 0) v = sum_partials(h, slot / kTileW, slot % kTileW, nlp, bb, chunk0, nchunk, part);
        red[cc][h] = v;
        if (nl == 0 && cell < ncells) L[(size_t)cell * nlh + h] = v;
    }
    if (nl == 0) return;
    __syncthreads();
    for (int it = threadIdx.x; it < kHarmCells * nl; it += blockDim.x) {
        const int cc = it / nl, n = it % nl, cell = c0 + cc;
        if (cell >= ncells) break;
        const MultiIndex nn = k_mi.v[n];
        const int j = nn.z / 2, r = nn.z & 1;
        double acc = 0.0, c = 1.0;   // c = C(j, i)
        for (int i = 0; i <= j; ++i) {
            acc = fma(c, red[cc][hindex(nn.x + 2 * i, nn.y + 2 * (j - i), r)], acc);
            c = c * (j - i) / (i + 1);
        }
        L[(size_t)cell * nl + n] = (j & 1) ? -acc : acc;
    }
}

hipError_t launch_m2l_combine(fmm_tree *t, hipStream_t s)
{
    const int nl = nterms(t->p - t->order);
    const int64_t nc = t->ht.ncells();
    const bool f32 = t->prec == FMM_PREC_MIXED, harm = t->basis == FMM_M2L_HARMONIC;
    M2LVariant v;
    if (!m2l_lookup(t->p, t->order, f32, harm, &v, t->mfma)) return hipErrorInvalidValue;
    BlockBounds bb;
    for (int i = 0; i < 17; ++i) bb.lo[i] = v.blo[i];
    bb.nb = v.nblocks;
    if (harm) {
        const unsigned g = (unsigned)((nc + kHarmCells - 1) / kHarmCells);
        const int nlh = hterms(t->p - t->order);
        // the locals stay reduced (nl = 0 asks for the n_z <= 1 part only)
#define COMBINE_H(T)                                                                                            \
    hipLaunchKernelGGL(m2l_combine_h_kernel<T>, dim3(g), dim3(256), 0, s, (int)nc, 0, nlh, v.nl_pad, bb,         \
                       t->d_cell_slot, t->d_tile_chunk0, t->d_tile_nchunk, (const T *)t->d_part, t->d_L64)
        if (f32) COMBINE_H(float);
        else COMBINE_H(double);
#undef COMBINE_H
        return hipGetLastError();
    }
    const size_t tot = (size_t)nc * nl;
    const unsigned g = (unsigned)((tot + 255) / 256);
#define COMBINE(T)                                                                                              \
    hipLaunchKernelGGL(m2l_combine_kernel<T>, dim3(g), dim3(256), 0, s, (int)nc, nl, v.nl_pad, bb,              \
                       t->d_cell_slot, t->d_tile_chunk0, t->d_tile_nchunk, (const T *)t->d_part, t->d_L64)
    if (f32) COMBINE(float);
    else COMBINE(double);
#undef COMBINE
    return hipGetLastError();
}
