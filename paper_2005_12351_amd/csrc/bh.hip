// Multipolar Barnes-Hut evaluation (Section 3.2 of Pepper & Fangohr, arXiv
// 2005.12351): every particle walks the tree from the root; a cell that
// satisfies r_A < theta |x - z_A| (Eq. 12; r = half the side, z = geometric
// centre) and does not contain the particle contributes through M2P (Eq. 6),
// an unaccepted leaf through direct interaction, any other cell is opened.
//
// GPU layout: one wavefront = 64 consecutive particles in Morton order, which
// are spatially close.  The wave walks the union of its particles' traversals
// with an LDS stack of (cell, lane mask); each lane takes its own acceptance
// decision, in FP64 with the same rounding sequence as the definition above,
// so every particle accepts exactly the cells it would accept alone and sees
// them in the same depth-first order.  The cell's multipole and the leaf's
// sources are identical for all lanes and are read through scalar loads.
#include <cmath>

#include "fmm_internal.h"
#include "pair_kernels.h"
#include "bh_m2p.h"

namespace {

struct BHGeo {
    double lo[3];
    double h;
};

struct BHArgs {
    const DevCell *cells;
    const double *xs;       // sorted positions, SoA
    const double *m64;      // sorted moments FP64 (w per particle)
    const float *m32;       // sorted moments FP32 (8 per particle)
    const void *M;          // normalised multipoles (harmonic basis: folded), rows of nmp
    const int32_t *perm;
    double *phi, *field;
    int n, nmp, outputs;
    double theta2;
    BHGeo g;
    unsigned long long *counts;   // [0] accepted (particle, cell) pairs, [1] direct pairs
    int mask, w;                  // source orders present (bit mask), FP64 moments per particle
};

constexpr int kStack = 8 * (kMaxLevel + 3);

__device__ __forceinline__ void wave_sync_bh()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// H: the rows are folded onto the harmonic basis and contracted by M2PEvalH
template <int P, int S, typename T, bool H>
__global__ __launch_bounds__(64) void bh_kernel(BHArgs a)
{
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int W = S == 0 ? 1 : (S == 1 ? 3 : 6);
    __shared__ int stk_c[kStack];
    __shared__ unsigned long long stk_m[kStack];
    const int lane = threadIdx.x;
    const int i = blockIdx.x * 64 + lane;
    const bool valid = i < a.n;
    const int ii = valid ? i : a.n - 1;
    const size_t n = a.n;
    const double xi = a.xs[ii], yi = a.xs[n + ii], zi = a.xs[2 * n + ii];
    double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    const unsigned long long live = __ballot(valid);
    int sp = 0;
    if (lane == 0) {
        stk_c[0] = 0;
        stk_m[0] = live;
    }
    sp = 1;
    wave_sync_bh();
    const T *Mb = (const T *)a.M;
    unsigned int n_m2p = 0, n_p2p = 0;
    while (sp > 0) {
        --sp;
        const int c = stk_c[sp];
        const unsigned long long mask = stk_m[sp];
        wave_sync_bh();
        const DevCell cell = a.cells[c];
        const bool mine = (mask >> lane) & 1ull;
        const double rc = ldexp(1.0, kMaxLevel - cell.level);
        const double zx = __dadd_rn(a.g.lo[0], __dmul_rn((double)(2 * cell.ix + 1) * rc, a.g.h));
        const double zy = __dadd_rn(a.g.lo[1], __dmul_rn((double)(2 * cell.iy + 1) * rc, a.g.h));
        const double zz = __dadd_rn(a.g.lo[2], __dmul_rn((double)(2 * cell.iz + 1) * rc, a.g.h));
        const double r = __dmul_rn(rc, a.g.h);
        const double dx = __dsub_rn(xi, zx), dy = __dsub_rn(yi, zy), dz = __dsub_rn(zi, zz);
        const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        const bool inside = i >= cell.first && i < cell.first + cell.count;
        const bool accept = mine && !inside && (__dmul_rn(r, r) < __dmul_rn(a.theta2, d2));
        const unsigned long long acc_m = __ballot(accept);
        const unsigned long long rest = mask & ~acc_m;
        if (accept) {
            ++n_m2p;
            // M2P in the normalised form: u = (x - z)/r, phi = (1/r) sum M~ D(u),
            // E = -(1/r^2) sum M~ D_{+e}(u)
            const double ir = 1.0 / r;
            T p_, x_, y_, z_;
            if constexpr (H)
                M2PEvalH<P, S, T>::eval(Mb + (size_t)c * a.nmp, (T)(dx * ir), (T)(dy * ir), (T)(dz * ir), p_, x_, y_,
                                        z_);
            else
                M2PEval<P, S, T>::eval(Mb + (size_t)c * a.nmp, (T)(dx * ir), (T)(dy * ir), (T)(dz * ir), p_, x_, y_,
                                       z_);
            ph += (double)p_ * ir;
            const double ir2 = ir * ir;
            ex -= (double)x_ * ir2;
            ey -= (double)y_ * ir2;
            ez -= (double)z_ * ir2;
        }
        if (rest) {
            if (cell.nchild == 0) {
                if ((rest >> lane) & 1ull) {
                    n_p2p += (unsigned)cell.count - (inside ? 1u : 0u);
                    if (a.mask != (1 << S)) {
                        // several source orders: each order's closed form, FP64
                        for (int j = cell.first; j < cell.first + cell.count; ++j) {
                            if (j == i) continue;
                            const double *mj = a.m64 + (size_t)j * a.w;
                            const double rx = xi - a.xs[j], ry = yi - a.xs[n + j], rz = zi - a.xs[2 * n + j];
                            int off = 0;
                            if (a.mask & 1) p2p_pair_f64<0>(rx, ry, rz, mj + off++, ph, ex, ey, ez);
                            if (a.mask & 2) {
                                p2p_pair_f64<1>(rx, ry, rz, mj + off, ph, ex, ey, ez);
                                off += 3;
                            }
                            if (a.mask & 4) p2p_pair_f64<2>(rx, ry, rz, mj + off, ph, ex, ey, ez);
                        }
                    } else if (F32) {
                        // sources in units of the leaf radius, FP32 block sum
                        const double ir = 1.0 / r;
                        float bp = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
                        for (int j = cell.first; j < cell.first + cell.count; ++j) {
                            if (j == i) continue;
                            const float rx = (float)((xi - a.xs[j]) * ir), ry = (float)((yi - a.xs[n + j]) * ir),
                                        rz = (float)((zi - a.xs[2 * n + j]) * ir);
                            const float r2 = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, rz * rz));
                            const float4 *m4 = reinterpret_cast<const float4 *>(a.m32) + 2 * (size_t)j;
                            p2p_pair_f32<S>(rx, ry, rz, __builtin_amdgcn_rsqf(r2), m4[0], m4[1], bp, bx, by, bz);
                        }
                        const double sphi = S == 0 ? ir : (S == 1 ? ir * ir : ir * ir * ir), sfld = sphi * ir;
                        ph += (double)bp * sphi;
                        ex += (double)bx * sfld;
                        ey += (double)by * sfld;
                        ez += (double)bz * sfld;
                    } else {
                        for (int j = cell.first; j < cell.first + cell.count; ++j) {
                            if (j == i) continue;
                            p2p_pair_f64<S>(xi - a.xs[j], yi - a.xs[n + j], zi - a.xs[2 * n + j],
                                            a.m64 + (size_t)j * W, ph, ex, ey, ez);
                        }
                    }
                }
            } else {
                // children in reverse, so that they are visited in octant order
                if (lane == 0)
                    for (int k = cell.nchild - 1; k >= 0; --k) {
                        stk_c[sp + (cell.nchild - 1 - k)] = cell.child0 + k;
                        stk_m[sp + (cell.nchild - 1 - k)] = rest;
                    }
                sp += cell.nchild;
                wave_sync_bh();
            }
        }
    }
    // interaction counts of the wave, one atomic per wave
    unsigned long long c0 = n_m2p, c1 = n_p2p;
    for (int o = 32; o > 0; o >>= 1) {
        c0 += __shfl_down(c0, o, 64);
        c1 += __shfl_down(c1, o, 64);
    }
    if (lane == 0) {
        atomicAdd(&a.counts[0], c0);
        atomicAdd(&a.counts[1], c1);
    }
    if (valid) {
        const size_t o = (size_t)a.perm[i];
        if (a.outputs & FMM_POT) a.phi[o] = ph;
        if (a.outputs & FMM_FIELD) {
            a.field[3 * o] = ex;
            a.field[3 * o + 1] = ey;
            a.field[3 * o + 2] = ez;
        }
    }
}

// counters are cleared by a kernel, not a memset, so that the launch
// sequence can be captured into a graph
__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

typedef void (*bh_fn)(BHArgs);

template <int P, int S>
bh_fn pick(bool f32, bool h)
{
    if (h) return f32 ? (bh_fn)bh_kernel<P, S, float, true> : (bh_fn)bh_kernel<P, S, double, true>;
    return f32 ? (bh_fn)bh_kernel<P, S, float, false> : (bh_fn)bh_kernel<P, S, double, false>;
}

template <int S, int P = (S > 1 ? S : 1)>
bh_fn pick_p(int p, bool f32, bool h)
{
    if constexpr (P > FMM_P_MAX) {
        return nullptr;
    } else {
        if (p == P) return pick<P, S>(f32, h);
        return pick_p<S, P + 1>(p, f32, h);
    }
}

}  // namespace

hipError_t launch_bh(fmm_tree *t, int outputs, double *phi, double *field, hipStream_t s)
{
    const bool f32 = t->prec == FMM_PREC_MIXED, h = t->basis == FMM_M2L_HARMONIC;
    bh_fn k = t->order == 0 ? pick_p<0>(t->p, f32, h)
                            : (t->order == 1 ? pick_p<1>(t->p, f32, h) : pick_p<2>(t->p, f32, h));
    if (!k) return hipErrorInvalidValue;
    BHArgs a;
    a.cells = t->d_cells;
    a.xs = t->d_x;
    a.m64 = t->d_mom;
    a.m32 = t->d_mom32;
    a.M = h ? (const void *)t->d_Mh : (f32 ? (const void *)t->d_M32 : (const void *)t->d_M64);
    a.perm = t->d_perm;
    a.phi = phi;
    a.field = field;
    a.n = (int)t->ht.n;
    a.nmp = h ? (hterms(t->p) - hterms(t->order - 1) + 3) / 4 * 4 : (nterms(t->p) - nterms(t->order - 1) + 3) / 4 * 4;
    a.outputs = outputs;
    a.theta2 = t->theta * t->theta;
    for (int d = 0; d < 3; ++d) a.g.lo[d] = t->ht.lo[d];
    a.g.h = t->ht.h;
    a.counts = t->d_bhcount;
    a.mask = t->smask;
    a.w = mask_width(t->smask);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, t->d_bhcount, 2);
    hipLaunchKernelGGL(k, dim3((unsigned)((t->ht.n + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}
