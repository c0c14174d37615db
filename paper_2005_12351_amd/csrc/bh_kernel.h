// Multipolar Barnes-Hut evaluation kernel (Section 3.2 of Pepper & Fangohr,
// arXiv 2005.12351), shared by bh.hip (potential and field) and bh_grad.hip
// (with the field gradient): every particle walks the tree from the root; a
// cell that satisfies r_A < theta |x - z_A| (Eq. 12; r = half the side, z =
// geometric centre) and does not contain the particle contributes through
// M2P (Eq. 6), an unaccepted leaf through direct interaction, any other cell
// is opened.
//
// GPU layout: one wavefront = 64 consecutive particles in Morton order, which
// are spatially close.  The wave walks the union of its particles' traversals
// with an LDS stack of (cell, lane mask); each lane takes its own acceptance
// decision, in FP64 with the same rounding sequence as the definition above,
// so every particle accepts exactly the cells it would accept alone and sees
// them in the same depth-first order.  The cell's multipole and the leaf's
// sources are identical for all lanes and are read through scalar loads.
#pragma once
#include <cmath>

#include "fmm_internal.h"
#include "pair_kernels.h"
#include "bh_m2p.h"

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
    double *grad;                 // field gradient (n x 6), kernels with GRAD only
};

constexpr int kStack = 8 * (kMaxLevel + 3);

typedef void (*bh_fn)(BHArgs);

__device__ __forceinline__ void wave_sync_bh()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// H: the rows are folded onto the harmonic basis and contracted by M2PEvalH
// GRAD: also the field gradient, G_ij = -(1/r^3) sum M~ D_{n+e_i+e_j}(u) for
// an accepted cell and the pairs' closed forms for a leaf
template <int P, int S, typename T, bool H, bool GRAD>
__global__ __launch_bounds__(64) void bh_kernel(BHArgs a)
{
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int W = (S + 1) * (S + 2) / 2;
    __shared__ int stk_c[kStack];
    __shared__ unsigned long long stk_m[kStack];
    const int lane = threadIdx.x;
    const int i = blockIdx.x * 64 + lane;
    const bool valid = i < a.n;
    const int ii = valid ? i : a.n - 1;
    const size_t n = a.n;
    const double xi = a.xs[ii], yi = a.xs[n + ii], zi = a.xs[2 * n + ii];
    double ph = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
            const T *Mc = Mb + (size_t)c * a.nmp;
            const T ux = (T)(dx * ir), uy = (T)(dy * ir), uz = (T)(dz * ir);
            if constexpr (GRAD) {
                T gg[6];
                if constexpr (H) M2PEvalGH<P, S, T>::eval(Mc, ux, uy, uz, p_, x_, y_, z_, gg);
                else M2PEvalG<P, S, T>::eval(Mc, ux, uy, uz, p_, x_, y_, z_, gg);
                const double ir3 = ir * ir * ir;
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] -= (double)gg[q] * ir3;
            } else if constexpr (H) {
                M2PEvalH<P, S, T>::eval(Mc, ux, uy, uz, p_, x_, y_, z_);
            } else {
                M2PEval<P, S, T>::eval(Mc, ux, uy, uz, p_, x_, y_, z_);
            }
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
                            if (a.mask & 1) {
                                p2p_pair_f64<0>(rx, ry, rz, mj + off, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_f64<0>(rx, ry, rz, mj + off, g);
                                off += 1;
                            }
                            if (a.mask & 2) {
                                p2p_pair_f64<1>(rx, ry, rz, mj + off, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_f64<1>(rx, ry, rz, mj + off, g);
                                off += 3;
                            }
                            if (a.mask & 4) {
                                p2p_pair_f64<2>(rx, ry, rz, mj + off, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_f64<2>(rx, ry, rz, mj + off, g);
                                off += 6;
                            }
                            if (a.mask & 8) {
                                p2p_pair_oct_f64(rx, ry, rz, mj + off, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_oct_f64(rx, ry, rz, mj + off, g);
                            }
                        }
                    } else if (F32) {
                        // sources in units of the leaf radius, FP32 block sum
                        const double ir = 1.0 / r;
                        float bp = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
                        float bg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                        for (int j = cell.first; j < cell.first + cell.count; ++j) {
                            if (j == i) continue;
                            const float rx = (float)((xi - a.xs[j]) * ir), ry = (float)((yi - a.xs[n + j]) * ir),
                                        rz = (float)((zi - a.xs[2 * n + j]) * ir);
                            const float r2 = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, rz * rz));
                            const float4 *m4 =
                                reinterpret_cast<const float4 *>(a.m32) + (size_t)(m32_width(1 << S) / 4) * j;
                            const float inv = __builtin_amdgcn_rsqf(r2);
                            if constexpr (S == 3) {
                                p2p_pair_oct_f32(rx, ry, rz, inv, m4[0], m4[1], m4[2], m4[3], bp, bx, by, bz);
                                if constexpr (GRAD) p2p_pair_grad_oct_f32(rx, ry, rz, inv, m4[0], m4[1], m4[2], m4[3], bg);
                            } else {
                                p2p_pair_f32<S>(rx, ry, rz, inv, m4[0], m4[1], bp, bx, by, bz);
                                if constexpr (GRAD) p2p_pair_grad_f32<S>(rx, ry, rz, inv, m4[0], m4[1], bg);
                            }
                        }
                        double sphi = ir;
#pragma unroll
                        for (int q = 0; q < S; ++q) sphi *= ir;
                        const double sfld = sphi * ir;
                        ph += (double)bp * sphi;
                        ex += (double)bx * sfld;
                        ey += (double)by * sfld;
                        ez += (double)bz * sfld;
                        if constexpr (GRAD) {
                            const double sgrd = sfld * ir;
#pragma unroll
                            for (int q = 0; q < 6; ++q) g[q] += (double)bg[q] * sgrd;
                        }
                    } else {
                        for (int j = cell.first; j < cell.first + cell.count; ++j) {
                            if (j == i) continue;
                            const double rx = xi - a.xs[j], ry = yi - a.xs[n + j], rz = zi - a.xs[2 * n + j];
                            if constexpr (S == 3) {
                                p2p_pair_oct_f64(rx, ry, rz, a.m64 + (size_t)j * W, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_oct_f64(rx, ry, rz, a.m64 + (size_t)j * W, g);
                            } else {
                                p2p_pair_f64<S>(rx, ry, rz, a.m64 + (size_t)j * W, ph, ex, ey, ez);
                                if constexpr (GRAD) p2p_pair_grad_f64<S>(rx, ry, rz, a.m64 + (size_t)j * W, g);
                            }
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
        if constexpr (GRAD) {
            if (a.outputs & FMM_GRAD)
#pragma unroll
                for (int q = 0; q < 6; ++q) a.grad[6 * o + q] = g[q];
        }
    }
}

// the kernel for (p, s, precision, basis), p in [max(s,1), FMM_P_MAX]
template <bool GRAD, int P, int S>
bh_fn bh_pick(bool f32, bool h)
{
    if (h) return f32 ? (bh_fn)bh_kernel<P, S, float, true, GRAD> : (bh_fn)bh_kernel<P, S, double, true, GRAD>;
    return f32 ? (bh_fn)bh_kernel<P, S, float, false, GRAD> : (bh_fn)bh_kernel<P, S, double, false, GRAD>;
}

template <bool GRAD, int S, int P = (S > 1 ? S : 1)>
bh_fn bh_pick_p(int p, bool f32, bool h)
{
    if constexpr (P > FMM_P_MAX) {
        return nullptr;
    } else {
        if (p == P) return bh_pick<GRAD, P, S>(f32, h);
        return bh_pick_p<GRAD, S, P + 1>(p, f32, h);
    }
}

// one per (field gradient, source order), each in its own generated
// translation unit (gen_bh.py)
bh_fn bh_select_f_s0(int p, bool f32, bool h);
bh_fn bh_select_f_s1(int p, bool f32, bool h);
bh_fn bh_select_f_s2(int p, bool f32, bool h);
bh_fn bh_select_f_s3(int p, bool f32, bool h);
bh_fn bh_select_g_s0(int p, bool f32, bool h);
bh_fn bh_select_g_s1(int p, bool f32, bool h);
bh_fn bh_select_g_s2(int p, bool f32, bool h);
bh_fn bh_select_g_s3(int p, bool f32, bool h);
