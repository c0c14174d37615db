// GPU kernels of libfmm.so other than M2L and Barnes-Hut: particle and
// moment preparation, P2M, M2M, L2L, P2P and L2P (Pepper & Fangohr, arXiv
// 2005.12351, Section 2 and Section 3.2).
//
// All expansions on the GPU are kept in a dimensionless form:
//   M~_n(A) = M_n(A) / r_A^|n|,  L~_n(B) = L_n(B) * r_B^(|n|+1),
// with r the cell radius (half side).  Child and parent centres differ by
// exactly +-r_child per axis, so M2M and L2L become fixed rational operators
// per octant and the M2L derivative tensor depends only on the dimensionless
// pair geometry.  P2M, M2M, L2L, L2P run in FP64.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "fmm_internal.h"
#include "pair_kernels.h"

// ------------------------------------------------------------------ tables
struct HalfTable {
    double v[kPTable + 2];
};
constexpr HalfTable make_half()
{
    HalfTable t{};
    double f = 1.0;
    for (int a = 0; a <= kPTable + 1; ++a) {
        if (a > 0) f = f * 0.5 / a;
        t.v[a] = f;
    }
    return t;
}
static __constant__ MITable k_mi = make_mi();
__constant__ HalfTable k_half = make_half();   // (1/2)^a / a!

__device__ __forceinline__ double cell_radius(int level, double h) { return ldexp(1.0, kMaxLevel - level) * h; }

// real centre, computed exactly as the canonical definition: lo + c * h
__device__ __forceinline__ void cell_center(const DevCell &c, const double *lo, double h, double *z)
{
    const double r = ldexp(1.0, kMaxLevel - c.level);
    z[0] = __dadd_rn(lo[0], __dmul_rn((double)(2 * c.ix + 1) * r, h));
    z[1] = __dadd_rn(lo[1], __dmul_rn((double)(2 * c.iy + 1) * r, h));
    z[2] = __dadd_rn(lo[2], __dmul_rn((double)(2 * c.iz + 1) * r, h));
}

struct Geo {
    double lo[3];
    double h;
};

// ------------------------------------------------------------------ fill
__global__ void fill_kernel(double *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void zero_ints_kernel(int *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

hipError_t launch_fill(double *p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ particles
// sorted SoA positions
__global__ void prep_particles_kernel(int n, const double *__restrict__ pos, const int32_t *__restrict__ perm,
                                      double *__restrict__ xs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    xs[i] = pos[3 * (size_t)j];
    xs[n + i] = pos[3 * (size_t)j + 1];
    xs[2 * (size_t)n + i] = pos[3 * (size_t)j + 2];
}

hipError_t launch_prep_positions(fmm_tree *t, const double *pos, hipStream_t s)
{
    const int n = (int)t->ht.n;
    hipLaunchKernelGGL(prep_particles_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, t->d_perm, t->d_x);
    return hipGetLastError();
}

// Sorted moments of particle i (sorted order; perm maps it to the caller's
// row): FP64 (the caller's row of w values) and FP32 in the layout m32_width
// describes.  P2M writes them while it visits every particle once; the near
// field reads them.
__device__ __forceinline__ void sort_moments(size_t i, int mask, const double *__restrict__ r,
                                             double *__restrict__ m64, float *__restrict__ m32)
{
    const int w = mask_width(mask), wf = m32_width(mask);
    float v[28];
#pragma unroll
    for (int k = 0; k < 28; ++k) v[k] = 0.f;
    for (int k = 0; k < w; ++k) m64[i * w + k] = r[k];
    // the octupole block: ten components and the trace vector
    auto oct = [&](const double *o, int at) {
        for (int k = 0; k < 10; ++k) v[at + k] = (float)o[k];
        v[at + 10] = (float)(o[0] + o[3] + o[5]);
        v[at + 11] = (float)(o[1] + o[6] + o[8]);
        v[at + 12] = (float)(o[2] + o[7] + o[9]);
    };
    if (mask == 8) {
        oct(r, 0);
    } else if (mask_single(mask)) {
        for (int k = 0; k < w; ++k) v[k] = (float)r[k];
        if (w == 6) v[6] = (float)(r[0] + r[3] + r[5]);
    } else {
        int off = 0;
        if (mask & 1) v[0] = (float)r[off++];
        if (mask & 2) {
            v[1] = (float)r[off];
            v[2] = (float)r[off + 1];
            v[3] = (float)r[off + 2];
            off += 3;
        }
        if (mask & 4) {
            for (int k = 0; k < 6; ++k) v[4 + k] = (float)r[off + k];
            v[10] = (float)(r[off] + r[off + 3] + r[off + 5]);
            off += 6;
        }
        if (mask & 8) oct(r + off, 12);
    }
    float4 *o = reinterpret_cast<float4 *>(m32) + (size_t)(wf / 4) * i;
    for (int k = 0; k < wf / 4; ++k) o[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// ------------------------------------------------------------------ P2M
// M~_n = sum_j sum_k r^-k sum_{sigma <= n, |sigma| = k} zeta_j^(n-sigma)/(n-sigma)! S_sigma(j)
// with zeta = (z - x_j)/r and S_sigma = (-1)^k T_sigma / sigma! (Eq. 3, Eq. 5),
// k over the source orders present (MASK bit k), so a system with several
// orders adds each part's expansion.  One workgroup per leaf; particles are
// staged in LDS 32 at a time as per-axis tables X_a = zeta_x^a/a! (and Y, Z).
// Two kernels, chosen by the source orders:
// - p2m_coef_kernel (charges and dipoles, and any system with octupoles): a
//   thread owns one or more coefficients n and adds every particle's term,
//   1 + 3 (+ 6 + 10) products of table entries per particle;
// - p2m_kernel (any quadrupole part): the monomial factorises over the axes
//   and sigma has at most two units, so for a fixed column (ax, ay) the
//   particle's contribution to every coefficient (ax, ay, az) is
//   A0 Z_az + A1 Z_{az-1} + A2 Z_{az-2}, with
//   A0 = S_0 X0 Y0 + S_ex X1 Y0 + S_ey X0 Y1 + S_2ex X2 Y0 + S_ex+ey X1 Y1 + S_2ey X0 Y2,
//   A1 = S_ez X0 Y0 + S_ex+ez X1 Y0 + S_ey+ez X0 Y1, A2 = S_2ez X0 Y0
//   (Xk = X_{ax-k}, Yk = Y_{ay-k}).  A thread owns a block of consecutive az
//   of one column and forms A0..A2 once per particle; when the blocks fill
//   less than half the workgroup, groups of threads take every ngroups-th
//   particle and their sums are added in group order at the end (a fixed
//   order).  With quadrupoles this is 25 % faster than the per-coefficient
//   form (ten terms per coefficient and particle there); with dipoles it is
//   not, so those keep the simpler kernel.
constexpr int kP2MThreads = 128;
constexpr int kP2MStage = 32;                    // particles staged per pass
constexpr int kP2MBlk = 6;                       // longest column block
constexpr int kAxWc = FMM_P_MAX + 2;             // axis table row of the per-coefficient kernel: X_0..X_p
constexpr int kAxW = FMM_P_MAX + kP2MBlk + 4;    // of the column kernel: X_-2, X_-1 (zero), X_0..X_p, zero padding

struct InvTable {
    double v[kPTable + 2];
};
constexpr InvTable make_inv()
{
    InvTable t{};
    t.v[0] = 1.0;
    for (int a = 1; a <= kPTable + 1; ++a) t.v[a] = 1.0 / a;
    return t;
}
__constant__ InvTable k_inv = make_inv();   // 1/a

static __constant__ FoldTable k_fold = make_fold();
static_assert(make_fold().start[hterms(kPTable)] == kFoldTerms, "fold table size");

// component h of the harmonic-basis fold of a multipole row (row indexed by
// multi-index)
__device__ __forceinline__ double fold_component(const double *row, int h)
{
    double acc = 0.0;
    for (int e = k_fold.start[h]; e < k_fold.start[h + 1]; ++e) acc = fma((double)k_fold.w[e], row[k_fold.idx[e]], acc);
    return acc;
}

template <int MASK>
__global__ __launch_bounds__(kP2MThreads) void p2m_coef_kernel(int p, int nmp, const int32_t *__restrict__ leaves,
                                                          const DevCell *__restrict__ cells, Geo g,
                                                          const double *__restrict__ xs, int n,
                                                          const double *__restrict__ mom_user,
                                                          const int32_t *__restrict__ perm, double *__restrict__ mom64,
                                                          float *__restrict__ mom32, double *__restrict__ M,
                                                          float *__restrict__ M32, int nhp, float *__restrict__ Mh32,
                                                          double *__restrict__ Mh64)
{
    constexpr int W = mask_width(MASK);
    constexpr int S = mask_min_order(MASK);
    constexpr bool Q0 = MASK & 1, Q1 = MASK & 2, Q2 = MASK & 4, Q3 = MASK & 8;
    // source tensor slots: 0 order 0; 1..3 order 1; 4..9 order 2; 10..19
    // order 3 (index order within each order)
    __shared__ double pw[kP2MStage][3][kAxWc];
    __shared__ double sv[kP2MStage][20];
    const int c = leaves[blockIdx.x];
    const DevCell cell = cells[c];
    double z[3];
    cell_center(cell, g.lo, g.h, z);
    const double r = cell_radius(cell.level, g.h);
    const double ir = 1.0 / r;
    const int n0 = nterms(S - 1), nm = nterms(p) - n0;
    constexpr int KMAX = (nterms(FMM_P_MAX) + kP2MThreads - 1) / kP2MThreads;
    double acc[KMAX];
    int ix[KMAX], iy[KMAX], iz[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        acc[k] = 0.0;
        const int i = threadIdx.x + k * kP2MThreads;
        const MultiIndex nn = k_mi.v[i < nm ? n0 + i : 0];
        ix[k] = nn.x;
        iy[k] = nn.y;
        iz[k] = nn.z;
    }
    for (int base = 0; base < cell.count; base += kP2MStage) {
        const int cnt = min(kP2MStage, cell.count - base);
        __syncthreads();
        for (int it = threadIdx.x; it < 3 * cnt; it += kP2MThreads) {
            // item -> (particle, axis): zeta^a / a! for a = 0..p
            const int t = it / 3, d = it % 3;
            const size_t j = (size_t)cell.first + base + t;
            const double zeta = (z[d] - xs[(size_t)d * n + j]) * ir;
            double f = 1.0;
            pw[t][d][0] = 1.0;
            for (int a = 1; a <= p; ++a) {
                f = f * zeta * k_inv.v[a];
                pw[t][d][a] = f;
            }
        }
        if ((int)threadIdx.x < cnt) {
            const int t = threadIdx.x;
            const size_t i = (size_t)cell.first + base + t;
            const double *m = mom_user + (size_t)perm[i] * W;
            sort_moments(i, MASK, m, mom64, mom32);
            int off = 0;
            if (Q0) sv[t][0] = m[off++];
            if (Q1) {
                sv[t][1] = -m[off] * ir;
                sv[t][2] = -m[off + 1] * ir;
                sv[t][3] = -m[off + 2] * ir;
                off += 3;
            }
            if (Q2) {
                const double ir2 = ir * ir;
                sv[t][4] = 0.5 * m[off] * ir2;       // (2,0,0)
                sv[t][5] = m[off + 1] * ir2;         // (1,1,0)
                sv[t][6] = m[off + 2] * ir2;         // (1,0,1)
                sv[t][7] = 0.5 * m[off + 3] * ir2;   // (0,2,0)
                sv[t][8] = m[off + 4] * ir2;         // (0,1,1)
                sv[t][9] = 0.5 * m[off + 5] * ir2;   // (0,0,2)
                off += 6;
            }
            if (Q3) {
                // S_m = -O_m / m!: m! = 6 for (3,0,0)-type, 2 for (2,1,0)-type,
                // 1 for (1,1,1)
                const double ir3 = ir * ir * ir;
                constexpr double kInvF[10] = {1.0 / 6, 0.5, 0.5, 0.5, 1.0, 0.5, 1.0 / 6, 0.5, 0.5, 1.0 / 6};
#pragma unroll
                for (int q = 0; q < 10; ++q) sv[t][10 + q] = -m[off + q] * kInvF[q] * ir3;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if ((int)threadIdx.x + k * kP2MThreads >= nm) break;
            const int ax = ix[k], ay = iy[k], az = iz[k];
            double a = acc[k];
            for (int t = 0; t < cnt; ++t) {
                // a zero table entry stands for a negative index
                const double px0 = pw[t][0][ax], py0 = pw[t][1][ay], pz0 = pw[t][2][az];
                if (Q0) a = fma(px0 * py0, pz0 * sv[t][0], a);
                if (Q1 || Q2 || Q3) {
                    const double px1 = ax >= 1 ? pw[t][0][ax - 1] : 0.0, py1 = ay >= 1 ? pw[t][1][ay - 1] : 0.0,
                                 pz1 = az >= 1 ? pw[t][2][az - 1] : 0.0;
                    if (Q1) {
                        a = fma(px1 * py0, pz0 * sv[t][1], a);
                        a = fma(px0 * py1, pz0 * sv[t][2], a);
                        a = fma(px0 * py0, pz1 * sv[t][3], a);
                    }
                    if (Q2) {
                        const double px2 = ax >= 2 ? pw[t][0][ax - 2] : 0.0, py2 = ay >= 2 ? pw[t][1][ay - 2] : 0.0,
                                     pz2 = az >= 2 ? pw[t][2][az - 2] : 0.0;
                        a = fma(px2 * py0, pz0 * sv[t][4], a);
                        a = fma(px1 * py1, pz0 * sv[t][5], a);
                        a = fma(px1 * py0, pz1 * sv[t][6], a);
                        a = fma(px0 * py2, pz0 * sv[t][7], a);
                        a = fma(px0 * py1, pz1 * sv[t][8], a);
                        a = fma(px0 * py0, pz2 * sv[t][9], a);
                    }
                    if (Q3) {
                        const double px2 = ax >= 2 ? pw[t][0][ax - 2] : 0.0, py2 = ay >= 2 ? pw[t][1][ay - 2] : 0.0,
                                     pz2 = az >= 2 ? pw[t][2][az - 2] : 0.0;
                        const double px3 = ax >= 3 ? pw[t][0][ax - 3] : 0.0, py3 = ay >= 3 ? pw[t][1][ay - 3] : 0.0,
                                     pz3 = az >= 3 ? pw[t][2][az - 3] : 0.0;
                        a = fma(px3 * py0, pz0 * sv[t][10], a);   // (3,0,0)
                        a = fma(px2 * py1, pz0 * sv[t][11], a);   // (2,1,0)
                        a = fma(px2 * py0, pz1 * sv[t][12], a);   // (2,0,1)
                        a = fma(px1 * py2, pz0 * sv[t][13], a);   // (1,2,0)
                        a = fma(px1 * py1, pz1 * sv[t][14], a);   // (1,1,1)
                        a = fma(px1 * py0, pz2 * sv[t][15], a);   // (1,0,2)
                        a = fma(px0 * py3, pz0 * sv[t][16], a);   // (0,3,0)
                        a = fma(px0 * py2, pz1 * sv[t][17], a);   // (0,2,1)
                        a = fma(px0 * py1, pz2 * sv[t][18], a);   // (0,1,2)
                        a = fma(px0 * py0, pz3 * sv[t][19], a);   // (0,0,3)
                    }
                }
            }
            acc[k] = a;
        }
    }
    __shared__ double row[nterms(FMM_P_MAX)];   // the finished row, indexed by multi-index
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if ((int)threadIdx.x + k * kP2MThreads < nm) {
            const size_t o = (size_t)c * nmp + threadIdx.x + k * kP2MThreads;
            M[o] = acc[k];
            if (M32) M32[o] = (float)acc[k];   // the copy the full-basis mixed-precision M2L reads
            row[n0 + threadIdx.x + k * kP2MThreads] = acc[k];
        }
    if (Mh32 || Mh64) {
        // the harmonic-basis row the M2L reads (in its precision)
        __syncthreads();
        const int h0 = hterms(S - 1), nh = hterms(p) - h0;
        for (int h = threadIdx.x; h < nh; h += kP2MThreads) {
            const double v = fold_component(row, h + h0);
            if (Mh32) Mh32[(size_t)c * nhp + h] = (float)v;
            else Mh64[(size_t)c * nhp + h] = v;
        }
    }
}

// Column blocks of every (p, s), fixed at compile time: for each pair the
// block length with the fewest multiply-add steps per particle (about 10 to
// form A0..A2 plus 3 per block entry, divided by the groups of threads that
// share the particles), then the blocks in column order, (ax, ay, az0, nb).
struct P2MItem {
    int8_t ax, ay, az0, nb;
};
constexpr int kP2MPlanMax = 3 * (FMM_P_MAX + 1) * kP2MThreads;
struct P2MPlan {
    int16_t start[FMM_P_MAX + 1][3];
    int16_t nitems[FMM_P_MAX + 1][3];
    int8_t blk[FMM_P_MAX + 1][3];
    int8_t ngroups[FMM_P_MAX + 1][3];
    P2MItem items[kP2MPlanMax];
};
constexpr int p2m_count(int p, int S, int blk)
{
    int cnt = 0;
    for (int x = 0; x <= p; ++x)
        for (int y = 0; y <= p - x; ++y) {
            const int lo = S - x - y > 0 ? S - x - y : 0, hi = p - x - y;
            cnt += (hi - lo + blk) / blk;
        }
    return cnt;
}
constexpr P2MPlan make_p2m_plan()
{
    P2MPlan pl{};
    int pos = 0;
    for (int p = 0; p <= FMM_P_MAX; ++p)
        for (int S = 0; S < 3; ++S) {
            pl.start[p][S] = (int16_t)pos;
            if (S > p) continue;
            int best_b = kP2MBlk, best_n = p2m_count(p, S, kP2MBlk);
            double best = (10.0 + 3.0 * kP2MBlk) / (kP2MThreads / best_n);
            for (int bl = 2; bl < kP2MBlk; ++bl) {
                const int ni = p2m_count(p, S, bl);
                if (ni > kP2MThreads) continue;
                const double cost = (10.0 + 3.0 * bl) / (kP2MThreads / ni);
                if (cost < best) {
                    best = cost;
                    best_b = bl;
                    best_n = ni;
                }
            }
            pl.blk[p][S] = (int8_t)best_b;
            pl.nitems[p][S] = (int16_t)best_n;
            pl.ngroups[p][S] = (int8_t)(kP2MThreads / best_n);
            for (int x = 0; x <= p; ++x)
                for (int y = 0; y <= p - x; ++y) {
                    const int lo = S - x - y > 0 ? S - x - y : 0, hi = p - x - y;
                    for (int z0 = lo; z0 <= hi; z0 += best_b)
                        pl.items[pos++] = P2MItem{(int8_t)x, (int8_t)y, (int8_t)z0,
                                                  (int8_t)(hi + 1 - z0 < best_b ? hi + 1 - z0 : best_b)};
                }
        }
    return pl;
}
static __constant__ P2MPlan k_p2m = make_p2m_plan();
static constexpr P2MPlan kP2MPlanHost = make_p2m_plan();
// the longest block always fits: at p = 10, s = 0 it makes 81 blocks
static_assert(p2m_count(FMM_P_MAX, 0, kP2MBlk) <= kP2MThreads, "P2M blocks exceed the workgroup");

template <int MASK>
__global__ __launch_bounds__(kP2MThreads) void p2m_kernel(int p, int nmp, int blk, int nitems, int ngroups,
                                                          const int32_t *__restrict__ leaves,
                                                          const DevCell *__restrict__ cells, Geo g,
                                                          const double *__restrict__ xs, int n,
                                                          const double *__restrict__ mom_user,
                                                          const int32_t *__restrict__ perm, double *__restrict__ mom64,
                                                          float *__restrict__ mom32, double *__restrict__ M,
                                                          float *__restrict__ M32, int nhp, float *__restrict__ Mh32,
                                                          double *__restrict__ Mh64)
{
    constexpr int W = mask_width(MASK);
    constexpr int S = mask_min_order(MASK);
    constexpr bool Q0 = MASK & 1, Q1 = MASK & 2, Q2 = MASK & 4;
    // source tensor slots: 0 order 0; 1..3 order 1; 4..9 order 2
    __shared__ double pw[kP2MStage][3][kAxW];
    __shared__ double sv[kP2MStage][10];
    __shared__ double gsum[kP2MThreads * kP2MBlk];   // sums of groups 1.. (ngroups > 1)
    __shared__ double row[nterms(FMM_P_MAX)];          // the finished row, indexed by multi-index
    const int c = leaves[blockIdx.x];
    const DevCell cell = cells[c];
    double z[3];
    cell_center(cell, g.lo, g.h, z);
    const double r = cell_radius(cell.level, g.h);
    const double ir = 1.0 / r;
    const int n0 = nterms(S - 1);
    const int item = (int)threadIdx.x % nitems, grp = (int)threadIdx.x / nitems;
    const bool act = grp < ngroups;
    const P2MItem pi = k_p2m.items[k_p2m.start[p][S] + item];
    const int ax = pi.ax, ay = pi.ay, az0 = pi.az0, nb = pi.nb;
    double acc[kP2MBlk];
#pragma unroll
    for (int k = 0; k < kP2MBlk; ++k) acc[k] = 0.0;
    for (int base = 0; base < cell.count; base += kP2MStage) {
        const int cnt = min(kP2MStage, cell.count - base);
        __syncthreads();
        for (int it = threadIdx.x; it < 3 * cnt; it += kP2MThreads) {
            // item -> (particle, axis): two zeros, zeta^a / a! for a = 0..p, zeros
            const int t = it / 3, d = it % 3;
            const size_t j = (size_t)cell.first + base + t;
            const double zeta = (z[d] - xs[(size_t)d * n + j]) * ir;
            double *row_t = pw[t][d];
            double f = 1.0;
            row_t[0] = 0.0;
            row_t[1] = 0.0;
            row_t[2] = 1.0;
            for (int e = 1; e <= p; ++e) {
                f = f * zeta * k_inv.v[e];
                row_t[2 + e] = f;
            }
            for (int e = p + 3; e < kAxW; ++e) row_t[e] = 0.0;
        }
        if ((int)threadIdx.x < cnt) {
            const int t = threadIdx.x;
            const size_t i = (size_t)cell.first + base + t;
            const double *m = mom_user + (size_t)perm[i] * W;
            sort_moments(i, MASK, m, mom64, mom32);
            int off = 0;
            if (Q0) sv[t][0] = m[off++];
            if (Q1) {
                sv[t][1] = -m[off] * ir;
                sv[t][2] = -m[off + 1] * ir;
                sv[t][3] = -m[off + 2] * ir;
                off += 3;
            }
            if (Q2) {
                const double ir2 = ir * ir;
                sv[t][4] = 0.5 * m[off] * ir2;       // (2,0,0)
                sv[t][5] = m[off + 1] * ir2;         // (1,1,0)
                sv[t][6] = m[off + 2] * ir2;         // (1,0,1)
                sv[t][7] = 0.5 * m[off + 3] * ir2;   // (0,2,0)
                sv[t][8] = m[off + 4] * ir2;         // (0,1,1)
                sv[t][9] = 0.5 * m[off + 5] * ir2;   // (0,0,2)
            }
        }
        __syncthreads();
        if (act) {
            for (int t = grp; t < cnt; t += ngroups) {
                const double *X = pw[t][0], *Y = pw[t][1], *Z = pw[t][2] + az0;
                const double x0 = X[ax + 2], y0 = Y[ay + 2];
                const double x0y0 = x0 * y0;
                double A0 = 0.0, A1 = 0.0, A2 = 0.0;
                if (Q0) A0 = sv[t][0] * x0y0;
                if (Q1 || Q2) {
                    const double x1 = X[ax + 1], y1 = Y[ay + 1];
                    const double x1y0 = x1 * y0, x0y1 = x0 * y1;
                    if (Q1) {
                        A0 = fma(sv[t][1], x1y0, A0);
                        A0 = fma(sv[t][2], x0y1, A0);
                        A1 = sv[t][3] * x0y0;
                    }
                    if (Q2) {
                        const double x2 = X[ax], y2 = Y[ay];
                        A0 = fma(sv[t][4], x2 * y0, A0);
                        A0 = fma(sv[t][5], x1 * y1, A0);
                        A0 = fma(sv[t][7], x0 * y2, A0);
                        A1 = fma(sv[t][6], x1y0, A1);
                        A1 = fma(sv[t][8], x0y1, A1);
                        A2 = sv[t][9] * x0y0;
                    }
                }
                // Z[k + 2] = Z_{az0+k}; blocks past the column's end read
                // real or zero table entries into sums that are not written
#pragma unroll
                for (int k = 0; k < kP2MBlk; ++k) {
                    if (k >= blk) break;
                    double v = fma(A0, Z[k + 2], acc[k]);
                    if (Q1 || Q2) v = fma(A1, Z[k + 1], v);
                    if (Q2) v = fma(A2, Z[k], v);
                    acc[k] = v;
                }
            }
        }
    }
    if (ngroups > 1) {
        __syncthreads();
        if (act && grp > 0)
#pragma unroll
            for (int k = 0; k < kP2MBlk; ++k)
                if (k < blk) gsum[((grp - 1) * nitems + item) * kP2MBlk + k] = acc[k];
        __syncthreads();
        if (act && grp == 0)
            for (int q = 1; q < ngroups; ++q)
#pragma unroll
                for (int k = 0; k < kP2MBlk; ++k)
                    if (k < blk) acc[k] += gsum[((q - 1) * nitems + item) * kP2MBlk + k];
    }
    if (act && grp == 0)
#pragma unroll
        for (int k = 0; k < kP2MBlk; ++k) {
            if (k >= nb) break;
            const int i = mindex(ax, ay, az0 + k);
            const size_t o = (size_t)c * nmp + (i - n0);
            M[o] = acc[k];
            if (M32) M32[o] = (float)acc[k];   // the copy the full-basis mixed-precision M2L reads
            row[i] = acc[k];
        }
    if (Mh32 || Mh64) {
        // the harmonic-basis row the M2L reads (in its precision)
        __syncthreads();
        const int h0 = hterms(S - 1), nh = hterms(p) - h0;
        for (int h = threadIdx.x; h < nh; h += kP2MThreads) {
            const double v = fold_component(row, h + h0);
            if (Mh32) Mh32[(size_t)c * nhp + h] = (float)v;
            else Mh64[(size_t)c * nhp + h] = v;
        }
    }
}

// harmonic-basis rows written beside M64 by P2M and M2M (null when unused)
struct HarmOut {
    int nhp;
    float *h32;
    double *h64;
};
static HarmOut harm_out(const fmm_tree *t)
{
    HarmOut o{0, nullptr, nullptr};
    if (t->basis != FMM_M2L_HARMONIC || !t->d_Mh) return o;
    o.nhp = t->nhp;
    if (t->prec == FMM_PREC_MIXED) o.h32 = (float *)t->d_Mh;
    else o.h64 = (double *)t->d_Mh;
    return o;
}

template <int MASK>
static void p2m_launch(fmm_tree *t, hipStream_t s)
{
    Geo g{{t->ht.lo[0], t->ht.lo[1], t->ht.lo[2]}, t->ht.h};
    const int nmp = (nterms(t->p) - nterms(t->order - 1) + 3) / 4 * 4;
    float *m32 = t->prec == FMM_PREC_MIXED ? t->d_M32 : nullptr;
    const HarmOut ho = harm_out(t);
    if constexpr (!(MASK & 4) || (MASK & 8)) {
        hipLaunchKernelGGL(p2m_coef_kernel<MASK>, dim3((unsigned)t->nleaves), dim3(kP2MThreads), 0, s, t->p, nmp,
                           t->d_leaves, t->d_cells, g, t->d_x, (int)t->ht.n, t->mom_user, t->d_perm, t->d_mom,
                           t->d_mom32, t->d_M64, m32, ho.nhp, ho.h32, ho.h64);
        return;
    }
    const int S = t->order;
    const int blk = kP2MPlanHost.blk[t->p][S], nitems = kP2MPlanHost.nitems[t->p][S];
    const int ngroups = kP2MPlanHost.ngroups[t->p][S];
    hipLaunchKernelGGL(p2m_kernel<MASK>, dim3((unsigned)t->nleaves), dim3(kP2MThreads), 0, s, t->p, nmp, blk, nitems,
                       ngroups, t->d_leaves,
                       t->d_cells, g, t->d_x, (int)t->ht.n, t->mom_user, t->d_perm, t->d_mom, t->d_mom32,
                       t->d_M64, m32, ho.nhp, ho.h32, ho.h64);
}

hipError_t launch_p2m(fmm_tree *t, hipStream_t s)
{
    switch (t->smask) {
    case 1: p2m_launch<1>(t, s); break;
    case 2: p2m_launch<2>(t, s); break;
    case 3: p2m_launch<3>(t, s); break;
    case 4: p2m_launch<4>(t, s); break;
    case 5: p2m_launch<5>(t, s); break;
    case 6: p2m_launch<6>(t, s); break;
    case 7: p2m_launch<7>(t, s); break;
    case 8: p2m_launch<8>(t, s); break;
    case 9: p2m_launch<9>(t, s); break;
    case 10: p2m_launch<10>(t, s); break;
    case 11: p2m_launch<11>(t, s); break;
    case 12: p2m_launch<12>(t, s); break;
    case 13: p2m_launch<13>(t, s); break;
    case 14: p2m_launch<14>(t, s); break;
    case 15: p2m_launch<15>(t, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ M2M / L2L
// Both shifts act per child octant sigma (child centre = parent centre +
// sigma r_child) and factorise over the axes, so each is applied as three 1-D
// passes over a coefficient row held in LDS.  One workgroup per parent cell:
// threadIdx.y = child slot (up to 8), threadIdx.x = coefficient slot; every
// thread keeps the multi-indices of its coefficients and its child's octant
// signs in registers, so the passes touch LDS only.
constexpr int kShiftX = 128;                     // coefficient slots per child
constexpr int kShiftItems = (nterms(kPTable) + kShiftX - 1) / kShiftX;

struct ShiftItems {
    int n;                                       // items owned by this thread
    int m[kShiftItems][3];
    int k[kShiftItems];
};

__device__ __forceinline__ void shift_items(int nt, ShiftItems &it)
{
    it.n = 0;
#pragma unroll
    for (int j = 0; j < kShiftItems; ++j) {
        const int i = threadIdx.x + j * kShiftX;
        const MultiIndex nn = k_mi.v[i < nt ? i : 0];
        it.m[j][0] = nn.x;
        it.m[j][1] = nn.y;
        it.m[j][2] = nn.z;
        it.k[j] = nn.k;
        if (i < nt) it.n = j + 1;
    }
}

// M~_n(P) = sum_children 2^-|n| sum_{k <= n} prod_d (-sigma_d)^k_d / k_d! M~_{n-k}(C)
// (Eq. 4 read with new-minus-old centre; radii halve from child to parent).
// Children are summed in octant order in FP64.
// (8 waves per SIMD: two 1024-thread workgroups fit a CU)
__global__ __launch_bounds__(kShiftX * 8, 8) void m2m_kernel(int p, int s, int nmp, const int32_t *__restrict__ parents,
                                                          const DevCell *__restrict__ cells, double *__restrict__ M,
                                                          float *__restrict__ M32, int nhp, float *__restrict__ Mh32,
                                                          double *__restrict__ Mh64)
{
    extern __shared__ double sm[];   // X[8][nt], Y[8][nt]
    const int nt = nterms(p), n0 = nterms(s - 1);
    double *X = sm, *Y = sm + 8 * nt;
    __shared__ double inv_fact[kPTable + 2];
    const int P = parents[blockIdx.x];
    const int nch = cells[P].nchild, kid0 = cells[P].child0;
    const int k = threadIdx.y;
    const int tid = threadIdx.y * kShiftX + threadIdx.x;
    if (tid <= kPTable + 1) {
        double f = 1.0;
        for (int a = 1; a <= tid; ++a) f *= k_inv.v[a];
        inv_fact[tid] = f;
    }
    ShiftItems it;
    shift_items(nt, it);
    double sg[3] = {1.0, 1.0, 1.0};   // -sigma_d
    if (k < nch) {
        const DevCell cc = cells[kid0 + k];
        sg[0] = (cc.ix & 1) ? -1.0 : 1.0;
        sg[1] = (cc.iy & 1) ? -1.0 : 1.0;
        sg[2] = (cc.iz & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int j = 0; j < kShiftItems; ++j) {
            if (j >= it.n) break;
            const int i = threadIdx.x + j * kShiftX;
            X[k * nt + i] = i < n0 ? 0.0 : M[(size_t)(kid0 + k) * nmp + (i - n0)];
        }
    }
    __syncthreads();
    // pass d: dst_n = sum_{a <= n_d} (-sigma_d)^a / a! src_{n - a e_d}
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *src = (d == 1 ? Y : X) + k * nt;
        double *dst = (d == 1 ? X : Y) + k * nt;
        if (k < nch) {
#pragma unroll
            for (int j = 0; j < kShiftItems; ++j) {
                if (j >= it.n) break;
                int mx = it.m[j][0], my = it.m[j][1], mz = it.m[j][2];
                const int nd = d == 0 ? mx : (d == 1 ? my : mz);
                double acc = 0.0, sp = 1.0;
                for (int a = 0; a <= nd; ++a) {
                    acc = fma(sp * inv_fact[a], src[mindex(mx, my, mz)], acc);
                    mx -= d == 0;
                    my -= d == 1;
                    mz -= d == 2;
                    sp *= sg[d];
                }
                dst[threadIdx.x + j * kShiftX] = acc;
            }
        }
        __syncthreads();
    }
    if (k == 0)
#pragma unroll
        for (int j = 0; j < kShiftItems; ++j) {
            if (j >= it.n) break;
            const int i = threadIdx.x + j * kShiftX;
            if (i < n0) continue;
            double acc = 0.0;
            for (int c = 0; c < nch; ++c) acc += Y[c * nt + i];
            const double v = ldexp(acc, -it.k[j]);
            M[(size_t)P * nmp + (i - n0)] = v;
            if (M32) M32[(size_t)P * nmp + (i - n0)] = (float)v;
            X[i] = v;   // X is free after the last pass
        }
    if (Mh32 || Mh64) {
        // the harmonic-basis row the M2L reads (in its precision)
        __syncthreads();
        const int h0 = hterms(s - 1), nh = hterms(p) - h0;
        for (int h = tid; h < nh; h += kShiftX * 8) {
            const double v = fold_component(X, h + h0);
            if (Mh32) Mh32[(size_t)P * nhp + h] = (float)v;
            else Mh64[(size_t)P * nhp + h] = v;
        }
    }
}

hipError_t launch_m2m_level(fmm_tree *t, int level, hipStream_t s)
{
    const int a = t->level_nonleaf_ptr[level], b = t->level_nonleaf_ptr[level + 1];
    if (b <= a) return hipSuccess;
    const int nmp = (nterms(t->p) - nterms(t->order - 1) + 3) / 4 * 4;
    const size_t lds = (size_t)16 * nterms(t->p) * sizeof(double);
    const HarmOut ho = harm_out(t);
    hipLaunchKernelGGL(m2m_kernel, dim3(b - a), dim3(kShiftX, 8), lds, s, t->p, t->order, nmp, t->d_nonleaf + a,
                       t->d_cells, t->d_M64, t->prec == FMM_PREC_MIXED ? t->d_M32 : nullptr, ho.nhp, ho.h32, ho.h64);
    return hipGetLastError();
}

// L~_n(C) += sum_{a: |n+a| <= q} prod_d sigma_d^a_d / a_d! * 2^-(|n+a|+1) L~_{n+a}(P)
// (Taylor shift of the local expansion to the child centre, in the
// normalised form).  The parent row is scaled once and shared by the
// children of the workgroup.
__global__ __launch_bounds__(kShiftX * 8, 8) void l2l_kernel(int q, const int32_t *__restrict__ parents,
                                                          const DevCell *__restrict__ cells, double *__restrict__ L)
{
    extern __shared__ double sm[];   // Pr[nl], X[8][nl], Y[8][nl]
    const int nl = nterms(q);
    double *Pr = sm, *X = sm + nl, *Y = sm + 9 * nl;
    __shared__ double inv_fact[kPTable + 2];
    const int P = parents[blockIdx.x];
    const int nch = cells[P].nchild, kid0 = cells[P].child0;
    const int k = threadIdx.y;
    const int tid = threadIdx.y * kShiftX + threadIdx.x;
    if (tid <= kPTable + 1) {
        double f = 1.0;
        for (int a = 1; a <= tid; ++a) f *= k_inv.v[a];
        inv_fact[tid] = f;
    }
    ShiftItems it;
    shift_items(nl, it);
    if (k == 0)
#pragma unroll
        for (int j = 0; j < kShiftItems; ++j) {
            if (j >= it.n) break;
            const int i = threadIdx.x + j * kShiftX;
            Pr[i] = ldexp(L[(size_t)P * nl + i], -(it.k[j] + 1));
        }
    double sg[3] = {1.0, 1.0, 1.0};   // sigma_d
    if (k < nch) {
        const DevCell cc = cells[kid0 + k];
        sg[0] = (cc.ix & 1) ? 1.0 : -1.0;
        sg[1] = (cc.iy & 1) ? 1.0 : -1.0;
        sg[2] = (cc.iz & 1) ? 1.0 : -1.0;
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *src = d == 0 ? Pr : (d == 1 ? Y : X) + k * nl;
        double *dst = (d == 1 ? X : Y) + k * nl;
        if (k < nch) {
#pragma unroll
            for (int j = 0; j < kShiftItems; ++j) {
                if (j >= it.n) break;
                int mx = it.m[j][0], my = it.m[j][1], mz = it.m[j][2];
                double acc = 0.0, sp = 1.0;
                for (int a = 0; a <= q - it.k[j]; ++a) {
                    acc = fma(sp * inv_fact[a], src[mindex(mx, my, mz)], acc);
                    mx += d == 0;
                    my += d == 1;
                    mz += d == 2;
                    sp *= sg[d];
                }
                dst[threadIdx.x + j * kShiftX] = acc;
            }
        }
        __syncthreads();
    }
    if (k < nch)
#pragma unroll
        for (int j = 0; j < kShiftItems; ++j) {
            if (j >= it.n) break;
            const int i = threadIdx.x + j * kShiftX;
            L[(size_t)(kid0 + k) * nl + i] += Y[k * nl + i];
        }
}

// children at `level` receive from their parents at level - 1
hipError_t launch_l2l_level(fmm_tree *t, int level, hipStream_t s)
{
    const int a = t->level_nonleaf_ptr[level - 1], b = t->level_nonleaf_ptr[level];
    if (b <= a) return hipSuccess;
    const int q = t->p - t->order;
    const size_t lds = (size_t)17 * nterms(q) * sizeof(double);
    hipLaunchKernelGGL(l2l_kernel, dim3(b - a), dim3(kShiftX, 8), lds, s, q, t->d_nonleaf + a, t->d_cells, t->d_L64);
    return hipGetLastError();
}


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
    const float *m32;       // 8 per particle
    const double *xs;       // SoA
    const double *m64;
    double *near;           // 4 per particle (phi, E)
    double *near_g;         // 6 per particle (field gradient), gradient kernels only
    int n;
    double h, lo[3];
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
// offset of the target leaf's own entry (-1 if absent).  Returns the number
// of staged sources of the window.
__device__ int p2p_window(const P2PArgs &a, const DevCell &cb, int b, int w0, int nw, int *wstart, int *wfirst,
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
    if (q < nw) wstart[q] = st;
    __syncthreads();
    if (q < nw && *wself == -2 - q) *wself = st;
    __syncthreads();
    return tot;
}

// entry of window source j: the last q with wstart[q] <= j
__device__ __forceinline__ int p2p_entry(const int *wstart, int nw, int j)
{
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if (wstart[m] <= j) lo = m;
        else hi = m - 1;
    }
    return lo;
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
    __shared__ double sbuf[3 * kPChunk32];
    double *const spx = sbuf, *const spy = sbuf + CH, *const spz = sbuf + 2 * CH;
    static_assert(NO * kPT <= 3 * kPChunk32, "reduction buffer exceeds the staging area");
    double (*const red)[kPT] = reinterpret_cast<double (*)[kPT]>(sbuf);
    __shared__ float4 spm[NV][CH];
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
            const int cstep = (CH / ns) * ns;
            for (int c0 = 0; c0 < nsw; c0 += cstep) {
                const int nc = min(cstep, nsw - c0);
                const int per = (nc + ns - 1) / ns;   // sources per slice
                __syncthreads();
                for (int j = tid; j < per * ns; j += kPT) {
                    if (j < nc) {
                        const int q = p2p_entry(wstart, nw, c0 + j);
                        const size_t pj = (size_t)wfirst[q] + (c0 + j - wstart[q]);
                        spx[j] = (a.xs[pj] - zb[0]) * irb;
                        spy[j] = (a.xs[n + pj] - zb[1]) * irb;
                        spz[j] = (a.xs[2 * n + pj] - zb[2]) * irb;
#pragma unroll
                        for (int v = 0; v < NV; ++v) spm[v][j] = m4[MW * pj + v];
                    } else {
                        spx[j] = spy[j] = spz[j] = 1.0e4;
#pragma unroll
                        for (int v = 0; v < NV; ++v) spm[v][j] = make_float4(0.f, 0.f, 0.f, 0.f);
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
                        const float rx = (float)(tx - spx[j]), ry = (float)(ty - spy[j]), rz = (float)(tz - spz[j]);
                        const float r2 = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, rz * rz));
                        const float inv = (decltype(check)::value && j == jself) ? 0.f : __builtin_amdgcn_rsqf(r2);
                        float4 mv[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) mv[v] = spm[v][j];
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

static hipError_t launch_p2p_range(fmm_tree *t, hipStream_t s, bool grad, int first, int count,
                                   double *near_g = nullptr);

hipError_t launch_p2p(fmm_tree *t, hipStream_t s, bool grad, double *near_g)
{
    return launch_p2p_range(t, s, grad, 0, -1, near_g);
}

hipError_t launch_p2p_part(fmm_tree *t, hipStream_t s, int first, int count)
{
    return launch_p2p_range(t, s, false, first, count);
}

// Near-field gradient of the allocation-free fmm_evaluate_grad variant: every
// particle's six values are written by the gradient pass before the L2P reads
// them, so nothing needs clearing between calls.  Calls that overlap on one
// device share it and race.
static __device__ __align__(256) double scratch[(size_t)kNoAllocMaxN * 6];

hipError_t noalloc_scratch(int device, double **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        // each device holds its own copy of the array; its host-side name is
        // no device address, so kernels get this one
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

static hipError_t launch_p2p_range(fmm_tree *t, hipStream_t s, bool grad, int first, int count, double *near_g)
{
    if (count < 0) count = (int)t->nleaves - first;
    if (first < 0 || count < 0 || first + count > t->nleaves) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    P2PArgs a;
    a.leaves = t->d_leaves;
    a.ptr = t->d_p2p_ptr;
    a.src = t->d_p2p_src;
    a.cells = t->d_cells;
    for (int d = 0; d < 3; ++d) a.lo[d] = t->ht.lo[d];
    a.m32 = t->d_mom32;
    a.xs = t->d_x;
    a.m64 = t->d_mom;
    a.near = t->d_near;
    a.near_g = near_g ? near_g : t->d_near_g;
    a.n = (int)t->ht.n;
    a.h = t->ht.h;
    a.order = t->d_p2p_order + first;
    const dim3 g((unsigned)count), bl(kPT);
    const bool f32 = t->prec == FMM_PREC_MIXED;
#define P2P_CASE(M)                                                                         \
    case M:                                                                                 \
        if (f32 && grad) hipLaunchKernelGGL((p2p_f32_kernel<M, true>), g, bl, 0, s, a);     \
        else if (f32) hipLaunchKernelGGL((p2p_f32_kernel<M, false>), g, bl, 0, s, a);       \
        else if (grad) hipLaunchKernelGGL((p2p_f64_kernel<M, true>), g, bl, 0, s, a);       \
        else hipLaunchKernelGGL((p2p_f64_kernel<M, false>), g, bl, 0, s, a);                \
        break;
    switch (t->smask) {
        P2P_CASE(1)
        P2P_CASE(2)
        P2P_CASE(3)
        P2P_CASE(4)
        P2P_CASE(5)
        P2P_CASE(6)
        P2P_CASE(7)
        P2P_CASE(8)
        P2P_CASE(9)
        P2P_CASE(10)
        P2P_CASE(11)
        P2P_CASE(12)
        P2P_CASE(13)
        P2P_CASE(14)
        P2P_CASE(15)
    default: return hipErrorInvalidValue;
    }
#undef P2P_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ L2P
// phi = (1/r) sum_{|n|<=q} eta^n/n! L~_n, E_d = -(1/r^2) sum eta^n/n! L~_{n+e_d}
// (Eq. 9, Eq. 10 with |k| = 1), eta = (x - z)/r, plus the near field, written
// to the caller's particle order.  One wave per pack of consecutive leaves
// holding at most 64 particles together (the host packs them, so that most
// lanes work although leaves hold ~ncrit/3 particles on average).  Each
// leaf's L~ is unpacked into LDS, zero beyond the simplex, so that for fixed
// (n_x, n_y) the sums over n_z of L~_n and of its neighbours n + e_d (+ e_d')
// are unit-stride from one base each; the loop structure is the same for
// every lane.  Two layouts (COLS):
// - a dense (q+2)^3 cube: the neighbours sit at fixed offsets from the base,
//   immediates of the LDS reads;
// - packed columns: for every (n_x, n_y) with n_x + n_y <= q + 2 the entries
//   n_z = 0 .. q + 2 - n_x - n_y lie contiguously, (q+3)(q+4)(q+5)/6 values,
//   a third of the cube, but each neighbour column costs an address add.
// The cube is used while every wave of the launch fits on the chip at once
// under its LDS share (100k particles), the columns when that share limits
// the resident waves (1M and more), where they are about 25 % faster.
// The leaves per pack are what a 16 KB budget of cubes allows in both cases.
// Compiled per q = p - s.
constexpr int kL2PMaxLeaves = 8;
constexpr int kL2PPackBudget = 16384;   // bytes of (q+2)^3 cubes that fix the leaves per pack

// values of one leaf's columns, and the start of column (x, y) (K = q + 3:
// column (x', y') holds K - x' - y' values)
__host__ __device__ constexpr int l2p_cols(int q) { return (q + 3) * (q + 4) * (q + 5) / 6; }
__host__ __device__ constexpr int l2p_col(int q, int x, int y)
{
    const int K = q + 3, kx = K - x;
    return K * (K + 1) * (K + 2) / 6 - kx * (kx + 1) * (kx + 2) / 6 + y * kx - y * (y - 1) / 2;
}
__host__ __device__ constexpr int l2p_cube(int q) { return (q + 2) * (q + 2) * (q + 2); }
int l2p_pack_limit(int q) { return std::max(1, std::min(kL2PMaxLeaves, kL2PPackBudget / (8 * l2p_cube(q)))); }
constexpr int kLdsPerCU = 160 * 1024;
bool l2p_columns_pay(int q, int npacks, int ncu)
{
    const int cube_bytes = l2p_pack_limit(q) * l2p_cube(q) * 8;
    return (int64_t)npacks > (int64_t)ncu * std::max(1, kLdsPerCU / cube_bytes);
}

// GRAD: also the field gradient, -(1/r^3) sum_{|n|<=q-2} eta^n/n! L~_{n+e_i+e_j}
// (the second derivatives of the expansion, the general-k form of Eq. 10),
// plus the near field's gradient; its sums read the same cube (indices stay
// inside the simplex, so no larger edge is needed)
template <int Q, bool GRAD, bool COLS>
__global__ __launch_bounds__(64) void l2p_kernel(int outputs, const int32_t *__restrict__ pack,
                                                 const int32_t *__restrict__ leaves, const DevCell *__restrict__ cells,
                                                 Geo g, const double *__restrict__ xs, int n,
                                                 const double *__restrict__ L, const double *__restrict__ near,
                                                 const int32_t *__restrict__ perm, double *__restrict__ phi,
                                                 double *__restrict__ field, const double *__restrict__ near_g,
                                                 double *__restrict__ grad)
{
    constexpr int NL = nterms(Q);
    constexpr int E = Q + 2;                     // cube edge: room for n + e_d
    constexpr int NC = COLS ? l2p_cols(Q) : E * E * E;   // values per leaf
    // start of the n_z run of (x, y)
    auto at = [](int x, int y) { return COLS ? l2p_col(Q, x, y) : (x * E + y) * E; };
    extern __shared__ double cubes[];            // one cube or set of columns per leaf of the pack
    __shared__ int lfirst[kL2PMaxLeaves], lstart[kL2PMaxLeaves + 1];
    __shared__ double lgeo[kL2PMaxLeaves][4];    // centre, 1 / radius
    const int p0 = pack[blockIdx.x], nlv = pack[blockIdx.x + 1] - p0;
    for (int i = threadIdx.x; i < nlv * NC; i += blockDim.x) cubes[i] = 0.0;
    if ((int)threadIdx.x < nlv) {
        const DevCell c = cells[leaves[p0 + threadIdx.x]];
        double z[3];
        cell_center(c, g.lo, g.h, z);
        lfirst[threadIdx.x] = c.first;
        lstart[threadIdx.x + 1] = c.count;
        lgeo[threadIdx.x][0] = z[0];
        lgeo[threadIdx.x][1] = z[1];
        lgeo[threadIdx.x][2] = z[2];
        lgeo[threadIdx.x][3] = 1.0 / cell_radius(c.level, g.h);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        lstart[0] = 0;
        for (int q = 0; q < nlv; ++q) lstart[q + 1] += lstart[q];
    }
    for (int q = 0; q < nlv; ++q) {
        const size_t c = (size_t)leaves[p0 + q];
        for (int i = threadIdx.x; i < NL; i += blockDim.x) {
            const MultiIndex nn = k_mi.v[i];
            cubes[q * NC + at(nn.x, nn.y) + nn.z] = L[c * NL + i];
        }
    }
    __syncthreads();
    const int tot = lstart[nlv];
    for (int k = threadIdx.x; k < tot; k += blockDim.x) {
        int q = 0;
        while (q + 1 < nlv && k >= lstart[q + 1]) ++q;
        const int i = lfirst[q] + (k - lstart[q]);
        const double *cube = cubes + q * NC;
        const double ir = lgeo[q][3];
        const double ex = (xs[i] - lgeo[q][0]) * ir, ey = (xs[n + i] - lgeo[q][1]) * ir,
                     ez = (xs[2 * (size_t)n + i] - lgeo[q][2]) * ir;
        double pz[Q + 1];
        pz[0] = 1.0;
#pragma unroll
        for (int a = 1; a <= Q; ++a) pz[a] = pz[a - 1] * ez * (1.0 / a);
        double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        double G[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // xx, xy, xz, yy, yz, zz
        double px = 1.0;
#pragma unroll 1
        for (int nx = 0; nx <= Q; ++nx) {
            if (nx) px *= ex * k_inv.v[nx];
            double py = px;
#pragma unroll 1
            for (int ny = 0; ny <= Q - nx; ++ny) {
                if (ny) py *= ey * k_inv.v[ny];
                // columns (nx, ny), (nx+1, ny), (nx, ny+1) and, for the
                // gradient, (nx+2, ny), (nx+1, ny+1), (nx, ny+2)
                const double *b = cube + at(nx, ny);
                const double *bx = cube + at(nx + 1, ny), *by = cube + at(nx, ny + 1);
                const int lim = Q - nx - ny;
                // entries beyond the simplex are zero, so the field sums may
                // run to the same bound as the potential sum
                double tp = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
                for (int nz = 0; nz <= Q; ++nz) {
                    if (nz > lim) break;
                    tp = fma(pz[nz], b[nz], tp);
                    tx = fma(pz[nz], bx[nz], tx);
                    ty = fma(pz[nz], by[nz], ty);
                    tz = fma(pz[nz], b[nz + 1], tz);
                }
                ph = fma(py, tp, ph);
                fx = fma(py, tx, fx);
                fy = fma(py, ty, fy);
                fz = fma(py, tz, fz);
                if constexpr (GRAD) {
                    double tg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    const double *bxx = cube + at(nx + 2, ny), *bxy = cube + at(nx + 1, ny + 1),
                                 *byy = cube + at(nx, ny + 2);
#pragma unroll
                    for (int nz = 0; nz + 2 <= Q; ++nz) {
                        if (nz > lim - 2) break;
                        tg[0] = fma(pz[nz], bxx[nz], tg[0]);
                        tg[1] = fma(pz[nz], bxy[nz], tg[1]);
                        tg[2] = fma(pz[nz], bx[nz + 1], tg[2]);
                        tg[3] = fma(pz[nz], byy[nz], tg[3]);
                        tg[4] = fma(pz[nz], by[nz + 1], tg[4]);
                        tg[5] = fma(pz[nz], b[nz + 2], tg[5]);
                    }
#pragma unroll
                    for (int c = 0; c < 6; ++c) G[c] = fma(py, tg[c], G[c]);
                }
            }
        }
        const double *nr = near + 4 * (size_t)i;
        const size_t o = (size_t)perm[i];
        if (outputs & FMM_POT) phi[o] = ph * ir + nr[0];
        if (outputs & FMM_FIELD) {
            const double ir2 = ir * ir;
            field[3 * o] = -fx * ir2 + nr[1];
            field[3 * o + 1] = -fy * ir2 + nr[2];
            field[3 * o + 2] = -fz * ir2 + nr[3];
        }
        if constexpr (GRAD) {
            const double ir3 = ir * ir * ir;
            const double *ng = near_g + 6 * (size_t)i;
#pragma unroll
            for (int c = 0; c < 6; ++c) grad[6 * o + c] = -G[c] * ir3 + ng[c];
        }
    }
}

template <int Q, bool COLS>
static void l2p_launch_layout(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s,
                              const double *near_g)
{
    Geo g{{t->ht.lo[0], t->ht.lo[1], t->ht.lo[2]}, t->ht.h};
    const size_t lds = (size_t)l2p_pack_limit(Q) * (COLS ? l2p_cols(Q) : l2p_cube(Q)) * sizeof(double);
    if constexpr (Q >= 2) {
        if (outputs & FMM_GRAD) {
            hipLaunchKernelGGL((l2p_kernel<Q, true, COLS>), dim3((unsigned)t->l2p_npacks), dim3(64), lds, s, outputs,
                               t->d_l2p_pack, t->d_leaves, t->d_cells, g, t->d_x, (int)t->ht.n, t->d_L64, t->d_near,
                               t->d_perm, phi, field, near_g, grad);
            return;
        }
    }
    hipLaunchKernelGGL((l2p_kernel<Q, false, COLS>), dim3((unsigned)t->l2p_npacks), dim3(64), lds, s, outputs,
                       t->d_l2p_pack, t->d_leaves, t->d_cells, g, t->d_x, (int)t->ht.n, t->d_L64, t->d_near, t->d_perm,
                       phi, field, nullptr, nullptr);
}

template <int Q>
static void l2p_launch(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s,
                       const double *near_g)
{
    if (t->l2p_columns) l2p_launch_layout<Q, true>(t, outputs, phi, field, grad, s, near_g);
    else l2p_launch_layout<Q, false>(t, outputs, phi, field, grad, s, near_g);
}

hipError_t launch_l2p_final(fmm_tree *t, int outputs, double *phi, double *field, double *grad, hipStream_t s,
                            const double *near_g)
{
    if ((outputs & FMM_GRAD) && t->p - t->order < 2) return hipErrorInvalidValue;
    if (!near_g) near_g = t->d_near_g;
    switch (t->p - t->order) {
    case 0: l2p_launch<0>(t, outputs, phi, field, grad, s, near_g); break;
    case 1: l2p_launch<1>(t, outputs, phi, field, grad, s, near_g); break;
    case 2: l2p_launch<2>(t, outputs, phi, field, grad, s, near_g); break;
    case 3: l2p_launch<3>(t, outputs, phi, field, grad, s, near_g); break;
    case 4: l2p_launch<4>(t, outputs, phi, field, grad, s, near_g); break;
    case 5: l2p_launch<5>(t, outputs, phi, field, grad, s, near_g); break;
    case 6: l2p_launch<6>(t, outputs, phi, field, grad, s, near_g); break;
    case 7: l2p_launch<7>(t, outputs, phi, field, grad, s, near_g); break;
    case 8: l2p_launch<8>(t, outputs, phi, field, grad, s, near_g); break;
    case 9: l2p_launch<9>(t, outputs, phi, field, grad, s, near_g); break;
    case 10: l2p_launch<10>(t, outputs, phi, field, grad, s, near_g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

