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
            if (M) M[o] = acc[k];              // full basis: the FP64 upward state
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
            if (Mh64) Mh64[(size_t)c * nhp + h] = v;
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
            if (M) M[o] = acc[k];              // full basis: the FP64 upward state
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
            if (Mh64) Mh64[(size_t)c * nhp + h] = v;
        }
    }
}

// harmonic-basis rows written by P2M and M2M (null when unused): the FP64
// folded rows (the upward state of that basis; in FP64 precision also what
// the M2L reads) and, in MIXED, their FP32 copy the M2L reads
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
    if (t->prec == FMM_PREC_MIXED) {
        o.h32 = (float *)t->d_Mh;
        o.h64 = t->d_Mf64;
    } else {
        o.h64 = (double *)t->d_Mh;
    }
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
// Children are summed in octant order in FP64.  Harmonic basis (M null): the
// children's folded rows Mh64, lifted with zeros at m_z >= 2, are shifted
// and the parent's row is folded again (the fold commutes with the shift:
// what it drops is r^2 times a lower row, which the shift keeps so).
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
            double v = 0.0;
            if (i >= n0) {
                if (M) v = M[(size_t)(kid0 + k) * nmp + (i - n0)];
                else if (it.m[j][2] <= 1)
                    v = Mh64[(size_t)(kid0 + k) * nhp + hindex(it.m[j][0], it.m[j][1], it.m[j][2]) - hterms(s - 1)];
            }
            X[k * nt + i] = v;
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
            if (M) M[(size_t)P * nmp + (i - n0)] = v;
            if (M32) M32[(size_t)P * nmp + (i - n0)] = (float)v;
            X[i] = v;   // X is free after the last pass
        }
    if (Mh32 || Mh64) {
        // the harmonic-basis rows: the FP64 state and the M2L's copy
        __syncthreads();
        const int h0 = hterms(s - 1), nh = hterms(p) - h0;
        for (int h = tid; h < nh; h += kShiftX * 8) {
            const double v = fold_component(X, h + h0);
            if (Mh32) Mh32[(size_t)P * nhp + h] = (float)v;
            if (Mh64) Mh64[(size_t)P * nhp + h] = v;
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

// (-1)^j C(j, i) for j <= FMM_P_MAX / 2: the weights that rebuild a
// harmonic row's component (a, b, 2j + r) from those with n_z <= 1
struct RebuildTable {
    double w[FMM_P_MAX / 2 + 1][FMM_P_MAX / 2 + 1];
};
constexpr RebuildTable make_rebuild()
{
    RebuildTable t{};
    for (int j = 0; j <= FMM_P_MAX / 2; ++j) {
        double c = 1.0;
        for (int i = 0; i <= j; ++i) {
            t.w[j][i] = (j & 1) ? -c : c;
            c = c * (j - i) / (i + 1);
        }
    }
    return t;
}
__constant__ RebuildTable k_rebuild = make_rebuild();

// rebuilt component (a, b, 2j + r) of a harmonic local row from its n_z <= 1
// components R (stride 1, harmonic order): (-1)^j sum_i C(j, i)
// R[(a + 2i, b + 2(j - i), r)]
__device__ __forceinline__ double rebuild_local(const double *R, int a, int b, int c)
{
    const int j = c >> 1, r = c & 1;
    double acc = 0.0;
    for (int i = 0; i <= j; ++i) acc = fma(k_rebuild.w[j][i], R[hindex(a + 2 * i, b + 2 * (j - i), r)], acc);
    return acc;
}

// L~_n(C) += sum_{a: |n+a| <= q} prod_d sigma_d^a_d / a_d! * 2^-(|n+a|+1) L~_{n+a}(P)
// (Taylor shift of the local expansion to the child centre, in the
// normalised form).  The parent row is scaled once and shared by the
// children of the workgroup.  Harmonic basis (nlh > 0): rows hold the n_z
// <= 1 components; the parent's row is rebuilt in LDS and only the
// children's n_z <= 1 components are updated (the shift keeps the row
// harmonic, so the others follow from them).
__global__ __launch_bounds__(kShiftX * 8, 8) void l2l_kernel(int q, int nlh, const int32_t *__restrict__ parents,
                                                          const DevCell *__restrict__ cells, double *__restrict__ L)
{
    extern __shared__ double sm[];   // Pr[nl], X[8][nl], Y[8][nl], R[nlh]
    const int nl = nterms(q);
    double *Pr = sm, *X = sm + nl, *Y = sm + 9 * nl, *R = sm + 17 * nl;
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
    if (nlh > 0) {
        for (int h = tid; h < nlh; h += kShiftX * 8) R[h] = L[(size_t)P * nlh + h];
        __syncthreads();
    }
    if (nlh > 0) {
        // the parent's row rebuilt by the whole workgroup
        for (int i = tid; i < nl; i += kShiftX * 8) {
            const MultiIndex nn = k_mi.v[i];
            Pr[i] = ldexp(rebuild_local(R, nn.x, nn.y, nn.z), -(nn.k + 1));
        }
    } else if (k == 0) {
#pragma unroll
        for (int j = 0; j < kShiftItems; ++j) {
            if (j >= it.n) break;
            const int i = threadIdx.x + j * kShiftX;
            Pr[i] = ldexp(L[(size_t)P * nl + i], -(it.k[j] + 1));
        }
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
    if (k < nch) {
        if (nlh > 0) {
            for (int h = threadIdx.x; h < nlh; h += kShiftX) {
                int a, b, c;
                hmulti(h, a, b, c);
                L[(size_t)(kid0 + k) * nlh + h] += Y[k * nl + mindex(a, b, c)];
            }
        } else {
#pragma unroll
            for (int j = 0; j < kShiftItems; ++j) {
                if (j >= it.n) break;
                const int i = threadIdx.x + j * kShiftX;
                L[(size_t)(kid0 + k) * nl + i] += Y[k * nl + i];
            }
        }
    }
}

// children at `level` receive from their parents at level - 1
hipError_t launch_l2l_level(fmm_tree *t, int level, hipStream_t s)
{
    const int a = t->level_nonleaf_ptr[level - 1], b = t->level_nonleaf_ptr[level];
    if (b <= a) return hipSuccess;
    const int q = t->p - t->order;
    const int nlh = t->basis == FMM_M2L_HARMONIC ? hterms(q) : 0;
    const size_t lds = (size_t)(17 * nterms(q) + nlh) * sizeof(double);
    hipLaunchKernelGGL(l2l_kernel, dim3(b - a), dim3(kShiftX, 8), lds, s, q, nlh, t->d_nonleaf + a, t->d_cells,
                       t->d_L64);
    return hipGetLastError();
}


#include "p2p_kernel.h"

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
    const bool f32 = t->prec == FMM_PREC_MIXED;
    if (!p2p_dispatch_lo(t->smask, f32, grad, (unsigned)count, s, a) &&
        !p2p_dispatch_oct(t->smask, f32, grad, (unsigned)count, s, a))
        return hipErrorInvalidValue;
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
// The columns are used when they pack more leaves into a wave than the cube
// (high orders, where one leaf's cube fills the 16 KB budget: at p - s = 9
// a cube is 10.6 KB and a wave would take one leaf of ~24 particles), or when
// the cube's LDS share limits the resident waves (1M particles and more,
// where they are about 25 % faster); the cube otherwise.  The leaves per pack
// are what a 16 KB budget of the layout allows.
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
int l2p_pack_limit(int q, bool cols)
{
    return std::max(1, std::min(kL2PMaxLeaves, kL2PPackBudget / (8 * (cols ? l2p_cols(q) : l2p_cube(q)))));
}
constexpr int kLdsPerCU = 160 * 1024;
bool l2p_columns_pay(int q, int npacks, int ncu)
{
    const int cube_bytes = l2p_pack_limit(q, false) * l2p_cube(q) * 8;
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
                                                 const double *__restrict__ L, int nlh,
                                                 const double *__restrict__ near, const int32_t *__restrict__ perm,
                                                 double *__restrict__ phi, double *__restrict__ field,
                                                 const double *__restrict__ near_g, double *__restrict__ grad)
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
        if (nlh > 0) {
            // harmonic basis: the n_z <= 1 components, the rest below
            for (int h = threadIdx.x; h < nlh; h += blockDim.x) {
                int a, b, z;
                hmulti(h, a, b, z);
                cubes[q * NC + at(a, b) + z] = L[c * nlh + h];
            }
        } else {
            for (int i = threadIdx.x; i < NL; i += blockDim.x) {
                const MultiIndex nn = k_mi.v[i];
                cubes[q * NC + at(nn.x, nn.y) + nn.z] = L[c * NL + i];
            }
        }
    }
    if (nlh > 0) {
        // (a, b, 2j + r) = (-1)^j sum_i C(j, i) (a + 2i, b + 2(j - i), r):
        // reads only n_z <= 1 entries, writes only n_z >= 2 ones
        __syncthreads();
        for (int it = threadIdx.x; it < nlv * NL; it += blockDim.x) {
            const int q = it / NL;
            const MultiIndex nn = k_mi.v[it % NL];
            if (nn.z < 2) continue;
            double *cube = cubes + q * NC;
            const int j = nn.z >> 1, r = nn.z & 1;
            double acc = 0.0;
            for (int i = 0; i <= j; ++i) acc = fma(k_rebuild.w[j][i], cube[at(nn.x + 2 * i, nn.y + 2 * (j - i)) + r], acc);
            cube[at(nn.x, nn.y) + nn.z] = acc;
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
    const size_t lds = (size_t)l2p_pack_limit(Q, COLS) * (COLS ? l2p_cols(Q) : l2p_cube(Q)) * sizeof(double);
    const int nlh = t->basis == FMM_M2L_HARMONIC ? hterms(Q) : 0;
    if constexpr (Q >= 2) {
        if (outputs & FMM_GRAD) {
            hipLaunchKernelGGL((l2p_kernel<Q, true, COLS>), dim3((unsigned)t->l2p_npacks), dim3(64), lds, s, outputs,
                               t->d_l2p_pack, t->d_leaves, t->d_cells, g, t->d_x, (int)t->ht.n, t->d_L64, nlh,
                               t->d_near, t->d_perm, phi, field, near_g, grad);
            return;
        }
    }
    hipLaunchKernelGGL((l2p_kernel<Q, false, COLS>), dim3((unsigned)t->l2p_npacks), dim3(64), lds, s, outputs,
                       t->d_l2p_pack, t->d_leaves, t->d_cells, g, t->d_x, (int)t->ht.n, t->d_L64, nlh, t->d_near,
                       t->d_perm, phi, field, nullptr, nullptr);
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

