// Derivatives of the potential of order K = 1..3 at every particle (Pepper &
// Fangohr, arXiv 2005.12351, Section 2: the derivatives of the potential of
// order |k| follow from the local expansion, Eq. 10; the near field adds the
// same derivatives of the pair potentials).  For each multi-index k with
// |k| = K, in the index order of that order:
//   far:  d^k phi = r^-(K+1) sum_{|n| <= q-K} eta^n/n! L~_{n+k},
//         eta = (x - z)/r, q = p - s, L~ the normalised local of the leaf;
//   near: d^k phi = sum_j sum_{|m|=s} S_m D_{m+k}(x - x_j), S the source
//         tensor S_m = (-1)^|m| T_m / m! of the physical moment T, D the
//         derivatives of 1/r (Eq. 6 applied to a point source's own
//         expansion).
// FP64 throughout, from the tree's FP64 locals and sorted FP64 moments, in
// both precisions of the tree.  One workgroup per leaf: the leaf's local row
// is staged in LDS and every thread (one target) walks the leaf's P2P list.
#include "fmm_internal.h"

namespace {

constexpr int kDT = 64;   // threads per leaf

struct DerivArgs {
    const int32_t *leaves, *ptr, *src, *perm;
    const DevCell *cells;
    const double *xs;      // sorted positions, SoA
    const double *mom;     // sorted moments, w per particle
    const double *L;       // normalised locals, nl per cell
    double *out;           // nk per particle, caller order
    int n, nl, q, w, smask;
    double h, lo[3];
};

// D_k(r) = d^k (1/|r|) by the Hermite form of the derivatives of f(r^2/2),
// f(u) = (2u)^-1/2:  d^k f = sum_{a <= k/2} prod_d c(k_d, a_d) x_d^(k_d-2a_d)
// f^(|k|-|a|)(u),  c(n, a) = n! / (2^a a! (n-2a)!),
// f^(j) = (-1)^j (2j-1)!! r^-(2j+1)
// c(n, a) for n <= 7, a <= 3
__constant__ double kHc[8][4] = {{1, 0, 0, 0},   {1, 0, 0, 0},    {1, 1, 0, 0},     {1, 3, 0, 0},
                                 {1, 6, 3, 0},   {1, 10, 15, 0},  {1, 15, 45, 15},  {1, 21, 105, 105}};

__device__ __forceinline__ double hcoef(int n, int a) { return kHc[n][a]; }

template <int Q>
__device__ __forceinline__ double dtensor_k(int kx, int ky, int kz, const double (&px)[Q + 1],
                                            const double (&py)[Q + 1], const double (&pz)[Q + 1],
                                            const double (&F)[Q + 1])
{
    double acc = 0.0;
    const int kk = kx + ky + kz;
    for (int ax = 0; 2 * ax <= kx; ++ax)
        for (int ay = 0; 2 * ay <= ky; ++ay)
            for (int az = 0; 2 * az <= kz; ++az)
                acc += hcoef(kx, ax) * hcoef(ky, ay) * hcoef(kz, az) * px[kx - 2 * ax] * py[ky - 2 * ay] *
                       pz[kz - 2 * az] * F[kk - ax - ay - az];
    return acc;
}

// the source tensor of one order from its physical moments (S_0 = q,
// S_{e_i} = -mu_i, S_{e_i+e_j} = Q_ij / (e_i+e_j)!), in the index order of
// that order
__device__ __forceinline__ void source_of(int s, const double *t, double (&S)[6])
{
    if (s == 0) {
        S[0] = t[0];
    } else if (s == 1) {
        S[0] = -t[0];
        S[1] = -t[1];
        S[2] = -t[2];
    } else {   // (2,0,0) (1,1,0) (1,0,1) (0,2,0) (0,1,1) (0,0,2)
        S[0] = 0.5 * t[0];
        S[1] = t[1];
        S[2] = t[2];
        S[3] = 0.5 * t[3];
        S[4] = t[4];
        S[5] = 0.5 * t[5];
    }
}

// multi-index number c of order K in the index order (n_x descending, then n_y)
__device__ __forceinline__ void mi_of(int K, int c, int &nx, int &ny, int &nz)
{
    nx = K;
    int left = c;
    while (left > K - nx) {
        left -= K - nx + 1;
        --nx;
    }
    ny = K - nx - left;
    nz = K - nx - ny;
}

template <int K>
__global__ __launch_bounds__(kDT) void derivs_kernel(DerivArgs a)
{
    constexpr int NK = (K + 1) * (K + 2) / 2;
    constexpr int Q = K + 2;                 // highest derivative order a pair needs (quadrupoles)
    __shared__ double sL[nterms(FMM_P_MAX)];
    const int lk = blockIdx.x;
    const int b = a.leaves[lk];
    const DevCell cb = a.cells[b];
    for (int i = threadIdx.x; i < a.nl; i += kDT) sL[i] = a.L[(size_t)b * a.nl + i];
    __syncthreads();
    const double r = ldexp(1.0, kMaxLevel - cb.level) * a.h;
    const double zb[3] = {a.lo[0] + (double)(2 * cb.ix + 1) * r, a.lo[1] + (double)(2 * cb.iy + 1) * r,
                          a.lo[2] + (double)(2 * cb.iz + 1) * r};
    const size_t n = a.n;
    int kidx[NK][3];
#pragma unroll
    for (int c = 0; c < NK; ++c) mi_of(K, c, kidx[c][0], kidx[c][1], kidx[c][2]);
    for (int t = threadIdx.x; t < cb.count; t += kDT) {
        const int i = cb.first + t;
        const double x = a.xs[i], y = a.xs[n + i], z = a.xs[2 * n + i];
        double acc[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) acc[c] = 0.0;
        // far field: Eq. 10 on the normalised local
        if (K <= a.q) {
            const double e[3] = {(x - zb[0]) / r, (y - zb[1]) / r, (z - zb[2]) / r};
            const int qk = a.q - K;
            double ax = 1.0;
            for (int nx = 0; nx <= qk; ++nx) {
                double ay = ax;
                for (int ny = 0; nx + ny <= qk; ++ny) {
                    double az = ay;
                    for (int nz = 0; nx + ny + nz <= qk; ++nz) {
#pragma unroll
                        for (int c = 0; c < NK; ++c)
                            acc[c] = fma(az, sL[mindex(nx + kidx[c][0], ny + kidx[c][1], nz + kidx[c][2])], acc[c]);
                        az *= e[2] / (nz + 1);
                    }
                    ay *= e[1] / (ny + 1);
                }
                ax *= e[0] / (nx + 1);
            }
            const double sc = pow(r, -(double)(K + 1));
#pragma unroll
            for (int c = 0; c < NK; ++c) acc[c] *= sc;
        }
        // near field: every source of the leaf's P2P list but the target
        for (int e = a.ptr[lk]; e < a.ptr[lk + 1]; ++e) {
            const DevCell cs = a.cells[a.src[e]];
            for (int j = cs.first; j < cs.first + cs.count; ++j) {
                if (j == i) continue;
                const double rx = x - a.xs[j], ry = y - a.xs[n + j], rz = z - a.xs[2 * n + j];
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double ir = 1.0 / sqrt(r2), ir2 = ir * ir;
                double px[Q + 1], py[Q + 1], pz[Q + 1], F[Q + 1];
                px[0] = py[0] = pz[0] = 1.0;
                F[0] = ir;
#pragma unroll
                for (int d = 1; d <= Q; ++d) {
                    px[d] = px[d - 1] * rx;
                    py[d] = py[d - 1] * ry;
                    pz[d] = pz[d - 1] * rz;
                    F[d] = -F[d - 1] * (2.0 * d - 1.0) * ir2;
                }
                const double *mj = a.mom + (size_t)a.w * j;
                int off = 0;
                for (int s = 0; s < 3; ++s) {
                    if (!(a.smask & (1 << s))) continue;
                    double S[6];
                    source_of(s, mj + off, S);
                    off += s == 0 ? 1 : (s == 1 ? 3 : 6);
                    const int nm = (s + 1) * (s + 2) / 2;
                    for (int mi = 0; mi < nm; ++mi) {
                        int mx, my, mz;
                        mi_of(s, mi, mx, my, mz);
#pragma unroll
                        for (int c = 0; c < NK; ++c)
                            acc[c] = fma(S[mi], dtensor_k<Q>(mx + kidx[c][0], my + kidx[c][1], mz + kidx[c][2], px, py, pz, F),
                                         acc[c]);
                    }
                }
            }
        }
        double *o = a.out + (size_t)NK * a.perm[i];
#pragma unroll
        for (int c = 0; c < NK; ++c) o[c] = acc[c];
    }
}

}  // namespace

hipError_t launch_derivs(fmm_tree *t, int K, double *out, hipStream_t s)
{
    if (t->nleaves == 0) return hipSuccess;
    DerivArgs a;
    a.leaves = t->d_leaves;
    a.ptr = t->d_p2p_ptr;
    a.src = t->d_p2p_src;
    a.perm = t->d_perm;
    a.cells = t->d_cells;
    a.xs = t->d_x;
    a.mom = t->d_mom;
    a.L = t->d_L64;
    a.out = out;
    a.n = (int)t->ht.n;
    a.q = t->p - t->order;
    a.nl = nterms(a.q);
    a.w = mask_width(t->smask);
    a.smask = t->smask;
    a.h = t->ht.h;
    for (int d = 0; d < 3; ++d) a.lo[d] = t->ht.lo[d];
    const dim3 g((unsigned)t->nleaves), bl(kDT);
    switch (K) {
    case 1: hipLaunchKernelGGL(derivs_kernel<1>, g, bl, 0, s, a); break;
    case 2: hipLaunchKernelGGL(derivs_kernel<2>, g, bl, 0, s, a); break;
    case 3: hipLaunchKernelGGL(derivs_kernel<3>, g, bl, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
