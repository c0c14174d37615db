// Derivatives of the potential of order K = 1..3 at every particle (Pepper &
// Fangohr, arXiv 2005.12351, Section 2: the derivatives of the potential of
// order |k| follow from the local expansion, Eq. 10; the near field adds the
// same derivatives of the pair potentials).  For each multi-index k with
// |k| = K, in the index order of that order:
//   FMM far:  d^k phi = r^-(K+1) sum_{|n| <= q-K} eta^n/n! L~_{n+k},
//             eta = (x - z)/r, q = p - s, L~ the normalised local of the leaf;
//   BH far:   d^k phi = r^-(K+1) sum_{s <= |n| <= p} M~_n D_{n+k}(u),
//             u = (x - z_A)/r, for every cell the particle accepts (Eq. 6
//             differentiated K times, the traversal of Eq. 12);
//   near:     d^k phi = sum_j sum_{|m|=s} S_m D_{m+k}(x - x_j), S the source
//             tensor S_m = (-1)^|m| T_m / m! of the physical moment T, D the
//             derivatives of 1/r (Eq. 6 applied to a point source's own
//             expansion).
// FP64 throughout, from the tree's FP64 expansions and sorted FP64 moments,
// in both precisions of the tree.  FMM: one workgroup per leaf, the leaf's
// local row staged in LDS, every thread one target walking the leaf's P2P
// list.  Barnes-Hut: one wavefront per particle; the wave walks the
// particle's traversal, builds an accepted cell's derivative tensor in LDS
// (one component per lane) and contracts it with the cell's multipole row
// (one term per lane), and splits an unaccepted leaf's sources over lanes.
#include "fmm_internal.h"

namespace {

constexpr int kDT = 64;   // threads per leaf

struct DerivArgs {
    const int32_t *leaves, *ptr, *src, *perm;
    const DevCell *cells;
    const double *xs;      // sorted positions, SoA
    const double *mom;     // sorted moments, w per particle
    const double *L;       // normalised locals, nl per cell (harmonic basis: nlh, the n_z <= 1 part)
    double *out;           // nk per particle, caller order
    int n, nl, nlh, q, w, smask;
    double h, lo[3];
};

// D_k(r) = d^k (1/|r|) by the Hermite form of the derivatives of f(r^2/2),
// f(u) = (2u)^-1/2:  d^k f = sum_{a <= k/2} prod_d c(k_d, a_d) x_d^(k_d-2a_d)
// f^(|k|-|a|)(u),  c(n, a) = n! / (2^a a! (n-2a)!),
// f^(j) = (-1)^j (2j-1)!! r^-(2j+1)
// c(n, a) for n <= FMM_P_MAX + 3 = 13, a <= 6
constexpr int kQMax = FMM_P_MAX + 3;
__constant__ double kHc[kQMax + 1][kQMax / 2 + 1] = {
    {1, 0, 0, 0, 0, 0, 0},           {1, 0, 0, 0, 0, 0, 0},
    {1, 1, 0, 0, 0, 0, 0},           {1, 3, 0, 0, 0, 0, 0},
    {1, 6, 3, 0, 0, 0, 0},           {1, 10, 15, 0, 0, 0, 0},
    {1, 15, 45, 15, 0, 0, 0},        {1, 21, 105, 105, 0, 0, 0},
    {1, 28, 210, 420, 105, 0, 0},    {1, 36, 378, 1260, 945, 0, 0},
    {1, 45, 630, 3150, 4725, 945, 0},  {1, 55, 990, 6930, 17325, 10395, 0},
    {1, 66, 1485, 13860, 51975, 62370, 10395},  {1, 78, 2145, 25740, 135135, 270270, 135135}};

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
// S_{e_i} = -mu_i, S_{e_i+e_j} = Q_ij / (e_i+e_j)!, S_m = -O_m / m! for an
// octupole), in the index order of that order
__device__ __forceinline__ void source_of(int s, const double *t, double (&S)[10])
{
    if (s == 3) {
        constexpr double kInvF[10] = {1.0 / 6, 0.5, 0.5, 0.5, 1.0, 0.5, 1.0 / 6, 0.5, 0.5, 1.0 / 6};
#pragma unroll
        for (int q = 0; q < 10; ++q) S[q] = -t[q] * kInvF[q];
    } else if (s == 0) {
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

// multi-index of position idx in the ordering by total order
__device__ __forceinline__ void mi_at(int idx, int &nx, int &ny, int &nz)
{
    int o = 0;
    while (nterms(o) <= idx) ++o;
    mi_of(o, idx - nterms(o - 1), nx, ny, nz);
}

// the K-th derivatives of the pair potentials of one source (every order
// its mask holds) at displacement (rx, ry, rz), added to acc
template <int K>
__device__ __forceinline__ void pair_derivs_add(double rx, double ry, double rz, const double *mj, int smask,
                                                const int (&kidx)[(K + 1) * (K + 2) / 2][3],
                                                double (&acc)[(K + 1) * (K + 2) / 2])
{
    constexpr int NK = (K + 1) * (K + 2) / 2;
    constexpr int Q = K + 3;                 // highest derivative order a pair needs (octupoles)
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
    int off = 0;
    for (int s = 0; s < 4; ++s) {
        if (!(smask & (1 << s))) continue;
        double S[10];
        source_of(s, mj + off, S);
        off += (s + 1) * (s + 2) / 2;
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

template <int K>
__global__ __launch_bounds__(kDT) void derivs_kernel(DerivArgs a)
{
    constexpr int NK = (K + 1) * (K + 2) / 2;
    __shared__ double sL[nterms(FMM_P_MAX)];
    const int lk = blockIdx.x;
    const int b = a.leaves[lk];
    const DevCell cb = a.cells[b];
    if (a.nlh > 0) {
        // harmonic basis: the row is rebuilt from its n_z <= 1 components,
        // (a, b, 2j + r) = (-1)^j sum_i C(j, i) (a + 2i, b + 2(j - i), r)
        const double *R = a.L + (size_t)b * a.nlh;
        for (int i = threadIdx.x; i < a.nl; i += kDT) {
            int nx, ny, nz;
            mi_at(i, nx, ny, nz);
            const int j = nz >> 1, r = nz & 1;
            double acc = 0.0, w = 1.0;
            for (int k = 0; k <= j; ++k) {
                acc = fma(w, R[hindex(nx + 2 * k, ny + 2 * (j - k), r)], acc);
                w = w * (j - k) / (k + 1);
            }
            sL[i] = (j & 1) ? -acc : acc;
        }
    } else {
        for (int i = threadIdx.x; i < a.nl; i += kDT) sL[i] = a.L[(size_t)b * a.nl + i];
    }
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
                pair_derivs_add<K>(rx, ry, rz, a.mom + (size_t)a.w * j, a.smask, kidx, acc);
            }
        }
        double *o = a.out + (size_t)NK * a.perm[i];
#pragma unroll
        for (int c = 0; c < NK; ++c) o[c] = acc[c];
    }
}

constexpr int kBW = 4;                                  // wavefronts (particles) per workgroup
constexpr int kDMax = nterms(kQMax);                    // derivative tensor to order p + K
constexpr int kBStack = 8 * (kMaxLevel + 3);

struct BHDerivArgs {
    const DevCell *cells;
    const double *xs;      // sorted positions, SoA
    const double *mom;     // sorted moments, w per particle
    const double *M;       // normalised multipoles, rows of nmp from order s (folded: harmonic order)
    const int32_t *perm;
    double *out;           // nk per particle, caller order
    int n, p, s, nmp, w, smask, folded;
    double theta2, h, lo[3];
};

__device__ __forceinline__ void wave_sync_d()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


template <int K>
__global__ __launch_bounds__(64 * kBW) void bh_derivs_kernel(BHDerivArgs a)
{
    constexpr int NK = (K + 1) * (K + 2) / 2;
    __shared__ double sD[kBW][kDMax];
    __shared__ double sPow[kBW][4][kQMax + 1];   // u_x^e, u_y^e, u_z^e and f^(e) at |u|
    __shared__ int stk[kBW][kBStack];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int i = blockIdx.x * kBW + wv;
    if (i >= a.n) return;   // the whole wavefront: it synchronises only with itself
    const size_t n = a.n;
    const double xi = a.xs[i], yi = a.xs[n + i], zi = a.xs[2 * n + i];
    int kidx[NK][3];
#pragma unroll
    for (int c = 0; c < NK; ++c) mi_of(K, c, kidx[c][0], kidx[c][1], kidx[c][2]);
    double acc[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) acc[c] = 0.0;
    const int Q = a.p + K;
    const int d0 = nterms(a.s + K - 1), d1 = nterms(Q);   // the derivative orders a contraction reads
    const int n0 = nterms(a.s - 1), n1 = nterms(a.p);
    double *D = sD[wv];
    if (lane == 0) stk[wv][0] = 0;
    int sp = 1;
    wave_sync_d();
    while (sp > 0) {
        --sp;
        const int c = stk[wv][sp];
        wave_sync_d();
        const DevCell cell = a.cells[c];
        // the acceptance test of Eq. 12 in the rounding sequence of the
        // Barnes-Hut evaluation kernel, so both accept the same cells
        const double rc = ldexp(1.0, kMaxLevel - cell.level);
        const double zx = __dadd_rn(a.lo[0], __dmul_rn((double)(2 * cell.ix + 1) * rc, a.h));
        const double zy = __dadd_rn(a.lo[1], __dmul_rn((double)(2 * cell.iy + 1) * rc, a.h));
        const double zz = __dadd_rn(a.lo[2], __dmul_rn((double)(2 * cell.iz + 1) * rc, a.h));
        const double r = __dmul_rn(rc, a.h);
        const double dx = __dsub_rn(xi, zx), dy = __dsub_rn(yi, zy), dz = __dsub_rn(zi, zz);
        const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        const bool inside = i >= cell.first && i < cell.first + cell.count;
        if (!inside && (__dmul_rn(r, r) < __dmul_rn(a.theta2, d2))) {
            const double ir = 1.0 / r;
            const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
            if (lane <= Q) {
                const double iu2 = 1.0 / (ux * ux + uy * uy + uz * uz);
                double px = 1.0, py = 1.0, pz = 1.0, F = sqrt(iu2);
                for (int e = 1; e <= lane; ++e) {
                    px *= ux;
                    py *= uy;
                    pz *= uz;
                    F *= -(2.0 * e - 1.0) * iu2;
                }
                sPow[wv][0][lane] = px;
                sPow[wv][1][lane] = py;
                sPow[wv][2][lane] = pz;
                sPow[wv][3][lane] = F;
            }
            wave_sync_d();
            const double *PX = sPow[wv][0], *PY = sPow[wv][1], *PZ = sPow[wv][2], *FF = sPow[wv][3];
            for (int idx = d0 + lane; idx < d1; idx += 64) {
                int kx, ky, kz;
                mi_at(idx, kx, ky, kz);
                const int kk = kx + ky + kz;
                double v = 0.0;
                for (int ax = 0; 2 * ax <= kx; ++ax) {
                    const double cx = kHc[kx][ax] * PX[kx - 2 * ax];
                    for (int ay = 0; 2 * ay <= ky; ++ay) {
                        const double cxy = cx * kHc[ky][ay] * PY[ky - 2 * ay];
                        for (int az = 0; 2 * az <= kz; ++az)
                            v = fma(cxy * kHc[kz][az] * PZ[kz - 2 * az], FF[kk - ax - ay - az], v);
                    }
                }
                D[idx] = v;
            }
            wave_sync_d();
            double tq[NK];
#pragma unroll
            for (int q = 0; q < NK; ++q) tq[q] = 0.0;
            // a folded row holds the m_z <= 1 components: D_{.+k} is
            // harmonic, so contracting them gives the same sums
            const int j0 = a.folded ? hterms(a.s - 1) : n0, j1 = a.folded ? hterms(a.p) : n1;
            const double *Mc = a.M + (size_t)c * a.nmp - j0;
            for (int j = j0 + lane; j < j1; j += 64) {
                int mx, my, mz;
                if (a.folded) hmulti(j, mx, my, mz);
                else mi_at(j, mx, my, mz);
                const double mv = Mc[j];
#pragma unroll
                for (int q = 0; q < NK; ++q)
                    tq[q] = fma(mv, D[mindex(mx + kidx[q][0], my + kidx[q][1], mz + kidx[q][2])], tq[q]);
            }
            double sc = ir;
#pragma unroll
            for (int e = 0; e < K; ++e) sc *= ir;
#pragma unroll
            for (int q = 0; q < NK; ++q) acc[q] = fma(tq[q], sc, acc[q]);
            wave_sync_d();   // D and sPow are rewritten by the next accepted cell
        } else if (cell.nchild == 0) {
            for (int j = cell.first + lane; j < cell.first + cell.count; j += 64) {
                if (j == i) continue;
                pair_derivs_add<K>(xi - a.xs[j], yi - a.xs[n + j], zi - a.xs[2 * n + j], a.mom + (size_t)a.w * j,
                                   a.smask, kidx, acc);
            }
        } else {
            // children in reverse, so that they are visited in octant order
            if (lane == 0)
                for (int k = cell.nchild - 1; k >= 0; --k) stk[wv][sp + (cell.nchild - 1 - k)] = cell.child0 + k;
            sp += cell.nchild;
            wave_sync_d();
        }
    }
#pragma unroll
    for (int q = 0; q < NK; ++q)
        for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_down(acc[q], o, 64);
    if (lane == 0) {
        double *o = a.out + (size_t)NK * a.perm[i];
#pragma unroll
        for (int q = 0; q < NK; ++q) o[q] = acc[q];
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
    a.nlh = t->basis == FMM_M2L_HARMONIC ? hterms(a.q) : 0;
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

hipError_t launch_bh_derivs(fmm_tree *t, int K, double *out, hipStream_t s)
{
    if (t->ht.n == 0) return hipSuccess;
    BHDerivArgs a;
    a.cells = t->d_cells;
    a.xs = t->d_x;
    a.mom = t->d_mom;
    a.folded = t->basis == FMM_M2L_HARMONIC;
    // the FP64 upward state: full rows, or folded ones in the harmonic basis
    a.M = a.folded ? (t->prec == FMM_PREC_MIXED ? t->d_Mf64 : (const double *)t->d_Mh) : t->d_M64;
    a.perm = t->d_perm;
    a.out = out;
    a.n = (int)t->ht.n;
    a.p = t->p;
    a.s = t->order;
    a.nmp = a.folded ? t->nhp : (nterms(t->p) - nterms(t->order - 1) + 3) / 4 * 4;
    a.w = mask_width(t->smask);
    a.smask = t->smask;
    a.theta2 = t->theta * t->theta;
    a.h = t->ht.h;
    for (int d = 0; d < 3; ++d) a.lo[d] = t->ht.lo[d];
    const dim3 g((unsigned)((t->ht.n + kBW - 1) / kBW)), bl(64 * kBW);
    switch (K) {
    case 1: hipLaunchKernelGGL(bh_derivs_kernel<1>, g, bl, 0, s, a); break;
    case 2: hipLaunchKernelGGL(bh_derivs_kernel<2>, g, bl, 0, s, a); break;
    case 3: hipLaunchKernelGGL(bh_derivs_kernel<3>, g, bl, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
