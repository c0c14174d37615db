/*
 * Plain CPU reference ("oracle") for the Cartesian Fast Multipole and
 * multipolar Barnes-Hut method of Pepper & Fangohr, "fmmgen: Automatic Code
 * Generation of Operators for Cartesian Fast Multipole and Barnes-Hut
 * Methods" (arXiv 2005.12351).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or generator with the GPU library; the GPU path never calls
 * it.  Everything is IEEE double, written for readability, not speed
 * (OpenMP only over independent targets, so results do not depend on the
 * thread count).  Build with -ffp-contract=off.
 *
 * Conventions (the readings of the paper that both implementations follow):
 *  - kernel 1/|r| with no 1/(4 pi) factor (Section 2, Eq. 1);
 *  - field E = -grad(phi);
 *  - multi-indices ordered by total order, then n_x descending, then n_y
 *    descending (Section 3.1 lists the first terms of this order);
 *  - the source tensor of a point source of order s is
 *    S_n = (-1)^|n| T_n / n!, T the physical moment (q; mu; Q_ij), which is
 *    Eq. 3 applied to the source's own charge distribution;
 *  - P2M: M_n(z) = sum_{sigma<=n, |sigma|=s} (z-x)^(n-sigma)/(n-sigma)! S_sigma
 *    (Eq. 5), M2M: M_n(z') = sum_{k<=n} (z'-z)^k/k! M_{n-k}(z) (Eq. 4, with
 *    the shift taken as new-minus-old centre, as Eq. 3 implies);
 *  - M2L: L_n = sum_m M_m D_{n+m}(z_B - z_A), s<=|m|<=p-|n|, |n|<=p-s (Eq. 8,
 *    the form the printed p=1 operator uses), D_k = d^k (1/|r|);
 *  - L2L: L_n(z') = sum_{k>=n,|k|<=p-s} (z'-z)^(k-n)/(k-n)! L_k(z);
 *  - L2P: phi = sum_{|n|<=p-s} (x-z)^n/n! L_n, derivatives by Eq. 10;
 *  - M2P: phi = sum_{s<=|n|<=p} M_n D_n(x - z_A) (Eq. 6 without the
 *    duplicated factors), E_i = -sum M_n D_{n+e_i};
 *  - tree: cube root box, 21 bits per axis, Morton key with x as the most
 *    significant bit of each octal digit, stable sort, split while
 *    count > ncrit (depth cap 21), geometric cell centres (Section 3.2);
 *  - cell radius = half the side; FMM acceptance (r_A + r_B) < theta R
 *    (Eq. 13), BH acceptance r_A < theta |x - z_A| (Eq. 12), both strict;
 *    a BH cell that contains the target particle is always opened;
 *  - dual-tree traversal splits the larger cell, both on a tie.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXLEVEL 21

/* ------------------------------------------------------------------ */
/* Multi-index algebra (Section 2)                                      */
/* ------------------------------------------------------------------ */

int orc_nterms(int p) { return p < 0 ? 0 : (p + 1) * (p + 2) * (p + 3) / 6; }

/* position of n = (nx,ny,nz) in the ordering by total order, then nx
 * descending, then ny descending */
int orc_index(int nx, int ny, int nz)
{
    int k = nx + ny + nz;
    int a = k - nx;                 /* = ny + nz */
    return k * (k + 1) * (k + 2) / 6 + a * (a + 1) / 2 + nz;
}

/* multi-index of every position, filled once when the library loads */
#define ORC_TABLE_P 30
static int mi_table[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) * (ORC_TABLE_P + 3) / 6][3];

__attribute__((constructor)) static void fill_mi_table(void)
{
    for (int k = 0; k <= ORC_TABLE_P; ++k)
        for (int nx = k; nx >= 0; --nx)
            for (int ny = k - nx; ny >= 0; --ny) {
                int i = orc_index(nx, ny, k - nx - ny);
                mi_table[i][0] = nx;
                mi_table[i][1] = ny;
                mi_table[i][2] = k - nx - ny;
            }
}

void orc_multi_index(int idx, int *n)
{
    n[0] = mi_table[idx][0];
    n[1] = mi_table[idx][1];
    n[2] = mi_table[idx][2];
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* r^n / n! for all |n| <= p */
static void monomials(int p, const double *r, double *out)
{
    int nt = orc_nterms(p);
    for (int i = 0; i < nt; ++i) {
        int n[3];
        orc_multi_index(i, n);
        out[i] = ipow(r[0], n[0]) * ipow(r[1], n[1]) * ipow(r[2], n[2]) /
                 (factorial(n[0]) * factorial(n[1]) * factorial(n[2]));
    }
}

/* ------------------------------------------------------------------ */
/* Derivatives of the Green's function (Section 3.1, Eq. 11 context)    */
/* ------------------------------------------------------------------ */

/* D_k = d^k (1/|r|) for all |k| <= q.  Written from r^2 d_i(1/r) = -r_i/r
 * differentiated with Leibniz' rule and symmetrised over the axes:
 *   |k| r^2 D_k = -(2|k|-1) sum_j k_j r_j D_{k-e_j}
 *                 -(|k|-1) sum_j k_j (k_j-1) D_{k-2e_j}.
 * This is not one of the recursions the paper cites, on purpose. */
void orc_dtensor(int q, double x, double y, double z, double *D)
{
    double r[3] = {x, y, z};
    double r2 = x * x + y * y + z * z;
    D[0] = 1.0 / sqrt(r2);
    for (int k = 1; k <= q; ++k)
        for (int nx = k; nx >= 0; --nx)
            for (int ny = k - nx; ny >= 0; --ny) {
                int n[3] = {nx, ny, k - nx - ny};
                double s1 = 0.0, s2 = 0.0;
                for (int j = 0; j < 3; ++j) {
                    if (n[j] >= 1) {
                        int m[3] = {n[0], n[1], n[2]};
                        m[j] -= 1;
                        s1 += n[j] * r[j] * D[orc_index(m[0], m[1], m[2])];
                    }
                    if (n[j] >= 2) {
                        int m[3] = {n[0], n[1], n[2]};
                        m[j] -= 2;
                        s2 += (double)n[j] * (n[j] - 1) * D[orc_index(m[0], m[1], m[2])];
                    }
                }
                D[orc_index(n[0], n[1], n[2])] = (-(2.0 * k - 1.0) * s1 - (k - 1.0) * s2) / (k * r2);
            }
}

/* ------------------------------------------------------------------ */
/* Direct interaction of point sources (Eq. 1 and its derivatives)      */
/* ------------------------------------------------------------------ */

/* ------------------------------------------------------------------ */
/* Source order codes                                                    */
/* ------------------------------------------------------------------ */
/* A code is a single source order (0 charge, 1 dipole, 2 quadrupole,
 * 3 octupole) or
 * ORC_MIXED plus a bit mask of the orders present in one system (bit k:
 * order k).  A moment row then holds the physical moments of the present
 * orders, in ascending order, concatenated.  Every operator is linear in the
 * source, so a mixed source acts as the sum of its single-order parts; the
 * expansions start at the lowest order present (Section 2). */
#define ORC_MIXED 16

static int code_mask(int o) { return o >= ORC_MIXED ? o - ORC_MIXED : 1 << o; }
static int width_of(int order) { return (order + 1) * (order + 2) / 2; }
static int mom_width(int o)
{
    int m = code_mask(o), w = 0;
    for (int k = 0; k < 4; ++k)
        if (m & (1 << k)) w += width_of(k);
    return w;
}
int orc_min_order(int o)
{
    int m = code_mask(o);
    return (m & 1) ? 0 : ((m & 2) ? 1 : ((m & 4) ? 2 : 3));
}
int orc_code_valid(int o)
{
    return (o >= 0 && o <= 3) || (o > ORC_MIXED && o < ORC_MIXED + 16);
}

/* the full symmetric octupole tensor O_ijk from its ten components, stored
 * in the index order of order 3 (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz) */
static void octupole_tensor(const double *mom, double O[3][3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                int c[3] = {0, 0, 0};
                c[i]++;
                c[j]++;
                c[k]++;
                O[i][j][k] = mom[orc_index(c[0], c[1], c[2]) - orc_nterms(2)];
            }
}

/* potential and field at a target displaced by r = x_target - x_source from
 * a source of one order with physical moment mom */
static void pair_single(int order, const double *r, const double *mom, double *phi, double *E)
{
    if (order == 3) {
        /* phi = -(1/6) sum_ijk O_ijk d_i d_j d_k (1/r)
         *     = 5/2 O(r,r,r) / r^7 - 3/2 (t.r) / r^5,   t_k = sum_i O_iik;
         * E = -grad phi = -15/2 V / r^7 + 35/2 O(r,r,r) r / r^9
         *                 + 3/2 t / r^5 - 15/2 (t.r) r / r^7,
         * V_k = sum_ij O_ijk r_i r_j */
        double O[3][3][3], V[3] = {0, 0, 0}, t[3] = {0, 0, 0};
        octupole_tensor(mom, O);
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) {
                t[k] += O[i][i][k];
                for (int j = 0; j < 3; ++j) V[k] += O[i][j][k] * r[i] * r[j];
            }
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double rinv = 1.0 / sqrt(r2);
        double r5 = rinv * rinv * rinv * rinv * rinv, r7 = r5 * rinv * rinv, r9 = r7 * rinv * rinv;
        double C = V[0] * r[0] + V[1] * r[1] + V[2] * r[2];
        double tr = t[0] * r[0] + t[1] * r[1] + t[2] * r[2];
        *phi = 2.5 * C * r7 - 1.5 * tr * r5;
        for (int k = 0; k < 3; ++k) E[k] = -7.5 * V[k] * r7 + 17.5 * C * r[k] * r9 + 1.5 * t[k] * r5 - 7.5 * tr * r[k] * r7;
        return;
    }
    double x = r[0], y = r[1], z = r[2];
    double r2 = x * x + y * y + z * z;
    double rinv = 1.0 / sqrt(r2);
    double r3 = rinv * rinv * rinv;
    if (order == 0) {
        double q = mom[0];
        *phi = q * rinv;
        E[0] = q * x * r3;
        E[1] = q * y * r3;
        E[2] = q * z * r3;
    } else if (order == 1) {
        /* phi = mu.r / r^3 ; E = (3 (mu.r) r - r^2 mu) / r^5 */
        double mr = mom[0] * x + mom[1] * y + mom[2] * z;
        double r5 = r3 * rinv * rinv;
        *phi = mr * r3;
        E[0] = (3.0 * mr * x - r2 * mom[0]) * r5;
        E[1] = (3.0 * mr * y - r2 * mom[1]) * r5;
        E[2] = (3.0 * mr * z - r2 * mom[2]) * r5;
    } else {
        /* phi = 1/2 sum_ij Q_ij d_i d_j (1/r) = (3 r.Q.r - r^2 tr Q) / (2 r^5)
         * E   = 15/2 (r.Q.r) r / r^7 - 3 Q r / r^5 - 3/2 tr Q r / r^5 */
        double qxx = mom[0], qxy = mom[1], qxz = mom[2], qyy = mom[3], qyz = mom[4], qzz = mom[5];
        double Qr[3] = {qxx * x + qxy * y + qxz * z, qxy * x + qyy * y + qyz * z,
                        qxz * x + qyz * y + qzz * z};
        double rQr = x * Qr[0] + y * Qr[1] + z * Qr[2];
        double tr = qxx + qyy + qzz;
        double r5 = r3 * rinv * rinv;
        double r7 = r5 * rinv * rinv;
        *phi = 0.5 * (3.0 * rQr - r2 * tr) * r5;
        E[0] = 7.5 * rQr * x * r7 - 3.0 * Qr[0] * r5 - 1.5 * tr * x * r5;
        E[1] = 7.5 * rQr * y * r7 - 3.0 * Qr[1] * r5 - 1.5 * tr * y * r5;
        E[2] = 7.5 * rQr * z * r7 - 3.0 * Qr[2] * r5 - 1.5 * tr * z * r5;
    }
}

/* the same for a source of any order code: the sum over its parts */
void orc_p2p_pair(int o, const double *r, const double *mom, double *phi, double *E)
{
    int m = code_mask(o), off = 0;
    *phi = 0.0;
    E[0] = E[1] = E[2] = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (!(m & (1 << k))) continue;
        double ph, e[3];
        pair_single(k, r, mom + off, &ph, e);
        *phi += ph;
        E[0] += e[0];
        E[1] += e[1];
        E[2] += e[2];
        off += width_of(k);
    }
}

/* Field gradient G_ij = d_i E_j = -d_i d_j phi (symmetric; stored xx, xy,
 * xz, yy, yz, zz) at a target displaced by r from a source of one order: the
 * second derivatives of the closed forms above (Section 2 asks for
 * derivatives of the potential of any order; order 2 is the one after the
 * field).
 *   charge:     q (delta_ij r^2 - 3 r_i r_j) / r^5
 *   dipole:     3 (mu_i r_j + mu_j r_i + (mu.r) delta_ij) / r^5
 *               - 15 (mu.r) r_i r_j / r^7
 *   quadrupole: phi = A + B, A = 3/2 (r.Q.r) / r^5, B = -tr Q / (2 r^3);
 *     d_i d_j A = 3 Q_ij / r^5 - 15 ((Qr)_i r_j + (Qr)_j r_i) / r^7
 *                 - 15/2 (r.Q.r) delta_ij / r^7 + 105/2 (r.Q.r) r_i r_j / r^9
 *     d_i d_j B = 3/2 tr Q (delta_ij / r^5 - 5 r_i r_j / r^7)          */
static void pair_grad_single(int order, const double *r, const double *mom, double *G)
{
    static const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rinv = 1.0 / sqrt(r2);
    double r3 = rinv * rinv * rinv, r5 = r3 * rinv * rinv, r7 = r5 * rinv * rinv, r9 = r7 * rinv * rinv;
    if (order == 3) {
        /* octupole, phi = 5/2 C / r^7 - 3/2 (t.r) / r^5 with C = O(r,r,r),
         * W_ij = sum_k O_ijk r_k, V = W r:
         *   d_i d_j (C / r^7) = 6 W_ij / r^7 - 21 (V_i r_j + V_j r_i) / r^9
         *                       - 7 C delta_ij / r^9 + 63 C r_i r_j / r^11
         *   d_i d_j ((t.r) / r^5) = -5 (t_i r_j + t_j r_i) / r^7
         *                           - 5 (t.r) delta_ij / r^7 + 35 (t.r) r_i r_j / r^9 */
        double O[3][3][3], W[3][3], V[3] = {0, 0, 0}, t[3] = {0, 0, 0};
        octupole_tensor(mom, O);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) W[i][j] = O[i][j][0] * r[0] + O[i][j][1] * r[1] + O[i][j][2] * r[2];
        for (int i = 0; i < 3; ++i) {
            V[i] = W[i][0] * r[0] + W[i][1] * r[1] + W[i][2] * r[2];
            t[i] = O[0][0][i] + O[1][1][i] + O[2][2][i];
        }
        double C = V[0] * r[0] + V[1] * r[1] + V[2] * r[2];
        double tr = t[0] * r[0] + t[1] * r[1] + t[2] * r[2];
        double r11 = r9 * rinv * rinv;
        for (int k = 0; k < 6; ++k) {
            int i = I[k], j = J[k];
            double dij = i == j ? 1.0 : 0.0;
            double ddC = 6.0 * W[i][j] * r7 - 21.0 * (V[i] * r[j] + V[j] * r[i]) * r9 - 7.0 * C * dij * r9 +
                         63.0 * C * r[i] * r[j] * r11;
            double ddT = -5.0 * (t[i] * r[j] + t[j] * r[i]) * r7 - 5.0 * tr * dij * r7 + 35.0 * tr * r[i] * r[j] * r9;
            G[k] = -(2.5 * ddC - 1.5 * ddT);
        }
        return;
    }
    for (int k = 0; k < 6; ++k) {
        int i = I[k], j = J[k];
        double dij = i == j ? 1.0 : 0.0;
        if (order == 0) {
            G[k] = mom[0] * (dij * r2 - 3.0 * r[i] * r[j]) * r5;
        } else if (order == 1) {
            double mr = mom[0] * r[0] + mom[1] * r[1] + mom[2] * r[2];
            G[k] = 3.0 * (mom[i] * r[j] + mom[j] * r[i] + mr * dij) * r5 - 15.0 * mr * r[i] * r[j] * r7;
        } else {
            double Q[3][3] = {{mom[0], mom[1], mom[2]}, {mom[1], mom[3], mom[4]}, {mom[2], mom[4], mom[5]}};
            double Qr[3], rQr = 0.0, tr = mom[0] + mom[3] + mom[5];
            for (int a = 0; a < 3; ++a) Qr[a] = Q[a][0] * r[0] + Q[a][1] * r[1] + Q[a][2] * r[2];
            for (int a = 0; a < 3; ++a) rQr += r[a] * Qr[a];
            double ddA = 3.0 * Q[i][j] * r5 - 15.0 * (Qr[i] * r[j] + Qr[j] * r[i]) * r7 - 7.5 * rQr * dij * r7 +
                         52.5 * rQr * r[i] * r[j] * r9;
            double ddB = 1.5 * tr * (dij * r5 - 5.0 * r[i] * r[j] * r7);
            G[k] = -(ddA + ddB);
        }
    }
}

void orc_p2p_pair_grad(int o, const double *r, const double *mom, double *G)
{
    int m = code_mask(o), off = 0;
    for (int k = 0; k < 6; ++k) G[k] = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (!(m & (1 << k))) continue;
        double g[6];
        pair_grad_single(k, r, mom + off, g);
        for (int c = 0; c < 6; ++c) G[c] += g[c];
        off += width_of(k);
    }
}

/* O(N^2) field gradient at the listed targets (all if targets == NULL),
 * ascending j, j != i; grad is nt x 6 (xx, xy, xz, yy, yz, zz). */
void orc_direct_grad(int64_t n, const double *pos, int order, const double *mom, int64_t nt,
                     const int64_t *targets, double *grad)
{
    int w = mom_width(order);
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = targets ? targets[t] : t;
        double sg[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            double g[6];
            orc_p2p_pair_grad(order, r, mom + w * j, g);
            for (int c = 0; c < 6; ++c) sg[c] += g[c];
        }
        for (int c = 0; c < 6; ++c) grad[6 * t + c] = sg[c];
    }
}

/* O(N^2) sum over all sources j != i for the listed targets (all if
 * targets == NULL), ascending j. */
void orc_direct(int64_t n, const double *pos, int order, const double *mom,
                int64_t nt, const int64_t *targets, double *phi, double *field)
{
    int w = mom_width(order);
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = targets ? targets[t] : t;
        double sp = 0.0, se[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            double ph, e[3];
            orc_p2p_pair(order, r, mom + w * j, &ph, e);
            sp += ph;
            se[0] += e[0];
            se[1] += e[1];
            se[2] += e[2];
        }
        if (phi) phi[t] = sp;
        if (field) {
            field[3 * t] = se[0];
            field[3 * t + 1] = se[1];
            field[3 * t + 2] = se[2];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Expansion operators, physical units, all |n| <= p stored             */
/* ------------------------------------------------------------------ */

/* source tensor S_sigma for |sigma| = order, written into S (nterms(order)) */
static void source_tensor(int order, const double *mom, double *S)
{
    memset(S, 0, sizeof(double) * orc_nterms(order));
    if (order == 0) {
        S[0] = mom[0];
    } else if (order == 1) {
        S[orc_index(1, 0, 0)] = -mom[0];
        S[orc_index(0, 1, 0)] = -mom[1];
        S[orc_index(0, 0, 1)] = -mom[2];
    } else if (order == 2) {
        S[orc_index(2, 0, 0)] = mom[0] / 2.0;
        S[orc_index(1, 1, 0)] = mom[1];
        S[orc_index(1, 0, 1)] = mom[2];
        S[orc_index(0, 2, 0)] = mom[3] / 2.0;
        S[orc_index(0, 1, 1)] = mom[4];
        S[orc_index(0, 0, 2)] = mom[5] / 2.0;
    } else {
        /* octupole: the ten components O_m in the index order of order 3,
         * S_m = -O_m / m! */
        for (int c = 0; c < 10; ++c) {
            int m[3];
            orc_multi_index(orc_nterms(2) + c, m);
            S[orc_nterms(2) + c] = -mom[c] / (factorial(m[0]) * factorial(m[1]) * factorial(m[2]));
        }
    }
}

/* P2M (Eq. 5): add the expansion about z of np sources into M (nterms(p));
 * a mixed source contributes each of its single-order parts */
void orc_p2m(int p, int o, const double *z, int64_t np, const double *pos,
             const double *mom, double *M)
{
    int w = mom_width(o);
    int nt = orc_nterms(p);
    int mask = code_mask(o);
    double *mono = malloc(sizeof(double) * nt);
    double S[20];
    for (int64_t j = 0; j < np; ++j) {
        double d[3] = {z[0] - pos[3 * j], z[1] - pos[3 * j + 1], z[2] - pos[3 * j + 2]};
        monomials(p, d, mono);
        int off = 0;
        for (int order = 0; order < 4; ++order) {
        if (!(mask & (1 << order))) continue;
        source_tensor(order, mom + w * j + off, S);
        off += width_of(order);
        for (int i = orc_nterms(order - 1); i < nt; ++i) {
            int n[3];
            orc_multi_index(i, n);
            double acc = 0.0;
            for (int sx = order; sx >= 0; --sx)
                for (int sy = order - sx; sy >= 0; --sy) {
                    int sz = order - sx - sy;
                    if (sx > n[0] || sy > n[1] || sz > n[2]) continue;
                    acc += mono[orc_index(n[0] - sx, n[1] - sy, n[2] - sz)] * S[orc_index(sx, sy, sz)];
                }
            M[i] += acc;
        }
        }
    }
    free(mono);
}

/* M2M (Eq. 4): add the expansion Mc about zc, re-centred at zp, into Mp */
void orc_m2m(int p, const double *zc, const double *Mc, const double *zp, double *Mp)
{
    int nt = orc_nterms(p);
    double *mono = malloc(sizeof(double) * nt);
    double d[3] = {zp[0] - zc[0], zp[1] - zc[1], zp[2] - zc[2]};
    monomials(p, d, mono);
    for (int i = 0; i < nt; ++i) {
        int n[3];
        orc_multi_index(i, n);
        double acc = 0.0;
        for (int kx = 0; kx <= n[0]; ++kx)
            for (int ky = 0; ky <= n[1]; ++ky)
                for (int kz = 0; kz <= n[2]; ++kz)
                    acc += mono[orc_index(kx, ky, kz)] * Mc[orc_index(n[0] - kx, n[1] - ky, n[2] - kz)];
        Mp[i] += acc;
    }
    free(mono);
}

/* M2L (Eq. 8): add the local expansion about zB of the multipole MA about zA */
void orc_m2l(int p, int s, const double *zA, const double *MA, const double *zB, double *LB)
{
    double *D = malloc(sizeof(double) * orc_nterms(p));
    orc_dtensor(p, zB[0] - zA[0], zB[1] - zA[1], zB[2] - zA[2], D);
    for (int i = 0; i < orc_nterms(p - s); ++i) {
        int n[3];
        orc_multi_index(i, n);
        int kn = n[0] + n[1] + n[2];
        double acc = 0.0;
        for (int j = orc_nterms(s - 1); j < orc_nterms(p - kn); ++j) {
            int m[3];
            orc_multi_index(j, m);
            acc += MA[j] * D[orc_index(n[0] + m[0], n[1] + m[1], n[2] + m[2])];
        }
        LB[i] += acc;
    }
    free(D);
}

/* L2L: add the local expansion LP about zP, re-centred at zC, into LC */
void orc_l2l(int p, int s, const double *zP, const double *LP, const double *zC, double *LC)
{
    int q = p - s;
    double *mono = malloc(sizeof(double) * orc_nterms(q));
    double d[3] = {zC[0] - zP[0], zC[1] - zP[1], zC[2] - zP[2]};
    monomials(q, d, mono);
    for (int i = 0; i < orc_nterms(q); ++i) {
        int n[3];
        orc_multi_index(i, n);
        double acc = 0.0;
        for (int j = 0; j < orc_nterms(q); ++j) {
            int k[3];
            orc_multi_index(j, k);
            if (k[0] < n[0] || k[1] < n[1] || k[2] < n[2]) continue;
            acc += mono[orc_index(k[0] - n[0], k[1] - n[1], k[2] - n[2])] * LP[j];
        }
        LC[i] += acc;
    }
    free(mono);
}

/* L2P (Eq. 9, Eq. 10 with |k| = 1): potential and field at x */
void orc_l2p(int p, int s, const double *z, const double *L, const double *x, double *phi, double *E)
{
    int q = p - s;
    double *mono = malloc(sizeof(double) * orc_nterms(q));
    double d[3] = {x[0] - z[0], x[1] - z[1], x[2] - z[2]};
    monomials(q, d, mono);
    double ph = 0.0, e[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < orc_nterms(q); ++i) ph += mono[i] * L[i];
    for (int i = 0; i < orc_nterms(q - 1); ++i) {
        int n[3];
        orc_multi_index(i, n);
        e[0] -= mono[i] * L[orc_index(n[0] + 1, n[1], n[2])];
        e[1] -= mono[i] * L[orc_index(n[0], n[1] + 1, n[2])];
        e[2] -= mono[i] * L[orc_index(n[0], n[1], n[2] + 1)];
    }
    *phi = ph;
    E[0] = e[0];
    E[1] = e[1];
    E[2] = e[2];
    free(mono);
}

/* Field gradient of the local expansion at x: the derivative of order
 * k = e_i + e_j of the L2P sum (the general-k form of Eq. 10),
 * d_i d_j phi = sum_{|n| <= p-s-2} (x-z)^n/n! L_{n+e_i+e_j}, G_ij = -that.
 * For p - s < 2 the truncated expansion has no second derivative: G = 0. */
void orc_l2p_grad(int p, int s, const double *z, const double *L, const double *x, double *G)
{
    static const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
    int q = p - s;
    for (int k = 0; k < 6; ++k) G[k] = 0.0;
    if (q < 2) return;
    double *mono = malloc(sizeof(double) * orc_nterms(q));
    double d[3] = {x[0] - z[0], x[1] - z[1], x[2] - z[2]};
    monomials(q, d, mono);
    for (int i = 0; i < orc_nterms(q - 2); ++i) {
        int n[3];
        orc_multi_index(i, n);
        for (int k = 0; k < 6; ++k) {
            int a[3] = {n[0], n[1], n[2]};
            a[I[k]] += 1;
            a[J[k]] += 1;
            G[k] -= mono[i] * L[orc_index(a[0], a[1], a[2])];
        }
    }
    free(mono);
}

/* M2P (Eq. 6): potential and field at x of the multipole M about zA */
void orc_m2p(int p, int s, const double *zA, const double *M, const double *x, double *phi, double *E)
{
    double *D = malloc(sizeof(double) * orc_nterms(p + 1));
    orc_dtensor(p + 1, x[0] - zA[0], x[1] - zA[1], x[2] - zA[2], D);
    double ph = 0.0, e[3] = {0.0, 0.0, 0.0};
    for (int j = orc_nterms(s - 1); j < orc_nterms(p); ++j) {
        int m[3];
        orc_multi_index(j, m);
        ph += M[j] * D[j];
        e[0] -= M[j] * D[orc_index(m[0] + 1, m[1], m[2])];
        e[1] -= M[j] * D[orc_index(m[0], m[1] + 1, m[2])];
        e[2] -= M[j] * D[orc_index(m[0], m[1], m[2] + 1)];
    }
    *phi = ph;
    E[0] = e[0];
    E[1] = e[1];
    E[2] = e[2];
    free(D);
}

/* Field gradient of the multipole M about zA at x: the second derivatives
 * of the M2P sum, d_i d_j phi = sum M_n D_{n+e_i+e_j}(x - zA), G_ij = -that
 * (derivative tensor to order p + 2). */
void orc_m2p_grad(int p, int s, const double *zA, const double *M, const double *x, double *G)
{
    static const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
    double *D = malloc(sizeof(double) * orc_nterms(p + 2));
    orc_dtensor(p + 2, x[0] - zA[0], x[1] - zA[1], x[2] - zA[2], D);
    for (int k = 0; k < 6; ++k) G[k] = 0.0;
    for (int j = orc_nterms(s - 1); j < orc_nterms(p); ++j) {
        int m[3];
        orc_multi_index(j, m);
        for (int k = 0; k < 6; ++k) {
            int a[3] = {m[0], m[1], m[2]};
            a[I[k]] += 1;
            a[J[k]] += 1;
            G[k] -= M[j] * D[orc_index(a[0], a[1], a[2])];
        }
    }
    free(D);
}

/* ------------------------------------------------------------------ */
/* Octree and interaction lists (Section 3.2)                           */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t *v;
    int64_t n, cap;
} ivec;

static void ivec_push(ivec *a, int64_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 16;
        a->v = realloc(a->v, sizeof(int64_t) * a->cap);
    }
    a->v[a->n++] = x;
}

typedef struct orc_tree {
    int64_t n;
    double lo[3], W, h;          /* root corner, root side, half grid unit */
    uint64_t *key;               /* sorted keys */
    int64_t *perm;               /* perm[i] = input index of sorted particle i */
    int64_t *iperm;              /* inverse */
    int32_t *q;                  /* quantised coords of sorted particles (3 per) */
    double *xs;                  /* sorted positions (3 per) */
    int64_t ncells, nlevels;
    int32_t *level, *ix;         /* ix: 3 per cell */
    int64_t *first, *count, *parent, *child0;
    int32_t *nchild;
    int64_t *level_ptr;          /* cells of level l: [level_ptr[l], level_ptr[l+1]) */
    int64_t *leaf_of;            /* leaf of each sorted particle */
    /* lists (filled by orc_tree_lists) */
    double theta;
    int64_t *m2l_ptr, *m2l_src, *p2p_ptr, *p2p_src;
} orc_tree;

typedef struct {
    uint64_t key;
    int64_t idx;
} keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *x = a, *y = b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static uint64_t morton(int64_t qx, int64_t qy, int64_t qz)
{
    uint64_t k = 0;
    for (int b = 0; b < ORC_MAXLEVEL; ++b) {
        k |= (uint64_t)((qx >> b) & 1) << (3 * b + 2);
        k |= (uint64_t)((qy >> b) & 1) << (3 * b + 1);
        k |= (uint64_t)((qz >> b) & 1) << (3 * b);
    }
    return k;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->key); free(t->perm); free(t->iperm); free(t->q); free(t->xs);
    free(t->level); free(t->ix); free(t->first); free(t->count); free(t->parent);
    free(t->child0); free(t->nchild); free(t->level_ptr); free(t->leaf_of);
    free(t->m2l_ptr); free(t->m2l_src); free(t->p2p_ptr); free(t->p2p_src);
    free(t);
}

orc_tree *orc_tree_build(int64_t n, const double *pos, int ncrit)
{
    if (n < 1 || ncrit < 1) return NULL;
    orc_tree *t = calloc(1, sizeof(orc_tree));
    t->n = n;
    double hi[3];
    for (int d = 0; d < 3; ++d) { t->lo[d] = pos[d]; hi[d] = pos[d]; }
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (pos[3 * i + d] < t->lo[d]) t->lo[d] = pos[3 * i + d];
            if (pos[3 * i + d] > hi[d]) hi[d] = pos[3 * i + d];
        }
    double W = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - t->lo[d] > W) W = hi[d] - t->lo[d];
    if (W == 0.0) W = 1.0;
    t->W = W;
    t->h = ldexp(W, -22);
    double scale = ldexp(1.0, ORC_MAXLEVEL) / W;
    const int64_t qmax = ((int64_t)1 << ORC_MAXLEVEL) - 1;

    int32_t *qin = malloc(sizeof(int32_t) * 3 * n);
    keyidx *ki = malloc(sizeof(keyidx) * n);
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double v = (pos[3 * i + d] - t->lo[d]) * scale;
            int64_t qi = (int64_t)floor(v);
            if (qi > qmax) qi = qmax;
            if (qi < 0) qi = 0;
            qin[3 * i + d] = (int32_t)qi;
        }
        ki[i].key = morton(qin[3 * i], qin[3 * i + 1], qin[3 * i + 2]);
        ki[i].idx = i;
    }
    qsort(ki, n, sizeof(keyidx), cmp_keyidx);
    t->key = malloc(sizeof(uint64_t) * n);
    t->perm = malloc(sizeof(int64_t) * n);
    t->iperm = malloc(sizeof(int64_t) * n);
    t->q = malloc(sizeof(int32_t) * 3 * n);
    t->xs = malloc(sizeof(double) * 3 * n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = ki[i].idx;
        t->key[i] = ki[i].key;
        t->perm[i] = j;
        t->iperm[j] = i;
        for (int d = 0; d < 3; ++d) {
            t->q[3 * i + d] = qin[3 * j + d];
            t->xs[3 * i + d] = pos[3 * j + d];
        }
    }
    free(qin);
    free(ki);

    /* cells, level by level; canonical order = level-major, ascending key */
    ivec lev = {0}, ix = {0}, first = {0}, count = {0}, parent = {0};
    ivec lptr = {0};
    ivec_push(&lptr, 0);
    ivec_push(&lev, 0); ivec_push(&ix, 0); ivec_push(&ix, 0); ivec_push(&ix, 0);
    ivec_push(&first, 0); ivec_push(&count, n); ivec_push(&parent, -1);
    int64_t lbeg = 0, lend = 1;
    int l = 0;
    for (;;) {
        ivec_push(&lptr, lend);
        if (l == ORC_MAXLEVEL) break;
        for (int64_t c = lbeg; c < lend; ++c) {
            if (count.v[c] <= ncrit) continue;
            int shift = 3 * (ORC_MAXLEVEL - (l + 1));
            int64_t f = first.v[c], e = first.v[c] + count.v[c];
            int64_t i = f;
            while (i < e) {
                int dig = (int)((t->key[i] >> shift) & 7);
                int64_t j = i;
                while (j < e && (int)((t->key[j] >> shift) & 7) == dig) ++j;
                ivec_push(&lev, l + 1);
                ivec_push(&ix, 2 * ix.v[3 * c] + ((dig >> 2) & 1));
                ivec_push(&ix, 2 * ix.v[3 * c + 1] + ((dig >> 1) & 1));
                ivec_push(&ix, 2 * ix.v[3 * c + 2] + (dig & 1));
                ivec_push(&first, i);
                ivec_push(&count, j - i);
                ivec_push(&parent, c);
                i = j;
            }
        }
        if (lev.n == lend) break;
        lbeg = lend;
        lend = lev.n;
        ++l;
    }
    t->ncells = lev.n;
    t->nlevels = lptr.n - 1;
    int64_t nc = t->ncells;
    t->level = malloc(sizeof(int32_t) * nc);
    t->ix = malloc(sizeof(int32_t) * 3 * nc);
    t->first = first.v;
    t->count = count.v;
    t->parent = parent.v;
    t->child0 = malloc(sizeof(int64_t) * nc);
    t->nchild = calloc(nc, sizeof(int32_t));
    for (int64_t c = 0; c < nc; ++c) {
        t->level[c] = (int32_t)lev.v[c];
        for (int d = 0; d < 3; ++d) t->ix[3 * c + d] = (int32_t)ix.v[3 * c + d];
        t->child0[c] = -1;
    }
    for (int64_t c = 0; c < nc; ++c) {
        int64_t pa = t->parent[c];
        if (pa >= 0) {
            if (t->child0[pa] < 0) t->child0[pa] = c;
            t->nchild[pa]++;
        }
    }
    t->level_ptr = lptr.v;
    free(lev.v);
    free(ix.v);
    t->leaf_of = malloc(sizeof(int64_t) * n);
    for (int64_t c = 0; c < nc; ++c)
        if (t->nchild[c] == 0)
            for (int64_t i = t->first[c]; i < t->first[c] + t->count[c]; ++i) t->leaf_of[i] = c;
    return t;
}

/* integer geometry in units of the half grid step h = W 2^-22 */
static void cell_geom(const orc_tree *t, int64_t c, int64_t *cen, int64_t *rad)
{
    int l = t->level[c];
    *rad = (int64_t)1 << (ORC_MAXLEVEL - l);
    for (int d = 0; d < 3; ++d) cen[d] = (2 * (int64_t)t->ix[3 * c + d] + 1) * (*rad);
}

void orc_cell_center(const orc_tree *t, int64_t c, double *z, double *r)
{
    int64_t cen[3], rad;
    cell_geom(t, c, cen, &rad);
    for (int d = 0; d < 3; ++d) z[d] = t->lo[d] + (double)cen[d] * t->h;
    *r = (double)rad * t->h;
}

static int is_leaf(const orc_tree *t, int64_t c) { return t->nchild[c] == 0; }

static void dual_traverse(const orc_tree *t, int64_t A, int64_t B, double th2, ivec *m2l, ivec *p2p)
{
    int64_t cA[3], cB[3], rA, rB;
    cell_geom(t, A, cA, &rA);
    cell_geom(t, B, cB, &rB);
    int64_t d2 = 0;
    for (int d = 0; d < 3; ++d) d2 += (cB[d] - cA[d]) * (cB[d] - cA[d]);
    double lhs = (double)(rA + rB);
    lhs = lhs * lhs;
    double rhs = th2 * (double)d2;
    int la = is_leaf(t, A), lb = is_leaf(t, B);
    if (lhs < rhs) {
        ivec_push(&m2l[B], A);
    } else if (la && lb) {
        ivec_push(&p2p[B], A);
    } else if (lb || (!la && rA > rB)) {
        for (int64_t a = t->child0[A]; a < t->child0[A] + t->nchild[A]; ++a)
            dual_traverse(t, a, B, th2, m2l, p2p);
    } else if (la || rB > rA) {
        for (int64_t b = t->child0[B]; b < t->child0[B] + t->nchild[B]; ++b)
            dual_traverse(t, A, b, th2, m2l, p2p);
    } else {
        for (int64_t a = t->child0[A]; a < t->child0[A] + t->nchild[A]; ++a)
            for (int64_t b = t->child0[B]; b < t->child0[B] + t->nchild[B]; ++b)
                dual_traverse(t, a, b, th2, m2l, p2p);
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static void to_csr(ivec *lists, int64_t nc, int64_t **ptr, int64_t **src)
{
    *ptr = malloc(sizeof(int64_t) * (nc + 1));
    (*ptr)[0] = 0;
    for (int64_t c = 0; c < nc; ++c) (*ptr)[c + 1] = (*ptr)[c] + lists[c].n;
    *src = malloc(sizeof(int64_t) * ((*ptr)[nc] + 1));
    for (int64_t c = 0; c < nc; ++c) {
        qsort(lists[c].v, lists[c].n, sizeof(int64_t), cmp_i64);
        if (lists[c].n) memcpy(*src + (*ptr)[c], lists[c].v, sizeof(int64_t) * lists[c].n);
        free(lists[c].v);
    }
}

int orc_tree_lists(orc_tree *t, double theta)
{
    if (!t || !(theta > 0.0 && theta < 1.0)) return 1;
    free(t->m2l_ptr); free(t->m2l_src); free(t->p2p_ptr); free(t->p2p_src);
    t->theta = theta;
    int64_t nc = t->ncells;
    ivec *m2l = calloc(nc, sizeof(ivec));
    ivec *p2p = calloc(nc, sizeof(ivec));
    double th2 = theta * theta;
    dual_traverse(t, 0, 0, th2, m2l, p2p);
    to_csr(m2l, nc, &t->m2l_ptr, &t->m2l_src);
    to_csr(p2p, nc, &t->p2p_ptr, &t->p2p_src);
    free(m2l);
    free(p2p);
    return 0;
}

/* sizes: n, ncells, nlevels, n_m2l, n_p2p, nleaves */
void orc_tree_info(const orc_tree *t, int64_t *info)
{
    info[0] = t->n;
    info[1] = t->ncells;
    info[2] = t->nlevels;
    info[3] = t->m2l_ptr ? t->m2l_ptr[t->ncells] : 0;
    info[4] = t->p2p_ptr ? t->p2p_ptr[t->ncells] : 0;
    int64_t nl = 0;
    for (int64_t c = 0; c < t->ncells; ++c) nl += is_leaf(t, c);
    info[5] = nl;
}

/* copy the canonical tree out; any pointer may be NULL */
void orc_tree_export(const orc_tree *t, double *geom /* lo[3], W */, uint64_t *key, int64_t *perm,
                     int32_t *level, int32_t *ix, int64_t *first, int64_t *count, int64_t *parent,
                     int64_t *child0, int32_t *nchild, int64_t *m2l_ptr, int64_t *m2l_src,
                     int64_t *p2p_ptr, int64_t *p2p_src)
{
    int64_t n = t->n, nc = t->ncells;
    if (geom) { geom[0] = t->lo[0]; geom[1] = t->lo[1]; geom[2] = t->lo[2]; geom[3] = t->W; }
    if (key) memcpy(key, t->key, sizeof(uint64_t) * n);
    if (perm) memcpy(perm, t->perm, sizeof(int64_t) * n);
    if (level) memcpy(level, t->level, sizeof(int32_t) * nc);
    if (ix) memcpy(ix, t->ix, sizeof(int32_t) * 3 * nc);
    if (first) memcpy(first, t->first, sizeof(int64_t) * nc);
    if (count) memcpy(count, t->count, sizeof(int64_t) * nc);
    if (parent) memcpy(parent, t->parent, sizeof(int64_t) * nc);
    if (child0) memcpy(child0, t->child0, sizeof(int64_t) * nc);
    if (nchild) memcpy(nchild, t->nchild, sizeof(int32_t) * nc);
    if (t->m2l_ptr) {
        if (m2l_ptr) memcpy(m2l_ptr, t->m2l_ptr, sizeof(int64_t) * (nc + 1));
        if (m2l_src) memcpy(m2l_src, t->m2l_src, sizeof(int64_t) * t->m2l_ptr[nc]);
        if (p2p_ptr) memcpy(p2p_ptr, t->p2p_ptr, sizeof(int64_t) * (nc + 1));
        if (p2p_src) memcpy(p2p_src, t->p2p_src, sizeof(int64_t) * t->p2p_ptr[nc]);
    }
}

/* ------------------------------------------------------------------ */
/* Upward pass, FMM and BH evaluation                                   */
/* ------------------------------------------------------------------ */

/* M for every cell (ncells x nterms(p)), from sorted moments */
static double *upward(const orc_tree *t, int order, const double *mom_sorted, int p)
{
    int nt = orc_nterms(p);
    int w = mom_width(order);
    double *M = calloc((size_t)t->ncells * nt, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < t->ncells; ++c) {
        if (!is_leaf(t, c)) continue;
        double z[3], r;
        orc_cell_center(t, c, z, &r);
        orc_p2m(p, order, z, t->count[c], t->xs + 3 * t->first[c], mom_sorted + w * t->first[c],
                M + (size_t)c * nt);
    }
    for (int64_t l = t->nlevels - 2; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t c = t->level_ptr[l]; c < t->level_ptr[l + 1]; ++c) {
            double zp[3], rp;
            orc_cell_center(t, c, zp, &rp);
            for (int64_t ch = t->child0[c]; ch >= 0 && ch < t->child0[c] + t->nchild[c]; ++ch) {
                double zc[3], rc;
                orc_cell_center(t, ch, zc, &rc);
                orc_m2m(p, zc, M + (size_t)ch * nt, zp, M + (size_t)c * nt);
            }
        }
    }
    return M;
}

static double *sorted_moments(const orc_tree *t, int order, const double *mom)
{
    int w = mom_width(order);
    double *ms = malloc(sizeof(double) * w * t->n);
    for (int64_t i = 0; i < t->n; ++i)
        for (int k = 0; k < w; ++k) ms[w * i + k] = mom[w * t->perm[i] + k];
    return ms;
}

/* Multipoles of every cell in canonical order (physical units). */
int orc_upward(const orc_tree *t, int order, const double *mom, int p, double *M_out)
{
    double *ms = sorted_moments(t, order, mom);
    double *M = upward(t, order, ms, p);
    memcpy(M_out, M, sizeof(double) * (size_t)t->ncells * orc_nterms(p));
    free(M);
    free(ms);
    return 0;
}

/* FMM potential/field at the listed targets (input indices; all if
 * targets == NULL).  L_out (ncells x nterms(p-s)), if given, receives the
 * local expansions of the cells that were needed (others zero).  grad, if
 * given (nt x 6), receives the field gradient: the second derivatives of the
 * local expansion plus the near field's closed forms. */
int orc_fmm_eval(const orc_tree *t, int order, const double *mom, int p, int64_t nt_,
                 const int64_t *targets, double *phi, double *field, double *L_out, double *grad)
{
    if (!orc_code_valid(order)) return 1;
    int s = orc_min_order(order);
    if (!t->m2l_ptr || p < s + 1) return 1;
    int w = mom_width(order);
    int ntM = orc_nterms(p), ntL = orc_nterms(p - s);
    double *ms = sorted_moments(t, order, mom);
    double *M = upward(t, order, ms, p);
    int64_t nc = t->ncells;
    int64_t cnt = targets ? nt_ : t->n;
    char *need = calloc(nc, 1);
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? t->iperm[targets[k]] : k;
        for (int64_t c = t->leaf_of[i]; c >= 0 && !need[c]; c = t->parent[c]) need[c] = 1;
    }
    double *L = calloc((size_t)nc * ntL, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nc; ++b) {
        if (!need[b]) continue;
        double zB[3], rB;
        orc_cell_center(t, b, zB, &rB);
        for (int64_t e = t->m2l_ptr[b]; e < t->m2l_ptr[b + 1]; ++e) {
            int64_t a = t->m2l_src[e];
            double zA[3], rA;
            orc_cell_center(t, a, zA, &rA);
            orc_m2l(p, s, zA, M + (size_t)a * ntM, zB, L + (size_t)b * ntL);
        }
    }
    for (int64_t l = 1; l < t->nlevels; ++l) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t c = t->level_ptr[l]; c < t->level_ptr[l + 1]; ++c) {
            if (!need[c]) continue;
            int64_t pa = t->parent[c];
            double zP[3], zC[3], r;
            orc_cell_center(t, pa, zP, &r);
            orc_cell_center(t, c, zC, &r);
            orc_l2l(p, s, zP, L + (size_t)pa * ntL, zC, L + (size_t)c * ntL);
        }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? t->iperm[targets[k]] : k;
        int64_t out = targets ? k : t->perm[i];
        int64_t b = t->leaf_of[i];
        double zB[3], rB;
        orc_cell_center(t, b, zB, &rB);
        const double *x = t->xs + 3 * i;
        double ph, e[3], g[6];
        orc_l2p(p, s, zB, L + (size_t)b * ntL, x, &ph, e);
        if (grad) orc_l2p_grad(p, s, zB, L + (size_t)b * ntL, x, g);
        for (int64_t q = t->p2p_ptr[b]; q < t->p2p_ptr[b + 1]; ++q) {
            int64_t a = t->p2p_src[q];
            for (int64_t j = t->first[a]; j < t->first[a] + t->count[a]; ++j) {
                if (j == i) continue;
                double r[3] = {x[0] - t->xs[3 * j], x[1] - t->xs[3 * j + 1], x[2] - t->xs[3 * j + 2]};
                double pp, ee[3];
                orc_p2p_pair(order, r, ms + w * j, &pp, ee);
                ph += pp;
                e[0] += ee[0];
                e[1] += ee[1];
                e[2] += ee[2];
                if (grad) {
                    double gg[6];
                    orc_p2p_pair_grad(order, r, ms + w * j, gg);
                    for (int c = 0; c < 6; ++c) g[c] += gg[c];
                }
            }
        }
        if (grad)
            for (int c = 0; c < 6; ++c) grad[6 * out + c] = g[c];
        if (phi) phi[out] = ph;
        if (field) {
            field[3 * out] = e[0];
            field[3 * out + 1] = e[1];
            field[3 * out + 2] = e[2];
        }
    }
    if (L_out) memcpy(L_out, L, sizeof(double) * (size_t)nc * ntL);
    free(L);
    free(need);
    free(M);
    free(ms);
    return 0;
}

/* does cell c contain sorted particle i (integer test on the quantised grid) */
static int cell_contains(const orc_tree *t, int64_t c, int64_t i)
{
    int sh = ORC_MAXLEVEL - t->level[c];
    for (int d = 0; d < 3; ++d)
        if ((t->q[3 * i + d] >> sh) != t->ix[3 * c + d]) return 0;
    return 1;
}

/* Multipolar Barnes-Hut (Section 3.2, Eq. 12) at the listed targets. */
int orc_bh_eval(const orc_tree *t, int order, const double *mom, int p, double theta_bh,
                int64_t nt_, const int64_t *targets, double *phi, double *field, double *grad)
{
    if (!orc_code_valid(order)) return 1;
    int s = orc_min_order(order);
    if (p < s || !(theta_bh > 0.0 && theta_bh < 1.0)) return 1;
    int w = mom_width(order);
    int ntM = orc_nterms(p);
    double *ms = sorted_moments(t, order, mom);
    double *M = upward(t, order, ms, p);
    int64_t cnt = targets ? nt_ : t->n;
    double th2 = theta_bh * theta_bh;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? t->iperm[targets[k]] : k;
        int64_t out = targets ? k : t->perm[i];
        const double *x = t->xs + 3 * i;
        double ph = 0.0, e[3] = {0.0, 0.0, 0.0}, g[6] = {0, 0, 0, 0, 0, 0};
        int64_t stack[8 * (ORC_MAXLEVEL + 2)];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            int64_t a = stack[--sp];
            double zA[3], rA;
            orc_cell_center(t, a, zA, &rA);
            double d[3] = {x[0] - zA[0], x[1] - zA[1], x[2] - zA[2]};
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            int accept = !cell_contains(t, a, i) && (rA * rA < th2 * d2);
            if (accept) {
                double pp, ee[3];
                orc_m2p(p, s, zA, M + (size_t)a * ntM, x, &pp, ee);
                ph += pp;
                e[0] += ee[0];
                e[1] += ee[1];
                e[2] += ee[2];
                if (grad) {
                    double gg[6];
                    orc_m2p_grad(p, s, zA, M + (size_t)a * ntM, x, gg);
                    for (int c = 0; c < 6; ++c) g[c] += gg[c];
                }
            } else if (is_leaf(t, a)) {
                for (int64_t j = t->first[a]; j < t->first[a] + t->count[a]; ++j) {
                    if (j == i) continue;
                    double r[3] = {x[0] - t->xs[3 * j], x[1] - t->xs[3 * j + 1], x[2] - t->xs[3 * j + 2]};
                    double pp, ee[3];
                    orc_p2p_pair(order, r, ms + w * j, &pp, ee);
                    ph += pp;
                    e[0] += ee[0];
                    e[1] += ee[1];
                    e[2] += ee[2];
                    if (grad) {
                        double gg[6];
                        orc_p2p_pair_grad(order, r, ms + w * j, gg);
                        for (int c = 0; c < 6; ++c) g[c] += gg[c];
                    }
                }
            } else {
                /* push in reverse so that children are visited in octant order */
                for (int64_t ch = t->child0[a] + t->nchild[a] - 1; ch >= t->child0[a]; --ch) stack[sp++] = ch;
            }
        }
        if (phi) phi[out] = ph;
        if (field) {
            field[3 * out] = e[0];
            field[3 * out + 1] = e[1];
            field[3 * out + 2] = e[2];
        }
        if (grad)
            for (int c = 0; c < 6; ++c) grad[6 * out + c] = g[c];
    }
    free(M);
    free(ms);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Derivatives of the potential of any order K (Section 2, Eq. 10)      */
/* ------------------------------------------------------------------ */
/* Every function below writes d^k phi for each multi-index k of order
 * exactly K, in the index order of that order (position
 * orc_index(k) - orc_nterms(K-1)), (K+1)(K+2)/2 values per target.  Order 1
 * is -E and order 2 is -G of the functions above, which are written from
 * closed forms and so check these independently. */

/* One source of one order at displacement r.  The multipole of a point
 * source about its own position is its source tensor (Eq. 5 with z = x), so
 * Eq. 6 gives phi(r) = sum_{|m|=s} S_m D_m(r) and d^k phi = sum_m S_m D_{m+k}. */
static void pair_derivs_single(int order, int K, const double *r, const double *mom, double *out)
{
    int q = order + K;
    double *D = malloc(sizeof(double) * orc_nterms(q));
    double S[20];
    orc_dtensor(q, r[0], r[1], r[2], D);
    source_tensor(order, mom, S);
    int nk = (K + 1) * (K + 2) / 2, k0 = orc_nterms(K - 1);
    for (int c = 0; c < nk; ++c) {
        int k[3];
        orc_multi_index(k0 + c, k);
        double acc = 0.0;
        for (int mi = orc_nterms(order - 1); mi < orc_nterms(order); ++mi) {
            int m[3];
            orc_multi_index(mi, m);
            acc += S[mi] * D[orc_index(k[0] + m[0], k[1] + m[1], k[2] + m[2])];
        }
        out[c] = acc;
    }
    free(D);
}

/* the same for a source of any order code: the sum over its parts */
void orc_pair_derivs(int o, int K, const double *r, const double *mom, double *out)
{
    int m = code_mask(o), off = 0, nk = (K + 1) * (K + 2) / 2;
    double part[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2];
    for (int c = 0; c < nk; ++c) out[c] = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (!(m & (1 << k))) continue;
        pair_derivs_single(k, K, r, mom + off, part);
        for (int c = 0; c < nk; ++c) out[c] += part[c];
        off += width_of(k);
    }
}

/* O(N^2) derivatives of order K at the listed targets (all if targets is
 * NULL), sources j != i in ascending order */
void orc_direct_derivs(int64_t n, const double *pos, int order, const double *mom, int K, int64_t nt,
                       const int64_t *targets, double *out)
{
    int w = mom_width(order), nk = (K + 1) * (K + 2) / 2;
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? targets[k] : k;
        double acc[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2], part[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2];
        for (int c = 0; c < nk; ++c) acc[c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1], pos[3 * i + 2] - pos[3 * j + 2]};
            orc_pair_derivs(order, K, r, mom + w * j, part);
            for (int c = 0; c < nk; ++c) acc[c] += part[c];
        }
        for (int c = 0; c < nk; ++c) out[(size_t)nk * k + c] = acc[c];
    }
}

/* Eq. 10 for |k| = K: d^k phi = sum_{|n| <= p-s-K} (x-z)^n/n! L_{n+k}
 * (the local expansion is a polynomial of degree p-s: zero for K > p-s) */
void orc_l2p_derivs(int p, int s, const double *z, const double *L, const double *x, int K, double *out)
{
    int q = p - s, nk = (K + 1) * (K + 2) / 2, k0 = orc_nterms(K - 1);
    for (int c = 0; c < nk; ++c) out[c] = 0.0;
    if (K > q) return;
    double *mono = malloc(sizeof(double) * orc_nterms(q - K));
    double d[3] = {x[0] - z[0], x[1] - z[1], x[2] - z[2]};
    monomials(q - K, d, mono);
    for (int c = 0; c < nk; ++c) {
        int k[3];
        orc_multi_index(k0 + c, k);
        double acc = 0.0;
        for (int i = 0; i < orc_nterms(q - K); ++i) {
            int n[3];
            orc_multi_index(i, n);
            acc += mono[i] * L[orc_index(n[0] + k[0], n[1] + k[1], n[2] + k[2])];
        }
        out[c] = acc;
    }
    free(mono);
}

/* FMM derivatives of order K at the listed targets: Eq. 10 on each target's
 * leaf local expansion plus the pairs of its P2P list (j != i) */
int orc_fmm_derivs(const orc_tree *t, int order, const double *mom, int p, int K, int64_t nt_,
                   const int64_t *targets, double *out)
{
    if (!orc_code_valid(order) || K < 1 || K > ORC_TABLE_P) return 1;
    int s = orc_min_order(order);
    if (!t->m2l_ptr || p < s + 1) return 1;
    int w = mom_width(order), ntL = orc_nterms(p - s), nk = (K + 1) * (K + 2) / 2;
    double *L = calloc((size_t)t->ncells * ntL, sizeof(double));
    int rc = orc_fmm_eval(t, order, mom, p, nt_, targets, NULL, NULL, L, NULL);
    if (rc) {
        free(L);
        return rc;
    }
    double *ms = sorted_moments(t, order, mom);
    int64_t cnt = targets ? nt_ : t->n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? t->iperm[targets[k]] : k;
        int64_t o = targets ? k : t->perm[i];
        int64_t b = t->leaf_of[i];
        double zB[3], rB;
        orc_cell_center(t, b, zB, &rB);
        const double *x = t->xs + 3 * i;
        double acc[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2], part[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2];
        orc_l2p_derivs(p, s, zB, L + (size_t)b * ntL, x, K, acc);
        for (int64_t e = t->p2p_ptr[b]; e < t->p2p_ptr[b + 1]; ++e) {
            int64_t a = t->p2p_src[e];
            for (int64_t j = t->first[a]; j < t->first[a] + t->count[a]; ++j) {
                if (j == i) continue;
                double r[3] = {x[0] - t->xs[3 * j], x[1] - t->xs[3 * j + 1], x[2] - t->xs[3 * j + 2]};
                orc_pair_derivs(order, K, r, ms + w * j, part);
                for (int c = 0; c < nk; ++c) acc[c] += part[c];
            }
        }
        for (int c = 0; c < nk; ++c) out[(size_t)nk * o + c] = acc[c];
    }
    free(ms);
    free(L);
    return 0;
}

/* Eq. 6 differentiated K times: d^k phi = sum_{s<=|n|<=p} M_n D_{n+k}(x - zA)
 * for |k| = K (derivative tensor to order p + K) */
void orc_m2p_derivs(int p, int s, const double *zA, const double *M, const double *x, int K, double *out)
{
    int nk = (K + 1) * (K + 2) / 2, k0 = orc_nterms(K - 1);
    double *D = malloc(sizeof(double) * orc_nterms(p + K));
    orc_dtensor(p + K, x[0] - zA[0], x[1] - zA[1], x[2] - zA[2], D);
    for (int c = 0; c < nk; ++c) {
        int k[3];
        orc_multi_index(k0 + c, k);
        double acc = 0.0;
        for (int j = orc_nterms(s - 1); j < orc_nterms(p); ++j) {
            int m[3];
            orc_multi_index(j, m);
            acc += M[j] * D[orc_index(m[0] + k[0], m[1] + k[1], m[2] + k[2])];
        }
        out[c] = acc;
    }
    free(D);
}

/* Barnes-Hut derivatives of order K at the listed targets: the traversal of
 * orc_bh_eval (Eq. 12, the target's own cell never accepted), with the K-th
 * derivatives of M2P for an accepted cell and of the pair potentials for an
 * unaccepted leaf */
int orc_bh_derivs(const orc_tree *t, int order, const double *mom, int p, double theta_bh, int K, int64_t nt_,
                  const int64_t *targets, double *out)
{
    if (!orc_code_valid(order) || K < 1 || K > ORC_TABLE_P) return 1;
    int s = orc_min_order(order);
    if (p < s || !(theta_bh > 0.0 && theta_bh < 1.0)) return 1;
    int w = mom_width(order), ntM = orc_nterms(p), nk = (K + 1) * (K + 2) / 2;
    double *ms = sorted_moments(t, order, mom);
    double *M = upward(t, order, ms, p);
    int64_t cnt = targets ? nt_ : t->n;
    double th2 = theta_bh * theta_bh;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? t->iperm[targets[k]] : k;
        int64_t o = targets ? k : t->perm[i];
        const double *x = t->xs + 3 * i;
        double acc[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2], part[(ORC_TABLE_P + 1) * (ORC_TABLE_P + 2) / 2];
        for (int c = 0; c < nk; ++c) acc[c] = 0.0;
        int64_t stack[8 * (ORC_MAXLEVEL + 2)];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            int64_t a = stack[--sp];
            double zA[3], rA;
            orc_cell_center(t, a, zA, &rA);
            double d[3] = {x[0] - zA[0], x[1] - zA[1], x[2] - zA[2]};
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!cell_contains(t, a, i) && (rA * rA < th2 * d2)) {
                orc_m2p_derivs(p, s, zA, M + (size_t)a * ntM, x, K, part);
                for (int c = 0; c < nk; ++c) acc[c] += part[c];
            } else if (is_leaf(t, a)) {
                for (int64_t j = t->first[a]; j < t->first[a] + t->count[a]; ++j) {
                    if (j == i) continue;
                    double r[3] = {x[0] - t->xs[3 * j], x[1] - t->xs[3 * j + 1], x[2] - t->xs[3 * j + 2]};
                    orc_pair_derivs(order, K, r, ms + w * j, part);
                    for (int c = 0; c < nk; ++c) acc[c] += part[c];
                }
            } else {
                for (int64_t ch = t->child0[a] + t->nchild[a] - 1; ch >= t->child0[a]; --ch) stack[sp++] = ch;
            }
        }
        for (int c = 0; c < nk; ++c) out[(size_t)nk * o + c] = acc[c];
    }
    free(M);
    free(ms);
    return 0;
}
