// Closed-form potential and field of one point source of order S (0 charge,
// 1 dipole, 2 quadrupole, 3 octupole) at displacement r = x_target -
// x_source, used by the near-field kernels (Eq. 1 of Pepper & Fangohr, arXiv
// 2005.12351, and its derivatives; phi = q/r, mu.r/r^3,
// (3 r.Q.r - r^2 tr Q)/(2 r^5), 5/2 O(r,r,r)/r^7 - 3/2 t.r/r^5 with
// t_k = sum_i O_iik; E = -grad phi).
#pragma once
#include <hip/hip_runtime.h>

template <int S>
__device__ __forceinline__ void p2p_pair_f32(float rx, float ry, float rz, float inv, const float4 &m0, const float4 &m1,
                                             float &ph, float &ex, float &ey, float &ez)
{
    const float inv2 = inv * inv;
    const float inv3 = inv * inv2;
    if (S == 0) {
        const float q3 = m0.x * inv3;
        ph = __builtin_fmaf(m0.x, inv, ph);
        ex = __builtin_fmaf(q3, rx, ex);
        ey = __builtin_fmaf(q3, ry, ey);
        ez = __builtin_fmaf(q3, rz, ez);
    } else if (S == 1) {
        const float mr = __builtin_fmaf(m0.x, rx, __builtin_fmaf(m0.y, ry, m0.z * rz));
        ph = __builtin_fmaf(mr, inv3, ph);
        const float t1 = 3.0f * mr * inv2;
        ex = __builtin_fmaf(inv3, __builtin_fmaf(t1, rx, -m0.x), ex);
        ey = __builtin_fmaf(inv3, __builtin_fmaf(t1, ry, -m0.y), ey);
        ez = __builtin_fmaf(inv3, __builtin_fmaf(t1, rz, -m0.z), ez);
    } else {
        // m0 = (xx, xy, xz, yy), m1 = (yz, zz, tr, -)
        const float qx = __builtin_fmaf(m0.x, rx, __builtin_fmaf(m0.y, ry, m0.z * rz));
        const float qy = __builtin_fmaf(m0.y, rx, __builtin_fmaf(m0.w, ry, m1.x * rz));
        const float qz = __builtin_fmaf(m0.z, rx, __builtin_fmaf(m1.x, ry, m1.y * rz));
        const float rqr = __builtin_fmaf(rx, qx, __builtin_fmaf(ry, qy, rz * qz));
        const float inv5 = inv3 * inv2;
        const float r2 = rx * rx + ry * ry + rz * rz;
        ph = __builtin_fmaf(0.5f * inv5, __builtin_fmaf(3.0f, rqr, -r2 * m1.z), ph);
        const float a = __builtin_fmaf(7.5f * rqr, inv2, -1.5f * m1.z);
        ex = __builtin_fmaf(inv5, __builtin_fmaf(a, rx, -3.0f * qx), ex);
        ey = __builtin_fmaf(inv5, __builtin_fmaf(a, ry, -3.0f * qy), ey);
        ez = __builtin_fmaf(inv5, __builtin_fmaf(a, rz, -3.0f * qz), ez);
    }
}

template <int S>
__device__ __forceinline__ void p2p_pair_f64(double rx, double ry, double rz, const double *m, double &ph, double &ex,
                                             double &ey, double &ez)
{
    const double r2 = rx * rx + ry * ry + rz * rz;
    // hardware reciprocal square root estimate, two Newton steps
    double inv = __builtin_amdgcn_rsq(r2);
    const double hr = 0.5 * r2;
    inv = inv * __builtin_fma(-hr * inv, inv, 1.5);
    inv = inv * __builtin_fma(-hr * inv, inv, 1.5);
    const double inv2 = inv * inv;
    const double inv3 = inv * inv2;
    if (S == 0) {
        ph += m[0] * inv;
        ex += m[0] * rx * inv3;
        ey += m[0] * ry * inv3;
        ez += m[0] * rz * inv3;
    } else if (S == 1) {
        const double mr = m[0] * rx + m[1] * ry + m[2] * rz;
        const double inv5 = inv3 * inv2;
        ph += mr * inv3;
        ex += (3.0 * mr * rx - r2 * m[0]) * inv5;
        ey += (3.0 * mr * ry - r2 * m[1]) * inv5;
        ez += (3.0 * mr * rz - r2 * m[2]) * inv5;
    } else {
        const double qx = m[0] * rx + m[1] * ry + m[2] * rz;
        const double qy = m[1] * rx + m[3] * ry + m[4] * rz;
        const double qz = m[2] * rx + m[4] * ry + m[5] * rz;
        const double rqr = rx * qx + ry * qy + rz * qz;
        const double tr = m[0] + m[3] + m[5];
        const double inv5 = inv3 * inv2;
        const double inv7 = inv5 * inv2;
        ph += 0.5 * (3.0 * rqr - r2 * tr) * inv5;
        ex += 7.5 * rqr * rx * inv7 - 3.0 * qx * inv5 - 1.5 * tr * rx * inv5;
        ey += 7.5 * rqr * ry * inv7 - 3.0 * qy * inv5 - 1.5 * tr * ry * inv5;
        ez += 7.5 * rqr * rz * inv7 - 3.0 * qz * inv5 - 1.5 * tr * rz * inv5;
    }
}


// Field gradient G_ij = d_i E_j = -d_i d_j phi of the same sources (the
// second derivatives of the potentials above), accumulated into
// g[0..5] = xx, xy, xz, yy, yz, zz:
//   charge:     q (delta_ij / r^3 - 3 r_i r_j / r^5)
//   dipole:     3 (mu_i r_j + mu_j r_i + (mu.r) delta_ij) / r^5 - 15 (mu.r) r_i r_j / r^7
//   quadrupole: -3 Q_ij / r^5 + 15 ((Qr)_i r_j + (Qr)_j r_i) / r^7
//               + (7.5 r.Q.r / r^7 - 1.5 tr Q / r^5) delta_ij
//               + (7.5 tr Q / r^7 - 52.5 r.Q.r / r^9) r_i r_j
template <int S, typename T>
__device__ __forceinline__ void pair_grad_terms(T rx, T ry, T rz, T inv, T m0, T m1, T m2, T m3, T m4, T m5, T tr,
                                                T (&g)[6])
{
    const T inv2 = inv * inv;
    const T inv3 = inv * inv2;
    const T inv5 = inv3 * inv2;
    const T r[3] = {rx, ry, rz};
    if (S == 0) {
        const T a = m0 * inv3, b = (T)3 * m0 * inv5;
        g[0] += a - b * rx * rx;
        g[1] -= b * rx * ry;
        g[2] -= b * rx * rz;
        g[3] += a - b * ry * ry;
        g[4] -= b * ry * rz;
        g[5] += a - b * rz * rz;
    } else if (S == 1) {
        const T mu[3] = {m0, m1, m2};
        const T mr = m0 * rx + m1 * ry + m2 * rz;
        const T a = (T)3 * inv5, b = (T)15 * mr * inv5 * inv2;
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j, ++k)
                g[k] += a * (mu[i] * r[j] + mu[j] * r[i] + (i == j ? mr : (T)0)) - b * r[i] * r[j];
    } else {
        // m0..m5 = xx, xy, xz, yy, yz, zz
        const T Q[3][3] = {{m0, m1, m2}, {m1, m3, m4}, {m2, m4, m5}};
        T Qr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Qr[i] = Q[i][0] * rx + Q[i][1] * ry + Q[i][2] * rz;
        const T rqr = rx * Qr[0] + ry * Qr[1] + rz * Qr[2];
        const T inv7 = inv5 * inv2;
        const T cq = (T)-3 * inv5, cx = (T)15 * inv7;
        const T cd = (T)7.5 * rqr * inv7 - (T)1.5 * tr * inv5;
        const T cr = (T)7.5 * tr * inv7 - (T)52.5 * rqr * inv7 * inv2;
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j, ++k)
                g[k] += cq * Q[i][j] + cx * (Qr[i] * r[j] + Qr[j] * r[i]) + (i == j ? cd : (T)0) + cr * r[i] * r[j];
    }
}

// FP32 near field: positions in units of the target leaf radius, moments as
// staged (charge m0.x; dipole m0.xyz; quadrupole m0 = (xx, xy, xz, yy),
// m1 = (yz, zz, tr, -))
template <int S>
__device__ __forceinline__ void p2p_pair_grad_f32(float rx, float ry, float rz, float inv, const float4 &m0,
                                                  const float4 &m1, float (&g)[6])
{
    if (S == 2) pair_grad_terms<2, float>(rx, ry, rz, inv, m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, g);
    else pair_grad_terms<S, float>(rx, ry, rz, inv, m0.x, m0.y, m0.z, 0.f, 0.f, 0.f, 0.f, g);
}

// FP64 near field: physical positions and moments (w values of one order)
template <int S>
__device__ __forceinline__ void p2p_pair_grad_f64(double rx, double ry, double rz, const double *m, double (&g)[6])
{
    const double r2 = rx * rx + ry * ry + rz * rz;
    double inv = __builtin_amdgcn_rsq(r2);
    const double hr = 0.5 * r2;
    inv = inv * __builtin_fma(-hr * inv, inv, 1.5);
    inv = inv * __builtin_fma(-hr * inv, inv, 1.5);
    if (S == 2) pair_grad_terms<2, double>(rx, ry, rz, inv, m[0], m[1], m[2], m[3], m[4], m[5], m[0] + m[3] + m[5], g);
    else if (S == 1) pair_grad_terms<1, double>(rx, ry, rz, inv, m[0], m[1], m[2], 0.0, 0.0, 0.0, 0.0, g);
    else pair_grad_terms<0, double>(rx, ry, rz, inv, m[0], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, g);
}


// ------------------------------------------------------------------ octupoles
// O given by its ten components (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz) and
// its trace vector t; W_ij = sum_k O_ijk r_k, V = W r, C = r.V:
//   phi = 5/2 C / r^7 - 3/2 t.r / r^5
//   E   = -15/2 V / r^7 + (35/2 C / r^9 - 15/2 t.r / r^7) r + 3/2 t / r^5
//   G_ij = -d_i d_j phi = -15 W_ij / r^7 + 105/2 (V_i r_j + V_j r_i) / r^9
//          - 15/2 (t_i r_j + t_j r_i) / r^7 + (35/2 C / r^9 - 15/2 t.r / r^7) delta_ij
//          + (105/2 t.r / r^9 - 315/2 C / r^11) r_i r_j
template <typename T>
struct OctW {
    T W[6];   // xx xy xz yy yz zz
    T V[3], C, tr;
};

template <typename T>
__device__ __forceinline__ OctW<T> oct_contract(T rx, T ry, T rz, const T (&o)[10], const T (&t)[3])
{
    OctW<T> w;
    w.W[0] = o[0] * rx + o[1] * ry + o[2] * rz;
    w.W[1] = o[1] * rx + o[3] * ry + o[4] * rz;
    w.W[2] = o[2] * rx + o[4] * ry + o[5] * rz;
    w.W[3] = o[3] * rx + o[6] * ry + o[7] * rz;
    w.W[4] = o[4] * rx + o[7] * ry + o[8] * rz;
    w.W[5] = o[5] * rx + o[8] * ry + o[9] * rz;
    w.V[0] = w.W[0] * rx + w.W[1] * ry + w.W[2] * rz;
    w.V[1] = w.W[1] * rx + w.W[3] * ry + w.W[4] * rz;
    w.V[2] = w.W[2] * rx + w.W[4] * ry + w.W[5] * rz;
    w.C = w.V[0] * rx + w.V[1] * ry + w.V[2] * rz;
    w.tr = t[0] * rx + t[1] * ry + t[2] * rz;
    return w;
}

template <typename T>
__device__ __forceinline__ void oct_field(T rx, T ry, T rz, T inv, const T (&o)[10], const T (&t)[3], T &ph, T &ex,
                                          T &ey, T &ez)
{
    const OctW<T> w = oct_contract<T>(rx, ry, rz, o, t);
    const T inv2 = inv * inv;
    const T inv5 = inv2 * inv2 * inv;
    const T inv7 = inv5 * inv2;
    ph += ((T)2.5 * w.C * inv2 - (T)1.5 * w.tr) * inv5;
    const T a = ((T)17.5 * w.C * inv2 - (T)7.5 * w.tr) * inv7;
    ex += a * rx - (T)7.5 * w.V[0] * inv7 + (T)1.5 * t[0] * inv5;
    ey += a * ry - (T)7.5 * w.V[1] * inv7 + (T)1.5 * t[1] * inv5;
    ez += a * rz - (T)7.5 * w.V[2] * inv7 + (T)1.5 * t[2] * inv5;
}

template <typename T>
__device__ __forceinline__ void oct_grad(T rx, T ry, T rz, T inv, const T (&o)[10], const T (&t)[3], T (&g)[6])
{
    const OctW<T> w = oct_contract<T>(rx, ry, rz, o, t);
    const T inv2 = inv * inv;
    const T inv7 = inv2 * inv2 * inv2 * inv;
    const T inv9 = inv7 * inv2;
    const T r[3] = {rx, ry, rz};
    const T cd = (T)17.5 * w.C * inv9 - (T)7.5 * w.tr * inv7;
    const T cr = ((T)52.5 * w.tr - (T)157.5 * w.C * inv2) * inv9;
    int k = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j, ++k)
            g[k] += (T)-15 * w.W[k] * inv7 + (T)52.5 * (w.V[i] * r[j] + w.V[j] * r[i]) * inv9 -
                    (T)7.5 * (t[i] * r[j] + t[j] * r[i]) * inv7 + (i == j ? cd : (T)0) + cr * r[i] * r[j];
}

// FP32: the staged block [O xxx xxy xxz xyy] [xyz xzz yyy yyz] [yzz zzz t_x t_y] [t_z - - -]
__device__ __forceinline__ void oct_unpack_f32(const float4 &a, const float4 &b, const float4 &c, const float4 &d,
                                               float (&o)[10], float (&t)[3])
{
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
    o[8] = c.x; o[9] = c.y;
    t[0] = c.z; t[1] = c.w; t[2] = d.x;
}

__device__ __forceinline__ void p2p_pair_oct_f32(float rx, float ry, float rz, float inv, const float4 &a,
                                                 const float4 &b, const float4 &c, const float4 &d, float &ph,
                                                 float &ex, float &ey, float &ez)
{
    float o[10], t[3];
    oct_unpack_f32(a, b, c, d, o, t);
    oct_field<float>(rx, ry, rz, inv, o, t, ph, ex, ey, ez);
}

__device__ __forceinline__ void p2p_pair_grad_oct_f32(float rx, float ry, float rz, float inv, const float4 &a,
                                                      const float4 &b, const float4 &c, const float4 &d, float (&g)[6])
{
    float o[10], t[3];
    oct_unpack_f32(a, b, c, d, o, t);
    oct_grad<float>(rx, ry, rz, inv, o, t, g);
}

// FP64: physical positions and the ten physical components
__device__ __forceinline__ double rsq_f64(double r2)
{
    double inv = __builtin_amdgcn_rsq(r2);
    const double hr = 0.5 * r2;
    inv = inv * __builtin_fma(-hr * inv, inv, 1.5);
    return inv * __builtin_fma(-hr * inv, inv, 1.5);
}

__device__ __forceinline__ void p2p_pair_oct_f64(double rx, double ry, double rz, const double *m, double &ph,
                                                 double &ex, double &ey, double &ez)
{
    double o[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) o[k] = m[k];
    const double t[3] = {m[0] + m[3] + m[5], m[1] + m[6] + m[8], m[2] + m[7] + m[9]};
    oct_field<double>(rx, ry, rz, rsq_f64(rx * rx + ry * ry + rz * rz), o, t, ph, ex, ey, ez);
}

__device__ __forceinline__ void p2p_pair_grad_oct_f64(double rx, double ry, double rz, const double *m,
                                                      double (&g)[6])
{
    double o[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) o[k] = m[k];
    const double t[3] = {m[0] + m[3] + m[5], m[1] + m[6] + m[8], m[2] + m[7] + m[9]};
    oct_grad<double>(rx, ry, rz, rsq_f64(rx * rx + ry * ry + rz * rz), o, t, g);
}
