// Closed-form potential and field of one point source of order S (0 charge,
// 1 dipole, 2 quadrupole) at displacement r = x_target - x_source, used by
// the near-field kernels (Eq. 1 of Pepper & Fangohr, arXiv 2005.12351, and
// its derivatives; phi = q/r, mu.r/r^3, (3 r.Q.r - r^2 tr Q)/(2 r^5);
// E = -grad phi).
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

