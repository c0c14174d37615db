"""Writes the M2P evaluators of the Barnes-Hut kernel (a build step).

M2P (Eq. 6 of Pepper & Fangohr, arXiv 2005.12351, read as
phi = sum_n M_n D_n(x - z_A), E_i = -sum_n M_n D_{n+e_i}(x - z_A)) needs the
derivatives D_k = d^k (1/|u|) up to order p + 1 at a point that differs for
every particle, so they are computed in registers.  This generator writes
them from the closed (Hermite-type) form of the derivatives of a function of
u^2 / 2: with f(v) = (2v)^(-1/2) and F_m = f^(m) = (-1)^m (2m-1)!! |u|^-(2m+1),

    D_n = sum_{k_d <= n_d / 2} prod_d [ n_d! / (2^k_d k_d! (n_d - 2 k_d)!) u_d^(n_d - 2 k_d) ] F_{|n| - |k|},

followed by the contraction with the cell's (uniform, scalar-loaded)
multipole coefficients.  One specialisation per (p, s, precision).

M2PEvalH is the same for the harmonic basis: the cell's row is folded onto
its components with m_z <= 1 (see P2M / M2M), so only those are contracted
and only the derivatives with k_z <= 2 (those with m_z <= 1 and their
gradient) are formed; D being harmonic, the result is the same.
M2PEvalG / M2PEvalGH also return sum M_n D_{n+e_i+e_j} (the field gradient,
derivatives to order p + 2; harmonic: k_z <= 3) in g[0..5] = xx, xy, xz,
yy, yz, zz.

Usage: python gen_bh.py OUTDIR -> OUTDIR/bh_m2p.h, bh_m2p_s{0..3}.h and the
translation units bh_inst_{f,g}_s{0..3}.hip
"""
import math
import os
import sys

P_MAX = 10


def orders(p):
    out = []
    for k in range(p + 1):
        for nx in range(k, -1, -1):
            for ny in range(k - nx, -1, -1):
                out.append((nx, ny, k - nx - ny))
    return out


def nterms(p):
    return 0 if p < 0 else (p + 1) * (p + 2) * (p + 3) // 6


def idx(n):
    k = sum(n)
    a = n[1] + n[2]
    return nterms(k - 1) + a * (a + 1) // 2 + n[2]


def hcoef(n, k):
    return math.factorial(n) // (2 ** k * math.factorial(k) * math.factorial(n - 2 * k))


def lit(v, fp32):
    s = repr(float(v))
    return s + "f" if fp32 else s


def gen_spec(p, s, fp32, harmonic=False, grad=False):
    T = "float" if fp32 else "double"
    q = p + 2 if grad else p + 1
    L = []
    name = "M2PEval" + ("G" if grad else "") + ("H" if harmonic else "")
    L.append(f"template <> struct {name}<{p}, {s}, {T}> {{")
    L.append(f"    static __device__ __forceinline__ void eval(const {T} *__restrict__ M, {T} ux, {T} uy, {T} uz, "
             f"{T} &ph, {T} &ex, {T} &ey, {T} &ez" + (f", {T} (&g)[6])" if grad else ")"))
    L.append("    {")
    if fp32:
        L.append("        const float r2 = ux * ux + uy * uy + uz * uz;")
        L.append("        const float ri = __builtin_amdgcn_rsqf(r2);")
    else:
        L.append("        const double r2 = ux * ux + uy * uy + uz * uz;")
        L.append("        const double ri = 1.0 / sqrt(r2);")
    L.append(f"        const {T} ri2 = ri * ri;")
    L.append(f"        {T} F0 = ri;")
    for m in range(1, q + 1):
        L.append(f"        const {T} F{m} = F{m - 1} * ri2 * {lit(-(2 * m - 1), fp32)};")
    for d, v in (("X", "ux"), ("Y", "uy"), ("Z", "uz")):
        L.append(f"        const {T} {d}0 = 1;")
        for a in range(1, q + 1):
            L.append(f"        const {T} {d}{a} = {d}{a - 1} * {v};")
    for n in orders(q):
        if harmonic and n[2] > (3 if grad else 2):
            continue
        terms = []
        for kx in range(n[0] // 2 + 1):
            for ky in range(n[1] // 2 + 1):
                for kz in range(n[2] // 2 + 1):
                    c = hcoef(n[0], kx) * hcoef(n[1], ky) * hcoef(n[2], kz)
                    m = sum(n) - kx - ky - kz
                    terms.append(f"{lit(c, fp32)} * (X{n[0] - 2 * kx} * Y{n[1] - 2 * ky}) * (Z{n[2] - 2 * kz} * F{m})")
        L.append(f"        const {T} D{idx(n)} = " + " + ".join(terms) + ";")
    # contraction with the multipole (orders s..p), field needs one order more
    ms = orders(p)[nterms(s - 1):]
    if harmonic:
        ms = [m for m in ms if m[2] <= 1]
    L.append(f"        {T} a0 = 0, a1 = 0, a2 = 0, a3 = 0;")
    for j, m in enumerate(ms):
        L.append(f"        {{ const {T} mm = M[{j}];")
        L.append(f"          a0 = {('__builtin_fmaf' if fp32 else '__builtin_fma')}(mm, D{idx(m)}, a0);")
        for c, (dx, dy, dz) in zip(("a1", "a2", "a3"), ((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            L.append(f"          {c} = {('__builtin_fmaf' if fp32 else '__builtin_fma')}(mm, "
                     f"D{idx((m[0] + dx, m[1] + dy, m[2] + dz))}, {c}); ")
        L.append("        }")
    if grad:
        fm = '__builtin_fmaf' if fp32 else '__builtin_fma'
        L.append(f"        {T} b0 = 0, b1 = 0, b2 = 0, b3 = 0, b4 = 0, b5 = 0;")
        pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        for j, m in enumerate(ms):
            L.append(f"        {{ const {T} mm = M[{j}];")
            for c, (i1, i2) in enumerate(pairs):
                k = list(m)
                k[i1] += 1
                k[i2] += 1
                L.append(f"          b{c} = {fm}(mm, D{idx(tuple(k))}, b{c});")
            L.append("        }")
        for c in range(6):
            L.append(f"        g[{c}] = b{c};")
    L.append("        ph = a0;")
    L.append("        ex = a1;")
    L.append("        ey = a2;")
    L.append("        ez = a3;")
    L.append("    }")
    L.append("};")
    return "\n".join(L)


def _write(fn, txt):
    old = open(fn).read() if os.path.exists(fn) else None
    if old != txt:
        with open(fn, "w") as f:
            f.write(txt)


def main(outdir):
    """Writes bh_m2p.h (the primary templates), bh_m2p_s{s}.h (the
    specialisations of one source order) and one translation unit per
    (source order, with or without the field gradient) that instantiates the
    Barnes-Hut kernels of that pair, so that they compile in parallel;
    returns the translation units."""
    os.makedirs(outdir, exist_ok=True)
    head = ["// Generated by gen_bh.py; do not edit.", "#pragma once", "",
            "template <int P, int S, typename T> struct M2PEval;",
            "template <int P, int S, typename T> struct M2PEvalH;",
            "template <int P, int S, typename T> struct M2PEvalG;",
            "template <int P, int S, typename T> struct M2PEvalGH;", ""]
    _write(os.path.join(outdir, "bh_m2p.h"), "\n".join(head) + "\n")
    tus = []
    for s in (0, 1, 2, 3):
        parts = ["// Generated by gen_bh.py; do not edit.", "#pragma once", '#include "bh_m2p.h"', ""]
        for p in range(max(s, 1), P_MAX + 1):
            for fp32 in (True, False):
                for h in (False, True):
                    for gr in (False, True):
                        parts.append(gen_spec(p, s, fp32, h, gr))
                        parts.append("")
        _write(os.path.join(outdir, f"bh_m2p_s{s}.h"), "\n".join(parts) + "\n")
        for gr in (False, True):
            g = "g" if gr else "f"
            what = "with the field gradient" if gr else "potential and field"
            tu = (f"// Generated by gen_bh.py; do not edit.  Barnes-Hut kernels of source\n"
                  f"// order {s}, {what} (bh_kernel.h).\n"
                  f'#include "bh_kernel.h"\n#include "bh_m2p_s{s}.h"\n\n'
                  f"bh_fn bh_select_{g}_s{s}(int p, bool f32, bool h) {{ return bh_pick_p<{'true' if gr else 'false'}, {s}>(p, f32, h); }}\n")
            fn = os.path.join(outdir, f"bh_inst_{g}_s{s}.hip")
            _write(fn, tu)
            tus.append(fn)
    return tus


if __name__ == "__main__":
    print(main(sys.argv[1] if len(sys.argv) > 1 else "_build/gen"))
