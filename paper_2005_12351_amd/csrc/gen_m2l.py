"""Writes the unrolled M2L kernels of libfmm.so (a build step).

The multipole-to-local translation (Eq. 8 of Pepper & Fangohr, arXiv
2005.12351) is, for target cell B and source cell A,

    L_n(B) += sum_{s <= |m| <= p - |n|} M_m(A) D_{n+m}(z_B - z_A),  |n| <= p - s,

with D_k the derivatives of 1/r.  In the normalised form used on the GPU
(M~_m = M_m / r_A^|m|, L~_n = L_n r_B^(|n|+1), rho = r_A / r_B) it reads

    L~_n(B) += sum_m D_{n+m}((z_B - z_A) / r_B) * rho^|m| * M~_m(A).

In each generated kernel a 64-wide wavefront works on one tile: lane l owns
the target cell of tile slot l and keeps its local coefficients (or one block
of them) in registers; the wave walks the tile's translation classes, and at
each step every lane streams the multipole of its own source while the
derivative tensor of the class, identical for all lanes, comes through scalar
loads.  The contraction is written out term by term (one fused multiply-add
each), so no index arithmetic is left at run time.  The grid has exactly as
many workgroups as the device keeps resident; the host cuts the concatenated
(tile, output block, entry) work into equally expensive pieces, one per
workgroup, so every SIMD finishes together although the blocks differ in
work by up to 10x.  The wgw waves of a workgroup split each piece's entries
and add their sums in LDS; a piece writes partial sums only where it crosses
a (tile, block) boundary.

Harmonic basis.  The derivative tensor of 1/r is harmonic: for every k,
D_{k+2e_x} + D_{k+2e_y} + D_{k+2e_z} = 0, hence
D_{k+2j e_z} = (-1)^j sum_i C(j,i) D_{k+2i e_x+2(j-i) e_y}.  A multipole
row folded onto the components with m_z <= 1 (done once per cell, as P2M
and M2M write the row) therefore gives the same sums, and the locals, whose
truncation |m| <= p - |n| is the same for n+2e_x, n+2e_y and n+2e_z, obey
the same identity, so only their components with n_z <= 1 are computed and
the rest is rebuilt afterwards.  Order l then holds 2l+1 components instead
of (l+1)(l+2)/2: the irreducible count the paper's Discussion refers to.
The "_h" kernels contract these reduced rows; the term lists are the same
construction restricted to the reduced components.

Usage: python gen_m2l.py OUTDIR  -> OUTDIR/m2l_s{0,1,2}_{f32,f64}[_h].hip
"""
import os
import sys

P_MAX = 10
TILE = 64

# code-shape options (register blocking, scalar-load pipelining, waves per
# workgroup); the defaults are the measured best on gfx950
DEFAULTS = {"acc32": 128, "m32": 64, "acc64": 64, "m64": 32, "dgroup32": 32, "dgroup64": 16, "pipeline": 1,
            "mpre": 0, "launder": 1, "scale_branch": 0, "minwaves": 0, "wgw": 4, "fairprio": 1}


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


def pad(x, m):
    return (x + m - 1) // m * m


def reduced(mis):
    """The components with n_z <= 1 (the harmonic basis), in storage order."""
    return [n for n in mis if n[2] <= 1]


def split_blocks(nl, max_acc):
    """Fewest contiguous n-ranges [a, b) of nearly equal size with at most
    max_acc accumulators each (every block re-reads the multipole
    coefficients it needs, so fewer blocks means less gather traffic)."""
    nb = max(1, -(-nl // max_acc))
    assert nb <= 16, 'at most 16 output blocks'
    return [(nl * i // nb, nl * (i + 1) // nb) for i in range(nb)]


def gen_kernel(p, s, fp32, opt=None, harmonic=False):
    """One kernel per (p, s, precision).  Work split: blockIdx.x = work item
    (tile, entry range, output row), blockIdx.y = block of output
    coefficients.  Inside a block the needed multipole coefficients are loaded
    into registers in chunks; within a chunk the multiply-adds are emitted in
    bands of equal total derivative order |n| + |m|, so that only one band of
    the (uniform) derivative tensor is live in scalar registers at a time; an
    scheduling barrier (not a memory clobber, so the tensor stays eligible
    for scalar loads) separates the groups so that the compiler cannot hoist
    every scalar load to the top of the loop."""
    T = "float" if fp32 else "double"
    V = "float4" if fp32 else "double2"
    VW = 4 if fp32 else 2
    fma = "__builtin_fmaf" if fp32 else "__builtin_fma"
    suf = "f32" if fp32 else "f64"
    ns = orders(p - s)
    ms = orders(p)[nterms(s - 1):]
    if harmonic:
        ns, ms = reduced(ns), reduced(ms)
    nm = len(ms)
    nl = len(ns)
    nmp = pad(nm, 4)
    nlp = pad(nl, 4)
    nd = pad(nterms(p), 16)
    scw = pad(p + 1, 4)
    opt = dict(DEFAULTS, **(opt or {}))
    max_acc = opt["acc32"] if fp32 else opt["acc64"]
    max_m = opt["m32"] if fp32 else opt["m64"]
    dgroup = opt["dgroup32"] if fp32 else opt["dgroup64"]
    blocks = split_blocks(nl, max_acc)
    name = f"m2l_p{p}_s{s}_{suf}" + ("_h" if harmonic else "")
    L = []
    # minwaves > 0: resident waves per SIMD the register allocation must allow
    wgw = opt["wgw"]
    NT = TILE * wgw
    lb = f"{NT}, {opt['minwaves']}" if opt["minwaves"] else f"{NT}"
    L.append(f"__global__ __launch_bounds__({lb}) void {name}(M2LArgs a)")
    L.append("{")
    L.append(f"    const int lane = threadIdx.x % {TILE};")
    if wgw > 1:
        # the waves of a workgroup split every item's entries and add their
        # partial sums in LDS (in wave order) before one row set is written;
        # the wave index is read from the first lane so that the compiler
        # knows it is uniform (else the piece bounds, class ids and table
        # pointer derived from it leave the scalar unit)
        L.append(f"    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / {TILE});")
        L.append(f"    __shared__ {T} red[{max(b - a for a, b in blocks)} * {TILE}];")
    L.append(f"    const {T} *__restrict__ Mb = (const {T} *)a.M;")
    L.append(f"    const {T} *__restrict__ Db = (const {T} *)a.D;")
    L.append(f"    const {T} *__restrict__ Sb = (const {T} *)a.sc;")
    L.append("    // this wave's pieces (equal total cost per wave, fixed by the host)")
    L.append("    const int p0 = a.wave_ptr[blockIdx.x], p1 = a.wave_ptr[blockIdx.x + 1];")
    L.append("    for (int item = p0; item < p1; ++item) {")
    L.append("    const int4 w = a.work[item];")
    L.append("    const int blk = w.x >> 24;")
    L.append(f"    {T} *__restrict__ out = ({T} *)a.part + ((size_t)w.w + lane) * {nlp};")
    for bi, (n0, n1) in enumerate(blocks):
        kw = "if" if bi == 0 else "else if"
        L.append(f"    {kw} (blk == {bi}) {{")
        for i in range(n0, n1):
            L.append(f"        {T} c{i} = 0;")
        minord = min(sum(ns[i]) for i in range(n0, n1))
        need = [j for j, m in enumerate(ms) if sum(m) + minord <= p]
        # chunks of the needed m, aligned to the vector width
        chunks, cur = [], []
        for j in need:
            if cur and (len(cur) >= max_m and j % VW == 0):
                chunks.append(cur)
                cur = []
            cur.append(j)
        if cur:
            chunks.append(cur)
        if wgw > 1:
            L.append(f"        const int uspan = w.z - w.y;")
            L.append(f"        const int ub = w.y + uspan * wv / {wgw}, ue = w.y + uspan * (wv + 1) / {wgw};")
            L.append("        for (int u = ub; u < ue; ++u) {")
        else:
            L.append("        for (int u = w.y; u < w.z; ++u) {")
        if opt["fairprio"] and wgw > 1:
            # issue priority falls as the wave works through its entries, so
            # a wave that lags (the younger workgroup's, which loses the
            # age-ordered arbitration) catches up instead of finishing alone
            L.append("            {")
            L.append("                const int stage = (u - ub) * 4 / (ue - ub);")
            L.append("                if (stage == 0) __builtin_amdgcn_s_setprio(3);")
            L.append("                else if (stage == 1) __builtin_amdgcn_s_setprio(2);")
            L.append("                else if (stage == 2) __builtin_amdgcn_s_setprio(1);")
            L.append("                else __builtin_amdgcn_s_setprio(0);")
            L.append("            }")
        L.append("            const int cls = a.ucls[u];")
        # the class tables are read-only for the whole kernel: reading them
        # through the constant address space lets the uniform loads go
        # through the scalar unit into SGPRs (an operand of every FMA)
        L.append(f"            const {T} __attribute__((address_space(4))) *const D = "
                 f"(const {T} __attribute__((address_space(4))) *)(Db + (size_t)cls * {nd});")
        L.append(f"            const {T} __attribute__((address_space(4))) *sc = "
                 f"(const {T} __attribute__((address_space(4))) *)(Sb + (size_t)cls * {scw});")
        L.append(f"            const {T} *__restrict__ Mr = Mb + (size_t)a.usrc[(size_t)u * {TILE} + lane] * {nmp};")
        comps = "xyzw"
        SB = '            __builtin_amdgcn_sched_barrier(0);'

        def mload(ch):
            return [f"            const {V} v{g} = *(const {V} *)(Mr + {g * VW});" for g in sorted(set(j // VW for j in ch))]

        def mscale(ch):
            if opt["scale_branch"]:
                # rho = r_A / r_B is 1 for pairs of one level: skip the scaling then
                out = [f"            {T} m{j} = v{j // VW}.{comps[j % VW]};" for j in ch]
                out.append("            if (sc[1] != 1) {")
                out += [f"                m{j} *= sc[{sum(ms[j])}];" for j in ch]
                out.append("            }")
                return out
            return [f"            const {T} m{j} = v{j // VW}.{comps[j % VW]} * sc[{sum(ms[j])}];" for j in ch]

        def chunk_groups(ch):
            # multiply-adds of this chunk, ordered by derivative index k = n + m
            # (bands of equal |k| are contiguous in the coefficient order),
            # in groups of at most dgroup distinct k, never spanning two bands
            terms = []
            for i in range(n0, n1):
                n = ns[i]
                for j in ch:
                    m = ms[j]
                    if sum(n) + sum(m) > p:
                        continue
                    terms.append((idx((n[0] + m[0], n[1] + m[1], n[2] + m[2])), i, j))
            terms.sort()
            groups, cur, curk = [], [], []
            for k, i, j in terms:
                band = sum(orders(p)[k])
                if curk and k != curk[-1] and (len(curk) >= dgroup or sum(orders(p)[curk[-1]]) != band):
                    groups.append((curk, cur))
                    cur, curk = [], []
                if not curk or curk[-1] != k:
                    curk.append(k)
                cur.append((k, i, j))
            if cur:
                groups.append((curk, cur))
            return groups

        def loads(g):
            base = f"D{g[2]}" if opt["launder"] else "D"
            return [f"            const {T} d{g[2]}_{k} = {base}[{k}];" for k in g[0]]

        def fmas(g):
            return [f"            c{i} = {fma}(d{g[2]}_{k}, m{j}, c{i});" for k, i, j in g[1]]

        mode = opt["pipeline"]
        mpre = opt["mpre"]
        if mpre:
            L.extend(mload(chunks[0]))
        for ci, ch in enumerate(chunks):
            if opt["launder"]:
                # a table pointer per chunk that the compiler cannot prove
                # equal to the previous one: it reloads the derivatives each
                # chunk needs instead of keeping the whole tensor live in
                # scalar registers
                L.append(f"            const {T} __attribute__((address_space(4))) *const D{ci} = D + (size_t)(a.zero * {ci + 1});")
            if not mpre:
                L.extend(mload(ch))
            L.extend(mscale(ch))
            groups = [(ks, ts, ci) for ks, ts in chunk_groups(ch)]
            mid = len(groups) // 2
            nxt = chunks[ci + 1] if ci + 1 < len(chunks) else None
            if mode == 0:
                for gi, g in enumerate(groups):
                    L.append(SB)
                    L.extend(loads(g))
                    L.extend(fmas(g))
                    if mpre and nxt and gi == mid:
                        L.append(SB)
                        L.extend(mload(nxt))
            elif mode == 1:
                # loads of group g+1 are issued before the multiply-adds of group g
                L.append(SB)
                L.extend(loads(groups[0]))
                for gi, g in enumerate(groups):
                    L.append(SB)
                    if gi + 1 < len(groups):
                        L.extend(loads(groups[gi + 1]))
                    L.extend(fmas(g))
                    if mpre and nxt and gi == mid:
                        L.append(SB)
                        L.extend(mload(nxt))
            else:
                # loads of group g+1 are issued half way through the
                # multiply-adds of group g: scalar loads complete out of
                # order, so the wait before group g+1 covers every scalar
                # load in flight; this way only group g+1's are
                L.append(SB)
                L.extend(loads(groups[0]))
                for gi, g in enumerate(groups):
                    f_ = fmas(g)
                    h = len(f_) // 2
                    L.append(SB)
                    L.extend(f_[:h])
                    L.append(SB)
                    if gi + 1 < len(groups):
                        L.extend(loads(groups[gi + 1]))
                    if mpre and nxt and gi == mid:
                        L.extend(mload(nxt))
                    L.append(SB)
                    L.extend(f_[h:])
        L.append("        }")
        if wgw > 1:
            for q in range(wgw):
                last = q == wgw - 1
                L.append(f"        if (wv == {q}) {{")
                for i in range(n0, n1):
                    slot = f"red[{i - n0} * {TILE} + lane]"
                    if q == 0:
                        L.append(f"            {slot} = c{i};")
                    elif not last:
                        L.append(f"            {slot} += c{i};")
                    else:
                        L.append(f"            out[{i}] = {slot} + c{i};")
                L.append("        }")
                if not last:
                    L.append("        __syncthreads();")
            L.append("        __syncthreads();   // red is reused by the next item")
        else:
            for i in range(n0, n1):
                L.append(f"        out[{i}] = c{i};")
        L.append("    }")
    L.append("    }")
    L.append("}")
    launcher = f"""
static hipError_t launch_{name}(const M2LArgs &a, int nwaves, hipStream_t st)
{{
    hipLaunchKernelGGL({name}, dim3(nwaves), dim3({NT}), 0, st, a);
    return hipGetLastError();
}}

static int occ_{name}()
{{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, {name}, {NT}, 0) != hipSuccess) return 1;
    return per_cu > 0 ? per_cu : 1;
}}
"""
    fma_per_block = []
    for (n0, n1) in blocks:
        fma_per_block.append(sum(1 for i in range(n0, n1) for m in ms if sum(m) + sum(ns[i]) <= p))
    meta = dict(name=name, nl_pad=nlp, nm_pad=nmp, nd=nd, nblocks=len(blocks), scw=scw,
                blo=[b[0] for b in blocks] + [blocks[-1][1]], bfma=fma_per_block)
    return "\n".join(L) + "\n" + launcher, meta


def gen_file(s, fp32, opt=None, harmonic=False):
    suf = ("f32" if fp32 else "f64") + ("_h" if harmonic else "")
    parts = ["// Generated by gen_m2l.py; do not edit.", "#include <algorithm>", '#include "fmm_internal.h"', ""]
    metas = []
    for p in range(s + 1, P_MAX + 1):
        code, meta = gen_kernel(p, s, fp32, opt, harmonic)
        parts.append(code)
        metas.append((p, meta))
    parts.append(f"bool m2l_lookup_s{s}_{suf}(int p, M2LVariant *v)")
    parts.append("{")
    parts.append("    switch (p) {")
    for p, m in metas:
        blo = ", ".join(str(x) for x in m["blo"] + [0] * (17 - len(m["blo"])))
        bf = ", ".join(str(x) for x in m["bfma"] + [0] * (16 - len(m["bfma"])))
        parts.append(f"    case {p}: *v = M2LVariant{{launch_{m['name']}, occ_{m['name']}, {m['nl_pad']}, {m['nm_pad']}, "
                     f"{m['nd']}, {m['nblocks']}, {{{blo}}}, {{{bf}}}}}; return true;")
    parts.append("    default: return false;")
    parts.append("    }")
    parts.append("}")
    return "\n".join(parts) + "\n"


def main(outdir, opt=None):
    os.makedirs(outdir, exist_ok=True)
    written = []
    for s in (0, 1, 2):
        for fp32, h in ((True, False), (False, False), (True, True), (False, True)):
            fn = os.path.join(outdir, f"m2l_s{s}_{'f32' if fp32 else 'f64'}{'_h' if h else ''}.hip")
            txt = gen_file(s, fp32, opt, h)
            old = open(fn).read() if os.path.exists(fn) else None
            if old != txt:
                with open(fn, "w") as f:
                    f.write(txt)
            written.append(fn)
    return written


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "_build/gen")
