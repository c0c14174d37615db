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

Matrix cores.  The "_hm" kernels compute the same FP32 harmonic-basis
contraction on the MFMA units.  v_mfma_f32_4x4x1_16b_f32 is a batch of
sixteen 4x4 outer products: block b of the wave gets D[r][c] += A[r] B[c],
with A[r] from lane 4b+r and B[c] from lane 4b+c.  Lane l = 4b+c holds the
scaled multipole coefficient m_j of its own target's source (B) and four
accumulators, the local outputs 4g..4g+3 of its target; the class operand
A[r] = D_{n_{4g+r}+m_j} is the same for every block, so it is broadcast from
one block (CBSZ = 4, ABID = k): a single VGPR holds the operands of sixteen
consecutive multiply-add slots (j, g), gathered per lane from the class's
derivative row through a fixed index table (an index past the tensor reads a
zero for outputs a slot does not reach).  Per slot: 64 targets x 4 outputs
in one instruction, twice the FP32 multiply-add rate of the vector unit.

Usage: python gen_m2l.py OUTDIR  -> OUTDIR/m2l_s{0,1,2}_{f32,f64}[_h].hip, m2l_s{0,1,2}_f32_hm.hip
"""
import os
import sys

P_MAX = 10
TILE = 64

# code-shape options (register blocking, scalar-load pipelining, waves per
# workgroup); the defaults are the measured best on gfx950
DEFAULTS = {"acc32": 128, "m32": 64, "acc64": 64, "m64": 32, "dgroup32": 32, "dgroup64": 16, "pipeline": 1,
            "mpre": 0, "launder": 1, "scale_branch": 0, "minwaves": 0, "wgw": 4, "fairprio": 1,
            "mch": 32, "mdist": 4, "mwaves": 2, "mbarrier": 1, "mbalance": 0, "mpipe": 1, "malign": 1}


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


def mfma_schedule(p, s, mch, dist, balance=False):
    """Multiply-add slots (j, g) of the harmonic contraction for the matrix
    cores, in issue order, with accumulator copies: a slot whose output group
    was used fewer than `dist` slots before goes to another copy of that
    group's accumulators (added together at the end), so that no MFMA waits
    for the previous one's result.  Returns the chunks of the multipole row
    (lists of j, at most `mch`, starting at multiples of 4) and per chunk the
    slots as (j, g, copy).  balance: the chunks take whole quads of j (one
    vector load each) so that they hold about the same number of slots,
    low orders (many slots) beside high orders (few)."""
    ns = reduced(orders(p - s))
    ms = reduced(orders(p)[nterms(s - 1):])
    nl = len(ns)
    ng = (nl + 3) // 4
    chunks = [list(range(c, min(len(ms), c + mch))) for c in range(0, len(ms), mch)]
    if balance:
        def nslots(j):
            return sum(1 for g in range(ng)
                       if any(sum(ns[i]) + sum(ms[j]) <= p for i in range(4 * g, min(nl, 4 * g + 4))))
        quads = [list(range(q, min(len(ms), q + 4))) for q in range(0, len(ms), 4)]
        k = len(chunks)
        cost = sorted(((sum(nslots(j) for j in qd), qi) for qi, qd in enumerate(quads)), reverse=True)
        bins = [[] for _ in range(k)]
        load = [0] * k
        for c, qi in cost:
            b = min((b for b in range(k) if len(bins[b]) < mch // 4), key=lambda b: load[b])
            bins[b].append(qi)
            load[b] += c
        chunks = [[j for qi in sorted(bn) for j in quads[qi]] for bn in bins if bn]
    out = []
    for ch in chunks:
        queues = {}
        for j in ch:
            for g in range(ng):
                if any(sum(ns[i]) + sum(ms[j]) <= p for i in range(4 * g, min(nl, 4 * g + 4))):
                    queues.setdefault(g, []).append(j)
        last = {}            # (g, copy) -> step of its last use
        ncopy = {g: 1 for g in queues}
        seq, step = [], 0
        while any(queues.values()):
            # the group with the most remaining slots that has a free copy
            best = None
            for g, q in sorted(queues.items(), key=lambda kv: -len(kv[1])):
                if not q:
                    continue
                free = [c for c in range(ncopy[g]) if step - last.get((g, c), -dist) >= dist]
                if free:
                    best = (g, free[0])
                    break
            if best is None:
                g = max((g for g in queues if queues[g]), key=lambda g: len(queues[g]))
                if ncopy[g] < 4:
                    ncopy[g] += 1
                    best = (g, ncopy[g] - 1)
                else:
                    best = (g, min(range(ncopy[g]), key=lambda c: last.get((g, c), -dist)))
            g, c = best
            j = queues[g].pop(0)
            seq.append((j, g, c))
            last[(g, c)] = step
            step += 1
        out.append(seq)
    return chunks, out


def gen_kernel_mfma(p, s, opt=None):
    """FP32 harmonic-basis M2L on the matrix cores (see the module header).
    Same arguments, work items, waves per workgroup and partial rows as the
    vector kernels (one output block holding every local output)."""
    opt = dict(DEFAULTS, **(opt or {}))
    ns = reduced(orders(p - s))
    ms = reduced(orders(p)[nterms(s - 1):])
    nl, nm = len(ns), len(ms)
    # rows aligned to 128-byte lines: a chunk of 32 coefficients is one line
    nlp, nmp = pad(nl, 4), pad(nm, 32 if opt["malign"] else 4)
    nd = pad(nterms(p), 16)
    scw = pad(p + 1, 4)
    zero = nterms(p)          # an entry of every derivative row that is zero (nd > nterms(p))
    assert zero < nd
    ng = (nl + 3) // 4
    assert 4 * ng == nlp
    chunks, sched = mfma_schedule(p, s, opt["mch"], opt["mdist"], opt["mbalance"])
    # operand groups: 16 consecutive slots of a chunk share one VGPR
    groups = []              # per group: list of (j, g, copy)
    for seq in sched:
        for k in range(0, len(seq), 16):
            groups.append(seq[k:k + 16])
    nw = len(groups)
    itab = []
    for grp in groups:
        row = []
        for slot in range(16):
            for r in range(4):
                v = zero
                if slot < len(grp):
                    j, g, _ = grp[slot]
                    i = 4 * g + r
                    if i < nl and sum(ns[i]) + sum(ms[j]) <= p:
                        n, m = ns[i], ms[j]
                        v = idx((n[0] + m[0], n[1] + m[1], n[2] + m[2]))
                row.append(4 * v)      # byte offset in the class's row
        itab.append(row)
    copies = {}
    for seq in sched:
        for j, g, c in seq:
            copies[g] = max(copies.get(g, 0), c + 1)
    wgw = opt["wgw"]
    NT = TILE * wgw
    name = f"m2l_p{p}_s{s}_f32_hm"
    L = []
    # operand byte offsets, two 16-bit values per word: group 2k in the low half
    words = []
    for k in range(0, nw, 2):
        lo = itab[k]
        hi = itab[k + 1] if k + 1 < nw else [0] * 64
        words.append([a | (b << 16) for a, b in zip(lo, hi)])
    assert max(max(r) for r in itab) < 65536
    flat = ", ".join(str(v) for w_ in words for v in w_)
    L.append(f"static __device__ const unsigned kIdx_{name}[{len(words) * 64}] = {{{flat}}};")
    L.append(f"__global__ __launch_bounds__({NT}, {opt['mwaves']}) void {name}(M2LArgs a)")
    L.append("{")
    L.append(f"    const int lane = threadIdx.x % {TILE};")
    L.append(f"    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / {TILE});")
    L.append(f"    __shared__ float red[{nlp} * {TILE}];")
    # the operand index table, read from LDS where a group of slots needs it
    L.append(f"    __shared__ unsigned ixs[{len(words) * 64}];")
    L.append(f"    for (int k = threadIdx.x; k < {len(words) * 64}; k += {NT}) ixs[k] = kIdx_{name}[k];")
    L.append("    __syncthreads();")
    L.append("    const float *__restrict__ Mb = (const float *)a.M;")
    L.append("    const char *__restrict__ Db = (const char *)a.D;")
    L.append("    const float *__restrict__ Sb = (const float *)a.sc;")
    L.append("    const int p0 = a.wave_ptr[blockIdx.x], p1 = a.wave_ptr[blockIdx.x + 1];")
    L.append("    for (int item = p0; item < p1; ++item) {")
    L.append("    const int4 w = a.work[item];")
    L.append(f"    float *__restrict__ out = a.part ? (float *)a.part + ((size_t)w.w + lane) * {nlp} : nullptr;")
    for g in range(ng):
        for c in range(copies.get(g, 1)):
            L.append(f"    f32x4 acc{g}_{c} = {{0.f, 0.f, 0.f, 0.f}};")
    L.append("    const int uspan = w.z - w.y;")
    L.append(f"    const int ub = w.y + uspan * wv / {wgw}, ue = w.y + uspan * (wv + 1) / {wgw};")
    L.append("    for (int u = ub; u < ue; ++u) {")
    if opt["fairprio"]:
        L.append("        {")
        L.append("            const int stage = (u - ub) * 4 / (ue - ub);")
        L.append("            if (stage == 0) __builtin_amdgcn_s_setprio(3);")
        L.append("            else if (stage == 1) __builtin_amdgcn_s_setprio(2);")
        L.append("            else if (stage == 2) __builtin_amdgcn_s_setprio(1);")
        L.append("            else __builtin_amdgcn_s_setprio(0);")
        L.append("        }")
    L.append("        const int cls = a.ucls[u];")
    L.append(f"        const char *__restrict__ Dr = Db + (size_t)cls * {nd * 4};")
    L.append(f"        const float __attribute__((address_space(4))) *sc = "
             f"(const float __attribute__((address_space(4))) *)(Sb + (size_t)cls * {scw});")
    L.append(f"        const float *__restrict__ Mr = Mb + (size_t)a.usrc[(size_t)u * {TILE} + lane] * {nmp};")
    comps = "xyzw"
    # operand groups of each chunk (first global group index, count)
    gstart, gi = [], 0
    for seq in sched:
        gstart.append(gi)
        gi += (len(seq) + 15) // 16

    def loads(ci, mr="Mr", dr="Dr", decl=True):
        ch, seq = chunks[ci], sched[ci]
        out = []
        kw = "const " if decl else ""
        t4, t1 = ("float4 ", "float ") if decl else ("", "")
        for q in sorted(set(j // 4 for j in ch)):
            out.append(f"        {kw}{t4}v{q} = *(const float4 *)({mr} + {4 * q});")
        for k in range((len(seq) + 15) // 16):
            wk = gstart[ci] + k
            word = f"ixs[{(wk // 2) * 64} + lane]"
            half = f"({word} & 0xffffu)" if wk % 2 == 0 else f"({word} >> 16)"
            out.append(f"        {kw}{t1}w{wk} = *(const float *)({dr} + {half});")
        return out

    def mfmas(ci):
        ch, seq = chunks[ci], sched[ci]
        out = []
        for j in ch:
            out.append(f"        const float m{j} = v{j // 4}.{comps[j % 4]} * sc[{sum(ms[j])}];")
        for k in range((len(seq) + 15) // 16):
            wk = gstart[ci] + k
            for slot, (j, g, c) in enumerate(seq[16 * k:16 * k + 16]):
                out.append(f"        acc{g}_{c} = __builtin_amdgcn_mfma_f32_4x4x1f32(w{wk}, m{j}, acc{g}_{c}, 4, {slot}, 0);")
        return out

    def entry_ptrs(u, suf):
        return [f"        const char *__restrict__ Dr{suf} = Db + (size_t)a.ucls[{u}] * {nd * 4};",
                f"        const float *__restrict__ Mr{suf} = Mb + (size_t)a.usrc[(size_t)({u}) * {TILE} + lane] * {nmp};"]

    SB = "        __builtin_amdgcn_sched_barrier(0);"
    nchunk = len(chunks)
    mpipe = opt["mpipe"] if nchunk > 1 else min(opt["mpipe"], 1)
    if mpipe == 2:
        # the first chunk's operands of entry u+1 load while entry u's last
        # chunk multiplies (loop-carried registers); every other chunk's
        # while the previous chunk of the same entry multiplies
        pre = [x.replace("        ", "    ", 1) for x in loads(0, "Mr0", "Dr0", False)]
        decl = [f"    float4 v{q};" for q in sorted(set(j // 4 for j in chunks[0]))]
        decl += [f"    float w{gstart[0] + k};" for k in range((len(sched[0]) + 15) // 16)]
        i_loop = L.index("    for (int u = ub; u < ue; ++u) {")
        head = decl + ["    if (ub < ue) {"] + ["    " + x for x in entry_ptrs("ub", "0")] + ["    " + x for x in pre] + ["    }"]
        L[i_loop:i_loop] = head
        for ci in range(nchunk):
            L.append(SB)
            if ci + 1 < nchunk:
                L.extend(loads(ci + 1))
            else:
                L.append("        {")
                L.append("        const int un = u + 1 < ue ? u + 1 : u;")
                L.extend(["    " + x for x in entry_ptrs("un", "0")])
                L.extend(["    " + x for x in loads(0, "Mr0", "Dr0", False)])
                L.append("        }")
            L.extend(mfmas(ci))
    elif mpipe == 1:
        # the loads of chunk c+1 are issued before the multiply-adds of chunk c
        L.extend(loads(0))
        for ci in range(nchunk):
            L.append(SB)
            if ci + 1 < nchunk:
                L.extend(loads(ci + 1))
            L.extend(mfmas(ci))
    else:
        for ci in range(nchunk):
            if opt["mbarrier"] and ci > 0:
                # keeps the next chunk's loads from being hoisted above this
                # point, which would hold every chunk's operands at once
                L.append(SB)
            L.extend(loads(ci))
            L.extend(mfmas(ci))
    L.append("    }")
    for g in range(ng):
        for c in range(1, copies.get(g, 1)):
            L.append(f"    acc{g}_0 += acc{g}_{c};")
    for q in range(wgw):
        last = q == wgw - 1
        L.append(f"    if (wv == {q}) {{")
        for g in range(ng):
            for r in range(4):
                i = 4 * g + r
                slot_ = f"red[{i} * {TILE} + lane]"
                if q == 0:
                    L.append(f"        {slot_} = acc{g}_0[{r}];")
                elif not last:
                    L.append(f"        {slot_} += acc{g}_0[{r}];")
                else:
                    L.append(f"        out[{i}] = {slot_} + acc{g}_0[{r}];")
        L.append("    }")
        if not last:
            L.append("    __syncthreads();")
    L.append("    __syncthreads();   // red is reused by the next item")
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
    nslots = sum(len(q) for q in sched)
    meta = dict(name=name, nl_pad=nlp, nm_pad=nmp, nd=nd, nblocks=1, scw=scw, blo=[0, nl], bfma=[4 * nslots])
    return "\n".join(L) + "\n" + launcher, meta


def gen_file(s, fp32, opt=None, harmonic=False, mfma=False):
    suf = ("f32" if fp32 else "f64") + ("_h" if harmonic else "") + ("m" if mfma else "")
    parts = ["// Generated by gen_m2l.py; do not edit.", "#include <algorithm>", '#include "fmm_internal.h"', ""]
    if mfma:
        parts.append("typedef float f32x4 __attribute__((ext_vector_type(4)));")
        parts.append("")
    metas = []
    for p in range(s + 1, P_MAX + 1):
        code, meta = gen_kernel_mfma(p, s, opt) if mfma else gen_kernel(p, s, fp32, opt, harmonic)
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
    for s in (0, 1, 2, 3):
        for fp32, h, mf in ((True, False, False), (False, False, False), (True, True, False), (False, True, False),
                            (True, True, True)):
            fn = os.path.join(outdir, f"m2l_s{s}_{'f32' if fp32 else 'f64'}{'_h' if h else ''}{'m' if mf else ''}.hip")
            txt = gen_file(s, fp32, opt, h, mf)
            old = open(fn).read() if os.path.exists(fn) else None
            if old != txt:
                with open(fn, "w") as f:
                    f.write(txt)
            written.append(fn)
    return written


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "_build/gen")
