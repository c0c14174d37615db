// Host construction of the canonical octree, the dual-tree interaction lists
// and the M2L work tiling (Section 3.2 of Pepper & Fangohr, arXiv 2005.12351).
//
// Canonical definitions (shared by specification, not by code, with the
// test oracle): cube root box of side W = largest extent, corner lo; 21-bit
// integer coordinates floor((x - lo) * 2^21 / W) clamped to 2^21 - 1; Morton
// key with x as the most significant bit of every octal digit; stable sort
// by key; a cell is split when it holds more than ncrit particles and is
// above level 21; empty children are not created; cells are stored
// level-major in ascending key order.  Geometry in units of h = W 2^-22:
// centre (2 i + 1) 2^(21-l), radius (half side) 2^(21-l).
//
// This file must be compiled without floating-point contraction: the
// quantisation and the acceptance test have to round exactly as specified.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "fmm_internal.h"

namespace {

// spread the low 21 bits of v so that bit b lands at bit 3b
inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

inline uint64_t morton_key(uint32_t qx, uint32_t qy, uint32_t qz)
{
    return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

}  // namespace

int host_build_tree(const double *pos, int64_t n, int ncrit, HostTree &t)
{
    t = HostTree();
    t.n = n;
    double hi[3];
    for (int d = 0; d < 3; ++d) t.lo[d] = hi[d] = pos[d];
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            t.lo[d] = std::min(t.lo[d], pos[3 * i + d]);
            hi[d] = std::max(hi[d], pos[3 * i + d]);
        }
    double W = std::max(hi[0] - t.lo[0], std::max(hi[1] - t.lo[1], hi[2] - t.lo[2]));
    if (W == 0.0) W = 1.0;
    t.W = W;
    t.h = std::ldexp(W, -22);
    const double scale = std::ldexp(1.0, kMaxLevel) / W;
    const int64_t qmax = (int64_t(1) << kMaxLevel) - 1;

    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            double v = (pos[3 * i + d] - t.lo[d]) * scale;
            int64_t qi = (int64_t)std::floor(v);
            q[d] = (uint32_t)std::min(std::max(qi, (int64_t)0), qmax);
        }
        key[i] = morton_key(q[0], q[1], q[2]);
    }
    t.perm.resize(n);
    std::iota(t.perm.begin(), t.perm.end(), 0);
    std::stable_sort(t.perm.begin(), t.perm.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    t.key.resize(n);
    for (int64_t i = 0; i < n; ++i) t.key[i] = key[t.perm[i]];

    // cells level by level
    auto push = [&](int l, int32_t x, int32_t y, int32_t z, int64_t f, int64_t c, int64_t par) {
        t.level.push_back(l);
        t.ix.push_back(x);
        t.ix.push_back(y);
        t.ix.push_back(z);
        t.first.push_back(f);
        t.count.push_back(c);
        t.parent.push_back(par);
    };
    push(0, 0, 0, 0, 0, n, -1);
    t.level_ptr.push_back(0);
    int64_t lb = 0, le = 1;
    for (int l = 0;; ++l) {
        t.level_ptr.push_back(le);
        if (l == kMaxLevel) break;
        const int shift = 3 * (kMaxLevel - l - 1);
        for (int64_t c = lb; c < le; ++c) {
            if (t.count[c] <= ncrit) continue;
            const uint64_t *kb = t.key.data() + t.first[c];
            const uint64_t *ke = kb + t.count[c];
            for (int dig = 0; dig < 8; ++dig) {
                // sorted keys: the particles with this digit form one run
                const uint64_t *a = std::partition_point(kb, ke, [&](uint64_t k) { return (int)((k >> shift) & 7) < dig; });
                const uint64_t *b = std::partition_point(a, ke, [&](uint64_t k) { return (int)((k >> shift) & 7) <= dig; });
                if (a == b) continue;
                push(l + 1, 2 * t.ix[3 * c] + (dig >> 2), 2 * t.ix[3 * c + 1] + ((dig >> 1) & 1),
                     2 * t.ix[3 * c + 2] + (dig & 1), (int64_t)(a - t.key.data()), (int64_t)(b - a), c);
            }
        }
        if ((int64_t)t.level.size() == le) break;
        lb = le;
        le = (int64_t)t.level.size();
    }
    const int64_t nc = t.ncells();
    t.child0.assign(nc, -1);
    t.nchild.assign(nc, 0);
    for (int64_t c = 1; c < nc; ++c) {
        int64_t pa = t.parent[c];
        if (t.child0[pa] < 0) t.child0[pa] = c;
        t.nchild[pa]++;
    }
    return FMM_OK;
}

void host_dual_traversal(HostTree &t, double theta)
{
    const int64_t nc = t.ncells();
    std::vector<std::vector<int64_t>> m2l(nc), p2p(nc);
    const double th2 = theta * theta;
    auto geom = [&](int64_t c, int64_t *cen) {
        const int64_t r = int64_t(1) << (kMaxLevel - t.level[c]);
        for (int d = 0; d < 3; ++d) cen[d] = (2 * (int64_t)t.ix[3 * c + d] + 1) * r;
        return r;
    };
    std::vector<std::pair<int64_t, int64_t>> stack;   // (source A, target B)
    stack.emplace_back(0, 0);
    while (!stack.empty()) {
        auto [A, B] = stack.back();
        stack.pop_back();
        int64_t ca[3], cb[3];
        const int64_t ra = geom(A, ca), rb = geom(B, cb);
        int64_t d2 = 0;
        for (int d = 0; d < 3; ++d) d2 += (cb[d] - ca[d]) * (cb[d] - ca[d]);
        const double s = (double)(ra + rb);
        const bool leafA = t.nchild[A] == 0, leafB = t.nchild[B] == 0;
        if (s * s < th2 * (double)d2) {
            m2l[B].push_back(A);
        } else if (leafA && leafB) {
            p2p[B].push_back(A);
        } else if (leafB || (!leafA && ra > rb)) {
            for (int64_t a = t.child0[A]; a < t.child0[A] + t.nchild[A]; ++a) stack.emplace_back(a, B);
        } else if (leafA || rb > ra) {
            for (int64_t b = t.child0[B]; b < t.child0[B] + t.nchild[B]; ++b) stack.emplace_back(A, b);
        } else {
            for (int64_t a = t.child0[A]; a < t.child0[A] + t.nchild[A]; ++a)
                for (int64_t b = t.child0[B]; b < t.child0[B] + t.nchild[B]; ++b) stack.emplace_back(a, b);
        }
    }
    auto csr = [&](std::vector<std::vector<int64_t>> &lists, std::vector<int64_t> &ptr, std::vector<int64_t> &src) {
        ptr.assign(nc + 1, 0);
        for (int64_t c = 0; c < nc; ++c) ptr[c + 1] = ptr[c] + (int64_t)lists[c].size();
        src.resize(ptr[nc]);
        for (int64_t c = 0; c < nc; ++c) {
            std::sort(lists[c].begin(), lists[c].end());
            std::copy(lists[c].begin(), lists[c].end(), src.begin() + ptr[c]);
        }
    };
    csr(m2l, t.m2l_ptr, t.m2l_src);
    csr(p2p, t.p2p_ptr, t.p2p_src);
}

// ---------------------------------------------------------------------------
// M2L tiling.  Target cells with a non-empty M2L list are grouped 64 to a
// tile (one GPU lane per target).  Cells of one level and one position
// inside their parent have identical relative source layouts away from the
// domain boundary, so tiles are formed in that order.  A tile iterates over
// the union of its targets' translation classes; a class is the exact
// dimensionless geometry of a pair, ((z_B - z_A) / r_B, r_A / r_B), so one
// derivative tensor serves every lane at a given step.
void build_m2l_tiling(const HostTree &t, M2LTiling &out)
{
    out = M2LTiling();
    const int64_t nc = t.ncells();
    std::vector<int32_t> tg;
    for (int64_t c = 0; c < nc; ++c)
        if (t.m2l_ptr[c + 1] > t.m2l_ptr[c]) tg.push_back((int32_t)c);
    auto oct = [&](int32_t c) { return ((t.ix[3 * c] & 1) << 2) | ((t.ix[3 * c + 1] & 1) << 1) | (t.ix[3 * c + 2] & 1); };
    // a cell whose list is shorter than most of its level's lists sits near
    // the domain boundary; list length (coarsely) groups cells with similar
    // truncated neighbourhoods, which shrinks the per-tile union
    std::stable_sort(tg.begin(), tg.end(), [&](int32_t a, int32_t b) {
        if (t.level[a] != t.level[b]) return t.level[a] < t.level[b];
        if (oct(a) != oct(b)) return oct(a) < oct(b);
        const int64_t la = t.m2l_ptr[a + 1] - t.m2l_ptr[a], lb = t.m2l_ptr[b + 1] - t.m2l_ptr[b];
        return la > lb;
    });
    out.ntiles = (int)((tg.size() + kTileW - 1) / kTileW);
    out.tile_cell.assign((size_t)out.ntiles * kTileW, -1);
    for (size_t i = 0; i < tg.size(); ++i) out.tile_cell[i] = tg[i];

    struct Key {
        int64_t dx, dy, dz;
        int dl;
        bool operator==(const Key &o) const { return dx == o.dx && dy == o.dy && dz == o.dz && dl == o.dl; }
    };
    struct KeyHash {
        size_t operator()(const Key &k) const
        {
            uint64_t h = (uint64_t)k.dx * 0x9E3779B97F4A7C15ULL ^ (uint64_t)k.dy * 0xC2B2AE3D27D4EB4FULL ^
                         (uint64_t)k.dz * 0x165667B19E3779F9ULL ^ (uint64_t)(k.dl + 64) * 0x27D4EB2F165667C5ULL;
            return (size_t)(h ^ (h >> 29));
        }
    };
    std::unordered_map<Key, int32_t, KeyHash> cls;
    auto class_of = [&](int64_t A, int64_t B) {
        const int la = t.level[A], lb = t.level[B];
        const int lmax = std::max(la, lb);
        // offsets in units of the smaller radius 2^(21 - lmax)
        int64_t d[3];
        for (int k = 0; k < 3; ++k) {
            const int64_t cb = (2 * (int64_t)t.ix[3 * B + k] + 1) << (lmax - lb);
            const int64_t ca = (2 * (int64_t)t.ix[3 * A + k] + 1) << (lmax - la);
            d[k] = cb - ca;
        }
        Key key{d[0], d[1], d[2], lb - la};
        auto it = cls.find(key);
        if (it != cls.end()) return it->second;
        int32_t id = (int32_t)cls.size();
        cls.emplace(key, id);
        const double unit = std::ldexp(1.0, lb - lmax);   // smaller radius / r_B
        out.cls_geom.push_back((double)d[0] * unit);
        out.cls_geom.push_back((double)d[1] * unit);
        out.cls_geom.push_back((double)d[2] * unit);
        out.cls_geom.push_back(std::ldexp(1.0, lb - la));  // r_A / r_B
        return id;
    };

    out.tile_uoff.assign(out.ntiles + 1, 0);
    std::vector<std::pair<int32_t, int32_t>> ent;   // (class, lane) -> source
    std::vector<int32_t> entsrc;
    for (int ti = 0; ti < out.ntiles; ++ti) {
        ent.clear();
        entsrc.clear();
        std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> items;
        for (int l = 0; l < kTileW; ++l) {
            const int32_t B = out.tile_cell[(size_t)ti * kTileW + l];
            if (B < 0) continue;
            for (int64_t e = t.m2l_ptr[B]; e < t.m2l_ptr[B + 1]; ++e) {
                const int64_t A = t.m2l_src[e];
                items.push_back({{class_of(A, B), l}, (int32_t)A});
                out.pairs++;
            }
        }
        std::sort(items.begin(), items.end());
        int32_t prev = -1;
        for (auto &it : items) {
            const int32_t c = it.first.first;
            if (c != prev) {
                out.ucls.push_back(c);
                out.usrc.insert(out.usrc.end(), kTileW, (int32_t)nc);   // zero row
                prev = c;
            }
            out.usrc[out.usrc.size() - kTileW + it.first.second] = it.second;
        }
        out.tile_uoff[ti + 1] = (int32_t)out.ucls.size();
    }
    out.nclasses = (int)cls.size();
    out.nentries = (int64_t)out.ucls.size();

}

void build_m2l_work(const M2LTiling &tl, const M2LVariant &v, int nwaves, M2LWork &out)
{
    out = M2LWork();
    const int nb = v.nblocks;
    // cost of one list entry in output block b: its multiply-adds plus a fixed
    // overhead for the gather and the loop
    std::vector<double> ecost(nb);
    for (int b = 0; b < nb; ++b) ecost[b] = (double)v.bfma[b] + 32.0;
    double total = 0.0;
    for (int ti = 0; ti < tl.ntiles; ++ti)
        for (int b = 0; b < nb; ++b) total += (double)(tl.tile_uoff[ti + 1] - tl.tile_uoff[ti]) * ecost[b];
    nwaves = std::max(1, nwaves);
    const double per = total / nwaves;
    out.chunk0.assign((size_t)tl.ntiles * nb, 0);
    out.nchunk.assign((size_t)tl.ntiles * nb, 0);
    out.wave_ptr.push_back(0);
    int64_t rowset = 0;
    int wave = 0;
    double acc = 0.0;   // cost already given to the current wave
    for (int ti = 0; ti < tl.ntiles; ++ti)
        for (int b = 0; b < nb; ++b) {
            const size_t g = (size_t)ti * nb + b;
            out.chunk0[g] = (int32_t)rowset;
            int64_t u = tl.tile_uoff[ti];
            const int64_t ue = tl.tile_uoff[ti + 1];
            while (u < ue) {
                // entries this wave can still take
                int64_t take = (int64_t)std::ceil((per - acc) / ecost[b] - 1e-9);
                if (wave == nwaves - 1) take = ue - u;
                take = std::max<int64_t>(1, std::min<int64_t>(take, ue - u));
                out.work.insert(out.work.end(), {ti | (b << 24), (int32_t)u, (int32_t)(u + take), (int32_t)(rowset * kTileW)});
                ++rowset;
                out.nchunk[g]++;
                u += take;
                acc += (double)take * ecost[b];
                if (acc >= per - 1e-9 && wave < nwaves - 1) {
                    out.wave_ptr.push_back((int32_t)(out.work.size() / 4));
                    ++wave;
                    acc = 0.0;
                }
            }
        }
    while ((int)out.wave_ptr.size() < nwaves + 1) out.wave_ptr.push_back((int32_t)(out.work.size() / 4));
    out.nwaves = nwaves;
    out.nrows = rowset * kTileW;
}
