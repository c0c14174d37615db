// Host scheduling of the M2L work (Section 3.2 of Pepper & Fangohr, arXiv
// 2005.12351): target cells grouped into 64-lane tiles, the translation
// classes of every tile, and the cut of the tiled work into equal-cost pieces
// per wave.  The tree and the lists themselves are built on the GPU.
//
// Compiled without floating-point contraction, like the rest of the host
// code: the class geometry is formed from exact integers and powers of two.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "fmm_internal.h"

// ---------------------------------------------------------------------------
// M2L tiling.  Target cells with a non-empty M2L list are grouped 64 to a
// tile (one GPU lane per target).  Cells of one level and one position
// inside their parent have identical relative source layouts away from the
// domain boundary, and near it equal truncations (see below), so tiles are
// formed in that order.  A tile iterates over
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
    // Near the domain boundary a cell's list is truncated on the sides that
    // touch the boundary.  Its neighbourhood signature, the smallest and
    // largest offset per axis of its same-level sources, identifies the
    // truncation (in a uniform region cells with equal signatures have equal
    // class sets), so tiles are formed in (level, octant, signature) order;
    // the list length breaks ties.
    struct Key {
        int32_t lo[3], hi[3];
        int64_t len;
    };
    std::vector<Key> key(nc);
    for (int32_t c : tg) {
        Key k{{0, 0, 0}, {0, 0, 0}, t.m2l_ptr[c + 1] - t.m2l_ptr[c]};
        bool any = false;
        for (int64_t e = t.m2l_ptr[c]; e < t.m2l_ptr[c + 1]; ++e) {
            const int64_t A = t.m2l_src[e];
            if (t.level[A] != t.level[c]) continue;
            for (int d = 0; d < 3; ++d) {
                const int32_t o = t.ix[3 * A + d] - t.ix[3 * c + d];
                k.lo[d] = any ? std::min(k.lo[d], o) : o;
                k.hi[d] = any ? std::max(k.hi[d], o) : o;
            }
            any = true;
        }
        key[c] = k;
    }
    std::stable_sort(tg.begin(), tg.end(), [&](int32_t a, int32_t b) {
        if (t.level[a] != t.level[b]) return t.level[a] < t.level[b];
        if (oct(a) != oct(b)) return oct(a) < oct(b);
        const Key &ka = key[a], &kb = key[b];
        for (int d = 0; d < 3; ++d) {
            if (ka.lo[d] != kb.lo[d]) return ka.lo[d] < kb.lo[d];
            if (ka.hi[d] != kb.hi[d]) return ka.hi[d] < kb.hi[d];
        }
        return ka.len > kb.len;
    });
    out.ntiles = (int)((tg.size() + kTileW - 1) / kTileW);
    out.tile_cell.assign((size_t)out.ntiles * kTileW, -1);
    for (size_t i = 0; i < tg.size(); ++i) out.tile_cell[i] = tg[i];

    // translation classes: flat open-addressing table keyed by the exact
    // integer pair geometry (offsets in units of the smaller radius, level
    // difference); ids in order of first appearance
    struct Slot {
        int64_t dx, dy, dz;
        int32_t dl, id;
    };
    std::vector<Slot> table(4096, Slot{0, 0, 0, 0, -1});
    size_t mask = table.size() - 1, used = 0;
    auto hash = [](int64_t dx, int64_t dy, int64_t dz, int dl) {
        uint64_t h = (uint64_t)dx * 0x9E3779B97F4A7C15ULL ^ (uint64_t)dy * 0xC2B2AE3D27D4EB4FULL ^
                     (uint64_t)dz * 0x165667B19E3779F9ULL ^ (uint64_t)(dl + 64) * 0x27D4EB2F165667C5ULL;
        return (size_t)(h ^ (h >> 29));
    };
    auto grow = [&]() {
        std::vector<Slot> old(std::move(table));
        table.assign(old.size() * 2, Slot{0, 0, 0, 0, -1});
        mask = table.size() - 1;
        for (const Slot &e : old)
            if (e.id >= 0) {
                size_t i = hash(e.dx, e.dy, e.dz, e.dl) & mask;
                while (table[i].id >= 0) i = (i + 1) & mask;
                table[i] = e;
            }
    };
    auto class_of = [&](int64_t A, int64_t B) {
        const int la = t.level[A], lb = t.level[B];
        const int lmax = std::max(la, lb);
        int64_t d[3];
        for (int k = 0; k < 3; ++k) {
            const int64_t cb = (2 * (int64_t)t.ix[3 * B + k] + 1) << (lmax - lb);
            const int64_t ca = (2 * (int64_t)t.ix[3 * A + k] + 1) << (lmax - la);
            d[k] = cb - ca;
        }
        const int dl = lb - la;
        size_t i = hash(d[0], d[1], d[2], dl) & mask;
        while (table[i].id >= 0) {
            const Slot &e = table[i];
            if (e.dx == d[0] && e.dy == d[1] && e.dz == d[2] && e.dl == dl) return e.id;
            i = (i + 1) & mask;
        }
        const int32_t id = (int32_t)used++;
        table[i] = Slot{d[0], d[1], d[2], dl, id};
        const double unit = std::ldexp(1.0, lb - lmax);   // smaller radius / r_B
        out.cls_geom.push_back((double)d[0] * unit);
        out.cls_geom.push_back((double)d[1] * unit);
        out.cls_geom.push_back((double)d[2] * unit);
        out.cls_geom.push_back(std::ldexp(1.0, lb - la));  // r_A / r_B
        if (2 * used > table.size()) grow();
        return id;
    };

    out.tile_uoff.assign(out.ntiles + 1, 0);
    // per tile: its distinct classes in ascending id order, then one entry
    // (a row of 64 sources, the zero row where a lane lacks the class) each
    struct Item {
        int32_t cls, lane, src;
    };
    std::vector<Item> items;
    std::vector<int32_t> tile_cls, seen, slot;
    for (int ti = 0; ti < out.ntiles; ++ti) {
        items.clear();
        tile_cls.clear();
        for (int l = 0; l < kTileW; ++l) {
            const int32_t B = out.tile_cell[(size_t)ti * kTileW + l];
            if (B < 0) continue;
            for (int64_t e = t.m2l_ptr[B]; e < t.m2l_ptr[B + 1]; ++e) {
                const int64_t A = t.m2l_src[e];
                const int32_t c = class_of(A, B);
                if ((size_t)c >= seen.size()) {
                    seen.resize(used, -1);
                    slot.resize(used, 0);
                }
                if (seen[c] != ti) {
                    seen[c] = ti;
                    tile_cls.push_back(c);
                }
                items.push_back(Item{c, l, (int32_t)A});
                out.pairs++;
            }
        }
        std::sort(tile_cls.begin(), tile_cls.end());
        const size_t base = out.ucls.size();
        for (size_t k = 0; k < tile_cls.size(); ++k) slot[tile_cls[k]] = (int32_t)k;
        out.ucls.insert(out.ucls.end(), tile_cls.begin(), tile_cls.end());
        out.usrc.resize((base + tile_cls.size()) * kTileW, (int32_t)nc);   // zero row by default
        for (const Item &it : items) out.usrc[(base + slot[it.cls]) * kTileW + it.lane] = it.src;
        out.tile_uoff[ti + 1] = (int32_t)out.ucls.size();
    }
    out.nclasses = (int)used;
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
