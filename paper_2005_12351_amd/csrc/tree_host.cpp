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
#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>

#include "fmm_internal.h"

// ---------------------------------------------------------------------------
// Host threads for the scheduling passes: a fixed set of workers, started on
// first use and kept for the life of the process, takes blocks of work items
// [0, n) from a shared counter; the calling thread takes blocks too, so a
// loop completes even while every worker serves another build's loop (the
// serving slots build trees at once).  Every result slot is written by
// exactly one item, so the outcome does not depend on which thread ran it.
class HostPool {
public:
    static HostPool &get()
    {
        static HostPool p;
        return p;
    }
    template <typename F>
    void run(int64_t n, F &&f)
    {
        const int64_t grain = std::max<int64_t>(1, n / (4 * (int64_t)(workers_.size() + 1)));
        if (workers_.empty() || n <= grain) {
            for (int64_t i = 0; i < n; ++i) f(i);
            return;
        }
        Task task;
        task.n = n;
        task.grain = grain;
        task.body = [&f](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i) f(i);
        };
        {
            std::lock_guard<std::mutex> lk(mu_);
            tasks_.push_back(&task);
        }
        cv_.notify_all();
        work_on(task);
        {
            // no worker joins once the task has left the queue; wait for
            // those that joined before
            std::lock_guard<std::mutex> lk(mu_);
            auto it = std::find(tasks_.begin(), tasks_.end(), &task);
            if (it != tasks_.end()) tasks_.erase(it);
        }
        std::unique_lock<std::mutex> tl(task.m);
        task.cv.wait(tl, [&] { return task.active == 0; });
    }

private:
    struct Task {
        int64_t n = 0, grain = 1;
        std::function<void(int64_t, int64_t)> body;
        std::atomic<int64_t> next{0};
        int active = 0;   // workers inside; guarded by m
        std::mutex m;
        std::condition_variable cv;
    };
    HostPool()
    {
        const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (int k = 0; k + 1 < hw; ++k) workers_.emplace_back([this] { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &w : workers_) w.join();
    }
    static void work_on(Task &t)
    {
        for (;;) {
            const int64_t a = t.next.fetch_add(t.grain);
            if (a >= t.n) return;
            t.body(a, std::min(t.n, a + t.grain));
        }
    }
    void loop()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !tasks_.empty(); });
            if (stop_) return;
            Task *t = tasks_.front();
            if (t->next.load() >= t->n) {
                tasks_.pop_front();   // nothing left to take; its owner finishes it
                continue;
            }
            {
                std::lock_guard<std::mutex> tl(t->m);
                ++t->active;
            }
            lk.unlock();
            work_on(*t);
            {
                std::lock_guard<std::mutex> tl(t->m);
                if (--t->active == 0) t->cv.notify_all();
            }
            lk.lock();
        }
    }
    std::vector<std::thread> workers_;
    std::deque<Task *> tasks_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool stop_ = false;
};

template <typename F>
static void parallel_for(int64_t n, F f)
{
    HostPool::get().run(n, f);
}

void host_parallel_for(int64_t n, const std::function<void(int64_t)> &f, int64_t serial_below)
{
    if (n < serial_below) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    parallel_for(n, [&](int64_t i) { f(i); });
}

// Exact integer geometry of a pair (source A, target B): the centre offset
// in units of the smaller radius and the level difference.  It determines
// ((z_B - z_A) / r_B, r_A / r_B) exactly.
struct ClassKey {
    int64_t d[3];
    int32_t dl;
    bool operator<(const ClassKey &o) const
    {
        if (dl != o.dl) return dl < o.dl;
        for (int k = 0; k < 3; ++k)
            if (d[k] != o.d[k]) return d[k] < o.d[k];
        return false;
    }
    bool operator==(const ClassKey &o) const
    {
        return dl == o.dl && d[0] == o.d[0] && d[1] == o.d[1] && d[2] == o.d[2];
    }
    uint64_t hash() const
    {
        uint64_t h = (uint64_t)d[0] * 0x9E3779B97F4A7C15ULL ^ (uint64_t)d[1] * 0xC2B2AE3D27D4EB4FULL ^
                     (uint64_t)d[2] * 0x165667B19E3779F9ULL ^ (uint64_t)(dl + 64) * 0x27D4EB2F165667C5ULL;
        return h ^ (h >> 29);
    }
};

static ClassKey class_key(const HostTree &t, int64_t A, int64_t B)
{
    const int la = t.level[A], lb = t.level[B];
    const int lmax = std::max(la, lb);
    ClassKey k;
    for (int d = 0; d < 3; ++d) {
        const int64_t cb = (2 * (int64_t)t.ix[3 * B + d] + 1) << (lmax - lb);
        const int64_t ca = (2 * (int64_t)t.ix[3 * A + d] + 1) << (lmax - la);
        k.d[d] = cb - ca;
    }
    k.dl = lb - la;
    return k;
}

// Map ClassKey -> int (one per thread and tile).  Pairs of one level with
// offsets of at most kNear cells per axis (nearly all M2L pairs) index a
// dense table; the rest go through open addressing.
constexpr int kNear = 8;
constexpr int kNearW = 2 * kNear + 1;
static int near_index(const ClassKey &k)
{
    if (k.dl != 0) return -1;
    int idx = 0;
    for (int d = 0; d < 3; ++d) {
        const int64_t o = k.d[d] / 2;   // same level: offsets are 2 * (cell offset)
        if (o < -kNear || o > kNear) return -1;
        idx = idx * kNearW + (int)(o + kNear);
    }
    return idx;
}

struct KeyMap {
    std::vector<int32_t> nearv;
    std::vector<ClassKey> key;
    std::vector<int32_t> val;
    size_t mask = 0, used = 0;
    void reset(size_t want)
    {
        nearv.assign((size_t)kNearW * kNearW * kNearW, -1);
        size_t cap = 64;
        while (cap < 2 * want) cap *= 2;
        key.assign(cap, ClassKey{});
        val.assign(cap, -1);
        mask = cap - 1;
        used = 0;
    }
    // value of k, inserting it with value v if absent
    int32_t get_or_put(const ClassKey &k, int32_t v)
    {
        const int ni = near_index(k);
        if (ni >= 0) {
            if (nearv[ni] < 0) nearv[ni] = v;
            return nearv[ni];
        }
        if (2 * (used + 1) > key.size()) grow();
        size_t i = k.hash() & mask;
        while (val[i] >= 0) {
            if (key[i] == k) return val[i];
            i = (i + 1) & mask;
        }
        key[i] = k;
        val[i] = v;
        ++used;
        return v;
    }
    int32_t get(const ClassKey &k) const
    {
        const int ni = near_index(k);
        if (ni >= 0) return nearv[ni];
        size_t i = k.hash() & mask;
        while (val[i] >= 0) {
            if (key[i] == k) return val[i];
            i = (i + 1) & mask;
        }
        return -1;
    }
    void grow()
    {
        std::vector<ClassKey> ok(std::move(key));
        std::vector<int32_t> ov(std::move(val));
        key.assign(ok.size() * 2, ClassKey{});
        val.assign(ok.size() * 2, -1);
        mask = key.size() - 1;
        for (size_t j = 0; j < ok.size(); ++j)
            if (ov[j] >= 0) {
                size_t i = ok[j].hash() & mask;
                while (val[i] >= 0) i = (i + 1) & mask;
                key[i] = ok[j];
                val[i] = ov[j];
            }
    }
};

// ---------------------------------------------------------------------------
// M2L tiling.  Target cells with a non-empty M2L list are grouped 64 to a
// tile (one GPU lane per target).  Cells of one level and one position
// inside their parent have identical relative source layouts away from the
// domain boundary, and near it equal truncations (see below), so tiles are
// formed in that order.  A tile iterates over the union of its targets'
// translation classes; a class is the exact dimensionless geometry of a
// pair, ((z_B - z_A) / r_B, r_A / r_B), so one derivative tensor serves
// every lane at a given step.  Class ids follow the sorted order of the
// exact pair geometry, so they and everything built from them are the same
// for any number of host threads.
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
    parallel_for((int64_t)tg.size(), [&](int64_t q) {
        const int32_t c = tg[q];
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
    });
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
    const int ntl = out.ntiles;

    // pass 1 (per tile): the tile's distinct pair geometries, sorted
    std::vector<std::vector<ClassKey>> tkeys(ntl);
    std::vector<int64_t> tpairs(ntl, 0);
    parallel_for(ntl, [&](int64_t ti) {
        KeyMap m;
        m.reset(256);
        std::vector<ClassKey> &u = tkeys[ti];
        for (int l = 0; l < kTileW; ++l) {
            const int32_t B = out.tile_cell[(size_t)ti * kTileW + l];
            if (B < 0) continue;
            for (int64_t e = t.m2l_ptr[B]; e < t.m2l_ptr[B + 1]; ++e) {
                const ClassKey k = class_key(t, t.m2l_src[e], B);
                if (m.get_or_put(k, (int32_t)u.size()) == (int32_t)u.size()) u.push_back(k);
                tpairs[ti]++;
            }
        }
        std::sort(u.begin(), u.end());
    });
    // class ids: ranks in the sorted union of all tiles' geometries
    std::vector<ClassKey> all;
    {
        KeyMap seen;
        seen.reset(1024);
        for (const auto &u : tkeys)
            for (const ClassKey &k : u)
                if (seen.get_or_put(k, (int32_t)all.size()) == (int32_t)all.size()) all.push_back(k);
        std::sort(all.begin(), all.end());
    }
    out.nclasses = (int)all.size();
    out.cls_geom.resize((size_t)4 * all.size());
    for (size_t c = 0; c < all.size(); ++c) {
        const ClassKey &k = all[c];
        const double unit = std::ldexp(1.0, std::min(0, k.dl));   // smaller radius / r_B
        out.cls_geom[4 * c] = (double)k.d[0] * unit;
        out.cls_geom[4 * c + 1] = (double)k.d[1] * unit;
        out.cls_geom[4 * c + 2] = (double)k.d[2] * unit;
        out.cls_geom[4 * c + 3] = std::ldexp(1.0, k.dl);           // r_A / r_B
    }
    out.tile_uoff.assign(ntl + 1, 0);
    for (int ti = 0; ti < ntl; ++ti) {
        out.tile_uoff[ti + 1] = out.tile_uoff[ti] + (int32_t)tkeys[ti].size();
        out.pairs += tpairs[ti];
    }
    out.nentries = out.tile_uoff[ntl];
    out.ucls.assign((size_t)out.nentries, 0);
    out.usrc.resize((size_t)out.nentries * kTileW);
    // pass 2 (per tile): class ids of its entries (ascending) and the source
    // of every lane at each entry
    parallel_for(ntl, [&](int64_t ti) {
        const std::vector<ClassKey> &u = tkeys[ti];
        const size_t base = (size_t)out.tile_uoff[ti];
        std::fill(out.usrc.begin() + base * kTileW, out.usrc.begin() + (base + u.size()) * kTileW,
                  (int32_t)nc);   // the zero row where a lane lacks the class
        KeyMap m;
        m.reset(u.size());
        for (size_t j = 0; j < u.size(); ++j) {
            m.get_or_put(u[j], (int32_t)j);
            out.ucls[base + j] = (int32_t)(std::lower_bound(all.begin(), all.end(), u[j]) - all.begin());
        }
        for (int l = 0; l < kTileW; ++l) {
            const int32_t B = out.tile_cell[(size_t)ti * kTileW + l];
            if (B < 0) continue;
            for (int64_t e = t.m2l_ptr[B]; e < t.m2l_ptr[B + 1]; ++e) {
                const int64_t A = t.m2l_src[e];
                out.usrc[(base + (size_t)m.get(class_key(t, A, B))) * kTileW + l] = (int32_t)A;
            }
        }
    });
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
