// CPU model of the transport kernel's LDS write-back tally cache, with
// std::atomic words and host threads standing in for the lanes of a
// workgroup.  The update protocol is restated here (not included from the
// library) so that the test exercises the protocol as documented:
//
//   word = (voxel + 1) << vbits | partial sum, 0 = empty;
//   a deposit of at least 2^(vbits-12) goes straight to the global tally;
//   hit  (the word read holds the voxel): atomic add of the deposit;
//   miss: atomic exchange installs (voxel, deposit); the evicted sum goes to
//         the global tally, unless it is the same voxel's (installed by another
//         lane an instant earlier), which is added back into the word;
//   after an add whose returned word holds another key, the deposit is added
//   to the lane's own voxel and subtracted from that key's voxel (a modular
//   repair, settled when that word is flushed);
//   an add that takes a sum to half its field exchanges the word with 0 and
//   flushes it; flushes skip words whose key is 0.
// At the end every slot is flushed.  The global tally must equal the exact
// per-voxel sums (mod 2^64) for every thread count, slot count, voxel set and
// field width.  Usage: cache_model threads slots voxels vbits adds_per_thread seed
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

namespace {

struct Model {
    std::vector<std::atomic<uint64_t>> cache;
    std::vector<std::atomic<uint64_t>> tally;
    uint32_t n, vbits, nvox;

    Model(uint32_t slots, uint32_t voxels, uint32_t bits) : cache(slots), tally(voxels), n(slots), vbits(bits), nvox(voxels)
    {
        for (auto &w : cache) w.store(0);
        for (auto &t : tally) t.store(0);
    }

    uint64_t vmask() const { return (uint64_t(1) << vbits) - 1; }

    // slot: a hash of the voxel's row plus its x index (rows of nx = 16 voxels)
    uint32_t slot(uint32_t v) const
    {
        const uint32_t ix = v % 16u;
        uint32_t row = v - ix;
        row ^= row >> 15;
        row *= 0x2c1b3c6du;
        row ^= row >> 12;
        const uint32_t s = (uint32_t)(((uint64_t)row * n) >> 32) + ix;
        return s < n ? s : s % n;
    }

    void to_global(uint32_t v, uint64_t val) { tally[v].fetch_add(val, std::memory_order_relaxed); }

    void flush_word(uint64_t w)
    {
        const uint32_t kv = (uint32_t)(w >> vbits);
        const uint64_t val = w & vmask();
        if (kv != 0 && kv <= nvox && val != 0) to_global(kv - 1, val);
    }

    void settle(std::atomic<uint64_t> &c, uint32_t v, uint64_t key, uint64_t val, bool hit, uint64_t o)
    {
        if (!hit) {
            flush_word(o);
            return;
        }
        if ((o & ~vmask()) != key) {
            to_global(v, val);
            const uint32_t kv = (uint32_t)(o >> vbits);
            if (kv != 0 && kv <= nvox) to_global(kv - 1, 0 - val);
        }
        if ((o & vmask()) + val >= (uint64_t(1) << (vbits - 1))) flush_word(c.exchange(0));
    }

    void add(uint32_t v, uint64_t dep)
    {
        if (dep == 0) return;
        const uint64_t lim = uint64_t(1) << (vbits - 12);
        if (dep >= lim) {
            to_global(v, dep);
            return;
        }
        std::atomic<uint64_t> &c = cache[slot(v)];
        const uint64_t key = (uint64_t)(v + 1) << vbits;
        const uint64_t w = c.load();
        const bool hit = (w & ~vmask()) == key;
        uint64_t o = hit ? c.fetch_add(dep) : c.exchange(key | dep);
        uint64_t a = dep;
        bool h = hit;
        if (!hit && (o & ~vmask()) == key && (o & vmask()) < lim) {
            a = o & vmask();
            h = true;
            o = c.fetch_add(a);
        }
        settle(c, v, key, a, h, o);
    }
};

} // namespace

int main(int argc, char **argv)
{
    if (argc != 7) {
        std::fprintf(stderr, "usage: cache_model threads slots voxels vbits adds_per_thread seed\n");
        return 2;
    }
    const int threads = std::atoi(argv[1]);
    const uint32_t slots = (uint32_t)std::atoi(argv[2]);
    const uint32_t voxels = (uint32_t)std::atoi(argv[3]);
    const uint32_t vbits = (uint32_t)std::atoi(argv[4]);
    const long adds = std::atol(argv[5]);
    const uint64_t seed = (uint64_t)std::atoll(argv[6]);
    Model m(slots, voxels, vbits);
    std::vector<std::vector<uint64_t>> expect(threads, std::vector<uint64_t>(voxels, 0));
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            std::mt19937_64 rng(seed * 1000003u + (uint64_t)t);
            const uint64_t lim = uint64_t(1) << (vbits - 12);
            for (long i = 0; i < adds; ++i) {
                // neighbouring voxels in bursts (as a wave walking together), sometimes far ones
                const uint32_t v = (uint32_t)(rng() % voxels);
                const uint64_t r = rng() % 100;
                const uint64_t dep = r < 2 ? lim + rng() % (4 * lim)       // too large for the cache
                                   : r < 4 ? 0                              // zero deposits are skipped
                                   : 1 + rng() % (lim - 1);
                expect[t][v] += dep;
                m.add(v, dep);
            }
        });
    for (auto &th : pool) th.join();
    for (uint32_t s = 0; s < slots; ++s) m.flush_word(m.cache[s].load());
    long bad = 0;
    for (uint32_t v = 0; v < voxels; ++v) {
        uint64_t e = 0;
        for (int t = 0; t < threads; ++t) e += expect[t][v];
        if (m.tally[v].load() != e) ++bad;
    }
    std::printf("%s threads=%d slots=%u voxels=%u vbits=%u adds=%ld mismatches=%ld\n", bad ? "FAIL" : "ok", threads,
                slots, voxels, vbits, adds, bad);
    return bad ? 1 : 0;
}
