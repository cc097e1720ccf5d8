// Optional processing order of a run's histories by start position.
//
// A wave unit normally takes 64 consecutive histories of a spot, which share
// one database track (Section 2.3: a stored history re-traced for many
// incident protons; Section 4: one history per thread group).  For a broad
// field (say the 4 cm circular field of Section 2.5 on 1 mm voxels) those 64
// histories start centimetres apart, so the lanes of a wave deposit into
// unrelated voxels and the workgroup's LDS tally cache finds little to merge.
// In this order the lanes of a wave (and the waves of a workgroup) start next
// to each other; each lane then reads its own track.  Every random number
// stays keyed by the history's identity and the tallies are integer sums, so
// the order cannot change a result bit.
//
// Every history's lateral start offset is drawn exactly as the walk draws it
// and binned on a square grid over the spot (+-4 sigma for a Gaussian spot,
// the diameter for a disk field) in Morton order; each history's offset is
// written at its place in the per-unit lane table order[unit * 64 + lane]
// (0xFFFFFFFF for the lanes past the item's end, filled beforehand).
//  - An item of at most 65536 histories is ordered chunk by chunk (16384
//    histories, 256 units each): one workgroup per chunk counts the bins in
//    LDS, scans them and places the histories (about four per cell, at most
//    64 x 64 cells).
//  - A larger item is ordered as a whole, so that neighbouring units start
//    next to each other across the entire spot: a histogram of about 16
//    histories per cell (at most 256 x 256 cells) in device memory, counted
//    by one workgroup per chunk of histories with device atomics, scanned by
//    one workgroup per item, and the histories placed by a second pass over
//    the chunks.  The histogram of item i starts at first_i / 16 + i (first_i:
//    the item's first history among the run's), so a run needs at most
//    n / 16 + items + 1 counters.
// With secondary trajectories in the database, the histories whose track has
// any come after those whose track has none, each group in Morton order at
// half the spatial resolution (the top bit of the key): a wave replays its
// primaries and then its secondaries, so a wave of which only some lanes
// have secondaries would idle the others meanwhile.
// A fixed number of launches, so the sequence can be captured in a graph.
// Within a cell the order follows the atomics and may differ between runs;
// tallies cannot.
#include "fdc_device.h"

namespace fdc {

namespace {

constexpr uint32_t kChunk = kOrderChunk;    // histories per ordering workgroup (256 units)
constexpr uint32_t kThreads = 1024;
constexpr uint32_t kPer = kChunk / kThreads; // histories per thread
constexpr uint32_t kMaxHalfBits = 6;        // up to 64 x 64 cells

__device__ inline uint32_t spread(uint32_t x)     // bits 0..7 -> even bits
{
    x &= 0xFFu;
    x = (x | (x << 4)) & 0x0F0Fu;
    x = (x | (x << 2)) & 0x3333u;
    x = (x | (x << 1)) & 0x5555u;
    return x;
}

// cells per axis 2^hb over the spot; the offset is drawn exactly as the walk draws it
__device__ inline uint32_t start_cell(const DevSpot &sp, unsigned long long h, uint32_t hb, uint32_t seed_lo,
                                      uint32_t seed_hi)
{
    const uint4 xs = philox4x32_10(make_uint4((uint32_t)h, (uint32_t)(h >> 32), sp.spot,
                                              (sp.plan << 4) | kTagSource), seed_lo, seed_hi);
    const double r = sp.sigma >= 0.f ? sqrt(-2.0 * log(u01(xs.x))) : sqrt(u01(xs.x));
    double sa, ca;
    sincos(2.0 * M_PI * u01(xs.y), &sa, &ca);
    const double n = (double)(1u << hb);
    const double per = sp.sigma >= 0.f ? n / 8.0 : n / 2.0;    // cells per unit of the offset
    const double hi = n - 1.0;
    const double qx = fmin(fmax(floor(r * ca * per) + 0.5 * n, 0.0), hi);
    const double qy = fmin(fmax(floor(r * sa * per) + 0.5 * n, 0.0), hi);
    return spread((uint32_t)qx) | (spread((uint32_t)qy) << 1);
}

// 1 when the history's track has secondary trajectories (the track drawn as the walk draws it)
__device__ inline uint32_t has_secondaries(const DevSpot &sp, unsigned long long h, const OrderTracks &ot,
                                           uint32_t seed_lo, uint32_t seed_hi)
{
    const unsigned long long c = h / ot.R;
    const uint4 xt = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)(c >> 32), sp.spot, (sp.plan << 4) | kTagTrack),
                                   seed_lo, seed_hi);
    const uint32_t first = ot.bin_first[sp.bin];
    const uint32_t nb = ot.bin_first[sp.bin + 1] - first;
    const uint32_t t = first + (uint32_t)(((uint64_t)xt.x * nb) >> 32);
    return ot.sec_first[t + 1] > ot.sec_first[t] ? 1u : 0u;
}

// the sort key of a history among 4^hb bins (at least 2 with secondaries)
__device__ inline uint32_t order_key(const DevSpot &sp, unsigned long long h, uint32_t hb, const OrderTracks &ot,
                                     uint32_t seed_lo, uint32_t seed_hi)
{
    const uint32_t cell = start_cell(sp, h, hb, seed_lo, seed_hi);
    if (!ot.sec_first) return cell;
    const uint32_t sec = has_secondaries(sp, h, ot, seed_lo, seed_hi);
    return hb ? ((cell >> 1) | (sec << (2 * hb - 1))) : sec;
}

// the item holding chunk c: largest i with items[i].chunk0 <= c
__device__ inline uint32_t item_of_chunk(const WorkItem *items, uint32_t n_items, uint32_t c)
{
    uint32_t lo = 0, hi = n_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].chunk0 <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// half the bits of a large item's cell count: 4^hb <= n / 16, at most 256 x 256 cells
__device__ inline uint32_t large_half_bits(unsigned long long n)
{
    uint32_t hb = 0;
    while (hb < 8 && (16ull << (2 * (hb + 1))) <= n) ++hb;
    return hb;
}

// count (PLACE false) or place (PLACE true) the histories of one chunk of a large item
template <bool PLACE>
__global__ void __launch_bounds__(kThreads) order_large_kernel(const WorkItem *__restrict__ items, uint32_t n_items,
                                                               const DevSpot *__restrict__ spots,
                                                               const unsigned long long *__restrict__ hnext,
                                                               uint32_t seed_lo, uint32_t seed_hi,
                                                               uint32_t *__restrict__ hist, uint32_t *__restrict__ order,
                                                               OrderTracks ot)
{
    const uint32_t i = item_of_chunk(items, n_items, blockIdx.x);
    const WorkItem it = items[i];
    if (it.n <= kOrderWholeSpot) return;                             // (uniform: the whole block)
    const unsigned long long j0 = (unsigned long long)(blockIdx.x - it.chunk0) * kChunk;
    if (j0 >= it.n) return;
    const uint32_t len = (uint32_t)min((unsigned long long)kChunk, it.n - j0);
    const DevSpot &sp = spots[it.gspot];
    const uint32_t hb = large_half_bits(it.n);
    uint32_t *h = hist + (it.first >> 4) + i;
    const unsigned long long hbase = it.h0 + (hnext ? hnext[it.gspot] : 0ull) + j0;
    for (uint32_t e = threadIdx.x; e < len; e += kThreads) {
        const uint32_t cell = order_key(sp, hbase + e, hb, ot, seed_lo, seed_hi);
        if (PLACE) {
            const unsigned long long p = atomicAdd(h + cell, 1u);
            order[(it.unit0 + p / kWave) * kWave + (p % kWave)] = (uint32_t)(j0 + e);
        } else {
            atomicAdd(h + cell, 1u);
        }
    }
}

// exclusive scan of each large item's histogram, one workgroup per item
__global__ void __launch_bounds__(kThreads) order_scan_kernel(const WorkItem *__restrict__ items,
                                                              uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_wave[kThreads / kWave];
    const WorkItem it = items[blockIdx.x];
    if (it.n <= kOrderWholeSpot) return;
    const uint32_t ncell = 1u << (2 * large_half_bits(it.n));
    uint32_t *h = hist + (it.first >> 4) + blockIdx.x;
    const uint32_t per = (ncell + kThreads - 1) / kThreads;         // 1 .. 64 consecutive cells per thread
    const uint32_t t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    const uint32_t c0 = t * per;
    uint32_t mine = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (c0 + k < ncell) mine += h[c0 + k];
    uint32_t incl = mine;
#pragma unroll
    for (uint32_t off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += v;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint32_t run = incl - mine;
    for (uint32_t w = 0; w < wave; ++w) run += s_wave[w];
    for (uint32_t k = 0; k < per; ++k) {
        if (c0 + k < ncell) {
            const uint32_t c = h[c0 + k];
            h[c0 + k] = run;
            run += c;
        }
    }
}

__global__ void __launch_bounds__(kThreads) order_chunk_kernel(const WorkItem *__restrict__ items, uint32_t n_items,
                                                               const DevSpot *__restrict__ spots,
                                                               const unsigned long long *__restrict__ hnext,
                                                               uint32_t seed_lo, uint32_t seed_hi,
                                                               uint32_t *__restrict__ order, OrderTracks ot)
{
    __shared__ uint32_t s_cnt[1u << (2 * kMaxHalfBits)];
    __shared__ uint32_t s_wave[kThreads / kWave];
    const uint32_t t = threadIdx.x;
    const WorkItem it = items[item_of_chunk(items, n_items, blockIdx.x)];
    const DevSpot &sp = spots[it.gspot];
    if (it.n > kOrderWholeSpot) return;                              // ordered as a whole (uniform: the whole block)
    const unsigned long long j0 = (unsigned long long)(blockIdx.x - it.chunk0) * kChunk;
    if (j0 >= it.n) return;
    const uint32_t len = (uint32_t)min((unsigned long long)kChunk, it.n - j0);
    // about four histories per cell: 4^hb <= len / 4
    uint32_t hb = 0;
    while (hb < kMaxHalfBits && (4u << (2 * (hb + 1))) <= len) ++hb;
    const uint32_t nbins = ot.sec_first && hb == 0 ? 2u : 1u << (2 * hb);
    const unsigned long long hbase = it.h0 + (hnext ? hnext[it.gspot] : 0ull) + j0;

    for (uint32_t b = t; b < nbins; b += kThreads) s_cnt[b] = 0;
    __syncthreads();
    uint32_t cell[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t e = t + r * kThreads;
        cell[r] = 0;
        if (e < len) {
            cell[r] = order_key(sp, hbase + e, hb, ot, seed_lo, seed_hi);
            atomicAdd(&s_cnt[cell[r]], 1u);
        }
    }
    __syncthreads();
    // exclusive scan of the bin counts: each thread sums up to four
    // consecutive bins, the threads' sums are scanned per wave with shuffles
    // and across waves through LDS
    const uint32_t per_t = (nbins + kThreads - 1) / kThreads;      // 1 or 4
    const uint32_t b0 = t * per_t;
    uint32_t mine = 0;
    for (uint32_t k = 0; k < per_t; ++k)
        if (b0 + k < nbins) mine += s_cnt[b0 + k];
    const uint32_t lane = t & (kWave - 1), wave = t / kWave;
    uint32_t incl = mine;
#pragma unroll
    for (uint32_t off = 1; off < kWave; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += v;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (uint32_t w = 0; w < wave; ++w) wbase += s_wave[w];
    uint32_t run = wbase + incl - mine;                            // exclusive prefix of this thread's bins
    __syncthreads();                                               // every count read before the rewrite
    for (uint32_t k = 0; k < per_t; ++k) {
        if (b0 + k < nbins) {
            const uint32_t c = s_cnt[b0 + k];
            s_cnt[b0 + k] = run;
            run += c;
        }
    }
    __syncthreads();
    // each history at its place: unit = item's first unit + place / 64
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t e = t + r * kThreads;
        if (e < len) {
            const unsigned long long p = j0 + atomicAdd(&s_cnt[cell[r]], 1u);
            order[(it.unit0 + p / kWave) * kWave + (p % kWave)] = (uint32_t)(j0 + e);
        }
    }
}

} // namespace

hipError_t launch_source_order(const WorkItem *items, uint32_t n_items, uint32_t n_chunks, unsigned long long n_units,
                               const DevSpot *spots, const unsigned long long *hnext, uint32_t seed_lo,
                               uint32_t seed_hi, uint32_t *order, uint32_t *hist, unsigned long long hist_words,
                               bool large, const OrderTracks &tracks, hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    // lanes past an item's end: none (the table is 64 x n_units words, an even count)
    hipError_t e = launch_fill_u64((unsigned long long *)order, n_units * kWave / 2, ~0ull, s);
    if (e != hipSuccess || n_chunks == 0) return e;
    if (large) {                                         // items of more than one chunk: whole-item histograms
        e = launch_fill_u64((unsigned long long *)hist, (hist_words + 1) / 2, 0ull, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(order_large_kernel<false>, dim3(n_chunks), dim3(kThreads), 0, s, items, n_items, spots,
                           hnext, seed_lo, seed_hi, hist, order, tracks);
        hipLaunchKernelGGL(order_scan_kernel, dim3(n_items), dim3(kThreads), 0, s, items, hist);
        hipLaunchKernelGGL(order_large_kernel<true>, dim3(n_chunks), dim3(kThreads), 0, s, items, n_items, spots,
                           hnext, seed_lo, seed_hi, hist, order, tracks);
    }
    hipLaunchKernelGGL(order_chunk_kernel, dim3(n_chunks), dim3(kThreads), 0, s, items, n_items, spots, hnext,
                       seed_lo, seed_hi, order, tracks);
    return hipGetLastError();
}

} // namespace fdc
