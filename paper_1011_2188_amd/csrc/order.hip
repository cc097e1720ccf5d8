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
// Each work item's histories are cut in chunks of 16384 (a multiple of the
// 64-history unit, so a chunk fills whole units); one workgroup orders one
// chunk: it draws every history's lateral start offset exactly as the walk
// draws it, bins it on a square grid over the spot (+-4 sigma for a Gaussian
// spot, the diameter for a disk field) in Morton order, counts the bins in
// LDS, scans them and writes each history's offset at its place in the
// per-unit lane table order[unit * 64 + lane] (0xFFFFFFFF for the lanes past
// the item's end, filled beforehand).  The grid has about four histories per
// cell (at most 64 x 64 cells).  Chunks are ordered independently: no global
// histogram or scan, no scratch memory, and a fixed number of launches, so
// the sequence can be captured in a graph.  Within a cell the order follows
// the LDS atomics and may differ between runs; tallies cannot.
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

__global__ void __launch_bounds__(kThreads) order_chunk_kernel(const WorkItem *__restrict__ items, uint32_t n_items,
                                                               const DevSpot *__restrict__ spots,
                                                               const unsigned long long *__restrict__ hnext,
                                                               uint32_t seed_lo, uint32_t seed_hi,
                                                               uint32_t *__restrict__ order)
{
    __shared__ uint32_t s_cnt[1u << (2 * kMaxHalfBits)];
    __shared__ uint32_t s_wave[kThreads / kWave];
    const uint32_t t = threadIdx.x;
    // the item holding this chunk: largest i with items[i].chunk0 <= blockIdx.x
    uint32_t lo = 0, hi = n_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].chunk0 <= blockIdx.x) lo = mid; else hi = mid;
    }
    const WorkItem it = items[lo];
    const DevSpot &sp = spots[it.gspot];
    const unsigned long long j0 = (unsigned long long)(blockIdx.x - it.chunk0) * kChunk;
    if (j0 >= it.n) return;                                          // (uniform: the whole block)
    const uint32_t len = (uint32_t)min((unsigned long long)kChunk, it.n - j0);
    // about four histories per cell: 4^hb <= len / 4
    uint32_t hb = 0;
    while (hb < kMaxHalfBits && (4u << (2 * (hb + 1))) <= len) ++hb;
    const uint32_t nbins = 1u << (2 * hb);
    const unsigned long long hbase = it.h0 + (hnext ? hnext[it.gspot] : 0ull) + j0;

    for (uint32_t b = t; b < nbins; b += kThreads) s_cnt[b] = 0;
    __syncthreads();
    uint32_t cell[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t e = t + r * kThreads;
        cell[r] = 0;
        if (e < len) {
            cell[r] = start_cell(sp, hbase + e, hb, seed_lo, seed_hi);
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
                               uint32_t seed_hi, uint32_t *order, hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    // lanes past an item's end: none (the table is 64 x n_units words, an even count)
    hipError_t e = launch_fill_u64((unsigned long long *)order, n_units * kWave / 2, ~0ull, s);
    if (e != hipSuccess || n_chunks == 0) return e;
    hipLaunchKernelGGL(order_chunk_kernel, dim3(n_chunks), dim3(kThreads), 0, s, items, n_items, spots, hnext,
                       seed_lo, seed_hi, order);
    return hipGetLastError();
}

} // namespace fdc
