// Optional processing order of a run's histories by start position.
//
// A wave unit normally takes 64 consecutive histories of a spot, which share
// one database track (Section 2.3: a stored history re-traced for many
// incident protons; Section 4: one history per thread group).  For a broad
// field (say the 4 cm circular field of Section 2.5 on 1 mm voxels) those 64
// histories start centimetres apart, so the lanes of a wave deposit into
// unrelated voxels and the workgroup's LDS tally cache finds little to merge.
// With this order the histories of each work item are sorted by a Morton code
// of their lateral start offset on a fine grid, so the lanes of a wave (and
// the waves of a workgroup) start next to each other; each lane then reads its
// own track.  Every random number stays keyed by the history's identity and
// the tallies are integer sums, so the order cannot change a result bit.
//
// Three steps per run: keys (one thread per history), a device radix sort of
// (item << 16 | morton, offset) pairs (32-bit keys while the run has fewer
// than 2^16 work items, else 64-bit), and a scatter into the per-unit table
// order[unit * 64 + lane] = offset of the lane's history in its item
// (0xFFFFFFFF for the lanes past the item's end).  The Morton code covers the
// spot's lateral offset in units of its width: 256 cells over +-4 sigma for a
// Gaussian spot, over the diameter for a disk field.
#include <hipcub/hipcub.hpp>

#include "fdc_device.h"

namespace fdc {

namespace {

__device__ inline uint32_t spread16(uint32_t x)     // bits 0..15 -> even bits
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__device__ inline uint32_t item_of(const WorkItem *items, uint32_t n_items, unsigned long long g)
{
    uint32_t lo = 0, hi = n_items;              // largest i with items[i].first <= g
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].first <= g) lo = mid; else hi = mid;
    }
    return lo;
}

template <class Key>
__global__ void order_keys_kernel(const WorkItem *items, uint32_t n_items,
                                  unsigned long long n_total, const DevSpot *spots, const unsigned long long *hnext,
                                  uint32_t seed_lo, uint32_t seed_hi, Key *keys, uint32_t *vals)
{
    const unsigned long long g = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    const uint32_t i = item_of(items, n_items, g);
    const WorkItem it = items[i];
    const DevSpot sp = spots[it.gspot];
    const unsigned long long j = g - it.first;
    const unsigned long long h = it.h0 + (hnext ? hnext[it.gspot] : 0ull) + j;
    // the lateral start offset drawn exactly as the transport draws it
    const uint4 xs = philox4x32_10(make_uint4((uint32_t)h, (uint32_t)(h >> 32), sp.spot,
                                              (sp.plan << 4) | kTagSource), seed_lo, seed_hi);
    const double r = sp.sigma >= 0.f ? sqrt(-2.0 * log(u01(xs.x))) : sqrt(u01(xs.x));
    double sa, ca;
    sincos(2.0 * M_PI * u01(xs.y), &sa, &ca);
    const double cells = sp.sigma >= 0.f ? 32.0 : 128.0;          // per unit of the offset
    const double qx = fmin(fmax(floor(r * ca * cells) + 128.0, 0.0), 255.0);
    const double qy = fmin(fmax(floor(r * sa * cells) + 128.0, 0.0), 255.0);
    const uint32_t morton = spread16((uint32_t)qx) | (spread16((uint32_t)qy) << 1);
    keys[g] = ((Key)i << 16) | (Key)morton;
    vals[g] = (uint32_t)j;
}

__global__ void order_scatter_kernel(const WorkItem *items, uint32_t n_items,
                                     unsigned long long n_slots, const uint32_t *sorted, uint32_t *order)
{
    const unsigned long long q = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (q >= n_slots) return;
    const unsigned long long unit = q / kWave;
    uint32_t lo = 0, hi = n_items;              // the item owning this unit
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].unit0 <= unit) lo = mid; else hi = mid;
    }
    const WorkItem it = items[lo];
    const unsigned long long j = (unit - it.unit0) * kWave + (q % kWave);
    order[q] = j < it.n ? sorted[it.first + j] : 0xFFFFFFFFu;
}

} // namespace

static bool narrow_keys(uint32_t n_items) { return n_items < (1u << 16); }

static int key_bits(uint32_t n_items) { return 16 + (32 - __builtin_clz(n_items | 1u)); }

size_t source_order_temp_bytes(unsigned long long n_total, uint32_t n_items)
{
    size_t bytes = 0;
    if (narrow_keys(n_items))
        hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                           (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)n_total, 0,
                                           key_bits(n_items));
    else
        hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const unsigned long long *)nullptr,
                                           (unsigned long long *)nullptr, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (int)n_total, 0, key_bits(n_items));
    return bytes;
}

template <class Key>
static hipError_t keys_and_sort(const WorkItem *items, uint32_t n_items, unsigned long long n_total,
                                const DevSpot *spots, const unsigned long long *hnext, uint32_t seed_lo,
                                uint32_t seed_hi, Key *keys_a, Key *keys_b, uint32_t *vals_a, uint32_t *vals_b,
                                void *temp, size_t temp_bytes, hipStream_t s)
{
    const unsigned int tb = 256;
    hipLaunchKernelGGL(order_keys_kernel<Key>, dim3((unsigned)((n_total + tb - 1) / tb)), dim3(tb), 0, s, items,
                       n_items, n_total, spots, hnext, seed_lo, seed_hi, keys_a, vals_a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_a, keys_b, vals_a, vals_b, (int)n_total, 0,
                                              key_bits(n_items), s);
}

// keys_a and keys_b hold n_total 64-bit keys each (the 32-bit form uses their first halves)
hipError_t launch_source_order(const WorkItem *items, uint32_t n_items,
                               unsigned long long n_total, unsigned long long n_units, const DevSpot *spots,
                               const unsigned long long *hnext, uint32_t seed_lo, uint32_t seed_hi,
                               unsigned long long *keys_a, unsigned long long *keys_b, uint32_t *vals_a,
                               uint32_t *vals_b, void *temp, size_t temp_bytes, uint32_t *order, hipStream_t s)
{
    if (n_total == 0) return hipSuccess;
    const hipError_t e =
        narrow_keys(n_items)
            ? keys_and_sort<uint32_t>(items, n_items, n_total, spots, hnext, seed_lo, seed_hi, (uint32_t *)keys_a,
                                      (uint32_t *)keys_b, vals_a, vals_b, temp, temp_bytes, s)
            : keys_and_sort<unsigned long long>(items, n_items, n_total, spots, hnext, seed_lo, seed_hi, keys_a,
                                                keys_b, vals_a, vals_b, temp, temp_bytes, s);
    if (e != hipSuccess) return e;
    const unsigned int tb = 256;
    const unsigned long long n_slots = n_units * kWave;
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)((n_slots + tb - 1) / tb)), dim3(tb), 0, s, items, n_items,
                       n_slots, vals_b, order);
    return hipGetLastError();
}

} // namespace fdc
