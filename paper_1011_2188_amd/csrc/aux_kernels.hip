// Set-up and finishing kernels: material table, HU -> table index, track
// energies, dose and Eq. (2) variance, integer reductions, Philox test.
#include "fdc_device.h"

namespace fdc {

namespace {

// pts: n_pts rows of (hu, rho, rsp, rscp); piecewise linear, clamped at the ends
__device__ double table_value(const double *pts, int n_pts, int col, double h)
{
    if (h <= pts[0]) return pts[col];
    if (h >= pts[4 * (n_pts - 1)]) return pts[4 * (n_pts - 1) + col];
    int j = 0;
    while (!(h < pts[4 * (j + 1)])) ++j;
    const double h0 = pts[4 * j], h1 = pts[4 * (j + 1)];
    const double v0 = pts[4 * j + col], v1 = pts[4 * (j + 1) + col];
    return v0 + (v1 - v0) * (h - h0) / (h1 - h0);
}

__global__ void build_lut_kernel(const double *pts, int n_pts, double vacuum_below, float2 *lut,
                                 float *rho)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kLutSize) return;
    const double h = (double)(i + kHuMin);
    rho[i] = (float)table_value(pts, n_pts, 1, h);
    if (h < vacuum_below) {
        lut[i] = make_float2(0.f, 0.f);
        return;
    }
    const double s = table_value(pts, n_pts, 2, h);
    const double c = table_value(pts, n_pts, 3, h);
    lut[i] = s > 0.0 ? make_float2((float)s, (float)(c / s)) : make_float2(0.f, 0.f);
}

__global__ void hu_to_index_kernel(const int16_t *__restrict__ hu, uint16_t *__restrict__ idx, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int h = min(max((int)hu[i], kHuMin), kHuMin + kLutSize - 1);
        idx[i] = (uint16_t)(h - kHuMin);
    }
}

// vacuum-skip bits: seed (0 for non-vacuum voxels, the cap for vacuum), then
// relaxation passes skip(v) = min(skip(v), 1 + min over the 26 neighbours
// inside the box).  Every value stays an upper bound of the true distance and
// a voxel at distance d is exact after pass d, so after kMaxSkip passes every
// voxel holds min(distance, kMaxSkip) whatever order the updates run in (a
// pass may already see neighbours updated in the same pass).
__global__ void skip_seed_kernel(uint16_t *__restrict__ idx, const float2 *__restrict__ lut, size_t n)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const uint32_t h = hu_index(idx[v]);
        idx[v] = (uint16_t)(h | ((lut[h].x == 0.f ? kMaxSkip : 0u) << kHuBits));
    }
}

__global__ void skip_relax_kernel(uint16_t *idx, int nx, int ny, int nz)
{
    const size_t n = (size_t)nx * ny * nz;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const uint16_t w = idx[v];
        uint32_t k = vacuum_skip(w);
        if (k <= 1u) continue;                   // non-vacuum, or already next to material
        const int x = (int)(v % (size_t)nx), y = (int)((v / (size_t)nx) % (size_t)ny), z = (int)(v / ((size_t)nx * ny));
        uint32_t best = k;
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = z + dz;
            if (zz < 0 || zz >= nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx;
                    if (xx < 0 || xx >= nx || (dx | dy | dz) == 0) continue;
                    const uint32_t kn = vacuum_skip(idx[((size_t)zz * ny + yy) * nx + xx]);
                    best = min(best, kn + 1u);
                }
            }
        }
        if (best < k) idx[v] = (uint16_t)(hu_index(w) | (best << kHuBits));
    }
}

__global__ void track_energy_kernel(const float4 *__restrict__ steps, const unsigned long long *__restrict__ off,
                                    long long *__restrict__ T, uint32_t n_tracks)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tracks) return;
    long long s = 0;
    for (unsigned long long k = off[t]; k < off[t + 1]; ++k) s += to_fp(steps[k].y);
    T[t] = s;
}

// the stored steps, in place, as the walk reads them: (dx, dE, theta, phi) ->
// (dx, fixed-point dE as int32 bits, theta cos phi, theta sin phi).  One
// 16-byte record per step carries everything the walk needs (the energy in
// the form it is split in, and the deflection without a per-step sincos).
__global__ void compact_steps_kernel(float4 *__restrict__ steps, unsigned long long n)
{
    for (unsigned long long k = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; k < n;
         k += (unsigned long long)gridDim.x * blockDim.x) {
        const float4 r = steps[k];
        float sp, cp;
        sincosf(r.w, &sp, &cp);
        steps[k] = make_float4(r.x, __int_as_float((int)to_fp(r.y)), r.z * cp, r.z * sp);
    }
}

// dose per primary = E / (rho V) / N and Eq. (2) variance of that mean; N is
// the plan's device history count
__global__ void dose_kernel(const uint16_t *__restrict__ idx, const unsigned long long *__restrict__ E,
                            const unsigned long long *__restrict__ E2, const float2 *__restrict__ lut,
                            const float *__restrict__ rho_lut, size_t nvox, double vol_cm3,
                            const unsigned long long *__restrict__ n_hist, double *__restrict__ dose,
                            double *__restrict__ var)
{
    const double N = (double)n_hist[0];
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const uint32_t m = hu_index(idx[v]);
        const bool vac = lut[m].x == 0.f || N <= 0.0;
        const double mass_kg = (double)rho_lut[m] * vol_cm3 * 1e-3;
        const double per = kMeVToJ / mass_kg;                // Gy per MeV in this voxel
        const double s1 = vac ? 0.0 : (double)(long long)E[v] * kFpMeV * per;
        if (dose) dose[v] = vac ? 0.0 : s1 / N;
        if (var) {
            const double s2 = vac || !E2 ? 0.0 : (double)E2[v] * kFpMeV * per * per;
            const double mean = vac ? 0.0 : s1 / N;
            var[v] = N > 1.0 ? (s2 / N - mean * mean) / (N - 1.0) : 0.0;
        }
    }
}

// after a transport launch: every item's spot counter moves past its histories
// and its plan's history count grows
__global__ void advance_kernel(const WorkItem *__restrict__ items, uint32_t n_items,
                               unsigned long long *__restrict__ hnext, const DevSpot *__restrict__ spots,
                               const DevPlan *__restrict__ plans)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const WorkItem it = items[i];
    hnext[it.gspot] += it.n;                 // one item per spot and launch: no race
    atomicAdd(plans[spots[it.gspot].plan].acc + 3, it.n);
}

// Work table of a run built on the device: one workgroup walks the listed
// spots in range order, each thread a contiguous run of them; a spot with
// histories becomes an item whose unit, history and ordering-chunk offsets are
// exclusive prefix sums (per thread, then across the workgroup's lanes and
// waves) of units_for(n), n and source_order_chunks(n).
constexpr uint32_t kItemThreads = 1024;

struct ItemSums {
    unsigned long long items, hist, units, chunks;
};

__device__ inline ItemSums wave_scan_incl(ItemSums v, uint32_t lane)
{
#pragma unroll
    for (uint32_t off = 1; off < kWave; off <<= 1) {
        const unsigned long long a = __shfl_up(v.items, off, kWave), b = __shfl_up(v.hist, off, kWave);
        const unsigned long long c = __shfl_up(v.units, off, kWave), d = __shfl_up(v.chunks, off, kWave);
        if (lane >= off) { v.items += a; v.hist += b; v.units += c; v.chunks += d; }
    }
    return v;
}

__global__ void __launch_bounds__(kItemThreads) build_items_kernel(const DevSpot *__restrict__ spots, SpotRanges r,
                                                                   WorkItem *__restrict__ items)
{
    __shared__ ItemSums s_wave[kItemThreads / kWave];
    const uint32_t t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    uint32_t total = 0;
    for (uint32_t i = 0; i < r.n; ++i) total += r.count[i];
    const uint32_t per = (total + kItemThreads - 1) / kItemThreads;
    const uint32_t j0 = min(total, t * per), j1 = min(total, j0 + per);
    // the DevSpot index of list position j
    auto gspot_of = [&](uint32_t j) {
        uint32_t i = 0;
        while (j >= r.count[i]) { j -= r.count[i]; ++i; }
        return r.first[i] + j;
    };
    ItemSums mine{0, 0, 0, 0};
    for (uint32_t j = j0; j < j1; ++j) {
        const unsigned long long n = spots[gspot_of(j)].n_hist;
        if (!n) continue;
        mine.items += 1;
        mine.hist += n;
        mine.units += units_for(n);
        mine.chunks += source_order_chunks(n);
    }
    const ItemSums incl = wave_scan_incl(mine, lane);
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    ItemSums run{incl.items - mine.items, incl.hist - mine.hist, incl.units - mine.units, incl.chunks - mine.chunks};
    for (uint32_t w = 0; w < wave; ++w) {
        run.items += s_wave[w].items;
        run.hist += s_wave[w].hist;
        run.units += s_wave[w].units;
        run.chunks += s_wave[w].chunks;
    }
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t g = gspot_of(j);
        const unsigned long long n = spots[g].n_hist;
        if (!n) continue;
        WorkItem w{};
        w.h0 = 0;                              // the spot's device counter is added
        w.n = n;
        w.unit0 = run.units;
        w.first = run.hist;
        w.gspot = g;
        w.chunk0 = (uint32_t)run.chunks;
        items[run.items] = w;
        run.items += 1;
        run.hist += n;
        run.units += units_for(n);
        run.chunks += source_order_chunks(n);
    }
}

__global__ void fill_u64_kernel(unsigned long long *__restrict__ p, size_t n, unsigned long long value)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// density per voxel from the HU index (vacuum voxels report their table density)
__global__ void density_kernel(const uint16_t *__restrict__ idx, const float *__restrict__ rho_lut, size_t n,
                               float *__restrict__ rho)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        rho[v] = rho_lut[hu_index(idx[v])];
}

// denoiser input: channel 0 = dose * scale, channel 1 = density / 2
__global__ void denoise_input_kernel(const double *__restrict__ dose, const float *__restrict__ rho, size_t n,
                                     double scale, float *__restrict__ out)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        out[v] = (float)(dose[v] * scale);
        out[n + v] = 0.5f * rho[v];
    }
}

__global__ void sum_i64_kernel(const unsigned long long *__restrict__ x, size_t n, unsigned long long *out)
{
    __shared__ unsigned long long part[16];
    unsigned long long s = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        s += x[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        atomicAdd(out, t);
    }
}

__global__ void philox_test_kernel(const uint4 *ctr, uint4 *out, uint32_t n, uint32_t k0, uint32_t k1)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

uint32_t grid_for(size_t n, uint32_t block, uint32_t cap = 65536)
{
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

} // namespace

hipError_t launch_build_lut(const double *pts, int n_pts, double vacuum_below, float2 *lut, float *rho,
                            hipStream_t s)
{
    hipLaunchKernelGGL(build_lut_kernel, dim3(kLutSize / 256), dim3(256), 0, s, pts, n_pts, vacuum_below, lut, rho);
    return hipGetLastError();
}

hipError_t launch_hu_to_index(const int16_t *hu, uint16_t *idx, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(hu_to_index_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, hu, idx, n);
    return hipGetLastError();
}

hipError_t launch_compact_steps(float4 *steps, unsigned long long n, hipStream_t s)
{
    hipLaunchKernelGGL(compact_steps_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, steps, n);
    return hipGetLastError();
}

hipError_t launch_track_energy(const float4 *steps, const unsigned long long *off, long long *T,
                               uint32_t n_tracks, hipStream_t s)
{
    hipLaunchKernelGGL(track_energy_kernel, dim3((n_tracks + 255) / 256), dim3(256), 0, s, steps, off, T, n_tracks);
    return hipGetLastError();
}

hipError_t launch_dose(const uint16_t *idx, const unsigned long long *E, const unsigned long long *E2,
                       const float2 *lut, const float *rho_lut, size_t nvox, double vol,
                       const unsigned long long *n_hist, double *dose, double *var, hipStream_t s)
{
    hipLaunchKernelGGL(dose_kernel, dim3(grid_for(nvox, 256, 8192)), dim3(256), 0, s, idx, E, E2, lut, rho_lut,
                       nvox, vol, n_hist, dose, var);
    return hipGetLastError();
}

hipError_t launch_advance(const WorkItem *items, uint32_t n_items, unsigned long long *hnext, const DevSpot *spots,
                          const DevPlan *plans, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3((n_items + 255) / 256), dim3(256), 0, s, items, n_items, hnext, spots,
                       plans);
    return hipGetLastError();
}

hipError_t launch_vacuum_skip(uint16_t *idx, const float2 *lut, int nx, int ny, int nz, hipStream_t s)
{
    const size_t n = (size_t)nx * ny * nz;
    hipLaunchKernelGGL(skip_seed_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, idx, lut, n);
    for (uint32_t pass = 0; pass < kMaxSkip; ++pass)
        hipLaunchKernelGGL(skip_relax_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, idx, nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_build_items(const DevSpot *spots, const SpotRanges &r, WorkItem *items, hipStream_t s)
{
    hipLaunchKernelGGL(build_items_kernel, dim3(1), dim3(kItemThreads), 0, s, spots, r, items);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long value, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t launch_density(const uint16_t *idx, const float *rho_lut, size_t n, float *rho, hipStream_t s)
{
    hipLaunchKernelGGL(density_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, idx, rho_lut, n, rho);
    return hipGetLastError();
}

hipError_t launch_denoise_input(const double *dose, const float *rho, size_t n, double scale, float *out,
                                hipStream_t s)
{
    hipLaunchKernelGGL(denoise_input_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, dose, rho, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_sum_i64(const unsigned long long *x, size_t n, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_i64_kernel, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_philox_test(const uint4 *ctr, uint4 *out, uint32_t n, uint32_t k0, uint32_t k1, hipStream_t s)
{
    hipLaunchKernelGGL(philox_test_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctr, out, n, k0, k1);
    return hipGetLastError();
}

} // namespace fdc
