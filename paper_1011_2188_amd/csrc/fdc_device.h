// Internal layout shared by the library's host runtime and its kernels.
// Not part of the public ABI (include/fdc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdc {

constexpr int kLutSize = 4096;        // HU index = clamp(HU, -1024, 3071) + 1024
constexpr int kHuMin = -1024;
constexpr int kWave = 64;             // CDNA wavefront
constexpr uint32_t kTagTrack = 2u;    // Philox counter tags (word 3, low 4 bits)
constexpr uint32_t kTagSource = 3u;
constexpr uint32_t kFlagVariance = 1u;
constexpr uint32_t kFlagRotate = 2u;
constexpr int kMaxTablePts = 64;
constexpr size_t kMaxLdsBytes = 160 * 1024;   // LDS per workgroup on gfx950
constexpr size_t kLdsFixedBytes = 64;          // besides the material table and the tally: the ticket words
constexpr double kMeVToJ = 1.602176634e-13;
constexpr double kFpMeV = 1.0 / 16777216.0;   // one fixed-point unit in MeV

// A voxel's 16-bit word: the HU index (clamp(HU, -1024, 3071) + 1024) in the
// low 12 bits; in the high 4 bits, for a vacuum voxel, its Chebyshev distance
// in voxels to the nearest non-vacuum voxel of the plan, capped at 15 (0 for
// non-vacuum voxels): every voxel within distance skip - 1 is vacuum too.
constexpr uint32_t kHuBits = 12;
constexpr uint32_t kMaxSkip = 15;
__host__ __device__ inline uint32_t hu_index(uint16_t w) { return w & ((1u << kHuBits) - 1u); }
__host__ __device__ inline uint32_t vacuum_skip(uint16_t w) { return (uint32_t)w >> kHuBits; }

// one phantom + its tallies, as seen by the kernels
struct DevPlan {
    const uint16_t *idx;             // voxel word (HU index | vacuum skip << 12), x-fastest
    unsigned long long *E;           // int64 energy tally (two's complement in u64 adds)
    unsigned long long *E2;          // uint64 sum of squared per-visit deposits
    unsigned long long *acc;         // [0] incident, [1] escaped (fixed point), [2] scratch,
                                     // [3] histories run since the last reset, [4..6] work
                                     // counters (steps, voxel visits, flushes), [7] unused
    const float4 *ps;                // listed protons: (x, y, z, E MeV), (dx, dy, dz, 0) each
    int n[3];
    float vox[3];
    float inv_vox[3];                // 1 / vox (FP32)
    float org[3];
    double vox_d[3];
    double org_d[3];
};

// one spot with everything task 1 needs that does not depend on the history
struct DevSpot {
    double pos[3];
    double e1[3], e2[3], d[3];      // lateral axes and direction (double, for the source)
    float m[9];                     // field matrix, columns e1 e2 d (row-major m[r*3+c])
    float sigma;
    uint32_t bin;
    uint32_t plan;                  // plan id (Philox counter word 3)
    uint32_t spot;                  // spot index inside its plan (counter word 2)
    long long skip;                 // fp(E_bin) - fp(E_spot)
    unsigned long long n_hist;      // histories per run (the device-built work table reads it)
    // a source of listed protons (kind 1): history h is proton ps_first + h % ps_count
    // of the plan's list, which brings its own start, direction and energy
    uint32_t kind;                  // 0 spot, 1 listed protons
    int32_t dev;                    // beam-line device the spot's histories pass, -1 none
    long long bin_fp;               // fp(E_bin)
    unsigned long long ps_first, ps_count;
};

// a beam-line device upstream of the phantom (fdc_beam_device): its face
// plane, lateral axes and pixel grid, in FP64 like the source
struct DevDevice {
    double o[3], nrm[3], u1[3], u2[3];
    double pitch[2];
    int npix[2];
    double rsp, g;                  // compensator RSP and RScP / RSP
    const float *pix;               // < 0 closed, else thickness (cm) along nrm
};

// a secondary trajectory of the track database: a particle that starts at
// the end of one of its track's primary steps and replays steps of its own,
// kept behind the primary steps in the same step array
constexpr uint32_t kMaxSecPerTrack = 4;
struct DevSec {
    unsigned long long k0, k1;      // its steps: steps[k0 .. k1)
    unsigned long long kb;          // the primary step at whose end it starts (~0: the end marker)
    long long T;                    // its energy, fixed point
    float ct, st, cph, sph;         // cos and sin of its polar and azimuthal emission angles
};

// a contiguous range of histories of one spot, cut in wave units of 64
// histories aligned to multiples of 64.  The range starts at h0, plus the
// spot's device history counter hnext[gspot] when the launch has one (runs;
// debug end-point replays give h0 explicitly).  An item owns units_for(n)
// units, enough for any alignment of its start, so a captured launch stays
// valid while the counters advance.
struct WorkItem {
    unsigned long long h0;
    unsigned long long n;
    unsigned long long unit0;       // index of this item's first wave unit
    unsigned long long first;       // index of this item's first history among the run's
    uint32_t gspot;                 // index into the DevSpot array
    uint32_t chunk0;                // index of this item's first ordering chunk (start-position order)
};

__host__ __device__ inline unsigned long long units_for(unsigned long long n)
{
    return n ? (n + 62) / 64 + 1 : 0;
}

// start-position order: a spot's histories are ordered in chunks of this many
// (a multiple of the 64-history unit), one ordering workgroup per chunk
constexpr uint32_t kOrderChunk = 16384;
// spots of more histories than this are ordered as a whole (a device-memory
// histogram); smaller ones chunk by chunk in LDS (at most four chunks)
constexpr unsigned long long kOrderWholeSpot = 4ull * kOrderChunk;
__host__ __device__ inline unsigned long long source_order_chunks(unsigned long long n)
{
    return (n + kOrderChunk - 1) / kOrderChunk;
}

// The spots of one run as ranges of the DevSpot array (one per listed plan),
// for the work table built on the device (allocation-free runs).
constexpr uint32_t kMaxRangePlans = 64;
struct SpotRanges {
    uint32_t n;                          // ranges used
    uint32_t first[kMaxRangePlans];      // first DevSpot index of each listed plan
    uint32_t count[kMaxRangePlans];      // its spots
};

struct TransportArgs {
    const float4 *steps;                 // per step: (dx, fixed-point dE as int32 bits,
                                         // theta cos phi, theta sin phi), made at load
    const unsigned long long *track_off; // n_tracks + 1
    const long long *track_T;            // sum of fp(dE) per track
    const uint32_t *bin_first;           // n_bins + 1
    const DevPlan *plans;
    const DevSpot *spots;
    const WorkItem *items;
    const unsigned long long *hnext;     // per DevSpot: next history index (null: h0 is absolute)
    const float2 *lut;                   // (rsp, g) per HU index; rsp == 0 is vacuum
    unsigned long long n_units;
    unsigned long long *queue;           // persistent mode: next unit counter
    uint32_t n_items;
    uint32_t seed_lo, seed_hi;
    uint32_t R;
    uint32_t flags;
    float *ep_xyz;                       // endpoint mode outputs (else null)
    int *ep_reason;
    const uint32_t *order;               // per unit and lane: offset of the lane's history in its
                                         // item, 0xFFFFFFFF = none (null: consecutive histories)
    const DevDevice *devices;            // beam-line devices (DevSpot::dev indexes them)
    const uint32_t *sec_first;           // per track: its first secondary (null: none loaded)
    const DevSec *secs;                  // secondaries by track and branch step, then an end marker
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies with a Weyl key schedule.
__host__ __device__ inline void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                             uint32_t k0, uint32_t k1)
{
    const uint64_t a = (uint64_t)0xD2511F53u * c0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
}

__host__ __device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(c.x, c.y, c.z, c.w, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24 random bits mapped to the open interval (0, 1)
__host__ __device__ inline double u01(uint32_t x)
{
    return (double)(x >> 8) * 0x1p-24 + 0x1p-25;
}

// Global-memory views of device pointers.  The plan buffers are reached
// through pointers stored in device memory, which the compiler would otherwise
// access as generic (flat) pointers; a flat access also counts against the LDS
// wait counter, so an LDS lookup issued after a flat tally atomic would stall
// until that atomic completes.  (The qualifier applies to the device pass only;
// the host pass sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define FDC_AS_GLOBAL __attribute__((address_space(1)))
#else
#define FDC_AS_GLOBAL
#endif

__host__ __device__ inline uint16_t load_global(const uint16_t *p, uint32_t i)
{
    return ((const FDC_AS_GLOBAL uint16_t *)p)[i];
}

// relaxed device-scope 64-bit add without a return value
__device__ inline void add_global(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add((FDC_AS_GLOBAL unsigned long long *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// rintf(x) converted to int64, and int64 -> float; both take the 32-bit
// conversion when it gives the same result (values below 2^31 in magnitude),
// which is a few instructions instead of the general 64-bit sequence
__host__ __device__ inline long long rint_ll(float x)
{
    const float r = rintf(x);
    if (fabsf(r) < 2147483648.f) return (long long)(int)r;
    return (long long)r;
}

__host__ __device__ inline float ll_to_f(long long e)
{
    if (e == (long long)(int)e) return (float)(int)e;
    return (float)e;
}

// Reciprocal and reciprocal square root: the hardware approximations
// (v_rcp_f32, v_rsq_f32, about 1 ulp) in device code, exact division in the
// host pass (which only CPU checks of the walk compile).
__host__ __device__ inline float fast_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.f / x;
#endif
}

__host__ __device__ inline float fast_rsq(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.f / sqrtf(x);
#endif
}

__host__ __device__ inline float fast_sqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);          // v_sqrt_f32
#else
    return sqrtf(x);
#endif
}

// sin and cos of a small angle: Taylor series to x^9 and x^10 (truncation
// below 2e-11 for |x| <= 0.5, under FP32 rounding); sincosf beyond.
__host__ __device__ inline void small_sincos(float x, float *s, float *c)
{
    if (fabsf(x) <= 0.5f) {
        const float x2 = x * x;
        *s = x * fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.f / 362880.f, -1.f / 5040.f), 1.f / 120.f), -1.f / 6.f), 1.f);
        *c = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, -1.f / 3628800.f, 1.f / 40320.f), -1.f / 720.f),
                                    1.f / 24.f), -0.5f), 1.f);
    } else {
        sincosf(x, s, c);
    }
}

// energy in MeV (float) -> fixed point; exact for every float input
__host__ __device__ inline long long to_fp(float mev)
{
    return rint_ll(mev * 16777216.0f);
}

// kernels' host-side launchers (implemented next to their kernels)
hipError_t launch_transport(const TransportArgs &a, uint32_t waves_per_block, uint32_t grid_blocks,
                            bool variance, bool endpoints, hipStream_t s, bool count = false);
hipError_t launch_transport_lds(const TransportArgs &a, uint32_t waves_per_block, uint32_t grid_blocks,
                                uint32_t slots, uint32_t units_per_wave, bool variance, uint32_t mode, hipStream_t s);
size_t lds_tally_bytes(uint32_t slots, bool variance, uint32_t mode);
hipError_t cache_kernel_occupancy(uint32_t waves_per_block, uint32_t slots, bool variance, int *blocks);
hipError_t prepare_lds_kernels();
hipError_t launch_build_lut(const double *pts, int n_pts, double vacuum_below, float2 *lut, float *rho,
                            hipStream_t s);
hipError_t launch_hu_to_index(const int16_t *hu, uint16_t *idx, size_t n, hipStream_t s);
// the vacuum-skip bits of every voxel word of a plan, from the material table
hipError_t launch_vacuum_skip(uint16_t *idx, const float2 *lut, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_compact_steps(float4 *steps, unsigned long long n, hipStream_t s);
hipError_t launch_track_energy(const float4 *steps, const unsigned long long *off, long long *T,
                               uint32_t n_tracks, hipStream_t s);
hipError_t launch_dose(const uint16_t *idx, const unsigned long long *E, const unsigned long long *E2,
                       const float2 *lut, const float *rho_lut, size_t nvox, double voxel_volume_cm3,
                       const unsigned long long *n_hist, double *dose, double *var, hipStream_t s);
// processing order of a run's histories by start position (order.hip): the
// launches (fill of the per-unit lane table, one workgroup per chunk; with
// `large`, the whole-item histograms of the items of more than one chunk, in
// hist: hist_words = order_hist_words(...) counters)
// what the start-position order needs to tell histories whose track has secondary
// trajectories (sec_first null: the database has none)
struct OrderTracks {
    const uint32_t *bin_first;
    const uint32_t *sec_first;
    uint32_t R;
};
hipError_t launch_source_order(const WorkItem *items, uint32_t n_items, uint32_t n_chunks, unsigned long long n_units,
                               const DevSpot *spots, const unsigned long long *hnext, uint32_t seed_lo,
                               uint32_t seed_hi, uint32_t *order, uint32_t *hist, unsigned long long hist_words,
                               bool large, const OrderTracks &tracks, hipStream_t s);
// counters the whole-item histograms of a run of n histories in n_items items need
__host__ __device__ inline unsigned long long order_hist_words(unsigned long long n, unsigned long long n_items)
{
    return (n >> 4) + n_items + 1;
}
// the work table of a run over the spots of `r` (every spot with histories,
// in range order), built by one workgroup from the spots' n_hist; the same
// items the host builds for fdc_run_histories
hipError_t launch_build_items(const DevSpot *spots, const SpotRanges &r, WorkItem *items, hipStream_t s);
hipError_t launch_advance(const WorkItem *items, uint32_t n_items, unsigned long long *hnext, const DevSpot *spots,
                          const DevPlan *plans, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long value, hipStream_t s);
hipError_t launch_density(const uint16_t *idx, const float *rho_lut, size_t n, float *rho, hipStream_t s);
hipError_t launch_denoise_input(const double *dose, const float *rho, size_t n, double scale, float *out,
                                hipStream_t s);
hipError_t launch_sum_i64(const unsigned long long *x, size_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_dmax(const double *d, const uint16_t *idx, const float2 *lut, size_t n, double *part,
                       double *out3, hipStream_t s);
hipError_t launch_mean_uncertainty(const double *d, const double *var, const uint16_t *idx, const float2 *lut,
                                   size_t n, double frac, double *scratch, double *out3, hipStream_t s);
size_t metrics_scratch_doubles();
hipError_t launch_batch_uncertainty(const double *doses, uint32_t nb, size_t n, double *mean, double *sigma,
                                    hipStream_t s);
hipError_t launch_gamma(const double *ref, const double *ev, const uint16_t *idx, const float2 *lut, int nx, int ny,
                        int nz, const int4 *offs, const double *offd2, int n_offs, const double *dmax_out,
                        double dose_frac, double cutoff_frac, float *gamma, unsigned long long *counts,
                        hipStream_t s);
hipError_t launch_philox_test(const uint4 *ctr, uint4 *out, uint32_t n, uint32_t k0, uint32_t k1,
                              hipStream_t s);

} // namespace fdc
