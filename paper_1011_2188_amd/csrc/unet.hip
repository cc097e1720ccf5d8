// Dose denoiser: a 3-level 3D U-Net (16/32/64 channels) trained and run with
// hand-written BF16 MFMA kernels accumulating in FP32 (CDNA4
// v_mfma_f32_16x16x32_bf16).
//
// Activations are bfloat16, channels-last: element (voxel v, channel c) of a
// view is p[v * pitch + c], channel counts padded to multiples of 8 so that a
// lane loads 8 channels (16 bytes) at once; the network's two input channels
// are kept unpadded for the first convolution (and padded for its weight
// gradients).  A decoder's input, the concatenation of the up-convolution's
// output and the skip, is two dense buffers that the kernels stage as one (no
// copies).  Weights live as FP32 master copies in the canonical
// layout of the network description (per layer: weights, then biases) and are
// packed to bfloat16 GEMM operands after every update.
//
// Kernels:
//   igemm    implicit GEMM, rows = voxels, cols = output channels, K = kernel
//            offsets x input channels.  Operand gathers: 3x3x3 neighbours with
//            zero padding, 1x1, or the 8 fine voxels of a coarse voxel.
//            Epilogues: bias, ReLU, a 0/1 mask (ReLU backward), bf16 store, or
//            a depth-to-space store (transposed convolution).
//   wgrad    weight gradient sum_v P[v][i] * Q[map(v, o)][j] over voxels, tiles
//            transposed through LDS, per-slab partials summed in a fixed order.
//   small kernels: input packing, the adjoint of the 2x2x2 average pool (the
//            pool itself runs in the epilogue of the convolution before it), the
//            1x1 head with residual and MSE loss, bias gradients, Adam.
#include "fdc.h"
#include "fdc_device.h"

#include <algorithm>
#include <cmath>
#include <random>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace fdc {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

enum { A_CONV3 = 0, A_CONV1 = 1, A_S2D = 2 };
enum { E_STORE = 0, E_D2S = 1 };

struct Grid {
    int nx, ny, nz;
};

__device__ inline u16 f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);            // round to nearest even
    return (u16)(u >> 16);
}

__device__ inline float bf2f(u16 b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

__device__ inline bf16x8 load8(const u16 *p)
{
    const uint4 q = *(const uint4 *)p;
    return __builtin_bit_cast(bf16x8, q);
}

// zero the bf16 elements of v whose mask element is not > 0 (8 at a time)
__device__ inline uint4 mask8(uint4 v, uint4 m)
{
    uint32_t vv[4] = {v.x, v.y, v.z, v.w};
    const uint32_t mm[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t keep = (bf2f((u16)(mm[i] & 0xFFFFu)) > 0.f ? 0x0000FFFFu : 0u) |
                              (bf2f((u16)(mm[i] >> 16)) > 0.f ? 0xFFFF0000u : 0u);
        vv[i] &= keep;
    }
    return make_uint4(vv[0], vv[1], vv[2], vv[3]);
}

__device__ inline bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// ---------------------------------------------------------------------------
// implicit GEMM.  One wave computes 16*MT consecutive rows x 16*NT columns.
// Rows index the row grid g (output voxels; coarse voxels for D2S and S2D).
// Operand A[row][k], k = o * cpad + c (o: kernel offset, c: source channel):
//   A_CONV3: source voxel = row voxel + (dz-1, dy-1, dx-1), o = (dz*3+dy)*3+dx
//   A_CONV1: source voxel = row voxel
//   A_S2D  : source grid is 2x finer, source voxel = 2*row + (a>>2, (a>>1)&1, a&1), o = a
// Operand B[k][n] = wpk[n * kpad + k] (packed weights, zero padded).
// v_mfma_f32_16x16x32_bf16 lane layout: A[i][k] in lane i + 16*(k/8), element
// k%8; B[k][j] in lane j + 16*(k/8), element k%8; D[i][j] in lane j +
// 16*(i/4), element i%4.
// Columns are split over blockIdx.y in blocks of 16*NT.
template <int AM, int EM, int MT, int NT>
__global__ void __launch_bounds__(256) igemm_kernel(const u16 *__restrict__ src, int src_pitch, int cpad, Grid g,
                                                    const u16 *__restrict__ wpk, int kpad, int n_cols,
                                                    const float *__restrict__ bias, int relu,
                                                    const u16 *__restrict__ mask, int mask_pitch,
                                                    u16 *__restrict__ dst, int dst_pitch, int d2s_cout)
{
    const int n_base = blockIdx.y * 16 * NT;
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long n_rows = (long)g.nx * g.ny * g.nz;
    const long row0 = (long)wave * (16 * MT);
    if (row0 >= n_rows) return;
    const int li = lane & 15, lg = lane >> 4;
    const int n_off = AM == A_CONV3 ? 27 : AM == A_S2D ? 8 : 1;
    const int kvalid = n_off * cpad;
    const int fx = 2 * g.nx, fy = 2 * g.ny;     // fine grid (A_S2D sources)

    // (grids hold fewer than 2^31 rows, checked by the host: 32-bit divisions)
    const uint32_t unx = (uint32_t)g.nx, uny = (uint32_t)g.ny;
    int rz[MT], ry[MT], rx[MT];
    bool rok[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const long r = row0 + 16 * m + li;
        rok[m] = r < n_rows;
        const uint32_t rr = rok[m] ? (uint32_t)r : 0u;
        const uint32_t q = rr / unx;
        rx[m] = (int)(rr - q * unx);
        ry[m] = (int)(q % uny);
        rz[m] = (int)(q / uny);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < kpad; k0 += 32) {
        const int k = k0 + 8 * lg;
        const int o = k / cpad, c = k - o * cpad;
        bf16x8 a[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            a[m] = zero8();
            if (k < kvalid && rok[m]) {
                long sv = -1;
                if (AM == A_CONV3) {
                    const int z = rz[m] + o / 9 - 1, y = ry[m] + (o / 3) % 3 - 1, x = rx[m] + o % 3 - 1;
                    if (z >= 0 && z < g.nz && y >= 0 && y < g.ny && x >= 0 && x < g.nx)
                        sv = ((long)z * g.ny + y) * g.nx + x;
                } else if (AM == A_CONV1) {
                    sv = ((long)rz[m] * g.ny + ry[m]) * g.nx + rx[m];
                } else {
                    const int z = 2 * rz[m] + (o >> 2), y = 2 * ry[m] + ((o >> 1) & 1), x = 2 * rx[m] + (o & 1);
                    sv = ((long)z * fy + y) * fx + x;
                }
                if (sv >= 0) a[m] = load8(src + sv * src_pitch + c);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = n_base + 16 * t + li;
            const bf16x8 b = n < n_cols ? load8(wpk + (long)n * kpad + k) : zero8();
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][t], 0, 0, 0);
        }
    }
    // epilogue: lane holds D[4*lg + e][li] of every (m, t) tile.  The bias
    // (one value per column) and the masks are loaded before any use, so their
    // round trips overlap instead of queueing one per element.
    float bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = n_base + 16 * t + li;
        const int co = EM == E_STORE ? n : n - (n / d2s_cout) * d2s_cout;
        bv[t] = (bias && n < n_cols) ? bias[co] : 0.f;
    }
    if constexpr (EM == E_D2S) {
        // The columns of a row are (sub-voxel a8, channel co) of 8 fine voxels.
        // Per-element stores would write 2 bytes per lane, scattered over 8
        // fine voxels; the wave instead places its tile in LDS (bf16, rows of
        // 16 NT columns) and then writes 16-byte runs of 8 channels of one
        // fine voxel per lane.  Needs d2s_cout, dst_pitch and dst 8-element
        // aligned (checked by the host).  The tile is private to the wave.
        constexpr int TP = 16 * NT + 8;                     // row pitch (16-byte rows, skewed banks)
        __shared__ __attribute__((aligned(16))) u16 stile[4][16 * MT * TP];
        u16 *tl = stile[threadIdx.x >> 6];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[m][t][e] + bv[t];
                    if (relu) v = fmaxf(v, 0.f);
                    tl[(16 * m + 4 * lg + e) * TP + 16 * t + li] = f2bf(v);
                }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr int CH = 2 * NT;                          // 16-byte chunks per row
#pragma unroll
        for (int q0 = 0; q0 < 16 * MT * CH; q0 += 64) {
            const int q = q0 + lane, rl = q / CH, cc = q % CH;
            const long r = row0 + rl;
            const int n = n_base + 8 * cc;
            if (r >= n_rows || n >= n_cols) continue;
            const int a8 = n / d2s_cout, co = n - a8 * d2s_cout;
            const uint32_t r32 = (uint32_t)r, qy = r32 / unx;
            const int x = (int)(r32 - qy * unx), y = (int)(qy % uny), z = (int)(qy / uny);
            const long fv = ((long)(2 * z + (a8 >> 2)) * fy + (2 * y + ((a8 >> 1) & 1))) * fx + 2 * x + (a8 & 1);
            *(uint4 *)(dst + fv * dst_pitch + co) = *(const uint4 *)(tl + rl * TP + 8 * cc);
        }
        return;
    }
    u16 mk[MT][NT][4];
    if (mask) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const long r = row0 + 16 * m + 4 * lg + e;
                    const int n = n_base + 16 * t + li;
                    const bool in = r < n_rows && n < n_cols;
                    mk[m][t][e] = mask[(in ? r : 0) * mask_pitch + (in ? n : 0)];
                }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = n_base + 16 * t + li;
            if (n >= n_cols) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long r = row0 + 16 * m + 4 * lg + e;
                if (r >= n_rows) continue;
                float v = acc[m][t][e] + bv[t];
                if (relu) v = fmaxf(v, 0.f);
                if (mask && !(bf2f(mk[m][t][e]) > 0.f)) v = 0.f;
                dst[r * dst_pitch + n] = f2bf(v);
            }
        }
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution (forward and backward-data) with the input tile in LDS.
// A block computes an output tile of 16 (x) x TY (y) x 4 (z) voxels for 16*NT
// output channels: it stages the tile and a one-voxel halo, (TY+2) x 6 x 18
// voxels of all input channels, into LDS once (channels-last, 16-byte rows),
// then every kernel tap is an offset into that copy instead of a new gather
// through the caches.  Wave w computes the z slice w; its m-th MFMA row tile
// is the 16 voxels of x at y = m.  K = 27 taps x cpad channels, in steps of 32
// (lane group lg takes 8 channels of tap (k0 + 8 lg) / cpad).  Weights (the
// B operand) come from the packed table in global memory, as in igemm.
// Copy `total` 16-byte items into LDS, B per thread in flight: all loads of a
// batch are issued before its stores (a load followed by its own store would
// serialise the global round trips).  src(t): global address or null (zeros);
// dst(t): LDS address.
template <int B, class Src, class Dst>
__device__ inline void stage16(int total, Src src, Dst dst)
{
    for (int t0 = threadIdx.x; t0 < total; t0 += B * (int)blockDim.x) {
        uint4 v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int t = t0 + b * (int)blockDim.x;
            const u16 *p = t < total ? src(t) : nullptr;
            v[b] = p ? *(const uint4 *)p : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int t = t0 + b * (int)blockDim.x;
            if (t < total) *(uint4 *)dst(t) = v[b];
        }
    }
}

// CS < CP: the input channels are staged CS at a time (phases of all 27 taps
// over CS channels), so the tile fits LDS with room for more blocks per CU.
// Input channels from `split` on come from a second buffer (src2, its own
// pitch, channel c - split): a decoder's input is the concatenation of the
// up-convolution's output and the skip, kept as two dense buffers so that
// their producers write whole cache lines.
template <int NT, int TY, int CP, int CS = CP>
__global__ void __launch_bounds__(256) conv3_kernel(const u16 *__restrict__ src, int src_pitch,
                                                    const u16 *__restrict__ src2, int src2_pitch, int split, Grid g,
                                                    const u16 *__restrict__ wpk, int kpad, int n_cols,
                                                    const float *__restrict__ bias, int relu,
                                                    const u16 *__restrict__ mask, int mask_pitch,
                                                    u16 *__restrict__ dst, int dst_pitch, int vec,
                                                    u16 *__restrict__ pool_dst, int pool_pitch,
                                                    const float *__restrict__ head_w,
                                                    const float *__restrict__ head_in, float *__restrict__ head_out)
{
    constexpr int TX = 16, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    static_assert(CP % CS == 0 && (CS == CP || CS % 32 == 0), "phases of whole K steps");
    // NARROW (two input channels, the network's input): the tile holds 4 bytes
    // per voxel, and a lane group's 8 K elements are the two channels of four
    // consecutive taps, K = 54 in two steps instead of 27 x 8 in seven
    constexpr bool NARROW = CP == 2;
    static_assert(!NARROW || CS == 2, "two channels in one phase");
    constexpr int HP = NARROW ? 2 : CS + 8;                // LDS channel pitch (16-byte rows, skewed banks)
    constexpr int GSHIFT = CS == 8 ? 0 : CS == 16 ? 1 : CS == 32 ? 2 : 3;   // CS / 8 = 1 << GSHIFT
    constexpr int KVALID = 27 * CS;                        // K of one phase
    constexpr int STEPS = (KVALID + 31) / 32;              // K steps of 32 per phase
    constexpr int PH = CP / CS;                            // phases
    constexpr int TOTAL = PH * STEPS;
    constexpr int D0 = NT == 1 ? 8 : NT == 2 ? 4 : 2;
    constexpr int D = D0 < TOTAL ? D0 : TOTAL;             // weight look-ahead, in K steps
    extern __shared__ __attribute__((aligned(16))) u16 sh[];
    const int tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
    const int bx = blockIdx.x % tiles_x, by = (blockIdx.x / tiles_x) % tiles_y, bz = blockIdx.x / (tiles_x * tiles_y);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int n_base = blockIdx.y * 16 * NT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int z = z0 + w;                                  // the wave's output slice
    const u16 *wrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = n_base + 16 * t + li;
        wrow[t] = wpk + (long)(n < n_cols ? n : 0) * kpad;
    }
    // weight fragments of K step gs (phase gs / STEPS): the lane group's 8
    // channels c of tap o sit at k = o CP + CS phase + c of the packed table.
    // Plain loads (no select on the loaded value, which would make the wave
    // wait for it at once).  The packed table is zero from 27 CP to kpad, and
    // columns past n_cols are never stored.
    auto load_w = [&](bf16x8 *b, int gs) {
        const int kl = 32 * (gs % STEPS) + 8 * lg;
        const int k = (kl / CS) * CP + (gs / STEPS) * CS + kl % CS;
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = load8(wrow[t] + k);
    };
    // Staged output (see the epilogue): 16 TY voxels x 16 NT channels per wave
    // in the input tile's LDS, 16-byte chunks of 8 channels of one voxel.
    constexpr int TP = 16 * NT + 8;                        // voxel pitch (16-byte rows, skewed banks)
    // the output tiles fit (a NARROW launch allocates LDS for them)
    constexpr bool STAGE = NARROW || 4 * 16 * TY * TP <= HZ * HY * HX * HP;
    constexpr int CH = 2 * NT;                             // chunks per voxel
    constexpr int NQ = STAGE ? 16 * TY * CH / 64 : 1;      // chunks per lane
    static_assert(!STAGE || (16 * TY * CH) % 64 == 0, "whole chunk rounds");
    // Everything the block reads from global memory besides the input tile
    // (the first D weight steps, the bias, the mask chunks) is requested
    // before the tile, so the block waits for one round trip, not four.
    bf16x8 ring[D][NT];
#pragma unroll
    for (int j = 0; j < D; ++j) load_w(ring[j], j);
    float bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = n_base + 16 * t + li;
        bv[t] = (bias && n < n_cols) ? bias[n] : 0.f;
    }
    uint4 mq[NQ];
    if (STAGE && vec && mask) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = 64 * i + lane, vl = q / CH, cc = q % CH;
            const int x = x0 + (vl & 15), y = y0 + (vl >> 4), n = n_base + 8 * cc;
            const bool in = x < g.nx && y < g.ny && z < g.nz && n < n_cols;
            const long r = in ? ((long)z * g.ny + y) * g.nx + x : 0;
            mq[i] = *(const uint4 *)(mask + r * mask_pitch + (in ? n : 0));
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // channels CS ph .. CS ph + CS - 1 of the tile and its halo into LDS
    auto stage = [&](int ph) {
        if constexpr (NARROW) {
            // one 4-byte item per tile voxel, eight loads in flight per thread
            constexpr int NV = HZ * HY * HX;
            for (int t0 = threadIdx.x; t0 < NV; t0 += 8 * (int)blockDim.x) {
                uint32_t q[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int h = t0 + b * (int)blockDim.x;
                    const int x = x0 - 1 + h % HX, y = y0 - 1 + (h / HX) % HY, z = z0 - 1 + h / (HX * HY);
                    const bool in = h < NV && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
                    q[b] = in ? *(const uint32_t *)(src + (((long)z * g.ny + y) * g.nx + x) * src_pitch) : 0u;
                }
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int h = t0 + b * (int)blockDim.x;
                    if (h < NV) *(uint32_t *)(sh + h * HP) = q[b];
                }
            }
            return;
        }
        stage16<8>((HZ * HY * HX) << GSHIFT,
                [&](int t) -> const u16 * {
                    const int h = t >> GSHIFT, cg = t & ((1 << GSHIFT) - 1);
                    const int x = x0 - 1 + h % HX, y = y0 - 1 + (h / HX) % HY, z = z0 - 1 + h / (HX * HY);
                    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz) return nullptr;
                    const long v = ((long)z * g.ny + y) * g.nx + x;
                    const int c = CS * ph + 8 * cg;
                    return c < split ? src + v * src_pitch + c : src2 + v * src2_pitch + (c - split);
                },
                [&](int t) { return sh + (t >> GSHIFT) * HP + 8 * (t & ((1 << GSHIFT) - 1)); });
    };
    stage(0);
    __syncthreads();
    // element offset of this lane's row in each m tile at tap 0
    int base[TY];
#pragma unroll
    for (int m = 0; m < TY; ++m) base[m] = ((w * HY + m) * HX + li) * HP;
    f32x4 acc[TY][NT];
#pragma unroll
    for (int m = 0; m < TY; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // LDS element offset of the lane's A fragment in step st of a phase: tap
    // o = (32 st + 8 lg) / CS at halo offset ((o/9) HY + (o/3)%3) HX + o%3,
    // channel (32 st + 8 lg) % CS.  For CS >= 32 the tap does not depend on the
    // lane; for smaller CS the lane group picks one of 32/CS taps of the step.
    auto a_off = [&](int st) {
        const int k = 32 * st + 8 * lg;
        const int o = k / CS, c = k % CS;
        return (((o / 9) * HY + (o / 3) % 3) * HX + o % 3) * HP + c;
    };
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
        if (ph > 0) {                                      // every wave is done with the previous channels
            __syncthreads();
            stage(ph);
            __syncthreads();
        }
#pragma unroll
        for (int st = 0; st < STEPS; ++st) {
            const int gs = ph * STEPS + st;
            const bool kv = 32 * st + 8 * lg < KVALID;    // false only in a last, partial step
            const int off = kv ? a_off(st) : 0;
            bf16x8 a[TY];
#pragma unroll
            for (int m = 0; m < TY; ++m) a[m] = NARROW ? zero8() : load8(sh + base[m] + off);
            if constexpr (NARROW) {
                // taps 16 st + 4 lg + j, j = 0..3, both channels of each (zero past the 27th)
                int to[4];
                bool tv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = 16 * st + 4 * lg + j;
                    tv[j] = o < 27;
                    const int oc = tv[j] ? o : 0;
                    to[j] = (((oc / 9) * HY + (oc / 3) % 3) * HX + oc % 3) * HP;
                }
#pragma unroll
                for (int m = 0; m < TY; ++m) {
                    uint32_t q[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) q[j] = tv[j] ? *(const uint32_t *)(sh + base[m] + to[j]) : 0u;
                    a[m] = __builtin_bit_cast(bf16x8, make_uint4(q[0], q[1], q[2], q[3]));
                }
            }
#pragma unroll
            for (int m = 0; m < TY; ++m) {
                const bf16x8 am = (32 * st + 32 <= KVALID || kv) ? a[m] : zero8();
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, ring[gs % D][t], acc[m][t], 0, 0, 0);
            }
            if (gs + D < TOTAL) load_w(ring[gs % D], gs + D);
            // keep each step's loads in their step: the scheduler would otherwise
            // sink the look-ahead loads next to their use
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // epilogue: lane holds D[4 lg + e][li] of every (m, t) tile: voxel x = x0 + 4 lg + e.
    if (STAGE && vec) {
        // Staged output: each wave writes its 16 TY voxels x 16 NT channels
        // (bias, ReLU applied, bf16) into the LDS the input tile used, then
        // stores 16-byte runs of 8 channels of one voxel per lane, the mask
        // applied 8 channels at a time.  Per-element stores would write
        // 2 bytes per lane in 32-byte pieces of 4 voxels.  vec needs n_cols,
        // the pitches and the dst and mask pointers 8-element aligned (the
        // host checks).
        __syncthreads();                                   // every wave is done with the input tile
        u16 *tl = sh + w * (16 * TY * TP);
#pragma unroll
        for (int m = 0; m < TY; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[m][t][e] + bv[t];
                    if (relu) v = fmaxf(v, 0.f);
                    tl[(16 * m + 4 * lg + e) * TP + 16 * t + li] = f2bf(v);
                }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (pool_dst) {
            // fused 2x2x2 average pool of the block's (pool-aligned) output tile:
            // pool_dst[coarse v][c] = bf16(0.125 * sum of the 8 stored bf16 values),
            // summed in FP32 over a = 4 dz + 2 dy + dx = 0 .. 7
            __syncthreads();                               // every wave's slice is in LDS
            const int ch = (int)threadIdx.x, cq = ch % CH, cv = ch / CH;   // chunk of 8 channels, coarse voxel
            const int cx = cv % (TX / 2), cy = (cv / (TX / 2)) % (TY / 2), cz = cv / ((TX / 2) * (TY / 2));
            const int gx = x0 / 2 + cx, gy = y0 / 2 + cy, gz = z0 / 2 + cz, n = n_base + 8 * cq;
            if (cz < TZ / 2 && gx < g.nx / 2 && gy < g.ny / 2 && gz < g.nz / 2 && n < n_cols) {
                float acc8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const int wz = 2 * cz + (a >> 2), vy = 2 * cy + ((a >> 1) & 1), vx = 2 * cx + (a & 1);
                    const uint4 q = *(const uint4 *)(sh + wz * (16 * TY * TP) + (vy * 16 + vx) * TP + 8 * cq);
                    const u16 *hq = (const u16 *)&q;
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc8[k] += bf2f(hq[k]);
                }
                uint4 o;
                u16 *oh = (u16 *)&o;
#pragma unroll
                for (int k = 0; k < 8; ++k) oh[k] = f2bf(acc8[k] * 0.125f);
                const long cvox = ((long)gz * (g.ny / 2) + gy) * (g.nx / 2) + gx;
                *(uint4 *)(pool_dst + cvox * pool_pitch + n) = o;
            }
        }
        if (z >= g.nz) return;
        if (NT == 1 && TY == 4 && head_out) {
            // the network's 1x1 head (16 channels -> 1, bias) and the residual,
            // fused for inference: lane = voxel of the wave's 16 x 4 slice, its
            // 16 channels one row of the staged tile (the head kernel's sum order)
            const int x = x0 + (lane & 15), y = y0 + (lane >> 4);
            if (x < g.nx && y < g.ny) {
                const long r = ((long)z * g.ny + y) * g.nx + x;
                float yv = head_w[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) yv += head_w[c] * bf2f(tl[lane * TP + c]);
                head_out[r] = yv + head_in[r];
            }
        }
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = 64 * i + lane, vl = q / CH, cc = q % CH;
            const int x = x0 + (vl & 15), y = y0 + (vl >> 4), n = n_base + 8 * cc;
            if (x >= g.nx || y >= g.ny || n >= n_cols) continue;
            const long r = ((long)z * g.ny + y) * g.nx + x;
            uint4 o = *(const uint4 *)(tl + vl * TP + 8 * cc);
            if (mask) o = mask8(o, mq[i]);
            *(uint4 *)(dst + r * dst_pitch + n) = o;
        }
        return;
    }
    // per-element path.  The masks are loaded before any use, so their round
    // trips overlap instead of queueing one per element.
    if (z >= g.nz) return;
    u16 mk[TY][NT][4];
    if (mask) {
#pragma unroll
        for (int m = 0; m < TY; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int y = y0 + m, x = x0 + 4 * lg + e, n = n_base + 16 * t + li;
                    const bool in = y < g.ny && x < g.nx && n < n_cols;
                    const long r = ((long)z * g.ny + (in ? y : 0)) * g.nx + (in ? x : 0);
                    mk[m][t][e] = mask[r * mask_pitch + (in ? n : 0)];
                }
    }
#pragma unroll
    for (int m = 0; m < TY; ++m) {
        const int y = y0 + m;
        if (y >= g.ny) continue;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = n_base + 16 * t + li;
            if (n >= n_cols) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = x0 + 4 * lg + e;
                if (x >= g.nx) continue;
                const long r = ((long)z * g.ny + y) * g.nx + x;
                float v = acc[m][t][e] + bv[t];
                if (relu) v = fmaxf(v, 0.f);
                if (mask && !(bf2f(mk[m][t][e]) > 0.f)) v = 0.f;
                dst[r * dst_pitch + n] = f2bf(v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[slab][o][i][j] = sum over the slab's rows v of
// P[v][i] * Q[src(v, o)][j], with src as in the igemm gathers:
//   A_CONV3: Q on the row grid, neighbour o (zero outside);  A_S2D: Q on the
//   2x finer grid, sub-voxel o.  i < pc, j < qc (multiples of 16, zero padded).
// 32 rows at a time are staged in LDS transposed ([channel][row]) so that a
// lane's 8 consecutive rows of one channel are one 16-byte read.
template <int AM>
__global__ void __launch_bounds__(256) wgrad_kernel(const u16 *__restrict__ P, int p_pitch, int p_ch,
                                                    const u16 *__restrict__ Q, int q_pitch, int q_ch, Grid g,
                                                    long rows_per_slab, float *__restrict__ part, int pc, int qc)
{
    __shared__ __attribute__((aligned(16))) u16 sP[64 * 32];
    __shared__ __attribute__((aligned(16))) u16 sQ[64 * 32];
    const int o = blockIdx.x;
    const int slab = blockIdx.y;
    const int n_off = gridDim.x;
    const long n_rows = (long)g.nx * g.ny * g.nz;
    const long r_begin = (long)slab * rows_per_slab;
    const long r_end = std::min<long>(n_rows, r_begin + rows_per_slab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int tiles_i = pc / 16, tiles_j = qc / 16, n_tiles = tiles_i * tiles_j;
    const int fx = 2 * g.nx, fy = 2 * g.ny;
    f32x4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (long r0 = r_begin; r0 < r_end; r0 += 32) {
        // stage: thread -> (row 0..31, channel group of 8)
        for (int s = threadIdx.x; s < 32 * 8; s += blockDim.x) {
            const int rr = s & 31, cg = s >> 5;            // cg 0..7 -> channels 8cg..8cg+7
            const long r = r0 + rr;
            uint4 vp = make_uint4(0, 0, 0, 0), vq = make_uint4(0, 0, 0, 0);
            if (r < r_end) {
                if (8 * cg < p_ch) vp = *(const uint4 *)(P + r * p_pitch + 8 * cg);
                if (8 * cg < q_ch) {
                    // (grids hold fewer than 2^31 rows: 32-bit divisions)
                    const uint32_t r32 = (uint32_t)r, qy = r32 / (uint32_t)g.nx;
                    const int x = (int)(r32 - qy * (uint32_t)g.nx), y = (int)(qy % (uint32_t)g.ny),
                              z = (int)(qy / (uint32_t)g.ny);
                    long sv = -1;
                    if (AM == A_CONV3) {
                        const int zz = z + o / 9 - 1, yy = y + (o / 3) % 3 - 1, xx = x + o % 3 - 1;
                        if (zz >= 0 && zz < g.nz && yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx)
                            sv = ((long)zz * g.ny + yy) * g.nx + xx;
                    } else {
                        sv = ((long)(2 * z + (o >> 2)) * fy + (2 * y + ((o >> 1) & 1))) * fx + 2 * x + (o & 1);
                    }
                    if (sv >= 0) vq = *(const uint4 *)(Q + sv * q_pitch + 8 * cg);
                }
            }
            const u16 *hp = (const u16 *)&vp, *hq = (const u16 *)&vq;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                sP[(8 * cg + e) * 32 + rr] = hp[e];
                sQ[(8 * cg + e) * 32 + rr] = hq[e];
            }
        }
        __syncthreads();
        // MFMA over the 32 staged rows: K = rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int tile = wave + 4 * q;
            if (tile < n_tiles) {
                const int ti = tile / tiles_j, tj = tile % tiles_j;
                const bf16x8 a = load8(sP + (16 * ti + li) * 32 + 8 * lg);
                const bf16x8 b = load8(sQ + (16 * tj + li) * 32 + 8 * lg);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int tile = wave + 4 * q;
        if (tile >= n_tiles) continue;
        const int ti = tile / tiles_j, tj = tile % tiles_j;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * ti + 4 * lg + e, j = 16 * tj + li;
            part[(((long)slab * n_off + o) * pc + i) * qc + j] = acc[q][e];
        }
    }
}

// MFMA operands from row-major LDS tiles with the gfx950 LDS transpose read
// (ds_read_b64_tr_b16): within a 16-lane group, lane r addresses row R + r/4,
// channels c0 + 4 (r%4) .. +3, and lane i receives rows R..R+3 of channel
// c0 + i - four consecutive contraction elements, as the 16x16x32 bf16 MFMA
// operands want them (two reads give the lane's eight).

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s lds_v4s;

__device__ inline bf16x8 tr_frag(const u16 *tile, int pitch, int row, int col)
{
    // row: first of the lane group's 8 rows; col: channel base of the 16-wide tile
    const int lane = threadIdx.x & 63, li = lane & 15;
    const u16 *p0 = tile + (row + (li >> 2)) * pitch + col + 4 * (li & 3);
    const u16 *p1 = p0 + 4 * pitch;
    const v4s a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(__attribute__((address_space(3))) u16 *)p0);
    const v4s b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(__attribute__((address_space(3))) u16 *)p1);
    typedef short v8s __attribute__((ext_vector_type(8)));
    const v8s c = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf16x8, c);
}

// Weight gradient of a 3x3x3 convolution over 3D tiles.  A block loops over
// tiles of 16 (x) x TY x TZ voxels (tile t = blockIdx.x + k * gridDim.x) and
// owns the taps og * G .. og * G + G - 1 and the Q channels
// 16 qs oq .. 16 qs (oq + 1) - 1 (blockIdx.y = og * (qc / 16 / qs) + oq).  Per
// tile it stages the output gradient P of the tile (all its channels) and the
// block's channels of the input Q over the tile plus a one-voxel halo
// (row-major, 16-byte copies); the contraction runs over the
// tile's voxels in x-fastest order, 32 at a time.  Eight consecutive
// contraction voxels are 8 consecutive x of one row, and for every tap their
// shifted neighbours are 8 consecutive halo rows, so both MFMA operands come
// straight from ds_read_b64_tr_b16 with no boundary masks (the halo holds the
// zeros).  Q channels from q_split on come from Q2 (a concatenation kept as
// two buffers, as in conv3_kernel).  Accumulators stay in registers across the block's tiles;
// part[blockIdx.x][o][i][j] receives the block's sums.
template <int TY, int TZ, int PT>
__global__ void __launch_bounds__(256) wgrad3t_kernel(const u16 *__restrict__ P, int p_pitch, int p_ch,
                                                      const u16 *__restrict__ Q, int q_pitch, int q_ch,
                                                      const u16 *__restrict__ Q2, int q2_pitch, int q_split, Grid g,
                                                      float *__restrict__ part, int pc, int qc, int G, int qs)
{
    constexpr int TX = 16, HX = TX + 2, HY = TY + 2, HZ = TZ + 2, TV = TX * TY * TZ;
    extern __shared__ __attribute__((aligned(16))) u16 lds[];
    const int nq = qc / (16 * qs);                             // Q channel slices
    const int o0 = (blockIdx.y / nq) * G, q_off = 16 * qs * (blockIdx.y % nq);
    const int sp_pitch = pc + 8, sq_pitch = 16 * qs + 8;
    u16 *sP = lds;
    u16 *sQ = lds + TV * sp_pitch;
    const int tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY, tiles_z = (g.nz + TZ - 1) / TZ;
    const int n_tiles_grid = tiles_x * tiles_y * tiles_z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lg = lane >> 4;
    // Accumulators: PT = pc / 16 P channel tiles.  The block's work is G qs
    // groups (tap, Q channel tile); wave w owns groups w, w + 4, ... and, for
    // each, the PT tiles (ti, tj): one Q fragment read serves PT MFMAs, and the
    // PT P fragments of a K step are read once for all groups.
    const int n_grp = G * qs;                                  // <= 4 kMaxAcc / PT (the host picks G, qs)
    const int pcg = pc / 8, qcg = 2 * qs;
    // accumulator tiles per wave: 14 for the 16 x 4 x 2 tiles (16 x 32 channel layers keep all 27
    // taps in one block), 12 elsewhere (more registers slow the other shapes down)
    constexpr int kMaxAcc = (TY == 4 && TZ == 2) ? 14 : 12;
    constexpr int RMAX = kMaxAcc / PT;                         // groups per wave
    f32x4 acc[RMAX * PT];
#pragma unroll
    for (int q = 0; q < RMAX * PT; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int t = blockIdx.x; t < n_tiles_grid; t += gridDim.x) {
        const int bx = t % tiles_x, by = (t / tiles_x) % tiles_y, bz = t / (tiles_x * tiles_y);
        const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
        stage16<4>(TV * pcg,
                [&](int u) -> const u16 * {
                    const int k = u / pcg, cg = u - k * pcg;
                    const int x = x0 + k % TX, y = y0 + (k / TX) % TY, z = z0 + k / (TX * TY);
                    if (x >= g.nx || y >= g.ny || z >= g.nz || 8 * cg >= p_ch) return nullptr;
                    return P + (((long)z * g.ny + y) * g.nx + x) * p_pitch + 8 * cg;
                },
                [&](int u) { return sP + (u / pcg) * sp_pitch + 8 * (u % pcg); });
        stage16<4>(HZ * HY * HX * qcg,
                [&](int u) -> const u16 * {
                    const int h = u / qcg, cg = u - h * qcg;
                    const int x = x0 - 1 + h % HX, y = y0 - 1 + (h / HX) % HY, z = z0 - 1 + h / (HX * HY);
                    const int c = q_off + 8 * cg;
                    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz || c >= q_ch) return nullptr;
                    const long v = ((long)z * g.ny + y) * g.nx + x;
                    return c < q_split ? Q + v * q_pitch + c : Q2 + v * q2_pitch + (c - q_split);
                },
                [&](int u) { return sQ + (u / qcg) * sq_pitch + 8 * (u % qcg); });
        __syncthreads();
#pragma unroll 1
        for (int kb = 0; kb < TV / 32; ++kb) {
            // the lane group's 8 contraction voxels: x = 8 (lg % 2) .. +7 of tile row (y, z)
            const int k0 = 32 * kb + 8 * lg;
            const int xr = k0 % TX, yr = (k0 / TX) % TY, zr = k0 / (TX * TY);
            bf16x8 a[PT];                                      // the step's P fragments
#pragma unroll
            for (int ti = 0; ti < PT; ++ti) a[ti] = tr_frag(sP, sp_pitch, k0, 16 * ti);
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                const int gi = wave + 4 * r;
                if (gi < n_grp) {
                    const int o = o0 + gi / qs, tj = gi % qs;
                    const int dz = o / 9, dy = (o / 3) % 3, dx = o % 3;     // halo shift = tap
                    const int hrow = ((zr + dz) * HY + (yr + dy)) * HX + (xr + dx);
                    const bf16x8 b = tr_frag(sQ, sq_pitch, hrow, 16 * tj);
#pragma unroll
                    for (int ti = 0; ti < PT; ++ti)
                        acc[r * PT + ti] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti], b, acc[r * PT + ti], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    const int li = lane & 15;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const int gi = wave + 4 * r;
        if (gi >= n_grp) continue;
        const int o = o0 + gi / qs, tj = gi % qs;
#pragma unroll
        for (int ti = 0; ti < PT; ++ti)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * ti + 4 * lg + e, j = q_off + 16 * tj + li;
                part[(((long)blockIdx.x * 27 + o) * pc + i) * qc + j] = acc[r * PT + ti][e];
            }
    }
}

// sum the slabs in a fixed order, sum_s part[s][o][i][j] for element x = (o pc + i) qc + j,
// and store it as the canonical weight gradient (i < ni, j < nj; padding dropped):
//   conv3: i = co, j = ci  -> gw[co][ci][o];   tconv: i = ci, j = co -> gw[ci][co][o]
// Block = 64 elements x 8 waves: wave w adds slabs w, w + 8, ... (coalesced rows),
// then the 8 partial sums are added in wave order (reproducible).
__global__ void __launch_bounds__(512) slab_sum_kernel(const float *__restrict__ part, int slabs, long per_slab,
                                                       int pc, int qc, int ni, int nj, float *__restrict__ gw)
{
    __shared__ float red[8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long x = blockIdx.x * 64L + lane;
    float s = 0.f;
    if (x < per_slab) {
#pragma unroll 8
        for (int k = w; k < slabs; k += 8) s += part[k * per_slab + x];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && x < per_slab) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) t += red[k][lane];
        const int j = (int)(x % qc), i = (int)((x / qc) % pc), o = (int)(x / ((long)pc * qc));
        const int n_off = (int)(per_slab / ((long)pc * qc));
        if (i < ni && j < nj) gw[((long)i * nj + j) * n_off + o] = t;
    }
}

// Bias gradients of all layers, two launches for the whole backward pass.
// Job = one layer's output gradient G (n voxels x C channels, C a multiple of
// 8 up to 64, 16-byte aligned rows) and its bias gradient gb; its blocks are
// b0 .. b0 + nb - 1, per voxels each.
struct BiasJob {
    const u16 *G;
    float *gb;
    long n, per;
    int pitch, C, b0, nb;
};
constexpr int kMaxBiasJobs = 16;
constexpr int kMaxBiasBlocks = 512;                    // per job
struct BiasJobs {
    BiasJob j[kMaxBiasJobs];
    int n;
};

// partials: part[block][c] (stride 64) = sum over the block's voxels of G[v][c].
// Thread t reads 8 channels (16 bytes) of voxel v0 + t / (C/8) + k * (256 / (C/8)),
// so consecutive threads read consecutive bytes; the per-thread sums are then
// added per channel in a fixed order (reproducible).
__global__ void __launch_bounds__(256) bias_part_kernel(BiasJobs jobs, float *__restrict__ part)
{
    __shared__ float red[256][8];
    int jb = 0;
    while (jb + 1 < jobs.n && (int)blockIdx.x >= jobs.j[jb + 1].b0) ++jb;
    const BiasJob J = jobs.j[jb];
    const int C = J.C, cgs = C / 8, per_step = 256 / cgs;
    const int cg = threadIdx.x % cgs, vo = threadIdx.x / cgs;
    const long v0 = (long)((int)blockIdx.x - J.b0) * J.per, v1 = std::min<long>(J.n, v0 + J.per);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (vo < per_step) {
#pragma unroll 4
        for (long v = v0 + vo; v < v1; v += per_step) {
            const uint4 q = *(const uint4 *)(J.G + v * J.pitch + 8 * cg);
            const u16 *h = (const u16 *)&q;
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] += bf2f(h[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[threadIdx.x][e] = acc[e];
    __syncthreads();
    if ((int)threadIdx.x < C) {
        const int c = threadIdx.x, g8 = c / 8, e = c % 8;
        float sum = 0.f;
        for (int k = 0; k < per_step; ++k) sum += red[k * cgs + g8][e];
        part[(long)blockIdx.x * 64 + c] = sum;
    }
}

// FP32 [2][n] channels-first input -> bf16 channels-last, pitch 2 or 8 (zeros beyond 2)
__global__ void pack_input_kernel(const float *__restrict__ in, long n, u16 *__restrict__ x, int pitch)
{
    for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
        const uint32_t lo = f2bf(in[v]), hi = f2bf(in[n + v]);
        if (pitch == 2)
            *(uint32_t *)(x + v * 2) = lo | (hi << 16);
        else
            *(uint4 *)(x + v * 8) = make_uint4(lo | (hi << 16), 0u, 0u, 0u);
    }
}

// adjoint of the pool plus the skip-connection gradient, masked by ReLU:
// ge[fine v][c] = bf16( (bf16(gp[coarse(v)][c] / 8) + skip[v][c]) * (e[v][c] > 0) )
// 8 channels (16 bytes of every operand) per thread: C, the pitches and the
// pointers are 8-element aligned (the host checks).
__global__ void pool_back_kernel(const u16 *__restrict__ gp, int gp_pitch, const u16 *__restrict__ skip,
                                 int skip_pitch, const u16 *__restrict__ e, int e_pitch, int C, Grid fine,
                                 u16 *__restrict__ ge, int ge_pitch)
{
    const long n = (long)fine.nx * fine.ny * fine.nz;
    const int cx = fine.nx / 2, cy = fine.ny / 2, cgs = C / 8;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n * cgs; t += (long)gridDim.x * blockDim.x) {
        const long v = t / cgs;
        const int c = 8 * (int)(t - v * cgs);
        const int x = (int)(v % fine.nx), y = (int)((v / fine.nx) % fine.ny), z = (int)(v / ((long)fine.nx * fine.ny));
        const long cv = ((long)(z / 2) * cy + y / 2) * cx + x / 2;
        const uint4 g4 = *(const uint4 *)(gp + cv * gp_pitch + c);
        const uint4 s4 = *(const uint4 *)(skip + v * skip_pitch + c);
        const uint4 e4 = *(const uint4 *)(e + v * e_pitch + c);
        const u16 *gh = (const u16 *)&g4, *sh = (const u16 *)&s4, *eh = (const u16 *)&e4;
        uint4 o4;
        u16 *oh = (u16 *)&o4;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float up = bf2f(f2bf(bf2f(gh[k]) * 0.125f));
            const float sum = bf2f(sh[k]) + up;
            oh[k] = f2bf(bf2f(eh[k]) > 0.f ? sum : 0.f);
        }
        *(uint4 *)(ge + v * ge_pitch + c) = o4;
    }
}

// head: y = w . d1 + b + dose; loss partials; gy = 2 (y - t) / N; the head's
// input gradient w * gy masked by d1 > 0 (bf16) and its weight/bias partials
__global__ void head_kernel(const u16 *__restrict__ d1, int pitch, const float *__restrict__ in, long n,
                            const float *__restrict__ w, const float *__restrict__ target, float *__restrict__ y_out,
                            u16 *__restrict__ gd1, double *__restrict__ loss_part, float *__restrict__ gw_part,
                            long per_block)
{
    __shared__ double s_loss[256];
    __shared__ float s_g[256][17];
    const long v0 = blockIdx.x * per_block, v1 = std::min<long>(n, v0 + per_block);
    double l = 0.0;
    float gwl[17];
    for (int c = 0; c < 17; ++c) gwl[c] = 0.f;
    const double inv_n = 1.0 / (double)n;
    // a voxel's 16 channels are read and written as two 16-byte halves (pitch
    // and buffers 8-element aligned: the head runs on the pitch-16 d1 buffers)
    for (long v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        const uint4 q[2] = {*(const uint4 *)(d1 + v * pitch), *(const uint4 *)(d1 + v * pitch + 8)};
        const u16 *hq = (const u16 *)q;
        float h[16];
        float y = w[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            h[c] = bf2f(hq[c]);
            y += w[c] * h[c];
        }
        y += in[v];
        if (y_out) y_out[v] = y;
        if (target) {
            const float d = y - target[v];
            l += (double)d * d;
            const float gy = (float)(2.0 * d * inv_n);
            uint4 o[2];
            u16 *oh = (u16 *)o;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                gwl[c] += gy * h[c];
                oh[c] = f2bf(h[c] > 0.f ? w[c] * gy : 0.f);
            }
            *(uint4 *)(gd1 + v * pitch) = o[0];
            *(uint4 *)(gd1 + v * pitch + 8) = o[1];
            gwl[16] += gy;
        }
    }
    if (!target) return;
    s_loss[threadIdx.x] = l;
    for (int c = 0; c < 17; ++c) s_g[threadIdx.x][c] = gwl[c];
    __syncthreads();
    for (int wdt = blockDim.x / 2; wdt > 0; wdt >>= 1) {
        if ((int)threadIdx.x < wdt) {
            s_loss[threadIdx.x] += s_loss[threadIdx.x + wdt];
            for (int c = 0; c < 17; ++c) s_g[threadIdx.x][c] += s_g[threadIdx.x + wdt][c];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss_part[blockIdx.x] = s_loss[0] * inv_n;
        for (int c = 0; c < 17; ++c) gw_part[blockIdx.x * 17 + c] = s_g[0][c];
    }
}

__global__ void head_finish_kernel(const double *__restrict__ loss_part, const float *__restrict__ gw_part, int nb,
                                   double *__restrict__ loss, float *__restrict__ grad_head)
{
    const int c = threadIdx.x;
    // sequential sums (a fixed order), unrolled so that several loads are in flight
    if (c < 17) {
        float s = 0.f;
#pragma unroll 8
        for (int b = 0; b < nb; ++b) s += gw_part[b * 17 + c];
        grad_head[c] = s;
    }
    if (c == 0) {
        double l = 0.0;
#pragma unroll 8
        for (int b = 0; b < nb; ++b) l += loss_part[b];
        *loss = l;
    }
}

// Adam with bias correction (Kingma and Ba 2015) on the FP32 master copy
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ s, long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float si = b2 * s[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        s[i] = si;
        p[i] -= lr * (mi / c1) / (sqrtf(si / c2) + eps);
    }
}

// Pack FP32 canonical weights into bf16 GEMM operands wpk[n * kpad + k].
//   mode 0: conv3 forward   n = co,            k = o * cpad_in + ci,   w[co][ci][o]
//   mode 1: conv3 backward  n = ci,            k = o * cpad_out + co,  w[co][ci][26 - o]
//   mode 2: tconv forward   n = a * cout + co, k = ci,                 w[ci][co][a]
//   mode 3: tconv backward  n = ci,            k = a * cpad_out + co,  w[ci][co][a]
// One packing job per (layer, direction); all of them run in one launch, each
// job on its own contiguous range of blocks starting at b0.
struct PackJob {
    const float *w;
    u16 *wpk;
    int mode, cin, cout, cpad, n_cols, kpad, b0;
};
constexpr int kMaxPackJobs = 32;
struct PackJobs {
    PackJob j[kMaxPackJobs];
    int n;
};

__global__ void pack_kernel(PackJobs jobs)
{
    int jb = 0;
    while (jb + 1 < jobs.n && (int)blockIdx.x >= jobs.j[jb + 1].b0) ++jb;
    const PackJob J = jobs.j[jb];
    const int nb = (jb + 1 < jobs.n ? jobs.j[jb + 1].b0 : (int)gridDim.x) - J.b0;
    const long total = (long)J.n_cols * J.kpad;
    for (long t = (blockIdx.x - J.b0) * (long)blockDim.x + threadIdx.x; t < total; t += (long)nb * blockDim.x) {
        const int n = (int)(t / J.kpad), k = (int)(t - (long)n * J.kpad);
        float v = 0.f;
        if (J.mode == 0) {
            const int o = k / J.cpad, ci = k % J.cpad;
            if (o < 27 && ci < J.cin) v = J.w[((long)n * J.cin + ci) * 27 + o];
        } else if (J.mode == 1) {
            const int o = k / J.cpad, co = k % J.cpad;
            if (o < 27 && co < J.cout) v = J.w[((long)co * J.cin + n) * 27 + (26 - o)];
        } else if (J.mode == 2) {
            const int a = n / J.cout, co = n % J.cout;
            if (k < J.cin) v = J.w[((long)k * J.cout + co) * 8 + a];
        } else {
            const int a = k / J.cpad, co = k % J.cpad;
            if (a < 8 && co < J.cout) v = J.w[((long)n * J.cout + co) * 8 + a];
        }
        J.wpk[t] = f2bf(v);
    }
}

// head parameters as the head kernel reads them: bf16-rounded weights, FP32 bias
__global__ void head_weights_kernel(const float *__restrict__ p, float *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c < 16) out[c] = bf2f(f2bf(p[c]));
    if (c == 16) out[16] = p[16];
}

// gb[c] = sum over the job's nb partials, one block per job; 256 threads: thread t
// sums channel t % C over partials b = t / C, t / C + 256 / C, ... and the groups
// are added in a fixed order (reproducible)
__global__ void __launch_bounds__(256) bias_finish_kernel(BiasJobs jobs, const float *__restrict__ part)
{
    __shared__ float red[256];
    const BiasJob J = jobs.j[blockIdx.x];
    const int C = J.C, groups = 256 / C, c = threadIdx.x % C, j = threadIdx.x / C;
    float s = 0.f;
    if (j < groups) {
#pragma unroll 8
        for (int b = j; b < J.nb; b += groups) s += part[(long)(J.b0 + b) * 64 + c];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < C) {
        float t = 0.f;
        for (int k = 0; k < groups; ++k) t += red[k * C + threadIdx.x];
        J.gb[threadIdx.x] = t;
    }
}

// ------------------------------------------------------------------ host --
enum { K_CONV3 = 0, K_TCONV = 1, K_CONV1 = 2 };

struct LayerDesc {
    const char *name;
    int kind, cin, cout;
};

// the network, in the canonical parameter order (weights then biases per layer)
const LayerDesc kLayers[] = {
    {"enc1a", K_CONV3, 2, 16}, {"enc1b", K_CONV3, 16, 16}, {"enc2a", K_CONV3, 16, 32}, {"enc2b", K_CONV3, 32, 32},
    {"mida", K_CONV3, 32, 64}, {"midb", K_CONV3, 64, 64},  {"up2", K_TCONV, 64, 32},   {"dec2a", K_CONV3, 64, 32},
    {"dec2b", K_CONV3, 32, 32}, {"up1", K_TCONV, 32, 16},  {"dec1a", K_CONV3, 32, 16}, {"dec1b", K_CONV3, 16, 16},
    {"head", K_CONV1, 16, 1}};
constexpr int kNumLayers = 13;
static_assert(2 * kNumLayers <= kMaxPackJobs, "one forward and one backward packing job per layer");
enum { L_E1A, L_E1B, L_E2A, L_E2B, L_MA, L_MB, L_UP2, L_D2A, L_D2B, L_UP1, L_D1A, L_D1B, L_HEAD };

inline int pad8(int c) { return (c + 7) & ~7; }
inline int pad16(int c) { return (c + 15) & ~15; }
inline int pad32(int k) { return (k + 31) & ~31; }
// channels per tap in a 3x3x3 layer's forward K: the network's two input
// channels unpadded (the two-channel kernel), else padded to 8
inline int fwd_cpad(int cin) { return cin == 2 ? 2 : pad8(cin); }

long weight_count(const LayerDesc &L)
{
    return (long)L.cin * L.cout * (L.kind == K_CONV3 ? 27 : L.kind == K_TCONV ? 8 : 1);
}

long total_params()
{
    long n = 0;
    for (const LayerDesc &L : kLayers) n += weight_count(L) + L.cout;
    return n;
}

struct View {
    u16 *p;
    int pitch;
    int ch;
    // a concatenation held as two dense buffers: channels from `split` on are
    // channel c - split of p2 (pitch pitch2)
    u16 *p2 = nullptr;
    int pitch2 = 0;
    int split = 0;
};

} // namespace nn
} // namespace fdc

using namespace fdc;
using namespace fdc::nn;

struct fdc_unet {
    int device = 0;
    Grid g[3];                      // full, half, quarter resolution
    long nv[3];
    std::string err;
    long n_params = 0;
    long w_off[kNumLayers], b_off[kNumLayers];
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_s = nullptr;
    int step = 0;
    u16 *wpk_f[kNumLayers] = {}, *wpk_b[kNumLayers] = {};
    int kpad_f[kNumLayers] = {}, ncol_f[kNumLayers] = {}, kpad_b[kNumLayers] = {}, ncol_b[kNumLayers] = {};
    std::vector<void *> allocs;
    // activations (bf16, channels-last); x2: the input's two channels (the
    // forward pass), x: the same padded to 8 (weight gradients of the first layer)
    u16 *x, *x2, *e1a, *c1, *p1, *e2a, *c2, *p2, *ma, *m, *d2a, *d2, *d1a, *d1;
    // activation gradients
    u16 *gd1, *gd1a, *gc1, *gd2, *gd2a, *gc2, *gm, *gma, *gp2, *ge2, *ge2a, *gp1, *ge1, *ge1a;
    float *wpart = nullptr, *bpart = nullptr, *hpart = nullptr, *hw = nullptr;
    double *lpart = nullptr, *loss = nullptr;
    size_t wpart_n = 0;
};

namespace {

int ufail(fdc_unet *u, int code, const char *msg, hipError_t e = hipSuccess)
{
    if (u) u->err = std::string(msg) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : "");
    return code;
}

template <class T> T *ualloc(fdc_unet *u, size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    u->allocs.push_back(p);
    return (T *)p;
}

uint32_t blocks_for(long n, int per = 256, long cap = 16384) { return (uint32_t)std::max<long>(1, std::min<long>(cap, (n + per - 1) / per)); }

// one implicit-GEMM launch: rows on grid g, n_cols output columns
// the network's head fused into the last convolution's epilogue (inference)
struct HeadFuse {
    const float *w;     // 16 weights and the bias, as the head kernel reads them
    const float *in;    // the input's first channel (the residual)
    float *out;
};

hipError_t igemm(int am, int em, const View &src, int cpad, const Grid &g, const u16 *wpk, int kpad, int n_cols,
                 const float *bias, bool relu, const View *mask, const View &dst, int d2s_cout, hipStream_t s,
                 const View *pool = nullptr, const HeadFuse *head = nullptr)
{
    const long rows = (long)g.nx * g.ny * g.nz;
    const long waves = (rows + 31) / 32;                  // MT = 2: 32 rows per wave
    const int nt = n_cols >= 64 ? 4 : n_cols >= 32 ? 2 : 1;
    const dim3 grid((uint32_t)((waves + 3) / 4), (uint32_t)((n_cols + 16 * nt - 1) / (16 * nt)));
    const u16 *mp = mask ? mask->p : nullptr;
    const int mpitch = mask ? mask->pitch : 0;
#define IG(AM_, EM_, NT_) hipLaunchKernelGGL((igemm_kernel<AM_, EM_, 2, NT_>), grid, dim3(256), 0, s, src.p, src.pitch, \
                                             cpad, g, wpk, kpad, n_cols, bias, (int)relu, mp, mpitch, dst.p, dst.pitch, d2s_cout)
#define IGN(AM_, EM_) do { if (nt == 4) IG(AM_, EM_, 4); else if (nt == 2) IG(AM_, EM_, 2); else IG(AM_, EM_, 1); } while (0)
    if (src.p2 && am != A_CONV3) return hipErrorInvalidValue;          // two-buffer sources: 3x3x3 only
    if (em == E_D2S) {
        // the staged epilogue writes 8 channels of one fine voxel as 16 bytes
        if (am != A_CONV1 || d2s_cout % 8 || dst.pitch % 8 || ((uintptr_t)dst.p & 15)) return hipErrorInvalidValue;
        IGN(A_CONV1, E_D2S);
    } else if (am == A_CONV3) {
        // LDS-tiled kernel: 16 x 4 x 4 output voxels per block, compiled per
        // padded channel count so that the K loop unrolls; 64 input channels
        // are staged 32 at a time, so the tile and its halo take 52 KB of LDS
        const int ty = 4, cs = std::min(cpad, 32);
        if (cpad != 2 && cpad != 8 && cpad != 16 && cpad != 32 && cpad != 64) return hipErrorInvalidValue;
        if (cpad == 2 && (pool || src.p2 || src.pitch < 2 || ((uintptr_t)src.p & 3))) return hipErrorInvalidValue;
        if (kpad < (27 * cpad + 31) / 32 * 32) return hipErrorInvalidValue;   // the K loop reads 32-wide steps
        const uint32_t tiles = (uint32_t)(((g.nx + 15) / 16) * ((g.ny + ty - 1) / ty) * ((g.nz + 3) / 4));
        const dim3 cgrid(tiles, (uint32_t)((n_cols + 16 * nt - 1) / (16 * nt)));
        // (two input channels: a 4-byte tile, the LDS sized for the staged output)
        const size_t lds = cpad == 2 ? (size_t)std::max(6 * (ty + 2) * 18 * 2, 4 * 16 * ty * (16 * nt + 8)) * sizeof(u16)
                                     : (size_t)6 * (ty + 2) * 18 * (cs + 8) * sizeof(u16);
        // 16-byte output stores (and mask loads) need 8-element alignment throughout
        const auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
        const int vec = n_cols % 8 == 0 && dst.pitch % 8 == 0 && al(dst.p) && (!mp || (mpitch % 8 == 0 && al(mp)));
        // the fused pool needs the staged epilogue, a grid divisible by 2 and one
        // thread per (coarse voxel, 8 channels) of the block: 32 coarse voxels x 2 nt
        if (pool && (!vec || pool->pitch % 8 || !al(pool->p) || g.nx % 2 || g.ny % 2 || g.nz % 2 || nt > 4 ||
                     16 * ty * (16 * nt + 8) * 4 > 6 * (ty + 2) * 18 * (cs + 8)))
            return hipErrorInvalidValue;
        u16 *pp = pool ? pool->p : nullptr;
        const int ppitch = pool ? pool->pitch : 0;
        // the fused head needs one 16-channel tile per block, 16 x 4 voxels per wave, the staged epilogue
        if (head && (nt != 1 || n_cols != 16 || !vec || pool || mp || !head->w || !head->in || !head->out))
            return hipErrorInvalidValue;
        const float *hw = head ? head->w : nullptr, *hin = head ? head->in : nullptr;
        float *hout = head ? head->out : nullptr;
        // a two-buffer source: its parts split at a whole 16-byte channel group
        if (src.p2 && (src.split % 8 || src.split <= 0 || src.split >= cpad || src.pitch2 % 8 ||
                       ((uintptr_t)src.p2 & 15)))
            return hipErrorInvalidValue;
        const u16 *s2 = src.p2 ? src.p2 : src.p;
        const int s2pitch = src.p2 ? src.pitch2 : src.pitch, split = src.p2 ? src.split : cpad;
#define CV(NT_, TY_, CP_, CS_) hipLaunchKernelGGL((conv3_kernel<NT_, TY_, CP_, CS_>), cgrid, dim3(256), lds, s, src.p, \
                                                  src.pitch, s2, s2pitch, split, g, wpk, kpad, n_cols, bias, (int)relu, \
                                                  mp, mpitch, dst.p, \
                                                  dst.pitch, vec, pp, ppitch, hw, hin, hout)
#define CVN(TY_, CP_, CS_) do { if (nt == 4) CV(4, TY_, CP_, CS_); else if (nt == 2) CV(2, TY_, CP_, CS_); \
                                else CV(1, TY_, CP_, CS_); } while (0)
        if (cpad == 2) CVN(4, 2, 2);
        else if (cpad == 8) CVN(4, 8, 8);
        else if (cpad == 16) CVN(4, 16, 16);
        else if (cpad == 32) CVN(4, 32, 32);
        else CVN(4, 64, 32);
#undef CVN
#undef CV
    } else if (am == A_S2D) {
        IGN(A_S2D, E_STORE);
    } else {
        IGN(A_CONV1, E_STORE);
    }
#undef IGN
#undef IG
    return hipGetLastError();
}

} // namespace

namespace {

hipError_t wgrad(int am, const View &P, int p_ch, const View &Q, int q_ch, const Grid &g, int n_off, fdc_unet *u,
                 bool transposed_layer, int ni, int nj, float *gw_out, hipStream_t s)
{
    const long rows = (long)g.nx * g.ny * g.nz;
    const int pc = pad16(p_ch), qc = pad16(q_ch);
    if (P.p2 || (Q.p2 && am != A_CONV3)) return hipErrorInvalidValue;      // two-buffer sources: 3x3x3 Q only
    long slabs = 1, per = rows;
    if (am != A_CONV3) {
        // slabs of at least 256 rows (8 rounds of 32), at most 1024 of them and
        // as many as the partials buffer holds: enough blocks to fill the chip
        const long cap = (long)(u->wpart_n / ((size_t)n_off * pc * qc));
        if (cap < 1) return hipErrorInvalidValue;
        slabs = std::min<long>({1024L, cap, std::max<long>(1, rows / 256)});
        per = (rows + slabs - 1) / slabs;
        per = (per + 31) & ~31L;
        slabs = (rows + per - 1) / per;
    } else {
        // Tile shape (16 x 4 x 4, 16 x 4 x 2 or 16 x 2 x 2 voxels), taps per block G
        // and Q channel tiles per block qs: the feasible choice (G qs groups of
        // pc/16 accumulator tiles over 4 waves, at most 14 tiles per wave for
        // 16 x 4 x 2 tiles, 12 otherwise; P tile and Q halo slice within 64 KB of LDS)
        // that stages the fewest elements per voxel of the layer,
        // (27 / G) (qc / 16 / qs) (TV pc + HV 16 qs) / TV; within 15% the choice
        // with fewer blocks per tile wins (more MFMA work per staged tile), and
        // exact ties go to the larger tile.
        if (pc != 16 && pc != 32 && pc != 64) return hipErrorInvalidValue;   // the kernel's PT = pc / 16
        const int shapes[3][2] = {{4, 4}, {4, 2}, {2, 2}};
        int ty = 0, tz = 0, G = 0, qs = 0, best_ny = 0;
        double best = 0.0;
        for (const auto &sh : shapes) {
            const int tv = 16 * sh[0] * sh[1], hv = 18 * (sh[0] + 2) * (sh[1] + 2);
            const int rmax = ((sh[0] == 4 && sh[1] == 2) ? 14 : 12) / (pc / 16);   // groups per wave
            for (int gg : {27, 9, 3})
                for (int q = qc / 16; q >= 1; q /= 2) {
                    if ((qc / 16) % q || (gg * q + 3) / 4 > rmax) continue;
                    if (((size_t)tv * (pc + 8) + (size_t)hv * (16 * q + 8)) * sizeof(u16) > 65536) continue;
                    const int nyb = (27 / gg) * (qc / 16 / q);
                    const double cost = (double)nyb * ((double)tv * pc + (double)hv * 16 * q) / tv;
                    if (!G || cost < 0.85 * best || (cost < 1.15 * best && nyb < best_ny)) {
                        best = cost; best_ny = nyb; ty = sh[0]; tz = sh[1]; G = gg; qs = q;
                    }
                }
        }
        if (!G) return hipErrorInvalidValue;
        const int ny_blocks = (27 / G) * (qc / (16 * qs));
        const long tiles = ((g.nx + 15) / 16) * (long)((g.ny + ty - 1) / ty) * ((g.nz + tz - 1) / tz);
        const long cap = (long)(u->wpart_n / ((size_t)27 * pc * qc));
        slabs = std::max<long>(1, std::min<long>({tiles, cap, std::max(1L, 2048L / ny_blocks)}));
        const size_t lds = ((size_t)16 * ty * tz * (pc + 8) + (size_t)18 * (ty + 2) * (tz + 2) * (16 * qs + 8)) * sizeof(u16);
        const dim3 grid((uint32_t)slabs, (uint32_t)ny_blocks);
        // a two-buffer Q: its parts split at a whole 16-byte channel group
        if (Q.p2 && (Q.split % 8 || Q.split <= 0 || Q.pitch2 % 8 || ((uintptr_t)Q.p2 & 15))) return hipErrorInvalidValue;
        const u16 *q2 = Q.p2 ? Q.p2 : Q.p;
        const int q2pitch = Q.p2 ? Q.pitch2 : Q.pitch, qsplit = Q.p2 ? Q.split : qc;
#define WTP(TY_, TZ_, PT_) hipLaunchKernelGGL((wgrad3t_kernel<TY_, TZ_, PT_>), grid, dim3(256), lds, s, P.p, P.pitch, \
                                              p_ch, Q.p, Q.pitch, q_ch, q2, q2pitch, qsplit, g, u->wpart, pc, qc, G, qs)
#define WT(TY_, TZ_) do { if (pc == 16) WTP(TY_, TZ_, 1); else if (pc == 32) WTP(TY_, TZ_, 2); else WTP(TY_, TZ_, 4); } while (0)
        if (ty == 4 && tz == 4) WT(4, 4); else if (ty == 4) WT(4, 2); else WT(2, 2);
#undef WT
#undef WTP
    }
    if (am != A_CONV3)
        hipLaunchKernelGGL((wgrad_kernel<A_S2D>), dim3(n_off, (uint32_t)slabs), dim3(256), 0, s, P.p, P.pitch, p_ch,
                           Q.p, Q.pitch, q_ch, g, per, u->wpart, pc, qc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long per_slab = (long)n_off * pc * qc;
    hipLaunchKernelGGL(slab_sum_kernel, dim3((uint32_t)((per_slab + 63) / 64)), dim3(512), 0, s, u->wpart, (int)slabs,
                       per_slab, pc, qc, ni, nj, gw_out);
    (void)transposed_layer;
    return hipGetLastError();
}

// queue the bias gradient of one layer (computed by bias_grad_all)
hipError_t add_bias_job(BiasJobs &bj, int &blocks, const View &G, int C, long n, float *gb)
{
    if (C % 8 || C > 64 || G.pitch % 8 || ((uintptr_t)G.p & 15) || bj.n >= kMaxBiasJobs) return hipErrorInvalidValue;
    // at most kMaxBiasBlocks blocks, each a whole number of rounds of its 256
    // threads over C/8 channel groups, at least one round
    const long per_step = 256 / (C / 8);
    long per = (n + kMaxBiasBlocks - 1) / kMaxBiasBlocks;
    per = std::max(per_step, (per + per_step - 1) / per_step * per_step);
    const int nb = (int)((n + per - 1) / per);
    bj.j[bj.n++] = BiasJob{G.p, gb, n, per, G.pitch, C, blocks, nb};
    blocks += nb;
    return hipSuccess;
}

hipError_t bias_grad_all(const BiasJobs &bj, int blocks, fdc_unet *u, hipStream_t s)
{
    if (!bj.n) return hipSuccess;
    hipLaunchKernelGGL(bias_part_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, bj, u->bpart);
    hipLaunchKernelGGL(bias_finish_kernel, dim3((uint32_t)bj.n), dim3(256), 0, s, bj, u->bpart);
    return hipGetLastError();
}

hipError_t pack_all(fdc_unet *u, hipStream_t s)
{
    PackJobs jobs{};
    int blocks = 0;
    auto add = [&](const float *w, u16 *wpk, int mode, int cin, int cout, int cpad, int n_cols, int kpad) {
        PackJob &J = jobs.j[jobs.n++];
        J = PackJob{w, wpk, mode, cin, cout, cpad, n_cols, kpad, blocks};
        blocks += (int)blocks_for((long)n_cols * kpad, 256, 1024);
    };
    for (int l = 0; l < kNumLayers; ++l) {
        const LayerDesc &L = kLayers[l];
        const float *w = u->params + u->w_off[l];
        if (L.kind == K_CONV3) {
            add(w, u->wpk_f[l], 0, L.cin, L.cout, fwd_cpad(L.cin), u->ncol_f[l], u->kpad_f[l]);
            if (u->wpk_b[l]) add(w, u->wpk_b[l], 1, L.cin, L.cout, pad8(L.cout), u->ncol_b[l], u->kpad_b[l]);
        } else if (L.kind == K_TCONV) {
            add(w, u->wpk_f[l], 2, L.cin, L.cout, pad8(L.cin), u->ncol_f[l], u->kpad_f[l]);
            add(w, u->wpk_b[l], 3, L.cin, L.cout, pad8(L.cout), u->ncol_b[l], u->kpad_b[l]);
        }
    }
    hipLaunchKernelGGL(pack_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

// views of the activation buffers (concatenations share one buffer)
struct Views {
    View x, e1a, u1, e1, c1, p1, e2a, u2, e2, c2, p2, ma, m, d2a, d2, d1a, d1;
    View gd1, gd1a, gc1, gu1, ge1s, gd2, gd2a, gc2, gu2, ge2s, gm, gma, gp2, ge2, ge2a, gp1, ge1, ge1a;
};

Views views(const fdc_unet *u)
{
    Views v;
    v.x = {u->x, 8, 2};
    v.e1a = {u->e1a, 16, 16};
    // decoder inputs: up-convolution output | skip, each half dense
    v.u1 = {u->c1, 16, 16};
    v.e1 = {u->c1 + u->nv[0] * 16, 16, 16};
    v.c1 = {v.u1.p, 16, 32, v.e1.p, 16, 16};
    v.p1 = {u->p1, 16, 16};
    v.e2a = {u->e2a, 32, 32};
    v.u2 = {u->c2, 32, 32};
    v.e2 = {u->c2 + u->nv[1] * 32, 32, 32};
    v.c2 = {v.u2.p, 32, 64, v.e2.p, 32, 32};
    v.p2 = {u->p2, 32, 32};
    v.ma = {u->ma, 64, 64};
    v.m = {u->m, 64, 64};
    v.d2a = {u->d2a, 32, 32};
    v.d2 = {u->d2, 32, 32};
    v.d1a = {u->d1a, 16, 16};
    v.d1 = {u->d1, 16, 16};
    v.gd1 = {u->gd1, 16, 16};
    v.gd1a = {u->gd1a, 16, 16};
    v.gc1 = {u->gc1, 32, 32};
    v.gu1 = {u->gc1, 32, 16};
    v.ge1s = {u->gc1 + 16, 32, 16};
    v.gd2 = {u->gd2, 32, 32};
    v.gd2a = {u->gd2a, 32, 32};
    v.gc2 = {u->gc2, 64, 64};
    v.gu2 = {u->gc2, 64, 32};
    v.ge2s = {u->gc2 + 32, 64, 32};
    v.gm = {u->gm, 64, 64};
    v.gma = {u->gma, 64, 64};
    v.gp2 = {u->gp2, 32, 32};
    v.ge2 = {u->ge2, 32, 32};
    v.ge2a = {u->ge2a, 32, 32};
    v.gp1 = {u->gp1, 16, 16};
    v.ge1 = {u->ge1, 16, 16};
    v.ge1a = {u->ge1a, 16, 16};
    return v;
}

hipError_t conv_fwd(fdc_unet *u, int l, const View &src, const Grid &g, const View &dst, hipStream_t s,
                    const View *pool = nullptr, const HeadFuse *head = nullptr)
{
    const LayerDesc &L = kLayers[l];
    return igemm(A_CONV3, E_STORE, src, fwd_cpad(L.cin), g, u->wpk_f[l], u->kpad_f[l], L.cout, u->params + u->b_off[l],
                 true, nullptr, dst, 0, s, pool, head);
}

// out: the network's output (inference: the head runs in dec1b's epilogue),
// or null (training: the head kernel follows with the loss and its gradient)
hipError_t forward_pass(fdc_unet *u, const float *in, hipStream_t s, float *out = nullptr)
{
    const Views v = views(u);
    const Grid *g = u->g;
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks_for(u->nv[0])), dim3(256), 0, s, in, u->nv[0], u->x2, 2);
    hipError_t e = hipGetLastError();
    if (!e) e = conv_fwd(u, L_E1A, View{u->x2, 2, 2}, g[0], v.e1a, s);
    if (!e) e = conv_fwd(u, L_E1B, v.e1a, g[0], v.e1, s, &v.p1);    // pool 1 fused into the epilogue
    if (!e) e = conv_fwd(u, L_E2A, v.p1, g[1], v.e2a, s);
    if (!e) e = conv_fwd(u, L_E2B, v.e2a, g[1], v.e2, s, &v.p2);    // pool 2 fused into the epilogue
    if (!e) e = conv_fwd(u, L_MA, v.p2, g[2], v.ma, s);
    if (!e) e = conv_fwd(u, L_MB, v.ma, g[2], v.m, s);
    if (!e) e = igemm(A_CONV1, E_D2S, v.m, 64, g[2], u->wpk_f[L_UP2], u->kpad_f[L_UP2], u->ncol_f[L_UP2],
                      u->params + u->b_off[L_UP2], false, nullptr, v.u2, 32, s);
    if (!e) e = conv_fwd(u, L_D2A, v.c2, g[1], v.d2a, s);
    if (!e) e = conv_fwd(u, L_D2B, v.d2a, g[1], v.d2, s);
    if (!e) e = igemm(A_CONV1, E_D2S, v.d2, 32, g[1], u->wpk_f[L_UP1], u->kpad_f[L_UP1], u->ncol_f[L_UP1],
                      u->params + u->b_off[L_UP1], false, nullptr, v.u1, 16, s);
    if (!e) e = conv_fwd(u, L_D1A, v.c1, g[0], v.d1a, s);
    if (out) {
        // the head reads bf16-rounded weights like every other layer (its bias stays FP32)
        hipLaunchKernelGGL(head_weights_kernel, dim3(1), dim3(64), 0, s, u->params + u->w_off[L_HEAD], u->hw);
        if (!e) e = hipGetLastError();
        const HeadFuse hf{u->hw, in, out};
        if (!e) e = conv_fwd(u, L_D1B, v.d1a, g[0], v.d1, s, nullptr, &hf);
    } else if (!e) {
        e = conv_fwd(u, L_D1B, v.d1a, g[0], v.d1, s);
    }
    return e;
}

// pool adjoint + skip gradient + ReLU mask on the fine grid g (16-byte accesses)
hipError_t pool_back(const View &gp, const View &skip, const View &e, int C, const Grid &g, const View &ge,
                     hipStream_t s)
{
    const auto al = [](const View &v) { return v.pitch % 8 == 0 && ((uintptr_t)v.p & 15) == 0; };
    if (C % 8 || !al(gp) || !al(skip) || !al(e) || !al(ge)) return hipErrorInvalidValue;
    const long n = (long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(pool_back_kernel, dim3(blocks_for(n * (C / 8))), dim3(256), 0, s, gp.p, gp.pitch, skip.p,
                       skip.pitch, e.p, e.pitch, C, g, ge.p, ge.pitch);
    return hipGetLastError();
}

hipError_t backward_pass(fdc_unet *u, const float *in, hipStream_t s)
{
    const Views v = views(u);
    const Grid *g = u->g;
    float *G = u->grads;
    auto gw = [&](int l) { return G + u->w_off[l]; };
    auto gb = [&](int l) { return G + u->b_off[l]; };
    auto bwd = [&](int l, const View &gout, const Grid &gr, const View *mask, const View &gin) {
        const LayerDesc &L = kLayers[l];
        return igemm(A_CONV3, E_STORE, gout, pad8(L.cout), gr, u->wpk_b[l], u->kpad_b[l], L.cin, nullptr, false, mask,
                     gin, 0, s);
    };
    // bias gradients are queued and computed together at the end (every output
    // gradient buffer is written once per backward pass)
    BiasJobs bj{};
    int bias_blocks = 0;
    auto wg3 = [&](int l, const View &gout, const View &in_v, const Grid &gr) {
        const LayerDesc &L = kLayers[l];
        hipError_t e = wgrad(A_CONV3, gout, L.cout, in_v, L.cin, gr, 27, u, false, L.cout, L.cin, gw(l), s);
        if (!e) e = add_bias_job(bj, bias_blocks, gout, L.cout, (long)gr.nx * gr.ny * gr.nz, gb(l));
        return e;
    };
    // the input padded to 8 channels, for the first layer's weight gradients
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks_for(u->nv[0])), dim3(256), 0, s, in, u->nv[0], u->x, 8);
    hipError_t e = hipGetLastError();
    // dec1b, dec1a
    if (!e) e = bwd(L_D1B, v.gd1, g[0], &v.d1a, v.gd1a);
    if (!e) e = wg3(L_D1B, v.gd1, v.d1a, g[0]);
    if (!e) e = bwd(L_D1A, v.gd1a, g[0], nullptr, v.gc1);
    if (!e) e = wg3(L_D1A, v.gd1a, v.c1, g[0]);
    // up1: transposed conv 32 -> 16 (coarse rows on g[1])
    if (!e) e = igemm(A_S2D, E_STORE, v.gu1, 16, g[1], u->wpk_b[L_UP1], u->kpad_b[L_UP1], 32, nullptr, false, &v.d2,
                      v.gd2, 0, s);
    if (!e) e = wgrad(A_S2D, v.d2, 32, v.gu1, 16, g[1], 8, u, true, 32, 16, gw(L_UP1), s);
    if (!e) e = add_bias_job(bj, bias_blocks, v.gu1, 16, u->nv[0], gb(L_UP1));
    // dec2b, dec2a
    if (!e) e = bwd(L_D2B, v.gd2, g[1], &v.d2a, v.gd2a);
    if (!e) e = wg3(L_D2B, v.gd2, v.d2a, g[1]);
    if (!e) e = bwd(L_D2A, v.gd2a, g[1], nullptr, v.gc2);
    if (!e) e = wg3(L_D2A, v.gd2a, v.c2, g[1]);
    // up2: transposed conv 64 -> 32 (coarse rows on g[2])
    if (!e) e = igemm(A_S2D, E_STORE, v.gu2, 32, g[2], u->wpk_b[L_UP2], u->kpad_b[L_UP2], 64, nullptr, false, &v.m,
                      v.gm, 0, s);
    if (!e) e = wgrad(A_S2D, v.m, 64, v.gu2, 32, g[2], 8, u, true, 64, 32, gw(L_UP2), s);
    if (!e) e = add_bias_job(bj, bias_blocks, v.gu2, 32, u->nv[1], gb(L_UP2));
    // mid
    if (!e) e = bwd(L_MB, v.gm, g[2], &v.ma, v.gma);
    if (!e) e = wg3(L_MB, v.gm, v.ma, g[2]);
    if (!e) e = bwd(L_MA, v.gma, g[2], nullptr, v.gp2);
    if (!e) e = wg3(L_MA, v.gma, v.p2, g[2]);
    // pool 2 adjoint + skip, enc2
    if (!e) {
        e = pool_back(v.gp2, v.ge2s, v.e2, 32, g[1], v.ge2, s);
    }
    if (!e) e = bwd(L_E2B, v.ge2, g[1], &v.e2a, v.ge2a);
    if (!e) e = wg3(L_E2B, v.ge2, v.e2a, g[1]);
    if (!e) e = bwd(L_E2A, v.ge2a, g[1], nullptr, v.gp1);
    if (!e) e = wg3(L_E2A, v.ge2a, v.p1, g[1]);
    // pool 1 adjoint + skip, enc1
    if (!e) {
        e = pool_back(v.gp1, v.ge1s, v.e1, 16, g[0], v.ge1, s);
    }
    if (!e) e = bwd(L_E1B, v.ge1, g[0], &v.e1a, v.ge1a);
    if (!e) e = wg3(L_E1B, v.ge1, v.e1a, g[0]);
    if (!e) e = wg3(L_E1A, v.ge1a, v.x, g[0]);
    if (!e) e = bias_grad_all(bj, bias_blocks, u, s);
    return e;
}

hipError_t head(fdc_unet *u, const float *in, const float *target, float *out, hipStream_t s)
{
    const long per = 8192;
    const int nb = (int)((u->nv[0] + per - 1) / per);
    // the head reads bf16-rounded weights like every other layer (its bias stays FP32)
    hipLaunchKernelGGL(head_weights_kernel, dim3(1), dim3(64), 0, s, u->params + u->w_off[L_HEAD], u->hw);
    hipLaunchKernelGGL(head_kernel, dim3(nb), dim3(256), 0, s, u->d1, 16, in, u->nv[0], u->hw, target, out, u->gd1,
                       u->lpart, u->hpart, per);
    hipError_t e = hipGetLastError();
    if (!e && target) {
        hipLaunchKernelGGL(head_finish_kernel, dim3(1), dim3(64), 0, s, u->lpart, u->hpart, nb, u->loss,
                           u->grads + u->w_off[L_HEAD]);
        e = hipGetLastError();
    }
    return e;
}

} // namespace

extern "C" {

int64_t fdc_unet_num_params(void) { return total_params(); }

const char *fdc_unet_last_error(const fdc_unet *u) { return u ? u->err.c_str() : "null"; }

int fdc_unet_destroy(fdc_unet *u)
{
    if (!u) return FDC_E_ARG;
    (void)hipSetDevice(u->device);
    (void)hipDeviceSynchronize();
    for (void *p : u->allocs) (void)hipFree(p);
    delete u;
    return FDC_OK;
}

int fdc_unet_create(fdc_unet **out, int hip_device, int nx, int ny, int nz)
{
    if (!out) return FDC_E_ARG;
    *out = nullptr;
    if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 4 || ny % 4 || nz % 4) return FDC_E_ARG;
    if ((long)nx * ny * nz >= (1L << 31)) return FDC_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        (void)hipGetLastError();
        return FDC_E_HIP;
    }
    fdc_unet *u = new (std::nothrow) fdc_unet();
    if (!u) return FDC_E_NOMEM;
    u->device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess) { delete u; return FDC_E_HIP; }
    for (int r = 0; r < 3; ++r) {
        u->g[r] = Grid{nx >> r, ny >> r, nz >> r};
        u->nv[r] = (long)u->g[r].nx * u->g[r].ny * u->g[r].nz;
    }
    long o = 0;
    for (int l = 0; l < kNumLayers; ++l) {
        u->w_off[l] = o;
        o += weight_count(kLayers[l]);
        u->b_off[l] = o;
        o += kLayers[l].cout;
    }
    u->n_params = o;
    bool ok = true;
    auto A16 = [&](long n) { u16 *p = ualloc<u16>(u, (size_t)n); ok = ok && p; return p; };
    u->params = ualloc<float>(u, o);
    u->grads = ualloc<float>(u, o);
    u->adam_m = ualloc<float>(u, o);
    u->adam_s = ualloc<float>(u, o);
    ok = u->params && u->grads && u->adam_m && u->adam_s;
    for (int l = 0; l < kNumLayers; ++l) {
        const LayerDesc &L = kLayers[l];
        if (L.kind == K_CONV3) {
            u->ncol_f[l] = L.cout; u->kpad_f[l] = pad32(27 * fwd_cpad(L.cin));
            u->ncol_b[l] = L.cin;  u->kpad_b[l] = pad32(27 * pad8(L.cout));
            u->wpk_f[l] = A16((long)u->ncol_f[l] * u->kpad_f[l]);
            if (l != L_E1A) u->wpk_b[l] = A16((long)u->ncol_b[l] * u->kpad_b[l]);
        } else if (L.kind == K_TCONV) {
            u->ncol_f[l] = 8 * L.cout; u->kpad_f[l] = pad32(pad8(L.cin));
            u->ncol_b[l] = L.cin;      u->kpad_b[l] = pad32(8 * pad8(L.cout));
            u->wpk_f[l] = A16((long)u->ncol_f[l] * u->kpad_f[l]);
            u->wpk_b[l] = A16((long)u->ncol_b[l] * u->kpad_b[l]);
        }
    }
    const long n0 = u->nv[0], n1 = u->nv[1], n2 = u->nv[2];
    u->x = A16(n0 * 8); u->x2 = A16(n0 * 2);
    u->e1a = A16(n0 * 16); u->c1 = A16(n0 * 32); u->p1 = A16(n1 * 16); u->e2a = A16(n1 * 32);
    u->c2 = A16(n1 * 64); u->p2 = A16(n2 * 32); u->ma = A16(n2 * 64); u->m = A16(n2 * 64); u->d2a = A16(n1 * 32);
    u->d2 = A16(n1 * 32); u->d1a = A16(n0 * 16); u->d1 = A16(n0 * 16);
    u->gd1 = A16(n0 * 16); u->gd1a = A16(n0 * 16); u->gc1 = A16(n0 * 32); u->gd2 = A16(n1 * 32);
    u->gd2a = A16(n1 * 32); u->gc2 = A16(n1 * 64); u->gm = A16(n2 * 64); u->gma = A16(n2 * 64);
    u->gp2 = A16(n2 * 32); u->ge2 = A16(n1 * 32); u->ge2a = A16(n1 * 32); u->gp1 = A16(n1 * 16);
    u->ge1 = A16(n0 * 16); u->ge1a = A16(n0 * 16);
    u->wpart_n = (size_t)64 * 27 * 64 * 64;
    u->wpart = ualloc<float>(u, u->wpart_n);
    u->bpart = ualloc<float>(u, (size_t)kMaxBiasJobs * kMaxBiasBlocks * 64);
    u->hpart = ualloc<float>(u, (size_t)((n0 + 8191) / 8192) * 17);
    u->lpart = ualloc<double>(u, (size_t)((n0 + 8191) / 8192));
    u->loss = ualloc<double>(u, 1);
    u->hw = ualloc<float>(u, 32);
    ok = ok && u->hw && u->wpart && u->bpart && u->hpart && u->lpart && u->loss;
    if (!ok) { fdc_unet_destroy(u); return FDC_E_NOMEM; }
    if (hipMemset(u->params, 0, o * 4) != hipSuccess || hipMemset(u->grads, 0, o * 4) != hipSuccess ||
        hipMemset(u->adam_m, 0, o * 4) != hipSuccess || hipMemset(u->adam_s, 0, o * 4) != hipSuccess) {
        fdc_unet_destroy(u);
        return FDC_E_HIP;
    }
    *out = u;
    return FDC_OK;
}

int fdc_unet_set_params(fdc_unet *u, const float *host, void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    if (!host) return ufail(u, FDC_E_ARG, "set_params: NULL");
    for (long i = 0; i < u->n_params; ++i)
        if (!std::isfinite(host[i])) return ufail(u, FDC_E_ARG, "set_params: non-finite value");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(u->device);
    if (!e) e = hipMemcpyAsync(u->params, host, u->n_params * 4, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemsetAsync(u->adam_m, 0, u->n_params * 4, s);
    if (!e) e = hipMemsetAsync(u->adam_s, 0, u->n_params * 4, s);
    if (!e) e = pack_all(u, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return ufail(u, FDC_E_HIP, "set_params", e);
    u->step = 0;
    return FDC_OK;
}

int fdc_unet_init_params(fdc_unet *u, uint64_t seed, void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    std::vector<float> v(u->n_params, 0.f);
    std::mt19937_64 gen(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < kNumLayers; ++l) {
        const LayerDesc &L = kLayers[l];
        const int taps = L.kind == K_CONV3 ? 27 : L.kind == K_TCONV ? 8 : 1;
        const double sd = std::sqrt(2.0 / (double)(L.cin * taps)) * (l == L_HEAD ? 0.1 : 1.0);
        for (long i = 0; i < weight_count(L); ++i) v[u->w_off[l] + i] = (float)(sd * nd(gen));
    }
    return fdc_unet_set_params(u, v.data(), hip_stream);
}

static int copy_out(fdc_unet *u, const float *src, float *host, void *hip_stream, const char *what)
{
    if (!u) return FDC_E_ARG;
    if (!host) return ufail(u, FDC_E_ARG, what);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(u->device);
    if (!e) e = hipMemcpyAsync(host, src, u->n_params * 4, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return ufail(u, FDC_E_HIP, what, e);
    return FDC_OK;
}

int fdc_unet_get_params(fdc_unet *u, float *host, void *s) { return copy_out(u, u ? u->params : nullptr, host, s, "get_params"); }
int fdc_unet_get_grads(fdc_unet *u, float *host, void *s) { return copy_out(u, u ? u->grads : nullptr, host, s, "get_grads"); }

int fdc_unet_forward(fdc_unet *u, const float *in_dev, float *out_dev, void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    if (!in_dev || !out_dev) return ufail(u, FDC_E_ARG, "forward: NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(u->device);
    if (!e) e = forward_pass(u, in_dev, s, out_dev);
    if (e) return ufail(u, FDC_E_HIP, "forward", e);
    return FDC_OK;
}

int fdc_unet_backward(fdc_unet *u, const float *in_dev, const float *target_dev, float *out_dev, double *loss_host,
                      void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    if (!in_dev || !target_dev) return ufail(u, FDC_E_ARG, "backward: NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(u->device);
    if (!e) e = forward_pass(u, in_dev, s);
    if (!e) e = head(u, in_dev, target_dev, out_dev, s);
    if (!e) e = backward_pass(u, in_dev, s);
    if (!e && loss_host) e = hipMemcpyAsync(loss_host, u->loss, 8, hipMemcpyDeviceToHost, s);
    if (!e && loss_host) e = hipStreamSynchronize(s);
    if (e) return ufail(u, FDC_E_HIP, "backward", e);
    return FDC_OK;
}

int fdc_unet_debug_buffer(fdc_unet *u, int index, uint16_t *host_out, int64_t *n_voxels, int32_t *pitch,
                          void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    u16 *const bufs[] = {u->x, u->e1a, u->c1, u->p1, u->e2a, u->c2, u->p2, u->ma, u->m, u->d2a, u->d2, u->d1a, u->d1,
                         u->gd1, u->gd1a, u->gc1, u->gd2, u->gd2a, u->gc2, u->gm, u->gma, u->gp2, u->ge2, u->ge2a,
                         u->gp1, u->ge1, u->ge1a};
    const int lvl[] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 0, 0, 0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 1, 0, 0};
    const int pit[] = {8, 16, 32, 16, 32, 64, 32, 64, 64, 32, 32, 16, 16, 16, 16, 32, 32, 32, 64, 64, 64, 32, 32, 32,
                       16, 16, 16};
    if (index < 0 || index >= (int)(sizeof(lvl) / sizeof(int))) return ufail(u, FDC_E_ARG, "debug_buffer: index");
    const long n = u->nv[lvl[index]];
    if (n_voxels) *n_voxels = n;
    if (pitch) *pitch = pit[index];
    if (!host_out) return FDC_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(u->device);
    if (index == 0 || index == 2 || index == 5) {
        // the input as the forward pass read it (two channels, returned in rows
        // of 8), or a concatenation held as two dense halves (returned
        // interleaved): contiguous copies, rearranged here
        const size_t h = index == 0 ? 2 : (size_t)pit[index] / 2, parts = index == 0 ? 1 : 2;
        std::vector<u16> tmp;
        try {
            tmp.resize((size_t)n * h * parts);
        } catch (const std::bad_alloc &) {
            return ufail(u, FDC_E_NOMEM, "debug_buffer: host staging");
        }
        const u16 *src = index == 0 ? u->x2 : bufs[index];
        if (!e) e = hipMemcpyAsync(tmp.data(), src, tmp.size() * 2, hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (!e) {
            u16 *o = (u16 *)host_out;
            const size_t P = (size_t)pit[index];
            std::memset(o, 0, (size_t)n * P * 2);
            for (size_t part = 0; part < parts; ++part)
                for (size_t v = 0; v < (size_t)n; ++v)
                    std::memcpy(o + v * P + part * h, tmp.data() + (part * (size_t)n + v) * h, h * 2);
        }
    } else if (!e) {
        e = hipMemcpyAsync(host_out, bufs[index], (size_t)n * pit[index] * 2, hipMemcpyDeviceToHost, s);
    }
    if (!e) e = hipStreamSynchronize(s);
    if (e) return ufail(u, FDC_E_HIP, "debug_buffer", e);
    return FDC_OK;
}

int fdc_unet_adam(fdc_unet *u, float lr, float beta1, float beta2, float eps, void *hip_stream)
{
    if (!u) return FDC_E_ARG;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return ufail(u, FDC_E_ARG, "adam: bad hyper-parameters");
    hipStream_t s = (hipStream_t)hip_stream;
    u->step++;
    const float c1 = 1.f - std::pow(beta1, (float)u->step), c2 = 1.f - std::pow(beta2, (float)u->step);
    hipError_t e = hipSetDevice(u->device);
    if (!e) {
        hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(u->n_params)), dim3(256), 0, s, u->params, u->grads, u->adam_m,
                           u->adam_s, u->n_params, lr, beta1, beta2, eps, c1, c2);
        e = hipGetLastError();
    }
    if (!e) e = pack_all(u, s);
    if (e) return ufail(u, FDC_E_HIP, "adam", e);
    return FDC_OK;
}

} // extern "C"
