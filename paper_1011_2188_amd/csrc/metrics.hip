// Dose-distribution metrics (Section 2.4): the mean dose uncertainty (mean of
// sigma_D / D over voxels above half the maximum dose), the batch uncertainty
// of Eq. (1), and the gamma index (Low et al. 1998) with a global dose
// criterion.  Reductions run in a fixed order so results are reproducible.
#include "fdc_device.h"

namespace fdc {

namespace {

constexpr int kRedBlocks = 1024;   // fixed grid of the fixed-order reductions
constexpr int kRedThreads = 256;

__device__ inline bool is_vacuum(const uint16_t *idx, const float2 *lut, size_t v)
{
    return lut[hu_index(idx[v])].x == 0.f;
}

// per-block maximum of non-vacuum doses (doses are >= 0, so the max of their
// bit patterns as unsigned integers is the max of the values)
__global__ void dmax_partial_kernel(const double *__restrict__ d, const uint16_t *__restrict__ idx,
                                    const float2 *__restrict__ lut, size_t n, double *__restrict__ part)
{
    __shared__ double s[kRedThreads];
    double m = 0.0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        if (!is_vacuum(idx, lut, v)) m = fmax(m, d[v]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// per-block sum of sigma/D and count over non-vacuum voxels with D > thr,
// where thr = frac * max(part_max[*]) is recomputed by every block
__global__ void unc_partial_kernel(const double *__restrict__ d, const double *__restrict__ var,
                                   const uint16_t *__restrict__ idx, const float2 *__restrict__ lut, size_t n,
                                   const double *__restrict__ part_max, int n_part, double frac,
                                   double *__restrict__ part_sum, unsigned long long *__restrict__ part_cnt)
{
    __shared__ double s[kRedThreads];
    __shared__ unsigned long long c[kRedThreads];
    __shared__ double s_thr;
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < n_part; ++i) m = fmax(m, part_max[i]);
        s_thr = frac * m;
    }
    __syncthreads();
    const double thr = s_thr;
    double acc = 0.0;
    unsigned long long cnt = 0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const double dv = d[v];
        if (dv > thr && !is_vacuum(idx, lut, v)) {
            acc += sqrt(fmax(var[v], 0.0)) / dv;
            ++cnt;
        }
    }
    s[threadIdx.x] = acc;
    c[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[threadIdx.x] += s[threadIdx.x + w];
            c[threadIdx.x] += c[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_sum[blockIdx.x] = s[0];
        part_cnt[blockIdx.x] = c[0];
    }
}

// final fixed-order sums: out[0] = max, out[1] = sum, out[2] = count (as double)
__global__ void finish_kernel(const double *__restrict__ part_max, const double *__restrict__ part_sum,
                              const unsigned long long *__restrict__ part_cnt, int n_part, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = 0.0, sum = 0.0;
    unsigned long long cnt = 0;
    for (int i = 0; i < n_part; ++i) {
        m = fmax(m, part_max[i]);
        if (part_sum) sum += part_sum[i];
        if (part_cnt) cnt += part_cnt[i];
    }
    out[0] = m;
    out[1] = sum;
    out[2] = (double)cnt;
}

// Eq. (1): per voxel, mean over n batches and sqrt(sum (D_i - mean)^2 / (n (n-1)))
__global__ void batch_kernel(const double *__restrict__ doses, uint32_t nb, size_t n, double *__restrict__ mean,
                             double *__restrict__ sigma)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        double m = 0.0;
        for (uint32_t i = 0; i < nb; ++i) m += doses[i * n + v];
        m /= nb;
        double s = 0.0;
        for (uint32_t i = 0; i < nb; ++i) {
            const double x = doses[i * n + v] - m;
            s += x * x;
        }
        if (mean) mean[v] = m;
        if (sigma) sigma[v] = sqrt(s / ((double)nb * (nb - 1)));
    }
}

// Gamma index of each reference voxel against the evaluated dose upsampled
// twice per axis by trilinear interpolation (points at half-voxel spacing).
// offs: candidate offsets in half-voxel units with their squared distance /
// DTA^2, sorted by that distance term, so the search stops once the distance
// term alone reaches the best gamma^2 found.  gamma = -1 for voxels not
// evaluated (vacuum or reference dose below the cutoff).
__global__ void gamma_kernel(const double *__restrict__ ref, const double *__restrict__ ev,
                             const uint16_t *__restrict__ idx, const float2 *__restrict__ lut, int nx, int ny,
                             int nz, const int4 *__restrict__ offs, const double *__restrict__ offd2, int n_offs,
                             const double *__restrict__ dmax_out, double dose_frac, double cutoff_frac,
                             float *__restrict__ gamma, unsigned long long *__restrict__ counts)
{
    const size_t n = (size_t)nx * ny * nz;
    const double dmax = dmax_out[0];
    const double dd = dose_frac * dmax;
    const double inv_dd2 = 1.0 / (dd * dd);
    unsigned long long n_eval = 0, n_pass = 0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const double dr = ref[v];
        if (is_vacuum(idx, lut, v) || !(dr >= cutoff_frac * dmax)) {
            if (gamma) gamma[v] = -1.f;
            continue;
        }
        const int ix = (int)(v % nx), iy = (int)((v / nx) % ny), iz = (int)(v / ((size_t)nx * ny));
        const int hx = 2 * ix, hy = 2 * iy, hz = 2 * iz;
        double best = __builtin_huge_val();
        for (int k = 0; k < n_offs; ++k) {
            const double d2 = offd2[k];
            if (d2 >= best) break;
            const int4 o = offs[k];
            const int px = hx + o.x, py = hy + o.y, pz = hz + o.z;
            if (px < 0 || py < 0 || pz < 0 || px > 2 * (nx - 1) || py > 2 * (ny - 1) || pz > 2 * (nz - 1)) continue;
            const int x0 = px >> 1, y0 = py >> 1, z0 = pz >> 1;
            const int x1 = x0 + (px & 1), y1 = y0 + (py & 1), z1 = z0 + (pz & 1);
            const size_t r00 = ((size_t)z0 * ny + y0) * nx, r01 = ((size_t)z0 * ny + y1) * nx;
            const size_t r10 = ((size_t)z1 * ny + y0) * nx, r11 = ((size_t)z1 * ny + y1) * nx;
            const double e = 0.125 * (ev[r00 + x0] + ev[r00 + x1] + ev[r01 + x0] + ev[r01 + x1] +
                                      ev[r10 + x0] + ev[r10 + x1] + ev[r11 + x0] + ev[r11 + x1]);
            const double diff = e - dr;
            const double g2 = d2 + diff * diff * inv_dd2;
            best = fmin(best, g2);
        }
        const double g = sqrt(best);
        if (gamma) gamma[v] = (float)g;
        ++n_eval;
        n_pass += g <= 1.0;
    }
    atomicAdd(counts + 0, n_eval);
    atomicAdd(counts + 1, n_pass);
}

} // namespace

hipError_t launch_dmax(const double *d, const uint16_t *idx, const float2 *lut, size_t n, double *part,
                       double *out3, hipStream_t s)
{
    hipLaunchKernelGGL(dmax_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, d, idx, lut, n, part);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, part, (const double *)nullptr,
                       (const unsigned long long *)nullptr, kRedBlocks, out3);
    return hipGetLastError();
}

hipError_t launch_mean_uncertainty(const double *d, const double *var, const uint16_t *idx, const float2 *lut,
                                   size_t n, double frac, double *scratch, double *out3, hipStream_t s)
{
    double *part_max = scratch, *part_sum = scratch + kRedBlocks;
    unsigned long long *part_cnt = (unsigned long long *)(scratch + 2 * kRedBlocks);
    hipLaunchKernelGGL(dmax_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, d, idx, lut, n, part_max);
    hipLaunchKernelGGL(unc_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, d, var, idx, lut, n, part_max,
                       kRedBlocks, frac, part_sum, part_cnt);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, part_max, part_sum, part_cnt, kRedBlocks, out3);
    return hipGetLastError();
}

size_t metrics_scratch_doubles() { return 3 * kRedBlocks + 8; }

hipError_t launch_batch_uncertainty(const double *doses, uint32_t nb, size_t n, double *mean, double *sigma,
                                    hipStream_t s)
{
    const size_t g = std::min<size_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(batch_kernel, dim3((uint32_t)std::max<size_t>(g, 1)), dim3(256), 0, s, doses, nb, n, mean,
                       sigma);
    return hipGetLastError();
}

hipError_t launch_gamma(const double *ref, const double *ev, const uint16_t *idx, const float2 *lut, int nx, int ny,
                        int nz, const int4 *offs, const double *offd2, int n_offs, const double *dmax_out,
                        double dose_frac, double cutoff_frac, float *gamma, unsigned long long *counts,
                        hipStream_t s)
{
    const size_t n = (size_t)nx * ny * nz;
    const size_t g = std::min<size_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(gamma_kernel, dim3((uint32_t)std::max<size_t>(g, 1)), dim3(256), 0, s, ref, ev, idx, lut,
                       nx, ny, nz, offs, offd2, n_offs, dmax_out, dose_frac, cutoff_frac, gamma, counts);
    return hipGetLastError();
}

} // namespace fdc
