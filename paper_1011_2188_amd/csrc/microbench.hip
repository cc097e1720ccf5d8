// Microbenchmarks of the ceilings that bound the transport kernel:
//   copy       - HBM stream copy (also the reference for HBM byte counters)
//   atom_rand  - 64-bit global atomic adds at pseudo-random addresses of a
//                tally-sized array (distinct addresses, like scattered flushes)
//   atom_coal  - 64-bit global atomic adds, lane i -> consecutive addresses
//   atom_wave  - 64-bit global atomic adds, every lane of a wave on one address
//   atom_hot   - 64-bit global atomic adds at random addresses among 4096
//   lds_atom   - 64-bit LDS atomic adds at random slots of a 4096-entry table
// Prints one JSON line per test.  Usage: fdc_microbench [tally_MB ...]
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHK(x)                                                                     \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            exit(1);                                                               \
        }                                                                          \
    } while (0)

__device__ inline uint32_t mix(uint32_t x)
{
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    return x;
}

__global__ void copy_kernel(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void atom_rand(unsigned long long *t, uint32_t n, int k)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < k; ++j) atomicAdd(t + mix(g * 977u + j) % n, 1ull);
}

__global__ void atom_coal(unsigned long long *t, uint32_t n, int k)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < k; ++j) atomicAdd(t + ((uint64_t)g + (uint64_t)j * gridDim.x * blockDim.x) % n, 1ull);
}

__global__ void atom_wave(unsigned long long *t, uint32_t n, int k)
{
    const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    for (int j = 0; j < k; ++j) atomicAdd(t + mix(w * 131u + j) % n, 1ull);
}

__global__ void atom_hot(unsigned long long *t, uint32_t, int k)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < k; ++j) atomicAdd(t + (mix(g * 977u + j) & 4095u), 1ull);
}

__global__ void lds_atom(unsigned long long *out, uint32_t, int k)
{
    __shared__ unsigned long long s[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s[i] = 0;
    __syncthreads();
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < k; ++j) atomicAdd(s + (mix(g * 977u + j) & 4095u), 1ull);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, s[g & 4095u]);
}

typedef void (*akernel)(unsigned long long *, uint32_t, int);

static float time_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

int main(int argc, char **argv)
{
    std::vector<double> sizes_mb;
    for (int i = 1; i < argc; ++i) sizes_mb.push_back(atof(argv[i]));
    if (sizes_mb.empty()) sizes_mb = {2.1, 16.8, 67.1};
    hipDeviceProp_t prop;
    CHK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));

    // HBM copy: 2 GiB read + 2 GiB written
    {
        const size_t n = (size_t(2) << 30) / sizeof(float4);
        float4 *a, *b;
        CHK(hipMalloc(&a, n * sizeof(float4)));
        CHK(hipMalloc(&b, n * sizeof(float4)));
        CHK(hipMemset(a, 1, n * sizeof(float4)));
        const int grid = cus * 32;
        hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, 0, a, b, n);
        CHK(hipDeviceSynchronize());
        float best = 1e30f;
        for (int r = 0; r < 5; ++r) {
            CHK(hipEventRecord(e0));
            hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, 0, a, b, n);
            CHK(hipEventRecord(e1));
            CHK(hipEventSynchronize(e1));
            best = fminf(best, time_ms(e0, e1));
        }
        printf("{\"test\": \"copy\", \"bytes_read\": %zu, \"bytes_written\": %zu, \"ms\": %.4f, \"GBps\": %.1f}\n",
               n * sizeof(float4), n * sizeof(float4), best, 2.0 * n * sizeof(float4) / (best * 1e-3) / 1e9);
        CHK(hipFree(a));
        CHK(hipFree(b));
    }

    const struct { const char *name; akernel k; } tests[] = {
        {"atom_rand", atom_rand}, {"atom_coal", atom_coal}, {"atom_wave", atom_wave},
        {"atom_hot", atom_hot}, {"lds_atom", lds_atom}};
    for (double mb : sizes_mb) {
        const uint32_t n = (uint32_t)(mb * 1e6 / 8.0);
        unsigned long long *t;
        CHK(hipMalloc(&t, (size_t)n * 8));
        CHK(hipMemset(t, 0, (size_t)n * 8));
        for (const auto &T : tests) {
            const int k = 64;
            const int grid = cus * 64;
            const int block = 256;
            hipLaunchKernelGGL(T.k, dim3(grid), dim3(block), 0, 0, t, n, 4);
            CHK(hipDeviceSynchronize());
            float best = 1e30f;
            for (int r = 0; r < 3; ++r) {
                CHK(hipEventRecord(e0));
                hipLaunchKernelGGL(T.k, dim3(grid), dim3(block), 0, 0, t, n, k);
                CHK(hipEventRecord(e1));
                CHK(hipEventSynchronize(e1));
                best = fminf(best, time_ms(e0, e1));
            }
            const double ops = (double)grid * block * k;
            printf("{\"test\": \"%s\", \"tally_MB\": %.1f, \"atomics\": %.0f, \"ms\": %.4f, \"atomics_per_s\": %.4g}\n",
                   T.name, mb, ops, best, ops / (best * 1e-3));
            fflush(stdout);
        }
        CHK(hipFree(t));
    }
    return 0;
}
