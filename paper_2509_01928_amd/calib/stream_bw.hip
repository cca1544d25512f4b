// stream_bw.hip -- HBM streaming ceilings of the device, used to calibrate
// the bandwidth figures of the DOCH kernels:
//   copy   : b[i] = a[i]        (16-byte loads and stores)
//   read   : per-workgroup sums of a (16-byte loads, one store per workgroup)
//   write  : b[i] = constant    (16-byte stores)
// Usage: stream_bw [MiB per buffer = 2048] [repetitions = 20]
// Prints one line per kernel with the best and mean GB/s (10^9 bytes/s).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));    \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy_kernel(const f4* __restrict__ a, f4* __restrict__ b,
                                                   long n4) {
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n4;
         i += static_cast<long>(gridDim.x) * 256)
        b[i] = __builtin_nontemporal_load(a + i);
}

__global__ __launch_bounds__(256) void read_kernel(const f4* __restrict__ a, float* __restrict__ out,
                                                   long n4) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n4;
         i += static_cast<long>(gridDim.x) * 256)
        acc += __builtin_nontemporal_load(a + i);
    __shared__ float red[256];
    red[threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void write_kernel(f4* __restrict__ b, long n4, float v) {
    const f4 val = {v, v, v, v};
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n4;
         i += static_cast<long>(gridDim.x) * 256)
        b[i] = val;
}

int main(int argc, char** argv) {
    const long mib = argc > 1 ? std::atol(argv[1]) : 2048;
    const int reps = argc > 2 ? std::atoi(argv[2]) : 20;
    const long bytes = mib * 1024L * 1024L;
    const long n4 = bytes / 16;
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    f4 *a = nullptr, *b = nullptr;
    float* out = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    const int grid = cus * 8;
    CHECK(hipMalloc(&out, grid * sizeof(float)));
    hipLaunchKernelGGL(write_kernel, dim3(grid), dim3(256), 0, 0, a, n4, 1.0f);
    hipLaunchKernelGGL(write_kernel, dim3(grid), dim3(256), 0, 0, b, n4, 0.0f);
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char* names[3] = {"copy", "read", "write"};
    const double moved[3] = {2.0 * bytes, 1.0 * bytes, 1.0 * bytes};
    for (int k = 0; k < 3; ++k) {
        double best = 0.0, sum = 0.0;
        for (int r = 0; r < reps + 2; ++r) {
            CHECK(hipEventRecord(e0, 0));
            if (k == 0) hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, 0, a, b, n4);
            if (k == 1) hipLaunchKernelGGL(read_kernel, dim3(grid), dim3(256), 0, 0, a, out, n4);
            if (k == 2) hipLaunchKernelGGL(write_kernel, dim3(grid), dim3(256), 0, 0, b, n4, 2.0f);
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (r < 2) continue;      // warm-up
            const double gbs = moved[k] / (ms * 1e-3) / 1e9;
            sum += gbs;
            if (gbs > best) best = gbs;
        }
        std::printf("%-5s %6ld MiB  best %8.1f GB/s  mean %8.1f GB/s  (grid %d x 256)\n", names[k],
                    mib, best, sum / reps, grid);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(out));
    return 0;
}
