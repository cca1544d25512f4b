// lattice_mix_bw -- what the lattice DOCH step's access pattern can stream.
//
// Per row i the step reads a 16-byte chunk of column indices and one of
// values, the row offset, the iterate and the field (4 bytes each) and
// writes the new iterate (4 bytes): 48 bytes per row, 92% of them reads.
// This program streams exactly that mix over 10^8 rows with no arithmetic to
// speak of, in four access orders:
//   plain         the whole grid sweeps the rows together
//   partitioned   XCD c (workgroups w with w mod 8 = c) owns the c-th eighth
//   gathers       plain, plus the four lattice neighbours x[i+-1], x[i+-L]
//   part+gathers  both
// at 2, 3, 4 and 8 resident workgroups per CU, and prints GB/s of the 48
// algorithmic bytes per row.  Usage: lattice_mix_bw [rows] [L]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef float f4 __attribute__((ext_vector_type(4)));

#define CK(x)                                                                 \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            std::printf("%s: %s\n", #x, hipGetErrorString(e_));              \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

template <bool PART, bool GATH>
__global__ __launch_bounds__(256) void mix_kernel(const f4* __restrict__ c, const f4* __restrict__ v,
                                                  const float* __restrict__ r, const float* __restrict__ x,
                                                  const float* __restrict__ h, float* __restrict__ out,
                                                  long n, long L) {
    long hi = n, first = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    long stride = static_cast<long>(gridDim.x) * 256;
    if (PART) {
        const unsigned xcd = blockIdx.x & 7u, slot = blockIdx.x >> 3;
        const long lo = n * xcd / 8;
        hi = n * (xcd + 1) / 8;
        first = lo + static_cast<long>(slot) * 256 + threadIdx.x;
        stride = static_cast<long>(gridDim.x >> 3) * 256;
    }
    for (long i = first; i < hi; i += stride) {
        const f4 a = __builtin_nontemporal_load(c + i), b = __builtin_nontemporal_load(v + i);
        const float p = __builtin_nontemporal_load(r + i), q = x[i], s = __builtin_nontemporal_load(h + i);
        float z = a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w + p + q + s;
        if (GATH) {
            const long im = i == 0 ? n - 1 : i - 1, ip = i + 1 == n ? 0 : i + 1;
            const long iu = i >= L ? i - L : i - L + n, id = i + L < n ? i + L : i + L - n;
            z += x[im] + x[ip] + x[iu] + x[id];
        }
        __builtin_nontemporal_store(z, out + i);
    }
}

int main(int argc, char** argv) {
    const long n = argc > 1 ? std::atol(argv[1]) : 100000000L;
    const long L = argc > 2 ? std::atol(argv[2]) : 10000L;
    if (n < 1 || L < 1 || L >= n) {
        std::printf("need 1 <= L < rows\n");
        return 1;
    }
    f4 *c, *v;
    float *r, *x, *h, *o;
    CK(hipMalloc(&c, n * 16));
    CK(hipMalloc(&v, n * 16));
    CK(hipMalloc(&r, n * 4));
    CK(hipMalloc(&x, n * 4));
    CK(hipMalloc(&h, n * 4));
    CK(hipMalloc(&o, n * 4));
    CK(hipMemset(c, 0, n * 16));
    CK(hipMemset(v, 0, n * 16));
    CK(hipMemset(r, 0, n * 4));
    CK(hipMemset(x, 0, n * 4));
    CK(hipMemset(h, 0, n * 4));
    int cus = 0;
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const double bytes = n * 48.0;
    auto timed = [&](const char* name, int g, auto launch) {
        for (int w = 0; w < 2; ++w) launch();
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0));
        for (int k = 0; k < 10; ++k) launch();
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        ms /= 10;
        std::printf("%-13s grid %5d %8.1f us %8.1f GB/s\n", name, g, ms * 1e3, bytes / (ms * 1e-3) / 1e9);
        std::fflush(stdout);
    };
    for (int occ : {2, 3, 4, 8}) {
        const int g = cus * occ;
        timed("plain", g, [&] {
            hipLaunchKernelGGL((mix_kernel<false, false>), dim3(g), dim3(256), 0, 0, c, v, r, x, h, o, n, L);
        });
        timed("partitioned", g, [&] {
            hipLaunchKernelGGL((mix_kernel<true, false>), dim3(g), dim3(256), 0, 0, c, v, r, x, h, o, n, L);
        });
        timed("gathers", g, [&] {
            hipLaunchKernelGGL((mix_kernel<false, true>), dim3(g), dim3(256), 0, 0, c, v, r, x, h, o, n, L);
        });
        timed("part+gathers", g, [&] {
            hipLaunchKernelGGL((mix_kernel<true, true>), dim3(g), dim3(256), 0, 0, c, v, r, x, h, o, n, L);
        });
    }
    CK(hipGetLastError());
    return 0;
}
