// device_common.h -- device helpers shared by the gfx950 kernels:
// deterministic wavefront/workgroup reductions, the coherent last-workgroup
// hand-off, IEEE-exact scalar arithmetic and streaming loads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace doch {

constexpr int kWave = 64;

// Native 16/32-byte vectors for wide streaming loads.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef signed char i8x4 __attribute__((ext_vector_type(4)));
template <> struct Vec4<int> { using type = i32x4; };
template <> struct Vec4<int8_t> { using type = i8x4; };
template <> struct Vec4<int16_t> { using type = i16x4; };
template <> struct Vec4<float> { using type = f32x4; };
template <> struct Vec4<double> { using type = f64x4; };

// Four consecutive elements starting at a 4-element-aligned index, streamed
// past the caches.
template <typename T>
__device__ __forceinline__ typename Vec4<T>::type ld_stream4(const T* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename Vec4<T>::type*>(p));
}

// Round-to-nearest double operations that the compiler may not contract into
// FMAs, so the update matches its defining expression operation by operation.
__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ double dsub(double a, double b) { return __dsub_rn(a, b); }
__device__ __forceinline__ double ddiv(double a, double b) { return __ddiv_rn(a, b); }

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ double to_d(T v) { return static_cast<double>(v); }

template <typename XT>
__device__ __forceinline__ void store_x(XT* p, double v) { *p = static_cast<XT>(v); }

// Butterfly sum over the 64 lanes of a wavefront.  Lane 0 always performs the
// same sequence of additions, so its result is reproducible run to run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = dadd(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Sum K values over a workgroup of NT threads in a fixed order; the result
// is valid in thread 0.  `lds` must hold K * (NT / 64) doubles.
template <int K, int NT>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) lds[q * NW + wave] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s = dadd(s, lds[q * NW + w]);
            v[q] = s;
        }
    }
    __syncthreads();
}

// Coherent (agent-scope) accesses used for the partial sums that cross
// workgroups -- and therefore XCDs and their private L2 caches.
__device__ __forceinline__ void store_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Handing partial results to the last workgroup of a launch.  The arriving
// wave has stored its workgroup's partials with store_agent, which writes
// through to the device's point of coherence; it waits until those stores
// have completed, then counts itself in with a relaxed atomic.  The arrival
// that completes the count reads every partial with load_agent, which reads
// at the point of coherence.  No L2 write-back or invalidate is involved, so
// a workgroup pays one store round trip and one atomic.
__device__ __forceinline__ void wait_stores_complete() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

__device__ __forceinline__ bool arrive_last(unsigned int* ticket, unsigned int count) {
    wait_stores_complete();
    const unsigned int prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return prev == count - 1;
}

// The same for a 1-D grid of any size, counted in two levels so that no
// single counter takes more than about grid/8 arrivals: workgroup w counts in
// group w mod 8 (one group per XCD under round-robin dispatch), the last of
// each group counts at the top.  tickets[0] is the top, group g's counter is
// tickets[kTicketStride * (1 + g)]; all nine start at zero and are zero again
// when the launch is over.
constexpr int kTicketStride = 32;                 // one counter per 128-byte line
constexpr int kGridTickets = 9 * kTicketStride;   // counters a grouped ticket spans

__device__ __forceinline__ bool arrive_last_grid(unsigned int* tickets, unsigned int grid) {
    const unsigned int g = blockIdx.x & 7u;
    const unsigned int per = (grid - g + 7u) / 8u;   // workgroups in group g (g < grid here)
    const unsigned int groups = grid < 8u ? grid : 8u;
    wait_stores_complete();
    unsigned int* gt = tickets + kTicketStride * (1 + g);
    if (__hip_atomic_fetch_add(gt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != per - 1) return false;
    __hip_atomic_store(gt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_fetch_add(tickets, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1;
}

__device__ __forceinline__ void reset_ticket(unsigned int* ticket) {
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last workgroup of a column block (64 restarts): reduce the K per-row-tile
// partials of each restart in row-tile order.  Thread (q, c) owns quantity q
// of restart c; its loads are issued B at a time so the latency (these loads
// read at the device's point of coherence) is paid once per batch of B row
// tiles.
template <int K, int B = 32>
__device__ __forceinline__ double column_partial_sum(const double* __restrict__ partials, int Rp,
                                                     int c, int q, int tiles) {
    double s = 0.0;
    for (int t0 = 0; t0 < tiles; t0 += B) {
        double v[B];
#pragma unroll
        for (int b = 0; b < B; ++b)
            v[b] = t0 + b < tiles ? load_agent(partials + (static_cast<size_t>(t0 + b) * Rp + c) * K + q) : 0.0;
#pragma unroll
        for (int b = 0; b < B; ++b) s = dadd(s, v[b]);
    }
    return s;
}

}  // namespace doch
