// Device-wide exclusive scans (reduce -> scan partials -> downsweep).
#include "svr_internal.h"

namespace svr {
namespace {

constexpr int kThreads = 256;
constexpr int kPer = 8;
constexpr int kChunk = kThreads * kPer;

struct L2 {
    long long x, y;
};
__device__ inline L2 l2add(L2 a, L2 b) { return L2{a.x + b.x, a.y + b.y}; }

__device__ inline L2 wave_incl_scan(L2 v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        long long ux = __shfl_up(v.x, o, 64);
        long long uy = __shfl_up(v.y, o, 64);
        if (lane >= o) { v.x += ux; v.y += uy; }
    }
    return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix
// and writes the block total to *total (all threads).
__device__ inline L2 block_excl_scan(L2 v, L2* total) {
    __shared__ L2 s_w[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    L2 inc = wave_incl_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    L2 base{0, 0}, tot{0, 0};
    for (int k = 0; k < kThreads / 64; ++k) {
        if (k < w) base = l2add(base, s_w[k]);
        tot = l2add(tot, s_w[k]);
    }
    __syncthreads();
    *total = tot;
    return L2{base.x + inc.x - v.x, base.y + inc.y - v.y};
}

template <typename T>
__device__ inline L2 load2(const T* p, int64_t i);
template <>
__device__ inline L2 load2<int2>(const int2* p, int64_t i) {
    int2 v = p[i];
    return L2{v.x, v.y};
}
template <>
__device__ inline L2 load2<int>(const int* p, int64_t i) {
    return L2{p[i], 0};
}
template <typename T>
__device__ inline void store2(T* p, int64_t i, L2 v);
template <>
__device__ inline void store2<int2>(int2* p, int64_t i, L2 v) {
    p[i] = make_int2((int)v.x, (int)v.y);
}
template <>
__device__ inline void store2<int>(int* p, int64_t i, L2 v) {
    p[i] = (int)v.x;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_reduce(const T* __restrict__ in, int64_t n,
                                                     L2* __restrict__ partial) {
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kPer;
    // the thread's loads in flight at once (index clamped, past the end unused)
    L2 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = load2(in, min(base + k, n - 1));
    L2 s{0, 0};
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (base + k < n) s = l2add(s, v[k]);
    L2 tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(L2* __restrict__ partial, int64_t nb,
                                                            long long* __restrict__ totals) {
    L2 carry{0, 0};
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        const int64_t b = b0 + threadIdx.x;
        L2 v = (b < nb) ? partial[b] : L2{0, 0};
        L2 tot;
        L2 ex = block_excl_scan(v, &tot);
        if (b < nb) partial[b] = l2add(ex, carry);
        carry = l2add(carry, tot);
    }
    if (threadIdx.x == 0 && totals) {
        totals[0] = carry.x;
        totals[1] = carry.y;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_down(const T* __restrict__ in, T* __restrict__ out,
                                                   int64_t n, const L2* __restrict__ partial) {
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kPer;
    L2 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = load2(in, min(base + k, n - 1));  // in flight at once
    L2 s{0, 0};
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (base + k >= n) v[k] = L2{0, 0};
        s = l2add(s, v[k]);
    }
    L2 tot;
    L2 ex = l2add(block_excl_scan(s, &tot), partial[blockIdx.x]);
    for (int k = 0; k < kPer; ++k) {
        if (base + k < n) store2(out, base + k, ex);
        ex = l2add(ex, v[k]);
    }
}

template <typename T>
hipError_t scan_impl(const T* in, T* out, int64_t n, long long* totals, void* tmp, hipStream_t st) {
    const int64_t nb = (n + kChunk - 1) / kChunk;
    L2* partial = (L2*)tmp;
    if (n <= 0) {
        if (totals) {
            hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, st, partial, (int64_t)0, totals);
            return hipGetLastError();
        }
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)nb), dim3(kThreads), 0, st, in, n, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, st, partial, nb, totals);
    hipLaunchKernelGGL(k_down<T>, dim3((unsigned)nb), dim3(kThreads), 0, st, in, out, n,
                       (const L2*)partial);
    return hipGetLastError();
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
    const int64_t nb = (n + kChunk - 1) / kChunk;
    return sizeof(L2) * (size_t)(nb + 1);
}

hipError_t launch_scan_int2(const int2* in, int2* out, int64_t n, long long* totals, void* tmp,
                            hipStream_t st) {
    return scan_impl<int2>(in, out, n, totals, tmp, st);
}

hipError_t launch_scan_int(const int* in, int* out, int64_t n, long long* totals, void* tmp,
                           hipStream_t st) {
    return scan_impl<int>(in, out, n, totals, tmp, st);
}

}  // namespace svr
