// Device-side status of the library's calls: finite checks of parameters and
// outputs, and the capacity check of fixed-capacity binning (no host
// synchronisation).  gfx950.
#include "svr_internal.h"

namespace svr {
namespace {

__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ x, int64_t n,
                                                      DevStatus* __restrict__ st) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !(fabsf(x[i]) <= 3.4028235e38f);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->bits, kStatusNonfinite);
}

// One thread per Gaussian: when the counts of this binning exceed the
// capacity, every Gaussian's record and instance counts and offsets become 0
// (no later stage then reads a record or instance slot: the per-Gaussian
// kernels find a Gaussian's records from its offset and the next one's) and
// the needed counts are recorded.
__global__ __launch_bounds__(256) void k_fixed_capacity(const long long* __restrict__ totals, int64_t cap_rec,
                                                        int64_t cap_inst, int2* __restrict__ counts,
                                                        int2* __restrict__ offsets, int64_t n,
                                                        DevStatus* __restrict__ st) {
    const long long nr = totals[0], ni = totals[1];
    const bool over = nr > cap_rec || ni > cap_inst;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->overflow = over ? 1 : 0;
        if (over) {
            atomicOr(&st->bits, kStatusCapacity);
            st->need_rec = nr;
            st->need_inst = ni;
        }
    }
    if (over && j < n) {
        counts[j] = make_int2(0, 0);
        offsets[j] = make_int2(0, 0);
    }
}

// Instance slots the binning did not fill get the padding key (above every
// tile id, sorted last and skipped by the tile stages).
__global__ __launch_bounds__(256) void k_pad_instances(uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       int64_t cap, const long long* __restrict__ totals,
                                                       const DevStatus* __restrict__ st) {
    const int64_t valid = st->overflow ? 0 : totals[1];
    for (int64_t i = valid + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap;
         i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = 0xffffffffu;
        vals[i] = 0u;
    }
}

}  // namespace

hipError_t launch_check_finite(const float* x, int64_t n, DevStatus* st, hipStream_t s) {
    if (n <= 0 || !x) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, x, n, st);
    return hipGetLastError();
}

hipError_t launch_fixed_capacity(const long long* totals, int64_t cap_rec, int64_t cap_inst, int2* counts,
                                 int2* offsets, int64_t n, DevStatus* st, hipStream_t s) {
    const int64_t blocks = std::max<int64_t>((n + 255) / 256, 1);
    hipLaunchKernelGGL(k_fixed_capacity, dim3((unsigned)blocks), dim3(256), 0, s, totals, cap_rec, cap_inst, counts,
                       offsets, n, st);
    return hipGetLastError();
}

hipError_t launch_pad_instances(uint32_t* keys, uint32_t* vals, int64_t cap, const long long* totals,
                                const DevStatus* st, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((cap + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pad_instances, dim3((unsigned)blocks), dim3(256), 0, s, keys, vals, cap, totals, st);
    return hipGetLastError();
}

}  // namespace svr
