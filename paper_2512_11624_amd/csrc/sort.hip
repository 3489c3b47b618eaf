// Stable LSD radix sort of 32-bit (key, value) pairs for tile binning.  The
// binning sort also carries each pair's input position as a second payload
// (generated on the first pass), so later stages can find an instance's
// emission slot without an inverse permutation.
//
// Each pass sorts on an 8-bit digit:
//   1. upsweep: per-block digit histogram in LDS  -> hist[digit * nblocks + block]
//   2. exclusive scan of hist (digit-major), giving every (digit, block) its
//      global output offset
//   3. downsweep: every wave ranks its 1024 keys in input order with ballot
//      "match" masks (lanes holding the same digit), keeps per-wave digit
//      counters in LDS, scatters the block's keys into LDS in digit order and
//      writes them out with coalesced runs per digit.
// Ranking follows input order inside a wave (iteration by iteration, lane by
// lane), waves are ordered inside a block and blocks by the scan, so the sort
// is stable and deterministic.
#include "svr_internal.h"

namespace svr {
hipError_t launch_scan_int(const int* in, int* out, int64_t n, long long* totals, void* tmp,
                           hipStream_t st);
size_t scan_tmp_bytes(int64_t n);

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kIters = 16;
constexpr int kItems = kThreads * kIters;  // 4096 keys per block
constexpr int kRadix = 256;

__global__ __launch_bounds__(kThreads) void k_upsweep(const uint32_t* __restrict__ keys, int64_t n,
                                                      int shift, int* __restrict__ hist, int nb) {
    __shared__ int s_h[kRadix];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kItems;
    for (int k = 0; k < kIters; ++k) {
        const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = s_h[threadIdx.x];
}

template <int kIdx>  // 0: no second payload; 1: second payload read; 2: second payload = input index
__global__ __launch_bounds__(kThreads) void k_downsweep(const uint32_t* __restrict__ keys_in,
                                                        const uint32_t* __restrict__ vals_in,
                                                        uint32_t* __restrict__ keys_out,
                                                        uint32_t* __restrict__ vals_out,
                                                        const uint32_t* __restrict__ idx_in,
                                                        uint32_t* __restrict__ idx_out, int64_t n,
                                                        int shift, int nbits,
                                                        const int* __restrict__ offs, int nb) {
    __shared__ int s_cnt[kWaves][kRadix];
    __shared__ int s_dstart[kRadix];
    __shared__ int s_gofs[kRadix];
    __shared__ int s_wsum[kWaves];
    __shared__ uint32_t s_k[kItems];
    __shared__ uint32_t s_v[kItems];
    __shared__ uint32_t s_x[kIdx ? kItems : 1];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = 0; q < kWaves; ++q) s_cnt[q][tid] = 0;
    s_gofs[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kItems;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t kk[kIters], vv[kIters], xx[kIdx ? kIters : 1];
    int rk[kIters];
    for (int it = 0; it < kIters; ++it) {
        const int64_t i = base + (int64_t)w * (kIters * 64) + (int64_t)it * 64 + lane;
        const bool valid = i < n;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const uint32_t val = valid ? vals_in[i] : 0u;
        if (kIdx == 1) xx[it] = valid ? idx_in[i] : 0u;
        if (kIdx == 2) xx[it] = (uint32_t)i;
        const int d = (int)((key >> shift) & (kRadix - 1));
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        if (!valid) peers = 0ull;
        const int rank = __popcll(peers & lt_mask);
        const int cnt = __popcll(peers);
        const int leader = valid ? (__ffsll((long long)peers) - 1) : lane;
        int basec = 0;
        if (valid && lane == leader) {
            basec = s_cnt[w][d];
            s_cnt[w][d] = basec + cnt;
        }
        basec = __shfl(basec, leader, 64);
        kk[it] = key;
        vv[it] = val;
        rk[it] = valid ? basec + rank : -1;
    }
    __syncthreads();
    // exclusive prefix over waves for every digit, and digit totals
    int tot = 0;
    for (int q = 0; q < kWaves; ++q) {
        const int c = s_cnt[q][tid];
        s_cnt[q][tid] = tot;
        tot += c;
    }
    // exclusive scan of totals over digits (one digit per thread)
    int incl = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wsum[w] = incl;
    __syncthreads();
    int wbase = 0;
    for (int q = 0; q < w; ++q) wbase += s_wsum[q];
    s_dstart[tid] = wbase + incl - tot;
    __syncthreads();
    for (int it = 0; it < kIters; ++it) {
        if (rk[it] >= 0) {
            const int d = (int)((kk[it] >> shift) & (kRadix - 1));
            const int pos = s_dstart[d] + s_cnt[w][d] + rk[it];
            s_k[pos] = kk[it];
            s_v[pos] = vv[it];
            if (kIdx) s_x[pos] = xx[it];
        }
    }
    __syncthreads();
    const int64_t rem = n - base;
    const int nvalid = rem < kItems ? (int)rem : kItems;
    for (int p = tid; p < nvalid; p += kThreads) {
        const uint32_t key = s_k[p];
        const int d = (int)((key >> shift) & (kRadix - 1));
        const int64_t g = (int64_t)s_gofs[d] + (p - s_dstart[d]);
        keys_out[g] = key;
        vals_out[g] = s_v[p];
        if (kIdx) idx_out[g] = s_x[p];
    }
}

}  // namespace

size_t sort_tmp_bytes(int64_t n) {
    const int64_t nb = (n + kItems - 1) / kItems;
    const int64_t nh = nb * kRadix;
    size_t a = sizeof(int) * (size_t)nh * 2;  // hist + offsets
    a = (a + 255) & ~(size_t)255;
    return a + scan_tmp_bytes(nh) + 256;
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             int64_t n, int key_bits, void* tmp, bool* result_in_alt,
                             hipStream_t st, uint32_t* idx, uint32_t* idx_alt) {
    *result_in_alt = false;
    if (n <= 0 || key_bits <= 0) return hipSuccess;
    const int64_t nb = (n + kItems - 1) / kItems;
    const int64_t nh = nb * kRadix;
    int* hist = (int*)tmp;
    int* offs = hist + nh;
    size_t a = sizeof(int) * (size_t)nh * 2;
    a = (a + 255) & ~(size_t)255;
    void* stmp = (char*)tmp + a;
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    uint32_t *xi = idx, *xo = idx_alt;
    bool alt = false;
    bool first = true;
    for (int shift = 0; shift < key_bits; shift += 8) {
        const int nbits = (key_bits - shift) < 8 ? (key_bits - shift) : 8;
        hipLaunchKernelGGL(k_upsweep, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, n, shift, hist, (int)nb);
        hipError_t e = launch_scan_int(hist, offs, nh, nullptr, stmp, st);
        if (e != hipSuccess) return e;
        if (!idx)
            hipLaunchKernelGGL(k_downsweep<0>, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                               (const uint32_t*)nullptr, (uint32_t*)nullptr, n, shift, nbits, (const int*)offs, (int)nb);
        else if (first)
            hipLaunchKernelGGL(k_downsweep<2>, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                               (const uint32_t*)nullptr, xo, n, shift, nbits, (const int*)offs, (int)nb);
        else
            hipLaunchKernelGGL(k_downsweep<1>, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                               (const uint32_t*)xi, xo, n, shift, nbits, (const int*)offs, (int)nb);
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        t = xi; xi = xo; xo = t;
        alt = !alt;
        first = false;
    }
    *result_in_alt = alt;
    return hipGetLastError();
}

}  // namespace svr
