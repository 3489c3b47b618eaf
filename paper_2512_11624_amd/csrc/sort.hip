// Stable LSD radix sort of 32-bit (key, value) pairs for tile binning.  The
// binning sort also carries each pair's input position as a second payload
// (generated on the first pass), so later stages can find an instance's
// emission slot without an inverse permutation.
//
// The key is cut into as few digits of 8 or 9 bits as cover it (a 16-bit key
// takes two 8-bit passes, an 18-bit key two 9-bit passes; wider digits make
// the histogram scan and the per-block LDS footprint grow faster than a pass
// costs).  Each pass:
//   1. upsweep: per-block digit histogram in LDS  -> hist[digit * nblocks + block]
//   2. exclusive scan of hist (digit-major), giving every (digit, block) its
//      global output offset
//   3. downsweep: every wave ranks its 512 keys in input order with ballot
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
constexpr int kIters = 8;
constexpr int kItems = kThreads * kIters;  // 2048 keys per block (a block's LDS then allows 4-5 blocks per CU)
constexpr int kMaxDigitBits = 9;

template <int kBits>
__global__ __launch_bounds__(kThreads) void k_upsweep(const uint32_t* __restrict__ keys, int64_t n,
                                                      int shift, int nbits, int* __restrict__ hist, int nb) {
    constexpr int kRadix = 1 << kBits, D = kRadix / kThreads;
    const uint32_t dmask = (1u << nbits) - 1u;
    // one histogram per wave: neighbouring keys often share a digit, and the
    // LDS serialises atomics on one address
    __shared__ int s_h[kWaves][kRadix];
    const int w = threadIdx.x >> 6;
    for (int q = 0; q < kWaves; ++q)
        for (int j = 0; j < D; ++j) s_h[q][threadIdx.x * D + j] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kItems;
    // all of the thread's key loads in flight at once (index clamped, result
    // unused past the end), then the counts
    uint32_t kk[kIters];
#pragma unroll
    for (int k = 0; k < kIters; ++k) kk[k] = keys[min(base + (int64_t)k * kThreads + threadIdx.x, n - 1)];
#pragma unroll
    for (int k = 0; k < kIters; ++k)
        if (base + (int64_t)k * kThreads + threadIdx.x < n) atomicAdd(&s_h[w][(kk[k] >> shift) & dmask], 1);
    __syncthreads();
    for (int j = 0; j < D; ++j) {
        const int d = j * kThreads + threadIdx.x;  // coalesced over the block index for fixed j
        int c = 0;
        for (int q = 0; q < kWaves; ++q) c += s_h[q][d];
        hist[(int64_t)d * nb + blockIdx.x] = c;
    }
}

// kIdx: 0 no second payload; 1 second payload read; 2 second payload = input index
template <int kBits, int kIdx>
__global__ __launch_bounds__(kThreads) void k_downsweep(const uint32_t* __restrict__ keys_in,
                                                        const uint32_t* __restrict__ vals_in,
                                                        uint32_t* __restrict__ keys_out,
                                                        uint32_t* __restrict__ vals_out,
                                                        const uint32_t* __restrict__ idx_in,
                                                        uint32_t* __restrict__ idx_out, int64_t n,
                                                        int shift, int nbits,
                                                        const int* __restrict__ offs, int nb) {
    constexpr int kRadix = 1 << kBits, D = kRadix / kThreads;
    const uint32_t dmask = (1u << nbits) - 1u;  // bits of the key above the sorted ones are ignored
    __shared__ int s_cnt[kWaves][kRadix];
    __shared__ int s_dstart[kRadix];
    __shared__ int s_gofs[kRadix];
    __shared__ int s_wsum[kWaves];
    __shared__ uint32_t s_k[kItems];
    __shared__ uint32_t s_v[kItems];
    __shared__ uint32_t s_x[kIdx ? kItems : 1];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = 0; q < kWaves; ++q)
        for (int j = 0; j < D; ++j) s_cnt[q][j * kThreads + tid] = 0;
    for (int j = 0; j < D; ++j) {
        const int d = j * kThreads + tid;
        s_gofs[d] = offs[(int64_t)d * nb + blockIdx.x];
    }
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kItems;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t kk[kIters], vv[kIters], xx[kIdx ? kIters : 1];
    int rk[kIters];
    // all of the thread's loads in flight at once (index clamped, results
    // selected), then the ranking
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int64_t i = base + (int64_t)w * (kIters * 64) + (int64_t)it * 64 + lane;
        const int64_t ic = min(i, n - 1);
        kk[it] = keys_in[ic];
        vv[it] = vals_in[ic];
        if (kIdx == 1) xx[it] = idx_in[ic];
        if (kIdx == 2) xx[it] = (uint32_t)i;
    }
    __builtin_amdgcn_sched_barrier(0);
    for (int it = 0; it < kIters; ++it) {
        const int64_t i = base + (int64_t)w * (kIters * 64) + (int64_t)it * 64 + lane;
        const bool valid = i < n;
        const uint32_t key = valid ? kk[it] : 0u;
        const uint32_t val = valid ? vv[it] : 0u;
        const int d = (int)((key >> shift) & dmask);
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
    // exclusive prefix over waves for every digit (thread owns digits
    // tid*D .. tid*D+D-1), then an exclusive scan of the digit totals
    int tots[D];
    int local = 0;
    for (int j = 0; j < D; ++j) {
        const int d = tid * D + j;
        int tot = 0;
        for (int q = 0; q < kWaves; ++q) {
            const int c = s_cnt[q][d];
            s_cnt[q][d] = tot;
            tot += c;
        }
        tots[j] = tot;
        local += tot;
    }
    int incl = local;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wsum[w] = incl;
    __syncthreads();
    int run = incl - local;
    for (int q = 0; q < w; ++q) run += s_wsum[q];
    for (int j = 0; j < D; ++j) {
        s_dstart[tid * D + j] = run;
        run += tots[j];
    }
    __syncthreads();
    for (int it = 0; it < kIters; ++it) {
        if (rk[it] >= 0) {
            const int d = (int)((kk[it] >> shift) & dmask);
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
        const int d = (int)((key >> shift) & dmask);
        const int64_t g = (int64_t)s_gofs[d] + (p - s_dstart[d]);
        keys_out[g] = key;
        vals_out[g] = s_v[p];
        if (kIdx) idx_out[g] = s_x[p];
    }
}

template <int kBits>
hipError_t sort_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, const uint32_t* xi,
                     uint32_t* xo, int idx_mode, int64_t n, int shift, int nbits, int* hist, int* offs,
                     void* stmp, int nb, hipStream_t st) {
    hipLaunchKernelGGL(k_upsweep<kBits>, dim3((unsigned)nb), dim3(kThreads), 0, st, ki, n, shift, nbits, hist, nb);
    hipError_t e = launch_scan_int(hist, offs, (int64_t)nb << kBits, nullptr, stmp, st);
    if (e != hipSuccess) return e;
    if (idx_mode == 0)
        hipLaunchKernelGGL((k_downsweep<kBits, 0>), dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                           (const uint32_t*)nullptr, (uint32_t*)nullptr, n, shift, nbits, (const int*)offs, nb);
    else if (idx_mode == 2)
        hipLaunchKernelGGL((k_downsweep<kBits, 2>), dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                           (const uint32_t*)nullptr, xo, n, shift, nbits, (const int*)offs, nb);
    else
        hipLaunchKernelGGL((k_downsweep<kBits, 1>), dim3((unsigned)nb), dim3(kThreads), 0, st, ki, vi, ko, vo,
                           xi, xo, n, shift, nbits, (const int*)offs, nb);
    return hipGetLastError();
}

}  // namespace

int radix_digit_bits(int key_bits) {
    if (key_bits <= 8) return 8;
    const int passes = (key_bits + kMaxDigitBits - 1) / kMaxDigitBits;
    const int width = (key_bits + passes - 1) / passes;
    return width < 8 ? 8 : width;
}

size_t sort_tmp_bytes(int64_t n) {
    const int64_t nb = (n + kItems - 1) / kItems;
    const int64_t nh = nb << kMaxDigitBits;
    size_t a = sizeof(int) * (size_t)nh * 2;  // hist + offsets
    a = (a + 255) & ~(size_t)255;
    return a + scan_tmp_bytes(nh) + 256;
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             int64_t n, int key_bits, void* tmp, bool* result_in_alt,
                             hipStream_t st, uint32_t* idx, uint32_t* idx_alt, int first_bit) {
    *result_in_alt = false;
    if (n <= 0 || key_bits <= first_bit || first_bit < 0) return hipSuccess;
    const int64_t nb = (n + kItems - 1) / kItems;
    const int64_t nh = nb << kMaxDigitBits;
    int* hist = (int*)tmp;
    int* offs = hist + nh;
    size_t a = sizeof(int) * (size_t)nh * 2;
    a = (a + 255) & ~(size_t)255;
    void* stmp = (char*)tmp + a;
    const int width = radix_digit_bits(key_bits - first_bit);
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    uint32_t *xi = idx, *xo = idx_alt;
    bool alt = false;
    bool first = true;
    for (int shift = first_bit; shift < key_bits; shift += width) {
        const int nbits = (key_bits - shift) < width ? (key_bits - shift) : width;
        const int mode = !idx ? 0 : (first ? 2 : 1);
        hipError_t e;
        switch (width) {
            case 8: e = sort_pass<8>(ki, vi, ko, vo, xi, xo, mode, n, shift, nbits, hist, offs, stmp, (int)nb, st); break;
            case 9: e = sort_pass<9>(ki, vi, ko, vo, xi, xo, mode, n, shift, nbits, hist, offs, stmp, (int)nb, st); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
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
