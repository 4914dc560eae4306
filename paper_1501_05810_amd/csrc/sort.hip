// Device-wide exclusive scan and LSD radix sort of (uint32 key, uint32 value) pairs.
//
// Both are deterministic (integer arithmetic only; the sort is stable), which
// makes the cell list, the canonical contact order and the colour-major order
// reproducible run to run.  The sort ranks keys inside a wavefront with
// 64-bit ballots: eight ballots, one per digit bit, leave every lane the mask
// of the lanes holding the same 8-bit digit, whose population count below the
// lane is its stable rank.
#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

constexpr int kRadixBlock = 256;
constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kRadixBlock * kRadixRounds;
constexpr int kRadixDigits = 256;
constexpr int kWaves = kRadixBlock / 64;

__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan over the block's threads; *total receives the block sum.
__device__ inline int block_exclusive_scan(int v, int *lds, int *total) {
    const int inc = wave_inclusive_scan(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        int s = lds[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const int32_t *in, int64_t n, int32_t *block_sums) {
    __shared__ int lds[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) s += in[i];
    }
    int total;
    (void)block_exclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t *in, int64_t n, const int32_t *block_offsets,
                                                           int32_t *out, int32_t *total_dev) {
    __shared__ int lds[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int vals[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        vals[k] = i < n ? in[i] : 0;
        s += vals[k];
    }
    int total;
    int run = block_exclusive_scan(s, lds, &total) + (block_offsets ? block_offsets[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += vals[k];
    }
    if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) *total_dev = run;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t exclusive_scan_tmp_bytes(int64_t n) {
    size_t bytes = 0;
    int64_t m = n;
    while (m > kScanTile) {
        int64_t nb = ceil_div(m, kScanTile);
        bytes += 2 * (size_t)nb * sizeof(int32_t);
        m = nb;
    }
    return bytes + 256;
}

nbgs_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev, void *tmp,
                               size_t tmp_bytes, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) NBGS_HIP(hipMemsetAsync(total_dev, 0, sizeof(int32_t), s));
        return NBGS_OK;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb == 1) {
        k_scan_apply<<<1, kScanBlock, 0, s>>>(in, n, nullptr, out, total_dev);
        NBGS_HIP(hipGetLastError());
        return NBGS_OK;
    }
    if (2 * (size_t)nb * sizeof(int32_t) > tmp_bytes) {
        set_error("scan scratch too small");
        return NBGS_ERR_CAPACITY;
    }
    int32_t *sums = (int32_t *)tmp;
    int32_t *offs = sums + nb;
    k_scan_reduce<<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, sums);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sums, offs, nb, nullptr, (void *)(offs + nb),
                                tmp_bytes - 2 * (size_t)nb * sizeof(int32_t), s));
    k_scan_apply<<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, offs, out, total_dev);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

namespace {

__global__ void __launch_bounds__(kRadixBlock) k_radix_hist(const uint32_t *keys, int64_t n, int shift,
                                                            int32_t *hist, int nblocks) {
    __shared__ int cnt[kRadixDigits];
    for (int d = threadIdx.x; d < kRadixDigits; d += kRadixBlock) cnt[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        int64_t i = base + (int64_t)r * kRadixBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadixDigits; d += kRadixBlock)
        hist[(int64_t)d * nblocks + blockIdx.x] = cnt[d];
}

// Stable scatter of one tile of kRadixTile elements.  Element order inside
// the tile is (round, wave, lane), the input order; each element's place in
// the tile sorted by digit (the tile's digit starts plus its stable rank) is
// found with ballots and LDS counts, the tile is rearranged in LDS, and then
// written out so that neighbouring threads store neighbouring elements of one
// digit's run.  The global start of (digit, tile) comes from the digit-major
// scan of the histograms; the tile's count of a digit is the difference of two
// neighbouring scan entries (the last one's end is n).
__global__ void __launch_bounds__(kRadixBlock) k_radix_scatter(const uint32_t *keys, const uint32_t *vals,
                                                               uint32_t *okeys, uint32_t *ovals, int64_t n, int shift,
                                                               const int32_t *offs, int nblocks) {
    __shared__ uint32_t lk[kRadixTile], lv[kRadixTile];
    __shared__ int gstart[kRadixDigits], lstart[kRadixDigits], run[kRadixDigits];
    __shared__ int wcnt[kWaves][kRadixDigits];
    __shared__ int scan_lds[kRadixBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    static_assert(kRadixBlock == kRadixDigits, "one thread per digit");
    {
        const int64_t idx = (int64_t)tid * nblocks + blockIdx.x;
        const int g = offs[idx];
        const int next = idx + 1 < (int64_t)kRadixDigits * nblocks ? offs[idx + 1] : (int)n;
        gstart[tid] = g;
        int total;
        lstart[tid] = block_exclusive_scan(next - g, scan_lds, &total);
        run[tid] = 0;
    }
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < kRadixRounds; ++r) {
        for (int d = tid; d < kWaves * kRadixDigits; d += kRadixBlock) (&wcnt[0][0])[d] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * kRadixBlock + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? keys[i] : 0u;
        const uint32_t v = valid ? vals[i] : 0u;
        const uint32_t dig = (k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (dig >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = lstart[dig] + run[dig] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
            lk[pos] = k;
            lv[pos] = v;
        }
        __syncthreads();
        {
            int add = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
            run[tid] += add;
        }
        __syncthreads();  // before the next round clears the wave counts
    }
    const int tile_n = (int)(n - base < (int64_t)kRadixTile ? n - base : (int64_t)kRadixTile);
    for (int j = tid; j < tile_n; j += kRadixBlock) {
        const uint32_t k = lk[j];
        const uint32_t d = (k >> shift) & 255u;
        const int dst = gstart[d] + (j - lstart[d]);
        okeys[dst] = k;
        ovals[dst] = lv[j];
    }
}

}  // namespace

size_t radix_hist_entries(int64_t n) { return (size_t)kRadixDigits * (size_t)ceil_div(n > 0 ? n : 1, kRadixTile); }

nbgs_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n,
                             int32_t key_bits, int32_t *hist_tmp, void *scan_tmp, size_t scan_tmp_bytes,
                             bool *result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1 || key_bits <= 0) return NBGS_OK;
    const int nblocks = (int)ceil_div(n, kRadixTile);
    const int passes = (key_bits + 7) / 8;
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        k_radix_hist<<<nblocks, kRadixBlock, 0, s>>>(ki, n, shift, hist_tmp, nblocks);
        NBGS_HIP(hipGetLastError());
        NBGS_TRY(exclusive_scan_i32(hist_tmp, hist_tmp, (int64_t)kRadixDigits * nblocks, nullptr, scan_tmp,
                                    scan_tmp_bytes, s));
        k_radix_scatter<<<nblocks, kRadixBlock, 0, s>>>(ki, vi, ko, vo, n, shift, hist_tmp, nblocks);
        NBGS_HIP(hipGetLastError());
        uint32_t *t = ki;
        ki = ko;
        ko = t;
        t = vi;
        vi = vo;
        vo = t;
    }
    *result_in_alt = (passes % 2) == 1;
    return NBGS_OK;
}

}  // namespace nbgs
