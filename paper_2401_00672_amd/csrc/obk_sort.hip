// Device primitives used by the plan: exclusive prefix sums and a stable LSD
// radix sort of (uint32 key, uint32 value) pairs.  Both are deterministic:
// the result never depends on scheduling.
#include "obk_internal.h"

namespace obk {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // 2048

// Inclusive scan of one value per thread across a 256-thread block.
// Returns the inclusive prefix; *total receives the block total.
template <class T>
__device__ T block_inclusive_scan(T v, T* lds_waves, T* total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        T u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    if (lane == 63) lds_waves[wave] = v;
    __syncthreads();
    T add = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; w++) {
        T s = lds_waves[w];
        if (w < wave) add += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return v + add;
}

__global__ void k_tile_sums(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ sums) {
    __shared__ int64_t lw[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_inclusive_scan<int64_t>(s, lw, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_tile_scan(const int64_t* in, int64_t n, const int64_t* __restrict__ offsets,
                            int64_t* out) {
    __shared__ int64_t lw[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t incl = block_inclusive_scan<int64_t>(s, lw, &tot);
    int64_t run = incl - s + (offsets ? offsets[blockIdx.x] : 0);
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

__global__ void k_widen_i32(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

void scan_rec(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_tile_scan<<<1, kScanThreads, 0, s>>>(in, n, nullptr, out);
        OBK_HIP(hipGetLastError());
        return;
    }
    DevArray<int64_t> sums;
    sums.alloc(nb);
    k_tile_sums<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums.get());
    OBK_HIP(hipGetLastError());
    scan_rec(sums.get(), sums.get(), nb, s);
    k_tile_scan<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums.get(), out);
    OBK_HIP(hipGetLastError());
    sync_for_free(s);   // sums is freed on return
}

// *out = *a (+ *b when b is given); one thread
__global__ void k_total(const int64_t* a, const int64_t* b, int64_t* out) {
    const int64_t v = *a;
    *out = b ? v + *b : v;
}

// ------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 2048
constexpr int kDigitBits = 4;
constexpr int kBins = 1 << kDigitBits;                 // 16

__global__ void k_digit_hist(const uint32_t* __restrict__ keys, int64_t n, int shift, int64_t nblocks,
                             int64_t* __restrict__ counts) {
    __shared__ int hist[kBins];
    if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    for (int k = 0; k < kSortItems; k++) {
        int64_t i = base + k;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & (kBins - 1)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kBins) counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter: element order within a block is (thread, item); per-thread
// digit counts are packed four digits to a uint64 (16-bit fields: a block
// holds 2048 elements, so no field can overflow) and scanned across threads.
__global__ void k_digit_scatter(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
                                uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n,
                                int shift, int64_t nblocks, const int64_t* __restrict__ offsets) {
    __shared__ uint64_t lw[kSortThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    // loads are unconditional at clamped in-range indices (predicated form)
    uint32_t k[kSortItems];
    uint32_t v[kSortItems];
    int dig[kSortItems];
    uint64_t packed[kBins / 4] = {0, 0, 0, 0};
    for (int j = 0; j < kSortItems; j++) {
        const int64_t i = base + j;
        const int64_t ic = i < n ? i : n - 1;
        k[j] = keys_in[ic];
        v[j] = vals_in ? vals_in[ic] : 0u;
        const int d = (int)((k[j] >> shift) & (kBins - 1));
        dig[j] = i < n ? d : -1;
        const uint64_t one = i < n ? 1ull : 0ull;
        for (int q = 0; q < kBins / 4; q++)
            packed[q] += (q == (d >> 2)) ? (one << (16 * (d & 3))) : 0ull;
    }
    uint64_t excl[kBins / 4];
    for (int q = 0; q < kBins / 4; q++) {
        uint64_t tot;
        uint64_t incl = block_inclusive_scan<uint64_t>(packed[q], lw, &tot);
        excl[q] = incl - packed[q];
    }
    for (int j = 0; j < kSortItems; j++) {
        const int d = dig[j];
        const int dd = d < 0 ? 0 : d;
        // running count of digit dd among this thread's earlier items
        int before = 0;
        for (int t = 0; t < j; t++) before += (dig[t] == dd) ? 1 : 0;
        uint64_t ex = 0;
        for (int q = 0; q < kBins / 4; q++) ex = (q == (dd >> 2)) ? excl[q] : ex;
        const int64_t pos = offsets[(int64_t)dd * nblocks + blockIdx.x] +
                            (int64_t)((ex >> (16 * (dd & 3))) & 0xFFFF) + before;
        if (d >= 0) {
            keys_out[pos] = k[j];
            if (vals_in) vals_out[pos] = v[j];
        }
    }
}

}  // namespace

int bits_for(uint64_t max_value) {
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) b++;
    return b;
}

int64_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return 0;
    // total = in[n-1] + out[n-1], formed on the device (in may alias out)
    DevArray<int64_t> last;
    last.alloc(1);
    k_total<<<1, 1, 0, s>>>(in + n - 1, nullptr, last.get());
    OBK_HIP(hipGetLastError());
    scan_rec(in, out, n, s);
    k_total<<<1, 1, 0, s>>>(last.get(), out + n - 1, last.get());
    OBK_HIP(hipGetLastError());
    int64_t* h = static_cast<int64_t*>(pinned_stage(sizeof(int64_t)));
    OBK_HIP(hipMemcpyAsync(h, last.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    return *h;
}

int64_t scan_counts_i32(const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return 0;
    k_widen_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
    OBK_HIP(hipGetLastError());
    return scan_exclusive_i64(out, out, n, s);
}

void radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits, hipStream_t s) {
    if (n <= 1 || key_bits <= 0) return;
    const int64_t nblocks = (n + kSortTile - 1) / kSortTile;
    DevArray<uint32_t> k2, v2;
    k2.alloc(n);
    if (vals) v2.alloc(n);
    DevArray<int64_t> counts;
    counts.alloc(kBins * nblocks);
    uint32_t *ki = keys, *vi = vals, *ko = k2.get(), *vo = vals ? v2.get() : nullptr;
    const int passes = (key_bits + kDigitBits - 1) / kDigitBits;
    for (int p = 0; p < passes; p++) {
        const int shift = p * kDigitBits;
        k_digit_hist<<<(unsigned)nblocks, kSortThreads, 0, s>>>(ki, n, shift, nblocks, counts.get());
        OBK_HIP(hipGetLastError());
        scan_rec(counts.get(), counts.get(), kBins * nblocks, s);
        k_digit_scatter<<<(unsigned)nblocks, kSortThreads, 0, s>>>(ki, vi, ko, vo, n, shift, nblocks,
                                                                  counts.get());
        OBK_HIP(hipGetLastError());
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    if (ki != keys) {
        OBK_HIP(hipMemcpyAsync(keys, ki, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        if (vals) OBK_HIP(hipMemcpyAsync(vals, vi, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    sync_for_free(s);   // k2, v2 and counts are freed on return
}

}  // namespace obk
