// Cuthill-McKee order on the device, level by level (Section 3.2: the
// reordering step).  The sequential breadth-first search takes the vertices
// of one level in queue order and appends, for each, its unvisited
// neighbours by ascending (degree, index).  A vertex of the next level is
// therefore appended by the earliest vertex of the current level adjacent to
// it, and the next level is ordered by (position of that parent, degree,
// index).  One level step here forms exactly that order:
//   expand   -- every unvisited neighbour u of the frontier gets
//               parent[u] = min frontier position adjacent to it, and the
//               first thread to reach u puts it on a list (in any order)
//   sort     -- by the key (parent, degree, index), which is unique, so the
//               order of the list does not matter: one workgroup sorts a
//               short level in LDS; a long one takes stable radix passes
//   append   -- they become the next frontier at the end of the sequence
// A component ends when the next level is empty; the next one starts at the
// unvisited vertex of least (degree, index).  Vertices of degree 0 are such
// one-vertex components, and they come first in index order, so they are
// placed in one step.
//
// Each level costs a fixed number of launches and one host synchronisation,
// so the device form only pays on graphs whose levels are wide.  The driver
// gives up once the levels stay narrow and hands the exact state (sequence so
// far, visited flags, unexpanded frontier) to the host loop, which resumes
// where the device stopped; the sequence is the same either way.
#include <climits>
#include <cstring>
#include <vector>

#include "obk_internal.h"

namespace obk {

namespace {

constexpr int kRT = 256;
inline unsigned rblk(int64_t n) { return (unsigned)((n + kRT - 1) / kRT); }

__global__ void k_deg_stats(int64_t n, const int32_t* __restrict__ deg, int32_t* __restrict__ zero_flag,
                            unsigned* __restrict__ maxdeg) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t d = deg[v];
    zero_flag[v] = d == 0 ? 1 : 0;
    atomicMax(maxdeg, (unsigned)d);
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_fill_i32(int64_t n, int32_t* __restrict__ p, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// parent[u] = min over frontier positions i adjacent to unvisited u; the
// first thread to claim u (cand[u] 0 -> 1) appends it to list
__global__ void k_expand(int64_t nf, const int32_t* __restrict__ frontier, const int64_t* __restrict__ gptr,
                         const int32_t* __restrict__ gadj, const uint8_t* __restrict__ vis,
                         int32_t* __restrict__ parent, int32_t* __restrict__ cand, uint32_t* __restrict__ list,
                         unsigned* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int32_t v = frontier[i];
    const int64_t k1 = gptr[v + 1];
    for (int64_t k = gptr[v]; k < k1; k++) {
        const int32_t u = gadj[k];
        if (!vis[u]) {
            atomicMin(&parent[u], (int32_t)i);
            if (atomicExch(&cand[u], 1) == 0) list[atomicAdd(count, 1u)] = (uint32_t)u;
        }
    }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

// One workgroup sorts a short level (m <= kSmallLevel) by the 64-bit key
// parent << (db + ub) | degree << ub | index (bitonic network over the next
// power of two, padded with the largest key) and appends it: seq, visited,
// parent and claim reset.
constexpr int kSmallLevel = 4096;
constexpr int kSortWG = 1024;
__global__ __launch_bounds__(kSortWG) void k_sort_append_small(
    int32_t m, const uint32_t* __restrict__ list, const int32_t* __restrict__ deg, int32_t* __restrict__ parent,
    int32_t* __restrict__ cand, int db, int ub, int32_t* __restrict__ seq, uint8_t* __restrict__ vis) {
    __shared__ unsigned long long key[kSmallLevel];
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += kSortWG) {
        unsigned long long k = ULLONG_MAX;
        if (i < m) {
            const uint32_t u = list[i];
            k = ((unsigned long long)(uint32_t)parent[u] << (db + ub)) |
                ((unsigned long long)(uint32_t)deg[u] << ub) | u;
        }
        key[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < p2; i += kSortWG) {
                const int j = i ^ stride;
                if (j > i) {
                    const unsigned long long a = key[i], b = key[j];
                    const bool up = (i & size) == 0;
                    if ((a > b) == up) { key[i] = b; key[j] = a; }
                }
            }
            __syncthreads();
        }
    }
    const uint64_t umask = (ub >= 64) ? ~0ull : ((1ull << ub) - 1ull);
    for (int i = threadIdx.x; i < m; i += kSortWG) {
        const int32_t u = (int32_t)(key[i] & umask);
        seq[i] = u;
        vis[u] = 1;
        parent[u] = INT_MAX;
        cand[u] = 0;
    }
}

// out[off[u]] = u for every flagged u (ascending u); the flags are cleared
__global__ void k_emit(int64_t n, int32_t* __restrict__ cand, const int64_t* __restrict__ off,
                       uint32_t* __restrict__ out) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || !cand[u]) return;
    out[off[u]] = (uint32_t)u;
    cand[u] = 0;
}

template <bool kParent>
__global__ void k_key_of(int64_t m, const uint32_t* __restrict__ vals, const int32_t* __restrict__ deg,
                         const int32_t* __restrict__ parent, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) keys[i] = (uint32_t)(kParent ? parent[vals[i]] : deg[vals[i]]);
}

// the sorted new vertices join the sequence: visited, parent and claim reset
__global__ void k_append(int64_t m, const uint32_t* __restrict__ vals, int32_t* __restrict__ seq,
                         uint8_t* __restrict__ vis, int32_t* __restrict__ parent, int32_t* __restrict__ cand) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t u = (int32_t)vals[i];
    seq[i] = u;
    vis[u] = 1;
    parent[u] = INT_MAX;
    cand[u] = 0;
}

// (degree << ub | index) when that fits 32 bits, else the index alone
template <bool kPacked>
__global__ void k_key_deg_index(int64_t m, const uint32_t* __restrict__ vals, const int32_t* __restrict__ deg,
                                int ub, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) keys[i] = kPacked ? (((uint32_t)deg[vals[i]] << ub) | vals[i]) : vals[i];
}

// least (degree << 32 | index) over the unvisited vertices
__global__ __launch_bounds__(kRT) void k_argmin_unvisited(int64_t n, const int32_t* __restrict__ deg,
                                                          const uint8_t* __restrict__ vis,
                                                          unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[kRT];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long key = ULLONG_MAX;
    if (v < n && !vis[v]) key = ((unsigned long long)(uint32_t)deg[v] << 32) | (uint32_t)v;
    red[threadIdx.x] = key;
    __syncthreads();
    for (int st = kRT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != ULLONG_MAX) atomicMin(out, red[0]);
}

__global__ void k_start(int32_t s, int32_t* __restrict__ seq, uint8_t* __restrict__ vis) {
    *seq = s;
    vis[s] = 1;
}

template <class T> T d2h_one(const T* d, hipStream_t s) {
    T* h = static_cast<T*>(pinned_stage(sizeof(T)));
    OBK_HIP(hipMemcpyAsync(h, d, sizeof(T), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    return *h;
}

template <class T> void d2h(T* h, const T* d, size_t n, hipStream_t s) {
    if (!n) return;
    stage_d2h(h, d, n * sizeof(T), s);
}

}  // namespace

void device_rcm(int64_t n, const int32_t* adj, const int32_t* deg, bool give_up, hipStream_t s, int32_t* perm) {
    if (n <= 0) return;
    DevArray<int64_t> gptr, off;
    gptr.alloc(n + 1);
    off.alloc(n);
    const int64_t mu = scan_counts_i32(deg, gptr.get(), n, s);
    k_set_i64<<<1, 1, 0, s>>>(gptr.get() + n, mu);
    DevArray<int32_t> seq, parent, cand;
    DevArray<uint8_t> vis;
    DevArray<uint32_t> keys, vals;
    DevArray<unsigned> maxdeg, count;
    DevArray<unsigned long long> best;
    seq.alloc(n); parent.alloc(n); cand.alloc(n); vis.alloc(n); keys.alloc(n); vals.alloc(n);
    maxdeg.alloc(1); count.alloc(1); best.alloc(1);
    OBK_HIP(hipMemsetAsync(vis.get(), 0, n, s));
    OBK_HIP(hipMemsetAsync(maxdeg.get(), 0, sizeof(unsigned), s));
    k_fill_i32<<<rblk(n), kRT, 0, s>>>(n, parent.get(), INT_MAX);
    // degree-0 vertices first, ascending; cand holds their flags
    k_deg_stats<<<rblk(n), kRT, 0, s>>>(n, deg, cand.get(), maxdeg.get());
    OBK_HIP(hipGetLastError());
    const int deg_bits = bits_for(d2h_one(maxdeg.get(), s));
    const int ub = bits_for((uint64_t)(n - 1));
    const int64_t n0 = scan_counts_i32(cand.get(), off.get(), n, s);
    if (n0 > 0) {
        k_emit<<<rblk(n), kRT, 0, s>>>(n, cand.get(), off.get(), vals.get());
        k_append<<<rblk(n0), kRT, 0, s>>>(n0, vals.get(), seq.get(), vis.get(), parent.get(), cand.get());
        OBK_HIP(hipGetLastError());
    }

    int64_t head = n0, tail = n0, levels = 0;
    bool resumed = false;
    while (tail < n) {
        if (head == tail) {   // a new component at the least (degree, index) unvisited vertex
            k_set_u64<<<1, 1, 0, s>>>(best.get(), ULLONG_MAX);
            k_argmin_unvisited<<<rblk(n), kRT, 0, s>>>(n, deg, vis.get(), best.get());
            OBK_HIP(hipGetLastError());
            const int32_t st = (int32_t)(d2h_one(best.get(), s) & 0xffffffffu);
            k_start<<<1, 1, 0, s>>>(st, seq.get() + tail, vis.get());
            tail++;
            levels++;
        }
        const int64_t nf = tail - head;
        k_zero_u32<<<1, 1, 0, s>>>(count.get());
        k_expand<<<rblk(nf), kRT, 0, s>>>(nf, seq.get() + head, gptr.get(), adj, vis.get(), parent.get(),
                                          cand.get(), vals.get(), count.get());
        OBK_HIP(hipGetLastError());
        const int64_t m = d2h_one(count.get(), s);
        const int pb = bits_for((uint64_t)(nf - 1));
        if (m > 0 && m <= kSmallLevel && pb + deg_bits + ub <= 64) {
            k_sort_append_small<<<1, kSortWG, 0, s>>>((int32_t)m, vals.get(), deg, parent.get(), cand.get(),
                                                      deg_bits, ub, seq.get() + tail, vis.get());
            OBK_HIP(hipGetLastError());
        } else if (m > 0) {
            // stable passes: (degree, index), then parent
            if (deg_bits + ub <= 32) {
                k_key_deg_index<true><<<rblk(m), kRT, 0, s>>>(m, vals.get(), deg, ub, keys.get());
                radix_sort_pairs(keys.get(), vals.get(), m, deg_bits + ub, s);
            } else {
                k_key_deg_index<false><<<rblk(m), kRT, 0, s>>>(m, vals.get(), deg, ub, keys.get());
                radix_sort_pairs(keys.get(), vals.get(), m, ub, s);
                k_key_of<false><<<rblk(m), kRT, 0, s>>>(m, vals.get(), deg, parent.get(), keys.get());
                radix_sort_pairs(keys.get(), vals.get(), m, deg_bits, s);
            }
            k_key_of<true><<<rblk(m), kRT, 0, s>>>(m, vals.get(), deg, parent.get(), keys.get());
            OBK_HIP(hipGetLastError());
            radix_sort_pairs(keys.get(), vals.get(), m, pb, s);
            k_append<<<rblk(m), kRT, 0, s>>>(m, vals.get(), seq.get() + tail, vis.get(), parent.get(), cand.get());
            OBK_HIP(hipGetLastError());
        }
        const int64_t prev = tail - head;
        head = tail;
        tail += m;
        levels++;
        // narrow levels that no longer grow fast: a level step costs about as
        // much as a few thousand vertices of the host loop
        if (give_up && tail < n && levels >= 4 && (tail - n0) < kDeviceRcmMinWidth * levels && m < 2 * prev) {
            resumed = true;
            break;
        }
    }
    std::vector<int32_t> cm(n);
    if (!resumed) {
        d2h(cm.data(), seq.get(), n, s);
    } else {
        std::vector<uint8_t> seen(n);
        std::vector<int32_t> hdeg(n), hadj(mu);
        std::vector<int64_t> hptr(n + 1, 0);
        d2h(cm.data(), seq.get(), tail, s);
        d2h(seen.data(), vis.get(), n, s);
        d2h(hdeg.data(), deg, n, s);
        d2h(hadj.data(), adj, mu, s);
        for (int64_t i = 0; i < n; i++) hptr[i + 1] = hptr[i] + hdeg[i];
        host_cm_resume(n, hptr.data(), hadj.data(), cm.data(), seen.data(), head, tail);
    }
    for (int64_t t = 0; t < n; t++) perm[t] = cm[n - 1 - t];
}

}  // namespace obk
