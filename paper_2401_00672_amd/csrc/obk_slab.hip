// Banded sweep engine: the orthogonal-group sweep (eq. 3.3 with one-row
// blocks) on a matrix whose reverse Cuthill-McKee order (Section 3.2) keeps
// every row's columns near the diagonal, run by one persistent launch per
// call in which each workgroup owns a contiguous slab of the reordered
// unknowns.
//
// Slab k owns rows and columns O_k = [a_k, b_k).  It keeps in LDS
//   - the x window H_k = [hlo_k, hhi_k): its own columns and every column
//     its rows touch (the RCM band makes this a short range around O_k);
//   - for the group g being swept, the weights w of every row of g that
//     touches a column of H_k.  These rows lie in R_k = [rlo_k, rhi_k),
//     which the plan checks to lie within the slabs k-1, k, k+1.
// A group step is
//   phase R  w_i = (f_i - sum_c a_ic x_c) / ||a_i||^2 for the own rows of g,
//            x_c read from the LDS window (ascending column order);
//   exchange the own rows' w that a neighbour needs are published to it
//            (stored by phase R itself), and the neighbours' w are
//            received (one flag per slab, raised at each step that
//            publishes);
//   phase S  x_c = x_c + sum_i w_i a_ic (ascending row order) for every
//            column of H_k that g touches: own columns, and halo columns,
//            which the owning neighbour updates identically, so the window
//            stays exact without a second exchange.  Columns whose rows are
//            all own rows are updated before the wait for the neighbours,
//            the others after it.
// A step exchanges only in the directions that carry rows, except at the
// first group of every sweep, where every pair of neighbours synchronises:
// a slab is therefore never more than one sweep ahead of a neighbour, and
// the exchange buffers, kept per (group, sweep parity), are never
// overwritten before they are read.
// Every sum runs in the oracle's order with no contraction, so the iterate
// equals the per-group phase kernels' and the oracle's bit for bit.
//
// The exchange goes through global memory with agent-scope relaxed atomic
// stores and loads (coherent across XCDs without whole-cache write-back or
// invalidation); each thread waits for its own stores to complete before
// the workgroup barrier that precedes the flag store, and readers load the
// data only after a barrier that follows the flag observation.  Waits are
// bounded: a timeout sets an error flag and every workgroup leaves.
//
// Matrix data are streamed once per phase from a plan-time layout: per
// (slab, group, phase) a list of items (a row in R, a touched column in S),
// sorted by length and cut into rounds of Q * 448 items (Q items per
// computing thread: 5 rows in R, 9 columns in S, whose items are shorter) whose
// entries are stored entry-major (ELL) with 16-bit window indices.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "obk_internal.h"

namespace obk {

namespace {

constexpr int kSlabThreads = 512;
// Wave 0 of a workgroup runs the neighbour exchange (flag, wait, receive)
// while the other waves sweep the interior columns; those waves run every
// phase, and phase R publishes the rows the neighbours need.
constexpr int kCommThreads = 64, kCompThreads = kSlabThreads - kCommThreads;
constexpr int kQR = 5, kKPR = 6;                     // phase R: rows per thread per round, entries per pass
constexpr int kQS = 9, kKPS = 4;                     // phase S: columns per thread per round, entries per pass
__host__ __device__ constexpr int phase_qt(bool isR) { return (isR ? kQR : kQS) * kCompThreads; }
constexpr int kFlagStride = 32;                      // one flag per 128-byte line
constexpr long kSpinLimit = 1L << 22;                // polls before a wait gives up

__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Byte layout of a phase copied to the LDS cache (offsets from its block,
// doubles first so that every array stays aligned): f per item (R only), the
// entry values, then the 16-bit item targets, lengths and entry indices.
struct CacheLayout {
    int32_t f, val, tgt, len, idx, bytes;
};
__host__ __device__ __forceinline__ CacheLayout cache_layout(bool isR, int32_t count, int32_t ents) {
    CacheLayout c;
    c.f = 0;
    c.val = isR ? 8 * count : 0;
    c.tgt = c.val + 8 * ents;
    c.len = c.tgt + 2 * count;
    c.idx = c.len + 2 * count;
    c.bytes = (c.idx + 2 * ents + 15) & ~15;
    return c;
}

// Registers of one round: per item (Q per thread) its slot, length, f and
// ||a||^2 (R, summed from the row's entries) and running sum; one pass of
// KP entries each.
template <int Q, int KP>
struct RoundRegs {
    bool act[Q];
    int tg[Q], ln[Q];
    double fa[Q], nu[Q], acc[Q];
    int ix[Q][KP];
    double v[Q][KP];
};

// Where phase R also stores the w of the own rows a neighbour's window
// needs: slots [lo0, lo1) of the w window go to lo[slot - lo0] (for k-1),
// slots [hi0, hi1) to hi[slot - hi0] (for k+1); empty ranges store nothing.
struct PubRange {
    double* lo;
    double* hi;
    int lo0, lo1, hi0, hi1;
};

// The global arrays a streamed phase reads its items and entries from.
struct PhaseSrc {
    const uint16_t* tgt;
    const uint16_t* len;
    const double* f;
    const uint16_t* idx;
    const double* val;
};

template <bool kR, int Q, int KP>
__device__ __forceinline__ void round_items(const PhaseSrc& s, const SlabPhase& ph, int r, int nr,
                                            RoundRegs<Q, KP>& R) {
    const int t = (int)threadIdx.x - kCommThreads;
    const int64_t io = ph.item_off + (int64_t)r * phase_qt(kR);
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int j = q * kCompThreads + t;
        R.act[q] = j < nr;
        R.tg[q] = 0;
        R.ln[q] = 0;
        R.fa[q] = 0.0;
        R.nu[q] = 0.0;
        R.acc[q] = 0.0;
        if (R.act[q]) {
            R.tg[q] = s.tgt[io + j];
            R.ln[q] = s.len[io + j];
            if (kR) R.fa[q] = s.f[io + j];
        }
    }
}

template <int Q, int KP>
__device__ __forceinline__ void round_entries(const PhaseSrc& s, int64_t ent_off, int K, int nr, int e0,
                                              RoundRegs<Q, KP>& R) {
    const int t = (int)threadIdx.x - kCommThreads;
    const int64_t eo = ent_off;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int j = q * kCompThreads + t;
#pragma unroll
        for (int e = 0; e < KP; e++) {
            R.ix[q][e] = 0;
            R.v[q][e] = 0.0;
            if (R.act[q] & (e0 + e < K)) {
                const int64_t at = eo + (int64_t)(e0 + e) * nr + j;
                R.ix[q][e] = s.idx[at];
                R.v[q][e] = s.val[at];
            }
        }
    }
}

// Phase R also sums each row's ||a||^2 from its entries, in the same order
// as the plan's norms (ascending column, no contraction).
template <bool kR, int Q, int KP>
__device__ __forceinline__ void round_accumulate(RoundRegs<Q, KP>& R, int e0, const double* src) {
#pragma unroll
    for (int q = 0; q < Q; q++)
#pragma unroll
        for (int e = 0; e < KP; e++)
            if (e0 + e < R.ln[q]) {
                R.acc[q] = R.acc[q] + R.v[q][e] * src[R.ix[q][e]];
                if (kR) R.nu[q] = R.nu[q] + R.v[q][e] * R.v[q][e];
            }
}

// The rest of round r once its items and first entry pass are in R: the
// other passes, then the writes.  R writes w = (f - sum) * inv into dst (the
// w window) at each item's slot; S adds the sum into dst (the x window) at
// each item's column.  src is the window the entries index (x in R, w in
// S); the oracle's product a * v commutes exactly.
template <bool kR, int Q, int KP>
__device__ __forceinline__ void finish_round(const PhaseSrc& s, const SlabRound& rd, int nr, const double* src,
                                             double* dst, RoundRegs<Q, KP>& R, double omega, const PubRange& pb) {
    const int K = __builtin_amdgcn_readfirstlane(rd.K);
    round_accumulate<kR>(R, 0, src);
    for (int e0 = KP; e0 < K; e0 += KP) {
        round_entries(s, rd.ent_off, K, nr, e0, R);
        round_accumulate<kR>(R, e0, src);
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
        if (R.act[q]) {
            if (kR) {
                const double wv = ((R.fa[q] - R.acc[q]) * (1.0 / R.nu[q])) * omega;
                const int tg = R.tg[q];
                dst[tg] = wv;
                if ((tg >= pb.lo0) & (tg < pb.lo1)) st_agent(pb.lo + (tg - pb.lo0), wv);
                if ((tg >= pb.hi0) & (tg < pb.hi1)) st_agent(pb.hi + (tg - pb.hi0), wv);
            } else {
                dst[R.tg[q]] = dst[R.tg[q]] + R.acc[q];
            }
        }
}

// Rounds [r0, nrounds) of a streamed phase (run by the computing threads,
// t >= kCommThreads).  rounds are the slab's rounds in
// LDS (index minus the slab's first).
template <bool kR>
__device__ __forceinline__ void run_phase(const PhaseSrc& s, const SlabPhase& ph, const SlabRound* rounds,
                                          int32_t round_first, const double* src, double* dst, double omega,
                                          const PubRange& pb) {
    constexpr int Q = kR ? kQR : kQS, KP = kR ? kKPR : kKPS;
    RoundRegs<Q, KP> R;
    for (int r = 0; r < ph.nrounds; r++) {
        const SlabRound& rd = rounds[ph.round0 + r - round_first];
        const int nr = min(phase_qt(kR), ph.count - r * phase_qt(kR));
        round_items<kR, Q, KP>(s, ph, r, nr, R);
        round_entries<Q, KP>(s, rd.ent_off, __builtin_amdgcn_readfirstlane(rd.K), nr, 0, R);
        finish_round<kR, Q, KP>(s, rd, nr, src, dst, R, omega, pb);
    }
}

// A phase whose items and entries were copied to its LDS block: the same
// arithmetic, reading one entry at a time (LDS latency is short, and no
// register arrays are held).
template <bool kR>
__device__ __forceinline__ void run_cached(const char* b, const SlabPhase& ph, const SlabRound* rounds,
                                           int32_t round_first, const double* src, double* dst, double omega,
                                           const PubRange& pb) {
    const CacheLayout c = cache_layout(kR, ph.count, ph.ents);
    const uint16_t* tgt = reinterpret_cast<const uint16_t*>(b + c.tgt);
    const uint16_t* len = reinterpret_cast<const uint16_t*>(b + c.len);
    const double* f = reinterpret_cast<const double*>(b + c.f);
    const uint16_t* idx = reinterpret_cast<const uint16_t*>(b + c.idx);
    const double* val = reinterpret_cast<const double*>(b + c.val);
    const int t = (int)threadIdx.x - kCommThreads;
    const int64_t ebase = ph.nrounds ? rounds[ph.round0 - round_first].ent_off : 0;
    for (int r = 0; r < ph.nrounds; r++) {
        const SlabRound& rd = rounds[ph.round0 + r - round_first];
        const int nr = min(phase_qt(kR), ph.count - r * phase_qt(kR));
        const int64_t eo = rd.ent_off - ebase;
        for (int j = t; j < nr; j += kCompThreads) {
            const int li = r * phase_qt(kR) + j;
            const int ln = len[li];
            double acc = 0.0, nu = 0.0;
            for (int e = 0; e < ln; e++) {
                const int64_t at = eo + (int64_t)e * nr + j;
                const double v = val[at];
                acc = acc + v * src[idx[at]];
                if (kR) nu = nu + v * v;
            }
            if (kR) {
                const double wv = ((f[li] - acc) * (1.0 / nu)) * omega;
                const int tg = tgt[li];
                dst[tg] = wv;
                if ((tg >= pb.lo0) & (tg < pb.lo1)) st_agent(pb.lo + (tg - pb.lo0), wv);
                if ((tg >= pb.hi0) & (tg < pb.hi1)) st_agent(pb.hi + (tg - pb.hi0), wv);
            } else {
                dst[tgt[li]] = dst[tgt[li]] + acc;
            }
        }
    }
}

// The communication wave's copy of a neighbour's published values into the
// w window, kCommBatch values per lane in flight.
constexpr int kCommBatch = 16;
__device__ __forceinline__ void comm_receive(double* dst, const double* src, int n, int t) {
    for (int base = 0; base < n; base += kCommBatch * kCommThreads) {
        double v[kCommBatch];
#pragma unroll
        for (int m = 0; m < kCommBatch; m++) {
            const int i = base + m * kCommThreads + t;
            v[m] = i < n ? ld_agent(src + i) : 0.0;
        }
#pragma unroll
        for (int m = 0; m < kCommBatch; m++) {
            const int i = base + m * kCommThreads + t;
            if (i < n) dst[i] = v[m];
        }
    }
}

// Zero the step flags and the error flag before a launch (a kernel rather
// than a memset, so that the pair can be captured in a graph).
__global__ void k_slab_reset(int32_t S, uint32_t* flags, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) flags[(int64_t)i * kFlagStride] = 0u;
    if (i == 0) err[0] = 0;
}

struct SlabArgs {
    const SlabDesc* desc;
    const SlabGroup* grp;
    const SlabRound* rounds;
    const uint16_t* tgt;
    const uint16_t* len;
    const double* f;
    const uint16_t* idx;
    const double* val;
    double* xbuf;
    uint32_t* flags;
    int* err;
    int64_t cap;
    int32_t S, G;
    int32_t wwin_off;        // LDS offsets in doubles (w window) and bytes (descriptors, cache)
    int32_t meta_off, cache_off;
    double omega;            // relaxation of the row steps
};

__device__ __forceinline__ PhaseSrc global_src(const SlabArgs& a) {
    return PhaseSrc{a.tgt, a.len, a.f, a.idx, a.val};
}

// copy a phase's items and entries into its LDS block
template <bool kR>
__device__ __forceinline__ void cache_fill(const SlabArgs& a, char* cache, const SlabPhase& ph,
                                           const SlabRound* rounds, int32_t round_first) {
    if (ph.cache < 0 || ph.count == 0) return;
    const CacheLayout c = cache_layout(kR, ph.count, ph.ents);
    char* b = cache + ph.cache;
    const int64_t e0 = rounds[ph.round0 - round_first].ent_off;
    for (int i = threadIdx.x; i < ph.count; i += kSlabThreads) {
        reinterpret_cast<uint16_t*>(b + c.tgt)[i] = a.tgt[ph.item_off + i];
        reinterpret_cast<uint16_t*>(b + c.len)[i] = a.len[ph.item_off + i];
        if (kR) reinterpret_cast<double*>(b + c.f)[i] = a.f[ph.item_off + i];
    }
    for (int i = threadIdx.x; i < ph.ents; i += kSlabThreads) {
        reinterpret_cast<uint16_t*>(b + c.idx)[i] = a.idx[e0 + i];
        reinterpret_cast<double*>(b + c.val)[i] = a.val[e0 + i];
    }
}

__global__ __launch_bounds__(kSlabThreads) void k_slab_sweeps(SlabArgs a, int64_t sweeps, double* x) {
    extern __shared__ double lds[];
    double* xw = lds;
    double* ww = lds + a.wwin_off;
    char* lb = reinterpret_cast<char*>(lds);
    SlabGroup* gl = reinterpret_cast<SlabGroup*>(lb + a.meta_off);
    SlabRound* rl = reinterpret_cast<SlabRound*>(lb + a.meta_off + (int64_t)a.G * sizeof(SlabGroup));
    char* cache = lb + a.cache_off;
    __shared__ int bail;
    const int k = blockIdx.x, t = threadIdx.x, G = a.G, S = a.S;
    const SlabDesc d = a.desc[k];
    for (int j = t; j < d.xcount; j += kSlabThreads) xw[j] = x[(int64_t)d.xlo + j];
    for (int g = t; g < G; g += kSlabThreads) gl[g] = a.grp[(int64_t)k * G + g];
    for (int r = t; r < d.round_count; r += kSlabThreads) rl[r] = a.rounds[d.round_first + r];
    if (t == 0) bail = 0;
    __syncthreads();
    for (int g = 0; g < G; g++) {
        cache_fill<true>(a, cache, gl[g].r, rl, d.round_first);
        cache_fill<false>(a, cache, gl[g].s, rl, d.round_first);
        cache_fill<false>(a, cache, gl[g].sb, rl, d.round_first);
    }
    __syncthreads();
    // exchange buffers: [slab][0: prefix for k-1, 1: suffix for k+1][sweep parity], each
    // holding every group's values at the group's offset
    auto buf = [&](int slab, int dir, int g, int par) {
        return a.xbuf + (((int64_t)slab * 2 + dir) * 2 + par) * a.cap + gl[g].xoff;
    };
    const bool comp = t >= kCommThreads;
    for (int64_t sw = 0; sw < sweeps; sw++) {
        for (int g = 0; g < G; g++) {
            const uint32_t step = (uint32_t)(sw * G + g) + 1u;
            const int par = (int)(sw & 1);
            const SlabGroup& gd = gl[g];
            const bool sync = g == 0;
            const bool send = sync | (gd.pre_cnt > 0) | (gd.suf_cnt > 0);
            // phase R of the own rows of g; the first pre_cnt own rows also go
            // to the buffer k-1 reads and the last suf_cnt to the one k+1
            // reads, and each wave waits for its stores before the barrier
            if (comp) {
                const int own0 = gd.lo_cnt, own1 = gd.lo_cnt + gd.own_cnt;
                const PubRange pb{buf(k, 0, g, par), buf(k, 1, g, par), own0, own0 + gd.pre_cnt,
                                  own1 - gd.suf_cnt, own1};
                if (gd.r.cache >= 0)
                    run_cached<true>(cache + gd.r.cache, gd.r, rl, d.round_first, xw, ww, a.omega, pb);
                else
                    run_phase<true>(global_src(a), gd.r, rl, d.round_first, xw, ww, a.omega, pb);
                __builtin_amdgcn_s_waitcnt(0);
            }
            __syncthreads();
            if (!comp) {
                // wave 0: the published values are stored and complete (every
                // computing wave waited for its stores before the barrier):
                // raise the flag, wait for the neighbours' and receive k-1's
                // suffix before the own rows and k+1's prefix after them
                // (every pair of neighbours meets at the first group of a sweep)
                if (send) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // the flag stays after the barrier
                    if (t == 0)
                        __hip_atomic_store(a.flags + (int64_t)k * kFlagStride, step, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                const int nb = (t == 0) ? k - 1 : k + 1;
                const bool need = (t == 0) ? (sync | (gd.lo_cnt > 0)) : (sync | (gd.hi_cnt > 0));
                bool late = false;
                if ((t < 2) & (nb >= 0) & (nb < S) & need) {
                    const uint32_t* fl = a.flags + (int64_t)nb * kFlagStride;
                    long spins = 0;
#pragma clang loop unroll(disable)
                    while (__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < step) {
                        if (++spins > kSpinLimit) {
                            late = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // the data loads follow the wait
                if (__any(late)) {
                    if (t == 0) {
                        atomicOr(a.err, 1);
                        bail = 1;
                    }
                } else {
                    if (gd.lo_cnt) comm_receive(ww, buf(k - 1, 1, g, par), gd.lo_cnt, t);
                    if (gd.hi_cnt) comm_receive(ww + gd.lo_cnt + gd.own_cnt, buf(k + 1, 0, g, par), gd.hi_cnt, t);
                }
            } else {
                // the other waves: the columns whose rows are all own rows,
                // which need no neighbour
                if (gd.s.cache >= 0) run_cached<false>(cache + gd.s.cache, gd.s, rl, d.round_first, ww, xw, a.omega, PubRange{});
                else run_phase<false>(global_src(a), gd.s, rl, d.round_first, ww, xw, a.omega, PubRange{});
            }
            __syncthreads();
            if (bail) return;
            // phase S over the window columns with halo rows
            if (comp) {
                if (gd.sb.cache >= 0) run_cached<false>(cache + gd.sb.cache, gd.sb, rl, d.round_first, ww, xw, a.omega, PubRange{});
                else run_phase<false>(global_src(a), gd.sb, rl, d.round_first, ww, xw, a.omega, PubRange{});
            }
            __syncthreads();
        }
    }
    for (int j = t; j < d.own_cnt; j += kSlabThreads) x[(int64_t)d.xlo + d.own_lo + j] = xw[d.own_lo + j];
}

// ------------------------------------------------------------ plan time
template <class T> void upload(DevArray<T>& d, const std::vector<T>& h, hipStream_t s) {
    d.alloc(h.size());
    if (!h.empty()) OBK_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T> std::vector<T> download(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) OBK_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    return h;
}

// slab boundaries and windows for S slabs of (near) equal width
struct SlabGeom {
    std::vector<int64_t> a;           // [S+1] own ranges
    std::vector<int64_t> hlo, hhi;    // x windows
    std::vector<int64_t> rlo, rhi;    // rows touching a window column
};

// The geometry of S slabs, or false when a slab's window rows reach past its
// neighbours or a window exceeds 16-bit indices.
bool slab_geometry(int64_t n, int32_t S, const std::vector<int64_t>& rowmin, const std::vector<int64_t>& rowmax,
                   const std::vector<int64_t>& colmin, const std::vector<int64_t>& colmax, SlabGeom& sg) {
    sg.a.assign(S + 1, 0);
    for (int32_t k = 0; k <= S; k++) sg.a[k] = (int64_t)((__int128)n * k / S);
    sg.hlo.assign(S, 0); sg.hhi.assign(S, 0); sg.rlo.assign(S, 0); sg.rhi.assign(S, 0);
    for (int32_t k = 0; k < S; k++) {
        const int64_t a = sg.a[k], b = sg.a[k + 1];
        if (b <= a) return false;
        int64_t hlo = a, hhi = b;
        for (int64_t i = a; i < b; i++)
            if (rowmin[i] <= rowmax[i]) { hlo = std::min(hlo, rowmin[i]); hhi = std::max(hhi, rowmax[i] + 1); }
        int64_t rlo = a, rhi = b;
        for (int64_t c = hlo; c < hhi; c++)
            if (colmin[c] <= colmax[c]) { rlo = std::min(rlo, colmin[c]); rhi = std::max(rhi, colmax[c] + 1); }
        const int64_t lo_ok = k > 0 ? sg.a[k - 1] : 0, hi_ok = k + 1 < S ? sg.a[k + 2] : n;
        if (rlo < lo_ok || rhi > hi_ok) return false;
        if (hhi - hlo > 65535 || rhi - rlo > 65535) return false;
        sg.hlo[k] = hlo; sg.hhi[k] = hhi; sg.rlo[k] = rlo; sg.rhi[k] = rhi;
    }
    return true;
}

}  // namespace

// Host image of the banded engine's data (built on the host, uploaded by
// slab_setup, and run on the host by slab_emulate in the CPU tests).
struct SlabHost {
    int32_t S = 0, G = 0;
    int64_t xmax = 0, wmax = 0, cap = 1;
    int64_t meta_bytes = 0, cache_bytes = 0;   // LDS: descriptors and rounds, cached phases (per slab, max)
    double bytes = 0;                 // streamed per sweep
    double bytes_launch = 0;          // read once per launch (windows, descriptors, cached phases)
    std::string why;                  // why the engine does not apply (S = 0)
    std::vector<SlabDesc> desc;
    std::vector<SlabGroup> grp;
    std::vector<SlabRound> rounds;
    std::vector<uint16_t> tgt, len, idx;
    std::vector<double> f, inv, val;
};

// Build the banded engine's data for the group-major system (gptr: group
// row ranges; hrptr/col/val: group-major CSR with reordered column ids;
// rf/rinv: f~ and 1/||a||^2 per group-major row; grow: reordered row of each
// group-major row).  forced_S > 0 tries that slab count only.
SlabHost slab_build(int64_t n, int32_t G, const std::vector<int64_t>& gptr, const std::vector<int64_t>& hrptr,
                    const std::vector<int32_t>& grow, const std::vector<int32_t>& col, const std::vector<double>& val,
                    const std::vector<double>& rf, const std::vector<double>& rinv, int64_t bandwidth, int cus,
                    int64_t lds_budget, int32_t forced_S) {
    SlabHost h;
    const int64_t m = gptr[G];
    if (n < 1 || m < 1 || G < 1) { h.why = "empty system"; return h; }
    if (G > kSlabMaxGroups) { h.why = "too many groups"; return h; }
    const int64_t bw = std::max<int64_t>(bandwidth, 1);
    // per reordered row: column range; per column: row range (active rows)
    std::vector<int64_t> rowmin(n, n), rowmax(n, -1), colmin(n, n), colmax(n, -1);
    for (int64_t p = 0; p < m; p++) {
        const int64_t i = grow[p];
        for (int64_t e = hrptr[p]; e < hrptr[p + 1]; e++) {
            const int64_t c = col[e];
            rowmin[i] = std::min(rowmin[i], c); rowmax[i] = std::max(rowmax[i], c);
            colmin[c] = std::min(colmin[c], i); colmax[c] = std::max(colmax[c], i);
        }
    }
    // the most slabs (at most one per CU) whose windows fit
    SlabGeom sg;
    int32_t S = forced_S > 0 ? forced_S
                             : (int32_t)std::min<int64_t>(cus, std::max<int64_t>(1, n / std::max<int64_t>(2 * bw, 256)));
    bool ok = false;
    while (S >= 1) {
        if (S <= n && slab_geometry(n, S, rowmin, rowmax, colmin, colmax, sg)) {
            int64_t xmax = 0, wmax = 0;
            for (int32_t k = 0; k < S; k++) xmax = std::max(xmax, sg.hhi[k] - sg.hlo[k]);
            for (int32_t g = 0; g < G; g++) {
                const int32_t* gb = grow.data() + gptr[g];
                const int32_t* ge = grow.data() + gptr[g + 1];
                for (int32_t k = 0; k < S; k++)
                    wmax = std::max<int64_t>(wmax, std::lower_bound(gb, ge, (int32_t)sg.rhi[k]) -
                                                       std::lower_bound(gb, ge, (int32_t)sg.rlo[k]));
            }
            if ((xmax + wmax) * 8 + (int64_t)G * (int64_t)sizeof(SlabGroup) + 4096 <= lds_budget) {
                ok = true; h.xmax = xmax; h.wmax = wmax; break;
            }
        }
        if (forced_S > 0) break;
        S = (S > 8) ? S * 3 / 4 : S - 1;
    }
    if (!ok) { h.why = "no slab count whose windows fit"; return h; }

    h.S = S;
    h.G = G;
    h.desc.resize(S);
    h.grp.resize((size_t)S * G);
    std::vector<uint16_t> s_tgt, s_len;      // S items, appended after the R items
    struct Item { int32_t len; int32_t tgt; int64_t src; };

    // items of one phase: sort by length (descending, stable), cut into
    // rounds, lay the entries out entry-major within each round
    auto emit = [&](std::vector<Item>& items, bool isR, const std::vector<int32_t>& pidx,
                    const std::vector<double>& pval, const std::vector<int64_t>& pstart, SlabPhase& ph) {
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.len > y.len; });
        ph.count = (int32_t)items.size();
        ph.round0 = (int32_t)h.rounds.size();
        const int64_t qt = phase_qt(isR);
        ph.nrounds = (int32_t)((items.size() + qt - 1) / qt);
        ph.item_off = isR ? (int64_t)h.tgt.size() : (int64_t)s_tgt.size();
        ph.ents = 0;
        ph.cache = -1;
        ph.pad = 0;
        for (int32_t r = 0; r < ph.nrounds; r++) {
            const size_t b = (size_t)r * qt, e = std::min(items.size(), b + (size_t)qt);
            const int64_t nr = (int64_t)(e - b);
            SlabRound rd;
            rd.K = items[b].len;
            rd.pad = 0;
            rd.ent_off = (int64_t)h.idx.size();
            h.idx.resize(h.idx.size() + (size_t)rd.K * nr, 0);
            h.val.resize(h.val.size() + (size_t)rd.K * nr, 0.0);
            for (size_t j = b; j < e; j++) {
                const Item& it = items[j];
                for (int32_t q = 0; q < it.len; q++) {
                    const size_t at = (size_t)rd.ent_off + (size_t)q * nr + (j - b);
                    h.idx[at] = (uint16_t)pidx[pstart[it.src] + q];
                    h.val[at] = pval[pstart[it.src] + q];
                }
            }
            h.rounds.push_back(rd);
            h.bytes += (double)rd.K * nr * 10.0;
            ph.ents += (int32_t)(rd.K * nr);
        }
        for (const Item& it : items) {
            if (isR) {
                h.tgt.push_back((uint16_t)it.tgt);
                h.len.push_back((uint16_t)it.len);
                h.f.push_back(rf[it.src]);
                h.inv.push_back(rinv[it.src]);     // kept on the host for the emulation's check
                h.bytes += 12.0;
            } else {
                s_tgt.push_back((uint16_t)it.tgt);
                s_len.push_back((uint16_t)it.len);
                h.bytes += 4.0;
            }
        }
    };

    std::vector<int32_t> rloc(col.size());
    for (int32_t k = 0; k < S; k++) {
        const int64_t a = sg.a[k], b = sg.a[k + 1], hlo = sg.hlo[k], hhi = sg.hhi[k];
        h.desc[k].xlo = (int32_t)hlo;
        h.desc[k].xcount = (int32_t)(hhi - hlo);
        h.desc[k].own_lo = (int32_t)(a - hlo);
        h.desc[k].own_cnt = (int32_t)(b - a);
        h.desc[k].round_first = (int32_t)h.rounds.size();
        h.desc[k].cache_bytes = 0;
        h.desc[k].pad = 0;
        for (int32_t g = 0; g < G; g++) {
            SlabGroup& gd = h.grp[(size_t)k * G + g];
            std::memset(&gd, 0, sizeof(gd));
            const int32_t* gb = grow.data() + gptr[g];
            const int32_t* ge = grow.data() + gptr[g + 1];
            auto at = [&](int64_t i) { return (int64_t)(std::lower_bound(gb, ge, (int32_t)i) - grow.data()); };
            const int64_t wlo = at(sg.rlo[k]), plo = at(a), phi = at(b), whi = at(sg.rhi[k]);
            gd.lo_cnt = (int32_t)(plo - wlo);
            gd.own_cnt = (int32_t)(phi - plo);
            gd.hi_cnt = (int32_t)(whi - phi);
            // R: own rows of g, columns as window positions
            std::vector<Item> items;
            items.reserve((size_t)(phi - plo));
            for (int64_t p = plo; p < phi; p++) {
                for (int64_t e = hrptr[p]; e < hrptr[p + 1]; e++) rloc[e] = (int32_t)(col[e] - hlo);
                items.push_back({(int32_t)(hrptr[p + 1] - hrptr[p]), (int32_t)(gd.lo_cnt + (p - plo)), p});
            }
            emit(items, true, rloc, val, hrptr, gd.r);
            // S: window columns touched by rows of g in the w window, each
            // column's entries by ascending row (counting sort by column)
            const int64_t xc = hhi - hlo;
            std::vector<int64_t> cnt(xc + 1, 0);
            for (int64_t p = wlo; p < whi; p++)
                for (int64_t e = hrptr[p]; e < hrptr[p + 1]; e++)
                    if (col[e] >= hlo && col[e] < hhi) cnt[col[e] - hlo + 1]++;
            for (int64_t c = 0; c < xc; c++) cnt[c + 1] += cnt[c];
            std::vector<int32_t> sidx(cnt[xc]);
            std::vector<double> sval(cnt[xc]);
            std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
            for (int64_t p = wlo; p < whi; p++)
                for (int64_t e = hrptr[p]; e < hrptr[p + 1]; e++)
                    if (col[e] >= hlo && col[e] < hhi) {
                        const int64_t q = fillp[col[e] - hlo]++;
                        sidx[q] = (int32_t)(p - wlo);
                        sval[q] = val[e];
                    }
            // columns whose rows are all own rows (w slots [lo_cnt, lo_cnt + own_cnt))
            // need no neighbour; the others wait for the exchange
            items.clear();
            std::vector<Item> bitems;
            for (int64_t c = 0; c < xc; c++) {
                if (cnt[c + 1] == cnt[c]) continue;
                bool own_only = true;
                for (int64_t q = cnt[c]; q < cnt[c + 1]; q++)
                    own_only = own_only && sidx[q] >= gd.lo_cnt && sidx[q] < gd.lo_cnt + gd.own_cnt;
                (own_only ? items : bitems).push_back({(int32_t)(cnt[c + 1] - cnt[c]), (int32_t)c, c});
            }
            emit(items, false, sidx, sval, cnt, gd.s);
            emit(bitems, false, sidx, sval, cnt, gd.sb);
        }
        h.desc[k].round_count = (int32_t)h.rounds.size() - h.desc[k].round_first;
        h.meta_bytes = std::max<int64_t>(h.meta_bytes, (int64_t)G * (int64_t)sizeof(SlabGroup) +
                                                           (int64_t)h.desc[k].round_count * (int64_t)sizeof(SlabRound));
        h.bytes_launch += 8.0 * (double)(hhi - hlo + (b - a)) + (double)G * sizeof(SlabGroup) +
                          (double)h.desc[k].round_count * sizeof(SlabRound);
    }
    h.meta_bytes = (h.meta_bytes + 15) & ~(int64_t)15;
    if ((h.xmax + h.wmax) * 8 + h.meta_bytes > lds_budget) {
        SlabHost none;
        none.why = "descriptors do not fit in LDS";
        return none;
    }
    // LDS cache: per slab, the smallest phases first, while they fit beside
    // the windows and descriptors; a cached phase is read once per launch
    const int64_t cache_budget = lds_budget - ((h.xmax + h.wmax) * 8 + 15) / 16 * 16 - h.meta_bytes;
    struct Cand { int64_t bytes; SlabPhase* ph; bool isR; };
    for (int32_t k = 0; k < S; k++) {
        std::vector<Cand> cand;
        for (int32_t g = 0; g < G; g++) {
            SlabGroup& gd = h.grp[(size_t)k * G + g];
            if (gd.r.count > 0) cand.push_back({cache_layout(true, gd.r.count, gd.r.ents).bytes, &gd.r, true});
            if (gd.s.count > 0) cand.push_back({cache_layout(false, gd.s.count, gd.s.ents).bytes, &gd.s, false});
            if (gd.sb.count > 0) cand.push_back({cache_layout(false, gd.sb.count, gd.sb.ents).bytes, &gd.sb, false});
        }
        std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) { return x.bytes < y.bytes; });
        int64_t used = 0;
        for (const Cand& c : cand) {
            if (used + c.bytes > cache_budget) break;
            c.ph->cache = (int32_t)used;
            used += c.bytes;
            // streamed bytes of the phase move from every sweep to the launch
            const double streamed = (double)c.ph->count * (c.isR ? 20.0 : 4.0) + (double)c.ph->ents * 10.0;
            h.bytes -= streamed;
            h.bytes_launch += streamed;
        }
        h.desc[k].cache_bytes = (int32_t)used;
        h.cache_bytes = std::max(h.cache_bytes, used);
    }
    // publication counts: what each neighbour's window takes from the own
    // rows; each group's values sit at the same offset in every buffer
    std::vector<int64_t> gcap(G, 0);
    for (int32_t k = 0; k < S; k++)
        for (int32_t g = 0; g < G; g++) {
            SlabGroup& gd = h.grp[(size_t)k * G + g];
            gd.pre_cnt = k > 0 ? h.grp[(size_t)(k - 1) * G + g].hi_cnt : 0;
            gd.suf_cnt = k + 1 < S ? h.grp[(size_t)(k + 1) * G + g].lo_cnt : 0;
            if (gd.pre_cnt > gd.own_cnt || gd.suf_cnt > gd.own_cnt)
                fail(OBK_E_HIP, "banded engine: inconsistent neighbour windows");
            gcap[g] = std::max<int64_t>(gcap[g], std::max(gd.pre_cnt, gd.suf_cnt));
            h.bytes += 16.0 * (gd.pre_cnt + gd.suf_cnt);
        }
    int64_t total_cap = 0;
    for (int32_t g = 0; g < G; g++) {
        for (int32_t k = 0; k < S; k++) h.grp[(size_t)k * G + g].xoff = (int32_t)total_cap;
        total_cap += gcap[g];
    }
    h.cap = std::max<int64_t>(1, total_cap);
    // S items follow the R items in the item arrays
    const int64_t nR = (int64_t)h.tgt.size();
    for (auto& gd : h.grp) {
        gd.s.item_off += nR;
        gd.sb.item_off += nR;
    }
    h.tgt.insert(h.tgt.end(), s_tgt.begin(), s_tgt.end());
    h.len.insert(h.len.end(), s_len.begin(), s_len.end());
    if (h.idx.empty()) { h.idx.push_back(0); h.val.push_back(0.0); }
    if (h.f.empty()) { h.f.push_back(0.0); h.inv.push_back(0.0); }
    if (h.tgt.empty()) { h.tgt.push_back(0); h.len.push_back(0); }
    return h;
}

// The banded kernel's arithmetic and exchange run on the host, step by step
// in the kernel's order (every slab's phase R, the publications, every
// slab's phase S), on x (reordered coordinates).  Cached phases are copied
// into a per-slab byte image of the LDS cache with the kernel's layout and
// read from there, the rounds from the slab's own copy.  Used by the CPU
// tests to check the builder's indexing against the oracle without a device.
void slab_emulate(const SlabHost& h, int64_t sweeps, double omega, double* x) {
    const int32_t S = h.S, G = h.G;
    std::vector<std::vector<double>> xw(S), ww(S);
    std::vector<std::vector<char>> cache(S);
    std::vector<std::vector<SlabRound>> rl(S);
    auto fill = [&](int32_t k, const SlabPhase& ph, bool isR) {
        if (ph.cache < 0 || ph.count == 0) return;
        const CacheLayout c = cache_layout(isR, ph.count, ph.ents);
        if (ph.cache + c.bytes > h.desc[k].cache_bytes) fail(OBK_E_HIP, "banded engine: cache block out of range");
        char* b = cache[k].data() + ph.cache;
        const int64_t e0 = rl[k].at(ph.round0 - h.desc[k].round_first).ent_off;
        for (int32_t i = 0; i < ph.count; i++) {
            std::memcpy(b + c.tgt + 2 * i, &h.tgt[ph.item_off + i], 2);
            std::memcpy(b + c.len + 2 * i, &h.len[ph.item_off + i], 2);
            if (isR) std::memcpy(b + c.f + 8 * i, &h.f[ph.item_off + i], 8);
        }
        for (int32_t i = 0; i < ph.ents; i++) {
            std::memcpy(b + c.idx + 2 * (int64_t)i, &h.idx[e0 + i], 2);
            std::memcpy(b + c.val + 8 * (int64_t)i, &h.val[e0 + i], 8);
        }
    };
    for (int32_t k = 0; k < S; k++) {
        xw[k].assign(x + h.desc[k].xlo, x + h.desc[k].xlo + h.desc[k].xcount);
        ww[k].assign(h.wmax, 0.0);
        cache[k].assign(h.desc[k].cache_bytes, 0);
        rl[k].assign(h.rounds.begin() + h.desc[k].round_first,
                     h.rounds.begin() + h.desc[k].round_first + h.desc[k].round_count);
        for (int32_t g = 0; g < G; g++) {
            fill(k, h.grp[(size_t)k * G + g].r, true);
            fill(k, h.grp[(size_t)k * G + g].s, false);
            fill(k, h.grp[(size_t)k * G + g].sb, false);
        }
    }
    auto phase = [&](int32_t k, const SlabPhase& ph, bool isR, const std::vector<double>& src,
                     std::vector<double>& dst) {
        const bool cached = ph.cache >= 0;
        const CacheLayout c = cache_layout(isR, ph.count, ph.ents);
        const char* b = cached ? cache[k].data() + ph.cache : nullptr;
        const int64_t ebase = (cached && ph.nrounds) ? rl[k].at(ph.round0 - h.desc[k].round_first).ent_off : 0;
        auto rd16 = [&](const char* p, int64_t i) { uint16_t v; std::memcpy(&v, p + 2 * i, 2); return v; };
        auto rd64 = [&](const char* p, int64_t i) { double v; std::memcpy(&v, p + 8 * i, 8); return v; };
        for (int32_t r = 0; r < ph.nrounds; r++) {
            const SlabRound& rd = rl[k].at(ph.round0 + r - h.desc[k].round_first);
            const int64_t qt = phase_qt(isR);
            const int64_t nr = std::min<int64_t>(qt, ph.count - (int64_t)r * qt);
            for (int64_t j = 0; j < nr; j++) {
                const int64_t it = ph.item_off + (int64_t)r * qt + j;
                const int64_t li = it - ph.item_off;
                const int ln = cached ? rd16(b + c.len, li) : h.len.at(it);
                double acc = 0.0, nu = 0.0;
                for (int32_t e = 0; e < ln; e++) {
                    const int64_t at = rd.ent_off + (int64_t)e * nr + j;
                    const double v = cached ? rd64(b + c.val, at - ebase) : h.val.at(at);
                    const int ix = cached ? rd16(b + c.idx, at - ebase) : h.idx.at(at);
                    acc = acc + v * src.at(ix);
                    nu = nu + v * v;
                }
                const int tg = cached ? rd16(b + c.tgt, li) : h.tgt.at(it);
                if (isR) {
                    const double fa = cached ? rd64(b + c.f, li) : h.f.at(it);
                    const double ia = 1.0 / nu;
                    // the engine's 1/||a||^2, formed from the row's entries,
                    // is the plan's (and the oracle's) bit for bit
                    if (ia != h.inv.at(it))
                        fail(OBK_E_ARG, "banded engine: a row's 1/||a||^2 differs from the given one");
                    dst.at(tg) = ((fa - acc) * ia) * omega;
                } else {
                    dst.at(tg) = dst.at(tg) + acc;
                }
            }
        }
    };
    for (int64_t sw = 0; sw < sweeps; sw++)
        for (int32_t g = 0; g < G; g++) {
            for (int32_t k = 0; k < S; k++) phase(k, h.grp[(size_t)k * G + g].r, true, xw[k], ww[k]);
            std::vector<std::vector<double>> pre(S), suf(S);
            for (int32_t k = 0; k < S; k++) {
                const SlabGroup& gd = h.grp[(size_t)k * G + g];
                pre[k].assign(ww[k].begin() + gd.lo_cnt, ww[k].begin() + gd.lo_cnt + gd.pre_cnt);
                suf[k].assign(ww[k].begin() + gd.lo_cnt + gd.own_cnt - gd.suf_cnt, ww[k].begin() + gd.lo_cnt + gd.own_cnt);
            }
            for (int32_t k = 0; k < S; k++) {
                const SlabGroup& gd = h.grp[(size_t)k * G + g];
                for (int32_t i = 0; i < gd.lo_cnt; i++) ww[k].at(i) = suf.at(k - 1).at(i);
                for (int32_t i = 0; i < gd.hi_cnt; i++) ww[k].at(gd.lo_cnt + gd.own_cnt + i) = pre.at(k + 1).at(i);
            }
            for (int32_t k = 0; k < S; k++) {
                phase(k, h.grp[(size_t)k * G + g].s, false, ww[k], xw[k]);
                phase(k, h.grp[(size_t)k * G + g].sb, false, ww[k], xw[k]);
            }
        }
    for (int32_t k = 0; k < S; k++)
        for (int32_t j = 0; j < h.desc[k].own_cnt; j++) x[h.desc[k].xlo + h.desc[k].own_lo + j] = xw[k][h.desc[k].own_lo + j];
}

// Build the banded engine's data for a real FP64 plan when its RCM band is
// narrow enough; otherwise leave P.slab_S = 0 (the per-group phase kernels
// run).  hrptr: group-major row offsets; grow: reordered row of each
// group-major row.
void slab_setup(obk_plan_s& P, const std::vector<int64_t>& hrptr, const std::vector<int32_t>& grow,
                const std::vector<int32_t>& pos, hipStream_t s) {
    (void)pos;
    P.slab_S = 0;
    const int mode = P.opts.sweep_kernel;
    // FP32 refinement plans sweep with the phase kernels (FP32 arithmetic);
    // their FP64 sweeps, after a switch of precision, do too
    if (mode == 1 || P.cplx || P.block_form() || P.opts.precision != OBK_FP64) return;
    auto reject = [&](const std::string& why) {
        if (mode == 2) fail(OBK_E_ARG, "sweep_kernel = 2: the banded engine does not apply: " + why);
    };
    int dev = 0, cus = 0, max_lds = 0;
    OBK_HIP(hipGetDevice(&dev));
    OBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    OBK_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t lds_budget = std::min<int64_t>(max_lds, 160 * 1024) - 1024;   // static LDS and slack
    // quick rejection without the download: a window pair of a single slab
    // of a scattered matrix is the whole system
    if (std::min<int64_t>(P.n, 4 * std::max<int64_t>(P.bandwidth, 1) + 1) * 16 > lds_budget)
        return reject("band too wide for the LDS windows");
    const int64_t m = P.m;
    if (m < 1) return reject("empty system");
    const std::vector<int32_t> col = download(P.rcol.get(), (size_t)hrptr[m], s);
    const std::vector<double> val = download(P.rval.get(), (size_t)hrptr[m], s);
    const std::vector<double> rf = download(P.rf.get(), (size_t)m, s);
    const std::vector<double> rinv = download(P.rinv.get(), (size_t)m, s);
    SlabHost h = slab_build(P.n, P.ngroups, P.h_gptr, hrptr, grow, col, val, rf, rinv, P.bandwidth, cus, lds_budget,
                            0);
    if (!h.S) return reject(h.why);
    // LDS: x window, w window, descriptors and rounds, cached phases
    const int64_t meta_off = ((h.xmax + h.wmax) * 8 + 15) / 16 * 16;
    const int64_t cache_off = meta_off + h.meta_bytes;
    const int64_t lds = cache_off + h.cache_bytes;
    OBK_HIP(hipFuncSetAttribute((const void*)k_slab_sweeps, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int occ = 0;
    OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_slab_sweeps, kSlabThreads, (size_t)lds));
    if ((int64_t)occ * cus < h.S) return reject("slabs not co-resident");
    upload(P.sl_desc, h.desc, s);
    upload(P.sl_grp, h.grp, s);
    upload(P.sl_round, h.rounds, s);
    upload(P.sl_tgt, h.tgt, s);
    upload(P.sl_len, h.len, s);
    upload(P.sl_f, h.f, s);
    upload(P.sl_idx, h.idx, s);
    upload(P.sl_val, h.val, s);
    P.sl_xbuf.alloc((size_t)h.S * 4 * h.cap);
    P.sl_flags.alloc((size_t)h.S * kFlagStride);
    P.sl_err.alloc(1);
    OBK_HIP(hipMemsetAsync(P.sl_flags.get(), 0, (size_t)h.S * kFlagStride * sizeof(uint32_t), s));
    OBK_HIP(hipMemsetAsync(P.sl_err.get(), 0, sizeof(int), s));
    OBK_HIP(hipStreamSynchronize(s));
    P.slab_xmax = h.xmax;
    P.slab_wmax = h.wmax;
    P.slab_cap = h.cap;
    P.slab_lds = lds;
    P.slab_meta_off = meta_off;
    P.slab_cache_off = cache_off;
    P.slab_bytes_per_sweep = h.bytes;
    P.slab_bytes_per_launch = h.bytes_launch;
    P.slab_S = h.S;
}

static SlabArgs slab_args(obk_plan_s& P) {
    SlabArgs a;
    a.desc = P.sl_desc.get();
    a.grp = P.sl_grp.get();
    a.rounds = P.sl_round.get();
    a.tgt = P.sl_tgt.get();
    a.len = P.sl_len.get();
    a.f = P.sl_f.get();
    a.idx = P.sl_idx.get();
    a.val = P.sl_val.get();
    a.xbuf = P.sl_xbuf.get();
    a.flags = P.sl_flags.get();
    a.err = P.sl_err.get();
    a.cap = P.slab_cap;
    a.S = P.slab_S;
    a.G = P.ngroups;
    a.wwin_off = (int32_t)P.slab_xmax;
    a.meta_off = (int32_t)P.slab_meta_off;
    a.cache_off = (int32_t)P.slab_cache_off;
    a.omega = P.opts.omega;
    return a;
}

// `sweeps` sweeps on x (device, reordered coordinates) in one launch,
// preceded by the flag reset; both are graph-capturable.
void slab_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    if (sweeps <= 0) return;
    const int32_t S = P.slab_S;
    k_slab_reset<<<(S + 255) / 256, 256, 0, s>>>(S, P.sl_flags.get(), P.sl_err.get());
    k_slab_sweeps<<<S, kSlabThreads, (size_t)P.slab_lds, s>>>(slab_args(P), sweeps, x);
    OBK_HIP(hipGetLastError());
}

// The same launch with an event pair on its dispatch packet (for the
// per-kernel roofline); returns the launch's seconds.  Synchronises s.
double slab_profile(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    const int32_t S = P.slab_S;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    OBK_HIP(hipEventCreate(&e0));
    OBK_HIP(hipEventCreate(&e1));
    k_slab_reset<<<(S + 255) / 256, 256, 0, s>>>(S, P.sl_flags.get(), P.sl_err.get());
    hipExtLaunchKernelGGL(k_slab_sweeps, dim3(S), dim3(kSlabThreads), (size_t)P.slab_lds, s, e0, e1, 0,
                          slab_args(P), sweeps, x);
    OBK_HIP(hipGetLastError());
    OBK_HIP(hipStreamSynchronize(s));
    float ms = 0;
    OBK_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    slab_check(P, s);
    return ms * 1e-3;
}

// Report a timed-out neighbour wait of the last launches (synchronises s).
void slab_check(obk_plan_s& P, hipStream_t s) {
    if (!P.slab_S) return;
    int h = 0;
    OBK_HIP(hipMemcpyAsync(&h, P.sl_err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    if (h) fail(OBK_E_HIP, "banded sweep: a neighbour wait timed out (workgroups not co-resident?)");
}

}  // namespace obk

extern "C" obk_status obk_banded_emulate_host(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                                              const double* f, const double* inv, const int32_t* group,
                                              int32_t ngroups, int32_t slabs, int64_t sweeps, double omega,
                                              double* x, int64_t* stats) {
    try {
        if (n < 1 || !rp || !col || !val || !f || !inv || !group || !x || ngroups < 1 || slabs < 1 || sweeps < 0)
            obk::fail(OBK_E_ARG, "bad argument");
        // group-major layout: rows of each group in ascending reordered order
        std::vector<int64_t> gptr(ngroups + 1, 0);
        for (int64_t i = 0; i < n; i++)
            if (group[i] >= 0) {
                if (group[i] >= ngroups) obk::fail(OBK_E_ARG, "group out of range");
                gptr[group[i] + 1]++;
            }
        for (int32_t g = 0; g < ngroups; g++) gptr[g + 1] += gptr[g];
        const int64_t m = gptr[ngroups];
        std::vector<int32_t> grow(m);
        std::vector<int64_t> fillg(gptr.begin(), gptr.end() - 1);
        for (int64_t i = 0; i < n; i++)
            if (group[i] >= 0) grow[fillg[group[i]]++] = (int32_t)i;
        std::vector<int64_t> hrptr(m + 1, 0);
        for (int64_t p = 0; p < m; p++) hrptr[p + 1] = hrptr[p] + (rp[grow[p] + 1] - rp[grow[p]]);
        std::vector<int32_t> gcol(hrptr[m]);
        std::vector<double> gval(hrptr[m]), rf(m), rinv(m);
        int64_t bw = 0;
        for (int64_t p = 0; p < m; p++) {
            const int64_t i = grow[p];
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
                gcol[hrptr[p] + (e - rp[i])] = col[e];
                gval[hrptr[p] + (e - rp[i])] = val[e];
                bw = std::max<int64_t>(bw, std::abs((int64_t)col[e] - i));
            }
            rf[p] = f[i];
            rinv[p] = inv[i];
        }
        obk::SlabHost h = obk::slab_build(n, ngroups, gptr, hrptr, grow, gcol, gval, rf, rinv, bw, slabs,
                                          159 * 1024, slabs);
        if (stats) {
            int64_t cached = 0, streamed = 0;
            for (const auto& gd : h.grp)
                for (const obk::SlabPhase* ph : {&gd.r, &gd.s, &gd.sb})
                    if (ph->count > 0) (ph->cache >= 0 ? cached : streamed)++;
            stats[0] = h.S;
            stats[1] = cached;
            stats[2] = streamed;
            stats[3] = ((h.xmax + h.wmax) * 8 + 15) / 16 * 16 + h.meta_bytes + h.cache_bytes;
        }
        if (!h.S) obk::fail(OBK_E_ARG, "the banded engine does not apply: " + h.why);
        obk::slab_emulate(h, sweeps, omega, x);
        obk::set_last_error("");
        return OBK_OK;
    } catch (const obk::Error& e) {
        obk::set_last_error(e.msg);
        return e.code;
    } catch (...) {
        obk::set_last_error("unexpected internal error");
        return OBK_E_HIP;
    }
}
