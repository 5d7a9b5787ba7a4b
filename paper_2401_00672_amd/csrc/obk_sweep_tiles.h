// Device bodies of the two sweep phases over tiles, shared by the per-group
// kernels (defined at the end of this file) and the batched team kernel.  T
// is the arithmetic type (double, or float in the inner sweeps of iterative
// refinement).
//
// phase R (one group): for each row a of the tile, from the same x,
//   w_a = ((f_a - sum_k a_ak x_k) * inv_a) * omega   (omega = 1: the paper's step)
// phase S (one group): for each touched column c of the tile,
//   x_c = x_c + sum over the group's rows a holding c of w_a a_ac
//
// A tile is worked on by one 256-thread sub-block.  Thread t owns segments
// (rows in R, columns in S) t, t + 256, ..., Q of them; entries are staged
// through LDS in chunks of 256*E values, E per thread, and each segment is
// then reduced by its owner in ascending entry order, so the result depends
// neither on Q, E nor on the tile schedule.  The per-group kernels use plan
// tiles (Q = 1, E = 8, which keeps enough tiles per phase to fill the chip);
// the batched kernel, whose parallelism comes from many systems, uses
// merged tiles (Q = 2, E = 16) to keep twice the loads in flight per round
// trip.  Every load that depends only on the tile (row bounds, f,
// 1/||a||^2, the column owned) is issued before the entry loads.  Written in
// predicated form: every load is issued at an in-range index.  An empty tile
// {0,0,0,0} may be passed for an idle sub-block (segment 0 must exist).
#pragma once

#include <type_traits>

#include "obk_internal.h"

namespace obk {

constexpr int kPlanE = kTileEntries / kTileThreads;    // entries per thread for plan tiles
constexpr int kPlanQ = kTileSegs / kTileThreads;       // segments per thread for plan tiles

template <int E = kPlanE>
__device__ __forceinline__ int tile_chunks(const Tile& t) {
    constexpr int64_t C = (int64_t)kTileThreads * E;
    return (int)((t.ent_end - t.ent_begin + C - 1) / C);
}

// In the FP32 sweeps a streamed entry (column or row index, value), read
// once per phase, is loaded with the non-temporal hint, so that it displaces
// less of the gathered x and w from L2: phase R of a scattered 2M-row system
// gathers from 8 MB of FP32 x against a 4 MiB L2 per XCD, and the batched
// engine keeps every system's x there.  The FP64 and complex sweeps keep the
// plain load (on the banded stencil, whose x windows already stay in L2, the
// hint cost 7% of the sweep rate).
template <bool kNT, class V>
__device__ __forceinline__ V entry_ld(const V* p) {
    if constexpr (kNT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Stage one chunk of products into LDS: prod[q] = val[q] * v[idx[q]] for
// q < len.  All index and value loads of the thread are issued first, then all
// gathers, so a chunk costs two dependent memory round trips, not one pair per
// entry.  Loads are exec-masked (q < len), never issued out of range.
template <class T, int E = kPlanE>
__device__ __forceinline__ void stage_r(T* prod, int me, int len, const int32_t* __restrict__ idx,
                                        const T* __restrict__ val, const T* __restrict__ v) {
    int32_t ix[E];
    T va[E], g[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        ix[e] = 0;
        va[e] = T(0);
        if (q < len) {
            ix[e] = entry_ld<std::is_same<T, float>::value>(idx + q);
            va[e] = entry_ld<std::is_same<T, float>::value>(val + q);
        }
    }
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        g[e] = T(0);
        if (q < len) g[e] = v[ix[e]];
    }
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        if (q < len) prod[q] = va[e] * g[e];
    }
}

// Same for phase S, where the product is w[row] * val (operand order kept).
template <class T, int E = kPlanE>
__device__ __forceinline__ void stage_s(T* prod, int me, int len, const int32_t* __restrict__ idx,
                                        const T* __restrict__ val, const T* __restrict__ v) {
    int32_t ix[E];
    T va[E], g[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        ix[e] = 0;
        va[e] = T(0);
        if (q < len) {
            ix[e] = entry_ld<std::is_same<T, float>::value>(idx + q);
            va[e] = entry_ld<std::is_same<T, float>::value>(val + q);
        }
    }
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        g[e] = T(0);
        if (q < len) g[e] = v[ix[e]];
    }
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = me + e * kTileThreads;
        if (q < len) prod[q] = g[e] * va[e];
    }
}

template <class T, int Q = kPlanQ, int E = kPlanE>
__device__ __forceinline__ void tile_phase_r(const Tile& t, int nchunks, T* prod, const int64_t* __restrict__ rptr,
                                             const int32_t* __restrict__ rcol, const T* __restrict__ rval,
                                             const T* __restrict__ rf, const T* __restrict__ rinv,
                                             const T* __restrict__ x, T* __restrict__ w, T omega) {
    constexpr int64_t C = (int64_t)kTileThreads * E;     // entries per chunk
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x & (kTileThreads - 1);
    bool own[Q];
    int64_t a[Q], k0[Q], k1[Q];
    T fa[Q], ia[Q], acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int sg = me + q * kTileThreads;
        own[q] = sg < nseg;
        a[q] = t.seg_begin + (own[q] ? sg : 0);
        k0[q] = rptr[a[q]];
        k1[q] = rptr[a[q] + 1];
        fa[q] = rf[a[q]];
        ia[q] = rinv[a[q]];
        acc[q] = T(0);
    }
    for (int c = 0; c < nchunks; c++) {
        const int64_t base = t.ent_begin + (int64_t)c * C;
        const int len = (int)max<int64_t>(0, min<int64_t>(C, t.ent_end - base));
        stage_r<T, E>(prod, me, len, rcol + base, rval + base, x);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int64_t lo = max(k0[q], base), hi = own[q] ? min(k1[q], base + len) : lo;
            for (int64_t k = lo; k < hi; k++) acc[q] = acc[q] + prod[k - base];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
        if (own[q]) w[a[q]] = ((fa[q] - acc[q]) * ia[q]) * omega;
}

template <class T, int Q = kPlanQ, int E = kPlanE>
__device__ __forceinline__ void tile_phase_s(const Tile& t, int nchunks, T* prod, const int64_t* __restrict__ sptr,
                                             const int32_t* __restrict__ srow, const T* __restrict__ sval,
                                             const int32_t* __restrict__ tcol, const T* __restrict__ w,
                                             T* __restrict__ x) {
    constexpr int64_t C = (int64_t)kTileThreads * E;     // entries per chunk
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x & (kTileThreads - 1);
    bool own[Q];
    int64_t k0[Q], k1[Q];
    int32_t col[Q];
    T xc[Q], acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int sg = me + q * kTileThreads;
        own[q] = sg < nseg;
        const int64_t s = t.seg_begin + (own[q] ? sg : 0);
        k0[q] = sptr[s];
        k1[q] = sptr[s + 1];
        col[q] = tcol[s];
        xc[q] = x[col[q]];      // each column has one owner in the phase
        acc[q] = T(0);
    }
    for (int c = 0; c < nchunks; c++) {
        const int64_t base = t.ent_begin + (int64_t)c * C;
        const int len = (int)max<int64_t>(0, min<int64_t>(C, t.ent_end - base));
        stage_s<T, E>(prod, me, len, srow + base, sval + base, w);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int64_t lo = max(k0[q], base), hi = own[q] ? min(k1[q], base + len) : lo;
            for (int64_t k = lo; k < hi; k++) acc[q] = acc[q] + prod[k - base];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
        if (own[q]) x[col[q]] = xc[q] + acc[q];
}

// FP64 residual of one R tile: r_a = f_a - a_a . x for each row of the tile,
// each row summed in ascending entry order exactly as in phase R.  r (may be
// null) receives r_a.  The tile's sum of r_a^2 and maximum of |r_a| are formed
// by a fixed tree over the row slots and returned to every thread of the
// sub-block (prod is reused as the tree's scratch).  A nonfinite r_a sets
// *nonfinite.
__device__ __forceinline__ void tile_resid(const Tile& t, int nchunks, double* prod,
                                           const int64_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                                           const double* __restrict__ rval, const double* __restrict__ rf,
                                           const double* __restrict__ x, double* __restrict__ r,
                                           int* __restrict__ nonfinite, double& sum_sq, double& max_abs) {
    static_assert(kTileSegs == kTileThreads, "one row per thread");
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x & (kTileThreads - 1);
    const bool own = me < nseg;
    const int64_t a = t.seg_begin + (own ? me : 0);
    const int64_t k0 = rptr[a], k1 = rptr[a + 1];
    const double fa = rf[a];
    double acc = 0.0;
    for (int c = 0; c < nchunks; c++) {
        const int64_t base = t.ent_begin + (int64_t)c * kTileEntries;
        const int len = (int)max<int64_t>(0, min<int64_t>(kTileEntries, t.ent_end - base));
        stage_r(prod, me, len, rcol + base, rval + base, x);
        __syncthreads();
        const int64_t lo = max(k0, base), hi = own ? min(k1, base + len) : lo;
        for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        __syncthreads();
    }
    const double ra = fa - acc;
    if (own) {
        if (r) r[a] = ra;
        if (!isfinite(ra)) atomicOr(nonfinite, 1);
    }
    double* red = prod;
    double* mx = prod + kTileThreads;
    red[me] = own ? ra * ra : 0.0;
    mx[me] = own ? fabs(ra) : 0.0;
    __syncthreads();
    for (int st = kTileThreads / 2; st > 0; st >>= 1) {
        if (me < st) {
            red[me] = red[me] + red[me + st];
            mx[me] = fmax(mx[me], mx[me + st]);
        }
        __syncthreads();
    }
    sum_sq = red[0];
    max_abs = mx[0];
    __syncthreads();
}

// Tile of workgroup b when workgroups are dealt to the 8 XCDs in turn
// (b -> XCD b % 8): XCD x takes one contiguous run of the tiles, so tiles
// that share a window of x (or w) share that XCD's L2.  A bijection on
// [0, n) for any n.
__host__ __device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n) {
    const int32_t q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
    return x * q + min(x, r) + j;
}

// A phase of at most kInlineTiles tiles carries its tile list in the kernel
// arguments, already in the order of xcd_tile: workgroup b reads entry b at
// kernel start together with the other arguments, one dependent load sooner
// than through the tile array (whose index needs the grid size, itself an
// argument), which shortens the latency-bound phases of small groups.
constexpr int kInlineTiles = 32;
struct TileList {
    Tile t[kInlineTiles];
};

namespace {

// Phase R / phase S kernels over the tiles of one group: one tile per
// 256-thread workgroup, from tiles[] or, for kInl, from tl.
// (kInl: the tile list is in the arguments; the two instances differ only in
// where the tile is read, so neither carries the other's load.)
template <class T, bool kInl>
__global__ __launch_bounds__(kTileThreads) void k_phase_r(
    const Tile* __restrict__ tiles, TileList tl, const int64_t* __restrict__ rptr,
    const int32_t* __restrict__ rcol, const T* __restrict__ rval, const T* __restrict__ rf,
    const T* __restrict__ rinv, const T* __restrict__ x, T* __restrict__ w, T omega) {
    __shared__ T prod[kTileEntries];
    const Tile t = kInl ? tl.t[blockIdx.x] : tiles[xcd_tile(blockIdx.x, gridDim.x)];
    tile_phase_r<T>(t, tile_chunks(t), prod, rptr, rcol, rval, rf, rinv, x, w, omega);
}

template <class T, bool kInl>
__global__ __launch_bounds__(kTileThreads) void k_phase_s(
    const Tile* __restrict__ tiles, TileList tl, const int64_t* __restrict__ sptr,
    const int32_t* __restrict__ srow, const T* __restrict__ sval, const int32_t* __restrict__ tcol,
    const T* __restrict__ w, T* __restrict__ x) {
    __shared__ T prod[kTileEntries];
    const Tile t = kInl ? tl.t[blockIdx.x] : tiles[xcd_tile(blockIdx.x, gridDim.x)];
    tile_phase_s<T>(t, tile_chunks(t), prod, sptr, srow, sval, tcol, w, x);
}

// FP64 residual over all R tiles of a plan, one tile per workgroup: r
// (may be null) gets r_a; psum/pmax get the per-tile sum of r_a^2 and max |r_a|.
__global__ __launch_bounds__(kTileThreads) void k_resid_tiles(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
    const double* __restrict__ rval, const double* __restrict__ rf, const double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ psum, double* __restrict__ pmax, int* __restrict__ nonfinite) {
    __shared__ double prod[kTileEntries];
    const Tile t = tiles[blockIdx.x];
    double s2, mx;
    tile_resid(t, tile_chunks(t), prod, rptr, rcol, rval, rf, x, r, nonfinite, s2, mx);
    if (threadIdx.x == 0) { psum[blockIdx.x] = s2; pmax[blockIdx.x] = mx; }
}

}  // namespace

}  // namespace obk
