// Block form of Algorithm 4 (Section 3.3): k uniform chunks of the reordered
// system, the |cos| table of their centroids, the pairing into Oclass and
// Nclass, and sweeps of exact block projections (eq. 3.3).
//
// Planning (block_setup; the shared stages have already kept the reordered
// rows in order, m = n, and built the per-block CSC with rows ascending):
//   * every per-block column segment is summed in ascending row order: these
//     are the block's column sums, its centroid times its row count (a scale
//     the cosine does not see);
//   * for every pair of blocks whose touched-column ranges intersect, one
//     workgroup forms the dot product of their column sums by looking up each
//     column of one block in the sorted column list of the other; all other
//     pairs share no column and their cosine is exactly 0;
//   * the host forms |cos| and pairs the blocks;
//   * (block_factor) for each block, the host puts its rows in the reverse
//     Cuthill-McKee order of its Gram graph and forms the banded Cholesky
//     factor of A_t A_t^T in the unit-diagonal form U D U^T, when the block
//     has full row rank to the pivot test and a band within the limits.
//
// Sweeps with factors (k_block_direct, or k_block_sweeps<1> when only some
// blocks have one): a projection is r = f_t - A_t x~, U z = r, z *= D^-1,
// U^T y = z, x~ += A_t^T y, by one workgroup (project_direct).
//
// Sweeps by CG (k_block_sweeps): one launch of G workgroups (cooperative for
// G > 1) runs every projection of the call.  Projection onto block t (rows R, touched columns
// S): res = f_R - A_R x~ (all-zero rows: 0), then conjugate gradients on
// A_R A_R^T y = res in the form that moves x~ itself (x~ += alpha A_R^T d):
//   phase A (columns of S)  u = A_R^T (res + beta p)              |u|^2
//   -- grid barrier --      alpha = |res|^2 / |u|^2
//   phase B (columns of S)  x~ += alpha u
//           (rows of R)     p = res + beta p; res -= alpha A_R u   |res|^2
//   -- grid barrier --      beta = |res_new|^2 / |res|^2
// (p holds the previous direction; u = A_R^T d with d = res + beta p is the
// current one, so alpha = |res|^2 / d^T A_R A_R^T d = |res|^2 / |u|^2.)
// Rows and column segments of a block are cut into G contiguous ranges, one
// per workgroup; each row and each column is reduced sequentially in
// ascending index order.  Every workgroup reduces the G partial sums itself
// in one fixed order, so all of them take the same decisions with no further
// synchronisation, and a solve is bitwise repeatable for a given G.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <system_error>
#include <thread>
#include <vector>

#include "obk_internal.h"

namespace obk {

namespace {

constexpr int kBT = 1024;             // threads per workgroup of the projection launch
constexpr long kBlockSpin = 1L << 22; // bound on one barrier wait (polls)

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// A double moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over a wave in a fixed order, the same value in every lane: pairs
// within quads (lanes i, i^1, then i, i^2), quads within half rows (lane i
// with 7 - i), half rows within rows of 16 (i with 15 - i) -- each step adds
// two values in an order that commutes, so all lanes of a row agree -- then
// the four row sums in ascending order.
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp_f64<0xB1>(v);       // quad_perm [1,0,3,2]
    v = v + dpp_f64<0x4E>(v);       // quad_perm [2,3,0,1]
    v = v + dpp_f64<0x141>(v);      // row_half_mirror
    v = v + dpp_f64<0x140>(v);      // row_mirror
    return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}

// Sum over the workgroup in a fixed order (each wave's sum, then the wave
// sums in ascending order); every thread gets the same value.  Called by
// every thread of the workgroup.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* lds) {
    v = wave_sum(v);
    __syncthreads();                       // lds is free again
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) t = t + lds[i];
    return t;
}

// sum over e in [e0, e1) of val[e] * gather(idx[e]), accumulated in
// ascending e; four entries at a time have their loads issued together.
template <class I, class F>
__device__ __forceinline__ double dot_seq(int64_t e0, int64_t e1, const double* val, const I* idx, F gather) {
    double s = 0.0;
    int64_t e = e0;
    for (; e + 4 <= e1; e += 4) {
        const double v0 = val[e], v1 = val[e + 1], v2 = val[e + 2], v3 = val[e + 3];
        const double g0 = gather(idx[e]), g1 = gather(idx[e + 1]), g2 = gather(idx[e + 2]),
                     g3 = gather(idx[e + 3]);
        s = s + v0 * g0;
        s = s + v1 * g1;
        s = s + v2 * g2;
        s = s + v3 * g3;
    }
    for (; e < e1; e++) s = s + val[e] * gather(idx[e]);
    return s;
}

// Barrier over the whole (co-resident) grid on a monotonic arrival counter:
// at its e-th barrier a workgroup adds 1 and waits until the counter reaches
// e G.  Every wave fences at agent scope on both sides (its own stores out
// before the arrival, the others' stores in after the wait); wave 0 waits,
// in wave-uniform control flow.  Returns false when the wait timed out or
// another workgroup reported a timeout: the caller then leaves the kernel,
// so every workgroup exits after at most one bound.
__device__ __forceinline__ bool grid_barrier(uint64_t* bar, int* err, int* lds_flag, uint64_t& episode) {
    if (gridDim.x == 1) {
        __syncthreads();
        return true;
    }
    episode++;
    const uint64_t target = episode * gridDim.x;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x) >> 6;
    if (wave == 0) {
        if (threadIdx.x == 0) __hip_atomic_fetch_add(bar, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t cur = 0;
        int bad = 0;
        long spins = 0;
#pragma clang loop unroll(disable)
        do {
            __builtin_amdgcn_s_sleep(1);
            cur = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            spins++;
        } while ((cur < target) & (bad == 0) & (spins <= kBlockSpin));
        const int ok = cur >= target ? 1 : 0;
        if (threadIdx.x == 0) {
            if (!ok) atomicOr(err, 1);
            *lds_flag = ok;
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *lds_flag != 0;
}

struct BlockArgs {
    const int64_t* rptr;      // reordered CSR (rows in order), [n+1]
    const int32_t* rcol;
    const double* rval;
    const double* rf;
    const double* rinv;       // 0 marks an all-zero row
    const int64_t* bptr;      // rows of block b: [bptr[b], bptr[b+1])
    const int64_t* btptr;     // column segments of block b: [btptr[b], btptr[b+1])
    const int32_t* tcol;
    const int64_t* sptr;
    const int32_t* srow;
    const double* sval;
    const int32_t* order;     // blocks in projection order
    double* x;
    double* res;
    double* p;
    double* u;
    double* part;             // [4 G] partial sums: |u|^2, |res|^2 in the loop, |res_0|^2 (two)
    uint64_t* bar;            // arrival counter (zero at launch)
    int* err;
    int64_t* iters;           // CG iterations per block, accumulated
    const int32_t* lseg;      // per CSR entry: its column's index in the block's segment list
    const int32_t* fit;       // per block: 1 if it is projected from LDS
    const int32_t* direct;    // per block: 1 if it is projected from its Cholesky factor
    const int32_t* dbw;       // per block: the factor's bandwidth
    const int64_t* doff;      // per block: offset of the factor in lfc / lfr
    const double* lfc;        // factors by columns: [off + c (bw+1) + d] = L[c+d][c]
    const double* lfr;        // factors by rows: [off + i (bw+1) + bw - (i-j)] = L[i][j]
    const double* ldinv;      // 1 / L[k][k] per factor position [n]
    const int32_t* lperm;     // per factor position k of a block: its block row [n]
    const int32_t* lpos;      // per block row: its factor position [n]
    int64_t sweeps;
    int32_t lds_path;         // 1: single-workgroup launch with dynamic LDS for the fitting blocks
    int32_t k;
    int32_t maxit;            // 0: 4 rows + 100
    double tol2;              // squared relative stopping tolerance
};

// Dynamic LDS bytes of a block projected from LDS (nb rows, ns touched
// columns, eb entries): entry values of the CSR and CSC copies, res, p, u and
// the touched x in FP64; row and segment offsets in int32; local column and
// row indices in uint16.
__host__ __device__ inline int64_t lds_bytes_for(int64_t nb, int64_t ns, int64_t eb) {
    return 8 * (2 * eb + 2 * nb + 2 * ns) + 4 * (nb + ns + 2) + 4 * eb;
}

// The local indices of up to C entries of one row or column segment, held in
// registers for a whole projection (entries past C are read from LDS), so
// that a dot's gathers can be issued without first loading the indices.
template <int C>
struct RegCache {
    int e0, n, hi;          // first entry, cached count, end of the segment
    int idx[C];
};

template <int C>
__device__ __forceinline__ void cache_load(RegCache<C>& c, int e0, int e1, const uint16_t* idx) {
    c.e0 = e0;
    c.n = min(e1 - e0, C);
    c.hi = e1;
#pragma unroll
    for (int k = 0; k < C; k++) c.idx[k] = (k < c.n) ? (int)idx[e0 + k] : 0;
}

// sum over the segment's entries, ascending, of val * vec[idx]; the value
// loads and gathers of the cached entries are issued together
template <int C, class F>
__device__ __forceinline__ double cache_dot(const RegCache<C>& c, const double* val, const uint16_t* idx, F vec) {
    double g[C], v[C];
#pragma unroll
    for (int k = 0; k < C; k++) {
        g[k] = (k < c.n) ? vec(c.idx[k]) : 0.0;
        v[k] = (k < c.n) ? val[c.e0 + k] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < C; k++)
        if (k < c.n) s = s + v[k] * g[k];
    for (int e = c.e0 + c.n; e < c.hi; e++) s = s + val[e] * vec(idx[e]);
    return s;
}

constexpr int kCache = 6;

// One projection by a single workgroup with the block resident in LDS: the
// block's CSR and CSC (local indices), res, p, u and the touched entries of
// x~ are staged once; the CG iterations then touch no global memory; x~ is
// written back at the end.  Same operations in the same order as the
// global-memory form with one workgroup.  Returns the CG iterations.
__device__ int64_t project_lds(const BlockArgs& a, int32_t b, double* dyn, double* lds) {
    const int t = threadIdx.x;
    const int64_t r0 = a.bptr[b], nb = a.bptr[b + 1] - r0;
    const int64_t s0 = a.btptr[b], ns = a.btptr[b + 1] - s0;
    const int64_t e0 = a.rptr[r0], eb = a.rptr[r0 + nb] - e0;
    const int64_t q0 = a.sptr[s0];
    double* rv = dyn;
    double* sv = rv + eb;
    double* res = sv + eb;
    double* pv = res + nb;
    double* u = pv + nb;
    double* xs = u + ns;
    int32_t* roff = reinterpret_cast<int32_t*>(xs + ns);
    int32_t* soff = roff + nb + 1;
    uint16_t* lcol = reinterpret_cast<uint16_t*>(soff + ns + 1);
    uint16_t* lrow = lcol + eb;
    for (int64_t i = t; i <= nb; i += kBT) roff[i] = (int32_t)(a.rptr[r0 + i] - e0);
    for (int64_t q = t; q <= ns; q += kBT) soff[q] = (int32_t)(a.sptr[s0 + q] - q0);
    for (int64_t e = t; e < eb; e += kBT) {
        rv[e] = a.rval[e0 + e];
        lcol[e] = (uint16_t)a.lseg[e0 + e];
        sv[e] = a.sval[q0 + e];
        lrow[e] = (uint16_t)(a.srow[q0 + e] - r0);
    }
    for (int64_t q = t; q < ns; q += kBT) xs[q] = a.x[a.tcol[s0 + q]];
    __syncthreads();
    // registers hold the indices of the first owned row and the first two owned segments
    const int64_t qa = t, qb = t + kBT;
    RegCache<kCache> rc, sca, scb;
    cache_load(rc, t < nb ? roff[t] : 0, t < nb ? roff[t + 1] : 0, lcol);
    cache_load(sca, qa < ns ? soff[qa] : 0, qa < ns ? soff[qa + 1] : 0, lrow);
    cache_load(scb, qb < ns ? soff[qb] : 0, qb < ns ? soff[qb + 1] : 0, lrow);
    auto gx = [&](int c) { return xs[c]; };
    auto gu = [&](int c) { return u[c]; };
    auto gp = [&](int i) { return pv[i]; };
    double acc = 0.0;
    // the residual of each owned row (the first from its cached indices);
    // all-zero rows take no part; the first direction is res + beta p with
    // beta = 0, p = 0
    if (t < nb) {
        const double d = cache_dot(rc, rv, lcol, gx);
        const double r = (a.rinv[r0 + t] != 0.0) ? a.rf[r0 + t] - d : 0.0;
        res[t] = r;
        pv[t] = r + 0.0 * 0.0;
        acc = acc + r * r;
    }
    for (int64_t i = t + kBT; i < nb; i += kBT) {
        double d = 0.0;
        for (int32_t e = roff[i]; e < roff[i + 1]; e++) d = d + rv[e] * xs[lcol[e]];
        const double r = (a.rinv[r0 + i] != 0.0) ? a.rf[r0 + i] - d : 0.0;
        res[i] = r;
        pv[i] = r + 0.0 * 0.0;
        acc = acc + r * r;
    }
    double rr = wg_sum<kBT>(acc, lds);
    const double rr0 = rr;
    const int64_t cap = a.maxit > 0 ? a.maxit : 4 * nb + 100;
    int64_t it = 0;
    // pv holds the current direction d = res + beta p, formed once per row
    // after beta is known (the global-memory form forms the same value at
    // every use), so phase A gathers one vector
    while (rr0 > 0.0 && rr > a.tol2 * rr0 && it < cap) {
        acc = 0.0;
        if (qa < ns) {
            const double sum = cache_dot(sca, sv, lrow, gp);
            u[qa] = sum;
            acc = acc + sum * sum;
        }
        if (qb < ns) {
            const double sum = cache_dot(scb, sv, lrow, gp);
            u[qb] = sum;
            acc = acc + sum * sum;
        }
        for (int64_t q = t + 2 * kBT; q < ns; q += kBT) {
            double sum = 0.0;
            for (int32_t e = soff[q]; e < soff[q + 1]; e++) sum = sum + sv[e] * pv[lrow[e]];
            u[q] = sum;
            acc = acc + sum * sum;
        }
        const double uu = wg_sum<kBT>(acc, lds);
        if (!(uu > 0.0)) break;
        const double alpha = rr / uu;
        for (int64_t q = t; q < ns; q += kBT) xs[q] = xs[q] + alpha * u[q];
        acc = 0.0;
        if (t < nb) {
            const double rn = res[t] - alpha * cache_dot(rc, rv, lcol, gu);
            res[t] = rn;
            acc = acc + rn * rn;
        }
        for (int64_t i = t + kBT; i < nb; i += kBT) {
            double d = 0.0;
            for (int32_t e = roff[i]; e < roff[i + 1]; e++) d = d + rv[e] * u[lcol[e]];
            const double rn = res[i] - alpha * d;
            res[i] = rn;
            acc = acc + rn * rn;
        }
        const double rn2 = wg_sum<kBT>(acc, lds);
        const double beta = rn2 / rr;
        rr = rn2;
        it++;
        for (int64_t i = t; i < nb; i += kBT) pv[i] = res[i] + beta * pv[i];
        __syncthreads();
    }
    for (int64_t q = t; q < ns; q += kBT) a.x[a.tcol[s0 + q]] = xs[q];
    __syncthreads();
    return it;
}

// Dynamic LDS bytes of a direct projection of a block of nb rows: y, and
// two buffers for the diagonal block of a panel and its inverse pivots.
constexpr int kPanel = 64;
// a panel's diagonal block, rows padded to 65 doubles so that lane k reading
// row k stays off the other lanes' banks, then 1 / L[k][k]
constexpr int kDStride = kPanel + 1;
constexpr int kDiagBuf = kPanel * kDStride + kPanel;
__host__ __device__ inline int64_t direct_lds_for(int64_t nb) { return 8 * (nb + 2 * kDiagBuf); }

// One exact projection by a single workgroup from the block's banded
// Cholesky factor L (L L^T = A_t A_t^T):
//   r = f_t - A_t x~  ->  L z = r  ->  L^T y = z  ->  x~ += A_t^T y
// The triangular solves go by panels of 64 rows: the panel's diagonal block
// is staged in LDS and solved by wave 0 lane by lane (lane k holds row k;
// step c broadcasts the finished value of row c), then the rows of the band
// beyond the panel are updated, four threads to a row (16 panel columns
// each, the four partial sums added in lane order).  Neither the factor
// entries of that update nor the next panel's diagonal block depend on the
// solve, so every thread loads them into registers before wave 0 starts and
// the solve hides their latency; the diagonal blocks alternate between two
// LDS buffers.  y lives in LDS throughout.
constexpr int kPart = 4;                       // threads per updated row
constexpr int kPartCols = kPanel / kPart;      // panel columns per thread
constexpr int kStagePer = kPanel * kPanel / kBT;
constexpr int64_t kRowsPerPass = kBT / kPart;  // updated rows per pass

// Factor entries of the update of row j (this thread's 16 panel columns);
// lfac(j, c) gives the entry's index, or -1 outside the band.
template <class F>
__device__ __forceinline__ void band_load(double (&lv)[kPartCols], int j, bool row_ok, int pw,
                                          const double* __restrict__ Lf, F lfac) {
    const int part = threadIdx.x % kPart;
#pragma unroll
    for (int u = 0; u < kPartCols; u++) {
        const int c = part * kPartCols + u;
        const int k = (row_ok && c < pw) ? lfac(j, c) : -1;
        const double l = Lf[k >= 0 ? k : 0];
        lv[u] = k >= 0 ? l : 0.0;
    }
}

// z[j] -= sum over the panel columns c of L(j, c) z[p0 + c]; the four lanes
// of a row call it together
__device__ __forceinline__ void band_apply(const double (&lv)[kPartCols], double* z, int p0, int pw, int j,
                                           bool row_ok) {
    const int part = threadIdx.x % kPart;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kPartCols; u++) {
        const int c = part * kPartCols + u;
        acc = acc + lv[u] * z[p0 + (c < pw ? c : 0)];
    }
    const double a1 = __shfl_down(acc, 1, kPart);
    const double a2 = __shfl_down(acc, 2, kPart);
    const double a3 = __shfl_down(acc, 3, kPart);
    if (row_ok && part == 0) z[j] = z[j] - (((acc + a1) + a2) + a3);
}

// The diagonal block D[k][c] (64 x 64) of the panel at row p0 (pw rows) and
// its inverse pivots: lfac(k, c) gives the entry's index, or -1 for a zero.
template <class F>
__device__ __forceinline__ void stage_load(double (&v)[kStagePer], double& dv, const double* __restrict__ Lf,
                                           const double* __restrict__ dinv, int p0, int pw, F lfac) {
#pragma unroll
    for (int u = 0; u < kStagePer; u++) {
        const int q = threadIdx.x + u * kBT;
        const int k = lfac(q / kPanel, q % kPanel);
        const double l = Lf[k >= 0 ? k : 0];
        v[u] = k >= 0 ? l : 0.0;
    }
    const int k = (int)threadIdx.x;
    const double d = dinv[p0 + (k < pw ? k : 0)];
    dv = k < pw ? d : 0.0;
}
__device__ __forceinline__ void stage_store(double* D, const double (&v)[kStagePer], double dv) {
#pragma unroll
    for (int u = 0; u < kStagePer; u++) {
        const int q = threadIdx.x + u * kBT;
        D[(q / kPanel) * kDStride + q % kPanel] = v[u];
    }
    if (threadIdx.x < kPanel) D[kPanel * kDStride + threadIdx.x] = dv;
}

// Unit triangular solve with a band narrower than a wave (bw < 64), in place
// on z (LDS): forward U z = r (kFwd) or backward U^T y = z.  Wave 0 keeps the
// 64 rows at and after the current one (before it, backward) in a circular
// window: row j lives in lane j mod 64.  Step k broadcasts row k's finished
// value from its lane, updates the rows of the band with one FMA each, and
// the lane takes the row 64 further on.  The other waves copy the band, 64
// rows at a time, into the LDS buffer wave 0 is not reading.
template <bool kFwd>
__device__ __forceinline__ void window_solve(double* z, int nb, int bw, const double* __restrict__ Lf,
                                             const double* __restrict__ dinv, double* buf0, double* buf1) {
    const int t = threadIdx.x, W = bw + 1;
    const int nch = (nb + kPanel - 1) / kPanel;
    // chunk ci covers rows [cb, ce): ascending chunks forward, descending backward
    auto range = [&](int ci, int& cb, int& ce) {
        if (kFwd) { cb = ci * kPanel; ce = min(nb, cb + kPanel); }
        else { ce = nb - ci * kPanel; cb = max(0, ce - kPanel); }
    };
    // copy a chunk's band rows (at most 64 x 64 values) and inverse pivots:
    // every load of the thread is issued before its stores
    constexpr int kPer = (kPanel * kPanel + (kBT - kPanel) - 1) / (kBT - kPanel);
    auto stage = [&](int ci, double* B, int first, int stride) {
        int cb, ce;
        range(ci, cb, ce);
        const int len = (ce - cb) * W;
        double v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int q = first + u * stride;
            v[u] = Lf[cb * W + (q < len ? q : 0)];
        }
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int q = first + u * stride;
            if (q < len) B[q] = v[u];
        }
    };
    // wave 0 is the solving wave; the test is wave-uniform by construction
    const bool solver = (__builtin_amdgcn_readfirstlane(threadIdx.x) >> 6) == 0;
    double w = 0.0;
    if (solver) {
        const int j = kFwd ? t : (nb - 1) - ((nb - 1 - t) & (kPanel - 1));
        w = (j >= 0 && j < nb) ? z[j] : 0.0;
    }
    stage(0, buf0, t, kBT);
    __syncthreads();
    for (int ci = 0; ci < nch; ci++) {
        double* B = (ci & 1) ? buf1 : buf0;
        if (!solver) {
            if (ci + 1 < nch) stage(ci + 1, (ci & 1) ? buf0 : buf1, t - kPanel, kBT - kPanel);
        } else {
            int cb, ce;
            range(ci, cb, ce);
            const int cw = ce - cb;
            // this lane's row is finished at step my_s (if my_s < cw); it then
            // takes the row 64 further on, whose right-hand side is read now,
            // off the chain of dependent steps
            const int my_s = kFwd ? ((t - cb) & (kPanel - 1)) : ((ce - 1 - t) & (kPanel - 1));
            const int my_k = kFwd ? cb + my_s : ce - 1 - my_s;
            const int nxt = kFwd ? my_k + kPanel : my_k - kPanel;
            const double nv = z[(my_s < cw && nxt >= 0 && nxt < nb) ? nxt : 0];
            const double nval = (my_s < cw && nxt >= 0 && nxt < nb) ? nv : 0.0;
            // forward: the finished value is stored already scaled by D^-1,
            // the right-hand side of the backward solve
            const double dk = kFwd ? dinv[(my_s < cw) ? my_k : 0] : 1.0;
            double fin = 0.0;
            // a lane that finishes a row gets its first update for the next
            // row 64 - bw steps later, so for bw <= 56 the lanes finished in
            // a group of 8 steps take their next rows together after it
            const bool grouped = bw <= kPanel - 8;
            auto load_group = [&](int s0, double (&lv)[8]) {
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int st = s0 + u;
                    const int kk = st < cw ? (kFwd ? st : cw - 1 - st) : 0;
                    const int k = cb + kk;
                    const int d = kFwd ? ((t - k) & (kPanel - 1)) : ((k - t) & (kPanel - 1));
                    const bool ok = st < cw && d >= 1 && d <= bw;
                    const double x = B[ok ? kk * W + (kFwd ? d : bw - d) : 0];
                    lv[u] = ok ? x : 0.0;
                }
            };
            double lv[8], ln[8];
            load_group(0, lv);
            for (int s0 = 0; s0 < cw; s0 += 8) {
                // the next group's band entries are read while this group's steps run
                load_group(s0 + 8, ln);
                auto step = [&](int u, bool replace) {
                    const int st = s0 + u;
                    const int k = cb + (kFwd ? st : cw - 1 - st);
                    const int src = k & (kPanel - 1);
                    const double zk = readlane_f64(w, src);
                    w = __builtin_fma(-lv[u], zk, w);
                    fin = (t == src) ? zk : fin;
                    if (replace) w = (t == src) ? nval : w;
                };
                if (s0 + 8 <= cw && grouped) {
#pragma unroll
                    for (int u = 0; u < 8; u++) step(u, false);
                    const bool mine = my_s >= s0 && my_s < s0 + 8;
                    w = mine ? nval : w;
                } else {
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        if (u < cw - s0) step(u, true);
                }
#pragma unroll
                for (int u = 0; u < 8; u++) lv[u] = ln[u];
            }
            if (my_s < cw) z[my_k] = kFwd ? fin * dk : fin;
        }
        __syncthreads();
    }
}

// The triangular solves by panels of 64 rows (any bandwidth), in place on z.
__device__ __forceinline__ void panel_solves(double* z, int nb, int bw, const double* __restrict__ Lc,
                                             const double* __restrict__ Lr, const double* __restrict__ dinv,
                                             double* const (&Dbuf)[2], double (&sv)[kStagePer],
                                             double (&lv)[kPartCols], double& sd) {
    const int t = threadIdx.x, W = bw + 1;
    const int np = (nb + kPanel - 1) / kPanel;
    auto fwd_diag = [=](int p0, int pw) {
        return [=](int k, int c) -> int { return (k < pw && c <= k && k - c <= bw) ? (p0 + k) * W + bw - (k - c) : -1; };
    };
    auto bwd_diag = [=](int p0, int pw) {
        return [=](int k, int c) -> int { return (c < pw && c >= k && c - k <= bw) ? (p0 + k) * W + (c - k) : -1; };
    };
    // L z = r, panels from the top
    for (int ip = 0; ip < np; ip++) {
        const int p0 = ip * kPanel;
        const int pw = min(kPanel, nb - p0);
        const double* D = Dbuf[ip & 1];
        // rows below the panel that the band reaches: [p0 + pw, je)
        const int je = min(nb, p0 + pw + bw);
        auto below = [=](int j, int c) -> int {
            const int d = j - (p0 + c);
            return d <= bw ? (p0 + c) * W + d : -1;
        };
        const int j0 = p0 + pw + t / kPart;
        band_load(lv, j0, j0 < je, pw, Lc, below);
        if (ip + 1 < np) {
            const int q0 = p0 + kPanel, qw = min(kPanel, nb - q0);
            stage_load(sv, sd, Lr, dinv, q0, qw, fwd_diag(q0, qw));
        }
        if (t < kPanel) {
            // reads LDS only: the prefetches above stay in flight
            double v = t < pw ? z[p0 + t] : 0.0;
            for (int c0 = 0; c0 < pw; c0 += 8) {
                double dr[8];
#pragma unroll
                for (int u = 0; u < 8; u++) dr[u] = D[t * kDStride + c0 + u];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = c0 + u;
                    if (c < pw) {
                        const double zc = readlane_f64(v, c);
                        const double upd = v - dr[u] * zc;
                        v = (t == c) ? zc : ((t > c) ? upd : v);
                    }
                }
            }
            if (t < pw) z[p0 + t] = v;
        }
        __syncthreads();
        band_apply(lv, z, p0, pw, j0, j0 < je);
        for (int jp = p0 + pw + (int)kRowsPerPass; jp < je; jp += (int)kRowsPerPass) {   // bands over 256 rows
            const int j = jp + t / kPart;
            band_load(lv, j, j < je, pw, Lc, below);
            band_apply(lv, z, p0, pw, j, j < je);
        }
        if (ip + 1 < np) stage_store(Dbuf[(ip + 1) & 1], sv, sd);
        __syncthreads();
    }
    // D^-1 between the two unit triangular solves
    for (int k = t; k < nb; k += kBT) z[k] = z[k] * dinv[k];
    __syncthreads();
    // U^T y = z, panels from the bottom
    {
        const int p0 = (np - 1) * kPanel;
        stage_load(sv, sd, Lc, dinv, p0, nb - p0, bwd_diag(p0, nb - p0));
        stage_store(Dbuf[0], sv, sd);
        __syncthreads();
    }
    for (int ip = np - 1; ip >= 0; ip--) {
        const int p0 = ip * kPanel;
        const int pw = min(kPanel, nb - p0);
        const double* D = Dbuf[(np - 1 - ip) & 1];
        // rows above the panel that the band reaches: [jb, p0)
        const int jb = max(0, p0 - bw);
        auto above = [=](int j, int c) -> int {
            const int d = (p0 + c) - j;
            return d <= bw ? (p0 + c) * W + bw - d : -1;
        };
        const int j0 = jb + t / kPart;
        band_load(lv, j0, j0 < p0, pw, Lr, above);
        if (ip > 0) stage_load(sv, sd, Lc, dinv, p0 - kPanel, kPanel, bwd_diag(p0 - kPanel, kPanel));
        if (t < kPanel) {
            double v = t < pw ? z[p0 + t] : 0.0;
            for (int c1 = pw; c1 > 0; c1 -= 8) {
                double dr[8];
#pragma unroll
                for (int u = 0; u < 8; u++) dr[u] = D[t * kDStride + max(c1 - 1 - u, 0)];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = c1 - 1 - u;
                    if (c >= 0) {
                        const double yc = readlane_f64(v, c);
                        const double upd = v - dr[u] * yc;
                        v = (t == c) ? yc : ((t < c) ? upd : v);
                    }
                }
            }
            if (t < pw) z[p0 + t] = v;
        }
        __syncthreads();
        band_apply(lv, z, p0, pw, j0, j0 < p0);
        for (int jp = jb + (int)kRowsPerPass; jp < p0; jp += (int)kRowsPerPass) {
            const int j = jp + t / kPart;
            band_load(lv, j, j < p0, pw, Lr, above);
            band_apply(lv, z, p0, pw, j, j < p0);
        }
        if (ip > 0) stage_store(Dbuf[(np - ip) & 1], sv, sd);
        __syncthreads();
    }
}

__device__ void project_direct(const BlockArgs& a, int32_t b, double* dyn) {
    static_assert(kPanel * kPanel % kBT == 0 && kPanel == 64, "panel of one wave");
    const int t = threadIdx.x;
    // in-block indices fit 32 bits: a block has at most 8192 rows and 2^24 band entries
    const int64_t r0 = a.bptr[b];
    const int nb = (int)(a.bptr[b + 1] - r0);
    const int64_t s0 = a.btptr[b];
    const int ns = (int)(a.btptr[b + 1] - s0);
    const int bw = a.dbw[b], W = bw + 1;
    const double* Lc = a.lfc + a.doff[b];
    const double* Lr = a.lfr + a.doff[b];
    const double* dinv = a.ldinv + r0;
    double* z = dyn;
    double* Dbuf[2] = {dyn + nb, dyn + nb + kDiagBuf};
    double sv[kStagePer], lv[kPartCols], sd = 0.0;
    const bool narrow = bw < kPanel;
    // r = f_t - A_t x~ in factor order (all-zero rows: 0); for the panel
    // solves, the first diagonal block meanwhile
    if (!narrow) {
        const int pw = min(kPanel, nb);
        stage_load(sv, sd, Lr, dinv, 0, pw, [=](int k, int c) -> int {
            return (k < pw && c <= k && k - c <= bw) ? k * W + bw - (k - c) : -1;
        });
    }
    for (int k = t; k < nb; k += kBT) {
        const int64_t i = r0 + a.lperm[r0 + k];
        double r = 0.0;
        if (a.rinv[i] != 0.0) {
            const double d = dot_seq(a.rptr[i], a.rptr[i + 1], a.rval, a.rcol, [&](int32_t c) { return a.x[c]; });
            r = a.rf[i] - d;
        }
        z[k] = r;
    }
    if (!narrow) stage_store(Dbuf[0], sv, sd);
    __syncthreads();
    if (narrow) {
        window_solve<true>(z, nb, bw, Lc, dinv, Dbuf[0], Dbuf[1]);     // stores D^-1 z
        window_solve<false>(z, nb, bw, Lr, dinv, Dbuf[0], Dbuf[1]);
    } else {
        panel_solves(z, nb, bw, Lc, Lr, dinv, Dbuf, sv, lv, sd);
    }
    // x~ += A_t^T y on the touched columns, rows in ascending order
    for (int q = t; q < ns; q += kBT) {
        const int64_t sg = s0 + q;
        double acc = 0.0;
        for (int64_t e = a.sptr[sg]; e < a.sptr[sg + 1]; e++) acc = acc + a.sval[e] * z[a.lpos[a.srow[e]]];
        const int32_t c = a.tcol[sg];
        a.x[c] = a.x[c] + acc;
    }
    __syncthreads();
}

// Every projection of a call from the blocks' factors, one workgroup.
__global__ __launch_bounds__(kBT) void k_block_direct(BlockArgs a) {
    extern __shared__ double dyn[];
    for (int64_t sw = 0; sw < a.sweeps; sw++)
        for (int32_t j = 0; j < a.k; j++) project_direct(a, a.order[j], dyn);
}

// kMix = 1: blocks with a factor are projected from it (one-workgroup
// launches), the rest by CG; kMix = 0: CG for all (kept apart so that the CG
// forms keep their registers).
template <int kMix>
__global__ __launch_bounds__(kBT) void k_block_sweeps(BlockArgs a) {
    extern __shared__ double dyn[];
    __shared__ double lds[kBT / 64];
    __shared__ int flag;
    uint64_t episode = 0;
    const int64_t G = gridDim.x, w = blockIdx.x;
    const int t = threadIdx.x;
    // Each reduction reads, after a barrier, partials written before it; a
    // workgroup may already write the next partials while a slower one still
    // reads, so consecutive reductions never share a buffer: the loop
    // alternates pu and pr, and the start of a projection alternates between
    // two buffers of its own (it can follow a reduction of either kind, or
    // the start of the previous projection).
    double* pu = a.part;
    double* pr = a.part + G;
    for (int64_t sw = 0; sw < a.sweeps; sw++) {
        for (int32_t j = 0; j < a.k; j++) {
            double* p0 = a.part + (2 + ((sw * a.k + j) & 1)) * G;
            const int32_t b = a.order[j];
            if (kMix == 1 && a.lds_path && a.direct[b]) {
                project_direct(a, b, dyn);
                continue;
            }
            if (a.lds_path && a.fit[b]) {
                const int64_t it = project_lds(a, b, dyn, lds);
                if (t == 0) a.iters[b] += it;
                continue;
            }
            const int64_t r0 = a.bptr[b], nb = a.bptr[b + 1] - r0;
            const int64_t s0 = a.btptr[b], ns = a.btptr[b + 1] - s0;
            const int64_t ra = r0 + nb * w / G, rb = r0 + nb * (w + 1) / G;
            const int64_t sa = s0 + ns * w / G, sb = s0 + ns * (w + 1) / G;
            // res = f_R - A_R x~, p = 0
            double acc = 0.0;
            for (int64_t i = ra + t; i < rb; i += kBT) {
                double r = 0.0;
                if (a.rinv[i] != 0.0) {
                    const double d = dot_seq(a.rptr[i], a.rptr[i + 1], a.rval, a.rcol,
                                             [&](int32_t c) { return a.x[c]; });
                    r = a.rf[i] - d;
                }
                a.res[i] = r;
                a.p[i] = 0.0;
                acc = acc + r * r;
            }
            acc = wg_sum<kBT>(acc, lds);
            if (t == 0) p0[w] = acc;
            if (!grid_barrier(a.bar, a.err, &flag, episode)) return;
            double rr = wg_sum<kBT>(t < G ? p0[t] : 0.0, lds);
            const double rr0 = rr;
            const int64_t cap = a.maxit > 0 ? a.maxit : 4 * nb + 100;
            double beta = 0.0;
            int64_t it = 0;
            while (rr0 > 0.0 && rr > a.tol2 * rr0 && it < cap) {
                // phase A: u = A_R^T (res + beta p) on the touched columns
                acc = 0.0;
                for (int64_t q = sa + t; q < sb; q += kBT) {
                    const double s = dot_seq(a.sptr[q], a.sptr[q + 1], a.sval, a.srow,
                                             [&](int32_t i) { return a.res[i] + beta * a.p[i]; });
                    a.u[a.tcol[q]] = s;
                    acc = acc + s * s;
                }
                acc = wg_sum<kBT>(acc, lds);
                if (t == 0) pu[w] = acc;
                if (!grid_barrier(a.bar, a.err, &flag, episode)) return;
                const double uu = wg_sum<kBT>(t < G ? pu[t] : 0.0, lds);
                if (!(uu > 0.0)) break;
                const double alpha = rr / uu;
                // phase B: x~ += alpha u; p = res + beta p; res -= alpha A_R u
                for (int64_t q = sa + t; q < sb; q += kBT) {
                    const int32_t c = a.tcol[q];
                    a.x[c] = a.x[c] + alpha * a.u[c];
                }
                acc = 0.0;
                for (int64_t i = ra + t; i < rb; i += kBT) {
                    if (a.rinv[i] == 0.0) continue;
                    const double ri = a.res[i];
                    a.p[i] = ri + beta * a.p[i];
                    const double d = dot_seq(a.rptr[i], a.rptr[i + 1], a.rval, a.rcol,
                                             [&](int32_t c) { return a.u[c]; });
                    const double rn = ri - alpha * d;
                    a.res[i] = rn;
                    acc = acc + rn * rn;
                }
                acc = wg_sum<kBT>(acc, lds);
                if (t == 0) pr[w] = acc;
                if (!grid_barrier(a.bar, a.err, &flag, episode)) return;
                const double rn2 = wg_sum<kBT>(t < G ? pr[t] : 0.0, lds);
                beta = rn2 / rr;
                rr = rn2;
                it++;
            }
            if (w == 0 && t == 0) a.iters[b] += it;
        }
    }
}

// local index of each CSR entry's column in its block's (ascending) segment list
__global__ void k_block_local_seg(int64_t n, int32_t k, const int64_t* __restrict__ bptr,
                                  const int64_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                                  const int64_t* __restrict__ btptr, const int32_t* __restrict__ tcol,
                                  int32_t* __restrict__ lseg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = k;                // block b: bptr[b] <= i < bptr[b+1]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (bptr[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int64_t q0 = btptr[lo], q1 = btptr[lo + 1];
    for (int64_t e = rptr[i]; e < rptr[i + 1]; e++) {
        const int32_t c = rcol[e];
        int64_t a = q0, z = q1;
        while (a < z) {
            const int64_t mid = a + ((z - a) >> 1);
            if (tcol[mid] < c) a = mid + 1;
            else z = mid;
        }
        lseg[e] = (int32_t)(a - q0);
    }
}

// sum of each column segment, ascending rows
__global__ void k_seg_sums(int64_t T, const int64_t* __restrict__ sptr, const double* __restrict__ sval,
                           double* __restrict__ ssum) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    double s = 0.0;
    for (int64_t e = sptr[q]; e < sptr[q + 1]; e++) s = s + sval[e];
    ssum[q] = s;
}

// first and last touched column of each block (lo > hi: no column)
__global__ void k_block_col_range(int32_t k, const int64_t* __restrict__ btptr, const int32_t* __restrict__ tcol,
                                  int32_t* __restrict__ lohi) {
    const int32_t b = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= k) return;
    const int64_t q0 = btptr[b], q1 = btptr[b + 1];
    lohi[2 * b] = q1 > q0 ? tcol[q0] : 1;
    lohi[2 * b + 1] = q1 > q0 ? tcol[q1 - 1] : 0;
}

// Gram entry of the column sums of blocks (pairs[2p], pairs[2p+1]); one
// workgroup per pair; the columns of each block's segment list ascend.
__global__ __launch_bounds__(256) void k_block_gram(const int32_t* __restrict__ pairs,
                                                    const int64_t* __restrict__ btptr,
                                                    const int32_t* __restrict__ tcol,
                                                    const double* __restrict__ ssum, double* __restrict__ gram) {
    __shared__ double lds[4];
    const int32_t ba = pairs[2 * blockIdx.x], bb = pairs[2 * blockIdx.x + 1];
    const int64_t a0 = btptr[ba], a1 = btptr[ba + 1], b0 = btptr[bb], b1 = btptr[bb + 1];
    double acc = 0.0;
    for (int64_t q = a0 + threadIdx.x; q < a1; q += blockDim.x) {
        const int32_t c = tcol[q];
        int64_t lo = b0, hi = b1;          // first position with tcol >= c
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (tcol[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        if (lo < b1 && tcol[lo] == c) acc = acc + ssum[q] * ssum[lo];
    }
    acc = wg_sum<256>(acc, lds);
    if (threadIdx.x == 0) gram[blockIdx.x] = acc;
}

template <class T> std::vector<T> dev_to_host(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) {
        OBK_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
        OBK_HIP(hipStreamSynchronize(s));
    }
    return h;
}

template <class T> void host_to_dev(DevArray<T>& d, const std::vector<T>& h, hipStream_t s) {
    d.alloc(h.size());
    if (!h.empty()) {
        OBK_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
        OBK_HIP(hipStreamSynchronize(s));
    }
}

int32_t block_grid(const obk_plan_s& P) {
    int dev = 0, cus = 256;
    OBK_HIP(hipGetDevice(&dev));
    OBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int32_t cap = std::max(1, std::min(kBT, std::max(1, P.block_occ) * cus));
    if (P.opts.block_wgs > 0) return std::min(P.opts.block_wgs, cap);
    int64_t rows = 0;
    for (size_t b = 0; b + 1 < P.h_bptr.size(); b++) rows = std::max(rows, P.h_bptr[b + 1] - P.h_bptr[b]);
    // about two rows per thread
    return (int32_t)std::min<int64_t>(cap, std::max<int64_t>(1, (rows + 2 * kBT - 1) / (2 * kBT)));
}

// The projection kernel of a launch of G workgroups: the factors serve
// one-workgroup launches only.
struct BlockKernel { const void* fn; const char* name; };
BlockKernel block_kernel(const obk_plan_s& P, int32_t G) {
    int32_t nd = 0;
    for (int32_t d : P.h_bdirect) nd += d;
    if (G == 1 && nd > 0 && nd == P.opts.block_k)
        return {reinterpret_cast<const void*>(k_block_direct), "k_block_direct"};
    if (G == 1 && nd > 0) return {reinterpret_cast<const void*>(k_block_sweeps<1>), "k_block_sweeps"};
    return {reinterpret_cast<const void*>(k_block_sweeps<0>), "k_block_sweeps"};
}

}  // namespace

// Block ranges, centroid cosines, pairing and the projection workspace.
void block_setup(obk_plan_s& P, hipStream_t s) {
    const int32_t K = P.opts.block_k;
    const int64_t n = P.n;
    const int64_t T = P.h_tptr[K];
    host_to_dev(P.d_bptr, P.h_bptr, s);
    host_to_dev(P.d_btptr, P.h_tptr, s);
    // column sums per segment, column range per block
    DevArray<double> ssum; ssum.alloc(T);
    if (T) {
        k_seg_sums<<<nblk(T), 256, 0, s>>>(T, P.sptr.get(), P.sval.get(), ssum.get());
        OBK_HIP(hipGetLastError());
    }
    DevArray<int32_t> lohi; lohi.alloc(2 * (size_t)K);
    k_block_col_range<<<nblk(K), 256, 0, s>>>(K, P.d_btptr.get(), P.tcol.get(), lohi.get());
    OBK_HIP(hipGetLastError());
    std::vector<int32_t> hl = dev_to_host(lohi.get(), 2 * (size_t)K, s);
    // pairs of blocks that can share a column (a <= b)
    std::vector<int32_t> pairs;
    for (int32_t a = 0; a < K; a++) {
        if (hl[2 * a] > hl[2 * a + 1]) continue;
        for (int32_t b = a; b < K; b++)
            if (hl[2 * b] <= hl[2 * b + 1] && hl[2 * b] <= hl[2 * a + 1] && hl[2 * a] <= hl[2 * b + 1]) {
                pairs.push_back(a);
                pairs.push_back(b);
            }
    }
    const int64_t np = (int64_t)pairs.size() / 2;
    std::vector<double> gram;
    if (np) {
        DevArray<int32_t> dpairs; host_to_dev(dpairs, pairs, s);
        DevArray<double> dgram; dgram.alloc(np);
        k_block_gram<<<(unsigned)np, 256, 0, s>>>(dpairs.get(), P.d_btptr.get(), P.tcol.get(), ssum.get(),
                                                 dgram.get());
        OBK_HIP(hipGetLastError());
        gram = dev_to_host(dgram.get(), np, s);
    }
    std::vector<double> diag(K, 0.0);
    for (int64_t q = 0; q < np; q++)
        if (pairs[2 * q] == pairs[2 * q + 1]) diag[pairs[2 * q]] = gram[q];
    P.h_bcos.assign((size_t)K * K, 0.0);
    for (int64_t q = 0; q < np; q++) {
        const int32_t a = pairs[2 * q], b = pairs[2 * q + 1];
        if (diag[a] > 0.0 && diag[b] > 0.0) {
            const double c = std::fabs(gram[q]) / (std::sqrt(diag[a]) * std::sqrt(diag[b]));
            P.h_bcos[(size_t)a * K + b] = c;
            P.h_bcos[(size_t)b * K + a] = c;
        }
    }
    // pairing: a block not yet paired takes the least later free block with
    // |cos| below the threshold; the rest form Nclass
    P.h_partner.assign(K, -1);
    P.h_border.clear();
    for (int32_t a = 0; a < K; a++) {
        if (P.h_partner[a] >= 0) continue;
        for (int32_t b = a + 1; b < K; b++)
            if (P.h_partner[b] < 0 && P.h_bcos[(size_t)a * K + b] < P.delta) {
                P.h_partner[a] = b;
                P.h_partner[b] = a;
                P.h_border.push_back(a);
                P.h_border.push_back(b);
                break;
            }
    }
    for (int32_t a = 0; a < K; a++)
        if (P.h_partner[a] < 0) P.h_border.push_back(a);
    host_to_dev(P.d_border, P.h_border, s);
    // blocks small enough to be projected from LDS by a one-workgroup launch
    {
        const int64_t nnz_act = P.rcol.count;
        P.blseg.alloc(nnz_act);
        if (n) {
            k_block_local_seg<<<nblk(n), 256, 0, s>>>(n, K, P.d_bptr.get(), P.rptr.get(), P.rcol.get(),
                                                     P.d_btptr.get(), P.tcol.get(), P.blseg.get());
            OBK_HIP(hipGetLastError());
        }
        int dev = 0, max_lds = 0;
        OBK_HIP(hipGetDevice(&dev));
        OBK_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const int64_t budget = (int64_t)max_lds - 1024;      // room for the kernel's static LDS
        std::vector<int64_t> rp = dev_to_host(P.rptr.get(), n + 1, s);
        P.h_bfit.assign(K, 0);
        P.h_bnnz.assign(K, 0);
        P.block_lds = 0;
        for (int32_t b = 0; b < K; b++) {
            const int64_t nb = P.h_bptr[b + 1] - P.h_bptr[b];
            const int64_t ns = P.h_tptr[b + 1] - P.h_tptr[b];
            const int64_t eb = rp[P.h_bptr[b + 1]] - rp[P.h_bptr[b]];
            P.h_bnnz[b] = eb;
            const int64_t bytes = lds_bytes_for(nb, ns, eb);
            if (nb <= 65535 && ns <= 65535 && bytes <= budget) {
                P.h_bfit[b] = 1;
                P.block_lds = std::max(P.block_lds, bytes);
            }
        }
        host_to_dev(P.d_bfit, P.h_bfit, s);
        if (P.block_lds > 0)
            OBK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_block_sweeps<0>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.block_lds));
    }
    // projection workspace
    P.bres.alloc(n); P.bp.alloc(n); P.bu.alloc(n);
    P.bpart.alloc(4 * kBT);
    P.bbar.alloc(1);
    P.berr.alloc(1);
    P.biters.alloc(K);
    OBK_HIP(hipMemsetAsync(P.bu.get(), 0, std::max<int64_t>(n, 1) * sizeof(double), s));
    OBK_HIP(hipMemsetAsync(P.biters.get(), 0, K * sizeof(int64_t), s));
    OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&P.block_occ, k_block_sweeps<0>, kBT, 0));
    if (P.block_occ < 1) fail(OBK_E_HIP, "the block projection kernel cannot be resident");
    OBK_HIP(hipStreamSynchronize(s));
}

// Banded Cholesky factor of B B^T for the rows [r0, r0 + nb) of the
// reordered CSR.  The rows are first put in the reverse Cuthill-McKee order
// of the block's own Gram graph (two rows adjacent when they share a
// column): the block's rows follow the global order, which for a band of
// the matrix runs across the block, while the local order runs along it and
// keeps the factor's band narrow.  perm[k] is the block row at position k.
// Gram entries are accumulated over the columns in ascending order, then L
// row by row.  Returns the bandwidth, or -1 when the block is rank deficient
// to the pivot test, too wide, or too large.  All-zero rows (rinv 0) get a
// unit diagonal: they are decoupled and their y is 0.
constexpr int64_t kDirectMaxRows = 8192;
constexpr int64_t kDirectMaxBand = int64_t(1) << 24;     // band entries per block
constexpr int64_t kDirectMaxTotal = int64_t(1) << 27;    // band entries per plan
constexpr int64_t kDirectMaxWork = int64_t(1) << 36;     // factorisation work (rows x band^2) per plan
constexpr double kPivotTol = 1e-8;

// A block's entries (column, row within the block, value), sorted by
// (column, row) in the block's factor order once block_order has run.
struct FactorEnt { int32_t c, i; double v; };

// First stage of a block's factor: the reverse Cuthill-McKee order of its
// Gram graph (rows adjacent when they share a column) and the bandwidth of
// A_t A_t^T in that order; -1 when the block has too many rows, or its
// columns give too many row pairs, or the band would be too large (the block
// keeps CG).  Cheap next to the factorisation, so the plan-wide limits can
// be applied before any block is factored.
static int64_t block_order(int64_t r0, int64_t nb, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                           const std::vector<double>& va, std::vector<FactorEnt>& es, std::vector<int32_t>& perm) {
    if (nb <= 0 || nb > kDirectMaxRows) return -1;
    using Ent = FactorEnt;
    es.reserve((size_t)(rp[r0 + nb] - rp[r0]));
    for (int64_t i = 0; i < nb; i++)
        for (int64_t k = rp[r0 + i]; k < rp[r0 + i + 1]; k++) es.push_back({ci[k], (int32_t)i, va[k]});
    auto by_col = [](const Ent& x, const Ent& y) { return x.c != y.c ? x.c < y.c : x.i < y.i; };
    std::sort(es.begin(), es.end(), by_col);
    // a column with c entries in the block gives c^2 row pairs: a block with
    // dense columns keeps CG rather than building a large Gram graph
    int64_t pairs = 0;
    for (size_t a = 0; a < es.size();) {
        size_t e = a;
        while (e < es.size() && es[e].c == es[a].c) e++;
        pairs += (int64_t)(e - a) * (int64_t)(e - a);
        a = e;
    }
    if (pairs > kDirectMaxBand) return -1;
    // the Gram graph and its reverse Cuthill-McKee order
    std::vector<uint64_t> edges;
    for (size_t a = 0; a < es.size();) {
        size_t e = a;
        while (e < es.size() && es[e].c == es[a].c) e++;
        for (size_t p = a; p < e; p++)
            for (size_t q = a; q < e; q++)
                if (p != q) edges.push_back(((uint64_t)(uint32_t)es[p].i << 32) | (uint32_t)es[q].i);
        a = e;
    }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    std::vector<int64_t> gptr(nb + 1, 0);
    std::vector<int32_t> gadj(edges.size());
    for (size_t q = 0; q < edges.size(); q++) {
        gptr[(edges[q] >> 32) + 1]++;
        gadj[q] = (int32_t)(edges[q] & 0xffffffffu);
    }
    for (int64_t i = 0; i < nb; i++) gptr[i + 1] += gptr[i];
    perm.assign((size_t)nb, 0);
    host_rcm(nb, gptr.data(), gadj.data(), perm.data());
    std::vector<int32_t> pos((size_t)nb);
    for (int64_t k = 0; k < nb; k++) pos[perm[k]] = (int32_t)k;
    for (Ent& e : es) e.i = pos[e.i];
    std::sort(es.begin(), es.end(), by_col);
    int64_t bw = 0;
    for (size_t a = 0; a < es.size();) {
        size_t e = a;
        while (e < es.size() && es[e].c == es[a].c) e++;
        bw = std::max<int64_t>(bw, es[e - 1].i - es[a].i);
        a = e;
    }
    if (nb * (bw + 1) > kDirectMaxBand) return -1;
    return bw;
}

// Second stage: the banded Cholesky factor of A_t A_t^T in the block's order
// (row products accumulated in ascending column order); false when a pivot
// falls below kPivotTol of its diagonal (rank deficient to working accuracy).
static bool factor_block(int64_t r0, int64_t nb, int64_t bw, const std::vector<FactorEnt>& es,
                         const std::vector<double>& rinv, const std::vector<int32_t>& perm, std::vector<double>& L) {
    const int64_t W = bw + 1;
    L.assign((size_t)(nb * W), 0.0);
    auto at = [&](int64_t i, int64_t j) -> double& { return L[(size_t)(i * W + bw - (i - j))]; };
    for (size_t a = 0; a < es.size();) {
        size_t e = a;
        while (e < es.size() && es[e].c == es[a].c) e++;
        for (size_t p = a; p < e; p++)
            for (size_t q = a; q <= p; q++) at(es[p].i, es[q].i) += es[p].v * es[q].v;
        a = e;
    }
    for (int64_t k = 0; k < nb; k++)
        if (rinv[r0 + perm[k]] == 0.0) at(k, k) = 1.0;
    for (int64_t i = 0; i < nb; i++) {
        const int64_t jlo = std::max<int64_t>(0, i - bw);
        const double gii = at(i, i);
        for (int64_t j = jlo; j <= i; j++) {
            double sum = at(i, j);
            for (int64_t k = std::max<int64_t>(jlo, j - bw); k < j; k++) sum -= at(i, k) * at(j, k);
            if (j < i) {
                at(i, j) = sum / at(j, j);
            } else {
                if (!(sum > kPivotTol * gii)) return false;
                at(i, i) = std::sqrt(sum);
            }
        }
    }
    return true;
}

void block_factor(obk_plan_s& P, hipStream_t s) {
    const int32_t K = P.opts.block_k;
    P.h_bdirect.assign(K, 0);
    P.h_bbw.assign(K, -1);
    P.direct_lds = 0;
    std::vector<std::vector<double>> fac(K);
    std::vector<std::vector<int32_t>> perms(K);
    std::vector<std::vector<FactorEnt>> ents(K);
    // factors serve one-workgroup launches only: a plan whose launch spans
    // several workgroups keeps CG for every block and builds none
    const bool want = P.opts.block_solver == 0 && K > 0 && block_grid(P) == 1;
    auto parallel = [&](auto&& body) {
        std::atomic<int32_t> next{0};
        std::atomic<bool> failed{false};
        auto worker = [&] {
            for (int32_t b; (b = next.fetch_add(1)) < K;) {
                try {
                    body(b);
                } catch (...) {
                    failed = true;
                }
            }
        };
        const int nt = (int)std::max(1u, std::min<unsigned>(16u, std::min<unsigned>(
                                               (unsigned)K, std::thread::hardware_concurrency())));
        std::vector<std::thread> pool;
        for (int i = 1; i < nt; i++) {
            try {
                pool.emplace_back(worker);
            } catch (const std::system_error&) {
                break;     // fewer helper threads; the calling thread takes the rest
            }
        }
        worker();
        for (auto& th : pool) th.join();
        if (failed) fail(OBK_E_NOMEM, "host memory for the block factors");
    };
    if (want) {
        const int64_t n = P.n;
        const std::vector<int64_t> rp = dev_to_host(P.rptr.get(), n + 1, s);
        const std::vector<int32_t> ci = dev_to_host(P.rcol.get(), rp[n], s);
        const std::vector<double> va = dev_to_host(P.rval.get(), rp[n], s);
        const std::vector<double> ri = dev_to_host(P.rinv.get(), n, s);
        // 1. orders and bands of every block
        parallel([&](int32_t b) {
            P.h_bbw[b] = block_order(P.h_bptr[b], P.h_bptr[b + 1] - P.h_bptr[b], rp, ci, va, ents[b], perms[b]);
        });
        // 2. the plan-wide limits, in block order, before any factorisation:
        // the band storage and the factorisation work (rows x band^2)
        int64_t band_total = 0, work_total = 0;
        for (int32_t b = 0; b < K; b++) {
            const int64_t nb = P.h_bptr[b + 1] - P.h_bptr[b], bw = P.h_bbw[b];
            if (bw < 0) continue;
            const int64_t work = nb * (bw + 1) * (bw + 1);
            if (band_total + nb * (bw + 1) > kDirectMaxTotal || work_total + work > kDirectMaxWork) {
                P.h_bbw[b] = -1;
                std::vector<FactorEnt>().swap(ents[b]);
                continue;
            }
            band_total += nb * (bw + 1);
            work_total += work;
        }
        // 3. factors of the blocks still in; a failed pivot test releases its factor
        parallel([&](int32_t b) {
            if (P.h_bbw[b] < 0) return;
            const int64_t nb = P.h_bptr[b + 1] - P.h_bptr[b];
            if (!factor_block(P.h_bptr[b], nb, P.h_bbw[b], ents[b], ri, perms[b], fac[b])) {
                P.h_bbw[b] = -1;
                std::vector<double>().swap(fac[b]);
            }
            std::vector<FactorEnt>().swap(ents[b]);
        });
    }
    // the device footprint must stay within hbm_budget
    std::vector<int64_t> off(K, 0);
    int64_t total = 0;
    for (int32_t b = 0; b < K; b++) {
        const int64_t nb = P.h_bptr[b + 1] - P.h_bptr[b];
        if (P.h_bbw[b] < 0) continue;
        off[b] = total;
        total += nb * (P.h_bbw[b] + 1);
        P.h_bdirect[b] = 1;
    }
    const size_t extra = (size_t)(2 * total + P.n) * sizeof(double) + (size_t)(2 * P.n) * sizeof(int32_t);
    if (total > 0 && P.opts.hbm_budget && P.device_bytes() + extra > P.opts.hbm_budget) {
        P.h_bdirect.assign(K, 0);
        P.h_bbw.assign(K, -1);
        total = 0;
    }
    std::vector<int32_t> hbw(K, 0);
    for (int32_t b = 0; b < K; b++) hbw[b] = (int32_t)std::max<int64_t>(0, P.h_bbw[b]);
    host_to_dev(P.d_bdirect, P.h_bdirect, s);
    host_to_dev(P.d_bbw, hbw, s);
    host_to_dev(P.d_boff, off, s);
    std::vector<double> lc((size_t)total), lr((size_t)total), dinv((size_t)P.n, 0.0);
    std::vector<int32_t> hperm((size_t)P.n, 0), hpos((size_t)P.n, 0);
    for (int32_t b = 0; b < K; b++) {
        if (!P.h_bdirect[b]) continue;
        const int64_t nb = P.h_bptr[b + 1] - P.h_bptr[b], bw = P.h_bbw[b], W = bw + 1;
        // the unit lower factor U = L diag(1 / L[j][j]) (so that A_t A_t^T =
        // U D U^T with D = diag(L[j][j]^2)) and D^-1
        std::vector<double>& L = fac[b];
        std::vector<double> piv((size_t)nb);
        for (int64_t c = 0; c < nb; c++) piv[c] = L[(size_t)(c * W + bw)];
        for (int64_t i = 0; i < nb; i++)
            for (int64_t d = 1; d <= bw && d <= i; d++) L[(size_t)(i * W + bw - d)] /= piv[i - d];
        for (int64_t i = 0; i < nb; i++) L[(size_t)(i * W + bw)] = 1.0;
        std::copy(L.begin(), L.end(), lr.begin() + off[b]);
        for (int64_t c = 0; c < nb; c++) {
            for (int64_t d = 0; d <= bw; d++)
                lc[(size_t)(off[b] + c * W + d)] = c + d < nb ? L[(size_t)((c + d) * W + bw - d)] : 0.0;
            dinv[(size_t)(P.h_bptr[b] + c)] = 1.0 / (piv[c] * piv[c]);
            hperm[(size_t)(P.h_bptr[b] + c)] = perms[b][c];
            hpos[(size_t)(P.h_bptr[b] + perms[b][c])] = (int32_t)c;
        }
        P.direct_lds = std::max(P.direct_lds, direct_lds_for(nb));
    }
    host_to_dev(P.lfc, lc, s);
    host_to_dev(P.lfr, lr, s);
    host_to_dev(P.ldinv, dinv, s);
    host_to_dev(P.d_lperm, hperm, s);
    host_to_dev(P.d_lpos, hpos, s);
    const int64_t shmem = std::max(P.block_lds, P.direct_lds);
    if (P.direct_lds > 0) {
        OBK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_block_sweeps<1>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
        OBK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_block_direct),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.direct_lds));
    }
}

// `sweeps` block sweeps on x (device, reordered coordinates); synchronises
// the stream to check the launch's barrier flag.  ms (may be null) receives
// the launch's event time.
void block_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, float* ms) {
    if (sweeps <= 0 || P.opts.block_k <= 0) return;
    const int32_t G = block_grid(P);
    BlockArgs a{};
    a.rptr = P.rptr.get(); a.rcol = P.rcol.get(); a.rval = P.rval.get(); a.rf = P.rf.get(); a.rinv = P.rinv.get();
    a.bptr = P.d_bptr.get(); a.btptr = P.d_btptr.get();
    a.tcol = P.tcol.get(); a.sptr = P.sptr.get(); a.srow = P.srow.get(); a.sval = P.sval.get();
    a.order = P.d_border.get();
    a.x = x; a.res = P.bres.get(); a.p = P.bp.get(); a.u = P.bu.get();
    a.part = P.bpart.get(); a.bar = P.bbar.get(); a.err = P.berr.get(); a.iters = P.biters.get();
    a.sweeps = sweeps;
    a.k = P.opts.block_k;
    a.maxit = std::max(0, P.opts.block_maxit);
    a.tol2 = P.opts.block_tol * P.opts.block_tol;
    a.lseg = P.blseg.get();
    a.fit = P.d_bfit.get();
    a.direct = P.d_bdirect.get();
    a.dbw = P.d_bbw.get();
    a.doff = P.d_boff.get();
    a.lfc = P.lfc.get();
    a.lfr = P.lfr.get();
    a.ldinv = P.ldinv.get();
    a.lperm = P.d_lperm.get();
    a.lpos = P.d_lpos.get();
    const int64_t lds_need = std::max(P.block_lds, P.direct_lds);
    a.lds_path = (G == 1 && lds_need > 0) ? 1 : 0;
    const BlockKernel kern = block_kernel(P, G);
    const unsigned shmem = kern.fn == reinterpret_cast<const void*>(k_block_direct) ? (unsigned)P.direct_lds
                           : a.lds_path ? (unsigned)lds_need : 0u;
    OBK_HIP(hipMemsetAsync(P.bbar.get(), 0, sizeof(uint64_t), s));
    OBK_HIP(hipMemsetAsync(P.berr.get(), 0, sizeof(int), s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        OBK_HIP(hipEventCreate(&e0));
        OBK_HIP(hipEventCreate(&e1));
    }
    hipError_t le = hipSuccess;
    if (G == 1) {
        // one workgroup needs no co-residency guarantee: a plain launch, with
        // the events on its own dispatch packet
        if (kern.fn == reinterpret_cast<const void*>(k_block_direct))
            hipExtLaunchKernelGGL(k_block_direct, dim3(1), dim3(kBT), shmem, s, e0, e1, 0, a);
        else if (kern.fn == reinterpret_cast<const void*>(k_block_sweeps<1>))
            hipExtLaunchKernelGGL(k_block_sweeps<1>, dim3(1), dim3(kBT), shmem, s, e0, e1, 0, a);
        else
            hipExtLaunchKernelGGL(k_block_sweeps<0>, dim3(1), dim3(kBT), shmem, s, e0, e1, 0, a);
        le = hipGetLastError();
    } else {
        void* args[] = {&a};
        if (ms) OBK_HIP(hipEventRecord(e0, s));
        le = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_block_sweeps<0>), dim3(G), dim3(kBT), args,
                                        shmem, s);
        if (ms) OBK_HIP(hipEventRecord(e1, s));
    }
    auto* h = static_cast<int*>(pinned_stage(sizeof(int)));
    *h = 0;
    if (le == hipSuccess) le = hipMemcpyAsync(h, P.berr.get(), sizeof(int), hipMemcpyDeviceToHost, s);
    const hipError_t se = hipStreamSynchronize(s);
    if (ms && le == hipSuccess && se == hipSuccess) (void)hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    check_hip(le, kern.name);
    check_hip(se, "hipStreamSynchronize");
    if (*h) fail(OBK_E_HIP, "a grid barrier of the block projection launch timed out");
}

// Event time and algorithmic bytes of block sweeps (formula in obk.h).
int32_t profile_block(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                      int32_t max_out) {
    const int32_t K = P.opts.block_k;
    std::vector<int64_t> it0 = dev_to_host(P.biters.get(), K, s);
    float ms = 0;
    block_sweeps(P, x, sweeps, s, &ms);
    std::vector<int64_t> it1 = dev_to_host(P.biters.get(), K, s);
    const double sv = 8, so = 4;
    double bytes = 0;
    const bool one_wg = block_grid(P) == 1;
    for (int32_t b = 0; b < K; b++) {
        const double nb = (double)(P.h_bptr[b + 1] - P.h_bptr[b]);
        const double eb = (double)P.h_bnnz[b];
        const double tb = (double)(P.h_tptr[b + 1] - P.h_tptr[b]);
        if (one_wg && b < (int32_t)P.h_bdirect.size() && P.h_bdirect[b]) {
            // residual; the band and 1/L[i][i] once per triangular solve; x~ += A_t^T y
            const double band = nb * (double)(P.h_bbw[b] + 1);
            bytes += (double)sweeps * (eb * (sv + so) + nb * (so + 2 * sv) + tb * sv + 2 * band * sv +
                                       2 * nb * sv + eb * (sv + so) + tb * (2 * so + 2 * sv));
            continue;
        }
        const double start = eb * (sv + so) + nb * (so + 3 * sv) + tb * sv;
        const double iter = 2 * eb * (sv + so) + nb * (so + 6 * sv) + tb * (3 * so + 5 * sv);
        bytes += (double)sweeps * start + (double)(it1[b] - it0[b]) * iter;
    }
    if (max_out < 1) return 0;
    std::memset(&out[0], 0, sizeof(out[0]));
    std::strncpy(out[0].name, block_kernel(P, block_grid(P)).name, sizeof(out[0].name) - 1);
    out[0].launches = 1;
    out[0].seconds = ms * 1e-3;
    out[0].bytes = bytes;
    return 1;
}

}  // namespace obk
