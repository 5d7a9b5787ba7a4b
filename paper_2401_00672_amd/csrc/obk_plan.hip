// obk_plan: RCM reordering, row norms, row-cosine conflicts, grouping and the
// group-major relayout (Algorithm 4, first four steps, with one-row blocks).
//
// Built with -ffp-contract=off: the norms and cosines decide the grouping,
// which must come out identical to any other IEEE-754 evaluation of the same
// sums in the same (ascending column) order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "obk_internal.h"

namespace obk {
namespace {

constexpr int kT = 256;
inline unsigned nblk(int64_t n, int t = kT) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

enum : int { BAD_ROWPTR = 1, BAD_COL = 2, BAD_VAL = 4, BAD_F = 8, DUPLICATE = 16 };

// ------------------------------------------------------------- small helpers
// cptr[i] = ccount[trp[i]] (exclusive count of conflicts before row i's first
// entry), nconf when row i starts past the last entry (empty trailing rows)
__global__ void k_row_conflict_ptr(int64_t n, int64_t nnz, int64_t nconf, const int64_t* __restrict__ trp,
                                   const int64_t* __restrict__ ccount, int64_t* __restrict__ cptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) {
        const int64_t k = trp[i];
        const bool in = k < nnz;
        const int64_t c = ccount[in ? k : 0];
        cptr[i] = in ? c : nconf;
    }
}

__global__ void k_iota_u32(int64_t n, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint32_t)i;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

// ---------------------------------------------------------------- ingest
// rows nr..n-1 of the extended system: empty, right-hand side 0
__global__ void k_extend_rows(int64_t nr, int64_t n, int64_t* __restrict__ rp, double* __restrict__ f) {
    const int64_t i = nr + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        rp[i + 1] = rp[nr];
        f[i] = 0.0;
    }
}

// n: rows of the (extended) square system; ncols: columns of the caller's matrix
__global__ void k_validate(int64_t n, int64_t ncols, int64_t nnz, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v,
                           const double* __restrict__ f, int* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i <= n) {
        int64_t r = rp[i];
        if ((i == 0 && r != 0) || (i == n && r != nnz) || r < 0 || r > nnz) bad |= BAD_ROWPTR;
        if (i < n && rp[i + 1] < r) bad |= BAD_ROWPTR;
        if (i < n && !isfinite(f[i])) bad |= BAD_F;
    }
    if (i < nnz) {
        if (ci[i] < 0 || (int64_t)ci[i] >= ncols) bad |= BAD_COL;
        if (!isfinite(v[i])) bad |= BAD_VAL;
    }
    if (bad) atomicOr(flags, bad);
}

// row id of every entry of a CSR
__global__ void k_row_of(int64_t n, const int64_t* __restrict__ rp, int32_t* __restrict__ row) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) row[k] = (int32_t)i;
}

// ----------------------------------------------------- graph of A + A^T
__global__ void k_offdiag_flag(int64_t nnz, const int32_t* __restrict__ row, const int32_t* __restrict__ ci,
                               int64_t* __restrict__ flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) flag[k] = (row[k] != ci[k]) ? 2 : 0;
}

__global__ void k_offdiag_emit(int64_t nnz, const int32_t* __restrict__ row, const int32_t* __restrict__ ci,
                               const int64_t* __restrict__ pos, uint32_t* __restrict__ ra, uint32_t* __restrict__ cb) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    int32_t r = row[k], c = ci[k];
    if (r == c) return;
    int64_t p = pos[k];
    ra[p] = (uint32_t)r; cb[p] = (uint32_t)c;
    ra[p + 1] = (uint32_t)c; cb[p + 1] = (uint32_t)r;
}

// after sorting by (r, c): keep the first of each run of equal pairs
__global__ void k_unique_flag(int64_t m, const uint32_t* __restrict__ ra, const uint32_t* __restrict__ cb,
                              int64_t* __restrict__ flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t kp = k > 0 ? k - 1 : 0;
    const uint32_t r = ra[k], c = cb[k], rp = ra[kp], cp = cb[kp];
    flag[k] = ((k == 0) | (r != rp) | (c != cp)) ? 1 : 0;
}

// Written without short-circuit branches around loads: every load is issued
// unconditionally at an in-range index and the condition is combined with
// bitwise operators (the HIP compiler of ROCm 7.2 miscompiles some
// short-circuit forms; see the design notes).
__global__ void k_unique_emit(int64_t m, const uint32_t* __restrict__ ra, const uint32_t* __restrict__ cb,
                              const int64_t* __restrict__ pos, int32_t* __restrict__ adj, int32_t* __restrict__ deg) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t kp = k > 0 ? k - 1 : 0;
    const uint32_t r = ra[k], c = cb[k], rp = ra[kp], cp = cb[kp];
    const int64_t p = pos[k];
    const bool head = (k == 0) | (r != rp) | (c != cp);
    if (head) {
        adj[p] = (int32_t)c;
        atomicAdd(&deg[r], 1);
    }
}

// --------------------------------------------------- symmetric permutation
__global__ void k_inverse_perm(int64_t n, const int32_t* __restrict__ p, int32_t* __restrict__ q) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) q[p[t]] = (int32_t)t;
}

__global__ void k_perm_lengths(int64_t n, const int32_t* __restrict__ p, const int64_t* __restrict__ rp,
                               int64_t* __restrict__ len) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) len[t] = rp[p[t] + 1] - rp[p[t]];
}

// gather row p[t] into new row t, relabel columns through q
__global__ void k_perm_gather(int64_t n, const int32_t* __restrict__ p, const int32_t* __restrict__ q,
                              const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const int64_t* __restrict__ trp, uint32_t* __restrict__ key_col,
                              uint32_t* __restrict__ entry, int32_t* __restrict__ trow,
                              const double* __restrict__ f, double* __restrict__ tf) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t src = rp[p[t]], dst = trp[t], len = trp[t + 1] - trp[t];
    for (int64_t k = 0; k < len; k++) {
        key_col[dst + k] = (uint32_t)q[ci[src + k]];
        entry[dst + k] = (uint32_t)(src + k);
        trow[dst + k] = (int32_t)t;
    }
    tf[t] = f[p[t]];
}

__global__ void k_gather_u32_by(int64_t m, const uint32_t* __restrict__ idx, const int32_t* __restrict__ src,
                                uint32_t* __restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = (uint32_t)src[idx[k]];
}

// final permuted CSR entries: order[] lists original entry ids in (row, col) order
__global__ void k_perm_finish(int64_t nnz, const uint32_t* __restrict__ order, const int32_t* __restrict__ ci,
                              const int32_t* __restrict__ q, const double* __restrict__ v,
                              const int32_t* __restrict__ trow, int32_t* __restrict__ tci,
                              double* __restrict__ tv, int* flags, unsigned long long* bw) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    uint32_t e = order[k];
    int32_t c = q[ci[e]];
    tci[k] = c;
    tv[k] = v[e];
    int32_t r = trow[k];
    unsigned long long d = (unsigned long long)(r > c ? r - c : c - r);
    atomicMax(bw, d);
    (void)flags;
}

__global__ void k_dup_check(int64_t nnz, const int32_t* __restrict__ trow, const int32_t* __restrict__ tci,
                            int* flags) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int64_t kp = k > 0 ? k - 1 : 0;
    const int32_t r = trow[k], c = tci[k], rp = trow[kp], cp = tci[kp];
    if ((k > 0) & (r == rp) & (c == cp)) atomicOr(flags, DUPLICATE);
}

// --------------------------------------------------------------- norms
// nu_i = sum_k a_ik^2 in ascending k; inv_i = 1/nu_i (denominator of eq. 1.2)
__global__ void k_norms(int64_t n, const int64_t* __restrict__ trp, const double* __restrict__ tv,
                        double* __restrict__ nu, double* __restrict__ inv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t k = trp[i]; k < trp[i + 1]; k++) s = s + tv[k] * tv[k];
    nu[i] = s;
    inv[i] = (s != 0.0) ? 1.0 / s : 0.0;
}

// ------------------------------------------------------------------ CSC
__global__ void k_hist_i32(int64_t m, const uint32_t* __restrict__ key, int64_t* __restrict__ cnt) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) atomicAdd((unsigned long long*)&cnt[key[k]], 1ull);
}

__global__ void k_csc_fill(int64_t nnz, const uint32_t* __restrict__ order, const int32_t* __restrict__ trow,
                           int32_t* __restrict__ crow) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) crow[k] = trow[order[k]];
}

// CSC position of every CSR entry (the inverse of the CSC order)
__global__ void k_csc_pos(int64_t nnz, const uint32_t* __restrict__ order, uint32_t* __restrict__ cpos) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) cpos[order[k]] = (uint32_t)k;
}

// ------------------------------------------ cosine pass, per entry
// Plans of short rows (fewer than kGramMinRowLen entries per row on
// average) take these kernels: a wavefront per row would leave most lanes
// idle, while one thread per entry keeps the device full.
// One thread per entry (i, c) of A~.  For every row j < i stored in column c,
// the sparse dot a_i . a_j is taken over the common columns in ascending
// order; the pair is handled only by the entry of its first common column,
// so each pair is evaluated once.  |cos| = |d| / sqrt(nu_i * nu_j) (Section
// 3.3, one-row blocks); the pair conflicts iff |cos| >= delta.
template <bool kFill>
__global__ void k_conflicts(int64_t nnz, const int64_t* __restrict__ trp, const int32_t* __restrict__ tci,
                            const double* __restrict__ tv, const int32_t* __restrict__ trow,
                            const int64_t* __restrict__ cptr, const int32_t* __restrict__ crow,
                            const double* __restrict__ nu, double delta, int64_t* __restrict__ count,
                            const int64_t* __restrict__ out_pos, int32_t* __restrict__ out_idx) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t i = trow[e];
    const int32_t c = tci[e];
    const double nui = nu[i];
    const int64_t ia0 = trp[i], ia1 = trp[i + 1];
    const int64_t s0 = cptr[c], s1 = cptr[c + 1];
    // rows of column c are ascending: those below i are a prefix
    int64_t s_end = s0;
    for (int64_t s = s0; s < s1; s++) s_end += (crow[s] < i) ? 1 : 0;
    if (nui == 0.0) s_end = s0;
    int64_t found = 0;
    int64_t wpos = 0;
    if (kFill) wpos = out_pos[e];
    for (int64_t s = s0; s < s_end; s++) {
        const int32_t j = crow[s];
        const double nuj = nu[j];
        int64_t a = ia0, b = trp[j];
        const int64_t b1 = trp[j + 1];
        int32_t first = -1;
        double d = 0.0;
        while ((a < ia1) & (b < b1)) {
            const int32_t ca = tci[a], cb = tci[b];
            const double va = tv[a], vb = tv[b];
            const bool eq = (ca == cb);
            if (eq) d = d + va * vb;
            first = (eq & (first < 0)) ? ca : first;
            a += (ca <= cb) ? 1 : 0;
            b += (cb <= ca) ? 1 : 0;
        }
        const double cs = fabs(d) / __dsqrt_rn(nui * nuj);
        const bool conflict = (first == c) & (nuj != 0.0) & (cs >= delta);
        if (kFill && conflict) out_idx[wpos] = j;
        wpos += conflict ? 1 : 0;
        found += conflict ? 1 : 0;
    }
    if (!kFill) count[e] = found;
}

// ------------------------------------------------- group Gram row sums
// For the bound on the largest eigenvalue of B_g B_g^T (B_g: the rows of
// group g scaled to unit norm): one thread per entry (i, c); over every other
// row j of column c in i's group whose first column shared with row i is c,
// the sum of |cos(a_i, a_j)| (complex: |a_i^H a_j| / (|a_i| |a_j|)).  Each
// pair of a row's Gram row is so counted at exactly one of its entries.
// Complex plans form the bound at plan time with it; real plans form theirs
// on request (k_gm_group_cos below, the same sums over the arrays they keep).
template <bool kCplx>
__global__ void k_group_cos(int64_t nnz, const int64_t* __restrict__ trp, const int32_t* __restrict__ tci,
                            const double* __restrict__ tv, const double* __restrict__ tvi,
                            const int32_t* __restrict__ trow, const int64_t* __restrict__ cptr,
                            const int32_t* __restrict__ crow, const double* __restrict__ nu,
                            const int32_t* __restrict__ group, double* __restrict__ part) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t i = trow[e];
    const int32_t c = tci[e];
    const int32_t gi = group[i];
    double acc = 0.0;
    if (gi >= 0) {
        const double nui = nu[i];
        const int64_t ia0 = trp[i], ia1 = trp[i + 1];
        for (int64_t s = cptr[c]; s < cptr[c + 1]; s++) {
            const int32_t j = crow[s];
            if ((j == i) | (group[j] != gi)) continue;
            int64_t a = ia0, b = trp[j];
            const int64_t b1 = trp[j + 1];
            int32_t first = -1;
            double dr = 0.0, di = 0.0;
            while ((a < ia1) & (b < b1)) {
                const int32_t ca = tci[a], cb = tci[b];
                if (ca == cb) {
                    if (first < 0) first = ca;
                    if (kCplx) {   // conj(a_i) a_j
                        dr = dr + (tv[a] * tv[b] + tvi[a] * tvi[b]);
                        di = di + (tv[a] * tvi[b] - tvi[a] * tv[b]);
                    } else {
                        dr = dr + tv[a] * tv[b];
                    }
                }
                a += (ca <= cb) ? 1 : 0;
                b += (cb <= ca) ? 1 : 0;
            }
            if (first == c) {
                const double mag = kCplx ? __dsqrt_rn(dr * dr + di * di) : fabs(dr);
                acc = acc + mag / __dsqrt_rn(nui * nu[j]);
            }
        }
    }
    part[e] = acc;
}

// ------------------------------------------ cosine pass, per row
// Sparse rows of the Gram matrix A~ A~^T, one wavefront per row i (Section
// 3.3, one-row blocks: |cos_ij| = |a_i . a_j| / sqrt(nu_i nu_j)).  The
// candidates of row i are the rows j of its columns (below i for conflicts,
// other than i for the group sums), listed entry by entry in ascending column
// order and, within a column, in ascending row order; the CSC position of
// entry (i, c) (cpos) gives the rows of column c below i without a search.
// A row of at most 64 entries and kGramMaxCand candidates (counted with
// repeats) gathers its candidates into LDS at once (all loads in flight
// together), then adds a_ic a_jc into an LDS hash table keyed by j, one
// column after the other, so that every d_ij = a_i . a_j is summed over the
// common columns in ascending order -- the order of the pairwise dot
// product.  Other rows take the pairwise path: 64 candidates at a time, one
// lane each merges rows i and j, and the pair counts at its first common
// column only.
//   kGramCount: conflicts (rows j < i, nu_j != 0, |cos_ij| >= delta) per row;
//   kGramFill:  the conflict lists at row_pos[i] (hash path: ascending j;
//               pairwise path: in the order the candidates are listed).
constexpr int kGramWaves = 4;
constexpr int kGramMinRowLen = 7;    // plans with fewer entries per row on average: per-entry kernels
constexpr int kGramSlots = 512;
constexpr int kGramMaxCand = 384;
enum : int { kGramCount = 0, kGramFill = 1 };

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}
__device__ __forceinline__ int32_t wave_excl_scan(int32_t v, int lane, int32_t* total) {
    int32_t incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    *total = __shfl(incl, 63, 64);
    return incl - v;
}
// the entry e of [0, ne) whose candidate range [eoff[e], eoff[e + 1]) holds q
// (ne <= 64; a fixed number of predicated halvings)
__device__ __forceinline__ int entry_of(const int32_t* eoff, int ne, int32_t q) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int c = lo + step;
        const bool ok = (c < ne) & (eoff[c < 64 ? c : 64] <= q);
        lo = ok ? c : lo;
    }
    return lo;
}

struct GramLds {
    int32_t key[kGramSlots];
    double val[kGramSlots];
    int32_t cj[kGramMaxCand];        // candidate row, -1: not counted; later the conflict list
    double cp[kGramMaxCand];         // its product a_ic a_jc
    int32_t eoff[65];                // first candidate of each entry of the chunk
    int32_t ecol[64];
    int64_t es0[64];                 // CSC position of the entry's first candidate
    double ea[64];
};

// Written in predicated form (loads at clamped in-range indices, conditions
// combined bitwise, per-row values wave-uniform), like every kernel here.
template <int kMode>
__global__ __launch_bounds__(kGramWaves * 64) void k_row_gram(
    int64_t n, const int64_t* __restrict__ trp, const int32_t* __restrict__ tci, const double* __restrict__ tv,
    const int64_t* __restrict__ cptr, const uint32_t* __restrict__ cpos, const int32_t* __restrict__ crow,
    const double* __restrict__ cval, const double* __restrict__ nu, double delta, int64_t* __restrict__ row_count,
    const int64_t* __restrict__ row_pos, int32_t* __restrict__ out_idx) {
    __shared__ GramLds lds_all[kGramWaves];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    GramLds& L = lds_all[w];
    const int64_t row = (int64_t)blockIdx.x * kGramWaves + w;
    if (row >= n) return;                    // whole wavefronts; no block barrier follows
    const int32_t i = (int32_t)row;
    const int64_t ia0 = trp[i], ia1 = trp[i + 1];
    const double nui = nu[i];
    const bool idle = (ia0 == ia1) | (nui == 0.0);
    if (idle) {
        if (kMode == kGramCount && lane == 0) row_count[i] = 0;
        return;
    }
    int64_t found = 0;                       // conflicts so far (pairwise path)
    int64_t wpos = (kMode == kGramFill) ? row_pos[i] : 0;
    for (int64_t kb = ia0; kb < ia1; kb += 64) {
        // this chunk's entries: one lane each
        const int ne = (int)min<int64_t>(64, ia1 - kb);
        const bool kin = lane < ne;
        const int64_t k = kb + (kin ? lane : ne - 1);
        const int32_t c = tci[k];
        const double a = tv[k];
        const int64_t s0 = cptr[c];
        const int64_t pk = (int64_t)cpos[k];
        const int32_t cnt = kin ? (int32_t)(pk - s0) : 0;      // rows of column c below i
        int32_t total = 0;
        const int32_t off = wave_excl_scan(cnt, lane, &total);
        total = __builtin_amdgcn_readfirstlane(total);
        L.eoff[lane] = off;
        if (lane == 63) L.eoff[64] = total;
        L.ecol[lane] = c;
        L.es0[lane] = s0;
        L.ea[lane] = a;
        wave_sync();
        if ((kb == ia0) & (ia1 - ia0 <= 64) & (total <= kGramMaxCand)) {
            // ---- hash path: the whole row is this chunk
            for (int t = lane; t < kGramSlots; t += 64) L.key[t] = -1;
            for (int32_t qb = 0; qb < total; qb += 64) {
                const int32_t q = qb + lane;
                const bool valid = q < total;
                const int32_t qc = valid ? q : total - 1;
                const int e = entry_of(L.eoff, ne, qc);
                const int64_t sp = L.es0[e] + (qc - L.eoff[e]);
                const int32_t j = crow[sp];
                const double cv = cval[sp];
                const bool keep = j != i;
                if (valid) {
                    L.cj[q] = keep ? j : -1;
                    L.cp[q] = L.ea[e] * cv;
                }
            }
            wave_sync();
            for (int e = 0; e < ne; e++) {   // columns in ascending order
                const int32_t q0 = __builtin_amdgcn_readfirstlane(L.eoff[e]);
                const int32_t q1 = __builtin_amdgcn_readfirstlane(L.eoff[e + 1]);
                for (int32_t qb = q0; qb < q1; qb += 64) {
                    const int32_t q = qb + lane;
                    const bool valid = q < q1;
                    const int32_t qc = valid ? q : q1 - 1;
                    const int32_t j = L.cj[qc];
                    const double prod = L.cp[qc];
                    if (valid & (j >= 0)) {
                        uint32_t h = ((uint32_t)j * 0x9E3779B1u) >> (32 - 9);
                        bool done = false;
                        do {
                            const int32_t prev = atomicCAS(&L.key[h], -1, j);
                            const bool fresh = prev == -1;
                            const bool hit = fresh | (prev == j);
                            const double old = L.val[h];
                            if (hit) L.val[h] = (fresh ? 0.0 : old) + prod;
                            done = hit;
                            h = hit ? h : ((h + 1) & (kGramSlots - 1));
                        } while (!done);
                    }
                }
                wave_sync();                 // column e's sums land before column e + 1's
            }
            uint32_t mine = 0;               // bit r: slot lane + 64 r conflicts
#pragma unroll
            for (int r = 0; r < kGramSlots / 64; r++) {
                const int t = lane + 64 * r;
                const int32_t j = L.key[t];
                const double nuj = nu[j >= 0 ? j : i];
                const double cs = fabs(L.val[t]) / __dsqrt_rn(nui * nuj);
                const bool conf = (j >= 0) & (nuj != 0.0) & (cs >= delta);
                mine |= conf ? (1u << r) : 0u;
            }
            if (kMode == kGramCount) {
                const int64_t cntc = wave_sum_i64(__popc(mine));
                if (lane == 0) row_count[i] = cntc;
                return;
            }
            // compact the conflicts into cj, then place each at its rank (ascending j)
            int m = 0;
#pragma unroll
            for (int r = 0; r < kGramSlots / 64; r++) {
                const bool bit = (mine >> r) & 1u;
                const uint64_t bal = __ballot(bit);
                if (bit) L.cj[m + __popcll(bal & __lanemask_lt())] = L.key[lane + 64 * r];
                m += __popcll(bal);
            }
            wave_sync();
            for (int tb = 0; tb < m; tb += 64) {
                const int t = tb + lane;
                const bool valid = t < m;
                const int32_t j = L.cj[valid ? t : 0];
                int rank = 0;
                for (int u = 0; u < m; u++) rank += L.cj[u] < j ? 1 : 0;
                if (valid) out_idx[wpos + rank] = j;
            }
            return;
        }
        // ---- pairwise path: this chunk's candidates, 64 at a time
        for (int32_t qb = 0; qb < total; qb += 64) {
            const int32_t q = qb + lane;
            const bool valid = q < total;
            const int32_t qc = valid ? q : total - 1;
            const int e = entry_of(L.eoff, ne, qc);
            const int64_t sp = L.es0[e] + (qc - L.eoff[e]);
            const int32_t ce = L.ecol[e];
            const int32_t j = crow[sp];
            const bool take = valid & (j != i);
            int64_t x = ia0, y = trp[j];
            const int64_t y1 = take ? trp[j + 1] : y;
            int32_t first = -1;
            double d = 0.0;
            while ((x < ia1) & (y < y1)) {
                const int32_t cx = tci[x], cy = tci[y];
                const double vx = tv[x], vy = tv[y];
                const bool eq = cx == cy;
                d = eq ? d + vx * vy : d;
                first = (eq & (first < 0)) ? cx : first;
                x += (cx <= cy) ? 1 : 0;
                y += (cy <= cx) ? 1 : 0;
            }
            const double nuj = nu[j];
            const double cs = fabs(d) / __dsqrt_rn(nui * nuj);
            const bool hit = take & (first == ce) & (nuj != 0.0) & (cs >= delta);
            const uint64_t bal = __ballot(hit);
            if ((kMode == kGramFill) & hit) out_idx[wpos + __popcll(bal & __lanemask_lt())] = j;
            wpos += __popcll(bal);
            found += __popcll(bal);
        }
        wave_sync();                         // the chunk's LDS lists are read before the next chunk's
    }
    if (kMode == kGramCount && lane == 0) row_count[i] = found;
}

// 1 + the row's sum, folded into its group's maximum (non-negative doubles
// order as their bit patterns, so the maximum does not depend on the order).
// One thread per group-major row: a block whose rows all belong to one group
// (all but the blocks at group boundaries) reduces in LDS and folds once.
constexpr int kCosMaxThreads = 256;
__global__ void __launch_bounds__(kCosMaxThreads)
k_group_cos_max(int64_t m, const int32_t* __restrict__ grow, const int64_t* __restrict__ trp,
                const double* __restrict__ part, const int32_t* __restrict__ group,
                unsigned long long* __restrict__ gmax) {
    __shared__ unsigned long long red[kCosMaxThreads];
    __shared__ int g0, uniform;
    const int t = threadIdx.x;
    const int64_t a = (int64_t)blockIdx.x * kCosMaxThreads + t;
    const bool valid = a < m;
    int32_t g = -1;
    unsigned long long r = 0ull;
    if (valid) {
        const int32_t i = grow[a];
        g = group[i];
        double s = 1.0;
        for (int64_t e = trp[i]; e < trp[i + 1]; e++) s = s + part[e];
        r = (unsigned long long)__double_as_longlong(s);
    }
    if (t == 0) {
        g0 = g;
        uniform = 1;
    }
    __syncthreads();
    if (valid && g != g0) uniform = 0;
    red[t] = r;
    __syncthreads();
    if (!uniform) {
        if (valid) atomicMax(gmax + g, r);
        return;
    }
    for (int w = kCosMaxThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = red[t] > red[t + w] ? red[t] : red[t + w];
        __syncthreads();
    }
    if (t == 0) atomicMax(gmax + g0, red[0]);
}

__global__ void k_zero_u64(int64_t m, unsigned long long* __restrict__ p) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) p[k] = 0ull;
}

// ------------------------------------------ relaxation bound, on request
// A real plan forms its per-group Gershgorin bounds when they are first asked
// for, from the arrays it keeps: the group-major rows (columns ascending) and
// each group's column segments (rows ascending).  ||a||^2 of a group-major row,
// summed as the plan's norms are (ascending column, no contraction).
__global__ void k_gm_norms(int64_t m, const int64_t* __restrict__ rptr, const double* __restrict__ rval,
                           double* __restrict__ nu) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < m) {
        double s = 0.0;
        for (int64_t k = rptr[a]; k < rptr[a + 1]; k++) s = s + rval[k] * rval[k];
        nu[a] = s;
    }
}

// One thread per group-major entry (a, c) of row a in group g: over the other
// rows j of g's segment of column c whose first column shared with row a is
// c, the sum of |cos(a_a, a_j)| -- the plan-time per-entry sums, term for term
// (a group's rows keep their reordered order in its segments).
__global__ void k_gm_group_cos(int64_t nnz, const int32_t* __restrict__ erow, const int32_t* __restrict__ rgrp,
                               const int64_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                               const double* __restrict__ rval, const int64_t* __restrict__ tptr,
                               const int32_t* __restrict__ tcol, const int64_t* __restrict__ sptr,
                               const int32_t* __restrict__ srow, const double* __restrict__ nu,
                               double* __restrict__ part) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t a = erow[e];
    const int32_t g = rgrp[a];
    const int32_t c = rcol[e];
    // the segment of column c among the group's (present: row a touches c)
    int64_t lo = tptr[g], hi = tptr[g + 1];
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const bool less = tcol[mid] < c;
        lo = less ? mid + 1 : lo;
        hi = less ? hi : mid;
    }
    const int64_t s0 = sptr[lo], s1 = sptr[lo + 1];
    const double nua = nu[a];
    const int64_t a0 = rptr[a], a1 = rptr[a + 1];
    double acc = 0.0;
    for (int64_t sp = s0; sp < s1; sp++) {
        const int32_t j = srow[sp];
        const bool take = j != a;
        int64_t x = a0, y = rptr[j];
        const int64_t y1 = take ? rptr[j + 1] : y;
        int32_t first = -1;
        double d = 0.0;
        while ((x < a1) & (y < y1)) {
            const int32_t cx = rcol[x], cy = rcol[y];
            const double vx = rval[x], vy = rval[y];
            const bool eq = cx == cy;
            d = eq ? d + vx * vy : d;
            first = (eq & (first < 0)) ? cx : first;
            x += (cx <= cy) ? 1 : 0;
            y += (cy <= cx) ? 1 : 0;
        }
        const double cs = fabs(d) / __dsqrt_rn(nua * nu[j]);
        acc = (take & (first == c)) ? acc + cs : acc;
    }
    part[e] = acc;
}

// 1 + the row's sum of its entries' parts, in entry order
__global__ void k_gm_rowsum(int64_t m, const int64_t* __restrict__ rptr, const double* __restrict__ part,
                            double* __restrict__ out) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < m) {
        double s = 1.0;
        for (int64_t k = rptr[a]; k < rptr[a + 1]; k++) s = s + part[k];
        out[a] = s;
    }
}

// --------------------------------------------------------------- relayout
__global__ void k_gm_lengths(int64_t m, const int32_t* __restrict__ grow, const int64_t* __restrict__ trp,
                             int64_t* __restrict__ len) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < m) len[a] = trp[grow[a] + 1] - trp[grow[a]];
}

__global__ void k_gm_gather(int64_t m, const int32_t* __restrict__ grow, const int64_t* __restrict__ trp,
                            const int32_t* __restrict__ tci, const double* __restrict__ tv,
                            const double* __restrict__ tf, const double* __restrict__ inv,
                            const int64_t* __restrict__ rptr, int32_t* __restrict__ rcol, double* __restrict__ rval,
                            double* __restrict__ rf, double* __restrict__ rinv) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    int32_t t = grow[a];
    int64_t src = trp[t], dst = rptr[a], len = rptr[a + 1] - rptr[a];
    for (int64_t k = 0; k < len; k++) {
        rcol[dst + k] = tci[src + k];
        rval[dst + k] = tv[src + k];
    }
    rf[a] = tf[t];
    rinv[a] = inv[t];
}

// CSC entries of active rows, keyed by the group of their row
__global__ void k_csc_group_keys(int64_t nnz, const int32_t* __restrict__ crow, const int32_t* __restrict__ group,
                                 int64_t* __restrict__ keep) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) keep[k] = group[crow[k]] >= 0 ? 1 : 0;
}

__global__ void k_csc_group_emit(int64_t nnz, const int32_t* __restrict__ crow, const int32_t* __restrict__ group,
                                 const int64_t* __restrict__ pos, uint32_t* __restrict__ gkey,
                                 uint32_t* __restrict__ cidx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    int32_t g = group[crow[k]];
    if (g < 0) return;
    gkey[pos[k]] = (uint32_t)g;
    cidx[pos[k]] = (uint32_t)k;
}

// column of each CSC position: from the CSC column pointers
__global__ void k_csc_col_of(int64_t n, const int64_t* __restrict__ cptr, int32_t* __restrict__ ccol) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int64_t k = cptr[c]; k < cptr[c + 1]; k++) ccol[k] = (int32_t)c;
}

// after the stable sort by group: entries are in (group, column, row) order
__global__ void k_seg_flag(int64_t me, const uint32_t* __restrict__ gkey, const uint32_t* __restrict__ cidx,
                           const int32_t* __restrict__ ccol, int64_t* __restrict__ flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= me) return;
    const int64_t kp = k > 0 ? k - 1 : 0;
    const uint32_t g = gkey[k], gp = gkey[kp];
    const int32_t c = ccol[cidx[k]], cp = ccol[cidx[kp]];
    flag[k] = ((k == 0) | (g != gp) | (c != cp)) ? 1 : 0;
}

__global__ void k_seg_emit(int64_t me, const uint32_t* __restrict__ gkey, const uint32_t* __restrict__ cidx,
                           const int32_t* __restrict__ ccol, const int32_t* __restrict__ crow,
                           const double* __restrict__ cval, const int32_t* __restrict__ pos_of_row,
                           const int64_t* __restrict__ segpos, int32_t* __restrict__ tcol,
                           int64_t* __restrict__ sptr, int32_t* __restrict__ srow, double* __restrict__ sval,
                           int64_t* __restrict__ group_first_seg) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= me) return;
    const int64_t kp = k > 0 ? k - 1 : 0;
    const uint32_t e = cidx[k], ep = cidx[kp];
    const uint32_t g = gkey[k], gp = gkey[kp];
    const int32_t c = ccol[e], cp = ccol[ep];
    const int64_t sidx = segpos[k];
    const int32_t row_pos = pos_of_row[crow[e]];
    const double val = cval[e];
    const bool head = (k == 0) | (g != gp) | (c != cp);
    if (head) {
        tcol[sidx] = c;
        sptr[sidx] = k;
    }
    // the first entry of a group opens the group's first segment (one writer per group)
    if ((k == 0) | (g != gp)) group_first_seg[g] = sidx;
    srow[k] = row_pos;
    sval[k] = val;
}

__global__ void k_gather_f64(int64_t m, const uint32_t* __restrict__ idx, const double* __restrict__ src,
                             double* __restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = src[idx[k]];
}

__global__ void k_sumsq_rows(int64_t n, const double* __restrict__ f, const double* __restrict__ nu,
                             int only_zero_rows, double* __restrict__ partial) {
    __shared__ double red[kT];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n && (!only_zero_rows || nu[i] == 0.0)) v = f[i] * f[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_to_f32(int64_t m, const double* __restrict__ src, float* __restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = (float)src[k];
}

// Host <-> device copies of the plan go through the calling thread's pinned
// staging buffer, so that concurrent plan builds on several threads do not
// share the runtime's pageable-copy path.
template <class T> void h2d(T* d, const T* h, size_t n, hipStream_t s) {
    stage_h2d(d, h, n * sizeof(T), s);
}
template <class T> void to_device(DevArray<T>& d, const T* h, size_t n, hipStream_t s) {
    d.alloc(n);
    h2d(d.get(), h, n, s);
}
template <class T> void copy_in(DevArray<T>& d, const T* src, size_t n, bool on_dev, hipStream_t s) {
    d.alloc(n);
    if (!n) return;
    if (on_dev)
        OBK_HIP(hipMemcpyAsync(d.get(), src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
    else
        h2d(d.get(), src, n, s);
}
template <class T> std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    stage_d2h(h.data(), d, n * sizeof(T), s);
    return h;
}

double host_sum_ordered(const std::vector<double>& v) {
    double s = 0.0;
    for (double x : v) s = s + x;
    return s;
}

}  // namespace

// Deterministic sum of f_i^2 (all rows, or only rows with nu_i = 0).
double sum_squares(const double* f, const double* nu, int64_t n, bool only_zero_rows, hipStream_t s) {
    if (n <= 0) return 0.0;
    DevArray<double> part;
    part.alloc(nblk(n));
    k_sumsq_rows<<<nblk(n), kT, 0, s>>>(n, f, nu, only_zero_rows ? 1 : 0, part.get());
    OBK_HIP(hipGetLastError());
    return host_sum_ordered(to_host(part.get(), nblk(n), s));
}

// FP32 copies of the values, 1/||a||^2 and the workspace of the refinement mode
void ensure_fp32(obk_plan_s& P, hipStream_t s) {
    if (P.rval32.get()) return;
    const int64_t nnz_act = (int64_t)P.rval.count, me = (int64_t)P.sval.count, m = P.m, n = P.n;
    const size_t extra = (size_t)(nnz_act + me) * 4 + (size_t)m * 16 + (size_t)n * 4 + (size_t)m * 8;
    if (P.opts.hbm_budget && P.device_bytes() + extra > P.opts.hbm_budget)
        fail(OBK_E_NOMEM, "FP32 copies would exceed hbm_budget");
    P.rval32.alloc(nnz_act); P.rinv32.alloc(m); P.sval32.alloc(me);
    k_to_f32<<<nblk(nnz_act), kT, 0, s>>>(nnz_act, P.rval.get(), P.rval32.get());
    k_to_f32<<<nblk(m), kT, 0, s>>>(m, P.rinv.get(), P.rinv32.get());
    k_to_f32<<<nblk(me), kT, 0, s>>>(me, P.sval.get(), P.sval32.get());
    OBK_HIP(hipGetLastError());
    P.b32.alloc(m); P.d32.alloc(n); P.w32.alloc(m); P.r64.alloc(m);
    OBK_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Optional stage timing of the plan (OBK_PLAN_TRACE=1 in the environment):
// the stream is synchronised at each stage boundary and the wall time of each
// stage is printed to stderr when the plan is complete.
struct PlanTrace {
    bool on = false;
    hipStream_t s = nullptr;
    std::chrono::steady_clock::time_point t0, last;
    std::vector<std::pair<const char*, double>> marks;
    explicit PlanTrace(hipStream_t st) : s(st) {
        const char* e = std::getenv("OBK_PLAN_TRACE");
        on = e && e[0] && e[0] != '0';
        if (on) t0 = last = std::chrono::steady_clock::now();
    }
    void mark(const char* what) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        auto now = std::chrono::steady_clock::now();
        marks.emplace_back(what, std::chrono::duration<double, std::milli>(now - last).count());
        last = now;
    }
    void report(int64_t n, int64_t nnz) {
        if (!on) return;
        double tot = std::chrono::duration<double, std::milli>(last - t0).count();
        std::fprintf(stderr, "[obk-plan] n=%lld nnz=%lld total %.2f ms:", (long long)n, (long long)nnz, tot);
        for (auto& m : marks) std::fprintf(stderr, " %s %.2f", m.first, m.second);
        std::fprintf(stderr, "\n");
    }
};

// The per-group bounds of a real one-row-group plan, formed on first request
// (the largest of 1 + row sum over each group's rows).
void lambda_bound_on_request(obk_plan_s& P, hipStream_t s) {
    const int32_t G = P.ngroups;
    const int64_t m = P.m;
    const int64_t nnz = (int64_t)P.rcol.count;
    std::vector<double> bound(G, 0.0);
    if (m > 0) {
        std::vector<int32_t> rgrp(m);
        for (int32_t g = 0; g < G; g++)
            for (int64_t a = P.h_gptr[g]; a < P.h_gptr[g + 1]; a++) rgrp[a] = g;
        DevArray<int32_t> drgrp; to_device(drgrp, rgrp.data(), m, s);
        DevArray<int64_t> dtptr; to_device(dtptr, P.h_tptr.data(), (size_t)G + 1, s);
        DevArray<double> nu; nu.alloc(m);
        DevArray<double> rowsum; rowsum.alloc(m);
        DevArray<int32_t> erow; erow.alloc(nnz);
        DevArray<double> part; part.alloc(nnz);
        k_gm_norms<<<nblk(m), kT, 0, s>>>(m, P.rptr.get(), P.rval.get(), nu.get());
        k_row_of<<<nblk(m), kT, 0, s>>>(m, P.rptr.get(), erow.get());
        OBK_HIP(hipGetLastError());
        if (nnz > 0)
            k_gm_group_cos<<<nblk(nnz), kT, 0, s>>>(nnz, erow.get(), drgrp.get(), P.rptr.get(), P.rcol.get(),
                                                    P.rval.get(), dtptr.get(), P.tcol.get(), P.sptr.get(),
                                                    P.srow.get(), nu.get(), part.get());
        k_gm_rowsum<<<nblk(m), kT, 0, s>>>(m, P.rptr.get(), part.get(), rowsum.get());
        OBK_HIP(hipGetLastError());
        const std::vector<double> rs = to_host(rowsum.get(), m, s);
        for (int32_t g = 0; g < G; g++)
            for (int64_t a = P.h_gptr[g]; a < P.h_gptr[g + 1]; a++) bound[g] = std::max(bound[g], rs[a]);
    }
    P.h_lambda_bound = bound;
}

void build_plan(obk_plan_s& P, const obk_csr& A, const double* f, double delta, hipStream_t s) {
    // an m x n system with m != n is solved as its extended square system
    // (Section 4): [A, O] for m > n, [A; O] with f^ = [f; 0] for m < n
    const int64_t nr = A.n_rows, nc = A.n_cols, nnz = A.nnz;
    const int64_t n = std::max(nr, nc);
    const bool dev = A.on_device != 0;
    P.n = n; P.n_in = nc; P.m_in = nr; P.nnz = nnz; P.delta = delta; P.input_on_device = dev;
    OBK_HIP(hipGetDevice(&P.device));
    AllocScope pool(s);
    PlanTrace tr(s);

    // ---- a1: ingest and validate (square checked by the caller)
    // complex systems: values and f arrive interleaved (re, im) and travel
    // through the structural stages as separate real and imaginary arrays
    const bool cplx = P.cplx;
    DevArray<int64_t> rp; DevArray<int32_t> ci; DevArray<double> v, fd, v_im, fd_im;
    rp.alloc(n + 1);
    fd.alloc(n);
    if (cplx) fd_im.alloc(n);
    if (cplx) {
        DevArray<double> fz;
        copy_in(fz, f, 2 * nr, dev, s);
        z_split(fz.get(), nr, fd.get(), fd_im.get(), s);
        z_fill_zero(fd_im.get() + nr, n - nr, s);
        sync_for_free(s);
    }
    if (dev) {
        OBK_HIP(hipMemcpyAsync(rp.get(), A.row_ptr, (nr + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        if (nr && !cplx) OBK_HIP(hipMemcpyAsync(fd.get(), f, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        h2d(rp.get(), A.row_ptr, nr + 1, s);
        if (nr && !cplx) h2d(fd.get(), f, nr, s);
    }
    if (n > nr) {   // appended empty rows with a zero right-hand side
        k_extend_rows<<<nblk(n - nr), kT, 0, s>>>(nr, n, rp.get(), fd.get());
        OBK_HIP(hipGetLastError());
    }
    copy_in(ci, A.col, nnz, dev, s);
    if (cplx) {
        DevArray<double> vz;
        copy_in(vz, A.val, 2 * nnz, dev, s);
        v.alloc(nnz);
        v_im.alloc(nnz);
        z_split(vz.get(), nnz, v.get(), v_im.get(), s);
        sync_for_free(s);
    } else {
        copy_in(v, A.val, nnz, dev, s);
    }
    DevArray<int> flags; flags.alloc(1);
    OBK_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int), s));
    k_validate<<<nblk(std::max(n + 1, nnz)), kT, 0, s>>>(n, nc, nnz, rp.get(), ci.get(), v.get(), fd.get(),
                                                          flags.get());
    OBK_HIP(hipGetLastError());
    if (cplx) {
        z_finite(v_im.get(), nnz, flags.get(), BAD_VAL, s);
        z_finite(fd_im.get(), n, flags.get(), BAD_F, s);
    }
    int hflags = to_host(flags.get(), 1, s)[0];
    if (hflags & BAD_ROWPTR) fail(OBK_E_CSR, "row_ptr is not a monotone offset array from 0 to nnz");
    if (hflags & BAD_COL) fail(OBK_E_CSR, "column index out of range");
    if (hflags & (BAD_VAL | BAD_F)) fail(OBK_E_NONFINITE, "NaN or Inf in the matrix values or in f");

    DevArray<int32_t> row; row.alloc(nnz);
    k_row_of<<<nblk(n), kT, 0, s>>>(n, rp.get(), row.get());
    OBK_HIP(hipGetLastError());
    const int nbits = bits_for((uint64_t)std::max<int64_t>(n - 1, 0));

    tr.mark("ingest");
    // ---- a2: RCM on the pattern of A + A^T without the diagonal
    std::vector<int32_t> perm(n);
    if (P.opts.use_rcm && n > 0) {
        DevArray<int64_t> flag; flag.alloc(nnz + 1);
        k_offdiag_flag<<<nblk(nnz), kT, 0, s>>>(nnz, row.get(), ci.get(), flag.get());
        OBK_HIP(hipGetLastError());
        int64_t m2 = scan_exclusive_i64(flag.get(), flag.get(), nnz, s);
        DevArray<uint32_t> ra, cb; ra.alloc(m2); cb.alloc(m2);
        k_offdiag_emit<<<nblk(nnz), kT, 0, s>>>(nnz, row.get(), ci.get(), flag.get(), ra.get(), cb.get());
        OBK_HIP(hipGetLastError());
        // (r, c) order: stable by c, then stable by r
        radix_sort_pairs(cb.get(), ra.get(), m2, nbits, s);
        radix_sort_pairs(ra.get(), cb.get(), m2, nbits, s);
        DevArray<int64_t> uflag; uflag.alloc(m2 + 1);
        k_unique_flag<<<nblk(m2), kT, 0, s>>>(m2, ra.get(), cb.get(), uflag.get());
        OBK_HIP(hipGetLastError());
        int64_t mu = scan_exclusive_i64(uflag.get(), uflag.get(), m2, s);
        DevArray<int32_t> adj, deg; adj.alloc(mu); deg.alloc(n);
        OBK_HIP(hipMemsetAsync(deg.get(), 0, n * sizeof(int32_t), s));
        k_unique_emit<<<nblk(m2), kT, 0, s>>>(m2, ra.get(), cb.get(), uflag.get(), adj.get(), deg.get());
        OBK_HIP(hipGetLastError());
        tr.mark("rcm_graph");
        const int mode = P.opts.use_rcm;
        if (mode == 2 || (mode == 1 && n >= kDeviceRcmMinN)) {
            device_rcm(n, adj.get(), deg.get(), mode == 1, s, perm.data());
        } else {
            std::vector<int32_t> hdeg = to_host(deg.get(), n, s);
            std::vector<int32_t> hadj = to_host(adj.get(), mu, s);
            std::vector<int64_t> gptr(n + 1, 0);
            for (int64_t i = 0; i < n; i++) gptr[i + 1] = gptr[i] + hdeg[i];
            tr.mark("rcm_copy");
            host_rcm(n, gptr.data(), hadj.data(), perm.data());
        }
    } else {
        for (int64_t t = 0; t < n; t++) perm[t] = (int32_t)t;
    }
    P.h_perm = perm;
    to_device(P.perm, perm.data(), n, s);

    tr.mark("rcm");
    // ---- a3: A~ = P A P^T with rows sorted by the new column index
    DevArray<int32_t> q; q.alloc(n);
    k_inverse_perm<<<nblk(n), kT, 0, s>>>(n, P.perm.get(), q.get());
    DevArray<int64_t> trp; trp.alloc(n + 1);
    k_perm_lengths<<<nblk(n), kT, 0, s>>>(n, P.perm.get(), rp.get(), trp.get());
    OBK_HIP(hipGetLastError());
    int64_t tot = scan_exclusive_i64(trp.get(), trp.get(), n, s);
    k_set_i64<<<1, 1, 0, s>>>(trp.get() + n, tot);
    DevArray<uint32_t> kcol, entry, krow; kcol.alloc(nnz); entry.alloc(nnz); krow.alloc(nnz);
    DevArray<int32_t> trow; trow.alloc(nnz);
    DevArray<double> tf; tf.alloc(n);
    k_perm_gather<<<nblk(n), kT, 0, s>>>(n, P.perm.get(), q.get(), rp.get(), ci.get(), trp.get(), kcol.get(),
                                          entry.get(), trow.get(), fd.get(), tf.get());
    OBK_HIP(hipGetLastError());
    // sort entries by (new row, new column): stable by column, then by row
    radix_sort_pairs(kcol.get(), entry.get(), nnz, nbits, s);
    // row of each entry in the current order: the new row of the original entry
    {
        k_gather_u32_by<<<nblk(nnz), kT, 0, s>>>(nnz, entry.get(), row.get(), krow.get());   // old row ids
        OBK_HIP(hipGetLastError());
        // map old row -> new row through q
        DevArray<uint32_t> tmp; tmp.alloc(nnz);
        k_gather_u32_by<<<nblk(nnz), kT, 0, s>>>(nnz, krow.get(), q.get(), tmp.get());
        OBK_HIP(hipGetLastError());
        OBK_HIP(hipMemcpyAsync(krow.get(), tmp.get(), nnz * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        sync_for_free(s);   // tmp is freed here
    }
    radix_sort_pairs(krow.get(), entry.get(), nnz, nbits, s);
    DevArray<int32_t> tci; DevArray<double> tv; tci.alloc(nnz); tv.alloc(nnz);
    DevArray<unsigned long long> bw; bw.alloc(1);
    OBK_HIP(hipMemsetAsync(bw.get(), 0, sizeof(unsigned long long), s));
    k_perm_finish<<<nblk(nnz), kT, 0, s>>>(nnz, entry.get(), ci.get(), q.get(), v.get(), trow.get(), tci.get(),
                                           tv.get(), flags.get(), bw.get());
    OBK_HIP(hipGetLastError());
    DevArray<double> tv_im, tf_im;
    if (cplx) {
        tv_im.alloc(nnz);
        tf_im.alloc(n);
        z_gather_u32(nnz, entry.get(), v_im.get(), tv_im.get(), s);
        z_gather_i32(n, P.perm.get(), fd_im.get(), tf_im.get(), s);
    }
    k_dup_check<<<nblk(nnz), kT, 0, s>>>(nnz, trow.get(), tci.get(), flags.get());
    OBK_HIP(hipGetLastError());
    hflags = to_host(flags.get(), 1, s)[0];
    if (hflags & DUPLICATE) fail(OBK_E_CSR, "duplicate (row, col) entry");
    P.bandwidth = (int64_t)to_host(bw.get(), 1, s)[0];
    // free what the rest of the plan no longer needs
    rp = DevArray<int64_t>(); ci = DevArray<int32_t>(); v = DevArray<double>(); fd = DevArray<double>();
    v_im = DevArray<double>(); fd_im = DevArray<double>();
    row = DevArray<int32_t>(); kcol = DevArray<uint32_t>(); krow = DevArray<uint32_t>();
    entry = DevArray<uint32_t>();

    tr.mark("permute");
    // ---- a4: row norms
    DevArray<double> nu, inv; nu.alloc(n); inv.alloc(n);
    if (cplx) {
        z_norms(n, trp.get(), tv.get(), tv_im.get(), nu.get(), inv.get(), s);
    } else {
        k_norms<<<nblk(n), kT, 0, s>>>(n, trp.get(), tv.get(), nu.get(), inv.get());
        OBK_HIP(hipGetLastError());
    }
    P.fnorm2 = sum_squares(tf.get(), nu.get(), n, false, s);
    P.zero_rows_f2 = sum_squares(tf.get(), nu.get(), n, true, s);
    if (cplx) {   // |f_i|^2 = re^2 + im^2: the two parts summed apart, then added
        P.fnorm2 = P.fnorm2 + sum_squares(tf_im.get(), nu.get(), n, false, s);
        P.zero_rows_f2 = P.zero_rows_f2 + sum_squares(tf_im.get(), nu.get(), n, true, s);
    }
    {
        std::vector<double> hf = to_host(tf.get(), n, s), hn = to_host(nu.get(), n, s);
        double mx = 0.0;
        for (int64_t i = 0; i < n; i++) if (hn[i] == 0.0) mx = std::max(mx, std::fabs(hf[i]));
        P.zero_rows_fmax = mx;
    }
    if (P.opts.reject_inconsistent && P.zero_rows_f2 != 0.0)
        fail(OBK_E_INCONSISTENT, "an all-zero row has a nonzero right-hand side");

    tr.mark("norms");
    // ---- a5: CSC of A~ (rows ascending within a column), then conflicts
    DevArray<int64_t> cptr; cptr.alloc(n + 1);
    DevArray<int32_t> crow; crow.alloc(nnz);
    DevArray<double> cval; cval.alloc(nnz);
    DevArray<uint32_t> order; order.alloc(nnz);
    DevArray<uint32_t> cpos; cpos.alloc(nnz);
    int64_t csc_total = 0;
    {
        DevArray<uint32_t> ckey; ckey.alloc(nnz);
        OBK_HIP(hipMemcpyAsync(ckey.get(), tci.get(), nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        k_iota_u32<<<nblk(nnz), kT, 0, s>>>(nnz, order.get());
        OBK_HIP(hipGetLastError());
        radix_sort_pairs(ckey.get(), order.get(), nnz, nbits, s);
        OBK_HIP(hipMemsetAsync(cptr.get(), 0, (n + 1) * sizeof(int64_t), s));
        k_hist_i32<<<nblk(nnz), kT, 0, s>>>(nnz, ckey.get(), cptr.get());
        OBK_HIP(hipGetLastError());
        csc_total = scan_exclusive_i64(cptr.get(), cptr.get(), n, s);
        k_set_i64<<<1, 1, 0, s>>>(cptr.get() + n, csc_total);
        k_csc_fill<<<nblk(nnz), kT, 0, s>>>(nnz, order.get(), trow.get(), crow.get());
        OBK_HIP(hipGetLastError());
        k_gather_f64<<<nblk(nnz), kT, 0, s>>>(nnz, order.get(), tv.get(), cval.get());
        OBK_HIP(hipGetLastError());
        k_csc_pos<<<nblk(nnz), kT, 0, s>>>(nnz, order.get(), cpos.get());
        OBK_HIP(hipGetLastError());
    }
    DevArray<double> cval_im;
    if (cplx) {
        cval_im.alloc(nnz);
        z_gather_u32(nnz, order.get(), tv_im.get(), cval_im.get(), s);
    }
    std::vector<int32_t> group(n);
    if (P.block_form()) {
        // ---- block form: k uniform chunks in order (Section 3.3), the first
        // k - 1 of floor(n / k) rows, the last of the rest; every row, zero or
        // not, belongs to its block, and the residual tiles cover all rows
        const int32_t K = P.opts.block_k;
        if (K > n) fail(OBK_E_ARG, "block_k exceeds the number of rows");
        P.h_bptr.assign(K + 1, 0);
        for (int32_t b = 0; b <= K; b++) P.h_bptr[b] = (int64_t)b * (n / K);
        P.h_bptr[K] = n;
        for (int32_t b = 0; b < K; b++)
            for (int64_t i = P.h_bptr[b]; i < P.h_bptr[b + 1]; i++) group[i] = b;
        P.ngroups = K;
        P.nconflicts = 0;
        P.zero_rows_f2 = 0.0;
        P.zero_rows_fmax = 0.0;
        P.h_group = group;
        tr.mark("conflicts");
        tr.mark("groups");
    } else {
        // per-row conflict counts, their exclusive scan (the row offsets of
        // the lists, nconf at [n]), then the lists; plans of short rows take
        // one thread per entry instead of a wavefront per row
        const bool per_row_gram = nnz >= (int64_t)kGramMinRowLen * n;
        DevArray<int64_t> rconf; rconf.alloc(n + 1);
        DevArray<int32_t> cidx;
        int64_t nconf = 0;
        if (cplx || !per_row_gram) {
            // one thread per entry: counts per entry, their scan, the lists
            DevArray<int64_t> ccount; ccount.alloc(nnz + 1);
            if (cplx)
                z_conflicts(false, nnz, trp.get(), tci.get(), tv.get(), tv_im.get(), trow.get(), cptr.get(),
                            crow.get(), nu.get(), delta, ccount.get(), nullptr, nullptr, s);
            else if (nnz > 0)
                k_conflicts<false><<<nblk(nnz), kT, 0, s>>>(nnz, trp.get(), tci.get(), tv.get(), trow.get(),
                                                            cptr.get(), crow.get(), nu.get(), delta, ccount.get(),
                                                            nullptr, nullptr);
            OBK_HIP(hipGetLastError());
            nconf = scan_exclusive_i64(ccount.get(), ccount.get(), nnz, s);
            cidx.alloc(nconf);
            if (cplx)
                z_conflicts(true, nnz, trp.get(), tci.get(), tv.get(), tv_im.get(), trow.get(), cptr.get(),
                            crow.get(), nu.get(), delta, nullptr, ccount.get(), cidx.get(), s);
            else if (nnz > 0)
                k_conflicts<true><<<nblk(nnz), kT, 0, s>>>(nnz, trp.get(), tci.get(), tv.get(), trow.get(),
                                                           cptr.get(), crow.get(), nu.get(), delta, nullptr,
                                                           ccount.get(), cidx.get());
            OBK_HIP(hipGetLastError());
            // row offsets: the exclusive count at the row's first entry
            // (conflicts are emitted in entry order), nconf past the last entry
            k_row_conflict_ptr<<<nblk(n + 1), kT, 0, s>>>(n, nnz, nconf, trp.get(), ccount.get(), rconf.get());
            OBK_HIP(hipGetLastError());
            sync_for_free(s);
        } else {
            const unsigned gb = (unsigned)std::max<int64_t>(1, (n + kGramWaves - 1) / kGramWaves);
            if (n > 0)
                k_row_gram<kGramCount><<<gb, kGramWaves * 64, 0, s>>>(n, trp.get(), tci.get(), tv.get(), cptr.get(),
                                                                      cpos.get(), crow.get(), cval.get(), nu.get(),
                                                                      delta, rconf.get(), nullptr, nullptr);
            OBK_HIP(hipGetLastError());
            nconf = scan_exclusive_i64(rconf.get(), rconf.get(), n, s);
            k_set_i64<<<1, 1, 0, s>>>(rconf.get() + n, nconf);
            cidx.alloc(nconf);
            if (n > 0 && nconf > 0)
                k_row_gram<kGramFill><<<gb, kGramWaves * 64, 0, s>>>(n, trp.get(), tci.get(), tv.get(), cptr.get(),
                                                                     cpos.get(), crow.get(), cval.get(), nu.get(),
                                                                     delta, nullptr, rconf.get(), cidx.get());
            OBK_HIP(hipGetLastError());
        }
        P.nconflicts = nconf;
        tr.mark("conflicts");
        // ---- a6: first-fit grouping on the host
        std::vector<int64_t> hcptr = to_host(rconf.get(), n + 1, s);
        std::vector<int32_t> hcidx = to_host(cidx.get(), nconf, s);
        std::vector<double> hnu = to_host(nu.get(), n, s);
        std::vector<uint8_t> active(n);
        for (int64_t i = 0; i < n; i++) active[i] = hnu[i] != 0.0;
        P.ngroups = host_first_fit(n, hcptr.data(), hcidx.data(), active.data(), group.data());
        P.h_group = group;
        rconf = DevArray<int64_t>(); cidx = DevArray<int32_t>();

        tr.mark("groups");
    }
    // ---- a7: group-major relayout
    const int32_t G = P.ngroups;
    std::vector<int64_t> gsize(G + 1, 0);
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) gsize[group[i] + 1]++;
    P.h_gptr.assign(G + 1, 0);
    for (int32_t g = 0; g < G; g++) P.h_gptr[g + 1] = P.h_gptr[g] + gsize[g + 1];
    const int64_t m = P.h_gptr[G];
    P.m = m;
    std::vector<int32_t> grow(m), pos_of_row(n, -1);
    {
        std::vector<int64_t> fill(P.h_gptr.begin(), P.h_gptr.end());
        for (int64_t i = 0; i < n; i++)
            if (group[i] >= 0) { int64_t a = fill[group[i]]++; grow[a] = (int32_t)i; pos_of_row[i] = (int32_t)a; }
    }
    // device footprint check before the persistent arrays are allocated
    {
        int64_t me_est = nnz;
        size_t est = (size_t)(m + 1) * 8 + (size_t)nnz * 12 + (size_t)m * 24 + (size_t)nnz * 12 +
                     (size_t)std::min<int64_t>(me_est, (int64_t)G * n + 1) * 12 + (size_t)n * 12;
        if (cplx) est += (size_t)nnz * 16 + (size_t)m * 16 + (size_t)n * 8;   // imaginary parts, x~ and w
        if (P.block_form()) est += (size_t)n * 24 + (size_t)nnz * 4;         // CG vectors, local indices
        if (P.opts.hbm_budget && est > P.opts.hbm_budget)
            fail(OBK_E_NOMEM, "plan footprint " + std::to_string(est) + " B exceeds hbm_budget");
    }
    DevArray<int32_t> dgrow; to_device(dgrow, grow.data(), m, s);
    DevArray<int32_t> dpos; to_device(dpos, pos_of_row.data(), n, s);
    DevArray<int32_t> dgroup; to_device(dgroup, group.data(), n, s);
    if (cplx && G > 0) {
        // per-group Gershgorin bound on lambda_max(B_g B_g^H) (real plans
        // form theirs on request, from the arrays they keep)
        DevArray<double> part; part.alloc(nnz);
        DevArray<unsigned long long> gmax; gmax.alloc(G);
        k_zero_u64<<<nblk(G), kT, 0, s>>>(G, gmax.get());
        if (nnz > 0)
            k_group_cos<true><<<nblk(nnz), kT, 0, s>>>(nnz, trp.get(), tci.get(), tv.get(), tv_im.get(),
                                                       trow.get(), cptr.get(), crow.get(), nu.get(), dgroup.get(),
                                                       part.get());
        OBK_HIP(hipGetLastError());
        if (m > 0)
            k_group_cos_max<<<(unsigned)((m + kCosMaxThreads - 1) / kCosMaxThreads), kCosMaxThreads, 0, s>>>(
                m, dgrow.get(), trp.get(), part.get(), dgroup.get(), gmax.get());
        OBK_HIP(hipGetLastError());
        std::vector<unsigned long long> hm = to_host(gmax.get(), G, s);
        P.h_lambda_bound.resize(G);
        for (int32_t g = 0; g < G; g++) std::memcpy(&P.h_lambda_bound[g], &hm[g], sizeof(double));
        sync_for_free(s);
    }
    P.rptr.alloc(m + 1);
    k_gm_lengths<<<nblk(m), kT, 0, s>>>(m, dgrow.get(), trp.get(), P.rptr.get());
    OBK_HIP(hipGetLastError());
    int64_t nnz_act = scan_exclusive_i64(P.rptr.get(), P.rptr.get(), m, s);
    k_set_i64<<<1, 1, 0, s>>>(P.rptr.get() + m, nnz_act);
    P.rcol.alloc(nnz_act); P.rval.alloc(nnz_act); P.rf.alloc(m); P.rinv.alloc(m);
    k_gm_gather<<<nblk(m), kT, 0, s>>>(m, dgrow.get(), trp.get(), tci.get(), tv.get(), tf.get(), inv.get(),
                                        P.rptr.get(), P.rcol.get(), P.rval.get(), P.rf.get(), P.rinv.get());
    OBK_HIP(hipGetLastError());
    if (cplx) {   // interleaved values and f~; the real-only arrays are dropped
        P.rvalz.alloc(2 * nnz_act);
        P.rfz.alloc(2 * m);
        z_relayout(m, dgrow.get(), trp.get(), tv.get(), tv_im.get(), tf.get(), tf_im.get(), P.rptr.get(),
                   P.rvalz.get(), P.rfz.get(), s);
        sync_for_free(s);
        P.rval = DevArray<double>();
        P.rf = DevArray<double>();
    }

    tr.mark("relayout");
    // per-group CSC: CSC entries of active rows, stable-sorted by group
    DevArray<int64_t> keep; keep.alloc(nnz + 1);
    k_csc_group_keys<<<nblk(nnz), kT, 0, s>>>(nnz, crow.get(), dgroup.get(), keep.get());
    OBK_HIP(hipGetLastError());
    int64_t me = scan_exclusive_i64(keep.get(), keep.get(), nnz, s);
    DevArray<uint32_t> gkey, gidx; gkey.alloc(me); gidx.alloc(me);
    k_csc_group_emit<<<nblk(nnz), kT, 0, s>>>(nnz, crow.get(), dgroup.get(), keep.get(), gkey.get(), gidx.get());
    OBK_HIP(hipGetLastError());
    radix_sort_pairs(gkey.get(), gidx.get(), me, bits_for((uint64_t)std::max(G - 1, 0)), s);
    DevArray<int32_t> ccol; ccol.alloc(nnz);
    k_csc_col_of<<<nblk(n), kT, 0, s>>>(n, cptr.get(), ccol.get());
    OBK_HIP(hipGetLastError());
    DevArray<int64_t> segflag; segflag.alloc(me + 1);
    k_seg_flag<<<nblk(me), kT, 0, s>>>(me, gkey.get(), gidx.get(), ccol.get(), segflag.get());
    OBK_HIP(hipGetLastError());
    int64_t T = scan_exclusive_i64(segflag.get(), segflag.get(), me, s);
    P.tcol.alloc(T); P.sptr.alloc(T + 1); P.srow.alloc(me); P.sval.alloc(me);
    DevArray<int64_t> segs_g; segs_g.alloc(std::max(G, 1));
    OBK_HIP(hipMemsetAsync(segs_g.get(), 0xFF, std::max(G, 1) * sizeof(int64_t), s));   // -1: no segment
    k_seg_emit<<<nblk(me), kT, 0, s>>>(me, gkey.get(), gidx.get(), ccol.get(), crow.get(), cval.get(), dpos.get(),
                                        segflag.get(), P.tcol.get(), P.sptr.get(), P.srow.get(), P.sval.get(),
                                        segs_g.get());
    OBK_HIP(hipGetLastError());
    k_set_i64<<<1, 1, 0, s>>>(P.sptr.get() + T, me);
    if (cplx) {
        DevArray<double> sval_im; sval_im.alloc(me);
        z_gather_u32(me, gidx.get(), cval_im.get(), sval_im.get(), s);
        P.svalz.alloc(2 * me);
        z_pack(me, P.sval.get(), sval_im.get(), true, P.svalz.get(), s);   // conj(a)
        sync_for_free(s);
        P.sval = DevArray<double>();
    }
    std::vector<int64_t> hfirst = to_host(segs_g.get(), std::max(G, 1), s);
    // every group has at least one row with a nonzero entry, hence a segment;
    // a block of the block form may have none (its range is then empty)
    P.h_tptr.assign(G + 1, 0);
    P.h_tptr[G] = T;
    for (int32_t g = G - 1; g >= 0; g--) P.h_tptr[g] = hfirst[g] >= 0 ? hfirst[g] : P.h_tptr[g + 1];
    for (int32_t g = 0; g < G; g++)
        if (P.h_tptr[g] > P.h_tptr[g + 1] || P.h_tptr[g] < 0)
            fail(OBK_E_HIP, "inconsistent per-group column segments");

    tr.mark("group_csc");
    // ---- sweep schedule: tiles per group for both phases
    std::vector<int64_t> hrptr = to_host(P.rptr.get(), m + 1, s);
    std::vector<int64_t> hsptr = to_host(P.sptr.get(), T + 1, s);
    P.h_rtile_ptr.assign(G + 1, 0);
    P.h_stile_ptr.assign(G + 1, 0);
    for (int32_t g = 0; g < G; g++) {
        build_tiles(P.h_gptr[g], P.h_gptr[g + 1], hrptr.data(), P.h_rtiles);
        P.h_rtile_ptr[g + 1] = (int32_t)P.h_rtiles.size();
        build_tiles(P.h_tptr[g], P.h_tptr[g + 1], hsptr.data(), P.h_stiles);
        P.h_stile_ptr[g + 1] = (int32_t)P.h_stiles.size();
    }
    to_device(P.rtiles, P.h_rtiles.data(), P.h_rtiles.size(), s);
    to_device(P.stiles, P.h_stiles.data(), P.h_stiles.size(), s);
    to_device(P.d_rtile_ptr, P.h_rtile_ptr.data(), P.h_rtile_ptr.size(), s);
    to_device(P.d_stile_ptr, P.h_stile_ptr.data(), P.h_stile_ptr.size(), s);

    tr.mark("tiles");
    // OBK_VALIDATE=1: check the layout against its definition (host, slow)
    const char* val_env = std::getenv("OBK_VALIDATE");
    if (val_env && std::string(val_env) == "1" && !P.block_form()) {
        const int64_t ne = hrptr[m], me_ = hsptr[T];
        std::vector<int32_t> hrcol = to_host(P.rcol.get(), ne, s);
        std::vector<double> hrval = cplx ? to_host(P.rvalz.get(), 2 * ne, s) : to_host(P.rval.get(), ne, s);
        std::vector<int32_t> htcol = to_host(P.tcol.get(), T, s);
        std::vector<int32_t> hsrow = to_host(P.srow.get(), me_, s);
        std::vector<double> hsval = cplx ? to_host(P.svalz.get(), 2 * me_, s) : to_host(P.sval.get(), me_, s);
        LayoutView L;
        L.n = n; L.ngroups = G; L.gptr = P.h_gptr.data(); L.grow = grow.data(); L.group_of_row = P.h_group.data();
        L.rptr = hrptr.data(); L.rcol = hrcol.data(); L.rval = hrval.data();
        L.tptr = P.h_tptr.data(); L.tcol = htcol.data(); L.sptr = hsptr.data(); L.srow = hsrow.data();
        L.sval = hsval.data(); L.cplx = cplx; L.sval_conj = cplx; L.delta = delta;
        L.rtiles = P.h_rtiles.data(); L.rtile_ptr = P.h_rtile_ptr.data();
        L.stiles = P.h_stiles.data(); L.stile_ptr = P.h_stile_ptr.data();
        try {
            validate_layout(L);
        } catch (const Error& e) {
            fail(OBK_E_HIP, e.msg);
        }
        tr.mark("validate");
    }
    if (!cplx && !P.block_form()) slab_setup(P, hrptr, grow, pos_of_row, s);
    tr.mark("banded_engine");
    if (P.block_form()) {
        block_setup(P, s);
        block_factor(P, s);
    }
    // ---- FP32 copies for the refinement mode
    if (P.has_fp32()) ensure_fp32(P, s);

    // ---- workspace
    P.x.alloc(cplx ? 2 * n : n);
    P.w.alloc(cplx ? 2 * m : m);
    P.red.alloc(2 * std::max<size_t>(P.h_rtiles.size(), 1) + 16);   // residual partials per R tile
    OBK_HIP(hipStreamSynchronize(s));
    tr.mark("fp32_workspace");
    tr.report(n, nnz);
}

}  // namespace obk
