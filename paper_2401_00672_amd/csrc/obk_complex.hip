// Complex FP64 systems.  The paper applies Algorithm 4 unchanged to the
// complex matrix kim1 (its discussion of Table 4); over C the row norm is
// sum |a_ik|^2, the cosine of rows i, j is |a_i^H a_j| / (||a_i|| ||a_j||),
// and the row projection of eq. 1.2 is x + (f_i - a_i x) / ||a_i||^2 a_i^H.
//
// The plan reuses every structural stage of the real plan (RCM on the
// pattern, permutation, CSC, grouping, group-major relayout, tiles): values
// travel through it as separate real and imaginary arrays, and the stages
// that compute with values (norms, cosines) have complex forms here.  The
// finished plan holds the matrix values, f~, x~ and the group weights
// interleaved (re, im) so that the sweep loads one 16-byte value per entry.
//
// Every complex sum is accumulated in ascending index order with these
// operations (a = matrix entry, b = the other row's entry, x, w complex):
//   norm     s += re a re a + im a im a
//   cosine   re d += re a re b + im a im b,  im d += re a im b - im a re b
//            (d = a_i^H a_j), |cos| = sqrt(re d^2 + im d^2) / sqrt(nu_i nu_j)
//   phase R  re s += re a re x - im a im x,  im s += re a im x + im a re x,
//            w = (f - s) / ||a||^2
//   phase S  t = sum of w conj(a), x_c += t, with conj(a) stored in the
//            per-group CSC and w conj(a) formed as the plain product:
//            re = re w re a - im w (-im a), im = re w (-im a) + im w re a,
//            which equals re w re a + im w im a and im w re a - re w im a
//            bit for bit (negation is exact and a two-term sum commutes)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "obk_internal.h"
#include "obk_sweep_tiles.h"

namespace obk {

// Complex FP64 value with exactly the component operations listed above; the
// tile bodies of the real sweep run on it unchanged (the per-group CSC of a
// complex plan holds conj(a), so phase S's product w * conj(a) is the plain
// product).
struct alignas(16) zdouble {
    double re, im;
    zdouble() = default;
    __host__ __device__ constexpr zdouble(double r) : re(r), im(0.0) {}
    __host__ __device__ constexpr zdouble(double r, double i) : re(r), im(i) {}
};
__device__ __forceinline__ zdouble operator*(zdouble a, zdouble b) {
    return zdouble(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ zdouble operator+(zdouble a, zdouble b) { return zdouble(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ zdouble operator-(zdouble a, zdouble b) { return zdouble(a.re - b.re, a.im - b.im); }

namespace {

constexpr int kZT = kTileThreads;

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// ------------------------------------------------------------ plan kernels
__global__ void k_split(int64_t n, const double* __restrict__ in, double* __restrict__ re, double* __restrict__ im) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        re[i] = in[2 * i];
        im[i] = in[2 * i + 1];
    }
}

__global__ void k_fill_zero(int64_t n, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_finite(int64_t n, const double* __restrict__ a, int* __restrict__ flags, int bit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(flags, bit);
}

template <class I>
__global__ void k_gather(int64_t n, const I* __restrict__ idx, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_norms_z(int64_t n, const int64_t* __restrict__ trp, const double* __restrict__ tv,
                          const double* __restrict__ tvi, double* __restrict__ nu, double* __restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t k = trp[i]; k < trp[i + 1]; k++) s = s + (tv[k] * tv[k] + tvi[k] * tvi[k]);
    nu[i] = s;
    inv[i] = (s != 0.0) ? 1.0 / s : 0.0;
}

// One thread per entry (i, c): as the real cosine pass, with the Hermitian
// dot over the common columns of rows i and j < i.
template <bool kFill>
__global__ void k_conflicts_z(int64_t nnz, const int64_t* __restrict__ trp, const int32_t* __restrict__ tci,
                              const double* __restrict__ tv, const double* __restrict__ tvi,
                              const int32_t* __restrict__ trow, const int64_t* __restrict__ cptr,
                              const int32_t* __restrict__ crow, const double* __restrict__ nu, double delta,
                              int64_t* __restrict__ count, const int64_t* __restrict__ out_pos,
                              int32_t* __restrict__ out_idx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t i = trow[e];
    const int32_t c = tci[e];
    const double nui = nu[i];
    const int64_t ia0 = trp[i], ia1 = trp[i + 1];
    const int64_t s0 = cptr[c], s1 = cptr[c + 1];
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
        double dr = 0.0, di = 0.0;
        while ((a < ia1) & (b < b1)) {
            const int32_t ca = tci[a], cb = tci[b];
            const double ar = tv[a], ai = tvi[a], br = tv[b], bi = tvi[b];
            const bool eq = (ca == cb);
            if (eq) {
                dr = dr + (ar * br + ai * bi);
                di = di + (ar * bi - ai * br);
            }
            first = (eq & (first < 0)) ? ca : first;
            a += (ca <= cb) ? 1 : 0;
            b += (cb <= ca) ? 1 : 0;
        }
        const double cs = __dsqrt_rn(dr * dr + di * di) / __dsqrt_rn(nui * nuj);
        const bool conflict = (first == c) & (nuj != 0.0) & (cs >= delta);
        if (kFill && conflict) out_idx[wpos] = j;
        wpos += conflict ? 1 : 0;
        found += conflict ? 1 : 0;
    }
    if (!kFill) count[e] = found;
}

// group-major relayout of the values: entries and f~ interleaved
__global__ void k_gm_gather_z(int64_t m, const int32_t* __restrict__ grow, const int64_t* __restrict__ trp,
                              const double* __restrict__ tv, const double* __restrict__ tvi,
                              const double* __restrict__ tf, const double* __restrict__ tfi,
                              const int64_t* __restrict__ rptr, double2* __restrict__ rvalz,
                              double2* __restrict__ rfz) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    const int32_t t = grow[a];
    const int64_t src = trp[t], dst = rptr[a], len = rptr[a + 1] - rptr[a];
    for (int64_t k = 0; k < len; k++) rvalz[dst + k] = make_double2(tv[src + k], tvi[src + k]);
    rfz[a] = make_double2(tf[t], tfi[t]);
}

__global__ void k_pack(int64_t n, const double* __restrict__ re, const double* __restrict__ im, double sign,
                       double2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_double2(re[i], sign * im[i]);
}

// ----------------------------------------------------------- sweep kernels
// Phase R over one tile of rows: the real tile body (entries staged through
// LDS, each row summed by its owner in ascending entry order) on complex
// values, with the real scale 1/||a||^2: w_a = ((f_a - a_a x~) / ||a_a||^2) omega.
__global__ __launch_bounds__(kZT) void k_phase_r_z(const Tile* __restrict__ tiles, const int64_t* __restrict__ rptr,
                                                   const int32_t* __restrict__ rcol,
                                                   const zdouble* __restrict__ rval,
                                                   const zdouble* __restrict__ rf, const double* __restrict__ rinv,
                                                   const zdouble* __restrict__ x, zdouble* __restrict__ w,
                                                   double omega) {
    __shared__ zdouble prod[kTileEntries];
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    constexpr int64_t C = kTileEntries;
    const int nchunks = tile_chunks(t);
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x;
    const bool own = me < nseg;
    const int64_t a = t.seg_begin + (own ? me : 0);
    const int64_t k0 = rptr[a], k1 = rptr[a + 1];
    const zdouble fa = rf[a];
    const double ia = rinv[a];
    zdouble acc(0.0);
    for (int c = 0; c < nchunks; c++) {
        const int64_t base = t.ent_begin + (int64_t)c * C;
        const int len = (int)max<int64_t>(0, min<int64_t>(C, t.ent_end - base));
        stage_r<zdouble>(prod, me, len, rcol + base, rval + base, x);
        __syncthreads();
        const int64_t lo = max(k0, base), hi = own ? min(k1, base + len) : lo;
        for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        __syncthreads();
    }
    if (own) {
        const zdouble d = fa - acc;
        w[a] = zdouble((d.re * ia) * omega, (d.im * ia) * omega);
    }
}

// Phase S over one tile of touched columns: x~_c += sum over the group's rows
// (ascending) of w_a conj(a_ac), the generic tile body on conj(a).
__global__ __launch_bounds__(kZT) void k_phase_s_z(const Tile* __restrict__ tiles, const int64_t* __restrict__ sptr,
                                                   const int32_t* __restrict__ srow,
                                                   const zdouble* __restrict__ sval_conj,
                                                   const int32_t* __restrict__ tcol, const zdouble* __restrict__ w,
                                                   zdouble* __restrict__ x) {
    __shared__ zdouble prod[kTileEntries];
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    tile_phase_s<zdouble>(t, tile_chunks(t), prod, sptr, srow, sval_conj, tcol, w, x);
}

// FP64 residual over one tile of rows: sum of |r_a|^2 in a fixed tree order
// per tile, and a flag for a non-finite residual.
__global__ __launch_bounds__(kZT) void k_resid_z(const Tile* __restrict__ tiles, const int64_t* __restrict__ rptr,
                                                 const int32_t* __restrict__ rcol, const double2* __restrict__ rval,
                                                 const double2* __restrict__ rf, const double2* __restrict__ x,
                                                 double* __restrict__ psum, int* __restrict__ nonfinite) {
    __shared__ double red[kZT];
    const Tile t = tiles[blockIdx.x];
    const int64_t a = t.seg_begin + threadIdx.x;
    double r2 = 0.0;
    if (a < t.seg_end) {
        double sr = 0.0, si = 0.0;
        const int64_t e1 = rptr[a + 1];
        for (int64_t e = rptr[a]; e < e1; e++) {
            const double2 v = rval[e];
            const double2 xv = x[rcol[e]];
            sr = sr + (v.x * xv.x - v.y * xv.y);
            si = si + (v.x * xv.y + v.y * xv.x);
        }
        const double2 f = rf[a];
        const double er = f.x - sr, ei = f.y - si;
        r2 = er * er + ei * ei;
        if (!isfinite(r2)) atomicOr(nonfinite, 1);
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int st = kZT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) psum[blockIdx.x] = red[0];
}

// ordered sum of the per-tile partials by one block
__global__ void k_sum_partials(int64_t np, const double* __restrict__ psum, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) s = s + psum[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// x~ = P [x0; 0] (x0 interleaved, may be null), and x = (P^T x~)(1 : n_in)
__global__ void k_permute_in_z(int64_t n, int64_t n_in, const int32_t* __restrict__ p,
                               const double2* __restrict__ x0, double2* __restrict__ xt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = (x0 != nullptr) & (n_in > 0);     // uniform
    if (t < n) {
        const int32_t pt = p[t];
        const bool mine = pt < n_in;
        double2 val = make_double2(0.0, 0.0);
        if (have) {
            const double2 g = x0[mine ? pt : 0];
            val = mine ? g : make_double2(0.0, 0.0);
        }
        xt[t] = val;
    }
}

__global__ void k_permute_out_z(int64_t n, int64_t n_in, const int32_t* __restrict__ p,
                                const double2* __restrict__ xt, double2* __restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int32_t pt = p[t];
        if (pt < n_in) x[pt] = xt[t];
    }
}

}  // namespace

// ------------------------------------------------------ plan-stage helpers
void z_split(const double* in, int64_t n, double* re, double* im, hipStream_t s) {
    if (n <= 0) return;
    k_split<<<nblk(n), 256, 0, s>>>(n, in, re, im);
    OBK_HIP(hipGetLastError());
}

void z_fill_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_zero<<<nblk(n), 256, 0, s>>>(n, p);
    OBK_HIP(hipGetLastError());
}

void z_finite(const double* a, int64_t n, int* flags, int bit, hipStream_t s) {
    if (n <= 0) return;
    k_finite<<<nblk(n), 256, 0, s>>>(n, a, flags, bit);
    OBK_HIP(hipGetLastError());
}

void z_gather_i32(int64_t n, const int32_t* idx, const double* src, double* dst, hipStream_t s) {
    if (n <= 0) return;
    k_gather<int32_t><<<nblk(n), 256, 0, s>>>(n, idx, src, dst);
    OBK_HIP(hipGetLastError());
}

void z_gather_u32(int64_t n, const uint32_t* idx, const double* src, double* dst, hipStream_t s) {
    if (n <= 0) return;
    k_gather<uint32_t><<<nblk(n), 256, 0, s>>>(n, idx, src, dst);
    OBK_HIP(hipGetLastError());
}

void z_norms(int64_t n, const int64_t* trp, const double* tv, const double* tvi, double* nu, double* inv,
             hipStream_t s) {
    if (n <= 0) return;
    k_norms_z<<<nblk(n), 256, 0, s>>>(n, trp, tv, tvi, nu, inv);
    OBK_HIP(hipGetLastError());
}

void z_conflicts(bool fill, int64_t nnz, const int64_t* trp, const int32_t* tci, const double* tv, const double* tvi,
                 const int32_t* trow, const int64_t* cptr, const int32_t* crow, const double* nu, double delta,
                 int64_t* count, const int64_t* out_pos, int32_t* out_idx, hipStream_t s) {
    if (nnz <= 0) return;
    if (fill)
        k_conflicts_z<true><<<nblk(nnz), 256, 0, s>>>(nnz, trp, tci, tv, tvi, trow, cptr, crow, nu, delta, nullptr,
                                                      out_pos, out_idx);
    else
        k_conflicts_z<false><<<nblk(nnz), 256, 0, s>>>(nnz, trp, tci, tv, tvi, trow, cptr, crow, nu, delta, count,
                                                       nullptr, nullptr);
    OBK_HIP(hipGetLastError());
}

void z_relayout(int64_t m, const int32_t* grow, const int64_t* trp, const double* tv, const double* tvi,
                const double* tf, const double* tfi, const int64_t* rptr, double* rvalz, double* rfz,
                hipStream_t s) {
    if (m <= 0) return;
    k_gm_gather_z<<<nblk(m), 256, 0, s>>>(m, grow, trp, tv, tvi, tf, tfi, rptr, reinterpret_cast<double2*>(rvalz),
                                          reinterpret_cast<double2*>(rfz));
    OBK_HIP(hipGetLastError());
}

void z_pack(int64_t n, const double* re, const double* im, bool conjugate, double* out, hipStream_t s) {
    if (n <= 0) return;
    k_pack<<<nblk(n), 256, 0, s>>>(n, re, im, conjugate ? -1.0 : 1.0, reinterpret_cast<double2*>(out));
    OBK_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ sweeps
static void enqueue_sweeps_zt(const obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    const zdouble* rv = reinterpret_cast<const zdouble*>(P.rvalz.get());
    const zdouble* rf = reinterpret_cast<const zdouble*>(P.rfz.get());
    const zdouble* sv = reinterpret_cast<const zdouble*>(P.svalz.get());
    zdouble* xz = reinterpret_cast<zdouble*>(x);
    zdouble* wz = reinterpret_cast<zdouble*>(P.w.get());
    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < P.ngroups; g++) {
            const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
            const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
            if (r1 > r0)
                k_phase_r_z<<<r1 - r0, kZT, 0, s>>>(P.rtiles.get() + r0, P.rptr.get(), P.rcol.get(), rv, rf,
                                                    P.rinv.get(), xz, wz, P.opts.omega);
            if (s1 > s0)
                k_phase_s_z<<<s1 - s0, kZT, 0, s>>>(P.stiles.get() + s0, P.sptr.get(), P.srow.get(), sv,
                                                    P.tcol.get(), wz, xz);
        }
    }
    OBK_HIP(hipGetLastError());
}

// `sweeps` complex sweeps on x (device, reordered, interleaved), replayed from
// graphs of whole sweeps captured per iterate pointer and sweep count
void enqueue_sweeps_z(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    if (sweeps <= 0 || P.ngroups == 0) return;
    constexpr int64_t kChunkZ = 8;
    auto graph_for = [&](int64_t count) -> hipGraphExec_t {
        for (auto& g : P.graphs)
            if (g.x == (const void*)x && g.sweeps == count && g.elem == 16 && g.exec) return g.exec;
        if (!P.capture_stream) OBK_HIP(hipStreamCreateWithFlags(&P.capture_stream, hipStreamNonBlocking));
        obk_plan_s::SweepGraph sg;
        sg.x = x; sg.sweeps = count; sg.elem = 16;
        OBK_HIP(hipStreamBeginCapture(P.capture_stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_sweeps_zt(P, x, count, P.capture_stream);
        } catch (...) {
            hipGraph_t dummy = nullptr;
            (void)hipStreamEndCapture(P.capture_stream, &dummy);
            if (dummy) (void)hipGraphDestroy(dummy);
            throw;
        }
        OBK_HIP(hipStreamEndCapture(P.capture_stream, &sg.graph));
        OBK_HIP(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
        P.graphs.push_back(sg);
        return sg.exec;
    };
    // both graphs are captured on the iterate's first use (see run_sweeps)
    hipGraphExec_t chunk = graph_for(kChunkZ), one = graph_for(1);
    for (int64_t i = 0; i + kChunkZ <= sweeps; i += kChunkZ) OBK_HIP(hipGraphLaunch(chunk, s));
    for (int64_t i = 0; i < sweeps % kChunkZ; i++) OBK_HIP(hipGraphLaunch(one, s));
}

// Eager complex sweeps with an event pair on every kernel's dispatch packet;
// per-kernel sums of event time and algorithmic bytes (formulas in obk.h,
// with s = 16 for values, f~, w and x~).
int32_t profile_sweeps_z(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                         int32_t max_out) {
    const int32_t G = P.ngroups;
    const double sv = 16, so = 4;
    std::vector<double> rbytes(G, 0.0), sbytes(G, 0.0);
    for (int32_t g = 0; g < G; g++) {
        double ng = 0, eg = 0, tg = 0;
        for (int32_t t = P.h_rtile_ptr[g]; t < P.h_rtile_ptr[g + 1]; t++) {
            ng += P.h_rtiles[t].seg_end - P.h_rtiles[t].seg_begin;
            eg += (double)(P.h_rtiles[t].ent_end - P.h_rtiles[t].ent_begin);
        }
        for (int32_t t = P.h_stile_ptr[g]; t < P.h_stile_ptr[g + 1]; t++)
            tg += P.h_stiles[t].seg_end - P.h_stiles[t].seg_begin;
        // R: values and columns; offset, f~, w per row and 1/||a||^2 (8 B); x~ once per touched column
        rbytes[g] = eg * (sv + so) + ng * (so + 2 * sv + 8) + tg * sv;
        // S: values and row ids; offset, id, x~ read and write per touched column; w once per row
        sbytes[g] = eg * (sv + so) + tg * (2 * so + 2 * sv) + ng * sv;
    }
    const zdouble* rv = reinterpret_cast<const zdouble*>(P.rvalz.get());
    const zdouble* rf = reinterpret_cast<const zdouble*>(P.rfz.get());
    const zdouble* svz = reinterpret_cast<const zdouble*>(P.svalz.get());
    zdouble* xz = reinterpret_cast<zdouble*>(x);
    zdouble* wz = reinterpret_cast<zdouble*>(P.w.get());
    struct L { int kind; double bytes; hipEvent_t a, b; };
    std::vector<L> ls;
    struct Guard {
        std::vector<L>& v;
        ~Guard() { for (auto& l : v) { if (l.a) (void)hipEventDestroy(l.a); if (l.b) (void)hipEventDestroy(l.b); } }
    } guard{ls};
    for (int64_t it = 0; it < sweeps; it++)
        for (int32_t g = 0; g < G; g++) {
            const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
            const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
            if (r1 > r0) {
                L l{0, rbytes[g], nullptr, nullptr};
                OBK_HIP(hipEventCreate(&l.a));
                OBK_HIP(hipEventCreate(&l.b));
                ls.push_back(l);
                hipExtLaunchKernelGGL(k_phase_r_z, dim3(r1 - r0), dim3(kZT), 0, s, l.a, l.b, 0,
                                      (const Tile*)(P.rtiles.get() + r0), (const int64_t*)P.rptr.get(),
                                      (const int32_t*)P.rcol.get(), rv, rf, (const double*)P.rinv.get(),
                                      (const zdouble*)xz, wz, P.opts.omega);
            }
            if (s1 > s0) {
                L l{1, sbytes[g], nullptr, nullptr};
                OBK_HIP(hipEventCreate(&l.a));
                OBK_HIP(hipEventCreate(&l.b));
                ls.push_back(l);
                hipExtLaunchKernelGGL(k_phase_s_z, dim3(s1 - s0), dim3(kZT), 0, s, l.a, l.b, 0,
                                      (const Tile*)(P.stiles.get() + s0), (const int64_t*)P.sptr.get(),
                                      (const int32_t*)P.srow.get(), svz, (const int32_t*)P.tcol.get(),
                                      (const zdouble*)wz, xz);
            }
        }
    OBK_HIP(hipGetLastError());
    OBK_HIP(hipStreamSynchronize(s));
    const char* names[2] = {"k_phase_r_z", "k_phase_s_z"};
    obk_kernel_profile acc[2];
    for (int j = 0; j < 2; j++) {
        std::memset(&acc[j], 0, sizeof(acc[j]));
        std::strncpy(acc[j].name, names[j], sizeof(acc[j].name) - 1);
    }
    for (auto& l : ls) {
        float ms = 0;
        OBK_HIP(hipEventElapsedTime(&ms, l.a, l.b));
        acc[l.kind].launches++;
        acc[l.kind].seconds += ms * 1e-3;
        acc[l.kind].bytes += l.bytes;
    }
    int32_t nout = 0;
    for (int j = 0; j < 2 && nout < max_out; j++)
        if (acc[j].launches) out[nout++] = acc[j];
    return nout;
}

// relative residual ||f~ - A~ x~|| / ||f~|| over C (synchronises the stream)
static double relres_z(const obk_plan_s& P, const double* x, hipStream_t s, bool* nonfinite) {
    const int64_t nt = (int64_t)P.h_rtiles.size();
    double* psum = P.red.get();
    double* out = psum + std::max<int64_t>(nt, 1);
    int* flag = reinterpret_cast<int*>(out + 2);
    OBK_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    if (nt)
        k_resid_z<<<(unsigned)nt, kZT, 0, s>>>(P.rtiles.get(), P.rptr.get(), P.rcol.get(),
                                               reinterpret_cast<const double2*>(P.rvalz.get()),
                                               reinterpret_cast<const double2*>(P.rfz.get()),
                                               reinterpret_cast<const double2*>(x), psum, flag);
    k_sum_partials<<<1, 256, 0, s>>>(nt, psum, out);
    OBK_HIP(hipGetLastError());
    auto* h = static_cast<double*>(pinned_stage(2 * sizeof(double)));
    OBK_HIP(hipMemcpyAsync(h, out, sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipMemcpyAsync(h + 1, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    int nf = 0;
    std::memcpy(&nf, h + 1, sizeof(int));
    const double r2 = h[0] + P.zero_rows_f2;
    if (nonfinite) *nonfinite = nf != 0 || !std::isfinite(r2);
    if (P.fnorm2 == 0.0) return r2 == 0.0 ? 0.0 : INFINITY;
    return std::sqrt(r2) / std::sqrt(P.fnorm2);
}

// obk_solve on a complex plan (x0 and x interleaved, n_in complex entries)
void solve_complex(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = P.n;
    const bool dev = P.input_on_device;
    obk_info inf{};
    inf.relres = -1;
    DevArray<double> x0d, xd;
    const double* x0dev = nullptr;
    if (x0) {
        if (dev) x0dev = x0;
        else {
            x0d.alloc(2 * P.n_in);
            OBK_HIP(hipMemcpyAsync(x0d.get(), x0, 2 * P.n_in * sizeof(double), hipMemcpyHostToDevice, s));
            x0dev = x0d.get();
        }
    }
    k_permute_in_z<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), reinterpret_cast<const double2*>(x0dev),
                                           reinterpret_cast<double2*>(P.x.get()));
    OBK_HIP(hipGetLastError());
    bool nf = false;
    inf.relres0 = relres_z(P, P.x.get(), s, &nf);
    inf.relres = inf.relres0;
    inf.status = OBK_MAXIT;
    const int64_t every = std::max(1, P.opts.check_every);
    int64_t done = 0;
    if (nf) inf.status = OBK_NONFINITE_ITERATE;
    else if (tol > 0 && inf.relres0 <= tol) inf.status = OBK_CONVERGED;
    while (done < maxit && inf.status == OBK_MAXIT) {
        const int64_t chunk = (tol > 0) ? std::min(every, maxit - done) : (maxit - done);
        enqueue_sweeps_z(P, P.x.get(), chunk, s);
        done += chunk;
        if (tol > 0) {
            inf.outer_steps++;
            inf.relres = relres_z(P, P.x.get(), s, &nf);
            if (nf) inf.status = OBK_NONFINITE_ITERATE;
            else if (inf.relres <= tol) inf.status = OBK_CONVERGED;
            else if (inf.relres > 1e3 * inf.relres0 && inf.relres0 > 0) inf.status = OBK_DIVERGED;
        }
    }
    if (tol <= 0) inf.relres = relres_z(P, P.x.get(), s, &nf);
    inf.sweeps = done;
    double* xout = x;
    if (!dev) { xd.alloc(2 * P.n_in); xout = xd.get(); }
    k_permute_out_z<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), reinterpret_cast<const double2*>(P.x.get()),
                                            reinterpret_cast<double2*>(xout));
    OBK_HIP(hipGetLastError());
    if (!dev) OBK_HIP(hipMemcpyAsync(x, xd.get(), 2 * P.n_in * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
}

}  // namespace obk
