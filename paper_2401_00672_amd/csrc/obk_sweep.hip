// The orthogonal-group block Kaczmarz sweep (eq. 3.3 with one-row blocks;
// eq. 1.3 when a group's rows are exactly orthogonal) and its residual.
//
// One sweep = for every group g in ascending order
//   phase R: w_a = (f_a - sum_k a_ak x_k) / ||a_a||^2 for every row a of g,
//            all from the same x (rows are stored group-major, so a group is
//            one contiguous CSR range);
//   phase S: for every column c touched by g, x_c += sum_a w_a a_ac, owned by
//            exactly one thread (the group's CSC), so no atomics are needed.
// Both phases stream their entries through LDS in tiles and reduce each row
// (column) sequentially in ascending entry order.
#include <chrono>
#include <cmath>
#include <vector>

#include "obk_internal.h"

namespace obk {

double sum_squares(const double* f, const double* nu, int64_t n, bool only_zero_rows, hipStream_t s);

namespace {

constexpr int kT = kTileThreads;
inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// Phase R over the tiles of one group.
__global__ __launch_bounds__(kT) void k_phase_r(const Tile* __restrict__ tiles, const int64_t* __restrict__ rptr,
                                                const int32_t* __restrict__ rcol, const double* __restrict__ rval,
                                                const double* __restrict__ rf, const double* __restrict__ rinv,
                                                const double* __restrict__ x, double* __restrict__ w) {
    __shared__ double prod[kTileEntries];
    const Tile t = tiles[blockIdx.x];
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x;
    int64_t k0 = 0, k1 = 0;
    if (me < nseg) { k0 = rptr[t.seg_begin + me]; k1 = rptr[t.seg_begin + me + 1]; }
    double acc = 0.0;
    for (int64_t base = t.ent_begin; base < t.ent_end; base += kTileEntries) {
        const int len = (int)min<int64_t>(kTileEntries, t.ent_end - base);
        for (int q = me; q < len; q += kT) prod[q] = rval[base + q] * x[rcol[base + q]];
        __syncthreads();
        if (me < nseg) {
            const int64_t lo = max(k0, base), hi = min(k1, base + len);
            for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        }
        __syncthreads();
    }
    if (me < nseg) {
        const int64_t a = t.seg_begin + me;
        w[a] = (rf[a] - acc) * rinv[a];
    }
}

// Phase S over the tiles of one group's touched columns.
__global__ __launch_bounds__(kT) void k_phase_s(const Tile* __restrict__ tiles, const int64_t* __restrict__ sptr,
                                                const int32_t* __restrict__ srow, const double* __restrict__ sval,
                                                const int32_t* __restrict__ tcol, const double* __restrict__ w,
                                                double* __restrict__ x) {
    __shared__ double prod[kTileEntries];
    const Tile t = tiles[blockIdx.x];
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x;
    int64_t k0 = 0, k1 = 0;
    if (me < nseg) { k0 = sptr[t.seg_begin + me]; k1 = sptr[t.seg_begin + me + 1]; }
    double acc = 0.0;
    for (int64_t base = t.ent_begin; base < t.ent_end; base += kTileEntries) {
        const int len = (int)min<int64_t>(kTileEntries, t.ent_end - base);
        for (int q = me; q < len; q += kT) prod[q] = w[srow[base + q]] * sval[base + q];
        __syncthreads();
        if (me < nseg) {
            const int64_t lo = max(k0, base), hi = min(k1, base + len);
            for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        }
        __syncthreads();
    }
    if (me < nseg) {
        const int32_t c = tcol[t.seg_begin + me];
        x[c] = x[c] + acc;
    }
}

// r_a = f_a - a_a . x over the group-major rows; per-block sums of r_a^2
__global__ __launch_bounds__(256) void k_resid(int64_t m, const int64_t* __restrict__ rptr,
                                               const int32_t* __restrict__ rcol, const double* __restrict__ rval,
                                               const double* __restrict__ rf, const double* __restrict__ x,
                                               double* __restrict__ partial, int* __restrict__ nonfinite) {
    __shared__ double red[256];
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r2 = 0.0;
    if (a < m) {
        double s = 0.0;
        for (int64_t k = rptr[a]; k < rptr[a + 1]; k++) s = s + rval[k] * x[rcol[k]];
        double r = rf[a] - s;
        if (!isfinite(r)) atomicOr(nonfinite, 1);
        r2 = r * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ordered sum of the partials by one block (deterministic)
__global__ void k_sum_partials(int64_t np, const double* __restrict__ partial, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) s = s + partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_permute_in(int64_t n, const int32_t* __restrict__ p, const double* __restrict__ x0,
                             double* __restrict__ xt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) xt[t] = x0 ? x0[p[t]] : 0.0;
}

__global__ void k_permute_out(int64_t n, const int32_t* __restrict__ p, const double* __restrict__ xt,
                              double* __restrict__ x) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[p[t]] = xt[t];
}

}  // namespace

// enqueue `sweeps` sweeps on x (device, reordered coordinates)
void enqueue_sweeps(const obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < P.ngroups; g++) {
            const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
            const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
            if (r1 > r0)
                k_phase_r<<<r1 - r0, kT, 0, s>>>(P.rtiles.get() + r0, P.rptr.get(), P.rcol.get(), P.rval.get(),
                                                  P.rf.get(), P.rinv.get(), x, P.w.get());
            if (s1 > s0)
                k_phase_s<<<s1 - s0, kT, 0, s>>>(P.stiles.get() + s0, P.sptr.get(), P.srow.get(), P.sval.get(),
                                                  P.tcol.get(), P.w.get(), x);
        }
    }
    OBK_HIP(hipGetLastError());
}

// relative residual ||f~ - A~ x|| / ||f~|| (synchronises the stream); sets *nonfinite
double relres(const obk_plan_s& P, const double* x, hipStream_t s, bool* nonfinite) {
    const int64_t m = P.m;
    const unsigned nb = nblk(m);
    double* part = P.red.get();
    int* flag = reinterpret_cast<int*>(part + nb + 8);
    OBK_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_resid<<<nb, 256, 0, s>>>(m, P.rptr.get(), P.rcol.get(), P.rval.get(), P.rf.get(), x, part, flag);
    k_sum_partials<<<1, 256, 0, s>>>(nb, part, part + nb);
    OBK_HIP(hipGetLastError());
    double r2 = 0;
    int nf = 0;
    OBK_HIP(hipMemcpyAsync(&r2, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipMemcpyAsync(&nf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    r2 = r2 + P.zero_rows_f2;
    if (nonfinite) *nonfinite = (nf != 0) || !std::isfinite(r2);
    if (P.fnorm2 == 0.0) return r2 == 0.0 ? 0.0 : INFINITY;
    return std::sqrt(r2) / std::sqrt(P.fnorm2);
}

void solve_fp64(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = P.n;
    const bool dev = P.input_on_device;
    obk_info inf{};
    inf.relres = -1;
    // x~0 = P x0 (Section 3.5 starts from 0)
    DevArray<double> x0d, xd;
    const double* x0dev = nullptr;
    if (x0) {
        if (dev) x0dev = x0;
        else {
            x0d.alloc(n);
            OBK_HIP(hipMemcpyAsync(x0d.get(), x0, n * sizeof(double), hipMemcpyHostToDevice, s));
            x0dev = x0d.get();
        }
    }
    k_permute_in<<<nblk(n), 256, 0, s>>>(n, P.perm.get(), x0dev, P.x.get());
    OBK_HIP(hipGetLastError());
    bool nf = false;
    inf.relres0 = relres(P, P.x.get(), s, &nf);
    inf.relres = inf.relres0;
    inf.status = OBK_MAXIT;
    const int64_t every = std::max(1, P.opts.check_every);
    int64_t done = 0;
    if (nf) inf.status = OBK_NONFINITE_ITERATE;
    else if (tol > 0 && inf.relres0 <= tol) inf.status = OBK_CONVERGED;
    while (done < maxit && inf.status == OBK_MAXIT) {
        int64_t chunk = (tol > 0) ? std::min(every, maxit - done) : (maxit - done);
        enqueue_sweeps(P, P.x.get(), chunk, s);
        done += chunk;
        if (tol > 0) {
            inf.outer_steps++;
            inf.relres = relres(P, P.x.get(), s, &nf);
            if (nf) inf.status = OBK_NONFINITE_ITERATE;
            else if (inf.relres <= tol) inf.status = OBK_CONVERGED;
            else if (inf.relres > 1e3 * inf.relres0 && inf.relres0 > 0) inf.status = OBK_DIVERGED;
        }
    }
    if (tol <= 0) inf.relres = relres(P, P.x.get(), s, &nf);
    inf.sweeps = done;
    // x = P^T x~ (Algorithm 4, last step)
    double* xout = x;
    if (!dev) { xd.alloc(n); xout = xd.get(); }
    k_permute_out<<<nblk(n), 256, 0, s>>>(n, P.perm.get(), P.x.get(), xout);
    OBK_HIP(hipGetLastError());
    if (!dev) OBK_HIP(hipMemcpyAsync(x, xd.get(), n * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
}

}  // namespace obk
