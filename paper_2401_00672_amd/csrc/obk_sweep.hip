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
#include <hip/hip_ext.h>

#include <chrono>
#include <mutex>
#include <string>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <vector>

#include "obk_internal.h"
#include "obk_sweep_tiles.h"

namespace obk {

constexpr int kT = kTileThreads;

double sum_squares(const double* f, const double* nu, int64_t n, bool only_zero_rows, hipStream_t s);

namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

__global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0) p[0] = 0;
}

// x~ = P x^0 over the extended system of size n, where x^0 = [x0; 0] and x0
// (may be null: 0) holds the caller's n_in unknowns
__global__ void k_permute_in(int64_t n, int64_t n_in, const int32_t* __restrict__ p, const double* __restrict__ x0,
                             double* __restrict__ xt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = (x0 != nullptr) & (n_in > 0);     // uniform
    if (t < n) {
        const int32_t pt = p[t];
        const bool mine = pt < n_in;
        double val = 0.0;
        if (have) {
            const double g = x0[mine ? pt : 0];
            val = mine ? g : 0.0;
        }
        xt[t] = val;
    }
}

// x = (P^T x~)(1 : n_in): the caller's unknowns of the extended solution
__global__ void k_permute_out(int64_t n, int64_t n_in, const int32_t* __restrict__ p,
                              const double* __restrict__ xt, double* __restrict__ x) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int32_t pt = p[t];
        if (pt < n_in) x[pt] = xt[t];
    }
}

// ordered reduction of the per-tile partials by one block (deterministic; the
// batched engine reduces each system's partials in the same order)
__global__ void k_sum_max_partials(int64_t np, const double* __restrict__ psum, const double* __restrict__ pmax,
                                   double* __restrict__ out) {
    __shared__ double red[256];
    __shared__ double mx[256];
    double s = 0.0, m = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) { s = s + psum[i]; m = fmax(m, pmax[i]); }
    red[threadIdx.x] = s;
    mx[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = red[0]; out[1] = mx[0]; }
}

// right-hand side of the correction system, b = (float)(r / sigma), and d = 0
__global__ void k_make_rhs(int64_t m, int64_t n, const double* __restrict__ r, double sigma,
                           float* __restrict__ b, float* __restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) b[i] = (float)(r[i] / sigma);
    if (i < n) d[i] = 0.0f;
}

// x += sigma * d (FP64)
__global__ void k_update_x(int64_t n, double sigma, const float* __restrict__ d, double* __restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + sigma * (double)d[i];
}

}  // namespace

// The tiles [t0, t1) of a phase as a kernel argument list in workgroup order
// (empty when the phase has more than kInlineTiles tiles and reads them from
// the tile array).
static TileList tile_list(const std::vector<Tile>& tiles, int32_t t0, int32_t t1, int32_t& inl) {
    TileList tl;
    std::memset(&tl, 0, sizeof(tl));
    inl = (t1 - t0 <= kInlineTiles) ? 1 : 0;
    if (inl)
        for (int32_t b = 0; b < t1 - t0; b++) tl.t[b] = tiles[t0 + xcd_tile(b, t1 - t0)];
    return tl;
}

template <class T>
static void enqueue_sweeps_t(obk_plan_s& P, const T* rval, const T* rf, const T* rinv, const T* sval,
                             T* x, T* w, int64_t sweeps, hipStream_t s) {
    if constexpr (std::is_same<T, double>::value) {
        if (P.slab_S > 0) return slab_sweeps(P, x, sweeps, s);     // the banded engine, one launch
    }
    const int32_t G = P.ngroups;
    std::vector<TileList> rl(G), sl(G);
    std::vector<int32_t> rin(G), sin(G);
    for (int32_t g = 0; g < G; g++) {
        rl[g] = tile_list(P.h_rtiles, P.h_rtile_ptr[g], P.h_rtile_ptr[g + 1], rin[g]);
        sl[g] = tile_list(P.h_stiles, P.h_stile_ptr[g], P.h_stile_ptr[g + 1], sin[g]);
    }
    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < G; g++) {
            const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
            const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
            if (r1 > r0) {
                if (rin[g])
                    k_phase_r<T, true><<<r1 - r0, kT, 0, s>>>(P.rtiles.get() + r0, rl[g], P.rptr.get(), P.rcol.get(),
                                                               rval, rf, rinv, x, w, (T)P.opts.omega);
                else
                    k_phase_r<T, false><<<r1 - r0, kT, 0, s>>>(P.rtiles.get() + r0, rl[g], P.rptr.get(),
                                                                P.rcol.get(), rval, rf, rinv, x, w, (T)P.opts.omega);
            }
            if (s1 > s0) {
                if (sin[g])
                    k_phase_s<T, true><<<s1 - s0, kT, 0, s>>>(P.stiles.get() + s0, sl[g], P.sptr.get(), P.srow.get(),
                                                               sval, P.tcol.get(), w, x);
                else
                    k_phase_s<T, false><<<s1 - s0, kT, 0, s>>>(P.stiles.get() + s0, sl[g], P.sptr.get(),
                                                                P.srow.get(), sval, P.tcol.get(), w, x);
            }
        }
    }
    OBK_HIP(hipGetLastError());
}

// Sweeps are replayed from captured graphs: one graph per (iterate, sweep
// count, precision) holding kChunk (or 1) whole sweeps as kernel nodes; the
// host then launches ceil(sweeps / kChunk) graphs instead of 2 G kernels per
// sweep.
constexpr int64_t kChunk = 8;

template <class T>
static hipGraphExec_t sweep_graph(obk_plan_s& P, const T* rval, const T* rf, const T* rinv, const T* sval, T* x,
                                  T* w, int64_t sweeps) {
    for (auto& g : P.graphs)
        if (g.x == (const void*)x && g.sweeps == sweeps && g.elem == (int)sizeof(T) && g.exec) return g.exec;
    if (!P.capture_stream) OBK_HIP(hipStreamCreateWithFlags(&P.capture_stream, hipStreamNonBlocking));
    obk_plan_s::SweepGraph sg;
    sg.x = x; sg.sweeps = sweeps; sg.elem = (int)sizeof(T);
    OBK_HIP(hipStreamBeginCapture(P.capture_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_sweeps_t<T>(P, rval, rf, rinv, sval, x, w, sweeps, P.capture_stream);
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
}

template <class T>
static void run_sweeps(obk_plan_s& P, const T* rval, const T* rf, const T* rinv, const T* sval, T* x, T* w,
                       int64_t sweeps, hipStream_t s, bool eager = false) {
    if (sweeps <= 0 || P.ngroups == 0) return;
    if (eager) return enqueue_sweeps_t<T>(P, rval, rf, rinv, sval, x, w, sweeps, s);
    // both graphs of this iterate are captured on its first use, so no later
    // call (whatever its sweep count) captures or instantiates on the host
    hipGraphExec_t chunk = sweep_graph<T>(P, rval, rf, rinv, sval, x, w, kChunk);
    hipGraphExec_t one = sweep_graph<T>(P, rval, rf, rinv, sval, x, w, 1);
    for (int64_t i = 0; i + kChunk <= sweeps; i += kChunk) OBK_HIP(hipGraphLaunch(chunk, s));
    for (int64_t i = 0; i < sweeps % kChunk; i++) OBK_HIP(hipGraphLaunch(one, s));
}

// enqueue `sweeps` sweeps on x (device, reordered coordinates)
void enqueue_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s) {
    if (P.block_form()) return block_sweeps(P, x, sweeps, s, nullptr);
    run_sweeps<double>(P, P.rval.get(), P.rf.get(), P.rinv.get(), P.sval.get(), x, P.w.get(), sweeps, s);
}

// Eager FP64 sweeps with an event pair around every launch; per-kernel sums
// of event time and algorithmic bytes (formulas in obk.h).
int32_t profile_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                       int32_t max_out) {
    if (P.block_form()) return profile_block(P, x, sweeps, s, out, max_out);
    if (P.slab_S > 0) {
        if (max_out < 1) return 0;
        obk_kernel_profile& o = out[0];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, "k_slab_sweeps", sizeof(o.name) - 1);
        o.launches = 1;
        o.seconds = slab_profile(P, x, sweeps, s);
        o.bytes = P.slab_bytes_per_sweep * (double)sweeps + P.slab_bytes_per_launch;
        return 1;
    }
    const int32_t G = P.ngroups;
    struct Launch { int kind; double bytes; };
    std::vector<Launch> plan_launches;
    const double sv = 8, so = 4;
    for (int32_t g = 0; g < G; g++) {
        const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
        const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
        double ng = 0, eg = 0, tg = 0;
        for (int32_t t = r0; t < r1; t++) {
            ng += P.h_rtiles[t].seg_end - P.h_rtiles[t].seg_begin;
            eg += (double)(P.h_rtiles[t].ent_end - P.h_rtiles[t].ent_begin);
        }
        for (int32_t t = s0; t < s1; t++) tg += P.h_stiles[t].seg_end - P.h_stiles[t].seg_begin;
        if (r1 > r0) plan_launches.push_back({0, eg * (sv + so) + ng * (so + 3 * sv) + tg * sv});
        if (s1 > s0) plan_launches.push_back({1, eg * (sv + so) + tg * (2 * so + 2 * sv) + ng * sv});
    }
    const size_t nl = plan_launches.size() * (size_t)sweeps;
    std::vector<hipEvent_t> ev(2 * nl, nullptr);
    struct EvGuard {
        std::vector<hipEvent_t>& e;
        ~EvGuard() { for (auto x : e) if (x) (void)hipEventDestroy(x); }
    } guard{ev};
    for (auto& e : ev) OBK_HIP(hipEventCreate(&e));
    size_t k = 0;
    for (int64_t it = 0; it < sweeps; it++) {
        size_t li = 0;
        for (int32_t g = 0; g < G; g++) {
            const int32_t r0 = P.h_rtile_ptr[g], r1 = P.h_rtile_ptr[g + 1];
            const int32_t s0 = P.h_stile_ptr[g], s1 = P.h_stile_ptr[g + 1];
            // the events ride on the kernel's own dispatch packet: they time the
            // kernel, not the packets around it
            int32_t rin = 0, sin = 0;
            const TileList rl = tile_list(P.h_rtiles, r0, r1, rin), sl = tile_list(P.h_stiles, s0, s1, sin);
            if (r1 > r0) {
                hipExtLaunchKernelGGL(rin ? k_phase_r<double, true> : k_phase_r<double, false>, dim3(r1 - r0),
                                      dim3(kT), 0, s, ev[2 * k], ev[2 * k + 1], 0,
                                      (const Tile*)(P.rtiles.get() + r0), rl, (const int64_t*)P.rptr.get(),
                                      (const int32_t*)P.rcol.get(), (const double*)P.rval.get(),
                                      (const double*)P.rf.get(), (const double*)P.rinv.get(), (const double*)x,
                                      P.w.get(), P.opts.omega);
                k++, li++;
            }
            if (s1 > s0) {
                hipExtLaunchKernelGGL(sin ? k_phase_s<double, true> : k_phase_s<double, false>, dim3(s1 - s0),
                                      dim3(kT), 0, s, ev[2 * k], ev[2 * k + 1], 0,
                                      (const Tile*)(P.stiles.get() + s0), sl, (const int64_t*)P.sptr.get(),
                                      (const int32_t*)P.srow.get(), (const double*)P.sval.get(),
                                      (const int32_t*)P.tcol.get(), (const double*)P.w.get(), x);
                k++, li++;
            }
        }
        (void)li;
    }
    OBK_HIP(hipGetLastError());
    OBK_HIP(hipStreamSynchronize(s));
    const char* names[2] = {"k_phase_r<double>", "k_phase_s<double>"};
    obk_kernel_profile acc[2];
    for (int j = 0; j < 2; j++) {
        std::memset(&acc[j], 0, sizeof(acc[j]));
        std::strncpy(acc[j].name, names[j], sizeof(acc[j].name) - 1);
    }
    for (size_t i = 0; i < nl; i++) {
        const Launch& L = plan_launches[i % plan_launches.size()];
        float ms = 0;
        OBK_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        acc[L.kind].launches++;
        acc[L.kind].seconds += ms * 1e-3;
        acc[L.kind].bytes += L.bytes;
    }
    int32_t n = 0;
    for (int j = 0; j < 2 && n < max_out; j++)
        if (acc[j].launches) out[n++] = acc[j];
    return n;
}

}  // namespace obk

obk_plan_s::~obk_plan_s() {
    for (auto& g : graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

namespace obk {

// FP64 residual over the plan's R tiles (every active row): r (may be null)
// receives r_a; *sum_sq gets sum r_a^2 over the active rows, *max_abs max |r_a|,
// *nonfinite whether any r_a is not finite.  Synchronises the stream.
// With ws (the no-allocation solve), the partials live in ws->red and the
// sums come back through a stack buffer instead of the pinned stage.
static void resid_tiles(const obk_plan_s& P, const double* x, double* r, hipStream_t s, double* sum_sq,
                        double* max_abs, bool* nonfinite, const SolveWs* ws) {
    const int64_t nt = (int64_t)P.h_rtiles.size();
    double* psum = ws ? ws->red : P.red.get();
    double* pmax = psum + std::max<int64_t>(nt, 1);
    double* out = pmax + std::max<int64_t>(nt, 1);
    int* flag = reinterpret_cast<int*>(out + 4);
    k_zero_int<<<1, 64, 0, s>>>(flag);
    if (nt)
        k_resid_tiles<<<(unsigned)nt, kT, 0, s>>>(P.rtiles.get(), P.rptr.get(), P.rcol.get(), P.rval.get(),
                                                  P.rf.get(), x, r, psum, pmax, flag);
    k_sum_max_partials<<<1, 256, 0, s>>>(nt, psum, pmax, out);
    OBK_HIP(hipGetLastError());
    double hstack[4];
    auto* h = ws ? hstack : static_cast<double*>(pinned_stage(4 * sizeof(double)));
    OBK_HIP(hipMemcpyAsync(h, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipMemcpyAsync(h + 2, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    int nf = 0;
    std::memcpy(&nf, h + 2, sizeof(int));
    *sum_sq = h[0];
    *max_abs = h[1];
    *nonfinite = nf != 0;
}

// relative residual ||f~ - A~ x|| / ||f~|| (synchronises the stream); sets *nonfinite
double relres(obk_plan_s& P, const double* x, hipStream_t s, bool* nonfinite, const SolveWs* ws) {
    slab_check(P, s);
    double r2 = 0, mx = 0;
    bool nf = false;
    resid_tiles(P, x, nullptr, s, &r2, &mx, &nf, ws);
    r2 = r2 + P.zero_rows_f2;
    if (nonfinite) *nonfinite = nf || !std::isfinite(r2);
    if (P.fnorm2 == 0.0) return r2 == 0.0 ? 0.0 : INFINITY;
    return std::sqrt(r2) / std::sqrt(P.fnorm2);
}

void solve_fp64(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                hipStream_t s, const SolveWs* ws) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = P.n;
    const bool dev = P.input_on_device || ws;
    obk_info inf{};
    inf.relres = -1;
    // x~0 = P x0 (Section 3.5 starts from 0)
    DevArray<double> x0d, xd;
    const double* x0dev = nullptr;
    if (x0) {
        if (dev) x0dev = x0;
        else {
            x0d.alloc(P.n_in);
            OBK_HIP(hipMemcpyAsync(x0d.get(), x0, P.n_in * sizeof(double), hipMemcpyHostToDevice, s));
            x0dev = x0d.get();
        }
    }
    k_permute_in<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), x0dev, P.x.get());
    OBK_HIP(hipGetLastError());
    bool nf = false;
    inf.relres0 = relres(P, P.x.get(), s, &nf, ws);
    inf.relres = inf.relres0;
    inf.status = OBK_MAXIT;
    const int64_t every = std::max(1, P.opts.check_every);
    int64_t done = 0;
    if (nf) inf.status = OBK_NONFINITE_ITERATE;
    else if (tol > 0 && inf.relres0 <= tol) inf.status = OBK_CONVERGED;
    while (done < maxit && inf.status == OBK_MAXIT) {
        int64_t chunk = (tol > 0) ? std::min(every, maxit - done) : (maxit - done);
        if (ws) run_sweeps<double>(P, P.rval.get(), P.rf.get(), P.rinv.get(), P.sval.get(), P.x.get(), P.w.get(),
                                   chunk, s, true);
        else enqueue_sweeps(P, P.x.get(), chunk, s);
        done += chunk;
        if (tol > 0) {
            inf.outer_steps++;
            inf.relres = relres(P, P.x.get(), s, &nf, ws);
            if (nf) inf.status = OBK_NONFINITE_ITERATE;
            else if (inf.relres <= tol) inf.status = OBK_CONVERGED;
            else if (inf.relres > 1e3 * inf.relres0 && inf.relres0 > 0) inf.status = OBK_DIVERGED;
        }
    }
    if (tol <= 0) inf.relres = relres(P, P.x.get(), s, &nf, ws);
    inf.sweeps = done;
    // x = P^T x~ (Algorithm 4, last step)
    double* xout = x;
    if (!dev) { xd.alloc(P.n_in); xout = xd.get(); }
    k_permute_out<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), P.x.get(), xout);
    OBK_HIP(hipGetLastError());
    if (!dev) OBK_HIP(hipMemcpyAsync(x, xd.get(), P.n_in * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
}

// Iterative refinement with FP32 inner sweeps (residual, norms, scale and
// update in FP64): r = f - A x; sigma = max |r_i|; `inner_sweeps` FP32
// sweeps on A d = r / sigma from d = 0; x += sigma d.  Stops when
// ||r|| / ||f|| <= tol or after maxit refinement steps.
void solve_fp32_ir(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s, const SolveWs* ws) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = P.n, m = P.m;
    const bool dev = P.input_on_device || ws;
    obk_info inf{};
    DevArray<double> x0d, xd;
    const double* x0dev = nullptr;
    if (x0) {
        if (dev) x0dev = x0;
        else {
            x0d.alloc(P.n_in);
            OBK_HIP(hipMemcpyAsync(x0d.get(), x0, P.n_in * sizeof(double), hipMemcpyHostToDevice, s));
            x0dev = x0d.get();
        }
    }
    k_permute_in<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), x0dev, P.x.get());
    OBK_HIP(hipGetLastError());
    auto residual = [&](double* rho, double* sigma, bool* nonfinite) {
        double r2 = 0, mx = 0;
        bool nf = false;
        resid_tiles(P, P.x.get(), P.r64.get(), s, &r2, &mx, &nf, ws);
        r2 = r2 + P.zero_rows_f2;
        *sigma = std::max(mx, P.zero_rows_fmax);
        *nonfinite = nf || !std::isfinite(r2);
        *rho = (P.fnorm2 == 0.0) ? (r2 == 0.0 ? 0.0 : INFINITY) : std::sqrt(r2) / std::sqrt(P.fnorm2);
    };
    double rho = 0, sigma = 0;
    bool nf = false;
    residual(&rho, &sigma, &nf);
    inf.relres0 = rho;
    inf.relres = rho;
    inf.status = OBK_MAXIT;
    if (nf) inf.status = OBK_NONFINITE_ITERATE;
    else if (tol > 0 && rho <= tol) inf.status = OBK_CONVERGED;
    const int inner = std::max(1, P.opts.inner_sweeps);
    while (inf.status == OBK_MAXIT && inf.outer_steps < maxit && sigma > 0.0) {
        k_make_rhs<<<nblk(std::max(m, n)), 256, 0, s>>>(m, n, P.r64.get(), sigma, P.b32.get(), P.d32.get());
        run_sweeps<float>(P, P.rval32.get(), P.b32.get(), P.rinv32.get(), P.sval32.get(), P.d32.get(),
                          P.w32.get(), inner, s, ws != nullptr);
        k_update_x<<<nblk(n), 256, 0, s>>>(n, sigma, P.d32.get(), P.x.get());
        OBK_HIP(hipGetLastError());
        inf.outer_steps++;
        inf.sweeps += inner;
        residual(&rho, &sigma, &nf);
        inf.relres = rho;
        if (nf) inf.status = OBK_NONFINITE_ITERATE;
        else if (tol > 0 && rho <= tol) inf.status = OBK_CONVERGED;
        else if (rho > 1e3 * inf.relres0 && inf.relres0 > 0) inf.status = OBK_DIVERGED;
    }
    if (inf.status == OBK_MAXIT && sigma == 0.0) inf.status = OBK_CONVERGED;
    double* xout = x;
    if (!dev) { xd.alloc(P.n_in); xout = xd.get(); }
    k_permute_out<<<nblk(n), 256, 0, s>>>(n, P.n_in, P.perm.get(), P.x.get(), xout);
    OBK_HIP(hipGetLastError());
    if (!dev) OBK_HIP(hipMemcpyAsync(x, xd.get(), P.n_in * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
}

// ------------------------------------------------- the no-allocation solve
// Device scratch of the no-allocation solve (obk_solve_noalloc): the
// residual partials of up to kScratchTiles row tiles and the reduced sums.
// One copy per GPU, held until the process ends; every call on a GPU uses
// it, so calls that overlap on one GPU race.  Host code reaches it only
// through the address hipGetSymbolAddress returns on each device.
constexpr int64_t kScratchDoubles = int64_t(1) << 17;          // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int64_t kScratchTiles = (kScratchDoubles - 16) / 2;

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch;        // per device: the address of scratch there

// The device address of scratch on the current device (looked up once per
// device, with that device current).
static double* scratch_address() {
    int dev = 0;
    OBK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(OBK_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

// obk_solve on device iterates with no allocation: the residual partials in
// the static scratch, sweeps launched eagerly (no graph is captured), sums
// read back through a stack buffer.  The plan's own workspace is used as in
// obk_solve.
void solve_noalloc(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s) {
    const int64_t nt = (int64_t)P.h_rtiles.size();
    if (nt > kScratchTiles)
        fail(OBK_E_ARG, "the plan has " + std::to_string(nt) + " row tiles; the static scratch holds the partials of " +
                            std::to_string(kScratchTiles));
    SolveWs ws;
    ws.red = scratch_address();
    if (P.opts.precision == OBK_FP32_IR) solve_fp32_ir(P, x0, tol, maxit, x, info, s, &ws);
    else solve_fp64(P, x0, tol, maxit, x, info, s, &ws);
}

}  // namespace obk
