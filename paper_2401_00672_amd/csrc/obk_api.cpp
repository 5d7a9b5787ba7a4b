// The C ABI of libobk: argument checks, error conversion, plan lifecycle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "obk_internal.h"

namespace obk {
const char* last_error_cstr();
void build_plan(obk_plan_s& P, const obk_csr& A, const double* f, double delta, hipStream_t s);
void solve_fp64(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                hipStream_t s, const SolveWs* ws = nullptr);
void enqueue_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);
int32_t profile_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                       int32_t max_out);
void solve_fp32_ir(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s, const SolveWs* ws = nullptr);
void ensure_fp32(obk_plan_s& P, hipStream_t s);
void lambda_bound_on_request(obk_plan_s& P, hipStream_t s);
void batch_create(obk_batch_s& B, const obk_plan_t* plans, int count, const obk_batch_opts* opts);
void batch_reset(obk_batch_s& B, const obk_plan_t* plans, int count, hipStream_t s);
void batch_begin(obk_batch_s& B, const double* const* x0, hipStream_t s);
void batch_step(obk_batch_s& B, double tol, double* relres_out, int32_t* active_out, hipStream_t s);
void batch_result(obk_batch_s& B, int index, double* x, hipStream_t s);
void batch_set_enabled(obk_batch_s& B, const int32_t* enabled, hipStream_t s);
void batch_start(obk_batch_s& B, int index, const double* x0, hipStream_t s);
}  // namespace obk

// the batch object is defined with its kernels; only pointers cross here
struct obk_batch_s;
obk_batch_s* obk_batch_new();
void obk_batch_delete(obk_batch_s*);
bool* obk_batch_busy(obk_batch_s*);
int obk_batch_count(obk_batch_s*);

size_t obk_plan_s::device_bytes() const {
    return perm.bytes() + rptr.bytes() + rcol.bytes() + rval.bytes() + rf.bytes() + rinv.bytes() +
           tcol.bytes() + sptr.bytes() + srow.bytes() + sval.bytes() + rtiles.bytes() + stiles.bytes() +
           d_rtile_ptr.bytes() + d_stile_ptr.bytes() +
           x.bytes() + w.bytes() + red.bytes() + rval32.bytes() + rinv32.bytes() + sval32.bytes() +
           b32.bytes() + d32.bytes() + w32.bytes() + r64.bytes() + d_bptr.bytes() + d_btptr.bytes() +
           d_border.bytes() + bres.bytes() + bp.bytes() + bu.bytes() + bpart.bytes() + bbar.bytes() + berr.bytes() +
           biters.bytes() + blseg.bytes() + d_bfit.bytes() + rvalz.bytes() + svalz.bytes() + rfz.bytes() +
           d_bdirect.bytes() + d_bbw.bytes() + d_boff.bytes() + lfc.bytes() + lfr.bytes() + ldinv.bytes() +
           d_lperm.bytes() + d_lpos.bytes() + sl_desc.bytes() + sl_grp.bytes() + sl_round.bytes() +
           sl_tgt.bytes() + sl_len.bytes() + sl_idx.bytes() + sl_f.bytes() + sl_val.bytes() +
           sl_xbuf.bytes() + sl_flags.bytes() + sl_err.bytes();
}

namespace {

const char* status_name(obk_status st) {
    switch (st) {
        case OBK_OK: return "OBK_OK";
        case OBK_E_ARG: return "OBK_E_ARG";
        case OBK_E_CSR: return "OBK_E_CSR";
        case OBK_E_NOT_SQUARE: return "OBK_E_NOT_SQUARE";
        case OBK_E_NONFINITE: return "OBK_E_NONFINITE";
        case OBK_E_NOMEM: return "OBK_E_NOMEM";
        case OBK_E_HIP: return "OBK_E_HIP";
        case OBK_E_BUSY: return "OBK_E_BUSY";
        case OBK_E_INCONSISTENT: return "OBK_E_INCONSISTENT";
    }
    return "OBK_E_?";
}

obk_status failed(obk_status code, const std::string& msg) {
    obk::set_last_error(msg);
    obk::log_line(1, "error %s: %s", status_name(code), msg.c_str());
    return code;
}

template <class F> obk_status guarded(F&& body) {
    try {
        body();
        obk::set_last_error("");
        return OBK_OK;
    } catch (const obk::Error& e) {
        (void)hipGetLastError();
        return failed(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return failed(OBK_E_NOMEM, "host allocation failed");
    } catch (...) {
        return failed(OBK_E_HIP, "unexpected internal error");
    }
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

hipStream_t as_hip(obk_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// Definitions 1 and 2 on the plan's centroid cosine table
void block_criteria(const obk_plan_s& P, double* zn, double* nn) {
    const size_t num = P.h_bcos.size();
    size_t n2 = 0;
    double sum = 0.0;
    for (double c : P.h_bcos)
        if (c != 0.0) {
            n2++;
            sum += c;
        }
    const double nm = n2 ? sum / (double)n2 : 0.0;
    if (zn) *zn = num ? (double)(num - n2) / (double)num : 0.0;
    if (nn) *nn = num ? (double)n2 * nm / (double)num : 0.0;
}

void check_block_opts(const obk_opts& o) {
    if (o.block_k < 0 || o.block_k > 4096) obk::fail(OBK_E_ARG, "block_k must be in [0, 4096]");
    if (o.block_k > 0 && o.precision != OBK_FP64) obk::fail(OBK_E_ARG, "the block form runs in OBK_FP64 only");
    if (o.block_wgs < 0 || o.block_maxit < 0) obk::fail(OBK_E_ARG, "block_wgs and block_maxit must be >= 0");
    if (!(o.block_tol >= 0.0) || !std::isfinite(o.block_tol)) obk::fail(OBK_E_ARG, "block_tol must be finite and >= 0");
    if (o.block_solver != 0 && o.block_solver != 1) obk::fail(OBK_E_ARG, "block_solver must be 0 or 1");
    if (o.sweep_kernel < 0 || o.sweep_kernel > 2) obk::fail(OBK_E_ARG, "sweep_kernel must be 0, 1 or 2");
}

// the fields every entry point that takes an obk_opts checks the same way
void check_common_opts(const obk_opts& o) {
    if (!(o.omega > 0.0 && o.omega < 2.0)) obk::fail(OBK_E_ARG, "omega must lie in (0, 2)");
    if (o.max_group != 0 && o.max_group != 2) obk::fail(OBK_E_ARG, "max_group must be 0 or 2");
    if (o.deterministic != 0 && o.deterministic != 1) obk::fail(OBK_E_ARG, "deterministic must be 0 or 1");
    if ((o.alloc == nullptr) != (o.dealloc == nullptr))
        obk::fail(OBK_E_ARG, "alloc and dealloc must both be set or both be NULL");
    if (o.block_k > 0 && o.omega != 1.0) obk::fail(OBK_E_ARG, "the block form takes no relaxation (omega = 1)");
    if (o.block_k > 0 && o.sweep_kernel == 2) obk::fail(OBK_E_ARG, "the banded engine runs one-row-block plans only");
}

// RAII marker for the one-solve-at-a-time rule
struct BusyGuard {
    obk_plan_s* p;
    explicit BusyGuard(obk_plan_s* plan) : p(plan) {
        if (__atomic_exchange_n(&p->busy, true, __ATOMIC_ACQ_REL)) obk::fail(OBK_E_BUSY, "a solve on this plan is running");
    }
    ~BusyGuard() { __atomic_store_n(&p->busy, false, __ATOMIC_RELEASE); }
};

}  // namespace

extern "C" {

obk_status obk_opts_default(obk_opts* opts) {
    if (!opts) { obk::set_last_error("opts is NULL"); return OBK_E_ARG; }
    std::memset(opts, 0, sizeof(*opts));
    opts->use_rcm = 1;
    opts->precision = OBK_FP64;
    opts->inner_sweeps = 8;
    opts->check_every = 1;
    opts->reject_inconsistent = 0;
    opts->hbm_budget = 0;
    opts->block_k = 0;
    opts->block_wgs = 0;
    opts->block_maxit = 0;
    opts->block_tol = 1e-14;
    opts->block_solver = 0;
    opts->sweep_kernel = 0;
    opts->omega = 1.0;
    opts->max_group = 0;
    opts->deterministic = 1;
    opts->alloc = nullptr;
    opts->dealloc = nullptr;
    opts->ctx = nullptr;
    return OBK_OK;
}

static obk_status plan_impl(const obk_csr* A, const double* f, double delta, const obk_opts* opts,
                            obk_stream_t stream, obk_plan_t* out, bool cplx);

obk_status obk_plan(const obk_csr* A, const double* f, double delta, const obk_opts* opts, obk_stream_t stream,
                    obk_plan_t* out) {
    return plan_impl(A, f, delta, opts, stream, out, false);
}

obk_status obk_plan_complex(const obk_csr* A, const double* f, double delta, const obk_opts* opts,
                            obk_stream_t stream, obk_plan_t* out) {
    return plan_impl(A, f, delta, opts, stream, out, true);
}

static obk_status plan_impl(const obk_csr* A, const double* f, double delta, const obk_opts* opts,
                            obk_stream_t stream, obk_plan_t* out, bool cplx) {
    if (out) *out = nullptr;
    obk_plan_s* P = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    obk_status st = guarded([&] {
        if (!A || !out) obk::fail(OBK_E_ARG, "A and out must not be NULL");
        if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) obk::fail(OBK_E_ARG, "negative size");
        if (std::max(A->n_rows, A->n_cols) >= std::numeric_limits<int32_t>::max() ||
            A->nnz >= std::numeric_limits<int32_t>::max())
            obk::fail(OBK_E_ARG, "n_rows, n_cols and nnz must be below 2^31 - 1");
        if (A->n_rows > 0 && (!A->row_ptr || !f)) obk::fail(OBK_E_ARG, "row_ptr and f must not be NULL");
        if (A->nnz > 0 && (!A->col || !A->val)) obk::fail(OBK_E_ARG, "col and val must not be NULL");
        if (!(delta > 0.0) || !std::isfinite(delta)) obk::fail(OBK_E_ARG, "delta must be finite and > 0");
        obk_opts o;
        obk_opts_default(&o);
        if (opts) o = *opts;
        if (o.precision != OBK_FP64 && o.precision != OBK_FP32_IR) obk::fail(OBK_E_ARG, "unknown precision");
        if (o.inner_sweeps < 1 || o.check_every < 1) obk::fail(OBK_E_ARG, "inner_sweeps and check_every must be >= 1");
        if (o.use_rcm < 0 || o.use_rcm > 3) obk::fail(OBK_E_ARG, "use_rcm must be 0, 1, 2 or 3");
        if (o.max_group == 2) {
            // the paper's pair rule: the block form with one-row blocks
            const int64_t N = std::max(A->n_rows, A->n_cols);
            if (o.block_k != 0) obk::fail(OBK_E_ARG, "max_group = 2 is the block form with k = n; leave block_k 0");
            if (N > 4096 || N < 1) obk::fail(OBK_E_ARG, "max_group = 2 needs 1 <= n <= 4096 (k = n blocks)");
            o.block_k = (int)N;
        }
        check_block_opts(o);
        check_common_opts(o);
        if (o.block_k > std::max(A->n_rows, A->n_cols)) obk::fail(OBK_E_ARG, "block_k exceeds the number of rows");
        if (cplx && o.precision != OBK_FP64) obk::fail(OBK_E_ARG, "complex systems run in OBK_FP64 only");
        if (cplx && o.block_k > 0) obk::fail(OBK_E_ARG, "the block form takes real systems only");
        if (cplx && o.sweep_kernel == 2) obk::fail(OBK_E_ARG, "the banded engine runs real systems only");
        P = new obk_plan_s();
        P->opts = o;
        P->cplx = cplx;
        obk::UserAllocScope ua(o.alloc, o.dealloc, o.ctx, as_hip(stream));
        obk::build_plan(*P, *A, f, delta, as_hip(stream));
    });
    if (st != OBK_OK) {
        if (P) {
            (void)hipStreamSynchronize(as_hip(stream));   // no kernel may still use the plan's buffers
            (void)hipGetLastError();
        }
        delete P;
        return st;
    }
    *out = P;
    obk::log_line(2, "plan%s n=%lld nnz=%lld groups=%d conflicts=%lld bytes=%zu block_k=%d %.2f ms",
                  cplx ? " (complex)" : "", (long long)P->n, (long long)P->nnz, (int)P->ngroups,
                  (long long)P->nconflicts, P->device_bytes(), P->opts.block_k, 1e3 * seconds_since(t0));
    return OBK_OK;
}

obk_status obk_solve(obk_plan_t plan, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                     obk_stream_t stream) {
    return guarded([&] {
        if (!plan || !x) obk::fail(OBK_E_ARG, "plan and x must not be NULL");
        if (maxit < 0 || std::isnan(tol)) obk::fail(OBK_E_ARG, "maxit must be >= 0 and tol a number");
        BusyGuard busy(plan);
        OBK_HIP(hipSetDevice(plan->device));
        obk::UserAllocScope ua(plan->opts.alloc, plan->opts.dealloc, plan->opts.ctx, as_hip(stream));
        obk_info local{};
        obk_info* inf = info ? info : &local;
        if (plan->cplx)
            obk::solve_complex(*plan, x0, tol, maxit, x, inf, as_hip(stream));
        else if (plan->opts.precision == OBK_FP32_IR)
            obk::solve_fp32_ir(*plan, x0, tol, maxit, x, inf, as_hip(stream));
        else
            obk::solve_fp64(*plan, x0, tol, maxit, x, inf, as_hip(stream));
        obk::log_line(2, "solve n=%lld status=%d sweeps=%lld outer_steps=%lld relres0=%.3e relres=%.3e %.3f ms",
                      (long long)plan->n, inf->status, (long long)inf->sweeps, (long long)inf->outer_steps,
                      inf->relres0, inf->relres, 1e3 * inf->seconds);
    });
}

obk_status obk_solve_noalloc(obk_plan_t plan, const double* x0, double tol, int64_t maxit, double* x,
                             obk_info* info, obk_stream_t stream) {
    return guarded([&] {
        if (!plan || !x) obk::fail(OBK_E_ARG, "plan and x must not be NULL");
        if (maxit < 0 || std::isnan(tol)) obk::fail(OBK_E_ARG, "maxit must be >= 0 and tol a number");
        if (plan->cplx || plan->block_form())
            obk::fail(OBK_E_ARG, "obk_solve_noalloc takes real plans with one-row blocks");
        BusyGuard busy(plan);
        OBK_HIP(hipSetDevice(plan->device));
        obk::solve_noalloc(*plan, x0, tol, maxit, x, info, as_hip(stream));
    });
}

obk_status obk_plan_set_opts(obk_plan_t plan, const obk_opts* opts) {
    return guarded([&] {
        if (!plan || !opts) obk::fail(OBK_E_ARG, "NULL argument");
        if (opts->precision != OBK_FP64 && opts->precision != OBK_FP32_IR) obk::fail(OBK_E_ARG, "unknown precision");
        if (opts->inner_sweeps < 1 || opts->check_every < 1) obk::fail(OBK_E_ARG, "inner_sweeps and check_every must be >= 1");
        obk_opts o = *opts;
        o.block_k = plan->opts.block_k;   // a plan-time option
        check_block_opts(o);
        if (plan->cplx && o.precision != OBK_FP64) obk::fail(OBK_E_ARG, "complex systems run in OBK_FP64 only");
        BusyGuard busy(plan);
        OBK_HIP(hipSetDevice(plan->device));
        plan->opts.precision = opts->precision;
        plan->opts.inner_sweeps = opts->inner_sweeps;
        plan->opts.check_every = opts->check_every;
        plan->opts.hbm_budget = opts->hbm_budget;
        plan->opts.block_wgs = opts->block_wgs;
        plan->opts.block_maxit = opts->block_maxit;
        plan->opts.block_tol = opts->block_tol;
        obk::UserAllocScope ua(plan->opts.alloc, plan->opts.dealloc, plan->opts.ctx, nullptr);
        if (plan->has_fp32()) obk::ensure_fp32(*plan, nullptr);
    });
}

obk_status obk_sweep_device(obk_plan_t plan, double* x_tilde_dev, int64_t sweeps, obk_stream_t stream) {
    return guarded([&] {
        if (!plan || !x_tilde_dev) obk::fail(OBK_E_ARG, "plan and x_tilde_dev must not be NULL");
        if (sweeps < 0) obk::fail(OBK_E_ARG, "sweeps must be >= 0");
        BusyGuard busy(plan);
        OBK_HIP(hipSetDevice(plan->device));
        obk::UserAllocScope ua(plan->opts.alloc, plan->opts.dealloc, plan->opts.ctx, as_hip(stream));
        if (plan->cplx) obk::enqueue_sweeps_z(*plan, x_tilde_dev, sweeps, as_hip(stream));
        else obk::enqueue_sweeps(*plan, x_tilde_dev, sweeps, as_hip(stream));
    });
}

obk_status obk_sweep_profile(obk_plan_t plan, double* x_tilde_dev, int64_t sweeps, obk_stream_t stream,
                             obk_kernel_profile* out, int32_t max_out, int32_t* n_out) {
    return guarded([&] {
        if (!plan || !x_tilde_dev || !out || !n_out) obk::fail(OBK_E_ARG, "NULL argument");
        if (sweeps < 1 || sweeps > 4096) obk::fail(OBK_E_ARG, "sweeps must be in [1, 4096]");
        if (max_out < 1) obk::fail(OBK_E_ARG, "max_out must be >= 1");
        OBK_HIP(hipSetDevice(plan->device));
        BusyGuard busy(plan);
        obk::UserAllocScope ua(plan->opts.alloc, plan->opts.dealloc, plan->opts.ctx, as_hip(stream));
        *n_out = plan->cplx ? obk::profile_sweeps_z(*plan, x_tilde_dev, sweeps, as_hip(stream), out, max_out)
                            : obk::profile_sweeps(*plan, x_tilde_dev, sweeps, as_hip(stream), out, max_out);
    });
}

void obk_free(obk_plan_t plan) {
    if (!plan) return;
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    delete plan;
}

obk_status obk_free_async(obk_plan_t plan, obk_stream_t stream) {
    return guarded([&] {
        if (!plan) return;
        OBK_HIP(hipSetDevice(plan->device));
        if (__atomic_load_n(&plan->busy, __ATOMIC_ACQUIRE)) obk::fail(OBK_E_BUSY, "a solve on this plan is running");
        hipStream_t s = as_hip(stream);
        // the caller's deallocator takes blocks back at once: the work queued
        // on s must be done first
        if (plan->opts.alloc) OBK_HIP(hipStreamSynchronize(s));
        // pool blocks go back in stream order on s
        obk::AllocScope scope(s);
        delete plan;
    });
}

obk_status obk_plan_perm(obk_plan_t plan, int32_t* p_host) {
    return guarded([&] {
        if (!plan || (!p_host && plan->n > 0)) obk::fail(OBK_E_ARG, "NULL argument");
        if (plan->n) std::memcpy(p_host, plan->h_perm.data(), plan->n * sizeof(int32_t));
    });
}

obk_status obk_plan_groups(obk_plan_t plan, int32_t* group_of_row_host, int32_t* n_groups) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (group_of_row_host && plan->n)
            std::memcpy(group_of_row_host, plan->h_group.data(), plan->n * sizeof(int32_t));
        if (n_groups) *n_groups = plan->ngroups;
    });
}

obk_status obk_plan_blocks(obk_plan_t plan, int32_t* k, int64_t* bptr, int32_t* partner, double* cos,
                           int64_t* cg_iters) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (!plan->block_form()) obk::fail(OBK_E_ARG, "the plan is not in block form");
        const int32_t K = plan->opts.block_k;
        if (k) *k = K;
        if (bptr) std::memcpy(bptr, plan->h_bptr.data(), (K + 1) * sizeof(int64_t));
        if (partner) std::memcpy(partner, plan->h_partner.data(), K * sizeof(int32_t));
        if (cos) std::memcpy(cos, plan->h_bcos.data(), (size_t)K * K * sizeof(double));
        if (cg_iters) {
            OBK_HIP(hipSetDevice(plan->device));
            OBK_HIP(hipMemcpy(cg_iters, plan->biters.get(), K * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
    });
}

obk_status obk_plan_block_solvers(obk_plan_t plan, int32_t* direct, int64_t* bandwidth) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (!plan->block_form()) obk::fail(OBK_E_ARG, "the plan is not in block form");
        const int32_t K = plan->opts.block_k;
        for (int32_t b = 0; b < K; b++) {
            const bool d = b < (int32_t)plan->h_bdirect.size() && plan->h_bdirect[b];
            if (direct) direct[b] = d ? 1 : 0;
            if (bandwidth) bandwidth[b] = d ? plan->h_bbw[b] : -1;
        }
    });
}

obk_status obk_block_zn_nn(obk_plan_t plan, double* zn, double* nn) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (!plan->block_form()) obk::fail(OBK_E_ARG, "the plan is not in block form");
        block_criteria(*plan, zn, nn);
    });
}

obk_status obk_block_select_k(const obk_csr* A, const double* f, double thr, const int32_t* candidates,
                              int32_t n_candidates, const obk_opts* opts, obk_stream_t stream, int32_t* best_k,
                              double* zn, double* nn) {
    return guarded([&] {
        if (!best_k) obk::fail(OBK_E_ARG, "best_k must not be NULL");
        if (n_candidates < 1 || !candidates) obk::fail(OBK_E_ARG, "no candidate block counts");
        for (int32_t i = 0; i < n_candidates; i++)
            if (candidates[i] < 1 || candidates[i] > 4096) obk::fail(OBK_E_ARG, "a candidate is outside [1, 4096]");
        obk_opts o;
        obk_opts_default(&o);
        if (opts) o = *opts;
        double bz = 0.0, bn = 0.0;
        int32_t bk = -1;
        for (int32_t i = 0; i < n_candidates; i++) {
            o.block_k = candidates[i];
            obk_plan_t P = nullptr;
            const obk_status st = obk_plan(A, f, thr, &o, stream, &P);
            if (st != OBK_OK) obk::fail(st, obk::last_error_cstr());
            double z = 0.0, q = 0.0;
            block_criteria(*P, &z, &q);
            obk_free(P);
            if (zn) zn[i] = z;
            if (nn) nn[i] = q;
            const int32_t k = candidates[i];
            if (bk < 0 || z > bz || (z == bz && (q < bn || (q == bn && k < bk)))) {
                bk = k;
                bz = z;
                bn = q;
            }
        }
        *best_k = bk;
    });
}

obk_status obk_select_delta(const obk_csr* A, const double* f, const double* candidates, int32_t n_candidates,
                            double tol, int64_t maxit, const obk_opts* opts, obk_stream_t stream, double* best_delta,
                            double* seconds, int64_t* sweeps, double* relres) {
    return guarded([&] {
        if (!A || !best_delta) obk::fail(OBK_E_ARG, "A and best_delta must not be NULL");
        if (n_candidates < 1 || !candidates) obk::fail(OBK_E_ARG, "no candidate thresholds");
        for (int32_t i = 0; i < n_candidates; i++)
            if (!(candidates[i] > 0.0) || !std::isfinite(candidates[i]))
                obk::fail(OBK_E_ARG, "a candidate threshold is not finite and > 0");
        if (!(tol > 0.0) || maxit < 1) obk::fail(OBK_E_ARG, "tol must be > 0 and maxit >= 1");
        const int64_t n_x = A->n_cols;
        // solution buffer in the input's memory space
        obk::DevArray<double> xd;
        std::vector<double> xh;
        double* x = nullptr;
        if (A->on_device) {
            xd.alloc((size_t)n_x);
            x = xd.get();
        } else {
            xh.assign((size_t)std::max<int64_t>(n_x, 1), 0.0);
            x = xh.data();
        }
        int32_t best = -1;
        double best_s = 0.0, best_r = 0.0;
        bool best_conv = false;
        for (int32_t i = 0; i < n_candidates; i++) {
            const auto t0 = std::chrono::steady_clock::now();
            obk_plan_t P = nullptr;
            obk_status st = obk_plan(A, f, candidates[i], opts, stream, &P);
            if (st != OBK_OK) obk::fail(st, obk::last_error_cstr());
            obk_info info{};
            st = obk_solve(P, nullptr, tol, maxit, x, &info, stream);
            const std::string msg = st != OBK_OK ? obk::last_error_cstr() : "";
            obk_free(P);
            if (st != OBK_OK) obk::fail(st, msg);
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (seconds) seconds[i] = sec;
            if (sweeps) sweeps[i] = info.sweeps;
            if (relres) relres[i] = info.relres;
            const bool conv = info.status == OBK_CONVERGED;
            const bool better = best < 0 || (conv && !best_conv) ||
                                (conv == best_conv && (conv ? sec < best_s : info.relres < best_r));
            if (better) {
                best = i;
                best_s = sec;
                best_r = info.relres;
                best_conv = conv;
            }
        }
        *best_delta = candidates[best];
    });
}

obk_status obk_plan_bytes(obk_plan_t plan, size_t* device_bytes) {
    return guarded([&] {
        if (!plan || !device_bytes) obk::fail(OBK_E_ARG, "NULL argument");
        *device_bytes = plan->device_bytes();
    });
}

obk_status obk_plan_stats(obk_plan_t plan, int64_t* n, int64_t* nnz, int32_t* n_groups, int64_t* bandwidth,
                          int64_t* n_conflicts) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (n) *n = plan->n;
        if (nnz) *nnz = plan->nnz;
        if (n_groups) *n_groups = plan->ngroups;
        if (bandwidth) *bandwidth = plan->bandwidth;
        if (n_conflicts) *n_conflicts = plan->nconflicts;
    });
}

obk_status obk_plan_lambda_bound(obk_plan_t plan, double* bound, double* per_group) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (plan->block_form()) obk::fail(OBK_E_ARG, "the bound concerns one-row groups; a block-form plan has none");
        if (!plan->cplx && plan->ngroups > 0 && plan->h_lambda_bound.empty()) {
            // formed on first request, on a stream of its own
            BusyGuard busy(plan);
            OBK_HIP(hipSetDevice(plan->device));
            hipStream_t s = nullptr;
            OBK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            struct SD { hipStream_t s; ~SD() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } } sd{s};
            obk::UserAllocScope ua(plan->opts.alloc, plan->opts.dealloc, plan->opts.ctx, s);
            obk::lambda_bound_on_request(*plan, s);
        }
        double b = 0.0;
        for (double v : plan->h_lambda_bound) b = std::max(b, v);
        if (bound) *bound = b;
        if (per_group && !plan->h_lambda_bound.empty())
            std::memcpy(per_group, plan->h_lambda_bound.data(), plan->h_lambda_bound.size() * sizeof(double));
    });
}

obk_status obk_plan_engine(obk_plan_t plan, int32_t* engine, int32_t* slabs) {
    return guarded([&] {
        if (!plan) obk::fail(OBK_E_ARG, "NULL plan");
        if (engine) *engine = plan->slab_S > 0 ? 2 : 1;
        if (slabs) *slabs = plan->slab_S;
    });
}

obk_status obk_rcm_host(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* perm) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!gptr || !perm))) obk::fail(OBK_E_ARG, "bad argument");
        if (n > 0 && gptr[n] > 0 && !gadj) obk::fail(OBK_E_ARG, "gadj is NULL");
        obk::host_rcm(n, gptr, gadj, perm);
    });
}

obk_status obk_validate_layout_host(int64_t n, int32_t n_groups, const int64_t* gptr, const int32_t* grow,
                                   const int32_t* group_of_row, const int64_t* rptr, const int32_t* rcol,
                                   const double* rval, const int64_t* tptr, const int32_t* tcol, const int64_t* sptr,
                                   const int32_t* srow, const double* sval, int32_t cplx, double delta) {
    return guarded([&] {
        if (n < 0 || n_groups < 0 || !gptr || !rptr || !tptr || !sptr || (n > 0 && !group_of_row) ||
            (gptr[n_groups] > 0 && (!grow || !rcol || !rval)) || (tptr[n_groups] > 0 && (!tcol || !srow || !sval)))
            obk::fail(OBK_E_ARG, "bad argument");
        obk::LayoutView L;
        L.n = n; L.ngroups = n_groups; L.gptr = gptr; L.grow = grow; L.group_of_row = group_of_row;
        L.rptr = rptr; L.rcol = rcol; L.rval = rval; L.tptr = tptr; L.tcol = tcol; L.sptr = sptr; L.srow = srow;
        L.sval = sval; L.cplx = cplx != 0; L.sval_conj = cplx != 0; L.delta = delta;
        obk::validate_layout(L);
    });
}

obk_status obk_first_fit_host(int64_t n, const int64_t* cptr, const int32_t* cidx, const uint8_t* active,
                              int32_t* group, int32_t* n_groups) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!cptr || !active || !group))) obk::fail(OBK_E_ARG, "bad argument");
        if (n > 0 && cptr[n] > 0 && !cidx) obk::fail(OBK_E_ARG, "cidx is NULL");
        int32_t ng = obk::host_first_fit(n, cptr, cidx, active, group);
        if (n_groups) *n_groups = ng;
    });
}

obk_status obk_batch_create(const obk_plan_t* plans, int count, const obk_batch_opts* opts, obk_batch_t* out) {
    if (out) *out = nullptr;
    obk_batch_s* B = nullptr;
    obk_status st = guarded([&] {
        if (!out || count < 0 || (count > 0 && !plans)) obk::fail(OBK_E_ARG, "bad argument");
        B = obk_batch_new();
        obk::batch_create(*B, plans, count, opts);
    });
    if (st != OBK_OK) { obk_batch_delete(B); return st; }
    *out = B;
    return OBK_OK;
}

obk_status obk_batch_reset(obk_batch_t batch, const obk_plan_t* plans, int count, obk_stream_t stream) {
    return guarded([&] {
        if (!batch || count < 0 || (count > 0 && !plans)) obk::fail(OBK_E_ARG, "bad argument");
        bool* busy = obk_batch_busy(batch);
        if (__atomic_exchange_n(busy, true, __ATOMIC_ACQ_REL)) obk::fail(OBK_E_BUSY, "a step on this batch is running");
        try {
            obk::batch_reset(*batch, plans, count, as_hip(stream));
        } catch (...) {
            __atomic_store_n(busy, false, __ATOMIC_RELEASE);
            throw;
        }
        __atomic_store_n(busy, false, __ATOMIC_RELEASE);
    });
}

obk_status obk_batch_begin(obk_batch_t batch, const double* const* x0, obk_stream_t stream) {
    return guarded([&] {
        if (!batch) obk::fail(OBK_E_ARG, "NULL batch");
        obk::batch_begin(*batch, x0, as_hip(stream));
    });
}

obk_status obk_batch_start(obk_batch_t batch, int index, const double* x0, obk_stream_t stream) {
    return guarded([&] {
        if (!batch || index < 0 || index >= obk_batch_count(batch)) obk::fail(OBK_E_ARG, "bad argument");
        obk::batch_start(*batch, index, x0, as_hip(stream));
    });
}

obk_status obk_batch_step(obk_batch_t batch, double tol, double* relres, int32_t* active, obk_stream_t stream) {
    return guarded([&] {
        if (!batch || std::isnan(tol)) obk::fail(OBK_E_ARG, "bad argument");
        bool* busy = obk_batch_busy(batch);
        if (__atomic_exchange_n(busy, true, __ATOMIC_ACQ_REL)) obk::fail(OBK_E_BUSY, "a step on this batch is running");
        try {
            obk::batch_step(*batch, tol, relres, active, as_hip(stream));
        } catch (...) {
            __atomic_store_n(busy, false, __ATOMIC_RELEASE);
            throw;
        }
        __atomic_store_n(busy, false, __ATOMIC_RELEASE);
    });
}

obk_status obk_batch_enable(obk_batch_t batch, const int32_t* enabled, obk_stream_t stream) {
    return guarded([&] {
        if (!batch || (!enabled && obk_batch_count(batch) > 0)) obk::fail(OBK_E_ARG, "bad argument");
        obk::batch_set_enabled(*batch, enabled, as_hip(stream));
    });
}

obk_status obk_batch_result(obk_batch_t batch, int index, double* x, obk_stream_t stream) {
    return guarded([&] {
        if (!batch || !x || index < 0 || index >= obk_batch_count(batch)) obk::fail(OBK_E_ARG, "bad argument");
        obk::batch_result(*batch, index, x, as_hip(stream));
    });
}

void obk_batch_free(obk_batch_t batch) {
    if (!batch) return;
    (void)hipDeviceSynchronize();
    obk_batch_delete(batch);
}

obk_status obk_solve_batch(const obk_plan_t* plans, int count, const double* const* x0, double tol, int64_t maxit,
                           double* const* x, obk_info* infos, const obk_batch_opts* opts, obk_stream_t stream) {
    return guarded([&] {
        if (count < 0 || (count > 0 && (!plans || !x)) || maxit < 0 || std::isnan(tol))
            obk::fail(OBK_E_ARG, "bad argument");
        auto t0 = std::chrono::steady_clock::now();
        obk_batch_s* B = obk_batch_new();
        struct Del { obk_batch_s* b; ~Del() { obk_batch_delete(b); } } del{B};
        obk::batch_create(*B, plans, count, opts);
        hipStream_t s = as_hip(stream);
        obk::batch_begin(*B, x0, s);
        std::vector<double> rr(count), first(count, -1.0);
        std::vector<int32_t> act(count), done(count, 0), steps(count, 0);
        std::vector<obk_info> inf(count);
        int remaining = count;
        for (int64_t it = 0; it < maxit && remaining > 0; it++) {
            obk::batch_step(*B, tol, rr.data(), act.data(), s);
            for (int i = 0; i < count; i++) {
                if (done[i]) continue;
                if (first[i] < 0) first[i] = rr[i];
                if (!act[i]) {
                    done[i] = 1;
                    remaining--;
                    inf[i].relres = rr[i];
                    inf[i].status = !std::isfinite(rr[i]) ? OBK_NONFINITE_ITERATE : OBK_CONVERGED;
                } else {
                    steps[i]++;
                }
            }
        }
        if (remaining > 0) {     // residual of the systems still running (no further update)
            obk::batch_step(*B, INFINITY, rr.data(), act.data(), s);
            for (int i = 0; i < count; i++)
                if (!done[i]) {
                    inf[i].relres = rr[i];
                    inf[i].status = !std::isfinite(rr[i]) ? OBK_NONFINITE_ITERATE
                                    : (tol > 0 && rr[i] <= tol) ? OBK_CONVERGED : OBK_MAXIT;
                    if (first[i] < 0) first[i] = rr[i];
                }
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < count; i++) {
            obk::batch_result(*B, i, x[i], s);
            const bool ir = plans[i]->opts.precision == OBK_FP32_IR;
            inf[i].outer_steps = steps[i];
            inf[i].sweeps = steps[i] * (ir ? plans[i]->opts.inner_sweeps : plans[i]->opts.check_every);
            inf[i].relres0 = first[i];
            inf[i].seconds = secs;
            if (infos) infos[i] = inf[i];
        }
    });
}

obk_status obk_batch_tune(const obk_plan_t* plans, int count, obk_batch_opts* best, double* seconds) {
    return guarded([&] {
        if (count <= 0 || !plans || !best) obk::fail(OBK_E_ARG, "bad argument");
        hipStream_t s = nullptr;
        OBK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        struct SD { hipStream_t s; ~SD() { (void)hipStreamDestroy(s); } } sd{s};
        double best_t = INFINITY;
        obk_batch_opts best_o{};
        for (int sub : {1, 2, 4}) {
            for (int per_cu : {1, 2, 4, 8}) {
                if (sub * per_cu > 16) continue;
                for (int64_t tw : {int64_t(0), int64_t(1) << 18, int64_t(1) << 20, int64_t(1) << 30}) {
                    obk_batch_opts o{per_cu, tw, 16, sub};
                    obk_batch_s* B = obk_batch_new();
                    struct Del { obk_batch_s* b; ~Del() { obk_batch_delete(b); } } del{B};
                    obk::batch_create(*B, plans, count, &o);
                    obk::batch_begin(*B, nullptr, s);
                    obk::batch_step(*B, -1.0, nullptr, nullptr, s);            // warm-up
                    auto t0 = std::chrono::steady_clock::now();
                    for (int r = 0; r < 2; r++) obk::batch_step(*B, -1.0, nullptr, nullptr, s);
                    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / 2;
                    if (t < best_t) { best_t = t; best_o = o; }
                }
            }
        }
        *best = best_o;
        if (seconds) *seconds = best_t;
        for (int i = 0; i < count; i++) {     // leave the iterates at zero
            obk_batch_s* B = obk_batch_new();
            struct Del { obk_batch_s* b; ~Del() { obk_batch_delete(b); } } del{B};
            obk::batch_create(*B, plans + i, 1, &best_o);
            obk::batch_begin(*B, nullptr, s);
        }
    });
}

const char* obk_last_error(void) { return obk::last_error_cstr(); }

}  // extern "C"
