// The C ABI of libobk: argument checks, error conversion, plan lifecycle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>

#include "obk_internal.h"

namespace obk {
const char* last_error_cstr();
void build_plan(obk_plan_s& P, const obk_csr& A, const double* f, double delta, hipStream_t s);
void solve_fp64(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                hipStream_t s);
void enqueue_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);
void solve_fp32_ir(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s);
}  // namespace obk

size_t obk_plan_s::device_bytes() const {
    return perm.bytes() + rptr.bytes() + rcol.bytes() + rval.bytes() + rf.bytes() + rinv.bytes() +
           tcol.bytes() + sptr.bytes() + srow.bytes() + sval.bytes() + rtiles.bytes() + stiles.bytes() +
           x.bytes() + w.bytes() + red.bytes() + rval32.bytes() + rinv32.bytes() + sval32.bytes() +
           b32.bytes() + d32.bytes() + w32.bytes() + r64.bytes();
}

namespace {

template <class F> obk_status guarded(F&& body) {
    try {
        body();
        obk::set_last_error("");
        return OBK_OK;
    } catch (const obk::Error& e) {
        obk::set_last_error(e.msg);
        (void)hipGetLastError();
        return e.code;
    } catch (const std::bad_alloc&) {
        obk::set_last_error("host allocation failed");
        return OBK_E_NOMEM;
    } catch (...) {
        obk::set_last_error("unexpected internal error");
        return OBK_E_HIP;
    }
}

hipStream_t as_hip(obk_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

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
    return OBK_OK;
}

obk_status obk_plan(const obk_csr* A, const double* f, double delta, const obk_opts* opts, obk_stream_t stream,
                    obk_plan_t* out) {
    if (out) *out = nullptr;
    obk_plan_s* P = nullptr;
    obk_status st = guarded([&] {
        if (!A || !out) obk::fail(OBK_E_ARG, "A and out must not be NULL");
        if (A->n_rows != A->n_cols) obk::fail(OBK_E_NOT_SQUARE, "the method needs a square matrix");
        if (A->n_rows < 0 || A->nnz < 0) obk::fail(OBK_E_ARG, "negative size");
        if (A->n_rows >= std::numeric_limits<int32_t>::max() || A->nnz >= std::numeric_limits<int32_t>::max())
            obk::fail(OBK_E_ARG, "n and nnz must be below 2^31 - 1");
        if (A->n_rows > 0 && (!A->row_ptr || !f)) obk::fail(OBK_E_ARG, "row_ptr and f must not be NULL");
        if (A->nnz > 0 && (!A->col || !A->val)) obk::fail(OBK_E_ARG, "col and val must not be NULL");
        if (!(delta > 0.0) || !std::isfinite(delta)) obk::fail(OBK_E_ARG, "delta must be finite and > 0");
        obk_opts o;
        obk_opts_default(&o);
        if (opts) o = *opts;
        if (o.precision != OBK_FP64 && o.precision != OBK_FP32_IR) obk::fail(OBK_E_ARG, "unknown precision");
        if (o.inner_sweeps < 1 || o.check_every < 1) obk::fail(OBK_E_ARG, "inner_sweeps and check_every must be >= 1");
        P = new obk_plan_s();
        P->opts = o;
        obk::build_plan(*P, *A, f, delta, as_hip(stream));
    });
    if (st != OBK_OK) {
        delete P;
        return st;
    }
    *out = P;
    return OBK_OK;
}

obk_status obk_solve(obk_plan_t plan, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                     obk_stream_t stream) {
    return guarded([&] {
        if (!plan || !x) obk::fail(OBK_E_ARG, "plan and x must not be NULL");
        if (maxit < 0 || std::isnan(tol)) obk::fail(OBK_E_ARG, "maxit must be >= 0 and tol a number");
        BusyGuard busy(plan);
        OBK_HIP(hipSetDevice(plan->device));
        if (plan->opts.precision == OBK_FP32_IR)
            obk::solve_fp32_ir(*plan, x0, tol, maxit, x, info, as_hip(stream));
        else
            obk::solve_fp64(*plan, x0, tol, maxit, x, info, as_hip(stream));
    });
}

obk_status obk_sweep_device(obk_plan_t plan, double* x_tilde_dev, int64_t sweeps, obk_stream_t stream) {
    return guarded([&] {
        if (!plan || !x_tilde_dev) obk::fail(OBK_E_ARG, "plan and x_tilde_dev must not be NULL");
        if (sweeps < 0) obk::fail(OBK_E_ARG, "sweeps must be >= 0");
        OBK_HIP(hipSetDevice(plan->device));
        obk::enqueue_sweeps(*plan, x_tilde_dev, sweeps, as_hip(stream));
    });
}

void obk_free(obk_plan_t plan) {
    if (!plan) return;
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    delete plan;
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

obk_status obk_rcm_host(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* perm) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!gptr || !perm))) obk::fail(OBK_E_ARG, "bad argument");
        if (n > 0 && gptr[n] > 0 && !gadj) obk::fail(OBK_E_ARG, "gadj is NULL");
        obk::host_rcm(n, gptr, gadj, perm);
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

const char* obk_last_error(void) { return obk::last_error_cstr(); }

}  // extern "C"
