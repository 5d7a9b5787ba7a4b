// Internal declarations of libobk (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/obk.h"
#include "obk_tile.h"

namespace obk {

// ---------------------------------------------------------------- errors
// Thrown inside the library only; every ABI entry point catches and converts.
struct Error {
    obk_status code;
    std::string msg;
};
[[noreturn]] void fail(obk_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define OBK_HIP(call) ::obk::check_hip((call), #call)
void set_last_error(const std::string& msg);
// OBK_LOG (environment, read once): 0 silent (default), 1 every failed call
// with its status and message, 2 also a line per plan, solve and batch
// (re)formation, 3 also a line per batched step.  Lines go to stderr.
int log_level();
void log_line(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// ------------------------------------------------------- device memory
// Owning device buffer; all plan memory goes through it so that the plan
// can report its footprint.
//
// While an AllocScope is active on the calling thread, buffers are taken from
// the device's stream-ordered pool (hipMallocAsync on the scope's stream) and
// returned with hipFreeAsync: on the scope's stream while it is active, else on
// the null stream, after the owner has synchronised the device (obk_free
// does).  Plan building on one thread then never waits for work that other
// threads run on the device, as a synchronous hipFree may.  Inside the scope,
// a released buffer is kept by the scope (by size class) and serves the next
// request of its class there: all of the scope's work runs on its stream, so
// the new owner's work is ordered after the old owner's.  The pool's own
// calls cost tens of microseconds each and serialise across threads; a plan
// makes over a hundred temporaries.  When the scope ends it synchronises its
// stream and leaves what it keeps to a process-wide store of idle blocks (at
// most 1 GiB, by device and size class), from which later scopes on any
// thread and stream take before they ask the pool.
struct AllocScope {
    hipStream_t prev_stream;
    bool prev_on;
    void* prev_cache;
    explicit AllocScope(hipStream_t s);
    ~AllocScope();
};
// True while an AllocScope is active on this thread: temporaries are then
// freed in stream order and need no synchronisation before they go.
bool alloc_scoped();
// Synchronise s unless temporaries are freed in stream order.
void sync_for_free(hipStream_t s);
// Pinned host staging buffer of the calling thread (grown on demand, kept
// until the thread ends); every user completes its copy before returning.
void* pinned_stage(size_t bytes);
// Host <-> device copies through that buffer, in chunks of at most 8 MiB with
// two in flight (a large array needs no pinned buffer of its own size:
// pinning hundreds of megabytes costs more than the copy); both return with
// the copy complete and the stream synchronised.
void stage_h2d(void* d, const void* h, size_t bytes, hipStream_t s);
void stage_d2h(void* h, const void* d, size_t bytes, hipStream_t s);

// While a UserAllocScope is active on the calling thread, buffers come from
// the caller's allocator (obk_opts.alloc / dealloc / ctx) instead; each
// buffer keeps its dealloc, and a temporary released while the scope is
// active first waits for the scope's stream.
struct UserAllocScope {
    void* (*prev_alloc)(size_t, void*);
    void (*prev_dealloc)(void*, void*);
    void* prev_ctx;
    hipStream_t prev_stream;
    UserAllocScope(void* (*alloc)(size_t, void*), void (*dealloc)(void*, void*), void* ctx, hipStream_t s);
    ~UserAllocScope();
};

struct DevMem {
    void* ptr = nullptr;
    size_t bytes = 0;
    size_t cap = 0;          // block size when it came from an AllocScope's size classes
    bool pooled = false;
    void (*dealloc)(void*, void*) = nullptr;   // the caller's deallocator, when it came from alloc
    void* ctx = nullptr;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    DevMem(DevMem&& o) noexcept
        : ptr(o.ptr), bytes(o.bytes), cap(o.cap), pooled(o.pooled), dealloc(o.dealloc), ctx(o.ctx) {
        o.ptr = nullptr; o.bytes = 0; o.cap = 0; o.pooled = false; o.dealloc = nullptr; o.ctx = nullptr;
    }
    DevMem& operator=(DevMem&& o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr; bytes = o.bytes; cap = o.cap; pooled = o.pooled; dealloc = o.dealloc; ctx = o.ctx;
            o.ptr = nullptr; o.bytes = 0; o.cap = 0; o.pooled = false; o.dealloc = nullptr; o.ctx = nullptr;
        }
        return *this;
    }
    ~DevMem() { release(); }
    void alloc(size_t b);
    void release();
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

template <class T> struct DevArray {
    DevMem mem;
    size_t count = 0;
    void alloc(size_t n) { mem.alloc(n * sizeof(T) + (n == 0 ? sizeof(T) : 0)); count = n; }
    T* get() const { return mem.as<T>(); }
    size_t bytes() const { return mem.bytes; }
};

// ------------------------------------------------------- device primitives
// Exclusive prefix sum of n int64 values (in -> out, may alias); returns the
// total on the host (synchronises the stream).
int64_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
// Same for int32 counts producing int64 offsets.
int64_t scan_counts_i32(const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs by the low `key_bits` bits of
// the uint32 keys.  keys/vals are sorted in place (scratch of equal size is
// allocated internally).  vals may be null (keys only).
void radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits, hipStream_t s);
int bits_for(uint64_t max_value);

// ----------------------------------------------------------- host graph
// Reverse Cuthill-McKee order of an undirected graph given as a symmetric
// adjacency structure without self loops (gptr[n+1], gadj[gptr[n]]).
// Tie-break: start at the unvisited vertex of least (degree, index); visit
// unvisited neighbours by ascending (degree, index); reverse the whole
// Cuthill-McKee sequence.  perm[t] = old index of new position t.
void host_rcm(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* perm);
// The same Cuthill-McKee sequence (not reversed) continued from a state of
// the search: cm[0, tail) appended so far, seen[] their flags, cm[head, tail)
// not yet expanded.  (0, 0) with no vertex seen starts it.
void host_cm_resume(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* cm, uint8_t* seen, int64_t head,
                    int64_t tail);
// The reverse Cuthill-McKee order of the same graph formed on the device, one
// breadth-first level per step (adj, deg: device adjacency in row order and
// degrees).  With give_up, once at least 4 levels are done, they hold fewer
// than kDeviceRcmMinWidth vertices each on average and the last one is less
// than twice the one before, the host loop finishes the search from the
// device's state.  perm is host memory.
constexpr int64_t kDeviceRcmMinWidth = 2048;
constexpr int64_t kDeviceRcmMinN = 16384;     // use_rcm = 1: smaller graphs go to the host loop
void device_rcm(int64_t n, const int32_t* adj, const int32_t* deg, bool give_up, hipStream_t s, int32_t* perm);
// First-fit colouring in row order: row i takes the least colour not used
// by any conflicting row j < i (conflict lists cptr[n+1], cidx).  Rows with
// active[i] == 0 get colour -1.  Returns the number of colours.
int32_t host_first_fit(int64_t n, const int64_t* cptr, const int32_t* cidx, const uint8_t* active,
                       int32_t* colour);

// --------------------------------------------------------- sweep schedule
// Split segments [0, nseg) with offsets off[nseg+1] into tiles of at most
// kTileSegs segments and (unless a single segment is longer) at most
// kTileEntries entries.
void build_tiles(int64_t seg0, int64_t seg1, const int64_t* off, std::vector<Tile>& out);

// The group-major layout of a one-row-block plan, as host arrays, for the
// plan validator.  rval/sval: one value per entry, or (re, im) pairs when
// cplx; sval_conj: the column copies hold conj(a).  Tiles may be null.
struct LayoutView {
    int64_t n = 0;
    int32_t ngroups = 0;
    const int64_t* gptr = nullptr;        // [G+1] group-major rows of each group
    const int32_t* grow = nullptr;        // [m] reordered row of each group-major row
    const int32_t* group_of_row = nullptr;   // [n] group of each reordered row (-1: none)
    const int64_t* rptr = nullptr;        // [m+1]
    const int32_t* rcol = nullptr;
    const double* rval = nullptr;
    const int64_t* tptr = nullptr;        // [G+1] column segments of each group
    const int32_t* tcol = nullptr;        // [T]
    const int64_t* sptr = nullptr;        // [T+1]
    const int32_t* srow = nullptr;        // group-major row of each column entry
    const double* sval = nullptr;
    bool cplx = false, sval_conj = false;
    double delta = 0.0;
    const Tile* rtiles = nullptr;
    const int32_t* rtile_ptr = nullptr;   // [G+1]
    const Tile* stiles = nullptr;
    const int32_t* stile_ptr = nullptr;   // [G+1]
};
void validate_layout(const LayoutView& L);

}  // namespace obk

struct obk_plan_s;
namespace obk {
// Complex systems: plan-stage helpers (values as separate real and imaginary
// arrays) and the solve on a complex plan (interleaved values).
void z_split(const double* in, int64_t n, double* re, double* im, hipStream_t s);
void z_fill_zero(double* p, int64_t n, hipStream_t s);
void z_finite(const double* a, int64_t n, int* flags, int bit, hipStream_t s);
void z_gather_i32(int64_t n, const int32_t* idx, const double* src, double* dst, hipStream_t s);
void z_gather_u32(int64_t n, const uint32_t* idx, const double* src, double* dst, hipStream_t s);
void z_norms(int64_t n, const int64_t* trp, const double* tv, const double* tvi, double* nu, double* inv,
             hipStream_t s);
void z_conflicts(bool fill, int64_t nnz, const int64_t* trp, const int32_t* tci, const double* tv, const double* tvi,
                 const int32_t* trow, const int64_t* cptr, const int32_t* crow, const double* nu, double delta,
                 int64_t* count, const int64_t* out_pos, int32_t* out_idx, hipStream_t s);
void z_relayout(int64_t m, const int32_t* grow, const int64_t* trp, const double* tv, const double* tvi,
                const double* tf, const double* tfi, const int64_t* rptr, double* rvalz, double* rfz,
                hipStream_t s);
void z_pack(int64_t n, const double* re, const double* im, bool conjugate, double* out, hipStream_t s);
void solve_complex(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s);
void enqueue_sweeps_z(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);
int32_t profile_sweeps_z(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                         int32_t max_out);

// Centroid cosines, pairing and projection workspace of a block-form plan
// (after the shared plan stages).
void block_setup(obk_plan_s& P, hipStream_t s);
// Banded Cholesky factors of A_t A_t^T for the blocks that have one (full row
// rank to the pivot test, band within the size limits); sets h_bdirect.
void block_factor(obk_plan_s& P, hipStream_t s);
// `sweeps` block sweeps on x (device, reordered); synchronises the stream.
// ms (may be null) receives the launch's event time in milliseconds.
void block_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, float* ms);
int32_t profile_block(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s, obk_kernel_profile* out,
                      int32_t max_out);
// Banded sweep engine (obk_slab.hip): one persistent launch in which each
// workgroup owns a contiguous slab of the reordered unknowns.
struct SlabPhase {           // one phase (R or S) of one group on one slab
    int64_t item_off;        // first item in the item arrays
    int32_t count;           // items (rows in R, touched window columns in S)
    int32_t round0, nrounds; // rounds in the round table
    int32_t ents;            // entries of all its rounds (ELL, padding included)
    int32_t cache;           // byte offset of its copy in the LDS cache, -1: streamed
    int32_t pad;
};
struct SlabRound {           // items [r * QT, ...) of a phase, entry-major
    int64_t ent_off;         // first entry of the round
    int32_t K;               // entries per item in the round (its longest item)
    int32_t pad;
};
struct SlabGroup {           // one group on one slab
    SlabPhase r;             // phase R: the own rows of the group
    SlabPhase s, sb;         // phase S: window columns whose rows are all own rows (s, run
                             // before the exchange) and those with halo rows (sb, after it)
    int32_t lo_cnt, own_cnt, hi_cnt;   // w window: [lower halo | own rows | upper halo]
    int32_t pre_cnt, suf_cnt;          // own rows published to slab k-1 (first) and k+1 (last)
    int32_t xoff;                      // the group's offset in every exchange buffer (same on all slabs)
};
struct SlabDesc {            // one slab
    int32_t xlo, xcount;     // x window: reordered columns [xlo, xlo + xcount)
    int32_t own_lo, own_cnt; // own columns: window positions [own_lo, own_lo + own_cnt)
    int32_t round_first, round_count;   // the slab's rounds (contiguous in the round table)
    int32_t cache_bytes;     // bytes of its phases copied to LDS at launch start
    int32_t pad;
};
constexpr int32_t kSlabMaxGroups = 64;

// Workspace of the no-allocation solve: the residual partials (static
// device scratch) instead of the plan's.
struct SolveWs {
    double* red = nullptr;
};
void solve_noalloc(obk_plan_s& P, const double* x0, double tol, int64_t maxit, double* x, obk_info* info,
                   hipStream_t s);
void slab_setup(obk_plan_s& P, const std::vector<int64_t>& hrptr, const std::vector<int32_t>& grow,
                const std::vector<int32_t>& pos, hipStream_t s);
void slab_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);
double slab_profile(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);
void slab_check(obk_plan_s& P, hipStream_t s);
}  // namespace obk

// --------------------------------------------------------------- the plan
struct obk_plan_s {
    int device = 0;
    int64_t n = 0, nnz = 0;      // n: size of the (extended) square system
    int64_t n_in = 0, m_in = 0;  // unknowns and equations of the caller's system
    int64_t m = 0;              // rows that take part in a group (nonzero rows)
    int32_t ngroups = 0;
    int64_t bandwidth = 0;
    int64_t nconflicts = 0;
    obk_opts opts{};
    double delta = 0;
    bool cplx = false;           // complex system: values, f~, x~, w interleaved (re, im)
    bool input_on_device = false;
    bool busy = false;

    // host copies (introspection, schedule)
    std::vector<int32_t> h_perm;       // new -> old
    std::vector<int32_t> h_group;      // group of each reordered row (-1 zero row)
    std::vector<double> h_lambda_bound;   // per group: Gershgorin bound on lambda_max(B_g B_g^T)
    std::vector<int64_t> h_gptr;       // group g = group-major rows [gptr[g], gptr[g+1])
    std::vector<int64_t> h_tptr;       // touched columns of group g: [tptr[g], tptr[g+1])
    std::vector<obk::Tile> h_rtiles, h_stiles;
    std::vector<int32_t> h_rtile_ptr, h_stile_ptr;   // tiles of group g

    // device: permutation
    obk::DevArray<int32_t> perm;       // new -> old
    // device: group-major CSR of A~ (columns in reordered numbering, rows sorted)
    obk::DevArray<int64_t> rptr;       // [m+1]
    obk::DevArray<int32_t> rcol;       // [nnz]
    obk::DevArray<double> rval;        // [nnz]
    obk::DevArray<double> rf;          // f~ in group-major order [m]
    obk::DevArray<double> rinv;        // 1/||a||^2 in group-major order [m]
    // device: per-group CSC (scatter-owner lists)
    obk::DevArray<int32_t> tcol;       // touched column of each segment [T]
    obk::DevArray<int64_t> sptr;       // [T+1]
    obk::DevArray<int32_t> srow;       // group-major row of each entry [nnz]
    obk::DevArray<double> sval;        // [nnz]
    // device: tiles, and the tile range of each group
    obk::DevArray<obk::Tile> rtiles, stiles;
    obk::DevArray<int32_t> d_rtile_ptr, d_stile_ptr;   // [G+1]
    // device: workspace
    obk::DevArray<double> x;           // reordered iterate [n]
    obk::DevArray<double> w;           // group weights [m]
    obk::DevArray<double> red;         // reduction scratch
    double fnorm2 = 0;                 // ||f~||^2
    double zero_rows_f2 = 0;           // sum of f_i^2 over all-zero rows
    double zero_rows_fmax = 0;         // max |f_i| over all-zero rows

    // FP32 copies and workspace for iterative refinement (precision OBK_FP32_IR)
    obk::DevArray<float> rval32;       // [nnz]
    obk::DevArray<float> rinv32;       // [m]
    obk::DevArray<float> sval32;       // [nnz]
    obk::DevArray<float> b32;          // scaled residual, group-major [m]
    obk::DevArray<float> d32;          // correction, reordered [n]
    obk::DevArray<float> w32;          // group weights [m]
    obk::DevArray<double> r64;         // FP64 residual, group-major [m]

    // complex plans: interleaved values of the group-major CSR and the
    // per-group CSC, and f~ (rval, sval, rf stay empty)
    obk::DevArray<double> rvalz;       // [2 nnz]
    obk::DevArray<double> svalz;       // [2 nnz], conj(a): phase S adds w conj(a)
    obk::DevArray<double> rfz;         // [2 m]

    // block form (opts.block_k > 0): groups are the k blocks, rows stay in
    // reordered order (m = n) and the per-group CSC is the per-block CSC
    std::vector<int64_t> h_bptr;       // block b = rows [bptr[b], bptr[b+1])  [k+1]
    std::vector<double> h_bcos;        // |cos| of the block centroids, row-major [k*k]
    std::vector<int32_t> h_partner;    // paired block (-1: Nclass) [k]
    std::vector<int32_t> h_border;     // blocks in projection order of a sweep [k]
    std::vector<int64_t> h_bnnz;       // entries of each block [k]
    obk::DevArray<int64_t> d_bptr, d_btptr;   // row and segment ranges per block [k+1]
    obk::DevArray<int32_t> d_border;
    obk::DevArray<double> bres, bp, bu;       // CG residual and direction [n], A_t^T p [n]
    obk::DevArray<double> bpart;              // per-workgroup partial sums
    obk::DevArray<uint64_t> bbar;             // grid barrier arrival counter [1]
    obk::DevArray<int> berr;                  // [1]: a barrier wait timed out
    obk::DevArray<int64_t> biters;            // CG iterations per block [k]
    obk::DevArray<int32_t> blseg;             // per CSR entry: local index of its column in its block
    obk::DevArray<int32_t> d_bfit;            // per block: projected from LDS in one-workgroup launches
    std::vector<int32_t> h_bfit;
    int64_t block_lds = 0;                    // dynamic LDS bytes of a one-workgroup launch (0: none fits)
    int block_occ = 0;                        // resident workgroups per CU of the projection launch
    // direct projections (opts.block_solver = 0): banded Cholesky factor L of
    // P A_t A_t^T P^T per block (P: the reverse Cuthill-McKee order of the
    // block's Gram graph), bandwidth bw_b, stored twice: by columns,
    // lfc[off_b + c (bw_b+1) + d] = L[c+d][c], and by rows,
    // lfr[off_b + i (bw_b+1) + bw_b - (i-j)] = L[i][j] (zero outside the band);
    // ldinv[row] = 1 / L[i][i]
    std::vector<int32_t> h_bdirect;           // per block: 1 when projected from its factor [k]
    std::vector<int64_t> h_bbw;               // per block: factor bandwidth, -1 without one [k]
    obk::DevArray<int32_t> d_bdirect, d_bbw;
    obk::DevArray<int64_t> d_boff;            // per block: offset of its factor in lfc / lfr
    obk::DevArray<double> lfc, lfr, ldinv;
    obk::DevArray<int32_t> d_lperm, d_lpos;   // factor order of each block's rows, and its inverse [n]
    int64_t direct_lds = 0;                   // dynamic LDS bytes of a direct projection (0: none)

    // banded sweep engine (slab_S > 0 when it runs the FP64 sweeps)
    int32_t slab_S = 0;                       // slabs (workgroups) of the launch
    int64_t slab_xmax = 0, slab_wmax = 0;     // largest x and w windows (LDS doubles)
    int64_t slab_cap = 0;                     // exchange buffer doubles per (slab, side, parity)
    int64_t slab_lds = 0;                     // dynamic LDS bytes
    int64_t slab_meta_off = 0, slab_cache_off = 0;   // LDS byte offsets of descriptors and cached phases
    double slab_bytes_per_sweep = 0;          // bytes one sweep streams (items, entries, exchange)
    double slab_bytes_per_launch = 0;         // bytes read once per launch (windows, cached phases)
    obk::DevArray<obk::SlabDesc> sl_desc;
    obk::DevArray<obk::SlabGroup> sl_grp;
    obk::DevArray<obk::SlabRound> sl_round;
    obk::DevArray<uint16_t> sl_tgt, sl_len, sl_idx;
    obk::DevArray<double> sl_f, sl_val, sl_xbuf;
    obk::DevArray<uint32_t> sl_flags;
    obk::DevArray<int> sl_err;

    // captured sweep sequences (hipGraph), keyed by iterate pointer, sweep
    // count and element size; replayed on the caller's stream
    struct SweepGraph {
        const void* x = nullptr;
        int64_t sweeps = 0;
        int elem = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<SweepGraph> graphs;
    hipStream_t capture_stream = nullptr;

    obk_plan_s() = default;
    obk_plan_s(const obk_plan_s&) = delete;
    obk_plan_s& operator=(const obk_plan_s&) = delete;
    ~obk_plan_s();
    size_t device_bytes() const;
    bool has_fp32() const { return opts.precision == OBK_FP32_IR; }
    bool block_form() const { return opts.block_k > 0; }
};
