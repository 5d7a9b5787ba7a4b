// Batched solves: many independent plans advanced in shared launches.
//
// A refinement step over a batch (all plans OBK_FP32_IR):
//   1. one launch computes r = f~ - A~ x~ in FP64 for every system (row blocks
//      of all systems) with per-block sums of r^2 and maxima of |r|;
//   2. one launch reduces them per system (fixed order): relres, sigma and the
//      system's active flag (relres > tol, sigma > 0, finite);
//   3. one launch forms b = (float)(r / sigma) and d = 0 for active systems;
//   4. ONE persistent launch runs the inner FP32 sweeps of every active
//      system: each system is owned by a team of workgroups placed on one XCD
//      (team size from the system's work), teams synchronise only among
//      themselves between the phases of a sweep;
//   5. one launch applies x~ += sigma d in FP64.
// With OBK_FP64 plans, step 4 runs check_every FP64 sweeps on x~ directly and
// steps 3 and 5 are skipped.
//
// Team barriers are generation barriers in device memory (agent-scope
// release/acquire); a workgroup's task list is ordered by team id, so a team
// can always complete once its lowest-numbered members arrive.  Every wait is
// bounded: past the bound the kernel records an error and leaves, and the host
// reports OBK_E_HIP.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "obk_internal.h"
#include "obk_sweep_tiles.h"

namespace obk {

void enqueue_sweeps(obk_plan_s& P, double* x, int64_t sweeps, hipStream_t s);

namespace {

constexpr long kSpinLimit = 1L << 22;
// Merged tiles of the batched sweep: up to kBatchQ * 256 segments (kBatchQ
// per thread) and kBatchChunk entries; FP32 stages them in one chunk of 16
// entries per thread, FP64 (twice the registers per value) in two of 8.
constexpr int kBatchQ = 2;
constexpr int kBatchChunk = kTileThreads * 16;
template <class T> constexpr int batch_e() { return sizeof(T) == 4 ? 16 : 8; }

template <class T> struct BatchSys {
    const Tile* rtiles;
    const Tile* stiles;
    const int32_t* rtile_ptr;
    const int32_t* stile_ptr;
    const int64_t* rptr;
    const int32_t* rcol;
    const T* rval;
    const T* rf;
    const T* rinv;
    const int64_t* sptr;
    const int32_t* srow;
    const T* sval;
    const int32_t* tcol;
    T* x;
    T* w;
    int32_t ngroups;
    int32_t team;
    uint32_t* bar;           // [0] arrivals, [1] generation
    T omega;                 // relaxation of the row steps
};

struct TeamTask {
    int32_t sys;
    int32_t rank;
};

struct Block {               // a range of rows or columns of one system
    int32_t sys;
    int32_t begin;
    int32_t end;
};

struct ResSys {              // FP64 arrays for residual, scaling and update
    const Tile* rtiles;
    const int64_t* rptr;
    const int32_t* rcol;
    const double* rval;
    const double* rf;
    double* x;
    double* r;
    float* b;
    float* d;
    double fnorm2, zero_f2, zero_fmax;
};

// Barrier of a system's team; false (for every thread of the workgroup) when
// the wait timed out, after which the launch is abandoned: the workgroup
// leaves, its teammates time out in turn, and the host reports the error flag.
__device__ __forceinline__ bool team_barrier(uint32_t* bar, int team, int* err) {
    __shared__ int timed_out;
    __syncthreads();
    if (team > 1) {
        if (threadIdx.x == 0) timed_out = 0;
        if (threadIdx.x == 0) {
            const uint32_t gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t arrived =
                __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == (uint32_t)team - 1) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                // bounded wait for the generation to move on
                uint32_t cur = gen;
                long spins = 0;
#pragma clang loop unroll(disable)
                do {
                    __builtin_amdgcn_s_sleep(1);
                    cur = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    spins++;
                } while ((cur == gen) & (spins <= kSpinLimit));
                if (cur == gen) {
                    atomicOr(err, 1);
                    timed_out = 1;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        return timed_out == 0;
    }
    return true;
}

// Tiles of one phase handled by team member `rank`: r0 + rank + j * team for
// j = 0, 1, ...; a workgroup takes SUB of them per pass, one per sub-block.
template <class T, int SUB, bool kR>
__device__ __forceinline__ void team_phase(const BatchSys<T>& S, int32_t g, int32_t rank, T* prod) {
    const Tile* tiles = kR ? S.rtiles : S.stiles;
    const int32_t r0 = kR ? S.rtile_ptr[g] : S.stile_ptr[g];
    const int32_t r1 = kR ? S.rtile_ptr[g + 1] : S.stile_ptr[g + 1];
    const int32_t mine = (r1 - r0 > rank) ? (r1 - r0 - rank + S.team - 1) / S.team : 0;
    const int32_t passes = (mine + SUB - 1) / SUB;
    const int sb = threadIdx.x / kTileThreads;
    __shared__ int chunks[SUB];
    for (int32_t p = 0; p < passes; p++) {
        // each sub-block loads its own tile (clamped index: pass p always has j = p * SUB < mine)
        const int32_t j = p * SUB + sb;
        const bool ok = j < mine;
        const Tile tb = tiles[r0 + rank + (ok ? j : p * SUB) * S.team];
        Tile mt;
        mt.seg_begin = ok ? tb.seg_begin : 0;
        mt.seg_end = ok ? tb.seg_end : 0;
        mt.ent_begin = ok ? tb.ent_begin : 0;
        mt.ent_end = ok ? tb.ent_end : 0;
        constexpr int E = batch_e<T>();
        if ((threadIdx.x & (kTileThreads - 1)) == 0) chunks[sb] = tile_chunks<E>(mt);
        __syncthreads();
        int nchunks = 0;
        for (int b = 0; b < SUB; b++) nchunks = max(nchunks, chunks[b]);
        if (kR)
            tile_phase_r<T, kBatchQ, E>(mt, nchunks, prod, S.rptr, S.rcol, S.rval, S.rf, S.rinv, S.x, S.w, S.omega);
        else
            tile_phase_s<T, kBatchQ, E>(mt, nchunks, prod, S.sptr, S.srow, S.sval, S.tcol, S.w, S.x);
    }
}

template <class T, int SUB>
__global__ __launch_bounds__(kTileThreads * SUB) void k_batch_sweeps(const BatchSys<T>* __restrict__ systems,
                                                                     const int32_t* __restrict__ task_ptr,
                                                                     const TeamTask* __restrict__ tasks,
                                                                     const uint8_t* __restrict__ active, int sweeps,
                                                                     int* err, uint64_t* __restrict__ trace) {
    constexpr int chunk = kTileThreads * batch_e<T>();
    __shared__ T prod_all[SUB * chunk];
    T* prod = prod_all + (threadIdx.x / kTileThreads) * chunk;
    const int32_t t0 = task_ptr[blockIdx.x], t1 = task_ptr[blockIdx.x + 1];
    if (trace && threadIdx.x == 0) trace[2 * blockIdx.x] = wall_clock64();
    for (int32_t ti = t0; ti < t1; ti++) {
        const TeamTask tk = tasks[ti];
        if (!active[tk.sys]) continue;
        const BatchSys<T> S = systems[tk.sys];
        for (int sw = 0; sw < sweeps; sw++) {
            for (int32_t g = 0; g < S.ngroups; g++) {
                team_phase<T, SUB, true>(S, g, tk.rank, prod);
                if (!team_barrier(S.bar, S.team, err)) return;
                team_phase<T, SUB, false>(S, g, tk.rank, prod);
                if (!team_barrier(S.bar, S.team, err)) return;
            }
        }
    }
    if (trace && threadIdx.x == 0) trace[2 * blockIdx.x + 1] = wall_clock64();
}

// FP64 residual of one R tile of one system per workgroup (block = {system,
// tile}); the per-tile partials are those of the single-system solve, so the
// per-system reduction in k_batch_reduce gives the same relative residual.
__global__ __launch_bounds__(kTileThreads) void k_batch_resid(const int64_t* __restrict__ dims,
                                                              const ResSys* __restrict__ sys,
                                                              const Block* __restrict__ blocks,
                                                              double* __restrict__ psum, double* __restrict__ pmax,
                                                              int* __restrict__ nonfinite) {
    __shared__ double prod[kTileEntries];
    if ((int64_t)blockIdx.x >= dims[0]) return;
    const Block bk = blocks[blockIdx.x];
    const ResSys S = sys[bk.sys];
    const Tile t = S.rtiles[bk.begin];
    double s2, mx;
    tile_resid(t, tile_chunks(t), prod, S.rptr, S.rcol, S.rval, S.rf, S.x, S.r, nonfinite, s2, mx);
    if (threadIdx.x == 0) { psum[blockIdx.x] = s2; pmax[blockIdx.x] = mx; }
}

__global__ __launch_bounds__(256) void k_batch_reduce(const int64_t* __restrict__ dims,
                                                      const ResSys* __restrict__ sys,
                                                      const int32_t* __restrict__ blk_ptr,
                                                      const double* __restrict__ psum,
                                                      const double* __restrict__ pmax, double tol,
                                                      const uint8_t* __restrict__ enabled,
                                                      double* __restrict__ relres, double* __restrict__ sigma,
                                                      uint8_t* __restrict__ active) {
    __shared__ double red[256];
    __shared__ double mx[256];
    if ((int64_t)blockIdx.x >= dims[1]) return;
    const int s = blockIdx.x;
    const int32_t b0 = blk_ptr[s], b1 = blk_ptr[s + 1];
    double acc = 0.0, m = 0.0;
    for (int32_t b = b0 + threadIdx.x; b < b1; b += 256) { acc = acc + psum[b]; m = fmax(m, pmax[b]); }
    red[threadIdx.x] = acc;
    mx[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + st]);
        }
        __syncthreads();
    }
    // every thread derives the (uniform) results; thread 0 stores them
    const ResSys S = sys[s];
    const double r2 = red[0] + S.zero_f2;
    const double sg = fmax(mx[0], S.zero_fmax);
    const double denom = (S.fnorm2 == 0.0) ? 1.0 : S.fnorm2;
    const double q = sqrt(r2) / sqrt(denom);
    const double rho = (S.fnorm2 == 0.0) ? ((r2 == 0.0) ? 0.0 : INFINITY) : q;
    const bool go = enabled[s] && isfinite(rho) && (rho > tol) && (sg > 0.0);
    if (threadIdx.x == 0) {
        relres[s] = rho;
        sigma[s] = sg;
        active[s] = go ? 1 : 0;
    }
}

__global__ void k_batch_rhs(const int64_t* __restrict__ dims, const ResSys* __restrict__ sys,
                            const Block* __restrict__ rows, const double* __restrict__ sigma,
                            const uint8_t* __restrict__ active) {
    if ((int64_t)blockIdx.x >= dims[2]) return;
    const Block bk = rows[blockIdx.x];
    const int64_t a = bk.begin + (int64_t)threadIdx.x;
    if (a >= bk.end || !active[bk.sys]) return;
    const ResSys S = sys[bk.sys];
    S.b[a] = (float)(S.r[a] / sigma[bk.sys]);
}

__global__ void k_batch_cols(const int64_t* __restrict__ dims, const ResSys* __restrict__ sys,
                             const Block* __restrict__ cols, const double* __restrict__ sigma,
                             const uint8_t* __restrict__ active, int update) {
    if ((int64_t)blockIdx.x >= dims[3]) return;
    const Block bk = cols[blockIdx.x];
    const int64_t c = bk.begin + (int64_t)threadIdx.x;
    if (c >= bk.end || !active[bk.sys]) return;
    const ResSys S = sys[bk.sys];
    if (update) S.x[c] = S.x[c] + sigma[bk.sys] * (double)S.d[c];
    else S.d[c] = 0.0f;
}

// x~ = P [x0; 0] over the extended system (n entries; x0 holds the caller's
// n_in unknowns, may be null: 0)
__global__ void k_batch_permute_in(int64_t n, int64_t n_in, const int32_t* __restrict__ p,
                                   const double* __restrict__ x0, double* __restrict__ xt) {
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

// x = (P^T x~)(1 : n_in)
__global__ void k_batch_permute_out(int64_t n, int64_t n_in, const int32_t* __restrict__ p,
                                    const double* __restrict__ xt, double* __restrict__ x) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int32_t pt = p[t];
        if (pt < n_in) x[pt] = xt[t];
    }
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// Tiles of the batched sweep for one system: rt/st (device) with per-group
// offsets rp/sp (device, G + 1 each).
struct TileView {
    const Tile* rt;
    const Tile* st;
    const int32_t* rp;
    const int32_t* sp;
};

template <class T> BatchSys<T> sys_view(obk_plan_s& P, const TileView& tv, uint32_t* bar, int team);
template <> BatchSys<float> sys_view<float>(obk_plan_s& P, const TileView& tv, uint32_t* bar, int team) {
    return BatchSys<float>{tv.rt, tv.st, tv.rp, tv.sp, P.rptr.get(), P.rcol.get(), P.rval32.get(), P.b32.get(),
                           P.rinv32.get(), P.sptr.get(), P.srow.get(), P.sval32.get(), P.tcol.get(), P.d32.get(),
                           P.w32.get(), P.ngroups, team, bar, (float)P.opts.omega};
}
template <> BatchSys<double> sys_view<double>(obk_plan_s& P, const TileView& tv, uint32_t* bar, int team) {
    return BatchSys<double>{tv.rt, tv.st, tv.rp, tv.sp, P.rptr.get(), P.rcol.get(), P.rval.get(), P.rf.get(),
                            P.rinv.get(), P.sptr.get(), P.srow.get(), P.sval.get(), P.tcol.get(), P.x.get(),
                            P.w.get(), P.ngroups, team, bar, P.opts.omega};
}

// Join consecutive tiles of one group while the result keeps at most
// kBatchQ * 256 segments and kBatchChunk entries (a tile already over the
// entry bound stays alone); appends to out, and the group offsets (relative
// to the first tile appended) to optr.
void merge_tiles(const std::vector<Tile>& in, const std::vector<int32_t>& ptr, int32_t G, std::vector<Tile>& out,
                 std::vector<int32_t>& optr) {
    const size_t base = out.size();
    optr.push_back(0);
    for (int32_t g = 0; g < G; g++) {
        int32_t k = ptr[g];
        while (k < ptr[g + 1]) {
            Tile m = in[k++];
            while (k < ptr[g + 1]) {
                const Tile& nx = in[k];
                const int64_t segs = (int64_t)nx.seg_end - m.seg_begin;
                const int64_t ents = nx.ent_end - m.ent_begin;
                if (segs > (int64_t)kBatchQ * kTileThreads || ents > kBatchChunk) break;
                m.seg_end = nx.seg_end;
                m.ent_end = nx.ent_end;
                k++;
            }
            out.push_back(m);
        }
        optr.push_back((int32_t)(out.size() - base));
    }
}

}  // namespace
}  // namespace obk

// ------------------------------------------------------------------ engine
struct obk_batch_s {
    std::vector<obk_plan_s*> plans;
    obk_batch_opts opts{};
    bool fp32 = false;
    int device = 0;
    int nwg = 0;
    std::vector<int32_t> team;               // team size per system
    obk::DevArray<uint8_t> enabled, active;  // per system
    obk::DevArray<double> relres, sigma;     // per system
    obk::DevArray<uint32_t> bars;            // 2 per system
    obk::DevArray<int32_t> task_ptr;
    obk::DevArray<char> tasks, sys_sweep, sys_res;
    obk::DevArray<char> rowblocks, colblocks, resblocks;
    obk::DevArray<char> mtiles_r, mtiles_s, mptr_r, mptr_s;   // merged sweep tiles
    obk::DevArray<int32_t> rowblk_ptr;
    obk::DevArray<double> psum, pmax;
    obk::DevArray<int> err;
    int64_t n_rowblocks = 0, n_colblocks = 0, n_resblocks = 0;
    // Launch grids of the residual, reduction, right-hand-side and column
    // kernels: at least the block counts of the current members, which the
    // kernels read from dims (blocks past them return at once), so that a
    // reset over new members keeps the captured graphs while the grids and
    // buffers are large enough.  Buffers and grids only grow.
    int64_t g_res = 0, g_sys = 0, g_rows = 0, g_cols = 0;
    obk::DevArray<int64_t> dims;         // {residual blocks, systems, row blocks, column blocks}
    int occ_fp32 = -1, occ = 0;          // occupancy of the sweep kernel, cached per precision
    std::vector<uint8_t> h_enabled;
    bool busy = false;
    obk::DevArray<uint64_t> trace;       // per workgroup start/end (OBK_TRACE=1)
    int sub = 4;                         // tiles in flight per workgroup
    // captured steps (one per tolerance and sweep count); OBK_BATCH_EAGER=1
    // launches eagerly
    struct StepGraph {
        double tol = 0;
        int sweeps = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<StepGraph> graphs;
    hipStream_t capture_stream = nullptr;
    bool use_graph = true;
    obk_batch_s() = default;
    obk_batch_s(const obk_batch_s&) = delete;
    obk_batch_s& operator=(const obk_batch_s&) = delete;
    void drop_graphs() {
        for (auto& g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        graphs.clear();
    }
    ~obk_batch_s() {
        drop_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }
};

namespace obk {
namespace {

// OBK_TRACE=1: per-workgroup wall-clock spans of the persistent launch and the
// event time of the launch, summarised on stderr after each step
bool trace_enabled() {
    const char* v = std::getenv("OBK_TRACE");
    return v && v[0] && v[0] != '0';
}

// Grow-only device storage: true when d had to be (re)allocated.  A first
// allocation is exact; a later one takes at least `headroom` times the old
// size, so that a stream of resets over similar member lists settles.
template <class T> bool reserve(DevArray<T>& d, size_t n, double headroom) {
    if (d.get() && d.count >= n) return false;
    size_t c = std::max<size_t>(n, 1);
    if (d.get()) c = std::max(c, (size_t)((double)d.count * headroom));
    d.alloc(c);
    return true;
}
bool grow_grid(int64_t& g, int64_t need, double headroom) {
    if (need <= g) return false;
    g = g == 0 ? need : std::max(need, (int64_t)((double)g * headroom));
    return true;
}
template <class T> void put(DevArray<char>& d, const std::vector<T>& h, hipStream_t s) {
    if (!h.empty()) OBK_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T> void put(DevArray<T>& d, const std::vector<T>& h, hipStream_t s) {
    if (!h.empty()) OBK_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

int sweep_occupancy(bool fp32, int sub) {
    int occ = 0;
    if (fp32) {
        if (sub == 1) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<float, 1>, kTileThreads, 0));
        if (sub == 2) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<float, 2>, 2 * kTileThreads, 0));
        if (sub == 4) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<float, 4>, 4 * kTileThreads, 0));
    } else {
        if (sub == 1) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<double, 1>, kTileThreads, 0));
        if (sub == 2) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<double, 2>, 2 * kTileThreads, 0));
        if (sub == 4) OBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_sweeps<double, 4>, 4 * kTileThreads, 0));
    }
    return occ;
}

// Team sizing and placement.  Work of a system per sweep ~ its entries in
// both phases; a system gets ceil(work / team_work) workgroups (at most
// max_team; team_work defaults to the average work per workgroup), all on one
// XCD (workgroup b runs on XCD b % 8).  A workgroup joins at most one team and
// runs that task first, so the members of a team start it together and never
// wait at a team barrier for a member still busy with another system.
// Single-workgroup systems then go to the least-loaded workgroups.
//
// The host arrays are formed first, then the device storage is grown where
// it is too small (which drops the captured step graphs: they hold its
// addresses and grids), then everything goes over in asynchronous copies on
// `st`, which is synchronised before returning.  The batch must be idle.
// Returns whether any storage or launch grid had to grow.
bool build_schedule(obk_batch_s& B, hipStream_t st, double headroom) {
    const int count = (int)B.plans.size();
    int dev = 0, cus = 256;
    OBK_HIP(hipGetDevice(&dev));
    OBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = B.opts.wgs_per_cu > 0 ? B.opts.wgs_per_cu : 2;
    // every workgroup of the persistent launch must be resident at once
    if (B.occ_fp32 != (int)B.fp32) {
        B.occ = sweep_occupancy(B.fp32, B.sub);
        B.occ_fp32 = (int)B.fp32;
    }
    per_cu = std::max(1, std::min(per_cu, B.occ));
    const int nxcd = 8;
    int nwg = std::max(nxcd, cus * per_cu);
    nwg -= nwg % nxcd;
    bool changed = nwg != B.nwg;
    B.nwg = nwg;
    std::vector<int64_t> work(count);
    int64_t total = 0;
    for (int s = 0; s < count; s++) {
        work[s] = 2 * B.plans[s]->nnz + 2 * B.plans[s]->m;
        total += work[s];
    }
    // default: a system gets about work / (average work per workgroup) members
    const int64_t team_work =
        B.opts.team_work > 0 ? B.opts.team_work : std::max<int64_t>(1, (total + nwg - 1) / nwg);
    const int max_team = std::max(1, std::min(B.opts.max_team > 0 ? B.opts.max_team : 16, nwg / nxcd));
    B.team.assign(count, 1);
    std::vector<std::vector<TeamTask>> per_wg(nwg);
    std::vector<int64_t> load(nwg, 0);
    std::vector<uint8_t> teamed(nwg, 0);     // a workgroup joins at most one team
    // large systems first
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    const int slots = nwg / nxcd;
    for (int s : order) {
        int k = (int)std::min<int64_t>(max_team, std::max<int64_t>(1, (work[s] + team_work - 1) / team_work));
        std::vector<int> pick;
        if (k > 1) {
            // the XCD with the most free slots (ties: least loaded); the team
            // shrinks to the free slots there
            int best_x = -1, best_free = 0;
            int64_t best_l = INT64_MAX;
            for (int x = 0; x < nxcd; x++) {
                int nfree = 0;
                int64_t l = 0;
                for (int j = 0; j < slots; j++) {
                    const int b = x + nxcd * j;
                    if (!teamed[b]) { nfree++; l += load[b]; }
                }
                if (nfree > best_free || (nfree == best_free && nfree > 0 && l < best_l)) {
                    best_free = nfree; best_l = l; best_x = x;
                }
            }
            k = std::min(k, best_free);
            if (k > 1) {
                std::vector<int> ids;
                for (int j = 0; j < slots; j++) {
                    const int b = best_x + nxcd * j;
                    if (!teamed[b]) ids.push_back(b);
                }
                std::partial_sort(ids.begin(), ids.begin() + k, ids.end(),
                                  [&](int a, int b) { return load[a] < load[b]; });
                pick.assign(ids.begin(), ids.begin() + k);
            }
        }
        if (k > 1) {
            B.team[s] = k;
            for (int j = 0; j < k; j++) {
                per_wg[pick[j]].push_back(TeamTask{s, j});
                teamed[pick[j]] = 1;
                load[pick[j]] += (work[s] + k - 1) / k;
            }
        } else {
            int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            per_wg[best].push_back(TeamTask{s, 0});
            load[best] += work[s];
        }
    }
    std::vector<int32_t> tptr(nwg + 1, 0);
    std::vector<TeamTask> flat;
    for (int b = 0; b < nwg; b++) {
        // one global order for all workgroups: larger teams first, then system id
        std::sort(per_wg[b].begin(), per_wg[b].end(), [&](const TeamTask& a, const TeamTask& c) {
            if (B.team[a.sys] != B.team[c.sys]) return B.team[a.sys] > B.team[c.sys];
            return a.sys < c.sys;
        });
        for (auto& t : per_wg[b]) flat.push_back(t);
        tptr[b + 1] = (int32_t)flat.size();
    }
    // merged tiles of every system, R then S, in one array each
    std::vector<Tile> mr, ms;
    std::vector<int32_t> mrp, msp;
    std::vector<size_t> rbase(count), sbase(count), rpbase(count), spbase(count);
    for (int s = 0; s < count; s++) {
        obk_plan_s& P = *B.plans[s];
        rbase[s] = mr.size(); rpbase[s] = mrp.size();
        merge_tiles(P.h_rtiles, P.h_rtile_ptr, P.ngroups, mr, mrp);
        sbase[s] = ms.size(); spbase[s] = msp.size();
        merge_tiles(P.h_stiles, P.h_stile_ptr, P.ngroups, ms, msp);
    }
    // residual, right-hand-side and column blocks
    std::vector<Block> rows, cols, res;
    std::vector<int32_t> rptr(count + 1, 0);
    for (int s = 0; s < count; s++) {
        obk_plan_s& P = *B.plans[s];
        for (int64_t a = 0; a < std::max<int64_t>(P.m, 1); a += 256)
            rows.push_back(Block{s, (int32_t)a, (int32_t)std::min<int64_t>(a + 256, P.m)});
        // residual blocks: the system's R tiles in plan order (all groups)
        for (size_t k = 0; k < P.h_rtiles.size(); k++) res.push_back(Block{s, (int32_t)k, 0});
        rptr[s + 1] = (int32_t)res.size();
        for (int64_t c = 0; c < P.n; c += 256)
            cols.push_back(Block{s, (int32_t)c, (int32_t)std::min<int64_t>(c + 256, P.n)});
    }
    B.n_rowblocks = (int64_t)rows.size();
    B.n_colblocks = (int64_t)cols.size();
    B.n_resblocks = (int64_t)res.size();
    changed |= grow_grid(B.g_res, B.n_resblocks, headroom);
    changed |= grow_grid(B.g_sys, count, headroom);
    changed |= grow_grid(B.g_rows, B.n_rowblocks, headroom);
    changed |= grow_grid(B.g_cols, B.n_colblocks, headroom);
    // device storage (grown where too small)
    const size_t sysb = B.fp32 ? sizeof(BatchSys<float>) : sizeof(BatchSys<double>);
    changed |= reserve(B.task_ptr, (size_t)nwg + 1, headroom);
    changed |= reserve(B.tasks, flat.size() * sizeof(TeamTask), headroom);
    changed |= reserve(B.bars, 2 * (size_t)std::max(count, 1), headroom);
    changed |= reserve(B.mtiles_r, mr.size() * sizeof(Tile), headroom);
    changed |= reserve(B.mtiles_s, ms.size() * sizeof(Tile), headroom);
    changed |= reserve(B.mptr_r, mrp.size() * sizeof(int32_t), headroom);
    changed |= reserve(B.mptr_s, msp.size() * sizeof(int32_t), headroom);
    changed |= reserve(B.sys_sweep, (size_t)count * sysb, headroom);
    changed |= reserve(B.sys_res, (size_t)count * sizeof(ResSys), headroom);
    changed |= reserve(B.rowblocks, rows.size() * sizeof(Block), headroom);
    changed |= reserve(B.colblocks, cols.size() * sizeof(Block), headroom);
    changed |= reserve(B.resblocks, res.size() * sizeof(Block), headroom);
    changed |= reserve(B.rowblk_ptr, (size_t)count + 1, headroom);
    changed |= reserve(B.psum, (size_t)B.g_res, headroom);
    changed |= reserve(B.pmax, (size_t)B.g_res, headroom);
    changed |= reserve(B.relres, (size_t)B.g_sys, headroom);
    changed |= reserve(B.sigma, (size_t)B.g_sys, headroom);
    changed |= reserve(B.active, (size_t)B.g_sys, headroom);
    changed |= reserve(B.enabled, (size_t)B.g_sys, headroom);
    changed |= reserve(B.err, 2, headroom);
    changed |= reserve(B.dims, 4, headroom);
    if (changed) B.drop_graphs();
    // per-system views (device addresses of the merged tiles and barriers)
    auto view = [&](int s) {
        return TileView{reinterpret_cast<const Tile*>(B.mtiles_r.get()) + rbase[s],
                        reinterpret_cast<const Tile*>(B.mtiles_s.get()) + sbase[s],
                        reinterpret_cast<const int32_t*>(B.mptr_r.get()) + rpbase[s],
                        reinterpret_cast<const int32_t*>(B.mptr_s.get()) + spbase[s]};
    };
    std::vector<BatchSys<float>> v32;
    std::vector<BatchSys<double>> v64;
    for (int s = 0; s < count; s++) {
        if (B.fp32) v32.push_back(sys_view<float>(*B.plans[s], view(s), B.bars.get() + 2 * s, B.team[s]));
        else v64.push_back(sys_view<double>(*B.plans[s], view(s), B.bars.get() + 2 * s, B.team[s]));
    }
    std::vector<ResSys> rs;
    for (int s = 0; s < count; s++) {
        obk_plan_s& P = *B.plans[s];
        rs.push_back(ResSys{P.rtiles.get(), P.rptr.get(), P.rcol.get(), P.rval.get(), P.rf.get(), P.x.get(),
                            P.r64.get(), P.b32.get(), P.d32.get(), P.fnorm2, P.zero_rows_f2, P.zero_rows_fmax});
    }
    const std::vector<int64_t> dims{B.n_resblocks, count, B.n_rowblocks, B.n_colblocks};
    B.h_enabled.assign(count, 1);
    put(B.task_ptr, tptr, st);
    put(B.tasks, flat, st);
    put(B.mtiles_r, mr, st);
    put(B.mtiles_s, ms, st);
    put(B.mptr_r, mrp, st);
    put(B.mptr_s, msp, st);
    if (B.fp32) put(B.sys_sweep, v32, st);
    else put(B.sys_sweep, v64, st);
    put(B.sys_res, rs, st);
    put(B.rowblocks, rows, st);
    put(B.colblocks, cols, st);
    put(B.resblocks, res, st);
    put(B.rowblk_ptr, rptr, st);
    put(B.enabled, B.h_enabled, st);
    put(B.dims, dims, st);
    // team barriers start from zero; [0]: a team barrier timed out, [1]: a
    // residual was not finite (per system in relres)
    OBK_HIP(hipMemsetAsync(B.bars.get(), 0, 2 * sizeof(uint32_t) * std::max(count, 1), st));
    OBK_HIP(hipMemsetAsync(B.err.get(), 0, 2 * sizeof(int), st));
    if (trace_enabled()) {
        (void)reserve(B.trace, 2 * (size_t)B.nwg, headroom);     // eager launches only: no graph holds it
        OBK_HIP(hipMemsetAsync(B.trace.get(), 0, 2 * sizeof(uint64_t) * B.nwg, st));
    }
    // the host arrays above must outlive the copies
    OBK_HIP(hipStreamSynchronize(st));
    return changed;
}

}  // namespace

namespace {

hipEvent_t g_ev[2] = {nullptr, nullptr};

void ev_record(obk_batch_s& B, int which, hipStream_t s) {
    if (!B.trace.get()) return;
    if (!g_ev[which]) OBK_HIP(hipEventCreate(&g_ev[which]));
    OBK_HIP(hipEventRecord(g_ev[which], s));
}

void trace_report(obk_batch_s& B) {
    std::vector<uint64_t> t(2 * (size_t)B.nwg);
    OBK_HIP(hipMemcpy(t.data(), B.trace.get(), t.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
    int rate_khz = 100000;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, B.device);
    const double us = 1e3 / (double)rate_khz;
    uint64_t t0 = UINT64_MAX, t1 = 0;
    std::vector<double> dur;
    for (int b = 0; b < B.nwg; b++) {
        t0 = std::min(t0, t[2 * b]);
        t1 = std::max(t1, t[2 * b + 1]);
        dur.push_back((double)(t[2 * b + 1] - t[2 * b]) * us);
    }
    std::vector<double> sd = dur;
    std::sort(sd.begin(), sd.end());
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g_ev[0], g_ev[1]);
    std::fprintf(stderr, "[obk-trace] batched launch: %.1f us (event), span %.1f us, per-WG us: min %.1f "
                         "median %.1f p90 %.1f max %.1f over %d WGs\n",
                 ms * 1e3, (double)(t1 - t0) * us, sd.front(), sd[sd.size() / 2], sd[sd.size() * 9 / 10],
                 sd.back(), B.nwg);
}
}  // namespace

template <class T>
void launch_sweeps(obk_batch_s& B, int sweeps, hipStream_t s) {
    const BatchSys<T>* sys = (const BatchSys<T>*)B.sys_sweep.get();
    const TeamTask* tasks = (const TeamTask*)B.tasks.get();
    if (B.sub == 1)
        k_batch_sweeps<T, 1><<<B.nwg, kTileThreads, 0, s>>>(sys, B.task_ptr.get(), tasks, B.active.get(), sweeps,
                                                             B.err.get(), B.trace.get());
    else if (B.sub == 2)
        k_batch_sweeps<T, 2><<<B.nwg, 2 * kTileThreads, 0, s>>>(sys, B.task_ptr.get(), tasks, B.active.get(),
                                                                 sweeps, B.err.get(), B.trace.get());
    else
        k_batch_sweeps<T, 4><<<B.nwg, 4 * kTileThreads, 0, s>>>(sys, B.task_ptr.get(), tasks, B.active.get(),
                                                                 sweeps, B.err.get(), B.trace.get());
    OBK_HIP(hipGetLastError());
}

// The checks every member list passes (obk_batch_create and obk_batch_reset).
static void check_members(const obk_batch_s& B, const obk_plan_t* plans, int count) {
    for (int s = 0; s < count; s++) {
        if (!plans[s]) fail(OBK_E_ARG, "NULL plan in batch");
        if (plans[s]->device != B.device) fail(OBK_E_ARG, "plans of a batch must live on the current device");
        if (plans[s]->block_form()) fail(OBK_E_ARG, "plans in block form cannot be batched");
        if (plans[s]->cplx) fail(OBK_E_ARG, "complex plans cannot be batched");
        if (s > 0 && plans[s]->opts.precision != plans[0]->opts.precision)
            fail(OBK_E_ARG, "plans of a batch must share one precision");
    }
    std::vector<const obk_plan_s*> sorted(plans, plans + count);
    std::sort(sorted.begin(), sorted.end(), std::less<const obk_plan_s*>());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        fail(OBK_E_ARG, "a plan appears twice in a batch");
}

void batch_create(obk_batch_s& B, const obk_plan_t* plans, int count, const obk_batch_opts* opts) {
    if (opts) B.opts = *opts;
    B.sub = B.opts.tiles_per_wg > 0 ? B.opts.tiles_per_wg : 4;
    if (B.sub != 1 && B.sub != 2 && B.sub != 4) fail(OBK_E_ARG, "tiles_per_wg must be 1, 2 or 4");
    OBK_HIP(hipGetDevice(&B.device));
    check_members(B, plans, count);
    B.plans.assign(plans, plans + count);
    B.fp32 = count > 0 && plans[0]->opts.precision == OBK_FP32_IR;
    {
        const char* e = std::getenv("OBK_BATCH_EAGER");
        B.use_graph = !(e && e[0] && e[0] != '0');
    }
    build_schedule(B, nullptr, 1.0);
    log_line(2, "batch create systems=%d workgroups=%d %s", count, B.nwg, B.fp32 ? "fp32-ir" : "fp64");
}

// A new member list for an existing batch object (continuous batching): the
// schedule is formed again, the device storage and the captured step graphs
// are kept unless the new members outgrow them.  Members keep their iterates
// (they live in the plans); every member is enabled afterwards.
void batch_reset(obk_batch_s& B, const obk_plan_t* plans, int count, hipStream_t s) {
    int dev = 0;
    OBK_HIP(hipGetDevice(&dev));
    if (dev != B.device) fail(OBK_E_ARG, "a batch must be reset on the device it was created on");
    check_members(B, plans, count);
    const bool fp32 = count > 0 ? plans[0]->opts.precision == OBK_FP32_IR : B.fp32;
    if (fp32 != B.fp32) {
        // another kernel instantiation: the captured graphs no longer apply
        B.drop_graphs();
        B.fp32 = fp32;
    }
    B.plans.assign(plans, plans + count);
    try {
        const bool grown = build_schedule(B, s, 1.5);
        log_line(2, "batch reset systems=%d workgroups=%d storage %s", count, B.nwg,
                 grown ? "grown (step graphs captured again)" : "kept");
    } catch (...) {
        // a failed reset leaves an empty batch, never one whose descriptors
        // and member list disagree
        B.plans.clear();
        B.h_enabled.clear();
        B.drop_graphs();
        throw;
    }
}

// x~ = P x0 for one system (x0 NULL: 0)
static void start_one(obk_plan_s& P, const double* x0, hipStream_t s) {
    const double* src = x0;
    DevArray<double> tmp;
    if (src && !P.input_on_device) {
        tmp.alloc(P.n_in);
        OBK_HIP(hipMemcpyAsync(tmp.get(), src, P.n_in * sizeof(double), hipMemcpyHostToDevice, s));
        src = tmp.get();
    }
    k_batch_permute_in<<<nblk(P.n), 256, 0, s>>>(P.n, P.n_in, P.perm.get(), src, P.x.get());
    OBK_HIP(hipGetLastError());
    if (tmp.get()) OBK_HIP(hipStreamSynchronize(s));
}

// x~ = P x0 for every system (x0 entries may be NULL: 0)
void batch_begin(obk_batch_s& B, const double* const* x0, hipStream_t s) {
    for (size_t i = 0; i < B.plans.size(); i++) start_one(*B.plans[i], x0 ? x0[i] : nullptr, s);
    B.h_enabled.assign(B.plans.size(), 1);
    if (!B.plans.empty())
        OBK_HIP(hipMemcpyAsync(B.enabled.get(), B.h_enabled.data(), B.plans.size(), hipMemcpyHostToDevice, s));
    OBK_HIP(hipStreamSynchronize(s));
}

// One step for all enabled systems; relres/active (host, may be NULL) receive
// each system's relative residual at the start of the step and whether the
// step advanced it.
// The kernels of one step: residual, reduction (relative residual, sigma and
// the active flags), right-hand side and correction reset (FP32 refinement),
// the persistent sweep launch, and the update.
static int step_sweeps(const obk_batch_s& B) {
    return B.fp32 ? std::max(1, B.plans[0]->opts.inner_sweeps) : std::max(1, B.plans[0]->opts.check_every);
}

static void enqueue_step(obk_batch_s& B, double tol, hipStream_t s) {
    const int64_t* dims = B.dims.get();
    const ResSys* rs = (const ResSys*)B.sys_res.get();
    if (B.g_res)
        k_batch_resid<<<(unsigned)B.g_res, kTileThreads, 0, s>>>(dims, rs, (const Block*)B.resblocks.get(),
                                                                 B.psum.get(), B.pmax.get(), B.err.get() + 1);
    k_batch_reduce<<<(unsigned)B.g_sys, 256, 0, s>>>(dims, rs, B.rowblk_ptr.get(), B.psum.get(), B.pmax.get(),
                                                     tol > 0 ? tol : -1.0, B.enabled.get(), B.relres.get(),
                                                     B.sigma.get(), B.active.get());
    OBK_HIP(hipGetLastError());
    if (B.fp32) {
        k_batch_rhs<<<(unsigned)B.g_rows, 256, 0, s>>>(dims, rs, (const Block*)B.rowblocks.get(), B.sigma.get(),
                                                       B.active.get());
        if (B.g_cols)
            k_batch_cols<<<(unsigned)B.g_cols, 256, 0, s>>>(dims, rs, (const Block*)B.colblocks.get(),
                                                            B.sigma.get(), B.active.get(), 0);
        ev_record(B, 0, s);
        launch_sweeps<float>(B, step_sweeps(B), s);
        ev_record(B, 1, s);
        if (B.g_cols)
            k_batch_cols<<<(unsigned)B.g_cols, 256, 0, s>>>(dims, rs, (const Block*)B.colblocks.get(),
                                                            B.sigma.get(), B.active.get(), 1);
    } else {
        ev_record(B, 0, s);
        launch_sweeps<double>(B, step_sweeps(B), s);
        ev_record(B, 1, s);
    }
    OBK_HIP(hipGetLastError());
}

// The step's kernels captured once per tolerance and sweep count into a graph
// on the batch's own capture stream and replayed afterwards (no memset nodes:
// the flags the kernels read are written by kernels or by host copies and
// fills outside the graph).  The graph holds the batch's device addresses and
// grids, so it survives a reset until the storage has to grow.
static hipGraphExec_t step_graph(obk_batch_s& B, double tol) {
    const int sweeps = step_sweeps(B);
    for (auto& g : B.graphs)
        if (g.tol == tol && g.sweeps == sweeps && g.exec) return g.exec;
    if (!B.capture_stream) OBK_HIP(hipStreamCreateWithFlags(&B.capture_stream, hipStreamNonBlocking));
    obk_batch_s::StepGraph sg;
    sg.tol = tol;
    sg.sweeps = sweeps;
    OBK_HIP(hipStreamBeginCapture(B.capture_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_step(B, tol, B.capture_stream);
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(B.capture_stream, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    OBK_HIP(hipStreamEndCapture(B.capture_stream, &sg.graph));
    OBK_HIP(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
    B.graphs.push_back(sg);
    return sg.exec;
}

void batch_step(obk_batch_s& B, double tol, double* relres_out, int32_t* active_out, hipStream_t s) {
    const int count = (int)B.plans.size();
    if (count == 0) return;
    if (B.use_graph && !B.trace.get())
        OBK_HIP(hipGraphLaunch(step_graph(B, tol), s));
    else
        enqueue_step(B, tol, s);
    OBK_HIP(hipGetLastError());
    std::vector<double> rr(count);
    std::vector<uint8_t> act(count);
    int herr = 0;
    OBK_HIP(hipMemcpyAsync(rr.data(), B.relres.get(), count * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipMemcpyAsync(act.data(), B.active.get(), count, hipMemcpyDeviceToHost, s));
    OBK_HIP(hipMemcpyAsync(&herr, B.err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
    if (herr & 1) fail(OBK_E_HIP, "a team barrier of the batched sweep timed out");
    if (B.trace.get()) trace_report(B);
    if (log_level() >= 3) {
        int act_n = 0;
        for (int i = 0; i < count; i++) act_n += act[i] ? 1 : 0;
        log_line(3, "batch step systems=%d advanced=%d", count, act_n);
    }
    for (int i = 0; i < count; i++) {
        if (relres_out) relres_out[i] = rr[i];
        if (active_out) active_out[i] = act[i];
    }
}

void batch_result(obk_batch_s& B, int index, double* x, hipStream_t s) {
    obk_plan_s& P = *B.plans[index];
    DevArray<double> tmp;
    double* dst = x;
    if (!P.input_on_device) { tmp.alloc(P.n_in); dst = tmp.get(); }
    k_batch_permute_out<<<nblk(P.n), 256, 0, s>>>(P.n, P.n_in, P.perm.get(), P.x.get(), dst);
    OBK_HIP(hipGetLastError());
    if (!P.input_on_device) OBK_HIP(hipMemcpyAsync(x, tmp.get(), P.n_in * sizeof(double), hipMemcpyDeviceToHost, s));
    OBK_HIP(hipStreamSynchronize(s));
}

// Start one system (continuous batching); the others are untouched.
void batch_start(obk_batch_s& B, int index, const double* x0, hipStream_t s) {
    start_one(*B.plans[index], x0, s);
    B.h_enabled[index] = 1;
    OBK_HIP(hipMemcpyAsync(B.enabled.get() + index, &B.h_enabled[index], 1, hipMemcpyHostToDevice, s));
    OBK_HIP(hipStreamSynchronize(s));
}

// Disable systems from further steps (e.g. after they converged).
void batch_set_enabled(obk_batch_s& B, const int32_t* enabled, hipStream_t s) {
    for (size_t i = 0; i < B.plans.size(); i++) B.h_enabled[i] = enabled[i] ? 1 : 0;
    OBK_HIP(hipMemcpyAsync(B.enabled.get(), B.h_enabled.data(), B.plans.size(), hipMemcpyHostToDevice, s));
    OBK_HIP(hipStreamSynchronize(s));
}

}  // namespace obk

obk_batch_s* obk_batch_new() { return new obk_batch_s(); }
void obk_batch_delete(obk_batch_s* b) { delete b; }
bool* obk_batch_busy(obk_batch_s* b) { return &b->busy; }
int obk_batch_count(obk_batch_s* b) { return (int)b->plans.size(); }
