// Host parts of the plan: the two inherently sequential graph passes (reverse
// Cuthill-McKee, first-fit grouping), the sweep tile schedule, errors and
// device-memory bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "obk_internal.h"

namespace obk {

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

// ----------------------------------------------------------------- logging
int log_level() {
    static const int level = [] {
        const char* v = std::getenv("OBK_LOG");
        if (!v || !v[0]) return 0;
        const int l = std::atoi(v);
        return l < 0 ? 0 : (l > 3 ? 3 : l);
    }();
    return level;
}

void log_line(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[obk] %s\n", buf);
    std::fflush(stderr);
}

void fail(obk_status code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        obk_status code = (e == hipErrorOutOfMemory) ? OBK_E_NOMEM : OBK_E_HIP;
        fail(code, std::string(what) + ": " + hipGetErrorString(e));
    }
}

namespace {
thread_local hipStream_t g_alloc_stream = nullptr;
thread_local bool g_alloc_scoped = false;
thread_local void* (*g_user_alloc)(size_t, void*) = nullptr;
thread_local void (*g_user_dealloc)(void*, void*) = nullptr;
thread_local void* g_user_ctx = nullptr;
thread_local hipStream_t g_user_stream = nullptr;
}  // namespace

UserAllocScope::UserAllocScope(void* (*alloc)(size_t, void*), void (*dealloc)(void*, void*), void* ctx,
                               hipStream_t s)
    : prev_alloc(g_user_alloc), prev_dealloc(g_user_dealloc), prev_ctx(g_user_ctx), prev_stream(g_user_stream) {
    if (alloc) {
        g_user_alloc = alloc;
        g_user_dealloc = dealloc;
        g_user_ctx = ctx;
        g_user_stream = s;
    }
}

UserAllocScope::~UserAllocScope() {
    g_user_alloc = prev_alloc;
    g_user_dealloc = prev_dealloc;
    g_user_ctx = prev_ctx;
    g_user_stream = prev_stream;
}

namespace {
// Buffers released inside the active AllocScope, by size class.
struct ScopeCache {
    hipStream_t stream = nullptr;
    int device = 0;
    std::multimap<size_t, void*> blocks;
};
thread_local ScopeCache* g_scope_cache = nullptr;

// Pool blocks that no queued work uses any more (the stream of their last use
// was synchronised), by (device, size class), shared by every thread: a
// scope takes from here before it asks the pool and leaves its blocks here
// when it ends.  At most kIdleCap bytes are kept; beyond that blocks go back
// to the pool.
constexpr size_t kIdleCap = (size_t)1 << 30;
struct IdleBlocks {
    std::mutex mu;
    std::multimap<std::pair<int, size_t>, void*> blocks;
    size_t bytes = 0;
};
IdleBlocks& idle_blocks() {
    static IdleBlocks* b = new IdleBlocks();   // never destroyed: kept blocks may outlive static destruction
    return *b;
}

// Size classes: multiples of 256 B up to 4 KiB, then four per power of two
// (at most 25% over the request).
size_t size_class(size_t b) {
    if (b <= 4096) return (b + 255) & ~(size_t)255;
    const size_t p = (size_t)1 << (63 - __builtin_clzll((unsigned long long)b));
    const size_t step = p / 4;
    return (b + step - 1) / step * step;
}
}  // namespace

AllocScope::AllocScope(hipStream_t s)
    : prev_stream(g_alloc_stream), prev_on(g_alloc_scoped), prev_cache(g_scope_cache) {
    g_alloc_stream = s;
    g_alloc_scoped = true;
    // a scope nested on the same stream shares the outer cache; on another
    // stream it keeps none (a buffer of the outer scope may still be in use there)
    if (!g_scope_cache || g_scope_cache->stream != s) {
        g_scope_cache = (prev_cache && static_cast<ScopeCache*>(prev_cache)->stream != s) ? nullptr
                                                                                         : new ScopeCache();
        if (g_scope_cache) {
            g_scope_cache->stream = s;
            if (hipGetDevice(&g_scope_cache->device) != hipSuccess) (void)hipGetLastError();
        }
    }
}

AllocScope::~AllocScope() {
    if (g_scope_cache && g_scope_cache != prev_cache) {
        ScopeCache* c = g_scope_cache;
        if (!c->blocks.empty()) {
            // once the scope's stream is idle its blocks are free of any queued
            // use and may serve any later scope, on any stream of the device
            const bool idle = hipStreamSynchronize(c->stream) == hipSuccess;
            if (!idle) (void)hipGetLastError();
            IdleBlocks& ib = idle_blocks();
            std::lock_guard<std::mutex> lk(ib.mu);
            for (auto& kv : c->blocks) {
                if (idle && ib.bytes + kv.first <= kIdleCap) {
                    ib.blocks.emplace(std::make_pair(c->device, kv.first), kv.second);
                    ib.bytes += kv.first;
                } else {
                    (void)hipFreeAsync(kv.second, c->stream);
                }
            }
        }
        delete c;
    }
    g_scope_cache = static_cast<ScopeCache*>(prev_cache);
    g_alloc_stream = prev_stream;
    g_alloc_scoped = prev_on;
}

bool alloc_scoped() { return g_alloc_scoped; }

void sync_for_free(hipStream_t s) {
    if (!g_alloc_scoped) OBK_HIP(hipStreamSynchronize(s));
}

namespace {
struct PinnedStage {
    void* p = nullptr;
    size_t cap = 0;
    ~PinnedStage() { if (p) (void)hipHostFree(p); }
};
thread_local PinnedStage g_stage;
}  // namespace

void* pinned_stage(size_t bytes) {
    if (bytes > g_stage.cap) {
        if (g_stage.p) (void)hipHostFree(g_stage.p);
        g_stage.p = nullptr;
        g_stage.cap = 0;
        const size_t want = std::max<size_t>(bytes, (size_t)1 << 20);
        OBK_HIP(hipHostMalloc(&g_stage.p, want, hipHostMallocDefault));
        g_stage.cap = want;
    }
    return g_stage.p;
}

namespace {
// Two events per thread and device mark when each half of the staging buffer
// is free again (created once and never destroyed: two events per thread).
struct StageEvents {
    int device = -1;
    hipEvent_t e[2] = {nullptr, nullptr};
};
thread_local StageEvents g_stage_ev;
hipEvent_t stage_event(int k) {
    int dev = 0;
    OBK_HIP(hipGetDevice(&dev));
    if (g_stage_ev.device != dev) {
        g_stage_ev = StageEvents{};
        g_stage_ev.device = dev;
    }
    if (!g_stage_ev.e[k]) OBK_HIP(hipEventCreateWithFlags(&g_stage_ev.e[k], hipEventDisableTiming));
    return g_stage_ev.e[k];
}
constexpr size_t kStageChunk = (size_t)8 << 20;
}  // namespace

void stage_h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if (bytes <= kStageChunk) {
        void* st = pinned_stage(bytes);
        std::memcpy(st, h, bytes);
        OBK_HIP(hipMemcpyAsync(d, st, bytes, hipMemcpyHostToDevice, s));
        OBK_HIP(hipStreamSynchronize(s));     // the stage is reused by the next copy
        return;
    }
    char* st = static_cast<char*>(pinned_stage(2 * kStageChunk));
    bool busy[2] = {false, false};
    int k = 0;
    for (size_t off = 0; off < bytes; off += kStageChunk, k ^= 1) {
        const size_t len = std::min(kStageChunk, bytes - off);
        if (busy[k]) OBK_HIP(hipEventSynchronize(stage_event(k)));      // half k's last copy is done
        std::memcpy(st + k * kStageChunk, static_cast<const char*>(h) + off, len);
        OBK_HIP(hipMemcpyAsync(static_cast<char*>(d) + off, st + k * kStageChunk, len, hipMemcpyHostToDevice, s));
        OBK_HIP(hipEventRecord(stage_event(k), s));
        busy[k] = true;
    }
    OBK_HIP(hipStreamSynchronize(s));
}

void stage_d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
    if (!bytes) {
        OBK_HIP(hipStreamSynchronize(s));
        return;
    }
    if (bytes <= kStageChunk) {
        void* st = pinned_stage(bytes);
        OBK_HIP(hipMemcpyAsync(st, d, bytes, hipMemcpyDeviceToHost, s));
        OBK_HIP(hipStreamSynchronize(s));
        std::memcpy(h, st, bytes);
        return;
    }
    char* st = static_cast<char*>(pinned_stage(2 * kStageChunk));
    size_t pend_off[2] = {0, 0}, pend_len[2] = {0, 0};
    int k = 0;
    auto drain = [&](int q) {
        if (!pend_len[q]) return;
        OBK_HIP(hipEventSynchronize(stage_event(q)));
        std::memcpy(static_cast<char*>(h) + pend_off[q], st + q * kStageChunk, pend_len[q]);
        pend_len[q] = 0;
    };
    for (size_t off = 0; off < bytes; off += kStageChunk, k ^= 1) {
        const size_t len = std::min(kStageChunk, bytes - off);
        drain(k);                             // half k holds an earlier chunk still to copy out
        OBK_HIP(hipMemcpyAsync(st + k * kStageChunk, static_cast<const char*>(d) + off, len, hipMemcpyDeviceToHost, s));
        OBK_HIP(hipEventRecord(stage_event(k), s));
        pend_off[k] = off;
        pend_len[k] = len;
    }
    drain(k);                                 // the older of the two in flight first
    drain(k ^ 1);
    OBK_HIP(hipStreamSynchronize(s));
}

void DevMem::alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    void* p = nullptr;
    if (g_user_alloc) {
        p = g_user_alloc(b, g_user_ctx);
        if (!p) fail(OBK_E_NOMEM, "the caller's allocator returned NULL for " + std::to_string(b) + " bytes");
        ptr = p;
        bytes = b;
        pooled = false;
        dealloc = g_user_dealloc;
        ctx = g_user_ctx;
        return;
    }
    const bool use_pool = g_alloc_scoped;
    size_t want = b;
    if (use_pool && g_scope_cache) {
        want = size_class(b);
        void* hit = nullptr;
        auto it = g_scope_cache->blocks.find(want);
        if (it != g_scope_cache->blocks.end()) {
            hit = it->second;
            g_scope_cache->blocks.erase(it);
        } else {
            IdleBlocks& ib = idle_blocks();
            std::lock_guard<std::mutex> lk(ib.mu);
            auto jt = ib.blocks.find(std::make_pair(g_scope_cache->device, want));
            if (jt != ib.blocks.end()) {
                hit = jt->second;
                ib.blocks.erase(jt);
                ib.bytes -= want;
            }
        }
        if (hit) {
            ptr = hit;
            bytes = b;
            cap = want;
            pooled = true;
            return;
        }
    }
    hipError_t e = use_pool ? hipMallocAsync(&p, want, g_alloc_stream) : hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(OBK_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    ptr = p;
    bytes = b;
    cap = (use_pool && g_scope_cache) ? want : 0;
    pooled = use_pool;
}

void DevMem::release() {
    if (ptr && dealloc) {
        // a temporary released during a call: no queued work may still use it
        if (g_user_alloc) (void)hipStreamSynchronize(g_user_stream);
        dealloc(ptr, ctx);
    } else if (ptr) {
        if (pooled && cap && g_alloc_scoped && g_scope_cache && g_scope_cache->stream == g_alloc_stream)
            g_scope_cache->blocks.emplace(cap, ptr);       // kept for the scope's next request of its class
        else if (pooled)
            (void)hipFreeAsync(ptr, g_alloc_scoped ? g_alloc_stream : nullptr);
        else
            (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
    cap = 0;
    pooled = false;
    dealloc = nullptr;
    ctx = nullptr;
}

// --------------------------------------------------------------------- RCM
// Section 3.2 names reverse Cuthill-McKee without a tie-break; this file
// fixes one (stated in obk.h and below) so that the order is unique.
void host_cm_resume(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* cm, uint8_t* seen, int64_t head,
                    int64_t tail) {
    if (n <= 0) return;
    // Degrees once; neighbours are then ordered by the 64-bit key
    // (degree << 32 | index), which is the (degree, index) order.
    std::vector<uint32_t> deg(n);
    uint32_t maxdeg = 0;
    for (int64_t v = 0; v < n; v++) {
        deg[v] = (uint32_t)(gptr[v + 1] - gptr[v]);
        maxdeg = std::max(maxdeg, deg[v]);
    }
    // Vertices ordered by (degree, index): counting sort on the degree keeps
    // ascending index within a degree.
    std::vector<int64_t> bucket((size_t)maxdeg + 2, 0);
    for (int64_t v = 0; v < n; v++) bucket[deg[v] + 1]++;
    for (uint32_t d = 0; d <= maxdeg; d++) bucket[d + 1] += bucket[d];
    std::vector<int32_t> by_degree(n);
    for (int64_t v = 0; v < n; v++) by_degree[bucket[deg[v]]++] = (int32_t)v;

    // cm is the Cuthill-McKee sequence and doubles as the FIFO: [head, tail)
    // are the vertices appended but not yet expanded
    std::vector<uint64_t> fresh;
    fresh.reserve(256);
    int64_t next_start = 0;
    while (tail < n) {
        if (head == tail) {               // new component
            while (seen[by_degree[next_start]]) next_start++;
            int32_t s = by_degree[next_start];
            seen[s] = 1;
            cm[tail++] = s;
        }
        int32_t v = cm[head++];
        // the queue ahead is known: start fetching the adjacency of a vertex
        // a few places further on while this one is expanded
        if (head + 4 < tail) {
            const int32_t ahead = cm[head + 4];
            __builtin_prefetch(gadj + gptr[ahead]);
            __builtin_prefetch(&gptr[cm[head + 8 < tail ? head + 8 : head + 4]]);
        }
        fresh.clear();
        for (int64_t k = gptr[v]; k < gptr[v + 1]; k++) {
            int32_t u = gadj[k];
            if (!seen[u]) {
                seen[u] = 1;
                fresh.push_back(((uint64_t)deg[u] << 32) | (uint32_t)u);
            }
        }
        if (fresh.size() <= 32) {          // short lists: insertion sort
            for (size_t a = 1; a < fresh.size(); a++) {
                uint64_t key = fresh[a];
                size_t b = a;
                while (b > 0 && key < fresh[b - 1]) { fresh[b] = fresh[b - 1]; b--; }
                fresh[b] = key;
            }
        } else {
            std::sort(fresh.begin(), fresh.end());
        }
        for (uint64_t key : fresh) cm[tail++] = (int32_t)(key & 0xffffffffu);
    }
}

void host_rcm(int64_t n, const int64_t* gptr, const int32_t* gadj, int32_t* perm) {
    if (n <= 0) return;
    std::vector<int32_t> cm(n);
    std::vector<uint8_t> seen(n, 0);
    host_cm_resume(n, gptr, gadj, cm.data(), seen.data(), 0, 0);
    for (int64_t t = 0; t < n; t++) perm[t] = cm[n - 1 - t];
}

// -------------------------------------------------------- first-fit groups
// Section 3.3 puts each block with the first later block it is (near-)
// orthogonal to; taken to maximal classes this is first-fit colouring in
// row order.
int32_t host_first_fit(int64_t n, const int64_t* cptr, const int32_t* cidx, const uint8_t* active,
                       int32_t* colour) {
    std::vector<int64_t> stamp;   // stamp[c] == i: colour c is taken by a conflicting row of i
    int32_t ncol = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!active[i]) { colour[i] = -1; continue; }
        for (int64_t t = cptr[i]; t < cptr[i + 1]; t++) {
            int32_t c = colour[cidx[t]];
            if (c >= 0) {
                if ((size_t)c >= stamp.size()) stamp.resize((size_t)c + 1, -1);
                stamp[c] = i;
            }
        }
        int32_t c = 0;
        while ((size_t)c < stamp.size() && stamp[c] == i) c++;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// ---------------------------------------------------------------- tiles
void build_tiles(int64_t seg0, int64_t seg1, const int64_t* off, std::vector<Tile>& out) {
    int64_t s = seg0;
    while (s < seg1) {
        int64_t e = s + 1;
        while (e < seg1 && e - s < kTileSegs && off[e + 1] - off[s] <= kTileEntries) e++;
        Tile t;
        t.seg_begin = (int32_t)s;
        t.seg_end = (int32_t)e;
        t.ent_begin = off[s];
        t.ent_end = off[e];
        out.push_back(t);
        s = e;
    }
}

// The plan validator: the group-major layout of a one-row-block plan against
// its definition (Section 3.3 grouping, eq. 3.3 sweep data).  Throws an Error
// (OBK_E_ARG) naming the first violation.
void validate_layout(const LayoutView& L) {
    auto bad = [](const std::string& why) { fail(OBK_E_ARG, "plan validator: " + why); };
    const int64_t n = L.n;
    const int32_t G = L.ngroups;
    if (G < 0 || !L.gptr || L.gptr[0] != 0) bad("group offsets do not start at 0");
    for (int32_t g = 0; g < G; g++)
        if (L.gptr[g + 1] < L.gptr[g]) bad("group offsets decrease at group " + std::to_string(g));
    const int64_t m = L.gptr[G];
    // 1. every active row exactly once, in its group, ascending within it
    std::vector<uint8_t> seen(n, 0);
    for (int32_t g = 0; g < G; g++)
        for (int64_t a = L.gptr[g]; a < L.gptr[g + 1]; a++) {
            const int64_t r = L.grow[a];
            if (r < 0 || r >= n) bad("group-major row " + std::to_string(a) + " names row " + std::to_string(r));
            if (L.group_of_row[r] != g)
                bad("row " + std::to_string(r) + " is laid out in group " + std::to_string(g) + " but belongs to " +
                    std::to_string(L.group_of_row[r]));
            if (a > L.gptr[g] && L.grow[a - 1] >= r) bad("rows of group " + std::to_string(g) + " not ascending");
            if (seen[r]++) bad("row " + std::to_string(r) + " laid out twice");
        }
    for (int64_t r = 0; r < n; r++)
        if (L.group_of_row[r] >= 0 && !seen[r]) bad("active row " + std::to_string(r) + " missing");
    // 2. rows: columns ascending, in range
    if (L.rptr[0] != 0) bad("row offsets do not start at 0");
    for (int64_t a = 0; a < m; a++) {
        if (L.rptr[a + 1] <= L.rptr[a]) bad("group-major row " + std::to_string(a) + " has no entry");
        for (int64_t e = L.rptr[a]; e < L.rptr[a + 1]; e++) {
            if (L.rcol[e] < 0 || L.rcol[e] >= n) bad("column out of range in row " + std::to_string(a));
            if (e > L.rptr[a] && L.rcol[e] <= L.rcol[e - 1]) bad("columns of row " + std::to_string(a) + " not ascending");
        }
    }
    const int vs = L.cplx ? 2 : 1;
    auto rv = [&](int64_t e, int part) { return L.rval[vs * e + part]; };
    // 3. the per-group columns: every entry of a group's rows owned by exactly
    // one segment entry, with the same value (conjugated where stored so)
    const int64_t T = L.tptr[G];
    const int64_t me = L.sptr[T];
    std::vector<uint8_t> used(me, 0);
    for (int32_t g = 0; g < G; g++) {
        const int64_t s0 = L.tptr[g], s1 = L.tptr[g + 1];
        if (s1 < s0) bad("segment offsets decrease at group " + std::to_string(g));
        for (int64_t sg = s0; sg < s1; sg++) {
            if (sg > s0 && L.tcol[sg] <= L.tcol[sg - 1]) bad("columns of group " + std::to_string(g) + " not ascending");
            for (int64_t k = L.sptr[sg]; k < L.sptr[sg + 1]; k++) {
                if (L.srow[k] < L.gptr[g] || L.srow[k] >= L.gptr[g + 1])
                    bad("segment of group " + std::to_string(g) + " holds a row of another group");
                if (k > L.sptr[sg] && L.srow[k] <= L.srow[k - 1]) bad("rows of a segment not ascending");
            }
        }
        for (int64_t a = L.gptr[g]; a < L.gptr[g + 1]; a++)
            for (int64_t e = L.rptr[a]; e < L.rptr[a + 1]; e++) {
                const int32_t c = L.rcol[e];
                const int32_t* tb = L.tcol + s0;
                const int32_t* te = L.tcol + s1;
                const int32_t* it = std::lower_bound(tb, te, c);
                if (it == te || *it != c)
                    bad("entry (" + std::to_string(a) + ", " + std::to_string(c) + ") has no column segment");
                const int64_t sg = s0 + (it - tb);
                const int32_t* rb = L.srow + L.sptr[sg];
                const int32_t* re = L.srow + L.sptr[sg + 1];
                const int32_t* jt = std::lower_bound(rb, re, (int32_t)a);
                if (jt == re || *jt != a)
                    bad("entry (" + std::to_string(a) + ", " + std::to_string(c) + ") missing from its column");
                const int64_t k = L.sptr[sg] + (jt - rb);
                if (used[k]++) bad("a column entry is owned twice");
                const double sr = L.sval[vs * k], si = L.cplx ? L.sval[vs * k + 1] : 0.0;
                const double er = rv(e, 0), ei = L.cplx ? rv(e, 1) : 0.0;
                if (sr != er || si != (L.sval_conj ? -ei : ei))
                    bad("entry (" + std::to_string(a) + ", " + std::to_string(c) + ") has another value in its column");
            }
    }
    for (int64_t k = 0; k < me; k++)
        if (!used[k]) bad("a column entry belongs to no row entry");
    // 4. no two rows of a group conflict: |cos| < delta for every pair that
    // shares a column (the others are orthogonal)
    std::vector<double> nu(m, 0.0);
    for (int64_t a = 0; a < m; a++)
        for (int64_t e = L.rptr[a]; e < L.rptr[a + 1]; e++)
            nu[a] = nu[a] + (rv(e, 0) * rv(e, 0) + (L.cplx ? rv(e, 1) * rv(e, 1) : 0.0));
    for (int64_t sg = 0; sg < T; sg++)
        for (int64_t i = L.sptr[sg]; i < L.sptr[sg + 1]; i++)
            for (int64_t j = i + 1; j < L.sptr[sg + 1]; j++) {
                const int64_t a = L.srow[i], b = L.srow[j];
                double dr = 0.0, di = 0.0;
                int64_t p = L.rptr[a], q = L.rptr[b];
                while (p < L.rptr[a + 1] && q < L.rptr[b + 1]) {
                    if (L.rcol[p] == L.rcol[q]) {
                        dr = dr + (rv(p, 0) * rv(q, 0) + (L.cplx ? rv(p, 1) * rv(q, 1) : 0.0));
                        if (L.cplx) di = di + (rv(p, 0) * rv(q, 1) - rv(p, 1) * rv(q, 0));
                        p++, q++;
                    } else if (L.rcol[p] < L.rcol[q]) {
                        p++;
                    } else {
                        q++;
                    }
                }
                const double cs = std::sqrt(dr * dr + di * di) / std::sqrt(nu[a] * nu[b]);
                if (!(cs < L.delta))
                    bad("group-major rows " + std::to_string(a) + " and " + std::to_string(b) +
                        " share a group with |cos| = " + std::to_string(cs) + " >= delta");
            }
    // 5. tiles cover each group's rows (columns) once, in order
    auto cover = [&](const Tile* tl, const int32_t* tp, const int64_t* seg, const int64_t* off, const char* what) {
        if (!tl || !tp) return;
        for (int32_t g = 0; g < G; g++) {
            int64_t at = seg[g];
            for (int32_t t = tp[g]; t < tp[g + 1]; t++) {
                if (tl[t].seg_begin != at || tl[t].seg_end <= tl[t].seg_begin)
                    bad(std::string(what) + " tiles of group " + std::to_string(g) + " leave a gap or overlap");
                if (tl[t].ent_begin != off[tl[t].seg_begin] || tl[t].ent_end != off[tl[t].seg_end])
                    bad(std::string(what) + " tile entry range differs from its segments");
                at = tl[t].seg_end;
            }
            if (at != seg[g + 1]) bad(std::string(what) + " tiles of group " + std::to_string(g) + " stop short");
        }
    };
    cover(L.rtiles, L.rtile_ptr, L.gptr, L.rptr, "row");
    cover(L.stiles, L.stile_ptr, L.tptr, L.sptr, "column");
}

}  // namespace obk
