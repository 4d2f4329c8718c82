// msz_api.hip -- host driver and C ABI of libmsz (declared in include/msz.h).
//
// The schedule of the correction loop (Sec. 5) runs on the device (the
// engine in msz_kernels.hip): every step runs one operation per field, and
// the next operation of each field follows from its counters (decided inside
// the step kernel for one field, by a decide kernel for a batch) --
//   C phase  sub-loops FPmax, FPmin, FNmax, FNmin, each until it finds no case
//            of its type, repeated until no false critical point remains (or,
//            with MSZ_FLAG_MERGED_C, rounds over all four types at once);
//   R phase  labels of g, then troublemaker detection, which also edits the
//            troublemakers' targets; back to the C phase whenever those edits
//            created a false critical point.
// The host captures kGraphSteps steps in a HIP graph and relaunches it until
// the device clears a done word in pinned host memory; a batch has one graph
// and one stream per chain (its 2D fields, its 3D fields), each relaunched
// on its own.  msz_fix runs the same schedule for one field.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/msz.h"
#include "msz_internal.h"

namespace msz {

constexpr int64_t kMaxVertices = (int64_t(1) << 31) - (int64_t(1) << 16);

bool make_grid(const msz_dims& d, Grid& gr) {
    if (d.ndim != 2 && d.ndim != 3) return false;
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return false;
    if (d.ndim == 2 && d.nz != 1) return false;
    const int64_t n = static_cast<int64_t>(d.nx) * d.ny * d.nz;
    // headroom below 2^31: vertex counts rounded up to whole work chunks,
    // flag words and tiles are formed in 32-bit arithmetic
    if (n > kMaxVertices) return false;
    gr.ndim = d.ndim;
    gr.nx = d.nx;
    gr.ny = d.ny;
    gr.nz = d.nz;
    gr.nxy = d.nx * d.ny;
    gr.n = static_cast<int>(n);
    const int64_t X = 1, Y = d.nx, Z = static_cast<int64_t>(d.nx) * d.ny;
    const int64_t off[16] = {X,      -X,      Y,          -Y,          X + Y,          -X - Y,
                             Z,      -Z,      Z + X,      -Z - X,      Z + Y,          -Z - Y,
                             Z + Y + X, -Z - Y - X, 0, 0};
    // offsets that do not fit 32 bits belong to slots no in-grid vertex can use
    for (int k = 0; k < 16; ++k) gr.off[k] = static_cast<int>(off[k] < INT32_MIN || off[k] > INT32_MAX ? 0 : off[k]);
    return true;
}

namespace {

#define MSZ_HIP(x)                                 \
    do {                                           \
        if ((x) != hipSuccess) return MSZ_EDEVICE; \
    } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Option flags accepted by the correction entry points.
constexpr int32_t kFixFlags = MSZ_FLAG_TIMING | MSZ_FLAG_MERGED_C | MSZ_FLAG_COUNT_INIT | MSZ_FLAG_PREEMPTIVE;

// The kernels move four vertices per dwordx4 access.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Workspace of one field.
struct Layout {
    size_t L, g, dirs_f, dirs_g, marks, cases, dirty, chunk_dirty, chunk_cnt, chunk_unk, tile_dirty, Mf, mf, qu, qd, total;
};

Layout layout_for(const Grid& gr) {
    const int64_t n = gr.n;
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    l.L = take(n * 4);
    l.g = take(n * 4);
    l.dirs_f = take(n);
    l.dirs_g = take(n);
    l.marks = take((n + 15) & ~int64_t(15));
    l.cases = take((n + 15) & ~int64_t(15));
    l.dirty = take((n + 15) & ~int64_t(15));
    l.chunk_dirty = take(((n + kEngChunk - 1) / kEngChunk) * 4);
    l.chunk_cnt = take(((n + kEngChunk - 1) / kEngChunk) * 8);
    l.chunk_unk = take(((n + kEngChunk - 1) / kEngChunk) * 4);
    l.tile_dirty = take(label_tile_count(gr));
    l.Mf = take(n * 4);
    l.mf = take(n * 4);
    l.qu = take(n * 4);
    l.qd = take(n * 4);
    l.total = o;
    return l;
}

// Pinned host copy of the counter block (all slots, then the summed counters
// in the last kCntSlots words), one per host thread.
unsigned* host_counters() {
    thread_local unsigned* p = nullptr;
    if (!p) {
        void* q = nullptr;
        if (hipHostMalloc(&q, (kCntBlockWords + kCntSlots) * sizeof(unsigned), hipHostMallocDefault) !=
            hipSuccess)
            return nullptr;
        p = static_cast<unsigned*>(q);
    }
    return p + kCntBlockWords;  // the summed view; the raw slots precede it
}

// Copies the counter slots back, waits, and sums them into host[0..kCntSlots).
int read_counters(const unsigned* dev, unsigned* host, hipStream_t s) {
    unsigned* raw = host - kCntBlockWords;
    MSZ_HIP(hipGetLastError());
    MSZ_HIP(hipMemcpyAsync(raw, dev, kCntBlockWords * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    MSZ_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < kCntSlots; ++k) host[k] = 0;
    for (int b = 0; b < kSlots; ++b) {
        const unsigned* slot = raw + b * kSlotStride;
        for (int k = 0; k < kCntSlots; ++k) host[k] = k == kCntErr ? (host[k] | slot[k]) : host[k] + slot[k];
    }
    return MSZ_OK;
}

int clear_counters(unsigned* dev, hipStream_t s) {
    MSZ_HIP(hipMemsetAsync(dev, 0, kCntBlockWords * sizeof(unsigned), s));
    return MSZ_OK;
}

// Scratch owned for the duration of one call.
struct Scratch {
    void* p = nullptr;
    hipStream_t s = nullptr;
    bool owned = false;
    ~Scratch() {
        if (owned && p) (void)hipFreeAsync(p, s);
    }
    int get(void* user, size_t user_bytes, size_t need, hipStream_t stream) {
        s = stream;
        if (user) {
            if (user_bytes < need) return MSZ_EINVAL;
            p = user;
            return MSZ_OK;
        }
        if (hipMallocAsync(&p, need, stream) != hipSuccess) {
            p = nullptr;
            return MSZ_ENOMEM;
        }
        owned = true;
        return MSZ_OK;
    }
};

int check_xi(float xi) {
    if (!(std::fabs(xi) <= kValueLimit)) return MSZ_ENONFINITE;
    if (xi < 0.0f) return MSZ_EINVAL;
    return MSZ_OK;
}

// ------------------------------------------------------------- engine ---

constexpr int kGraphSteps = kEngTimeSlots;  // steps per graph launch (even: parities line up)
static_assert(kGraphSteps % 2 == 0, "states alternate between two buffers");
// a batch chain's block prefix of one step: nf + 1 prefix sums, then the
// number of fields given blocks; two of them, by step parity
constexpr int kPreWords = kEngMaxFields + 2;

// Per host thread and device: the engine's control block (device), a pinned
// read-back word, and the graph of kGraphSteps steps for the last topology.
struct EngineCtx {
    int device = -1;
    char* ctl_mem = nullptr;  // fields, states, stats, pre2, pre3, tick2, tick3, ctl, oplog
    EngField* fields = nullptr;
    EngState* states = nullptr;
    EngStats* stats = nullptr;
    int *pre2 = nullptr, *pre3 = nullptr, *ctl = nullptr, *oplog = nullptr;
    int *tick2 = nullptr, *tick3 = nullptr;  // a chain's tickets: kEngMaxFields + 1 words
    unsigned long long* tstamp = nullptr;  // profiling: kEngStampWords words per step
    unsigned* counters = nullptr;          // kCntBlockWords per field
    int* host = nullptr;  // pinned: [0] ctl, [1 .. kGraphSteps] oplog, then 2 * kGraphSteps stamps
    // pinned, device-mapped: [0] 1 while a single field is active, [1], [2] 1
    // while a batch's 2D / 3D chain is active (the device clears them), final
    // statistics of a single field from word kHostStatsWord
    int* hflag = nullptr;
    int* hflag_dev = nullptr;  // its device address
    // ev[0]: end of the last graph launch of a single field; ev[1], ev[2]: of
    // each batch chain; ev[3]: the caller's stream reached the batch's start
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t cs[2] = {nullptr, nullptr};  // the batch chains' streams (default priority)
    // cached graphs: a single field's, or one per batch chain
    int g_nf = -1, g_n2 = -1, g_grid2 = 0, g_grid3 = 0;
    bool g_timing = false;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};

    void drop_graph() {
        for (int d = 0; d < 2; ++d) {
            if (exec[d]) (void)hipGraphExecDestroy(exec[d]);
            if (graph[d]) (void)hipGraphDestroy(graph[d]);
            exec[d] = nullptr;
            graph[d] = nullptr;
        }
        g_nf = -1;
    }
    // No destructor work: at process exit the HIP runtime may already be torn
    // down, and the device memory (about 0.4 MB per host thread) is reclaimed
    // with the process.

    static size_t host_bytes() { return 256 + stamp_bytes(); }
    // per step, a stamp block for each of the two step kernels (a batch's 2D
    // and 3D kernels; a single field uses the first)
    static size_t stamp_bytes() { return sizeof(unsigned long long) * kEngStampWords * 2 * kGraphSteps; }
    unsigned long long* host_stamps() const { return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(host) + 256); }

    int init(int dev) {
        if (device == dev && ctl_mem) return MSZ_OK;
        drop_graph();
        if (ctl_mem) (void)hipFree(ctl_mem);
        ctl_mem = nullptr;
        size_t o = 0;
        auto take = [&](size_t b) {
            const size_t r = o;
            o += align256(b);
            return r;
        };
        const size_t of = take(sizeof(EngField) * kEngMaxFields);
        const size_t os = take(sizeof(EngState) * 2 * kEngMaxFields);
        const size_t ost = take(sizeof(EngStats) * kEngMaxFields);
        const size_t op2 = take(sizeof(int) * 2 * kPreWords);
        const size_t op3 = take(sizeof(int) * 2 * kPreWords);
        const size_t ot2 = take(sizeof(int) * (kEngMaxFields + 1));
        const size_t ot3 = take(sizeof(int) * (kEngMaxFields + 1));
        const size_t oc = take(sizeof(int) * 4);
        const size_t ol = take(sizeof(int) * kGraphSteps * kEngMaxFields);
        const size_t ot = take(stamp_bytes());
        const size_t oc2 = take(sizeof(unsigned) * kCntBlockWords * kEngMaxFields);
        void* p = nullptr;
        if (hipMalloc(&p, o) != hipSuccess) return MSZ_ENOMEM;
        ctl_mem = static_cast<char*>(p);
        fields = reinterpret_cast<EngField*>(ctl_mem + of);
        states = reinterpret_cast<EngState*>(ctl_mem + os);
        stats = reinterpret_cast<EngStats*>(ctl_mem + ost);
        pre2 = reinterpret_cast<int*>(ctl_mem + op2);
        pre3 = reinterpret_cast<int*>(ctl_mem + op3);
        tick2 = reinterpret_cast<int*>(ctl_mem + ot2);
        tick3 = reinterpret_cast<int*>(ctl_mem + ot3);
        ctl = reinterpret_cast<int*>(ctl_mem + oc);
        oplog = reinterpret_cast<int*>(ctl_mem + ol);
        tstamp = reinterpret_cast<unsigned long long*>(ctl_mem + ot);
        counters = reinterpret_cast<unsigned*>(ctl_mem + oc2);
        if (!host) {
            void* h = nullptr;
            if (hipHostMalloc(&h, host_bytes(), hipHostMallocDefault) != hipSuccess)
                return MSZ_ENOMEM;
            host = static_cast<int*>(h);
        }
        if (!hflag) {
            void* h = nullptr;
            void* d = nullptr;
            static_assert((kHostStatsWord + sizeof(EngStats) / 4) * 4 <= 512, "host word block");
            if (hipHostMalloc(&h, 512, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return MSZ_ENOMEM;
            if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) return MSZ_EDEVICE;
            hflag = static_cast<int*>(h);
            hflag_dev = static_cast<int*>(d);
        }
        for (hipEvent_t& e : ev)
            if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MSZ_EDEVICE;
        for (hipStream_t& c : cs)
            if (!c && hipStreamCreateWithFlags(&c, hipStreamNonBlocking) != hipSuccess) return MSZ_EDEVICE;
        device = dev;
        return MSZ_OK;
    }

    // (Re)builds the graphs when the topology changed.  A batch's table holds
    // its n2 2D fields first, then its 3D fields.
    int graph_for(int nf, int n2, bool timing, int grid2, int grid3) {
        if (g_nf == nf && g_n2 == n2 && g_timing == timing && g_grid2 == grid2 && g_grid3 == grid3)
            return MSZ_OK;
        drop_graph();
        hipGraph_t gcur = nullptr;
        hipGraphNode_t last = nullptr;
        // a kernel node after the last one added to the current graph
        auto add_kernel = [&](const void* fn, dim3 g, dim3 b, void** args) -> bool {
            hipKernelNodeParams p{};
            p.func = const_cast<void*>(fn);
            p.gridDim = g;
            p.blockDim = b;
            p.sharedMemBytes = 0;
            p.kernelParams = args;
            hipGraphNode_t n = nullptr;
            if (hipGraphAddKernelNode(&n, gcur, last ? &last : nullptr, last ? 1 : 0, &p) != hipSuccess)
                return false;
            last = n;
            return true;
        };
        if (nf == 1) {  // one field: one step kernel per step, deciding for itself
            const bool has3 = n2 == 0;
            if (hipGraphCreate(&graph[0], 0) != hipSuccess) return MSZ_EDEVICE;
            gcur = graph[0];
            const void* fn = eng_step1_kernel(has3 ? 3 : 2);
            const int grid = has3 ? grid3 : grid2;
            for (int st = 0; st < kGraphSteps; ++st) {
                unsigned long long* ts = timing ? tstamp + 2 * st * kEngStampWords : nullptr;
                int* log = timing ? oplog : nullptr;
                int stp = st;
                void* a[] = {&fields, &states, &states, &stats, &counters, &ctl, &hflag_dev, &log, &stp, &ts};
                if (!add_kernel(fn, dim3(grid), dim3(256), a)) return MSZ_EDEVICE;
            }
            if (hipGraphInstantiate(&exec[0], graph[0], nullptr, nullptr, 0) != hipSuccess) return MSZ_EDEVICE;
        }
        // A batch: one graph per dimension's chain of steps, each launched on
        // its own stream, so that the chains never wait for each other (not
        // even where a launch ends).  Per step: one kernel, which also takes
        // the decisions and forms the next step's block prefix.
        for (int d = 0; nf > 1 && d < 2; ++d) {
            int cnt = d == 0 ? n2 : nf - n2;
            if (cnt == 0) continue;
            const int off = d == 0 ? 0 : n2;
            if (hipGraphCreate(&graph[d], 0) != hipSuccess) return MSZ_EDEVICE;
            gcur = graph[d];
            last = nullptr;
            int* word = hflag_dev + 1 + d;
            for (int st = 0; st < kGraphSteps; ++st) {
                const int par = st & 1;
                EngField* fp = fields + off;
                EngState* cur = states + par * nf + off;
                EngState* nxt = states + (par ^ 1) * nf + off;
                EngStats* sp = stats + off;
                int* pre = (d == 0 ? pre2 : pre3) + par * kPreWords;
                int* pre_next = (d == 0 ? pre2 : pre3) + (par ^ 1) * kPreWords;
                int* tick = d == 0 ? tick2 : tick3;
                unsigned long long* ts = timing ? tstamp + (2 * st + d) * kEngStampWords : nullptr;
                int* log = timing ? oplog + (d == 0 ? 0 : kGraphSteps * n2) : nullptr;
                int stp = st;
                void* a[] = {&fp, &cur, &nxt, &sp, &pre, &pre_next, &cnt, &tick, &word, &log, &stp, &ts};
                if (!add_kernel(eng_step_kernel(d == 0 ? 2 : 3), dim3(d == 0 ? grid2 : grid3), dim3(256), a))
                    return MSZ_EDEVICE;
            }
            if (hipGraphInstantiate(&exec[d], graph[d], nullptr, nullptr, 0) != hipSuccess) return MSZ_EDEVICE;
        }
        g_nf = nf;
        g_n2 = n2;
        g_timing = timing;
        g_grid2 = grid2;
        g_grid3 = grid3;
        return MSZ_OK;
    }
};

EngineCtx& engine_ctx() {
    thread_local EngineCtx ctx;
    return ctx;
}

int phase_of_op(int op) {
    switch (op) {
        case kOpPreA: return MSZ_PHASE_VALIDATE;
        case kOpPreA2: return MSZ_PHASE_DIRS;
        case kOpPreB: case kOpRTile: return MSZ_PHASE_LABEL_TILE;
        case kOpPreD: return MSZ_PHASE_LABEL_FINAL;
        case kOpApplyC: return MSZ_PHASE_APPLY;
        case kOpPreE: case kOpFullC: case kOpFullR: return MSZ_PHASE_DIRS_DETECT;
        case kOpRefreshC: case kOpRefreshR: return MSZ_PHASE_REFRESH;
        case kOpRDetect: return MSZ_PHASE_DETECT_R;
        case kOpDelta: return MSZ_PHASE_DELTA;
        default: return -1;
    }
}

// Step-kernel grid of one dimension: the blocks that fit on the device at once.
// (single: the one-field step kernel.)
int step_grid(int dev, int ndim, bool single) {
    thread_local int cached_dev = -1, cached[4] = {0, 0, 0, 0};
    if (cached_dev != dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
        for (int k = 0; k < 4; ++k) {
            int b = 0;
            const void* fn = k < 2 ? eng_step_kernel(2 + k) : eng_step1_kernel(k);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, 256, 0) != hipSuccess) return 0;
            cached[k] = cus * std::max(1, b);
        }
        cached_dev = dev;
    }
    return cached[(single ? 2 : 0) + (ndim == 3 ? 1 : 0)];
}

// Schedule of the calling thread's last timed single-field run: the phase of
// every step (-1 for the idle steps that close the last graph launch).
std::vector<int32_t>& last_schedule() {
    thread_local std::vector<int32_t> v;
    return v;
}

// Every step-kernel launch of the calling thread's last timed run.
std::vector<msz_launch>& last_launches() {
    thread_local std::vector<msz_launch> v;
    return v;
}

// One engine run over hf.size() fields whose workspaces are already bound.
// Fills st[] (one per field).  With timing, every step-kernel launch is
// recorded (last_launches: duration from its clock stamps, algorithmic bytes)
// and, for one field, the per-step durations are added to ms[] / launches[]
// by phase.
int run_engine(std::vector<EngField>& hf, std::vector<EngStats>& st, bool timing, double* ms, int64_t* launches,
               int64_t max_steps, hipStream_t s) {
    const int nf = static_cast<int>(hf.size());
    int dev = 0;
    MSZ_HIP(hipGetDevice(&dev));
    EngineCtx& E = engine_ctx();
    if (int rc = E.init(dev)) return rc;
    const bool single = nf == 1;
    int grid2 = step_grid(dev, 2, single), grid3 = step_grid(dev, 3, single);
    if (grid2 < 1 || grid3 < 1) return MSZ_EDEVICE;
    // The device table holds the 2D fields first, then the 3D fields (each
    // dimension is one chain of steps); order[p] is the caller's index of
    // table entry p.
    std::vector<int> order(nf);
    for (int j = 0; j < nf; ++j) order[j] = j;
    std::stable_partition(order.begin(), order.end(), [&](int j) { return hf[j].gr.ndim == 2; });
    std::vector<EngField> tab(nf);
    for (int p = 0; p < nf; ++p) tab[p] = hf[order[p]];
    int n2 = 0;
    std::vector<EngState> hs(2 * nf);
    std::vector<int64_t> u2, u3;  // a batch: each chain's fields' units (items x weight) of the first step
    for (int j = 0; j < nf; ++j) {
        const int items = eng_items_host(tab[j], kOpPreA);
        hs[j] = EngState{kOpPreA, 0, items, 0};
        hs[nf + j] = EngState{kOpDone, 0, 0, 0};
        const bool three = tab[j].gr.ndim == 3;
        n2 += !three;
        (three ? u3 : u2).push_back(static_cast<int64_t>(items) * eng_weight_host(tab[j], kOpPreA));
    }
    const int n3 = nf - n2;
    const bool has2 = n2 > 0, has3 = n3 > 0;
    if (!single) {
        // batch step kernels: twice as many blocks as fit on the device at
        // once, so the 2D and 3D chains running side by side keep each
        // other's idle slots filled (the 96-field batch: 61.9 ms against 68.1
        // with one resident grid each, 89.7 with half, 43.6 against 45.7
        // after the items were weighted by cost).  The single-field kernel
        // stays at one resident grid: each of its blocks takes the schedule
        // decision itself, and twice as many cost 38% more.
        grid2 *= 2;
        grid3 *= 2;
        // every field of a chain needs a block of its own in a step
        grid2 = std::max(grid2, n2 + 1);
        grid3 = std::max(grid3, n3 + 1);
    }
    // the first step's blocks per field, as the step kernel assigns them for
    // the steps after it, and the number of fields given blocks
    auto block_prefix = [](const std::vector<int64_t>& u, int grid) {
        const int m = static_cast<int>(u.size());
        int64_t total = 0;
        for (int64_t x : u) total += x;
        const int64_t slots = grid > m ? grid - m : 1;
        const int64_t per = total > 0 ? (total + slots - 1) / slots : 1;
        std::vector<int> p(m + 2, 0);
        for (int i = 0; i < m; ++i) {
            const int nb = static_cast<int>((u[i] + per - 1) / per);
            p[i + 1] = p[i] + nb;
            p[m + 1] += nb > 0;
        }
        return p;
    };
    const std::vector<int> p2 = block_prefix(u2, grid2), p3 = block_prefix(u3, grid3);
    if (timing) {
        last_schedule().clear();
        last_launches().clear();
    }
    for (int j = 0; j < nf; ++j) tab[j].cnt = E.counters + static_cast<size_t>(j) * kCntBlockWords;
    // a single field keeps chunk summaries of its flag arrays when each block
    // of the step kernel scans at least kSelectChunks chunks
    if (single) {
        const int64_t chunks = (static_cast<int64_t>(tab[0].gr.n) + kEngChunk - 1) / kEngChunk;
        tab[0].sum = chunks >= static_cast<int64_t>(kSelectChunks) * (has3 ? grid3 : grid2) ? 1 : 0;
    }
    if (int rc = E.graph_for(nf, n2, timing, grid2, grid3)) {
        E.drop_graph();
        return rc;
    }
    volatile int* flag = E.hflag;
    *flag = 1;  // cleared by the device when the work is done
    volatile int* chain_word = E.hflag + 1;  // a batch: each chain's done word
    chain_word[0] = has2 ? 1 : 0;
    chain_word[1] = has3 ? 1 : 0;
    if (single) {
        // one setup kernel: field entry, start states, counters, statistics,
        // marks, case bytes and dirty flags (no uploads, no memsets)
        EngField F = tab[0];
        EngField* fp = E.fields;
        EngState* sp = E.states;
        EngStats* tp = E.stats;
        unsigned* cp = E.counters;
        int* lp = E.ctl;
        int* no_word = nullptr;  // the done word is in pinned host memory, raised above
        void* a[] = {&F, &fp, &sp, &tp, &cp, &lp, &no_word};
        const int nw = (F.gr.n + 15) >> 4;
        MSZ_HIP(hipLaunchKernel(eng_setup1_kernel(), dim3(std::max(1, std::min(2048, (nw + 255) / 256))), dim3(256),
                                a, 0, s));
    } else {
        // the chains' active words (a chain without fields is inactive from the start)
        const int active[2] = {has2 ? 1 : 0, has3 ? 1 : 0};
        MSZ_HIP(hipMemcpyAsync(E.fields, tab.data(), sizeof(EngField) * nf, hipMemcpyHostToDevice, s));
        MSZ_HIP(hipMemcpyAsync(E.states, hs.data(), sizeof(EngState) * 2 * nf, hipMemcpyHostToDevice, s));
        MSZ_HIP(hipMemcpyAsync(E.pre2, p2.data(), sizeof(int) * p2.size(), hipMemcpyHostToDevice, s));
        MSZ_HIP(hipMemcpyAsync(E.pre3, p3.data(), sizeof(int) * p3.size(), hipMemcpyHostToDevice, s));
        // the tickets (every step resets the ones it draws; cleared here as well)
        MSZ_HIP(hipMemsetAsync(E.tick2, 0, sizeof(int) * (kEngMaxFields + 1), s));
        MSZ_HIP(hipMemsetAsync(E.tick3, 0, sizeof(int) * (kEngMaxFields + 1), s));
        MSZ_HIP(hipMemcpyAsync(E.ctl, active, sizeof(active), hipMemcpyHostToDevice, s));
        MSZ_HIP(hipMemsetAsync(E.stats, 0, sizeof(EngStats) * nf, s));
        int total = 0;
        for (const EngField& F : tab) total = std::max(total, (F.gr.n + 15) >> 4);
        EngField* fp = E.fields;
        int nfv = nf;
        void* a[] = {&fp, &nfv};
        MSZ_HIP(hipLaunchKernel(eng_init_kernel(), dim3(std::max(1, std::min(2048, (total + 255) / 256))), dim3(256),
                                a, 0, s));
    }
    int wall_khz = 0;
    if (timing && (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0))
        return MSZ_EDEVICE;
    int64_t steps = 0;
    int rc = MSZ_OK;
    // a batch: the chains start once the caller's stream reaches this point,
    // and the caller's stream waits for them at the end
    bool live[2] = {!single && has2, !single && has3};
    int64_t chain_steps[2] = {0, 0};
    auto chains_after_caller = [&]() {
        if (hipEventRecord(E.ev[3], s) != hipSuccess) return false;
        for (int d = 0; d < 2; ++d)
            if (live[d] && hipStreamWaitEvent(E.cs[d], E.ev[3], 0) != hipSuccess) return false;
        return true;
    };
    auto launch_chain = [&](int d) {
        chain_steps[d] += kGraphSteps;
        return hipGraphLaunch(E.exec[d], E.cs[d]) == hipSuccess && hipEventRecord(E.ev[1 + d], E.cs[d]) == hipSuccess;
    };
    auto caller_after_chains = [&]() {
        for (int d = 0; d < 2; ++d)
            if ((d == 0 ? has2 : has3) && hipStreamWaitEvent(s, E.ev[1 + d], 0) != hipSuccess) return false;
        return true;
    };
    if (!timing && single) {
        // Relaunch until the device clears the done word (pinned host memory):
        // no read-back copy per launch.
        for (;;) {
            if (hipGraphLaunch(E.exec[0], s) != hipSuccess || hipEventRecord(E.ev[0], s) != hipSuccess ||
                hipEventSynchronize(E.ev[0]) != hipSuccess) {
                rc = MSZ_EDEVICE;
                break;
            }
            steps += kGraphSteps;
            if (*flag == 0) break;
            if (steps > max_steps) { rc = MSZ_EDEVICE; break; }
        }
    }
    if (!timing && !single) {
        // Each chain is relaunched as soon as its last launch has ended and
        // its done word is still raised, independently of the other chain.
        bool ok = chains_after_caller();
        for (int d = 0; ok && d < 2; ++d)
            if (live[d]) ok = launch_chain(d);
        while (ok && (live[0] || live[1])) {
            for (int d = 0; ok && d < 2; ++d) {
                if (!live[d]) continue;
                const hipError_t q = hipEventQuery(E.ev[1 + d]);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) { ok = false; break; }
                if (chain_word[d] == 0) { live[d] = false; continue; }
                if (chain_steps[d] > max_steps) { ok = false; break; }
                ok = launch_chain(d);
            }
        }
        if (!ok) {
            rc = MSZ_EDEVICE;
            for (int d = 0; d < 2; ++d) (void)hipStreamSynchronize(E.cs[d]);
        }
        if (!caller_after_chains()) rc = MSZ_EDEVICE;
    }
    std::vector<int> batch_log;  // timed batch: the operation of every field in every step of a launch
    std::vector<int> pos(nf);    // table position of the caller's field j
    for (int p = 0; p < nf; ++p) pos[order[p]] = p;
    if (timing && !single) batch_log.resize(static_cast<size_t>(kGraphSteps) * nf);
    while (timing) {  // one launch at a time, with the schedule and clock stamps of each step read back
        if (hipMemsetAsync(E.tstamp, 0, EngineCtx::stamp_bytes(), s) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        bool launched[2] = {live[0], live[1]};
        if (single) {
            if (hipGraphLaunch(E.exec[0], s) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        } else {
            bool ok = chains_after_caller();
            for (int d = 0; ok && d < 2; ++d)
                if (live[d]) ok = launch_chain(d);
            if (!ok || !caller_after_chains()) { rc = MSZ_EDEVICE; break; }
        }
        if (hipMemcpyAsync(E.host, E.ctl, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(E.host + 1, E.oplog, sizeof(int) * kGraphSteps, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(E.host_stamps(), E.tstamp, EngineCtx::stamp_bytes(), hipMemcpyDeviceToHost, s) !=
                hipSuccess) {
            rc = MSZ_EDEVICE;
            break;
        }
        if (!single && hipMemcpyAsync(batch_log.data(), E.oplog, sizeof(int) * batch_log.size(),
                                      hipMemcpyDeviceToHost, s) != hipSuccess) {
            rc = MSZ_EDEVICE;
            break;
        }
        if (hipStreamSynchronize(s) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        for (int k = 0; k < kGraphSteps; ++k) {
            const int ph = single ? phase_of_op(E.host[1 + k]) : -1;
            if (single) last_schedule().push_back(ph);
            // a batch logs each chain's steps apart: [step][field of the
            // chain]; a chain that was not launched (done) logs nothing
            for (int j = 0; !single && j < nf; ++j) {
                const int p = pos[j];
                const bool two = p < n2;
                int op = kOpDone;
                if (launched[two ? 0 : 1])
                    op = two ? batch_log[k * n2 + p] : batch_log[kGraphSteps * n2 + k * n3 + (p - n2)];
                last_schedule().push_back(phase_of_op(op));
            }
            for (int d = 0; d < 2; ++d) {
                if (single ? d != 0 : !launched[d]) continue;
                const unsigned long long* t = E.host_stamps() + (2 * k + d) * kEngStampWords;
                unsigned long long end = 0;
                for (int w = 1; w <= kEngEndSlots; ++w) end = std::max(end, t[w]);
                const unsigned long long t0 = t[0];
                const double dms = end >= t0 && t0 ? static_cast<double>(end - t0) / wall_khz : 0.0;
                msz_launch rec{};
                rec.kernel = single ? (has3 ? MSZ_KERNEL_STEP1_3D : MSZ_KERNEL_STEP1_2D)
                                    : (d == 0 ? MSZ_KERNEL_BATCH_2D : MSZ_KERNEL_BATCH_3D);
                rec.phase = ph;
                rec.us = dms * 1e3;
                rec.bytes = static_cast<int64_t>(t[kEngBytesWord]);
                last_launches().push_back(rec);
                if (single && ph >= 0 && end >= t[0]) {
                    ms[ph] += dms;
                    launches[ph] += 1;
                }
            }
        }
        steps += kGraphSteps;
        if (single) {
            if (E.host[0] == 0) break;
        } else {
            for (int d = 0; d < 2; ++d)
                if (live[d] && chain_word[d] == 0) live[d] = false;
            if (!live[0] && !live[1]) break;
        }
        if (steps > max_steps) { rc = MSZ_EDEVICE; break; }
    }
    if (rc != MSZ_OK) {
        E.drop_graph();
        return rc;
    }
    st.resize(nf);
    if (single) {
        // the step kernel wrote the final statistics into the pinned host words
        // before clearing the done word; the launch that did so has completed
        if (timing) MSZ_HIP(hipStreamSynchronize(s));
        std::memcpy(st.data(), const_cast<const int*>(E.hflag) + kHostStatsWord, sizeof(EngStats));
        return MSZ_OK;
    }
    std::vector<EngStats> by_pos(nf);
    MSZ_HIP(hipMemcpyAsync(by_pos.data(), E.stats, sizeof(EngStats) * nf, hipMemcpyDeviceToHost, s));
    MSZ_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < nf; ++p) st[order[p]] = by_pos[p];
    return MSZ_OK;
}

void bind_field(EngField& F, char* w) {
    const Layout l = layout_for(F.gr);
    F.L = reinterpret_cast<float*>(w + l.L);
    F.g = reinterpret_cast<float*>(w + l.g);
    F.dirs_f = reinterpret_cast<uint8_t*>(w + l.dirs_f);
    F.dirs_g = reinterpret_cast<uint8_t*>(w + l.dirs_g);
    F.marks = reinterpret_cast<uint8_t*>(w + l.marks);
    F.cases = reinterpret_cast<uint8_t*>(w + l.cases);
    F.dirty = reinterpret_cast<uint8_t*>(w + l.dirty);
    F.chunk_dirty = reinterpret_cast<unsigned*>(w + l.chunk_dirty);
    F.chunk_cnt = reinterpret_cast<unsigned*>(w + l.chunk_cnt);
    F.chunk_unk = reinterpret_cast<unsigned*>(w + l.chunk_unk);
    F.tile_dirty = reinterpret_cast<uint8_t*>(w + l.tile_dirty);
    F.Mf = reinterpret_cast<int*>(w + l.Mf);
    F.mf = reinterpret_cast<int*>(w + l.mf);
    F.qu = reinterpret_cast<int*>(w + l.qu);
    F.qd = reinterpret_cast<int*>(w + l.qd);
}

void copy_stats(const EngStats& e, bool counted_init, msz_stats* out) {
    for (int t = 0; t < 4; ++t) out->rounds[t] = e.rounds[t], out->false_init[t] = e.false_init[t];
    out->mislabel_init = counted_init ? e.mislabel_init : -1;
    out->rounds_r = e.rounds_r;
    out->outer_iters = e.outer_iters;
    out->n_edited = e.n_edited;
    out->n_inexact = e.n_inexact;
    out->status = e.status;
}

// Upper bound on steps: every round takes at most 8 steps; the bound only
// stops a runaway schedule.
int64_t step_bound(int64_t cap) {
    const int64_t b = 16 * std::min<int64_t>(cap, int64_t(1) << 24) + 4096;
    return std::min<int64_t>(b, int64_t(1) << 26);
}

// ------------------------------------------------ no-allocation variant ---
// msz_fix_noalloc keeps everything beyond its inputs and outputs in `scratch`:
// a one-field control block (field entry, the two step states, three
// statistics records, the active word, three round-counter sets, and the
// done word with the final statistics) and, after it, the field's workspace.
// In host code `scratch` names a host-side stand-in; its device address comes
// from hipGetSymbolAddress, once per device.

struct NoAllocCtl {
    size_t fields, states, stats, ctl, cnt3, words, work;  // byte offsets; work = start of the workspace
};

NoAllocCtl noalloc_ctl() {
    NoAllocCtl c{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += align256(b);
        return r;
    };
    c.fields = take(sizeof(EngField));
    c.states = take(sizeof(EngState) * 2);
    c.stats = take(sizeof(EngStats) * 3);
    c.ctl = take(sizeof(int) * 4);
    c.cnt3 = take(sizeof(unsigned) * 3 * kCntBlockWords);
    c.words = take(512);
    c.work = o;
    return c;
}

}  // namespace
}  // namespace msz

static __device__ __align__(256) char scratch[MSZ_NOALLOC_SCRATCH_BYTES];

namespace msz {
namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up on the first
// call on that device; nullptr if the lookup failed.
char* scratch_base(int dev) {
    static std::mutex mu;
    static char* base[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!base[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        base[dev] = static_cast<char*>(p);
    }
    return base[dev];
}

// The one-field schedule on the control block at `base`: the setup kernel,
// then the step kernel launched kGraphSteps times between checks of the done
// word (copied back into host stack memory), until the device lowers it.
int run_noalloc(EngField F, char* base, int64_t max_steps, EngStats& out, hipStream_t s) {
    int dev = 0;
    MSZ_HIP(hipGetDevice(&dev));
    const NoAllocCtl c = noalloc_ctl();
    EngField* fp = reinterpret_cast<EngField*>(base + c.fields);
    EngState* sp = reinterpret_cast<EngState*>(base + c.states);
    EngStats* tp = reinterpret_cast<EngStats*>(base + c.stats);
    int* lp = reinterpret_cast<int*>(base + c.ctl);
    unsigned* cp = reinterpret_cast<unsigned*>(base + c.cnt3);
    int* wp = reinterpret_cast<int*>(base + c.words);
    const int grid = step_grid(dev, F.gr.ndim, true);
    if (grid < 1) return MSZ_EDEVICE;
    F.cnt = cp;
    {
        void* a[] = {&F, &fp, &sp, &tp, &cp, &lp, &wp};
        const int nw = (F.gr.n + 15) >> 4;
        MSZ_HIP(hipLaunchKernel(eng_setup1_kernel(), dim3(std::max(1, std::min(2048, (nw + 255) / 256))), dim3(256),
                                a, 0, s));
    }
    const void* fn = eng_step1_kernel(F.gr.ndim);
    int* no_log = nullptr;
    unsigned long long* no_stamps = nullptr;
    int words[128];
    static_assert(sizeof(words) == 512, "the done word block");
    for (int64_t steps = 0;;) {
        for (int k = 0; k < kGraphSteps; ++k) {
            int kk = k;
            void* a[] = {&fp, &sp, &sp, &tp, &cp, &lp, &wp, &no_log, &kk, &no_stamps};
            MSZ_HIP(hipLaunchKernel(fn, dim3(grid), dim3(256), a, 0, s));
        }
        MSZ_HIP(hipMemcpyAsync(words, wp, sizeof(words), hipMemcpyDeviceToHost, s));
        MSZ_HIP(hipStreamSynchronize(s));
        steps += kGraphSteps;
        if (words[0] == 0) break;
        if (steps > max_steps) return MSZ_EDEVICE;
    }
    std::memcpy(&out, words + kHostStatsWord, sizeof(EngStats));
    return MSZ_OK;
}

}  // namespace
}  // namespace msz

using namespace msz;

extern "C" {

const char* msz_strerror(int code) {
    switch (code) {
        case MSZ_OK: return "ok";
        case MSZ_EINVAL: return "invalid argument";
        case MSZ_ENONFINITE: return "non-finite or too large value";
        case MSZ_EBOUND: return "error bound violated by the input";
        case MSZ_ESTALL: return "stalled: every target at its floor";
        case MSZ_ENOCONV: return "round cap reached";
        case MSZ_EDEVICE: return "HIP runtime error";
        case MSZ_ENOMEM: return "out of device memory";
        case MSZ_ETOOBIG: return "field too large for the static scratch of msz_fix_noalloc";
        default: return "unknown error";
    }
}

size_t msz_workspace_bytes(msz_dims d) {
    Grid gr;
    if (!make_grid(d, gr)) return 0;
    return layout_for(gr).total;
}

int msz_tile_variants(int32_t ndim) {
    if (ndim != 2 && ndim != 3) return 0;
    return tile_variant_count(ndim);
}

int msz_fix(const float* f, const float* fhat, msz_dims d, float xi, float* edits_out,
            const msz_options* opt, msz_stats* stats, void* stream) {
    if (!stats) return MSZ_EINVAL;
    std::memset(stats, 0, sizeof(*stats));
    auto done = [&](int rc) {
        stats->status = rc;
        return rc;
    };
    Grid gr;
    if (!make_grid(d, gr) || !f || !fhat || !edits_out) return done(MSZ_EINVAL);
    msz_options o{};
    if (opt) o = *opt;
    if (!aligned16(f) || !aligned16(fhat) || !aligned16(edits_out) || !aligned16(o.warm_start) ||
        !aligned16(o.g_out) || !aligned16(o.workspace))
        return done(MSZ_EINVAL);
    if ((o.flags & ~kFixFlags) != 0 || o.tile_override < 0 ||
        o.tile_override > tile_variant_count(d.ndim))
        return done(MSZ_EINVAL);
    if (int rc = check_xi(xi)) return done(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout l = layout_for(gr);
    Scratch ws;
    if (int rc = ws.get(o.workspace, o.workspace_bytes, l.total, s)) return done(rc);
    std::vector<EngField> hf(1);
    EngField& F = hf[0];
    F = EngField{};
    F.gr = gr;
    F.variant = o.tile_override;
    F.preempt = (o.flags & MSZ_FLAG_PREEMPTIVE) != 0;
    F.merged = (o.flags & MSZ_FLAG_MERGED_C) != 0 || F.preempt;
    F.count_init = (o.flags & MSZ_FLAG_COUNT_INIT) != 0;
    F.flabels = 1;
    F.xi = xi;
    F.cap = o.max_rounds > 0 ? o.max_rounds : (int64_t(1) << 30);
    F.f = f;
    F.fhat = fhat;
    F.warm = o.warm_start;
    F.edits = edits_out;
    F.g_out = o.g_out;
    bind_field(F, static_cast<char*>(ws.p));
    const bool timing = (o.flags & MSZ_FLAG_TIMING) != 0;
    double ms[MSZ_N_PHASES] = {};
    int64_t launches[MSZ_N_PHASES] = {};
    std::vector<EngStats> st;
    if (int rc = run_engine(hf, st, timing, ms, launches, step_bound(F.cap), s)) return done(rc);
    copy_stats(st[0], F.count_init != 0, stats);
    for (int k = 0; k < MSZ_N_PHASES; ++k) {
        stats->phase_ms[k] = static_cast<float>(ms[k]);
        stats->phase_launches[k] = static_cast<int32_t>(launches[k]);
    }
    return stats->status;
}

int msz_fix_noalloc(const float* f, const float* fhat, msz_dims d, float xi, float* edits_out,
                    const msz_options* opt, msz_stats* stats, void* stream) {
    if (!stats) return MSZ_EINVAL;
    std::memset(stats, 0, sizeof(*stats));
    auto done = [&](int rc) {
        stats->status = rc;
        return rc;
    };
    Grid gr;
    if (!make_grid(d, gr) || !f || !fhat || !edits_out) return done(MSZ_EINVAL);
    msz_options o{};
    if (opt) o = *opt;
    if (!aligned16(f) || !aligned16(fhat) || !aligned16(edits_out) || !aligned16(o.warm_start) ||
        !aligned16(o.g_out))
        return done(MSZ_EINVAL);
    if (o.workspace || o.workspace_bytes || (o.flags & ~(kFixFlags & ~MSZ_FLAG_TIMING)) != 0 ||
        o.tile_override < 0 || o.tile_override > tile_variant_count(d.ndim))
        return done(MSZ_EINVAL);
    if (int rc = check_xi(xi)) return done(rc);
    const NoAllocCtl c = noalloc_ctl();
    if (c.work + layout_for(gr).total > MSZ_NOALLOC_SCRATCH_BYTES) return done(MSZ_ETOOBIG);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return done(MSZ_EDEVICE);
    char* base = scratch_base(dev);
    if (!base) return done(MSZ_EDEVICE);
    EngField F{};
    F.gr = gr;
    F.variant = o.tile_override;
    F.preempt = (o.flags & MSZ_FLAG_PREEMPTIVE) != 0;
    F.merged = (o.flags & MSZ_FLAG_MERGED_C) != 0 || F.preempt;
    F.count_init = (o.flags & MSZ_FLAG_COUNT_INIT) != 0;
    F.flabels = 1;
    F.xi = xi;
    F.cap = o.max_rounds > 0 ? o.max_rounds : (int64_t(1) << 30);
    F.f = f;
    F.fhat = fhat;
    F.warm = o.warm_start;
    F.edits = edits_out;
    F.g_out = o.g_out;
    bind_field(F, base + c.work);
    EngStats st{};
    if (int rc = run_noalloc(F, base, step_bound(F.cap), st, static_cast<hipStream_t>(stream))) return done(rc);
    copy_stats(st, F.count_init != 0, stats);
    return stats->status;
}

int32_t msz_last_launches(msz_launch* out, int32_t max) {
    const std::vector<msz_launch>& v = last_launches();
    const int32_t n = static_cast<int32_t>(v.size());
    if (out)
        for (int32_t k = 0; k < n && k < max; ++k) out[k] = v[k];
    return n;
}

int32_t msz_last_schedule(int32_t* phases_out, int32_t max) {
    const std::vector<int32_t>& v = last_schedule();
    const int32_t n = static_cast<int32_t>(v.size());
    if (phases_out)
        for (int32_t k = 0; k < n && k < max; ++k) phases_out[k] = v[k];
    return n;
}

size_t msz_batch_workspace_bytes(const msz_job* jobs, int32_t n_jobs) {
    if (!jobs || n_jobs <= 0 || n_jobs > kEngMaxFields) return 0;
    size_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        Grid gr;
        if (!make_grid(jobs[j].d, gr)) return 0;
        total += layout_for(gr).total;
    }
    return total;
}

int msz_fix_batch(const msz_job* jobs, int32_t n_jobs, const msz_options* opt, void* stream) {
    if (!jobs || n_jobs <= 0 || n_jobs > kEngMaxFields) return MSZ_EINVAL;
    msz_options o{};
    if (opt) o = *opt;
    if (o.warm_start || o.g_out || (o.flags & ~kFixFlags) || o.tile_override || !aligned16(o.workspace))
        return MSZ_EINVAL;
    for (int j = 0; j < n_jobs; ++j) {
        Grid gr;
        const msz_job& J = jobs[j];
        if (!J.stats || !make_grid(J.d, gr) || !J.f || !J.fhat || !J.edits_out || !aligned16(J.f) ||
            !aligned16(J.fhat) || !aligned16(J.edits_out) || !aligned16(J.g_out) || J.tile < 0 ||
            J.tile > tile_variant_count(J.d.ndim))
            return MSZ_EINVAL;
        std::memset(J.stats, 0, sizeof(msz_stats));
    }
    for (int j = 0; j < n_jobs; ++j)
        if (int rc = check_xi(jobs[j].xi)) {
            jobs[j].stats->status = rc;
            return rc;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t need = msz_batch_workspace_bytes(jobs, n_jobs);
    if (need == 0) return MSZ_EINVAL;
    Scratch ws;
    if (int rc = ws.get(o.workspace, o.workspace_bytes, need, s)) return rc;
    char* w = static_cast<char*>(ws.p);
    const int64_t cap = o.max_rounds > 0 ? o.max_rounds : (int64_t(1) << 30);
    std::vector<EngField> hf(n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const msz_job& J = jobs[j];
        EngField& F = hf[j];
        F = EngField{};
        make_grid(J.d, F.gr);
        F.variant = J.tile;
        F.preempt = (o.flags & MSZ_FLAG_PREEMPTIVE) != 0;
        F.merged = (o.flags & MSZ_FLAG_MERGED_C) != 0 || F.preempt;
        F.count_init = (o.flags & MSZ_FLAG_COUNT_INIT) != 0;
        // a batch's troublemaker passes follow f's chains where they need f's
        // labels: cheaper than one more full step for every field (a field
        // corrected alone, whose R rounds resolve many labels, resolves them
        // once instead)
        F.flabels = 0;
        F.xi = J.xi;
        F.cap = cap;
        F.f = J.f;
        F.fhat = J.fhat;
        F.warm = nullptr;
        F.edits = J.edits_out;
        F.g_out = J.g_out;
        bind_field(F, w);
        w += layout_for(F.gr).total;
    }
    std::vector<EngStats> st;
    double ms[MSZ_N_PHASES] = {};
    int64_t launches[MSZ_N_PHASES] = {};
    int rc = run_engine(hf, st, (o.flags & MSZ_FLAG_TIMING) != 0, ms, launches, step_bound(cap), s);
    int first = rc;
    for (int j = 0; j < n_jobs; ++j) {
        msz_stats* out = jobs[j].stats;
        if (rc == MSZ_OK) copy_stats(st[j], (o.flags & MSZ_FLAG_COUNT_INIT) != 0, out);
        else out->status = rc;
        if (first == MSZ_OK && out->status != MSZ_OK) first = out->status;
    }
    return first;
}

int msz_labels(const float* field, msz_dims d, int32_t* max_label, int32_t* min_label, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !field || !max_label || !min_label) return MSZ_EINVAL;
    if (!aligned16(max_label) || !aligned16(min_label)) return MSZ_EINVAL;
    unsigned* hc = host_counters();
    if (!hc) return MSZ_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t need = align256(kCntBlockWords * sizeof(unsigned)) + align256(gr.n);
    Scratch ws;
    if (int rc = ws.get(nullptr, 0, need, s)) return rc;
    unsigned* cnt = static_cast<unsigned*>(ws.p);
    uint8_t* dirs = static_cast<uint8_t*>(ws.p) + align256(kCntBlockWords * sizeof(unsigned));
    if (clear_counters(cnt, s)) return MSZ_EDEVICE;
    launch_check_finite(field, gr.n, cnt, s);
    launch_dirs(field, gr, 0, dirs, s);
    launch_label_forests(dirs, gr, max_label, min_label, cnt, s);
    launch_label_final(max_label, min_label, gr, max_label, min_label, cnt, s);
    if (int rc = read_counters(cnt, hc, s)) return rc;
    if (hc[kCntErr] & kErrWalk) return MSZ_EDEVICE;
    return hc[kCntErr] ? MSZ_ENONFINITE : MSZ_OK;
}

int msz_count_false(const float* f, const float* g, msz_dims d, msz_false_counts* out, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !f || !g || !out) return MSZ_EINVAL;
    std::memset(out, 0, sizeof(*out));
    unsigned* hc = host_counters();
    if (!hc) return MSZ_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t c0 = align256(kCntBlockWords * sizeof(unsigned));
    const size_t nb = align256(gr.n), ni = align256(size_t(gr.n) * 4);
    Scratch ws;
    if (int rc = ws.get(nullptr, 0, c0 + 2 * nb + 4 * ni, s)) return rc;
    char* p = static_cast<char*>(ws.p);
    unsigned* cnt = reinterpret_cast<unsigned*>(p);
    uint8_t* df = reinterpret_cast<uint8_t*>(p + c0);
    uint8_t* dg = df + nb;
    int* qfu = reinterpret_cast<int*>(p + c0 + 2 * nb);
    int* qfd = reinterpret_cast<int*>(p + c0 + 2 * nb + ni);
    int* qgu = reinterpret_cast<int*>(p + c0 + 2 * nb + 2 * ni);
    int* qgd = reinterpret_cast<int*>(p + c0 + 2 * nb + 3 * ni);
    if (clear_counters(cnt, s)) return MSZ_EDEVICE;
    launch_check_finite(f, gr.n, cnt, s);
    launch_check_finite(g, gr.n, cnt, s);
    launch_dirs(f, gr, 0, df, s);
    launch_dirs(g, gr, 0, dg, s);
    launch_label_forests(df, gr, qfu, qfd, cnt, s);
    launch_label_forests(dg, gr, qgu, qgd, cnt, s);
    launch_compare(df, dg, qfu, qfd, qgu, qgd, gr.n, cnt, s);
    if (int rc = read_counters(cnt, hc, s)) return rc;
    if (hc[kCntErr] & kErrWalk) return MSZ_EDEVICE;
    if (hc[kCntErr]) return MSZ_ENONFINITE;
    out->fp_max = hc[kCntCase + 0];
    out->fp_min = hc[kCntCase + 1];
    out->fn_max = hc[kCntCase + 2];
    out->fn_min = hc[kCntCase + 3];
    out->wrong_max = hc[kCntWrongMax];
    out->wrong_min = hc[kCntWrongMin];
    out->wrong_any = hc[kCntWrong];
    return MSZ_OK;
}

}  // extern "C"
