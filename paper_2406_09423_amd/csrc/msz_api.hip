// msz_api.hip -- host driver and C ABI of libmsz (declared in include/msz.h).
//
// The correction loop is driven from the host, one synchronisation per round:
// the detection of a round leaves its counters in a 256-byte block that is
// read back together with the number of values the previous apply changed,
// and the host decides the next step of the schedule (Sec. 5):
//   C phase  sub-loops FPmax, FPmin, FNmax, FNmin, each until it finds no case
//            of its type; repeated until no false critical point remains;
//   R phase  labels of g, troublemaker detection, one apply; back to the C
//            phase whenever the apply created a false critical point.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/msz.h"
#include "msz_internal.h"

namespace msz {

bool make_grid(const msz_dims& d, Grid& gr) {
    if (d.ndim != 2 && d.ndim != 3) return false;
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return false;
    if (d.ndim == 2 && d.nz != 1) return false;
    const int64_t n = static_cast<int64_t>(d.nx) * d.ny * d.nz;
    if (n >= (int64_t(1) << 31)) return false;
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

// The kernels move four vertices per dwordx4 access.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Workspace of one field.
struct Layout {
    size_t L, g, dirs_f, dirs_g, marks, Mf, mf, qu, qd, cnt, total;
};

Layout layout_for(int64_t n) {
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    l.cnt = take(kCntBlockWords * sizeof(unsigned));
    l.L = take(n * 4);
    l.g = take(n * 4);
    l.dirs_f = take(n);
    l.dirs_g = take(n);
    l.marks = take((n + 15) & ~int64_t(15));
    l.Mf = take(n * 4);
    l.mf = take(n * 4);
    l.qu = take(n * 4);
    l.qd = take(n * 4);
    l.total = o;
    return l;
}

// Optional hipEvent timing of every launch, summed per kernel kind.
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> phase_of;  // one entry per recorded (start, stop) pair
    double ms[MSZ_N_PHASES] = {};
    int64_t n[MSZ_N_PHASES] = {};
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int ph, hipStream_t s) {
        if (!on) return;
        hipEvent_t a = take();
        hipEvent_t b = take();  // reserved for end()
        if (!a || !b) {
            on = false;
            return;
        }
        (void)b;
        phase_of.push_back(ph);
        (void)hipEventRecord(a, s);
    }
    void end(hipStream_t s) {
        if (!on) return;
        (void)hipEventRecord(pool[2 * phase_of.size() - 1], s);
    }
    void collect() {  // call after the stream has been synchronised
        if (!on) return;
        for (size_t k = 0; k < phase_of.size(); ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
                ms[phase_of[k]] += t;
                n[phase_of[k]]++;
            }
        }
        phase_of.clear();
        used = 0;
    }
    void store(msz_stats* st) const {
        for (int k = 0; k < MSZ_N_PHASES; ++k) {
            st->phase_ms[k] = static_cast<float>(ms[k]);
            st->phase_launches[k] = static_cast<int32_t>(n[k]);
        }
    }
    ~Timing() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

#define TIMED(F, ph, s, call)      \
    do {                           \
        (F).tm->begin((ph), (s));  \
        call;                      \
        (F).tm->end(s);            \
    } while (0)

struct Field {
    Timing* tm;
    Grid gr;
    int variant;
    const float *f, *fhat, *warm;
    float xi;
    float *edits, *g_out;
    float *L, *g;
    uint8_t *dirs_f, *dirs_g, *marks;
    int *Mf, *mf, *qu, *qd;
    unsigned* cnt;
};

void bind(Field& F, char* ws, const Layout& l) {
    F.cnt = reinterpret_cast<unsigned*>(ws + l.cnt);
    F.L = reinterpret_cast<float*>(ws + l.L);
    F.g = reinterpret_cast<float*>(ws + l.g);
    F.dirs_f = reinterpret_cast<uint8_t*>(ws + l.dirs_f);
    F.dirs_g = reinterpret_cast<uint8_t*>(ws + l.dirs_g);
    F.marks = reinterpret_cast<uint8_t*>(ws + l.marks);
    F.Mf = reinterpret_cast<int*>(ws + l.Mf);
    F.mf = reinterpret_cast<int*>(ws + l.mf);
    F.qu = reinterpret_cast<int*>(ws + l.qu);
    F.qd = reinterpret_cast<int*>(ws + l.qd);
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
int read_counters(const unsigned* dev, unsigned* host, hipStream_t s, Timing* tm = nullptr) {
    unsigned* raw = host - kCntBlockWords;
    MSZ_HIP(hipGetLastError());
    MSZ_HIP(hipMemcpyAsync(raw, dev, kCntBlockWords * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    MSZ_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < kCntSlots; ++k) host[k] = 0;
    for (int b = 0; b < kSlots; ++b) {
        const unsigned* slot = raw + b * kSlotStride;
        for (int k = 0; k < kCntSlots; ++k) host[k] = k == kCntErr ? (host[k] | slot[k]) : host[k] + slot[k];
    }
    if (tm) tm->collect();
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

// Validation, floors, start field, directions and labels of f.
int precompute(Field& F, unsigned* hc, hipStream_t s) {
    const int n = F.gr.n;
    if (clear_counters(F.cnt, s)) return MSZ_EDEVICE;
    MSZ_HIP(hipMemsetAsync(F.marks, 0, (n + 15) & ~15, s));
    TIMED(F, MSZ_PHASE_VALIDATE, s, launch_validate_init(F.f, F.fhat, F.warm, F.xi, n, F.L, F.g, F.cnt, s));
    TIMED(F, MSZ_PHASE_DIRS, s, launch_dirs(F.f, F.gr, F.variant, F.dirs_f, s));
    TIMED(F, MSZ_PHASE_LABEL_TILE, s, launch_label_tile(F.dirs_f, F.gr, F.qu, F.qd, s));
    TIMED(F, MSZ_PHASE_LABEL_JUMP, s, launch_label_compress(F.gr, F.qu, F.qd, F.cnt, s));
    TIMED(F, MSZ_PHASE_LABEL_FINAL, s, launch_label_final(F.qu, F.qd, F.gr, F.Mf, F.mf, s));
    int rc = read_counters(F.cnt, hc, s, F.tm);
    if (rc) return rc;
    const unsigned e = hc[kCntErr];
    if (e & kErrWalk) return MSZ_EDEVICE;
    if (e & kErrNonFinite) return MSZ_ENONFINITE;
    if (e & kErrBound) return MSZ_EBOUND;
    if (e & kErrWarmNonFinite) return MSZ_ENONFINITE;
    if (e & kErrWarmBound) return MSZ_EBOUND;
    return MSZ_OK;
}

// The schedule.  Returns the status; stats are filled as it goes.
int run_loop(Field& F, int64_t cap, msz_stats* st, unsigned* hc, hipStream_t s) {
    const Grid& gr = F.gr;
    unsigned c[kCntSlots];
    auto step_read = [&]() -> int {
        int rc = read_counters(F.cnt, hc, s, F.tm);
        if (rc) return rc;
        std::memcpy(c, hc, sizeof(c));
        return MSZ_OK;
    };
    auto begin = [&]() { return clear_counters(F.cnt, s); };

    int type = 0;
    if (begin()) return MSZ_EDEVICE;
    TIMED(F, MSZ_PHASE_DIRS_DETECT, s,
          launch_dirs_detect(F.g, gr, F.variant, F.dirs_g, F.dirs_f, type, F.marks, F.cnt, s));
    if (int rc = step_read()) return rc;
    for (int t = 0; t < 4; ++t) st->false_init[t] = c[kCntCase + t];

    int64_t rounds = 0;
    bool in_c = true;
    st->outer_iters = 1;
    for (;;) {
        if (in_c) {
            if (c[kCntCase + type] > 0) {
                if (rounds >= cap) return MSZ_ENOCONV;
                if (begin()) return MSZ_EDEVICE;
                TIMED(F, MSZ_PHASE_APPLY, s,
                      launch_apply(F.g, F.L, F.marks, gr.n, F.cnt, s));
                TIMED(F, MSZ_PHASE_DIRS_DETECT, s,
                      launch_dirs_detect(F.g, gr, F.variant, F.dirs_g, F.dirs_f, type, F.marks, F.cnt, s));
                if (int rc = step_read()) return rc;
                if (c[kCntChanged] == 0) return MSZ_ESTALL;
                ++rounds;
                st->rounds[type]++;
                continue;
            }
            if (type < 3) {
                ++type;
            } else if (c[kCntCase + 0] + c[kCntCase + 1] + c[kCntCase + 2] > 0) {
                type = 0;  // the C phase repeats until no type has a case
            } else {
                in_c = false;
            }
            if (in_c) {
                if (begin()) return MSZ_EDEVICE;
                TIMED(F, MSZ_PHASE_DETECT, s,
                      launch_detect_only(F.dirs_f, F.dirs_g, gr, type, F.marks, F.cnt, s));
                if (int rc = step_read()) return rc;
                continue;
            }
        }
        // R phase: labels of g from its current directions, then troublemakers
        if (begin()) return MSZ_EDEVICE;
        TIMED(F, MSZ_PHASE_LABEL_TILE, s, launch_label_tile(F.dirs_g, gr, F.qu, F.qd, s));
        TIMED(F, MSZ_PHASE_LABEL_JUMP, s, launch_label_compress(gr, F.qu, F.qd, F.cnt, s));
        TIMED(F, MSZ_PHASE_DETECT_R, s,
              launch_detect_r(F.dirs_f, F.dirs_g, F.qu, F.qd, F.Mf, F.mf, gr, F.marks, F.cnt, s));
        if (int rc = step_read()) return rc;
        if (c[kCntErr] & kErrWalk) return MSZ_EDEVICE;
        if (c[kCntWrong] == 0) return MSZ_OK;
        if (rounds >= cap) return MSZ_ENOCONV;
        if (begin()) return MSZ_EDEVICE;
        TIMED(F, MSZ_PHASE_APPLY, s,
              launch_apply(F.g, F.L, F.marks, gr.n, F.cnt, s));
        type = 0;
        TIMED(F, MSZ_PHASE_DIRS_DETECT, s,
              launch_dirs_detect(F.g, gr, F.variant, F.dirs_g, F.dirs_f, type, F.marks, F.cnt, s));
        if (int rc = step_read()) return rc;
        if (c[kCntChanged] == 0) return MSZ_ESTALL;
        ++rounds;
        st->rounds_r++;
        if (c[kCntCase + 0] + c[kCntCase + 1] + c[kCntCase + 2] + c[kCntCase + 3] > 0) {
            in_c = true;  // Sec. 5.3: the R edit created false critical points
            st->outer_iters++;
        }
    }
}

int finish(Field& F, msz_stats* st, unsigned* hc, hipStream_t s) {
    if (clear_counters(F.cnt, s)) return MSZ_EDEVICE;
    TIMED(F, MSZ_PHASE_DELTA, s, launch_delta(F.g, F.fhat, F.gr.n, F.edits, F.g_out, F.cnt, s));
    if (int rc = read_counters(F.cnt, hc, s, F.tm)) return rc;
    st->n_edited = hc[kCntEdited];
    st->n_inexact = hc[kCntInexact];
    return MSZ_OK;
}

int check_xi(float xi) {
    if (!(std::fabs(xi) <= kValueLimit)) return MSZ_ENONFINITE;
    if (xi < 0.0f) return MSZ_EINVAL;
    return MSZ_OK;
}

int fix_one(Field& F, int64_t cap, msz_stats* st, unsigned* hc, hipStream_t s) {
    int rc = precompute(F, hc, s);
    if (rc == MSZ_OK) {
        const int status = run_loop(F, cap, st, hc, s);
        rc = status;
        if (status != MSZ_EDEVICE) {
            const int frc = finish(F, st, hc, s);
            if (frc) rc = frc;
        }
    }
    F.tm->store(st);
    return rc;
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
        default: return "unknown error";
    }
}

size_t msz_workspace_bytes(msz_dims d) {
    Grid gr;
    if (!make_grid(d, gr)) return 0;
    return layout_for(gr.n).total;
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
    if ((o.flags & ~MSZ_FLAG_TIMING) != 0 || o.tile_override < 0 ||
        o.tile_override > tile_variant_count(d.ndim))
        return done(MSZ_EINVAL);
    if (int rc = check_xi(xi)) return done(rc);
    unsigned* hc = host_counters();
    if (!hc) return done(MSZ_EDEVICE);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout l = layout_for(gr.n);
    Scratch ws;
    if (int rc = ws.get(o.workspace, o.workspace_bytes, l.total, s)) return done(rc);
    Timing tm;
    tm.on = (o.flags & MSZ_FLAG_TIMING) != 0;
    Field F{};
    F.tm = &tm;
    F.gr = gr;
    F.variant = o.tile_override;
    F.f = f;
    F.fhat = fhat;
    F.warm = o.warm_start;
    F.xi = xi;
    F.edits = edits_out;
    F.g_out = o.g_out;
    bind(F, static_cast<char*>(ws.p), l);
    const int64_t cap = o.max_rounds > 0 ? o.max_rounds : (int64_t(1) << 30);
    return done(fix_one(F, cap, stats, hc, s));
}

namespace {

// Batch workspace: the engine's tables, then one field workspace per job.
struct BatchLayout {
    size_t fields, states, stats, tickets, bar, field0, total;
    std::vector<size_t> field_off;
};

bool batch_layout(const msz_job* jobs, int32_t n, BatchLayout& bl) {
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += align256(b);
        return r;
    };
    bl.fields = take(sizeof(EngField) * n);
    bl.states = take(sizeof(EngState) * 2 * n);
    bl.stats = take(sizeof(EngStats) * n);
    bl.tickets = take(sizeof(unsigned) * 2 * n);
    bl.bar = take(sizeof(unsigned) * 4);
    bl.field0 = o;
    bl.field_off.resize(n);
    for (int j = 0; j < n; ++j) {
        Grid gr;
        if (!make_grid(jobs[j].d, gr)) return false;
        bl.field_off[j] = take(layout_for(gr.n).total + align256(2 * kEngSet * sizeof(unsigned)));
    }
    bl.total = o;
    return true;
}

int run_engine(const EngField* dev_fields, EngState* states, EngStats* stats, unsigned* tickets, unsigned* bar,
               int nf, int max_steps, hipStream_t s) {
    int dev = 0, cus = 0, bpc = 0, coop = 0;
    MSZ_HIP(hipGetDevice(&dev));
    MSZ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MSZ_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    MSZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, engine_kernel(), 256, 0));
    if (!coop || bpc < 1 || cus < 1) return MSZ_EDEVICE;
    const int grid = cus * (bpc < 2 ? bpc : 2);  // every block resident: the barrier needs it
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = MSZ_OK;
    if (hipGraphCreate(&graph, 0) != hipSuccess) return MSZ_EDEVICE;
    do {
        // node 1: clear marks, counters, tickets and the barrier (a kernel, not a memset node)
        hipGraphNode_t init = nullptr, eng = nullptr;
        void* a1[] = {const_cast<EngField**>(&dev_fields), &nf, &tickets, &bar};
        hipKernelNodeParams p1{};
        p1.func = const_cast<void*>(engine_init_kernel());
        p1.gridDim = dim3(1024);
        p1.blockDim = dim3(256);
        p1.kernelParams = a1;
        if (hipGraphAddKernelNode(&init, graph, nullptr, 0, &p1) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        // node 2: the persistent engine, one cooperative launch
        void* a2[] = {const_cast<EngField**>(&dev_fields), &states, &stats, &tickets, &bar, &nf, &max_steps};
        hipKernelNodeParams p2{};
        p2.func = const_cast<void*>(engine_kernel());
        p2.gridDim = dim3(grid);
        p2.blockDim = dim3(256);
        p2.kernelParams = a2;
        if (hipGraphAddKernelNode(&eng, graph, &init, 1, &p2) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        hipKernelNodeAttrValue v{};
        v.cooperative = 1;
        if (hipGraphKernelNodeSetAttribute(eng, hipKernelNodeAttributeCooperative, &v) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        if (hipGraphLaunch(exec, s) != hipSuccess) { rc = MSZ_EDEVICE; break; }
        if (hipStreamSynchronize(s) != hipSuccess) { rc = MSZ_EDEVICE; break; }
    } while (false);
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return rc;
}

}  // namespace

size_t msz_batch_workspace_bytes(const msz_job* jobs, int32_t n_jobs) {
    if (!jobs || n_jobs <= 0 || n_jobs > kEngMaxFields) return 0;
    BatchLayout bl;
    if (!batch_layout(jobs, n_jobs, bl)) return 0;
    return bl.total;
}

int msz_fix_batch(const msz_job* jobs, int32_t n_jobs, const msz_options* opt, void* stream) {
    if (!jobs || n_jobs <= 0 || n_jobs > kEngMaxFields) return MSZ_EINVAL;
    msz_options o{};
    if (opt) o = *opt;
    if (o.warm_start || o.g_out || (o.flags & ~MSZ_FLAG_TIMING) || o.tile_override) return MSZ_EINVAL;
    for (int j = 0; j < n_jobs; ++j) {
        Grid gr;
        const msz_job& J = jobs[j];
        if (!J.stats || !make_grid(J.d, gr) || !J.f || !J.fhat || !J.edits_out || !aligned16(J.f) ||
            !aligned16(J.fhat) || !aligned16(J.edits_out) || !aligned16(J.g_out) || J.tile < 0 ||
            J.tile > tile_variant_count(J.d.ndim))
            return MSZ_EINVAL;
        std::memset(J.stats, 0, sizeof(msz_stats));
        if (int rc = check_xi(J.xi)) {
            J.stats->status = rc;
            return rc;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchLayout bl;
    if (!batch_layout(jobs, n_jobs, bl)) return MSZ_EINVAL;
    Scratch ws;
    if (int rc = ws.get(o.workspace, o.workspace_bytes, bl.total, s)) return rc;
    char* base = static_cast<char*>(ws.p);
    const long long cap = o.max_rounds > 0 ? o.max_rounds : (1ll << 30);
    std::vector<EngField> hf(n_jobs);
    std::vector<EngState> hs(2 * n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const msz_job& J = jobs[j];
        EngField& F = hf[j];
        make_grid(J.d, F.gr);
        F.variant = J.tile;
        F.xi = J.xi;
        F.cap = cap;
        F.f = J.f;
        F.fhat = J.fhat;
        F.edits = J.edits_out;
        F.g_out = J.g_out;
        char* w = base + bl.field_off[j];
        const Layout l = layout_for(F.gr.n);
        F.L = reinterpret_cast<float*>(w + l.L);
        F.g = reinterpret_cast<float*>(w + l.g);
        F.dirs_f = reinterpret_cast<uint8_t*>(w + l.dirs_f);
        F.dirs_g = reinterpret_cast<uint8_t*>(w + l.dirs_g);
        F.marks = reinterpret_cast<uint8_t*>(w + l.marks);
        F.Mf = reinterpret_cast<int*>(w + l.Mf);
        F.mf = reinterpret_cast<int*>(w + l.mf);
        F.qu = reinterpret_cast<int*>(w + l.qu);
        F.qd = reinterpret_cast<int*>(w + l.qd);
        F.cnt = reinterpret_cast<unsigned*>(w + l.total);
        hs[j] = EngState{kOpPreA, 0, eng_items_host(F, kOpPreA), 0};
        hs[n_jobs + j] = EngState{kOpDone, 0, 0, 0};
    }
    EngField* dev_fields = reinterpret_cast<EngField*>(base + bl.fields);
    EngState* states = reinterpret_cast<EngState*>(base + bl.states);
    EngStats* stats = reinterpret_cast<EngStats*>(base + bl.stats);
    unsigned* tickets = reinterpret_cast<unsigned*>(base + bl.tickets);
    unsigned* bar = reinterpret_cast<unsigned*>(base + bl.bar);
    MSZ_HIP(hipMemcpyAsync(dev_fields, hf.data(), sizeof(EngField) * n_jobs, hipMemcpyHostToDevice, s));
    MSZ_HIP(hipMemcpyAsync(states, hs.data(), sizeof(EngState) * 2 * n_jobs, hipMemcpyHostToDevice, s));
    MSZ_HIP(hipMemsetAsync(stats, 0, sizeof(EngStats) * n_jobs, s));
    // every round takes at most 8 steps; the bound only stops a runaway batch
    const long long steps = 16 * cap + 4096;
    const int max_steps = static_cast<int>(steps < (1 << 20) ? steps : (1 << 20));
    int rc = run_engine(dev_fields, states, stats, tickets, bar, n_jobs, max_steps, s);
    std::vector<EngStats> st(n_jobs);
    std::vector<EngState> fin(2 * n_jobs);
    unsigned hbar[4] = {0, 0, 0, 0};
    if (rc == MSZ_OK) {
        MSZ_HIP(hipMemcpyAsync(st.data(), stats, sizeof(EngStats) * n_jobs, hipMemcpyDeviceToHost, s));
        MSZ_HIP(hipMemcpyAsync(fin.data(), states, sizeof(EngState) * 2 * n_jobs, hipMemcpyDeviceToHost, s));
        MSZ_HIP(hipMemcpyAsync(hbar, bar, sizeof(hbar), hipMemcpyDeviceToHost, s));
        MSZ_HIP(hipStreamSynchronize(s));
    }
    int first = rc;
    for (int j = 0; j < n_jobs; ++j) {
        msz_stats* out = jobs[j].stats;
        if (rc == MSZ_OK) {
            const EngStats& e = st[j];
            for (int t = 0; t < 4; ++t) out->rounds[t] = e.rounds[t], out->false_init[t] = e.false_init[t];
            out->rounds_r = e.rounds_r;
            out->outer_iters = e.outer_iters;
            out->n_edited = e.n_edited;
            out->n_inexact = e.n_inexact;
            out->status = e.status;
            // a field the engine did not finish (aborted barrier or step bound) is an error
            const bool done = fin[0 * n_jobs + j].op == kOpDone || fin[1 * n_jobs + j].op == kOpDone;
            if (hbar[2] || !done) out->status = MSZ_EDEVICE;
        } else {
            out->status = rc;
        }
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
    launch_label_final(max_label, min_label, gr, max_label, min_label, s);
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
