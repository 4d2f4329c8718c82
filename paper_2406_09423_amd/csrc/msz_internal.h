// msz_internal.h -- declarations shared by the kernels and the host driver of libmsz.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msz {

constexpr unsigned kSelf = 15u;        // direction slot meaning "the vertex itself"
constexpr int kTileX = 64;             // x extent of a direction tile (16 threads x 4 vertices)
constexpr float kValueLimit = 1.2676506002282294e30f;  // 2^100: inputs above it are rejected

// Round counters.  The device block holds kSlots copies of kCntSlots counters,
// kSlotStride uint32 apart (one 128-byte line each); a launch's blocks add into
// slot blockIdx % kSlots and the host sums the slots (error bits are OR-ed).
constexpr int kSlots = 64;
constexpr int kSlotStride = 32;
constexpr int kCntBlockWords = kSlots * kSlotStride;
constexpr int kGridCap = 2048;  // grid-stride kernels: 8 blocks per compute unit
enum : int {
    kCntCase = 0,      // 0..3: false critical points per C type (a full pass), or their change (a refresh)
    kCntChanged = 5,   // values changed by the last apply
    kCntWrong = 6,     // mislabelled vertices (R detection) / wrong_any (compare)
    kCntRCases = 7,    // R-loop troublemaker hits
    kCntErr = 8,       // validation error bits
    kCntEdited = 9,
    kCntInexact = 10,
    kCntWrongMax = 11,
    kCntWrongMin = 12,
    kCntSlots = 16
};
enum : unsigned { kErrNonFinite = 1u, kErrBound = 2u, kErrWarmNonFinite = 4u, kErrWarmBound = 8u, kErrWalk = 16u };

struct Grid {
    int ndim, nx, ny, nz, nxy, n;
    int off[16];  // linear id offset of each neighbour slot; off[15] = 0 (self)
};

// Work items of a persistent grid, XCD-aware: blocks are dealt to the 8 XCDs
// round-robin, so the items are cut into K = min(8, blocks) contiguous ranges
// and the blocks with blockIdx % K == k walk range k with stride "blocks in
// the range".  Neighbouring items then share an L2.  Every item in
// [0, nitems) is visited exactly once.
struct ItemRange {
    int first, hi, stride;
};
__device__ __forceinline__ ItemRange xcd_items(int nitems) {
    const int nb = gridDim.x;
    const int K = nb < 8 ? nb : 8;
    const int k = blockIdx.x % K, slot = blockIdx.x / K;
    const int per = (nb - k + K - 1) / K;  // blocks b < nb with b % K == k
    const int lo = static_cast<int>(static_cast<long>(nitems) * k / K);
    const int hi = static_cast<int>(static_cast<long>(nitems) * (k + 1) / K);
    return {lo + slot, hi, per};
}

// Exact float helpers shared by the loop and the warm start.
__device__ __forceinline__ float f32_next_up(float x) {
    if (x == 0.0f) return __int_as_float(1);
    int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b + 1 : b - 1);
}

__device__ __forceinline__ float f32_next_down(float x) {
    if (x == 0.0f) return -__int_as_float(1);
    int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b - 1 : b + 1);
}

// Error-free difference a - b = s + e in binary64 (two-sum; no fused ops).
__device__ __forceinline__ void exact_diff(float a, float b, double& s, double& e) {
    const double da = a, nb = -static_cast<double>(b);
    s = __dadd_rn(da, nb);
    const double bv = __dadd_rn(s, -da);
    const double av = __dadd_rn(s, -bv);
    e = __dadd_rn(__dadd_rn(da, -av), __dadd_rn(nb, -bv));
}

// a - b <= c and a - b >= c, decided exactly.
__device__ __forceinline__ bool diff_at_most(float a, float b, float c) {
    double s, e;
    exact_diff(a, b, s, e);
    return s < static_cast<double>(c) || (s == static_cast<double>(c) && e <= 0.0);
}
__device__ __forceinline__ bool diff_at_least(float a, float b, float c) {
    double s, e;
    exact_diff(a, b, s, e);
    return s > static_cast<double>(c) || (s == static_cast<double>(c) && e >= 0.0);
}

// Smallest float32 L with L >= f - xi (the float reading of Eq. 1's bound).
__device__ __forceinline__ float floor_bound(float f, float xi) {
    float x = __double2float_rn(__dadd_rn(static_cast<double>(f), -static_cast<double>(xi)));
    for (int k = 0; k < 4 && !diff_at_most(f, x, xi); ++k) x = f32_next_up(x);
    for (int k = 0; k < 4; ++k) {
        const float y = f32_next_down(x);
        if (!diff_at_most(f, y, xi)) break;
        x = y;
    }
    return x;
}

__device__ __forceinline__ bool value_ok(float v) {
    return fabsf(v) <= kValueLimit;  // false for NaN and +-Inf
}

int tile_variant_count(int ndim);

}  // namespace msz
#include "../../include/msz.h"
namespace msz {
// Validates dims (ndim 2 or 3, nz == 1 in 2D, positive sides, n <= 2^31 - 2^16) and fills gr.
bool make_grid(const msz_dims& d, Grid& gr);

void launch_check_finite(const float* h, int n, unsigned* cnt, hipStream_t s);
void launch_dirs(const float* h, const Grid& gr, int variant, uint8_t* dirs_out, hipStream_t s);
void launch_label_tile(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, hipStream_t s);
void launch_label_compress(const Grid& gr, int* q_up, int* q_dn, unsigned* cnt, hipStream_t s);
void launch_label_forests(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, unsigned* cnt,
                          hipStream_t s);
void launch_label_final(const int* q_up, const int* q_dn, const Grid& gr, int* M, int* m, unsigned* cnt,
                        hipStream_t s);
void launch_compare(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* qfu, const int* qfd,
                    const int* qgu, const int* qgd, int n, unsigned* cnt, hipStream_t s);

}  // namespace msz

namespace msz {

// ------------------------------------------------------------ batch engine ---
// The correction schedule on the device: per step, k_eng_step<2>/<3> run the
// current operation of every field of a chain, pick each field's next one and
// split the next step's items over the blocks (see the engine in msz_kernels.hip).
constexpr int kEngMaxFields = 1024;
constexpr int kEngTimeSlots = 48;                   // steps per graph launch (a multiple of 2 and 3)
constexpr int kEngEndSlots = 64;                    // per timed step: start, 64 slots of block ends,
constexpr int kEngBytesWord = 1 + kEngEndSlots;     // then the algorithmic bytes the step's blocks visited
constexpr int kEngStampWords = 2 + kEngEndSlots;
constexpr int kEngChunkShift = 12;
constexpr int kEngChunk = 1 << kEngChunkShift;      // vertices per flat work item
constexpr int kSelectChunks = 8;                    // a block's range of chunks from which flag scans select
constexpr int kHostStatsWord = 32;                  // final statistics in the host word block, from word 32

enum EngOp : int {
    kOpPreA = 0,   // validation, floors, start field
    kOpPreA2,      // directions of f
    kOpPreB,       // label tiles of f (the pointers of f's forests)
    kOpPreD,       // labels of f, in place (fields with flabels)
    kOpPreE,       // directions of g and the case bytes of every vertex
    kOpApplyC,     // C-loop apply: the targets of every case of the current type
    kOpRefreshC,   // directions and cases of the vertices around the last C edits
    kOpFullC,      // the same for every vertex (after an apply that changed many)
    kOpRTile,      // label tiles of g (the changed ones)
    kOpRDetect,    // troublemakers (labels by following the exit chains), and the edits of their targets
    kOpRefreshR,   // directions and cases of the vertices around the last R edits
    kOpFullR,      // the same for every vertex
    kOpDelta,      // output
    kOpDone,
    kOpStart       // before the first step (its successor is kOpPreA)
};

// EngState.type of a merged C round (all four case types at once); 0..3 are
// the sub-loop types FPmax, FPmin, FNmax, FNmin.
constexpr int kTypeMerged = 4;

struct EngField {
    Grid gr;
    int variant;
    int merged;      // 1: merged C rounds
    int preempt;     // 1: shared targets edited without claims (preemptive mode; implies merged)
    int count_init;  // 1: label the start field once and count its mislabelled vertices
    int sum;         // 1: keep chunk summaries of the flag arrays and skip empty chunks (large single fields)
    int flabels;     // 1: resolve f's labels once before the loop (else the troublemaker passes follow f's chains)
    float xi;
    long long cap;
    const float *f, *fhat, *warm;
    float *edits, *g_out;
    float *L, *g;
    uint8_t *dirs_f, *dirs_g, *marks;
    uint8_t *cases;  // per vertex: bit t set when it is a case of type t (FPmax, FPmin, FNmax, FNmin)
    uint8_t *dirty;  // per vertex: its directions in g must be recomputed (it or a neighbour was edited)
    unsigned* chunk_dirty;  // per kEngChunk vertices: 1 when some dirty flag of the chunk may be set
    unsigned* chunk_cnt;    // per kEngChunk vertices, 2 words: the number of cases of types 0, 1 (16-bit
                            // halves of word 0) and 2, 3 (word 1) in the chunk -- exact unless chunk_unk
    unsigned* chunk_unk;    // per kEngChunk vertices: 1 when the counts are not known (after a full pass)
    uint8_t *tile_dirty;  // per label tile: a direction of g in it changed since its last tile pass
    int *Mf, *mf, *qu, *qd;  // pointers of f's (Mf, mf) and g's (qu, qd) ascending / descending forests
    unsigned* cnt;  // kCntBlockWords words (kSlots slots), in the engine's control block
};

struct EngState {
    int op, type, items;
    int init;  // 1 while the start field's labels are computed and counted (MSZ_FLAG_COUNT_INIT)
};

struct EngStats {
    long long rounds[4], rounds_r, outer_iters, n_edited, false_init[4], n_inexact, rounds_total, mislabel_init;
    int cases[4];  // current number of cases of each type (kept up to date by the refresh steps)
    int status, pad;
};

// Number of work items of operation op for one field (device and host).
int eng_items_host(const EngField& F, int op);
int eng_weight_host(const EngField& F, int op);  // cost units of one item (batch splits)
int label_tile_count(const Grid& gr);   // label tiles of the grid
// k_eng_step<ndim>(fields, cur, nxt, stats, pre, pre_next, nf, tick, word, oplog, step, ts)
const void* eng_step_kernel(int ndim);
const void* eng_init_kernel();          // k_eng_init(fields, nf)
const void* eng_setup1_kernel();        // k_eng_setup1(F, fields, states, stats, cnt3, ctl, done_word)
const void* eng_step1_kernel(int ndim); // k_eng_step1<ndim>(fields, states, states, stats, cnt3, ctl, hflag, oplog, k, ts)

}  // namespace msz
