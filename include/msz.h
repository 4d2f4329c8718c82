/*
 * msz.h -- C ABI of the MI355X (gfx950) MSz correction library, libmsz.so.
 *
 * The library corrects an error-bounded decompression fhat of a piecewise
 * linear scalar field f so that the ascending and descending Morse-Smale
 * segmentations of the edited field g = fhat + delta equal those of f, while
 * |f - g| <= xi holds at every vertex (MSz, arXiv 2406.09423, Problem
 * Statement).  Every step runs in HIP kernels on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids: row-major with x fastest, vertex id i = x + nx*(y + ny*z).
 *    ndim == 2 (nz must be 1): every quad is split along its (0,0)-(1,1)
 *    diagonal, so interior vertices have 6 neighbours.  ndim == 3: Freudenthal
 *    split of every cube along (0,0,0)-(1,1,1), 14 neighbours (Sec. 3, the PL
 *    setting).  No periodic wrap.  nx, ny, nz >= 1 and nx*ny*nz <= 2^31 - 2^16.
 *  - Order (Sec. 4, simulation of simplicity): vertex a is above b iff
 *    h_a > h_b, or h_a == h_b and a > b.  -0 and +0 compare equal.
 *  - Arrays: float32 / int32, DEVICE pointers, owned by the caller, at least
 *    n = nx*ny*nz elements.  The arrays of msz_fix / msz_fix_batch (f, fhat,
 *    edits_out, warm_start, g_out, workspace) and the label arrays of
 *    msz_labels must be 16-byte aligned (every hipMalloc / torch allocation
 *    is); MSZ_EINVAL otherwise.  Host structs (stats, counts) are filled
 *    before the call returns.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  All work is enqueued on it; each call synchronises on it
 *    before returning.  The schedule of the loop runs on the device: a HIP
 *    graph of 48 steps is relaunched until the device clears a done word in
 *    pinned host memory.
 *  - Memory: the library allocates scratch per call when no workspace is
 *    given (hipMallocAsync on the stream), and keeps one control block
 *    (about 9 MB: field table, step states, round counters, statistics, the
 *    cached graph) and 512 bytes of pinned, device-mapped host memory (the
 *    done word and the final statistics of one-field runs) per host thread
 *    and device for the life of the process.  msz_fix_noalloc allocates
 *    nothing: it works in a static device array instead (see there).
 *  - Errors: the return code is the only error channel; no global state
 *    besides the control block above.  msz_strerror() names a code.  Inputs
 *    must be finite with magnitude at most 2^100 (so that no edit can
 *    overflow float32).
 *  - Concurrency: calls on different streams with separate workspaces are
 *    independent; calls from one host thread run one after another (each
 *    returns after its device work).  Calls sharing a workspace must not
 *    overlap.
 */
#ifndef MSZ_H
#define MSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MSZ_OK = 0,
    MSZ_EINVAL = -1,     /* bad dims, NULL pointer, bad option or workspace too small */
    MSZ_ENONFINITE = -2, /* NaN / Inf (or |v| > 2^100) in f, fhat, warm start or xi */
    MSZ_EBOUND = -3,     /* |f - fhat| > xi somewhere, or warm start outside [L, fhat] */
    MSZ_ESTALL = -4,     /* a round had targets but every target sat at its floor L */
    MSZ_ENOCONV = -5,    /* max_rounds productive rounds were not enough */
    MSZ_EDEVICE = -6,    /* a HIP runtime call failed */
    MSZ_ENOMEM = -7,     /* the library could not allocate scratch memory */
    MSZ_ETOOBIG = -8     /* msz_fix_noalloc: the field's scratch exceeds MSZ_NOALLOC_SCRATCH_BYTES */
};

/* Steps timed under MSZ_FLAG_TIMING (indices of msz_stats.phase_ms).  The
 * loop runs as a sequence of device-scheduled steps, each running one
 * operation; a timed step kernel stamps its first block's start and its last
 * block's end with the GPU's constant-rate clock. */
enum {
    MSZ_PHASE_VALIDATE = 0,     /* input contract, floors L, start field */
    MSZ_PHASE_DIRS = 1,         /* steepest directions of f */
    MSZ_PHASE_DIRS_DETECT = 2,  /* directions and case bytes of every vertex of g */
    MSZ_PHASE_REFRESH = 3,      /* directions and case bytes around the last edits */
    MSZ_PHASE_APPLY = 4,        /* halving of a C round's targets (from the case bytes) */
    MSZ_PHASE_LABEL_TILE = 5,   /* in-LDS pointer jumping per changed tile */
    MSZ_PHASE_LABEL_JUMP = 6,   /* (unused: the loop's labels follow the tiles' exit chains) */
    MSZ_PHASE_LABEL_FINAL = 7,  /* labels of f */
    MSZ_PHASE_DETECT_R = 8,     /* labels of g along the exit chains, troublemakers and the halving of their targets */
    MSZ_PHASE_DELTA = 9,        /* output deltas */
    MSZ_PHASE_NET = 10,         /* learned warm start: features, 3 conv layers, g0 */
    MSZ_N_PHASES = 11
};

/* msz_options.flags bits. */
#define MSZ_FLAG_TIMING 1 /* time every step kernel (adds a little overhead): msz_stats.phase_ms, msz_last_launches */
/* Merged C rounds (the parallel C-loop of Sec. 6.1): each C round finds the
 * false critical points of all four types on one snapshot of g and halves the
 * union of their targets once, instead of running the FPmax, FPmin, FNmax and
 * FNmin sub-loops in turn.  Deterministic; the result is bit-identical to the
 * oracle's merged schedule (not to the default one) and still has zero
 * segmentation error within xi.  stats.rounds[t] then counts the C rounds in
 * which type t had a case.  Accepted by msz_fix, msz_fix_batch and
 * msz_fix_learned. */
#define MSZ_FLAG_MERGED_C 2
/* Count the mislabelled vertices of the start field (stats.mislabel_init:
 * the N_f of the right-labelled ratio before any edit, Appendix B).  This
 * costs one extra labelling of the start field (a label tile pass, the face
 * compression and a comparison pass), so it is opt-in; without the flag
 * stats.mislabel_init is -1.  Accepted by msz_fix, msz_fix_batch and
 * msz_fix_learned (there the start field is the network's warm start). */
#define MSZ_FLAG_COUNT_INIT 4
/* Preemptive mode (Sec. 6.1): merged C rounds (implied) in which a target
 * proposed by several cases -- a C round's or an R round's -- is edited by
 * each of them without a claim, so they race: cases that read the same value
 * write the same halving (one edit survives and the lost ones are found again
 * in a later round), and a case that reads another's result halves it once
 * more.  The result is not deterministic; every run still ends with zero
 * segmentation error, |f - g| <= xi and g <= fhat (every value written is a
 * halving of a value no larger than the round's snapshot, so each round
 * lowers what it changes and the loop ends as the synchronous one does).
 * Accepted by msz_fix, msz_fix_batch, msz_fix_learned and msz_fix_noalloc. */
#define MSZ_FLAG_PREEMPTIVE 8

typedef struct {
    int32_t ndim;        /* 2 or 3 */
    int32_t nx, ny, nz;  /* nz == 1 when ndim == 2 */
} msz_dims;

/* Statistics of one correction (the per-type round counts mirror the paper's
 * per-iteration breakdown, Sec. 8 / Fig. 12). */
typedef struct {
    int64_t rounds[4];     /* productive rounds of the FPmax, FPmin, FNmax, FNmin sub-loops */
    int64_t rounds_r;      /* productive R-loop rounds */
    int64_t outer_iters;   /* times the C phase was entered */
    int64_t n_edited;      /* vertices whose final g differs from fhat */
    int64_t false_init[4]; /* false critical points of each type in the start field */
    int64_t mislabel_init; /* vertices of the start field with a wrong max or min label (N_f of
                              Appendix B); -1 unless MSZ_FLAG_COUNT_INIT was set */
    int64_t n_inexact;     /* vertices where no float32 delta gives fl(fhat + delta) == g */
    int32_t status;        /* the return code of the call */
    int32_t pad;
    /* Filled only with MSZ_FLAG_TIMING: summed GPU time (ms, from the GPU clock
     * stamps of each device step) and step count of each operation, indexed by
     * MSZ_PHASE_*. */
    float phase_ms[MSZ_N_PHASES];
    int32_t phase_launches[MSZ_N_PHASES];
} msz_stats;

/* Counts returned by msz_count_false (Defs. 1-3; Appendix B right-labelled ratio). */
typedef struct {
    int64_t fp_max, fp_min, fn_max, fn_min; /* false critical points of g w.r.t. f */
    int64_t wrong_max, wrong_min;           /* vertices whose max / min label differs */
    int64_t wrong_any;                      /* vertices with either label wrong (N_f) */
} msz_false_counts;

/* Options; pass NULL for all defaults. */
typedef struct {
    int64_t max_rounds;       /* cap on productive rounds; <= 0 means 2^30 */
    const float* warm_start;  /* DEVICE start field g0 with L <= g0 <= fhat, or NULL for fhat */
    float* g_out;             /* DEVICE array receiving the edited field g, or NULL */
    void* workspace;          /* DEVICE scratch of >= msz_workspace_bytes(dims), or NULL */
    size_t workspace_bytes;   /* size of `workspace` */
    int32_t tile_override;    /* 0: autotuned/default tile; k > 0: tile variant k (see msz_tile_variants) */
    int32_t flags;            /* MSZ_FLAG_* bits */
} msz_options;

/*
 * msz_fix -- the correction loop (Sec. 5: C-loops and R-loops alternated
 * until no false critical point and no mislabelled vertex remains).
 *
 *  f, fhat    DEVICE float32[n]: original field and its decompression; the
 *             input contract is |f_i - fhat_i| <= xi (checked exactly).
 *  d          grid description.
 *  xi         absolute error bound, finite, >= 0.
 *  edits_out  DEVICE float32[n]: receives delta with fl32(fhat + delta) == g
 *             wherever a float achieves it (stats->n_inexact counts the rest).
 *  opt        options or NULL.
 *  stats      HOST struct, required.
 *
 * Edits only ever lower values: g_i lies in [L_i, fhat_i], where L_i is the
 * smallest float32 >= f_i - xi (Eq. 1).  Each round works on a snapshot of g
 * and halves every proposed target once: g <- fl(fl(g + L)/2), snapped to L
 * when rounding makes no progress (Eqs. 2-6).  Sub-loop order FPmax, FPmin,
 * FNmax, FNmin (Sec. 5.1); an FPmin lowers the vertex's descent neighbour in
 * f; an FNmax lowers the vertex's ascent neighbour in g; the R-loop lowers
 * dn_f(u) for a wrong-minimum troublemaker u and up_g(u) for a wrong-maximum
 * one (Sec. 5.2, Eq. 6).  The result is bit-identical to the serial oracle's.
 * On MSZ_ESTALL / MSZ_ENOCONV, edits_out still holds a valid, bounded delta.
 */
int msz_fix(const float* f, const float* fhat, msz_dims d, float xi, float* edits_out,
            const msz_options* opt, msz_stats* stats, void* stream);

/*
 * msz_fix_noalloc -- msz_fix for callers that cannot allocate memory: code
 * running while a stream is being captured into a graph elsewhere, tight
 * serving loops, harnesses that forbid allocation.  It calls no hipMalloc,
 * hipFree, hipHostMalloc or graph instantiation: its workspace and control
 * block live in one static device array of MSZ_NOALLOC_SCRATCH_BYTES bytes,
 * which every device the library runs on holds from module load until the
 * process ends, and it launches the step kernels directly.
 *
 * Arguments and results are those of msz_fix, and so is the result: g,
 * edits_out and every statistic are bit-identical to msz_fix's.  Differences:
 *  - opt->workspace must be NULL and opt->workspace_bytes 0, and
 *    MSZ_FLAG_TIMING is not accepted (MSZ_EINVAL);
 *  - a field whose workspace plus the control block exceeds the array
 *    returns MSZ_ETOOBIG before any device work.  The limit admits fields of
 *    up to about 3.4e6 vertices, e.g. 150^3 or 1850 x 1850 (the workspace
 *    takes 29 bytes per vertex: msz_workspace_bytes);
 *  - every call on a device shares that device's array, and a call leaves
 *    its contents behind (each call clears what it needs cleared).  Calls
 *    that overlap on one device, from several host threads or streams,
 *    race on the array and give undefined results: serialise them.
 * The call synchronises on the stream before returning, as msz_fix does.
 */
#define MSZ_NOALLOC_SCRATCH_BYTES (96u << 20)
int msz_fix_noalloc(const float* f, const float* fhat, msz_dims d, float xi, float* edits_out,
                    const msz_options* opt, msz_stats* stats, void* stream);

/* Profiling aid: every step-kernel launch of the calling host thread's last
 * msz_fix or msz_fix_batch call that ran with MSZ_FLAG_TIMING, in launch
 * order (a batch: per step index, the 2D chain's launch, then the 3D
 * chain's).  A step kernel records, from the GPU's constant-rate clock, its first
 * block's start and its last block's end, and the algorithmic bytes of the
 * units its blocks visited: per operation, the compulsory reads and writes of
 * each vertex of a visited direction or label tile, each scanned flag byte,
 * edit attempt, recomputed vertex, face-layer pointer, the two forests'
 * pointers of each vertex whose labels the troublemaker search resolves, and
 * each pointer load of an exit-chain walk or load or store of a compression
 * walk (halo and cache re-reads not counted). */
enum {
    MSZ_KERNEL_STEP1_2D = 0, /* one field: the step kernel of a 2D field (decides and runs) */
    MSZ_KERNEL_STEP1_3D = 1,
    MSZ_KERNEL_BATCH_2D = 2, /* a batch: the step kernel of the 2D fields */
    MSZ_KERNEL_BATCH_3D = 3
};
typedef struct {
    int32_t kernel;  /* MSZ_KERNEL_* */
    int32_t phase;   /* MSZ_PHASE_* of a one-field step; -1 for a batch step (mixed) or an idle step */
    double us;       /* first block's start to last block's end, microseconds (0 if no block ran) */
    int64_t bytes;   /* algorithmic bytes of the units the launch visited */
} msz_launch;
/* Writes at most max records (out may be NULL); returns the number recorded. */
int32_t msz_last_launches(msz_launch* out, int32_t max);

/* Profiling aid: the step schedule of the calling host thread's last msz_fix
 * or msz_fix_batch that ran with MSZ_FLAG_TIMING.  Every step of the device
 * schedule runs one operation per field; for one field, step k is
 * phases_out[k] (an MSZ_PHASE_* index, or -1 for the idle steps that end the
 * last graph launch), and the entries line up one to one with the step-kernel
 * dispatches of that call in a kernel trace; for a batch of n_jobs fields,
 * phases_out[k * n_jobs + j] is field j's operation in step k of its
 * dimension's chain of steps (-1 once it is done).  Writes at most max entries (phases_out may be NULL) and returns the
 * number of entries recorded. */
int32_t msz_last_schedule(int32_t* phases_out, int32_t max);

/*
 * msz_labels -- ascending / descending segmentation labels of one field
 * (Sec. 3): max_label[i] (min_label[i]) is the id of the maximum (minimum)
 * that the steepest ascending (descending) integral line from i reaches.
 * field: DEVICE float32[n]; max_label, min_label: DEVICE int32[n].
 */
int msz_labels(const float* field, msz_dims d, int32_t* max_label, int32_t* min_label,
               void* stream);

/*
 * msz_count_false -- false critical points of g with respect to f (Defs. 1-3)
 * and mislabelled vertices (Problem Statement; wrong_any is N_f of the
 * right-labelled ratio 1 - N_f/N, Appendix B).  f, g: DEVICE float32[n];
 * out: HOST struct.
 */
int msz_count_false(const float* f, const float* g, msz_dims d, msz_false_counts* out,
                    void* stream);

/* One field of a batch. */
typedef struct {
    const float* f;      /* DEVICE float32[n] */
    const float* fhat;   /* DEVICE float32[n] */
    msz_dims d;
    float xi;
    int32_t tile;        /* direction tile variant for this field (0 = default, see msz_tile_variants) */
    float* edits_out;    /* DEVICE float32[n] */
    float* g_out;        /* DEVICE float32[n] or NULL */
    msz_stats* stats;    /* HOST, required */
} msz_job;

/*
 * msz_fix_batch -- corrects n_jobs (<= 1024) independent fields of uneven
 * sizes together: every device step advances each unfinished field by one
 * operation of the schedule msz_fix follows, so each field's result is
 * bit-identical to its own msz_fix.  The 2D fields and the 3D fields form two
 * chains of steps that run side by side without waiting for each other; per
 * step of a chain, one step kernel runs the work items of all its fields as
 * one index space split over the blocks by each operation's cost; in the
 * same kernel the last block of each field picks the field's next operation
 * and the last field decided splits the next step's items over the blocks.  Each chain's steps run from a HIP graph on a stream of the
 * library's own, relaunched until its fields are done; the chains start
 * after the work already queued on `stream` and the work queued on it
 * afterwards waits for them.  opt->workspace (if given) must hold
 * msz_batch_workspace_bytes(jobs, n_jobs) bytes; opt->warm_start, opt->g_out
 * and opt->tile_override must be unset (use msz_job.g_out / msz_job.tile);
 * opt->max_rounds, MSZ_FLAG_MERGED_C and MSZ_FLAG_PREEMPTIVE apply to every field
 * (MSZ_FLAG_TIMING records the step-kernel launches for msz_last_launches and
 * fills no per-field timings).
 * Returns MSZ_OK when every field converged, else the first failing field's
 * code (see each stats; per-phase timings are not filled).
 */
int msz_fix_batch(const msz_job* jobs, int32_t n_jobs, const msz_options* opt, void* stream);

/* Scratch bytes msz_fix needs for dims d (0 for invalid dims). */
size_t msz_workspace_bytes(msz_dims d);

/* Scratch bytes msz_fix_batch needs for these jobs (0 if any dims are invalid). */
size_t msz_batch_workspace_bytes(const msz_job* jobs, int32_t n_jobs);

/* Number of tile variants selectable through msz_options.tile_override for ndim. */
int msz_tile_variants(int32_t ndim);

/*
 * Lossless encoding of the edits (Sec. 6.3: the edits are stored as key-value
 * pairs; the keys, sorted, as their differences, entropy coded; the values
 * separately).  An edit is an entry of edits[] whose bits are not those of +0
 * (msz_fix leaves +0 at every unedited vertex).  Format (little-endian):
 *   header, 576 bytes: uint32 magic "MSZE" (0x455A534D), version 1, n, m (the
 *     number of edits), chunk count ceil(m / 256), edits per chunk (256);
 *     then the code lengths (uint8) of the 32 gap symbols and of the 512 value
 *     symbols; zero padding;
 *   chunk table: per chunk {uint32 word offset in the bit stream, int32 index
 *     of the chunk's first edit};
 *   bit stream: uint32 words, each chunk starting on its own word.
 * In index order, each edit of a chunk is: for all but the chunk's first, the
 * Huffman code of b = floor(log2(d)), d = index - previous index, then the b
 * low bits of d; then the Huffman code of the edit's 9 high bits (sign and
 * exponent) and its 23 mantissa bits.  Fields are written most significant
 * bit first; emitted bit j of a chunk is bit j % 32 of its word j / 32.  The
 * Huffman codes are canonical (ordered by length, then symbol), at most 20
 * bits long: built by merging the two lightest nodes (ties to the older node;
 * leaves, by symbol, are older than merged nodes), and while a code is too long
 * every count is halved rounding up and the code rebuilt.  Chunks decode
 * independently (one GPU thread each).
 */
typedef struct {
    int64_t n;           /* entries scanned */
    int64_t n_edits;     /* edits found (m) */
    int64_t bytes;       /* encoded size */
    int64_t index_bits;  /* stream bits spent on index gaps */
    int64_t value_bits;  /* stream bits spent on values */
} msz_edit_stats;

/* Upper bound of the encoded size of n entries (0 if n is out of range). */
size_t msz_edits_bound(int64_t n);

/* Encodes the edits of edits[0..n) (DEVICE float32, 16-byte aligned) into out
 * (DEVICE, 16-byte aligned, capacity bytes).  *out_bytes (HOST) receives the
 * encoded size; MSZ_EINVAL if it exceeds capacity (msz_edits_bound(n) always
 * suffices) or if the stream would pass 2^32 words (more than about 1.4e9
 * edits).  stats (HOST) may be NULL.  Allocates its scratch per call
 * (about 12 bytes per entry) on the stream and synchronises before returning. */
int msz_encode_edits(const float* edits, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                     msz_edit_stats* stats, void* stream);

/* Decodes in[0..in_bytes) (DEVICE, 16-byte aligned) into the dense edits_out
 * (DEVICE float32[n], 16-byte aligned; +0 wherever no edit).  MSZ_EINVAL when
 * the header does not match n, or the stream is malformed (a code outside the
 * tables, a read past a chunk, an index outside [0, n)); the decoder never
 * reads or writes outside the given buffers. */
int msz_decode_edits(const void* in, size_t in_bytes, float* edits_out, int64_t n, void* stream);

/* ------------------------------------------------------------------------
 * Learned edit proposal (warm start).  Every edit of the correction loop
 * moves g_i one step down the chain fhat_i, halve(fhat_i), ... towards L_i
 * (Eqs. 2-6), so an edit is a count of halvings.  A 3-layer 3x3x3
 * convolution network (16 -> 16 -> 16 -> 1 channels, ReLU after the two
 * hidden layers, a linear output, zero padding) predicts p, the count of
 * every vertex; the correction loop then starts from g0_i = fhat_i halved
 * k_i times, k_i = floor(fl(p_i - p_min)) + 1 clamped to [0, 64] (0 for a
 * NaN p), and, as always, runs to zero segmentation error within xi.
 * Weights and activations are BF16 (round to nearest even), sums FP32, on
 * MFMA.
 *
 * Parameters: MSZ_NET_PARAMS FP32 values, DEVICE, in this order
 *   W0[27][16][16] b0[16]
 *   W1[27][16][16] b1[16]
 *   W2[27][16]     b2[1]
 * with tap = (dz+1)*9 + (dy+1)*3 + (dx+1) and W[tap][in][out].
 * Features: MSZ_NET_FEATURES BF16 values per vertex, DEVICE, [vertex][16]
 * (box = the 3x3x3 block around the vertex clipped to the grid; every
 * clamp is to [-8, 8]; u ranges over the neighbours of the vertex i):
 *   0  (fhat - mean of fhat over the box) / xi
 *   1  log10(xi / (max f - min f)) / 4 + 1
 *   2..5  false-critical-point flags of fhat against f (FPmax, FPmin, FNmax, FNmin)
 *   6  (fhat - f) / xi
 *   7  (f - mean of f over the box) / xi
 *   8  i = dn_f(u) for an FPmin vertex u      9  i = up_fhat(u) for an FNmax vertex u
 *   10 i = dn_f(u) for a u with dn_fhat(u) != dn_f(u)
 *   11 i = up_fhat(u) for a u with up_fhat(u) != up_f(u)
 *   12..15 zero
 * 2D grids are treated as 3D grids with nz = 1.  All pointers 16-byte aligned.
 * ------------------------------------------------------------------------ */
#define MSZ_NET_PARAMS 14289
#define MSZ_NET_FEATURES 16

/* DEVICE scratch the net entry points need for dims d (0 for invalid dims). */
size_t msz_net_workspace_bytes(msz_dims d);

/* feat[n][16] (BF16 bits) from f, fhat and xi. */
int msz_net_features(const float* f, const float* fhat, msz_dims d, float xi, uint16_t* feat,
                     void* workspace, size_t workspace_bytes, void* stream);

/* p_out[n] = the network's prediction; act1_out / act2_out (optional, [n][16]
 * BF16) receive the two hidden activations. */
int msz_net_forward(const float* params, const uint16_t* feat, msz_dims d, float* p_out,
                    uint16_t* act1_out, uint16_t* act2_out, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Gradient of the weighted mean squared error mean_i w_i (p_i - target_i)^2,
 * w_i = 1 + edit_weight where target_i > 0, else 1, with respect to the
 * parameters (grad_out: DEVICE, MSZ_NET_PARAMS floats, same layout);
 * *loss_out (HOST) receives the loss. */
int msz_net_gradients(const float* params, const uint16_t* feat, const float* target, float edit_weight,
                      msz_dims d, float* grad_out, float* loss_out, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Training target: k_out[i] = the number of halvings that take fhat_i to g_i
 * (L from f and xi as in msz_fix), or -1 where g_i is not on that chain
 * within 256 steps.  All arrays DEVICE, n floats; scratch: n floats. */
int msz_net_halvings(const float* f, const float* fhat, const float* g, msz_dims d, float xi,
                     float* k_out, void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1)
 * on n FP32 parameters with first / second moments m, v (DEVICE). */
int msz_net_adam(float* params, const float* grad, float* m, float* v, int32_t n, int32_t step,
                 float lr, void* stream);

/* Scratch bytes of msz_fix_learned for dims d. */
size_t msz_learned_workspace_bytes(msz_dims d);

/* msz_fix started from the network's warm start (params: DEVICE; p_min: the
 * count threshold, see above, 0.5 rounds p to the nearest count).  opt->warm_start
 * must be NULL; opt->workspace, if given, must hold
 * msz_learned_workspace_bytes(d).  With MSZ_FLAG_TIMING the network's kernels
 * are reported under MSZ_PHASE_NET. */
int msz_fix_learned(const float* f, const float* fhat, msz_dims d, float xi, const float* params,
                    float p_min, float* edits_out, const msz_options* opt, msz_stats* stats,
                    void* stream);

/* Human-readable name of a return code (static string). */
const char* msz_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MSZ_H */
