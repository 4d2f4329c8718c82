/*
 * msz_ref.h -- serial CPU oracle for the MSz correction loop.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no source with the GPU library.
 *
 * Paper: "MSz: An Efficient Parallel Algorithm for Correcting Morse-Smale
 * Segmentations in Error-Bounded Lossy Compressors" (arXiv 2406.09423).
 * Every entry point cites the section / equation / definition it follows.
 *
 * All pointers are HOST pointers owned by the caller.  Grids are row-major
 * with x fastest: vertex id i = x + nx*(y + ny*z).  ndim is 2 or 3; for
 * ndim == 2, nz must be 1.  n = nx*ny*nz must be < 2^31.
 */
#ifndef MSZ_REF_H
#define MSZ_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes (same numeric meaning as the GPU library's). */
#define MSZ_REF_OK          0
#define MSZ_REF_EINVAL     -1   /* bad dims / pointer / option */
#define MSZ_REF_ENONFINITE -2   /* NaN or Inf in f, fhat or xi, or |value| too large */
#define MSZ_REF_EBOUND     -3   /* |f - fhat| > xi, or warm start outside [L, fhat] */
#define MSZ_REF_ESTALL     -4   /* a round had targets but changed no value */
#define MSZ_REF_ENOCONV    -5   /* round cap reached */
#define MSZ_REF_ENOMEM     -7

/* False-case types of the C-loop sub-loops (Sec. 5.1, in the order they run). */
#define MSZ_REF_FPMAX 0
#define MSZ_REF_FPMIN 1
#define MSZ_REF_FNMAX 2
#define MSZ_REF_FNMIN 3

typedef struct {
    int64_t max_rounds;        /* productive rounds allowed (<=0: 1<<30) */
    const float* warm_start;   /* optional start field g0 with L <= g0 <= fhat */
    float* g_out;              /* optional: receives the edited field g */
    int32_t fpmin_literal;     /* 1: FPmin lowers the highest neighbour (literal Eq. 3); test use */
    int32_t merged_c;          /* 1: each C round fixes the cases of all four types at once (Sec. 6.1) */
    int32_t threads;           /* threads of the per-vertex direction loop (<= 1: serial); results
                                  do not depend on it */
    int32_t pad;
} msz_ref_options;

typedef struct {
    int64_t rounds[4];      /* productive rounds of each C sub-loop type (merged_c: the C rounds
                               in which that type had a case) */
    int64_t rounds_r;       /* productive R-loop rounds */
    int64_t outer_iters;    /* number of times the C phase was entered */
    int64_t n_edited;       /* vertices whose final g differs from fhat */
    int64_t false_init[4];  /* false critical points of each type in the start field */
    int64_t mislabel_init;  /* vertices of the start field with a wrong max or min label */
    int64_t n_inexact;      /* vertices where no float delta reproduces g exactly */
    int32_t status;
    int32_t pad;
} msz_ref_stats;

typedef struct {
    int64_t fp_max, fp_min, fn_max, fn_min;
    int64_t wrong_max, wrong_min, wrong_any;
} msz_ref_false_counts;

/* Lower bound L_i = smallest float32 >= f_i - xi (exact real comparison). */
int msz_ref_lower_bound(const float* f, int64_t n, float xi, float* L);

/* One decreasing edit: (g + L)/2 in float32, snapped to L when it makes no progress. */
float msz_ref_halve(float g, float L);

/* Steepest ascent/descent neighbour ids (self when critical). */
int msz_ref_dirs(const float* h, int ndim, int nx, int ny, int nz, int32_t* up, int32_t* dn);

/* Ascending (max) and descending (min) segmentation labels = extremum vertex ids. */
int msz_ref_labels(const float* h, int ndim, int nx, int ny, int nz, int32_t* max_label, int32_t* min_label);

/* False critical points and mislabelled vertices of g with respect to f. */
int msz_ref_count_false(const float* f, const float* g, int ndim, int nx, int ny, int nz,
                        msz_ref_false_counts* out);

/* delta such that fl32(fhat + delta) == g when some float achieves it. Returns 1 if exact. */
int msz_ref_delta(float g, float fhat, float* delta);

/* The full correction loop (Sec. 5, synchronous-round schedule). */
int msz_ref_fix(const float* f, const float* fhat, int ndim, int nx, int ny, int nz, float xi,
                float* edits_out, const msz_ref_options* opt, msz_ref_stats* stats);

/* Per-vertex flags of the four C-loop predicates and the two R-loop predicates for (f, g):
 * bit t (t = 0..3) set when vertex i is a false case of C type t, bit 4: R-min, bit 5: R-max. */
int msz_ref_case_flags(const float* f, const float* g, int ndim, int nx, int ny, int nz, uint8_t* flags);

#ifdef __cplusplus
}
#endif
#endif
