/*
 * msz_ref.c -- serial CPU oracle for the MSz correction loop (arXiv 2406.09423).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
 * It is deliberately plain and slow: naive neighbour loops, a memoised walk
 * for the labels, one full pass over the grid per detection.  No blocking,
 * fusion or reordering beyond what the definitions state.  The one loop that
 * may run on several threads (option `threads`) is the per-vertex direction
 * loop of the correction loop: every vertex's directions depend only on the
 * field, so the split changes no result; everything else runs serially.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared (no
 * fast-math: the halving chain runs through subnormals, and every float
 * operation must be a single IEEE binary32/binary64 operation with
 * round-to-nearest-even).
 *
 * Readings of the paper that this file fixes (the paper is silent or
 * ambiguous on them) are marked "Reading:".
 */
#include "msz_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 3: PL field on a triangulation).                               */
/* Reading: 2D grids split every quad along its (0,0)-(1,1) diagonal, giving  */
/* the 6 neighbours +-(1,0), +-(0,1), +-(1,1); 3D grids use the Freudenthal  */
/* split of every cube along its (0,0,0)-(1,1,1) diagonal, giving the 14     */
/* neighbours whose offsets have all components in {0,1} or all in {0,-1}.   */
/* Boundaries are not periodic: offsets leaving the grid are dropped.        */
/* ------------------------------------------------------------------------ */
static const int OFFSETS_3D[14][3] = {
    {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},
    {-1, -1, 0}, {1, 0, 1},  {-1, 0, -1}, {0, 1, 1},  {0, -1, -1}, {1, 1, 1},  {-1, -1, -1}};

typedef struct {
    int ndim, nx, ny, nz;
    int64_t n;
} grid_t;

static int make_grid(int ndim, int nx, int ny, int nz, grid_t* gr) {
    if (ndim != 2 && ndim != 3) return MSZ_REF_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return MSZ_REF_EINVAL;
    if (ndim == 2 && nz != 1) return MSZ_REF_EINVAL;
    int64_t n = (int64_t)nx * ny * nz;
    if (n >= ((int64_t)1 << 31)) return MSZ_REF_EINVAL;
    gr->ndim = ndim;
    gr->nx = nx;
    gr->ny = ny;
    gr->nz = nz;
    gr->n = n;
    return MSZ_REF_OK;
}

/* Fill nb[] with the ids of the in-grid neighbours of vertex i; returns their count. */
static int neighbours(const grid_t* gr, int64_t i, int64_t* nb) {
    int64_t x = i % gr->nx;
    int64_t y = (i / gr->nx) % gr->ny;
    int64_t z = i / ((int64_t)gr->nx * gr->ny);
    int cnt = 0;
    for (int k = 0; k < 14; ++k) {
        int dx = OFFSETS_3D[k][0], dy = OFFSETS_3D[k][1], dz = OFFSETS_3D[k][2];
        if (gr->ndim == 2 && dz != 0) continue;
        int64_t xx = x + dx, yy = y + dy, zz = z + dz;
        if (xx < 0 || xx >= gr->nx || yy < 0 || yy >= gr->ny || zz < 0 || zz >= gr->nz) continue;
        nb[cnt++] = xx + gr->nx * (yy + (int64_t)gr->ny * zz);
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Total order (Sec. 4: Morse assumption, ties resolved by simulation of     */
/* simplicity).  Reading: i precedes j iff h_i < h_j, or h_i == h_j and      */
/* i < j (the larger index counts as higher).                                */
/* ------------------------------------------------------------------------ */
static int above(const float* h, int64_t a, int64_t b) { /* a strictly above b */
    if (h[a] > h[b]) return 1;
    if (h[a] < h[b]) return 0;
    return a > b;
}

/* ------------------------------------------------------------------------ */
/* Exact real-number comparisons on float inputs.                            */
/* Knuth's TwoSum gives s + e == a - b exactly (binary64, round to nearest, */
/* no fused operations), so "a - b <= c" can be decided without rounding.   */
/* ------------------------------------------------------------------------ */
static void two_diff(double a, double b, double* s, double* e) {
    double nb = -b;
    double sum = a + nb;
    double bv = sum - a;
    double av = sum - bv;
    *s = sum;
    *e = (a - av) + (nb - bv);
}

/* a - b <= c as real numbers (a, b, c are float32 values). */
static int diff_le(float a, float b, float c) {
    double s, e;
    two_diff((double)a, (double)b, &s, &e);
    if (s < (double)c) return 1;
    if (s > (double)c) return 0;
    return e <= 0.0;
}

/* a - b >= c as real numbers. */
static int diff_ge(float a, float b, float c) {
    double s, e;
    two_diff((double)a, (double)b, &s, &e);
    if (s > (double)c) return 1;
    if (s < (double)c) return 0;
    return e >= 0.0;
}

/* Input magnitudes are limited so that g + L can never overflow float32. */
#define VALUE_LIMIT 1.2676506002282294e30 /* 2^100 */

static int value_ok(float v) { return isfinite(v) && fabs((double)v) <= VALUE_LIMIT; }

/* Eq. 1 bounds every edited value from below by f - xi.  Reading: in float32 the
 * bound is the smallest float L with L >= f - xi, so |f - g| <= xi holds exactly
 * for every g >= L (Problem Statement, global error bound). */
static float lower_bound_one(float f, float xi) {
    float x = (float)((double)f - (double)xi);
    while (!diff_le(f, x, xi)) x = nextafterf(x, INFINITY);            /* need f - x <= xi */
    while (diff_le(f, nextafterf(x, -INFINITY), xi)) x = nextafterf(x, -INFINITY);
    return x;
}

int msz_ref_lower_bound(const float* f, int64_t n, float xi, float* L) {
    if (!f || !L || n < 0) return MSZ_REF_EINVAL;
    for (int64_t i = 0; i < n; ++i) L[i] = lower_bound_one(f[i], xi);
    return MSZ_REF_OK;
}

/* Eqs. 2-6: g <- (g + f - xi) / 2, i.e. halfway to the lower bound.
 * Reading: evaluated as fl32(fl32(g + L) * 0.5); when rounding leaves g
 * unchanged the value snaps to L, so every edit strictly lowers g until g == L. */
float msz_ref_halve(float g, float L) {
    volatile float s = g + L;
    volatile float h = s * 0.5f;
    if (h == g) return L;
    return h;
}

/* ------------------------------------------------------------------------ */
/* Steepest directions (Sec. 3 integral lines; Sec. 6.1 "updating            */
/* directions").  Reading: "steepest" is the highest / lowest neighbour by   */
/* value (the order above), not the slope; a vertex is its own ascent       */
/* (descent) target when it is a maximum (minimum).                          */
/* ------------------------------------------------------------------------ */
static void dirs_of(const float* h, const grid_t* gr, int32_t* up, int32_t* dn, int threads) {
#pragma omp parallel for num_threads(threads > 1 ? threads : 1) schedule(static)
    for (int64_t i = 0; i < gr->n; ++i) {
        int64_t nb[14];
        int64_t u = i, d = i;
        int cnt = neighbours(gr, i, nb);
        for (int k = 0; k < cnt; ++k) {
            if (above(h, nb[k], u)) u = nb[k];
            if (above(h, d, nb[k])) d = nb[k];
        }
        up[i] = (int32_t)u;
        dn[i] = (int32_t)d;
    }
}

int msz_ref_dirs(const float* h, int ndim, int nx, int ny, int nz, int32_t* up, int32_t* dn) {
    grid_t gr;
    int rc = make_grid(ndim, nx, ny, nz, &gr);
    if (rc) return rc;
    if (!h || !up || !dn) return MSZ_REF_EINVAL;
    dirs_of(h, &gr, up, dn, 1);
    return MSZ_REF_OK;
}

/* Segmentation labels (Sec. 3): the extremum an integral line reaches.  A
 * memoised walk: follow the pointers until a vertex with a known label or a
 * fixed point, then label the whole walked path. */
static void follow(const int32_t* ptr, int64_t n, int32_t* lab, int32_t* path) {
    for (int64_t i = 0; i < n; ++i) lab[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (lab[i] >= 0) continue;
        int64_t len = 0;
        int32_t v = (int32_t)i;
        while (lab[v] < 0 && ptr[v] != v) {
            path[len++] = v;
            v = ptr[v];
        }
        int32_t root = lab[v] >= 0 ? lab[v] : v;
        lab[v] = root;
        for (int64_t k = 0; k < len; ++k) lab[path[k]] = root;
    }
}

int msz_ref_labels(const float* h, int ndim, int nx, int ny, int nz, int32_t* max_label,
                   int32_t* min_label) {
    grid_t gr;
    int rc = make_grid(ndim, nx, ny, nz, &gr);
    if (rc) return rc;
    if (!h || !max_label || !min_label) return MSZ_REF_EINVAL;
    int32_t* up = malloc(sizeof(int32_t) * gr.n);
    int32_t* dn = malloc(sizeof(int32_t) * gr.n);
    int32_t* path = malloc(sizeof(int32_t) * gr.n);
    if (!up || !dn || !path) {
        free(up), free(dn), free(path);
        return MSZ_REF_ENOMEM;
    }
    msz_ref_dirs(h, ndim, nx, ny, nz, up, dn);
    follow(up, gr.n, max_label, path);
    follow(dn, gr.n, min_label, path);
    free(up), free(dn), free(path);
    return MSZ_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* False cases.                                                              */
/*  FPmax (Def. 1): maximum in g, not in f.        edit target: the vertex   */
/*  FPmin (Def. 2): minimum in g, not in f.        edit target: see below    */
/*  FNmax (Def. 3): maximum in f, not in g.        edit target: its highest  */
/*                  neighbour in g (Eq. 4)                                   */
/*  FNmin (Def. 3): minimum in f, not in g.        edit target: the vertex   */
/*                  (Eq. 5)                                                  */
/* Reading (FPmin, Eq. 3): the printed rule lowers i's highest neighbour in  */
/* g, which cannot end i's minimality unless that neighbour's floor lies     */
/* below g_i and can stall.  Following Lemma 1, the target is i's descent    */
/* neighbour in f, whose floor is below i's.  The printed rule is kept as an */
/* option (fpmin_literal) to show the stall.                                 */
/* ------------------------------------------------------------------------ */
static int is_case(int type, int64_t i, const int32_t* upf, const int32_t* dnf, const int32_t* upg,
                   const int32_t* dng) {
    switch (type) {
        case MSZ_REF_FPMAX: return upg[i] == i && upf[i] != i;
        case MSZ_REF_FPMIN: return dng[i] == i && dnf[i] != i;
        case MSZ_REF_FNMAX: return upf[i] == i && upg[i] != i;
        default:            return dnf[i] == i && dng[i] != i;
    }
}

static int64_t case_target(int type, int64_t i, const int32_t* dnf, const int32_t* upg, int literal) {
    switch (type) {
        case MSZ_REF_FPMAX: return i;
        case MSZ_REF_FPMIN: return literal ? upg[i] : dnf[i];
        case MSZ_REF_FNMAX: return upg[i];
        default:            return i;
    }
}

/* Sec. 5.2 R-loop.  A vertex u is a troublemaker for minima when its descent in
 * g leaves the descent in f (dn_g(u) != dn_f(u)) while its minimum label is wrong;
 * the first divergence on any mislabelled vertex's integral line is exactly such
 * a vertex.  Reading of Eq. 6's "descending (ascending) neighbour" under
 * value-lowering edits: a wrong minimum is rerouted by lowering dn_f(u), a wrong
 * maximum by lowering up_g(u). */
static int is_rmin(int64_t i, const int32_t* dnf, const int32_t* dng, const int32_t* mf,
                   const int32_t* mg) {
    return dng[i] != dnf[i] && mg[i] != mf[i];
}
static int is_rmax(int64_t i, const int32_t* upf, const int32_t* upg, const int32_t* Mf,
                   const int32_t* Mg) {
    return upg[i] != upf[i] && Mg[i] != Mf[i];
}

int msz_ref_case_flags(const float* f, const float* g, int ndim, int nx, int ny, int nz,
                       uint8_t* flags) {
    grid_t gr;
    int rc = make_grid(ndim, nx, ny, nz, &gr);
    if (rc) return rc;
    if (!f || !g || !flags) return MSZ_REF_EINVAL;
    int64_t n = gr.n;
    int32_t* a = malloc(sizeof(int32_t) * n * 8);
    if (!a) return MSZ_REF_ENOMEM;
    int32_t *upf = a, *dnf = a + n, *upg = a + 2 * n, *dng = a + 3 * n;
    int32_t *Mf = a + 4 * n, *mf = a + 5 * n, *Mg = a + 6 * n, *mg = a + 7 * n;
    msz_ref_dirs(f, ndim, nx, ny, nz, upf, dnf);
    msz_ref_dirs(g, ndim, nx, ny, nz, upg, dng);
    msz_ref_labels(f, ndim, nx, ny, nz, Mf, mf);
    msz_ref_labels(g, ndim, nx, ny, nz, Mg, mg);
    for (int64_t i = 0; i < n; ++i) {
        uint8_t b = 0;
        for (int t = 0; t < 4; ++t)
            if (is_case(t, i, upf, dnf, upg, dng)) b |= (uint8_t)(1u << t);
        if (is_rmin(i, dnf, dng, mf, mg)) b |= 16;
        if (is_rmax(i, upf, upg, Mf, Mg)) b |= 32;
        flags[i] = b;
    }
    free(a);
    return MSZ_REF_OK;
}

int msz_ref_count_false(const float* f, const float* g, int ndim, int nx, int ny, int nz,
                        msz_ref_false_counts* out) {
    grid_t gr;
    int rc = make_grid(ndim, nx, ny, nz, &gr);
    if (rc) return rc;
    if (!f || !g || !out) return MSZ_REF_EINVAL;
    int64_t n = gr.n;
    int32_t* a = malloc(sizeof(int32_t) * n * 8);
    if (!a) return MSZ_REF_ENOMEM;
    int32_t *upf = a, *dnf = a + n, *upg = a + 2 * n, *dng = a + 3 * n;
    int32_t *Mf = a + 4 * n, *mf = a + 5 * n, *Mg = a + 6 * n, *mg = a + 7 * n;
    msz_ref_dirs(f, ndim, nx, ny, nz, upf, dnf);
    msz_ref_dirs(g, ndim, nx, ny, nz, upg, dng);
    msz_ref_labels(f, ndim, nx, ny, nz, Mf, mf);
    msz_ref_labels(g, ndim, nx, ny, nz, Mg, mg);
    memset(out, 0, sizeof(*out));
    for (int64_t i = 0; i < n; ++i) {
        out->fp_max += is_case(MSZ_REF_FPMAX, i, upf, dnf, upg, dng);
        out->fp_min += is_case(MSZ_REF_FPMIN, i, upf, dnf, upg, dng);
        out->fn_max += is_case(MSZ_REF_FNMAX, i, upf, dnf, upg, dng);
        out->fn_min += is_case(MSZ_REF_FNMIN, i, upf, dnf, upg, dng);
        int wM = Mg[i] != Mf[i], wm = mg[i] != mf[i];
        out->wrong_max += wM;
        out->wrong_min += wm;
        out->wrong_any += (wM || wm); /* Appendix B: a vertex is wrong if either label is */
    }
    free(a);
    return MSZ_REF_OK;
}

/* Problem statement: g = fhat + delta.  Reading: delta starts as fl32(g - fhat); when
 * fl32(fhat + delta) misses g (the difference is not representable), the nearest
 * floats up to two ulps either side are tried in the order +1, -1, +2, -2 ulps. */
int msz_ref_delta(float g, float fhat, float* delta) {
    volatile float d0 = g - fhat;
    volatile float r = fhat + d0;
    if (r == g) {
        *delta = d0;
        return 1;
    }
    static const int steps[4] = {1, -1, 2, -2};
    for (int k = 0; k < 4; ++k) {
        float d = d0;
        int s = steps[k];
        for (int j = 0; j < abs(s); ++j) d = nextafterf(d, s > 0 ? INFINITY : -INFINITY);
        volatile float rr = fhat + d;
        if (rr == g) {
            *delta = d;
            return 1;
        }
    }
    *delta = d0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The correction loop (Sec. 5; schedule readings below).                   */
/*  - Every round works on a snapshot of g: the directions of g are computed */
/*    first, then every false case of the current type proposes its target,  */
/*    then each proposed target is halved exactly once.  Proposals for one   */
/*    target from one snapshot are identical, so this is what keeping "the   */
/*    most significant edit" (Sec. 6.1) amounts to.                          */
/*  - C phase (Sec. 5.1): sub-loops FPmax, FPmin, FNmax, FNmin in that order,*/
/*    each repeated until it finds no case of its type; the C phase repeats  */
/*    until no false critical point of any type remains.                     */
/*  - Merged C phase (option merged_c; the parallel C-loop of Sec. 6.1): one */
/*    round finds the false critical points of all four types on the same   */
/*    snapshot and halves the union of their targets once; it repeats until */
/*    no false critical point remains.                                       */
/*  - R phase (Sec. 5.2): one round lowers the targets of both the min and   */
/*    the max troublemakers; after it, if any false critical point appeared, */
/*    control returns to the C phase (Sec. 5.3), else the R phase goes on.   */
/*  - The loop ends when both segmentations of g equal those of f.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    grid_t gr;
    const float* L;
    float* g;
    int32_t *upf, *dnf, *upg, *dng, *Mf, *mf, *Mg, *mg, *path;
    uint8_t* mark;
    int threads;
} loop_t;

static void refresh_dirs(loop_t* s) { dirs_of(s->g, &s->gr, s->upg, s->dng, s->threads); }

static int64_t mark_c_targets(loop_t* s, int type, int literal) {
    int64_t count = 0;
    for (int64_t i = 0; i < s->gr.n; ++i) {
        if (is_case(type, i, s->upf, s->dnf, s->upg, s->dng)) {
            s->mark[case_target(type, i, s->dnf, s->upg, literal)] = 1;
            ++count;
        }
    }
    return count;
}

static int any_c_case(loop_t* s) {
    for (int64_t i = 0; i < s->gr.n; ++i)
        for (int t = 0; t < 4; ++t)
            if (is_case(t, i, s->upf, s->dnf, s->upg, s->dng)) return 1;
    return 0;
}

/* Halve every marked target once; returns how many values changed. */
static int64_t apply_marks(loop_t* s) {
    int64_t changed = 0;
    for (int64_t i = 0; i < s->gr.n; ++i) {
        if (!s->mark[i]) continue;
        float h = msz_ref_halve(s->g[i], s->L[i]);
        if (h != s->g[i]) ++changed;
        s->g[i] = h;
        s->mark[i] = 0;
    }
    return changed;
}

int msz_ref_fix(const float* f, const float* fhat, int ndim, int nx, int ny, int nz, float xi,
                float* edits_out, const msz_ref_options* opt, msz_ref_stats* stats) {
    grid_t gr;
    int rc = make_grid(ndim, nx, ny, nz, &gr);
    if (rc) return rc;
    if (!f || !fhat || !edits_out || !stats) return MSZ_REF_EINVAL;
    memset(stats, 0, sizeof(*stats));
    msz_ref_options o;
    memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    int64_t cap = o.max_rounds > 0 ? o.max_rounds : ((int64_t)1 << 30);
    int64_t n = gr.n;

    /* Input contract (Problem Statement): finite values, |f - fhat| <= xi. */
    if (!value_ok(xi)) return stats->status = MSZ_REF_ENONFINITE;
    if (xi < 0.0f) return stats->status = MSZ_REF_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!value_ok(f[i]) || !value_ok(fhat[i])) return stats->status = MSZ_REF_ENONFINITE;
    for (int64_t i = 0; i < n; ++i)
        if (!diff_le(f[i], fhat[i], xi) || !diff_ge(f[i], fhat[i], -xi))
            return stats->status = MSZ_REF_EBOUND;

    float* L = malloc(sizeof(float) * n);
    float* g = malloc(sizeof(float) * n);
    int32_t* ia = malloc(sizeof(int32_t) * n * 9);
    uint8_t* mark = calloc((size_t)n, 1);
    if (!L || !g || !ia || !mark) {
        free(L), free(g), free(ia), free(mark);
        return stats->status = MSZ_REF_ENOMEM;
    }
    msz_ref_lower_bound(f, n, xi, L);
    int status = MSZ_REF_OK;
    if (o.warm_start) {
        for (int64_t i = 0; i < n; ++i) {
            float w = o.warm_start[i];
            if (!value_ok(w)) {
                status = MSZ_REF_ENONFINITE;
                break;
            }
            if (!(w >= L[i] && w <= fhat[i])) {
                status = MSZ_REF_EBOUND;
                break;
            }
            g[i] = w;
        }
        if (status) {
            free(L), free(g), free(ia), free(mark);
            return stats->status = status;
        }
    } else {
        memcpy(g, fhat, sizeof(float) * n);
    }

    loop_t s;
    s.gr = gr;
    s.L = L;
    s.g = g;
    s.upf = ia, s.dnf = ia + n, s.upg = ia + 2 * n, s.dng = ia + 3 * n;
    s.Mf = ia + 4 * n, s.mf = ia + 5 * n, s.Mg = ia + 6 * n, s.mg = ia + 7 * n;
    s.path = ia + 8 * n;
    s.mark = mark;
    s.threads = o.threads;

    dirs_of(f, &gr, s.upf, s.dnf, s.threads);
    follow(s.upf, n, s.Mf, s.path);
    follow(s.dnf, n, s.mf, s.path);
    refresh_dirs(&s);
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < 4; ++t) stats->false_init[t] += is_case(t, i, s.upf, s.dnf, s.upg, s.dng);
    /* Appendix B: vertices of the start field whose max or min label differs from f's */
    follow(s.upg, n, s.Mg, s.path);
    follow(s.dng, n, s.mg, s.path);
    for (int64_t i = 0; i < n; ++i) stats->mislabel_init += s.Mg[i] != s.Mf[i] || s.mg[i] != s.mf[i];

    int64_t rounds = 0;
    for (;;) {
        /* C phase */
        stats->outer_iters++;
        while (o.merged_c) {
            refresh_dirs(&s);
            int64_t cnt[4], total = 0;
            for (int t = 0; t < 4; ++t) total += cnt[t] = mark_c_targets(&s, t, o.fpmin_literal);
            if (total == 0) break;
            if (rounds >= cap) {
                memset(mark, 0, (size_t)n);
                status = MSZ_REF_ENOCONV;
                goto done;
            }
            if (apply_marks(&s) == 0) {
                status = MSZ_REF_ESTALL;
                goto done;
            }
            ++rounds;
            for (int t = 0; t < 4; ++t) stats->rounds[t] += cnt[t] > 0;
        }
        while (!o.merged_c) {
            for (int t = 0; t < 4; ++t) {
                for (;;) {
                    refresh_dirs(&s);
                    int64_t cnt = mark_c_targets(&s, t, o.fpmin_literal);
                    if (cnt == 0) break;
                    if (rounds >= cap) {
                        memset(mark, 0, (size_t)n);
                        status = MSZ_REF_ENOCONV;
                        goto done;
                    }
                    if (apply_marks(&s) == 0) {
                        status = MSZ_REF_ESTALL;
                        goto done;
                    }
                    ++rounds;
                    stats->rounds[t]++;
                }
            }
            if (!any_c_case(&s)) break; /* directions are current: the last FNmin pass saw g */
        }
        /* R phase */
        for (;;) {
            follow(s.upg, n, s.Mg, s.path);
            follow(s.dng, n, s.mg, s.path);
            int64_t wrong = 0;
            for (int64_t i = 0; i < n; ++i) {
                int rmin = is_rmin(i, s.dnf, s.dng, s.mf, s.mg);
                int rmax = is_rmax(i, s.upf, s.upg, s.Mf, s.Mg);
                if (s.Mg[i] != s.Mf[i] || s.mg[i] != s.mf[i]) ++wrong;
                if (rmin) mark[s.dnf[i]] = 1;
                if (rmax) mark[s.upg[i]] = 1;
            }
            if (wrong == 0) goto done;
            if (rounds >= cap) {
                memset(mark, 0, (size_t)n);
                status = MSZ_REF_ENOCONV;
                goto done;
            }
            if (apply_marks(&s) == 0) {
                status = MSZ_REF_ESTALL;
                goto done;
            }
            ++rounds;
            stats->rounds_r++;
            refresh_dirs(&s);
            if (any_c_case(&s)) break; /* Sec. 5.3: back to the C phase */
        }
    }
done:
    for (int64_t i = 0; i < n; ++i) {
        if (g[i] != fhat[i]) stats->n_edited++;
        if (!msz_ref_delta(g[i], fhat[i], &edits_out[i])) stats->n_inexact++;
    }
    if (o.g_out) memcpy(o.g_out, g, sizeof(float) * n);
    stats->status = status;
    free(L), free(g), free(ia), free(mark);
    return status;
}
