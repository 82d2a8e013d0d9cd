/*
 * Seeded synthetic inputs for the symmetric-SpMM / LOBPCG hot path.
 *
 * This file generates test and benchmark inputs only.  It holds none of the
 * method's arithmetic (no products, no Gram matrices, no eigen-solves); both
 * the FP64 oracle and the HIP path consume what it writes.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to (key, counter).  Every draw is a pure
 * function of (seed, stream, counter), so results do not depend on the
 * number of OpenMP threads.
 *
 * Matrices are returned as the upper triangle of a symmetric H in CSR form,
 * diagonal included, columns ascending within each row, the diagonal first.
 * Three families:
 *   rs    : each row draws `draws` distinct off-diagonal partners uniformly;
 *           pair values N(0,1)*scale are summed into the symmetric position.
 *   tiled : T x T tiles; each tile-row draws `tile_draws` distinct tile
 *           columns; every present tile is filled Bernoulli(p) per entry.
 *   zipf  : full-row degrees L_i = clip(Zipf(a), lmin, lmax); row i draws
 *           ceil(L_i/2) partners with probability proportional to L_j.
 * The diagonal is d = sort(Uniform[0, dmax)), generated as normalised
 * cumulative sums of exponential spacings (the order statistics of n
 * uniforms), which is exact in distribution and O(n).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* ---------------- counter-based generator ---------------- */
static inline uint64_t sm64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline uint64_t rkey(uint64_t seed, uint64_t stream) {
    return sm64(sm64(seed * 0x2545f4914f6cdd1dULL + 0x1234567ULL) ^ sm64(stream + 0x51ed27ULL));
}
static inline uint64_t rbits(uint64_t key, uint64_t ctr) { return sm64(key + ctr * 0x9e3779b97f4a7c15ULL); }
/* uniform in [0,1) */
static inline double u01(uint64_t b) { return (double)(b >> 11) * 0x1.0p-53; }
/* uniform in (0,1] */
static inline double u01_open0(uint64_t b) { return ((double)(b >> 11) + 1.0) * 0x1.0p-53; }
static inline double gauss(uint64_t key, uint64_t ctr) {
    double u1 = u01_open0(rbits(key, 2 * ctr));
    double u2 = u01(rbits(key, 2 * ctr + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

/* ---------------- handle ---------------- */
typedef struct {
    int64_t n, nnz;
    int64_t *row_ptr;   /* n+1 */
    int32_t *col;       /* nnz */
    double *val64;      /* nnz (when !f32) */
    float *val32;       /* nnz (when f32) */
    double *diag;       /* n */
    int f32;
} synth_csr;

int64_t synth_csr_n(const synth_csr *h) { return h->n; }
int64_t synth_csr_nnz(const synth_csr *h) { return h->nnz; }
int64_t *synth_csr_row_ptr(synth_csr *h) { return h->row_ptr; }
int32_t *synth_csr_col(synth_csr *h) { return h->col; }
void *synth_csr_val(synth_csr *h) { return h->f32 ? (void *)h->val32 : (void *)h->val64; }
double *synth_csr_diag(synth_csr *h) { return h->diag; }
int synth_csr_is_f32(const synth_csr *h) { return h->f32; }
void synth_csr_free(synth_csr *h) {
    if (!h) return;
    free(h->row_ptr); free(h->col); free(h->val64); free(h->val32); free(h->diag);
    free(h);
}

/* sorted Uniform[0,dmax) of length n via exponential spacings */
static void sorted_uniform(int64_t n, uint64_t seed, double dmax, double *out) {
    uint64_t key = rkey(seed, 0xd1a9ULL);
    int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt + 1, sizeof(double));
    double total_last = 0.0;
    #pragma omp parallel
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t lo = n * t / T, hi = n * (t + 1) / T;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) { s += -log(u01_open0(rbits(key, (uint64_t)i))); out[i] = s; }
        part[t + 1] = s;
        #pragma omp barrier
        #pragma omp single
        {
            for (int q = 1; q <= T; ++q) part[q] += part[q - 1];
            total_last = part[T] - log(u01_open0(rbits(key, (uint64_t)n)));
        }
        double off = part[t];
        for (int64_t i = lo; i < hi; ++i) out[i] = dmax * (out[i] + off) / total_last;
    }
    free(part);
}

void synth_sorted_uniform(int64_t n, uint64_t seed, double dmax, double *out) { sorted_uniform(n, seed, dmax, out); }

/* n x k row-major block of N(0,1); stream `seed` */
void synth_gaussian_block(int64_t n, int64_t k, uint64_t seed, double *out) {
    uint64_t key = rkey(seed, 0xb10cULL);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n * k; ++i) out[i] = gauss(key, (uint64_t)i);
}
void synth_gaussian_block_f32(int64_t n, int64_t k, uint64_t seed, float *out) {
    uint64_t key = rkey(seed, 0xb10cULL);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n * k; ++i) out[i] = (float)gauss(key, (uint64_t)i);
}

/* ---------------- shared assembly: raw (lo, hi, v) pairs -> CSR ---------------- */
typedef struct { int32_t c; float v32; double v; } ent_t;
/* order by column, ties by value, so that summing repeated pairs is reproducible */
static int ent_cmp(const void *a, const void *b) {
    const ent_t *x = (const ent_t *)a, *y = (const ent_t *)b;
    if (x->c != y->c) return (x->c > y->c) - (x->c < y->c);
    return (x->v > y->v) - (x->v < y->v);
}

/* bucket raw pairs (already counted in cnt[lo]) and assemble the CSR */
typedef void (*pair_emit_fn)(void *ctx, int64_t row, void (*emit)(void *, int64_t, int64_t, double), void *ectx);

typedef struct { int64_t *cursor; int32_t *hi; double *v; } scatter_ctx;
static void emit_count(void *ectx, int64_t lo, int64_t hi, double v) {
    (void)hi; (void)v;
    int64_t *cnt = (int64_t *)ectx;
    #pragma omp atomic
    cnt[lo] += 1;
}
static void emit_scatter(void *ectx, int64_t lo, int64_t hi, double v) {
    scatter_ctx *s = (scatter_ctx *)ectx;
    int64_t pos;
    #pragma omp atomic capture
    pos = s->cursor[lo]++;
    s->hi[pos] = (int32_t)hi;
    s->v[pos] = v;
}

/* stage lines on stderr when SYNTH_PROGRESS is set (large matrices take minutes) */
static void progress(const char *stage, int64_t n, int64_t count) {
    if (!getenv("SYNTH_PROGRESS")) return;
    fprintf(stderr, "[synth] n=%lld: %s (%lld)\n", (long long)n, stage, (long long)count);
    fflush(stderr);
}

/* rows done in a generator pass; a stage line at every tenth of the rows */
static void rows_done(const char *stage, int64_t n, int64_t *done, int64_t add) {
    int64_t before;
    #pragma omp atomic capture
    { before = *done; *done += add; }
    const int64_t step = n / 10 > 0 ? n / 10 : 1;
    if ((before + add) / step != before / step) progress(stage, n, before + add);
}

static synth_csr *assemble(int64_t n, const double *diag, pair_emit_fn gen, void *gctx, int f32) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return NULL;
    int64_t done = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < n; b += 4096) {
        const int64_t e = b + 4096 < n ? b + 4096 : n;
        for (int64_t i = b; i < e; ++i) gen(gctx, i, emit_count, cnt);
        rows_done("counting pairs, rows", n, &done, e - b);
    }
    progress("pairs counted", n, n);
    int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    int64_t raw = off[n];
    scatter_ctx sc;
    sc.cursor = cnt;
    for (int64_t i = 0; i < n; ++i) cnt[i] = off[i];
    sc.hi = (int32_t *)malloc((size_t)(raw ? raw : 1) * sizeof(int32_t));
    sc.v = (double *)malloc((size_t)(raw ? raw : 1) * sizeof(double));
    if (!sc.hi || !sc.v) { free(cnt); free(off); free(sc.hi); free(sc.v); return NULL; }
    done = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < n; b += 4096) {
        const int64_t e = b + 4096 < n ? b + 4096 : n;
        for (int64_t i = b; i < e; ++i) gen(gctx, i, emit_scatter, &sc);
        rows_done("placing pairs, rows", n, &done, e - b);
    }
    progress("pairs placed", n, raw);
    /* sort each bucket by column, merge duplicate pairs by summation */
    int64_t *fcnt = cnt; /* reuse: final off-diagonal count per row */
    done = 0;
    #pragma omp parallel
    {
        size_t cap = 0; ent_t *buf = NULL;
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if ((i & 4095) == 4095) rows_done("sorting rows", n, &done, 4096);
            int64_t b = off[i], e = off[i + 1], m = e - b;
            if ((size_t)m > cap) { cap = (size_t)m * 2; buf = (ent_t *)realloc(buf, cap * sizeof(ent_t)); }
            for (int64_t q = 0; q < m; ++q) { buf[q].c = sc.hi[b + q]; buf[q].v = sc.v[b + q]; }
            qsort(buf, (size_t)m, sizeof(ent_t), ent_cmp);
            int64_t w = 0;
            for (int64_t q = 0; q < m; ++q) {
                if (w > 0 && buf[w - 1].c == buf[q].c) {
                    buf[w - 1].v += buf[q].v;
                } else buf[w++] = buf[q];
            }
            for (int64_t q = 0; q < w; ++q) { sc.hi[b + q] = buf[q].c; sc.v[b + q] = buf[q].v; }
            fcnt[i] = w;
        }
        free(buf);
    }
    progress("rows sorted and merged", n, n);
    synth_csr *h = (synth_csr *)calloc(1, sizeof(synth_csr));
    h->n = n; h->f32 = f32;
    h->row_ptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    h->row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) h->row_ptr[i + 1] = h->row_ptr[i] + 1 + fcnt[i];
    h->nnz = h->row_ptr[n];
    h->col = (int32_t *)malloc((size_t)h->nnz * sizeof(int32_t));
    if (f32) h->val32 = (float *)malloc((size_t)h->nnz * sizeof(float));
    else h->val64 = (double *)malloc((size_t)h->nnz * sizeof(double));
    h->diag = (double *)malloc((size_t)n * sizeof(double));
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = h->row_ptr[i];
        double dv = diag[i];
        if (f32) dv = (double)(float)dv;
        h->diag[i] = dv;
        h->col[p] = (int32_t)i;
        if (f32) h->val32[p] = (float)dv; else h->val64[p] = dv;
        for (int64_t q = 0; q < fcnt[i]; ++q) {
            h->col[p + 1 + q] = sc.hi[off[i] + q];
            if (f32) h->val32[p + 1 + q] = (float)sc.v[off[i] + q];
            else h->val64[p + 1 + q] = sc.v[off[i] + q];
        }
    }
    free(cnt); free(off); free(sc.hi); free(sc.v);
    progress("CSR built", n, h->nnz);
    return h;
}

/* ---------------- family rs ---------------- */
typedef struct { int64_t n, draws; uint64_t key; double scale; } rs_ctx;

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* row i draws `draws` distinct partners j != i; returns them in draw order */
static void rs_row_partners(const rs_ctx *c, int64_t i, int64_t *js, int64_t *tmp) {
    uint64_t rk = rbits(c->key, (uint64_t)i);
    uint64_t ctr = 0;
    int64_t m = c->draws, have = 0;
    while (have < m) {
        for (int64_t q = have; q < m; ++q) {
            int64_t j = (int64_t)(u01(rbits(rk, ctr++)) * (double)(c->n - 1));
            if (j >= c->n - 1) j = c->n - 2;
            if (j >= i) j += 1;
            js[q] = j;
        }
        /* drop repeats, keeping first occurrence in draw order */
        memcpy(tmp, js, (size_t)m * sizeof(int64_t));
        qsort(tmp, (size_t)m, sizeof(int64_t), cmp_i64);
        int dup = 0;
        for (int64_t q = 1; q < m; ++q) if (tmp[q] == tmp[q - 1]) { dup = 1; break; }
        if (!dup) { have = m; break; }
        int64_t w = 0;
        for (int64_t q = 0; q < m; ++q) {
            int seen = 0;
            for (int64_t r = 0; r < w; ++r) if (js[r] == js[q]) { seen = 1; break; }
            if (!seen) js[w++] = js[q];
        }
        have = w;
    }
}

static void rs_gen(void *gctx, int64_t i, void (*emit)(void *, int64_t, int64_t, double), void *ectx) {
    const rs_ctx *c = (const rs_ctx *)gctx;
    int64_t stackj[512], stackt[512];
    int64_t *js = c->draws <= 512 ? stackj : (int64_t *)malloc((size_t)c->draws * sizeof(int64_t));
    int64_t *tmp = c->draws <= 512 ? stackt : (int64_t *)malloc((size_t)c->draws * sizeof(int64_t));
    rs_row_partners(c, i, js, tmp);
    uint64_t vk = rbits(c->key ^ 0x5bd1e995ULL, (uint64_t)i);
    for (int64_t q = 0; q < c->draws; ++q) {
        double v = gauss(vk, (uint64_t)q) * c->scale;
        int64_t j = js[q];
        if (j < i) emit(ectx, j, i, v); else emit(ectx, i, j, v);
    }
    if (js != stackj) { free(js); free(tmp); }
}

synth_csr *synth_rs(int64_t n, int64_t draws, uint64_t seed, double dmax, double scale, int f32) {
    if (n < 2 || draws < 0 || draws > n - 1) return NULL;
    double *d = (double *)malloc((size_t)n * sizeof(double));
    sorted_uniform(n, seed, dmax, d);
    rs_ctx c = { n, draws, rkey(seed, 0x7273ULL), scale };
    synth_csr *h = assemble(n, d, rs_gen, &c, f32);
    free(d);
    return h;
}

/* ---------------- family zipf ---------------- */
typedef struct {
    int64_t n; uint64_t key; double scale;
    const int32_t *deg;       /* full-row degree target per row */
    const double *cum;        /* cumulative degree weights, n+1 */
} zipf_ctx;

static int64_t pick_weighted(const double *cum, int64_t n, double u) {
    double t = u * cum[n];
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (cum[mid + 1] > t) hi = mid; else lo = mid + 1; }
    return lo;
}

static void zipf_gen(void *gctx, int64_t i, void (*emit)(void *, int64_t, int64_t, double), void *ectx) {
    const zipf_ctx *c = (const zipf_ctx *)gctx;
    int64_t m = (c->deg[i] + 1) / 2;
    uint64_t rk = rbits(c->key, (uint64_t)i);
    uint64_t vk = rbits(c->key ^ 0x5bd1e995ULL, (uint64_t)i);
    int64_t stackj[1024];
    int64_t *js = m <= 1024 ? stackj : (int64_t *)malloc((size_t)m * sizeof(int64_t));
    uint64_t ctr = 0;
    int64_t have = 0;
    while (have < m) {
        int64_t j = pick_weighted(c->cum, c->n, u01(rbits(rk, ctr++)));
        if (j == i) continue;
        int seen = 0;
        /* small rows: linear check; hub rows: accept repeats as summed duplicates */
        if (m <= 64) for (int64_t r = 0; r < have; ++r) if (js[r] == j) { seen = 1; break; }
        if (seen) continue;
        js[have++] = j;
        if (ctr > (uint64_t)(64 * m + 1024)) break;
    }
    for (int64_t q = 0; q < have; ++q) {
        double v = gauss(vk, (uint64_t)q) * c->scale;
        int64_t j = js[q];
        if (j < i) emit(ectx, j, i, v); else emit(ectx, i, j, v);
    }
    if (js != stackj) free(js);
}

synth_csr *synth_zipf(int64_t n, double a, int64_t lmin, int64_t lmax, uint64_t seed, double dmax,
                      double scale, int f32) {
    if (n < 2 || a <= 1.0 || lmin < 1 || lmax < lmin) return NULL;
    int32_t *deg = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint64_t dk = rkey(seed, 0x21f5ULL);
    /* Zipf(a) by rejection (Devroye, Non-Uniform Random Variate Generation, X.6.1) */
    double b = pow(2.0, a - 1.0);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr = 0;
        double x;
        for (;;) {
            double u = 1.0 - u01(rbits(dk, ((uint64_t)i << 8) + ctr++));
            double v = u01(rbits(dk, ((uint64_t)i << 8) + ctr++));
            x = floor(pow(u, -1.0 / (a - 1.0)));
            if (x > 1e12) continue;
            double t = pow(1.0 + 1.0 / x, a - 1.0);
            if (v * x * (t - 1.0) / (b - 1.0) <= t / b) break;
        }
        if (x < (double)lmin) x = (double)lmin;
        if (x > (double)lmax) x = (double)lmax;
        if (x > (double)(n - 1)) x = (double)(n - 1);
        deg[i] = (int32_t)x;
    }
    double *cum = (double *)malloc(((size_t)n + 1) * sizeof(double));
    cum[0] = 0.0;
    for (int64_t i = 0; i < n; ++i) cum[i + 1] = cum[i] + (double)deg[i];
    double *d = (double *)malloc((size_t)n * sizeof(double));
    sorted_uniform(n, seed, dmax, d);
    zipf_ctx c = { n, rkey(seed, 0x7a69ULL), scale, deg, cum };
    synth_csr *h = assemble(n, d, zipf_gen, &c, f32);
    free(d); free(cum); free(deg);
    return h;
}

/* ---------------- family tiled ---------------- */
/* tile-row I draws `tile_draws` distinct tile columns J != I; the pattern is
   symmetric: a tile (lo, hi) is present when either end drew the other. */
static int32_t *tiled_pattern(int64_t nt, int64_t tile_draws, uint64_t seed, int64_t **tptr_out) {
    rs_ctx c = { nt, tile_draws, rkey(seed, 0x7469ULL), 0.0 };
    int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    #pragma omp parallel
    {
        int64_t *js = (int64_t *)malloc((size_t)(tile_draws + 1) * sizeof(int64_t));
        int64_t *tmp = (int64_t *)malloc((size_t)(tile_draws + 1) * sizeof(int64_t));
        #pragma omp for schedule(static)
        for (int64_t I = 0; I < nt; ++I) {
            rs_row_partners(&c, I, js, tmp);
            for (int64_t q = 0; q < tile_draws; ++q) {
                int64_t lo = js[q] < I ? js[q] : I;
                #pragma omp atomic
                cnt[lo] += 1;
            }
        }
        free(js); free(tmp);
    }
    int64_t *off = (int64_t *)malloc(((size_t)nt + 1) * sizeof(int64_t));
    off[0] = 0;
    for (int64_t I = 0; I < nt; ++I) off[I + 1] = off[I] + cnt[I];
    for (int64_t I = 0; I < nt; ++I) cnt[I] = off[I];
    int32_t *hi = (int32_t *)malloc((size_t)(off[nt] ? off[nt] : 1) * sizeof(int32_t));
    #pragma omp parallel
    {
        int64_t *js = (int64_t *)malloc((size_t)(tile_draws + 1) * sizeof(int64_t));
        int64_t *tmp = (int64_t *)malloc((size_t)(tile_draws + 1) * sizeof(int64_t));
        #pragma omp for schedule(static)
        for (int64_t I = 0; I < nt; ++I) {
            rs_row_partners(&c, I, js, tmp);
            for (int64_t q = 0; q < tile_draws; ++q) {
                int64_t lo = js[q] < I ? js[q] : I, h = js[q] < I ? I : js[q];
                int64_t pos;
                #pragma omp atomic capture
                pos = cnt[lo]++;
                hi[pos] = (int32_t)h;
            }
        }
        free(js); free(tmp);
    }
    /* sort + dedupe per tile-row */
    int64_t *fc = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    #pragma omp parallel
    {
        int64_t cap = 0; int64_t *b64 = NULL;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t I = 0; I < nt; ++I) {
            int64_t b = off[I], m = off[I + 1] - b;
            if (m > cap) { cap = 2 * m; b64 = (int64_t *)realloc(b64, (size_t)cap * sizeof(int64_t)); }
            for (int64_t q = 0; q < m; ++q) b64[q] = hi[b + q];
            qsort(b64, (size_t)m, sizeof(int64_t), cmp_i64);
            int64_t w = 0;
            for (int64_t q = 0; q < m; ++q) if (w == 0 || b64[w - 1] != b64[q]) b64[w++] = b64[q];
            for (int64_t q = 0; q < w; ++q) hi[b + q] = (int32_t)b64[q];
            fc[I] = w;
        }
        free(b64);
    }
    int64_t *tptr = (int64_t *)malloc(((size_t)nt + 1) * sizeof(int64_t));
    tptr[0] = 0;
    for (int64_t I = 0; I < nt; ++I) tptr[I + 1] = tptr[I] + fc[I];
    int32_t *tj = (int32_t *)malloc((size_t)(tptr[nt] ? tptr[nt] : 1) * sizeof(int32_t));
    for (int64_t I = 0; I < nt; ++I) memcpy(tj + tptr[I], hi + off[I], (size_t)fc[I] * sizeof(int32_t));
    free(cnt); free(off); free(hi); free(fc);
    *tptr_out = tptr;
    return tj;
}

/* Bernoulli(p) positions in [c0, T) of one tile row, by geometric skipping */
static inline int tile_row_positions(uint64_t rk, int c0, int T, double lq, int *pos) {
    int m = 0; uint64_t ctr = 0;
    int c = c0 - 1;
    for (;;) {
        double u = u01_open0(rbits(rk, ctr++));
        double g = floor(log(u) / lq);
        if (g > (double)T) break;
        c += 1 + (int)g;
        if (c >= T) break;
        pos[m++] = c;
    }
    return m;
}

synth_csr *synth_tiled(int64_t n, int64_t T, int64_t tile_draws, double p, uint64_t seed, double dmax,
                       double scale, int f32) {
    if (T < 1 || T > 4096 || n % T != 0 || n / T < 2 || p <= 0.0 || p >= 1.0) return NULL;
    int64_t nt = n / T;
    if (tile_draws > nt - 1) return NULL;
    int64_t *tptr = NULL;
    int32_t *tj = tiled_pattern(nt, tile_draws, seed, &tptr);
    double *d = (double *)malloc((size_t)n * sizeof(double));
    sorted_uniform(n, seed, dmax, d);
    double lq = log1p(-p);
    uint64_t pk = rkey(seed, 0x9057ULL), vk = rkey(seed, 0x7661ULL);
    synth_csr *h = (synth_csr *)calloc(1, sizeof(synth_csr));
    h->n = n; h->f32 = f32;
    h->row_ptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *rc = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    /* pass 1: count per row */
    #pragma omp parallel
    {
        int *pos = (int *)malloc((size_t)T * sizeof(int));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t I = 0; I < nt; ++I) {
            for (int64_t r = 0; r < T; ++r) {
                int64_t i = I * T + r, cnt = 1;
                /* diagonal tile: strict upper part */
                cnt += tile_row_positions(rbits(pk, (uint64_t)((I * nt + I) * T + r)), (int)r + 1, (int)T, lq, pos);
                for (int64_t q = tptr[I]; q < tptr[I + 1]; ++q) {
                    int64_t J = tj[q];
                    cnt += tile_row_positions(rbits(pk, (uint64_t)((I * nt + J) * T + r)), 0, (int)T, lq, pos);
                }
                rc[i] = cnt;
            }
        }
        free(pos);
    }
    h->row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) h->row_ptr[i + 1] = h->row_ptr[i] + rc[i];
    h->nnz = h->row_ptr[n];
    h->col = (int32_t *)malloc((size_t)h->nnz * sizeof(int32_t));
    if (f32) h->val32 = (float *)malloc((size_t)h->nnz * sizeof(float));
    else h->val64 = (double *)malloc((size_t)h->nnz * sizeof(double));
    h->diag = (double *)malloc((size_t)n * sizeof(double));
    /* pass 2: fill */
    #pragma omp parallel
    {
        int *pos = (int *)malloc((size_t)T * sizeof(int));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t I = 0; I < nt; ++I) {
            for (int64_t r = 0; r < T; ++r) {
                int64_t i = I * T + r, p0 = h->row_ptr[i];
                double dv = f32 ? (double)(float)d[i] : d[i];
                h->diag[i] = dv;
                h->col[p0] = (int32_t)i;
                if (f32) h->val32[p0] = (float)dv; else h->val64[p0] = dv;
                int64_t w = p0 + 1;
                for (int64_t q = tptr[I] - 1; q < tptr[I + 1]; ++q) {
                    int64_t J = q < tptr[I] ? I : tj[q];
                    uint64_t tid = (uint64_t)((I * nt + J) * T + r);
                    int m = tile_row_positions(rbits(pk, tid), J == I ? (int)r + 1 : 0, (int)T, lq, pos);
                    uint64_t vrk = rbits(vk, tid);
                    for (int e = 0; e < m; ++e) {
                        double v = gauss(vrk, (uint64_t)pos[e]) * scale;
                        h->col[w] = (int32_t)(J * T + pos[e]);
                        if (f32) h->val32[w] = (float)v; else h->val64[w] = v;
                        ++w;
                    }
                }
            }
        }
        free(pos);
    }
    free(rc); free(d); free(tptr); free(tj);
    return h;
}
