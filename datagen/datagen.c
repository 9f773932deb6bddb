/*
 * Seeded synthetic column generators: the inputs of every test and benchmark.
 *
 * This module produces data and nothing else.  It holds none of the
 * aggregation arithmetic (no sums, minima or maxima of columns), so the GPU
 * library and the CPU oracle can both take their inputs from it without
 * sharing any of the method.
 *
 * Randomness is counter based: element i of a column is a pure function of
 * (seed, i), so a column can be produced in any number of threads and comes
 * out identical.  The stream is SplitMix64 (G. L. Steele, D. Lea and
 * C. H. Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * evaluated at counter values: the state for counter c is key + c * gamma and
 * the output is the published 64-bit finaliser of that state.
 *
 * Distributions (the workload shapes of the paper's key column and of the
 * precision study):
 *   DG_UNIFORM          ints uniform in [lo, hi); with lo == hi == 0 the
 *                       default range per type: i32 [-2^20, 2^20),
 *                       i64 [-2^32, 2^32), f32 k/8 - 2^20 for k uniform in
 *                       [0, 2^24) (exactly representable values);
 *   DG_ZIPF             bounded Zipf, rank k in [1, 2^20] with
 *                       P(k) proportional to k^-1.1, value = k;
 *   DG_SORTED           the DG_UNIFORM column of the same seed, sorted
 *                       ascending (a permutation of it);
 *   DG_NORMAL_OUTLIERS  f32: with probability 1/100 the value is +-1e6 with
 *                       a fair sign, otherwise N(0,1) by the Box-Muller
 *                       transform in double precision, rounded to float.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { DG_I32 = 0, DG_I64 = 1, DG_F32 = 2 };
enum { DG_UNIFORM = 0, DG_ZIPF = 1, DG_SORTED = 2, DG_NORMAL_OUTLIERS = 3 };

#define DG_OK 0
#define DG_EINVAL -1
#define DG_ENOMEM -2

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Output number `ctr` of the SplitMix64 stream whose key is `key`. */
static inline uint64_t sm64_at(uint64_t key, uint64_t ctr) {
    return sm64_mix(key + (ctr + 1) * GOLDEN_GAMMA);
}

/* Independent stream keys derived from the user seed. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed ^ sm64_mix(stream * GOLDEN_GAMMA + 0x5851F42D4C957F2DULL));
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* Integer uniform in [0, span) by the multiply-shift map (span < 2^63). */
static inline uint64_t below(uint64_t r, uint64_t span) {
    return (uint64_t)(((unsigned __int128)r * span) >> 64);
}

/* ------------------------------------------------------------------ */
/* Bounded Zipf(1.1) on ranks [1, 2^20]: inverse CDF with a guide table. */

#define ZIPF_K (1 << 20)
#define ZIPF_S 1.1
#define ZIPF_GUIDE (1 << 20)

typedef struct {
    double* cdf;      /* cdf[k] = P(rank <= k + 1), cdf[ZIPF_K - 1] == 1 */
    int32_t* guide;   /* guide[g] = first k with cdf[k] > g / ZIPF_GUIDE */
} zipf_table;

static int zipf_build(zipf_table* z) {
    z->cdf = (double*)malloc(sizeof(double) * ZIPF_K);
    z->guide = (int32_t*)malloc(sizeof(int32_t) * ZIPF_GUIDE);
    if (!z->cdf || !z->guide) { free(z->cdf); free(z->guide); return DG_ENOMEM; }
    double acc = 0.0;
    for (int k = 0; k < ZIPF_K; ++k) { acc += pow((double)(k + 1), -ZIPF_S); z->cdf[k] = acc; }
    for (int k = 0; k < ZIPF_K; ++k) z->cdf[k] /= acc;
    z->cdf[ZIPF_K - 1] = 1.0;
    int k = 0;
    for (int g = 0; g < ZIPF_GUIDE; ++g) {
        double t = (double)g / (double)ZIPF_GUIDE;
        while (z->cdf[k] <= t) ++k;
        z->guide[g] = k;
    }
    return DG_OK;
}

static inline int64_t zipf_draw(const zipf_table* z, uint64_t r) {
    double u = u01(r);
    int64_t k = z->guide[(int64_t)(u * ZIPF_GUIDE)];
    while (z->cdf[k] <= u) ++k;
    return k + 1;
}

/* ------------------------------------------------------------------ */

typedef struct {
    void* out;
    int64_t lo_i, hi_i;      /* element range of this thread */
    int dtype, dist;
    uint64_t seed;
    int64_t lo, hi;          /* value range for DG_UNIFORM ints */
    const zipf_table* zipf;
} fill_job;

static void* fill_worker(void* arg) {
    fill_job* j = (fill_job*)arg;
    const uint64_t k0 = stream_key(j->seed, 0);
    const uint64_t k1 = stream_key(j->seed, 1);
    const uint64_t k2 = stream_key(j->seed, 2);
    int32_t* o32 = (int32_t*)j->out;
    int64_t* o64 = (int64_t*)j->out;
    float* of = (float*)j->out;
    for (int64_t i = j->lo_i; i < j->hi_i; ++i) {
        uint64_t r = sm64_at(k0, (uint64_t)i);
        if (j->dist == DG_UNIFORM) {
            if (j->dtype == DG_F32) {
                uint64_t k = r >> 40; /* 24 bits */
                of[i] = (float)((double)k * 0.125 - 1048576.0);
            } else if (j->lo == 0 && j->hi == 0) {
                if (j->dtype == DG_I32) o32[i] = (int32_t)((int64_t)(r >> 43) - (1LL << 20));
                else o64[i] = (int64_t)(r >> 31) - (1LL << 32);
            } else {
                int64_t v = j->lo + (int64_t)below(r, (uint64_t)(j->hi - j->lo));
                if (j->dtype == DG_I32) o32[i] = (int32_t)v; else o64[i] = v;
            }
        } else if (j->dist == DG_ZIPF) {
            int64_t k = zipf_draw(j->zipf, r);
            if (j->dtype == DG_I32) o32[i] = (int32_t)k;
            else if (j->dtype == DG_I64) o64[i] = k;
            else of[i] = (float)k;
        } else { /* DG_NORMAL_OUTLIERS, f32 only */
            if ((r >> 11) < (uint64_t)(0.01 * 9007199254740992.0)) {
                of[i] = (r & 1) ? -1.0e6f : 1.0e6f;
            } else {
                double u1 = 1.0 - u01(sm64_at(k1, (uint64_t)i)); /* (0, 1] */
                double u2 = u01(sm64_at(k2, (uint64_t)i));
                double zv = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                of[i] = (float)zv;
            }
        }
    }
    return NULL;
}

static int run_threads(void* (*fn)(void*), void* jobs, size_t job_size, int nt) {
    pthread_t th[256];
    for (int t = 0; t < nt; ++t)
        if (pthread_create(&th[t], NULL, fn, (char*)jobs + job_size * t)) {
            for (int u = 0; u < t; ++u) pthread_join(th[u], NULL);
            return DG_ENOMEM;
        }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return DG_OK;
}

/* ------------------------------------------------------------------ */
/* Sorting for DG_SORTED: a parallel LSD radix sort (11-bit digits) on an
 * unsigned key that is a monotone function of the value:
 * ints key = value - keybase; f32 (1/8 grid of [-2^20, 2^20)) key = 8x + 2^23. */

typedef struct {
    const void* in; void* out;
    int64_t lo_i, hi_i;
    int dtype;
    int shift;            /* radix pass: digit = (key >> shift) & 2047 */
    int64_t* hist;        /* per-thread histogram, 2048 entries */
    int64_t* pos;         /* per-thread scatter positions */
    int64_t keybase;
} radix_job;

static inline uint64_t radix_key(const void* a, int dtype, int64_t i, int64_t keybase) {
    if (dtype == DG_I32) return (uint64_t)((int64_t)((const int32_t*)a)[i] - keybase);
    if (dtype == DG_I64) return (uint64_t)(((const int64_t*)a)[i] - keybase);
    return (uint64_t)(((double)((const float*)a)[i] + 1048576.0) * 8.0);
}

static void* radix_hist_worker(void* arg) {
    radix_job* j = (radix_job*)arg;
    memset(j->hist, 0, sizeof(int64_t) * 2048);
    for (int64_t i = j->lo_i; i < j->hi_i; ++i)
        j->hist[(radix_key(j->in, j->dtype, i, j->keybase) >> j->shift) & 2047]++;
    return NULL;
}

static void* radix_scatter_worker(void* arg) {
    radix_job* j = (radix_job*)arg;
    for (int64_t i = j->lo_i; i < j->hi_i; ++i) {
        uint64_t d = (radix_key(j->in, j->dtype, i, j->keybase) >> j->shift) & 2047;
        int64_t p = j->pos[d]++;
        if (j->dtype == DG_I64) ((int64_t*)j->out)[p] = ((const int64_t*)j->in)[i];
        else ((int32_t*)j->out)[p] = ((const int32_t*)j->in)[i]; /* 4-byte copy (i32 / f32) */
    }
    return NULL;
}

static int radix_sort(void* a, int64_t n, int dtype, int64_t keybase, int key_bits, int nt) {
    size_t w = dtype == DG_I64 ? 8 : 4;
    void* tmp = malloc((size_t)n * w);
    int64_t* hist = (int64_t*)malloc(sizeof(int64_t) * 2048 * (size_t)nt * 2);
    radix_job* jobs = (radix_job*)calloc((size_t)nt, sizeof(radix_job));
    if (!tmp || !hist || !jobs) { free(tmp); free(hist); free(jobs); return DG_ENOMEM; }
    void* src = a; void* dst = tmp;
    int passes = (key_bits + 10) / 11;
    int rc = DG_OK;
    for (int p = 0; p < passes && rc == DG_OK; ++p) {
        for (int t = 0; t < nt; ++t) {
            jobs[t].in = src; jobs[t].out = dst; jobs[t].dtype = dtype;
            jobs[t].lo_i = n * t / nt; jobs[t].hi_i = n * (t + 1) / nt;
            jobs[t].shift = 11 * p; jobs[t].keybase = keybase;
            jobs[t].hist = hist + 2048 * t; jobs[t].pos = hist + 2048 * (nt + t);
        }
        rc = run_threads(radix_hist_worker, jobs, sizeof(radix_job), nt);
        if (rc != DG_OK) break;
        int64_t off = 0;
        for (int d = 0; d < 2048; ++d)
            for (int t = 0; t < nt; ++t) { jobs[t].pos[d] = off; off += jobs[t].hist[d]; }
        rc = run_threads(radix_scatter_worker, jobs, sizeof(radix_job), nt);
        void* s = src; src = dst; dst = s;
    }
    if (rc == DG_OK && src != a) memcpy(a, src, (size_t)n * w);
    free(tmp); free(hist); free(jobs);
    return rc;
}

/* ------------------------------------------------------------------ */

/* Fill out[0..n) with column `dist` of type `dtype` from `seed`.
 * lo/hi: value range [lo, hi) for integer DG_UNIFORM / DG_SORTED
 * (0, 0 = default range).  nthreads <= 0 means 1.  Returns 0 or < 0. */
int dg_fill(void* out, int64_t n, int dtype, int dist, uint64_t seed,
            int64_t lo, int64_t hi, int nthreads) {
    if (n < 0 || (n > 0 && !out)) return DG_EINVAL;
    if (dtype < DG_I32 || dtype > DG_F32) return DG_EINVAL;
    if (dist < DG_UNIFORM || dist > DG_NORMAL_OUTLIERS) return DG_EINVAL;
    if (dist == DG_NORMAL_OUTLIERS && dtype != DG_F32) return DG_EINVAL;
    if ((lo != 0 || hi != 0) && (dtype == DG_F32 || hi <= lo)) return DG_EINVAL;
    if (dtype == DG_I32 && (lo < INT32_MIN || hi - 1 > INT32_MAX)) return DG_EINVAL;
    if (n == 0) return DG_OK;
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    if (n < 65536) nt = 1;

    zipf_table z = {0, 0};
    if (dist == DG_ZIPF && zipf_build(&z) != DG_OK) return DG_ENOMEM;
    fill_job jobs[256];
    for (int t = 0; t < nt; ++t) {
        fill_job j = {out, n * t / nt, n * (t + 1) / nt, dtype,
                      dist == DG_SORTED ? DG_UNIFORM : dist, seed, lo, hi, &z};
        jobs[t] = j;
    }
    int rc = run_threads(fill_worker, jobs, sizeof(fill_job), nt);
    free(z.cdf); free(z.guide);
    if (rc != DG_OK || dist != DG_SORTED) return rc;

    if (dtype == DG_F32) return radix_sort(out, n, dtype, 0, 24, nt);
    if (lo == 0 && hi == 0) {
        if (dtype == DG_I32) return radix_sort(out, n, dtype, -(1LL << 20), 21, nt);
        return radix_sort(out, n, dtype, -(1LL << 32), 33, nt);
    }
    int bits = 1;
    while (bits < 63 && ((uint64_t)1 << bits) < (uint64_t)(hi - lo)) ++bits;
    return radix_sort(out, n, dtype, lo, bits, nt);
}

/* Raw SplitMix64 output `ctr` for `seed`'s first stream (for generator tests). */
uint64_t dg_raw(uint64_t seed, uint64_t ctr) { return sm64_at(stream_key(seed, 0), ctr); }
