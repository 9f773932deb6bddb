/*
 * CPU oracle of the aggregation scan.  TEST INFRASTRUCTURE ONLY: the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark call it;
 * the GPU library never links, includes or calls it, and the two share no
 * code.  It is plain and slow on purpose, so that it can be checked by eye
 * against the definitions below.
 *
 * What is computed (Section 2.1 and Figure 4 of the paper: scan every item
 * of a column and fold it with an aggregation function into one summary,
 * r = aggregate(r, input[i]) over all i):
 *
 *   COUNT   n.  Columns are non-nullable, like the paper's key column.
 *   SUM     integer columns: the two's-complement sum mod 2^64 of the items
 *           widened to int64.  Addition mod 2^64 is associative and
 *           commutative, so this plain definition is the exact answer of any
 *           evaluation order.
 *           f32 columns: the exact real sum of the items, rounded once to the
 *           nearest double (ties to even).  The exact sum is held in a
 *           fixed-point superaccumulator: every finite float is m * 2^(k-149)
 *           with m < 2^24 and 0 <= k <= 253, so it is added as the integer
 *           m << k into a multi-digit integer.
 *   MIN/MAX the smallest / largest item.  f32: NaN items are skipped (IEEE
 *           minNum / maxNum); the result is NaN only if every item is NaN.
 *   AVG     RN(RN(SUM) / RN(n)) in double: the SUM above converted to double,
 *           divided by n converted to double.  Null when n == 0.
 *   ABS_SUM (f32 only) the exact sum of |x_i| rounded once to double, for
 *           the condition number kappa = sum|x| / |sum x| of the error report.
 *
 * Empty columns: SUM = 0, COUNT = 0, MIN / MAX / AVG are null.
 * Non-finite f32 items: any NaN, or both +Inf and -Inf, give a NaN sum;
 * otherwise an infinite item gives that infinity.
 *
 * Threads split [0, n) into contiguous ranges.  Every per-range result is
 * exact (integer sum mod 2^64, superaccumulator, min, max), so merging them
 * gives the same bits for any thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { O_I32 = 0, O_I64 = 1, O_F32 = 2 };
enum { O_SUM = 0, O_MIN = 1, O_MAX = 2, O_COUNT = 3, O_AVG = 4, O_ABS_SUM = 5 };

#define O_OK 0
#define O_EINVAL -1
#define O_ENOMEM -2

typedef struct {
    int64_t i64;     /* integer result (SUM / MIN / MAX of ints, COUNT) */
    double f64;      /* floating result (f32 SUM / MIN / MAX / ABS_SUM, AVG) */
    int64_t count;   /* n */
    int32_t is_null; /* 1 for MIN / MAX / AVG of an empty column */
    int32_t reserved;
} oracle_result;

/* ------------------------------------------------------------------ */
/* Superaccumulator: value = sum_k d[k] * 2^(32k) * 2^-149.
 * Each added float touches two digits by less than 2^32 each, so after at
 * most 2^30 additions every digit is below 2^62 in magnitude; sa_normalize()
 * is called before that.  12 digits = 384 bits hold 2^34 additions of the
 * largest float (24 + 253 + 34 = 311 bits plus sign). */

#define SA_DIGITS 12
#define SA_RENORM (1LL << 30)

typedef struct {
    int64_t d[SA_DIGITS];
    int64_t pending;             /* additions since the last normalisation */
    int64_t nan, pinf, ninf;     /* non-finite items seen */
} superacc;

static void sa_init(superacc* a) { memset(a, 0, sizeof *a); }

/* Carry-propagate so that d[0..SA_DIGITS-2] lie in [0, 2^32); the top digit
 * keeps the sign.  The value is unchanged. */
static void sa_normalize(superacc* a) {
    for (int k = 0; k < SA_DIGITS - 1; ++k) {
        int64_t carry = a->d[k] >> 32;            /* floor(d / 2^32) */
        a->d[k] -= carry * 4294967296LL;
        a->d[k + 1] += carry;
    }
    a->pending = 0;
}

static void sa_add_float(superacc* a, float x) {
    uint32_t bits;
    memcpy(&bits, &x, sizeof bits);
    uint32_t biased = (bits >> 23) & 0xFFu;
    uint32_t frac = bits & 0x7FFFFFu;
    int negative = (int)(bits >> 31);
    if (biased == 0xFFu) {
        if (frac) a->nan++;
        else if (negative) a->ninf++;
        else a->pinf++;
        return;
    }
    uint64_t m;  /* |x| = m * 2^(k - 149) */
    int k;
    if (biased == 0) { m = frac; k = 0; }              /* subnormal or zero */
    else { m = frac | 0x800000u; k = (int)biased - 1; } /* normal */
    uint64_t v = m << (k % 32);                        /* < 2^55 */
    int64_t lo = (int64_t)(v & 0xFFFFFFFFu);
    int64_t hi = (int64_t)(v >> 32);
    if (negative) { lo = -lo; hi = -hi; }
    a->d[k / 32] += lo;
    a->d[k / 32 + 1] += hi;
    if (++a->pending >= SA_RENORM) sa_normalize(a);
}

static void sa_merge(superacc* into, superacc* from) {
    sa_normalize(into);
    sa_normalize(from);
    for (int k = 0; k < SA_DIGITS; ++k) into->d[k] += from->d[k];
    into->nan += from->nan; into->pinf += from->pinf; into->ninf += from->ninf;
    sa_normalize(into);
}

static int sa_bit(const int64_t* d, int b) { return (int)((d[b / 32] >> (b % 32)) & 1); }

/* The exact value rounded to the nearest double, ties to even. */
static double sa_to_double(superacc* a) {
    if (a->nan || (a->pinf && a->ninf)) return NAN;
    if (a->pinf) return INFINITY;
    if (a->ninf) return -INFINITY;
    sa_normalize(a);
    int64_t d[SA_DIGITS];
    memcpy(d, a->d, sizeof d);
    int negative = d[SA_DIGITS - 1] < 0;
    if (negative) {  /* negate, then carry-propagate: all digits become >= 0 */
        for (int k = 0; k < SA_DIGITS; ++k) d[k] = -d[k];
        for (int k = 0; k < SA_DIGITS - 1; ++k) {
            int64_t carry = d[k] >> 32;
            d[k] -= carry * 4294967296LL;
            d[k + 1] += carry;
        }
    }
    int top = -1;  /* highest set bit of the magnitude */
    for (int b = 32 * SA_DIGITS - 1; b >= 0; --b)
        if (sa_bit(d, b)) { top = b; break; }
    if (top < 0) return 0.0;
    uint64_t mant = 0;
    int e;  /* magnitude ~ mant * 2^e * 2^-149 */
    if (top <= 52) {
        for (int b = top; b >= 0; --b) mant = (mant << 1) | (uint64_t)sa_bit(d, b);
        e = 0;
    } else {
        for (int b = top; b >= top - 52; --b) mant = (mant << 1) | (uint64_t)sa_bit(d, b);
        e = top - 52;
        int round = sa_bit(d, top - 53);
        int sticky = 0;
        for (int b = top - 54; b >= 0; --b) if (sa_bit(d, b)) { sticky = 1; break; }
        if (round && (sticky || (mant & 1))) {
            mant += 1;
            if (mant == (1ULL << 53)) { mant >>= 1; e += 1; }
        }
    }
    double r = ldexp((double)mant, e - 149);  /* exact: mant < 2^53, in range */
    return negative ? -r : r;
}

/* ------------------------------------------------------------------ */

typedef struct {
    const void* col;
    int64_t lo, hi;
    int dtype, op;
    uint64_t wrap_sum;       /* integer SUM mod 2^64 */
    int64_t imin, imax;      /* integer MIN / MAX */
    float fmin, fmax;        /* f32 MIN / MAX (NaN = nothing seen yet) */
    superacc sa;             /* f32 SUM / ABS_SUM */
} range_job;

static int64_t item_i64(const void* col, int dtype, int64_t i) {
    if (dtype == O_I32) return (int64_t)((const int32_t*)col)[i];
    return ((const int64_t*)col)[i];
}

static void* range_worker(void* arg) {
    range_job* j = (range_job*)arg;
    j->wrap_sum = 0;
    j->imin = INT64_MAX;
    j->imax = INT64_MIN;
    j->fmin = NAN;
    j->fmax = NAN;
    sa_init(&j->sa);
    for (int64_t i = j->lo; i < j->hi; ++i) {
        if (j->dtype == O_F32) {
            float x = ((const float*)j->col)[i];
            if (j->op == O_SUM || j->op == O_AVG) sa_add_float(&j->sa, x);
            else if (j->op == O_ABS_SUM) sa_add_float(&j->sa, fabsf(x));
            else if (j->op == O_MIN) { if (!isnan(x) && (isnan(j->fmin) || x < j->fmin)) j->fmin = x; }
            else if (j->op == O_MAX) { if (!isnan(x) && (isnan(j->fmax) || x > j->fmax)) j->fmax = x; }
        } else {
            int64_t x = item_i64(j->col, j->dtype, i);
            if (j->op == O_SUM || j->op == O_AVG) j->wrap_sum += (uint64_t)x;
            else if (j->op == O_MIN) { if (x < j->imin) j->imin = x; }
            else if (j->op == O_MAX) { if (x > j->imax) j->imax = x; }
        }
    }
    return NULL;
}

/* Aggregate col[0..n) of `dtype` with `op` using `nthreads` threads. */
int oracle_aggregate(const void* col, int64_t n, int dtype, int op, int nthreads,
                     oracle_result* out) {
    if (!out || n < 0 || (n > 0 && !col)) return O_EINVAL;
    if (dtype < O_I32 || dtype > O_F32 || op < O_SUM || op > O_ABS_SUM) return O_EINVAL;
    if (op == O_ABS_SUM && dtype != O_F32) return O_EINVAL;
    memset(out, 0, sizeof *out);
    out->count = n;
    if (op == O_COUNT) { out->i64 = n; out->f64 = (double)n; return O_OK; }

    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    if (n < 65536) nt = 1;
    range_job* jobs = (range_job*)calloc((size_t)nt, sizeof(range_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return O_ENOMEM; }
    for (int t = 0; t < nt; ++t) {
        jobs[t].col = col; jobs[t].dtype = dtype; jobs[t].op = op;
        jobs[t].lo = n * t / nt; jobs[t].hi = n * (t + 1) / nt;
    }
    int started = 0;
    for (int t = 1; t < nt; ++t) {
        if (pthread_create(&th[t], NULL, range_worker, &jobs[t])) break;
        started = t;
    }
    for (int t = started + 1; t < nt; ++t) range_worker(&jobs[t]);  /* no thread: run here */
    range_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);

    /* Merge in range order; every merge below is exact. */
    range_job* m = &jobs[0];
    for (int t = 1; t < nt; ++t) {
        m->wrap_sum += jobs[t].wrap_sum;
        if (jobs[t].imin < m->imin) m->imin = jobs[t].imin;
        if (jobs[t].imax > m->imax) m->imax = jobs[t].imax;
        if (!isnan(jobs[t].fmin) && (isnan(m->fmin) || jobs[t].fmin < m->fmin)) m->fmin = jobs[t].fmin;
        if (!isnan(jobs[t].fmax) && (isnan(m->fmax) || jobs[t].fmax > m->fmax)) m->fmax = jobs[t].fmax;
        if (dtype == O_F32) sa_merge(&m->sa, &jobs[t].sa);
    }

    if (dtype == O_F32) {
        double s = (op == O_SUM || op == O_AVG || op == O_ABS_SUM) ? sa_to_double(&m->sa) : 0.0;
        if (op == O_SUM || op == O_ABS_SUM) out->f64 = s;
        else if (op == O_AVG) { if (n == 0) out->is_null = 1; else out->f64 = s / (double)n; }
        else if (op == O_MIN) { if (n == 0) out->is_null = 1; else out->f64 = (double)m->fmin; }
        else if (op == O_MAX) { if (n == 0) out->is_null = 1; else out->f64 = (double)m->fmax; }
    } else {
        int64_t s = (int64_t)m->wrap_sum;
        if (op == O_SUM) { out->i64 = s; out->f64 = (double)s; }
        else if (op == O_AVG) { if (n == 0) out->is_null = 1; else out->f64 = (double)s / (double)n; }
        else if (op == O_MIN) { if (n == 0) out->is_null = 1; else { out->i64 = m->imin; out->f64 = (double)m->imin; } }
        else if (op == O_MAX) { if (n == 0) out->is_null = 1; else { out->i64 = m->imax; out->f64 = (double)m->imax; } }
    }
    free(jobs);
    free(th);
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Group-by: for every distinct key k of keys[0..n), the aggregate of the
 * values whose key is k (the same per-group definitions as above: integer
 * SUM mod 2^64, MIN, MAX, COUNT, AVG = RN(RN(SUM)/RN(count)); float SUM
 * exact then rounded once; float MIN / MAX skip NaN).  Groups come out in
 * ascending key order.  Plain method: sort the item indices by key, then
 * fold each run of equal keys. */

typedef struct {
    int64_t key;
    int64_t i64;     /* integer SUM / MIN / MAX */
    double f64;      /* float SUM / MIN / MAX, AVG, integer results converted */
    int64_t count;
} oracle_group;

static const void* g_sort_keys;
static int g_sort_key_dtype;

static int64_t key_at(const void* keys, int dt, int64_t i) {
    return dt == O_I32 ? (int64_t)((const int32_t*)keys)[i] : ((const int64_t*)keys)[i];
}

static int cmp_index(const void* a, const void* b) {
    int64_t ka = key_at(g_sort_keys, g_sort_key_dtype, *(const int64_t*)a);
    int64_t kb = key_at(g_sort_keys, g_sort_key_dtype, *(const int64_t*)b);
    return (ka > kb) - (ka < kb);
}

/* Returns the number of groups (>= 0), or a negative code; at most
 * max_groups are written (the count returned is the true number). */
int64_t oracle_groupby(const void* keys, int key_dtype, const void* vals, int val_dtype, int64_t n, int op,
                       oracle_group* out, int64_t max_groups) {
    if (n < 0 || (n > 0 && (!keys || !vals)) || (key_dtype != O_I32 && key_dtype != O_I64)) return O_EINVAL;
    if (val_dtype < O_I32 || val_dtype > O_F32 || op < O_SUM || op > O_AVG) return O_EINVAL;
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!idx) return O_ENOMEM;
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    g_sort_keys = keys;
    g_sort_key_dtype = key_dtype;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_index);
    int64_t ngroups = 0;
    int64_t i = 0;
    while (i < n) {
        const int64_t k = key_at(keys, key_dtype, idx[i]);
        int64_t j = i;
        uint64_t wrap = 0;
        int64_t imin = INT64_MAX, imax = INT64_MIN;
        float fmin = NAN, fmax = NAN;
        superacc sa;
        sa_init(&sa);
        for (; j < n && key_at(keys, key_dtype, idx[j]) == k; ++j) {
            const int64_t r = idx[j];
            if (val_dtype == O_F32) {
                const float x = ((const float*)vals)[r];
                sa_add_float(&sa, x);
                if (!isnan(x) && (isnan(fmin) || x < fmin)) fmin = x;
                if (!isnan(x) && (isnan(fmax) || x > fmax)) fmax = x;
            } else {
                const int64_t x = item_i64(vals, val_dtype, r);
                wrap += (uint64_t)x;
                if (x < imin) imin = x;
                if (x > imax) imax = x;
            }
        }
        if (ngroups < max_groups && out) {
            oracle_group* g = &out[ngroups];
            g->key = k;
            g->count = j - i;
            g->i64 = 0;
            g->f64 = 0.0;
            if (op == O_COUNT) {
                g->i64 = j - i;
                g->f64 = (double)(j - i);
            } else if (val_dtype == O_F32) {
                const double s = sa_to_double(&sa);
                if (op == O_SUM) g->f64 = s;
                else if (op == O_AVG) g->f64 = s / (double)(j - i);
                else g->f64 = (double)(op == O_MIN ? fmin : fmax);
            } else {
                const int64_t s = (int64_t)wrap;
                if (op == O_SUM) { g->i64 = s; g->f64 = (double)s; }
                else if (op == O_AVG) { g->i64 = s; g->f64 = (double)s / (double)(j - i); }
                else { g->i64 = op == O_MIN ? imin : imax; g->f64 = (double)g->i64; }
            }
        }
        ++ngroups;
        i = j;
    }
    free(idx);
    return ngroups;
}

/* ------------------------------------------------------------------ */
/* Block tables: out[j] = SUM (mod 2^64), MIN or MAX of the integer items
 * col[j*block, min((j+1)*block, n)), for j = 0 .. ceil(n/block) - 1 -- the
 * same definitions as oracle_aggregate, applied to each block.  They let a
 * test check many aggregations of sub-ranges of one large column: a range is
 * its partial end blocks (aggregated directly) plus whole blocks (combined
 * from the table; exact, since sum mod 2^64, min and max are associative). */

typedef struct {
    const void* col;
    int64_t n, block, jlo, jhi;
    int dtype, op;
    int64_t* out;
} block_job;

static void* block_worker(void* arg) {
    block_job* b = (block_job*)arg;
    for (int64_t j = b->jlo; j < b->jhi; ++j) {
        const int64_t lo = j * b->block;
        const int64_t hi = lo + b->block < b->n ? lo + b->block : b->n;
        uint64_t wrap = 0;
        int64_t mn = INT64_MAX, mx = INT64_MIN;
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t x = item_i64(b->col, b->dtype, i);
            wrap += (uint64_t)x;
            if (x < mn) mn = x;
            if (x > mx) mx = x;
        }
        b->out[j] = b->op == O_SUM ? (int64_t)wrap : (b->op == O_MIN ? mn : mx);
    }
    return NULL;
}

int oracle_block_aggregate(const void* col, int64_t n, int dtype, int op, int64_t block, int64_t* out,
                           int nthreads) {
    if (n < 0 || (n > 0 && (!col || !out)) || block < 1) return O_EINVAL;
    if ((dtype != O_I32 && dtype != O_I64) || (op != O_SUM && op != O_MIN && op != O_MAX)) return O_EINVAL;
    const int64_t nb = (n + block - 1) / block;
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    if (nb < nt) nt = nb > 0 ? (int)nb : 1;
    block_job* jobs = (block_job*)calloc((size_t)nt, sizeof(block_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return O_ENOMEM; }
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (block_job){col, n, block, nb * t / nt, nb * (t + 1) / nt, dtype, op, out};
    }
    int started = 0;
    for (int t = 1; t < nt; ++t) {
        if (pthread_create(&th[t], NULL, block_worker, &jobs[t])) break;
        started = t;
    }
    for (int t = started + 1; t < nt; ++t) block_worker(&jobs[t]);
    block_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Host memory read ceiling for the CPU baseline: `nthreads` threads read
 * contiguous ranges of the buffer 64 bits at a time (8 independent xor
 * chains each, so the loop is bound by memory, not by a dependency); the xor
 * of everything is returned so the reads cannot be dropped.  Not part of any
 * aggregation result. */

typedef struct {
    const uint64_t* p;
    int64_t lo, hi;
    uint64_t acc;
} read_job;

static void* read_worker(void* arg) {
    read_job* r = (read_job*)arg;
    uint64_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = r->lo;
    for (; i + 8 <= r->hi; i += 8)
        for (int k = 0; k < 8; ++k) a[k] ^= r->p[i + k];
    for (; i < r->hi; ++i) a[0] ^= r->p[i];
    r->acc = a[0] ^ a[1] ^ a[2] ^ a[3] ^ a[4] ^ a[5] ^ a[6] ^ a[7];
    return NULL;
}

int oracle_read_ceiling(const void* buf, int64_t bytes, int nthreads, uint64_t* xor_out) {
    if (bytes < 0 || (bytes > 0 && !buf) || !xor_out) return O_EINVAL;
    const int64_t words = bytes / 8;
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    read_job* jobs = (read_job*)calloc((size_t)nt, sizeof(read_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return O_ENOMEM; }
    for (int t = 0; t < nt; ++t) jobs[t] = (read_job){(const uint64_t*)buf, words * t / nt, words * (t + 1) / nt, 0};
    int started = 0;
    for (int t = 1; t < nt; ++t) {
        if (pthread_create(&th[t], NULL, read_worker, &jobs[t])) break;
        started = t;
    }
    for (int t = started + 1; t < nt; ++t) read_worker(&jobs[t]);
    read_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    uint64_t x = 0;
    for (int t = 0; t < nt; ++t) x ^= jobs[t].acc;
    *xor_out = x;
    free(jobs);
    free(th);
    return O_OK;
}
