/*
 * CPU oracle for hybrid tensor network (h-TN) contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  It shares no code with the GPU library;
 * only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.
 *
 * A network: n_t tensors, tensor i has ranks[i] modes whose labels are
 * labels[off_i .. off_i + ranks[i]) (off_i = sum of earlier ranks); dims[l]
 * is the extent of label l; data[i] is row-major with the last mode fastest.
 * The result is indexed by out_labels (row-major, last fastest); a label
 * that is not an output label is summed.  A label carried by several
 * tensors is one index summed once (hyperedge semantics, Sec. 2.2).
 *
 *  oracle_naive   The knitting sum written out (Sec. 2.1, Eq. knitting):
 *                 for every output assignment, the sum over every assignment
 *                 of every summed label of the product of one entry of every
 *                 tensor.  Neumaier-compensated FP64 accumulation.
 *  oracle_ve      Variable (bucket) elimination: repeatedly pick a summed
 *                 label, multiply every factor that carries it and sum the
 *                 label out.  mode 1 runs in double-double arithmetic
 *                 (reference values), mode 0 in plain FP64 (timed baseline).
 *                 Exact in exact arithmetic by the distributive law, so it
 *                 equals oracle_naive up to rounding.
 *
 * Double-double arithmetic follows the published error-free transformations:
 * Knuth's TwoSum, TwoProd via fused multiply-add, and the double-double
 * add/multiply of Hida, Li and Bailey (QD library paper, 2001).  Build
 * without -ffast-math and with -ffp-contract=off so that the error-free
 * transformations are not rewritten by the compiler.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EARG -1
#define OR_ENOMEM -2

/* ------------------------------------------------------------------ */
/* error-free transformations and double-double                        */
/* ------------------------------------------------------------------ */

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = {s, e};
    return r;
}

static inline dd quick_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    dd r = {s, e};
    return r;
}

static inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd r = {p, e};
    return r;
}

static inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

static inline dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

/* Neumaier's improved Kahan summation. */
typedef struct { double s, c; } neum;

static inline void neum_add(neum *acc, double x) {
    double t = acc->s + x;
    if (fabs(acc->s) >= fabs(x))
        acc->c += (acc->s - t) + x;
    else
        acc->c += (x - t) + acc->s;
    acc->s = t;
}

/* ------------------------------------------------------------------ */
/* shared validation                                                   */
/* ------------------------------------------------------------------ */

static int check_net(int n_t, const int *ranks, const int *labels, int n_labels,
                     const int64_t *dims, int n_out, const int *out_labels) {
    if (n_t <= 0 || n_labels < 0 || !ranks || !dims) return OR_EARG;
    int off = 0;
    for (int i = 0; i < n_t; ++i) {
        if (ranks[i] < 0) return OR_EARG;
        for (int a = 0; a < ranks[i]; ++a) {
            int l = labels[off + a];
            if (l < 0 || l >= n_labels) return OR_EARG;
            for (int b = 0; b < a; ++b)
                if (labels[off + b] == l) return OR_EARG;
        }
        off += ranks[i];
    }
    for (int l = 0; l < n_labels; ++l)
        if (dims[l] <= 0) return OR_EARG;
    for (int a = 0; a < n_out; ++a) {
        if (out_labels[a] < 0 || out_labels[a] >= n_labels) return OR_EARG;
        for (int b = 0; b < a; ++b)
            if (out_labels[b] == out_labels[a]) return OR_EARG;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* naive knitting sum                                                  */
/* ------------------------------------------------------------------ */

/*
 * out[o] (o over out_labels, row-major) =
 *     sum over assignments of summed labels of  prod_i data[i][entry].
 * Summed labels = labels carried by some tensor and not in out_labels.
 * n_terms (optional) receives the number of (output, summed) assignments;
 * n_mults (optional) the multiplications the loop performed, counted as
 * they are made (each term is the product of its n_t factors: n_t - 1
 * multiplications, the |C| (s + n_g - 1) of Sec. 2.1 for s QTs and n_g
 * coefficient tensors).
 */
int oracle_naive(int n_t, const int *ranks, const int *labels, int n_labels,
                 const int64_t *dims, const double *const *data, int n_out,
                 const int *out_labels, double *out, int64_t *n_terms, int64_t *n_mults) {
    int st = check_net(n_t, ranks, labels, n_labels, dims, n_out, out_labels);
    if (st) return st;
    if (!data || !out) return OR_EARG;

    int *is_out = calloc((size_t)n_labels + 1, sizeof(int));
    int *used = calloc((size_t)n_labels + 1, sizeof(int));
    int *sum_labels = malloc(sizeof(int) * ((size_t)n_labels + 1));
    int *toff = malloc(sizeof(int) * (size_t)n_t);
    if (!is_out || !used || !sum_labels || !toff) {
        free(is_out); free(used); free(sum_labels); free(toff);
        return OR_ENOMEM;
    }
    for (int a = 0; a < n_out; ++a) is_out[out_labels[a]] = 1;
    int off = 0;
    for (int i = 0; i < n_t; ++i) {
        toff[i] = off;
        for (int a = 0; a < ranks[i]; ++a) used[labels[off + a]] = 1;
        off += ranks[i];
    }
    int n_sum = 0;
    for (int l = 0; l < n_labels; ++l)
        if (used[l] && !is_out[l]) sum_labels[n_sum++] = l;

    int64_t n_o = 1, n_s = 1;
    for (int a = 0; a < n_out; ++a) n_o *= dims[out_labels[a]];
    for (int a = 0; a < n_sum; ++a) n_s *= dims[sum_labels[a]];
    if (n_terms) *n_terms = n_o * n_s;

    /* Parallelise over fixed chunks of the summed space so the result does
     * not depend on the thread count. */
    const int64_t n_chunks = n_s < 64 ? n_s : 64;
    int64_t mults = 0;
    for (int64_t o = 0; o < n_o; ++o) {
        neum *part = calloc((size_t)n_chunks, sizeof(neum));
        int64_t *part_mults = calloc((size_t)n_chunks, sizeof(int64_t));
        if (!part || !part_mults) { free(part); free(part_mults); st = OR_ENOMEM; break; }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t ch = 0; ch < n_chunks; ++ch) {
            int64_t *idx = malloc(sizeof(int64_t) * ((size_t)n_labels + 1));
            int64_t s0 = n_s * ch / n_chunks, s1 = n_s * (ch + 1) / n_chunks;
            int64_t cnt = 0;
            neum acc = {0.0, 0.0};
            /* output label digits */
            int64_t r = o;
            for (int a = n_out - 1; a >= 0; --a) {
                int l = out_labels[a];
                idx[l] = r % dims[l];
                r /= dims[l];
            }
            for (int64_t s = s0; s < s1; ++s) {
                int64_t q = s;
                for (int a = n_sum - 1; a >= 0; --a) {
                    int l = sum_labels[a];
                    idx[l] = q % dims[l];
                    q /= dims[l];
                }
                double prod = 0.0;
                for (int i = 0; i < n_t; ++i) {
                    int64_t e = 0;
                    for (int a = 0; a < ranks[i]; ++a) {
                        int l = labels[toff[i] + a];
                        e = e * dims[l] + idx[l];
                    }
                    if (i == 0) {
                        prod = data[i][e];
                    } else {
                        prod *= data[i][e];
                        ++cnt;
                    }
                }
                neum_add(&acc, prod);
            }
            part[ch] = acc;
            part_mults[ch] = cnt;
            free(idx);
        }
        for (int64_t ch = 0; ch < n_chunks; ++ch) mults += part_mults[ch];
        free(part_mults);
        neum tot = {0.0, 0.0};
        for (int64_t ch = 0; ch < n_chunks; ++ch) {
            neum_add(&tot, part[ch].s);
            neum_add(&tot, part[ch].c);
        }
        out[o] = tot.s + tot.c;
        free(part);
    }
    if (n_mults) *n_mults = mults;
    free(is_out); free(used); free(sum_labels); free(toff);
    return st;
}

/* ------------------------------------------------------------------ */
/* variable elimination                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    int rank;
    int *lab;     /* ascending label ids */
    int64_t size;
    dd *v;        /* row-major over lab, last fastest */
} factor;

static void factor_free(factor *f) {
    free(f->lab);
    free(f->v);
    f->lab = NULL;
    f->v = NULL;
}

static inline dd mul_mode(dd a, dd b, int mode) {
    if (mode) return dd_mul(a, b);
    dd r = {a.hi * b.hi, 0.0};
    return r;
}

static inline dd add_mode(dd a, dd b, int mode) {
    if (mode) return dd_add(a, b);
    dd r = {a.hi + b.hi, 0.0};
    return r;
}

/* Offset of factor f's entry at the full assignment idx[]. */
static inline int64_t factor_off(const factor *f, const int64_t *dims, const int64_t *idx) {
    int64_t e = 0;
    for (int a = 0; a < f->rank; ++a) e = e * dims[f->lab[a]] + idx[f->lab[a]];
    return e;
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/*
 * Multiply the factors listed in sel[0..n_sel) into one factor over the
 * union of their labels, summing out label `elim` (elim < 0: sum nothing).
 */
static int combine(factor *fs, const int *sel, int n_sel, int elim, const int64_t *dims,
                   int n_labels, int mode, factor *res) {
    int *mark = calloc((size_t)n_labels + 1, sizeof(int));
    if (!mark) return OR_ENOMEM;
    for (int k = 0; k < n_sel; ++k)
        for (int a = 0; a < fs[sel[k]].rank; ++a) mark[fs[sel[k]].lab[a]] = 1;
    int rank = 0;
    for (int l = 0; l < n_labels; ++l)
        if (mark[l] && l != elim) ++rank;
    res->rank = rank;
    res->lab = malloc(sizeof(int) * ((size_t)rank + 1));
    int p = 0;
    res->size = 1;
    for (int l = 0; l < n_labels; ++l)
        if (mark[l] && l != elim) {
            res->lab[p++] = l;
            res->size *= dims[l];
        }
    free(mark);
    res->v = malloc(sizeof(dd) * (size_t)res->size);
    if (!res->lab || !res->v) return OR_ENOMEM;
    const int64_t d_elim = elim >= 0 ? dims[elim] : 1;
    int st = OR_OK;
#pragma omp parallel
    {
        int64_t *idx = malloc(sizeof(int64_t) * ((size_t)n_labels + 1));
        if (!idx) {
#pragma omp atomic write
            st = OR_ENOMEM;
        } else {
#pragma omp for schedule(static)
            for (int64_t o = 0; o < res->size; ++o) {
                int64_t r = o;
                for (int a = rank - 1; a >= 0; --a) {
                    idx[res->lab[a]] = r % dims[res->lab[a]];
                    r /= dims[res->lab[a]];
                }
                dd acc = {0.0, 0.0};
                for (int64_t v = 0; v < d_elim; ++v) {
                    if (elim >= 0) idx[elim] = v;
                    dd prod = {1.0, 0.0};
                    for (int k = 0; k < n_sel; ++k) {
                        const factor *f = &fs[sel[k]];
                        prod = mul_mode(prod, f->v[factor_off(f, dims, idx)], mode);
                    }
                    acc = add_mode(acc, prod, mode);
                }
                res->v[o] = acc;
            }
            free(idx);
        }
    }
    return st;
}

/*
 * Elimination order: among summed labels still present, the one whose
 * elimination produces the smallest new factor; ties go to the lower label
 * id.  Result written as out_hi[o] + out_lo[o] (out_lo may be NULL).
 */
int oracle_ve(int n_t, const int *ranks, const int *labels, int n_labels,
              const int64_t *dims, const double *const *data, int n_out,
              const int *out_labels, int mode, double *out_hi, double *out_lo) {
    int st = check_net(n_t, ranks, labels, n_labels, dims, n_out, out_labels);
    if (st) return st;
    if (!data || !out_hi) return OR_EARG;

    int cap = n_t + 1;
    factor *fs = calloc((size_t)cap, sizeof(factor));
    int *alive = calloc((size_t)cap, sizeof(int));
    int *is_out = calloc((size_t)n_labels + 1, sizeof(int));
    int *sel = malloc(sizeof(int) * (size_t)cap);
    if (!fs || !alive || !is_out || !sel) {
        free(fs); free(alive); free(is_out); free(sel);
        return OR_ENOMEM;
    }
    for (int a = 0; a < n_out; ++a) is_out[out_labels[a]] = 1;

    /* Load inputs as factors with ascending label order. */
    int off = 0;
    for (int i = 0; i < n_t; ++i) {
        factor *f = &fs[i];
        f->rank = ranks[i];
        f->lab = malloc(sizeof(int) * ((size_t)ranks[i] + 1));
        memcpy(f->lab, labels + off, sizeof(int) * (size_t)ranks[i]);
        qsort(f->lab, (size_t)f->rank, sizeof(int), cmp_int);
        f->size = 1;
        for (int a = 0; a < f->rank; ++a) f->size *= dims[f->lab[a]];
        f->v = malloc(sizeof(dd) * (size_t)f->size);
        int64_t *idx = calloc((size_t)n_labels + 1, sizeof(int64_t));
        for (int64_t e = 0; e < f->size; ++e) {
            /* source entry e in the caller's mode order */
            int64_t r = e;
            for (int a = ranks[i] - 1; a >= 0; --a) {
                int l = labels[off + a];
                idx[l] = r % dims[l];
                r /= dims[l];
            }
            dd x = {data[i][e], 0.0};
            f->v[factor_off(f, dims, idx)] = x;
        }
        free(idx);
        alive[i] = 1;
        off += ranks[i];
    }
    int n_f = n_t;

    for (;;) {
        /* candidate labels: summed and present in some live factor */
        int best = -1;
        double best_size = 0.0;
        for (int l = 0; l < n_labels; ++l) {
            if (is_out[l]) continue;
            int present = 0;
            double sz = 1.0;
            int *mark = calloc((size_t)n_labels + 1, sizeof(int));
            for (int k = 0; k < n_f; ++k) {
                if (!alive[k]) continue;
                int has = 0;
                for (int a = 0; a < fs[k].rank; ++a)
                    if (fs[k].lab[a] == l) has = 1;
                if (!has) continue;
                present = 1;
                for (int a = 0; a < fs[k].rank; ++a) mark[fs[k].lab[a]] = 1;
            }
            for (int m = 0; m < n_labels; ++m)
                if (mark[m] && m != l) sz *= (double)dims[m];
            free(mark);
            if (present && (best < 0 || sz < best_size)) {
                best = l;
                best_size = sz;
            }
        }
        if (best < 0) break;
        int n_sel = 0;
        for (int k = 0; k < n_f; ++k) {
            if (!alive[k]) continue;
            for (int a = 0; a < fs[k].rank; ++a)
                if (fs[k].lab[a] == best) { sel[n_sel++] = k; break; }
        }
        factor res;
        memset(&res, 0, sizeof(res));
        st = combine(fs, sel, n_sel, best, dims, n_labels, mode, &res);
        if (st) { factor_free(&res); goto done; }
        for (int k = 0; k < n_sel; ++k) {
            factor_free(&fs[sel[k]]);
            alive[sel[k]] = 0;
        }
        /* reuse the first freed slot */
        fs[sel[0]] = res;
        alive[sel[0]] = 1;
    }

    /* Remaining factors carry output labels only: take their product. */
    {
        int n_sel = 0;
        for (int k = 0; k < n_f; ++k)
            if (alive[k]) sel[n_sel++] = k;
        factor res;
        memset(&res, 0, sizeof(res));
        st = combine(fs, sel, n_sel, -1, dims, n_labels, mode, &res);
        if (st) { factor_free(&res); goto done; }
        /* Output labels carried by no tensor are broadcast. */
        int64_t n_o = 1;
        for (int a = 0; a < n_out; ++a) n_o *= dims[out_labels[a]];
        int64_t *idx = calloc((size_t)n_labels + 1, sizeof(int64_t));
        for (int64_t o = 0; o < n_o; ++o) {
            int64_t r = o;
            for (int a = n_out - 1; a >= 0; --a) {
                int l = out_labels[a];
                idx[l] = r % dims[l];
                r /= dims[l];
            }
            dd x = res.v[factor_off(&res, dims, idx)];
            out_hi[o] = x.hi;
            if (out_lo) out_lo[o] = x.lo;
        }
        free(idx);
        factor_free(&res);
    }
done:
    for (int k = 0; k < n_f; ++k)
        if (alive[k]) factor_free(&fs[k]);
    free(fs); free(alive); free(is_out); free(sel);
    return st;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
