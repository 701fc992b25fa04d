/*
 * CPU oracle for the loop-of-stencil-reduce pattern -- TEST INFRASTRUCTURE ONLY.
 * See lsr_oracle.h for the contract. Build: gcc -O2 -ffp-contract=off -fopenmp.
 *
 * Structure follows the paper's functional semantics (Sect. 3.1):
 *   loop-of-stencil-reduce-d-s:
 *     s = init; repeat { b = stencil(sigma_1, f'):a ; d = alpha(delta):b ;
 *                        a = alpha(fst):b ; s = update } until c(/(+):d, s)
 * with one full sweep into a distinct array (a stencil cannot run in place,
 * Sect. 3.1), then a separate reduce pass, then the condition. No fusion, no
 * blocking: each step is its own loop over the whole grid.
 */
#include "lsr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* A check happens every check_every sweeps and always at the sweep cap
 * (the -s variant's state is the sweep count n). */
static int is_check_sweep(int64_t n, int check_every, int64_t max_iter) {
    return (n % check_every) == 0 || n == max_iter;
}

/* max that keeps a NaN once one is seen, whatever the order of the operands */
static double max_nan(double acc, double d) {
    return (d > acc || d != d) ? d : acc;
}

/* ---------------------------------------------------------------------------
 * Reduce /(+) over delta(b, a) (Sect. 3.1, -d variant). Per-row partials are
 * formed left to right and combined top to bottom, so the value does not depend
 * on the number of threads.
 * ------------------------------------------------------------------------- */
static double reduce_delta(int op, const double *b, const double *a, int64_t rows, int64_t cols) {
    double *part = (double *)malloc(sizeof(double) * (size_t)rows);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < cols; ++j) {
            double d = b[i * cols + j] - a[i * cols + j];
            if (op == ORC_RED_MAX_ABS_DELTA) acc = max_nan(acc, fabs(d));
            else if (op == ORC_RED_L2_DELTA) acc = acc + d * d;
            else acc = acc + fabs(d);
        }
        part[i] = acc;
    }
    double r = 0.0;
    for (int64_t i = 0; i < rows; ++i)
        r = (op == ORC_RED_MAX_ABS_DELTA) ? max_nan(r, part[i]) : r + part[i];
    free(part);
    if (op == ORC_RED_L2_DELTA) r = sqrt(r);
    if (op == ORC_RED_MEAN_ABS_DELTA) r = r / ((double)rows * (double)cols);
    return r;
}

/* ---------------------------------------------------------------------------
 * 5-point Jacobi sweep (Helmholtz solver of Sect. 4.1, Laplace as alpha = 0,
 * f = 0). The outer ring is boundary data: copied, never updated.
 * ------------------------------------------------------------------------- */
/* The right-hand side of the -i form (index-aware elemental function, Sect. 3.1):
 * g(i, j) = c2 * (c1 * (p_i * q_j)), evaluated from the cell's indices. */
typedef struct {
    const double *p, *q;
    double c1, c2;
} sep_source;

static void jacobi_sweep(int helmholtz, const double *a, double *b, const double *g,
                         const sep_source *sep, int64_t rows, int64_t cols, double rd) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            int64_t p = i * cols + j;
            if (i == 0 || j == 0 || i == rows - 1 || j == cols - 1) {
                b[p] = a[p];
                continue;
            }
            double nn = a[p - cols], ss = a[p + cols], ww = a[p - 1], ee = a[p + 1];
            if (sep) {
                double gij = sep->c2 * (sep->c1 * (sep->p[i] * sep->q[j]));
                b[p] = (((nn + ss) + (ww + ee)) + gij) * rd;
            } else if (helmholtz) {
                b[p] = (((nn + ss) + (ww + ee)) + g[p]) * rd;
            } else {
                b[p] = 0.25 * ((nn + ss) + (ww + ee));
            }
        }
    }
}

static int jacobi_loop(int helmholtz, double *a, const double *g, const sep_source *sep,
                       int64_t rows, int64_t cols, double alpha, double h, int reduce_op,
                       int cond_kind, double thr, int check_every, int64_t max_iter,
                       double *trace, int64_t trace_cap, orc_result *out);

int orc_jacobi_run(int helmholtz, double *a, const double *g, int64_t rows, int64_t cols,
                   double alpha, double h, int reduce_op, int cond_kind, double thr,
                   int check_every, int64_t max_iter, double *trace, int64_t trace_cap,
                   orc_result *out) {
    if (helmholtz && !g) return -1;
    return jacobi_loop(helmholtz, a, g, NULL, rows, cols, alpha, h, reduce_op, cond_kind, thr,
                       check_every, max_iter, trace, trace_cap, out);
}

int orc_jacobi_sep_run(double *a, const double *p, const double *q, double c1, double c2,
                       int64_t rows, int64_t cols, double alpha, double h, int reduce_op,
                       int cond_kind, double thr, int check_every, int64_t max_iter,
                       double *trace, int64_t trace_cap, orc_result *out) {
    if (!p || !q) return -1;
    sep_source sep = {p, q, c1, c2};
    return jacobi_loop(1, a, NULL, &sep, rows, cols, alpha, h, reduce_op, cond_kind, thr,
                       check_every, max_iter, trace, trace_cap, out);
}

static int jacobi_loop(int helmholtz, double *a, const double *g, const sep_source *sep,
                       int64_t rows, int64_t cols, double alpha, double h, int reduce_op,
                       int cond_kind, double thr, int check_every, int64_t max_iter,
                       double *trace, int64_t trace_cap, orc_result *out) {
    if (!a || !out || rows < 3 || cols < 3 || check_every < 1 || max_iter < 1) return -1;
    if (reduce_op != ORC_RED_MAX_ABS_DELTA && reduce_op != ORC_RED_L2_DELTA &&
        reduce_op != ORC_RED_MEAN_ABS_DELTA) return -1;
    if (cond_kind != ORC_COND_BELOW && cond_kind != ORC_COND_NEVER) return -1;
    double rd = 1.0 / (4.0 + alpha * (h * h));
    size_t bytes = sizeof(double) * (size_t)(rows * cols);
    double *cur = (double *)malloc(bytes), *nxt = (double *)malloc(bytes);
    memcpy(cur, a, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    int64_t n = 0;
    int stop = 0;
    do {
        jacobi_sweep(helmholtz, cur, nxt, g, sep, rows, cols, rd);     /* b = stencil(f'):a */
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            double r = reduce_delta(reduce_op, nxt, cur, rows, cols);  /* /(+):alpha(delta):b */
            if (trace && out->checks < trace_cap) trace[out->checks] = r;
            out->checks += 1;
            out->r = r;
            if (isnan(r) || isinf(r)) { out->numeric_error = 1; stop = 1; }
            else if (cond_kind == ORC_COND_BELOW && r < thr) { out->converged = 1; stop = 1; }
        }
        double *t = cur; cur = nxt; nxt = t;                            /* a = alpha(fst):b */
    } while (!stop && n < max_iter);
    memcpy(a, cur, bytes);
    out->n = n;
    free(cur);
    free(nxt);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Game of Life (Fig. 1): count live neighbours of the 3x3 window, then
 * alive' = (count == 3) || (alive && count == 2).
 * ------------------------------------------------------------------------- */
/* Index of the neighbour at offset d in {-1, 0, 1} of position x on an axis of
 * length n: wrapped on a torus, -1 (absent) past a dead border. */
static int64_t neighbour_index(int bc, int64_t x, int d, int64_t n) {
    int64_t y = x + d;
    if (y >= 0 && y < n) return y;
    if (bc != ORC_BC_TORUS) return -1;
    return y < 0 ? y + n : y - n;
}

static void life_sweep(int bc, const uint8_t *a, uint8_t *b, int64_t rows, int64_t cols) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        /* the rows above, at and below i (NULL: out of range, all dead) */
        const uint8_t *nb_row[3];
        for (int di = -1; di <= 1; ++di) {
            int64_t ii = neighbour_index(bc, i, di, rows);
            nb_row[di + 1] = ii < 0 ? NULL : a + ii * cols;
        }
        for (int64_t j = 0; j < cols; ++j) {
            int64_t jl = neighbour_index(bc, j, -1, cols), jr = neighbour_index(bc, j, 1, cols);
            int count = 0;
            for (int r = 0; r < 3; ++r) {
                const uint8_t *row = nb_row[r];
                if (!row) continue;
                if (jl >= 0) count += row[jl] != 0;
                if (r != 1) count += row[j] != 0; /* the cell itself is not its neighbour */
                if (jr >= 0) count += row[jr] != 0;
            }
            int alive = a[i * cols + j] != 0;
            b[i * cols + j] = (uint8_t)(count == 3 || (alive && count == 2));
        }
    }
}

static uint64_t live_count(const uint8_t *a, int64_t rows, int64_t cols) {
    uint64_t c = 0;
#pragma omp parallel for reduction(+ : c) schedule(static)
    for (int64_t i = 0; i < rows * cols; ++i) c += a[i] != 0;
    return c;
}

int orc_life_run(uint8_t *a, int64_t rows, int64_t cols, int bc, int cond_kind,
                 int stable_window, int check_every, int64_t max_iter,
                 uint64_t *trace, int64_t trace_cap, orc_result *out) {
    if (!a || !out || rows < 1 || cols < 1 || check_every < 1 || max_iter < 1) return -1;
    if (bc != ORC_BC_TORUS && bc != ORC_BC_BOTTOM) return -1;
    if (cond_kind != ORC_COND_STABLE_FOR && cond_kind != ORC_COND_NEVER) return -1;
    if (cond_kind == ORC_COND_STABLE_FOR && stable_window < 1) return -1;
    size_t bytes = (size_t)(rows * cols);
    uint8_t *cur = (uint8_t *)malloc(bytes), *nxt = (uint8_t *)malloc(bytes);
    memcpy(cur, a, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    uint64_t prev = live_count(cur, rows, cols); /* s = init: count before the first sweep */
    int64_t n = 0;
    int run = 0, stop = 0;
    do {
        life_sweep(bc, cur, nxt, rows, cols);
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            uint64_t count = live_count(nxt, rows, cols);
            if (trace && out->checks < trace_cap) trace[out->checks] = count;
            out->checks += 1;
            run = (count == prev) ? run + 1 : 0;                     /* s = update */
            prev = count;
            out->count = count;
            out->r = (double)count;
            if (cond_kind == ORC_COND_STABLE_FOR && run >= stable_window) {
                out->converged = 1;
                stop = 1;
            }
        }
        uint8_t *t = cur; cur = nxt; nxt = t;
    } while (!stop && n < max_iter);
    memcpy(a, cur, bytes);
    out->n = n;
    out->run = run;
    free(cur);
    free(nxt);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Adaptive median detection (Sect. 4.3, first phase; window grown to a static
 * bound as Sect. 3.2 describes). Windows hold only in-range pixels.
 * ------------------------------------------------------------------------- */
static void insertion_sort_u8(uint8_t *v, int n) {
    for (int i = 1; i < n; ++i) {
        uint8_t x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) { v[j + 1] = v[j]; --j; }
        v[j + 1] = x;
    }
}

int orc_amf_detect(const uint8_t *y, int64_t rows, int64_t cols, int w_max,
                   uint8_t *mask, uint8_t *u0) {
    if (!y || !mask || !u0 || rows < 1 || cols < 1 || w_max < 3 || (w_max % 2) == 0) return -1;
#pragma omp parallel
    {
        uint8_t *win = (uint8_t *)malloc((size_t)w_max * (size_t)w_max);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < rows; ++i) {
            for (int64_t j = 0; j < cols; ++j) {
                uint8_t yv = y[i * cols + j], lo = 0, hi = 0, med = 0;
                int decided = 0;
                for (int w = 3; w <= w_max && !decided; w += 2) {
                    int k = w / 2, cnt = 0;
                    for (int64_t ii = i - k; ii <= i + k; ++ii) {
                        if (ii < 0 || ii >= rows) continue;
                        for (int64_t jj = j - k; jj <= j + k; ++jj) {
                            if (jj < 0 || jj >= cols) continue;
                            win[cnt++] = y[ii * cols + jj];
                        }
                    }
                    insertion_sort_u8(win, cnt);
                    lo = win[0];
                    hi = win[cnt - 1];
                    med = win[(cnt - 1) / 2];
                    if (lo < med && med < hi) {
                        mask[i * cols + j] = (uint8_t)!(lo < yv && yv < hi);
                        decided = 1;
                    }
                }
                if (!decided) mask[i * cols + j] = (uint8_t)(yv == lo || yv == hi);
                u0[i * cols + j] = mask[i * cols + j] ? med : yv;
            }
        }
        free(win);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Restoration update (Sect. 4.3, second phase): the value minimising the sum of
 * phi over the neighbourhood, i.e. the root of the (strictly increasing)
 * derivative sum phi'(t - v_m), found by bisection on [min v, max v].
 * ------------------------------------------------------------------------- */
static double dphi_sum(const double *v, int count, double t, double beta, int quadratic) {
    double s = 0.0;
    for (int m = 0; m < count; ++m) {
        double d = t - v[m];
        s = s + (quadratic ? 2.0 * d : d / sqrt(beta + d * d));
    }
    return s;
}

double orc_restore_argmin(const double *v, int count, double beta, int quadratic) {
    if (count <= 0) return NAN;
    double lo = v[0], hi = v[0];
    for (int m = 1; m < count; ++m) {
        if (v[m] < lo) lo = v[m];
        if (v[m] > hi) hi = v[m];
    }
    if (!(lo < hi)) return lo;
    for (;;) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        double gm = dphi_sum(v, count, mid, beta, quadratic);
        if (gm == 0.0) return mid;
        if (gm < 0.0) lo = mid; else hi = mid;
    }
    double glo = fabs(dphi_sum(v, count, lo, beta, quadratic));
    double ghi = fabs(dphi_sum(v, count, hi, beta, quadratic));
    return (glo <= ghi) ? lo : hi;
}

static void restore_sweep(const double *a, double *b, const uint8_t *mask, int64_t rows,
                          int64_t cols, double beta, int quadratic) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            int64_t p = i * cols + j;
            if (!mask[p]) { b[p] = a[p]; continue; }
            double v[8];
            int cnt = 0;
            for (int di = -1; di <= 1; ++di) {
                for (int dj = -1; dj <= 1; ++dj) {
                    if (di == 0 && dj == 0) continue;
                    int64_t ii = i + di, jj = j + dj;
                    if (ii < 0 || jj < 0 || ii >= rows || jj >= cols) continue; /* bottom */
                    v[cnt++] = a[ii * cols + jj];
                }
            }
            b[p] = cnt ? orc_restore_argmin(v, cnt, beta, quadratic) : a[p];
        }
    }
}

int orc_restore_run(double *u, const uint8_t *mask, int64_t rows, int64_t cols, double beta,
                    int quadratic, int reduce_op, int cond_kind, double thr, int check_every,
                    int64_t max_iter, double *trace, int64_t trace_cap, orc_result *out) {
    if (!u || !mask || !out || rows < 1 || cols < 1 || check_every < 1 || max_iter < 1) return -1;
    if (reduce_op != ORC_RED_MAX_ABS_DELTA && reduce_op != ORC_RED_MEAN_ABS_DELTA) return -1;
    if (cond_kind != ORC_COND_BELOW && cond_kind != ORC_COND_NEVER) return -1;
    size_t bytes = sizeof(double) * (size_t)(rows * cols);
    double *cur = (double *)malloc(bytes), *nxt = (double *)malloc(bytes);
    memcpy(cur, u, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    int64_t n = 0;
    int stop = 0;
    do {
        restore_sweep(cur, nxt, mask, rows, cols, beta, quadratic);
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            double r = reduce_delta(reduce_op, nxt, cur, rows, cols);
            if (trace && out->checks < trace_cap) trace[out->checks] = r;
            out->checks += 1;
            out->r = r;
            if (isnan(r) || isinf(r)) { out->numeric_error = 1; stop = 1; }
            else if (cond_kind == ORC_COND_BELOW && r < thr) { out->converged = 1; stop = 1; }
        }
        double *t = cur; cur = nxt; nxt = t;
    } while (!stop && n < max_iter);
    memcpy(u, cur, bytes);
    out->n = n;
    free(cur);
    free(nxt);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sobel edge detector (Sect. 4.2): a single-iteration stencil on a u8 image.  */
/* Gx and Gy are the two 3x3 Sobel derivative masks; a sample outside the     */
/* image is bottom and counts as 0 (the convention of Fig. 1). The output is  */
/* the gradient magnitude floor(sqrt(Gx^2 + Gy^2)) clamped to 255, computed   */
/* exactly in integers. The reduce is the plain variant over the new image:   */
/* the sum of its values (u64).                                               */
/* ------------------------------------------------------------------------- */

static int pixel_or_zero(const uint8_t *a, int64_t rows, int64_t cols, int64_t i, int64_t j) {
    if (i < 0 || j < 0 || i >= rows || j >= cols) return 0;
    return a[i * cols + j];
}

static int isqrt_floor(int m) {
    int s = 0;
    while ((s + 1) * (s + 1) <= m) s = s + 1;
    return s;
}

static void sobel_sweep(const uint8_t *a, uint8_t *b, int64_t rows, int64_t cols) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            int nw = pixel_or_zero(a, rows, cols, i - 1, j - 1);
            int n = pixel_or_zero(a, rows, cols, i - 1, j);
            int ne = pixel_or_zero(a, rows, cols, i - 1, j + 1);
            int w = pixel_or_zero(a, rows, cols, i, j - 1);
            int e = pixel_or_zero(a, rows, cols, i, j + 1);
            int sw = pixel_or_zero(a, rows, cols, i + 1, j - 1);
            int s = pixel_or_zero(a, rows, cols, i + 1, j);
            int se = pixel_or_zero(a, rows, cols, i + 1, j + 1);
            int gx = (ne + 2 * e + se) - (nw + 2 * w + sw);
            int gy = (sw + 2 * s + se) - (nw + 2 * n + ne);
            int mag = isqrt_floor(gx * gx + gy * gy);
            b[i * cols + j] = (uint8_t)(mag > 255 ? 255 : mag);
        }
    }
}

static uint64_t value_sum(const uint8_t *a, int64_t rows, int64_t cols) {
    uint64_t total = 0;
    for (int64_t i = 0; i < rows * cols; ++i) total += a[i];
    return total;
}

int orc_sobel_run(uint8_t *a, int64_t rows, int64_t cols, int check_every, int64_t max_iter,
                  uint64_t *trace, int64_t trace_cap, orc_result *out) {
    if (!a || !out || rows < 1 || cols < 1 || check_every < 1 || max_iter < 1) return -1;
    size_t bytes = (size_t)(rows * cols);
    uint8_t *cur = (uint8_t *)malloc(bytes), *nxt = (uint8_t *)malloc(bytes);
    memcpy(cur, a, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    int64_t n = 0;
    do {
        sobel_sweep(cur, nxt, rows, cols);
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            uint64_t total = value_sum(nxt, rows, cols);
            if (trace && out->checks < trace_cap) trace[out->checks] = total;
            out->checks += 1;
            out->count = total;
            out->r = (double)total;
        }
        uint8_t *t = cur; cur = nxt; nxt = t;
    } while (n < max_iter);
    memcpy(a, cur, bytes);
    out->n = n;
    free(cur);
    free(nxt);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Radius-k box stencil (sigma_k of Sect. 3.1 with k > 1): every cell at least */
/* k from the edge takes the mean of its (2k+1) x (2k+1) neighbourhood; the     */
/* outer band of width k is boundary data, never updated. Summation order:     */
/* each row of the box left to right, then the row sums top to bottom, then one */
/* division by the cell count (2k+1)^2.                                         */
/* ------------------------------------------------------------------------- */
static void box_sweep(const double *a, double *b, int64_t rows, int64_t cols, int k) {
    const double cnt = (double)((2 * k + 1) * (2 * k + 1));
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            int64_t p = i * cols + j;
            if (i < k || j < k || i >= rows - k || j >= cols - k) {
                b[p] = a[p];
                continue;
            }
            double total = 0.0;
            for (int di = -k; di <= k; ++di) {
                double row = 0.0;
                for (int dj = -k; dj <= k; ++dj) row = row + a[(i + di) * cols + (j + dj)];
                total = total + row;
            }
            b[p] = total / cnt;
        }
    }
}

int orc_box_run(double *a, int64_t rows, int64_t cols, int k, int reduce_op, int cond_kind,
                double thr, int check_every, int64_t max_iter, double *trace, int64_t trace_cap,
                orc_result *out) {
    if (!a || !out || k < 1 || rows < 2 * k + 1 || cols < 2 * k + 1 || check_every < 1 ||
        max_iter < 1) return -1;
    if (reduce_op != ORC_RED_MAX_ABS_DELTA && reduce_op != ORC_RED_L2_DELTA &&
        reduce_op != ORC_RED_MEAN_ABS_DELTA) return -1;
    if (cond_kind != ORC_COND_BELOW && cond_kind != ORC_COND_NEVER) return -1;
    size_t bytes = sizeof(double) * (size_t)(rows * cols);
    double *cur = (double *)malloc(bytes), *nxt = (double *)malloc(bytes);
    memcpy(cur, a, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    int64_t n = 0;
    int stop = 0;
    do {
        box_sweep(cur, nxt, rows, cols, k);
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            double r = reduce_delta(reduce_op, nxt, cur, rows, cols);
            if (trace && out->checks < trace_cap) trace[out->checks] = r;
            out->checks += 1;
            out->r = r;
            if (isnan(r) || isinf(r)) { out->numeric_error = 1; stop = 1; }
            else if (cond_kind == ORC_COND_BELOW && r < thr) { out->converged = 1; stop = 1; }
        }
        double *t = cur; cur = nxt; nxt = t;
    } while (!stop && n < max_iter);
    memcpy(a, cur, bytes);
    out->n = n;
    free(cur);
    free(nxt);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 3D 7-point Jacobi (Laplace): a grid of nz planes of ny rows of nx cells,     */
/* stored plane after plane; the six faces are boundary data. Interior update:  */
/* b = (((W + E) + (N + S)) + (U + D)) / 6, W/E along x, N/S along y, U/D along  */
/* z. reduce and condition as for the 2D Jacobi.                                */
/* ------------------------------------------------------------------------- */
static void jacobi3d_sweep(const double *a, double *b, int64_t nz, int64_t ny, int64_t nx) {
    const int64_t plane = ny * nx;
    int64_t z;
#pragma omp parallel for schedule(static)
    for (z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                int64_t p = z * plane + y * nx + x;
                if (z == 0 || y == 0 || x == 0 || z == nz - 1 || y == ny - 1 || x == nx - 1) {
                    b[p] = a[p];
                    continue;
                }
                double w = a[p - 1], e = a[p + 1], n = a[p - nx], s = a[p + nx];
                double u = a[p - plane], d = a[p + plane];
                b[p] = (((w + e) + (n + s)) + (u + d)) / 6.0;
            }
        }
    }
}

int orc_jacobi3d_run(double *a, int64_t nz, int64_t ny, int64_t nx, int reduce_op, int cond_kind,
                     double thr, int check_every, int64_t max_iter, double *trace,
                     int64_t trace_cap, orc_result *out) {
    if (!a || !out || nz < 3 || ny < 3 || nx < 3 || check_every < 1 || max_iter < 1) return -1;
    if (reduce_op != ORC_RED_MAX_ABS_DELTA && reduce_op != ORC_RED_L2_DELTA &&
        reduce_op != ORC_RED_MEAN_ABS_DELTA) return -1;
    if (cond_kind != ORC_COND_BELOW && cond_kind != ORC_COND_NEVER) return -1;
    size_t bytes = sizeof(double) * (size_t)(nz * ny * nx);
    double *cur = (double *)malloc(bytes), *nxt = (double *)malloc(bytes);
    memcpy(cur, a, bytes);
    memset(out, 0, sizeof *out);
    out->r = NAN;
    int64_t n = 0;
    int stop = 0;
    do {
        jacobi3d_sweep(cur, nxt, nz, ny, nx);
        n = n + 1;
        if (is_check_sweep(n, check_every, max_iter)) {
            /* the reduce runs over all cells; faces contribute a zero change */
            double r = reduce_delta(reduce_op, nxt, cur, nz * ny, nx);
            if (trace && out->checks < trace_cap) trace[out->checks] = r;
            out->checks += 1;
            out->r = r;
            if (isnan(r) || isinf(r)) { out->numeric_error = 1; stop = 1; }
            else if (cond_kind == ORC_COND_BELOW && r < thr) { out->converged = 1; stop = 1; }
        }
        double *t = cur; cur = nxt; nxt = t;
    } while (!stop && n < max_iter);
    memcpy(a, cur, bytes);
    out->n = n;
    free(cur);
    free(nxt);
    return 0;
}
