/*
 * CPU oracle for the loop-of-stencil-reduce pattern -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-pass-per-step CPU implementation of what the pattern
 * computes (Aldinucci et al., "A Parallel Pattern for Iterative Stencil +
 * Reduce", Sect. 3.1: the loop-of-stencil-reduce procedure and its -d, -i and -s
 * variants). Only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg may call it. It shares no code, header or constant with the GPU
 * library; inputs reach both sides as identical bytes from the seeded generators.
 *
 * Every array is host memory, row-major and dense (pitch == cols). All floating
 * point is IEEE double, built with -ffp-contract=off so the expression order
 * written here is the one evaluated.
 *
 * Pins (what each function is checked against, besides itself) are listed in the
 * test-suite. Parity unpinned by the paper: the restoration functional
 * phi(t) = sqrt(beta + t^2), the detection window bound w_max and the adaptive
 * median edge rules (the paper names the method but gives none of these); they
 * are pinned only by closed forms and brute force on small inputs.
 */
#ifndef LSR_ORACLE_H
#define LSR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_RED_MAX_ABS_DELTA = 1, ORC_RED_L2_DELTA = 2, ORC_RED_SUM = 3, ORC_RED_MEAN_ABS_DELTA = 4 };
enum { ORC_COND_BELOW = 1, ORC_COND_STABLE_FOR = 2, ORC_COND_NEVER = 3 };
enum { ORC_BC_RING = 0, ORC_BC_TORUS = 1, ORC_BC_BOTTOM = 2 };

typedef struct {
    int64_t n;              /* sweeps performed */
    double r;               /* reduce value at the last check (NaN if never checked) */
    uint64_t count;         /* life: live cells after the last sweep */
    int32_t converged;      /* 1 if the condition held at the stop */
    int32_t run;            /* life: consecutive checks with an unchanged count */
    int64_t checks;         /* number of checks evaluated */
    int32_t numeric_error;  /* 1 if r became NaN or Inf (the loop stops there) */
    int32_t pad;
} orc_result;

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int orc_threads(void);
void orc_set_threads(int n);

/*
 * 5-point Jacobi on a grid with a fixed boundary ring (Dirichlet data that is
 * never updated). helmholtz = 0: Laplace, b = 0.25*((N+S)+(W+E)).
 * helmholtz = 1: b = (((N+S)+(W+E)) + g) * rd with rd = 1/(4 + alpha*(h*h)),
 * g = h^2 f read from env (may be NULL for Laplace).
 * reduce: MAX_ABS_DELTA (max|b-a|), L2_DELTA (sqrt of the sum of (b-a)^2) or
 * MEAN_ABS_DELTA (sum|b-a| / (rows*cols)); ring cells contribute 0.
 * cond: BELOW (stop when r < thr) or NEVER. a is in/out; trace (may be NULL)
 * receives r at each check, up to trace_cap entries.
 * Returns 0, or -1 on bad arguments.
 */
int orc_jacobi_run(int helmholtz, double *a, const double *g, int64_t rows, int64_t cols,
                   double alpha, double h, int reduce_op, int cond_kind, double thr,
                   int check_every, int64_t max_iter, double *trace, int64_t trace_cap,
                   orc_result *out);

/*
 * The -i form of the Helmholtz sweep (Sect. 3.1: the elemental function also
 * receives the cell's index): the right-hand side is evaluated from the indices
 * as g(i, j) = c2 * (c1 * (p[i] * q[j])) instead of being read from an env
 * array; everything else as orc_jacobi_run with helmholtz = 1.
 */
int orc_jacobi_sep_run(double *a, const double *p, const double *q, double c1, double c2,
                       int64_t rows, int64_t cols, double alpha, double h, int reduce_op,
                       int cond_kind, double thr, int check_every, int64_t max_iter,
                       double *trace, int64_t trace_cap, orc_result *out);

/*
 * Conway's Life B3/S23 (the rule of the paper's Fig. 1). bc = TORUS wraps both
 * axes; bc = BOTTOM treats out-of-range cells as dead (Fig. 1's guards).
 * A cell is alive iff its byte is non-zero; the output holds 0/1.
 * reduce is the live-cell count of the new generation (u64).
 * cond: STABLE_FOR (stop once the count has been equal at stable_window
 * consecutive checks, the count before the first sweep being the initial
 * reference) or NEVER. trace receives the count at each check.
 */
int orc_life_run(uint8_t *a, int64_t rows, int64_t cols, int bc, int cond_kind,
                 int stable_window, int check_every, int64_t max_iter,
                 uint64_t *trace, int64_t trace_cap, orc_result *out);

/*
 * Adaptive-median impulse detection (phase 1 of the two-phase restoration,
 * Sect. 4.3). Per pixel, windows w = 3, 5, ..., w_max of in-range pixels;
 * lower median med = sorted[(cnt-1)/2]. The first w with min < med < max
 * decides: flag = !(min < y < max), init = med. If no window qualifies,
 * flag = (y == min || y == max) and init = med of the w_max window.
 * Writes mask (0/1) and init (u8).
 */
int orc_amf_detect(const uint8_t *y, int64_t rows, int64_t cols, int w_max,
                   uint8_t *mask, uint8_t *init);

/*
 * Phase 2: each flagged pixel p takes argmin_t sum_{m in V_p} phi(t - u_m) over
 * its in-range 8-neighbourhood V_p, from the previous iterate only (Jacobi).
 * phi(t) = sqrt(beta + t^2) (quadratic = 0) or t^2 (quadratic = 1, test form).
 * The root of the derivative is found by bisection on [min v, max v] until the
 * midpoint equals an end point. Unflagged pixels never change.
 * reduce: MAX_ABS_DELTA or MEAN_ABS_DELTA over the whole image.
 */
int orc_restore_run(double *u, const uint8_t *mask, int64_t rows, int64_t cols, double beta,
                    int quadratic, int reduce_op, int cond_kind, double thr, int check_every,
                    int64_t max_iter, double *trace, int64_t trace_cap, orc_result *out);

/* One restoration update of a single pixel from explicit neighbour values. */
double orc_restore_argmin(const double *v, int count, double beta, int quadratic);

/*
 * Sobel edge detector (Sect. 4.2) as a loop-of-stencil-reduce on a u8 image:
 * each sweep writes floor(sqrt(Gx^2 + Gy^2)) clamped to 255 for every pixel,
 * where Gx, Gy are the 3x3 Sobel derivative masks and samples outside the image
 * are 0; at a check (every check_every sweeps and at max_iter) the reduce is the
 * sum of the new image's values (u64, in out->count and out->r). The paper's use
 * is max_iter = 1. a is updated in place with the last image.
 */
int orc_sobel_run(uint8_t *a, int64_t rows, int64_t cols, int check_every, int64_t max_iter,
                  uint64_t *trace, int64_t trace_cap, orc_result *out);

/*
 * Radius-k box stencil (sigma_k, k >= 1): cells at least k from the edge take the
 * mean of their (2k+1)^2 neighbourhood (rows of the box summed left to right, the
 * row sums top to bottom, one division by (2k+1)^2); the band of width k at the
 * edge is fixed. reduce / cond as orc_jacobi_run.
 */
int orc_box_run(double *a, int64_t rows, int64_t cols, int k, int reduce_op, int cond_kind,
                double thr, int check_every, int64_t max_iter, double *trace, int64_t trace_cap,
                orc_result *out);

/*
 * 3D 7-point Jacobi on nz planes of ny x nx cells (plane after plane, row-major);
 * the faces are fixed; b = (((W+E) + (N+S)) + (U+D)) / 6 inside. reduce / cond as
 * orc_jacobi_run, over all cells.
 */
int orc_jacobi3d_run(double *a, int64_t nz, int64_t ny, int64_t nx, int reduce_op, int cond_kind,
                     double thr, int check_every, int64_t max_iter, double *trace,
                     int64_t trace_cap, orc_result *out);

#ifdef __cplusplus
}
#endif
#endif
