/*
 * si_oracle.c -- FP64 reference for spin-image generation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only tests, the smoke check and the benchmark's CPU
 * baseline may build, load or call it; the library never does, and the two
 * share no code.
 *
 * What it computes is the plain definition of the parallel spin-image
 * algorithm (Section 2.1, Algorithm 1; the same body restricted to
 * [start, end) is Algorithm 2): for each of the N chosen oriented points
 * P = (p, n) and for every one of the M oriented points X = (x, n_x),
 *
 *   c     = n . n_x                          support-angle test on the normals
 *   beta  = n . (x - p)                      signed height above P's tangent plane
 *   alpha = sqrt(|x - p|^2 - beta^2)         distance from P's normal axis
 *
 * X contributes to P's W x W image if the angle between the normals is at
 * most S and its bin lies inside the image.  Everything is evaluated in
 * double precision from the float32 inputs (widening is exact).
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *   - angle test acos(c) <= S is evaluated as c >= cos(S), the same predicate
 *     for S in [0, pi]; for S >= pi every pair passes (the paper runs with
 *     S = 2 pi, Section 4.1);
 *   - the row coordinate is v = W/2 - beta/B, i.e. the dimensionally
 *     consistent form of the printed (W/2 - beta)/B, and the column
 *     coordinate is u = alpha/B;
 *   - the inner loop runs over all M points, so the self-pair (x = p) counts;
 *   - normals are used as given, not renormalised;
 *   - SI_BIN_CEIL is the printed binning: k = ceil(v), l = ceil(u), counted
 *     if 0 <= k < W and 0 <= l < W, image[k][l] += 1;
 *   - SI_BIN_BILINEAR spreads a unit weight over the four grid nodes around
 *     (v, u) (Johnson's bilinear interpolation, which this paper does not
 *     print); a pair counts only if the whole 2x2 footprint lies inside the
 *     image, 0 <= v < W-1 and u < W-1, so image mass equals the count.
 *
 * Boundary flags.  Float32 evaluation may legitimately decide differently
 * from float64 for pairs that lie within eps of a decision boundary.  With
 * eps > 0, every condition whose argument lies within eps of its threshold is
 * "unsure".  A pair with a surely-false condition is out; a pair whose
 * outcome depends on an unsure support condition is ambiguous (counted in
 * cnt_amb, excluded from img_sure, and every bin it might touch gets
 * touch += 1).  In ceil mode a surely-in pair whose bin is unsure (beta or
 * alpha within eps of a bin edge, or 0 < |alpha^2| < 1e-6 near the axis) is
 * counted in cnt_sure but, too, only recorded in touch.  eps = 0 turns all
 * flags off (designed inputs whose values are exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define SIO_BILINEAR 0
#define SIO_CEIL 1

/* condition states */
#define C_FALSE 0
#define C_TRUE 1
#define C_UNSURE 2

static int cond(int value, double dist, double eps)
{
    if (eps > 0.0 && fabs(dist) < eps)
        return C_UNSURE;
    return value ? C_TRUE : C_FALSE;
}

static void touch_box(int32_t* t, int W, long r0, long r1, long c0, long c1)
{
    if (!t)
        return;
    if (r0 < 0) r0 = 0;
    if (c0 < 0) c0 = 0;
    if (r1 > W - 1) r1 = W - 1;
    if (c1 > W - 1) c1 = W - 1;
    for (long r = r0; r <= r1; ++r)
        for (long c = c0; c <= c1; ++c)
            t[r * W + c] += 1;
}

/*
 * Returns 0 on success, -1 on invalid arguments.
 *   xyz, nrm : M x 3 float32, row-major
 *   idx      : N int32 indices into [0, M)
 *   img_sure : N x W x W doubles (zeroed here)
 *   cnt_sure, cnt_amb : N int64 each
 *   touch    : N x W x W int32 (zeroed here) or NULL
 */
/* Everything one image's loop needs (the widened thresholds of its call). */
typedef struct {
    const float* xyz;
    const float* nrm;
    int64_t M;
    const int32_t* idx;
    int32_t W;
    int32_t mode;
    double eps, B, cosS, half, WW, beta_hi, beta_lo, alpha_max;
    int vacuous;
    double* img_sure;
    int64_t* cnt_sure;
    int64_t* cnt_amb;
    int32_t* touch;
} Job;

/* Checks the arguments and fills the job; 0 or -1. */
static int make_job(Job* jb, const float* xyz, const float* nrm, int64_t M,
                    const int32_t* idx, int64_t N, int32_t W, float bin,
                    float support_angle, int32_t mode, double eps, double* img_sure,
                    int64_t* cnt_sure, int64_t* cnt_amb, int32_t* touch)
{
    if (M <= 0 || N < 0 || W < 1 || !(bin > 0.0f) || !(support_angle >= 0.0f))
        return -1;
    if (mode != SIO_BILINEAR && mode != SIO_CEIL)
        return -1;
    for (int64_t i = 0; i < N; ++i)
        if (idx[i] < 0 || idx[i] >= M)
            return -1;
    jb->xyz = xyz;
    jb->nrm = nrm;
    jb->M = M;
    jb->idx = idx;
    jb->W = W;
    jb->mode = mode;
    jb->eps = eps;
    jb->B = (double)bin;
    const double S = (double)support_angle;
    jb->vacuous = S >= M_PI;
    jb->cosS = cos(S);
    jb->half = 0.5 * (double)W;
    jb->WW = (double)W;
    /* support thresholds in scene units */
    jb->beta_hi = (mode == SIO_CEIL) ? jb->B * (jb->half + 1.0) : jb->B * jb->half;
    jb->beta_lo = jb->B * (1.0 - jb->half);
    jb->alpha_max = jb->B * (jb->WW - 1.0);
    jb->img_sure = img_sure;
    jb->cnt_sure = cnt_sure;
    jb->cnt_amb = cnt_amb;
    jb->touch = touch;
    return 0;
}

/* One image's running state: P = (p, n), its image, touch counts and counts. */
typedef struct {
    double px, py, pz, nx, ny, nz;
    double* img;
    int32_t* tch;
    int64_t sure, amb;
} ImageAcc;

static void image_begin(const Job* jb, int64_t i, ImageAcc* a)
{
    const int32_t W = jb->W;
    a->img = jb->img_sure + (size_t)i * W * W;
    a->tch = jb->touch ? jb->touch + (size_t)i * W * W : NULL;
    memset(a->img, 0, sizeof(double) * (size_t)W * W);
    if (a->tch)
        memset(a->tch, 0, sizeof(int32_t) * (size_t)W * W);
    a->sure = 0;
    a->amb = 0;
    const int64_t pi = jb->idx[i];
    a->px = jb->xyz[3 * pi];
    a->py = jb->xyz[3 * pi + 1];
    a->pz = jb->xyz[3 * pi + 2];
    a->nx = jb->nrm[3 * pi];
    a->ny = jb->nrm[3 * pi + 1];
    a->nz = jb->nrm[3 * pi + 2];
}

static void image_end(const Job* jb, int64_t i, const ImageAcc* a)
{
    jb->cnt_sure[i] = a->sure;
    jb->cnt_amb[i] = a->amb;
}

/* The body of Algorithm 1's inner loop: the pair (P, X_j). */
static inline void pair_update(const Job* jb, ImageAcc* a, int64_t j)
{
    const float* xyz = jb->xyz;
    const float* nrm = jb->nrm;
    const int32_t W = jb->W;
    const double eps = jb->eps, B = jb->B, cosS = jb->cosS, half = jb->half, WW = jb->WW;
    const double beta_hi = jb->beta_hi, beta_lo = jb->beta_lo, alpha_max = jb->alpha_max;
    const int vacuous = jb->vacuous;
    const int32_t mode = jb->mode;
    double* img = a->img;
    int32_t* tch = a->tch;
    const double px = a->px, py = a->py, pz = a->pz;
    const double nx = a->nx, ny = a->ny, nz = a->nz;

    const double qx = xyz[3 * j], qy = xyz[3 * j + 1], qz = xyz[3 * j + 2];
    const double mx = nrm[3 * j], my = nrm[3 * j + 1], mz = nrm[3 * j + 2];

    const double c = nx * mx + ny * my + nz * mz;
    const double dx = qx - px, dy = qy - py, dz = qz - pz;
    const double beta = nx * dx + ny * dy + nz * dz;
    const double dd = dx * dx + dy * dy + dz * dz;
    const double a2 = dd - beta * beta;
    const double alpha = sqrt(a2 > 0.0 ? a2 : 0.0);
    const double v = half - beta / B;
    const double u = alpha / B;

    int ca = vacuous ? C_TRUE : cond(c >= cosS, c - cosS, eps);
    int c1, c2, c3;
    if (mode == SIO_CEIL) {
        const double kk = ceil(v), ll = ceil(u);
        c1 = cond(kk >= 0.0, beta - beta_hi, eps);      /* k >= 0 */
        c2 = cond(kk < WW, beta - beta_lo, eps);        /* k < W  */
        c3 = cond(ll >= 0.0 && ll < WW, alpha - alpha_max, eps);
    } else {
        c1 = cond(v >= 0.0, beta - beta_hi, eps);
        c2 = cond(v < WW - 1.0, beta - beta_lo, eps);
        c3 = cond(u < WW - 1.0, alpha - alpha_max, eps);
    }
    if (ca == C_FALSE || c1 == C_FALSE || c2 == C_FALSE || c3 == C_FALSE)
        return;
    const int unsure = (ca == C_UNSURE) || (c1 == C_UNSURE) ||
                       (c2 == C_UNSURE) || (c3 == C_UNSURE);

    if (mode == SIO_CEIL) {
        const long k = (long)ceil(v), l = (long)ceil(u);
        if (unsure) {
            ++a->amb;
            touch_box(tch, W, k - 1, k + 1, l - 1, l + 1);
            return;
        }
        ++a->sure;
        int row_unsure = 0, col_unsure = 0;
        /* x == p (the self-pair, duplicate points) is exact in any
           precision: beta = alpha = 0, never ambiguous */
        if (eps > 0.0 && (dx != 0.0 || dy != 0.0 || dz != 0.0)) {
            const double m = nearbyint(v);             /* nearest row edge */
            row_unsure = fabs(beta - B * (half - m)) < eps;
            const double q = nearbyint(u);             /* nearest column edge */
            col_unsure = (q >= 1.0 && fabs(alpha - B * q) < eps) ||
                         (a2 != 0.0 && fabs(a2) < 1e-6);
        }
        if (row_unsure || col_unsure) {
            touch_box(tch, W, row_unsure ? k - 1 : k, row_unsure ? k + 1 : k,
                      col_unsure ? l - 1 : l, col_unsure ? l + 1 : l);
        } else {
            img[k * W + l] += 1.0;
        }
    } else {
        const double fi = floor(v), fj = floor(u);
        if (unsure) {
            ++a->amb;
            touch_box(tch, W, (long)fi - 1, (long)fi + 2, (long)fj - 1, (long)fj + 2);
            return;
        }
        ++a->sure;
        const long i0 = (long)fi, j0 = (long)fj;
        const double wa = v - fi, wb = u - fj;
        img[i0 * W + j0] += (1.0 - wa) * (1.0 - wb);
        img[(i0 + 1) * W + j0] += wa * (1.0 - wb);
        img[i0 * W + j0 + 1] += (1.0 - wa) * wb;
        img[(i0 + 1) * W + j0 + 1] += wa * wb;
    }
}

/* The inner loop of Algorithm 1 for image i: P = OP[idx[i]] against all M points. */
static void one_image(const Job* jb, int64_t i)
{
    ImageAcc a;
    image_begin(jb, i, &a);
    for (int64_t j = 0; j < jb->M; ++j)
        pair_update(jb, &a, j);
    image_end(jb, i, &a);
}

/*
 * Returns 0 on success, -1 on invalid arguments.
 *   xyz, nrm : M x 3 float32, row-major
 *   idx      : N int32 indices into [0, M)
 *   img_sure : N x W x W doubles (zeroed here)
 *   cnt_sure, cnt_amb : N int64 each
 *   touch    : N x W x W int32 (zeroed here) or NULL
 */
int sio_generate(const float* xyz, const float* nrm, int64_t M,
                 const int32_t* idx, int64_t N,
                 int32_t W, float bin, float support_angle, int32_t mode,
                 double eps, double* img_sure, int64_t* cnt_sure,
                 int64_t* cnt_amb, int32_t* touch, int32_t nthreads)
{
    Job jb;
    if (make_job(&jb, xyz, nrm, M, idx, N, W, bin, support_angle, mode, eps, img_sure,
                 cnt_sure, cnt_amb, touch) != 0)
        return -1;
    (void)nthreads;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t i = 0; i < N; ++i)
        one_image(&jb, i);
    return 0;
}

/*
 * The same loop with its iterations distributed over the host threads by a
 * loop-scheduling technique of Section 2.2 (the paper's experiment on one
 * node, threads in place of MPI workers):
 *   sched 0  STATIC: one contiguous, balanced block per thread;
 *   sched 1  SS: one iteration per request;
 *   sched 2  GSS: each request takes ceil(remaining / threads) iterations
 *            (OpenMP's guided schedule with chunk 1);
 *   sched 3  a table of chunks: chunk_starts[0..n_chunks] ascending from 0
 *            to N, chunks requested one at a time (FAC2 from the table).
 * Results are those of sio_generate; returns -1 on invalid arguments.
 */
int sio_generate_sched(const float* xyz, const float* nrm, int64_t M,
                       const int32_t* idx, int64_t N,
                       int32_t W, float bin, float support_angle, int32_t mode,
                       double eps, double* img_sure, int64_t* cnt_sure,
                       int64_t* cnt_amb, int32_t* touch, int32_t nthreads,
                       int32_t sched, const int64_t* chunk_starts, int64_t n_chunks)
{
    Job jb;
    if (make_job(&jb, xyz, nrm, M, idx, N, W, bin, support_angle, mode, eps, img_sure,
                 cnt_sure, cnt_amb, touch) != 0)
        return -1;
    if (sched < 0 || sched > 3)
        return -1;
    if (sched == 3) {
        if (!chunk_starts || n_chunks < 0 || chunk_starts[0] != 0 ||
            chunk_starts[n_chunks] != N)
            return -1;
        for (int64_t c = 0; c < n_chunks; ++c)
            if (chunk_starts[c + 1] < chunk_starts[c])
                return -1;
    }
    (void)nthreads;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    if (sched == 3) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < n_chunks; ++c)
            for (int64_t i = chunk_starts[c]; i < chunk_starts[c + 1]; ++i)
                one_image(&jb, i);
        return 0;
    }
    omp_set_schedule(sched == 0 ? omp_sched_static
                     : sched == 1 ? omp_sched_dynamic : omp_sched_guided,
                     sched == 0 ? 0 : 1);
#pragma omp parallel for schedule(runtime)
    for (int64_t i = 0; i < N; ++i)
        one_image(&jb, i);
#else
    for (int64_t i = 0; i < N; ++i)
        one_image(&jb, i);
#endif
    return 0;
}

/*
 * Grid-accelerated form of sio_generate, for scenes where brute force is too
 * slow (millions of images): the same pair arithmetic (pair_update) applied
 * to the points of the 7 x 7 x 7 block of grid cells around p's cell only.
 * No pair outside that block can change the result:
 *   - every pair that is surely in support, or flagged, has |x - p| below
 *     R_c = sqrt(max(|beta_hi|, |beta_lo|)^2 + alpha_max^2) + 4 eps, because
 *     beta must lie within eps of [beta_lo, beta_hi] and alpha within eps
 *     below alpha_max (otherwise one extent condition is surely false);
 *   - the cells are cubes of edge h >= (R_c (1 + 1e-6) + 1e-9) / 3 over the
 *     bounding box of the finite points, so a point within R_c of p lies in
 *     a cell at most three steps from p's along every axis;
 *   - points with a non-finite coordinate are never in support and never
 *     flagged (every comparison with NaN or an infinite distance is false),
 *     and an image whose P is not finite is empty: both are left out.
 * Counts, ambiguous counts and touch counts are therefore identical to
 * sio_generate; image bins are the same sums taken in another order (cells
 * in z, y, x order, points in index order within a cell), so they agree to
 * FP64 rounding.  The grid is coarsened while it would exceed 2^26 cells.
 * Returns -1 on invalid arguments, -2 when memory runs out.
 */
int sio_generate_grid(const float* xyz, const float* nrm, int64_t M,
                      const int32_t* idx, int64_t N,
                      int32_t W, float bin, float support_angle, int32_t mode,
                      double eps, double* img_sure, int64_t* cnt_sure,
                      int64_t* cnt_amb, int32_t* touch, int32_t nthreads)
{
    Job jb;
    if (make_job(&jb, xyz, nrm, M, idx, N, W, bin, support_angle, mode, eps, img_sure,
                 cnt_sure, cnt_amb, touch) != 0)
        return -1;
    const double bmax = fmax(fabs(jb.beta_hi), fabs(jb.beta_lo));
    const double Rc = sqrt(bmax * bmax + jb.alpha_max * jb.alpha_max) + 4.0 * (eps > 0 ? eps : 0);
    const int64_t reach = 3;
    double h = (Rc * (1.0 + 1e-6) + 1e-9) / (double)reach;

    /* bounding box of the finite points */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = 0; j < M; ++j) {
        const double x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z))
            continue;
        const double q[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            if (q[a] < lo[a]) lo[a] = q[a];
            if (q[a] > hi[a]) hi[a] = q[a];
        }
    }
    int any = lo[0] <= hi[0];
    int64_t dims[3] = {1, 1, 1};
    if (any) {
        for (;;) {
            double cells = 1.0;
            for (int a = 0; a < 3; ++a) {
                dims[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
                cells *= (double)dims[a];
            }
            if (cells <= (double)(1 << 26))
                break;
            h *= cbrt(cells / (double)(1 << 26)) * 1.01;
        }
    }
    const int64_t ncell = dims[0] * dims[1] * dims[2];
    int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
    int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* pts = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
    if (!cell_of || !start || !pts) {
        free(cell_of);
        free(start);
        free(pts);
        return -2;
    }
    for (int64_t j = 0; j < M; ++j) {
        const double q[3] = {xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2]};
        if (!any || !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2])) {
            cell_of[j] = -1;
            continue;
        }
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int64_t)floor((q[a] - lo[a]) / h);
            if (c[a] < 0) c[a] = 0;
            if (c[a] > dims[a] - 1) c[a] = dims[a] - 1;
        }
        cell_of[j] = (c[2] * dims[1] + c[1]) * dims[0] + c[0];
        start[cell_of[j] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c)
        start[c + 1] += start[c];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
        if (!fill) {
            free(cell_of);
            free(start);
            free(pts);
            return -2;
        }
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t j = 0; j < M; ++j)
            if (cell_of[j] >= 0)
                pts[fill[cell_of[j]]++] = j;
        free(fill);
    }
    (void)nthreads;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < N; ++i) {
        ImageAcc acc;
        image_begin(&jb, i, &acc);
        const int64_t pc = cell_of[idx[i]];
        if (pc >= 0) {
            const int64_t cx = pc % dims[0], cy = (pc / dims[0]) % dims[1],
                          cz = pc / (dims[0] * dims[1]);
            for (int64_t z = cz - reach; z <= cz + reach; ++z) {
                if (z < 0 || z >= dims[2]) continue;
                for (int64_t y = cy - reach; y <= cy + reach; ++y) {
                    if (y < 0 || y >= dims[1]) continue;
                    for (int64_t x = cx - reach; x <= cx + reach; ++x) {
                        if (x < 0 || x >= dims[0]) continue;
                        const int64_t c = (z * dims[1] + y) * dims[0] + x;
                        for (int64_t k = start[c]; k < start[c + 1]; ++k)
                            pair_update(&jb, &acc, pts[k]);
                    }
                }
            }
        }
        image_end(&jb, i, &acc);
    }
    free(cell_of);
    free(start);
    free(pts);
    return 0;
}

int sio_abi_version(void) { return 1; }

/* threads an OpenMP parallel region of this library would use */
int sio_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
