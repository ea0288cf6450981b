/*
 * FP64 CPU oracle for ABX discriminability -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the bench's CPU-baseline leg load
 * this file's shared library.  The HIP library never includes, links or calls
 * it, and it shares no code with the HIP library.
 *
 * What it computes (plain definitions, FP64, no blocking or reordering):
 *   - angular distance between two frames (the distance named "angular" in the
 *     Score interface, library-overview section), as theta/pi with theta the
 *     angle between the two vectors;
 *   - the DTW alignment cost between two frame sequences (the recurrence of
 *     the "Dynamic Time Warping on GPU" section), optionally divided by the
 *     length of the optimal alignment path;
 *   - the time-pooled alternative (same section: "pool along the time
 *     domain"): angular distance of the per-item mean frames;
 *   - the Euclidean distance between two frames (the Score interface names
 *     "euclidean" beside "angular"): the square root of the sequential sum of
 *     squared differences, on the raw frames (or raw means), in either mode;
 *   - for discrete units (the paper says ABX works with discrete
 *     representations but gives no distance for them): frames are unit codes
 *     (D = 1) and the frame distance is 0 for equal codes, 1 otherwise; DTW
 *     mode only.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every sum is the plain sequential sum written below).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* pi rounded to the nearest double */
#define ORACLE_PI 3.14159265358979323846
#define ORACLE_OK 0
#define ORACLE_EDOMAIN (-3)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EINVAL (-1)

/* ---------------------------------------------------------------- frames -- */

/* u / ||u|| with ||u|| = sqrt of the sequential sum of squares (FP64).
 * Returns ORACLE_EDOMAIN for a zero vector: the angle is undefined there. */
static int unit_from_f64(const double *u, int D, double *out)
{
    double s = 0.0;
    for (int k = 0; k < D; ++k)
        s += u[k] * u[k];
    double n = sqrt(s);
    if (!(n > 0.0))
        return ORACLE_EDOMAIN;
    for (int k = 0; k < D; ++k)
        out[k] = u[k] / n;
    return ORACLE_OK;
}

static int unit_from_f32(const float *u, int D, double *tmp, double *out)
{
    for (int k = 0; k < D; ++k)
        tmp[k] = (double)u[k];
    return unit_from_f64(tmp, D, out);
}

/* Angle between two unit vectors, divided by pi (so the distance lies in
 * [0, 1]).  Where |cos| is close to 1, acos loses accuracy, so the angle is
 * taken from the half-chord form theta = 2 atan2(|u - v|, |u + v|), which is
 * exact 0 for identical vectors and exact pi for opposite ones. */
static double angular_unit(const double *u, const double *v, int D)
{
    double c = 0.0;
    for (int k = 0; k < D; ++k)
        c += u[k] * v[k];
    double theta;
    if (fabs(c) < 1.0 - 0x1p-20) {
        theta = acos(c);
    } else {
        double sm = 0.0, sp = 0.0;
        for (int k = 0; k < D; ++k) {
            double dm = u[k] - v[k];
            double dp = u[k] + v[k];
            sm += dm * dm;
            sp += dp * dp;
        }
        theta = 2.0 * atan2(sqrt(sm), sqrt(sp));
    }
    return theta / ORACLE_PI;
}

/* Euclidean distance of two raw vectors: sqrt of the sequential sum of
 * (u_k - v_k)^2. */
static double euclidean(const double *u, const double *v, int D)
{
    double s = 0.0;
    for (int k = 0; k < D; ++k) {
        double d = u[k] - v[k];
        s += d * d;
    }
    return sqrt(s);
}

/* Discrete units: 0 when the two codes are equal, else 1. */
static double unit_mismatch(const double *u, const double *v)
{
    return u[0] == v[0] ? 0.0 : 1.0;
}

/* Exported for the closed-form pins: distance of two raw vectors
 * (distance 0 = angular, 1 = Euclidean, 2 = unit mismatch with D = 1). */
int oracle_frame_distance(const double *u, const double *v, int D, int distance, double *out)
{
    if (D <= 0 || distance < 0 || distance > 2 || (distance == 2 && D != 1))
        return ORACLE_EINVAL;
    if (distance == 2) {
        *out = unit_mismatch(u, v);
        return ORACLE_OK;
    }
    if (distance == 1) {
        *out = euclidean(u, v, D);
        return ORACLE_OK;
    }
    double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)D);
    if (!buf)
        return ORACLE_ENOMEM;
    int rc = unit_from_f64(u, D, buf);
    if (rc == ORACLE_OK)
        rc = unit_from_f64(v, D, buf + D);
    if (rc == ORACLE_OK)
        *out = angular_unit(buf, buf + D, D);
    free(buf);
    return rc;
}

/* ------------------------------------------------------------------- DTW -- */

/*
 * DTW over a frame-distance matrix d[N][M] (rows = x frames, cols = y frames).
 *   c[0][0] = d[0][0]
 *   c[i][0] = c[i-1][0] + d[i][0],  c[0][j] = c[0][j-1] + d[0][j]
 *   c[i][j] = d[i][j] + min(c[i-1][j-1], c[i][j-1], c[i-1][j])   (i, j >= 1)
 * The predecessor is the first of (diagonal, left, up) that attains the
 * minimum; len counts the cells of the path that follows predecessors back to
 * (0, 0).  norm == 0 returns c[N-1][M-1] / len, norm == 1 returns c[N-1][M-1].
 */
int oracle_dtw(const double *d, int N, int M, int norm, double *out, int64_t *len_out)
{
    if (N <= 0 || M <= 0)
        return ORACLE_EINVAL;
    double *c = (double *)malloc(sizeof(double) * (size_t)N * M);
    int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * M);
    if (!c || !len) {
        free(c);
        free(len);
        return ORACLE_ENOMEM;
    }
    c[0] = d[0];
    len[0] = 1;
    for (int i = 1; i < N; ++i) {
        c[(size_t)i * M] = c[(size_t)(i - 1) * M] + d[(size_t)i * M];
        len[(size_t)i * M] = i + 1;
    }
    for (int j = 1; j < M; ++j) {
        c[j] = c[j - 1] + d[j];
        len[j] = j + 1;
    }
    for (int i = 1; i < N; ++i) {
        for (int j = 1; j < M; ++j) {
            size_t here = (size_t)i * M + j;
            size_t dg = (size_t)(i - 1) * M + (j - 1);
            size_t lf = (size_t)i * M + (j - 1);
            size_t up = (size_t)(i - 1) * M + j;
            size_t pred;
            if (c[dg] <= c[lf] && c[dg] <= c[up])
                pred = dg;
            else if (c[lf] <= c[up])
                pred = lf;
            else
                pred = up;
            c[here] = d[here] + c[pred];
            len[here] = len[pred] + 1;
        }
    }
    size_t last = (size_t)N * M - 1;
    if (len_out)
        *len_out = len[last];
    *out = norm == 0 ? c[last] / (double)len[last] : c[last];
    free(c);
    free(len);
    return ORACLE_OK;
}

/* ----------------------------------------------------- per-group pairs -- */

/*
 * Item-pair distances, one BY group at a time.
 *
 * feat      float32 [n_frames][D] (bf16 inputs are widened exactly by the caller)
 * offsets   int64 [n_items + 1]: frames of item i are offsets[i] .. offsets[i+1]-1
 * gptr      int64 [n_groups + 1] into gitems: the items of group g
 * gitems    int64 item ids
 * pptr      int64 [n_groups + 1] into px / py / out: the pairs of group g
 * px, py    int32 positions inside the group's item list (x = rows, y = cols)
 * mode      0 = DTW over frames, 1 = distance of mean frames
 * norm      0 = divide by path length, 1 = raw cost (DTW mode only)
 * distance  0 = angular (frames or means made unit first), 1 = Euclidean
 *           (raw frames or means)
 * out       float64 distances, one per pair
 * bad_item  on ORACLE_EDOMAIN, an item holding a zero frame (or zero mean)
 *
 * Groups run in parallel (OpenMP); each pair is plain sequential code.
 */
int oracle_pair_distances(const float *feat, const int64_t *offsets, int D,
                          int64_t n_groups, const int64_t *gptr, const int64_t *gitems,
                          const int64_t *pptr, const int32_t *px, const int32_t *py,
                          int mode, int norm, int distance, double *out, int64_t *bad_item)
{
    int status = ORACLE_OK;
    if (D <= 0 || n_groups < 0 || distance < 0 || distance > 2 || (distance == 2 && (D != 1 || mode != 0)))
        return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < n_groups; ++g) {
        int local_status;
#pragma omp atomic read
        local_status = status;
        if (local_status != ORACLE_OK)
            continue;
        int64_t n = gptr[g + 1] - gptr[g];
        const int64_t *items = gitems + gptr[g];
        /* frames (DTW) or means (pooled) of every item in the group: made
           unit for the angular distance, kept raw for the Euclidean one */
        int64_t *ustart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        ustart[0] = 0;
        for (int64_t a = 0; a < n; ++a) {
            int64_t L = offsets[items[a] + 1] - offsets[items[a]];
            ustart[a + 1] = ustart[a] + (mode == 0 ? L : 1);
        }
        double *uf = (double *)malloc(sizeof(double) * (size_t)ustart[n] * D);
        double *tmp = (double *)malloc(sizeof(double) * (size_t)D);
        int rc = ORACLE_OK;
        for (int64_t a = 0; a < n && rc == ORACLE_OK; ++a) {
            int64_t it = items[a];
            int64_t f0 = offsets[it], L = offsets[it + 1] - offsets[it];
            if (mode == 0) {
                for (int64_t t = 0; t < L && rc == ORACLE_OK; ++t) {
                    const float *f = feat + (size_t)(f0 + t) * D;
                    double *u = uf + (size_t)(ustart[a] + t) * D;
                    if (distance >= 1)
                        for (int k = 0; k < D; ++k)
                            u[k] = (double)f[k];
                    else
                        rc = unit_from_f32(f, D, tmp, u);
                }
            } else {
                for (int k = 0; k < D; ++k)
                    tmp[k] = 0.0;
                for (int64_t t = 0; t < L; ++t)
                    for (int k = 0; k < D; ++k)
                        tmp[k] += (double)feat[(size_t)(f0 + t) * D + k];
                for (int k = 0; k < D; ++k)
                    tmp[k] = tmp[k] / (double)L;
                double *u = uf + (size_t)ustart[a] * D;
                if (distance == 1)
                    memcpy(u, tmp, sizeof(double) * (size_t)D);
                else
                    rc = unit_from_f64(tmp, D, u);
            }
            if (rc != ORACLE_OK && bad_item) {
#pragma omp critical
                *bad_item = it;
            }
        }
        if (rc == ORACLE_OK) {
            double *dm = NULL;
            size_t dm_cap = 0;
            for (int64_t p = pptr[g]; p < pptr[g + 1]; ++p) {
                int64_t a = px[p], b = py[p];
                const double *ux = uf + (size_t)ustart[a] * D;
                const double *uy = uf + (size_t)ustart[b] * D;
                if (mode == 1) {
                    out[p] = distance == 1 ? euclidean(ux, uy, D) : angular_unit(ux, uy, D);
                    continue;
                }
                int N = (int)(ustart[a + 1] - ustart[a]);
                int M = (int)(ustart[b + 1] - ustart[b]);
                if ((size_t)N * M > dm_cap) {
                    dm_cap = (size_t)N * M;
                    free(dm);
                    dm = (double *)malloc(sizeof(double) * dm_cap);
                }
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < M; ++j)
                        dm[(size_t)i * M + j] =
                            distance == 2   ? unit_mismatch(ux + (size_t)i * D, uy + (size_t)j * D)
                            : distance == 1 ? euclidean(ux + (size_t)i * D, uy + (size_t)j * D, D)
                                            : angular_unit(ux + (size_t)i * D, uy + (size_t)j * D, D);
                oracle_dtw(dm, N, M, norm, &out[p], NULL);
            }
            free(dm);
        } else {
#pragma omp atomic write
            status = rc;
        }
        free(ustart);
        free(uf);
        free(tmp);
    }
    return status;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
