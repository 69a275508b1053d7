/*
 * smki_oracle.c -- CPU correctness oracle for the S-BKI semantic map update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * GPU library.
 *
 * What it computes is the plain definition from Gan et al., "Bayesian Spatial
 * Kernel Smoothing for Scalable Dense Semantic Mapping" (arXiv 1909.04631):
 *
 *   - Sec. III, Eq. (1)-(2): categorical likelihood with a Dirichlet prior;
 *     the semantic counting sensor model (S-CSM) counts, per grid cell, the
 *     one-hot labels of the measurements that fall in the cell.
 *   - Sec. III, Eq. (3)-(4): mode, mean and variance of the Dirichlet posterior.
 *   - Sec. III (text after Eq. (4)): free-space measurements are points
 *     interpolated linearly along every sensor beam and labelled "free".
 *   - Sec. IV, Eq. (7): the S-BKI posterior concentration at a query point is
 *     the prior plus the kernel-weighted sum of the one-hot labels of all
 *     training points; Eq. (8): the sparse kernel, zero at and beyond l.
 *   - Sec. IV (text after Eq. (8)): query points are the grid centroids and the
 *     concentrations are updated recursively, scan after scan.
 *
 * Everything is double precision, with three exceptions that are *inputs* of
 * the method rather than its arithmetic and therefore follow the binary32
 * contract of the library boundary bit for bit (compile with
 * -ffp-contract=off and without fast-math):
 *   - the free-space sample positions (reading R4 below),
 *   - the voxel / cell index of a point, floor_f32(x / res)  (reading R5/R6),
 *   - all parameters arrive as binary32 values and are promoted exactly.
 *
 * Readings of places where the paper is silent or garbled:
 *   R1  Eq. (8) as printed puts (1 - d/l) on the cosine term only and is then
 *       discontinuous at d = l.  The sparse kernel the paper cites (Melkumyan &
 *       Ramos) is  k = sigma0 [ (2 + cos(2 pi r)) (1 - r) / 3 + sin(2 pi r)/(2 pi) ]
 *       for r = d/l < 1, which is 1 at r = 0, 0 with zero slope at r = 1,
 *       monotone and within [0, sigma0].  That reading is used.
 *   R2  support is strictly d < l.
 *   R3  the training set of a voxel is every training point with d < l (the
 *       paper's face-adjacent "extended block" is a search shortcut that can
 *       drop in-support points; the definition, Eq. (7), has no such cut).
 *   R4  free samples along the beam from origin o to hit p:  v = p - o,
 *       L = sqrt((vx*vx + vy*vy) + vz*vz),  n = ceil(L/s) - 1 (0 if L or s is
 *       not positive), t_j = j*s, w_j = t_j / L, q_j = o + w_j*v (per axis,
 *       multiply then add), j = 1..n; every operation binary32, round to
 *       nearest, no fused multiply-add.  The origin and the hit are not
 *       samples.  n > 2^20 is an input error.
 *   R5/R6  voxel (i,j,k) of a point is floor_f32(x/res) per axis (IEEE
 *       division); voxel centres are ((i+1/2) res, ...) in double from the
 *       binary32 res; blocks are B^3 voxels, block index = floor(i / B).
 *       Voxel indices must lie in [-2^20, 2^20).
 *   R8  the free class is an explicit index (0 in every workload here).
 *   R9  the prior alpha0 is the same for every class.
 *   R10 label -1 drops the hit and its beam.
 *   R11 label = argmax of the mean (lowest index on ties); the mode exists
 *       only when every alpha^k > 1 (NaN otherwise); occupancy probability =
 *       1 - mean of the free class (the sum over the occupied classes).
 *   R12 the recursive update is plain addition.
 *   R23 per-class kernel parameters (Sec. V-D and VI): rows of class k use
 *       their own l_k and sigma0_k, alpha^k = alpha0 + sum_{y_t = k} sigma0_k
 *       f(d / l_k); the loss takes the gradient per class.
 *   R22 soft measurements (Sec. VI): a hit carries a vector of non-negative
 *       class weights instead of one label and adds each class's weight
 *       times the kernel (the linear-pooling form); weights are used as given,
 *       without renormalisation, so a one-hot vector is the hard update.
 *   R14-R16 differentiable form: the loss is the mean negative log predictive
 *       probability  -log(alpha^{y}/S)  of held-out labelled points queried
 *       at their own (continuous) positions; every training row is an input
 *       with its own gradient.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_OOM (-2)
#define OR_E_INPUT (-5)
#define OR_E_RANGE (-6)

#define OR_PI 3.14159265358979323846
#define OR_COORD_LIM (1 << 20)
#define OR_MAX_SAMPLES_PER_RAY (1 << 20)

/* ------------------------------------------------------------------------ */
/* Eq. (8), reading R1                                                        */
/* ------------------------------------------------------------------------ */

/* f(r) with k(d) = sigma0 f(d/l):  (2 + cos 2 pi r)(1 - r)/3 + sin(2 pi r)/(2 pi)
 * for 0 <= r < 1, and 0 for r >= 1.  Near r = 1 the direct double expression
 * can round to a value of order -1e-17; the kernel maps into [0, 1], so the
 * result is clamped at 0. */
double oracle_kernel_f(double r)
{
    if (r < 0.0) r = -r;
    if (r >= 1.0) return 0.0;
    double a = 2.0 * OR_PI * r;
    double f = (2.0 + cos(a)) * (1.0 - r) / 3.0 + sin(a) / (2.0 * OR_PI);
    return f > 0.0 ? f : 0.0;
}

/* df/dr on [0, 1): -(2 pi/3)(1 - r) sin(2 pi r) + (cos(2 pi r) - 1)(2/3);
 * zero for r >= 1 (the kernel and its slope vanish at the support edge). */
double oracle_kernel_df(double r)
{
    if (r < 0.0 || r >= 1.0) return 0.0;
    double a = 2.0 * OR_PI * r;
    double s = sin(OR_PI * r);
    /* cos(2 pi r) - 1 = -2 sin^2(pi r): same value, no cancellation near r = 0 */
    return -(2.0 * OR_PI / 3.0) * (1.0 - r) * sin(a) - (4.0 / 3.0) * s * s;
}

/* (df/dr)/r, with its limit -(4 pi^2)/3 at r = 0 (used for d/dx, where the
 * direction (x - x')/d is multiplied by df/dr). */
double oracle_kernel_df_over_r(double r)
{
    if (r < 0.0 || r >= 1.0) return 0.0;
    if (r < 1e-8) return -4.0 * OR_PI * OR_PI / 3.0;
    return oracle_kernel_df(r) / r;
}

/* k(x, x') = sigma0 f(d/l) if d < l else 0 (Eq. 8). */
double oracle_kernel_k(double d, double l, double sigma0)
{
    if (!(d < l)) return 0.0;
    return sigma0 * oracle_kernel_f(d / l);
}

/* ------------------------------------------------------------------------ */
/* Free-space samples along each beam (Sec. III, reading R4), binary32        */
/* ------------------------------------------------------------------------ */

static int ray_count_f32(const float *p, const float *o, float s, int64_t *n_out)
{
    volatile float vx = p[0] - o[0];
    volatile float vy = p[1] - o[1];
    volatile float vz = p[2] - o[2];
    volatile float xx = vx * vx;
    volatile float yy = vy * vy;
    volatile float zz = vz * vz;
    volatile float a = xx + yy;
    volatile float L2 = a + zz;
    float L = sqrtf(L2);
    if (!(L > 0.0f) || !(s > 0.0f)) { *n_out = 0; return OR_OK; }
    volatile float q = L / s;
    float c = ceilf(q);
    if (!(c - 1.0f <= (float)OR_MAX_SAMPLES_PER_RAY)) return OR_E_INPUT;
    *n_out = (int64_t)c - 1;
    return OR_OK;
}

static int label_ok(int32_t y, int32_t K) { return y == -1 || (y >= 0 && y < K); }
static int finite3(const float *p) { return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]); }

/* Number of free samples of every beam (0 for dropped hits), and the total. */
int oracle_free_counts(const float *xyz, const int32_t *label, int64_t n, const float *origin,
                       float free_step, int32_t K, int64_t *counts /*n, nullable*/,
                       int64_t *total)
{
    if (n < 0 || !total || (n > 0 && (!xyz || !label)) || !origin) return OR_E_ARG;
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!label_ok(label[i], K) || !finite3(xyz + 3 * i)) return OR_E_INPUT;
        int64_t c = 0;
        if (label[i] != -1) {
            int rc = ray_count_f32(xyz + 3 * i, origin, free_step, &c);
            if (rc) return rc;
        }
        if (counts) counts[i] = c;
        tot += c;
    }
    *total = tot;
    return OR_OK;
}

/* The samples themselves, in (hit, j) order; parent[i] = index of the hit. */
int oracle_free_samples(const float *xyz, const int32_t *label, int64_t n, const float *origin,
                        float free_step, int32_t K, float *out_xyz, int64_t *out_parent)
{
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!label_ok(label[i], K) || !finite3(xyz + 3 * i)) return OR_E_INPUT;
        if (label[i] == -1) continue;
        int64_t c = 0;
        int rc = ray_count_f32(xyz + 3 * i, origin, free_step, &c);
        if (rc) return rc;
        if (c == 0) continue;
        const float *p = xyz + 3 * i;
        volatile float vx = p[0] - origin[0];
        volatile float vy = p[1] - origin[1];
        volatile float vz = p[2] - origin[2];
        volatile float xx = vx * vx, yy = vy * vy, zz = vz * vz;
        volatile float a = xx + yy;
        volatile float L2 = a + zz;
        float L = sqrtf(L2);
        for (int64_t j = 1; j <= c; ++j) {
            volatile float t = (float)j * free_step;
            volatile float wj = t / L;
            volatile float mx = wj * vx, my = wj * vy, mz = wj * vz;
            volatile float qx = origin[0] + mx;
            volatile float qy = origin[1] + my;
            volatile float qz = origin[2] + mz;
            out_xyz[3 * w + 0] = qx;
            out_xyz[3 * w + 1] = qy;
            out_xyz[3 * w + 2] = qz;
            if (out_parent) out_parent[w] = i;
            ++w;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Voxel index of a point, floor_f32(x / res) (readings R5/R6)                */
/* ------------------------------------------------------------------------ */

static int voxel_of(const float *p, float res, int32_t *ijk)
{
    for (int a = 0; a < 3; ++a) {
        volatile float q = p[a] / res;
        float f = floorf(q);
        if (!(f >= -(float)OR_COORD_LIM && f < (float)OR_COORD_LIM)) return OR_E_RANGE;
        ijk[a] = (int32_t)f;
    }
    return OR_OK;
}

int oracle_voxel_coords(const float *xyz, int64_t n, float res, int32_t *out_ijk)
{
    if (n < 0 || !(res > 0.0f)) return OR_E_ARG;
    for (int64_t i = 0; i < n; ++i) {
        if (!finite3(xyz + 3 * i)) return OR_E_INPUT;
        int rc = voxel_of(xyz + 3 * i, res, out_ijk + 3 * i);
        if (rc) return rc;
    }
    return OR_OK;
}

/* Packed 64-bit key of a voxel index (21 bits per axis, biased by 2^20). */
static inline uint64_t pack_key(int64_t i, int64_t j, int64_t k)
{
    return ((uint64_t)(i + OR_COORD_LIM) << 42) | ((uint64_t)(j + OR_COORD_LIM) << 21) |
           (uint64_t)(k + OR_COORD_LIM);
}
static inline void unpack_key(uint64_t key, int32_t *ijk)
{
    ijk[0] = (int32_t)((key >> 42) & 0x1FFFFF) - OR_COORD_LIM;
    ijk[1] = (int32_t)((key >> 21) & 0x1FFFFF) - OR_COORD_LIM;
    ijk[2] = (int32_t)(key & 0x1FFFFF) - OR_COORD_LIM;
}

int oracle_pack_keys(const int32_t *ijk, int64_t n, uint64_t *keys)
{
    for (int64_t i = 0; i < n; ++i) keys[i] = pack_key(ijk[3 * i], ijk[3 * i + 1], ijk[3 * i + 2]);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. (7) by definition at arbitrary query points: all training points       */
/* ------------------------------------------------------------------------ */

/* alpha[q][k] = alpha0 + sum over training points t with d(q,t) < l of
 * sigma0 f(d/l) [y_t = k].  n_in[q] counts those t; n_band[q] counts the t
 * with |d^2/l^2 - 1| <= 1e-5 (pairs whose in/out status can flip between a
 * binary32 and a double evaluation; their weight is below 1e-25 sigma0).
 * Every query sums its terms in training-point order. */
/* Gather form of Eq. (7) with row weights w (NULL: every row weighs 1). */
static int alpha_at_impl(const float *train_xyz, const int32_t *train_label, const double *w,
                         int64_t n_train, const double *query_xyz, int64_t n_query, int32_t K,
                         float l, float sigma0, float alpha0, double *alpha, int64_t *n_in,
                         int64_t *n_band)
{
    if (n_train < 0 || n_query < 0 || K < 1 || !(l > 0) || !alpha) return OR_E_ARG;
    for (int64_t t = 0; t < n_train; ++t) {
        if (train_label[t] < 0 || train_label[t] >= K) return OR_E_INPUT;
        if (w && !(isfinite(w[t]) && w[t] >= 0.0)) return OR_E_INPUT;
    }
    const double L = l, S0 = sigma0, A0 = alpha0, L2 = L * L;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_query; ++q) {
        double *a = alpha + q * K;
        for (int k = 0; k < K; ++k) a[k] = A0;
        int64_t cin = 0, cband = 0;
        const double qx = query_xyz[3 * q], qy = query_xyz[3 * q + 1], qz = query_xyz[3 * q + 2];
        for (int64_t t = 0; t < n_train; ++t) {
            double dx = (double)train_xyz[3 * t] - qx;
            double dy = (double)train_xyz[3 * t + 1] - qy;
            double dz = (double)train_xyz[3 * t + 2] - qz;
            double d2 = dx * dx + dy * dy + dz * dz;
            if (fabs(d2 / L2 - 1.0) <= 1e-5) ++cband;
            if (!(d2 < L2)) continue;
            double d = sqrt(d2);
            a[train_label[t]] += (w ? w[t] : 1.0) * (S0 * oracle_kernel_f(d / L));
            ++cin;
        }
        if (n_in) n_in[q] = cin;
        if (n_band) n_band[q] = cband;
    }
    return OR_OK;
}

int oracle_alpha_at(const float *train_xyz, const int32_t *train_label, int64_t n_train,
                    const double *query_xyz, int64_t n_query, int32_t K, float l, float sigma0,
                    float alpha0, double *alpha, int64_t *n_in, int64_t *n_band)
{
    return alpha_at_impl(train_xyz, train_label, NULL, n_train, query_xyz, n_query, K, l, sigma0,
                         alpha0, alpha, n_in, n_band);
}

/* Voxel centres ((i+1/2) res, ...) in double from the binary32 res (R6). */
int oracle_voxel_centres(const int32_t *ijk, int64_t n, float res, double *out)
{
    const double r = res;
    for (int64_t i = 0; i < 3 * n; ++i) out[i] = ((double)ijk[i] + 0.5) * r;
    return OR_OK;
}

/* Eq. (7) at the centroids of the given voxels (Sec. IV: queries are the grid
 * centroids). */
int oracle_alpha_at_voxels(const float *train_xyz, const int32_t *train_label, int64_t n_train,
                           const int32_t *ijk, int64_t n_query, float res, int32_t K, float l,
                           float sigma0, float alpha0, double *alpha, int64_t *n_in,
                           int64_t *n_band)
{
    double *c = (double *)malloc(sizeof(double) * 3 * (size_t)(n_query > 0 ? n_query : 1));
    if (!c) return OR_E_OOM;
    oracle_voxel_centres(ijk, n_query, res, c);
    int rc = oracle_alpha_at(train_xyz, train_label, n_train, c, n_query, K, l, sigma0, alpha0,
                             alpha, n_in, n_band);
    free(c);
    return rc;
}

/* The same with row weights (soft measurements, reading R22). */
int oracle_alpha_at_voxels_w(const float *train_xyz, const int32_t *train_label,
                             const double *train_w, int64_t n_train, const int32_t *ijk,
                             int64_t n_query, float res, int32_t K, float l, float sigma0,
                             float alpha0, double *alpha, int64_t *n_in, int64_t *n_band)
{
    double *c = (double *)malloc(sizeof(double) * 3 * (size_t)(n_query > 0 ? n_query : 1));
    if (!c) return OR_E_OOM;
    oracle_voxel_centres(ijk, n_query, res, c);
    int rc = alpha_at_impl(train_xyz, train_label, train_w, n_train, c, n_query, K, l, sigma0,
                           alpha0, alpha, n_in, n_band);
    free(c);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Training set of one scan: labelled hits, then their free samples (R4,R10)  */
/* ------------------------------------------------------------------------ */

/* Two calls: with out_xyz == NULL only *n_out is set.  Order: the kept hits in
 * input order, then the free samples in (hit, j) order.  out_parent (nullable)
 * gets the index of the source hit of every row. */
int oracle_training_set(const float *xyz, const int32_t *label, int64_t n, const float *origin,
                        float free_step, int32_t K, int32_t free_class, int64_t *n_out,
                        float *out_xyz, int32_t *out_label, int64_t *out_parent)
{
    if (n < 0 || !n_out || K < 1 || free_class < 0 || free_class >= K) return OR_E_ARG;
    int64_t nf = 0;
    int rc = oracle_free_counts(xyz, label, n, origin, free_step, K, NULL, &nf);
    if (rc) return rc;
    int64_t nh = 0;
    for (int64_t i = 0; i < n; ++i) nh += label[i] != -1;
    *n_out = nh + nf;
    if (!out_xyz) return OR_OK;
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] == -1) continue;
        memcpy(out_xyz + 3 * w, xyz + 3 * i, 3 * sizeof(float));
        out_label[w] = label[i];
        if (out_parent) out_parent[w] = i;
        ++w;
    }
    rc = oracle_free_samples(xyz, label, n, origin, free_step, K, out_xyz + 3 * w,
                             out_parent ? out_parent + w : NULL);
    if (rc) return rc;
    for (int64_t j = 0; j < nf; ++j) out_label[w + j] = free_class;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* The map: Eq. (7) at every grid centroid, accumulated scan after scan        */
/* ------------------------------------------------------------------------ */
/* Stored are only voxels that received at least one in-support term; every
 * other voxel holds the prior alpha0 by definition.  The sum is enumerated
 * from the training-point side: for a point x, every voxel whose centre can
 * lie within l of x has its index in [floor((x - l)/res - 1/2), ceil((x + l)/res
 * - 1/2)] per axis (a box around the ball, widened by one voxel); each
 * candidate's exact double distance decides.  The result is the same sum as
 * Eq. (7) per voxel, in training-point order. */

typedef struct {
    uint64_t key;    /* packed voxel index; UINT64_MAX = empty */
    int64_t idx;     /* row into the value arrays */
} or_slot;

typedef struct oracle_map {
    int32_t K, B;
    double res, l, sigma0, alpha0;
    float res32, l32, sigma032, alpha032;
    or_slot *tab;
    int64_t cap;     /* table slots (power of two) */
    int64_t n;       /* stored voxels */
    int64_t rows;    /* row capacity */
    uint64_t *keys;
    double *alpha;   /* rows * K */
    int64_t *nv, *nband;
    int scsm;        /* 1: S-CSM map (Eq. 2), 0: S-BKI map (Eq. 7) */
    int face_blocks; /* 1: a voxel's training rows are those in its block and the six
                        face-adjacent blocks (the extended block of Sec. IV's
                        implementation notes), 0: every row (exact Eq. 7) */
    double *lk, *s0k; /* [K] length-scale and scale of each class's kernel (reading R23);
                         all equal to l and sigma0 unless set per class */
    int64_t *stamp;   /* per stored voxel: the last S-CSM insert that touched it */
    int64_t stamp_now;
    int64_t last[4];  /* counters of the last insert (oracle_map_last_insert) */
} oracle_map;

/* floor(a / b) for b > 0 */
static int64_t fdiv_floor(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

void oracle_map_destroy(oracle_map *m);

oracle_map *oracle_map_create(int32_t K, float res, int32_t block_size, float l, float sigma0,
                              float alpha0, int32_t scsm, int32_t face_blocks)
{
    if (K < 1 || !(res > 0) || !(l > 0) || block_size < 1) return NULL;
    oracle_map *m = (oracle_map *)calloc(1, sizeof(oracle_map));
    if (!m) return NULL;
    m->K = K; m->B = block_size;
    m->res32 = res; m->l32 = l; m->sigma032 = sigma0; m->alpha032 = alpha0;
    m->res = res; m->l = l; m->sigma0 = sigma0; m->alpha0 = alpha0;
    m->scsm = scsm;
    m->face_blocks = face_blocks;
    m->cap = 1 << 16;
    m->tab = (or_slot *)malloc(sizeof(or_slot) * m->cap);
    for (int64_t i = 0; i < m->cap; ++i) m->tab[i].key = UINT64_MAX;
    m->rows = 1 << 15;
    m->keys = (uint64_t *)malloc(sizeof(uint64_t) * m->rows);
    m->alpha = (double *)malloc(sizeof(double) * m->rows * K);
    m->nv = (int64_t *)malloc(sizeof(int64_t) * m->rows);
    m->nband = (int64_t *)malloc(sizeof(int64_t) * m->rows);
    m->stamp = (int64_t *)malloc(sizeof(int64_t) * m->rows);
    m->lk = (double *)malloc(sizeof(double) * K);
    m->s0k = (double *)malloc(sizeof(double) * K);
    if (!m->tab || !m->keys || !m->alpha || !m->nv || !m->nband || !m->stamp || !m->lk || !m->s0k) {
        oracle_map_destroy(m);
        return NULL;
    }
    for (int32_t k = 0; k < K; ++k) { m->lk[k] = m->l; m->s0k[k] = m->sigma0; }
    return m;
}

/* Per-class kernel parameters (reading R23): rows of class k use length-scale
 * l[k] and scale sigma0[k] (binary32 inputs, promoted exactly), each finite and
 * positive.  Applies to later inserts. */
int oracle_map_set_class_params(oracle_map *m, const float *l, const float *sigma0)
{
    if (!m || !l || !sigma0) return OR_E_ARG;
    for (int32_t k = 0; k < m->K; ++k)
        if (!(isfinite(l[k]) && l[k] > 0.0f && isfinite(sigma0[k]) && sigma0[k] > 0.0f))
            return OR_E_ARG;
    for (int32_t k = 0; k < m->K; ++k) { m->lk[k] = l[k]; m->s0k[k] = sigma0[k]; }
    return OR_OK;
}

void oracle_map_destroy(oracle_map *m)
{
    if (!m) return;
    free(m->tab); free(m->keys); free(m->alpha); free(m->nv); free(m->nband);
    free(m->stamp); free(m->lk); free(m->s0k);
    free(m);
}

static int map_grow_table(oracle_map *m)
{
    int64_t nc = m->cap * 2;
    or_slot *t = (or_slot *)malloc(sizeof(or_slot) * nc);
    if (!t) return OR_E_OOM;
    for (int64_t i = 0; i < nc; ++i) t[i].key = UINT64_MAX;
    for (int64_t i = 0; i < m->cap; ++i) {
        if (m->tab[i].key == UINT64_MAX) continue;
        uint64_t h = mix64(m->tab[i].key) & (uint64_t)(nc - 1);
        while (t[h].key != UINT64_MAX) h = (h + 1) & (uint64_t)(nc - 1);
        t[h] = m->tab[i];
    }
    free(m->tab);
    m->tab = t;
    m->cap = nc;
    return OR_OK;
}

/* Row of a voxel, created (alpha = alpha0) if absent; -1 on allocation failure. */
static int64_t map_row(oracle_map *m, uint64_t key)
{
    if (2 * (m->n + 1) > m->cap && map_grow_table(m)) return -1;
    uint64_t h = mix64(key) & (uint64_t)(m->cap - 1);
    while (m->tab[h].key != UINT64_MAX) {
        if (m->tab[h].key == key) return m->tab[h].idx;
        h = (h + 1) & (uint64_t)(m->cap - 1);
    }
    if (m->n == m->rows) {
        int64_t nr = m->rows * 2;
        uint64_t *k2 = (uint64_t *)realloc(m->keys, sizeof(uint64_t) * nr);
        if (!k2) return -1;
        m->keys = k2;
        double *a2 = (double *)realloc(m->alpha, sizeof(double) * nr * m->K);
        if (!a2) return -1;
        m->alpha = a2;
        int64_t *n2 = (int64_t *)realloc(m->nv, sizeof(int64_t) * nr);
        if (!n2) return -1;
        m->nv = n2;
        int64_t *b2 = (int64_t *)realloc(m->nband, sizeof(int64_t) * nr);
        if (!b2) return -1;
        m->nband = b2;
        int64_t *s2 = (int64_t *)realloc(m->stamp, sizeof(int64_t) * nr);
        if (!s2) return -1;
        m->stamp = s2;
        m->rows = nr;
    }
    int64_t r = m->n++;
    m->tab[h].key = key;
    m->tab[h].idx = r;
    m->keys[r] = key;
    for (int k = 0; k < m->K; ++k) m->alpha[r * m->K + k] = m->alpha0;
    m->nv[r] = 0;
    m->nband[r] = 0;
    m->stamp[r] = 0;
    return r;
}

/* Add one training set (rows already expanded: hits + free samples). */
/* Rows t = 0..n-1 with class label[t] and measurement weight w[t] (1 for every
 * row when w is NULL): alpha^y += w sigma0 f(d / l) at every voxel centre
 * within l (Eq. (7)), or alpha^y += w in the row's own cell (Eq. (2)).  A
 * one-hot row has w = 1; a soft row contributes its class probability
 * (reading R22).
 *
 * Every row is validated before anything is written, so a failed insert leaves
 * the map unchanged.  The S-BKI sum is split over square tiles of voxel columns
 * (x, y) so that several threads can work at once; each tile adds, for each of
 * its voxels, the terms of the rows in row order starting from the voxel's
 * value before the insert, which is exactly the serial order: the result does
 * not depend on the number of threads. */

/* Box of voxel indices around the ball of radius L at x (widened by one voxel). */
static void row_box(const double x[3], double L, double res, int64_t lo[3], int64_t hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = (int64_t)floor((x[a] - L) / res - 0.5) - 1;
        hi[a] = (int64_t)ceil((x[a] + L) / res - 0.5) + 1;
    }
}

/* The voxels one tile touches during one insert: packed key -> entry, each
 * entry the running concentrations, the map's counts plus this insert's, and
 * this insert's in-support and band counts. */
typedef struct {
    uint64_t *hk;      /* hash slots: key, UINT64_MAX empty */
    int64_t *hv;       /* hash slots: entry */
    int64_t hcap, n, cap;
    uint64_t *key;     /* [cap] */
    double *alpha;     /* [cap * K] */
    int64_t *nv, *nb;  /* cumulative counts */
    int64_t *snv, *snb;/* this insert's counts */
} or_tile;

static void tile_free(or_tile *t)
{
    free(t->hk); free(t->hv); free(t->key); free(t->alpha);
    free(t->nv); free(t->nb); free(t->snv); free(t->snb);
    memset(t, 0, sizeof(*t));
}

static int tile_grow_entries(or_tile *t, int32_t K)
{
    int64_t nc = t->cap ? 2 * t->cap : 256;
    uint64_t *k2 = (uint64_t *)realloc(t->key, sizeof(uint64_t) * nc);
    if (!k2) return OR_E_OOM;
    t->key = k2;
    double *a2 = (double *)realloc(t->alpha, sizeof(double) * nc * K);
    if (!a2) return OR_E_OOM;
    t->alpha = a2;
    int64_t **arr[4] = {&t->nv, &t->nb, &t->snv, &t->snb};
    for (int i = 0; i < 4; ++i) {
        int64_t *q = (int64_t *)realloc(*arr[i], sizeof(int64_t) * nc);
        if (!q) return OR_E_OOM;
        *arr[i] = q;
    }
    t->cap = nc;
    return OR_OK;
}

static int tile_grow_hash(or_tile *t)
{
    int64_t nc = t->hcap ? 2 * t->hcap : 512;
    uint64_t *hk = (uint64_t *)malloc(sizeof(uint64_t) * nc);
    int64_t *hv = (int64_t *)malloc(sizeof(int64_t) * nc);
    if (!hk || !hv) { free(hk); free(hv); return OR_E_OOM; }
    for (int64_t i = 0; i < nc; ++i) hk[i] = UINT64_MAX;
    for (int64_t e = 0; e < t->n; ++e) {
        uint64_t h = mix64(t->key[e]) & (uint64_t)(nc - 1);
        while (hk[h] != UINT64_MAX) h = (h + 1) & (uint64_t)(nc - 1);
        hk[h] = t->key[e];
        hv[h] = e;
    }
    free(t->hk); free(t->hv);
    t->hk = hk; t->hv = hv; t->hcap = nc;
    return OR_OK;
}

/* Row of the stored map for a key, or -1 (read only). */
static int64_t map_find(const oracle_map *m, uint64_t key)
{
    uint64_t h = mix64(key) & (uint64_t)(m->cap - 1);
    while (m->tab[h].key != UINT64_MAX) {
        if (m->tab[h].key == key) return m->tab[h].idx;
        h = (h + 1) & (uint64_t)(m->cap - 1);
    }
    return -1;
}

/* Entry of a voxel in a tile, created from the map's current value (alpha0 and
 * zero counts for a voxel the map does not store); -1 on allocation failure. */
static int64_t tile_entry(or_tile *t, const oracle_map *m, uint64_t key)
{
    if (2 * (t->n + 1) > t->hcap && tile_grow_hash(t)) return -1;
    uint64_t h = mix64(key) & (uint64_t)(t->hcap - 1);
    while (t->hk[h] != UINT64_MAX) {
        if (t->hk[h] == key) return t->hv[h];
        h = (h + 1) & (uint64_t)(t->hcap - 1);
    }
    if (t->n == t->cap && tile_grow_entries(t, m->K)) return -1;
    const int64_t e = t->n++;
    t->hk[h] = key;
    t->hv[h] = e;
    t->key[e] = key;
    const int64_t r = map_find(m, key);
    for (int k = 0; k < m->K; ++k) t->alpha[e * m->K + k] = r < 0 ? m->alpha0 : m->alpha[r * m->K + k];
    t->nv[e] = r < 0 ? 0 : m->nv[r];
    t->nb[e] = r < 0 ? 0 : m->nband[r];
    t->snv[e] = 0;
    t->snb[e] = 0;
    return e;
}

/* The terms of rows rows[0..nr) (ascending) for the voxels of columns
 * i in [i0, i1], j in [j0, j1]. */
static int tile_accumulate(or_tile *t, const oracle_map *m, const float *xyz,
                           const int32_t *label, const double *w, const int64_t *rows,
                           int64_t nr, int64_t i0, int64_t i1, int64_t j0, int64_t j1)
{
    const double res = m->res;
    for (int64_t q = 0; q < nr; ++q) {
        const int64_t t_ = rows[q];
        const float *p = xyz + 3 * t_;
        const double wt = w ? w[t_] : 1.0;
        const double L = m->lk[label[t_]], L2 = L * L, S0 = m->s0k[label[t_]];
        const double x[3] = {p[0], p[1], p[2]};
        int32_t pv[3] = {0, 0, 0};
        if (m->face_blocks && voxel_of(p, m->res32, pv)) return OR_E_RANGE;
        int64_t lo[3], hi[3];
        row_box(x, L, res, lo, hi);
        if (lo[0] < i0) lo[0] = i0;
        if (hi[0] > i1) hi[0] = i1;
        if (lo[1] < j0) lo[1] = j0;
        if (hi[1] > j1) hi[1] = j1;
        for (int64_t i = lo[0]; i <= hi[0]; ++i) {
            double dx = x[0] - ((double)i + 0.5) * res;
            for (int64_t j = lo[1]; j <= hi[1]; ++j) {
                double dy = x[1] - ((double)j + 0.5) * res;
                for (int64_t k = lo[2]; k <= hi[2]; ++k) {
                    double dz = x[2] - ((double)k + 0.5) * res;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (m->face_blocks) {
                        /* the row must lie in the voxel's block or one sharing a face */
                        const int64_t B = m->B;
                        const int64_t db = llabs(fdiv_floor(pv[0], B) - fdiv_floor(i, B)) +
                                           llabs(fdiv_floor(pv[1], B) - fdiv_floor(j, B)) +
                                           llabs(fdiv_floor(pv[2], B) - fdiv_floor(k, B));
                        if (db > 1) continue;
                    }
                    int band = fabs(d2 / L2 - 1.0) <= 1e-5;
                    if (!(d2 < L2) && !band) continue;
                    int64_t e = tile_entry(t, m, pack_key(i, j, k));
                    if (e < 0) return OR_E_OOM;
                    if (band) { t->nb[e] += 1; t->snb[e] += 1; }
                    if (!(d2 < L2)) continue;
                    t->alpha[e * m->K + label[t_]] += wt * (S0 * oracle_kernel_f(sqrt(d2) / L));
                    t->nv[e] += 1;
                    t->snv[e] += 1;
                }
            }
        }
    }
    return OR_OK;
}

static int insert_rows(oracle_map *m, const float *xyz, const int32_t *label, const double *w,
                       int64_t n)
{
    if (!m || n < 0) return OR_E_ARG;
    const double res = m->res;
    memset(m->last, 0, sizeof(m->last));
    for (int64_t t = 0; t < n; ++t) {
        if (label[t] < 0 || label[t] >= m->K) return OR_E_INPUT;
        if (!finite3(xyz + 3 * t)) return OR_E_INPUT;
        if (w && !(isfinite(w[t]) && w[t] >= 0.0)) return OR_E_INPUT;
        int32_t v[3];
        int rc = voxel_of(xyz + 3 * t, m->res32, v);
        if (rc) return rc;
        if (!m->scsm) {
            const double x[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
            int64_t lo[3], hi[3];
            row_box(x, m->lk[label[t]], res, lo, hi);
            for (int a = 0; a < 3; ++a)
                if (lo[a] < -OR_COORD_LIM || hi[a] >= OR_COORD_LIM) return OR_E_RANGE;
        }
    }
    if (n == 0) return OR_OK;
    if (m->scsm) {
        /* Eq. (2): each measurement counts in the cell it falls into. */
        ++m->stamp_now;
        for (int64_t t = 0; t < n; ++t) {
            int32_t v[3];
            (void)voxel_of(xyz + 3 * t, m->res32, v);
            int64_t r = map_row(m, pack_key(v[0], v[1], v[2]));
            if (r < 0) return OR_E_OOM;
            m->alpha[r * m->K + label[t]] += w ? w[t] : 1.0;
            m->nv[r] += 1;
            if (m->stamp[r] != m->stamp_now) { m->stamp[r] = m->stamp_now; m->last[0] += 1; }
            m->last[1] += 1;
        }
        return OR_OK;
    }
    /* tiles of W x W voxel columns covering the rows' boxes */
    int64_t ti0 = INT64_MAX, ti1 = INT64_MIN, tj0 = INT64_MAX, tj1 = INT64_MIN;
    int64_t W = 16;
    int64_t vlo[2] = {INT64_MAX, INT64_MAX}, vhi[2] = {INT64_MIN, INT64_MIN};
    for (int64_t t = 0; t < n; ++t) {
        const double x[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
        int64_t lo[3], hi[3];
        row_box(x, m->lk[label[t]], res, lo, hi);
        for (int a = 0; a < 2; ++a) {
            if (lo[a] < vlo[a]) vlo[a] = lo[a];
            if (hi[a] > vhi[a]) vhi[a] = hi[a];
        }
    }
    for (;;) {
        ti0 = fdiv_floor(vlo[0], W); ti1 = fdiv_floor(vhi[0], W);
        tj0 = fdiv_floor(vlo[1], W); tj1 = fdiv_floor(vhi[1], W);
        if ((ti1 - ti0 + 1) * (tj1 - tj0 + 1) <= (1 << 20)) break;
        W *= 2;
    }
    const int64_t nti = ti1 - ti0 + 1, ntj = tj1 - tj0 + 1, ntiles = nti * ntj;
    int64_t *start = (int64_t *)calloc((size_t)ntiles + 1, sizeof(int64_t));
    if (!start) return OR_E_OOM;
    for (int64_t t = 0; t < n; ++t) {
        const double x[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
        int64_t lo[3], hi[3];
        row_box(x, m->lk[label[t]], res, lo, hi);
        for (int64_t a = fdiv_floor(lo[0], W); a <= fdiv_floor(hi[0], W); ++a)
            for (int64_t b = fdiv_floor(lo[1], W); b <= fdiv_floor(hi[1], W); ++b)
                start[(a - ti0) * ntj + (b - tj0) + 1] += 1;
    }
    for (int64_t i = 0; i < ntiles; ++i) start[i + 1] += start[i];
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(start[ntiles] > 0 ? start[ntiles] : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)ntiles);
    or_tile *tiles = (or_tile *)calloc((size_t)ntiles, sizeof(or_tile));
    int64_t *busy = (int64_t *)malloc(sizeof(int64_t) * (size_t)ntiles);
    if (!rows || !cur || !tiles || !busy) {
        free(start); free(rows); free(cur); free(tiles); free(busy);
        return OR_E_OOM;
    }
    memcpy(cur, start, sizeof(int64_t) * (size_t)ntiles);
    for (int64_t t = 0; t < n; ++t) {   /* each tile's rows in row order */
        const double x[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
        int64_t lo[3], hi[3];
        row_box(x, m->lk[label[t]], res, lo, hi);
        for (int64_t a = fdiv_floor(lo[0], W); a <= fdiv_floor(hi[0], W); ++a)
            for (int64_t b = fdiv_floor(lo[1], W); b <= fdiv_floor(hi[1], W); ++b)
                rows[cur[(a - ti0) * ntj + (b - tj0)]++] = t;
    }
    int64_t nbusy = 0;
    for (int64_t i = 0; i < ntiles; ++i)
        if (start[i + 1] > start[i]) busy[nbusy++] = i;
    int err = OR_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nbusy; ++q) {
        const int64_t i = busy[q];
        const int64_t a = i / ntj + ti0, b = i % ntj + tj0;
        int rc = tile_accumulate(&tiles[i], m, xyz, label, w, rows + start[i],
                                 start[i + 1] - start[i], a * W, a * W + W - 1, b * W,
                                 b * W + W - 1);
        if (rc) {
            #pragma omp critical
            err = rc;
        }
    }
    /* write back tile by tile (tiles own disjoint voxels) */
    for (int64_t q = 0; q < nbusy && !err; ++q) {
        or_tile *t = &tiles[busy[q]];
        for (int64_t e = 0; e < t->n; ++e) {
            int64_t r = map_row(m, t->key[e]);
            if (r < 0) { err = OR_E_OOM; break; }
            memcpy(m->alpha + r * m->K, t->alpha + e * m->K, sizeof(double) * m->K);
            m->nv[r] = t->nv[e];
            m->nband[r] = t->nb[e];
            m->last[0] += t->snv[e] > 0;
            m->last[1] += t->snv[e];
            m->last[2] += t->snb[e] > 0;
            m->last[3] += t->snb[e];
        }
    }
    for (int64_t q = 0; q < nbusy; ++q) tile_free(&tiles[busy[q]]);
    free(start); free(rows); free(cur); free(tiles); free(busy);
    return err;
}

/* Counters of the last insert: [0] voxels with at least one in-support row
 * (S-CSM: voxels holding at least one row), [1] in-support (voxel, row) pairs
 * (S-CSM: rows), [2] voxels with a pair in the rounding band |d^2/l^2 - 1| <=
 * 1e-5, [3] such pairs. */
int oracle_map_last_insert(const oracle_map *m, int64_t *out)
{
    if (!m || !out) return OR_E_ARG;
    memcpy(out, m->last, sizeof(m->last));
    return OR_OK;
}

/* One scan: its training set (hits + free samples) into the map. */
int oracle_map_insert_training(oracle_map *m, const float *xyz, const int32_t *label, int64_t n)
{
    return insert_rows(m, xyz, label, NULL, n);
}

/* Training rows of one scan of soft measurements (reading R22): probs[i][k]
 * >= 0 is the weight of class k in hit i.  Every class with a positive weight
 * gives the hit one row of that class and weight (hits in input order, classes
 * ascending); a hit whose weights are all zero is dropped with its beam (as
 * label -1); then the free samples of the kept beams, free-class rows of
 * weight 1.  Negative or non-finite weights are input errors.  Two calls: with
 * out_xyz == NULL only *n_out is set. */
int oracle_training_set_soft(const float *xyz, const float *probs, int64_t n, const float *origin,
                             float free_step, int32_t K, int32_t free_class, int64_t *n_out,
                             float *out_xyz, int32_t *out_label, double *out_w)
{
    if (n < 0 || !n_out || K < 1 || free_class < 0 || free_class >= K) return OR_E_ARG;
    if (n > 0 && (!xyz || !probs)) return OR_E_ARG;
    int32_t *keep = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!keep) return OR_E_OOM;
    int64_t nrows = 0;
    for (int64_t i = 0; i < n; ++i) {
        int any = 0;
        for (int32_t k = 0; k < K; ++k) {
            const float p = probs[i * K + k];
            if (!(isfinite(p) && p >= 0.0f)) { free(keep); return OR_E_INPUT; }
            if (p > 0.0f) { any = 1; ++nrows; }
        }
        keep[i] = any ? 0 : -1;   /* any class index marks a kept beam */
    }
    int64_t nf = 0;
    int rc = oracle_free_counts(xyz, keep, n, origin, free_step, K, NULL, &nf);
    if (rc || !out_xyz) {
        *n_out = nrows + nf;
        free(keep);
        return rc;
    }
    int64_t r = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < K; ++k) {
            const float p = probs[i * K + k];
            if (!(p > 0.0f)) continue;
            memcpy(out_xyz + 3 * r, xyz + 3 * i, 3 * sizeof(float));
            out_label[r] = k;
            out_w[r] = (double)p;
            ++r;
        }
    rc = oracle_free_samples(xyz, keep, n, origin, free_step, K, out_xyz + 3 * r, NULL);
    for (int64_t j = 0; j < nf; ++j) { out_label[r + j] = free_class; out_w[r + j] = 1.0; }
    *n_out = nrows + nf;
    free(keep);
    return rc;
}

/* One scan of soft measurements: the rows above, inserted with their weights. */
int oracle_map_insert_scan_soft(oracle_map *m, const float *xyz, const float *probs, int64_t n,
                                const float *origin, float free_step, int32_t free_class)
{
    if (!m || n < 0 || (n > 0 && (!xyz || !probs)) || !origin) return OR_E_ARG;
    if (free_class < 0 || free_class >= m->K) return OR_E_ARG;
    int64_t nt = 0;
    int rc = oracle_training_set_soft(xyz, probs, n, origin, free_step, m->K, free_class, &nt,
                                      NULL, NULL, NULL);
    if (rc) return rc;
    float *tx = (float *)malloc(sizeof(float) * 3 * (size_t)(nt > 0 ? nt : 1));
    int32_t *ty = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
    double *tw = (double *)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    if (!tx || !ty || !tw) { free(tx); free(ty); free(tw); return OR_E_OOM; }
    rc = oracle_training_set_soft(xyz, probs, n, origin, free_step, m->K, free_class, &nt, tx, ty,
                                  tw);
    if (!rc) rc = insert_rows(m, tx, ty, tw, nt);
    free(tx); free(ty); free(tw);
    return rc;
}

int oracle_map_insert_scan(oracle_map *m, const float *xyz, const int32_t *label, int64_t n,
                           const float *origin, float free_step, int32_t free_class)
{
    int64_t nt = 0;
    int rc = oracle_training_set(xyz, label, n, origin, free_step, m->K, free_class, &nt, NULL,
                                 NULL, NULL);
    if (rc) return rc;
    float *tx = (float *)malloc(sizeof(float) * 3 * (size_t)(nt > 0 ? nt : 1));
    int32_t *ty = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
    if (!tx || !ty) { free(tx); free(ty); return OR_E_OOM; }
    rc = oracle_training_set(xyz, label, n, origin, free_step, m->K, free_class, &nt, tx, ty, NULL);
    if (!rc) rc = oracle_map_insert_training(m, tx, ty, nt);
    free(tx);
    free(ty);
    return rc;
}

int64_t oracle_map_size(const oracle_map *m) { return m ? m->n : -1; }

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* Stored voxels sorted by packed key (x-major, z fastest). */
int oracle_map_export(const oracle_map *m, int32_t *ijk, double *alpha, int64_t *nv,
                      int64_t *nband)
{
    if (!m) return OR_E_ARG;
    uint64_t *ks = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m->n > 0 ? m->n : 1));
    if (!ks) return OR_E_OOM;
    memcpy(ks, m->keys, sizeof(uint64_t) * m->n);
    qsort(ks, (size_t)m->n, sizeof(uint64_t), cmp_u64);
    for (int64_t i = 0; i < m->n; ++i) {
        uint64_t key = ks[i];
        uint64_t h = mix64(key) & (uint64_t)(m->cap - 1);
        while (m->tab[h].key != key) h = (h + 1) & (uint64_t)(m->cap - 1);
        int64_t r = m->tab[h].idx;
        if (ijk) unpack_key(key, ijk + 3 * i);
        if (alpha) memcpy(alpha + i * m->K, m->alpha + r * m->K, sizeof(double) * m->K);
        if (nv) nv[i] = m->nv[r];
        if (nband) nband[i] = m->nband[r];
    }
    free(ks);
    return OR_OK;
}

/* alpha of arbitrary voxels (alpha0 where the map stores nothing). */
int oracle_map_lookup(const oracle_map *m, const int32_t *ijk, int64_t n, double *alpha)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t key = pack_key(ijk[3 * i], ijk[3 * i + 1], ijk[3 * i + 2]);
        uint64_t h = mix64(key) & (uint64_t)(m->cap - 1);
        int64_t r = -1;
        while (m->tab[h].key != UINT64_MAX) {
            if (m->tab[h].key == key) { r = m->tab[h].idx; break; }
            h = (h + 1) & (uint64_t)(m->cap - 1);
        }
        for (int k = 0; k < m->K; ++k)
            alpha[i * m->K + k] = r < 0 ? m->alpha0 : m->alpha[r * m->K + k];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Readout, Eq. (3)-(4) and reading R11                                       */
/* ------------------------------------------------------------------------ */
int oracle_readout(const double *alpha, int64_t n, int32_t K, int32_t free_class, double *mean,
                   double *var, double *mode, int32_t *label, double *p_occ)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *a = alpha + i * K;
        double S = 0.0;
        int all_gt1 = 1;
        for (int k = 0; k < K; ++k) { S += a[k]; all_gt1 &= a[k] > 1.0; }
        int best = 0;
        for (int k = 0; k < K; ++k) {
            double e = a[k] / S;
            if (mean) mean[i * K + k] = e;
            if (var) var[i * K + k] = e * (1.0 - e) / (S + 1.0);
            if (mode) mode[i * K + k] = all_gt1 ? (a[k] - 1.0) / (S - K) : NAN;
            if (a[k] > a[best]) best = k;
        }
        if (label) label[i] = best;
        if (p_occ) p_occ[i] = 1.0 - a[free_class] / S;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Differentiable form (readings R14-R16): predictive loss and its gradient   */
/* ------------------------------------------------------------------------ */
/* alpha_h = Eq. (7) at held-out point x_h from all training rows;
 * loss = -(1/H) sum_h log(alpha_h^{y_h} / S_h).
 * With G_hk = dloss/dalpha_hk = -(1/H)(delta_{k,y_h}/alpha_hk - 1/S_h), and
 * for each in-support pair (h, t), r = d/l:
 *   dloss/dsigma0 += G_{h,y_t} f(r)
 *   dloss/dl      += G_{h,y_t} sigma0 f'(r) (-r/l)
 *   dloss/dx_t    += G_{h,y_t} sigma0 (f'(r)/r) (x_t - x_h) / l^2
 *   dloss/dx_h    -= the same vector.
 * Coordinates are double here so that finite differences can perturb them. */
int oracle_loss(const double *train_xyz, const int32_t *train_label, int64_t n_train,
                const double *query_xyz, const int32_t *query_label, int64_t n_query, int32_t K,
                double l, double sigma0, double alpha0, double *loss, double *alpha_q,
                double *grad_l, double *grad_sigma0, double *grad_train, double *grad_query)
{
    if (n_train < 0 || n_query <= 0 || K < 1 || !(l > 0)) return OR_E_ARG;
    for (int64_t t = 0; t < n_train; ++t)
        if (train_label[t] < 0 || train_label[t] >= K) return OR_E_INPUT;
    for (int64_t h = 0; h < n_query; ++h)
        if (query_label[h] < 0 || query_label[h] >= K) return OR_E_INPUT;
    double *A = alpha_q ? alpha_q : (double *)malloc(sizeof(double) * n_query * K);
    double *G = (double *)malloc(sizeof(double) * n_query * K);
    if (!A || !G) return OR_E_OOM;
    const double L2 = l * l, H = (double)n_query;
    double tot = 0.0;
    for (int64_t h = 0; h < n_query; ++h) {
        double *a = A + h * K;
        for (int k = 0; k < K; ++k) a[k] = alpha0;
        for (int64_t t = 0; t < n_train; ++t) {
            double dx = train_xyz[3 * t] - query_xyz[3 * h];
            double dy = train_xyz[3 * t + 1] - query_xyz[3 * h + 1];
            double dz = train_xyz[3 * t + 2] - query_xyz[3 * h + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 < L2)) continue;
            a[train_label[t]] += sigma0 * oracle_kernel_f(sqrt(d2) / l);
        }
        double S = 0.0;
        for (int k = 0; k < K; ++k) S += a[k];
        tot += -log(a[query_label[h]] / S);
        for (int k = 0; k < K; ++k)
            G[h * K + k] = -((k == query_label[h] ? 1.0 / a[k] : 0.0) - 1.0 / S) / H;
    }
    if (loss) *loss = tot / H;
    double gl = 0.0, gs = 0.0;
    if (grad_train) memset(grad_train, 0, sizeof(double) * 3 * n_train);
    if (grad_query) memset(grad_query, 0, sizeof(double) * 3 * n_query);
    for (int64_t h = 0; h < n_query; ++h) {
        for (int64_t t = 0; t < n_train; ++t) {
            double dx = train_xyz[3 * t] - query_xyz[3 * h];
            double dy = train_xyz[3 * t + 1] - query_xyz[3 * h + 1];
            double dz = train_xyz[3 * t + 2] - query_xyz[3 * h + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 < L2)) continue;
            double r = sqrt(d2) / l;
            double g = G[h * K + train_label[t]];
            gs += g * oracle_kernel_f(r);
            gl += g * sigma0 * oracle_kernel_df(r) * (-r / l);
            double c = g * sigma0 * oracle_kernel_df_over_r(r) / L2;
            if (grad_train) {
                grad_train[3 * t] += c * dx;
                grad_train[3 * t + 1] += c * dy;
                grad_train[3 * t + 2] += c * dz;
            }
            if (grad_query) {
                grad_query[3 * h] -= c * dx;
                grad_query[3 * h + 1] -= c * dy;
                grad_query[3 * h + 2] -= c * dz;
            }
        }
    }
    if (grad_l) *grad_l = gl;
    if (grad_sigma0) *grad_sigma0 = gs;
    if (!alpha_q) free(A);
    free(G);
    return OR_OK;
}

/* The predictive loss with per-class kernel parameters (reading R23):
 * alpha_q[h][k] = alpha0 + sum_{t: y_t = k} sigma0[k] f(|x_t - x_h| / l[k]),
 * loss = -(1/H) sum_h log(alpha_q[h][y_h] / S_h), and its gradient with respect
 * to every l[k], sigma0[k] and coordinate, all pairs, double throughout. */
int oracle_loss_classes(const double *train_xyz, const int32_t *train_label, int64_t n_train,
                        const double *query_xyz, const int32_t *query_label, int64_t n_query,
                        int32_t K, const double *l, const double *sigma0, double alpha0,
                        double *loss, double *alpha_q, double *grad_l, double *grad_sigma0,
                        double *grad_train, double *grad_query)
{
    if (n_train < 0 || n_query <= 0 || K < 1 || !l || !sigma0) return OR_E_ARG;
    for (int32_t k = 0; k < K; ++k)
        if (!(l[k] > 0) || !(sigma0[k] > 0)) return OR_E_ARG;
    for (int64_t t = 0; t < n_train; ++t)
        if (train_label[t] < 0 || train_label[t] >= K) return OR_E_INPUT;
    for (int64_t h = 0; h < n_query; ++h)
        if (query_label[h] < 0 || query_label[h] >= K) return OR_E_INPUT;
    double *A = alpha_q ? alpha_q : (double *)malloc(sizeof(double) * n_query * K);
    double *G = (double *)malloc(sizeof(double) * n_query * K);
    if (!A || !G) { if (!alpha_q) free(A); free(G); return OR_E_OOM; }
    const double H = (double)n_query;
    double tot = 0.0;
    for (int64_t h = 0; h < n_query; ++h) {
        double *a = A + h * K;
        for (int k = 0; k < K; ++k) a[k] = alpha0;
        for (int64_t t = 0; t < n_train; ++t) {
            const int32_t y = train_label[t];
            double dx = train_xyz[3 * t] - query_xyz[3 * h];
            double dy = train_xyz[3 * t + 1] - query_xyz[3 * h + 1];
            double dz = train_xyz[3 * t + 2] - query_xyz[3 * h + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 < l[y] * l[y])) continue;
            a[y] += sigma0[y] * oracle_kernel_f(sqrt(d2) / l[y]);
        }
        double S = 0.0;
        for (int k = 0; k < K; ++k) S += a[k];
        tot += -log(a[query_label[h]] / S);
        for (int k = 0; k < K; ++k)
            G[h * K + k] = -((k == query_label[h] ? 1.0 / a[k] : 0.0) - 1.0 / S) / H;
    }
    if (loss) *loss = tot / H;
    if (grad_l) memset(grad_l, 0, sizeof(double) * K);
    if (grad_sigma0) memset(grad_sigma0, 0, sizeof(double) * K);
    if (grad_train) memset(grad_train, 0, sizeof(double) * 3 * n_train);
    if (grad_query) memset(grad_query, 0, sizeof(double) * 3 * n_query);
    for (int64_t h = 0; h < n_query; ++h) {
        for (int64_t t = 0; t < n_train; ++t) {
            const int32_t y = train_label[t];
            const double L = l[y], S0 = sigma0[y];
            double dx = train_xyz[3 * t] - query_xyz[3 * h];
            double dy = train_xyz[3 * t + 1] - query_xyz[3 * h + 1];
            double dz = train_xyz[3 * t + 2] - query_xyz[3 * h + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 < L * L)) continue;
            double r = sqrt(d2) / L;
            double g = G[h * K + y];
            if (grad_sigma0) grad_sigma0[y] += g * oracle_kernel_f(r);
            if (grad_l) grad_l[y] += g * S0 * oracle_kernel_df(r) * (-r / L);
            double c = g * S0 * oracle_kernel_df_over_r(r) / (L * L);
            if (grad_train) {
                grad_train[3 * t] += c * dx;
                grad_train[3 * t + 1] += c * dy;
                grad_train[3 * t + 2] += c * dz;
            }
            if (grad_query) {
                grad_query[3 * h] -= c * dx;
                grad_query[3 * h + 1] -= c * dy;
                grad_query[3 * h + 2] -= c * dz;
            }
        }
    }
    if (!alpha_q) free(A);
    free(G);
    return OR_OK;
}

/* Threads of the tile-parallel map insert (results do not depend on it). */
int oracle_set_num_threads(int n)
{
    if (n < 1) return OR_E_ARG;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return OR_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
