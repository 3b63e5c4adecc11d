/*
 * CPU oracle of the permutohedral-lattice E-step (FilterReg, Sec. 4).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant generator with the GPU library.
 *
 * What it computes (Sec. 4.1-4.2, Eq. 6, 8, 9, 11, 14):
 *   G(f_x) = sum_y K(f_x, f_y) v_y,   v_y = [1, y, n_y]
 * where K is the kernel of a permutohedral lattice that is built ONCE from the
 * observation Y (splat) and read at the model points X (slice), with no blur
 * (the reading of the customised filter; Sec. 3.2 builds the index once, Sec.
 * 4.2 says the customisation removes the per-iteration rebuild).
 *
 * Numerics.  The lattice key of a point is an integer decided by floating
 * point, so it is taken in the precision of the GPU kernel: every operation of
 * the key path (scale, elevate, round, rank) is one IEEE binary32 operation in
 * a fixed order, and this file is compiled with -ffp-contract=off so that no
 * multiply-add is fused.  Everything downstream of the integer decision
 * (barycentric weights, splat sums, slice sums) is binary64.
 *
 * Embedding (the permutohedral lattice of Adams et al. 2010, cited in Sec. 4.2):
 *   1. cf_i = p_i * k_i  (k_i folds the feature normalisation 1/sigma_i and the
 *      lattice scale sqrt(2/3) (d+1) / sqrt((i+1)(i+2)))
 *   2. elevate into the hyperplane sum(e) = 0 of R^(d+1):
 *      e_j = (cf_j + ... + cf_(d-1)) - j cf_(j-1) for j = d..1, e_0 = sum cf
 *   3. g_j = multiple of (d+1) nearest to e_j (ties to the lower one)
 *   4. rank_j = #{i : delta_i > delta_j} + #{i < j : delta_i == delta_j},
 *      delta = e - g
 *   5. s = sum(g)/(d+1); rank_j += s; a rank that leaves [0, d] wraps by (d+1)
 *      and moves g_j by -/+ (d+1)
 *   6. barycentric weights from the rank-sorted deltas (units of d+1):
 *      b_k = u_(d-k) - u_(d-k+1) for k >= 1, b_0 = 1 + u_(d) - u_(0),
 *      u_(r) = delta of the coordinate of rank r, divided by d+1
 *   7. vertex k: v_k[j] = g_j + k - (d+1) [rank_j > d - k]; its key is the
 *      first d coordinates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 32

/* k_i = sqrt(2/3) (d+1) / (sigma_i sqrt((i+1)(i+2))), rounded once to binary32. */
void or_scale_factors(int d, const double *sigma, float *k)
{
    for (int i = 0; i < d; i++)
        k[i] = (float)(sqrt(2.0 / 3.0) * (double)(d + 1) / (sigma[i] * sqrt((double)((i + 1) * (i + 2)))));
}

/*
 * Embed one d-dimensional raw feature p (positions, then normals) with
 * per-dimension factors k.  Writes the d+1 vertex keys (row k holds d int32
 * coordinates), their barycentric weights b (binary64) and, if elev != NULL,
 * the elevated binary32 coordinates e.
 */
void or_embed(int d, const float *p, const float *k, int32_t *keys, double *b, float *elev)
{
    const int D = d + 1;
    float e[OR_MAXD + 1];
    float S = 0.0f;
    for (int j = d; j >= 1; j--) {
        float cf = p[j - 1] * k[j - 1];
        float jc = (float)j * cf;
        e[j] = S - jc;
        S = S + cf;
    }
    e[0] = S;

    const float invD = (float)(1.0 / (double)D);
    const float fD = (float)D;
    int32_t g[OR_MAXD + 1];
    int32_t sum_g = 0;
    for (int j = 0; j < D; j++) {
        float v = e[j] * invD;
        float up = ceilf(v) * fD;
        float dn = floorf(v) * fD;
        float du = up - e[j];
        float dd = e[j] - dn;
        g[j] = (du < dd) ? (int32_t)up : (int32_t)dn;
        sum_g += g[j];
    }
    const int32_t s = sum_g / D;

    float delta[OR_MAXD + 1];
    for (int j = 0; j < D; j++)
        delta[j] = e[j] - (float)g[j];

    int32_t rank[OR_MAXD + 1];
    for (int j = 0; j < D; j++) {
        int32_t r = 0;
        for (int i = 0; i < D; i++) {
            if (delta[i] > delta[j]) r++;
            else if (i < j && delta[i] == delta[j]) r++;
        }
        rank[j] = r;
    }

    for (int j = 0; j < D; j++) {
        rank[j] += s;
        if (rank[j] < 0) { rank[j] += D; g[j] += D; }
        else if (rank[j] > d) { rank[j] -= D; g[j] -= D; }
    }

    double u[OR_MAXD + 1] = {0};
    for (int j = 0; j < D; j++)
        u[rank[j]] = ((double)e[j] - (double)g[j]) / (double)D;
    b[0] = 1.0 + u[d] - u[0];
    for (int kk = 1; kk <= d; kk++)
        b[kk] = u[d - kk] - u[d - kk + 1];

    for (int kk = 0; kk < D; kk++)
        for (int j = 0; j < d; j++)
            keys[kk * d + j] = g[j] + kk - ((rank[j] > d - kk) ? D : 0);

    if (elev)
        for (int j = 0; j < D; j++) elev[j] = e[j];
}

/* ----------------------------------------------------------------------- */
/* Splat: the lattice built from the observation (Sec. 3.2, Eq. 14).        */
/* ----------------------------------------------------------------------- */

typedef struct {
    int32_t key[OR_MAXD];
    int64_t point;
    int32_t vertex;   /* which of the d+1 simplex vertices */
    double b;
} or_record;

static int g_sort_d;

static int cmp_keys(const int32_t *a, const int32_t *b, int d)
{
    for (int j = 0; j < d; j++) {
        if (a[j] < b[j]) return -1;
        if (a[j] > b[j]) return 1;
    }
    return 0;
}

static int cmp_record(const void *pa, const void *pb)
{
    const or_record *a = (const or_record *)pa, *b = (const or_record *)pb;
    int c = cmp_keys(a->key, b->key, g_sort_d);
    if (c) return c;
    if (a->point != b->point) return a->point < b->point ? -1 : 1;
    return a->vertex - b->vertex;
}

/*
 * Build the lattice of n observation points.
 *   feat : n x d raw features (row-major binary32)
 *   vals : n x nv values per point (binary64; [1, y, n_y] for the E-step)
 * Every point adds to all d+1 vertices of its simplex, including those whose
 * weight is zero; occupancy counts these incidences, so sum(occ) = (d+1) n.
 * Outputs (capacity (d+1) n rows): the distinct keys in lexicographic order,
 * their occupancy, and the per-vertex sums of b * vals accumulated in the
 * order of increasing point index.  Returns the number of vertices.
 */
int64_t or_lattice_build(int d, int nv, int64_t n, const float *feat, const double *vals, const float *k,
                         int32_t *keys_out, int32_t *occ_out, double *vals_out)
{
    const int D = d + 1;
    if (n <= 0) return 0;
    or_record *rec = (or_record *)malloc(sizeof(or_record) * (size_t)(n * D));
    if (!rec) return -1;
    int32_t keys[(OR_MAXD + 1) * OR_MAXD];
    double b[OR_MAXD + 1];
    for (int64_t i = 0; i < n; i++) {
        or_embed(d, feat + i * d, k, keys, b, NULL);
        for (int kk = 0; kk < D; kk++) {
            or_record *r = &rec[i * D + kk];
            memset(r->key, 0, sizeof(r->key));
            memcpy(r->key, keys + kk * d, sizeof(int32_t) * (size_t)d);
            r->point = i;
            r->vertex = kk;
            r->b = b[kk];
        }
    }
    g_sort_d = d;
    qsort(rec, (size_t)(n * D), sizeof(or_record), cmp_record);

    int64_t nvtx = -1;
    for (int64_t r = 0; r < n * D; r++) {
        if (r == 0 || cmp_keys(rec[r].key, rec[r - 1].key, d) != 0) {
            nvtx++;
            memcpy(keys_out + nvtx * d, rec[r].key, sizeof(int32_t) * (size_t)d);
            occ_out[nvtx] = 0;
            for (int c = 0; c < nv; c++) vals_out[nvtx * nv + c] = 0.0;
        }
        occ_out[nvtx] += 1;
        for (int c = 0; c < nv; c++)
            vals_out[nvtx * nv + c] += rec[r].b * vals[rec[r].point * nv + c];
    }
    free(rec);
    return nvtx + 1;
}

/* ----------------------------------------------------------------------- */
/* Slice: read the lattice at query points (Eq. 6, 9 via Eq. 11).          */
/* ----------------------------------------------------------------------- */

static int64_t find_key(const int32_t *keys, int64_t n_v, int d, const int32_t *q)
{
    int64_t lo = 0, hi = n_v - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_keys(keys + mid * d, q, d);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * out[i] = sum_k b_k(q_i) * lattice_vals[v_k(q_i)] over the vertices present
 * in the lattice (absent vertices contribute nothing).  If touched != NULL it
 * must hold n_v bytes; a vertex found by any lookup is marked 1.
 */
void or_slice(int d, int nv, int64_t n_v, const int32_t *keys, const double *lat_vals, int64_t m,
              const float *feat, const float *k, double *out, uint8_t *touched)
{
    const int D = d + 1;
    int32_t vk[(OR_MAXD + 1) * OR_MAXD];
    double b[OR_MAXD + 1];
    for (int64_t i = 0; i < m; i++) {
        double *o = out + i * nv;
        for (int c = 0; c < nv; c++) o[c] = 0.0;
        or_embed(d, feat + i * d, k, vk, b, NULL);
        for (int kk = 0; kk < D; kk++) {
            int64_t v = find_key(keys, n_v, d, vk + kk * d);
            if (v < 0) continue;
            if (touched) touched[v] = 1;
            for (int c = 0; c < nv; c++) o[c] += b[kk] * lat_vals[v * nv + c];
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Blur: the uncustomised permutohedral filter (the cited Adams et al.      */
/* method, referred to by Sec. 4.2 and rebuilt per iteration in Sec. 3.1).  */
/* ----------------------------------------------------------------------- */

/*
 * The d+1 lattice directions of the (d+1)-scaled A*_d lattice are the vectors
 * with every coordinate +1 except coordinate j, which is -d (they sum to zero
 * and connect a vertex to its nearest neighbours of the same remainder class).
 * A pass along direction j replaces each vertex value by
 *   1/2 v(x) + 1/4 v(x + e_j) + 1/4 v(x - e_j),
 * reading the previous pass's values; vertices absent from the lattice read as
 * 0 and are not created.  Passes run for j = 0..d in order; the values are
 * finally multiplied by `scale`.  `vals` (n_v x nv) is updated in place; keys
 * must be in lexicographic order (as or_lattice_build leaves them).  Returns
 * 0, or -1 when out of memory.
 */
int or_blur(int d, int nv, int64_t n_v, const int32_t *keys, double *vals, double scale)
{
    if (n_v <= 0) return 0;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n_v * nv));
    if (!tmp) return -1;
    int32_t up[OR_MAXD], dn[OR_MAXD];
    for (int j = 0; j <= d; j++) {
        for (int64_t v = 0; v < n_v; v++) {
            const int32_t *key = keys + v * d;
            for (int i = 0; i < d; i++) {
                up[i] = key[i] + 1;
                dn[i] = key[i] - 1;
            }
            if (j < d) {
                up[j] = key[j] - d;
                dn[j] = key[j] + d;
            }
            const int64_t a = find_key(keys, n_v, d, up);
            const int64_t b = find_key(keys, n_v, d, dn);
            for (int c = 0; c < nv; c++) {
                double s = 0.5 * vals[v * nv + c];
                if (a >= 0) s += 0.25 * vals[a * nv + c];
                if (b >= 0) s += 0.25 * vals[b * nv + c];
                tmp[v * nv + c] = s;
            }
        }
        memcpy(vals, tmp, sizeof(double) * (size_t)(n_v * nv));
    }
    for (int64_t q = 0; q < n_v * nv; q++) vals[q] *= scale;
    free(tmp);
    return 0;
}

/*
 * Brute force of the same kernel, with no lattice at all:
 *   out[i] = sum_j K(q_i, y_j) vals_j,
 *   K(q, y) = sum over vertex pairs (k, l) with v_k(q) == v_l(y) of b_k(q) b_l(y).
 * O(m n (d+1)^2); only for tiny inputs.  It pins splat + slice: the two must
 * agree up to binary64 rounding.
 */
void or_bf_lattice_sum(int d, int nv, int64_t n, const float *fy, const double *vals, int64_t m,
                       const float *fx, const float *k, double *out)
{
    const int D = d + 1;
    int32_t *ky = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n * D * d) + 1);
    double *by = (double *)malloc(sizeof(double) * (size_t)(n * D) + 1);
    for (int64_t j = 0; j < n; j++)
        or_embed(d, fy + j * d, k, ky + j * D * d, by + j * D, NULL);
    int32_t kx[(OR_MAXD + 1) * OR_MAXD];
    double bx[OR_MAXD + 1];
    for (int64_t i = 0; i < m; i++) {
        double *o = out + i * nv;
        for (int c = 0; c < nv; c++) o[c] = 0.0;
        or_embed(d, fx + i * d, k, kx, bx, NULL);
        for (int64_t j = 0; j < n; j++) {
            double K = 0.0;
            for (int a = 0; a < D; a++)
                for (int l = 0; l < D; l++)
                    if (cmp_keys(kx + a * d, ky + (j * D + l) * d, d) == 0)
                        K += bx[a] * by[j * D + l];
            if (K != 0.0)
                for (int c = 0; c < nv; c++) o[c] += K * vals[j * nv + c];
        }
    }
    free(ky);
    free(by);
}

/* Pinned binary32 rigid transform: p' = ((R0 x + R1 y) + R2 z) + t, no fused multiply-add. */
void or_transform_f32(int64_t m, const float *mat /* 12: row-major [R | t] */, const float *p, float *out,
                      int with_translation)
{
    for (int64_t i = 0; i < m; i++) {
        const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
        for (int r = 0; r < 3; r++) {
            float a = mat[4 * r + 0] * x;
            float bb = mat[4 * r + 1] * y;
            float c = mat[4 * r + 2] * z;
            float s = a + bb;
            s = s + c;
            if (with_translation) s = s + mat[4 * r + 3];
            out[3 * i + r] = s;
        }
    }
}

/* Embed n points (row-major n x d); keys n x (d+1) x d, b n x (d+1), elev n x (d+1) or NULL. */
void or_embed_many(int d, int64_t n, const float *feat, const float *k, int32_t *keys, double *b, float *elev)
{
    const int D = d + 1;
    for (int64_t i = 0; i < n; i++)
        or_embed(d, feat + i * d, k, keys + i * D * d, b + i * D, elev ? elev + i * D : NULL);
}
