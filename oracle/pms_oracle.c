/*
 * CPU oracle for boundary-matrix reduction over F2 and for the filtrations
 * that feed it.  TEST INFRASTRUCTURE ONLY: it is loaded by the test suite,
 * the smoke check and the CPU baseline of the benchmark, never by the GPU
 * library, and it shares no code with it.
 *
 * Everything here is deliberately plain and sequential:
 *   - oracle_reduce_standard : the standard reduction (Alg. "Standard
 *     reduction", Sec. 1).  Columns are processed left to right; a column
 *     is repeatedly added the earlier column that shares its low until it
 *     is zero or its low is unique.  The result low* is the entrywise
 *     minimum of low (eq. "low"), a property of the complex (Sec. 2.3).
 *   - oracle_reduce_twist    : the same reduction with the twist / clearing
 *     order (Alg. "Standard reduction with a twist", Sec. 2.4): dimensions
 *     from high to low, and column low(j) is zeroed once column j is reduced.
 *   - builders for Vietoris-Rips (Sec. 2.2, diam <= 2r, i.e. monotone in the
 *     squared diameter) and for lower-star filtrations of a Freudenthal grid
 *     triangulation, ordered compatibly (faces before cofaces, Sec. 2.2) by
 *     the key (value, dimension, lexicographic vertex tuple), with the
 *     boundary matrix of eq. "def:boundary_matrix" in CSC form.
 *
 * Index convention: 0-based; -1 stands for the paper's 0 ("no entry").
 * Compile with -ffp-contract=off: the FP32 squared distances are computed as
 * d_k = x_ak - x_bk, s = ((d_0*d_0) + d_1*d_1) + ..., each step rounded.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOT_COMPATIBLE (-2)
#define ORC_ERR_OOM (-3)

/* ------------------------------------------------------------------ */
/* growable int32 vector                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t *a;
    int64_t n, cap;
} ivec;

static int ivec_reserve(ivec *v, int64_t cap)
{
    if (cap <= v->cap) return 0;
    int64_t nc = v->cap ? v->cap : 8;
    while (nc < cap) nc *= 2;
    int32_t *p = (int32_t *)realloc(v->a, (size_t)nc * sizeof(int32_t));
    if (!p) return -1;
    v->a = p;
    v->cap = nc;
    return 0;
}

/* Sum of two F2 columns stored as ascending row lists: the sorted
 * symmetric difference.  Rows present in both cancel (1 + 1 = 0). */
static int64_t f2_add(const int32_t *x, int64_t nx, const int32_t *y, int64_t ny, int32_t *out)
{
    int64_t i = 0, j = 0, k = 0;
    while (i < nx && j < ny) {
        if (x[i] < y[j]) out[k++] = x[i++];
        else if (y[j] < x[i]) out[k++] = y[j++];
        else { i++; j++; }
    }
    while (i < nx) out[k++] = x[i++];
    while (j < ny) out[k++] = y[j++];
    return k;
}

/* Input check shared by both reductions: rows of every column strictly
 * ascending and strictly above the diagonal (the matrix of a compatibly
 * ordered filtration is strictly upper triangular); when dims are given, a
 * row of column j must have dimension dim[j] - 1 (codimension-1 faces). */
static int check_boundary(int64_t m, const int64_t *col_ptr, const int32_t *rows, const int8_t *dim)
{
    if (m < 0 || (m > 0 && (!col_ptr || (!rows && col_ptr[m] > 0)))) return ORC_ERR_ARG;
    if (m == 0) return ORC_OK;
    if (col_ptr[0] != 0) return ORC_ERR_ARG;
    for (int64_t j = 0; j < m; j++) {
        if (col_ptr[j + 1] < col_ptr[j]) return ORC_ERR_ARG;
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
            int32_t r = rows[p];
            if (r < 0 || (int64_t)r >= j) return ORC_ERR_NOT_COMPATIBLE;
            if (p > col_ptr[j] && rows[p - 1] >= r) return ORC_ERR_NOT_COMPATIBLE;
            if (dim && dim[r] != dim[j] - 1) return ORC_ERR_NOT_COMPATIBLE;
        }
    }
    return ORC_OK;
}

/*
 * Standard reduction.  stats (optional, 2 entries): [0] number of column
 * additions, [1] number of non-trivial scalar XORs (entries of the union of
 * the two supports, i.e. the operations 1+1, 1+0, 0+1 of Sec. 4.1).
 */
int oracle_reduce_standard(int64_t m, const int64_t *col_ptr, const int32_t *rows,
                           int32_t *low_star, int64_t *stats)
{
    int rc = check_boundary(m, col_ptr, rows, NULL);
    if (rc) return rc;
    int64_t adds = 0, xors = 0;
    ivec *R = (ivec *)calloc((size_t)(m > 0 ? m : 1), sizeof(ivec));
    int32_t *piv = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    ivec cur = {0}, tmp = {0};
    if (!R || !piv) { rc = ORC_ERR_OOM; goto done; }
    for (int64_t i = 0; i < m; i++) piv[i] = -1;

    for (int64_t j = 0; j < m; j++) {
        int64_t len = col_ptr[j + 1] - col_ptr[j];
        if (ivec_reserve(&cur, len)) { rc = ORC_ERR_OOM; goto done; }
        memcpy(cur.a, rows + col_ptr[j], (size_t)len * sizeof(int32_t));
        cur.n = len;
        /* while some earlier column has the same low, add it */
        while (cur.n > 0 && piv[cur.a[cur.n - 1]] >= 0) {
            const ivec *src = &R[piv[cur.a[cur.n - 1]]];
            if (ivec_reserve(&tmp, cur.n + src->n)) { rc = ORC_ERR_OOM; goto done; }
            int64_t k = f2_add(cur.a, cur.n, src->a, src->n, tmp.a);
            adds++;
            xors += (cur.n + src->n + k) / 2; /* |x u y| = (|x|+|y|+|x (+) y|)/2 */
            tmp.n = k;
            ivec t = cur; cur = tmp; tmp = t;
        }
        if (cur.n > 0) {
            low_star[j] = cur.a[cur.n - 1];
            piv[cur.a[cur.n - 1]] = (int32_t)j;
            R[j] = cur; /* keep the reduced column as a future source */
            memset(&cur, 0, sizeof(cur));
        } else {
            low_star[j] = -1;
        }
    }
    if (stats) { stats[0] = adds; stats[1] = xors; }
done:
    if (R) { for (int64_t j = 0; j < m; j++) free(R[j].a); free(R); }
    free(piv); free(cur.a); free(tmp.a);
    return rc;
}

/*
 * Standard reduction with a twist: dimensions from the top down; after a
 * column j is reduced to a non-zero column, column low(j) is known to be
 * positive and is set to zero without being reduced (clearing).
 */
int oracle_reduce_twist(int64_t m, const int64_t *col_ptr, const int32_t *rows, const int8_t *dim,
                        int32_t *low_star, int64_t *stats)
{
    if (!dim && m > 0) return ORC_ERR_ARG;
    int rc = check_boundary(m, col_ptr, rows, dim);
    if (rc) return rc;
    int64_t adds = 0, xors = 0;
    int maxd = 0;
    for (int64_t j = 0; j < m; j++) if (dim[j] > maxd) maxd = dim[j];
    ivec *R = (ivec *)calloc((size_t)(m > 0 ? m : 1), sizeof(ivec));
    int32_t *piv = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    char *cleared = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    ivec cur = {0}, tmp = {0};
    if (!R || !piv || !cleared) { rc = ORC_ERR_OOM; goto done; }
    for (int64_t i = 0; i < m; i++) { piv[i] = -1; low_star[i] = -1; }

    for (int d = maxd; d >= 1; d--) {
        for (int64_t j = 0; j < m; j++) {
            if (dim[j] != d) continue;
            if (cleared[j]) { low_star[j] = -1; continue; }
            int64_t len = col_ptr[j + 1] - col_ptr[j];
            if (ivec_reserve(&cur, len)) { rc = ORC_ERR_OOM; goto done; }
            memcpy(cur.a, rows + col_ptr[j], (size_t)len * sizeof(int32_t));
            cur.n = len;
            while (cur.n > 0 && piv[cur.a[cur.n - 1]] >= 0) {
                const ivec *src = &R[piv[cur.a[cur.n - 1]]];
                if (ivec_reserve(&tmp, cur.n + src->n)) { rc = ORC_ERR_OOM; goto done; }
                int64_t k = f2_add(cur.a, cur.n, src->a, src->n, tmp.a);
                adds++;
                xors += (cur.n + src->n + k) / 2;
                tmp.n = k;
                ivec t = cur; cur = tmp; tmp = t;
            }
            if (cur.n > 0) {
                int32_t i = cur.a[cur.n - 1];
                low_star[j] = i;
                piv[i] = (int32_t)j;
                cleared[i] = 1; /* column i is positive: zero it */
                R[j] = cur;
                memset(&cur, 0, sizeof(cur));
            } else {
                low_star[j] = -1;
            }
        }
    }
    if (stats) { stats[0] = adds; stats[1] = xors; }
done:
    if (R) { for (int64_t j = 0; j < m; j++) free(R[j].a); free(R); }
    free(piv); free(cleared); free(cur.a); free(tmp.a);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Filtrations                                                         */
/* ------------------------------------------------------------------ */
#define ORC_MAXV 4 /* simplices of dimension <= 3 */

typedef struct {
    double value;   /* filtration value (int64 squared distance or f32, exact in double) */
    int32_t dim;
    int32_t v[ORC_MAXV]; /* ascending vertex ids, -1 padded */
} simplex_rec;

typedef struct {
    int64_t m, nnz;
    int64_t *col_ptr; /* [m+1] */
    int32_t *rows;    /* [nnz] ascending per column */
    int8_t *dim;      /* [m] */
    double *value;    /* [m] */
    int32_t *verts;   /* [m * 4], ascending, -1 padded */
} oracle_filtration;

typedef struct {
    simplex_rec *s;
    int64_t n, cap;
} svec;

static int svec_push(svec *sv, double value, int dim, const int32_t *v)
{
    if (sv->n == sv->cap) {
        int64_t nc = sv->cap ? 2 * sv->cap : 1024;
        simplex_rec *p = (simplex_rec *)realloc(sv->s, (size_t)nc * sizeof(simplex_rec));
        if (!p) return -1;
        sv->s = p;
        sv->cap = nc;
    }
    simplex_rec *r = &sv->s[sv->n++];
    r->value = value;
    r->dim = dim;
    for (int k = 0; k < ORC_MAXV; k++) r->v[k] = k <= dim ? v[k] : -1;
    return 0;
}

static int cmp_lex(const simplex_rec *a, const simplex_rec *b)
{
    for (int k = 0; k < ORC_MAXV; k++) {
        if (a->v[k] < b->v[k]) return -1;
        if (a->v[k] > b->v[k]) return 1;
    }
    return 0;
}

/* Filtration order: value, then dimension, then lexicographic vertex tuple.
 * (value, dim) already puts every face before its cofaces. */
static int cmp_filtration(const void *pa, const void *pb)
{
    const simplex_rec *a = (const simplex_rec *)pa, *b = (const simplex_rec *)pb;
    if (a->value < b->value) return -1;
    if (a->value > b->value) return 1;
    if (a->dim != b->dim) return a->dim < b->dim ? -1 : 1;
    return cmp_lex(a, b);
}

typedef struct {
    int32_t dim;
    int32_t v[ORC_MAXV];
    int64_t index;
} tuple_index;

static int cmp_tuple(const void *pa, const void *pb)
{
    const tuple_index *a = (const tuple_index *)pa, *b = (const tuple_index *)pb;
    if (a->dim != b->dim) return a->dim < b->dim ? -1 : 1;
    for (int k = 0; k < ORC_MAXV; k++) {
        if (a->v[k] < b->v[k]) return -1;
        if (a->v[k] > b->v[k]) return 1;
    }
    return 0;
}

/* Sort the simplices into filtration order and write the boundary matrix:
 * column j holds the filtration indices of the codimension-1 faces of
 * simplex j, ascending. */
static int finish_filtration(svec *sv, oracle_filtration *out)
{
    int64_t m = sv->n;
    memset(out, 0, sizeof(*out));
    qsort(sv->s, (size_t)m, sizeof(simplex_rec), cmp_filtration);
    tuple_index *tab = (tuple_index *)malloc((size_t)(m > 0 ? m : 1) * sizeof(tuple_index));
    if (!tab) return ORC_ERR_OOM;
    int64_t nnz = 0;
    for (int64_t j = 0; j < m; j++) {
        tab[j].dim = sv->s[j].dim;
        memcpy(tab[j].v, sv->s[j].v, sizeof(tab[j].v));
        tab[j].index = j;
        nnz += sv->s[j].dim > 0 ? sv->s[j].dim + 1 : 0;
    }
    qsort(tab, (size_t)m, sizeof(tuple_index), cmp_tuple);
    out->m = m;
    out->nnz = nnz;
    out->col_ptr = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    out->rows = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    out->dim = (int8_t *)malloc((size_t)(m > 0 ? m : 1));
    out->value = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    out->verts = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * ORC_MAXV * sizeof(int32_t));
    if (!out->col_ptr || !out->rows || !out->dim || !out->value || !out->verts) {
        free(tab);
        return ORC_ERR_OOM;
    }
    int64_t p = 0;
    out->col_ptr[0] = 0;
    for (int64_t j = 0; j < m; j++) {
        const simplex_rec *s = &sv->s[j];
        out->dim[j] = (int8_t)s->dim;
        out->value[j] = s->value;
        memcpy(out->verts + j * ORC_MAXV, s->v, sizeof(s->v));
        if (s->dim > 0) {
            int32_t face_rows[ORC_MAXV];
            for (int drop = 0; drop <= s->dim; drop++) {
                tuple_index key;
                key.dim = s->dim - 1;
                int q = 0;
                for (int k = 0; k <= s->dim; k++) if (k != drop) key.v[q++] = s->v[k];
                for (; q < ORC_MAXV; q++) key.v[q] = -1;
                tuple_index *hit = (tuple_index *)bsearch(&key, tab, (size_t)m, sizeof(tuple_index), cmp_tuple);
                if (!hit) { free(tab); return ORC_ERR_NOT_COMPATIBLE; } /* face missing: not a complex */
                face_rows[drop] = (int32_t)hit->index;
            }
            /* insertion sort: ascending row order */
            for (int a = 1; a <= s->dim; a++) {
                int32_t x = face_rows[a];
                int b = a - 1;
                while (b >= 0 && face_rows[b] > x) { face_rows[b + 1] = face_rows[b]; b--; }
                face_rows[b + 1] = x;
            }
            for (int k = 0; k <= s->dim; k++) out->rows[p++] = face_rows[k];
        }
        out->col_ptr[j + 1] = p;
    }
    free(tab);
    return ORC_OK;
}

void oracle_filtration_free(oracle_filtration *f)
{
    if (!f) return;
    free(f->col_ptr); free(f->rows); free(f->dim); free(f->value); free(f->verts);
    memset(f, 0, sizeof(*f));
}

/* Vietoris-Rips complex up to maxdim (<= 3) on a point cloud.  The value of
 * a simplex is its squared diameter (the largest squared pairwise distance
 * of its vertices); a simplex is present when that value is <= thr.  Vertices
 * have value 0.  edge_value holds the n x n squared-distance matrix. */
static int vr_from_distances(const double *edge_value, int32_t n, double thr, int has_thr,
                             int32_t maxdim, oracle_filtration *out)
{
    svec sv = {0};
    int32_t v[ORC_MAXV];
    char *adj = (char *)calloc((size_t)n * (size_t)n, 1);
    if (!adj) return ORC_ERR_OOM;
#define EV(a, b) edge_value[(int64_t)(a) * n + (b)]
#define ADJ(a, b) adj[(int64_t)(a) * n + (b)]
    for (int32_t a = 0; a < n; a++)
        for (int32_t b = 0; b < n; b++)
            ADJ(a, b) = (a != b) && (!has_thr || EV(a, b) <= thr);
    int rc = ORC_OK;
    for (int32_t a = 0; a < n; a++) {
        v[0] = a;
        if (svec_push(&sv, 0.0, 0, v)) { rc = ORC_ERR_OOM; goto fail; }
    }
    if (maxdim >= 1)
        for (int32_t a = 0; a < n; a++)
            for (int32_t b = a + 1; b < n; b++) {
                if (!ADJ(a, b)) continue;
                v[0] = a; v[1] = b;
                if (svec_push(&sv, EV(a, b), 1, v)) { rc = ORC_ERR_OOM; goto fail; }
            }
    if (maxdim >= 2)
        for (int32_t a = 0; a < n; a++)
            for (int32_t b = a + 1; b < n; b++) {
                if (!ADJ(a, b)) continue;
                for (int32_t c = b + 1; c < n; c++) {
                    if (!ADJ(a, c) || !ADJ(b, c)) continue;
                    double val = EV(a, b);
                    if (EV(a, c) > val) val = EV(a, c);
                    if (EV(b, c) > val) val = EV(b, c);
                    v[0] = a; v[1] = b; v[2] = c;
                    if (svec_push(&sv, val, 2, v)) { rc = ORC_ERR_OOM; goto fail; }
                    if (maxdim >= 3)
                        for (int32_t d = c + 1; d < n; d++) {
                            if (!ADJ(a, d) || !ADJ(b, d) || !ADJ(c, d)) continue;
                            double w = val;
                            if (EV(a, d) > w) w = EV(a, d);
                            if (EV(b, d) > w) w = EV(b, d);
                            if (EV(c, d) > w) w = EV(c, d);
                            v[3] = d;
                            if (svec_push(&sv, w, 3, v)) { rc = ORC_ERR_OOM; goto fail; }
                        }
                }
            }
#undef EV
#undef ADJ
    rc = finish_filtration(&sv, out);
fail:
    free(adj);
    free(sv.s);
    return rc;
}

/* Integer point cloud: exact int64 squared distances. thr < 0: no threshold. */
int oracle_build_vr_i32(const int32_t *pts, int32_t n, int32_t D, int64_t thr, int32_t maxdim,
                        oracle_filtration *out)
{
    if (n < 0 || D < 1 || maxdim < 0 || maxdim > 3 || (n > 0 && !pts) || !out) return ORC_ERR_ARG;
    double *ev = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!ev) return ORC_ERR_OOM;
    for (int32_t a = 0; a < n; a++)
        for (int32_t b = 0; b < n; b++) {
            int64_t s = 0;
            for (int32_t k = 0; k < D; k++) {
                int64_t d = (int64_t)pts[(int64_t)a * D + k] - (int64_t)pts[(int64_t)b * D + k];
                s += d * d;
            }
            ev[(int64_t)a * n + b] = (double)s; /* exact: s < 2^53 */
        }
    int rc = vr_from_distances(ev, n, (double)thr, thr >= 0, maxdim, out);
    free(ev);
    return rc;
}

/* FP32 point cloud: squared distance rounded to float step by step, with
 * the coordinates taken in index order. thr < 0: no threshold. */
int oracle_build_vr_f32(const float *pts, int32_t n, int32_t D, float thr, int32_t maxdim,
                        oracle_filtration *out)
{
    if (n < 0 || D < 1 || maxdim < 0 || maxdim > 3 || (n > 0 && !pts) || !out) return ORC_ERR_ARG;
    double *ev = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!ev) return ORC_ERR_OOM;
    for (int32_t a = 0; a < n; a++)
        for (int32_t b = 0; b < n; b++) {
            volatile float s = 0.0f;
            for (int32_t k = 0; k < D; k++) {
                volatile float d = pts[(int64_t)a * D + k] - pts[(int64_t)b * D + k];
                volatile float sq = d * d;
                s = s + sq;
            }
            ev[(int64_t)a * n + b] = (double)s;
        }
    int rc = vr_from_distances(ev, n, (double)thr, thr >= 0.0f, maxdim, out);
    free(ev);
    return rc;
}

/* Same cloud in FP64 (reference for gradients): squared distances in double. */
int oracle_build_vr_f64(const double *pts, int32_t n, int32_t D, double thr, int32_t maxdim,
                        oracle_filtration *out)
{
    if (n < 0 || D < 1 || maxdim < 0 || maxdim > 3 || (n > 0 && !pts) || !out) return ORC_ERR_ARG;
    double *ev = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!ev) return ORC_ERR_OOM;
    for (int32_t a = 0; a < n; a++)
        for (int32_t b = 0; b < n; b++) {
            double s = 0.0;
            for (int32_t k = 0; k < D; k++) {
                double d = pts[(int64_t)a * D + k] - pts[(int64_t)b * D + k];
                s = s + d * d;
            }
            ev[(int64_t)a * n + b] = s;
        }
    int rc = vr_from_distances(ev, n, thr, thr >= 0.0, maxdim, out);
    free(ev);
    return rc;
}

/* Lower-star filtration of the Freudenthal triangulation of an
 * nx x ny x nz vertex grid (x fastest: id = x + nx*(y + ny*z)).  The
 * simplices are the chains v0 < v1 < ... < vk of grid vertices whose
 * successive differences are non-zero 0/1 vectors with disjoint supports;
 * every such chain is a face of a maximal chain that starts at v0 and
 * raises one coordinate at a time.  The value of a simplex is the largest
 * value of its vertices. */
int oracle_build_lowerstar(const float *grid, int32_t nx, int32_t ny, int32_t nz, oracle_filtration *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !grid || !out) return ORC_ERR_ARG;
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int32_t ext[3] = {nx, ny, nz};
    int64_t nv = (int64_t)nx * ny * nz;
    for (int64_t i = 0; i < nv; i++)
        if (grid[i] != grid[i]) return ORC_ERR_ARG; /* NaN */
    svec sv = {0};
    int rc = ORC_OK;
    for (int32_t z = 0; z < nz; z++)
        for (int32_t y = 0; y < ny; y++)
            for (int32_t x = 0; x < nx; x++) {
                for (int p = 0; p < 6; p++) {
                    int32_t chain[4];
                    int len = 0;
                    int32_t c[3] = {x, y, z};
                    chain[len++] = x + nx * (y + ny * z);
                    for (int s = 0; s < 3; s++) {
                        c[perms[p][s]] += 1;
                        if (c[perms[p][s]] >= ext[perms[p][s]]) break;
                        chain[len++] = c[0] + nx * (c[1] + ny * c[2]);
                    }
                    /* every subset of the chain that contains its first vertex */
                    for (int mask = 0; mask < (1 << (len - 1)); mask++) {
                        int32_t v[ORC_MAXV];
                        int k = 0;
                        v[k++] = chain[0];
                        for (int b = 1; b < len; b++)
                            if (mask & (1 << (b - 1))) v[k++] = chain[b];
                        float val = grid[v[0]];
                        for (int q = 1; q < k; q++) if (grid[v[q]] > val) val = grid[v[q]];
                        if (val == 0.0f) val = 0.0f; /* -0 and +0 are one value */
                        if (svec_push(&sv, (double)val, k - 1, v)) { rc = ORC_ERR_OOM; goto fail; }
                    }
                }
            }
    /* remove duplicates (the same simplex is reached from several chains) */
    {
        qsort(sv.s, (size_t)sv.n, sizeof(simplex_rec), cmp_filtration);
        int64_t w = 0;
        for (int64_t r = 0; r < sv.n; r++) {
            if (w > 0 && sv.s[w - 1].dim == sv.s[r].dim && cmp_lex(&sv.s[w - 1], &sv.s[r]) == 0) continue;
            sv.s[w++] = sv.s[r];
        }
        sv.n = w;
    }
    rc = finish_filtration(&sv, out);
fail:
    free(sv.s);
    return rc;
}
