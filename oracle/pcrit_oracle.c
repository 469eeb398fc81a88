/*
 * pcrit_oracle.c -- plain CPU oracle for PL critical-point classification.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The GPU library never links,
 * includes or calls it, and it shares no code, header or table with it.
 *
 * What it computes (Lukasczyk et al., "Localized Topological Simplification
 * of Scalar Data", Section 3.1 and Section 4.1):
 *   - the input is a PL scalar field given at the vertices of a triangulated
 *     domain (Section 3.1);
 *   - vertices are totally ordered by value, equal values being ordered by
 *     their position in memory, i.e. by the full-resolution linear index
 *     idx = x + nx*(y + ny*z) (Section 4.1, order field);
 *   - the star of v is the set of simplices having v as a face, and the link
 *     is the set of faces of star simplices that do not meet v; the lower
 *     (upper) link is the part of the link whose vertices all come before
 *     (after) v in that order (Section 3.1);
 *   - v is regular iff both lower and upper link are non-empty and simply
 *     connected; a minimum has an empty lower link, a maximum an empty upper
 *     link, every other critical vertex is a saddle, degenerate when a link
 *     part has more than two components (Section 3.1, Fig. 3).
 *
 * The grid triangulation and the level hierarchy are readings, not paper
 * content: each cube [c, c+1]^3 of the level-k grid (stride 2^k) is cut into
 * the six tetrahedra c -> c+e_a -> c+e_a+e_b -> c+(1,1,1), one per
 * permutation (a,b,c) of the axes; a square [c, c+1]^2 is cut along its
 * (1,1) diagonal.  Level k holds the samples whose coordinates are all
 * multiples of 2^k.
 *
 * Nothing here is blocked, vectorised or table-driven: for every vertex the
 * star is enumerated cell by cell, the link simplices are collected
 * explicitly, and the components of the lower and upper link are counted
 * with a union-find over the link edges.
 *
 * Output per level vertex v: one code byte
 *   bits 0-2  #components of the lower link
 *   bits 3-5  #components of the upper link
 *   bit  6    v lies on the boundary of the level grid
 *   bit  7    v is a boundary vertex whose lower or upper link has a hole
 *             (first Betti number > 0), i.e. is connected but not simply
 *             connected
 * and the ascending list of full-resolution indices of critical vertices.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_DIMS (-2)
#define OR_E_LEVEL (-3)
#define OR_E_CAPACITY (-4)
#define OR_E_NAN (-5)
#define OR_E_OOM (-7)

typedef struct {
    int dim;          /* 2 or 3 */
    int64_t n[3];     /* full-resolution sizes along x, y, z (n[2] = 1 in 2D) */
    int64_t s;        /* stride of the level, 2^level */
    int64_t m[3];     /* number of level samples along x, y, z */
} grid_t;

/* -------------------------------------------------------------------------
 * Generic part: classify a vertex from an explicit link complex.
 * ------------------------------------------------------------------------- */

typedef struct {
    int n_lower, n_upper;       /* connected components of Lk-(v), Lk+(v) */
    int chi_lower, chi_upper;   /* Euler characteristics V - E + F */
    int b1_lower, b1_upper;     /* first Betti numbers */
    int critical;               /* not regular in the sense of Section 3.1 */
} link_result_t;

static int uf_find(int *p, int a)
{
    while (p[a] != a) {
        p[a] = p[p[a]];
        a = p[a];
    }
    return a;
}

/*
 * nv link vertices, lower[i] = 1 if link vertex i comes before v in the order
 * (else it comes after v); ne edges as pairs of link-vertex ids; nt triangles
 * as triples.  link_dim = 1 for a 1-dimensional link (2D domains), 2 for a
 * 2-dimensional link (3D domains).  link_closed = 1 if the link is a closed
 * manifold (a circle or a 2-sphere: v interior), 0 if it is a path or a disk.
 *
 * The Betti numbers use: a 1-complex has b1 = E - V + b0; a subcomplex X of a
 * 2-sphere or of a disk has b2(X) = 1 exactly when X is the whole sphere, and
 * b1 = b0 + b2 - chi.
 */
static void classify_link_part(int nv, const int *in_part, int ne,
                               const int (*edges)[2], int nt,
                               const int (*tris)[3], int link_dim,
                               int link_closed, int *n_comp, int *chi,
                               int *b1)
{
    int parent[64];
    int V = 0, E = 0, F = 0;
    for (int i = 0; i < nv; i++) {
        parent[i] = i;
        V += in_part[i];
    }
    for (int e = 0; e < ne; e++) {
        int a = edges[e][0], b = edges[e][1];
        if (in_part[a] && in_part[b]) {
            E++;
            int ra = uf_find(parent, a), rb = uf_find(parent, b);
            if (ra != rb)
                parent[ra] = rb;
        }
    }
    for (int t = 0; t < nt; t++)
        if (in_part[tris[t][0]] && in_part[tris[t][1]] && in_part[tris[t][2]])
            F++;
    int c = 0;
    for (int i = 0; i < nv; i++)
        if (in_part[i] && uf_find(parent, i) == i)
            c++;
    *n_comp = c;
    *chi = V - E + F;
    if (link_dim == 1) {
        *b1 = E - V + c;
    } else {
        int b2 = (link_closed && V == nv && F == nt) ? 1 : 0;
        *b1 = c + b2 - (V - E + F);
    }
}

static void classify_link(int nv, const int *lower, int ne,
                          const int (*edges)[2], int nt, const int (*tris)[3],
                          int link_dim, int link_closed, link_result_t *r)
{
    int upper[64];
    for (int i = 0; i < nv; i++)
        upper[i] = !lower[i];
    classify_link_part(nv, lower, ne, edges, nt, tris, link_dim, link_closed,
                       &r->n_lower, &r->chi_lower, &r->b1_lower);
    classify_link_part(nv, upper, ne, edges, nt, tris, link_dim, link_closed,
                       &r->n_upper, &r->chi_upper, &r->b1_upper);
    /* regular iff both parts are non-empty, connected and without holes */
    int regular = r->n_lower == 1 && r->n_upper == 1 && r->b1_lower == 0 &&
                  r->b1_upper == 0;
    r->critical = !regular;
}

/* Exported for the tests: classify from a hand-written link (e.g. the link
 * of Fig. 3).  out[6] = {n_lower, n_upper, chi_lower, chi_upper, b1_lower,
 * b1_upper}; returns 1 if critical, 0 if regular, <0 on bad arguments. */
int oracle_classify_link(int nv, const int *lower, int ne, const int *edges,
                         int nt, const int *tris, int link_dim,
                         int link_closed, int *out)
{
    if (nv < 0 || nv > 64 || ne < 0 || nt < 0 || !lower || !out ||
        (ne && !edges) || (nt && !tris) || (link_dim != 1 && link_dim != 2))
        return OR_E_ARG;
    for (int e = 0; e < 2 * ne; e++)
        if (edges[e] < 0 || edges[e] >= nv)
            return OR_E_ARG;
    for (int t = 0; t < 3 * nt; t++)
        if (tris[t] < 0 || tris[t] >= nv)
            return OR_E_ARG;
    link_result_t r;
    classify_link(nv, lower, ne, (const int(*)[2])edges, nt,
                  (const int(*)[3])tris, link_dim, link_closed, &r);
    out[0] = r.n_lower;
    out[1] = r.n_upper;
    out[2] = r.chi_lower;
    out[3] = r.chi_upper;
    out[4] = r.b1_lower;
    out[5] = r.b1_upper;
    return r.critical;
}

/* -------------------------------------------------------------------------
 * Grid part: the star and link of a level vertex, collected cell by cell.
 * ------------------------------------------------------------------------- */

static int64_t full_index(const grid_t *g, const int64_t q[3])
{
    return g->s * q[0] + g->n[0] * (g->s * q[1] + g->n[1] * (g->s * q[2]));
}

static float value_at(const grid_t *g, const float *f, const int64_t q[3])
{
    return f[full_index(g, q)];
}

typedef struct {
    int nv, ne, nt;
    int64_t vert[64][3];   /* link vertices, level-local coordinates */
    int edges[96][2];
    int tris[64][3];
} link_t;

static int link_vertex_id(link_t *L, const int64_t q[3])
{
    for (int i = 0; i < L->nv; i++)
        if (L->vert[i][0] == q[0] && L->vert[i][1] == q[1] &&
            L->vert[i][2] == q[2])
            return i;
    L->vert[L->nv][0] = q[0];
    L->vert[L->nv][1] = q[1];
    L->vert[L->nv][2] = q[2];
    return L->nv++;
}

static void link_add_edge(link_t *L, int a, int b)
{
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
    for (int e = 0; e < L->ne; e++)
        if (L->edges[e][0] == a && L->edges[e][1] == b)
            return;
    L->edges[L->ne][0] = a;
    L->edges[L->ne][1] = b;
    L->ne++;
}

static const int PERMS[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

/* Collect the link of level vertex v (level-local coordinates). */
static void build_link(const grid_t *g, const int64_t v[3], link_t *L)
{
    L->nv = L->ne = L->nt = 0;
    if (g->dim == 3) {
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) {
                    int64_t c[3] = {v[0] - dx, v[1] - dy, v[2] - dz};
                    int inside = 1;
                    for (int a = 0; a < 3; a++)
                        if (c[a] < 0 || c[a] + 1 > g->m[a] - 1)
                            inside = 0;
                    if (!inside)
                        continue;
                    for (int p = 0; p < 6; p++) {
                        int64_t q[4][3];
                        for (int a = 0; a < 3; a++)
                            q[0][a] = c[a];
                        for (int k = 1; k < 4; k++) {
                            for (int a = 0; a < 3; a++)
                                q[k][a] = q[k - 1][a];
                            q[k][PERMS[p][k - 1]] += 1;
                        }
                        int at = -1;
                        for (int k = 0; k < 4; k++)
                            if (q[k][0] == v[0] && q[k][1] == v[1] &&
                                q[k][2] == v[2])
                                at = k;
                        if (at < 0)
                            continue;
                        int ids[3], n = 0;
                        for (int k = 0; k < 4; k++)
                            if (k != at)
                                ids[n++] = link_vertex_id(L, q[k]);
                        L->tris[L->nt][0] = ids[0];
                        L->tris[L->nt][1] = ids[1];
                        L->tris[L->nt][2] = ids[2];
                        L->nt++;
                        link_add_edge(L, ids[0], ids[1]);
                        link_add_edge(L, ids[0], ids[2]);
                        link_add_edge(L, ids[1], ids[2]);
                    }
                }
    } else {
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
                int64_t c[3] = {v[0] - dx, v[1] - dy, 0};
                if (c[0] < 0 || c[0] + 1 > g->m[0] - 1 || c[1] < 0 ||
                    c[1] + 1 > g->m[1] - 1)
                    continue;
                /* triangles (c, c+ex, c+ex+ey) and (c, c+ey, c+ex+ey) */
                for (int t = 0; t < 2; t++) {
                    int64_t q[3][3] = {{c[0], c[1], 0},
                                       {c[0] + (t == 0), c[1] + (t == 1), 0},
                                       {c[0] + 1, c[1] + 1, 0}};
                    int at = -1;
                    for (int k = 0; k < 3; k++)
                        if (q[k][0] == v[0] && q[k][1] == v[1])
                            at = k;
                    if (at < 0)
                        continue;
                    int ids[2], n = 0;
                    for (int k = 0; k < 3; k++)
                        if (k != at)
                            ids[n++] = link_vertex_id(L, q[k]);
                    link_add_edge(L, ids[0], ids[1]);
                }
            }
    }
}

static int on_boundary(const grid_t *g, const int64_t v[3])
{
    for (int a = 0; a < g->dim; a++)
        if (v[a] == 0 || v[a] == g->m[a] - 1)
            return 1;
    return 0;
}

typedef struct {
    link_result_t r;
    int boundary, nsc;
    uint8_t code;
    int nv, ne, nt;
} vertex_result_t;

static void classify_vertex(const grid_t *g, const float *f,
                            const int64_t v[3], vertex_result_t *out)
{
    link_t L;
    build_link(g, v, &L);
    float fv = value_at(g, f, v);
    int64_t iv = full_index(g, v);
    int lower[64];
    for (int i = 0; i < L.nv; i++) {
        float fu = value_at(g, f, L.vert[i]);
        int64_t iu = full_index(g, L.vert[i]);
        lower[i] = (fu < fv) || (fu == fv && iu < iv);
    }
    int boundary = on_boundary(g, v);
    classify_link(L.nv, lower, L.ne, (const int(*)[2])L.edges, L.nt,
                  (const int(*)[3])L.tris, g->dim == 3 ? 2 : 1, !boundary,
                  &out->r);
    out->boundary = boundary;
    out->nsc = boundary && (out->r.b1_lower > 0 || out->r.b1_upper > 0);
    out->code = (uint8_t)((out->r.n_lower & 7) | ((out->r.n_upper & 7) << 3) |
                          (boundary << 6) | (out->nsc << 7));
    out->nv = L.nv;
    out->ne = L.ne;
    out->nt = L.nt;
}

/* -------------------------------------------------------------------------
 * Level geometry and the exported grid entry points.
 * ------------------------------------------------------------------------- */

static int make_grid(int64_t nx, int64_t ny, int64_t nz, int level, grid_t *g)
{
    if (nx < 2 || ny < 2 || nz < 1)
        return OR_E_DIMS;
    if (nx > (1LL << 32) || ny > (1LL << 32) || nz > (1LL << 32) ||
        (double)nx * (double)ny * (double)nz > 4294967295.0)
        return OR_E_DIMS;
    g->dim = nz == 1 ? 2 : 3;
    g->n[0] = nx;
    g->n[1] = ny;
    g->n[2] = nz;
    if (level < 0 || level > 40)
        return OR_E_LEVEL;
    g->s = (int64_t)1 << level;
    for (int a = 0; a < 3; a++) {
        if (a == 2 && g->dim == 2) {
            g->m[2] = 1;
            continue;
        }
        if (g->s > g->n[a] - 1)
            return OR_E_LEVEL;
        g->m[a] = (g->n[a] - 1) / g->s + 1;
    }
    return OR_OK;
}

/* Number of samples per axis at a level; returns <0 if the level is invalid. */
int oracle_level_dims(int64_t nx, int64_t ny, int64_t nz, int level,
                      int64_t *m_out)
{
    grid_t g;
    int st = make_grid(nx, ny, nz, level, &g);
    if (st)
        return st;
    m_out[0] = g.m[0];
    m_out[1] = g.m[1];
    m_out[2] = g.m[2];
    return OR_OK;
}

/* Per-vertex detail for a list of level-local vertices (tests).
 * out row (12 ints): code, n_lower, n_upper, chi_lower, chi_upper, b1_lower,
 * b1_upper, boundary, nsc, critical, #link vertices, #link edges + 1000 *
 * #link triangles. */
int oracle_vertex_detail(const float *f, int64_t nx, int64_t ny, int64_t nz,
                         int level, int64_t count, const int64_t *coords,
                         int *out)
{
    grid_t g;
    int st = make_grid(nx, ny, nz, level, &g);
    if (st)
        return st;
    if (!f || !coords || !out || count < 0)
        return OR_E_ARG;
    for (int64_t i = 0; i < count; i++) {
        int64_t v[3] = {coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]};
        for (int a = 0; a < 3; a++)
            if (v[a] < 0 || v[a] >= g.m[a])
                return OR_E_ARG;
        vertex_result_t r;
        classify_vertex(&g, f, v, &r);
        int *o = out + 12 * i;
        o[0] = r.code;
        o[1] = r.r.n_lower;
        o[2] = r.r.n_upper;
        o[3] = r.r.chi_lower;
        o[4] = r.r.chi_upper;
        o[5] = r.r.b1_lower;
        o[6] = r.r.b1_upper;
        o[7] = r.boundary;
        o[8] = r.nsc;
        o[9] = r.r.critical;
        o[10] = r.nv;
        o[11] = r.ne + 1000 * r.nt;
    }
    return OR_OK;
}

typedef struct {
    const grid_t *g;
    const float *f;
    int64_t slow_begin, slow_end; /* range of the slowest level axis */
    uint8_t *codes;               /* full resolution, may be NULL */
    int8_t *chi_lower, *chi_upper;/* level-local, may be NULL */
    uint8_t *critical;            /* level-local scratch */
    int64_t base;                 /* level-local index of the range start */
    int nan_seen;
} work_t;

static void *worker(void *arg)
{
    work_t *w = (work_t *)arg;
    const grid_t *g = w->g;
    int slow = g->dim == 3 ? 2 : 1;
    for (int64_t t = w->slow_begin; t < w->slow_end; t++) {
        int64_t v[3] = {0, 0, 0};
        v[slow] = t;
        int64_t mid_n = g->dim == 3 ? g->m[1] : 1;
        for (int64_t y = 0; y < mid_n; y++) {
            if (g->dim == 3)
                v[1] = y;
            for (int64_t x = 0; x < g->m[0]; x++) {
                v[0] = x;
                int64_t loc = v[0] + g->m[0] * (v[1] + g->m[1] * v[2]);
                if (isnan(value_at(g, w->f, v))) {
                    w->nan_seen = 1;
                    continue;
                }
                vertex_result_t r;
                classify_vertex(g, w->f, v, &r);
                if (w->codes)
                    w->codes[full_index(g, v)] = r.code;
                if (w->chi_lower)
                    w->chi_lower[loc] = (int8_t)r.r.chi_lower;
                if (w->chi_upper)
                    w->chi_upper[loc] = (int8_t)r.r.chi_upper;
                w->critical[loc - w->base] = (uint8_t)r.r.critical;
            }
        }
    }
    return NULL;
}

/*
 * Classify every level-`level` vertex whose slowest level coordinate (z in
 * 3D, y in 2D) lies in [slow_begin, slow_end) (slow_end < 0: to the end).
 *   codes      full-resolution array of nx*ny*nz bytes; only level positions
 *              in the range are written.  May be NULL.
 *   chi_lower, chi_upper  level-local arrays (m_x*m_y*m_z int8), may be NULL.
 *   crit       ascending full-resolution indices of critical vertices.
 *   crit_count receives the number of critical vertices (also when it
 *              exceeds crit_cap, in which case OR_E_CAPACITY is returned and
 *              only the first crit_cap entries are written).
 * Returns OR_E_NAN if a level sample in the range is NaN.
 */
int oracle_classify(const float *f, int64_t nx, int64_t ny, int64_t nz,
                    int level, int64_t slow_begin, int64_t slow_end,
                    uint8_t *codes, int8_t *chi_lower, int8_t *chi_upper,
                    uint32_t *crit, int64_t crit_cap, int64_t *crit_count,
                    int nthreads)
{
    grid_t g;
    int st = make_grid(nx, ny, nz, level, &g);
    if (st)
        return st;
    if (!f || !crit_count || crit_cap < 0 || (crit_cap > 0 && !crit))
        return OR_E_ARG;
    int slow = g.dim == 3 ? 2 : 1;
    if (slow_end < 0 || slow_end > g.m[slow])
        slow_end = g.m[slow];
    if (slow_begin < 0)
        slow_begin = 0;
    if (slow_begin > slow_end)
        return OR_E_ARG;
    int64_t plane = g.m[0] * (g.dim == 3 ? g.m[1] : 1);
    int64_t base = slow_begin * plane;
    int64_t count = (slow_end - slow_begin) * plane;
    uint8_t *critical = (uint8_t *)calloc((size_t)(count > 0 ? count : 1), 1);
    if (!critical)
        return OR_E_OOM;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    int64_t rows = slow_end - slow_begin;
    if (nthreads > rows)
        nthreads = rows > 0 ? (int)rows : 1;
    pthread_t th[256];
    work_t wk[256];
    for (int t = 0; t < nthreads; t++) {
        wk[t].g = &g;
        wk[t].f = f;
        wk[t].slow_begin = slow_begin + rows * t / nthreads;
        wk[t].slow_end = slow_begin + rows * (t + 1) / nthreads;
        wk[t].codes = codes;
        wk[t].chi_lower = chi_lower;
        wk[t].chi_upper = chi_upper;
        wk[t].critical = critical;
        wk[t].base = base;
        wk[t].nan_seen = 0;
    }
    if (nthreads == 1) {
        worker(&wk[0]);
    } else {
        for (int t = 0; t < nthreads; t++)
            pthread_create(&th[t], NULL, worker, &wk[t]);
        for (int t = 0; t < nthreads; t++)
            pthread_join(th[t], NULL);
    }
    int nan_seen = 0;
    for (int t = 0; t < nthreads; t++)
        nan_seen |= wk[t].nan_seen;
    /* level-local lexicographic order is the full-resolution index order
     * restricted to the level, so a scan in level order is ascending */
    int64_t n = 0;
    for (int64_t i = 0; i < count; i++) {
        if (!critical[i])
            continue;
        int64_t loc = base + i;
        int64_t v[3];
        v[0] = loc % g.m[0];
        v[1] = (loc / g.m[0]) % g.m[1];
        v[2] = loc / (g.m[0] * g.m[1]);
        if (n < crit_cap)
            crit[n] = (uint32_t)full_index(&g, v);
        n++;
    }
    free(critical);
    *crit_count = n;
    if (nan_seen)
        return OR_E_NAN;
    return n > crit_cap ? OR_E_CAPACITY : OR_OK;
}
