/*
 * paper_cpu.c -- a plain single-threaded CPU implementation of the paper's
 * algorithm (U. Bauer, "Ripser: efficient computation of Vietoris-Rips
 * persistence barcodes", arXiv:1908.02518), written from the paper as a
 * performance baseline. It is timed beside the GPU library and the oracle;
 * nothing here is used by the GPU library, and it uses nothing of it.
 *
 * What it follows from the paper:
 *   - simplices indexed in the combinatorial number system (section
 *     "Indexing simplices in the combinatorial number system"), ordered by
 *     the lexicographic refinement of the Rips filtration (diameter, then
 *     index, the larger index older: "Lexicographic refinement ...");
 *   - persistent cohomology with clearing: Algorithm 2 around Algorithm 1 on
 *     the coboundary matrices in increasing dimension (sections "Clearing
 *     inessential birth columns", "Persistent Cohomology");
 *   - implicit matrix reduction: coboundary columns are generated on the fly
 *     from the stored reduction matrix V, the working column is a binary
 *     heap with lazy cancellation (sections "Implicit matrix reduction",
 *     "Column and matrix data structures", "Pivot extraction");
 *   - the shortcuts for zero-persistence apparent pairs and emergent pairs
 *     (sections "Apparent pairs", "Emergent persistence pairs", "Shortcuts
 *     for apparent and emergent pairs");
 *   - dimension 0 by union-find over the edges in filtration order (elder
 *     rule), the enclosing-radius threshold ("Input").
 * The conventions (threshold clamp, inclusive diameters, orientation, output
 * order) are the ones the oracle and the GPU library use, so the bars are
 * comparable bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define PC_MAXD 3

typedef struct {
    float diam;
    int64_t idx;
    uint32_t coef;
} entry;

/* ---------------------------------------------------------------- context */

typedef struct {
    int n;
    const float *D; /* lower triangle, (i, j) i > j at i(i-1)/2 + j */
    float t;
    uint32_t p;
    int64_t *B; /* B[j * (n + 1) + i] = C(i, j), j <= PC_MAXD + 2 */
    int *nb_off, *nb_idx; /* neighbours within t, ascending */
    uint32_t *inv;
} ctx;

static float dist(const ctx *c, int a, int b) {
    if (a == b) return 0.0f;
    if (a < b) {
        int s = a;
        a = b;
        b = s;
    }
    return c->D[(int64_t)a * (a - 1) / 2 + b];
}

static int64_t binom(const ctx *c, int i, int j) {
    if (i < 0 || j < 0 || i < j) return 0;
    return c->B[(int64_t)j * (c->n + 1) + i];
}

/* vertices decreasing -> index */
static int64_t index_of(const ctx *c, const int *v, int k) {
    int64_t s = 0;
    for (int m = 0; m <= k; ++m) s += binom(c, v[m], k - m + 1);
    return s;
}

/* index -> vertices decreasing: the largest vertex is the largest i with
   C(i, k+1) <= idx, then the rest recursively */
static void vertices_of(const ctx *c, int64_t idx, int k, int *v) {
    int hi = c->n - 1;
    for (int l = k; l >= 0; --l) {
        int lo = l, top = hi;
        while (lo < top) { /* largest i in [l, hi] with C(i, l+1) <= idx */
            int mid = (lo + top + 1) / 2;
            if (binom(c, mid, l + 1) <= idx) lo = mid;
            else top = mid - 1;
        }
        v[k - l] = lo;
        idx -= binom(c, lo, l + 1);
        hi = lo - 1;
    }
}

static float diameter(const ctx *c, const int *v, int k) {
    float m = 0.0f;
    for (int a = 0; a <= k; ++a)
        for (int b = a + 1; b <= k; ++b) {
            float d = dist(c, v[a], v[b]);
            if (d > m) m = d;
        }
    return m;
}

static int older(float da, int64_t ia, float db, int64_t ib) {
    return da < db || (da == db && ia > ib);
}

/* ------------------------------------------------------- cofacets, facets */

/* Cofacets of sigma (k-simplex, vertices v decreasing, diameter dm) within
   t: the candidates are the neighbours of sigma's vertex with the fewest of
   them. For each: index, diameter and (-1)^(vertices of sigma below j). */
typedef struct {
    int64_t idx;
    float diam;
    int sign; /* 0: +1, 1: -1 */
    int j;    /* the added vertex */
} cof;

static int cofacets(const ctx *c, const int *v, int k, float dm, cof *out) {
    int u = v[0], du = c->nb_off[v[0] + 1] - c->nb_off[v[0]];
    for (int m = 1; m <= k; ++m) {
        int d = c->nb_off[v[m] + 1] - c->nb_off[v[m]];
        if (d < du) {
            du = d;
            u = v[m];
        }
    }
    int cnt = 0;
    const int *L = c->nb_idx + c->nb_off[u];
    for (int q = 0; q < du; ++q) {
        int j = L[q], in = 0;
        float nd = dm;
        for (int m = 0; m <= k && !in; ++m) {
            if (v[m] == j) in = 1;
            else {
                float d = dist(c, v[m], j);
                if (d > nd) nd = d;
            }
        }
        if (in || !(nd <= c->t)) continue;
        /* insert j: vertices above j move up one binomial order */
        int64_t s = 0;
        int below = 0;
        for (int m = 0; m <= k; ++m) {
            if (v[m] > j) s += binom(c, v[m], k - m + 2);
            else {
                s += binom(c, v[m], k - m + 1);
                ++below;
            }
        }
        s += binom(c, j, below + 1);
        out[cnt].idx = s;
        out[cnt].diam = nd;
        out[cnt].sign = below & 1;
        out[cnt].j = j;
        ++cnt;
    }
    return cnt;
}

/* oldest cofacet of sigma with diameter dm (the zero-persistence candidate):
   the one with the largest added vertex; -1 if none */
static int64_t zero_cofacet(const ctx *c, const int *v, int k, float dm, int *jout) {
    int u = v[0], du = c->nb_off[v[0] + 1] - c->nb_off[v[0]];
    for (int m = 1; m <= k; ++m) {
        int d = c->nb_off[v[m] + 1] - c->nb_off[v[m]];
        if (d < du) {
            du = d;
            u = v[m];
        }
    }
    const int *L = c->nb_idx + c->nb_off[u];
    for (int q = du - 1; q >= 0; --q) { /* largest j first: the oldest */
        int j = L[q], ok = 1;
        for (int m = 0; m <= k && ok; ++m) ok = v[m] != j && dist(c, v[m], j) <= dm;
        if (!ok) continue;
        int tv[PC_MAXD + 3], w = 0, placed = 0;
        for (int m = 0; m <= k; ++m) {
            if (!placed && j > v[m]) {
                tv[w++] = j;
                placed = 1;
            }
            tv[w++] = v[m];
        }
        if (!placed) tv[w++] = j;
        *jout = j;
        return index_of(c, tv, k + 1);
    }
    return -1;
}

/* youngest facet of tau (vertices tv decreasing, k+1-simplex) with
   diameter dm: remove the largest vertex possible; returns the position
   removed or -1 */
static int zero_facet(const ctx *c, const int *tv, int k1, float dm) {
    for (int m = 0; m <= k1; ++m) {
        int rv[PC_MAXD + 3], w = 0;
        for (int q = 0; q <= k1; ++q)
            if (q != m) rv[w++] = tv[q];
        if (diameter(c, rv, k1 - 1) == dm) return m;
    }
    return -1;
}

/* (sigma, tau) is a zero-persistence apparent pair: tau is sigma's oldest
   cofacet, of sigma's diameter, and sigma is tau's youngest facet, of the
   same diameter */
static int apparent_cofacet(const ctx *c, const int *v, int k, float dm, int64_t *tau) {
    int j;
    int64_t t = zero_cofacet(c, v, k, dm, &j);
    if (t < 0) return 0;
    int tv[PC_MAXD + 3];
    vertices_of(c, t, k + 1, tv);
    int m = zero_facet(c, tv, k + 1, dm);
    if (m < 0 || tv[m] != j) return 0;
    *tau = t;
    return 1;
}

/* tau (a (k+1)-simplex) has a zero apparent facet rho: returns rho's index
   and the position m removed, or -1 */
static int64_t apparent_facet(const ctx *c, int64_t tau, int k1, float dm, int *mout) {
    int tv[PC_MAXD + 3];
    vertices_of(c, tau, k1, tv);
    int m = zero_facet(c, tv, k1, dm);
    if (m < 0) return -1;
    int rv[PC_MAXD + 3], w = 0;
    for (int q = 0; q <= k1; ++q)
        if (q != m) rv[w++] = tv[q];
    int j;
    int64_t t2 = zero_cofacet(c, rv, k1 - 1, dm, &j);
    if (t2 != tau) return -1;
    *mout = m;
    return index_of(c, rv, k1 - 1);
}

/* ------------------------------------------------------------ hash table */

typedef struct {
    int64_t *keys;
    int64_t *vals;
    uint64_t mask;
} hmap;

static uint64_t mixh(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

static void hmap_init(hmap *h, int64_t n) {
    uint64_t cap = 64;
    while (cap < (uint64_t)(2 * n + 64)) cap <<= 1;
    h->keys = (int64_t *)malloc(cap * 8);
    h->vals = (int64_t *)malloc(cap * 8);
    for (uint64_t i = 0; i < cap; ++i) h->keys[i] = -1;
    h->mask = cap - 1;
}

static void hmap_free(hmap *h) {
    free(h->keys);
    free(h->vals);
}

static int64_t hmap_get(const hmap *h, int64_t key) {
    for (uint64_t s = mixh((uint64_t)key) & h->mask;; s = (s + 1) & h->mask) {
        if (h->keys[s] == key) return h->vals[s];
        if (h->keys[s] == -1) return -1;
    }
}

static void hmap_put(hmap *h, int64_t key, int64_t val) {
    for (uint64_t s = mixh((uint64_t)key) & h->mask;; s = (s + 1) & h->mask) {
        if (h->keys[s] == -1 || h->keys[s] == key) {
            h->keys[s] = key;
            h->vals[s] = val;
            return;
        }
    }
}

/* ---------------------------------------------------------------- heap */

typedef struct {
    entry *a;
    int64_t n, cap;
} heap;

/* the oldest entry on top */
static void heap_push(heap *h, entry e) {
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (entry *)realloc(h->a, h->cap * sizeof(entry));
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (!older(e.diam, e.idx, h->a[par].diam, h->a[par].idx)) break;
        h->a[i] = h->a[par];
        i = par;
    }
    h->a[i] = e;
}

static entry heap_pop(heap *h) {
    entry top = h->a[0], last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        entry be = last;
        if (l < h->n && older(h->a[l].diam, h->a[l].idx, be.diam, be.idx)) {
            b = l;
            be = h->a[l];
        }
        if (r < h->n && older(h->a[r].diam, h->a[r].idx, be.diam, be.idx)) b = r;
        if (b == i) break;
        h->a[i] = h->a[b];
        i = b;
    }
    if (h->n) h->a[i] = last;
    return top;
}

/* pivot with lazy cancellation: pop equal indices, sum, drop zeros; the
   pivot (nonzero sum) is pushed back and returned; coef 0 = empty */
static entry heap_pivot(heap *h, uint32_t p) {
    while (h->n) {
        entry e = heap_pop(h);
        uint32_t s = e.coef % p;
        while (h->n && h->a[0].idx == e.idx) s = (s + heap_pop(h).coef) % p;
        if (s != 0) {
            e.coef = s;
            heap_push(h, e);
            return e;
        }
    }
    entry none = {0.0f, -1, 0};
    return none;
}

/* ---------------------------------------------------------------- result */

typedef struct {
    float birth, death;
    int64_t bs, ds;
} bar;

typedef struct {
    bar *b;
    int64_t n, cap;
} barlist;

static void bar_push(barlist *L, float b, float d, int64_t bs, int64_t ds) {
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->b = (bar *)realloc(L->b, L->cap * sizeof(bar));
    }
    L->b[L->n].birth = b;
    L->b[L->n].death = d;
    L->b[L->n].bs = bs;
    L->b[L->n].ds = ds;
    L->n++;
}

static int cmp_bar(const void *x, const void *y) {
    const bar *a = (const bar *)x, *b = (const bar *)y;
    if (a->birth != b->birth) return a->birth < b->birth ? -1 : 1;
    return (a->bs < b->bs) - (a->bs > b->bs); /* birth simplex index descending */
}

typedef struct {
    int max_dim;
    float t_eff;
    barlist bars[PC_MAXD + 1];
    int64_t columns[PC_MAXD + 1], additions[PC_MAXD + 1];
} pc_result;

/* ---------------------------------------------------------------- simplex lists */

typedef struct {
    int64_t *idx;
    float *diam;
    int64_t n, cap;
} slist;

static void sl_push(slist *s, int64_t idx, float dm) {
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 4096;
        s->idx = (int64_t *)realloc(s->idx, s->cap * 8);
        s->diam = (float *)realloc(s->diam, s->cap * 4);
    }
    s->idx[s->n] = idx;
    s->diam[s->n] = dm;
    s->n++;
}

/* reverse filtration order of the columns: diameter descending, index
   ascending */
static const slist *g_sort_list;
static int cmp_rev(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    float da = g_sort_list->diam[a], db = g_sort_list->diam[b];
    if (da != db) return da > db ? -1 : 1;
    int64_t ia = g_sort_list->idx[a], ib = g_sort_list->idx[b];
    return (ia > ib) - (ia < ib);
}

/* ---------------------------------------------------------------- dimension 0 */

static int uf_find(int *par, int x) {
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

typedef struct {
    float d;
    int64_t idx;
    int a, b;
} edge;

static int cmp_edge(const void *x, const void *y) {
    const edge *a = (const edge *)x, *b = (const edge *)y;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    return (a->idx < b->idx) - (a->idx > b->idx); /* larger index older */
}

/* ---------------------------------------------------------------- main routine */

pc_result *pc_run(const float *D, int32_t n, int32_t max_dim, float threshold, uint32_t p) {
    if (n < 1 || max_dim < 0 || max_dim > PC_MAXD || p < 2) return NULL;
    pc_result *res = (pc_result *)calloc(1, sizeof(pc_result));
    res->max_dim = max_dim;
    ctx c;
    c.n = n;
    c.D = D;
    c.p = p;
    /* threshold clamped to the enclosing radius */
    float renc = INFINITY;
    for (int i = 0; i < n; ++i) {
        float m = 0.0f;
        for (int j = 0; j < n; ++j) {
            float d = dist(&c, i, j);
            if (d > m) m = d;
        }
        if (m < renc) renc = m;
    }
    if (n == 1) renc = 0.0f;
    c.t = threshold < renc ? threshold : renc;
    res->t_eff = c.t;
    c.B = (int64_t *)calloc((size_t)(PC_MAXD + 3) * (n + 1), 8);
    for (int i = 0; i <= n; ++i) {
        c.B[i] = 1;
        for (int j = 1; j <= PC_MAXD + 2; ++j)
            c.B[(int64_t)j * (n + 1) + i] =
                i == 0 ? 0 : c.B[(int64_t)j * (n + 1) + i - 1] + c.B[(int64_t)(j - 1) * (n + 1) + i - 1];
    }
    c.inv = (uint32_t *)malloc(p * 4);
    for (uint32_t a = 1; a < p; ++a) {
        uint64_t r = 1, b = a, e = p - 2;
        while (e) {
            if (e & 1) r = r * b % p;
            b = b * b % p;
            e >>= 1;
        }
        c.inv[a] = (uint32_t)r;
    }
    /* neighbour lists within t */
    c.nb_off = (int *)calloc(n + 1, sizeof(int));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (j != i && dist(&c, i, j) <= c.t) c.nb_off[i + 1]++;
    for (int i = 0; i < n; ++i) c.nb_off[i + 1] += c.nb_off[i];
    c.nb_idx = (int *)malloc(sizeof(int) * (c.nb_off[n] + 1));
    for (int i = 0, w = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (j != i && dist(&c, i, j) <= c.t) c.nb_idx[w++] = j;

    /* ---- dimension 0: union-find over the edges in filtration order */
    slist lo;
    memset(&lo, 0, sizeof(lo));
    int64_t ne = 0;
    edge *E = (edge *)malloc(sizeof(edge) * ((int64_t)c.nb_off[n] / 2 + 1));
    for (int a = 1; a < n; ++a)
        for (int b = 0; b < a; ++b) {
            float d = dist(&c, a, b);
            if (d <= c.t) {
                E[ne].d = d;
                E[ne].idx = (int64_t)a * (a - 1) / 2 + b;
                E[ne].a = a;
                E[ne].b = b;
                ++ne;
            }
        }
    qsort(E, ne, sizeof(edge), cmp_edge);
    int *par = (int *)malloc(sizeof(int) * n);
    int *oldest = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) {
        par[i] = i;
        oldest[i] = i;
    }
    hmap prev; /* pivots of the previous dimension (cleared columns) */
    hmap_init(&prev, ne + n);
    for (int64_t e = 0; e < ne; ++e) {
        int ra = uf_find(par, E[e].a), rb = uf_find(par, E[e].b);
        if (ra == rb) continue;
        /* elder rule: the component whose oldest vertex is younger dies;
           vertices all have diameter 0, the larger index is older */
        int oa = oldest[ra], ob = oldest[rb];
        int young = oa < ob ? oa : ob;
        if (E[e].d > 0.0f) bar_push(&res->bars[0], 0.0f, E[e].d, young, E[e].idx);
        par[ra] = rb;
        oldest[rb] = oa > ob ? oa : ob;
        hmap_put(&prev, E[e].idx, 0);
    }
    for (int i = 0; i < n; ++i)
        if (uf_find(par, i) == i) bar_push(&res->bars[0], 0.0f, INFINITY, oldest[i], -1);
    for (int64_t e = 0; e < ne; ++e) sl_push(&lo, E[e].idx, E[e].d);
    free(E);
    free(par);
    free(oldest);

    /* ---- dimensions 1 .. max_dim: cohomology with clearing */
    cof *cbuf = (cof *)malloc(sizeof(cof) * (n + 1));
    heap W;
    memset(&W, 0, sizeof(W));
    for (int k = 1; k <= max_dim; ++k) {
        /* the k-simplices: lo holds them for k = 1; else expand the
           (k-1)-simplices by cofacets above their top vertex */
        slist cur;
        memset(&cur, 0, sizeof(cur));
        if (k == 1) {
            cur = lo;
            memset(&lo, 0, sizeof(lo));
        } else {
            for (int64_t q = 0; q < lo.n; ++q) {
                int v[PC_MAXD + 3];
                vertices_of(&c, lo.idx[q], k - 1, v);
                int cnt = cofacets(&c, v, k - 1, lo.diam[q], cbuf);
                for (int r = 0; r < cnt; ++r)
                    if (cbuf[r].j > v[0]) sl_push(&cur, cbuf[r].idx, cbuf[r].diam);
            }
            free(lo.idx);
            free(lo.diam);
        }
        /* columns: not cleared, not in a zero apparent pair (sigma, tau) and
           not the tau of one of the previous dimension (those are pivots
           there too) */
        int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (cur.n + 1));
        int64_t nc = 0;
        hmap app; /* zero apparent pairs (sigma, tau) of this dimension: tau -> sigma */
        hmap_init(&app, cur.n);
        for (int64_t q = 0; q < cur.n; ++q) {
            if (hmap_get(&prev, cur.idx[q]) >= 0) continue;
            int v[PC_MAXD + 3];
            vertices_of(&c, cur.idx[q], k, v);
            int64_t tau;
            if (apparent_cofacet(&c, v, k, cur.diam[q], &tau)) {
                hmap_put(&app, tau, cur.idx[q]);
                continue;
            }
            ord[nc++] = q;
        }
        g_sort_list = &cur;
        qsort(ord, nc, sizeof(int64_t), cmp_rev);
        res->columns[k] = nc;
        hmap piv; /* pivot -> column */
        hmap_init(&piv, nc);
        /* V columns of the paired columns: (index, coefficient) lists */
        int64_t **vidx = (int64_t **)calloc(nc + 1, sizeof(int64_t *));
        uint32_t **vcoef = (uint32_t **)calloc(nc + 1, sizeof(uint32_t *));
        int64_t *vlen = (int64_t *)calloc(nc + 1, sizeof(int64_t));
        uint32_t *pivc = (uint32_t *)calloc(nc + 1, sizeof(uint32_t));
        int64_t *vi = NULL;
        uint32_t *vc = NULL;
        int64_t vn = 0, vcap = 0;
        for (int64_t col = 0; col < nc; ++col) {
            const int64_t sidx = cur.idx[ord[col]];
            const float sdm = cur.diam[ord[col]];
            int v[PC_MAXD + 3];
            vertices_of(&c, sidx, k, v);
            /* emergent shortcut: the oldest cofacet of sigma's diameter,
               free (not a pivot, no zero apparent facet), pairs at once */
            {
                int j;
                int64_t tau = zero_cofacet(&c, v, k, sdm, &j);
                int mm;
                if (tau >= 0 && hmap_get(&piv, tau) < 0 && apparent_facet(&c, tau, k + 1, sdm, &mm) < 0) {
                    hmap_put(&piv, tau, col);
                    vidx[col] = (int64_t *)malloc(8);
                    vcoef[col] = (uint32_t *)malloc(4);
                    vidx[col][0] = sidx;
                    vcoef[col][0] = 1;
                    vlen[col] = 1;
                    /* coefficient of tau in the coboundary of sigma */
                    int below = 0;
                    for (int m = 0; m <= k; ++m) below += v[m] < j;
                    pivc[col] = (below & 1) ? p - 1 : 1;
                    continue;
                }
            }
            /* the working column: the coboundary of sigma, then additions */
            W.n = 0;
            vn = 0;
            {
                int cnt = cofacets(&c, v, k, sdm, cbuf);
                for (int r = 0; r < cnt; ++r) {
                    entry e = {cbuf[r].diam, cbuf[r].idx, cbuf[r].sign ? p - 1 : 1};
                    heap_push(&W, e);
                }
            }
            if (vn == vcap) {
                vcap = vcap ? 2 * vcap : 64;
                vi = (int64_t *)realloc(vi, vcap * 8);
                vc = (uint32_t *)realloc(vc, vcap * 4);
            }
            vi[vn] = sidx;
            vc[vn++] = 1;
            for (;;) {
                entry pv = heap_pivot(&W, p);
                if (pv.coef == 0) { /* zero column: essential class */
                    bar_push(&res->bars[k], sdm, INFINITY, sidx, -1);
                    break;
                }
                int64_t o = hmap_get(&piv, pv.idx);
                int mm = -1;
                int64_t rho = o < 0 ? apparent_facet(&c, pv.idx, k + 1, pv.diam, &mm) : -1;
                if (o < 0 && rho < 0) { /* pair */
                    if (pv.diam > sdm) bar_push(&res->bars[k], sdm, pv.diam, sidx, pv.idx);
                    hmap_put(&piv, pv.idx, col);
                    pivc[col] = pv.coef;
                    vidx[col] = (int64_t *)malloc(sizeof(int64_t) * vn);
                    vcoef[col] = (uint32_t *)malloc(sizeof(uint32_t) * vn);
                    memcpy(vidx[col], vi, sizeof(int64_t) * vn);
                    memcpy(vcoef[col], vc, sizeof(uint32_t) * vn);
                    vlen[col] = vn;
                    break;
                }
                /* W -= lambda (coboundary of V_o) or lambda (coboundary of rho),
                   lambda = pivot(W) / pivot of the added column */
                res->additions[k]++;
                int64_t an;
                const int64_t *ai;
                const uint32_t *ac;
                int64_t one_i;
                uint32_t one_c = 1, pc;
                if (o >= 0) {
                    an = vlen[o];
                    ai = vidx[o];
                    ac = vcoef[o];
                    pc = pivc[o];
                } else {
                    one_i = rho;
                    an = 1;
                    ai = &one_i;
                    ac = &one_c;
                    /* tau = rho u {tau[m]}: vertices of rho below tau[m] = k + 1 - m */
                    pc = ((k + 1 - mm) & 1) ? p - 1 : 1;
                }
                uint32_t lam = (uint32_t)((uint64_t)pv.coef * c.inv[pc] % p);
                uint32_t neg = (p - lam) % p;
                for (int64_t q = 0; q < an; ++q) {
                    uint32_t f = (uint32_t)((uint64_t)neg * ac[q] % p);
                    if (vn == vcap) {
                        vcap = vcap ? 2 * vcap : 64;
                        vi = (int64_t *)realloc(vi, vcap * 8);
                        vc = (uint32_t *)realloc(vc, vcap * 4);
                    }
                    vi[vn] = ai[q];
                    vc[vn++] = f;
                    int sv[PC_MAXD + 3];
                    vertices_of(&c, ai[q], k, sv);
                    float sd = diameter(&c, sv, k);
                    int cnt = cofacets(&c, sv, k, sd, cbuf);
                    for (int r = 0; r < cnt; ++r) {
                        entry e = {cbuf[r].diam, cbuf[r].idx,
                                   (uint32_t)(cbuf[r].sign ? (uint64_t)f * (p - 1) % p : f)};
                        if (e.coef) heap_push(&W, e);
                    }
                }
            }
        }
        /* the pivots of this dimension clear columns of the next */
        hmap_free(&prev);
        hmap_init(&prev, nc + app.mask);
        for (uint64_t s = 0; s <= piv.mask; ++s)
            if (piv.keys[s] >= 0) hmap_put(&prev, piv.keys[s], 0);
        for (uint64_t s = 0; s <= app.mask; ++s)
            if (app.keys[s] >= 0) hmap_put(&prev, app.keys[s], 0);
        for (int64_t q = 0; q < nc; ++q) {
            free(vidx[q]);
            free(vcoef[q]);
        }
        free(vidx);
        free(vcoef);
        free(vlen);
        free(pivc);
        free(vi);
        free(vc);
        hmap_free(&piv);
        hmap_free(&app);
        free(ord);
        lo = cur;
    }
    free(lo.idx);
    free(lo.diam);
    free(W.a);
    free(cbuf);
    hmap_free(&prev);
    for (int k = 0; k <= max_dim; ++k) qsort(res->bars[k].b, res->bars[k].n, sizeof(bar), cmp_bar);
    free(c.B);
    free(c.inv);
    free(c.nb_off);
    free(c.nb_idx);
    return res;
}

void pc_free(pc_result *r) {
    if (!r) return;
    for (int k = 0; k <= PC_MAXD; ++k) free(r->bars[k].b);
    free(r);
}

float pc_threshold(const pc_result *r) { return r->t_eff; }
int64_t pc_num_bars(const pc_result *r, int k) { return r->bars[k].n; }
int64_t pc_num_columns(const pc_result *r, int k) { return r->columns[k]; }
int64_t pc_num_additions(const pc_result *r, int k) { return r->additions[k]; }

void pc_get_bars(const pc_result *r, int k, float *b, float *d, int64_t *bs, int64_t *ds) {
    for (int64_t i = 0; i < r->bars[k].n; ++i) {
        b[i] = r->bars[k].b[i].birth;
        d[i] = r->bars[k].b[i].death;
        bs[i] = r->bars[k].b[i].bs;
        ds[i] = r->bars[k].b[i].ds;
    }
}
