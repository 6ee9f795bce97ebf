/*
 * rips_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, explicit CPU computation of Vietoris-Rips persistence over
 * the prime field Z/p, written from U. Bauer, "Ripser: efficient computation
 * of Vietoris-Rips persistence barcodes" (arXiv:1908.02518). Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it. It shares
 * no code, header, table or helper with the GPU library, and never calls it.
 *
 * What is computed, with no shortcut of the paper's implementation section:
 *   1. distances d(x_i, x_j) in float32, sum over coordinates in increasing
 *      order, every product and sum rounded (built with -ffp-contract=off),
 *      then a correctly rounded square root ("Input" paragraph; values are
 *      32-bit floats);
 *   2. the threshold t_eff = min(t, r_enc), r_enc = min_x max_y d(x, y), the
 *      enclosing radius above which the complex is a cone ("Input"), with
 *      diam <= t_eff inclusive (definition of Rips_t);
 *   3. explicit lists K_k of all k-simplices of diameter <= t_eff for
 *      k = 0 .. max_dim+1, each indexed in the combinatorial number system
 *      (section "Indexing simplices in the combinatorial number system");
 *   4. the lexicographically refined order: diameter, then dimension, then
 *      reverse colexicographic order, i.e. within a dimension (diam asc,
 *      CNS index desc) (section "Lexicographic refinement");
 *   5. explicit coboundary matrices delta_k = (boundary_{k+1})^T with rows
 *      and columns in reverse filtration order (section "Persistent
 *      cohomology"), standard orientation: the entry of sigma in the
 *      coboundary of sigma u {j} is (-1)^(number of vertices of sigma below j);
 *   6. Algorithm 2 (reduction with clearing) applied to delta_k for
 *      k = 0, 1, ..., max_dim, each step running Algorithm 1 (column
 *      reduction) on explicit sorted sparse columns;
 *   7. bars [diam sigma, diam tau) for pairs with diam tau > diam sigma, and
 *      [diam sigma, +inf) for essential sigma (Proposition on simplexwise
 *      refinements).
 * Besides, from the definition of apparent pairs (youngest facet / oldest
 * cofacet) it reports which simplices lie in a zero-persistence apparent
 * pair, and the set of columns left after clearing and after removing those
 * simplices; and, for small inputs, the homology pairs from Algorithm 1 on
 * the explicit boundary matrices (the duality cross-check).
 *
 * Readings where the paper is loose (each also listed in the design notes):
 *  - the pivot of a column is the lowest nonzero entry, i.e. the largest row
 *    position; a zero column has no pivot (sentinel -1, not 0);
 *  - the threshold is always clamped to the enclosing radius (bars with
 *    nonzero persistence are unchanged by this);
 *  - H0 birth simplices follow from the reduction of delta_0 itself;
 *  - bars of one dimension are listed by birth ascending, then birth simplex
 *    CNS index descending (the refined order of the birth simplex).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 8 /* largest max_dim accepted */

typedef struct {
    int64_t count;
    int32_t k;      /* dimension */
    int32_t *verts; /* count x (k+1), each row strictly decreasing */
    int64_t *idx;   /* CNS index */
    float *diam;
} slist;

typedef struct {
    int64_t len, cap;
    int64_t *row;
    uint32_t *val;
} scol;

typedef struct {
    int32_t n, max_dim;
    uint32_t p;
    float r_enc, t_eff;
    int64_t count[OR_MAXD + 2];
    /* bars per dimension, canonical order */
    int64_t nbars[OR_MAXD + 1];
    float *birth[OR_MAXD + 1], *death[OR_MAXD + 1];
    int64_t *bsimp[OR_MAXD + 1], *dsimp[OR_MAXD + 1];
    /* columns that remain after clearing and after dropping simplices in a
       zero-persistence apparent pair; listed in reduction order */
    int64_t ncols[OR_MAXD + 1];
    int64_t *col_idx[OR_MAXD + 1];
    float *col_diam[OR_MAXD + 1];
    /* counters */
    int64_t npairs[OR_MAXD + 1];        /* all pairs (k, k+1), zero persistence included */
    int64_t nessential[OR_MAXD + 1];
    int64_t ncleared[OR_MAXD + 1];      /* k-simplices that were pivots in dimension k-1 */
    int64_t nreduced_cols[OR_MAXD + 1]; /* columns fed to Algorithm 1 in dimension k */
    int64_t nzero_app_col[OR_MAXD + 1]; /* sigma in a zero apparent pair (sigma, tau) */
    int64_t nzero_app_piv[OR_MAXD + 1]; /* sigma in a zero apparent pair (rho, sigma) */
    /* all pairs (k, k+1) as CNS indices (for cross-checks), reduction order */
    int64_t *pair_lo[OR_MAXD + 1], *pair_hi[OR_MAXD + 1];
    int64_t *ess[OR_MAXD + 1];
    /* all apparent pairs (k, k+1), any persistence, from the definition */
    int64_t napp[OR_MAXD + 1];
    int64_t *app_lo[OR_MAXD + 1], *app_hi[OR_MAXD + 1];
    /* homology cross-check results (only when requested) */
    int32_t have_hom;
    int64_t hom_npairs[OR_MAXD + 1], hom_ness[OR_MAXD + 1];
    int64_t *hom_lo[OR_MAXD + 1], *hom_hi[OR_MAXD + 1], *hom_ess[OR_MAXD + 1];
    char err[256];
} oracle_result;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) abort();
    return p;
}

static void *xrealloc(void *q, size_t n) {
    void *p = realloc(q, n ? n : 1);
    if (!p) abort();
    return p;
}

/* C(a, b) for a, b >= 0 by the multiplicative formula; 0 when b > a. */
static int64_t choose(int64_t a, int64_t b) {
    if (b < 0 || a < b) return 0;
    if (b > a - b) b = a - b;
    __int128 r = 1;
    for (int64_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return (int64_t)r;
}

/* CNS index of a simplex with vertices v[0] > v[1] > ... > v[k]:
   sum over l of C(i_l, l+1) where i_l is the l-th smallest vertex. */
static int64_t cns_index(const int32_t *v, int k, const int64_t *tab, int64_t tabw) {
    int64_t s = 0;
    for (int m = 0; m <= k; ++m) {
        int l = k - m; /* v[m] is i_l */
        s += tab[(int64_t)(l + 1) * tabw + v[m]];
    }
    return s;
}

static uint32_t pow_mod(uint32_t a, uint32_t e, uint32_t p) {
    uint64_t r = 1 % p, b = a % p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return (uint32_t)r;
}

static int is_prime(uint32_t p) {
    if (p < 2) return 0;
    for (uint32_t q = 2; (uint64_t)q * q <= p; ++q)
        if (p % q == 0) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* distances                                                           */
/* ------------------------------------------------------------------ */

/* Lower triangle, row-major: entry (i, j), i > j, at i*(i-1)/2 + j. */
void oracle_distances(const float *x, int64_t n, int64_t m, float *out_lower) {
    for (int64_t i = 1; i < n; ++i) {
        for (int64_t j = 0; j < i; ++j) {
            float s = 0.0f;
            for (int64_t c = 0; c < m; ++c) {
                float t = x[i * m + c] - x[j * m + c];
                float sq = t * t;
                s = s + sq;
            }
            out_lower[i * (i - 1) / 2 + j] = sqrtf(s);
        }
    }
}

/* ------------------------------------------------------------------ */
/* simplex lists                                                       */
/* ------------------------------------------------------------------ */

static void slist_free(slist *s) {
    free(s->verts);
    free(s->idx);
    free(s->diam);
    memset(s, 0, sizeof(*s));
}

typedef struct {
    float diam;
    int64_t idx;
    int64_t orig;
} sortrec;

/* refined order inside one dimension: diameter ascending, then CNS index
   descending (reverse colexicographic) */
static int cmp_refined(const void *a, const void *b) {
    const sortrec *x = (const sortrec *)a, *y = (const sortrec *)b;
    if (x->diam < y->diam) return -1;
    if (x->diam > y->diam) return 1;
    if (x->idx > y->idx) return -1;
    if (x->idx < y->idx) return 1;
    return 0;
}

static void slist_sort_refined(slist *s) {
    int64_t c = s->count;
    int w = s->k + 1;
    sortrec *r = (sortrec *)xmalloc(sizeof(sortrec) * c);
    for (int64_t i = 0; i < c; ++i) {
        r[i].diam = s->diam[i];
        r[i].idx = s->idx[i];
        r[i].orig = i;
    }
    qsort(r, c, sizeof(sortrec), cmp_refined);
    int32_t *nv = (int32_t *)xmalloc(sizeof(int32_t) * c * w);
    int64_t *ni = (int64_t *)xmalloc(sizeof(int64_t) * c);
    float *nd = (float *)xmalloc(sizeof(float) * c);
    for (int64_t i = 0; i < c; ++i) {
        memcpy(nv + i * w, s->verts + r[i].orig * w, sizeof(int32_t) * w);
        ni[i] = r[i].idx;
        nd[i] = r[i].diam;
    }
    free(r);
    free(s->verts);
    free(s->idx);
    free(s->diam);
    s->verts = nv;
    s->idx = ni;
    s->diam = nd;
}

/* index lookup: CNS index -> refined position, via a copy sorted by index */
typedef struct {
    int64_t count;
    int64_t *idx; /* ascending */
    int64_t *pos;
} lookup;

typedef struct {
    int64_t idx, pos;
} idxpos;

static int cmp_idxpos(const void *a, const void *b) {
    const idxpos *x = (const idxpos *)a, *y = (const idxpos *)b;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static void lookup_build(lookup *L, const slist *s) {
    idxpos *t = (idxpos *)xmalloc(sizeof(idxpos) * s->count);
    for (int64_t i = 0; i < s->count; ++i) {
        t[i].idx = s->idx[i];
        t[i].pos = i;
    }
    qsort(t, s->count, sizeof(idxpos), cmp_idxpos);
    L->count = s->count;
    L->idx = (int64_t *)xmalloc(sizeof(int64_t) * s->count);
    L->pos = (int64_t *)xmalloc(sizeof(int64_t) * s->count);
    for (int64_t i = 0; i < s->count; ++i) {
        L->idx[i] = t[i].idx;
        L->pos[i] = t[i].pos;
    }
    free(t);
}

static int64_t lookup_find(const lookup *L, int64_t idx) {
    int64_t lo = 0, hi = L->count - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (L->idx[mid] == idx) return L->pos[mid];
        if (L->idx[mid] < idx) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static void lookup_free(lookup *L) {
    free(L->idx);
    free(L->pos);
    memset(L, 0, sizeof(*L));
}

/* ------------------------------------------------------------------ */
/* sparse columns over Z/p                                             */
/* ------------------------------------------------------------------ */

static void scol_push(scol *c, int64_t row, uint32_t v) {
    if (c->len == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 4;
        c->row = (int64_t *)xrealloc(c->row, sizeof(int64_t) * c->cap);
        c->val = (uint32_t *)xrealloc(c->val, sizeof(uint32_t) * c->cap);
    }
    c->row[c->len] = row;
    c->val[c->len] = v;
    c->len++;
}

static void scol_free(scol *c) {
    free(c->row);
    free(c->val);
    memset(c, 0, sizeof(*c));
}

/* insertion-free sort of a column by row ascending (rows are distinct) */
typedef struct {
    int64_t row;
    uint32_t val;
} rv;

static int cmp_rv(const void *a, const void *b) {
    const rv *x = (const rv *)a, *y = (const rv *)b;
    return (x->row > y->row) - (x->row < y->row);
}

static void scol_sort(scol *c) {
    rv *t = (rv *)xmalloc(sizeof(rv) * c->len);
    for (int64_t i = 0; i < c->len; ++i) {
        t[i].row = c->row[i];
        t[i].val = c->val[i];
    }
    qsort(t, c->len, sizeof(rv), cmp_rv);
    for (int64_t i = 0; i < c->len; ++i) {
        c->row[i] = t[i].row;
        c->val[i] = t[i].val;
    }
    free(t);
}

/* a := a - lambda * b  (mod p); both sorted by row ascending */
static void scol_axpy(scol *a, uint32_t lambda, const scol *b, uint32_t p) {
    scol r = {0, 0, NULL, NULL};
    int64_t i = 0, j = 0;
    uint32_t neg = (p - lambda % p) % p; /* -lambda mod p */
    while (i < a->len || j < b->len) {
        if (j >= b->len || (i < a->len && a->row[i] < b->row[j])) {
            scol_push(&r, a->row[i], a->val[i]);
            ++i;
        } else if (i >= a->len || b->row[j] < a->row[i]) {
            uint32_t v = (uint32_t)((uint64_t)neg * b->val[j] % p);
            if (v) scol_push(&r, b->row[j], v);
            ++j;
        } else {
            uint32_t v = (uint32_t)((a->val[i] + (uint64_t)neg * b->val[j]) % p);
            if (v) scol_push(&r, a->row[i], v);
            ++i;
            ++j;
        }
    }
    scol_free(a);
    *a = r;
}

/* ------------------------------------------------------------------ */
/* the computation                                                     */
/* ------------------------------------------------------------------ */

static float dist_of(const float *D, int64_t n, int32_t a, int32_t b) {
    (void)n;
    if (a == b) return 0.0f;
    if (a < b) {
        int32_t t = a;
        a = b;
        b = t;
    }
    return D[(int64_t)a * (a - 1) / 2 + b];
}

/* all (k+1)-simplices of diameter <= t from the k-simplices, each exactly
   once: append a vertex j above the current largest vertex */
static void expand(const slist *s, slist *out, const float *D, int64_t n, float t,
                   const int64_t *tab, int64_t tabw) {
    int k = s->k, w = k + 2;
    int64_t cap = 16, c = 0;
    out->k = k + 1;
    out->verts = (int32_t *)xmalloc(sizeof(int32_t) * cap * w);
    out->idx = (int64_t *)xmalloc(sizeof(int64_t) * cap);
    out->diam = (float *)xmalloc(sizeof(float) * cap);
    int32_t v[OR_MAXD + 3];
    for (int64_t i = 0; i < s->count; ++i) {
        const int32_t *sv = s->verts + i * (k + 1);
        for (int32_t j = sv[0] + 1; j < n; ++j) {
            float dm = s->diam[i];
            int ok = 1;
            for (int m = 0; m <= k; ++m) {
                float d = dist_of(D, n, j, sv[m]);
                if (!(d <= t)) {
                    ok = 0;
                    break;
                }
                if (d > dm) dm = d;
            }
            if (!ok) continue;
            if (c == cap) {
                cap *= 2;
                out->verts = (int32_t *)xrealloc(out->verts, sizeof(int32_t) * cap * w);
                out->idx = (int64_t *)xrealloc(out->idx, sizeof(int64_t) * cap);
                out->diam = (float *)xrealloc(out->diam, sizeof(float) * cap);
            }
            v[0] = j;
            for (int m = 0; m <= k; ++m) v[m + 1] = sv[m];
            memcpy(out->verts + c * w, v, sizeof(int32_t) * w);
            out->idx[c] = cns_index(v, k + 1, tab, tabw);
            out->diam[c] = dm;
            ++c;
        }
    }
    out->count = c;
}

/* Explicit coboundary matrix of K_k -> K_{k+1}: column c holds the
   cofacets of the k-simplex at reversed position c (c = |K_k|-1-pos), rows
   are reversed positions in K_{k+1}; entries sorted by row. */
static scol *build_coboundary(const slist *lo, const slist *hi, const lookup *Llo, uint32_t p,
                              const int64_t *tab, int64_t tabw) {
    int64_t nc = lo->count, nr = hi->count;
    int k = lo->k;
    scol *cols = (scol *)calloc(nc ? nc : 1, sizeof(scol));
    int32_t f[OR_MAXD + 3];
    for (int64_t r = 0; r < nr; ++r) {
        int64_t pos_tau = r;
        int64_t row = nr - 1 - pos_tau;
        const int32_t *tv = hi->verts + r * (k + 2);
        for (int m = 0; m <= k + 1; ++m) {
            /* facet tau \ {tv[m]}; tv[m] has (k+1-m) facet vertices below it */
            int q = 0;
            for (int u = 0; u <= k + 1; ++u)
                if (u != m) f[q++] = tv[u];
            int64_t fidx = cns_index(f, k, tab, tabw);
            int64_t fpos = lookup_find(Llo, fidx);
            if (fpos < 0) abort(); /* a complex is closed under faces */
            int64_t col = nc - 1 - fpos;
            uint32_t coeff = ((k + 1 - m) % 2 == 0) ? 1u % p : (p - 1) % p;
            scol_push(&cols[col], row, coeff);
        }
    }
    for (int64_t c = 0; c < nc; ++c) scol_sort(&cols[c]);
    return cols;
}

typedef struct {
    float diam;
    int64_t bidx, didx;
    float death;
} barrec;

static int cmp_bar(const void *a, const void *b) {
    const barrec *x = (const barrec *)a, *y = (const barrec *)b;
    if (x->diam < y->diam) return -1;
    if (x->diam > y->diam) return 1;
    return (x->bidx < y->bidx) - (x->bidx > y->bidx);
}

/* Algorithm 1 on explicit columns (in place). owner[row] receives the
   column whose reduced pivot is that row. skip[c] = 1 removes column c
   (clearing). */
static void reduce_columns(scol *cols, int64_t nc, int64_t nr, const uint8_t *skip, uint32_t p,
                           int64_t *owner) {
    for (int64_t r = 0; r < nr; ++r) owner[r] = -1;
    for (int64_t j = 0; j < nc; ++j) {
        if (skip && skip[j]) {
            scol_free(&cols[j]);
            continue;
        }
        scol *R = &cols[j];
        while (R->len > 0) {
            int64_t piv = R->row[R->len - 1];
            int64_t o = owner[piv];
            if (o < 0) break;
            const scol *Ro = &cols[o];
            uint32_t inv = pow_mod(Ro->val[Ro->len - 1], p - 2, p);
            uint32_t lambda = (uint32_t)((uint64_t)R->val[R->len - 1] * inv % p);
            scol_axpy(R, lambda, Ro, p);
        }
        if (R->len > 0) owner[R->row[R->len - 1]] = j;
    }
}

static void result_set_err(oracle_result *res, const char *m) {
    strncpy(res->err, m, sizeof(res->err) - 1);
}

void oracle_free(oracle_result *r) {
    if (!r) return;
    for (int k = 0; k <= OR_MAXD; ++k) {
        free(r->birth[k]);
        free(r->death[k]);
        free(r->bsimp[k]);
        free(r->dsimp[k]);
        free(r->col_idx[k]);
        free(r->col_diam[k]);
        free(r->pair_lo[k]);
        free(r->pair_hi[k]);
        free(r->ess[k]);
        free(r->app_lo[k]);
        free(r->app_hi[k]);
        free(r->hom_lo[k]);
        free(r->hom_hi[k]);
        free(r->hom_ess[k]);
    }
    free(r);
}

/*
 * Main entry. D: lower triangle of the distance matrix (see
 * oracle_distances). threshold: +inf for none. clamp: 1 clamps to the
 * enclosing radius (the normal mode); 0 keeps the given threshold (used by
 * tests that need the full complex). homology: 1 also runs the homology
 * cross-check (small inputs only).
 */
oracle_result *oracle_run(const float *D, int32_t n, int32_t max_dim, float threshold, uint32_t p,
                          int32_t clamp, int32_t homology) {
    oracle_result *res = (oracle_result *)calloc(1, sizeof(oracle_result));
    if (!res) return NULL;
    if (n < 1 || max_dim < 0 || max_dim > OR_MAXD) {
        result_set_err(res, "bad n or max_dim");
        return res;
    }
    if (!is_prime(p) || p >= 65536) {
        result_set_err(res, "p must be a prime < 65536");
        return res;
    }
    int64_t npairs_tri = (int64_t)n * (n - 1) / 2;
    for (int64_t e = 0; e < npairs_tri; ++e)
        if (!(D[e] >= 0.0f) || isinf(D[e])) {
            result_set_err(res, "distances must be finite and >= 0");
            return res;
        }
    res->n = n;
    res->max_dim = max_dim;
    res->p = p;

    /* enclosing radius: min over x of max over y of d(x, y) */
    float r_enc = INFINITY;
    if (n == 1) r_enc = 0.0f;
    for (int32_t x = 0; x < n && n > 1; ++x) {
        float mx = 0.0f;
        for (int32_t y = 0; y < n; ++y)
            if (y != x) {
                float d = dist_of(D, n, x, y);
                if (d > mx) mx = d;
            }
        if (mx < r_enc) r_enc = mx;
    }
    float t = threshold;
    if (clamp && r_enc < t) t = r_enc;
    res->r_enc = r_enc;
    res->t_eff = t;

    /* binomial table C(i, j), j <= max_dim + 2, i <= n */
    int64_t tabw = (int64_t)n + 1;
    int64_t *tab = (int64_t *)xmalloc(sizeof(int64_t) * (max_dim + 3) * tabw);
    for (int j = 0; j <= max_dim + 2; ++j)
        for (int64_t i = 0; i <= n; ++i) tab[j * tabw + i] = choose(i, j);

    /* explicit simplex lists */
    int top = max_dim + 1;
    slist K[OR_MAXD + 2];
    memset(K, 0, sizeof(K));
    K[0].k = 0;
    K[0].count = n;
    K[0].verts = (int32_t *)xmalloc(sizeof(int32_t) * n);
    K[0].idx = (int64_t *)xmalloc(sizeof(int64_t) * n);
    K[0].diam = (float *)xmalloc(sizeof(float) * n);
    for (int32_t i = 0; i < n; ++i) {
        K[0].verts[i] = i;
        K[0].idx[i] = i;
        K[0].diam[i] = 0.0f;
    }
    for (int k = 0; k < top; ++k) expand(&K[k], &K[k + 1], D, n, t, tab, tabw);
    for (int k = 0; k <= top; ++k) {
        slist_sort_refined(&K[k]);
        res->count[k] = K[k].count;
    }
    lookup L[OR_MAXD + 2];
    for (int k = 0; k <= top; ++k) lookup_build(&L[k], &K[k]);

    /* pivots of dimension k-1, as reversed positions in K_k */
    uint8_t *cleared = (uint8_t *)calloc(K[0].count ? K[0].count : 1, 1);

    for (int k = 0; k <= max_dim; ++k) {
        int64_t nc = K[k].count, nr = K[k + 1].count;
        scol *cols = build_coboundary(&K[k], &K[k + 1], &L[k], p, tab, tabw);

        /* zero-persistence apparent pairs, from the definition: sigma's
           oldest cofacet tau (largest row of the unreduced column) has
           sigma as its youngest facet (smallest column among its facets) */
        uint8_t *app_col = (uint8_t *)calloc(nc ? nc : 1, 1);
        {
            /* youngest facet of each row: min column over its entries */
            int64_t *young = (int64_t *)xmalloc(sizeof(int64_t) * (nr ? nr : 1));
            for (int64_t r = 0; r < nr; ++r) young[r] = INT64_MAX;
            for (int64_t c = 0; c < nc; ++c)
                for (int64_t e = 0; e < cols[c].len; ++e)
                    if (c < young[cols[c].row[e]]) young[cols[c].row[e]] = c;
            res->app_lo[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
            res->app_hi[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
            for (int64_t c = 0; c < nc; ++c) {
                if (cols[c].len == 0) continue;
                int64_t r = cols[c].row[cols[c].len - 1];
                if (young[r] != c) continue;
                int64_t spos = nc - 1 - c, tpos = nr - 1 - r;
                res->app_lo[k][res->napp[k]] = K[k].idx[spos];
                res->app_hi[k][res->napp[k]] = K[k + 1].idx[tpos];
                res->napp[k]++;
                if (K[k].diam[spos] == K[k + 1].diam[tpos]) {
                    app_col[c] = 1;
                    res->nzero_app_col[k]++;
                }
            }
            free(young);
        }
        /* sigma in a zero apparent pair (rho, sigma): recomputed from the
           unreduced coboundary of dimension k-1 */
        uint8_t *app_piv = (uint8_t *)calloc(nc ? nc : 1, 1);
        if (k >= 1) {
            int64_t pc = K[k - 1].count;
            scol *pcols = build_coboundary(&K[k - 1], &K[k], &L[k - 1], p, tab, tabw);
            int64_t *young = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
            for (int64_t r = 0; r < nc; ++r) young[r] = INT64_MAX;
            for (int64_t c = 0; c < pc; ++c)
                for (int64_t e = 0; e < pcols[c].len; ++e)
                    if (c < young[pcols[c].row[e]]) young[pcols[c].row[e]] = c;
            for (int64_t c = 0; c < pc; ++c) {
                if (pcols[c].len == 0) continue;
                int64_t r = pcols[c].row[pcols[c].len - 1];
                if (young[r] != c) continue;
                int64_t rpos = pc - 1 - c, spos = nc - 1 - r;
                if (K[k - 1].diam[rpos] == K[k].diam[spos]) {
                    app_piv[r] = 1;
                    res->nzero_app_piv[k]++;
                }
            }
            free(young);
            for (int64_t c = 0; c < pc; ++c) scol_free(&pcols[c]);
            free(pcols);
        }

        /* columns left after clearing and after dropping zero apparent pairs */
        res->col_idx[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
        res->col_diam[k] = (float *)xmalloc(sizeof(float) * (nc ? nc : 1));
        for (int64_t c = 0; c < nc; ++c) {
            if (cleared[c]) res->ncleared[k]++;
            if (cleared[c] || app_col[c] || app_piv[c]) continue;
            int64_t pos = nc - 1 - c;
            res->col_idx[k][res->ncols[k]] = K[k].idx[pos];
            res->col_diam[k][res->ncols[k]] = K[k].diam[pos];
            res->ncols[k]++;
        }
        free(app_col);
        free(app_piv);

        /* Algorithm 2: clear, then Algorithm 1 on the remaining columns */
        int64_t *owner = (int64_t *)xmalloc(sizeof(int64_t) * (nr ? nr : 1));
        for (int64_t c = 0; c < nc; ++c)
            if (!cleared[c]) res->nreduced_cols[k]++;
        reduce_columns(cols, nc, nr, cleared, p, owner);

        barrec *bars = (barrec *)xmalloc(sizeof(barrec) * (nc ? nc : 1));
        int64_t nb = 0;
        res->pair_lo[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
        res->pair_hi[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
        res->ess[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nc ? nc : 1));
        for (int64_t c = 0; c < nc; ++c) {
            if (cleared[c]) continue;
            int64_t spos = nc - 1 - c;
            if (cols[c].len > 0) {
                int64_t r = cols[c].row[cols[c].len - 1];
                int64_t tpos = nr - 1 - r;
                res->pair_lo[k][res->npairs[k]] = K[k].idx[spos];
                res->pair_hi[k][res->npairs[k]] = K[k + 1].idx[tpos];
                res->npairs[k]++;
                if (K[k + 1].diam[tpos] > K[k].diam[spos]) {
                    bars[nb].diam = K[k].diam[spos];
                    bars[nb].bidx = K[k].idx[spos];
                    bars[nb].didx = K[k + 1].idx[tpos];
                    bars[nb].death = K[k + 1].diam[tpos];
                    ++nb;
                }
            } else {
                res->ess[k][res->nessential[k]++] = K[k].idx[spos];
                bars[nb].diam = K[k].diam[spos];
                bars[nb].bidx = K[k].idx[spos];
                bars[nb].didx = -1;
                bars[nb].death = INFINITY;
                ++nb;
            }
        }
        qsort(bars, nb, sizeof(barrec), cmp_bar);
        res->nbars[k] = nb;
        res->birth[k] = (float *)xmalloc(sizeof(float) * (nb ? nb : 1));
        res->death[k] = (float *)xmalloc(sizeof(float) * (nb ? nb : 1));
        res->bsimp[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nb ? nb : 1));
        res->dsimp[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nb ? nb : 1));
        for (int64_t b = 0; b < nb; ++b) {
            res->birth[k][b] = bars[b].diam;
            res->death[k][b] = bars[b].death;
            res->bsimp[k][b] = bars[b].bidx;
            res->dsimp[k][b] = bars[b].didx;
        }
        free(bars);

        /* the pivots of this dimension clear columns of the next */
        free(cleared);
        cleared = (uint8_t *)calloc(nr ? nr : 1, 1);
        for (int64_t r = 0; r < nr; ++r)
            if (owner[r] >= 0) cleared[r] = 1;
        free(owner);
        for (int64_t c = 0; c < nc; ++c) scol_free(&cols[c]);
        free(cols);
    }
    free(cleared);

    /* homology cross-check: Algorithm 1 on the explicit boundary matrices in
       filtration order (rows/columns = refined positions), no clearing */
    if (homology) {
        res->have_hom = 1;
        int64_t *zero_col_prev = NULL; /* per k-simplex: 1 if its column of d_k is zero */
        uint8_t *is_piv = NULL;
        /* boundary of K_{k+1} -> K_k for k = 0..max_dim; a k-simplex is
           essential iff its d_k column is zero and it is no pivot of d_{k+1} */
        uint8_t *zero_k = (uint8_t *)xmalloc(K[0].count ? K[0].count : 1);
        memset(zero_k, 1, K[0].count ? K[0].count : 1); /* vertices: d_0 = 0 */
        for (int k = 0; k <= max_dim; ++k) {
            int64_t nrow = K[k].count, ncol = K[k + 1].count;
            /* column pos_tau: facets of tau as refined positions in K_k */
            scol *cols = (scol *)calloc(ncol ? ncol : 1, sizeof(scol));
            int32_t f[OR_MAXD + 3];
            for (int64_t c = 0; c < ncol; ++c) {
                const int32_t *tv = K[k + 1].verts + c * (k + 2);
                for (int m = 0; m <= k + 1; ++m) {
                    int q = 0;
                    for (int u = 0; u <= k + 1; ++u)
                        if (u != m) f[q++] = tv[u];
                    int64_t fpos = lookup_find(&L[k], cns_index(f, k, tab, tabw));
                    /* standard orientation: removing the vertex that is
                       (k+1-m)-th in increasing order */
                    uint32_t coeff = ((k + 1 - m) % 2 == 0) ? 1u % p : (p - 1) % p;
                    scol_push(&cols[c], fpos, coeff);
                }
                scol_sort(&cols[c]);
            }
            int64_t *owner = (int64_t *)xmalloc(sizeof(int64_t) * (nrow ? nrow : 1));
            reduce_columns(cols, ncol, nrow, NULL, p, owner);
            is_piv = (uint8_t *)calloc(nrow ? nrow : 1, 1);
            res->hom_lo[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nrow ? nrow : 1));
            res->hom_hi[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nrow ? nrow : 1));
            res->hom_ess[k] = (int64_t *)xmalloc(sizeof(int64_t) * (nrow ? nrow : 1));
            for (int64_t c = 0; c < ncol; ++c)
                if (cols[c].len > 0) {
                    int64_t r = cols[c].row[cols[c].len - 1];
                    is_piv[r] = 1;
                    res->hom_lo[k][res->hom_npairs[k]] = K[k].idx[r];
                    res->hom_hi[k][res->hom_npairs[k]] = K[k + 1].idx[c];
                    res->hom_npairs[k]++;
                }
            for (int64_t r = 0; r < nrow; ++r)
                if (zero_k[r] && !is_piv[r]) res->hom_ess[k][res->hom_ness[k]++] = K[k].idx[r];
            free(zero_k);
            zero_k = (uint8_t *)xmalloc(ncol ? ncol : 1);
            for (int64_t c = 0; c < ncol; ++c) zero_k[c] = cols[c].len == 0;
            for (int64_t c = 0; c < ncol; ++c) scol_free(&cols[c]);
            free(cols);
            free(owner);
            free(is_piv);
            is_piv = NULL;
        }
        free(zero_k);
        (void)zero_col_prev;
    }

    for (int k = 0; k <= top; ++k) {
        lookup_free(&L[k]);
        slist_free(&K[k]);
    }
    free(tab);
    return res;
}

/* ------------------------------------------------------------------ */
/* accessors for the ctypes wrapper                                    */
/* ------------------------------------------------------------------ */

const char *oracle_error(const oracle_result *r) { return r->err; }
float oracle_threshold(const oracle_result *r) { return r->t_eff; }
float oracle_enclosing_radius(const oracle_result *r) { return r->r_enc; }
int64_t oracle_simplex_count(const oracle_result *r, int k) { return r->count[k]; }
int64_t oracle_num_bars(const oracle_result *r, int k) { return r->nbars[k]; }
int64_t oracle_num_columns(const oracle_result *r, int k) { return r->ncols[k]; }
int64_t oracle_num_pairs(const oracle_result *r, int k) { return r->npairs[k]; }
int64_t oracle_num_essential(const oracle_result *r, int k) { return r->nessential[k]; }
int64_t oracle_num_apparent(const oracle_result *r, int k) { return r->napp[k]; }
int64_t oracle_num_hom_pairs(const oracle_result *r, int k) { return r->hom_npairs[k]; }
int64_t oracle_num_hom_essential(const oracle_result *r, int k) { return r->hom_ness[k]; }

void oracle_counters(const oracle_result *r, int k, int64_t *out6) {
    out6[0] = r->ncleared[k];
    out6[1] = r->nzero_app_col[k];
    out6[2] = r->nzero_app_piv[k];
    out6[3] = r->nreduced_cols[k];
    out6[4] = r->npairs[k];
    out6[5] = r->nessential[k];
}

void oracle_get_bars(const oracle_result *r, int k, float *birth, float *death, int64_t *bs,
                     int64_t *ds) {
    int64_t nb = r->nbars[k];
    memcpy(birth, r->birth[k], sizeof(float) * nb);
    memcpy(death, r->death[k], sizeof(float) * nb);
    memcpy(bs, r->bsimp[k], sizeof(int64_t) * nb);
    memcpy(ds, r->dsimp[k], sizeof(int64_t) * nb);
}

void oracle_get_columns(const oracle_result *r, int k, int64_t *idx, float *diam) {
    memcpy(idx, r->col_idx[k], sizeof(int64_t) * r->ncols[k]);
    memcpy(diam, r->col_diam[k], sizeof(float) * r->ncols[k]);
}

void oracle_get_pairs(const oracle_result *r, int k, int64_t *lo, int64_t *hi, int64_t *ess) {
    memcpy(lo, r->pair_lo[k], sizeof(int64_t) * r->npairs[k]);
    memcpy(hi, r->pair_hi[k], sizeof(int64_t) * r->npairs[k]);
    memcpy(ess, r->ess[k], sizeof(int64_t) * r->nessential[k]);
}

void oracle_get_hom_pairs(const oracle_result *r, int k, int64_t *lo, int64_t *hi, int64_t *ess) {
    memcpy(lo, r->hom_lo[k], sizeof(int64_t) * r->hom_npairs[k]);
    memcpy(hi, r->hom_hi[k], sizeof(int64_t) * r->hom_npairs[k]);
    memcpy(ess, r->hom_ess[k], sizeof(int64_t) * r->hom_ness[k]);
}

void oracle_get_apparent(const oracle_result *r, int k, int64_t *lo, int64_t *hi) {
    memcpy(lo, r->app_lo[k], sizeof(int64_t) * r->napp[k]);
    memcpy(hi, r->app_hi[k], sizeof(int64_t) * r->napp[k]);
}

/* CNS index of the simplex with the k+1 given vertices in decreasing order
   (section "Indexing simplices in the combinatorial number system"). */
int64_t oracle_cns_index(const int32_t *verts_desc, int32_t k) {
    int64_t s = 0;
    for (int m = 0; m <= k; ++m) s += choose(verts_desc[m], k - m + 1);
    return s;
}

/* All simplices of dimension <= top with diameter <= t (t used as given), in
   the lexicographically refined order (diameter, dimension, reverse colex).
   Returns the count; if out_* are non-NULL they receive dim, CNS index and
   diameter (capacity cap). */
int64_t oracle_filtration(const float *D, int32_t n, int32_t top, float t, int32_t *out_dim,
                          int64_t *out_idx, float *out_diam, int64_t cap) {
    if (n < 1 || top < 0 || top > OR_MAXD + 1) return -1;
    int64_t tabw = (int64_t)n + 1;
    int64_t *tab = (int64_t *)xmalloc(sizeof(int64_t) * (top + 2) * tabw);
    for (int j = 0; j <= top + 1; ++j)
        for (int64_t i = 0; i <= n; ++i) tab[j * tabw + i] = choose(i, j);
    slist K[OR_MAXD + 2];
    memset(K, 0, sizeof(K));
    K[0].k = 0;
    K[0].count = n;
    K[0].verts = (int32_t *)xmalloc(sizeof(int32_t) * n);
    K[0].idx = (int64_t *)xmalloc(sizeof(int64_t) * n);
    K[0].diam = (float *)xmalloc(sizeof(float) * n);
    for (int32_t i = 0; i < n; ++i) {
        K[0].verts[i] = i;
        K[0].idx[i] = i;
        K[0].diam[i] = 0.0f;
    }
    for (int k = 0; k < top; ++k) expand(&K[k], &K[k + 1], D, n, t, tab, tabw);
    int64_t total = 0;
    for (int k = 0; k <= top; ++k) {
        slist_sort_refined(&K[k]);
        total += K[k].count;
    }
    if (out_idx && total <= cap) {
        /* merge the per-dimension lists: diameter, then dimension */
        int64_t at[OR_MAXD + 2] = {0};
        for (int64_t o = 0; o < total; ++o) {
            int best = -1;
            for (int k = 0; k <= top; ++k) {
                if (at[k] >= K[k].count) continue;
                if (best < 0 || K[k].diam[at[k]] < K[best].diam[at[best]]) best = k;
            }
            out_dim[o] = best;
            out_idx[o] = K[best].idx[at[best]];
            out_diam[o] = K[best].diam[at[best]];
            at[best]++;
        }
    }
    for (int k = 0; k <= top; ++k) slist_free(&K[k]);
    free(tab);
    return total;
}
