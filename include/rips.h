/*
 * rips.h -- C ABI of the MI355X (gfx950) Vietoris-Rips persistence library.
 *
 * The library computes persistence barcodes of the lexicographically refined
 * Vietoris-Rips filtration of a finite metric space over the prime field Z/p,
 * following U. Bauer, "Ripser: efficient computation of Vietoris-Rips
 * persistence barcodes" (arXiv:1908.02518):
 *   - simplices are indexed in the combinatorial number system (section
 *     "Indexing simplices in the combinatorial number system");
 *   - the filtration is refined by diameter, then dimension, then reverse
 *     colexicographic order (section "Lexicographic refinement");
 *   - persistence is computed as relative cohomology with clearing, in
 *     increasing dimension (Algorithm 2 applied to coboundary matrices,
 *     section "Persistent cohomology"), with implicit coboundary columns
 *     (section "Implicit matrix reduction"), columns in zero-persistence
 *     apparent pairs skipped (section "Apparent pairs", Proposition on zero
 *     apparent pairs; "Assembling column indices") and the emergent-pair
 *     shortcut (Proposition on emergent pairs);
 *   - with no threshold the enclosing radius min_x max_y d(x, y) is used
 *     ("Input" paragraph); a finite threshold is also clamped to it, which
 *     changes no bar of nonzero persistence.
 * Every step runs in hand-written HIP kernels on the GPU; there is no CPU
 * fallback. All entry points return a rips_status; no exception crosses the
 * ABI. Error details for the calling thread: rips_last_error().
 *
 * Conventions shared by all entry points
 *   - Distances are float32, d(i, j) = sqrt(sum_c (x_ic - x_jc)^2) with the
 *     sum taken over c in increasing order, each product and sum rounded to
 *     float32 (no fused multiply-add) and a correctly rounded square root.
 *   - A simplex is reported by its CNS index within its dimension; a vertex
 *     v has index v. For a bar of dimension d the birth simplex is a
 *     d-simplex, the death simplex a (d+1)-simplex (-1 for an infinite bar).
 *   - Bars of zero persistence (death == birth in float32) are not reported.
 *   - Within a dimension bars are ordered by the refined order of their birth
 *     simplex: birth ascending, then birth simplex index descending.
 *   - H0 birth simplices follow the elder rule of the reduction: when two
 *     components merge, the one whose oldest vertex (largest index) is
 *     younger dies.
 *   - Limits: 1 <= n <= RIPS_MAX_POINTS, 0 <= max_dim <= RIPS_MAX_DIM,
 *     2 <= p < 65536 prime, and C(n, max_dim + 2) < 2^63 (simplex indices are
 *     64-bit, "Vertices and simplices" paragraph).
 */
#ifndef RIPS_H
#define RIPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RIPS_MAX_DIM 3
#define RIPS_MAX_POINTS 65535

typedef enum {
    RIPS_OK = 0,
    RIPS_E_INVALID_ARG = -1,    /* bad size, dimension, pointer or layout */
    RIPS_E_NOT_PRIME = -2,      /* p is not a prime in [2, 65536) */
    RIPS_E_INDEX_OVERFLOW = -3, /* C(n, max_dim + 2) does not fit in int64 */
    RIPS_E_NONFINITE = -4,      /* NaN/Inf coordinate or distance, or a negative distance */
    RIPS_E_OOM = -5,            /* device or host allocation failed */
    RIPS_E_CAPACITY = -6,       /* a caller-provided output buffer is too small; see `needed` */
    RIPS_E_HIP = -7             /* a HIP runtime call failed */
} rips_status;

/* Bars of one dimension (host memory owned by the rips_result). */
typedef struct {
    int64_t count;
    float *birth;
    float *death;           /* +INFINITY for an essential class */
    int64_t *birth_simplex; /* CNS index of a d-simplex */
    int64_t *death_simplex; /* CNS index of a (d+1)-simplex, -1 if essential */
} rips_bars;

/* Per-dimension counters (Table "counts of pairs" of the paper is of this kind). */
typedef struct {
    int64_t candidates;     /* d-simplices of diameter <= threshold */
    int64_t cleared;        /* candidates that were pivots in dimension d-1 (clearing) */
    int64_t apparent_col;   /* candidates sigma in a zero apparent pair (sigma, tau) */
    int64_t apparent_pivot; /* candidates sigma in a zero apparent pair (rho, sigma), d >= 2 */
    int64_t columns;        /* columns left for the reduction */
    int64_t emergent;       /* columns resolved by the emergent shortcut */
    int64_t reduced;        /* columns that needed at least one column addition */
    int64_t additions;      /* column additions in total */
    int64_t bars_nonzero;   /* finite bars of nonzero persistence */
    int64_t essential;      /* infinite bars */
    int64_t entries_added;  /* entries added to working columns by the reduction */
    int64_t entries_stored; /* entries of the stored reduction columns (V and R parts) */
} rips_dim_stats;

typedef struct {
    int32_t n;
    int32_t max_dim;
    uint32_t p;
    int32_t sparse;          /* 1 if neighbour lists were used for cofacets */
    float threshold_used;    /* min(threshold, enclosing radius) */
    float enclosing_radius;
    rips_bars *dims;         /* max_dim + 1 entries */
    rips_dim_stats *stats;   /* max_dim + 1 entries */
    int64_t *simplex_count;  /* max_dim + 1 entries: |K_d| at threshold_used */
    /* columns left for the reduction in each dimension, in reduction order
       (diameter descending, then CNS index ascending) */
    int64_t *column_count;   /* max_dim + 1 entries */
    int64_t **column_index;  /* max_dim + 1 arrays */
    float **column_diam;     /* max_dim + 1 arrays */
} rips_result;

/*
 * rips_barcode -- barcode of one point cloud or distance matrix (host memory).
 *   data      dim > 0: n x dim float32 points, row-major;
 *             dim == 0: n x n float32 distance matrix, row-major; only the
 *             entries (i, j) with i > j are read.
 *   threshold +INFINITY for none; simplices with diameter <= threshold.
 *   p         prime coefficient field Z/p, 2 <= p < 65536.
 *   out       receives a library-allocated result (free with
 *             rips_result_free); *out = NULL on error.
 * Inputs are copied; no caller pointer is kept. Runs on the current HIP device.
 */
rips_status rips_barcode(const float *data, int64_t n, int32_t dim, int32_t max_dim,
                         float threshold, uint32_t p, rips_result **out);

void rips_result_free(rips_result *r);

/*
 * Representative cocycles of the bars of one dimension d >= 1 (section
 * "Matrix reduction": the columns V_j of the reduction matrix, together with
 * the reduced columns, form a basis of the filtered complex; here, in
 * cohomology, the columns of the coboundary matrix). For the bar born at the
 * d-simplex sigma_j and dying at tau, the cochain V_j (sigma_j plus the
 * combination of the columns added to it) has tau as the oldest simplex of
 * its coboundary: it is a cocycle on every simplex older than tau. For an
 * essential bar, V_j is a cocycle. Runs rips_barcode up to dimension d.
 * data, n, dim, threshold, p: as for rips_barcode. Bars of dimension d in the
 * same canonical order; the cocycle of bar b is entries
 * [offsets[b], offsets[b + 1]) of simplex (CNS indices of d-simplices) and
 * coef (in Z/p, nonzero). The library allocates *out; rips_cocycles_free
 * releases it. d < 1 or out of range: RIPS_E_INVALID_ARG; *out = NULL on
 * error. Uses the shortcuts set by rips_set_shortcuts (V_j is the same).
 */
typedef struct {
    int32_t dim;
    int64_t count;
    float *birth, *death;
    int64_t *birth_simplex, *death_simplex;
    int64_t *offsets; /* count + 1 */
    int64_t *simplex; /* offsets[count] */
    uint32_t *coef;
} rips_cocycles;
rips_status rips_barcode_cocycles(const float *data, int64_t n, int32_t dim, int32_t d, float threshold,
                                  uint32_t p, rips_cocycles **out);
void rips_cocycles_free(rips_cocycles *c);
const char *rips_status_string(rips_status s);
const char *rips_last_error(void);

/*
 * rips_barcode_device -- one cloud, device-resident input and output.
 * Same computation and arguments as rips_barcode, but `d_data` is device
 * memory and the bars are written to caller-owned device buffers:
 *   birth/death/birth_simplex/death_simplex hold (max_dim + 1) * cap entries;
 *   dimension d uses entries [d * cap, d * cap + count[d]).
 * Host-side results: count[d], stats[d], simplex_count[d], threshold_used.
 * On RIPS_E_CAPACITY nothing is written to the bar buffers and needed_cap
 * holds the capacity that suffices. All work is queued on `hip_stream`
 * (a hipStream_t, NULL = default stream); the call returns after the stream
 * has finished. Scratch memory is owned by a per-device context that grows
 * on demand and is reused by later calls.
 */
typedef struct {
    int64_t cap;
    float *birth;
    float *death;
    int64_t *birth_simplex;
    int64_t *death_simplex;
    int64_t count[RIPS_MAX_DIM + 1];
    rips_dim_stats stats[RIPS_MAX_DIM + 1];
    int64_t simplex_count[RIPS_MAX_DIM + 1];
    float threshold_used;
    int32_t sparse;
    int64_t needed_cap;
} rips_device_out;

rips_status rips_barcode_device(const float *d_data, int64_t n, int32_t dim, int32_t max_dim,
                                float threshold, uint32_t p, rips_device_out *out,
                                void *hip_stream);

/*
 * rips_barcode_device_noalloc -- rips_barcode_device for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same computation, arguments, outputs and
 * error behaviour as rips_barcode_device; the call itself allocates nothing:
 * no hipMalloc, hipFree, pinned host memory or library allocation. All its
 * scratch memory is carved from one fixed device array of
 * RIPS_NOALLOC_SCRATCH_MIB MiB that the library holds on every GPU it runs on
 * until the process ends (its device address is taken at the first call on
 * each device). Limits: n <= RIPS_NOALLOC_MAX_POINTS and
 * max_dim <= RIPS_NOALLOC_MAX_DIM (else RIPS_E_INVALID_ARG); an input whose
 * scratch does not fit the array returns RIPS_E_CAPACITY. The reduction runs
 * in one workgroup. Every call on a GPU reuses that GPU's array, which keeps
 * the last call's contents (everything that must start at zero is cleared by
 * the call); calls are serialized per device by the library, and concurrent
 * use of the array by other means would race. Kernel profiling
 * (rips_profile_enable) does not time this entry point.
 */
#define RIPS_NOALLOC_SCRATCH_MIB 64
#define RIPS_NOALLOC_MAX_POINTS 256
#define RIPS_NOALLOC_MAX_DIM 1
rips_status rips_barcode_device_noalloc(const float *d_data, int64_t n, int32_t dim, int32_t max_dim,
                                        float threshold, uint32_t p, rips_device_out *out,
                                        void *hip_stream);

/*
 * rips_simplex_counts_device -- |K_d| for d = 0 .. top (top <= RIPS_MAX_DIM + 1)
 * at threshold min(threshold, enclosing radius), counted on the GPU without
 * storing the top dimension. Used for throughput accounting
 * (simplices of the explicit filtration). counts: host array of top + 1.
 */
rips_status rips_simplex_counts_device(const float *d_data, int64_t n, int32_t dim, int32_t top,
                                       float threshold, int64_t *counts, void *hip_stream);

/*
 * rips_barcode_batched_device -- barcodes of B point clouds of uneven sizes
 * in one persistent launch (one workgroup per cloud from a queue ordered by
 * decreasing size), replayed from a cached hipGraph when the arguments
 * repeat. Same method and conventions as rips_barcode, per cloud.
 *   d_points   device float32, all clouds' points concatenated row-major
 *              (dim coordinates each); cloud b has rows
 *              [d_offsets[b], d_offsets[b+1]).
 *   d_offsets  device int64, B + 1 entries, nondecreasing, d_offsets[0] = 0.
 *   n_max      an upper bound on every cloud's size, 1 <= n_max <= 2048
 *              (sizes scratch memory; clouds above it give RIPS_E_INVALID_ARG).
 *   max_dim    0 or 1.
 *   out        caller-owned device arrays:
 *                birth/death/birth_simplex/death_simplex: cap entries;
 *                bar_offsets: B * (max_dim + 1) + 1 entries; the bars of
 *                  cloud b in dimension d are [bar_offsets[b*(max_dim+1)+d],
 *                  bar_offsets[b*(max_dim+1)+d+1]), canonical order inside;
 *                stats: B * (max_dim + 1) entries, or NULL;
 *                threshold_used: B entries, or NULL.
 *              `needed` (host) receives the total number of bars; if it
 *              exceeds cap the call returns RIPS_E_CAPACITY and the bar
 *              arrays are not written (bar_offsets are).
 * Work is queued on `hip_stream`; the call returns after it has finished.
 */
typedef struct {
    int64_t cap;
    float *birth;
    float *death;
    int64_t *birth_simplex;
    int64_t *death_simplex;
    int64_t *bar_offsets;
    rips_dim_stats *stats;
    float *threshold_used;
    int64_t needed;
} rips_batch_out;

rips_status rips_barcode_batched_device(const float *d_points, const int64_t *d_offsets, int32_t B,
                                        int32_t dim, int32_t n_max, int32_t max_dim,
                                        float threshold, uint32_t p, rips_batch_out *out,
                                        void *hip_stream);

/*
 * rips_backward_device -- gradient of a loss through the bars. The paper
 * does not differentiate barcodes; the reading here: every finite bar
 * endpoint equals the length of one edge of its simplex, its critical edge
 * (the edge of largest float32 length, as the forward computes it, ties to
 * the smallest CNS edge index), so d(loss)/d(endpoint) flows to the two
 * points of that edge: d||x_u - x_v||/dx_u = (x_u - x_v)/||x_u - x_v|| and
 * the negative for x_v (nothing at zero length). Vertex births (k = 0) and
 * absent simplices (index -1) contribute nothing.
 *   d_data        the forward's device input: points (rows x dim) or, with
 *                 dim == 0, the n x n distance matrix; then the gradient goes
 *                 to matrix entry (u, v), u > v, the entry the forward read.
 *   n             points per cloud (an upper bound for batched clouds).
 *   nbars         bars; k_birth: dimension of their birth simplices (death
 *                 simplices have k_birth + 1).
 *   d_row0        per bar, the row of its cloud's first point (batched
 *                 bars), or NULL for one cloud; must be NULL when dim == 0.
 *   d_birth_simplex, d_death_simplex   device int64 CNS indices per bar.
 *   d_grad_birth, d_grad_death         device float32 d(loss)/d(endpoint).
 *   d_grad        device float32, same shape as d_data; accumulated into
 *                 (+=) with float32 atomics (summation order unspecified).
 * Indices must come from the forward on the same input; every vertex read
 * is below n. Returns after the stream has finished.
 */
rips_status rips_backward_device(const float *d_data, int64_t n, int32_t dim, int64_t nbars,
                                 int32_t k_birth, const int64_t *d_row0,
                                 const int64_t *d_birth_simplex, const int64_t *d_death_simplex,
                                 const float *d_grad_birth, const float *d_grad_death,
                                 float *d_grad, void *hip_stream);

/*
 * Workgroups of the single-cloud reduction (per device, the current one).
 * 0 (default): one per compute unit. Each takes the next column in the
 * reduction order and reduces it against the pivot table as it stands; a
 * column commits its pivot only once no earlier column can still end with
 * it, which gives exactly the pairs of the column-by-column order
 * (Algorithm 2 on the coboundary matrix, section "Persistent cohomology",
 * with the shortcut of section "Emergent persistence pairs"). 1: the
 * columns one after another in one workgroup.
 * Results are bit-identical either way. Returns RIPS_E_INVALID_ARG for a
 * negative count; rips_get_reduce_workgroups reads the setting back.
 */
rips_status rips_set_reduce_workgroups(int32_t workgroups);
rips_status rips_get_reduce_workgroups(int32_t *workgroups);

/*
 * Shortcuts of the single-cloud path (per device, the current one), as the
 * ablation switches of the experiments section (Table 3): the barcode is the
 * same with any of them off, only the work changes.
 *   RIPS_SHORTCUT_APPARENT: zero apparent pairs (section "Apparent pairs") are
 *     found by the data-parallel filter and never become columns, and a pivot
 *     in such a pair is added from its facet without a column of its own.
 *     Off: every candidate that is not cleared is a column, and the pivot
 *     test uses the pivot table only.
 *   RIPS_SHORTCUT_EMERGENT: a column whose oldest cofacet no column owns
 *     pairs with it without enumerating its coboundary (paragraph "Emergent
 *     persistence pairs").
 *   RIPS_SHORTCUT_CLEARING: a simplex that is a pivot of the dimension below
 *     gets no column (section "Clearing inessential birth columns"). Off:
 *     its column is reduced, to zero, and gives no bar.
 * Default: all three. flags outside the three bits: RIPS_E_INVALID_ARG;
 * rips_get_shortcuts reads the setting back. The batched path always uses
 * all three. Cohomology is always computed.
 */
#define RIPS_SHORTCUT_APPARENT 1
#define RIPS_SHORTCUT_EMERGENT 2
#define RIPS_SHORTCUT_CLEARING 4
rips_status rips_set_shortcuts(int32_t flags);
rips_status rips_get_shortcuts(int32_t *flags);

/*
 * When the single-cloud path keeps a death column's reduced column R_j beside
 * V_j (Table 3: implicit reduction storing, or discarding, the reduced
 * matrix; section "Implicit matrix reduction"). An addition of column j
 * later adds the stored R_j, or recomputes the coboundaries of V_j's
 * simplices.
 *   RIPS_R_AUTO (default): R_j is kept when it is cheaper to add than those
 *     coboundaries are to recompute (and fits the working column's LDS part);
 *   RIPS_R_DISCARD: never kept;
 *   RIPS_R_STORE: kept whenever it fits the working column's LDS part;
 *   RIPS_R_EXPLICIT: explicit matrix reduction (the "explicit" column of
 *     Table 3): before each dimension is reduced, the coboundary columns of
 *     all its columns (after clearing) are built in device memory, and every
 *     reduced column is stored and used for the additions. The apparent and
 *     emergent shortcuts do not apply (rips_set_shortcuts' clearing bit
 *     does). A coboundary column of more than 4096 cofacets <= threshold
 *     returns RIPS_E_CAPACITY. stats: emergent, apparent_col and
 *     apparent_pivot are 0; entries_stored counts the entries of the
 *     coboundary matrix and of the stored reduced columns.
 *     rips_barcode_cocycles keeps the implicit reduction in this mode.
 * The bars are the same in every mode. Other values: RIPS_E_INVALID_ARG.
 * The batched path always uses RIPS_R_AUTO.
 */
#define RIPS_R_AUTO 0
#define RIPS_R_DISCARD 1
#define RIPS_R_STORE 2
#define RIPS_R_EXPLICIT 3
rips_status rips_set_reduced_storage(int32_t mode);
rips_status rips_get_reduced_storage(int32_t *mode);

/*
 * The working column of the dimension-1 reduction (per device, the current
 * one; single-cloud and batched paths). Its rows are triangles, and over
 * Z/2 with every shortcut on it can be held direct-mapped: one bit per
 * (longest edge, third vertex), the edges <= t in order of length, so that
 * an addition is one XOR per entry and the oldest entry is the highest bit
 * of the first nonempty edge (the refined order of section "Lexicographic
 * refinement"; the implicit columns of section "Implicit matrix
 * reduction").
 *   RIPS_WORKING_COLUMN_AUTO (default): direct-mapped where it applies and
 *     fits (n <= 1920, at most 2^18 edges <= t, its bitmaps within 8 GiB),
 *     else the general working column;
 *   RIPS_WORKING_COLUMN_GENERAL: always the general one (LDS delta, sorted
 *     base, far list).
 * The bars are the same either way. Other values: RIPS_E_INVALID_ARG.
 */
#define RIPS_WORKING_COLUMN_AUTO 0
#define RIPS_WORKING_COLUMN_GENERAL 1
rips_status rips_set_working_column(int32_t mode);
rips_status rips_get_working_column(int32_t *mode);

/*
 * The homology variant, for the ablation of the sections "Clearing
 * inessential birth columns" and "Cohomology": the filtration boundary
 * matrices are reduced with clearing (Algorithm 2 on boundary matrices),
 * from dimension max_dim + 1 down to 1, one column after another, with the
 * reduced columns stored explicitly. The pairs of a filtration and of its
 * dual coincide, so the bars equal rips_barcode's (same canonical order);
 * what differs is the work: clearing cannot skip any column of the top
 * dimension, which cohomology never reduces. Arguments and result as for
 * rips_barcode, with max_dim <= 2 (else RIPS_E_INVALID_ARG); the shortcuts
 * of rips_set_shortcuts do not apply. stats[d] describes the boundary of the
 * (d+1)-simplices: candidates = their number, cleared = columns skipped
 * (pivots of the boundary above), columns = columns reduced, reduced =
 * columns left nonzero (every pair of dimension d), additions = column
 * additions, bars_nonzero = pairs of positive length, essential = essential
 * bars of dimension d, entries_stored = entries of the stored columns; the
 * other fields are 0. column_count is 0. RIPS_E_CAPACITY when a reduced
 * column exceeds 2048 entries or 2^24 additions.
 */
rips_status rips_barcode_homology(const float *data, int64_t n, int32_t dim, int32_t max_dim,
                                  float threshold, uint32_t p, rips_result **out);

/*
 * Launch configuration of the batched path (per device, the current one):
 *   delta_slots        LDS slots of each workgroup's working-column delta:
 *                      512, 1024 or 2048 (0 = default, 2048);
 *   workgroups_per_cu  persistent workgroups per compute unit, 1..4
 *                      (0 = default 1).
 * Results do not depend on the configuration (bit-identical bars); only
 * speed does. Returns RIPS_E_INVALID_ARG for other values.
 */
rips_status rips_batched_set_config(int32_t delta_slots, int32_t workgroups_per_cu);
rips_status rips_batched_get_config(int32_t *delta_slots, int32_t *workgroups_per_cu);

/*
 * Workgroups per cloud of the batched path (per device, the current one).
 * mode 0 (default): a batch of B clouds with at least two compute units per
 * cloud spreads each cloud over min(8, CUs / B) workgroups: one of them runs
 * the cloud's distances, H0, enumeration filter, column sort and edge order,
 * and all of them reduce its columns together (the spread-out reduction of
 * rips_set_reduce_workgroups); larger batches keep one workgroup per cloud.
 * mode 1: always one workgroup per cloud. The bars are the same either way.
 * Other values: RIPS_E_INVALID_ARG.
 */
rips_status rips_batched_set_spread(int32_t mode);

/*
 * rips_batched_autotune -- time the batched launch on the caller's batch
 * (same arguments as rips_barcode_batched_device) for every configuration
 * of delta_slots in {512, 1024, 2048} x workgroups_per_cu in {1, 2, 4},
 * `reps` timed replays each (hipEvents, after one untimed run), keep the
 * fastest with rips_batched_set_config and report it. Every configuration's
 * bar offsets are compared with the first one's; a mismatch returns
 * RIPS_E_HIP. `out` receives the bars of the last run. best_ms: mean
 * milliseconds per launch of the chosen configuration (any pointer may be
 * NULL).
 */
rips_status rips_batched_autotune(const float *d_points, const int64_t *d_offsets, int32_t B,
                                  int32_t dim, int32_t n_max, int32_t max_dim, float threshold,
                                  uint32_t p, rips_batch_out *out, void *hip_stream, int32_t reps,
                                  int32_t *best_delta_slots, int32_t *best_workgroups_per_cu,
                                  float *best_ms);

/*
 * Diagnostics: GPU time per kernel class of the calls made while profiling
 * is on, from hipEvents recorded around each launch on the caller's stream.
 * rips_profile_enable(1) clears the totals and starts recording; (0) stops.
 * Classes are numbered 0 .. rips_profile_count()-1 and named
 * ("distances", "h0", "filter_d2", "reduce_d2", ...). Not thread-safe with
 * concurrent rips_* calls on other threads.
 */
void rips_profile_enable(int on);
int rips_profile_count(void);
const char *rips_profile_name(int i);
double rips_profile_ms(int i);      /* total milliseconds */
int64_t rips_profile_calls(int i);  /* launches timed */

#ifdef __cplusplus
}
#endif

#endif /* RIPS_H */
