// rips_kernels.hpp -- buffers shared by the host driver and the kernels of
// the single-cloud path, and the launcher declarations.
#pragma once

#include "rips_device.hpp"

namespace rips {

enum {
    kStatCleared = 0,
    kStatAppCol,
    kStatAppPiv,
    kStatEmergent,
    kStatReduced,
    kStatAdditions,
    kStatBarsNonzero,
    kStatEssential,
    kStatGlobalCols, // columns that outgrew the LDS working tables
    kStatMaxV,       // longest stored V column
    kStatMaxR,       // most entries touched by one working column
    kStatPulls,      // far-list pulls
    kStatMerges,     // delta merges into the sorted base
    kStatSplits,     // sorted-base splits into the far list
    kStatPulled,     // far-list entries scanned by pulls
    kStatAdded,      // entries added to working columns
    kStatTime,       // kRedTimers phase timers of the reduction (wall-clock ticks)
    kNumStats = kStatTime + 24
};

// Device scalars of one call; read back by the host after a dimension ends.
struct Scalars {
    u32 renc_bits;    // enclosing radius as float bits (atomicMin target)
    int bad;          // nonfinite / negative input seen
    int status;       // reduction: 0 ok, 1 working column overflow, 2 V overflow
    float r_enc;
    float t_eff;
    unsigned long long edges;     // edges <= t (may exceed capacity)
    unsigned long long list;      // expanded simplices (may exceed capacity)
    unsigned long long cob;       // coboundary-list entries reserved (may exceed capacity)
    unsigned long long survivors; // columns left by the filter
    unsigned long long vcount;    // entries appended to V
    unsigned long long mst;       // forest edges
    int64_t nbars;                // bars of the current dimension
    int maxdeg;                   // largest vertex degree at the threshold
    unsigned long long stat[kNumStats];
};

struct EdgeList {
    int64_t *idx;
    float *diam;
    int *a; // larger vertex
    int *b; // smaller vertex
};

struct SimplexList {
    int64_t *idx;
    float *diam;
};

struct Columns {
    int64_t *idx;
    float *diam;
    int *j;         // zero pivot cofacet vertex, -1 if none
    uint8_t *tapp;  // 1 if that cofacet lies in a zero apparent pair
};

// Reduced columns R_j of the non-emergent death columns, kept once column j
// is final: an addition of column o then touches |R_o| entries. Emergent
// columns keep len = -1: their R_o is the coboundary of sigma_o (implicit).
// Stored columns of the reduction. Column j keeps V_j (the simplices whose
// coboundaries sum to R_j) and, when that is cheaper to add later, R_j
// itself. Entries (simplex index, diameter, coefficient) live in one append
// pool.
struct VStore {
    int64_t *off;   // per column: V_j in the pool
    int *len;       // -1: V_j is the column's own simplex (emergent pair)
    int64_t *roff;  // per column: R_j in the pool
    int *rlen;      // -1: R_j not stored
    u32 *pivcoef;   // inverse of the pivot entry of R_j (mod p)
    int64_t *idx;   // append pool
    float *diam;
    u32 *coef;
    int64_t cap;
};

struct BarBuf {
    float *birth;
    float *death;
    int64_t *bs;
    int64_t *ds;
};

struct H0Scratch {
    int *comp;
    int *hook;
    u64 *best;
    u64 *mst, *mst2;
    u32 *hi, *hi2, *val, *val2;
    int *parent;
    int *maxv;
    float *hdeath;
    int64_t *hdsimp;
    u32 *bits; // forest edges by edge index (clearing of dimension 1)
};

void launch_binom(u64 *B, int stride, int n, int jmax, hipStream_t st);
void launch_backward(const float *X, int m, int64_t nrow, int nmax, Binom B, int64_t nbars,
                     int kb, const int64_t *row0, const int64_t *bs, const int64_t *ds,
                     const float *gb, const float *gd, float *grad, hipStream_t st);
void launch_inverse(u32 *inv, u32 p, hipStream_t st);
void launch_dist(const float *data, int n, int m, float *D, int *bad, hipStream_t st);
void launch_init_scalars(Scalars *s, hipStream_t st);
void launch_reset_dim(Scalars *s, hipStream_t st);
void launch_threshold(const float *D, int n, float t, Scalars *s, hipStream_t st);
void launch_edges(const float *D, int n, Scalars *s, EdgeList E, int64_t cap, int *deg,
                  hipStream_t st);
void launch_csr(const float *D, int n, Scalars *s, const int *deg, int *off, int *nbr,
                hipStream_t st);
void launch_h0(EdgeList E, Scalars *s, int n, H0Scratch W, BarBuf out, int64_t nbits_words,
               hipStream_t st);
void launch_fill_i64(int64_t *a, int64_t n, int64_t v, hipStream_t st);
// rho's coboundary list for every slot of the apparent-pair table (app.cob,
// ckey, cdia; count = entries used, to be zeroed before)
void launch_cob_lists(const Ctx<DistFull> &c, int k, PairHash app, int64_t *ckey, float *cdia,
                      unsigned long long *count, int64_t cap, hipStream_t st);
void launch_fill_u32(u32 *a, int64_t n, u32 v, hipStream_t st);
void launch_filter(int G, const Ctx<DistFull> &c, int k, SimplexList in, int64_t count,
                   const u32 *bits, PivotHash prev, Scalars *s, Columns out, PairHash app, int flags,
                   hipStream_t st);
void launch_expand(int G, const Ctx<DistFull> &c, int k, SimplexList in, int64_t count, Scalars *s,
                   SimplexList out, int64_t cap, bool count_only, hipStream_t st);
void launch_bm_edge_order(EdgeList E, int nE, int n, SortBufs sb, int *pos, u32 *verts, float *len, u32 *run,
                          PairHash app_tab, int *app, hipStream_t st);
void launch_sort_columns(Columns in, Scalars *s, SortBufs sb, int lo_bytes, Columns out,
                         hipStream_t st);
void launch_emit(BarBuf in, Scalars *s, int reverse, BarBuf out, hipStream_t st);

// ---- the homology variant (rips_homology.hip)
constexpr int kHomThreads = 256;
constexpr int kHomCap = 2048;            // entries of the working column and of a stored one
constexpr int64_t kHomMaxAdds = 1 << 24; // additions per column
constexpr int kHomOk = 0, kHomFull = 1, kHomPool = 2, kHomTable = 3, kHomBound = 4;

struct HomOut {
    int status; // kHomOk, or what stopped the reduction
    int pad;
    long long pairs;     // bars of dimension k-1 (pairs of distinct diameters)
    long long nonzero;   // columns left nonzero (every pair)
    long long essential; // essential bars of dimension k
    long long cleared;   // columns skipped by clearing
    long long reduced;   // columns reduced
    long long additions; // column additions
    long long stored;    // entries of the stored columns
    long long longest;   // longest reduced column
};

struct HomJob {
    Ctx<DistFull> c;
    int k;               // columns are k-simplices
    const int64_t *cidx; // the k-simplices <= t, younger first
    const float *cdia;
    int64_t ncols;
    u32 p;
    const u32 *inv;
    PivotHash clear;     // pivots of the boundary of the (k+1)-simplices (keys null: none)
    PivotHash piv;       // this boundary's pivots -> stored column
    int64_t *roff;       // stored column s: entries [roff[s], roff[s] + rlen[s]) of the pool
    int *rlen;
    int64_t *pidx;       // the pool, younger first within a column
    float *pdia;
    u32 *pcoef;
    int64_t pcap;
    BarBuf pairs;        // dimension k-1
    int64_t pairs_cap;
    BarBuf ess;          // dimension k (used when essential != 0)
    int64_t ess_cap;
    int essential;
    HomOut *out;
};

size_t hom_lds_bytes();
hipError_t launch_hom_reduce(const HomJob &J, hipStream_t st);
void launch_hom_vertices(int n, PivotHash piv, BarBuf ess, HomOut *o, hipStream_t st);
void launch_hom_iota(int *a, int64_t n, hipStream_t st);
void launch_hom_gather(BarBuf in, const int *perm, int64_t n, BarBuf out, hipStream_t st);

// ---- explicit matrix reduction (rips_explicit.hip)
constexpr int kExpThreads = 256;
constexpr int kExpBuildCap = 4096;        // cofacets <= t of one column
constexpr int64_t kExpMaxAdds = 1 << 24;  // additions per column
constexpr int kExpOk = 0, kExpFull = 1, kExpPool = 2, kExpTable = 3, kExpBound = 4;

// The coboundary matrix of one dimension's columns: column c holds entries
// [off[c], off[c+1]), oldest first.
struct ExpMatrix {
    const int64_t *off;
    int64_t *idx;
    float *diam;
    u32 *coef;
};

struct ExpOut {
    int status; // kExpOk, or what stopped the reduction
    int pad;
    long long bars;      // bars of dimension k (finite and essential)
    long long nonzero;   // columns left nonzero
    long long essential; // essential bars
    long long reduced;   // columns with at least one addition
    long long additions; // column additions
    long long added;     // entries of the added columns
    long long stored;    // entries of the stored reduced columns
    unsigned long long longest; // longest coboundary column (build)
};

struct ExpJob {
    int k;               // columns are k-simplices
    u32 p;
    const u32 *inv;
    const int64_t *cidx; // the columns, younger first
    const float *cdia;
    int64_t ncols;
    ExpMatrix D;
    PivotHash piv;       // pivot -> column position (final)
    PivotHash prev;      // pivots of dimension k-1 (k >= 2)
    const u32 *prev_bits; // forest edges (k = 1)
    int clearing;        // columns that are pivots below were removed
    int64_t *roff;       // per column: its stored R in the pool
    int *rlen;
    int64_t *pidx;       // the pool, oldest first within a column
    float *pdia;
    u32 *pcoef;
    int64_t pcap;
    int64_t *wi[2];      // working column and merge target (global)
    float *wd[2];
    u32 *wc[2];
    int wcap;
    BarBuf bars;
    ExpOut *out;
};

void launch_exp_count(const Ctx<DistFull> &c, int k, const int64_t *cidx, const float *cdia, int64_t S,
                      int64_t *cnt, unsigned long long *longest, hipStream_t st);
void launch_exp_offsets(const int64_t *cnt, int64_t S, int64_t *off, hipStream_t st);
void launch_exp_fill(const Ctx<DistFull> &c, int k, u32 p, const int64_t *cidx, const float *cdia, int64_t S,
                     const int64_t *off, ExpMatrix D, hipStream_t st);
void launch_exp_reduce(const ExpJob &J, hipStream_t st);

constexpr int kRedThreads = 256;

} // namespace rips
