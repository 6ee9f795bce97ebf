// rips_reduce.hpp -- the reduction of the surviving coboundary columns over
// Z/p as a workgroup-level device routine (Algorithm 1 on the implicit
// coboundary matrix of one dimension, columns already cleared; the emergent
// shortcut; pivot lookup = pivot table, then zero apparent facet). Used by
// the single-cloud kernel and by the batched persistent kernel.
//
// Stored columns (the implicit representation of the paper's reduction
// section): column j keeps V_j, the combination of simplices whose
// coboundaries sum to its reduced column R_j, and re-enumerates those
// coboundaries when R_j is added to a later column. R_j itself is kept as
// well when it is cheaper to add than to recompute.
//
// The working column R_j is split at a diameter bound kd:
//  - near part (diameter <= kd): a delta D in LDS (open addressing keyed by
//    simplex index, with the list of used slots; every near addition goes
//    here) plus a sorted base S in global memory (age ascending: diameter
//    ascending, then index descending) read from a front pointer f;
//  - far part (diameter > kd): an unsorted append-only list F in global
//    memory; repeated keys are combined only when they are pulled in.
// The pivot of R_j is its oldest entry with a nonzero coefficient, so it is
// in the near part whenever the near part has a live entry. During the
// reduction of one column the pivot only moves to younger rows (an addition
// cancels the pivot and brings in younger entries only), so entries of S
// before f are dead for good. Maintenance:
//  - D holds more than an eighth of its slots: its live entries are sorted
//    in LDS and merged into S;
//  - S holds more than capD live entries: kd drops to the diameter in the
//    middle of S and the tail moves to F;
//  - the near part has no live entry: kd rises (a diameter histogram of F
//    picks the bound) and the entries under it move from F into D.
// Each entry is thus touched O(1) times in the far list and the near part
// stays small, whatever the size of the column.
#pragma once

#include "rips_kernels.hpp"

namespace rips {

// Open-addressing table keyed by simplex index, with the list of its used
// slots (so that scans, clearing and compaction cost O(entries touched)).
// Coefficients accumulate with atomics and are reduced mod p when read (XOR
// for p = 2). WorkCol lives in global memory (the V table), LdsCol in LDS
// (the delta); the routines below are templates over both.
struct WorkCol {
    int64_t *keys;
    u32 *coef;
    float *diam;
    u32 *slots;
    LDS int *nslots;
    u32 mask;
};

struct LdsCol {
    LDS int64_t *keys;
    LDS u32 *coef;
    LDS float *diam;
    LDS u32 *slots;
    LDS int *nslots;
    u32 mask;
};

// Merge staging in LDS (capacity = a quarter of the delta's slots).
struct Staging {
    LDS int64_t *idx;
    LDS float *dia;
    LDS u32 *coef;
    LDS u32 *cnt; // cap + 1
    LDS int *nd;  // cap + 1
    int cap;
};

// Sorted base in LDS: entries [f, len) of cap, age ascending. A merge stages
// the live part in registers (at most kSPer entries per thread) and writes
// the result back in place.
struct SortedBase {
    LDS int64_t *idx;
    LDS float *dia;
    LDS u32 *coef;
    int cap;
};

constexpr int kSPer = 10;        // base entries per thread during a merge
constexpr u32 kMaxDelta = 2048;  // largest delta: its base (1.25x) fits kSPer x 256 threads
constexpr int kPullUnroll = 8;   // far-list entries in flight per thread in a pull

// Far list in global memory, two buffers of cap entries each.
struct FarList {
    int64_t *idx[2];
    float *dia[2];
    u32 *coef[2];
    int64_t cap;
};

// Global scratch of one workgroup's reduction as the host allocates it and
// passes it to the kernel. It holds no LDS pointer: those are 32 bits wide on
// the device and 64 on the host, so a kernel argument holding one would be
// laid out differently on the two sides.
struct ReduceBuffers {
    FarList F;
    int64_t *vw_keys; // working V column (table used when V_j is too large for LDS)
    u32 *vw_coef;
    float *vw_diam;
    u32 *vw_slots;
    int64_t vw_cap;   // power of two
    // log of one column's additions: key -2 - o = "V_o of column o", key >= 0
    // = "the simplex with that index"; coefficient; diameter (simplices)
    int64_t *lkey;
    u32 *lcoef;
    float *ldia;
    int64_t lcap;
};

// The device view of a workgroup's scratch: the sorted base (LDS), the far
// list, the working V column (its slot count in LDS) and the addition log.
struct ReduceScratch {
    SortedBase SB;
    FarList F;
    WorkCol Vw;
    int64_t *lkey;
    u32 *lcoef;
    float *ldia;
    int64_t lcap;
};

__device__ __forceinline__ ReduceScratch make_scratch(const ReduceBuffers &b, SortedBase sb,
                                                      LDS int *vw_nslots) {
    ReduceScratch sc;
    sc.SB = sb;
    sc.F = b.F;
    sc.Vw = WorkCol{b.vw_keys, b.vw_coef, b.vw_diam, b.vw_slots, vw_nslots, (u32)b.vw_cap - 1};
    sc.lkey = b.lkey;
    sc.lcoef = b.lcoef;
    sc.ldia = b.ldia;
    sc.lcap = b.lcap;
    return sc;
}

// The shortcuts of the reduction, each of which leaves the barcode as it is
// (an ablation switch per shortcut): pivots in zero apparent pairs added from
// their facet rho without a column of their own ("Apparent pairs"; the filter
// then also skips the columns of such pairs), and the emergent pair of a
// column whose oldest cofacet nobody owns ("Emergent persistence pairs").
constexpr int kShortApparent = 1;
constexpr int kShortEmergent = 2;
// Clearing ("Clearing inessential birth columns"): a simplex that is a pivot
// of the dimension below gets no column. Without it that column reduces to
// zero and is not an essential class.
constexpr int kShortClearing = 4;
// When a death column's reduced column R_j is stored beside V_j (the
// "storing R" and "discarding R" rows of Table 3): when it is cheaper to add
// than V_j's coboundaries are to recompute, never, or whenever it has no far
// part
constexpr int kRStoreAuto = 0, kRStoreNever = 1, kRStoreAlways = 2;
// (the single-cloud path's explicit matrix reduction: no implicit reduction runs)
constexpr int kRStoreExplicit = 3;

// Additions one column may take before the reduction reports an error: every
// addition moves the pivot to a strictly younger row, so the loop ends; the
// bound only turns a fault into an error. The addition log (one entry per
// addition) grows on demand up to it.
constexpr int kMaxAdditions = 1 << 24;

// Result codes of the reduction.
enum : int {
    kRedOk = 0,
    kRedBaseFull = 1,  // sorted base or delta full (cannot happen: sizes are bounded)
    kRedStoreFull = 2, // column store too small
    kRedBound = 3,     // addition bound reached
    kRedFarFull = 4,   // far list too small
    kRedVFull = 5,     // working V table too small
    kRedLogFull = 6,   // addition log too small
    kRedAbort = 7,     // another workgroup of the launch failed
    kRedWait = 8,      // a wait for the columns before exceeded its bound
    kRedNoPull = 9,    // a pull of the far part moved nothing (cannot happen)
    kRedOrder = 10,    // a column after j owns a pivot j looks up (cannot happen)
    kRedRefill = 11,   // the middle level came out of a refill empty (cannot happen)
    kRedNoTable = 12,  // apparent shortcut without the filter's pair table (cannot happen)
};

// Bound of one wait in the spread-out reduction, in wall-clock ticks
// (100 MHz): far above any wait a correct run has, it only turns a fault
// into an error.
constexpr unsigned long long kWaitTicks = 1000000000ull;

// LDS bytes of a delta of capD slots, its merge staging (capD / 4 entries)
// and the sorted base (capD + capD / 4 entries).
__host__ __device__ constexpr size_t reduce_lds_bytes(u32 capD) {
    return (size_t)capD * 20 + (size_t)(capD / 4) * 16 + 2 * ((size_t)(capD / 4) + 1) * 4 +
           (size_t)(capD + capD / 4) * 16;
}

// Carve the delta, its staging and the sorted base out of an LDS block
// (capD a power of two, 256 <= capD <= kMaxDelta).
__device__ __forceinline__ void carve_reduce_lds(unsigned char *smem, u32 capD, LDS int *nslots,
                                                 LdsCol *D, Staging *G, SortedBase *SB) {
    LDS unsigned char *q = (LDS unsigned char *)smem;
    const size_t c = capD, m = capD / 4, sc = capD + capD / 4;
    D->keys = (LDS int64_t *)q;
    q += c * 8;
    G->idx = (LDS int64_t *)q;
    q += m * 8;
    SB->idx = (LDS int64_t *)q;
    q += sc * 8;
    D->coef = (LDS u32 *)q;
    q += c * 4;
    D->diam = (LDS float *)q;
    q += c * 4;
    D->slots = (LDS u32 *)q;
    q += c * 4;
    G->dia = (LDS float *)q;
    q += m * 4;
    G->coef = (LDS u32 *)q;
    q += m * 4;
    SB->dia = (LDS float *)q;
    q += sc * 4;
    SB->coef = (LDS u32 *)q;
    q += sc * 4;
    G->cnt = (LDS u32 *)q;
    q += (m + 1) * 4;
    G->nd = (LDS int *)q;
    G->cap = (int)m;
    SB->cap = (int)sc;
    D->nslots = nslots;
    D->mask = capD - 1;
}

template <class T>
__device__ __forceinline__ bool wc_add(const T &h, int64_t key, float dm, u32 c, u32 p) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = ld(&h.keys[s]);
        bool mine = cur == key;
        if (!mine && cur == kEmpty) {
            int64_t expected = kEmpty;
            if (__hip_atomic_compare_exchange_strong(&h.keys[s], &expected, key, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
                h.diam[s] = dm;
                const int q = __hip_atomic_fetch_add(h.nslots, 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
                if ((u32)q <= h.mask) h.slots[q] = s;
                mine = true;
            } else mine = expected == key;
        }
        if (mine) {
            if (p == 2)
                __hip_atomic_fetch_xor(&h.coef[s], c & 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_add(&h.coef[s], c, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            return true;
        }
        s = (s + 1) & h.mask;
    }
    return false;
}

// slot holding key, or -1
template <class T>
__device__ __forceinline__ int wc_find(const T &h, int64_t key) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = ld(&h.keys[s]);
        if (cur == key) return (int)s;
        if (cur == kEmpty) return -1;
        s = (s + 1) & h.mask;
    }
    return -1;
}

// one of two buffers, selected without indexing an array (which would put
// the pointer pair in scratch memory)
template <class T>
__device__ __forceinline__ T *pick(T *const (&a)[2], int b) {
    return b ? a[1] : a[0];
}

// Entry order: older first = (diameter ascending, index descending).
__device__ __forceinline__ bool older_key(float da, int64_t ia, float db, int64_t ib) {
    return da < db || (da == db && ia > ib);
}

// Everything the routine needs about one dimension of one cloud.
// State shared by the workgroups of a reduction spread over a launch. Each
// workgroup takes the next column in order and reduces it against the pivot
// table as it stands. Pivots only move to younger rows while a column is
// reduced (every addition clears the pivot and adds entries younger than it),
// so a column whose current pivot has a larger diameter than tau can never
// end with tau. A column whose pivot tau is free therefore waits until every
// column before it is committed or has its pivot past tau's diameter, looks
// tau up once more, and then either adds the owner's column or commits:
// every pair is the one the column-by-column order gives.
constexpr u32 kColDone = 0xffffffffu;
enum : int { kCtlNext = 0, kCtlFront = 1, kCtlAbort = 2, kCtlWords = 4 };
struct ParState {
    u32 *cst; // per column: float bits of a lower bound of its final pivot's diameter
              // (0 before it starts), kColDone once committed
    u32 *ctl; // kCtlWords words: column cursor, frontier (columns below it are
              // committed; only raised), abort flag
};

// The edges <= t in order of length, for the direct-mapped working column of
// dimension 1 (rips_reduce_bm.hpp): pos[a * n + b] = pos[b * n + a] = the
// position of the edge {a, b} (-1 for an edge longer than t; a row is
// contiguous in its second vertex, so the positions of the edges {a, w} of
// all w load together), position -> vertices (a << 16 | b, a > b) and length.
// E == 0: not in use.
struct EdgeOrder {
    const int *pos;
    const u32 *verts;
    const float *len;
    const u32 *run; // position -> first position of its run of equal lengths,
                    // with kRunTie set when the next position has the same length
    const int *app; // position -> the third vertex c of the edge's zero apparent
                    // cofacet (the edge and {a, b, c} are a zero apparent pair), or -1
    int E;
    int W; // 32-bit words of one edge's bitmap: ceil(n / 32)
    int n; // points: the row length of pos
};
constexpr u32 kRunTie = 0x80000000u;

// The summary of the direct-mapped working column in LDS: one bit per edge
// position (l1, n1 words) and one per first-level word (l2, n2 words).
struct BmLds {
    LDS u32 *l1;
    LDS u32 *l2;
    int n1, n2, E;
};

__host__ __device__ constexpr size_t bm_lds_bytes(int64_t E) {
    return E <= 0 ? 0 : (size_t)(((E + 31) / 32) + ((E + 1023) / 1024)) * 4;
}

// Carve the summary after `at` bytes of the block and clear it (all threads).
__device__ __forceinline__ BmLds carve_bm_lds(unsigned char *smem, size_t at, int E) {
    BmLds L;
    L.E = E;
    L.n1 = (E + 31) / 32;
    L.n2 = (L.n1 + 31) / 32;
    L.l1 = (LDS u32 *)((LDS unsigned char *)smem + at);
    L.l2 = L.l1 + L.n1;
    for (int i = threadIdx.x; i < L.n1 + L.n2; i += blockDim.x) L.l1[i] = 0u;
    __syncthreads();
    return L;
}

template <class Dist>
struct ReduceJob {
    Ctx<Dist> c;
    int k;
    u32 p;
    const u32 *inv;
    Columns cols;
    int ncols;
    PivotHash ph;
    VStore V;
    unsigned long long *vcount; // column-store append counter (global)
    BarBuf bars;                // capacity ncols
    float cand_avg;             // mean coboundary candidates of a k-simplex
    PairHash app;               // zero apparent pairs (rho, tau) of this dimension, or none
    ParState par;               // reduction spread over workgroups (cst null: one workgroup)
    int shortcuts;              // kShortApparent | kShortEmergent | kShortClearing: those in use
    int keep_essential_v;       // also store V_j of zero columns (their cocycles)
    int rstore;                 // kRStoreAuto, kRStoreNever or kRStoreAlways: when R_j is kept
#if RIPS_COLUMN_TRACE
    unsigned long long *trace;  // per column: pick and commit clock, additions, clock spent waiting
#endif
    // the pivots of the dimension below (read only without clearing): forest
    // edges of H0 as bits (k = 1), else that dimension's pivot table
    const u32 *prev_bits;
    PivotHash prev;
    // direct-mapped working column (dimension 1, Z/2, every shortcut on):
    // bm_bits == null means the general working column is used
    EdgeOrder eo = {nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
    u32 *bm_bits = nullptr; // eo.E * eo.W words per workgroup, all zero between columns
    int64_t bm_stride = 0;  // words per workgroup (workgroup blockIdx.x uses its own)
};

constexpr int kRedTimers = 24;

// Shared state of the routine (one per workgroup).
template <int BT>
struct RedShared {
    int base, full, abort, m, nbars, cur, merged, nit, vns, refine;
    int nlog, gen;
    int64_t vest;
    int fw, fwn;    // far list: buffer appended to, entries in it
    int fr, nr, pn; // far list being pulled: buffer, entries; entries pulled
    // middle level of the far part: the top quarter of each far buffer holds
    // the far entries of diameter bits <= mb (when mon), the rest the others
    int mw, mwn, mon;
    u32 mb;
    int pcount, nr2; // far_bound: entries at or under the bound; running count
    float kd;       // near part = entries older than (kd, kidx)
    int64_t kidx;
    int64_t len, f; // sorted base: length and front
    int64_t owner, qsplit, appv;
    int64_t tau;    // spread-out reduction: emergent candidate
    u32 tcoef, pub; // its coefficient; diameter bits published for this column
    int wbad, wopen, wstop;
#if RIPS_COLUMN_TRACE
    unsigned long long wacc;
#endif
    int fa_n, fa_r; // apparent steps of wave 0: additions made, result
    int bmf;        // direct-mapped working column: front position of the pivot search
    u32 lo, bound;
    int shift;
    unsigned long long vbase;
    PivotCand wp[BT / kWave];
    PivotCand piv, spiv;
    int w[BT / kWave + 1];
    u32 mm[2][BT / kWave];
    unsigned long long stat[13];
    unsigned long long tm[kRedTimers]; // wall-clock ticks: pivot, add, merge, pull, split, store, setup, apparent, emergent, reset, total, owner; merge: gather, rank, base pass, prefix; apparent addition, wait, apparent run; its pivot search, table lookup, coboundary
    u32 hist[256];
    // simplices whose coboundaries are added next: vertices, coefficient,
    // diameter, candidate source (vertex with the fewest neighbours, -1 =
    // all vertices) and prefix offsets of their candidate counts
    int it_v[BT][kMaxDim + 1];
    u32 it_coef[BT];
    float it_diam[BT];
    int it_u[BT];
    int it_start[BT]; // first candidate of the item in the neighbour list
    int it_off[BT + 1];
};

// Phase timers (thread 0, wall clock), compiled in only with
// RIPS_PHASE_TIMERS=1: reading the clock waits for the wave's outstanding
// LDS and scalar loads, which costs about 5 % of the reduction's time.
#ifndef RIPS_PHASE_TIMERS
#define RIPS_PHASE_TIMERS 0
#endif
#if RIPS_PHASE_TIMERS
#define RED_T0(v) const unsigned long long v = threadIdx.x == 0 ? wall_clock64() : 0ull
#define RED_T1(S, i, v)                                                                            \
    do {                                                                                           \
        if (threadIdx.x == 0) (S).tm[i] += wall_clock64() - v;                                     \
    } while (0)
// the same for any thread (cond), accumulated atomically
#define RED_TW0(v, cond) const unsigned long long v = (cond) ? wall_clock64() : 0ull
#define RED_TW1(S, i, v, cond)                                                                     \
    do {                                                                                           \
        if (cond) atomicAdd(&(S).tm[i], wall_clock64() - v);                                       \
    } while (0)
#else
#define RED_TW0(v, cond) const unsigned long long v = 0ull
#define RED_TW1(S, i, v, cond)                                                                     \
    do {                                                                                           \
        (void)(v);                                                                                 \
    } while (0)
#define RED_T0(v) const unsigned long long v = 0ull
#define RED_T1(S, i, v)                                                                            \
    do {                                                                                           \
        (void)(v);                                                                                 \
    } while (0)
#endif

template <int BT>
__device__ __forceinline__ int block_scan_excl(int x, int *s_w, int *total) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int inc = wave_scan_incl(x);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int q = 0; q < BT / kWave; ++q) {
            int t = s_w[q];
            s_w[q] = acc;
            acc += t;
        }
        s_w[BT / kWave] = acc;
    }
    __syncthreads();
    const int r = s_w[w] + inc - x;
    *total = s_w[BT / kWave];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// tables (all threads of the block)
// ---------------------------------------------------------------------------
template <int BT, class T>
__device__ __forceinline__ void wc_reset(const T &h) {
    const int ns = min(*h.nslots, (int)h.mask + 1);
    for (int i = threadIdx.x; i < ns; i += BT) {
        const u32 s = h.slots[i];
        st(&h.keys[s], kEmpty);
        st(&h.coef[s], 0u);
    }
    gsync();
    if (threadIdx.x == 0) *h.nslots = 0;
    __syncthreads();
}

template <int BT, class T>
__device__ __forceinline__ void wc_clear_all(const T &h) {
    for (u32 q = threadIdx.x; q <= h.mask; q += BT) {
        st(&h.keys[q], kEmpty);
        st(&h.coef[q], 0u);
    }
    gsync();
    if (threadIdx.x == 0) *h.nslots = 0;
    __syncthreads();
}

// Oldest live entry of the delta (block-wide). Coefficients are normalised
// mod p on the way (no addition runs concurrently).
template <int BT>
__device__ __forceinline__ PivotCand wc_oldest(const LdsCol &R, u32 p, RedShared<BT> &S) {
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    PivotCand best;
    best.idx = kEmpty;
    best.diam = 0.0f;
    best.coef = 0;
    const int ns = min(*R.nslots, (int)R.mask + 1);
    for (int i = tid; i < ns; i += BT) {
        const u32 s = R.slots[i];
        u32 cf = ld(&R.coef[s]);
        if (p != 2 && cf >= p) {
            cf %= p;
            st(&R.coef[s], cf);
        }
        if (cf == 0) continue;
        PivotCand x;
        x.idx = ld(&R.keys[s]);
        x.diam = R.diam[s];
        x.coef = cf;
        if (older(x, best)) best = x;
    }
    best = wave_oldest(best);
    if (lane == 0) S.wp[w] = best;
    __syncthreads();
    if (tid == 0) {
        PivotCand b = S.wp[0];
        for (int q = 1; q < BT / kWave; ++q)
            if (older(S.wp[q], b)) b = S.wp[q];
        S.piv = b;
    }
    __syncthreads();
    return S.piv;
}

// Is (dm, key) in the near part, i.e. older than the boundary (kd, kidx)?
template <int BT>
__device__ __forceinline__ bool is_near(const RedShared<BT> &S, float dm, int64_t key) {
    return older_key(dm, key, S.kd, S.kidx);
}

// The far part has two levels in each of its two buffers: the bottom holds
// the far list proper, the top quarter (from far_mbase) a middle level with
// every far entry of diameter bits <= mb while it is in use. A pull then
// scans the middle level only; when that runs empty, one pass over the far
// list moves its oldest entries up. Buffers too small for a middle level
// keep the far list alone.
__device__ __forceinline__ int64_t far_mcap(const FarList &F) {
    return F.cap >= (int64_t)16 * kMaxDelta ? F.cap / 4 : 0;
}

// One wave's appends with pred to one level: one atomic per wave. Positions
// at or past lim fail.
__device__ __forceinline__ bool far_level_append(const FarList &F, int *count, int buf, int64_t base,
                                                 int64_t lim, bool pred, int64_t key, float dm, u32 c) {
    const u64 m = __ballot(pred);
    if (!m) return true;
    const int lane = lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    int at = 0;
    if (lane == leader) at = atomicAdd(count, __popcll(m));
    at = lane_bcast(at, leader);
    if (!pred) return true;
    const int64_t pos = at + __popcll(m & ((1ull << lane) - 1ull));
    if (pos >= lim) return false;
    pick(F.idx, buf)[base + pos] = key;
    pick(F.dia, buf)[base + pos] = dm;
    pick(F.coef, buf)[base + pos] = c;
    return true;
}

// Append the lanes' entries with pred to the far part, each to its level.
// Every lane of the wave must call it. Returns false on the lanes whose
// entry did not fit.
template <int BT>
__device__ __forceinline__ bool far_append_w(const FarList &F, RedShared<BT> &S, bool pred,
                                             int64_t key, float dm, u32 c) {
    const int64_t mcap = far_mcap(F);
    const bool mid = pred && S.mon && __float_as_uint(dm) <= S.mb;
    // the far list stays below the middle level; the middle level keeps a
    // segment of slack at its top for the entries a pull reads from there
    const bool a = far_level_append(F, &S.fwn, S.fw, 0, F.cap - mcap, pred && !mid, key, dm, c);
    const bool b = far_level_append(F, &S.mwn, S.mw, F.cap - mcap, mcap - kMaxDelta / 8, mid, key, dm,
                                    c);
    return a && b;
}

// Add the lanes' entries (act) to the working column: near -> delta, far ->
// far list. Every lane of the wave must call it. Returns 0 or a result code.
template <int BT>
__device__ __forceinline__ int add_entry_w(const LdsCol &D, const FarList &F, RedShared<BT> &S,
                                           bool act, int64_t key, float dm, u32 c, u32 p) {
    const bool near = act && is_near(S, dm, key);
    int r = kRedOk;
    if (near && !wc_add(D, key, dm, c, p)) r = kRedBaseFull;
    if (!far_append_w<BT>(F, S, act && !near, key, dm, c)) r = kRedFarFull;
    return r;
}

// ---------------------------------------------------------------------------
// sorted base
// ---------------------------------------------------------------------------

// Wave 0 moves the front of S past entries whose total coefficient (S + D)
// is zero; the delta's copies of those keys are zeroed, since their part of
// the sum is spent. S.spiv = the first live entry with its total, if any.
template <int BT, class Dist>
__device__ __forceinline__ PivotCand base_advance(const ReduceJob<Dist> &J, const LdsCol &D,
                                                  const SortedBase &SB, u32 p, RedShared<BT> &S) {
    (void)J;
    PivotCand out;
    out.idx = kEmpty;
    out.diam = 0.0f;
    out.coef = 0;
    if (threadIdx.x >= kWave) return out;
    wave_sync(); // S.f: lane 0 may have moved it, in this wave's own run
    const int lane = lane_id();
    int64_t f = S.f;
    const int64_t len = S.len;
    while (f < len) {
        const int64_t q = f + lane;
        const bool valid = q < len;
        u32 total = 0;
        int slot = -1;
        int64_t id = 0;
        float dm = 0.0f;
        if (valid) {
            id = SB.idx[q];
            dm = SB.dia[q];
            slot = wc_find(D, id);
            const u32 cd = slot >= 0 ? ld(&D.coef[slot]) % p : 0u;
            total = (SB.coef[q] + cd) % p;
        }
        const u64 live = __ballot(valid && total != 0);
        const int first = live ? __ffsll((unsigned long long)live) - 1 : kWave;
        if (valid && lane < first && slot >= 0) st(&D.coef[slot], 0u);
        if (live) {
            out.idx = lane_bcast(id, first);
            out.diam = lane_bcast(dm, first);
            out.coef = lane_bcast(total, first);
            f += first;
            break;
        }
        f += kWave;
    }
    if (f > len) f = len;
    if (lane == 0) {
        S.f = f;
        S.spiv = out;
    }
    return out; // the same in every lane of wave 0
}

// Merge the live entries of D into S[f, len) (all threads); D is empty
// afterwards and S starts at 0. Returns 0 or a result code.
template <int BT>
__device__ __forceinline__ int base_merge(const LdsCol &D, const Staging &G, const SortedBase &SB, u32 p,
                          RedShared<BT> &S) {
    static_assert(kSPer * BT >= (int)(kMaxDelta + kMaxDelta / 4), "base does not fit the staging");
    RED_T0(t_mrg);
    const int tid = threadIdx.x;
    const int ns = min(*D.nslots, (int)D.mask + 1);
    RED_T0(t_m1);
    // 1. gather the live entries into the staging area, unsorted
    int cnt = 0;
    for (int i = tid; i < ns; i += BT) cnt += (ld(&D.coef[D.slots[i]]) % p) != 0 ? 1 : 0;
    int m;
    int at = block_scan_excl<BT>(cnt, S.w, &m);
    const int f = (int)S.f, sl = (int)(S.len - S.f);
    if (m > G.cap || sl + m > SB.cap) return kRedBaseFull; // bounded by construction
    for (int i = tid; i < ns; i += BT) {
        const u32 s = D.slots[i];
        const u32 cf = ld(&D.coef[s]) % p;
        if (cf != 0) {
            G.idx[at] = ld(&D.keys[s]);
            G.dia[at] = D.diam[s];
            G.coef[at] = cf;
            ++at;
        }
    }
    __syncthreads();
    RED_T1(S, 12, t_m1);
    RED_T0(t_m2);
    // 2. sort into M = D's first m slots (keys are distinct): every wave
    // sorts 64-entry chunks of the staging area in place with a bitonic
    // network over shuffles; an entry's rank is then its place in its chunk
    // plus, for every other chunk, how many of its entries are older
    LDS int64_t *Mi = D.keys;
    LDS float *Md = D.diam;
    LDS u32 *Mc = D.coef;
    {
        const int lane = lane_id(), w = tid / kWave;
        const int nc = (m + kWave - 1) / kWave;
        for (int ch = w; ch < nc; ch += BT / kWave) {
            const int e = ch * kWave + lane;
            const bool real = e < m;
            float d = real ? G.dia[e] : INFINITY;
            int64_t id = real ? G.idx[e] : (int64_t)-1;
            u32 cf = real ? G.coef[e] : 0u;
            for (int kk = 2; kk <= kWave; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    const float pd = __shfl_xor(d, jj, kWave);
                    const int64_t pi = __shfl_xor(id, jj, kWave);
                    const u32 pc = (u32)__shfl_xor((int)cf, jj, kWave);
                    const bool up = (lane & kk) == 0;
                    const bool lower = (lane & jj) == 0;
                    const bool p_older = older_key(pd, pi, d, id);
                    if (lower == up ? p_older : (!p_older && (pd != d || pi != id))) {
                        d = pd;
                        id = pi;
                        cf = pc;
                    }
                }
            }
            if (real) {
                G.dia[e] = d;
                G.idx[e] = id;
                G.coef[e] = cf;
            }
        }
        __syncthreads();
        for (int e = tid; e < m; e += BT) {
            const int ch = e / kWave;
            const float de = G.dia[e];
            const int64_t ie = G.idx[e];
            int r = e - ch * kWave;
            for (int c2 = 0; c2 < nc; ++c2) {
                if (c2 == ch) continue;
                int lo = c2 * kWave, hi = min(m, lo + kWave); // first entry not older
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (older_key(G.dia[mid], G.idx[mid], de, ie)) lo = mid + 1;
                    else hi = mid;
                }
                r += lo - c2 * kWave;
            }
            Mi[r] = ie;
            Md[r] = de;
            Mc[r] = G.coef[e];
        }
    }
    for (int i = tid; i <= m; i += BT) G.cnt[i] = 0;
    __syncthreads();
    RED_T1(S, 13, t_m2);
    RED_T0(t_m3);
    // 3. every base entry into registers with its lower bound in M (first
    // entry not older than it); counts; duplicate flag (bit 31 of M's
    // coefficient)
    int64_t rid[kSPer];
    float rdm[kSPer];
    u32 rcf[kSPer];
    int rlo[kSPer];
#pragma unroll
    for (int i = 0; i < kSPer; ++i) {
        const int r = tid + i * BT;
        rlo[i] = -1;
        rid[i] = 0;
        rdm[i] = 0.0f;
        rcf[i] = 0;
        if (r < sl) {
            rid[i] = SB.idx[f + r];
            rdm[i] = SB.dia[f + r];
            rcf[i] = SB.coef[f + r];
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (older_key(Md[mid], Mi[mid], rdm[i], rid[i])) lo = mid + 1;
                else hi = mid;
            }
            rlo[i] = lo;
            __hip_atomic_fetch_add(&G.cnt[lo], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lo < m && Mi[lo] == rid[i])
                __hip_atomic_fetch_or(&Mc[lo], 0x80000000u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    RED_T1(S, 14, t_m3);
    RED_T0(t_m4);
    // 4. inclusive prefix of the counts (base entries older than M[i] for a
    // non-duplicate i), exclusive prefix of the non-duplicates
    int carry_c = 0, carry_n = 0;
    for (int b0 = 0; b0 <= m; b0 += BT) {
        const int i = b0 + tid;
        const int c = i <= m ? (int)G.cnt[i] : 0;
        const int nd = i < m ? ((Mc[i] & 0x80000000u) ? 0 : 1) : 0;
        int tc, tn;
        const int ec = block_scan_excl<BT>(c, S.w, &tc);
        const int en = block_scan_excl<BT>(nd, S.w, &tn);
        if (i <= m) {
            G.cnt[i] = (u32)(carry_c + ec + c);
            G.nd[i] = carry_n + en;
        }
        carry_c += tc;
        carry_n += tn;
    }
    __syncthreads();
    RED_T1(S, 15, t_m4);
    // 5. write in place (every base entry was read in step 3): base entry r
    // goes to r + (non-duplicates before its lower bound); non-duplicate M[i]
    // goes to (base entries older) + (non-duplicates before it)
#pragma unroll
    for (int i = 0; i < kSPer; ++i) {
        const int r = tid + i * BT;
        if (r < sl) {
            const int lo = rlo[i];
            u32 cf = rcf[i];
            if (lo < m && Mi[lo] == rid[i]) cf = (cf + (Mc[lo] & 0x7fffffffu)) % p;
            const int dst = r + G.nd[lo];
            SB.idx[dst] = rid[i];
            SB.dia[dst] = rdm[i];
            SB.coef[dst] = cf;
        }
    }
    for (int i = tid; i < m; i += BT) {
        const u32 cf = Mc[i];
        if (cf & 0x80000000u) continue;
        const int dst = (int)G.cnt[i] + G.nd[i];
        SB.idx[dst] = Mi[i];
        SB.dia[dst] = Md[i];
        SB.coef[dst] = cf;
    }
    const int nondup = carry_n;
    __syncthreads();
    if (tid == 0) {
        S.f = 0;
        S.len = sl + nondup;
        S.merged = 1;
        S.gen += 1;
        S.stat[9] += 1;
    }
    wc_clear_all<BT>(D);
    RED_T1(S, 2, t_mrg);
    return kRedOk;
}

// S longer than smax live entries: lower kd to the diameter in the middle
// of S and move the entries above it to the far list (D is empty here).
template <int BT>
__device__ __forceinline__ int base_split(const SortedBase &SB, const FarList &F, u32 p, int smax,
                                          RedShared<BT> &S) {
    const int tid = threadIdx.x;
    if (S.len - S.f <= smax) return kRedOk;
    RED_T0(t_spl);
    // the entry in the middle becomes the boundary: it and everything
    // younger move to the far list (the key includes the index, so blocks of
    // equal diameters split too)
    const int q = (int)S.f + smax / 2, len = (int)S.len;
    const float kd = SB.dia[q];
    const int64_t kidx = SB.idx[q];
    bool ok = true;
    for (int b0 = q; b0 < len; b0 += BT) {
        const int r = b0 + tid;
        const bool act = r < len;
        const u32 cf = act ? SB.coef[r] % p : 0u;
        ok = far_append_w<BT>(F, S, cf != 0, act ? SB.idx[r] : 0, act ? SB.dia[r] : 0.0f, cf) && ok;
    }
    if (!ok) S.abort = kRedFarFull;
    gsync();
    if (S.abort) return S.abort;
    if (tid == 0) {
        S.len = q;
        S.kd = kd;
        S.kidx = kidx;
        S.merged = 1;
        S.gen += 1;
        S.stat[10] += 1;
    }
    __syncthreads();
    RED_T1(S, 4, t_spl);
    return kRedOk;
}

// Rehash D's live entries in place when there are at most `most` of them
// (all threads; most <= G.cap). Returns the number of live entries; D is
// unchanged when that is above `most`.
template <int BT>
__device__ __forceinline__ int delta_compact(const LdsCol &D, const Staging &G, u32 p, int most,
                             RedShared<BT> &S) {
    const int tid = threadIdx.x;
    const int ns = min(*D.nslots, (int)D.mask + 1);
    int cnt = 0;
    for (int i = tid; i < ns; i += BT) cnt += (ld(&D.coef[D.slots[i]]) % p) != 0 ? 1 : 0;
    int m;
    int at = block_scan_excl<BT>(cnt, S.w, &m);
    if (m > most) return m;
    for (int i = tid; i < ns; i += BT) {
        const u32 s = D.slots[i];
        const u32 cf = ld(&D.coef[s]) % p;
        if (cf != 0) {
            G.idx[at] = ld(&D.keys[s]);
            G.dia[at] = D.diam[s];
            G.coef[at] = cf;
            ++at;
        }
    }
    __syncthreads();
    for (int i = tid; i < ns; i += BT) {
        const u32 s = D.slots[i];
        st(&D.keys[s], kEmpty);
        st(&D.coef[s], 0u);
    }
    __syncthreads();
    if (tid == 0) *D.nslots = 0;
    __syncthreads();
    for (int e = tid; e < m; e += BT) wc_add(D, G.idx[e], G.dia[e], G.coef[e], p);
    __syncthreads();
    return m;
}

// keep D at most an eighth full (compacting it when few of its entries are
// live, else merging it into S) and S at most capD live entries
template <int BT>
__device__ __forceinline__ int delta_check(const LdsCol &D, const Staging &G,
                                           const ReduceScratch &SC, u32 p, RedShared<BT> &S) {
    const int capD = (int)D.mask + 1;
    if (*D.nslots <= capD / 8) return kRedOk;
    {
        RED_T0(t_cmp);
        const int live = delta_compact<BT>(D, G, p, capD / 32, S);
        RED_T1(S, 2, t_cmp);
        if (live <= capD / 32) return kRedOk;
    }
    int r = base_merge<BT>(D, G, SC.SB, p, S);
    if (r) return r;
    return base_split<BT>(SC.SB, SC.F, p, capD, S);
}

// Bound of a histogram over the diameter bit patterns (non-negative floats
// order like their bits) of n far entries fd[0, n), over [lo, hi]: the
// smallest bin top with about `target` entries at or under it, refined while
// the chosen bin alone holds more than `factor` times the target. Sets
// S.bound (capped at cap_bits) and S.pcount, the entries at or under it.
template <int BT>
__device__ __forceinline__ void far_bound(const float *fd, int n, u32 lo, u32 hi, u32 cap_bits,
                                          int target, int factor, RedShared<BT> &S) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        const u32 span = max(lo, hi) - lo;
        const int nb = span ? 32 - __clz(span) : 0;
        S.lo = lo;
        S.shift = nb > 8 ? nb - 8 : 0;
        S.refine = 1;
    }
    __syncthreads();
    int below = 0; // entries under S.lo (all taken)
    while (S.refine) {
        for (int i = tid; i < 256; i += BT) S.hist[i] = 0;
        __syncthreads();
        const u32 l = S.lo;
        const int sh = S.shift;
        // kPullUnroll independent loads in flight per thread
        for (int b0 = 0; b0 < n; b0 += kPullUnroll * BT) {
            u32 bb[kPullUnroll];
#pragma unroll
            for (int u = 0; u < kPullUnroll; ++u) {
                const int r = b0 + u * BT + tid;
                bb[u] = r < n ? __float_as_uint(fd[r]) : 0xffffffffu;
            }
#pragma unroll
            for (int u = 0; u < kPullUnroll; ++u) {
                if (bb[u] == 0xffffffffu || bb[u] < l) continue;
                const u32 bin = (bb[u] - l) >> sh;
                atomicAdd(&S.hist[bin < 256 ? bin : 255], 1u);
            }
        }
        __syncthreads();
        if (tid == 0) {
            int cum = below, i = 0;
            for (; i < 256; ++i) {
                cum += (int)S.hist[i];
                if (cum >= target) break;
            }
            if (i == 256) i = 255;
            const int before = cum - (int)S.hist[i];
            if (cum > factor * target && sh > 0 && S.hist[i] > 1) {
                // bin i alone is far too full: split it
                S.lo = l + ((u32)i << sh);
                S.shift = sh > 8 ? sh - 8 : 0;
                S.nr2 = before; // the running count below lo
            } else {
                // the last bin takes everything up to cap_bits (+inf for the
                // far list: its bits bound every finite diameter, and a larger
                // pattern would be a NaN boundary, which nothing is older than)
                const u64 top = i == 255 ? (u64)cap_bits : (u64)l + ((u64)(i + 1) << sh) - 1;
                S.bound = (u32)(top > (u64)cap_bits ? (u64)cap_bits : top);
                // entries in bin 255 above cap_bits cannot exist: every source
                // holds entries at or under its cap only
                S.pcount = cum;
                S.refine = 0;
            }
        }
        __syncthreads();
        below = S.refine ? S.nr2 : below;
        __syncthreads();
    }
}

// Pull from n entries at src (buffer sb, from offset so): raise the boundary
// to S.bound, move the entries at or under it to the top of buffer db and
// append the rest to the far part (far_append_w puts each in its level),
// then feed the moved ones into the delta in segments. `room` is the space
// the top of db may take (a segment of slack included).
template <int BT>
__device__ __forceinline__ int far_pull_core(const LdsCol &D, const Staging &G, const ReduceScratch &SC,
                                             u32 p, int sb, int64_t so, int n, int db, int64_t room,
                                             RedShared<BT> &S) {
    const FarList &F = SC.F;
    const int tid = threadIdx.x;
    if ((int64_t)n + ((int)D.mask + 1) / 8 > room) return kRedFarFull;
    if (tid == 0) {
        // new boundary (d, -1): every entry of diameter <= d is near
        S.kd = __uint_as_float(S.bound);
        S.kidx = -1;
        S.pn = 0;
    }
    __syncthreads();
    // partition without barriers: entries under the bound go to the top of
    // buffer db (slot cap - 1 - i for the i-th), the rest to the far part
    const u32 bound = S.bound;
    bool ok = true;
    const int64_t *fi = pick(F.idx, sb) + so;
    const float *fd = pick(F.dia, sb) + so;
    const u32 *fc = pick(F.coef, sb) + so;
    for (int b0 = 0; b0 < n; b0 += kPullUnroll * BT) {
        int64_t ids[kPullUnroll];
        float dms[kPullUnroll];
        u32 cfs[kPullUnroll];
#pragma unroll
        for (int u = 0; u < kPullUnroll; ++u) {
            const int r = b0 + u * BT + tid;
            const bool act = r < n;
            ids[u] = act ? fi[r] : 0;
            dms[u] = act ? fd[r] : 0.0f;
            cfs[u] = act ? fc[r] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPullUnroll; ++u) {
            const int r = b0 + u * BT + tid;
            const bool act = r < n;
            const bool pull = act && __float_as_uint(dms[u]) <= bound;
            ok = far_append_w<BT>(F, S, act && !pull, ids[u], dms[u], cfs[u]) && ok;
            const u64 m = __ballot(pull);
            if (m) {
                const int lane = lane_id();
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&S.pn, __popcll(m));
                base = lane_bcast(base, leader);
                if (pull) {
                    const int64_t pos = F.cap - 1 - (base + __popcll(m & ((1ull << lane) - 1ull)));
                    pick(F.idx, db)[pos] = ids[u];
                    pick(F.dia, db)[pos] = dms[u];
                    pick(F.coef, db)[pos] = cfs[u];
                }
            }
        }
    }
    if (!ok) S.abort = kRedFarFull;
    gsync();
    if (S.abort) return S.abort;
    // the pulled entries into D, in segments, read upwards from the lowest
    // slot: whatever a split sends back to the bottom of the level stays
    // below the part not read yet (both come out of the same n entries)
    const int pn = S.pn;
    // the entries of the smallest diameter in the source are under the
    // bound, so a pull always moves some; one that moved none would repeat
    // forever: report it instead. (The near part may still end up empty:
    // copies of one key in the far part can cancel. The caller then pulls
    // again, from a far part that has shrunk.)
    if (pn == 0) return kRedNoPull;
    const int64_t pbase = F.cap - pn;
    const int seg = ((int)D.mask + 1) / 8;
    for (int s0 = 0; s0 < pn; s0 += seg) {
        const int s1 = min(pn, s0 + seg);
        int bad = 0;
        for (int b0 = s0; b0 < s1; b0 += BT) {
            const int e = b0 + tid;
            const bool act = e < s1;
            const int64_t pos = pbase + e;
            const int rr = add_entry_w<BT>(D, F, S, act, act ? pick(F.idx, db)[pos] : 0,
                                           act ? pick(F.dia, db)[pos] : 0.0f,
                                           act ? pick(F.coef, db)[pos] : 0u, p);
            if (rr) bad = rr;
        }
        if (bad) S.abort = bad;
        gsync();
        if (S.abort) return S.abort;
        const int r = delta_check<BT>(D, G, SC, p, S);
        if (r) return r;
    }
    return kRedOk;
}

// The near part is empty and the far part is not: raise the boundary to a
// diameter d such that about `target` far entries have diameter <= d, and
// move those into the delta. From the middle level while it holds entries;
// when it is empty and the far list is long, one pass first moves the far
// list's oldest entries (about sqrt(far list x target) of them) up into it;
// otherwise straight from the far list.
template <int BT>
__device__ __forceinline__ int far_pull(const LdsCol &D, const Staging &G,
                                        const ReduceScratch &SC, u32 p, int target, float tmax,
                                        RedShared<BT> &S) {
    const FarList &F = SC.F;
    const int tid = threadIdx.x;
    const int64_t mcap = far_mcap(F);
    const int64_t mbase = F.cap - mcap;
    RED_T0(t_pull);
    // every thread reads the middle level's count before thread 0 rewrites it
    const int mwn0 = S.mwn;
    __syncthreads();
    if (mwn0 == 0) {
        // middle level empty: the far list's buffers swap
        if (tid == 0) {
            S.fr = S.fw;
            S.nr = S.fwn;
            S.fw = S.fw ^ 1;
            S.fwn = 0;
            S.mon = 0;
            S.merged = 1;
            S.stat[8] += 1;
            S.stat[11] += S.nr;
        }
        __syncthreads();
        const int fr = S.fr, nr = S.nr;
        const u32 lo = __float_as_uint(S.kd);
        const u32 hi = max(lo, __float_as_uint(tmax));
        const int64_t want = (int64_t)sqrtf((float)nr * (float)target);
        bool refilled = false;
        if (mcap > 0 && nr > 8 * target && want > 2 * (int64_t)target) {
            const int tm = (int)min(want, mcap / 4);
            far_bound<BT>(pick(F.dia, fr), nr, lo, hi, 0x7f800000u, tm, 2, S);
            if (S.pcount > 0 && (int64_t)S.pcount <= mcap / 2) {
                // refill: everything goes back to the far part, the entries
                // at or under mb into the middle level (empty before)
                if (tid == 0) {
                    S.mon = 1;
                    S.mb = S.bound;
                    S.mw = 0;
                    S.mwn = 0;
                }
                __syncthreads();
                bool ok = true;
                const int64_t *fi = pick(F.idx, fr);
                const float *fd = pick(F.dia, fr);
                const u32 *fc = pick(F.coef, fr);
                for (int b0 = 0; b0 < nr; b0 += kPullUnroll * BT) {
#pragma unroll
                    for (int u = 0; u < kPullUnroll; ++u) {
                        const int r = b0 + u * BT + tid;
                        const bool act = r < nr;
                        ok = far_append_w<BT>(F, S, act, act ? fi[r] : 0, act ? fd[r] : 0.0f,
                                              act ? fc[r] : 0u) &&
                             ok;
                    }
                }
                if (!ok) S.abort = kRedFarFull;
                gsync();
                if (S.abort) return S.abort;
                // pcount entries are at or under mb: the middle level holds them
                const int got = S.mwn;
                __syncthreads(); // read by every thread before the pull below rewrites it
                if (got == 0) return kRedRefill;
                refilled = true;
            }
        }
        if (!refilled) {
            // straight from the far list (the middle level is off and empty,
            // so the top of the new buffer is free)
            far_bound<BT>(pick(F.dia, fr), nr, lo, hi, 0x7f800000u, target, 8, S);
            RED_T1(S, 3, t_pull);
            return far_pull_core<BT>(D, G, SC, p, fr, 0, nr, S.fw, F.cap, S);
        }
    }
    // from the middle level: its buffers swap; the bound stays at or under mb
    if (tid == 0) {
        S.nr = S.mwn;
        S.fr = S.mw;
        S.mw = S.mw ^ 1;
        S.mwn = 0;
        S.merged = 1;
        S.stat[8] += 1;
        S.stat[11] += S.nr;
    }
    __syncthreads();
    const int mr = S.fr, nm = S.nr;
    const u32 lo = __float_as_uint(S.kd);
    far_bound<BT>(pick(F.dia, mr) + mbase, nm, lo, max(lo, S.mb), S.mb, target, 8, S);
    RED_T1(S, 3, t_pull);
    return far_pull_core<BT>(D, G, SC, p, mr, mbase, nm, S.mw, mcap, S);
}

// ---------------------------------------------------------------------------
// additions
// ---------------------------------------------------------------------------

// Add the coboundaries of the S.nit simplices in S.it_* (each times its
// coefficient) to the working column. The (item, candidate) pairs are spread
// over the workgroup, in segments of an eighth of D with maintenance
// between. Cofacet sigma u {j} gets (-1)^(vertices of sigma below j) times
// the item's coefficient. Dense candidates: all vertices; sparse: the
// neighbours of the item's vertex with the fewest.
template <int BT, class Dist>
__device__ __forceinline__ int add_items(const ReduceJob<Dist> &J, RedShared<BT> &S, const LdsCol &D,
                         const Staging &G, const ReduceScratch &SC) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x;
    const int nit = S.nit;
    int cnt = 0;
    if (tid < nit) {
        if (c.nb.off == nullptr) {
            S.it_u[tid] = -1;
            S.it_start[tid] = 0;
            cnt = c.n;
        } else {
            int u = S.it_v[tid][0];
            int lo = c.nb.off[u];
            int du = c.nb.off[u + 1] - lo;
            for (int m = 1; m <= k; ++m) {
                const int vm = S.it_v[tid][m];
                const int lm = c.nb.off[vm];
                const int dd = c.nb.off[vm + 1] - lm;
                if (dd < du) {
                    du = dd;
                    u = vm;
                    lo = lm;
                }
            }
            S.it_u[tid] = u;
            S.it_start[tid] = lo;
            cnt = du;
        }
    }
    int total;
    if (nit == 1) {
        // one item (an apparent facet, a single simplex): no scan
        if (tid == 0) {
            S.it_off[0] = 0;
            S.it_off[1] = cnt;
        }
        __syncthreads();
        total = S.it_off[1];
    } else {
        const int off = block_scan_excl<BT>(cnt, S.w, &total);
        if (tid < nit) S.it_off[tid] = off;
        if (tid == 0) S.it_off[nit] = total;
        __syncthreads();
    }
    const int seg = ((int)D.mask + 1) / 8;
    for (int s0 = 0; s0 < total; s0 += seg) {
        const int s1 = min(total, s0 + seg);
        int bad = 0;
        unsigned long long added = 0;
        for (int b0 = s0; b0 < s1; b0 += BT) {
            const int fl = b0 + tid;
            bool act = fl < s1;
            int64_t ci = 0;
            float nd = 0.0f;
            u32 cc = 0;
            if (act) {
                int lo = 0, hi = nit - 1; // last item with it_off <= fl
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (S.it_off[mid] <= fl) lo = mid;
                    else hi = mid - 1;
                }
                const int it = lo;
                const int q = fl - S.it_off[it];
                const int u = S.it_u[it];
                const int j = u < 0 ? q : c.nb.idx[S.it_start[it] + q];
                const int *v = S.it_v[it];
                bool in = false;
                nd = S.it_diam[it];
                for (int m = 0; m <= k; ++m) {
                    in = in || (j == v[m]);
                    nd = fmaxf(nd, c.d(v[m], j));
                }
                act = !in && nd <= c.t;
                if (act) {
                    int below;
                    ci = cofacet_index(v, k, j, c.B, &below);
                    const u32 coef = S.it_coef[it];
                    cc = (below & 1) ? (p - coef) % p : coef;
                    ++added;
                }
            }
            const int rr = add_entry_w<BT>(D, SC.F, S, act, ci, nd, cc, p);
            if (rr) bad = rr;
        }
        if (added) atomicAdd(&S.stat[12], added);
        if (bad) S.abort = bad;
        gsync();
        if (S.abort) return S.abort;
        const int r = delta_check<BT>(D, G, SC, p, S);
        if (r) return r;
    }
    __syncthreads(); // the items are read before anyone rewrites them
    return kRedOk;
}

// Add mul times the coboundaries of the simplices of a stored V column.
template <int BT, class Dist>
__device__ __forceinline__ int add_vcolumn(const ReduceJob<Dist> &J, RedShared<BT> &S, const LdsCol &D,
                           const Staging &G, const ReduceScratch &SC, int64_t off, int len,
                           u32 mul) {
    const int tid = threadIdx.x;
    const u32 p = J.p;
    for (int c0 = 0; c0 < len; c0 += BT) {
        const int nit = min(BT, len - c0);
        if (tid < nit) {
            const int64_t e = off + c0 + tid;
            decode(J.V.idx[e], J.k, J.c.n, J.c.B, S.it_v[tid]);
            S.it_diam[tid] = J.V.diam[e];
            S.it_coef[tid] = (u32)((u64)mul * J.V.coef[e] % p);
        }
        if (tid == 0) S.nit = nit;
        __syncthreads();
        const int r = add_items<BT>(J, S, D, G, SC);
        if (r) return r;
    }
    return kRedOk;
}

// Add neg times the stored R column entries [off, off + len), in segments.
template <int BT, class Dist>
__device__ __forceinline__ int add_rcolumn(const ReduceJob<Dist> &J, RedShared<BT> &S, const LdsCol &D,
                           const Staging &G, const ReduceScratch &SC, int64_t off, int len,
                           u32 neg) {
    const u32 p = J.p;
    const int seg = ((int)D.mask + 1) / 8;
    for (int s0 = 0; s0 < len; s0 += seg) {
        const int s1 = min(len, s0 + seg);
        int bad = 0;
        for (int b0 = s0; b0 < s1; b0 += BT) {
            const int e = b0 + threadIdx.x;
            const bool act = e < s1;
            const u32 cc = act ? (u32)((u64)neg * J.V.coef[off + e] % p) : 0u;
            const int rr = add_entry_w<BT>(D, SC.F, S, act, act ? J.V.idx[off + e] : 0,
                                           act ? J.V.diam[off + e] : 0.0f, cc, p);
            if (rr) bad = rr;
        }
        if (threadIdx.x == 0) S.stat[12] += (unsigned long long)(s1 - s0);
        if (bad) S.abort = bad;
        gsync();
        if (S.abort) return S.abort;
        const int r = delta_check<BT>(D, G, SC, p, S);
        if (r) return r;
    }
    return kRedOk;
}

// Append the live entries of a table (V_j) or of the sorted base to the
// column store; returns the count, or -1 when the store is full.
template <int BT, class Tb>
__device__ __forceinline__ int store_table(const Tb &T, const VStore &V, unsigned long long *vcount, u32 p,
                           RedShared<BT> &S, int64_t *off_out) {
    const int tid = threadIdx.x;
    const int ns = min(*T.nslots, (int)T.mask + 1);
    int cnt = 0;
    for (int i = tid; i < ns; i += BT) cnt += (ld(&T.coef[T.slots[i]]) % p) != 0 ? 1 : 0;
    int tot;
    int at = block_scan_excl<BT>(cnt, S.w, &tot);
    if (tid == 0) S.vbase = atomicAdd(vcount, (unsigned long long)tot);
    __syncthreads();
    const int64_t vb = (int64_t)S.vbase;
    if (vb + tot > V.cap) return -1;
    for (int i = tid; i < ns; i += BT) {
        const u32 s = T.slots[i];
        const u32 cf = ld(&T.coef[s]) % p;
        if (cf != 0) {
            V.idx[vb + at] = ld(&T.keys[s]);
            V.diam[vb + at] = T.diam[s];
            V.coef[vb + at] = cf;
            ++at;
        }
    }
    *off_out = vb;
    return tot;
}

template <int BT>
__device__ __forceinline__ int store_base(const SortedBase &SB, const VStore &V, unsigned long long *vcount,
                          u32 p, RedShared<BT> &S, int64_t *off_out) {
    const int tid = threadIdx.x;
    const int64_t f0 = S.f, nsrc = S.len - S.f;
    int cnt = 0;
    for (int64_t i = tid; i < nsrc; i += BT) cnt += (SB.coef[f0 + i] % p) != 0 ? 1 : 0;
    int tot;
    int at = block_scan_excl<BT>(cnt, S.w, &tot);
    if (tid == 0) S.vbase = atomicAdd(vcount, (unsigned long long)tot);
    __syncthreads();
    const int64_t vb = (int64_t)S.vbase;
    if (vb + tot > V.cap) return -1;
    for (int64_t i = tid; i < nsrc; i += BT) {
        const u32 cf = SB.coef[f0 + i] % p;
        if (cf != 0) {
            V.idx[vb + at] = SB.idx[f0 + i];
            V.diam[vb + at] = SB.dia[f0 + i];
            V.coef[vb + at] = cf;
            ++at;
        }
    }
    *off_out = vb;
    return tot;
}

// live entries of the working column's near part (D merged into S first
// when S is in use); -1 on failure
template <int BT, class Tb>
__device__ __forceinline__ int count_live(const Tb &T, u32 p, RedShared<BT> &S) {
    const int ns = min(*T.nslots, (int)T.mask + 1);
    int cnt = 0;
    for (int i = threadIdx.x; i < ns; i += BT) cnt += (ld(&T.coef[T.slots[i]]) % p) != 0 ? 1 : 0;
    int tot;
    (void)block_scan_excl<BT>(cnt, S.w, &tot);
    return tot;
}

template <int BT>
__device__ __forceinline__ int64_t count_live_base(const SortedBase &SB, u32 p, RedShared<BT> &S) {
    int cnt = 0;
    for (int64_t i = S.f + threadIdx.x; i < S.len; i += BT) cnt += (SB.coef[i] % p) != 0;
    int tot;
    (void)block_scan_excl<BT>(cnt, S.w, &tot);
    return tot;
}

// Append one addition to the column's log (thread 0). False when full.
template <int BT>
__device__ __forceinline__ bool log_add(const ReduceScratch &SC, RedShared<BT> &S, int64_t key,
                                        u32 coef, float dm, int64_t vlen) {
    if ((int64_t)S.nlog >= SC.lcap) return false;
    SC.lkey[S.nlog] = key;
    SC.lcoef[S.nlog] = coef;
    SC.ldia[S.nlog] = dm;
    S.nlog += 1;
    S.vest += vlen;
    return true;
}

// V_j = sigma_j + the logged combination, summed into table T (all threads).
// Returns false when T overflowed (T is then in an unspecified state).
template <int BT, class Dist, class Tb>
__device__ __forceinline__ bool materialize_v(const ReduceJob<Dist> &J, const ReduceScratch &SC, const Tb &T,
                              int64_t sidx, float sdm, RedShared<BT> &S) {
    const u32 p = J.p;
    bool ok = true;
    if (threadIdx.x == 0) ok = wc_add(T, sidx, sdm, 1u, p);
    const int nl = S.nlog;
    for (int e = threadIdx.x; e < nl; e += BT) {
        const int64_t key = SC.lkey[e];
        const u32 cf = SC.lcoef[e];
        if (key >= 0) {
            ok = ok && wc_add(T, key, SC.ldia[e], cf, p);
            continue;
        }
        const int o = (int)(-2 - key);
        const int vlen = J.V.len[o];
        if (vlen < 0) {
            ok = ok && wc_add(T, J.cols.idx[o], J.cols.diam[o], cf, p);
        } else {
            const int64_t vo = J.V.off[o];
            for (int q = 0; q < vlen && ok; ++q)
                ok = wc_add(T, J.V.idx[vo + q], J.V.diam[vo + q],
                            (u32)((u64)cf * J.V.coef[vo + q] % p), p);
        }
    }
    if (!ok) S.abort = 1;
    gsync();
    const bool res = S.abort == 0;
    __syncthreads();
    if (threadIdx.x == 0) S.abort = 0;
    __syncthreads();
    return res;
}

// Steps of the reduction of column j taken by wave 0 alone, without
// workgroup barriers, while the pivot tau lies in a zero apparent pair
// (rho, tau) recorded by the filter: R_j -= lambda coboundary(rho), the same
// addition the general step makes there (such a tau is never in the pivot
// table). It stops, leaving the pivot to the general step, at a pivot that
// is not such a tau, at an empty near part, at a coboundary that does not
// fit the delta before its next maintenance, once that maintenance is due,
// or after `budget` additions. Returns the additions made (the same in every
// lane); *res gets 0 or a result code.
constexpr int kRunScan = 4; // delta slots an apparent run scans, in units of a wave

template <int BT, class Dist, bool kPar>
__device__ __forceinline__ int apparent_run(const ReduceJob<Dist> &J, const LdsCol &D,
                                            const ReduceScratch &SC, int j, int budget,
                                            RedShared<BT> &S, int *res) {
    // values, not references into the job: read once per run and kept in
    // registers (the job itself lives in scratch memory)
    const Ctx<Dist> c = J.c;
    const PairHash app = J.app;
    const int k = J.k;
    const u32 p = J.p;
    const u32 *inv = J.inv;
    const FarList F = SC.F;
    const SortedBase SB = SC.SB;
    const int lane = lane_id();
    const int capD = (int)D.mask + 1;
    int nadd = 0;
    *res = kRedOk;
    while (nadd < budget) {
        // the last step's additions (other lanes' slots, diameters, counts)
        wave_sync();
        const int ns0 = min(*D.nslots, capD);
        if (ns0 > capD / 8) break; // maintenance due
        RED_T0(t_r0);
        const PivotCand smin = base_advance<BT>(J, D, SB, p, S);
        PivotCand best;
        best.idx = kEmpty;
        best.diam = 0.0f;
        best.coef = 0;
        const int ns = min(*D.nslots, capD);
        if (ns <= kRunScan * kWave) {
            // at most capD / 8 <= 256 slots here: every load is issued at
            // once, two LDS round trips in all instead of three per 64
            // slots. Lanes past ns read list entry 0, which may never have
            // been written: the mask keeps that slot inside the table, and
            // the lane's result is dropped.
            u32 sl[kRunScan];
#pragma unroll
            for (int r = 0; r < kRunScan; ++r) {
                const int i = lane + r * kWave;
                sl[r] = D.slots[i < ns ? i : 0] & D.mask;
            }
            u32 cfs[kRunScan];
            int64_t kys[kRunScan];
            float dgs[kRunScan];
#pragma unroll
            for (int r = 0; r < kRunScan; ++r) {
                cfs[r] = ld(&D.coef[sl[r]]);
                kys[r] = ld(&D.keys[sl[r]]);
                dgs[r] = D.diam[sl[r]];
            }
#pragma unroll
            for (int r = 0; r < kRunScan; ++r) {
                if (lane + r * kWave >= ns) continue;
                u32 cf = cfs[r];
                if (p != 2 && cf >= p) {
                    cf %= p;
                    st(&D.coef[sl[r]], cf);
                }
                if (cf == 0) continue;
                PivotCand x;
                x.idx = kys[r];
                x.diam = dgs[r];
                x.coef = cf;
                if (older(x, best)) best = x;
            }
        } else {
            for (int i = lane; i < ns; i += kWave) {
                const u32 sl = D.slots[i];
                u32 cf = ld(&D.coef[sl]);
                if (p != 2 && cf >= p) {
                    cf %= p;
                    st(&D.coef[sl], cf);
                }
                if (cf == 0) continue;
                PivotCand x;
                x.idx = ld(&D.keys[sl]);
                x.diam = D.diam[sl];
                x.coef = cf;
                if (older(x, best)) best = x;
            }
        }
        const PivotCand dmin = wave_oldest(best);
        const bool from_base = smin.idx != kEmpty &&
                               (dmin.idx == kEmpty || dmin.idx == smin.idx || !older(dmin, smin));
        const PivotCand piv = from_base ? smin : dmin;
        if (piv.idx == kEmpty) break;
        if (kPar && lane == 0 && __float_as_uint(piv.diam) > S.pub) {
            S.pub = __float_as_uint(piv.diam);
            st_dev(&J.par.cst[j], S.pub);
        }
        RED_T1(S, 19, t_r0);
        RED_T0(t_r1);
        PairHit hit{-1, kNoVerts, 0, kNoList};
        if (lane == 0) hit = pair_find_all(app, piv.idx);
        const int64_t a = lane_bcast(hit.val, 0);
        RED_T1(S, 20, t_r1);
        if (a < 0) break;
        RED_T0(t_r2);
        const u64 vw = lane_bcast(hit.verts, 0);
        const u64 nbw = lane_bcast(hit.nbr, 0);
        const u64 cbw = lane_bcast(hit.cob, 0);
        // rho's vertices, and the candidate source: the neighbour list of its
        // vertex with the fewest neighbours (all vertices when dense), both
        // from the table slot
        int rv[kMaxVerts];
        if (vw != kNoVerts) {
            for (int q = 0; q <= k; ++q) rv[q] = (int)((vw >> (16 * q)) & 0xffffu);
        } else {
            decode(a >> 3, k, c.n, c.B, rv);
        }
        const int u = c.nb.off == nullptr ? -1 : 0;
        // rho's coboundary: its list from the table when there is one, else
        // the candidates of its shortest neighbour list
        const bool listed = cbw != kNoList;
        const int64_t loff = listed ? (int64_t)(cbw >> 24) : 0;
        const int lo = u < 0 ? 0 : (int)(nbw >> 32);
        const int du = listed ? (int)(cbw & 0xffffffu) : (u < 0 ? c.n : (int)(u32)nbw);
        if (ns + du > capD / 4) break; // more than the delta takes before its maintenance
        // tau = rho u {tau[m]}; vertices of rho below tau[m]: k + 1 - m
        const int m = (int)(a & 7);
        const u32 lam = p == 2 ? 1u : (u32)((u64)piv.coef * inv[coeff_sign(k + 1 - m, p)] % p);
        const u32 neg = (p - lam) % p;
        int bad = 0;
        if (lane == 0 && !log_add(SC, S, a >> 3, neg, piv.diam, 1)) bad = kRedLogFull;
        int added = 0;
        for (int q0 = 0; q0 < du; q0 += kWave) {
            const int q = q0 + lane;
            bool act = q < du;
            int64_t ci = 0;
            float nd = 0.0f;
            u32 cc = 0;
            if (act && listed) {
                const int64_t key = app.ckey[loff + q];
                ci = key & kCobIdx;
                nd = app.cdia[loff + q];
                cc = (key >> 62) ? (p - neg) % p : neg;
            } else if (act) {
                const int jv = u < 0 ? q : c.nb.idx[lo + q];
                bool in = false;
                nd = piv.diam;
                for (int mm = 0; mm <= k; ++mm) {
                    in = in || (jv == rv[mm]);
                    nd = fmaxf(nd, c.d(rv[mm], jv));
                }
                act = !in && nd <= c.t;
                if (act) {
                    int below;
                    ci = cofacet_index(rv, k, jv, c.B, &below);
                    cc = (below & 1) ? (p - neg) % p : neg;
                }
            }
            added += __popcll(__ballot(act));
            const int rr = add_entry_w<BT>(D, F, S, act, ci, nd, cc, p);
            if (rr) bad = rr;
        }
        if (lane == 0) S.stat[12] += (unsigned long long)added;
        RED_T1(S, 21, t_r2);
        ++nadd;
        // a failure in any lane ends the run
        const u64 fail = __ballot(bad != 0);
        if (fail) {
            *res = lane_bcast(bad, __ffsll((unsigned long long)fail) - 1);
            break;
        }
    }
    return nadd;
}

// Block-wide minimum of two values (all threads; every thread gets both).
template <int BT>
__device__ __forceinline__ void block_min2(int &a, int &b, RedShared<BT> &S) {
    // both are column positions (>= 0): unsigned minima
    a = (int)wave_min_u32((u32)a);
    b = (int)wave_min_u32((u32)b);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        S.mm[0][w] = (u32)a;
        S.mm[1][w] = (u32)b;
    }
    __syncthreads();
    for (int q = 0; q < BT / kWave; ++q) {
        a = min(a, (int)S.mm[0][q]);
        b = min(b, (int)S.mm[1][q]);
    }
    __syncthreads();
}

// Spread-out reduction: wait until no column before j can still end with a
// pivot of diameter bits <= dbits, i.e. each one is committed or its current
// pivot is past that diameter (a column's published bound only grows).
// Returns 0, or kRedAbort / kRedWait (all threads get the same answer).
// (The column words come by value: a job struct whose address reached this
// out-of-line call would be copied to scratch memory, and every read of it
// in the caller would become a scratch load.)
template <int BT>
__device__ int par_wait(const ParState par, RedShared<BT> &S, int j, u32 dbits) {
    const int tid = threadIdx.x;
    u32 *ctl = par.ctl;
    if (tid == 0) S.wbad = (int)ld_dev(&ctl[kCtlFront]);
    __syncthreads();
    int from = min(S.wbad, j);
    const unsigned long long t0 = tid == 0 ? wall_clock64() : 0ull;
#if RIPS_COLUMN_TRACE
    struct WaitClock {
        RedShared<BT> &S;
        unsigned long long t0;
        int tid;
        __device__ ~WaitClock() {
            if (tid == 0) S.wacc += wall_clock64() - t0;
        }
    } wclock{S, t0, tid};
#endif
    for (bool first = true;; first = false) {
        int bad = j, open = j;
        for (int o = from + tid; o < j; o += BT) {
            const u32 st = ld_dev(&par.cst[o]);
            if (st != kColDone) open = min(open, o);
            if (st <= dbits) bad = min(bad, o);
        }
        block_min2<BT>(bad, open, S);
        // the frontier may move up only past columns this scan saw committed
        if (tid == 0 && first && open > from) atomicMax(&ctl[kCtlFront], (u32)open);
        if (bad == j) break;
        // the columns in [from, bad) stay past dbits: scan from bad next time
        from = bad;
        if (tid == 0) {
            S.wstop = 0;
            if (ld_dev(&ctl[kCtlAbort])) S.wstop = kRedAbort;
            else if (wall_clock64() - t0 > kWaitTicks) S.wstop = kRedWait;
        }
        __syncthreads();
        const int stop = S.wstop;
        __syncthreads();
        if (stop) return stop;
        __builtin_amdgcn_s_sleep(8);
    }
    return 0;
}

// V_j = sigma_j + the logged combination, summed (in D's LDS slots when it
// fits comfortably, else in the global table) and appended to the column
// store. Returns its length, or minus a result code (all threads).
template <int BT, class Dist>
__device__ __forceinline__ int store_v(const ReduceJob<Dist> &J, const LdsCol &D, const ReduceScratch &SC,
                                      int64_t sidx, float sdm, RedShared<BT> &S, int64_t *voff) {
    wc_reset<BT>(D);
    const bool try_lds = S.vest <= (int64_t)(D.mask + 1) / 2;
    const bool used_lds = try_lds && materialize_v<BT>(J, SC, D, sidx, sdm, S);
    if (!used_lds) {
        if (try_lds) wc_clear_all<BT>(D); // the failed attempt left D unspecified
        if (!materialize_v<BT>(J, SC, SC.Vw, sidx, sdm, S)) {
            wc_clear_all<BT>(SC.Vw);
            return -kRedVFull;
        }
    }
    const int vn = used_lds ? store_table<BT>(D, J.V, J.vcount, J.p, S, voff)
                            : store_table<BT>(SC.Vw, J.V, J.vcount, J.p, S, voff);
    if (!used_lds) wc_reset<BT>(SC.Vw);
    return vn < 0 ? -kRedStoreFull : vn;
}

// Full reduction of column j. Returns a result code; on anything but kRedOk
// nothing of column j has been published.
//
// V_j is not kept up to date at every addition: the additions are logged
// (column o with its factor, or an apparent facet rho) and V_j is summed
// once, when the column pairs.
template <int BT, class Dist, bool kPar>
__device__ __forceinline__ int reduce_one(const ReduceJob<Dist> &J, const LdsCol &D, const Staging &G,
                          const ReduceScratch &SC, int j, RedShared<BT> &S) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const int64_t sidx = J.cols.idx[j];
    const float sdm = J.cols.diam[j];
    RED_T0(t_setup);
    if (tid == 0) {
        S.abort = 0;
        S.len = 0;
        S.f = 0;
        S.merged = 0;
        S.kd = INFINITY;
        S.kidx = -1;
        S.fw = 0;
        S.fwn = 0;
        S.mw = 0;
        S.mwn = 0;
        S.mon = 0;
        S.mb = 0;
        S.nlog = 0;
        S.vest = 1;
        S.nit = 1;
        S.it_coef[0] = 1u;
        S.it_diam[0] = sdm;
        decode(sidx, k, c.n, c.B, S.it_v[0]);
        if (kPar) {
            // every cofacet of sigma is at least as old as sigma
            S.pub = __float_as_uint(sdm);
            st_dev(&J.par.cst[j], S.pub);
        }
    }
    __syncthreads();
    int result = add_items<BT>(J, S, D, G, SC);
    RED_T1(S, 6, t_setup);
    int nadd = 0;
    while (result == kRedOk) {
        __syncthreads();
        // every addition moves the pivot to a strictly younger row, so the
        // loop ends; the bound only turns a fault into an error
        if (nadd > kMaxAdditions) {
            result = kRedBound;
            break;
        }
        if (J.app.keys != nullptr) {
            // the run of pivots in zero apparent pairs, by wave 0 alone
            RED_T0(t_fast);
            if (w == 0) {
                int r;
                const int na = apparent_run<BT, Dist, kPar>(J, D, SC, j, kMaxAdditions + 1 - nadd, S, &r);
                if (lane == 0) {
                    S.fa_n = na;
                    S.fa_r = r;
                }
            }
            __syncthreads();
            const int na = S.fa_n;
            result = S.fa_r;
            RED_T1(S, 18, t_fast);
            if (result) break;
            nadd += na;
            if (na > 0) {
                result = delta_check<BT>(D, G, SC, p, S);
                if (result) break;
                __syncthreads();
            }
        }
        PivotCand piv;
        bool from_base = false;
        RED_T0(t_piv);
        for (;;) {
            base_advance<BT>(J, D, SC.SB, p, S);
            __syncthreads();
            const PivotCand dmin = wc_oldest<BT>(D, p, S);
            const PivotCand smin = S.spiv;
            from_base = smin.idx != kEmpty &&
                        (dmin.idx == kEmpty || dmin.idx == smin.idx || !older(dmin, smin));
            piv = from_base ? smin : dmin;
            if (piv.idx != kEmpty || (S.fwn == 0 && S.mwn == 0)) break;
            result = far_pull<BT>(D, G, SC, p, ((int)D.mask + 1) / 2, c.t, S);
            if (result) break;
        }
        RED_T1(S, 0, t_piv);
        if (result) break;
        if (piv.idx == kEmpty) {
            // zero column: essential class born at sigma (final as it is:
            // nothing is left to look up); its cocycle V_j is stored only
            // when asked for. Without clearing, the zero column of a pivot
            // of the dimension below is no class at all.
            const bool lower = !(J.shortcuts & kShortClearing) &&
                               (k == 1 ? ((J.prev_bits[sidx >> 5] >> (sidx & 31)) & 1u) != 0
                                       : ph_find(J.prev, sidx) >= 0);
            int64_t voff = 0;
            int vn = -1;
            if (J.keep_essential_v && !lower) {
                __syncthreads();
                vn = store_v<BT>(J, D, SC, sidx, sdm, S, &voff);
                if (vn < 0) {
                    result = -vn;
                    break;
                }
            }
            if (kPar) {
                if (tid == 0) {
                    J.bars.birth[j] = sdm;
                    J.bars.death[j] = INFINITY;
                    J.bars.bs[j] = lower ? -1 : sidx; // -1: no bar
                    J.bars.ds[j] = -1;
                    if (!lower) S.stat[4] += 1;
                    if (J.keep_essential_v) {
                        J.V.off[j] = voff;
                        J.V.len[j] = vn;
                    }
                }
                fence_release_dev();
                __syncthreads();
                if (tid == 0) st_dev(&J.par.cst[j], kColDone);
            } else if (tid == 0 && !lower) {
                if (S.nbars < J.ncols) {
                    J.bars.birth[S.nbars] = sdm;
                    J.bars.death[S.nbars] = INFINITY;
                    J.bars.bs[S.nbars] = sidx;
                    J.bars.ds[S.nbars] = -1;
                    S.nbars++;
                }
                S.stat[4] += 1;
                if (J.keep_essential_v) {
                    J.V.off[j] = voff;
                    J.V.len[j] = vn;
                }
            }
            break;
        }
        if (kPar && tid == 0 && __float_as_uint(piv.diam) > S.pub) {
            S.pub = __float_as_uint(piv.diam);
            st_dev(&J.par.cst[j], S.pub);
        }
        RED_T0(t_own);
        // pivot table and apparent-pair table, read by two waves at once
        // (spread out: a cached copy can only miss an entry, and a miss is
        // checked again below after the wait)
        if (tid == 0) S.owner = ph_find(J.ph, piv.idx);
        if (tid == kWave) S.appv = J.app.keys ? pair_find(J.app, piv.idx) : -1;
        __syncthreads();
        if (kPar && S.owner < 0 && S.appv < 0) {
            // free pivot: final once no column before can still take it
            RED_T0(t_w);
            result = par_wait<BT>(J.par, S, j, __float_as_uint(piv.diam));
            RED_T1(S, 17, t_w);
            if (result) break;
            if (tid == 0) S.owner = ph_find_dev(J.ph, piv.idx);
            __syncthreads();
        }
        RED_T1(S, 11, t_own);
        const int64_t o = S.owner;
        if (kPar && o >= j) {
            result = kRedOrder; // only a column before j can own a pivot j looks up
            break;
        }
        if (kPar && o >= 0) fence_acquire_dev(); // the owner's published column
        if (o >= 0) {
            // R_j -= lambda R_o (and V_j -= lambda V_o), lambda = piv / pivot(R_o)
            // over Z/2 every nonzero entry is 1: no lookup
            const u32 lam = p == 2 ? 1u : (u32)((u64)piv.coef * J.V.pivcoef[o] % p);
            const u32 neg = (p - lam) % p;
            const int vlen = J.V.len[o];
            const int rlen = J.V.rlen[o];
            if (tid == 0 && !log_add(SC, S, -2 - o, neg, 0.0f, vlen < 0 ? 1 : vlen))
                S.abort = kRedLogFull;
            RED_T0(t_add);
            if (rlen >= 0) {
                result = add_rcolumn<BT>(J, S, D, G, SC, J.V.roff[o], rlen, neg);
            } else if (vlen < 0) {
                // emergent column: R_o is the coboundary of sigma_o
                if (tid == 0) {
                    S.nit = 1;
                    S.it_coef[0] = neg;
                    S.it_diam[0] = J.cols.diam[o];
                    decode(J.cols.idx[o], k, c.n, c.B, S.it_v[0]);
                }
                __syncthreads();
                result = add_items<BT>(J, S, D, G, SC);
            } else {
                result = add_vcolumn<BT>(J, S, D, G, SC, J.V.off[o], vlen, neg);
            }
            RED_T1(S, 1, t_add);
            __syncthreads();
            if (result == kRedOk && S.abort) result = S.abort;
            ++nadd;
            continue;
        }
        // not in the table: is the pivot in a zero apparent pair (rho, tau)?
        RED_T0(t_app);
        if (J.app.keys) {
            // recorded by the filter: tau -> (rho, position m of the added vertex)
            if (tid == 0) {
                const int64_t a = S.appv;
                S.m = a < 0 ? -1 : (int)(a & 7);
                if (a >= 0) {
                    const int m = (int)(a & 7);
                    decode(a >> 3, k, c.n, c.B, S.it_v[0]);
                    // tau = rho u {tau[m]}; vertices of rho below tau[m]: k + 1 - m
                    const u32 crho = coeff_sign(k + 1 - m, p);
                    const u32 lam = (u32)((u64)piv.coef * J.inv[crho] % p);
                    S.nit = 1;
                    S.it_coef[0] = (p - lam) % p;
                    S.it_diam[0] = piv.diam;
                    if (!log_add(SC, S, a >> 3, (p - lam) % p, piv.diam, 1)) S.abort = kRedLogFull;
                }
            }
        } else if (!(J.shortcuts & kShortApparent)) {
            if (tid == 0) S.m = -1; // no apparent shortcut: the pivot is free
        } else if (tid == 0) {
            // every caller that keeps the shortcut passes the filter's table
            S.m = -1;
            S.abort = kRedNoTable;
        }
        __syncthreads();
        RED_T1(S, 7, t_app);
        if (S.abort) {
            result = S.abort;
            break;
        }
        if (S.m >= 0) {
            RED_T0(t_aa);
            result = add_items<BT>(J, S, D, G, SC);
            RED_T1(S, 16, t_aa);
            ++nadd;
            continue;
        }
        // unowned pivot: persistence pair (sigma_j, pivot). R_j is stored
        // when it has no far part and is cheaper to add than V_j's
        // coboundaries are to recompute (|V_j| estimated from the log); then
        // V_j is summed from the log and stored.
        RED_T0(t_st);
        int64_t roff = 0;
        int rn = -1;
        if (S.fwn == 0 && S.mwn == 0 && J.rstore != kRStoreNever) {
            if (S.len > 0 && *D.nslots > 0) {
                result = base_merge<BT>(D, G, SC.SB, p, S);
                if (result) break;
            }
            __syncthreads();
            const bool rb = S.len > 0;
            const int64_t live = rb ? count_live_base<BT>(SC.SB, p, S)
                                    : (int64_t)count_live<BT>(D, p, S);
            const bool keep_r = J.rstore == kRStoreAlways ||
                                (J.rstore == kRStoreAuto && (float)live <= 2.0f * (float)S.vest * J.cand_avg);
            if (keep_r) {
                rn = rb ? store_base<BT>(SC.SB, J.V, J.vcount, p, S, &roff)
                        : store_table<BT>(D, J.V, J.vcount, p, S, &roff);
                if (rn < 0) {
                    result = kRedStoreFull;
                    break;
                }
            }
        }
        __syncthreads();
        int64_t voff = 0;
        const int vn = store_v<BT>(J, D, SC, sidx, sdm, S, &voff);
        if (vn < 0) {
            result = -vn;
            break;
        }
        if (kPar) {
            // publish V_j, R_j and the bar, then the table entry, then "done"
            if (tid == 0) {
                if ((unsigned long long)vn > S.stat[6]) S.stat[6] = vn;
                J.bars.birth[j] = sdm;
                J.bars.death[j] = piv.diam;
                J.bars.bs[j] = piv.diam > sdm ? sidx : -1; // -1: no bar
                J.bars.ds[j] = piv.idx;
                if (piv.diam > sdm) S.stat[3] += 1;
                J.V.pivcoef[j] = J.inv[piv.coef];
                J.V.off[j] = voff;
                J.V.len[j] = vn;
                J.V.roff[j] = roff;
                J.V.rlen[j] = rn;
            }
            fence_release_dev();
            __syncthreads();
            if (tid == 0) {
                ph_insert_dev(J.ph, piv.idx, j);
                fence_release_dev();
                st_dev(&J.par.cst[j], kColDone);
            }
        } else if (tid == 0) {
            if ((unsigned long long)vn > S.stat[6]) S.stat[6] = vn;
            if (piv.diam > sdm) {
                if (S.nbars < J.ncols) {
                    J.bars.birth[S.nbars] = sdm;
                    J.bars.death[S.nbars] = piv.diam;
                    J.bars.bs[S.nbars] = sidx;
                    J.bars.ds[S.nbars] = piv.idx;
                    S.nbars++;
                }
                S.stat[3] += 1;
            }
            ph_insert(J.ph, piv.idx, j);
            J.V.pivcoef[j] = J.inv[piv.coef];
            J.V.off[j] = voff;
            J.V.len[j] = vn;
            J.V.roff[j] = roff;
            J.V.rlen[j] = rn;
        }
        RED_T1(S, 5, t_st);
        break;
    }
    if (tid == 0) {
        if (result == kRedOk) {
            S.stat[1] += nadd > 0 ? 1 : 0;
            S.stat[2] += nadd;
            if (S.merged) S.stat[5] += 1;
        }
        const unsigned long long sz = (unsigned long long)(S.len - S.f + S.fwn + S.mwn + *D.nslots);
        if (sz > S.stat[7]) S.stat[7] = sz;
    }
    __syncthreads();
    RED_T0(t_rst);
    wc_reset<BT>(D);
    RED_T1(S, 9, t_rst);
    return result;
}

// The reduction of J.ncols columns by one workgroup of BT threads, with the
// delta D (and its staging G) in LDS and the rest of the working column in
// global scratch. Returns a result code. Stats: S.stat = emergent, reduced,
// additions, bars_nonzero, essential, columns that used the sorted base or
// far list, largest stored V column, largest working column.
} // namespace rips

#include "rips_reduce_bm.hpp"

namespace rips {

template <int BT, class Dist>
__device__ __forceinline__ int reduce_columns(const ReduceJob<Dist> &J, const LdsCol &D, const Staging &G,
                              const ReduceScratch &SC, const BmLds &L, RedShared<BT> &S) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    wc_clear_all<BT>(D);
    wc_clear_all<BT>(SC.Vw);
    if (tid == 0) {
        S.base = 0;
        S.abort = 0;
        S.nbars = 0;
        S.len = 0;
        S.f = 0;
        S.gen = 0;
    }
    if (tid < 13) S.stat[tid] = 0;
    if (tid < kRedTimers) S.tm[tid] = 0;
    int status = 0;
    gsync();
    RED_T0(t_total);
    for (;;) {
        __syncthreads();
        const int base = S.base;
        const int stop = base >= J.ncols;
        __syncthreads(); // everyone has read the cursor before wave 0 moves it
        if (stop || status) break;
        RED_T0(t_em);
        // ---- emergent shortcut for up to 64 columns at once (wave 0): a
        // column whose zero pivot cofacet is free (not in the pivot table,
        // not in a zero apparent pair, not taken by a lower column of the
        // batch) pairs with it; the batch stops at the first other column
        if (w == 0) {
            const int col = base + lane;
            const bool valid = col < J.ncols;
            bool ok = false;
            int64_t tau = kEmpty;
            u32 tcoef = 0;
            // no probe at all when the first column cannot be emergent (no
            // zero pivot cofacet, or that cofacet is in an apparent pair)
            const bool cand = (J.shortcuts & kShortEmergent) && valid && J.cols.j[col] >= 0 &&
                              !J.cols.tapp[col];
            if (lane_bcast((int)cand, 0)) {
                const int j = J.cols.j[col];
                if (cand) {
                    int v[kMaxVerts];
                    decode(J.cols.idx[col], k, c.n, c.B, v);
                    int below;
                    tau = cofacet_index(v, k, j, c.B, &below);
                    tcoef = coeff_sign(below, p);
                    ok = ph_find(J.ph, tau) < 0;
                }
            }
            for (int l = 0; l < kWave - 1; ++l) {
                const int64_t tl = lane_bcast(tau, l);
                const int okl = lane_bcast((int)ok, l);
                if (l < lane && okl && tl == tau) ok = false;
            }
            const u64 bad = __ballot(!ok);
            const int first_bad = bad ? __ffsll((unsigned long long)bad) - 1 : kWave;
            if (lane < first_bad) {
                ph_insert(J.ph, tau, col);
                J.V.pivcoef[col] = J.inv[tcoef];
                J.V.len[col] = -1; // V_col = sigma_col, R_col = its coboundary
                J.V.off[col] = 0;
                J.V.rlen[col] = -1;
                J.V.roff[col] = 0;
            }
            if (lane == 0) {
                S.base = base + first_bad;
                S.full = (first_bad < kWave) && (base + first_bad < J.ncols);
                S.stat[0] += first_bad;
            }
        }
        gsync(); // column metadata of the batch is visible to every wave
        RED_T1(S, 8, t_em);
        if (!S.full) continue;
        const int j = S.base;
        status = J.bm_bits ? reduce_one_bm<BT, Dist, false>(J, D, SC, L, j, S)
                           : reduce_one<BT, Dist, false>(J, D, G, SC, j, S);
        if (tid == 0) S.base = j + 1;
        gsync(); // V_j and the table entry are visible before the next column
    }
    gsync();
    RED_T1(S, 10, t_total);
    return status;
}

// The same reduction spread over the workgroups of a launch (ParState):
// each workgroup takes the next column from the cursor and reduces it; a
// column whose zero pivot cofacet tau is not in a zero apparent pair takes
// the emergent shortcut when tau is still free after the wait. Bars go to
// the column's own slot of J.bars (birth simplex -1: none). Returns a result
// code; on failure the abort flag stops the other workgroups.
template <int BT, class Dist>
__device__ __forceinline__ int reduce_columns_par(const ReduceJob<Dist> &J, const LdsCol &D,
                                                  const Staging &G, const ReduceScratch &SC,
                                                  const BmLds &L, RedShared<BT> &S) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x;
    wc_clear_all<BT>(D);
    wc_clear_all<BT>(SC.Vw);
    if (tid == 0) {
        S.abort = 0;
        S.nbars = 0;
        S.len = 0;
        S.f = 0;
        S.gen = 0;
    }
    if (tid < 13) S.stat[tid] = 0;
    if (tid < kRedTimers) S.tm[tid] = 0;
#if RIPS_COLUMN_TRACE
    if (tid == 0) S.wacc = 0;
#endif
    int status = 0;
    gsync();
    RED_T0(t_total);
    for (;;) {
        if (tid == 0) {
            int col = J.ncols;
            if (ld_dev(&J.par.ctl[kCtlAbort]) == 0) col = (int)min(atomicAdd(&J.par.ctl[kCtlNext], 1u), (u32)J.ncols);
            S.cur = col;
            S.m = 0;
            if ((J.shortcuts & kShortEmergent) && col < J.ncols && J.cols.j[col] >= 0 &&
                !J.cols.tapp[col]) {
                // emergent candidate: tau = sigma u {j}, at sigma's diameter
                int v[kMaxVerts];
                decode(J.cols.idx[col], k, c.n, c.B, v);
                int below;
                S.tau = cofacet_index(v, k, J.cols.j[col], c.B, &below);
                S.tcoef = coeff_sign(below, p);
                S.m = 1;
                st_dev(&J.par.cst[col], __float_as_uint(J.cols.diam[col]));
            }
        }
        __syncthreads();
        const int col = S.cur;
        const int emerg = S.m;
        __syncthreads();
        if (col >= J.ncols) break;
#if RIPS_COLUMN_TRACE
        unsigned long long tr0 = 0, tra = 0, trw = 0;
        if (tid == 0) {
            tr0 = wall_clock64();
            tra = S.stat[2];
            trw = S.wacc;
        }
        struct ColClock {
            const ReduceJob<Dist> &J;
            RedShared<BT> &S;
            int col, tid;
            unsigned long long t0, a0, w0;
            __device__ ~ColClock() {
                if (tid == 0 && J.trace) {
                    J.trace[4 * col + 0] = t0;
                    J.trace[4 * col + 1] = wall_clock64();
                    J.trace[4 * col + 2] = S.stat[2] - a0;
                    J.trace[4 * col + 3] = S.wacc - w0;
                }
            }
        } cclock{J, S, col, tid, tr0, tra, trw};
#endif
        if (emerg) {
            RED_T0(t_em);
            RED_T0(t_w);
            status = par_wait<BT>(J.par, S, col, __float_as_uint(J.cols.diam[col]));
            RED_T1(S, 17, t_w);
            if (status) break;
            if (tid == 0) S.owner = ph_find_dev(J.ph, S.tau);
            __syncthreads();
            const bool free = S.owner < 0;
            if (free) {
                // V_col = sigma_col, R_col = its coboundary; zero persistence
                if (tid == 0) {
                    J.V.pivcoef[col] = J.inv[S.tcoef];
                    J.V.len[col] = -1;
                    J.V.off[col] = 0;
                    J.V.rlen[col] = -1;
                    J.V.roff[col] = 0;
                    J.bars.bs[col] = -1;
                    S.stat[0] += 1;
                }
                fence_release_dev();
                __syncthreads();
                if (tid == 0) {
                    ph_insert_dev(J.ph, S.tau, col);
                    fence_release_dev();
                    st_dev(&J.par.cst[col], kColDone);
                }
            }
            __syncthreads();
            RED_T1(S, 8, t_em);
            if (free) continue;
        }
        status = J.bm_bits ? reduce_one_bm<BT, Dist, true>(J, D, SC, L, col, S)
                           : reduce_one<BT, Dist, true>(J, D, G, SC, col, S);
        if (status) break;
    }
    if (status && status != kRedAbort && tid == 0) st_dev(&J.par.ctl[kCtlAbort], 1u);
    __syncthreads();
    RED_T1(S, 10, t_total);
    return status;
}

hipError_t launch_reduce(const ReduceJob<DistFull> &J, u32 capD, ReduceBuffers RB, Scalars *s,
                         hipStream_t st);
// J.bars: one slot per column; the bars are compacted into `out` in column
// order and s->nbars set
hipError_t launch_reduce_par(const ReduceJob<DistFull> &J, u32 capD, ReduceBuffers RB, int groups,
                             BarBuf out, Scalars *s, hipStream_t st);

} // namespace rips
