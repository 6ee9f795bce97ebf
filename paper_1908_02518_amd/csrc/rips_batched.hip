// rips_batched.hip -- many point clouds of uneven sizes in one persistent
// launch. Each workgroup takes the next cloud from a queue ordered by
// decreasing size (longest processing time first) and runs the whole path on
// it: distances (packed lower triangle in LDS for n <= 256, a full matrix in
// its global scratch otherwise), enclosing radius, H0 (Boruvka + elder rule),
// the enumeration / apparent-pair filter of dimension 1, the column sort and
// the Z/p reduction (reduce_columns). Bars go to an unordered buffer with one
// segment per (cloud, dimension); a final pass lays them out in cloud order.
#include "../../include/rips.h"
#include "rips_batched.hpp"

namespace rips {

constexpr int kBT = 256;         // threads per workgroup
constexpr int kBatchFilterG = 8; // lanes per candidate edge in the filter

struct BatchShared {
    int cloud, n, nsurv, nbars0, flag, m;
    float t;
    unsigned long long mcount;
    unsigned long long cnt[4];
    int w[kBT / kWave + 1];
};

__device__ __forceinline__ void pair_of(int64_t e, int *a, int *b) {
    int x = (int)((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);
    while ((int64_t)x * (x - 1) / 2 > e) --x;
    while ((int64_t)(x + 1) * x / 2 <= e) ++x;
    *a = x;
    *b = (int)(e - (int64_t)x * (x - 1) / 2);
}

__device__ __forceinline__ u64 bkey(float d, u32 idx) {
    return ((u64)__float_as_uint(d) << 32) | (u64)(0xffffffffu - idx);
}

// d(i, j) for i != j: coordinates in increasing order, each product and sum
// rounded to float32, correctly rounded square root
__device__ __forceinline__ float point_dist(const float *X, int m, int i, int j) {
    float s = 0.0f;
    for (int c = 0; c < m; ++c) {
        const float t = X[i * m + c] - X[j * m + c];
        const float sq = t * t;
        s = s + sq;
    }
    return __builtin_sqrtf(s);
}

template <class Dist>
struct CloudDist;

template <>
struct CloudDist<DistPacked> {
    static __device__ DistPacked make(float *lds, float *, int n) { return DistPacked{lds, n}; }
};
template <>
struct CloudDist<DistFull> {
    static __device__ DistFull make(float *, float *g, int n) { return DistFull{g, n}; }
};

// The reduction job of the cloud whose data-parallel passes workgroup wgL
// ran: its columns, pivot table, apparent-pair table, column store, edge
// order and staged bars live in wgL's slices. The distances are read from
// wgL's global slice (the packed variant copies its LDS triangle there).
template <class Dist>
__device__ __forceinline__ ReduceJob<Dist> batch_job(const BatchArgs &A, int wgL, int n, float t, int S,
                                                    int nE) {
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    float *Dgw = A.Dg + (int64_t)wgL * A.d_stride;
    ReduceJob<Dist> J;
    J.c.d = CloudDist<Dist>::make(Dgw, Dgw, n);
    J.c.B = A.binom;
    J.c.nb.off = nullptr;
    J.c.nb.idx = nullptr;
    J.c.n = n;
    J.c.t = t;
    J.k = 1;
    J.p = A.p;
    J.inv = A.inv;
    const int64_t co = (int64_t)wgL * A.col_stride;
    J.cols = Columns{A.c_idx1 + co, A.c_dm1 + co, A.c_j1 + co, A.c_t1 + co};
    J.ncols = S;
    u32 phcap = 64;
    while (phcap < 2u * (u32)S + 64u && (int64_t)phcap < A.ph_stride) phcap <<= 1;
    J.ph = PivotHash{A.ph_keys + (int64_t)wgL * A.ph_stride, A.ph_vals + (int64_t)wgL * A.ph_stride,
                     phcap - 1};
    J.V.off = A.v_off + co;
    J.V.len = A.v_len + co;
    J.V.pivcoef = A.v_piv + co;
    J.V.roff = A.v_roff + co;
    J.V.rlen = A.v_rlen + co;
    J.V.idx = A.v_idx + (int64_t)wgL * A.v_stride;
    J.V.diam = A.v_diam + (int64_t)wgL * A.v_stride;
    J.V.coef = A.v_coef + (int64_t)wgL * A.v_stride;
    J.V.cap = A.v_stride;
    J.vcount = &A.v_count[wgL];
    const int64_t so = (int64_t)wgL * A.st_stride + n;
    J.bars = BarBuf{A.st_b + so, A.st_d + so, A.st_bs + so, A.st_ds + so};
    J.cand_avg = (float)n;
    u32 appcap = 64;
    while (appcap < 2u * (u32)npairs + 64u && (int64_t)appcap < A.ph_stride) appcap <<= 1;
    J.app = PairHash{A.app_keys + (int64_t)wgL * A.ph_stride, A.app_vals + (int64_t)wgL * A.ph_stride,
                     A.app_verts + (int64_t)wgL * A.ph_stride, nullptr, nullptr, nullptr, nullptr,
                     appcap - 1};
    J.par = A.spread > 1 ? ParState{A.par_cst + co, A.par_ctl + (int64_t)wgL * kCtlWords}
                         : ParState{nullptr, nullptr};
    J.shortcuts = kShortApparent | kShortEmergent | kShortClearing;
    J.keep_essential_v = 0;
    J.rstore = kRStoreAuto;
#if RIPS_COLUMN_TRACE
    J.trace = nullptr;
#endif
    J.prev_bits = nullptr;
    J.prev = PivotHash{nullptr, nullptr, 0};
    const int64_t to = (int64_t)wgL * A.bm_tab_stride;
    J.eo = A.bm_bits ? EdgeOrder{A.bm_pos + (int64_t)wgL * A.bm_pos_stride, A.bm_verts + to, A.bm_len + to,
                                 A.bm_run + to, A.bm_app + to, nE, (n + 31) / 32, n}
                     : EdgeOrder{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
    J.bm_bits = A.bm_bits;
    J.bm_stride = A.bm_stride;
    return J;
}

// This workgroup's own reduction scratch (blockIdx.x's slices) and the LDS
// of its working column.
__device__ __forceinline__ void batch_scratch(const BatchArgs &A, unsigned char *smem, LDS int *nsl,
                                              RedShared<kBT> &RS, int nE, LdsCol *Dw, Staging *Gs,
                                              ReduceScratch *SC, BmLds *L) {
    const int64_t wg = blockIdx.x;
    carve_reduce_lds(smem, A.capD, nsl, Dw, Gs, &SC->SB);
    *L = carve_bm_lds(smem, reduce_lds_bytes(A.capD), A.bm_bits ? nE : 0);
    for (int h = 0; h < 2; ++h) {
        SC->F.idx[h] = A.f_idx[h] + wg * A.f_stride;
        SC->F.dia[h] = A.f_dia[h] + wg * A.f_stride;
        SC->F.coef[h] = A.f_coef[h] + wg * A.f_stride;
    }
    SC->F.cap = A.f_stride;
    SC->Vw.keys = A.vw_keys + wg * A.vw_stride;
    SC->Vw.coef = A.vw_coef + wg * A.vw_stride;
    SC->Vw.diam = A.vw_diam + wg * A.vw_stride;
    SC->Vw.slots = A.vw_slots + wg * A.vw_stride;
    SC->Vw.nslots = (LDS int *)&RS.vns;
    SC->Vw.mask = (u32)A.vw_stride - 1;
    SC->lkey = A.log_key + wg * A.log_stride;
    SC->lcoef = A.log_coef + wg * A.log_stride;
    SC->ldia = A.log_dia + wg * A.log_stride;
    SC->lcap = A.log_stride;
}

// A reduction's status as a status bit of the batch (the host grows the
// buffer behind it and runs again).
__device__ __forceinline__ void batch_red_status(const BatchArgs &A, int rstat) {
    if (!rstat || rstat == kRedAbort || threadIdx.x != 0) return;
    const int bit = rstat == kRedBaseFull    ? 1
                    : rstat == kRedStoreFull ? 2
                    : rstat == kRedFarFull   ? 32
                    : rstat == kRedVFull     ? 64
                    : rstat == kRedLogFull   ? 128
                                             : 8;
    atomicOr(A.status, bit);
}

// Bounded wait of thread 0 until *w >= want (agent scope); false after
// kWaitTicks, with the batch status marked.
__device__ __forceinline__ bool batch_wait(const BatchArgs &A, const int *w, int want) {
    const unsigned long long t0 = wall_clock64();
    while (ld_dev(w) < want) {
        if (wall_clock64() - t0 > kWaitTicks) {
            atomicOr(A.status, 8);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// The counters of one workgroup's share of a spread-out reduction, summed
// into its cloud's (the leader's) counters.
__device__ __forceinline__ void batch_par_stats(const BatchArgs &A, int wgL, const RedShared<kBT> &RS) {
    if (threadIdx.x != 0) return;
    unsigned long long *ps = A.par_stat + (int64_t)wgL * kSyncStats;
    atomicAdd(&ps[0], RS.stat[0]);   // emergent
    atomicAdd(&ps[1], RS.stat[1]);   // reduced
    atomicAdd(&ps[2], RS.stat[2]);   // additions
    atomicAdd(&ps[3], RS.stat[3]);   // bars of nonzero persistence
    atomicAdd(&ps[4], RS.stat[4]);   // essential
    atomicAdd(&ps[12], RS.stat[12]); // entries added
}

// The dimension-1 enumeration / apparent-pair filter: survivors appended
// through *nsurv, zero apparent pairs inserted into app, the counts of
// candidates, cleared and apparent columns added to cnt[0..2]; with appe (the
// direct-mapped column), appe[e] = the third vertex of edge e's zero
// apparent cofacet, or -1, for every edge it looks at. The edges: with
// chunk == null, this workgroup's whole pass over all of them; otherwise
// runs of kFilterChunk edges handed out through *chunk (an agent-scope
// counter the cloud's workgroups share). bits (the forest edges of H0, which
// clearing skips) or null: then a forest edge comes out as a survivor (it is
// in no zero apparent pair, being paired in dimension 0), and the caller
// drops it. Every thread calls it.
constexpr int kFilterChunk = 128;

template <class Dist>
__device__ __forceinline__ void batch_filter(const BatchArgs &A, const Ctx<Dist> &c, float t, int64_t npairs,
                                             const u32 *bits, const Columns &surv, const PairHash &app,
                                             int *appe, int *chunk, int *nsurv, unsigned long long *cnt) {
    const int tid = threadIdx.x, lane = lane_id();
    const Dist dist = c.d;
    const bool leader = (lane & (kBatchFilterG - 1)) == 0;
    unsigned long long n_clear = 0, n_acol = 0, n_cand = 0;
    // one edge per group of kBatchFilterG lanes; the loop is uniform in
    // the wave and the tests are predicates (the scans need every lane)
    constexpr int kGroups = kWave / kBatchFilterG;
    int64_t e0 = (int64_t)(tid / kWave) * kGroups, cend = npairs;
    if (chunk) {
        int base = 0;
        if (lane == 0) base = atomicAdd(chunk, kFilterChunk);
        base = __shfl(base, 0, kWave);
        e0 = base;
        cend = min<int64_t>(npairs, (int64_t)base + kFilterChunk);
    }
    for (;;) {
        if (e0 >= cend) {
            if (!chunk || cend >= npairs) break;
            int base = 0;
            if (lane == 0) base = atomicAdd(chunk, kFilterChunk);
            base = __shfl(base, 0, kWave);
            e0 = base;
            cend = min<int64_t>(npairs, (int64_t)base + kFilterChunk);
            if (e0 >= cend) break;
        }
        const int64_t e = e0 + lane / kBatchFilterG;
        e0 += chunk ? kGroups : (int64_t)(kBT / kWave) * kGroups;
        bool live = e < cend;
        int v[2] = {0, 0};
        float dm = 0.0f;
        if (live) {
            pair_of(e, &v[0], &v[1]);
            dm = dist(v[0], v[1]);
            live = dm <= t;
        }
        if (live) {
            n_cand += leader;
            if (bits && ((bits[e >> 5] >> (e & 31)) & 1u)) {
                n_clear += leader;
                live = false;
            }
        }
        const int j = scan_max_k<kBatchFilterG, 1>(c, v, dm, -1, live);
        int tv[3];
        int pos = 0;
        insert_k<1>(v, j, tv, pos);
        const bool zap = live && j >= 0 && zero_pivot_facet_k<2>(c, tv, dm) == pos;
        if (zap) {
            n_acol += leader;
            live = false;
            // capacity is at least twice the pairs: the insert cannot fail
            if (leader)
                (void)pair_insert(app, simplex_index(tv, 2, c.B), (e << 3) | pos,
                                  (u64)(u32)v[0] | ((u64)(u32)v[1] << 16), 0);
        }
        if (appe != nullptr && leader && e < cend) appe[e] = zap ? j : -1;
        // is the zero pivot cofacet itself in a zero apparent pair (for
        // the emergent shortcut)?
        const bool tj = live && j >= 0;
        const int mt = tj ? zero_pivot_facet_k<2>(c, tv, dm) : -1;
        int rt[2];
        remove_k<2>(tv, mt < 0 ? 0 : mt, rt);
        const bool ttest = tj && mt >= 0;
        const int jt = scan_max_k<kBatchFilterG, 1>(c, rt, dm, pick_vertex(tv, mt), ttest);
        if (live && leader) {
            const int slot = atomicAdd(nsurv, 1);
            if (slot < A.col_stride) {
                surv.idx[slot] = e;
                surv.diam[slot] = dm;
                surv.j[slot] = j;
                surv.tapp[slot] = (ttest && jt < 0) ? 1 : 0;
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        n_clear += __shfl_xor(n_clear, off, kWave);
        n_acol += __shfl_xor(n_acol, off, kWave);
        n_cand += __shfl_xor(n_cand, off, kWave);
    }
    if (lane == 0) {
        atomicAdd(&cnt[0], n_cand);
        atomicAdd(&cnt[1], n_clear);
        atomicAdd(&cnt[2], n_acol);
    }
}

// Per position of workgroup wgT's edge order, the third vertex of the
// edge's zero apparent cofacet, from the filter's per-edge values (the edge
// of position q is sb.val[ce][q]); after the whole filter. Every thread
// calls it.
__device__ __forceinline__ void batch_map_app(const BatchArgs &A, SortBufs sb, int ce, int nE, int wgT) {
    const int *appe = A.bm_appe + (int64_t)wgT * A.bm_tab_stride;
    int *app = A.bm_app + (int64_t)wgT * A.bm_tab_stride;
    for (int q = threadIdx.x; q < nE; q += kBT) app[q] = appe[sb.val[ce][q]];
    gsync();
}

// The edges <= t in order of length, for the direct-mapped working column,
// into workgroup wgT's tables (edge index -> position, -1 for an edge longer
// than t; position -> vertices, length and run word); sb are the calling
// workgroup's sort buffers, *ce the one that holds the order. Each thread
// keeps a contiguous range of pair indices, so that the stable sort leaves
// equal lengths in index order. Every thread calls it; returns the number
// of edges.
template <class Dist>
__device__ __forceinline__ int batch_edge_order(const BatchArgs &A, const Dist &dist, float t, int n, int64_t npairs,
                                                SortBufs sb, SortShared<kBT> &SS, int *scan_w, int wgT,
                                                int *ce_out) {
    const int tid = threadIdx.x;
    const int64_t chunk = (npairs + kBT - 1) / kBT;
    const int64_t e0 = (int64_t)tid * chunk, e1 = min(npairs, e0 + chunk);
    int cnt = 0;
    for (int64_t e = e0; e < e1; ++e) {
        int a, cc;
        pair_of(e, &a, &cc);
        cnt += dist(a, cc) <= t ? 1 : 0;
    }
    int nE;
    int at = block_scan_excl<kBT>(cnt, scan_w, &nE);
    int *bpos = A.bm_pos + (int64_t)wgT * A.bm_pos_stride;
    for (int64_t e = e0; e < e1; ++e) {
        int a, cc;
        pair_of(e, &a, &cc);
        const float d = dist(a, cc);
        if (d <= t) {
            sb.lo[0][at] = 0;
            sb.hi[0][at] = __float_as_uint(d);
            sb.val[0][at] = (u32)e;
            ++at;
        } else {
            bpos[(int64_t)a * n + cc] = -1;
            bpos[(int64_t)cc * n + a] = -1;
        }
    }
    gsync();
    const int ce = block_radix_sort<kBT>(sb, nE, 0, 4, SS);
    *ce_out = ce;
    u32 *bv = A.bm_verts + (int64_t)wgT * A.bm_tab_stride;
    float *bl = A.bm_len + (int64_t)wgT * A.bm_tab_stride;
    u32 *br = A.bm_run + (int64_t)wgT * A.bm_tab_stride;
    for (int q = tid; q < nE; q += kBT) {
        const u32 e = sb.val[ce][q];
        int a, cc;
        pair_of(e, &a, &cc);
        bpos[(int64_t)a * n + cc] = q;
        bpos[(int64_t)cc * n + a] = q;
        bv[q] = ((u32)a << 16) | (u32)cc;
        bl[q] = __uint_as_float(sb.hi[ce][q]);
    }
    gsync();
    // runs of equal lengths: first position, and whether the next
    // position continues the run (keys are the length bits)
    for (int q = tid; q < nE; q += kBT) {
        const u32 key = sb.hi[ce][q];
        int r = q;
        while (r > 0 && sb.hi[ce][r - 1] == key) --r;
        const bool tie = q + 1 < nE && sb.hi[ce][q + 1] == key;
        br[q] = (u32)r | (tie ? kRunTie : 0u);
    }
    gsync();
    return nE;
}

// A workgroup that helps its cloud's leader (spread > 1). With the
// distances in global memory it first filters its share of the edges (after
// the leader's distances and H0); then it waits for the leader's sorted
// columns, reduces columns from the shared cursor with its own scratch, adds
// its counters and reports done.
template <class Dist>
__device__ void batch_follow(const BatchArgs &A, int wgL, int role, unsigned char *smem, BatchShared &Sh,
                             RedShared<kBT> &RS, SortShared<kBT> &SS) {
    constexpr bool kLds = std::is_same<Dist, DistPacked>::value;
    const int tid = threadIdx.x;
    // with three or more workgroups the second builds the edge order
    const bool ordering = A.spread >= 3 && A.bm_bits != nullptr;
    const bool order_role = ordering && role == 1;
    if (A.max_dim < 1) return; // no reduction: the leader waits for nobody
    int *sw = A.sync + (int64_t)wgL * kSyncWords;
    __shared__ int s_go;
    if (!kLds) {
        if (tid == 0) {
            // the front flag, or the skip flag of a rejected cloud
            const unsigned long long t0 = wall_clock64();
            int go = 1;
            while (ld_dev(&sw[kSyncFront]) == 0 && ld_dev(&sw[kSyncSkip]) == 0) {
                if (wall_clock64() - t0 > kWaitTicks) {
                    atomicOr(A.status, 8);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            s_go = go && ld_dev(&sw[kSyncSkip]) == 0;
        }
        __syncthreads();
        if (s_go) {
            fence_acquire_dev(); // the leader's distances, forest edges and table
            const int n = __builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncN]));
            const float t = __int_as_float(__builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncT])));
            const int64_t npairs = (int64_t)n * (n - 1) / 2;
            float *Dgw = A.Dg + (int64_t)wgL * A.d_stride;
            Ctx<Dist> c;
            c.d = CloudDist<Dist>::make(Dgw, Dgw, n);
            c.B = A.binom;
            c.nb.off = nullptr;
            c.nb.idx = nullptr;
            c.n = n;
            c.t = t;
            const int64_t co = (int64_t)wgL * A.col_stride;
            const Columns surv{A.c_idx0 + co, A.c_dm0 + co, A.c_j0 + co, A.c_t0 + co};
            u32 appcap = 64;
            while (appcap < 2u * (u32)npairs + 64u && (int64_t)appcap < A.ph_stride) appcap <<= 1;
            const PairHash app{A.app_keys + (int64_t)wgL * A.ph_stride, A.app_vals + (int64_t)wgL * A.ph_stride,
                               A.app_verts + (int64_t)wgL * A.ph_stride, nullptr, nullptr, nullptr, nullptr,
                               appcap - 1};
            SortBufs sb_o;
            int ce_o = 0, nE_o = 0;
            if (order_role) {
                // first the edge order, into the leader's tables, with this
                // workgroup's sort buffers
                const int64_t wo = (int64_t)blockIdx.x * A.col_stride;
                sb_o.lo[0] = A.s_lo0 + wo;
                sb_o.lo[1] = A.s_lo1 + wo;
                sb_o.hi[0] = A.s_hi0 + wo;
                sb_o.hi[1] = A.s_hi1 + wo;
                sb_o.val[0] = A.s_v0 + wo;
                sb_o.val[1] = A.s_v1 + wo;
                nE_o = batch_edge_order<Dist>(A, c.d, t, n, npairs, sb_o, SS, Sh.w, wgL, &ce_o);
            }
            // runs of edges from the shared counter until none is left (no
            // clearing: the leader drops the forest edges); then done
            int *appe = A.bm_bits ? A.bm_appe + (int64_t)wgL * A.bm_tab_stride : nullptr;
            batch_filter<Dist>(A, c, t, npairs, nullptr, surv, app, appe, &sw[kSyncChunk], &sw[kSyncSurv],
                               A.par_stat + (int64_t)wgL * kSyncStats + 8);
            fence_release_dev();
            __syncthreads();
            if (tid == 0) atomicAdd(&sw[kSyncFiltered], 1);
            if (order_role) {
                // the apparent vertices by position, once every workgroup
                // of the cloud is done filtering
                if (tid == 0) (void)batch_wait(A, &sw[kSyncFiltered], A.spread);
                __syncthreads();
                fence_acquire_dev();
                batch_map_app(A, sb_o, ce_o, nE_o, wgL);
                if (tid == 0) sw[kSyncE] = nE_o;
            }
        }
        // the edge order, then done
        fence_release_dev();
        __syncthreads();
        if (order_role && tid == 0) atomicAdd(&sw[kSyncOrdered], 1);
    }
    if (tid == 0) s_go = batch_wait(A, &sw[kSyncReady], 1) ? 1 : 0;
    __syncthreads();
    if (s_go) {
        fence_acquire_dev(); // the leader's columns, tables and words
        const int skip = __builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncSkip]));
        if (!skip) {
            const int n = __builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncN]));
            const float t = __int_as_float(__builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncT])));
            const int S = __builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncS]));
            const int nE = __builtin_amdgcn_readfirstlane(ld_dev(&sw[kSyncE]));
            const ReduceJob<Dist> J = batch_job<Dist>(A, wgL, n, t, S, nE);
            __shared__ int s_nsl;
            LdsCol Dw;
            Staging Gs;
            ReduceScratch SC;
            BmLds L;
            batch_scratch(A, smem, (LDS int *)&s_nsl, RS, nE, &Dw, &Gs, &SC, &L);
            gsync();
            const int rstat = reduce_columns_par<kBT>(J, Dw, Gs, SC, L, RS);
            batch_red_status(A, rstat);
            batch_par_stats(A, wgL, RS);
        }
    }
    // the column slots and the column store written here, then done
    fence_release_dev();
    __syncthreads();
    if (tid == 0) atomicAdd(&sw[kSyncDone], 1);
}

// One cloud by one workgroup. kLdsD: distances in LDS (packed) for the
// enumeration and H0 phases, then copied to global for the reduction.
template <class Dist>
__device__ void batch_cloud(const BatchArgs &A, int b, unsigned char *smem, BatchShared &Sh,
                            RedShared<kBT> &RS, SortShared<kBT> &SS) {
    constexpr bool kLds = std::is_same<Dist, DistPacked>::value;
    const int tid = threadIdx.x, lane = lane_id();
    const int wg = blockIdx.x;
    // max_dim and the cloud index are uniform: held in scalar registers they
    // are never copied between vector registers by the register allocator.
    // (A copy of max_dim into an accumulation register, placed at the end of
    // a divergent loop before the exec mask was restored, once left it
    // undefined in the lanes outside that loop; those lanes then took the
    // dimension-1 branch alone.)
    const int max_dim = __builtin_amdgcn_readfirstlane(A.max_dim);
    b = __builtin_amdgcn_readfirstlane(b);
    const int D1 = max_dim + 1;
    const int64_t o0 = A.offsets[b];
    const int64_t nn = A.offsets[b + 1] - o0;
    if (nn < 1 || nn > A.nmax) {
        // rejected by the order pass (status bit 16); publish empty segments
        if (threadIdx.x == 0) {
            for (int d = 0; d < D1; ++d) {
                A.seg_start[(int64_t)b * D1 + d] = 0;
                A.seg_count[(int64_t)b * D1 + d] = 0;
            }
            if (A.spread > 1) {
                int *sw = A.sync + (int64_t)wg * kSyncWords;
                st_dev(&sw[kSyncSkip], 1);
                fence_release_dev();
                st_dev(&sw[kSyncReady], 1);
            }
        }
        __syncthreads();
        return;
    }
    const int n = __builtin_amdgcn_readfirstlane((int)nn);
    const int m = A.m;
    const float *X = A.X + o0 * m;
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    float *Dl = (float *)smem;                       // packed D in LDS (kLds)
    float *Dgw = A.Dg + (int64_t)wg * A.d_stride;    // this workgroup's global D
    // ---- distances
    bool fin = true;
    if (kLds) {
        for (int64_t e = tid; e < npairs; e += kBT) {
            int a, c;
            pair_of(e, &a, &c);
            const float d = point_dist(X, m, a, c);
            fin = fin && isfinite(d);
            Dl[e] = d;
        }
    } else {
        for (int64_t q = tid; q < (int64_t)n * n; q += kBT) {
            const int i = (int)(q / n), j = (int)(q % n);
            const float d = i == j ? 0.0f : point_dist(X, m, i, j);
            fin = fin && isfinite(d);
            Dgw[q] = d;
        }
    }
    if (!fin) atomicOr(A.status, 4);
    if (tid == 0) {
        Sh.flag = 0x7f800000; // enclosing radius as float bits
        for (int q = 0; q < 4; ++q) Sh.cnt[q] = 0;
    }
    gsync();
    const Dist dist = CloudDist<Dist>::make(Dl, Dgw, n);
    // ---- enclosing radius min_x max_y d(x, y)
    for (int i = tid; i < n; i += kBT) {
        float mx = 0.0f;
        for (int j = 0; j < n; ++j)
            if (j != i) mx = fmaxf(mx, dist(i, j));
        atomicMin((unsigned *)&Sh.flag, __float_as_uint(mx));
    }
    __syncthreads();
    const float renc = n > 1 ? __uint_as_float((u32)Sh.flag) : 0.0f;
    const float t = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(fminf(A.threshold, renc))));
    // with the distances in global memory the cloud's other workgroups start
    // the dimension-1 filter now, while this one computes H0: its apparent-
    // pair table is emptied first, then n, t and the front flag are published
    const bool share = A.spread > 1 && !kLds && max_dim >= 1;
    u32 appcap = 64;
    while (appcap < 2u * (u32)npairs + 64u && (int64_t)appcap < A.ph_stride) appcap <<= 1;
    int *sw0 = A.sync + (int64_t)wg * kSyncWords;
    unsigned long long *fcnt = A.par_stat + (int64_t)wg * kSyncStats + 8;
    if (max_dim >= 1) {
        int64_t *akeys = A.app_keys + (int64_t)wg * A.ph_stride;
        for (u32 q = tid; q < appcap; q += kBT) akeys[q] = kEmpty;
    }
    if (share) {
        if (tid < 3) fcnt[tid] = 0ull;
        if (tid == 0) {
            sw0[kSyncN] = n;
            sw0[kSyncT] = __float_as_int(t);
        }
        fence_release_dev();
        gsync();
        if (tid == 0) st_dev(&sw0[kSyncFront], 1);
    }
    // ---- H0: Boruvka on the pairs <= t, union-find state in LDS
    const int nm = A.nmax;
    const int64_t npairs_max = (int64_t)nm * (nm - 1) / 2;
    unsigned char *after = smem + (kLds ? ((size_t)npairs_max * 4 + 15) / 16 * 16 : 0);
    u64 *best = (u64 *)after;
    int *comp = (int *)(best + nm);
    int *hook = comp + nm;
    u32 *bits = kLds ? (u32 *)(hook + nm) : A.bits_g + (int64_t)wg * A.bits_stride;
    const int64_t nwords = npairs / 32 + 1;
    u64 *mst = A.s_lo0 + (int64_t)wg * A.col_stride;
    for (int v = tid; v < n; v += kBT) st(&comp[v], v);
    for (int64_t q = tid; q < nwords; q += kBT) bits[q] = 0;
    if (tid == 0) Sh.mcount = 0;
    __syncthreads();
    for (int round = 0; round < 40; ++round) {
        for (int v = tid; v < n; v += kBT) st(&best[v], ~0ull);
        __syncthreads();
        for (int64_t e = tid; e < npairs; e += kBT) {
            int a, c;
            pair_of(e, &a, &c);
            const float d = dist(a, c);
            if (!(d <= t)) continue;
            const int ca = ld(&comp[a]), cb = ld(&comp[c]);
            if (ca != cb) {
                const u64 key = bkey(d, (u32)e);
                atomicMin(&best[ca], key);
                atomicMin(&best[cb], key);
            }
        }
        if (tid == 0) Sh.flag = 0;
        __syncthreads();
        for (int v = tid; v < n; v += kBT) {
            const int cv = ld(&comp[v]);
            int h = cv;
            const u64 key = ld(&best[v]);
            if (cv == v && key != ~0ull) {
                int a, c;
                pair_of(0xffffffffu - (u32)(key & 0xffffffffu), &a, &c);
                const int ca = ld(&comp[a]), cb = ld(&comp[c]);
                const int other = ca == v ? cb : ca;
                const bool mutual = ld(&best[other]) == key;
                if (!mutual || v > other) {
                    h = other;
                    const unsigned long long slot = atomicAdd(&Sh.mcount, 1ull);
                    if (slot < (unsigned long long)n) mst[slot] = key;
                    Sh.flag = 1;
                }
            }
            st(&hook[v], h);
        }
        gsync();
        if (!Sh.flag) break;
        for (int v = tid; v < n; v += kBT) st(&comp[v], ld(&hook[v]));
        for (int jump = 0; jump < 40; ++jump) {
            __syncthreads();
            if (tid == 0) Sh.flag = 0;
            __syncthreads();
            for (int v = tid; v < n; v += kBT) {
                const int c = ld(&comp[v]), cc = ld(&comp[c]);
                if (c != cc) {
                    st(&comp[v], cc);
                    Sh.flag = 1;
                }
            }
            __syncthreads();
            if (!Sh.flag) break;
        }
    }
    gsync();
    const int mm = (int)min(Sh.mcount, (unsigned long long)(n > 0 ? n - 1 : 0));
    SortBufs sb;
    sb.lo[0] = mst;
    sb.lo[1] = A.s_lo1 + (int64_t)wg * A.col_stride;
    sb.hi[0] = A.s_hi0 + (int64_t)wg * A.col_stride;
    sb.hi[1] = A.s_hi1 + (int64_t)wg * A.col_stride;
    sb.val[0] = A.s_v0 + (int64_t)wg * A.col_stride;
    sb.val[1] = A.s_v1 + (int64_t)wg * A.col_stride;
    for (int e = tid; e < mm; e += kBT) {
        sb.hi[0][e] = 0;
        sb.val[0][e] = 0;
    }
    gsync();
    const int cur = block_radix_sort<kBT>(sb, mm, 8, 0, SS);
    const u64 *keys = sb.lo[cur];
    // elder rule on wave 0 (parent = comp, maxv = hook arrays)
    int *parent = comp, *maxv = hook;
    float *hdeath = (float *)best;          // reuse: n floats
    int64_t *hds = (int64_t *)(A.st_ds + (int64_t)wg * A.st_stride + A.st_stride - n);
    for (int v = tid; v < n; v += kBT) {
        st(&parent[v], v);
        st(&maxv[v], v);
        hdeath[v] = -1.0f;
    }
    __syncthreads();
    if (tid < kWave) {
        for (int base = 0; base < mm; base += kWave) {
            const int e = base + lane;
            const bool valid = e < mm;
            int ra = 0, rb = 0, ma = -1, mb = -1;
            u32 idx = 0;
            float dm = 0.0f;
            if (valid) {
                const u64 key = keys[e];
                idx = 0xffffffffu - (u32)(key & 0xffffffffu);
                dm = __uint_as_float((u32)(key >> 32));
                int a, c;
                pair_of(idx, &a, &c);
                a = min(a, n - 1);
                c = min(c, n - 1);
                ra = a;
                for (int g = 0; g < n && ld(&parent[ra]) != ra; ++g) ra = ld(&parent[ra]);
                rb = c;
                for (int g = 0; g < n && ld(&parent[rb]) != rb; ++g) rb = ld(&parent[rb]);
                ma = ld(&maxv[ra]);
                mb = ld(&maxv[rb]);
            }
            const int cnt = min(kWave, mm - base);
            int my_loser = 0, my_winner = 0, my_newmax = 0, my_birth = 0;
            for (int q = 0; q < cnt; ++q) {
                const int RA = __shfl(ra, q, kWave), RB = __shfl(rb, q, kWave);
                const int MA = __shfl(ma, q, kWave), MB = __shfl(mb, q, kWave);
                const int winner = MA > MB ? RA : RB;
                const int loser = MA > MB ? RB : RA;
                const int newmax = MA > MB ? MA : MB;
                if (lane == q) {
                    my_loser = loser;
                    my_winner = winner;
                    my_newmax = newmax;
                    my_birth = MA > MB ? MB : MA;
                }
                if (ra == RA || ra == RB) {
                    ra = winner;
                    ma = newmax;
                }
                if (rb == RA || rb == RB) {
                    rb = winner;
                    mb = newmax;
                }
            }
            if (valid) {
                st(&parent[my_loser], my_winner);
                atomicMax(&maxv[my_winner], my_newmax);
                if (dm > 0.0f) {
                    hdeath[my_birth] = dm;
                    hds[my_birth] = (int64_t)idx;
                }
                if ((int64_t)idx < npairs) atomicOr(&bits[idx >> 5], 1u << (idx & 31));
            }
        }
    }
    gsync();
    for (int v = tid; v < n; v += kBT)
        if (ld(&parent[v]) == v) {
            const int bb = ld(&maxv[v]);
            hdeath[bb] = INFINITY;
            hds[bb] = -1;
        }
    gsync();
    // H0 bars into the stage, by birth vertex descending
    float *sb_b = A.st_b + (int64_t)wg * A.st_stride;
    float *sb_d = A.st_d + (int64_t)wg * A.st_stride;
    int64_t *sb_bs = A.st_bs + (int64_t)wg * A.st_stride;
    int64_t *sb_ds = A.st_ds + (int64_t)wg * A.st_stride;
    {
        int at = 0, nz = 0, ne = 0;
        for (int base = 0; base < n; base += kBT) {
            const int v = n - 1 - (base + tid);
            const float hd = v >= 0 ? hdeath[v] : -1.0f;
            const bool has = hd >= 0.0f;
            int tot;
            const int ex = block_scan_excl<kBT>(has ? 1 : 0, Sh.w, &tot);
            if (has) {
                sb_b[at + ex] = 0.0f;
                sb_d[at + ex] = hd;
                sb_bs[at + ex] = v;
                sb_ds[at + ex] = hds[v];
                if (isinf(hd)) ++ne;
                else ++nz;
            }
            at += tot;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            nz += __shfl_xor(nz, off, kWave);
            ne += __shfl_xor(ne, off, kWave);
        }
        if (lane == 0) {
            atomicAdd(&Sh.cnt[0], (unsigned long long)nz);
            atomicAdd(&Sh.cnt[1], (unsigned long long)ne);
        }
        if (tid == 0) Sh.nbars0 = at;
    }
    gsync();
    if (tid == 0) {
        rips_dim_stats &s0 = A.stats[(int64_t)b * D1];
        s0.candidates = n;
        s0.cleared = 0;
        s0.apparent_col = 0;
        s0.apparent_pivot = 0;
        s0.columns = n;
        s0.emergent = 0;
        s0.reduced = 0;
        s0.additions = 0;
        s0.bars_nonzero = (int64_t)Sh.cnt[0];
        s0.essential = (int64_t)Sh.cnt[1];
        s0.entries_added = 0;
        s0.entries_stored = 0;
        A.t_used[b] = t;
        Sh.nsurv = 0;
        Sh.cnt[0] = Sh.cnt[1] = Sh.cnt[2] = Sh.cnt[3] = 0;
    }
    __syncthreads();
    int nb1 = 0;
    if (max_dim >= 1) {
        // ---- dimension 1: enumeration / apparent-pair filter over the edges
        Ctx<Dist> c;
        c.d = dist;
        c.B = A.binom;
        c.nb.off = nullptr;
        c.nb.idx = nullptr;
        c.n = n;
        c.t = t;
        Columns surv{A.c_idx0 + (int64_t)wg * A.col_stride, A.c_dm0 + (int64_t)wg * A.col_stride,
                     A.c_j0 + (int64_t)wg * A.col_stride, A.c_t0 + (int64_t)wg * A.col_stride};
        // the zero apparent pairs (rho, tau) found here serve the reduction's
        // pivot tests (one lookup instead of facet and cofacet scans); the
        // table was emptied before H0
        const PairHash app{A.app_keys + (int64_t)wg * A.ph_stride, A.app_vals + (int64_t)wg * A.ph_stride,
                           A.app_verts + (int64_t)wg * A.ph_stride, nullptr, nullptr, nullptr, nullptr,
                           appcap - 1};
        gsync();
        // spread out, every workgroup of the cloud takes runs of edges from
        // the shared counter (the edge-order workgroup once its order is
        // built), with no clearing: the forest edges are dropped below
        int *appe = A.bm_bits ? A.bm_appe + (int64_t)wg * A.bm_tab_stride : nullptr;
        batch_filter<Dist>(A, c, t, npairs, share ? nullptr : bits, surv, app, appe,
                           share ? &sw0[kSyncChunk] : nullptr, share ? &sw0[kSyncSurv] : &Sh.nsurv,
                           share ? fcnt : Sh.cnt);
        if (share) {
            // this workgroup done filtering, then every other
            fence_release_dev();
            __syncthreads();
            if (tid == 0) {
                atomicAdd(&sw0[kSyncFiltered], 1);
                (void)batch_wait(A, &sw0[kSyncFiltered], A.spread);
            }
            __syncthreads();
            fence_acquire_dev();
            if (tid == 0) {
                Sh.nsurv = ld_dev(&sw0[kSyncSurv]);
                Sh.cnt[0] = ld_dev(&fcnt[0]);
                Sh.cnt[1] = ld_dev(&fcnt[1]);
                Sh.cnt[2] = ld_dev(&fcnt[2]);
            }
        }
        gsync();
        const int S0 = min(Sh.nsurv, (int)A.col_stride);
        // ---- sort: diameter descending, then index ascending (a forest edge,
        // when the filter did not clear it, after every column: bit 31 of its
        // key; the count of those is the cleared count)
        if (share && tid == 0) Sh.cnt[3] = 0;
        gsync();
        int nforest = 0;
        for (int e = tid; e < S0; e += kBT) {
            const int64_t ix = surv.idx[e];
            const bool forest = share && ((bits[ix >> 5] >> (ix & 31)) & 1u);
            nforest += forest ? 1 : 0;
            sb.lo[0][e] = (u64)ix | (forest ? (1ull << 31) : 0ull);
            sb.hi[0][e] = forest ? ~0u : ~__float_as_uint(surv.diam[e]);
            sb.val[0][e] = (u32)e;
        }
        if (nforest) atomicAdd(&Sh.cnt[3], (unsigned long long)nforest);
        gsync();
        if (share && tid == 0) Sh.cnt[1] = Sh.cnt[3];
        const int S = S0 - (share ? (int)Sh.cnt[3] : 0);
        const int cs = block_radix_sort<kBT>(sb, S0, 4, 4, SS);
        Columns cols{A.c_idx1 + (int64_t)wg * A.col_stride, A.c_dm1 + (int64_t)wg * A.col_stride,
                     A.c_j1 + (int64_t)wg * A.col_stride, A.c_t1 + (int64_t)wg * A.col_stride};
        for (int q = tid; q < S0; q += kBT) {
            const u32 e = sb.val[cs][q];
            cols.idx[q] = surv.idx[e];
            cols.diam[q] = surv.diam[e];
            cols.j[q] = surv.j[e];
            cols.tapp[q] = surv.tapp[e];
        }
        // ---- the edges <= t in order of length, for the direct-mapped
        // working column (by the cloud's second workgroup, during the
        // filter, when the cloud has three or more)
        const bool offload = share && A.spread >= 3 && A.bm_bits;
        EdgeOrder eo{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
        if (A.bm_bits) {
            int nE;
            if (offload) {
                if (tid == 0) (void)batch_wait(A, &sw0[kSyncOrdered], 1);
                __syncthreads();
                fence_acquire_dev();
                nE = __builtin_amdgcn_readfirstlane(ld_dev(&sw0[kSyncE]));
            } else {
                int ce;
                nE = batch_edge_order<Dist>(A, dist, t, n, npairs, sb, SS, Sh.w, wg, &ce);
                batch_map_app(A, sb, ce, nE, wg);
            }
            const int64_t to = (int64_t)wg * A.bm_tab_stride;
            eo = EdgeOrder{A.bm_pos + (int64_t)wg * A.bm_pos_stride, A.bm_verts + to, A.bm_len + to,
                           A.bm_run + to, A.bm_app + to, nE, (n + 31) / 32, n};
        }
        // ---- the reduction reads D from global; LDS now holds its working column
        if (kLds)
            for (int64_t e = tid; e < npairs; e += kBT) Dgw[e] = Dl[e];
        const int spread = A.spread;
        const ReduceJob<Dist> J = batch_job<Dist>(A, wg, n, t, S, eo.E);
        for (u32 q = tid; q <= J.ph.mask; q += kBT) {
            st(&J.ph.keys[q], kEmpty);
            if (spread > 1) st(&J.ph.vals[q], -1); // spread out: -1 = no value yet
        }
        if (tid == 0) A.v_count[wg] = 0;
        int *sw = A.sync + (int64_t)wg * kSyncWords;
        if (spread > 1) {
            // column states, control words and counters of the shared
            // reduction, then the words the other workgroups build their job
            // from, then the ready flag
            for (int q = tid; q < S; q += kBT) J.par.cst[q] = 0u;
            if (tid < kCtlWords) J.par.ctl[tid] = 0u;
            if (tid < kSyncStats) A.par_stat[(int64_t)wg * kSyncStats + tid] = 0ull;
            if (tid == 0) {
                sw[kSyncN] = n;
                sw[kSyncT] = __float_as_int(t);
                sw[kSyncS] = S;
                sw[kSyncE] = eo.E;
            }
            fence_release_dev();
            gsync();
            if (tid == 0) st_dev(&sw[kSyncReady], 1);
        }
        __shared__ int s_nsl;
        LdsCol Dw;
        Staging Gs;
        ReduceScratch SC;
        BmLds L;
        batch_scratch(A, smem, (LDS int *)&s_nsl, RS, eo.E, &Dw, &Gs, &SC, &L);
        gsync();
        unsigned long long st5[6];
        if (spread > 1) {
            const int rstat = reduce_columns_par<kBT>(J, Dw, Gs, SC, L, RS);
            batch_red_status(A, rstat);
            batch_par_stats(A, wg, RS);
            // the other workgroups' column slots, then the bars compacted in
            // column order (each slot has birth simplex -1 when it gives none)
            if (tid == 0) (void)batch_wait(A, &sw[kSyncDone], spread - 1);
            __syncthreads();
            fence_acquire_dev();
            int base = 0;
            for (int c0 = 0; c0 < S; c0 += kBT) {
                const int q = c0 + tid;
                float bb = 0.0f, bd = 0.0f;
                int64_t bbs = -1, bds = -1;
                if (q < S) {
                    bb = J.bars.birth[q];
                    bd = J.bars.death[q];
                    bbs = J.bars.bs[q];
                    bds = J.bars.ds[q];
                }
                const bool keep = q < S && bbs >= 0;
                int tot;
                const int at = block_scan_excl<kBT>(keep ? 1 : 0, Sh.w, &tot);
                if (keep) {
                    J.bars.birth[base + at] = bb;
                    J.bars.death[base + at] = bd;
                    J.bars.bs[base + at] = bbs;
                    J.bars.ds[base + at] = bds;
                }
                base += tot;
                gsync();
            }
            nb1 = base;
            const unsigned long long *ps = A.par_stat + (int64_t)wg * kSyncStats;
            st5[0] = ld_dev(&ps[0]);
            st5[1] = ld_dev(&ps[1]);
            st5[2] = ld_dev(&ps[2]);
            st5[3] = ld_dev(&ps[3]);
            st5[4] = ld_dev(&ps[4]);
            st5[5] = ld_dev(&ps[12]);
        } else {
            const int rstat = reduce_columns<kBT>(J, Dw, Gs, SC, L, RS);
            batch_red_status(A, rstat);
            nb1 = RS.nbars;
            st5[0] = RS.stat[0];
            st5[1] = RS.stat[1];
            st5[2] = RS.stat[2];
            st5[3] = RS.stat[3];
            st5[4] = RS.stat[4];
            st5[5] = RS.stat[12];
        }
        if (tid == 0) {
            rips_dim_stats &s1 = A.stats[(int64_t)b * D1 + 1];
            s1.candidates = (int64_t)Sh.cnt[0];
            s1.cleared = (int64_t)Sh.cnt[1];
            s1.apparent_col = (int64_t)Sh.cnt[2];
            s1.apparent_pivot = 0;
            s1.columns = S;
            s1.emergent = (int64_t)st5[0];
            s1.reduced = (int64_t)st5[1];
            s1.additions = (int64_t)st5[2];
            s1.bars_nonzero = (int64_t)st5[3];
            s1.entries_added = (int64_t)st5[5];
            s1.entries_stored = (int64_t)ld_dev(&A.v_count[wg]);
            s1.essential = (int64_t)st5[4];
        }
    }
    // ---- publish: one segment per dimension in the unordered buffer
    const int nb0 = Sh.nbars0;
    __shared__ unsigned long long s_base;
    if (tid == 0) s_base = atomicAdd(A.ucount, (unsigned long long)(nb0 + nb1));
    gsync();
    const int64_t base = (int64_t)s_base;
    const bool fits = base + nb0 + nb1 <= A.ucap;
    for (int q = tid; q < nb0 && fits; q += kBT) {
        A.ub[base + q] = sb_b[q];
        A.ud[base + q] = sb_d[q];
        A.ubs[base + q] = sb_bs[q];
        A.uds[base + q] = sb_ds[q];
    }
    // dimension 1: column order is youngest first, the canonical order its reverse
    for (int q = tid; q < nb1 && fits; q += kBT) {
        const int src = n + nb1 - 1 - q;
        A.ub[base + nb0 + q] = sb_b[src];
        A.ud[base + nb0 + q] = sb_d[src];
        A.ubs[base + nb0 + q] = sb_bs[src];
        A.uds[base + nb0 + q] = sb_ds[src];
    }
    if (tid == 0) {
        A.seg_start[(int64_t)b * D1] = base;
        A.seg_count[(int64_t)b * D1] = nb0;
        if (D1 > 1) {
            A.seg_start[(int64_t)b * D1 + 1] = base + nb0;
            A.seg_count[(int64_t)b * D1 + 1] = nb1;
        }
    }
    gsync();
}

template <class Dist>
__global__ void __launch_bounds__(kBT) k_batched(BatchArgs A) {
    extern __shared__ unsigned char smem[];
    __shared__ BatchShared Sh;
    __shared__ RedShared<kBT> RS;
    __shared__ SortShared<kBT> SS;
    if (A.spread > 1) {
        // a fixed workgroup set per cloud, all resident together (the grid
        // is at most the resident workgroups of the chip)
        const int w = blockIdx.x;
        const int slot = w / A.spread, role = w - slot * A.spread;
        if (slot >= A.B) return;
        if (role == 0) batch_cloud<Dist>(A, A.order[slot], smem, Sh, RS, SS);
        else batch_follow<Dist>(A, w - role, role, smem, Sh, RS, SS);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) Sh.cloud = (int)atomicAdd(A.queue, 1ull);
        __syncthreads();
        const int qi = Sh.cloud;
        __syncthreads();
        if (qi >= A.B) break;
        batch_cloud<Dist>(A, A.order[qi], smem, Sh, RS, SS);
    }
}

// clouds by decreasing size (longest processing time first); one block
__global__ void __launch_bounds__(1024) k_lpt_order(const int64_t *offsets, int B, SortBufs sb,
                                                    int *order, unsigned long long *queue,
                                                    unsigned long long *ucount, int *status,
                                                    int nmax) {
    __shared__ SortShared<1024> S;
    for (int b = threadIdx.x; b < B; b += 1024) {
        const int64_t n = offsets[b + 1] - offsets[b];
        if (n < 1 || n > nmax) atomicOr(status, 16);
        sb.lo[0][b] = (u64)b;
        sb.hi[0][b] = 0xffffffffu - (u32)(n < 0 ? 0 : n);
        sb.val[0][b] = (u32)b;
    }
    if (threadIdx.x == 0) {
        *queue = 0;
        *ucount = 0;
    }
    gsync();
    const int cur = block_radix_sort<1024>(sb, B, 4, 4, S);
    for (int q = threadIdx.x; q < B; q += 1024) order[q] = (int)sb.val[cur][q];
}

__global__ void k_batch_status_reset(int *status) { *status = 0; }

__global__ void k_batch_zero_words(int *w, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0;
}

int batched_spread(int B, int slots, int max_dim) {
    if (max_dim < 1 || B < 1) return 1;
    const int s = slots / B;
    return s < 2 ? 1 : (s > 8 ? 8 : s);
}

// canonical layout: segments in (cloud, dimension) order
__global__ void __launch_bounds__(1024) k_batch_offsets(const int64_t *seg_count, int nseg,
                                                        int64_t *offsets, int64_t *total) {
    __shared__ int64_t s_w[1024 / kWave + 1];
    int64_t carry = 0;
    for (int base = 0; base < nseg; base += 1024) {
        const int i = base + threadIdx.x;
        const int64_t x = i < nseg ? seg_count[i] : 0;
        const int lane = lane_id(), w = threadIdx.x / kWave;
        int64_t inc = x;
        for (int o = 1; o < kWave; o <<= 1) {
            int64_t t = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t acc = 0;
            for (int q = 0; q < 1024 / kWave; ++q) {
                int64_t t = s_w[q];
                s_w[q] = acc;
                acc += t;
            }
            s_w[1024 / kWave] = acc;
        }
        __syncthreads();
        if (i < nseg) offsets[i] = carry + s_w[w] + inc - x;
        carry += s_w[1024 / kWave];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        offsets[nseg] = carry;
        *total = carry;
    }
}

__global__ void k_batch_copy(const int64_t *seg_start, const int64_t *seg_count,
                             const int64_t *offsets, int nseg, const float *ub, const float *ud,
                             const int64_t *ubs, const int64_t *uds, int64_t cap, float *ob,
                             float *od, int64_t *obs, int64_t *ods) {
    const int sgi = blockIdx.x;
    if (sgi >= nseg) return;
    const int64_t src = seg_start[sgi], cnt = seg_count[sgi], dst = offsets[sgi];
    if (dst + cnt > cap) return;
    for (int64_t q = threadIdx.x; q < cnt; q += blockDim.x) {
        ob[dst + q] = ub[src + q];
        od[dst + q] = ud[src + q];
        obs[dst + q] = ubs[src + q];
        ods[dst + q] = uds[src + q];
    }
}

size_t batched_lds_bytes(bool lds_d, int nmax, u32 capD, bool bm) {
    const size_t npairs = (size_t)nmax * (nmax - 1) / 2;
    const size_t dpart = lds_d ? (npairs * 4 + 15) / 16 * 16 : 0;
    const size_t uf = (size_t)nmax * (8 + 4 + 4) + (lds_d ? (npairs / 32 + 1) * 4 : 0);
    return std::max(dpart + uf, reduce_lds_bytes(capD) + (bm ? bm_lds_bytes((int64_t)npairs) : 0));
}

// The direct-mapped working column needs W = ceil(nmax / 32) <= 60 words per
// edge (the pivot search reads one edge's bitmap words and four more words
// of the edge with one wave), a summary of
// C(nmax, 2) bits in LDS beside the general working column's, and
// C(nmax, 2) * W words of bitmaps and an nmax x nmax position table per
// workgroup (at most 8 GiB in all).
bool batched_bm_fits(int nmax, int max_dim, u32 p, int64_t grid) {
    const int64_t npairs = (int64_t)nmax * (nmax - 1) / 2;
    const int64_t W = (nmax + 31) / 32;
    return p == 2 && max_dim >= 1 && W <= 60 && npairs <= (1 << 18) &&
           grid * (npairs * W + (int64_t)nmax * nmax) * 4 <= (8ll << 30);
}

// default delta: the largest (kMaxDelta slots, about 94 KB of LDS with its
// staging and sorted base)
u32 batched_default_capD(bool lds_d, int nmax) {
    (void)lds_d;
    (void)nmax;
    return kMaxDelta;
}

hipError_t batched_prepare(bool lds_d, int nmax, u32 capD, bool bm) {
    const size_t lds = batched_lds_bytes(lds_d, nmax, capD, bm);
    return hipFuncSetAttribute(lds_d ? (const void *)k_batched<DistPacked>
                                     : (const void *)k_batched<DistFull>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

void launch_batched(const BatchArgs &A, bool lds_d, int grid, SortBufs lpt, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_status_reset, dim3(1), dim3(1), 0, st, A.status);
    if (A.spread > 1)
        hipLaunchKernelGGL(k_batch_zero_words, dim3(((int64_t)grid * kSyncWords + 255) / 256), dim3(256), 0,
                           st, A.sync, (int64_t)grid * kSyncWords);
    hipLaunchKernelGGL(k_lpt_order, dim3(1), dim3(1024), 0, st, A.offsets, A.B, lpt,
                       (int *)A.order, A.queue, A.ucount, A.status, A.nmax);
    const size_t lds = batched_lds_bytes(lds_d, A.nmax, A.capD, A.bm_bits != nullptr);
    if (lds_d) hipLaunchKernelGGL(k_batched<DistPacked>, dim3(grid), dim3(kBT), lds, st, A);
    else hipLaunchKernelGGL(k_batched<DistFull>, dim3(grid), dim3(kBT), lds, st, A);
}

void launch_batch_finalize(const BatchArgs &A, int64_t *offsets_out, int64_t *total, int64_t cap,
                           float *ob, float *od, int64_t *obs, int64_t *ods, hipStream_t st) {
    const int nseg = A.B * (A.max_dim + 1);
    hipLaunchKernelGGL(k_batch_offsets, dim3(1), dim3(1024), 0, st, A.seg_count, nseg, offsets_out,
                       total);
    hipLaunchKernelGGL(k_batch_copy, dim3(nseg), dim3(256), 0, st, A.seg_start, A.seg_count,
                       offsets_out, nseg, A.ub, A.ud, A.ubs, A.uds, cap, ob, od, obs, ods);
}

} // namespace rips
