// rips_batched.hpp -- arguments of the batched persistent kernel.
#pragma once

#include "../../include/rips.h"
#include "rips_reduce.hpp"

namespace rips {

constexpr int kBatchMaxN = 2048; // largest cloud of the batched path
constexpr int kBatchLdsN = 256;  // clouds up to this size keep D in LDS

struct BatchArgs {
    const float *X;          // points, cloud b at rows [offsets[b], offsets[b+1])
    const int64_t *offsets;  // B + 1
    int B, m, max_dim;
    float threshold;
    u32 p;
    const u32 *inv;
    Binom binom;             // table for n <= nmax
    int nmax;
    const int *order;        // clouds by decreasing size
    unsigned long long *queue;
    // per-workgroup scratch, indexed by blockIdx.x
    float *Dg;               // packed (LDS variant) or full (global variant) distances
    int64_t d_stride;
    int64_t *c_idx0, *c_idx1;  // candidate columns / sorted columns (idx)
    float *c_dm0, *c_dm1;
    int *c_j0, *c_j1;
    uint8_t *c_t0, *c_t1;
    u64 *s_lo0, *s_lo1;
    u32 *s_hi0, *s_hi1, *s_v0, *s_v1;
    int64_t col_stride;      // C(nmax, 2)
    int64_t *ph_keys;
    int32_t *ph_vals;
    int64_t ph_stride;       // power of two >= 2 C(nmax,2) + 64
    int64_t *app_keys;       // zero apparent pairs of dimension 1 (PairHash), ph_stride slots
    int64_t *app_vals;
    u64 *app_verts;
    int64_t *v_off;
    int *v_len;
    u32 *v_piv;
    int64_t *v_idx;
    float *v_diam;
    u32 *v_coef;
    int64_t v_stride;        // column-store capacity per workgroup
    unsigned long long *v_count; // per workgroup
    u32 *bits_g;             // forest-edge bitmap per workgroup (global variant)
    int64_t bits_stride;
    u32 capD;                // LDS delta slots of the working column (power of two)
    int64_t *f_idx[2];       // far list of the working column, two buffers
    float *f_dia[2];
    u32 *f_coef[2];
    int64_t f_stride;        // far-list entries per workgroup and buffer
    int64_t *vw_keys;        // working V column (table)
    u32 *vw_coef;
    float *vw_diam;
    u32 *vw_slots;
    int64_t vw_stride;       // its slots per workgroup (power of two)
    int64_t *v_roff;         // per column: stored R_j, if any
    int *v_rlen;
    int64_t *log_key;        // addition log of the column being reduced
    u32 *log_coef;
    float *log_dia;
    int64_t log_stride;
    float *st_b, *st_d;      // staged bars of the current cloud
    int64_t *st_bs, *st_ds;
    int64_t st_stride;       // nmax + C(nmax, 2)
    // results
    float *ub, *ud;          // unordered bars
    int64_t *ubs, *uds;
    int64_t ucap;
    unsigned long long *ucount;
    int64_t *seg_start, *seg_count; // B * (max_dim + 1)
    rips_dim_stats *stats;          // B * (max_dim + 1)
    float *t_used;                  // B
    int *status;
    // direct-mapped working column of dimension 1 (Z/2), or bm_bits == null:
    // per workgroup the edge order (C(nmax, 2) entries each) and the bitmaps
    int *bm_pos;
    u32 *bm_verts;
    float *bm_len;
    u32 *bm_run;
    int64_t bm_pos_stride;          // nmax * nmax: the n x n position table of each workgroup
    int *bm_app;                    // position -> third vertex of its zero apparent cofacet, or -1
    int *bm_appe;                   // the same by edge index, written by the filter
    int64_t bm_tab_stride;          // C(nmax, 2)
    u32 *bm_bits;                   // all zero between columns
    int64_t bm_stride;              // C(nmax, 2) * ceil(nmax / 32) words
    // workgroups per cloud: 1 = one workgroup per cloud, clouds from the
    // queue; s > 1 (a batch smaller than the chip) = workgroup w works on
    // cloud order[w / s]: w % s == 0 leads it (distances to edge order) and
    // all s reduce its columns together (the spread-out reduction)
    int spread;
    int *sync;                      // kSyncWords per workgroup (its cloud's leader's are used)
    u32 *par_cst;                   // per workgroup col_stride words: column states
    u32 *par_ctl;                   // per workgroup kCtlWords words: cursor, frontier, abort
    unsigned long long *par_stat;   // per workgroup kSyncStats counters of the reduction
};

// The words a cloud's leader shares with the other workgroups of its cloud
// (spread > 1), zeroed before every launch: ready flag (columns sorted, the
// reduction may start), n, t (bits), columns, edges of the edge order, skip
// (the cloud has no reduction), reductions done; with the distances in
// global memory also: front flag (distances and threshold done, the filter
// may start), survivors appended, workgroups done filtering, edge order
// done, edges handed out to the filter.
enum : int { kSyncReady = 0, kSyncN = 1, kSyncT = 2, kSyncS = 3, kSyncE = 4, kSyncSkip = 5,
             kSyncDone = 6, kSyncFront = 7, kSyncSurv = 8, kSyncFiltered = 9, kSyncOrdered = 10,
             kSyncChunk = 11, kSyncWords = 16 };
constexpr int kSyncStats = 16;


size_t batched_lds_bytes(bool lds_d, int nmax, u32 capD, bool bm);
u32 batched_default_capD(bool lds_d, int nmax);
hipError_t batched_prepare(bool lds_d, int nmax, u32 capD, bool bm);
void launch_batched(const BatchArgs &A, bool lds_d, int grid, SortBufs lpt, hipStream_t st);
// workgroups per cloud for a batch of B clouds on `slots` resident workgroups
int batched_spread(int B, int slots, int max_dim);
// whether the batched path can use the direct-mapped working column
bool batched_bm_fits(int nmax, int max_dim, u32 p, int64_t grid);
void launch_batch_finalize(const BatchArgs &A, int64_t *offsets_out, int64_t *total, int64_t cap,
                           float *ob, float *od, int64_t *obs, int64_t *ods, hipStream_t st);

} // namespace rips
