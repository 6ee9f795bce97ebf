// rips_reduce.hpp -- the reduction of the surviving coboundary columns over
// Z/p as a workgroup-level device routine (Algorithm 1 on the implicit
// coboundary matrix of one dimension, columns already cleared; the emergent
// shortcut; pivot lookup = pivot table, then zero apparent facet). Used by
// the single-cloud kernel and by the batched persistent kernel.
#pragma once

#include "rips_kernels.hpp"

namespace rips {

// Working column (R_j or V_j): open addressing keyed by simplex index plus
// the list of used slots, so that pivot search, clearing and compaction cost
// O(entries touched) instead of O(capacity). Coefficients accumulate with
// atomics and are reduced mod p when read (XOR for p = 2).
struct WorkCol {
    int64_t *keys;
    u32 *coef;
    float *diam; // null for V (diameters recomputed when needed)
    u32 *slots;
    int *nslots; // in LDS
    u32 mask;
};

__device__ __forceinline__ bool wc_add(const WorkCol &h, int64_t key, float dm, u32 c, u32 p) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = ld(&h.keys[s]);
        bool mine = cur == key;
        if (!mine && cur == kEmpty) {
            const u64 prev = atomicCAS((u64 *)&h.keys[s], (u64)kEmpty, (u64)key);
            if (prev == (u64)kEmpty) {
                if (h.diam) h.diam[s] = dm;
                const int q = atomicAdd(h.nslots, 1);
                if ((u32)q <= h.mask) h.slots[q] = s;
                mine = true;
            } else mine = prev == (u64)key;
        }
        if (mine) {
            if (p == 2) atomicXor(&h.coef[s], c & 1u);
            else atomicAdd(&h.coef[s], c);
            return true;
        }
        s = (s + 1) & h.mask;
    }
    return false;
}

// Everything the routine needs about one dimension of one cloud.
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
    unsigned long long *vcount; // V append counter (global)
    BarBuf bars;                // capacity ncols
};

// Shared state of the routine (one per workgroup).
template <int BT>
struct RedShared {
    int base, full, abort, m, nbars, nitems, total;
    int64_t owner;
    unsigned long long vbase;
    PivotCand wp[BT / kWave];
    PivotCand piv;
    int w[BT / kWave + 1];
    unsigned long long stat[8];
    // one batch of coboundaries to add: simplex, coefficient, candidate
    // source and prefix offsets into the flattened (item, candidate) space
    int64_t it_idx[BT];
    u32 it_coef[BT];
    int it_v[BT][kMaxDim + 1];
    float it_diam[BT];
    int it_off[BT + 1];
    int it_u[BT];
};

template <int BT>
__device__ __forceinline__ int block_scan_excl(int x, int *s_w, int *total) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int inc = x;
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
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

// Barrier of the routine: a plain workgroup barrier while the working
// columns live in LDS, a fenced one when they live in global memory.
__device__ __forceinline__ void rsync(bool global) {
    if (global) gsync();
    else __syncthreads();
}

// Add the coboundaries of S.nitems simplices (S.it_*) with their
// coefficients to R: the (item, candidate) pairs are spread over the whole
// workgroup. Dense candidates: all n vertices; sparse: the neighbours of the
// item's vertex with the fewest neighbours. Coefficient of sigma u {j}:
// (-1)^(vertices of sigma below j) times the item's coefficient.
template <int BT, class Dist>
__device__ bool add_items(const ReduceJob<Dist> &J, RedShared<BT> &S, const WorkCol &R) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x;
    // per item: candidate source and count
    int cnt = 0;
    if (tid < S.nitems) {
        if (c.nb.off == nullptr) {
            cnt = c.n;
            S.it_u[tid] = -1;
        } else {
            int u = S.it_v[tid][0];
            int du = c.nb.off[u + 1] - c.nb.off[u];
            for (int m = 1; m <= k; ++m) {
                const int vm = S.it_v[tid][m];
                const int dd = c.nb.off[vm + 1] - c.nb.off[vm];
                if (dd < du) {
                    du = dd;
                    u = vm;
                }
            }
            S.it_u[tid] = u;
            cnt = du;
        }
    }
    int total;
    const int off = block_scan_excl<BT>(cnt, S.w, &total);
    if (tid < S.nitems) S.it_off[tid] = off;
    if (tid == 0) S.it_off[S.nitems] = total;
    __syncthreads();
    bool ok = true;
    for (int f = tid; f < total; f += BT) {
        // item holding flat index f: last it with it_off[it] <= f
        int lo = 0, hi = S.nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.it_off[mid] <= f) lo = mid;
            else hi = mid - 1;
        }
        const int it = lo;
        const int q = f - S.it_off[it];
        const int u = S.it_u[it];
        const int j = u < 0 ? q : c.nb.idx[c.nb.off[u] + q];
        const int *v = S.it_v[it];
        bool in = false;
        float nd = S.it_diam[it];
        for (int m = 0; m <= k; ++m) {
            in = in || (j == v[m]);
            nd = fmaxf(nd, c.d(v[m], j));
        }
        if (in || !(nd <= c.t)) continue;
        int below;
        const int64_t ci = cofacet_index(v, k, j, c.B, &below);
        const u32 coef = S.it_coef[it];
        const u32 cc = (below & 1) ? (p - coef) % p : coef;
        ok = ok && wc_add(R, ci, nd, cc, p);
    }
    return ok;
}

// Oldest nonzero entry of R (block-wide); coefficients normalised mod p.
template <int BT>
__device__ PivotCand wc_pivot(const WorkCol &R, u32 p, RedShared<BT> &S, bool g) {
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
    rsync(g);
    if (tid == 0) {
        PivotCand b = S.wp[0];
        for (int q = 1; q < BT / kWave; ++q)
            if (older(S.wp[q], b)) b = S.wp[q];
        S.piv = b;
    }
    rsync(g);
    return S.piv;
}

// Empty the used slots of a working column.
template <int BT>
__device__ void wc_reset(const WorkCol &h, bool g) {
    const int ns = min(*h.nslots, (int)h.mask + 1);
    for (int i = threadIdx.x; i < ns; i += BT) {
        const u32 s = h.slots[i];
        st(&h.keys[s], kEmpty);
        st(&h.coef[s], 0u);
    }
    rsync(g);
    if (threadIdx.x == 0) *h.nslots = 0;
    rsync(g);
}

// Empty a whole table (its contents are unknown).
template <int BT>
__device__ void wc_clear_all(const WorkCol &h, bool g) {
    for (u32 q = threadIdx.x; q <= h.mask; q += BT) {
        st(&h.keys[q], kEmpty);
        st(&h.coef[q], 0u);
    }
    rsync(g);
    if (threadIdx.x == 0) *h.nslots = 0;
    rsync(g);
}

// Drop the entries whose coefficient cancelled to zero once more than half
// the table is in use. Each thread moves at most kPer entries; tables hold at
// most 2 * kPer * BT slots.
template <int BT, int kPer>
__device__ void wc_compact(const WorkCol &h, u32 p, int *nslots_shared, bool g) {
    const int ns = min(*h.nslots, (int)h.mask + 1);
    if (2 * ns <= (int)h.mask + 1) return;
    if ((int)h.mask + 1 > 2 * kPer * BT) return; // larger tables are not compacted
    int64_t kk[kPer];
    u32 cc[kPer];
    float dd[kPer];
    int mine = 0;
    for (int i = threadIdx.x; i < ns && mine < kPer; i += BT) {
        const u32 s = h.slots[i];
        const u32 cf = ld(&h.coef[s]) % p;
        if (cf != 0) {
            kk[mine] = ld(&h.keys[s]);
            cc[mine] = cf;
            dd[mine] = h.diam ? h.diam[s] : 0.0f;
            ++mine;
        }
    }
    rsync(g);
    for (int i = threadIdx.x; i < ns; i += BT) {
        const u32 s = h.slots[i];
        st(&h.keys[s], kEmpty);
        st(&h.coef[s], 0u);
    }
    rsync(g);
    if (threadIdx.x == 0) *nslots_shared = 0;
    rsync(g);
    for (int q = 0; q < mine; ++q) wc_add(h, kk[q], dd[q], cc[q], p);
    rsync(g);
}

// Full reduction of column j with the working column R. Returns 0 when
// done, 1 on working-column overflow (nothing of column j has been published
// then), 2 on column store overflow, 3 on the addition bound.
template <int BT, class Dist>
__device__ int reduce_one(const ReduceJob<Dist> &J, const WorkCol &R, bool g, int j,
                          RedShared<BT> &S) {
    constexpr int kPer = 16;
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const int64_t sidx = J.cols.idx[j];
    const float sdm = J.cols.diam[j];
    if (tid == 0) {
        S.abort = 0;
        S.nitems = 1;
        S.it_idx[0] = sidx;
        S.it_coef[0] = 1u;
        S.it_diam[0] = sdm;
        decode(sidx, k, c.n, c.B, S.it_v[0]);
    }
    __syncthreads();
    if (!add_items<BT>(J, S, R)) S.abort = 1;
    int nadd = 0;
    int result = 0;
    for (;;) {
        rsync(g);
        if (S.abort) {
            result = S.abort;
            break;
        }
        // every addition moves the pivot to a strictly younger row, so the
        // loop ends; the bound only turns a fault into an error
        if (nadd > (1 << 16)) {
            result = 3;
            break;
        }
        wc_compact<BT, kPer>(R, p, R.nslots, g);
        const PivotCand piv = wc_pivot<BT>(R, p, S, g);
        if (piv.idx == kEmpty) {
            // zero column: essential class born at sigma
            if (tid == 0) {
                if (S.nbars < J.ncols) {
                    J.bars.birth[S.nbars] = sdm;
                    J.bars.death[S.nbars] = INFINITY;
                    J.bars.bs[S.nbars] = sidx;
                    J.bars.ds[S.nbars] = -1;
                    S.nbars++;
                }
                S.stat[4] += 1;
            }
            break;
        }
        if (tid == 0) S.owner = ph_find(J.ph, piv.idx);
        __syncthreads();
        const int64_t o = S.owner;
        if (o >= 0) {
            // R_j -= lambda R_o, lambda = piv / pivot(R_o)
            const u32 lam = (u32)((u64)piv.coef * J.inv[J.V.pivcoef[o]] % p);
            const u32 neg = (p - lam) % p;
            const int len = J.V.len[o];
            if (len < 0) {
                // emergent column: R_o is the coboundary of sigma_o
                if (tid == 0) {
                    S.nitems = 1;
                    S.it_idx[0] = J.cols.idx[o];
                    S.it_coef[0] = neg;
                    S.it_diam[0] = J.cols.diam[o];
                    decode(J.cols.idx[o], k, c.n, c.B, S.it_v[0]);
                }
                __syncthreads();
                if (!add_items<BT>(J, S, R)) S.abort = 1;
            } else {
                const int64_t off = J.V.off[o];
                bool ok = true;
                for (int e = tid; e < len; e += BT) {
                    const u32 cc = (u32)((u64)neg * J.V.coef[off + e] % p);
                    ok = ok && wc_add(R, J.V.idx[off + e], J.V.diam[off + e], cc, p);
                }
                if (!ok) S.abort = 1;
            }
            ++nadd;
            continue;
        }
        // not in the table: is the pivot in a zero apparent pair (rho, tau)?
        if (w == 0) {
            int tv[kMaxVerts];
            decode(piv.idx, k + 1, c.n, c.B, tv);
            const int m = zero_apparent_facet<kWave>(c, tv, k + 1, piv.diam);
            if (lane == 0) {
                S.m = m;
                if (m >= 0) {
                    int rv[kMaxVerts];
                    remove_vertex(tv, k + 1, m, rv);
                    // tau = rho u {tau[m]}; vertices of rho below tau[m]: k + 1 - m
                    const u32 crho = coeff_sign(k + 1 - m, p);
                    const u32 lam = (u32)((u64)piv.coef * J.inv[crho] % p);
                    S.nitems = 1;
                    for (int q = 0; q <= k; ++q) S.it_v[0][q] = rv[q];
                    S.it_idx[0] = simplex_index(rv, k, c.B);
                    S.it_coef[0] = (p - lam) % p;
                    S.it_diam[0] = piv.diam;
                }
            }
        }
        __syncthreads();
        if (S.m >= 0) {
            if (!add_items<BT>(J, S, R)) S.abort = 1;
            ++nadd;
            continue;
        }
        // unowned pivot: persistence pair (sigma_j, pivot); keep R_j
        const int ns = min(*R.nslots, (int)R.mask + 1);
        int cnt = 0;
        for (int i = tid; i < ns; i += BT) cnt += (ld(&R.coef[R.slots[i]]) % p) != 0 ? 1 : 0;
        int tot;
        const int ex = block_scan_excl<BT>(cnt, S.w, &tot);
        if (tid == 0) S.vbase = atomicAdd(J.vcount, (unsigned long long)tot);
        __syncthreads();
        const int64_t vb = (int64_t)S.vbase;
        if (vb + tot > J.V.cap) {
            result = 2;
            break;
        }
        int at = ex;
        for (int i = tid; i < ns; i += BT) {
            const u32 s = R.slots[i];
            const u32 cf = ld(&R.coef[s]) % p;
            if (cf != 0) {
                J.V.idx[vb + at] = ld(&R.keys[s]);
                J.V.diam[vb + at] = R.diam[s];
                J.V.coef[vb + at] = cf;
                ++at;
            }
        }
        if (tid == 0) {
            if ((unsigned long long)tot > S.stat[6]) S.stat[6] = tot;
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
            J.V.pivcoef[j] = piv.coef;
            J.V.off[j] = vb;
            J.V.len[j] = tot;
        }
        break;
    }
    if (tid == 0 && result == 0) {
        S.stat[1] += nadd > 0 ? 1 : 0;
        S.stat[2] += nadd;
    }
    if (tid == 0 && (unsigned long long)*R.nslots > S.stat[7]) S.stat[7] = *R.nslots;
    wc_reset<BT>(R, g);
    return result;
}

// The reduction of J.ncols columns by one workgroup of BT threads. A working
// column starts in the LDS table Rl; a column that outgrows it is redone with
// the global table Rg. Returns 0, or 1 (global working column overflow), 2
// (column store overflow), 3 (addition bound).
// Stats: S.stat = emergent, reduced, additions, bars_nonzero, essential.
template <int BT, class Dist>
__device__ int reduce_columns(const ReduceJob<Dist> &J, const WorkCol &Rl, const WorkCol &Rg,
                              RedShared<BT> &S) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const u32 p = J.p;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const bool lds_ok = Rl.keys != nullptr;
    if (lds_ok) wc_clear_all<BT>(Rl, false);
    bool g_clean = false;
    if (tid == 0) {
        S.base = 0;
        S.abort = 0;
        S.nbars = 0;
    }
    if (tid < 8) S.stat[tid] = 0;
    int status = 0;
    gsync();
    for (;;) {
        __syncthreads();
        const int base = S.base;
        const int stop = base >= J.ncols;
        __syncthreads(); // everyone has read the cursor before wave 0 moves it
        if (stop || status) break;
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
            if (valid) {
                const int j = J.cols.j[col];
                if (j >= 0 && !J.cols.tapp[col]) {
                    int v[kMaxVerts];
                    decode(J.cols.idx[col], k, c.n, c.B, v);
                    int below;
                    tau = cofacet_index(v, k, j, c.B, &below);
                    tcoef = coeff_sign(below, p);
                    ok = ph_find(J.ph, tau) < 0;
                }
            }
            for (int l = 0; l < kWave - 1; ++l) {
                const int64_t tl = __shfl(tau, l, kWave);
                const int okl = __shfl((int)ok, l, kWave);
                if (l < lane && okl && tl == tau) ok = false;
            }
            const u64 bad = __ballot(!ok);
            const int first_bad = bad ? __ffsll((unsigned long long)bad) - 1 : kWave;
            if (lane < first_bad) {
                ph_insert(J.ph, tau, col);
                J.V.pivcoef[col] = tcoef;
                J.V.len[col] = -1; // R_col is the coboundary of sigma_col
                J.V.off[col] = 0;
            }
            if (lane == 0) {
                S.base = base + first_bad;
                S.full = (first_bad < kWave) && (base + first_bad < J.ncols);
                S.stat[0] += first_bad;
            }
        }
        gsync(); // V metadata of the batch is visible to every wave
        if (!S.full) continue;
        const int j = S.base;
        int r = 1;
        if (lds_ok) r = reduce_one<BT>(J, Rl, false, j, S);
        if (r == 1) {
            if (tid == 0) S.stat[5] += 1;
            if (!g_clean) {
                wc_clear_all<BT>(Rg, true);
                g_clean = true;
            }
            r = reduce_one<BT>(J, Rg, true, j, S);
        }
        status = r;
        if (tid == 0) S.base = j + 1;
        gsync(); // V_j and the table entry are visible before the next column
    }
    gsync();
    return status;
}

size_t reduce_lds_bytes(u32 capR);
hipError_t launch_reduce(const ReduceJob<DistFull> &J, WorkCol Rl, WorkCol Rg, int use_lds,
                         Scalars *s, hipStream_t st);

} // namespace rips
