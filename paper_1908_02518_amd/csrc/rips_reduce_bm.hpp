// rips_reduce_bm.hpp -- the reduction of the dimension-1 columns over Z/2
// with a direct-mapped working column (included by rips_reduce.hpp).
//
// The rows of a dimension-1 coboundary column are triangles. The edges <= t
// are put in order of length once per dimension (position = rank; equal
// lengths in any order). A triangle's "owner" is its edge of the latest
// position, so the triangle's diameter (the length of its longest edge) is
// the owner's length, and among the triangles of one edge {a, b} the CNS
// index grows with the third vertex c. The working column R_j is therefore
// held as one bit per (owner position, third vertex): bit c of position e is
// set when the triangle {a_e, b_e, c} is in R_j (over Z/2 an addition is an
// XOR), and a triangle's coordinate needs the positions of its three edges
// only, no distances. The oldest entry (smallest diameter, then largest
// index) is the highest set bit of the first edge position with a set bit,
// compared across the run of positions of exactly that length. A summary in
// LDS marks the positions that may hold set bits (one bit per position, and
// one bit per 32 of those); it is cleared lazily as the pivot search finds
// positions empty. The pivot only moves to younger rows while a column is
// reduced, so the search starts from a front that only moves forward.
//
// Zero apparent pairs (section "Apparent pairs"): when no other edge has the
// owner's length, a triangle's only facet of its own diameter is its owner,
// so the triangle is in a zero apparent pair exactly when it is the owner's
// zero apparent cofacet. The third vertex of that cofacet is kept per
// position (EdgeOrder::app) and read in the same round trip as the bitmap
// words, so such a pivot needs no table lookup; a pivot in a run of equal
// lengths, or not paired so, is looked up in the pair and pivot tables.
//
// Compared with the general working column (delta, sorted base, far list)
// there is no merge, no sorting and no spill: an addition costs one XOR per
// entry, and the column's size does not matter. The memory is
// (edges <= t) x ceil(n / 32) words per workgroup and an n x n table of edge
// positions, so the engine is used when that fits; the rest of the reduction (the pivot and apparent-pair tables,
// the addition log, V_j, the commit of the spread-out reduction) is the
// general one's.
#pragma once

namespace rips {

// Triangle {a, b, c} (any order) -> CNS index: with x > y > z,
// C(x, 3) + C(y, 2) + C(z, 1).
__device__ __forceinline__ int64_t bm_tri_index(int a, int b, int c) {
    int x = a, y = b, z = c, t;
    if (x < y) { t = x; x = y; y = t; }
    if (y < z) { t = y; y = z; z = t; }
    if (x < y) { t = x; x = y; y = t; }
    return (int64_t)x * (x - 1) * (x - 2) / 6 + (int64_t)y * (y - 1) / 2 + z;
}

__device__ __forceinline__ int64_t bm_edge_index(int a, int b) {
    const int x = max(a, b), y = min(a, b);
    return (int64_t)x * (x - 1) / 2 + y;
}

// Bitmap coordinate of the triangle {u, v, w}, puv the position of the edge
// uv: the owner is the edge of the latest position, the coordinate its
// position and the vertex off it; -1 when w is u or v, or when an edge is
// longer than t (no position).
__device__ __forceinline__ int64_t bm_coord(const EdgeOrder &eo, int u, int v, int puv, int w) {
    if (w == u || w == v) return -1;
    const int puw = gp(eo.pos)[(int64_t)u * eo.n + w];
    const int pvw = gp(eo.pos)[(int64_t)v * eo.n + w];
    if (puw < 0 || pvw < 0) return -1;
    int po = puv, cc = w;
    if (puw > po) {
        po = puw;
        cc = v;
    }
    if (pvw > po) {
        po = pvw;
        cc = u;
    }
    return ((int64_t)po << 16) | cc;
}

// XOR one entry into the working column and mark its position in the
// summary (any thread; LDS and global atomics at workgroup scope).
__device__ __forceinline__ void bm_flip(u32 *bits, const BmLds &L, int W, int64_t coord) {
    const int pos = (int)(coord >> 16), cc = (int)(coord & 0xffff);
    __hip_atomic_fetch_xor(gp(&bits[(int64_t)pos * W + (cc >> 5)]), 1u << (cc & 31), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_or(&L.l1[pos >> 5], 1u << (pos & 31), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_or(&L.l2[pos >> 10], 1u << ((pos >> 5) & 31), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until every memory operation the wave issued has completed, the
// XORs of bm_flip included (s_waitcnt vmcnt(0) expcnt(0) lgkmcnt(0)); the
// words they changed are read next, by this wave or, after a barrier, by
// the others.
__device__ __forceinline__ void bm_wait_flips() { __builtin_amdgcn_s_waitcnt(0); }

// First position >= f whose summary bit is set, or -1 (wave 0; the result
// in every lane). Stale second-level bits met on the way are cleared.
__device__ __forceinline__ int bm_next(const BmLds &L, int f) {
    const int lane = lane_id();
    if (f >= L.E) return -1;
    wave_sync(); // summary bits lane 0 cleared in this wave's last look
    int w1 = f >> 5;
    const u32 first = L.l1[w1] & (~0u << (f & 31));
    if (first) return (w1 << 5) + __ffs((int)first) - 1;
    int i = w1 + 1; // next first-level word to look at
    while (i < L.n1) {
        // second level from bit i: 64 words of it at a time
        const int w2 = (i >> 5) + lane;
        u32 x = w2 < L.n2 ? L.l2[w2] : 0u;
        if (lane == 0) x &= ~0u << (i & 31);
        const u64 nz = __ballot(x != 0);
        if (!nz) {
            i = ((i >> 5) + kWave) << 5;
            continue;
        }
        const int ln = __ffsll((unsigned long long)nz) - 1;
        const u32 xw = lane_bcast(x, ln);
        const int j = (((i >> 5) + ln) << 5) + __ffs((int)xw) - 1; // first-level word
        const u32 y = L.l1[j];
        if (y) return (j << 5) + __ffs((int)y) - 1;
        if (lane == 0)
            __hip_atomic_fetch_and(&L.l2[j >> 5], ~(1u << (j & 31)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        wave_sync();
        i = j + 1;
    }
    return -1;
}

// The oldest live entry of the working column (wave 0 calls it; the result
// in every lane of wave 0): smallest diameter, then largest index. The
// marked positions from *front on are checked a few at a time: one round
// trip reads the bitmaps of up to kBmSlots of them (W lanes each) with each
// one's length, run word, vertices and apparent vertex (four more lanes).
// Empty ones are unmarked and passed; *front then stays at the first
// position of the pivot's run of equal lengths, where an entry younger than
// the pivot may still be added (never before it).
constexpr int kBmSlots = 6;
constexpr u32 kNoRho = 0xffffffffu;
constexpr int kBmStoreAdds = 256; // longest column whose R_j is stored (V_j always is)

// The highest set bit of a position's bitmap (lanes base .. base+W-1 hold
// its words, nz their nonzero mask): the third vertex of its oldest entry.
__device__ __forceinline__ int bm_top_vertex(u32 w, u64 nz, int base) {
    const int hl = 63 - __clzll((long long)nz);
    const u32 hw = lane_bcast(w, hl);
    return (hl - base) * 32 + 31 - __clz((int)hw);
}

// *rho: when the pivot is in a zero apparent pair found through
// EdgeOrder::app, the vertices (a << 16 | b) of its partner edge; else kNoRho.
__device__ __forceinline__ PivotCand bm_pivot(const EdgeOrder &eo, const u32 *bits, const BmLds &L,
                                              int *front, u32 *rho) {
    const int lane = lane_id();
    const int W = eo.W;
    // a slot: W bitmap words, then length, run word, vertices, apparent vertex
    const int SL = W + 4;
    const int P = min(kBmSlots, kWave / SL);
    PivotCand out;
    out.idx = kEmpty;
    out.diam = 0.0f;
    out.coef = 1u;
    *rho = kNoRho;
    int f = *front;
    for (;;) {
        // up to P marked positions from f (LDS only)
        int ps[kBmSlots];
        int np = 0, g = f;
#pragma unroll
        for (int q = 0; q < kBmSlots; ++q) {
            ps[q] = -1;
            if (q < P && g >= 0) {
                const int pp = bm_next(L, g);
                ps[q] = pp;
                np += pp >= 0 ? 1 : 0;
                g = pp >= 0 ? pp + 1 : -1;
            }
        }
        if (np == 0) {
            f = L.E;
            break;
        }
        // one round trip: slot q = lanes [q*SL, q*SL + W) bitmap words,
        // then (lanes q*SL + W ..) its length, run word, vertices and the
        // third vertex of its zero apparent cofacet
        const int q = lane / SL, r = lane - q * SL;
        int mypos = -1;
#pragma unroll
        for (int qq = 0; qq < kBmSlots; ++qq) mypos = qq == q ? ps[qq] : mypos;
        u32 w = 0, mw = 0;
        if (q < np && mypos >= 0) {
            if (r < W) w = ld(gp(&bits[(int64_t)mypos * W + r]));
            else if (r == W) mw = __float_as_uint(gp(eo.len)[mypos]);
            else if (r == W + 1) mw = gp(eo.run)[mypos];
            else if (r == W + 2) mw = gp(eo.verts)[mypos];
            else mw = (u32)gp(eo.app)[mypos];
        }
        const u64 nz = __ballot(w != 0);
        // first slot with a set bit
        int live = -1;
        for (int qq = 0; qq < np; ++qq) {
            const u64 m = ((1ull << W) - 1) << (qq * SL);
            if (nz & m) {
                live = qq;
                break;
            }
        }
        // unmark the empty slots before it
        const int nempty = live < 0 ? np : live;
        if (lane == 0)
            for (int qq = 0; qq < nempty; ++qq) {
                int pp = -1;
#pragma unroll
                for (int z = 0; z < kBmSlots; ++z) pp = z == qq ? ps[z] : pp;
                const u32 bit = 1u << (pp & 31);
                const u32 was = __hip_atomic_fetch_and(&L.l1[pp >> 5], ~bit, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if ((was & ~bit) == 0)
                    __hip_atomic_fetch_and(&L.l2[pp >> 10], ~(1u << ((pp >> 5) & 31)), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        if (live < 0) {
            int last = -1;
#pragma unroll
            for (int z = 0; z < kBmSlots; ++z) last = z == np - 1 ? ps[z] : last;
            f = last + 1;
            continue;
        }
        int pos = -1;
#pragma unroll
        for (int z = 0; z < kBmSlots; ++z) pos = z == live ? ps[z] : pos;
        const int base = live * SL;
        const u64 mlive = (((1ull << W) - 1) << base) & nz;
        const int cc = bm_top_vertex(w, mlive, base);
        const float dm = __uint_as_float(lane_bcast(mw, base + W));
        const u32 run = lane_bcast(mw, base + W + 1);
        const u32 ab = lane_bcast(mw, base + W + 2);
        const int app = (int)lane_bcast(mw, base + W + 3);
        out.idx = bm_tri_index((int)(ab >> 16), (int)(ab & 0xffffu), cc);
        out.diam = dm;
        f = (int)(run & ~kRunTie);
        // alone in its run: the pivot's only facet of its diameter is the
        // owner edge, and EdgeOrder::app decides the zero apparent pair
        if ((run & kRunTie) == 0 && f == pos && app == cc) *rho = ab;
        // positions after pos of exactly the same length: their triangles tie
        // on the diameter, and the largest index among them is the oldest
        bool tie = (run & kRunTie) != 0;
        for (int qp = pos + 1; tie && qp < eo.E; ++qp) {
            const u32 rq = gp(eo.run)[qp];
            if ((L.l1[qp >> 5] >> (qp & 31)) & 1u) {
                u32 wq = 0;
                if (lane < W) wq = ld(gp(&bits[(int64_t)qp * W + lane]));
                const u64 nq = __ballot(wq != 0);
                if (nq) {
                    const u32 abq = gp(eo.verts)[qp];
                    const int64_t iq =
                        bm_tri_index((int)(abq >> 16), (int)(abq & 0xffffu), bm_top_vertex(wq, nq, 0));
                    if (iq > out.idx) out.idx = iq;
                }
            }
            tie = (rq & kRunTie) != 0;
        }
        break;
    }
    *front = f;
    return out;
}

// Add the coboundaries of the S.nit edges in S.it_v to the working column:
// the (edge, candidate vertex) pairs are spread over the workgroup; dense
// candidates are all vertices, sparse ones the neighbours of the edge's
// vertex with the fewer neighbours (as in add_items).
template <int BT, class Dist>
__device__ __forceinline__ void bm_add_items(const ReduceJob<Dist> &J, RedShared<BT> &S, u32 *bits,
                                             const BmLds &L) {
    // values, not references into the job (which may live in scratch memory)
    const Ctx<Dist> c = J.c;
    const EdgeOrder eo = J.eo;
    const int tid = threadIdx.x;
    const int nit = S.nit;
    // one edge, every vertex a candidate: each thread loads the edge
    // positions of up to kRounds candidates at once, then flips (no barrier
    // before: the item was written before the caller's barrier)
    constexpr int kRounds = 8;
    if (nit == 1 && c.nb.off == nullptr && c.n <= kRounds * BT) {
        RED_TW0(t_fl, tid == 0);
        const int u = S.it_v[0][0], v = S.it_v[0][1];
        const int puv = gp(eo.pos)[(int64_t)u * eo.n + v];
        const int rounds = (c.n + BT - 1) / BT;
        int64_t cd[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int w = r * BT + tid;
            cd[r] = (r < rounds && w < c.n) ? bm_coord(eo, u, v, puv, w) : -1;
        }
        unsigned long long added = 0;
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            if (cd[r] >= 0) {
                bm_flip(bits, L, eo.W, cd[r]);
                ++added;
            }
        }
        if (added) atomicAdd(&S.stat[12], added);
        bm_wait_flips();
        RED_TW1(S, 21, t_fl, tid == 0);
        __syncthreads(); // the flips are done, and the item read, before anyone goes on
        return;
    }
    int cnt = 0;
    if (tid < nit) {
        if (c.nb.off == nullptr) {
            S.it_u[tid] = -1;
            S.it_start[tid] = 0;
            cnt = c.n;
        } else {
            const int u = S.it_v[tid][0], v = S.it_v[tid][1];
            const int lu = c.nb.off[u], du = c.nb.off[u + 1] - lu;
            const int lv = c.nb.off[v], dv = c.nb.off[v + 1] - lv;
            S.it_u[tid] = dv < du ? v : u;
            S.it_start[tid] = dv < du ? lv : lu;
            cnt = dv < du ? dv : du;
        }
    }
    int total;
    const int off = block_scan_excl<BT>(cnt, S.w, &total);
    if (tid < nit) S.it_off[tid] = off;
    if (tid == 0) S.it_off[nit] = total;
    __syncthreads();
    unsigned long long added = 0;
    for (int fl = tid; fl < total; fl += BT) {
        int lo = 0, hi = nit - 1; // last item with it_off <= fl
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.it_off[mid] <= fl) lo = mid;
            else hi = mid - 1;
        }
        const int q = fl - S.it_off[lo];
        const int w = S.it_u[lo] < 0 ? q : c.nb.idx[S.it_start[lo] + q];
        const int u = S.it_v[lo][0], v = S.it_v[lo][1];
        const int64_t cd = bm_coord(eo, u, v, gp(eo.pos)[(int64_t)u * eo.n + v], w);
        if (cd >= 0) {
            bm_flip(bits, L, eo.W, cd);
            ++added;
        }
    }
    if (added) atomicAdd(&S.stat[12], added);
    bm_wait_flips();
    __syncthreads(); // the flips are done, and the items read, before anyone goes on
}

// Add a stored reduced column R_o (entries in bitmap coordinates).
template <int BT>
__device__ __forceinline__ void bm_add_r(const VStore &V, int64_t off, int len, u32 *bits,
                                         const BmLds &L, int W, RedShared<BT> &S) {
    for (int e = threadIdx.x; e < len; e += BT) bm_flip(bits, L, W, gp(V.idx)[off + e]);
    if (threadIdx.x == 0) S.stat[12] += (unsigned long long)len;
    bm_wait_flips();
    __syncthreads();
}

// Live entries of the working column from the front on (all threads).
template <int BT>
__device__ __forceinline__ int64_t bm_count(const u32 *bits, const BmLds &L, int W, int f,
                                            RedShared<BT> &S) {
    int cnt = 0;
    for (int i = (f >> 5) + threadIdx.x; i < L.n1; i += BT) {
        u32 m = L.l1[i];
        while (m) {
            const int pos = (i << 5) + __ffs((int)m) - 1;
            m &= m - 1;
            for (int q = 0; q < W; ++q) cnt += __popc(ld(gp(&bits[(int64_t)pos * W + q])));
        }
    }
    int tot;
    (void)block_scan_excl<BT>(cnt, S.w, &tot);
    return tot;
}

// Append the live entries (bitmap coordinates) to the column store; returns
// the count, or -1 when the store is full (all threads).
template <int BT>
__device__ __forceinline__ int bm_store(const u32 *bits, const BmLds &L, int W, int f, const VStore &V,
                                        unsigned long long *vcount, RedShared<BT> &S, int64_t *off_out) {
    int cnt = 0;
    for (int i = (f >> 5) + threadIdx.x; i < L.n1; i += BT) {
        u32 m = L.l1[i];
        while (m) {
            const int pos = (i << 5) + __ffs((int)m) - 1;
            m &= m - 1;
            for (int q = 0; q < W; ++q) cnt += __popc(ld(gp(&bits[(int64_t)pos * W + q])));
        }
    }
    int tot;
    int at = block_scan_excl<BT>(cnt, S.w, &tot);
    if (threadIdx.x == 0) S.vbase = atomicAdd(vcount, (unsigned long long)tot);
    __syncthreads();
    const int64_t vb = (int64_t)S.vbase;
    if (vb + tot > V.cap) return -1;
    for (int i = (f >> 5) + threadIdx.x; i < L.n1; i += BT) {
        u32 m = L.l1[i];
        while (m) {
            const int pos = (i << 5) + __ffs((int)m) - 1;
            m &= m - 1;
            for (int q = 0; q < W; ++q) {
                u32 x = ld(gp(&bits[(int64_t)pos * W + q]));
                while (x) {
                    const int cc = q * 32 + __ffs((int)x) - 1;
                    x &= x - 1;
                    gp(V.idx)[vb + at] = ((int64_t)pos << 16) | cc;
                    gp(V.diam)[vb + at] = 0.0f;
                    gp(V.coef)[vb + at] = 1u;
                    ++at;
                }
            }
        }
    }
    *off_out = vb;
    return tot;
}

// Empty the working column: the bitmaps of every marked position, then the
// summary (all threads). A position whose summary bit is clear has an empty
// bitmap, so this clears everything.
template <int BT>
__device__ __forceinline__ void bm_clear(u32 *bits, const BmLds &L, int W) {
    for (int i = threadIdx.x; i < L.n1; i += BT) {
        u32 m = L.l1[i];
        while (m) {
            const int pos = (i << 5) + __ffs((int)m) - 1;
            m &= m - 1;
            for (int q = 0; q < W; ++q) st(gp(&bits[(int64_t)pos * W + q]), 0u);
        }
    }
    bm_wait_flips();
    __syncthreads();
    for (int i = threadIdx.x; i < L.n1; i += BT) L.l1[i] = 0u;
    for (int i = threadIdx.x; i < L.n2; i += BT) L.l2[i] = 0u;
    __syncthreads();
}

// Full reduction of column j with the direct-mapped working column: the
// steps of reduce_one (same pivot tests, additions, log, stores and commit),
// for k = 1 over Z/2 with every shortcut on.
template <int BT, class Dist, bool kPar>
__device__ __forceinline__ int reduce_one_bm(const ReduceJob<Dist> &J, const LdsCol &D,
                                             const ReduceScratch &SC, const BmLds &L, int j,
                                             RedShared<BT> &S) {
    const Ctx<Dist> &c = J.c;
    const int k = J.k;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const int W = J.eo.W;
    u32 *bits = J.bm_bits + (int64_t)blockIdx.x * J.bm_stride;
    const int64_t sidx = J.cols.idx[j];
    const float sdm = J.cols.diam[j];
    if (tid == 0) {
        S.abort = 0;
        S.bmf = 0;
        S.nlog = 0;
        S.vest = 1;
        S.nit = 1;
        S.it_coef[0] = 1u;
        S.it_diam[0] = sdm;
        decode(sidx, k, c.n, c.B, S.it_v[0]);
        if (kPar) {
            S.pub = __float_as_uint(sdm);
            st_dev(&J.par.cst[j], S.pub);
        }
    }
    __syncthreads();
    bm_add_items<BT>(J, S, bits, L);
    int result = kRedOk;
    int nadd = 0;
    for (;;) {
        if (nadd > kMaxAdditions) {
            result = kRedBound;
            break;
        }
        // the pivot and both table lookups, by wave 0 (one barrier)
        RED_T0(t_piv);
        if (w == 0) {
            int f = S.bmf;
            const EdgeOrder eo = J.eo;
            u32 rho;
            RED_TW0(t_bp, lane == 0);
            const PivotCand pv = bm_pivot(eo, bits, L, &f, &rho);
            RED_TW1(S, 19, t_bp, lane == 0);
            int64_t own = -1;
            PairHit hit{-1, kNoVerts, 0, kNoList};
            if (pv.idx != kEmpty && rho == kNoRho) {
                if (lane == 0) own = ph_find(J.ph, pv.idx);
                if (lane == 32) hit = pair_find_all(J.app, pv.idx);
            }
            own = lane_bcast(own, 0);
            int64_t av = lane_bcast(hit.val, 32);
            u64 avw = lane_bcast(hit.verts, 32);
            if (rho != kNoRho) {
                // a zero apparent pair (rho, pivot) read with the pivot (a
                // pivot of a zero apparent pair is never in the pivot table)
                av = bm_edge_index((int)(rho >> 16), (int)(rho & 0xffffu)) << 3;
                avw = (u64)(rho >> 16) | ((u64)(rho & 0xffffu) << 16);
            }
            if (lane == 0) {
                S.bmf = f;
                S.piv = pv;
                S.owner = own;
                S.appv = av;
                if (pv.idx != kEmpty && own < 0 && av >= 0) {
                    // the addition of delta(rho): its item, set up here
                    if (avw != kNoVerts) {
                        S.it_v[0][0] = (int)(avw & 0xffffu);
                        S.it_v[0][1] = (int)((avw >> 16) & 0xffffu);
                    } else {
                        decode(av >> 3, k, c.n, c.B, S.it_v[0]);
                    }
                    S.nit = 1;
                    S.it_coef[0] = 1u;
                    S.it_diam[0] = pv.diam;
                }
            }
        }
        __syncthreads();
        RED_T1(S, 0, t_piv);
        const PivotCand piv = S.piv;
        if (piv.idx == kEmpty) {
            // zero column: an essential class born at sigma
            int64_t voff = 0;
            int vn = -1;
            if (J.keep_essential_v) {
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
                    J.bars.bs[j] = sidx;
                    J.bars.ds[j] = -1;
                    S.stat[4] += 1;
                    if (J.keep_essential_v) {
                        J.V.off[j] = voff;
                        J.V.len[j] = vn;
                    }
                }
                fence_release_dev();
                __syncthreads();
                if (tid == 0) st_dev(&J.par.cst[j], kColDone);
            } else if (tid == 0) {
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
        if (kPar && S.owner < 0 && S.appv < 0) {
            RED_T0(t_w);
            result = par_wait<BT>(J.par, S, j, __float_as_uint(piv.diam));
            if (result) break;
            if (tid == 0) S.owner = ph_find_dev(J.ph, piv.idx);
            __syncthreads();
            RED_T1(S, 17, t_w);
        }
        const int64_t o = S.owner;
        if (kPar && o >= j) {
            result = kRedOrder;
            break;
        }
        if (kPar && o >= 0) fence_acquire_dev();
        if (o >= 0) {
            // R_j += R_o (Z/2)
            RED_T0(t_add);
            const int vlen = J.V.len[o];
            const int rlen = J.V.rlen[o];
            if (tid == 0 && !log_add(SC, S, -2 - o, 1u, 0.0f, vlen < 0 ? 1 : vlen)) S.abort = kRedLogFull;
            if (rlen >= 0) {
                bm_add_r<BT>(J.V, J.V.roff[o], rlen, bits, L, W, S);
            } else if (vlen < 0) {
                // emergent column: R_o is the coboundary of sigma_o
                if (tid == 0) {
                    S.nit = 1;
                    S.it_coef[0] = 1u;
                    S.it_diam[0] = J.cols.diam[o];
                    decode(J.cols.idx[o], k, c.n, c.B, S.it_v[0]);
                }
                __syncthreads();
                bm_add_items<BT>(J, S, bits, L);
            } else {
                const int64_t voff = J.V.off[o];
                for (int c0 = 0; c0 < vlen; c0 += BT) {
                    const int nit = min(BT, vlen - c0);
                    if (tid < nit) {
                        const int64_t e = voff + c0 + tid;
                        decode(J.V.idx[e], k, c.n, c.B, S.it_v[tid]);
                        S.it_diam[tid] = J.V.diam[e];
                        S.it_coef[tid] = 1u;
                    }
                    if (tid == 0) S.nit = nit;
                    __syncthreads();
                    bm_add_items<BT>(J, S, bits, L);
                }
            }
            RED_T1(S, 1, t_add);
            if (S.abort) {
                result = S.abort;
                break;
            }
            ++nadd;
            continue;
        }
        if (S.appv >= 0) {
            RED_T0(t_app);
            // the pivot tau is in a zero apparent pair (rho, tau): add the
            // coboundary of rho (its item was set up with the pivot); the
            // last wave writes the log entry, so that wave 0 has no store
            // outstanding when it loads
            if (tid == BT - kWave && !log_add(SC, S, S.appv >> 3, 1u, piv.diam, 1)) S.abort = kRedLogFull;
            bm_add_items<BT>(J, S, bits, L);
            RED_T1(S, 16, t_app);
            if (S.abort) {
                result = S.abort;
                break;
            }
            ++nadd;
            continue;
        }
        // free pivot: the pair (sigma_j, pivot). R_j is stored (in bitmap
        // coordinates) when it is cheaper to add than V_j's coboundaries are
        // to recompute; then V_j is summed from the log and stored.
        RED_T0(t_st);
        int64_t roff = 0;
        int rn = -1;
        // a column of more than kBmStoreAdds additions stores V_j only: its
        // summary marks nearly every position after the front (an entry
        // stays marked after it cancels), so counting and storing R_j would
        // scan the whole bitmap at the end of the longest chain of additions,
        // and a later addition of it recomputes it from V_j
        const int64_t live = nadd > kBmStoreAdds ? INT64_MAX : bm_count<BT>(bits, L, W, S.bmf, S);
        if ((float)live <= 2.0f * (float)S.vest * J.cand_avg) {
            rn = bm_store<BT>(bits, L, W, S.bmf, J.V, J.vcount, S, &roff);
            if (rn < 0) {
                result = kRedStoreFull;
                break;
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
            if (tid == 0) {
                if ((unsigned long long)vn > S.stat[6]) S.stat[6] = vn;
                J.bars.birth[j] = sdm;
                J.bars.death[j] = piv.diam;
                J.bars.bs[j] = piv.diam > sdm ? sidx : -1;
                J.bars.ds[j] = piv.idx;
                if (piv.diam > sdm) S.stat[3] += 1;
                J.V.pivcoef[j] = 1u;
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
            J.V.pivcoef[j] = 1u;
            J.V.off[j] = voff;
            J.V.len[j] = vn;
            J.V.roff[j] = roff;
            J.V.rlen[j] = rn;
        }
        RED_T1(S, 5, t_st);
        break;
    }
    if (tid == 0 && result == kRedOk) {
        S.stat[1] += nadd > 0 ? 1 : 0;
        S.stat[2] += nadd;
    }
    __syncthreads();
    RED_T0(t_clr);
    bm_clear<BT>(bits, L, W);
    RED_T1(S, 9, t_clr);
    return result;
}

} // namespace rips
