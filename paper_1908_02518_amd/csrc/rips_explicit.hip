// rips_explicit.hip -- explicit matrix reduction, the first column of the
// ablation in Table 3 of the paper (section "Experiments", paragraph
// "Implicit reduction matrix"): before dimension k is reduced, the
// coboundary columns of every column left by clearing are built in HBM as a
// compressed sparse column matrix (each column's cofacets <= t, oldest first
// in the refined order of the "Filtrations" paragraph, with the coefficients
// of the standard orientation), and the reduction adds stored reduced
// columns R_o, which is Algorithm 1 on an explicit matrix. Cohomology and
// clearing are kept; the apparent and emergent shortcuts are not, since both
// rest on the implicit matrix. The pairs are those of the implicit path; the
// memory (every coboundary entry and every reduced column at once) is what
// the implicit path avoids.
//
// Build: one wave per column counts the cofacets; a single workgroup turns
// the counts into column offsets; one workgroup per column writes its
// entries into LDS, ranks them by counting and writes them out sorted.
// Reduction: one workgroup takes the columns one after another (column j
// reads the final pivots of all columns before it). The working column is a
// sorted list in global memory (it can outgrow LDS by far); an addition is
// a merge of two sorted lists, every entry finding its place in the other
// by binary search, and a block scan compacts the result.
#include "rips_reduce.hpp"
#include "rips_kernels.hpp"

namespace rips {

// older first: smaller diameter, then larger index
__device__ __forceinline__ bool exp_older(float da, int64_t ia, float db, int64_t ib) {
    return da < db || (da == db && ia > ib);
}

// candidate vertices of sigma's cofacets: all vertices (dense), or the
// neighbours of v[0] within t (sparse); every vertex of a cofacet <= t is a
// neighbour of v[0]
__device__ __forceinline__ int exp_ncand(const Ctx<DistFull> &c, int v0) {
    return c.nb.off == nullptr ? c.n : c.nb.off[v0 + 1] - c.nb.off[v0];
}

__device__ __forceinline__ int exp_cand(const Ctx<DistFull> &c, int v0, int q) {
    return c.nb.off == nullptr ? q : c.nb.idx[c.nb.off[v0] + q];
}

// j extends sigma (vertices v[0..k]) to a cofacet <= t; its diameter in *dm
__device__ __forceinline__ bool exp_cofacet(const Ctx<DistFull> &c, const int *v, int k, int j, float sd,
                                            float *dm) {
    float m = sd;
    for (int a = 0; a <= k; ++a) {
        if (v[a] == j) return false;
        m = fmaxf(m, c.d(j, v[a]));
    }
    *dm = m;
    return m <= c.t;
}

__global__ void __launch_bounds__(256) k_exp_count(Ctx<DistFull> c, int k, const int64_t *cidx,
                                                   const float *cdia, int64_t S, int64_t *cnt,
                                                   unsigned long long *longest) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    const int64_t waves = (int64_t)gridDim.x * (256 / kWave);
    for (int64_t col = wave; col < S; col += waves) {
        int v[kMaxVerts];
        decode(cidx[col], k, c.n, c.B, v);
        const float sd = cdia[col];
        const int nc = exp_ncand(c, v[0]);
        int64_t count = 0;
        for (int q0 = 0; q0 < nc; q0 += kWave) {
            const int q = q0 + lane;
            float dm;
            const bool ok = q < nc && exp_cofacet(c, v, k, exp_cand(c, v[0], q), sd, &dm);
            count += __popcll(__ballot(ok));
        }
        if (lane == 0) {
            cnt[col] = count;
            atomicMax(longest, (unsigned long long)count);
        }
    }
}

// off[i] = cnt[0] + ... + cnt[i-1], i = 0..S (one workgroup of 1024: each
// thread sums a contiguous stretch, the stretch sums are scanned in LDS)
__global__ void __launch_bounds__(1024) k_exp_offsets(const int64_t *cnt, int64_t S, int64_t *off) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (S + 1023) / 1024;
    const int64_t lo = (int64_t)tid * per < S ? (int64_t)tid * per : S;
    const int64_t hi = lo + per < S ? lo + per : S;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int64_t run = part[tid] - s; // exclusive
    for (int64_t i = lo; i < hi; ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (tid == 1023) off[S] = part[1023];
}

// One workgroup per column: the cofacets <= t in LDS (compacted in vertex
// order), then each written to its rank in the refined order, oldest first.
__global__ void __launch_bounds__(kExpThreads) k_exp_fill(Ctx<DistFull> c, int k, u32 p, const int64_t *cidx,
                                                          const float *cdia, int64_t S, const int64_t *off,
                                                          ExpMatrix D) {
    __shared__ int64_t li[kExpBuildCap];
    __shared__ float ld_[kExpBuildCap];
    __shared__ u32 lc[kExpBuildCap];
    __shared__ int s_w[kExpThreads / kWave + 1];
    const int tid = threadIdx.x;
    for (int64_t col = blockIdx.x; col < S; col += gridDim.x) {
        int v[kMaxVerts];
        decode(cidx[col], k, c.n, c.B, v);
        const float sd = cdia[col];
        const int nc = exp_ncand(c, v[0]);
        int len = 0;
        for (int q0 = 0; q0 < nc; q0 += kExpThreads) {
            const int q = q0 + tid;
            float dm = 0.0f;
            int j = -1;
            const bool ok = q < nc && exp_cofacet(c, v, k, j = exp_cand(c, v[0], q), sd, &dm);
            int tot;
            const int at = block_scan_excl<kExpThreads>(ok ? 1 : 0, s_w, &tot);
            if (ok && len + at < kExpBuildCap) {
                int below;
                li[len + at] = cofacet_index(v, k, j, c.B, &below);
                ld_[len + at] = dm;
                lc[len + at] = coeff_sign(below, p);
            }
            len += tot;
        }
        __syncthreads();
        // the host sized the build for the longest column; a longer one
        // would be a count / fill mismatch, and is cut to what fits
        if (len > kExpBuildCap) len = kExpBuildCap;
        const int64_t base = off[col];
        for (int e = tid; e < len; e += kExpThreads) {
            const int64_t ie = li[e];
            const float de = ld_[e];
            int r = 0;
            for (int f = 0; f < len; ++f) r += exp_older(ld_[f], li[f], de, ie) ? 1 : 0;
            D.idx[base + r] = ie;
            D.diam[base + r] = de;
            D.coef[base + r] = lc[e];
        }
        __syncthreads(); // the LDS lists are rewritten for the next column
    }
}

// The reduction of one dimension's columns, in the order given (youngest
// first), by one workgroup.
__global__ void __launch_bounds__(kExpThreads) k_exp_reduce(ExpJob J) {
    __shared__ int s_w[kExpThreads / kWave + 1];
    __shared__ int s_owner, s_bad;
    const int tid = threadIdx.x;
    const u32 p = J.p;
    const int k = J.k;
    int64_t *Wi = J.wi[0], *Ti = J.wi[1];
    float *Wd = J.wd[0], *Td = J.wd[1];
    u32 *Wc = J.wc[0], *Tc = J.wc[1];
    unsigned long long n_add = 0, n_red = 0, n_added = 0, n_nonzero = 0, n_bars = 0, n_ess = 0;
    int64_t pool = 0;
    int status = kExpOk;
    if (tid == 0) s_bad = 0;
    for (int64_t jj = 0; jj < J.ncols; ++jj) {
        const int64_t sidx = J.cidx[jj];
        const float sdm = J.cdia[jj];
        const int64_t d0 = J.D.off[jj];
        int len = (int)(J.D.off[jj + 1] - d0);
        if (len > J.wcap) {
            status = kExpFull;
            break;
        }
        for (int e = tid; e < len; e += kExpThreads) {
            Wi[e] = J.D.idx[d0 + e];
            Wd[e] = J.D.diam[d0 + e];
            Wc[e] = J.D.coef[d0 + e];
        }
        __syncthreads();
        int64_t adds = 0;
        // while the pivot (oldest entry) is the pivot of an earlier column o:
        // W -= lambda R_o with lambda = W's pivot coefficient over R_o's
        while (len > 0) {
            if (tid == 0) s_owner = ph_find(J.piv, Wi[0]);
            __syncthreads();
            const int32_t o = s_owner;
            if (o < 0) break;
            if (++adds > kExpMaxAdds) {
                status = kExpBound;
                break;
            }
            const int64_t ro = J.roff[o];
            const int rl = J.rlen[o];
            if (len + rl > J.wcap) {
                status = kExpFull;
                break;
            }
            const int64_t *Ri = J.pidx + ro;
            const float *Rd = J.pdia + ro;
            const u32 *Rc = J.pcoef + ro;
            const u32 lam = (u32)((u64)Wc[0] * J.inv[Rc[0]] % p);
            n_added += (unsigned long long)rl;
            for (int e = tid; e < len + rl; e += kExpThreads) Tc[e] = 0u;
            __syncthreads();
            // merged place of W[a]: a + (entries of R_o older than it); the
            // entry of R_o equal to W[a], if any, is added into it
            for (int a = tid; a < len; a += kExpThreads) {
                const int64_t ia = Wi[a];
                const float da = Wd[a];
                int lo = 0, hi = rl;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (exp_older(Rd[mid], Ri[mid], da, ia)) lo = mid + 1;
                    else hi = mid;
                }
                u32 cf = Wc[a];
                if (lo < rl && Ri[lo] == ia) cf = (u32)((cf + (u64)(p - (u64)lam * Rc[lo] % p)) % p);
                Ti[a + lo] = ia;
                Td[a + lo] = da;
                Tc[a + lo] = cf;
            }
            for (int b = tid; b < rl; b += kExpThreads) {
                const int64_t ib = Ri[b];
                const float db = Rd[b];
                int lo = 0, hi = len;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (exp_older(Wd[mid], Wi[mid], db, ib)) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < len && Wi[lo] == ib) continue;
                Ti[b + lo] = ib;
                Td[b + lo] = db;
                Tc[b + lo] = (u32)((p - (u64)lam * Rc[b] % p) % p);
            }
            __syncthreads();
            // nonzero entries, in order, become the working column
            const int tot = len + rl;
            int nl = 0;
            for (int b0 = 0; b0 < tot; b0 += kExpThreads) {
                const int e = b0 + tid;
                const int live = (e < tot && Tc[e] != 0u) ? 1 : 0;
                int t2;
                const int at = block_scan_excl<kExpThreads>(live, s_w, &t2);
                if (live) {
                    Wi[nl + at] = Ti[e];
                    Wd[nl + at] = Td[e];
                    Wc[nl + at] = Tc[e];
                }
                nl += t2;
            }
            __syncthreads();
            len = nl;
        }
        n_add += (unsigned long long)adds;
        if (adds > 0) ++n_red;
        if (status != kExpOk) break;
        if (len == 0) {
            // an essential class born at sigma, unless (without clearing)
            // sigma is a pivot of the dimension below and so no class at all
            const bool lower = !J.clearing && (k == 1 ? ((J.prev_bits[sidx >> 5] >> (sidx & 31)) & 1u) != 0
                                                      : ph_find(J.prev, sidx) >= 0);
            if (!lower) {
                if (tid == 0) {
                    J.bars.birth[n_bars] = sdm;
                    J.bars.death[n_bars] = INFINITY;
                    J.bars.bs[n_bars] = sidx;
                    J.bars.ds[n_bars] = -1;
                }
                ++n_bars;
                ++n_ess;
            }
            __syncthreads();
            continue;
        }
        // R_j is stored and its pivot recorded; (sigma, pivot) is a bar when
        // the diameters differ
        if (pool + len > J.pcap) {
            status = kExpPool;
            break;
        }
        for (int e = tid; e < len; e += kExpThreads) {
            J.pidx[pool + e] = Wi[e];
            J.pdia[pool + e] = Wd[e];
            J.pcoef[pool + e] = Wc[e];
        }
        const float pd = Wd[0];
        const int64_t pi = Wi[0];
        if (tid == 0) {
            J.roff[jj] = pool;
            J.rlen[jj] = len;
            if (!ph_insert(J.piv, pi, (int32_t)jj)) s_bad = 1;
            if (pd > sdm) {
                J.bars.birth[n_bars] = sdm;
                J.bars.death[n_bars] = pd;
                J.bars.bs[n_bars] = sidx;
                J.bars.ds[n_bars] = pi;
            }
        }
        if (pd > sdm) ++n_bars;
        ++n_nonzero;
        pool += len;
        // the stored column and the table entry are read by later columns
        __syncthreads();
        if (s_bad) {
            status = kExpTable;
            break;
        }
    }
    if (tid == 0) {
        ExpOut *o = J.out;
        o->status = status;
        o->bars = (long long)n_bars;
        o->nonzero = (long long)n_nonzero;
        o->essential = (long long)n_ess;
        o->additions = (long long)n_add;
        o->reduced = (long long)n_red;
        o->added = (long long)n_added;
        o->stored = pool;
    }
}

void launch_exp_count(const Ctx<DistFull> &c, int k, const int64_t *cidx, const float *cdia, int64_t S,
                      int64_t *cnt, unsigned long long *longest, hipStream_t st) {
    int64_t blocks = (S + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_exp_count, dim3((unsigned)blocks), dim3(256), 0, st, c, k, cidx, cdia, S, cnt,
                       longest);
}

void launch_exp_offsets(const int64_t *cnt, int64_t S, int64_t *off, hipStream_t st) {
    hipLaunchKernelGGL(k_exp_offsets, dim3(1), dim3(1024), 0, st, cnt, S, off);
}

void launch_exp_fill(const Ctx<DistFull> &c, int k, u32 p, const int64_t *cidx, const float *cdia, int64_t S,
                     const int64_t *off, ExpMatrix D, hipStream_t st) {
    int64_t blocks = S < 1 ? 1 : (S > 16384 ? 16384 : S);
    hipLaunchKernelGGL(k_exp_fill, dim3((unsigned)blocks), dim3(kExpThreads), 0, st, c, k, p, cidx, cdia, S,
                       off, D);
}

void launch_exp_reduce(const ExpJob &J, hipStream_t st) {
    hipLaunchKernelGGL(k_exp_reduce, dim3(1), dim3(kExpThreads), 0, st, J);
}

} // namespace rips
