// rips_homology.hip -- the homology variant of the single-cloud path, kept
// for the ablation against cohomology: the filtration boundary matrices are
// reduced with clearing (Algorithm 2 of the section "Clearing inessential
// birth columns" applied to boundary matrices), from the top dimension down,
// with the reduced columns R_j stored explicitly (the "explicit" row of
// Table 3). It reaches the same persistence pairs as the cohomology path
// (the pairs of a filtration and of its dual coincide, section
// "Cohomology"), but has to reduce every column of the top dimension, which
// clearing cannot touch: the asymmetry the column counters show.
//
// One workgroup takes the columns one after another (the reduction of
// column j reads the final pivots of all columns before it). The working
// column lives in LDS as a list sorted younger first; adding a stored column
// is a merge of two sorted lists: every entry finds its place in the other
// list by binary search, the merged list is compacted by a block scan.
#include "rips_reduce.hpp"
#include "rips_kernels.hpp"

namespace rips {

// younger first: larger diameter, then smaller index (the refined order of
// the "Filtrations" paragraph, reversed)
__device__ __forceinline__ bool younger_key(float da, int64_t ia, float db, int64_t ib) {
    return da > db || (da == db && ia < ib);
}

// Reduction of the boundary matrix of the k-simplices (rows: (k-1)-simplices).
__global__ void __launch_bounds__(kHomThreads) k_hom_reduce(HomJob J) {
    extern __shared__ unsigned char smem[];
    __shared__ int s_w[kHomThreads / kWave + 1];
    __shared__ int s_len, s_bad;
    LDS unsigned char *q = (LDS unsigned char *)smem;
    LDS int64_t *Wi = (LDS int64_t *)q;
    q += kHomCap * 8;
    LDS int64_t *Bi = (LDS int64_t *)q;
    q += kHomCap * 8;
    LDS int64_t *Ti = (LDS int64_t *)q;
    q += 2 * kHomCap * 8;
    LDS float *Wd = (LDS float *)q;
    q += kHomCap * 4;
    LDS float *Bd = (LDS float *)q;
    q += kHomCap * 4;
    LDS float *Td = (LDS float *)q;
    q += 2 * kHomCap * 4;
    LDS u32 *Wc = (LDS u32 *)q;
    q += kHomCap * 4;
    LDS u32 *Bc = (LDS u32 *)q;
    q += kHomCap * 4;
    LDS u32 *Tc = (LDS u32 *)q;

    const int tid = threadIdx.x;
    const int k = J.k;
    const u32 p = J.p;
    if (tid == 0) s_bad = 0;
    // counters (the same in every thread; thread 0 writes them out)
    unsigned long long n_pairs = 0, n_nonzero = 0, n_ess = 0, n_clear = 0, n_red = 0, n_add = 0;
    int64_t pool = 0, longest = 0;
    int32_t nstored = 0;
    int status = kHomOk;
    for (int64_t jj = J.ncols - 1; jj >= 0; --jj) {
        // oldest column first: the list is sorted younger first
        const int64_t tidx = J.cidx[jj];
        const float tdia = J.cdia[jj];
        if (J.clear.keys != nullptr && ph_find(J.clear, tidx) >= 0) {
            ++n_clear; // a pivot of the boundary above: its column reduces to zero
            continue;
        }
        ++n_red;
        // the boundary: facet m drops vertex v[m]; with the vertices below
        // v[m] counted, its coefficient is (-1)^(k - m)
        if (tid == 0) {
            int v[kMaxVerts];
            decode(tidx, k, J.c.n, J.c.B, v);
            int cnt = 0;
            for (int m = 0; m <= k; ++m) {
                int f[kMaxVerts];
                int r = 0;
                for (int u = 0; u <= k; ++u)
                    if (u != m) f[r++] = v[u];
                float fd = 0.0f;
                for (int a = 0; a < k; ++a)
                    for (int b = a + 1; b < k; ++b) fd = fmaxf(fd, J.c.d(f[a], f[b]));
                const int64_t fi = k == 1 ? (int64_t)f[0] : simplex_index(f, k - 1, J.c.B);
                const u32 fc = ((k - m) & 1) ? p - 1 : 1u;
                int at = cnt;
                while (at > 0 && younger_key(fd, fi, Wd[at - 1], Wi[at - 1])) {
                    Wi[at] = Wi[at - 1];
                    Wd[at] = Wd[at - 1];
                    Wc[at] = Wc[at - 1];
                    --at;
                }
                Wi[at] = fi;
                Wd[at] = fd;
                Wc[at] = fc;
                ++cnt;
            }
            s_len = cnt;
        }
        __syncthreads();
        int len = s_len;
        int64_t adds = 0;
        // while the pivot (youngest entry) is owned by an earlier column:
        // W -= lambda R_o, lambda = W's pivot coefficient over R_o's
        while (len > 0) {
            const int32_t o = ph_find(J.piv, Wi[0]);
            if (o < 0) break;
            if (++adds > kHomMaxAdds) {
                status = kHomBound;
                break;
            }
            const int64_t off = J.roff[o];
            const int rl = J.rlen[o];
            if (rl > kHomCap) {
                status = kHomFull;
                break;
            }
            const u32 lam = (u32)((u64)Wc[0] * J.inv[J.pcoef[off]] % p);
            for (int e = tid; e < rl; e += kHomThreads) {
                Bi[e] = J.pidx[off + e];
                Bd[e] = J.pdia[off + e];
                Bc[e] = (u32)((p - (u64)lam * J.pcoef[off + e] % p) % p);
            }
            for (int e = tid; e < len + rl; e += kHomThreads) Tc[e] = 0u;
            __syncthreads();
            // merged place of W[a]: a + (entries of B younger than it); an
            // entry of B equal to W[a] is added into it and leaves a hole
            for (int a = tid; a < len; a += kHomThreads) {
                const int64_t ia = Wi[a];
                const float da = Wd[a];
                int lo = 0, hi = rl;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (younger_key(Bd[mid], Bi[mid], da, ia)) lo = mid + 1;
                    else hi = mid;
                }
                u32 cf = Wc[a];
                if (lo < rl && Bi[lo] == ia) cf = (cf + Bc[lo]) % p;
                Ti[a + lo] = ia;
                Td[a + lo] = da;
                Tc[a + lo] = cf;
            }
            for (int b = tid; b < rl; b += kHomThreads) {
                const int64_t ib = Bi[b];
                const float db = Bd[b];
                int lo = 0, hi = len;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (younger_key(Wd[mid], Wi[mid], db, ib)) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < len && Wi[lo] == ib) continue;
                Ti[b + lo] = ib;
                Td[b + lo] = db;
                Tc[b + lo] = Bc[b];
            }
            __syncthreads();
            // nonzero entries back into W, in order
            const int tot = len + rl;
            int nl = 0;
            for (int b0 = 0; b0 < tot; b0 += kHomThreads) {
                const int e = b0 + tid;
                const int live = (e < tot && Tc[e] != 0u) ? 1 : 0;
                int t2;
                const int at = block_scan_excl<kHomThreads>(live, s_w, &t2);
                if (live && nl + at < kHomCap) {
                    Wi[nl + at] = Ti[e];
                    Wd[nl + at] = Td[e];
                    Wc[nl + at] = Tc[e];
                }
                nl += t2;
            }
            __syncthreads();
            if (nl > kHomCap) {
                status = kHomFull;
                break;
            }
            len = nl;
        }
        n_add += (unsigned long long)adds;
        if (status != kHomOk) break;
        if (len > longest) longest = len;
        if (len == 0) {
            // a cycle that no column of the boundary above kills: essential
            if (J.essential) {
                if (n_ess >= (unsigned long long)J.ess_cap) {
                    status = kHomTable;
                    break;
                }
                if (tid == 0) {
                    J.ess.birth[n_ess] = tdia;
                    J.ess.death[n_ess] = INFINITY;
                    J.ess.bs[n_ess] = tidx;
                    J.ess.ds[n_ess] = -1;
                }
                ++n_ess;
            }
            __syncthreads();
            continue;
        }
        // store R_j and its pivot; the pair (pivot, tau) is a bar when its
        // diameters differ
        if (pool + len > J.pcap) {
            status = kHomPool;
            break;
        }
        for (int e = tid; e < len; e += kHomThreads) {
            J.pidx[pool + e] = Wi[e];
            J.pdia[pool + e] = Wd[e];
            J.pcoef[pool + e] = Wc[e];
        }
        const bool bar = tdia > Wd[0];
        if (bar && n_pairs >= (unsigned long long)J.pairs_cap) {
            status = kHomTable;
            break;
        }
        if (tid == 0) {
            J.roff[nstored] = pool;
            J.rlen[nstored] = len;
            if (!ph_insert(J.piv, Wi[0], nstored)) s_bad = 1;
            if (bar) {
                J.pairs.birth[n_pairs] = Wd[0];
                J.pairs.death[n_pairs] = tdia;
                J.pairs.bs[n_pairs] = Wi[0];
                J.pairs.ds[n_pairs] = tidx;
            }
        }
        if (bar) ++n_pairs;
        ++n_nonzero;
        pool += len;
        ++nstored;
        // the stored column and the table entry are read by the next columns
        __syncthreads();
        if (s_bad) {
            status = kHomTable;
            break;
        }
    }
    if (tid == 0) {
        HomOut *o = J.out;
        o->status = status;
        o->pairs = (long long)n_pairs;
        o->nonzero = (long long)n_nonzero;
        o->essential = (long long)n_ess;
        o->cleared = (long long)n_clear;
        o->reduced = (long long)n_red;
        o->additions = (long long)n_add;
        o->stored = pool;
        o->longest = longest;
    }
}

// H0 classes that never die: vertices that are no pivot of the edge boundary.
__global__ void k_hom_vertices(int n, PivotHash piv, BarBuf ess, HomOut *o) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (ph_find(piv, v) >= 0) continue;
        const long long at = atomicAdd((unsigned long long *)&o->essential, 1ull);
        ess.birth[at] = 0.0f;
        ess.death[at] = INFINITY;
        ess.bs[at] = v;
        ess.ds[at] = -1;
    }
}

__global__ void k_hom_iota(int *a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int)i;
}

// bars in canonical order: the sort left them youngest birth simplex first
// (its j carries the bar's slot); the canonical order is the reverse
__global__ void k_hom_gather(BarBuf in, const int *perm, int64_t n, BarBuf out) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int e = perm[n - 1 - q];
        out.birth[q] = in.birth[e];
        out.death[q] = in.death[e];
        out.bs[q] = in.bs[e];
        out.ds[q] = in.ds[e];
    }
}

size_t hom_lds_bytes() { return (size_t)kHomCap * (8 + 8 + 16 + 4 + 4 + 8 + 4 + 4 + 8); }

hipError_t launch_hom_reduce(const HomJob &J, hipStream_t st) {
    const size_t lds = hom_lds_bytes();
    hipError_t e = hipFuncSetAttribute((const void *)k_hom_reduce,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hom_reduce, dim3(1), dim3(kHomThreads), lds, st, J);
    return hipGetLastError();
}

void launch_hom_vertices(int n, PivotHash piv, BarBuf ess, HomOut *o, hipStream_t st) {
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_hom_vertices, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, n, piv, ess, o);
}

void launch_hom_iota(int *a, int64_t n, hipStream_t st) {
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_hom_iota, dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b))), dim3(256), 0,
                       st, a, n);
}

void launch_hom_gather(BarBuf in, const int *perm, int64_t n, BarBuf out, hipStream_t st) {
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_hom_gather, dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b))), dim3(256), 0,
                       st, in, perm, n, out);
}

} // namespace rips
