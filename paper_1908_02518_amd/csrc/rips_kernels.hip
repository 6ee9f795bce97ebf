// rips_kernels.hip -- gfx950 kernels of the single-cloud Vietoris-Rips path.
//
// Data layout in HBM (one cloud):
//   D        n x n float32, row-major (rows contiguous: coalesced scans of
//            candidate vertices for a fixed simplex vertex)
//   B        binomial table, (kMaxDim + 3) x (n + 1) uint64
//   edges    SoA (idx int64, diam f32, a i32, b i32) of the edges <= t
//   nbr      CSR neighbour lists <= t, ascending (sparse path only)
//   lists    SoA (idx int64, diam f32) of all k-simplices <= t, k >= 2
//   columns  SoA (idx, diam, j*, tau-apparent flag) of the surviving columns
//   pivots   open-addressing table pivot -> column per dimension
//   V        death columns of the reduction matrix, CSR-like append buffer
#include "rips_reduce.hpp"

namespace rips {

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------

__device__ __forceinline__ u64 gcd64(u64 a, u64 b) {
    while (b) {
        u64 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// C(i, j) for 0 <= i <= n, 0 <= j <= jmax, by C(i, j) = C(i, j-1) (i-j+1) / j
// with the gcd split so that no intermediate exceeds the result.
__global__ void k_binom(u64 *B, int stride, int n, int jmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    u64 r = 1;
    B[i] = 1;
    for (int j = 1; j <= jmax; ++j) {
        if (j > i) r = 0;
        else {
            const u64 g = gcd64(r, (u64)j);
            r = (r / g) * ((u64)(i - j + 1) / ((u64)j / g));
        }
        B[(int64_t)j * stride + i] = r;
    }
}

// multiplicative inverses mod p (the paper's multiplicative_inverse_vector)
__global__ void k_inverse(u32 *inv, u32 p) {
    const u32 a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= p) return;
    if (a == 0) {
        inv[0] = 0;
        return;
    }
    u64 r = 1, b = a, e = p - 2;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    inv[a] = (u32)r;
}

// ---------------------------------------------------------------------------
// distances
// ---------------------------------------------------------------------------

// d(i, j) = sqrt(sum_c (x_ic - x_jc)^2): coordinates in increasing order,
// every product and sum rounded to float32 (built with -ffp-contract=off),
// correctly rounded square root. Full square matrix; (x_i - x_j)^2 equals
// (x_j - x_i)^2 exactly, so D is bitwise symmetric.
__global__ void k_dist_points(const float *__restrict__ X, int n, int m, float *__restrict__ D,
                              int *bad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    const float *xi = X + (int64_t)i * m;
    const float *xj = X + (int64_t)j * m;
    float s = 0.0f;
    bool fin = true;
    for (int c = 0; c < m; ++c) {
        const float a = xi[c], b = xj[c];
        fin = fin && isfinite(a) && isfinite(b);
        const float t = a - b;
        const float sq = t * t;
        s = s + sq;
    }
    if (!fin) atomicOr(bad, 1);
    D[(int64_t)i * n + j] = __builtin_sqrtf(s);
}

// Distance-matrix input: entries (i, j), i > j, of a row-major n x n matrix.
__global__ void k_dist_matrix(const float *__restrict__ M, int n, float *__restrict__ D, int *bad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    float v;
    if (i > j) v = M[(int64_t)i * n + j];
    else if (i < j) v = M[(int64_t)j * n + i];
    else v = 0.0f;
    if (!(v >= 0.0f) || isinf(v)) atomicOr(bad, 1);
    D[(int64_t)i * n + j] = v;
}

// ---------------------------------------------------------------------------
// threshold: enclosing radius min_x max_y d(x, y); t_eff = min(t, r_enc)
// ---------------------------------------------------------------------------
__global__ void k_init_scalars(Scalars *s) {
    s->renc_bits = 0x7f800000u; // +inf
    s->bad = 0;
    s->status = 0;
    s->edges = 0;
    s->list = 0;
    s->survivors = 0;
    s->vcount = 0;
    s->mst = 0;
    s->nbars = 0;
    s->maxdeg = 0;
    for (int q = 0; q < kNumStats; ++q) s->stat[q] = 0;
}

// per-dimension counters back to zero (the host has read them)
__global__ void k_reset_dim(Scalars *s) {
    s->status = 0;
    s->list = 0;
    s->survivors = 0;
    s->vcount = 0;
    s->nbars = 0;
    for (int q = 0; q < kNumStats; ++q) s->stat[q] = 0;
}

__global__ void k_rowmax(const float *__restrict__ D, int n, Scalars *s) {
    const int wpb = blockDim.x / kWave;
    const int i = blockIdx.x * wpb + threadIdx.x / kWave;
    if (i >= n) return;
    const int lane = lane_id();
    const float *row = D + (int64_t)i * n;
    float mx = 0.0f;
    for (int j = lane; j < n; j += kWave) mx = fmaxf(mx, row[j]);
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    if (lane == 0) atomicMin(&s->renc_bits, __float_as_uint(mx));
}

__global__ void k_set_teff(Scalars *s, float t) {
    const float r = __uint_as_float(s->renc_bits);
    s->r_enc = r;
    s->t_eff = fminf(t, r);
}

// ---------------------------------------------------------------------------
// edges <= t_eff (k = 1 candidates; Kruskal/Boruvka input), degrees
// ---------------------------------------------------------------------------
__global__ void k_edges(const float *__restrict__ D, int n, Scalars *s, EdgeList E, int64_t cap,
                        int *deg) {
    const int wpb = blockDim.x / kWave;
    const int i = blockIdx.x * wpb + threadIdx.x / kWave;
    if (i >= n) return;
    const float t = s->t_eff;
    const int lane = lane_id();
    const float *row = D + (int64_t)i * n;
    int mine = 0;
    for (int j0 = 0; j0 < i; j0 += kWave) {
        const int j = j0 + lane;
        const float d = j < i ? row[j] : INFINITY;
        const bool ok = d <= t;
        const int64_t slot = wave_append(&s->edges, ok);
        if (ok) {
            if (slot < cap) {
                E.idx[slot] = (int64_t)i * (i - 1) / 2 + j;
                E.diam[slot] = d;
                E.a[slot] = i;
                E.b[slot] = j;
            }
            atomicAdd(&deg[j], 1);
            ++mine;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) mine += __shfl_xor(mine, off, kWave);
    if (lane == 0 && mine) atomicAdd(&deg[i], mine);
}

__global__ void k_zero_int(int *a, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = 0;
}

__global__ void k_fill_u32(u32 *a, int64_t n, u32 v) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

__global__ void k_fill_i64(int64_t *a, int64_t n, int64_t v) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

// ---------------------------------------------------------------------------
// block-wide exclusive scan helper (BT threads, one value each)
// ---------------------------------------------------------------------------
template <int BT>
__device__ __forceinline__ int block_exclusive_scan(int x, int *s_w, int *total) {
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

// exclusive scan of deg[0..n) into off[0..n], single block
__global__ void __launch_bounds__(1024) k_scan_deg(const int *deg, int n, int *off) {
    __shared__ int s_w[1024 / kWave + 1];
    int carry = 0;
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        const int x = i < n ? deg[i] : 0;
        int tot;
        const int ex = block_exclusive_scan<1024>(x, s_w, &tot);
        if (i < n) off[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) off[n] = carry;
}

// neighbour lists: one block per vertex, ascending neighbour order
__global__ void __launch_bounds__(256) k_csr_fill(const float *__restrict__ D, int n, Scalars *s,
                                                  const int *off, int *nbr) {
    __shared__ int s_w[256 / kWave + 1];
    const int i = blockIdx.x;
    const float t = s->t_eff;
    const float *row = D + (int64_t)i * n;
    int at = off[i];
    const int end = off[i + 1];
    for (int base = 0; base < n; base += 256) {
        const int j = base + threadIdx.x;
        const bool ok = j < n && j != i && row[j] <= t;
        int tot;
        const int ex = block_exclusive_scan<256>(ok ? 1 : 0, s_w, &tot);
        if (ok && at + ex < end) nbr[at + ex] = j;
        at += tot;
    }
}

// ---------------------------------------------------------------------------
// H0: minimum spanning forest by Boruvka rounds on the refined edge order
// (diameter, then larger CNS index = older first), then the elder rule on the
// forest's edges in that order (Kruskal with union-find, "Persistence pairs"
// paragraph). One block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 edge_key(float d, u32 idx) {
    return ((u64)__float_as_uint(d) << 32) | (u64)(0xffffffffu - idx);
}

__device__ __forceinline__ void edge_vertices(u32 idx, int *a, int *b) {
    // largest a with a(a-1)/2 <= idx
    int x = (int)((1.0 + sqrt(1.0 + 8.0 * (double)idx)) * 0.5);
    while ((int64_t)x * (x - 1) / 2 > (int64_t)idx) --x;
    while ((int64_t)(x + 1) * x / 2 <= (int64_t)idx) ++x;
    *a = x;
    *b = (int)((int64_t)idx - (int64_t)x * (x - 1) / 2);
}

__device__ __forceinline__ int uf_find(int *parent, int v, int n) {
    int p = ld(&parent[v]);
    for (int guard = 0; p != v && guard < n; ++guard) {
        v = p;
        p = ld(&parent[v]);
    }
    return v;
}

constexpr int kH0Threads = 1024;
constexpr int kH0LdsMax = 2048; // union-find state of up to this many vertices lives in LDS

__global__ void __launch_bounds__(kH0Threads) k_h0(EdgeList E, Scalars *s, int n, H0Scratch W,
                                                    BarBuf out) {
    __shared__ SortShared<kH0Threads> S;
    __shared__ int s_flag;
    __shared__ int s_w[kH0Threads / kWave + 1];
    __shared__ int l_comp[kH0LdsMax];
    __shared__ int l_hook[kH0LdsMax];
    __shared__ u64 l_best[kH0LdsMax];
    const bool in_lds = n <= kH0LdsMax;
    // every word below that is touched by an atomic is only ever accessed
    // atomically; phases are separated by gsync()
    int *comp = in_lds ? l_comp : W.comp;
    int *hook = in_lds ? l_hook : W.hook;
    u64 *best = in_lds ? l_best : W.best;
    const int tid = threadIdx.x;
    const int64_t ne = s->edges;
    const int64_t all_edges = (int64_t)n * (n - 1) / 2;
    for (int v = tid; v < n; v += kH0Threads) st(&comp[v], v);
    gsync();
    // Boruvka: every component picks its oldest outgoing edge. Each round at
    // least halves the number of components that still have an edge; the
    // round bound only guards against a fault.
    for (int round = 0; round < 40; ++round) {
        for (int v = tid; v < n; v += kH0Threads) st(&best[v], ~0ull);
        gsync();
        for (int64_t e = tid; e < ne; e += kH0Threads) {
            const int ca = ld(&comp[E.a[e]]), cb = ld(&comp[E.b[e]]);
            if (ca != cb) {
                const u64 key = edge_key(E.diam[e], (u32)E.idx[e]);
                atomicMin(&best[ca], key);
                atomicMin(&best[cb], key);
            }
        }
        if (tid == 0) s_flag = 0;
        gsync();
        for (int v = tid; v < n; v += kH0Threads) {
            const int cv = ld(&comp[v]);
            int h = cv; // non-roots keep pointing at their root
            const u64 key = ld(&best[v]);
            if (cv == v && key != ~0ull) {
                int a, b;
                edge_vertices(0xffffffffu - (u32)(key & 0xffffffffu), &a, &b);
                const int ca = ld(&comp[a]), cb = ld(&comp[b]);
                const int other = ca == v ? cb : ca;
                const bool mutual = ld(&best[other]) == key;
                // mutual choices form 2-cycles: the larger root hooks
                if (!mutual || v > other) {
                    h = other;
                    const u64 slot = atomicAdd(&s->mst, 1ull);
                    if (slot < (u64)n) W.mst[slot] = key;
                    s_flag = 1;
                }
            }
            st(&hook[v], h);
        }
        gsync();
        if (!s_flag) break;
        for (int v = tid; v < n; v += kH0Threads) st(&comp[v], ld(&hook[v]));
        for (int jump = 0; jump < 40; ++jump) {
            gsync();
            if (tid == 0) s_flag = 0;
            gsync();
            for (int v = tid; v < n; v += kH0Threads) {
                const int c = ld(&comp[v]), cc = ld(&comp[c]);
                if (c != cc) {
                    st(&comp[v], cc);
                    s_flag = 1;
                }
            }
            gsync();
            if (!s_flag) break;
        }
    }
    gsync();
    // sort the forest edges by key: refined filtration order
    const u64 mcount = ld(&s->mst);
    if (mcount > (u64)(n > 0 ? n - 1 : 0) && tid == 0) s->status = 4; // cannot happen
    const int m = (int)(mcount < (u64)n ? mcount : (u64)(n > 0 ? n - 1 : 0));
    SortBufs sb;
    sb.lo[0] = W.mst;
    sb.lo[1] = W.mst2;
    sb.hi[0] = W.hi;
    sb.hi[1] = W.hi2;
    sb.val[0] = W.val;
    sb.val[1] = W.val2;
    for (int e = tid; e < m; e += kH0Threads) {
        W.hi[e] = 0;
        W.val[e] = 0;
    }
    gsync();
    const int cur = block_radix_sort<kH0Threads>(sb, m, 8, 0, S);
    const u64 *keys = sb.lo[cur];
    // elder rule, 64 forest edges per step on wave 0: roots at the start of
    // the step come from the shared union-find; the merges inside the step
    // are resolved in order with wave shuffles
    int *parent = comp;
    int *maxv = hook;
    for (int v = tid; v < n; v += kH0Threads) {
        st(&parent[v], v);
        st(&maxv[v], v);
        W.hdeath[v] = -1.0f; // no bar (yet) born at v
    }
    gsync();
    if (tid < kWave) {
        const int lane = tid;
        for (int base = 0; base < m; base += kWave) {
            const int e = base + lane;
            const bool valid = e < m;
            int ra = 0, rb = 0, ma = -1, mb = -1;
            u32 idx = 0;
            float dm = 0.0f;
            if (valid) {
                const u64 key = keys[e];
                idx = 0xffffffffu - (u32)(key & 0xffffffffu);
                dm = __uint_as_float((u32)(key >> 32));
                int a, b;
                edge_vertices(idx, &a, &b);
                a = a < n ? a : n - 1;
                b = b < n ? b : n - 1;
                ra = uf_find(parent, a, n);
                rb = uf_find(parent, b, n);
                ma = ld(&maxv[ra]);
                mb = ld(&maxv[rb]);
            }
            const int cnt = min(kWave, m - base);
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
                    W.hdeath[my_birth] = dm;
                    W.hdsimp[my_birth] = (int64_t)idx;
                }
                if ((int64_t)idx < all_edges) atomicOr(&W.bits[idx >> 5], 1u << (idx & 31));
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        }
    }
    gsync();
    // essential classes: one per component, born at its oldest vertex
    for (int v = tid; v < n; v += kH0Threads)
        if (ld(&parent[v]) == v) {
            const int b = ld(&maxv[v]);
            W.hdeath[b] = INFINITY;
            W.hdsimp[b] = -1;
        }
    gsync();
    // bars by birth simplex descending (canonical order: all births are 0)
    int at = 0;
    int nz = 0, ness = 0;
    for (int base = 0; base < n; base += kH0Threads) {
        const int v = n - 1 - (base + tid);
        const float hd = v >= 0 ? W.hdeath[v] : -1.0f;
        const bool has = hd >= 0.0f;
        int tot;
        const int ex = block_exclusive_scan<kH0Threads>(has ? 1 : 0, s_w, &tot);
        if (has && at + ex < n) {
            out.birth[at + ex] = 0.0f;
            out.death[at + ex] = hd;
            out.bs[at + ex] = v;
            out.ds[at + ex] = W.hdsimp[v];
            if (isinf(hd)) ++ness;
            else ++nz;
        }
        at += tot;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        nz += __shfl_xor(nz, off, kWave);
        ness += __shfl_xor(ness, off, kWave);
    }
    if (lane_id() == 0) {
        atomicAdd(&s->stat[kStatBarsNonzero], (u64)nz);
        atomicAdd(&s->stat[kStatEssential], (u64)ness);
    }
    if (tid == 0) s->nbars = at < n ? at : n;
}

// ---------------------------------------------------------------------------
// expansion: all k-simplices <= t from the (k-1)-simplices, each exactly once
// as the cofacet sigma u {j} with j above sigma's largest vertex ("Assembling
// column indices": cofacets enumerated with all_cofacets = false).
// ---------------------------------------------------------------------------
template <int G, class Dist>
__global__ void __launch_bounds__(256) k_expand(Ctx<Dist> c, int k, SimplexList in, int64_t count,
                                                Scalars *s, SimplexList out, int64_t cap) {
    const int gpb = blockDim.x / G;
    const int lg = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * gpb;
    for (int64_t e = blockIdx.x * (int64_t)gpb + threadIdx.x / G; e < count; e += stride) {
        const int64_t idx = in.idx[e];
        const float dm0 = in.diam[e];
        int v[kMaxVerts];
        decode(idx, k - 1, c.n, c.B, v);
        const int top = v[0];
        const int *L = nullptr;
        int lo = top + 1, hi = c.n; // candidate range [lo, hi)
        if (c.nb.off != nullptr) {
            L = c.nb.idx + c.nb.off[top];
            const int len = c.nb.off[top + 1] - c.nb.off[top];
            // first neighbour above top
            int a = 0, b = len;
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (L[mid] <= top) a = mid + 1;
                else b = mid;
            }
            lo = a;
            hi = len;
        }
        for (int q0 = lo; q0 < hi; q0 += G) {
            const int q = q0 + lg;
            bool ok = q < hi;
            int j = 0;
            float nd = dm0;
            if (ok) {
                j = L ? L[q] : q;
                for (int m = 0; m < k; ++m) {
                    const float d = c.d(v[m], j);
                    ok = ok && (d <= c.t);
                    nd = fmaxf(nd, d);
                }
            }
            const int64_t slot = wave_append(&s->list, ok);
            if (ok && slot < cap) {
                out.idx[slot] = (int64_t)c.B(j, k + 1) + idx;
                out.diam[slot] = nd;
            }
        }
    }
}

// counting-only variant for the top dimension (throughput accounting)
template <int G, class Dist>
__global__ void __launch_bounds__(256) k_expand_count(Ctx<Dist> c, int k, SimplexList in,
                                                      int64_t count, Scalars *s) {
    const int gpb = blockDim.x / G;
    const int lg = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * gpb;
    u64 mine = 0;
    for (int64_t e = blockIdx.x * (int64_t)gpb + threadIdx.x / G; e < count; e += stride) {
        int v[kMaxVerts];
        decode(in.idx[e], k - 1, c.n, c.B, v);
        const int top = v[0];
        const int *L = nullptr;
        int lo = top + 1, hi = c.n;
        if (c.nb.off != nullptr) {
            L = c.nb.idx + c.nb.off[top];
            const int len = c.nb.off[top + 1] - c.nb.off[top];
            int a = 0, b = len;
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (L[mid] <= top) a = mid + 1;
                else b = mid;
            }
            lo = a;
            hi = len;
        }
        for (int q0 = lo; q0 < hi; q0 += G) {
            const int q = q0 + lg;
            bool ok = q < hi;
            if (ok) {
                const int j = L ? L[q] : q;
                for (int m = 0; m < k; ++m) ok = ok && (c.d(v[m], j) <= c.t);
            }
            mine += ok ? 1 : 0;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) mine += __shfl_xor(mine, off, kWave);
    if (lane_id() == 0 && mine) atomicAdd(&s->list, mine);
}

// ---------------------------------------------------------------------------
// The enumeration / apparent-pair pass (the hot data-parallel pass): for each
// candidate k-simplex sigma (diam <= t):
//   - cleared: sigma is a pivot of dimension k-1 (clearing; k = 1: a forest
//     edge of H0);
//   - sigma in a zero apparent pair (sigma, tau): tau = sigma u {j}, j the
//     largest vertex extending sigma at the same diameter, and sigma is tau's
//     first same-diameter facet;
//   - sigma in a zero apparent pair (rho, sigma) (k >= 2);
//   - otherwise sigma is a column to reduce; its zero pivot cofacet j (or -1)
//     and whether that cofacet is itself in a zero apparent pair are kept for
//     the emergent shortcut of the reduction.
// G lanes cooperate on one candidate (G candidate vertices per step); the
// dimension k is a template parameter, so vertex tuples stay in registers.
// The loop over candidates is uniform in the wave (one candidate per group
// per turn) and the tests are predicates, as the scans need every lane.
// ---------------------------------------------------------------------------
constexpr int kFilterLdsBinom = 8;                // flag of k_filter (beside the shortcut bits)
constexpr size_t kFilterLdsBinomMax = 16384;       // largest table staged in LDS

template <int G, int K, class Dist>
__global__ void __launch_bounds__(256) k_filter(Ctx<Dist> c, SimplexList in, int64_t count,
                                                const u32 *mst_bits, PivotHash prev, Scalars *s,
                                                Columns out, PairHash app, int flags) {
    // flags: kShortApparent (zero apparent pairs are no columns), kShortClearing,
    // kFilterLdsBinom (the binomial rows 0..K+2 staged in LDS, dynamic shared
    // memory; the launcher sets it for small tables only)
    extern __shared__ u64 btab[];
    if (flags & kFilterLdsBinom) {
        const int total = (K + 3) * c.B.stride;
        for (int i = threadIdx.x; i < total; i += blockDim.x) btab[i] = c.B.t[i];
        __syncthreads();
        c.B.t = btab;
    }
    const bool apparent = (flags & kShortApparent) != 0;
    const bool clearing = (flags & kShortClearing) != 0;
    constexpr int kGroups = kWave / G; // groups per wave
    const int lane = lane_id();
    const bool leader = (lane & (G - 1)) == 0;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    u64 n_clear = 0, n_acol = 0, n_apiv = 0;
    for (int64_t e0 = wave * kGroups; e0 < count; e0 += nwaves * kGroups) {
        const int64_t e = e0 + lane / G;
        bool live = e < count;
        int64_t idx = 0;
        float dm = 0.0f;
        int v[K + 1];
#pragma unroll
        for (int q = 0; q <= K; ++q) v[q] = 0;
        if (live) {
            idx = in.idx[e];
            dm = in.diam[e];
            bool cleared;
            if constexpr (K == 1) {
                edge_vertices((u32)idx, &v[0], &v[1]);
                cleared = (mst_bits[idx >> 5] >> (idx & 31)) & 1u;
            } else {
                decode(idx, K, c.n, c.B, v);
                cleared = ph_find(prev, idx) >= 0;
            }
            if (clearing && cleared) {
                n_clear += leader;
                live = false;
            }
        }
        // sigma's zero pivot cofacet sigma u {j}, if any
        const int j = scan_max_k<G, K>(c, v, dm, -1, live);
        int tv[K + 2];
        int pos = 0;
        insert_k<K>(v, j, tv, pos);
        if (apparent && live && j >= 0 && zero_pivot_facet_k<K + 1>(c, tv, dm) == pos) {
            // (sigma, sigma u {j}) is a zero apparent pair
            n_acol += leader;
            live = false;
            if (leader && app.keys) {
                // capacity is twice the candidates: the insert cannot fail
                u64 packed = kNoVerts;
                if (c.n <= 65536) {
                    packed = 0;
#pragma unroll
                    for (int q = 0; q <= K; ++q) packed |= (u64)(u32)v[q] << (16 * q);
                }
                u64 nbr = 0;
                if (c.nb.off != nullptr) {
                    int lo = c.nb.off[v[0]], du = c.nb.off[v[0] + 1] - lo;
#pragma unroll
                    for (int q = 1; q <= K; ++q) {
                        const int lq = c.nb.off[v[q]];
                        const int dq = c.nb.off[v[q] + 1] - lq;
                        if (dq < du) {
                            du = dq;
                            lo = lq;
                        }
                    }
                    nbr = ((u64)(u32)lo << 32) | (u32)du;
                }
                (void)pair_insert(app, simplex_index(tv, K + 1, c.B), (idx << 3) | pos, packed, nbr);
            }
        }
        if constexpr (K >= 2) {
            // sigma in a zero apparent pair (rho, sigma): rho = sigma's zero
            // pivot facet, and no vertex above the removed one extends rho at
            // the same diameter
            const int m = live && apparent ? zero_pivot_facet_k<K>(c, v, dm) : -1;
            int rv[K];
            remove_k<K>(v, m < 0 ? 0 : m, rv);
            const bool test = live && m >= 0;
            const int jr = scan_max_k<G, K - 1>(c, rv, dm, pick_vertex(v, m), test);
            if (test && jr < 0) {
                n_apiv += leader;
                live = false;
            }
        }
        // the same test for the zero pivot cofacet, for the emergent shortcut
        // (without the apparent shortcut, that cofacet's pair is a column too)
        const bool tj = apparent && live && j >= 0;
        const int mt = tj ? zero_pivot_facet_k<K + 1>(c, tv, dm) : -1;
        int rt[K + 1];
        remove_k<K + 1>(tv, mt < 0 ? 0 : mt, rt);
        const bool ttest = tj && mt >= 0;
        const int jt = scan_max_k<G, K>(c, rt, dm, pick_vertex(tv, mt), ttest);
        const uint8_t tapp = (ttest && jt < 0) ? 1 : 0;
        // survivors: one atomic per wave
        const u64 keep = __ballot(live && leader);
        if (keep) {
            unsigned long long base = 0;
            const int first = __ffsll((unsigned long long)keep) - 1;
            if (lane == first) base = atomicAdd(&s->survivors, (unsigned long long)__popcll(keep));
            base = __shfl(base, first, kWave);
            if (live && leader) {
                const u64 slot = base + (u64)__popcll(keep & ((1ull << lane) - 1ull));
                if (slot < (u64)count) { // one survivor per candidate at most
                    out.idx[slot] = idx;
                    out.diam[slot] = dm;
                    out.j[slot] = j;
                    out.tapp[slot] = tapp;
                }
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        n_clear += __shfl_xor(n_clear, off, kWave);
        n_acol += __shfl_xor(n_acol, off, kWave);
        n_apiv += __shfl_xor(n_apiv, off, kWave);
    }
    if (lane == 0) {
        if (n_clear) atomicAdd(&s->stat[kStatCleared], n_clear);
        if (n_acol) atomicAdd(&s->stat[kStatAppCol], n_acol);
        if (n_apiv) atomicAdd(&s->stat[kStatAppPiv], n_apiv);
    }
}

// ---------------------------------------------------------------------------
// sort of the columns: reverse filtration order, i.e. diameter descending,
// then CNS index ascending (youngest first). Keys: hi = ~diameter bits
// (diameters are >= +0, so bit order is value order), lo = index.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 1024;

__global__ void __launch_bounds__(kSortThreads) k_sort_columns(Columns in, Scalars *s,
                                                               SortBufs sb, int lo_bytes,
                                                               Columns out) {
    __shared__ SortShared<kSortThreads> S;
    const int N = (int)s->survivors;
    for (int e = threadIdx.x; e < N; e += kSortThreads) {
        sb.lo[0][e] = (u64)in.idx[e];
        sb.hi[0][e] = ~__float_as_uint(in.diam[e]);
        sb.val[0][e] = (u32)e;
    }
    __syncthreads();
    const int cur = block_radix_sort<kSortThreads>(sb, N, lo_bytes, 4, S);
    for (int q = threadIdx.x; q < N; q += kSortThreads) {
        const u32 e = sb.val[cur][q];
        out.idx[q] = in.idx[e];
        out.diam[q] = in.diam[e];
        out.j[q] = in.j[e];
        out.tapp[q] = in.tapp[e];
    }
}

// ---------------------------------------------------------------------------
// Reduction of the surviving columns over Z/p: one workgroup runs
// reduce_columns (rips_reduce.hpp) over the sorted columns of one dimension,
// with the working column's delta in LDS and its sorted base in global
// scratch.
// ---------------------------------------------------------------------------
// The job record of a reduction kernel, copied once into LDS and read from
// there. Read straight from the kernel arguments, its fields become
// wave-uniform scalar values, and that build of the reduction loses zero
// apparent pairs (the pivot lookups in the pair table miss, the columns end
// early, the bars are wrong; the same with SGPR spills to memory, without
// the VGPR live-range pass and at -O1); copied to LDS (or, as before, to
// scratch memory) the same source gives the oracle's bars, at the same
// speed. The cause is not found.
template <class Dist>
__device__ __forceinline__ const ReduceJob<Dist> &job_to_lds(const ReduceJob<Dist> &J) {
    __shared__ __align__(16) unsigned char jbuf[sizeof(ReduceJob<Dist>)];
    if (threadIdx.x == 0) __builtin_memcpy(jbuf, &J, sizeof(ReduceJob<Dist>));
    __syncthreads();
    return *reinterpret_cast<const ReduceJob<Dist> *>(jbuf);
}

template <class Dist>
__global__ void __launch_bounds__(kRedThreads) k_reduce(ReduceJob<Dist> J, u32 capD,
                                                       ReduceBuffers RB, Scalars *s) {
    extern __shared__ unsigned char smem[];
    __shared__ RedShared<kRedThreads> S;
    __shared__ int s_ns;
    LdsCol D;
    Staging G;
    SortedBase SB;
    carve_reduce_lds(smem, capD, (LDS int *)&s_ns, &D, &G, &SB);
    const BmLds L = carve_bm_lds(smem, reduce_lds_bytes(capD), J.bm_bits ? J.eo.E : 0);
    const ReduceScratch SC = make_scratch(RB, SB, (LDS int *)&S.vns);
    const ReduceJob<Dist> &Jl = job_to_lds(J);
    const int status = reduce_columns<kRedThreads>(Jl, D, G, SC, L, S);
    if (threadIdx.x == 0) {
        s->status = status;
        s->nbars = S.nbars;
        s->stat[kStatEmergent] += S.stat[0];
        s->stat[kStatReduced] += S.stat[1];
        s->stat[kStatAdditions] += S.stat[2];
        s->stat[kStatBarsNonzero] += S.stat[3];
        s->stat[kStatEssential] += S.stat[4];
        s->stat[kStatGlobalCols] += S.stat[5];
        s->stat[kStatMaxV] = S.stat[6];
        s->stat[kStatMaxR] = S.stat[7];
        s->stat[kStatPulls] += S.stat[8];
        s->stat[kStatMerges] += S.stat[9];
        s->stat[kStatSplits] += S.stat[10];
        s->stat[kStatPulled] += S.stat[11];
        s->stat[kStatAdded] += S.stat[12];
        for (int q = 0; q < kRedTimers; ++q) s->stat[kStatTime + q] += S.tm[q];
    }
}

// The reduction spread over a launch of `groups` workgroups (one per CU: the
// working column takes the LDS). Each workgroup has its own far list,
// working-V table and addition log, at blockIdx.x times their capacities.
template <class Dist>
__global__ void __launch_bounds__(kRedThreads) k_reduce_par(ReduceJob<Dist> J, u32 capD,
                                                           ReduceBuffers RB, Scalars *s) {
    extern __shared__ unsigned char smem[];
    __shared__ RedShared<kRedThreads> S;
    __shared__ int s_ns;
    LdsCol D;
    Staging G;
    SortedBase SB;
    carve_reduce_lds(smem, capD, (LDS int *)&s_ns, &D, &G, &SB);
    const int64_t g = blockIdx.x;
    ReduceBuffers R = RB;
    for (int b = 0; b < 2; ++b) {
        R.F.idx[b] += g * RB.F.cap;
        R.F.dia[b] += g * RB.F.cap;
        R.F.coef[b] += g * RB.F.cap;
    }
    R.vw_keys += g * RB.vw_cap;
    R.vw_coef += g * RB.vw_cap;
    R.vw_diam += g * RB.vw_cap;
    R.vw_slots += g * RB.vw_cap;
    R.lkey += g * RB.lcap;
    R.lcoef += g * RB.lcap;
    R.ldia += g * RB.lcap;
    const ReduceScratch SC = make_scratch(R, SB, (LDS int *)&S.vns);
    const BmLds L = carve_bm_lds(smem, reduce_lds_bytes(capD), J.bm_bits ? J.eo.E : 0);
    const ReduceJob<Dist> &Jl = job_to_lds(J);
    const int status = reduce_columns_par<kRedThreads>(Jl, D, G, SC, L, S);
    if (threadIdx.x == 0) {
        if (status && status != kRedAbort) atomicCAS(&s->status, 0, status);
        atomicAdd(&s->stat[kStatEmergent], S.stat[0]);
        atomicAdd(&s->stat[kStatReduced], S.stat[1]);
        atomicAdd(&s->stat[kStatAdditions], S.stat[2]);
        atomicAdd(&s->stat[kStatBarsNonzero], S.stat[3]);
        atomicAdd(&s->stat[kStatEssential], S.stat[4]);
        atomicAdd(&s->stat[kStatGlobalCols], S.stat[5]);
        atomicMax(&s->stat[kStatMaxV], S.stat[6]);
        atomicMax(&s->stat[kStatMaxR], S.stat[7]);
        atomicAdd(&s->stat[kStatPulls], S.stat[8]);
        atomicAdd(&s->stat[kStatMerges], S.stat[9]);
        atomicAdd(&s->stat[kStatSplits], S.stat[10]);
        atomicAdd(&s->stat[kStatPulled], S.stat[11]);
        atomicAdd(&s->stat[kStatAdded], S.stat[12]);
        for (int q = 0; q < kRedTimers; ++q) atomicAdd(&s->stat[kStatTime + q], S.tm[q]);
    }
}

// Bars of the spread-out reduction, one slot per column in column order
// (birth simplex -1: none), compacted in that order by one workgroup.
__global__ void __launch_bounds__(1024) k_compact_bars(BarBuf in, int64_t ncols, BarBuf out, Scalars *s) {
    __shared__ int s_w[1024 / kWave + 1];
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < ncols; c0 += 1024) {
        const int64_t q = c0 + threadIdx.x;
        const bool keep = q < ncols && in.bs[q] >= 0;
        int tot;
        const int at = block_exclusive_scan<1024>(keep ? 1 : 0, s_w, &tot);
        if (keep) {
            const int64_t d = base + at;
            out.birth[d] = in.birth[q];
            out.death[d] = in.death[q];
            out.bs[d] = in.bs[q];
            out.ds[d] = in.ds[q];
        }
        base += tot;
    }
    if (threadIdx.x == 0) s->nbars = base;
}

// The coboundary of the rho of every zero apparent pair (rho, tau) the filter
// recorded, listed once, in parallel: the reduction then adds such a
// coboundary by reading its list instead of scanning rho's neighbours. One
// wave per group of 64 table slots, one rho at a time (all control flow is
// uniform in the wave); a wave reserves room for its slots with one atomic.
// A slot whose list would not fit gets kNoList, and the reduction scans.
// spw (1..64) slots per wave: fewer slots give more waves, i.e. more
// independent chains of loads in flight. The room is reserved with one
// atomic per workgroup of 256 threads (one counter serializes its atomics).
template <class Dist>
__global__ void __launch_bounds__(256) k_cob_lists(Ctx<Dist> c, int k, PairHash app, int64_t *ckey,
                                                   float *cdia, unsigned long long *count, int64_t cap,
                                                   int spw) {
    constexpr int kWaves = 256 / kWave;
    __shared__ unsigned long long wsum[kWaves];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const bool dense = c.nb.off == nullptr;
    // block-uniform loop: every wave of a workgroup takes the same turns
    for (int64_t b0 = (int64_t)blockIdx.x * kWaves * spw; b0 <= (int64_t)app.mask;
         b0 += (int64_t)gridDim.x * kWaves * spw) {
        const int64_t s0 = b0 + (int64_t)w * spw;
        const int64_t s = s0 + lane;
        const bool full = lane < spw && s <= (int64_t)app.mask && app.keys[s] != kEmpty;
        // candidates of this lane's rho, then room for all of the block's lists
        int du = 0;
        if (full) du = dense ? c.n : (int)(u32)app.nbr[s];
        int incl = du;
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, kWave - 1, kWave);
        if (lane == 0) wsum[w] = (unsigned long long)total;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long run = 0;
            for (int q = 0; q < kWaves; ++q) {
                const unsigned long long t = wsum[q];
                wsum[q] = run;
                run += t;
            }
            const unsigned long long bbase = run > 0 ? atomicAdd(count, run) : 0ull;
            for (int q = 0; q < kWaves; ++q) wsum[q] += bbase;
        }
        __syncthreads();
        const unsigned long long wbase = wsum[w];
        __syncthreads(); // wsum is rewritten next turn
        const unsigned long long mybase = wbase + (unsigned long long)(incl - du);
        u64 todo = __ballot(full);
        while (todo) {
            const int l = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t slot = s0 + l;
            const unsigned long long base = __shfl(mybase, l, kWave);
            const int n_cand = __shfl(du, l, kWave);
            if ((int64_t)(base + n_cand) > cap || n_cand > 0xffffff) {
                if (lane == 0) app.cob[slot] = kNoList;
                continue;
            }
            int rv[kMaxVerts];
            const u64 vw = app.verts[slot];
            if (vw != kNoVerts) {
                for (int q = 0; q <= k; ++q) rv[q] = (int)((vw >> (16 * q)) & 0xffffu);
            } else {
                decode(app.vals[slot] >> 3, k, c.n, c.B, rv);
            }
            const float rd = diam_of(c, rv, k);
            const int lo = dense ? 0 : (int)(app.nbr[slot] >> 32);
            int w = 0;
            for (int q0 = 0; q0 < n_cand; q0 += kWave) {
                const int q = q0 + lane;
                bool ok = q < n_cand;
                int64_t ci = 0;
                float nd = rd;
                int below = 0;
                if (ok) {
                    const int jv = dense ? q : c.nb.idx[lo + q];
                    for (int m = 0; m <= k; ++m) {
                        ok = ok && jv != rv[m];
                        nd = fmaxf(nd, c.d(rv[m], jv));
                    }
                    ok = ok && nd <= c.t;
                    if (ok) ci = cofacet_index(rv, k, jv, c.B, &below);
                }
                const u64 b = __ballot(ok);
                if (ok) {
                    const int pos = w + __popcll(b & ((1ull << lane) - 1ull));
                    ckey[base + pos] = ci | ((int64_t)(below & 1) << 62);
                    cdia[base + pos] = nd;
                }
                w += __popcll(b);
            }
            if (lane == 0) app.cob[slot] = ((u64)base << 24) | (u64)w;
        }
    }
}

void launch_cob_lists(const Ctx<DistFull> &c, int k, PairHash app, int64_t *ckey, float *cdia,
                      unsigned long long *count, int64_t cap, hipStream_t st) {
    const int spw = 16; // table slots per wave
    const int64_t slots = (int64_t)app.mask + 1;
    const int64_t waves = (slots + spw - 1) / spw;
    int64_t blocks = (waves + 3) / 4; // 4 waves per workgroup of 256
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_cob_lists<DistFull>), dim3((unsigned)blocks), dim3(256), 0, st, c, k, app, ckey,
                       cdia, count, cap, spw);
}

// ---------------------------------------------------------------------------
// Backward: d(loss)/d(bar endpoint) scattered onto the critical edge of the
// endpoint's simplex (the edge of largest float32 length, ties to the
// smallest CNS edge index, i.e. the edge whose arrival gives the simplex its
// diameter in the refined order). One thread per (bar, endpoint).
// Points input: d ||x_u - x_v|| / d x_u = (x_u - x_v) / ||x_u - x_v||,
// the negative for x_v (no contribution at zero length). Distance-matrix
// input (m = 0): the gradient goes to entry (u, v), u > v, of the n x n
// matrix the forward read.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bw_dist(const float *X, int m, const float *M, int64_t nrow,
                                         int64_t u, int64_t v) {
    if (m == 0) return M[u * nrow + v];
    float s = 0.0f;
    for (int c = 0; c < m; ++c) {
        const float t = X[u * m + c] - X[v * m + c];
        const float sq = t * t;
        s = s + sq;
    }
    return __builtin_sqrtf(s);
}

__global__ void k_backward(const float *X, int m, int64_t nrow, int nmax, Binom B, int64_t nbars,
                           int kb, const int64_t *row0, const int64_t *bs, const int64_t *ds,
                           const float *gb, const float *gd, float *grad) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 2 * nbars) return;
    const int64_t bar = t >> 1;
    const bool death = t & 1;
    const int k = death ? kb + 1 : kb;
    const int64_t idx = death ? ds[bar] : bs[bar];
    const float g = death ? gd[bar] : gb[bar];
    if (k < 1 || k > kMaxDim + 1 || idx < 0 || g == 0.0f) return;
    int v[kMaxVerts + 1];
    decode(idx, k, nmax, B, v); // decreasing vertices
    const int64_t r0 = row0 ? row0[bar] : 0;
    const float *Xc = m ? X + r0 * m : nullptr;
    const float *Mc = m ? nullptr : X;
    float best = -1.0f;
    int64_t beste = 0;
    int bu = 0, bv = 0;
    for (int a = 0; a <= k; ++a)
        for (int b = a + 1; b <= k; ++b) {
            const int u = v[a], w = v[b]; // u > w
            const float d = bw_dist(Xc, m, Mc, nrow, u, w);
            const int64_t e = (int64_t)B(u, 2) + w;
            if (d > best || (d == best && e < beste)) {
                best = d;
                beste = e;
                bu = u;
                bv = w;
            }
        }
    if (m == 0) {
        atomicAdd(&grad[(int64_t)bu * nrow + bv], g);
        return;
    }
    if (!(best > 0.0f)) return;
    const float sc = g / best;
    float *gu = grad + (r0 + bu) * m;
    float *gv = grad + (r0 + bv) * m;
    for (int c = 0; c < m; ++c) {
        const float diff = Xc[(int64_t)bu * m + c] - Xc[(int64_t)bv * m + c];
        const float q = sc * diff;
        atomicAdd(&gu[c], q);
        atomicAdd(&gv[c], -q);
    }
}

void launch_backward(const float *X, int m, int64_t nrow, int nmax, Binom B, int64_t nbars,
                     int kb, const int64_t *row0, const int64_t *bs, const int64_t *ds,
                     const float *gb, const float *gd, float *grad, hipStream_t st) {
    if (nbars <= 0) return;
    const int64_t threads = 2 * nbars;
    hipLaunchKernelGGL(k_backward, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, X, m,
                       nrow, nmax, B, nbars, kb, row0, bs, ds, gb, gd, grad);
}

// bars of one dimension into the caller's arrays; reverse = column order was
// youngest first, the canonical order is the reverse
__global__ void k_emit(BarBuf in, Scalars *s, int reverse, BarBuf out) {
    const int64_t nb = s->nbars;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nb;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t src = reverse ? nb - 1 - q : q;
        out.birth[q] = in.birth[src];
        out.death[q] = in.death[src];
        out.bs[q] = in.bs[src];
        out.ds[q] = in.ds[src];
    }
}

// ---------------------------------------------------------------------------
// instantiations / launchers
// ---------------------------------------------------------------------------
template <int G, int K>
static void launch_filter_gk(const Ctx<DistFull> &c, SimplexList in, int64_t count, PairHash app,
                             const u32 *bits, PivotHash prev, Scalars *s, Columns out, int flags,
                             hipStream_t st) {
    const int gpb = 256 / G;
    int64_t blocks = (count + gpb - 1) / gpb;
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    // the binomial rows the filter reads, in LDS when they are small: every
    // workgroup copies them first, and a large table costs occupancy (measured:
    // 3 KB, sphere-100: 23 -> 19 us; 40 KB, so3-1000 dimension 2: 180 -> 175 us;
    // 80 KB, torus4-2000 dimension 2: 196 -> 272 us)
    const size_t lds = (size_t)(K + 3) * c.B.stride * 8;
    const bool stage = lds <= kFilterLdsBinomMax;
    hipLaunchKernelGGL((k_filter<G, K, DistFull>), dim3((unsigned)blocks), dim3(256), stage ? lds : 0, st, c,
                       in, count, bits, prev, s, out, app, flags | (stage ? kFilterLdsBinom : 0));
}

template <int G>
static void launch_filter_g(const Ctx<DistFull> &c, int k, SimplexList in, int64_t count, PairHash app,
                            const u32 *bits, PivotHash prev, Scalars *s, Columns out, int flags,
                            hipStream_t st) {
    switch (k) {
    case 1: launch_filter_gk<G, 1>(c, in, count, app, bits, prev, s, out, flags, st); break;
    case 2: launch_filter_gk<G, 2>(c, in, count, app, bits, prev, s, out, flags, st); break;
    default: launch_filter_gk<G, 3>(c, in, count, app, bits, prev, s, out, flags, st); break;
    }
}

void launch_filter(int G, const Ctx<DistFull> &c, int k, SimplexList in, int64_t count,
                   const u32 *bits, PivotHash prev, Scalars *s, Columns out, PairHash app, int flags,
                   hipStream_t st) {
    switch (G) {
    case 1: launch_filter_g<1>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    case 2: launch_filter_g<2>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    case 4: launch_filter_g<4>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    case 8: launch_filter_g<8>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    case 16: launch_filter_g<16>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    case 32: launch_filter_g<32>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    default: launch_filter_g<64>(c, k, in, count, app, bits, prev, s, out, flags, st); break;
    }
}

template <int G>
static void launch_expand_g(const Ctx<DistFull> &c, int k, SimplexList in, int64_t count,
                            Scalars *s, SimplexList out, int64_t cap, bool count_only,
                            hipStream_t st) {
    const int gpb = 256 / G;
    int64_t blocks = (count + gpb - 1) / gpb;
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    if (count_only)
        hipLaunchKernelGGL((k_expand_count<G, DistFull>), dim3((unsigned)blocks), dim3(256), 0, st,
                           c, k, in, count, s);
    else
        hipLaunchKernelGGL((k_expand<G, DistFull>), dim3((unsigned)blocks), dim3(256), 0, st, c, k,
                           in, count, s, out, cap);
}

void launch_expand(int G, const Ctx<DistFull> &c, int k, SimplexList in, int64_t count, Scalars *s,
                   SimplexList out, int64_t cap, bool count_only, hipStream_t st) {
    switch (G) {
    case 8: launch_expand_g<8>(c, k, in, count, s, out, cap, count_only, st); break;
    case 16: launch_expand_g<16>(c, k, in, count, s, out, cap, count_only, st); break;
    case 32: launch_expand_g<32>(c, k, in, count, s, out, cap, count_only, st); break;
    default: launch_expand_g<64>(c, k, in, count, s, out, cap, count_only, st); break;
    }
}

void launch_binom(u64 *B, int stride, int n, int jmax, hipStream_t st) {
    hipLaunchKernelGGL(k_binom, dim3((n + 1 + 255) / 256), dim3(256), 0, st, B, stride, n, jmax);
}

void launch_inverse(u32 *inv, u32 p, hipStream_t st) {
    hipLaunchKernelGGL(k_inverse, dim3((p + 255) / 256), dim3(256), 0, st, inv, p);
}

void launch_dist(const float *data, int n, int m, float *D, int *bad, hipStream_t st) {
    dim3 grid((n + 255) / 256, n);
    if (m > 0) hipLaunchKernelGGL(k_dist_points, grid, dim3(256), 0, st, data, n, m, D, bad);
    else hipLaunchKernelGGL(k_dist_matrix, grid, dim3(256), 0, st, data, n, D, bad);
}

void launch_init_scalars(Scalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(1), 0, st, s);
}

void launch_reset_dim(Scalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_dim, dim3(1), dim3(1), 0, st, s);
}

void launch_threshold(const float *D, int n, float t, Scalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_rowmax, dim3((n + 3) / 4), dim3(256), 0, st, D, n, s);
    hipLaunchKernelGGL(k_set_teff, dim3(1), dim3(1), 0, st, s, t);
}

void launch_edges(const float *D, int n, Scalars *s, EdgeList E, int64_t cap, int *deg,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_zero_int, dim3(64), dim3(256), 0, st, deg, (int64_t)n + 1);
    hipLaunchKernelGGL(k_edges, dim3((n + 3) / 4), dim3(256), 0, st, D, n, s, E, cap, deg);
}

void launch_csr(const float *D, int n, Scalars *s, const int *deg, int *off, int *nbr,
                hipStream_t st) {
    hipLaunchKernelGGL(k_scan_deg, dim3(1), dim3(1024), 0, st, deg, n, off);
    hipLaunchKernelGGL(k_csr_fill, dim3(n), dim3(256), 0, st, D, n, s, off, nbr);
}

__global__ void k_reset_mst(Scalars *s) { s->mst = 0; }

void launch_h0(EdgeList E, Scalars *s, int n, H0Scratch W, BarBuf out, int64_t nbits_words,
               hipStream_t st) {
    hipLaunchKernelGGL(k_zero_int, dim3(256), dim3(256), 0, st, (int *)W.bits, nbits_words);
    hipLaunchKernelGGL(k_reset_mst, dim3(1), dim3(1), 0, st, s);
    hipLaunchKernelGGL(k_h0, dim3(1), dim3(kH0Threads), 0, st, E, s, n, W, out);
}

void launch_fill_i64(int64_t *a, int64_t n, int64_t v, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)blocks), dim3(256), 0, st, a, n, v);
}

void launch_fill_u32(u32 *a, int64_t n, u32 v, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, a, n, v);
}


// The edges <= t in order of length for the direct-mapped working column of
// dimension 1 (one workgroup): a sort on the length bits, then position ->
// vertices, length and run word, and (a, b) -> position in the n x n table.
__global__ void __launch_bounds__(1024) k_bm_edge_order(EdgeList E, int nE, int n, SortBufs sb, int *pos,
                                                        u32 *verts, float *len, u32 *run) {
    __shared__ SortShared<1024> S;
    for (int q = threadIdx.x; q < nE; q += 1024) {
        sb.lo[0][q] = (u64)E.idx[q];
        sb.hi[0][q] = __float_as_uint(E.diam[q]);
        sb.val[0][q] = (u32)q;
    }
    gsync();
    // equal lengths may come in any order (the pivot search scans a run of
    // them whole), so the length bits alone are the key
    const int cur = block_radix_sort<1024>(sb, nE, 0, 4, S);
    for (int q = threadIdx.x; q < nE; q += 1024) {
        const u32 e = sb.val[cur][q];
        pos[(int64_t)E.a[e] * n + E.b[e]] = q;
        pos[(int64_t)E.b[e] * n + E.a[e]] = q;
        verts[q] = ((u32)E.a[e] << 16) | (u32)E.b[e];
        len[q] = E.diam[e];
    }
    gsync();
    for (int q = threadIdx.x; q < nE; q += 1024) {
        const u32 key = sb.hi[cur][q];
        int r = q;
        while (r > 0 && sb.hi[cur][r - 1] == key) --r;
        const bool tie = q + 1 < nE && sb.hi[cur][q + 1] == key;
        run[q] = (u32)r | (tie ? kRunTie : 0u);
    }
}

// Per edge position, the third vertex of the edge's zero apparent cofacet:
// for every pair (rho, tau) of the table, app[pos(rho)] = the vertex of tau
// off rho (app holds -1 elsewhere).
__global__ void k_bm_app(PairHash tab, const int *pos, int n, int *app) {
    const u32 cap = tab.mask + 1;
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < cap; q += gridDim.x * blockDim.x) {
        const int64_t tau = tab.keys[q];
        if (tau == kEmpty) continue;
        const int64_t rho = tab.vals[q] >> 3;
        int a, b;
        edge_vertices((u32)rho, &a, &b);
        // tau = C(x, 3) + C(y, 2) + z with x > y > z
        int x = (int)cbrt(6.0 * (double)tau) + 1;
        while ((int64_t)x * (x - 1) * (x - 2) / 6 > tau) --x;
        while ((int64_t)(x + 1) * x * (x - 1) / 6 <= tau) ++x;
        int y, z;
        edge_vertices((u32)(tau - (int64_t)x * (x - 1) * (x - 2) / 6), &y, &z);
        const int c = (x != a && x != b) ? x : (y != a && y != b) ? y : z;
        const int p = pos[(int64_t)a * n + b];
        if (p >= 0) app[p] = c;
    }
}

void launch_bm_edge_order(EdgeList E, int nE, int n, SortBufs sb, int *pos, u32 *verts, float *len, u32 *run,
                          PairHash app_tab, int *app, hipStream_t st) {
    launch_fill_u32((u32 *)pos, (int64_t)n * n, 0xffffffffu, st);
    launch_fill_u32((u32 *)app, nE, 0xffffffffu, st);
    hipLaunchKernelGGL(k_bm_edge_order, dim3(1), dim3(1024), 0, st, E, nE, n, sb, pos, verts, len, run);
    if (app_tab.keys) {
        const int64_t cap = (int64_t)app_tab.mask + 1;
        const unsigned blocks = (unsigned)std::min<int64_t>(1024, (cap + 255) / 256);
        hipLaunchKernelGGL(k_bm_app, dim3(blocks), dim3(256), 0, st, app_tab, (const int *)pos, n, app);
    }
}

void launch_sort_columns(Columns in, Scalars *s, SortBufs sb, int lo_bytes, Columns out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_sort_columns, dim3(1), dim3(kSortThreads), 0, st, in, s, sb, lo_bytes,
                       out);
}

hipError_t launch_reduce(const ReduceJob<DistFull> &J, u32 capD, ReduceBuffers RB, Scalars *s,
                         hipStream_t st) {
    const size_t lds = reduce_lds_bytes(capD) + (J.bm_bits ? bm_lds_bytes(J.eo.E) : 0);
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce<DistFull>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce<DistFull>), dim3(1), dim3(kRedThreads), lds, st, J, capD, RB, s);
    return hipGetLastError();
}

hipError_t launch_reduce_par(const ReduceJob<DistFull> &J, u32 capD, ReduceBuffers RB, int groups,
                             BarBuf out, Scalars *s, hipStream_t st) {
    const size_t lds = reduce_lds_bytes(capD) + (J.bm_bits ? bm_lds_bytes(J.eo.E) : 0);
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce_par<DistFull>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_par<DistFull>), dim3(groups), dim3(kRedThreads), lds, st, J, capD, RB,
                       s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_bars, dim3(1), dim3(1024), 0, st, J.bars, (int64_t)J.ncols,
                       out, s);
    return hipGetLastError();
}

void launch_emit(BarBuf in, Scalars *s, int reverse, BarBuf out, hipStream_t st) {
    hipLaunchKernelGGL(k_emit, dim3(64), dim3(256), 0, st, in, s, reverse, out);
}

} // namespace rips
