// rips_device.hpp -- device building blocks of the gfx950 Vietoris-Rips
// persistence path (wave64, CDNA4). Written from U. Bauer, "Ripser: efficient
// computation of Vietoris-Rips persistence barcodes" (arXiv:1908.02518).
//
// Everything here is integer and comparison work: combinatorial-number-system
// (CNS) encoding and decoding, cofacet and facet enumeration, the zero
// apparent pair tests, open-addressing hash tables, and a block-wide LSD
// radix sort. No floating point arithmetic beyond comparisons happens on
// distances here; distances are computed once (rips_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rips {

typedef unsigned long long u64;
typedef uint32_t u32;

constexpr int kWave = 64;
constexpr int kMaxDim = 3;             // largest homology dimension
constexpr int kMaxVerts = kMaxDim + 2; // vertices of a cofacet of a top-dimension column
constexpr int64_t kEmpty = -1;         // empty hash slot / "no simplex"

// ---------------------------------------------------------------------------
// Binomial coefficient table, C(i, j) at t[j * stride + i], 0 <= i <= n,
// 0 <= j <= kMaxDim + 2 (the table of the "Vertices and simplices" paragraph).
// ---------------------------------------------------------------------------
struct Binom {
    const u64 *t;
    int stride;
    __host__ __device__ __forceinline__ u64 operator()(int i, int j) const {
        return t[(int64_t)j * stride + i];
    }
};

// ---------------------------------------------------------------------------
// Distance access.
// ---------------------------------------------------------------------------

// Full n x n row-major float32 matrix in global memory (HBM, L2/MALL
// resident for the sizes of one cloud). Row v is contiguous, so a wave that
// scans candidate vertices j for a fixed simplex vertex v reads coalesced.
struct DistFull {
    const float *D;
    int n;
    __device__ __forceinline__ float operator()(int a, int b) const {
        return D[(int64_t)a * n + b];
    }
};

// Packed lower triangle (entry (a, b), a > b, at a(a-1)/2 + b, which is the
// CNS index of the edge {a, b}), used when one cloud's matrix lives in LDS.
struct DistPacked {
    const float *D;
    int n;
    __device__ __forceinline__ float operator()(int a, int b) const {
        if (a == b) return 0.0f;
        int hi = a > b ? a : b, lo = a > b ? b : a;
        return D[hi * (hi - 1) / 2 + lo];
    }
};

// Neighbour lists within the threshold, ascending by neighbour index (the
// adjacency lists of the "sparse distance matrix"); off == nullptr means
// dense enumeration over all vertices.
struct Nbrs {
    const int *off;
    const int *idx;
};

template <class Dist>
struct Ctx {
    Dist d;
    Binom B;
    Nbrs nb;
    int n;
    float t;
};

// ---------------------------------------------------------------------------
// Combinatorial number system.
// A k-simplex is the decreasing tuple v[0] > v[1] > ... > v[k]; with i_l the
// l-th smallest vertex its index is sum_l C(i_l, l + 1).
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ int64_t simplex_index(const int *v, int k, Binom B) {
    int64_t s = 0;
    for (int m = 0; m <= k; ++m) s += (int64_t)B(v[m], k - m + 1);
    return s;
}

// Largest i in [lo, hi] with C(i, r) <= x, 2 <= r <= 5. The start comes
// from C(i, r) ~ (i - (r - 1) / 2)^r / r! in double precision and is then
// corrected against the exact table: two independent table reads in the
// usual case instead of a binary search's chain of dependent ones.
__host__ __device__ __forceinline__ int top_vertex(u64 x, int r, int lo, int hi, Binom B) {
    const double xd = (double)x;
    double g;
    if (r == 2) g = 0.5 + sqrt(2.0 * xd + 0.25);
    else if (r == 3) g = cbrt(6.0 * xd) + 1.0;
    else if (r == 4) g = sqrt(sqrt(24.0 * xd)) + 1.5;
    else g = pow(120.0 * xd, 0.2) + 2.0;
    int i = g < (double)lo ? lo : (g > (double)hi ? hi : (int)g);
    u64 a = B(i, r);
    u64 b = i < hi ? B(i + 1, r) : ~0ull;
    while (a > x && i > lo) {
        --i;
        b = a;
        a = B(i, r);
    }
    while (b <= x && i < hi) {
        ++i;
        a = b;
        b = i < hi ? B(i + 1, r) : ~0ull;
    }
    return i;
}

// Vertices of the k-simplex with index idx on n vertices, decreasing: the
// largest vertex is the largest i with C(i, k+1) <= idx (Lemma of the
// "Vertices and simplices" paragraph); then recurse on the rest.
__host__ __device__ __forceinline__ void decode(int64_t idx, int k, int n, Binom B, int *v) {
    int hi = n - 1;
    for (int l = k; l >= 1; --l) {
        const int i = top_vertex((u64)(idx < 0 ? 0 : idx), l + 1, l, hi < l ? l : hi, B);
        v[k - l] = i;
        idx -= (int64_t)B(i, l + 1);
        hi = i - 1;
    }
    // valid indices leave 0 <= idx <= hi; the clamp only keeps a corrupted
    // index from addressing outside the distance matrix
    v[k] = (int)(idx < 0 ? 0 : (idx > hi ? hi : idx));
}

// Index of the cofacet sigma u {j}, j not in sigma (section "Enumerating
// cofacets and facets"): vertices above j move up one binomial order. The
// number of vertices of sigma below j is returned in *below; the coefficient
// of the cofacet in the coboundary is (-1)^below (standard orientation).
__host__ __device__ __forceinline__ int64_t cofacet_index(const int *v, int k, int j, Binom B,
                                                         int *below) {
    int64_t s = 0;
    int nb = 0;
    for (int m = 0; m <= k; ++m) {
        int l = k - m;
        if (v[m] > j) s += (int64_t)B(v[m], l + 2);
        else {
            s += (int64_t)B(v[m], l + 1);
            ++nb;
        }
    }
    s += (int64_t)B(j, nb + 1);
    *below = nb;
    return s;
}

// Insert j into the decreasing tuple v[0..k]; returns the position of j.
__host__ __device__ __forceinline__ int insert_vertex(const int *v, int k, int j, int *out) {
    int q = 0, pos = -1;
    for (int m = 0; m <= k; ++m) {
        if (pos < 0 && j > v[m]) {
            pos = q;
            out[q++] = j;
        }
        out[q++] = v[m];
    }
    if (pos < 0) {
        pos = q;
        out[q] = j;
    }
    return pos;
}

__host__ __device__ __forceinline__ void remove_vertex(const int *v, int k, int m, int *out) {
    int q = 0;
    for (int u = 0; u <= k; ++u)
        if (u != m) out[q++] = v[u];
}

__host__ __device__ __forceinline__ u32 coeff_sign(int below, u32 p) {
    return (below & 1) ? (p - 1) : 1u;
}

template <class Dist>
__device__ __forceinline__ float diam_of(const Ctx<Dist> &c, const int *v, int k) {
    float m = 0.0f;
    for (int a = 0; a < k + 1; ++a)
        for (int b = a + 1; b < k + 1; ++b) m = fmaxf(m, c.d(v[a], v[b]));
    return m;
}

// Zero pivot facet: the first facet in forward colexicographic order (i.e.
// removing v[0], then v[1], ...) whose diameter equals the simplex's. Returns
// the position of the removed vertex or -1.
template <class Dist>
__device__ __forceinline__ int zero_pivot_facet(const Ctx<Dist> &c, const int *v, int k, float dm) {
    float pd[kMaxVerts][kMaxVerts];
    for (int a = 0; a <= k; ++a)
        for (int b = a + 1; b <= k; ++b) pd[a][b] = c.d(v[a], v[b]);
    for (int m = 0; m <= k; ++m) {
        float mx = 0.0f;
        for (int a = 0; a <= k; ++a)
            for (int b = a + 1; b <= k; ++b)
                if (a != m && b != m) mx = fmaxf(mx, pd[a][b]);
        if (mx == dm) return m;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Wave / group helpers. A "group" is G consecutive lanes of one wave64 that
// cooperate on one simplex; every lane of a group follows the same control
// flow, different groups of a wave may diverge.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Barrier for phases that hand data between the waves of one workgroup
// through global memory. The workgroup barrier's release/acquire fences
// cover global memory as well as LDS, and a workgroup's scratch is its own,
// so workgroup scope is enough. An agent-scope fence writes back (release)
// or invalidates (acquire) the L2 of the XCD, whose L2s are not coherent
// with each other: it is kept to the few places where workgroups of one
// launch hand data to each other (the reduction spread over workgroups).
__device__ __forceinline__ void gsync() { __syncthreads(); }

// Agent-scope relaxed loads / stores, for words that workgroups of one
// launch exchange (they bypass the non-coherent caches), and agent-scope
// fences that order the plain accesses around them.
template <class T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void st_dev(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void fence_release_dev() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire_dev() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Relaxed workgroup-scope atomic load / store, for words that other waves
// of the workgroup update with atomics (atomics execute in L2; these loads
// do not return a stale L1 copy).
template <class T>
__device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <class T>
__device__ __forceinline__ void st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Pointers into LDS carry the local address space, so that accesses compile
// to ds_* instructions rather than flat ones (a flat access also waits for
// every outstanding global load of the wave).
#define LDS __attribute__((address_space(3)))

template <class T>
__device__ __forceinline__ T ld(const LDS T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <class T>
__device__ __forceinline__ void st(LDS T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Pointers into global memory carry the global address space where it
// matters. A pointer read from memory (the reduction's job record is copied
// to LDS) is generic, and a generic access compiles to a flat instruction,
// which counts on the LDS counter as well as on the vector-memory counter:
// every later LDS wait of the wave then also waits for that global access
// (an atomic to a line in HBM, say). gp() casts a pointer that is known to
// point to global memory.
#define GLB __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ GLB T *gp(T *p) {
    return (GLB T *)p;
}

template <class T>
__device__ __forceinline__ const GLB T *gp(const T *p) {
    return (const GLB T *)p;
}

template <class T>
__device__ __forceinline__ T ld(const GLB T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <class T>
__device__ __forceinline__ void st(GLB T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Hand-over point between the lanes of one wave, for code that one wave
// runs alone (no workgroup barrier): values that other lanes stored to
// shared or global memory before it are read after it. Without it the
// compiler, reasoning about each lane on its own, may serve a later load
// from a value loaded earlier (a lane that did not store sees no reason to
// load again) or move the access across the other lanes' stores. A
// wavefront-scope fence is such a point for the compiler and costs no
// instruction (a wave's memory accesses execute in order); the wave barrier
// keeps the scheduler from moving work across it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Lanes of this lane's group of G in a wave-wide mask.
template <int G>
__device__ __forceinline__ u64 group_mask() {
    if (G >= 64) return ~0ull;
    const int base = lane_id() & ~(G - 1);
    return ((1ull << (G & 63)) - 1) << base;
}

// ---------------------------------------------------------------------------
// The zero apparent pair tests with the dimension K fixed at compile time, for the
// enumeration / apparent-pair pass: every tuple is indexed by constants, so
// it stays in registers. The scans are called by every lane of the wave at
// once; their loops run until every group of the wave is done, so no lane
// leaves a loop holding a wave operation while others stay in it.
// ---------------------------------------------------------------------------

// v[m] for a run-time m, by selects over constant positions.
template <int N>
__device__ __forceinline__ int pick_vertex(const int (&v)[N], int m) {
    int r = v[0];
#pragma unroll
    for (int q = 1; q < N; ++q) r = q == m ? v[q] : r;
    return r;
}

// sigma u {j} for the decreasing tuple v of a K-simplex, j not in v; pos =
// the position of j (the number of vertices above it).
template <int K>
__device__ __forceinline__ void insert_k(const int (&v)[K + 1], int j, int (&out)[K + 2], int &pos) {
    int above = 0;
#pragma unroll
    for (int m = 0; m <= K; ++m) above += v[m] > j ? 1 : 0;
    pos = above;
#pragma unroll
    for (int q = 0; q <= K + 1; ++q) {
        const int lo = v[q <= K ? q : K];     // v[q], when q < above
        const int hi = v[q >= 1 ? q - 1 : 0]; // v[q - 1], when q > above
        out[q] = q < above ? lo : (q == above ? j : hi);
    }
}

// The facet of the K-simplex v without v[m].
template <int K>
__device__ __forceinline__ void remove_k(const int (&v)[K + 1], int m, int (&out)[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] = q < m ? v[q] : v[q + 1];
}

// Position of the removed vertex of the zero pivot facet of the K-simplex v
// (diameter dm): the first facet, removing v[0], v[1], ..., whose diameter
// is dm; -1 if none.
template <int K, class Dist>
__device__ __forceinline__ int zero_pivot_facet_k(const Ctx<Dist> &c, const int (&v)[K + 1], float dm) {
    float pd[K + 1][K + 1];
#pragma unroll
    for (int a = 0; a <= K; ++a)
#pragma unroll
        for (int b = a + 1; b <= K; ++b) pd[a][b] = c.d(v[a], v[b]);
    int res = -1;
#pragma unroll
    for (int m = K; m >= 0; --m) {
        float mx = 0.0f;
#pragma unroll
        for (int a = 0; a <= K; ++a)
#pragma unroll
            for (int b = a + 1; b <= K; ++b)
                if (a != m && b != m) mx = fmaxf(mx, pd[a][b]);
        if (mx == dm) res = m;
    }
    return res;
}

// Largest vertex j > jmin, j not in the K-simplex v, with d(j, v_m) <= bound
// for every m; -1 if none, or if the group is not active. Candidates are
// scanned in decreasing order (decreasing CNS order of the cofacets
// v u {j}), G at a time, and the scan of a group stops at its first chunk
// with a hit (the early exit of the apparent-pair test); dense: all
// vertices, sparse: the neighbour list of the vertex of v with the fewest
// neighbours. All lanes of a group get the same result.
template <int G, int K, class Dist>
__device__ __forceinline__ int scan_max_k(const Ctx<Dist> &c, const int (&v)[K + 1], float bound,
                                          int jmin, bool active) {
    const int lg = lane_id() & (G - 1);
    const u64 gm = group_mask<G>();
    const bool dense = c.nb.off == nullptr;
    const int *L = nullptr;
    int top = c.n - 1; // dense: next vertex; sparse: next position in L
    if (active && !dense) {
        int u = v[0];
        int du = c.nb.off[u + 1] - c.nb.off[u];
#pragma unroll
        for (int m = 1; m <= K; ++m) {
            const int dq = c.nb.off[v[m] + 1] - c.nb.off[v[m]];
            if (dq < du) {
                du = dq;
                u = v[m];
            }
        }
        L = c.nb.idx + c.nb.off[u];
        top = du - 1;
    }
    int res = -1;
    bool done = !active;
    while (__ballot(!done) != 0) {
        bool ok = false;
        int j = -1;
        if (!done) {
            // the rest of a sparse list is smaller still once its top is <= jmin
            if (dense ? top <= jmin : (top < 0 || L[top] <= jmin)) {
                done = true;
            } else {
                const int q = top - lg;
                j = dense ? q : (q >= 0 ? L[q] : -1);
                ok = j > jmin;
#pragma unroll
                for (int m = 0; m <= K; ++m) ok = ok && j != v[m];
                if (ok) {
#pragma unroll
                    for (int m = 0; m <= K; ++m) ok = ok && c.d(v[m], j) <= bound;
                }
            }
        }
        const u64 hit = __ballot(ok) & gm;
        const int jj = __shfl(j, hit ? __ffsll((unsigned long long)hit) - 1 : lane_id(), kWave);
        if (!done) {
            if (hit) {
                res = jj;
                done = true;
            } else {
                top -= G;
            }
        }
    }
    return res;
}

// ---------------------------------------------------------------------------
// Hashing.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ u32 mix64(u64 x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return (u32)x;
}

// Pivot table of one dimension: pivot (a (k+1)-simplex) -> column position.
// Apparent pairs are never stored (section "Implementation", persistence
// pairs paragraph); the table only holds pivots found by the reduction.
struct PivotHash {
    int64_t *keys; // kEmpty when free
    int32_t *vals;
    u32 mask;      // capacity - 1, capacity a power of two
};

__device__ __forceinline__ int32_t ph_find(const PivotHash &h, int64_t key) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = ld(&h.keys[s]);
        if (cur == key) return ld(&h.vals[s]);
        if (cur == kEmpty) return -1;
        s = (s + 1) & h.mask;
    }
    return -1;
}

__device__ __forceinline__ bool ph_insert(const PivotHash &h, int64_t key, int32_t val) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const u64 prev = atomicCAS((u64 *)&h.keys[s], (u64)kEmpty, (u64)key);
        if (prev == (u64)kEmpty || prev == (u64)key) {
            st(&h.vals[s], val);
            return true;
        }
        s = (s + 1) & h.mask;
    }
    return false;
}

// The same table shared by the workgroups of one launch. A slot's value is
// -1 until its writer stores it, and a reader takes -1 for "not there": the
// writer stores the value after everything it publishes with it, behind an
// agent-scope release fence, and a reader that finds a value and then reads
// what it refers to issues an agent-scope acquire fence first.
__device__ __forceinline__ int32_t ph_find_dev(const PivotHash &h, int64_t key) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = ld_dev(&h.keys[s]);
        if (cur == key) return ld_dev(&h.vals[s]);
        if (cur == kEmpty) return -1;
        s = (s + 1) & h.mask;
    }
    return -1;
}

__device__ __forceinline__ bool ph_insert_dev(const PivotHash &h, int64_t key, int32_t val) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        int64_t expect = kEmpty;
        const bool won = __hip_atomic_compare_exchange_strong(&h.keys[s], &expect, key, __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (won || expect == key) {
            st_dev(&h.vals[s], val);
            return true;
        }
        s = (s + 1) & h.mask;
    }
    return false;
}

// Zero apparent pairs (rho, tau) of one dimension, recorded by the filter:
// tau -> (rho << 3) | m, m = position in tau's decreasing vertex list of the
// vertex tau adds to rho. Sized at twice the candidates, so inserts never
// fail; the reduction then finds whether its pivot is such a tau with one
// lookup. Beside the value, each slot keeps what the addition of rho's
// coboundary needs next, so that it costs no further dependent load: rho's
// vertices (decreasing, 16 bits each; kNoVerts when n > 65536) and, with
// neighbour lists, the list of rho's vertex with the fewest neighbours
// (first entry << 32 | length). Either array may be absent (null).
constexpr u64 kNoVerts = ~0ull;

struct PairHash {
    int64_t *keys; // kEmpty when free; null = no table
    int64_t *vals;
    u64 *verts;
    u64 *nbr;
    u64 *cob;          // rho's coboundary list: offset << 24 | length, kNoList when absent
    const int64_t *ckey; // the lists: cofacet index | (orientation bit << 62)
    const float *cdia;   // and cofacet diameter
    u32 mask;
};
constexpr u64 kNoList = ~0ull;
constexpr int64_t kCobIdx = (1ll << 62) - 1; // index bits of a list key

// Everything a slot holds for a key (val -1: not there).
struct PairHit {
    int64_t val;
    u64 verts, nbr, cob;
};

__device__ __forceinline__ PairHit pair_find_all(const PairHash &h, int64_t key) {
    u32 s = mix64((u64)key) & h.mask;
    PairHit r{-1, kNoVerts, 0, kNoList};
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        // the slot's words are loaded together: one round trip per probe
        const int64_t cur = h.keys[s];
        const int64_t v = h.vals[s];
        const u64 w = h.verts ? h.verts[s] : kNoVerts;
        const u64 nb = h.nbr ? h.nbr[s] : 0;
        const u64 cb = h.cob ? h.cob[s] : kNoList;
        if (cur == key) {
            r.val = v;
            r.verts = w;
            r.nbr = nb;
            r.cob = cb;
            return r;
        }
        if (cur == kEmpty) return r;
        s = (s + 1) & h.mask;
    }
    return r;
}

// The table is read-only while the reduction runs (the filter wrote it in an
// earlier kernel, or earlier in the same workgroup behind a barrier), so
// plain loads serve, and the value is loaded with the key.
__device__ __forceinline__ int64_t pair_find(const PairHash &h, int64_t key) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const int64_t cur = h.keys[s];
        const int64_t v = h.vals[s];
        if (cur == key) return v;
        if (cur == kEmpty) return -1;
        s = (s + 1) & h.mask;
    }
    return -1;
}

__device__ __forceinline__ bool pair_insert(const PairHash &h, int64_t key, int64_t val, u64 verts,
                                            u64 nbr) {
    u32 s = mix64((u64)key) & h.mask;
    for (u32 probe = 0; probe <= h.mask; ++probe) {
        const u64 prev = atomicCAS((u64 *)&h.keys[s], (u64)kEmpty, (u64)key);
        if (prev == (u64)kEmpty || prev == (u64)key) {
            h.vals[s] = val;
            if (h.verts) h.verts[s] = verts;
            if (h.nbr) h.nbr[s] = nbr;
            return true;
        }
        s = (s + 1) & h.mask;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Block-wide reductions of a (diameter, index) pivot candidate: the oldest
// entry of a coboundary column is the one of smallest diameter, then largest
// CNS index (refined order).
// ---------------------------------------------------------------------------
struct PivotCand {
    float diam;
    int64_t idx; // kEmpty = none
    u32 coef;
};

__device__ __forceinline__ bool older(const PivotCand &a, const PivotCand &b) {
    if (a.idx == kEmpty) return false;
    if (b.idx == kEmpty) return true;
    if (a.diam != b.diam) return a.diam < b.diam;
    return a.idx > b.idx;
}

// Wave reductions over DPP lane moves (no LDS round trips): row shifts by
// 1, 2, 4 and 8 leave each row's minimum (maximum) in its last lane, and the
// row broadcasts of lanes 15 and 31 carry those to lane 63. Lanes whose
// source lies outside the row get the identity. Every lane of the wave must
// be active; every lane gets the result.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ u32 dpp_min_step(u32 x) {
    const u32 y = (u32)__builtin_amdgcn_update_dpp(-1, (int)x, kCtrl, kRowMask, 0xf, false);
    return y < x ? y : x;
}

__device__ __forceinline__ u32 wave_min_u32(u32 x) {
    x = dpp_min_step<0x111, 0xf>(x); // row_shr:1
    x = dpp_min_step<0x112, 0xf>(x); // row_shr:2
    x = dpp_min_step<0x114, 0xf>(x); // row_shr:4
    x = dpp_min_step<0x118, 0xf>(x); // row_shr:8
    x = dpp_min_step<0x142, 0xa>(x); // row_bcast:15 into rows 1 and 3
    x = dpp_min_step<0x143, 0xc>(x); // row_bcast:31 into rows 2 and 3
    return (u32)__builtin_amdgcn_readlane((int)x, kWave - 1);
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ void dpp_max64_step(u32 &lo, u32 &hi) {
    const u32 ylo = (u32)__builtin_amdgcn_update_dpp(0, (int)lo, kCtrl, kRowMask, 0xf, false);
    const u32 yhi = (u32)__builtin_amdgcn_update_dpp(0, (int)hi, kCtrl, kRowMask, 0xf, false);
    if (((u64)yhi << 32 | ylo) > ((u64)hi << 32 | lo)) {
        lo = ylo;
        hi = yhi;
    }
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
    u32 lo = (u32)v, hi = (u32)(v >> 32);
    dpp_max64_step<0x111, 0xf>(lo, hi);
    dpp_max64_step<0x112, 0xf>(lo, hi);
    dpp_max64_step<0x114, 0xf>(lo, hi);
    dpp_max64_step<0x118, 0xf>(lo, hi);
    dpp_max64_step<0x142, 0xa>(lo, hi);
    dpp_max64_step<0x143, 0xc>(lo, hi);
    const u32 rlo = (u32)__builtin_amdgcn_readlane((int)lo, kWave - 1);
    const u32 rhi = (u32)__builtin_amdgcn_readlane((int)hi, kWave - 1);
    return (u64)rhi << 32 | rlo;
}

// Inclusive prefix sum over the wave with the same DPP moves.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_add_step(int x) {
    return x + __builtin_amdgcn_update_dpp(0, x, kCtrl, kRowMask, 0xf, false);
}

__device__ __forceinline__ int wave_scan_incl(int x) {
    x = dpp_add_step<0x111, 0xf>(x);
    x = dpp_add_step<0x112, 0xf>(x);
    x = dpp_add_step<0x114, 0xf>(x);
    x = dpp_add_step<0x118, 0xf>(x);
    x = dpp_add_step<0x142, 0xa>(x);
    x = dpp_add_step<0x143, 0xc>(x);
    return x;
}

// Lane l's value in every lane, through the scalar unit (v_readlane): for a
// source lane that is the same in the whole wave, in place of an LDS shuffle.
__device__ __forceinline__ int lane_bcast(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ u32 lane_bcast(u32 x, int l) { return (u32)__builtin_amdgcn_readlane((int)x, l); }
__device__ __forceinline__ float lane_bcast(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ u64 lane_bcast(u64 x, int l) {
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)x, l);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(x >> 32), l);
    return (u64)hi << 32 | lo;
}
__device__ __forceinline__ int64_t lane_bcast(int64_t x, int l) { return (int64_t)lane_bcast((u64)x, l); }

// The oldest candidate of the wave (smallest diameter, then largest index),
// in every lane. Diameters are >= +0, so their bit patterns order as the
// values do. All 64 lanes must be active.
__device__ __forceinline__ PivotCand wave_oldest(PivotCand x) {
    const u32 dk = x.idx == kEmpty ? 0xffffffffu : __float_as_uint(x.diam);
    const u32 mn = wave_min_u32(dk);
    PivotCand r;
    r.idx = kEmpty;
    r.diam = 0.0f;
    r.coef = 0;
    if (mn == 0xffffffffu) return r;
    const u64 key = dk == mn ? (u64)x.idx + 1ull : 0ull; // 0 = not of the smallest diameter
    const u64 mx = wave_max_u64(key);
    const u64 win = __ballot(key == mx);
    r.idx = (int64_t)(mx - 1ull);
    r.diam = __uint_as_float(mn);
    r.coef = (u32)__builtin_amdgcn_readlane((int)x.coef, __ffsll((unsigned long long)win) - 1);
    return r;
}

// ---------------------------------------------------------------------------
// Block-wide stable LSD radix sort (8-bit digits) of up to 2^31 records with
// 96-bit keys (hi: 32 bits, lo: 64 bits), ascending by (hi, lo), carrying a
// 32-bit payload. Runs in one workgroup of BT threads over global ping-pong
// buffers; histograms and per-wave digit counts live in LDS. Within a tile of
// BT records, ranks of equal digits come from 8 ballots per wave (a
// match-any on the digit), which keeps the scatter stable.
// ---------------------------------------------------------------------------
struct SortBufs {
    u64 *lo[2];
    u32 *hi[2];
    u32 *val[2];
};

template <int BT>
struct SortShared {
    u32 hist[256];
    u32 off[256];
    u32 wcnt[BT / kWave][256];
};

template <int BT>
__device__ __attribute__((noinline)) int block_radix_sort(SortBufs b, int N, int lo_bytes, int hi_bytes, SortShared<BT> &S) {
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int lane = lane_id();
    const u64 lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int cur = 0;
    for (int pass = 0; pass < lo_bytes + hi_bytes; ++pass) {
        const bool on_lo = pass < lo_bytes;
        const int sh = 8 * (on_lo ? pass : pass - lo_bytes);
        for (int d = tid; d < 256; d += BT) S.hist[d] = 0;
        gsync();
        for (int e = tid; e < N; e += BT) {
            const u32 dg = on_lo ? (u32)((b.lo[cur][e] >> sh) & 255) : ((b.hi[cur][e] >> sh) & 255);
            atomicAdd(&S.hist[dg], 1u);
        }
        __syncthreads();
        if (tid < kWave) {
            // exclusive scan of 256 bins by one wave, 4 bins per lane
            u32 v0 = S.hist[4 * lane], v1 = S.hist[4 * lane + 1], v2 = S.hist[4 * lane + 2],
                v3 = S.hist[4 * lane + 3];
            u32 sum = v0 + v1 + v2 + v3, inc = sum;
            for (int o = 1; o < kWave; o <<= 1) {
                u32 t = __shfl_up(inc, o, kWave);
                if (lane >= o) inc += t;
            }
            u32 ex = inc - sum;
            S.off[4 * lane] = ex;
            S.off[4 * lane + 1] = ex + v0;
            S.off[4 * lane + 2] = ex + v0 + v1;
            S.off[4 * lane + 3] = ex + v0 + v1 + v2;
        }
        __syncthreads();
        const int nxt = cur ^ 1;
        for (int base = 0; base < N; base += BT) {
            const int e = base + tid;
            const bool valid = e < N;
            u32 dg = 0;
            u64 klo = 0;
            u32 khi = 0, kv = 0;
            if (valid) {
                klo = b.lo[cur][e];
                khi = b.hi[cur][e];
                kv = b.val[cur][e];
                dg = on_lo ? (u32)((klo >> sh) & 255) : ((khi >> sh) & 255);
            }
            u64 same = __ballot(valid);
            for (int bit = 0; bit < 8; ++bit) {
                const u64 bb = __ballot(valid && ((dg >> bit) & 1));
                same &= ((dg >> bit) & 1) ? bb : ~bb;
            }
            for (int d = tid; d < (BT / kWave) * 256; d += BT) (&S.wcnt[0][0])[d] = 0;
            __syncthreads();
            const u32 rank_w = __popcll(same & lt);
            if (valid && rank_w == 0) S.wcnt[w][dg] = __popcll(same);
            __syncthreads();
            if (valid) {
                u32 r = rank_w;
                for (int ww = 0; ww < w; ++ww) r += S.wcnt[ww][dg];
                const u32 dst = S.off[dg] + r;
                if (dst < (u32)N) {
                    b.lo[nxt][dst] = klo;
                    b.hi[nxt][dst] = khi;
                    b.val[nxt][dst] = kv;
                }
            }
            __syncthreads();
            for (int d = tid; d < 256; d += BT) {
                u32 s = 0;
                for (int ww = 0; ww < BT / kWave; ++ww) s += S.wcnt[ww][d];
                S.off[d] += s;
            }
            __syncthreads();
        }
        gsync();
        cur = nxt;
    }
    gsync();
    return cur; // buffer index holding the sorted data
}

// Wave-aggregated append: lanes with pred get consecutive slots of *counter
// (one atomic per wave). Returns the slot or -1.
__device__ __forceinline__ int64_t wave_append(unsigned long long *counter, bool pred) {
    const u64 m = __ballot(pred);
    if (!m) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, kWave);
    const u64 lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    return pred ? (int64_t)(base + __popcll(m & lt)) : -1;
}

} // namespace rips
