// rips_api.hip -- host driver and C ABI (include/rips.h) of the single-cloud
// path. The host validates arguments, owns a per-device context whose
// buffers only grow (steady-state calls allocate nothing), queues the kernels
// of rips_kernels.hip on the caller's stream and reads back one small
// scalar block per stage to size the next one. No step of the method runs on
// the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rips.h"
#include "rips_kernels.hpp"

using namespace rips;

namespace {

thread_local std::string g_err;

rips_status fail(rips_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? RIPS_E_OOM : RIPS_E_HIP,                       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

enum BufId {
    B_INPUT,
    B_D,
    B_BINOM,
    B_INV,
    B_SCAL,
    B_E_IDX,
    B_E_DIAM,
    B_E_A,
    B_E_B,
    B_DEG,
    B_OFF,
    B_NBR,
    B_H0_COMP,
    B_H0_HOOK,
    B_H0_BEST,
    B_H0_MST,
    B_H0_MST2,
    B_H0_HI,
    B_H0_HI2,
    B_H0_VAL,
    B_H0_VAL2,
    B_H0_PARENT,
    B_H0_MAXV,
    B_H0_HDEATH,
    B_H0_HDSIMP,
    B_BITS,
    B_LIST_IDX,  // + k (k = 2..kMaxDim), two slots per k
    B_LIST_DIAM = B_LIST_IDX + kMaxDim + 1,
    B_SURV_IDX = B_LIST_DIAM + kMaxDim + 1,
    B_SURV_DIAM,
    B_SURV_J,
    B_SURV_TAPP,
    B_COL_IDX,   // + k
    B_COL_DIAM = B_COL_IDX + kMaxDim + 1,
    B_COL_J = B_COL_DIAM + kMaxDim + 1,
    B_COL_TAPP = B_COL_J + kMaxDim + 1,
    B_SORT_LO0 = B_COL_TAPP + kMaxDim + 1,
    B_SORT_LO1,
    B_SORT_HI0,
    B_SORT_HI1,
    B_SORT_V0,
    B_SORT_V1,
    B_PH_KEYS0,  // two pivot tables, alternating by dimension
    B_PH_KEYS1,
    B_PH_VALS0,
    B_PH_VALS1,
    B_V_OFF,
    B_V_LEN,
    B_V_PIV,
    B_V_IDX,
    B_V_COEF,
    B_WR_KEYS,
    B_WR_COEF,
    B_WR_DIAM,
    B_WV_KEYS,
    B_WV_COEF,
    B_WV_DIAM,
    B_BAR_BIRTH, // + d
    B_BAR_DEATH = B_BAR_BIRTH + kMaxDim + 1,
    B_BAR_BS = B_BAR_DEATH + kMaxDim + 1,
    B_BAR_DS = B_BAR_BS + kMaxDim + 1,
    B_STAGE = B_BAR_DS + kMaxDim + 1,
    B_NUM
};

struct DevCtx {
    std::mutex mu;
    void *buf[B_NUM] = {};
    size_t cap[B_NUM] = {};
    Scalars *host_scal = nullptr;
    int64_t hint_edges = 0;
    int64_t hint_list[kMaxDim + 2] = {};
    int64_t hint_v = 0;

    hipError_t ensure(int id, size_t bytes, void **out) {
        if (bytes == 0) bytes = 16;
        if (cap[id] < bytes) {
            if (buf[id]) {
                hipError_t e = hipFree(buf[id]);
                if (e != hipSuccess) return e;
                buf[id] = nullptr;
                cap[id] = 0;
            }
            size_t want = bytes + bytes / 4;
            hipError_t e = hipMalloc(&buf[id], want);
            if (e != hipSuccess) {
                buf[id] = nullptr;
                return e;
            }
            cap[id] = want;
        }
        *out = buf[id];
        return hipSuccess;
    }
};

std::mutex g_ctx_mu;
DevCtx *g_ctx[64];

rips_status get_ctx(DevCtx **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(RIPS_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (!g_ctx[dev]) {
        DevCtx *c = new DevCtx();
        HIP_TRY(hipHostMalloc((void **)&c->host_scal, sizeof(Scalars), hipHostMallocDefault));
        g_ctx[dev] = c;
    }
    *out = g_ctx[dev];
    return RIPS_OK;
}

bool is_prime_u32(uint32_t p) {
    if (p < 2) return false;
    for (uint32_t q = 2; (uint64_t)q * q <= p; ++q)
        if (p % q == 0) return false;
    return true;
}

// C(n, k) as long double (overflow test only)
long double choose_ld(int64_t n, int k) {
    if (k < 0 || n < k) return 0.0L;
    long double r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (long double)(n - k + i) / (long double)i;
    return r;
}

int64_t choose_i64(int64_t n, int k) {
    if (k < 0 || n < k) return 0;
    __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int64_t)r;
}

rips_status validate(int64_t n, int32_t dim, int32_t max_dim, float threshold, uint32_t p,
                     int top_extra) {
    if (n < 1 || n > RIPS_MAX_POINTS)
        return fail(RIPS_E_INVALID_ARG, "n must be in [1, " + std::to_string(RIPS_MAX_POINTS) + "]");
    if (dim < 0) return fail(RIPS_E_INVALID_ARG, "dim must be >= 0");
    if (max_dim < 0 || max_dim > RIPS_MAX_DIM + top_extra)
        return fail(RIPS_E_INVALID_ARG, "max_dim out of range");
    if (std::isnan(threshold)) return fail(RIPS_E_INVALID_ARG, "threshold is NaN");
    if (!is_prime_u32(p) || p >= 65536)
        return fail(RIPS_E_NOT_PRIME, "p must be a prime in [2, 65536)");
    if (choose_ld(n, max_dim + 2) >= 9.2e18L)
        return fail(RIPS_E_INDEX_OVERFLOW, "C(n, max_dim + 2) does not fit in int64");
    return RIPS_OK;
}

uint32_t next_pow2(uint64_t x) {
    uint64_t r = 1;
    while (r < x) r <<= 1;
    return (uint32_t)r;
}

int bytes_for(uint64_t maxval) {
    int b = 1;
    while (b < 8 && (maxval >> (8 * b)) != 0) ++b;
    return b;
}

template <class T>
T *as(void *p) {
    return static_cast<T *>(p);
}

struct RunOut {
    int n, max_dim;
    float t_eff, r_enc;
    int sparse;
    int64_t count[kMaxDim + 1];
    int64_t ncols[kMaxDim + 1];
    int64_t simplex_count[kMaxDim + 2];
    rips_dim_stats stats[kMaxDim + 1];
};

rips_status read_scalars(DevCtx &C, Scalars *d_scal, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(C.host_scal, d_scal, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RIPS_OK;
}

__global__ void k_set_counter(unsigned long long *p, unsigned long long v) { *p = v; }

__global__ void k_maxdeg(const int *deg, int n, int *out) {
    int m = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = max(m, deg[i]);
    atomicMax(out, m);
}

struct Prepared {
    float *D;
    u64 *B;
    u32 *inv;
    Scalars *scal;
    EdgeList E;
    int64_t nedges;
    int *deg, *off, *nbr;
    int maxdeg;
    int sparse;
    Ctx<DistFull> ctx;
};

// distances, threshold, edges (and neighbour lists): everything up to H0
rips_status prepare(DevCtx &C, const float *d_in, int n, int m, int jmax, float t, uint32_t p,
                    hipStream_t st, Prepared &P) {
    void *q;
    const int stride = n + 1;
    HIP_TRY(C.ensure(B_BINOM, (size_t)(jmax + 1) * stride * 8, &q));
    P.B = as<u64>(q);
    launch_binom(P.B, stride, n, jmax, st);
    HIP_TRY(C.ensure(B_INV, (size_t)p * 4, &q));
    P.inv = as<u32>(q);
    launch_inverse(P.inv, p, st);
    HIP_TRY(C.ensure(B_D, (size_t)n * n * 4, &q));
    P.D = as<float>(q);
    HIP_TRY(C.ensure(B_SCAL, sizeof(Scalars), &q));
    P.scal = as<Scalars>(q);
    launch_init_scalars(P.scal, st);
    launch_dist(d_in, n, m, P.D, &P.scal->bad, st);
    launch_threshold(P.D, n, t, P.scal, st);
    const int64_t all_edges = (int64_t)n * (n - 1) / 2;
    int64_t cap = C.hint_edges > 0 ? C.hint_edges : std::min<int64_t>(all_edges, 1 << 16);
    if (cap > all_edges) cap = all_edges;
    HIP_TRY(C.ensure(B_DEG, (size_t)(n + 1) * 4, &q));
    P.deg = as<int>(q);
    for (int attempt = 0; attempt < 3; ++attempt) {
        HIP_TRY(C.ensure(B_E_IDX, (size_t)cap * 8, &q));
        P.E.idx = as<int64_t>(q);
        HIP_TRY(C.ensure(B_E_DIAM, (size_t)cap * 4, &q));
        P.E.diam = as<float>(q);
        HIP_TRY(C.ensure(B_E_A, (size_t)cap * 4, &q));
        P.E.a = as<int>(q);
        HIP_TRY(C.ensure(B_E_B, (size_t)cap * 4, &q));
        P.E.b = as<int>(q);
        hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->edges, 0ull);
        launch_edges(P.D, n, P.scal, P.E, cap, P.deg, st);
        hipLaunchKernelGGL(k_maxdeg, dim3(1), dim3(256), 0, st, P.deg, n, &P.scal->maxdeg);
        rips_status rs = read_scalars(C, P.scal, st);
        if (rs) return rs;
        if (C.host_scal->bad)
            return fail(RIPS_E_NONFINITE, "input holds NaN/Inf or a negative distance");
        if ((int64_t)C.host_scal->edges <= cap) break;
        cap = (int64_t)C.host_scal->edges;
    }
    P.nedges = (int64_t)C.host_scal->edges;
    if (P.nedges > C.hint_edges) C.hint_edges = P.nedges;
    P.maxdeg = C.host_scal->maxdeg;
    // neighbour lists pay off once the complex is sparse
    P.sparse = n > 64 && P.nedges * 10 < all_edges * 3;
    P.off = P.nbr = nullptr;
    if (P.sparse) {
        HIP_TRY(C.ensure(B_OFF, (size_t)(n + 1) * 4, &q));
        P.off = as<int>(q);
        HIP_TRY(C.ensure(B_NBR, (size_t)(2 * P.nedges + 1) * 4, &q));
        P.nbr = as<int>(q);
        launch_csr(P.D, n, P.scal, P.deg, P.off, P.nbr, st);
    }
    P.ctx.d.D = P.D;
    P.ctx.d.n = n;
    P.ctx.B.t = P.B;
    P.ctx.B.stride = stride;
    P.ctx.nb.off = P.off;
    P.ctx.nb.idx = P.nbr;
    P.ctx.n = n;
    P.ctx.t = C.host_scal->t_eff;
    return RIPS_OK;
}

int group_size_for(const Prepared &P) {
    // lanes per candidate: about the expected early-exit scan length
    const char *env = getenv("RIPS_GROUP");
    if (env) {
        int g = atoi(env);
        if (g == 4 || g == 8 || g == 16 || g == 32 || g == 64) return g;
    }
    if (P.sparse) return 16;
    return P.ctx.n <= 128 ? 16 : 32;
}

rips_status run_single(DevCtx &C, const float *d_in, int n, int m, int max_dim, float t, uint32_t p,
                       hipStream_t st, RunOut &o) {
    memset(&o, 0, sizeof(o));
    o.n = n;
    o.max_dim = max_dim;
    Prepared P;
    rips_status rs = prepare(C, d_in, n, m, max_dim + 2, t, p, st, P);
    if (rs) return rs;
    o.t_eff = C.host_scal->t_eff;
    o.r_enc = C.host_scal->r_enc;
    o.sparse = P.sparse;
    o.simplex_count[0] = n;
    if (max_dim + 1 >= 1) o.simplex_count[1] = P.nedges;
    void *q;
    // ---- H0
    H0Scratch W;
    HIP_TRY(C.ensure(B_H0_COMP, (size_t)n * 4, &q));
    W.comp = as<int>(q);
    HIP_TRY(C.ensure(B_H0_HOOK, (size_t)n * 4, &q));
    W.hook = as<int>(q);
    HIP_TRY(C.ensure(B_H0_BEST, (size_t)n * 8, &q));
    W.best = as<u64>(q);
    HIP_TRY(C.ensure(B_H0_MST, (size_t)n * 8, &q));
    W.mst = as<u64>(q);
    HIP_TRY(C.ensure(B_H0_MST2, (size_t)n * 8, &q));
    W.mst2 = as<u64>(q);
    HIP_TRY(C.ensure(B_H0_HI, (size_t)n * 4, &q));
    W.hi = as<u32>(q);
    HIP_TRY(C.ensure(B_H0_HI2, (size_t)n * 4, &q));
    W.hi2 = as<u32>(q);
    HIP_TRY(C.ensure(B_H0_VAL, (size_t)n * 4, &q));
    W.val = as<u32>(q);
    HIP_TRY(C.ensure(B_H0_VAL2, (size_t)n * 4, &q));
    W.val2 = as<u32>(q);
    HIP_TRY(C.ensure(B_H0_PARENT, (size_t)n * 4, &q));
    W.parent = as<int>(q);
    HIP_TRY(C.ensure(B_H0_MAXV, (size_t)n * 4, &q));
    W.maxv = as<int>(q);
    HIP_TRY(C.ensure(B_H0_HDEATH, (size_t)n * 4, &q));
    W.hdeath = as<float>(q);
    HIP_TRY(C.ensure(B_H0_HDSIMP, (size_t)n * 8, &q));
    W.hdsimp = as<int64_t>(q);
    const int64_t nwords = ((int64_t)n * (n - 1) / 2) / 32 + 1;
    HIP_TRY(C.ensure(B_BITS, (size_t)nwords * 4, &q));
    W.bits = as<u32>(q);
    BarBuf bars[kMaxDim + 1];
    auto ensure_bars = [&](int d, int64_t cap) -> rips_status {
        HIP_TRY(C.ensure(B_BAR_BIRTH + d, (size_t)cap * 4, &q));
        bars[d].birth = as<float>(q);
        HIP_TRY(C.ensure(B_BAR_DEATH + d, (size_t)cap * 4, &q));
        bars[d].death = as<float>(q);
        HIP_TRY(C.ensure(B_BAR_BS + d, (size_t)cap * 8, &q));
        bars[d].bs = as<int64_t>(q);
        HIP_TRY(C.ensure(B_BAR_DS + d, (size_t)cap * 8, &q));
        bars[d].ds = as<int64_t>(q);
        return RIPS_OK;
    };
    if ((rs = ensure_bars(0, n))) return rs;
    launch_reset_dim(P.scal, st);
    launch_h0(P.E, P.scal, n, W, bars[0], nwords, st);
    if ((rs = read_scalars(C, P.scal, st))) return rs;
    if (getenv("RIPS_DEBUG") && n <= 64) {
        // diagnostics: H0 internals of small inputs
        const int m = (int)C.host_scal->mst;
        std::vector<unsigned long long> k0(n), k1(n);
        std::vector<int> par(n), mx(n);
        std::vector<float> hd(n);
        (void)hipMemcpy(k0.data(), W.mst, 8 * n, hipMemcpyDeviceToHost);
        (void)hipMemcpy(k1.data(), W.mst2, 8 * n, hipMemcpyDeviceToHost);
        (void)hipMemcpy(par.data(), W.parent, 4 * n, hipMemcpyDeviceToHost);
        (void)hipMemcpy(mx.data(), W.maxv, 4 * n, hipMemcpyDeviceToHost);
        (void)hipMemcpy(hd.data(), W.hdeath, 4 * n, hipMemcpyDeviceToHost);
        fprintf(stderr, "[rips h0] n=%d edges=%lld forest=%d nbars=%lld\n", n,
                (long long)P.nedges, m, (long long)C.host_scal->nbars);
        for (int i = 0; i < m; ++i)
            fprintf(stderr, "[rips h0] key[%d] %016llx / %016llx\n", i, k0[i], k1[i]);
        for (int v = 0; v < n; ++v)
            fprintf(stderr, "[rips h0] v=%d parent=%d maxv=%d hdeath=%g\n", v, par[v], mx[v], hd[v]);
    }
    o.count[0] = C.host_scal->nbars;
    o.ncols[0] = n;
    o.stats[0].candidates = n;
    o.stats[0].columns = n;
    o.stats[0].bars_nonzero = (int64_t)C.host_scal->stat[kStatBarsNonzero];
    o.stats[0].essential = (int64_t)C.host_scal->stat[kStatEssential];
    o.stats[0].emergent = 0;

    const int G = group_size_for(P);
    SimplexList prev_list{P.E.idx, P.E.diam};
    int64_t prev_count = P.nedges;
    PivotHash ph_prev{nullptr, nullptr, 0};
    for (int k = 1; k <= max_dim; ++k) {
        launch_reset_dim(P.scal, st);
        SimplexList cand;
        int64_t ncand;
        if (k == 1) {
            cand = prev_list;
            ncand = prev_count;
        } else {
            int64_t cap = C.hint_list[k] > 0 ? C.hint_list[k] : std::max<int64_t>(prev_count * 4, 1024);
            for (int attempt = 0; attempt < 3; ++attempt) {
                HIP_TRY(C.ensure(B_LIST_IDX + k, (size_t)cap * 8, &q));
                cand.idx = as<int64_t>(q);
                HIP_TRY(C.ensure(B_LIST_DIAM + k, (size_t)cap * 4, &q));
                cand.diam = as<float>(q);
                hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->list, 0ull);
                launch_expand(G, P.ctx, k, prev_list, prev_count, P.scal, cand, cap, false, st);
                if ((rs = read_scalars(C, P.scal, st))) return rs;
                if ((int64_t)C.host_scal->list <= cap) break;
                cap = (int64_t)C.host_scal->list;
            }
            ncand = (int64_t)C.host_scal->list;
            if (ncand > C.hint_list[k]) C.hint_list[k] = ncand;
        }
        o.simplex_count[k] = ncand;
        // ---- enumeration / apparent-pair pass
        Columns surv, cols;
        HIP_TRY(C.ensure(B_SURV_IDX, (size_t)ncand * 8, &q));
        surv.idx = as<int64_t>(q);
        HIP_TRY(C.ensure(B_SURV_DIAM, (size_t)ncand * 4, &q));
        surv.diam = as<float>(q);
        HIP_TRY(C.ensure(B_SURV_J, (size_t)ncand * 4, &q));
        surv.j = as<int>(q);
        HIP_TRY(C.ensure(B_SURV_TAPP, (size_t)ncand, &q));
        surv.tapp = as<uint8_t>(q);
        launch_filter(G, P.ctx, k, cand, ncand, W.bits, ph_prev, P.scal, surv, st);
        if ((rs = read_scalars(C, P.scal, st))) return rs;
        const int64_t S = std::min<int64_t>((int64_t)C.host_scal->survivors, ncand);
        if (S > 0x7fffffff) return fail(RIPS_E_CAPACITY, "too many columns");
        o.ncols[k] = S;
        o.stats[k].candidates = ncand;
        o.stats[k].cleared = (int64_t)C.host_scal->stat[kStatCleared];
        o.stats[k].apparent_col = (int64_t)C.host_scal->stat[kStatAppCol];
        o.stats[k].apparent_pivot = (int64_t)C.host_scal->stat[kStatAppPiv];
        o.stats[k].columns = S;
        // ---- sort
        HIP_TRY(C.ensure(B_COL_IDX + k, (size_t)S * 8, &q));
        cols.idx = as<int64_t>(q);
        HIP_TRY(C.ensure(B_COL_DIAM + k, (size_t)S * 4, &q));
        cols.diam = as<float>(q);
        HIP_TRY(C.ensure(B_COL_J + k, (size_t)S * 4, &q));
        cols.j = as<int>(q);
        HIP_TRY(C.ensure(B_COL_TAPP + k, (size_t)S, &q));
        cols.tapp = as<uint8_t>(q);
        SortBufs sb;
        HIP_TRY(C.ensure(B_SORT_LO0, (size_t)S * 8, &q));
        sb.lo[0] = as<u64>(q);
        HIP_TRY(C.ensure(B_SORT_LO1, (size_t)S * 8, &q));
        sb.lo[1] = as<u64>(q);
        HIP_TRY(C.ensure(B_SORT_HI0, (size_t)S * 4, &q));
        sb.hi[0] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_HI1, (size_t)S * 4, &q));
        sb.hi[1] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_V0, (size_t)S * 4, &q));
        sb.val[0] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_V1, (size_t)S * 4, &q));
        sb.val[1] = as<u32>(q);
        const int lo_bytes = bytes_for((uint64_t)choose_i64(n, k + 1));
        launch_sort_columns(surv, P.scal, sb, lo_bytes, cols, st);
        // ---- reduction
        const int slot = k & 1;
        PivotHash ph;
        const uint32_t phcap = next_pow2((uint64_t)2 * S + 64);
        HIP_TRY(C.ensure(B_PH_KEYS0 + slot, (size_t)phcap * 8, &q));
        ph.keys = as<int64_t>(q);
        HIP_TRY(C.ensure(B_PH_VALS0 + slot, (size_t)phcap * 4, &q));
        ph.vals = as<int32_t>(q);
        ph.mask = phcap - 1;
        VStore V;
        HIP_TRY(C.ensure(B_V_OFF, (size_t)S * 8, &q));
        V.off = as<int64_t>(q);
        HIP_TRY(C.ensure(B_V_LEN, (size_t)S * 4, &q));
        V.len = as<int>(q);
        HIP_TRY(C.ensure(B_V_PIV, (size_t)S * 4, &q));
        V.pivcoef = as<u32>(q);
        int64_t vcap = std::max<int64_t>(C.hint_v, 4 * S + 4096);
        if ((rs = ensure_bars(k, S))) return rs;
        const int bound = P.sparse ? P.maxdeg : n;
        uint32_t capR = next_pow2(std::max<uint64_t>(256, 4ull * (uint64_t)bound));
        uint32_t capV = 1024;
        int use_lds = reduce_lds_bytes(capR, capV) <= 150 * 1024;
        for (int attempt = 0;; ++attempt) {
            if (attempt > 8) return fail(RIPS_E_CAPACITY, "reduction scratch kept overflowing");
            HIP_TRY(C.ensure(B_V_IDX, (size_t)vcap * 8, &q));
            V.idx = as<int64_t>(q);
            HIP_TRY(C.ensure(B_V_COEF, (size_t)vcap * 4, &q));
            V.coef = as<u32>(q);
            V.cap = vcap;
            WorkHash Rg{nullptr, nullptr, nullptr, capR - 1}, Vg{nullptr, nullptr, nullptr, capV - 1};
            if (!use_lds) {
                HIP_TRY(C.ensure(B_WR_KEYS, (size_t)capR * 8, &q));
                Rg.keys = as<int64_t>(q);
                HIP_TRY(C.ensure(B_WR_COEF, (size_t)capR * 4, &q));
                Rg.coef = as<u32>(q);
                HIP_TRY(C.ensure(B_WR_DIAM, (size_t)capR * 4, &q));
                Rg.diam = as<float>(q);
                HIP_TRY(C.ensure(B_WV_KEYS, (size_t)capV * 8, &q));
                Vg.keys = as<int64_t>(q);
                HIP_TRY(C.ensure(B_WV_COEF, (size_t)capV * 4, &q));
                Vg.coef = as<u32>(q);
                HIP_TRY(C.ensure(B_WV_DIAM, (size_t)capV * 4, &q));
                Vg.diam = as<float>(q);
            }
            launch_fill_i64(ph.keys, phcap, kEmpty, st);
            launch_reset_dim(P.scal, st);
            launch_reduce(P.ctx, k, p, P.inv, cols, (int)S, ph, V, Rg, Vg, use_lds, capR, capV,
                          P.scal, bars[k], st);
            HIP_TRY(hipGetLastError());
            if ((rs = read_scalars(C, P.scal, st))) return rs;
            const int status = C.host_scal->status;
            if (status == 0) break;
            if (status == 1) {
                use_lds = 0;
                capR = capR < (1u << 26) ? capR * 8 : capR;
                capV = capV < (1u << 24) ? capV * 8 : capV;
            } else if (status == 2) {
                vcap *= 4;
            } else {
                return fail(RIPS_E_HIP, "reduction exceeded its addition bound");
            }
        }
        if ((int64_t)C.host_scal->vcount > C.hint_v) C.hint_v = (int64_t)C.host_scal->vcount;
        o.count[k] = C.host_scal->nbars;
        o.stats[k].emergent = (int64_t)C.host_scal->stat[kStatEmergent];
        o.stats[k].reduced = (int64_t)C.host_scal->stat[kStatReduced];
        o.stats[k].additions = (int64_t)C.host_scal->stat[kStatAdditions];
        o.stats[k].bars_nonzero = (int64_t)C.host_scal->stat[kStatBarsNonzero];
        o.stats[k].essential = (int64_t)C.host_scal->stat[kStatEssential];
        ph_prev = ph;
        prev_list = cand;
        prev_count = ncand;
    }
    return RIPS_OK;
}

BarBuf internal_bars(DevCtx &C, int d) {
    BarBuf b;
    b.birth = as<float>(C.buf[B_BAR_BIRTH + d]);
    b.death = as<float>(C.buf[B_BAR_DEATH + d]);
    b.bs = as<int64_t>(C.buf[B_BAR_BS + d]);
    b.ds = as<int64_t>(C.buf[B_BAR_DS + d]);
    return b;
}

// set the device "nbars" scalar before an emit
__global__ void k_set_nbars(Scalars *s, int64_t v) { s->nbars = v; }

} // namespace

extern "C" {

const char *rips_status_string(rips_status s) {
    switch (s) {
    case RIPS_OK: return "ok";
    case RIPS_E_INVALID_ARG: return "invalid argument";
    case RIPS_E_NOT_PRIME: return "p is not a prime in [2, 65536)";
    case RIPS_E_INDEX_OVERFLOW: return "simplex index overflow";
    case RIPS_E_NONFINITE: return "non-finite or negative input";
    case RIPS_E_OOM: return "out of memory";
    case RIPS_E_CAPACITY: return "output capacity too small";
    case RIPS_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *rips_last_error(void) { return g_err.c_str(); }

rips_status rips_barcode_device(const float *d_data, int64_t n, int32_t dim, int32_t max_dim,
                                float threshold, uint32_t p, rips_device_out *out,
                                void *hip_stream) {
    g_err.clear();
    if (!d_data || !out) return fail(RIPS_E_INVALID_ARG, "null pointer");
    rips_status rs = validate(n, dim, max_dim, threshold, p, 0);
    if (rs) return rs;
    DevCtx *C;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    RunOut o;
    rs = run_single(*C, d_data, (int)n, dim, max_dim, threshold, p, st, o);
    if (rs) return rs;
    int64_t need = 0;
    for (int d = 0; d <= max_dim; ++d) need = std::max(need, o.count[d]);
    out->needed_cap = need;
    for (int d = 0; d <= max_dim; ++d) {
        out->count[d] = o.count[d];
        out->stats[d] = o.stats[d];
        out->simplex_count[d] = o.simplex_count[d];
    }
    out->threshold_used = o.t_eff;
    out->sparse = o.sparse;
    if (need > out->cap) return fail(RIPS_E_CAPACITY, "bar capacity too small");
    if (!out->birth || !out->death || !out->birth_simplex || !out->death_simplex)
        return fail(RIPS_E_INVALID_ARG, "null output buffer");
    Scalars *scal = as<Scalars>(C->buf[B_SCAL]);
    for (int d = 0; d <= max_dim; ++d) {
        BarBuf dst{out->birth + d * out->cap, out->death + d * out->cap,
                   out->birth_simplex + d * out->cap, out->death_simplex + d * out->cap};
        hipLaunchKernelGGL(k_set_nbars, dim3(1), dim3(1), 0, st, scal, o.count[d]);
        launch_emit(internal_bars(*C, d), scal, d > 0 ? 1 : 0, dst, st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return RIPS_OK;
}

rips_status rips_barcode(const float *data, int64_t n, int32_t dim, int32_t max_dim,
                         float threshold, uint32_t p, rips_result **out) {
    g_err.clear();
    if (!out) return fail(RIPS_E_INVALID_ARG, "null out");
    *out = nullptr;
    if (!data) return fail(RIPS_E_INVALID_ARG, "null data");
    rips_status rs = validate(n, dim, max_dim, threshold, p, 0);
    if (rs) return rs;
    DevCtx *C;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    hipStream_t st = nullptr;
    void *q;
    const size_t in_elems = dim > 0 ? (size_t)n * dim : (size_t)n * n;
    HIP_TRY(C->ensure(B_INPUT, in_elems * 4, &q));
    float *d_in = as<float>(q);
    HIP_TRY(hipMemcpyAsync(d_in, data, in_elems * 4, hipMemcpyHostToDevice, st));
    RunOut o;
    rs = run_single(*C, d_in, (int)n, dim, max_dim, threshold, p, st, o);
    if (rs) return rs;
    rips_result *r = (rips_result *)calloc(1, sizeof(rips_result));
    if (!r) return fail(RIPS_E_OOM, "host allocation");
    r->n = (int32_t)n;
    r->max_dim = max_dim;
    r->p = p;
    r->sparse = o.sparse;
    r->threshold_used = o.t_eff;
    r->enclosing_radius = o.r_enc;
    const int nd = max_dim + 1;
    r->dims = (rips_bars *)calloc(nd, sizeof(rips_bars));
    r->stats = (rips_dim_stats *)calloc(nd, sizeof(rips_dim_stats));
    r->simplex_count = (int64_t *)calloc(nd, sizeof(int64_t));
    r->column_count = (int64_t *)calloc(nd, sizeof(int64_t));
    r->column_index = (int64_t **)calloc(nd, sizeof(int64_t *));
    r->column_diam = (float **)calloc(nd, sizeof(float *));
    if (!r->dims || !r->stats || !r->simplex_count || !r->column_count || !r->column_index ||
        !r->column_diam) {
        rips_result_free(r);
        return fail(RIPS_E_OOM, "host allocation");
    }
    Scalars *scal = as<Scalars>(C->buf[B_SCAL]);
    for (int d = 0; d < nd; ++d) {
        const int64_t c = o.count[d];
        r->stats[d] = o.stats[d];
        r->simplex_count[d] = o.simplex_count[d];
        rips_bars &b = r->dims[d];
        b.count = c;
        b.birth = (float *)malloc(sizeof(float) * (c ? c : 1));
        b.death = (float *)malloc(sizeof(float) * (c ? c : 1));
        b.birth_simplex = (int64_t *)malloc(sizeof(int64_t) * (c ? c : 1));
        b.death_simplex = (int64_t *)malloc(sizeof(int64_t) * (c ? c : 1));
        const int64_t nc = d == 0 ? 0 : o.ncols[d];
        r->column_count[d] = nc;
        r->column_index[d] = (int64_t *)malloc(sizeof(int64_t) * (nc ? nc : 1));
        r->column_diam[d] = (float *)malloc(sizeof(float) * (nc ? nc : 1));
        if (!b.birth || !b.death || !b.birth_simplex || !b.death_simplex ||
            !r->column_index[d] || !r->column_diam[d]) {
            rips_result_free(r);
            return fail(RIPS_E_OOM, "host allocation");
        }
        if (c > 0) {
            if (C->ensure(B_STAGE, (size_t)c * 24, &q) != hipSuccess) {
                rips_result_free(r);
                return fail(RIPS_E_OOM, "staging buffer");
            }
            char *sg = as<char>(q);
            BarBuf dst{(float *)sg, (float *)(sg + c * 4), (int64_t *)(sg + c * 8),
                       (int64_t *)(sg + c * 16)};
            hipLaunchKernelGGL(k_set_nbars, dim3(1), dim3(1), 0, st, scal, c);
            launch_emit(internal_bars(*C, d), scal, d > 0 ? 1 : 0, dst, st);
            hipError_t e1 = hipMemcpyAsync(b.birth, dst.birth, c * 4, hipMemcpyDeviceToHost, st);
            hipError_t e2 = hipMemcpyAsync(b.death, dst.death, c * 4, hipMemcpyDeviceToHost, st);
            hipError_t e3 = hipMemcpyAsync(b.birth_simplex, dst.bs, c * 8, hipMemcpyDeviceToHost, st);
            hipError_t e4 = hipMemcpyAsync(b.death_simplex, dst.ds, c * 8, hipMemcpyDeviceToHost, st);
            hipError_t e5 = hipStreamSynchronize(st);
            if (e1 || e2 || e3 || e4 || e5) {
                rips_result_free(r);
                return fail(RIPS_E_HIP, "copying bars to the host");
            }
        }
        if (nc > 0) {
            hipError_t e1 = hipMemcpyAsync(r->column_index[d], C->buf[B_COL_IDX + d], nc * 8,
                                           hipMemcpyDeviceToHost, st);
            hipError_t e2 = hipMemcpyAsync(r->column_diam[d], C->buf[B_COL_DIAM + d], nc * 4,
                                           hipMemcpyDeviceToHost, st);
            hipError_t e3 = hipStreamSynchronize(st);
            if (e1 || e2 || e3) {
                rips_result_free(r);
                return fail(RIPS_E_HIP, "copying columns to the host");
            }
        }
    }
    *out = r;
    return RIPS_OK;
}

void rips_result_free(rips_result *r) {
    if (!r) return;
    const int nd = r->max_dim + 1;
    if (r->dims)
        for (int d = 0; d < nd; ++d) {
            free(r->dims[d].birth);
            free(r->dims[d].death);
            free(r->dims[d].birth_simplex);
            free(r->dims[d].death_simplex);
        }
    if (r->column_index)
        for (int d = 0; d < nd; ++d) free(r->column_index[d]);
    if (r->column_diam)
        for (int d = 0; d < nd; ++d) free(r->column_diam[d]);
    free(r->dims);
    free(r->stats);
    free(r->simplex_count);
    free(r->column_count);
    free(r->column_index);
    free(r->column_diam);
    free(r);
}

rips_status rips_simplex_counts_device(const float *d_data, int64_t n, int32_t dim, int32_t top,
                                       float threshold, int64_t *counts, void *hip_stream) {
    g_err.clear();
    if (!d_data || !counts) return fail(RIPS_E_INVALID_ARG, "null pointer");
    rips_status rs = validate(n, dim, top - 1 < 0 ? 0 : top - 1, threshold, 2, 0);
    if (rs) return rs;
    if (top < 0 || top > RIPS_MAX_DIM + 1) return fail(RIPS_E_INVALID_ARG, "top out of range");
    DevCtx *C;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    Prepared P;
    rs = prepare(*C, d_data, (int)n, dim, std::max(top + 1, 2), threshold, 2, st, P);
    if (rs) return rs;
    counts[0] = n;
    if (top >= 1) counts[1] = P.nedges;
    SimplexList prev{P.E.idx, P.E.diam};
    int64_t prev_count = P.nedges;
    void *q;
    for (int k = 2; k <= top; ++k) {
        const bool last = k == top;
        SimplexList cur{nullptr, nullptr};
        int64_t cap = 0;
        if (!last) {
            cap = C->hint_list[k] > 0 ? C->hint_list[k] : std::max<int64_t>(prev_count * 4, 1024);
        }
        for (int attempt = 0; attempt < 3; ++attempt) {
            if (!last) {
                HIP_TRY(C->ensure(B_LIST_IDX + k, (size_t)cap * 8, &q));
                cur.idx = as<int64_t>(q);
                HIP_TRY(C->ensure(B_LIST_DIAM + k, (size_t)cap * 4, &q));
                cur.diam = as<float>(q);
            }
            hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->list, 0ull);
            launch_expand(16, P.ctx, k, prev, prev_count, P.scal, cur, cap, last, st);
            if ((rs = read_scalars(*C, P.scal, st))) return rs;
            if (last || (int64_t)C->host_scal->list <= cap) break;
            cap = (int64_t)C->host_scal->list;
        }
        counts[k] = (int64_t)C->host_scal->list;
        if (!last && counts[k] > C->hint_list[k]) C->hint_list[k] = counts[k];
        prev = cur;
        prev_count = counts[k];
    }
    return RIPS_OK;
}

} // extern "C"
