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
#include <unordered_map>

#include "../../include/rips.h"
#include "rips_batched.hpp"

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
    B_BW_BINOM, // binomial table of the backward entry
    B_APP_KEYS, // zero apparent pairs of the current dimension
    B_APP_VALS,
    B_APP_VERTS, // rho's vertices, per slot
    B_APP_NBR,   // rho's shortest neighbour list, per slot
    B_APP_COB,   // rho's coboundary list, per slot
    B_COB_KEY,   // the coboundary lists
    B_COB_DIA,
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
    B_V_DIAM,
    B_F_IDX0, // far list of the working column, two buffers
    B_F_IDX1,
    B_F_DIA0,
    B_F_DIA1,
    B_F_COEF0,
    B_F_COEF1,
    B_VW_KEYS, // working V column
    B_VW_COEF,
    B_VW_DIAM,
    B_VW_SLOTS,
    B_V_ROFF,
    B_V_RLEN,
    B_LOG_KEY, // addition log of the column being reduced
    B_LOG_COEF,
    B_LOG_DIA,
    B_CBAR_BIRTH, // per-column bar slots of the spread-out reduction
    B_CBAR_DEATH,
    B_CBAR_BS,
    B_CBAR_DS,
    B_CST,        // per-column state of the spread-out reduction
    B_CTL,        // its cursor, frontier and abort flag
    B_BAR_BIRTH, // + d
    B_BAR_DEATH = B_BAR_BIRTH + kMaxDim + 1,
    B_BAR_BS = B_BAR_DEATH + kMaxDim + 1,
    B_BAR_DS = B_BAR_BS + kMaxDim + 1,
    B_STAGE = B_BAR_DS + kMaxDim + 1,
    // batched path
    BB_DG,
    BB_C_IDX0,
    BB_C_IDX1,
    BB_C_DM0,
    BB_C_DM1,
    BB_C_J0,
    BB_C_J1,
    BB_C_T0,
    BB_C_T1,
    BB_S_LO0,
    BB_S_LO1,
    BB_S_HI0,
    BB_S_HI1,
    BB_S_V0,
    BB_S_V1,
    BB_PH_KEYS,
    BB_PH_VALS,
    BB_APP_KEYS,
    BB_APP_VALS,
    BB_APP_VERTS,
    BB_V_OFF,
    BB_V_LEN,
    BB_V_PIV,
    BB_V_IDX,
    BB_V_DIAM,
    BB_V_COEF,
    BB_V_COUNT,
    BB_BITS,
    BB_F_IDX0,
    BB_F_IDX1,
    BB_F_DIA0,
    BB_F_DIA1,
    BB_F_COEF0,
    BB_F_COEF1,
    BB_VW_KEYS,
    BB_VW_COEF,
    BB_VW_DIAM,
    BB_VW_SLOTS,
    BB_V_ROFF,
    BB_V_RLEN,
    BB_LOG_KEY,
    BB_LOG_COEF,
    BB_LOG_DIA,
    BB_ST_B,
    BB_ST_D,
    BB_ST_BS,
    BB_ST_DS,
    BB_UB,
    BB_UD,
    BB_UBS,
    BB_UDS,
    BB_SEG_START,
    BB_SEG_COUNT,
    BB_STATS,
    BB_TUSED,
    BB_LPT_LO0,
    BB_LPT_LO1,
    BB_LPT_HI0,
    BB_LPT_HI1,
    BB_LPT_V0,
    BB_LPT_V1,
    BB_ORDER,
    BB_SCAL,
    BB_BINOM,
    BB_INV,
    // direct-mapped working column of dimension 1 (batched path)
    BB_BM_POS,
    BB_BM_VERTS,
    BB_BM_LEN,
    BB_BM_RUN,
    BB_BM_APP,
    BB_BM_APPE,
    BB_BM_BITS,
    // workgroups that share one cloud (spread-out batched reduction)
    BB_SYNC,
    BB_PAR_CST,
    BB_PAR_CTL,
    BB_PAR_STAT,
    // the same for the single-cloud path, and its edge sort
    B_BM_POS,
    B_BM_VERTS,
    B_BM_LEN,
    B_BM_RUN,
    B_BM_APP,
    B_BM_BITS,
    B_BM_SORT_LO0,
    B_BM_SORT_LO1,
    B_BM_SORT_HI0,
    B_BM_SORT_HI1,
    B_BM_SORT_V0,
    B_BM_SORT_V1,
    // homology variant
    B_HOM_OUT,
    B_HOM_PERM,
    B_HOM_PERM2,
    B_HOM_TAPP,
    // explicit matrix reduction
    B_EXP_CNT,
    B_EXP_OFF,
    B_EXP_OUT,
    B_EXP_IDX,
    B_EXP_DIA,
    B_EXP_COEF,
    B_EXP_WI0,
    B_EXP_WI1,
    B_EXP_WD0,
    B_EXP_WD1,
    B_EXP_WC0,
    B_EXP_WC1,
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
    int64_t hint_far = 0;
    int64_t hint_vw = 0;
    int64_t hint_log = 0;
    int64_t hint_cob = 0;
    int64_t hint_exp_w = 0;
    int lds_per_block = 0;
    int num_cus = 0;
    int reduce_groups = 0; // workgroups of the single-cloud reduction: 0 = one per CU
    int shortcuts = kShortApparent | kShortEmergent | kShortClearing; // of the single-cloud path
    int cocycle_dim = -1; // dimension whose zero columns also store V_j (cocycle requests)
    int rstore = kRStoreAuto; // when the single-cloud path stores R_j beside V_j
    hipStream_t capture_stream = nullptr;
    // cached graph of the batched launch and the arguments it was built for
    hipGraphExec_t batch_exec = nullptr;
    std::vector<unsigned char> batch_key;
    int64_t batch_vstride = 0;
    int64_t batch_fstride = 0;
    int64_t batch_vwstride = 0;
    int64_t batch_logstride = 0;
    u32 batch_capD = 0; // 0 = default delta size of the batched reduction
    int batch_wgpcu = 0; // 0 = default (1 persistent workgroup per CU)
    int batch_spread_off = 0; // 1 = one workgroup per cloud even for a small batch
    int working_column = RIPS_WORKING_COLUMN_AUTO; // rips_set_working_column
    // the bitmap buffers are zero between columns; these record what was
    // zeroed after the last allocation (pointer and bytes) per path
    void *bm_zero_ptr[2] = {nullptr, nullptr};
    size_t bm_zero_bytes[2] = {0, 0};

    // No-allocation mode (the context of rips_barcode_device_noalloc): every
    // buffer is carved from one fixed device region instead of hipMalloc;
    // reset_arena() at the start of each call forgets the carving.
    unsigned char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    int arena_last = -1;  // buffer carved last (it can grow in place)
    bool arena_full = false;

    void reset_arena() {
        for (int i = 0; i < B_NUM; ++i) {
            buf[i] = nullptr;
            cap[i] = 0;
        }
        arena_used = 0;
        arena_last = -1;
        arena_full = false;
    }

    hipError_t carve(int id, size_t bytes, void **out) {
        const size_t al = 256;
        if (id == arena_last && buf[id]) {
            // the last region grows in place
            const size_t at = (size_t)((unsigned char *)buf[id] - arena);
            if (at + bytes <= arena_cap) {
                arena_used = (at + bytes + al - 1) / al * al;
                cap[id] = bytes;
                *out = buf[id];
                return hipSuccess;
            }
        } else {
            const size_t at = (arena_used + al - 1) / al * al;
            if (at + bytes <= arena_cap) {
                buf[id] = arena + at;
                cap[id] = bytes;
                arena_used = (at + bytes + al - 1) / al * al;
                arena_last = id;
                *out = buf[id];
                return hipSuccess;
            }
        }
        arena_full = true;
        return hipErrorOutOfMemory;
    }

    hipError_t ensure(int id, size_t bytes, void **out) {
        if (bytes == 0) bytes = 16;
        if (arena) {
            if (cap[id] >= bytes) {
                *out = buf[id];
                return hipSuccess;
            }
            return carve(id, bytes, out);
        }
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
        HIP_TRY(hipDeviceGetAttribute(&c->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      dev));
        HIP_TRY(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
        g_ctx[dev] = c;
    }
    *out = g_ctx[dev];
    return RIPS_OK;
}

// Device memory of the no-allocation entry point (rips_barcode_device_noalloc):
// one fixed region per GPU, held until the process ends. In host code the
// symbol is only a stand-in; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kNoAllocBytes = (size_t)RIPS_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

DevCtx *g_ctx_na[64];
Scalars g_na_scal[64]; // host copies of the scalars (pageable: nothing is allocated)

// The context of the no-allocation entry point on the current device: set up
// at its first call there (the device address of `scratch`, the device
// attributes), with no allocation of device or pinned memory.
rips_status get_ctx_noalloc(DevCtx **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(RIPS_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (!g_ctx_na[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(RIPS_E_HIP, "no device address for the no-allocation scratch");
        static DevCtx ctx_store[64];
        DevCtx *c = &ctx_store[dev];
        c->arena = (unsigned char *)ptr;
        c->arena_cap = kNoAllocBytes;
        c->host_scal = &g_na_scal[dev];
        HIP_TRY(hipDeviceGetAttribute(&c->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      dev));
        HIP_TRY(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
        g_ctx_na[dev] = c;
    }
    *out = g_ctx_na[dev];
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

// ---------------------------------------------------------------------------
// Optional per-kernel-class GPU timing (rips_profile_*): hipEvents recorded
// on the caller's stream around each launch, resolved at the sync points.
// ---------------------------------------------------------------------------
enum ProfId {
    P_TABLES,
    P_DIST,
    P_THRESHOLD,
    P_EDGES,
    P_CSR,
    P_H0,
    P_EXPAND1, // expansion to dimension k at P_EXPAND1 + k - 1 (k = 2..)
    P_FILTER1 = P_EXPAND1 + kMaxDim + 1,
    P_SORT1 = P_FILTER1 + kMaxDim,
    P_REDUCE1 = P_SORT1 + kMaxDim,
    P_COB1 = P_REDUCE1 + kMaxDim,
    P_EXP_BUILD1 = P_COB1 + kMaxDim, // explicit coboundary matrix of dimension k
    P_EMIT = P_EXP_BUILD1 + kMaxDim,
    P_BATCHED,
    P_NUM
};

const char *prof_name(int i) {
    static char names[P_NUM][32];
    static bool init = false;
    if (!init) {
        for (int q = 0; q < P_NUM; ++q) snprintf(names[q], 32, "k%d", q);
        snprintf(names[P_TABLES], 32, "tables");
        snprintf(names[P_DIST], 32, "distances");
        snprintf(names[P_THRESHOLD], 32, "threshold");
        snprintf(names[P_EDGES], 32, "edges");
        snprintf(names[P_CSR], 32, "neighbour_lists");
        snprintf(names[P_H0], 32, "h0");
        for (int k = 1; k <= kMaxDim + 1; ++k) snprintf(names[P_EXPAND1 + k - 1], 32, "expand_d%d", k);
        for (int k = 1; k <= kMaxDim; ++k) {
            snprintf(names[P_FILTER1 + k - 1], 32, "filter_d%d", k);
            snprintf(names[P_SORT1 + k - 1], 32, "sort_d%d", k);
            snprintf(names[P_REDUCE1 + k - 1], 32, "reduce_d%d", k);
            snprintf(names[P_COB1 + k - 1], 32, "cob_lists_d%d", k);
            snprintf(names[P_EXP_BUILD1 + k - 1], 32, "explicit_build_d%d", k);
        }
        snprintf(names[P_EMIT], 32, "emit");
        snprintf(names[P_BATCHED], 32, "batched_graph");
        init = true;
    }
    return (i >= 0 && i < P_NUM) ? names[i] : "";
}

struct Profiler {
    std::mutex mu;
    bool on = false;
    double ms[P_NUM] = {};
    int64_t calls[P_NUM] = {};
    std::vector<hipEvent_t> pool;
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    size_t next = 0;
    hipEvent_t get() {
        if (next == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[next++];
    }
};
Profiler g_prof;
// set while the no-allocation entry point runs: its launches are not timed
// (timing would create events and grow the profiler's lists)
thread_local bool g_prof_quiet = false;

struct ProfScope {
    hipStream_t st;
    int id;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int id_, hipStream_t st_) : st(st_), id(id_) {
        if (!g_prof.on || g_prof_quiet) return;
        a = g_prof.get();
        b = g_prof.get();
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        g_prof.pending.push_back({id, a, b});
    }
};

// after a stream synchronize: fold the finished intervals into the totals
void prof_resolve() {
    if (!g_prof.on || g_prof_quiet) return;
    for (auto &r : g_prof.pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof.ms[r.id] += ms;
            g_prof.calls[r.id] += 1;
        }
    }
    g_prof.pending.clear();
    g_prof.next = 0;
}

#define PROF_CAT2(a, b) a##b
#define PROF_CAT(a, b) PROF_CAT2(a, b)
#define PROF(id) ProfScope PROF_CAT(prof_scope_, __LINE__)((id), st)

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
    prof_resolve();
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
    {
        PROF(P_TABLES);
        launch_binom(P.B, stride, n, jmax, st);
    }
    HIP_TRY(C.ensure(B_INV, (size_t)p * 4, &q));
    P.inv = as<u32>(q);
    {
        PROF(P_TABLES);
        launch_inverse(P.inv, p, st);
    }
    HIP_TRY(C.ensure(B_D, (size_t)n * n * 4, &q));
    P.D = as<float>(q);
    HIP_TRY(C.ensure(B_SCAL, sizeof(Scalars), &q));
    P.scal = as<Scalars>(q);
    launch_init_scalars(P.scal, st);
    {
        PROF(P_DIST);
        launch_dist(d_in, n, m, P.D, &P.scal->bad, st);
    }
    {
        PROF(P_THRESHOLD);
        launch_threshold(P.D, n, t, P.scal, st);
    }
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
        {
            PROF(P_EDGES);
            launch_edges(P.D, n, P.scal, P.E, cap, P.deg, st);
        }
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
        PROF(P_CSR);
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
    if (P.sparse) return 16;
    return P.ctx.n <= 128 ? 16 : 32;
}

// Lanes per candidate of the apparent-pair filter. Its time goes into the
// per-candidate tests every lane of a group repeats, more than into the
// scan, so groups are narrower than the expansion's: one lane per candidate
// for sparse dimensions >= 2, four for edges, eight for small dense clouds.
int filter_group_size_for(const Prepared &P, int k) {
    if (P.sparse) return k == 1 ? 4 : 1;
    return P.ctx.n <= 128 ? 8 : 32;
}

// Explicit matrix reduction of dimension k (the first column of Table 3):
// the coboundary matrix of the S columns is built in HBM, then reduced by
// adding stored reduced columns. Fills bars (column order), o.count[k] and
// o.stats[k]; ph receives the pivots (clearing of dimension k+1).
rips_status reduce_explicit(DevCtx &C, const Prepared &P, int k, uint32_t p, const Columns &cols, int64_t S,
                            PivotHash ph, uint32_t phcap, const u32 *prev_bits, PivotHash prev, BarBuf bars,
                            hipStream_t st, RunOut &o) {
    void *q;
    HIP_TRY(C.ensure(B_EXP_CNT, (size_t)(S + 1) * 8, &q));
    int64_t *cnt = as<int64_t>(q);
    HIP_TRY(C.ensure(B_EXP_OFF, (size_t)(S + 1) * 8, &q));
    int64_t *off = as<int64_t>(q);
    HIP_TRY(C.ensure(B_EXP_OUT, sizeof(ExpOut), &q));
    ExpOut *hout = as<ExpOut>(q);
    HIP_TRY(hipMemsetAsync(hout, 0, sizeof(ExpOut), st));
    int64_t nnz = 0;
    ExpOut h{};
    {
        PROF(P_EXP_BUILD1 + k - 1);
        launch_exp_count(P.ctx, k, cols.idx, cols.diam, S, cnt, &hout->longest, st);
        launch_exp_offsets(cnt, S, off, st);
        HIP_TRY(hipMemcpyAsync(&nnz, off + S, 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&h, hout, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (h.longest > (unsigned long long)kExpBuildCap)
        return fail(RIPS_E_CAPACITY, "a column of the explicit coboundary matrix exceeds " +
                                         std::to_string(kExpBuildCap) + " entries");
    ExpJob J{};
    J.k = k;
    J.p = p;
    J.inv = P.inv;
    J.cidx = cols.idx;
    J.cdia = cols.diam;
    J.ncols = S;
    HIP_TRY(C.ensure(B_EXP_IDX, (size_t)std::max<int64_t>(nnz, 1) * 8, &q));
    J.D.idx = as<int64_t>(q);
    HIP_TRY(C.ensure(B_EXP_DIA, (size_t)std::max<int64_t>(nnz, 1) * 4, &q));
    J.D.diam = as<float>(q);
    HIP_TRY(C.ensure(B_EXP_COEF, (size_t)std::max<int64_t>(nnz, 1) * 4, &q));
    J.D.coef = as<u32>(q);
    J.D.off = off;
    {
        PROF(P_EXP_BUILD1 + k - 1);
        launch_exp_fill(P.ctx, k, p, cols.idx, cols.diam, S, off, J.D, st);
    }
    J.piv = ph;
    J.prev = prev;
    J.prev_bits = prev_bits;
    J.clearing = (C.shortcuts & kShortClearing) ? 1 : 0;
    HIP_TRY(C.ensure(B_V_ROFF, (size_t)std::max<int64_t>(S, 1) * 8, &q));
    J.roff = as<int64_t>(q);
    HIP_TRY(C.ensure(B_V_RLEN, (size_t)std::max<int64_t>(S, 1) * 4, &q));
    J.rlen = as<int>(q);
    J.bars = bars;
    J.out = hout;
    int64_t pcap = std::max<int64_t>(C.hint_v, nnz + 4096);
    int64_t wcap = std::max<int64_t>(C.hint_exp_w, 4 * (int64_t)h.longest + 4096);
    for (int attempt = 0;; ++attempt) {
        if (attempt > 12) return fail(RIPS_E_CAPACITY, "explicit reduction scratch kept overflowing");
        HIP_TRY(C.ensure(B_V_IDX, (size_t)pcap * 8, &q));
        J.pidx = as<int64_t>(q);
        HIP_TRY(C.ensure(B_V_DIAM, (size_t)pcap * 4, &q));
        J.pdia = as<float>(q);
        HIP_TRY(C.ensure(B_V_COEF, (size_t)pcap * 4, &q));
        J.pcoef = as<u32>(q);
        J.pcap = pcap;
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(C.ensure(B_EXP_WI0 + b, (size_t)wcap * 8, &q));
            J.wi[b] = as<int64_t>(q);
            HIP_TRY(C.ensure(B_EXP_WD0 + b, (size_t)wcap * 4, &q));
            J.wd[b] = as<float>(q);
            HIP_TRY(C.ensure(B_EXP_WC0 + b, (size_t)wcap * 4, &q));
            J.wc[b] = as<u32>(q);
        }
        J.wcap = (int)wcap;
        launch_fill_i64(ph.keys, phcap, kEmpty, st);
        {
            PROF(P_REDUCE1 + k - 1);
            launch_exp_reduce(J, st);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&h, hout, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h.status == kExpPool) {
            pcap *= 4;
        } else if (h.status == kExpFull && wcap < (1ll << 28)) {
            wcap = std::min<int64_t>(wcap * 4, 1ll << 28);
        } else {
            break;
        }
    }
    if (h.status == kExpFull) return fail(RIPS_E_CAPACITY, "a working column of the explicit reduction exceeded 2^28 entries");
    if (h.status == kExpBound) return fail(RIPS_E_CAPACITY, "reduction: a column exceeded the bound of 2^24 additions");
    if (h.status != kExpOk) return fail(RIPS_E_HIP, "explicit reduction: internal consistency check failed");
    if (h.stored > C.hint_v) C.hint_v = h.stored;
    if (wcap > C.hint_exp_w) C.hint_exp_w = wcap;
    o.count[k] = h.bars;
    o.stats[k].emergent = 0;
    o.stats[k].reduced = h.reduced;
    o.stats[k].additions = h.additions;
    o.stats[k].bars_nonzero = h.bars - h.essential;
    o.stats[k].essential = h.essential;
    o.stats[k].entries_added = h.added;
    o.stats[k].entries_stored = nnz + h.stored;
    return RIPS_OK;
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
    {
        PROF(P_H0);
        launch_h0(P.E, P.scal, n, W, bars[0], nwords, st);
    }
    if ((rs = read_scalars(C, P.scal, st))) return rs;
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
                {
                    PROF(P_EXPAND1 + k - 1);
                    launch_expand(G, P.ctx, k, prev_list, prev_count, P.scal, cand, cap, false, st);
                }
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
        // zero apparent pairs (rho, tau) found by the filter, for the
        // reduction's pivot test; twice the candidates, so inserts never fail
        // (none without the apparent shortcut: those pairs are columns then)
        // (the explicit matrix has no use for them: its columns are all built)
        // (cocycle requests keep the implicit reduction, which stores V_j)
        const bool explicit_matrix = C.rstore == kRStoreExplicit && C.cocycle_dim < 0;
        const bool apparent = (C.shortcuts & kShortApparent) != 0 && !explicit_matrix;
        PairHash app{};
        int64_t *ckey_w = nullptr;
        float *cdia_w = nullptr;
        int64_t cobcap = 0;
        if (ncand > (1ll << 30)) return fail(RIPS_E_CAPACITY, "too many candidate simplices");
        // table sizes are 32-bit powers of two
        if ((uint64_t)2 * ncand + 64 > (1ull << 31)) return fail(RIPS_E_CAPACITY, "too many candidates");
        const uint32_t appcap = next_pow2((uint64_t)2 * ncand + 64);
        if (apparent) {
            HIP_TRY(C.ensure(B_APP_KEYS, (size_t)appcap * 8, &q));
            app.keys = as<int64_t>(q);
            HIP_TRY(C.ensure(B_APP_VALS, (size_t)appcap * 8, &q));
            app.vals = as<int64_t>(q);
            HIP_TRY(C.ensure(B_APP_VERTS, (size_t)appcap * 8, &q));
            app.verts = as<u64>(q);
            HIP_TRY(C.ensure(B_APP_NBR, (size_t)appcap * 8, &q));
            app.nbr = as<u64>(q);
            HIP_TRY(C.ensure(B_APP_COB, (size_t)appcap * 8, &q));
            app.cob = as<u64>(q);
            // room for the coboundary lists of the apparent pairs: a slot reserves
            // as many entries as rho has candidates (grown from the last call's need)
            const int64_t per = P.sparse ? std::min<int64_t>(std::max(P.maxdeg, 1), 64) : n;
            cobcap = std::max<int64_t>(C.hint_cob, std::min<int64_t>(ncand * per, 1ll << 25));
            // no-allocation mode: a small list buffer (a slot whose list does
            // not fit gets none; the reduction then enumerates it)
            if (C.arena) cobcap = std::min<int64_t>(cobcap, 1ll << 18);
            HIP_TRY(C.ensure(B_COB_KEY, (size_t)cobcap * 8, &q));
            app.ckey = as<int64_t>(q);
            ckey_w = as<int64_t>(q);
            HIP_TRY(C.ensure(B_COB_DIA, (size_t)cobcap * 4, &q));
            app.cdia = as<float>(q);
            cdia_w = as<float>(q);
            app.mask = appcap - 1;
            launch_fill_i64(app.keys, appcap, kEmpty, st);
        }
        {
            PROF(P_FILTER1 + k - 1);
            launch_filter(filter_group_size_for(P, k), P.ctx, k, cand, ncand, W.bits, ph_prev, P.scal, surv,
                          app, (apparent ? kShortApparent : 0) | (C.shortcuts & kShortClearing), st);
        }
        // the coboundary lists serve the general working column's apparent
        // runs; a dimension that the direct-mapped column will reduce (the
        // same conditions as below, with every workgroup counted) has no use
        // for them
        const int64_t bm_w = (n + 31) / 32;
        const int64_t bm_groups = C.reduce_groups > 0 ? C.reduce_groups : std::max(1, C.num_cus);
        const size_t bm_budget = C.lds_per_block > 16384 ? (size_t)C.lds_per_block - 12288 : 0;
        const bool bm_ahead = k == 1 && p == 2 && !C.arena && !P.sparse &&
                              C.working_column == RIPS_WORKING_COLUMN_AUTO &&
                              C.shortcuts == (kShortApparent | kShortEmergent | kShortClearing) &&
                              C.rstore == kRStoreAuto && bm_w <= 60 && P.nedges > 0 && P.nedges <= (1 << 18) &&
                              bm_groups * P.nedges * bm_w * 4 <= (8ll << 30) &&
                              reduce_lds_bytes(256) + bm_lds_bytes(P.nedges) <= bm_budget;
        if (apparent && !bm_ahead) {
            PROF(P_COB1 + k - 1);
            hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->cob, 0ull);
            launch_cob_lists(P.ctx, k, app, ckey_w, cdia_w, &P.scal->cob, cobcap, st);
        } else if (apparent) {
            app.cob = nullptr;
            app.ckey = nullptr;
            app.cdia = nullptr;
        }
        if ((rs = read_scalars(C, P.scal, st))) return rs;
        if ((int64_t)C.host_scal->cob > C.hint_cob)
            C.hint_cob = std::min<int64_t>((int64_t)C.host_scal->cob, 1ll << 28);
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
        {
            PROF(P_SORT1 + k - 1);
            launch_sort_columns(surv, P.scal, sb, lo_bytes, cols, st);
        }
        // ---- reduction
        const int slot = k & 1;
        PivotHash ph;
        if ((uint64_t)2 * S + 64 > (1ull << 31)) return fail(RIPS_E_CAPACITY, "too many columns");
        const uint32_t phcap = next_pow2((uint64_t)2 * S + 64);
        HIP_TRY(C.ensure(B_PH_KEYS0 + slot, (size_t)phcap * 8, &q));
        ph.keys = as<int64_t>(q);
        HIP_TRY(C.ensure(B_PH_VALS0 + slot, (size_t)phcap * 4, &q));
        ph.vals = as<int32_t>(q);
        ph.mask = phcap - 1;
        if (explicit_matrix) {
            if ((rs = ensure_bars(k, S))) return rs;
            if ((rs = reduce_explicit(C, P, k, p, cols, S, ph, phcap, W.bits, ph_prev, bars[k], st, o)))
                return rs;
            ph_prev = ph;
            prev_list = cand;
            prev_count = ncand;
            continue;
        }
        VStore V;
        HIP_TRY(C.ensure(B_V_OFF, (size_t)S * 8, &q));
        V.off = as<int64_t>(q);
        HIP_TRY(C.ensure(B_V_LEN, (size_t)S * 4, &q));
        V.len = as<int>(q);
        HIP_TRY(C.ensure(B_V_PIV, (size_t)S * 4, &q));
        V.pivcoef = as<u32>(q);
        HIP_TRY(C.ensure(B_V_ROFF, (size_t)S * 8, &q));
        V.roff = as<int64_t>(q);
        HIP_TRY(C.ensure(B_V_RLEN, (size_t)S * 4, &q));
        V.rlen = as<int>(q);
        int64_t vcap = std::max<int64_t>(C.hint_v, C.arena ? 16 * S + 16384 : 64 * S + 65536);
        if ((rs = ensure_bars(k, S))) return rs;
        const int bound = P.sparse ? P.maxdeg : n;
        // working column: the delta in LDS (as large as a workgroup's share
        // allows), the sorted base in global scratch (grown on overflow)
        const size_t lds_budget = C.lds_per_block > 16384 ? (size_t)C.lds_per_block - 12288 : 0;
        // the columns spread over one workgroup per CU, each with its own
        // scratch (smaller first sizes, grown on overflow), or one workgroup
        // (no-allocation mode: one workgroup, whose scratch is small)
        const int64_t want = C.arena ? 1 : C.reduce_groups > 0 ? C.reduce_groups : std::max(1, C.num_cus);
        const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(want, S));
        const bool spread = groups > 1;
        // the direct-mapped working column of dimension 1 (Z/2, every
        // shortcut and the default storage), where its bitmaps and summary fit
        const int64_t nE = P.nedges;
        const int64_t bmW = (n + 31) / 32;
        // (dense clouds: sparse ones keep the general column, whose apparent
        // runs read the precomputed coboundary lists of the filter)
        const bool bm = k == 1 && p == 2 && S > 0 && !C.arena && !P.sparse &&
                        C.working_column == RIPS_WORKING_COLUMN_AUTO &&
                        C.shortcuts == (kShortApparent | kShortEmergent | kShortClearing) &&
                        C.rstore == kRStoreAuto && bmW <= 60 && nE > 0 && nE <= (1 << 18) &&
                        groups * nE * bmW * 4 <= (8ll << 30) &&
                        reduce_lds_bytes(256) + bm_lds_bytes(nE) <= lds_budget;
        uint32_t capD = kMaxDelta;
        while (capD > 256 && reduce_lds_bytes(capD) + (bm ? bm_lds_bytes(nE) : 0) > lds_budget) capD >>= 1;
        EdgeOrder eo{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, 0};
        u32 *bm_bits = nullptr;
        if (bm) {
            HIP_TRY(C.ensure(B_BM_POS, (size_t)n * n * 4 + 16, &q));
            int *bpos = as<int>(q);
            HIP_TRY(C.ensure(B_BM_VERTS, (size_t)nE * 4, &q));
            u32 *bverts = as<u32>(q);
            HIP_TRY(C.ensure(B_BM_LEN, (size_t)nE * 4, &q));
            float *blen = as<float>(q);
            HIP_TRY(C.ensure(B_BM_RUN, (size_t)nE * 4, &q));
            u32 *brun = as<u32>(q);
            HIP_TRY(C.ensure(B_BM_APP, (size_t)nE * 4, &q));
            int *bapp = as<int>(q);
            SortBufs eb;
            HIP_TRY(C.ensure(B_BM_SORT_LO0, (size_t)nE * 8, &q));
            eb.lo[0] = as<u64>(q);
            HIP_TRY(C.ensure(B_BM_SORT_LO1, (size_t)nE * 8, &q));
            eb.lo[1] = as<u64>(q);
            HIP_TRY(C.ensure(B_BM_SORT_HI0, (size_t)nE * 4, &q));
            eb.hi[0] = as<u32>(q);
            HIP_TRY(C.ensure(B_BM_SORT_HI1, (size_t)nE * 4, &q));
            eb.hi[1] = as<u32>(q);
            HIP_TRY(C.ensure(B_BM_SORT_V0, (size_t)nE * 4, &q));
            eb.val[0] = as<u32>(q);
            HIP_TRY(C.ensure(B_BM_SORT_V1, (size_t)nE * 4, &q));
            eb.val[1] = as<u32>(q);
            const size_t need = (size_t)(groups * nE * bmW * 4);
            HIP_TRY(C.ensure(B_BM_BITS, need, &q));
            bm_bits = as<u32>(q);
            if (C.bm_zero_ptr[0] != (void *)bm_bits || C.bm_zero_bytes[0] < need) {
                HIP_TRY(hipMemsetAsync(bm_bits, 0, need, st));
                C.bm_zero_ptr[0] = (void *)bm_bits;
                C.bm_zero_bytes[0] = need;
            }
            {
                PROF(P_SORT1);
                launch_bm_edge_order(P.E, (int)nE, n, eb, bpos, bverts, blen, brun, app, bapp, st);
            }
            eo = EdgeOrder{bpos, bverts, blen, brun, bapp, (int)nE, (int)bmW, n};
        }
        int64_t fcap = spread ? std::max<int64_t>(C.hint_far, 1 << 16)
                              : std::max<int64_t>(C.hint_far, std::max<int64_t>(1 << 18, 256ll * bound));
        int64_t vwcap = std::max<int64_t>(C.hint_vw, 1 << 14);
        // one log entry per addition: the log grows on overflow, up to the addition bound
        const int64_t lmax = (int64_t)kMaxAdditions + 64;
        int64_t lcap = std::max<int64_t>(C.hint_log, spread ? 1 << 14 : (1 << 18) + 64);
        BarBuf cbars = bars[k];
        if (spread) {
            HIP_TRY(C.ensure(B_CBAR_BIRTH, (size_t)S * 4, &q));
            cbars.birth = as<float>(q);
            HIP_TRY(C.ensure(B_CBAR_DEATH, (size_t)S * 4, &q));
            cbars.death = as<float>(q);
            HIP_TRY(C.ensure(B_CBAR_BS, (size_t)S * 8, &q));
            cbars.bs = as<int64_t>(q);
            HIP_TRY(C.ensure(B_CBAR_DS, (size_t)S * 8, &q));
            cbars.ds = as<int64_t>(q);
        }
#if RIPS_COLUMN_TRACE
        unsigned long long *trace_buf = nullptr;
#endif
        for (int attempt = 0;; ++attempt) {
            if (attempt > 12) return fail(RIPS_E_CAPACITY, "reduction scratch kept overflowing");
            HIP_TRY(C.ensure(B_V_IDX, (size_t)vcap * 8, &q));
            V.idx = as<int64_t>(q);
            HIP_TRY(C.ensure(B_V_DIAM, (size_t)vcap * 4, &q));
            V.diam = as<float>(q);
            HIP_TRY(C.ensure(B_V_COEF, (size_t)vcap * 4, &q));
            V.coef = as<u32>(q);
            V.cap = vcap;
            ReduceBuffers RB;
            // one far list, working-V table and log per workgroup
            for (int b = 0; b < 2; ++b) {
                HIP_TRY(C.ensure(B_F_IDX0 + b, (size_t)(groups * fcap) * 8, &q));
                RB.F.idx[b] = as<int64_t>(q);
                HIP_TRY(C.ensure(B_F_DIA0 + b, (size_t)(groups * fcap) * 4, &q));
                RB.F.dia[b] = as<float>(q);
                HIP_TRY(C.ensure(B_F_COEF0 + b, (size_t)(groups * fcap) * 4, &q));
                RB.F.coef[b] = as<u32>(q);
            }
            RB.F.cap = fcap;
            HIP_TRY(C.ensure(B_VW_KEYS, (size_t)(groups * vwcap) * 8, &q));
            RB.vw_keys = as<int64_t>(q);
            HIP_TRY(C.ensure(B_VW_COEF, (size_t)(groups * vwcap) * 4, &q));
            RB.vw_coef = as<u32>(q);
            HIP_TRY(C.ensure(B_VW_DIAM, (size_t)(groups * vwcap) * 4, &q));
            RB.vw_diam = as<float>(q);
            HIP_TRY(C.ensure(B_VW_SLOTS, (size_t)(groups * vwcap) * 4, &q));
            RB.vw_slots = as<u32>(q);
            RB.vw_cap = vwcap;
            HIP_TRY(C.ensure(B_LOG_KEY, (size_t)(groups * lcap) * 8, &q));
            RB.lkey = as<int64_t>(q);
            HIP_TRY(C.ensure(B_LOG_COEF, (size_t)(groups * lcap) * 4, &q));
            RB.lcoef = as<u32>(q);
            HIP_TRY(C.ensure(B_LOG_DIA, (size_t)(groups * lcap) * 4, &q));
            RB.ldia = as<float>(q);
            RB.lcap = lcap;
            launch_fill_i64(ph.keys, phcap, kEmpty, st);
            launch_reset_dim(P.scal, st);
            ParState par{nullptr, nullptr};
            if (spread) {
                HIP_TRY(C.ensure(B_CST, (size_t)S * 4, &q));
                par.cst = as<u32>(q);
                HIP_TRY(C.ensure(B_CTL, (size_t)kCtlWords * 4, &q));
                par.ctl = as<u32>(q);
                launch_fill_u32(par.cst, S, 0u, st);
                launch_fill_u32(par.ctl, kCtlWords, 0u, st);
                launch_fill_u32((u32 *)ph.vals, phcap, 0xffffffffu, st); // -1: no value yet
            }
            ReduceJob<DistFull> J;
            J.c = P.ctx;
            J.k = k;
            J.p = p;
            J.inv = P.inv;
            J.cols = cols;
            J.ncols = (int)S;
            J.ph = ph;
            J.V = V;
            J.vcount = &P.scal->vcount;
            J.bars = spread ? cbars : bars[k];
            J.app = app;
            J.par = par;
            J.shortcuts = C.shortcuts;
#if RIPS_COLUMN_TRACE
            // profiling builds only: per-column clocks of the spread-out reduction
            if (trace_buf) (void)hipFree(trace_buf);
            trace_buf = nullptr;
            if (getenv("RIPS_COLUMN_TRACE_OUT") && hipMalloc(&trace_buf, (size_t)S * 32 + 32) == hipSuccess)
                (void)hipMemset(trace_buf, 0, (size_t)S * 32 + 32);
            J.trace = trace_buf;
#endif
            J.keep_essential_v = k == C.cocycle_dim ? 1 : 0;
            J.rstore = C.rstore;
            J.prev_bits = W.bits;
            J.prev = ph_prev;
            J.cand_avg = P.sparse ? (float)(2.0 * (double)P.nedges / (double)std::max<int64_t>(n, 1))
                                  : (float)n;
            if (bm) {
                J.eo = eo;
                J.bm_bits = bm_bits;
                J.bm_stride = nE * bmW;
            }
            {
                PROF(P_REDUCE1 + k - 1);
                if (spread) HIP_TRY(launch_reduce_par(J, capD, RB, (int)groups, bars[k], P.scal, st));
                else HIP_TRY(launch_reduce(J, capD, RB, P.scal, st));
            }
            if ((rs = read_scalars(C, P.scal, st))) return rs;
            const int status = C.host_scal->status;
            if (status == 0) break;
            if (status == kRedStoreFull) {
                vcap *= 4;
            } else if (status == kRedFarFull) {
                fcap *= 4;
                C.hint_far = fcap;
            } else if (status == kRedVFull) {
                vwcap *= 4;
                C.hint_vw = vwcap;
            } else if (status == kRedLogFull && lcap < lmax) {
                lcap = std::min(lmax, lcap * 4);
                C.hint_log = lcap;
            } else if (status == kRedLogFull) {
                return fail(RIPS_E_HIP, "reduction log overflow");
            } else if (status == kRedWait) {
                return fail(RIPS_E_HIP, "reduction: a wait for earlier columns exceeded its bound");
            } else if (status == kRedBound) {
                return fail(RIPS_E_CAPACITY, "reduction: a column exceeded the bound of 2^24 additions");
            } else {
                char msg[96];
                snprintf(msg, sizeof(msg), "reduction: internal consistency check %d failed", status);
                return fail(RIPS_E_HIP, msg);
            }
        }
        if ((int64_t)C.host_scal->vcount > C.hint_v) C.hint_v = (int64_t)C.host_scal->vcount;
#if RIPS_PHASE_TIMERS
        // profiling build: the reduction's counters and phase clocks
        if (getenv("RIPS_PHASE_REPORT"))
            fprintf(stderr,
                    "[rips reduce d%d] cols=%lld capD=%u lds_per_block=%d "
                    "base_cols=%llu entries=%llu maxV=%llu maxR=%llu additions=%llu pulls=%llu "
                    "merges=%llu splits=%llu pulled=%llu\n",
                    k, (long long)S, capD, C.lds_per_block,
                    C.host_scal->stat[kStatGlobalCols], C.host_scal->vcount,
                    C.host_scal->stat[kStatMaxV], C.host_scal->stat[kStatMaxR],
                    C.host_scal->stat[kStatAdditions], C.host_scal->stat[kStatPulls],
                    C.host_scal->stat[kStatMerges], C.host_scal->stat[kStatSplits],
                    C.host_scal->stat[kStatPulled]);
        if (getenv("RIPS_PHASE_REPORT")) {
            int khz = 0;
            (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0);
            const double f = khz > 0 ? 1.0 / khz : 1e-5;
            const unsigned long long *T = C.host_scal->stat + kStatTime;
            fprintf(stderr,
                    "[rips reduce d%d] ms (clock %d kHz): total %.2f setup %.2f pivot %.2f "
                    "owner %.2f add %.2f apparent %.2f store %.2f reset %.2f emergent %.2f | "
                    "merge %.2f (gather %.2f rank %.2f base %.2f prefix %.2f) pull %.2f split %.2f "
                    "apparent-add %.2f wait %.2f apparent-run %.2f (pivot %.2f lookup %.2f add %.2f) "
                    "(summed over %lld workgroups)\n",
                    k, khz, T[10] * f, T[6] * f, T[0] * f, T[11] * f, T[1] * f, T[7] * f,
                    T[5] * f, T[9] * f, T[8] * f, T[2] * f, T[12] * f, T[13] * f, T[14] * f,
                    T[15] * f, T[3] * f, T[4] * f, T[16] * f, T[17] * f, T[18] * f, T[19] * f, T[20] * f, T[21] * f,
                    (long long)groups);
        }
#endif
        o.count[k] = C.host_scal->nbars;
#if RIPS_COLUMN_TRACE
        if (trace_buf) {
            std::vector<unsigned long long> tb((size_t)S * 4);
            if (hipMemcpy(tb.data(), trace_buf, (size_t)S * 32, hipMemcpyDeviceToHost) == hipSuccess) {
                const std::string path = std::string(getenv("RIPS_COLUMN_TRACE_OUT")) + "_d" + std::to_string(k) + ".bin";
                if (FILE *fp = fopen(path.c_str(), "wb")) {
                    fwrite(tb.data(), 8, tb.size(), fp);
                    fclose(fp);
                }
            }
            (void)hipFree(trace_buf);
        }
#endif
        o.stats[k].emergent = (int64_t)C.host_scal->stat[kStatEmergent];
        o.stats[k].reduced = (int64_t)C.host_scal->stat[kStatReduced];
        o.stats[k].additions = (int64_t)C.host_scal->stat[kStatAdditions];
        o.stats[k].bars_nonzero = (int64_t)C.host_scal->stat[kStatBarsNonzero];
        o.stats[k].essential = (int64_t)C.host_scal->stat[kStatEssential];
        o.stats[k].entries_added = (int64_t)C.host_scal->stat[kStatAdded];
        o.stats[k].entries_stored = (int64_t)C.host_scal->vcount;
        ph_prev = ph;
        prev_list = cand;
        prev_count = ncand;
    }
    return RIPS_OK;
}

// ---------------------------------------------------------------------------
// The homology variant (ablation): boundary matrices with clearing, from the
// top dimension down (section "Clearing inessential birth columns"); the
// same bars as the cohomology path, with column counters that show what
// clearing leaves to reduce in homology.
// ---------------------------------------------------------------------------
struct HomRun {
    float t_eff, r_enc;
    int sparse;
    int64_t count[kMaxDim + 1];          // bars per dimension (unordered in B_BAR_* + d)
    int64_t simplex_count[kMaxDim + 2];
    rips_dim_stats stats[kMaxDim + 1];
};

rips_status run_homology(DevCtx &C, const float *d_in, int n, int m, int max_dim, float t, uint32_t p,
                         hipStream_t st, HomRun &o) {
    memset(&o, 0, sizeof(o));
    Prepared P;
    rips_status rs = prepare(C, d_in, n, m, max_dim + 2, t, p, st, P);
    if (rs) return rs;
    o.t_eff = C.host_scal->t_eff;
    o.r_enc = C.host_scal->r_enc;
    o.sparse = P.sparse;
    void *q;
    const int top = max_dim + 1;
    // the simplices of every dimension up to the top
    SimplexList list[kMaxDim + 2];
    int64_t cnt[kMaxDim + 2] = {};
    cnt[0] = n;
    list[1] = SimplexList{P.E.idx, P.E.diam};
    cnt[1] = P.nedges;
    const int G = group_size_for(P);
    for (int k = 2; k <= top; ++k) {
        int64_t cap = C.hint_list[k] > 0 ? C.hint_list[k] : std::max<int64_t>(cnt[k - 1] * 4, 1024);
        bool fits = false;
        for (int attempt = 0; attempt < 3 && !fits; ++attempt) {
            HIP_TRY(C.ensure(B_LIST_IDX + k, (size_t)cap * 8, &q));
            list[k].idx = as<int64_t>(q);
            HIP_TRY(C.ensure(B_LIST_DIAM + k, (size_t)cap * 4, &q));
            list[k].diam = as<float>(q);
            hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->list, 0ull);
            launch_expand(G, P.ctx, k, list[k - 1], cnt[k - 1], P.scal, list[k], cap, false, st);
            if ((rs = read_scalars(C, P.scal, st))) return rs;
            fits = (int64_t)C.host_scal->list <= cap;
            if (!fits) cap = (int64_t)C.host_scal->list;
        }
        if (!fits) return fail(RIPS_E_CAPACITY, "simplex list did not fit");
        cnt[k] = (int64_t)C.host_scal->list;
        if (cnt[k] > C.hint_list[k]) C.hint_list[k] = cnt[k];
    }
    for (int k = 0; k <= top; ++k) o.simplex_count[k] = cnt[k];
    // each dimension's simplices younger first (the column sort)
    Columns sorted[kMaxDim + 2] = {};
    for (int k = 1; k <= top; ++k) {
        const int64_t N = cnt[k];
        if (N > 0x7fffffff) return fail(RIPS_E_CAPACITY, "too many simplices for the homology variant");
        Columns in{list[k].idx, list[k].diam, nullptr, nullptr}, out;
        HIP_TRY(C.ensure(B_SURV_J, (size_t)N * 4, &q));
        in.j = as<int>(q);
        HIP_TRY(C.ensure(B_SURV_TAPP, (size_t)N, &q));
        in.tapp = as<uint8_t>(q);
        HIP_TRY(C.ensure(B_COL_IDX + k, (size_t)N * 8, &q));
        out.idx = as<int64_t>(q);
        HIP_TRY(C.ensure(B_COL_DIAM + k, (size_t)N * 4, &q));
        out.diam = as<float>(q);
        HIP_TRY(C.ensure(B_COL_J + k, (size_t)N * 4, &q));
        out.j = as<int>(q);
        HIP_TRY(C.ensure(B_COL_TAPP + k, (size_t)N, &q));
        out.tapp = as<uint8_t>(q);
        sorted[k] = out;
        if (N == 0) continue;
        SortBufs sb;
        HIP_TRY(C.ensure(B_SORT_LO0, (size_t)N * 8, &q));
        sb.lo[0] = as<u64>(q);
        HIP_TRY(C.ensure(B_SORT_LO1, (size_t)N * 8, &q));
        sb.lo[1] = as<u64>(q);
        HIP_TRY(C.ensure(B_SORT_HI0, (size_t)N * 4, &q));
        sb.hi[0] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_HI1, (size_t)N * 4, &q));
        sb.hi[1] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_V0, (size_t)N * 4, &q));
        sb.val[0] = as<u32>(q);
        HIP_TRY(C.ensure(B_SORT_V1, (size_t)N * 4, &q));
        sb.val[1] = as<u32>(q);
        hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &P.scal->survivors, (unsigned long long)N);
        launch_sort_columns(in, P.scal, sb, bytes_for((uint64_t)choose_i64(n, k + 1)), out, st);
    }
    // bars of dimension d: at most one per d-simplex
    BarBuf bars[kMaxDim + 1];
    int64_t bcap[kMaxDim + 1];
    for (int d = 0; d <= max_dim; ++d) {
        bcap[d] = std::max<int64_t>(cnt[d], 1);
        HIP_TRY(C.ensure(B_BAR_BIRTH + d, (size_t)bcap[d] * 4, &q));
        bars[d].birth = as<float>(q);
        HIP_TRY(C.ensure(B_BAR_DEATH + d, (size_t)bcap[d] * 4, &q));
        bars[d].death = as<float>(q);
        HIP_TRY(C.ensure(B_BAR_BS + d, (size_t)bcap[d] * 8, &q));
        bars[d].bs = as<int64_t>(q);
        HIP_TRY(C.ensure(B_BAR_DS + d, (size_t)bcap[d] * 8, &q));
        bars[d].ds = as<int64_t>(q);
    }
    HIP_TRY(C.ensure(B_HOM_OUT, sizeof(HomOut), &q));
    HomOut *hout = as<HomOut>(q);
    int64_t npairs[kMaxDim + 1] = {}, ness[kMaxDim + 1] = {};
    PivotHash above{nullptr, nullptr, 0};
    for (int k = top; k >= 1; --k) {
        const int64_t N = cnt[k];
        if ((uint64_t)2 * N + 64 > (1ull << 31)) return fail(RIPS_E_CAPACITY, "too many columns");
        const uint32_t phcap = next_pow2((uint64_t)2 * N + 64);
        const int slot = k & 1;
        HomJob J{};
        HIP_TRY(C.ensure(B_PH_KEYS0 + slot, (size_t)phcap * 8, &q));
        J.piv.keys = as<int64_t>(q);
        HIP_TRY(C.ensure(B_PH_VALS0 + slot, (size_t)phcap * 4, &q));
        J.piv.vals = as<int32_t>(q);
        J.piv.mask = phcap - 1;
        HIP_TRY(C.ensure(B_V_OFF, (size_t)std::max<int64_t>(N, 1) * 8, &q));
        J.roff = as<int64_t>(q);
        HIP_TRY(C.ensure(B_V_LEN, (size_t)std::max<int64_t>(N, 1) * 4, &q));
        J.rlen = as<int>(q);
        J.c = P.ctx;
        J.k = k;
        J.cidx = sorted[k].idx;
        J.cdia = sorted[k].diam;
        J.ncols = N;
        J.p = p;
        J.inv = P.inv;
        J.clear = above;
        J.pairs = bars[k - 1];
        J.pairs_cap = bcap[k - 1];
        J.essential = k <= max_dim ? 1 : 0;
        if (J.essential) {
            J.ess = BarBuf{bars[k].birth + npairs[k], bars[k].death + npairs[k], bars[k].bs + npairs[k],
                           bars[k].ds + npairs[k]};
            J.ess_cap = bcap[k] - npairs[k];
        }
        J.out = hout;
        int64_t pcap = std::max<int64_t>(C.hint_v, 8 * N + 4096);
        HomOut h{};
        for (int attempt = 0; attempt < 6; ++attempt) {
            HIP_TRY(C.ensure(B_V_IDX, (size_t)pcap * 8, &q));
            J.pidx = as<int64_t>(q);
            HIP_TRY(C.ensure(B_V_DIAM, (size_t)pcap * 4, &q));
            J.pdia = as<float>(q);
            HIP_TRY(C.ensure(B_V_COEF, (size_t)pcap * 4, &q));
            J.pcoef = as<u32>(q);
            J.pcap = pcap;
            launch_fill_i64(J.piv.keys, phcap, kEmpty, st);
            HIP_TRY(launch_hom_reduce(J, st));
            HIP_TRY(hipMemcpyAsync(&h, hout, sizeof(h), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (h.status != kHomPool) break;
            pcap *= 4;
        }
        if (h.status == kHomPool) return fail(RIPS_E_CAPACITY, "stored columns exceed the pool");
        if (h.status == kHomFull)
            return fail(RIPS_E_CAPACITY, "a column of the homology variant exceeded " +
                                             std::to_string(kHomCap) + " entries");
        if (h.status == kHomBound)
            return fail(RIPS_E_CAPACITY, "a column of the homology variant exceeded 2^24 additions");
        if (h.status != kHomOk) return fail(RIPS_E_HIP, "homology variant: internal consistency check failed");
        if (h.stored > C.hint_v) C.hint_v = h.stored;
        npairs[k - 1] = h.pairs;
        if (J.essential) ness[k] = h.essential;
        rips_dim_stats &sd = o.stats[k - 1];
        sd.candidates = N;
        sd.cleared = h.cleared;
        sd.columns = h.reduced;
        sd.reduced = h.nonzero;
        sd.additions = h.additions;
        sd.bars_nonzero = h.pairs;
        sd.entries_stored = h.stored;
        above = J.piv;
    }
    // dimension 0: vertices that no edge column has as its pivot
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, (unsigned long long *)&hout->essential, 0ull);
    launch_hom_vertices(n, above, BarBuf{bars[0].birth + npairs[0], bars[0].death + npairs[0],
                                         bars[0].bs + npairs[0], bars[0].ds + npairs[0]},
                        hout, st);
    {
        HomOut h{};
        HIP_TRY(hipMemcpyAsync(&h, hout, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ness[0] = h.essential;
    }
    for (int d = 0; d <= max_dim; ++d) {
        o.count[d] = npairs[d] + ness[d];
        o.stats[d].essential = ness[d];
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

rips_status batched_once(DevCtx &Cref, const float *d_points, const int64_t *d_offsets,
                                int32_t B, int32_t dim, int32_t n_max, int32_t max_dim,
                                float threshold, uint32_t p, rips_batch_out *out, void *hip_stream,
                                bool *retry) {
    DevCtx *C = &Cref;
    hipStream_t st = (hipStream_t)hip_stream;
    const int D1 = max_dim + 1;
    const bool lds_d = n_max <= kBatchLdsN;
    // a batch smaller than the chip spreads each cloud over several
    // workgroups, at most one per CU in all (they wait for each other, so all
    // of them must be resident at once)
    const int slots = std::max(1, C->num_cus) * std::max(1, C->batch_wgpcu);
    const int spread = C->batch_spread_off ? 1 : batched_spread(B, std::max(1, C->num_cus), max_dim);
    int grid = spread > 1 ? B * spread : std::min(slots, B);
    const int64_t npairs = (int64_t)n_max * (n_max - 1) / 2;
    const int64_t col_stride = npairs + n_max + 16;
    int64_t ph_stride = 64;
    while (ph_stride < 2 * col_stride + 64) ph_stride <<= 1;
    const int64_t v_stride = std::max<int64_t>(C->batch_vstride, std::max<int64_t>(1 << 18, 4 * col_stride));
    const u32 capD = C->batch_capD ? C->batch_capD : batched_default_capD(lds_d, n_max);
    const int64_t f_stride =
        std::max<int64_t>(C->batch_fstride, std::max<int64_t>(1 << 15, 64ll * n_max));
    const int64_t vw_stride = std::max<int64_t>(C->batch_vwstride, 1 << 12);
    const int64_t log_stride = std::max<int64_t>(C->batch_logstride, 1 << 14);
    const int64_t st_stride = 2 * (int64_t)n_max + npairs + 16;
    const int64_t d_stride = lds_d ? npairs + 4 : (int64_t)n_max * n_max + 4;
    const int64_t bits_stride = npairs / 32 + 2;
    const int64_t G = grid;
    void *q;
    BatchArgs A;
    memset(&A, 0, sizeof(A));
    A.X = d_points;
    A.offsets = d_offsets;
    A.B = B;
    A.m = dim;
    A.max_dim = max_dim;
    A.threshold = threshold;
    A.p = p;
    A.nmax = n_max;
#define ENS(id, bytes, field, T)                                                                   \
    do {                                                                                           \
        HIP_TRY(C->ensure(id, (size_t)(bytes), &q));                                               \
        field = as<T>(q);                                                                          \
    } while (0)
    ENS(BB_BINOM, (size_t)4 * (n_max + 1) * 8, A.binom.t, const u64);
    A.binom.stride = n_max + 1;
    u32 *inv;
    ENS(BB_INV, (size_t)p * 4, inv, u32);
    A.inv = inv;
    ENS(BB_DG, G * d_stride * 4, A.Dg, float);
    A.d_stride = d_stride;
    ENS(BB_C_IDX0, G * col_stride * 8, A.c_idx0, int64_t);
    ENS(BB_C_IDX1, G * col_stride * 8, A.c_idx1, int64_t);
    ENS(BB_C_DM0, G * col_stride * 4, A.c_dm0, float);
    ENS(BB_C_DM1, G * col_stride * 4, A.c_dm1, float);
    ENS(BB_C_J0, G * col_stride * 4, A.c_j0, int);
    ENS(BB_C_J1, G * col_stride * 4, A.c_j1, int);
    ENS(BB_C_T0, G * col_stride, A.c_t0, uint8_t);
    ENS(BB_C_T1, G * col_stride, A.c_t1, uint8_t);
    ENS(BB_S_LO0, G * col_stride * 8, A.s_lo0, u64);
    ENS(BB_S_LO1, G * col_stride * 8, A.s_lo1, u64);
    ENS(BB_S_HI0, G * col_stride * 4, A.s_hi0, u32);
    ENS(BB_S_HI1, G * col_stride * 4, A.s_hi1, u32);
    ENS(BB_S_V0, G * col_stride * 4, A.s_v0, u32);
    ENS(BB_S_V1, G * col_stride * 4, A.s_v1, u32);
    A.col_stride = col_stride;
    ENS(BB_PH_KEYS, G * ph_stride * 8, A.ph_keys, int64_t);
    ENS(BB_PH_VALS, G * ph_stride * 4, A.ph_vals, int32_t);
    A.ph_stride = ph_stride;
    ENS(BB_APP_KEYS, G * ph_stride * 8, A.app_keys, int64_t);
    ENS(BB_APP_VALS, G * ph_stride * 8, A.app_vals, int64_t);
    ENS(BB_APP_VERTS, G * ph_stride * 8, A.app_verts, u64);
    ENS(BB_V_OFF, G * col_stride * 8, A.v_off, int64_t);
    ENS(BB_V_LEN, G * col_stride * 4, A.v_len, int);
    ENS(BB_V_PIV, G * col_stride * 4, A.v_piv, u32);
    ENS(BB_V_IDX, G * v_stride * 8, A.v_idx, int64_t);
    ENS(BB_V_DIAM, G * v_stride * 4, A.v_diam, float);
    ENS(BB_V_COEF, G * v_stride * 4, A.v_coef, u32);
    A.v_stride = v_stride;
    ENS(BB_V_COUNT, G * 8, A.v_count, unsigned long long);
    ENS(BB_BITS, G * bits_stride * 4, A.bits_g, u32);
    A.bits_stride = bits_stride;
    A.capD = capD;
    for (int h = 0; h < 2; ++h) {
        ENS(BB_F_IDX0 + h, G * f_stride * 8, A.f_idx[h], int64_t);
        ENS(BB_F_DIA0 + h, G * f_stride * 4, A.f_dia[h], float);
        ENS(BB_F_COEF0 + h, G * f_stride * 4, A.f_coef[h], u32);
    }
    A.f_stride = f_stride;
    ENS(BB_VW_KEYS, G * vw_stride * 8, A.vw_keys, int64_t);
    ENS(BB_VW_COEF, G * vw_stride * 4, A.vw_coef, u32);
    ENS(BB_VW_DIAM, G * vw_stride * 4, A.vw_diam, float);
    ENS(BB_VW_SLOTS, G * vw_stride * 4, A.vw_slots, u32);
    A.vw_stride = vw_stride;
    ENS(BB_V_ROFF, G * col_stride * 8, A.v_roff, int64_t);
    ENS(BB_V_RLEN, G * col_stride * 4, A.v_rlen, int);
    ENS(BB_LOG_KEY, G * log_stride * 8, A.log_key, int64_t);
    ENS(BB_LOG_COEF, G * log_stride * 4, A.log_coef, u32);
    ENS(BB_LOG_DIA, G * log_stride * 4, A.log_dia, float);
    A.log_stride = log_stride;
    ENS(BB_ST_B, G * st_stride * 4, A.st_b, float);
    ENS(BB_ST_D, G * st_stride * 4, A.st_d, float);
    ENS(BB_ST_BS, G * st_stride * 8, A.st_bs, int64_t);
    ENS(BB_ST_DS, G * st_stride * 8, A.st_ds, int64_t);
    A.st_stride = st_stride;
    const int64_t ucap = std::max<int64_t>(out->cap, 1);
    ENS(BB_UB, ucap * 4, A.ub, float);
    ENS(BB_UD, ucap * 4, A.ud, float);
    ENS(BB_UBS, ucap * 8, A.ubs, int64_t);
    ENS(BB_UDS, ucap * 8, A.uds, int64_t);
    A.ucap = out->cap;
    ENS(BB_SEG_START, (int64_t)B * D1 * 8, A.seg_start, int64_t);
    ENS(BB_SEG_COUNT, (int64_t)B * D1 * 8, A.seg_count, int64_t);
    if (out->stats) A.stats = out->stats;
    else ENS(BB_STATS, (int64_t)B * D1 * sizeof(rips_dim_stats), A.stats, rips_dim_stats);
    if (out->threshold_used) A.t_used = out->threshold_used;
    else ENS(BB_TUSED, (int64_t)B * 4, A.t_used, float);
    SortBufs lpt;
    ENS(BB_LPT_LO0, (int64_t)B * 8, lpt.lo[0], u64);
    ENS(BB_LPT_LO1, (int64_t)B * 8, lpt.lo[1], u64);
    ENS(BB_LPT_HI0, (int64_t)B * 4, lpt.hi[0], u32);
    ENS(BB_LPT_HI1, (int64_t)B * 4, lpt.hi[1], u32);
    ENS(BB_LPT_V0, (int64_t)B * 4, lpt.val[0], u32);
    ENS(BB_LPT_V1, (int64_t)B * 4, lpt.val[1], u32);
    int *order;
    ENS(BB_ORDER, (int64_t)B * 4, order, int);
    A.order = order;
    A.spread = spread;
    if (spread > 1) {
        ENS(BB_SYNC, G * kSyncWords * 4, A.sync, int);
        ENS(BB_PAR_CST, G * col_stride * 4, A.par_cst, u32);
        ENS(BB_PAR_CTL, G * kCtlWords * 4, A.par_ctl, u32);
        ENS(BB_PAR_STAT, G * kSyncStats * 8, A.par_stat, unsigned long long);
    }
    // the direct-mapped working column of dimension 1, where it fits
    const bool bm = C->working_column == RIPS_WORKING_COLUMN_AUTO &&
                    batched_bm_fits(n_max, max_dim, p, G);
    if (bm) {
        const int64_t W = (n_max + 31) / 32;
        ENS(BB_BM_POS, G * (int64_t)n_max * n_max * 4, A.bm_pos, int);
        A.bm_pos_stride = (int64_t)n_max * n_max;
        ENS(BB_BM_VERTS, G * npairs * 4, A.bm_verts, u32);
        ENS(BB_BM_LEN, G * npairs * 4, A.bm_len, float);
        ENS(BB_BM_RUN, G * npairs * 4, A.bm_run, u32);
        ENS(BB_BM_APP, G * npairs * 4, A.bm_app, int);
        ENS(BB_BM_APPE, G * npairs * 4, A.bm_appe, int);
        A.bm_tab_stride = npairs;
        ENS(BB_BM_BITS, G * npairs * W * 4, A.bm_bits, u32);
        A.bm_stride = npairs * W;
        const size_t need = (size_t)(G * npairs * W * 4);
        if (C->bm_zero_ptr[1] != (void *)A.bm_bits || C->bm_zero_bytes[1] < need) {
            HIP_TRY(hipMemsetAsync(A.bm_bits, 0, need, st));
            C->bm_zero_ptr[1] = (void *)A.bm_bits;
            C->bm_zero_bytes[1] = need;
        }
    }
    struct BatchScal {
        unsigned long long queue, ucount;
        int64_t total;
        int status;
    };
    BatchScal *bs;
    ENS(BB_SCAL, sizeof(BatchScal), bs, BatchScal);
    A.queue = &bs->queue;
    A.ucount = &bs->ucount;
    A.status = &bs->status;
#undef ENS
    HIP_TRY(batched_prepare(lds_d, n_max, capD, bm));
    // the graph is keyed by every argument and buffer address it captures
    std::vector<unsigned char> key(sizeof(A) + sizeof(lpt) + 6 * sizeof(void *) + 16);
    {
        unsigned char *kp = key.data();
        memcpy(kp, &A, sizeof(A));
        kp += sizeof(A);
        memcpy(kp, &lpt, sizeof(lpt));
        kp += sizeof(lpt);
        const void *ptrs[6] = {out->birth, out->death, out->birth_simplex, out->death_simplex,
                               out->bar_offsets, (void *)(intptr_t)grid};
        memcpy(kp, ptrs, sizeof(ptrs));
        kp += sizeof(ptrs);
        memcpy(kp, &out->cap, 8);
        memcpy(kp + 8, &lds_d, 1);
    }
    if (!C->batch_exec || C->batch_key != key) {
        if (C->batch_exec) {
            (void)hipGraphExecDestroy(C->batch_exec);
            C->batch_exec = nullptr;
        }
        // tables are built outside the graph (they depend only on n_max, p)
        launch_binom((u64 *)A.binom.t, A.binom.stride, n_max, 3, st);
        launch_inverse(inv, p, st);
        HIP_TRY(hipStreamSynchronize(st));
        hipGraph_t graph;
        HIP_TRY(hipStreamBeginCapture(C->capture_stream, hipStreamCaptureModeThreadLocal));
        launch_batched(A, lds_d, grid, lpt, C->capture_stream);
        launch_batch_finalize(A, out->bar_offsets, &bs->total, out->cap, out->birth, out->death,
                              out->birth_simplex, out->death_simplex, C->capture_stream);
        HIP_TRY(hipStreamEndCapture(C->capture_stream, &graph));
        hipError_t e = hipGraphInstantiate(&C->batch_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            C->batch_exec = nullptr;
            return fail(RIPS_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        C->batch_key = key;
    }
    {
        PROF(P_BATCHED);
        HIP_TRY(hipGraphLaunch(C->batch_exec, st));
    }
    struct {
        int64_t total;
        int status;
    } hs;
    HIP_TRY(hipMemcpyAsync(&hs.total, &bs->total, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hs.status, &bs->status, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    prof_resolve();
    out->needed = hs.total;
    if (hs.status & 16) return fail(RIPS_E_INVALID_ARG, "a cloud is empty or larger than n_max");
    if (hs.status & 4) return fail(RIPS_E_NONFINITE, "input holds NaN/Inf");
    if (hs.status & 2) {
        // column store too small for some cloud: grow and run again
        C->batch_vstride = v_stride * 4;
        if (C->batch_vstride > (1ll << 26)) return fail(RIPS_E_CAPACITY, "column store overflow");
        *retry = true;
        return RIPS_E_CAPACITY;
    }
    if (hs.status & 1) return fail(RIPS_E_HIP, "batched reduction: delta or sorted base overflow");
    if (hs.status & 32) {
        C->batch_fstride = f_stride * 4;
        if (C->batch_fstride > (1ll << 28)) return fail(RIPS_E_CAPACITY, "far list overflow");
        *retry = true;
        return RIPS_E_CAPACITY;
    }
    if (hs.status & 64) {
        C->batch_vwstride = vw_stride * 4;
        if (C->batch_vwstride > (1ll << 24)) return fail(RIPS_E_CAPACITY, "V table overflow");
        *retry = true;
        return RIPS_E_CAPACITY;
    }
    if (hs.status & 128) {
        C->batch_logstride = log_stride * 4;
        if (C->batch_logstride > (1ll << 20)) return fail(RIPS_E_CAPACITY, "addition log overflow");
        *retry = true;
        return RIPS_E_CAPACITY;
    }
    if (hs.status & 8) return fail(RIPS_E_HIP, "batched reduction exceeded its addition bound");
    if (hs.total > out->cap) return fail(RIPS_E_CAPACITY, "bar capacity too small");
    return RIPS_OK;
}


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

// One cloud from device memory into the caller's device buffers, with the
// scratch of context C (the caller holds C's lock).
rips_status device_barcode(DevCtx *C, const float *d_data, int64_t n, int32_t dim, int32_t max_dim,
                           float threshold, uint32_t p, rips_device_out *out, hipStream_t st) {
    RunOut o;
    rips_status rs = run_single(*C, d_data, (int)n, dim, max_dim, threshold, p, st, o);
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
        PROF(P_EMIT);
        hipLaunchKernelGGL(k_set_nbars, dim3(1), dim3(1), 0, st, scal, o.count[d]);
        launch_emit(internal_bars(*C, d), scal, d > 0 ? 1 : 0, dst, st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    prof_resolve();
    return RIPS_OK;
}

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
    return device_barcode(C, d_data, n, dim, max_dim, threshold, p, out, (hipStream_t)hip_stream);
}

rips_status rips_barcode_device_noalloc(const float *d_data, int64_t n, int32_t dim, int32_t max_dim,
                                        float threshold, uint32_t p, rips_device_out *out,
                                        void *hip_stream) {
    g_err.clear();
    if (!d_data || !out) return fail(RIPS_E_INVALID_ARG, "null pointer");
    rips_status rs = validate(n, dim, max_dim, threshold, p, 0);
    if (rs) return rs;
    if (n > RIPS_NOALLOC_MAX_POINTS)
        return fail(RIPS_E_INVALID_ARG, "no-allocation entry point: n must be <= " +
                                            std::to_string(RIPS_NOALLOC_MAX_POINTS));
    if (max_dim > RIPS_NOALLOC_MAX_DIM)
        return fail(RIPS_E_INVALID_ARG, "no-allocation entry point: max_dim must be <= " +
                                            std::to_string(RIPS_NOALLOC_MAX_DIM));
    DevCtx *C;
    if ((rs = get_ctx_noalloc(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->reset_arena();
    g_prof_quiet = true;
    rs = device_barcode(C, d_data, n, dim, max_dim, threshold, p, out, (hipStream_t)hip_stream);
    g_prof_quiet = false;
    if (rs != RIPS_OK && C->arena_full)
        return fail(RIPS_E_CAPACITY, "no-allocation entry point: the input needs more than the " +
                                         std::to_string(kNoAllocBytes >> 20) + " MiB of its scratch");
    return rs;
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

rips_status rips_barcode_homology(const float *data, int64_t n, int32_t dim, int32_t max_dim,
                                  float threshold, uint32_t p, rips_result **out) {
    g_err.clear();
    if (!out) return fail(RIPS_E_INVALID_ARG, "null out");
    *out = nullptr;
    if (!data) return fail(RIPS_E_INVALID_ARG, "null data");
    rips_status rs = validate(n, dim, max_dim, threshold, p, 0);
    if (rs) return rs;
    if (max_dim > 2) return fail(RIPS_E_INVALID_ARG, "the homology variant computes dimensions 0-2");
    DevCtx *C;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    hipStream_t st = nullptr;
    void *q;
    const size_t in_elems = dim > 0 ? (size_t)n * dim : (size_t)n * n;
    HIP_TRY(C->ensure(B_INPUT, in_elems * 4, &q));
    float *d_in = as<float>(q);
    HIP_TRY(hipMemcpyAsync(d_in, data, in_elems * 4, hipMemcpyHostToDevice, st));
    HomRun o;
    rs = run_homology(*C, d_in, (int)n, dim, max_dim, threshold, p, st, o);
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
        r->column_index[d] = (int64_t *)malloc(sizeof(int64_t));
        r->column_diam[d] = (float *)malloc(sizeof(float));
        if (!b.birth || !b.death || !b.birth_simplex || !b.death_simplex || !r->column_index[d] ||
            !r->column_diam[d]) {
            rips_result_free(r);
            return fail(RIPS_E_OOM, "host allocation");
        }
        if (c == 0) continue;
        // canonical order: sort by birth simplex (younger first, carrying
        // the bar's slot), then gather in reverse
        const BarBuf in = internal_bars(*C, d);
        Columns ci{in.bs, in.birth, nullptr, nullptr}, co;
        hipError_t e = hipSuccess;
        auto need = [&](int id, size_t bytes) -> void * {
            void *pp = nullptr;
            if (e == hipSuccess) e = C->ensure(id, bytes, &pp);
            return pp;
        };
        ci.j = (int *)need(B_HOM_PERM, (size_t)c * 4);
        ci.tapp = (uint8_t *)need(B_SURV_TAPP, (size_t)c);
        co.idx = (int64_t *)need(B_SURV_IDX, (size_t)c * 8);
        co.diam = (float *)need(B_SURV_DIAM, (size_t)c * 4);
        co.j = (int *)need(B_HOM_PERM2, (size_t)c * 4);
        co.tapp = (uint8_t *)need(B_HOM_TAPP, (size_t)c);
        SortBufs sb;
        sb.lo[0] = (u64 *)need(B_SORT_LO0, (size_t)c * 8);
        sb.lo[1] = (u64 *)need(B_SORT_LO1, (size_t)c * 8);
        sb.hi[0] = (u32 *)need(B_SORT_HI0, (size_t)c * 4);
        sb.hi[1] = (u32 *)need(B_SORT_HI1, (size_t)c * 4);
        sb.val[0] = (u32 *)need(B_SORT_V0, (size_t)c * 4);
        sb.val[1] = (u32 *)need(B_SORT_V1, (size_t)c * 4);
        char *sg = (char *)need(B_STAGE, (size_t)c * 24);
        if (e != hipSuccess) {
            rips_result_free(r);
            return fail(RIPS_E_OOM, "sort buffers");
        }
        launch_hom_iota(ci.j, c, st);
        hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, &scal->survivors, (unsigned long long)c);
        launch_sort_columns(ci, scal, sb, bytes_for((uint64_t)choose_i64(n, d + 1)), co, st);
        BarBuf dst{(float *)sg, (float *)(sg + c * 4), (int64_t *)(sg + c * 8), (int64_t *)(sg + c * 16)};
        launch_hom_gather(in, co.j, c, dst, st);
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
    *out = r;
    return RIPS_OK;
}

void rips_cocycles_free(rips_cocycles *c) {
    if (!c) return;
    free(c->birth);
    free(c->death);
    free(c->birth_simplex);
    free(c->death_simplex);
    free(c->offsets);
    free(c->simplex);
    free(c->coef);
    free(c);
}

rips_status rips_barcode_cocycles(const float *data, int64_t n, int32_t dim, int32_t d, float threshold,
                                  uint32_t p, rips_cocycles **out) {
    g_err.clear();
    if (!out) return fail(RIPS_E_INVALID_ARG, "null out");
    *out = nullptr;
    if (!data) return fail(RIPS_E_INVALID_ARG, "null data");
    if (d < 1) return fail(RIPS_E_INVALID_ARG, "cocycles are given for dimensions >= 1");
    rips_status rs = validate(n, dim, d, threshold, p, 0);
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
    C->cocycle_dim = d;
    rs = run_single(*C, d_in, (int)n, dim, d, threshold, p, st, o);
    C->cocycle_dim = -1;
    if (rs) return rs;
    // the bars of dimension d in the canonical order
    const int64_t c = o.count[d];
    std::vector<float> birth(c), death(c);
    std::vector<int64_t> bs(c), ds(c);
    if (c > 0) {
        HIP_TRY(C->ensure(B_STAGE, (size_t)c * 24, &q));
        char *sg = as<char>(q);
        BarBuf dst{(float *)sg, (float *)(sg + c * 4), (int64_t *)(sg + c * 8), (int64_t *)(sg + c * 16)};
        Scalars *scal = as<Scalars>(C->buf[B_SCAL]);
        hipLaunchKernelGGL(k_set_nbars, dim3(1), dim3(1), 0, st, scal, c);
        launch_emit(internal_bars(*C, d), scal, 1, dst, st);
        HIP_TRY(hipMemcpyAsync(birth.data(), dst.birth, c * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(death.data(), dst.death, c * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(bs.data(), dst.bs, c * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(ds.data(), dst.ds, c * 8, hipMemcpyDeviceToHost, st));
    }
    // the columns of dimension d (still resident: d is the last dimension
    // run) and the stored V_j of each
    const int64_t S = o.ncols[d];
    const int64_t nv = o.stats[d].entries_stored;
    std::vector<int64_t> cidx(S), voff(S), vidx(nv);
    std::vector<int> vlen(S);
    std::vector<u32> vcoef(nv);
    if (S > 0) {
        HIP_TRY(hipMemcpyAsync(cidx.data(), C->buf[B_COL_IDX + d], S * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(voff.data(), C->buf[B_V_OFF], S * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(vlen.data(), C->buf[B_V_LEN], S * 4, hipMemcpyDeviceToHost, st));
    }
    if (nv > 0) {
        HIP_TRY(hipMemcpyAsync(vidx.data(), C->buf[B_V_IDX], nv * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(vcoef.data(), C->buf[B_V_COEF], nv * 4, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    std::unordered_map<int64_t, int64_t> col_of;
    col_of.reserve((size_t)S * 2);
    for (int64_t j = 0; j < S; ++j) col_of[cidx[j]] = j;
    std::vector<int64_t> offs(c + 1, 0), simp;
    std::vector<u32> cf;
    for (int64_t b = 0; b < c; ++b) {
        auto it = col_of.find(bs[b]);
        if (it == col_of.end()) return fail(RIPS_E_HIP, "cocycles: a bar without a column");
        const int64_t j = it->second;
        if (vlen[j] < 0) {
            // emergent column: V_j is its own simplex
            simp.push_back(bs[b]);
            cf.push_back(1u);
        } else {
            if (voff[j] < 0 || voff[j] + vlen[j] > nv) return fail(RIPS_E_HIP, "cocycles: column store out of range");
            for (int e = 0; e < vlen[j]; ++e) {
                simp.push_back(vidx[voff[j] + e]);
                cf.push_back(vcoef[voff[j] + e] % p);
            }
        }
        offs[b + 1] = (int64_t)simp.size();
    }
    rips_cocycles *r = (rips_cocycles *)calloc(1, sizeof(rips_cocycles));
    if (!r) return fail(RIPS_E_OOM, "host allocation");
    const int64_t ne = (int64_t)simp.size();
    r->dim = d;
    r->count = c;
    r->birth = (float *)malloc(sizeof(float) * (c ? c : 1));
    r->death = (float *)malloc(sizeof(float) * (c ? c : 1));
    r->birth_simplex = (int64_t *)malloc(sizeof(int64_t) * (c ? c : 1));
    r->death_simplex = (int64_t *)malloc(sizeof(int64_t) * (c ? c : 1));
    r->offsets = (int64_t *)malloc(sizeof(int64_t) * (c + 1));
    r->simplex = (int64_t *)malloc(sizeof(int64_t) * (ne ? ne : 1));
    r->coef = (uint32_t *)malloc(sizeof(uint32_t) * (ne ? ne : 1));
    if (!r->birth || !r->death || !r->birth_simplex || !r->death_simplex || !r->offsets || !r->simplex ||
        !r->coef) {
        rips_cocycles_free(r);
        return fail(RIPS_E_OOM, "host allocation");
    }
    if (c) {
        memcpy(r->birth, birth.data(), c * 4);
        memcpy(r->death, death.data(), c * 4);
        memcpy(r->birth_simplex, bs.data(), c * 8);
        memcpy(r->death_simplex, ds.data(), c * 8);
    }
    memcpy(r->offsets, offs.data(), (c + 1) * 8);
    if (ne) {
        memcpy(r->simplex, simp.data(), ne * 8);
        memcpy(r->coef, cf.data(), ne * 4);
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

rips_status rips_barcode_batched_device(const float *d_points, const int64_t *d_offsets, int32_t B,
                                        int32_t dim, int32_t n_max, int32_t max_dim,
                                        float threshold, uint32_t p, rips_batch_out *out,
                                        void *hip_stream) {
    g_err.clear();
    if (!d_points || !d_offsets || !out || !out->bar_offsets)
        return fail(RIPS_E_INVALID_ARG, "null pointer");
    if (B < 1 || B > (1 << 24)) return fail(RIPS_E_INVALID_ARG, "B out of range");
    if (dim < 1) return fail(RIPS_E_INVALID_ARG, "batched clouds are point clouds (dim >= 1)");
    if (n_max < 1 || n_max > kBatchMaxN)
        return fail(RIPS_E_INVALID_ARG, "n_max must be in [1, 2048]");
    if (max_dim < 0 || max_dim > 1) return fail(RIPS_E_INVALID_ARG, "batched max_dim is 0 or 1");
    if (std::isnan(threshold)) return fail(RIPS_E_INVALID_ARG, "threshold is NaN");
    if (!is_prime_u32(p) || p >= 65536) return fail(RIPS_E_NOT_PRIME, "p must be a prime < 65536");
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    for (int attempt = 0;; ++attempt) {
        bool retry = false;
        rs = batched_once(*C, d_points, d_offsets, B, dim, n_max, max_dim, threshold, p, out,
                          hip_stream, &retry);
        if (!retry || attempt > 8) return rs;
    }
}

rips_status rips_backward_device(const float *d_data, int64_t n, int32_t dim, int64_t nbars,
                                 int32_t k_birth, const int64_t *d_row0,
                                 const int64_t *d_birth_simplex, const int64_t *d_death_simplex,
                                 const float *d_grad_birth, const float *d_grad_death,
                                 float *d_grad, void *hip_stream) {
    g_err.clear();
    if (n < 1 || n > RIPS_MAX_POINTS) return fail(RIPS_E_INVALID_ARG, "n out of range");
    if (dim < 0) return fail(RIPS_E_INVALID_ARG, "dim < 0");
    if (dim == 0 && d_row0) return fail(RIPS_E_INVALID_ARG, "distance input has one cloud");
    if (k_birth < 0 || k_birth > RIPS_MAX_DIM)
        return fail(RIPS_E_INVALID_ARG, "k_birth out of range");
    if (nbars < 0) return fail(RIPS_E_INVALID_ARG, "nbars < 0");
    if (nbars == 0) return RIPS_OK;
    if (!d_data || !d_birth_simplex || !d_death_simplex || !d_grad_birth || !d_grad_death ||
        !d_grad)
        return fail(RIPS_E_INVALID_ARG, "null pointer");
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const int jmax = kMaxDim + 2;
    const int stride = (int)n + 1;
    void *q;
    HIP_TRY(C->ensure(B_BW_BINOM, (size_t)(jmax + 1) * stride * 8, &q));
    Binom B{as<u64>(q), stride};
    launch_binom(as<u64>(q), stride, (int)n, jmax, st);
    launch_backward(d_data, dim, n, (int)n, B, nbars, k_birth, d_row0, d_birth_simplex,
                    d_death_simplex, d_grad_birth, d_grad_death, d_grad, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return RIPS_OK;
}

rips_status rips_set_reduce_workgroups(int32_t workgroups) {
    g_err.clear();
    if (workgroups < 0) return fail(RIPS_E_INVALID_ARG, "workgroups must be >= 0");
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->reduce_groups = workgroups;
    return RIPS_OK;
}

rips_status rips_get_reduce_workgroups(int32_t *workgroups) {
    g_err.clear();
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    if (workgroups) *workgroups = C->reduce_groups;
    return RIPS_OK;
}

rips_status rips_set_shortcuts(int32_t flags) {
    g_err.clear();
    if (flags < 0 || flags > (RIPS_SHORTCUT_APPARENT | RIPS_SHORTCUT_EMERGENT | RIPS_SHORTCUT_CLEARING))
        return fail(RIPS_E_INVALID_ARG, "unknown shortcut flags");
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->shortcuts = (flags & RIPS_SHORTCUT_APPARENT ? kShortApparent : 0) |
                   (flags & RIPS_SHORTCUT_EMERGENT ? kShortEmergent : 0) |
                   (flags & RIPS_SHORTCUT_CLEARING ? kShortClearing : 0);
    return RIPS_OK;
}

rips_status rips_set_reduced_storage(int32_t mode) {
    g_err.clear();
    if (mode != RIPS_R_AUTO && mode != RIPS_R_DISCARD && mode != RIPS_R_STORE && mode != RIPS_R_EXPLICIT)
        return fail(RIPS_E_INVALID_ARG, "unknown storage mode");
    DevCtx *C;
    rips_status rs = get_ctx(&C);
    if (rs) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->rstore = mode == RIPS_R_DISCARD    ? kRStoreNever
                : mode == RIPS_R_STORE    ? kRStoreAlways
                : mode == RIPS_R_EXPLICIT ? kRStoreExplicit
                                          : kRStoreAuto;
    return RIPS_OK;
}

rips_status rips_set_working_column(int32_t mode) {
    g_err.clear();
    if (mode != RIPS_WORKING_COLUMN_AUTO && mode != RIPS_WORKING_COLUMN_GENERAL)
        return fail(RIPS_E_INVALID_ARG, "unknown working-column mode");
    DevCtx *C;
    rips_status rs = get_ctx(&C);
    if (rs) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->working_column = mode;
    return RIPS_OK;
}

rips_status rips_get_working_column(int32_t *mode) {
    g_err.clear();
    if (!mode) return fail(RIPS_E_INVALID_ARG, "null mode");
    DevCtx *C;
    rips_status rs = get_ctx(&C);
    if (rs) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    *mode = C->working_column;
    return RIPS_OK;
}

rips_status rips_get_reduced_storage(int32_t *mode) {
    g_err.clear();
    if (!mode) return fail(RIPS_E_INVALID_ARG, "null mode");
    DevCtx *C;
    rips_status rs = get_ctx(&C);
    if (rs) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    *mode = C->rstore == kRStoreNever      ? RIPS_R_DISCARD
            : C->rstore == kRStoreAlways   ? RIPS_R_STORE
            : C->rstore == kRStoreExplicit ? RIPS_R_EXPLICIT
                                           : RIPS_R_AUTO;
    return RIPS_OK;
}

rips_status rips_get_shortcuts(int32_t *flags) {
    g_err.clear();
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    if (flags)
        *flags = (C->shortcuts & kShortApparent ? RIPS_SHORTCUT_APPARENT : 0) |
                 (C->shortcuts & kShortEmergent ? RIPS_SHORTCUT_EMERGENT : 0) |
                 (C->shortcuts & kShortClearing ? RIPS_SHORTCUT_CLEARING : 0);
    return RIPS_OK;
}

rips_status rips_batched_set_config(int32_t delta_slots, int32_t workgroups_per_cu) {
    g_err.clear();
    if (!(delta_slots == 0 || delta_slots == 512 || delta_slots == 1024 || delta_slots == 2048))
        return fail(RIPS_E_INVALID_ARG, "delta_slots must be 0, 512, 1024 or 2048");
    if (workgroups_per_cu < 0 || workgroups_per_cu > 4)
        return fail(RIPS_E_INVALID_ARG, "workgroups_per_cu must be in [0, 4]");
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->batch_capD = (u32)delta_slots;
    C->batch_wgpcu = workgroups_per_cu;
    return RIPS_OK;
}

rips_status rips_batched_set_spread(int32_t mode) {
    g_err.clear();
    if (mode != 0 && mode != 1) return fail(RIPS_E_INVALID_ARG, "spread mode is 0 (auto) or 1 (off)");
    DevCtx *C;
    rips_status rs = get_ctx(&C);
    if (rs) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    C->batch_spread_off = mode;
    return RIPS_OK;
}

rips_status rips_batched_get_config(int32_t *delta_slots, int32_t *workgroups_per_cu) {
    g_err.clear();
    DevCtx *C;
    rips_status rs;
    if ((rs = get_ctx(&C))) return rs;
    std::lock_guard<std::mutex> lk(C->mu);
    if (delta_slots) *delta_slots = (int32_t)C->batch_capD;
    if (workgroups_per_cu) *workgroups_per_cu = C->batch_wgpcu;
    return RIPS_OK;
}

rips_status rips_batched_autotune(const float *d_points, const int64_t *d_offsets, int32_t B,
                                  int32_t dim, int32_t n_max, int32_t max_dim, float threshold,
                                  uint32_t p, rips_batch_out *out, void *hip_stream, int32_t reps,
                                  int32_t *best_delta_slots, int32_t *best_workgroups_per_cu,
                                  float *best_ms) {
    g_err.clear();
    if (reps < 1 || reps > 1000) return fail(RIPS_E_INVALID_ARG, "reps must be in [1, 1000]");
    if (!out || !out->bar_offsets) return fail(RIPS_E_INVALID_ARG, "null pointer");
    const int32_t slots[3] = {512, 1024, 2048};
    const int32_t wgs[3] = {1, 2, 4};
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t noff = (int64_t)B * (max_dim + 1) + 1;
    std::vector<int64_t> ref, cur;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RIPS_E_HIP, "hipEventCreate failed");
    float best = -1.0f;
    int32_t bs = 0, bw = 0;
    rips_status rs = RIPS_OK;
    for (int a = 0; a < 3 && rs == RIPS_OK; ++a) {
        for (int b = 0; b < 3 && rs == RIPS_OK; ++b) {
            if ((rs = rips_batched_set_config(slots[a], wgs[b]))) break;
            // untimed run: builds the graph and grows scratch
            if ((rs = rips_barcode_batched_device(d_points, d_offsets, B, dim, n_max, max_dim,
                                                  threshold, p, out, hip_stream)))
                break;
            cur.resize(noff);
            if (hipMemcpy(cur.data(), out->bar_offsets, noff * 8, hipMemcpyDeviceToHost) !=
                hipSuccess) {
                rs = fail(RIPS_E_HIP, "copy of bar offsets failed");
                break;
            }
            if (ref.empty()) ref = cur;
            else if (ref != cur) {
                rs = fail(RIPS_E_HIP, "configurations disagree on the bar counts");
                break;
            }
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && rs == RIPS_OK; ++r)
                rs = rips_barcode_batched_device(d_points, d_offsets, B, dim, n_max, max_dim,
                                                 threshold, p, out, hip_stream);
            if (rs) break;
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)reps;
            if (best < 0.0f || ms < best) {
                best = ms;
                bs = slots[a];
                bw = wgs[b];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs) {
        const std::string err = g_err;
        (void)rips_batched_set_config(0, 0);
        g_err = err;
        return rs;
    }
    if ((rs = rips_batched_set_config(bs, bw))) return rs;
    if (best_delta_slots) *best_delta_slots = bs;
    if (best_workgroups_per_cu) *best_workgroups_per_cu = bw;
    if (best_ms) *best_ms = best;
    return RIPS_OK;
}

void rips_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.clear();
    g_prof.next = 0;
    if (on) {
        for (int i = 0; i < P_NUM; ++i) {
            g_prof.ms[i] = 0.0;
            g_prof.calls[i] = 0;
        }
    }
    g_prof.on = on != 0;
}

int rips_profile_count(void) { return P_NUM; }
const char *rips_profile_name(int i) { return prof_name(i); }
double rips_profile_ms(int i) { return (i >= 0 && i < P_NUM) ? g_prof.ms[i] : 0.0; }
int64_t rips_profile_calls(int i) { return (i >= 0 && i < P_NUM) ? g_prof.calls[i] : 0; }

} // extern "C"
