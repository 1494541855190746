// C-ABI of the DMS library: context, buffers, stage orchestration.
// Declarations and the contract of every entry point are in include/dms.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dms.h"
#include "dms_internal.h"
#include "d1.h"

using namespace dms;

namespace {

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

enum { EV_START = 0, EV_ORDER, EV_GK, EV_GRAD, EV_SORT, EV_D02, EV_D1, EV_OUT, NEV };

}  // namespace

struct dms_ctx {
    int device = 0;
    hipStream_t st = nullptr;
    // a second stream of the context's own (default priority) and the events
    // that fork D0 onto it and join it back: D0 and D2 run concurrently
    hipStream_t st2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t budget = 0;
    size_t used = 0;
    std::string err;
    GridDev g{};
    int bpr = 1;
    int stage = 0;  // 0: nothing, 1: gradient, 2: D0/D2, 3: D1
    bool batched = false;  // the last run was a batch (super-grid ids)
    bool flat = false;     // the last grid was 2D (nz = 1)
    int64_t ncrit[4] = {0, 0, 0, 0};
    uint32_t cap[4] = {0, 0, 0, 0};
    Buf rank, keysA, keysB, valsA, valsB, G, hist, part, flags, counters, stats;
    Buf keysA2, keysB2, valsA2, valsB2, hist2, part2;  // a second sort's scratch (concurrent critical sorts)
    Buf cid[4], ck[4];          // unsorted critical ids and their keys (CritLists)
    Buf csorted[4];             // ids sorted by the lexicographic order
    Buf cpos[4];                // cpos[d][i] = sorted position of cid[d][i] (d = 1, 2)
    uint32_t* order = nullptr;  // rank -> vertex (inside valsA / valsB)
    // D0 / D2
    Buf na0, nb0, owner0, bnd0, paired1, na2, nb2, owner2, bnd2, paired2, tet2pos, jump0, jump2;
    int64_t n_d0_pairs = 0, n_d2_pairs = 0;
    // D1
    D1State d1;
    bool opt_d1_small = false, opt_log = false;  // debug options (dms_set_option)
    bool opt_no_sandwich = false, opt_no_cache = false;  // ablation variants of D1 (dms_set_option)
    int64_t opt_heap_keys = 0;  // debug: D1's first publication heap, in keys (0: default sizing)
    bool virtual_max = true;  // DMS_VIRTUAL_MAX of the last gradient call (Sec. 5.2)
    // output staging
    Buf ob, od, okey, ocnt;
    // gradient scatter
    Buf gk0, gk1, gv0, gv1, ghist, gpart, gflag;
    // batching: super field, owner map, slot table, super pairs, demux scratch
    Buf bfield, bowner, bslots, bpairs[3], bkey, bdeath, bitem, bkept;
    BatchLayout blayout;
    // captured order + gradient stage per (super grid, buffer generation, caps)
    struct GraphEntry {
        int X, Y, Z;
        std::vector<const void*> sig;  // every buffer the captured kernels touch
        uint32_t cap[4];
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    int64_t binfo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipEvent_t ev[NEV] = {};
    bool ev_ok[NEV] = {};
    float ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace {

int fail(dms_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ctx, DMS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int ensure(dms_ctx* ctx, Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return DMS_OK;
    size_t want = bytes + bytes / 8;
    const size_t held = ctx->used + ctx->d1.bytes;  // the context's buffers and D1's
    if (ctx->budget && held - b.cap + want > ctx->budget) {
        want = bytes;
        if (held - b.cap + want > ctx->budget)
            return fail(ctx, DMS_E_NOMEM, "HBM budget exceeded (" + std::to_string(held - b.cap + want) +
                                              " > " + std::to_string(ctx->budget) + " bytes)");
    }
    if (b.p) {
        hipError_t e = hipFree(b.p);
        (void)e;
        ctx->used -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, DMS_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    b.cap = want;
    ctx->used += want;
    return DMS_OK;
}

#define ENSURE(buf, bytes)                                   \
    do {                                                     \
        int r_ = ensure(ctx, (buf), (size_t)(bytes));        \
        if (r_ != DMS_OK) return r_;                         \
    } while (0)

template <typename T>
T* P(Buf& b) {
    return (T*)b.p;
}

void record(dms_ctx* ctx, int i) {
    if (hipEventRecord(ctx->ev[i], ctx->st) == hipSuccess) ctx->ev_ok[i] = true;
}

int bits_for(uint64_t v) {
    int b = 1;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

// ---- output assembly kernels ------------------------------------------------
constexpr int OB = 256;
inline unsigned nb_of(int64_t n) { return (unsigned)((n + OB - 1) / OB); }

// D0: paired column j -> (vertex of dying minimum, edge); unowned minima ->
// infinite classes (key bit 32 set so that they sort last).
constexpr int EMIT_ITEMS = 16;  // items per lane of the emit kernels: one list atomic per 4096 items
inline unsigned nb_emit(int64_t n) { return (unsigned)((n + OB * EMIT_ITEMS - 1) / (OB * EMIT_ITEMS)); }

__global__ __launch_bounds__(OB) void k_emit_d0(const uint64_t* bnd, const uint8_t* paired, const uint32_t* order,
                                                const uint32_t* c1, int64_t m1, const uint32_t* c0,
                                                const uint32_t* rank, const uint32_t* owner0, int64_t m0,
                                                uint64_t* key, uint32_t* death, uint32_t* cnt) {
    const int64_t first = (int64_t)blockIdx.x * OB * EMIT_ITEMS;
    block_append<OB, EMIT_ITEMS>(
        cnt, first, m1, [&](int64_t i, uint64_t& p) {
            if (!paired[i]) return false;
            p = bnd[i] >> 32;
            return true;
        },
        [&](int64_t i, uint64_t p, uint32_t at) {
            key[at] = order[(uint32_t)p];
            death[at] = c1[i];
        });
    block_append<OB, EMIT_ITEMS>(
        cnt, first, m0,
        [&](int64_t i, uint64_t& p) {
            p = c0[i];
            return owner0[rank[p]] == EMPTY32;
        },
        [&](int64_t, uint64_t p, uint32_t at) {
            key[at] = (1ull << 32) | p;
            death[at] = EMPTY32;
        });
}

// D2: paired column j (decreasing triangles) -> (triangle, tet of the pivot age).
__global__ __launch_bounds__(OB) void k_emit_d2(const uint64_t* bnd, const uint8_t* paired, const uint32_t* c2,
                                                int64_t m2, const uint32_t* c3, int64_t m3, uint64_t* key,
                                                uint32_t* death, uint32_t* cnt) {
    block_append<OB, EMIT_ITEMS>(
        cnt, (int64_t)blockIdx.x * OB * EMIT_ITEMS, m2, [&](int64_t j, uint64_t&) { return paired[j] != 0; },
        [&](int64_t j, uint64_t, uint32_t at) {
            const uint32_t pos = (uint32_t)(bnd[j] >> 32);  // 1 = highest maximum
            key[at] = c2[m2 - 1 - j];
            death[at] = c3[m3 - pos];
        });
}

// 2D, D1: paired column j (decreasing edges) -> (edge, triangle of the pivot
// age); then the edges paired neither here nor in D0 (infinite classes)
__global__ __launch_bounds__(OB) void k_emit_flat1(const uint64_t* bnd, const uint8_t* paired, const uint32_t* c1,
                                                   int64_t m1, const uint32_t* c2, int64_t m2,
                                                   const uint8_t* paired0, uint64_t* key, uint32_t* death,
                                                   uint32_t* cnt) {
    const int64_t first = (int64_t)blockIdx.x * OB * EMIT_ITEMS;
    block_append<OB, EMIT_ITEMS>(
        cnt, first, m1, [&](int64_t j, uint64_t&) { return paired[j] != 0; },
        [&](int64_t j, uint64_t, uint32_t at) {
            const uint32_t pos = (uint32_t)(bnd[j] >> 32);  // 1 = highest maximum
            key[at] = c1[m1 - 1 - j];
            death[at] = c2[m2 - pos];
        });
    block_append<OB, EMIT_ITEMS>(
        cnt, first, m1, [&](int64_t i, uint64_t&) { return !paired0[i] && !paired[m1 - 1 - i]; },
        [&](int64_t i, uint64_t, uint32_t at) {
            key[at] = (1ull << 32) | c1[i];
            death[at] = EMPTY32;
        });
}

// 2D, D2: maxima no saddle killed (none with the virtual maximum on)
__global__ __launch_bounds__(OB) void k_emit_flat2(const uint32_t* owner, const uint32_t* c2, int64_t m2,
                                                   uint64_t* key, uint32_t* death, uint32_t* cnt) {
    block_append<OB, EMIT_ITEMS>(
        cnt, (int64_t)blockIdx.x * OB * EMIT_ITEMS, m2,
        [&](int64_t i, uint64_t&) { return owner[m2 - i] == EMPTY32; },  // position m2 - i is c2[i]
        [&](int64_t i, uint64_t, uint32_t at) {
            key[at] = (1ull << 32) | c2[i];
            death[at] = EMPTY32;
        });
}

__device__ inline int64_t max_vertex_of(const GridDev& g, const uint32_t* rank, int dim, int64_t id) {
    const int64_t a = id / ntypes(dim);
    const int t = (int)(id % ntypes(dim));
    int st[3] = {0, 0, 0};
    if (dim == 1) st[0] = t + 1;
    if (dim == 2) { st[0] = tri_step(t, 0); st[1] = tri_step(t, 1); }
    if (dim == 3) { st[0] = tet_step(t, 0); st[1] = tet_step(t, 1); st[2] = tet_step(t, 2); }
    int64_t v = a, best = a;
    for (int s = 0; s < dim; ++s) {
        v += lin_of_mask(g, st[s]);
        if (rank[v] > rank[best]) best = v;
    }
    return best;
}

__global__ void k_write_pairs(const uint64_t* key_sorted, const uint32_t* idx, const uint32_t* death, int64_t n,
                              dms_pair* out, int64_t* bv, int64_t* dv, float* bval, float* dval, GridDev g,
                              const uint32_t* rank, const float* field, float fmax_dummy, int dim,
                              const uint32_t* order) {
    const int64_t i = (int64_t)blockIdx.x * OB + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = key_sorted[i];
    const int64_t b = (int64_t)(k & 0xFFFFFFFFull);
    const uint32_t d = death[idx[i]];
    const int64_t dd = d == EMPTY32 ? -1 : (int64_t)d;
    out[i].birth = b;
    out[i].death = dd;
    if (bv || bval) {
        const int64_t v = max_vertex_of(g, rank, dim, b);
        if (bv) bv[i] = v;
        if (bval) bval[i] = field[v];
    }
    if (dv || dval) {
        const int64_t v = dd < 0 ? -1 : max_vertex_of(g, rank, dim + 1, dd);
        if (dv) dv[i] = v;
        if (dval) dval[i] = v < 0 ? field[order[g.V - 1]] : field[v];
    }
    (void)fmax_dummy;
}

}  // namespace

// ---- internal helpers used by the entry points --------------------------------

// the context's second stream and the events that fork work onto it and join it back
static int ensure_second_stream(dms_ctx* ctx) {
    if (ctx->st2) return DMS_OK;
    HIPCHK(hipStreamCreateWithFlags(&ctx->st2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    return DMS_OK;
}

// the scratch of one sort: keys, values (double-buffered), tile histograms, scan partials
struct SortScratch {
    Buf *keysA, *keysB, *valsA, *valsB, *hist, *part;
};

static int sort_scratch(dms_ctx* ctx, const SortScratch& S, int64_t m) {
    ENSURE(*S.keysA, 8 * m);
    ENSURE(*S.keysB, 8 * m);
    ENSURE(*S.valsA, 4 * m);
    ENSURE(*S.valsB, 4 * m);
    ENSURE(*S.hist, 4 * 256 * sort_tiles(m));
    ENSURE(*S.part, 4 * scan_part_size(256 * sort_tiles(m)));
    return DMS_OK;
}

// sort C_d by the lexicographic order on stream st with scratch S (sized
// beforehand with sort_scratch)
static int sort_ids_on(dms_ctx* ctx, int d, hipStream_t st, const SortScratch& S) {
    const int64_t m = ctx->ncrit[d];
    if (m == 0) return DMS_OK;
    uint32_t* hist = P<uint32_t>(*S.hist);
    uint32_t* part = P<uint32_t>(*S.part);
    const int bpr = ctx->bpr;
    uint32_t* perm = nullptr;
    if (d == 0) {
        int r = radix_sort_pairs<uint32_t>(P<uint32_t>(ctx->ck[0]), P<uint32_t>(*S.valsA), P<uint32_t>(*S.keysA),
                                           P<uint32_t>(*S.valsB), m, 0, bpr, true, hist, part, st);
        perm = r ? P<uint32_t>(*S.valsB) : P<uint32_t>(*S.valsA);
    } else {
        // rank of the highest vertex, then 4-bit labels of the others (CritLists)
        int r = radix_sort_pairs<uint64_t>(P<uint64_t>(ctx->ck[d]), P<uint32_t>(*S.valsA), P<uint64_t>(*S.keysA),
                                           P<uint32_t>(*S.valsB), m, 0, bpr + 4 * d, true, hist, part, st);
        perm = r ? P<uint32_t>(*S.valsB) : P<uint32_t>(*S.valsA);
    }
    gather_u32(P<uint32_t>(ctx->cid[d]), perm, P<uint32_t>(ctx->csorted[d]), m, st);
    if (d == 1 || d == 2) inverse_perm(perm, m, P<uint32_t>(ctx->cpos[d]), st);
    return DMS_OK;
}

// Sort emitted (key, death) pairs by key and write them out.
static int finish_pairs(dms_ctx* ctx, int dim, int64_t n, dms_pair* out, int64_t* bv, int64_t* dv, float* bval,
                        float* dval, const float* field) {
    hipStream_t st = ctx->st;
    if (n == 0) return DMS_OK;
    ENSURE(ctx->hist, 4 * 256 * sort_tiles(n));
    ENSURE(ctx->part, 4 * scan_part_size(256 * sort_tiles(n)));
    ENSURE(ctx->keysB, 8 * n);
    ENSURE(ctx->valsA, 4 * n);
    ENSURE(ctx->valsB, 4 * n);
    int r = radix_sort_pairs<uint64_t>(P<uint64_t>(ctx->okey), P<uint32_t>(ctx->valsA), P<uint64_t>(ctx->keysB),
                                       P<uint32_t>(ctx->valsB), n, 0, 40, true, P<uint32_t>(ctx->hist),
                                       P<uint32_t>(ctx->part), st);
    uint64_t* ks = r ? P<uint64_t>(ctx->keysB) : P<uint64_t>(ctx->okey);
    uint32_t* idx = r ? P<uint32_t>(ctx->valsB) : P<uint32_t>(ctx->valsA);
    hipLaunchKernelGGL(k_write_pairs, dim3(nb_of(n)), dim3(OB), 0, st, ks, idx, P<uint32_t>(ctx->od), n, out, bv, dv,
                       bval, dval, ctx->g, P<uint32_t>(ctx->rank), field, 0.0f, dim, ctx->order);
    return DMS_OK;
}

static int read_counter(dms_ctx* ctx, uint32_t* host) {
    HIPCHK(hipMemcpyAsync(host, ctx->ocnt.p, 4, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return DMS_OK;
}

static int check_flags(dms_ctx* ctx) {
    uint32_t f = 0;
    HIPCHK(hipMemcpyAsync(&f, ctx->flags.p, 4, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (f & FLAG_NAN) return fail(ctx, DMS_E_NAN, "the scalar field holds a NaN");
    if (f & FLAG_GUARD) return fail(ctx, DMS_E_INTERNAL, "a pairing loop exceeded its iteration bound");
    if (f & FLAG_HEAP) return fail(ctx, DMS_E_INTERNAL, "the D1 boundary heap overflowed");
    return DMS_OK;
}

extern "C" {

int dms_create(dms_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes) {
    if (!out) return DMS_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DMS_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return DMS_E_HIP;
    dms_ctx* ctx = new dms_ctx();
    ctx->device = device;
    ctx->st = (hipStream_t)hip_stream;
    ctx->budget = hbm_budget_bytes;
    for (int i = 0; i < NEV; ++i)
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            delete ctx;
            return DMS_E_HIP;
        }
    ctx->err.reserve(512);  // messages fit without a host allocation later
    if (noalloc_scratch_init(device) != 0) {  // address of this device's scatter scratch
        delete ctx;
        return DMS_E_HIP;
    }
    int r = ensure(ctx, ctx->flags, 64);
    if (r == DMS_OK) r = ensure(ctx, ctx->counters, 64);
    if (r == DMS_OK) r = ensure(ctx, ctx->stats, 64);
    if (r == DMS_OK) r = ensure(ctx, ctx->ocnt, 64);
    if (r != DMS_OK) {
        delete ctx;
        return r;
    }
    *out = ctx;
    return DMS_OK;
}

void dms_destroy(dms_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->st);
    Buf* all[] = {&ctx->rank, &ctx->keysA, &ctx->keysB, &ctx->valsA, &ctx->valsB, &ctx->G, &ctx->hist,
                  &ctx->part, &ctx->flags, &ctx->counters, &ctx->stats, &ctx->keysA2, &ctx->keysB2, &ctx->valsA2,
                  &ctx->valsB2, &ctx->hist2, &ctx->part2, &ctx->na0, &ctx->nb0, &ctx->owner0, &ctx->bnd0,
                  &ctx->paired1, &ctx->na2, &ctx->nb2, &ctx->owner2, &ctx->bnd2, &ctx->paired2, &ctx->tet2pos,
                  &ctx->jump0, &ctx->jump2, &ctx->ob, &ctx->od, &ctx->okey, &ctx->ocnt, &ctx->gk0, &ctx->gk1, &ctx->gv0, &ctx->gv1,
                  &ctx->ghist, &ctx->gpart, &ctx->gflag, &ctx->bfield, &ctx->bowner, &ctx->bslots, &ctx->bpairs[0],
                  &ctx->bpairs[1], &ctx->bpairs[2], &ctx->bkey, &ctx->bdeath, &ctx->bitem, &ctx->bkept};
    for (auto& e : ctx->graphs) (void)hipGraphExecDestroy(e.exec);
    for (Buf* b : all)
        if (b->p) (void)hipFree(b->p);
    for (int d = 0; d < 4; ++d) {
        if (ctx->cid[d].p) (void)hipFree(ctx->cid[d].p);
        if (ctx->ck[d].p) (void)hipFree(ctx->ck[d].p);
        if (ctx->csorted[d].p) (void)hipFree(ctx->csorted[d].p);
        if (ctx->cpos[d].p) (void)hipFree(ctx->cpos[d].p);
    }
    d1_free(ctx->d1);
    for (int i = 0; i < NEV; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->st2) {
        (void)hipStreamSynchronize(ctx->st2);
        (void)hipStreamDestroy(ctx->st2);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    delete ctx;
}

const char* dms_last_error(const dms_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

// ---- a0-a3 in three parts: buffers, the enqueued kernels (no host sync, no
// allocation, no memset: a hipGraph may capture them), and the count
// read-back with the critical sort ----

static int gradient_setup(dms_ctx* ctx, dms_grid grid) {
    const int64_t V = (int64_t)grid.nx * grid.ny * grid.nz;
    ctx->stage = 0;
    ctx->g.nx = grid.nx;
    ctx->g.ny = grid.ny;
    ctx->g.nz = grid.nz;
    ctx->g.V = V;
    ctx->g.sy = grid.nx;
    ctx->g.sz = (int64_t)grid.nx * grid.ny;
    ctx->bpr = bits_for((uint64_t)(V - 1));
    for (int i = 0; i < NEV; ++i) ctx->ev_ok[i] = false;
    ENSURE(ctx->rank, 4 * V);
    ENSURE(ctx->keysA, 8 * V);
    ENSURE(ctx->keysB, 8 * V);
    ENSURE(ctx->valsA, 4 * V);
    ENSURE(ctx->valsB, 4 * V);
    ENSURE(ctx->hist, 4 * 256 * sort_tiles(V));
    ENSURE(ctx->part, 4 * scan_part_size(256 * sort_tiles(V)));
    ENSURE(ctx->ob, 4 * V);
    ENSURE(ctx->G, (size_t)PLANES * V);
    for (int d = 0; d < 4; ++d) {
        if (ctx->cap[d] == 0)
            ctx->cap[d] = (uint32_t)std::min<int64_t>(V / (d == 0 || d == 3 ? 4 : 2) + 256, 0xF0000000ll);
        ENSURE(ctx->cid[d], 4ull * ctx->cap[d]);
        ENSURE(ctx->ck[d], (d == 0 ? 4ull : 8ull) * ctx->cap[d]);
    }
    ctx->order = P<uint32_t>(ctx->ob);
    return DMS_OK;
}

static void gradient_enqueue(dms_ctx* ctx, const float* d_field, const uint32_t* owner, bool events) {
    hipStream_t st = ctx->st;
    const int64_t V = ctx->g.V;
    fill_u32(P<uint32_t>(ctx->flags), 0, 16, st);
    if (events) record(ctx, EV_START);
    float_keys(d_field, owner, V, P<uint32_t>(ctx->keysA), P<uint32_t>(ctx->flags), st);
    int r = radix_sort_pairs<uint32_t>(P<uint32_t>(ctx->keysA), P<uint32_t>(ctx->valsA), P<uint32_t>(ctx->keysB),
                                       P<uint32_t>(ctx->valsB), V, 0, 32, true, P<uint32_t>(ctx->hist),
                                       P<uint32_t>(ctx->part), st);
    uint32_t* order = r ? P<uint32_t>(ctx->valsB) : P<uint32_t>(ctx->valsA);
    rank_scatter(order, V, P<uint32_t>(ctx->rank), st);
    if (events) record(ctx, EV_ORDER);
    // keep the order (rank -> vertex) in a buffer of its own
    (void)hipMemcpyAsync(ctx->ob.p, order, 4 * V, hipMemcpyDeviceToDevice, st);
    CritLists cl;
    cl.count = P<uint32_t>(ctx->counters);
    for (int d = 0; d < 4; ++d) cl.cap[d] = ctx->cap[d];
    cl.id0 = P<uint32_t>(ctx->cid[0]);
    cl.key0 = P<uint32_t>(ctx->ck[0]);
    cl.id1 = P<uint32_t>(ctx->cid[1]);
    cl.key1 = P<uint64_t>(ctx->ck[1]);
    cl.id2 = P<uint32_t>(ctx->cid[2]);
    cl.key2 = P<uint64_t>(ctx->ck[2]);
    cl.id3 = P<uint32_t>(ctx->cid[3]);
    cl.key3 = P<uint64_t>(ctx->ck[3]);
    fill_u32(P<uint32_t>(ctx->counters), 0, 4, st);
    if (events) record(ctx, EV_GK);
    launch_gradient(ctx->g, P<uint32_t>(ctx->rank), P<uint8_t>(ctx->G), ctx->bpr, cl, st);
    if (events) record(ctx, EV_GRAD);
}

// reads the counts; *over is set when a critical list overflowed (the caps
// are raised: set up and enqueue again)
static int gradient_counts(dms_ctx* ctx, bool* over) {
    hipStream_t st = ctx->st;
    uint32_t cnt[4];
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(cnt, ctx->counters.p, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *over = false;
    for (int d = 0; d < 4; ++d) {
        ctx->ncrit[d] = cnt[d];
        if (cnt[d] > ctx->cap[d]) {
            *over = true;
            ctx->cap[d] = cnt[d] + 256;
        }
    }
    return DMS_OK;
}

static int gradient_finish(dms_ctx* ctx, dms_gradient_info* info) {
    int r = check_flags(ctx);
    if (r != DMS_OK) return r;
    // ---- a3: sort critical simplices by the lexicographic order ----
    // Without an HBM budget the 2-saddles sort on the second stream, with a
    // scratch of their own, while the other lists sort on the main stream.
    const int64_t* m = ctx->ncrit;
    for (int d = 0; d < 4; ++d) {
        ENSURE(ctx->csorted[d], 4 * m[d]);
        if (d == 1 || d == 2) ENSURE(ctx->cpos[d], 4 * m[d]);
    }
    const bool two = ctx->budget == 0 && m[2] > 0;
    const SortScratch A{&ctx->keysA, &ctx->keysB, &ctx->valsA, &ctx->valsB, &ctx->hist, &ctx->part};
    const SortScratch B{&ctx->keysA2, &ctx->keysB2, &ctx->valsA2, &ctx->valsB2, &ctx->hist2, &ctx->part2};
    r = sort_scratch(ctx, A, std::max(std::max(m[0], m[1]), std::max(m[3], two ? (int64_t)0 : m[2])));
    if (r != DMS_OK) return r;
    if (two) {
        r = sort_scratch(ctx, B, m[2]);
        if (r == DMS_OK) r = ensure_second_stream(ctx);
        if (r != DMS_OK) return r;
        HIPCHK(hipEventRecord(ctx->ev_fork, ctx->st));
        HIPCHK(hipStreamWaitEvent(ctx->st2, ctx->ev_fork, 0));
        sort_ids_on(ctx, 2, ctx->st2, B);
    }
    for (int d = 0; d < 4; ++d)
        if (d != 2 || !two) sort_ids_on(ctx, d, ctx->st, A);
    if (two) {
        HIPCHK(hipEventRecord(ctx->ev_join, ctx->st2));
        HIPCHK(hipStreamWaitEvent(ctx->st, ctx->ev_join, 0));
    }
    record(ctx, EV_SORT);
    HIPCHK(hipStreamSynchronize(ctx->st));
    HIPCHK(hipGetLastError());
    if (info)
        for (int d = 0; d < 4; ++d) info->n_crit[d] = ctx->ncrit[d];
    ctx->stage = 1;
    return DMS_OK;
}

static int check_grid(dms_ctx* ctx, dms_grid grid, uint32_t flags) {
    if (grid.nx < 2 || grid.ny < 2 || grid.nz < 1)
        return fail(ctx, DMS_E_INVAL, "nx and ny must be >= 2 and nz >= 1 (nz = 1: a 2D grid)");
    const int64_t V = (int64_t)grid.nx * grid.ny * grid.nz;
    if (12 * V >= (int64_t)0xFFFFFFFFll) return fail(ctx, DMS_E_INVAL, "grid too large: 12*V must stay below 2^32");
    if (flags & ~(uint32_t)DMS_VIRTUAL_MAX) return fail(ctx, DMS_E_INVAL, "unknown flags");
    return DMS_OK;
}

int dms_gradient(dms_ctx* ctx, const float* d_field, dms_grid grid, uint32_t flags, dms_gradient_info* info) {
    if (!ctx) return DMS_E_INVAL;
    if (!d_field) return fail(ctx, DMS_E_INVAL, "d_field is NULL");
    int r = check_grid(ctx, grid, flags);
    if (r != DMS_OK) return r;
    HIPCHK(hipSetDevice(ctx->device));
    ctx->batched = false;
    ctx->flat = grid.nz == 1;
    ctx->virtual_max = (flags & DMS_VIRTUAL_MAX) != 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        r = gradient_setup(ctx, grid);
        if (r != DMS_OK) return r;
        gradient_enqueue(ctx, d_field, nullptr, true);
        bool over = false;
        r = gradient_counts(ctx, &over);
        if (r != DMS_OK) return r;
        if (!over) return gradient_finish(ctx, info);
    }
    return fail(ctx, DMS_E_INTERNAL, "critical list capacity");
}

static int run_d0_d2(dms_ctx* ctx) {
    hipStream_t st = ctx->st;
    const int64_t V = ctx->g.V;
    const int64_t m0 = ctx->ncrit[0], m1 = ctx->ncrit[1], m2 = ctx->ncrit[2], m3 = ctx->ncrit[3];
    HIPCHK(hipMemsetAsync(ctx->stats.p, 0, 64, st));
    unsigned long long* stats = P<unsigned long long>(ctx->stats);
    // work counters of the tracing and reduction kernels (bytes 32..63 of the counters)
    unsigned long long* next = P<unsigned long long>(ctx->counters) + 4;
    fill_u32(P<uint32_t>(ctx->counters) + 8, 0, 8, st);
    // D0 (Sec. 5.1)
    ENSURE(ctx->na0, 4 * m1);
    ENSURE(ctx->nb0, 4 * m1);
    ENSURE(ctx->owner0, 4 * V);
    ENSURE(ctx->bnd0, 8 * m1);
    ENSURE(ctx->paired1, m1);
    ENSURE(ctx->jump0, 8 * V);
    // In 3D, D0 and D2 only share read-only inputs and the error flags until
    // D1: D0 runs on the context's second stream, concurrently with D2 on the
    // main one (their tails and gathers overlap). Every buffer of both chains
    // is sized before the fork, so nothing is freed or allocated while the
    // second stream runs and no early return leaves it running.
    hipStream_t d0_st = st;
    if (!ctx->flat) {
        ENSURE(ctx->tet2pos, 4 * 6 * V);
        ENSURE(ctx->na2, 4 * m2);
        ENSURE(ctx->nb2, 4 * m2);
        ENSURE(ctx->owner2, 4 * (m3 + 1));
        ENSURE(ctx->bnd2, 8 * m2);
        ENSURE(ctx->paired2, m2);
        ENSURE(ctx->jump2, 8 * (m3 + 1));
        int r2 = ensure_second_stream(ctx);
        if (r2 != DMS_OK) return r2;
        HIPCHK(hipEventRecord(ctx->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(ctx->st2, ctx->ev_fork, 0));
        d0_st = ctx->st2;
    }
    trace_d0(ctx->g, P<uint8_t>(ctx->G), P<uint32_t>(ctx->rank), P<uint32_t>(ctx->cid[1]), P<uint32_t>(ctx->cpos[1]),
             m1, P<uint32_t>(ctx->na0), P<uint32_t>(ctx->nb0), P<uint32_t>(ctx->flags), next, d0_st);
    fill_u32(P<uint32_t>(ctx->owner0), EMPTY32, V, d0_st);
    fill_u64(P<uint64_t>(ctx->bnd0), EMPTY64, m1, d0_st);
    fill_u64(P<uint64_t>(ctx->jump0), EMPTY64, V, d0_st);
    reduce_pairs(P<uint32_t>(ctx->na0), P<uint32_t>(ctx->nb0), m1, P<uint32_t>(ctx->owner0), P<uint64_t>(ctx->bnd0),
                 P<uint64_t>(ctx->jump0), P<uint32_t>(ctx->flags), stats, next + 2, d0_st);
    settled_columns(P<uint64_t>(ctx->bnd0), P<uint32_t>(ctx->owner0), m1, P<uint8_t>(ctx->paired1), d0_st);
    if (ctx->flat) {
        // 2D: the maxima's diagram is D1, from the stable sets of the 1-saddles
        // (Sec. 5.2 one dimension down; no sandwich, Sec. 3); virtual maximum = age 0
        ENSURE(ctx->tet2pos, 4 * 2 * V);
        ENSURE(ctx->na2, 4 * m1);
        ENSURE(ctx->nb2, 4 * m1);
        ENSURE(ctx->owner2, 4 * (m2 + 1));
        ENSURE(ctx->bnd2, 8 * m1);
        ENSURE(ctx->paired2, m1);
        tri_positions_flat(P<uint32_t>(ctx->csorted[2]), m2, P<uint32_t>(ctx->tet2pos), st);
        trace_flat(ctx->g, P<uint8_t>(ctx->G), P<uint32_t>(ctx->tet2pos), P<uint32_t>(ctx->cid[1]),
                   P<uint32_t>(ctx->cpos[1]), m1, P<uint32_t>(ctx->na2), P<uint32_t>(ctx->nb2),
                   P<uint32_t>(ctx->flags), next + 1, st);
        ENSURE(ctx->jump2, 8 * (m2 + 1));
        fill_u32(P<uint32_t>(ctx->owner2), EMPTY32, m2 + 1, st);
        fill_u64(P<uint64_t>(ctx->bnd2), EMPTY64, m1, st);
        fill_u64(P<uint64_t>(ctx->jump2), EMPTY64, m2 + 1, st);
        reduce_pairs(P<uint32_t>(ctx->na2), P<uint32_t>(ctx->nb2), m1, P<uint32_t>(ctx->owner2),
                     P<uint64_t>(ctx->bnd2), P<uint64_t>(ctx->jump2), P<uint32_t>(ctx->flags), stats + 2, next + 3,
                     st, !ctx->virtual_max,
                     // without the virtual maximum a 1-saddle D0 paired could join two components
                     // here; it is the death of its D0 pair and is left out (with it, the rule
                     // leaves it out by itself)
                     ctx->virtual_max ? nullptr : P<uint8_t>(ctx->paired1));
        settled_columns(P<uint64_t>(ctx->bnd2), P<uint32_t>(ctx->owner2), m1, P<uint8_t>(ctx->paired2), st);
        (void)m3;
        return DMS_OK;
    }
    // D2 (Sec. 5.2), virtual maximum = age 0 (buffers sized before the fork)
    tet_positions(P<uint32_t>(ctx->csorted[3]), m3, P<uint32_t>(ctx->tet2pos), st);
    trace_d2(ctx->g, P<uint8_t>(ctx->G), P<uint32_t>(ctx->tet2pos), P<uint32_t>(ctx->cid[2]), P<uint32_t>(ctx->cpos[2]),
             m2, P<uint32_t>(ctx->na2), P<uint32_t>(ctx->nb2), P<uint32_t>(ctx->flags), next + 1, st);
    fill_u32(P<uint32_t>(ctx->owner2), EMPTY32, m3 + 1, st);
    fill_u64(P<uint64_t>(ctx->bnd2), EMPTY64, m2, st);
    fill_u64(P<uint64_t>(ctx->jump2), EMPTY64, m3 + 1, st);
    reduce_pairs(P<uint32_t>(ctx->na2), P<uint32_t>(ctx->nb2), m2, P<uint32_t>(ctx->owner2), P<uint64_t>(ctx->bnd2),
                 P<uint64_t>(ctx->jump2), P<uint32_t>(ctx->flags), stats + 2, next + 3, st, !ctx->virtual_max);
    settled_columns(P<uint64_t>(ctx->bnd2), P<uint32_t>(ctx->owner2), m2, P<uint8_t>(ctx->paired2), st);
    if (d0_st != st) {  // D1 needs D0: join the second stream
        HIPCHK(hipEventRecord(ctx->ev_join, d0_st));
        HIPCHK(hipStreamWaitEvent(st, ctx->ev_join, 0));
    }
    (void)m0;
    return DMS_OK;
}

static int emit_d0(dms_ctx* ctx, dms_pair* d0, int64_t cap0, int64_t* n0, int64_t* bv, int64_t* dv, float* bval,
                   float* dval, const float* field) {
    hipStream_t st = ctx->st;
    const int64_t m0 = ctx->ncrit[0], m1 = ctx->ncrit[1];
    const int64_t cap = m0 + 16;
    ENSURE(ctx->okey, 8 * cap);
    ENSURE(ctx->od, 4 * cap);
    HIPCHK(hipMemsetAsync(ctx->ocnt.p, 0, 4, st));
    const int64_t n = std::max(m0, m1);
    if (n > 0)
        hipLaunchKernelGGL(k_emit_d0, dim3(nb_emit(n)), dim3(OB), 0, st, P<uint64_t>(ctx->bnd0),
                           P<uint8_t>(ctx->paired1), ctx->order, P<uint32_t>(ctx->csorted[1]), m1,
                           P<uint32_t>(ctx->csorted[0]), P<uint32_t>(ctx->rank), P<uint32_t>(ctx->owner0), m0,
                           P<uint64_t>(ctx->okey), P<uint32_t>(ctx->od), P<uint32_t>(ctx->ocnt));
    uint32_t cnt = 0;
    int r = read_counter(ctx, &cnt);
    if (r != DMS_OK) return r;
    *n0 = cnt;
    if ((int64_t)cnt > cap0) return fail(ctx, DMS_E_CAPACITY, "D0 output buffer too small");
    return finish_pairs(ctx, 0, cnt, d0, bv, dv, bval, dval, field);
}

static int emit_d2(dms_ctx* ctx, dms_pair* d2, int64_t cap2, int64_t* n2, int64_t* bv, int64_t* dv, float* bval,
                   float* dval, const float* field, bool with_essential) {
    hipStream_t st = ctx->st;
    const int64_t m2 = ctx->ncrit[2], m3 = ctx->ncrit[3];
    const int64_t cap = m2 + 16;
    ENSURE(ctx->okey, 8 * cap);
    ENSURE(ctx->od, 4 * cap);
    HIPCHK(hipMemsetAsync(ctx->ocnt.p, 0, 4, st));
    if (ctx->flat) {
        if (m2 > 0)
            hipLaunchKernelGGL(k_emit_flat2, dim3(nb_emit(m2)), dim3(OB), 0, st, P<uint32_t>(ctx->owner2),
                               P<uint32_t>(ctx->csorted[2]), m2, P<uint64_t>(ctx->okey), P<uint32_t>(ctx->od),
                               P<uint32_t>(ctx->ocnt));
        with_essential = false;
    } else if (m2 > 0)
        hipLaunchKernelGGL(k_emit_d2, dim3(nb_emit(m2)), dim3(OB), 0, st, P<uint64_t>(ctx->bnd2),
                           P<uint8_t>(ctx->paired2), P<uint32_t>(ctx->csorted[2]), m2, P<uint32_t>(ctx->csorted[3]),
                           m3, P<uint64_t>(ctx->okey), P<uint32_t>(ctx->od), P<uint32_t>(ctx->ocnt));
    if (with_essential) d1_emit_essential2(ctx->d1, m2, P<uint8_t>(ctx->paired2), P<uint32_t>(ctx->csorted[2]),
                                           P<uint64_t>(ctx->okey), P<uint32_t>(ctx->od), P<uint32_t>(ctx->ocnt), st);
    uint32_t cnt = 0;
    int r = read_counter(ctx, &cnt);
    if (r != DMS_OK) return r;
    *n2 = cnt;
    if ((int64_t)cnt > cap2) return fail(ctx, DMS_E_CAPACITY, "D2 output buffer too small");
    return finish_pairs(ctx, 2, cnt, d2, bv, dv, bval, dval, field);
}

int dms_pairs_d0_d2(dms_ctx* ctx, dms_pair* d0, int64_t cap0, int64_t* n0, dms_pair* d2, int64_t cap2,
                    int64_t* n2) {
    if (!ctx) return DMS_E_INVAL;
    if (ctx->stage < 1) return fail(ctx, DMS_E_STATE, "dms_pairs_d0_d2 needs dms_gradient first");
    if (!n0 || !n2) return fail(ctx, DMS_E_INVAL, "n0 / n2 is NULL");
    HIPCHK(hipSetDevice(ctx->device));
    int r = run_d0_d2(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D02);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 2;
    int64_t a = 0, b = 0;
    int r0 = emit_d0(ctx, d0, cap0, &a, nullptr, nullptr, nullptr, nullptr, nullptr);
    *n0 = a;
    if (r0 != DMS_OK && r0 != DMS_E_CAPACITY) return r0;
    int r2 = emit_d2(ctx, d2, cap2, &b, nullptr, nullptr, nullptr, nullptr, nullptr, false);
    *n2 = b;
    if (r2 != DMS_OK && r2 != DMS_E_CAPACITY) return r2;
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (r0 == DMS_E_CAPACITY || r2 == DMS_E_CAPACITY) return fail(ctx, DMS_E_CAPACITY, "output buffer too small");
    return DMS_OK;
}

// device bytes D1 may hold under the context's budget (0 = no budget; at
// least 1, so that an exhausted budget still limits)
static size_t d1_limit(const dms_ctx* ctx) {
    if (!ctx->budget) return 0;
    return std::max<size_t>(1, ctx->budget - std::min(ctx->budget, ctx->used));
}

static int run_d1(dms_ctx* ctx) {
    if (ctx->flat) {  // 2D: D1 came from the dual tracing with D0 (no sandwich)
        ctx->d1.ncols = 0;
        ctx->d1.gen_n = -1;
        return DMS_OK;
    }
    // Without the virtual maximum, D2 from the dual union-find is not the
    // plain reduction's D2 (reading of Sec. 5.2 / App. A), so D1 over every
    // 2-saddle would give other pairs: the ablation is defined with it only.
    if (ctx->opt_no_sandwich && !ctx->virtual_max)
        return fail(ctx, DMS_E_INVAL, "DMS_OPT_D1_NO_SANDWICH needs DMS_VIRTUAL_MAX");
    D1Inputs in;
    in.g = ctx->g;
    in.G = P<uint8_t>(ctx->G);
    in.rank = P<uint32_t>(ctx->rank);
    in.order = ctx->order;
    in.c1 = P<uint32_t>(ctx->csorted[1]);
    in.m1 = ctx->ncrit[1];
    in.c2 = P<uint32_t>(ctx->csorted[2]);
    in.m2 = ctx->ncrit[2];
    in.paired1 = P<uint8_t>(ctx->paired1);
    in.paired2_desc = P<uint8_t>(ctx->paired2);
    in.bpr = ctx->bpr;
    in.flags = P<uint32_t>(ctx->flags);
    in.small_passes = ctx->opt_d1_small;
    in.log_passes = ctx->opt_log;
    in.no_sandwich = ctx->opt_no_sandwich;
    in.no_cache = ctx->opt_no_cache;
    in.heap_keys = ctx->opt_heap_keys;
    std::string err;
    int r = d1_run(ctx->d1, in, ctx->st, d1_limit(ctx), err);
    if (r != DMS_OK) return fail(ctx, r, err);
    return DMS_OK;
}

static int emit_d1(dms_ctx* ctx, dms_pair* d1, int64_t cap1, int64_t* n1, int64_t* bv, int64_t* dv, float* bval,
                   float* dval, const float* field) {
    hipStream_t st = ctx->st;
    const int64_t m1 = ctx->ncrit[1];
    const int64_t cap = m1 + 16;
    ENSURE(ctx->okey, 8 * cap);
    ENSURE(ctx->od, 4 * cap);
    HIPCHK(hipMemsetAsync(ctx->ocnt.p, 0, 4, st));
    if (ctx->flat) {
        if (m1 > 0)
            hipLaunchKernelGGL(k_emit_flat1, dim3(nb_emit(m1)), dim3(OB), 0, st, P<uint64_t>(ctx->bnd2),
                               P<uint8_t>(ctx->paired2), P<uint32_t>(ctx->csorted[1]), m1,
                               P<uint32_t>(ctx->csorted[2]), ctx->ncrit[2], P<uint8_t>(ctx->paired1),
                               P<uint64_t>(ctx->okey), P<uint32_t>(ctx->od), P<uint32_t>(ctx->ocnt));
    } else {
        d1_emit(ctx->d1, m1, P<uint8_t>(ctx->paired1), P<uint32_t>(ctx->csorted[1]), P<uint64_t>(ctx->okey),
                P<uint32_t>(ctx->od), P<uint32_t>(ctx->ocnt), st);
    }
    uint32_t cnt = 0;
    int r = read_counter(ctx, &cnt);
    if (r != DMS_OK) return r;
    *n1 = cnt;
    if ((int64_t)cnt > cap1) return fail(ctx, DMS_E_CAPACITY, "D1 output buffer too small");
    return finish_pairs(ctx, 1, cnt, d1, bv, dv, bval, dval, field);
}

int dms_pairs_d1(dms_ctx* ctx, dms_pair* d1, int64_t cap1, int64_t* n1) {
    if (!ctx) return DMS_E_INVAL;
    if (ctx->stage < 2) return fail(ctx, DMS_E_STATE, "dms_pairs_d1 needs dms_pairs_d0_d2 first");
    if (!n1) return fail(ctx, DMS_E_INVAL, "n1 is NULL");
    HIPCHK(hipSetDevice(ctx->device));
    int r = run_d1(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D1);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 3;
    r = emit_d1(ctx, d1, cap1, n1, nullptr, nullptr, nullptr, nullptr, nullptr);
    HIPCHK(hipStreamSynchronize(ctx->st));
    return r;
}

int dms_d1_generators(dms_ctx* ctx, int64_t* d_offsets, int64_t cap_offsets, int64_t* d_edges, int64_t cap_edges,
                      int64_t* n_pairs, int64_t* n_edges) {
    if (!ctx) return DMS_E_INVAL;
    if (!n_pairs || !n_edges) return fail(ctx, DMS_E_INVAL, "n_pairs or n_edges is NULL");
    if (cap_offsets < 0 || cap_edges < 0 || (cap_offsets > 0 && !d_offsets) || (cap_edges > 0 && !d_edges))
        return fail(ctx, DMS_E_INVAL, "an output buffer is NULL or a capacity is negative");
    if (ctx->stage < 3 || ctx->batched)
        return fail(ctx, DMS_E_STATE, "dms_d1_generators needs dms_pairs_d1 or dms_diagram on one field first");
    if (ctx->flat)
        return fail(ctx, DMS_E_STATE, "generators come from the sandwich of 3D grids; on a 2D grid D1 is dual");
    HIPCHK(hipSetDevice(ctx->device));
    std::string err;
    ctx->d1.limit = d1_limit(ctx);
    int r = d1_generators(ctx->d1, d_offsets, cap_offsets, d_edges, cap_edges, n_pairs, n_edges,
                          P<uint32_t>(ctx->flags), ctx->st, err);
    if (r < 0) return fail(ctx, r, err);
    if (r == 1) return fail(ctx, DMS_E_CAPACITY, "generator output buffers too small");
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    HIPCHK(hipGetLastError());
    return DMS_OK;
}

int dms_diagram(dms_ctx* ctx, const float* d_field, dms_grid grid, uint32_t flags, dms_diagram_out* out) {
    if (!ctx) return DMS_E_INVAL;
    if (!out) return fail(ctx, DMS_E_INVAL, "out is NULL");
    int r = dms_gradient(ctx, d_field, grid, flags, nullptr);
    if (r != DMS_OK) return r;
    r = run_d0_d2(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D02);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 2;
    r = run_d1(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D1);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 3;
    int64_t n[3] = {0, 0, 0};
    int rr[3];
    rr[0] = emit_d0(ctx, out->pairs[0], out->cap[0], &n[0], out->birth_vertex[0], out->death_vertex[0],
                    out->birth_value[0], out->death_value[0], d_field);
    rr[1] = emit_d1(ctx, out->pairs[1], out->cap[1], &n[1], out->birth_vertex[1], out->death_vertex[1],
                    out->birth_value[1], out->death_value[1], d_field);
    rr[2] = emit_d2(ctx, out->pairs[2], out->cap[2], &n[2], out->birth_vertex[2], out->death_vertex[2],
                    out->birth_value[2], out->death_value[2], d_field, true);
    record(ctx, EV_OUT);
    HIPCHK(hipStreamSynchronize(ctx->st));
    bool cap_fail = false;
    for (int d = 0; d < 3; ++d) {
        out->n[d] = n[d];
        if (rr[d] == DMS_E_CAPACITY) cap_fail = true;
        else if (rr[d] != DMS_OK) return rr[d];
    }
    if (cap_fail) return fail(ctx, DMS_E_CAPACITY, "an output buffer is too small; n[] holds the need");
    return DMS_OK;
}

// the tetrahedra of the gradient storage (by id) -> 6 planes indexed by anchor
__global__ void k_tet_planes(const uint8_t* __restrict__ by_id, int64_t V, uint8_t* __restrict__ planes) {
    const int64_t i = (int64_t)blockIdx.x * OB + threadIdx.x;
    if (i >= 6 * V) return;
    const int64_t type = i / V, anchor = i - type * V;
    planes[i] = by_id[anchor * 6 + type];
}

int64_t dms_debug_copy(dms_ctx* ctx, int what, void* dst, int64_t cap) {
    if (!ctx) return DMS_E_INVAL;
    const int64_t V = ctx->g.V;
    void* src = nullptr;
    int64_t bytes = 0;
    switch (what) {
        case DMS_BUF_RANK: src = ctx->rank.p; bytes = 4 * V; break;
        case DMS_BUF_GRADIENT: src = ctx->G.p; bytes = (int64_t)PLANES * V; break;
        case DMS_BUF_CRIT0: case DMS_BUF_CRIT1: case DMS_BUF_CRIT2: case DMS_BUF_CRIT3: {
            const int d = what - DMS_BUF_CRIT0;
            src = ctx->csorted[d].p;
            bytes = 4 * ctx->ncrit[d];
            break;
        }
        case DMS_BUF_ARCS0: bytes = 8 * ctx->ncrit[1]; break;
        case DMS_BUF_ARCS2: bytes = 8 * ctx->ncrit[ctx->flat ? 1 : 2]; break;  // 2D: the 1-saddles' dual arcs
        case DMS_BUF_STATS: {
            if (ctx->stage < 1) return fail(ctx, DMS_E_STATE, "no gradient computed yet");
            bytes = 8 * 48;
            if (!dst) return bytes;
            if (cap < bytes) return fail(ctx, DMS_E_CAPACITY, "destination too small");
            uint64_t* h = (uint64_t*)dst;
            std::memset(h, 0, bytes);
            HIPCHK(hipStreamSynchronize(ctx->st));
            HIPCHK(hipMemcpyAsync(h, ctx->stats.p, 32, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            for (int i = 0; i < 6; ++i) h[4 + i] = ctx->d1.stats[i];
            for (int i = 0; i < 5; ++i) {
                h[10 + 2 * i] = ctx->d1.pass_work[i];
                h[11 + 2 * i] = ctx->d1.pass_us[i];
            }
            for (int i = 0; i < 3; ++i) h[20 + i] = ctx->d1.wide[i];
            for (int i = 0; i < 6; ++i) h[23 + i] = ctx->d1.wide_t[i];
            for (int i = 0; i < 12; ++i) h[29 + i] = ctx->d1.wide_ph[i];
            h[41] = ctx->d1.wide[3];
            h[42] = ctx->d1.pass_work[5];
            h[43] = ctx->d1.pass_us[5];
            h[44] = ctx->d1.coop[0];
            h[45] = ctx->d1.coop[1];
            h[46] = ctx->d1.nc_fallbacks;
            return bytes;
        }
        case DMS_BUF_D1LEN: {
            if (ctx->stage < 3) return fail(ctx, DMS_E_STATE, "no D1 computed yet");
            bytes = 8 * ctx->d1.ncols;
            if (!dst) return bytes;
            if (cap < bytes) return fail(ctx, DMS_E_CAPACITY, "destination too small");
            HIPCHK(hipStreamSynchronize(ctx->st));
            if (bytes) HIPCHK(hipMemcpyAsync(dst, ctx->d1.bndptr, bytes, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            return bytes;
        }
        default: return fail(ctx, DMS_E_INVAL, "unknown buffer");
    }
    if (ctx->stage < 1) return fail(ctx, DMS_E_STATE, "no gradient computed yet");
    if (!dst) return bytes;
    if (cap < bytes) return fail(ctx, DMS_E_CAPACITY, "destination too small");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (what == DMS_BUF_ARCS0 || what == DMS_BUF_ARCS2) {
        if (ctx->stage < 2) return fail(ctx, DMS_E_STATE, "no D0/D2 computed yet");
        const int64_t m = bytes / 8;
        uint32_t* h = (uint32_t*)dst;
        Buf& a = what == DMS_BUF_ARCS0 ? ctx->na0 : ctx->na2;
        Buf& b = what == DMS_BUF_ARCS0 ? ctx->nb0 : ctx->nb2;
        if (m) {
            HIPCHK(hipMemcpyAsync(h, a.p, 4 * m, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipMemcpyAsync(h + m, b.p, 4 * m, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
        }
        return bytes;
    }
    if (what == DMS_BUF_GRADIENT && V > 0) {  // the tetrahedra go out as planes, like the rest
        ENSURE(ctx->keysB, 6 * V);
        hipLaunchKernelGGL(k_tet_planes, dim3(nb_of(6 * V)), dim3(OB), 0, ctx->st, P<uint8_t>(ctx->G) + 20 * V, V,
                           P<uint8_t>(ctx->keysB));
        HIPCHK(hipMemcpyAsync(dst, src, 20 * V, hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipMemcpyAsync((uint8_t*)dst + 20 * V, ctx->keysB.p, 6 * V, hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        return bytes;
    }
    if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return bytes;
}

int dms_scatter_grad(dms_ctx* ctx, int64_t n, const int64_t* d_vertex, const float* d_grad, int64_t nvert,
                     float* d_grad_field) {
    if (!ctx) return DMS_E_INVAL;
    if (n < 0 || nvert < 1 || nvert > ((int64_t)1 << 32) || !d_grad_field || (n > 0 && (!d_vertex || !d_grad)))
        return fail(ctx, DMS_E_INVAL, "dms_scatter_grad: bad sizes or null pointers");
    if (n > ((int64_t)1 << 32) - 1) return fail(ctx, DMS_E_INVAL, "dms_scatter_grad: too many contributions");
    HIPCHK(hipSetDevice(ctx->device));
    int r = DMS_OK;
    const int64_t m = n > 0 ? n : 1;
    if ((r = ensure(ctx, ctx->gk0, 4 * m)) || (r = ensure(ctx, ctx->gk1, 4 * m)) || (r = ensure(ctx, ctx->gv0, 4 * m)) ||
        (r = ensure(ctx, ctx->gv1, 4 * m)) || (r = ensure(ctx, ctx->ghist, 4 * 256 * sort_tiles(m))) ||
        (r = ensure(ctx, ctx->gpart, 4 * scan_part_size(256 * sort_tiles(m)))) || (r = ensure(ctx, ctx->gflag, 64)))
        return r;
    uint32_t* flag = P<uint32_t>(ctx->gflag);
    fill_u32(flag, 0, 1, ctx->st);
    scatter_grad(d_vertex, d_grad, n, nvert, d_grad_field, P<uint32_t>(ctx->gk0), P<uint32_t>(ctx->gv0),
                 P<uint32_t>(ctx->gk1), P<uint32_t>(ctx->gv1), P<uint32_t>(ctx->ghist), P<uint32_t>(ctx->gpart), flag,
                 ctx->st);
    HIPCHK(hipGetLastError());
    uint32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (h) return fail(ctx, DMS_E_INVAL, "dms_scatter_grad: vertex index out of range (gradient left zero there)");
    return DMS_OK;
}

// The error messages below fit the capacity reserved at dms_create, so
// reporting an error allocates nothing either.
static int fail_noalloc(dms_ctx* ctx, int code, const char* msg) {
    ctx->err.assign(msg);
    return code;
}

int dms_scatter_grad_noalloc(dms_ctx* ctx, int64_t n, const int64_t* d_vertex, const float* d_grad, int64_t nvert,
                             float* d_grad_field) {
    if (!ctx) return DMS_E_INVAL;
    if (n < 0 || nvert < 1 || nvert > ((int64_t)1 << 32) || !d_grad_field || (n > 0 && (!d_vertex || !d_grad)))
        return fail_noalloc(ctx, DMS_E_INVAL, "dms_scatter_grad_noalloc: bad sizes or null pointers");
    if (n > NOALLOC_MAX_CONTRIB)
        return fail_noalloc(ctx, DMS_E_INVAL,
                            "dms_scatter_grad_noalloc: more than 4194304 contributions (use dms_scatter_grad)");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail_noalloc(ctx, DMS_E_HIP, "hipSetDevice failed");
    uint32_t* flag = nullptr;
    if (scatter_grad_noalloc(ctx->device, d_vertex, d_grad, n, nvert, d_grad_field, &flag, ctx->st) != 0)
        return fail_noalloc(ctx, DMS_E_STATE, "dms_scatter_grad_noalloc: scratch of this device not set up");
    if (hipGetLastError() != hipSuccess) return fail_noalloc(ctx, DMS_E_HIP, "dms_scatter_grad_noalloc: launch failed");
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, ctx->st) != hipSuccess ||
        hipStreamSynchronize(ctx->st) != hipSuccess)
        return fail_noalloc(ctx, DMS_E_HIP, "dms_scatter_grad_noalloc: read-back failed");
    if (h)
        return fail_noalloc(ctx, DMS_E_INVAL,
                            "dms_scatter_grad_noalloc: vertex index out of range (gradient left zero there)");
    return DMS_OK;
}

static int batch_layout(dms_ctx* ctx, const dms_item* items, int32_t nitems, const dms_batch_opts* opts,
                        BatchLayout& L) {
    if (!items || nitems < 1) return fail(ctx, DMS_E_INVAL, "dms batch: no items");
    std::vector<int32_t> dims(3 * (size_t)nitems);
    int mx = 0, my = 0;
    for (int i = 0; i < nitems; ++i) {
        dims[3 * i] = items[i].nx;
        dims[3 * i + 1] = items[i].ny;
        dims[3 * i + 2] = items[i].nz;
        mx = std::max(mx, items[i].nx);
        my = std::max(my, items[i].ny);
    }
    int X = opts && opts->cross_x > 0 ? opts->cross_x : (mx + 1 + 15) / 16 * 16;
    int Y = opts && opts->cross_y > 0 ? opts->cross_y : (my + 1 + 15) / 16 * 16;
    const int zq = opts && opts->z_quantum > 0 ? opts->z_quantum : 16;
    std::string err;
    if (pack_layers(dims.data(), nitems, X, Y, zq, L, err)) return fail(ctx, DMS_E_INVAL, "dms batch: " + err);
    return DMS_OK;
}

int dms_batch_layout(const dms_item* items, int32_t nitems, const dms_batch_opts* opts, int32_t dims[3],
                     int32_t* origins) {
    if (!dims) return DMS_E_INVAL;
    BatchLayout L;
    const int r = batch_layout(nullptr, items, nitems, opts, L);
    if (r != DMS_OK) return r;
    dims[0] = L.X;
    dims[1] = L.Y;
    dims[2] = L.Z;
    if (origins)
        for (int i = 0; i < nitems; ++i) {
            origins[3 * i] = L.slots[i].ox;
            origins[3 * i + 1] = L.slots[i].oy;
            origins[3 * i + 2] = L.slots[i].oz;
        }
    return DMS_OK;
}

int dms_diagram_batch(dms_ctx* ctx, const float* d_fields, const dms_item* items, int32_t nitems, uint32_t flags,
                      const dms_batch_opts* opts, dms_batch_out* out) {
    if (!ctx) return DMS_E_INVAL;
    if (!d_fields || !out) return fail(ctx, DMS_E_INVAL, "dms_diagram_batch: NULL fields or output");
    for (int d = 0; d < 3; ++d)
        if (!out->item_start[d] || (out->cap[d] > 0 && !out->pairs[d]))
            return fail(ctx, DMS_E_INVAL, "dms_diagram_batch: NULL output array");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->st;
    BatchLayout& L = ctx->blayout;
    int r = batch_layout(ctx, items, nitems, opts, L);
    if (r != DMS_OK) return r;
    int64_t real = 0;
    for (int i = 0; i < nitems; ++i) {
        if (items[i].offset < 0) return fail(ctx, DMS_E_INVAL, "dms_diagram_batch: negative field offset");
        L.slots[i].src_off = items[i].offset;
        real += (int64_t)items[i].nx * items[i].ny * items[i].nz;
    }
    const dms_grid sg = {L.X, L.Y, L.Z};
    r = check_grid(ctx, sg, flags);
    if (r != DMS_OK) return r;
    // the separator region closes every box the way the virtual maximum
    // closes a grid, so a batch computes the diagrams with it on
    if (!(flags & DMS_VIRTUAL_MAX))
        return fail(ctx, DMS_E_INVAL, "dms_diagram_batch: DMS_VIRTUAL_MAX is required");
    ctx->virtual_max = true;
    const int64_t V = (int64_t)L.X * L.Y * L.Z;
    ENSURE(ctx->bfield, 4 * V);
    ENSURE(ctx->bowner, 4 * V);
    ENSURE(ctx->bslots, sizeof(BatchSlot) * (size_t)nitems);
    ENSURE(ctx->bitem, 4 * (size_t)nitems);
    ENSURE(ctx->bkept, 64);
    HIPCHK(hipMemcpyAsync(ctx->bslots.p, L.slots.data(), sizeof(BatchSlot) * (size_t)nitems, hipMemcpyHostToDevice,
                          st));
    launch_pack(d_fields, P<BatchSlot>(ctx->bslots), nitems, L.nrows, L, P<float>(ctx->bfield),
                P<uint32_t>(ctx->bowner), st);
    ctx->binfo[0] = L.X;
    ctx->binfo[1] = L.Y;
    ctx->binfo[2] = L.Z;
    ctx->binfo[3] = real;
    ctx->binfo[7] = nitems;

    // ---- a0-a3 on the super grid; the kernels before the count read-back are
    // replayed from a captured graph when the super grid repeats ----
    const bool use_graph = opts && opts->use_graph && st != nullptr;
    bool done = false;
    for (int attempt = 0; attempt < 2 && !done; ++attempt) {
        r = gradient_setup(ctx, sg);
        if (r != DMS_OK) return r;
        if (use_graph) {
            // the buffers the captured kernels read and write
            std::vector<const void*> sig = {ctx->bfield.p, ctx->bowner.p, ctx->flags.p, ctx->keysA.p, ctx->keysB.p, ctx->valsA.p,
                                            ctx->valsB.p, ctx->hist.p, ctx->part.p, ctx->rank.p, ctx->ob.p,
                                            ctx->counters.p, ctx->G.p};
            for (int d = 0; d < 4; ++d) {
                sig.push_back(ctx->cid[d].p);
                sig.push_back(ctx->ck[d].p);
            }
            dms_ctx::GraphEntry* hit = nullptr;
            for (auto& e : ctx->graphs)
                if (e.X == L.X && e.Y == L.Y && e.Z == L.Z && e.sig == sig && std::equal(e.cap, e.cap + 4, ctx->cap))
                    hit = &e;
            if (!hit) {
                hipGraph_t graph = nullptr;
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                gradient_enqueue(ctx, P<float>(ctx->bfield), P<uint32_t>(ctx->bowner), false);
                HIPCHK(hipStreamEndCapture(st, &graph));
                hipGraphExec_t exec = nullptr;
                const hipError_t ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                HIPCHK(ge);
                if (ctx->graphs.size() >= 8) {
                    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
                    ctx->graphs.erase(ctx->graphs.begin());
                }
                dms_ctx::GraphEntry e{L.X, L.Y, L.Z, sig, {ctx->cap[0], ctx->cap[1], ctx->cap[2], ctx->cap[3]},
                                      exec};
                ctx->graphs.push_back(e);
                hit = &ctx->graphs.back();
                ++ctx->binfo[5];
            }
            HIPCHK(hipGraphLaunch(hit->exec, st));
            ++ctx->binfo[4];
        } else {
            gradient_enqueue(ctx, P<float>(ctx->bfield), P<uint32_t>(ctx->bowner), true);
            ++ctx->binfo[6];
        }
        bool over = false;
        r = gradient_counts(ctx, &over);
        if (r != DMS_OK) return r;
        if (!over) done = true;
    }
    if (!done) return fail(ctx, DMS_E_INTERNAL, "critical list capacity");
    r = gradient_finish(ctx, nullptr);
    if (r != DMS_OK) return r;
    r = run_d0_d2(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D02);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 2;
    r = run_d1(ctx);
    if (r != DMS_OK) return r;
    record(ctx, EV_D1);
    r = check_flags(ctx);
    if (r != DMS_OK) return r;
    ctx->stage = 3;
    ctx->batched = true;

    // ---- pairs of the super grid, then per item ----
    int64_t ns[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) ENSURE(ctx->bpairs[d], sizeof(dms_pair) * (size_t)(ctx->ncrit[d] + 16));
    r = emit_d0(ctx, P<dms_pair>(ctx->bpairs[0]), ctx->ncrit[0] + 16, &ns[0], nullptr, nullptr, nullptr, nullptr,
                nullptr);
    if (r != DMS_OK) return r;
    r = emit_d1(ctx, P<dms_pair>(ctx->bpairs[1]), ctx->ncrit[1] + 16, &ns[1], nullptr, nullptr, nullptr, nullptr,
                nullptr);
    if (r != DMS_OK) return r;
    r = emit_d2(ctx, P<dms_pair>(ctx->bpairs[2]), ctx->ncrit[2] + 16, &ns[2], nullptr, nullptr, nullptr, nullptr,
                nullptr, true);
    if (r != DMS_OK) return r;
    const int kbits = 33 + bits_for((uint64_t)std::max(1, nitems - 1));
    bool cap_fail = false;
    std::vector<uint32_t> cnt(nitems);
    for (int d = 0; d < 3; ++d) {
        const int64_t n = ns[d];
        ENSURE(ctx->bkey, 8 * std::max<int64_t>(n, 1));
        ENSURE(ctx->bdeath, 8 * std::max<int64_t>(n, 1));
        ENSURE(ctx->keysB, 8 * std::max<int64_t>(n, 1));
        ENSURE(ctx->valsA, 4 * std::max<int64_t>(n, 1));
        ENSURE(ctx->valsB, 4 * std::max<int64_t>(n, 1));
        ENSURE(ctx->hist, 4 * 256 * sort_tiles(std::max<int64_t>(n, 1)));
        ENSURE(ctx->part, 4 * scan_part_size(256 * sort_tiles(std::max<int64_t>(n, 1))));
        fill_u32(P<uint32_t>(ctx->bitem), 0, nitems, st);
        fill_u32(P<uint32_t>(ctx->bkept), 0, 1, st);
        launch_demux(P<dms_pair>(ctx->bpairs[d]), n, d, ctx->g, P<uint32_t>(ctx->bowner), P<BatchSlot>(ctx->bslots),
                     P<uint64_t>(ctx->bkey), P<int64_t>(ctx->bdeath), P<uint32_t>(ctx->bitem),
                     P<uint32_t>(ctx->bkept), st);
        const int w = radix_sort_pairs<uint64_t>(P<uint64_t>(ctx->bkey), P<uint32_t>(ctx->valsA),
                                                 P<uint64_t>(ctx->keysB), P<uint32_t>(ctx->valsB), n, 0, kbits, true,
                                                 P<uint32_t>(ctx->hist), P<uint32_t>(ctx->part), st);
        uint32_t kept = 0;
        HIPCHK(hipMemcpyAsync(&kept, ctx->bkept.p, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(cnt.data(), ctx->bitem.p, 4 * (size_t)nitems, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        out->n[d] = kept;
        out->item_start[d][0] = 0;
        for (int i = 0; i < nitems; ++i) out->item_start[d][i + 1] = out->item_start[d][i] + cnt[i];
        if ((int64_t)kept > out->cap[d]) {
            cap_fail = true;
            continue;
        }
        launch_demux_write(w ? P<uint64_t>(ctx->keysB) : P<uint64_t>(ctx->bkey),
                           w ? P<uint32_t>(ctx->valsB) : P<uint32_t>(ctx->valsA), P<int64_t>(ctx->bdeath), kept,
                           out->pairs[d], st);
    }
    record(ctx, EV_OUT);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    if (cap_fail) return fail(ctx, DMS_E_CAPACITY, "an output buffer is too small; n[] holds the need");
    return DMS_OK;
}

int dms_batch_info(const dms_ctx* ctx, int64_t info[8]) {
    if (!ctx || !info) return DMS_E_INVAL;
    for (int i = 0; i < 8; ++i) info[i] = ctx->binfo[i];
    return DMS_OK;
}

int dms_set_option(dms_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return DMS_E_INVAL;
    switch (option) {
        case DMS_OPT_D1_SMALL_PASSES: ctx->opt_d1_small = value != 0; return DMS_OK;
        case DMS_OPT_LOG_PASSES: ctx->opt_log = value != 0; return DMS_OK;
        case DMS_OPT_D1_NO_SANDWICH: ctx->opt_no_sandwich = value != 0; return DMS_OK;
        case DMS_OPT_D1_NO_CACHE: ctx->opt_no_cache = value != 0; return DMS_OK;
        case DMS_OPT_D1_HEAP_KEYS:
            if (value < 0) return fail(ctx, DMS_E_INVAL, "dms_set_option: DMS_OPT_D1_HEAP_KEYS must be >= 0");
            ctx->opt_heap_keys = value;
            return DMS_OK;
        default: return fail(ctx, DMS_E_INVAL, "dms_set_option: unknown option");
    }
}

int dms_stage_ms(const dms_ctx* ctx, float ms[8]) {
    if (!ctx || !ms) return DMS_E_INVAL;
    const int pairs[6][2] = {{EV_START, EV_ORDER}, {EV_ORDER, EV_GRAD}, {EV_GRAD, EV_SORT},
                             {EV_SORT, EV_D02},    {EV_D02, EV_D1},     {EV_D1, EV_OUT}};
    ms[7] = -1.0f;
    if (ctx->ev_ok[EV_GK] && ctx->ev_ok[EV_GRAD]) {
        float t = 0;
        if (hipEventElapsedTime(&t, ctx->ev[EV_GK], ctx->ev[EV_GRAD]) == hipSuccess) ms[7] = t;
    }
    for (int i = 0; i < 6; ++i) {
        ms[i] = -1.0f;
        if (ctx->ev_ok[pairs[i][0]] && ctx->ev_ok[pairs[i][1]]) {
            float t = 0;
            if (hipEventElapsedTime(&t, ctx->ev[pairs[i][0]], ctx->ev[pairs[i][1]]) == hipSuccess) ms[i] = t;
        }
    }
    ms[6] = -1.0f;
    int last = -1;
    for (int i = NEV - 1; i > 0; --i)
        if (ctx->ev_ok[i]) { last = i; break; }
    if (ctx->ev_ok[EV_START] && last > 0) {
        float t = 0;
        if (hipEventElapsedTime(&t, ctx->ev[EV_START], ctx->ev[last]) == hipSuccess) ms[6] = t;
    }
    return DMS_OK;
}

}  // extern "C"
