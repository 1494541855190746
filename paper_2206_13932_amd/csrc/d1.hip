// D1 by PairCriticalSimplices (Alg. "PairCriticalSimplices", Sec. 4) on the
// critical triangles left unpaired by D2 -- the sandwich of Sec. 3 -- with
// boundary caching (Sec. 4.1(b)) and clearing (Sec. 4.1(a)).
//
// A column is a 2-saddle; its boundary is a set of edges keyed by their
// lexicographic key (rank of the higher vertex, rank of the lower one). Its
// highest edge tau decides the step:
//   tau regular (tail of an edge-triangle vector) -> add the boundary of the
//       paired triangle;
//   tau critical, owned by an earlier column     -> add that column's cached
//       boundary;
//   tau critical, free or owned by a later one   -> cache the boundary and
//       claim tau with compare-and-swap; a later owner is evicted and its
//       reduction is carried on by this thread (Sec. 7.2).
// The working boundary is a max-heap in per-thread scratch (contiguous per
// thread), with mod-2 cancellation of equal keys when they meet at
// the top. Cached boundaries are immutable arrays (sorted decreasing) bump-
// allocated from a publication heap and accessed with coherent (agent-scope)
// loads and stores, so a reader that finds tau at their head has a complete
// copy. A column whose boundary outgrows its thread's heap is saved to the
// publication heap and deferred to a later pass with larger heaps and fewer
// threads; the result does not depend on when a column is processed.
//
// The result equals the sequential algorithm: with the expansion-based
// gradient, the highest edge of a boundary whose top is critical is also the
// top of its projection onto the Morse complex (all smaller edges of that
// lower star were classified before the critical one was popped, so their
// v-paths only reach smaller critical edges); the loop is therefore a column
// reduction of the Morse boundary matrix, whose pivots do not depend on the
// order in which earlier columns are added.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "d1.h"
#include "dms_internal.h"

namespace dms {

namespace {

constexpr int DB = 256;
constexpr uint32_t OWN_D0 = 0xFFFFFFFEu;
constexpr uint64_t NONE = ~0ull;
constexpr int MAX_PASSES = 6;
// one pass of the D1 plan: heap capacity (keys), lanes or workgroups, block
// size, thread-per-column (heaps in LDS) or workgroup-per-column
struct PassPlan {
    int64_t k, t;
    int db;
    bool lane;
};
constexpr int LDS_K = 20;   // keys per thread in the first pass (LDS heaps)
constexpr int LDS_K2 = 48;  // ... and in the second
constexpr uint32_t MAX_RETRIES = 1u << 16;  // consecutive look-agains before a column is declared corrupt
inline unsigned nblocks(int64_t n) { return (unsigned)((n + DB - 1) / DB); }

// counters in D1State::ctrs
enum { C_HEAP = 0, C_NEXT = 1, C_DEFER = 2, C_STEPS = 3, C_EVICT = 4, C_ADDS = 5, C_ROUNDS = 6, C_EXPANDED = 7,
       C_MOVED = 8, C_TMAX = 9, C_TSUM = 10, C_RMAX = 11, C_AMAX = 12, C_NMAX = 13, C_SLOW = 14, C_LONG = 15, C_PHASE = 16,
       N_PHASE = 10, C_RSTOP = 28, C_RCAP = 29, C_RTAKEN = 30, C_ACTIVE = 31, N_CTRS = 32 };
// The publication heap is split into NSEG segments with one bump counter each
// (counters 128 bytes apart, after the N_CTRS counters above), so that
// millions of publications do not serialise on one atomic.
constexpr int NSEG = 64;
constexpr int SEG_STRIDE = 16;
constexpr int SEG_BASE = N_CTRS;
// Job board of the cooperative merges (after the segment counters): NJ slots
// of BSLOT words (one 128-byte line each): [0] control (sequence << 32 | next
// part), [1] parts done, [2] holder (0 = free), [3] sequence << 32 | parts,
// [4] A, [5] |A|, [6] B (stored decreasing), [7] |B|, [8] output, [9] part
// status words, [10] part span. An odd sequence marks an open job.
constexpr int NJ = 64;
constexpr int BSLOT = 16;
constexpr int BOARD_BASE = SEG_BASE + SEG_STRIDE * NSEG;
// own line: open jobs, then (counted over a run) parts merged by helpers and
// cooperative merges
constexpr int OPEN_JOBS = BOARD_BASE + NJ * BSLOT, HELPED_PARTS = OPEN_JOBS + 1, COOP_MERGES = OPEN_JOBS + 2,
              GUARD_REASON = OPEN_JOBS + 3,  // the first consistency check that failed (one of G_*)
              NC_FALLBACKS = OPEN_JOBS + 4;  // uncached additions whose pivot came back (ablation)
constexpr int N_CTR_WORDS = OPEN_JOBS + 16;

// consistency checks of the D1 kernels
enum : uint32_t { G_STEPS = 1, G_RETRIES, G_KEY, G_VPARTNER, G_D0, G_EVICT_HEAD, G_WSTEPS, G_WRETRIES, G_WTOP,
                  G_LOOKBACK, G_JOBWAIT, G_HEAPPTR, G_COUNT };
static const char* const kGuardName[G_COUNT] = {
    "unknown", "a column ran out of steps", "a look-again did not resolve", "a key is no edge",
    "a vertex's partner edge at the top", "a D0-paired edge at the top", "an evicted column's cached head moved",
    "a workgroup column ran out of steps", "a workgroup look-again did not resolve",
    "a workgroup column's top is no critical edge", "a merge part's look-back wait ran out",
    "a merge job's wait for its parts ran out", "a boundary pointer lies outside the publication heap"};
// record the first failed check and flag the call
__device__ inline void guard_fail(unsigned long long* ctrs, uint32_t* flags, uint32_t why) {
    atomicCAS(&ctrs[GUARD_REASON], 0ull, (unsigned long long)why);
    atomicOr(flags, FLAG_GUARD);
}

struct D1K {
    GridDev g;
    const uint8_t* G;
    const uint32_t* rank;
    const uint32_t* order;
    const uint32_t* cols;
    int64_t ncols;
    // work of this pass: columns 0..ncols-1 (first pass) or deferred records
    const uint64_t* work;  // heap offset of each deferred record, or null in the first pass
    const uint32_t* work_col;  // its column
    const uint32_t* work_len;  // its length
    int64_t nwork;
    uint64_t* defer;  // records deferred by this pass: heap offset, column, length
    uint32_t* defer_col;
    uint32_t* defer_len;
    int bpr;
    uint32_t* owner1;
    uint64_t* bndptr;
    uint64_t* heap;
    uint64_t heap_cap;  // entries
    uint64_t seg_cap;   // entries per segment
    uint64_t* scratch;
    int64_t K;
    int64_t nthreads;
    uint32_t long_add;  // cached boundaries longer than this are added by one full merge
    int64_t nslots;     // workgroups of a workgroup pass that take columns; the others only help
    uint32_t part_span; // merged positions per part of a cooperative merge
    uint64_t coop_min;  // full merges of at least this many entries are split into parts
    int coop_always;    // split them even when no idle workgroup may help (debug)
    uint32_t pcap;      // pending keys that trigger a flush into low (PCAP; smaller for debugging)
    int no_cache;       // ablation: add the boundary of an earlier owner's 2-saddle, not its cached one
    unsigned long long* ctrs;
    uint32_t* flags;
};

__device__ inline uint32_t ld_rlx(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_rlx64(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_rlx64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Publish order: the data a claim makes visible is written with agent-scope
// atomic stores (sc1, coherent across the XCDs' L2s); vmcnt(0) makes the
// hardware finish them before the claiming atomic is issued, and the two
// signal fences (compiler-only barriers) keep the compiler from moving any
// memory operation across the wait. A release CAS at agent scope would also
// order them, but it adds an L2 writeback (buffer_wbl2) per claim.
__device__ inline void wait_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ inline bool cas32(uint32_t* p, uint32_t expect, uint32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t ekey_r(int bpr, uint32_t ra, uint32_t rb) {
    return ra > rb ? (((uint64_t)ra << bpr) | rb) : (((uint64_t)rb << bpr) | ra);
}

// edge key -> endpoints (va higher), anchor, step mask, id
struct EdgeDec {
    int64_t va, vb, lo;
    uint32_t ra, rb;
    int mask;
    uint32_t id;
};
// step mask and anchor of the edge {a, b} of the triangulation (vertex ids)
__device__ inline int edge_mask(const GridDev& g, int64_t a, int64_t b, int64_t& lo) {
    lo = a < b ? a : b;
    int64_t d = (a < b ? b : a) - lo;
    int m = 0;
    if (d >= g.sz) { m |= 4; d -= g.sz; }
    if (d >= g.sy) { m |= 2; d -= g.sy; }
    if (d >= 1) { m |= 1; }
    return m;
}
// the same when the endpoints' vertex ids are known (va of rank ra, vb of rb)
__device__ inline EdgeDec edecode_ids(const GridDev& g, int bpr, uint64_t key, int64_t va, int64_t vb) {
    EdgeDec e;
    e.ra = (uint32_t)(key >> bpr);
    e.rb = (uint32_t)(key & ((1ull << bpr) - 1));
    e.va = va;
    e.vb = vb;
    e.lo = e.va < e.vb ? e.va : e.vb;
    int64_t d = (e.va < e.vb ? e.vb : e.va) - e.lo;
    int m = 0;
    if (d >= g.sz) { m |= 4; d -= g.sz; }
    if (d >= g.sy) { m |= 2; d -= g.sy; }
    if (d >= 1) { m |= 1; }
    e.mask = m;
    e.id = (uint32_t)(e.lo * 7 + (m - 1));
    return e;
}
// (mask 0: the key holds a rank outside the grid or twice; the lookups then
// read ranks 0 and 1 instead, so that no address depends on it)
__device__ inline EdgeDec edecode(const GridDev& g, const uint32_t* order, int bpr, uint64_t key) {
    EdgeDec e;
    e.ra = (uint32_t)(key >> bpr);
    e.rb = (uint32_t)(key & ((1ull << bpr) - 1));
    const bool ok = !(key >> (2 * bpr)) && (int64_t)e.ra < g.V && (int64_t)e.rb < g.V && e.ra != e.rb;
    e.va = order[ok ? e.ra : 0u];
    e.vb = order[ok ? e.rb : 1u];
    e.lo = e.va < e.vb ? e.va : e.vb;
    int64_t d = (e.va < e.vb ? e.vb : e.va) - e.lo;
    int m = 0;
    if (d >= g.sz) { m |= 4; d -= g.sz; }
    if (d >= g.sy) { m |= 2; d -= g.sy; }
    if (d >= 1) { m |= 1; }
    e.mask = ok ? m : 0;
    e.id = (uint32_t)(e.lo * 7 + (m - 1));
    return e;
}

// ---- per-lane max-heap in LDS with mod-2 cancellation ------------------------
// The lane passes' dynamic LDS: lane t's heap is lds_heaps[t K .. t K + K).
// Elements are reached through the shared array itself (not through a
// pointer that could be global memory), so that they compile to LDS
// instructions, which wait apart from the lane's global loads.
extern __shared__ uint64_t lds_heaps[];
struct Heap {
    uint32_t base;  // element i at lds_heaps[base + i]
    int32_t n;
    int32_t K;
    __device__ uint64_t& at(int32_t i) { return lds_heaps[base + (uint32_t)i]; }
    __device__ void push(uint64_t x) {
        int32_t i = n++;
        while (i > 0) {
            const int32_t p = (i - 1) >> 1;
            const uint64_t hp = at(p);
            if (hp >= x) break;
            at(i) = hp;
            i = p;
        }
        at(i) = x;
    }
    __device__ uint64_t pop() {
        const uint64_t top = at(0);
        const uint64_t x = at(--n);
        int32_t i = 0;
        for (;;) {
            const int32_t l = 2 * i + 1;
            if (l >= n) break;
            int32_t c = l;
            uint64_t hc = at(l);
            if (l + 1 < n) {
                const uint64_t hr = at(l + 1);
                if (hr > hc) { c = l + 1; hc = hr; }
            }
            if (hc <= x) break;
            at(i) = hc;
            i = c;
        }
        if (n > 0) at(i) = x;
        return top;
    }
    // highest key present an odd number of times, removed; NONE if empty
    __device__ uint64_t extract_max() {
        while (n > 0) {
            const uint64_t t = pop();
            int cnt = 1;
            while (n > 0 && at(0) == t) {
                pop();
                ++cnt;
            }
            if (cnt & 1) return t;
        }
        return NONE;
    }
    // rewrite the heap as its cancelled contents sorted decreasingly (a
    // decreasing array is a valid max-heap)
    __device__ void compact() {
        const int32_t n0 = n;
        int32_t out = 0;
        for (;;) {
            const uint64_t t = extract_max();
            if (t == NONE) break;
            at(n0 - 1 - out) = t;
            ++out;
        }
        for (int32_t i = 0; i < out / 2; ++i) {
            const uint64_t a = at(n0 - out + i);
            at(n0 - out + i) = at(n0 - 1 - i);
            at(n0 - 1 - i) = a;
        }
        for (int32_t i = 0; i < out; ++i) at(i) = at(n0 - out + i);
        n = out;
    }
    __device__ bool room(int64_t extra) {
        if (n + extra <= K) return true;
        compact();
        return n + extra <= K;
    }
};

// keys of the three edges of triangle t (the boundary of a 2-saddle)
__device__ __forceinline__ void tri_edge_keys(const D1K& P, uint32_t t, uint64_t (&k)[3]) {
    const int64_t a = t / 12;
    const int ty = t % 12;
    const int64_t v1 = a + lin_of_mask(P.g, tri_step(ty, 0));
    const int64_t v2 = v1 + lin_of_mask(P.g, tri_step(ty, 1));
    const uint32_t r0 = P.rank[a], r1 = P.rank[v1], r2 = P.rank[v2];
    k[0] = ekey_r(P.bpr, r0, r1);
    k[1] = ekey_r(P.bpr, r1, r2);
    k[2] = ekey_r(P.bpr, r0, r2);
}

// Reserve len entries of the publication heap, in segment seg or, when it is
// full, in the following ones; NONE when every segment is full.
__device__ inline uint64_t heap_alloc(const D1K& P, uint32_t seg, uint64_t len) {
    for (int k = 0; k < NSEG; ++k) {
        const uint32_t sg = (seg + k) % NSEG;
        unsigned long long* ctr = &P.ctrs[SEG_BASE + SEG_STRIDE * sg];
        if (ld_rlx64((const uint64_t*)ctr) + len > P.seg_cap) continue;  // full: skip without growing it
        const uint64_t off = atomicAdd(ctr, (unsigned long long)len);
        if (off + len <= P.seg_cap) return (uint64_t)sg * P.seg_cap + off;
    }
    return NONE;
}

// A packed boundary pointer (offset << 24 | length) whose entries lie inside
// the publication heap. Pointers come from other columns' publications; one
// that does not is reported as a failed check instead of being followed.
__device__ inline bool heap_span_ok(const D1K& P, uint64_t packed) {
    const uint64_t off = packed >> 24, len = packed & 0xFFFFFF;
    return packed != EMPTY64 && len > 0 && off + len <= (uint64_t)P.heap_cap;
}

// Copy {top (optional)} + the heap array as it stands to the publication
// heap; returns the packed (offset << 24 | length) or NONE when the heap is
// full. The copy is neither sorted nor cancelled (the lane's wavefront runs
// this whenever any of its lanes claims, so it must be short): entries after
// the head form a valid max-heap and count mod 2. Lane passes read such
// boundaries as heaps; the workgroup passes sort and cancel every boundary of
// up to NW entries they load (longer ones come only from workgroup passes,
// which publish them sorted and cancelled).
__device__ inline uint64_t publish(const D1K& P, Heap& H, bool with_top, uint64_t top) {
    const uint64_t len = (uint64_t)H.n + (with_top ? 1 : 0);
    if (len >= (1ull << 24)) return NONE;
    const uint64_t off = heap_alloc(P, (uint32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), len);
    if (off == NONE) return NONE;
    uint64_t* A = P.heap + off;
    int64_t k = 0;
    if (with_top) st_rlx64(&A[k++], top);
    for (int64_t i = 0; i < H.n; ++i) st_rlx64(&A[k++], H.at(i));
    wait_stores();
    return (off << 24) | len;
}

__device__ inline void defer_column(const D1K& P, uint32_t c, uint64_t off, uint64_t len) {
    const uint64_t d = atomicAdd(&P.ctrs[C_DEFER], 1ull);
    P.defer[d] = off;
    P.defer_col[d] = c;
    P.defer_len[d] = (uint32_t)len;
}

// One lane per column; each iteration of the loop is one reduction step of
// the lane's column, and a lane whose column is done takes the next one at
// once (one atomic per wavefront for all lanes that need work), so the lanes
// of a wavefront do not wait for each other's columns.
template <bool NC>  // NC: the ablation without caching
__global__ __launch_bounds__(DB) void k_d1(D1K P) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the lanes beyond nthreads take no work
    const bool real = tid < P.nthreads;
    Heap H;
    H.base = (uint32_t)(threadIdx.x * P.K);
    H.K = (int32_t)P.K;
    H.n = 0;
    const int64_t V = P.g.V;
    unsigned long long steps = 0, evictions = 0, adds = 0;
    bool active = false, exhausted = !real, stop = false;
    uint32_t c = 0;
    bool have = false;
    uint64_t tau = 0;
    int64_t guard = 0;
    uint32_t retries = 0;
    int64_t pb = 0, pe = 0;  // the wavefront's chunk of column numbers
    // keys of the last two edges pushed by an expansion, with their endpoints
    // (va: the endpoint of the higher rank)
    uint64_t hint_key[2] = {NONE, NONE};
    uint64_t nc_min = NONE;  // ablation without caching: the lowest pivot re-reduced in place
    uint32_t fallbacks = 0;
    int64_t hint_va[2] = {0, 0}, hint_vb[2] = {0, 0};

    // one step of column c: 0 = go on, 1 = the column is done, 2 = error
    auto step = [&]() -> int {
        if (++guard > ((int64_t)1 << 24) || retries > MAX_RETRIES) {
            guard_fail(P.ctrs, P.flags, retries > MAX_RETRIES ? G_RETRIES : G_STEPS);
            return 2;
        }
        ++steps;
        if (!have) {
            tau = H.extract_max();
            if (tau == NONE) return 1;  // zero column
            have = true;
        }
        // The two edges an expansion pushes are often the next top (the v-path
        // goes on): their vertex ids are kept, which saves the order lookups,
        // one dependent global load, on the lane's chain of loads.
        const EdgeDec e = tau == hint_key[0]   ? edecode_ids(P.g, P.bpr, tau, hint_va[0], hint_vb[0])
                          : tau == hint_key[1] ? edecode_ids(P.g, P.bpr, tau, hint_va[1], hint_vb[1])
                                               : edecode(P.g, P.order, P.bpr, tau);
        if (e.mask == 0) {  // not an edge: corrupted key
            guard_fail(P.ctrs, P.flags, G_KEY);
            return 2;
        }
        const uint8_t code = P.G[(int64_t)e.mask * V + e.lo];
        bool defer = false;
        if (code != CODE_CRIT) {
            if (code >= 27) {  // the top of a cycle cannot be a vertex's partner
                guard_fail(P.ctrs, P.flags, G_VPARTNER);
                return 2;
            }
            const int64_t w = e.lo + lin27(P.g, code);
            if (H.room(2)) {
                have = false;  // tau cancels against the boundary of its partner
                const uint32_t rw = P.rank[w];
                hint_key[0] = ekey_r(P.bpr, e.ra, rw);
                hint_key[1] = ekey_r(P.bpr, e.rb, rw);
                hint_va[0] = e.ra > rw ? e.va : w;
                hint_vb[0] = e.ra > rw ? w : e.va;
                hint_va[1] = e.rb > rw ? e.vb : w;
                hint_vb[1] = e.rb > rw ? w : e.vb;
                // The larger new key, when it is above every heap entry, is the
                // boundary's highest key, present once: it is the next top as
                // extract_max would return it, and it stays out of the heap
                // (a push and the next step's pop saved).
                const uint64_t kmax = hint_key[0] > hint_key[1] ? hint_key[0] : hint_key[1];
                const uint64_t kmin = hint_key[0] > hint_key[1] ? hint_key[1] : hint_key[0];
                H.push(kmin);
                if (kmax > H.at(0)) {
                    tau = kmax;
                    have = true;
                } else {
                    H.push(kmax);
                }
                return 0;
            }
            defer = true;
        } else {
            const uint32_t o = ld_rlx(&P.owner1[e.id]);
            if (o == OWN_D0) {
                guard_fail(P.ctrs, P.flags, G_D0);
                return 2;
            }
            if (o == EMPTY32 || o > c) {
                // cache Boundary(c) = {tau} + heap, then claim tau
                const uint64_t b = publish(P, H, true, tau);
                if (b == NONE) {
                    atomicOr(P.flags, FLAG_HEAP);
                    return 2;
                }
                st_rlx64(&P.bndptr[c], b);
                wait_stores();
                if (!cas32(&P.owner1[e.id], o, c)) {  // owner changed: look again
                    ++retries;
                    return 0;
                }
                if (o == EMPTY32) return 1;  // column settled
                // evicted o: carry on reducing it from its cached boundary
                ++evictions;
                const uint64_t bo = ld_rlx64(&P.bndptr[o]);
                if (!heap_span_ok(P, bo)) {
                    guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                    return 2;
                }
                const uint64_t* B = P.heap + (bo >> 24);
                const int64_t bl = (int64_t)(bo & 0xFFFFFF);
                if (ld_rlx64(&B[0]) != tau) {
                    guard_fail(P.ctrs, P.flags, G_EVICT_HEAD);
                    return 2;
                }
                c = o;
                retries = 0;
                nc_min = NONE;
                if (bl > H.K) {  // too large for this pass: defer it as it stands
                    defer_column(P, c, bo >> 24, bl);
                    return 1;
                }
                for (int32_t i = 1; i < (int32_t)bl; ++i) H.at(i - 1) = ld_rlx64(&B[i]);
                H.n = (int32_t)bl - 1;
                have = true;  // tau (= B[0]) is its top
                return 0;
            }
            // o < c: add the cached boundary of the earlier owner, or, in the
            // ablation without caching, the boundary of o's 2-saddle (its top
            // is at or above tau), which is then reduced again: tau goes back
            // into the heap and cancels when that reduction brings it back.
            // The re-reduction follows the owners of the moment, which
            // evictions may have changed since o's own reduction, so it can
            // miss tau; so re-reduction happens only below every pivot
            // re-reduced before in this column: pivots met inside it, and a
            // pivot that comes back, get cached boundaries (the uncached
            // pivots then strictly decrease, and the loop ends).
            const bool uncached = NC && tau < nc_min;
            fallbacks += (NC && !uncached) ? 1 : 0;
            const uint64_t* B = nullptr;
            int64_t need = 4;
            if (!uncached) {
                const uint64_t b = ld_rlx64(&P.bndptr[o]);
                if (b == EMPTY64) {
                    ++retries;
                    return 0;
                }
                if (!heap_span_ok(P, b)) {
                    guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                    return 2;
                }
                B = P.heap + (b >> 24);
                if (ld_rlx64(&B[0]) != tau) {  // o moved on: look again
                    ++retries;
                    return 0;
                }
                need = (int64_t)(b & 0xFFFFFF) - 1;
            }
            retries = 0;
            if (H.room(need)) {
                have = false;
                ++adds;
                if (B) {
                    for (int64_t i = 1; i <= need; ++i) H.push(ld_rlx64(&B[i]));
                } else {
                    uint64_t k3[3];
                    tri_edge_keys(P, P.cols[o], k3);
                    nc_min = tau;
                    H.push(tau);
                    H.push(k3[0]);
                    H.push(k3[1]);
                    H.push(k3[2]);
                }
                return 0;
            }
            defer = true;
        }
        // save {tau} + heap and hand the column to the next pass
        (void)defer;
        const uint64_t b = publish(P, H, have, tau);
        if (b == NONE) {
            atomicOr(P.flags, FLAG_HEAP);
            return 2;
        }
        defer_column(P, c, b >> 24, b & 0xFFFFFF);
        return 1;
    };

    for (;;) {
        // lanes without a column take the next ones, from chunks of 128
        // consecutive columns per wavefront. Columns are taken in increasing
        // order: the frontier of columns in flight stays narrow, which keeps
        // evictions rare
        const bool need = !active && !exhausted && !stop;
        int64_t next = 0;
        if (!wave_take<128>(need, &P.ctrs[C_NEXT], P.nwork, next, pb, pe)) {
            exhausted = true;
        } else if (need) {
            H.n = 0;
            have = false;
            guard = 0;
            retries = 0;
            nc_min = NONE;
            active = true;
            if (!P.work) {
                c = (uint32_t)next;
                uint64_t k3[3];
                tri_edge_keys(P, P.cols[c], k3);
                H.push(k3[0]);
                H.push(k3[1]);
                H.push(k3[2]);
            } else {
                // resume a deferred column from its saved boundary
                c = P.work_col[next];
                const uint64_t off = P.work[next];
                const int64_t len = P.work_len[next];
                if (len > H.K) {
                    atomicOr(P.flags, FLAG_WORK);
                    active = false;
                    stop = true;
                } else if (off + (uint64_t)len > (uint64_t)P.heap_cap) {
                    guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                    active = false;
                    stop = true;
                } else {
                    // a saved boundary is {tau} + a heap array: pushed entry by entry
                    for (int64_t i = 0; i < len; ++i) H.push(ld_rlx64(P.heap + off + i));
                }
            }
        }
        if (!__ballot(active)) break;  // every lane is out of work (or stopped)
        if (active) {
            const int r = step();
            if (r != 0) active = false;
            if (r == 2) stop = true;
        }
    }
    atomicAdd(&P.ctrs[C_STEPS], steps);
    atomicAdd(&P.ctrs[C_EVICT], evictions);
    atomicAdd(&P.ctrs[C_ADDS], adds);
    if (fallbacks) atomicAdd(&P.ctrs[NC_FALLBACKS], (unsigned long long)fallbacks);
}


// ---- one workgroup per large column ------------------------------------------
// The boundary is kept sorted ascending in two parts: its largest entries
// (up to TOPCAP) in LDS ("top"), the rest in per-block global scratch ("low";
// every low key is below every top key). A round looks at the top WB edges:
// every regular tail above the first critical (or non-tail) edge is expanded
// at once -- adding the boundary of a partner triangle leaves the column's
// Morse projection unchanged, so the expansions commute -- and the new edges
// are sorted, cancelled mod 2 and merged in: keys above the low part's
// maximum into the top (LDS to LDS), the others into the low part (staged
// through LDS in segments). A top that outgrows TOPCAP spills its smaller
// entries to the end of the low part; a top that falls below WB entries is
// refilled from it. When the top is critical, the owner rule runs as in k_d1,
// with cached boundaries merged in chunks. Published boundaries keep the
// decreasing layout (top first). Block-wide scans and counts use wave
// ballots and shuffles with one barrier each.
constexpr int WB = 256;
constexpr int NWAVE = WB / 64;
constexpr int NW = 4 * WB;  // keys merged per step
constexpr int IPW = NW / WB;
constexpr int TOPCAP = 2048;  // LDS top capacity; also the staging segment of low merges
constexpr int TOPKEEP = 1024; // top entries kept after a spill, or loaded by a refill
constexpr int PCAP = NW;      // pending keys below the top, merged into low in batches
constexpr uint32_t BATCH_ADD_MAX = 512;  // longest cached boundary added out of order in a round
constexpr int CHAIN = 6;  // same-star continuation steps of one expansion in a round
constexpr uint64_t PAD = ~0ull;
constexpr uint32_t LONG_ADD = 2 * PCAP;  // default of D1K::long_add
static_assert(TOPKEEP >= WB && TOPKEEP + WB <= TOPCAP, "top refill must fit");

// rows of WideShared::ws (wave totals); a row is written again only after
// another barrier has passed
enum { WS_CNT0 = 0, WS_CNT1 = 1, WS_ROUND = 2, WS_SORT = 3, WS_MERGE = 4, WS_ROWS = 5 };

struct WideShared {
    uint64_t top[2][TOPCAP];  // the top (one buffer) and a merge target / staging area
    uint64_t raw[NW];   // new keys of a round, sorted here
    uint64_t src[NW];   // keys to merge (ascending, unique)
    uint64_t surv[NW];  // keys of src not present in the target; heap offsets while a round is built
    uint32_t lb[NW];    // number of target entries smaller than src[j]
    uint32_t lbs[NW];   // lb of the survivors
    uint32_t canc[NW];  // target indices cancelled by src, ascending
    uint32_t flag[NW];
    uint32_t ws[WS_ROWS][NWAVE];
    uint32_t wstop[NWAVE];
    uint32_t wcnt[NWAVE];
    uint32_t wend[NWAVE];
    int ints[8];
    uint64_t u64s[4];
    uint64_t srch[4];   // search ranges of the part bounds, then the bounds
    uint32_t wcount[NWAVE];
    uint64_t job[12];   // the job a helper works on
    uint32_t nextra;    // keys of a round's same-star continuations, after the entries' own keys
};

// inclusive prefix sum over the 64 lanes of a wave with DPP row shifts and
// row broadcasts (no LDS round trips)
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return v;
}

// value of lane (lane ^ d) of the same wave, d a power of two below 64: quad
// permutes, row shifts and the gfx950 permlane swaps, all without LDS
__device__ inline uint32_t lane_xor(uint32_t x, uint32_t d) {
    const uint32_t lane = threadIdx.x & 63;
    switch (d) {
    case 1: return __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    case 2: return __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    case 4: {
        const uint32_t a = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xf, 0xf, false);  // row_shl:4
        const uint32_t b = __builtin_amdgcn_update_dpp(x, x, 0x114, 0xf, 0xf, false);  // row_shr:4
        return (lane & 4) ? b : a;
    }
    case 8: {
        const uint32_t a = __builtin_amdgcn_update_dpp(x, x, 0x108, 0xf, 0xf, false);  // row_shl:8
        const uint32_t b = __builtin_amdgcn_update_dpp(x, x, 0x118, 0xf, 0xf, false);  // row_shr:8
        return (lane & 8) ? b : a;
    }
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    default: {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
    }
}

// exclusive prefix sum of v over the block; ws is a row of wave totals
__device__ inline uint32_t block_excl_scan(uint32_t* ws, uint32_t v, uint32_t& total) {
    const int t = threadIdx.x, w = t >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if ((t & 63) == 63) ws[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) {
        const uint32_t s = ws[i];
        before += i < w ? s : 0u;
        tot += s;
    }
    total = tot;
    return before + inc - v;
}

// number of threads of the block with pred set
__device__ inline uint32_t block_count(uint32_t* ws, bool pred) {
    const uint64_t b = __ballot(pred);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) tot += ws[i];
    return tot;
}

// number of elements of the ascending array A[0..n) smaller than x (LDS)
template <typename T>
__device__ inline uint32_t count_less(const T* A, uint32_t n, T x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The same for an array in global memory, found by the whole block: each
// level loads one sample per thread (the last entry of WB equal segments)
// and keeps the segment where the samples cross x.
__device__ uint32_t count_less_block(WideShared& L, const uint64_t* A, uint32_t n, uint64_t x) {
    const uint32_t t = threadIdx.x;
    uint32_t lo = 0, len = n;
    int row = 0;
    while (len > (uint32_t)WB) {
        const uint32_t step = (len + WB - 1) / WB;
        const uint32_t nseg = (len + step - 1) / step;
        bool pred = false;
        if (t < nseg) pred = A[lo + min((t + 1) * step, len) - 1] < x;
        const uint32_t c = block_count(L.ws[WS_CNT0 + row], pred);
        row ^= 1;
        if (c == nseg) return lo + len;
        lo += c * step;
        len = min(step, len - c * step);
    }
    const bool pred = t < len && A[lo + t] < x;
    return lo + block_count(L.ws[WS_CNT0 + row], pred);
}

// dst[0..len) <- src[0..len) (global to LDS), by the block, len <= TOPCAP
__device__ inline void stage(uint64_t* dst, const uint64_t* src, uint32_t len) {
    if (len == 0) return;
    const uint32_t t = threadIdx.x;
    uint64_t v[TOPCAP / WB];
#pragma unroll
    for (int q = 0; q < TOPCAP / WB; ++q) v[q] = src[min((uint32_t)(q * WB) + t, len - 1)];
#pragma unroll
    for (int q = 0; q < TOPCAP / WB; ++q)
        if ((uint32_t)(q * WB) + t < len) dst[q * WB + t] = v[q];
}

// Merge X[0..len) (LDS) with S[0..m) (LDS; both ascending, unique; equal
// keys cancel). Output entries o < sp go to gdst[o], the others to
// ldst[o - sp], where sp = 0 if the result fits in cap entries and
// result - keep otherwise (cap = 0: everything to gdst). Returns the
// result length; sp is set. The caller synchronises before the outputs or
// the shared arrays are used again. When sp > 0, L.u64s[0] receives the
// largest key sent to gdst.
__device__ uint32_t merge_seg(WideShared& L, const uint64_t* X, uint32_t len, const uint64_t* S, uint32_t m,
                              uint64_t* gdst, uint64_t* ldst, uint32_t cap, uint32_t keep, uint32_t& sp) {
    const uint32_t t = threadIdx.x;
    for (uint32_t j = t; j < m; j += WB) {
        const uint32_t c = count_less<uint64_t>(X, len, S[j]);
        L.lb[j] = c;
        L.flag[j] = (c < len && X[c] == S[j]) ? 1u : 0u;
    }
    __syncthreads();
    uint32_t fc = 0, sc = 0;
    for (int q = 0; q < IPW; ++q) {
        const uint32_t j = IPW * t + q;
        if (j < m) {
            fc += L.flag[j];
            sc += 1 - L.flag[j];
        }
    }
    // both counts in one scan (each at most NW < 2^16)
    uint32_t both;
    const uint32_t ex = block_excl_scan(L.ws[WS_MERGE], fc | (sc << 16), both);
    const uint32_t nc = both & 0xFFFF, ns = both >> 16;
    {
        uint32_t a = ex & 0xFFFF, b = ex >> 16;
        for (int q = 0; q < IPW; ++q) {
            const uint32_t j = IPW * t + q;
            if (j >= m) break;
            if (L.flag[j]) L.canc[a++] = L.lb[j];
            else {
                L.surv[b] = S[j];
                L.lbs[b] = L.lb[j];
                ++b;
            }
        }
    }
    __syncthreads();
    const uint32_t r = len - nc + ns;
    const uint32_t split = cap == 0 ? r : (r > cap ? r - keep : 0u);
    sp = split;
    auto put = [&](uint32_t o, uint64_t x) {
        if (o < split) {
            gdst[o] = x;
            if (o + 1 == split) L.u64s[0] = x;
        } else {
            ldst[o - split] = x;
        }
    };
    // canc (indices of cancelled entries) and lbs (entries placed before each
    // survivor) are ascending: each thread walks a contiguous run of X with
    // two cursors. Entry i moves to i - #(cancelled before i) + #(survivors
    // with lbs <= i); survivor k goes to k + lbs[k] - #(cancelled before lbs[k]).
    {
        const uint32_t per = (len + WB - 1) / WB;
        const uint32_t i0 = min(len, t * per), i1 = min(len, i0 + per);
        if (i0 < i1) {
            uint32_t cc = count_less<uint32_t>(L.canc, nc, i0);
            uint32_t ss = count_less<uint32_t>(L.lbs, ns, i0 + 1);
            uint32_t nextc = cc < nc ? L.canc[cc] : ~0u;
            uint32_t nexts = ss < ns ? L.lbs[ss] : ~0u;
            for (uint32_t i = i0; i < i1; ++i) {
                const uint64_t x = X[i];
                while (nexts <= i) {
                    ++ss;
                    nexts = ss < ns ? L.lbs[ss] : ~0u;
                }
                if (nextc == i) {
                    ++cc;
                    nextc = cc < nc ? L.canc[cc] : ~0u;
                    continue;
                }
                put(i - cc + ss, x);
            }
        }
    }
    for (uint32_t k = t; k < ns; k += WB) {
        const uint32_t cl = count_less<uint32_t>(L.canc, nc, L.lbs[k]);
        put(k + L.lbs[k] - cl, L.surv[k]);
    }
    return r;
}

// cooperative full merge (defined below with the job board)
__device__ __noinline__ uint32_t coop_merge(WideShared& L, unsigned long long* ctrs, uint32_t* flags, const uint64_t* b,
                                            uint32_t span, const uint64_t* low, uint32_t na, uint32_t nb, uint64_t* tmp,
                                            uint64_t* stat, int xb);
// may other workgroups help with a merge now? (the pass has dedicated
// helpers, or its queue of columns is exhausted)
__device__ inline bool coop_possible(const D1K& P) {
    return P.coop_always || (int64_t)gridDim.x > P.nslots ||
           ld_rlx64((const uint64_t*)&P.ctrs[C_NEXT]) >= (uint64_t)P.nwork;
}

// low[0..n) ^= S[0..m) (S in LDS; both ascending, unique), in place in global
// memory; returns the new size. Only the suffix from S[0] changes. The top
// TOPCAP entries of low are staged in LDS (in stg); when the suffix lies
// inside them it is merged straight back. A longer suffix is found by a block
// search and merged segment by segment (TOPCAP entries each, with the keys
// below the next segment's first key) into tmp. Then either the merged
// suffix is copied back, or, when the unchanged prefix is shorter, the prefix
// is copied in front of it and the two buffers swap roles.
__device__ __forceinline__ uint32_t merge_low(const D1K& P, WideShared& L, uint64_t*& low, uint32_t n, const uint64_t* S,
                                              uint32_t m, uint64_t*& tmp, uint64_t* stg, uint64_t* sbuf,
                                              uint64_t* stat, unsigned long long& moved) {
    const uint32_t t = threadIdx.x;
    if (m == 0) return n;
    uint32_t sp;
    const uint32_t h = min(n, (uint32_t)TOPCAP);
    stage(stg, low + (n - h), h);
    __syncthreads();
    if (h == n || S[0] > stg[0]) {
        const uint32_t q = count_less<uint64_t>(stg, h, S[0]);
        moved += h - q;
        const uint32_t r = merge_seg(L, stg + q, h - q, S, m, low + (n - h + q), nullptr, 0, 0, sp);
        __syncthreads();
        return n - h + q + r;
    }
    const uint32_t p = count_less_block(L, low, n, S[0]);
    uint64_t* Bp = low + p;
    const uint32_t len = n - p;
    if (len >= P.coop_min && coop_possible(P)) {
        // a long suffix changes: merge all of low with S by parts into tmp. S is
        // staged decreasing in sbuf (coherent stores: parts read it coherently)
        for (uint32_t k = t; k < m; k += WB) st_rlx64(sbuf + (m - 1 - k), S[k]);
        __syncthreads();
        moved += n + m;
        const uint32_t out = coop_merge(L, P.ctrs, P.flags, sbuf, P.part_span, low, n, m, tmp, stat,
                                        stg == L.top[1] ? 1 : 0);
        if (out == ~0u) return 0;  // a wait ran out; the consistency flag is set
        uint64_t* w = low;
        low = tmp;
        tmp = w;
        __syncthreads();
        return out;
    }
    const bool swap = p < len;
    uint64_t* dst = swap ? tmp + p : tmp;
    moved += len;
    uint32_t out = 0, j0 = 0;
    for (uint32_t sb = 0; sb < len; sb += TOPCAP) {
        const uint32_t sl = min((uint32_t)TOPCAP, len - sb);
        stage(stg, Bp + sb, sl);
        uint32_t ja = m;
        if (sb + sl < len) ja = j0 + count_less<uint64_t>(S + j0, m - j0, Bp[sb + sl]);
        __syncthreads();
        out += merge_seg(L, stg, sl, S + j0, ja - j0, dst + out, nullptr, 0, 0, sp);
        __syncthreads();
        j0 = ja;
    }
    if (swap) {
        for (uint32_t base = 0; base < p; base += 8 * WB) {
            uint64_t v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t i = base + q * WB + t;
                v[q] = i < p ? low[i] : 0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t i = base + q * WB + t;
                if (i < p) tmp[i] = v[q];
            }
        }
        __syncthreads();
        uint64_t* w = low;
        low = tmp;
        tmp = w;
        return p + out;
    }
    for (uint32_t base = 0; base < out; base += 8 * WB) {
        uint64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t i = base + q * WB + t;
            v[q] = i < out ? tmp[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t i = base + q * WB + t;
            if (i < out) Bp[i] = v[q];
        }
    }
    __syncthreads();
    return p + out;
}

// sort L.raw[0..total) ascending (total <= NW) and cancel equal keys mod 2
// into out (which may be L.raw); returns the number of keys kept. A bitonic network over the next
// power of two (PAD beyond total), each thread holding IPW consecutive
// entries: exchanges inside a thread are register moves, inside a wave lane
// permutes, and only strides of a wave's span or more go through LDS.
__device__ inline uint64_t lane_xor64(uint64_t x, uint32_t d) {
    const uint32_t lo = lane_xor((uint32_t)x, d), hi = lane_xor((uint32_t)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}
// the bitonic network over NP entries (NP a power of two, 4 <= NP <= NW),
// unrolled so that every exchange distance is a compile-time constant
template <uint32_t NP>
__device__ inline void bitonic(WideShared& L, uint64_t (&e)[IPW]) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t k = 2; k <= NP; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            uint64_t b[IPW];
            if (j == 1) {
                b[0] = e[1], b[1] = e[0], b[2] = e[3], b[3] = e[2];
            } else if (j == 2) {
                b[0] = e[2], b[1] = e[3], b[2] = e[0], b[3] = e[1];
            } else if (j < (uint32_t)(IPW * 64)) {
#pragma unroll
                for (int q = 0; q < IPW; ++q) b[q] = lane_xor64(e[q], j / IPW);
            } else {
#pragma unroll
                for (int q = 0; q < IPW; ++q) L.raw[IPW * t + q] = e[q];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < IPW; ++q) b[q] = L.raw[(IPW * t + q) ^ j];
                __syncthreads();
            }
#pragma unroll
            for (int q = 0; q < IPW; ++q) {
                const uint32_t i = IPW * t + q;
                const bool asc = (i & k) == 0, first = (i & j) == 0;
                const uint64_t lo = e[q] < b[q] ? e[q] : b[q], hi = e[q] < b[q] ? b[q] : e[q];
                e[q] = first == asc ? lo : hi;
            }
        }
    }
}

// the same with one entry per thread (entry index = thread index), NP <= WB
template <uint32_t NP>
__device__ inline void bitonic1(WideShared& L, uint64_t& x) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t k = 2; k <= NP; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            uint64_t b;
            if (j < 64) {
                b = lane_xor64(x, j);
            } else {
                L.raw[t] = x;
                __syncthreads();
                b = L.raw[t ^ j];
                __syncthreads();
            }
            const bool asc = (t & k) == 0, first = (t & j) == 0;
            const uint64_t lo = x < b ? x : b, hi = x < b ? b : x;
            x = first == asc ? lo : hi;
        }
    }
}

// the same with two entries per thread (entry index = 2 * thread + q), NP <= 2 * WB
template <uint32_t NP>
__device__ inline void bitonic2(WideShared& L, uint64_t (&e)[2]) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t k = 2; k <= NP; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            uint64_t b[2];
            if (j == 1) {
                b[0] = e[1], b[1] = e[0];
            } else if (j < 128) {
                b[0] = lane_xor64(e[0], j / 2);
                b[1] = lane_xor64(e[1], j / 2);
            } else {
                L.raw[2 * t] = e[0];
                L.raw[2 * t + 1] = e[1];
                __syncthreads();
                b[0] = L.raw[(2 * t) ^ j];
                b[1] = L.raw[(2 * t + 1) ^ j];
                __syncthreads();
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t i = 2 * t + q;
                const bool asc = (i & k) == 0, first = (i & j) == 0;
                const uint64_t lo = e[q] < b[q] ? e[q] : b[q], hi = e[q] < b[q] ? b[q] : e[q];
                e[q] = first == asc ? lo : hi;
            }
        }
    }
}

// the LDS buffer that receives sort_cancel's output (named, not passed as a
// pointer, so that its stores compile to LDS instructions)
enum SortOut { TO_RAW, TO_SRC, TO_TOP0, TO_TOP1 };
__device__ uint32_t sort_cancel(WideShared& L, uint32_t total, SortOut to) {
    static_assert(IPW == 4 && WB == 256 && NW == 1024, "exchange distances assume 4 entries per thread");
    const uint32_t t = threadIdx.x;
    uint64_t* const out = to == TO_RAW ? L.raw : to == TO_SRC ? L.src : L.top[to == TO_TOP1 ? 1 : 0];
    if (total <= (uint32_t)WB) {
        uint64_t x = t < total ? L.raw[t] : PAD;
        __syncthreads();  // raw is reused below
        if (total <= 64) bitonic1<64>(L, x);
        else if (total <= 128) bitonic1<128>(L, x);
        else bitonic1<256>(L, x);
        L.raw[t] = x;
        __syncthreads();
        uint32_t k = 0;
        if (t < total && (t == 0 || L.raw[t - 1] != x)) {
            uint32_t r = 1;
            while (t + r < total && L.raw[t + r] == x) ++r;
            k = r & 1;
        }
        uint32_t kept;
        const uint32_t ex = block_excl_scan(L.ws[WS_SORT], k, kept);
        if (k) out[ex] = x;
        __syncthreads();
        return kept;
    }
    if (total <= 2u * WB) {
        uint64_t e2[2];
        e2[0] = 2 * t < total ? L.raw[2 * t] : PAD;
        e2[1] = 2 * t + 1 < total ? L.raw[2 * t + 1] : PAD;
        __syncthreads();  // raw is reused below
        bitonic2<2 * WB>(L, e2);
        L.raw[2 * t] = e2[0];
        L.raw[2 * t + 1] = e2[1];
        __syncthreads();
        uint32_t keep2[2], kc2 = 0;
        for (int q = 0; q < 2; ++q) {
            const uint32_t j = 2 * t + q;
            uint32_t kk = 0;
            if (j < total && (j == 0 || L.raw[j - 1] != e2[q])) {
                uint32_t r = 1;
                while (j + r < total && L.raw[j + r] == e2[q]) ++r;
                kk = r & 1;
            }
            keep2[q] = kk;
            kc2 += kk;
        }
        uint32_t kept;
        const uint32_t ex = block_excl_scan(L.ws[WS_SORT], kc2, kept);
        uint32_t a = ex;
        for (int q = 0; q < 2; ++q)
            if (keep2[q]) out[a++] = e2[q];
        __syncthreads();
        return kept;
    }
    uint64_t e[IPW];
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
        const uint32_t i = IPW * t + q;
        e[q] = i < total ? L.raw[i] : PAD;
    }
    __syncthreads();  // raw is reused below
    bitonic<1024>(L, e);
#pragma unroll
    for (int q = 0; q < IPW; ++q) L.raw[IPW * t + q] = e[q];
    __syncthreads();
    uint32_t keep[IPW];
    uint32_t kc = 0;
    for (int q = 0; q < IPW; ++q) {
        const uint32_t j = IPW * t + q;
        uint32_t k = 0;
        if (j < total) {
            const uint64_t x = e[q];
            if (j == 0 || L.raw[j - 1] != x) {
                uint32_t r = 1;
                while (j + r < total && L.raw[j + r] == x) ++r;
                k = r & 1;
            }
        }
        keep[q] = k;
        kc += k;
    }
    uint32_t kept;
    const uint32_t ex = block_excl_scan(L.ws[WS_SORT], kc, kept);
    uint32_t a = ex;
    for (int q = 0; q < IPW; ++q)
        if (keep[q]) out[a++] = e[q];
    __syncthreads();
    return kept;
}

// The boundary of the column being reduced is top ^ low ^ pend: top (LDS
// buffer cur, nt entries, ascending), low (global, nl entries, ascending,
// every key below every top key; lmax = its largest key, 0 when empty, keys
// are never 0) and pend (global, np unsorted keys, each at most lmax when it
// was added; pend is empty whenever low is).
struct Col {
    int cur;
    uint32_t nt, nl, np;
    uint64_t lmax;
    __device__ uint32_t n() const { return nt + nl + np; }
};

// Merge pend into low: sort and cancel it in LDS, then one low merge.
__device__ __forceinline__ void flush(const D1K& P, WideShared& L, Col& C, uint64_t*& low, uint64_t* pend, uint64_t*& tmp,
                                      uint64_t* stat,
                      unsigned long long& moved) {
    if (C.np == 0) return;
    const uint32_t t = threadIdx.x;
    __syncthreads();  // pend entries appended by other threads are complete
    {
        uint64_t v[IPW];
#pragma unroll
        for (int q = 0; q < IPW; ++q) {
            const uint32_t i = q * WB + t;
            v[q] = i < C.np ? pend[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < IPW; ++q) {
            const uint32_t i = q * WB + t;
            if (i < C.np) L.raw[i] = v[q];
        }
    }
    __syncthreads();
    // sorted in place: the low merge does not use raw
    const uint32_t m = sort_cancel(L, C.np, TO_RAW);
    C.np = 0;
    if (m == 0) return;
    C.nl = merge_low(P, L, low, C.nl, L.raw, m, tmp, L.top[C.cur ^ 1], pend, stat, moved);
    C.lmax = C.nl ? low[C.nl - 1] : 0;
    __syncthreads();
}

// Boundary ^= L.src[0..m) (ascending, unique): keys up to lmax are appended
// to pend (which is flushed first when they would not fit), the others are
// merged into the top, which spills its smaller entries to low when it
// outgrows TOPCAP.
// t_low and t_top accumulate the time of the two parts (100 MHz clock ticks
// since tp, which is advanced).
__device__ __forceinline__ void merge_col(const D1K& P, WideShared& L, Col& C, uint64_t*& low, uint64_t* pend,
                                          uint64_t* stat, uint32_t m, uint64_t*& tmp,
                          unsigned long long& moved, uint64_t& t_low, uint64_t& t_top, uint64_t& tp) {
    auto lap = [&](uint64_t& acc) {
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        acc += now - tp;
        tp = now;
    };
    if (m == 0) return;
    const uint32_t t = threadIdx.x;
    uint32_t s0 = C.nl ? count_less<uint64_t>(L.src, m, C.lmax + 1) : 0u;
    if (s0 > 0) {
        if (C.np + s0 > P.pcap) {
            flush(P, L, C, low, pend, tmp, stat, moved);
            s0 = C.nl ? count_less<uint64_t>(L.src, m, C.lmax + 1) : 0u;
        }
        for (uint32_t i = t; i < s0; i += WB) pend[C.np + i] = L.src[i];
        C.np += s0;
        __syncthreads();  // L.src is rewritten by the caller next
        lap(t_low);
    }
    if (s0 < m) {
        uint32_t sp;
        const uint32_t r =
            merge_seg(L, L.top[C.cur], C.nt, L.src + s0, m - s0, low + C.nl, L.top[C.cur ^ 1], TOPCAP, TOPKEEP, sp);
        moved += C.nt;
        __syncthreads();
        if (sp > 0) {
            C.nl += sp;
            C.lmax = L.u64s[0];
        }
        C.nt = r - sp;
        C.cur ^= 1;
        __syncthreads();  // L.u64s[0] read by all before it is written again
        lap(t_top);
    }
}

// Load a boundary stored at src[0..len): the largest TOPKEEP entries into the
// top, the rest into low. One of more than NW entries is stored decreasing
// and cancelled; a shorter one is sorted and cancelled here.
__device__ __forceinline__ void load_col(WideShared& L, Col& C, uint64_t* low, const uint64_t* src, uint32_t len) {
    const uint32_t t = threadIdx.x;
    if (len <= (uint32_t)NW) {  // possibly a lane pass's unsorted copy: sort and cancel it
        for (uint32_t i = t; i < len; i += WB) L.raw[i] = ld_rlx64(src + i);
        __syncthreads();
        C.nt = sort_cancel(L, len, C.cur ? TO_TOP1 : TO_TOP0);
        C.nl = 0;
        C.np = 0;
        C.lmax = 0;
        return;
    }
    C.nt = min(len, (uint32_t)TOPKEEP);
    C.nl = len - C.nt;
    C.np = 0;
    {
        uint64_t v[TOPKEEP / WB];
#pragma unroll
        for (int q = 0; q < TOPKEEP / WB; ++q) {
            const uint32_t i = q * WB + t;
            v[q] = i < C.nt ? ld_rlx64(src + (C.nt - 1 - i)) : 0;
        }
#pragma unroll
        for (int q = 0; q < TOPKEEP / WB; ++q) {
            const uint32_t i = q * WB + t;
            if (i < C.nt) L.top[C.cur][i] = v[q];
        }
    }
    for (uint32_t base = 0; base < C.nl; base += 8 * WB) {
        uint64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t i = base + q * WB + t;
            v[q] = i < C.nl ? ld_rlx64(src + (len - 1 - i)) : 0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t i = base + q * WB + t;
            if (i < C.nl) low[i] = v[q];
        }
    }
    C.lmax = C.nl ? ld_rlx64(src + C.nt) : 0;
    __syncthreads();
}

// Flush pend, then move the largest low entries below the top until it holds
// TOPKEEP more entries (or low is empty).
__device__ __forceinline__ void refill(const D1K& P, WideShared& L, Col& C, uint64_t*& low, uint64_t* pend, uint64_t*& tmp,
                                       uint64_t* stat,
                       unsigned long long& moved) {
    flush(P, L, C, low, pend, tmp, stat, moved);
    if (C.nl == 0) return;
    const uint32_t t = threadIdx.x;
    const uint32_t r = min(C.nl, (uint32_t)TOPKEEP);
    uint64_t* nt = L.top[C.cur ^ 1];
    const uint64_t* ot = L.top[C.cur];
    stage(nt, low + (C.nl - r), r);
    for (uint32_t i = t; i < C.nt; i += WB) nt[r + i] = ot[i];
    C.nl -= r;
    C.nt += r;
    C.cur ^= 1;
    C.lmax = C.nl ? low[C.nl - 1] : 0;
    __syncthreads();
}

// Flush pend and save the boundary (C.n() entries afterwards) to the
// publication heap in the decreasing layout; returns the offset or PAD when
// the heap is full.
__device__ __forceinline__ uint64_t save_col(const D1K& P, WideShared& L, Col& C, uint64_t*& low, uint64_t* pend,
                                             uint64_t* stat,
                             uint64_t*& tmp, unsigned long long& moved) {
    flush(P, L, C, low, pend, tmp, stat, moved);
    const uint32_t t = threadIdx.x;
    const uint32_t n = C.n();
    if (t == 0) L.u64s[1] = heap_alloc(P, blockIdx.x, n);
    __syncthreads();
    const uint64_t off = L.u64s[1];
    __syncthreads();
    if (off == NONE) return PAD;
    const uint64_t* T = L.top[C.cur];
    for (uint32_t i = t; i < C.nt; i += WB) st_rlx64(P.heap + off + i, T[C.nt - 1 - i]);
    for (uint32_t i = t; i < C.nl; i += WB) st_rlx64(P.heap + off + C.nt + i, low[C.nl - 1 - i]);
    wait_stores();
    __syncthreads();
    return off;
}

// ---- cooperative full merges ------------------------------------------------
// A full merge low ^ B (both ascending and unique, B stored decreasing) is cut
// into parts of part_span consecutive positions of the merged order (merge
// path), moved by one so that two equal keys, which cancel, always fall in the
// same part. Each part is merged in LDS by one workgroup; the parts' output
// offsets come from a single-pass scan with decoupled look-back over one
// status word per part (flag << 62 | count: 1 = the part's own count, 2 = the
// count of every part up to it). The column's workgroup posts the job on the
// board and takes parts itself; workgroups without a column take parts of
// open jobs. A part waits only for the statuses of lower parts, which were
// taken earlier by running workgroups, so every wait ends. Data moves between
// workgroups with agent-scope release fences (after the writes) and acquire
// fences (before the reads) around the board's atomics.
constexpr uint64_t ST_AGG = 1ull << 62, ST_INC = 2ull << 62, ST_VAL = (1ull << 62) - 1;
constexpr uint32_t PART_SPAN = 2040;   // positions per part: a part's A and B entries fit in TOPCAP LDS keys
constexpr uint32_t SUB = 8;            // positions per thread inside a part
constexpr uint64_t COOP_MIN = 1u << 16;  // smaller full merges stay with the column's workgroup
constexpr uint32_t WAIT_SPIN = 1u << 24;  // bounded waits of the look-back and of the job's end
constexpr uint32_t HELP_SPIN = 1u << 22;  // polls of an idle helper before it gives up helping
static_assert(WB * SUB == TOPCAP && PART_SPAN + 1 <= TOPCAP, "a part fits one top buffer");
static_assert(offsetof(WideShared, flag) + sizeof(uint32_t) * NW - offsetof(WideShared, surv) >= 8 * TOPCAP,
              "the part output stage (surv .. flag) holds a part");

struct Job {
    const uint64_t* a;
    uint64_t na;
    const uint64_t* b;  // decreasing: ascending entry j is b[nb - 1 - j]
    uint64_t nb;
    uint64_t* out;
    uint64_t* stat;
    uint32_t span, nparts;
    int coh;  // a helper: A is read and the output written with coherent accesses
};
__device__ inline uint64_t aget(const Job& J, uint64_t i) { return J.coh ? ld_rlx64(J.a + i) : J.a[i]; }
// B lives in the publication heap: read coherently (a line of it may have
// been cached before it was published)
__device__ inline uint64_t bget(const Job& J, uint64_t j) { return ld_rlx64(J.b + (J.nb - 1 - j)); }

// Bounds (i, j) of the merged prefixes of d0 and d1 positions (A entries
// before equal B entries, then an equal pair kept together), by two 128-ary
// searches over A, one per half of the block.
__device__ void part_bounds(WideShared& L, const Job& J, uint64_t d0, uint64_t d1) {
    const uint32_t t = threadIdx.x, h = t >> 7, k = t & 127;
    const uint64_t d = h ? d1 : d0;
    if (k == 0) {
        L.srch[2 * h] = d > J.nb ? d - J.nb : 0;
        L.srch[2 * h + 1] = d < J.na ? d : J.na;
    }
    __syncthreads();
    for (;;) {
        const uint64_t lo = L.srch[2 * h], hi = L.srch[2 * h + 1];
        if (L.srch[0] >= L.srch[1] && L.srch[2] >= L.srch[3]) break;  // both found
        // f(i) = A[i] <= B[d - 1 - i] holds for a prefix of the range: the
        // answer is the first i where it fails
        const uint64_t n = hi - lo, step = (n + 127) / 128;
        bool f = false;
        if (n > 0) {
            const uint64_t i = lo + k * step;
            if (i < hi) f = aget(J, i) <= bget(J, d - 1 - i);
        }
        const uint64_t bal = __ballot(f);
        if ((t & 63) == 0) L.wcount[t >> 6] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (k == 0 && n > 0) {
            const uint64_t c = L.wcount[2 * h] + L.wcount[2 * h + 1];
            if (c == 0) {
                L.srch[2 * h + 1] = lo;
            } else {
                L.srch[2 * h] = lo + (c - 1) * step + 1;
                L.srch[2 * h + 1] = min(hi, lo + c * step);
            }
        }
        __syncthreads();
    }
    if (k == 0) {
        const uint64_t i = L.srch[2 * h];
        uint64_t j = d - i;
        if (i > 0 && j < J.nb && aget(J, i - 1) == bget(J, j)) ++j;  // the equal pair stays together
        L.srch[2 * h + 1] = j;
    }
    __syncthreads();
}

// the same inside a part held in LDS (XA[0..la), XB[0..lb) ascending), for one
// thread: bounds of the first e merged positions
__device__ inline void local_bound(const uint64_t* XA, uint32_t la, const uint64_t* XB, uint32_t lb, uint32_t e,
                                   uint32_t& i, uint32_t& j) {
    uint32_t lo = e > lb ? e - lb : 0, hi = min(e, la);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (XA[mid] <= XB[e - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    i = lo;
    j = e - lo;
    if (i > 0 && j < lb && XA[i - 1] == XB[j]) ++j;
}

// Merge part p of job J (by the whole block) into J.out at its scanned offset,
// staging its entries in top buffer xb (named by index, so that its accesses
// compile to LDS instructions). Returns false when a look-back wait ran out
// (the kernel's consistency flag is then set).
__device__ __noinline__ bool merge_part(WideShared& L, const Job J, uint32_t p, unsigned long long* ctrs, uint32_t* flags,
                                        int xb) {
    const uint32_t t = threadIdx.x;
    uint64_t* const X = L.top[xb];
    const uint64_t tot = J.na + J.nb;
    const uint64_t d0 = (uint64_t)p * J.span, d1 = min(tot, d0 + J.span);
    part_bounds(L, J, d0, d1);
    const uint64_t i0 = L.srch[0], j0 = L.srch[1], i1 = L.srch[2], j1 = L.srch[3];
    const uint32_t la = (uint32_t)(i1 - i0), lb = (uint32_t)(j1 - j0);
    // X (a free top buffer): A entries, then B entries (ascending)
    for (uint32_t q = t; q < la; q += WB) X[q] = aget(J, i0 + q);
    for (uint32_t q = t; q < lb; q += WB) X[la + q] = bget(J, j0 + q);
    __syncthreads();
    const uint64_t* XA = X;
    const uint64_t* XB = X + la;
    const uint32_t n = la + lb;
    uint32_t si, sj, ei, ej;
    local_bound(XA, la, XB, lb, min(t * SUB, n), si, sj);
    local_bound(XA, la, XB, lb, min(t * SUB + SUB, n), ei, ej);
    // count, then write: a thread's range holds at most SUB + 1 entries
    uint32_t cnt = 0;
    {
        uint32_t i = si, j = sj;
        for (uint32_t q = 0; q <= SUB; ++q) {
            if (i < ei || j < ej) {
                const uint64_t a = i < ei ? XA[i] : PAD, b = j < ej ? XB[j] : PAD;
                if (a < b) { ++cnt; ++i; }
                else if (b < a) { ++cnt; ++j; }
                else { ++i; ++j; }
            }
        }
    }
    uint32_t total;
    const uint32_t off = block_excl_scan(L.ws[WS_SORT], cnt, total);
    // decoupled look-back by wave 0: 64 predecessors per step; the nearest
    // inclusive status ends it, a missing one closer than that is waited for
    bool ok = true;
    if (t < 64) {
        const uint32_t lane = t;
        uint64_t excl = 0;
        if (p == 0) {
            if (lane == 0) st_rlx64(&J.stat[0], ST_INC | total);
        } else {
            if (lane == 0) st_rlx64(&J.stat[p], ST_AGG | total);
            int64_t q = (int64_t)p - 1;  // the window is q, q - 1, ..., q - 63
            uint32_t spin = 0;
            for (;;) {
                const int64_t r = q - (int64_t)lane;
                const uint64_t w = r >= 0 ? ld_rlx64(&J.stat[r]) : ST_INC;  // before part 0: an empty prefix
                const uint64_t inc = __ballot((w & ~ST_VAL) == ST_INC), miss = __ballot(w == 0);
                const uint32_t first = inc ? (uint32_t)__builtin_ctzll(inc) : 64u;
                const uint64_t below = first == 64 ? ~0ull : ((2ull << first) - 1);  // lanes 0 .. first
                if (miss & below) {
                    if (++spin > WAIT_SPIN) {
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint64_t v = ((below >> lane) & 1) ? (w & ST_VAL) : 0;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) v += lane_xor64(v, (uint32_t)d);
                excl += v;
                if (first < 64) break;
                q -= 64;
            }
            if (lane == 0) {
                if (ok) st_rlx64(&J.stat[p], ST_INC | (excl + total));
                else guard_fail(ctrs, flags, G_LOOKBACK);
            }
        }
        if (lane == 0) {
            L.u64s[0] = excl;
            L.ints[0] = ok ? 1 : 0;
        }
    }
    // output stage: surv .. flag (src may hold a round's new keys while its
    // column flushes pend)
    uint64_t* O = &L.surv[0];
    {
        uint32_t i = si, j = sj, o = off;
        for (uint32_t q = 0; q <= SUB; ++q) {
            if (i < ei || j < ej) {
                const uint64_t a = i < ei ? XA[i] : PAD, b = j < ej ? XB[j] : PAD;
                if (a < b) { O[o++] = a; ++i; }
                else if (b < a) { O[o++] = b; ++j; }
                else { ++i; ++j; }
            }
        }
    }
    __syncthreads();
    const uint64_t base = L.u64s[0];
    ok = L.ints[0] != 0;
    if (J.coh) {
        for (uint32_t q = t; q < total; q += WB) st_rlx64(J.out + base + q, O[q]);
        wait_stores();  // complete before the part is counted as done
    } else {
        for (uint32_t q = t; q < total; q += WB) J.out[base + q] = O[q];
    }
    __syncthreads();
    return ok;
}

__device__ inline uint64_t* board_slot(unsigned long long* ctrs, int s) { return (uint64_t*)ctrs + BOARD_BASE + s * BSLOT; }

// low[0..na) ^ b (nb keys stored decreasing) -> tmp by parts, with idle
// workgroups helping when a board slot is free. Returns the output length, or
// ~0u when a wait ran out.
__device__ __noinline__ uint32_t coop_merge(WideShared& L, unsigned long long* ctrs, uint32_t* flags, const uint64_t* b,
                                            uint32_t span, const uint64_t* low, uint32_t na, uint32_t nb, uint64_t* tmp,
                                            uint64_t* stat, int xb) {
    const uint32_t t = threadIdx.x;
    Job J;
    J.a = low;
    J.na = na;
    J.b = b;
    J.nb = nb;
    J.out = tmp;
    J.stat = stat;
    J.span = span;
    J.coh = 0;
    J.nparts = (uint32_t)((na + (uint64_t)nb + J.span - 1) / J.span);
    if (t == 0) atomicAdd(&ctrs[COOP_MERGES], 1ull);
    for (uint32_t q = t; q < J.nparts; q += WB) st_rlx64(&stat[q], 0);
    // every wave: its stores (low, the staged B, the cleared statuses) are
    // complete and written back before the job opens (a barrier waits for LDS
    // operations only)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (t == 0) {
        int slot = -1;
        for (int k = 0; k < NJ; ++k) {
            const int q = (int)((blockIdx.x + k) % NJ);
            if (atomicCAS((unsigned long long*)&board_slot(ctrs, q)[2], 0ull, 1ull) == 0ull) {
                slot = q;
                break;
            }
        }
        if (slot >= 0) {
            uint64_t* B = board_slot(ctrs, slot);
            const uint64_t seq = (ld_rlx64(&B[0]) >> 32) + 1;  // odd: open
            st_rlx64(&B[1], 0);
            st_rlx64(&B[3], (seq << 32) | J.nparts);
            st_rlx64(&B[4], (uint64_t)J.a);
            st_rlx64(&B[5], J.na);
            st_rlx64(&B[6], (uint64_t)J.b);
            st_rlx64(&B[7], J.nb);
            st_rlx64(&B[8], (uint64_t)J.out);
            st_rlx64(&B[9], (uint64_t)J.stat);
            st_rlx64(&B[10], J.span);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicExch((unsigned long long*)&B[0], (unsigned long long)(seq << 32));
            atomicAdd(&ctrs[OPEN_JOBS], 1ull);
        }
        L.ints[1] = slot;
    }
    __syncthreads();
    const int slot = L.ints[1];
    __syncthreads();
    uint64_t* B = slot >= 0 ? board_slot(ctrs, slot) : nullptr;
    bool ok = true;
    for (uint32_t next = 0;;) {
        if (t == 0) {
            uint32_t k = next++;
            if (B) k = (uint32_t)atomicAdd((unsigned long long*)&B[0], 1ull);
            L.ints[2] = (int)min(k, J.nparts);
        }
        __syncthreads();
        const uint32_t k = (uint32_t)L.ints[2];
        __syncthreads();
        if (k >= J.nparts) break;
        ok = merge_part(L, J, k, ctrs, flags, xb) && ok;
        if (B && t == 0) atomicAdd((unsigned long long*)&B[1], 1ull);
    }
    if (t == 0 && B) {
        // every part taken by a helper ends: wait for them, then close the job
        for (uint32_t spin = 0; ld_rlx64(&B[1]) < J.nparts; ++spin) {
            if (spin > WAIT_SPIN) {
                guard_fail(ctrs, flags, G_JOBWAIT);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        const uint64_t seq = ld_rlx64(&B[0]) >> 32;
        atomicExch((unsigned long long*)&B[0], (unsigned long long)((seq + 1) << 32));  // even: closed
        atomicAdd(&ctrs[OPEN_JOBS], ~0ull);
        atomicExch((unsigned long long*)&B[2], 0ull);
    }
    if (t == 0) L.ints[3] = ok ? (int)(uint32_t)(ld_rlx64(&stat[J.nparts - 1]) & ST_VAL) : -1;
    __syncthreads();
    if (B) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the helpers' output, before it is read
    const int r = L.ints[3];
    __syncthreads();
    return r < 0 ? ~0u : (uint32_t)r;
}

// Take parts of open jobs until the pass has no column left in work (or
// nothing to take for a long time, after which helping stops).
__device__ __noinline__ void help(WideShared& L, unsigned long long* ctrs, int64_t nwork, uint32_t* flags) {
    const uint32_t t = threadIdx.x;
    for (uint32_t idle = 0;;) {
        if (t == 0) L.ints[4] = ld_rlx64((const uint64_t*)&ctrs[OPEN_JOBS]) != 0;
        __syncthreads();
        const bool any = L.ints[4] != 0;
        __syncthreads();
        if (!any) {
            // done when no column is left or in work, or when the call failed
            // (a full publication heap stops every column workgroup before
            // the queue is empty: the host grows the heap and runs again)
            if (t == 0)
                L.ints[5] = (ld_rlx64((const uint64_t*)&ctrs[C_NEXT]) >= (uint64_t)nwork &&
                             ld_rlx64((const uint64_t*)&ctrs[C_ACTIVE]) == 0) ||
                            (ld_rlx(flags) & (FLAG_HEAP | FLAG_GUARD | FLAG_WORK)) != 0;
            __syncthreads();
            const bool fin = L.ints[5] != 0;
            __syncthreads();
            if (fin || ++idle > HELP_SPIN) break;
            __builtin_amdgcn_s_sleep(32);
            continue;
        }
        if (t < 64) {
            const int s = (int)((t + blockIdx.x) % NJ);
            const uint64_t* B = board_slot(ctrs, s);
            const uint64_t c = ld_rlx64(&B[0]), sp = ld_rlx64(&B[3]);
            const bool cand = ((c >> 32) & 1) && (c >> 32) == (sp >> 32) && (uint32_t)c < (uint32_t)sp;
            const uint64_t bal = __ballot(cand);
            if (t == 0) {
                int part = -1, slot = -1, done = 0;
                if (bal) {
                    slot = (int)((__builtin_ctzll(bal) + blockIdx.x) % NJ);
                    uint64_t* Bs = board_slot(ctrs, slot);
                    const uint64_t r = atomicAdd((unsigned long long*)&Bs[0], 1ull);
                    if ((r >> 32) & 1) {
                        const uint64_t sp2 = ld_rlx64(&Bs[3]);
                        if ((sp2 >> 32) == (r >> 32) && (uint32_t)r < (uint32_t)sp2) {
                            part = (int)(uint32_t)r;
                            for (int q = 0; q < 12; ++q) L.job[q] = ld_rlx64(&Bs[q]);
                        }
                    }
                }
                L.ints[0] = part;
                L.ints[1] = slot;
                L.ints[2] = done;
            }
        }
        __syncthreads();
        const int part = L.ints[0], slot = L.ints[1], done = L.ints[2];
        Job J;
        if (part >= 0) {
            J.a = (const uint64_t*)L.job[4];
            J.na = L.job[5];
            J.b = (const uint64_t*)L.job[6];
            J.nb = L.job[7];
            J.out = (uint64_t*)L.job[8];
            J.stat = (uint64_t*)L.job[9];
            J.span = (uint32_t)L.job[10];
            J.nparts = (uint32_t)L.job[3];
            J.coh = 1;
        }
        __syncthreads();
        if (part >= 0) {
            merge_part(L, J, (uint32_t)part, ctrs, flags, 0);
            if (t == 0) {  // the part's coherent stores are complete (merge_part waited)
                atomicAdd((unsigned long long*)&board_slot(ctrs, slot)[1], 1ull);
                atomicAdd(&ctrs[HELPED_PARTS], 1ull);
            }
            idle = 0;
            continue;
        }
        if (done || ++idle > HELP_SPIN) break;
        __builtin_amdgcn_s_sleep(4);
    }
}

// Boundary ^= the cached boundary stored decreasingly at P.heap[aoff ..
// aoff + alen), by one merge of the whole column: pend is flushed, the top
// is appended to low, and low and the cached boundary are merged into tmp,
// which becomes low (the two buffers swap). Each step stages TOPCAP low keys
// and NW cached keys and merges those up to the smaller of the two segments'
// last keys, so equal keys are always in the same step and every step
// consumes a full segment of one side. Adding a long boundary in NW-key
// chunks instead rewrites the low part once per chunk.
__device__ __forceinline__ bool add_long(const D1K& P, WideShared& L, Col& C, uint64_t*& low, uint64_t*& tmp, uint64_t* pend,
                         uint64_t* stat, uint64_t aoff, uint32_t alen, unsigned long long& moved) {
    const uint32_t t = threadIdx.x;
    flush(P, L, C, low, pend, tmp, stat, moved);
    {
        const uint64_t* T = L.top[C.cur];
        for (uint32_t i = t; i < C.nt; i += WB) low[C.nl + i] = T[i];
        C.nl += C.nt;
        C.nt = 0;
    }
    __syncthreads();
    // a long merge is split into parts when other workgroups may help: the
    // pass has dedicated helpers, or its queue of columns is exhausted
    if ((uint64_t)C.nl + alen >= P.coop_min && coop_possible(P)) {
        const uint64_t* b = P.heap + aoff;
        uint32_t nb = alen;
        if (alen <= (uint32_t)NW) {
            // possibly a lane pass's unsorted copy: sorted and cancelled, then
            // staged decreasing in pend (empty after the flush above)
            for (uint32_t k = t; k < alen; k += WB) L.raw[k] = ld_rlx64(P.heap + aoff + k);
            __syncthreads();
            nb = sort_cancel(L, alen, TO_SRC);
            // (coherent stores: the parts read B with coherent loads)
            for (uint32_t k = t; k < nb; k += WB) st_rlx64(pend + (nb - 1 - k), L.src[k]);
            __syncthreads();
            b = pend;
        }
        moved += C.nl + alen;
        if (nb == 0) return true;  // everything cancelled
        const uint32_t out = coop_merge(L, P.ctrs, P.flags, b, P.part_span, low, C.nl, nb, tmp, stat, 0);
        if (out == ~0u) return false;
        uint64_t* sw = low;
        low = tmp;
        tmp = sw;
        C.nl = out;
        C.lmax = out ? low[out - 1] : 0;
        __syncthreads();
        return true;
    }
    // a boundary of up to NW entries may be a lane pass's unsorted copy: it is
    // sorted and cancelled into L.src once; a longer one is stored decreasing
    const bool small = alen <= (uint32_t)NW;
    uint32_t nb = alen;
    if (small) {
        for (uint32_t k = t; k < alen; k += WB) L.raw[k] = ld_rlx64(P.heap + aoff + k);
        __syncthreads();
        nb = sort_cancel(L, alen, TO_SRC);
    }
    const uint32_t na = C.nl;
    uint64_t* X = L.top[0];
    uint32_t i = 0, j = 0, out = 0;
    while (i < na || j < nb) {
        const uint32_t la = min((uint32_t)TOPCAP, na - i), lb = min((uint32_t)NW, nb - j);
        stage(X, low + i, la);
        if (!small) {
            uint64_t v[IPW];
#pragma unroll
            for (int q = 0; q < IPW; ++q) {
                const uint32_t k = q * WB + t;
                v[q] = k < lb ? ld_rlx64(P.heap + aoff + (alen - 1 - (j + k))) : 0;
            }
#pragma unroll
            for (int q = 0; q < IPW; ++q) {
                const uint32_t k = q * WB + t;
                if (k < lb) L.src[k] = v[q];
            }
        }
        __syncthreads();
        const uint64_t* S = small ? L.src + j : L.src;  // this step's segment of the boundary
        uint64_t bound = PAD;  // keys are below PAD
        if (i + la < na) bound = X[la - 1];
        if (j + lb < nb) bound = min(bound, S[lb - 1]);
        const uint32_t ta = bound == PAD ? la : count_less<uint64_t>(X, la, bound + 1);
        const uint32_t tb = bound == PAD ? lb : count_less<uint64_t>(S, lb, bound + 1);
        uint32_t sp;
        out += merge_seg(L, X, ta, S, tb, tmp + out, nullptr, 0, 0, sp);
        __syncthreads();
        i += ta;
        j += tb;
    }
    moved += na + alen;
    uint64_t* sw = low;
    low = tmp;
    tmp = sw;
    C.nl = out;
    C.lmax = out ? low[out - 1] : 0;
    __syncthreads();
    return true;
}

__global__ __launch_bounds__(WB, 2) void k_d1_wide(D1K P) {
    __shared__ WideShared L;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    // per column slot: low, tmp, pend, and the part statuses of cooperative merges
    const int64_t slot_words = 2 * P.K + PCAP + P.K / P.part_span + 2;
    uint64_t* low = P.scratch + (int64_t)blockIdx.x * slot_words;
    uint64_t* tmp = low + P.K;
    uint64_t* pend = tmp + P.K;
    uint64_t* stat = pend + PCAP;
    const int64_t V = P.g.V;
    unsigned long long steps = 0, evictions = 0, adds = 0, rounds = 0, expanded = 0, moved = 0, longs = 0;
    unsigned long long r_stop = 0, r_cap = 0, r_taken = 0;  // rounds ended at an edge / by the merge list; entries taken
    for (;;) {
        if ((int64_t)blockIdx.x >= P.nslots) break;  // a helper only
        // no new column once the call has failed (it is run again or reported)
        if (t == 0)
            L.u64s[0] = (ld_rlx(P.flags) & (FLAG_HEAP | FLAG_GUARD | FLAG_WORK)) ? (uint64_t)P.nwork
                                                                                 : atomicAdd(&P.ctrs[C_NEXT], 1ull);
        __syncthreads();
        const uint64_t next = L.u64s[0];
        __syncthreads();
        if ((int64_t)next >= P.nwork) break;
        // Deferred columns are taken last-deferred first: the column that ran
        // longest in the previous pass before outgrowing it tends to be the
        // longest here too, and its chain of rounds then starts with the pass
        // instead of after thousands of short columns (smooth512: 43 -> 35 ms).
        const uint64_t wi = (uint64_t)P.nwork - 1 - next;
        uint32_t c = P.work_col[wi];
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();  // 100 MHz clock
        // time per phase (thread 0): window, sort, round merge, owner rule, additions, claims
        uint64_t ph[N_PHASE] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        uint64_t tp = t0;
        auto lap = [&](int i) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            ph[i] += now - tp;
            tp = now;
        };
        const unsigned long long rounds0 = rounds, adds0 = adds;
        uint32_t nmax = 0;
        uint64_t nc_min = PAD;  // ablation without caching: the lowest pivot re-reduced in place
        Col C;
        C.cur = 0;
        {
            const uint64_t off = P.work[wi];
            const uint32_t n0 = P.work_len[wi];
            if ((int64_t)n0 > P.K) {
                if (t == 0) atomicOr(P.flags, FLAG_WORK);
                break;
            }
            if (off + n0 > (uint64_t)P.heap_cap) {
                if (t == 0) guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                break;
            }
            if (t == 0) atomicAdd(&P.ctrs[C_ACTIVE], 1ull);
            load_col(L, C, low, P.heap + off, n0);
        }
        bool stop = false;
        uint32_t retries = 0;
        for (int64_t guard = 0;; ++guard) {
            if (guard > ((int64_t)1 << 24)) {
                if (t == 0) guard_fail(P.ctrs, P.flags, G_WSTEPS);
                stop = true;
                break;
            }
            ++steps;
            if (C.n() == 0) break;  // zero column
            if (C.nt < (uint32_t)WB && (C.nl > 0 || C.np > 0)) {
                refill(P, L, C, low, pend, tmp, stat, moved);
                lap(9);
                if (C.n() == 0) break;  // everything cancelled in the flush
            }
            // a look-again (an owner that moved on, a lost claim) resolves once the
            // other column has published; a long run of them means corrupted state
            if (retries > MAX_RETRIES) {
                if (t == 0) guard_fail(P.ctrs, P.flags, G_WRETRIES);
                stop = true;
                break;
            }
            const uint64_t* T = L.top[C.cur];
            // Scan the top window. Above the first stopping edge, every regular tail
            // (add its partner's boundary) and every critical edge owned by an earlier
            // column with a short cached boundary (add it) is processed this round.
            // Edges that are never a pivot (vertex partners, D0-paired edges) are
            // kept without stopping. A possible pivot (free or later-owned critical
            // edge) stops the round, and so does an earlier-owned one with a long
            // cached boundary, which is added in order when it reaches the top: adding
            // long boundaries out of order inflates the boundaries cached later. The
            // top must be processable, otherwise the owner rule runs. The window
            // entries above the stop leave the top; the kept ones come back with the
            // new keys.
            const uint32_t k = min(C.nt, (uint32_t)WB);
            uint64_t wkey = 0, nk0 = PAD, nk1 = PAD, zoff = 0;
            int64_t cva = 0, cw = 0;  // a regular entry: its higher endpoint and its partner's third vertex
            uint32_t cra = 0, crw = 0;
            uint32_t nkeys = 0;  // keys this entry contributes when processed
            bool batched = false;
            int cls = 0;  // 0 none/stop, 1 processable, 2 kept (never a pivot)
            if ((uint32_t)t < k) {
                wkey = T[C.nt - 1 - t];
                const EdgeDec e = edecode(P.g, P.order, P.bpr, wkey);
                // the gradient code and the owner are loaded together
                const uint8_t code = e.mask ? P.G[(int64_t)e.mask * V + e.lo] : (uint8_t)0xFE;
                const uint32_t o = e.mask ? ld_rlx(&P.owner1[e.id]) : EMPTY32;
                if (code < 27) {
                    cw = e.lo + lin27(P.g, code);
                    const uint32_t rw = P.rank[cw];
                    nk0 = ekey_r(P.bpr, e.ra, rw);
                    nk1 = ekey_r(P.bpr, e.rb, rw);
                    cva = e.va;
                    cra = e.ra;
                    crw = rw;
                    nkeys = 2;
                    cls = 1;
                } else if (code == CODE_CRIT) {
                    if (o == OWN_D0) {
                        cls = 2;
                    } else if (o != EMPTY32 && o < c && !P.no_cache) {
                        // (the top too: its short cached boundary is added in the
                        // round like the others'). The cached boundary's head is
                        // checked against wkey when its entries are loaded.
                        const uint64_t bo = ld_rlx64(&P.bndptr[o]);
                        const uint32_t zl = (uint32_t)(bo & 0xFFFFFF) - 1;
                        // (a pointer outside the heap is not batched: the
                        // addition at the top reports it)
                        if (heap_span_ok(P, bo) && zl <= BATCH_ADD_MAX) {
                            zoff = bo >> 24;
                            nkeys = zl;
                            batched = true;
                            cls = 1;
                        }
                    }
                } else if (code >= 0x80 && code < 0xFE) {
                    cls = 2;  // vertex partner
                }
            }
            if (cls == 2) nkeys = 1;
            // first stopping entry (t >= k counts as one) and, per wave, the slots of
            // the entries before its own first stop
            const bool stopbit = (uint32_t)t >= k || cls == 0;
            const uint64_t sm = __ballot(stopbit);
            const bool stop_in_wave_before = (sm & ((1ull << lane) - 1)) != 0;
            const uint32_t need = (!stopbit && !stop_in_wave_before) ? nkeys : 0u;
            const uint32_t inc = wave_incl_scan(need);
            if (lane == 63) L.ws[WS_ROUND][wv] = inc;
            if (lane == 0) L.wstop[wv] = sm ? (uint32_t)(wv * 64 + __builtin_ctzll(sm)) : (uint32_t)WB;
            if (t == 0) {
                L.ints[0] = cls;
                L.ints[3] = 0;
                L.nextra = 0;
            }
            __syncthreads();
            uint32_t stop0 = WB, before = 0;
#pragma unroll
            for (int i = 0; i < NWAVE; ++i) {
                stop0 = min(stop0, L.wstop[i]);
                before += i < wv ? L.ws[WS_ROUND][i] : 0u;
            }
            const bool top_go = L.ints[0] == 1;
            lap(0);
            if (top_go) {
                // entries t < stop0 whose keys fit in the merge list take part; the
                // slot ends grow with t, so they form a prefix of the window
                const uint32_t slot = before + inc - need;
                const bool incl = (uint32_t)t < stop0 && slot + need <= (uint32_t)NW;
                const bool go = incl && cls == 1;
                // Keys of the entries before the stop (waves up to the stop's
                // wave: entries after a wave's first stop need nothing). When
                // they all fit, every entry above the stop key is processed this
                // round, and an expansion may go on along its lower star: the
                // edge {va, w} it leaves is replaced by {w, w'} and {va, w'} via
                // the partner {va, w, w'} while {va, w} is regular and above the
                // stop key (up to CHAIN times; the extra keys go after the
                // entries' own). Such an edge, if it is in the column, is a
                // regular window entry expanded by its own thread this round, so
                // the two expansions cancel mod 2 and nothing unexpanded is left
                // twice; below the stop key that would not hold.
                uint32_t total_base = 0;
#pragma unroll
                for (int i = 0; i < NWAVE; ++i) total_base += i <= (int)(min(stop0, (uint32_t)(WB - 1)) >> 6) ? L.ws[WS_ROUND][i] : 0u;
                const bool chains = total_base <= (uint32_t)NW;
                if (go && !batched && chains) {
                    const uint64_t stopkey = stop0 < C.nt ? T[C.nt - 1 - stop0] : (C.nl ? C.lmax : 0ull);
                    int64_t w = cw;
                    uint32_t rw = crw;
                    if (ekey_r(P.bpr, cra, rw) > stopkey) {
                        int64_t lo;
                        uint8_t c2 = P.G[(int64_t)edge_mask(P.g, cva, w, lo) * V + lo];
                        for (int q = 0; q < CHAIN && c2 < 27; ++q) {  // {va, w} regular
                            const uint32_t sl = total_base + atomicAdd(&L.nextra, 1u);
                            if (sl >= (uint32_t)NW) break;
                            const int64_t w2 = lo + lin27(P.g, c2);
                            // the rank of w' and the code of {va, w'} are loaded together
                            int64_t lo2;
                            const uint8_t c3 = P.G[(int64_t)edge_mask(P.g, cva, w2, lo2) * V + lo2];
                            const uint32_t rw2 = P.rank[w2];
                            L.raw[sl] = ekey_r(P.bpr, rw, rw2);
                            L.surv[sl] = NONE;
                            w = w2;
                            rw = rw2;
                            lo = lo2;
                            c2 = c3;
                            if (ekey_r(P.bpr, cra, rw) <= stopkey) break;
                        }
                    }
                    nk0 = ekey_r(P.bpr, cra, rw);
                }
                if (incl) {
                    if (batched) {
                        for (uint32_t j = 0; j < nkeys; ++j) L.surv[slot + j] = zoff + 1 + j;
                    } else if (go) {
                        L.raw[slot] = nk0;
                        L.raw[slot + 1] = nk1;
                        L.surv[slot] = NONE;
                        L.surv[slot + 1] = NONE;
                    } else {
                        L.raw[slot] = wkey;  // kept: re-inserted
                        L.surv[slot] = NONE;
                    }
                }
                // included entries form a prefix: count them, and the last one of
                // each wave gives the end of its slots
                {
                    const uint64_t im = __ballot(incl);
                    if (lane == 0) {
                        L.wcnt[wv] = (uint32_t)__popcll(im);
                        if (!im) L.wend[wv] = 0;
                    }
                    if (incl && (im >> lane) == 1ull) L.wend[wv] = slot + need;
                }
                __syncthreads();
                lap(1);
                uint32_t stop_at = 0, total = 0;
#pragma unroll
                for (int i = 0; i < NWAVE; ++i) {
                    stop_at += L.wcnt[i];
                    total = max(total, L.wend[i]);
                }
                if (chains) total = min((uint32_t)NW, total_base + L.nextra);
                // entries of the batched cached boundaries, one load per slot, and
                // the boundaries' heads, all in flight together
                {
                    uint64_t v[IPW];
#pragma unroll
                    for (int q = 0; q < IPW; ++q) {
                        const uint32_t j = q * WB + t;
                        const uint64_t a = j < total ? L.surv[j] : NONE;
                        v[q] = a != NONE ? ld_rlx64(P.heap + a) : 0;
                    }
                    const uint64_t head = (incl && batched) ? ld_rlx64(P.heap + zoff) : wkey;
#pragma unroll
                    for (int q = 0; q < IPW; ++q) {
                        const uint32_t j = q * WB + t;
                        if (j < total && L.surv[j] != NONE) L.raw[j] = v[q];
                    }
                    if (head != wkey) L.ints[3] = 1;  // the owner moved on
                }
                __syncthreads();
                const bool retry = L.ints[3] != 0;
                __syncthreads();  // L.ints[3] is reset by the next round
                lap(2);
                if (retry) {  // nothing changed yet: look again
                    ++retries;
                    continue;
                }
                retries = 0;
                expanded += go ? 1 : 0;
                const uint32_t m = sort_cancel(L, total, TO_SRC);
                lap(3);
                ++rounds;
                if ((int64_t)(C.n() - stop_at) + m > P.K) {
                    // no room: save the column unchanged for the next pass
                    const uint64_t off = save_col(P, L, C, low, pend, stat, tmp, moved);
                    if (off == PAD) {
                        if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                        stop = true;
                        break;
                    }
                    if (t == 0) defer_column(P, c, off, C.n());
                    break;
                }
                r_stop += stop0 < k ? 1 : 0;
                r_cap += stop_at < stop0 ? 1 : 0;
                r_taken += stop_at;
                C.nt -= stop_at;  // the window entries above the stop leave
                merge_col(P, L, C, low, pend, stat, m, tmp, moved, ph[4], ph[5], tp);
                nmax = max(nmax, C.n());
                continue;
            }
            // the top edge is not a regular tail
            const uint64_t tau = T[C.nt - 1];
            if (t == 0) {
                const EdgeDec te = edecode(P.g, P.order, P.bpr, tau);
                const uint8_t code = te.mask ? P.G[(int64_t)te.mask * V + te.lo] : (uint8_t)0xFE;
                int action = 0;
                uint32_t o = 0;
                if (code != CODE_CRIT) {
                    action = -1;  // the top of a cycle cannot be a vertex's partner
                } else {
                    o = ld_rlx(&P.owner1[te.id]);
                    if (o == OWN_D0) action = -1;
                    else if (o == EMPTY32 || o > c) action = 1;  // claim
                    else action = 2;                             // add the owner's boundary
                }
                L.ints[4] = action;
                L.ints[5] = (int)o;
                L.ints[6] = (int)te.id;
            }
            __syncthreads();
            const int action = L.ints[4];
            const uint32_t o = (uint32_t)L.ints[5];
            const uint32_t eid = (uint32_t)L.ints[6];
            __syncthreads();
            lap(6);
            if (action < 0) {
                if (t == 0) guard_fail(P.ctrs, P.flags, G_WTOP);
                stop = true;
                break;
            }
            if (action == 1) {
                const uint64_t off = save_col(P, L, C, low, pend, stat, tmp, moved);
                const uint32_t n = C.n();
                if (off == PAD) {
                    if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                    stop = true;
                    break;
                }
                if (t == 0) {
                    st_rlx64(&P.bndptr[c], (off << 24) | n);
                    wait_stores();
                    L.ints[7] = cas32(&P.owner1[eid], o, c) ? 1 : 0;
                    if (L.ints[7] && o != EMPTY32) L.u64s[2] = ld_rlx64(&P.bndptr[o]);
                }
                __syncthreads();
                lap(8);
                const int won = L.ints[7];
                const uint64_t bo = L.u64s[2];
                __syncthreads();
                if (!won) {
                    ++retries;
                    continue;
                }
                if (o == EMPTY32) break;  // settled
                if (!heap_span_ok(P, bo)) {
                    if (t == 0) guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                    stop = true;
                    break;
                }
                ++evictions;
                c = o;
                nc_min = PAD;
                const uint32_t bl = (uint32_t)(bo & 0xFFFFFF);
                const uint64_t boff = bo >> 24;
                if ((int64_t)bl > P.K) {
                    if (t == 0) defer_column(P, c, boff, bl);
                    break;
                }
                load_col(L, C, low, P.heap + boff, bl);
                lap(8);
                continue;
            }
            if (P.no_cache && tau >= nc_min && t == 0) atomicAdd(&P.ctrs[NC_FALLBACKS], 1ull);
            if (P.no_cache && tau < nc_min) {
                // ablation without caching: add the boundary of o's 2-saddle
                // (its three edges, the top at or above tau) and reduce it
                // again, below every pivot re-reduced before in this column
                // (the re-reduction follows owners that evictions may have
                // changed: pivots met inside it, and one that comes back, get
                // cached boundaries)
                nc_min = tau;
                if ((int64_t)C.n() + 3 > P.K) {
                    const uint64_t off = save_col(P, L, C, low, pend, stat, tmp, moved);
                    if (off == PAD) {
                        if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                        stop = true;
                        break;
                    }
                    if (t == 0) defer_column(P, c, off, C.n());
                    break;
                }
                ++adds;
                if (t < 3) {
                    uint64_t k3[3];
                    tri_edge_keys(P, P.cols[o], k3);
                    L.raw[t] = t == 0 ? k3[0] : t == 1 ? k3[1] : k3[2];
                }
                __syncthreads();
                const uint32_t m = sort_cancel(L, 3, TO_SRC);
                uint64_t tq = 0, u0 = 0, u1 = 0;
                merge_col(P, L, C, low, pend, stat, m, tmp, moved, u0, u1, tq);
                nmax = max(nmax, C.n());
                lap(7);
                continue;
            }
            // action 2: boundary += Boundary(o), merged in chunks (largest keys first)
            if (t == 0) {
                const uint64_t b = ld_rlx64(&P.bndptr[o]);
                L.u64s[3] = b;
                L.ints[7] = b == EMPTY64 ? 0 : !heap_span_ok(P, b) ? 2 : ld_rlx64(P.heap + (b >> 24)) == tau ? 1 : 0;
            }
            __syncthreads();
            const uint64_t b = L.u64s[3];
            const int ok = L.ints[7];
            __syncthreads();
            if (ok == 2) {
                if (t == 0) guard_fail(P.ctrs, P.flags, G_HEAPPTR);
                stop = true;
                break;
            }
            if (!ok) {  // o moved on: look again
                ++retries;
                continue;
            }
            retries = 0;
            const uint64_t aoff = b >> 24;
            const uint32_t alen = (uint32_t)(b & 0xFFFFFF);
            if ((int64_t)C.n() + alen > P.K) {
                // the sum might not fit: hand the column, unchanged, to the next pass
                const uint64_t off = save_col(P, L, C, low, pend, stat, tmp, moved);
                if (off == PAD) {
                    if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                    stop = true;
                    break;
                }
                if (t == 0) defer_column(P, c, off, C.n());
                break;
            }
            ++adds;
            if (alen > P.long_add) {
                ++longs;
                if (!add_long(P, L, C, low, tmp, pend, stat, aoff, alen, moved)) {
                    stop = true;
                    break;
                }
                nmax = max(nmax, C.n());
                lap(7);
                continue;
            }
            if (alen <= (uint32_t)NW) {  // possibly unsorted: sort and cancel, then merge
                for (uint32_t k = t; k < alen; k += WB) L.raw[k] = ld_rlx64(P.heap + aoff + k);
                __syncthreads();
                const uint32_t m = sort_cancel(L, alen, TO_SRC);
                uint64_t tq = 0, u0 = 0, u1 = 0;
                merge_col(P, L, C, low, pend, stat, m, tmp, moved, u0, u1, tq);
                nmax = max(nmax, C.n());
                lap(7);
                continue;
            }
            for (uint32_t base = 0; base < alen; base += NW) {
                const uint32_t m = min((uint32_t)NW, alen - base);
                uint64_t v[IPW];
#pragma unroll
                for (int q = 0; q < IPW; ++q) {
                    const uint32_t j = q * WB + t;
                    v[q] = j < m ? ld_rlx64(P.heap + aoff + base + (m - 1 - j)) : 0;
                }
#pragma unroll
                for (int q = 0; q < IPW; ++q) {
                    const uint32_t j = q * WB + t;
                    if (j < m) L.src[j] = v[q];
                }
                __syncthreads();
                uint64_t tq = 0;
                uint64_t u0 = 0, u1 = 0;
                merge_col(P, L, C, low, pend, stat, m, tmp, moved, u0, u1, tq);
            }
            nmax = max(nmax, C.n());
            lap(7);
        }
        __syncthreads();
        if (t == 0) {
            atomicAdd(&P.ctrs[C_ACTIVE], ~0ull);  // this column is done
            const uint64_t dt = __builtin_amdgcn_s_memrealtime() - t0;
            atomicMax(&P.ctrs[C_TMAX], (unsigned long long)dt);
            atomicAdd(&P.ctrs[C_TSUM], (unsigned long long)dt);
            atomicMax(&P.ctrs[C_RMAX], rounds - rounds0);
            atomicMax(&P.ctrs[C_AMAX], adds - adds0);
            atomicMax(&P.ctrs[C_NMAX], (unsigned long long)nmax);
            if (dt > 100000) {
                atomicAdd(&P.ctrs[C_SLOW], 1ull);
                atomicAdd(&P.ctrs[C_PHASE + N_PHASE], rounds - rounds0);
                atomicAdd(&P.ctrs[C_PHASE + N_PHASE + 1], adds - adds0);
                for (int i = 0; i < N_PHASE; ++i) atomicAdd(&P.ctrs[C_PHASE + i], (unsigned long long)ph[i]);
            }
        }
        if (stop) break;
    }
    help(L, P.ctrs, P.nwork, P.flags);
    if (expanded) atomicAdd(&P.ctrs[C_EXPANDED], expanded);
    if (t == 0) {
        atomicAdd(&P.ctrs[C_STEPS], steps);
        atomicAdd(&P.ctrs[C_EVICT], evictions);
        atomicAdd(&P.ctrs[C_ADDS], adds);
        atomicAdd(&P.ctrs[C_ROUNDS], rounds);
        atomicAdd(&P.ctrs[C_MOVED], moved);
        atomicAdd(&P.ctrs[C_LONG], longs);
        atomicAdd(&P.ctrs[C_RSTOP], r_stop);
        atomicAdd(&P.ctrs[C_RCAP], r_cap);
        atomicAdd(&P.ctrs[C_RTAKEN], r_taken);
    }
}

// paired1 null (no sandwich): no 1-saddle is set aside
__global__ void k_init_owner(const uint32_t* c1, const uint8_t* paired1, int64_t m1, uint32_t* owner1) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i < m1) owner1[c1[i]] = (paired1 && paired1[i]) ? OWN_D0 : EMPTY32;
}

// paired2_desc null (no sandwich): every 2-saddle is a column
__global__ void k_colflags(const uint8_t* paired2_desc, int64_t m2, uint32_t* flag) {
    const int64_t k = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (k < m2) flag[k] = (paired2_desc && paired2_desc[m2 - 1 - k]) ? 0u : 1u;
}

__global__ void k_compact(const uint32_t* c2, const uint8_t* paired2_desc, const uint32_t* pos, int64_t m2,
                          uint32_t* cols) {
    const int64_t k = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (k < m2 && !(paired2_desc && paired2_desc[m2 - 1 - k])) cols[pos[k]] = c2[k];
}

constexpr int EMIT_ITEMS = 16;  // columns per lane of k_emit_pairs: one list atomic per 4096 columns

__global__ __launch_bounds__(DB) void k_emit_pairs(GridDev g, const uint32_t* order, int bpr, const uint32_t* cols,
                                                   int64_t ncols, const uint64_t* bndptr, const uint64_t* heap,
                                                   const uint32_t* owner1, uint64_t* key, uint32_t* death,
                                                   uint32_t* cnt) {
    block_append<DB, EMIT_ITEMS>(
        cnt, (int64_t)blockIdx.x * DB * EMIT_ITEMS, ncols,
        [&](int64_t c, uint64_t& p) {
            const uint64_t b = bndptr[c];
            if (b == EMPTY64) return false;
            const EdgeDec e = edecode(g, order, bpr, heap[b >> 24]);
            p = e.id;
            return owner1[e.id] == (uint32_t)c;
        },
        [&](int64_t c, uint64_t p, uint32_t at) {
            key[at] = p;
            death[at] = cols[c];
        });
}

__global__ void k_emit_ess1(const uint32_t* c1, const uint8_t* paired1, int64_t m1, const uint32_t* owner1,
                            uint64_t* key, uint32_t* death, uint32_t* cnt) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i >= m1 || paired1[i]) return;
    if (owner1[c1[i]] != EMPTY32) return;
    const uint32_t at = wave_append(true, cnt);
    key[at] = (1ull << 32) | c1[i];
    death[at] = EMPTY32;
}

// paired2_desc non-null: the columns are every 2-saddle (no sandwich), and
// those D2 paired are no essential class
__global__ void k_emit_ess2(GridDev g, const uint32_t* order, int bpr, const uint32_t* cols, int64_t ncols,
                            const uint64_t* bndptr, const uint64_t* heap, const uint32_t* owner1,
                            const uint8_t* paired2_desc, uint64_t* key, uint32_t* death, uint32_t* cnt) {
    const int64_t c = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (c >= ncols) return;
    if (paired2_desc && paired2_desc[ncols - 1 - c]) return;
    const uint64_t b = bndptr[c];
    if (b != EMPTY64) {
        const EdgeDec e = edecode(g, order, bpr, heap[b >> 24]);
        if (owner1[e.id] == (uint32_t)c) return;
    }
    const uint32_t at = wave_append(true, cnt);
    key[at] = (1ull << 32) | cols[c];
    death[at] = EMPTY32;
}

// ---- persistent 1-cycle generators (Sec. 8) -------------------------------
// The cycle of a finite D1 pair is the boundary its 2-saddle published when
// it claimed the birth edge: a lane pass publishes {pivot} + its working heap
// as it stood (entries may repeat and count mod 2), a workgroup pass a
// sorted, cancelled list. The export gathers those entries per pair, sorts
// them by (pair, edge id) and keeps the keys that occur an odd number of times.

// (birth edge id, column) of every column that owns its pivot
__global__ __launch_bounds__(DB) void k_gen_pairs(GridDev g, const uint32_t* order, int bpr, int64_t ncols,
                                                  const uint64_t* bndptr, const uint64_t* heap,
                                                  const uint32_t* owner1, uint32_t* edge, uint32_t* col,
                                                  uint32_t* cnt) {
    block_append<DB, EMIT_ITEMS>(
        cnt, (int64_t)blockIdx.x * DB * EMIT_ITEMS, ncols,
        [&](int64_t c, uint64_t& p) {
            const uint64_t b = bndptr[c];
            if (b == EMPTY64) return false;
            const EdgeDec e = edecode(g, order, bpr, heap[b >> 24]);
            p = e.id;
            return owner1[e.id] == (uint32_t)c;
        },
        [&](int64_t c, uint64_t p, uint32_t at) {
            edge[at] = (uint32_t)p;
            col[at] = (uint32_t)c;
        });
}

// published length of the boundary of pair i
__global__ void k_gen_len(const uint32_t* col, int64_t n, const uint64_t* bndptr, uint32_t* len) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i < n) len[i] = (uint32_t)(bndptr[col[i]] & 0xFFFFFFull);
}

// entry j of the concatenated boundaries -> pair << 32 | edge id; off is the
// exclusive scan of the lengths, every one of which is at least 1
__global__ void k_gen_gather(GridDev g, const uint32_t* order, int bpr, const uint32_t* col, const uint32_t* off,
                             int64_t n, int64_t total, const uint64_t* bndptr, const uint64_t* heap,
                             uint64_t* key) {
    const int64_t j = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (j >= total) return;
    int64_t lo = 0, hi = n - 1;  // the last pair whose offset is <= j
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const uint64_t b = bndptr[col[lo]];
    const EdgeDec e = edecode(g, order, bpr, heap[(b >> 24) + (uint64_t)(j - (int64_t)off[lo])]);
    key[j] = ((uint64_t)lo << 32) | e.id;
}

// sorted keys: one copy of every key that occurs an odd number of times
__global__ void k_gen_keep(const uint64_t* key, int64_t total, uint32_t* keep) {
    const int64_t j = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (j >= total) return;
    const uint64_t k = key[j];
    uint32_t odd = 0;
    if (j == 0 || key[j - 1] != k) {
        int64_t r = j + 1;
        while (r < total && key[r] == k) ++r;
        odd = (uint32_t)((r - j) & 1);
    }
    keep[j] = odd;
}

__global__ void k_gen_write(const uint64_t* key, const uint32_t* keep, const uint32_t* pos, int64_t total,
                            int64_t* edges, uint32_t* pair_of) {
    const int64_t j = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (j >= total || !keep[j]) return;
    const uint32_t p = pos[j];
    edges[p] = (int64_t)(key[j] & 0xFFFFFFFFull);
    pair_of[p] = (uint32_t)(key[j] >> 32);
}

// offsets[i] = the first output position of pair i; offsets[n] = ne
__global__ void k_gen_offsets(const uint32_t* pair_of, int64_t ne, int64_t n, int64_t* offsets) {
    const int64_t p = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (p == 0) offsets[n] = ne;
    if (p >= ne) return;
    const uint32_t i = pair_of[p];
    if (p == 0 || pair_of[p - 1] != i) offsets[i] = p;
}

// every cycle holds at least its birth edge: an offset left at -1 is a fault
__global__ void k_gen_check(const int64_t* offsets, int64_t n, uint32_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i < n && offsets[i] < 0) atomicOr(flags, FLAG_GUARD);
}

// (re)allocate p to at least `bytes`; total counts the bytes D1 holds and may
// not pass limit (0 = no limit): the context's HBM budget left for D1
int grow(void*& p, size_t& cap, size_t bytes, size_t& total, size_t limit) {
    if (cap >= bytes) return 0;
    if (limit && total - cap + bytes > limit) return -1;
    if (p) (void)hipFree(p);
    total -= cap;
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    cap = bytes;
    total += bytes;
    return 0;
}

}  // namespace

int d1_run(D1State& s, const D1Inputs& in, hipStream_t st, size_t budget_left, std::string& err) {
    s.gen_n = -1;  // generators of an earlier run are stale
    s.limit = budget_left;
    const int64_t V = in.g.V;
    const int64_t m2 = in.m2;
    s.g = in.g;
    s.order = in.order;
    s.bpr = in.bpr;
    auto oom = [&](const char* what) {
        err = std::string("D1: cannot allocate ") + what;
        return -3;  // DMS_E_NOMEM
    };
    const size_t ctr_bytes = 8 * (size_t)N_CTR_WORDS;
    if (!s.ctrs && hipMalloc(&s.ctrs, ctr_bytes) != hipSuccess) return oom("counters");
    if (grow(s.colflag, s.colflag_cap, 4 * (m2 + 1), s.bytes, s.limit)) return oom("column flags");
    if (grow(s.cols, s.cols_cap, 4 * (m2 + 1), s.bytes, s.limit)) return oom("columns");
    if (grow(s.scanpart, s.scanpart_cap, 4 * scan_part_size(m2 + 1), s.bytes, s.limit)) return oom("scan");
    if (grow(s.owner1, s.owner1_cap, 4 * 7 * V, s.bytes, s.limit)) return oom("owners");
    for (int d = 0; d < 6; ++d) s.stats[d] = 0;
    for (int d = 0; d < MAX_PASSES; ++d) s.pass_work[d] = s.pass_us[d] = 0;
    for (int d = 0; d < 4; ++d) s.wide[d] = 0;
    for (int d = 0; d < 6; ++d) s.wide_t[d] = 0;
    for (int d = 0; d < 12; ++d) s.wide_ph[d] = 0;
    s.coop[0] = s.coop[1] = 0;
    s.nc_fallbacks = 0;
    // unpaired 2-saddles (every 2-saddle without the sandwich), ascending
    const uint8_t* p2 = in.no_sandwich ? nullptr : in.paired2_desc;
    const uint8_t* p1 = in.no_sandwich ? nullptr : in.paired1;
    s.all_cols = in.no_sandwich;
    uint32_t* flag = (uint32_t*)s.colflag;
    uint32_t* cols = (uint32_t*)s.cols;
    int64_t ncols = 0;
    if (m2 > 0) {
        hipLaunchKernelGGL(k_colflags, dim3(nblocks(m2)), dim3(DB), 0, st, p2, m2, flag);
        uint32_t* pos = cols;  // scan output; the compacted list goes through flag's buffer
        exclusive_scan_u32(flag, pos, m2, (uint32_t*)s.scanpart, st);
        uint32_t last_pos = 0, last_flag = 0;
        if (hipMemcpyAsync(&last_pos, pos + m2 - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&last_flag, flag + m2 - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = "D1: count read-back failed";
            return -5;
        }
        ncols = (int64_t)last_pos + last_flag;
        hipLaunchKernelGGL(k_compact, dim3(nblocks(m2)), dim3(DB), 0, st, in.c2, p2, pos, m2, flag);
        if (ncols > 0 && hipMemcpyAsync(cols, flag, 4 * ncols, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            err = "D1: copy failed";
            return -5;
        }
    }
    s.ncols = ncols;
    if (grow(s.bndptr, s.bndptr_cap, 8 * (ncols + 1), s.bytes, s.limit)) return oom("boundary pointers");
    // two deferral queues (this pass / next pass): u64 (column, offset) + u32 length
    if (grow(s.dq, s.dq_cap, 2 * (size_t)(ncols + 1) * 16, s.bytes, s.limit)) return oom("deferral queues");
    if (in.heap_keys > 0) {
        // debug: a heap of exactly the given size, so that small grids overflow
        // it and go through the restart below
        const size_t want = (size_t)8 * (size_t)std::max<int64_t>(in.heap_keys, 64);
        if (s.heap_cap != want) {
            if (s.heap) (void)hipFree(s.heap);
            s.bytes -= s.heap_cap;
            s.heap = nullptr;
            s.heap_cap = 0;
            if (grow(s.heap, s.heap_cap, want, s.bytes, s.limit)) return oom("boundary heap");
        }
    } else if (s.heap_cap < (size_t)8 * 32 * ncols) {
        if (grow(s.heap, s.heap_cap, std::max<size_t>((size_t)8 << 22, (size_t)8 * 32 * ncols), s.bytes, s.limit))
            return oom("boundary heap");
    }
    if (in.m1 > 0)
        hipLaunchKernelGGL(k_init_owner, dim3(nblocks(in.m1)), dim3(DB), 0, st, in.c1, p1, in.m1,
                           (uint32_t*)s.owner1);
    if (ncols == 0) return 0;
    for (int restart = 0; restart < 4; ++restart) {
        if (hipMemsetAsync(s.ctrs, 0, ctr_bytes, st) != hipSuccess || hipMemsetAsync(in.flags, 0, 4, st) != hipSuccess) {
            err = "D1: counter reset failed";
            return -5;
        }
        fill_u64((uint64_t*)s.bndptr, EMPTY64, ncols, st);
        if (restart > 0 && in.m1 > 0)
            hipLaunchKernelGGL(k_init_owner, dim3(nblocks(in.m1)), dim3(DB), 0, st, in.c1, p1, in.m1,
                               (uint32_t*)s.owner1);
        uint64_t* q[2] = {(uint64_t*)s.dq, (uint64_t*)s.dq + (ncols + 1)};
        uint32_t* qlen = (uint32_t*)((uint64_t*)s.dq + 2 * (ncols + 1));
        uint32_t* qcol = qlen + 2 * (ncols + 1);
        uint32_t* qc[2] = {qcol, qcol + (ncols + 1)};
        uint32_t* ql[2] = {qlen, qlen + (ncols + 1)};
        int64_t nwork = ncols;
        int cur = 0;
        bool overflow = false;
        unsigned long long hc[N_CTRS] = {0};
        // pass plan: thread-per-column with heaps of k keys in LDS (lane
        // passes), then one workgroup per column with boundaries
        // of up to k entries (lengths stay below 2^24: the cached length field).
        // t = lanes or workgroups: as many lanes as the LDS heaps leave resident
        // (160 KB per CU: 4 workgroups of 256 lanes x 20 keys, or 6 of 64 lanes x
        // 48 keys).
        PassPlan plan[MAX_PASSES] = {
            {LDS_K, 256 * 4 * 256, 256, true},
            {LDS_K2, 256 * 6 * 64, 64, true},
            {(int64_t)1 << 15, 1024, WB, false},
            {(int64_t)1 << 20, 512, WB, false},
            {((int64_t)1 << 24) - 1024, 64, WB, false},
            {0, 0, 0, false},
        };
        uint32_t long_add = LONG_ADD, part_span = PART_SPAN;
        uint64_t coop_min = COOP_MIN;
        int coop_always = 0;
        uint32_t pcap = PCAP;
        if (in.small_passes) {  // debug option: tiny capacities, every pass used
            plan[0].k = 3;
            plan[1].k = 4;
            plan[2].k = 24;
            long_add = 2;
            part_span = 40;
            coop_min = 4;
            coop_always = 1;
            pcap = 8;
        }
        // workgroup passes run at least two workgroups per compute unit: the
        // ones beyond the column slots only help with long merges
        int ncu = 256;
        {
            int dev = 0;
            if (hipGetDevice(&dev) == hipSuccess) {
                int v = 0;
                if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                    ncu = v;
            }
        }
        for (int pass = 0; pass < MAX_PASSES && nwork > 0; ++pass) {
            const int64_t K = plan[pass].k;
            if (K == 0) break;
            const int64_t T = std::max<int64_t>(1, std::min<int64_t>(nwork, plan[pass].t));
            const auto t_pass = std::chrono::steady_clock::now();
            const bool lane_pass = plan[pass].lane;
            const size_t need = lane_pass ? 8 : (size_t)8 * T * (2 * K + PCAP + K / part_span + 2);
            if (grow(s.scratch, s.scratch_cap, need, s.bytes, s.limit)) return oom("working boundaries");
            D1K P;
            P.g = in.g;
            P.G = in.G;
            P.rank = in.rank;
            P.order = in.order;
            P.cols = cols;
            P.ncols = ncols;
            P.work = pass == 0 ? nullptr : q[cur];
            P.work_len = pass == 0 ? nullptr : ql[cur];
            P.work_col = pass == 0 ? nullptr : qc[cur];
            P.nwork = nwork;
            P.defer = q[cur ^ 1];
            P.defer_len = ql[cur ^ 1];
            P.defer_col = qc[cur ^ 1];
            P.bpr = in.bpr;
            P.owner1 = (uint32_t*)s.owner1;
            P.bndptr = (uint64_t*)s.bndptr;
            P.heap = (uint64_t*)s.heap;
            P.heap_cap = s.heap_cap / 8;
            P.seg_cap = P.heap_cap / NSEG;
            P.scratch = (uint64_t*)s.scratch;
            P.K = K;
            P.nthreads = T;
            P.long_add = long_add;
            P.nslots = T;
            P.part_span = part_span;
            P.coop_min = coop_min;
            P.coop_always = coop_always;
            P.pcap = pcap;
            P.no_cache = in.no_cache ? 1 : 0;
            P.ctrs = (unsigned long long*)s.ctrs;
            P.flags = in.flags;
            // fresh work cursor, deferral count and work counters for this pass
            if (hipMemsetAsync((unsigned long long*)s.ctrs + C_NEXT, 0, 8 * (N_CTRS - C_NEXT), st) != hipSuccess) {
                err = "D1: counter reset failed";
                return -5;
            }
            if (lane_pass)
                hipLaunchKernelGGL(in.no_cache ? k_d1<true> : k_d1<false>,
                                   dim3((unsigned)((T + plan[pass].db - 1) / plan[pass].db)), dim3(plan[pass].db),
                                   (size_t)8 * plan[pass].db * K, st, P);
            else
                hipLaunchKernelGGL(k_d1_wide, dim3((unsigned)std::max<int64_t>(T, 2 * ncu)), dim3(WB), 0, st, P);
            uint32_t f = 0;
            if (hipMemcpyAsync(&f, in.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(hc, s.ctrs, sizeof(hc), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                err = "D1: kernel failed";
                return -5;
            }
            if (f & FLAG_GUARD) {
                unsigned long long why = 0;
                if (hipMemcpyAsync(&why, (unsigned long long*)s.ctrs + GUARD_REASON, 8, hipMemcpyDeviceToHost, st) !=
                        hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    why = 0;
                err = std::string("D1: consistency check failed (") + kGuardName[why < G_COUNT ? why : 0] +
                      ", pass " + std::to_string(pass) + ")";
                return -7;
            }
            if (in.log_passes) {
                std::fprintf(stderr, "[dms] D1 pass %d: %lld columns, heap %lld entries/thread, %.1f ms\n", pass,
                             (long long)nwork, (long long)K,
                             std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_pass)
                                 .count());
                if (!lane_pass) {
                    std::fprintf(stderr,
                                 "[dms]   rounds %llu (at an edge %llu, merge list full %llu, entries %llu), adds %llu "
                                 "(full merges %llu), keys moved %llu, deferred %llu\n",
                                 hc[C_ROUNDS], hc[C_RSTOP], hc[C_RCAP], hc[C_RTAKEN], hc[C_ADDS], hc[C_LONG],
                                 hc[C_MOVED], hc[C_DEFER]);
                    std::fprintf(stderr,
                                 "[dms]   longest column %.3f ms, max rounds %llu, max adds %llu, max length %llu, "
                                 "columns over 1 ms %llu; their us per phase:",
                                 hc[C_TMAX] / 1e5, hc[C_RMAX], hc[C_AMAX], hc[C_NMAX], hc[C_SLOW]);
                    for (int i = 0; i < N_PHASE; ++i) std::fprintf(stderr, " %llu", hc[C_PHASE + i] / 100);
                    std::fprintf(stderr, "\n");
                }
            }
            s.pass_work[pass] = (uint64_t)nwork;
            s.pass_us[pass] = (uint64_t)std::chrono::duration_cast<std::chrono::microseconds>(
                                  std::chrono::steady_clock::now() - t_pass)
                                  .count();
            s.stats[0] += hc[C_STEPS];
            s.stats[1] += hc[C_EVICT];
            s.stats[2] += hc[C_ADDS];
            s.stats[3] += hc[C_DEFER];
            s.wide[0] += hc[C_ROUNDS];
            s.wide[1] += hc[C_EXPANDED];
            s.wide[2] += hc[C_MOVED];
            s.wide[3] += hc[C_LONG];
            s.wide_t[0] = std::max<uint64_t>(s.wide_t[0], hc[C_TMAX] / 100);
            s.wide_t[1] += hc[C_TSUM] / 100;
            s.wide_t[2] = std::max<uint64_t>(s.wide_t[2], hc[C_RMAX]);
            s.wide_t[3] = std::max<uint64_t>(s.wide_t[3], hc[C_AMAX]);
            s.wide_t[4] = std::max<uint64_t>(s.wide_t[4], hc[C_NMAX]);
            s.wide_t[5] += hc[C_SLOW];
            for (int i = 0; i < N_PHASE; ++i) s.wide_ph[i] += hc[C_PHASE + i] / 100;
            s.wide_ph[10] += hc[C_PHASE + N_PHASE];
            s.wide_ph[11] += hc[C_PHASE + N_PHASE + 1];
            if (f & (FLAG_HEAP | FLAG_WORK)) {
                overflow = true;
                break;
            }
            nwork = (int64_t)hc[C_DEFER];
            cur ^= 1;
        }
        {
            uint64_t used = 0, segs[SEG_STRIDE * NSEG];
            if (hipMemcpyAsync(segs, (unsigned long long*)s.ctrs + SEG_BASE, sizeof(segs), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                err = "D1: heap counter read-back failed";
                return -5;
            }
            for (int q = 0; q < NSEG; ++q) used += segs[SEG_STRIDE * q];
            hc[C_HEAP] = used;
            uint64_t coop[5];
            if (hipMemcpyAsync(coop, (unsigned long long*)s.ctrs + OPEN_JOBS, sizeof(coop), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                err = "D1: counter read-back failed";
                return -5;
            }
            s.coop[0] = coop[2];
            s.coop[1] = coop[1];
            s.nc_fallbacks = coop[4];
        }
        s.stats[4] = hc[C_HEAP];
        s.stats[5] = restart;
        if (!overflow) {
            if (nwork > 0) {
                err = "D1: columns left after the last pass";
                return -7;
            }
            return 0;
        }
        // publication heap exhausted: grow it and redo D1 from the start
        const size_t want = std::max<size_t>(2 * s.heap_cap, (size_t)16 * hc[C_HEAP]);  // segments fill unevenly
        if (grow(s.heap, s.heap_cap, want, s.bytes, s.limit)) return oom("boundary heap");
    }
    err = "D1: boundary storage kept overflowing";
    return -3;
}

void d1_emit(D1State& s, int64_t m1, const uint8_t* paired1, const uint32_t* c1, uint64_t* key, uint32_t* death,
             uint32_t* cnt, hipStream_t st) {
    if (s.ncols > 0)
        hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)((s.ncols + DB * EMIT_ITEMS - 1) / (DB * EMIT_ITEMS))),
                           dim3(DB), 0, st, s.g, s.order, s.bpr,
                           (const uint32_t*)s.cols, s.ncols, (const uint64_t*)s.bndptr, (const uint64_t*)s.heap,
                           (const uint32_t*)s.owner1, key, death, cnt);
    if (m1 > 0)
        hipLaunchKernelGGL(k_emit_ess1, dim3(nblocks(m1)), dim3(DB), 0, st, c1, paired1, m1,
                           (const uint32_t*)s.owner1, key, death, cnt);
}

void d1_emit_essential2(D1State& s, int64_t m2, const uint8_t* paired2_desc, const uint32_t* c2, uint64_t* key,
                        uint32_t* death, uint32_t* cnt, hipStream_t st) {
    (void)c2;
    // without the sandwich the columns are all m2 2-saddles in C2 order
    const uint8_t* p2 = (s.all_cols && s.ncols == m2) ? paired2_desc : nullptr;
    if (s.ncols > 0)
        hipLaunchKernelGGL(k_emit_ess2, dim3(nblocks(s.ncols)), dim3(DB), 0, st, s.g, s.order, s.bpr,
                           (const uint32_t*)s.cols, s.ncols, (const uint64_t*)s.bndptr, (const uint64_t*)s.heap,
                           (const uint32_t*)s.owner1, p2, key, death, cnt);
}

int d1_generators(D1State& s, int64_t* offsets, int64_t cap_off, int64_t* edges, int64_t cap_edges,
                  int64_t* n_pairs, int64_t* n_edges, uint32_t* flags, hipStream_t st, std::string& err) {
    enum { G_EDGE, G_COL, G_EDGE2, G_COL2, G_LEN, G_OFF, G_KEY0, G_KEY1, G_VAL0, G_VAL1, G_HIST, G_PART };
    static_assert(G_PART < (int)(sizeof(s.gbuf) / sizeof(s.gbuf[0])), "generator buffers");
    auto buf = [&](int k, size_t bytes) -> void* {
        if (grow(s.gbuf[k], s.gcap[k], std::max<size_t>(bytes, 64), s.bytes, s.limit)) return nullptr;
        return s.gbuf[k];
    };
    auto hip_fail = [&](const char* what) {
        err = std::string("generators: ") + what;
        return -5;  // DMS_E_HIP
    };
    auto oom = [&]() {
        err = "generators: cannot allocate working buffers";
        return -3;  // DMS_E_NOMEM
    };
    *n_pairs = 0;
    *n_edges = 0;
    if (s.gen_n < 0) {  // build the cycles of the last D1 run once; later calls only copy them out
        const int64_t nc = s.ncols;
        if (s.stats[4] >= (1ull << 32)) {
            err = "generators: more than 2^32 published boundary entries";
            return -7;  // DMS_E_INTERNAL
        }
        // 1. finite pairs: (birth edge, column)
        uint32_t* ecol[4];
        for (int k = 0; k < 4; ++k)
            if (!(ecol[k] = (uint32_t*)buf(G_EDGE + k, 4 * (size_t)(nc + 1)))) return oom();
        uint32_t* len = (uint32_t*)buf(G_LEN, 4 * (size_t)(nc + 1));
        uint32_t* off = (uint32_t*)buf(G_OFF, 4 * (size_t)(nc + 1));
        if (!len || !off) return oom();
        if (hipMemsetAsync(len, 0, 4, st) != hipSuccess) return hip_fail("counter reset");
        if (nc > 0)
            hipLaunchKernelGGL(k_gen_pairs, dim3((unsigned)((nc + DB * EMIT_ITEMS - 1) / (DB * EMIT_ITEMS))),
                               dim3(DB), 0, st, s.g, s.order, s.bpr, nc, (const uint64_t*)s.bndptr,
                               (const uint64_t*)s.heap, (const uint32_t*)s.owner1, ecol[0], ecol[1], len);
        uint32_t n32 = 0;
        if (hipMemcpyAsync(&n32, len, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return hip_fail("pair count");
        const int64_t n = n32;
        int64_t total = 0, ne = 0;
        int r2 = 0;
        if (n > 0) {
            // 2. pairs in increasing birth-edge order (the order of the D1 output)
            const int ebits = 64 - __builtin_clzll((unsigned long long)(7 * s.g.V));
            const int pbits = 64 - __builtin_clzll((unsigned long long)n);
            uint32_t *hist = nullptr, *part = nullptr;
            auto scratch_for = [&](int64_t m) {
                const int64_t hn = 256 * sort_tiles(m);
                hist = (uint32_t*)buf(G_HIST, 4 * (size_t)hn);
                part = (uint32_t*)buf(G_PART, 4 * (size_t)std::max(scan_part_size(hn), scan_part_size(m)));
                return hist && part;
            };
            if (!scratch_for(n)) return oom();
            const int r1 = radix_sort_pairs<uint32_t>(ecol[0], ecol[1], ecol[2], ecol[3], n, 0, ebits, false, hist,
                                                      part, st);
            const uint32_t* col = r1 ? ecol[3] : ecol[1];
            // 3. published lengths and their offsets
            hipLaunchKernelGGL(k_gen_len, dim3(nblocks(n)), dim3(DB), 0, st, col, n, (const uint64_t*)s.bndptr, len);
            exclusive_scan_u32(len, off, n, part, st);
            uint32_t tail[2] = {0, 0};
            if (hipMemcpyAsync(&tail[0], off + n - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&tail[1], len + n - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return hip_fail("boundary sizes");
            total = (int64_t)tail[0] + tail[1];
            // 4. (pair, edge) keys of every published entry, sorted
            uint64_t* k0 = (uint64_t*)buf(G_KEY0, 8 * (size_t)total);
            uint64_t* k1 = (uint64_t*)buf(G_KEY1, 8 * (size_t)total);
            uint32_t* v0 = (uint32_t*)buf(G_VAL0, 4 * (size_t)total);
            uint32_t* v1 = (uint32_t*)buf(G_VAL1, 4 * (size_t)total);
            if (!k0 || !k1 || !v0 || !v1 || !scratch_for(std::max(n, total))) return oom();
            hipLaunchKernelGGL(k_gen_gather, dim3(nblocks(total)), dim3(DB), 0, st, s.g, s.order, s.bpr, col,
                               (const uint32_t*)off, n, total, (const uint64_t*)s.bndptr, (const uint64_t*)s.heap,
                               k0);
            r2 = radix_sort_pairs<uint64_t>(k0, v0, k1, v1, total, 0, 32 + pbits, true, hist, part, st);
            // 5. mod-2 cancellation: keep flags (v0), output positions (v1)
            hipLaunchKernelGGL(k_gen_keep, dim3(nblocks(total)), dim3(DB), 0, st, r2 ? k1 : k0, total, v0);
            exclusive_scan_u32(v0, v1, total, part, st);
            if (hipMemcpyAsync(&tail[0], v1 + total - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&tail[1], v0 + total - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return hip_fail("cycle sizes");
            ne = (int64_t)tail[0] + tail[1];
        }
        s.gen_n = n;
        s.gen_ne = ne;
        s.gen_total = total;
        s.gen_sorted = r2;
    }
    const int64_t n = s.gen_n, ne = s.gen_ne, total = s.gen_total;
    *n_pairs = n;
    *n_edges = ne;
    if (cap_off < n + 1 || cap_edges < ne) return 1;
    if (n == 0) {
        fill_u64((uint64_t*)offsets, 0, 1, st);
        return 0;
    }
    // 6. edges and offsets (pair_of: the key buffer that does not hold the keys)
    const uint64_t* key = (const uint64_t*)s.gbuf[s.gen_sorted ? G_KEY1 : G_KEY0];
    uint32_t* pair_of = (uint32_t*)s.gbuf[s.gen_sorted ? G_KEY0 : G_KEY1];
    fill_u64((uint64_t*)offsets, ~0ull, n, st);
    hipLaunchKernelGGL(k_gen_write, dim3(nblocks(total)), dim3(DB), 0, st, key, (const uint32_t*)s.gbuf[G_VAL0],
                       (const uint32_t*)s.gbuf[G_VAL1], total, edges, pair_of);
    hipLaunchKernelGGL(k_gen_offsets, dim3(nblocks(std::max<int64_t>(ne, 1))), dim3(DB), 0, st,
                       (const uint32_t*)pair_of, ne, n, offsets);
    hipLaunchKernelGGL(k_gen_check, dim3(nblocks(n)), dim3(DB), 0, st, (const int64_t*)offsets, n, flags);
    if (hipGetLastError() != hipSuccess) return hip_fail("kernel launch");
    return 0;
}

void d1_free(D1State& s) {
    void* ps[] = {s.cols, s.colflag, s.scanpart, s.owner1, s.bndptr, s.heap, s.scratch, s.ctrs, s.dq};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (void* p : s.gbuf)
        if (p) (void)hipFree(p);
    s = D1State();
}

}  // namespace dms
