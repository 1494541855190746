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
// The working boundary is a max-heap in per-thread scratch (interleaved
// across threads), with mod-2 cancellation of equal keys when they meet at
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
constexpr int MAX_PASSES = 5;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + DB - 1) / DB); }

// counters in D1State::ctrs
enum { C_HEAP = 0, C_NEXT = 1, C_DEFER = 2, C_STEPS = 3, C_EVICT = 4, C_ADDS = 5, C_ROUNDS = 6, C_EXPANDED = 7,
       C_MOVED = 8 };
// The publication heap is split into NSEG segments with one bump counter each
// (counters 128 bytes apart, after the 16 counters above), so that millions of
// publications do not serialise on one atomic.
constexpr int NSEG = 64;
constexpr int SEG_STRIDE = 16;
constexpr int SEG_BASE = 16;

struct D1K {
    GridDev g;
    const uint8_t* G;
    const uint32_t* rank;
    const uint32_t* order;
    const uint32_t* cols;
    int64_t ncols;
    // work of this pass: columns 0..ncols-1 (first pass) or deferred records
    const uint64_t* work;  // (column << 40 | record offset), or null in the first pass
    const uint32_t* work_len;
    int64_t nwork;
    uint64_t* defer;  // deferred (column << 40 | offset) of this pass
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
    int lds;  // working heaps in LDS (K entries per thread) instead of global scratch
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
__device__ inline void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */ }
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
__device__ inline EdgeDec edecode(const GridDev& g, const uint32_t* order, int bpr, uint64_t key) {
    EdgeDec e;
    e.ra = (uint32_t)(key >> bpr);
    e.rb = (uint32_t)(key & ((1ull << bpr) - 1));
    e.va = order[e.ra];
    e.vb = order[e.rb];
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

// ---- per-thread max-heap with mod-2 cancellation -----------------------------
struct Heap {
    uint64_t* base;  // element i at base[i * stride]
    int64_t stride;
    int64_t n;
    int64_t K;
    __device__ uint64_t& at(int64_t i) { return base[i * stride]; }
    __device__ void push(uint64_t x) {
        int64_t i = n++;
        while (i > 0) {
            const int64_t p = (i - 1) >> 1;
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
        int64_t i = 0;
        for (;;) {
            const int64_t l = 2 * i + 1;
            if (l >= n) break;
            int64_t c = l;
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
        const int64_t n0 = n;
        int64_t out = 0;
        for (;;) {
            const uint64_t t = extract_max();
            if (t == NONE) break;
            at(n0 - 1 - out) = t;
            ++out;
        }
        for (int64_t i = 0; i < out / 2; ++i) {
            const uint64_t a = at(n0 - out + i);
            at(n0 - out + i) = at(n0 - 1 - i);
            at(n0 - 1 - i) = a;
        }
        for (int64_t i = 0; i < out; ++i) at(i) = at(n0 - out + i);
        n = out;
    }
    __device__ bool room(int64_t extra) {
        if (n + extra <= K) return true;
        compact();
        return n + extra <= K;
    }
};

// Reserve len entries of the publication heap in segment seg; NONE when full.
__device__ inline uint64_t heap_alloc(const D1K& P, uint32_t seg, uint64_t len) {
    const uint64_t off = atomicAdd(&P.ctrs[SEG_BASE + SEG_STRIDE * (seg % NSEG)], (unsigned long long)len);
    if (off + len > P.seg_cap) return NONE;
    return (uint64_t)(seg % NSEG) * P.seg_cap + off;
}

// Copy {top (optional)} + heap (compacted) to the publication heap; returns
// the packed (offset << 24 | length) or NONE when the heap is full.
__device__ inline uint64_t publish(const D1K& P, Heap& H, bool with_top, uint64_t top) {
    H.compact();
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
    P.defer[d] = ((uint64_t)c << 40) | off;
    P.defer_len[d] = (uint32_t)len;
}

__global__ __launch_bounds__(DB) void k_d1(D1K P) {
    extern __shared__ uint64_t lds_heaps[];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= P.nthreads) return;  // scratch exists for nthreads lanes only
    Heap H;
    if (P.lds) {
        H.base = lds_heaps + (int64_t)threadIdx.x * P.K;
        H.stride = 1;
    } else {
        H.base = P.scratch + tid;
        H.stride = P.nthreads;
    }
    H.K = P.K;
    const int64_t V = P.g.V;
    unsigned long long steps = 0, evictions = 0, adds = 0;
    for (;;) {
        // columns are taken in increasing order: the frontier of columns in flight
        // stays narrow, which keeps evictions rare
        const int64_t next = (int64_t)atomicAdd(&P.ctrs[C_NEXT], 1ull);
        if (next >= P.nwork) break;
        uint32_t c;
        H.n = 0;
        if (!P.work) {
            c = (uint32_t)next;
            const uint32_t t = P.cols[c];
            const int64_t a = t / 12;
            const int ty = t % 12;
            const int64_t v1 = a + lin_of_mask(P.g, tri_step(ty, 0));
            const int64_t v2 = v1 + lin_of_mask(P.g, tri_step(ty, 1));
            const uint32_t r0 = P.rank[a], r1 = P.rank[v1], r2 = P.rank[v2];
            H.push(ekey_r(P.bpr, r0, r1));
            H.push(ekey_r(P.bpr, r1, r2));
            H.push(ekey_r(P.bpr, r0, r2));
        } else {
            // resume a deferred column from its saved, decreasing boundary
            const uint64_t w = P.work[next];
            c = (uint32_t)(w >> 40);
            const uint64_t off = w & ((1ull << 40) - 1);
            const int64_t len = P.work_len[next];
            if (len > H.K) {
                atomicOr(P.flags, FLAG_WORK);
                break;
            }
            for (int64_t i = 0; i < len; ++i) H.at(i) = ld_rlx64(P.heap + off + i);
            H.n = len;
        }
        bool have = false;
        uint64_t tau = 0;
        bool stop = false;  // leave the thread (error)
        for (int64_t guard = 0;; ++guard) {
            if (guard > ((int64_t)1 << 24)) {
                atomicOr(P.flags, FLAG_GUARD);
                stop = true;
                break;
            }
            ++steps;
            if (!have) {
                tau = H.extract_max();
                if (tau == NONE) break;  // zero column
                have = true;
            }
            const EdgeDec e = edecode(P.g, P.order, P.bpr, tau);
            if (e.mask == 0) {  // not an edge: corrupted key
                atomicOr(P.flags, FLAG_GUARD);
                stop = true;
                break;
            }
            const uint8_t code = P.G[(int64_t)e.mask * V + e.lo];
            bool defer = false;
            if (code != CODE_CRIT) {
                if (code >= 27) {  // the top of a cycle cannot be a vertex's partner
                    atomicOr(P.flags, FLAG_GUARD);
                    stop = true;
                    break;
                }
                const int64_t w = e.lo + lin27(P.g, code);
                if (H.room(2)) {
                    have = false;  // tau cancels against the boundary of its partner
                    const uint32_t rw = P.rank[w];
                    H.push(ekey_r(P.bpr, e.ra, rw));
                    H.push(ekey_r(P.bpr, e.rb, rw));
                    continue;
                }
                defer = true;
            } else {
                const uint32_t o = ld_rlx(&P.owner1[e.id]);
                if (o == OWN_D0) {
                    atomicOr(P.flags, FLAG_GUARD);
                    stop = true;
                    break;
                }
                if (o == EMPTY32 || o > c) {
                    // cache Boundary(c) = {tau} + heap, then claim tau
                    const uint64_t b = publish(P, H, true, tau);
                    if (b == NONE) {
                        atomicOr(P.flags, FLAG_HEAP);
                        stop = true;
                        break;
                    }
                    st_rlx64(&P.bndptr[c], b);
                    wait_stores();
                    if (!cas32(&P.owner1[e.id], o, c)) continue;  // owner changed: look again
                    if (o == EMPTY32) break;                       // column settled
                    // evicted o: carry on reducing it from its cached boundary
                    ++evictions;
                    const uint64_t bo = ld_rlx64(&P.bndptr[o]);
                    const uint64_t* B = P.heap + (bo >> 24);
                    const int64_t bl = (int64_t)(bo & 0xFFFFFF);
                    if (ld_rlx64(&B[0]) != tau) {
                        atomicOr(P.flags, FLAG_GUARD);
                        stop = true;
                        break;
                    }
                    c = o;
                    if (bl > H.K) {  // too large for this pass: defer it as it stands
                        defer_column(P, c, bo >> 24, bl);
                        break;
                    }
                    for (int64_t i = 1; i < bl; ++i) H.at(i - 1) = ld_rlx64(&B[i]);
                    H.n = bl - 1;
                    have = true;  // tau (= B[0]) is its top
                    continue;
                }
                // o < c: add the cached boundary of the earlier owner
                const uint64_t b = ld_rlx64(&P.bndptr[o]);
                if (b == EMPTY64) continue;
                const uint64_t* B = P.heap + (b >> 24);
                const int64_t bl = (int64_t)(b & 0xFFFFFF);
                if (ld_rlx64(&B[0]) != tau) continue;  // o moved on: look again
                if (H.room(bl - 1)) {
                    have = false;
                    ++adds;
                    for (int64_t i = 1; i < bl; ++i) H.push(ld_rlx64(&B[i]));
                    continue;
                }
                defer = true;
            }
            if (defer) {
                // save {tau} + heap and hand the column to the next pass
                const uint64_t b = publish(P, H, have, tau);
                if (b == NONE) {
                    atomicOr(P.flags, FLAG_HEAP);
                    stop = true;
                    break;
                }
                defer_column(P, c, b >> 24, b & 0xFFFFFF);
                break;
            }
        }
        if (stop) break;
    }
    atomicAdd(&P.ctrs[C_STEPS], steps);
    atomicAdd(&P.ctrs[C_EVICT], evictions);
    atomicAdd(&P.ctrs[C_ADDS], adds);
}


// ---- one workgroup per large column ------------------------------------------
// The boundary is a sorted array, ascending, in per-block global scratch, so
// that its top is at the end and a merge only rewrites the suffix from the
// smallest key it inserts or removes. A round looks at the top WB edges:
// every regular tail above the first critical (or non-tail) edge is expanded
// at once -- adding the boundary of a partner triangle leaves the column's
// Morse projection unchanged, so the expansions commute -- and the new edges
// are sorted, cancelled mod 2 and merged in. When the top is critical, the
// owner rule runs as in k_d1, with cached boundaries merged in chunks.
// Published boundaries keep the decreasing layout (top first).
constexpr int WB = 256;
constexpr int NW = 4 * WB;  // keys merged per step: 2 new keys + 1 kept entry per window slot
constexpr int IPW = NW / WB;
constexpr uint32_t BATCH_ADD_MAX = 32;  // longest cached boundary added out of order in a round
constexpr uint64_t PAD = ~0ull;

struct WideShared {
    uint64_t raw[NW];   // new keys of a round, sorted here
    uint64_t src[NW];   // keys to merge (ascending, unique)
    uint64_t surv[NW];  // keys of src not present in B
    uint32_t lb[NW];    // number of B-suffix elements smaller than src[j]
    uint32_t lbs[NW];   // lb of the survivors
    uint32_t canc[NW];  // B-suffix indices cancelled by src, ascending
    uint32_t flag[NW];
    uint32_t scan[WB];
    uint64_t scan64[WB];
    uint64_t zoff[WB];  // per window entry: cached boundary to add (offset of its second entry)
    uint32_t zlen[WB];  //   and the number of entries after its head; 0 = none
    int ints[8];
    uint64_t u64s[4];
};

__device__ inline uint32_t block_excl_scan(WideShared& L, uint32_t v, uint32_t& total) {
    const int t = threadIdx.x;
    L.scan[t] = v;
    __syncthreads();
    for (int d = 1; d < WB; d <<= 1) {
        const uint32_t a = t >= d ? L.scan[t - d] : 0;
        __syncthreads();
        L.scan[t] += a;
        __syncthreads();
    }
    total = L.scan[WB - 1];
    const uint32_t ex = L.scan[t] - v;
    __syncthreads();
    return ex;
}

// exclusive prefix maximum of v over the block (0 for thread 0)
__device__ inline uint64_t block_excl_max(WideShared& L, uint64_t v) {
    const int t = threadIdx.x;
    L.scan64[t] = v;
    __syncthreads();
    for (int d = 1; d < WB; d <<= 1) {
        const uint64_t a = t >= d ? L.scan64[t - d] : 0;
        __syncthreads();
        if (a > L.scan64[t]) L.scan64[t] = a;
        __syncthreads();
    }
    const uint64_t ex = t > 0 ? L.scan64[t - 1] : 0;
    __syncthreads();
    return ex;
}

// number of elements of the ascending array A[0..n) smaller than x
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

// B[0..n) ^= L.src[0..m) (both ascending, unique), in place, tmp holding the
// rewritten suffix; returns the new size.
__device__ uint32_t merge_xor(WideShared& L, uint64_t* B, uint32_t n, uint32_t m, uint64_t* tmp,
                              unsigned long long& moved) {
    const int t = threadIdx.x;
    if (m == 0) return n;
    const uint32_t p = count_less<uint64_t>(B, n, L.src[0]);
    uint64_t* Bp = B + p;
    const uint32_t len = n - p;
    moved += len;
    for (uint32_t j = t; j < (uint32_t)NW; j += WB) {
        uint32_t c = 0, f = 0;
        if (j < m) {
            c = count_less<uint64_t>(Bp, len, L.src[j]);
            f = (c < len && Bp[c] == L.src[j]) ? 1u : 0u;
        }
        L.lb[j] = c;
        L.flag[j] = f;
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
    uint32_t nc, ns;
    const uint32_t ec = block_excl_scan(L, fc, nc);
    const uint32_t es = block_excl_scan(L, sc, ns);
    {
        uint32_t a = ec, b = es;
        for (int q = 0; q < IPW; ++q) {
            const uint32_t j = IPW * t + q;
            if (j >= m) break;
            if (L.flag[j]) L.canc[a++] = L.lb[j];
            else {
                L.surv[b] = L.src[j];
                L.lbs[b] = L.lb[j];
                ++b;
            }
        }
    }
    __syncthreads();
    for (uint32_t i = t; i < len; i += WB) {
        const uint64_t x = Bp[i];
        const uint32_t cl = count_less<uint32_t>(L.canc, nc, i);
        if (cl < nc && L.canc[cl] == i) continue;  // cancelled
        const uint32_t sl = count_less<uint64_t>(L.surv, ns, x);
        tmp[i - cl + sl] = x;
    }
    for (uint32_t k = t; k < ns; k += WB) {
        const uint32_t cl = count_less<uint32_t>(L.canc, nc, L.lbs[k]);
        tmp[k + L.lbs[k] - cl] = L.surv[k];
    }
    __syncthreads();
    const uint32_t r = len - nc + ns;
    for (uint32_t i = t; i < r; i += WB) Bp[i] = tmp[i];
    __syncthreads();
    return p + r;
}

// sort L.raw[0..np) ascending (np a power of two, PAD last), cancel equal keys
// mod 2 into L.src; returns the number of keys kept
__device__ uint32_t sort_cancel(WideShared& L, int np) {
    const int t = threadIdx.x;
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int pp = t; pp < np / 2; pp += WB) {
                const int i = 2 * pp - (pp & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = L.raw[i], b = L.raw[j];
                if ((a > b) == asc) {
                    L.raw[i] = b;
                    L.raw[j] = a;
                }
            }
            __syncthreads();
        }
    }
    uint32_t keep[IPW];
    uint32_t kc = 0;
    for (int q = 0; q < IPW; ++q) {
        const int j = IPW * t + q;
        const uint64_t x = j < np ? L.raw[j] : PAD;
        uint32_t k = 0;
        if (x != PAD && (j == 0 || L.raw[j - 1] != x)) {
            int r = 1;
            while (j + r < np && L.raw[j + r] == x) ++r;
            k = r & 1;
        }
        keep[q] = k;
        kc += k;
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan(L, kc, total);
    uint32_t a = ex;
    for (int q = 0; q < IPW; ++q)
        if (keep[q]) L.src[a++] = L.raw[IPW * t + q];
    __syncthreads();
    return total;
}

// Save the ascending boundary B[0..n) to the publication heap in the
// decreasing layout; returns the offset or PAD when the heap is full.
__device__ uint64_t save_desc(const D1K& P, WideShared& L, const uint64_t* B, uint32_t n) {
    const int t = threadIdx.x;
    if (t == 0) L.u64s[1] = heap_alloc(P, blockIdx.x, n);
    __syncthreads();
    const uint64_t off = L.u64s[1];
    __syncthreads();
    if (off == NONE) return PAD;
    for (uint32_t i = t; i < n; i += WB) st_rlx64(P.heap + off + i, B[n - 1 - i]);
    wait_stores();
    __syncthreads();
    return off;
}

__global__ __launch_bounds__(WB) void k_d1_wide(D1K P) {
    __shared__ WideShared L;
    const int t = threadIdx.x;
    uint64_t* B = P.scratch + (int64_t)blockIdx.x * 2 * P.K;
    uint64_t* tmp = B + P.K;
    const int64_t V = P.g.V;
    unsigned long long steps = 0, evictions = 0, adds = 0, rounds = 0, expanded = 0, moved = 0;
    for (;;) {
        if (t == 0) L.u64s[0] = atomicAdd(&P.ctrs[C_NEXT], 1ull);
        __syncthreads();
        const uint64_t next = L.u64s[0];
        __syncthreads();
        if ((int64_t)next >= P.nwork) break;
        const uint64_t w = P.work[next];
        uint32_t c = (uint32_t)(w >> 40);
        uint32_t n;
        {
            const uint64_t off = w & ((1ull << 40) - 1);
            n = P.work_len[next];
            if ((int64_t)n > P.K) {
                if (t == 0) atomicOr(P.flags, FLAG_WORK);
                break;
            }
            for (uint32_t i = t; i < n; i += WB) B[i] = ld_rlx64(P.heap + off + (n - 1 - i));
        }
        __syncthreads();
        bool stop = false;
        for (int64_t guard = 0;; ++guard) {
            if (guard > ((int64_t)1 << 24)) {
                if (t == 0) atomicOr(P.flags, FLAG_GUARD);
                stop = true;
                break;
            }
            ++steps;
            if (n == 0) break;  // zero column
            // scan the top window. Above the first stopping edge, every regular tail
            // (add its partner's boundary) and every critical edge owned by an earlier
            // column with a short cached boundary (add it) is processed this round.
            // Edges that are never a pivot (vertex partners, D0-paired edges) are
            // kept without stopping. A possible pivot (free or later-owned critical
            // edge) stops the round, and so does an earlier-owned one with a long
            // cached boundary, which is added in order when it reaches the top: adding
            // long boundaries out of order inflates the boundaries cached later. The
            // top must be processable, otherwise the owner rule runs.
            const uint32_t k = n < (uint32_t)WB ? n : (uint32_t)WB;
            for (int q = 0; q < IPW; ++q) L.raw[IPW * t + q] = PAD;
            L.zlen[t] = 0;
            L.flag[t] = 0;
            if (t == 0) L.ints[0] = WB;
            __syncthreads();
            uint64_t wkey = 0;
            uint64_t nk0 = PAD, nk1 = PAD;
            int cls = 0;  // 0 none/stop, 1 processable, 2 kept (never a pivot)
            if ((uint32_t)t < k) {
                wkey = B[n - 1 - t];
                const EdgeDec e = edecode(P.g, P.order, P.bpr, wkey);
                const uint8_t code = e.mask ? P.G[(int64_t)e.mask * V + e.lo] : (uint8_t)0xFE;
                if (code < 27) {
                    const uint32_t rw = P.rank[e.lo + lin27(P.g, code)];
                    nk0 = ekey_r(P.bpr, e.ra, rw);
                    nk1 = ekey_r(P.bpr, e.rb, rw);
                    cls = 1;
                } else if (code == CODE_CRIT) {
                    const uint32_t o = ld_rlx(&P.owner1[e.id]);
                    if (o == OWN_D0) {
                        cls = 2;
                    } else if (o != EMPTY32 && o < c && t > 0) {
                        // (a critical top goes through the owner rule below)
                        const uint64_t bo = ld_rlx64(&P.bndptr[o]);
                        const uint32_t zl = (uint32_t)(bo & 0xFFFFFF) - 1;
                        if (bo != EMPTY64 && zl <= BATCH_ADD_MAX && ld_rlx64(P.heap + (bo >> 24)) == wkey) {
                            L.zoff[t] = (bo >> 24) + 1;
                            L.zlen[t] = zl;
                            cls = 1;
                        }
                    }
                } else if (code >= 0x80 && code < 0xFE) {
                    cls = 2;  // vertex partner
                }
            }
            if ((uint32_t)t < k && cls == 0) atomicMin(&L.ints[0], t);
            __syncthreads();
            uint32_t stop_at = (uint32_t)L.ints[0];
            // room in the merge list: every window entry reserves one slot (a kept
            // entry needs exactly that); a processed tail needs one more, a batched
            // cached boundary its length minus one more. Stop where it would overflow.
            {
                uint32_t extra = 0;
                if ((uint32_t)t < k && cls == 1) extra = (L.zlen[t] ? L.zlen[t] : 2) - 1;
                uint32_t tot;
                const uint32_t ex = block_excl_scan(L, extra, tot);
                if (t == 0) L.ints[1] = WB;
                __syncthreads();
                if ((uint32_t)t < k && k + ex + extra > (uint32_t)NW) atomicMin(&L.ints[1], t);
                __syncthreads();
                if ((uint32_t)L.ints[1] < stop_at) stop_at = (uint32_t)L.ints[1];
                __syncthreads();
            }
            uint32_t slot = 0;
            {
                uint32_t need = 0;
                const bool go = (uint32_t)t < k && cls == 1 && (uint32_t)t < stop_at;
                if ((uint32_t)t < k) need = go ? (L.zlen[t] ? L.zlen[t] : 2) : 1;
                uint32_t tot;
                slot = block_excl_scan(L, need, tot);
                L.ints[7] = (int)tot;  // same value from every thread
                if ((uint32_t)t < k) {
                    if (go) {
                        if (L.zlen[t]) {
                            const uint64_t zo = L.zoff[t];
                            for (uint32_t j = 0; j < L.zlen[t]; ++j) L.raw[slot + j] = ld_rlx64(P.heap + zo + j);
                        } else {
                            L.raw[slot] = nk0;
                            L.raw[slot + 1] = nk1;
                        }
                    } else {
                        L.raw[slot] = wkey;  // kept: re-inserted below
                    }
                }
                L.flag[t] = go ? 1u : 0u;
            }
            __syncthreads();
            const bool top_go = L.flag[0] != 0;
            __syncthreads();
            if (top_go) {
                const uint32_t total = (uint32_t)L.ints[7];
                uint32_t nproc;
                block_excl_scan(L, L.flag[t], nproc);
                int np = 2;
                while (np < (int)total) np <<= 1;
                const uint32_t m = sort_cancel(L, np);
                ++rounds;
                expanded += nproc;
                if ((int64_t)(n - k) + m > P.K) {
                    // no room: save the column unchanged for the next pass
                    const uint64_t off = save_desc(P, L, B, n);
                    if (off == PAD) {
                        if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                        stop = true;
                        break;
                    }
                    if (t == 0) defer_column(P, c, off, n);
                    break;
                }
                // the window leaves; new keys, batched boundaries and kept entries come in
                n = merge_xor(L, B, n - k, m, tmp, moved);
                continue;
            }
            // the top edge is not a regular tail
            if (t == 0) {
                const EdgeDec te = edecode(P.g, P.order, P.bpr, B[n - 1]);
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
                L.ints[2] = action;
                L.ints[3] = (int)o;
                L.ints[4] = (int)te.id;
            }
            __syncthreads();
            const int action = L.ints[2];
            const uint32_t o = (uint32_t)L.ints[3];
            const uint32_t eid = (uint32_t)L.ints[4];
            const uint64_t tau = B[n - 1];
            __syncthreads();
            if (action < 0) {
                if (t == 0) atomicOr(P.flags, FLAG_GUARD);
                stop = true;
                break;
            }
            if (action == 1) {
                const uint64_t off = save_desc(P, L, B, n);
                if (off == PAD) {
                    if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                    stop = true;
                    break;
                }
                if (t == 0) {
                    st_rlx64(&P.bndptr[c], (off << 24) | n);
                    wait_stores();
                    L.ints[5] = cas32(&P.owner1[eid], o, c) ? 1 : 0;
                    if (L.ints[5] && o != EMPTY32) L.u64s[2] = ld_rlx64(&P.bndptr[o]);
                }
                __syncthreads();
                const int won = L.ints[5];
                const uint64_t bo = L.u64s[2];
                __syncthreads();
                if (!won) continue;
                if (o == EMPTY32) break;  // settled
                ++evictions;
                c = o;
                const uint32_t bl = (uint32_t)(bo & 0xFFFFFF);
                const uint64_t boff = bo >> 24;
                if ((int64_t)bl > P.K) {
                    if (t == 0) defer_column(P, c, boff, bl);
                    break;
                }
                for (uint32_t i = t; i < bl; i += WB) B[i] = ld_rlx64(P.heap + boff + (bl - 1 - i));
                __syncthreads();
                n = bl;
                continue;
            }
            // action 2: B += Boundary(o), merged in chunks (largest keys first)
            if (t == 0) {
                const uint64_t b = ld_rlx64(&P.bndptr[o]);
                L.u64s[3] = b;
                L.ints[6] = (b != EMPTY64 && ld_rlx64(P.heap + (b >> 24)) == tau) ? 1 : 0;
            }
            __syncthreads();
            const uint64_t b = L.u64s[3];
            const int ok = L.ints[6];
            __syncthreads();
            if (!ok) continue;  // o moved on: look again
            const uint64_t aoff = b >> 24;
            const uint32_t alen = (uint32_t)(b & 0xFFFFFF);
            if ((int64_t)n + alen > P.K) {
                // the sum might not fit: hand the column, unchanged, to the next pass
                const uint64_t off = save_desc(P, L, B, n);
                if (off == PAD) {
                    if (t == 0) atomicOr(P.flags, FLAG_HEAP);
                    stop = true;
                    break;
                }
                if (t == 0) defer_column(P, c, off, n);
                break;
            }
            ++adds;
            for (uint32_t base = 0; base < alen; base += NW) {
                const uint32_t m = min((uint32_t)NW, alen - base);
                for (uint32_t j = t; j < m; j += WB) L.src[j] = ld_rlx64(P.heap + aoff + base + (m - 1 - j));
                __syncthreads();
                n = merge_xor(L, B, n, m, tmp, moved);
            }
        }
        __syncthreads();
        if (stop) break;
    }
    if (t == 0) {
        atomicAdd(&P.ctrs[C_STEPS], steps);
        atomicAdd(&P.ctrs[C_EVICT], evictions);
        atomicAdd(&P.ctrs[C_ADDS], adds);
        atomicAdd(&P.ctrs[C_ROUNDS], rounds);
        atomicAdd(&P.ctrs[C_EXPANDED], expanded);
        atomicAdd(&P.ctrs[C_MOVED], moved);
    }
}

__global__ void k_init_owner(const uint32_t* c1, const uint8_t* paired1, int64_t m1, uint32_t* owner1) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i < m1) owner1[c1[i]] = paired1[i] ? OWN_D0 : EMPTY32;
}

__global__ void k_colflags(const uint8_t* paired2_desc, int64_t m2, uint32_t* flag) {
    const int64_t k = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (k < m2) flag[k] = paired2_desc[m2 - 1 - k] ? 0u : 1u;
}

__global__ void k_compact(const uint32_t* c2, const uint8_t* paired2_desc, const uint32_t* pos, int64_t m2,
                          uint32_t* cols) {
    const int64_t k = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (k < m2 && !paired2_desc[m2 - 1 - k]) cols[pos[k]] = c2[k];
}

__global__ void k_emit_pairs(GridDev g, const uint32_t* order, int bpr, const uint32_t* cols, int64_t ncols,
                             const uint64_t* bndptr, const uint64_t* heap, const uint32_t* owner1, uint64_t* key,
                             uint32_t* death, uint32_t* cnt) {
    const int64_t c = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (c >= ncols) return;
    const uint64_t b = bndptr[c];
    if (b == EMPTY64) return;
    const EdgeDec e = edecode(g, order, bpr, heap[b >> 24]);
    if (owner1[e.id] != (uint32_t)c) return;
    const uint32_t at = atomicAdd(cnt, 1u);
    key[at] = e.id;
    death[at] = cols[c];
}

__global__ void k_emit_ess1(const uint32_t* c1, const uint8_t* paired1, int64_t m1, const uint32_t* owner1,
                            uint64_t* key, uint32_t* death, uint32_t* cnt) {
    const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (i >= m1 || paired1[i]) return;
    if (owner1[c1[i]] != EMPTY32) return;
    const uint32_t at = atomicAdd(cnt, 1u);
    key[at] = (1ull << 32) | c1[i];
    death[at] = EMPTY32;
}

__global__ void k_emit_ess2(GridDev g, const uint32_t* order, int bpr, const uint32_t* cols, int64_t ncols,
                            const uint64_t* bndptr, const uint64_t* heap, const uint32_t* owner1, uint64_t* key,
                            uint32_t* death, uint32_t* cnt) {
    const int64_t c = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (c >= ncols) return;
    const uint64_t b = bndptr[c];
    if (b != EMPTY64) {
        const EdgeDec e = edecode(g, order, bpr, heap[b >> 24]);
        if (owner1[e.id] == (uint32_t)c) return;
    }
    const uint32_t at = atomicAdd(cnt, 1u);
    key[at] = (1ull << 32) | cols[c];
    death[at] = EMPTY32;
}

int grow(void*& p, size_t& cap, size_t bytes, size_t& total) {
    if (cap >= bytes) return 0;
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
    (void)budget_left;
    const int64_t V = in.g.V;
    const int64_t m2 = in.m2;
    s.g = in.g;
    s.order = in.order;
    s.bpr = in.bpr;
    auto oom = [&](const char* what) {
        err = std::string("D1: cannot allocate ") + what;
        return -3;  // DMS_E_NOMEM
    };
    const size_t ctr_bytes = 8 * (SEG_BASE + SEG_STRIDE * NSEG);
    if (!s.ctrs && hipMalloc(&s.ctrs, ctr_bytes) != hipSuccess) return oom("counters");
    if (grow(s.colflag, s.colflag_cap, 4 * (m2 + 1), s.bytes)) return oom("column flags");
    if (grow(s.cols, s.cols_cap, 4 * (m2 + 1), s.bytes)) return oom("columns");
    if (grow(s.scanpart, s.scanpart_cap, 4 * scan_part_size(m2 + 1), s.bytes)) return oom("scan");
    if (grow(s.owner1, s.owner1_cap, 4 * 7 * V, s.bytes)) return oom("owners");
    for (int d = 0; d < 6; ++d) s.stats[d] = 0;
    for (int d = 0; d < 5; ++d) s.pass_work[d] = s.pass_us[d] = 0;
    for (int d = 0; d < 3; ++d) s.wide[d] = 0;
    // unpaired 2-saddles, ascending
    uint32_t* flag = (uint32_t*)s.colflag;
    uint32_t* cols = (uint32_t*)s.cols;
    int64_t ncols = 0;
    if (m2 > 0) {
        hipLaunchKernelGGL(k_colflags, dim3(nblocks(m2)), dim3(DB), 0, st, in.paired2_desc, m2, flag);
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
        hipLaunchKernelGGL(k_compact, dim3(nblocks(m2)), dim3(DB), 0, st, in.c2, in.paired2_desc, pos, m2, flag);
        if (ncols > 0 && hipMemcpyAsync(cols, flag, 4 * ncols, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            err = "D1: copy failed";
            return -5;
        }
    }
    s.ncols = ncols;
    if (grow(s.bndptr, s.bndptr_cap, 8 * (ncols + 1), s.bytes)) return oom("boundary pointers");
    // two deferral queues (this pass / next pass): u64 (column, offset) + u32 length
    if (grow(s.dq, s.dq_cap, 2 * (size_t)(ncols + 1) * 12, s.bytes)) return oom("deferral queues");
    if (s.heap_cap < (size_t)8 * 32 * ncols) {
        if (grow(s.heap, s.heap_cap, std::max<size_t>((size_t)8 << 22, (size_t)8 * 32 * ncols), s.bytes))
            return oom("boundary heap");
    }
    const int64_t lanes = (int64_t)1 << 18;  // first pass: 262144 threads x 256 entries
    const int64_t k0 = 256;
    if (in.m1 > 0)
        hipLaunchKernelGGL(k_init_owner, dim3(nblocks(in.m1)), dim3(DB), 0, st, in.c1, in.paired1, in.m1,
                           (uint32_t*)s.owner1);
    if (ncols == 0) return 0;
    for (int restart = 0; restart < 4; ++restart) {
        if (hipMemsetAsync(s.ctrs, 0, ctr_bytes, st) != hipSuccess) return -5;
        if (hipMemsetAsync(in.flags, 0, 4, st) != hipSuccess) return -5;
        fill_u64((uint64_t*)s.bndptr, EMPTY64, ncols, st);
        if (restart > 0 && in.m1 > 0)
            hipLaunchKernelGGL(k_init_owner, dim3(nblocks(in.m1)), dim3(DB), 0, st, in.c1, in.paired1, in.m1,
                               (uint32_t*)s.owner1);
        uint64_t* q[2] = {(uint64_t*)s.dq, (uint64_t*)s.dq + (ncols + 1)};
        uint32_t* qlen = (uint32_t*)((uint64_t*)s.dq + 2 * (ncols + 1));
        uint32_t* ql[2] = {qlen, qlen + (ncols + 1)};
        int64_t nwork = ncols;
        int cur = 0;
        bool overflow = false;
        unsigned long long hc[16] = {0};
        // pass plan: thread-per-column with small heaps, then one workgroup per
        // column with boundaries of up to plan_k entries
        int64_t plan_k[MAX_PASSES] = {k0, (int64_t)1 << 15, (int64_t)1 << 20, (int64_t)1 << 24, 0};
        int64_t plan_t[MAX_PASSES] = {lanes, 1024, 32, 2, 0};
        if (std::getenv("DMS_D1_TEST_PLAN")) {  // test hook: tiny capacities, every pass used
            plan_k[0] = 4;
            plan_k[1] = 24;
        }
        for (int pass = 0; pass < MAX_PASSES && nwork > 0; ++pass) {
            const int64_t K = plan_k[pass];
            if (K == 0) break;
            const int64_t T = std::max<int64_t>(1, std::min<int64_t>(nwork, plan_t[pass]));
            const auto t_pass = std::chrono::steady_clock::now();
            const size_t need = pass == 0 ? (size_t)8 * T * K : (size_t)8 * 2 * T * K;
            if (grow(s.scratch, s.scratch_cap, need, s.bytes)) return oom("working boundaries");
            D1K P;
            P.g = in.g;
            P.G = in.G;
            P.rank = in.rank;
            P.order = in.order;
            P.cols = cols;
            P.ncols = ncols;
            P.work = pass == 0 ? nullptr : q[cur];
            P.work_len = pass == 0 ? nullptr : ql[cur];
            P.nwork = nwork;
            P.defer = q[cur ^ 1];
            P.defer_len = ql[cur ^ 1];
            P.bpr = in.bpr;
            P.owner1 = (uint32_t*)s.owner1;
            P.bndptr = (uint64_t*)s.bndptr;
            P.heap = (uint64_t*)s.heap;
            P.heap_cap = s.heap_cap / 8;
            P.seg_cap = P.heap_cap / NSEG;
            P.scratch = (uint64_t*)s.scratch;
            P.K = K;
            P.nthreads = T;
            P.lds = 0;
            P.ctrs = (unsigned long long*)s.ctrs;
            P.flags = in.flags;
            // fresh work cursor, deferral count and work counters for this pass
            if (hipMemsetAsync((unsigned long long*)s.ctrs + C_NEXT, 0, 8 * 8, st) != hipSuccess) return -5;
            if (pass == 0)
                hipLaunchKernelGGL(k_d1, dim3(nblocks(T)), dim3(DB), 0, st, P);
            else
                hipLaunchKernelGGL(k_d1_wide, dim3((unsigned)T), dim3(WB), 0, st, P);
            uint32_t f = 0;
            if (hipMemcpyAsync(&f, in.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(hc, s.ctrs, 128, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                err = "D1: kernel failed";
                return -5;
            }
            if (f & FLAG_GUARD) {
                err = "D1: consistency check failed";
                return -7;
            }
            if (std::getenv("DMS_LOG"))
                std::fprintf(stderr, "[dms] D1 pass %d: %lld columns, heap %lld entries/thread, %.1f ms\n", pass,
                             (long long)nwork, (long long)K,
                             std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_pass)
                                 .count());
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
            if (f & (FLAG_HEAP | FLAG_WORK)) {
                overflow = true;
                break;
            }
            nwork = (int64_t)hc[C_DEFER];
            cur ^= 1;
        }
        {
            uint64_t used = 0, segs[SEG_STRIDE * NSEG];
            if (hipMemcpy(segs, (unsigned long long*)s.ctrs + SEG_BASE, sizeof(segs), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return -5;
            for (int q = 0; q < NSEG; ++q) used += segs[SEG_STRIDE * q];
            hc[C_HEAP] = used;
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
        if (grow(s.heap, s.heap_cap, want, s.bytes)) return oom("boundary heap");
    }
    err = "D1: boundary storage kept overflowing";
    return -3;
}

void d1_emit(D1State& s, int64_t m1, const uint8_t* paired1, const uint32_t* c1, uint64_t* key, uint32_t* death,
             uint32_t* cnt, hipStream_t st) {
    if (s.ncols > 0)
        hipLaunchKernelGGL(k_emit_pairs, dim3(nblocks(s.ncols)), dim3(DB), 0, st, s.g, s.order, s.bpr,
                           (const uint32_t*)s.cols, s.ncols, (const uint64_t*)s.bndptr, (const uint64_t*)s.heap,
                           (const uint32_t*)s.owner1, key, death, cnt);
    if (m1 > 0)
        hipLaunchKernelGGL(k_emit_ess1, dim3(nblocks(m1)), dim3(DB), 0, st, c1, paired1, m1,
                           (const uint32_t*)s.owner1, key, death, cnt);
}

void d1_emit_essential2(D1State& s, int64_t m2, const uint8_t* paired2_desc, const uint32_t* c2, uint64_t* key,
                        uint32_t* death, uint32_t* cnt, hipStream_t st) {
    (void)m2;
    (void)paired2_desc;
    (void)c2;
    if (s.ncols > 0)
        hipLaunchKernelGGL(k_emit_ess2, dim3(nblocks(s.ncols)), dim3(DB), 0, st, s.g, s.order, s.bpr,
                           (const uint32_t*)s.cols, s.ncols, (const uint64_t*)s.bndptr, (const uint64_t*)s.heap,
                           (const uint32_t*)s.owner1, key, death, cnt);
}

void d1_free(D1State& s) {
    void* ps[] = {s.cols, s.colflag, s.scanpart, s.owner1, s.bndptr, s.heap, s.scratch, s.ctrs, s.dq};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    s = D1State();
}

}  // namespace dms
