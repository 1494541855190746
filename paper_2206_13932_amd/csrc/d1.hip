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
// The boundary is a max-heap in a per-thread global scratch region, with
// mod-2 cancellation of equal keys when they meet at the top. Cached
// boundaries are immutable, bump-allocated arrays (sorted decreasing), so a
// reader that sees tau at their head has a consistent copy.
//
// The result equals the sequential algorithm: with the expansion-based
// gradient, the highest edge of a boundary whose top is critical is also
// the top of its projection onto the Morse complex (all smaller edges of
// that lower star were classified before the critical one was popped, so
// their v-paths only reach smaller critical edges); the loop is therefore a
// column reduction of the Morse boundary matrix, whose pivots do not depend
// on the order in which earlier columns are added.
#include "d1.h"
#include "dms_internal.h"

namespace dms {

namespace {

constexpr int DB = 256;
constexpr uint32_t OWN_D0 = 0xFFFFFFFEu;
constexpr uint64_t NONE = ~0ull;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + DB - 1) / DB); }

struct D1K {
    GridDev g;
    const uint8_t* G;
    const uint32_t* rank;
    const uint32_t* order;
    const uint32_t* cols;
    int64_t ncols;
    int bpr;
    uint32_t* owner1;
    uint64_t* bndptr;
    uint64_t* heap;
    uint64_t heap_cap;
    uint64_t* scratch;
    int64_t K;
    int64_t nthreads;
    unsigned long long* ctrs;
    uint32_t* flags;
};

__device__ inline uint32_t ld_acq(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_acq64(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_rel64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool cas32(uint32_t* p, uint32_t expect, uint32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t ekey(const D1K& P, int64_t a, int64_t b) {
    const uint32_t ra = P.rank[a], rb = P.rank[b];
    return ra > rb ? (((uint64_t)ra << P.bpr) | rb) : (((uint64_t)rb << P.bpr) | ra);
}

// edge key -> endpoints (va higher), anchor, step mask, id
struct EdgeDec {
    int64_t va, vb, lo;
    int mask;
    uint32_t id;
};
__device__ inline EdgeDec edecode(const GridDev& g, const uint32_t* order, int bpr, uint64_t key) {
    EdgeDec e;
    e.va = order[key >> bpr];
    e.vb = order[key & ((1ull << bpr) - 1)];
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
    uint64_t* h;
    int64_t n;
    int64_t K;
    __device__ void push(uint64_t x) {
        int64_t i = n++;
        while (i > 0) {
            const int64_t p = (i - 1) >> 1;
            const uint64_t hp = h[p];
            if (hp >= x) break;
            h[i] = hp;
            i = p;
        }
        h[i] = x;
    }
    __device__ uint64_t pop() {
        const uint64_t top = h[0];
        const uint64_t x = h[--n];
        int64_t i = 0;
        for (;;) {
            const int64_t l = 2 * i + 1;
            if (l >= n) break;
            int64_t c = l;
            uint64_t hc = h[l];
            if (l + 1 < n) {
                const uint64_t hr = h[l + 1];
                if (hr > hc) { c = l + 1; hc = hr; }
            }
            if (hc <= x) break;
            h[i] = hc;
            i = c;
        }
        if (n > 0) h[i] = x;
        return top;
    }
    // highest key present an odd number of times, removed; NONE if empty
    __device__ uint64_t extract_max() {
        while (n > 0) {
            const uint64_t t = pop();
            int cnt = 1;
            while (n > 0 && h[0] == t) {
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
            h[n0 - 1 - out] = t;
            ++out;
        }
        // outputs sit in [n0-out, n0), increasing from left; reverse, then shift
        for (int64_t i = 0; i < out / 2; ++i) {
            const uint64_t a = h[n0 - out + i];
            h[n0 - out + i] = h[n0 - 1 - i];
            h[n0 - 1 - i] = a;
        }
        for (int64_t i = 0; i < out; ++i) h[i] = h[n0 - out + i];
        n = out;
    }
    __device__ bool room(int64_t extra) {
        if (n + extra <= K) return true;
        compact();
        return n + extra <= K;
    }
};

__global__ __launch_bounds__(DB) void k_d1(D1K P) {
    const int64_t tid = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (tid >= P.nthreads) return;  // scratch exists for nthreads lanes only
    Heap H;
    H.h = P.scratch + tid * P.K;
    H.K = P.K;
    const int64_t V = P.g.V;
    for (;;) {
        const uint64_t next = atomicAdd(&P.ctrs[1], 1ull);
        if ((int64_t)next >= P.ncols) return;
        uint32_t c = (uint32_t)next;
        H.n = 0;
        {
            const uint32_t t = P.cols[c];
            const int64_t a = t / 12;
            const int ty = t % 12;
            const int64_t v1 = a + lin_of_mask(P.g, tri_step(ty, 0));
            const int64_t v2 = v1 + lin_of_mask(P.g, tri_step(ty, 1));
            H.push(ekey(P, a, v1));
            H.push(ekey(P, v1, v2));
            H.push(ekey(P, a, v2));
        }
        bool have = false;
        uint64_t tau = 0;
        for (int64_t guard = 0;; ++guard) {
            if (guard > ((int64_t)1 << 24)) {
                atomicOr(P.flags, FLAG_GUARD);
                return;
            }
            if (!have) {
                tau = H.extract_max();
                if (tau == NONE) break;  // zero column
                have = true;
            }
            const EdgeDec e = edecode(P.g, P.order, P.bpr, tau);
            if (e.mask == 0) {  // not an edge: corrupted key
                atomicOr(P.flags, FLAG_GUARD);
                return;
            }
            const uint8_t code = P.G[(int64_t)e.mask * V + e.lo];
            if (code != CODE_CRIT) {
                if (code >= 27) {  // the top of a cycle cannot be a vertex's partner
                    atomicOr(P.flags, FLAG_GUARD);
                    return;
                }
                const int64_t w = e.lo + lin27(P.g, code);
                have = false;  // tau cancels against the boundary of its partner
                if (!H.room(2)) {
                    atomicOr(P.flags, FLAG_HEAP);
                    return;
                }
                H.push(ekey(P, e.va, w));
                H.push(ekey(P, e.vb, w));
                continue;
            }
            const uint32_t o = ld_acq(&P.owner1[e.id]);
            if (o == OWN_D0) {
                atomicOr(P.flags, FLAG_GUARD);
                return;
            }
            if (o == EMPTY32 || o > c) {
                // cache Boundary(c) = {tau} + heap, then claim tau
                H.compact();
                const uint64_t len = (uint64_t)H.n + 1;
                const uint64_t off = atomicAdd(&P.ctrs[0], (unsigned long long)len);
                if (off + len > P.heap_cap || len >= (1ull << 24)) {
                    atomicOr(P.flags, FLAG_HEAP);
                    return;
                }
                uint64_t* A = P.heap + off;
                A[0] = tau;
                for (int64_t i = 0; i < H.n; ++i) A[i + 1] = H.h[i];
                st_rel64(&P.bndptr[c], (off << 24) | len);
                if (!cas32(&P.owner1[e.id], o, c)) continue;  // owner changed: look again
                if (o == EMPTY32) break;                       // column settled
                // evicted o: carry on reducing it from its cached boundary
                const uint64_t b = ld_acq64(&P.bndptr[o]);
                const uint64_t* B = P.heap + (b >> 24);
                const int64_t bl = (int64_t)(b & 0xFFFFFF);
                if (B[0] != tau) {
                    atomicOr(P.flags, FLAG_GUARD);
                    return;
                }
                if (bl - 1 > H.K) {
                    atomicOr(P.flags, FLAG_HEAP);
                    return;
                }
                for (int64_t i = 1; i < bl; ++i) H.h[i - 1] = B[i];
                H.n = bl - 1;
                c = o;
                have = true;  // tau (= B[0]) is its top
                continue;
            }
            // o < c: add the cached boundary of the earlier owner
            const uint64_t b = ld_acq64(&P.bndptr[o]);
            if (b == EMPTY64) continue;
            const uint64_t* B = P.heap + (b >> 24);
            const int64_t bl = (int64_t)(b & 0xFFFFFF);
            if (B[0] != tau) continue;  // o moved on: look again
            have = false;
            if (!H.room(bl - 1)) {
                atomicOr(P.flags, FLAG_HEAP);
                return;
            }
            for (int64_t i = 1; i < bl; ++i) H.push(B[i]);
        }
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
    if (!s.ctrs && hipMalloc(&s.ctrs, 64) != hipSuccess) return oom("counters");
    if (grow(s.colflag, s.colflag_cap, 4 * (m2 + 1), s.bytes)) return oom("column flags");
    if (grow(s.cols, s.cols_cap, 4 * (m2 + 1), s.bytes)) return oom("columns");
    if (grow(s.scanpart, s.scanpart_cap, 4 * scan_part_size(m2 + 1), s.bytes)) return oom("scan");
    if (grow(s.owner1, s.owner1_cap, 4 * 7 * V, s.bytes)) return oom("owners");
    // unpaired 2-saddles, ascending
    uint32_t* flag = (uint32_t*)s.colflag;
    uint32_t* cols = (uint32_t*)s.cols;
    int64_t ncols = 0;
    if (m2 > 0) {
        hipLaunchKernelGGL(k_colflags, dim3(nblocks(m2)), dim3(DB), 0, st, in.paired2_desc, m2, flag);
        // positions into cols (reuse cols as scan output would alias: use a second region after flags)
        uint32_t* pos = cols;  // scan in place into cols, then compact into flag space reversed below
        exclusive_scan_u32(flag, pos, m2, (uint32_t*)s.scanpart, st);
        uint32_t last_pos = 0, last_flag = 0;
        if (hipMemcpyAsync(&last_pos, pos + m2 - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&last_flag, flag + m2 - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = "D1: count read-back failed";
            return -5;
        }
        ncols = (int64_t)last_pos + last_flag;
        // compact: cols must not alias pos, so scatter into flag's buffer then copy
        hipLaunchKernelGGL(k_compact, dim3(nblocks(m2)), dim3(DB), 0, st, in.c2, in.paired2_desc, pos, m2, flag);
        if (ncols > 0 && hipMemcpyAsync(cols, flag, 4 * ncols, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            err = "D1: copy failed";
            return -5;
        }
    }
    s.ncols = ncols;
    if (grow(s.bndptr, s.bndptr_cap, 8 * (ncols + 1), s.bytes)) return oom("boundary pointers");
    if (s.heap_cap == 0) {
        size_t want = (size_t)8 * std::max<int64_t>(1 << 22, 64 * ncols);
        if (grow(s.heap, s.heap_cap, want, s.bytes)) return oom("boundary heap");
    }
    for (int attempt = 0; attempt < 6; ++attempt) {
        const int64_t T = std::max<int64_t>(1, std::min<int64_t>(ncols, s.threads));
        if (grow(s.scratch, s.scratch_cap, (size_t)8 * T * s.work_k, s.bytes)) return oom("working heaps");
        if (hipMemsetAsync(s.ctrs, 0, 64, st) != hipSuccess) return -5;
        if (hipMemsetAsync(in.flags, 0, 4, st) != hipSuccess) return -5;
        fill_u64((uint64_t*)s.bndptr, EMPTY64, ncols, st);
        if (in.m1 > 0)
            hipLaunchKernelGGL(k_init_owner, dim3(nblocks(in.m1)), dim3(DB), 0, st, in.c1, in.paired1, in.m1,
                               (uint32_t*)s.owner1);
        if (ncols == 0) return 0;
        D1K P;
        P.g = in.g;
        P.G = in.G;
        P.rank = in.rank;
        P.order = in.order;
        P.cols = cols;
        P.ncols = ncols;
        P.bpr = in.bpr;
        P.owner1 = (uint32_t*)s.owner1;
        P.bndptr = (uint64_t*)s.bndptr;
        P.heap = (uint64_t*)s.heap;
        P.heap_cap = s.heap_cap / 8;
        P.scratch = (uint64_t*)s.scratch;
        P.K = s.work_k;
        P.nthreads = T;
        P.ctrs = (unsigned long long*)s.ctrs;
        P.flags = in.flags;
        hipLaunchKernelGGL(k_d1, dim3(nblocks(T)), dim3(DB), 0, st, P);
        uint32_t f = 0;
        if (hipMemcpyAsync(&f, in.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = "D1: kernel failed";
            return -5;
        }
        if (f & FLAG_GUARD) {
            err = "D1: consistency check failed";
            return -7;
        }
        if (!(f & FLAG_HEAP)) return 0;
        // overflow: larger working heaps (fewer threads) and a larger cache
        s.work_k *= 4;
        s.threads = std::max<int64_t>(1024, s.threads / 2);
        if (grow(s.heap, s.heap_cap, s.heap_cap * 4, s.bytes)) return oom("boundary heap");
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
    void* ps[] = {s.cols, s.colflag, s.scanpart, s.owner1, s.bndptr, s.heap, s.scratch, s.ctrs};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    s = D1State();
}

}  // namespace dms
