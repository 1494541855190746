// D1: PairCriticalSimplices on the 2-saddles left unpaired by D2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dms_device.h"

namespace dms {

struct D1Inputs {
    GridDev g;
    const uint8_t* G;
    const uint32_t* rank;
    const uint32_t* order;
    const uint32_t* c1;   // critical edges, ascending
    int64_t m1;
    const uint32_t* c2;   // critical triangles, ascending
    int64_t m2;
    const uint8_t* paired1;       // per C1 position: paired in D0
    const uint8_t* paired2_desc;  // per decreasing C2 position: paired in D2
    int bpr;
    uint32_t* flags;
    bool small_passes = false;  // debug: tiny pass capacities, every pass used
    bool log_passes = false;    // debug: one stderr line per pass
    bool no_sandwich = false;   // ablation: every 2-saddle is a column, no D0 set-aside
    bool no_cache = false;      // ablation: add earlier owners' 2-saddle boundaries, not their cached ones
    int64_t heap_keys = 0;      // debug: the publication heap starts with this many keys (0: default sizing)
};

struct D1State {
    void* cols = nullptr;     // u32 unpaired 2-saddles (ascending)
    size_t cols_cap = 0;
    void* colflag = nullptr;  // u32 scratch for compaction
    size_t colflag_cap = 0;
    void* scanpart = nullptr;
    size_t scanpart_cap = 0;
    void* owner1 = nullptr;   // u32[7V] owner column of a critical edge (sparse)
    size_t owner1_cap = 0;
    void* bndptr = nullptr;   // u64 per column: published boundary (offset << 24 | length)
    size_t bndptr_cap = 0;
    void* heap = nullptr;     // u64 published boundaries (bump allocated)
    size_t heap_cap = 0;      // bytes
    void* scratch = nullptr;  // u64 per-thread working heaps (interleaved)
    size_t scratch_cap = 0;
    void* dq = nullptr;       // deferral queues
    size_t dq_cap = 0;
    void* ctrs = nullptr;     // u64 counters (heap top, work cursor, deferrals, work counts)
    int64_t ncols = 0;
    size_t bytes = 0;         // device bytes held by D1 (ctrs aside)
    size_t limit = 0;         // most bytes D1 may hold (0 = no limit)
    // last run: [0] loop steps, [1] evictions, [2] cached-boundary additions,
    // [3] deferrals, [4] published entries, [5] restarts
    uint64_t stats[6] = {0, 0, 0, 0, 0, 0};
    // per pass: columns to process, microseconds
    uint64_t pass_work[6] = {0, 0, 0, 0, 0, 0};
    uint64_t pass_us[6] = {0, 0, 0, 0, 0, 0};
    // workgroup passes: rounds, edges expanded, boundary entries moved by merges
    uint64_t wide[4] = {0, 0, 0, 0};
    // workgroup passes, per column taken from the queue: longest (us), total (us),
    // most rounds, most cached-boundary additions, longest boundary, columns over 1 ms
    uint64_t wide_t[6] = {0, 0, 0, 0, 0, 0};
    // microseconds per phase summed over the columns over 1 ms: window scan,
    // slot assignment, batched loads, sort, merge into the low part, merge into
    // the top, owner rule, cached-boundary additions, claims and reloads,
    // refills; then those columns' rounds and additions
    uint64_t wide_ph[12] = {0};
    // cooperative full merges, and their parts merged by helping workgroups
    uint64_t coop[2] = {0, 0};
    bool all_cols = false;  // last run had every 2-saddle as a column (no sandwich)
    uint64_t nc_fallbacks = 0;  // ablation without caching: pivots that came back and got the cached boundary
    // per-run data for emission
    GridDev g{};
    const uint32_t* order = nullptr;
    int bpr = 1;
    // working buffers of the generator export, and what they hold: the
    // cancelled (pair, edge) keys of the last run once gen_n >= 0
    void* gbuf[12] = {nullptr};
    size_t gcap[12] = {0};
    int64_t gen_n = -1, gen_ne = 0, gen_total = 0;
    int gen_sorted = 0;  // which key buffer holds the sorted keys
};

// budget_left: most device bytes D1 may hold (0 = no limit); more is DMS_E_NOMEM
int d1_run(D1State& s, const D1Inputs& in, hipStream_t st, size_t budget_left, std::string& err);
void d1_emit(D1State& s, int64_t m1, const uint8_t* paired1, const uint32_t* c1, uint64_t* key, uint32_t* death,
             uint32_t* cnt, hipStream_t st);
void d1_emit_essential2(D1State& s, int64_t m2, const uint8_t* paired2_desc, const uint32_t* c2, uint64_t* key,
                        uint32_t* death, uint32_t* cnt, hipStream_t st);
// Persistent 1-cycle generators of the finite D1 pairs (Sec. 8): for the
// i-th finite pair in increasing birth-edge order, the edge ids (ascending)
// of the boundary cached when its 2-saddle claimed the birth edge, mod-2
// cancelled. Writes offsets[0..n] and edges[0..E) only when cap_off >= n + 1
// and cap_edges >= E; always sets *n_pairs and *n_edges. Returns 0, 1 when
// a buffer is too small, or a negative DMS error code (message in err).
int d1_generators(D1State& s, int64_t* offsets, int64_t cap_off, int64_t* edges, int64_t cap_edges,
                  int64_t* n_pairs, int64_t* n_edges, uint32_t* flags, hipStream_t st, std::string& err);
void d1_free(D1State& s);

}  // namespace dms
