/*
 * dms.h -- C ABI of the Discrete Morse Sandwich library for MI355X (gfx950).
 *
 * Computes the persistence diagrams D0, D1 and D2 of a piecewise-linear scalar
 * field on a 3D regular grid, triangulated implicitly (Freudenthal/Kuhn, 6
 * tetrahedra per cube; Sec. 2.1 of Guillou, Vidal, Tierny, "Discrete Morse
 * Sandwich"). The problem statement (Sec. 1 and 2.4): a scalar field on the
 * vertices of a simplicial complex goes in; persistence pairs (birth
 * p-simplex, death (p+1)-simplex) per dimension come out, plus the classes of
 * infinite persistence (Sec. 6).
 *
 * Conventions (part of the ABI):
 *  - Vertex id v = x + nx*(y + ny*z), x fastest; a field is float32,
 *    contiguous, shaped [nz][ny][nx].
 *  - Vertex order: by (f(v), v), ties broken by the lower id (the paper's
 *    symbolic perturbation, Sec. 2.1); -0 == +0; NaN is an error.
 *  - Simplex id = anchor * T_k + type, T = {1, 7, 12, 6} for k = 0..3, the
 *    anchor being the vertex with the smallest coordinates. A simplex is the
 *    chain anchor, anchor+s0, anchor+s0+s1, ... with steps given as axis masks
 *    (bit0 = x, bit1 = y, bit2 = z):
 *      edges      type t: step (t+1)
 *      triangles  types 0..11: (1,2) (1,4) (1,6) (2,1) (2,4) (2,5) (3,4) (4,1)
 *                              (4,2) (4,3) (5,2) (6,1)
 *      tetrahedra types 0..5:  (1,2,4) (1,4,2) (2,1,4) (2,4,1) (4,1,2) (4,2,1)
 *  - Pairs are sorted by (birth, death) as int64, classes of infinite
 *    persistence (death = -1) last.
 *  - A grid with nz = 1 is a 2D grid: the plane z = 0 of the same
 *    triangulation (edges of types 0, 1, 2; triangles of types 0 and 3).
 *    There the method computes D0 and, from the stable sets of the
 *    1-saddles, D1 (Sec. 3: the sandwich is for 3D data only); D2 is empty.
 *  - All pointers named d_* are device pointers on the context's device.
 *    The caller owns them; the library only borrows them for the duration of
 *    the call's work on the context's stream.
 *
 * Errors: every call returns DMS_OK or a negative code; dms_last_error()
 * returns a text. A context is not thread-safe: use one context per stream.
 */
#ifndef DMS_H
#define DMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dms_ctx dms_ctx;

typedef struct {
    int32_t nx, ny, nz; /* vertex counts per axis: nx, ny >= 2; nz >= 2, or 1 for a
                           2D grid; 12*nx*ny*nz < 2^32 */
} dms_grid;

typedef struct {
    int64_t birth, death; /* simplex ids; death = -1 for infinite persistence */
} dms_pair;

typedef struct {
    int64_t n_crit[4]; /* critical simplices per dimension (Alg. "Zero-persistence skip") */
} dms_gradient_info;

typedef struct {
    /* caller-owned device buffers, one per dimension (D0, D1, D2) */
    dms_pair* pairs[3];
    int64_t cap[3];  /* capacity in pairs */
    int64_t n[3];    /* out: pairs written, or required on DMS_E_CAPACITY */
    /* optional (NULL allowed): highest vertex of birth / death simplex (-1 for
       infinite death) and its value (infinite death: the maximum of f, Sec. 6) */
    int64_t* birth_vertex[3];
    int64_t* death_vertex[3];
    float* birth_value[3];
    float* death_value[3];
} dms_diagram_out;

enum {
    DMS_OK = 0,
    DMS_E_INVAL = -1,    /* bad argument (grid too small or too large, NULL)        */
    DMS_E_NAN = -2,      /* the field holds a NaN                                    */
    DMS_E_NOMEM = -3,    /* the hbm_budget_bytes of the context would be exceeded    */
    DMS_E_CAPACITY = -4, /* an output buffer is too small; n[] holds the need        */
    DMS_E_HIP = -5,      /* a HIP runtime call failed                                */
    DMS_E_STATE = -6,    /* calls out of order (pairs before gradient, D1 before D0/D2) */
    DMS_E_INTERNAL = -7  /* an internal consistency check failed                     */
};

/* flags of dms_gradient / dms_diagram (other bits: DMS_E_INVAL).
 * DMS_VIRTUAL_MAX set: the outside of the domain is one maximum of value
 *   +inf (Sec. 5.2, "Domains with boundary"): the exact diagrams of the
 *   lower-star filtration of the grid. The usual choice.
 * DMS_VIRTUAL_MAX clear: the adjustment is off (App. A, "Boundary
 *   perturbations"; the paper's more stable option for the global maximum):
 *   the outside is no node of the dual union-find, so a 2-saddle whose stable
 *   set reaches the boundary joins nothing there. The rest runs as is; what
 *   stays unpaired is a class of infinite persistence (Sec. 6): a 2-saddle
 *   whose boundary reduces to zero in D1 is an infinite D2 class (3D), such a
 *   1-saddle an infinite D1 class (2D); maxima never killed are infinite D2
 *   classes on a 2D grid and are not reported on a 3D grid (there is no D3).
 *   D0 is the same in both modes. dms_diagram_batch requires the flag. */
enum {
    DMS_VIRTUAL_MAX = 1u << 0
};

/* Create a context on `device`, enqueuing on `hip_stream` (NULL = the null
 * stream). hbm_budget_bytes = 0 means no limit; otherwise it bounds all the
 * device memory the context holds (D1's boundary storage and the generator
 * export's working buffers included), and a call that would pass it fails
 * with DMS_E_NOMEM. The context owns all internal
 * device state (order, gradient, critical sets, union-find owners, boundary
 * heap), which persists from dms_gradient() to the next dms_gradient() /
 * dms_diagram() or dms_destroy(). */
int dms_create(dms_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes);
void dms_destroy(dms_ctx* ctx);
const char* dms_last_error(const dms_ctx* ctx);

/* Vertex order (Sec. 2.1), discrete gradient by expansions and critical
 * simplices sorted by the lexicographic order (Sec. 2.2, 2.6 and Alg.
 * "Zero-persistence skip"). d_field: nx*ny*nz floats. info may be NULL. */
int dms_gradient(dms_ctx* ctx, const float* d_field, dms_grid grid, uint32_t flags, dms_gradient_info* info);

/* D0 (Sec. 5.1) and D2 (Sec. 5.2) from the gradient left by dms_gradient.
 * On a 2D grid the stable sets of the 1-saddles are traced here as well and
 * D2 holds only maxima no saddle kills (none with DMS_VIRTUAL_MAX). Without
 * DMS_VIRTUAL_MAX the infinite D2 classes of a 3D grid come with D1 (the
 * 2-saddles left after it), so this call reports none.
 * Writes the pairs (sorted, infinite classes last) to d0 / d2 (device).
 * On DMS_E_CAPACITY the required counts are in *n0 / *n2 and nothing is
 * written. Returns DMS_E_STATE without a prior dms_gradient. */
int dms_pairs_d0_d2(dms_ctx* ctx, dms_pair* d0, int64_t cap0, int64_t* n0, dms_pair* d2, int64_t cap2,
                    int64_t* n2);

/* D1 by PairCriticalSimplices on the 2-saddles left unpaired by D2 (Sec. 3
 * and 4, Alg. "PairCriticalSimplices"), with boundary caching and clearing;
 * on a 2D grid, the (1-saddle, maximum) pairs of the dual union-find over
 * the stable sets (Sec. 5.2 one dimension down).
 * Requires dms_pairs_d0_d2 first (DMS_E_STATE otherwise). */
int dms_pairs_d1(dms_ctx* ctx, dms_pair* d1, int64_t cap1, int64_t* n1);

/* The whole pipeline: gradient, D0/D2, D1, infinite classes (Sec. 6). */
int dms_diagram(dms_ctx* ctx, const float* d_field, dms_grid grid, uint32_t flags, dms_diagram_out* out);

/* Persistent 1-cycle generators (Sec. 8): for a D1 pair (tau, sigma), the
 * boundary of sigma as it stood when sigma was paired with tau. It is a
 * 1-cycle whose highest edge is tau, and it differs from the boundary of
 * sigma by boundaries of triangles that precede sigma in the filtration.
 * Which such cycle is returned depends on the order in which concurrent
 * columns were reduced; the birth edge, the death triangle and the three
 * properties above do not.
 *
 * Needs dms_pairs_d1 or dms_diagram on one 3D field (not a batch, not a 2D
 * grid, where D1 comes from the dual union-find) first: DMS_E_STATE
 * otherwise. Cycle i belongs to the i-th finite pair of the D1
 * list those calls write (finite pairs come first, in increasing birth-edge
 * id). Output, device memory owned by the caller:
 *   d_offsets[0..n_pairs]  int64, cycle i = d_edges[d_offsets[i] .. d_offsets[i+1])
 *   d_edges[0..n_edges)    int64 edge ids (anchor * 7 + type), ascending per cycle
 * *n_pairs and *n_edges are always set. If cap_offsets < n_pairs + 1 or
 * cap_edges < n_edges, nothing is written and DMS_E_CAPACITY is returned
 * (NULL buffers with zero capacities ask for the sizes). Working memory grows
 * with the total length of the cycles and stays with the context. */
int dms_d1_generators(dms_ctx* ctx, int64_t* d_offsets, int64_t cap_offsets, int64_t* d_edges, int64_t cap_edges,
                      int64_t* n_pairs, int64_t* n_edges);

/* ---- Batching: many grids in one pipeline run ----
 * The grids are placed as disjoint boxes in one super grid of cross-section
 * cross_x * cross_y, separated by planes of separator vertices; one pipeline
 * run computes all diagrams. Separators are ordered above every real value,
 * +inf included (items may hold +-inf), so in the lower-star filtration they
 * come after every real vertex and a real vertex's lower star stays inside
 * its box: every pair is the pair the grid has alone, with the same local
 * simplex ids; around each box the separator region closes the boundary as
 * the virtual maximum of D2 does (Sec. 5.2), and a grid's infinite D0 class
 * is reported
 * as infinite (death = -1). */
typedef struct {
    int32_t nx, ny, nz; /* the item's grid, each side >= 2                       */
    int32_t reserved;
    int64_t offset;     /* element offset of its field [nz][ny][nx] in d_fields  */
} dms_item;

typedef struct {
    int32_t cross_x, cross_y; /* super-grid cross-section (>= every side + 1);
                                 0 = the smallest multiple of 16 that fits     */
    int32_t z_quantum;        /* depth rounded up to a multiple (0 = 16) so
                                 that super grids repeat                       */
    int32_t use_graph;        /* replay the order + gradient kernels from a
                                 captured hipGraph per super grid (needs a
                                 non-default stream)                           */
} dms_batch_opts;

typedef struct {
    dms_pair* pairs[3];       /* device, caller-owned: every item's pairs of
                                 dimension d, item after item, each item's in
                                 the order of dms_diagram                       */
    int64_t cap[3];
    int64_t n[3];             /* pairs written (or needed on DMS_E_CAPACITY)   */
    int64_t* item_start[3];   /* host, caller-owned, nitems + 1 entries: item
                                 i's pairs are [item_start[d][i], [i + 1])      */
} dms_batch_out;

/* Diagrams of nitems grids whose float32 fields lie in d_fields (device).
 * items and opts are host memory (opts may be NULL). DMS_E_INVAL for an item
 * wider than the cross-section or a super grid over the size limit. */
int dms_diagram_batch(dms_ctx* ctx, const float* d_fields, const dms_item* items, int32_t nitems, uint32_t flags,
                      const dms_batch_opts* opts, dms_batch_out* out);

/* The super grid (X, Y, Z) a batch would use, computed on the host only; its
 * X*Y*Z vertices set the batch's device footprint. origins (host, 3*nitems,
 * may be NULL) receives each item's box origin (x, y, z) in the super grid. */
int dms_batch_layout(const dms_item* items, int32_t nitems, const dms_batch_opts* opts, int32_t dims[3],
                     int32_t* origins);

/* Last batch: [0..2] super grid X, Y, Z, [3] real vertices, [4] graph
 * launches, [5] graph captures, [6] runs without a graph, [7] items. */
int dms_batch_info(const dms_ctx* ctx, int64_t info[8]);

/* Backward of the persistence map (the pair values are f at the highest
 * vertices of the birth and death simplices, Sec. 2.1 and Sec. 6): writes
 * d_grad_field[v] = sum of d_grad[i] over the i with d_vertex[i] == v, for
 * v in [0, nvert), and 0 elsewhere. All pointers are device pointers on the
 * context's device: d_vertex int64[n], d_grad float[n], d_grad_field
 * float[nvert] (owned by the caller; fully overwritten). Deterministic: each
 * vertex's contributions are added in increasing i, in float32, starting
 * from 0. n may be 0. A vertex outside [0, nvert) is DMS_E_INVAL (its
 * contribution is dropped). Synchronises the context's stream. */
int dms_scatter_grad(dms_ctx* ctx, int64_t n, const int64_t* d_vertex, const float* d_grad, int64_t nvert,
                     float* d_grad_field);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): dms_scatter_grad with the same arguments, result and errors,
 * but it calls no hipMalloc / hipFree and no allocating library routine. Its
 * sort buffers live in one static device array per GPU (65 MiB + 64 KiB,
 * held from the first dms_create on that GPU until the process ends), so
 * n <= 4194304 (2^22) contributions; more is DMS_E_INVAL, nothing enqueued.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other contexts, other threads) race and must be
 * serialised by the caller. The array keeps the last call's contents; the
 * call clears what must start at zero. Synchronises the context's stream. */
int dms_scatter_grad_noalloc(dms_ctx* ctx, int64_t n, const int64_t* d_vertex, const float* d_grad, int64_t nvert,
                             float* d_grad_field);

/* Inspection of internal state for tests: copies the device buffer `what`
 * (see DMS_BUF_*) to host memory `dst` of `cap` bytes; returns the byte
 * size of the buffer (or a negative error). */
enum {
    DMS_BUF_RANK = 0,      /* u32[V] vertex order                                 */
    DMS_BUF_GRADIENT = 1,  /* u8[26*V] gradient byte planes                       */
    DMS_BUF_CRIT0 = 2,     /* u32 critical ids sorted by the lexicographic order, */
    DMS_BUF_CRIT1 = 3,     /*   dimensions 0..3 (2..5)                            */
    DMS_BUF_CRIT2 = 4,
    DMS_BUF_CRIT3 = 5,
    DMS_BUF_ARCS0 = 6,     /* u32[2*n] D0 arcs (rank of minimum a, b) per C1      */
    DMS_BUF_ARCS2 = 7,     /* u32[2*n] D2 arcs (age of maximum a, b), C2 reversed
                              (2D grids: the dual arcs of the 1-saddles, C1 reversed) */
    DMS_BUF_STATS = 8,     /* u64[48] work counters of the last call: D0 steps,
                              evictions; D2 steps, evictions; D1 steps, evictions,
                              boundary additions, deferrals, published entries,
                              restarts; per D1 pass (columns, microseconds);
                              workgroup rounds, edges expanded, entries moved;
                              per column of the workgroup passes: longest and
                              total microseconds, most rounds, most boundary
                              additions, longest boundary, columns over 1 ms;
                              microseconds of those columns per phase (window
                              scan, slot assignment, batched loads, sort, low
                              merge, top merge, owner rule, additions, claims
                              and reloads, refills), then their rounds and
                              additions; additions made by one full merge;
                              the sixth D1 pass (columns, microseconds);
                              cooperative full merges, their parts merged by
                              helping workgroups; additions made with the cached
                              boundary under DMS_OPT_D1_NO_CACHE                */
    DMS_BUF_D1LEN = 9      /* u64 per D1 column: last cached boundary
                              (offset << 24 | length)                             */
};
int64_t dms_debug_copy(dms_ctx* ctx, int what, void* dst, int64_t cap);

/* Debug and ablation options of a context (inspection, tests and the
 * variant measurements of Sec. 9.2; a new context has all of them 0). They
 * change no result, only how the work is split, logged or how much of it
 * there is:
 *   DMS_OPT_D1_SMALL_PASSES  value != 0: the D1 passes get tiny capacities
 *       (lane heaps of 3 and 4 keys, first workgroup pass 24 keys, cached
 *       boundaries of more than 2 keys added by full merges), so that small
 *       grids go through every pass of PairCriticalSimplices;
 *   DMS_OPT_LOG_PASSES       value != 0: one line per D1 pass on stderr;
 *   DMS_OPT_D1_NO_SANDWICH   value != 0: PairCriticalSimplices without the
 *       sandwich (Sec. 3): every 2-saddle is a column, also those D2 already
 *       paired (their columns reduce to zero), and 1-saddles paired by D0 are
 *       not set aside (they never become a pivot). Defined with
 *       DMS_VIRTUAL_MAX only: a D1 call without it returns DMS_E_INVAL
 *       (without the outside node, D2 from the dual union-find is not the
 *       plain reduction's, so D1 over every 2-saddle would differ);
 *   DMS_OPT_D1_NO_CACHE      value != 0: PairCriticalSimplices without
 *       boundary caching (Sec. 4.1(b)): when a column's top is the pivot of an
 *       earlier column, the boundary of that column's 2-saddle (its three
 *       edges) is added and reduced again instead of the earlier column's
 *       cached reduced boundary. In the lock-free reduction that
 *       re-reduction follows the owners of the moment, which evictions may
 *       have changed since the earlier column's own reduction, so it can miss
 *       the pivot: a column re-reduces only below every pivot it re-reduced
 *       before, and pivots met inside a re-reduction, or one that comes back,
 *       are added with cached boundaries (counted in DMS_BUF_STATS). The work
 *       can grow steeply on noisy fields; the kernels' step bounds then end
 *       the call with DMS_E_INTERNAL;
 *   DMS_OPT_D1_HEAP_KEYS     value > 0: every later D1 run starts with a
 *       publication heap (the cached boundaries) of that many keys, at least
 *       64, instead of 32 keys per column with a floor of 4 M keys. A small
 *       grid then overflows it and goes through D1's restart: the heap grows
 *       and D1 runs again from its first pass, up to three times (DMS_E_NOMEM
 *       after that); the restarts are counted in DMS_BUF_STATS. 0 restores the
 *       default sizing (a heap larger than it is kept); a negative value
 *       returns DMS_E_INVAL.
 * Returns DMS_OK, or DMS_E_INVAL for an unknown option or a NULL ctx. */
enum {
    DMS_OPT_D1_SMALL_PASSES = 1,
    DMS_OPT_LOG_PASSES = 2,
    DMS_OPT_D1_NO_SANDWICH = 3,
    DMS_OPT_D1_NO_CACHE = 4,
    DMS_OPT_D1_HEAP_KEYS = 5
};
int dms_set_option(dms_ctx* ctx, int32_t option, int64_t value);

/* Milliseconds of the last call's stages, measured with HIP events on the
 * context's stream: [0] order, [1] gradient+critical (with the count
 * read-back), [2] critical sort, [3] D0+D2, [4] D1, [5] output assembly,
 * [6] total, [7] the gradient kernel alone. -1 for a stage not run. */
int dms_stage_ms(const dms_ctx* ctx, float ms[8]);

#ifdef __cplusplus
}
#endif

#endif /* DMS_H */
