// Internal host/device interfaces of the DMS library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dms_device.h"

namespace dms {

// Critical-cell lists written by the gradient kernel, with packed
// lexicographic keys (bpr = bits per rank):
//   C0 key = rank; C1 key = (r0 << bpr) | r1;
//   C2 key = hi (r0 << bpr) | r1, lo r2; C3 key = hi (r0 << bpr) | r1, lo (r2 << bpr) | r3
// with r0 > r1 > r2 > r3 the vertex ranks in decreasing order.
struct CritLists {
    uint32_t* count;  // 4 device counters
    uint32_t cap[4];
    uint32_t* id0;
    uint32_t* key0;
    uint32_t* id1;
    uint64_t* key1;
    uint32_t* id2;
    uint64_t* key2hi;
    uint32_t* key2lo;
    uint32_t* id3;
    uint64_t* key3hi;
    uint64_t* key3lo;
};

constexpr uint32_t EMPTY32 = 0xFFFFFFFFu;
constexpr uint64_t EMPTY64 = ~0ull;

// error flag bits
enum : uint32_t { FLAG_NAN = 1u, FLAG_GUARD = 2u, FLAG_HEAP = 4u, FLAG_WORK = 8u };

// gradient.hip
void launch_gradient(const GridDev& g, const uint32_t* rank, uint8_t* G, int bpr, const CritLists& cl,
                     hipStream_t st);

// sort.hip
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t m, uint32_t* part, hipStream_t st);
int64_t scan_part_size(int64_t m);
int64_t sort_tiles(int64_t n);
template <typename K>
int radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int bit_begin, int bit_end,
                     bool implicit_vals, uint32_t* hist, uint32_t* part, hipStream_t st);

// misc.hip
void iota_u32(uint32_t* out, int64_t n, hipStream_t st);
void fill_u32(uint32_t* out, uint32_t v, int64_t n, hipStream_t st);
void fill_u64(uint64_t* out, uint64_t v, int64_t n, hipStream_t st);
void float_keys(const float* f, int64_t n, uint32_t* keys, uint32_t* flags, hipStream_t st);
void rank_scatter(const uint32_t* order, int64_t n, uint32_t* rank, hipStream_t st);
void gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, int64_t n, hipStream_t st);
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t st);

// pairs.hip -- D0 / D2
void trace_d0(const GridDev& g, const uint8_t* G, const uint32_t* rank, const uint32_t* c1, int64_t m,
              uint32_t* na, uint32_t* nb, uint32_t* flags, hipStream_t st);
void tet_positions(const uint32_t* c3_sorted, int64_t m, uint32_t* tet2pos, hipStream_t st);
void trace_d2(const GridDev& g, const uint8_t* G, const uint32_t* tet2pos, const uint32_t* c2_sorted, int64_t m,
              uint32_t* na, uint32_t* nb, uint32_t* flags, hipStream_t st);
void reduce_pairs(const uint32_t* na, const uint32_t* nb, int64_t m, uint32_t* owner, uint64_t* bnd,
                  uint32_t* flags, unsigned long long* stats, hipStream_t st);
void settled_columns(const uint64_t* bnd, const uint32_t* owner, int64_t m, uint8_t* paired, hipStream_t st);

// grad.hip
void scatter_grad(const int64_t* vertex, const float* grad, int64_t n, int64_t nvert, float* out, uint32_t* k0,
                  uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* hist, uint32_t* part, uint32_t* flags,
                  hipStream_t st);

}  // namespace dms
