// Small streaming kernels: float -> order key, rank scatter, fills, gathers.
#include "dms_internal.h"

namespace dms {

namespace {

constexpr int MB = 256;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + MB - 1) / MB); }

__global__ void k_iota(uint32_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) out[i] = (uint32_t)i;
}
__global__ void k_fill32(uint32_t* out, uint32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) out[i] = v;
}
__global__ void k_fill64(uint64_t* out, uint64_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) out[i] = v;
}

// Sec. 2.1: the symbolic perturbation orders equal values by vertex id; the
// stable sort over (key, implicit index) realises it. -0 == +0; NaN flagged.
// With an owner map (batched grids), a vertex that belongs to no grid gets
// the key 0xFFFFFFFF, above float_key(+inf) = 0xFF800000 (NaN keys, the only
// ones above that, are rejected): separator vertices come after every real
// vertex, +inf included.
__global__ void k_float_keys(const float* __restrict__ f, const uint32_t* __restrict__ owner, int64_t n,
                             uint32_t* __restrict__ keys, uint32_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i >= n) return;
    if (owner && owner[i] == EMPTY32) {
        keys[i] = 0xFFFFFFFFu;
        return;
    }
    const float v = f[i];
    if (is_nan_bits(v)) atomicOr(flags, FLAG_NAN);
    keys[i] = float_key(v);
}

__global__ void k_inverse(const uint32_t* __restrict__ perm, int64_t n, uint32_t* __restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) inv[perm[i]] = (uint32_t)i;
}

__global__ void k_rank_scatter(const uint32_t* __restrict__ order, int64_t n, uint32_t* __restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) rank[order[i]] = (uint32_t)i;
}

template <typename T>
__global__ void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ idx, T* __restrict__ dst,
                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

void iota_u32(uint32_t* out, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_iota, dim3(nblocks(n)), dim3(MB), 0, st, out, n);
}
void fill_u32(uint32_t* out, uint32_t v, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill32, dim3(nblocks(n)), dim3(MB), 0, st, out, v, n);
}
void fill_u64(uint64_t* out, uint64_t v, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill64, dim3(nblocks(n)), dim3(MB), 0, st, out, v, n);
}
void float_keys(const float* f, const uint32_t* owner, int64_t n, uint32_t* keys, uint32_t* flags, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_float_keys, dim3(nblocks(n)), dim3(MB), 0, st, f, owner, n, keys, flags);
}
void inverse_perm(const uint32_t* perm, int64_t n, uint32_t* inv, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_inverse, dim3(nblocks(n)), dim3(MB), 0, st, perm, n, inv);
}
void rank_scatter(const uint32_t* order, int64_t n, uint32_t* rank, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_rank_scatter, dim3(nblocks(n)), dim3(MB), 0, st, order, n, rank);
}
void gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_gather<uint32_t>, dim3(nblocks(n)), dim3(MB), 0, st, src, idx, dst, n);
}
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_gather<uint64_t>, dim3(nblocks(n)), dim3(MB), 0, st, src, idx, dst, n);
}

}  // namespace dms
