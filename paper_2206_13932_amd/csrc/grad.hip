// Backward of the persistence map: the value of a pair's birth (death) is
// f at the highest vertex of its birth (death) simplex, so dL/df collects,
// for every vertex, the derivatives of the pair values it carries. The sum
// is made deterministic: contributions are stably sorted by vertex and each
// vertex's run is added up in the order the contributions were given.
#include "dms_internal.h"

namespace dms {

namespace {

constexpr int GB = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + GB - 1) / GB); }

__global__ void k_grad_keys(const int64_t* __restrict__ vertex, int64_t n, int64_t nvert, uint32_t* __restrict__ keys,
                            uint32_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
    if (i >= n) return;
    const int64_t v = vertex[i];
    if (v < 0 || v >= nvert) {
        atomicOr(flags, FLAG_GUARD);
        keys[i] = 0;  // kept in range; the call reports the error
        return;
    }
    keys[i] = (uint32_t)v;
}

__global__ void k_fill_f32(float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
    if (i < n) out[i] = 0.0f;
}

// one thread per run of equal keys, summing in the original order
__global__ void k_grad_runs(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ perm,
                            const float* __restrict__ grad, int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) return;
    float s = 0.0f;
    for (int64_t j = i; j < n && keys[j] == k; ++j) s += grad[perm[j]];
    out[k] = s;
}

}  // namespace

void scatter_grad(const int64_t* vertex, const float* grad, int64_t n, int64_t nvert, float* out, uint32_t* k0,
                  uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* hist, uint32_t* part, uint32_t* flags,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(nvert)), dim3(GB), 0, st, out, nvert);
    if (n == 0) return;
    hipLaunchKernelGGL(k_grad_keys, dim3(nblocks(n)), dim3(GB), 0, st, vertex, n, nvert, k0, flags);
    int bits = 8;
    while (bits < 32 && ((uint64_t)1 << bits) < (uint64_t)nvert) bits += 8;
    const int which = radix_sort_pairs<uint32_t>(k0, v0, k1, v1, n, 0, bits, true, hist, part, st);
    const uint32_t* ks = which ? k1 : k0;
    const uint32_t* vs = which ? v1 : v0;
    hipLaunchKernelGGL(k_grad_runs, dim3(nblocks(n)), dim3(GB), 0, st, ks, vs, grad, n, out);
}

}  // namespace dms
