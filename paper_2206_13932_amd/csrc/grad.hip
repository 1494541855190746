// Backward of the persistence map: the value of a pair's birth (death) is
// f at the highest vertex of its birth (death) simplex, so dL/df collects,
// for every vertex, the derivatives of the pair values it carries. The sum
// is made deterministic: contributions are stably sorted by vertex and each
// vertex's run is added up in the order the contributions were given.
#include <mutex>

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

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[MAX_DEVICES] = {nullptr};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Scratch of the allocation-free scatter (dms_scatter_grad_noalloc): sort
// keys and values, tile histograms, scan partials and the error flag for up
// to NOALLOC_MAX_CONTRIB contributions, as one array in device memory that
// each GPU the library runs on holds until the process ends. Host code must
// not use its name as an address: the per-device pointer comes from
// hipGetSymbolAddress (noalloc_scratch_init).
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

int noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return -1;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    // the layout for the largest input must fit the array
    const int64_t N = NOALLOC_MAX_CONTRIB;
    const size_t need = 4 * align256(4 * (size_t)N) + align256(4 * 256 * (size_t)sort_tiles(N)) +
                        align256(4 * (size_t)scan_part_size(256 * sort_tiles(N))) + 256;
    if (need > NOALLOC_SCRATCH_BYTES) return -2;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -3;
    g_scratch_ptr[device] = (uint8_t*)p;
    return 0;
}

int scatter_grad_noalloc(int device, const int64_t* vertex, const float* grad, int64_t n, int64_t nvert, float* out,
                         uint32_t** flag, hipStream_t st) {
    uint8_t* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (device >= 0 && device < MAX_DEVICES) base = g_scratch_ptr[device];
    }
    if (!base) return -1;
    // fixed carving for NOALLOC_MAX_CONTRIB, whatever n is
    const int64_t N = NOALLOC_MAX_CONTRIB;
    const size_t kv = align256(4 * (size_t)N);
    uint32_t* k0 = (uint32_t*)base;
    uint32_t* v0 = (uint32_t*)(base + kv);
    uint32_t* k1 = (uint32_t*)(base + 2 * kv);
    uint32_t* v1 = (uint32_t*)(base + 3 * kv);
    uint8_t* rest = base + 4 * kv;
    uint32_t* hist = (uint32_t*)rest;
    rest += align256(4 * 256 * (size_t)sort_tiles(N));
    uint32_t* part = (uint32_t*)rest;
    rest += align256(4 * (size_t)scan_part_size(256 * sort_tiles(N)));
    *flag = (uint32_t*)rest;
    fill_u32(*flag, 0, 1, st);  // the previous call's flag is still there
    scatter_grad(vertex, grad, n, nvert, out, k0, v0, k1, v1, hist, part, *flag, st);
    return 0;
}

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
