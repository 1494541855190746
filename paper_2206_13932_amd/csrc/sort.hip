// Stable LSD radix sort of (key, u32 value) pairs, 8-bit digits, and the
// device-wide exclusive scan it needs. Used for the vertex order (the
// paper's first stage, a global sort -- Sec. 7.1/7.2) and for sorting the
// critical simplices by their lexicographic keys (Alg. "Zero-persistence
// skip").
//
// Each pass: (1) per-tile digit histogram, (2) exclusive scan of the
// digit-major histogram table, (3) stable scatter. A tile is 4 wavefronts x
// 16 rounds x 64 lanes; stability inside a tile comes from ordering by
// (wave, round, lane) with ballot-based digit matching inside a wavefront
// and per-wave running counts in LDS.
#include "dms_internal.h"

namespace dms {

namespace {

constexpr int SB = 256;           // threads per block
constexpr int IPT = 16;           // rounds per wave
constexpr int TILE = SB * IPT;    // 4096 elements per tile
constexpr int WAVES = SB / 64;
constexpr int WTILE = 64 * IPT;   // 1024 elements per wave

template <typename K>
__device__ inline uint32_t digit_of(K k, int shift) {
    return (uint32_t)(k >> shift) & 0xFFu;
}

template <typename K>
__global__ __launch_bounds__(SB) void k_hist(const K* __restrict__ keys, int64_t n, int shift,
                                            uint32_t* __restrict__ hist, int64_t nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t i = base + w * WTILE + r * 64 + lane;
        if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile. Each element's rank among the tile's elements
// with the same digit comes from ballot matching inside its wavefront and
// per-wave running counts; the tile is then reordered by digit in LDS and
// written out from there, so that consecutive lanes write consecutive
// addresses of a digit's bucket (an element-order scatter writes 64
// different buckets per store instruction).
template <typename K>
__global__ __launch_bounds__(SB) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                               K* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
                                               int shift, const uint32_t* __restrict__ offs, int64_t nblk) {
    __shared__ uint32_t wcnt[WAVES][256];  // per-wave digit counts, then per-wave offsets in the digit
    __shared__ uint32_t dstart[256];       // first tile position of each digit
    __shared__ uint32_t wsum[WAVES];
    __shared__ K sk[TILE];
    __shared__ uint32_t sv[TILE];
    for (int i = threadIdx.x; i < WAVES * 256; i += SB) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    // Workgroups are dispatched to the 8 XCDs in turn, each with its own L2:
    // XCD k takes the k-th eighth of the tiles, in order, so that the runs
    // that neighbouring tiles write into one digit's bucket (consecutive
    // addresses) meet in one L2 and leave it as whole lines.
    int64_t tile;
    {
        const int64_t nt = gridDim.x, q = nt / 8, r = nt % 8, k = blockIdx.x % 8;
        tile = k * q + (k < r ? k : r) + blockIdx.x / 8;
    }
    const int64_t base = tile * TILE;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    K kk[IPT];
    uint32_t vv[IPT];
    uint32_t loc[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t i = base + w * WTILE + r * 64 + lane;
        const bool valid = i < n;
        K k = valid ? kin[i] : (K)0;
        vv[r] = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
        kk[r] = k;
        const uint32_t d = digit_of(k, shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        const uint32_t lr = (uint32_t)__popcll(peers & lt);
        uint32_t pre = 0;
        if (valid) pre = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && lr == 0) wcnt[w][d] = pre + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        loc[r] = pre + lr;
    }
    __syncthreads();
    {
        // digit d = thread: offsets of the waves inside the digit, then the
        // tile-wide exclusive scan over digits
        const int d = threadIdx.x;  // SB == 256 digits
        uint32_t acc = 0;
        for (int ww = 0; ww < WAVES; ++ww) {
            const uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = acc;
            acc += c;
        }
        uint32_t inc = acc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int ww = 0; ww < w; ++ww) before += wsum[ww];
        dstart[d] = before + inc - acc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t i = base + w * WTILE + r * 64 + lane;
        if (i < n) {
            const uint32_t d = digit_of(kk[r], shift);
            const uint32_t p = dstart[d] + wcnt[w][d] + loc[r];
            sk[p] = kk[r];
            sv[p] = vv[r];
        }
    }
    __syncthreads();
    const int64_t cnt = n - base < TILE ? n - base : TILE;
    for (int j = threadIdx.x; j < cnt; j += SB) {
        const K k = sk[j];
        const uint32_t d = digit_of(k, shift);
        const int64_t dst = (int64_t)offs[(int64_t)d * nblk + tile] + (j - dstart[d]);
        kout[dst] = k;
        vout[dst] = sv[j];
    }
}

// ---- exclusive scan of u32 (total must fit in u32) --------------------------
constexpr int CH = SB * 8;  // elements per scan block

__device__ inline uint32_t block_exclusive(uint32_t v, uint32_t* sh, uint32_t& total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < SB; d <<= 1) {
        uint32_t a = (t >= d) ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[SB - 1];
    uint32_t ex = sh[t] - v;
    __syncthreads();
    return ex;
}

__global__ __launch_bounds__(SB) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t m,
                                                   uint32_t* __restrict__ part) {
    __shared__ uint32_t sh[SB];
    const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x * 8;
    uint32_t s = 0;
    for (int j = 0; j < 8; ++j)
        if (base + j < m) s += in[base + j];
    uint32_t tot;
    block_exclusive(s, sh, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SB) void k_scan_partials(uint32_t* __restrict__ part, int64_t np) {
    __shared__ uint32_t sh[SB];
    uint32_t carry = 0;
    for (int64_t b = 0; b < np; b += SB) {
        const int64_t i = b + threadIdx.x;
        uint32_t v = i < np ? part[i] : 0;
        uint32_t tot;
        uint32_t ex = block_exclusive(v, sh, tot);
        if (i < np) part[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(SB) void k_scan_apply(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                  int64_t m, const uint32_t* __restrict__ part) {
    __shared__ uint32_t sh[SB];
    const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x * 8;
    uint32_t v[8];
    uint32_t s = 0;
    for (int j = 0; j < 8; ++j) {
        v[j] = (base + j < m) ? in[base + j] : 0;
        s += v[j];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive(s, sh, tot) + part[blockIdx.x];
    for (int j = 0; j < 8; ++j) {
        if (base + j < m) out[base + j] = ex;
        ex += v[j];
    }
}

}  // namespace

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t m, uint32_t* part, hipStream_t st) {
    if (m <= 0) return;
    const int64_t nb = (m + CH - 1) / CH;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SB), 0, st, in, m, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SB), 0, st, part, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SB), 0, st, in, out, m, part);
}

int64_t scan_part_size(int64_t m) { return (m + CH - 1) / CH + 1; }
int64_t sort_tiles(int64_t n) { return (n + TILE - 1) / TILE; }

template <typename K>
int radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int bit_begin, int bit_end,
                     bool implicit_vals, uint32_t* hist, uint32_t* part, hipStream_t st) {
    // returns 0 if the result is in (k0, v0), 1 if it is in (k1, v1)
    if (n <= 0) return 0;
    const int64_t nblk = sort_tiles(n);
    int cur = 0;
    K* kb[2] = {k0, k1};
    uint32_t* vb[2] = {v0, v1};
    bool first = true;
    for (int shift = bit_begin; shift < bit_end; shift += 8) {
        hipLaunchKernelGGL(k_hist<K>, dim3((unsigned)nblk), dim3(SB), 0, st, kb[cur], n, shift, hist, nblk);
        exclusive_scan_u32(hist, hist, 256 * nblk, part, st);
        const uint32_t* vin = (first && implicit_vals) ? nullptr : vb[cur];
        hipLaunchKernelGGL(k_scatter<K>, dim3((unsigned)nblk), dim3(SB), 0, st, kb[cur], vin, kb[cur ^ 1],
                           vb[cur ^ 1], n, shift, hist, nblk);
        cur ^= 1;
        first = false;
    }
    if (first && implicit_vals) iota_u32(v0, n, st);  // zero passes: identity permutation
    return cur;
}

template int radix_sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t, int, int, bool,
                                        uint32_t*, uint32_t*, hipStream_t);
template int radix_sort_pairs<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, int64_t, int, int, bool,
                                        uint32_t*, uint32_t*, hipStream_t);

}  // namespace dms
