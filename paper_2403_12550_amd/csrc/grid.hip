// Uniform-grid spatial hash: cell keys, a stable LSD radix sort of 24-bit keys
// (three 8-bit digit passes), and the open-addressing cell table.
//
// Radix sort design for wave64: each pass is (1) a per-tile digit histogram
// (tile-major [tiles][256]), (2) one workgroup per digit that scans that
// digit's counts over the tiles and records the digit total, and (3) a stable
// scatter whose workgroups add the scanned digit totals to their offsets.  Within a tile, elements are processed in rounds of
// 256 (one per lane, in order); lanes holding the same digit are found with
// eight wavefront ballots, their rank is the popcount of the lower lanes of
// the match mask, and per-wave digit totals in LDS order the four waves.
// Equal digits therefore keep input order, which makes the sort stable.
// Tiles of 1024 keys keep a 60k-point frame at ~60 workgroups.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kIpt = 4;                        // rounds (elements per thread) per tile
constexpr int kTile = kSortThreads * kIpt;     // 1024

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Lanes of this wavefront whose (valid) digit equals mine.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                          int shift, int ntiles, uint32_t* __restrict__ counts) {
    __shared__ uint32_t s_hist[kDigits];
    for (int i = threadIdx.x; i < kDigits; i += kSortThreads) s_hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kIpt; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const uint32_t d = valid ? (keys[i] >> shift) & (kDigits - 1) : 0u;
        const uint64_t m = match_digit(d, valid);
        if (valid && (m & lanemask_lt()) == 0) atomicAdd(&s_hist[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kDigits; i += kSortThreads) counts[(int64_t)blockIdx.x * kDigits + i] = s_hist[i];
}

// Inclusive scan of x over a 256-thread workgroup (4 wavefronts); s_w holds
// the wavefront totals.
__device__ __forceinline__ uint32_t block_scan_256(uint32_t x, uint32_t* s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    for (int w = 0; w < wave; ++w) x += s_w[w];
    return x;
}

// Per-digit scan over the tiles: workgroup d writes offsets[t][d] = number
// of keys with digit d in tiles before t, and totals[d].  Each thread scans a
// contiguous run of tiles.
__global__ __launch_bounds__(kSortThreads) void k_rs_digit_scan(const uint32_t* __restrict__ counts, int ntiles,
                                                                uint32_t* __restrict__ offsets,
                                                                uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_w[kSortWaves];
    const int d = blockIdx.x;
    const int per = (ntiles + kSortThreads - 1) / kSortThreads;
    const int t0 = min(ntiles, (int)threadIdx.x * per), t1 = min(ntiles, t0 + per);
    uint32_t sum = 0;
    for (int t = t0; t < t1; ++t) sum += counts[(int64_t)t * kDigits + d];
    const uint32_t incl = block_scan_256(sum, s_w);
    uint32_t run = incl - sum;
    for (int t = t0; t < t1; ++t) {
        const uint32_t c = counts[(int64_t)t * kDigits + d];
        offsets[(int64_t)t * kDigits + d] = run;
        run += c;
    }
    if (threadIdx.x == kSortThreads - 1) totals[d] = incl;
}

__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin, int64_t n,
                                                             int shift, int ntiles,
                                                             const uint32_t* __restrict__ offsets,
                                                             const uint32_t* __restrict__ totals,
                                                             uint32_t* __restrict__ kout,
                                                             uint32_t* __restrict__ vout) {
    static_assert(kSortThreads == kDigits, "one thread per digit");
    __shared__ uint32_t s_base[kDigits];
    __shared__ uint32_t s_wcount[kSortWaves][kDigits];
    __shared__ uint32_t s_w[kSortWaves];
    {
        // start of digit d in the output: keys with a lower digit, then
        // keys with digit d in earlier tiles
        const int d = threadIdx.x;
        const uint32_t tot = totals[d];
        const uint32_t below = block_scan_256(tot, s_w) - tot;
        s_base[d] = below + offsets[(int64_t)blockIdx.x * kDigits + d];
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s_wcount[w][d] = 0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kIpt; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & (kDigits - 1);
        const uint64_t m = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
        const uint32_t cnt = (uint32_t)__popcll(m);
        const bool leader = valid && rank == 0;
        if (leader) s_wcount[wave][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t off = s_base[d] + rank;
            for (int w = 0; w < wave; ++w) off += s_wcount[w][d];
            if (off < (uint64_t)n) {   // always true for a consistent scan; guards the write
                kout[off] = key;
                vout[off] = val;
            }
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&s_base[d], cnt);
            s_wcount[wave][d] = 0;
        }
        __syncthreads();
    }
}

__global__ void k_cell_keys(SegSet S, int64_t total, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            int* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int p = S.find(i);
    const Seg sg = S.get(p);
    const int64_t j = i - sg.off;
    const float x = sg.xyz[j], y = sg.xyz[sg.n + j], z = sg.xyz[2 * sg.n + j];
    if (!finite3(x, y, z)) atomicOr(err, kErrNonFinite);
    const Cell c = cell_of(x, y, z, sg.inv_h);
    keys[i] = ((uint32_t)p << (3 * kCellBits)) | cell_key(c.x, c.y, c.z);
    vals[i] = (uint32_t)i;
}

__global__ void k_table_clear(uint4* __restrict__ table, uint32_t cap) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) table[i] = make_uint4(kEmptyKey, 0u, 0u, 0u);
}

__global__ void k_table_build(const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ svals, int64_t total,
                              SegSet S, float4* __restrict__ spts, uint4* __restrict__ table, uint32_t mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    uint32_t v = svals[i];
    if (v >= (uint64_t)total) v = 0;   // always a permutation; guards the gather
    const Seg sg = S.get(S.find(v));
    const int64_t j = (int64_t)v - sg.off;
    spts[i] = make_float4(sg.xyz[j], sg.xyz[sg.n + j], sg.xyz[2 * sg.n + j], __uint_as_float((uint32_t)j));
    const uint32_t key = skeys[i];
    if (i == 0 || skeys[i - 1] != key) {
        uint32_t cnt = 1;
        while (i + cnt < total && skeys[i + cnt] == key) ++cnt;
        uint32_t s = hash_slot(key, mask);
        while (true) {
            const uint32_t prev = atomicCAS(&table[s].x, kEmptyKey, key);
            if (prev == kEmptyKey) {
                table[s].y = (uint32_t)i;
                table[s].z = cnt;
                break;
            }
            s = (s + 1u) & mask;
        }
    }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t radix_scratch_bytes(int64_t n) {
    const int64_t ntiles = std::max<int64_t>(1, ceil_div(n, kTile));
    return (size_t)(2 * ntiles * kDigits + kDigits + 64) * sizeof(uint32_t);
}

hipError_t radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, int64_t n,
                      int passes, void* scratch, hipStream_t s, uint32_t** keys_out, uint32_t** vals_out) {
    *keys_out = keys_a;
    *vals_out = vals_a;
    if (n <= 0) return hipSuccess;
    const int ntiles = (int)ceil_div(n, kTile);
    uint32_t* counts = static_cast<uint32_t*>(scratch);
    uint32_t* offs = counts + (int64_t)ntiles * kDigits;
    uint32_t* totals = offs + (int64_t)ntiles * kDigits;
    uint32_t* kin = keys_a;
    uint32_t* vin = vals_a;
    uint32_t* kout = keys_b;
    uint32_t* vout = vals_b;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * kDigitBits;
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(kSortThreads), 0, s, kin, n, shift, ntiles, counts);
        hipLaunchKernelGGL(k_rs_digit_scan, dim3(kDigits), dim3(kSortThreads), 0, s, (const uint32_t*)counts, ntiles,
                           offs, totals);
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, kin, vin, n, shift, ntiles,
                           (const uint32_t*)offs, (const uint32_t*)totals, kout, vout);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    *keys_out = kin;
    *vals_out = vin;
    return hipGetLastError();
}

hipError_t launch_cell_keys(const SegSet& S, int64_t total, uint32_t* keys, uint32_t* vals, int* err,
                            hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_keys, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, S, total, keys, vals, err);
    return hipGetLastError();
}

hipError_t launch_table_clear(uint4* table, uint32_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_table_clear, dim3((cap + 255) / 256), dim3(256), 0, s, table, cap);
    return hipGetLastError();
}

hipError_t launch_table_build(const uint32_t* skeys, const uint32_t* svals, int64_t total, const SegSet& S,
                              float4* spts, uint4* table, uint32_t mask, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_build, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, skeys, svals, total, S,
                       spts, table, mask);
    return hipGetLastError();
}

}  // namespace gicp
