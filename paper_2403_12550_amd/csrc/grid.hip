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
    // (the strided counts are loaded eight at a time: one memory round trip
    // per eight tiles instead of one per tile)
    constexpr int kU = 8;
    uint32_t sum = 0;
    for (int t = t0; t < t1; t += kU) {
        uint32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) c[u] = t + u < t1 ? counts[(int64_t)(t + u) * kDigits + d] : 0u;
#pragma unroll
        for (int u = 0; u < kU; ++u) sum += c[u];
    }
    const uint32_t incl = block_scan_256(sum, s_w);
    uint32_t run = incl - sum;
    for (int t = t0; t < t1; t += kU) {
        uint32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) c[u] = t + u < t1 ? counts[(int64_t)(t + u) * kDigits + d] : 0u;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (t + u < t1) {
                offsets[(int64_t)(t + u) * kDigits + d] = run;
                run += c[u];
            }
        }
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

// ---------------------------------------------------------------------------
// Incremental map update: the new points, sorted by cell key on their own,
// are merged into the map's sorted run.  An old point moves forward by the
// number of new keys below its key, a new point by the number of old keys at
// or below its key, so equal keys keep the old points first (the order a
// stable sort of the concatenation [old; new] would give).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t count_below(const uint32_t* __restrict__ a, int64_t n, uint32_t key, bool or_equal) {
    int64_t lo = 0, hi = n;   // first index whose key is above (or at) `key`
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const bool before = or_equal ? (a[mid] <= key) : (a[mid] < key);
        if (before) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_merge_old(const uint32_t* __restrict__ okeys, const float4* __restrict__ opts,
                            const float4* __restrict__ ocov, int64_t m_old, const uint32_t* __restrict__ nkeys,
                            int64_t m_new, uint32_t* __restrict__ keys, float4* __restrict__ pts,
                            float4* __restrict__ cov) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m_old) return;
    const uint32_t k = okeys[i];
    const int64_t o = i + count_below(nkeys, m_new, k, false);
    keys[o] = k;
    pts[o] = opts[i];
    cov[2 * o] = ocov[2 * i];
    cov[2 * o + 1] = ocov[2 * i + 1];
}

__global__ void k_merge_new(const uint32_t* __restrict__ nkeys, const uint32_t* __restrict__ nvals,
                            const float* __restrict__ means, const float4* __restrict__ ncov, int64_t m_new,
                            const uint32_t* __restrict__ okeys, int64_t m_old, uint32_t* __restrict__ keys,
                            float4* __restrict__ pts, float4* __restrict__ cov) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_new) return;
    const uint32_t k = nkeys[j];
    uint32_t v = nvals[j];
    if (v >= (uint64_t)m_new) v = 0;   // always a permutation; guards the gather
    const int64_t o = j + count_below(okeys, m_old, k, true);
    keys[o] = k;
    pts[o] = make_float4(means[v], means[m_new + v], means[2 * m_new + v], __uint_as_float((uint32_t)(m_old + v)));
    cov[2 * o] = ncov[2 * j];
    cov[2 * o + 1] = ncov[2 * j + 1];
}

// Cell table from sorted keys alone (the points are already in place).
__global__ void k_table_runs(const uint32_t* __restrict__ skeys, int64_t total, uint4* __restrict__ table,
                             uint32_t mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const uint32_t key = skeys[i];
    if (i > 0 && skeys[i - 1] == key) return;
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

// ---------------------------------------------------------------------------
// Exclusive scan of 0/1 flags (stream compaction): per-tile sums, one
// workgroup scanning the tile sums, then per-tile block scans.
// ---------------------------------------------------------------------------
constexpr int kScanTile = 1024;

__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t* __restrict__ flags, int64_t n,
                                                   uint32_t* __restrict__ tile_sums) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t sum = 0;
    for (int r = 0; r < kScanTile / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) sum += flags[i];
    }
    const uint32_t incl = block_scan_256(sum, s_w);
    if (threadIdx.x == 255) tile_sums[blockIdx.x] = incl;
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t* __restrict__ tile_sums, int64_t ntiles,
                                                 uint32_t* __restrict__ total) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < ntiles; b += 256) {
        const int64_t i = b + threadIdx.x;
        const uint32_t x = i < ntiles ? tile_sums[i] : 0u;
        const uint32_t incl = block_scan_256(x, s_w);
        const uint32_t carry = s_carry;
        if (i < ntiles) tile_sums[i] = carry + incl - x;
        __syncthreads();
        if (threadIdx.x == 255) s_carry = carry + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ flags, int64_t n,
                                                   const uint32_t* __restrict__ tile_offs,
                                                   uint32_t* __restrict__ out) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = tile_offs[blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int r = 0; r < kScanTile / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const uint32_t x = i < n ? flags[i] : 0u;
        const uint32_t incl = block_scan_256(x, s_w);
        const uint32_t carry = s_carry;
        if (i < n) out[i] = carry + incl - x;
        __syncthreads();
        if (threadIdx.x == 255) s_carry = carry + incl;
        __syncthreads();
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

hipError_t launch_map_merge(const uint32_t* okeys, const float4* opts, const float4* ocov, int64_t m_old,
                            const uint32_t* nkeys, const uint32_t* nvals, const float* means, const float4* ncov,
                            int64_t m_new, uint32_t* keys, float4* pts, float4* cov, hipStream_t s) {
    if (m_old > 0)
        hipLaunchKernelGGL(k_merge_old, dim3((unsigned)ceil_div(m_old, 256)), dim3(256), 0, s, okeys, opts, ocov, m_old,
                           nkeys, m_new, keys, pts, cov);
    if (m_new > 0)
        hipLaunchKernelGGL(k_merge_new, dim3((unsigned)ceil_div(m_new, 256)), dim3(256), 0, s, nkeys, nvals, means, ncov,
                           m_new, okeys, m_old, keys, pts, cov);
    return hipGetLastError();
}

hipError_t launch_table_runs(const uint32_t* skeys, int64_t total, uint4* table, uint32_t mask, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_runs, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, skeys, total, table, mask);
    return hipGetLastError();
}

size_t flag_scan_scratch(int64_t n) { return (size_t)(ceil_div(std::max<int64_t>(n, 1), kScanTile) + 64) * 4; }

hipError_t launch_flag_scan(const uint32_t* flags, int64_t n, uint32_t* out, uint32_t* total, void* scratch,
                            hipStream_t s) {
    const int64_t ntiles = ceil_div(std::max<int64_t>(n, 1), kScanTile);
    uint32_t* tiles = static_cast<uint32_t*>(scratch);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, s, flags, n, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, tiles, ntiles, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(256), 0, s, flags, n, (const uint32_t*)tiles, out);
    return hipGetLastError();
}

}  // namespace gicp
