// Gauss-Newton iteration of G-ICP (Sec. 3, Eq. MLE_for_T):
//   k_gn_linearize : per source point, q = R x + t, the nearest map mean within
//                    r_max (exact over the map's cell grid, ties to the lower
//                    map index), Sigma = C_t + R C_s R^T, M = Sigma^-1,
//                    J = [[q]x, -I]; accumulation of the 21 unique terms of
//                    J^T M J, the 6 of J^T M d, d^T M d and the inlier count.
//                    FP32 per point; per-lane and per-wavefront sums are
//                    compensated (two-sum), the per-wave totals are summed in
//                    FP64 and written as one FP64 partial per workgroup.
//   k_gn_solve     : one workgroup; FP64 sum of the partials in a fixed order,
//                    6x6 Cholesky, xi = -H^-1 b, T <- Exp(xi) T, convergence.
// A registration runs (linearize, solve) max_it times; once the solve marks
// the state done, later launches return immediately.
#include <float.h>

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

// Knuth's two-sum: s + x = t + err exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& t, float& err) {
    t = a + b;
    const float bp = t - a;
    err = (a - (t - bp)) + (b - bp);
}

// Fixed-order sum of one column of the chunk's per-point values (kChunk
// values at stride `stride` in LDS), in the accumulation mode ACC:
//   TWOSUM: FP32 compensated summation (two-sum of every addition, the
//           compensations summed alongside), returned as s + c in FP64;
//   FP32:   plain FP32 summation;
//   FP64:   FP64 summation of the FP32 values.
// The sum is split over kSumParts consecutive lanes: lane `part` sums its
// kChunk / kSumParts rows in order, then the parts are combined pairwise
// through lane shuffles, ((p0 + p1) + (p2 + p3)); every lane of the four
// returns the same total (two-sum is exact, so its error term does not depend
// on the operand order).
constexpr int kSumParts = 4;

template <int ACC>
__device__ __forceinline__ double column_sum_split(const float* col, int stride, int part) {
    constexpr int rows = kChunk / kSumParts;
    const float* c0 = col + part * rows * stride;
    if (ACC == GICP_ACC_TWOSUM) {
        float s = 0.f, c = 0.f;
#pragma unroll
        for (int p = 0; p < rows; ++p) {
            float t, e;
            two_sum(s, c0[p * stride], t, e);
            s = t;
            c += e;
        }
#pragma unroll
        for (int o = 1; o < kSumParts; o <<= 1) {
            const float os = __shfl_xor(s, o, 64), oc = __shfl_xor(c, o, 64);
            float t, e;
            two_sum(s, os, t, e);
            s = t;
            c = (c + oc) + e;
        }
        return (double)s + (double)c;
    } else if (ACC == GICP_ACC_FP32) {
        float s = 0.f;
#pragma unroll
        for (int p = 0; p < rows; ++p) s += c0[p * stride];
#pragma unroll
        for (int o = 1; o < kSumParts; o <<= 1) s += __shfl_xor(s, o, 64);
        return (double)s;
    } else {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < rows; ++p) s += (double)c0[p * stride];
#pragma unroll
        for (int o = 1; o < kSumParts; o <<= 1) s += __shfl_xor(s, o, 64);
        return s;
    }
}

// Lanes per source point in the batched linearisation: the correspondence
// search's cells are split over them (fewer lanes keep the per-point
// arithmetic from being repeated on every lane; more shorten each point's
// chain of dependent lookups).
#ifndef GICP_LIN_GROUP
#define GICP_LIN_GROUP 2
#endif
constexpr int kLinGroup = GICP_LIN_GROUP;
// Lanes per source point in the sequential tracking launches: one frame
// leaves most of the chip idle, and a launch lasts as long as its slowest
// point's search, so four lanes split each search (measured on 68k-point
// frames: 40 us per launch against 51 us with two lanes, equal results).
constexpr int kTrackGroup = 4;
constexpr int kLinThreads = kChunk * kLinGroup;
static_assert(kLinGroup == 1 || kLinGroup == 2 || kLinGroup == 4, "lanes per point: 1, 2 or 4");
static_assert(kLinThreads >= kNumAcc * kSumParts, "the column sums take kSumParts threads per accumulated value");

// Exact 1-NN of q among the map means within the gate, searched by a group of
// G consecutive lanes (all holding the same q): lane l of the group scans
// every G-th cell (nearest cells first, skipping cells whose distance
// lower bound exceeds its best key so far or the gate), then the group takes
// the minimum (FP32 key, original index) with shuffles.  Exactness is proven
// on the group minimum from the block clearance; otherwise the next shell is
// split the same way, and after kMaxShell shells the whole map is scanned.
// Returns the sorted position of the nearest mean within the gate, or -1, on
// every lane of the group.
//
// With TRACK2 the search also bounds the second-nearest distance from below
// (the second-best key seen, the lower bounds of every pruned cell and the
// clearance of the scanned block) and returns in free_r a radius within
// which q can move without changing its nearest mean: with d1 the nearest
// and d2 that bound, |q' - q| < (d2 - d1) / 2 keeps every other mean farther
// than the nearest one (margins cover the FP32 keys and coordinates);
// free_r < 0 when there is no correspondence or no margin.
__device__ __forceinline__ float key_of(uint64_t w) { return w == kEmptyWord ? FLT_MAX : word_key(w); }

template <int G>
__device__ __forceinline__ void group_min(uint64_t& best, int32_t& pos) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const uint64_t ob = __shfl_xor(best, o, 64);
        const int32_t op = __shfl_xor(pos, o, 64);
        pos = ob < best ? op : pos;
        best = wmin(best, ob);
    }
}

// As group_min, also combining each lane's second-best word and pruned-cell
// bound (a word held by both lanes, such as the shared hint, counts once).
template <int G>
__device__ __forceinline__ void group_min2(uint64_t& best, int32_t& pos, uint64_t& sec, float& minlb) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const uint64_t ob = __shfl_xor(best, o, 64);
        const int32_t op = __shfl_xor(pos, o, 64);
        const uint64_t os = __shfl_xor(sec, o, 64);
        const float om = __shfl_xor(minlb, o, 64);
        minlb = fminf(minlb, om);
        sec = wmin(wmin(sec, os), ob == best ? kEmptyWord : wmax(best, ob));
        pos = ob < best ? op : pos;
        best = wmin(best, ob);
    }
}

// One candidate at sorted position pj with word v: the best word and its
// position, and with TRACK2 the second-best word, all without branches.
template <bool TRACK2>
__device__ __forceinline__ void take(uint64_t v, int32_t pj, uint64_t& best, int32_t& pos, uint64_t& sec) {
    pos = v < best ? pj : pos;
    if (TRACK2) sec = wmin(sec, wmax(best, v));
    best = wmin(best, v);
}

// `hint` (a map position, or -1) is a candidate evaluated first, typically the
// point's match of the previous iteration: with its key as the starting bound,
// pruning skips nearly every cell, and the search stays exact.
// Candidate loads in flight per lane in the 1-NN cell scan: eight with four
// or more lanes per point (the latency-bound single-problem launches), one
// with fewer (the batched launches, bound by instruction issue, where the
// extra registers cost occupancy: 7.9k -> 7.1k frames/s measured with eight).
template <int G>
constexpr int scan_batch() { return G >= 4 ? 8 : 1; }

template <bool TRACK2, int G = kGroup>
__device__ __forceinline__ int32_t nearest(const MapView& m, float qx, float qy, float qz, int l, int32_t hint,
                                           float* free_r = nullptr) {
    const GridView& g = m.g;
    const bool fin = finite3(qx, qy, qz);
    uint64_t best = kEmptyWord, sec = kEmptyWord;
    int32_t pos = -1;
    float minlb = FLT_MAX;
    // every lane starts from the hint (equal words are merged once by the
    // group reduction, and the lane owning the hint's cell skips it there)
    if (fin && hint >= 0 && hint < g.n) {
        const float4 p = gload(g.spts, hint);
        best = word(rank_key(qx, qy, qz, p.x, p.y, p.z), __float_as_uint(p.w));
        pos = hint;
    }
    const Cell c = cell_of(fin ? qx : 0.f, fin ? qy : 0.f, fin ? qz : 0.f, g.inv_h);
    const float slack = cell_slack(qx, qy, qz, kMaxShell, g.h);
    auto scan = [&](int cx, int cy, int cz) {
        const float bound = fminf(key_of(best), m.r_max2);
        const float lb = cell_lower_bound2(qx, qy, qz, cx, cy, cz, g.h, slack);
        if (cell_pruned(lb, bound)) {
            if (TRACK2) minlb = fminf(minlb, lb);
            return;
        }
        uint32_t start = 0;
        const uint32_t cnt = cell_lookup(g.table, g.mask, cell_key(cx, cy, cz), start);
        // the cell's candidates are loaded kB at a time before any is
        // ranked, so that a lane waits once per batch rather than once per
        // candidate (slots past the cell reload its first point and are not
        // ranked; a last batch of at most kB / 2 candidates loads kB / 2
        // slots); the (key, index) minimum does not depend on the order
        constexpr int kB = scan_batch<G>();
        auto batch = [&](uint32_t j0, auto width) __attribute__((always_inline)) {
            constexpr int W = decltype(width)::value;
            float4 pb[W];
#pragma unroll
            for (int u = 0; u < W; ++u) pb[u] = gload(g.spts, (int64_t)start + (j0 + u < cnt ? j0 + u : 0));
#pragma unroll
            for (int u = 0; u < W; ++u) {
                if (j0 + u < cnt) {
                    const int32_t pj = (int32_t)(start + j0 + u);
                    const float4 p = pb[u];
                    uint64_t v = word(rank_key(qx, qy, qz, p.x, p.y, p.z), __float_as_uint(p.w));
                    if (TRACK2) v = pj == pos ? kEmptyWord : v;   // the hint, already counted
                    take<TRACK2>(v, pj, best, pos, sec);
                }
            }
        };
        uint32_t j0 = 0;
        for (; j0 + kB / 2 < cnt; j0 += kB) batch(j0, std::integral_constant<int, kB>());
        if (kB > 1 && j0 < cnt) batch(j0, std::integral_constant<int, (kB > 1 ? kB / 2 : 1)>());
    };
    if (fin) {
        for (int j = l; j < 27; j += G) {
            int dx, dy, dz;
            block_offset(j, dx, dy, dz);
            scan(c.x + dx, c.y + dy, c.z + dz);
            // without a hint, the lanes share their best after the nearest
            // four cells, so that every lane prunes the rest with the group's
            // bound (a hint already gives every lane a tight bound)
            if (j == l && hint < 0) {
                if (TRACK2) group_min2<G>(best, pos, sec, minlb);
                else group_min<G>(best, pos);
            }
        }
    }
    if (TRACK2) group_min2<G>(best, pos, sec, minlb);
    else group_min<G>(best, pos);
    if (!fin) {
        if (free_r) *free_r = -1.f;
        return -1;
    }
    const float r_gate = m.r_max * 1.000001f + 1e-6f;
    // shells needed for the gate to end the search (the full scan below is
    // reached only when r_max exceeds kMaxGateShells cells)
    const int max_shell = min(max(kMaxShell, (int)ceilf(r_gate * g.inv_h) + 1), kMaxGateShells);
    float clr_end = FLT_MAX;   // every mean outside the scanned region is at least this far
    for (int R = 1;; ++R) {
        const float clr = block_clearance(qx, qy, qz, c, R, g.h);
        if (clr > 0.f) {
            if (clr >= r_gate) {
                clr_end = clr;
                break;
            }
            if (best != kEmptyWord) {
                const float bk = key_of(best);
                if (bk < clr * clr * (1.f - 1e-6f)) {
                    clr_end = clr;
                    break;
                }
            }
        }
        if (R >= max_shell) {
            // full scan (exact by construction), split across the group
            best = kEmptyWord;
            sec = kEmptyWord;
            pos = -1;
            minlb = FLT_MAX;
            for (int32_t j = l; j < g.n; j += G) {
                const float4 p = gload(g.spts, j);
                take<TRACK2>(word(rank_key(qx, qy, qz, p.x, p.y, p.z), __float_as_uint(p.w)), j, best, pos, sec);
            }
            if (TRACK2) group_min2<G>(best, pos, sec, minlb);
            else group_min<G>(best, pos);
            break;
        }
        const int S = R + 1;
        int idx = 0;
        for (int dz = -S; dz <= S; ++dz)
            for (int dy = -S; dy <= S; ++dy)
                for (int dx = -S; dx <= S; ++dx)
                    if (max(max(abs(dx), abs(dy)), abs(dz)) == S) {
                        if ((idx & (G - 1)) == l) scan(c.x + dx, c.y + dy, c.z + dz);
                        ++idx;
                    }
        if (TRACK2) group_min2<G>(best, pos, sec, minlb);
        else group_min<G>(best, pos);
    }
    const float bk = key_of(best);
    const int32_t res = (pos >= 0 && bk <= m.r_max2) ? pos : -1;
    if (TRACK2 && free_r) {
        float fr = -1.f;
        if (res >= 0) {
            const float k2 = fminf(fminf(key_of(sec), minlb), clr_end * clr_end);
            const float d1 = sqrtf(bk), d2 = sqrtf(k2);
            const float mag = fmaxf(fmaxf(fabsf(qx), fabsf(qy)), fabsf(qz));
            fr = 0.5f * (d2 * (1.f - 1e-5f) - d1 * (1.f + 1e-5f)) - 4e-6f * (1.f + mag);
        }
        *free_r = fr;
    }
    return res;
}

// The same search by a group of four lanes that scan cells together: in each
// round every lane takes one cell (the block's cells nearest first, then the
// shells'), tests it against the group's bound and looks it up, and the
// group then loads the round's candidates as one sequence, lane l taking
// candidates l, l + 4, l + 8, ...: the four lanes of a point read adjacent
// slots of the same cells, so that a wavefront's load touches about a
// quarter of the cache lines that four separate cell scans touch, and the
// group shares its best after every round, pruning the later cells with it.
// The result is the same exact (key, index) minimum, and the certified
// radius stays a valid bound (every mean is scanned, in a pruned cell, or
// beyond the block clearance).
template <bool TRACK2>
__device__ __forceinline__ int32_t nearest_coop4(const MapView& m, float qx, float qy, float qz, int l, int32_t hint,
                                                 float* free_r) {
    constexpr int G = 4;
    constexpr int kB = 6;
    const GridView& g = m.g;
    const bool fin = finite3(qx, qy, qz);
    const int lane0 = (int)(threadIdx.x & 63u) & ~(G - 1);
    uint64_t best = kEmptyWord, sec = kEmptyWord;
    int32_t pos = -1;
    float minlb = FLT_MAX;
    if (fin && hint >= 0 && hint < g.n) {
        const float4 p = gload(g.spts, hint);
        best = word(rank_key(qx, qy, qz, p.x, p.y, p.z), __float_as_uint(p.w));
        pos = hint;
    }
    const Cell c = cell_of(fin ? qx : 0.f, fin ? qy : 0.f, fin ? qz : 0.f, g.inv_h);
    const float slack = cell_slack(qx, qy, qz, kMaxShell, g.h);
    // one round: this lane's cell (when `own`), then the group's candidates
    auto round = [&](bool own, int cx, int cy, int cz) __attribute__((always_inline)) {
        uint32_t st = 0, cnt = 0;
        if (own) {
            const float lb = cell_lower_bound2(qx, qy, qz, cx, cy, cz, g.h, slack);
            if (cell_pruned(lb, fminf(key_of(best), m.r_max2))) {
                if (TRACK2) minlb = fminf(minlb, lb);
            } else {
                cnt = cell_lookup(g.table, g.mask, cell_key(cx, cy, cz), st);
            }
        }
        const uint32_t c0 = (uint32_t)__shfl((int)cnt, lane0, 64), c1 = (uint32_t)__shfl((int)cnt, lane0 + 1, 64);
        const uint32_t c2 = (uint32_t)__shfl((int)cnt, lane0 + 2, 64), c3 = (uint32_t)__shfl((int)cnt, lane0 + 3, 64);
        const uint32_t p1 = c0, p2 = p1 + c1, p3 = p2 + c2, total = p3 + c3;
        if (total) {
            // candidate t of the round sits at sorted position t + b(t), b the
            // offset of the cell holding it
            const uint32_t b0 = (uint32_t)__shfl((int)st, lane0, 64);
            const uint32_t b1 = (uint32_t)__shfl((int)st, lane0 + 1, 64) - p1;
            const uint32_t b2 = (uint32_t)__shfl((int)st, lane0 + 2, 64) - p2;
            const uint32_t b3 = (uint32_t)__shfl((int)st, lane0 + 3, 64) - p3;
            // (selects: the empty asm keeps the compiler from turning the
            // chain into an indexed load from a stack copy of b0..b3)
            auto at = [&](uint32_t t) __attribute__((always_inline)) {
                uint32_t x1 = b1, x2 = b2, x3 = b3;
                asm("" : "+v"(x1), "+v"(x2), "+v"(x3));
                uint32_t b = t >= p1 ? x1 : b0;
                b = t >= p2 ? x2 : b;
                b = t >= p3 ? x3 : b;
                return (int32_t)(t + b);
            };
            const int32_t first = at(0u);
            for (uint32_t t0 = 0; t0 < total; t0 += G * kB) {
                float4 pb[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const uint32_t t = t0 + (uint32_t)(l + G * u);
                    pb[u] = gload(g.spts, (int64_t)(t < total ? at(t) : first));
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const uint32_t t = t0 + (uint32_t)(l + G * u);
                    if (t < total) {
                        const int32_t pj = at(t);
                        uint64_t v = word(rank_key(qx, qy, qz, pb[u].x, pb[u].y, pb[u].z), __float_as_uint(pb[u].w));
                        if (TRACK2) v = pj == pos ? kEmptyWord : v;   // the hint, already counted
                        take<TRACK2>(v, pj, best, pos, sec);
                    }
                }
            }
        }
        if (TRACK2) group_min2<G>(best, pos, sec, minlb);
        else group_min<G>(best, pos);
    };
    if (fin) {
        for (int j0 = 0; j0 < 27; j0 += G) {
            const int j = j0 + l;
            int dx = 0, dy = 0, dz = 0;
            if (j < 27) block_offset(j, dx, dy, dz);
            round(j < 27, c.x + dx, c.y + dy, c.z + dz);
        }
    }
    if (!fin) {
        if (free_r) *free_r = -1.f;
        return -1;
    }
    const float r_gate = m.r_max * 1.000001f + 1e-6f;
    const int max_shell = min(max(kMaxShell, (int)ceilf(r_gate * g.inv_h) + 1), kMaxGateShells);
    float clr_end = FLT_MAX;
    for (int R = 1;; ++R) {
        const float clr = block_clearance(qx, qy, qz, c, R, g.h);
        if (clr > 0.f) {
            if (clr >= r_gate) {
                clr_end = clr;
                break;
            }
            if (best != kEmptyWord) {
                const float bk = key_of(best);
                if (bk < clr * clr * (1.f - 1e-6f)) {
                    clr_end = clr;
                    break;
                }
            }
        }
        if (R >= max_shell) {
            best = kEmptyWord;
            sec = kEmptyWord;
            pos = -1;
            minlb = FLT_MAX;
            for (int32_t jj = l; jj < g.n; jj += G) {
                const float4 p = gload(g.spts, jj);
                take<TRACK2>(word(rank_key(qx, qy, qz, p.x, p.y, p.z), __float_as_uint(p.w)), jj, best, pos, sec);
            }
            if (TRACK2) group_min2<G>(best, pos, sec, minlb);
            else group_min<G>(best, pos);
            break;
        }
        // the shell's cells in rounds of four, lane l taking the l-th of each
        // (the walk over the box is the same in the four lanes)
        const int S = R + 1;
        int k = 0, pdx = 0, pdy = 0, pdz = 0;
        for (int dz = -S; dz <= S; ++dz)
            for (int dy = -S; dy <= S; ++dy)
                for (int dx = -S; dx <= S; ++dx)
                    if (max(max(abs(dx), abs(dy)), abs(dz)) == S) {
                        if ((k & (G - 1)) == l) {
                            pdx = dx;
                            pdy = dy;
                            pdz = dz;
                        }
                        if ((k & (G - 1)) == G - 1) round(true, c.x + pdx, c.y + pdy, c.z + pdz);
                        ++k;
                    }
        if (k & (G - 1)) round((k & (G - 1)) > l, c.x + pdx, c.y + pdy, c.z + pdz);
    }
    const float bk = key_of(best);
    const int32_t res = (pos >= 0 && bk <= m.r_max2) ? pos : -1;
    if (TRACK2 && free_r) {
        float fr = -1.f;
        if (res >= 0) {
            const float k2 = fminf(fminf(key_of(sec), minlb), clr_end * clr_end);
            const float d1 = sqrtf(bk), d2 = sqrtf(k2);
            const float mag = fmaxf(fmaxf(fabsf(qx), fabsf(qy)), fabsf(qz));
            fr = 0.5f * (d2 * (1.f - 1e-5f) - d1 * (1.f + 1e-5f)) - 4e-6f * (1.f + mag);
        }
        *free_r = fr;
    }
    return res;
}

// Hand-over of values between workgroups of one launch without cache
// write-back.  An agent-scope fence writes back the whole L2 of the XCD
// (measured: a launch of 1,057 workgroups that each fence before a counter
// update takes 110 us against 44 us without), so the values handed over are
// written and read with agent-scope (device-coherent) atomic accesses, and the
// hand-over only orders them: the writer waits for its stores to complete
// before the counter update, and the reader's loads are not moved above the
// counter update.
__device__ __forceinline__ void store_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_dev(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt with vmcnt = 0 and the other counters left alone (gfx9 encoding)
constexpr int kWaitVm0 = (0x7 << 4) | (0xf << 8);
__device__ __forceinline__ void handover_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
}
__device__ __forceinline__ void handover_acquire() {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A value written (read) by one workgroup for others of the same launch:
// device-coherent when DEV, plain otherwise.
template <bool DEV, typename T>
__device__ __forceinline__ void sput(T* p, T v) {
    if (DEV) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool DEV, typename T>
__device__ __forceinline__ T sget(const T* p) {
    if (DEV) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
// A float4 as two device-coherent 8-byte words.
__device__ __forceinline__ float4 load4_dev(const float4* p) {
    const uint64_t* q = (const uint64_t*)p;
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float4 r;
    __builtin_memcpy(&r.x, &a, 8);
    __builtin_memcpy(&r.z, &b, 8);
    return r;
}
__device__ __forceinline__ void store4_dev(float4* p, float4 v) {
    uint64_t a, b;
    __builtin_memcpy(&a, &v.x, 8);
    __builtin_memcpy(&b, &v.z, 8);
    uint64_t* q = (uint64_t*)p;
    __hip_atomic_store(q, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The linearisation of one source point, in three parts that chunk_linearize
// runs on different lanes: the query point q = R x + t; the correspondence
// (kept from the previous iteration, or searched by a group of G lanes); and
// the terms.  On success point_terms leaves in v[0..29) the point's 21 unique
// terms of J^T M J, the 6 of J^T M d, d^T M d and 1 (the inlier count); it
// returns false (v untouched) when the point has no correspondence within
// r_max or a singular combined covariance.  Point i of the problem's
// processing order: the grid-cell order when the problem carries its sorted
// source (ssrc, sscov), else the caller's order.
__device__ __forceinline__ void point_query(const ProbDev& P, int64_t i, const float* R, const float* t, float& qx,
                                            float& qy, float& qz) {
    float x, y, z;
    if (P.ssrc) {
        const float4 p4 = gload(P.ssrc, i);
        x = p4.x;
        y = p4.y;
        z = p4.z;
    } else {
        x = gload(P.src, i);
        y = gload(P.src, P.n + i);
        z = gload(P.src, 2 * P.n + i);
    }
    qx = R[0] * x + R[1] * y + R[2] * z + t[0];
    qy = R[3] * x + R[4] * y + R[5] * z + t[1];
    qz = R[6] * x + R[7] * y + R[8] * z + t[2];
}

// The previous iteration's match of point i stands while q stays within the
// radius its search certified (the nearest mean cannot have changed): the
// match (reuse), or the search's starting candidate (hint, -1 for none).
template <bool COH>
__device__ __forceinline__ bool point_reuse(const ProbDev& P, int64_t i, float qx, float qy, float qz,
                                            int32_t& hint) {
    hint = P.fresh ? -1 : (COH ? sget<true>(P.nn_prev + i) : gload((const int32_t*)P.nn_prev, i));
    if (hint < 0) return false;
    const float4 cq = COH ? load4_dev(P.nn_cache + i) : gload((const float4*)P.nn_cache, i);
    const float ex = qx - cq.x, ey = qy - cq.y, ez = qz - cq.z;
    return sqrtf(ex * ex + ey * ey + ez * ez) < cq.w;
}

// The terms of point i (query q at the pose R) against the map Gaussian at
// sorted position pos; the gate is tested here (a kept match may have left
// it; a searched one passes by construction).
__device__ __forceinline__ bool point_terms(const ProbDev& P, int64_t i, const float* R, float qx, float qy,
                                            float qz, int32_t pos, float* v) {
    if (pos < 0) return false;
    const int64_t n = P.n;
    const float* cv = P.ssrc ? P.sscov : P.scov;
    const MapView& map = P.map;
    const float4 mu = gload(map.g.spts, pos);
    const float4 ca = gload(map.scov, 2 * (int64_t)pos);
    const float4 cb = gload(map.scov, 2 * (int64_t)pos + 1);
    const float c00 = gload(cv, i), c01 = gload(cv, n + i), c02 = gload(cv, 2 * n + i);
    const float c11 = gload(cv, 3 * n + i), c12 = gload(cv, 4 * n + i), c22 = gload(cv, 5 * n + i);
    if (!(rank_key(qx, qy, qz, mu.x, mu.y, mu.z) <= map.r_max2)) return false;
    // source covariance rotated: A = R Cs, S = A R^T
    const float a00 = R[0] * c00 + R[1] * c01 + R[2] * c02;
    const float a01 = R[0] * c01 + R[1] * c11 + R[2] * c12;
    const float a02 = R[0] * c02 + R[1] * c12 + R[2] * c22;
    const float a10 = R[3] * c00 + R[4] * c01 + R[5] * c02;
    const float a11 = R[3] * c01 + R[4] * c11 + R[5] * c12;
    const float a12 = R[3] * c02 + R[4] * c12 + R[5] * c22;
    const float a20 = R[6] * c00 + R[7] * c01 + R[8] * c02;
    const float a21 = R[6] * c01 + R[7] * c11 + R[8] * c12;
    const float a22 = R[6] * c02 + R[7] * c12 + R[8] * c22;
    const float s00 = ca.x + a00 * R[0] + a01 * R[1] + a02 * R[2];
    const float s01 = ca.y + a00 * R[3] + a01 * R[4] + a02 * R[5];
    const float s02 = ca.z + a00 * R[6] + a01 * R[7] + a02 * R[8];
    const float s11 = ca.w + a10 * R[3] + a11 * R[4] + a12 * R[5];
    const float s12 = cb.x + a10 * R[6] + a11 * R[7] + a12 * R[8];
    const float s22 = cb.y + a20 * R[6] + a21 * R[7] + a22 * R[8];
    // M = Sigma^-1 by cofactors
    const float k00 = s11 * s22 - s12 * s12;
    const float k01 = s02 * s12 - s01 * s22;
    const float k02 = s01 * s12 - s02 * s11;
    const float det = s00 * k00 + s01 * k01 + s02 * k02;
    if (!(det > 0.f)) return false;
    const float id = 1.f / det;
    const float m00 = k00 * id, m01 = k01 * id, m02 = k02 * id;
    const float m11 = (s00 * s22 - s02 * s02) * id;
    const float m12 = (s01 * s02 - s00 * s12) * id;
    const float m22 = (s00 * s11 - s01 * s01) * id;
    // residual
    const float dx = mu.x - qx, dy = mu.y - qy, dz = mu.z - qz;
    const float md0 = m00 * dx + m01 * dy + m02 * dz;
    const float md1 = m01 * dx + m11 * dy + m12 * dz;
    const float md2 = m02 * dx + m12 * dy + m22 * dz;
    // B = M [q]x, [q]x = [[0,-qz,qy],[qz,0,-qx],[-qy,qx,0]]
    const float b00 = m01 * qz - m02 * qy, b01 = m02 * qx - m00 * qz, b02 = m00 * qy - m01 * qx;
    const float b10 = m11 * qz - m12 * qy, b11 = m12 * qx - m01 * qz, b12 = m01 * qy - m11 * qx;
    const float b20 = m12 * qz - m22 * qy, b21 = m22 * qx - m02 * qz, b22 = m02 * qy - m12 * qx;
    // H_ww = [q]x^T B: row i of [q]x^T is column i of [q]x
    // column 0 of [q]x = (0, qz, -qy); column 1 = (-qz, 0, qx); column 2 = (qy, -qx, 0)
    const float h00 = qz * b10 - qy * b20;
    const float h01 = qz * b11 - qy * b21;
    const float h02 = qz * b12 - qy * b22;
    const float h11 = -qz * b01 + qx * b21;
    const float h12 = -qz * b02 + qx * b22;
    const float h22 = qy * b02 - qx * b12;
    // H_wv = -B^T, H_vv = M
    v[0] = h00; v[1] = h01; v[2] = h02;
    v[3] = -b00; v[4] = -b10; v[5] = -b20;
    v[6] = h11; v[7] = h12;
    v[8] = -b01; v[9] = -b11; v[10] = -b21;
    v[11] = h22;
    v[12] = -b02; v[13] = -b12; v[14] = -b22;
    v[15] = m00; v[16] = m01; v[17] = m02;
    v[18] = m11; v[19] = m12;
    v[20] = m22;
    // b = [ [q]x^T M d ; -M d ],  [q]x^T v = v x q
    v[21] = md1 * qz - md2 * qy;
    v[22] = md2 * qx - md0 * qz;
    v[23] = md0 * qy - md1 * qx;
    v[24] = -md0; v[25] = -md1; v[26] = -md2;
    v[27] = dx * md0 + dy * md1 + dz * md2;
    v[28] = 1.f;
    return true;
}


// One work item: the kChunk points [c*kChunk, (c+1)*kChunk) of a cloud, in
// a workgroup of kChunk x G threads.  One lane per point finds q and whether
// its match stands; the points that must search are packed, G lanes each,
// into the first groups (a wavefront whose points all keep their matches
// then runs no search code); one lane per point computes the terms into the
// point's LDS row (zeros when it is not an inlier), so the per-point
// arithmetic runs once per point, not once per lane; threads 0..28 then sum
// one column each over the 64 rows in a fixed order, and write the chunk's FP64 partial
// (with DEV device-coherently, completed before the closing barrier, for a
// hand-over within the launch; with COH also the points' reuse state, for
// a launch in which another workgroup may take the chunk's next iteration).
// The listed points' searches, GS lanes each (groups of GS consecutive
// threads; the groups beyond the list idle): each stores its point's match
// and certified radius (the reuse state) and the match in s_pos.
template <int GS, bool COH>
__device__ __forceinline__ void search_listed(const ProbDev& P, int64_t c, int ns, const int32_t* s_list,
                                              const int32_t* s_hint, const float (*s_q)[3], int32_t* s_pos) {
    const int tid = threadIdx.x;
    const int grp = tid / GS, l = tid & (GS - 1);
    if (grp >= ns) return;
    const int pt = s_list[grp];
    const int64_t i = c * kChunk + pt;
    const float qx = s_q[pt][0], qy = s_q[pt][1], qz = s_q[pt][2];
    float free_r;
    int32_t pos;
    if constexpr (GS == 4 && !COH) pos = nearest_coop4<true>(P.map, qx, qy, qz, l, s_hint[pt], &free_r);
    else pos = nearest<true, GS>(P.map, qx, qy, qz, l, s_hint[pt], &free_r);
    if (l == 0) {
        if (COH) {
            sput<true>(P.nn_prev + i, pos);
            store4_dev(P.nn_cache + i, make_float4(qx, qy, qz, free_r));
        } else {
            gstore(P.nn_prev, i, pos);
            gstore(P.nn_cache, i, make_float4(qx, qy, qz, free_r));
        }
        s_pos[pt] = pos;
    }
}

template <int ACC, int G = kGroup, bool DEV = false, bool COH = false>
__device__ __forceinline__ void chunk_linearize(const ProbDev& P, int64_t c, const float* R, const float* t,
                                                double* __restrict__ out) {
    static_assert(kChunk == 64, "one wavefront holds a work item's points");
    __shared__ float s_val[kChunk][kNumAcc + 1];
    __shared__ float s_q[kChunk][3];
    __shared__ int32_t s_pos[kChunk];
    __shared__ int32_t s_hint[kChunk];
    __shared__ int32_t s_list[kChunk];
    __shared__ int32_t s_nsearch;
    const int tid = threadIdx.x;
    // 1. one lane per point (the first wavefront): q, and whether the
    //    previous match stands; the points that must search are listed in
    //    point order
    if (tid < kChunk) {
        const int pt = tid;
        const int64_t i = c * kChunk + pt;
        int32_t pos = -1;
        bool need = false;
        if (i < P.n) {
            float qx, qy, qz;
            point_query(P, i, R, t, qx, qy, qz);
            s_q[pt][0] = qx;
            s_q[pt][1] = qy;
            s_q[pt][2] = qz;
            int32_t hint;
            if (point_reuse<COH>(P, i, qx, qy, qz, hint)) {
                pos = hint;
            } else {
                need = true;
                s_hint[pt] = hint;
            }
        }
        s_pos[pt] = pos;
        const uint64_t m = __ballot(need);
        if (need) s_list[__popcll(m & ((1ull << pt) - 1ull))] = pt;
        if (pt == 0) s_nsearch = (int32_t)__popcll(m);
    }
    __syncthreads();
    // 2. the searches, packed into the first groups, so that only the
    //    wavefronts holding them run search code; when few points search,
    //    each gets more lanes (a work item lasts as long as its slowest
    //    search: in iterations where most matches stand, the few searching
    //    points are the critical path)
    {
        // (four-lane launches only: they are latency-bound; the two-lane
        // ones are issue-bound, and the wider searches' registers would cost
        // them occupancy, as they would the work queue)
        constexpr int NT = kChunk * G;
        constexpr bool kWiden = G == 4 && !COH;
        const int ns = s_nsearch;
        if (ns > 0) {
            if (kWiden && ns * 16 <= NT) search_listed<kWiden ? 16 : G, COH>(P, c, ns, s_list, s_hint, s_q, s_pos);
            else if (kWiden && ns * 8 <= NT) search_listed<kWiden ? 8 : G, COH>(P, c, ns, s_list, s_hint, s_q, s_pos);
            else search_listed<G, COH>(P, c, ns, s_list, s_hint, s_q, s_pos);
        }
    }
    __syncthreads();
    // 3. one lane per point: the terms, stored as the point's LDS row (zeros
    //    when it is not an inlier)
    if (tid < kChunk) {
        const int pt = tid;
        const int64_t i = c * kChunk + pt;
        float v[kNumAcc];
        bool ok = false;
        if (i < P.n) ok = point_terms(P, i, R, s_q[pt][0], s_q[pt][1], s_q[pt][2], s_pos[pt], v);
#pragma unroll
        for (int j = 0; j < kNumAcc; ++j) s_val[pt][j] = ok ? v[j] : 0.f;
    }
    if (COH) handover_release();
    __syncthreads();
    if (threadIdx.x < kNumAcc * kSumParts) {
        const int col = threadIdx.x / kSumParts, part = threadIdx.x % kSumParts;
        const double r = column_sum_split<ACC>(&s_val[0][col], kNumAcc + 1, part);
        if (part == 0) {
            if (DEV) {
                store_dev(&out[col], r);
                handover_release();
            } else {
                out[col] = r;
            }
        }
    }
    __syncthreads();
}

template <int ACC>
__global__ __launch_bounds__(kBlock) void k_gn_linearize(ProbDev P, double* __restrict__ partials) {
    const RegState* st = P.st;
    if (st->done) return;
    float R[9], t[3];
#pragma unroll
    for (int j = 0; j < 9; ++j) R[j] = st->Rf[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) t[j] = st->tf[j];
    chunk_linearize<ACC>(P, blockIdx.x, R, t, partials + (int64_t)blockIdx.x * kNumAcc);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// FP64 solve and update.
// ---------------------------------------------------------------------------
// 1 / sqrt(s) for s > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - s y^2) / 2 (each roughly doubles the correct bits), in
// place of a square root and a division on the solve's single thread; tiny
// arguments, outside the estimate's normal range, take the plain division.
__device__ __forceinline__ double rsqrt_pos(double s) {
    if (!(s > 1e-280)) return 1.0 / sqrt(s);
    double y = __builtin_amdgcn_rsq(s);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-(s * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// The coefficients of the closed-form SE(3) exponential, A = sin(th)/th,
// B = (1 - cos th)/th^2, C = (th - sin th)/th^3, are even power series in
// th: below th = 0.25 their terms up to th^12 reach double precision (the
// first omitted term is below 3e-21 of the sum), with no sine, cosine or
// division on the solve's single thread; above, the closed forms.
constexpr double kExpSeriesMax2 = 0.0625;

__device__ __forceinline__ void exp_se3(const double xi[6], double T[16]) {
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double th2 = wx * wx + wy * wy + wz * wz;
    double A, B, C;
    if (th2 < kExpSeriesMax2) {
        // Horner in th^2 with the coefficients (-1)^k / (2k+1)!, (-1)^k / (2k+2)!, (-1)^k / (2k+3)!
        A = 1.0 + th2 * (-1.0 / 6.0 + th2 * (1.0 / 120.0 + th2 * (-1.0 / 5040.0 + th2 * (1.0 / 362880.0 +
            th2 * (-1.0 / 39916800.0 + th2 * (1.0 / 6227020800.0))))));
        B = 0.5 + th2 * (-1.0 / 24.0 + th2 * (1.0 / 720.0 + th2 * (-1.0 / 40320.0 + th2 * (1.0 / 3628800.0 +
            th2 * (-1.0 / 479001600.0 + th2 * (1.0 / 87178291200.0))))));
        C = 1.0 / 6.0 + th2 * (-1.0 / 120.0 + th2 * (1.0 / 5040.0 + th2 * (-1.0 / 362880.0 + th2 * (1.0 / 39916800.0 +
            th2 * (-1.0 / 6227020800.0 + th2 * (1.0 / 1307674368000.0))))));
    } else {
        const double th = sqrt(th2);
        const double sn = sin(th), cs = cos(th);
        A = sn / th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / (th2 * th);
    }
    const double W[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            const double id = (i == j) ? 1.0 : 0.0;
            T[4 * i + j] = id + A * W[3 * i + j] + B * W2[3 * i + j];
        }
        double v = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double id = (i == j) ? 1.0 : 0.0;
            v += (id + B * W[3 * i + j] + C * W2[3 * i + j]) * xi[3 + j];
        }
        T[4 * i + 3] = v;
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

}  // namespace

// The state fields the update reads, fetched by the reducing threads while
// their partials are in flight (the state was last written on another
// compute unit: fetched inside the update they would cost two more round
// trips on its single thread), one 8-byte word per thread: pose[16],
// conv_rot, conv_trans, and the word holding iters and max_it.
constexpr int kPreFields = 19;
static_assert(offsetof(RegState, conv_rot) % 8 == 0 && offsetof(RegState, conv_trans) % 8 == 0 &&
                  offsetof(RegState, iters) % 8 == 0 && offsetof(RegState, max_it) == offsetof(RegState, iters) + 4,
              "prefetched state words");

__device__ __forceinline__ int pre_word(int t) {
    return t < 16 ? t
                  : (t == 16 ? (int)(offsetof(RegState, conv_rot) / 8)
                             : (t == 17 ? (int)(offsetof(RegState, conv_trans) / 8) : (int)(offsetof(RegState, iters) / 8)));
}

// The results of one update, in LDS: the new pose itself is left in the
// workspace (H[0..16)) when `moved`.
struct SolveOut {
    int32_t iters, status, done, converged, moved;
};

// Thread-0 part of the solve: v holds the 29 reduced sums, pre the words
// above; H and L live in LDS (workspace of 72 doubles).  Computes only: the
// results go to `o` and H[0..16), and solve_publish stores them.
__device__ __forceinline__ void solve_update_inl(const double* v, const double* pre, double* H, double* L,
                                                 SolveOut* o) {
    int32_t im[2];
    __builtin_memcpy(im, &pre[18], 8);
    const int32_t iters = im[0] + 1;
    const int32_t max_it = im[1];
    const double conv_rot = pre[16], conv_trans = pre[17];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            H[6 * i + j] = v[q];
            H[6 * j + i] = v[q];
            ++q;
        }
    o->iters = iters;
    o->status = 0;
    o->done = 0;
    o->converged = 0;
    o->moved = 0;
    if (v[28] < 6.0) {
        o->status = GICP_E_NO_CORR;
        o->done = 1;
        return;
    }
    // Cholesky H = L L^T; a pivot not above 1e-12 * max(diag H) fails.  The
    // factor lives in registers (every index below is fixed after unrolling;
    // H stays in LDS, read off the dependency chain) and each column is
    // scaled by one reciprocal of its pivot.
    double Lr[36], inv[6];
#pragma unroll
    for (int i = 0; i < 36; ++i) Lr[i] = 0.0;
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) dmax = fmax(dmax, H[7 * i]);
    const double floor_ = 1e-12 * dmax;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = H[7 * j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= Lr[6 * j + k] * Lr[6 * j + k];
        if (!(s > floor_) || !isfinite(s)) {
            o->status = GICP_E_DEGENERATE;
            o->done = 1;
            return;
        }
        inv[j] = rsqrt_pos(s);   // the pivot L_jj itself is never needed, only its reciprocal
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double r = H[6 * i + j];
#pragma unroll
            for (int k = 0; k < j; ++k) r -= Lr[6 * i + k] * Lr[6 * j + k];
            Lr[6 * i + j] = r * inv[j];
        }
    }
    double y[6], xi[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double r = v[21 + i];
#pragma unroll
        for (int k = 0; k < i; ++k) r -= Lr[6 * i + k] * y[k];
        y[i] = r * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double r = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) r -= Lr[6 * k + i] * xi[k];
        xi[i] = r * inv[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) xi[i] = -xi[i];
    // T <- Exp(xi) T, with Exp in L[0..16) and the product in H[0..16) (both free now)
    double P[16];   // the current pose
#pragma unroll
    for (int i = 0; i < 16; ++i) P[i] = pre[i];
    double* E = L;
    double* T = H;
    exp_se3(xi, E);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) s += E[4 * i + k] * P[4 * k + j];
            T[4 * i + j] = s;
        }
    o->moved = 1;
    const double nw = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    const double nv = sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]);
    if (nw < conv_rot && nv < conv_trans) {
        o->converged = 1;
        o->done = 1;
    } else if (iters >= max_it) {
        o->done = 1;
    }
}

// The update's stores, spread over the workgroup's threads (called by every
// thread; at least 64): the new pose (and its FP32 copy) when it moved; when
// the registration ends, the last linearisation's H, b, cost and inliers
// (the values a caller reads, written once); iterations and flags.
template <bool DEV>
__device__ __forceinline__ void solve_publish(const SolveOut& o, const double* T, const double* v, RegState* st,
                                              int t) {
    if (o.moved) {
        if (t < 16) {
            sput<DEV>(&st->pose[t], T[t]);
        } else if (t < 25) {
            const int k = t - 16;
            sput<DEV>(&st->Rf[k], (float)T[4 * (k / 3) + k % 3]);
        } else if (t < 28) {
            const int k = t - 25;
            sput<DEV>(&st->tf[k], (float)T[4 * k + 3]);
        }
    }
    if (o.done && t >= 32 && t < 32 + kNumAcc) {
        const int j = t - 32;
        if (j < 21) sput<DEV>(&st->H[j], v[j]);
        else if (j < 27) sput<DEV>(&st->b[j - 21], v[j]);
        else if (j == 27) sput<DEV>(&st->cost, v[27]);
        else sput<DEV>(&st->n_inl, v[28]);
    }
    if (t == 63) {
        sput<DEV>(&st->iters, o.iters);
        if (o.status) sput<DEV>(&st->status, o.status);
        if (o.converged) sput<DEV>(&st->converged, 1);
        if (o.done) sput<DEV>(&st->done, 1);
    }
    if (DEV) handover_release();
}

// The update as a call, for the work queue: its registers then do not add
// to the queue kernel's.
__device__ __noinline__ void solve_update_call(const double* v, const double* pre, double* H, double* L, SolveOut* o) {
    solve_update_inl(v, pre, H, L, o);
}

namespace {

constexpr int kSolveThreads = 512;
constexpr int kSolveParts = 32;

}  // namespace

// Reduction of `nparts` FP64 partials (29 values each) in a fixed order, then
// (thread 0) the 6x6 Cholesky solve, the SE(3) update and the convergence
// test.  Called by all NT threads of one workgroup.
//
// The order: task (p, j), p < kSolveParts, sums value j of the partials p,
// p + 32, p + 64, ... in that order; then value j is the sum of the tasks'
// results in order of p.  Task q = p * 29 + j reads partials[q + 928 m] for
// m = 0, 1, ..., so the consecutive tasks of a wavefront read one contiguous
// span per load instruction.  A thread takes its tasks two at a time and
// issues KU loads for each before adding any: the partials come from other
// compute units' caches, so the rounds of loads set the time.  Both the FP32
// and the FP64 sums are formed (no branch on the accumulation mode ahead of
// the loads) and the mode picks one.  The result does not depend on NT or KU.
template <int NT, int KU, bool DEV = false>
__device__ __forceinline__ void solve_state(const double* __restrict__ partials, int nparts,
                                            RegState* __restrict__ st) {
    static_assert(NT >= kPreFields && NT >= kNumAcc && NT >= 64, "solve block size");
    __shared__ double s_part[kNumAcc][kSolveParts];
    __shared__ double s_v[kNumAcc];
    __shared__ double s_pre[kPreFields];
    __shared__ double s_HL[72];
    constexpr int kTasks = kNumAcc * kSolveParts;
    const int t = threadIdx.x;
    // the update's state words (loaded now, stored to LDS after the loop)
    const double pre =
        t < kPreFields ? (DEV ? sget<true>((const double*)st + pre_word(t)) : gload((const double*)st, pre_word(t)))
                       : 0.0;
    const int acc = gload(&st->acc, 0);
    for (int qa = t; qa < kTasks; qa += 2 * NT) {
        const int qb = qa + NT;
        const bool hb = qb < kTasks;
        const int pa = qa / kNumAcc, pb = hb ? qb / kNumAcc : pa;   // pb >= pa
        double va = 0.0, vb = 0.0;
        float fa = 0.f, fb = 0.f;
        for (int m0 = 0; pa + kSolveParts * m0 < nparts; m0 += KU) {
            double xa[KU], xb[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int64_t m = m0 + u;
                xa[u] = pa + kSolveParts * m < nparts ? (DEV ? load_dev(partials + qa + kTasks * m)
                                                             : gload(partials, qa + kTasks * m))
                                                      : 0.0;
                xb[u] = hb && pb + kSolveParts * m < nparts ? (DEV ? load_dev(partials + qb + kTasks * m)
                                                                   : gload(partials, qb + kTasks * m))
                                                            : 0.0;
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                if (pa + kSolveParts * (m0 + u) < nparts) {
                    fa += (float)xa[u];
                    va += xa[u];
                }
                if (hb && pb + kSolveParts * (m0 + u) < nparts) {
                    fb += (float)xb[u];
                    vb += xb[u];
                }
            }
        }
        s_part[qa % kNumAcc][pa] = acc == GICP_ACC_FP32 ? (double)fa : va;
        if (hb) s_part[qb % kNumAcc][pb] = acc == GICP_ACC_FP32 ? (double)fb : vb;
    }
    if (t < kPreFields) s_pre[t] = pre;
    __syncthreads();
    if (t < kNumAcc) {
        if (acc == GICP_ACC_FP32) {
            float f = 0.f;
            for (int p = 0; p < kSolveParts; ++p) f += (float)s_part[t][p];
            s_v[t] = (double)f;
        } else {
            double s = 0.0;
            for (int p = 0; p < kSolveParts; ++p) s += s_part[t][p];
            s_v[t] = s;
        }
    }
    __syncthreads();
    __shared__ SolveOut s_out;
    if (t == 0) {
        if (DEV) solve_update_call(s_v, s_pre, s_HL, s_HL + 36, &s_out);
        else solve_update_inl(s_v, s_pre, s_HL, s_HL + 36, &s_out);
    }
    __syncthreads();
    solve_publish<DEV>(s_out, s_HL, s_v, st, t);
    __syncthreads();
}

// The solve kernels' form: kSolveThreads threads, 20 loads in flight per task.
__device__ __forceinline__ void solve_block(const double* __restrict__ partials, int nparts,
                                            RegState* __restrict__ st) {
    solve_state<kSolveThreads, 20>(partials, nparts, st);
}

namespace {

__global__ __launch_bounds__(kSolveThreads) void k_gn_solve(const double* __restrict__ partials, int nblocks,
                                                            RegState* __restrict__ st) {
    if (st->done) return;
    solve_block(partials, nblocks, st);
}

// ---------------------------------------------------------------------------
// Persistent work queue over (problem, chunk) items.  Workers pop items in
// ticket order; an item is one chunk of kChunk source points of one problem at
// the problem's current pose.  The worker that completes the last chunk of a
// problem's iteration reduces that iteration's partials (fixed slots, fixed
// order: results do not depend on scheduling), solves, updates the pose and
// either pushes the problem's chunks for the next iteration or retires the
// problem.  Workers leave when every problem is retired.  Every wait is bounded
// (kSpinLimit sleeps) and sets the queue's error word when exhausted.
// ---------------------------------------------------------------------------
constexpr long long kSpinLimit = 1ll << 24;

// A value equal on every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// (registers bounded so that five workgroups fit on a CU)
template <int ACC, int G>
__global__ __launch_bounds__(kChunk * G) __attribute__((amdgpu_waves_per_eu(5))) void k_gn_queue(const ProbDev* __restrict__ probs, QueueDev* __restrict__ q,
                                                     uint32_t* __restrict__ items, uint32_t* __restrict__ arrive,
                                                     double* __restrict__ partials) {
    __shared__ uint32_t s_item;
    __shared__ int s_last;
    __shared__ uint32_t s_base;
    const uint32_t cap = q->cap;
    while (true) {
        if (threadIdx.x == 0) {
            const uint32_t tk = atomicAdd(&q->head, 1u);
            uint32_t it = 0;
            long long spins = 0;
            while (true) {
                if (tk < cap) it = load_agent(&items[tk]);
                if (it != 0u) break;
                if (load_agent(&q->remaining) == 0u || tk >= cap) break;
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) {
                    atomicOr(&q->error, 1u);
                    break;
                }
            }
            s_item = it;
        }
        __syncthreads();
        const uint32_t item = s_item;
        if (item == 0u) return;
        // the problem's state as of the push of this item: written by
        // another workgroup of this launch, read device-coherently (the
        // hand-overs below order, rather than fence, the values they pass:
        // an agent-scope fence would write back this XCD's whole L2 for
        // every item)
        handover_acquire();
        const uint32_t p = (item - 1u) >> kChunkBits, c = (item - 1u) & ((1u << kChunkBits) - 1u);
        const ProbDev P = probs[p];
        RegState* st = P.st;
        float R[9], t[3];
#pragma unroll
        for (int j = 0; j < 9; ++j) R[j] = uniform(sget<true>(&st->Rf[j]));
#pragma unroll
        for (int j = 0; j < 3; ++j) t[j] = uniform(sget<true>(&st->tf[j]));
        chunk_linearize<ACC, G, true, true>(P, c, R, t, partials + ((int64_t)P.part0 + c) * kNumAcc);
        if (threadIdx.x == 0) s_last = (atomicAdd(&arrive[p], 1u) == (uint32_t)P.nchunks - 1u) ? 1 : 0;
        __syncthreads();
        if (s_last) {
            handover_acquire();
            // (few loads in flight: this kernel's register budget is the linearisation's)
            solve_state<kChunk * G, 4, true>(partials + (int64_t)P.part0 * kNumAcc, P.nchunks, st);
            if (threadIdx.x == 0) {
                atomicExch(&arrive[p], 0u);
                handover_release();   // the new state complete before it is announced
                if (sget<true>(&st->done)) {
                    s_base = 0xFFFFFFFFu;
                    atomicSub(&q->remaining, 1u);
                } else {
                    s_base = atomicAdd(&q->tail, (uint32_t)P.nchunks);
                }
            }
            __syncthreads();
            const uint32_t base = s_base;
            if (base != 0xFFFFFFFFu) {
                for (int j = threadIdx.x; j < P.nchunks; j += kChunk * G)
                    if (base + (uint32_t)j < cap)
                        __hip_atomic_store(&items[base + j], ((p << kChunkBits) | (uint32_t)j) + 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// Queue set-up: zero the item ring and the arrival counters, post every
// problem's first-iteration chunks (item slots = partial slots), and reset the
// queue counters.
__global__ void k_queue_init(const ProbDev* __restrict__ probs, int nprob, QueueDev* __restrict__ q,
                             uint32_t* __restrict__ items, uint32_t cap, uint32_t first, uint32_t* __restrict__ arrive) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t j = i; j < cap; j += gridDim.x * blockDim.x) items[j] = 0u;
    for (uint32_t j = i; j < (uint32_t)nprob; j += gridDim.x * blockDim.x) arrive[j] = 0u;
    if (i == 0) {
        q->head = 0u;
        q->tail = first;
        q->remaining = (uint32_t)nprob;
        q->error = 0u;
        q->cap = cap;
    }
}

__global__ void k_queue_post(const ProbDev* __restrict__ probs, int nprob, uint32_t* __restrict__ items) {
    const int p = blockIdx.x;
    if (p >= nprob) return;
    const ProbDev P = probs[p];
    for (int c = threadIdx.x; c < P.nchunks; c += blockDim.x)
        items[P.part0 + c] = (((uint32_t)p << kChunkBits) | (uint32_t)c) + 1u;
}

// ---------------------------------------------------------------------------
// Batched iteration as two launches: one workgroup per chunk of every
// problem (problems already retired return at once), then one workgroup per
// problem for its solve.  Same chunking and summation order as the queue.
// ---------------------------------------------------------------------------
__global__ void k_chunk_map(const ProbDev* __restrict__ probs, int nprob, int32_t* __restrict__ chunk_prob) {
    const int p = blockIdx.x;
    if (p >= nprob) return;
    const ProbDev P = probs[p];
    for (int c = threadIdx.x; c < P.nchunks; c += blockDim.x) chunk_prob[P.part0 + c] = p;
}

template <int ACC, int G = kLinGroup>
__global__ __launch_bounds__(kChunk * G) void k_gn_linearize_batch(const ProbDev* __restrict__ probs,
                                                                 const int32_t* __restrict__ chunk_prob,
                                                                 double* __restrict__ partials) {
    const int b = blockIdx.x;
    const int p = chunk_prob[b];
    if (p < 0) return;   // padding of a graph-captured launch
    const ProbDev P = probs[p];
    const RegState* st = P.st;
    if (st->done) return;
    float R[9], t[3];
#pragma unroll
    for (int j = 0; j < 9; ++j) R[j] = st->Rf[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) t[j] = st->tf[j];
    chunk_linearize<ACC, G>(P, b - P.part0, R, t, partials + (int64_t)b * kNumAcc);
}

__global__ __launch_bounds__(kSolveThreads) void k_gn_solve_batch(const ProbDev* __restrict__ probs,
                                                                  const double* __restrict__ partials,
                                                                  int32_t* __restrict__ chunk_prob) {
    const ProbDev P = probs[blockIdx.x];
    if (P.st->done) return;
    solve_block(partials + (int64_t)P.part0 * kNumAcc, P.nchunks, P.st);
    __syncthreads();
    // a problem that finished leaves the linearisation grid: its work items
    // exit on their first load in the remaining launches
    if (P.st->done)
        for (int c = threadIdx.x; c < P.nchunks; c += blockDim.x) chunk_prob[P.part0 + c] = -1;
}

// ---------------------------------------------------------------------------
// Sequential tracking: the problems of a call run one after another, each
// from a pose predicted on the device from the results of the previous ones.
// Per problem: one k_track_begin (which problem is next comes from a device
// counter, so that the same launches, or one captured graph, serve every
// problem), then max_it pairs of k_gn_linearize_batch (grid = the largest
// problem's chunk count; every problem uses partial slots from 0) and
// k_gn_solve_track.
// ---------------------------------------------------------------------------
__device__ void predict_pose(const ProbDev* __restrict__ probs, int i, int motion);

__global__ __launch_bounds__(256) void k_track_begin(const ProbDev* __restrict__ probs, int nprob,
                                                    int32_t* __restrict__ counter, int32_t* __restrict__ chunk_prob,
                                                    int grid, int motion) {
    __shared__ int s_i;
    if (threadIdx.x == 0) s_i = *counter;
    __syncthreads();
    const int i = s_i;
    const int nch = i < nprob ? probs[i].nchunks : 0;
    for (int c = threadIdx.x; c < grid; c += blockDim.x) chunk_prob[c] = c < nch ? i : -1;
    if (threadIdx.x != 0 || i >= nprob) return;
    *counter = i + 1;
    if (i > 0) predict_pose(probs, i, motion);   // the first problem starts from its given pose
}

// Initial pose of problem i >= 1 from the results of the problems before it:
// the previous pose b; with constant velocity also the one before, a:
// T = b (a^-1 b), the last relative motion applied once more.
__device__ void predict_pose(const ProbDev* __restrict__ probs, int i, int motion) {
    const double* b = probs[i - 1].st->pose;
    double T[16];
    if (motion == GICP_MOTION_CONSTANT_VELOCITY && i >= 2) {
        const double* a = probs[i - 2].st->pose;
        double D[12];   // a^-1 b as [R | t] rows
        for (int r = 0; r < 3; ++r) {
            for (int col = 0; col < 3; ++col)
                D[4 * r + col] = a[r] * b[col] + a[4 + r] * b[4 + col] + a[8 + r] * b[8 + col];
            D[4 * r + 3] = a[r] * (b[3] - a[3]) + a[4 + r] * (b[7] - a[7]) + a[8 + r] * (b[11] - a[11]);
        }
        for (int r = 0; r < 3; ++r) {
            for (int col = 0; col < 3; ++col)
                T[4 * r + col] = b[4 * r] * D[col] + b[4 * r + 1] * D[4 + col] + b[4 * r + 2] * D[8 + col];
            T[4 * r + 3] = b[4 * r] * D[3] + b[4 * r + 1] * D[7] + b[4 * r + 2] * D[11] + b[4 * r + 3];
        }
    } else {
        for (int j = 0; j < 12; ++j) T[j] = b[j];
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
    RegState* st = probs[i].st;
    for (int j = 0; j < 16; ++j) st->pose[j] = T[j];
    for (int r = 0; r < 3; ++r) {
        for (int col = 0; col < 3; ++col) st->Rf[3 * r + col] = (float)T[4 * r + col];
        st->tf[r] = (float)T[4 * r + 3];
    }
}

__global__ __launch_bounds__(kSolveThreads) void k_gn_solve_track(const ProbDev* __restrict__ probs,
                                                                  const double* __restrict__ partials,
                                                                  int32_t* __restrict__ chunk_prob) {
    const int p = chunk_prob[0];
    if (p < 0) return;
    const ProbDev P = probs[p];
    if (P.st->done) return;
    solve_block(partials, P.nchunks, P.st);
    __syncthreads();
    if (P.st->done)
        for (int c = threadIdx.x; c < P.nchunks; c += blockDim.x) chunk_prob[c] = -1;
}

// ---------------------------------------------------------------------------
// Iteration slots: the default form of sequential tracking.  The host
// launches iterations without knowing which problem each serves: the
// device's `cur` names it.  One launch is a whole Gauss-Newton iteration:
// every workgroup linearises its chunk at the current pose and writes its
// partial; the last workgroup to finish a group of partials (p, p + 32,
// p + 64, ...) sums that group, and the last group to finish sums the
// groups and solves; in exactly the order of solve_state, so that the
// result is bitwise that of the other forms.  When a problem finishes
// (converged, max_it, or failed), its solve predicts the next problem's pose
// and advances `cur`, so the next launch already works on the next problem:
// a problem costs exactly its own iterations.  The solving workgroup also
// publishes the progress (problems finished, slots run) to host-mapped
// memory, from which the host decides how many more slots to launch.
// ---------------------------------------------------------------------------
// Per-call hand-over words of the iteration slots (zero between launches).
struct SlotSync {
    uint32_t group[kSolveParts];   // partials of group p written so far
    uint32_t groups;               // groups summed so far
    uint32_t pad[31];
    double gsum[kSolveParts][kNumAcc];
};
static_assert(sizeof(SlotSync) % 8 == 0, "slot words");

// Members of group p among nparts partials.
__device__ __forceinline__ int group_members(int p, int nparts) { return p < nparts ? (nparts - p + 31) / 32 : 0; }

// Thread j < 29 of an NT-thread workgroup returns value j of group p's sum
// (partials p + 32 m in order of m; FP32 or FP64 as the mode), read
// device-coherently and staged through s_rows (LDS) 64 partials at a time.
constexpr int kGroupRows = 64;
template <int NT>
__device__ __forceinline__ double group_sum(const double* __restrict__ partials, int p, int nparts, int acc,
                                            double (*s_rows)[kNumAcc]) {
    constexpr int kRows = kGroupRows;
    constexpr int kPer = (kRows * kNumAcc + NT - 1) / NT;
    const int t = threadIdx.x;
    const int members = group_members(p, nparts);
    double v = 0.0;
    float f = 0.f;
    for (int m0 = 0; m0 < members; m0 += kRows) {
        const int cnt = min(kRows, members - m0);
        double x[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = t + u * NT, mm = e / kNumAcc, j = e % kNumAcc;
            x[u] = mm < cnt ? load_dev(&partials[(int64_t)(p + kSolveParts * (m0 + mm)) * kNumAcc + j]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = t + u * NT;
            if (e < kRows * kNumAcc) s_rows[e / kNumAcc][e % kNumAcc] = x[u];
        }
        __syncthreads();
        if (t < kNumAcc)
            for (int mm = 0; mm < cnt; ++mm) {
                f += (float)s_rows[mm][t];
                v += s_rows[mm][t];
            }
        __syncthreads();
    }
    return acc == GICP_ACC_FP32 ? (double)f : v;
}

// ctl (device): [0] and [1] the current problem for launches of parity 0 and
// 1 (every workgroup of a launch reads its own word, which only the next
// launch's parity is written to: workgroups that start late still see the
// launch's problem), [2] slots run.  The kernel's registers are bounded so
// that five workgroups fit on a CU: a 77k-point frame's chunks all resident.
template <int ACC, int G>
__global__ __launch_bounds__(kChunk * G) __attribute__((amdgpu_waves_per_eu(5))) void k_slot_iterate(
    const ProbDev* __restrict__ probs, int nprob, int32_t* __restrict__ ctl, int parity, double* __restrict__ partials,
    SlotSync* __restrict__ sync, int motion, int32_t* __restrict__ progress) {
    constexpr int NT = kChunk * G;
    static_assert(NT >= kNumAcc && NT >= kPreFields && NT > kSolveParts && NT >= 64, "slot block size");
    static_assert(kGroupRows >= kSolveParts, "the group rows also hold the groups' sums");
    __shared__ int s_last;
    __shared__ double s_rows[kGroupRows][kNumAcc];
    __shared__ double s_v[kNumAcc];
    __shared__ double s_pre[kPreFields];
    __shared__ double s_HL[72];
    const int t = threadIdx.x;
    const int b = blockIdx.x;
    const int i = ctl[parity];
    bool solver = false;   // this workgroup completes the launch
    if (i < nprob) {
        const ProbDev P = probs[i];
        RegState* st = P.st;
        if (st->done) {
            solver = b == 0;   // finished before its first iteration: only move on
        } else {
            if (b >= P.nchunks) return;
            float R[9], tr[3];
#pragma unroll
            for (int j = 0; j < 9; ++j) R[j] = st->Rf[j];
#pragma unroll
            for (int j = 0; j < 3; ++j) tr[j] = st->tf[j];
            chunk_linearize<ACC, G, true>(P, b, R, tr, partials + (int64_t)b * kNumAcc);
            const int p = b % kSolveParts;
            if (t == 0)
                s_last = atomicAdd(&sync->group[p], 1u) == (uint32_t)group_members(p, P.nchunks) - 1u ? 1 : 0;
            __syncthreads();
            if (!s_last) return;
            handover_acquire();
            const int acc = st->acc;
            const double gs = group_sum<NT>(partials, p, P.nchunks, acc, s_rows);
            if (t < kNumAcc) {
                store_dev(&sync->gsum[p][t], gs);
                handover_release();
            }
            __syncthreads();
            const int ngroups = min(kSolveParts, P.nchunks);
            if (t == 0) s_last = atomicAdd(&sync->groups, 1u) == (uint32_t)ngroups - 1u ? 1 : 0;
            __syncthreads();
            if (!s_last) return;
            handover_acquire();
            // the last group: the groups' sums in order of p (empty groups
            // add zero, as in solve_state), then the update
            const double pre = t < kPreFields ? gload((const double*)st, pre_word(t)) : 0.0;
            for (int e = t; e < ngroups * kNumAcc; e += NT)
                s_rows[e / kNumAcc][e % kNumAcc] = load_dev(&sync->gsum[0][0] + e);
            if (t < kPreFields) s_pre[t] = pre;
            __syncthreads();
            if (t < kNumAcc) {
                if (acc == GICP_ACC_FP32) {
                    float f = 0.f;
                    for (int q = 0; q < kSolveParts; ++q) f += q < ngroups ? (float)s_rows[q][t] : 0.f;
                    s_v[t] = (double)f;
                } else {
                    double v = 0.0;
                    for (int q = 0; q < kSolveParts; ++q) v += q < ngroups ? s_rows[q][t] : 0.0;
                    s_v[t] = v;
                }
            }
            // the hand-over words back to zero for the next launch
            if (t < kSolveParts) __hip_atomic_store(&sync->group[t], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == kSolveParts) __hip_atomic_store(&sync->groups, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            __shared__ SolveOut s_out;
            if (t == 0) solve_update_inl(s_v, s_pre, s_HL, s_HL + 36, &s_out);
            __syncthreads();
            solve_publish<false>(s_out, s_HL, s_v, st, t);
            __syncthreads();
            solver = true;
        }
    } else {
        solver = b == 0;   // every problem finished: only count the slot
    }
    if (!solver || t != 0) return;
    const int slots = ctl[2] + 1;
    int next = i, done = i < nprob ? i : nprob;
    if (i < nprob && probs[i].st->done) {
        if (i + 1 < nprob) predict_pose(probs, i + 1, motion);
        next = i + 1;
        done = i + 1;
    }
    ctl[parity ^ 1] = next;
    ctl[2] = slots;
    // progress for the host (host-mapped memory, plain vector stores)
    __hip_atomic_store(&progress[0], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&progress[1], slots, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// Device-resident registration (gicp_register_dev): the problem descriptor and
// the initial state are written by a kernel from its arguments and the
// device initial pose, and the results are written by a kernel to device
// outputs, so that the whole call is stream-ordered device work that a HIP
// graph can capture.
// ---------------------------------------------------------------------------
__global__ void k_state_init(ProbDev pd, ProbDev* __restrict__ dst, StateInit si, const double* __restrict__ init,
                             RegState* __restrict__ st) {
    if (threadIdx.x != 0) return;
    *dst = pd;
    for (int j = 0; j < 16; ++j) st->pose[j] = init[j];
    for (int j = 0; j < 21; ++j) st->H[j] = 0.0;
    for (int j = 0; j < 6; ++j) st->b[j] = 0.0;
    st->cost = 0.0;
    st->n_inl = 0.0;
    st->conv_rot = si.conv_rot;
    st->conv_trans = si.conv_trans;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) st->Rf[3 * r + c] = (float)init[4 * r + c];
        st->tf[r] = (float)init[4 * r + 3];
    }
    st->iters = 0;
    st->max_it = si.max_it;
    st->done = si.max_it <= 0 ? 1 : 0;
    st->status = GICP_OK;
    st->converged = 0;
    st->acc = si.acc;
}

__global__ void k_state_out(const RegState* __restrict__ st, const int* __restrict__ err, double* __restrict__ pose,
                            double* __restrict__ H, double* __restrict__ b, gicp_stats* __restrict__ stats) {
    const int t = threadIdx.x;
    if (t < 16) pose[t] = st->pose[t];
    if (t < 36) {
        const int i = t / 6, j = t % 6;
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        H[t] = st->H[lo * 6 - lo * (lo - 1) / 2 + (hi - lo)];
    }
    if (t < 6) b[t] = st->b[t];
    if (t == 0 && stats) {
        gicp_stats o;
        o.iters = st->iters;
        o.n_inliers = (int32_t)st->n_inl;
        o.cost = st->cost;
        o.converged = st->converged;
        o.status = (*err & kErrNonFinite) ? GICP_E_NONFINITE : st->status;
        o.hip_error = 0;
        o.reserved = 0;
        *stats = o;
    }
}

// ---------------------------------------------------------------------------
// Keyframe Gaussians (Sec. 3.1.2, Keyframe Selection; Sec. 3.2.1, Scale Aligning)
// ---------------------------------------------------------------------------
// keep[i] = 1 when R x_i + t has no map mean within r_max (the point adds a
// new Gaussian), 0 when it has a correspondence.  kGroup lanes per point.
__global__ __launch_bounds__(kBlock) void k_overlap(MapView m, const float* __restrict__ src, int64_t n, Pose32 T,
                                                   uint32_t* __restrict__ keep) {
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t i = (int64_t)blockIdx.x * (kBlock / kGroup) + threadIdx.x / kGroup;
    if (i >= n) return;   // uniform over each lane group
    const float x = src[i], y = src[n + i], z = src[2 * n + i];
    const float qx = T.R[0] * x + T.R[1] * y + T.R[2] * z + T.t[0];
    const float qy = T.R[3] * x + T.R[4] * y + T.R[5] * z + T.t[1];
    const float qz = T.R[6] * x + T.R[7] * y + T.R[8] * z + T.t[2];
    const int32_t pos = nearest<false>(m, qx, qy, qz, l, -1);
    if (l == 0) keep[i] = pos < 0 ? 1u : 0u;
}

// Nearest map mean of arbitrary queries by the linearisation's own search
// (nearest<true, G>: G = 2 as the two-lane launches, 4, 8 or 16 as the
// four-lane ones, whose searches of few points take 8 or 16 lanes), with its
// certified radius: the match, its FP32
// key and the radius (the query can move by less than it without changing
// its nearest mean), or -1 / +inf / -1 when no mean lies within the gate.
template <int G>
__global__ __launch_bounds__(kBlock) void k_map_nearest(MapView m, const float* __restrict__ q, int64_t nq,
                                                       const int32_t* __restrict__ hints,
                                                       const int32_t* __restrict__ inv, int32_t* __restrict__ idx,
                                                       float* __restrict__ d2, float* __restrict__ radius) {
    const int l = threadIdx.x & (G - 1);
    const int64_t i = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
    if (i >= nq) return;   // uniform over each lane group
    const float qx = q[i], qy = q[nq + i], qz = q[2 * nq + i];
    int32_t hint = -1;
    if (hints) {
        const int32_t h = hints[i];
        if (h >= 0 && h < m.g.n) hint = inv[h];
    }
    float fr = -1.f;
    int32_t pos;
    if constexpr (G == 4) pos = nearest_coop4<true>(m, qx, qy, qz, l, hint, &fr);
    else pos = nearest<true, G>(m, qx, qy, qz, l, hint, &fr);
    if (l == 0) {
        if (pos >= 0) {
            const float4 p = gload(m.g.spts, pos);
            idx[i] = (int32_t)__float_as_uint(p.w);
            d2[i] = rank_key(qx, qy, qz, p.x, p.y, p.z);
        } else {
            idx[i] = -1;
            d2[i] = __builtin_inff();
        }
        if (radius) radius[i] = fr;
    }
}

__global__ void k_map_inverse(const float4* __restrict__ spts, int64_t m, int32_t* __restrict__ inv) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint32_t o = __float_as_uint(spts[j].w);
    if ((int64_t)o < m) inv[o] = (int32_t)j;
}

// The kept points, scale aligned in the camera frame (C / z^(2p), z the
// depth) and moved into the map frame (mu = R x + t, C = R C R^T), in FP64,
// written in point order at their compacted positions.
__global__ void k_keyframe_gaussians(const float* __restrict__ src, const float* __restrict__ covs, int64_t n,
                                     const uint32_t* __restrict__ keep, const uint32_t* __restrict__ pos, Pose64 T,
                                     double two_p, float* __restrict__ out_means, float* __restrict__ out_covs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const int64_t o = pos[i];
    const double x = src[i], y = src[n + i], z = src[2 * n + i];
    const double* R = T.R;
    out_means[o] = (float)(R[0] * x + R[1] * y + R[2] * z + T.t[0]);
    out_means[n + o] = (float)(R[3] * x + R[4] * y + R[5] * z + T.t[1]);
    out_means[2 * n + o] = (float)(R[6] * x + R[7] * y + R[8] * z + T.t[2]);
    const double sc = z > 0.0 ? pow(z, -two_p) : 1.0;
    const double C[9] = {covs[i] * sc,         covs[n + i] * sc,     covs[2 * n + i] * sc,
                         covs[n + i] * sc,     covs[3 * n + i] * sc, covs[4 * n + i] * sc,
                         covs[2 * n + i] * sc, covs[4 * n + i] * sc, covs[5 * n + i] * sc};
    double RC[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) RC[3 * a + b] = R[3 * a] * C[b] + R[3 * a + 1] * C[3 + b] + R[3 * a + 2] * C[6 + b];
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
        const int a = ia[e], b = ib[e];
        out_covs[e * n + o] = (float)(RC[3 * a] * R[3 * b] + RC[3 * a + 1] * R[3 * b + 1] + RC[3 * a + 2] * R[3 * b + 2]);
    }
}

}  // namespace

int gn_blocks(int64_t n) {
    const int64_t b = (n + kChunk - 1) / kChunk;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_gn_linearize(const ProbDev& pd, double* partials, int nblocks, int acc, hipStream_t s) {
    switch (acc) {
        case GICP_ACC_FP32:
            hipLaunchKernelGGL(k_gn_linearize<GICP_ACC_FP32>, dim3(nblocks), dim3(kBlock), 0, s, pd, partials);
            break;
        case GICP_ACC_FP64:
            hipLaunchKernelGGL(k_gn_linearize<GICP_ACC_FP64>, dim3(nblocks), dim3(kBlock), 0, s, pd, partials);
            break;
        default:
            hipLaunchKernelGGL(k_gn_linearize<GICP_ACC_TWOSUM>, dim3(nblocks), dim3(kBlock), 0, s, pd, partials);
    }
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t b = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

namespace {

// Launch tables over the accumulation mode (0..2) and the lanes per point
// (index 0: two, 1: four).
constexpr int lanes_index(int lanes) { return lanes == 4 ? 1 : 0; }

template <int ACC, int G>
void queue_t(unsigned workers, const ProbDev* probs, QueueDev* q, uint32_t* items, uint32_t* arrive,
             double* partials, hipStream_t s) {
    hipLaunchKernelGGL((k_gn_queue<ACC, G>), dim3(workers), dim3(kChunk * G), 0, s, probs, q, items, arrive, partials);
}
template <int ACC, int G>
int queue_occupancy() {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gn_queue<ACC, G>, kChunk * G, 0) != hipSuccess) return 0;
    return per;
}
using QueueFn = void (*)(unsigned, const ProbDev*, QueueDev*, uint32_t*, uint32_t*, double*, hipStream_t);
using OccFn = int (*)();
constexpr QueueFn kQueue[3][2] = {{queue_t<0, 2>, queue_t<0, 4>}, {queue_t<1, 2>, queue_t<1, 4>},
                                  {queue_t<2, 2>, queue_t<2, 4>}};
constexpr OccFn kQueueOcc[3][2] = {{queue_occupancy<0, 2>, queue_occupancy<0, 4>},
                                   {queue_occupancy<1, 2>, queue_occupancy<1, 4>},
                                   {queue_occupancy<2, 2>, queue_occupancy<2, 4>}};

template <int ACC, int G>
void lin_batch_t(unsigned grid, const ProbDev* probs, const int32_t* chunk_prob, double* partials, hipStream_t s) {
    hipLaunchKernelGGL((k_gn_linearize_batch<ACC, G>), dim3(grid), dim3(kChunk * G), 0, s, probs, chunk_prob, partials);
}
using LinFn = void (*)(unsigned, const ProbDev*, const int32_t*, double*, hipStream_t);
constexpr LinFn kLinBatch[3][2] = {{lin_batch_t<0, 2>, lin_batch_t<0, 4>}, {lin_batch_t<1, 2>, lin_batch_t<1, 4>},
                                   {lin_batch_t<2, 2>, lin_batch_t<2, 4>}};

template <int ACC, int G>
void slot_t(unsigned grid, const ProbDev* probs, int nprob, int32_t* ctl, int parity, double* partials, SlotSync* sy,
            int motion, int32_t* progress, hipStream_t s) {
    hipLaunchKernelGGL((k_slot_iterate<ACC, G>), dim3(grid), dim3(kChunk * G), 0, s, probs, nprob, ctl, parity,
                       partials, sy, motion, progress);
}
using SlotFn = void (*)(unsigned, const ProbDev*, int, int32_t*, int, double*, SlotSync*, int, int32_t*, hipStream_t);
constexpr SlotFn kSlot[3][2] = {{slot_t<0, 2>, slot_t<0, 4>}, {slot_t<1, 2>, slot_t<1, 4>},
                                {slot_t<2, 2>, slot_t<2, 4>}};

}  // namespace

int gn_queue_workers(int acc, int lanes) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    int per = kQueueOcc[acc][lanes_index(lanes)]();
    if (per < 1) per = 1;
    return cus * per;
}

hipError_t launch_gn_queue(const ProbDev* probs, int nprob, QueueDev* q, uint32_t* items, uint32_t cap,
                           uint32_t first, uint32_t* arrive, double* partials, int workers, int acc, int lanes,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_queue_init, dim3(64), dim3(256), 0, s, probs, nprob, q, items, cap, first, arrive);
    hipLaunchKernelGGL(k_queue_post, dim3(nprob), dim3(256), 0, s, probs, nprob, items);
    kQueue[acc][lanes_index(lanes)]((unsigned)workers, probs, q, items, arrive, partials, s);
    return hipGetLastError();
}

hipError_t launch_chunk_map(const ProbDev* probs, int nprob, int32_t* chunk_prob, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_map, dim3(nprob), dim3(256), 0, s, probs, nprob, chunk_prob);
    return hipGetLastError();
}

hipError_t launch_gn_iteration_batch(const ProbDev* probs, int nprob, int32_t* chunk_prob, int64_t chunks,
                                     double* partials, int acc, int lanes, bool linearize, bool solve, hipStream_t s) {
    if (linearize) kLinBatch[acc][lanes_index(lanes)]((unsigned)chunks, probs, chunk_prob, partials, s);
    if (solve)
        hipLaunchKernelGGL(k_gn_solve_batch, dim3(nprob), dim3(kSolveThreads), 0, s, probs, (const double*)partials,
                           chunk_prob);
    return hipGetLastError();
}

hipError_t launch_track_begin(const ProbDev* probs, int nprob, int32_t* counter, int32_t* chunk_prob, int64_t grid,
                              int motion, hipStream_t s) {
    hipLaunchKernelGGL(k_track_begin, dim3(1), dim3(256), 0, s, probs, nprob, counter, chunk_prob, (int)grid, motion);
    return hipGetLastError();
}

hipError_t launch_gn_track_iteration(const ProbDev* probs, int32_t* chunk_prob, int64_t grid, double* partials, int acc,
                                     int lanes, bool linearize, bool solve, hipStream_t s) {
    if (linearize) kLinBatch[acc][lanes_index(lanes)]((unsigned)grid, probs, chunk_prob, partials, s);
    if (solve)
        hipLaunchKernelGGL(k_gn_solve_track, dim3(1), dim3(kSolveThreads), 0, s, probs, (const double*)partials,
                           chunk_prob);
    return hipGetLastError();
}

hipError_t launch_track_slot(const ProbDev* probs, int nprob, int32_t* ctl, int parity, int64_t grid, double* partials,
                             int acc, int lanes, int motion, int32_t* progress, void* sync, hipStream_t s) {
    kSlot[acc][lanes_index(lanes)]((unsigned)grid, probs, nprob, ctl, parity, partials, (SlotSync*)sync, motion,
                                   progress, s);
    return hipGetLastError();
}

size_t slot_sync_bytes() { return sizeof(SlotSync); }

hipError_t launch_state_init(const ProbDev& pd, ProbDev* dst, const StateInit& si, const double* init, RegState* st,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, pd, dst, si, init, st);
    return hipGetLastError();
}

hipError_t launch_state_out(const RegState* st, const int* err, double* pose, double* H, double* b,
                            gicp_stats* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_state_out, dim3(1), dim3(64), 0, s, st, err, pose, H, b, stats);
    return hipGetLastError();
}

hipError_t launch_gn_solve(const double* partials, int nblocks, RegState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_gn_solve, dim3(1), dim3(kSolveThreads), 0, s, partials, nblocks, st);
    return hipGetLastError();
}

hipError_t launch_overlap(const MapView& m, const float* src, int64_t n, const Pose32& T, uint32_t* keep,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int per = kBlock / kGroup;
    hipLaunchKernelGGL(k_overlap, dim3((unsigned)((n + per - 1) / per)), dim3(kBlock), 0, s, m, src, n, T, keep);
    return hipGetLastError();
}

hipError_t launch_map_nearest(const MapView& m, const float* q, int64_t nq, const int32_t* hints, const int32_t* inv,
                              int32_t* idx, float* d2, float* radius, int lanes, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const int per = kBlock / lanes;
    const dim3 grid((unsigned)((nq + per - 1) / per));
    switch (lanes) {
    case 2: hipLaunchKernelGGL(k_map_nearest<2>, grid, dim3(kBlock), 0, s, m, q, nq, hints, inv, idx, d2, radius); break;
    case 4: hipLaunchKernelGGL(k_map_nearest<4>, grid, dim3(kBlock), 0, s, m, q, nq, hints, inv, idx, d2, radius); break;
    case 8: hipLaunchKernelGGL(k_map_nearest<8>, grid, dim3(kBlock), 0, s, m, q, nq, hints, inv, idx, d2, radius); break;
    case 16: hipLaunchKernelGGL(k_map_nearest<16>, grid, dim3(kBlock), 0, s, m, q, nq, hints, inv, idx, d2, radius); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_map_inverse(const float4* spts, int64_t m, int32_t* inv, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_inverse, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, spts, m, inv);
    return hipGetLastError();
}

hipError_t launch_keyframe_gaussians(const float* src, const float* covs, int64_t n, const uint32_t* keep,
                                     const uint32_t* pos, const Pose64& T, double two_p, float* out_means,
                                     float* out_covs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_keyframe_gaussians, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, covs, n, keep,
                       pos, T, two_p, out_means, out_covs);
    return hipGetLastError();
}

}  // namespace gicp
