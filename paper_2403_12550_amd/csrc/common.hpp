// Shared device/host definitions of the gfx950 G-ICP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gicp.h"

namespace gicp {

constexpr int kBlock = 256;           // threads per workgroup for the point kernels
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr int kCellBits = 8;          // wrapped cell coordinate bits per axis (24-bit keys)
constexpr uint32_t kCellMask = (1u << kCellBits) - 1u;
constexpr int kMaxShell = 8;          // k-NN grid shells searched before the overflow pass
constexpr int kMaxGateShells = 64;    // 1-NN: shells allowed for the gate to end the search
constexpr int kNumAcc = 29;           // 21 unique H terms, 6 b terms, cost, inlier count

// Error bits recorded on the device (context error word).
constexpr int kErrNonFinite = 1;
constexpr int kErrInexact = 2;
constexpr int kErrIndex = 4;       // an index argument read on the device was out of range

// ---------------------------------------------------------------------------
// Grid cells.  A point p lies in cell floor(p * inv_h) per axis; the cell key
// packs the three cell coordinates modulo 256 (8 bits each).  Wrapping cannot
// break exactness: candidates are always ranked by their real distance, and
// an aliased cell (256 cells away) only adds far-away candidates.
// ---------------------------------------------------------------------------
struct Cell {
    int x, y, z;
};

__device__ __forceinline__ Cell cell_of(float x, float y, float z, float inv_h) {
    Cell c;
    c.x = (int)floorf(x * inv_h);
    c.y = (int)floorf(y * inv_h);
    c.z = (int)floorf(z * inv_h);
    return c;
}

__device__ __forceinline__ uint32_t cell_key(int cx, int cy, int cz) {
    return ((uint32_t)cx & kCellMask) | (((uint32_t)cy & kCellMask) << kCellBits) |
           (((uint32_t)cz & kCellMask) << (2 * kCellBits));
}

// Knuth's multiplicative hashing: the slot is the top log2(capacity) bits of
// key * 2654435761 mod 2^32 (the low bits of the product would depend only on
// the low bits of the key, i.e. only on x and part of y).  mask = capacity - 1.
__device__ __forceinline__ uint32_t hash_slot(uint32_t key, uint32_t mask) {
    return (key * 2654435761u) >> (32 - __popc(mask));
}

// Loads and stores through a pointer the compiler cannot place in an address
// space (one read from a descriptor in memory) would be flat instructions;
// these go through the global address space, where every array of the
// library lives.
// (the element moves as a 4-, 8- or 16-byte word of the same size; HIP's
// vector types cannot be copied out of another address space directly)
template <int B>
struct GWord;
template <>
struct GWord<4> { typedef uint32_t type; };
template <>
struct GWord<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <>
struct GWord<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

template <class T>
__device__ __forceinline__ T gload(const T* p, int64_t i) {
    typedef typename GWord<sizeof(T)>::type W;
    const W w = ((const __attribute__((address_space(1))) W*)p)[i];
    T r;
    __builtin_memcpy(&r, &w, sizeof(T));
    return r;
}

template <class T>
__device__ __forceinline__ void gstore(T* p, int64_t i, const T& v) {
    typedef typename GWord<sizeof(T)>::type W;
    W w;
    __builtin_memcpy(&w, &v, sizeof(T));
    ((__attribute__((address_space(1))) W*)p)[i] = w;
}

// Cell table lookup: entry = {key, start, count, -}.  Returns count (0 if the
// cell is empty) and writes its start offset into the cell-sorted arrays.
__device__ __forceinline__ uint32_t cell_lookup(const uint4* __restrict__ table, uint32_t mask,
                                                uint32_t key, uint32_t& start) {
    uint32_t s = hash_slot(key, mask);
    while (true) {
        const uint4 e = gload(table, s);
        if (e.x == key) {
            start = e.y;
            return e.z;
        }
        if (e.x == kEmptyKey) return 0u;
        s = (s + 1u) & mask;
    }
}

// FP32 ranking key of the k-NN: fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) with
// dx = fl(q.x - p.x), every operation rounded on its own (no contraction into
// fused multiply-adds), so that the ranking is reproducible bit for bit.
__device__ __forceinline__ float rank_key(float qx, float qy, float qz, float px, float py, float pz) {
#pragma clang fp contract(off)
    const float dx = qx - px;
    const float dy = qy - py;
    const float dz = qz - pz;
    const float s = dx * dx + dy * dy;
    return s + dz * dz;
}

// Candidate words: (FP32 key bits + 2^20) << 32 | index.  Unsigned integer
// order is the (key, index) order, and the offset makes every word the bit
// pattern of a positive normal double (exponent field 0x001 .. 0x7F9 for keys
// from +0 to +inf), whose floating-point order is the same: the minimum and
// maximum of two words are single v_min_f64 / v_max_f64 instructions.  The
// empty word is +inf, above every word.
constexpr uint32_t kWordBias = 1u << 20;
constexpr uint64_t kEmptyWord = 0x7FF0000000000000ull;

__device__ __forceinline__ uint64_t word(float key, uint32_t idx) {
    return ((uint64_t)(__float_as_uint(key) + kWordBias) << 32) | (uint64_t)idx;
}

__device__ __forceinline__ float word_key(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32) - kWordBias); }

// Minimum and maximum of two words, written as the instructions on the raw
// registers: as doubles the words (no NaN, no denormal) compare exactly like
// the integers, and the compiler's own fmin / fmax would first quieten every
// operand.
__device__ __forceinline__ uint64_t wmin(uint64_t a, uint64_t b) {
    uint64_t r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ uint64_t wmax(uint64_t a, uint64_t b) {
    uint64_t r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// Distance from q to the boundary of the block of cells [c - R, c + R] per
// axis, minus a safety margin that covers the rounding of the cell
// assignment, and the FP32 key bound below which every point outside the
// block is provably ranked after the current k-th neighbour.
__device__ __forceinline__ float block_clearance(float qx, float qy, float qz, Cell c, int R, float h) {
    const float lox = (float)(c.x - R) * h, hix = (float)(c.x + R + 1) * h;
    const float loy = (float)(c.y - R) * h, hiy = (float)(c.y + R + 1) * h;
    const float loz = (float)(c.z - R) * h, hiz = (float)(c.z + R + 1) * h;
    float d = fminf(fminf(qx - lox, hix - qx), fminf(fminf(qy - loy, hiy - qy), fminf(qz - loz, hiz - qz)));
    const float mag = fmaxf(fmaxf(fabsf(qx), fabsf(qy)), fabsf(qz)) + (float)(R + 1) * h;
    d = d - 4e-6f * mag - 1e-6f * h;   // cell rounding slack (relative 4e-6 of the coordinate scale)
    return d;
}

// Slack of the cell assignment: a point assigned to cell c by floor(p * inv_h)
// lies within [c*h - slack, (c+1)*h + slack] per axis.
__device__ __forceinline__ float cell_slack(float qx, float qy, float qz, int R, float h) {
    const float mag = fmaxf(fmaxf(fabsf(qx), fabsf(qy)), fabsf(qz)) + (float)(R + 1) * h;
    return 4e-6f * mag + 1e-6f * h;
}

// Lower bound of the squared distance from q to any point assigned to cell
// (cx, cy, cz): the distance to the cell box grown by the slack.
__device__ __forceinline__ float cell_lower_bound2(float qx, float qy, float qz, int cx, int cy, int cz, float h,
                                                  float slack) {
    const float dx = fmaxf(fmaxf((float)cx * h - slack - qx, qx - (float)(cx + 1) * h - slack), 0.f);
    const float dy = fmaxf(fmaxf((float)cy * h - slack - qy, qy - (float)(cy + 1) * h - slack), 0.f);
    const float dz = fmaxf(fmaxf((float)cz * h - slack - qz, qz - (float)(cz + 1) * h - slack), 0.f);
    return dx * dx + dy * dy + dz * dz;
}

// A cell whose lower bound exceeds the current k-th key cannot hold a point
// that ranks before it (the FP32 key is within 3e-7 relative of the exact
// squared distance; the factor covers that and the rounding of the bound).
__device__ __forceinline__ bool cell_pruned(float lb2, float kth_key) { return lb2 * (1.f - 2e-6f) > kth_key; }

// The 27 offsets of the block around a cell, nearest first: the cell itself,
// 6 faces, 12 edges, 8 corners.  Offset j is packed in 5 bits as
// (dx+1) + 3(dy+1) + 9(dz+1), twelve to a 64-bit word (pure ALU; j is
// uniform across the wavefront).
__device__ __forceinline__ void block_offset(int j, int& dx, int& dy, int& dz) {
    const uint64_t w = (j < 12) ? 0x01c5eb4d8905398dull : (j < 24) ? 0x0920c2066670dea5ull : 0x0000000000006b14ull;
    const int o = (int)((w >> (5 * (j % 12))) & 31u);
    dx = o % 3 - 1;
    dy = (o / 3) % 3 - 1;
    dz = o / 9 - 1;
}

}  // namespace gicp
