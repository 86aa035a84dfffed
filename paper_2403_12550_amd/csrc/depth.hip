// Depth image -> tracking point cloud (Sec. 3, system overview: the current
// depth image is reprojected and downsampled into the cloud G-ICP tracks).
//
// Pinhole back-projection x = (u - cx) z / fx, y = (v - cy) z / fy in FP32
// (each operation rounded on its own, so the voxel a point falls into is
// reproducible), voxel (floor(x/s), floor(y/s), floor(z/s)); every occupied
// voxel yields the FP64 centroid of its points, rounded to FP32 once, and the
// voxels come out sorted by (ix, iy, iz).  The voxel coordinates are packed
// into a mixed-radix key over the occupied bounding box and sorted with the
// library's stable radix sort, so the points of a voxel stay in pixel order.
#include <climits>
#include <float.h>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

constexpr int kLimit = 1 << 30;   // |coordinate / voxel| bound (larger values are rejected)

// Back-projection, voxel coordinates and their bounding box.  bounds:
// [min x, min y, min z, max x, max y, max z] (ints, initialised by the caller).
__global__ void k_depth_points(const float* __restrict__ depth, int W, int H, float fx, float fy, float cx, float cy,
                               float voxel, float max_depth, float* __restrict__ pts, int* __restrict__ vox,
                               int* __restrict__ bounds) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)W * H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int u = (int)(i % W), v = (int)(i / W);
    const float z = depth[i];
    bool ok = isfinite(z) && z > 0.f && z <= max_depth;
    const float x = (((float)u - cx) * z) / fx;
    const float y = (((float)v - cy) * z) / fy;
    const float fx_ = x / voxel, fy_ = y / voxel, fz_ = z / voxel;
    ok = ok && isfinite(x) && isfinite(y) && fabsf(fx_) < (float)kLimit && fabsf(fy_) < (float)kLimit &&
         fabsf(fz_) < (float)kLimit;
    int ix = 0, iy = 0, iz = 0;
    if (ok) {
        ix = (int)floorf(fx_);
        iy = (int)floorf(fy_);
        iz = (int)floorf(fz_);
        atomicMin(&bounds[0], ix);
        atomicMin(&bounds[1], iy);
        atomicMin(&bounds[2], iz);
        atomicMax(&bounds[3], ix);
        atomicMax(&bounds[4], iy);
        atomicMax(&bounds[5], iz);
    }
    pts[i] = x;
    pts[n + i] = y;
    pts[2 * n + i] = z;
    vox[i] = ok ? ix : INT_MIN;   // INT_MIN marks an invalid pixel
    vox[n + i] = iy;
    vox[2 * n + i] = iz;
}

// Mixed-radix voxel key over the bounding box (invalid pixels: all ones).
__global__ void k_voxel_keys(const int* __restrict__ vox, int64_t n, const int* __restrict__ bounds, uint32_t dy,
                             uint32_t dz, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ix = vox[i];
    uint32_t key = 0xFFFFFFFFu;
    if (ix != INT_MIN) {
        const uint32_t a = (uint32_t)(ix - bounds[0]), b = (uint32_t)(vox[n + i] - bounds[1]),
                       c = (uint32_t)(vox[2 * n + i] - bounds[2]);
        key = (a * dy + b) * dz + c;
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
}

// flag[i] = 1 at the first sorted entry of every occupied voxel.
__global__ void k_voxel_starts(const uint32_t* __restrict__ skeys, int64_t n, uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = skeys[i];
    flags[i] = (k != 0xFFFFFFFFu && (i == 0 || skeys[i - 1] != k)) ? 1u : 0u;
}

// Centroid of each voxel: FP64 sums in pixel order, one thread per voxel.
__global__ void k_voxel_centroids(const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ svals, int64_t n,
                                  const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                                  const float* __restrict__ pts, float* __restrict__ out, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t k = skeys[i];
    double sx = 0, sy = 0, sz = 0;
    int64_t c = 0;
    for (int64_t j = i; j < n && skeys[j] == k; ++j, ++c) {
        uint32_t p = svals[j];
        if (p >= (uint64_t)n) p = 0;   // always a permutation; guards the gather
        sx += (double)pts[p];
        sy += (double)pts[n + p];
        sz += (double)pts[2 * n + p];
    }
    const int64_t o = pos[i];
    if (o >= m) return;
    out[o] = (float)(sx / (double)c);
    out[m + o] = (float)(sy / (double)c);
    out[2 * m + o] = (float)(sz / (double)c);
}

__global__ void k_init_bounds(int* b) {
    if (threadIdx.x < 3) b[threadIdx.x] = INT_MAX;
    else if (threadIdx.x < 6) b[threadIdx.x] = INT_MIN;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_depth_points(const float* depth, int W, int H, float fx, float fy, float cx, float cy, float voxel,
                               float max_depth, float* pts, int* vox, int* bounds, hipStream_t s) {
    const int64_t n = (int64_t)W * H;
    hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, s, bounds);
    hipLaunchKernelGGL(k_depth_points, dim3(blocks(n)), dim3(256), 0, s, depth, W, H, fx, fy, cx, cy, voxel, max_depth,
                       pts, vox, bounds);
    return hipGetLastError();
}

hipError_t launch_voxel_keys(const int* vox, int64_t n, const int* bounds, uint32_t dy, uint32_t dz, uint32_t* keys,
                             uint32_t* vals, hipStream_t s) {
    hipLaunchKernelGGL(k_voxel_keys, dim3(blocks(n)), dim3(256), 0, s, vox, n, bounds, dy, dz, keys, vals);
    return hipGetLastError();
}

hipError_t launch_voxel_starts(const uint32_t* skeys, int64_t n, uint32_t* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_voxel_starts, dim3(blocks(n)), dim3(256), 0, s, skeys, n, flags);
    return hipGetLastError();
}

hipError_t launch_voxel_centroids(const uint32_t* skeys, const uint32_t* svals, int64_t n, const uint32_t* flags,
                                  const uint32_t* pos, const float* pts, float* out, int64_t m, hipStream_t s) {
    hipLaunchKernelGGL(k_voxel_centroids, dim3(blocks(n)), dim3(256), 0, s, skeys, svals, n, flags, pos, pts, out, m);
    return hipGetLastError();
}

}  // namespace gicp
