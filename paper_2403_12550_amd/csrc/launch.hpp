// Host-side launchers of the gfx950 kernels (internal to libgicp.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace gicp {

// Scratch the radix sort needs for n keys (bytes), and the launcher.  Sorts
// keys of 8 * passes bits with their values stably, ping-ponging between the
// a and b buffers; *keys_out / *vals_out receive the buffers with the result.
size_t radix_scratch_bytes(int64_t n);
hipError_t radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, int64_t n,
                      int passes, void* scratch, hipStream_t s, uint32_t** keys_out, uint32_t** vals_out);

// One cloud of a (possibly segmented) grid.  Several clouds share one sort
// and one cell table: the cloud index occupies the top 8 bits of the cell
// key, so each cloud's points form the contiguous grid-order range
// [off, off + n) and cells of different clouds never mix.
struct Seg {
    const float* xyz;     // SoA [3][n]
    float* covs;          // SoA [6][n] covariance output in the cloud's order (k-NN covariance only)
    float* covs_sorted;   // nullable: SoA [6][n] covariance output in grid order
    int64_t off;          // first index of the cloud in the concatenation and in grid order
    int64_t n;
    float h, inv_h;       // the cloud's cell size
};

struct SegSet {
    Seg one;              // the cloud when count == 1
    const Seg* many;      // device array of `count` clouds when count > 1
    int count;

    __device__ __forceinline__ Seg get(int p) const { return count == 1 ? one : many[p]; }
    // cloud of grid-order position s: the top byte of its sorted cell key
    __device__ __forceinline__ int of_key(uint32_t key) const { return count == 1 ? 0 : (int)(key >> 24); }
    // cloud holding concatenated (or grid-order) index i
    __device__ __forceinline__ int find(int64_t i) const {
        if (count == 1) return 0;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (many[mid].off <= i) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
};

// at most 255 clouds per segmented grid: cloud 255 could form the key 0xFFFFFFFF, the empty-slot marker
constexpr int kMaxSegments = 255;

// Cell keys of the concatenated clouds (cloud index << 24 | cell key) with
// their concatenated indices as values.
hipError_t launch_cell_keys(const SegSet& S, int64_t total, uint32_t* keys, uint32_t* vals, int* err,
                            hipStream_t s);
// Fill the hash table with empty entries.
hipError_t launch_table_clear(uint4* table, uint32_t cap, hipStream_t s);
// Gather points into cell order (float4 x, y, z, index within the cloud) and
// insert the cell runs.
hipError_t launch_table_build(const uint32_t* skeys, const uint32_t* svals, int64_t total, const SegSet& S,
                              float4* spts, uint4* table, uint32_t mask, hipStream_t s);

// A built grid: cell-sorted points and the cell table.
struct GridView {
    const float4* spts;   // [n] x, y, z, original index (bits)
    const uint32_t* skeys;   // [n] sorted cell keys (cloud index in the top byte when segmented); may be null for maps
    const uint4* table;   // [mask+1] {key, start, count, -}
    uint32_t mask;
    int32_t n;
    float h, inv_h;
};

// Self k-NN + covariance + regularisation of every cloud of the grid; each
// cloud's Seg names its outputs.  raw: device float scratch [6 * total] (per
// cloud SoA [6][n] at 6 * off; may alias the clouds' covs_sorted, which the
// last pass rewrites in place).  work: device int32 [2 + 2 * total] with
// work[0] = work[1] = 0 set by the caller (retry and overflow lists).
hipError_t launch_knn_cov(const GridView& g, const SegSet& S, int k, int mode, float eps, float* raw, int32_t* work,
                          hipStream_t s);
constexpr int64_t knn_cov_work_ints(int64_t total) { return 2 + 2 * total; }
// k-NN of arbitrary queries (SoA [3][nq]) in a one-cloud grid; idx/d2
// row-major [nq][k]; overflow [1 + nq].
hipError_t launch_knn_query(const GridView& g, const Seg& cloud, const float* q, int64_t nq, int k, float r_max,
                            int32_t* idx, float* d2, int32_t* overflow, hipStream_t s);
struct KthJob {
    const float* xyz;   // SoA [3][n]
    int64_t n, step;    // cloud size; only every step-th point is scanned
    int j, ns;          // neighbour rank; number of strided samples (<= samples)
};
// For every job, the j-th neighbour distance of ns strided samples, into
// out[job * samples + sample]; jobs is a device array of njobs entries.
hipError_t launch_kth_distance(const KthJob* jobs, int njobs, int samples, float* out, hipStream_t s);
// Map Gaussians: regularise covariances and store them in cell order (2 x float4 each).
hipError_t launch_map_covs(const uint32_t* svals, int64_t m, const float* covs, int64_t stride, int mode,
                           float eps, float4* scov, int* err, hipStream_t s);

// Device state of one registration.
struct __align__(256) RegState {
    double pose[16];
    double H[21];
    double b[6];
    double cost;
    double n_inl;
    double conv_rot, conv_trans;
    float Rf[9];
    float tf[3];
    int32_t iters;
    int32_t max_it;
    int32_t done;
    int32_t status;
    int32_t converged;
    int32_t acc;
};

// The scalar settings of a registration state (gicp_register_dev).
struct StateInit {
    double conv_rot, conv_trans;
    int32_t max_it, acc;
};

struct MapView {
    GridView g;
    const float4* scov;   // [m][2]: {xx, xy, xz, yy}, {yz, zz, 0, 0}
    float r_max, r_max2;
};

// One registration problem of the work-queue kernel.
struct ProbDev {
    const float* src;     // SoA [3][n]
    const float* scov;    // SoA [6][n]
    const float4* ssrc;   // nullable: the source in grid-cell order (x, y, z, original index)
    const float* sscov;   // with ssrc: the source covariances in that order, SoA [6][n]
    int32_t* nn_prev;     // [n] map position matched by each point at its last search (-1: none)
    float4* nn_cache;     // [n] query point of that search and the radius it certified
    int64_t n;
    int32_t nchunks;      // ceil(n / kChunk)
    int32_t part0;        // first partial / item slot of the problem
    int32_t fresh;        // 1: search every correspondence afresh (no reuse of the previous match, no hint)
    int32_t pad_;
    MapView map;
    RegState* st;
};

struct QueueDev {
    uint32_t head;        // next ticket
    uint32_t tail;        // item slots reserved so far
    uint32_t remaining;   // problems not yet retired
    uint32_t error;       // set when a bounded wait ran out
    uint32_t cap;         // item ring capacity
    uint32_t pad[3];
};

constexpr int kGroup = 4;            // lanes that search the correspondence of one point together
constexpr int kChunk = kBlock / kGroup;   // source points per work item (64)
constexpr int kChunkBits = 20;       // item = ((problem << 20) | chunk) + 1
constexpr int kMaxProblems = 4096;

int gn_blocks(int64_t n);
hipError_t launch_chunk_map(const ProbDev* probs, int nprob, int32_t* chunk_prob, hipStream_t s);
// Lanes per source point in the linearisation (gicp_params.lanes 0 picks
// the form's default; 2 and 4 are built): batched launches, the work queue,
// sequential tracking.
constexpr int kBatchLanes = 2, kQueueLanes = 4, kTrackLanes = 4;
hipError_t launch_gn_iteration_batch(const ProbDev* probs, int nprob, int32_t* chunk_prob, int64_t chunks,
                                     double* partials, int acc, int lanes, bool linearize, bool solve, hipStream_t s);
int gn_queue_workers(int acc, int lanes);
hipError_t launch_gn_queue(const ProbDev* probs, int nprob, QueueDev* q, uint32_t* items, uint32_t cap,
                           uint32_t first, uint32_t* arrive, double* partials, int workers, int acc, int lanes,
                           hipStream_t s);
hipError_t launch_gn_linearize(const ProbDev& pd, double* partials, int nblocks, int acc, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_gn_solve(const double* partials, int nblocks, RegState* st, hipStream_t s);
// Device-resident registration: descriptor and state from kernel arguments
// and the device initial pose; results (H full symmetric [36]) to device
// outputs, the status NONFINITE when the context's error word holds it.
hipError_t launch_state_init(const ProbDev& pd, ProbDev* dst, const StateInit& si, const double* init, RegState* st,
                             hipStream_t s);
hipError_t launch_state_out(const RegState* st, const int* err, double* pose, double* H, double* b,
                            gicp_stats* stats, hipStream_t s);
// Sequential tracking (gicp_track): the next problem's chunk map and predicted
// pose, then its iterations over a grid of the largest problem's chunks.
hipError_t launch_track_begin(const ProbDev* probs, int nprob, int32_t* counter, int32_t* chunk_prob, int64_t grid,
                              int motion, hipStream_t s);
// One iteration slot of sequential tracking (one launch: linearisation,
// reduction and solve).  ctl: device int32[3] (the current problem for
// launches of parity 0 and 1, slots run; zero before the first slot); parity:
// the launch's index modulo 2; progress: host-mapped int32[2] receiving
// (problems finished, slots run); sync: slot_sync_bytes() of device memory,
// zero before the first slot (each slot leaves it zero).
hipError_t launch_track_slot(const ProbDev* probs, int nprob, int32_t* ctl, int parity, int64_t grid, double* partials,
                             int acc, int lanes, int motion, int32_t* progress, void* sync, hipStream_t s);
size_t slot_sync_bytes();
hipError_t launch_gn_track_iteration(const ProbDev* probs, int32_t* chunk_prob, int64_t grid, double* partials, int acc,
                                     int lanes, bool linearize, bool solve, hipStream_t s);

// Incremental map update (grid.hip): merge the map's sorted run (okeys,
// opts, ocov; m_old) with new points sorted on their own (nkeys, nvals into
// means [3][m_new], regularised covariances ncov in that sorted order) into
// (keys, pts, cov) of m_old + m_new entries; equal keys keep old points first.
hipError_t launch_map_merge(const uint32_t* okeys, const float4* opts, const float4* ocov, int64_t m_old,
                            const uint32_t* nkeys, const uint32_t* nvals, const float* means, const float4* ncov,
                            int64_t m_new, uint32_t* keys, float4* pts, float4* cov, hipStream_t s);
// Cell table from sorted keys (points already in cell order); table cleared by the caller.
hipError_t launch_table_runs(const uint32_t* skeys, int64_t total, uint4* table, uint32_t mask, hipStream_t s);
// Exclusive scan of 0/1 flags; *total (device) receives the sum.
size_t flag_scan_scratch(int64_t n);
hipError_t launch_flag_scan(const uint32_t* flags, int64_t n, uint32_t* out, uint32_t* total, void* scratch,
                            hipStream_t s);

// Keyframe Gaussians (gn.hip).
struct Pose32 {
    float R[9], t[3];
};
struct Pose64 {
    double R[9], t[3];
};
// keep[i] = 1 when R x_i + t has no map mean within m.r_max.
hipError_t launch_overlap(const MapView& m, const float* src, int64_t n, const Pose32& T, uint32_t* keep,
                          hipStream_t s);
// Correspondence search of the batched linearisation for arbitrary queries
// (map frame, SoA [3][nq]); hints are map indices (inv: index -> sorted
// position, required with hints); radius nullable.
// lanes: 2 (the search of the batched launches) or 4, 8, 16 (the wide search).
hipError_t launch_map_nearest(const MapView& m, const float* q, int64_t nq, const int32_t* hints, const int32_t* inv,
                              int32_t* idx, float* d2, float* radius, int lanes, hipStream_t s);
// inv[index of the point at sorted position j] = j for the m points of a map.
hipError_t launch_map_inverse(const float4* spts, int64_t m, int32_t* inv, hipStream_t s);
// Kept points -> map-frame means and scale-aligned, rotated covariances at
// out[pos[i]] (SoA with stride n).
hipError_t launch_keyframe_gaussians(const float* src, const float* covs, int64_t n, const uint32_t* keep,
                                     const uint32_t* pos, const Pose64& T, double two_p, float* out_means,
                                     float* out_covs, hipStream_t s);

// Depth image -> voxel centroids (depth.hip).  pts [3][W*H], vox [3][W*H],
// bounds [8] ints.
hipError_t launch_depth_points(const float* depth, int W, int H, float fx, float fy, float cx, float cy, float voxel,
                               float max_depth, float* pts, int* vox, int* bounds, hipStream_t s);
hipError_t launch_voxel_keys(const int* vox, int64_t n, const int* bounds, uint32_t dy, uint32_t dz, uint32_t* keys,
                             uint32_t* vals, hipStream_t s);
hipError_t launch_voxel_starts(const uint32_t* skeys, int64_t n, uint32_t* flags, hipStream_t s);
hipError_t launch_voxel_centroids(const uint32_t* skeys, const uint32_t* svals, int64_t n, const uint32_t* flags,
                                  const uint32_t* pos, const float* pts, float* out, int64_t m, hipStream_t s);

// Warm-start network (mlp.hip).
hipError_t launch_mlp_init(uint64_t seed, float* params, float* m, float* v, uint16_t* wb, hipStream_t s);
hipError_t launch_mlp_fragments(const float* params, uint16_t* wb, hipStream_t s);
hipError_t launch_mlp_pack(int B, const gicp_mlp_pair* pairs, uint16_t* X, double* centres, int* err,
                           hipStream_t s);
// pmax / parg: scratch [B][mlp_splits()][256]
hipError_t launch_mlp_forward(int B, const uint16_t* X, const float* params, const uint16_t* wb, float* pmax,
                              int* parg, const double* centres, float* y, float* cache, double* poses, hipStream_t s);
// gpair: scratch [B][GICP_MLP_PARAMS]; lpair: scratch [B]
hipError_t launch_mlp_backward(int B, const uint16_t* X, const float* params, const float* cache, const float* y,
                               const float* ystar, float* gpair, float* lpair, float* grad, float* loss,
                               hipStream_t s);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr, uint16_t* wb,
                           hipStream_t s);
int mlp_splits();

}  // namespace gicp
