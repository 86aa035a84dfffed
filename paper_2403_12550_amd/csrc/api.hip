// Host runtime and C ABI of libgicp.so: context and growable workspace, grid
// builds, map handles and the Gauss-Newton driver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

using namespace gicp;

namespace {

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

struct GridBufs {
    Buf keys_a, vals_a, keys_b, vals_b, scratch, spts, table;
    const uint32_t* sorted_vals = nullptr;   // original indices in cell order (last build)
};

struct HipError {
    hipError_t e;
};

inline void check(hipError_t e) {
    if (e != hipSuccess) throw HipError{e};
}

// Grow-only device buffer: reallocated (contents dropped) when too small.
template <typename T>
T* ensure(Buf& b, size_t count) {
    const size_t need = std::max<size_t>(count * sizeof(T), 256);
    if (need > b.cap) {
        if (b.p) check(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
        const size_t want = need + need / 4;
        check(hipMalloc(&b.p, want));
        b.cap = want;
    }
    return static_cast<T*>(b.p);
}

void release(Buf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

uint32_t table_capacity(int64_t n) {
    uint64_t c = 1024;
    while (c < (uint64_t)(2 * n)) c <<= 1;
    return (uint32_t)c;
}

}  // namespace

struct ProfMark {
    int group;
    hipEvent_t a, b;
    double units;
    int iter;    // Gauss-Newton iteration index (-1: not an iteration)
    int frame;   // tracked frame (gicp_track), else -1
};

// Fixed workspace of gicp_covariances_noalloc: one copy per GPU the library
// runs on, held until the process ends.  Host code never uses this name as an
// address; it uses the device address looked up once per device below.
constexpr size_t kNoAllocBytes = 13107200;   // 12.5 MiB: the layout for GICP_NOALLOC_MAX_POINTS fits
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

struct gicp_ctx {
    int device = 0;
    void* noalloc = nullptr;         // device address of `scratch` on this context's device
    int* d_err = nullptr;
    int* h_err = nullptr;
    GridBufs grid;
    Buf covs, partials, kth, ssrc, sscov, nn_prev, nn_cache, overflow;
    RegState* d_state = nullptr;     // [state_cap]
    RegState* h_state = nullptr;     // pinned [state_cap]
    ProbDev* d_probs = nullptr;      // [state_cap]
    ProbDev* h_probs = nullptr;      // pinned [state_cap]
    int state_cap = 0;
    QueueDev* d_queue = nullptr;
    Buf items, arrive, chunk_prob, track_counter, slot_sync;
    RegState* dev_state = nullptr;   // gicp_register_dev: its own state and descriptor, allocated once
    ProbDev* dev_probs = nullptr;    // (never reallocated, so graphs that capture the call stay valid)
    int32_t* h_progress = nullptr;   // host-mapped progress of the tracking slots: problems done, slots run
    int32_t* d_progress = nullptr;   // its device address
    double slot_work = 0.0;          // slots of the last tracking call that did work
    int queue_workers[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // per precision and lanes (2, 4)
    float* h_kth = nullptr;
    int h_kth_cap = 0;   // clouds the pinned estimate buffer holds
    KthJob* h_jobs = nullptr;   // pinned descriptors of the estimate launch
    int h_jobs_cap = 0;
    Buf kth_jobs;
    Seg* h_segs = nullptr;           // pinned [kMaxSegments]
    Buf segs;
    // warm-start network workspaces
    gicp_mlp_pair* h_pairs = nullptr;   // pinned [GICP_MLP_MAX_BATCH] staging of pair descriptors
    hipEvent_t pairs_ev = nullptr;      // recorded after the last upload of h_pairs
    bool pairs_pending = false;
    Buf mlp_pairs, mlp_pmax, mlp_parg, mlp_gpair, mlp_lpair;
    // depth, keyframe and map-insert workspaces
    Buf dep_pts, dep_vox, dep_flags, dep_pos, dep_scan, dep_misc, ins_cov;
    // graph-captured Gauss-Newton iterations, keyed by batch shape and workspace
    struct GraphEntry {
        int kind;   // 0: batched iterations, 1: one tracked frame
        int nprob, max_it, acc, motion, lanes;
        int64_t chunks;
        const void *probs, *chunk_prob, *part, *counter;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;
    double queue_units = 0.0;        // source points x iterations of the last queue launch
    std::vector<double> iter_units;  // per iteration: source points of the problems still running
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<ProfMark> marks;
    int64_t launches[GICP_PROF_GROUPS] = {0, 0, 0, 0};
    double ms[GICP_PROF_GROUPS] = {0, 0, 0, 0};
    double units[GICP_PROF_GROUPS] = {0, 0, 0, 0};
};

struct gicp_map {
    int device = 0;
    int64_t m = 0;
    int64_t cap = 0;                 // points the arrays below hold
    float h = 0.f;
    uint32_t mask = 0;
    int reg_mode = GICP_REG_NONE;    // applied to inserted covariances as at the build
    float eps = 1e-3f;
    float4* spts = nullptr;          // [cap] cell-sorted x, y, z, index
    uint4* table = nullptr;          // [mask + 1]
    float4* scov = nullptr;          // [2 cap] regularised covariances in cell order
    uint32_t* keys = nullptr;        // [cap] cell keys in cell order
    float4* spts2 = nullptr;         // spare arrays of the same capacity (merge target of gicp_map_insert)
    float4* scov2 = nullptr;
    uint32_t* keys2 = nullptr;
    int32_t* inv = nullptr;          // [m] index -> sorted position, built on demand (hinted queries)
    bool inv_ok = false;
};

namespace {

int status_of(const HipError& e) { return e.e == hipErrorOutOfMemory ? GICP_E_OOM : GICP_E_HIP; }

hipEvent_t next_event(gicp_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        check(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Opens a timed region on stream s (no-op unless profiling); returns its mark index.
int prof_open(gicp_ctx* c, int group, double units, int iter, hipStream_t s, int frame = -1) {
    if (!c->prof) return -1;
    ProfMark m{group, next_event(c), next_event(c), units, iter, frame};
    check(hipEventRecord(m.a, s));
    c->marks.push_back(m);
    return (int)c->marks.size() - 1;
}

void prof_close(gicp_ctx* c, int mark, hipStream_t s) {
    if (mark < 0) return;
    check(hipEventRecord(c->marks[mark].b, s));
}

// After a synchronisation: accumulate the marks; iterations at or beyond
// `iters_done` were launched but returned at once (converged) and are skipped.
void prof_collect(gicp_ctx* c, int iters_done) {
    for (const ProfMark& m : c->marks) {
        if (m.frame == -5) {
            // a tracking slot (iter = slot index): the first slot_work slots did
            // work, the rest found every problem finished
            if (m.iter >= c->slot_work) continue;
            float ms = 0.f;
            check(hipEventSynchronize(m.b));
            check(hipEventElapsedTime(&ms, m.a, m.b));
            c->launches[m.group] += 1;
            c->ms[m.group] += ms;
            c->units[m.group] += m.group == GICP_PROF_LINEARIZE ? c->queue_units / c->slot_work : 1.0;
            continue;
        }
        if (m.frame >= 0) {
            // a tracked frame: its launches after convergence did no work; a
            // graph replay (iter -2) covers all of the frame's iterations
            const int it = c->h_state[m.frame].iters;
            if (m.iter >= 0 && m.iter >= it) continue;
            float ms = 0.f;
            check(hipEventSynchronize(m.b));
            check(hipEventElapsedTime(&ms, m.a, m.b));
            c->launches[m.group] += 1;
            c->ms[m.group] += ms;
            c->units[m.group] += m.iter == -2 ? m.units * it : m.units;
            continue;
        }
        if (m.iter >= 0 && m.iter >= iters_done) continue;
        float ms = 0.f;
        check(hipEventSynchronize(m.b));
        check(hipEventElapsedTime(&ms, m.a, m.b));
        c->launches[m.group] += 1;
        c->ms[m.group] += ms;
        double u = m.units;
        if (m.iter == -2) u = c->queue_units;
        else if (m.iter >= 0 && m.group == GICP_PROF_LINEARIZE && m.iter < (int)c->iter_units.size())
            u = c->iter_units[m.iter];
        c->units[m.group] += u;
    }
    c->marks.clear();
    c->ev_used = 0;
}

void reserve_grid(GridBufs& gb, int64_t n) {
    ensure<uint32_t>(gb.keys_a, n);
    ensure<uint32_t>(gb.vals_a, n);
    ensure<uint32_t>(gb.keys_b, n);
    ensure<uint32_t>(gb.vals_b, n);
    ensure<uint8_t>(gb.scratch, radix_scratch_bytes(n));
    ensure<float4>(gb.spts, n);
    ensure<uint4>(gb.table, table_capacity(n));
}

// Builds the cell grid of the clouds of S (total points) into `gb`: keys,
// radix sort (3 passes for one cloud, 4 when the cloud index is part of the
// key), cell table and the points gathered into grid order.
// Device buffers of one grid build (keys and values ping-pong pairs, radix
// scratch, gathered points, table of `cap` entries).
struct GridPtrs {
    uint32_t *ka, *va, *kb, *vb;
    void* scr;
    float4* spts;
    uint4* table;
    uint32_t cap;
};

GridView build_grid_into(gicp_ctx* ctx, const GridPtrs& b, const SegSet& S, int64_t total, hipStream_t s,
                         uint32_t* keys_out, const uint32_t** sorted_vals, bool timed) {
    const int pm = timed ? prof_open(ctx, GICP_PROF_GRID, (double)total, -1, s) : -1;
    check(launch_cell_keys(S, total, b.ka, b.va, ctx->d_err, s));
    uint32_t *ks = nullptr, *vs = nullptr;
    check(radix_sort(b.ka, b.va, b.kb, b.vb, total, S.count > 1 ? 4 : 3, b.scr, s, &ks, &vs));
    check(launch_table_clear(b.table, b.cap, s));
    check(launch_table_build(ks, vs, total, S, b.spts, b.table, b.cap - 1, s));
    if (keys_out) check(hipMemcpyAsync(keys_out, ks, total * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    prof_close(ctx, pm, s);
    if (sorted_vals) *sorted_vals = vs;
    GridView g;
    g.spts = b.spts;
    g.skeys = ks;
    g.table = b.table;
    g.mask = b.cap - 1;
    g.n = (int32_t)total;
    g.h = S.one.h;
    g.inv_h = S.one.inv_h;
    return g;
}

GridView build_grid(gicp_ctx* ctx, GridBufs& gb, const SegSet& S, int64_t total, hipStream_t s,
                    float4* spts_out = nullptr, uint4* table_out = nullptr, uint32_t* keys_out = nullptr) {
    GridPtrs b;
    b.ka = ensure<uint32_t>(gb.keys_a, total);
    b.va = ensure<uint32_t>(gb.vals_a, total);
    b.kb = ensure<uint32_t>(gb.keys_b, total);
    b.vb = ensure<uint32_t>(gb.vals_b, total);
    b.scr = ensure<uint8_t>(gb.scratch, radix_scratch_bytes(total));
    b.cap = table_capacity(total);
    b.spts = spts_out ? spts_out : ensure<float4>(gb.spts, total);
    b.table = table_out ? table_out : ensure<uint4>(gb.table, b.cap);
    return build_grid_into(ctx, b, S, total, s, keys_out, &gb.sorted_vals, true);
}

SegSet one_cloud(const float* xyz, int64_t n, float h, float* covs = nullptr, float* covs_sorted = nullptr) {
    SegSet S;
    S.one.xyz = xyz;
    S.one.covs = covs;
    S.one.covs_sorted = covs_sorted;
    S.one.off = 0;
    S.one.n = n;
    S.one.h = h;
    S.one.inv_h = 1.0f / h;
    S.many = nullptr;
    S.count = 1;
    return S;
}

// Grid cell size for a k-NN search: 1.2 x the 75th percentile of the k-th
// neighbour distance of 256 strided sample points.  Above kEstimateScan
// points the distances are taken among every step-th point only, at the
// neighbour rank that covers the same area on a surface (rank k / step), so
// the estimate costs a fixed amount of work.  All clouds are estimated
// behind one synchronisation.
constexpr int kEstimateSamples = 256;
constexpr int64_t kEstimateScan = 16384;

// (dbuf / djobs: device buffers of count * kEstimateSamples floats and count
// descriptors to use instead of the context's workspace)
void estimate_cells(gicp_ctx* ctx, int count, const float* const* xyz, const int64_t* n, int k, hipStream_t s,
                    float* cells, float* dbuf = nullptr, KthJob* djobs_in = nullptr) {
    if (count <= 0) return;
    float* d = dbuf ? dbuf : ensure<float>(ctx->kth, (int64_t)count * kEstimateSamples);
    if (ctx->h_kth_cap < count) {
        if (ctx->h_kth) check(hipHostFree(ctx->h_kth));
        ctx->h_kth = nullptr;
        ctx->h_kth_cap = 0;
        check(hipHostMalloc(&ctx->h_kth, (size_t)count * kEstimateSamples * sizeof(float)));
        ctx->h_kth_cap = count;
    }
    // one launch for every cloud (the job descriptors go through pinned memory)
    if (ctx->h_jobs_cap < count) {
        if (ctx->h_jobs) check(hipHostFree(ctx->h_jobs));
        ctx->h_jobs = nullptr;
        ctx->h_jobs_cap = 0;
        check(hipHostMalloc(&ctx->h_jobs, (size_t)count * sizeof(KthJob)));
        ctx->h_jobs_cap = count;
    }
    std::vector<int> ns(count);
    for (int i = 0; i < count; ++i) {
        ns[i] = (int)std::min<int64_t>(kEstimateSamples, n[i]);
        const int64_t step = std::max<int64_t>(1, n[i] / kEstimateScan);
        const int j = std::max(1, (int)std::lround((double)std::min<int64_t>(k, n[i]) / (double)step));
        ctx->h_jobs[i] = KthJob{xyz[i], n[i], step, j, ns[i]};
    }
    KthJob* djobs = djobs_in ? djobs_in : ensure<KthJob>(ctx->kth_jobs, count);
    check(hipMemcpyAsync(djobs, ctx->h_jobs, count * sizeof(KthJob), hipMemcpyHostToDevice, s));
    check(launch_kth_distance(djobs, count, kEstimateSamples, d, s));
    check(hipMemcpyAsync(ctx->h_kth, d, (size_t)count * kEstimateSamples * sizeof(float), hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {
        std::vector<float> v(ctx->h_kth + (int64_t)i * kEstimateSamples,
                             ctx->h_kth + (int64_t)i * kEstimateSamples + ns[i]);
        std::sort(v.begin(), v.end());
        float c = v[(size_t)(0.75 * (ns[i] - 1))] * 1.2f;
        if (!(c > 1e-6f) || !std::isfinite(c)) c = 1e-3f;
        cells[i] = c;
    }
}

float estimate_cell(gicp_ctx* ctx, const float* xyz, int64_t n, int k, hipStream_t s) {
    float c = 0.f;
    estimate_cells(ctx, 1, &xyz, &n, k, s, &c);
    return c;
}

void ensure_states(gicp_ctx* c, int n) {
    if (n <= c->state_cap) return;
    const int cap = std::max(n, 2 * c->state_cap);
    if (c->d_state) check(hipFree(c->d_state));
    if (c->h_state) check(hipHostFree(c->h_state));
    if (c->d_probs) check(hipFree(c->d_probs));
    if (c->h_probs) check(hipHostFree(c->h_probs));
    c->d_state = nullptr;
    c->h_state = nullptr;
    c->d_probs = nullptr;
    c->h_probs = nullptr;
    c->state_cap = 0;
    check(hipMalloc(&c->d_state, cap * sizeof(RegState)));
    check(hipHostMalloc(&c->h_state, cap * sizeof(RegState)));
    check(hipMalloc(&c->d_probs, cap * sizeof(ProbDev)));
    check(hipHostMalloc(&c->h_probs, cap * sizeof(ProbDev)));
    c->state_cap = cap;
}

// neighbour counts: any k in [1, 64] for a search; at least 3 for a
// covariance (with fewer neighbours it has rank 0 or 1, and a regularised
// form would fix an arbitrary direction)
bool valid_k(int k) { return k >= 1 && k <= 64; }

// Device address of `scratch` on `device` (current), looked up on the first
// context created on that device and kept for the life of the process.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) throw HipError{hipErrorInvalidDevice};
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[device] = p;
    }
    return g_noalloc_ptr[device];
}

// Byte offsets of the workspace of one gicp_covariances call on n points
// inside the fixed array (each region 256-byte aligned).
struct NoAllocLayout {
    size_t ka, va, kb, vb, scr, spts, table, raw, work, kth, jobs, end;
    uint32_t cap;
};

NoAllocLayout noalloc_layout(int64_t n) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    NoAllocLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += up(bytes);
        return at;
    };
    L.cap = table_capacity(n);
    L.ka = take(n * sizeof(uint32_t));
    L.va = take(n * sizeof(uint32_t));
    L.kb = take(n * sizeof(uint32_t));
    L.vb = take(n * sizeof(uint32_t));
    L.scr = take(radix_scratch_bytes(n));
    L.spts = take(n * sizeof(float4));
    L.table = take((size_t)L.cap * sizeof(uint4));
    L.raw = take(6 * n * sizeof(float));
    L.work = take(knn_cov_work_ints(n) * sizeof(int32_t));
    L.kth = take(kEstimateSamples * sizeof(float));
    L.jobs = take(sizeof(KthJob));
    L.end = o;
    return L;
}

// Cell estimate of one cloud (as estimate_cell) with its device buffers
// given and host storage on the stack: no allocation.  Synchronises.
float estimate_cell_fixed(gicp_ctx* ctx, const float* xyz, int64_t n, int k, hipStream_t s, float* d, KthJob* djob) {
    const int ns = (int)std::min<int64_t>(kEstimateSamples, n);
    const int64_t step = std::max<int64_t>(1, n / kEstimateScan);
    const int j = std::max(1, (int)std::lround((double)std::min<int64_t>(k, n) / (double)step));
    ctx->h_jobs[0] = KthJob{xyz, n, step, j, ns};
    check(hipMemcpyAsync(djob, ctx->h_jobs, sizeof(KthJob), hipMemcpyHostToDevice, s));
    check(launch_kth_distance(djob, 1, kEstimateSamples, d, s));
    check(hipMemcpyAsync(ctx->h_kth, d, kEstimateSamples * sizeof(float), hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    float v[kEstimateSamples];
    std::memcpy(v, ctx->h_kth, ns * sizeof(float));
    std::sort(v, v + ns);
    float c = v[(size_t)(0.75 * (ns - 1))] * 1.2f;
    if (!(c > 1e-6f) || !std::isfinite(c)) c = 1e-3f;
    return c;
}
bool valid_cov_k(int k) { return k >= 3 && k <= 64; }
bool valid_mode(int m) { return m == GICP_REG_NONE || m == GICP_REG_PLANE || m == GICP_REG_ELLIPSE; }

}  // namespace

extern "C" {

void gicp_params_default(gicp_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->k = 20;
    p->eps = 1e-3f;
    p->r_max = 0.1f;
    p->max_it = 30;
    p->conv_rot = 0.0;
    p->conv_trans = 0.0;
    p->reg_mode = GICP_REG_PLANE;
    p->cell_src = 0.f;
    p->precision = GICP_ACC_TWOSUM;
}

const char* gicp_version(void) { return "gicp-gfx950 0.1"; }

const char* gicp_strerror(int st) {
    switch (st) {
        case GICP_OK: return "ok";
        case GICP_E_ARG: return "invalid argument";
        case GICP_E_NONFINITE: return "non-finite input";
        case GICP_E_NO_CORR: return "fewer than 6 correspondences";
        case GICP_E_DEGENERATE: return "degenerate system (Cholesky failed)";
        case GICP_E_OOM: return "device out of memory";
        case GICP_E_HIP: return "HIP runtime error";
        case GICP_E_INEXACT: return "k-NN not provably exact";
        case GICP_E_TOO_LARGE: return "input exceeds the fixed workspace of the no-allocation entry point";
        default: return "unknown status";
    }
}

int gicp_create(gicp_ctx** out, int device) {
    if (!out) return GICP_E_ARG;
    *out = nullptr;
    gicp_ctx* c = new (std::nothrow) gicp_ctx();
    if (!c) return GICP_E_OOM;
    try {
        c->device = device;
        check(hipSetDevice(device));
        check(hipMalloc(&c->d_err, 256));
        check(hipMemset(c->d_err, 0, 256));
        check(hipMalloc(&c->d_queue, sizeof(QueueDev)));
        check(hipMalloc(&c->dev_state, sizeof(RegState)));
        check(hipMalloc(&c->dev_probs, sizeof(ProbDev)));
        check(hipHostMalloc(&c->h_err, 256));
        check(hipHostMalloc(&c->h_kth, kEstimateSamples * sizeof(float)));
        c->h_kth_cap = 1;
        check(hipHostMalloc(&c->h_jobs, sizeof(KthJob)));
        c->h_jobs_cap = 1;
        c->noalloc = noalloc_scratch(device);
        if (noalloc_layout(GICP_NOALLOC_MAX_POINTS).end > kNoAllocBytes) throw HipError{hipErrorInvalidValue};
        check(hipHostMalloc(&c->h_segs, kMaxSegments * sizeof(Seg)));
        *out = c;
        return GICP_OK;
    } catch (const HipError& e) {
        gicp_destroy(c);
        return status_of(e);
    }
}

int gicp_destroy(gicp_ctx* c) {
    if (!c) return GICP_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (Buf* b : {&c->grid.keys_a, &c->grid.vals_a, &c->grid.keys_b, &c->grid.vals_b, &c->grid.scratch,
                   &c->grid.spts, &c->grid.table, &c->covs, &c->partials, &c->kth, &c->ssrc, &c->sscov,
                   &c->nn_prev, &c->nn_cache, &c->overflow, &c->mlp_pairs, &c->mlp_pmax, &c->mlp_parg, &c->mlp_gpair,
                   &c->mlp_lpair, &c->dep_pts, &c->dep_vox, &c->dep_flags, &c->dep_pos, &c->dep_scan, &c->dep_misc,
                   &c->ins_cov, &c->kth_jobs, &c->track_counter, &c->slot_sync})
        release(*b);
    for (auto& ge : c->graphs) (void)hipGraphExecDestroy(ge.exec);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->h_pairs) (void)hipHostFree(c->h_pairs);
    if (c->h_jobs) (void)hipHostFree(c->h_jobs);
    if (c->h_progress) (void)hipHostFree(c->h_progress);
    if (c->pairs_ev) (void)hipEventDestroy(c->pairs_ev);
    if (c->d_err) (void)hipFree(c->d_err);
    if (c->d_state) (void)hipFree(c->d_state);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->d_probs) (void)hipFree(c->d_probs);
    if (c->h_probs) (void)hipHostFree(c->h_probs);
    if (c->d_queue) (void)hipFree(c->d_queue);
    if (c->dev_state) (void)hipFree(c->dev_state);
    if (c->dev_probs) (void)hipFree(c->dev_probs);
    release(c->items);
    release(c->arrive);
    release(c->chunk_prob);
    if (c->h_err) (void)hipHostFree(c->h_err);
    if (c->h_kth) (void)hipHostFree(c->h_kth);
    if (c->h_segs) (void)hipHostFree(c->h_segs);
    release(c->segs);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return GICP_OK;
}

int gicp_sync_status(gicp_ctx* c, void* stream) {
    if (!c) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        check(hipMemcpyAsync(c->h_err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        if (c->prof) prof_collect(c, 0);
        const int e = *c->h_err;
        if (e) check(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
        check(hipStreamSynchronize(s));
        if (e & kErrNonFinite) return GICP_E_NONFINITE;
        if (e & kErrInexact) return GICP_E_INEXACT;
        if (e & kErrIndex) return GICP_E_ARG;
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_estimate_cell(gicp_ctx* c, const float* pts, int64_t n, int k, float* cell, void* stream) {
    if (!c || !pts || !cell || n < 1 || !valid_k(k)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        *cell = estimate_cell(c, pts, n, k, (hipStream_t)stream);
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_knn(gicp_ctx* c, const float* pts, int64_t n, const float* queries, int64_t nq, int k, float cell,
             float r_max, int32_t* idx, float* d2, void* stream) {
    if (!c || !pts || n < 1 || nq < 0 || !valid_k(k) || n >= (1ll << 31)) return GICP_E_ARG;
    if (nq > 0 && (!queries || !idx || !d2)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const float h = cell > 0.f ? cell : estimate_cell(c, pts, n, k, s);
        const SegSet S = one_cloud(pts, n, h);
        GridView g = build_grid(c, c->grid, S, n, s);
        int32_t* ovf = ensure<int32_t>(c->overflow, nq + 1);
        check(launch_fill_i32(ovf, 1, 0, s));
        check(launch_knn_query(g, S.one, queries, nq, k, r_max, idx, d2, ovf, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_covariances(gicp_ctx* c, const float* pts, int64_t n, int k, float cell, int reg_mode, float eps,
                     float* covs, void* stream) {
    if (!c || !pts || !covs || !valid_cov_k(k) || n < k || !valid_mode(reg_mode) || n >= (1ll << 31))
        return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const float h = cell > 0.f ? cell : estimate_cell(c, pts, n, k, s);
        const SegSet S = one_cloud(pts, n, h, covs);
        GridView g = build_grid(c, c->grid, S, n, s);
        const int pm = prof_open(c, GICP_PROF_KNN_COV, (double)n, -1, s);
        int32_t* work = ensure<int32_t>(c->overflow, knn_cov_work_ints(n));
        float* raw = ensure<float>(c->sscov, 6 * n);
        check(launch_fill_i32(work, 2, 0, s));
        check(launch_knn_cov(g, S, k, reg_mode, eps, raw, work, s));
        prof_close(c, pm, s);
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_covariances_noalloc(gicp_ctx* c, const float* pts, int64_t n, int k, float cell, int reg_mode, float eps,
                             float* covs, void* stream) {
    if (!c || !pts || !covs || !valid_cov_k(k) || n < k || !valid_mode(reg_mode)) return GICP_E_ARG;
    if (n > GICP_NOALLOC_MAX_POINTS) return GICP_E_TOO_LARGE;
    if (!c->noalloc) return GICP_E_HIP;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const NoAllocLayout L = noalloc_layout(n);
        uint8_t* base = static_cast<uint8_t*>(c->noalloc);
        const float h = cell > 0.f ? cell
                                   : estimate_cell_fixed(c, pts, n, k, s, reinterpret_cast<float*>(base + L.kth),
                                                         reinterpret_cast<KthJob*>(base + L.jobs));
        const SegSet S = one_cloud(pts, n, h, covs);
        GridPtrs b;
        b.ka = reinterpret_cast<uint32_t*>(base + L.ka);
        b.va = reinterpret_cast<uint32_t*>(base + L.va);
        b.kb = reinterpret_cast<uint32_t*>(base + L.kb);
        b.vb = reinterpret_cast<uint32_t*>(base + L.vb);
        b.scr = base + L.scr;
        b.spts = reinterpret_cast<float4*>(base + L.spts);
        b.table = reinterpret_cast<uint4*>(base + L.table);
        b.cap = L.cap;
        GridView g = build_grid_into(c, b, S, n, s, nullptr, nullptr, false);
        int32_t* work = reinterpret_cast<int32_t*>(base + L.work);
        check(launch_fill_i32(work, 2, 0, s));   // the retry and overflow counters start at zero on every call
        check(launch_knn_cov(g, S, k, reg_mode, eps, reinterpret_cast<float*>(base + L.raw), work, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_map_build(gicp_ctx* c, const float* means, const float* covs, int64_t m, float cell, int reg_mode,
                   float eps, gicp_map** out, void* stream) {
    if (!c || !means || !covs || !out || m < 1 || !valid_mode(reg_mode) || m >= (1ll << 31)) return GICP_E_ARG;
    *out = nullptr;
    gicp_map* mp = new (std::nothrow) gicp_map();
    if (!mp) return GICP_E_OOM;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const float h = cell > 0.f ? cell : estimate_cell(c, means, m, 8, s);
        const uint32_t cap = table_capacity(m);
        mp->device = c->device;
        mp->m = m;
        mp->cap = m;
        mp->h = h;
        mp->mask = cap - 1;
        mp->reg_mode = reg_mode;
        mp->eps = eps;
        check(hipMalloc(&mp->spts, m * sizeof(float4)));
        check(hipMalloc(&mp->table, (size_t)cap * sizeof(uint4)));
        check(hipMalloc(&mp->scov, 2 * m * sizeof(float4)));
        check(hipMalloc(&mp->keys, m * sizeof(uint32_t)));
        build_grid(c, c->grid, one_cloud(means, m, h), m, s, mp->spts, mp->table, mp->keys);
        check(launch_map_covs(c->grid.sorted_vals, m, covs, m, reg_mode, eps, mp->scov, c->d_err, s));
        *out = mp;
        return GICP_OK;
    } catch (const HipError& e) {
        gicp_map_destroy(mp);
        return status_of(e);
    }
}

int gicp_map_destroy(gicp_map* mp) {
    if (!mp) return GICP_OK;
    (void)hipSetDevice(mp->device);
    (void)hipDeviceSynchronize();
    if (mp->spts) (void)hipFree(mp->spts);
    if (mp->table) (void)hipFree(mp->table);
    if (mp->scov) (void)hipFree(mp->scov);
    if (mp->keys) (void)hipFree(mp->keys);
    if (mp->spts2) (void)hipFree(mp->spts2);
    if (mp->scov2) (void)hipFree(mp->scov2);
    if (mp->keys2) (void)hipFree(mp->keys2);
    if (mp->inv) (void)hipFree(mp->inv);
    delete mp;
    return GICP_OK;
}

int gicp_map_info(const gicp_map* mp, int64_t* m, float* cell) {
    if (!mp) return GICP_E_ARG;
    if (m) *m = mp->m;
    if (cell) *cell = mp->h;
    return GICP_OK;
}

}  // extern "C"

namespace {

MapView map_view(const gicp_map* map, const gicp_params* prm) {
    MapView mv;
    mv.g.spts = map->spts;
    mv.g.skeys = map->keys;
    mv.g.table = map->table;
    mv.g.mask = map->mask;
    mv.g.n = (int32_t)map->m;
    mv.g.h = map->h;
    mv.g.inv_h = 1.0f / map->h;
    mv.scov = map->scov;
    mv.r_max = prm->r_max;
    mv.r_max2 = prm->r_max * prm->r_max;
    return mv;
}

bool valid_params(const gicp_params* prm) {
    return prm && prm->max_it >= 0 && prm->r_max > 0.f && prm->precision >= 0 && prm->precision <= 2 &&
           (prm->lanes == 0 || prm->lanes == 2 || prm->lanes == 4) &&
           (prm->flags & ~(GICP_FLAG_MULTI_LAUNCH | GICP_FLAG_QUEUE | GICP_FLAG_GRAPH | GICP_FLAG_NO_REUSE)) == 0;
}

// Lanes per source point: the parameter, or the form's default.
int lanes_of(const gicp_params* prm, int dflt) { return prm->lanes ? prm->lanes : dflt; }
// Default lanes of the Gauss-Newton launches for nprob problems: one problem
// leaves most of the chip idle and its launches are latency-bound (four
// lanes: 1.78k against 1.44k frames/s for per-frame registration of the
// 68k-point C2 frames); batches are bound by instruction issue (two lanes:
// 8.0k against 7.9k frames/s for 50 frames a call).
int batch_lanes(int64_t nprob) { return nprob == 1 ? kTrackLanes : kBatchLanes; }

// Work-queue workers that fit on the device at once (asked once per shape).
int queue_workers(gicp_ctx* c, int acc, int lanes) {
    int& w = c->queue_workers[acc][lanes == 4 ? 1 : 0];
    if (!w) w = gn_queue_workers(acc, lanes);
    return w;
}

// Graph of the max_it batched iterations for this batch shape and these
// workspace addresses (captured once on a private stream, then cached).
constexpr int64_t kGraphBucket = 1024;   // launch grids are padded to a multiple of this many chunks
constexpr size_t kMaxGraphs = 16;

hipGraphExec_t iteration_graph(gicp_ctx* c, int nprob, int64_t grid, int max_it, int acc, int lanes,
                               int32_t* chunk_prob, double* part) {
    for (auto& e : c->graphs)
        if (e.kind == 0 && e.nprob == nprob && e.chunks == grid && e.max_it == max_it && e.acc == acc &&
            e.lanes == lanes && e.probs == c->d_probs && e.chunk_prob == chunk_prob && e.part == part)
            return e.exec;
    if (!c->capture_stream) check(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = c->capture_stream;
    hipGraph_t graph = nullptr;
    check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int it = 0; it < max_it && err == hipSuccess; ++it) {
        err = launch_gn_iteration_batch(c->d_probs, nprob, chunk_prob, grid, part, acc, lanes, true, false, cs);
        if (err == hipSuccess)
            err = launch_gn_iteration_batch(c->d_probs, nprob, chunk_prob, grid, part, acc, lanes, false, true, cs);
    }
    const hipError_t end = hipStreamEndCapture(cs, &graph);
    check(err);
    check(end);
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check(inst);
    if (c->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({0, nprob, max_it, acc, 0, lanes, grid, c->d_probs, chunk_prob, part, nullptr, exec});
    return exec;
}

// Graph of one tracked frame (k_track_begin, then max_it iterations), valid
// for every frame of a call: which frame runs comes from the device counter.
hipGraphExec_t track_graph(gicp_ctx* c, int nprob, int64_t grid, int max_it, int acc, int lanes, int motion,
                           int32_t* counter, int32_t* chunk_prob, double* part) {
    for (auto& e : c->graphs)
        if (e.kind == 1 && e.nprob == nprob && e.chunks == grid && e.max_it == max_it && e.acc == acc &&
            e.lanes == lanes && e.motion == motion && e.probs == c->d_probs && e.chunk_prob == chunk_prob &&
            e.part == part &&
            e.counter == counter)
            return e.exec;
    if (!c->capture_stream) check(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = c->capture_stream;
    hipGraph_t graph = nullptr;
    check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t err = launch_track_begin(c->d_probs, nprob, counter, chunk_prob, grid, motion, cs);
    for (int it = 0; it < max_it && err == hipSuccess; ++it)
        err = launch_gn_track_iteration(c->d_probs, chunk_prob, grid, part, acc, lanes, true, true, cs);
    const hipError_t end = hipStreamEndCapture(cs, &graph);
    check(err);
    check(end);
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check(inst);
    if (c->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({1, nprob, max_it, acc, motion, lanes, grid, c->d_probs, chunk_prob, part, counter, exec});
    return exec;
}

// Registers nprob problems (validated by the caller).  covs_out[p] (nullable)
// receives problem p's source covariances when the call computes them.
// Returns the per-problem statuses in stats (never null here).
// Per-problem source arrays after prepare_sources: the covariances the
// linearisation reads and, for problems whose covariances the call computed,
// the grid-order copies of points and covariances it walks instead.
struct Sources {
    std::vector<const float*> scov;
    std::vector<const float4*> ssrc;
    std::vector<const float*> sscov;
    int32_t* nnprev = nullptr;
    float4* nncache = nullptr;
};

// 1. source covariances where missing; such problems are then linearised in
// their grid-cell order (sorted copies of the points and covariances)
void prepare_sources(gicp_ctx* c, int nprob, const gicp_problem* probs, const gicp_params* prm,
                     float* const* covs_out, Sources& out, hipStream_t s) {
    int64_t nsorted = 0, ntot = 0;
    for (int p = 0; p < nprob; ++p) {
        ntot += probs[p].n;
        if (!probs[p].src_covs) nsorted += probs[p].n;
    }
    float4* wsrc = nsorted ? ensure<float4>(c->ssrc, nsorted) : nullptr;
    float* wscov = nsorted ? ensure<float>(c->sscov, 6 * nsorted) : nullptr;
    int32_t* nnprev = ensure<int32_t>(c->nn_prev, ntot);
    float4* nncache = ensure<float4>(c->nn_cache, ntot);
    // size the grid workspace for the largest source up front (a reallocation
    // between problems would synchronise the device)
    int64_t nmax = 0, run = 0;
    int in_group = 0;
    for (int p = 0; p < nprob; ++p) {
        if (probs[p].src_covs) continue;
        if (in_group == kMaxSegments) {
            in_group = 0;
            run = 0;
        }
        run += probs[p].n;
        ++in_group;
        nmax = std::max(nmax, run);
    }
    if (nmax > 0) {
        reserve_grid(c->grid, nmax);
        ensure<int32_t>(c->overflow, knn_cov_work_ints(nmax));
    }
    std::vector<const float*>& scov = out.scov;
    std::vector<const float4*>& ssrc = out.ssrc;
    std::vector<const float*>& sscov = out.sscov;
    scov.assign(nprob, nullptr);
    ssrc.assign(nprob, nullptr);
    sscov.assign(nprob, nullptr);
    out.nnprev = nnprev;
    out.nncache = nncache;
    // problems with caller covariances keep the caller's order
    for (int p = 0; p < nprob; ++p) {
        const gicp_problem& P = probs[p];
        float* out = covs_out ? covs_out[p] : nullptr;
        if (!P.src_covs) continue;
        scov[p] = P.src_covs;
        if (out && out != P.src_covs)
            check(hipMemcpyAsync(out, P.src_covs, 6 * P.n * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    // the others: one segmented grid and one k-NN covariance launch per group
    // of up to kMaxSegments sources
    std::vector<int> todo;
    for (int p = 0; p < nprob; ++p)
        if (!probs[p].src_covs) todo.push_back(p);
    // cell sizes of all sources at once (one synchronisation)
    std::vector<float> cells(nprob, prm->cell_src);
    if (prm->cell_src <= 0.f && !todo.empty()) {
        std::vector<const float*> xs;
        std::vector<int64_t> ns;
        for (int p : todo) {
            xs.push_back(probs[p].src);
            ns.push_back(probs[p].n);
        }
        std::vector<float> est(todo.size());
        estimate_cells(c, (int)todo.size(), xs.data(), ns.data(), prm->k, s, est.data());
        for (size_t q = 0; q < todo.size(); ++q) cells[todo[q]] = est[q];
    }
    for (size_t g0 = 0; g0 < todo.size(); g0 += kMaxSegments) {
        const size_t g1 = std::min(todo.size(), g0 + kMaxSegments);
        const int cnt = (int)(g1 - g0);
        int64_t total = 0;
        for (size_t q = g0; q < g1; ++q) {
            const int p = todo[q];
            const gicp_problem& P = probs[p];
            // the registration reads the cell-order copy; the caller's order is
            // written only when the caller asked for the covariances
            float* dst = covs_out ? covs_out[p] : nullptr;
            const float h = cells[p];
            Seg& sg = c->h_segs[q - g0];
            sg.xyz = P.src;
            sg.covs = dst;
            sg.covs_sorted = wscov + 6 * total;
            sg.off = total;
            sg.n = P.n;
            sg.h = h;
            sg.inv_h = 1.0f / h;
            scov[p] = dst;
            ssrc[p] = wsrc + total;
            sscov[p] = wscov + 6 * total;
            total += P.n;
        }
        SegSet S;
        S.one = c->h_segs[0];
        S.count = cnt;
        S.many = nullptr;
        if (cnt > 1) {
            Seg* dsegs = ensure<Seg>(c->segs, kMaxSegments);
            check(hipMemcpyAsync(dsegs, c->h_segs, cnt * sizeof(Seg), hipMemcpyHostToDevice, s));
            S.many = dsegs;
        }
        GridView g = build_grid(c, c->grid, S, total, s, wsrc);
        const int pm = prof_open(c, GICP_PROF_KNN_COV, (double)total, -1, s);
        int32_t* work = static_cast<int32_t*>(c->overflow.p);
        check(launch_fill_i32(work, 2, 0, s));
        check(launch_knn_cov(g, S, prm->k, prm->reg_mode, prm->eps, wscov, work, s));
        prof_close(c, pm, s);
        wsrc += total;
        wscov += 6 * total;
        if (g1 < todo.size()) check(hipStreamSynchronize(s));   // the staging array is reused
    }
    check(launch_fill_i32(nnprev, ntot, -1, s));
}

// 2. states and problem descriptors (host copies; the caller uploads them).
// part0 of problem p is the running chunk count unless shared_partials, where
// every problem starts at slot 0 (problems that run one after another).
// Returns the total chunk count (shared: the largest).
int64_t prepare_states(gicp_ctx* c, int nprob, const gicp_problem* probs, const gicp_params* prm,
                       const Sources& src, bool shared_partials) {
    ensure_states(c, nprob);
    int32_t* nnprev = src.nnprev;
    float4* nncache = src.nncache;
    int64_t chunks = 0;
    for (int p = 0; p < nprob; ++p) {
        const gicp_problem& P = probs[p];
        RegState& hs = c->h_state[p];
        std::memset(&hs, 0, sizeof(RegState));
        for (int i = 0; i < 16; ++i) hs.pose[i] = P.init_pose[i];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) hs.Rf[3 * i + j] = (float)P.init_pose[4 * i + j];
            hs.tf[i] = (float)P.init_pose[4 * i + 3];
        }
        hs.max_it = prm->max_it;
        hs.done = prm->max_it <= 0 ? 1 : 0;
        hs.conv_rot = prm->conv_rot;
        hs.conv_trans = prm->conv_trans;
        hs.acc = prm->precision;
        ProbDev& pd = c->h_probs[p];
        pd.src = P.src;
        pd.scov = src.scov[p];
        pd.ssrc = src.ssrc[p];
        pd.sscov = src.sscov[p];
        pd.nn_prev = nnprev;
        pd.nn_cache = nncache;
        nnprev += P.n;
        nncache += P.n;
        pd.n = P.n;
        pd.nchunks = (int32_t)((P.n + kChunk - 1) / kChunk);
        pd.part0 = shared_partials ? 0 : (int32_t)chunks;
        pd.fresh = (prm->flags & GICP_FLAG_NO_REUSE) ? 1 : 0;
        pd.pad_ = 0;
        pd.map = map_view(P.map, prm);
        pd.st = c->d_state + p;
        chunks = shared_partials ? std::max<int64_t>(chunks, pd.nchunks) : chunks + pd.nchunks;
    }
    return chunks;
}

// Host outputs of nprob registrations from the downloaded states.
void write_results(gicp_ctx* c, int nprob, bool nonfinite, bool qerr, double* poses, double* Hs, double* bs,
                   gicp_stats* stats) {
    for (int p = 0; p < nprob; ++p) {
        const RegState& hs = c->h_state[p];
        if (poses)
            for (int i = 0; i < 16; ++i) poses[16 * p + i] = hs.pose[i];
        if (Hs) {
            int q = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = i; j < 6; ++j) {
                    Hs[36 * p + 6 * i + j] = hs.H[q];
                    Hs[36 * p + 6 * j + i] = hs.H[q];
                    ++q;
                }
        }
        if (bs)
            for (int i = 0; i < 6; ++i) bs[6 * p + i] = hs.b[i];
        gicp_stats& st = stats[p];
        st.iters = hs.iters;
        st.n_inliers = (int32_t)hs.n_inl;
        st.cost = hs.cost;
        st.converged = hs.converged;
        st.status = nonfinite ? GICP_E_NONFINITE : qerr ? GICP_E_HIP : hs.status;
        st.hip_error = 0;
    }
}

void register_many(gicp_ctx* c, int nprob, const gicp_problem* probs, const gicp_params* prm,
                   float* const* covs_out, double* poses, double* Hs, double* bs, gicp_stats* stats, hipStream_t s) {
    Sources src;
    prepare_sources(c, nprob, probs, prm, covs_out, src, s);
    const int64_t chunks = prepare_states(c, nprob, probs, prm, src, false);
    check(hipMemcpyAsync(c->d_state, c->h_state, nprob * sizeof(RegState), hipMemcpyHostToDevice, s));
    // 3. Gauss-Newton
    const bool queue = (prm->flags & GICP_FLAG_QUEUE) && !(prm->flags & GICP_FLAG_MULTI_LAUNCH);
    if (prm->max_it > 0) {
        if (prm->flags & GICP_FLAG_MULTI_LAUNCH) {
            for (int p = 0; p < nprob; ++p) {
                const ProbDev& pd = c->h_probs[p];
                const int nb = gn_blocks(pd.n);
                double* part = ensure<double>(c->partials, (size_t)nb * kNumAcc);
                for (int it = 0; it < prm->max_it; ++it) {
                    const int pl = prof_open(c, GICP_PROF_LINEARIZE, (double)pd.n, nprob == 1 ? it : -3, s);
                    check(launch_gn_linearize(pd, part, nb, prm->precision, s));
                    prof_close(c, pl, s);
                    const int ps = prof_open(c, GICP_PROF_SOLVE, 1.0, nprob == 1 ? it : -3, s);
                    check(launch_gn_solve(part, nb, pd.st, s));
                    prof_close(c, ps, s);
                }
            }
        } else if (queue) {
            check(hipMemcpyAsync(c->d_probs, c->h_probs, nprob * sizeof(ProbDev), hipMemcpyHostToDevice, s));
            const uint64_t cap64 = (uint64_t)chunks * (uint64_t)prm->max_it;
            if (cap64 >= (1ull << 31)) throw HipError{hipErrorInvalidValue};
            const uint32_t cap = (uint32_t)cap64;
            uint32_t* items = ensure<uint32_t>(c->items, cap);
            uint32_t* arrive = ensure<uint32_t>(c->arrive, nprob);
            double* part = ensure<double>(c->partials, (size_t)chunks * kNumAcc);
            const int acc = prm->precision;
            const int lanes = lanes_of(prm, kQueueLanes);
            const int workers = (int)std::min<int64_t>(chunks, queue_workers(c, acc, lanes));
            const int pq = prof_open(c, GICP_PROF_LINEARIZE, 0.0, -2, s);
            check(launch_gn_queue(c->d_probs, nprob, c->d_queue, items, cap, (uint32_t)chunks, arrive, part, workers,
                                  acc, lanes, s));
            prof_close(c, pq, s);
        } else if (prm->flags & GICP_FLAG_GRAPH) {
            check(hipMemcpyAsync(c->d_probs, c->h_probs, nprob * sizeof(ProbDev), hipMemcpyHostToDevice, s));
            const int64_t grid = (chunks + kGraphBucket - 1) / kGraphBucket * kGraphBucket;
            int32_t* chunk_prob = ensure<int32_t>(c->chunk_prob, grid);
            double* part = ensure<double>(c->partials, (size_t)grid * kNumAcc);
            check(launch_chunk_map(c->d_probs, nprob, chunk_prob, s));
            if (grid > chunks) check(launch_fill_i32(chunk_prob + chunks, grid - chunks, -1, s));
            hipGraphExec_t ge =
                iteration_graph(c, nprob, grid, prm->max_it, prm->precision, lanes_of(prm, batch_lanes(nprob)), chunk_prob,
                                part);
            const int pl = prof_open(c, GICP_PROF_LINEARIZE, 0.0, -2, s);
            check(hipGraphLaunch(ge, s));
            prof_close(c, pl, s);
        } else {
            check(hipMemcpyAsync(c->d_probs, c->h_probs, nprob * sizeof(ProbDev), hipMemcpyHostToDevice, s));
            int32_t* chunk_prob = ensure<int32_t>(c->chunk_prob, chunks);
            double* part = ensure<double>(c->partials, (size_t)chunks * kNumAcc);
            check(launch_chunk_map(c->d_probs, nprob, chunk_prob, s));
            for (int it = 0; it < prm->max_it; ++it) {
                // units: the work of a launch is only known after the run; the
                // single-problem case marks its iterations, batches count all
                const int pl = prof_open(c, GICP_PROF_LINEARIZE, 0.0, it, s);
                check(launch_gn_iteration_batch(c->d_probs, nprob, chunk_prob, chunks, part, prm->precision,
                                                lanes_of(prm, batch_lanes(nprob)), true, false, s));
                prof_close(c, pl, s);
                const int ps = prof_open(c, GICP_PROF_SOLVE, 1.0, it, s);
                check(launch_gn_iteration_batch(c->d_probs, nprob, chunk_prob, chunks, part, prm->precision,
                                                lanes_of(prm, batch_lanes(nprob)), false, true, s));
                prof_close(c, ps, s);
            }
        }
    }
    check(hipMemcpyAsync(c->h_state, c->d_state, nprob * sizeof(RegState), hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(c->h_err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(c->h_err + 1, &c->d_queue->error, sizeof(int), hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    double units = 0.0;
    int iters_max = 0;
    c->iter_units.assign(std::max(prm->max_it, 0), 0.0);
    for (int p = 0; p < nprob; ++p) {
        const int it = c->h_state[p].iters;
        units += (double)probs[p].n * it;
        iters_max = std::max(iters_max, it);
        for (int j = 0; j < it && j < (int)c->iter_units.size(); ++j) c->iter_units[j] += (double)probs[p].n;
    }
    c->queue_units = units;
    const bool per_problem = (prm->flags & GICP_FLAG_MULTI_LAUNCH) && nprob > 1;
    if (c->prof) prof_collect(c, per_problem ? (1 << 30) : iters_max);
    const bool nonfinite = (c->h_err[0] & kErrNonFinite) != 0;
    const bool qerr = queue && prm->max_it > 0 && c->h_err[1] != 0;
    if (nonfinite) {
        check(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
        check(hipStreamSynchronize(s));
    }
    write_results(c, nprob, nonfinite, qerr, poses, Hs, bs, stats);
}

int fail(gicp_stats* stats, int nprob, const HipError& e) {
    const int st = status_of(e);
    if (stats)
        for (int p = 0; p < nprob; ++p) {
            stats[p].status = st;
            stats[p].hip_error = (int32_t)e.e;
        }
    return st;
}

}  // namespace

extern "C" {

int gicp_register(gicp_ctx* c, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                  const double init_pose[16], const gicp_params* prm, double pose[16], double H[36], double b[6],
                  float* src_covs_out, gicp_stats* stats, void* stream) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!c || !src || !map || !init_pose || !prm || !pose || !H || !b || n < 1 || n >= (1ll << 31))
        return GICP_E_ARG;
    if (!src_covs && (!valid_cov_k(prm->k) || n < prm->k || !valid_mode(prm->reg_mode))) return GICP_E_ARG;
    if (!valid_params(prm)) return GICP_E_ARG;
    if ((n + kChunk - 1) / kChunk >= (1ll << kChunkBits)) return GICP_E_ARG;
    gicp_problem P;
    P.src = src;
    P.src_covs = src_covs;
    P.n = n;
    P.map = map;
    for (int i = 0; i < 16; ++i) P.init_pose[i] = init_pose[i];
    gicp_stats st;
    std::memset(&st, 0, sizeof(st));
    float* outs[1] = {src_covs_out};
    try {
        check(hipSetDevice(c->device));
        register_many(c, 1, &P, prm, outs, pose, H, b, &st, (hipStream_t)stream);
    } catch (const HipError& e) {
        return fail(stats, 1, e);
    }
    if (stats) *stats = st;
    return st.status;
}

int gicp_register_dev(gicp_ctx* c, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                      const double* init_pose, const gicp_params* prm, double* pose, double* H, double* b,
                      float* src_covs_out, gicp_stats* stats, void* stream) {
    if (!c || !src || !map || !init_pose || !prm || !pose || !H || !b || n < 1 || n >= (1ll << 31))
        return GICP_E_ARG;
    if (!src_covs && (!valid_cov_k(prm->k) || n < prm->k || !valid_mode(prm->reg_mode))) return GICP_E_ARG;
    if (!valid_params(prm) || (prm->flags & GICP_FLAG_GRAPH)) return GICP_E_ARG;
    if ((n + kChunk - 1) / kChunk >= (1ll << kChunkBits)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        gicp_problem P;
        P.src = src;
        P.src_covs = src_covs;
        P.n = n;
        P.map = map;
        for (int i = 0; i < 16; ++i) P.init_pose[i] = (i % 5 == 0) ? 1.0 : 0.0;   // replaced on the device
        float* outs[1] = {src_covs_out};
        Sources srcs;
        prepare_sources(c, 1, &P, prm, outs, srcs, s);
        const int64_t chunks = prepare_states(c, 1, &P, prm, srcs, false);
        ProbDev pd = c->h_probs[0];
        pd.st = c->dev_state;
        StateInit si;
        si.conv_rot = prm->conv_rot;
        si.conv_trans = prm->conv_trans;
        si.max_it = prm->max_it;
        si.acc = prm->precision;
        check(launch_state_init(pd, c->dev_probs, si, init_pose, c->dev_state, s));
        if (prm->max_it > 0) {
            if (prm->flags & GICP_FLAG_MULTI_LAUNCH) {
                const int nb = gn_blocks(n);
                double* part = ensure<double>(c->partials, (size_t)nb * kNumAcc);
                for (int it = 0; it < prm->max_it; ++it) {
                    check(launch_gn_linearize(pd, part, nb, prm->precision, s));
                    check(launch_gn_solve(part, nb, c->dev_state, s));
                }
            } else if (prm->flags & GICP_FLAG_QUEUE) {
                const uint64_t cap64 = (uint64_t)chunks * (uint64_t)prm->max_it;
                if (cap64 >= (1ull << 31)) throw HipError{hipErrorInvalidValue};
                const uint32_t cap = (uint32_t)cap64;
                uint32_t* items = ensure<uint32_t>(c->items, cap);
                uint32_t* arrive = ensure<uint32_t>(c->arrive, 1);
                double* part = ensure<double>(c->partials, (size_t)chunks * kNumAcc);
                const int acc = prm->precision;
                const int lanes = lanes_of(prm, kQueueLanes);
                const int workers = (int)std::min<int64_t>(chunks, queue_workers(c, acc, lanes));
                check(launch_gn_queue(c->dev_probs, 1, c->d_queue, items, cap, (uint32_t)chunks, arrive, part, workers,
                                      acc, lanes, s));
            } else {
                int32_t* chunk_prob = ensure<int32_t>(c->chunk_prob, chunks);
                double* part = ensure<double>(c->partials, (size_t)chunks * kNumAcc);
                check(launch_chunk_map(c->dev_probs, 1, chunk_prob, s));
                for (int it = 0; it < prm->max_it; ++it)
                    check(launch_gn_iteration_batch(c->dev_probs, 1, chunk_prob, chunks, part, prm->precision,
                                                    lanes_of(prm, batch_lanes(1)), true, true, s));
            }
        }
        check(launch_state_out(c->dev_state, c->d_err, pose, H, b, stats, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_register_batch(gicp_ctx* c, int nprob, const gicp_problem* probs, const gicp_params* prm, double* poses,
                        double* Hs, double* bs, gicp_stats* stats, void* stream) {
    if (stats) std::memset(stats, 0, (size_t)std::max(nprob, 0) * sizeof(gicp_stats));
    if (!c || !probs || nprob < 1 || nprob > kMaxProblems || !valid_params(prm)) return GICP_E_ARG;
    for (int p = 0; p < nprob; ++p) {
        const gicp_problem& P = probs[p];
        if (!P.src || !P.map || P.n < 1 || P.n >= (1ll << 31)) return GICP_E_ARG;
        if ((P.n + kChunk - 1) / kChunk >= (1ll << kChunkBits)) return GICP_E_ARG;
        if (!P.src_covs && (!valid_cov_k(prm->k) || P.n < prm->k || !valid_mode(prm->reg_mode))) return GICP_E_ARG;
    }
    std::vector<gicp_stats> st(nprob);
    try {
        check(hipSetDevice(c->device));
        register_many(c, nprob, probs, prm, nullptr, poses, Hs, bs, st.data(), (hipStream_t)stream);
    } catch (const HipError& e) {
        return fail(stats, nprob, e);
    }
    if (stats) std::memcpy(stats, st.data(), nprob * sizeof(gicp_stats));
    for (int p = 0; p < nprob; ++p)
        if (st[p].status == GICP_E_HIP || st[p].status == GICP_E_NONFINITE) return st[p].status;
    return GICP_OK;
}

int gicp_track(gicp_ctx* c, int nframes, const gicp_frame* frames, const gicp_map* map, const double init_pose[16],
               int motion, const gicp_params* prm, double* poses, double* Hs, double* bs, gicp_stats* stats,
               void* stream) {
    if (stats) std::memset(stats, 0, (size_t)std::max(nframes, 0) * sizeof(gicp_stats));
    if (!c || !frames || !map || !init_pose || nframes < 1 || nframes > kMaxProblems || !valid_params(prm))
        return GICP_E_ARG;
    if (motion != GICP_MOTION_PREVIOUS && motion != GICP_MOTION_CONSTANT_VELOCITY) return GICP_E_ARG;
    if (prm->flags & GICP_FLAG_QUEUE) return GICP_E_ARG;
    std::vector<gicp_problem> probs(nframes);
    for (int i = 0; i < nframes; ++i) {
        const gicp_frame& F = frames[i];
        if (!F.src || F.n < 1 || F.n >= (1ll << 31)) return GICP_E_ARG;
        if ((F.n + kChunk - 1) / kChunk >= (1ll << kChunkBits)) return GICP_E_ARG;
        if (!F.src_covs && (!valid_cov_k(prm->k) || F.n < prm->k || !valid_mode(prm->reg_mode))) return GICP_E_ARG;
        gicp_problem& P = probs[i];
        P.src = F.src;
        P.src_covs = F.src_covs;
        P.n = F.n;
        P.map = map;
        for (int j = 0; j < 16; ++j) P.init_pose[j] = (i == 0) ? init_pose[j] : (j % 5 == 0 ? 1.0 : 0.0);
    }
    std::vector<gicp_stats> st(nframes);
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        Sources src;
        prepare_sources(c, nframes, probs.data(), prm, nullptr, src, s);
        const int64_t grid = prepare_states(c, nframes, probs.data(), prm, src, true);
        check(hipMemcpyAsync(c->d_state, c->h_state, nframes * sizeof(RegState), hipMemcpyHostToDevice, s));
        check(hipMemcpyAsync(c->d_probs, c->h_probs, nframes * sizeof(ProbDev), hipMemcpyHostToDevice, s));
        int32_t* chunk_prob = ensure<int32_t>(c->chunk_prob, grid);
        double* part = ensure<double>(c->partials, (size_t)grid * kNumAcc);
        int32_t* counter = ensure<int32_t>(c->track_counter, 3);
        check(launch_fill_i32(counter, 3, 0, s));
        bool stalled = false;
        const int acc = prm->precision;
        const int lanes = lanes_of(prm, kTrackLanes);
        if (prm->max_it > 0 && !(prm->flags & (GICP_FLAG_GRAPH | GICP_FLAG_MULTI_LAUNCH))) {
            // iteration slots: (linearise, solve) pairs whose problem the device
            // chooses; the host launches until every problem has finished,
            // at most kLead slots ahead of the device
            if (!c->h_progress) {
                check(hipHostMalloc(&c->h_progress, 2 * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent));
                check(hipHostGetDevicePointer((void**)&c->d_progress, c->h_progress, 0));
            }
            // the slots' hand-over words, zero (int32 words) before the first slot
            const int64_t sync_words = (int64_t)(slot_sync_bytes() / sizeof(int32_t));
            int32_t* sync = ensure<int32_t>(c->slot_sync, (size_t)sync_words);
            check(launch_fill_i32(sync, sync_words, 0, s));
            volatile int32_t* hp = c->h_progress;
            hp[0] = 0;
            hp[1] = 0;
            constexpr int64_t kLead = 16;
            const int64_t max_slots = (int64_t)nframes * prm->max_it;
            int64_t launched = 0;
            stalled = false;
            while (launched < max_slots && hp[0] < nframes) {
                if (launched - hp[1] >= kLead) {
                    // the device is behind: wait for it (bounded; a failed
                    // stream is reported by the synchronisation below)
                    const auto t0 = std::chrono::steady_clock::now();
                    while (launched - hp[1] >= kLead && hp[0] < nframes) {
                        std::this_thread::yield();
                        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) break;
                    }
                    if (launched - hp[1] >= kLead && hp[0] < nframes) {
                        stalled = true;
                        break;
                    }
                    continue;
                }
                const int pl = prof_open(c, GICP_PROF_LINEARIZE, 0.0, (int)launched, s, -5);
                check(launch_track_slot(c->d_probs, nframes, counter, (int)(launched & 1), grid, part, acc, lanes,
                                        motion, c->d_progress, sync, s));
                prof_close(c, pl, s);
                ++launched;
            }
        } else if (prm->max_it > 0 && (prm->flags & GICP_FLAG_GRAPH)) {
            hipGraphExec_t ge =
                track_graph(c, nframes, grid, prm->max_it, acc, lanes, motion, counter, chunk_prob, part);
            for (int i = 0; i < nframes; ++i) {
                const int pm = prof_open(c, GICP_PROF_LINEARIZE, (double)probs[i].n, -2, s, i);
                check(hipGraphLaunch(ge, s));
                prof_close(c, pm, s);
            }
        } else {
            for (int i = 0; i < nframes; ++i) {
                check(launch_track_begin(c->d_probs, nframes, counter, chunk_prob, grid, motion, s));
                for (int it = 0; it < prm->max_it; ++it) {
                    const int pl = prof_open(c, GICP_PROF_LINEARIZE, (double)probs[i].n, it, s, i);
                    check(launch_gn_track_iteration(c->d_probs, chunk_prob, grid, part, acc, lanes, true, false, s));
                    prof_close(c, pl, s);
                    const int ps = prof_open(c, GICP_PROF_SOLVE, 1.0, it, s, i);
                    check(launch_gn_track_iteration(c->d_probs, chunk_prob, grid, part, acc, lanes, false, true, s));
                    prof_close(c, ps, s);
                }
            }
        }
        check(hipMemcpyAsync(c->h_state, c->d_state, nframes * sizeof(RegState), hipMemcpyDeviceToHost, s));
        check(hipMemcpyAsync(c->h_err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        double units = 0.0, work = 0.0;
        for (int i = 0; i < nframes; ++i) {
            units += (double)probs[i].n * c->h_state[i].iters;
            work += c->h_state[i].iters;
        }
        c->queue_units = units;
        c->slot_work = work;
        if (c->prof) prof_collect(c, 1 << 30);
        const bool nonfinite = (c->h_err[0] & kErrNonFinite) != 0;
        if (nonfinite) {
            check(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
            check(hipStreamSynchronize(s));
        }
        if (stalled) throw HipError{hipErrorLaunchTimeOut};
        write_results(c, nframes, nonfinite, false, poses, Hs, bs, st.data());
    } catch (const HipError& e) {
        return fail(stats, nframes, e);
    }
    if (stats) std::memcpy(stats, st.data(), nframes * sizeof(gicp_stats));
    for (int i = 0; i < nframes; ++i)
        if (st[i].status == GICP_E_HIP || st[i].status == GICP_E_NONFINITE) return st[i].status;
    return GICP_OK;
}

int gicp_register_pair(gicp_ctx* c, const float* src, const float* src_covs, int64_t n, const float* map_means,
                       const float* map_covs, int64_t m, float map_cell, const double init_pose[16],
                       const gicp_params* prm, double pose[16], double H[36], double b[6], gicp_stats* stats,
                       void* stream) {
    gicp_map* mp = nullptr;
    int st = gicp_map_build(c, map_means, map_covs, m, map_cell, GICP_REG_NONE, 0.f, &mp, stream);
    if (st != GICP_OK) return st;
    st = gicp_register(c, src, src_covs, n, mp, init_pose, prm, pose, H, b, nullptr, stats, stream);
    gicp_map_destroy(mp);
    return st;
}

int gicp_map_nearest(gicp_ctx* c, gicp_map* mp, const float* queries, int64_t nq, float r_max,
                     const int32_t* hints, int32_t* idx, float* d2, float* radius, int32_t lanes, void* stream) {
    if (!c || !mp || nq < 0 || !(r_max > 0.f) || !std::isfinite(r_max) || nq >= (1ll << 31)) return GICP_E_ARG;
    if (lanes != 0 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16) return GICP_E_ARG;
    if (nq > 0 && (!queries || !idx || !d2)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const int32_t* inv = nullptr;
        if (hints && nq > 0) {
            if (!mp->inv) check(hipMalloc(&mp->inv, (size_t)std::max<int64_t>(mp->m, 1) * sizeof(int32_t)));
            if (!mp->inv_ok) {
                check(launch_map_inverse(mp->spts, mp->m, mp->inv, s));
                mp->inv_ok = true;
            }
            inv = mp->inv;
        }
        gicp_params prm;
        gicp_params_default(&prm);
        prm.r_max = r_max;
        check(launch_map_nearest(map_view(mp, &prm), queries, nq, hints, inv, idx, d2, radius, lanes ? lanes : 2, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_profile(gicp_ctx* c, int enable) {
    if (!c) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        check(hipDeviceSynchronize());
        c->prof = enable != 0;
        c->marks.clear();
        c->ev_used = 0;
        for (int g = 0; g < GICP_PROF_GROUPS; ++g) {
            c->launches[g] = 0;
            c->ms[g] = 0.0;
            c->units[g] = 0.0;
        }
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_profile_read(gicp_ctx* c, int group, int64_t* launches, double* total_ms, double* units) {
    if (!c || group < 0 || group >= GICP_PROF_GROUPS) return GICP_E_ARG;
    if (launches) *launches = c->launches[group];
    if (total_ms) *total_ms = c->ms[group];
    if (units) *units = c->units[group];
    return GICP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// warm-start network
// ---------------------------------------------------------------------------
namespace {
bool valid_batch(int B) { return B >= 1 && B <= GICP_MLP_MAX_BATCH; }
}  // namespace

int gicp_mlp_init(gicp_ctx* c, uint64_t seed, float* params, float* m, float* v, uint16_t* wbf16, void* stream) {
    if (!c || !params || !wbf16 || seed >= (1ull << 32)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        check(launch_mlp_init(seed, params, m, v, wbf16, (hipStream_t)stream));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_mlp_sync_weights(gicp_ctx* c, const float* params, uint16_t* wbf16, void* stream) {
    if (!c || !params || !wbf16) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        check(launch_mlp_fragments(params, wbf16, (hipStream_t)stream));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_mlp_pack(gicp_ctx* c, int B, const gicp_mlp_pair* pairs, uint16_t* X, double* centres, void* stream) {
    if (!c || !pairs || !X || !valid_batch(B)) return GICP_E_ARG;
    for (int i = 0; i < B; ++i) {
        const gicp_mlp_pair& P = pairs[i];
        if (!P.src || !P.tgt || !P.src_idx || !P.tgt_idx || P.n_src < 1 || P.n_tgt < 1) return GICP_E_ARG;
    }
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        if (!c->h_pairs) {
            check(hipHostMalloc(&c->h_pairs, GICP_MLP_MAX_BATCH * sizeof(gicp_mlp_pair)));
            check(hipEventCreateWithFlags(&c->pairs_ev, hipEventDisableTiming));
        }
        if (c->pairs_pending) check(hipEventSynchronize(c->pairs_ev));   // the staging copy is reused
        std::memcpy(c->h_pairs, pairs, B * sizeof(gicp_mlp_pair));
        gicp_mlp_pair* dp = ensure<gicp_mlp_pair>(c->mlp_pairs, GICP_MLP_MAX_BATCH);
        check(hipMemcpyAsync(dp, c->h_pairs, B * sizeof(gicp_mlp_pair), hipMemcpyHostToDevice, s));
        check(hipEventRecord(c->pairs_ev, s));
        c->pairs_pending = true;
        check(launch_mlp_pack(B, dp, X, centres, c->d_err, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_mlp_forward(gicp_ctx* c, int B, const uint16_t* X, const float* params, const uint16_t* wbf16,
                     const double* centres, float* y, float* cache, double* poses, void* stream) {
    if (!c || !X || !params || !wbf16 || !valid_batch(B) || (poses && !centres)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        const size_t np = (size_t)B * mlp_splits() * 256;
        float* pmax = ensure<float>(c->mlp_pmax, np);
        int* parg = ensure<int>(c->mlp_parg, np);
        check(launch_mlp_forward(B, X, params, wbf16, pmax, parg, centres, y, cache, poses, (hipStream_t)stream));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_mlp_backward(gicp_ctx* c, int B, const uint16_t* X, const float* params, const float* cache,
                      const float* y, const float* ystar, float* grad, float* loss, void* stream) {
    if (!c || !X || !params || !cache || !y || !ystar || !grad || !valid_batch(B)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        float* gpair = ensure<float>(c->mlp_gpair, (size_t)B * GICP_MLP_PARAMS);
        float* lpair = ensure<float>(c->mlp_lpair, (size_t)B);
        check(launch_mlp_backward(B, X, params, cache, y, ystar, gpair, lpair, grad, loss, (hipStream_t)stream));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_mlp_adam_step(gicp_ctx* c, float* params, float* m, float* v, const float* grad, int t, float lr,
                       uint16_t* wbf16, void* stream) {
    if (!c || !params || !m || !v || !grad || !wbf16 || t < 1 || !(lr > 0.f)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        check(launch_mlp_adam(params, m, v, grad, t, lr, wbf16, (hipStream_t)stream));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

// ---------------------------------------------------------------------------
// depth image -> point cloud; keyframe Gaussians; incremental map update
// ---------------------------------------------------------------------------
int gicp_depth_to_points(gicp_ctx* c, const float* depth, int width, int height, float fx, float fy, float cx,
                         float cy, float voxel, float max_depth, float* out_xyz, int64_t capacity, int64_t* n_out,
                         void* stream) {
    if (!c || !depth || !out_xyz || !n_out || width < 1 || height < 1 || !(voxel > 0.f) || !(fx != 0.f) ||
        !(fy != 0.f) || !(max_depth > 0.f) || (int64_t)width * height >= (1ll << 31))
        return GICP_E_ARG;
    *n_out = 0;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = (int64_t)width * height;
        float* pts = ensure<float>(c->dep_pts, 3 * n);
        int* vox = ensure<int>(c->dep_vox, 3 * n);
        int* misc = ensure<int>(c->dep_misc, 64);   // [0..6) bounds, [8] voxel count
        check(launch_depth_points(depth, width, height, fx, fy, cx, cy, voxel, max_depth, pts, vox, misc, s));
        int hb[6];
        check(hipMemcpyAsync(c->h_err + 8, misc, 6 * sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        std::memcpy(hb, c->h_err + 8, sizeof(hb));
        if (hb[0] > hb[3]) return GICP_OK;   // no valid pixel
        const uint64_t dx = (uint64_t)((int64_t)hb[3] - hb[0] + 1), dy = (uint64_t)((int64_t)hb[4] - hb[1] + 1),
                       dz = (uint64_t)((int64_t)hb[5] - hb[2] + 1);
        const double cells = (double)dx * (double)dy * (double)dz;
        if (cells >= 4294967295.0) return GICP_E_ARG;   // occupied box exceeds 32-bit voxel keys
        const uint64_t total = dx * dy * dz;
        int passes = 1;
        while (passes < 4 && (1ull << (8 * passes)) - 1 <= total) ++passes;
        GridBufs& gb = c->grid;
        uint32_t* ka = ensure<uint32_t>(gb.keys_a, n);
        uint32_t* va = ensure<uint32_t>(gb.vals_a, n);
        uint32_t* kb = ensure<uint32_t>(gb.keys_b, n);
        uint32_t* vb = ensure<uint32_t>(gb.vals_b, n);
        void* scr = ensure<uint8_t>(gb.scratch, radix_scratch_bytes(n));
        check(launch_voxel_keys(vox, n, misc, (uint32_t)dy, (uint32_t)dz, ka, va, s));
        uint32_t *ks = nullptr, *vs = nullptr;
        check(radix_sort(ka, va, kb, vb, n, passes, scr, s, &ks, &vs));
        uint32_t* flags = ensure<uint32_t>(c->dep_flags, n);
        uint32_t* pos = ensure<uint32_t>(c->dep_pos, n);
        void* sscr = ensure<uint8_t>(c->dep_scan, flag_scan_scratch(n));
        check(launch_voxel_starts(ks, n, flags, s));
        check(launch_flag_scan(flags, n, pos, reinterpret_cast<uint32_t*>(misc + 8), sscr, s));
        check(hipMemcpyAsync(c->h_err + 8, misc + 8, sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        const int64_t m = (int64_t)(uint32_t)c->h_err[8];
        if (m > capacity) return GICP_E_ARG;
        check(launch_voxel_centroids(ks, vs, n, flags, pos, pts, out_xyz, m, s));
        *n_out = m;
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_keyframe_gaussians(gicp_ctx* c, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                            const double pose[16], float r_overlap, float p, float* out_means, float* out_covs,
                            int64_t* n_out, double* inlier_ratio, void* stream) {
    if (!c || !src || !src_covs || !map || !pose || !out_means || !out_covs || !n_out || n < 1 ||
        !(r_overlap > 0.f) || !std::isfinite(p) || n >= (1ll << 31))
        return GICP_E_ARG;
    *n_out = 0;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        gicp_params prm;
        gicp_params_default(&prm);
        prm.r_max = r_overlap;
        const MapView mv = map_view(map, &prm);
        Pose32 T32;
        Pose64 T64;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                T32.R[3 * i + j] = (float)pose[4 * i + j];
                T64.R[3 * i + j] = pose[4 * i + j];
            }
            T32.t[i] = (float)pose[4 * i + 3];
            T64.t[i] = pose[4 * i + 3];
        }
        uint32_t* keep = ensure<uint32_t>(c->dep_flags, n);
        uint32_t* pos = ensure<uint32_t>(c->dep_pos, n);
        void* sscr = ensure<uint8_t>(c->dep_scan, flag_scan_scratch(n));
        int* misc = ensure<int>(c->dep_misc, 64);
        check(launch_overlap(mv, src, n, T32, keep, s));
        check(launch_flag_scan(keep, n, pos, reinterpret_cast<uint32_t*>(misc + 8), sscr, s));
        check(launch_keyframe_gaussians(src, src_covs, n, keep, pos, T64, 2.0 * (double)p, out_means, out_covs, s));
        check(hipMemcpyAsync(c->h_err + 8, misc + 8, sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        const int64_t kept = (int64_t)(uint32_t)c->h_err[8];
        *n_out = kept;
        if (inlier_ratio) *inlier_ratio = (double)(n - kept) / (double)n;
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_keyframe_policy(double inlier_ratio, int since_keyframe, int since_mapping, double threshold, int max_gap,
                         int mapping_gap) {
    if (inlier_ratio < threshold || (max_gap > 0 && since_keyframe >= max_gap)) return GICP_KEYFRAME;
    if (mapping_gap > 0 && since_mapping >= mapping_gap) return GICP_MAPPING_ONLY;
    return 0;
}

int gicp_map_insert(gicp_ctx* c, gicp_map* mp, const float* means, const float* covs, int64_t m_new, void* stream) {
    if (!c || !mp || !means || !covs || m_new < 1 || mp->m + m_new >= (1ll << 31)) return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const int64_t m_old = mp->m, total = m_old + m_new;
        // 1. the new points sorted by cell key on their own, their regularised covariances in that order
        GridBufs& gb = c->grid;
        uint32_t* ka = ensure<uint32_t>(gb.keys_a, m_new);
        uint32_t* va = ensure<uint32_t>(gb.vals_a, m_new);
        uint32_t* kb = ensure<uint32_t>(gb.keys_b, m_new);
        uint32_t* vb = ensure<uint32_t>(gb.vals_b, m_new);
        void* scr = ensure<uint8_t>(gb.scratch, radix_scratch_bytes(m_new));
        check(launch_cell_keys(one_cloud(means, m_new, mp->h), m_new, ka, va, c->d_err, s));
        uint32_t *ks = nullptr, *vs = nullptr;
        check(radix_sort(ka, va, kb, vb, m_new, 3, scr, s, &ks, &vs));
        float4* ncov = ensure<float4>(c->ins_cov, 2 * m_new);
        check(launch_map_covs(vs, m_new, covs, m_new, mp->reg_mode, mp->eps, ncov, c->d_err, s));
        // 2. merge into the spare arrays (grown together with the primary
        //    ones when the map outgrows them), then swap
        float4 *spts = mp->spts2, *scov = mp->scov2;
        uint32_t* keys = mp->keys2;
        int64_t cap = mp->cap;
        const bool grow = total > cap || !spts;
        if (grow) {
            cap = total > mp->cap ? std::max<int64_t>(total, mp->cap + mp->cap / 2) : mp->cap;
            spts = nullptr;
            scov = nullptr;
            keys = nullptr;
            try {
                check(hipMalloc(&spts, cap * sizeof(float4)));
                check(hipMalloc(&scov, 2 * cap * sizeof(float4)));
                check(hipMalloc(&keys, cap * sizeof(uint32_t)));
            } catch (const HipError&) {
                if (spts) (void)hipFree(spts);
                if (scov) (void)hipFree(scov);
                if (keys) (void)hipFree(keys);
                throw;
            }
        }
        uint4* table = mp->table;
        uint32_t tcap = mp->mask + 1;
        if (table_capacity(total) > tcap) {
            tcap = table_capacity(total);
            table = nullptr;
            check(hipMalloc(&table, (size_t)tcap * sizeof(uint4)));
        }
        check(launch_map_merge(mp->keys, mp->spts, mp->scov, m_old, ks, vs, means, ncov, m_new, keys, spts, scov, s));
        check(launch_table_clear(table, tcap, s));
        check(launch_table_runs(keys, total, table, tcap - 1, s));
        if (table != mp->table) {
            check(hipStreamSynchronize(s));
            (void)hipFree(mp->table);
        }
        if (grow) {
            // the old primary arrays were the merge source: free them after the merge,
            // and give the map a spare set of the new capacity
            check(hipStreamSynchronize(s));
            (void)hipFree(mp->spts);
            (void)hipFree(mp->scov);
            (void)hipFree(mp->keys);
            if (mp->spts2) (void)hipFree(mp->spts2);
            if (mp->scov2) (void)hipFree(mp->scov2);
            if (mp->keys2) (void)hipFree(mp->keys2);
            mp->spts2 = nullptr;
            mp->scov2 = nullptr;
            mp->keys2 = nullptr;
            mp->spts = spts;
            mp->scov = scov;
            mp->keys = keys;
            check(hipMalloc(&mp->spts2, cap * sizeof(float4)));
            check(hipMalloc(&mp->scov2, 2 * cap * sizeof(float4)));
            check(hipMalloc(&mp->keys2, cap * sizeof(uint32_t)));
        } else {
            std::swap(mp->spts, mp->spts2);
            std::swap(mp->scov, mp->scov2);
            std::swap(mp->keys, mp->keys2);
        }
        mp->table = table;
        mp->mask = tcap - 1;
        mp->m = total;
        mp->cap = cap;
        if (mp->inv) {
            check(hipStreamSynchronize(s));
            (void)hipFree(mp->inv);
            mp->inv = nullptr;
        }
        mp->inv_ok = false;
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}
