// Host runtime and C ABI of libgicp.so: context and growable workspace, grid
// builds, map handles and the Gauss-Newton driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
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

struct gicp_ctx {
    int device = 0;
    int* d_err = nullptr;
    int* h_err = nullptr;
    GridBufs grid;
    Buf covs, partials, kth;
    RegState* d_state = nullptr;
    RegState* h_state = nullptr;
    float* h_kth = nullptr;
};

struct gicp_map {
    int device = 0;
    int64_t m = 0;
    float h = 0.f;
    uint32_t mask = 0;
    float4* spts = nullptr;
    uint4* table = nullptr;
    float4* scov = nullptr;
};

namespace {

int status_of(const HipError& e) { return e.e == hipErrorOutOfMemory ? GICP_E_OOM : GICP_E_HIP; }

// Builds the cell grid of n points (SoA, row stride `stride`) into `gb`.
GridView build_grid(gicp_ctx* ctx, GridBufs& gb, const float* xyz, int64_t n, int64_t stride, float h,
                    hipStream_t s, float4* spts_out = nullptr, uint4* table_out = nullptr,
                    uint32_t* svals_keep = nullptr) {
    uint32_t* ka = ensure<uint32_t>(gb.keys_a, n);
    uint32_t* va = ensure<uint32_t>(gb.vals_a, n);
    uint32_t* kb = ensure<uint32_t>(gb.keys_b, n);
    uint32_t* vb = ensure<uint32_t>(gb.vals_b, n);
    void* scr = ensure<uint8_t>(gb.scratch, radix_scratch_bytes(n));
    const uint32_t cap = table_capacity(n);
    float4* spts = spts_out ? spts_out : ensure<float4>(gb.spts, n);
    uint4* table = table_out ? table_out : ensure<uint4>(gb.table, cap);
    const float inv_h = 1.0f / h;
    check(launch_cell_keys(xyz, n, stride, inv_h, ka, va, ctx->d_err, s));
    check(radix_sort_30(ka, va, kb, vb, n, scr, s));
    check(launch_table_clear(table, cap, s));
    check(launch_table_build(kb, vb, n, xyz, stride, spts, table, cap - 1, s));
    if (svals_keep) check(hipMemcpyAsync(svals_keep, vb, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    GridView g;
    g.spts = spts;
    g.table = table;
    g.mask = cap - 1;
    g.n = (int32_t)n;
    g.h = h;
    g.inv_h = inv_h;
    return g;
}

float estimate_cell(gicp_ctx* ctx, const float* xyz, int64_t n, int k, hipStream_t s) {
    const int ns = (int)std::min<int64_t>(256, n);
    float* d = ensure<float>(ctx->kth, ns);
    check(launch_kth_distance(xyz, n, std::min<int>(k, (int)n), ns, d, s));
    check(hipMemcpyAsync(ctx->h_kth, d, ns * sizeof(float), hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    std::vector<float> v(ctx->h_kth, ctx->h_kth + ns);
    std::sort(v.begin(), v.end());
    float c = v[(size_t)(0.75 * (ns - 1))] * 1.1f;
    if (!(c > 1e-6f) || !std::isfinite(c)) c = 1e-3f;
    return c;
}

bool valid_k(int k) { return k >= 1 && k <= 64; }
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
        check(hipMalloc(&c->d_state, sizeof(RegState)));
        check(hipHostMalloc(&c->h_state, sizeof(RegState)));
        check(hipHostMalloc(&c->h_err, 256));
        check(hipHostMalloc(&c->h_kth, 256 * sizeof(float)));
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
                   &c->grid.spts, &c->grid.table, &c->covs, &c->partials, &c->kth})
        release(*b);
    if (c->d_err) (void)hipFree(c->d_err);
    if (c->d_state) (void)hipFree(c->d_state);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_err) (void)hipHostFree(c->h_err);
    if (c->h_kth) (void)hipHostFree(c->h_kth);
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
        const int e = *c->h_err;
        if (e) check(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
        check(hipStreamSynchronize(s));
        if (e & kErrNonFinite) return GICP_E_NONFINITE;
        if (e & kErrInexact) return GICP_E_INEXACT;
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
        GridView g = build_grid(c, c->grid, pts, n, n, h, s);
        check(launch_knn_query(g, queries, nq, k, r_max, idx, d2, c->d_err, s));
        return GICP_OK;
    } catch (const HipError& e) {
        return status_of(e);
    }
}

int gicp_covariances(gicp_ctx* c, const float* pts, int64_t n, int k, float cell, int reg_mode, float eps,
                     float* covs, void* stream) {
    if (!c || !pts || !covs || !valid_k(k) || n < k || !valid_mode(reg_mode) || n >= (1ll << 31))
        return GICP_E_ARG;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const float h = cell > 0.f ? cell : estimate_cell(c, pts, n, k, s);
        GridView g = build_grid(c, c->grid, pts, n, n, h, s);
        check(launch_knn_cov(g, pts, n, k, reg_mode, eps, covs, c->d_err, s));
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
        mp->h = h;
        mp->mask = cap - 1;
        check(hipMalloc(&mp->spts, m * sizeof(float4)));
        check(hipMalloc(&mp->table, (size_t)cap * sizeof(uint4)));
        check(hipMalloc(&mp->scov, 2 * m * sizeof(float4)));
        build_grid(c, c->grid, means, m, m, h, s, mp->spts, mp->table);
        // the sorted values (original indices) are still in grid.vals_b
        check(launch_map_covs(static_cast<const uint32_t*>(c->grid.vals_b.p), m, covs, m, reg_mode, eps, mp->scov,
                              c->d_err, s));
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
    delete mp;
    return GICP_OK;
}

int gicp_map_info(const gicp_map* mp, int64_t* m, float* cell) {
    if (!mp) return GICP_E_ARG;
    if (m) *m = mp->m;
    if (cell) *cell = mp->h;
    return GICP_OK;
}

int gicp_register(gicp_ctx* c, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                  const double init_pose[16], const gicp_params* prm, double pose[16], double H[36], double b[6],
                  float* src_covs_out, gicp_stats* stats, void* stream) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!c || !src || !map || !init_pose || !prm || !pose || !H || !b || n < 1 || n >= (1ll << 31))
        return GICP_E_ARG;
    if (!src_covs && (!valid_k(prm->k) || n < prm->k || !valid_mode(prm->reg_mode))) return GICP_E_ARG;
    if (prm->max_it < 0 || !(prm->r_max > 0.f)) return GICP_E_ARG;
    if (prm->precision < 0 || prm->precision > 2) return GICP_E_ARG;
    int status = GICP_OK;
    try {
        check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        const float* scov = src_covs;
        if (!scov) {
            float* dst = src_covs_out ? src_covs_out : ensure<float>(c->covs, 6 * n);
            const float h = prm->cell_src > 0.f ? prm->cell_src : estimate_cell(c, src, n, prm->k, s);
            GridView g = build_grid(c, c->grid, src, n, n, h, s);
            check(launch_knn_cov(g, src, n, prm->k, prm->reg_mode, prm->eps, dst, c->d_err, s));
            scov = dst;
        } else if (src_covs_out && src_covs_out != src_covs) {
            check(hipMemcpyAsync(src_covs_out, src_covs, 6 * n * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
        RegState* hs = c->h_state;
        std::memset(hs, 0, sizeof(RegState));
        for (int i = 0; i < 16; ++i) hs->pose[i] = init_pose[i];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) hs->Rf[3 * i + j] = (float)init_pose[4 * i + j];
            hs->tf[i] = (float)init_pose[4 * i + 3];
        }
        hs->max_it = prm->max_it;
        hs->done = prm->max_it <= 0 ? 1 : 0;
        hs->conv_rot = prm->conv_rot;
        hs->conv_trans = prm->conv_trans;
        hs->acc = prm->precision;
        check(hipMemcpyAsync(c->d_state, hs, sizeof(RegState), hipMemcpyHostToDevice, s));
        MapView mv;
        mv.g.spts = map->spts;
        mv.g.table = map->table;
        mv.g.mask = map->mask;
        mv.g.n = (int32_t)map->m;
        mv.g.h = map->h;
        mv.g.inv_h = 1.0f / map->h;
        mv.scov = map->scov;
        mv.r_max = prm->r_max;
        mv.r_max2 = prm->r_max * prm->r_max;
        const int nb = gn_blocks(n);
        double* part = ensure<double>(c->partials, (size_t)nb * kNumAcc);
        for (int it = 0; it < prm->max_it; ++it)
            check(launch_gn_iteration(src, scov, n, mv, c->d_state, part, nb, prm->precision, s));
        check(hipMemcpyAsync(hs, c->d_state, sizeof(RegState), hipMemcpyDeviceToHost, s));
        check(hipMemcpyAsync(c->h_err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        for (int i = 0; i < 16; ++i) pose[i] = hs->pose[i];
        int q = 0;
        for (int i = 0; i < 6; ++i)
            for (int j = i; j < 6; ++j) {
                H[6 * i + j] = hs->H[q];
                H[6 * j + i] = hs->H[q];
                ++q;
            }
        for (int i = 0; i < 6; ++i) b[i] = hs->b[i];
        status = hs->status;
        if (*c->h_err & kErrNonFinite) {
            status = GICP_E_NONFINITE;
            check(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
            check(hipStreamSynchronize(s));
        }
        if (stats) {
            stats->iters = hs->iters;
            stats->n_inliers = (int32_t)hs->n_inl;
            stats->cost = hs->cost;
            stats->converged = hs->converged;
            stats->status = status;
        }
        return status;
    } catch (const HipError& e) {
        if (stats) {
            stats->status = status_of(e);
            stats->hip_error = (int32_t)e.e;
        }
        return status_of(e);
    }
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

}  // extern "C"
