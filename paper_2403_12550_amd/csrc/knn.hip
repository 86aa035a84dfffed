// k-nearest-neighbour search over the cell grid, fused with the per-point
// covariance and its scale regularisation (Sec. 3: covariance of the k nearest
// neighbours; Sec. 3.1: C = R Lambda^2 R^T, plane and ellipse forms).
//
// One lane per query.  Queries of the self k-NN are the cell-sorted points
// themselves, so neighbouring lanes visit the same cells and the candidate
// reads are served by the vector L1/L2.  Each lane keeps its k best
// candidates in registers as 64-bit (FP32 key, original index) words, sorted,
// and inserts with an unrolled compare-exchange chain.  After the 27-cell
// block the lane proves exactness (the k-th key is below the squared
// clearance of the scanned block); otherwise it scans the next shell of cells,
// and after kMaxShell shells the whole cloud.
#include <float.h>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

// Sorted list of the best candidates as 64-bit (FP32 key, original index)
// words.  For a runtime k < K the first K - k slots hold zero words, which sort
// before every candidate and never move, so the k best always occupy slots
// [K - k, K) and the k-th best is the last slot (a static register index).
template <int K>
struct TopK {
    uint64_t v[K];
    __device__ __forceinline__ void init(int k) {
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = (j < K - k) ? 0ull : ~0ull;
    }
    __device__ __forceinline__ void insert(uint64_t x) {
        if (x >= v[K - 1]) return;
        v[K - 1] = x;
#pragma unroll
        for (int j = K - 1; j > 0; --j) {
            const uint64_t a = v[j - 1], b = v[j];
            const bool sw = b < a;
            v[j - 1] = sw ? b : a;
            v[j] = sw ? a : b;
        }
    }
};

// Scan one cell into the top-k.
template <int K>
__device__ __forceinline__ void scan_cell(const GridView& g, uint32_t key, float qx, float qy, float qz,
                                          float gate2, TopK<K>& top) {
    uint32_t start = 0;
    const uint32_t cnt = cell_lookup(g.table, g.mask, key, start);
    for (uint32_t j = 0; j < cnt; ++j) {
        const float4 p = g.spts[start + j];
        const float d2 = rank_key(qx, qy, qz, p.x, p.y, p.z);
        if (d2 <= gate2) top.insert(lex(d2, __float_as_uint(p.w)));
    }
}

// Current pruning bound: the k-th key once the list is full (else +inf),
// capped by the gate.
template <int K>
__device__ __forceinline__ float prune_bound(const TopK<K>& top, float gate2) {
    const uint64_t w = top.v[K - 1];
    const float kth = (w == ~0ull) ? FLT_MAX : __uint_as_float((uint32_t)(w >> 32));
    return fminf(kth, gate2);
}

// Exact k-NN of q.  The 27-cell block is visited nearest cell first, and a
// cell is skipped when its distance lower bound already exceeds the current
// k-th key (or the gate).  Exactness is then proven from the block clearance;
// otherwise the next shell of cells is visited (with the same pruning), and
// after kMaxShell shells the whole cloud is scanned.
template <int K>
__device__ __forceinline__ void knn_search(const GridView& g, float qx, float qy, float qz, int k, float gate2,
                                           float r_gate, TopK<K>& top) {
    top.init(k);
    if (!finite3(qx, qy, qz)) return;   // no neighbour has a finite distance
    const Cell c = cell_of(qx, qy, qz, g.inv_h);
    const float slack = cell_slack(qx, qy, qz, kMaxShell, g.h);
    for (int j = 0; j < 27; ++j) {
        int dx, dy, dz;
        block_offset(j, dx, dy, dz);
        const float lb = cell_lower_bound2(qx, qy, qz, c.x + dx, c.y + dy, c.z + dz, g.h, slack);
        if (cell_pruned(lb, prune_bound(top, gate2))) continue;
        scan_cell<K>(g, cell_key(c.x + dx, c.y + dy, c.z + dz), qx, qy, qz, gate2, top);
    }
    for (int R = 1;; ++R) {
        const float clr = block_clearance(qx, qy, qz, c, R, g.h);
        if (clr > 0.f) {
            if (clr >= r_gate) return;   // every point within the gate has been seen
            const uint64_t kth = top.v[K - 1];
            if (kth != ~0ull) {
                const float kkey = __uint_as_float((uint32_t)(kth >> 32));
                if (kkey < clr * clr * (1.f - 1e-6f)) return;
            }
        }
        if (R >= kMaxShell) break;
        const int S = R + 1;
        for (int dz = -S; dz <= S; ++dz)
            for (int dy = -S; dy <= S; ++dy)
                for (int dx = -S; dx <= S; ++dx) {
                    if (max(max(abs(dx), abs(dy)), abs(dz)) != S) continue;
                    const float lb = cell_lower_bound2(qx, qy, qz, c.x + dx, c.y + dy, c.z + dz, g.h, slack);
                    if (cell_pruned(lb, prune_bound(top, gate2))) continue;
                    scan_cell<K>(g, cell_key(c.x + dx, c.y + dy, c.z + dz), qx, qy, qz, gate2, top);
                }
    }
    // full scan (exact by construction)
    top.init(k);
    for (int32_t j = 0; j < g.n; ++j) {
        const float4 p = g.spts[j];
        const float d2 = rank_key(qx, qy, qz, p.x, p.y, p.z);
        if (d2 <= gate2) top.insert(lex(d2, __float_as_uint(p.w)));
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (a00..a22 on
// entry; eigenvalues on the diagonal and eigenvectors in the columns of V on
// exit).
struct Sym3 {
    float a00, a01, a02, a11, a12, a22;
};

__device__ __forceinline__ void jrot(float& app, float& aqq, float& apq, float& arp, float& arq, float& v0p,
                                     float& v0q, float& v1p, float& v1q, float& v2p, float& v2q) {
    if (apq == 0.f) return;
    const float theta = (aqq - app) / (2.f * apq);
    const float t = copysignf(1.f, theta) / (fabsf(theta) + sqrtf(fmaf(theta, theta, 1.f)));
    const float c = 1.f / sqrtf(fmaf(t, t, 1.f));
    const float s = t * c;
    const float tau = s / (1.f + c);
    app -= t * apq;
    aqq += t * apq;
    apq = 0.f;
    const float rp = arp, rq = arq;
    arp = rp - s * (rq + tau * rp);
    arq = rq + s * (rp - tau * rq);
    float p, q;
    p = v0p; q = v0q; v0p = p - s * (q + tau * p); v0q = q + s * (p - tau * q);
    p = v1p; q = v1q; v1p = p - s * (q + tau * p); v1q = q + s * (p - tau * q);
    p = v2p; q = v2q; v2p = p - s * (q + tau * p); v2q = q + s * (p - tau * q);
}

__device__ __forceinline__ void jacobi3(Sym3 a, float lam[3], float V[3][3]) {
    float v00 = 1, v01 = 0, v02 = 0, v10 = 0, v11 = 1, v12 = 0, v20 = 0, v21 = 0, v22 = 1;
    for (int sweep = 0; sweep < 10; ++sweep) {
        const float off = fabsf(a.a01) + fabsf(a.a02) + fabsf(a.a12);
        const float diag = fabsf(a.a00) + fabsf(a.a11) + fabsf(a.a22);
        if (off <= 1e-9f * diag || off < 1e-36f) break;
        // (p,q) = (0,1), r = 2
        jrot(a.a00, a.a11, a.a01, a.a02, a.a12, v00, v01, v10, v11, v20, v21);
        // (p,q) = (0,2), r = 1
        jrot(a.a00, a.a22, a.a02, a.a01, a.a12, v00, v02, v10, v12, v20, v22);
        // (p,q) = (1,2), r = 0
        jrot(a.a11, a.a22, a.a12, a.a01, a.a02, v01, v02, v11, v12, v21, v22);
    }
    lam[0] = a.a00; lam[1] = a.a11; lam[2] = a.a22;
    V[0][0] = v00; V[0][1] = v01; V[0][2] = v02;
    V[1][0] = v10; V[1][1] = v11; V[1][2] = v12;
    V[2][0] = v20; V[2][1] = v21; V[2][2] = v22;
}

// Scale regularisation of a raw covariance (Sec. 3.1).  out: xx,xy,xz,yy,yz,zz.
__device__ __forceinline__ void regularise(const Sym3& C, int mode, float eps, float out[6]) {
    if (mode == GICP_REG_NONE) {
        out[0] = C.a00; out[1] = C.a01; out[2] = C.a02; out[3] = C.a11; out[4] = C.a12; out[5] = C.a22;
        return;
    }
    float lam[3], V[3][3];
    jacobi3(C, lam, V);
    if (mode == GICP_REG_PLANE) {
        // smallest eigenvalue's eigenvector (first index on ties)
        int i0 = 0;
        if (lam[1] < lam[i0]) i0 = 1;
        if (lam[2] < lam[i0]) i0 = 2;
        float nx = (i0 == 0) ? V[0][0] : (i0 == 1) ? V[0][1] : V[0][2];
        float ny = (i0 == 0) ? V[1][0] : (i0 == 1) ? V[1][1] : V[1][2];
        float nz = (i0 == 0) ? V[2][0] : (i0 == 1) ? V[2][1] : V[2][2];
        const float inv = 1.f / sqrtf(nx * nx + ny * ny + nz * nz);
        nx *= inv; ny *= inv; nz *= inv;
        const float w = 1.f - eps;
        out[0] = 1.f - w * nx * nx;
        out[1] = -w * nx * ny;
        out[2] = -w * nx * nz;
        out[3] = 1.f - w * ny * ny;
        out[4] = -w * ny * nz;
        out[5] = 1.f - w * nz * nz;
        return;
    }
    // ellipse: divide by the middle eigenvalue (clamped at 1e-6 of the largest)
    const float lo = fminf(fminf(lam[0], lam[1]), lam[2]);
    const float hi = fmaxf(fmaxf(lam[0], lam[1]), lam[2]);
    const float mid = lam[0] + lam[1] + lam[2] - lo - hi;
    const float den = fmaxf(mid, 1e-6f * hi);
    const float s = den > 0.f ? 1.f / den : 0.f;
    out[0] = C.a00 * s; out[1] = C.a01 * s; out[2] = C.a02 * s;
    out[3] = C.a11 * s; out[4] = C.a12 * s; out[5] = C.a22 * s;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_knn_cov(GridView g, const float* __restrict__ xyz, int64_t stride,
                                                    int k, int mode, float eps, float* __restrict__ covs,
                                                    int64_t cstride) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    const float4 q = g.spts[s];
    const uint32_t orig = __float_as_uint(q.w);
    TopK<K> top;
    knn_search<K>(g, q.x, q.y, q.z, k, FLT_MAX, FLT_MAX, top);
    // one pass, shifted by the query point (which is itself a neighbour)
    float s1x = 0, s1y = 0, s1z = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
    int found = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        // a slot stays empty only when fewer than k neighbours have a finite
        // distance (non-finite input, reported through the error word)
        if (j >= K - k && top.v[j] != ~0ull) {
            const uint32_t id = (uint32_t)(top.v[j] & 0xFFFFFFFFu);
            const float dx = xyz[id] - q.x, dy = xyz[stride + id] - q.y, dz = xyz[2 * stride + id] - q.z;
            s1x += dx; s1y += dy; s1z += dz;
            sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
            syy += dy * dy; syz += dy * dz; szz += dz * dz;
            ++found;
        }
    }
    const float ik = 1.f / (float)max(found, 1);
    const float mx = s1x * ik, my = s1y * ik, mz = s1z * ik;
    Sym3 C;
    C.a00 = sxx * ik - mx * mx;
    C.a01 = sxy * ik - mx * my;
    C.a02 = sxz * ik - mx * mz;
    C.a11 = syy * ik - my * my;
    C.a12 = syz * ik - my * mz;
    C.a22 = szz * ik - mz * mz;
    float out[6];
    regularise(C, mode, eps, out);
#pragma unroll
    for (int c = 0; c < 6; ++c) covs[(int64_t)c * cstride + orig] = out[c];
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_knn_query(GridView g, const float* __restrict__ q, int64_t nq,
                                                      int k, float gate2, float r_gate, int32_t* __restrict__ idx,
                                                      float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const float qx = q[i], qy = q[nq + i], qz = q[2 * nq + i];
    TopK<K> top;
    knn_search<K>(g, qx, qy, qz, k, gate2, r_gate, top);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= K - k) {
            const uint64_t v = top.v[j];
            const bool ok = v != ~0ull;
            const int64_t o = i * k + (j - (K - k));
            idx[o] = ok ? (int32_t)(v & 0xFFFFFFFFu) : -1;
            d2[o] = ok ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
        }
    }
}

// Brute-force distance to the k-th neighbour of `ns` strided samples: one
// workgroup per sample, each lane keeps its own top-k over a strided slice,
// then lane 0 merges the slices through LDS.
__global__ __launch_bounds__(256) void k_kth_distance(const float* __restrict__ xyz, int64_t n, int k, int ns,
                                                      float* __restrict__ out) {
    __shared__ float s_keys[256 * 8];
    const int64_t qi = (int64_t)blockIdx.x * n / ns;
    const float qx = xyz[qi], qy = xyz[n + qi], qz = xyz[2 * n + qi];
    // each lane: its 8 smallest keys (k-th of the union is found by repeated
    // selection below; k <= 64 needs at most 8 per lane only if the k smallest
    // are spread, so lanes keep 8 and the merge is exact for k <= 8 per lane)
    float best[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) best[j] = FLT_MAX;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const float d = rank_key(qx, qy, qz, xyz[j], xyz[n + j], xyz[2 * n + j]);
        if (d < best[7]) {
            best[7] = d;
#pragma unroll
            for (int t = 7; t > 0; --t) {
                const float a = best[t - 1], b = best[t];
                best[t - 1] = fminf(a, b);
                best[t] = fmaxf(a, b);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) s_keys[threadIdx.x * 8 + j] = best[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        // k-th smallest of the 2048 lane candidates by repeated extraction
        // (an upper bound of the true k-th when a lane held more than 8 of the
        // k smallest; used only to size grid cells)
        float last = -1.f;
        int taken = 0;
        float kth = FLT_MAX;
        while (taken < k) {
            float m = FLT_MAX;
            int cnt = 0;
            for (int j = 0; j < 256 * 8; ++j) {
                const float v = s_keys[j];
                if (v > last && v < m) { m = v; cnt = 0; }
                if (v == m) ++cnt;
            }
            if (m == FLT_MAX) break;
            taken += cnt;
            last = m;
            kth = m;
        }
        out[blockIdx.x] = sqrtf(kth);
    }
}

__global__ void k_map_covs(const uint32_t* __restrict__ svals, int64_t m, const float* __restrict__ covs,
                           int64_t stride, int mode, float eps, float4* __restrict__ scov, int* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t v = svals[i];
    Sym3 C;
    C.a00 = covs[v];
    C.a01 = covs[stride + v];
    C.a02 = covs[2 * stride + v];
    C.a11 = covs[3 * stride + v];
    C.a12 = covs[4 * stride + v];
    C.a22 = covs[5 * stride + v];
    if (!(finite3(C.a00, C.a01, C.a02) && finite3(C.a11, C.a12, C.a22))) atomicOr(err, kErrNonFinite);
    float o[6];
    regularise(C, mode, eps, o);
    scov[2 * i] = make_float4(o[0], o[1], o[2], o[3]);
    scov[2 * i + 1] = make_float4(o[4], o[5], 0.f, 0.f);
}

template <int K>
hipError_t knn_cov_t(const GridView& g, const float* xyz, int64_t stride, int k, int mode, float eps, float* covs,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_knn_cov<K>, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, xyz, stride, k,
                       mode, eps, covs, (int64_t)g.n);
    return hipGetLastError();
}

template <int K>
hipError_t knn_query_t(const GridView& g, const float* q, int64_t nq, int k, float gate2, float r_gate,
                       int32_t* idx, float* d2, hipStream_t s) {
    hipLaunchKernelGGL(k_knn_query<K>, dim3((unsigned)((nq + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, q, nq, k,
                       gate2, r_gate, idx, d2);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_knn_cov(const GridView& g, const float* xyz, int64_t stride, int k, int mode, float eps,
                          float* covs, int* /*err*/, hipStream_t s) {
    if (g.n <= 0) return hipSuccess;
    if (k == 20) return knn_cov_t<20>(g, xyz, stride, k, mode, eps, covs, s);
    if (k <= 8) return knn_cov_t<8>(g, xyz, stride, k, mode, eps, covs, s);
    if (k <= 16) return knn_cov_t<16>(g, xyz, stride, k, mode, eps, covs, s);
    if (k <= 32) return knn_cov_t<32>(g, xyz, stride, k, mode, eps, covs, s);
    return knn_cov_t<64>(g, xyz, stride, k, mode, eps, covs, s);
}

hipError_t launch_knn_query(const GridView& g, const float* q, int64_t nq, int k, float r_max, int32_t* idx,
                            float* d2, int* /*err*/, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    float gate2 = FLT_MAX, r_gate = FLT_MAX;
    if (r_max > 0.f) {
        gate2 = r_max * r_max;
        r_gate = r_max * 1.000001f + 1e-6f;
    }
    if (k == 20) return knn_query_t<20>(g, q, nq, k, gate2, r_gate, idx, d2, s);
    if (k <= 8) return knn_query_t<8>(g, q, nq, k, gate2, r_gate, idx, d2, s);
    if (k <= 16) return knn_query_t<16>(g, q, nq, k, gate2, r_gate, idx, d2, s);
    if (k <= 32) return knn_query_t<32>(g, q, nq, k, gate2, r_gate, idx, d2, s);
    return knn_query_t<64>(g, q, nq, k, gate2, r_gate, idx, d2, s);
}

hipError_t launch_kth_distance(const float* xyz, int64_t n, int k, int ns, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_kth_distance, dim3(ns), dim3(256), 0, s, xyz, n, k, ns, out);
    return hipGetLastError();
}

hipError_t launch_map_covs(const uint32_t* svals, int64_t m, const float* covs, int64_t stride, int mode, float eps,
                           float4* scov, int* err, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_covs, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, svals, m, covs, stride, mode,
                       eps, scov, err);
    return hipGetLastError();
}

}  // namespace gicp
