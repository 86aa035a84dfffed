// k-nearest-neighbour search over the cell grid, fused with the per-point
// covariance and its scale regularisation (Sec. 3: covariance of the k nearest
// neighbours; Sec. 3.1.1: C = R Lambda^2 R^T, plane and ellipse forms).
//
// A group of four consecutive lanes serves one query: the lanes split the
// candidates of the 27-cell block evenly, each keeps its own best candidates
// in registers as 64-bit (FP32 key, original index) words, sorted, inserted
// with an unrolled min/max sweep, and the four lists are merged through LDS.
// Queries of the self k-NN are the cell-sorted points themselves, so the
// groups of a wavefront visit the same cells and the candidate reads are
// served by the vector L1/L2.  After the 27-cell block the group proves
// exactness (the k-th key is below the squared clearance of the scanned
// block); otherwise it scans the next shell of cells, and after kMaxShell
// shells the query goes to a whole-cloud scan by one workgroup.
#include <float.h>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

// Sorted list of the best candidates as words (FP32 key, original index; the
// word encoding orders like doubles).  For a runtime k < K the first
// K - k slots hold zero words (+0.0), which sort before every candidate and
// never move, so the k best always occupy slots [K - k, K) and the k-th best
// is the last slot (a static register index).
template <int K>
struct TopK {
    uint64_t v[K];
    __device__ __forceinline__ void init(int k) {
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = (j < K - k) ? 0ull : kEmptyWord;
    }
    // One sweep from the front: slot j keeps min(v[j], t) and max(v[j], t)
    // moves on, which places x and drops the largest word, two instructions
    // per slot.  The min and max are written as v_min_f64 / v_max_f64 on the
    // raw registers: as doubles, the words (no NaN, no denormal) compare
    // exactly like the integers, and the compiler's own fmin / fmax would
    // first quieten every operand.
    __device__ __forceinline__ void insert(uint64_t x) {
        if (x >= v[K - 1]) return;
        uint64_t t = x;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            uint64_t hi;
            asm("v_max_f64 %0, %1, %2" : "=v"(hi) : "v"(v[j]), "v"(t));
            asm("v_min_f64 %0, %0, %1" : "+v"(v[j]) : "v"(t));
            t = hi;
        }
    }
};

// Scan the cnt cell-sorted points from `start` into the top-k, their loads
// issued four at a time (a cell's points are contiguous), so that a run of
// candidates costs a quarter of the dependent memory round trips.
template <int K>
__device__ __forceinline__ void scan_run(const GridView& g, uint32_t start, uint32_t cnt, float qx, float qy,
                                         float qz, float gate2, TopK<K>& top) {
    for (uint32_t i0 = 0; i0 < cnt; i0 += 4) {
        float4 pp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pp[u] = g.spts[start + (i0 + u < cnt ? i0 + u : 0u)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float d2 = rank_key(qx, qy, qz, pp[u].x, pp[u].y, pp[u].z);
            if (i0 + u < cnt && d2 <= gate2) top.insert(word(d2, __float_as_uint(pp[u].w)));
        }
    }
}

// Scan one cell into the top-k.
template <int K>
__device__ __forceinline__ void scan_cell(const GridView& g, uint32_t key, float qx, float qy, float qz,
                                          float gate2, TopK<K>& top) {
    uint32_t start = 0;
    const uint32_t cnt = cell_lookup(g.table, g.mask, key, start);
    scan_run<K>(g, start, cnt, qx, qy, qz, gate2, top);
}

// Current pruning bound: the k-th key once the list is full (else +inf),
// capped by the gate.
template <int K>
__device__ __forceinline__ float prune_bound(const TopK<K>& top, float gate2) {
    const uint64_t w = top.v[K - 1];
    const float kth = (w == kEmptyWord) ? FLT_MAX : word_key(w);
    return fminf(kth, gate2);
}

// Publish the lanes' sorted lists in `lists` (LDS, [kGroup][K]) and merge
// them into every lane's `top`.  A word present in several lists (the
// common prefix the lanes started a shell from) is taken once.
template <int K>
__device__ __forceinline__ void merge_lists(TopK<K>& top, int k, int l, uint64_t* lists) {
#pragma unroll
    for (int j = 0; j < K; ++j) lists[l * K + j] = top.v[j];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the real entries of every list sit in [K - k, K)
    int h0 = K - k, h1 = K - k, h2 = K - k, h3 = K - k;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < K - k) continue;   // dummy slots keep their zero words
        const uint64_t a0 = h0 < K ? lists[0 * K + h0] : kEmptyWord;
        const uint64_t a1 = h1 < K ? lists[1 * K + h1] : kEmptyWord;
        const uint64_t a2 = h2 < K ? lists[2 * K + h2] : kEmptyWord;
        const uint64_t a3 = h3 < K ? lists[3 * K + h3] : kEmptyWord;
        const uint64_t m = wmin(wmin(a0, a1), wmin(a2, a3));
        top.v[j] = m;
        h0 += (m == a0) ? 1 : 0;
        h1 += (m == a1) ? 1 : 0;
        h2 += (m == a2) ? 1 : 0;
        h3 += (m == a3) ? 1 : 0;
    }
    // the next publication overwrites the lists: every lane has read them
    __builtin_amdgcn_wave_barrier();
}

constexpr int kShellBatch = 8;   // table slots loaded together per lane in a batched shell scan

// Exact k-NN of q by a group of kGroup consecutive lanes (lane l; all hold
// q).  The lanes look up every kGroup-th cell of the 27-cell block (a cell
// whose distance lower bound exceeds the gate counts as empty), then split
// the block's candidates evenly: each lane fills its own top-k from a
// contiguous quarter of them, and the four lists are merged, so the group
// continues converged.  Exactness is then proven from the block clearance;
// otherwise the lanes split the cells of the next shell (every kGroup-th
// cell, skipping those beyond the current k-th key or the gate), starting
// from the merged list, and merge again.  Returns false when max_shell shells
// did not prove the result exact: the caller then hands the query on (to a
// later pass or to a whole-cloud scan).
template <int K>
__device__ __forceinline__ bool knn_search(const GridView& g, float h, float inv_h, uint32_t prefix, float qx,
                                           float qy, float qz, int k, float gate2, float r_gate, TopK<K>& top, int l,
                                           uint64_t* lists, int max_shell = kMaxShell, bool batched_shells = false) {
    top.init(k);
    const bool fin = finite3(qx, qy, qz);   // a non-finite query has no neighbour with a finite distance
    const Cell c = cell_of(fin ? qx : 0.f, fin ? qy : 0.f, fin ? qz : 0.f, inv_h);
    const float slack = cell_slack(qx, qy, qz, kMaxShell, h);
    if (fin) {
        // the lane's cells of the 27-cell block: all table slots are loaded
        // first, so the lookups' latencies overlap
        constexpr int kPer = (27 + kGroup - 1) / kGroup;
        uint4 ent[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = l + kGroup * q;
            ent[q] = make_uint4(kEmptyKey, 0u, 0u, 0u);
            if (j < 27) {
                int dx, dy, dz;
                block_offset(j, dx, dy, dz);
                const uint32_t key = prefix | cell_key(c.x + dx, c.y + dy, c.z + dz);
                ent[q] = g.table[hash_slot(key, g.mask)];
            }
        }
        // resolve them to (start, count); cells beyond the gate count 0
        uint32_t st[kPer], ct[kPer];
        uint32_t total = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = l + kGroup * q;
            st[q] = 0;
            ct[q] = 0;
            if (j < 27) {
                int dx, dy, dz;
                block_offset(j, dx, dy, dz);
                const float lb = cell_lower_bound2(qx, qy, qz, c.x + dx, c.y + dy, c.z + dz, h, slack);
                if (!cell_pruned(lb, gate2)) {
                    const uint32_t key = prefix | cell_key(c.x + dx, c.y + dy, c.z + dz);
                    if (ent[q].x == key) {
                        st[q] = ent[q].y;
                        ct[q] = ent[q].z;
                    } else if (ent[q].x != kEmptyKey) {
                        // another key in the slot: probe on
                        ct[q] = cell_lookup(g.table, g.mask, key, st[q]);
                    }
                }
            }
            total += ct[q];
        }
        // The group's non-empty cells, compacted lane by lane into the group's
        // words of `lists` (free until the merge below): entry order is lane 0's
        // cells, then lane 1's, ...  The concatenated candidates of all the
        // cells are then split evenly over the four lanes (lane l takes
        // positions [l T / 4, (l + 1) T / 4) of the T candidates), so that the
        // lanes of a query do equal work whatever the cells' counts.
        static_assert(kGroup == 4 && K * kGroup > 27, "the group's cells fit its list words");
        int nz = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) nz += ct[q] > 0u ? 1 : 0;
        const int lane0 = (int)(threadIdx.x & 63u) & ~(kGroup - 1);
        uint32_t cnt_of[kGroup];   // candidates of each lane's cells
        int nz_of[kGroup];         // non-empty cells of each lane
#pragma unroll
        for (int m = 0; m < kGroup; ++m) {
            cnt_of[m] = (uint32_t)__shfl((int)total, lane0 + m, 64);
            nz_of[m] = __shfl(nz, lane0 + m, 64);
        }
        uint32_t S[kGroup + 1];   // candidates before lane m's cells
        int E[kGroup + 1];        // entries before lane m's cells
        S[0] = 0;
        E[0] = 0;
#pragma unroll
        for (int m = 0; m < kGroup; ++m) {
            S[m + 1] = S[m] + cnt_of[m];
            E[m + 1] = E[m] + nz_of[m];
        }
        {
            int w = l == 0 ? E[0] : l == 1 ? E[1] : l == 2 ? E[2] : E[3];
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                if (ct[q] > 0u) {
                    lists[w] = ((uint64_t)ct[q] << 32) | (uint64_t)st[q];
                    ++w;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t T = S[kGroup];
        const uint32_t a0 = (T * (uint32_t)l) / kGroup, a1 = (T * (uint32_t)(l + 1)) / kGroup;
        const uint32_t n = a1 - a0;
        uint32_t cs = 0, cl = 0;   // position and remaining count in the current cell
        int e = 0;                 // the current entry
        if (n > 0) {
            // the entry holding position a0: first the lane block, then the cell
            const int m = (a0 >= S[1] ? 1 : 0) + (a0 >= S[2] ? 1 : 0) + (a0 >= S[3] ? 1 : 0);
            const uint32_t sm = m == 0 ? S[0] : m == 1 ? S[1] : m == 2 ? S[2] : S[3];
            const int em = m == 0 ? E[0] : m == 1 ? E[1] : m == 2 ? E[2] : E[3];
            uint32_t r = a0 - sm;
            e = em;
            while (true) {
                const uint64_t x = lists[e];
                const uint32_t c = (uint32_t)(x >> 32);
                if (r < c) {
                    cs = (uint32_t)x + r;
                    cl = c - r;
                    break;
                }
                r -= c;
                ++e;
            }
        }
        // one flat loop over the lane's n candidates, four a trip, their
        // loads issued together; the next entry is read ahead (the slot after
        // the last entry is never consumed)
        uint64_t nxt = lists[e + 1];
        for (uint32_t j0 = 0; j0 < n; j0 += 4) {
            uint32_t pos[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool valid = j0 + u < n;
                if (valid && cl == 0) {
                    cs = (uint32_t)nxt;
                    cl = (uint32_t)(nxt >> 32);
                    ++e;
                    nxt = lists[e + 1];
                }
                pos[u] = valid ? cs : 0u;   // position 0 exists whenever n > 0
                cs += valid ? 1u : 0u;
                cl -= valid ? 1u : 0u;
            }
            float4 pp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pp[u] = g.spts[pos[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float d2 = rank_key(qx, qy, qz, pp[u].x, pp[u].y, pp[u].z);
                const uint64_t w = word(d2, __float_as_uint(pp[u].w));   // keeps the four loads whole
                if (j0 + u < n && d2 <= gate2) top.insert(w);
            }
        }
        // every lane has read the entries before the merge reuses the words
        __builtin_amdgcn_wave_barrier();
    }
    merge_lists<K>(top, k, l, lists);
    if (!fin) return true;
    for (int R = 1;; ++R) {
        const float clr = block_clearance(qx, qy, qz, c, R, h);
        if (clr > 0.f) {
            if (clr >= r_gate) return true;   // every point within the gate has been seen
            const uint64_t kth = top.v[K - 1];
            if (kth != kEmptyWord) {
                const float kkey = word_key(kth);
                if (kkey < clr * clr * (1.f - 1e-6f)) return true;
            }
        }
        if (R >= max_shell) return false;
        // shell S = R + 1: the cells at Chebyshev distance S, every kGroup-th
        // one per lane (positions of the (2S+1)^3 cube, interior skipped)
        const int S = R + 1, W = 2 * S + 1;
        if (!batched_shells) {
            for (int t = l; t < W * W * W; t += kGroup) {
                const int dx = t % W - S, dy = (t / W) % W - S, dz = t / (W * W) - S;
                if (max(max(abs(dx), abs(dy)), abs(dz)) != S) continue;
                const float lb = cell_lower_bound2(qx, qy, qz, c.x + dx, c.y + dy, c.z + dz, h, slack);
                if (cell_pruned(lb, prune_bound(top, gate2))) continue;
                scan_cell<K>(g, prefix | cell_key(c.x + dx, c.y + dy, c.z + dz), qx, qy, qz, gate2, top);
            }
        } else {
            // up to kShellBatch unpruned cells of the lane at a time: their
            // table slots are loaded together, then the cells are scanned
            int t = l;
            while (t < W * W * W) {
                uint4 ent[kShellBatch];
                uint32_t key[kShellBatch];
#pragma unroll
                for (int b = 0; b < kShellBatch; ++b) {
                    key[b] = kEmptyKey;
                    while (t < W * W * W) {
                        const int dx = t % W - S, dy = (t / W) % W - S, dz = t / (W * W) - S;
                        t += kGroup;
                        if (max(max(abs(dx), abs(dy)), abs(dz)) != S) continue;
                        const float lb = cell_lower_bound2(qx, qy, qz, c.x + dx, c.y + dy, c.z + dz, h, slack);
                        if (cell_pruned(lb, prune_bound(top, gate2))) continue;
                        key[b] = prefix | cell_key(c.x + dx, c.y + dy, c.z + dz);
                        ent[b] = g.table[hash_slot(key[b], g.mask)];
                        break;
                    }
                }
#pragma unroll
                for (int b = 0; b < kShellBatch; ++b) {
                    if (key[b] == kEmptyKey) continue;
                    uint32_t start = ent[b].y, cnt = ent[b].z;
                    if (ent[b].x != key[b]) {
                        cnt = 0;
                        if (ent[b].x != kEmptyKey) cnt = cell_lookup(g.table, g.mask, key[b], start);
                    }
                    scan_run<K>(g, start, cnt, qx, qy, qz, gate2, top);
                }
            }
        }
        merge_lists<K>(top, k, l, lists);
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

// Scale regularisation of a raw covariance (Sec. 3.1.1).  out: xx,xy,xz,yy,yz,zz.
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

// Threads per workgroup of the k-NN kernels: the lane lists take
// threads * K * 8 bytes of LDS, kept within 64 KiB.
template <int K>
constexpr int knn_threads() {
    return K <= 32 ? 256 : 128;
}

// Covariance from the shifted moments m = (sum d, sum d d^T (xx,xy,xz,yy,yz,zz),
// count) with the 1/k normalisation and the neighbourhood mean.
__device__ __forceinline__ Sym3 moments_to_cov(const float m[10]) {
    const float ik = 1.f / fmaxf(m[9], 1.f);
    const float mx = m[0] * ik, my = m[1] * ik, mz = m[2] * ik;
    Sym3 C;
    C.a00 = m[3] * ik - mx * mx;
    C.a01 = m[4] * ik - mx * my;
    C.a02 = m[5] * ik - mx * mz;
    C.a11 = m[6] * ik - my * my;
    C.a12 = m[7] * ik - my * mz;
    C.a22 = m[8] * ik - mz * mz;
    return C;
}

// Moments of one neighbour slot, shifted by the query point.
__device__ __forceinline__ void add_moments(float m[10], uint64_t v, const float* __restrict__ xyz, int64_t stride,
                                            float qx, float qy, float qz) {
    const uint32_t id = (uint32_t)(v & 0xFFFFFFFFu);
    const float dx = xyz[id] - qx, dy = xyz[stride + id] - qy, dz = xyz[2 * stride + id] - qz;
    m[0] += dx; m[1] += dy; m[2] += dz;
    m[3] += dx * dx; m[4] += dx * dy; m[5] += dx * dz;
    m[6] += dy * dy; m[7] += dy * dz; m[8] += dz * dz;
    m[9] += 1.f;
}

// Raw covariance of the k neighbours in `top` (moments shifted by the query
// point q, which is itself a neighbour), by one thread, in the summation
// order of the lane-group version below (four strided partial sums combined
// as (s0 + s1) + (s2 + s3)), so that a point gets the same bits whichever
// pass finds its neighbours.
template <int K>
__device__ __forceinline__ Sym3 raw_from_topk(const TopK<K>& top, int k, const float* __restrict__ xyz,
                                              int64_t stride, float qx, float qy, float qz) {
    float part[kGroup][10];
#pragma unroll
    for (int l = 0; l < kGroup; ++l) {
#pragma unroll
        for (int c = 0; c < 10; ++c) part[l][c] = 0.f;
#pragma unroll
        for (int jj = 0; jj < K / kGroup; ++jj) {
            const int j = kGroup * jj + l;
            // a slot stays empty only when fewer than k neighbours have a
            // finite distance (non-finite input, reported through the error word)
            if (j >= K - k && top.v[j] != kEmptyWord) add_moments(part[l], top.v[j], xyz, stride, qx, qy, qz);
        }
    }
    float m[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) m[c] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
    return moments_to_cov(m);
}

__device__ __forceinline__ void store_cov(const float out[6], float* __restrict__ covs, float* __restrict__ covs_sorted,
                                          int64_t cstride, uint32_t orig, int32_t s) {
    if (covs) {
#pragma unroll
        for (int c = 0; c < 6; ++c) covs[(int64_t)c * cstride + orig] = out[c];
    }
    if (covs_sorted) {
#pragma unroll
        for (int c = 0; c < 6; ++c) covs_sorted[(int64_t)c * cstride + s] = out[c];
    }
}

// Slot 4*jj + l of the (group-uniform) sorted list, picked without dynamic
// register indexing.
template <int K>
__device__ __forceinline__ uint64_t lane_slot(const TopK<K>& top, int jj, int l) {
    const uint64_t a = top.v[4 * jj], b = top.v[4 * jj + 1], c = top.v[4 * jj + 2], d = top.v[4 * jj + 3];
    return l == 0 ? a : l == 1 ? b : l == 2 ? c : d;
}

// Raw covariance of the group's (uniform) top-k: every lane sums the moments
// of a quarter of the slots, and the four partial sums are combined across
// the group's lanes.
template <int K>
__device__ __forceinline__ Sym3 raw_from_topk_group(const TopK<K>& top, int k, int l, const float* __restrict__ xyz,
                                                    int64_t stride, float qx, float qy, float qz) {
    static_assert(K % kGroup == 0, "list length must split over the group lanes");
    float m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int jj = 0; jj < K / kGroup; ++jj) {
        const uint64_t v = lane_slot<K>(top, jj, l);
        if (kGroup * jj + l >= K - k && v != kEmptyWord) add_moments(m, v, xyz, stride, qx, qy, qz);
    }
    // lane l holds s_l; after the two exchanges every lane holds
    // (s0 + s1) + (s2 + s3) (additions commute bit for bit)
#pragma unroll
    for (int c = 0; c < 10; ++c) {
        m[c] += __shfl_xor(m[c], 1);
        m[c] += __shfl_xor(m[c], 2);
    }
    return moments_to_cov(m);
}

// Raw covariances go to `raw`, laid out per cloud as SoA [6][n] at 6 * off
// (cell order); the regularisation pass turns them into the outputs.
__device__ __forceinline__ void store_raw(const Sym3& C, float* __restrict__ raw, const Seg& sg, int64_t s) {
    float* r = raw + 6 * sg.off + (s - sg.off);
    r[0] = C.a00;
    r[sg.n] = C.a01;
    r[2 * sg.n] = C.a02;
    r[3 * sg.n] = C.a11;
    r[4 * sg.n] = C.a12;
    r[5 * sg.n] = C.a22;
}

// Work lists of the self k-NN: [0] retry count, [1] overflow count, then the
// retry list (n entries) and the overflow list (n entries).
__device__ __forceinline__ void push_work(int32_t* work, int64_t n, int which, int64_t s) {
    int32_t* list = work + 2 + which * n;
    list[atomicAdd(&work[which], 1)] = (int32_t)s;
}

// Gate of the first pass, as a multiple of the cell size: the cell is about
// 1.2 times the 75th-percentile k-th neighbour distance, so most points find their k
// neighbours inside it.
constexpr float kGateCells = 1.25f;

// Self k-NN + raw covariance, first pass.  A group of kGroup lanes serves one
// cell-sorted point.  Only candidates inside a key gate of (kGateCells h)^2
// enter the lists, which removes most insertions; the result is exact whenever
// the list fills up (every point ranked before the k-th then lies inside the
// gate and was seen).  Points whose list does not fill, or whose search did
// not finish, go to the retry list.
template <int K>
__global__ __launch_bounds__(knn_threads<K>()) void k_knn_cov(GridView g, SegSet S, int k, float* __restrict__ raw,
                                                              int32_t* __restrict__ work) {
    constexpr int kT = knn_threads<K>();
    __shared__ uint64_t s_lists[kT / kGroup][kGroup * K];
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t s = (int64_t)blockIdx.x * (kT / kGroup) + threadIdx.x / kGroup;
    if (s >= g.n) return;   // uniform over each lane group
    const int p = S.of_key(g.skeys[s]);
    const Seg sg = S.get(p);
    const float4 q = g.spts[s];
    const float gate = kGateCells * sg.h;
    const float gate2 = gate * gate;
    TopK<K> top;
    const bool ok = knn_search<K>(g, sg.h, sg.inv_h, (uint32_t)p << (3 * kCellBits), q.x, q.y, q.z, k, gate2,
                                  gate * 1.000001f + 1e-6f, top, l, s_lists[threadIdx.x / kGroup]);
    if (!ok || top.v[K - 1] == kEmptyWord) {
        if (l == 0) push_work(work, g.n, 0, s);
        return;
    }
    const Sym3 C = raw_from_topk_group<K>(top, k, l, sg.xyz, sg.n, q.x, q.y, q.z);
    if (l == 0) store_raw(C, raw, sg, s);
}

// Second pass over the retry list: the same search under a gate of
// kRetryGateCells cells.  The list is short, so its queries are spread one per
// workgroup of a small block first (query e goes to block e mod gridDim.x), to
// use every compute unit.  Points that still have fewer than k neighbours
// inside the gate (isolated points) or whose search did not finish go to the
// overflow list, whose whole-cloud scan needs no gate.
constexpr int kRetryThreads = 64;
constexpr float kRetryGateCells = 3.0f;

template <int K>
__global__ __launch_bounds__(kRetryThreads) void k_knn_cov_retry(GridView g, SegSet S, int k,
                                                                 float* __restrict__ raw,
                                                                 int32_t* __restrict__ work) {
    constexpr int kG = kRetryThreads / kGroup;
    __shared__ uint64_t s_lists[kG][kGroup * K];
    const int l = threadIdx.x & (kGroup - 1);
    const int grp = threadIdx.x / kGroup;
    const int count = work[0];
    const int32_t* list = work + 2;
    for (int64_t e = blockIdx.x + (int64_t)gridDim.x * grp; e < count; e += (int64_t)gridDim.x * kG) {
        const int64_t s = list[e];
        const int p = S.of_key(g.skeys[s]);
        const Seg sg = S.get(p);
        const float4 q = g.spts[s];
        TopK<K> top;
        const float gate = kRetryGateCells * sg.h;
        const float gate2 = gate * gate;
        if (!knn_search<K>(g, sg.h, sg.inv_h, (uint32_t)p << (3 * kCellBits), q.x, q.y, q.z, k, gate2,
                           gate * 1.000001f + 1e-6f, top, l, s_lists[grp], kMaxShell, true) ||
            top.v[K - 1] == kEmptyWord) {
            if (l == 0) push_work(work, g.n, 1, s);
            continue;
        }
        const Sym3 C = raw_from_topk_group<K>(top, k, l, sg.xyz, sg.n, q.x, q.y, q.z);
        if (l == 0) store_raw(C, raw, sg, s);
    }
}

// Regularisation pass, one lane per point in cell order: raw covariance ->
// scale-regularised covariance (Sec. 3.1.1), written in the cloud's order and,
// when requested, in cell order.
__global__ __launch_bounds__(kBlock) void k_cov_regularise(GridView g, SegSet S, int mode, float eps,
                                                           const float* __restrict__ raw) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n) return;
    const Seg sg = S.get(S.of_key(g.skeys[s]));
    const float* r = raw + 6 * sg.off + (s - sg.off);
    Sym3 C;
    C.a00 = r[0]; C.a01 = r[sg.n]; C.a02 = r[2 * sg.n]; C.a11 = r[3 * sg.n]; C.a12 = r[4 * sg.n]; C.a22 = r[5 * sg.n];
    float out[6];
    regularise(C, mode, eps, out);
    store_cov(out, sg.covs, sg.covs_sorted, sg.n, __float_as_uint(g.spts[s].w), (int32_t)(s - sg.off));
}

template <int K>
__device__ __forceinline__ void store_knn(const TopK<K>& top, int k, int64_t i, int32_t* __restrict__ idx,
                                          float* __restrict__ d2) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= K - k) {
            const uint64_t v = top.v[j];
            const bool ok = v != kEmptyWord;
            const int64_t o = i * k + (j - (K - k));
            idx[o] = ok ? (int32_t)(v & 0xFFFFFFFFu) : -1;
            d2[o] = ok ? word_key(v) : __builtin_inff();
        }
    }
}

template <int K>
__global__ __launch_bounds__(knn_threads<K>()) void k_knn_query(GridView g, float h, float inv_h,
                                                                const float* __restrict__ q, int64_t nq, int k,
                                                                float gate2, float r_gate, int32_t* __restrict__ idx,
                                                                float* __restrict__ d2,
                                                                int32_t* __restrict__ overflow) {
    constexpr int kT = knn_threads<K>();
    __shared__ uint64_t s_lists[kT / kGroup][kGroup * K];
    const int l = threadIdx.x & (kGroup - 1);
    const int64_t i = (int64_t)blockIdx.x * (kT / kGroup) + threadIdx.x / kGroup;
    if (i >= nq) return;   // uniform over each lane group
    const float qx = q[i], qy = q[nq + i], qz = q[2 * nq + i];
    TopK<K> top;
    if (!knn_search<K>(g, h, inv_h, 0u, qx, qy, qz, k, gate2, r_gate, top, l, s_lists[threadIdx.x / kGroup])) {
        if (l == 0) overflow[1 + atomicAdd(&overflow[0], 1)] = (int32_t)i;
        return;
    }
    if (l == 0) store_knn<K>(top, k, i, idx, d2);
}

// ---------------------------------------------------------------------------
// Overflow pass: the queries whose k-NN could not be proven exact from the
// grid shells.  One workgroup per query: every thread keeps the top-k of a
// strided slice of the whole cloud, then the lists are merged pairwise in LDS
// (log2(threads) rounds); thread 0 finishes the query.  Workgroups loop over
// the overflow list, whose length is read on the device.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void full_scan_topk(const GridView& g, int64_t lo, int64_t hi, float qx, float qy,
                                               float qz, int k, float gate2, TopK<K>& top, uint64_t* lists) {
    top.init(k);
    // eight points a trip, their loads issued together: a query scans the
    // whole cloud alone, so the loop is bound by memory round trips
    constexpr int kU = 8;
    const int64_t stride = blockDim.x;
    for (int64_t j0 = lo + threadIdx.x; j0 < hi; j0 += stride * kU) {
        float4 pp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t j = j0 + u * stride;
            pp[u] = g.spts[j < hi ? j : j0];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const float d2 = rank_key(qx, qy, qz, pp[u].x, pp[u].y, pp[u].z);
            if (j0 + u * stride < hi && d2 <= gate2) top.insert(word(d2, __float_as_uint(pp[u].w)));
        }
    }
    for (int half = blockDim.x / 2; half >= 1; half >>= 1) {
#pragma unroll
        for (int j = 0; j < K; ++j) lists[threadIdx.x * K + j] = top.v[j];
        __syncthreads();
        if (threadIdx.x < half) {
            const uint64_t* a = lists + threadIdx.x * K;
            const uint64_t* b = lists + (threadIdx.x + half) * K;
            int ha = K - k, hb = K - k;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (j < K - k) continue;
                const uint64_t va = ha < K ? a[ha] : kEmptyWord;
                const uint64_t vb = hb < K ? b[hb] : kEmptyWord;
                const bool ta = va <= vb;
                top.v[j] = ta ? va : vb;
                ha += ta ? 1 : 0;
                hb += ta ? 0 : 1;
            }
        }
        __syncthreads();
    }
}

template <int K>
__global__ __launch_bounds__(knn_threads<K>()) void k_knn_cov_overflow(GridView g, SegSet S, int k,
                                                                       float* __restrict__ raw,
                                                                       const int32_t* __restrict__ work) {
    __shared__ uint64_t s_lists[knn_threads<K>() * K];
    const int count = work[1];
    const int32_t* list = work + 2 + g.n;
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int64_t s = list[e];
        const int p = S.of_key(g.skeys[s]);
        const Seg sg = S.get(p);
        const float4 q = g.spts[s];
        TopK<K> top;
        full_scan_topk<K>(g, sg.off, sg.off + sg.n, q.x, q.y, q.z, k, FLT_MAX, top, s_lists);
        if (threadIdx.x == 0) store_raw(raw_from_topk<K>(top, k, sg.xyz, sg.n, q.x, q.y, q.z), raw, sg, s);
        __syncthreads();
    }
}

template <int K>
__global__ __launch_bounds__(knn_threads<K>()) void k_knn_query_overflow(GridView g, const float* __restrict__ q,
                                                                         int64_t nq, int k, float gate2,
                                                                         int32_t* __restrict__ idx,
                                                                         float* __restrict__ d2,
                                                                         const int32_t* __restrict__ overflow) {
    __shared__ uint64_t s_lists[knn_threads<K>() * K];
    const int count = overflow[0];
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int64_t i = overflow[1 + e];
        TopK<K> top;
        full_scan_topk<K>(g, 0, g.n, q[i], q[nq + i], q[2 * nq + i], k, gate2, top, s_lists);
        if (threadIdx.x == 0) store_knn<K>(top, k, i, idx, d2);
        __syncthreads();
    }
}

// Distance to the j-th neighbour of `ns` evenly strided samples among every
// `step`-th point of the cloud (brute force), one wavefront per sample: each
// lane keeps its 8 smallest keys over a strided slice, then the wavefront
// pops the smallest head j times (an upper bound of the true j-th when a lane
// held more than 8 of the j smallest; used only to size grid cells).
constexpr int kKthWaves = 4;

__global__ __launch_bounds__(64 * kKthWaves) void k_kth_distance(const KthJob* __restrict__ jobs, int samples,
                                                                 float* __restrict__ out_all) {
    // block -> (job, group of kKthWaves samples); one wavefront per sample
    const int per_job = (samples + kKthWaves - 1) / kKthWaves;
    const KthJob J = jobs[blockIdx.x / per_job];
    const float* __restrict__ xyz = J.xyz;
    const int64_t n = J.n, step = J.step;
    const int j = J.j, ns = J.ns;
    float* __restrict__ out = out_all + (int64_t)(blockIdx.x / per_job) * samples;
    const int sample = (blockIdx.x % per_job) * kKthWaves + threadIdx.x / 64;
    if (sample >= ns) return;   // uniform over the wavefront
    const int lane = threadIdx.x % 64;
    const int64_t qi = (int64_t)sample * n / ns;
    const float qx = xyz[qi], qy = xyz[n + qi], qz = xyz[2 * n + qi];
    float best[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) best[t] = FLT_MAX;
    for (int64_t i = lane * step; i < n; i += 64 * step) {
        const float d = rank_key(qx, qy, qz, xyz[i], xyz[n + i], xyz[2 * n + i]);
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
    int taken = 0;
    float kth = FLT_MAX;
    while (taken < j) {
        float m = best[0];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o));
        if (m == FLT_MAX) break;
        const bool mine = best[0] == m;
        taken += __popcll(__ballot(mine));
        kth = m;
        if (mine) {
#pragma unroll
            for (int t = 0; t < 7; ++t) best[t] = best[t + 1];
            best[7] = FLT_MAX;
        }
    }
    if (lane == 0) out[sample] = sqrtf(kth);
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

constexpr int kOverflowBlocks = 2048;

constexpr int kRetryBlocks = 1024;

template <int K>
hipError_t knn_cov_t(const GridView& g, const SegSet& S, int k, int mode, float eps, float* raw, int32_t* work,
                     hipStream_t s) {
    constexpr int kT = knn_threads<K>();
    const int per = kT / kGroup;
    hipLaunchKernelGGL(k_knn_cov<K>, dim3((g.n + per - 1) / per), dim3(kT), 0, s, g, S, k, raw, work);
    hipLaunchKernelGGL(k_knn_cov_retry<K>, dim3(kRetryBlocks), dim3(kRetryThreads), 0, s, g, S, k, raw, work);
    hipLaunchKernelGGL(k_knn_cov_overflow<K>, dim3(kOverflowBlocks), dim3(kT), 0, s, g, S, k, raw,
                       (const int32_t*)work);
    hipLaunchKernelGGL(k_cov_regularise, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, S, mode, eps,
                       (const float*)raw);
    return hipGetLastError();
}

template <int K>
hipError_t knn_query_t(const GridView& g, float h, const float* q, int64_t nq, int k, float gate2, float r_gate,
                       int32_t* idx, float* d2, int32_t* overflow, hipStream_t s) {
    constexpr int kT = knn_threads<K>();
    const int per = kT / kGroup;
    hipLaunchKernelGGL(k_knn_query<K>, dim3((unsigned)((nq + per - 1) / per)), dim3(kT), 0, s, g, h, 1.0f / h, q, nq,
                       k, gate2, r_gate, idx, d2, overflow);
    hipLaunchKernelGGL(k_knn_query_overflow<K>, dim3(kOverflowBlocks), dim3(kT), 0, s, g, q, nq, k, gate2, idx, d2,
                       (const int32_t*)overflow);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_knn_cov(const GridView& g, const SegSet& S, int k, int mode, float eps, float* raw, int32_t* work,
                          hipStream_t s) {
    if (g.n <= 0) return hipSuccess;
    if (k == 20) return knn_cov_t<20>(g, S, k, mode, eps, raw, work, s);
    if (k <= 8) return knn_cov_t<8>(g, S, k, mode, eps, raw, work, s);
    if (k <= 16) return knn_cov_t<16>(g, S, k, mode, eps, raw, work, s);
    if (k <= 32) return knn_cov_t<32>(g, S, k, mode, eps, raw, work, s);
    return knn_cov_t<64>(g, S, k, mode, eps, raw, work, s);
}

hipError_t launch_knn_query(const GridView& g, const Seg& cloud, const float* q, int64_t nq, int k, float r_max,
                            int32_t* idx, float* d2, int32_t* overflow, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    float gate2 = FLT_MAX, r_gate = FLT_MAX;
    if (r_max > 0.f) {
        gate2 = r_max * r_max;
        r_gate = r_max * 1.000001f + 1e-6f;
    }
    const float h = cloud.h;
    if (k == 20) return knn_query_t<20>(g, h, q, nq, k, gate2, r_gate, idx, d2, overflow, s);
    if (k <= 8) return knn_query_t<8>(g, h, q, nq, k, gate2, r_gate, idx, d2, overflow, s);
    if (k <= 16) return knn_query_t<16>(g, h, q, nq, k, gate2, r_gate, idx, d2, overflow, s);
    if (k <= 32) return knn_query_t<32>(g, h, q, nq, k, gate2, r_gate, idx, d2, overflow, s);
    return knn_query_t<64>(g, h, q, nq, k, gate2, r_gate, idx, d2, overflow, s);
}

hipError_t launch_kth_distance(const KthJob* jobs, int njobs, int samples, float* out, hipStream_t s) {
    const int per_job = (samples + kKthWaves - 1) / kKthWaves;
    hipLaunchKernelGGL(k_kth_distance, dim3(njobs * per_job), dim3(64 * kKthWaves), 0, s, jobs, samples, out);
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
