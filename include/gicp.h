/*
 * gicp.h — C ABI of the MI355X (gfx950) G-ICP tracking library, libgicp.so.
 *
 * The library computes the tracking step of "RGBD GS-ICP SLAM" (Ha, Yeon, Yu):
 *   1. k-nearest-neighbour search over a uniform-grid spatial hash built by
 *      radix sort (Sec. 3: the covariance of a point is the covariance matrix
 *      of its k nearest neighbours; correspondences come from nearest-
 *      neighbour search);
 *   2. per-point covariances with scale regularisation (Sec. 3.1.1, Scale
 *      Regularization: C = R Lambda^2 R^T; plane form with scales (1,1,eps),
 *      ellipse form with scales divided by their median);
 *   3. Gauss-Newton minimisation of the Mahalanobis objective of
 *      Eq. (MLE_for_T), sum_i d_i^T (C^t_i + R C^s_i R^T)^-1 d_i with
 *      d_i = x^t_i - T x^s_i, reduced per iteration to a 6x6 system.
 *
 * Conventions shared by every call
 * ---------------------------------
 * Points:        const float* xyz, structure of arrays [3][n]: x[0..n), then
 *                y[0..n), then z[0..n).  Device memory.
 * Covariances:   float* cov, structure of arrays [6][n] in the order
 *                xx, xy, xz, yy, yz, zz.  Device memory.
 * Pose:          double[16], 4x4 row-major, host memory; maps source (frame)
 *                coordinates into target (map) coordinates: q = R x + t.
 * H, b:          double[36] full symmetric row-major and double[6], host memory,
 *                in the tangent order [omega_x, omega_y, omega_z, v_x, v_y, v_z]
 *                of the left perturbation T <- Exp(xi) T.  They are the sums
 *                H = sum J^T M J, b = sum J^T M d of the last linearisation
 *                (the one that produced the final update), J = [[q]x, -I],
 *                M = (C^t + R C^s R^T)^-1.
 * Streams:       every call takes a hipStream_t (passed as void*; NULL is the
 *                default stream).  Calls that return device results are
 *                stream-ordered and do not synchronise the host unless stated.
 * Ownership:     every array argument is caller-owned and must stay valid
 *                until the stream work completes; the library never frees or
 *                retains a caller pointer past the call.  The library owns only
 *                gicp_ctx and gicp_map objects and their workspaces, which grow
 *                on demand and are reused (no allocation on a call whose sizes
 *                do not exceed the largest seen so far).
 * Threading:     a gicp_ctx is not thread-safe; use one per host thread.
 * Errors:        every call returns a gicp_status.  No C++ exception crosses
 *                the ABI.  Checks that need device data (non-finite inputs)
 *                are raised by the next synchronising call on the same
 *                context (gicp_register, gicp_sync_status).
 */
#ifndef GICP_H
#define GICP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gicp_status {
    GICP_OK = 0,
    GICP_E_ARG = 1,         /* null pointer, n < k, k outside [3,64] for a covariance ([1,64] for a
                               search), n <= 0, bad mode */
    GICP_E_NONFINITE = 2,   /* a NaN/Inf coordinate or covariance entry was seen */
    GICP_E_NO_CORR = 3,     /* fewer than 6 correspondences within r_max */
    GICP_E_DEGENERATE = 4,  /* Cholesky of H failed: a pivot <= 1e-12 * max(diag H) */
    GICP_E_OOM = 5,         /* device allocation failed */
    GICP_E_HIP = 6,         /* a HIP runtime call failed (code in gicp_stats.hip_error) */
    GICP_E_INEXACT = 7,     /* k-NN could not be proven exact (never expected; see gicp_knn) */
    GICP_E_TOO_LARGE = 8    /* input larger than the fixed workspace of gicp_covariances_noalloc */
} gicp_status;

typedef enum gicp_reg_mode {
    GICP_REG_NONE = 0,      /* raw k-NN covariance */
    GICP_REG_PLANE = 1,     /* eigenvalues replaced by (1, 1, eps): I - (1 - eps) n n^T (Sec. 3.1.1) */
    GICP_REG_ELLIPSE = 2    /* covariance divided by its middle eigenvalue (Sec. 3.1.1) */
} gicp_reg_mode;

typedef enum gicp_precision {
    GICP_ACC_TWOSUM = 0,    /* FP32 per point, compensated two-sum per lane and
                               wavefront, FP64 across wavefronts and blocks (default) */
    GICP_ACC_FP32 = 1,      /* FP32 per point, plain FP32 sums everywhere (study only) */
    GICP_ACC_FP64 = 2       /* FP32 per point, FP64 sums everywhere (study only) */
} gicp_precision;

typedef struct gicp_ctx gicp_ctx;
typedef struct gicp_map gicp_map;

typedef struct gicp_params {
    int32_t k;              /* neighbours per source covariance (self included), default 20 */
    float eps;              /* plane regularisation eps (covariance eigenvalue), default 1e-3 */
    float r_max;            /* correspondence gate in metres (inclusive: d^2 <= r_max^2), default 0.1 */
    int32_t max_it;         /* Gauss-Newton iterations, default 30 */
    double conv_rot;        /* stop when |omega| < conv_rot [rad] ... */
    double conv_trans;      /* ... and |v| < conv_trans [m]; 0 disables early exit */
    int32_t reg_mode;       /* gicp_reg_mode for source covariances computed by the call */
    float cell_src;         /* grid cell [m] for the source k-NN; <= 0: estimate (synchronises) */
    int32_t precision;      /* gicp_precision */
    int32_t flags;          /* GICP_FLAG_* */
    int32_t lanes;          /* lanes per source point in the linearisation: 2 or 4, or 0 for the
                               form's default (batched launches: 4 for a single problem, 2 for
                               several; work queue 4; gicp_track 4); the results do not depend
                               on it */
} gicp_params;

/* gicp_params.flags.  Default (0): each Gauss-Newton iteration of all the
 * call's problems is two launches (a linearisation launch over every chunk of
 * every unfinished problem, then one solve workgroup per problem), max_it
 * iterations per call; finished problems return at once. */
enum {
    /* One problem at a time, with a linearise and a solve launch per
     * iteration (the plain per-registration form; for comparison). */
    GICP_FLAG_MULTI_LAUNCH = 1,
    /* One persistent work-queue launch runs every iteration of every problem:
     * workers pop chunks, the last chunk of an iteration solves and posts the
     * problem's next iteration. */
    GICP_FLAG_QUEUE = 2,
    /* The default batched launches, with the max_it iterations recorded once
     * into a HIP graph (per batch shape and workspace) and replayed by one
     * graph launch.  Same kernels and results as the default form.  Kernel
     * timing, when enabled, covers the whole replay under group 0. */
    GICP_FLAG_GRAPH = 4,
    /* Search every correspondence afresh in every iteration.  By default a
     * point keeps its previous match while it stays within the radius that
     * match's search certified (no other mean can have become nearer), and a
     * search starts from the previous match as its first candidate; both
     * leave the exact nearest mean unchanged, so results are bitwise equal
     * with and without this flag (it exists to verify that, and costs the
     * full search in every iteration).  Combines with any form above. */
    GICP_FLAG_NO_REUSE = 8
};

/* One problem of a batched registration. */
typedef struct gicp_problem {
    const float* src;       /* SoA [3][n] source points (device) */
    const float* src_covs;  /* SoA [6][n] source covariances (device), or NULL: computed */
    int64_t n;
    const gicp_map* map;
    double init_pose[16];   /* row-major 4x4 (host) */
} gicp_problem;

typedef struct gicp_stats {
    int32_t iters;          /* Gauss-Newton iterations run */
    int32_t n_inliers;      /* correspondences in the last linearisation */
    double cost;            /* sum d^T M d of the last linearisation */
    int32_t converged;      /* 1 if the step fell below (conv_rot, conv_trans) */
    int32_t status;         /* gicp_status of the registration */
    int32_t hip_error;      /* hipError_t of the failing runtime call, else 0 */
    int32_t reserved;
} gicp_stats;

/* Fills a gicp_params with the defaults listed above. */
void gicp_params_default(gicp_params* p);

/* Library version string (static storage). */
const char* gicp_version(void);

/* Human-readable name of a status code (static storage). */
const char* gicp_strerror(int status);

/* Creates a context on HIP device `device` (it becomes current for the call).
 * Allocates a small fixed workspace; larger buffers grow on demand. */
int gicp_create(gicp_ctx** ctx, int device);
int gicp_destroy(gicp_ctx* ctx);

/* Synchronises `stream` and returns (then clears) any device-side error the
 * context recorded (GICP_E_NONFINITE) since the last synchronising call. */
int gicp_sync_status(gicp_ctx* ctx, void* stream);

/* Estimates a grid cell size for k-NN over `pts` (n points, SoA [3][n]):
 * the 75th percentile, over up to 256 evenly strided sample points, of the
 * distance to the k-th nearest neighbour (brute force), times 1.2.
 * Synchronises the stream; writes the result to *cell (host). */
int gicp_estimate_cell(gicp_ctx* ctx, const float* pts, int64_t n, int k, float* cell, void* stream);

/* k nearest neighbours of each query among `pts` (Sec. 3 nearest-neighbour
 * search).  Ranking key: the FP32 squared distance
 *   fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)),  dx = fl(q.x - p.x)
 * (round to nearest, no fused multiply-add), ties broken by the lower point
 * index.  Output row-major [nq][k]: idx (int32 point indices) and d2 (that
 * key).  Only neighbours with key <= fl(r_max*r_max) are reported when
 * r_max > 0; remaining slots hold idx -1 and d2 +inf.  `cell` is the grid cell
 * size in metres (<= 0: estimated, which synchronises).  The search visits grid
 * shells until the result is provably exact, then falls back to a full scan.
 * Returns GICP_E_ARG for null pointers, n < 1, nq < 0 or k outside [1,64]. */
int gicp_knn(gicp_ctx* ctx, const float* pts, int64_t n, const float* queries, int64_t nq,
             int k, float cell, float r_max, int32_t* idx, float* d2, void* stream);

/* Per-point covariances of `pts` from their k nearest neighbours, self
 * included (Sec. 3), with scale regularisation `reg_mode` (Sec. 3.1.1):
 * C = (1/k) sum_j (p_j - mu)(p_j - mu)^T over the neighbours, mu their mean;
 * PLANE: I - (1 - eps) n n^T with n the eigenvector of the smallest
 * eigenvalue; ELLIPSE: C / max(lambda_mid, 1e-6 lambda_max) (an all-zero C
 * stays zero).  Output covs SoA [6][n] (device).  Asynchronous.  `cell` as in
 * gicp_knn.  Returns GICP_E_ARG for null pointers, n < k or k outside [3,64]
 * (fewer than 3 neighbours give a covariance of rank 0 or 1, whose
 * regularised forms would fix an arbitrary direction). */
int gicp_covariances(gicp_ctx* ctx, const float* pts, int64_t n, int k, float cell,
                     int reg_mode, float eps, float* covs, void* stream);

/* gicp_covariances for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * gicp_covariances, but every workspace lives in one fixed device array of
 * the library (12.5 MiB per GPU, reserved when the library is loaded and held
 * until the process ends), and the call allocates nothing.
 *   n must not exceed GICP_NOALLOC_MAX_POINTS: larger inputs return
 *   GICP_E_TOO_LARGE.  cell <= 0 estimates the cell size, which synchronises
 *   the stream (and so cannot be captured); give cell > 0 for capture.
 * Every call on a GPU uses that GPU's one array, whatever the context: calls
 * that overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  The array keeps the last call's contents; each
 * call clears what it needs. */
#define GICP_NOALLOC_MAX_POINTS 131072
int gicp_covariances_noalloc(gicp_ctx* ctx, const float* pts, int64_t n, int k, float cell, int reg_mode,
                             float eps, float* covs, void* stream);

/* Builds a map handle from Gaussians (means SoA [3][m], covs SoA [6][m],
 * device): sorts them into grid cells of size `cell` (<= 0: estimated from
 * the 8-NN distance, which synchronises), builds the cell hash table, and
 * applies the target regularisation `reg_mode` (eps as above) once, so that
 * registrations against the map reuse it (Sec. 3: the map's covariances are
 * never recomputed; Sec. 3.1.1: target Gaussians are regularised for tracking).
 * The inputs may be freed once the stream has passed this call. */
int gicp_map_build(gicp_ctx* ctx, const float* means, const float* covs, int64_t m,
                   float cell, int reg_mode, float eps, gicp_map** out, void* stream);
int gicp_map_destroy(gicp_map* map);
/* Number of Gaussians and cell size of a map. */
int gicp_map_info(const gicp_map* map, int64_t* m, float* cell);

/* Nearest map mean of each query within r_max: the correspondence search of
 * the registration (Sec. 3: correspondences come from nearest-neighbour
 * search; Eq. MLE_for_T pairs each source point with one map Gaussian), run
 * by the same device code the Gauss-Newton iterations use, exposed so that
 * it can be checked and used on its own.
 *   queries  SoA [3][nq] (device), points already in the map frame (q = R x + t)
 *   r_max    gate in metres: a mean is accepted when its key <= fl(r_max * r_max)
 *   hints    nullable int32 [nq] (device): a map index per query tried as the
 *            first candidate (typically its previous match; -1 or an index
 *            outside [0, m): none).  A hint only speeds up the search; the
 *            result is the exact nearest mean either way.  The first call
 *            with hints on a map (and the first after gicp_map_insert)
 *            allocates and fills a 4-byte-per-Gaussian index table.
 *   idx      int32 [nq] (device): map index (order of gicp_map_build, then of
 *            the insertions) of the nearest mean by (FP32 key, index) as in
 *            gicp_knn, or -1 when none lies within the gate
 *   d2       float [nq] (device): that key, +inf when none
 *   radius   nullable float [nq] (device): a distance the query can move by
 *            (strictly less) without any other mean becoming nearer than the
 *            match, margins for FP32 rounding included -- the bound under
 *            which the registration keeps a match between iterations;
 *            -1 when there is no match or no margin
 *   lanes    lanes per query splitting its search: 0 or 2 (as in two-lane
 *            launches), 4, 8 or 16 (as in four-lane launches such as the
 *            tracking ones, whose searches of few points take 8 or 16 lanes);
 *            the matches and keys are the same, the radius may differ (each a
 *            valid bound)
 * Asynchronous.  GICP_E_ARG for null pointers, nq < 0, r_max <= 0 or lanes
 * outside {0, 2, 4, 8, 16}. */
int gicp_map_nearest(gicp_ctx* ctx, gicp_map* map, const float* queries, int64_t nq, float r_max,
                     const int32_t* hints, int32_t* idx, float* d2, float* radius, int32_t lanes,
                     void* stream);

/* Registers a source cloud against a map by Gauss-Newton on Eq. MLE_for_T.
 *   src        SoA [3][n] source points (device)
 *   src_covs   SoA [6][n] source covariances (device), or NULL: computed with
 *              params->k, params->reg_mode, params->eps, params->cell_src
 *   init_pose  initial T (host, row-major 4x4)
 *   pose, H, b outputs (host); pose holds the last valid iterate also when the
 *              status is GICP_E_NO_CORR or GICP_E_DEGENERATE
 *   src_covs_out  nullable SoA [6][n] (device): receives the covariances used
 *              (the ones the paper shares with the map)
 *   stats      nullable (host)
 * Per iteration: q_i = R x_i + t; the nearest map mean within r_max (exact,
 * ties to the lower map index); Sigma_i = C^t + R C^s_i R^T; accumulation of
 * H, b, e, n over inliers; then on the device an FP64 6x6 Cholesky solve,
 * xi = -H^-1 b, T <- Exp(xi) T, and the convergence test.  Synchronises the
 * stream once at the end (pose, H and b are host outputs).  Non-convergence
 * within max_it is not an error (stats->converged = 0). */
int gicp_register(gicp_ctx* ctx, const float* src, const float* src_covs, int64_t n,
                  const gicp_map* map, const double init_pose[16], const gicp_params* params,
                  double pose[16], double H[36], double b[6], float* src_covs_out,
                  gicp_stats* stats, void* stream);

/* gicp_register with the pose input and every output in device memory, for
 * callers that chain registrations on the device or capture them in a HIP
 * graph (Sec. 3, Eq. MLE_for_T: the same Gauss-Newton minimisation, the same
 * kernels and bitwise the same results as gicp_register).  Nothing is copied
 * to or from the host and the call does not synchronise the stream.
 *   init_pose  device double[16] (row-major), read when the stream reaches it
 *   pose, H, b device double[16], double[36] (full symmetric), double[6]
 *   stats      nullable device gicp_stats; stats->status carries the
 *              registration's status (GICP_E_NO_CORR, GICP_E_DEGENERATE, or
 *              GICP_E_NONFINITE for a non-finite input, which also stays
 *              recorded for the next gicp_sync_status)
 *   src_covs, src_covs_out  as gicp_register (device)
 * The return value reports only what the host can check (arguments, HIP
 * launch errors).  GICP_FLAG_GRAPH is refused (the call is itself meant for
 * capture); the default, GICP_FLAG_MULTI_LAUNCH and GICP_FLAG_QUEUE forms are
 * accepted.  For capture: params->cell_src > 0 (an estimated cell size
 * synchronises), and one call of at least the same sizes on the context
 * before capturing (its workspaces grow on demand, and an allocation cannot
 * be captured); a captured graph stays valid while no larger call on the
 * same context grows those workspaces. */
int gicp_register_dev(gicp_ctx* ctx, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                      const double* init_pose, const gicp_params* params, double* pose, double* H, double* b,
                      float* src_covs_out, gicp_stats* stats, void* stream);

/* Registers `nprob` independent problems in one call (same method and
 * parameters as gicp_register; problems may differ in size and map).  Source
 * covariances of all problems come from one segmented grid and one set of
 * k-NN launches; each Gauss-Newton iteration is one linearisation launch over
 * the 64-point work items of every unfinished problem and one solve
 * workgroup per problem, so problems finish at their own iteration counts
 * (params->flags selects the per-problem, work-queue or graph-replayed forms
 * described above, with identical results).  Outputs (host): poses [nprob][16],
 * Hs [nprob][36], bs [nprob][6] (each nullable), stats [nprob] (nullable).
 * Source covariances are computed first for problems whose src_covs is NULL.
 * Synchronises the stream once.  Returns GICP_E_ARG for nprob outside
 * [1, 4096] or an invalid problem; per-problem statuses are in stats. */
int gicp_register_batch(gicp_ctx* ctx, int nprob, const gicp_problem* probs, const gicp_params* params,
                        double* poses, double* Hs, double* bs, gicp_stats* stats, void* stream);

/* One frame of a tracked sequence. */
typedef struct gicp_frame {
    const float* src;       /* SoA [3][n] frame points in the camera frame (device) */
    const float* src_covs;  /* SoA [6][n] covariances (device), or NULL: computed */
    int64_t n;
} gicp_frame;

/* Motion models of gicp_track: the initial pose of frame i >= 1 is the
 * estimate of frame i-1 (PREVIOUS), or that estimate moved once more by the
 * last estimated relative motion, T_{i-1} T_{i-2}^-1 T_{i-1}
 * (CONSTANT_VELOCITY, from frame 2 on; frame 1 starts from frame 0's
 * estimate). */
enum { GICP_MOTION_PREVIOUS = 0, GICP_MOTION_CONSTANT_VELOCITY = 1 };

/* Frame-to-map tracking of a sequence (Sec. 3, Fig. 2: every frame is
 * registered against the map by G-ICP, Eq. MLE_for_T): the frames are
 * registered in order, each from an initial pose predicted on the device
 * from the estimates of the frames before it (`motion`), so that the whole
 * sequence runs without a host round trip between frames.  Frame 0 starts
 * from init_pose.  Covariances of frames without src_covs are computed first,
 * in batched launches (they do not depend on any pose).  Per frame the same
 * Gauss-Newton iterations as gicp_register, in one of three forms with equal
 * results.  Default: iteration slots -- (linearise, solve) launch pairs whose
 * frame the device picks; a frame's last solve predicts the next frame's pose
 * and moves the device on to it, so each frame costs exactly its own
 * iterations and the host launches pairs until the device reports (through
 * host-mapped memory) that every frame has finished, at most 16 pairs ahead
 * of it.  GICP_FLAG_MULTI_LAUNCH: max_it launch pairs per frame (pairs after
 * convergence return at once).  GICP_FLAG_GRAPH: those launches replayed
 * from one captured graph per frame.  GICP_FLAG_NO_REUSE as for
 * gicp_register; GICP_FLAG_QUEUE is refused.  Outputs (host): poses [nframes][16], Hs [nframes][36],
 * bs [nframes][6] (each nullable), stats [nframes] (nullable).  A frame whose
 * registration fails (NO_CORR, DEGENERATE) keeps its last valid iterate, and
 * the next frames predict from it.  Synchronises the stream once.
 * GICP_E_ARG for nframes outside [1, 4096], an invalid frame or motion. */
int gicp_track(gicp_ctx* ctx, int nframes, const gicp_frame* frames, const gicp_map* map,
               const double init_pose[16], int motion, const gicp_params* params, double* poses, double* Hs,
               double* bs, gicp_stats* stats, void* stream);

/* The problem statement form: builds a transient map from (map_means,
 * map_covs, m) with cell size `map_cell` (<= 0: estimated) and no target
 * regularisation, registers, and destroys the map. */
int gicp_register_pair(gicp_ctx* ctx, const float* src, const float* src_covs, int64_t n,
                       const float* map_means, const float* map_covs, int64_t m, float map_cell,
                       const double init_pose[16], const gicp_params* params,
                       double pose[16], double H[36], double b[6], gicp_stats* stats, void* stream);

/* Kernel timing.  While enabled, the context brackets its kernels with HIP
 * events on the stream they run on and accumulates, per kernel group, the
 * number of launches that did work, their summed duration and the work units
 * they processed.  Groups: 0 = correspondence + linearisation (unit: source
 * point per iteration), 1 = fused k-NN + covariance (unit: point), 2 = grid
 * build (cell keys, radix sort, cell table; unit: point), 3 = solve and update
 * (unit: iteration).  Durations are collected when the context synchronises
 * (gicp_register, gicp_sync_status).  gicp_profile(ctx, 1) enables and resets. */
enum { GICP_PROF_LINEARIZE = 0, GICP_PROF_KNN_COV = 1, GICP_PROF_GRID = 2, GICP_PROF_SOLVE = 3, GICP_PROF_GROUPS = 4 };
int gicp_profile(gicp_ctx* ctx, int enable);
int gicp_profile_read(gicp_ctx* ctx, int group, int64_t* launches, double* total_ms, double* units);

/* ------------------------------------------------------------------------
 * Frame preparation and map growth (Sec. 3 system overview; Sec. 3.1.2
 * Keyframe Selection; Sec. 3.2.1 Scale Aligning)
 * ------------------------------------------------------------------------ */

/* Depth image -> tracking point cloud (Sec. 3, Fig. 2: the depth image is
 * reprojected and downsampled).  depth: device float [height][width] in
 * metres; a pixel is valid when 0 < z <= max_depth and finite.  Pinhole
 * back-projection in FP32, x = (u - cx) z / fx, y = (v - cy) z / fy (each
 * operation rounded on its own); every occupied voxel (floor(x/voxel),
 * floor(y/voxel), floor(z/voxel)) yields the FP64 centroid of its points,
 * rounded to FP32.  Output: out_xyz, device SoA [3][*n_out] (stride *n_out),
 * voxels sorted by (ix, iy, iz); *n_out (host) the count.  Synchronises the
 * stream twice.  GICP_E_ARG when the count would exceed `capacity` points or
 * the occupied voxel box exceeds 2^32 - 1 voxels. */
int gicp_depth_to_points(gicp_ctx* ctx, const float* depth, int width, int height, float fx, float fy, float cx,
                         float cy, float voxel, float max_depth, float* out_xyz, int64_t capacity, int64_t* n_out,
                         void* stream);

/* The Gaussians a keyframe adds to the map (Sec. 3.1.2: only Gaussians that do
 * not overlap the current map; Sec. 3.2.1: scale aligning Lambda'' = Lambda' /
 * z^p, i.e. C'' = C' / z^(2p) with z the camera-frame depth).  src [3][n] and
 * src_covs [6][n] (device) are the frame's points and regularised
 * covariances in the camera frame; pose (host double[16]) maps camera to map.
 * A point overlaps when R x + t has a map mean within r_overlap (the FP32
 * correspondence test of the registration).  The non-overlapping points are
 * written in point order to out_means [3][n] / out_covs [6][n] (device, SoA
 * with stride n) as mu = R x + t and C = R C'' R^T (FP64 arithmetic); *n_out
 * (host) is their count and *inlier_ratio (host, nullable) the fraction of
 * points with a correspondence.  Synchronises the stream. */
int gicp_keyframe_gaussians(gicp_ctx* ctx, const float* src, const float* src_covs, int64_t n, const gicp_map* map,
                            const double pose[16], float r_overlap, float p, float* out_means, float* out_covs,
                            int64_t* n_out, double* inlier_ratio, void* stream);

/* Keyframe decision (Sec. 3.1.2 and Sec. 3.2.2, Additional Keyframe Selection for
 * Mapping): GICP_KEYFRAME when the correspondence ratio is below `threshold`
 * or `since_keyframe` >= max_gap (> 0); otherwise GICP_MAPPING_ONLY when
 * `since_mapping` (frames since the last keyframe of either kind) >=
 * mapping_gap (> 0); else 0.  Host-only. */
enum { GICP_KEYFRAME = 1, GICP_MAPPING_ONLY = 2 };
int gicp_keyframe_policy(double inlier_ratio, int since_keyframe, int since_mapping, double threshold, int max_gap,
                         int mapping_gap);

/* Adds m_new Gaussians (means [3][m_new], covariances [6][m_new], device,
 * map frame) to a map without re-sorting it: the new points are sorted on
 * their own and merged into the map's cell order (old points first among
 * equal cells), and the cell table is rebuilt from the merged keys.  Their
 * covariances get the regularisation the map was built with.  The result
 * equals gicp_map_build of the concatenation [old; new] (indices of new
 * points continue after the old ones).  May synchronise the stream when the
 * map's arrays grow. */
int gicp_map_insert(gicp_ctx* ctx, gicp_map* map, const float* means, const float* covs, int64_t m_new,
                    void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension: the paper starts every registration from
 * the previous pose).  A PointNet-style regressor maps a frame pair to its
 * relative pose, used as the initial pose of the registration; callers fall
 * back to the constant-velocity prediction when it fails.  Per pair, N =
 * GICP_MLP_POINTS rows X_r = [(s_r - c) * SCALE ; (t_r - c) * SCALE] (a chosen
 * source point, a chosen target point, c = mean of the chosen target points):
 *     H1 = relu(X W1 + b1) 6->64, H2 = relu(H1 W2 + b2) 64->128,
 *     H3 = relu(H2 W3 + b3) 128->256, g = max over rows of H3 (lowest row on
 *     ties), z = relu(g W4 + b4) 256->128, y = z W5 + b5 128->6.
 * y = [rotation vector ; translation (m)] of the relative pose in the centred
 * frame; in the original frame T = [R, t' - (R - I) c], R = exp([y0..2]x).
 * Loss: (1/B) sum_b 1/2 |y_b - y*_b|^2.  Adam (beta 0.9 / 0.999, eps 1e-8).
 * Precision: X, W1..W3 and H1, H2 stored as bf16; W2, W3 products on the
 * matrix cores with FP32 accumulation; everything else FP32.
 *
 * Buffers (device, caller-owned):
 *   params  float[GICP_MLP_PARAMS]  W1[6][64] b1[64] W2[64][128] b2[128]
 *           W3[128][256] b3[256] W4[256][128] b4[128] W5[128][6] b5[6]
 *   m, v    float[GICP_MLP_PARAMS]  Adam moments
 *   wbf16   uint16[GICP_MLP_BF16]   bf16 copies of W2, W3 in matrix-core
 *           fragment order, kept in step with params by the calls below
 *   X       uint16 (bf16 bits)[B][GICP_MLP_POINTS][6]
 *   cache   float[B][GICP_MLP_CACHE] forward values the backward pass needs
 * ------------------------------------------------------------------------ */
#define GICP_MLP_POINTS 4096
#define GICP_MLP_PARAMS 75462
#define GICP_MLP_BF16 40960
#define GICP_MLP_CACHE 640
#define GICP_MLP_SCALE 0.5
#define GICP_MLP_MAX_BATCH 4096

/* One pair for gicp_mlp_pack: device pointers; src_idx / tgt_idx hold
 * GICP_MLP_POINTS indices into the clouds (out-of-range indices are read as
 * 0 and reported as GICP_E_ARG by the next synchronising call). */
typedef struct gicp_mlp_pair {
    const float* src;        /* SoA [3][n_src] */
    int64_t n_src;
    const float* tgt;        /* SoA [3][n_tgt] */
    int64_t n_tgt;
    const int32_t* src_idx;  /* [GICP_MLP_POINTS] */
    const int32_t* tgt_idx;  /* [GICP_MLP_POINTS] */
} gicp_mlp_pair;

/* Draws the parameters: weight j of the flat vector is a (2u - 1) with
 * a = sqrt(6 / fan_in) and u = (SplitMix64(seed * 2^32 + j) >> 11) * 2^-53
 * (SplitMix64: Steele, Lea & Flood 2014); biases 0; m and v (nullable) 0;
 * fills wbf16. */
int gicp_mlp_init(gicp_ctx* ctx, uint64_t seed, float* params, float* m, float* v, uint16_t* wbf16, void* stream);
/* Refreshes wbf16 from params (after the caller changed params). */
int gicp_mlp_sync_weights(gicp_ctx* ctx, const float* params, uint16_t* wbf16, void* stream);
/* Packs B pairs (host array of descriptors, 1 <= B <= GICP_MLP_MAX_BATCH)
 * into X; centres (device double[B][3], nullable) receives c. */
int gicp_mlp_pack(gicp_ctx* ctx, int B, const gicp_mlp_pair* pairs, uint16_t* X, double* centres, void* stream);
/* Forward pass of B pairs: y (device float[B][6], nullable), cache (nullable;
 * required for gicp_mlp_backward), poses (device double[B][16], nullable:
 * the decoded relative poses, needs centres). */
int gicp_mlp_forward(gicp_ctx* ctx, int B, const uint16_t* X, const float* params, const uint16_t* wbf16,
                     const double* centres, float* y, float* cache, double* poses, void* stream);
/* Gradient of the loss against targets ystar (device float[B][6]) into grad
 * (device float[GICP_MLP_PARAMS], overwritten) and the loss (device float[1],
 * nullable).  Deterministic: per-pair gradients are summed in pair order. */
int gicp_mlp_backward(gicp_ctx* ctx, int B, const uint16_t* X, const float* params, const float* cache,
                      const float* y, const float* ystar, float* grad, float* loss, void* stream);
/* One Adam step (t = 1, 2, ...) with learning rate lr; refreshes wbf16. */
int gicp_mlp_adam_step(gicp_ctx* ctx, float* params, float* m, float* v, const float* grad, int t, float lr,
                       uint16_t* wbf16, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GICP_H */
