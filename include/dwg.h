/*
 * dwg.h -- C ABI of libdwg, an MI355X (gfx950) implementation of the hot path of
 * "Diffusing Winding Gradients" (DWG, arXiv 2405.13839): the all-pairs generalized
 * winding number (GWN) dipole sum and its gradient at every input point, the screened
 * kernel, the mean-GWN iso-value, the normal update iterated to convergence, and the
 * initial normals (random, or proposed by a small MLP from k-nearest-neighbour features).
 *
 * Conventions shared by every call
 *  - Point arrays are planar ("SoA") float32 device arrays of shape [3][n]: x at [0,n),
 *    y at [n,2n), z at [2n,3n) -- a contiguous (3, n) torch tensor. Point counts are below
 *    2^31 (int32 point indices; some calls state tighter limits).
 *  - Every pointer argument is a DEVICE pointer to caller-owned memory unless it says
 *    "host". The library never allocates, frees or keeps caller memory.
 *  - Scratch memory comes only from the caller's workspace `ws` of `ws_bytes` bytes
 *    (device memory, 256-byte aligned); dwg_workspace_bytes() says how much is needed.
 *    Its contents on entry do not matter and on return are unspecified.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls marked
 *    "async" only enqueue work on that stream; the caller synchronises.
 *  - Every argument is validated before the first HIP call. Errors never throw; each call
 *    returns a dwg_status, and dwg_last_error() gives a thread-local detail string.
 *  - No global mutable state besides that error string: calls are re-entrant, and the
 *    same inputs, parameters and device give bitwise-identical outputs (no atomics take
 *    part in any floating-point sum).
 */
#ifndef DWG_H
#define DWG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dwg_status {
  DWG_OK = 0,
  DWG_NOT_CONVERGED = 1,  /* dwg_iterate: max_iters reached; outputs are valid */
  DWG_E_INVALID = -1,     /* NULL required pointer, bad size or parameter */
  DWG_E_WORKSPACE = -2,   /* ws_bytes smaller than dwg_workspace_bytes() */
  DWG_E_DEVICE = -3,      /* a HIP call failed (message in dwg_last_error) */
  DWG_E_NONFINITE = -4,   /* a non-finite statistic: an input held NaN/Inf */
  DWG_E_UNSUPPORTED = -5  /* the device is not gfx950 */
} dwg_status;

/* Kernel parameters (Sec. 4.2 Eq. 5 screening; Sec. 5.2 modified Poisson kernel and
 * octree traversal). */
typedef struct dwg_kernel_params {
  float lambda;    /* screening coefficient >= 0; 0 = plain GWN (Eq. 2-3) */
  float eps;       /* >= 0: global floor on the kernel radius (the "small constant") */
  int compensated; /* 1 = Kahan-compensated accumulation of per-tile partial sums */
  int split;       /* all-pairs source splits: 0 = automatic, else 1..64 */
  float tree_beta; /* 0 = exact all-pairs sum; >= 1 = octree traversal (Sec. 5.2) with
                      opening radius max(tree_beta * r, r + dmax) per node (paper: 2.3) */
  int tree_leaf;   /* octree leaf capacity: 0 = 32, else 1..1024 */
  int reserved[2]; /* must be zero */
} dwg_kernel_params;

/* Iteration parameters (Algorithm 1; Sec. 5.1 "Model-independent Parameters"). */
typedef struct dwg_iterate_params {
  int max_iters;   /* >= 1 */
  int fixed_iters; /* 1 = run exactly max_iters; 0 = stop at the convergence test */
  double eps_deg;  /* convergence threshold in degrees (paper: 0.1) */
  double top_frac; /* fraction of largest normal changes averaged (paper: 0.01), (0,1] */
} dwg_iterate_params;

/* Per-iteration statistics, all computed in FP64 on the device. */
typedef struct dwg_iter_stat {
  double wmean;        /* Eq. 6: mean GWN over the input points (the iso-value) */
  double top_mean_deg; /* mean of the ceil(top_frac*n) largest angle changes (deg) */
  double mean_chord;   /* (1/n) sum |n_i^(t) - n_i^(t-1)| */
  double gwn_ms;       /* duration of this iteration's all-pairs kernel (HIP events on the
                          caller's stream), milliseconds */
} dwg_iter_stat;

typedef enum dwg_init_kind {
  DWG_INIT_RANDOM = 0,  /* i.i.d. uniform unit normals (Algorithm 1) */
  DWG_INIT_MLP = 1,     /* learned from anchor features (extension) */
  DWG_INIT_PCA = 2,     /* smallest-eigenvalue eigenvector of the 16-NN covariance (Sec. 5.1) */
  DWG_INIT_GAUSS = 3    /* Gauss map p / |p| about the origin (Sec. 5.1) */
} dwg_init_kind;

/* Library version string (static storage). */
const char* dwg_version(void);
/* Name of a status code (static storage). */
const char* dwg_status_string(int status);
/* Detail of the last error on the calling thread (thread-local storage; "" if none). */
const char* dwg_last_error(void);

/* Workspace bytes needed by any call below for n_src sources and n_qry queries with these
 * kernel parameters (NULL = defaults). Returns 0 for invalid sizes. */
size_t dwg_workspace_bytes(int64_t n_src, int64_t n_qry, const dwg_kernel_params* kp);

/*
 * dwg_gwn_eval -- GWN values w(q) at m queries (Sec. 3 Eq. 2-3; Sec. 4.2 Eq. 5). async.
 *   For query q and source j with d = p_j - q, r = |d|: a pair with r == 0 contributes
 *   nothing; rho = max(r, delta_j, eps); s = sqrt(lambda);
 *   w(q) = sum_j a_j e^{-s r} (1 + s r) <d, n_j> / (4 pi rho^3).
 *   P, N: sources and their normals [3][n]; area: a_j [n]; delta: per-source radius [n]
 *   or NULL (= 0); Q: queries [3][m]; w: output [m]; wmean: output, one double = the FP64
 *   mean of w, or NULL.
 *   Errors: DWG_E_INVALID (NULL P/N/area/Q/w, n or m outside [1, 2^31), lambda or eps
 *   negative or not finite, nonzero reserved), DWG_E_WORKSPACE, DWG_E_DEVICE.
 */
dwg_status dwg_gwn_eval(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kp,
                        float* w, double* wmean, void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_gwn_grad -- w(q) and its gradient with respect to q, the normals held fixed
 * (Sec. 4.1), at m queries. async. Same inputs as dwg_gwn_eval; per pair
 *   grad += a_j e^{-s r} [ (3 (1 + s r) / r^2 [rho == r] + s^2) <d,n_j> d - (1 + s r) n_j ]
 *           / (4 pi rho^3),
 * the derivative of the piecewise w term (the clamp makes it jump at r = delta_j).
 * w: output [m] or NULL; grad: output [3][m]; wmean: output or NULL.
 */
dwg_status dwg_gwn_grad(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kp,
                        float* w, float* grad, double* wmean, void* ws, size_t ws_bytes,
                        void* stream);

/*
 * dwg_gwn_grad_static -- dwg_gwn_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, outputs and errors as dwg_gwn_grad minus ws / ws_bytes.
 * Scratch comes from a static device array of 64 MiB that each GPU holds from the first call
 * on it until the process ends; the call itself allocates nothing. Calls with a scratch need
 * above 64 MiB return DWG_E_INVALID (split = 0 halves the automatic source split until the
 * need fits; for scale, n = m = 650,000 fits all-pairs, n = m = 170,000 in octree mode). All calls on one GPU share that array: calls
 * that overlap in time on one GPU (several streams or threads) race and must be serialised by
 * the caller. async. Results agree with dwg_gwn_grad to rounding (the split may differ).
 */
dwg_status dwg_gwn_grad_static(const float* P, const float* N, const float* area, const float* delta,
                               int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kp,
                               float* w, float* grad, double* wmean, void* stream);

/*
 * Octree mode (tree_beta > 0; Sec. 5.2 "Octree Traversal"). The sources are put in an
 * octree: root = the cube over their bounding box (side = the largest extent), cells down
 * to level 21 (Morton order of floor((x - lo) 2^21 / side), FP64), a node = a non-empty cell,
 * a leaf when it holds <= tree_leaf sources or sits at level 21; a cell whose sources all
 * lie in one child is represented by the deepest cell of that chain. Per node: area A,
 * centre c.m = sum a p / A, r = max |p - c.m|, dmax = max max(delta_j, eps), moment
 * M = sum a n. For each query, depth-first from the root: a node with
 * |q - c.m| > max(tree_beta r, r + dmax) counts as one dipole M at c.m (kernel without
 * clamp); otherwise its children are visited, or, at a leaf, its sources are summed one by
 * one exactly as in the all-pairs definition. Requires n < 2^30. The result approximates
 * the all-pairs sum (tree_beta -> infinity gives it back); `split` is ignored.
 */

/*
 * dwg_octree -- the octree of the octree mode for P [3][n] with leaf capacity `leaf`
 * (0 = 32). Synchronous. Outputs: perm [n] int32 (i-th source in Morton order); nodes
 * [cap][4] int32 = (start, end, level, skip) per node in depth-first pre-order, where
 * [start, end) is the node's range of sorted positions and skip the index of the first node
 * after its subtree; *count (HOST) = number of nodes, at most 2n - 1 (cap >= 2n always
 * suffices). Workspace: dwg_workspace_bytes(n, n, kp) for any kp with tree_beta > 0.
 * Errors: DWG_E_INVALID (NULL pointers, n < 1 or >= 2^30, leaf outside 0..1024, count > cap
 * -- *count is still set), DWG_E_WORKSPACE, DWG_E_DEVICE.
 */
dwg_status dwg_octree(const float* P, int64_t n, int leaf, int32_t* perm, int32_t* nodes, int64_t cap,
                      int64_t* count, void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_octree_work -- the work of the octree mode's traversal (Sec. 5.2) for m queries Q,
 * written to work[0..3] (HOST), each totalled over the queries:
 *   work[0] = (query, node) pairs the traversal takes as one dipole;
 *   work[1] = (query, source) pairs it sums one by one at leaves;
 *   work[2] = traversal steps at which at least one query of a wavefront (64 consecutive
 *             queries in the spatial order the evaluation uses) takes the node as a dipole:
 *             the evaluation runs the dipole arithmetic once per such step for all 64 lanes;
 *   work[3] = source iterations of the wavefronts' leaf loops: at a leaf of s sources that
 *             a of its queries open, a wavefront runs s iterations, or ceil(s / k) when the
 *             evaluation spreads the leaf over k = 2^j groups of a lanes (k a <= 64, k <= s,
 *             when that saves at least 2 iterations), each group taking every k-th source.
 * work[0] / (64 work[2]) and work[1] / (64 work[3]) are the fractions of lanes doing useful
 * work in those steps. The counts depend on the positions, areas, radii and kp (the opening
 * decisions), not on the normals. Synchronous. Requires kp->tree_beta > 0 and n < 2^30.
 * Workspace: dwg_workspace_bytes(n, m, kp). Errors as dwg_gwn_eval (work[] is set to 0
 * first).
 */
dwg_status dwg_octree_work(const float* P, const float* area, const float* delta, int64_t n, const float* Q,
                           int64_t m, const dwg_kernel_params* kp, int64_t* work, void* ws, size_t ws_bytes,
                           void* stream);

/* Grid of the level-set update (Sec. 4.3, Algorithm 1). */
typedef struct dwg_mc_params {
  int depth;    /* cells per axis = 2^depth over the octree frame, 1..16 (paper: 8-13) */
  int dilate;   /* rings of neighbour cells around the cells holding points, 0..2 */
  int k;        /* nearest input points per face, 1..16 (paper: 10) */
  int iso;      /* w_bar: 0 = mean of w over the input points, 1 = over the grid corners */
  int surface;  /* level-set extraction: 0 = Marching Cubes (the paper's), 1 = marching
                   tetrahedra (an option) */
} dwg_mc_params;

/*
 * Level-set update (Sec. 4.3 Eq. 6-7, Algorithm 1). The grid: the octree frame (lo =
 * bounding-box minimum, side = largest extent) cut into 2^depth cells per axis; the
 * evaluated cells are those holding points plus `dilate` rings of neighbours; their
 * corners sit at lo + c * side / 2^depth. One iteration: w at every corner (all-pairs, or
 * octree mode when kp->tree_beta > 0) with the current normals; w_bar = the FP64 mean of w
 * over the input points (iso = 0; evaluated in the same launch) or over the corners
 * (iso = 1, Eq. 6 over the grid nodes); the w_bar level set by Marching Cubes (a corner is
 * above when w > w_bar; on every face each run of above corners is cut off by one segment,
 * so a face whose above corners are diagonal separates them and the surface is closed; the
 * segments of a cube chain into loops, each cut into a fan of triangles; at most 5 per
 * cube), or by marching tetrahedra when surface = 1 (each cube cut into 6 tetrahedra around
 * its (0,0,0)-(1,1,1) diagonal); per face the cross product (q1 - q0) x (q2 - q0), wound to
 * point away from the above corners; each face's vector added to its k nearest input
 * points; n_i = normalize(sum), a point with no face (or a zero sum) keeps its normal. The
 * per-face sums use 64-bit fixed-point atomics, so results are deterministic.
 *
 * Workspace: dwg_mc_workspace_bytes(n, kp, mcp, cells) with the cell count `cells` from
 * dwg_mc_cells (cells = 0 gives the bytes dwg_mc_cells itself needs).
 */
size_t dwg_mc_workspace_bytes(int64_t n, const dwg_kernel_params* kp, const dwg_mc_params* mcp, int64_t cells);
/* Number of evaluated grid cells for P [3][n] (synchronous; *cells is HOST). */
dwg_status dwg_mc_cells(const float* P, int64_t n, const dwg_mc_params* mcp, int64_t* cells, void* ws,
                        size_t ws_bytes, void* stream);
/*
 * dwg_iterate_mc -- Algorithm 1 with the level-set update above; arguments, statistics and
 * return codes as dwg_iterate (wmean = w_bar, gwn_ms = the evaluation of w). Synchronous. Needs k < n < 2^31 / (2 dilate + 1)^3.
 */
dwg_status dwg_iterate_mc(const float* P, const float* area, const float* delta, int64_t n, float* N_inout,
                          const dwg_kernel_params* kp, const dwg_iterate_params* ip, const dwg_mc_params* mcp,
                          dwg_iter_stat* stats_host, int* iters_done, void* ws, size_t ws_bytes, void* stream);
/*
 * dwg_level_set -- the w_bar level set of the field of (P, N) on the grid above: triangles
 * [cap][9] float (three vertices q0, q1, q2 each, wound so that (q1 - q0) x (q2 - q0) points
 * away from w > w_bar, i.e. outwards for outward normals), *ntri (HOST) = the number of triangles (written even when it
 * exceeds cap; then only cap are stored and DWG_E_INVALID is returned), *iso (HOST) = w_bar.
 * Synchronous.
 */
dwg_status dwg_level_set(const float* P, const float* N, const float* area, const float* delta, int64_t n,
                         const dwg_kernel_params* kp, const dwg_mc_params* mcp, float* tri, int64_t cap,
                         int64_t* ntri, double* iso, void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_iterate -- Algorithm 1 with every input point as a query (Sec. 4.3). Synchronous.
 *   Iteration t: evaluate w and grad w at every p_i with the normals n^(t-1) (self pair
 *   excluded), w_bar = mean w (Eq. 6), n_i^(t) = -grad w(p_i) / |grad w(p_i)| (Eq. 7; a
 *   zero or non-finite gradient keeps the old normal), and the statistics; stop when
 *   top_mean_deg <= eps_deg unless fixed_iters.
 *   P [3][n], area [n], delta [n] or NULL; N_inout [3][n]: n^(0) in, n^(T) out (unit
 *   vectors). stats_host: HOST array [max_iters] or NULL; iters_done: HOST int or NULL.
 *   Returns DWG_OK (converged, or fixed_iters), DWG_NOT_CONVERGED, DWG_E_NONFINITE (N_inout
 *   holds the last iterate), or the errors of dwg_gwn_grad; DWG_E_INVALID also for
 *   max_iters < 1, eps_deg < 0, top_frac outside (0,1].
 *   The iteration's state is N_inout alone, so a solve may start from another's result: an
 *   octree-mode solve run to its test, then an all-pairs solve from its normals, reaches
 *   the all-pairs test in a few exact iterations (one workspace of the larger of the two
 *   modes' dwg_workspace_bytes serves both).
 */
dwg_status dwg_iterate(const float* P, const float* area, const float* delta, int64_t n,
                       float* N_inout, const dwg_kernel_params* kp, const dwg_iterate_params* ip,
                       dwg_iter_stat* stats_host, int* iters_done, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * dwg_init_normals -- initial normals n^(0) (Algorithm 1; Sec. 5.1 "Normal
 * Initialization"). async.
 *   DWG_INIT_RANDOM: i.i.d. uniform unit vectors from the counter-based SplitMix64 stream
 *     of `seed`: point i uses outputs 2i and 2i+1, u = (x >> 40) 2^-24, z = 1 - 2 u0,
 *     phi = 2 pi u1, n = (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z). P may be NULL.
 *   DWG_INIT_MLP: the MLP of dwg_mlp_infer applied to the features of dwg_features;
 *     mlp_params is the device FP32 parameter blob of dwg_mlp_param_count() floats.
 *   DWG_INIT_PCA: covariance (FP64) of p_i and its 16 nearest other points about their
 *     mean; the unit eigenvector of its smallest eigenvalue, turned to point away from the
 *     origin (n . p_i > 0; where n . p_i == 0, largest-magnitude component positive) --
 *     the paper leaves the sign open; needs n > 16 and the workspace. An isotropic
 *     neighbourhood gives (0, 0, 1) before the sign rule.
 *   DWG_INIT_GAUSS: p_i / |p_i| (projection onto the unit sphere about the origin); a point
 *     at the origin gets (0, 0, 1).
 *   N_out: output [3][n].
 */
dwg_status dwg_init_normals(dwg_init_kind kind, uint64_t seed, const float* P, int64_t n,
                            const float* mlp_params, float* N_out, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * dwg_knn -- k nearest reference points (k <= 16) of each query, exact, by a uniform
 * grid (Sec. 5.1 uses kNN for the kernel radius and the normal update). async.
 *   R: reference points [3][nr]; Q: queries [3][m]; self_skip: 1 when Q is R itself (then
 *   query i never returns reference i), else 0. idx: output int32 [m][k] (ascending
 *   distance); dist: output float32 [m][k] or NULL. Distances are Euclidean in FP32.
 */
dwg_status dwg_knn(const float* R, int64_t nr, const float* Q, int64_t m, int self_skip, int k,
                   int32_t* idx, float* dist, void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_delta_knn_window -- the paper's kernel radius (Sec. 5.2 "Poisson Kernels"): delta_i =
 * mean of those distances from p_i to its k nearest other points that lie in [vmin, vmax]
 * (paper: k = 10, vmin = 0.0015, vmax = 0.015 in the model's units); when none lies in the
 * window, the mean of all k clamped to [vmin, vmax]. async. P [3][n]; delta: output [n];
 * 1 <= k <= 16, k < n < 2^31, finite 0 <= vmin <= vmax. Workspace as dwg_workspace_bytes(n, n).
 */
dwg_status dwg_delta_knn_window(const float* P, int64_t n, int k, float vmin, float vmax, float* delta,
                                void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_voronoi_area -- area weights a_i (Sec. 5.1 "Computing Area Weights"). async. For each
 * p_i: its m nearest other points (paper: m = 15); the plane through p_i normal to the
 * smallest-eigenvalue eigenvector of the covariance (FP64) of p_i and those points about
 * their mean; the points projected onto the plane; a_i = area of p_i's cell in the 2D
 * Voronoi diagram of the projections, bounded by the square [-R, R]^2 around p_i, R = the
 * largest projected distance (so that a point with all neighbours on one side gets a finite
 * cell), whose axes are u = n x e_k / |n x e_k| (e_k = the coordinate axis with the smallest
 * |n_k|, the first on ties) and n x u. Coincident neighbours bound nothing; a_i = 0 when all are coincident with p_i.
 * P [3][n]; area: output [n]; 3 <= m <= 16, m < n < 2^31. Workspace as
 * dwg_workspace_bytes(n, n).
 */
dwg_status dwg_voronoi_area(const float* P, int64_t n, int m, float* area, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * dwg_delta_knn_mean -- per-point kernel radius delta_i = mean distance to the k nearest
 * other points (Sec. 5.2 "Poisson Kernels", without the absolute distance filter), times
 * `scale`. async. P [3][n]; delta: output [n]; 1 <= k <= 16, k < n; scale > 0.
 */
dwg_status dwg_delta_knn_mean(const float* P, int64_t n, int k, float scale, float* delta,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * dwg_delta_anchor_mean -- resolution-independent kernel radius: delta_i = scale x mean
 * distance from p_i to its k nearest "anchor" points (anchors = points whose index is a
 * multiple of stride = max(1, n / n_anchor); an anchor never counts itself). A reading of
 * the threshold of Sec. 5.2, whose absolute distance window assumes the paper's model
 * normalisation: a fixed anchor count fixes the neighbourhood scale relative to the shape,
 * as the paper's octree depth fixes the field's resolution. async. P [3][n]; delta: output
 * [n]; 1 <= k <= 16; n_anchor > k; scale > 0. Workspace: dwg_workspace_bytes(n, n, NULL)
 * covers n_anchor <= 4096; the anchor grid grows with n_anchor, and a workspace too small
 * for a larger count gives DWG_E_WORKSPACE with the size needed (dwg_last_error).
 */
dwg_status dwg_delta_anchor_mean(const float* P, int64_t n, int k, int64_t n_anchor, float scale,
                                 float* delta, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- learned initial normals
 * Features of point i: its 16 nearest "anchor" points (anchors = points whose index is a
 * multiple of `stride`, stride = max(1, n / n_anchor)), the anchor i itself excluded, as
 * relative positions (a_k - p_i) / s_i in ascending distance, s_i = their mean distance:
 * 48 floats. MLP 48 -> 128 -> 128 -> 3, ReLU, output normalised. BF16 operands on MFMA,
 * FP32 accumulation. Parameter blob (FP32, this order): W1[128][48], b1[128],
 * W2[128][128], b2[128], W3[3][128], b3[3].
 */
#define DWG_MLP_IN 48
#define DWG_MLP_HID 128
#define DWG_MLP_OUT 3
#define DWG_FEAT_K 16
/* Number of FP32 values in the parameter blob (the layout above). */
int64_t dwg_mlp_param_count(void);
/* Size in bytes of the parameter blob that dwg_init_normals (DWG_INIT_MLP), dwg_mlp_infer and
 * dwg_mlp_train_step read: dwg_mlp_param_count() * sizeof(float). */
size_t dwg_mlp_blob_bytes(void);

/* Features [n][48] (float32) of every point; n_anchor >= 17. async. Workspace as for
 * dwg_delta_anchor_mean. */
dwg_status dwg_features(const float* P, int64_t n, int64_t n_anchor, float* feat, void* ws,
                        size_t ws_bytes, void* stream);

/* MLP forward on B feature rows X [B][48] (float32, rounded to BF16 on load):
 * Y [B][3] = normalised output. async. */
dwg_status dwg_mlp_infer(const float* params, const float* X, int64_t B, float* Y, void* ws,
                         size_t ws_bytes, void* stream);

/*
 * One training step on a batch: loss = mean_b (1 - <y_b/|y_b|, t_b>) over rows with
 * weight 1 (mask[b] != 0; mask may be NULL = all), gradients by the library's backward
 * kernels, then Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with `step` >= 1)
 * on the FP32 master parameters. async.
 *   params [P] in/out; adam_m, adam_v [P] in/out (zero at step 1); X [B][48]; T [B][3]
 *   unit targets; grad_out [P] or NULL (the raw gradient, for checking); loss_out: one
 *   float or NULL.
 */
dwg_status dwg_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                              float lr, const float* X, const float* T, const uint8_t* mask,
                              int64_t B, float* grad_out, float* loss_out, void* ws,
                              size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DWG_H */
