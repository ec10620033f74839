/*
 * wn.h -- C ABI of the MI355X (gfx950) generalized-winding-number voxelizer.
 *
 * The library computes, for every query point q (the centres of a voxel grid or an
 * explicit point list), the generalized winding number of a triangle mesh (V, F)
 *
 *     W(q) = 1/(4 pi) * sum_f Omega_f(q)                 (arXiv 2407.11272, Section 2.2, Eq. 5)
 *     Omega_f(q) = 2 * ATAN2(det(e0, e1, e2), 1 + e0.e1 + e1.e2 + e2.e0),
 *     e_j = (v_j - q) / |v_j - q|                        (Eq. 7 with its half-angle factor 2; Eq. 8)
 *
 * maps it to occupancy (Eq. 3: W is the occupancy of a closed surface), and
 * returns the adjoint d(loss)/d(vertices) (the differentiability of Section 2.4).
 * Algorithm 1 of the paper states the per-point problem: mesh and query point in,
 * occupancy out.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named V, F, Q, W, occ, dLdW, dLdV, dLdT, target, loss and ws are
 *    DEVICE pointers owned by the caller.  `grid`, `desc` and `tune` are HOST
 *    pointers read only during the call.
 *  - V: float [nV][3] vertex positions.  F: int32 [nF][3] vertex indices.
 *    Q: float [nQ][3] query points.  All row-major and densely packed.
 *  - Exactly one of `grid` (host) or `Q` (device) is non-NULL (both may be NULL
 *    when nQ = 0, an empty point list).  With a grid the
 *    query points are the voxel centres lo + (idx + 1/2) (hi - lo) / n, flat index
 *    (i * n[1] + j) * n[2] + k (x slowest, z fastest), and nQ must be 0 or
 *    n[0] n[1] n[2].
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    call only enqueues work on that stream and never synchronises, except
 *    wn_get_device_error.
 *  - `ws`/`ws_bytes`: caller-owned device workspace of at least
 *    wn_workspace_size(op, ...) bytes, 256-byte aligned.  The library allocates
 *    no device memory.  One workspace must not be used by two calls that may run
 *    concurrently.
 *  - Face indices outside [0, nV) never cause an out-of-bounds read: they are
 *    replaced by 0 on the device and recorded in the workspace; read the record
 *    with wn_get_device_error after the call.
 *  - Errors: argument errors return WN_ERR_INVALID_ARG before anything is
 *    enqueued; a workspace that is too small returns WN_ERR_WORKSPACE; a HIP
 *    launch error returns WN_ERR_HIP.  NaN or Inf inputs are not checked and
 *    propagate to the outputs of the affected points.
 *  - Limits: nV, nF < 2^31; nQ <= 2^31 - 1.
 *  - Results are deterministic: the same inputs give bit-identical outputs, on
 *    the same GPU model, independent of launch tuning and of what else runs.
 */
#ifndef WN_H
#define WN_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define WN_API __attribute__((visibility("default")))
#else
#define WN_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wn_status;
#define WN_OK 0
#define WN_ERR_INVALID_ARG (-1)
#define WN_ERR_HIP (-2)
#define WN_ERR_WORKSPACE (-3)
#define WN_ERR_BAD_INDEX (-4)
#define WN_ERR_UNSUPPORTED (-5)

/* Occupancy maps (Eq. 3; the threshold or a sigmoid around tau). */
#define WN_OCC_NONE 0      /* no occupancy output                          */
#define WN_OCC_THRESHOLD 1 /* uint8 occ = (W > tau)                        */
#define WN_OCC_SIGMOID 2   /* float occ = 1 / (1 + exp(-k (W - tau)))      */

/* Operation codes for wn_workspace_size. */
#define WN_OP_VOXELIZE 0
#define WN_OP_BACKWARD 1
#define WN_OP_BATCHED 2
#define WN_OP_LOSS 3
#define WN_OP_FLIP 4
#define WN_OP_MORPH 5
#define WN_OP_CUBIFY 6 /* wn_workspace_size(WN_OP_CUBIFY, 0, 0, voxels) for a grid; see wn_cubify  */
#define WN_OP_SMOOTH 7 /* wn_workspace_size(WN_OP_SMOOTH, nV, nF, 0)                              */
#define WN_OP_SAMPLE 8 /* wn_workspace_size(WN_OP_SAMPLE, 0, nF, n samples)                       */
#define WN_OP_NN 9     /* wn_workspace_size(WN_OP_NN, |A|, |B|, 0)                                 */
#define WN_OP_NAIVE 10 /* wn_autotune of wn_voxelize_naive (its workspace is WN_OP_VOXELIZE's)     */

/* Which integral drives a morphing iteration (wn_morph_step). */
#define WN_INTEGRAL_GWN 0   /* Eq. 5 with Eq. 7 solid angles (wn_voxelize / wn_backward)      */
#define WN_INTEGRAL_NAIVE 1 /* Eq. 4 centroid samples (wn_voxelize_naive / wn_backward_naive) */

/* Axis-aligned voxel grid: n[d] cells spanning [lo[d], hi[d]]. */
typedef struct {
    float lo[3];
    float hi[3];
    int32_t n[3];
} wn_grid;

/* Bytes of device workspace an operation needs (WN_OP_VOXELIZE, WN_OP_BACKWARD,
 * WN_OP_LOSS, WN_OP_FLIP, WN_OP_MORPH, WN_OP_SMOOTH, WN_OP_SAMPLE, WN_OP_NN, and
 * WN_OP_CUBIFY for a cube grid of nQ voxels; a batched launch uses
 * wn_workspace_size_batched, a cube surface of any grid wn_workspace_size_cubify).
 * Returns 0 for an unknown op or negative sizes. */
WN_API size_t wn_workspace_size(int32_t op, int64_t nV, int64_t nF, int64_t nQ);

/*
 * Forward pass (Eq. 5, 7, 8; Algorithm 1 for every point).
 * Writes W[nQ] (float, overwritten).  If occ_mode != WN_OCC_NONE also writes occ[nQ]
 * (uint8 for WN_OCC_THRESHOLD, float for WN_OCC_SIGMOID) from the same W.
 * nF = 0 gives W = 0.  nQ = 0 (point-list mode) or an empty grid is a no-op.
 */
WN_API wn_status wn_voxelize(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                      const wn_grid *grid, const float *Q, int64_t nQ,
                      float *W, int32_t occ_mode, float tau, float k, void *occ,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Triangle-strip order of a mesh, built on the host from HOST face indices F
 * (int32 [nF][3], every index in [0, nV)).  The result is a stream of records, int32
 * pairs (vertex id, face id or -1): a record with a face id completes that face
 * together with the vertices of the two records before it; consecutive faces of a
 * strip share an edge, so the forward kernels evaluate one new vertex per face
 * instead of three.  It depends only on F (a mesh whose vertices move keeps it).
 * Every face appears exactly once; n_records <= 3 nF.  With records == NULL only
 * *n_records is set; otherwise capacity (in records) must be >= *n_records, else
 * WN_ERR_WORKSPACE.  Invalid indices return WN_ERR_INVALID_ARG.
 */
WN_API wn_status wn_build_strips(const int32_t *F, int64_t nF, int64_t nV, int32_t *records, int64_t capacity,
                                 int64_t *n_records);

/*
 * wn_voxelize with a strip stream from wn_build_strips (device int32 [n_records][2])
 * in place of the default three records per face.  Same outputs and conventions; W
 * agrees with wn_voxelize to rounding (the face order differs) and is deterministic
 * for a given stream.  Face ids in the stream must be < nF and vertex ids < nV (out of
 * range entries are replaced and recorded, as for F).  The workspace is
 * wn_workspace_size(WN_OP_VOXELIZE, nV, nF, nQ) for any stream of at most 3 nF records.
 */
WN_API wn_status wn_voxelize_strips(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                    const int32_t *strips, int64_t n_records,
                                    const wn_grid *grid, const float *Q, int64_t nQ,
                                    float *W, int32_t occ_mode, float tau, float k, void *occ,
                                    void *ws, size_t ws_bytes, void *stream);

/*
 * Occupancy map alone (Eq. 3): occ[i] = (W[i] > tau) as uint8 for
 * WN_OCC_THRESHOLD, or sigmoid(k (W[i] - tau)) as float for WN_OCC_SIGMOID.
 */
WN_API wn_status wn_occupancy(const float *W, int64_t n, int32_t mode, float tau, float k, void *occ,
                       void *stream);

/*
 * Adjoint of the soft occupancy map (WN_OCC_SIGMOID): for g = dL/d(occ) (float [n]),
 * dLdW[i] = g[i] k s (1 - s) with s = sigmoid(k (W[i] - tau)) recomputed from W as
 * wn_occupancy computes it; dLdW may alias g.  The chain rule from a soft-occupancy loss
 * to the winding numbers (Section 2.4 supervises the mesh by voxel occupancy).
 */
WN_API wn_status wn_occupancy_backward(const float *W, const float *g, int64_t n, float tau, float k, float *dLdW,
                                       void *stream);

/*
 * Soft-occupancy MSE loss L = (1/n) sum_i (sigmoid(k (W_i - tau)) - target_i)^2 and its
 * gradient dLdW[i] (both outputs optional: pass NULL to skip).  `loss` is one float
 * in device memory.  Needs a workspace of wn_workspace_size(WN_OP_LOSS, 0, 0, n).
 * (The loss that drives mesh morphing by voxel supervision, Section 2.4.)
 */
WN_API wn_status wn_sigmoid_mse(const float *W, const float *target, int64_t n, float tau, float k,
                         float *loss, float *dLdW, void *ws, size_t ws_bytes, void *stream);

/*
 * Adjoint of wn_voxelize's W (the gradients with respect to the input mesh that
 * Section 2.4 relies on).  For the given dLdW[nQ]:
 *   dLdT[f][j][c] = sum_q dLdW[q] * dW(q)/dv_{F[f][j]}[c]    (float [nF][9], optional)
 *   dLdV[v][c]    = sum over the corners (f, j) with F[f][j] = v of dLdT[f][j][c]
 * dLdV (float [nV][3]) is overwritten.  Solid angles are recomputed per tile; the
 * point x face matrix is never stored.  A corner whose vertex coincides with q, or a
 * face with q on an edge, contributes 0.
 */
WN_API wn_status wn_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                      const wn_grid *grid, const float *Q, int64_t nQ,
                      const float *dLdW, float *dLdV, float *dLdT,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * The adjoint of wn_backward in pieces, so that a scheduler can interleave a large
 * adjoint with other work (Section 2.4's gradients, served in slices).  The points are
 * taken in tiles of WN_BWD_TILE consecutive points, dealt in turn to the S =
 * wn_backward_splits(nF, nQ) splits of the adjoint (tile t to split t mod S; with pairs,
 * the count whose running sums fit the same space, about S nF / (2 n_pairs), or 1.5 times
 * that with WN_BWD_VERTEX_SUMS, 3 times when there are at least 12 tiles per split; at
 * most one split per tile); each split
 * keeps compensated running sums per face corner in the workspace between calls, and the
 * splits are added in split order at the end.  A sequence of calls on one workspace
 *     flags WN_BWD_BEGIN (pack the faces), then consecutive point ranges [p0, p0 + n) in
 *     increasing order that together cover [0, nQ) exactly once, the last with
 *     WN_BWD_END (add the splits, group corners per vertex, write dLdV and optionally
 *     dLdT)
 * gives the same bits as one call (p0 = 0, n = nQ, both flags), which is wn_backward.
 * Flags may be combined with a range in one call (BEGIN runs before the range, END
 * after it).  Ranges out of order or overlapping give wrong sums (a range that reaches a
 * split's first tile restarts that split); the library does not detect it.
 *   p0:    a multiple of WN_BWD_TILE;  n: a multiple of WN_BWD_TILE, or p0 + n = nQ;
 *   dLdW:  indexed by the global point number (only [p0, p0 + n) is read);
 *   pairs: NULL (one face per lane), or a device copy of wn_build_face_pairs' output
 *          (n_pairs of them) for two faces per lane; the same in every call of a
 *          sequence.  Pairs give the same gradient up to rounding (the per-face
 *          arithmetic is the same, the compiler's contractions may differ).  A face
 *          missing or repeated, or a pair without a shared edge, is recorded as a bad
 *          index (wn_get_device_error);
 *   V, F, grid / Q, nQ: the same in every call of a sequence;
 *   dLdV:  needed with WN_BWD_END; dLdT optional, as in wn_backward;
 *   flags: may add WN_BWD_VERTEX_SUMS (in every call of a sequence, or in none) when
 *          only dLdV is wanted: with pairs, the two faces of a pair then share their
 *          running sums at the shared edge's two vertices (12 instead of 18 per pair and
 *          split, fewer operations per point), so the sums per vertex stay exact up to
 *          rounding but those per corner do not; dLdT must then be NULL at WN_BWD_END
 *          (also without pairs, where the flag changes nothing else);
 *   ws:    wn_workspace_size(WN_OP_BACKWARD, nV, nF, nQ) bytes, holding the running sums.
 * A range of at least S tiles keeps every split busy (about nF / 256 x S workgroups).
 * Argument errors return WN_ERR_INVALID_ARG before any launch.
 */
#define WN_BWD_BEGIN 1
#define WN_BWD_END 2
#define WN_BWD_VERTEX_SUMS 4
#define WN_BWD_TILE 256
WN_API wn_status wn_backward_range(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                   const int32_t *pairs, int64_t n_pairs,
                                   const wn_grid *grid, const float *Q, int64_t nQ,
                                   const float *dLdW, int64_t p0, int64_t n,
                                   int32_t flags, float *dLdV, float *dLdT,
                                   void *ws, size_t ws_bytes, void *stream);

/*
 * Pairs of faces that share an edge, built on the host from HOST face indices F (int32
 * [nF][3], every index in [0, nV)), for the adjoint: with them wn_backward_range gives
 * each lane two faces and evaluates the shared edge's two vertices once for both (4
 * instead of 6 vertices per point).  Output int32 [n_pairs][2] = (f, g), pairs of faces
 * with three distinct vertex ids sharing exactly two (consecutive faces of the strips of
 * wn_build_strips, then left-over faces matched across an edge), followed by the
 * unpaired faces as (f, -1); every face appears exactly once, so ceil(nF / 2) <= n_pairs
 * <= nF.  A pure function of F.  With pairs == NULL only *n_pairs is set; otherwise
 * capacity (in pairs) must be >= *n_pairs, else WN_ERR_WORKSPACE.  Invalid indices
 * return WN_ERR_INVALID_ARG.
 */
WN_API wn_status wn_build_face_pairs(const int32_t *F, int64_t nF, int64_t nV, int32_t *pairs, int64_t capacity,
                                     int64_t *n_pairs);

/* The number of splits S of the adjoint of nF faces over nQ points (a pure function of the
 * sizes: about 32 768 waves of (face block, split) work, at most one split per tile, at
 * most 4096, and at most 256 MiB of running sums, 72 bytes per face per split; the
 * workspace holds twice that space when there are at least 12 tiles per split, for the
 * face-pair adjoint with WN_BWD_VERTEX_SUMS); -1 on invalid sizes. */
WN_API int64_t wn_backward_splits(int64_t nF, int64_t nQ);

/*
 * The naive discretisation of the flux integral (Section 2.1, Eq. 4): one sample per
 * face at its centroid c_f with the area-weighted normal N_f / 2,
 * N_f = (v1 - v0) x (v2 - v0):
 *     W(q) ~= 1/(8 pi) sum_f <N_f, c_f - q> / |c_f - q|^3,
 * a face whose centroid coincides with q contributing 0.  It approximates W away from
 * the surface and, unlike the exact field, has non-vanishing vertex gradients (the
 * paper uses it for mesh morphing, Section 2.4).  Same arguments, outputs and
 * workspace (wn_workspace_size(WN_OP_VOXELIZE, ...)) as wn_voxelize.
 */
WN_API wn_status wn_voxelize_naive(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                   const wn_grid *grid, const float *Q, int64_t nQ,
                                   float *W, int32_t occ_mode, float tau, float k, void *occ,
                                   void *ws, size_t ws_bytes, void *stream);

/*
 * Adjoint of wn_voxelize_naive: the same outputs as wn_backward (dLdV overwritten,
 * optional per-corner dLdT) for the Eq. 4 sum, with
 *   d term_f / d v_j = (N/|r|^3 - 3 <N, r> r/|r|^5) / 3 + (v_{j+1} - v_{j+2}) x r/|r|^3,
 * r = c_f - q.  Workspace: wn_workspace_size(WN_OP_BACKWARD, ...).
 */
WN_API wn_status wn_backward_naive(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                   const wn_grid *grid, const float *Q, int64_t nQ,
                                   const float *dLdW, float *dLdV, float *dLdT,
                                   void *ws, size_t ws_bytes, void *stream);

/* One mesh of a batched forward launch (host struct; pointers are device memory).
 * The launch evaluates the voxel centres with flat indices
 * [point_begin, point_begin + point_count) of the grid (point_count = 0: to the end of
 * the grid) and writes W and occ at those same flat indices of the full-grid arrays, so
 * a grid can be processed in slices.  A voxel's value does not depend on the slice. */
typedef struct {
    const float *V;
    int64_t nV;
    const int32_t *F;
    int64_t nF;
    wn_grid grid;      /* query points are always this grid's voxel centres */
    float *W;          /* [n0 n1 n2] output, required                        */
    void *occ;         /* occupancy output or NULL                           */
    int32_t occ_mode;  /* WN_OCC_*                                           */
    float tau;
    float k;
    int64_t point_begin;
    int64_t point_count;
    const int32_t *strips;    /* device strip stream from wn_build_strips, or NULL */
    int64_t n_strip_records;  /* records in strips (0 when strips is NULL)         */
} wn_mesh_desc;

/*
 * Forward pass for n meshes of uneven size in one persistent launch: a host-built
 * work list of (mesh, point block, face chunk) units, longest first, drained by
 * persistent workgroups; the launch sequence is captured once as a HIP graph per
 * workspace and replayed.  Each mesh's result is bit-identical to the same mesh
 * alone in a batched call (its chunking depends only on its own size).
 * Workspace: wn_workspace_size_batched(desc, n).  The table describing the batch is
 * copied on `stream` from a ring of library-owned pinned host buffers: a call takes a
 * buffer whose earlier copy has finished or adds one, so it does not wait on the host
 * (unless 64 copies for this workspace are still queued).  wn_release_workspace frees
 * the graphs and buffers.
 * flags: 0, or WN_BATCH_NO_GRAPH to launch without graph capture.
 * Every mesh needs W non-NULL and a grid with n[d] >= 1 and hi > lo.
 */
#define WN_BATCH_NO_GRAPH 1
WN_API wn_status wn_voxelize_batched(const wn_mesh_desc *desc, int32_t n, int32_t flags,
                              void *ws, size_t ws_bytes, void *stream);

/* Exact workspace bytes for wn_voxelize_batched of these meshes (0 if a descriptor
 * is invalid). */
WN_API size_t wn_workspace_size_batched(const wn_mesh_desc *desc, int32_t n);

/*
 * Frees what the library keeps on the host for a workspace that batched launches used:
 * its captured graphs and pinned staging buffers.  Call it before the workspace memory
 * is freed or reused for something else, once no launch using it is still running
 * (synchronise its stream first).  A workspace the library holds nothing for is a no-op.
 */
WN_API wn_status wn_release_workspace(void *ws);

/*
 * Launch autotuner.  Times each candidate launch configuration -- the point tile
 * (query points per lane 1/2/4) times the record tile (1/2/4 tiles of 60 vertex records
 * staged in LDS per barrier); for WN_OP_BATCHED also the fastest of those with at
 * most 2 persistent workgroups per CU; for WN_OP_NAIVE (wn_voxelize_naive) the point
 * tile alone -- on the given work (desc[0] alone for WN_OP_VOXELIZE and WN_OP_NAIVE,
 * all n meshes for WN_OP_BATCHED), and records the fastest for that
 * shape bucket (floor(log2) of faces and points, or of total pairs and mesh count).
 * Later calls of that op and bucket use it.  A configuration never changes results,
 * only speed: the report carries a checksum of every candidate's outputs and
 * "identical": true when they all agree.  With the environment variable
 * WN_AUTOTUNE_CACHE naming a file, choices persist there as JSON lines.  Writes the
 * outputs of desc as a side effect, synchronises `stream`, and writes the JSON report
 * to `report` (optional, NUL-terminated, truncated to report_len).
 */
WN_API wn_status wn_autotune(int32_t op, const wn_mesh_desc *desc, int32_t n, void *ws, size_t ws_bytes,
                             void *stream, char *report, size_t report_len);

/*
 * Flipping duplication of an open mesh (Algorithm 2 of the paper): writes
 *   V2 = [V ; V - eps * N]            (float [2 nV][3], N = unit vertex normals)
 *   F2 = [F ; flip(F) + nV]           (int32 [2 nF][3], flip(a, b, c) = (a, c, b))
 * so that (V2, F2) can be voxelized like a closed mesh; the slit between the two
 * layers is eps thick.  A vertex normal is the normalised sum of the area-weighted
 * normals (v1 - v0) x (v2 - v0) of the faces using the vertex (0 if none), summed in
 * FP64 in face order.  Out-of-range face indices are replaced by 0 and recorded.
 * Workspace: wn_workspace_size(WN_OP_FLIP, nV, nF, 0).
 */
WN_API wn_status wn_flip_duplicate(const float *V, int64_t nV, const int32_t *F, int64_t nF, float eps,
                                   float *V2, int32_t *F2, void *ws, size_t ws_bytes, void *stream);

/*
 * Adam (Kingma and Ba, 2015, Algorithm 1) on n parameters in place, for step number t >= 1:
 *   m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   x -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * x, m, v (float [n], updated) and g (float [n]) are device arrays; m and v start at 0
 * for t = 1.  The bias corrections are formed in FP64 on the host.  Needs
 * 0 <= beta1, beta2 < 1, eps > 0, lr finite; n = 0 is a no-op.  The optimiser of the
 * mesh-morphing loop (Section 2.4 deforms a mesh by gradients of a voxel loss).
 */
WN_API wn_status wn_adam(float *x, const float *g, float *m, float *v, int64_t n, int64_t t, float lr,
                         float beta1, float beta2, float eps, void *stream);

/*
 * Mesh morphing by voxel supervision (Section 2.4): `iters` iterations, each
 *   W = winding numbers of (V, F) at the voxel centres of `grid`
 *       (integral = WN_INTEGRAL_NAIVE: the Eq. 4 sum the paper uses for morphing, whose
 *        gradient does not vanish; WN_INTEGRAL_GWN: Eq. 5 and 7),
 *   L = (1/P) sum_q (sigmoid(k (W_q - tau)) - target_q)^2 and dL/dW (wn_sigmoid_mse),
 *   dL/dV by the adjoint of the chosen integral,
 *   Adam (wn_adam) on V in place, step numbers t0 + 1, ..., t0 + iters.
 * V (float [nV][3]) is updated in place; F (int32 [nF][3]) and target (float [P], P =
 * grid cells, C order) are read; m and v (float [nV][3]) are the Adam moments, zero
 * before the first step.  loss_history (optional, device float [iters]) receives L of
 * each iteration, evaluated before its update.  Everything stays on the device; the call
 * only enqueues work on `stream`.  Workspace: wn_workspace_size(WN_OP_MORPH, nV, nF, P).
 * Face indices out of range are replaced and recorded as in wn_voxelize.
 */
WN_API wn_status wn_morph_step(float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                               const float *target, int32_t integral, float tau, float k, float lr,
                               float beta1, float beta2, float eps, int64_t t0, int32_t iters, float *m,
                               float *v, float *loss_history, void *ws, size_t ws_bytes, void *stream);

/*
 * Evaluation chain of the paper's experiments (Section 3): each method's occupancy is
 * "cubified", smoothed with a Laplacian filter (10 iterations, lambda = 0.15), and
 * compared with the original mesh by Chamfer and Hausdorff distances over 20 000
 * surface samples.  The four calls below are those steps.
 */

/*
 * Cube surface of an occupancy grid: every face of an occupied voxel (occ[i] != 0,
 * uint8 [P], C order like the grid points) whose neighbour is empty or outside the grid
 * becomes two triangles facing outward.  Faces are ordered by voxel, then -x, +x, -y,
 * +y, -z, +z; vertices are the lattice corners used, numbered in lattice C order, at
 * lo + c (hi - lo) / n.  Writes counts[0] = nV, counts[1] = nF (device int64 [2]) and
 * the first capV vertices (float [capV][3]) and capF faces (int32 [capF][3]); nothing
 * beyond the capacities.  Bounds: nV <= (nx+1)(ny+1)(nz+1), nF <= 12 P.  The lattice must
 * have fewer than 2^31 corners.  Workspace: wn_workspace_size(WN_OP_CUBIFY, 0, 0, P) for
 * a cube grid; in general wn_workspace_size_cubify(grid).
 */
WN_API size_t wn_workspace_size_cubify(const wn_grid *grid);
WN_API wn_status wn_cubify(const uint8_t *occ, const wn_grid *grid, float *V, int64_t capV, int32_t *F,
                           int64_t capF, int64_t *counts, void *ws, size_t ws_bytes, void *stream);

/*
 * Marching cubes (the reconstruction Section 3 names when it motivates the measure) of a
 * field f (float [P], C order like the grid points, e.g. W or a soft occupancy) at a
 * level iso > 0: the surface between values > iso (inside) and values <= iso, the
 * centres surrounded by one layer of zeros so that it is closed.  Cells join 8
 * neighbouring centres; the triangles of each corner pattern come from one rule (on every
 * cell face, counter-clockwise from outside, each entry crossing is joined to the next
 * exit, which cuts inside corners off on their own; loops start at their lowest local
 * edge and are fanned from their first vertex with no diagonal inside a cell face).
 *   Vertices: one per crossed lattice edge, at the linear interpolation of the two
 *     values, numbered by edge id 3 * (padded lattice index) + axis, where the padded
 *     lattice has (n + 2) points per axis, point i at lo + (i - 1/2) h.
 *   Faces: cell by cell in padded C order, each cell's triangles in table order, facing
 *     outward (from inside to outside values).
 * Writes counts[0] = nV, counts[1] = nF (device int64 [2]) and the first capV vertices
 * (float [capV][3]) and capF faces (int32 [capF][3]).  Bounds: nV <= 3 L, nF <= 5 C with
 * L = (nx+2)(ny+2)(nz+2) lattice points (3 L < 2^31) and C = (nx+1)(ny+1)(nz+1) cells.
 * NaN values count as outside.  Workspace: wn_workspace_size_marching(grid) (0 when the
 * grid is invalid or too large).
 */
WN_API size_t wn_workspace_size_marching(const wn_grid *grid);
WN_API wn_status wn_marching_cubes(const float *f, const wn_grid *grid, float iso, float *V, int64_t capV,
                                   int32_t *F, int64_t capF, int64_t *counts, void *ws, size_t ws_bytes,
                                   void *stream);

/*
 * The Laplacian filter of the evaluation (Section 3): `iters` Jacobi steps of the
 * umbrella operator
 *   v <- v + lam (mean of the vertices joined to v by a face edge - v),
 * vertices without neighbours staying; with keep_volume = 1 (the filter's default in the
 * tool the paper names) each step is followed by a uniform scaling about the origin by
 * (V0 / V)^(1/3), V0 the volume the surface enclosed before the first step and V the one
 * after this step (sum over faces of v0 . (v1 x v2) / 6, FP64, fixed order), skipped when
 * V0 / V is not positive; keep_volume = 0 leaves the steps alone.  Each vertex adds its
 * neighbours in increasing id order, so the result is deterministic.  V (float [nV][3])
 * is read, Vout (float [nV][3], not aliasing V) written.  Out-of-range face indices are
 * replaced by 0 and recorded.  Workspace: wn_workspace_size(WN_OP_SMOOTH, nV, nF, 0).
 */
WN_API wn_status wn_laplacian_smooth(const float *V, int64_t nV, const int32_t *F, int64_t nF, float lam,
                                     int32_t iters, int32_t keep_volume, float *Vout, void *ws, size_t ws_bytes,
                                     void *stream);

/*
 * Area-uniform surface samples from caller-supplied uniform numbers u (device double
 * [n][3] in [0, 1)).  Face weights are w_f = floor(area_f 2^32 / max area) with areas in
 * FP64 from the FP32 coordinates (products rounded separately); sample s takes the
 * first face whose inclusive prefix of w exceeds min(floor(u0 W), W - 1), W = sum w, and
 * the point a + r1 (b - a) + r2 (c - a) with (r1, r2) = (u1, u2), reflected to
 * (1 - u1, 1 - u2) when u1 + u2 > 1.  Writes P (float [n][3]) and face (int32 [n]);
 * if every face has zero area, face = -1 and P = 0.  Needs nF > 0 when n > 0.
 * Workspace: wn_workspace_size(WN_OP_SAMPLE, 0, nF, n).
 */
WN_API wn_status wn_sample_surface(const float *V, int64_t nV, const int32_t *F, int64_t nF, const double *u,
                                   int64_t n, float *P, int32_t *face, void *ws, size_t ws_bytes, void *stream);

/*
 * Nearest-neighbour distances d[i] = min_j |A_i - B_j| (float [nA]; A float [nA][3],
 * B float [nB][3], nB > 0 when nA > 0), and the two metrics of the evaluation:
 * out[0] = Chamfer distance mean_a d(a, B) + mean_b d(b, A), out[1] = Hausdorff distance
 * max(max_a d(a, B), max_b d(b, A)) (device double [2]; nA, nB > 0).  Squared distances
 * are FP32; the minimum is exact for them; the means are FP64 sums in a fixed order.
 * Workspace: wn_workspace_size(WN_OP_NN, nA, nB, 0).
 */
WN_API wn_status wn_nn_distance(const float *A, int64_t nA, const float *B, int64_t nB, float *d, void *ws,
                                size_t ws_bytes, void *stream);
WN_API wn_status wn_chamfer_hausdorff(const float *A, int64_t nA, const float *B, int64_t nB, double *out,
                                      void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): wn_voxelize_strips without the
 * workspace arguments.  The workspace lives in a fixed device array of
 * WN_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from the first call on
 * that GPU until the process ends; the call allocates nothing.  Inputs and outputs are
 * the caller's, with the meaning, layout and results of wn_voxelize_strips (bit-identical
 * to it).  A stream of n_records records over nQ points needs the workspace
 * wn_voxelize_strips would need, at most wn_workspace_size(WN_OP_VOXELIZE, nV,
 * ceil(n_records / 3), nQ) bytes; a larger request returns WN_ERR_WORKSPACE before
 * anything is enqueued.  Every call on one GPU shares that GPU's array (the last call's
 * contents stay), so calls that may overlap on one GPU -- on different streams, or from
 * different threads without ordering -- race and must not be issued.  Its device error
 * record (an index out of range) is read with wn_get_device_error(NULL, stream) on the
 * same GPU.
 */
#define WN_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
WN_API wn_status wn_voxelize_strips_noalloc(const float *V, int64_t nV, const int32_t *F, int64_t nF,
                                            const int32_t *strips, int64_t n_records, const wn_grid *grid,
                                            const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau,
                                            float k, void *occ, void *stream);

/*
 * Reads and clears the device-side error record that the most recent call using
 * this workspace left (a face index out of range); ws = NULL reads the record of
 * wn_voxelize_strips_noalloc on the current GPU.  Synchronises `stream`.
 * Returns WN_OK or WN_ERR_BAD_INDEX.
 */
WN_API wn_status wn_get_device_error(void *ws, void *stream);

/* Static description of a status code. */
WN_API const char *wn_status_string(wn_status s);

/* Library version string and the GPU architecture the code objects target. */
WN_API const char *wn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WN_H */
