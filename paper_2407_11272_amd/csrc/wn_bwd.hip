// Adjoint of the winding number with respect to the mesh vertices.
//
// The paper (arXiv 2407.11272, Section 2.4) relies on the voxelization being
// differentiable in the vertices but gives no gradient formula.  With
// t = ATAN2(alpha, beta) the half solid angle of Eq. 7/8 and e_j = R_j / |R_j|:
//   dt = (beta dalpha - alpha dbeta) / (alpha^2 + beta^2)
//   dalpha/de_j = e_k x e_l,  dbeta/de_j = e_k + e_l        ((j, k, l) cyclic)
//   de_j/dv_j = (I - e_j e_j^T) / |R_j|
// so dt/dv_j = P_j (beta u_j - alpha s_j) / (|R_j| (alpha^2 + beta^2)) with
// u_j = e_k x e_l, s_j = e_k + e_l, P_j the projector orthogonal to e_j, and
// dW/dv_j = dt/dv_j / (2 pi) (W = sum t / (2 pi)).
//
// Layout of the work (this library's own design):
//   * one lane owns one face and keeps its 9 gradient sums in registers;
//   * query points (with their dL/dW) stream through LDS and are read by every
//     lane (broadcast), solid angles are recomputed per pair, nothing of size
//     points x faces is stored;
//   * the points are split over workgroups: the 256-point tiles are dealt to S
//     splits in turn (tile t to split t mod S), each split keeping its own
//     compensated sums per corner; the splits are added in a fixed order at the end,
//     then corners are grouped per vertex by a stable radix sort of their vertex ids
//     and summed in face order -- deterministic throughout.  A split's running sums
//     live in the workspace between calls, so the adjoint can also be computed over
//     consecutive point ranges (the served loop's units) with the same bits.
// With a face-pair list the point loop runs two faces per lane instead
// (wn_bwd_pairs.hip); the split reduction and the vertex gather here are shared.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "wn_internal.hpp"

namespace wn {

constexpr int kPointTile = kBwdTile;  // points staged per tile (one per thread)
static_assert(kBwdTile == kBlock && kBwdTile == WN_BWD_TILE, "one point per thread per tile");

// dL/dv running sums of one face over the tiles [t0, t1) of its split.  Grid: x = face
// blocks, y = the splits that own a tile of the range (split (t0 + y) mod S).  state
// layout: float2 (sum, compensation) [S][9][nF]; a split whose first tile (tile s) is
// in the range starts from zero, any other resumes its stored sums.
//
// Per pair the corner vector is gk r_j^-1 (beta u_j - alpha E - alpha (e_k . e_l) e_j)
// with E = e_0 + e_1 + e_2 and gk = dL/dW / (alpha^2 + beta^2) (the projection folded
// in: e_j . u_j = alpha and e_j . (e_k + e_l) = beta - 1 - e_k . e_l).  The first term
// is not summed per pair.  With w = gk beta / (r_0 r_1 r_2) it is w (R_k x R_l), and
// R_k x R_l = C_j + D_j x R_0 with D_j = v_k - v_l, C_0 = N = (v_1 - v_0) x (v_2 - v_0)
// and C_1 = C_2 = 0, so over a tile of points it is C_j sum(w) + D_j x sum(w R_0): four
// sums per pair instead of nine products.  alpha = (R_0 . N) / (r_0 r_1 r_2) (Eq. 7).
__global__ __launch_bounds__(kBlock) void k_wn_bwd(const FaceRec *__restrict__ soup, int32_t nF, PointSrc ps,
                                                   int64_t nQ, int32_t S, int64_t t0, int64_t t1,
                                                   const float *__restrict__ dLdW, float2 *__restrict__ state) {
    __shared__ float4 pts[kPointTile];
    const int tid = threadIdx.x;
    const int64_t tfirst = t0 + blockIdx.y;       // this block's first tile
    const int64_t sy = tfirst % S;                // its split
    int32_t f = (int32_t)blockIdx.x * kBlock + tid;
    const bool live = f < nF;
    f = live ? f : nF - 1;
    const FaceRec r = soup[f];
    const float v[3][3] = {{r.a.x, r.a.y, r.a.z}, {r.a.w, r.b.x, r.b.y}, {r.b.z, r.b.w, r.c.x}};
    const float N[3] = {r.c.y, r.c.z, r.c.w};

    float s[9], c[9];
    load_state(state, sy, nF, f, tfirst < S, s, c);

    for (int64_t t = tfirst; t < t1; t += S) {
        const int64_t q0 = t * kPointTile;
        const int nt = (int)min((int64_t)kPointTile, nQ - q0);
        __syncthreads();
        if (tid < nt) {
            float x, y, z;
            ps.get(q0 + tid, x, y, z);
            pts[tid] = make_float4(x, y, z, dLdW[q0 + tid]);
        }
        __syncthreads();
        float ts[9], sw = 0.0f, sq[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < 9; ++i) ts[i] = 0.0f;
        for (int i = 0; i < nt; ++i) {
            const float4 q = pts[i];
            float R[3][3], e[3][3], ri[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                R[j][0] = v[j][0] - q.x;
                R[j][1] = v[j][1] - q.y;
                R[j][2] = v[j][2] - q.z;
                const float l2 = R[j][0] * R[j][0] + R[j][1] * R[j][1] + R[j][2] * R[j][2];
                ri[j] = (l2 > 0.0f) ? __builtin_amdgcn_rsqf(l2) : 0.0f;
                e[j][0] = R[j][0] * ri[j];
                e[j][1] = R[j][1] * ri[j];
                e[j][2] = R[j][2] * ri[j];
            }
            const float rho = ri[0] * ri[1] * ri[2];
            const float alpha = rho * (R[0][0] * N[0] + R[0][1] * N[1] + R[0][2] * N[2]);
            float dd[3];  // dd[j] = e_k . e_l for (j, k, l) cyclic
            dd[2] = e[0][0] * e[1][0] + e[0][1] * e[1][1] + e[0][2] * e[1][2];
            dd[0] = e[1][0] * e[2][0] + e[1][1] * e[2][1] + e[1][2] * e[2][2];
            dd[1] = e[2][0] * e[0][0] + e[2][1] * e[0][1] + e[2][2] * e[0][2];
            const float beta = 1.0f + dd[2] + dd[0] + dd[1];
            const float den = alpha * alpha + beta * beta;
            const float gk = (den > 0.0f) ? q.w * __builtin_amdgcn_rcpf(den) : 0.0f;
            const float w = gk * beta * rho, nga = -(gk * alpha);
            sw += w;
#pragma unroll
            for (int d = 0; d < 3; ++d) sq[d] = __builtin_fmaf(w, R[0][d], sq[d]);
            float E[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) E[d] = e[0][d] + e[1][d] + e[2][d];
            // Two multiply-adds into each sum with the signs folded into the
            // coefficients, so each is a two-operand accumulate (dual-issuable).
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float nca = nga * ri[j], ncd = nca * dd[j];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    ts[3 * j + d] = __builtin_fmaf(nca, E[d], ts[3 * j + d]);
                    ts[3 * j + d] = __builtin_fmaf(ncd, e[j][d], ts[3 * j + d]);
                }
            }
        }
        // the beta u_j terms of the tile: C_j sum(w) + D_j x sum(w R_0)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int k = (j + 1) % 3, l = (j + 2) % 3;
            const float D[3] = {v[k][0] - v[l][0], v[k][1] - v[l][1], v[k][2] - v[l][2]};
            const float cj = (j == 0) ? sw : 0.0f;
            ts[3 * j + 0] += cj * N[0] + (D[1] * sq[2] - D[2] * sq[1]);
            ts[3 * j + 1] += cj * N[1] + (D[2] * sq[0] - D[0] * sq[2]);
            ts[3 * j + 2] += cj * N[2] + (D[0] * sq[1] - D[1] * sq[0]);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) neumaier_add(s[i], c[i], ts[i]);
    }
    if (live) store_state(state, sy, nF, f, s, c);
}

// T[f][i] = sum over splits (fixed order) of each split's total, * scale (1/(2 pi) for
// the exact field, 1/(8 pi) for Eq. 4).
__global__ __launch_bounds__(kBlock) void k_bwd_reduce(const float2 *__restrict__ state, int32_t split, int32_t nF,
                                                       float scale, float *__restrict__ T) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nF * 9) return;
    const int32_t i = (int32_t)(t / nF);
    const int32_t f = (int32_t)(t - (int64_t)i * nF);
    const float2 *p = state + (int64_t)i * nF + f;
    const int64_t stride = (int64_t)9 * nF;  // from one split to the next
    float s = 0.0f, c = 0.0f;
    int32_t k = 0;
    // kReduceBatch loads in flight, then added in split order (the same order as one at a time)
    for (; k + kReduceBatch <= split; k += kReduceBatch) {
        float2 x[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) x[u] = p[(int64_t)(k + u) * stride];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) neumaier_add(s, c, x[u].x + x[u].y);
    }
    for (; k < split; ++k) {
        const float2 x = p[(int64_t)k * stride];
        neumaier_add(s, c, x.x + x.y);
    }
    T[(int64_t)f * 9 + i] = (s + c) * scale;
}

// Sort keys: the vertex of each corner (out-of-range ids read as 0, as in packing).
__global__ __launch_bounds__(kBlock) void k_corner_keys(const int32_t *__restrict__ F, int64_t nC, int64_t nV,
                                                        int32_t *__restrict__ keys, int32_t *__restrict__ vals) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nC) return;
    const int32_t v = F[c];
    keys[c] = (v < 0 || (int64_t)v >= nV) ? 0 : v;
    vals[c] = (int32_t)c;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// Run boundaries of the sorted vertex ids.
__global__ __launch_bounds__(kBlock) void k_bounds(const int32_t *__restrict__ keys, int64_t nC,
                                                   int32_t *__restrict__ vstart, int32_t *__restrict__ vend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nC) return;
    const int32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) vstart[k] = (int32_t)i;
    if (i == nC - 1 || keys[i + 1] != k) vend[k] = (int32_t)(i + 1);
}

// dL/dV[v] = sum of the corner gradients of v in increasing corner order.
__global__ __launch_bounds__(kBlock) void k_gather(const float *__restrict__ T, const int32_t *__restrict__ corners,
                                                   const int32_t *__restrict__ vstart,
                                                   const int32_t *__restrict__ vend, int64_t nV,
                                                   float *__restrict__ dLdV) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    float s[3] = {0.0f, 0.0f, 0.0f}, c[3] = {0.0f, 0.0f, 0.0f};
    for (int32_t i = vstart[v]; i < vend[v]; ++i) {
        const int64_t cn = corners[i];
        for (int d = 0; d < 3; ++d) neumaier_add(s[d], c[d], T[3 * cn + d]);
    }
    for (int d = 0; d < 3; ++d) dLdV[3 * v + d] = s[d] + c[d];
}

// ------------------------------------------------- flipping duplication ---
//
// Algorithm 2 of the paper turns an open mesh into an almost closed one: each vertex is
// copied and moved by -eps along its vertex normal, and each face is copied onto the
// moved vertices with its orientation reversed.  The vertex normal is the normalised
// sum of the area-weighted face normals (v1 - v0) x (v2 - v0) of the faces that use
// the vertex (the paper does not fix the weighting), summed in FP64 in face order
// through the same stable corner sort as the adjoint, so the result is deterministic.

__global__ __launch_bounds__(kBlock) void k_face_normals(const float *__restrict__ V, int64_t nV,
                                                         const int32_t *__restrict__ F, int64_t nF,
                                                         double *__restrict__ Nf, WsHeader *hdr) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    int32_t id[3];
    bool bad = false;
    for (int j = 0; j < 3; ++j) {
        id[j] = F[3 * f + j];
        if (id[j] < 0 || (int64_t)id[j] >= nV) {
            bad = true;
            id[j] = 0;
        }
    }
    if (bad) atomicOr(&hdr->bad_index, 1);
    double v[3][3];
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) v[j][c] = V[3 * (int64_t)id[j] + c];
    const double e1x = v[1][0] - v[0][0], e1y = v[1][1] - v[0][1], e1z = v[1][2] - v[0][2];
    const double e2x = v[2][0] - v[0][0], e2y = v[2][1] - v[0][1], e2z = v[2][2] - v[0][2];
    Nf[3 * f + 0] = e1y * e2z - e1z * e2y;
    Nf[3 * f + 1] = e1z * e2x - e1x * e2z;
    Nf[3 * f + 2] = e1x * e2y - e1y * e2x;
}

// V2[v] = V[v];  V2[nV + v] = V[v] - eps * unit(sum of the normals of v's faces).
__global__ __launch_bounds__(kBlock) void k_flip_vertices(const double *__restrict__ Nf,
                                                          const int32_t *__restrict__ corners,
                                                          const int32_t *__restrict__ vstart,
                                                          const int32_t *__restrict__ vend,
                                                          const float *__restrict__ V, int64_t nV, float eps,
                                                          float *__restrict__ V2) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    double a[3] = {0.0, 0.0, 0.0};
    for (int32_t i = vstart[v]; i < vend[v]; ++i) {
        const int64_t f = corners[i] / 3;
        for (int d = 0; d < 3; ++d) a[d] += Nf[3 * f + d];
    }
    const double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int d = 0; d < 3; ++d) {
        const double n = len > 0.0 ? a[d] / len : 0.0;
        const float x = V[3 * v + d];
        V2[3 * v + d] = x;
        V2[3 * (nV + v) + d] = (float)((double)x - (double)eps * n);
    }
}

// F2[f] = F[f];  F2[nF + f] = (F[f][0], F[f][2], F[f][1]) + nV  (out-of-range ids -> 0).
__global__ __launch_bounds__(kBlock) void k_flip_faces(const int32_t *__restrict__ F, int64_t nF, int64_t nV,
                                                       int32_t *__restrict__ F2) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    int32_t id[3];
    for (int j = 0; j < 3; ++j) {
        id[j] = F[3 * f + j];
        if (id[j] < 0 || (int64_t)id[j] >= nV) id[j] = 0;
    }
    for (int j = 0; j < 3; ++j) F2[3 * f + j] = id[j];
    F2[3 * (nF + f) + 0] = id[0] + (int32_t)nV;
    F2[3 * (nF + f) + 1] = id[2] + (int32_t)nV;
    F2[3 * (nF + f) + 2] = id[1] + (int32_t)nV;
}

// ------------------------------------------------------------------ host

namespace {

struct BwdPlan {
    int split;      // S: tile t of the points belongs to split t mod S
    int64_t tiles;  // 256-point tiles of the points
    bool wide;      // running-sum space for twice the merged face-pair splits
    unsigned bits;
    size_t sort_tmp;
    size_t off_soup, off_part, off_T, off_keys, off_vals, off_keys2, off_vals2, off_tmp, off_vs, off_ve;
    size_t off_prec, off_pmeta, off_pcount, total;  // face-pair records, metadata, face counts
};

}  // namespace

// Splits of the points: about 32768 waves of (face block, split) work, so that several
// rounds of resident workgroups keep the last, partly filled round short (more splits
// cost more in the per-split sums than they save); at most one split per tile, at most
// 4096, and the running sums (8 B per corner per split) within kBwdStateBytes.  A pure
// function of (nF, nQ), so results never depend on how the points are cut into ranges.
constexpr int64_t kBwdStateBytes = int64_t(256) << 20;

int bwd_splits(int64_t nF, int64_t nQ) {
    const int64_t face_waves = (nF + 63) / 64;
    int64_t sp = (32768 + face_waves - 1) / (face_waves > 0 ? face_waves : 1);
    if (sp > 4096) sp = 4096;
    const int64_t tiles = (nQ + kPointTile - 1) / kPointTile;
    if (sp > tiles) sp = tiles;
    const int64_t by_mem = kBwdStateBytes / (72 * (nF > 0 ? nF : 1));
    if (sp > by_mem) sp = by_mem;
    return (int)(sp < 1 ? 1 : sp);
}

namespace {

BwdPlan plan_backward(int64_t nV, int64_t nF, int64_t nQ) {
    BwdPlan p{};
    p.split = bwd_splits(nF, nQ);
    p.tiles = (nQ + kPointTile - 1) / kPointTile;
    // With at least 12 tiles per split, twice the merged face-pair splits still leave each
    // about 4 tiles, and their shorter workgroups shorten the launch's tail (measured 3.5 %
    // at 128^3 x 5120 faces, nothing at 64^3): the running-sum space is doubled for them.
    p.wide = p.tiles >= 12 * (int64_t)p.split;
    unsigned bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < nV) ++bits;
    p.bits = bits;
    const int64_t nC = 3 * nF;
    size_t tmp = 0;
    if (nC > 0)
        (void)rocprim::radix_sort_pairs(nullptr, tmp, (int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                                  (int32_t *)nullptr, (size_t)nC, 0u, bits);
    p.sort_tmp = tmp;
    size_t o = kWsHeader;
    p.off_soup = o;
    o += align_up((size_t)nF * sizeof(FaceRec));
    p.off_part = o;
    o += align_up((size_t)p.split * 9 * (size_t)nF * sizeof(float2) * (p.wide ? 2 : 1));
    p.off_T = o;
    o += align_up((size_t)nF * 9 * sizeof(float));
    p.off_keys = o;
    o += align_up((size_t)nC * 4);
    p.off_vals = o;
    o += align_up((size_t)nC * 4);
    p.off_keys2 = o;
    o += align_up((size_t)nC * 4);
    p.off_vals2 = o;
    o += align_up((size_t)nC * 4);
    p.off_tmp = o;
    o += align_up(tmp);
    p.off_vs = o;
    o += align_up((size_t)nV * 4);
    p.off_ve = o;
    o += align_up((size_t)nV * 4);
    p.off_prec = o;
    o += align_up((size_t)nF * kPairRecBytes);
    p.off_pmeta = o;
    o += align_up((size_t)nF * kPairMetaBytes);
    p.off_pcount = o;
    o += align_up((size_t)nF * 4);
    p.total = o;
    return p;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t bwd_workspace(int64_t nV, int64_t nF, int64_t nQ) { return plan_backward(nV, nF, nQ).total; }

// The flip reuses the adjoint's layout with no points: the corner sort buffers, vertex
// bounds, and the face-normal table in place of the per-split partials.
size_t flip_workspace(int64_t nV, int64_t nF) {
    const BwdPlan p = plan_backward(nV, nF, 0);
    return p.total + align_up((size_t)nF * 3 * sizeof(double));
}

wn_status run_flip(const float *V, int64_t nV, const int32_t *F, int64_t nF, float eps, float *V2, int32_t *F2,
                   char *ws, size_t ws_bytes, hipStream_t s) {
    const BwdPlan p = plan_backward(nV, nF, 0);
    if (ws_bytes < flip_workspace(nV, nF)) return WN_ERR_WORKSPACE;
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    double *Nf = reinterpret_cast<double *>(ws + p.total);
    int32_t *keys = reinterpret_cast<int32_t *>(ws + p.off_keys);
    int32_t *vals = reinterpret_cast<int32_t *>(ws + p.off_vals);
    int32_t *keys2 = reinterpret_cast<int32_t *>(ws + p.off_keys2);
    int32_t *vals2 = reinterpret_cast<int32_t *>(ws + p.off_vals2);
    int32_t *vs = reinterpret_cast<int32_t *>(ws + p.off_vs);
    int32_t *ve = reinterpret_cast<int32_t *>(ws + p.off_ve);
    hipError_t e = launch_ws_reset(hdr, s);
    if (e != hipSuccess) return WN_ERR_HIP;
    const int64_t nC = 3 * nF;
    if (nV > 0) {
        k_fill_i32<<<blocks_for(nV), kBlock, 0, s>>>(vs, nV, 0);
        k_fill_i32<<<blocks_for(nV), kBlock, 0, s>>>(ve, nV, 0);
    }
    if (nF > 0) {
        k_face_normals<<<blocks_for(nF), kBlock, 0, s>>>(V, nV, F, nF, Nf, hdr);
        k_corner_keys<<<blocks_for(nC), kBlock, 0, s>>>(F, nC, nV, keys, vals);
        if ((e = hipGetLastError()) != hipSuccess) return WN_ERR_HIP;
        size_t tmp = p.sort_tmp;
        e = rocprim::radix_sort_pairs(ws + p.off_tmp, tmp, keys, keys2, vals, vals2, (size_t)nC, 0u, p.bits, s);
        if (e != hipSuccess) return WN_ERR_HIP;
        k_bounds<<<blocks_for(nC), kBlock, 0, s>>>(keys2, nC, vs, ve);
        k_flip_faces<<<blocks_for(nF), kBlock, 0, s>>>(F, nF, nV, F2);
    }
    if (nV > 0) k_flip_vertices<<<blocks_for(nV), kBlock, 0, s>>>(Nf, vals2, vs, ve, V, nV, eps, V2);
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status run_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *pairs, int64_t nP,
                       const PointSrc &ps, int64_t nQ, const float *dLdW, int64_t p0, int64_t n, int flags,
                       float *dLdV, float *dLdT, char *ws, size_t ws_bytes, hipStream_t s, bool naive) {
    const BwdPlan p = plan_backward(nV, nF, nQ);
    if (ws_bytes < p.total) return WN_ERR_WORKSPACE;
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    FaceRec *soup = reinterpret_cast<FaceRec *>(ws + p.off_soup);
    float2 *state = reinterpret_cast<float2 *>(ws + p.off_part);
    hipError_t e = hipSuccess;

    char *prec = ws + p.off_prec;
    char *pmeta = ws + p.off_pmeta;
    int32_t *pcount = reinterpret_cast<int32_t *>(ws + p.off_pcount);
    const bool use_pairs = pairs != nullptr && !naive && nP > 0;
    const bool merged = use_pairs && (flags & kBwdVertexSums);  // 12 running sums per pair
    // begin: face (or face-pair) records and the index checks for the whole call sequence
    if (flags & kBwdBegin) {
        if ((e = launch_ws_reset(hdr, s)) != hipSuccess) return WN_ERR_HIP;
        if (nV > 0 && nF > 0 && !use_pairs && (e = launch_pack(V, nV, F, nF, soup, hdr, s)) != hipSuccess)
            return WN_ERR_HIP;
        if (nV > 0 && nF > 0 && use_pairs &&
            (e = launch_pack_pairs(V, nV, F, nF, pairs, nP, prec, pmeta, pcount, hdr, s)) != hipSuccess)
            return WN_ERR_HIP;
    }
    // With pairs the running sums take 18 float2 per pair and split (12 when merged); the
    // split count is the largest that fits the space sized for 9 per face and split (the
    // same S when nP <= nF / 2 and not merged, 1.5 S merged; merged and wide, twice that in
    // the doubled space), and at most one split per tile.  More splits mean shorter
    // workgroups and a shorter tail of the launch.
    const int64_t per_pair = merged ? 12 : 18, space = (merged && p.wide) ? 2 : 1;
    const int S = use_pairs ? (int)std::max<int64_t>(
                                  1, std::min<int64_t>(p.tiles, space * ((int64_t)p.split * 9 * nF / (per_pair * nP))))
                            : p.split;
    // points [p0, p0 + n): its tiles [t0, t1), one workgroup row per split that owns one
    if (n > 0 && nV > 0 && nF > 0) {
        const int64_t t0 = p0 / kPointTile, t1 = (p0 + n + kPointTile - 1) / kPointTile;
        const int64_t rows = min((int64_t)S, t1 - t0);
        if (naive) {
            e = launch_naive_bwd(soup, (int32_t)nF, ps, nQ, p.split, t0, t1, (int32_t)rows, dLdW, state, s);
        } else if (use_pairs) {
            e = launch_bwd_pairs(prec, pmeta, (int32_t)nP, (int32_t)nF, ps, nQ, S, t0, t1, (int32_t)rows, dLdW, state,
                                 merged, s);
        } else {
            k_wn_bwd<<<dim3(blocks_for(nF), (unsigned)rows), kBlock, 0, s>>>(soup, (int32_t)nF, ps, nQ, p.split, t0,
                                                                              t1, dLdW, state);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return WN_ERR_HIP;
    }
    if (!(flags & kBwdEnd) || nV == 0) return WN_OK;

    // end: the splits added in order, then corners grouped per vertex
    if (nF == 0) {
        k_fill_i32<<<blocks_for(3 * nV), kBlock, 0, s>>>(reinterpret_cast<int32_t *>(dLdV), 3 * nV, 0);
        return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
    }
    float *T = dLdT ? dLdT : reinterpret_cast<float *>(ws + p.off_T);
    int32_t *keys = reinterpret_cast<int32_t *>(ws + p.off_keys);
    int32_t *vals = reinterpret_cast<int32_t *>(ws + p.off_vals);
    int32_t *keys2 = reinterpret_cast<int32_t *>(ws + p.off_keys2);
    int32_t *vals2 = reinterpret_cast<int32_t *>(ws + p.off_vals2);
    int32_t *vs = reinterpret_cast<int32_t *>(ws + p.off_vs);
    int32_t *ve = reinterpret_cast<int32_t *>(ws + p.off_ve);
    if (nQ > 0 && use_pairs) {
        if ((e = launch_reduce_pairs(state, S, (int32_t)nP, pmeta, kInv2Pi, T, merged, s)) != hipSuccess)
            return WN_ERR_HIP;
    } else if (nQ > 0) {
        k_bwd_reduce<<<blocks_for(9 * nF), kBlock, 0, s>>>(state, p.split, (int32_t)nF, naive ? kInv8Pi : kInv2Pi, T);
    } else {
        k_fill_i32<<<blocks_for(9 * nF), kBlock, 0, s>>>(reinterpret_cast<int32_t *>(T), 9 * nF, 0);
    }
    if ((e = hipGetLastError()) != hipSuccess) return WN_ERR_HIP;

    const int64_t nC = 3 * nF;
    k_corner_keys<<<blocks_for(nC), kBlock, 0, s>>>(F, nC, nV, keys, vals);
    if ((e = hipGetLastError()) != hipSuccess) return WN_ERR_HIP;
    size_t tmp = p.sort_tmp;
    e = rocprim::radix_sort_pairs(ws + p.off_tmp, tmp, keys, keys2, vals, vals2, (size_t)nC, 0u, p.bits, s);
    if (e != hipSuccess) return WN_ERR_HIP;
    k_fill_i32<<<blocks_for(nV), kBlock, 0, s>>>(vs, nV, 0);
    k_fill_i32<<<blocks_for(nV), kBlock, 0, s>>>(ve, nV, 0);
    k_bounds<<<blocks_for(nC), kBlock, 0, s>>>(keys2, nC, vs, ve);
    k_gather<<<blocks_for(nV), kBlock, 0, s>>>(T, vals2, vs, ve, nV, dLdV);
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

}  // namespace wn
