// Forward path on gfx950: mesh packing, the all-pairs winding-number kernel,
// the fixed-order split reduction, occupancy maps and the sigmoid-MSE loss.
//
// Section 2.2 of arXiv 2407.11272 (Eq. 5, 7, 8) and Algorithm 1 define the
// arithmetic; the layout and launch shapes are this library's own:
//   * one lane owns PPL query points and keeps their sums in registers;
//   * the mesh streams through LDS as vertex records (three per face, or triangle
//     strips with one per face), each record read by every lane of the workgroup
//     (a broadcast read, no bank conflicts);
//   * each tile's per-point sum is folded into a Neumaier-compensated total;
//   * when the point count alone cannot fill the GPU, the faces are split over
//     workgroups and the partial sums are added in a fixed order afterwards.
#include "wn_internal.hpp"

namespace wn {

// ------------------------------------------------------------------ kernels

__global__ void k_ws_reset(WsHeader *hdr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        hdr->bad_index = 0;
        hdr->cursor = 0ull;
    }
}

// One thread per face: gather its three vertices (indices outside [0, nV) are
// replaced by 0 and recorded), compute the face normal N = (v1 - v0) x (v2 - v0)
// in FP64 and store the 48-byte record.
__global__ __launch_bounds__(kBlock) void k_pack(const float *__restrict__ V, int64_t nV,
                                                 const int32_t *__restrict__ F, int64_t nF,
                                                 FaceRec *__restrict__ soup, WsHeader *hdr) {
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
    float v[3][3];
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) v[j][c] = V[3 * (int64_t)id[j] + c];
    const double e1x = (double)v[1][0] - v[0][0], e1y = (double)v[1][1] - v[0][1], e1z = (double)v[1][2] - v[0][2];
    const double e2x = (double)v[2][0] - v[0][0], e2y = (double)v[2][1] - v[0][1], e2z = (double)v[2][2] - v[0][2];
    const float nx = (float)(e1y * e2z - e1z * e2y);
    const float ny = (float)(e1z * e2x - e1x * e2z);
    const float nz = (float)(e1x * e2y - e1y * e2x);
    FaceRec r;
    r.a = make_float4(v[0][0], v[0][1], v[0][2], v[1][0]);
    r.b = make_float4(v[1][1], v[1][2], v[2][0], v[2][1]);
    r.c = make_float4(v[2][2], nx, ny, nz);
    soup[f] = r;
}

__global__ __launch_bounds__(kBlock) void k_pack_records(const float *__restrict__ V, int64_t nV,
                                                         const int32_t *__restrict__ F, int64_t nF,
                                                         const int32_t *__restrict__ R, int64_t nR,
                                                         VRec *__restrict__ recs, WsHeader *hdr) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    int32_t vid, fid;
    if (R) {
        vid = R[2 * r];
        fid = R[2 * r + 1];
        check_strip_record(R, r, F, nF, fid, hdr);
    } else {
        const int64_t f = r / 3;
        const int j = (int)(r - 3 * f);
        vid = F[3 * f + j];
        fid = j == 2 ? (int32_t)f : -1;
    }
    recs[r] = make_record(V, nV, F, nF, vid, fid, hdr);
}

// All-pairs forward.  Grid: x = point blocks of kBlock * PPL points, y = record splits.
// With split == 1 the kernel writes W (scaled by 1 / 2 pi) and the occupancy map;
// otherwise it writes the unscaled partial sum of split y to partials[y * nQ + idx].
template <int PPL, int DEPTH>
__global__ __launch_bounds__(kBlock) void k_wn_fwd(const VRec *__restrict__ recs, int64_t nR, int64_t chunk,
                                                   PointSrc ps, int64_t nQ, float *__restrict__ W,
                                                   float *__restrict__ partials, OccParams occ) {
    __shared__ float4 tile[kRecTile * 2 * DEPTH];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kBlock * PPL) + tid;
    const int64_t r0 = (int64_t)blockIdx.y * chunk;
    const int64_t r1 = min(nR, r0 + chunk);

    float qx[PPL], qy[PPL], qz[PPL], s[PPL], c[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int64_t idx = base + (int64_t)p * kBlock;
        idx = idx < nQ ? idx : nQ - 1;
        ps.get(idx, qx[p], qy[p], qz[p]);
        s[p] = 0.0f;
        c[p] = 0.0f;
    }
    sum_records<PPL, DEPTH>(reinterpret_cast<const float4 *>(recs), r0, r1, tile, qx, qy, qz, s, c);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int64_t idx = base + (int64_t)p * kBlock;
        if (idx >= nQ) continue;
        const float tot = s[p] + c[p];
        if (partials) {
            partials[(int64_t)blockIdx.y * nQ + idx] = tot;
        } else {
            const float w = tot * kInv2Pi;
            W[idx] = w;
            write_occ(occ, idx, w);
        }
    }
}

// Fixed-order sum of the split partials, scale to W, occupancy.
__global__ __launch_bounds__(kBlock) void k_wn_reduce(const float *__restrict__ partials, int32_t split,
                                                      int64_t nQ, float scale, float *__restrict__ W, OccParams occ) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nQ) return;
    float s = 0.0f, c = 0.0f;
    for (int32_t k = 0; k < split; ++k) neumaier_add(s, c, partials[(int64_t)k * nQ + idx]);
    const float w = (s + c) * scale;
    W[idx] = w;
    write_occ(occ, idx, w);
}

__global__ __launch_bounds__(kBlock) void k_occ(const float *__restrict__ W, int64_t n, OccParams occ) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    write_occ(occ, idx, W[idx]);
}

// Chain rule through the soft occupancy s = sigmoid(k (W - tau)): dL/dW = g k s (1 - s),
// with s recomputed from W as the forward map computes it.
__global__ __launch_bounds__(kBlock) void k_occ_bwd(const float *__restrict__ W, const float *__restrict__ g,
                                                    int64_t n, float tau, float k, float *__restrict__ dLdW) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float sg = sigmoidf(k * (W[idx] - tau));
    dLdW[idx] = g[idx] * k * sg * (1.0f - sg);
}

// Sigmoid-MSE: per block, a fixed-shape tree sum of (s - t)^2; per element dL/dW.
constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_sigmoid_mse(const float *__restrict__ W, const float *__restrict__ T,
                                                        int64_t n, float tau, float k, float inv_n,
                                                        float *__restrict__ dLdW, float *__restrict__ block_sums) {
    __shared__ float red[kBlock];
    float acc = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float sg = sigmoidf(k * (W[i] - tau));
        const float d = sg - T[i];
        acc += d * d;
        if (dLdW) dLdW[i] = 2.0f * d * inv_n * k * sg * (1.0f - sg);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_loss_final(const float *__restrict__ block_sums, int nb, float inv_n,
                                                       float *__restrict__ loss) {
    __shared__ float red[kBlock];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += block_sums[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * inv_n;
}

// ---------------------------------------------------------------- launchers

int fwd_split_count(int64_t nR, int64_t nQ) {
    // Aim for about 131072 wave64s of (point block, record split) units, about 16
    // rounds of resident workgroups, so that the last, partly filled round costs little
    // (one round of 8192 point blocks left the GPU 5-10 % idle at the end); never give a
    // split fewer than 2 tiles of records.  Depends only on (nR, nQ), so results do not
    // depend on the launch configuration.
    const int64_t waves = (nQ + 63) / 64;
    int64_t s = (131072 + waves - 1) / (waves > 0 ? waves : 1);
    const int64_t max_by_faces = (nR + 2 * kRecTile - 1) / (2 * kRecTile);
    if (s > max_by_faces) s = max_by_faces;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    return (int)s;
}

int64_t fwd_split_chunk(int64_t nR, int split) {
    const int64_t per = (nR + split - 1) / (split > 0 ? split : 1);
    const int64_t chunk = (per + kRecTile - 1) / kRecTile * kRecTile;
    return chunk > 0 ? chunk : kRecTile;
}

PointSrc make_point_src(const wn_grid *grid, const float *Q) {
    PointSrc ps{};
    ps.Q = Q;
    if (grid) {
        for (int d = 0; d < 3; ++d) {
            ps.lo[d] = grid->lo[d];
            ps.h[d] = (float)(((double)grid->hi[d] - (double)grid->lo[d]) / (double)grid->n[d]);
        }
        ps.n1 = grid->n[1];
        ps.n2 = grid->n[2];
    }
    return ps;
}

hipError_t launch_ws_reset(WsHeader *hdr, hipStream_t s) {
    k_ws_reset<<<1, 64, 0, s>>>(hdr);
    return hipGetLastError();
}

hipError_t launch_pack(const float *V, int64_t nV, const int32_t *F, int64_t nF, FaceRec *soup, WsHeader *hdr,
                       hipStream_t s) {
    if (nF <= 0) return hipSuccess;
    const int64_t blocks = (nF + kBlock - 1) / kBlock;
    k_pack<<<dim3((unsigned)blocks), kBlock, 0, s>>>(V, nV, F, nF, soup, hdr);
    return hipGetLastError();
}

hipError_t launch_pack_records(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *R,
                               int64_t nR, VRec *recs, WsHeader *hdr, hipStream_t s) {
    if (nR <= 0) return hipSuccess;
    const int64_t blocks = (nR + kBlock - 1) / kBlock;
    k_pack_records<<<dim3((unsigned)blocks), kBlock, 0, s>>>(V, nV, F, nF, R, nR, recs, hdr);
    return hipGetLastError();
}

hipError_t launch_fwd(const VRec *recs, int64_t nR, const PointSrc &ps, int64_t nQ, int split, float *W,
                      float *partials, const OccParams &occ, int ppl, int depth, hipStream_t s) {
    if (nQ <= 0) return hipSuccess;
    const int64_t chunk = fwd_split_chunk(nR, split);
    hipError_t e = with_config(ppl, depth, [&](auto P, auto D) {
        constexpr int kP = decltype(P)::value, kD = decltype(D)::value;
        const int64_t pblocks = (nQ + kBlock * kP - 1) / (kBlock * kP);
        k_wn_fwd<kP, kD><<<dim3((unsigned)pblocks, (unsigned)split), kBlock, 0, s>>>(
            recs, nR, chunk, ps, nQ, W, split > 1 ? partials : nullptr, occ);
        return hipGetLastError();
    });
    if (e != hipSuccess || split <= 1) return e;
    const int64_t rblocks = (nQ + kBlock - 1) / kBlock;
    k_wn_reduce<<<dim3((unsigned)rblocks), kBlock, 0, s>>>(partials, split, nQ, kInv2Pi, W, occ);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_checksum(const uint32_t *__restrict__ x, int64_t n,
                                                     unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += x[i];
    if (acc) atomicAdd(out, acc);  // integer sums: the result does not depend on the order
}

__global__ void k_checksum_reset(WsHeader *hdr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) hdr->checksum = 0ull;
}

hipError_t launch_checksum(const float *x, int64_t n, WsHeader *hdr, bool reset, hipStream_t s) {
    if (reset) k_checksum_reset<<<1, 64, 0, s>>>(hdr);
    if (n > 0) k_checksum<<<1024, kBlock, 0, s>>>(reinterpret_cast<const uint32_t *>(x), n, &hdr->checksum);
    return hipGetLastError();
}

hipError_t launch_split_reduce(const float *partials, int split, int64_t nQ, float scale, float *W,
                               const OccParams &occ, hipStream_t s) {
    const int64_t rblocks = (nQ + kBlock - 1) / kBlock;
    k_wn_reduce<<<dim3((unsigned)rblocks), kBlock, 0, s>>>(partials, split, nQ, scale, W, occ);
    return hipGetLastError();
}

hipError_t launch_occ(const float *W, int64_t n, const OccParams &occ, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_occ<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(W, n, occ);
    return hipGetLastError();
}

hipError_t launch_occ_bwd(const float *W, const float *g, int64_t n, float tau, float k, float *dLdW,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_occ_bwd<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(W, g, n, tau, k, dLdW);
    return hipGetLastError();
}

int loss_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > kLossBlocks) b = kLossBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_sigmoid_mse(const float *W, const float *target, int64_t n, float tau, float k, float *loss,
                              float *dLdW, float *scratch, hipStream_t s) {
    const int nb = loss_blocks(n);
    const float inv_n = n > 0 ? (float)(1.0 / (double)n) : 0.0f;
    k_sigmoid_mse<<<nb, kBlock, 0, s>>>(W, target, n, tau, k, inv_n, dLdW, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    k_loss_final<<<1, kBlock, 0, s>>>(scratch, nb, inv_n, loss);
    return hipGetLastError();
}

}  // namespace wn
