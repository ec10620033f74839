// Naive flux integral of Section 2.1, Eq. 4: one sample per face at its centroid c
// with the area-weighted normal N / 2, N = (v1 - v0) x (v2 - v0):
//   W(q) ~= 1/(8 pi) sum_f <N_f, c_f - q> / |c_f - q|^3.
// The paper uses it for mesh morphing (Section 2.4) because, unlike the exact solid
// angles, its gradient with respect to the vertices does not vanish.  A face whose
// centroid coincides with q contributes 0.
//
// Forward: the same layout as the exact kernel (PPL points per lane, face records
// broadcast from LDS, Neumaier fold per tile, fixed-order split reduction); per pair
// one rsqrt and about 15 FP32 operations.  Adjoint: one lane per face, points
// broadcast from LDS, per pair
//   dg/dv_j = (N/|r|^3 - 3 <N, r> r/|r|^5) / 3 + (v_{j+1} - v_{j+2}) x r/|r|^3,
// then the adjoint's fixed-order split reduction and deterministic corner gather.
#include "wn_internal.hpp"

namespace wn {

struct NaiveRec {
    float4 c;  // centroid (w = 0)
    float4 n;  // N = (v1 - v0) x (v2 - v0) (w = 0)
};

__global__ __launch_bounds__(kBlock) void k_pack_naive(const float *__restrict__ V, int64_t nV,
                                                       const int32_t *__restrict__ F, int64_t nF,
                                                       NaiveRec *__restrict__ recs, WsHeader *hdr) {
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
    NaiveRec r;
    r.c = make_float4((float)((v[0][0] + v[1][0] + v[2][0]) / 3.0), (float)((v[0][1] + v[1][1] + v[2][1]) / 3.0),
                      (float)((v[0][2] + v[1][2] + v[2][2]) / 3.0), 0.0f);
    r.n = make_float4((float)(e1y * e2z - e1z * e2y), (float)(e1z * e2x - e1x * e2z), (float)(e1x * e2y - e1y * e2x),
                      0.0f);
    recs[f] = r;
}

template <int PPL>
__global__ __launch_bounds__(kBlock) void k_naive_fwd(const NaiveRec *__restrict__ recs, int64_t nF, int64_t chunk,
                                                      PointSrc ps, int64_t nQ, float *__restrict__ W,
                                                      float *__restrict__ partials, OccParams occ) {
    __shared__ float4 tile[kFaceTile * 2];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kBlock * PPL) + tid;
    const int64_t f0 = (int64_t)blockIdx.y * chunk;
    const int64_t f1 = min(nF, f0 + chunk);
    float qx[PPL], qy[PPL], qz[PPL], s[PPL], c[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int64_t idx = base + (int64_t)p * kBlock;
        idx = idx < nQ ? idx : nQ - 1;
        ps.get(idx, qx[p], qy[p], qz[p]);
        s[p] = 0.0f;
        c[p] = 0.0f;
    }
    const float4 *src = reinterpret_cast<const float4 *>(recs);
    for (int64_t t0 = f0; t0 < f1; t0 += kFaceTile) {
        const int nt = (int)min((int64_t)kFaceTile, f1 - t0);
        __syncthreads();
        if (tid < 2 * nt) tile[tid] = src[2 * t0 + tid];
        __syncthreads();
        float ts[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) ts[p] = 0.0f;
#pragma unroll 4
        for (int i = 0; i < nt; ++i) {
            const float4 cc = tile[2 * i], n = tile[2 * i + 1];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const float rx = cc.x - qx[p], ry = cc.y - qy[p], rz = cc.z - qz[p];
                const float r2 = rx * rx + ry * ry + rz * rz;
                const float is = (r2 > 0.0f) ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                ts[p] += (n.x * rx + n.y * ry + n.z * rz) * (is * is * is);
            }
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) neumaier_add(s[p], c[p], ts[p]);
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int64_t idx = base + (int64_t)p * kBlock;
        if (idx >= nQ) continue;
        const float tot = s[p] + c[p];
        if (partials) {
            partials[(int64_t)blockIdx.y * nQ + idx] = tot;
        } else {
            const float w = tot * kInv8Pi;
            W[idx] = w;
            write_occ(occ, idx, w);
        }
    }
}

// Adjoint pair kernel: grid x = face blocks, y = the splits owning a tile of [t0, t1)
// (split (t0 + y) mod S, tiles of kBwdTile points dealt to the splits in turn); running
// sums in state, float2 [S][9][nF] (the layout of the exact adjoint).
__global__ __launch_bounds__(kBlock) void k_naive_bwd(const FaceRec *__restrict__ soup, int32_t nF, PointSrc ps,
                                                      int64_t nQ, int32_t S, int64_t t0, int64_t t1,
                                                      const float *__restrict__ dLdW, float2 *__restrict__ state) {
    __shared__ float4 pts[kBlock];
    const int tid = threadIdx.x;
    const int64_t tfirst = t0 + blockIdx.y;  // this block's first tile
    const int64_t sy = tfirst % S;           // its split
    int32_t f = (int32_t)blockIdx.x * kBlock + tid;
    const bool live = f < nF;
    f = live ? f : nF - 1;
    const FaceRec r = soup[f];
    const float v[3][3] = {{r.a.x, r.a.y, r.a.z}, {r.a.w, r.b.x, r.b.y}, {r.b.z, r.b.w, r.c.x}};
    const float N[3] = {r.c.y, r.c.z, r.c.w};
    const float third = 1.0f / 3.0f;
    const float cen[3] = {(v[0][0] + v[1][0] + v[2][0]) * third, (v[0][1] + v[1][1] + v[2][1]) * third,
                          (v[0][2] + v[1][2] + v[2][2]) * third};
    float e[3][3];  // e_j = v_{j+1} - v_{j+2}
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) e[j][d] = v[(j + 1) % 3][d] - v[(j + 2) % 3][d];
    float s[9], c[9];
    load_state(state, sy, nF, f, tfirst < S, s, c);
    for (int64_t t = tfirst; t < t1; t += S) {
        const int64_t q0 = t * kBwdTile;
        const int nt = (int)min((int64_t)kBwdTile, nQ - q0);
        __syncthreads();
        if (tid < nt) {
            float x, y, z;
            ps.get(q0 + tid, x, y, z);
            pts[tid] = make_float4(x, y, z, dLdW[q0 + tid]);
        }
        __syncthreads();
        // Per corner j the pair adds u + e_j x a, where u (the centroid part, shared by the
        // three corners) and a = g r/|r|^3 depend on the point and e_j does not; so the
        // tile sums U = sum u and A = sum a are formed first and corner j gets U + e_j x A.
        float U[3] = {0.0f, 0.0f, 0.0f}, A[3] = {0.0f, 0.0f, 0.0f};
        for (int i = 0; i < nt; ++i) {
            const float4 q = pts[i];
            const float rx = cen[0] - q.x, ry = cen[1] - q.y, rz = cen[2] - q.z;
            const float r2 = rx * rx + ry * ry + rz * rz;
            const float is = (r2 > 0.0f) ? __builtin_amdgcn_rsqf(r2) : 0.0f;
            const float is2 = is * is;
            const float is3g = is2 * is * q.w;                  // g / |r|^3
            const float nr = N[0] * rx + N[1] * ry + N[2] * rz;
            const float kr = -nr * is2 * is3g;                  // -g <N, r> / |r|^5
            // centroid part: g (N/|r|^3 - 3 <N,r> r/|r|^5) / 3 = third * (N is3g) + kr * r
            U[0] += third * N[0] * is3g + kr * rx;
            U[1] += third * N[1] * is3g + kr * ry;
            U[2] += third * N[2] * is3g + kr * rz;
            A[0] += rx * is3g;
            A[1] += ry * is3g;
            A[2] += rz * is3g;
        }
        float ts[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            ts[3 * j + 0] = U[0] + (e[j][1] * A[2] - e[j][2] * A[1]);
            ts[3 * j + 1] = U[1] + (e[j][2] * A[0] - e[j][0] * A[2]);
            ts[3 * j + 2] = U[2] + (e[j][0] * A[1] - e[j][1] * A[0]);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) neumaier_add(s[i], c[i], ts[i]);
    }
    if (live) store_state(state, sy, nF, f, s, c);
}

// ------------------------------------------------------------------ host

size_t naive_fwd_workspace(int64_t nF, int64_t nQ) {
    const int split = fwd_split_count(nF, nQ);
    size_t b = kWsHeader + align_up((size_t)nF * sizeof(NaiveRec));
    if (split > 1) b += align_up((size_t)split * (size_t)nQ * sizeof(float));
    return b;
}

template <int PPL>
static void launch_naive_ppl(const NaiveRec *recs, int64_t nF, int64_t chunk, int split, const PointSrc &ps,
                             int64_t nQ, float *W, float *partials, const OccParams &occ, hipStream_t s) {
    const int64_t pblocks = (nQ + kBlock * PPL - 1) / (kBlock * PPL);
    k_naive_fwd<PPL><<<dim3((unsigned)pblocks, (unsigned)split), kBlock, 0, s>>>(
        recs, nF, chunk, ps, nQ, W, split > 1 ? partials : nullptr, occ);
}

hipError_t launch_naive_fwd(const float *V, int64_t nV, const int32_t *F, int64_t nF, const PointSrc &ps,
                            int64_t nQ, float *W, const OccParams &occ, char *ws, int ppl, hipStream_t s) {
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    NaiveRec *recs = reinterpret_cast<NaiveRec *>(ws + kWsHeader);
    float *partials = reinterpret_cast<float *>(ws + kWsHeader + align_up((size_t)nF * sizeof(NaiveRec)));
    hipError_t e = launch_ws_reset(hdr, s);
    if (e != hipSuccess) return e;
    if (nF > 0) {
        k_pack_naive<<<dim3((unsigned)((nF + kBlock - 1) / kBlock)), kBlock, 0, s>>>(V, nV, F, nF, recs, hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (nQ <= 0) return hipSuccess;
    const int split = fwd_split_count(nF, nQ);
    const int64_t per = (nF + split - 1) / split;
    int64_t chunk = (per + kFaceTile - 1) / kFaceTile * kFaceTile;
    if (chunk < kFaceTile) chunk = kFaceTile;
    if (ppl == 1)
        launch_naive_ppl<1>(recs, nF, chunk, split, ps, nQ, W, partials, occ, s);
    else if (ppl == 4)
        launch_naive_ppl<4>(recs, nF, chunk, split, ps, nQ, W, partials, occ, s);
    else
        launch_naive_ppl<2>(recs, nF, chunk, split, ps, nQ, W, partials, occ, s);
    if ((e = hipGetLastError()) != hipSuccess || split <= 1) return e;
    return launch_split_reduce(partials, split, nQ, kInv8Pi, W, occ, s);
}

hipError_t launch_naive_bwd(const FaceRec *soup, int32_t nF, const PointSrc &ps, int64_t nQ, int32_t S, int64_t t0,
                            int64_t t1, int32_t rows, const float *dLdW, float2 *state, hipStream_t s) {
    k_naive_bwd<<<dim3((unsigned)((nF + kBlock - 1) / kBlock), (unsigned)rows), kBlock, 0, s>>>(soup, nF, ps, nQ, S,
                                                                                               t0, t1, dLdW, state);
    return hipGetLastError();
}

}  // namespace wn
