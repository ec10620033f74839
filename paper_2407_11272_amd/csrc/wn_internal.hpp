// Internal header of the gfx950 winding-number library: device arithmetic,
// workspace layout and the host-side launch interface shared by the .hip files.
//
// Per (query point q, face f) the kernels evaluate the half solid angle
//   t_f(q) = ATAN2(alpha, beta)        (Section 2.2, Eq. 7 and Eq. 8)
// in a scale-free form that needs no normalised vectors: with R_j = v_j - q,
// r_j = |R_j|, and the face normal N = (v1 - v0) x (v2 - v0) computed once per face,
//   alpha' = det(R0, R1, R2) = R0 . N
//   beta'  = r0 r1 r2 + (R0.R1) r2 + (R1.R2) r0 + (R2.R0) r1
// which are alpha and beta of Eq. 7 multiplied by the positive factor r0 r1 r2, so
// ATAN2(alpha', beta') = ATAN2(alpha, beta).  W(q) = sum_f t_f(q) / (2 pi) (Eq. 5 with
// Omega = 2 t).  A vertex that coincides with q makes r0 r1 r2 = 0; that face then
// contributes 0, as a zero-length direction contributes no determinant.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "wn.h"

namespace wn {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489662f;
constexpr float kInv2Pi = 0.159154943091895336f;
constexpr float kFltMin = 1.17549435e-38f;

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kFaceTile = 64;    // faces staged in LDS per tile (3 float4 each)
constexpr int kWsHeader = 256;   // bytes reserved at the start of every workspace

// Face record in device memory: 12 floats = 3 float4.
//   a = (v0.x, v0.y, v0.z, v1.x)  b = (v1.y, v1.z, v2.x, v2.y)  c = (v2.z, N.x, N.y, N.z)
struct FaceRec {
    float4 a, b, c;
};

// Header at the start of each workspace.
struct WsHeader {
    int32_t bad_index;            // set to non-zero by a pack kernel on an out-of-range face index
    int32_t pad0;
    unsigned long long cursor;    // work-unit cursor of the persistent kernel
    int32_t pad[60];
};
static_assert(sizeof(WsHeader) == kWsHeader, "header size");

// ---------------------------------------------------------------- device math

// atan(t) for t in [0, 1] as t P(t^2): minimax in relative error (Remez exchange,
// degree 7 in t^2; coefficients from gen_atan_poly.py, max relative error 2.2e-7
// when evaluated in FP32).
__device__ __forceinline__ float atan_unit(float t) {
    const float x = t * t;
    float p = -0.0046932762f;
    p = __builtin_fmaf(p, x, 0.024252404f);
    p = __builtin_fmaf(p, x, -0.059486393f);
    p = __builtin_fmaf(p, x, 0.09914293f);
    p = __builtin_fmaf(p, x, -0.1401948f);
    p = __builtin_fmaf(p, x, 0.19969724f);
    p = __builtin_fmaf(p, x, -0.3333199f);
    p = __builtin_fmaf(p, x, 0.9999999f);
    return p * t;
}

// ATAN2(y, x) with the case table of Eq. 8: ATAN2(+-0, +-0) = 0 and, for x < 0,
// y = -0 takes the y >= 0 branch (+pi).  Finite inputs; NaN propagates.
__device__ __forceinline__ float atan2_eq8(float y, float x) {
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float mn = __builtin_fminf(ax, ay);
    const float mx = __builtin_fmaxf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(__builtin_fmaxf(mx, kFltMin));
    float a = atan_unit(t);
    a = (ay > ax) ? (kHalfPi - a) : a;
    a = (x < 0.0f) ? (kPi - a) : a;
    return (y < 0.0f) ? -a : a;
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Half solid angle t_f(q) of one face record at point q (see the header comment).
__device__ __forceinline__ float half_solid_angle(const float4 &a, const float4 &b, const float4 &c,
                                                  float qx, float qy, float qz) {
    const float r0x = a.x - qx, r0y = a.y - qy, r0z = a.z - qz;
    const float r1x = a.w - qx, r1y = b.x - qy, r1z = b.y - qz;
    const float r2x = b.z - qx, r2y = b.w - qy, r2z = c.x - qz;
    const float l0 = fast_sqrt(r0x * r0x + r0y * r0y + r0z * r0z);
    const float l1 = fast_sqrt(r1x * r1x + r1y * r1y + r1z * r1z);
    const float l2 = fast_sqrt(r2x * r2x + r2y * r2y + r2z * r2z);
    const float d01 = r0x * r1x + r0y * r1y + r0z * r1z;
    const float d12 = r1x * r2x + r1y * r2y + r1z * r2z;
    const float d20 = r2x * r0x + r2y * r0y + r2z * r0z;
    const float p = l0 * l1 * l2;
    const float beta = p + d01 * l2 + d12 * l0 + d20 * l1;
    float alpha = r0x * c.y + r0y * c.z + r0z * c.w;
    alpha = (p == 0.0f) ? 0.0f : alpha;
    return atan2_eq8(alpha, beta);
}

// Neumaier step: (s, c) += x.
__device__ __forceinline__ void neumaier_add(float &s, float &c, float x) {
    const float t = s + x;
    const float big = (__builtin_fabsf(s) >= __builtin_fabsf(x)) ? s : x;
    const float small = (__builtin_fabsf(s) >= __builtin_fabsf(x)) ? x : s;
    c += (big - t) + small;
    s = t;
}

// Where the query points come from: an explicit list or the voxel centres of a grid.
struct PointSrc {
    const float *Q;      // [n][3] or nullptr for grid mode
    float lo[3];
    float h[3];          // (hi - lo) / n per axis
    int32_t n1, n2;      // cells along y and z

    __device__ __forceinline__ void get(int64_t idx, float &x, float &y, float &z) const {
        if (Q) {
            x = Q[3 * idx + 0];
            y = Q[3 * idx + 1];
            z = Q[3 * idx + 2];
        } else {
            const int64_t yz = (int64_t)n1 * n2;
            const int32_t i = (int32_t)(idx / yz);
            const int32_t rem = (int32_t)(idx - (int64_t)i * yz);
            const int32_t j = rem / n2;
            const int32_t k = rem - j * n2;
            x = __builtin_fmaf((float)i + 0.5f, h[0], lo[0]);
            y = __builtin_fmaf((float)j + 0.5f, h[1], lo[1]);
            z = __builtin_fmaf((float)k + 0.5f, h[2], lo[2]);
        }
    }
};

// Sum over faces [f0, f1) of the half solid angles at PPL points per lane.  The whole
// workgroup stages kFaceTile face records at a time through `tile` (LDS, kFaceTile * 3
// float4) and every lane reads each record (broadcast).  Each tile's per-point sum is
// folded into the Neumaier pair (s, c), so the summation order -- and the result --
// depends only on the face order and the tile boundaries, not on PPL or the launch.
template <int PPL>
__device__ __forceinline__ void sum_faces(const float4 *__restrict__ src, int32_t f0, int32_t f1, float4 *tile,
                                          const float (&qx)[PPL], const float (&qy)[PPL], const float (&qz)[PPL],
                                          float (&s)[PPL], float (&c)[PPL]) {
    const int tid = threadIdx.x;
    for (int32_t t0 = f0; t0 < f1; t0 += kFaceTile) {
        const int nt = min(kFaceTile, f1 - t0);
        __syncthreads();
        if (tid < 3 * nt) tile[tid] = src[3 * (int64_t)t0 + tid];
        __syncthreads();
        float ts[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) ts[p] = 0.0f;
#pragma unroll 2
        for (int i = 0; i < nt; ++i) {
            const float4 a = tile[3 * i], b = tile[3 * i + 1], cc = tile[3 * i + 2];
#pragma unroll
            for (int p = 0; p < PPL; ++p) ts[p] += half_solid_angle(a, b, cc, qx[p], qy[p], qz[p]);
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) neumaier_add(s[p], c[p], ts[p]);
    }
}

struct OccParams {
    void *occ;
    int32_t mode;
    float tau;
    float k;
};

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

__device__ __forceinline__ void write_occ(const OccParams &o, int64_t idx, float w) {
    if (o.mode == WN_OCC_THRESHOLD)
        static_cast<uint8_t *>(o.occ)[idx] = (w > o.tau) ? 1 : 0;
    else if (o.mode == WN_OCC_SIGMOID)
        static_cast<float *>(o.occ)[idx] = sigmoidf(o.k * (w - o.tau));
}

// ---------------------------------------------------------------- host side

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Partition of the faces over workgroups when there are too few point blocks to
// fill the GPU.  A pure function of (nF, nQ): results never depend on tuning.
int fwd_split_count(int64_t nF, int64_t nQ);
int32_t fwd_split_chunk(int64_t nF, int split);

PointSrc make_point_src(const wn_grid *grid, const float *Q);

// Forward pieces (wn_fwd.hip).
hipError_t launch_ws_reset(WsHeader *hdr, hipStream_t s);
hipError_t launch_pack(const float *V, int64_t nV, const int32_t *F, int64_t nF, FaceRec *soup,
                       WsHeader *hdr, hipStream_t s);
hipError_t launch_fwd(const FaceRec *soup, int64_t nF, const PointSrc &ps, int64_t nQ, int split,
                      float *W, float *partials, const OccParams &occ, int ppl, hipStream_t s);
hipError_t launch_occ(const float *W, int64_t n, const OccParams &occ, hipStream_t s);
hipError_t launch_sigmoid_mse(const float *W, const float *target, int64_t n, float tau, float k,
                              float *loss, float *dLdW, float *scratch, hipStream_t s);
int loss_blocks(int64_t n);

// Backward pieces (wn_bwd.hip).
size_t bwd_workspace(int64_t nV, int64_t nF, int64_t nQ);
wn_status run_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF, const PointSrc &ps,
                       int64_t nQ, const float *dLdW, float *dLdV, float *dLdT, char *ws, size_t ws_bytes,
                       hipStream_t s);

// Batched pieces (wn_batched.hip).
size_t batched_workspace(const wn_mesh_desc *d, int32_t n);
wn_status run_batched(const wn_mesh_desc *d, int32_t n, int32_t flags, char *ws, size_t ws_bytes,
                      hipStream_t s, const struct TuneConfig *force);

// Launch tuning (wn_tune.hip).  A configuration changes only how work is mapped to
// lanes and workgroups, never the per-point summation order, so results do not
// depend on it.
struct TuneConfig {
    int32_t ppl;        // query points per lane: 1, 2 or 4
    int32_t wg_per_cu;  // persistent workgroups per CU (0 = as many as fit)
};
TuneConfig default_config(int32_t op);
TuneConfig lookup_config(int32_t op, int64_t a, int64_t b);
void store_config(int32_t op, int64_t a, int64_t b, const TuneConfig &c);
bool valid_ppl(int32_t ppl);

}  // namespace wn
