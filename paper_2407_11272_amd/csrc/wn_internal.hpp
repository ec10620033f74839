// Internal header of the gfx950 winding-number library: device arithmetic,
// workspace layout and the host-side launch interface shared by the .hip files.
//
// Per (query point q, face f) the kernels evaluate the half solid angle
//   t_f(q) = ATAN2(alpha, beta)        (Section 2.2, Eq. 7 and Eq. 8)
// in a scale-free form that needs no normalised vectors: with R_j = v_j - q,
// r_j = |R_j|, and the face normal N = (v1 - v0) x (v2 - v0) computed once per face,
//   alpha' = det(R0, R1, R2) = R_j . N   (the same for every vertex j of the face)
//   beta'  = r0 r1 r2 + (R0.R1) r2 + (R1.R2) r0 + (R2.R0) r1
// which are alpha and beta of Eq. 7 multiplied by the positive factor r0 r1 r2, so
// ATAN2(alpha', beta') = ATAN2(alpha, beta).  W(q) = sum_f t_f(q) / (2 pi) (Eq. 5 with
// Omega = 2 t).  A vertex that coincides with q makes r0 r1 r2 = 0; that face then
// contributes 0, as a zero-length direction contributes no determinant.
//
// The forward kernels read the mesh as a stream of vertex records.  A record carries
// one vertex position and, if it completes a face, that face's normal: the face is the
// record's vertex with the vertices of the two records before it.  Three records per
// face (the default) or triangle strips (consecutive faces sharing an edge, one new
// vertex per face) describe the same faces; alpha' and beta' do not depend on the
// order of a face's vertices, and N keeps the face's own winding.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "wn.h"

namespace wn {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489662f;
constexpr float kInv2Pi = 0.159154943091895336f;
constexpr float kFltMin = 1.17549435e-38f;
constexpr float kTwoPi = 6.28318530717958648f;
constexpr float kPairMax = 4.2535296e37f;  // 2^125: the reciprocal of a larger value is not normal

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kFaceTile = 64;    // faces staged in LDS per tile (3 float4 each)
constexpr int kWsHeader = 256;   // bytes reserved at the start of every workspace

// Vertex record of the forward stream: p = (x, y, z, 1 if it completes a face else 0),
// n = (N.x, N.y, N.z, 0) of the completed face.
struct VRec {
    float4 p, n;
};
constexpr int kRecTile = 60;  // records staged in LDS per tile (a multiple of 6, at most 64)

// Face record in device memory (adjoint): 12 floats = 3 float4.
//   a = (v0.x, v0.y, v0.z, v1.x)  b = (v1.y, v1.z, v2.x, v2.y)  c = (v2.z, N.x, N.y, N.z)
struct FaceRec {
    float4 a, b, c;
};

// Header at the start of each workspace.
struct WsHeader {
    int32_t bad_index;            // set to non-zero by a pack kernel on an out-of-range face index
    int32_t pad0;
    unsigned long long cursor;    // work-unit cursor of the persistent kernel
    unsigned long long checksum;  // output checksum of an autotuner candidate
    int32_t pad[58];
};
static_assert(sizeof(WsHeader) == kWsHeader, "header size");

// ---------------------------------------------------------------- device math

// atan(t) for t in [0, 1] as t P(t^2): minimax in relative error (Remez exchange,
// degree 6 in t^2; coefficients from gen_atan_poly.py, max relative error 7.6e-7 and
// absolute error 5.9e-7 when evaluated in FP32).  The polynomial's share of the error in
// W is at most 7.6e-7 times the sum of |angle| / 2 pi over a point's faces: about 8e-7
// per closed surface around the point, 6e-6 inside eight stacked shells even with every
// error of one sign, against the 1e-4 bar.  Degree 7 (2.2e-7) cost one more FMA per ATAN2.
__device__ __forceinline__ float atan_unit(float t) {
    const float x = t * t;
    float p = 0.007863377f;
    p = __builtin_fmaf(p, x, -0.037013f);
    p = __builtin_fmaf(p, x, 0.08387119f);
    p = __builtin_fmaf(p, x, -0.13487191f);
    p = __builtin_fmaf(p, x, 0.19881482f);
    p = __builtin_fmaf(p, x, -0.33326516f);
    p = __builtin_fmaf(p, x, 0.99999934f);
    return p * t;
}

// |ATAN2(y, x)|: the angle of (|y|, x), in [0, pi].
__device__ __forceinline__ float atan2_mag(float y, float x) {
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float mn = __builtin_fminf(ax, ay);
    const float mx = __builtin_fmaxf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(__builtin_fmaxf(mx, kFltMin));
    float a = atan_unit(t);
    a = (ay > ax) ? (kHalfPi - a) : a;
    return (x < 0.0f) ? (kPi - a) : a;
}

// ATAN2(y, x) with the case table of Eq. 8: ATAN2(+-0, +-0) = 0 and, for x < 0,
// y = -0 takes the y >= 0 branch (+pi).  Finite inputs; NaN propagates.
__device__ __forceinline__ float atan2_eq8(float y, float x) {
    const float a = atan2_mag(y, x);
    return (y < 0.0f) ? -a : a;
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

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

// One vertex of the record window, per query point: R = v - q, r = |R|, and the dot
// product and length product with the previous record's vertex.
template <int PPL>
struct Slot {
    float x[PPL], y[PPL], z[PPL], r[PPL], dprev[PPL], rprev[PPL];
};

// Record v enters slot C (after B): R = v - q, r = |R|, and the dot and length products
// with B, per query point.
template <int PPL>
__device__ __forceinline__ void enter_vertex(const float4 v, const Slot<PPL> &B, Slot<PPL> &C, const float (&qx)[PPL],
                                             const float (&qy)[PPL], const float (&qz)[PPL]) {
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        C.x[p] = v.x - qx[p];
        C.y[p] = v.y - qy[p];
        C.z[p] = v.z - qz[p];
        C.r[p] = fast_sqrt(C.x[p] * C.x[p] + C.y[p] * C.y[p] + C.z[p] * C.z[p]);
        C.dprev[p] = B.x[p] * C.x[p] + B.y[p] * C.y[p] + B.z[p] * C.z[p];
        C.rprev[p] = B.r[p] * C.r[p];
    }
}

// Scale-free Eq. 7 terms of the face (A, B, C) with normal n: alpha' = R_A . N and
// beta' = r_A r_B r_C + (R_A.R_B) r_C + (R_B.R_C) r_A + (R_C.R_A) r_B; alpha' = 0 when a
// vertex coincides with the point.
template <int PPL>
__device__ __forceinline__ void face_terms(const float4 n, const Slot<PPL> &A, const Slot<PPL> &B, const Slot<PPL> &C,
                                           float (&al)[PPL], float (&be)[PPL]) {
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const float dca = C.x[p] * A.x[p] + C.y[p] * A.y[p] + C.z[p] * A.z[p];
        const float pr = B.rprev[p] * C.r[p];  // r_A r_B r_C
        be[p] = pr + B.dprev[p] * C.r[p] + C.dprev[p] * A.r[p] + dca * B.r[p];
        const float alpha = A.x[p] * n.x + A.y[p] * n.y + A.z[p] * n.z;
        al[p] = (pr == 0.0f) ? 0.0f : alpha;
    }
}

// Sum of two half solid angles from one ATAN2: the argument of the product
// (beta0 + i alpha0)(beta1 + i alpha1) is their sum up to a multiple of 2 pi.  The two
// angles lie in (-pi, pi]; their sum leaves that range exactly when both have the same
// sign and the product's imaginary part has the other sign, and then the principal
// value is off by 2 pi with the sign of the angles.  Eq. 8's zero cases (an angle of
// exactly 0 or pi, a face seen edge-on) and products outside the normal FP32 range take
// the two ATAN2s one by one.
__device__ __forceinline__ float pair_angle(float a0, float b0, float a1, float b1) {
    const float a01 = a0 * a1;
    const float pre = __builtin_fmaf(b0, b1, -a01);
    const float pim = a0 * b1 + b0 * a1;
    // Same sign: a01 > 0 (where it is not, |a01| < FLT_MIN or a zero angle, the two ATAN2s
    // are taken below).  A wrap has the angles' sign opposite to pim's, so the corrected
    // sum is the ATAN2's sign applied to (|angle| - 2 pi): one subtraction and one select,
    // with the same rounding as adding -+2 pi to the signed angle.
    const bool np = pim < 0.0f;
    float u = atan2_mag(pim, pre);
    if ((a01 > 0.0f) & ((a0 < 0.0f) != np)) u -= kTwoPi;
    float t = np ? -u : u;
    const float mx = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(pre), __builtin_fabsf(pim)), kFltMin);
    if (__builtin_expect(__builtin_fabsf(a01) < kFltMin || mx > kPairMax, 0))
        t = atan2_eq8(a0, b0) + atan2_eq8(a1, b1);
    return t;
}

// Record v enters slot C (after B, which follows A).  If it completes a face, that face
// is (A, B, C); its half solid angle at each point is added to ts.
template <int PPL>
__device__ __forceinline__ void push_record(const float4 v, const bool face, const float4 n, const Slot<PPL> &A,
                                            const Slot<PPL> &B, Slot<PPL> &C, const float (&qx)[PPL],
                                            const float (&qy)[PPL], const float (&qz)[PPL], float (&ts)[PPL]) {
    enter_vertex<PPL>(v, B, C, qx, qy, qz);
    if (face) {
        float al[PPL], be[PPL];
        face_terms<PPL>(n, A, B, C, al, be);
#pragma unroll
        for (int p = 0; p < PPL; ++p) ts[p] += atan2_eq8(al[p], be[p]);
    }
}

// Two consecutive records: x enters slot X2 (window X0, X1), then y enters X0 (window
// X1, X2).  Faces they complete are added to ts two at a time through pair_angle: both
// together, or a lone one with the lone face held over from an earlier pair (pa, pb;
// `pending` is wave-uniform, like the face bits).
template <int PPL>
__device__ __forceinline__ void push_pair(const float4 vx, const float4 nx, const float4 vy, const float4 ny,
                                          unsigned bits, Slot<PPL> &X0, Slot<PPL> &X1, Slot<PPL> &X2,
                                          const float (&qx)[PPL], const float (&qy)[PPL], const float (&qz)[PPL],
                                          float (&ts)[PPL], float (&pa)[PPL], float (&pb)[PPL], bool &pending) {
    float a0[PPL], b0[PPL], a1[PPL], b1[PPL];
    enter_vertex<PPL>(vx, X1, X2, qx, qy, qz);
    if (bits & 1u) face_terms<PPL>(nx, X0, X1, X2, a0, b0);
    enter_vertex<PPL>(vy, X2, X0, qx, qy, qz);
    if (bits & 2u) face_terms<PPL>(ny, X1, X2, X0, a1, b1);
    if ((bits & 3u) == 3u) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) ts[p] += pair_angle(a0[p], b0[p], a1[p], b1[p]);
    } else if (bits & 3u) {
        float a[PPL], b[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            a[p] = (bits & 1u) ? a0[p] : a1[p];
            b[p] = (bits & 1u) ? b0[p] : b1[p];
        }
        if (pending) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) ts[p] += pair_angle(pa[p], pb[p], a[p], b[p]);
            pending = false;
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                pa[p] = a[p];
                pb[p] = b[p];
            }
            pending = true;
        }
    }
}

// Face flags of a staged tile (record i's flag is bit i) as a wave-uniform mask, so the
// per-record branch costs no vector instruction.  Needs nt <= 64.
__device__ __forceinline__ unsigned long long tile_face_mask(const float4 *tile, int nt) {
    const int lane = threadIdx.x & 63;
    const float flag = lane < nt ? tile[2 * lane].w : 0.0f;
    return __builtin_amdgcn_ballot_w64(flag != 0.0f);
}

// Sum of the half solid angles of the faces completed by records [r0, r1), at PPL
// points per lane.  The two records before r0 (if any) prime the vertex window, so a
// range may start anywhere in the stream.  Records are staged through `tile` (LDS,
// 2 * kRecTile * DEPTH float4: DEPTH tiles per barrier) by the whole workgroup; each
// tile's per-point sum is folded into the Neumaier pair (s, c).  The result depends only
// on the record stream and the kRecTile boundaries, not on DEPTH.  The window's three
// slots rotate statically (records are taken six at a time; kRecTile is a multiple of
// six), so no register moves are needed.
template <int PPL, int DEPTH>
__device__ __forceinline__ void sum_records(const float4 *__restrict__ src, int64_t r0, int64_t r1, float4 *tile,
                                            const float (&qx)[PPL], const float (&qy)[PPL], const float (&qz)[PPL],
                                            float (&s)[PPL], float (&c)[PPL]) {
    if (r0 >= r1) return;  // empty range: nothing to prime or sum (uniform)
    const int tid = threadIdx.x;
    Slot<PPL> S0, S1, S2;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        S0.x[p] = S0.y[p] = S0.z[p] = S0.r[p] = S0.dprev[p] = S0.rprev[p] = 0.0f;
        S1.x[p] = S1.y[p] = S1.z[p] = S1.r[p] = S1.dprev[p] = S1.rprev[p] = 0.0f;
        S2.x[p] = S2.y[p] = S2.z[p] = S2.r[p] = S2.dprev[p] = S2.rprev[p] = 0.0f;
    }
    {
        float ts[PPL];
        const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (r0 >= 2) push_record<PPL>(src[2 * (r0 - 2)], false, zero, S2, S0, S1, qx, qy, qz, ts);
        if (r0 >= 1) push_record<PPL>(src[2 * (r0 - 1)], false, zero, S0, S1, S2, qx, qy, qz, ts);
    }
    // window now: A = S1, B = S2
    for (int64_t t0 = r0; t0 < r1; t0 += kRecTile * DEPTH) {
        const int nst = (int)min((int64_t)kRecTile * DEPTH, r1 - t0);
        __syncthreads();
        for (int x = tid; x < 2 * nst; x += kBlock) tile[x] = src[2 * t0 + x];
        __syncthreads();
#pragma unroll 1
        for (int sub = 0; sub < DEPTH && sub * kRecTile < nst; ++sub) {
        const float4 *tile_s = tile + 2 * sub * kRecTile;
        const int nt = min(kRecTile, nst - sub * kRecTile);
        const unsigned long long fmask = tile_face_mask(tile_s, nt);
        float ts[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) ts[p] = 0.0f;
        int i = 0;
        // six records per step: the window's slots return to their places after six
        float pa[PPL], pb[PPL];
        bool pending = false;
        for (; i + 6 <= nt; i += 6) {
            const float4 *g = tile_s + 2 * i;
            const unsigned bits = (unsigned)(fmask >> i);
            push_pair<PPL>(g[0], g[1], g[2], g[3], bits, S1, S2, S0, qx, qy, qz, ts, pa, pb, pending);
            push_pair<PPL>(g[4], g[5], g[6], g[7], bits >> 2, S0, S1, S2, qx, qy, qz, ts, pa, pb, pending);
            push_pair<PPL>(g[8], g[9], g[10], g[11], bits >> 4, S2, S0, S1, qx, qy, qz, ts, pa, pb, pending);
        }
        if (pending) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) ts[p] += atan2_eq8(pa[p], pb[p]);
        }
        // a partial step only occurs in the last tile of the range
        if (i < nt) {
            const float4 *g = tile_s + 2 * i;
            const unsigned bits = (unsigned)(fmask >> i);
            const int m = nt - i;
            push_record<PPL>(g[0], bits & 1u, g[1], S1, S2, S0, qx, qy, qz, ts);
            if (m > 1) push_record<PPL>(g[2], bits & 2u, g[3], S2, S0, S1, qx, qy, qz, ts);
            if (m > 2) push_record<PPL>(g[4], bits & 4u, g[5], S0, S1, S2, qx, qy, qz, ts);
            if (m > 3) push_record<PPL>(g[6], bits & 8u, g[7], S1, S2, S0, qx, qy, qz, ts);
            if (m > 4) push_record<PPL>(g[8], bits & 16u, g[9], S2, S0, S1, qx, qy, qz, ts);
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) neumaier_add(s[p], c[p], ts[p]);
        }
    }
}

// Vertex record r of the forward stream (see the header comment): vertex `vid` and,
// if fid >= 0, the normal of face fid in its own winding, computed in FP64.  Ids outside
// their ranges are replaced (vertex 0, "no face") and recorded in the workspace.
__device__ __forceinline__ VRec make_record(const float *__restrict__ V, int64_t nV, const int32_t *__restrict__ F,
                                            int64_t nF, int32_t vid, int32_t fid, WsHeader *hdr) {
    bool bad = false;
    if (vid < 0 || (int64_t)vid >= nV) {
        bad = true;
        vid = 0;
    }
    if (fid < -1 || (int64_t)fid >= nF) {
        bad = true;
        fid = -1;
    }
    VRec r;
    r.p = make_float4(V[3 * (int64_t)vid], V[3 * (int64_t)vid + 1], V[3 * (int64_t)vid + 2], fid >= 0 ? 1.0f : 0.0f);
    r.n = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (fid >= 0) {
        int32_t id[3];
        for (int j = 0; j < 3; ++j) {
            id[j] = F[3 * (int64_t)fid + j];
            if (id[j] < 0 || (int64_t)id[j] >= nV) {
                bad = true;
                id[j] = 0;
            }
        }
        double v[3][3];
        for (int j = 0; j < 3; ++j)
            for (int c = 0; c < 3; ++c) v[j][c] = V[3 * (int64_t)id[j] + c];
        const double e1x = v[1][0] - v[0][0], e1y = v[1][1] - v[0][1], e1z = v[1][2] - v[0][2];
        const double e2x = v[2][0] - v[0][0], e2y = v[2][1] - v[0][1], e2z = v[2][2] - v[0][2];
        r.n = make_float4((float)(e1y * e2z - e1z * e2y), (float)(e1z * e2x - e1x * e2z),
                          (float)(e1x * e2y - e1y * e2x), 0.0f);
    }
    if (bad) atomicOr(&hdr->bad_index, 1);
    return r;
}

// A strip record r whose face id fid is in range must complete F[fid]: the vertex ids of
// records r - 2, r - 1 and r are those of F[fid] in some order (a stale strip order or a
// hand-built stream that breaks this would give a silently wrong W).  Records 0 and 1
// have no such window.
__device__ __forceinline__ void sort3(int32_t &a, int32_t &b, int32_t &c) {
    int32_t t;
    if (a > b) t = a, a = b, b = t;
    if (b > c) t = b, b = c, c = t;
    if (a > b) t = a, a = b, b = t;
}

__device__ __forceinline__ bool strip_window_ok(const int32_t *__restrict__ R, int64_t r,
                                                const int32_t *__restrict__ F, int32_t fid) {
    if (r < 2) return false;
    int32_t a = R[2 * (r - 2)], b = R[2 * (r - 1)], c = R[2 * r];
    int32_t x = F[3 * (int64_t)fid], y = F[3 * (int64_t)fid + 1], z = F[3 * (int64_t)fid + 2];
    sort3(a, b, c);
    sort3(x, y, z);
    return a == x && b == y && c == z;
}

// Strip record r (vertex vid, face fid) checked against F before it is packed: a face
// whose window is not F[fid] is recorded as a bad index, and a face flag on record 0 or
// 1 is also dropped (its window would reach before the stream).
__device__ __forceinline__ void check_strip_record(const int32_t *__restrict__ R, int64_t r,
                                                   const int32_t *__restrict__ F, int64_t nF, int32_t &fid,
                                                   WsHeader *hdr) {
    if (fid < 0 || (int64_t)fid >= nF) return;  // no face, or out of range (make_record records it)
    if (!strip_window_ok(R, r, F, fid)) {
        atomicOr(&hdr->bad_index, 1);
        if (r < 2) fid = -1;
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
int fwd_split_count(int64_t nR, int64_t nQ);
int64_t fwd_split_chunk(int64_t nR, int split);

// Host triangle-strip builder (wn_strips.hip): records as int32 pairs.
int64_t build_strips(const int32_t *F, int64_t nF, std::vector<int32_t> &out);
// Host face pairing for the adjoint (wn_strips.hip): int32 pairs (f, g or -1).
int64_t build_face_pairs(const int32_t *F, int64_t nF, std::vector<int32_t> &out);

PointSrc make_point_src(const wn_grid *grid, const float *Q);

// Forward pieces (wn_fwd.hip).
hipError_t launch_ws_reset(WsHeader *hdr, hipStream_t s);
hipError_t launch_pack(const float *V, int64_t nV, const int32_t *F, int64_t nF, FaceRec *soup,
                       WsHeader *hdr, hipStream_t s);
// Vertex records from (V, F) and an optional strip stream R ([nR][2] = vertex, face or
// -1); with R == nullptr the stream is three records per face (nR = 3 nF).
hipError_t launch_pack_records(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *R,
                               int64_t nR, VRec *recs, WsHeader *hdr, hipStream_t s);
hipError_t launch_fwd(const VRec *recs, int64_t nR, const PointSrc &ps, int64_t nQ, int split,
                      float *W, float *partials, const OccParams &occ, int ppl, int depth, hipStream_t s);
// Order-free checksum (sum of the bit patterns) of n floats into hdr->checksum.
hipError_t launch_checksum(const float *x, int64_t n, WsHeader *hdr, bool reset, hipStream_t s);
hipError_t launch_occ(const float *W, int64_t n, const OccParams &occ, hipStream_t s);
hipError_t launch_occ_bwd(const float *W, const float *g, int64_t n, float tau, float k, float *dLdW,
                          hipStream_t s);
// Fixed-order sum of [split][nQ] partials times `scale` into W, plus occupancy.
hipError_t launch_split_reduce(const float *partials, int split, int64_t nQ, float scale, float *W,
                               const OccParams &occ, hipStream_t s);
hipError_t launch_sigmoid_mse(const float *W, const float *target, int64_t n, float tau, float k,
                              float *loss, float *dLdW, float *scratch, hipStream_t s);
int loss_blocks(int64_t n);

// Backward pieces (wn_bwd.hip).  `naive` selects the adjoint of the Eq. 4 sum instead of
// the exact solid-angle field.  The points' 256-point tiles are dealt to S = bwd_splits
// splits in turn (tile t to split t mod S); each split keeps compensated running sums
// per corner in the workspace, and the splits are added in split order at the end.  A
// call sequence BEGIN, consecutive point ranges of whole tiles in increasing order, END
// therefore gives the same bits as one call over all points.
// Two faces per lane (wn_bwd_pairs.hip): 80-byte pair records and 16-byte pair metadata
// in the adjoint's workspace; pack (with the every-face-once check), the point-split
// kernel over tiles [t0, t1), and the reduction of the 18 running sums per pair into T.
// `merged`: the two faces share their sums at the shared edge's vertices (12 per pair),
// which keeps the sums per vertex exact but not those per corner (dL/dV only).
constexpr size_t kPairRecBytes = 80, kPairMetaBytes = 16;
hipError_t launch_pack_pairs(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *pairs, int64_t nP,
                             char *recs, char *meta, int32_t *counts, WsHeader *hdr, hipStream_t s);
hipError_t launch_bwd_pairs(const char *recs, const char *meta, int32_t nP, int32_t nF, const PointSrc &ps, int64_t nQ,
                            int32_t S, int64_t t0, int64_t t1, int32_t rows, const float *dLdW, float2 *state,
                            bool merged, hipStream_t s);
hipError_t launch_reduce_pairs(const float2 *state, int32_t S, int32_t nP, const char *meta, float scale, float *T,
                               bool merged, hipStream_t s);
constexpr int kBwdBegin = 1, kBwdEnd = 2, kBwdVertexSums = 4;
// Loads in flight per thread in the reductions over the splits (each thread's loop over
// several hundred splits is bound by memory latency, not bandwidth).
constexpr int kReduceBatch = 32;
constexpr int kBwdTile = 256;
int bwd_splits(int64_t nF, int64_t nQ);
size_t bwd_workspace(int64_t nV, int64_t nF, int64_t nQ);
// `pairs` (device int32 [nP][2], optional): faces two per lane, each pair sharing an
// edge (wn_build_face_pairs); the exact adjoint only.
wn_status run_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *pairs, int64_t nP,
                       const PointSrc &ps, int64_t nQ, const float *dLdW, int64_t p0, int64_t n, int flags,
                       float *dLdV, float *dLdT, char *ws, size_t ws_bytes, hipStream_t s, bool naive = false);
inline wn_status run_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF, const PointSrc &ps,
                              int64_t nQ, const float *dLdW, float *dLdV, float *dLdT, char *ws, size_t ws_bytes,
                              hipStream_t s, bool naive = false) {
    return run_backward(V, nV, F, nF, nullptr, 0, ps, nQ, dLdW, 0, nQ, kBwdBegin | kBwdEnd, dLdV, dLdT, ws,
                        ws_bytes, s, naive);
}

// A split's running sums of face f: (sum, compensation) of its 9 corner components at
// state[(split * 9 + i) * nF + f] (coalesced over faces).  A split that starts here
// begins at zero.
__device__ __forceinline__ void load_state(const float2 *__restrict__ state, int64_t split, int32_t nF, int32_t f,
                                           bool fresh, float (&s)[9], float (&c)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float2 x = fresh ? make_float2(0.0f, 0.0f) : state[(split * 9 + i) * nF + f];
        s[i] = x.x;
        c[i] = x.y;
    }
}

__device__ __forceinline__ void store_state(float2 *__restrict__ state, int64_t split, int32_t nF, int32_t f,
                                            const float (&s)[9], const float (&c)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) state[(split * 9 + i) * nF + f] = make_float2(s[i], c[i]);
}

// Naive flux integral of Eq. 4 (wn_naive.hip).
constexpr float kInv8Pi = 0.0397887357729738340f;
hipError_t launch_naive_fwd(const float *V, int64_t nV, const int32_t *F, int64_t nF, const PointSrc &ps,
                            int64_t nQ, float *W, const OccParams &occ, char *ws, int ppl, hipStream_t s);
size_t naive_fwd_workspace(int64_t nF, int64_t nQ);
// Evaluation chain (wn_eval.hip): cube surface of an occupancy grid, Laplacian
// smoothing, area-uniform surface samples, nearest-neighbour distances and metrics.
size_t cubify_workspace(int64_t P, int64_t C);
size_t smooth_workspace(int64_t nV, int64_t nF);
size_t sample_workspace(int64_t nF);
size_t nn_workspace(int64_t nA, int64_t nB);
wn_status run_cubify(const uint8_t *occ, const int32_t n[3], const float lo[3], const float hi[3], float *V,
                     int64_t capV, int32_t *F, int64_t capF, int64_t *counts, char *ws, hipStream_t s);
wn_status run_smooth(const float *V, int64_t nV, const int32_t *F, int64_t nF, float lam, int32_t iters,
                     int32_t keep_volume, float *Vout, char *ws, hipStream_t s);
wn_status run_sample(const float *V, int64_t nV, const int32_t *F, int64_t nF, const double *u, int64_t n, float *P,
                     int32_t *face, char *ws, hipStream_t s);
wn_status run_nn(const float *A, int64_t nA, const float *B, int64_t nB, float *d, char *ws, hipStream_t s);
wn_status run_chamfer(const float *A, int64_t nA, const float *B, int64_t nB, double *out, char *ws, hipStream_t s);

// Adam over a flat parameter array (wn_morph.hip); t >= 1 is the step number.
hipError_t launch_adam(float *x, const float *g, float *m, float *v, int64_t n, int64_t t, float lr, float b1,
                       float b2, float eps, hipStream_t s);
// The adjoint pair kernel of Eq. 4 (defined in wn_naive.hip, launched by run_backward)
// over the tiles [t0, t1) with S splits, `rows` = min(S, t1 - t0).
hipError_t launch_naive_bwd(const FaceRec *soup, int32_t nF, const PointSrc &ps, int64_t nQ, int32_t S, int64_t t0,
                            int64_t t1, int32_t rows, const float *dLdW, float2 *state, hipStream_t s);

// Flipping duplication (wn_bwd.hip).
size_t flip_workspace(int64_t nV, int64_t nF);
wn_status run_flip(const float *V, int64_t nV, const int32_t *F, int64_t nF, float eps, float *V2, int32_t *F2,
                   char *ws, size_t ws_bytes, hipStream_t s);

// The forward entry point's checks and launch sequence (wn_api.hip): R == nullptr for
// three records per face; `force` overrides the tuned launch configuration.  The
// workspace of a stream of nR records over nQ points is voxelize_workspace(nR, nQ).
struct TuneConfig;
wn_status voxelize_impl(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *R, int64_t nR,
                        const wn_grid *grid, const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau,
                        float k, void *occ, void *ws, size_t ws_bytes, void *stream, const TuneConfig *force);
size_t voxelize_workspace(int64_t nR, int64_t nQ);
// Device address of the allocation-free entry point's scratch array on the current
// device (wn_noalloc.hip); its header carries that entry point's device error record.
wn_status noalloc_header(void **out);

// Batched pieces (wn_batched.hip).
size_t batched_workspace(const wn_mesh_desc *d, int32_t n);
// Frees what the library holds for a workspace (captured graphs, pinned staging).
wn_status release_batched(const void *ws);
wn_status run_batched(const wn_mesh_desc *d, int32_t n, int32_t flags, char *ws, size_t ws_bytes,
                      hipStream_t s, const struct TuneConfig *force);

// Launch tuning (wn_tune.hip).  A configuration changes only how work is mapped to
// lanes and workgroups, never the per-point summation order, so results do not
// depend on it.
struct TuneConfig {
    int32_t ppl;        // query points per lane: 1, 2 or 4
    int32_t wg_per_cu;  // persistent workgroups per CU (0 = as many as fit)
    int32_t depth;      // record tiles staged in LDS per barrier: 1, 2 or 4
};
TuneConfig default_config(int32_t op);
TuneConfig lookup_config(int32_t op, int64_t a, int64_t b);
void store_config(int32_t op, int64_t a, int64_t b, const TuneConfig &c);
bool valid_ppl(int32_t ppl);
bool valid_depth(int32_t depth);

// Calls f(PPL, DEPTH) with the configuration as compile-time constants
// (std::integral_constant); an invalid pair returns hipErrorInvalidValue.
template <typename Fn>
hipError_t with_config(int32_t ppl, int32_t depth, Fn &&f) {
    using std::integral_constant;
    switch (ppl * 10 + depth) {
        case 11: return f(integral_constant<int, 1>{}, integral_constant<int, 1>{});
        case 12: return f(integral_constant<int, 1>{}, integral_constant<int, 2>{});
        case 14: return f(integral_constant<int, 1>{}, integral_constant<int, 4>{});
        case 21: return f(integral_constant<int, 2>{}, integral_constant<int, 1>{});
        case 22: return f(integral_constant<int, 2>{}, integral_constant<int, 2>{});
        case 24: return f(integral_constant<int, 2>{}, integral_constant<int, 4>{});
        case 41: return f(integral_constant<int, 4>{}, integral_constant<int, 1>{});
        case 42: return f(integral_constant<int, 4>{}, integral_constant<int, 2>{});
        case 44: return f(integral_constant<int, 4>{}, integral_constant<int, 4>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wn
