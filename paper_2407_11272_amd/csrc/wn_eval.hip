// Evaluation chain of the paper's experiments (Section 3): an occupancy grid becomes a
// cube surface ("cubified"), which is smoothed by Laplacian filtering (10 iterations,
// lambda = 0.15 in the paper) and compared with the original mesh through surface
// samples (20 000 in the paper) by Chamfer and Hausdorff distances.
//
// All of it is memory- or latency-bound bookkeeping except the nearest-neighbour
// search, which is an all-pairs FP32 minimum (like the forward, ALU-bound and tiled
// through LDS).  Every result is deterministic:
//   * cube surface: counts per voxel and used lattice corners, two exclusive scans,
//     then each voxel writes its own faces at its scanned offset;
//   * smoothing: neighbour lists from a radix sort of the directed edges, then Jacobi
//     steps that add each vertex's neighbours in increasing id order, each optionally
//     followed by a scaling about the origin back to the starting enclosed volume (FP64
//     volume summed in a fixed order);
//   * sampling: integer area weights and an integer prefix sum, so the face choice is
//     exact; the areas are formed in FP64 without contraction;
//   * nearest neighbours: squared distances are non-negative floats, whose bit patterns
//     order like the values, so an integer atomic minimum gives the exact minimum.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "wn_internal.hpp"

namespace wn {

namespace {

unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_copy_f32(const float *__restrict__ a, float *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------------ cube surface

// Voxel faces in the order -x, +x, -y, +y, -z, +z: the axis, the side (0: the lower
// lattice plane of the voxel, 1: the upper), and in-plane axes (u, w) with u x w = +axis.
// A face's corners walk (0,0), (1,0), (1,1), (0,1) in (u, w).  Triangles (p0,p1,p2),
// (p0,p2,p3) face +axis; on the lower side they are reversed to face -axis.
__constant__ int8_t c_dir[6][4] = {{0, 0, 1, 2}, {0, 1, 1, 2}, {1, 0, 2, 0}, {1, 1, 2, 0}, {2, 0, 0, 1}, {2, 1, 0, 1}};

struct Lattice {
    int32_t n[3];
    __device__ int64_t corner(const int32_t (&c)[3]) const {
        return ((int64_t)c[0] * (n[1] + 1) + c[1]) * (int64_t)(n[2] + 1) + c[2];
    }
    __device__ void voxel(int64_t v, int32_t (&ijk)[3]) const {
        ijk[2] = (int32_t)(v % n[2]);
        const int64_t r = v / n[2];
        ijk[1] = (int32_t)(r % n[1]);
        ijk[0] = (int32_t)(r / n[1]);
    }
};

__device__ __forceinline__ int32_t boundary_mask(const uint8_t *__restrict__ occ, const Lattice &L, int64_t v) {
    if (!occ[v]) return 0;
    int32_t ijk[3];
    L.voxel(v, ijk);
    const int64_t stride[3] = {(int64_t)L.n[1] * L.n[2], (int64_t)L.n[2], 1};
    int32_t m = 0;
    for (int d = 0; d < 6; ++d) {
        const int a = c_dir[d][0];
        const bool up = c_dir[d][1] != 0;
        const bool inside = up ? ijk[a] + 1 < L.n[a] : ijk[a] > 0;
        if (!inside || !occ[v + (up ? stride[a] : -stride[a])]) m |= 1 << d;
    }
    return m;
}

// The 4 lattice corners of face d of voxel ijk, in walk order.
__device__ __forceinline__ void face_corners(const Lattice &L, const int32_t (&ijk)[3], int d, int64_t (&c)[4]) {
    const int a = c_dir[d][0], side = c_dir[d][1], u = c_dir[d][2], w = c_dir[d][3];
    const int du[4] = {0, 1, 1, 0}, dw[4] = {0, 0, 1, 1};
    for (int q = 0; q < 4; ++q) {
        int32_t p[3] = {ijk[0], ijk[1], ijk[2]};
        p[a] += side;
        p[u] += du[q];
        p[w] += dw[q];
        c[q] = L.corner(p);
    }
}

__global__ __launch_bounds__(kBlock) void k_cub_count(const uint8_t *__restrict__ occ, Lattice L, int64_t P,
                                                      int32_t *__restrict__ qcount, int32_t *__restrict__ used) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= P) return;
    const int32_t m = boundary_mask(occ, L, v);
    qcount[v] = __builtin_popcount(m);
    if (!m) return;
    int32_t ijk[3];
    L.voxel(v, ijk);
    for (int d = 0; d < 6; ++d) {
        if (!(m >> d & 1)) continue;
        int64_t c[4];
        face_corners(L, ijk, d, c);
        for (int q = 0; q < 4; ++q) used[c[q]] = 1;  // every writer stores the same value
    }
}

__global__ __launch_bounds__(kBlock) void k_cub_counts(const int32_t *__restrict__ qcount,
                                                       const int64_t *__restrict__ qoff, int64_t P,
                                                       const int32_t *__restrict__ used,
                                                       const int64_t *__restrict__ vid, int64_t C,
                                                       int64_t *__restrict__ counts) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    counts[0] = C > 0 ? vid[C - 1] + used[C - 1] : 0;
    counts[1] = P > 0 ? 2 * (qoff[P - 1] + qcount[P - 1]) : 0;
}

__global__ __launch_bounds__(kBlock) void k_cub_faces(const uint8_t *__restrict__ occ, Lattice L, int64_t P,
                                                      const int64_t *__restrict__ qoff,
                                                      const int64_t *__restrict__ vid, int32_t *__restrict__ F,
                                                      int64_t capF) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= P) return;
    const int32_t m = boundary_mask(occ, L, v);
    if (!m) return;
    int32_t ijk[3];
    L.voxel(v, ijk);
    int64_t t = 2 * qoff[v];
    for (int d = 0; d < 6; ++d) {
        if (!(m >> d & 1)) continue;
        int64_t c[4];
        face_corners(L, ijk, d, c);
        const int32_t p0 = (int32_t)vid[c[0]], p1 = (int32_t)vid[c[1]], p2 = (int32_t)vid[c[2]],
                      p3 = (int32_t)vid[c[3]];
        int32_t tri[2][3];
        if (c_dir[d][1]) {
            tri[0][0] = p0, tri[0][1] = p1, tri[0][2] = p2;
            tri[1][0] = p0, tri[1][1] = p2, tri[1][2] = p3;
        } else {
            tri[0][0] = p0, tri[0][1] = p2, tri[0][2] = p1;
            tri[1][0] = p0, tri[1][1] = p3, tri[1][2] = p2;
        }
        for (int h = 0; h < 2; ++h, ++t)
            if (t < capF)
                for (int j = 0; j < 3; ++j) F[3 * t + j] = tri[h][j];
    }
}

__global__ __launch_bounds__(kBlock) void k_cub_verts(const int32_t *__restrict__ used,
                                                      const int64_t *__restrict__ vid, Lattice L, int64_t C,
                                                      float3 lo, float3 h, float *__restrict__ V, int64_t capV) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || !used[c]) return;
    const int64_t id = vid[c];
    if (id >= capV) return;
    const int64_t k = c % (L.n[2] + 1);
    const int64_t r = c / (L.n[2] + 1);
    const int64_t j = r % (L.n[1] + 1);
    const int64_t i = r / (L.n[1] + 1);
    V[3 * id] = __builtin_fmaf((float)i, h.x, lo.x);
    V[3 * id + 1] = __builtin_fmaf((float)j, h.y, lo.y);
    V[3 * id + 2] = __builtin_fmaf((float)k, h.z, lo.z);
}

struct CubPlan {
    size_t tmp, off_qcount, off_qoff, off_used, off_vid, off_tmp, total;
};

CubPlan plan_cubify(int64_t P, int64_t C) {
    CubPlan p{};
    size_t t1 = 0, t2 = 0;
    if (P > 0)
        (void)rocprim::exclusive_scan(nullptr, t1, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                      (size_t)P, rocprim::plus<int64_t>());
    if (C > 0)
        (void)rocprim::exclusive_scan(nullptr, t2, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                      (size_t)C, rocprim::plus<int64_t>());
    p.tmp = t1 > t2 ? t1 : t2;
    size_t o = kWsHeader;
    p.off_qcount = o;
    o += align_up((size_t)P * 4);
    p.off_qoff = o;
    o += align_up((size_t)P * 8);
    p.off_used = o;
    o += align_up((size_t)C * 4);
    p.off_vid = o;
    o += align_up((size_t)C * 8);
    p.off_tmp = o;
    o += align_up(p.tmp > 0 ? p.tmp : 1);
    p.total = o;
    return p;
}

// ------------------------------------------------------------------ smoothing

__global__ __launch_bounds__(kBlock) void k_edge_keys(const int32_t *__restrict__ F, int64_t nF, int64_t nV,
                                                      uint64_t *__restrict__ keys, WsHeader *hdr) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    int32_t v[3];
    bool bad = false;
    for (int j = 0; j < 3; ++j) {
        v[j] = F[3 * f + j];
        if (v[j] < 0 || (int64_t)v[j] >= nV) {
            v[j] = 0;
            bad = true;
        }
    }
    if (bad) hdr->bad_index = 1;
    for (int j = 0; j < 3; ++j) {
        const uint32_t a = (uint32_t)v[j], b = (uint32_t)v[(j + 1) % 3];
        keys[6 * f + 2 * j] = (uint64_t)a << 32 | b;
        keys[6 * f + 2 * j + 1] = (uint64_t)b << 32 | a;
    }
}

// 1 where a sorted key starts a run and is not a self-loop; the source's degree counted.
__global__ __launch_bounds__(kBlock) void k_edge_unique(const uint64_t *__restrict__ keys, int64_t n,
                                                        int32_t *__restrict__ flag, int32_t *__restrict__ deg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    const bool keep = (i == 0 || keys[i - 1] != k) && (uint32_t)(k >> 32) != (uint32_t)k;
    flag[i] = keep ? 1 : 0;
    if (keep) atomicAdd(&deg[(uint32_t)(k >> 32)], 1);  // integer counts: order-free
}

__global__ __launch_bounds__(kBlock) void k_edge_compact(const uint64_t *__restrict__ keys, int64_t n,
                                                         const int32_t *__restrict__ flag,
                                                         const int64_t *__restrict__ pos, int32_t *__restrict__ nbr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) nbr[pos[i]] = (int32_t)(uint32_t)keys[i];
}

__global__ __launch_bounds__(kBlock) void k_smooth_step(const float *__restrict__ X, float *__restrict__ Y, int64_t nV,
                                                        const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ nbr, float lam) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const int64_t b = off[v], e = off[v + 1];
    const float x = X[3 * v], y = X[3 * v + 1], z = X[3 * v + 2];
    if (e == b) {
        Y[3 * v] = x, Y[3 * v + 1] = y, Y[3 * v + 2] = z;
        return;
    }
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int64_t i = b; i < e; ++i) {
        const int64_t u = nbr[i];
        sx += X[3 * u];
        sy += X[3 * u + 1];
        sz += X[3 * u + 2];
    }
    const float inv = 1.0f / (float)(e - b);
    Y[3 * v] = x + lam * (sx * inv - x);
    Y[3 * v + 1] = y + lam * (sy * inv - y);
    Y[3 * v + 2] = z + lam * (sz * inv - z);
}

// Enclosed volume of the surface (v0 . (v1 x v2) / 6 summed over faces, the divergence
// theorem), in FP64 and in a fixed order: kVolBlocks workgroups each sum a fixed strided
// set of faces per thread, then a fixed-shape tree; one workgroup adds the partials.
constexpr int kVolBlocks = 256;

__device__ __forceinline__ double block_sum_f64(double x) {
    __shared__ double red[kBlock];
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(kBlock) void k_volume_partial(const float *__restrict__ X, int64_t nV,
                                                           const int32_t *__restrict__ F, int64_t nF,
                                                           double *__restrict__ part) {
    double acc = 0.0;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nF; f += (int64_t)gridDim.x * blockDim.x) {
        double v[3][3];
        for (int j = 0; j < 3; ++j) {
            int64_t id = F[3 * f + j];
            id = (id < 0 || id >= nV) ? 0 : id;  // recorded by the edge pass
            for (int c = 0; c < 3; ++c) v[j][c] = X[3 * id + c];
        }
        const double cx = v[1][1] * v[2][2] - v[1][2] * v[2][1];
        const double cy = v[1][2] * v[2][0] - v[1][0] * v[2][2];
        const double cz = v[1][0] * v[2][1] - v[1][1] * v[2][0];
        acc += v[0][0] * cx + v[0][1] * cy + v[0][2] * cz;
    }
    const double t = block_sum_f64(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// vol[0] = the volume (first call), or scale[0] = cbrt(vol0 / vol) when that ratio is
// positive and finite, else 1 (a surface that encloses no volume is not rescaled).
__global__ __launch_bounds__(kBlock) void k_volume_final(const double *__restrict__ part, double *__restrict__ vol0,
                                                         double *__restrict__ scale, int first) {
    const double t = block_sum_f64(threadIdx.x < kVolBlocks ? part[threadIdx.x] : 0.0) / 6.0;
    if (threadIdx.x != 0) return;
    if (first) {
        vol0[0] = t;
    } else {
        const double r = t != 0.0 ? vol0[0] / t : 0.0;
        scale[0] = (r > 0.0 && r <= 1.79e308) ? cbrt(r) : 1.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_scale_f32(float *__restrict__ X, int64_t n,
                                                      const double *__restrict__ scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) X[i] = (float)((double)X[i] * scale[0]);
}
static_assert(kVolBlocks <= kBlock, "one thread per volume partial in the final sum");

struct SmoothPlan {
    unsigned bits;
    size_t sort_tmp, scan_tmp, scan2_tmp;
    size_t off_keys, off_keys2, off_flag, off_pos, off_nbr, off_deg, off_off, off_tmp, off_T, off_vol, total;
};

SmoothPlan plan_smooth(int64_t nV, int64_t nF) {
    SmoothPlan p{};
    const int64_t nE = 6 * nF;
    unsigned vb = 1;
    while (vb < 32 && ((int64_t)1 << vb) < nV) ++vb;
    p.bits = 32 + vb;
    if (nE > 0) {
        (void)rocprim::radix_sort_keys(nullptr, p.sort_tmp, (uint64_t *)nullptr, (uint64_t *)nullptr, (size_t)nE, 0u,
                                       p.bits);
        (void)rocprim::exclusive_scan(nullptr, p.scan_tmp, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                      (size_t)nE, rocprim::plus<int64_t>());
    }
    (void)rocprim::exclusive_scan(nullptr, p.scan2_tmp, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                  (size_t)(nV + 1), rocprim::plus<int64_t>());
    size_t tmp = p.sort_tmp;
    if (p.scan_tmp > tmp) tmp = p.scan_tmp;
    if (p.scan2_tmp > tmp) tmp = p.scan2_tmp;
    size_t o = kWsHeader;
    p.off_keys = o;
    o += align_up((size_t)nE * 8);
    p.off_keys2 = o;
    o += align_up((size_t)nE * 8);
    p.off_flag = o;
    o += align_up((size_t)nE * 4);
    p.off_pos = o;
    o += align_up((size_t)nE * 8);
    p.off_nbr = o;
    o += align_up((size_t)nE * 4);
    p.off_deg = o;
    o += align_up((size_t)(nV + 1) * 4);
    p.off_off = o;
    o += align_up((size_t)(nV + 1) * 8);
    p.off_tmp = o;
    o += align_up(tmp > 0 ? tmp : 1);
    p.off_T = o;
    o += align_up((size_t)nV * 12);
    p.off_vol = o;  // kVolBlocks partials, then vol0 and the scale
    o += align_up((size_t)(kVolBlocks + 2) * 8);
    p.total = o;
    return p;
}

// ------------------------------------------------------------------ sampling

// Triangle area in FP64 from FP32 coordinates, with every product rounded on its own
// (no contraction), so that any IEEE FP64 implementation gives the same bits.
__device__ double face_area64(const float *__restrict__ V, int64_t nV, const int32_t *__restrict__ F, int64_t f,
                              bool &bad) {
#pragma clang fp contract(off)
    int32_t id[3];
    for (int j = 0; j < 3; ++j) {
        id[j] = F[3 * f + j];
        if (id[j] < 0 || (int64_t)id[j] >= nV) {
            id[j] = 0;
            bad = true;
        }
    }
    double a[3], e1[3], e2[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = (double)V[3 * (int64_t)id[0] + c];
        e1[c] = (double)V[3 * (int64_t)id[1] + c] - a[c];
        e2[c] = (double)V[3 * (int64_t)id[2] + c] - a[c];
    }
    const double cx = e1[1] * e2[2] - e1[2] * e2[1];
    const double cy = e1[2] * e2[0] - e1[0] * e2[2];
    const double cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double s = (cx * cx + cy * cy) + cz * cz;
    return 0.5 * __builtin_sqrt(s);
}

__global__ __launch_bounds__(kBlock) void k_area(const float *__restrict__ V, int64_t nV, const int32_t *__restrict__ F,
                                                 int64_t nF, double *__restrict__ area,
                                                 unsigned long long *__restrict__ amax_bits, WsHeader *hdr) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    bool bad = false;
    const double a = face_area64(V, nV, F, f, bad);
    if (bad) hdr->bad_index = 1;
    area[f] = a;
    // non-negative doubles order like their bit patterns
    atomicMax(amax_bits, (unsigned long long)__double_as_longlong(a));
}

__global__ __launch_bounds__(kBlock) void k_area_weights(const double *__restrict__ area, int64_t nF,
                                                         const unsigned long long *__restrict__ amax_bits,
                                                         uint64_t *__restrict__ w) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    const double amax = __longlong_as_double((long long)*amax_bits);
    w[f] = amax > 0.0 ? (uint64_t)__builtin_floor(area[f] * (4294967296.0 / amax)) : 0;
}

__global__ __launch_bounds__(kBlock) void k_sample(const float *__restrict__ V, const int32_t *__restrict__ F,
                                                   int64_t nV, int64_t nF, const uint64_t *__restrict__ cdf,
                                                   const double *__restrict__ u, int64_t n, float *__restrict__ P,
                                                   int32_t *__restrict__ face) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t total = cdf[nF - 1];
    if (total == 0) {  // every face has zero area
        face[s] = -1;
        P[3 * s] = P[3 * s + 1] = P[3 * s + 2] = 0.0f;
        return;
    }
    const double tf = __builtin_floor(u[3 * s] * (double)total);
    const double last = (double)(total - 1);
    const uint64_t t = (uint64_t)(tf < last ? tf : last);
    // first face whose inclusive prefix exceeds t
    int64_t lo = 0, hi = nF - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    double r1 = u[3 * s + 1], r2 = u[3 * s + 2];
    if (r1 + r2 > 1.0) {
        r1 = 1.0 - r1;
        r2 = 1.0 - r2;
    }
    int32_t id[3];
    for (int j = 0; j < 3; ++j) {
        id[j] = F[3 * lo + j];
        if (id[j] < 0 || (int64_t)id[j] >= nV) id[j] = 0;
    }
    const float b1 = (float)r1, b2 = (float)r2;
    for (int c = 0; c < 3; ++c) {
        const float a = V[3 * (int64_t)id[0] + c];
        const float e1 = V[3 * (int64_t)id[1] + c] - a, e2 = V[3 * (int64_t)id[2] + c] - a;
        P[3 * s + c] = __builtin_fmaf(b2, e2, __builtin_fmaf(b1, e1, a));
    }
    face[s] = (int32_t)lo;
}

struct SamplePlan {
    size_t scan_tmp, off_area, off_w, off_cdf, off_max, off_tmp, total;
};

SamplePlan plan_sample(int64_t nF) {
    SamplePlan p{};
    if (nF > 0)
        (void)rocprim::inclusive_scan(nullptr, p.scan_tmp, (const uint64_t *)nullptr, (uint64_t *)nullptr, (size_t)nF,
                                      rocprim::plus<uint64_t>());
    size_t o = kWsHeader;
    p.off_area = o;
    o += align_up((size_t)nF * 8);
    p.off_w = o;
    o += align_up((size_t)nF * 8);
    p.off_cdf = o;
    o += align_up((size_t)nF * 8);
    p.off_max = o;
    o += 256;
    p.off_tmp = o;
    o += align_up(p.scan_tmp > 0 ? p.scan_tmp : 1);
    p.total = o;
    return p;
}

// ------------------------------------------------------------------ nearest neighbours

constexpr int kNNTile = 256;  // points of B staged per LDS tile

// best[i] = min over the B points of this block's chunk of |A_i - B_j|^2 (as bits).
__global__ __launch_bounds__(kBlock) void k_nn(const float *__restrict__ A, int64_t nA, const float *__restrict__ B,
                                               int64_t nB, int64_t chunk, uint32_t *__restrict__ best) {
    __shared__ float tile[3 * kNNTile];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < nB ? j0 + chunk : nB;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    if (i < nA) ax = A[3 * i], ay = A[3 * i + 1], az = A[3 * i + 2];
    float m = __builtin_inff();
    for (int64_t t0 = j0; t0 < j1; t0 += kNNTile) {
        const int nt = (int)(j1 - t0 < kNNTile ? j1 - t0 : kNNTile);
        __syncthreads();
        for (int x = threadIdx.x; x < 3 * nt; x += blockDim.x) tile[x] = B[3 * t0 + x];
        __syncthreads();
        for (int j = 0; j < nt; ++j) {
            const float dx = ax - tile[3 * j], dy = ay - tile[3 * j + 1], dz = az - tile[3 * j + 2];
            m = __builtin_fminf(m, __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
        }
    }
    if (i < nA) atomicMin(&best[i], __float_as_uint(m));
}

__global__ __launch_bounds__(kBlock) void k_nn_sqrt(const uint32_t *__restrict__ best, int64_t n,
                                                    float *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = __builtin_sqrtf(__uint_as_float(best[i]));
}

constexpr int kRedBlocks = 256;

// Per-block FP64 sums and FP32 maxima of d[0..n) in a fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_max(const float *__restrict__ d, int64_t n, double *__restrict__ psum,
                                                    float *__restrict__ pmax) {
    __shared__ double ss[kBlock];
    __shared__ float sm[kBlock];
    double s = 0.0;
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        s += (double)d[i];
        m = __builtin_fmaxf(m, d[i]);
    }
    ss[threadIdx.x] = s;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sm[threadIdx.x] = __builtin_fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) psum[blockIdx.x] = ss[0], pmax[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kBlock) void k_metrics(const double *__restrict__ psum, const float *__restrict__ pmax,
                                                    int64_t nA, int64_t nB, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sa = 0.0, sb = 0.0;
    float ma = 0.0f, mb = 0.0f;
    for (int b = 0; b < kRedBlocks; ++b) {
        sa += psum[b], ma = __builtin_fmaxf(ma, pmax[b]);
        sb += psum[kRedBlocks + b], mb = __builtin_fmaxf(mb, pmax[kRedBlocks + b]);
    }
    out[0] = sa / (double)nA + sb / (double)nB;
    out[1] = (double)__builtin_fmaxf(ma, mb);
}

struct NNPlan {
    size_t off_best, off_dA, off_dB, off_psum, off_pmax, total;
};

NNPlan plan_nn(int64_t nA, int64_t nB) {
    NNPlan p{};
    const int64_t nmax = nA > nB ? nA : nB;
    size_t o = kWsHeader;
    p.off_best = o;
    o += align_up((size_t)nmax * 4);
    p.off_dA = o;
    o += align_up((size_t)nA * 4);
    p.off_dB = o;
    o += align_up((size_t)nB * 4);
    p.off_psum = o;
    o += align_up(2 * kRedBlocks * 8);
    p.off_pmax = o;
    o += align_up(2 * kRedBlocks * 4);
    p.total = o;
    return p;
}

// Splits of B so that about 8192 wave64s run.
int64_t nn_chunk(int64_t nA, int64_t nB) {
    const int64_t waves = (nA + 63) / 64;
    int64_t split = (8192 + waves - 1) / (waves > 0 ? waves : 1);
    const int64_t max_split = (nB + kNNTile - 1) / kNNTile;
    if (split > max_split) split = max_split;
    if (split < 1) split = 1;
    int64_t chunk = (nB + split - 1) / split;
    return chunk > 0 ? chunk : 1;
}

hipError_t launch_nn(const float *A, int64_t nA, const float *B, int64_t nB, uint32_t *best, float *d, hipStream_t s) {
    if (nA == 0) return hipSuccess;
    k_fill_u32<<<nblocks(nA), kBlock, 0, s>>>(best, nA, 0x7f800000u);
    const int64_t chunk = nn_chunk(nA, nB);
    const int64_t split = (nB + chunk - 1) / chunk;
    k_nn<<<dim3(nblocks(nA), (unsigned)split), kBlock, 0, s>>>(A, nA, B, nB, chunk, best);
    k_nn_sqrt<<<nblocks(nA), kBlock, 0, s>>>(best, nA, d);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------ entry helpers

size_t cubify_workspace(int64_t P, int64_t C) { return plan_cubify(P, C).total; }
size_t smooth_workspace(int64_t nV, int64_t nF) { return plan_smooth(nV, nF).total; }
size_t sample_workspace(int64_t nF) { return plan_sample(nF).total; }
size_t nn_workspace(int64_t nA, int64_t nB) { return plan_nn(nA, nB).total; }

wn_status run_cubify(const uint8_t *occ, const int32_t n[3], const float lo[3], const float hi[3], float *V,
                     int64_t capV, int32_t *F, int64_t capF, int64_t *counts, char *ws, hipStream_t s) {
    const int64_t P = (int64_t)n[0] * n[1] * n[2];
    const int64_t C = (int64_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
    const CubPlan p = plan_cubify(P, C);
    int32_t *qcount = reinterpret_cast<int32_t *>(ws + p.off_qcount);
    int64_t *qoff = reinterpret_cast<int64_t *>(ws + p.off_qoff);
    int32_t *used = reinterpret_cast<int32_t *>(ws + p.off_used);
    int64_t *vid = reinterpret_cast<int64_t *>(ws + p.off_vid);
    Lattice L{{n[0], n[1], n[2]}};
    k_fill_u32<<<nblocks(C), kBlock, 0, s>>>(reinterpret_cast<uint32_t *>(used), C, 0u);
    if (P > 0) k_cub_count<<<nblocks(P), kBlock, 0, s>>>(occ, L, P, qcount, used);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return WN_ERR_HIP;
    size_t tmp = p.tmp;
    if (P > 0 && (e = rocprim::exclusive_scan(ws + p.off_tmp, tmp, qcount, qoff, (int64_t)0, (size_t)P,
                                              rocprim::plus<int64_t>(), s)) != hipSuccess)
        return WN_ERR_HIP;
    tmp = p.tmp;
    if ((e = rocprim::exclusive_scan(ws + p.off_tmp, tmp, used, vid, (int64_t)0, (size_t)C, rocprim::plus<int64_t>(),
                                     s)) != hipSuccess)
        return WN_ERR_HIP;
    k_cub_counts<<<1, kBlock, 0, s>>>(qcount, qoff, P, used, vid, C, counts);
    if (P > 0) {
        k_cub_faces<<<nblocks(P), kBlock, 0, s>>>(occ, L, P, qoff, vid, F, capF);
        const float3 lo3 = make_float3(lo[0], lo[1], lo[2]);
        const float3 h3 = make_float3((hi[0] - lo[0]) / (float)n[0], (hi[1] - lo[1]) / (float)n[1],
                                      (hi[2] - lo[2]) / (float)n[2]);
        k_cub_verts<<<nblocks(C), kBlock, 0, s>>>(used, vid, L, C, lo3, h3, V, capV);
    }
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status run_smooth(const float *V, int64_t nV, const int32_t *F, int64_t nF, float lam, int32_t iters,
                     int32_t keep_volume, float *Vout, char *ws, hipStream_t s) {
    const SmoothPlan p = plan_smooth(nV, nF);
    const int64_t nE = 6 * nF;
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    uint64_t *keys = reinterpret_cast<uint64_t *>(ws + p.off_keys);
    uint64_t *keys2 = reinterpret_cast<uint64_t *>(ws + p.off_keys2);
    int32_t *flag = reinterpret_cast<int32_t *>(ws + p.off_flag);
    int64_t *pos = reinterpret_cast<int64_t *>(ws + p.off_pos);
    int32_t *nbr = reinterpret_cast<int32_t *>(ws + p.off_nbr);
    int32_t *deg = reinterpret_cast<int32_t *>(ws + p.off_deg);
    int64_t *off = reinterpret_cast<int64_t *>(ws + p.off_off);
    float *T = reinterpret_cast<float *>(ws + p.off_T);
    double *vpart = reinterpret_cast<double *>(ws + p.off_vol);
    double *vol0 = vpart + kVolBlocks, *vscale = vol0 + 1;
    hipError_t e = launch_ws_reset(hdr, s);
    if (e != hipSuccess) return WN_ERR_HIP;
    if (nV == 0) return WN_OK;
    const bool rescale = keep_volume && nF > 0 && iters > 0;
    if (rescale) {
        k_volume_partial<<<kVolBlocks, kBlock, 0, s>>>(V, nV, F, nF, vpart);
        k_volume_final<<<1, kBlock, 0, s>>>(vpart, vol0, vscale, 1);
    }
    k_fill_u32<<<nblocks(nV + 1), kBlock, 0, s>>>(reinterpret_cast<uint32_t *>(deg), nV + 1, 0u);
    if (nE > 0) {
        k_edge_keys<<<nblocks(nF), kBlock, 0, s>>>(F, nF, nV, keys, hdr);
        if ((e = hipGetLastError()) != hipSuccess) return WN_ERR_HIP;
        size_t tmp = p.sort_tmp;
        if ((e = rocprim::radix_sort_keys(ws + p.off_tmp, tmp, keys, keys2, (size_t)nE, 0u, p.bits, s)) != hipSuccess)
            return WN_ERR_HIP;
        k_edge_unique<<<nblocks(nE), kBlock, 0, s>>>(keys2, nE, flag, deg);
        tmp = p.scan_tmp;
        if ((e = rocprim::exclusive_scan(ws + p.off_tmp, tmp, flag, pos, (int64_t)0, (size_t)nE,
                                         rocprim::plus<int64_t>(), s)) != hipSuccess)
            return WN_ERR_HIP;
        k_edge_compact<<<nblocks(nE), kBlock, 0, s>>>(keys2, nE, flag, pos, nbr);
    }
    // off = exclusive prefix of the degrees (deg[nV] = 0 makes off[nV] the edge count)
    size_t tmp = p.scan2_tmp;
    if ((e = rocprim::exclusive_scan(ws + p.off_tmp, tmp, deg, off, (int64_t)0, (size_t)(nV + 1),
                                     rocprim::plus<int64_t>(), s)) != hipSuccess)
        return WN_ERR_HIP;
    if (iters == 0) {
        k_copy_f32<<<nblocks(3 * nV), kBlock, 0, s>>>(V, Vout, 3 * nV);
    } else {
        const float *src = V;
        for (int32_t it = 0; it < iters; ++it) {
            float *dst = ((iters - 1 - it) % 2 == 0) ? Vout : T;
            k_smooth_step<<<nblocks(nV), kBlock, 0, s>>>(src, dst, nV, off, nbr, lam);
            if (rescale) {  // back to the starting volume, scaling about the origin
                k_volume_partial<<<kVolBlocks, kBlock, 0, s>>>(dst, nV, F, nF, vpart);
                k_volume_final<<<1, kBlock, 0, s>>>(vpart, vol0, vscale, 0);
                k_scale_f32<<<nblocks(3 * nV), kBlock, 0, s>>>(dst, 3 * nV, vscale);
            }
            src = dst;
        }
    }
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status run_sample(const float *V, int64_t nV, const int32_t *F, int64_t nF, const double *u, int64_t n, float *P,
                     int32_t *face, char *ws, hipStream_t s) {
    const SamplePlan p = plan_sample(nF);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    double *area = reinterpret_cast<double *>(ws + p.off_area);
    uint64_t *w = reinterpret_cast<uint64_t *>(ws + p.off_w);
    uint64_t *cdf = reinterpret_cast<uint64_t *>(ws + p.off_cdf);
    unsigned long long *amax = reinterpret_cast<unsigned long long *>(ws + p.off_max);
    hipError_t e = launch_ws_reset(hdr, s);
    if (e != hipSuccess) return WN_ERR_HIP;
    if (n == 0) return WN_OK;
    k_fill_u32<<<1, kBlock, 0, s>>>(reinterpret_cast<uint32_t *>(amax), 2, 0u);
    k_area<<<nblocks(nF), kBlock, 0, s>>>(V, nV, F, nF, area, amax, hdr);
    k_area_weights<<<nblocks(nF), kBlock, 0, s>>>(area, nF, amax, w);
    if ((e = hipGetLastError()) != hipSuccess) return WN_ERR_HIP;
    size_t tmp = p.scan_tmp;
    if ((e = rocprim::inclusive_scan(ws + p.off_tmp, tmp, w, cdf, (size_t)nF, rocprim::plus<uint64_t>(), s)) !=
        hipSuccess)
        return WN_ERR_HIP;
    k_sample<<<nblocks(n), kBlock, 0, s>>>(V, F, nV, nF, cdf, u, n, P, face);
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status run_nn(const float *A, int64_t nA, const float *B, int64_t nB, float *d, char *ws, hipStream_t s) {
    const NNPlan p = plan_nn(nA, nB);
    uint32_t *best = reinterpret_cast<uint32_t *>(ws + p.off_best);
    return launch_nn(A, nA, B, nB, best, d, s) == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status run_chamfer(const float *A, int64_t nA, const float *B, int64_t nB, double *out, char *ws, hipStream_t s) {
    const NNPlan p = plan_nn(nA, nB);
    uint32_t *best = reinterpret_cast<uint32_t *>(ws + p.off_best);
    float *dA = reinterpret_cast<float *>(ws + p.off_dA);
    float *dB = reinterpret_cast<float *>(ws + p.off_dB);
    double *psum = reinterpret_cast<double *>(ws + p.off_psum);
    float *pmax = reinterpret_cast<float *>(ws + p.off_pmax);
    if (launch_nn(A, nA, B, nB, best, dA, s) != hipSuccess) return WN_ERR_HIP;
    if (launch_nn(B, nB, A, nA, best, dB, s) != hipSuccess) return WN_ERR_HIP;
    k_sum_max<<<kRedBlocks, kBlock, 0, s>>>(dA, nA, psum, pmax);
    k_sum_max<<<kRedBlocks, kBlock, 0, s>>>(dB, nB, psum + kRedBlocks, pmax + kRedBlocks);
    k_metrics<<<1, kBlock, 0, s>>>(psum, pmax, nA, nB, out);
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

}  // namespace wn
