// Marching cubes of a field sampled at the voxel centres (the reconstruction the paper
// names when it motivates its accuracy measure, Section 3).
//
// The centres form a lattice; one layer of zeros is added around it so that the surface
// is closed.  The work is bookkeeping (memory- and latency-bound), done in fixed order:
//   * one thread per lattice point flags its three edges (+x, +y, +z) that the level
//     crosses (one endpoint above the level, the other at or below it);
//   * one thread per cell counts its triangles from its corner pattern (the table in
//     wn_mc_table.hpp, written by gen_mc_table.py from a per-face rule);
//   * two exclusive scans number the crossed edges (the vertices) and place each
//     cell's triangles;
//   * every crossed edge writes its vertex (linear interpolation of its two values) and
//     every cell writes its triangles.
// Vertex ids follow the edge numbering 3 * (padded lattice index) + axis, faces the cell
// order, so the output is deterministic.
#include <rocprim/device/device_scan.hpp>

#include "wn_internal.hpp"
#include "wn_mc_table.hpp"

namespace wn {

namespace {

unsigned mc_blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// The padded lattice: N[d] = n[d] + 2 points per axis, point (i, j, k) holding the value
// of voxel (i - 1, j - 1, k - 1) or 0 outside the grid.
struct McLattice {
    int32_t n[3];
    int64_t N[3];
    __device__ float value(const float *__restrict__ f, int64_t i, int64_t j, int64_t k) const {
        if (i < 1 || j < 1 || k < 1 || i > n[0] || j > n[1] || k > n[2]) return 0.0f;
        return f[((i - 1) * n[1] + (j - 1)) * (int64_t)n[2] + (k - 1)];
    }
    __device__ void point(int64_t p, int64_t (&ijk)[3]) const {
        ijk[2] = p % N[2];
        const int64_t r = p / N[2];
        ijk[1] = r % N[1];
        ijk[0] = r / N[1];
    }
    __device__ int64_t index(int64_t i, int64_t j, int64_t k) const { return (i * N[1] + j) * N[2] + k; }
};

__global__ __launch_bounds__(kBlock) void k_mc_edges(const float *__restrict__ f, McLattice L, int64_t nL, float iso,
                                                     int32_t *__restrict__ eflag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nL) return;
    int64_t c[3];
    L.point(p, c);
    const bool in = L.value(f, c[0], c[1], c[2]) > iso;
    for (int a = 0; a < 3; ++a) {
        int64_t q[3] = {c[0], c[1], c[2]};
        ++q[a];
        int32_t crossed = 0;
        if (q[a] < L.N[a]) crossed = (L.value(f, q[0], q[1], q[2]) > iso) != in;
        eflag[3 * p + a] = crossed;
    }
}

// Corner pattern of the cell whose lowest corner is padded point (i, j, k): bit
// a + 2b + 4c for the corner at offsets (a, b, c).
__device__ __forceinline__ int mc_pattern(const float *__restrict__ f, const McLattice &L, int64_t i, int64_t j,
                                          int64_t k, float iso) {
    int pat = 0;
    for (int c = 0; c < 8; ++c)
        if (L.value(f, i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)) > iso) pat |= 1 << c;
    return pat;
}

__device__ __forceinline__ void mc_cell(int64_t cell, const McLattice &L, int64_t (&ijk)[3]) {
    const int64_t M1 = L.N[1] - 1, M2 = L.N[2] - 1;
    ijk[2] = cell % M2;
    const int64_t r = cell / M2;
    ijk[1] = r % M1;
    ijk[0] = r / M1;
}

__global__ __launch_bounds__(kBlock) void k_mc_count(const float *__restrict__ f, McLattice L, int64_t nC, float iso,
                                                     int32_t *__restrict__ tcount) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nC) return;
    int64_t c[3];
    mc_cell(cell, L, c);
    tcount[cell] = c_mc_count[mc_pattern(f, L, c[0], c[1], c[2], iso)];
}

__global__ __launch_bounds__(kBlock) void k_mc_counts(const int32_t *__restrict__ eflag,
                                                      const int64_t *__restrict__ eoff, int64_t nE,
                                                      const int32_t *__restrict__ tcount,
                                                      const int64_t *__restrict__ toff, int64_t nC,
                                                      int64_t *__restrict__ counts) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    counts[0] = nE > 0 ? eoff[nE - 1] + eflag[nE - 1] : 0;
    counts[1] = nC > 0 ? toff[nC - 1] + tcount[nC - 1] : 0;
}

__global__ __launch_bounds__(kBlock) void k_mc_verts(const float *__restrict__ f, McLattice L, int64_t nE, float iso,
                                                     const int32_t *__restrict__ eflag,
                                                     const int64_t *__restrict__ eoff, float3 lo, float3 h,
                                                     float *__restrict__ V, int64_t capV) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE || !eflag[e]) return;
    const int64_t id = eoff[e];
    if (id >= capV) return;
    const int a = (int)(e % 3);
    int64_t c[3];
    L.point(e / 3, c);
    const float fa = L.value(f, c[0], c[1], c[2]);
    const float fb = L.value(f, c[0] + (a == 0), c[1] + (a == 1), c[2] + (a == 2));
    const float t = (iso - fa) / (fb - fa);
    // centre of padded point c: lo + (c - 1/2) h
    float x[3] = {(float)c[0] - 0.5f, (float)c[1] - 0.5f, (float)c[2] - 0.5f};
    x[a] += t;
    V[3 * id] = __builtin_fmaf(x[0], h.x, lo.x);
    V[3 * id + 1] = __builtin_fmaf(x[1], h.y, lo.y);
    V[3 * id + 2] = __builtin_fmaf(x[2], h.z, lo.z);
}

__global__ __launch_bounds__(kBlock) void k_mc_faces(const float *__restrict__ f, McLattice L, int64_t nC, float iso,
                                                     const int64_t *__restrict__ toff,
                                                     const int64_t *__restrict__ eoff, int32_t *__restrict__ F,
                                                     int64_t capF) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nC) return;
    int64_t c[3];
    mc_cell(cell, L, c);
    const int pat = mc_pattern(f, L, c[0], c[1], c[2], iso);
    const int nt = c_mc_count[pat];
    const int64_t t0 = toff[cell];
    for (int t = 0; t < nt; ++t) {
        if (t0 + t >= capF) return;
        for (int j = 0; j < 3; ++j) {
            // local edge e: along axis e / 4 from the corner whose other two offsets (in
            // increasing axis order) are (e & 1, e >> 1 & 1)
            const int e = c_mc_tris[pat][3 * t + j];
            const int a = e >> 2, u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
            int64_t q[3] = {c[0], c[1], c[2]};
            q[u] += e & 1;
            q[w] += (e >> 1) & 1;
            F[3 * (t0 + t) + j] = (int32_t)eoff[3 * L.index(q[0], q[1], q[2]) + a];
        }
    }
}

struct McPlan {
    size_t tmp, off_eflag, off_eoff, off_tcount, off_toff, off_tmp, total;
};

McPlan plan_mc(int64_t nE, int64_t nC) {
    McPlan p{};
    size_t t1 = 0, t2 = 0;
    if (nE > 0)
        (void)rocprim::exclusive_scan(nullptr, t1, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                      (size_t)nE, rocprim::plus<int64_t>());
    if (nC > 0)
        (void)rocprim::exclusive_scan(nullptr, t2, (const int32_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                                      (size_t)nC, rocprim::plus<int64_t>());
    p.tmp = t1 > t2 ? t1 : t2;
    size_t o = kWsHeader;
    p.off_eflag = o;
    o += align_up((size_t)nE * 4);
    p.off_eoff = o;
    o += align_up((size_t)nE * 8);
    p.off_tcount = o;
    o += align_up((size_t)nC * 4);
    p.off_toff = o;
    o += align_up((size_t)nC * 8);
    p.off_tmp = o;
    o += align_up(p.tmp > 0 ? p.tmp : 1);
    p.total = o;
    return p;
}

constexpr int64_t kMcMaxIndex = 2147483647LL;  // vertex ids are int32

// Lattice sizes of a grid, or false when they do not fit.
bool mc_sizes(const wn_grid *grid, int64_t &nL, int64_t &nC) {
    if (!grid) return false;
    nL = 1;
    nC = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 0) return false;
        nL *= (int64_t)grid->n[d] + 2;
        nC *= (int64_t)grid->n[d] + 1;
    }
    return 3 * nL <= kMcMaxIndex;
}

bool mc_aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

}  // namespace

}  // namespace wn

using namespace wn;

extern "C" {

size_t wn_workspace_size_marching(const wn_grid *grid) {
    int64_t nL, nC;
    if (!mc_sizes(grid, nL, nC)) return 0;
    return plan_mc(3 * nL, nC).total;
}

wn_status wn_marching_cubes(const float *f, const wn_grid *grid, float iso, float *V, int64_t capV, int32_t *F,
                            int64_t capF, int64_t *counts, void *ws, size_t ws_bytes, void *stream) {
    int64_t nL, nC;
    if (!mc_sizes(grid, nL, nC) || counts == nullptr || capV < 0 || capF < 0) return WN_ERR_INVALID_ARG;
    if (!(iso > 0.0f) || !(iso <= 3.4e38f)) return WN_ERR_INVALID_ARG;
    const int64_t P = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    if (P > 0 && f == nullptr) return WN_ERR_INVALID_ARG;
    if ((capV > 0 && V == nullptr) || (capF > 0 && F == nullptr)) return WN_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    const int64_t nE = 3 * nL;
    const McPlan p = plan_mc(nE, nC);
    if (ws == nullptr || !mc_aligned256(ws) || ws_bytes < p.total) return WN_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    int32_t *eflag = reinterpret_cast<int32_t *>(w + p.off_eflag);
    int64_t *eoff = reinterpret_cast<int64_t *>(w + p.off_eoff);
    int32_t *tcount = reinterpret_cast<int32_t *>(w + p.off_tcount);
    int64_t *toff = reinterpret_cast<int64_t *>(w + p.off_toff);
    McLattice L{{grid->n[0], grid->n[1], grid->n[2]},
                {(int64_t)grid->n[0] + 2, (int64_t)grid->n[1] + 2, (int64_t)grid->n[2] + 2}};
    k_mc_edges<<<mc_blocks(nL), kBlock, 0, s>>>(f, L, nL, iso, eflag);
    k_mc_count<<<mc_blocks(nC), kBlock, 0, s>>>(f, L, nC, iso, tcount);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return WN_ERR_HIP;
    size_t tmp = p.tmp;
    if ((e = rocprim::exclusive_scan(w + p.off_tmp, tmp, eflag, eoff, (int64_t)0, (size_t)nE,
                                     rocprim::plus<int64_t>(), s)) != hipSuccess)
        return WN_ERR_HIP;
    tmp = p.tmp;
    if ((e = rocprim::exclusive_scan(w + p.off_tmp, tmp, tcount, toff, (int64_t)0, (size_t)nC,
                                     rocprim::plus<int64_t>(), s)) != hipSuccess)
        return WN_ERR_HIP;
    k_mc_counts<<<1, kBlock, 0, s>>>(eflag, eoff, nE, tcount, toff, nC, counts);
    const float hx = grid->n[0] > 0 ? (grid->hi[0] - grid->lo[0]) / (float)grid->n[0] : 0.0f;
    const float hy = grid->n[1] > 0 ? (grid->hi[1] - grid->lo[1]) / (float)grid->n[1] : 0.0f;
    const float hz = grid->n[2] > 0 ? (grid->hi[2] - grid->lo[2]) / (float)grid->n[2] : 0.0f;
    if (capV > 0)
        k_mc_verts<<<mc_blocks(nE), kBlock, 0, s>>>(f, L, nE, iso, eflag, eoff,
                                                    make_float3(grid->lo[0], grid->lo[1], grid->lo[2]),
                                                    make_float3(hx, hy, hz), V, capV);
    if (capF > 0) k_mc_faces<<<mc_blocks(nC), kBlock, 0, s>>>(f, L, nC, iso, toff, eoff, F, capF);
    return hipGetLastError() == hipSuccess ? WN_OK : WN_ERR_HIP;
}

}  // extern "C"
