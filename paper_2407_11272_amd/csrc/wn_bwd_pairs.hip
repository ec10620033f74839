// Adjoint with two faces per lane (face pairs): pair records, the kernel and the
// reduction of its running sums.  The arithmetic per face is that of the one-face-per-
// lane adjoint (the chain rule through Eq. 7/8 for dW/dv, Section 2.4 of arXiv
// 2407.11272); this file is compiled with the backend's ILP-first scheduler, which
// orders this kernel's point loop better (and the one-face kernel's worse).
#include "wn_internal.hpp"

namespace wn {

constexpr int kPointTile = kBwdTile;

// ------------------------------------------- two faces per lane (face pairs) ---
//
// A lane owns a pair of faces f and g that share an edge.  Its four vertices (slots
// 0..3) are f = (s0, s1, s2) and g = (s3, s1, s2) up to g's winding, so the shared edge's
// two vertices (their distances, unit vectors and dot product) are evaluated once for
// both faces: 4 instead of 6 vertices and 5 instead of 6 dot products per point.  The
// per-face arithmetic is that of k_wn_bwd.  The corner vector of a face does not depend
// on the order of its corners (alpha through the face's own normal, beta and E are
// symmetric, dd_j = e_k . e_l), so the per-point work is the same for both windings of
// g; only the per-tile beta u_j terms and the output corner order use the winding.
//   rec: a = (s0.xyz, s1.x), b = (s1.yz, s2.xy), c = (s2.z, s3.xyz), d = (Nf.xyz, Ng.x),
//        e = (Ng.yz, 0, 0);  Nf, Ng = the faces' normals in their own windings.
//   meta: f; g (-1: f alone, slot 3 a copy of slot 2); code = rf | rg << 2 | flip << 4,
//        rf (rg) = f's (g's) corner at slot 0 (3) in F, flip = g's corners in F order
//        are (s3, s1, s2) (else (s3, s2, s1)).
//   state: float2 (sum, compensation) [S][18][nP], per pair f's 9 corner components in
//        rotated order, then g's by slot 1, 2, 3; k_bwd_reduce_pairs maps them to T.
//        Merged ([S][12][nP], dL/dV only): slot 0, slots 1 and 2 of both faces, g's slot 3.
struct PairRec {
    float4 a, b, c, d, e;
};
struct PairMeta {
    int32_t f, g, code, pad;
};
static_assert(sizeof(PairRec) == kPairRecBytes && sizeof(PairMeta) == kPairMetaBytes, "pair record sizes");

// Pair records from a list of (f, g or -1) face pairs.  Every face must appear exactly
// once and a pair must share exactly one edge of two distinct vertex ids; anything else
// is recorded as a bad index (a pair without a shared edge keeps only f).
__global__ __launch_bounds__(kBlock) void k_pack_pairs(const float *__restrict__ V, int64_t nV,
                                                       const int32_t *__restrict__ F, int64_t nF,
                                                       const int32_t *__restrict__ pairs, int64_t nP,
                                                       PairRec *__restrict__ recs, PairMeta *__restrict__ meta,
                                                       int32_t *__restrict__ counts, WsHeader *hdr) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nP) return;
    bool bad = false;
    int32_t f = pairs[2 * p], g = pairs[2 * p + 1];
    if (f < 0 || (int64_t)f >= nF) {
        atomicOr(&hdr->bad_index, 1);
        meta[p] = PairMeta{-1, -1, 0, 0};
        return;
    }
    if (g != -1 && (g < 0 || (int64_t)g >= nF || g == f)) {
        bad = true;
        g = -1;
    }
    int32_t a[3], b[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j) {
        a[j] = F[3 * (int64_t)f + j];
        if (a[j] < 0 || (int64_t)a[j] >= nV) bad = true, a[j] = 0;
    }
    int rf = 0, rg = 0, flip = 0;
    if (g >= 0) {
        for (int j = 0; j < 3; ++j) {
            b[j] = F[3 * (int64_t)g + j];
            if (b[j] < 0 || (int64_t)b[j] >= nV) bad = true, b[j] = 0;
        }
        int na = 0, nb = 0;  // corners of f not in g, and of g not in f
        for (int j = 0; j < 3; ++j) {
            const bool ina = a[j] == b[0] || a[j] == b[1] || a[j] == b[2];
            const bool inb = b[j] == a[0] || b[j] == a[1] || b[j] == a[2];
            if (!ina) rf = j, ++na;
            if (!inb) rg = j, ++nb;
        }
        const bool distinct = a[0] != a[1] && a[1] != a[2] && a[2] != a[0] && b[0] != b[1] && b[1] != b[2] &&
                              b[2] != b[0];
        if (na != 1 || nb != 1 || !distinct) {
            bad = true;
            g = -1;
            rf = 0;
        } else {
            flip = b[(rg + 1) % 3] == a[(rf + 1) % 3] ? 1 : 0;
        }
    }
    atomicAdd(&counts[f], 1);
    if (g >= 0) atomicAdd(&counts[g], 1);
    if (bad) atomicOr(&hdr->bad_index, 1);
    double s[4][3];
    const int32_t id[4] = {a[rf], a[(rf + 1) % 3], a[(rf + 2) % 3], g >= 0 ? b[rg] : a[(rf + 2) % 3]};
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) s[k][c] = V[3 * (int64_t)id[k] + c];
    auto cross = [](const double *u0, const double *u1, const double *u2, double *n) {
        const double ex = u1[0] - u0[0], ey = u1[1] - u0[1], ez = u1[2] - u0[2];
        const double fx = u2[0] - u0[0], fy = u2[1] - u0[1], fz = u2[2] - u0[2];
        n[0] = ey * fz - ez * fy;
        n[1] = ez * fx - ex * fz;
        n[2] = ex * fy - ey * fx;
    };
    double nf[3], ng[3] = {0.0, 0.0, 0.0};
    cross(s[0], s[1], s[2], nf);
    if (g >= 0) {
        if (flip)
            cross(s[3], s[1], s[2], ng);
        else
            cross(s[3], s[2], s[1], ng);
    }
    PairRec r;
    r.a = make_float4((float)s[0][0], (float)s[0][1], (float)s[0][2], (float)s[1][0]);
    r.b = make_float4((float)s[1][1], (float)s[1][2], (float)s[2][0], (float)s[2][1]);
    r.c = make_float4((float)s[2][2], (float)s[3][0], (float)s[3][1], (float)s[3][2]);
    r.d = make_float4((float)nf[0], (float)nf[1], (float)nf[2], (float)ng[0]);
    r.e = make_float4((float)ng[1], (float)ng[2], 0.0f, 0.0f);
    recs[p] = r;
    meta[p] = PairMeta{f, g, rf | (rg << 2) | (flip << 4), 0};
}

// N running sums of a lane, rows[i * nP + p] (i < N, rows wave-uniform): all N loaded,
// the tile's sums t[0..N) folded in (from zero when `first`), stored if `live`.
template <int N>
__device__ __forceinline__ void fold_rows(float2 *__restrict__ rows, int32_t nP, int32_t p, bool live, bool first,
                                          const float *t) {
    float2 x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = rows[(int64_t)i * nP + p];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (first) x[i] = make_float2(0.0f, 0.0f);
        neumaier_add(x[i].x, x[i].y, t[i]);
    }
    if (live) {
#pragma unroll
        for (int i = 0; i < N; ++i) rows[(int64_t)i * nP + p] = x[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_check_counts(const int32_t *__restrict__ counts, int64_t nF,
                                                         WsHeader *hdr) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nF && counts[f] != 1) atomicOr(&hdr->bad_index, 1);
}

// kMerge: the two faces add their sums at their shared vertices (slots 1 and 2): 12 rows
// per pair (slot 0, slots 1 and 2 merged, slot 3) instead of 18, for callers that want
// dL/dV only.  A lane without a second face has its normal Ng = 0, so that face's per-point
// corner terms are exactly zero; its tile sums of w (the beta u_j terms) are dropped.
// kThreads: lanes per workgroup, 256 or 64 (one wave); every wave stages the whole point
// tile, so the per-lane arithmetic and the bits do not depend on it.
template <bool kMerge, int kThreads>
__global__ __launch_bounds__(kThreads) void k_wn_bwd_pairs(const PairRec *__restrict__ recs,
                                                         const PairMeta *__restrict__ meta, int32_t nP, int32_t nF,
                                                         PointSrc ps, int64_t nQ, int32_t S, int64_t t0, int64_t t1,
                                                         const float *__restrict__ dLdW,
                                                         float2 *__restrict__ state) {
    __shared__ float4 pts[kPointTile];
    const int tid = threadIdx.x;
    const int64_t tfirst = t0 + blockIdx.y;
    const int64_t sy = tfirst % S;
    int32_t p = (int32_t)blockIdx.x * kThreads + tid;
    const bool live = p < nP;
    p = live ? p : nP - 1;
    const PairRec r = recs[p];
    const PairMeta m = meta[p];
    const bool has_g = m.g >= 0;
    const bool any_g = __builtin_amdgcn_ballot_w64(live && has_g) != 0ull;  // wave-uniform
    constexpr int kRows = kMerge ? 12 : 18;  // running sums per pair and split
    const int flip = (m.code >> 4) & 1;
    const float v[4][3] = {{r.a.x, r.a.y, r.a.z}, {r.a.w, r.b.x, r.b.y}, {r.b.z, r.b.w, r.c.x}, {r.c.y, r.c.z, r.c.w}};
    const float Nf[3] = {r.d.x, r.d.y, r.d.z}, Ng[3] = {r.d.w, r.e.x, r.e.y};

    // The running sums stay in the state array and each tile's sums are folded in there
    // (read, Neumaier step, write), which keeps 36 registers free for the point loop; the
    // split's first tile starts from zero.
    for (int64_t t = tfirst; t < t1; t += S) {
        const int64_t q0 = t * kPointTile;
        const int nt = (int)min((int64_t)kPointTile, nQ - q0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPointTile / kThreads; ++k) {
            const int j = tid + k * kThreads;
            if (j < nt) {
                float x, y, z;
                ps.get(q0 + j, x, y, z);
                pts[j] = make_float4(x, y, z, dLdW[q0 + j]);
            }
        }
        __syncthreads();
        float tf[9], tg[9], swf = 0.0f, swg = 0.0f, sqf[3] = {0.0f, 0.0f, 0.0f}, sqg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < 9; ++i) tf[i] = tg[i] = 0.0f;
        for (int i = 0; i < nt; ++i) {
            const float4 q = pts[i];
            float R[4][3], e[4][3], ri[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k == 3 && !any_g) break;
                R[k][0] = v[k][0] - q.x;
                R[k][1] = v[k][1] - q.y;
                R[k][2] = v[k][2] - q.z;
                const float l2 = R[k][0] * R[k][0] + R[k][1] * R[k][1] + R[k][2] * R[k][2];
                ri[k] = (l2 > 0.0f) ? __builtin_amdgcn_rsqf(l2) : 0.0f;
                e[k][0] = R[k][0] * ri[k];
                e[k][1] = R[k][1] * ri[k];
                e[k][2] = R[k][2] * ri[k];
            }
            const float d01 = e[0][0] * e[1][0] + e[0][1] * e[1][1] + e[0][2] * e[1][2];
            const float d12 = e[1][0] * e[2][0] + e[1][1] * e[2][1] + e[1][2] * e[2][2];
            const float d20 = e[2][0] * e[0][0] + e[2][1] * e[0][1] + e[2][2] * e[0][2];
            const float r12 = ri[1] * ri[2];
            float e12[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) e12[d] = e[1][d] + e[2][d];
            float ngaf = 0.0f, Ef[3] = {0.0f, 0.0f, 0.0f};  // kept for the merged slots 1, 2
            (void)ngaf;
            (void)Ef;
            {  // face f = (s0, s1, s2)
                const float rho = ri[0] * r12;
                const float alpha = rho * (R[0][0] * Nf[0] + R[0][1] * Nf[1] + R[0][2] * Nf[2]);
                const float beta = 1.0f + d01 + d12 + d20;
                const float den = alpha * alpha + beta * beta;
                const float gk = (den > 0.0f) ? q.w * __builtin_amdgcn_rcpf(den) : 0.0f;
                const float w = gk * beta * rho, nga = -(gk * alpha);
                swf += w;
#pragma unroll
                for (int d = 0; d < 3; ++d) sqf[d] = __builtin_fmaf(w, R[0][d], sqf[d]);
                float E[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) E[d] = e[0][d] + e12[d];
                const float dd[3] = {d12, d20, d01};  // e_k . e_l of corner j
                // merging with a second face in the wave: corners 1 and 2 go with g's slots
                const int jn = (kMerge && any_g) ? 1 : 3;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j >= jn) break;
                    const float nca = nga * ri[j], ncd = nca * dd[j];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        tf[3 * j + d] = __builtin_fmaf(nca, E[d], tf[3 * j + d]);
                        tf[3 * j + d] = __builtin_fmaf(ncd, e[j][d], tf[3 * j + d]);
                    }
                }
                if constexpr (kMerge) {
                    ngaf = nga;
#pragma unroll
                    for (int d = 0; d < 3; ++d) Ef[d] = E[d];
                }
            }
            if (any_g) {  // face g = (s3, s1, s2) up to winding; accumulators by slot 1, 2, 3
                const float d13 = e[1][0] * e[3][0] + e[1][1] * e[3][1] + e[1][2] * e[3][2];
                const float d23 = e[2][0] * e[3][0] + e[2][1] * e[3][1] + e[2][2] * e[3][2];
                const float rho = ri[3] * r12;
                const float alpha = rho * (R[3][0] * Ng[0] + R[3][1] * Ng[1] + R[3][2] * Ng[2]);
                const float beta = 1.0f + d13 + d12 + d23;
                const float den = alpha * alpha + beta * beta;
                const float gk = (den > 0.0f) ? q.w * __builtin_amdgcn_rcpf(den) : 0.0f;
                const float w = gk * beta * rho, nga = -(gk * alpha);
                swg += w;
#pragma unroll
                for (int d = 0; d < 3; ++d) sqg[d] = __builtin_fmaf(w, R[3][d], sqg[d]);
                float E[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) E[d] = e[3][d] + e12[d];
                const float dd[3] = {d23, d13, d12};  // slots 1, 2, 3
                const float rs[3] = {ri[1], ri[2], ri[3]};
                if constexpr (kMerge) {
                    // slots 1 and 2: f's corner and g's slot on the same vertex, one e_j term
                    const float ddf[2] = {d20, d01};
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const float ncf = ngaf * ri[j + 1], ncg = nga * rs[j];
                        const float ncd = ncf * ddf[j] + ncg * dd[j];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            tf[3 * (j + 1) + d] = __builtin_fmaf(ncf, Ef[d], tf[3 * (j + 1) + d]);
                            tf[3 * (j + 1) + d] = __builtin_fmaf(ncg, E[d], tf[3 * (j + 1) + d]);
                            tf[3 * (j + 1) + d] = __builtin_fmaf(ncd, e[j + 1][d], tf[3 * (j + 1) + d]);
                        }
                    }
                    const float nca = nga * rs[2], ncd = nca * dd[2];  // slot 3: g alone
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        tg[6 + d] = __builtin_fmaf(nca, E[d], tg[6 + d]);
                        tg[6 + d] = __builtin_fmaf(ncd, e[3][d], tg[6 + d]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const float nca = nga * rs[j], ncd = nca * dd[j];
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            tg[3 * j + d] = __builtin_fmaf(nca, E[d], tg[3 * j + d]);
                            tg[3 * j + d] = __builtin_fmaf(ncd, e[j + 1][d], tg[3 * j + d]);
                        }
                    }
                }
            }
        }
        // the tile's beta u_j terms: C_j sum(w) + D_j x sum(w R_c0) in each face's winding.
        // The edge vectors are formed here from opaque copies of the vertices, so that the
        // compiler does not keep 27 of them alive through the point loop.
        float u[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                u[k][d] = v[k][d];
                asm volatile("" : "+v"(u[k][d]));
            }
        {
            const float D[3][3] = {{u[1][0] - u[2][0], u[1][1] - u[2][1], u[1][2] - u[2][2]},
                                   {u[2][0] - u[0][0], u[2][1] - u[0][1], u[2][2] - u[0][2]},
                                   {u[0][0] - u[1][0], u[0][1] - u[1][1], u[0][2] - u[1][2]}};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float cj = (j == 0) ? swf : 0.0f;
                tf[3 * j + 0] += cj * Nf[0] + (D[j][1] * sqf[2] - D[j][2] * sqf[1]);
                tf[3 * j + 1] += cj * Nf[1] + (D[j][2] * sqf[0] - D[j][0] * sqf[2]);
                tf[3 * j + 2] += cj * Nf[2] + (D[j][0] * sqf[1] - D[j][1] * sqf[0]);
            }
        }
        if (any_g) {
            if constexpr (kMerge) {  // a lane without a second face: its w sums are dropped
                swg = has_g ? swg : 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) sqg[d] = has_g ? sqg[d] : 0.0f;
            }
            const float sgn = flip ? 1.0f : -1.0f;
            const float sq[3] = {sgn * sqg[0], sgn * sqg[1], sgn * sqg[2]};
            // slots 1, 2, 3: (v2 - v3), (v3 - v1), (v1 - v2), and C = Ng at slot 3
            const float D[3][3] = {{u[2][0] - u[3][0], u[2][1] - u[3][1], u[2][2] - u[3][2]},
                                   {u[3][0] - u[1][0], u[3][1] - u[1][1], u[3][2] - u[1][2]},
                                   {u[1][0] - u[2][0], u[1][1] - u[2][1], u[1][2] - u[2][2]}};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float cj = (j == 2) ? swg : 0.0f;
                float *acc = (kMerge && j < 2) ? &tf[3 * (j + 1)] : &tg[3 * j];  // merged slots 1, 2
                acc[0] += cj * Ng[0] + (D[j][1] * sq[2] - D[j][2] * sq[1]);
                acc[1] += cj * Ng[1] + (D[j][2] * sq[0] - D[j][0] * sq[2]);
                acc[2] += cj * Ng[2] + (D[j][0] * sq[1] - D[j][1] * sq[0]);
            }
        }
        // rows of the state are wave-uniform pointers (scalar registers), the lane adds p;
        // all loads are issued before the first add (a fresh split reads and discards)
        const bool first = t < S;  // tile t is its split's first: the sums start at zero
        fold_rows<9>(state + (int64_t)sy * kRows * nP, nP, p, live, first, tf);
        if constexpr (kMerge) {
            if (any_g) fold_rows<3>(state + ((int64_t)sy * kRows + 9) * nP, nP, p, live, first, tg + 6);
        } else {
            if (any_g) fold_rows<9>(state + ((int64_t)sy * kRows + 9) * nP, nP, p, live, first, tg);
        }
    }
}

// T from the pairs' running sums: each (sum, compensation) slot summed over the splits
// in split order, then written to its face's corner in F order (f by rotated corner, g by
// slot: slots 1, 2, 3 are g's rotated corners (flip ? 1 : 2), (flip ? 2 : 1), 0).  With
// rows == 12 (merged slots 1 and 2) the merged sums go to f's corners, g's corners at
// slots 1 and 2 get zero, and rows 9..11 are g's slot 3: the sums per vertex are exact,
// the split between the two corners of a shared vertex is not.
__global__ __launch_bounds__(kBlock) void k_bwd_reduce_pairs(const float2 *__restrict__ state, int32_t split,
                                                             int32_t nP, int32_t rows,
                                                             const PairMeta *__restrict__ meta, float scale,
                                                             float *__restrict__ T) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nP * rows) return;
    const int32_t i = (int32_t)(t / nP);
    const int32_t p = (int32_t)(t - (int64_t)i * nP);
    const PairMeta m = meta[p];
    const int rf = m.code & 3, rg = (m.code >> 2) & 3, flip = (m.code >> 4) & 1;
    auto g_corner = [&](int slot) {
        const int cj = slot == 3 ? 0 : (slot == 1 ? (flip ? 1 : 2) : (flip ? 2 : 1));
        return (cj + rg) % 3;
    };
    int32_t face;
    int corner;
    const int d = i % 3;
    if (i < 9) {
        face = m.f;
        corner = (i / 3 + rf) % 3;
        if (rows == 12 && i >= 3 && m.g >= 0) T[(int64_t)m.g * 9 + 3 * g_corner(i / 3) + d] = 0.0f;
    } else {
        face = m.g;
        corner = g_corner(rows == 12 ? 3 : (i - 9) / 3 + 1);
    }
    if (face < 0) return;
    const float2 *q = state + (int64_t)i * nP + p;
    const int64_t stride = (int64_t)rows * nP;  // from one split to the next
    float s = 0.0f, c = 0.0f;
    int32_t k = 0;
    for (; k + kReduceBatch <= split; k += kReduceBatch) {
        float2 x[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) x[u] = q[(int64_t)(k + u) * stride];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) neumaier_add(s, c, x[u].x + x[u].y);
    }
    for (; k < split; ++k) {
        const float2 x = q[(int64_t)k * stride];
        neumaier_add(s, c, x.x + x.y);
    }
    T[(int64_t)face * 9 + 3 * corner + d] = (s + c) * scale;
}


__global__ __launch_bounds__(kBlock) void k_zero_counts(int32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

namespace {
unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
}  // namespace

hipError_t launch_pack_pairs(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *pairs, int64_t nP,
                             char *recs, char *meta, int32_t *counts, WsHeader *hdr, hipStream_t s) {
    k_zero_counts<<<blocks_of(nF), kBlock, 0, s>>>(counts, nF);
    k_pack_pairs<<<blocks_of(nP), kBlock, 0, s>>>(V, nV, F, nF, pairs, nP, reinterpret_cast<PairRec *>(recs),
                                                  reinterpret_cast<PairMeta *>(meta), counts, hdr);
    k_check_counts<<<blocks_of(nF), kBlock, 0, s>>>(counts, nF, hdr);
    return hipGetLastError();
}

hipError_t launch_bwd_pairs(const char *recs, const char *meta, int32_t nP, int32_t nF, const PointSrc &ps, int64_t nQ,
                            int32_t S, int64_t t0, int64_t t1, int32_t rows, const float *dLdW, float2 *state,
                            bool merged, hipStream_t s) {
    static_assert(kPointTile % 64 == 0 && kBlock % 64 == 0, "whole waves");
    // One-wave workgroups avoid the idle waves of a last, mostly empty column of 256-lane
    // workgroups (C3: 2576 pairs, 44 waves for 41 of work); they cost about 2.5 % more per
    // wave otherwise (four times the workgroups, each staging the whole tile), so they are
    // taken only when that column would waste more than that.
    const int64_t waves_wide = (int64_t)(kBlock / 64) * ((nP + kBlock - 1) / kBlock), waves_narrow = (nP + 63) / 64;
    const bool narrow = waves_wide * 40 > waves_narrow * 41;
    const auto *r = reinterpret_cast<const PairRec *>(recs);
    const auto *m = reinterpret_cast<const PairMeta *>(meta);
    if (narrow) {
        const dim3 grid((unsigned)waves_narrow, (unsigned)rows);
        if (merged)
            k_wn_bwd_pairs<true, 64><<<grid, 64, 0, s>>>(r, m, nP, nF, ps, nQ, S, t0, t1, dLdW, state);
        else
            k_wn_bwd_pairs<false, 64><<<grid, 64, 0, s>>>(r, m, nP, nF, ps, nQ, S, t0, t1, dLdW, state);
    } else {
        const dim3 grid(blocks_of(nP), (unsigned)rows);
        if (merged)
            k_wn_bwd_pairs<true, kBlock><<<grid, kBlock, 0, s>>>(r, m, nP, nF, ps, nQ, S, t0, t1, dLdW, state);
        else
            k_wn_bwd_pairs<false, kBlock><<<grid, kBlock, 0, s>>>(r, m, nP, nF, ps, nQ, S, t0, t1, dLdW, state);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_pairs(const float2 *state, int32_t S, int32_t nP, const char *meta, float scale, float *T,
                               bool merged, hipStream_t s) {
    const int32_t rows = merged ? 12 : 18;
    k_bwd_reduce_pairs<<<blocks_of((int64_t)rows * nP), kBlock, 0, s>>>(
        state, S, nP, rows, reinterpret_cast<const PairMeta *>(meta), scale, T);
    return hipGetLastError();
}

}  // namespace wn
