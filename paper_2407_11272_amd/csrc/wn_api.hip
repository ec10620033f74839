// C ABI entry points declared in include/wn.h: argument checks, workspace
// layout and the launch sequence of each call.  No entry point allocates device
// memory or synchronises (except wn_get_device_error).
#include <stdio.h>
#include <cmath>
#include <algorithm>
#include <string.h>

#include <string>
#include <vector>

#include "wn_internal.hpp"

using namespace wn;

namespace {

constexpr int64_t kMaxCount = 2147483647LL;  // 2^31 - 1

bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

wn_status hip_status(hipError_t e) { return e == hipSuccess ? WN_OK : WN_ERR_HIP; }

// Number of query points described by (grid, Q, nQ), or -1 when inconsistent.
int64_t query_count(const wn_grid *grid, const float *Q, int64_t nQ) {
    if (nQ < 0) return -1;
    if (grid == nullptr && Q == nullptr) return nQ == 0 ? 0 : -1;  // empty point list
    if (grid != nullptr && Q != nullptr) return -1;
    if (!grid) return nQ <= kMaxCount ? nQ : -1;
    int64_t p = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 0) return -1;
        p *= grid->n[d];
        if (p > kMaxCount) return -1;
    }
    if (nQ != 0 && nQ != p) return -1;
    return p;
}

bool mesh_ok(const float *V, int64_t nV, const int32_t *F, int64_t nF) {
    if (nV < 0 || nF < 0 || nV > kMaxCount || nF > kMaxCount) return false;
    if (nF > 0 && (V == nullptr || F == nullptr || nV == 0)) return false;
    return true;
}

size_t voxelize_ws(int64_t nR, int64_t nQ) {
    const int split = fwd_split_count(nR, nQ);
    size_t b = kWsHeader + align_up((size_t)nR * sizeof(VRec));
    if (split > 1) b += align_up((size_t)split * (size_t)nQ * sizeof(float));
    return b;
}

size_t loss_ws(int64_t n) { return kWsHeader + align_up((size_t)loss_blocks(n) * sizeof(float)); }

// Morphing workspace: one region shared in turn by the forward, the loss and the
// adjoint (they run in order on one stream), then W, dL/dW, dL/dV and a loss slot.
struct MorphLayout {
    size_t sub, w, dldw, dldv, loss, total;
};

MorphLayout morph_layout(int64_t nV, int64_t nF, int64_t P) {
    MorphLayout l;
    size_t sub = voxelize_ws(3 * nF, P);
    sub = std::max(sub, naive_fwd_workspace(nF, P));
    sub = std::max(sub, bwd_workspace(nV, nF, P));
    sub = std::max(sub, loss_ws(P));
    l.sub = 0;
    l.w = align_up(sub);
    l.dldw = l.w + align_up((size_t)P * sizeof(float));
    l.dldv = l.dldw + align_up((size_t)P * sizeof(float));
    l.loss = l.dldv + align_up((size_t)nV * 3 * sizeof(float));
    l.total = l.loss + 256;
    return l;
}

}  // namespace

extern "C" {

size_t wn_workspace_size(int32_t op, int64_t nV, int64_t nF, int64_t nQ) {
    if (nV < 0 || nF < 0 || nQ < 0) return 0;
    switch (op) {
        case WN_OP_VOXELIZE:
            return voxelize_ws(3 * nF, nQ);
        case WN_OP_BACKWARD:
            return bwd_workspace(nV, nF, nQ);
        case WN_OP_LOSS:
            return kWsHeader + align_up((size_t)loss_blocks(nQ) * sizeof(float));
        case WN_OP_FLIP:
            return flip_workspace(nV, nF);
        case WN_OP_MORPH:
            if (nV > kMaxCount || nF > kMaxCount || nQ > kMaxCount) return 0;
            return morph_layout(nV, nF, nQ).total;
        case WN_OP_CUBIFY: {
            int64_t r = 0;
            while ((r + 1) * (r + 1) * (r + 1) <= nQ) ++r;
            if (r * r * r != nQ || nQ > kMaxCount) return 0;
            return cubify_workspace(nQ, (r + 1) * (r + 1) * (r + 1));
        }
        case WN_OP_SMOOTH:
            if (nV > kMaxCount || nF > kMaxCount / 6) return 0;
            return smooth_workspace(nV, nF);
        case WN_OP_SAMPLE:
            if (nF > kMaxCount || nQ > kMaxCount) return 0;
            return sample_workspace(nF);
        case WN_OP_NN:
            if (nV > kMaxCount || nF > kMaxCount) return 0;
            return nn_workspace(nV, nF);
        default:
            return 0;
    }
}

}  // extern "C"

namespace wn {

wn_status voxelize_impl(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *R, int64_t nR,
                        const wn_grid *grid, const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau,
                        float k, void *occ, void *ws, size_t ws_bytes, void *stream, const TuneConfig *force) {
    if (!mesh_ok(V, nV, F, nF)) return WN_ERR_INVALID_ARG;
    if (R == nullptr) {
        if (nR != 0) return WN_ERR_INVALID_ARG;
        nR = 3 * nF;
    } else if (nR < 0 || nR > kMaxCount || nF == 0) {
        return WN_ERR_INVALID_ARG;
    }
    const int64_t P = query_count(grid, Q, nQ);
    if (P < 0) return WN_ERR_INVALID_ARG;
    if (occ_mode != WN_OCC_NONE && occ_mode != WN_OCC_THRESHOLD && occ_mode != WN_OCC_SIGMOID)
        return WN_ERR_INVALID_ARG;
    if (P > 0 && W == nullptr) return WN_ERR_INVALID_ARG;
    if (P > 0 && occ_mode != WN_OCC_NONE && occ == nullptr) return WN_ERR_INVALID_ARG;
    if (grid)
        for (int d = 0; d < 3; ++d)
            if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    const size_t need = voxelize_ws(nR, P);
    if (ws == nullptr || !aligned256(ws) || ws_bytes < need) return WN_ERR_WORKSPACE;
    if (P == 0) return WN_OK;

    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(base);
    VRec *recs = reinterpret_cast<VRec *>(base + kWsHeader);
    float *partials = reinterpret_cast<float *>(base + kWsHeader + align_up((size_t)nR * sizeof(VRec)));
    const int split = fwd_split_count(nR, P);
    OccParams op{occ, occ_mode, tau, k};

    const TuneConfig cfg = force ? *force : lookup_config(WN_OP_VOXELIZE, nF, P);
    hipError_t e = launch_ws_reset(hdr, s);
    if (e == hipSuccess) e = launch_pack_records(V, nV, F, nF, R, nR, recs, hdr, s);
    if (e == hipSuccess)
        e = launch_fwd(recs, nR, make_point_src(grid, Q), P, split, W, partials, op, cfg.ppl, cfg.depth, s);
    return hip_status(e);
}

size_t voxelize_workspace(int64_t nR, int64_t nQ) { return voxelize_ws(nR, nQ); }

}  // namespace wn

extern "C" {

wn_status wn_voxelize(const float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                      const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau, float k, void *occ,
                      void *ws, size_t ws_bytes, void *stream) {
    return voxelize_impl(V, nV, F, nF, nullptr, 0, grid, Q, nQ, W, occ_mode, tau, k, occ, ws, ws_bytes, stream,
                         nullptr);
}

wn_status wn_voxelize_strips(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *strips,
                             int64_t n_records, const wn_grid *grid, const float *Q, int64_t nQ, float *W,
                             int32_t occ_mode, float tau, float k, void *occ, void *ws, size_t ws_bytes,
                             void *stream) {
    if (strips == nullptr) return WN_ERR_INVALID_ARG;
    return voxelize_impl(V, nV, F, nF, strips, n_records, grid, Q, nQ, W, occ_mode, tau, k, occ, ws, ws_bytes,
                         stream, nullptr);
}

wn_status wn_build_strips(const int32_t *F, int64_t nF, int64_t nV, int32_t *records, int64_t capacity,
                          int64_t *n_records) {
    if (n_records == nullptr || nF < 0 || nV < 0 || nF > kMaxCount || nV > kMaxCount) return WN_ERR_INVALID_ARG;
    if (nF > 0 && F == nullptr) return WN_ERR_INVALID_ARG;
    for (int64_t i = 0; i < 3 * nF; ++i)
        if (F[i] < 0 || (int64_t)F[i] >= nV) return WN_ERR_INVALID_ARG;
    std::vector<int32_t> out;
    const int64_t n = build_strips(F, nF, out);
    *n_records = n;
    if (records == nullptr) return WN_OK;
    if (capacity < n) return WN_ERR_WORKSPACE;
    if (n > 0) memcpy(records, out.data(), sizeof(int32_t) * 2 * (size_t)n);
    return WN_OK;
}

wn_status wn_build_face_pairs(const int32_t *F, int64_t nF, int64_t nV, int32_t *pairs, int64_t capacity,
                              int64_t *n_pairs) {
    if (n_pairs == nullptr || nF < 0 || nV < 0 || nF > kMaxCount || nV > kMaxCount) return WN_ERR_INVALID_ARG;
    if (nF > 0 && F == nullptr) return WN_ERR_INVALID_ARG;
    for (int64_t i = 0; i < 3 * nF; ++i)
        if (F[i] < 0 || (int64_t)F[i] >= nV) return WN_ERR_INVALID_ARG;
    std::vector<int32_t> out;
    const int64_t n = build_face_pairs(F, nF, out);
    *n_pairs = n;
    if (pairs == nullptr) return WN_OK;
    if (capacity < n) return WN_ERR_WORKSPACE;
    if (n > 0) memcpy(pairs, out.data(), sizeof(int32_t) * 2 * (size_t)n);
    return WN_OK;
}

wn_status wn_occupancy(const float *W, int64_t n, int32_t mode, float tau, float k, void *occ, void *stream) {
    if (n < 0) return WN_ERR_INVALID_ARG;
    if (mode != WN_OCC_THRESHOLD && mode != WN_OCC_SIGMOID) return WN_ERR_INVALID_ARG;
    if (n == 0) return WN_OK;
    if (W == nullptr || occ == nullptr) return WN_ERR_INVALID_ARG;
    OccParams op{occ, mode, tau, k};
    return hip_status(launch_occ(W, n, op, static_cast<hipStream_t>(stream)));
}

wn_status wn_occupancy_backward(const float *W, const float *g, int64_t n, float tau, float k, float *dLdW,
                                void *stream) {
    if (n < 0 || !std::isfinite(tau) || !std::isfinite(k)) return WN_ERR_INVALID_ARG;
    if (n == 0) return WN_OK;
    if (W == nullptr || g == nullptr || dLdW == nullptr) return WN_ERR_INVALID_ARG;
    return hip_status(launch_occ_bwd(W, g, n, tau, k, dLdW, static_cast<hipStream_t>(stream)));
}

wn_status wn_release_workspace(void *ws) {
    if (ws == nullptr) return WN_ERR_INVALID_ARG;
    return release_batched(ws);
}

wn_status wn_sigmoid_mse(const float *W, const float *target, int64_t n, float tau, float k, float *loss,
                         float *dLdW, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || n > kMaxCount) return WN_ERR_INVALID_ARG;
    if (n > 0 && (W == nullptr || target == nullptr)) return WN_ERR_INVALID_ARG;
    if (loss == nullptr && dLdW == nullptr) return WN_ERR_INVALID_ARG;
    const size_t need = kWsHeader + align_up((size_t)loss_blocks(n) * sizeof(float));
    if (ws == nullptr || !aligned256(ws) || ws_bytes < need) return WN_ERR_WORKSPACE;
    float *scratch = reinterpret_cast<float *>(static_cast<char *>(ws) + kWsHeader);
    return hip_status(launch_sigmoid_mse(W, target, n, tau, k, loss, dLdW, scratch, static_cast<hipStream_t>(stream)));
}

static_assert(kBwdBegin == WN_BWD_BEGIN && kBwdEnd == WN_BWD_END && kBwdVertexSums == WN_BWD_VERTEX_SUMS,
              "adjoint flags");

wn_status wn_backward_range(const float *V, int64_t nV, const int32_t *F, int64_t nF, const int32_t *pairs,
                            int64_t n_pairs, const wn_grid *grid, const float *Q, int64_t nQ, const float *dLdW,
                            int64_t p0, int64_t n, int32_t flags, float *dLdV, float *dLdT, void *ws,
                            size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF)) return WN_ERR_INVALID_ARG;
    if (pairs == nullptr ? n_pairs != 0 : (n_pairs < (nF + 1) / 2 || n_pairs > nF)) return WN_ERR_INVALID_ARG;
    const int64_t P = query_count(grid, Q, nQ);
    if (P < 0) return WN_ERR_INVALID_ARG;
    if (flags & ~(WN_BWD_BEGIN | WN_BWD_END | WN_BWD_VERTEX_SUMS)) return WN_ERR_INVALID_ARG;
    if ((flags & WN_BWD_VERTEX_SUMS) && (flags & WN_BWD_END) && dLdT != nullptr) return WN_ERR_INVALID_ARG;
    if (p0 < 0 || n < 0 || p0 > P || n > P - p0) return WN_ERR_INVALID_ARG;
    if (n > 0 && (p0 % WN_BWD_TILE != 0 || (p0 + n != P && n % WN_BWD_TILE != 0))) return WN_ERR_INVALID_ARG;
    if ((flags & WN_BWD_END) && nV > 0 && dLdV == nullptr) return WN_ERR_INVALID_ARG;
    if (n > 0 && nF > 0 && dLdW == nullptr) return WN_ERR_INVALID_ARG;
    if (grid)
        for (int d = 0; d < 3; ++d)
            if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    const size_t need = bwd_workspace(nV, nF, P);
    if (ws == nullptr || !aligned256(ws) || ws_bytes < need) return WN_ERR_WORKSPACE;
    return run_backward(V, nV, F, nF, pairs, n_pairs, make_point_src(grid, Q), P, dLdW, p0, n, flags, dLdV, dLdT,
                        static_cast<char *>(ws), ws_bytes, static_cast<hipStream_t>(stream));
}

wn_status wn_backward(const float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                      const float *Q, int64_t nQ, const float *dLdW, float *dLdV, float *dLdT, void *ws,
                      size_t ws_bytes, void *stream) {
    const int64_t P = query_count(grid, Q, nQ);
    return wn_backward_range(V, nV, F, nF, nullptr, 0, grid, Q, nQ, dLdW, 0, P < 0 ? 0 : P, WN_BWD_BEGIN | WN_BWD_END,
                             dLdV, dLdT, ws, ws_bytes, stream);
}

int64_t wn_backward_splits(int64_t nF, int64_t nQ) {
    if (nF < 0 || nQ < 0 || nF > kMaxCount || nQ > kMaxCount) return -1;
    return bwd_splits(nF, nQ);
}

}  // extern "C"

namespace {

wn_status naive_impl(const float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid, const float *Q,
                     int64_t nQ, float *W, int32_t occ_mode, float tau, float k, void *occ, void *ws, size_t ws_bytes,
                     void *stream, const TuneConfig *force) {
    if (!mesh_ok(V, nV, F, nF)) return WN_ERR_INVALID_ARG;
    const int64_t P = query_count(grid, Q, nQ);
    if (P < 0) return WN_ERR_INVALID_ARG;
    if (occ_mode != WN_OCC_NONE && occ_mode != WN_OCC_THRESHOLD && occ_mode != WN_OCC_SIGMOID)
        return WN_ERR_INVALID_ARG;
    if (P > 0 && W == nullptr) return WN_ERR_INVALID_ARG;
    if (P > 0 && occ_mode != WN_OCC_NONE && occ == nullptr) return WN_ERR_INVALID_ARG;
    if (grid)
        for (int d = 0; d < 3; ++d)
            if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < naive_fwd_workspace(nF, P)) return WN_ERR_WORKSPACE;
    if (P == 0) return WN_OK;
    OccParams op{occ, occ_mode, tau, k};
    const int ppl = (force ? *force : lookup_config(WN_OP_NAIVE, nF, P)).ppl;
    return hip_status(launch_naive_fwd(V, nV, F, nF, make_point_src(grid, Q), P, W, op, static_cast<char *>(ws), ppl,
                                       static_cast<hipStream_t>(stream)));
}

}  // namespace

extern "C" {

wn_status wn_voxelize_naive(const float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                            const float *Q, int64_t nQ, float *W, int32_t occ_mode, float tau, float k, void *occ,
                            void *ws, size_t ws_bytes, void *stream) {
    return naive_impl(V, nV, F, nF, grid, Q, nQ, W, occ_mode, tau, k, occ, ws, ws_bytes, stream, nullptr);
}

wn_status wn_backward_naive(const float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                            const float *Q, int64_t nQ, const float *dLdW, float *dLdV, float *dLdT, void *ws,
                            size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF)) return WN_ERR_INVALID_ARG;
    const int64_t P = query_count(grid, Q, nQ);
    if (P < 0) return WN_ERR_INVALID_ARG;
    if (nV > 0 && dLdV == nullptr) return WN_ERR_INVALID_ARG;
    if (P > 0 && nF > 0 && dLdW == nullptr) return WN_ERR_INVALID_ARG;
    if (grid)
        for (int d = 0; d < 3; ++d)
            if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    const size_t need = bwd_workspace(nV, nF, P);
    if (ws == nullptr || !aligned256(ws) || ws_bytes < need) return WN_ERR_WORKSPACE;
    return run_backward(V, nV, F, nF, make_point_src(grid, Q), P, dLdW, dLdV, dLdT, static_cast<char *>(ws),
                        ws_bytes, static_cast<hipStream_t>(stream), true);
}

wn_status wn_voxelize_batched(const wn_mesh_desc *desc, int32_t n, int32_t flags, void *ws, size_t ws_bytes,
                              void *stream) {
    if (n < 0 || (n > 0 && desc == nullptr)) return WN_ERR_INVALID_ARG;
    if (flags & ~WN_BATCH_NO_GRAPH) return WN_ERR_INVALID_ARG;
    if (n == 0) return WN_OK;
    if (ws == nullptr || !aligned256(ws)) return WN_ERR_WORKSPACE;
    return run_batched(desc, n, flags, static_cast<char *>(ws), ws_bytes, static_cast<hipStream_t>(stream), nullptr);
}

size_t wn_workspace_size_batched(const wn_mesh_desc *desc, int32_t n) {
    if (n < 0 || (n > 0 && desc == nullptr)) return 0;
    return batched_workspace(desc, n);
}

wn_status wn_autotune(int32_t op, const wn_mesh_desc *desc, int32_t n, void *ws, size_t ws_bytes, void *stream,
                      char *report, size_t report_len) {
    if (desc == nullptr || n < 1) return WN_ERR_INVALID_ARG;
    if (op != WN_OP_VOXELIZE && op != WN_OP_BATCHED && op != WN_OP_NAIVE) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws)) return WN_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    std::vector<TuneConfig> cands;
    for (int ppl : {1, 2, 4})
        for (int depth : {1, 2, 4})
            if (op != WN_OP_NAIVE || depth == 1) cands.push_back(TuneConfig{ppl, 0, depth});
    int64_t a = 0, b = 0;
    if (op == WN_OP_VOXELIZE || op == WN_OP_NAIVE) {
        a = desc[0].nF;
        b = (int64_t)desc[0].grid.n[0] * desc[0].grid.n[1] * desc[0].grid.n[2];
    } else {
        for (int32_t m = 0; m < n; ++m)
            a += desc[m].nF * (desc[m].point_count > 0
                                   ? desc[m].point_count
                                   : (int64_t)desc[m].grid.n[0] * desc[m].grid.n[1] * desc[m].grid.n[2]);
        b = n;
    }
    auto run = [&](const TuneConfig &c) -> wn_status {
        if (op == WN_OP_NAIVE) {
            const wn_mesh_desc &d = desc[0];
            return naive_impl(d.V, d.nV, d.F, d.nF, &d.grid, nullptr, 0, d.W, d.occ_mode, d.tau, d.k, d.occ, ws,
                              ws_bytes, stream, &c);
        }
        if (op == WN_OP_VOXELIZE) {
            const wn_mesh_desc &d = desc[0];
            return voxelize_impl(d.V, d.nV, d.F, d.nF, d.strips, d.strips ? d.n_strip_records : 0, &d.grid, nullptr,
                                 0, d.W, d.occ_mode, d.tau, d.k, d.occ, ws, ws_bytes, stream, &c);
        }
        return run_batched(desc, n, WN_BATCH_NO_GRAPH, static_cast<char *>(ws), ws_bytes, s, &c);
    };
    // Every candidate's outputs are checksummed (sum of the bit patterns of W), so the
    // report shows whether any configuration changed a result.
    auto checksum = [&](unsigned long long &out) -> wn_status {
        bool reset = true;
        for (int32_t m = 0; m < (op == WN_OP_BATCHED ? n : 1); ++m) {
            const wn_mesh_desc &d = desc[m];
            const int64_t P = (int64_t)d.grid.n[0] * d.grid.n[1] * d.grid.n[2];
            if (launch_checksum(d.W, P, hdr, reset, s) != hipSuccess) return WN_ERR_HIP;
            reset = false;
        }
        if (hipMemcpyAsync(&out, &hdr->checksum, sizeof out, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return WN_ERR_HIP;
        return WN_OK;
    };
    const int reps = op == WN_OP_BATCHED ? 1 : 2;  // a batch is long enough to time once
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return WN_ERR_HIP;
    std::string rep = "{\"op\": " + std::to_string(op) + ", \"candidates\": [";
    float best_ms = 0.0f;
    TuneConfig best = cands[0];
    wn_status st = WN_OK;
    bool identical = true;
    unsigned long long first_sum = 0;
    auto time_one = [&](const TuneConfig &c, size_t i) -> wn_status {
        wn_status r = run(c);  // warm-up (and code-object load)
        if (r != WN_OK) return r;
        unsigned long long sum = 0;
        if ((r = checksum(sum)) != WN_OK) return r;
        if (i == 0) first_sum = sum;
        identical = identical && sum == first_sum;
        if (hipEventRecord(e0, s) != hipSuccess) return WN_ERR_HIP;
        for (int k = 0; k < reps && r == WN_OK; ++k) r = run(c);
        if (r != WN_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return WN_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return WN_ERR_HIP;
        ms /= (float)reps;
        char buf[160];
        snprintf(buf, sizeof buf, "%s{\"ppl\": %d, \"wg\": %d, \"depth\": %d, \"ms\": %.4f, \"checksum\": %llu}",
                 i ? ", " : "", c.ppl, c.wg_per_cu, c.depth, ms, sum);
        rep += buf;
        if (i == 0 || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        return WN_OK;
    };
    for (size_t i = 0; i < cands.size() && st == WN_OK; ++i) st = time_one(cands[i], i);
    // for a batch, also try the fastest mapping with fewer persistent workgroups per CU
    if (st == WN_OK && op == WN_OP_BATCHED) st = time_one(TuneConfig{best.ppl, 2, best.depth}, cands.size());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != WN_OK) return st;
    store_config(op, a, b, best);
    char buf[192];
    snprintf(buf, sizeof buf, "], \"chosen\": {\"ppl\": %d, \"wg\": %d, \"depth\": %d, \"ms\": %.4f}, \"identical\": %s}",
             best.ppl, best.wg_per_cu, best.depth, best_ms, identical ? "true" : "false");
    rep += buf;
    if (report && report_len > 0) {
        strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return WN_OK;
}

wn_status wn_flip_duplicate(const float *V, int64_t nV, const int32_t *F, int64_t nF, float eps, float *V2,
                            int32_t *F2, void *ws, size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF)) return WN_ERR_INVALID_ARG;
    if (2 * nV > kMaxCount || 2 * nF > kMaxCount) return WN_ERR_INVALID_ARG;
    if (nV > 0 && V2 == nullptr) return WN_ERR_INVALID_ARG;
    if (nF > 0 && F2 == nullptr) return WN_ERR_INVALID_ARG;
    if (!(eps == eps)) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < flip_workspace(nV, nF)) return WN_ERR_WORKSPACE;
    return run_flip(V, nV, F, nF, eps, V2, F2, static_cast<char *>(ws), ws_bytes, static_cast<hipStream_t>(stream));
}

wn_status wn_adam(float *x, const float *g, float *m, float *v, int64_t n, int64_t t, float lr, float beta1,
                  float beta2, float eps, void *stream) {
    if (n < 0 || t < 1) return WN_ERR_INVALID_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && std::isfinite(lr)))
        return WN_ERR_INVALID_ARG;
    if (n == 0) return WN_OK;
    if (!x || !g || !m || !v) return WN_ERR_INVALID_ARG;
    return hip_status(launch_adam(x, g, m, v, n, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
}

wn_status wn_morph_step(float *V, int64_t nV, const int32_t *F, int64_t nF, const wn_grid *grid,
                        const float *target, int32_t integral, float tau, float k, float lr, float beta1,
                        float beta2, float eps, int64_t t0, int32_t iters, float *m, float *v, float *loss_history,
                        void *ws, size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF) || grid == nullptr) return WN_ERR_INVALID_ARG;
    if (integral != WN_INTEGRAL_GWN && integral != WN_INTEGRAL_NAIVE) return WN_ERR_INVALID_ARG;
    if (iters < 0 || t0 < 0 || t0 > kMaxCount) return WN_ERR_INVALID_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && std::isfinite(lr)))
        return WN_ERR_INVALID_ARG;
    const int64_t P = query_count(grid, nullptr, 0);
    if (P < 0) return WN_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    if (P > 0 && target == nullptr) return WN_ERR_INVALID_ARG;
    if (nV > 0 && (m == nullptr || v == nullptr)) return WN_ERR_INVALID_ARG;
    const MorphLayout l = morph_layout(nV, nF, P);
    if (ws == nullptr || !aligned256(ws) || ws_bytes < l.total) return WN_ERR_WORKSPACE;
    if (iters == 0) return WN_OK;

    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    char *sub = base + l.sub;
    const size_t sub_bytes = l.w - l.sub;
    float *W = reinterpret_cast<float *>(base + l.w);
    float *dLdW = reinterpret_cast<float *>(base + l.dldw);
    float *dLdV = reinterpret_cast<float *>(base + l.dldv);
    float *loss_slot = reinterpret_cast<float *>(base + l.loss);
    const PointSrc ps = make_point_src(grid, nullptr);
    const int ppl = lookup_config(WN_OP_NAIVE, nF, P).ppl;
    const bool naive = integral == WN_INTEGRAL_NAIVE;
    for (int32_t it = 0; it < iters; ++it) {
        wn_status st = WN_OK;
        if (P > 0) {
            if (naive) {
                OccParams none{nullptr, WN_OCC_NONE, tau, k};
                st = hip_status(launch_naive_fwd(V, nV, F, nF, ps, P, W, none, sub, ppl, s));
            } else {
                st = voxelize_impl(V, nV, F, nF, nullptr, 0, grid, nullptr, 0, W, WN_OCC_NONE, tau, k, nullptr, sub,
                                   sub_bytes, stream, nullptr);
            }
            if (st != WN_OK) return st;
        }
        float *loss = loss_history ? loss_history + it : loss_slot;
        float *scratch = reinterpret_cast<float *>(sub + kWsHeader);
        st = hip_status(launch_sigmoid_mse(W, target, P, tau, k, loss, dLdW, scratch, s));
        if (st != WN_OK) return st;
        st = run_backward(V, nV, F, nF, ps, P, dLdW, dLdV, nullptr, sub, sub_bytes, s, naive);
        if (st != WN_OK) return st;
        st = hip_status(launch_adam(V, dLdV, m, v, 3 * nV, t0 + 1 + it, lr, beta1, beta2, eps, s));
        if (st != WN_OK) return st;
    }
    return WN_OK;
}

size_t wn_workspace_size_cubify(const wn_grid *grid) {
    if (!grid) return 0;
    int64_t P = 1, C = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 0) return 0;
        P *= grid->n[d];
        C *= (int64_t)grid->n[d] + 1;
    }
    if (P > kMaxCount || C > kMaxCount) return 0;
    return cubify_workspace(P, C);
}

wn_status wn_cubify(const uint8_t *occ, const wn_grid *grid, float *V, int64_t capV, int32_t *F, int64_t capF,
                    int64_t *counts, void *ws, size_t ws_bytes, void *stream) {
    if (grid == nullptr || counts == nullptr || capV < 0 || capF < 0) return WN_ERR_INVALID_ARG;
    const size_t need = wn_workspace_size_cubify(grid);
    if (need == 0) return WN_ERR_INVALID_ARG;
    const int64_t P = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    if (P > 0 && occ == nullptr) return WN_ERR_INVALID_ARG;
    if ((capV > 0 && V == nullptr) || (capF > 0 && F == nullptr)) return WN_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (grid->n[d] > 0 && !(grid->hi[d] > grid->lo[d])) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < need) return WN_ERR_WORKSPACE;
    return run_cubify(occ, grid->n, grid->lo, grid->hi, V, capV, F, capF, counts, static_cast<char *>(ws),
                      static_cast<hipStream_t>(stream));
}

wn_status wn_laplacian_smooth(const float *V, int64_t nV, const int32_t *F, int64_t nF, float lam, int32_t iters,
                              int32_t keep_volume, float *Vout, void *ws, size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF) || nF > kMaxCount / 6 || iters < 0 || !std::isfinite(lam)) return WN_ERR_INVALID_ARG;
    if (keep_volume != 0 && keep_volume != 1) return WN_ERR_INVALID_ARG;
    if (nV > 0 && (Vout == nullptr || Vout == V)) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < smooth_workspace(nV, nF)) return WN_ERR_WORKSPACE;
    return run_smooth(V, nV, F, nF, lam, iters, keep_volume, Vout, static_cast<char *>(ws),
                      static_cast<hipStream_t>(stream));
}

wn_status wn_sample_surface(const float *V, int64_t nV, const int32_t *F, int64_t nF, const double *u, int64_t n,
                            float *P, int32_t *face, void *ws, size_t ws_bytes, void *stream) {
    if (!mesh_ok(V, nV, F, nF) || n < 0 || n > kMaxCount) return WN_ERR_INVALID_ARG;
    if (n > 0 && (nF == 0 || u == nullptr || P == nullptr || face == nullptr)) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < sample_workspace(nF)) return WN_ERR_WORKSPACE;
    return run_sample(V, nV, F, nF, u, n, P, face, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
}

wn_status wn_nn_distance(const float *A, int64_t nA, const float *B, int64_t nB, float *d, void *ws,
                         size_t ws_bytes, void *stream) {
    if (nA < 0 || nB < 0 || nA > kMaxCount || nB > kMaxCount) return WN_ERR_INVALID_ARG;
    if (nA > 0 && (A == nullptr || d == nullptr || nB == 0 || B == nullptr)) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < nn_workspace(nA, nB)) return WN_ERR_WORKSPACE;
    return run_nn(A, nA, B, nB, d, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
}

wn_status wn_chamfer_hausdorff(const float *A, int64_t nA, const float *B, int64_t nB, double *out, void *ws,
                               size_t ws_bytes, void *stream) {
    if (nA <= 0 || nB <= 0 || nA > kMaxCount || nB > kMaxCount) return WN_ERR_INVALID_ARG;
    if (A == nullptr || B == nullptr || out == nullptr) return WN_ERR_INVALID_ARG;
    if (ws == nullptr || !aligned256(ws) || ws_bytes < nn_workspace(nA, nB)) return WN_ERR_WORKSPACE;
    return run_chamfer(A, nA, B, nB, out, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
}

wn_status wn_get_device_error(void *ws, void *stream) {
    if (ws == nullptr) {  // the record of wn_voxelize_strips_noalloc on the current device
        const wn_status st = noalloc_header(&ws);
        if (st != WN_OK) return st;
    }
    if (!aligned256(ws)) return WN_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    WsHeader *hdr = static_cast<WsHeader *>(ws);
    int32_t flag = 0;
    if (hipMemcpyAsync(&flag, &hdr->bad_index, sizeof(flag), hipMemcpyDeviceToHost, s) != hipSuccess)
        return WN_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return WN_ERR_HIP;
    if (flag != 0) {
        if (launch_ws_reset(hdr, s) != hipSuccess) return WN_ERR_HIP;
        return WN_ERR_BAD_INDEX;
    }
    return WN_OK;
}

const char *wn_status_string(wn_status st) {
    switch (st) {
        case WN_OK:
            return "ok";
        case WN_ERR_INVALID_ARG:
            return "invalid argument";
        case WN_ERR_HIP:
            return "HIP runtime error";
        case WN_ERR_WORKSPACE:
            return "workspace missing, misaligned or too small";
        case WN_ERR_BAD_INDEX:
            return "face index out of range (replaced by 0 on the device)";
        case WN_ERR_UNSUPPORTED:
            return "unsupported";
        default:
            return "unknown status";
    }
}

const char *wn_version(void) { return "wn-gfx950 0.1"; }

}  // extern "C"
