// Batched forward: many meshes of uneven face count and grid size in one
// persistent launch.
//
// The cost of a mesh is points x faces (the paper observes time linear in the face
// count and cubic in the resolution), so work is cut into units of one point block
// (kBlock * PPL voxel centres) against one chunk of the mesh's vertex-record stream
// (kChunkRecords records; see wn_internal.hpp).  Units of the same (mesh, chunk) form a
// group; groups are ordered by chunk size, largest first, and persistent workgroups take units from a device cursor until none are
// left.  A mesh with several chunks writes per-chunk partial sums to fixed slots and
// a reduction adds them in chunk order, so each mesh's result depends only on its own
// record stream -- never on the rest of the batch or on the launch configuration.
//
// Everything the kernels need (mesh table, groups, offsets) lives in the workspace,
// copied there from a pinned staging buffer before each launch; the kernels take only
// the workspace pointer, so the launch sequence is captured once per workspace as a
// HIP graph and replayed for every batch.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "wn_internal.hpp"

namespace wn {

constexpr int64_t kChunkRecords = 4080;  // records per work unit (a multiple of kRecTile)
static_assert(kChunkRecords % kRecTile == 0, "chunk must hold whole tiles");

struct BMesh {
    const float *V;
    const int32_t *F;
    const int32_t *R;   // strip stream or nullptr (three records per face)
    float *W;
    void *occ;
    int64_t nV;
    int64_t p0;         // first flat voxel index of this slice
    int64_t P;          // voxels in this slice
    int64_t nR;         // records of this mesh
    int64_t rec_off;    // first record of this mesh in the batch stream
    int64_t part_off;   // first partial-sum float of this mesh (chunks > 1)
    PointSrc ps;
    int32_t nF;
    int32_t chunks;
    int32_t pblocks;
    int32_t occ_mode;
    float tau;
    float k;
};

struct BGroup {
    int64_t unit_begin;  // units [unit_begin, next group's unit_begin)
    int32_t mesh;
    int32_t chunk;
};

struct BatchHeader {
    int64_t n_units;
    int64_t total_records;
    int64_t total_reduce_points;
    int64_t off_meshes, off_groups, off_face_prefix, off_reduce_ids, off_reduce_prefix, off_soup, off_part;
    int32_t n_meshes;
    int32_t n_groups;
    int32_t n_reduce;
    int32_t ppl;
};

__device__ __forceinline__ const BatchHeader *bheader(const char *ws) {
    return reinterpret_cast<const BatchHeader *>(ws + kWsHeader);
}

// Largest i in [0, n) with prefix[i] <= x (prefix ascending, prefix[0] <= x).
template <typename T>
__device__ __forceinline__ int32_t upper_index(const T *prefix, int32_t n, T x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t upper_index_group(const BGroup *g, int32_t n, int64_t u) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (g[mid].unit_begin <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Vertex records of every mesh into one stream (same record rule as k_pack_records).
__global__ __launch_bounds__(kBlock) void k_batched_pack(char *ws) {
    const BatchHeader *bh = bheader(ws);
    const BMesh *meshes = reinterpret_cast<const BMesh *>(ws + bh->off_meshes);
    const int64_t *rpre = reinterpret_cast<const int64_t *>(ws + bh->off_face_prefix);
    VRec *recs = reinterpret_cast<VRec *>(ws + bh->off_soup);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    const int64_t total = bh->total_records;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = upper_index(rpre, bh->n_meshes, g);
        const BMesh &mh = meshes[m];
        const int64_t r = g - rpre[m];
        int32_t vid, fid;
        if (mh.R) {
            vid = mh.R[2 * r];
            fid = mh.R[2 * r + 1];
            check_strip_record(mh.R, r, mh.F, mh.nF, fid, hdr);
        } else {
            const int64_t f = r / 3;
            const int j = (int)(r - 3 * f);
            vid = mh.F[3 * f + j];
            fid = j == 2 ? (int32_t)f : -1;
        }
        recs[g] = make_record(mh.V, mh.nV, mh.F, mh.nF, vid, fid, hdr);
    }
}

// Persistent workgroups: take units from the cursor until the list is exhausted.
template <int PPL, int DEPTH>
__global__ __launch_bounds__(kBlock) void k_batched_persistent(char *ws) {
    __shared__ float4 tile[kRecTile * 2 * DEPTH];
    __shared__ int64_t s_unit;
    __shared__ int32_t s_group;
    const BatchHeader *bh = bheader(ws);
    const BMesh *meshes = reinterpret_cast<const BMesh *>(ws + bh->off_meshes);
    const BGroup *groups = reinterpret_cast<const BGroup *>(ws + bh->off_groups);
    const float4 *recs = reinterpret_cast<const float4 *>(ws + bh->off_soup);
    float *part = reinterpret_cast<float *>(ws + bh->off_part);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    const int64_t n_units = bh->n_units;
    const int32_t n_groups = bh->n_groups;
    const int tid = threadIdx.x;
    for (;;) {
        __syncthreads();  // the previous unit's tile reads and s_* reads are done
        if (tid == 0) {
            const int64_t u = (int64_t)atomicAdd(&hdr->cursor, 1ull);
            s_unit = u;
            s_group = u < n_units ? upper_index_group(groups, n_groups, u) : -1;
        }
        __syncthreads();
        const int64_t u = s_unit;
        if (u >= n_units) break;
        const BGroup gr = groups[s_group];
        const BMesh &mh = meshes[gr.mesh];
        const int64_t pblock = u - gr.unit_begin;
        const int64_t base = pblock * (kBlock * PPL) + tid;
        const int64_t r0 = (int64_t)gr.chunk * kChunkRecords;
        const int64_t r1 = min(mh.nR, r0 + kChunkRecords);
        float qx[PPL], qy[PPL], qz[PPL], s[PPL], c[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int64_t idx = base + (int64_t)p * kBlock;
            idx = idx < mh.P ? idx : mh.P - 1;
            mh.ps.get(mh.p0 + idx, qx[p], qy[p], qz[p]);
            s[p] = 0.0f;
            c[p] = 0.0f;
        }
        sum_records<PPL, DEPTH>(recs + 2 * mh.rec_off, r0, r1, tile, qx, qy, qz, s, c);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int64_t idx = base + (int64_t)p * kBlock;
            if (idx >= mh.P) continue;
            const float tot = s[p] + c[p];
            if (mh.chunks > 1) {
                part[mh.part_off + (int64_t)gr.chunk * mh.P + idx] = tot;
            } else {
                const float w = tot * kInv2Pi;
                mh.W[mh.p0 + idx] = w;
                write_occ(OccParams{mh.occ, mh.occ_mode, mh.tau, mh.k}, mh.p0 + idx, w);
            }
        }
    }
}

// Fixed-order sum of the chunk partials of every multi-chunk mesh, then occupancy.
__global__ __launch_bounds__(kBlock) void k_batched_reduce(char *ws) {
    const BatchHeader *bh = bheader(ws);
    const BMesh *meshes = reinterpret_cast<const BMesh *>(ws + bh->off_meshes);
    const int32_t *rids = reinterpret_cast<const int32_t *>(ws + bh->off_reduce_ids);
    const int64_t *rpre = reinterpret_cast<const int64_t *>(ws + bh->off_reduce_prefix);
    const float *part = reinterpret_cast<const float *>(ws + bh->off_part);
    const int64_t total = bh->total_reduce_points;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = upper_index(rpre, bh->n_reduce, g);
        const BMesh &mh = meshes[rids[r]];
        const int64_t idx = g - rpre[r];
        float s = 0.0f, c = 0.0f;
        for (int32_t k = 0; k < mh.chunks; ++k) neumaier_add(s, c, part[mh.part_off + (int64_t)k * mh.P + idx]);
        const float w = (s + c) * kInv2Pi;
        mh.W[mh.p0 + idx] = w;
        write_occ(OccParams{mh.occ, mh.occ_mode, mh.tau, mh.k}, mh.p0 + idx, w);
    }
}

// ------------------------------------------------------------------ host

namespace {

struct Plan {
    std::vector<char> tables;  // BatchHeader + tables, copied to ws + kWsHeader
    size_t total_bytes = 0;    // workspace bytes needed
    int64_t n_units = 0;
    int64_t total_faces = 0;
    int64_t total_reduce = 0;
};

bool desc_ok(const wn_mesh_desc &d) {
    if (d.nV < 0 || d.nF < 0 || d.nV > 2147483647LL || d.nF > 2147483647LL) return false;
    if (d.nF > 0 && (d.V == nullptr || d.F == nullptr || d.nV == 0)) return false;
    if (d.strips == nullptr ? d.n_strip_records != 0
                            : (d.n_strip_records < 0 || d.n_strip_records > 2147483647LL || d.nF == 0))
        return false;
    int64_t p = 1;
    for (int k = 0; k < 3; ++k) {
        if (d.grid.n[k] < 1) return false;
        if (!(d.grid.hi[k] > d.grid.lo[k])) return false;
        p *= d.grid.n[k];
        if (p > 2147483647LL) return false;
    }
    if (d.W == nullptr) return false;
    if (d.point_begin < 0 || d.point_count < 0 || d.point_begin > p) return false;
    if (d.point_count > p - d.point_begin) return false;
    if (d.point_count == 0 && d.point_begin == p) return false;  // empty slice
    if (d.occ_mode != WN_OCC_NONE && d.occ_mode != WN_OCC_THRESHOLD && d.occ_mode != WN_OCC_SIGMOID) return false;
    if (d.occ_mode != WN_OCC_NONE && d.occ == nullptr) return false;
    return true;
}

size_t tables_layout(int32_t n, int32_t n_groups, int32_t n_reduce, BatchHeader &h) {
    size_t o = align_up(sizeof(BatchHeader), 64);
    h.off_meshes = kWsHeader + o;
    o += align_up(sizeof(BMesh) * (size_t)n, 64);
    h.off_groups = kWsHeader + o;
    o += align_up(sizeof(BGroup) * (size_t)n_groups, 64);
    h.off_face_prefix = kWsHeader + o;
    o += align_up(sizeof(int64_t) * (size_t)(n + 1), 64);
    h.off_reduce_ids = kWsHeader + o;
    o += align_up(sizeof(int32_t) * (size_t)(n_reduce + 1), 64);
    h.off_reduce_prefix = kWsHeader + o;
    o += align_up(sizeof(int64_t) * (size_t)(n_reduce + 1), 64);
    return o;
}

int64_t mesh_records(const wn_mesh_desc &d) { return d.strips ? d.n_strip_records : 3 * d.nF; }

int32_t mesh_chunks(int64_t nR) { return nR > 0 ? (int32_t)((nR + kChunkRecords - 1) / kChunkRecords) : 1; }

// Build the tables; ppl only changes the unit count, not any result.
bool make_plan(const wn_mesh_desc *d, int32_t n, int32_t ppl, Plan &plan) {
    std::vector<BMesh> meshes((size_t)n);
    struct G {
        int32_t faces, mesh, chunk;
        int64_t units;
    };
    std::vector<G> gs;
    std::vector<int32_t> rids;
    std::vector<int64_t> fpre((size_t)n + 1, 0), rpre(1, 0);
    int64_t part = 0;
    for (int32_t m = 0; m < n; ++m) {
        if (!desc_ok(d[m])) return false;
        BMesh &b = meshes[(size_t)m];
        memset(&b, 0, sizeof b);
        b.V = d[m].V;
        b.F = d[m].F;
        b.W = d[m].W;
        b.occ = d[m].occ_mode == WN_OCC_NONE ? nullptr : d[m].occ;
        b.nV = d[m].nV;
        const int64_t full = (int64_t)d[m].grid.n[0] * d[m].grid.n[1] * d[m].grid.n[2];
        b.p0 = d[m].point_begin;
        b.P = d[m].point_count > 0 ? d[m].point_count : full - d[m].point_begin;
        b.R = d[m].strips;
        b.nR = mesh_records(d[m]);
        b.rec_off = fpre[(size_t)m];
        b.ps = make_point_src(&d[m].grid, nullptr);
        b.nF = (int32_t)d[m].nF;
        b.chunks = mesh_chunks(b.nR);
        b.pblocks = (int32_t)((b.P + kBlock * ppl - 1) / (kBlock * ppl));
        b.occ_mode = d[m].occ_mode;
        b.tau = d[m].tau;
        b.k = d[m].k;
        fpre[(size_t)m + 1] = fpre[(size_t)m] + b.nR;
        if (b.chunks > 1) {
            b.part_off = part;
            part += (int64_t)b.chunks * b.P;
            rids.push_back(m);
            rpre.push_back(rpre.back() + b.P);
        }
        for (int32_t c = 0; c < b.chunks; ++c) {
            const int32_t faces = (int32_t)std::min<int64_t>(kChunkRecords, b.nR - (int64_t)c * kChunkRecords);
            gs.push_back(G{faces, m, c, b.pblocks});
        }
    }
    // Largest units first (longest-processing-time order); ties in table order.
    std::stable_sort(gs.begin(), gs.end(), [](const G &a, const G &b) { return a.faces > b.faces; });
    std::vector<BGroup> groups(gs.size());
    int64_t units = 0;
    for (size_t i = 0; i < gs.size(); ++i) {
        groups[i] = BGroup{units, gs[i].mesh, gs[i].chunk};
        units += gs[i].units;
    }
    if (rids.empty()) rids.push_back(0);  // keep the tables non-empty; n_reduce stays 0
    BatchHeader h;
    memset(&h, 0, sizeof h);
    const int32_t n_reduce = (int32_t)rpre.size() - 1;
    const size_t tbytes = tables_layout(n, (int32_t)groups.size(), n_reduce, h);
    h.n_units = units;
    h.total_records = fpre[(size_t)n];
    h.total_reduce_points = rpre.back();
    h.n_meshes = n;
    h.n_groups = (int32_t)groups.size();
    h.n_reduce = n_reduce;
    h.ppl = ppl;
    h.off_soup = (int64_t)align_up(kWsHeader + tbytes);
    h.off_part = h.off_soup + (int64_t)align_up((size_t)h.total_records * sizeof(VRec));
    plan.total_bytes = (size_t)h.off_part + align_up((size_t)part * sizeof(float));
    plan.n_units = units;
    plan.total_faces = h.total_records;
    plan.total_reduce = h.total_reduce_points;
    plan.tables.assign(tbytes, 0);
    char *t = plan.tables.data();
    memcpy(t, &h, sizeof h);
    memcpy(t + (h.off_meshes - kWsHeader), meshes.data(), sizeof(BMesh) * meshes.size());
    memcpy(t + (h.off_groups - kWsHeader), groups.data(), sizeof(BGroup) * groups.size());
    memcpy(t + (h.off_face_prefix - kWsHeader), fpre.data(), sizeof(int64_t) * fpre.size());
    memcpy(t + (h.off_reduce_ids - kWsHeader), rids.data(), sizeof(int32_t) * rids.size());
    memcpy(t + (h.off_reduce_prefix - kWsHeader), rpre.data(), sizeof(int64_t) * rpre.size());
    return true;
}

// Per-workspace host state: a ring of pinned staging buffers for the tables, each with
// the event recorded after its copy, and the captured graphs.  A call takes a buffer
// whose copy has finished (hipEventQuery), or adds one to the ring, so it never waits on
// the host for an earlier call's copy.
struct Staging {
    void *buf = nullptr;
    size_t cap = 0;
    hipEvent_t copied = nullptr;
};

struct WsState {
    std::vector<Staging> ring;
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;  // (ppl, depth, persistent grid, device)
};

constexpr size_t kMaxStaging = 64;  // buffers per workspace ring

std::mutex g_mu;
std::map<const void *, WsState> g_state;
hipStream_t g_capture = nullptr;

int persistent_grid(int ppl, int depth, int wg_per_cu) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = with_config(ppl, depth, [&](auto P, auto D) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, k_batched_persistent<decltype(P)::value, decltype(D)::value>, kBlock, 0);
    });
    if (e != hipSuccess || per < 1) per = 1;
    if (wg_per_cu > 0 && wg_per_cu < per) per = wg_per_cu;
    return cus * per;
}

hipError_t enqueue_kernels(char *ws, int ppl, int depth, int grid, hipStream_t s) {
    hipError_t e = launch_ws_reset(reinterpret_cast<WsHeader *>(ws), s);
    if (e != hipSuccess) return e;
    k_batched_pack<<<1024, kBlock, 0, s>>>(ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = with_config(ppl, depth, [&](auto P, auto D) {
        k_batched_persistent<decltype(P)::value, decltype(D)::value><<<grid, kBlock, 0, s>>>(ws);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_batched_reduce<<<2048, kBlock, 0, s>>>(ws);
    return hipGetLastError();
}

}  // namespace

size_t batched_workspace(const wn_mesh_desc *d, int32_t n) {
    Plan p;
    if (n <= 0 || d == nullptr) return kWsHeader;
    if (!make_plan(d, n, 1, p)) return 0;
    return p.total_bytes;
}

wn_status run_batched(const wn_mesh_desc *d, int32_t n, int32_t flags, char *ws, size_t ws_bytes, hipStream_t s,
                      const TuneConfig *force) {
    int64_t tot_pairs = 0;
    for (int32_t m = 0; m < n; ++m) {
        tot_pairs += d[m].nF * (d[m].point_count > 0 ? d[m].point_count
                                                        : (int64_t)d[m].grid.n[0] * d[m].grid.n[1] * d[m].grid.n[2]);
    }
    const TuneConfig cfg = force ? *force : lookup_config(WN_OP_BATCHED, tot_pairs, n);
    const int ppl = valid_ppl(cfg.ppl) ? cfg.ppl : 1;
    const int depth = valid_depth(cfg.depth) ? cfg.depth : 1;
    Plan plan;
    if (!make_plan(d, n, ppl, plan)) return WN_ERR_INVALID_ARG;
    if (ws_bytes < plan.total_bytes) return WN_ERR_WORKSPACE;
    if (plan.n_units > (int64_t)1 << 40) return WN_ERR_UNSUPPORTED;
    const int grid = persistent_grid(ppl, depth, cfg.wg_per_cu);
    if (grid <= 0) return WN_ERR_HIP;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return WN_ERR_HIP;

    std::lock_guard<std::mutex> lk(g_mu);
    WsState &st = g_state[ws];
    const size_t tb = plan.tables.size();
    // a staging buffer whose previous copy has finished, else a new one in the ring
    Staging *sb = nullptr;
    for (Staging &x : st.ring) {
        const hipError_t q = hipEventQuery(x.copied);
        if (q == hipSuccess) {
            sb = &x;
            break;
        }
        if (q != hipErrorNotReady) return WN_ERR_HIP;
    }
    if (sb == nullptr) {
        if (st.ring.size() >= kMaxStaging) {  // a deep backlog of copies: wait for the oldest
            if (hipEventSynchronize(st.ring.front().copied) != hipSuccess) return WN_ERR_HIP;
            sb = &st.ring.front();
        } else {
            st.ring.emplace_back();
            sb = &st.ring.back();
            if (hipEventCreateWithFlags(&sb->copied, hipEventDisableTiming) != hipSuccess) {
                st.ring.pop_back();
                return WN_ERR_HIP;
            }
        }
    }
    if (sb->cap < tb) {
        if (sb->buf) (void)hipHostFree(sb->buf);
        sb->buf = nullptr;
        sb->cap = 0;
        const size_t cap = std::max<size_t>(tb, 64 * 1024);
        if (hipHostMalloc(&sb->buf, cap, hipHostMallocDefault) != hipSuccess) return WN_ERR_HIP;
        sb->cap = cap;
    }
    memcpy(sb->buf, plan.tables.data(), tb);
    if (hipMemcpyAsync(ws + kWsHeader, sb->buf, tb, hipMemcpyHostToDevice, s) != hipSuccess) return WN_ERR_HIP;
    if (hipEventRecord(sb->copied, s) != hipSuccess) return WN_ERR_HIP;

    if (flags & WN_BATCH_NO_GRAPH) return enqueue_kernels(ws, ppl, depth, grid, s) == hipSuccess ? WN_OK : WN_ERR_HIP;

    auto key = std::make_tuple(ppl, depth, grid, dev);
    auto it = st.graphs.find(key);
    if (it == st.graphs.end()) {
        if (!g_capture && hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking) != hipSuccess) return WN_ERR_HIP;
        if (hipStreamBeginCapture(g_capture, hipStreamCaptureModeRelaxed) != hipSuccess) return WN_ERR_HIP;
        hipError_t e = enqueue_kernels(ws, ppl, depth, grid, g_capture);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(g_capture, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return WN_ERR_HIP;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return WN_ERR_HIP;
        it = st.graphs.emplace(key, exec).first;
    }
    return hipGraphLaunch(it->second, s) == hipSuccess ? WN_OK : WN_ERR_HIP;
}

wn_status release_batched(const void *ws) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_state.find(ws);
    if (it == g_state.end()) return WN_OK;
    wn_status st = WN_OK;
    for (Staging &x : it->second.ring) {
        if (x.copied) {
            if (hipEventSynchronize(x.copied) != hipSuccess) st = WN_ERR_HIP;
            (void)hipEventDestroy(x.copied);
        }
        if (x.buf) (void)hipHostFree(x.buf);
    }
    for (auto &g : it->second.graphs) (void)hipGraphExecDestroy(g.second);
    g_state.erase(it);
    return st;
}

}  // namespace wn
