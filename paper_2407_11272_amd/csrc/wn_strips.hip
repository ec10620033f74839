// Triangle-strip order of a mesh (host code).
//
// The forward kernels consume a mesh as a stream of vertex records: a record whose
// face id is f completes face f together with the two records before it.  Along a
// strip, consecutive faces share an edge, so each new face costs one new vertex
// (one distance, one square root, two dot products) instead of three.  The order is
// a pure function of F, built once per topology (a morphing loop that moves the
// vertices keeps it).  Faces keep their own winding: the kernels take the face
// normal from F, so strip parity does not matter.
//
// Greedy construction: faces are visited in index order; from the first face not yet
// used, each of its three rotations is extended forward along unused neighbours
// across the trailing edge, then the sequence is reversed and extended from the other
// end; the longest of the three is kept.  Strips are capped at kMaxStrip faces.
#include <string.h>

#include <algorithm>
#include <vector>

#include "wn_internal.hpp"

namespace wn {

namespace {

constexpr int kMaxStrip = 1024;

struct Builder {
    const int32_t *F;
    int64_t nF;
    std::vector<int32_t> nbr;    // [3 nF]: face across edge (F[f][j], F[f][j+1]), or -1
    std::vector<uint8_t> done;   // face already placed in a strip
    std::vector<int32_t> stamp;  // face used by the current trial (value = trial id)
    int32_t trial = 0;

    // Edge adjacency from a sorted list of (undirected edge, corner): the faces on an
    // edge are paired in corner order (a non-manifold edge pairs its first two faces,
    // then the next two, ...), which keeps the order a pure function of F.
    void build_edges() {
        std::vector<std::pair<uint64_t, int64_t>> e;
        e.reserve((size_t)nF * 3);
        for (int64_t f = 0; f < nF; ++f)
            for (int j = 0; j < 3; ++j) {
                const int32_t u = F[3 * f + j], v = F[3 * f + (j + 1) % 3];
                if (u == v) continue;
                const uint32_t a = (uint32_t)(u < v ? u : v), b = (uint32_t)(u < v ? v : u);
                e.emplace_back(((uint64_t)a << 32) | b, 3 * f + j);
            }
        std::sort(e.begin(), e.end());
        nbr.assign((size_t)nF * 3, -1);
        for (size_t i = 0; i + 1 < e.size();) {
            if (e[i].first == e[i + 1].first) {
                nbr[(size_t)e[i].second] = (int32_t)(e[i + 1].second / 3);
                nbr[(size_t)e[i + 1].second] = (int32_t)(e[i].second / 3);
                i += 2;
            } else {
                i += 1;
            }
        }
    }

    // Unused face across edge (u, v) of face g; -1 if none.
    int32_t neighbour(int32_t g, int32_t u, int32_t v) const {
        for (int j = 0; j < 3; ++j) {
            const int32_t a = F[3 * (int64_t)g + j], b = F[3 * (int64_t)g + (j + 1) % 3];
            if ((a == u && b == v) || (a == v && b == u)) {
                const int32_t h = nbr[3 * (size_t)g + j];
                if (h >= 0 && !done[(size_t)h] && stamp[(size_t)h] != trial) return h;
                return -1;
            }
        }
        return -1;
    }

    // The vertex of face g that is neither u nor v (-1 if g is degenerate there).
    int32_t third(int32_t g, int32_t u, int32_t v) const {
        int32_t w = -1, count = 0;
        for (int j = 0; j < 3; ++j) {
            const int32_t x = F[3 * (int64_t)g + j];
            if (x != u && x != v) {
                w = x;
                ++count;
            }
        }
        return count == 1 ? w : -1;
    }

    void extend(std::vector<int32_t> &seq, std::vector<int32_t> &faces) {
        while ((int)faces.size() < kMaxStrip) {
            const int32_t u = seq[seq.size() - 2], v = seq[seq.size() - 1];
            const int32_t g = neighbour(faces.back(), u, v);
            if (g < 0) return;
            const int32_t w = third(g, u, v);
            if (w < 0) return;
            seq.push_back(w);
            faces.push_back(g);
            stamp[(size_t)g] = trial;
        }
    }
};

}  // namespace

// Writes the record stream as int32 pairs (vertex id, face id or -1).  Returns the
// number of records; with out == nullptr only counts.
int64_t build_strips(const int32_t *F, int64_t nF, std::vector<int32_t> &out) {
    Builder b;
    b.F = F;
    b.nF = nF;
    b.build_edges();
    b.done.assign((size_t)nF, 0);
    b.stamp.assign((size_t)nF, -1);
    out.clear();
    out.reserve((size_t)nF * 2 * 2 + 16);
    std::vector<int32_t> seq, faces, best_seq, best_faces;
    for (int64_t f = 0; f < nF; ++f) {
        if (b.done[(size_t)f]) continue;
        const int32_t *t = F + 3 * f;
        best_faces.clear();
        for (int r = 0; r < 3; ++r) {
            ++b.trial;
            seq.assign({t[r], t[(r + 1) % 3], t[(r + 2) % 3]});
            faces.assign({(int32_t)f});
            b.stamp[(size_t)f] = b.trial;
            b.extend(seq, faces);
            // reverse and extend the other end (faces keep their own winding)
            std::reverse(seq.begin(), seq.end());
            std::reverse(faces.begin(), faces.end());
            b.extend(seq, faces);
            if (faces.size() > best_faces.size()) {
                best_faces = faces;
                best_seq = seq;
            }
        }
        for (int32_t g : best_faces) b.done[(size_t)g] = 1;
        // records: two opening vertices, then one record per face
        out.push_back(best_seq[0]);
        out.push_back(-1);
        out.push_back(best_seq[1]);
        out.push_back(-1);
        for (size_t i = 0; i < best_faces.size(); ++i) {
            out.push_back(best_seq[i + 2]);
            out.push_back(best_faces[i]);
        }
    }
    return (int64_t)(out.size() / 2);
}

// Pairs of faces that share an edge, for the adjoint's two-faces-per-lane kernel (the
// shared edge's two vertices are evaluated once for both faces).  Consecutive faces of
// each strip are paired; the faces left over (one per strip of odd length) are then
// matched greedily, in face order, with a left-over face across one of their edges.
// Only faces with three distinct vertex ids sharing exactly two of them are paired.
// Output: int32 pairs (f, g), the pairs first, then the unpaired faces as (f, -1), so
// that every face appears exactly once.  A pure function of F.
int64_t build_face_pairs(const int32_t *F, int64_t nF, std::vector<int32_t> &out) {
    auto distinct = [&](int64_t f) {
        const int32_t *t = F + 3 * f;
        return t[0] != t[1] && t[1] != t[2] && t[2] != t[0];
    };
    auto shared = [&](int64_t f, int64_t g) {
        int n = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) n += F[3 * f + i] == F[3 * g + j];
        return n;
    };
    std::vector<int32_t> rec;
    build_strips(F, nF, rec);
    const int64_t nR = (int64_t)rec.size() / 2;
    std::vector<uint8_t> paired((size_t)nF, 0);
    out.clear();
    out.reserve((size_t)nF * 2 + 4);
    // consecutive faces of each strip: face records come in runs after two openers
    for (int64_t r = 0; r + 1 < nR; ++r) {
        const int32_t f = rec[2 * r + 1], g = rec[2 * r + 3];
        if (f < 0 || g < 0 || paired[(size_t)f] || paired[(size_t)g]) continue;
        if (!distinct(f) || !distinct(g) || shared(f, g) != 2) continue;
        paired[(size_t)f] = paired[(size_t)g] = 1;
        out.push_back(f);
        out.push_back(g);
        ++r;  // the next record's face is taken
    }
    // left-over faces: a greedy match across their edges
    Builder b;
    b.F = F;
    b.nF = nF;
    b.build_edges();
    for (int64_t f = 0; f < nF; ++f) {
        if (paired[(size_t)f] || !distinct(f)) continue;
        for (int j = 0; j < 3; ++j) {
            const int32_t g = b.nbr[3 * (size_t)f + j];
            if (g < 0 || g == f || paired[(size_t)g] || !distinct(g) || shared(f, g) != 2) continue;
            paired[(size_t)f] = paired[(size_t)g] = 1;
            out.push_back((int32_t)f);
            out.push_back(g);
            break;
        }
    }
    for (int64_t f = 0; f < nF; ++f)
        if (!paired[(size_t)f]) {
            out.push_back((int32_t)f);
            out.push_back(-1);
        }
    return (int64_t)(out.size() / 2);
}

}  // namespace wn
