// Launch-configuration cache and the autotuner entry point.
//
// A configuration (points per lane, record tiles staged per barrier, persistent
// workgroups per CU) only changes how work is mapped onto lanes, workgroups and LDS; the
// per-point order of the face sum is fixed by the record tiles and chunks, so every
// configuration gives bit-identical results.  Shapes are bucketed by floor(log2) of two size parameters.  With
// WN_AUTOTUNE_CACHE set, the cache is read from and written to that file as JSON
// lines {"arch": "gfx950", "op": o, "a": i, "b": j, "ppl": p, "wg": w, "depth": d}.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "wn_internal.hpp"

namespace wn {

namespace {

struct Key {
    int32_t op, a, b;
    bool operator<(const Key &o) const {
        if (op != o.op) return op < o.op;
        if (a != o.a) return a < o.a;
        return b < o.b;
    }
};

std::mutex g_mu;
std::map<Key, TuneConfig> g_cache;
bool g_loaded = false;

int32_t bucket(int64_t x) {
    int32_t b = 0;
    while (x > 1 && b < 62) {
        x >>= 1;
        ++b;
    }
    return b;
}

void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = getenv("WN_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char arch[32] = {0};
        int op, a, b, ppl, wg, depth = 1;
        const int got = sscanf(line,
                               " {\"arch\": \"%31[^\"]\", \"op\": %d, \"a\": %d, \"b\": %d, \"ppl\": %d, \"wg\": %d, "
                               "\"depth\": %d}",
                               arch, &op, &a, &b, &ppl, &wg, &depth);
        if (got >= 6 && strcmp(arch, "gfx950") == 0 && valid_ppl(ppl) && wg >= 0 && valid_depth(depth))
            g_cache[Key{op, a, b}] = TuneConfig{ppl, wg, depth};
    }
    fclose(f);
}

void save_locked() {
    const char *path = getenv("WN_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_cache)
        fprintf(f, "{\"arch\": \"gfx950\", \"op\": %d, \"a\": %d, \"b\": %d, \"ppl\": %d, \"wg\": %d, \"depth\": %d}\n",
                kv.first.op, kv.first.a, kv.first.b, kv.second.ppl, kv.second.wg_per_cu, kv.second.depth);
    fclose(f);
    rename(tmp.c_str(), path);
}

}  // namespace

bool valid_ppl(int32_t ppl) { return ppl == 1 || ppl == 2 || ppl == 4; }
bool valid_depth(int32_t depth) { return depth == 1 || depth == 2 || depth == 4; }

// Without a measurement: one point per lane for the exact field (its per-lane state is
// large), two for the naive sum (measured 1.35x faster than one on an MI355X).
TuneConfig default_config(int32_t op) { return op == WN_OP_NAIVE ? TuneConfig{2, 0, 1} : TuneConfig{1, 0, 1}; }

TuneConfig lookup_config(int32_t op, int64_t a, int64_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_cache.find(Key{op, bucket(a), bucket(b)});
    return it == g_cache.end() ? default_config(op) : it->second;
}

void store_config(int32_t op, int64_t a, int64_t b, const TuneConfig &c) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_cache[Key{op, bucket(a), bucket(b)}] = c;
    save_locked();
}

}  // namespace wn
