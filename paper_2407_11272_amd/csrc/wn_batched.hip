// Batched multi-mesh forward (persistent, graph-captured launch).
#include "wn_internal.hpp"

namespace wn {

size_t batched_workspace(int64_t, int64_t, int64_t) { return 0; }

wn_status run_batched(const wn_mesh_desc *, int32_t, int32_t, char *, size_t, hipStream_t) {
    return WN_ERR_UNSUPPORTED;
}

}  // namespace wn
