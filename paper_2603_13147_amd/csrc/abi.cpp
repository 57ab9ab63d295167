// abi.cpp - llp_workspace_bytes: scratch sizes per problem kind.
#include "llp_host.h"

namespace llp {
size_t graph_workspace_bytes(int64_t n, int64_t m, int chunk);
size_t sm_workspace_bytes(int64_t n);
size_t jobs_workspace_bytes(int64_t n, int64_t m, int chunk);
size_t tc_workspace_bytes(int64_t n);
size_t reduce_workspace_bytes(int64_t n);
size_t batch_workspace_bytes(int64_t count);
}  // namespace llp

extern "C" size_t llp_workspace_bytes(int kind, int64_t n, int64_t m, const llp_opts* opts) {
    const int chunk = opts ? opts->chunk : 0;
    switch (kind) {
        case LLP_KIND_SSSP:
        case LLP_KIND_BFS:
            return llp::graph_workspace_bytes(n, m, chunk);
        case LLP_KIND_SM:
            return llp::sm_workspace_bytes(n);
        case LLP_KIND_JOBS:
            return llp::jobs_workspace_bytes(n, m, chunk);
        case LLP_KIND_KNAPSACK:
            return 256;
        case LLP_KIND_TC:
            return llp::tc_workspace_bytes(n);
        case LLP_KIND_REDUCE:
            return llp::reduce_workspace_bytes(n);
        case LLP_KIND_BATCH:
            return llp::batch_workspace_bytes(m);
        default:
            return 0;
    }
}
