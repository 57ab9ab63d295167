// Workspace sizes of the problem kinds the emulated test library does not
// build (abi.cpp refers to them); the graph and job sweeps' own come from graph.hip and jobs.hip.
#include <stddef.h>
#include <stdint.h>
namespace llp {
void batch_release() {}
size_t sm_workspace_bytes(int64_t) { return 256; }
size_t tc_workspace_bytes(int64_t) { return 256; }
size_t reduce_workspace_bytes(int64_t) { return 256; }
size_t batch_workspace_bytes(int64_t) { return 256; }
}  // namespace llp
