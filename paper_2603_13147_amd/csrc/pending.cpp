// pending.cpp - scratch-size hooks for plugins not built yet (removed as they land).
#include <stddef.h>
#include <stdint.h>
namespace llp {
size_t sm_workspace_bytes(int64_t n) { return 256 + (size_t)n * 16; }
size_t jobs_workspace_bytes(int64_t n, int64_t m) { return 256 + (size_t)(n + m) * 16; }
size_t tc_workspace_bytes(int64_t n) { return 256 + (size_t)n * 16; }
size_t reduce_workspace_bytes(int64_t n) { return 256 + (size_t)n * 16; }
size_t batch_workspace_bytes(int64_t count) { return 256 + (size_t)count * 16; }
}  // namespace llp
