// Host-side internals of libpermgpu shared by perm_host.cpp and perm_server.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/perm.h"
#include "perm_internal.h"

namespace permgpu {

// Records the message for perm_last_error() and returns `code`.
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);

// Current device index, with tables built (once per device).
int prepare_device(hipStream_t s, int *device);

// Tuning lookups (process-wide table, defaults when unset).
int tuned_layer_t(int n);
int tuned_layer_remap(int n);
int tuned_layer_flags(int n);
uint32_t tuned_layer_thin(int n);
int tuned_batch_group(int n, size_t lds_bytes, int elem_bytes, int block);

// Complex solve of a device matrix into a device result, stream-ordered.
int solve_c128_device(int n, const void *a_dev, int64_t lda, void *result_dev, void *ws,
                      size_t ws_bytes, hipStream_t s, bool allow_profile = true);

// Workspace bytes of the complex path (both solve entry points).
size_t c128_workspace_bytes(int n);

// The 61-bit primes of the integer paths, largest first.
const std::vector<uint64_t> &primes61();

// Chinese remaindering of R residues (plus the redundant prime p[R] checked
// against res[R]) into a signed multi-limb integer, times the factors in
// *scale when given.
int crt_to_int(const uint64_t *res, const uint64_t *p, int R, perm_int_t *out,
               const std::vector<uint64_t> *scale = nullptr);

// Profiling hooks.
bool profiling_on();
// kind 0 c128 layer, 1 modp layer, 2 batch, 3 Ryser, 4 repeated-column c128 layer, 5 its modp layer
void profile_record(int kind, hipEvent_t start, hipEvent_t stop);
hipEvent_t profile_event();
// Adds to the count of plain 64-bit integer layers run (reported by
// perm_profile_read).
void profile_count_plain(int layers);

// Monotonic clock in seconds.
double now_seconds();

}  // namespace permgpu
