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
// allow_order: the cache-aware tile order may be used (its first use for an
// order builds and uploads a table, which allocates).
int solve_c128_device(int n, const void *a_dev, int64_t lda, void *result_dev, void *ws,
                      size_t ws_bytes, hipStream_t s, bool allow_profile = true, bool allow_order = true);

// Cache-aware tile order of the layer sweep (perm_order.cpp).
// z of the families of group (m high columns, tiles of ck outputs of
// value_bytes each) for nh high columns; 0: colex runs.
int order_z(int nh, int m, uint32_t ck, int value_bytes);
// Appends layer k's padded, interleaved tile list (all tiled groups) to out;
// false if building it failed (host memory).
bool tile_order_layer(int n, int k, int t, uint32_t thin, int chunk, int value_bytes,
                      std::vector<uint32_t> &out);
// Points a (planned with pad8) at the device copy of the order, building and
// uploading it on the first use of (device, n, t, thin, chunk, value_bytes).
int apply_tile_order(int n, int k, int t, uint32_t thin, int chunk, int value_bytes, hipStream_t s,
                     LayerArgs *a);

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
