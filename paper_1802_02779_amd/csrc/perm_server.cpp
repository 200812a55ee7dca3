// Continuous-batching server (filled in below; entry points return PERM_EINVAL until then).
#include "perm_host.h"

using namespace permgpu;

extern "C" {
int perm_server_create(const perm_server_config_t *, perm_server_t **) {
    return set_error(PERM_EINVAL, "server not built yet");
}
int perm_server_submit(perm_server_t *, perm_dtype_t, int, const void *, int64_t, uint64_t *) {
    return set_error(PERM_EINVAL, "server not built yet");
}
int perm_server_poll(perm_server_t *, uint64_t, void *, perm_req_stats_t *) {
    return set_error(PERM_EINVAL, "server not built yet");
}
int perm_server_destroy(perm_server_t *) { return set_error(PERM_EINVAL, "server not built yet"); }
}
