// Continuous-batching request server -- see include/ss.h.
#include "handle.hpp"

extern "C" {

int ss_server_create(size_t, int32_t, ss_server *out) {
    if (out) *out = nullptr;
    return SS_E_INVALID_ARG;
}
int ss_submit(ss_server, const ss_csr_z *, const ss_csr_z *, int32_t, int64_t, int32_t, double, const ss_options *,
              uint64_t *) {
    return SS_E_INVALID_ARG;
}
int ss_poll(ss_server, uint64_t, double *, ss_info *) { return SS_E_INVALID_ARG; }
int ss_server_drain(ss_server) { return SS_E_INVALID_ARG; }
void ss_server_destroy(ss_server) {}

}
