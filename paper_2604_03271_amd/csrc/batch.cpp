// batch.cpp -- batched and served paths (placeholders until the batched driver lands).
#include "host_common.hpp"

extern "C" smc_status smc_batch_run(const smc_problem*, int32_t, const smc_options*, double*) { return SMC_ESTATE; }
extern "C" smc_status smc_server_create(smc_server** out, uint64_t, const smc_options*) {
    if (out) *out = nullptr;
    return SMC_ESTATE;
}
extern "C" smc_status smc_server_submit(smc_server*, const smc_problem*, uint64_t) { return SMC_ESTATE; }
extern "C" smc_status smc_server_poll(smc_server*, smc_result*, int32_t, int32_t* n, int32_t) {
    if (n) *n = 0;
    return SMC_ESTATE;
}
extern "C" uint64_t smc_server_request_bytes(const smc_problem*, const smc_options*) { return 0; }
extern "C" void smc_server_destroy(smc_server*) {}
