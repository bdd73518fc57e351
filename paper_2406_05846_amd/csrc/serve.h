// serve.h -- continuous-batching request loop behind strom_submit / strom_poll.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/strom.h"

namespace strom {

struct Server;

Server *server_start(strom_ctx *ctx);
void server_stop(Server *s);
strom_status server_submit(Server *s, const strom_problem *P, const strom_opts *opts, uint64_t *ticket,
                           std::string &err);
strom_status server_poll(Server *s, uint64_t ticket, strom_info *out, double *X, double *y, double *S,
                         std::string &err);

// Instance hooks implemented next to the C ABI (api.cpp).
hipError_t sdp_enqueue(strom_sdp *s, int n_iter, bool kkt_last);
hipError_t sdp_read_state(strom_sdp *s);
void sdp_info(strom_sdp *s, strom_info *info);
const strom_opts &sdp_opts(strom_sdp *s);

}  // namespace strom
