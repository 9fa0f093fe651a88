// The request server (continuous batching within an HBM budget).
#pragma once

#include "core.hpp"

namespace llama {

struct Server;

Server* create_server(const llama_server_config* cfg, const llama_executor* exec = nullptr);
uint64_t server_submit(Server* s, const llama_copy_item* item);
// true when the request has finished (status and latency filled in); with
// `wait`, blocks until it has
bool server_poll(Server* s, uint64_t ticket, bool wait, int& status, double& latency);
void server_stats(Server* s, llama_server_stats& st);
void server_reset_stats(Server* s);
void destroy_server(Server* s);

// kernels.hip: one launch of the batch kernel over a serialised work table
void launch_batch_args(const BatchArgs& args, uint32_t grid, uint32_t threads, uint32_t lds_bytes, bool persistent,
                       void* stream);

} // namespace llama
