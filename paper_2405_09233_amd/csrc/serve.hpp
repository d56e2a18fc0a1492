// Serving loop (continuous batching) behind tsylv_submit / tsylv_poll.
#pragma once

#include "runtime.hpp"

namespace tsylv {

Scheduler* scheduler_create(Ctx& ctx);
void scheduler_destroy(Scheduler* s);  // cancels queued requests, finishes running ones
uint64_t scheduler_submit(Scheduler* s, const tsylv_request& r);
int scheduler_poll(Scheduler* s, uint64_t ticket, tsylv_info* info);

}  // namespace tsylv
