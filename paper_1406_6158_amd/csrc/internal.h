// internal.h -- library-internal entry points shared between the context
// implementation (api.hip) and the request server (serve.hip).  Not part of
// the C ABI.
#pragma once

#include <stdint.h>

#include "../../include/htree.h"

namespace htree {

// Records an error message for htree_last_error() and returns code.
htree_status set_error(htree_status code, const char *msg);

// htree_set_state with a row stride: d_x holds x, y, z rows of ldx >= n
// doubles each, of which the first n are used.
htree_status ctx_set_state(htree_ctx *c, const double *d_x, int64_t ldx, const float *d_v,
                           const float *d_m);

// What a finished solve reports back to the host (pinned memory).
struct CtxReport {
    unsigned long long tally[4];   // soft interactions, hard candidates, hard pairs, spare
    uint32_t status;               // sticky device status word
    uint32_t pad[7];
};

// Enqueues copies of the status word and the interaction tallies into *dst
// on the context's stream.
htree_status ctx_report_async(htree_ctx *c, CtxReport *dst);

// Maps a status word to HTREE_OK or an error (with its message).
htree_status status_code(uint32_t word);

}  // namespace htree
