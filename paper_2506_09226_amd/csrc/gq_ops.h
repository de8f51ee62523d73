// Internal operations shared between operator sources.
#pragma once

#include "gq_internal.h"

// In-place exclusive scan of n uint32 values (n >= 0); ws must hold
// gq_scan_u32_workspace(n) bytes and is zeroed by the call.
size_t gq_scan_u32_workspace(int64_t n);
gq_status gq_scan_u32(gq_ctx *ctx, uint32_t *data, int64_t n, void *ws, hipStream_t s);
