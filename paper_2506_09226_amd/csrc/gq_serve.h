// Internal interface between the shared-scan batch executor and the server.
#pragma once

#include "gq_internal.h"

constexpr int SV_MAX_BATCH = 16;          // queries per shared-scan batch
constexpr int SV_MAX_AGG_GROUPS = 512;    // groups per query of the small-group templates

struct gq_serve_tables {
    const int64_t *fk, *fk2;
    const int32_t *date;
    const int64_t *qty, *price, *disc;
    int64_t n;
    const void *dim1_table, *dim2_table;
    int dim1_log2, dim2_log2;             // log2 of the tables' slot counts
};

struct gq_serve_query_out {
    gq_groups groups;
    int64_t *topk_val;
    int32_t *topk_row;
    int64_t *topk_n;
};

struct gq_serve_query {
    int32_t kind;
    int32_t k;
    int64_t date_hi;
    int64_t max_groups;
    gq_serve_query_out out;
};

// Workspace of one batch (all queries of one kind) and its execution.
size_t gq_serve_batch_bytes(const gq_serve_tables &t, const gq_serve_query *q, int nq);
gq_status gq_serve_batch(gq_ctx *ctx, const gq_serve_tables &t, const gq_serve_query *q, int nq, void *ws,
                         size_t ws_bytes, hipStream_t s);
// The plain per-operator form of one query (the serial baseline).
size_t gq_serve_single_bytes(const gq_serve_tables &t, const gq_serve_query &q);
gq_status gq_serve_single(gq_ctx *ctx, const gq_serve_tables &t, const gq_serve_query &q, void *ws, size_t ws_bytes,
                          hipStream_t s);
