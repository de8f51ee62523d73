// The served path's error policy: what happens to each query of a batch
// that has finished.  Plain C++ (no HIP), so that its cases are checked on
// the host.
#pragma once

#include <cstdint>

#include "gq.h"

enum class gq_retire_action {
    complete,         // the query is done, with the batch's status
    rerun_alone,      // run it again by itself (a shared batch reported an error)
    rerun_doubled,    // run it again by itself with twice the group bound
};

struct gq_retire_case {
    gq_status batch_status;   // launch status, else the batch's device status word
    int batch_queries;        // queries in the batch
    bool aggregate;           // a group-by template (FILTER_TOPK is not)
    int64_t max_groups;       // the query's group bound in this run
    int64_t capacity;         // its output capacity
    bool doubled_fits;        // the query alone, with the doubled bound, fits the pool
};

// The doubled group bound of a rerun: twice the bound, at most the capacity.
inline int64_t gq_doubled_groups(int64_t max_groups, int64_t capacity)
{
    return 2 * max_groups < capacity ? 2 * max_groups : capacity;
}

// A failed shared batch does not charge its error to every query: each runs
// again alone.  A query alone whose groups overflowed runs again with twice
// the bound while its outputs have room and it still fits the pool.  Launch
// failures (GQ_ERR_HIP) and everything else complete with their status.
inline gq_retire_action gq_retire_decide(const gq_retire_case &c)
{
    if (c.batch_status == GQ_OK) return gq_retire_action::complete;
    if (c.batch_status != GQ_ERR_HIP && c.batch_queries > 1) return gq_retire_action::rerun_alone;
    if (c.batch_status == GQ_ERR_CAPACITY && c.aggregate && c.max_groups < c.capacity && c.doubled_fits)
        return gq_retire_action::rerun_doubled;
    return gq_retire_action::complete;
}
