// host_ip.h -- initial partitioning of the coarsest graph on the host.
#pragma once

#include "pm_internal.h"

namespace pm {

// Hierarchical multisection with a breadth-first split.  Host arrays; writes
// PE ids (not codes) to part_ids.
void host_initial_partition(int32_t n, const int64_t *xadj, const int32_t *adj,
                            const int32_t *vwgt, const Hier &h, int32_t *part_ids);

}  // namespace pm
