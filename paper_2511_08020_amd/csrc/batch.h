// Launch interface of the batched kernels (batch.hip).
#pragma once

#include "kernels.h"

namespace pdg {

// `count` consecutive entries, from `first`, of mesh `mesh`'s element list of one type
struct BatchItem {
    int32_t mesh, first, count;
};

// one phase (0 trace, 1 volume, 2 surface) of every item of one (type, N, equations) group;
// A[mesh] holds the mesh's kernel arguments for the current stage
hipError_t launch_batch_phase(int type, int N, bool ns, int phase, const StageArgs *A, const BatchItem *items,
                              int n_items, hipStream_t s);

}  // namespace pdg
