// Launch interface of the batched kernels (batch.hip).
#pragma once

#include "kernels.h"

namespace pdg {

// `count` consecutive entries, from `first`, of mesh `mesh`'s element list of one type
struct BatchItem {
    int32_t mesh, first, count;
};

// one phase (0 trace, 1 volume, 2 surface) of every item of one (type, N, equations, curved)
// group; A[mesh] holds the mesh's kernel arguments for the current stage; cv: the group's meshes
// have curved elements (per-node metrics, per-element mass matrices)
hipError_t launch_batch_phase(int type, int N, bool ns, bool cv, int phase, const StageArgs *A,
                              const BatchItem *items, int n_items, hipStream_t s);

}  // namespace pdg
