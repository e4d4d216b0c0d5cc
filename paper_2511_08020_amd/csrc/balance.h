// Load balance from measured work-queue times (host only).
//
// The work-queue schedule runs one workgroup per contiguous segment of the Hilbert-ordered
// element list; each queue kernel adds its workgroup's device wall-clock time to a per-queue,
// per-phase counter (the paper's loop timers, Sec. 3, Listing 1, taken per queue instead of
// per rank).  From those times this file attributes a cost to every element: the time of a
// queue in one phase is shared by its elements in proportion to per-type costs fitted over all
// queues (non-negative least squares, one fit per phase), which is the paper's attribution by
// loop participation with the modal overhead resolved by element type.  The integer weights
// derived from the element costs feed the prefix-sum partition.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pdg {

constexpr int kPhases = 3;  // trace, volume, surface

// Imbalance of per-phase queue loads L[ph][q]: sum over phases of the slowest queue over sum
// over phases of the mean queue, minus one (0 = perfect balance).
double queue_imbalance(const std::vector<double> &load, int32_t n_queues);

// Fits per-type costs and attributes the measured times to elements.
//   etype[n], qb[nq+1] (validated by the caller), qms[kPhases*nq] (>= 0, not all 0)
//   cost  <- [kPhases][n] element cost per phase, in the units of qms
//   type_cost[kPhases*4] <- fitted cost per element of each type and phase (0 for absent types)
void attribute_costs(int32_t n, const int8_t *etype, int32_t nq, const int32_t *qb, const double *qms,
                     std::vector<double> &cost, double type_cost[kPhases * 4]);

// Integer weights max(1, round(1024 c_e / mean c)) of the per-element total cost, at most 2^24.
void cost_weights(int32_t n, const std::vector<double> &cost, uint32_t *weight);

// Per-phase loads of the queues of schedule qb under per-element costs `cost`.
std::vector<double> queue_loads(int32_t n, const std::vector<double> &cost, int32_t nq, const int32_t *qb);

// Checks a queue schedule against n elements; returns an empty string or the error.
std::string check_schedule(int32_t n, int32_t nq, const int32_t *qb);

}  // namespace pdg
