// Exact coarsening criteria of a matching pass evaluated on the device (criteria.hip).
//
// The greedy walk of Algorithm alg:pwagg stays on the host; the criteria it asks for (mu_b of
// Lemma thm:mu2 for a pair, mu_g of Thm thm:mu1 for the union of two agglomerates) are
// independent of each other and are evaluated in batches, one GPU thread per pair or union, with
// the arithmetic of crit_core.hpp compiled for the device without contraction so that every value
// equals the host's bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>

#include "coarsen.hpp"

namespace eamg {

// Smallest batches worth a device launch (setup default): below them host threads finish first.
constexpr int kGpuCritMinPairs = 4096;
constexpr int kGpuCritMinUnions = 128;

// Batch evaluator on `s` (the device current at creation).  Device copies of the levels are kept
// until the evaluator is destroyed or another level is handed over.
std::unique_ptr<CritBatch> make_device_criteria(hipStream_t s);

}  // namespace eamg
