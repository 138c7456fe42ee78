// fk_chain.hpp -- chain rewriting done once per plan: the run-time tier's
// normalised op list and the match against the compile-time chains built
// into the library.  Plain C++ (no HIP), so host tests can build it with g++.
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/fk.h"
#include "fk_internal.hpp"

namespace fk {

// Run-time tier op list for a validated chain (see fk_chain.cpp); swap = 1
// when the read must exchange channels 0 and 2.
void normalise_chain(const fk_chain_desc *ch, bool strict, std::vector<OpRec> &ops, int32_t &swap);
// Executed records per code (loops unrolled) of a normalised list.
// Consecutive identical records (outside multi-record loop bodies) merged
// into one record repeated by a one-record LOOP; the last step of
// normalise_chain.
void merge_repeats(std::vector<OpRec> &ops);
void executed_counts(const std::vector<OpRec> &ops, double cnt[4]);
// FAM_NORMALIZE / FAM_MULADD / FAM_MULADD_LOOP with their constants (and
// op count, or the loop's count of pairs) when the chain is one of the
// compile-time chains, else FAM_RUNTIME.
int match_static(const fk_chain_desc *ch, std::vector<float> &consts, int &n_ops);

}  // namespace fk
