// c3x_batch_kernels.h -- records shared by the batch kernels and their host.
#pragma once

#include "c3x_internal.h"

namespace c3x {

// Batch status flags (device word, read after a run).
constexpr uint32_t kBFlagStale = 1u;  // a source outside its job's planned box
constexpr uint32_t kBFlagCap = 2u;    // a list outgrew the capacity planned for it

// A band candidate the FP64 recheck could not decide: for the host's
// binary128 decision.
struct alignas(8) BAmb {
    double raA, decA, raB, decB, r_arcsec;
    uint32_t i, j, idxA, idxB;
};

}  // namespace c3x
