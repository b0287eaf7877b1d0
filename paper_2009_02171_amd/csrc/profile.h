// Per-launch HIP-event timing scope (active only between csdyn_profile_begin
// and csdyn_profile_end).
#pragma once

#include "common.h"

namespace csd {

class ProfScope {
   public:
    // size: the launch's problem size (cells, box cells or vector length);
    // bytes: the algorithmic HBM bytes the launch must move.  Timings and
    // bytes are aggregated per (name, size).
    ProfScope(const char *name, int64_t size, double bytes, hipStream_t s, double flops = 0.0);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

   private:
    hipStream_t s_;
    int64_t slot_ = -1;
};

// While a thread captures a graph its launches are not timed (an event pair
// recorded during capture would become graph nodes).
void prof_suspend(bool on);

}  // namespace csd
