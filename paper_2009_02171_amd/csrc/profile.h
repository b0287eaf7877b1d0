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
// True while launches are being timed on this thread (profiling on, not suspended).
bool prof_active();

// Per-phase times of one solve (the breakdown of a preconditioned iteration
// into the outer operator, the fine RAS sweeps, the coarse solve and the
// fine/coarse transfers).  While a PhaseTimer is installed on a thread, each
// outermost PhaseScope records an event pair on its stream; scopes opened
// inside another scope (the operator and orthogonalisation of the inner
// coarse solve, inside the coarse-solve scope) are not recorded separately.
enum Phase { PH_OP = 0, PH_PCF = 1, PH_PCC = 2, PH_PCI = 3, PH_ORTH = 4, PH_COUNT = 5 };

class PhaseScope {
   public:
    PhaseScope(Phase ph, hipStream_t s);
    ~PhaseScope();
    PhaseScope(const PhaseScope &) = delete;
    PhaseScope &operator=(const PhaseScope &) = delete;

   private:
    hipStream_t s_ = nullptr;
    int slot_ = -1;
    bool counted_ = false;
};

// Installs the thread's phase timer and records the start of the span on s.
int32_t phase_timer_begin(hipStream_t s);
// Records the end of the span, waits for it, uninstalls the timer and sums the
// phases: t_ms[PH_*] and t_ms[PH_COUNT] = span minus the phases (stream time
// outside every phase: vector copies, read-back waits, the host's Givens
// steps, launch gaps); *span_ms = the whole span.
int32_t phase_timer_end(hipStream_t s, double t_ms[PH_COUNT + 1], double *span_ms);
// Uninstalls the timer without reading it (error paths).
void phase_timer_abort();

}  // namespace csd
