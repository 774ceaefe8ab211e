// Step tape and discrete adjoint of the batched BDF solve (abdf_tape_*).
//
// A recording solve stores, per cell, the accepted steps' (h, q) and the
// abundances after each step, plus copies of the inputs; the reverse sweep
// (Engine::reverse) then differentiates the frozen-sequence map through them.
// The tape holds `cap` steps per cell.  A cell with more is swept in windows
// of cap steps, last window first: before each pass a forward re-run of the
// cells that need it records their window (the solve is deterministic, so the
// re-run repeats the recorded steps bit for bit) and the adjoint rows and
// dL/dk carry over from one pass to the next.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>

#include "../../include/astrobdf.h"
#include "engine.hpp"

namespace abdf {

class Tape {
  public:
    Tape(const HostNetwork &net, const DeviceNet &dn) : net_(net), dn_(dn) {}
    ~Tape();
    // Forward solve of io with alpha (device [R], or null for the network's),
    // recording up to `cap` accepted steps per cell.  Returns an abdf_status.
    int record(const BatchIO &io, const double *alpha, const abdf_options &opt, int cap, hipStream_t st,
               std::string &err);
    // Reverse sweep for the loss gradient dLdx [C][S]; any output may be null.
    int adjoint(const double *dLdx, double *g_sum, double *g_cell, double *dx0, double *dphi, hipStream_t st,
                std::string &err);
    size_t bytes() const { return bytes_; }
    long long cells() const { return C_; }

  private:
    const HostNetwork &net_;
    DeviceNet dn_;   // the network's tables, with this tape's copy of alpha
    std::unique_ptr<Engine> eng_;
    abdf_options opt_{};
    long long C_ = 0;
    int cap_ = 0;
    void *base_ = nullptr;
    void *g_slots_ = nullptr;
    size_t bytes_ = 0;
    double *alpha_ = nullptr, *phi_ = nullptr, *x0_ = nullptr, *tape_x_ = nullptr, *tape_h_ = nullptr;
    int32_t *tape_q_ = nullptr, *len_ = nullptr, *status_ = nullptr;
    double *phis_ = nullptr, *t_end_ = nullptr, *hprev_ = nullptr;   // [5][C] inputs, [C] horizons, [C]
    int32_t *qprev_ = nullptr;                                       // [C]
    // buffers of windowed sweeps, allocated by the first sweep that needs them
    void *win_base_ = nullptr;
    size_t win_bytes_ = 0;
    int windowed_sweep(const AdjIO &io, hipStream_t st, std::string &err);
};

}  // namespace abdf
