// Host orchestration of the batched BDF solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "network.hpp"

struct abdf_options;
struct abdf_cell_stats;

namespace abdf {

// Device inputs/outputs of one batch solve (caller-owned device pointers).
struct BatchIO {
    long long n_cells;
    const double *T, *nH, *Av, *zeta, *G0, *x0, *t_end;
    double *x_out;
    int32_t *status;
    abdf_cell_stats *stats;
};

// Device inputs/outputs of one reverse sweep (tape-owned or caller-owned device pointers).
struct AdjIO {
    long long n_cells;
    const double *phi;        // [n][5]
    const double *dLdx;       // [n][S]
    const int32_t *status;    // [n] forward outcome
    double *g_cell;           // [n][R] gradient with respect to log alpha per cell, or null
    double *dx0;              // [n][S] or null
    double *dphi;             // [n][5] gradient with respect to T, n_H, A_V, zeta, G0, or null
};

// Host buffers of an engine that allocates nothing itself: the caller keeps
// them (static storage) and they hold up to max_slots slots.
struct HostBuffers {
    int32_t *cnt;            // [kCountSlots]
    int32_t *fin;            // [max_slots]
    int32_t *admit_slots;    // [max_slots]
    long long *admit_cells;  // [max_slots]
    int32_t *free_list;      // [max_slots]
    double *atol;            // [kMaxSpecies] per-species absolute tolerances
    int max_slots;
};
constexpr int kMaxSpecies = 512;   // the factorisation holds at most this order

// Process-wide kernel timers (abdf_profile_*).
struct Profiler {
    static bool on();
    static void enable(bool v);
    static void add(int kind, double ms);
    static void read(int64_t *launches, double *ms, bool reset);
};

// A pool of device slots for one network.  Cells are admitted into free
// slots, integrated by the step-attempt loop, and harvested when finished;
// freed slots are refilled from the pending cells (continuous batching).
class Engine {
  public:
    Engine(const HostNetwork &net, const DeviceNet &dn, int prec, int max_steps);
    ~Engine();
    // Allocates room for up to `nslots` slots; returns an abdf_status.  With
    // cache_workspace the device workspace is taken from the network's cache
    // on this device when large enough and returned to it by the destructor.
    int init(int nslots, std::string &err, bool cache_workspace = false);
    // Lays out `nslots` slots in caller-provided device memory (`bytes` at
    // `base`) with the host buffers `hb`, allocating nothing: no side stream,
    // no events, no kernel timers; the counters are cleared by a kernel on the
    // solve's stream.  Returns an abdf_status.
    int init_external(int nslots, void *base, size_t bytes, const HostBuffers &hb, std::string &err);
    // Device bytes of the workspace of n slots (as init lays it out).
    static size_t workspace_bytes(const DeviceNet &dn, long long n);
    // relative change of c within which a slot keeps its factorisation (0: none)
    void set_lu_reuse(double v) { lu_reuse_ = v; s_.lu_reuse = v; }
    // highest order the order selection may reach (1..5; 0 or out of range: 5)
    void set_max_order(int q) {
        max_order_ = (q >= 1 && q <= kMaxOrder) ? q : kMaxOrder;
        s_.max_order = max_order_;
    }
    // The method options of o (reuse threshold, order cap, step bounds and the
    // per-species absolute tolerances, read from the device now into atol_host,
    // kMaxSpecies doubles, or into storage of the engine's own when null).  Before init.
    int set_options(const abdf_options &o, std::string &err, double *atol_host = nullptr);
    // first step (0: heuristic) and bound on every step (0: none), seconds
    void set_step_bounds(double h0, double h_max) {
        h0_ = h0;
        h_max_ = h_max;
        s_.h0 = h0;
        s_.h_max = h_max;
    }
    // Bytes of device workspace per slot.
    static size_t bytes_per_slot(const DeviceNet &dn, int prec);
    // Solves every cell of io; returns an abdf_status.
    int solve(const BatchIO &io, const abdf_options &opt, hipStream_t st, std::string &err);

    // Reverse sweep of the recorded steps (the slots' tape pointers must be set).
    int reverse(const AdjIO &io, int check_every, hipStream_t st, std::string &err);

    // Building blocks of a driver loop (batch solve, server, adjoint).
    int nslots() const { return s_.nslots; }
    int free_count() const { return n_free_; }
    // Slots on the current attempt list (an upper bound until the next sync_counts).
    int running() const { return bound_; }
    int take_slot() { return free_[--n_free_]; }
    // Admits a.count cells into the slots a.slots (taken with take_slot).
    int admit_cells(const AdmitArgs &a, hipStream_t st, std::string &err);
    // One step attempt of every running slot (ESDIRK: one stage).
    int attempt(hipStream_t st, std::string &err);
    // Waits for the stream and reads the running and finished counts.
    int sync_counts(hipStream_t st, int &nfin, std::string &err);
    // Copies the nfin finished slots out (h.count = nfin, h.slots = the finished
    // list), waits, and returns the slots to the free list; their ids stay
    // readable in finished_slots() until the next harvest.
    int harvest(HarvestArgs h, hipStream_t st, std::string &err);
    const int32_t *finished_slots() const { return h_fin_; }
    const int32_t *device_finished_list() const { return s_.fin; }
    Slots &slots() { return s_; }
    const DeviceNet &net() const { return dn_; }
    int ring() const { return ring_; }
    // kernel timers: an event before a launch, and after it with its family
    hipEvent_t timer_begin(hipStream_t st);
    void timer_end(int kind, hipEvent_t a, hipStream_t st);
    void flush_timers();
    // Newton tolerance for a relative tolerance (option value if positive).
    static double newton_tolerance(const abdf_options &opt);

  private:
    int admit(const BatchIO &io, const abdf_options &opt, long long &next, hipStream_t st, std::string &err);
    int newton_iterations(int which, hipStream_t st, std::string &err);
    hipError_t control(hipStream_t st);   // the method's control kernel

    const HostNetwork &net_;
    const DeviceNet &dn_;
    int prec_, max_steps_;
    double lu_reuse_ = 0.0;
    int max_order_ = kMaxOrder;
    double h0_ = 0.0, h_max_ = 0.0;
    int method_ = 0;   // ABDF_METHOD_*
    int tvar_ = 0;
    double phi_exp_[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    std::vector<double> atol_store_;   // per-species absolute tolerances when the engine owns them
    const double *atol_sp_ = nullptr;  // host copy of the per-species tolerances, or null (scalar atol)
    Slots s_{};
    bool ext_ = false;                 // workspace and host buffers belong to the caller
    bool cached_ = false;              // the workspace goes back to the network's cache
    void *base_ = nullptr;
    size_t base_bytes_ = 0;
    int reset_counts(hipStream_t st, std::string &err);
    int layout(int nslots, void *base, std::string &err);
    int32_t *d_admit_slots_ = nullptr;
    long long *d_admit_cells_ = nullptr;
    int32_t *h_cnt_ = nullptr;          // pinned [kCountSlots]
    hipStream_t side_ = nullptr;        // Newton iterations of slots that do not factor (default priority)
    hipEvent_t ev_lists_ = nullptr, ev_side_ = nullptr;
    int32_t *h_fin_ = nullptr;          // pinned [nslots]
    int32_t *h_admit_slots_ = nullptr;  // pinned [nslots]
    long long *h_admit_cells_ = nullptr;
    std::vector<int32_t> free_store_;  // free-slot stack when the engine owns it
    int32_t *free_ = nullptr;
    int n_free_ = 0;
    int ring_ = 0;
    int bound_ = 0;
    // LDS and persistent grid sizes; the *64 / unsuffixed FP64 values serve the
    // FP64 variants, *32 / the main grids the FP32 ones in FP32-LU engines
    size_t lds_admit_ = 0, lds_factor_ = 0, lds_factor32_ = 0, lds_newton_ = 0, lds_solve_ = 0, lds_solve32_ = 0;
    int grid_factor_max_ = 256, grid_newton_max_ = 512, grid_solve_max_ = 1024;
    int grid_factor64_max_ = 256, grid_solve64_max_ = 1024, grid_solve_ref_max_ = 512, grid_adj_solve_max_ = 1024;
    // kernel timers of launches not yet read back
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> event_pool_;
};

}  // namespace abdf
