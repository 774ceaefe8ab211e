// Continuous-batching request server over one engine (abdf_server_*).
//
// A worker thread owns the engine and its stream.  Submitted requests wait in
// a FIFO; whenever slots are free, cells of the oldest requests are admitted
// (their inputs staged through pinned memory), so requests that arrive while
// others run share the device step loop.  Finished cells are harvested every
// few step attempts and written to the caller's output buffers; a request is
// complete when its last cell is.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/astrobdf.h"
#include "engine.hpp"

namespace abdf {

class Server {
  public:
    Server(const HostNetwork &net, const DeviceNet &dn, const abdf_server_options &opt, int device);
    ~Server();
    // Allocates the slot pool and starts the worker; returns an abdf_status.
    int start(int nslots, std::string &err);
    int submit(const abdf_request &req, uint64_t *id, std::string &err);
    int poll(abdf_completion *out, int max, int *n_out, int timeout_ms, std::string &err);
    int cancel(uint64_t id, std::string &err);
    void info(abdf_server_info *out);
    double now() const;

  private:
    struct Request {
        uint64_t id = 0;
        long long n = 0;           // cells to run (lowered to those admitted on cancellation)
        long long n_req = 0;       // cells submitted
        std::vector<double> in;    // [n][kIn]: T, n_H, A_V, zeta, G0, t_end, rtol, atol
        std::vector<double> x0;    // [n][S]
        double *x_out = nullptr;
        int32_t *status = nullptr;
        abdf_cell_stats *stats = nullptr;
        long long next = 0;        // next cell to admit
        long long done = 0;        // cells finished
        long long failed = 0;
        bool cancelled = false;
        double t_submit = 0.0, t_first_admit = -1.0;
    };
    static constexpr int kIn = 8;

    void run();
    int admit_pending(std::string &err);
    int collect(std::string &err);
    void complete(Request *r);
    void apply_cancels(const std::vector<uint64_t> &ids);

    const HostNetwork &net_;
    const DeviceNet &dn_;
    abdf_server_options opt_;
    int device_;
    std::chrono::steady_clock::time_point t0_;
    std::unique_ptr<Engine> eng_;
    hipStream_t st_ = nullptr;
    std::thread th_;

    // shared with callers, guarded by mu_
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<std::shared_ptr<Request>> incoming_;
    std::vector<uint64_t> cancel_ids_;
    std::deque<abdf_completion> completed_;
    bool stop_ = false;
    int error_ = ABDF_OK;
    std::string error_msg_;
    uint64_t next_id_ = 1;
    long long queued_cells_ = 0;      // submitted, not yet admitted
    long long completed_requests_ = 0;
    long long completed_cells_ = 0;
    long long occupied_shared_ = 0;   // copy of occupied_ for info()
    double busy_slot_seconds_ = 0.0;  // integral of occupied slots over time

    // worker only
    std::deque<std::shared_ptr<Request>> pending_;
    std::vector<std::pair<std::shared_ptr<Request>, long long>> owner_;   // per slot
    int occupied_ = 0;
    double t_last_ = 0.0;
    // staging: admission inputs and harvested outputs
    hipEvent_t admit_done_ = nullptr;                 // the last admission's copies have been issued before it
    double *h_in_ = nullptr, *d_in_ = nullptr;       // [kIn][count] columns, then x0 [count][S]
    int32_t *h_slots_ = nullptr, *d_slots_ = nullptr;
    long long *h_cells_ = nullptr, *d_cells_ = nullptr;
    double *h_x_ = nullptr, *d_x_ = nullptr;          // [nslots][S]
    int32_t *h_st_ = nullptr, *d_st_ = nullptr;
    abdf_cell_stats *h_stats_ = nullptr, *d_stats_ = nullptr;
};

}  // namespace abdf
