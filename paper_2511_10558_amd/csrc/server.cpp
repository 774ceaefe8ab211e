// Continuous-batching request server (see server.hpp).
#include "server.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace abdf {

#define HIP_TRY(expr)                                                           \
    do {                                                                        \
        hipError_t e__ = (expr);                                                \
        if (e__ != hipSuccess) {                                                \
            err = std::string(#expr ": ") + hipGetErrorString(e__);            \
            return ABDF_E_DEVICE;                                               \
        }                                                                       \
    } while (0)

Server::Server(const HostNetwork &net, const DeviceNet &dn, const abdf_server_options &opt, int device)
    : net_(net), dn_(dn), opt_(opt), device_(device), t0_(std::chrono::steady_clock::now()) {}

double Server::now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> l(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    if (th_.joinable()) th_.join();
    (void)hipSetDevice(device_);
    if (st_) (void)hipStreamSynchronize(st_);
    eng_.reset();
    if (d_in_) (void)hipFree(d_in_);
    if (h_in_) (void)hipHostFree(h_in_);
    if (h_x_) (void)hipHostFree(h_x_);
    if (h_st_) (void)hipHostFree(h_st_);
    if (h_stats_) (void)hipHostFree(h_stats_);
    if (admit_done_) (void)hipEventDestroy(admit_done_);
    if (st_) (void)hipStreamDestroy(st_);
}

int Server::start(int nslots, std::string &err) {
    HIP_TRY(hipSetDevice(device_));
    HIP_TRY(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&admit_done_, hipEventDisableTiming));
    eng_ = std::make_unique<Engine>(net_, dn_, opt_.solve.precision, opt_.solve.max_steps);
    int rc = eng_->set_options(opt_.solve, err);
    if (rc != ABDF_OK) return rc;
    rc = eng_->init(nslots, err);
    if (rc != ABDF_OK) return rc;
    const size_t n = size_t(nslots), S = size_t(dn_.S);
    // one device block: admission inputs, slot and cell lists, harvested outputs
    const size_t b_in = n * (kIn + S) * sizeof(double), b_sl = n * sizeof(int32_t), b_ce = n * sizeof(long long);
    const size_t b_x = n * S * sizeof(double), b_st = n * sizeof(int32_t), b_stats = n * sizeof(abdf_cell_stats);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t total = al(b_in) + al(b_sl) + al(b_ce) + al(b_x) + al(b_st) + al(b_stats);
    void *base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) {
        err = "server staging of " + std::to_string(total) + " bytes";
        return ABDF_E_NOMEM;
    }
    char *p = static_cast<char *>(base);
    d_in_ = reinterpret_cast<double *>(p);
    p += al(b_in);
    d_slots_ = reinterpret_cast<int32_t *>(p);
    p += al(b_sl);
    d_cells_ = reinterpret_cast<long long *>(p);
    p += al(b_ce);
    d_x_ = reinterpret_cast<double *>(p);
    p += al(b_x);
    d_st_ = reinterpret_cast<int32_t *>(p);
    p += al(b_st);
    d_stats_ = reinterpret_cast<abdf_cell_stats *>(p);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_in_), b_in + b_sl + b_ce, hipHostMallocDefault));
    h_slots_ = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(h_in_) + b_in);
    h_cells_ = reinterpret_cast<long long *>(reinterpret_cast<char *>(h_slots_) + b_sl);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_x_), b_x, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_st_), b_st, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_stats_), b_stats, hipHostMallocDefault));
    // h_slots_ and h_cells_ live inside the h_in_ allocation
    owner_.assign(n, {nullptr, 0});
    th_ = std::thread([this] { run(); });
    return ABDF_OK;
}

int Server::submit(const abdf_request &q, uint64_t *id, std::string &err) {
    if (q.n_cells < 0 || q.n_cells > (1LL << 31)) {
        err = "n_cells out of range";
        return ABDF_E_ARG;
    }
    if (q.n_cells > 0 && (!q.T || !q.n_H || !q.A_V || !q.zeta || !q.G0 || !q.x0 || !q.t_end || !q.x_out ||
                          !q.cell_status)) {
        err = "null request array";
        return ABDF_E_ARG;
    }
    if (!std::isfinite(q.rtol) || !std::isfinite(q.atol)) {
        err = "non-finite tolerance";
        return ABDF_E_ARG;
    }
    auto r = std::make_shared<Request>();
    const long long n = q.n_cells;
    const size_t S = size_t(dn_.S);
    const double rtol = q.rtol > 0 ? q.rtol : opt_.solve.rtol;
    const double atol = q.atol >= 0 ? q.atol : opt_.solve.atol;
    r->n = n;
    r->n_req = n;
    r->in.resize(size_t(n) * kIn);
    for (long long c = 0; c < n; ++c) {
        double *v = r->in.data() + size_t(c) * kIn;
        v[0] = q.T[c];
        v[1] = q.n_H[c];
        v[2] = q.A_V[c];
        v[3] = q.zeta[c];
        v[4] = q.G0[c];
        v[5] = q.t_end[c];
        v[6] = rtol;
        v[7] = atol;
    }
    r->x0.assign(q.x0, q.x0 + size_t(n) * S);
    r->x_out = q.x_out;
    r->status = q.cell_status;
    r->stats = q.stats;
    {
        std::lock_guard<std::mutex> l(mu_);
        if (error_ != ABDF_OK) {
            err = "server stopped: " + error_msg_;
            return error_;
        }
        if (opt_.max_queued_cells > 0 && queued_cells_ + n > opt_.max_queued_cells) {
            err = "server queue full";
            return ABDF_E_BUSY;
        }
        r->id = next_id_++;
        r->t_submit = now();
        *id = r->id;
        if (n == 0) {
            abdf_completion c{};
            c.id = r->id;
            c.t_submit = c.t_done = r->t_submit;
            c.t_first_admit = -1.0;
            completed_.push_back(c);
            ++completed_requests_;
            cv_done_.notify_all();
            return ABDF_OK;
        }
        queued_cells_ += n;
        incoming_.push_back(std::move(r));
    }
    cv_work_.notify_all();
    return ABDF_OK;
}

int Server::poll(abdf_completion *out, int max, int *n_out, int timeout_ms, std::string &err) {
    std::unique_lock<std::mutex> l(mu_);
    auto ready = [this] { return !completed_.empty() || error_ != ABDF_OK; };
    if (!ready() && timeout_ms != 0) {
        if (timeout_ms < 0)
            cv_done_.wait(l, ready);
        else
            cv_done_.wait_for(l, std::chrono::milliseconds(timeout_ms), ready);
    }
    int n = 0;
    while (n < max && !completed_.empty()) {
        out[n++] = completed_.front();
        completed_.pop_front();
    }
    *n_out = n;
    if (n == 0 && error_ != ABDF_OK) {
        err = "server stopped: " + error_msg_;
        return error_;
    }
    return ABDF_OK;
}

int Server::cancel(uint64_t id, std::string &err) {
    {
        std::lock_guard<std::mutex> l(mu_);
        if (id == 0 || id >= next_id_) {
            err = "unknown request id";
            return ABDF_E_ARG;
        }
        cancel_ids_.push_back(id);
    }
    cv_work_.notify_all();
    return ABDF_OK;
}

void Server::info(abdf_server_info *o) {
    std::lock_guard<std::mutex> l(mu_);
    o->slots = eng_ ? eng_->nslots() : 0;
    o->occupied = occupied_shared_;
    o->queued_cells = queued_cells_;
    o->completed_requests = completed_requests_;
    o->completed_cells = completed_cells_;
    o->busy_slot_seconds = busy_slot_seconds_;
    o->uptime = now();
}

void Server::complete(Request *r) {
    abdf_completion c{};
    c.id = r->id;
    c.n_cells = r->n_req;
    c.n_failed = r->failed;
    c.cancelled = r->cancelled ? 1 : 0;
    c.t_submit = r->t_submit;
    c.t_first_admit = r->t_first_admit;
    {
        std::lock_guard<std::mutex> l(mu_);
        c.t_done = now();
        completed_.push_back(c);
        ++completed_requests_;
        if (!r->cancelled) completed_cells_ += r->n_req;
    }
    cv_done_.notify_all();
}

int Server::admit_pending(std::string &err) {
    // plan: consecutive cells of the oldest requests, as many as slots are free
    struct Part { std::shared_ptr<Request> r; long long first, count; };
    std::vector<Part> plan;
    long long room = eng_->free_count(), total = 0;
    for (auto &rp : pending_) {
        if (room == 0) break;
        const long long take = std::min(room, rp->n - rp->next);
        if (take <= 0) continue;
        plan.push_back({rp, rp->next, take});
        room -= take;
        total += take;
    }
    if (total == 0) return ABDF_OK;
    // the previous admission's host-to-device copy must have left the staging buffer
    HIP_TRY(hipEventSynchronize(admit_done_));
    const size_t S = size_t(dn_.S), cnt = size_t(total);
    double *cols = h_in_;                 // [kIn][cnt], then x0 [cnt][S]
    double *x0 = h_in_ + kIn * cnt;
    const double t = now();
    size_t i = 0;
    for (const Part &p : plan) {
        if (p.r->t_first_admit < 0) p.r->t_first_admit = t;
        for (long long c = p.first; c < p.first + p.count; ++c, ++i) {
            const double *v = p.r->in.data() + size_t(c) * kIn;
            for (int k = 0; k < kIn; ++k) cols[k * cnt + i] = v[k];
            std::memcpy(x0 + i * S, p.r->x0.data() + size_t(c) * S, S * sizeof(double));
            const int slot = eng_->take_slot();
            h_slots_[i] = slot;
            h_cells_[i] = (long long)i;
            owner_[slot] = {p.r, c};
        }
        p.r->next += p.count;
    }
    HIP_TRY(hipMemcpyAsync(d_in_, h_in_, cnt * (kIn + S) * sizeof(double), hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(d_slots_, h_slots_, cnt * sizeof(int32_t), hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(d_cells_, h_cells_, cnt * sizeof(long long), hipMemcpyHostToDevice, st_));
    HIP_TRY(hipEventRecord(admit_done_, st_));
    AdmitArgs a{};
    a.count = int(cnt);
    a.slots = d_slots_;
    a.cells = d_cells_;
    a.T = d_in_;
    a.nH = d_in_ + cnt;
    a.Av = d_in_ + 2 * cnt;
    a.zeta = d_in_ + 3 * cnt;
    a.G0 = d_in_ + 4 * cnt;
    a.t_end = d_in_ + 5 * cnt;
    a.rtol_c = d_in_ + 6 * cnt;
    a.atol_c = d_in_ + 7 * cnt;
    a.x0 = d_in_ + kIn * cnt;
    a.newton_tol = opt_.solve.newton_tol;
    int rc = eng_->admit_cells(a, st_, err);
    if (rc != ABDF_OK) return rc;
    occupied_ += int(cnt);
    while (!pending_.empty() && pending_.front()->next >= pending_.front()->n) pending_.pop_front();
    {
        std::lock_guard<std::mutex> l(mu_);
        queued_cells_ -= total;
        occupied_shared_ = occupied_;
    }
    return ABDF_OK;
}

int Server::collect(std::string &err) {
    int nfin = 0;
    int rc = eng_->sync_counts(st_, nfin, err);
    if (rc != ABDF_OK) return rc;
    const double t = now();
    {
        std::lock_guard<std::mutex> l(mu_);
        busy_slot_seconds_ += occupied_ * (t - t_last_);
    }
    t_last_ = t;
    if (nfin == 0) return ABDF_OK;
    HarvestArgs h{};
    h.count = nfin;
    h.x_out = d_x_;
    h.status = d_st_;
    h.stats = d_stats_;
    h.compact = 1;
    rc = eng_->harvest(h, st_, err);
    if (rc != ABDF_OK) return rc;
    const size_t S = size_t(dn_.S);
    HIP_TRY(hipMemcpyAsync(h_x_, d_x_, size_t(nfin) * S * sizeof(double), hipMemcpyDeviceToHost, st_));
    HIP_TRY(hipMemcpyAsync(h_st_, d_st_, size_t(nfin) * sizeof(int32_t), hipMemcpyDeviceToHost, st_));
    HIP_TRY(hipMemcpyAsync(h_stats_, d_stats_, size_t(nfin) * sizeof(abdf_cell_stats), hipMemcpyDeviceToHost, st_));
    HIP_TRY(hipStreamSynchronize(st_));
    const int32_t *slots = eng_->finished_slots();
    for (int i = 0; i < nfin; ++i) {
        auto &own = owner_[slots[i]];
        std::shared_ptr<Request> r = std::move(own.first);
        const long long c = own.second;
        own = {nullptr, 0};
        --occupied_;
        if (!r) continue;
        if (!r->cancelled) {
            std::memcpy(r->x_out + size_t(c) * S, h_x_ + size_t(i) * S, S * sizeof(double));
            r->status[c] = h_st_[i];
            if (r->stats) r->stats[c] = h_stats_[i];
        }
        if (h_st_[i] != ABDF_CELL_OK) ++r->failed;
        ++r->done;
        if (r->done == r->next && (r->next == r->n || r->cancelled)) complete(r.get());
    }
    std::lock_guard<std::mutex> l(mu_);
    occupied_shared_ = occupied_;
    return ABDF_OK;
}

void Server::apply_cancels(const std::vector<uint64_t> &ids) {
    for (uint64_t id : ids) {
        // a request is cancellable while it is pending or has cells in slots
        Request *r = nullptr;
        for (auto &p : pending_)
            if (p->id == id) r = p.get();
        if (!r)
            for (auto &o : owner_)
                if (o.first && o.first->id == id) r = o.first.get();
        if (!r || r->cancelled) continue;
        r->cancelled = true;
        const long long dropped = r->n - r->next;
        {
            std::lock_guard<std::mutex> l(mu_);
            queued_cells_ -= dropped;
        }
        r->n = r->next;   // nothing more is admitted
        if (r->done == r->next) complete(r);
    }
    pending_.erase(std::remove_if(pending_.begin(), pending_.end(),
                                  [](const std::shared_ptr<Request> &p) { return p->cancelled; }),
                   pending_.end());
}

void Server::run() {
    std::string err;
    int rc = hipSetDevice(device_) == hipSuccess ? ABDF_OK : ABDF_E_DEVICE;
    if (rc != ABDF_OK) err = "hipSetDevice in the server worker";
    const int check_every = std::max(1, opt_.solve.check_every);
    int since = 0;
    t_last_ = now();
    while (rc == ABDF_OK) {
        std::vector<uint64_t> cancels;
        {
            std::unique_lock<std::mutex> l(mu_);
            cv_work_.wait(l, [&] {
                return stop_ || !incoming_.empty() || !cancel_ids_.empty() || !pending_.empty() || occupied_ > 0;
            });
            if (stop_) return;
            for (auto &r : incoming_) pending_.push_back(std::move(r));
            incoming_.clear();
            cancels.swap(cancel_ids_);
        }
        if (!cancels.empty()) apply_cancels(cancels);
        if (!pending_.empty() && eng_->free_count() > 0) {
            rc = admit_pending(err);
            if (rc != ABDF_OK) break;
        }
        if (eng_->running() > 0) {
            rc = eng_->attempt(st_, err);
            if (rc != ABDF_OK) break;
            ++since;
        }
        if (occupied_ > 0 && (eng_->running() == 0 || since >= check_every)) {
            since = 0;
            rc = collect(err);
        }
    }
    {
        std::lock_guard<std::mutex> l(mu_);
        error_ = rc;
        error_msg_ = err;
    }
    cv_done_.notify_all();
}

}  // namespace abdf
