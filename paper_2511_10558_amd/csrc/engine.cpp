// Host orchestration: slot pool, admission, the step-attempt loop and harvest.
//
// Every loop iteration performs one step attempt for every running slot:
//   k_factor   (slots whose Newton matrix is stale)
//   k_newton   x 4 (slots still iterating)
//   k_control  (accept / reject / order selection, next attempt queued)
// The slot lists are compacted on the device every attempt.  The host reads
// the running and finished counts back every `check_every` attempts, copies
// finished results out, and refills freed slots with pending cells.
#include "engine.hpp"

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/astrobdf.h"

namespace abdf {

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// A named host range for rocprofv3 --marker-trace (one library call each way
// when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

#define HIP_TRY(expr)                                                           \
    do {                                                                        \
        hipError_t e__ = (expr);                                                \
        if (e__ != hipSuccess) {                                                \
            err = std::string(#expr ": ") + hipGetErrorString(e__);            \
            return ABDF_E_DEVICE;                                               \
        }                                                                       \
    } while (0)
}  // namespace

namespace {
std::atomic<bool> g_prof_on{false};
std::mutex g_prof_mu;
int64_t g_prof_launches[ABDF_PROF_KINDS];
double g_prof_ms[ABDF_PROF_KINDS];
}  // namespace

bool Profiler::on() { return g_prof_on.load(std::memory_order_relaxed); }
void Profiler::enable(bool v) { g_prof_on.store(v); }
void Profiler::add(int kind, double ms) {
    std::lock_guard<std::mutex> l(g_prof_mu);
    g_prof_launches[kind] += 1;
    g_prof_ms[kind] += ms;
}
void Profiler::read(int64_t *launches, double *ms, bool reset) {
    std::lock_guard<std::mutex> l(g_prof_mu);
    for (int i = 0; i < ABDF_PROF_KINDS; ++i) {
        launches[i] = g_prof_launches[i];
        ms[i] = g_prof_ms[i];
        if (reset) { g_prof_launches[i] = 0; g_prof_ms[i] = 0.0; }
    }
}

hipEvent_t Engine::timer_begin(hipStream_t st) {
    if (ext_ || !Profiler::on()) return nullptr;
    hipEvent_t e = nullptr;
    if (!event_pool_.empty()) {
        e = event_pool_.back();
        event_pool_.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, st) != hipSuccess) {
        event_pool_.push_back(e);
        return nullptr;
    }
    return e;
}

void Engine::timer_end(int kind, hipEvent_t a, hipStream_t st) {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!event_pool_.empty()) {
        b = event_pool_.back();
        event_pool_.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
        event_pool_.push_back(a);
        return;
    }
    (void)hipEventRecord(b, st);
    pending_.push_back({kind, a, b});
}

// Called after the stream has been synchronised.
void Engine::flush_timers() {
    for (auto &p : pending_) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) Profiler::add(p.kind, double(ms));
        event_pool_.push_back(p.a);
        event_pool_.push_back(p.b);
    }
    pending_.clear();
}

Engine::Engine(const HostNetwork &net, const DeviceNet &dn, int prec, int max_steps)
    : net_(net), dn_(dn), prec_(prec), max_steps_(max_steps) {}

Engine::~Engine() {
    for (auto &p : pending_) {
        event_pool_.push_back(p.a);
        event_pool_.push_back(p.b);
    }
    for (hipEvent_t e : event_pool_) (void)hipEventDestroy(e);
    if (ext_) return;   // nothing below was allocated
    if (base_) {
        if (cached_)
            net_.keep_workspace(dn_.device, base_, base_bytes_);
        else
            (void)hipFree(base_);
    }
    if (h_cnt_) (void)hipHostFree(h_cnt_);
    if (h_fin_) (void)hipHostFree(h_fin_);
    if (h_admit_slots_) (void)hipHostFree(h_admit_slots_);
    if (h_admit_cells_) (void)hipHostFree(h_admit_cells_);
    if (ev_lists_) (void)hipEventDestroy(ev_lists_);
    if (ev_side_) (void)hipEventDestroy(ev_side_);
    if (side_) (void)hipStreamDestroy(side_);
}

// Factor storage per slot: FP64-sized in both forms, since an FP32-LU cell can
// fall back to FP64 factors.
size_t Engine::bytes_per_slot(const DeviceNet &dn, int prec) {
    (void)prec;
    const size_t S = dn.S, R = dn.R, NP = dn.NP;
    return sizeof(SlotCtl) + 5 * sizeof(double) + R * sizeof(double) + kDRows * S * sizeof(double) +
           6 * S * sizeof(double) + size_t(std::max(dn.nnzJ, 1)) * sizeof(double) + lu_bytes(int(NP), ABDF_PREC_FP64) +
           dinv_bytes(int(NP), ABDF_PREC_FP64) +
           NP * sizeof(int32_t) + 7 * sizeof(int32_t) + sizeof(long long);
}

int Engine::set_options(const abdf_options &o, std::string &err, double *atol_host) {
    set_lu_reuse(o.lu_reuse);
    set_max_order(o.max_order);
    set_step_bounds(o.h0, o.h_max);
    method_ = o.method;
    s_.method = method_;
    s_.newton_maxiter = method_ == ABDF_METHOD_ESDIRK5 ? kRkNewtonMaxIter : kNewtonMaxIter;
    tvar_ = o.phi_tc != nullptr;
    for (int j = 0; j < 5; ++j) phi_exp_[j] = o.phi_exp[j];
    s_.tvar = tvar_;
    for (int j = 0; j < 5; ++j) s_.phi_exp[j] = phi_exp_[j];
    atol_sp_ = nullptr;
    if (o.atol_species) {
        if (dn_.S > kMaxSpecies) {
            err = "network too large";
            return ABDF_E_ARG;
        }
        double *h = atol_host;
        if (!h) {
            atol_store_.resize(size_t(dn_.S));
            h = atol_store_.data();
        }
        HIP_TRY(hipMemcpy(h, o.atol_species, size_t(dn_.S) * sizeof(double), hipMemcpyDeviceToHost));
        for (int i = 0; i < dn_.S; ++i)
            if (!(h[i] >= 0.0) || !std::isfinite(h[i])) {
                err = "atol_species entries must be finite and >= 0";
                return ABDF_E_ARG;
            }
        atol_sp_ = h;
    }
    return ABDF_OK;
}

namespace {
// The slot arrays of n slots in the order init lays them out (each part
// 256-byte aligned).
struct Layout {
    size_t bytes[22];
    static constexpr int kParts = 22;
    Layout(const DeviceNet &dn, size_t n) {
        const size_t S = dn.S, R = dn.R, NP = dn.NP;
        const size_t lu_stride = lu_bytes(int(NP), ABDF_PREC_FP64), dinv_stride = dinv_bytes(int(NP), ABDF_PREC_FP64);
        const size_t b[kParts] = {
            n * sizeof(SlotCtl), n * 5 * sizeof(double), n * R * sizeof(double), n * kDRows * S * sizeof(double),
            n * S * sizeof(double), n * S * sizeof(double), n * S * sizeof(double), n * S * sizeof(double),
            n * S * sizeof(double), n * S * sizeof(double), n * size_t(std::max(dn.nnzJ, 1)) * sizeof(double),
            n * lu_stride, n * dinv_stride, n * NP * sizeof(int32_t), 3 * n * sizeof(int32_t),
            3 * n * sizeof(int32_t), 3 * n * sizeof(int32_t), n * sizeof(int32_t), kCountSlots * sizeof(int32_t),
            n * sizeof(int32_t), n * sizeof(long long), S * sizeof(double)};
        for (int i = 0; i < kParts; ++i) bytes[i] = b[i];
    }
    size_t total() const {
        size_t t = 0;
        for (size_t b : bytes) t += align256(b);
        return t;
    }
};
}  // namespace

size_t Engine::workspace_bytes(const DeviceNet &dn, long long n) { return Layout(dn, size_t(n)).total(); }

// Points the slot arrays into base (workspace_bytes(nslots) bytes) and sets
// the launch shapes.
int Engine::layout(int nslots, void *base, std::string &err) {
    const size_t n = size_t(nslots), S = dn_.S, NP = dn_.NP;
    const Layout lay(dn_, n);
    void *part[Layout::kParts];
    size_t off = 0;
    for (int i = 0; i < Layout::kParts; ++i) {
        part[i] = static_cast<char *>(base) + off;
        off += align256(lay.bytes[i]);
    }
    s_.nslots = nslots;
    s_.S = dn_.S;
    s_.R = dn_.R;
    s_.NP = dn_.NP;
    s_.prec = prec_;
    s_.max_steps = max_steps_;
    s_.ctl = static_cast<SlotCtl *>(part[0]);
    s_.phi = static_cast<double *>(part[1]);
    s_.k = static_cast<double *>(part[2]);
    s_.D = static_cast<double *>(part[3]);
    s_.x = static_cast<double *>(part[4]);
    s_.d = static_cast<double *>(part[5]);
    s_.psi = static_cast<double *>(part[6]);
    s_.scl = static_cast<double *>(part[7]);
    s_.xJ = static_cast<double *>(part[8]);
    s_.rb = static_cast<double *>(part[9]);
    s_.jval = static_cast<double *>(part[10]);
    s_.lu = part[11];
    s_.dinv = part[12];
    s_.lu_stride = lu_bytes(int(NP), ABDF_PREC_FP64);
    s_.dinv_stride = dinv_bytes(int(NP), ABDF_PREC_FP64);
    s_.perm = static_cast<int32_t *>(part[13]);
    s_.act = static_cast<int32_t *>(part[14]);
    s_.lul = static_cast<int32_t *>(part[15]);
    s_.nol = static_cast<int32_t *>(part[16]);
    s_.fin = static_cast<int32_t *>(part[17]);
    s_.cnt = static_cast<int32_t *>(part[18]);
    d_admit_slots_ = static_cast<int32_t *>(part[19]);
    d_admit_cells_ = static_cast<long long *>(part[20]);
    s_.lu_reuse = lu_reuse_;
    s_.max_order = max_order_;
    s_.h0 = h0_;
    s_.h_max = h_max_;
    s_.method = method_;
    s_.newton_maxiter = method_ == ABDF_METHOD_ESDIRK5 ? kRkNewtonMaxIter : kNewtonMaxIter;
    s_.tvar = tvar_;
    for (int j = 0; j < 5; ++j) s_.phi_exp[j] = phi_exp_[j];
    s_.atol_sp = nullptr;
    if (atol_sp_) {
        HIP_TRY(hipMemcpy(part[21], atol_sp_, S * sizeof(double), hipMemcpyHostToDevice));
        s_.atol_sp = static_cast<const double *>(part[21]);
    }
    lds_admit_ = admit_lds(dn_);
    lds_factor_ = factor_lds(dn_, ABDF_PREC_FP64);
    lds_factor32_ = factor_lds(dn_, ABDF_PREC_FP32_LU);
    lds_newton_ = newton_lds(dn_);
    lds_solve_ = solve_lds(dn_);
    lds_solve32_ = solve_lds32(dn_);
    if (dn_.NP > 512 || lds_admit_ > kMaxLds || lds_factor_ > kMaxLds || lds_newton_ > kMaxLds ||
        lds_solve32_ > kMaxLds) {
        err = "network too large for one workgroup's LDS";
        return ABDF_E_ARG;
    }
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    const bool f32 = prec_ == ABDF_PREC_FP32_LU;
    grid_factor64_max_ = cus * resident_per_cu(0, ABDF_PREC_FP64, lds_factor_);
    grid_solve64_max_ = cus * resident_per_cu(2, ABDF_PREC_FP64, lds_solve_);
    grid_factor_max_ = f32 ? cus * resident_per_cu(0, prec_, lds_factor32_) : grid_factor64_max_;
    grid_newton_max_ = cus * newton_rhs_resident_per_cu(dn_, prec_, lds_newton_);
    grid_solve_max_ = f32 ? cus * resident_per_cu(2, prec_, lds_solve_) : grid_solve64_max_;
    grid_solve_ref_max_ = cus * resident_per_cu(4, prec_, lds_solve32_);
    grid_adj_solve_max_ = cus * resident_per_cu(3, prec_, adj_solve_lds(dn_));
    n_free_ = 0;
    for (int i = nslots - 1; i >= 0; --i) free_[n_free_++] = i;
    (void)n;
    return ABDF_OK;
}

int Engine::init(int nslots, std::string &err, bool cache_workspace) {
    const size_t n = size_t(nslots);
    const size_t total = workspace_bytes(dn_, nslots);
    cached_ = cache_workspace;
    base_ = cached_ ? net_.take_workspace(dn_.device, total, &base_bytes_) : nullptr;
    if (!base_) {
        hipError_t e = hipMalloc(&base_, total);
        if (e != hipSuccess) {
            base_ = nullptr;
            err = "device workspace of " + std::to_string(total) + " bytes: " + hipGetErrorString(e);
            return ABDF_E_NOMEM;
        }
        base_bytes_ = total;
    }
    free_store_.resize(n);
    free_ = free_store_.data();
    int rc = layout(nslots, base_, err);
    if (rc != ABDF_OK) return rc;
    HIP_TRY(hipMemset(s_.cnt, 0, kCountSlots * sizeof(int32_t)));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_cnt_), kCountSlots * sizeof(int32_t), hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ev_lists_, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ev_side_, hipEventDisableTiming));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_fin_), n * sizeof(int32_t), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_admit_slots_), n * sizeof(int32_t), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h_admit_cells_), n * sizeof(long long), hipHostMallocDefault));
    return ABDF_OK;
}

int Engine::init_external(int nslots, void *base, size_t bytes, const HostBuffers &hb, std::string &err) {
    ext_ = true;
    if (nslots < 1 || nslots > hb.max_slots || workspace_bytes(dn_, nslots) > bytes) {
        err = "slot count beyond the external workspace";
        return ABDF_E_ARG;
    }
    base_ = base;
    base_bytes_ = bytes;
    free_ = hb.free_list;
    h_cnt_ = hb.cnt;
    h_fin_ = hb.fin;
    h_admit_slots_ = hb.admit_slots;
    h_admit_cells_ = hb.admit_cells;
    return layout(nslots, base, err);
}

int Engine::reset_counts(hipStream_t st, std::string &err) {
    HIP_TRY(launch_fill_i32(s_.cnt, 0, kCountSlots, st));
    return ABDF_OK;
}

double Engine::newton_tolerance(const abdf_options &opt) {
    return opt.newton_tol > 0 ? opt.newton_tol
                              : std::max(10.0 * kURound / opt.rtol, std::min(0.03, std::sqrt(opt.rtol)));
}

int Engine::admit_cells(const AdmitArgs &a, hipStream_t st, std::string &err) {
    if (a.count <= 0) return ABDF_OK;
    TraceRange tr("abdf admit");
    hipEvent_t t0 = timer_begin(st);
    HIP_TRY(launch_admit(s_, dn_, a, ring_, lds_admit_, st));
    timer_end(ABDF_PROF_ADMIT, t0, st);
    bound_ += a.count;
    return ABDF_OK;
}

int Engine::admit(const BatchIO &io, const abdf_options &opt, long long &next, hipStream_t st, std::string &err) {
    const long long want = std::min<long long>(static_cast<long long>(n_free_), io.n_cells - next);
    if (want <= 0) return ABDF_OK;
    for (long long i = 0; i < want; ++i) {
        h_admit_slots_[i] = take_slot();
        h_admit_cells_[i] = next + i;
    }
    HIP_TRY(hipMemcpyAsync(d_admit_slots_, h_admit_slots_, want * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_admit_cells_, h_admit_cells_, want * sizeof(long long), hipMemcpyHostToDevice, st));
    AdmitArgs a{};
    a.count = int(want);
    a.slots = d_admit_slots_;
    a.cells = d_admit_cells_;
    a.T = io.T;
    a.nH = io.nH;
    a.Av = io.Av;
    a.zeta = io.zeta;
    a.G0 = io.G0;
    a.x0 = io.x0;
    a.t_end = io.t_end;
    a.rtol = opt.rtol;
    a.atol = opt.atol;
    a.newton_tol = newton_tolerance(opt);
    a.tc = opt.phi_tc;
    // the pinned admission buffers are rewritten only after the next poll's synchronisation
    next += want;
    return admit_cells(a, st, err);
}

int Engine::newton_iterations(int which, hipStream_t st, std::string &err) {
    for (int m = 0; m < s_.newton_maxiter; ++m) {
        hipEvent_t t0 = timer_begin(st);
        HIP_TRY(launch_newton_rhs(s_, dn_, ring_, which, std::min(bound_, grid_newton_max_), lds_newton_, st));
        timer_end(which == kListNoFactor ? ABDF_PROF_RHS_SIDE : ABDF_PROF_RHS, t0, st);
        t0 = timer_begin(st);
        HIP_TRY(launch_newton_solve(s_, dn_, ring_, which, std::min(bound_, grid_solve_max_),
                                    std::min(bound_, grid_solve_ref_max_), lds_solve_, lds_solve32_, st));
        timer_end(which == kListNoFactor ? ABDF_PROF_NEWTON_SIDE : ABDF_PROF_NEWTON, t0, st);
    }
    return ABDF_OK;
}

hipError_t Engine::control(hipStream_t st) {
    return method_ == ABDF_METHOD_ESDIRK5 ? launch_control_rk(s_, ring_, bound_, st)
                                          : launch_control(s_, dn_, ring_, bound_, st);
}

// Below this many occupied slots an attempt runs on one stream.
constexpr int kSplitMinSlots = 32;

// One step attempt.  The slots whose factorisation is current iterate on the
// side stream while the others are factored on st: the factorisation kernel is
// LDS-bound at a few workgroups per CU and leaves CUs idle in its last round,
// which the side stream's kernels fill.  Control waits for both streams.
int Engine::attempt(hipStream_t st, std::string &err) {
    if (bound_ <= 0) return ABDF_OK;
    TraceRange tr("abdf attempt");
    if (bound_ < kSplitMinSlots || !side_) {
        // a handful of cells: launch latency dominates, one stream
        hipEvent_t t0 = timer_begin(st);
        HIP_TRY(launch_factor(s_, dn_, ring_, std::min(bound_, grid_factor_max_),
                              std::min(bound_, grid_factor64_max_), lds_factor_, lds_factor32_, st));
        timer_end(ABDF_PROF_FACTOR, t0, st);
        if (prec_ == ABDF_PREC_FP64) {
            t0 = timer_begin(st);
            HIP_TRY(launch_newton_fused(s_, dn_, ring_, kListAll, bound_, std::max(lds_newton_, lds_solve_), st));
            timer_end(ABDF_PROF_NEWTON, t0, st);
        } else {
            int rc = newton_iterations(kListAll, st, err);
            if (rc != ABDF_OK) return rc;
        }
        t0 = timer_begin(st);
        HIP_TRY(control(st));
        timer_end(ABDF_PROF_CONTROL, t0, st);
        ring_ = (ring_ + 1) % 3;
        return ABDF_OK;
    }
    HIP_TRY(hipEventRecord(ev_lists_, st));
    hipEvent_t t0 = timer_begin(st);
    HIP_TRY(launch_factor(s_, dn_, ring_, std::min(bound_, grid_factor_max_), std::min(bound_, grid_factor64_max_),
                          lds_factor_, lds_factor32_, st));
    timer_end(ABDF_PROF_FACTOR, t0, st);
    HIP_TRY(hipStreamWaitEvent(side_, ev_lists_, 0));
    int rc = newton_iterations(kListNoFactor, side_, err);
    if (rc != ABDF_OK) return rc;
    HIP_TRY(hipEventRecord(ev_side_, side_));
    rc = newton_iterations(kListFactor, st, err);
    if (rc != ABDF_OK) return rc;
    HIP_TRY(hipStreamWaitEvent(st, ev_side_, 0));
    t0 = timer_begin(st);
    HIP_TRY(control(st));
    timer_end(ABDF_PROF_CONTROL, t0, st);
    ring_ = (ring_ + 1) % 3;
    return ABDF_OK;
}

int Engine::sync_counts(hipStream_t st, int &nfin, std::string &err) {
    TraceRange tr("abdf poll");
    HIP_TRY(hipMemcpyAsync(h_cnt_, s_.cnt, kCountSlots * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    flush_timers();
    nfin = h_cnt_[6];
    bound_ = h_cnt_[ring_];
    return ABDF_OK;
}

int Engine::harvest(HarvestArgs h, hipStream_t st, std::string &err) {
    const int nfin = h.count;
    if (nfin <= 0) return ABDF_OK;
    TraceRange tr("abdf harvest");
    HIP_TRY(hipMemcpyAsync(h_fin_, s_.fin, nfin * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    h.slots = s_.fin;
    hipEvent_t t0 = timer_begin(st);
    HIP_TRY(launch_harvest(s_, h, st));
    timer_end(ABDF_PROF_HARVEST, t0, st);
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < nfin; ++i) free_[n_free_++] = h_fin_[i];
    return ABDF_OK;
}

int Engine::solve(const BatchIO &io, const abdf_options &opt, hipStream_t st, std::string &err) {
    TraceRange tr("abdf solve");
    ring_ = 0;
    bound_ = 0;
    long long next = 0;
    {
        // the slot lists start empty: an external workspace keeps the previous
        // call's contents, and an engine's earlier sweep leaves its last ring's counts
        int rc0 = reset_counts(st, err);
        if (rc0 != ABDF_OK) return rc0;
    }
    const int check_every = std::max(1, opt.check_every);
    int rc = admit(io, opt, next, st, err);
    if (rc != ABDF_OK) return rc;
    int since_poll = 0;
    while (true) {
        if (bound_ > 0) {
            rc = attempt(st, err);
            if (rc != ABDF_OK) return rc;
            ++since_poll;
        }
        if (bound_ == 0 || since_poll >= check_every) {
            since_poll = 0;
            int nfin = 0;
            rc = sync_counts(st, nfin, err);
            if (rc != ABDF_OK) return rc;
            HarvestArgs h{};
            h.count = nfin;
            h.x_out = io.x_out;
            h.status = io.status;
            h.stats = io.stats;
            rc = harvest(h, st, err);
            if (rc != ABDF_OK) return rc;
            rc = admit(io, opt, next, st, err);
            if (rc != ABDF_OK) return rc;
            if (bound_ == 0 && next >= io.n_cells) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(st));
    flush_timers();
    return ABDF_OK;
}

int Engine::reverse(const AdjIO &io, int check_every, hipStream_t st, std::string &err) {
    TraceRange tr("abdf reverse sweep");
    ring_ = 0;
    bound_ = 0;
    {
        int rc0 = reset_counts(st, err);
        if (rc0 != ABDF_OK) return rc0;
    }
    const size_t lds_adj = adj_lds(dn_), lds_adj_solve = adj_solve_lds(dn_);
    if (lds_adj > kMaxLds || lds_adj_solve > kMaxLds) {
        err = "network too large for one workgroup's LDS";
        return ABDF_E_ARG;
    }
    check_every = std::max(1, check_every);
    long long next = 0;
    auto admit_rev = [&]() -> int {
        const long long want = std::min<long long>(static_cast<long long>(n_free_), io.n_cells - next);
        if (want <= 0) return ABDF_OK;
        for (long long i = 0; i < want; ++i) {
            h_admit_slots_[i] = take_slot();
            h_admit_cells_[i] = next + i;
        }
        HIP_TRY(hipMemcpyAsync(d_admit_slots_, h_admit_slots_, want * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_admit_cells_, h_admit_cells_, want * sizeof(long long), hipMemcpyHostToDevice, st));
        AdjArgs a{int(want), d_admit_slots_, d_admit_cells_, io.phi, io.dLdx, io.status};
        hipEvent_t t0 = timer_begin(st);
        HIP_TRY(launch_adj_admit(s_, dn_, a, ring_, lds_adj, st));
        timer_end(ABDF_PROF_ADMIT, t0, st);
        next += want;
        bound_ += int(want);
        return ABDF_OK;
    };
    int rc = admit_rev();
    if (rc != ABDF_OK) return rc;
    int since = 0;
    while (true) {
        if (bound_ > 0) {
            TraceRange ts("abdf reverse step");
            hipEvent_t t0 = timer_begin(st);
            HIP_TRY(launch_factor(s_, dn_, ring_, std::min(bound_, grid_factor_max_),
                                  std::min(bound_, grid_factor64_max_), lds_factor_, lds_factor32_, st));
            timer_end(ABDF_PROF_FACTOR, t0, st);
            t0 = timer_begin(st);
            HIP_TRY(launch_adj_solve(s_, ring_, std::min(bound_, grid_adj_solve_max_), lds_adj_solve, st));
            timer_end(ABDF_PROF_ADJ_SOLVE, t0, st);
            t0 = timer_begin(st);
            HIP_TRY(launch_adj_step(s_, dn_, ring_, bound_, lds_adj, st));
            timer_end(ABDF_PROF_ADJ_STEP, t0, st);
            ring_ = (ring_ + 1) % 3;
            ++since;
        }
        if (bound_ == 0 || since >= check_every) {
            since = 0;
            int nfin = 0;
            rc = sync_counts(st, nfin, err);
            if (rc != ABDF_OK) return rc;
            if (nfin > 0) {
                HIP_TRY(hipMemcpyAsync(h_fin_, s_.fin, nfin * sizeof(int32_t), hipMemcpyDeviceToHost, st));
                AdjHarvestArgs h{nfin, s_.fin, io.g_cell, io.dx0, io.dphi};
                hipEvent_t t0 = timer_begin(st);
                HIP_TRY(launch_adj_harvest(s_, dn_, h, st));
                timer_end(ABDF_PROF_HARVEST, t0, st);
                HIP_TRY(hipStreamSynchronize(st));
                for (int i = 0; i < nfin; ++i) free_[n_free_++] = h_fin_[i];
            }
            rc = admit_rev();
            if (rc != ABDF_OK) return rc;
            if (bound_ == 0 && next >= io.n_cells) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(st));
    flush_timers();
    return ABDF_OK;
}

}  // namespace abdf
