// Step tape and discrete adjoint (see adjoint.hpp).
#include "adjoint.hpp"

#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace abdf {

#define HIP_TRY(expr)                                                           \
    do {                                                                        \
        hipError_t e__ = (expr);                                                \
        if (e__ != hipSuccess) {                                                \
            err = std::string(#expr ": ") + hipGetErrorString(e__);            \
            return ABDF_E_DEVICE;                                               \
        }                                                                       \
    } while (0)

Tape::~Tape() {
    eng_.reset();
    if (base_) (void)hipFree(base_);
    if (g_slots_) (void)hipFree(g_slots_);
    if (win_base_) (void)hipFree(win_base_);
}

int Tape::record(const BatchIO &io, const double *alpha, const abdf_options &opt, int cap, hipStream_t st,
                 std::string &err) {
    opt_ = opt;
    C_ = io.n_cells;
    cap_ = cap;
    const size_t C = size_t(C_), S = size_t(dn_.S), R = size_t(dn_.R);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_alpha = al(R * 8), b_phi = al(C * 5 * 8), b_x0 = al(C * S * 8), b_st = al(C * 4),
                 b_len = al(C * 4), b_tx = al(C * size_t(cap) * S * 8), b_th = al(C * size_t(cap) * 8),
                 b_tq = al(C * size_t(cap) * 4), b_phis = al(5 * C * 8), b_tend = al(C * 8), b_hp = al(C * 8),
                 b_qp = al(C * 4);
    const size_t total = b_alpha + b_phi + b_x0 + b_st + b_len + b_tx + b_th + b_tq + b_phis + b_tend + b_hp + b_qp;
    if (opt.hbm_budget_bytes > 0 && total >= opt.hbm_budget_bytes) {
        err = "the step tape alone (" + std::to_string(total) + " bytes) exceeds the workspace budget";
        return ABDF_E_BUDGET;
    }
    if (hipMalloc(&base_, total) != hipSuccess) {
        base_ = nullptr;
        err = "step tape of " + std::to_string(total) + " bytes";
        return ABDF_E_NOMEM;
    }
    bytes_ = total;
    char *p = static_cast<char *>(base_);
    alpha_ = reinterpret_cast<double *>(p);
    p += b_alpha;
    phi_ = reinterpret_cast<double *>(p);
    p += b_phi;
    x0_ = reinterpret_cast<double *>(p);
    p += b_x0;
    status_ = reinterpret_cast<int32_t *>(p);
    p += b_st;
    len_ = reinterpret_cast<int32_t *>(p);
    p += b_len;
    tape_x_ = reinterpret_cast<double *>(p);
    p += b_tx;
    tape_h_ = reinterpret_cast<double *>(p);
    p += b_th;
    tape_q_ = reinterpret_cast<int32_t *>(p);
    p += b_tq;
    phis_ = reinterpret_cast<double *>(p);
    p += b_phis;
    t_end_ = reinterpret_cast<double *>(p);
    p += b_tend;
    hprev_ = reinterpret_cast<double *>(p);
    p += b_hp;
    qprev_ = reinterpret_cast<int32_t *>(p);
    HIP_TRY(hipMemcpyAsync(alpha_, alpha ? alpha : dn_.alpha, R * 8, hipMemcpyDeviceToDevice, st));
    dn_.alpha = alpha_;
    const double *cols[5] = {io.T, io.nH, io.Av, io.zeta, io.G0};
    for (int j = 0; j < 5; ++j) {
        HIP_TRY(hipMemcpy2DAsync(phi_ + j, 5 * 8, cols[j], 8, 8, C, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(phis_ + size_t(j) * C, cols[j], C * 8, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(t_end_, io.t_end, C * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(x0_, io.x0, C * S * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(len_, 0, C * 4, st));

    // slots: what remains of the budget and of the free memory after the tape
    const size_t per = Engine::bytes_per_slot(dn_, opt.precision) + R * 8;
    long long nslots = C_;
    if (opt.hbm_budget_bytes > 0) nslots = std::min<long long>(nslots, (long long)((opt.hbm_budget_bytes - total) / per));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
        nslots = std::min<long long>(nslots, (long long)(0.85 * double(free_b) / double(per)));
    if (nslots < 1) {
        err = "not even one cell fits in the workspace budget beside the step tape";
        return ABDF_E_BUDGET;
    }
    if (hipMalloc(&g_slots_, size_t(nslots) * R * 8) != hipSuccess) {
        g_slots_ = nullptr;
        err = "reverse-sweep gradient slots";
        return ABDF_E_NOMEM;
    }
    eng_ = std::make_unique<Engine>(net_, dn_, opt.precision, opt.max_steps);
    int rc = eng_->set_options(opt, err);
    if (rc != ABDF_OK) return rc;
    rc = eng_->init(int(nslots), err);
    if (rc != ABDF_OK) return rc;
    Slots &s = eng_->slots();
    s.tape_cap = cap;
    s.tape_x = tape_x_;
    s.tape_h = tape_h_;
    s.tape_q = tape_q_;
    s.tape_len = len_;
    s.tape_x0 = x0_;
    s.g = static_cast<double *>(g_slots_);
    s.tape_hprev = hprev_;
    s.tape_qprev = qprev_;
    s.tape_overflow = 1;   // steps past the tape are integrated on, and swept in windows
    rc = eng_->solve(io, opt, st, err);
    if (rc != ABDF_OK) return rc;
    HIP_TRY(hipMemcpyAsync(status_, io.status, C * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ABDF_OK;
}

int Tape::adjoint(const double *dLdx, double *g_sum, double *g_cell, double *dx0, double *dphi, hipStream_t st,
                  std::string &err) {
    const size_t R = size_t(dn_.R);
    double *gc = g_cell;
    void *tmp = nullptr;
    if (!gc && g_sum) {
        if (hipMalloc(&tmp, std::max<size_t>(1, size_t(C_) * R * 8)) != hipSuccess) {
            err = "per-cell gradient scratch";
            return ABDF_E_NOMEM;
        }
        gc = static_cast<double *>(tmp);
    }
    AdjIO io{C_, phi_, dLdx, status_, gc, dx0, dphi};
    int rc = windowed_sweep(io, st, err);
    hipError_t e = hipSuccess;
    if (rc == ABDF_OK && g_sum) e = launch_grad_sum(gc, C_, int(R), g_sum, st);
    if (rc == ABDF_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    if (tmp) (void)hipFree(tmp);
    if (rc != ABDF_OK) return rc;
    if (e != hipSuccess) {
        err = std::string("gradient sum: ") + hipGetErrorString(e);
        return ABDF_E_DEVICE;
    }
    return ABDF_OK;
}

// The reverse sweep: one pass when every differentiated cell fits in the tape,
// else one pass per window (see adjoint.hpp).
int Tape::windowed_sweep(const AdjIO &io, hipStream_t st, std::string &err) {
    const size_t C = size_t(C_), S = size_t(dn_.S), R = size_t(dn_.R);
    std::vector<int32_t> len(C), status(C);
    HIP_TRY(hipMemcpyAsync(len.data(), len_, C * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(status.data(), status_, C * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool over = false;
    for (size_t c = 0; c < C; ++c) over |= status[c] == ABDF_CELL_OK && len[c] > cap_;
    Slots &s = eng_->slots();
    if (!over) return eng_->reverse(io, opt_.check_every, st, err);

    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_i = al(C * 4), b_lam = al(C * kDRows * S * 8), b_g = al(C * R * 8), b_x = al(C * S * 8);
    const size_t need = 4 * b_i + b_lam + b_g + b_x;
    if (!win_base_) {
        if (hipMalloc(&win_base_, need) != hipSuccess) {
            win_base_ = nullptr;
            err = "windowed sweep buffers of " + std::to_string(need) + " bytes";
            return ABDF_E_NOMEM;
        }
        win_bytes_ = need;
    }
    char *p = static_cast<char *>(win_base_);
    int32_t *d_w0 = reinterpret_cast<int32_t *>(p);
    int32_t *d_stop = reinterpret_cast<int32_t *>(p + b_i);
    int32_t *d_end = reinterpret_cast<int32_t *>(p + 2 * b_i);
    int32_t *d_rst = reinterpret_cast<int32_t *>(p + 3 * b_i);
    double *d_lam = reinterpret_cast<double *>(p + 4 * b_i);
    double *d_g = reinterpret_cast<double *>(p + 4 * b_i + b_lam);
    double *d_x = reinterpret_cast<double *>(p + 4 * b_i + b_lam + b_g);

    // w1: end of the window still to sweep (-1: done); holds: the window start
    // the cell's tape rows hold (0 after the recording).  A cell whose forward
    // solve failed takes the first pass with no steps, which writes its zeros.
    std::vector<int32_t> w1(C), holds(C, 0), w0(C), stop(C), end(C);
    for (size_t c = 0; c < C; ++c) w1[c] = status[c] == ABDF_CELL_OK ? len[c] : 0;
    int rc = ABDF_OK;
    for (int pass = 0;; ++pass) {
        bool active = false, rerun = false;
        for (size_t c = 0; c < C; ++c) {
            const bool in = w1[c] > 0 || (pass == 0 && w1[c] == 0);
            w0[c] = in && w1[c] > 0 ? (w1[c] - 1) / cap_ * cap_ : 0;
            end[c] = in ? w1[c] : -1;
            stop[c] = 0;
            if (in && holds[c] != w0[c]) {
                stop[c] = w1[c];
                holds[c] = w0[c];
                rerun = true;
            }
            active |= in;
        }
        if (!active) break;
        HIP_TRY(hipMemcpyAsync(d_w0, w0.data(), C * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_stop, stop.data(), C * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_end, end.data(), C * 4, hipMemcpyHostToDevice, st));
        s.tape_w0 = d_w0;
        if (rerun) {
            // forward re-run: each listed cell records its window and stops at its end
            s.tape_stop = d_stop;
            int32_t *keep_len = s.tape_len;
            s.tape_len = nullptr;
            BatchIO fio{C_, phis_, phis_ + C, phis_ + 2 * C, phis_ + 3 * C, phis_ + 4 * C, x0_, t_end_,
                        d_x, d_rst, nullptr};
            rc = eng_->solve(fio, opt_, st, err);
            s.tape_stop = nullptr;
            s.tape_len = keep_len;
            if (rc != ABDF_OK) break;
            // the re-run repeats the recorded solve, so each re-run cell ends OK
            std::vector<int32_t> rst(C);
            HIP_TRY(hipMemcpy(rst.data(), d_rst, C * 4, hipMemcpyDeviceToHost));
            for (size_t c = 0; c < C; ++c)
                if (stop[c] > 0 && rst[c] != ABDF_CELL_OK) {
                    err = "forward re-run of cell " + std::to_string(c) + " did not repeat the recorded solve";
                    rc = ABDF_E_DEVICE;
                }
            if (rc != ABDF_OK) break;
        }
        s.win_end = d_end;
        s.win_lam = d_lam;
        s.win_g = d_g;
        s.win_resume = pass > 0;
        rc = eng_->reverse(io, opt_.check_every, st, err);
        if (rc != ABDF_OK) break;
        for (size_t c = 0; c < C; ++c)
            if (end[c] >= 0) w1[c] = w0[c] > 0 ? w0[c] : -1;
    }
    // the slots go back to single-window sweeps of the recorded tape rows,
    // which the re-runs have overwritten for the cells that took part
    s.tape_w0 = nullptr;
    s.win_end = nullptr;
    s.win_lam = nullptr;
    s.win_g = nullptr;
    s.win_resume = 0;
    return rc;
}

}  // namespace abdf
