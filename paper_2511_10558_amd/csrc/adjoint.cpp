// Step tape and discrete adjoint (see adjoint.hpp).
#include "adjoint.hpp"

#include <algorithm>

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
                 b_tq = al(C * size_t(cap) * 4);
    const size_t total = b_alpha + b_phi + b_x0 + b_st + b_len + b_tx + b_th + b_tq;
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
    HIP_TRY(hipMemcpyAsync(alpha_, alpha ? alpha : dn_.alpha, R * 8, hipMemcpyDeviceToDevice, st));
    dn_.alpha = alpha_;
    const double *cols[5] = {io.T, io.nH, io.Av, io.zeta, io.G0};
    for (int j = 0; j < 5; ++j)
        HIP_TRY(hipMemcpy2DAsync(phi_ + j, 5 * 8, cols[j], 8, 8, C, hipMemcpyDeviceToDevice, st));
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
    int rc = eng_->reverse(io, opt_.check_every, st, err);
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

}  // namespace abdf
