// C-ABI entry points (include/astrobdf.h): argument checks, error reporting,
// workspace sizing and dispatch to the engine and the component kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <fstream>
#include <memory>
#include <new>
#include <sstream>
#include <string>

#include "../../include/astrobdf.h"
#include "engine.hpp"
#include "kernels.hpp"
#include "network.hpp"

struct abdf_network {
    abdf::HostNetwork host;
};

namespace {

thread_local std::string g_last_error;

abdf_status fail(abdf_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

abdf_status ok() {
    g_last_error.clear();
    return ABDF_OK;
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

#define CHECK_DEV(p, name)                                                          \
    do {                                                                            \
        if (!is_device_ptr(p)) return fail(ABDF_E_ARG, std::string(name) + " is not a device pointer"); \
    } while (0)

#define HIP_OR_FAIL(expr)                                                           \
    do {                                                                            \
        hipError_t e__ = (expr);                                                    \
        if (e__ != hipSuccess) return fail(ABDF_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e__)); \
    } while (0)

abdf_status check_opts(const abdf_options &o) {
    if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(ABDF_E_ARG, "rtol must be finite and > 0");
    if (!(o.atol >= 0.0) || !std::isfinite(o.atol)) return fail(ABDF_E_ARG, "atol must be finite and >= 0");
    if (o.max_steps < 1) return fail(ABDF_E_ARG, "max_steps must be >= 1");
    if (o.precision != ABDF_PREC_FP64 && o.precision != ABDF_PREC_FP32_LU)
        return fail(ABDF_E_ARG, "unknown precision");
    if (o.newton_tol < 0.0 || !std::isfinite(o.newton_tol)) return fail(ABDF_E_ARG, "newton_tol must be >= 0");
    return ABDF_OK;
}

}  // namespace

extern "C" {

void abdf_options_default(abdf_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->rtol = 1e-6;
    opt->atol = 1e-20;
    opt->max_steps = 100000;
    opt->precision = ABDF_PREC_FP64;
    opt->check_every = 8;
    opt->hbm_budget_bytes = 0;
    opt->newton_tol = 0.0;
}

const char *abdf_last_error(void) { return g_last_error.c_str(); }

abdf_status abdf_network_load_mem(const char *text, size_t len, abdf_network **out) {
    if (!text || !out) return fail(ABDF_E_ARG, "null argument");
    *out = nullptr;
    try {
        auto net = std::make_unique<abdf_network>();
        std::string err;
        int rc = net->host.parse(text, len, err);
        if (rc != ABDF_OK) return fail(static_cast<abdf_status>(rc), err);
        *out = net.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(ABDF_E_PARSE, e.what());
    }
}

abdf_status abdf_network_load(const char *path, abdf_network **out) {
    if (!path || !out) return fail(ABDF_E_ARG, "null argument");
    *out = nullptr;
    std::ifstream in(path, std::ios::binary);
    if (!in) return fail(ABDF_E_IO, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    return abdf_network_load_mem(text.data(), text.size(), out);
}

void abdf_network_free(abdf_network *net) { delete net; }

int32_t abdf_network_num_species(const abdf_network *net) { return net ? net->host.S : -1; }
int32_t abdf_network_num_reactions(const abdf_network *net) { return net ? net->host.R : -1; }
int32_t abdf_network_num_elements(const abdf_network *net) { return net ? net->host.E : -1; }

const char *abdf_network_species_name(const abdf_network *net, int32_t i) {
    if (!net || i < 0 || i >= net->host.S) return nullptr;
    return net->host.species[i].c_str();
}

abdf_status abdf_solve(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                       const double *A_V, const double *zeta, const double *G0, const double *x0,
                       const double *t_end, const abdf_options *opt, double *x_out, int32_t *cell_status,
                       abdf_cell_stats *stats, void *stream) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    abdf_options o;
    if (opt) o = *opt; else abdf_options_default(&o);
    abdf_status rc = check_opts(o);
    if (rc != ABDF_OK) return rc;
    if (n_cells == 0) return ok();
    CHECK_DEV(T, "T");
    CHECK_DEV(n_H, "n_H");
    CHECK_DEV(A_V, "A_V");
    CHECK_DEV(zeta, "zeta");
    CHECK_DEV(G0, "G0");
    CHECK_DEV(x0, "x0");
    CHECK_DEV(t_end, "t_end");
    CHECK_DEV(x_out, "x_out");
    CHECK_DEV(cell_status, "cell_status");
    if (stats) CHECK_DEV(stats, "stats");
    try {
        std::string err;
        const abdf::DeviceNet *dn = net->host.device_tables(err);
        if (!dn) return fail(ABDF_E_DEVICE, err);
        const size_t per = abdf::Engine::bytes_per_slot(*dn, o.precision);
        long long nslots = n_cells;
        if (o.hbm_budget_bytes > 0) nslots = std::min<long long>(nslots, (long long)(o.hbm_budget_bytes / per));
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
            nslots = std::min<long long>(nslots, (long long)(0.85 * double(free_b) / double(per)));
        if (nslots < 1) return fail(ABDF_E_BUDGET, "not even one cell fits in the workspace budget");
        abdf::Engine eng(net->host, *dn, o.precision, o.max_steps);
        int r = eng.init(int(nslots), err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        abdf::BatchIO io{n_cells, T, n_H, A_V, zeta, G0, x0, t_end, x_out, cell_status, stats};
        r = eng.solve(io, o, static_cast<hipStream_t>(stream), err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(ABDF_E_DEVICE, e.what());
    }
}

abdf_status abdf_rates(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                       const double *A_V, const double *zeta, const double *G0, double *k_out, void *stream) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    if (n_cells == 0) return ok();
    CHECK_DEV(T, "T");
    CHECK_DEV(n_H, "n_H");
    CHECK_DEV(A_V, "A_V");
    CHECK_DEV(zeta, "zeta");
    CHECK_DEV(G0, "G0");
    CHECK_DEV(k_out, "k_out");
    std::string err;
    const abdf::DeviceNet *dn = net->host.device_tables(err);
    if (!dn) return fail(ABDF_E_DEVICE, err);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OR_FAIL(abdf::launch_rates(*dn, abdf::PhysArgs{T, n_H, A_V, zeta, G0}, n_cells, k_out, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return ok();
}

abdf_status abdf_rhs(const abdf_network *net, int64_t n_cells, const double *k, const double *x, double *f_out,
                     void *stream) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    if (n_cells == 0) return ok();
    CHECK_DEV(k, "k");
    CHECK_DEV(x, "x");
    CHECK_DEV(f_out, "f_out");
    std::string err;
    const abdf::DeviceNet *dn = net->host.device_tables(err);
    if (!dn) return fail(ABDF_E_DEVICE, err);
    if (sizeof(double) * (size_t(dn->S) + dn->R + dn->n_seg) > abdf::kMaxLds)
        return fail(ABDF_E_ARG, "network too large for one workgroup's LDS");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OR_FAIL(abdf::launch_rhs(*dn, n_cells, k, x, f_out, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return ok();
}

abdf_status abdf_newton_matrix(const abdf_network *net, int64_t n_cells, const double *k, const double *x,
                               const double *c, double *M_out, void *stream) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    if (n_cells == 0) return ok();
    CHECK_DEV(k, "k");
    CHECK_DEV(x, "x");
    CHECK_DEV(c, "c");
    CHECK_DEV(M_out, "M_out");
    std::string err;
    const abdf::DeviceNet *dn = net->host.device_tables(err);
    if (!dn) return fail(ABDF_E_DEVICE, err);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *W = nullptr;
    HIP_OR_FAIL(hipMalloc(reinterpret_cast<void **>(&W), size_t(n_cells) * dn->NP * dn->NP * sizeof(double)));
    hipError_t e = abdf::launch_newton_matrix(*dn, n_cells, k, x, c, M_out, W, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(W);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, hipGetErrorString(e));
    return ok();
}

abdf_status abdf_lu_factor(int32_t n, int64_t batch, double *A, int32_t *perm, int32_t *info, int32_t precision,
                           void *stream) {
    if (n < 1 || n > 512 || batch < 0 || batch > 65535) return fail(ABDF_E_ARG, "n or batch out of range");
    if (precision != ABDF_PREC_FP64 && precision != ABDF_PREC_FP32_LU) return fail(ABDF_E_ARG, "unknown precision");
    if (batch == 0) return ok();
    CHECK_DEV(A, "A");
    CHECK_DEV(perm, "perm");
    if (info) CHECK_DEV(info, "info");
    const int NP = (n + 15) / 16 * 16;
    const size_t elt = precision == ABDF_PREC_FP32_LU ? sizeof(float) : sizeof(double);
    void *W = nullptr, *dinv = nullptr;
    int32_t *permW = nullptr;
    hipError_t e = hipMalloc(&W, size_t(batch) * NP * NP * elt);
    if (e == hipSuccess) e = hipMalloc(&dinv, size_t(batch) * abdf::dinv_bytes(NP, precision));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&permW), size_t(batch) * NP * sizeof(int32_t));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (e == hipSuccess) e = abdf::launch_lu_factor(n, NP, batch, A, W, permW, perm, dinv, info, precision, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (W) (void)hipFree(W);
    if (dinv) (void)hipFree(dinv);
    if (permW) (void)hipFree(permW);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, hipGetErrorString(e));
    return ok();
}

abdf_status abdf_lu_solve(int32_t n, int64_t batch, const double *LU, const int32_t *perm, double *b, void *stream) {
    if (n < 1 || n > 512 || batch < 0 || batch > 65535) return fail(ABDF_E_ARG, "n or batch out of range");
    if (batch == 0) return ok();
    CHECK_DEV(LU, "LU");
    CHECK_DEV(perm, "perm");
    CHECK_DEV(b, "b");
    const int NP = (n + 15) / 16 * 16;
    void *W = nullptr, *dinv = nullptr;
    int32_t *permW = nullptr;
    hipError_t e = hipMalloc(&W, size_t(batch) * NP * NP * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dinv, size_t(batch) * abdf::dinv_bytes(NP, ABDF_PREC_FP64));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&permW), size_t(batch) * NP * sizeof(int32_t));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (e == hipSuccess) e = abdf::launch_lu_solve(n, NP, batch, LU, perm, b, W, permW, dinv, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (W) (void)hipFree(W);
    if (dinv) (void)hipFree(dinv);
    if (permW) (void)hipFree(permW);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, hipGetErrorString(e));
    return ok();
}

void abdf_profile_enable(int32_t on) { abdf::Profiler::enable(on != 0); }

void abdf_profile_read(abdf_profile *out, int32_t reset) {
    if (!out) return;
    abdf::Profiler::read(out->launches, out->ms, reset != 0);
}

abdf_status abdf_selftest(void *stream) {
    int *bad = nullptr;
    HIP_OR_FAIL(hipMalloc(reinterpret_cast<void **>(&bad), sizeof(int)));
    hipStream_t st = static_cast<hipStream_t>(stream);
    int h = -1;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
    if (e == hipSuccess) e = abdf::launch_selftest(bad, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, hipGetErrorString(e));
    if (h != 0) return fail(ABDF_E_DEVICE, "matrix-core lane layout differs from the kernels' assumption");
    return ok();
}

}  // extern "C"
