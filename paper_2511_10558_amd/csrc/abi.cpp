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
#include "server.hpp"
#include "adjoint.hpp"
#include "noalloc.hpp"

struct abdf_network {
    abdf::HostNetwork host;
};

struct abdf_tape {
    std::unique_ptr<abdf::Tape> impl;
};

struct abdf_server {
    std::unique_ptr<abdf::Server> impl;
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
    if (o.method != ABDF_METHOD_BDF && o.method != ABDF_METHOD_ESDIRK5) return fail(ABDF_E_ARG, "unknown method");
    if (o.method == ABDF_METHOD_ESDIRK5) {
        if (o.lu_reuse != 0.0) return fail(ABDF_E_ARG, "the ESDIRK method factors every step attempt (lu_reuse must be 0)");
        if (o.phi_tc) return fail(ABDF_E_ARG, "the ESDIRK method takes constant conditions (phi_tc must be NULL)");
    }
    if (o.newton_tol < 0.0 || !std::isfinite(o.newton_tol)) return fail(ABDF_E_ARG, "newton_tol must be >= 0");
    if (!(o.lu_reuse >= 0.0 && o.lu_reuse < 1.0)) return fail(ABDF_E_ARG, "lu_reuse must be in [0, 1)");
    if (o.max_order < 0 || o.max_order > 5) return fail(ABDF_E_ARG, "max_order must be in 1..5 (0: 5)");
    if (!(o.h0 >= 0.0) || !std::isfinite(o.h0)) return fail(ABDF_E_ARG, "h0 must be finite and >= 0");
    if (!(o.h_max >= 0.0) || !std::isfinite(o.h_max)) return fail(ABDF_E_ARG, "h_max must be finite and >= 0");
    if (o.atol_species) CHECK_DEV(o.atol_species, "atol_species");
    if (o.phi_tc) CHECK_DEV(o.phi_tc, "phi_tc");
    for (double p : o.phi_exp)
        if (!std::isfinite(p)) return fail(ABDF_E_ARG, "phi_exp entries must be finite");
    return ABDF_OK;
}

// Slots that fit in the budget and in 85% of the device memory free (plus,
// for an engine that takes the network's cached workspace, the cached bytes),
// at most `want`.
long long slot_count(const abdf::HostNetwork &net, const abdf::DeviceNet &dn, const abdf_options &o, long long want,
                     size_t extra_per_slot = 0, bool uses_cache = false) {
    const size_t per = abdf::Engine::bytes_per_slot(dn, o.precision) + extra_per_slot;
    long long n = want;
    if (o.hbm_budget_bytes > 0) n = std::min<long long>(n, (long long)(o.hbm_budget_bytes / per));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
        if (uses_cache) free_b += net.cached_workspace_bytes(dn.device);
        n = std::min<long long>(n, (long long)(0.85 * double(free_b) / double(per)));
    }
    return n;
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
    opt->lu_reuse = 0.0;
    opt->max_order = 5;
    opt->h0 = 0.0;
    opt->h_max = 0.0;
    opt->atol_species = nullptr;
    opt->phi_tc = nullptr;
    for (double &p : opt->phi_exp) p = 0.0;
    opt->method = ABDF_METHOD_BDF;
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
        const long long nslots = slot_count(net->host, *dn, o, n_cells, 0, /*uses_cache=*/true);
        if (nslots < 1) return fail(ABDF_E_BUDGET, "not even one cell fits in the workspace budget");
        abdf::Engine eng(net->host, *dn, o.precision, o.max_steps);
        int r = eng.set_options(o, err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        r = eng.init(int(nslots), err, /*cache_workspace=*/true);
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

abdf_status abdf_solve_noalloc(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
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
    int dev = 0;
    HIP_OR_FAIL(hipGetDevice(&dev));
    const abdf::DeviceNet *dn = net->host.device_tables_present(dev);
    if (!dn)
        return fail(ABDF_E_ARG, "the network's tables are not on this device yet (they are uploaded by the first "
                                "call of any other solving entry point with this network on this device)");
    std::string err;
    void *scratch = nullptr;
    abdf::HostBuffers hb{};
    int r = abdf::noalloc_workspace(dev, &scratch, &hb, err);
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    // as many slots as the scratch array, its host buffers and the budget hold
    const size_t cap = o.hbm_budget_bytes > 0 ? std::min<size_t>(o.hbm_budget_bytes, abdf::kNoAllocScratchBytes)
                                              : abdf::kNoAllocScratchBytes;
    long long nslots = std::min<long long>(n_cells, hb.max_slots);
    const size_t per = abdf::Engine::bytes_per_slot(*dn, o.precision);
    nslots = std::min<long long>(nslots, (long long)(cap / per) + 1);
    while (nslots > 0 && abdf::Engine::workspace_bytes(*dn, nslots) > cap) --nslots;
    if (nslots < 1)
        return fail(ABDF_E_BUDGET, "one cell of this network needs " +
                                       std::to_string(abdf::Engine::workspace_bytes(*dn, 1)) +
                                       " bytes of workspace, more than the " + std::to_string(cap) +
                                       " bytes the no-allocation entry point may use");
    abdf::Engine eng(net->host, *dn, o.precision, o.max_steps);
    r = eng.set_options(o, err, hb.atol);
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    r = eng.init_external(int(nslots), scratch, cap, hb, err);
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    abdf::BatchIO io{n_cells, T, n_H, A_V, zeta, G0, x0, t_end, x_out, cell_status, stats};
    r = eng.solve(io, o, static_cast<hipStream_t>(stream), err);
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    return ok();
}

namespace {
abdf_status check_solve_args(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                             const double *A_V, const double *zeta, const double *G0, const double *x0,
                             const double *t_end, const double *x_out, const int32_t *cell_status,
                             const abdf_cell_stats *stats) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    if (n_cells == 0) return ABDF_OK;
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
    return ABDF_OK;
}
}  // namespace

abdf_status abdf_solve_record(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                              const double *A_V, const double *zeta, const double *G0, const double *x0,
                              const double *t_end, const double *alpha, const abdf_options *opt,
                              int32_t max_tape_steps, double *x_out, int32_t *cell_status, abdf_cell_stats *stats,
                              abdf_tape **tape, void *stream) {
    if (!tape) return fail(ABDF_E_ARG, "null tape pointer");
    *tape = nullptr;
    abdf_status rc = check_solve_args(net, n_cells, T, n_H, A_V, zeta, G0, x0, t_end, x_out, cell_status, stats);
    if (rc != ABDF_OK) return rc;
    if (n_cells == 0) return fail(ABDF_E_ARG, "a tape needs at least one cell");
    abdf_options o;
    if (opt) o = *opt; else abdf_options_default(&o);
    rc = check_opts(o);
    if (rc != ABDF_OK) return rc;
    if (o.precision != ABDF_PREC_FP64) return fail(ABDF_E_ARG, "recording solves use FP64 factorisations");
    if (o.phi_tc) return fail(ABDF_E_ARG, "recording solves take constant conditions (phi_tc must be NULL)");
    if (o.method != ABDF_METHOD_BDF) return fail(ABDF_E_ARG, "recording solves (the adjoint) use the BDF method");
    if (max_tape_steps < 0) return fail(ABDF_E_ARG, "max_tape_steps must be >= 0");
    if (alpha) CHECK_DEV(alpha, "alpha");
    try {
        std::string err;
        const abdf::DeviceNet *dn = net->host.device_tables(err);
        if (!dn) return fail(ABDF_E_DEVICE, err);
        auto t = std::make_unique<abdf_tape>();
        t->impl = std::make_unique<abdf::Tape>(net->host, *dn);
        abdf::BatchIO io{n_cells, T, n_H, A_V, zeta, G0, x0, t_end, x_out, cell_status, stats};
        int r = t->impl->record(io, alpha, o, max_tape_steps > 0 ? max_tape_steps : 2048,
                                static_cast<hipStream_t>(stream), err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        *tape = t.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(ABDF_E_DEVICE, e.what());
    }
}

abdf_status abdf_tape_adjoint(abdf_tape *tape, const double *dL_dx, double *dL_dlog_alpha,
                              double *dL_dlog_alpha_cell, double *dL_dx0, double *dL_dphi, void *stream) {
    if (!tape) return fail(ABDF_E_ARG, "null tape");
    CHECK_DEV(dL_dx, "dL_dx");
    if (dL_dlog_alpha) CHECK_DEV(dL_dlog_alpha, "dL_dlog_alpha");
    if (dL_dlog_alpha_cell) CHECK_DEV(dL_dlog_alpha_cell, "dL_dlog_alpha_cell");
    if (dL_dx0) CHECK_DEV(dL_dx0, "dL_dx0");
    if (dL_dphi) CHECK_DEV(dL_dphi, "dL_dphi");
    try {
        std::string err;
        int r = tape->impl->adjoint(dL_dx, dL_dlog_alpha, dL_dlog_alpha_cell, dL_dx0, dL_dphi,
                                    static_cast<hipStream_t>(stream), err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    }
}

int64_t abdf_tape_bytes(const abdf_tape *tape) { return tape ? int64_t(tape->impl->bytes()) : 0; }

void abdf_tape_free(abdf_tape *tape) { delete tape; }

abdf_status abdf_solve_adjoint(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                               const double *A_V, const double *zeta, const double *G0, const double *x0,
                               const double *t_end, const double *alpha, const abdf_options *opt,
                               const double *dL_dx, double *x_out, int32_t *cell_status, double *dL_dlog_alpha,
                               double *dL_dlog_alpha_cell, double *dL_dx0, double *dL_dphi, abdf_cell_stats *stats,
                               void *stream) {
    abdf_tape *tape = nullptr;
    abdf_status rc = abdf_solve_record(net, n_cells, T, n_H, A_V, zeta, G0, x0, t_end, alpha, opt, 0, x_out,
                                       cell_status, stats, &tape, stream);
    if (rc != ABDF_OK) return rc;
    rc = abdf_tape_adjoint(tape, dL_dx, dL_dlog_alpha, dL_dlog_alpha_cell, dL_dx0, dL_dphi, stream);
    abdf_tape_free(tape);
    return rc;
}

void abdf_server_options_default(abdf_server_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    abdf_options_default(&opt->solve);
    opt->solve.check_every = 4;
}

abdf_status abdf_server_create(const abdf_network *net, const abdf_server_options *opt, abdf_server **out) {
    if (!net || !out) return fail(ABDF_E_ARG, "null argument");
    *out = nullptr;
    abdf_server_options o;
    if (opt) o = *opt; else abdf_server_options_default(&o);
    abdf_status rc = check_opts(o.solve);
    if (rc != ABDF_OK) return rc;
    if (o.max_slots < 0 || o.max_slots > INT32_MAX || o.max_queued_cells < 0)
        return fail(ABDF_E_ARG, "max_slots or max_queued_cells out of range");
    if (o.solve.phi_tc) return fail(ABDF_E_ARG, "served requests take constant conditions (phi_tc must be NULL)");
    if (o.solve.method != ABDF_METHOD_BDF) return fail(ABDF_E_ARG, "the server uses the BDF method");
    try {
        std::string err;
        const abdf::DeviceNet *dn = net->host.device_tables(err);
        if (!dn) return fail(ABDF_E_DEVICE, err);
        // staging per slot: admission inputs (8 + S doubles), outputs (S doubles, status, stats)
        const size_t staging = (8 + 2 * size_t(dn->S)) * sizeof(double) + 16 + sizeof(abdf_cell_stats);
        long long nslots = slot_count(net->host, *dn, o.solve, o.max_slots > 0 ? o.max_slots : INT32_MAX, staging);
        if (nslots < 1) return fail(ABDF_E_BUDGET, "not even one cell fits in the workspace budget");
        int dev = 0;
        HIP_OR_FAIL(hipGetDevice(&dev));
        auto s = std::make_unique<abdf_server>();
        s->impl = std::make_unique<abdf::Server>(net->host, *dn, o, dev);
        int r = s->impl->start(int(nslots), err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        *out = s.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(ABDF_E_DEVICE, e.what());
    }
}

abdf_status abdf_server_submit(abdf_server *srv, const abdf_request *req, uint64_t *id) {
    if (!srv || !req || !id) return fail(ABDF_E_ARG, "null argument");
    try {
        std::string err;
        int r = srv->impl->submit(*req, id, err);
        if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(ABDF_E_NOMEM, "host allocation failed");
    }
}

abdf_status abdf_server_poll(abdf_server *srv, abdf_completion *out, int32_t max, int32_t *n_out, int32_t timeout_ms) {
    if (!srv || !n_out || (max > 0 && !out) || max < 0) return fail(ABDF_E_ARG, "bad argument");
    std::string err;
    int n = 0;
    int r = srv->impl->poll(out, max, &n, timeout_ms, err);
    *n_out = n;
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    return ok();
}

abdf_status abdf_server_cancel(abdf_server *srv, uint64_t id) {
    if (!srv) return fail(ABDF_E_ARG, "null server");
    std::string err;
    int r = srv->impl->cancel(id, err);
    if (r != ABDF_OK) return fail(static_cast<abdf_status>(r), err);
    return ok();
}

double abdf_server_clock(const abdf_server *srv) { return srv ? srv->impl->now() : 0.0; }

abdf_status abdf_server_info_get(abdf_server *srv, abdf_server_info *out) {
    if (!srv || !out) return fail(ABDF_E_ARG, "null argument");
    srv->impl->info(out);
    return ok();
}

void abdf_server_destroy(abdf_server *srv) { delete srv; }

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

abdf_status abdf_phys_gradient(const abdf_network *net, int64_t n_cells, const double *T, const double *n_H,
                               const double *A_V, const double *zeta, const double *G0,
                               const double *dL_dlog_alpha_cell, double *dL_dphi, void *stream) {
    if (!net) return fail(ABDF_E_ARG, "null network");
    if (n_cells < 0 || n_cells > INT32_MAX) return fail(ABDF_E_ARG, "n_cells out of range");
    if (n_cells == 0) return ok();
    CHECK_DEV(T, "T");
    CHECK_DEV(n_H, "n_H");
    CHECK_DEV(A_V, "A_V");
    CHECK_DEV(zeta, "zeta");
    CHECK_DEV(G0, "G0");
    CHECK_DEV(dL_dlog_alpha_cell, "dL_dlog_alpha_cell");
    CHECK_DEV(dL_dphi, "dL_dphi");
    std::string err;
    const abdf::DeviceNet *dn = net->host.device_tables(err);
    if (!dn) return fail(ABDF_E_DEVICE, err);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OR_FAIL(abdf::launch_phys_grad(*dn, abdf::PhysArgs{T, n_H, A_V, zeta, G0}, n_cells, dL_dlog_alpha_cell,
                                       dL_dphi, st));
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
    if (sizeof(double) * (size_t(dn->S) + dn->R) > abdf::kMaxLds)
        return fail(ABDF_E_ARG, "network too large for one workgroup's LDS");
    hipStream_t st = static_cast<hipStream_t>(stream);
    abdf::RhsPlan plan;
    hipError_t e = abdf::plan_rhs(*dn, n_cells, plan);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, std::string("abdf_rhs: ") + hipGetErrorString(e));
    // with the timers on, the dispatch records events at the kernel's start and end
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (abdf::Profiler::on() && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)) {
        for (hipEvent_t evt : ev)
            if (evt) (void)hipEventDestroy(evt);
        ev[0] = ev[1] = nullptr;
    }
    e = abdf::launch_rhs_planned(plan, *dn, n_cells, k, x, f_out, st, ev[0], ev[1]);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && ev[0]) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) abdf::Profiler::add(ABDF_PROF_RHS_EVAL, double(ms));
    }
    for (hipEvent_t evt : ev)
        if (evt) (void)hipEventDestroy(evt);
    if (e != hipSuccess) return fail(ABDF_E_DEVICE, std::string("abdf_rhs: ") + hipGetErrorString(e));
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
    double *jv = nullptr;
    HIP_OR_FAIL(hipMalloc(reinterpret_cast<void **>(&jv), size_t(n_cells) * std::max(dn->nnzJ, 1) * sizeof(double)));
    hipError_t e = abdf::launch_newton_matrix(*dn, n_cells, k, x, c, M_out, jv, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(jv);
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
