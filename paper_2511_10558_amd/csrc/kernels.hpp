// Kernel launchers shared by the host engine and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.hpp"
#include "network.hpp"

struct abdf_cell_stats;

namespace abdf {

struct AdmitArgs {
    int count;
    const int32_t *slots;       // [count] target slots
    const long long *cells;     // [count] source cell indices
    const double *T, *nH, *Av, *zeta, *G0, *x0, *t_end;
    const double *rtol_c, *atol_c;  // per-cell tolerances [cells], or null for rtol / atol
    double rtol, atol;
    double newton_tol;          // > 0: used as is; 0: from each cell's rtol
    const double *tc;           // [cells] expansion times of the conditions, or null (constant)
};

struct HarvestArgs {
    int count;
    const int32_t *slots;       // [count] finished slots
    double *x_out;
    int32_t *status;
    abdf_cell_stats *stats;
    int compact;                // 1: results of the i-th finished slot go to index i, else to its cell
};

// Reverse-sweep admission: cells into slots with their loss gradients.
struct AdjArgs {
    int count;
    const int32_t *slots;
    const long long *cells;
    const double *phi;          // [cells][5] T, n_H, A_V, zeta, G0
    const double *dLdx;         // [cells][S] gradient of the loss with respect to x(t_end)
    const int32_t *status;      // [cells] forward outcome; only ABDF_CELL_OK cells are differentiated
};

struct AdjHarvestArgs {
    int count;
    const int32_t *slots;
    double *g_cell;             // [cells][R] dL/dlog alpha, or null
    double *dx0;                // [cells][S] or null
    double *dphi;               // [cells][5] dL/d(T, n_H, A_V, zeta, G0), or null
};

struct PhysArgs {
    const double *T, *nH, *Av, *zeta, *G0;
};

// LDS bytes per kernel for a network
inline size_t admit_lds(const DeviceNet &n) { return sizeof(double) * (4 * size_t(n.S) + n.R); }
inline size_t newton_lds(const DeviceNet &n) {
    return sizeof(double) * (2 * size_t(n.S) + n.R);
}
inline size_t solve_lds(const DeviceNet &n) { return sizeof(double) * 2 * size_t(n.NP); }
// the refining FP32 variant also holds the second solution, x_J and the
// scratch of the Jacobian-vector product
inline size_t solve_lds32(const DeviceNet &n) {
    return sizeof(double) * (3 * size_t(n.NP) + n.S + n.R);
}
size_t factor_lds(const DeviceNet &n, int prec);

hipError_t launch_admit(const Slots &s, const DeviceNet &n, const AdmitArgs &a, int ring, size_t lds, hipStream_t st);
// FP32-LU engines launch the FP32 variant (grid, lds32) and then the FP64 one
// for the slots that fell back (grid64, lds); FP64 engines only the latter (grid).
hipError_t launch_factor(const Slots &s, const DeviceNet &n, int ring, int grid, int grid64, size_t lds,
                         size_t lds32, hipStream_t st);
// Newton kernels take the slot list to work on (kListAll / kListFactor / kListNoFactor).
hipError_t launch_newton_rhs(const Slots &s, const DeviceNet &n, int ring, int which, int grid, size_t lds,
                             hipStream_t st);
// FP32-LU engines launch the plain FP32 (grid), the refining FP32 (grid_ref,
// lds_ref) and the FP64 (grid64) variants; FP64 engines only the last (grid).
// All Newton iterations of the listed slots in one launch (FP64 engines; LDS:
// the larger of newton_lds and solve_lds).
hipError_t launch_newton_fused(const Slots &s, const DeviceNet &n, int ring, int which, int grid, size_t lds,
                               hipStream_t st);
hipError_t launch_newton_solve(const Slots &s, const DeviceNet &n, int ring, int which, int grid, int grid_ref,
                               size_t lds, size_t lds_ref, hipStream_t st);
hipError_t launch_control(const Slots &s, const DeviceNet &n, int ring, int grid, hipStream_t st);
// ESDIRK: the next stage (or the step decision) of every active slot
hipError_t launch_control_rk(const Slots &s, int ring, int grid, hipStream_t st);
hipError_t launch_harvest(const Slots &s, const HarvestArgs &h, hipStream_t st);

hipError_t launch_adj_admit(const Slots &s, const DeviceNet &n, const AdjArgs &a, int ring, size_t lds, hipStream_t st);
hipError_t launch_adj_solve(const Slots &s, int ring, int grid, size_t lds, hipStream_t st);
hipError_t launch_adj_step(const Slots &s, const DeviceNet &n, int ring, int grid, size_t lds, hipStream_t st);
hipError_t launch_adj_harvest(const Slots &s, const DeviceNet &n, const AdjHarvestArgs &h, hipStream_t st);
hipError_t launch_grad_sum(const double *g_cell, long long cells, int R, double *out, hipStream_t st);
// dL/dphi [cells][5] (T, n_H, A_V, zeta, G0) from per-cell dL/dlog alpha [cells][R].
hipError_t launch_phys_grad(const DeviceNet &n, const PhysArgs &p, long long cells, const double *g_cell,
                            double *out, hipStream_t st);
inline size_t adj_lds(const DeviceNet &n) { return sizeof(double) * (2 * size_t(n.S) + n.R); }
inline size_t adj_solve_lds(const DeviceNet &n) { return sizeof(double) * (2 * size_t(n.NP) + 5 * 64 + 64 * 65); }

hipError_t launch_rates(const DeviceNet &n, const PhysArgs &p, long long cells, double *k, hipStream_t st);
// The standalone right-hand side: the kernel and grid for a batch (host
// queries only), then its launch.
struct RhsPlan {
    const void *fn = nullptr;
    long long grid = 0;
    int threads = 0;
    size_t lds = 0;
};
hipError_t plan_rhs(const DeviceNet &n, long long cells, RhsPlan &p);
// start, stop: events (or null) the dispatch itself records at the kernel's
// start and end.
hipError_t launch_rhs_planned(const RhsPlan &p, const DeviceNet &n, long long cells, const double *k, const double *x,
                              double *f, hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// jv: scratch of cells * max(nnzJ, 1) doubles (the Jacobian nonzeros)
hipError_t launch_newton_matrix(const DeviceNet &n, long long cells, const double *k, const double *x,
                                const double *c, double *M, double *jv, hipStream_t st);
hipError_t launch_lu_factor(int n, int NP, long long batch, double *A, void *W, int32_t *permW, int32_t *perm,
                            void *dinv, int32_t *info, int prec, hipStream_t st);
hipError_t launch_lu_solve(int n, int NP, long long batch, const double *LU, const int32_t *perm, double *b,
                           void *W, int32_t *permW, void *dinv, hipStream_t st);
size_t dinv_bytes(int NP, int prec);
size_t lu_bytes(int NP, int prec);
// Workgroups resident per CU of the factor (which = 0), Newton residual (1),
// Newton solve (2), transposed adjoint solve (3) or refining FP32 Newton
// solve (4) kernel.
int resident_per_cu(int which, int prec, size_t lds);
// Workgroups per CU of the kernel launch_newton_rhs runs for this network
// (lds: the LDS of the non-streaming kernel, used when it is that one).
int newton_rhs_resident_per_cu(const DeviceNet &n, int prec, size_t lds);
hipError_t launch_selftest(int *bad, hipStream_t st);
hipError_t launch_fill_i32(int32_t *v, int32_t value, int n, hipStream_t st);
size_t lu_work_lds(int NP, int prec);

// Largest dynamic LDS one workgroup may use on the device.
constexpr size_t kMaxLds = 160 * 1024;

}  // namespace abdf
