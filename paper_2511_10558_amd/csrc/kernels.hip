// Device kernels of the batched BDF solver and the component entry points.
//
// One workgroup handles one cell (slot) in every per-cell kernel; vectors are
// slot-major so a workgroup's loads over species or reactions are coalesced.
//
// Integrator: variable-order, variable-step BDF in backward-difference form
// (quasi-constant step size, orders 1..5; the BDF family of paper Sec. 1 in
// the formulation of Shampine & Reichelt 1997, Sec. 2.1-2.3, kappa = 0).
// Per step attempt of a cell:
//   begin   clamp h to land on t_end, predictor x_p = sum_{j<=q} D_j,
//           psi = sum_{j=1..q} gamma_j D_j / gamma_q, c = h / gamma_q,
//           request a factorisation of M = I - c J when c changed
//   factor  form M from J at x_J and factor it (k_factor)
//   newton  <= 4 modified-Newton iterations d <- d + M^{-1}(c f(x) - psi - d)
//   control error test ||d / (q+1)|| <= 1, accept (update differences) or
//           reject (shrink h), order/step selection every q+1 equal steps,
//           Jacobian refresh or h halving on corrector failure.
#include "kernels.hpp"

#include "device_chem.hpp"
#include "device_common.hpp"
#include "device_lu.hpp"
#include "device_lu2.hpp"

#include "../../include/astrobdf.h"

namespace abdf {

// ------------------------------------------------------------ BDF helpers --

__device__ inline double bdf_gamma(int q) {
    double g = 0.0;
    for (int j = 1; j <= q; ++j) g += 1.0 / j;
    return g;
}

__device__ inline double growth(double err, int p) {
    if (err == 0.0) return INFINITY;
    if (!isfinite(err)) return 0.0;
    return pow(err, -1.0 / p);
}

// RU = R(rho) R(1) with R(rho)[i][j] = prod_{m=1..i} (m - 1 - rho j) / m, i, j in 0..q.
// Thread i * 6 + j (< 36) forms entry (i, j): the factors of R(rho)[i][m] and
// R(1)[m][j] in the order of the recurrence R[i][.] = R[i - 1][.] (i - 1 - rho .) / i,
// then the sum over m in order.  Static loop bounds keep everything in registers.
__device__ inline void interp_product(int q, double rho, double *RU) {
    const int t = threadIdx.x;
    if (t >= 36) return;
    const int i = t / 6, j = t % 6;
    if (i > q || j > q) return;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m <= kMaxOrder; ++m) {
        if (m <= q) {
            double rr = 1.0, r1 = 1.0;
#pragma unroll
            for (int k = 1; k <= kMaxOrder; ++k) {
                if (k <= i) rr = rr * (k - 1 - rho * m) / k;
                if (k <= m) r1 = r1 * (k - 1 - 1.0 * j) / k;
            }
            s += rr * r1;
        }
    }
    RU[i * 6 + j] = s;
}

// Rows 0..q of D (one slot) from spacing h to rho*h.  Cooperative.
__device__ __forceinline__ void rescale_D(double *D, int S, int q, double rho, double *RU) {
    interp_product(q, rho, RU);
    __syncthreads();
    // loops over all kMaxOrder + 1 rows with the rows above q masked, so that
    // the per-thread arrays stay in registers (a dynamic index would put them
    // in scratch memory); the sums run in the same order
    for (int i = threadIdx.x; i < S; i += kBlock) {
        double v[kMaxOrder + 1], w[kMaxOrder + 1];
#pragma unroll
        for (int j = 0; j <= kMaxOrder; ++j) v[j] = j <= q ? D[j * S + i] : 0.0;
#pragma unroll
        for (int a = 0; a <= kMaxOrder; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b <= kMaxOrder; ++b)
                if (b <= q) s += RU[b * 6 + a] * v[b];
            w[a] = s;
        }
#pragma unroll
        for (int j = 0; j <= kMaxOrder; ++j)
            if (j <= q) D[j * S + i] = w[j];
    }
    __syncthreads();
}

__device__ inline void finish_slot(const Slots &s, int slot, SlotCtl &cs, int status) {
    if (threadIdx.x == 0) {
        cs.status = status;
        const int p = atomicAdd(&s.cnt[6], 1);
        s.fin[p] = slot;
    }
}

// The conditions of a slot at time t into out[5] (LDS, thread 0): an
// expanding flow, phi_j(t) = phi_j(0) (1 + t / tc)^(-p_j), constant for tc = 0.
__device__ __forceinline__ void phi_at(const Slots &s, int slot, double tc, double t, double *out) {
    if (threadIdx.x == 0) {
        const double *p0 = s.phi + size_t(slot) * 5;
        const double sc = 1.0 + t / tc;
#pragma unroll
        for (int j = 0; j < 5; ++j) out[j] = tc > 0.0 ? p0[j] * pow(sc, -s.phi_exp[j]) : p0[j];
    }
}

// Starts the next step attempt of a running slot whose cs (LDS) is current:
// checks limits, lands on t_end, forms the predictor and queues the slot.
// With time-dependent conditions the slot's rate coefficients become those
// at the attempt's end, t + h (phit: 5 doubles of LDS).  Writes cs back to
// global memory.
__device__ __forceinline__ void begin_attempt(const Slots &s, const DeviceNet &n, int slot, SlotCtl &cs, int ring,
                                              double *RU, double *sh, double *phit) {
    const int S = s.S;
    double *D = s.D + size_t(slot) * kDRows * S;
    if (threadIdx.x == 0) {
        int st = kRunning;
        double rho = 0.0;
        if (cs.n_attempts >= s.max_steps) {
            st = ABDF_CELL_MAX_STEPS;
        } else {
            cs.n_attempts += 1;
            if (cs.h < 10.0 * kURound * fabs(cs.t)) {
                st = ABDF_CELL_STEP_TOO_SMALL;
            } else {
                cs.landing = 0;
                if (cs.t + cs.h >= cs.t_end) {
                    if (cs.t + cs.h > cs.t_end) {
                        rho = (cs.t_end - cs.t) / cs.h;
                        cs.h = cs.t_end - cs.t;
                        cs.n_equal = 0;
                    }
                    cs.landing = 1;
                }
            }
        }
        cs.status = st;
        sh[0] = rho;
    }
    __syncthreads();
    if (cs.status != kRunning) {
        finish_slot(s, slot, cs, cs.status);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    const int q = cs.q;
    if (sh[0] != 0.0) rescale_D(D, S, q, sh[0], RU);
    if (s.tvar && cs.tc > 0.0) {
        phi_at(s, slot, cs.tc, cs.t + cs.h, phit);
        __syncthreads();
        cell_rates(n, phit, s.k + size_t(slot) * n.R);
    }
    const double gq = bdf_gamma(q);
    double gam[kMaxOrder + 1];
#pragma unroll
    for (int j = 1; j <= kMaxOrder; ++j) gam[j] = bdf_gamma(j);
    const bool refresh = cs.jac_refresh != 0;
    double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S, *psi = s.psi + size_t(slot) * S;
    double *scl = s.scl + size_t(slot) * S, *xJ = s.xJ + size_t(slot) * S;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        double dj[kMaxOrder + 1];
#pragma unroll
        for (int j = 0; j <= kMaxOrder; ++j) dj[j] = j <= q ? D[j * S + i] : 0.0;
        double xp = dj[0];
#pragma unroll
        for (int j = 1; j <= kMaxOrder; ++j)
            if (j <= q) xp = xp + dj[j];
        double ps = 0.0;
#pragma unroll
        for (int j = 1; j <= kMaxOrder; ++j)
            if (j <= q) ps = ps + gam[j] * dj[j];
        ps = ps / gq;
        x[i] = xp;
        d[i] = 0.0;
        psi[i] = ps;
        scl[i] = atol_of(s, cs, i) + cs.rtol * fabs(xp);
        if (refresh) xJ[i] = xp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (refresh) { cs.jac_refresh = 0; cs.lu_valid = 0; cs.jv_valid = 0; }
        cs.c = cs.h / gq;
        cs.phase = kIter;
        cs.newton_iter = 0;
        cs.eta_old = 0.0;
        const int p = atomicAdd(&s.cnt[ring], 1);
        s.act[ring * s.nslots + p] = slot;
        const bool stale = s.lu_reuse > 0.0 ? !(fabs(cs.c - cs.c_lu) <= s.lu_reuse * cs.c_lu) : cs.c != cs.c_lu;
        if (!cs.lu_valid || stale) {
            const int pl = atomicAdd(&s.cnt[3 + ring], 1);
            s.lul[ring * s.nslots + pl] = slot;
        } else {
            const int pn = atomicAdd(&s.cnt[7 + ring], 1);
            s.nol[ring * s.nslots + pn] = slot;
        }
        s.ctl[slot] = cs;
    }
}

// ----------------------------------------------------------------- ESDIRK --
//
// Kvaerno's seven-stage ESDIRK 5(4) (BIT Numer. Math. 44, 2004): explicit
// first stage, diagonal gamma = 0.26, stiffly accurate pair (c_6 = c_7 = 1).
// One stage of every slot per pass of the attempt loop: stage 2 of an attempt
// queues the factorisation of I - h gamma J(x_n), stages 3..7 reuse it.  The
// slot's D rows hold x_n (0), F_1 = f(x_n) (1) and G_i = h f(Y_i) (2..7).

constexpr int kRkStages = 7;
constexpr double kRkGamma = 0.26;
__constant__ double kRkA[kRkStages][kRkStages] = {
    {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {0.26, 0.26, 0.0, 0.0, 0.0, 0.0, 0.0},
    {0.13, 0.84033320996790809, 0.26, 0.0, 0.0, 0.0, 0.0},
    {0.22371961478320505, 0.47675532319799699, -0.06470895363112615, 0.26, 0.0, 0.0, 0.0},
    {0.16648564323248321, 0.10450018841591720, 0.03631482272098715, -0.13090704451073998, 0.26, 0.0, 0.0},
    {0.13855640231268224, 0.0, -0.04245337201752043, 0.02446657898003141, 0.61943039072480676, 0.26, 0.0},
    {0.13659751177640291, 0.0, -0.05496908796538376, -0.04118626728321046, 0.62993304899016403,
     0.06962479448202728, 0.26}};

// Starts stage cs.stage (2..7) of a running slot whose cs (LDS) is current.
// Stage 2 opens a step attempt: the step budget, the step-size floor and the
// landing on t_end are checked, and after an accepted step the Jacobian point
// moves to x_n.  The stage starts from Y_i^0 = x_n + sum_{j<i} a_ij G_j +
// gamma G_{i-1} (its own equation with the previous stage's G, G_1 = h F_1)
// with psi = Y_i^0 - x_n - sum_{j<i} a_ij G_j and weights atol + rtol |Y_i^0|,
// so that the corrector kernels solve Y_i = x_n + sum_j a_ij G_j + h gamma f(Y_i)
// as a BDF corrector with c = h gamma.  Writes cs back to global memory.
__device__ __forceinline__ void begin_stage_rk(const Slots &s, int slot, SlotCtl &cs, int ring) {
    const int S = s.S;
    const int stage = cs.stage;
    if (threadIdx.x == 0 && stage == 2) {
        int st = kRunning;
        if (cs.n_attempts >= s.max_steps) {
            st = ABDF_CELL_MAX_STEPS;
        } else {
            cs.n_attempts += 1;
            if (cs.h < 10.0 * kURound * fabs(cs.t)) {
                st = ABDF_CELL_STEP_TOO_SMALL;
            } else {
                cs.landing = 0;
                if (cs.t + cs.h >= cs.t_end) {
                    cs.h = cs.t_end - cs.t;
                    cs.landing = 1;
                }
            }
        }
        cs.status = st;
    }
    __syncthreads();
    if (cs.status != kRunning) {
        finish_slot(s, slot, cs, cs.status);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    const double *D = s.D + size_t(slot) * kDRows * S;
    double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S, *psi = s.psi + size_t(slot) * S;
    double *scl = s.scl + size_t(slot) * S, *xJ = s.xJ + size_t(slot) * S;
    const bool first = stage == 2;
    const bool refresh = first && cs.jac_refresh != 0;
    const double h = cs.h;
    const double *a = kRkA[stage - 1];
    for (int i = threadIdx.x; i < S; i += kBlock) {
        // the stage starts from its own equation with the previous stage's G
        // in place of its own: x_n + sum_{j<i} a_ij G_j + gamma G_{i-1}
        const double xn = D[i];
        const double g1 = h * D[S + i];
        double sum = a[0] * g1;
        for (int j = 2; j < stage; ++j) sum = sum + a[j - 1] * D[j * S + i];
        const double gprev = first ? g1 : D[(stage - 1) * S + i];
        const double xp = (xn + sum) + kRkGamma * gprev;
        x[i] = xp;
        d[i] = 0.0;
        psi[i] = (xp - xn) - sum;
        scl[i] = atol_of(s, cs, i) + cs.rtol * fabs(xp);
        if (refresh) xJ[i] = xn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double c = h * kRkGamma;
        if (refresh) {
            cs.jac_refresh = 0;
            cs.jv_valid = 0;
            cs.lu_valid = 0;
            cs.n_jac += 1;
        }
        if (first && c != cs.c_lu) cs.lu_valid = 0;
        cs.c = c;
        cs.phase = kIter;
        cs.newton_iter = 0;
        cs.eta_old = 0.0;
        const int p = atomicAdd(&s.cnt[ring], 1);
        s.act[ring * s.nslots + p] = slot;
        if (!cs.lu_valid) {
            const int pl = atomicAdd(&s.cnt[3 + ring], 1);
            s.lul[ring * s.nslots + pl] = slot;
        } else {
            const int pn = atomicAdd(&s.cnt[7 + ring], 1);
            s.nol[ring * s.nslots + pn] = slot;
        }
        s.ctl[slot] = cs;
    }
}


// --------------------------------------------------------------- kernels --

// Admits cells into slots: copies inputs, rates, starting step, difference
// table, then the first attempt.  One workgroup per (slot, cell) pair.
__global__ void __launch_bounds__(kBlock) k_admit(Slots s, DeviceNet n, AdmitArgs a, int ring) {
    extern __shared__ double smem[];
    __shared__ SlotCtl cs;
    __shared__ double RU[36], red[kWaves], sh[2], phit[5];
    const int idx = blockIdx.x;
    if (idx >= a.count) return;
    const int slot = a.slots[idx];
    const long long cell = a.cells[idx];
    const int S = s.S;
    double *xs = smem;
    double *f0 = xs + S;
    double *rate = f0 + S;
    double *f1 = rate + n.R;
    double *phi = s.phi + size_t(slot) * 5;
    double *k = s.k + size_t(slot) * n.R;
    double *D = s.D + size_t(slot) * kDRows * S;
    if (threadIdx.x == 0) {
        phi[0] = a.T[cell]; phi[1] = a.nH[cell]; phi[2] = a.Av[cell]; phi[3] = a.zeta[cell]; phi[4] = a.G0[cell];
        SlotCtl z = {};
        z.t = 0.0;
        z.t_end = a.t_end[cell];
        z.rtol = a.rtol_c ? a.rtol_c[cell] : a.rtol;
        z.atol = a.atol_c ? a.atol_c[cell] : a.atol;
        z.newton_tol = a.newton_tol > 0.0 ? a.newton_tol
                                          : fmax(10.0 * kURound / z.rtol, fmin(0.03, sqrt(z.rtol)));
        z.q = s.method == ABDF_METHOD_ESDIRK5 ? 5 : 1;
        z.stage = 2;
        z.status = kRunning;
        z.j_fresh = 1;
        z.lu_valid = 0;
        z.cell = int32_t(cell);
        z.tc = a.tc ? a.tc[cell] : 0.0;
        cs = z;
    }
    bool bad = false;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double v = a.x0[size_t(cell) * S + i];
        xs[i] = v;
        D[i] = v;
        for (int j = 1; j < kDRows; ++j) D[j * S + i] = 0.0;
        s.xJ[size_t(slot) * S + i] = v;
        bad |= !isfinite(v);
    }
    __syncthreads();
    const double T = phi[0], nH = phi[1], Av = phi[2], zeta = phi[3], G0 = phi[4];
    bad |= !(isfinite(T) && T > 0.0 && isfinite(nH) && nH > 0.0 && isfinite(Av) && isfinite(zeta) &&
             zeta >= 0.0 && isfinite(G0) && G0 >= 0.0 && isfinite(cs.t_end) && cs.t_end >= 0.0 &&
             isfinite(cs.rtol) && cs.rtol > 0.0 && isfinite(cs.atol) && cs.atol >= 0.0 && isfinite(cs.tc) &&
             cs.tc >= 0.0);
    bad = block_any(bad, red);
    if (bad) {
        finish_slot(s, slot, cs, ABDF_CELL_BAD_INPUT);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (s.tape_stop && s.tape_stop[cell] <= 0) {
        // a forward re-run that does not need this cell
        finish_slot(s, slot, cs, ABDF_CELL_OK);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    cell_rates(n, phi, k);
    __syncthreads();
    if (cs.t_end == 0.0) {
        finish_slot(s, slot, cs, ABDF_CELL_OK);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    // starting step (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4), for
    // the method's order: 1 (BDF's first step) or 5 (ESDIRK)
    const bool rk = s.method == ABDF_METHOD_ESDIRK5;
    cell_rhs(n, k, xs, rate, f0);
    {
        // rates that overflow at the initial state leave no step to take
        bool nf = false;
        for (int i = threadIdx.x; i < S; i += kBlock) nf |= !isfinite(f0[i]);
        if (block_any(nf, red)) {
            if (threadIdx.x == 0) cs.n_rhs = 1;
            __syncthreads();
            finish_slot(s, slot, cs, ABDF_CELL_NONFINITE);
            __syncthreads();
            if (threadIdx.x == 0) s.ctl[slot] = cs;
            return;
        }
    }
    const double rtol = cs.rtol;
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double sc = atol_of(s, cs, i) + rtol * fabs(xs[i]);
        s0 += (xs[i] / sc) * (xs[i] / sc);
        s1 += (f0[i] / sc) * (f0[i] / sc);
    }
    const double d0 = sqrt(block_sum(s0, red) / S);
    const double d1 = sqrt(block_sum(s1, red) / S);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, cs.t_end);
    // x1 = x0 + h0 f0 (kept in f1 as scratch, then f1 = f(x1))
    double *x1 = f1 + S;
    for (int i = threadIdx.x; i < S; i += kBlock) x1[i] = xs[i] + h0 * f0[i];
    if (s.tvar && cs.tc > 0.0) {
        // the trial evaluation at t = h0
        phi_at(s, slot, cs.tc, h0, phit);
        __syncthreads();
        cell_rates(n, phit, k);
    }
    __syncthreads();
    cell_rhs(n, k, x1, rate, f1);
    double s2 = 0.0;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double sc = atol_of(s, cs, i) + rtol * fabs(xs[i]);
        const double v = (f1[i] - f0[i]) / sc;
        s2 += v * v;
    }
    const double d2 = sqrt(block_sum(s2, red) / S) / h0;
    const double mx = fmax(d1, d2);
    const double h1 = mx <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : (rk ? pow(0.01 / mx, 1.0 / 6.0) : sqrt(0.01 / mx));
    double h = s.h0 > 0.0 ? fmin(s.h0, cs.t_end) : fmin(fmin(100.0 * h0, h1), cs.t_end);
    if (s.h_max > 0.0) h = fmin(h, s.h_max);
    for (int i = threadIdx.x; i < S; i += kBlock) D[S + i] = rk ? f0[i] : h * f0[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        cs.h = h;
        cs.n_rhs = 2;
        cs.n_jac = 1;
    }
    __syncthreads();
    if (rk)
        begin_stage_rk(s, slot, cs, ring);
    else
        begin_attempt(s, n, slot, cs, ring, RU, sh, phit);
}

// Forms M = I - c J(x_J) for every queued slot and factors it (one workgroup
// per matrix: 512 threads in FP64, 1024 in FP32).
template <typename T>
__global__ void __launch_bounds__(lu_threads<T>) k_factor(Slots s, DeviceNet n, int ring) {
    extern __shared__ double smem[];
    const int count = s.cnt[3 + ring];
    const int S = s.S, NP = s.NP;
    // persistent: each workgroup takes every gridDim.x-th queued slot
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int slot = s.lul[ring * s.nslots + idx];
        // FP32-LU engines run both variants: each takes the slots of its precision
        if (s.prec == ABDF_PREC_FP32_LU && (sizeof(T) == sizeof(double)) != (s.ctl[slot].lu_mode == kLu64)) continue;
        const double c = s.ctl[slot].c;
        // x_J after the factorisation's own LDS; the Jacobian nonzeros go to the
        // slot's compact array and M = I - c J(x_J) is formed block column by
        // block column as the factorisation gathers it.  A factorisation for a
        // new c at the same x_J (modified Newton keeps J across steps) reuses
        // the nonzeros already there.
        double *jv = s.jval + size_t(slot) * n.nnzJ;
        if (!s.ctl[slot].jv_valid) {
            double *xs = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(smem) + lu2_lds_bytes<T>(NP));
            for (int i = threadIdx.x; i < S; i += lu_threads<T>) xs[i] = s.xJ[size_t(slot) * S + i];
            __syncthreads();
            jacobian_values<lu_threads<T>>(n, s.k + size_t(slot) * n.R, xs, jv);
            __syncthreads();
        }
        NewtonMatrixSource<T> src{n.jmask, n.jbase, n.nbw, jv, c};
        lu_factor_left<T>(slot_lu<T>(s, slot), NP, s.perm + size_t(slot) * NP, slot_dinv<T>(s, slot), nullptr,
                          reinterpret_cast<unsigned char *>(smem), src);
        if (threadIdx.x == 0) {
            s.ctl[slot].c_lu = c;
            s.ctl[slot].lu_valid = 1;
            s.ctl[slot].jv_valid = 1;
            s.ctl[slot].n_lu += 1;
            if (s.prec == ABDF_PREC_FP32_LU && sizeof(T) == sizeof(double)) s.ctl[slot].n_lu64 += 1;
        }
        __syncthreads();
    }
}

// Newton residual r = c f(x) - psi - d of one slot still iterating.  A
// non-finite f ends the attempt as a corrector failure.  Cooperative; ends with
// a barrier.  LDS: xs [S], rate [R], f [S]; red [kWaves].
template <int NT>
__device__ __forceinline__ void newton_rhs_cell(const Slots &s, const DeviceNet &n, int slot, double *smem,
                                                double *red) {
    const int S = s.S;
    double *xs = smem;
    double *rate = xs + S;
    double *f = rate + n.R;
    const double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S, *psi = s.psi + size_t(slot) * S;
    double *rb = s.rb + size_t(slot) * S;
    const double c = s.ctl[slot].c;
    for (int i = threadIdx.x; i < S; i += NT) xs[i] = x[i];
    __syncthreads();
    cell_rhs<NT>(n, s.k + size_t(slot) * n.R, xs, rate, f);
    bool nonfinite = false;
    for (int i = threadIdx.x; i < S; i += NT) {
        nonfinite |= !isfinite(f[i]);
        rb[i] = c * f[i] - psi[i] - d[i];
    }
    nonfinite = block_sum_nt<NT>(nonfinite ? 1.0 : 0.0, red) != 0.0;
    if (threadIdx.x == 0) {
        SlotCtl &g = s.ctl[slot];
        g.n_rhs += 1;
        if (nonfinite) {
            g.n_newton_iter += 1;
            g.newton_iter += 1;
            g.m_last = g.newton_iter;
            g.phase = kFailed;
        }
    }
    __syncthreads();
}

// Newton correction Delta = M^{-1} r of one slot, its weighted norm, the
// convergence and divergence tests, and the update x += Delta, d += Delta.
// The refining variant (FP32 factors after a corrector failure) refines once in FP64:
// Delta += M^{-1} (r - (Delta - c J(x_J) Delta)), J applied through the
// network's Jacobian term lists.  Cooperative; ends with a barrier.
// LDS: b, y [NP] (refining: y2 [NP], xs [S], drate [R]);
// red [kLuW + kWaves]; decision: one shared int.
template <typename T, bool kRefine>
__device__ __forceinline__ void newton_solve_cell(const Slots &s, const DeviceNet &n, int slot, double *smem,
                                                  double *red, int *decision) {
    const int S = s.S, NP = s.NP;
    double *b = smem;
    double *y = b + NP;
    double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S;
    const double *scl = s.scl + size_t(slot) * S, *rb = s.rb + size_t(slot) * S;
    for (int i = threadIdx.x; i < NP; i += kBlock) b[i] = i < S ? rb[i] : 0.0;
    __syncthreads();
    const int32_t *perm = s.perm + size_t(slot) * NP;
    const T *A = slot_lu<T>(s, slot);
    const T *Di = slot_dinv<T>(s, slot);
    const int N = min(NP, S + (S & 1));   // the padding past S is the identity's
    lu_solve_left<T>(A, Di, perm, perm, NP, N, b, y, red);
    if (kRefine) {
        double *y2 = y + NP, *xs = y2 + NP, *drate = xs + S;
        const double c = s.ctl[slot].c_lu;
        for (int i = threadIdx.x; i < S; i += kBlock) xs[i] = s.xJ[size_t(slot) * S + i];
        __syncthreads();
        cell_jvp(n, s.k + size_t(slot) * n.R, xs, y, drate, y2);   // y2 = J(x_J) y
        for (int i = threadIdx.x; i < NP; i += kBlock) b[i] = i < S ? rb[i] - (y[i] - c * y2[i]) : 0.0;
        __syncthreads();
        lu_solve_left<T>(A, Di, perm, perm, NP, N, b, y2, red);
        for (int i = threadIdx.x; i < NP; i += kBlock) y[i] = y[i] + y2[i];
        __syncthreads();
    }
    {
        // a factorisation kept from c_lu != c: the correction is scaled by
        // 2 / (1 + c / c_lu), the usual remedy for the lagged leading coefficient
        const double c = s.ctl[slot].c, c_lu = s.ctl[slot].c_lu;
        if (c != c_lu) {
            const double sc = 2.0 / (1.0 + c / c_lu);
            for (int i = threadIdx.x; i < S; i += kBlock) y[i] = y[i] * sc;
            __syncthreads();
        }
    }
    double acc = 0.0;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double v = y[i] / scl[i];
        acc += v * v;
    }
    const double eta = sqrt(block_sum(acc, red + kLuW) / S);
    if (threadIdx.x == 0) {
        SlotCtl &g = s.ctl[slot];
        const int m = g.newton_iter + 1;
        const double tol = g.newton_tol;
        bool fail = false, conv = false;
        double theta = -1.0;
        if (m > 1) {
            theta = eta / g.eta_old;
            fail = theta >= 1.0 || pow(theta, double(s.newton_maxiter - m)) / (1.0 - theta) * eta > tol;
        }
        if (!fail) conv = eta == 0.0 || (m > 1 && theta / (1.0 - theta) * eta < tol);
        if (!fail && !conv && m == s.newton_maxiter) fail = true;
        g.n_newton_iter += 1;
        g.newton_iter = m;
        g.m_last = m;
        g.eta_old = eta;
        *decision = fail ? kFailed : (conv ? kConverged : kIter);
        g.phase = *decision;
    }
    __syncthreads();
    // a failed attempt discards x and d, so they are only updated otherwise
    if (*decision != kFailed) {
        for (int i = threadIdx.x; i < S; i += kBlock) {
            x[i] = x[i] + y[i];
            d[i] = d[i] + y[i];
        }
    }
    __syncthreads();
}

// Newton residuals of every listed slot still iterating (persistent), with
// kRhsThreads per slot: the residual's LDS (the rates) allows two workgroups per
// CU, so each takes sixteen waves and the CU runs its full 32.
constexpr int kRhsThreads = 1024;
__global__ void __launch_bounds__(kRhsThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_newton_rhs(Slots s, DeviceNet n, int ring, int which) {
    extern __shared__ double smem[];
    __shared__ double red[kRhsThreads / 64];
    int count;
    const int32_t *list = slot_list(s, which, ring, count);
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int slot = list[idx];
        if (s.ctl[slot].phase != kIter) continue;
        newton_rhs_cell<kRhsThreads>(s, n, slot, smem, red);
    }
}

// Streaming right-hand sides (k_rhs_stream, k_newton_rhs_stream): a
// workgroup of kRhsStreamThreads evaluates one cell after another, and each
// thread keeps for the whole launch its reactant pairs and its wave's lane
// groups of the species sums (two 16-bit entries a register), so the sums read
// LDS only and the next cell's inputs can be in flight while they run.  The
// lanes sum the entries of species_gather in the same order; the padding
// reads a -0.0 placed after the rates instead of being skipped (adding -0.0
// changes no sum, signed zeros included), so no entry needs a test, and a
// one-reactant rate takes a 1.0 placed after x as its second factor.
// LDS: rate [R], -0.0, x [S], 1.0, from the start of the dynamic block.  A
// resident entry is the rate's LDS address | nu in 3 bits, two's complement,
// so the sums read LDS at the entry's own address (the kernels have no static
// LDS, so the dynamic block starts at address 0 and every address fits 16
// bits).  Requires S <= kRhsStreamThreads, R < 8191, at most kGPW * 8 lane
// groups of at most kRhsResidentLen entries, and R <= kKU * kRhsStreamThreads
// (rhs_stream_shape checks).
constexpr int kRhsStreamThreads = 512;
template <int kKU, int kGPW>
struct RhsResident {
    static constexpr int NT = kRhsStreamThreads, NW = NT / 64, kE = kRhsResidentLen / 2;
    static constexpr int kB = kGPW * kKU >= 16 ? 4 : 8;   // LDS reads in flight per lane, as registers allow
    uint32_t ab[kKU];
    uint32_t ent[kGPW][kE];
    int red[kGPW], L[kGPW], steps[kGPW];

    // reactant pairs as LDS byte offsets into x (the 1.0 at x[S] for none)
    __device__ __forceinline__ void load_pairs(const DeviceNet &n) {
#pragma unroll
        for (int u = 0; u < kKU; ++u) {
            const int r = threadIdx.x + u * NT;
            const int w = r < n.R ? n.rx_ab[r] : 0;
            const int a = w & 0xffff, b = (w >> 16) & 0xffff;
            ab[u] = uint32_t(a * 8) | (uint32_t(b == 0xffff ? n.S : b) * 8u << 16);
        }
    }

    __device__ __forceinline__ void load(const DeviceNet &n, const double *smem) {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int R = n.R;
        load_pairs(n);
        // the LDS address of rate[0]
        const uint32_t lds0 = uint32_t(size_t((const __attribute__((address_space(3))) char *)smem));
        const uint32_t pad = (lds0 + uint32_t(R) * 8u) | 1u;   // +1 times the -0.0 after the rates
        auto conv = [lds0](int32_t w) { return (lds0 + uint32_t(w & ~7)) | (uint32_t((w & 7) - 4) & 7u); };
#pragma unroll
        for (int gi = 0; gi < kGPW; ++gi) {
            const int g = wave + gi * NW;
            const bool has = g < n.n_sgroup;
            const int mine = has ? n.sg_lane[g * 64 + lane] : 0;
            red[gi] = has ? n.sg_red[g * 64 + lane] : -1;
            const int lw = has ? __builtin_amdgcn_readfirstlane(n.sg_len[g]) : 0;
            L[gi] = lw & 0xffffff;
            steps[gi] = lw >> 24;
            if (L[gi] > 0) {
                // every load in flight at once: indexes past the group's
                // longest lane are clamped to its last row, their values unused
                const int32_t *e = n.sg_ent + n.sg_base[g] + lane;
                int32_t v[kRhsResidentLen];
#pragma unroll
                for (int j = 0; j < kRhsResidentLen; ++j) v[j] = e[min(j, L[gi] - 1) * 64];
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    const uint32_t lo = 2 * j < mine ? conv(v[2 * j]) : pad;
                    const uint32_t hi = 2 * j + 1 < mine ? conv(v[2 * j + 1]) : pad;
                    ent[gi][j] = lo | (hi << 16);
                }
            } else {
#pragma unroll
                for (int j = 0; j < kE; ++j) ent[gi][j] = pad | (pad << 16);
            }
        }
    }

    __device__ __forceinline__ static void init_lds(const DeviceNet &n, double *smem) {
        if (threadIdx.x == 0) {
            smem[n.R] = -0.0;
            smem[n.R + 1 + n.S] = 1.0;
        }
    }

    // rate[r] = k_r x_a x_b for this thread's reactions (x in LDS)
    __device__ __forceinline__ void rates(const DeviceNet &n, const double (&kr)[kKU], double *smem) const {
        const char *xb = reinterpret_cast<const char *>(smem + n.R + 1);
#pragma unroll
        for (int u = 0; u < kKU; ++u) {
            const int r = threadIdx.x + u * NT;
            const double xa = *reinterpret_cast<const double *>(xb + (ab[u] & 0xffffu));
            const double xc = *reinterpret_cast<const double *>(xb + (ab[u] >> 16));
            if (r < n.R) smem[r] = kr[u] * xa * xc;
        }
    }

    // out_i = sum_r nu_ir rate_r, written by each species' first lane
    __device__ __forceinline__ void sums(const DeviceNet &n, const double *smem, double *out) {
        // the entries are opaque to the compiler from one cell to the next,
        // so that it keeps them packed instead of hoisting what it derives from
        // them (offsets, coefficients) out of the cell loop into registers
#pragma unroll
        for (int gi = 0; gi < kGPW; ++gi)
#pragma unroll
            for (int j = 0; j < kE; ++j) asm volatile("" : "+v"(ent[gi][j]));
#pragma unroll
        for (int gi = 0; gi < kGPW; ++gi) {
            if (L[gi] == 0) continue;
            double acc = 0.0;
#pragma unroll
            for (int jb = 0; jb < kRhsResidentLen; jb += kB) {
                if (jb < L[gi]) {   // the same for the whole wave
                    double vv[kB], cf[kB];
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        const int j = jb + u, sh = 16 * (j & 1);
                        const uint32_t w = ent[gi][j >> 1];
                        vv[u] = *(const __attribute__((address_space(3))) double *)size_t((w >> sh) & 0xfff8u);
                        cf[u] = double(int32_t(w << (29 - sh)) >> 29);
                    }
#pragma unroll
                    for (int u = 0; u < kB; ++u) acc += cf[u] * vv[u];
                }
            }
            const int q = red[gi] < 0 ? 0 : (red[gi] >> 7) & 127, m = red[gi] < 0 ? 1 : red[gi] & 127;
            for (int t = 0; t < steps[gi]; ++t) {
                const int off = 1 << t;
                const double o = __shfl_down(acc, off);
                if ((q & (2 * off - 1)) == 0 && q + off < m) acc += o;
            }
            if (red[gi] >= 0 && q == 0) out[red[gi] >> 14] = acc;
        }
    }
};

// Newton residuals of every listed slot still iterating, streaming: the
// workgroup first collects, NT list positions at a time, the slots of its
// positions (blockIdx.x, blockIdx.x + gridDim.x, ...) still iterating, then
// evaluates them one after another with the next slot's k and x loading while
// the current one's sums run.  Per slot the same arithmetic as newton_rhs_cell.
// LDS: the RhsResident layout, then f [S], then the list of slots to evaluate
// [NT], its length and a non-finite flag (no static LDS: see RhsResident).
template <int kKU, int kGPW>
__global__ void __launch_bounds__(kRhsStreamThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_newton_rhs_stream(Slots s, DeviceNet n, int ring, int which) {
    using RR = RhsResident<kKU, kGPW>;
    constexpr int NT = kRhsStreamThreads;
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int S = n.S, R = n.R;
    int count;
    const int32_t *list = slot_list(s, which, ring, count);
    RR rr;
    rr.load(n, smem);
    RR::init_lds(n, smem);
    double *xs = smem + R + 1, *f = xs + S + 1;
    int *todo = reinterpret_cast<int *>(f + S), &ntodo = todo[NT], &bad = todo[NT + 1];
    const long long stride = (long long)gridDim.x * NT;
    for (long long base = blockIdx.x; base < count; base += stride) {
        if (tid == 0) ntodo = 0;
        __syncthreads();
        {
            const long long p = base + (long long)tid * gridDim.x;
            if (p < count) {
                const int slot = list[p];
                if (s.ctl[slot].phase == kIter) todo[atomicAdd(&ntodo, 1)] = slot;
            }
        }
        __syncthreads();
        const int nt = ntodo;
        double kr[kKU], xr = 0.0;
        if (nt > 0) {
            const int slot = todo[0];
#pragma unroll
            for (int u = 0; u < kKU; ++u) kr[u] = tid + u * NT < R ? s.k[size_t(slot) * R + tid + u * NT] : 0.0;
            if (tid < S) xr = s.x[size_t(slot) * S + tid];
        }
        for (int j = 0; j < nt; ++j) {
            const int slot = todo[j];
            const double c = s.ctl[slot].c;
            if (tid == 0) bad = 0;
            if (tid < S) xs[tid] = xr;
            __syncthreads();
            rr.rates(n, kr, smem);
            __syncthreads();
            double psi_i = 0.0, d_i = 0.0;
            if (tid < S) {
                psi_i = s.psi[size_t(slot) * S + tid];
                d_i = s.d[size_t(slot) * S + tid];
            }
            if (j + 1 < nt) {
                const int nx = todo[j + 1];
#pragma unroll
                for (int u = 0; u < kKU; ++u)
                    if (tid + u * NT < R) kr[u] = s.k[size_t(nx) * R + tid + u * NT];
                if (tid < S) xr = s.x[size_t(nx) * S + tid];
            }
            rr.sums(n, smem, f);
            // the pairs are reloaded (from cache) for the next slot rather than
            // held through the sums, where registers are scarcest
            rr.load_pairs(n);
            __syncthreads();
            if (tid < S) {
                const double fv = f[tid];
                if (!isfinite(fv)) bad = 1;
                s.rb[size_t(slot) * S + tid] = c * fv - psi_i - d_i;
            }
            __syncthreads();
            if (tid == 0) {   // only thread 0 reads the flag: it clears it next
                SlotCtl &g = s.ctl[slot];
                g.n_rhs += 1;
                if (bad) {
                    g.n_newton_iter += 1;
                    g.newton_iter += 1;
                    g.m_last = g.newton_iter;
                    g.phase = kFailed;
                }
            }
        }
        __syncthreads();
    }
}

// Newton corrections of every listed slot still iterating (persistent).  In an
// FP32-LU engine the plain FP32 variant also takes the slots whose factors are
// FP64 (same LDS), so that they run beside the FP32 ones rather than in a
// launch of their own; the refining variant takes its own slots.
template <typename T, bool kRefine>
__global__ void __launch_bounds__(kBlock) k_newton_solve(Slots s, DeviceNet n, int ring, int which) {
    extern __shared__ double smem[];
    __shared__ double red[kLuW + kWaves];
    __shared__ int decision;
    constexpr int32_t kMode = sizeof(T) == sizeof(double) ? kLu64 : (kRefine ? kLuRefined32 : kLuPlain32);
    constexpr bool kTakes64 = sizeof(T) == sizeof(float) && !kRefine;
    int count;
    const int32_t *list = slot_list(s, which, ring, count);
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int slot = list[idx];
        if (s.ctl[slot].phase != kIter) continue;
        if (s.prec == ABDF_PREC_FP32_LU) {
            const int32_t mode = s.ctl[slot].lu_mode;
            if constexpr (kTakes64) {
                if (mode == kLu64) {
                    newton_solve_cell<double, false>(s, n, slot, smem, red, &decision);
                    continue;
                }
            }
            if (mode != kMode) continue;
        }
        newton_solve_cell<T, kRefine>(s, n, slot, smem, red, &decision);
    }
}

// Every Newton iteration of each listed slot in one launch (FP64 factors), for
// attempts of a few cells where launches dominate: per slot, the same sequence
// of residuals and corrections as the separate kernels.
__global__ void __launch_bounds__(kBlock) k_newton_fused(Slots s, DeviceNet n, int ring, int which) {
    extern __shared__ double smem[];
    __shared__ double red[kLuW + kWaves];
    __shared__ int decision;
    int count;
    const int32_t *list = slot_list(s, which, ring, count);
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int slot = list[idx];
        for (int m = 0; m < s.newton_maxiter; ++m) {
            if (s.ctl[slot].phase != kIter) break;
            newton_rhs_cell<kBlock>(s, n, slot, smem, red);
            if (s.ctl[slot].phase != kIter) break;
            newton_solve_cell<double, false>(s, n, slot, smem, red, &decision);
        }
    }
}

// Acts on the outcome of every active slot's attempt and starts its next one.
__global__ void __launch_bounds__(kBlock) k_control(Slots s, DeviceNet n, int ring) {
    __shared__ SlotCtl cs;
    __shared__ double RU[36], red[kWaves], sh[4], phit[5];
    const int next = (ring + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int old = (ring + 2) % 3;
        s.cnt[old] = 0;
        s.cnt[3 + old] = 0;
        s.cnt[7 + old] = 0;
    }
    const int idx = blockIdx.x;
    if (idx >= s.cnt[ring]) return;
    const int slot = s.act[ring * s.nslots + idx];
    const int S = s.S;
    if (threadIdx.x == 0) cs = s.ctl[slot];
    __syncthreads();
    double *D = s.D + size_t(slot) * kDRows * S;
    const double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S;
    if (cs.phase == kFailed) {
        if (threadIdx.x == 0) {
            cs.n_newton_fail += 1;
            if (!cs.j_fresh) {
                cs.j_fresh = 1;
                cs.jac_refresh = 1;
                cs.n_jac += 1;
                sh[0] = 0.0;
            } else if (s.lu_reuse > 0.0 && cs.c != cs.c_lu) {
                // fresh Jacobian, factorisation kept from another c: retry the
                // same step with the factorisation at the current c
                cs.lu_valid = 0;
                sh[0] = 0.0;
            } else if (s.prec == ABDF_PREC_FP32_LU && cs.lu_mode != kLu64) {
                // the corrector failed with a fresh Jacobian and FP32 factors:
                // the cell retries the same step with refined solves, then
                // with FP64 factors
                cs.lu_mode += 1;
                if (cs.lu_mode == kLu64) cs.lu_valid = 0;
                sh[0] = 0.0;
            } else {
                cs.h = 0.5 * cs.h;
                cs.n_equal = 0;
                if (s.lu_reuse == 0.0) cs.lu_valid = 0;   // else the change of c decides
                sh[0] = 0.5;
            }
        }
        __syncthreads();
        if (sh[0] != 0.0) rescale_D(D, S, cs.q, 0.5, RU);
        begin_attempt(s, n, slot, cs, next, RU, sh + 2, phit);
        return;
    }
    // converged: local error test
    const int q = cs.q;
    const double rtol = cs.rtol;
    const double eq = 1.0 / (q + 1);
    double acc = 0.0;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double sc = atol_of(s, cs, i) + rtol * fmax(fabs(D[i]), fabs(x[i]));
        const double v = eq * d[i] / sc;
        acc += v * v;
    }
    const double err = sqrt(block_sum(acc, red) / S);
    const int m = cs.m_last;
    const double safety = 0.9 * (2 * kNewtonMaxIter + 1) / (2 * kNewtonMaxIter + m);
    if (!isfinite(err)) {
        finish_slot(s, slot, cs, ABDF_CELL_NONFINITE);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (err > 1.0) {
        const double rho = fmax(kMinFactor, safety * growth(err, q + 1));
        if (threadIdx.x == 0) {
            cs.n_err_reject += 1;
            cs.h = cs.h * rho;
            cs.n_equal = 0;
            if (s.lu_reuse == 0.0) cs.lu_valid = 0;   // else the change of c decides
        }
        rescale_D(D, S, q, rho, RU);
        begin_attempt(s, n, slot, cs, next, RU, sh + 2, phit);
        return;
    }
    // accept: update the differences, collect the order-selection norms, and
    // record the step when a tape is attached and the step is in the cell's window
    const int rel = cs.n_steps - (s.tape_w0 ? s.tape_w0[cs.cell] : 0);
    if (s.tape_x && rel >= s.tape_cap && !s.tape_overflow) {
        finish_slot(s, slot, cs, ABDF_CELL_TAPE_FULL);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    double *tx = s.tape_x && rel >= 0 && rel < s.tape_cap ? s.tape_x + (size_t(cs.cell) * s.tape_cap + rel) * S
                                                         : nullptr;
    const double em_c = q > 1 ? 1.0 / q : 0.0;
    const double ep_c = 1.0 / (q + 2);
    double am = 0.0, ap = 0.0;
    bool nonfinite = false;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double sc = atol_of(s, cs, i) + rtol * fmax(fabs(D[i]), fabs(x[i]));
        // rows 0..q+2 of the difference table, with every index static (masks
        // and selects instead of v[q + 1] etc.) so that v stays in registers
        double v[kDRows];
#pragma unroll
        for (int j = 0; j < kDRows; ++j) v[j] = j <= q + 1 ? D[j * S + i] : 0.0;
        const double di = d[i];
        double vq1 = 0.0;
#pragma unroll
        for (int j = 0; j < kDRows; ++j) vq1 = j == q + 1 ? v[j] : vq1;
#pragma unroll
        for (int j = 0; j < kDRows; ++j) {
            if (j == q + 2) v[j] = di - vq1;
            if (j == q + 1) v[j] = di;
        }
#pragma unroll
        for (int j = kDRows - 2; j >= 0; --j)
            if (j <= q) v[j] = v[j] + v[j + 1];
#pragma unroll
        for (int j = 0; j < kDRows; ++j)
            if (j <= q + 2) D[j * S + i] = v[j];
        if (tx) tx[i] = v[0];
        double vq = 0.0, vq2 = 0.0;
#pragma unroll
        for (int j = 0; j < kDRows; ++j) {
            vq = j == q ? v[j] : vq;
            vq2 = j == q + 2 ? v[j] : vq2;
        }
        const double a1 = em_c * vq / sc, a2 = ep_c * vq2 / sc;
        am += a1 * a1;
        ap += a2 * a2;
        nonfinite |= !isfinite(v[0]);
    }
    const double sm = block_sum(am, red);
    const double sp = block_sum(ap, red);
    nonfinite = block_any(nonfinite, red);
    if (threadIdx.x == 0) {
        if (tx) {
            s.tape_h[size_t(cs.cell) * s.tape_cap + rel] = cs.h;
            s.tape_q[size_t(cs.cell) * s.tape_cap + rel] = q;
        } else if (s.tape_x && rel == -1 && s.tape_hprev) {
            s.tape_hprev[cs.cell] = cs.h;
            s.tape_qprev[cs.cell] = q;
        }
        cs.t = cs.landing ? cs.t_end : cs.t + cs.h;
        cs.n_steps += 1;
        cs.n_equal += 1;
        cs.j_fresh = 0;
    }
    __syncthreads();
    if (nonfinite) {
        finish_slot(s, slot, cs, ABDF_CELL_NONFINITE);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (cs.landing || (s.tape_stop && cs.n_steps >= s.tape_stop[cs.cell])) {
        // t_end reached, or a re-run has recorded its window
        finish_slot(s, slot, cs, ABDF_CELL_OK);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (cs.n_equal >= q + 1) {
        if (threadIdx.x == 0) {
            const double e_m = q > 1 ? sqrt(sm / S) : INFINITY;
            const double e_p = q < s.max_order ? sqrt(sp / S) : INFINITY;
            const double r0 = growth(e_m, q), r1 = growth(err, q + 1), r2 = growth(e_p, q + 2);
            int best = 1;
            double rb = r1;
            if (r0 > rb) { best = 0; rb = r0; }
            if (r2 > rb) { best = 2; rb = r2; }
            cs.q = q + best - 1;
            double rho = fmin(kMaxFactor, safety * rb);
            if (s.h_max > 0.0) rho = fmin(rho, s.h_max / cs.h);
            cs.h = cs.h * rho;
            cs.n_equal = 0;
            if (s.lu_reuse == 0.0) cs.lu_valid = 0;   // else the change of c decides
            sh[0] = rho;
        }
        __syncthreads();
        rescale_D(D, S, cs.q, sh[0], RU);
    }
    begin_attempt(s, n, slot, cs, next, RU, sh + 2, phit);
}

// Acts on the stage every active slot has just solved and starts its next
// stage: a converged stage stores G_i = (psi + d) / gamma (its own equation
// gives h f(Y_i)); after stage 7 the error test Y_7 - Y_6 decides the step.
__global__ void __launch_bounds__(kBlock) k_control_rk(Slots s, int ring) {
    __shared__ SlotCtl cs;
    __shared__ double red[kWaves];
    const int next = (ring + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int old = (ring + 2) % 3;
        s.cnt[old] = 0;
        s.cnt[3 + old] = 0;
        s.cnt[7 + old] = 0;
    }
    const int idx = blockIdx.x;
    if (idx >= s.cnt[ring]) return;
    const int slot = s.act[ring * s.nslots + idx];
    const int S = s.S;
    if (threadIdx.x == 0) cs = s.ctl[slot];
    __syncthreads();
    double *D = s.D + size_t(slot) * kDRows * S;
    const double *x = s.x + size_t(slot) * S, *d = s.d + size_t(slot) * S, *psi = s.psi + size_t(slot) * S;
    if (cs.phase == kFailed) {
        if (threadIdx.x == 0) {
            cs.n_newton_fail += 1;
            if (s.prec == ABDF_PREC_FP32_LU && cs.lu_mode != kLu64) {
                // FP32 factors: the same step again with refined solves, then
                // with FP64 factors
                cs.lu_mode += 1;
                if (cs.lu_mode == kLu64) cs.lu_valid = 0;
            } else {
                cs.h = 0.5 * cs.h;
                cs.rejected = 1;
            }
            cs.stage = 2;
        }
        __syncthreads();
        begin_stage_rk(s, slot, cs, next);
        return;
    }
    const int stage = cs.stage;
    for (int i = threadIdx.x; i < S; i += kBlock) D[stage * S + i] = (psi[i] + d[i]) / kRkGamma;
    if (stage < kRkStages) {
        __syncthreads();
        if (threadIdx.x == 0) cs.stage = stage + 1;
        __syncthreads();
        begin_stage_rk(s, slot, cs, next);
        return;
    }
    // error estimate Y_7 - Y_6 = sum_j (a_7j - a_6j) G_j, weights from x_n and Y_7
    const double h = cs.h, rtol = cs.rtol;
    double acc = 0.0;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        double e = (kRkA[6][0] - kRkA[5][0]) * (h * D[S + i]);
        for (int j = 2; j <= kRkStages; ++j) e = e + (kRkA[6][j - 1] - kRkA[5][j - 1]) * D[j * S + i];
        const double sc = atol_of(s, cs, i) + rtol * fmax(fabs(D[i]), fabs(x[i]));
        const double v = e / sc;
        acc += v * v;
    }
    const double err = sqrt(block_sum(acc, red) / S);
    if (!isfinite(err)) {
        finish_slot(s, slot, cs, ABDF_CELL_NONFINITE);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (err > 1.0) {
        if (threadIdx.x == 0) {
            cs.n_err_reject += 1;
            cs.h = cs.h * fmax(kMinFactor, 0.9 * pow(err, -0.2));
            cs.rejected = 1;
            cs.stage = 2;
        }
        __syncthreads();
        begin_stage_rk(s, slot, cs, next);
        return;
    }
    // accept: x_{n+1} = Y_7, and F_1 of the next step is G_7 / h
    bool nonfinite = false;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double xi = x[i];
        D[i] = xi;
        D[S + i] = D[kRkStages * S + i] / h;
        nonfinite |= !isfinite(xi);
    }
    nonfinite = block_any(nonfinite, red);
    if (threadIdx.x == 0) {
        cs.t = cs.landing ? cs.t_end : cs.t + h;
        cs.n_steps += 1;
        cs.jac_refresh = 1;
    }
    __syncthreads();
    if (nonfinite || cs.landing) {
        finish_slot(s, slot, cs, nonfinite ? ABDF_CELL_NONFINITE : ABDF_CELL_OK);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    if (threadIdx.x == 0) {
        double fac = err == 0.0 ? kMaxFactor : fmin(kMaxFactor, fmax(kMinFactor, 0.9 * pow(err, -0.2)));
        if (cs.rejected) {
            fac = fmin(1.0, fac);
            cs.rejected = 0;
        }
        cs.h = h * fac;
        if (s.h_max > 0.0) cs.h = fmin(cs.h, s.h_max);
        cs.stage = 2;
    }
    __syncthreads();
    begin_stage_rk(s, slot, cs, next);
}

// Copies results of finished slots to the caller's arrays.
__global__ void __launch_bounds__(kBlock) k_harvest(Slots s, HarvestArgs h) {
    const int idx = blockIdx.x;
    if (idx == 0 && threadIdx.x == 0) s.cnt[6] = 0;
    if (idx >= h.count) return;
    const int slot = h.slots[idx];
    const SlotCtl &c = s.ctl[slot];
    const long long cell = h.compact ? idx : c.cell;
    const int S = s.S;
    for (int i = threadIdx.x; i < S; i += kBlock) h.x_out[size_t(cell) * S + i] = s.D[size_t(slot) * kDRows * S + i];
    if (threadIdx.x == 0) {
        if (s.tape_len) s.tape_len[c.cell] = c.n_steps;
        h.status[cell] = c.status;
        if (h.stats) {
            abdf_cell_stats st;
            st.n_steps = c.n_steps;
            st.n_attempts = c.n_attempts;
            st.n_err_reject = c.n_err_reject;
            st.n_newton_fail = c.n_newton_fail;
            st.n_rhs = c.n_rhs;
            st.n_jac = c.n_jac;
            st.n_lu = c.n_lu;
            st.order = c.q;
            st.h = c.h;
            st.t = c.t;
            st.n_lu_fp64 = s.prec == ABDF_PREC_FP32_LU ? c.n_lu64 : c.n_lu;
            st.reserved = 0;
            h.stats[cell] = st;
        }
    }
}

// ---------------------------------------------------------------- adjoint --
//
// Reverse sweep of the frozen-sequence BDF map: the accepted (h_n, q_n) of a
// recorded solve, each corrector equation c f(x_{n+1}) - psi - d = 0 taken as
// solved exactly.  lambda_j (stored in D) is the adjoint of difference row j.
// Step n, in reverse:
//   difference update   lambda_{j+1} += lambda_j (j = 0..q), lambda_d =
//                       lambda_{q+1} + lambda_{q+2}, lambda_{q+1} = -lambda_{q+2},
//                       lambda_{q+2} = 0
//   corrector           mu = M^{-T} lambda_d with M = I - c J(x_{n+1}) factored afresh,
//                       solved as lambda_xp = mu - lambda_d = M^{-T} c J^T lambda_d
//   predictor           lambda_j += lambda_xp (j <= q), lambda_j -= gamma_j / gamma_q mu (1 <= j <= q)
//   parameters          dL/dk_r += c x_a x_b (nu_r . mu)   (x at x_{n+1}, x_b only for two reactants)
//   step-size change    lambda_{0..q} <- (R(rho) U) lambda when (h, q) changed from step n-1
// and finally, for D_0 = x_0 and D_1 = h_0 f(x_0):
//   dL/dk_r += h_0 x_a x_b (nu_r . lambda_1) at x_0,  dL/dx_0 = lambda_0 + h_0 J(x_0)^T lambda_1.
// The sweep accumulates the gradient with respect to the rate coefficients;
// dL/dlog alpha_r = k_r dL/dk_r (k_r is linear in alpha_r) and the gradient with
// respect to a cell's physical parameters, sum_r dL/dk_r dk_r/dphi, are formed
// when the cell finishes.  Neither divides by a parameter, so both stay finite
// where G0 = 0 or zeta = 0 switches a family of reactions off.

// x_a (x_b): the abundance factor of rate_r = k_r x_a (x_b), from the packed reactant pair
__device__ __forceinline__ double reactant_product(const DeviceNet &n, const double *xs, int r) {
    const int ab = n.rx_ab[r];
    const int a = ab & 0xffff, b = (ab >> 16) & 0xffff;
    double v = xs[a];
    if (b != 0xffff) v *= xs[b];
    return v;
}

// nu_r . v over the reaction's net stoichiometry
__device__ __forceinline__ double nu_dot(const DeviceNet &n, const double *v, int r) {
    double w = 0.0;
    for (int e = n.rnu_ptr[r]; e < n.rnu_ptr[r + 1]; ++e) {
        const int ent = n.rnu_ent[e];
        w += double((ent & 7) - 4) * v[ent >> 3];
    }
    return w;
}

// Reverse of rescale_D: lambda_old[b] = sum_a RU[b][a] lambda_new[a], rows 0..q.
__device__ __forceinline__ void rescale_adjoint(double *L, int S, int q, double rho, double *RU) {
    interp_product(q, rho, RU);
    __syncthreads();
    for (int i = threadIdx.x; i < S; i += kBlock) {
        double v[kMaxOrder + 1], w[kMaxOrder + 1];
#pragma unroll
        for (int j = 0; j <= kMaxOrder; ++j) v[j] = j <= q ? L[j * S + i] : 0.0;
#pragma unroll
        for (int b = 0; b <= kMaxOrder; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a <= kMaxOrder; ++a)
                if (a <= q) acc += RU[b * 6 + a] * v[a];
            w[b] = acc;
        }
#pragma unroll
        for (int j = 0; j <= kMaxOrder; ++j)
            if (j <= q) L[j * S + i] = w[j];
    }
    __syncthreads();
}

// c J(x)^T v (into out, global) for one slot: w_r = nu_r . v, then
// (J^T v)_j = sum over reactions r with reactant j of d rate_r / d x_j w_r.
// xs, v in LDS; w: LDS scratch [R].
__device__ __forceinline__ void jac_transpose_apply(const DeviceNet &n, const double *k, const double *xs,
                                                    const double *v, double *w, double c, double *out, int S) {
    for (int r = threadIdx.x; r < n.R; r += kBlock) w[r] = nu_dot(n, v, r);
    __syncthreads();
    for (int j = threadIdx.x; j < S; j += kBlock) {
        double jt = 0.0;
        for (int e = n.dcol_ptr[j]; e < n.dcol_ptr[j + 1]; ++e) {
            const int ent = n.dcol_ent[e];
            const int r = ent >> 16, o = (ent & 0xffff) - 1;
            double d = n.dcol_coef[e] * k[r];
            if (o >= 0) d *= xs[o];
            jt += d * w[r];
        }
        out[j] = c * jt;
    }
    __syncthreads();
}

// Queues reverse step cs.n_steps - 1 of a slot: the reverse of its difference
// update (lambda_d kept in psi), the corrector point, c, and the right-hand
// side c J(x_{n+1})^T lambda_d of the transposed solve.  The solve then
// yields lambda_xp = mu - lambda_d = M^{-T} c J^T lambda_d directly: the
// adjoint rows can be many orders of magnitude larger than lambda_xp, and
// forming mu first and subtracting lambda_d would lose it to cancellation.
// LDS: xs [S], ls [S], w [R].
__device__ __forceinline__ void adj_begin(const Slots &s, const DeviceNet &n, int slot, SlotCtl &cs, int ring,
                                          double *smem) {
    const int S = s.S;
    const int w0 = s.tape_w0 ? s.tape_w0[cs.cell] : 0;
    const size_t te = size_t(cs.cell) * s.tape_cap + (cs.n_steps - 1 - w0);
    const int q = s.tape_q[te];
    const double h = s.tape_h[te];
    const double c = h / bdf_gamma(q);
    double *L = s.D + size_t(slot) * kDRows * S;
    double *rb = s.rb + size_t(slot) * S, *xJ = s.xJ + size_t(slot) * S, *lam_d = s.psi + size_t(slot) * S;
    const double *xt = s.tape_x + te * S;
    double *xs = smem, *ls = xs + S, *w = ls + S;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        double v[kDRows];
        for (int j = 0; j <= q + 2; ++j) v[j] = L[j * S + i];
        for (int j = 0; j <= q; ++j) v[j + 1] = v[j + 1] + v[j];
        const double ld = v[q + 1] + v[q + 2];
        v[q + 1] = -v[q + 2];
        v[q + 2] = 0.0;
        for (int j = 0; j <= q + 2; ++j) L[j * S + i] = v[j];
        ls[i] = ld;
        lam_d[i] = ld;
        const double xv = xt[i];
        xs[i] = xv;
        xJ[i] = xv;
    }
    __syncthreads();
    jac_transpose_apply(n, s.k + size_t(slot) * n.R, xs, ls, w, c, rb, S);
    if (threadIdx.x == 0) {
        cs.h = h;
        cs.q = q;
        cs.c = c;
        cs.jv_valid = 0;   // x_J moved to the step's corrector point
        const int p = atomicAdd(&s.cnt[ring], 1);
        s.act[ring * s.nslots + p] = slot;
        const int pl = atomicAdd(&s.cnt[3 + ring], 1);
        s.lul[ring * s.nslots + pl] = slot;
        s.ctl[slot] = cs;
    }
}

// Contributions of the starting differences and dL/dx_0 (into s.x); ends the slot.
// LDS: xs [S], l1 [S], w [R].
__device__ __forceinline__ void adj_finish(const Slots &s, const DeviceNet &n, int slot, SlotCtl &cs, int len,
                                           double *smem) {
    const int S = s.S, R = n.R;
    double *L = s.D + size_t(slot) * kDRows * S;
    double *dx0 = s.x + size_t(slot) * S;
    if (len > 0) {
        double *xs = smem, *l1 = xs + S, *w = l1 + S;
        const double h0 = s.tape_h[size_t(cs.cell) * s.tape_cap];
        const double *x0 = s.tape_x0 + size_t(cs.cell) * S;
        const double *k = s.k + size_t(slot) * R;
        double *g = s.g + size_t(slot) * R;
        for (int i = threadIdx.x; i < S; i += kBlock) {
            xs[i] = x0[i];
            l1[i] = L[S + i];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < R; r += kBlock) g[r] += h0 * reactant_product(n, xs, r) * nu_dot(n, l1, r);
        __syncthreads();
        // dL/dx0 = lambda_0 + h0 J(x0)^T lambda_1 (dx0 first holds the second term)
        jac_transpose_apply(n, k, xs, l1, w, h0, dx0, S);
        for (int i = threadIdx.x; i < S; i += kBlock) dx0[i] = L[i] + dx0[i];
    } else {
        for (int i = threadIdx.x; i < S; i += kBlock) dx0[i] = L[i];
    }
    __syncthreads();
    finish_slot(s, slot, cs, cs.status == kRunning ? ABDF_CELL_OK : cs.status);
    __syncthreads();
    if (threadIdx.x == 0) s.ctl[slot] = cs;
}

// Places cells in slots for the reverse sweep: lambda_0 = dL/dx(t_end), rate
// coefficients, zero gradient, and the last recorded step queued.
__global__ void __launch_bounds__(kBlock) k_adj_admit(Slots s, DeviceNet n, AdjArgs a, int ring) {
    extern __shared__ double smem[];
    __shared__ SlotCtl cs;
    const int idx = blockIdx.x;
    if (idx >= a.count) return;
    const int slot = a.slots[idx];
    const long long cell = a.cells[idx];
    const int S = s.S, R = n.R;
    const bool ok = a.status[cell] == ABDF_CELL_OK;
    if (s.win_end && s.win_end[cell] < 0) {
        // windowed sweep: nothing of this cell in the pass
        if (threadIdx.x == 0) {
            SlotCtl z = {};
            z.cell = int32_t(cell);
            cs = z;
        }
        __syncthreads();
        finish_slot(s, slot, cs, kSitsOut);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
        return;
    }
    double *phi = s.phi + size_t(slot) * 5;
    if (threadIdx.x == 0) {
        for (int j = 0; j < 5; ++j) phi[j] = a.phi[cell * 5 + j];
        SlotCtl z = {};
        z.cell = int32_t(cell);
        z.n_steps = ok ? (s.win_end ? s.win_end[cell] : s.tape_len[cell]) : 0;
        z.status = ok ? kRunning : a.status[cell];
        z.q = 1;
        cs = z;
    }
    double *L = s.D + size_t(slot) * kDRows * S;
    double *g = s.g + size_t(slot) * R;
    if (ok && s.win_resume) {
        // the adjoint rows and dL/dk where the previous pass (the later window) left them
        const double *wl = s.win_lam + size_t(cell) * kDRows * S;
        for (int i = threadIdx.x; i < kDRows * S; i += kBlock) L[i] = wl[i];
        for (int r = threadIdx.x; r < R; r += kBlock) g[r] = s.win_g[size_t(cell) * R + r];
    } else {
        for (int i = threadIdx.x; i < S; i += kBlock) {
            L[i] = ok ? a.dLdx[cell * S + i] : 0.0;
            for (int j = 1; j < kDRows; ++j) L[j * S + i] = 0.0;
        }
        for (int r = threadIdx.x; r < R; r += kBlock) g[r] = 0.0;
    }
    __syncthreads();
    cell_rates(n, phi, s.k + size_t(slot) * R);
    __syncthreads();
    if (cs.n_steps == 0)
        adj_finish(s, n, slot, cs, 0, smem);
    else
        adj_begin(s, n, slot, cs, ring, smem);
}

// lambda_xp = M^{-T} (c J^T lambda_d) for every queued slot (persistent).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_solve(Slots s, int ring) {
    extern __shared__ double smem[];
    const int count = s.cnt[ring];
    const int S = s.S, NP = s.NP;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int slot = s.act[ring * s.nslots + idx];
        double *b = smem, *z = b + NP, *t = z + NP, *Db = t + 5 * kLuW;
        const double *rb = s.rb + size_t(slot) * S;
        for (int i = threadIdx.x; i < NP; i += kBlock) b[i] = i < S ? rb[i] : 0.0;
        __syncthreads();
        lu_solve_left_T<T>(slot_lu<T>(s, slot), s.perm + size_t(slot) * NP,
                           NP, b, z, t, Db);
        double *d = s.d + size_t(slot) * S;
        for (int i = threadIdx.x; i < S; i += kBlock) d[i] = z[i];
        __syncthreads();
    }
}

// Completes the current reverse step of every queued slot and queues the
// previous one (or finishes the slot).  One workgroup per slot.
__global__ void __launch_bounds__(kBlock) k_adj_step(Slots s, DeviceNet n, int ring) {
    extern __shared__ double smem[];
    __shared__ SlotCtl cs;
    __shared__ double RU[36];
    const int next = (ring + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int old = (ring + 2) % 3;
        s.cnt[old] = 0;
        s.cnt[3 + old] = 0;
        s.cnt[7 + old] = 0;
    }
    const int idx = blockIdx.x;
    if (idx >= s.cnt[ring]) return;
    const int slot = s.act[ring * s.nslots + idx];
    const int S = s.S, R = n.R;
    if (threadIdx.x == 0) cs = s.ctl[slot];
    __syncthreads();
    const int q = cs.q;
    const double c = cs.c, gq = bdf_gamma(q);
    double *L = s.D + size_t(slot) * kDRows * S;
    const double *lam_d = s.psi + size_t(slot) * S, *lxp_g = s.d + size_t(slot) * S, *xJ = s.xJ + size_t(slot) * S;
    double *xs = smem, *ms = xs + S;
    double gr[kMaxOrder + 1];
    for (int j = 1; j <= q; ++j) gr[j] = bdf_gamma(j) / gq;
    for (int i = threadIdx.x; i < S; i += kBlock) {
        const double lxp = lxp_g[i];
        const double m = lam_d[i] + lxp;
        xs[i] = xJ[i];
        ms[i] = m;
        L[i] = L[i] + lxp;
        for (int j = 1; j <= q; ++j) L[j * S + i] = L[j * S + i] + (lxp - gr[j] * m);
    }
    __syncthreads();
    double *g = s.g + size_t(slot) * R;
    for (int r = threadIdx.x; r < R; r += kBlock) g[r] += c * reactant_product(n, xs, r) * nu_dot(n, ms, r);
    __syncthreads();
    const int m = cs.n_steps - 1;
    const int w0 = s.tape_w0 ? s.tape_w0[cs.cell] : 0;
    if (m > 0) {
        // (h, q) of step m - 1: in the window, or the one recorded just before it
        const size_t te = size_t(cs.cell) * s.tape_cap + (m - 1 - w0);
        const double hp = m > w0 ? s.tape_h[te] : s.tape_hprev[cs.cell];
        const int qp = m > w0 ? s.tape_q[te] : s.tape_qprev[cs.cell];
        if (cs.h != hp || q != qp) rescale_adjoint(L, S, q, cs.h / hp, RU);
    }
    if (threadIdx.x == 0) cs.n_steps = m;
    __syncthreads();
    if (m > w0) {
        adj_begin(s, n, slot, cs, next, smem);
    } else if (m > 0) {
        // the window is swept: the earlier steps come in the next pass
        double *wl = s.win_lam + size_t(cs.cell) * kDRows * S;
        for (int i = threadIdx.x; i < kDRows * S; i += kBlock) wl[i] = L[i];
        for (int r = threadIdx.x; r < R; r += kBlock) s.win_g[size_t(cs.cell) * R + r] = g[r];
        __syncthreads();
        finish_slot(s, slot, cs, kWindowDone);
        __syncthreads();
        if (threadIdx.x == 0) s.ctl[slot] = cs;
    } else {
        adj_finish(s, n, slot, cs, 1, smem);
    }
}

// dk_r / dphi_j of one reaction for phi = (T, n_H, A_V, zeta, G0) (paper Sec. 2
// Kooij-Arrhenius and direct cosmic-ray laws, App. B.1 photo and cosmic-ray-
// induced photon laws), written without dividing by zeta or G0: the
// cosmic-ray and photo coefficients are linear in them.
__device__ __forceinline__ void rate_param_derivs(const DeviceNet &n, int r, const double *phi, double k,
                                                  double d[5]) {
    const double T = phi[0], nH = phi[1], Av = phi[2];
    const int t = n.rx_type[r];
    d[0] = d[1] = d[2] = d[3] = d[4] = 0.0;
    if (t == kTwoBody) {
        d[0] = k * (n.beta[r] + n.gamma[r] / T) / T;
        d[1] = k / nH;
    } else if (t == kCosmicRay) {
        d[3] = n.alpha[r];
    } else if (t == kCrPhoton) {
        d[0] = k * n.beta[r] / T;
        d[3] = n.alpha[r] * pow(T / 300.0, n.beta[r]) * (n.gamma[r] / (1.0 - n.albedo));
    } else {
        d[2] = -n.gamma[r] * k;
        d[4] = n.alpha[r] * exp(-n.gamma[r] * Av);
    }
}

// Copies the gradients of finished reverse slots to per-cell arrays: dL/dlog
// alpha_r = k_r dL/dk_r, dL/dx_0, and dL/dphi = sum_r dL/dk_r dk_r/dphi
// (per-thread sums in reaction order, then a fixed tree).
__global__ void __launch_bounds__(kBlock) k_adj_harvest(Slots s, DeviceNet n, AdjHarvestArgs h) {
    __shared__ double red[kWaves];
    const int idx = blockIdx.x;
    if (idx == 0 && threadIdx.x == 0) s.cnt[6] = 0;
    if (idx >= h.count) return;
    const int slot = h.slots[idx];
    const int32_t fin = s.ctl[slot].status;
    if (fin == kWindowDone || fin == kSitsOut) return;   // the cell's result comes in a later pass
    const long long cell = s.ctl[slot].cell;
    const int S = s.S, R = s.R;
    const double *gk = s.g + size_t(slot) * R, *k = s.k + size_t(slot) * R, *phi = s.phi + size_t(slot) * 5;
    // a cell whose forward solve failed contributes zeros (its coefficients
    // may not even be finite, e.g. for a non-physical temperature)
    const bool ok = s.ctl[slot].status == ABDF_CELL_OK;
    if (h.g_cell)
        for (int r = threadIdx.x; r < R; r += kBlock) h.g_cell[size_t(cell) * R + r] = ok ? k[r] * gk[r] : 0.0;
    if (h.dx0)
        for (int i = threadIdx.x; i < S; i += kBlock) h.dx0[size_t(cell) * S + i] = s.x[size_t(slot) * S + i];
    if (h.dphi) {
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int r = ok ? int(threadIdx.x) : R; r < R; r += kBlock) {
            double d[5];
            rate_param_derivs(n, r, phi, k[r], d);
            const double g = gk[r];
#pragma unroll
            for (int j = 0; j < 5; ++j) acc[j] += g * d[j];
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const double v = block_sum(acc[j], red);
            if (threadIdx.x == 0) h.dphi[size_t(cell) * 5 + j] = v;
        }
    }
}

// out[r] = sum over cells of g_cell[c][r], cells in order.
__global__ void k_grad_sum(const double *g_cell, long long cells, int R, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double acc = 0.0;
    for (long long c = 0; c < cells; ++c) acc += g_cell[size_t(c) * R + r];
    out[r] = acc;
}

constexpr int kAsmThreads = 512;   // workgroup of the stand-alone Newton-matrix assembly

// dL/dphi of one cell (one workgroup) from its dL/dlog alpha: five sums over
// reactions of g_r d log k_r / d phi_j (paper Sec. 2, App. B.1 rate laws).
__global__ void __launch_bounds__(kBlock) k_phys_grad(DeviceNet n, PhysArgs p, const double *g_cell, double *out) {
    __shared__ double red[kWaves];
    const long long c = blockIdx.x;
    const double T = p.T[c], nH = p.nH[c], zeta = p.zeta[c], G0 = p.G0[c];
    const double *g = g_cell + size_t(c) * n.R;
    double sT = 0.0, sN = 0.0, sA = 0.0, sZ = 0.0, sG = 0.0;
    for (int r = threadIdx.x; r < n.R; r += kBlock) {
        const int t = n.rx_type[r];
        const double gr = g[r];
        if (t == kTwoBody) {
            sT += gr * (n.beta[r] + n.gamma[r] / T) / T;
            sN += gr / nH;
        } else if (t == kCosmicRay) {
            sZ += gr / zeta;
        } else if (t == kCrPhoton) {
            sT += gr * n.beta[r] / T;
            sZ += gr / zeta;
        } else {
            sA += -n.gamma[r] * gr;
            sG += gr / G0;
        }
    }
    sT = block_sum(sT, red);
    sN = block_sum(sN, red);
    sA = block_sum(sA, red);
    sZ = block_sum(sZ, red);
    sG = block_sum(sG, red);
    if (threadIdx.x == 0) {
        double *o = out + size_t(c) * 5;
        o[0] = sT;
        o[1] = sN;
        o[2] = sA;
        o[3] = sZ;
        o[4] = sG;
    }
}

// ------------------------------------------------- component entry kernels --

__global__ void __launch_bounds__(kBlock) k_rates_only(DeviceNet n, PhysArgs p, double *k_out) {
    __shared__ double phi[5];
    const long long c = blockIdx.x;
    if (threadIdx.x == 0) {
        phi[0] = p.T[c]; phi[1] = p.nH[c]; phi[2] = p.Av[c]; phi[3] = p.zeta[c]; phi[4] = p.G0[c];
    }
    __syncthreads();
    cell_rates(n, phi, k_out + size_t(c) * n.R);
}

__global__ void __launch_bounds__(kRhsThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_rhs_only(DeviceNet n, const double *k, const double *x, double *f) {
    extern __shared__ double smem[];
    const long long c = blockIdx.x;
    double *xs = smem, *rate = xs + n.S;
    for (int i = threadIdx.x; i < n.S; i += kRhsThreads) xs[i] = x[size_t(c) * n.S + i];
    __syncthreads();
    cell_rhs<kRhsThreads, true>(n, k + size_t(c) * n.R, xs, rate, f + size_t(c) * n.S);
}

// The standalone right-hand side, streaming: each workgroup walks the cells
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next cell's k and x are loaded
// into registers while the current cell's sums run (RhsResident).
template <int kKU, int kGPW>
__global__ void __launch_bounds__(kRhsStreamThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_rhs_stream(DeviceNet n, long long C, const double *__restrict__ k, const double *__restrict__ x,
             double *__restrict__ f) {
    using RR = RhsResident<kKU, kGPW>;
    constexpr int NT = kRhsStreamThreads;
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int S = n.S, R = n.R;
    RR rr;
    rr.load(n, smem);
    RR::init_lds(n, smem);
    double *xs = smem + R + 1;
    long long c = blockIdx.x;
    double kr[kKU], xr = 0.0;
    if (c < C) {
#pragma unroll
        for (int u = 0; u < kKU; ++u) kr[u] = tid + u * NT < R ? k[size_t(c) * R + tid + u * NT] : 0.0;
        if (tid < S) xr = x[size_t(c) * S + tid];
    }
    for (; c < C; c += gridDim.x) {
        const long long cn = c + gridDim.x;
        if (tid < S) xs[tid] = xr;
        __syncthreads();
        rr.rates(n, kr, smem);
        __syncthreads();
        if (cn < C) {
#pragma unroll
            for (int u = 0; u < kKU; ++u)
                if (tid + u * NT < R) kr[u] = k[size_t(cn) * R + tid + u * NT];
            if (tid < S) xr = x[size_t(cn) * S + tid];
        }
        rr.sums(n, smem, f + size_t(c) * S);
        __syncthreads();
    }
}

// Writes the unpadded S x S Newton matrix of each cell through the solver's
// own path: the Jacobian nonzeros at x (jacobian_values, into the scratch jv of
// nnzJ doubles per cell), then every entry as NewtonMatrixSource yields it to
// the factorisation's gather.
__global__ void __launch_bounds__(kAsmThreads) k_newton_matrix_only(DeviceNet n, const double *k, const double *x,
                                                                  const double *cvec, double *jv, double *M) {
    extern __shared__ double smem[];
    const long long c = blockIdx.x;
    double *xs = smem;
    for (int i = threadIdx.x; i < n.S; i += kAsmThreads) xs[i] = x[size_t(c) * n.S + i];
    __syncthreads();
    double *jvc = jv + size_t(c) * max(n.nnzJ, 1);
    jacobian_values<kAsmThreads>(n, k + size_t(c) * n.R, xs, jvc);
    __syncthreads();
    const NewtonMatrixSource<double> src{n.jmask, n.jbase, n.nbw, jvc, cvec[c]};
    for (size_t e = threadIdx.x; e < size_t(n.S) * n.S; e += kAsmThreads) {
        const int i = int(e / n.S), j = int(e % n.S);
        M[size_t(c) * n.S * n.S + e] = src.entry(src.row(i, j & ~63), i, j);
    }
}

// Copies an n x n matrix into the padded NP x NP work matrix (identity padding) and back.
template <typename T>
__global__ void k_pad_in(int n, int NP, const double *A, T *W) {
    const long long b = blockIdx.y;
    for (long long e = blockIdx.x * blockDim.x + threadIdx.x; e < (long long)NP * NP; e += gridDim.x * blockDim.x) {
        const int i = int(e / NP), j = int(e % NP);
        double v = (i < n && j < n) ? A[(b * n + i) * n + j] : (i == j ? 1.0 : 0.0);
        W[b * NP * NP + e] = T(v);
    }
}

// Factors (rows in storage order, row i of P A at storage row permW[i]) back
// to the LAPACK layout: row i of the output is row i of P A.
template <typename T>
__global__ void k_pad_out(int n, int NP, const T *W, double *A, const int32_t *permW, int32_t *perm) {
    const long long b = blockIdx.y;
    for (long long e = blockIdx.x * blockDim.x + threadIdx.x; e < (long long)n * n; e += gridDim.x * blockDim.x) {
        const int i = int(e / n), j = int(e % n);
        A[(b * n + i) * n + j] = double(W[b * NP * NP + (long long)permW[b * NP + i] * NP + j]);
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < n; i += blockDim.x) perm[b * n + i] = permW[b * NP + i];
}

__global__ void k_copy_perm(int n, int NP, const int32_t *perm, int32_t *permW) {
    const long long b = blockIdx.x;
    for (int i = threadIdx.x; i < NP; i += blockDim.x) permW[b * NP + i] = i < n ? perm[b * n + i] : i;
}

template <typename T>
__global__ void __launch_bounds__(lu_threads<T>) k_lu_factor_only(int NP, T *W, int32_t *permW, T *dinv,
                                                              int32_t *info) {
    extern __shared__ double smem[];
    const long long b = blockIdx.x;
    T *A = W + b * NP * NP;
    lu_factor_left<T>(A, NP, permW + b * NP, dinv + b * lu2_dinv_elems<T>(NP), info ? info + b : nullptr,
                      reinterpret_cast<unsigned char *>(smem), DenseSource<T>{A, NP});
}

// Inverse diagonal blocks of LAPACK-layout factors (rows already in P A order).
__global__ void __launch_bounds__(lu_threads<double>) k_dinv_only(int NP, const double *W, double *dinv) {
    extern __shared__ double smem[];
    const long long b = blockIdx.x;
    double *Cb = smem, *Xb = Cb + kLuW * kLdb, *Yb = Xb + kLuW * kLdb, *Tb = Yb + kLuW * kLdb;
    for (int j = 0; j * kLuW < NP; ++j) {
        const int r0 = j * kLuW, Wj = min(kLuW, NP - r0);
        for (int e = threadIdx.x; e < Wj * Wj; e += lu_threads<double>)
            Cb[(e / Wj) * kLdb + e % Wj] = W[b * NP * NP + size_t(r0 + e / Wj) * NP + r0 + e % Wj];
        __syncthreads();
        diag_inverses<double>(Cb, Wj, dinv + b * lu2_dinv_elems<double>(NP) + size_t(j) * 2 * kLuW * kLuW, Xb, Yb,
                              Tb);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_lu_solve_only(int NP, int n, const double *W, const double *dinv,
                                                          const int32_t *permW, double *bvec) {
    extern __shared__ double smem[];
    __shared__ double t[kLuW];
    const long long bi = blockIdx.x;
    double *b = smem, *y = b + NP;
    for (int i = threadIdx.x; i < NP; i += kBlock) b[i] = i < n ? bvec[bi * n + i] : 0.0;
    __syncthreads();
    // the padding past n is the identity's (k_pad_in, k_copy_perm)
    lu_solve_left<double>(W + bi * NP * NP, dinv + bi * lu2_dinv_elems<double>(NP), nullptr, permW + bi * NP, NP,
                          min(NP, n + (n & 1)), b, y, t);
    for (int i = threadIdx.x; i < n; i += kBlock) bvec[bi * n + i] = y[i];
}

// Matrix-core lane-layout check: D = A B for integer-valued A (16x4), B (4x16).
__global__ void k_selftest(int *bad) {
    const int l = threadIdx.x;
    auto Aval = [](int i, int k) { return double((i * 7 + k * 3) % 11 - 5); };
    auto Bval = [](int k, int j) { return double((k * 5 + j * 2) % 13 - 6); };
    f64x4 cd = {0, 0, 0, 0};
    cd = Mfma<double>::mma(Aval(l & 15, l >> 4), Bval(l >> 4, l & 15), cd);
    f32x4 cf = {0, 0, 0, 0};
    cf = Mfma<float>::mma(float(Aval(l & 15, l >> 4)), float(Bval(l >> 4, l & 15)), cf);
    int nb = 0;
    for (int v = 0; v < 4; ++v) {
        const int j = l & 15;
        double ref_d = 0.0, ref_f = 0.0;
        const int id = Mfma<double>::row(l, v), jf = Mfma<float>::row(l, v);
        for (int k = 0; k < 4; ++k) {
            ref_d += Aval(id, k) * Bval(k, j);
            ref_f += Aval(jf, k) * Bval(k, j);
        }
        nb += (cd[v] != ref_d) + (double(cf[v]) != ref_f);
    }
    // wave arg-max: several value patterns with ties, checked against brute force
    for (int pat = 0; pat < 4; ++pat) {
        auto val = [pat](int i) {
            return pat == 0 ? double((i * 37) % 64) : pat == 1 ? double((i * 13) % 7) : pat == 2 ? 1.0 : double(i % 5 == 3 ? 9 : -1);
        };
        double v = val(l);
        int k = (l * 29 + pat) % 64;
        double bv = val(0);
        int bk = (pat) % 64;
        for (int i = 1; i < 64; ++i) {
            const double vi = val(i);
            const int ki = (i * 29 + pat) % 64;
            if (vi > bv || (vi == bv && ki < bk)) { bv = vi; bk = ki; }
        }
        double v2 = v;
        int k2 = k;
        wave_argmax(v, k);
        nb += (v != bv) + (k != bk);
        wave_argmax_ballot(v2, k2);
        nb += (v2 != bv) + (k2 != bk);
    }
    {
        double v = -1.0;     // no lane with a candidate
        int k = l;
        wave_argmax_ballot(v, k);
        nb += !(v < 0.0);
    }
    atomicAdd(bad, nb);
}

// v[0..n) = value (counters cleared by a kernel rather than a memset node)
__global__ void k_fill_i32(int32_t *v, int32_t value, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = value;
}

// ------------------------------------------------------------- launchers --

hipError_t launch_fill_i32(int32_t *v, int32_t value, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, v, value, n);
    return hipGetLastError();
}

size_t lu_work_lds(int NP, int prec) {
    return prec == ABDF_PREC_FP32_LU ? lu2_lds_bytes<float>(NP) : lu2_lds_bytes<double>(NP);
}

size_t factor_lds(const DeviceNet &n, int prec) {
    return lu_work_lds(n.NP, prec) + sizeof(double) * size_t(n.S);   // factorisation, then x_J
}

// The streaming right-hand sides' instantiation for a network: lanes groups
// per wave (1 or 2) and reactions per thread (ku), or false when the network
// does not fit them.
static bool rhs_stream_shape(const DeviceNet &n, int &ku, int &gpw) {
    constexpr int NW = kRhsStreamThreads / 64;
    if (n.S > kRhsStreamThreads || n.R >= 8191 || n.sg_maxlen > kRhsResidentLen || n.n_sgroup > 2 * NW) return false;
    gpw = n.n_sgroup <= NW ? 1 : 2;
    const int need = (n.R + kRhsStreamThreads - 1) / kRhsStreamThreads;
    ku = need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : 16;
    return !(gpw == 2 && ku > 12);   // <16, 2> would spill
}

#define ABDF_RHS_STREAM_PICK(K)                                                                              \
    (gpw == 1 ? (ku == 2 ? (const void *)&K<2, 1> : ku == 4 ? (const void *)&K<4, 1> : ku == 8 ? (const void *)&K<8, 1> \
                 : ku == 12 ? (const void *)&K<12, 1> : (const void *)&K<16, 1>)                                         \
              : (ku == 2 ? (const void *)&K<2, 2> : ku == 4 ? (const void *)&K<4, 2> : ku == 8 ? (const void *)&K<8, 2> \
                 : (const void *)&K<12, 2>))

static size_t newton_rhs_stream_lds(const DeviceNet &n) {
    return sizeof(double) * (2 * size_t(n.S) + n.R + 2) + sizeof(int) * (kRhsStreamThreads + 2);
}

int resident_per_cu(int which, int prec, size_t lds) {
    int nb = 0;
    hipError_t e;
    if (which == 0)
        e = prec == ABDF_PREC_FP32_LU
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_factor<float>, lu_threads<float>, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_factor<double>, lu_threads<double>, lds);
    else if (which == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_newton_rhs, kRhsThreads, lds);
    else if (which == 2)
        e = prec == ABDF_PREC_FP32_LU
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_newton_solve<float, false>, kBlock, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_newton_solve<double, false>, kBlock, lds);
    else if (which == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_newton_solve<float, true>, kBlock, lds);
    else
        e = prec == ABDF_PREC_FP32_LU
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_solve<float>, kBlock, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_solve<double>, kBlock, lds);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

size_t lu_bytes(int NP, int prec) {
    return size_t(NP) * NP * (prec == ABDF_PREC_FP32_LU ? sizeof(float) : sizeof(double));
}

size_t dinv_bytes(int NP, int prec) {
    return prec == ABDF_PREC_FP32_LU ? lu2_dinv_elems<float>(NP) * sizeof(float)
                                     : lu2_dinv_elems<double>(NP) * sizeof(double);
}

#define LAUNCH_CHECK() hipGetLastError()

hipError_t launch_admit(const Slots &s, const DeviceNet &n, const AdmitArgs &a, int ring, size_t lds, hipStream_t st) {
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_admit, dim3(a.count), dim3(kBlock), lds, st, s, n, a, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_factor(const Slots &s, const DeviceNet &n, int ring, int grid, int grid64, size_t lds,
                         size_t lds32, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (s.prec == ABDF_PREC_FP32_LU) {
        hipLaunchKernelGGL(k_factor<float>, dim3(grid), dim3(lu_threads<float>), lds32, st, s, n, ring);
        hipError_t e = LAUNCH_CHECK();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_factor<double>, dim3(s.prec == ABDF_PREC_FP32_LU ? grid64 : grid), dim3(lu_threads<double>), lds,
                       st, s, n, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_newton_rhs(const Slots &s, const DeviceNet &n, int ring, int which, int grid, size_t lds,
                             hipStream_t st) {
    if (grid == 0) return hipSuccess;
    int ku = 0, gpw = 0;
    if (rhs_stream_shape(n, ku, gpw)) {
        Slots ss = s;
        DeviceNet nn = n;
        int rr = ring, ww = which;
        void *args[] = {&ss, &nn, &rr, &ww};
        return hipLaunchKernel(ABDF_RHS_STREAM_PICK(k_newton_rhs_stream), dim3(grid), dim3(kRhsStreamThreads), args,
                               newton_rhs_stream_lds(n), st);
    }
    hipLaunchKernelGGL(k_newton_rhs, dim3(grid), dim3(kRhsThreads), lds, st, s, n, ring, which);
    return LAUNCH_CHECK();
}

int newton_rhs_resident_per_cu(const DeviceNet &n, int prec, size_t lds) {
    int ku = 0, gpw = 0;
    if (!rhs_stream_shape(n, ku, gpw)) return resident_per_cu(1, prec, lds);
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ABDF_RHS_STREAM_PICK(k_newton_rhs_stream),
                                                                      kRhsStreamThreads, newton_rhs_stream_lds(n));
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_newton_fused(const Slots &s, const DeviceNet &n, int ring, int which, int grid, size_t lds,
                               hipStream_t st) {
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_newton_fused, dim3(grid), dim3(kBlock), lds, st, s, n, ring, which);
    return LAUNCH_CHECK();
}

hipError_t launch_newton_solve(const Slots &s, const DeviceNet &n, int ring, int which, int grid, int grid_ref,
                               size_t lds, size_t lds_ref, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (s.prec == ABDF_PREC_FP32_LU) {
        hipLaunchKernelGGL((k_newton_solve<float, false>), dim3(grid), dim3(kBlock), lds, st, s, n, ring, which);
        hipError_t e = LAUNCH_CHECK();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_newton_solve<float, true>), dim3(grid_ref), dim3(kBlock), lds_ref, st, s, n, ring,
                           which);
        return LAUNCH_CHECK();   // FP64-mode slots went with the plain FP32 variant
    }
    hipLaunchKernelGGL((k_newton_solve<double, false>), dim3(grid), dim3(kBlock), lds, st, s, n, ring, which);
    return LAUNCH_CHECK();
}

hipError_t launch_control_rk(const Slots &s, int ring, int grid, hipStream_t st) {
    k_control_rk<<<grid, kBlock, 0, st>>>(s, ring);
    return hipGetLastError();
}

hipError_t launch_control(const Slots &s, const DeviceNet &n, int ring, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_control, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, st, s, n, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_harvest(const Slots &s, const HarvestArgs &h, hipStream_t st) {
    hipLaunchKernelGGL(k_harvest, dim3(h.count > 0 ? h.count : 1), dim3(kBlock), 0, st, s, h);
    return LAUNCH_CHECK();
}

hipError_t launch_adj_admit(const Slots &s, const DeviceNet &n, const AdjArgs &a, int ring, size_t lds, hipStream_t st) {
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_admit, dim3(a.count), dim3(kBlock), lds, st, s, n, a, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_adj_solve(const Slots &s, int ring, int grid, size_t lds, hipStream_t st) {
    if (grid == 0) return hipSuccess;
    if (s.prec == ABDF_PREC_FP32_LU)
        hipLaunchKernelGGL(k_adj_solve<float>, dim3(grid), dim3(kBlock), lds, st, s, ring);
    else
        hipLaunchKernelGGL(k_adj_solve<double>, dim3(grid), dim3(kBlock), lds, st, s, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_adj_step(const Slots &s, const DeviceNet &n, int ring, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_step, dim3(grid > 0 ? grid : 1), dim3(kBlock), lds, st, s, n, ring);
    return LAUNCH_CHECK();
}

hipError_t launch_adj_harvest(const Slots &s, const DeviceNet &n, const AdjHarvestArgs &h, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_harvest, dim3(h.count > 0 ? h.count : 1), dim3(kBlock), 0, st, s, n, h);
    return LAUNCH_CHECK();
}

hipError_t launch_grad_sum(const double *g_cell, long long cells, int R, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_grad_sum, dim3((R + 255) / 256), dim3(256), 0, st, g_cell, cells, R, out);
    return LAUNCH_CHECK();
}

hipError_t launch_phys_grad(const DeviceNet &n, const PhysArgs &p, long long cells, const double *g_cell,
                            double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_phys_grad, dim3(cells), dim3(kBlock), 0, st, n, p, g_cell, out);
    return LAUNCH_CHECK();
}

hipError_t launch_rates(const DeviceNet &n, const PhysArgs &p, long long cells, double *k, hipStream_t st) {
    hipLaunchKernelGGL(k_rates_only, dim3(cells), dim3(kBlock), 0, st, n, p, k);
    return LAUNCH_CHECK();
}

hipError_t plan_rhs(const DeviceNet &n, long long cells, RhsPlan &p) {
    int ku = 0, gpw = 0;
    p = RhsPlan{};
    if (rhs_stream_shape(n, ku, gpw)) {
        p.fn = ABDF_RHS_STREAM_PICK(k_rhs_stream);
        p.lds = sizeof(double) * (size_t(n.S) + n.R + 2);
        p.threads = kRhsStreamThreads;
        int dev = 0, ncu = 0, nb = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, p.fn, kRhsStreamThreads, p.lds);
        if (e != hipSuccess) return e;
        p.grid = std::min<long long>(cells, std::max(1LL, (long long)nb * ncu));
        return hipSuccess;
    }
    p.fn = reinterpret_cast<const void *>(&k_rhs_only);
    p.lds = sizeof(double) * (size_t(n.S) + n.R);
    p.threads = kRhsThreads;
    p.grid = cells;
    return hipSuccess;
}

hipError_t launch_rhs_planned(const RhsPlan &p, const DeviceNet &n, long long cells, const double *k, const double *x,
                              double *f, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
    DeviceNet nn = n;
    long long C = cells;
    const double *kk = k, *xx = x;
    double *ff = f;
    void *args_only[] = {&nn, &kk, &xx, &ff};
    void *args_stream[] = {&nn, &C, &kk, &xx, &ff};
    void **args = p.fn == reinterpret_cast<const void *>(&k_rhs_only) ? args_only : args_stream;
    return hipExtLaunchKernel(p.fn, dim3(unsigned(p.grid)), dim3(p.threads), args, p.lds, st, start, stop, 0);
}

hipError_t launch_newton_matrix(const DeviceNet &n, long long cells, const double *k, const double *x,
                                const double *c, double *M, double *jv, hipStream_t st) {
    const size_t lds = sizeof(double) * size_t(n.S);
    hipLaunchKernelGGL(k_newton_matrix_only, dim3(cells), dim3(kAsmThreads), lds, st, n, k, x, c, jv, M);
    return LAUNCH_CHECK();
}

hipError_t launch_lu_factor(int n, int NP, long long batch, double *A, void *W, int32_t *permW, int32_t *perm,
                            void *dinv, int32_t *info, int prec, hipStream_t st) {
    dim3 g(std::max(1, std::min(64, (NP * NP + 255) / 256)), unsigned(batch));
    if (prec == ABDF_PREC_FP32_LU) {
        hipLaunchKernelGGL(k_pad_in<float>, g, dim3(256), 0, st, n, NP, A, (float *)W);
        hipLaunchKernelGGL(k_lu_factor_only<float>, dim3(batch), dim3(lu_threads<float>), lu2_lds_bytes<float>(NP), st, NP,
                           (float *)W, permW, (float *)dinv, info);
        hipLaunchKernelGGL(k_pad_out<float>, g, dim3(256), 0, st, n, NP, (const float *)W, A, permW, perm);
    } else {
        hipLaunchKernelGGL(k_pad_in<double>, g, dim3(256), 0, st, n, NP, A, (double *)W);
        hipLaunchKernelGGL(k_lu_factor_only<double>, dim3(batch), dim3(lu_threads<double>), lu2_lds_bytes<double>(NP), st,
                           NP, (double *)W, permW, (double *)dinv, info);
        hipLaunchKernelGGL(k_pad_out<double>, g, dim3(256), 0, st, n, NP, (const double *)W, A, permW, perm);
    }
    return LAUNCH_CHECK();
}

hipError_t launch_lu_solve(int n, int NP, long long batch, const double *LU, const int32_t *perm, double *b,
                           void *W, int32_t *permW, void *dinv, hipStream_t st) {
    dim3 g(std::max(1, std::min(64, (NP * NP + 255) / 256)), unsigned(batch));
    hipLaunchKernelGGL(k_pad_in<double>, g, dim3(256), 0, st, n, NP, LU, (double *)W);
    hipLaunchKernelGGL(k_copy_perm, dim3(unsigned(batch)), dim3(256), 0, st, n, NP, perm, permW);
    hipLaunchKernelGGL(k_dinv_only, dim3(batch), dim3(lu_threads<double>), sizeof(double) * (3 * kLuW * kLdb + 1536), st,
                       NP, (const double *)W, (double *)dinv);
    hipLaunchKernelGGL(k_lu_solve_only, dim3(batch), dim3(kBlock), sizeof(double) * 2 * NP, st, NP, n,
                       (const double *)W, (const double *)dinv, permW, b);
    return LAUNCH_CHECK();
}

hipError_t launch_selftest(int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, st, bad);
    return LAUNCH_CHECK();
}

}  // namespace abdf
