// Device-side constants, per-slot state and block-wide reductions (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <limits>

namespace abdf {

constexpr int kBlock = 256;          // threads per workgroup in every per-cell kernel
constexpr int kWaves = kBlock / 64;
constexpr int kMaxOrder = 5;
constexpr int kDRows = kMaxOrder + 3;  // difference rows 0..q+2 at q = 5
constexpr int kNewtonMaxIter = 4;     // BDF corrector iterations per attempt
constexpr int kRkNewtonMaxIter = 10;  // ESDIRK iterations per stage
constexpr double kURound = 2.220446049250313e-16;  // 2^-52
constexpr double kMinFactor = 0.2;
constexpr double kMaxFactor = 10.0;

// status values: >= 0 are the public ABDF_CELL_* codes
constexpr int32_t kRunning = -1;

// Newton phase of the current step attempt
constexpr int32_t kIter = 0;
constexpr int32_t kConverged = 1;
constexpr int32_t kFailed = 2;

// Factor modes of a cell in an FP32-LU engine: FP32 factors with one solve
// per Newton iteration, FP32 factors with one FP64 refinement of each solve,
// FP64 factors.  A cell whose corrector fails with a fresh Jacobian moves to
// the next mode.  FP64 engines use FP64 factors throughout.
constexpr int32_t kLuPlain32 = 0;
constexpr int32_t kLuRefined32 = 1;
constexpr int32_t kLu64 = 2;

struct SlotCtl {
    double t, h, t_end, c, c_lu, eta_old, rtol, atol, newton_tol, err;
    double tc;        // expansion time of the conditions (0: constant)
    int32_t q, n_equal, status, phase, j_fresh, jac_refresh, landing, newton_iter;
    int32_t lu_valid, cell, m_last, lu_mode;   // FP32-LU engines: kLuPlain32, kLuRefined32 or kLu64
    int32_t n_steps, n_attempts, n_err_reject, n_newton_fail, n_rhs, n_jac, n_lu, n_newton_iter;
    int32_t n_lu64;                        // FP32-LU engines: factorisations done in FP64 after a fallback
    int32_t jv_valid;                      // the slot's Jacobian nonzeros are those of the current x_J
    int32_t stage;                         // ESDIRK: the stage being solved (2..7)
    int32_t rejected;                      // ESDIRK: the last attempt was rejected (no growth on the next accept)
};

// Device workspace for n slots of one network (all arrays slot-major).
struct Slots {
    int nslots, S, R, NP, prec, max_steps;
    double lu_reuse;  // keep the factorisation while |c / c_lu - 1| <= lu_reuse (0: while c == c_lu)
    int max_order;    // highest order the order selection may reach (1..kMaxOrder)
    double h0;        // first step (> 0 replaces the starting-step heuristic), seconds
    double h_max;     // bound on every step (0: none), seconds
    int method;       // ABDF_METHOD_BDF or ABDF_METHOD_ESDIRK5
    int newton_maxiter;  // Newton iterations per corrector (kNewtonMaxIter or kRkNewtonMaxIter)
    int tvar;         // cells may have time-dependent conditions (SlotCtl::tc > 0)
    double phi_exp[5];  // phi_j(t) = phi_j(0) (1 + t / tc)^(-phi_exp[j])
    const double *atol_sp;   // [S] per-species absolute tolerances, or null (each cell's atol)
    SlotCtl *ctl;
    double *phi;      // [n][5]: T, n_H, A_V, zeta, G0
    double *k;        // [n][R]
    double *D;        // [n][kDRows][S]: BDF differences; ESDIRK: x_n, F_1, G_2..G_7
    double *x;        // [n][S] Newton iterate
    double *d;        // [n][S] accumulated correction
    double *psi;      // [n][S]
    double *scl;      // [n][S] Newton weights atol + rtol |x_p|
    double *xJ;       // [n][S] point of the current Jacobian
    double *rb;       // [n][S] Newton residual c f(x) - psi - d
    double *jval;     // [n][nnzJ] Jacobian nonzeros at x_J (the factor kernel's input)
    void *lu;         // [n] factors (double or float, NP x NP), rows in storage order, lu_stride bytes apart
    void *dinv;       // [n] inverses of the diagonal blocks' triangles [NB][2][64][64], dinv_stride bytes apart
    size_t lu_stride, dinv_stride;
    int32_t *perm;    // [n][NP]
    int32_t *act;     // [3][n] active-slot lists (ring)
    int32_t *lul;     // [3][n] slots needing a factorisation (ring)
    int32_t *nol;     // [3][n] active slots whose factorisation is current (ring)
    int32_t *fin;     // [n] finished slots since the last harvest
    int32_t *cnt;     // [0..2] active counts, [3..5] factor counts, [6] finished count, [7..9] no-factor counts
    // step tape of the discrete adjoint (null when not recording), indexed by cell
    int tape_cap;     // accepted steps recorded per cell
    double *tape_x;   // [cells][tape_cap][S] x after each accepted step
    double *tape_h;   // [cells][tape_cap] its step size
    int32_t *tape_q;  // [cells][tape_cap] its order
    int32_t *tape_len;  // [cells] accepted steps recorded
    const double *tape_x0;   // [cells][S] initial abundances
    double *g;        // [n][R] reverse sweep: per-slot gradient with respect to log alpha
    // Windows of a cell with more accepted steps than tape_cap: its tape rows
    // hold steps [w0, w0 + tape_cap), w0 = tape_w0[cell]; a forward re-run
    // records the window and stops after tape_stop[cell] accepted steps; the
    // reverse sweep walks one window per pass and carries its adjoint rows and
    // dL/dk between passes in win_lam / win_g.
    const int32_t *tape_w0;    // [cells] window start, or null (0)
    const int32_t *tape_stop;  // [cells] re-run: stop after this many accepted steps (<= 0: not run), or null
    double *tape_hprev;        // [cells] h of the step before the window
    int32_t *tape_qprev;       // [cells] its order
    int tape_overflow;         // steps past the window go unrecorded (else the cell ends TAPE_FULL)
    const int32_t *win_end;    // [cells] reverse: the window's end (< 0: the cell sits the pass out), or null
    double *win_lam;           // [cells][kDRows][S] adjoint rows carried between passes
    double *win_g;             // [cells][R] dL/dk carried between passes
    int win_resume;            // reverse admission resumes from win_lam / win_g (else from dL/dx)
};

// Internal end states of a slot in a windowed reverse pass (never returned).
constexpr int32_t kWindowDone = 100;   // the window is swept; the cell continues in the next pass
constexpr int32_t kSitsOut = 101;      // the cell has no window in this pass

// The factor storage of a slot in element type T.
// Absolute tolerance of species i in a slot's error and Newton weights.
__device__ __forceinline__ double atol_of(const Slots &s, const SlotCtl &cs, int i) {
    return s.atol_sp ? s.atol_sp[i] : cs.atol;
}

template <typename T>
__device__ __forceinline__ T *slot_lu(const Slots &s, int slot) {
    return reinterpret_cast<T *>(static_cast<char *>(s.lu) + size_t(slot) * s.lu_stride);
}
template <typename T>
__device__ __forceinline__ T *slot_dinv(const Slots &s, int slot) {
    return reinterpret_cast<T *>(static_cast<char *>(s.dinv) + size_t(slot) * s.dinv_stride);
}

// Slot lists of the step-attempt loop: every active slot, those that factor
// this attempt, those that do not.
constexpr int kListAll = 0;
constexpr int kListFactor = 1;
constexpr int kListNoFactor = 2;
constexpr int kCountSlots = 16;   // ints in Slots::cnt

__device__ __forceinline__ const int32_t *slot_list(const Slots &s, int which, int ring, int &count) {
    if (which == kListFactor) {
        count = s.cnt[3 + ring];
        return s.lul + ring * s.nslots;
    }
    if (which == kListNoFactor) {
        count = s.cnt[7 + ring];
        return s.nol + ring * s.nslots;
    }
    count = s.cnt[ring];
    return s.act + ring * s.nslots;
}

// One step of a wave-wide arg-max (value descending, key ascending on ties)
// through a DPP lane permutation; lanes outside the pattern keep their pair.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_argmax_step(double &v, int &k) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
    const int ok = __builtin_amdgcn_update_dpp(k, k, CTRL, ROW_MASK, 0xf, false);
    const double ov = __hiloint2double(ohi, olo);
    // selects, not a branch: keeps the reduction free of exec-mask changes
    const bool take = (ov > v) | ((ov == v) & (ok < k));
    v = take ? ov : v;
    k = take ? ok : k;
}

// Arg-max over the 64 lanes of a wave, returned uniformly to every lane:
// swaps within quads, half-row and row mirrors, then the row broadcasts
// that leave the wave's result in lane 63.
__device__ __forceinline__ void wave_argmax(double &v, int &k) {
    dpp_argmax_step<0xB1, 0xf>(v, k);    // quad_perm [1,0,3,2]
    dpp_argmax_step<0x4E, 0xf>(v, k);    // quad_perm [2,3,0,1]
    dpp_argmax_step<0x141, 0xf>(v, k);   // row_half_mirror
    dpp_argmax_step<0x140, 0xf>(v, k);   // row_mirror
    dpp_argmax_step<0x142, 0xa>(v, k);   // row_bcast:15
    dpp_argmax_step<0x143, 0xc>(v, k);   // row_bcast:31
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    k = __builtin_amdgcn_readlane(k, 63);
    v = __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_max_step(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
    return fmax(v, __hiloint2double(ohi, olo));
}

// Arg-max with the result of wave_argmax for values v >= 0 (v < 0 marks a lane
// without a candidate; if no lane has one, v < 0 is returned and k is
// unspecified).  The maximum is reduced alone; the lanes holding it are found
// by a ballot, and only a tie among several of them reduces the keys.
__device__ __forceinline__ void wave_argmax_ballot(double &v, int &k) {
    double m = v;
    m = dpp_max_step<0xB1, 0xf>(m);
    m = dpp_max_step<0x4E, 0xf>(m);
    m = dpp_max_step<0x141, 0xf>(m);
    m = dpp_max_step<0x140, 0xf>(m);
    m = dpp_max_step<0x142, 0xa>(m);
    m = dpp_max_step<0x143, 0xc>(m);
    {
        const int lo = __builtin_amdgcn_readlane(__double2loint(m), 63);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(m), 63);
        m = __hiloint2double(hi, lo);
    }
    if (m < 0.0) {
        v = m;
        return;
    }
    const unsigned long long hit = __ballot(v == m);
    if (__popcll(hit) == 1) {
        k = __builtin_amdgcn_readlane(k, __ffsll(static_cast<unsigned long long>(hit)) - 1);
    } else {
        double tv = v == m ? 1.0 : -1.0;
        int tk = v == m ? k : 0x7fffffff;
        wave_argmax(tv, tk);
        k = tk;
    }
    v = m;
}

// Sum over the workgroup, identical on every thread; fixed reduction order.
// Sum over a workgroup of NT threads (red: NT / 64 doubles), identical on every
// thread; fixed reduction order.
template <int NT>
__device__ inline double block_sum_nt(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

__device__ inline double block_sum(double v, double *red) { return block_sum_nt<kBlock>(v, red); }

// Logical OR over the workgroup.
__device__ inline bool block_any(bool p, double *red) {
    return block_sum(p ? 1.0 : 0.0, red) != 0.0;
}

}  // namespace abdf
