// Left-looking blocked LU with partial pivoting, one workgroup per matrix
// (shape per element type: LuShape), and the matching triangular solves.  The matrix is read through a
// source functor when each block column is first gathered, so it can be
// formed on the fly (the Newton matrix) instead of being stored first.
//
// Storage.  The matrix keeps its rows where they are: row r of P A (the
// "logical" row r) is storage row perm[r].  Pivoting only swaps entries of
// perm, so no row of the matrix is ever moved in memory; every access to a
// factor row goes through perm.  After the factorisation, storage row perm[r]
// holds row r of L (strictly lower part, unit diagonal implied) and of U.
// For each 64-row diagonal block b the inverses of its unit-lower and upper
// triangles are stored in dinv[b][0] and dinv[b][1] (64 x 64, row-major), so
// the triangular solves are products with dense blocks.
//
// Factorisation of block column j (columns 64j .. 64j + Wj - 1):
//  1. the block column is gathered (rows through perm) into MFMA accumulator
//     registers: with W waves, wave w owns row tiles w, w + W, ..., and all 4
//     column tiles of 16;
//  2. for every earlier block i: U_ij = inv(L_ii) C_i (rows 64i..64i+63 of the
//     block column, staged through LDS), then the rows below block i are
//     updated C -= L_{:,i} U_ij on the matrix cores, L read from memory;
//  3. the panel (rows >= 64j) is factored in 16-column sub-panels, one thread
//     per row.  First on the diagonal: one wave factors the sub-panel's 16 x 16
//     diagonal block without row exchanges (lane k holds row k, the pivot row
//     broadcast from its lane), then every other row eliminates against those
//     U rows with no exchange between waves; this is accepted when every
//     multiplier of the sub-panel is at most kPivotThreshold in magnitude
//     (threshold pivoting, u = 1 / kPivotThreshold: the diagonal entry is at
//     least u times the largest candidate of its column).  Otherwise the
//     sub-panel is factored again from its saved entries with partial
//     pivoting: arg-max pivot search (ties to the smaller logical row, as
//     LAPACK's idamax), scaling and rank-1 update; rows keep their positions
//     and only their logical labels change.  After each sub-panel the rest of
//     the block column is updated on the matrix cores;
//  4. the inverses of the diagonal block's triangles are formed and stored,
//     and the block column is written back through perm.
#pragma once

#include "device_common.hpp"
#include "device_lu.hpp"

namespace abdf {

constexpr int kLuW = 64;          // block-column width
constexpr int kLuMaxNP = 512;     // one thread per row in the panel
// Largest multiplier with which a sub-panel keeps its diagonal pivots.  On the
// Newton matrices I - c J of the chemistry networks fewer than 1% of the
// sub-panels exceed it (at large c, late in an integration); the factors'
// backward error stays at the level of partial pivoting there.
constexpr double kPivotThreshold = 4.0;

// Workgroup shape of the factorisation per element type.  FP64: 8 waves of
// 256 VGPRs, each wave holding four row tiles of the block column.  FP32: 16
// waves of 128 VGPRs with two row tiles each (its accumulators are half the
// size), twice the waves to hide latency with.
template <typename T>
struct LuShape;
template <>
struct LuShape<double> { static constexpr int waves = 8, wave_bits = 3; };
template <>
struct LuShape<float> { static constexpr int waves = 16, wave_bits = 4; };
template <typename T>
constexpr int lu_waves = LuShape<T>::waves;
template <typename T>
constexpr int lu_threads = LuShape<T>::waves * 64;
template <typename T>
constexpr int lu_slots = kLuMaxNP / 16 / LuShape<T>::waves;   // row tiles per wave
constexpr int kLdb = 65;          // LDS leading dimension of 64-wide staging buffers

template <typename T>
struct V4;
template <>
struct V4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <>
struct V4<float> { typedef float type __attribute__((ext_vector_type(4))); };

// lane group and accumulator register holding row t (0..15) of a 16x16 tile
template <typename T>
__device__ inline int tile_row_group(int t);
template <>
__device__ inline int tile_row_group<double>(int t) { return t & 3; }
template <>
__device__ inline int tile_row_group<float>(int t) { return t >> 2; }
template <typename T>
__device__ inline int tile_row_reg(int t);
template <>
__device__ inline int tile_row_reg<double>(int t) { return t >> 2; }
template <>
__device__ inline int tile_row_reg<float>(int t) { return t & 3; }

// LDS layout of lu_factor_left (element type T for the staging region).
constexpr int kPanLd = 17;        // row stride of the 16-column sub-panel buffer
constexpr int kU12Ld = 49;        // row stride of the 16 x 48 sub-panel U block
constexpr int kCrowLd = 17;       // candidate pivot row: 16 entries and the pivot's reciprocal
template <typename T>
__host__ __device__ constexpr size_t lu2_work_elems(int NP) {
    return size_t(NP) * kPanLd + 16 * kU12Ld > 3 * size_t(kLuW) * kLdb + 1536
               ? size_t(NP) * kPanLd + 16 * kU12Ld
               : 3 * size_t(kLuW) * kLdb + 1536;
}
template <typename T>
__host__ __device__ constexpr size_t lu2_lds_bytes(int NP) {
    return 5 * size_t(NP) * sizeof(int32_t)                        // perm, sto, pos_log, log_pos, pidx
           + kLuW * sizeof(int32_t)                                // piv_pos
           + 2 * lu_waves<T> * (sizeof(double) + sizeof(int32_t))     // arg-max partials, double-buffered
           + 16 + 18 * sizeof(int32_t)                                // row flags; diagonal positions, flag
           + 2 * lu_waves<T> * kCrowLd * sizeof(T)                    // candidate pivot rows, double-buffered
           + 16 * kCrowLd * sizeof(T)                                 // factored diagonal block
           + lu2_work_elems<T>(NP) * sizeof(T) + 64;
}

// Orders one wave's LDS accesses before and after this point as written: the
// LDS executes a wave's instructions in issue order, so a value one lane
// writes is seen by every lane of the wave that reads it later; only the
// compiler must be kept from moving the accesses (no instruction is emitted).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Elements of the per-matrix inverse diagonal blocks.
template <typename T>
__host__ __device__ constexpr size_t lu2_dinv_elems(int NP) {
    return size_t((NP + kLuW - 1) / kLuW) * 2 * kLuW * kLuW;
}

// Inverses of the unit-lower and the upper triangle of the W x W diagonal block
// held in LDS (leading dimension kLdb), written to D[0] and D[1] (64 x 64
// row-major, global), block-recursively on 16 x 16 blocks: the diagonal
// blocks by substitution (the first half of the threads for inv(L), the second
// for inv(U), one lane per column), then the off-diagonal blocks level by
// level on the matrix cores, one wave per block,
// X_ij = -X_ii sum_k L_ik X_kj (lower) and Y_ij = -Y_ii sum_k U_ik Y_kj (upper).
// Xb, Yb: 64 x kLdb LDS outputs; Tb: 1536 elements of LDS scratch.  Every
// thread of the workgroup must call this (it contains barriers).
template <typename T>
__device__ __forceinline__ void diag_inverses(const T *Cb, int W, T *D, T *Xb, T *Yb, T *Tb) {
    constexpr int HALF = lu_threads<T> / 2;
    const int tid = threadIdx.x;
    const bool upper = tid >= HALF;
    const int h = tid % HALF;
    const int nb = W / 16;
    T *Z = upper ? Yb : Xb;
    T *Tz = Tb + (upper ? 768 : 0);
    // zero the outputs
    for (int e = h; e < 64 * 64; e += HALF) Z[(e >> 6) * kLdb + (e & 63)] = T(0);
    __syncthreads();
    // diagonal 16 x 16 blocks: one lane per column, the column's entries in
    // registers, by substitution (no barrier, no shuffle); lanes h < 64 of
    // each half, lane h holding column h of the 64 x 64 block
    if (h < 64) {
        const int b = h >> 4, kc = h & 15;
        if (b < nb) {
            const T *Bd = Cb + 16 * b * kLdb + 16 * b;     // the diagonal block, leading dimension kLdb
            double xs[16];
            if (!upper) {
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    double acc = 0.0;
#pragma unroll
                    for (int m = 0; m < t; ++m) {
                        const double p = double(Bd[t * kLdb + m]) * xs[m];
                        acc = m >= kc ? acc + p : acc;
                    }
                    xs[t] = t < kc ? 0.0 : (t == kc ? 1.0 : -acc);
                }
            } else {
#pragma unroll
                for (int t = 15; t >= 0; --t) {
                    double acc = 0.0;
#pragma unroll
                    for (int m = t + 1; m < 16; ++m) {
                        const double p = double(Bd[t * kLdb + m]) * xs[m];
                        acc = m <= kc ? acc + p : acc;
                    }
                    const double d = double(Bd[t * kLdb + t]);
                    xs[t] = t > kc ? 0.0 : (t == kc ? 1.0 / d : -acc / d);
                }
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) Z[(16 * b + t) * kLdb + 16 * b + kc] = T(xs[t]);
        }
    }
    __syncthreads();
    // off-diagonal blocks, by distance from the diagonal, one wave per block on
    // the matrix cores: the sum over the blocks between, then the product with
    // the diagonal block's inverse (lower X_ij = -X_ii sum_{k=j..i-1} L_ik X_kj,
    // upper Y_ij = -Y_ii sum_{k=i+1..j} U_ik Y_kj)
    {
        using Mt = Mfma<T>;
        using acc_t = typename Mt::acc_t;
        const int wave = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
        for (int d = 1; d < nb; ++d) {
            if (wave < 2 * (nb - d)) {
                const bool up = wave >= nb - d;
                const int bi = up ? wave - (nb - d) : wave;
                const int i = up ? bi : bi + d, jb = up ? bi + d : bi;
                const int k0 = up ? i + 1 : jb;
                T *Zt = up ? Yb : Xb;
                acc_t acc = acc_t{0, 0, 0, 0};
                for (int kb = 0; kb < d; ++kb) {
                    const int k = k0 + kb;
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        acc = Mt::mma(Cb[(16 * i + lr) * kLdb + 16 * k + 4 * st + lg],
                                      Zt[(16 * k + 4 * st + lg) * kLdb + 16 * jb + lr], acc);
                }
                acc_t acc2 = acc_t{0, 0, 0, 0};
                if constexpr (sizeof(T) == sizeof(double)) {
                    // the accumulator's register st holds rows 4 st + lane / 16:
                    // the B operand of step st as it stands
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        acc2 = Mt::mma(Zt[(16 * i + lr) * kLdb + 16 * i + 4 * st + lg], acc[st], acc2);
                } else {
                    T *Ts = Tb + 256 * wave;
#pragma unroll
                    for (int v = 0; v < 4; ++v) Ts[Mt::row(lane, v) * 16 + lr] = acc[v];
                    wave_lds_order();
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        acc2 = Mt::mma(Zt[(16 * i + lr) * kLdb + 16 * i + 4 * st + lg], Ts[(4 * st + lg) * 16 + lr],
                                       acc2);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) Zt[(16 * i + Mt::row(lane, v)) * kLdb + 16 * jb + lr] = -acc2[v];
            }
            __syncthreads();
        }
    }
    for (int e = h; e < 64 * 64; e += HALF) D[(upper ? kLuW * kLuW : 0) + e] = Z[(e >> 6) * kLdb + (e & 63)];
}

// The value v of lane src (a constant of the unrolled loops), on every lane.
__device__ __forceinline__ double lane_value(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Entries of the matrix to factor as stored in A (storage row, column).  A
// source yields an entry in two steps: row(r, c0), what the lanes of row r
// need for the 64 columns from c0 (a multiple of 64), and entry(that, r, col),
// so that the gather can issue every row's loads before the entry loads that
// depend on them.
template <typename T>
struct DenseSource {
    const T *A;
    int NP;
    struct Row { int32_t off; };
    __device__ __forceinline__ Row row(int r, int) const { return {r * NP}; }
    __device__ __forceinline__ T entry(const Row &w, int, int col) const { return A[w.off + col]; }
};

// Factors the matrix whose entries src yields (read once, when its block
// column is gathered) into A: A needs no initial contents.
template <typename T, typename Src>
__device__ __forceinline__ void lu_factor_left(T *__restrict__ A, int NP, int32_t *__restrict__ perm_out,
                                               T *__restrict__ dinv, int32_t *info, unsigned char *smem,
                                               const Src &src) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    using v4 = typename V4<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, lc = lane & 15;
    const int RT = NP / 16;
    const int NB = (NP + kLuW - 1) / kLuW;

    int32_t *perm = reinterpret_cast<int32_t *>(smem);    // logical row -> storage row
    int32_t *sto = perm + NP;                              // position -> storage row (this block column)
    int32_t *pos_log = sto + NP;                           // position -> logical row
    int32_t *log_pos = pos_log + NP;                       // logical row -> position
    int32_t *pidx = log_pos + NP;                          // position -> pivot column in this block, or -1
    int32_t *piv_pos = pidx + NP;                          // pivot column -> position
    double *redv = reinterpret_cast<double *>(piv_pos + kLuW);   // [2][waves]
    int32_t *redi = reinterpret_cast<int32_t *>(redv + 2 * lu_waves<T>);
    int32_t *rwave = redi + 2 * lu_waves<T>;                        // [2] wave holding logical row r;
                                                                 // [2] first zero pivot (1-based) or INT_MAX
    int32_t *dpos = rwave + 4;                                   // [16] positions of the diagonal pivot rows
    int32_t *spec_bad = dpos + 16;                               // [2] the diagonal pivots were refused
    T *crow = reinterpret_cast<T *>(dpos + 18);                  // [2][waves][kCrowLd] candidate rows
    T *Db = crow + 2 * lu_waves<T> * kCrowLd;                    // [16][kCrowLd] factored diagonal block
    T *work = Db + 16 * kCrowLd;
    T *Cb = work;                                          // [64][kLdb]   (left-looking, inverses)
    T *Ub = Cb + kLuW * kLdb;                              // [64][kLdb]
    T *Xb = Ub + kLuW * kLdb;                              // [64][kLdb]
    T *P = work;                                           // [NP][kPanLd] (panel)
    T *U12 = P + size_t(NP) * kPanLd;                      // [16][kU12Ld]

    for (int i = tid; i < NP; i += lu_threads<T>) perm[i] = i;
    if (tid < 16) dpos[tid] = 0;      // every position read from it stays in the panel
    if (tid == 0) rwave[2] = 0x7fffffff;
    __syncthreads();

    for (int j = 0; j < NB; ++j) {
        const int c0 = j * kLuW;
        const int Wj = min(kLuW, NP - c0);
        const int CTj = Wj / 16;
        for (int q = tid; q < NP; q += lu_threads<T>) {
            sto[q] = perm[q];
            pos_log[q] = q;
            log_pos[q] = q;
            pidx[q] = -1;
        }
        acc_t acc[lu_slots<T>][4];
        // 1. gather the block column (positions = logical rows at this point):
        //    what each of the lane's rows needs first, then every entry, so
        //    that each lane has all its row loads in flight together and then
        //    all its entry loads (the accumulators are not live yet).  Tiles
        //    outside the matrix read column c0 + lc of row 0 and are zeroed.
        {
            typename Src::Row rw[lu_slots<T>][4];
            int srow[lu_slots<T>][4];
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s) {
                const int rt = wave + lu_waves<T> * s;
#pragma unroll
                for (int v = 0; v < 4; ++v) srow[s][v] = rt < RT ? perm[16 * rt + M::row(lane, v)] : 0;
            }
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s)
#pragma unroll
                for (int v = 0; v < 4; ++v) rw[s][v] = src.row(srow[s][v], c0);
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s) {
                const int rt = wave + lu_waves<T> * s;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const T val = src.entry(rw[s][v], srow[s][v], c0 + 16 * (ct < CTj ? ct : 0) + lc);
                        acc[s][ct][v] = (rt < RT && ct < CTj) ? val : T(0);
                    }
            }
        }
        // 2. updates from the earlier block columns
        for (int i = 0; i < j; ++i) {
            const int r0 = i * kLuW;
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s) {
                const int rt = wave + lu_waves<T> * s;
                if (rt >= 4 * i && rt < 4 * i + 4) {
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        if (ct < CTj)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                Cb[(16 * (rt - 4 * i) + M::row(lane, v)) * kLdb + 16 * ct + lc] = acc[s][ct][v];
                }
            }
            __syncthreads();
            const T *Li = dinv + size_t(i) * 2 * kLuW * kLuW;   // inverse of the unit-lower block i
            {
                // the 16 tiles of U_ij = inv(L_ii) C_i, spread over all waves
                constexpr int TPW = 16 / lu_waves<T>;
                const int t0 = wave * TPW, tr = t0 >> 2;
                v4 a[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    a[kk] = *reinterpret_cast<const v4 *>(Li + (16 * tr + lc) * kLuW + 16 * kk + 4 * g);
#pragma unroll
                for (int k = 0; k < TPW; ++k) {
                    const int ct = (t0 + k) & 3;
                    if (ct < CTj) {
                        acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                u = M::mma(a[kk][e], Cb[(16 * kk + 4 * g + e) * kLdb + 16 * ct + lc], u);
#pragma unroll
                        for (int v = 0; v < 4; ++v) Ub[(16 * tr + M::row(lane, v)) * kLdb + 16 * ct + lc] = u[v];
                    }
                }
            }
            __syncthreads();
            // the rows of block i take their tiles of U_ij; the rows below are
            // updated C -= L_{:,i} U_ij
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s) {
                const int rt = wave + lu_waves<T> * s;
                if (rt >= 4 * i && rt < 4 * i + 4) {
                    const int tr = rt - 4 * i;
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        if (ct < CTj)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[s][ct][v] = Ub[(16 * tr + M::row(lane, v)) * kLdb + 16 * ct + lc];
                }
                if (rt >= 4 * (i + 1) && rt < RT) {
                    const T *Lrow = A + size_t(perm[16 * rt + lc]) * NP + r0;
                    v4 a[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) a[kk] = *reinterpret_cast<const v4 *>(Lrow + 16 * kk + 4 * g);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int ct = 0; ct < 4; ++ct)
                                if (ct < CTj)
                                    acc[s][ct] = M::mma(-a[kk][e], Ub[(16 * kk + 4 * g + e) * kLdb + 16 * ct + lc],
                                                        acc[s][ct]);
                }
            }
            __syncthreads();
        }
        // 3. panel factorisation, 16-column sub-panels.  Rows stay at their
        //    positions; pivoting assigns logical rows to positions.
#pragma unroll 1
        for (int sp = 0; sp < CTj; ++sp) {
            // (a) the sub-panel's column tile to LDS, one row per position (the
            //     accumulators keep it until (c), so it can be written again)
            auto panel_to_lds = [&]() {
#pragma unroll
                for (int s = 0; s < lu_slots<T>; ++s) {
                    const int rt = wave + lu_waves<T> * s;
                    if (rt >= 4 * j && rt < RT)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            T val = acc[s][0][v];
#pragma unroll
                            for (int ct = 1; ct < 4; ++ct)
                                if (ct == sp) val = acc[s][ct][v];
                            P[(16 * rt + M::row(lane, v)) * kPanLd + lc] = val;
                        }
                }
            };
            panel_to_lds();
            // (b) one thread per position factors the 16 columns.  Each
            //     thread knows the logical row of its position (mylog).
            const int q = tid;
            bool active = q >= c0 && q < NP && pidx[q] < 0;
            const bool participated = active;
            int mylog = active ? pos_log[q] : 0x7fffffff;
            // (b1) diagonal pivots: the rows of logical index rb .. rb + 15
            const int rb = c0 + 16 * sp;
            const bool is_diag = active && mylog >= rb && mylog < rb + 16;
            if (tid == 0) spec_bad[0] = 0;
            if (is_diag) dpos[mylog - rb] = q;
            __syncthreads();
            if (wave == 0) {
                // the 16 x 16 diagonal block in registers; column c: every entry
                // below row c takes its multiplier or its update from row c,
                // each lane reading what it needs from the lanes that hold it
                // before it changes its own; the factored block then goes to Db.
                // A pivot below the smallest normal number refuses the diagonal
                // (partial pivoting then forms such multipliers by division).
                bool bad = false;
                if constexpr (sizeof(T) == sizeof(float)) {
                    // FP32: lane i < 16 holds row i; the pivot and the rest of
                    // row c reach every lane by readlane
                    T a[16];
                    const bool row_lane = lane < 16;
#pragma unroll
                    for (int c = 0; c < 16; ++c) a[c] = P[dpos[row_lane ? lane : 0] * kPanLd + c];
                    T uii = T(1);
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const T piv = lane_value(a[c], c);
                        const bool normal = fabs(piv) >= std::numeric_limits<T>::min();
                        const T rinv = T(1) / (normal ? piv : T(1));
                        if (lane == c) uii = a[c];
                        const bool below = row_lane && lane > c;
                        const T l = a[c] * rinv;
                        bad |= !normal;
                        bad |= below && !(fabs(l) <= T(kPivotThreshold));
#pragma unroll
                        for (int j = c + 1; j < 16; ++j) {
                            const T ucj = lane_value(a[j], c);
                            if (below) a[j] = a[j] - l * ucj;
                        }
                        if (below) a[c] = l;
                    }
                    if (row_lane) {
#pragma unroll
                        for (int c = 0; c < 16; ++c) Db[lane * kCrowLd + c] = a[c];
                        Db[lane * kCrowLd + 16] = T(1) / uii;   // used only when every pivot is normal
                    }
                } else {
                    // FP64 (fewer registers): lane l holds the entries of rows
                    // i = 4 t + l / 16 (t = 0..3) in column j = l % 16, read by
                    // shuffles
                    const int jj = lane & 15, gg = lane >> 4;
                    T a[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) a[t] = P[dpos[4 * t + gg] * kPanLd + jj];
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const int tc = c >> 2, gc = c & 3;
                        const T piv = __shfl(a[tc], 16 * gc + c);
                        const bool normal = fabs(piv) >= std::numeric_limits<T>::min();
                        const T rinv = T(1) / (normal ? piv : T(1));
                        const T ucj = __shfl(a[tc], 16 * gc + jj);
                        T l[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) l[t] = __shfl(a[t], 16 * gg + c) * rinv;
                        bad |= !normal;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int i = 4 * t + gg;
                            if (i > c) {
                                if (jj == c) {
                                    bad |= !(fabs(l[t]) <= T(kPivotThreshold));
                                    a[t] = l[t];
                                } else if (jj > c) {
                                    a[t] = a[t] - l[t] * ucj;
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) Db[(4 * t + gg) * kCrowLd + jj] = a[t];
                    wave_lds_order();
                    if (lane < 16) Db[lane * kCrowLd + 16] = T(1) / Db[lane * kCrowLd + lane];   // used only when every pivot is normal
                }
                if (__ballot(bad) != 0 && lane == 0) spec_bad[0] = 1;
            }
            __syncthreads();
            // (b2) every other unpivoted row against the diagonal block's U
            //      rows (the elimination of the partial-pivoting loop below
            //      with its pivots fixed, so no exchange between waves), the
            //      result written over the row in LDS; the diagonal rows take
            //      their factored entries
            {
                bool bad = false;
                if (active && !is_diag) {
                    T x[16];
#pragma unroll
                    for (int c = 0; c < 16; ++c) x[c] = P[q * kPanLd + c];
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const T *urow = Db + c * kCrowLd;
                        const T l = x[c] * urow[16];
                        bad |= !(fabs(l) <= T(kPivotThreshold));
                        x[c] = l;
#pragma unroll
                        for (int cb = c + 1; cb < 16; cb += 4) {
                            T uv[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (cb + u < 16) uv[u] = urow[cb + u];
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (cb + u < 16) x[cb + u] -= l * uv[u];
                        }
                        // the U rows are the same for every row: keep the
                        // scheduler from hoisting all their loads at once
                        __builtin_amdgcn_sched_barrier(0);
                    }
#pragma unroll
                    for (int c = 0; c < 16; ++c) P[q * kPanLd + c] = x[c];
                } else if (is_diag) {
                    const int k = mylog - rb;
#pragma unroll
                    for (int c = 0; c < 16; ++c) P[q * kPanLd + c] = Db[k * kCrowLd + c];
                }
                if (__ballot(bad) != 0 && lane == 0) spec_bad[0] = 1;
            }
            __syncthreads();
            if (spec_bad[0] == 0) {
                // accepted: the diagonal rows are the pivots, labels unchanged
                if (is_diag) {
                    pidx[q] = 16 * sp + (mylog - rb);
                    piv_pos[16 * sp + (mylog - rb)] = q;
                }
                __syncthreads();
            } else {
            // (b3) refused: the sub-panel again from the accumulators, with
            //      partial pivoting.  The winner of the pivot search among a
            //      wave's lanes publishes its row, so one barrier per column
            //      suffices.  A wave without unpivoted rows only takes part in
            //      the barriers.
            panel_to_lds();
            __syncthreads();
            const bool busy = __ballot(active) != 0;
            if (!busy && lane == 0) {
                redv[wave] = -1.0;
                redv[lu_waves<T> + wave] = -1.0;
            }
            T x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = active ? P[q * kPanLd + c] : T(0);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int gc = 16 * sp + c;
                const int r = c0 + gc;
                const int buf = c & 1;
                if (busy) {
                    const double ax = fabs(double(x[c]));
                    double bv = (active && ax == ax) ? ax : -1.0;   // NaN never wins
                    int bl = mylog;
                    wave_argmax_ballot(bv, bl);
                    if (lane == 0) { redv[buf * lu_waves<T> + wave] = bv; redi[buf * lu_waves<T> + wave] = bl; }
                    if (active && mylog == r) rwave[buf] = wave;
                    // the wave's candidate row (or row r, kept when nothing is
                    // finite) with the reciprocal of its entry in column c, or 0
                    // where that is below the smallest normal number (then the
                    // multipliers are formed by division, as LAPACK does)
                    if (active && mylog == (bv < 0.0 ? r : bl)) {
                        T *cr = crow + (buf * lu_waves<T> + wave) * kCrowLd;
#pragma unroll
                        for (int cc = c; cc < 16; ++cc) cr[cc] = x[cc];
                        cr[16] = fabs(x[c]) >= std::numeric_limits<T>::min() ? T(1) / x[c] : T(0);
                    }
                }
                __syncthreads();
                if (!busy) continue;
                // cross-wave arg-max: lane w < 8 holds wave w's partial; ties go
                // to the smaller logical row
                int lp, wv;
                {
                    const double fv = lane < lu_waves<T> ? redv[buf * lu_waves<T> + lane] : -2.0;
                    const int fi = lane < lu_waves<T> ? redi[buf * lu_waves<T> + lane] : 0x7fffffff;
                    double m = dpp_max_step<0xB1, 0xf>(fv);    // quad_perm [1,0,3,2]
                    m = dpp_max_step<0x4E, 0xf>(m);            // quad_perm [2,3,0,1]
                    m = dpp_max_step<0x141, 0xf>(m);           // row_half_mirror: lanes 0..7 hold their max
                    if (lu_waves<T> > 8) m = dpp_max_step<0x140, 0xf>(m);   // row_mirror: lanes 0..15
                    {
                        const int lo = __builtin_amdgcn_readlane(__double2loint(m), 0);
                        const int hi = __builtin_amdgcn_readlane(__double2hiint(m), 0);
                        m = __hiloint2double(hi, lo);
                    }
                    if (m < 0.0) {          // no finite candidate: keep logical row r
                        lp = r;
                        wv = rwave[buf];
                    } else {
                        const unsigned long long hit = __ballot(lane < lu_waves<T> && fv == m);
                        if (__popcll(hit) == 1) {
                            wv = __ffsll(static_cast<unsigned long long>(hit)) - 1;
                            lp = __builtin_amdgcn_readlane(fi, wv);
                        } else {
                            double tv = (lane < lu_waves<T> && fv == m) ? 1.0 : -1.0;
                            int tk = (lane < lu_waves<T> && fv == m) ? (fi << LuShape<T>::wave_bits) + lane : 0x7fffffff;
                            wave_argmax(tv, tk);
                            lp = tk >> LuShape<T>::wave_bits;
                            wv = tk & (lu_waves<T> - 1);
                        }
                    }
                }
                const T *urow = crow + (buf * lu_waves<T> + wv) * kCrowLd;
                const T piv = urow[c];
                const T rinv = urow[16];
                if (lane == 0 && piv == T(0)) atomicMin(&rwave[2], r + 1);
                if (active) {
                    if (mylog == lp) {               // this position becomes logical row r
                        mylog = r;
                        active = false;
                        pidx[q] = gc;
                        piv_pos[gc] = q;
                    } else {
                        if (mylog == r) mylog = lp;  // row r moves to the pivot's old logical index
                        T l;
                        if (rinv != T(0))
                            l = x[c] * rinv;
                        else
                            l = piv != T(0) ? x[c] / piv : x[c];
                        x[c] = l;
                        // the pivot row in groups of four entries, each group's
                        // loads issued together before its updates
#pragma unroll
                        for (int cb = c + 1; cb < 16; cb += 4) {
                            T uv[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (cb + u < 16) uv[u] = urow[cb + u];
                            __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);   // the group's LDS reads
                            __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);   // then VALU
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (cb + u < 16) x[cb + u] -= l * uv[u];
                        }
                    }
                }
            }
            if (participated) {
#pragma unroll
                for (int c = 0; c < 16; ++c) P[q * kPanLd + c] = x[c];
                pos_log[q] = mylog;
            }
            __syncthreads();
            }   // partial pivoting
            // (c) back to the accumulators
#pragma unroll
            for (int s = 0; s < lu_slots<T>; ++s) {
                const int rt = wave + lu_waves<T> * s;
                if (rt >= 4 * j && rt < RT)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const T val = P[(16 * rt + M::row(lane, v)) * kPanLd + lc];
#pragma unroll
                        for (int ct = 0; ct < 4; ++ct)
                            if (ct == sp) acc[s][ct][v] = val;
                    }
            }
            // (d) the remaining column tiles of the block: U12 of this
            //     sub-panel's pivot rows, then the update of unused rows
            if (sp + 1 < CTj) {
                const int nct = CTj - sp - 1;
#pragma unroll
                for (int s = 0; s < lu_slots<T>; ++s) {
                    const int rt = wave + lu_waves<T> * s;
                    if (rt >= 4 * j && rt < RT)
#pragma unroll
                        for (int ct = 1; ct < 4; ++ct)
                            if (ct > sp && ct < CTj)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int pi = pidx[16 * rt + M::row(lane, v)] - 16 * sp;
                                    if (pi >= 0 && pi < 16)
                                        U12[pi * kU12Ld + 16 * (ct - sp - 1) + lc] = acc[s][ct][v];
                                }
                }
                __syncthreads();
                if (tid < 16 * nct) {
                    T u[16];
#pragma unroll
                    for (int i2 = 0; i2 < 16; ++i2) u[i2] = U12[i2 * kU12Ld + tid];
#pragma unroll
                    for (int i2 = 1; i2 < 16; ++i2) {
                        const T *Lr = P + piv_pos[16 * sp + i2] * kPanLd;
#pragma unroll
                        for (int m = 0; m < i2; ++m) u[i2] -= Lr[m] * u[m];
                    }
#pragma unroll
                    for (int i2 = 0; i2 < 16; ++i2) U12[i2 * kU12Ld + tid] = u[i2];
                }
                __syncthreads();
#pragma unroll
                for (int s = 0; s < lu_slots<T>; ++s) {
                    const int rt = wave + lu_waves<T> * s;
                    if (rt >= 4 * j && rt < RT) {
                        const bool unused = pidx[16 * rt + lc] < 0;
                        T a[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) a[e] = unused ? -P[(16 * rt + lc) * kPanLd + 4 * e + g] : T(0);
#pragma unroll
                        for (int ct = 1; ct < 4; ++ct) {
                            if (ct > sp && ct < CTj) {
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    acc[s][ct] = M::mma(a[e], U12[(4 * e + g) * kU12Ld + 16 * (ct - sp - 1) + lc],
                                                        acc[s][ct]);
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int pi = pidx[16 * rt + M::row(lane, v)] - 16 * sp;
                                    if (pi >= 0 && pi < 16) acc[s][ct][v] = U12[pi * kU12Ld + 16 * (ct - sp - 1) + lc];
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        // the last sub-panel's rows are read back from P before the staging
        // buffer below (which shares P's memory) is written
        __syncthreads();
        for (int q2 = tid; q2 < NP; q2 += lu_threads<T>)
            if (q2 >= c0) perm[pos_log[q2]] = sto[q2];
        // 4. diagonal block (logical rows c0 .. c0 + Wj - 1) to LDS, its
        //    triangles' inverses, and the block column back to its storage rows
#pragma unroll
        for (int s = 0; s < lu_slots<T>; ++s) {
            const int rt = wave + lu_waves<T> * s;
            if (rt >= 4 * j && rt < RT)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    if (ct < CTj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int lr = pos_log[16 * rt + M::row(lane, v)] - c0;
                            if (lr >= 0 && lr < Wj) Cb[lr * kLdb + 16 * ct + lc] = acc[s][ct][v];
                        }
        }
        // the block column goes back first, so that the accumulators are free
        // while the inverses are formed
#pragma unroll
        for (int s = 0; s < lu_slots<T>; ++s) {
            const int rt = wave + lu_waves<T> * s;
            if (rt < RT)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    if (ct < CTj)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            A[size_t(sto[16 * rt + M::row(lane, v)]) * NP + c0 + 16 * ct + lc] = acc[s][ct][v];
        }
        __syncthreads();
        diag_inverses<T>(Cb, Wj, dinv + size_t(j) * 2 * kLuW * kLuW, Xb, Ub, Xb + kLuW * kLdb);
        __syncthreads();
    }
    for (int i = tid; i < NP; i += lu_threads<T>) perm_out[i] = perm[i];
    if (tid == 0 && info) *info = rwave[2] == 0x7fffffff ? 0 : rwave[2];
}

// Solves (P^T L U) z = b for one matrix factored by lu_factor_left, with the
// kBlock threads of a per-cell workgroup.  Row r of the factors is storage row
// rowmap[r] (identity if rowmap is null); y starts as b[bperm[.]] (both are
// perm in the solver).  b[NP] (LDS, FP64) is read, the
// solution is left in y[NP] (LDS); t is 64 doubles of LDS scratch.  Factor
// entries are widened to FP64; the arithmetic is FP64.
// N (even, N <= NP) is the order of the padded matrix: its rows and columns
// from N on are the identity's, in the matrix and so in its factors (no
// pivot is taken from them before column N), and b is zero there; the
// products then stop at N and y keeps its zeros past N.  N = NP for factors
// of unknown padding.
template <typename T>
__device__ __forceinline__ void lu_solve_left(const T *__restrict__ A, const T *__restrict__ dinv, const int32_t *__restrict__ rowmap,
                              const int32_t *__restrict__ bperm, int NP, int N, const double *b, double *y, double *t) {
    const int tid = threadIdx.x;
    const int lane16 = tid & 15, row16 = tid >> 4;   // 16 lanes per row, 16 rows per pass
    constexpr int VW = 16 / int(sizeof(T));           // factor entries per 16-byte load
    for (int i = tid; i < NP; i += kBlock) y[i] = b[bperm[i]];
    __syncthreads();
    const int NB = (N + kLuW - 1) / kLuW;
    // t[rr] = y[r0 + rr] - A_row(r0 + rr)[c_begin, c_end) . vec for rr < W (rows through
    // rowmap); 16 lanes per row, each thread carries 4 rows so that four
    // 16-byte loads are in flight per step.
    auto gemv_off = [&](int r0, int W, int c_begin, int c_end, const double *vec) {
        // rows past W (last block) read row W - 1 again; their sums are not stored.
        // No load sits behind a condition, so all of them are in flight together.
        const T *rows[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int rr = min(row16 + 16 * p, W - 1);
            rows[p] = A + size_t(rowmap ? rowmap[r0 + rr] : r0 + rr) * NP;
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        // VW entries (16 bytes) per lane and load: c_begin is a multiple of 64
        // and rows are 64-byte aligned.  FP32 entries past c_end (at most
        // three, within the row) meet zeros of vec.
        for (int c = c_begin + VW * lane16; c < c_end; c += 16 * VW) {
            double yv[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) yv[k] = vec[c + k];
            T a[4][VW];
#pragma unroll
            for (int p = 0; p < 4; ++p) __builtin_memcpy(a[p], __builtin_assume_aligned(rows[p] + c, 16), 16);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if constexpr (VW == 2)
                    acc[p] += double(a[p][0]) * yv[0] + double(a[p][1]) * yv[1];
                else
                    acc[p] += (double(a[p][0]) * yv[0] + double(a[p][1]) * yv[1]) +
                              (double(a[p][2]) * yv[2] + double(a[p][3]) * yv[3]);
            }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double a = acc[p];
            for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o);
            const int rr = row16 + 16 * p;
            if (lane16 == 0 && rr < W) t[rr] = y[r0 + rr] - a;
        }
    };
    // D is the 64 x 64 inverse of the block's unit lower (lower) or upper
    // triangle.  Its other triangle is zero and is not read: a column on that
    // side of the diagonal loads the diagonal entry instead (a cache line the
    // row needs anyway) and contributes nothing.  Rows past W read row W - 1
    // again and are not stored.
    auto gemv_diag = [&](int r0, int W, const T *D, bool lower) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = VW * lane16; c < W; c += 16 * VW) {
            double tv[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) tv[k] = c + k < W ? t[c + k] : 0.0;
            // the 16 bytes holding the diagonal stand in for those on the zero side
            T a[4][VW];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int rr = min(row16 + 16 * p, W - 1), dq = rr & ~(VW - 1);
                __builtin_memcpy(a[p], __builtin_assume_aligned(D + rr * kLuW + (lower ? min(c, dq) : max(c, dq)), 16),
                                 16);
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int rr = min(row16 + 16 * p, W - 1);
                double term[VW];
#pragma unroll
                for (int k = 0; k < VW; ++k) {
                    const bool use = c + k < W && (lower ? c + k <= rr : c + k >= rr);
                    term[k] = use ? double(a[p][k]) * tv[k] : 0.0;
                }
                if constexpr (VW == 2)
                    acc[p] += term[0] + term[1];
                else
                    acc[p] += (term[0] + term[1]) + (term[2] + term[3]);
            }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double a = acc[p];
            for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o);
            const int rr = row16 + 16 * p;
            if (lane16 == 0 && rr < W) y[r0 + rr] = a;
        }
    };
    for (int ib = 0; ib < NB; ++ib) {
        const int r0 = ib * kLuW, W = min(kLuW, N - r0);
        gemv_off(r0, W, 0, r0, y);
        __syncthreads();
        gemv_diag(r0, W, dinv + size_t(ib) * 2 * kLuW * kLuW, true);
        __syncthreads();
    }
    for (int ib = NB - 1; ib >= 0; --ib) {
        const int r0 = ib * kLuW, W = min(kLuW, N - r0);
        gemv_off(r0, W, r0 + W, N, y);
        __syncthreads();
        gemv_diag(r0, W, dinv + size_t(ib) * 2 * kLuW * kLuW + kLuW * kLuW, false);
        __syncthreads();
    }
}


// Solves M^T z = b from the factors of P M = L U (M^T = U^T L^T P): forward
// substitution with U^T, back substitution with L^T, then z[rowmap[i]] = v[i].
// The off-diagonal blocks enter as column products (lane i & 63 owns column
// i of the current 64-column block, the four waves split the rows, so each
// wave reads 64 consecutive entries of a row); the diagonal blocks are solved
// by substitution (one wave, column by column, the block staged in LDS)
// rather than by their stored inverses: the reverse sweep of the BDF map
// amplifies solve errors strongly, and substitution keeps them at the level
// of a backward-stable solver.  b, z, t (>= 5 * kLuW doubles) and Db
// (kLuW * kLdb doubles) are in LDS; b is consumed.  256 threads.
template <typename T>
__device__ __forceinline__ void lu_solve_left_T(const T *__restrict__ A, const int32_t *__restrict__ rowmap, int NP,
                                                double *b, double *z, double *t, double *Db) {
    const int tid = threadIdx.x;
    const int col = tid & 63, grp = tid >> 6;
    const int NB = (NP + kLuW - 1) / kLuW;
    // t[col] = b[r0 + col] - sum_{r in [rb, re)} A_logical[r][r0 + col] vec[r]
    auto colgemv = [&](int r0, int W, int rb, int re, const double *vec) {
        double acc = 0.0;
        if (col < W) {
            int r = rb + grp;
            for (; r + 12 < re; r += 16) {
                const double a0 = double(A[size_t(rowmap[r]) * NP + r0 + col]);
                const double a1 = double(A[size_t(rowmap[r + 4]) * NP + r0 + col]);
                const double a2 = double(A[size_t(rowmap[r + 8]) * NP + r0 + col]);
                const double a3 = double(A[size_t(rowmap[r + 12]) * NP + r0 + col]);
                acc += a0 * vec[r] + a1 * vec[r + 4] + a2 * vec[r + 8] + a3 * vec[r + 12];
            }
            for (; r < re; r += 4) acc += double(A[size_t(rowmap[r]) * NP + r0 + col]) * vec[r];
        }
        t[kLuW + grp * kLuW + col] = acc;
        __syncthreads();
        if (tid < W) t[tid] = b[r0 + tid] - ((t[kLuW + tid] + t[2 * kLuW + tid]) + (t[3 * kLuW + tid] + t[4 * kLuW + tid]));
        __syncthreads();
    };
    // the W x W diagonal block of logical rows r0.. into Db (row-major, ld kLdb)
    auto stage = [&](int r0, int W) {
        for (int e = tid; e < W * kLuW; e += blockDim.x) {
            const int rr = e >> 6, cc = e & 63;
            if (cc < W) Db[rr * kLdb + cc] = double(A[size_t(rowmap[r0 + rr]) * NP + r0 + cc]);
        }
        __syncthreads();
    };
    auto bcast = [](double v, int k) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
        return __hiloint2double(hi, lo);
    };
    // U^T w = b: w_k = t_k / U_kk, then t_i -= U_ki w_k for i > k  (w kept in b)
    for (int ib = 0; ib < NB; ++ib) {
        const int r0 = ib * kLuW, W = min(kLuW, NP - r0);
        colgemv(r0, W, 0, r0, b);
        stage(r0, W);
        if (tid < 64) {
            double tv = col < W ? t[col] : 0.0;
            for (int k = 0; k < W; ++k) {
                const double wk = bcast(tv, k) / Db[k * kLdb + k];
                if (col == k) tv = wk;
                else if (col > k && col < W) tv -= Db[k * kLdb + col] * wk;
            }
            if (col < W) b[r0 + col] = tv;
        }
        __syncthreads();
    }
    // L^T v = w (unit diagonal): v_k = t_k, then t_i -= L_ki v_k for i < k  (v kept in b)
    for (int ib = NB - 1; ib >= 0; --ib) {
        const int r0 = ib * kLuW, W = min(kLuW, NP - r0);
        colgemv(r0, W, r0 + W, NP, b);
        stage(r0, W);
        if (tid < 64) {
            double tv = col < W ? t[col] : 0.0;
            for (int k = W - 1; k > 0; --k) {
                const double vk = bcast(tv, k);
                if (col < k) tv -= Db[k * kLdb + col] * vk;
            }
            if (col < W) b[r0 + col] = tv;
        }
        __syncthreads();
    }
    for (int i = tid; i < NP; i += blockDim.x) z[rowmap[i]] = b[i];
    __syncthreads();
}

}  // namespace abdf
