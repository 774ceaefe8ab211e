// Left-looking blocked LU with partial pivoting, one 1024-thread workgroup per
// matrix, and the matching triangular solves.
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
//     registers: 16 waves, wave w owns row tiles w and w + 16, all 4 column
//     tiles of 16;
//  2. for every earlier block i: U_ij = inv(L_ii) C_i (rows 64i..64i+63 of the
//     block column, staged through LDS), then the rows below block i are
//     updated C -= L_{:,i} U_ij on the matrix cores, L read from memory;
//  3. the panel (rows >= 64j) is factored in registers, one column at a time:
//     arg-max pivot search (ties to the smaller row, as LAPACK), row exchange
//     through LDS, scaling, rank-1 update;
//  4. the inverses of the diagonal block's triangles are formed and stored,
//     and the block column is written back through perm.
#pragma once

#include "device_common.hpp"
#include "device_lu.hpp"

namespace abdf {

constexpr int kLuWaves = 16;
constexpr int kLuThreads = kLuWaves * 64;
constexpr int kLuW = 64;          // block-column width
constexpr int kLuMaxNP = 512;     // two row tiles per wave
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

template <typename T>
__host__ __device__ constexpr size_t lu2_lds_bytes(int NP) {
    return size_t(NP) * sizeof(int32_t)                   // perm
           + kLuWaves * (sizeof(double) + sizeof(int32_t)) // arg-max partials
           + 2 * 2 * kLuW * sizeof(T)                     // pivot row / displaced row, double-buffered
           + 3 * size_t(kLuW) * kLdb * sizeof(T) + 64;    // C_i, U_ij and inverse staging
}

// Bytes of the per-matrix inverse diagonal blocks.
template <typename T>
__host__ __device__ constexpr size_t lu2_dinv_elems(int NP) {
    return size_t((NP + kLuW - 1) / kLuW) * 2 * kLuW * kLuW;
}

// Inverses of the unit-lower and the upper triangle of the W x W diagonal block
// held in LDS (leading dimension kLdb), written to D[0] and D[1] (64 x 64
// row-major, global).  Wave 0 forms inv(L) by columns, wave 1 inv(U); Xb and
// Yb are LDS scratch of 64 x kLdb.
template <typename T>
__device__ __forceinline__ void diag_inverses(const T *Cb, int W, T *D, T *Xb, T *Yb, int wave, int lane) {
    if (wave == 0 && lane < W) {
        const int k = lane;
        for (int i = 0; i < W; ++i) {
            double acc2 = 0.0;
            for (int m = 0; m < i; ++m)
                if (m >= k) acc2 += double(Cb[i * kLdb + m]) * double(Xb[m * kLdb + k]);
            const double xv = i < k ? 0.0 : (i == k ? 1.0 : -acc2);
            Xb[i * kLdb + k] = T(xv);
            D[i * kLuW + k] = T(xv);
        }
    } else if (wave == 1 && lane < W) {
        const int k = lane;
        for (int i = W - 1; i >= 0; --i) {
            double acc2 = 0.0;
            for (int m = i + 1; m < W; ++m)
                if (m <= k) acc2 += double(Cb[i * kLdb + m]) * double(Yb[m * kLdb + k]);
            const double d = double(Cb[i * kLdb + i]);
            const double yv = i > k ? 0.0 : (i == k ? 1.0 / d : -acc2 / d);
            Yb[i * kLdb + k] = T(yv);
            D[kLuW * kLuW + i * kLuW + k] = T(yv);
        }
    }
}

template <typename T>
__device__ __forceinline__ void lu_factor_left(T *__restrict__ A, int NP, int32_t *__restrict__ perm_out, T *__restrict__ dinv,
                               int32_t *info, unsigned char *smem) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    using v4 = typename V4<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, lc = lane & 15;
    const int RT = NP / 16;
    const int NB = (NP + kLuW - 1) / kLuW;

    int32_t *perm = reinterpret_cast<int32_t *>(smem);
    double *redv = reinterpret_cast<double *>(perm + NP + (NP & 1));
    int32_t *redi = reinterpret_cast<int32_t *>(redv + kLuWaves);
    T *rowb = reinterpret_cast<T *>(redi + kLuWaves);           // [2 buffers][2 rows][64]
    T *Cb = rowb + 2 * 2 * kLuW;                                  // [64][kLdb]
    T *Ub = Cb + kLuW * kLdb;                                     // [64][kLdb]
    T *Xb = Ub + kLuW * kLdb;                                     // [64][kLdb] inverse output

    for (int i = tid; i < NP; i += kLuThreads) perm[i] = i;
    int first_zero = 0;
    __syncthreads();

    for (int j = 0; j < NB; ++j) {
        const int c0 = j * kLuW;
        const int Wj = min(kLuW, NP - c0);
        const int CTj = Wj / 16;
        acc_t acc[2][4];
        // 1. gather the block column
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int rt = wave + 16 * s;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T val = T(0);
                    if (rt < RT && ct < CTj) {
                        const int row = 16 * rt + M::row(lane, v);
                        val = A[size_t(perm[row]) * NP + c0 + 16 * ct + lc];
                    }
                    acc[s][ct][v] = val;
                }
            }
        }
        // 2. updates from the earlier block columns
        for (int i = 0; i < j; ++i) {
            const int r0 = i * kLuW;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
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
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
                if (rt >= 4 * i && rt < 4 * i + 4) {
                    const int tr = rt - 4 * i;
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct) {
                        if (ct < CTj) {
                            acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk) {
                                const v4 a =
                                    *reinterpret_cast<const v4 *>(Li + (16 * tr + lc) * kLuW + 16 * kk + 4 * g);
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    u = M::mma(a[e], Cb[(16 * kk + 4 * g + e) * kLdb + 16 * ct + lc], u);
                            }
                            acc[s][ct] = u;
#pragma unroll
                            for (int v = 0; v < 4; ++v) Ub[(16 * tr + M::row(lane, v)) * kLdb + 16 * ct + lc] = u[v];
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
                if (rt >= 4 * (i + 1) && rt < RT) {
                    const T *Lrow = A + size_t(perm[16 * rt + lc]) * NP + r0;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const v4 a = *reinterpret_cast<const v4 *>(Lrow + 16 * kk + 4 * g);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int ct = 0; ct < 4; ++ct)
                                if (ct < CTj)
                                    acc[s][ct] = M::mma(-a[e], Ub[(16 * kk + 4 * g + e) * kLdb + 16 * ct + lc],
                                                        acc[s][ct]);
                    }
                }
            }
            __syncthreads();
        }
        // 3. panel factorisation in registers
        for (int c = 0; c < Wj; ++c) {
            const int r = c0 + c;
            const int ctc = c >> 4;
            const int buf = c & 1;
            double bv = -1.0;
            int bi = 0x7fffffff;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
                if (rt < RT && lc == (c & 15)) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * rt + M::row(lane, v);
                        T x = T(0);
#pragma unroll
                        for (int ct = 0; ct < 4; ++ct)
                            if (ct == ctc) x = acc[s][ct][v];
                        const double a = fabs(double(x));
                        if (row >= r && a > bv) { bv = a; bi = row; }
                    }
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { redv[wave] = bv; redi[wave] = bi; }
            __syncthreads();
            double fv = redv[0];
            int p = redi[0];
            for (int w = 1; w < kLuWaves; ++w)
                if (redv[w] > fv || (redv[w] == fv && redi[w] < p)) { fv = redv[w]; p = redi[w]; }
            if (fv < 0.0) p = r;   // no finite candidate: keep the row
            T *urow = rowb + buf * 2 * kLuW;
            T *rrow = urow + kLuW;
            // the pivot row and (if it moves) row r, to LDS
            const int tp = p & 15, tr_ = r & 15;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
                if (rt == (p >> 4) && g == tile_row_group<T>(tp)) {
                    const int vr = tile_row_reg<T>(tp);
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        if (ct < CTj) {
                            T x = T(0);
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                if (v == vr) x = acc[s][ct][v];
                            urow[16 * ct + lc] = x;
                        }
                }
                if (p != r && rt == (r >> 4) && g == tile_row_group<T>(tr_)) {
                    const int vr = tile_row_reg<T>(tr_);
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        if (ct < CTj) {
                            T x = T(0);
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                if (v == vr) x = acc[s][ct][v];
                            rrow[16 * ct + lc] = x;
                        }
                }
            }
            __syncthreads();
            if (tid == 0 && p != r) {
                const int t = perm[r];
                perm[r] = perm[p];
                perm[p] = t;
            }
            const T piv = urow[c];
            if (tid == 0 && piv == T(0) && first_zero == 0) first_zero = r + 1;
            T u[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) u[ct] = ct < CTj ? urow[16 * ct + lc] : T(0);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int rt = wave + 16 * s;
                if (rt < RT && 16 * rt + 15 >= r) {
                    // exchange of rows r and p
                    if (p != r) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * rt + M::row(lane, v);
                            if (row == r || row == p) {
#pragma unroll
                                for (int ct = 0; ct < 4; ++ct)
                                    if (ct < CTj) acc[s][ct][v] = row == r ? u[ct] : rrow[16 * ct + lc];
                            }
                        }
                    }
                    // multipliers of column c and the rank-1 update of the rows below r
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        T x = T(0);
#pragma unroll
                        for (int ct = 0; ct < 4; ++ct)
                            if (ct == ctc) x = acc[s][ct][v];
                        x = __shfl(x, (lane & 48) | (c & 15));
                        const int row = 16 * rt + M::row(lane, v);
                        if (row > r) {
                            const T l = piv != T(0) ? x / piv : x;
#pragma unroll
                            for (int ct = 0; ct < 4; ++ct) {
                                const int col = 16 * ct + lc;
                                if (ct < CTj) {
                                    if (col == c) acc[s][ct][v] = l;
                                    else if (col > c) acc[s][ct][v] -= l * u[ct];
                                }
                            }
                        }
                    }
                }
            }
        }
        // 4. diagonal-block inverses and write-back
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int rt = wave + 16 * s;
            if (rt >= 4 * j && rt < 4 * j + CTj) {
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    if (ct < CTj)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            Cb[(16 * (rt - 4 * j) + M::row(lane, v)) * kLdb + 16 * ct + lc] = acc[s][ct][v];
            }
        }
        __syncthreads();
        diag_inverses<T>(Cb, Wj, dinv + size_t(j) * 2 * kLuW * kLuW, Xb, Ub, wave, lane);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int rt = wave + 16 * s;
            if (rt < RT) {
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    if (ct < CTj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * rt + M::row(lane, v);
                            A[size_t(perm[row]) * NP + c0 + 16 * ct + lc] = acc[s][ct][v];
                        }
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < NP; i += kLuThreads) perm_out[i] = perm[i];
    if (tid == 0 && info) *info = first_zero;
}

// Solves (P^T L U) z = b for one matrix factored by lu_factor_left, with the
// kBlock threads of a per-cell workgroup.  Row r of the factors is storage row
// rowmap[r] (identity if rowmap is null); y starts as b[bperm[.]] (both are
// perm in the solver).  b[NP] (LDS, FP64) is read, the
// solution is left in y[NP] (LDS); t is 64 doubles of LDS scratch.  Factor
// entries are widened to FP64; the arithmetic is FP64.
template <typename T>
__device__ __forceinline__ void lu_solve_left(const T *__restrict__ A, const T *__restrict__ dinv, const int32_t *__restrict__ rowmap,
                              const int32_t *__restrict__ bperm, int NP, const double *b, double *y, double *t) {
    const int tid = threadIdx.x;
    const int lane16 = tid & 15, row16 = tid >> 4;   // 16 lanes per row, 16 rows per pass
    for (int i = tid; i < NP; i += kBlock) y[i] = b[bperm[i]];
    __syncthreads();
    const int NB = (NP + kLuW - 1) / kLuW;
    // y_rows -= A_rows[c_begin, c_end) . vec (rows through perm), result to t[0..W)
    auto gemv_off = [&](int r0, int W, int c_begin, int c_end, const double *vec) {
        for (int rr = row16; rr < W; rr += 16) {
            const T *row = A + size_t(rowmap ? rowmap[r0 + rr] : r0 + rr) * NP;
            double acc = 0.0;
            for (int c = c_begin + 2 * lane16; c < c_end; c += 32)
                acc += double(row[c]) * vec[c] + double(row[c + 1]) * vec[c + 1];
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (lane16 == 0) t[rr] = y[r0 + rr] - acc;
        }
    };
    auto gemv_diag = [&](int r0, int W, const T *D) {
        for (int rr = row16; rr < W; rr += 16) {
            const T *row = D + rr * kLuW;
            double acc = 0.0;
            for (int c = 2 * lane16; c < W; c += 32) acc += double(row[c]) * t[c] + double(row[c + 1]) * t[c + 1];
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (lane16 == 0) y[r0 + rr] = acc;
        }
    };
    for (int ib = 0; ib < NB; ++ib) {
        const int r0 = ib * kLuW, W = min(kLuW, NP - r0);
        gemv_off(r0, W, 0, r0, y);
        __syncthreads();
        gemv_diag(r0, W, dinv + size_t(ib) * 2 * kLuW * kLuW);
        __syncthreads();
    }
    for (int ib = NB - 1; ib >= 0; --ib) {
        const int r0 = ib * kLuW, W = min(kLuW, NP - r0);
        gemv_off(r0, W, r0 + W, NP, y);
        __syncthreads();
        gemv_diag(r0, W, dinv + size_t(ib) * 2 * kLuW * kLuW + kLuW * kLuW);
        __syncthreads();
    }
}

}  // namespace abdf
