// Dense LU with partial pivoting of one NP x NP row-major matrix per
// workgroup, and the matching triangular solves.
//
// Factorisation: right-looking, 16-column panels.  The panel is factored in
// LDS (pivot search as a block arg-max with ties to the smaller row, as
// LAPACK's idamax), its row interchanges are applied to the other columns, the
// 16-row block of U is formed by forward substitution, and the trailing
// matrix is updated on the matrix cores (16x16x4 MFMA, FP64 or FP32) in strips
// of four 16x16 tiles per wave.
#pragma once

#include "device_common.hpp"

namespace abdf {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Lane layouts of the 16x16x4 matrix-core operations (wave64):
//   A operand: lane l holds A[l % 16][l / 16];  B operand: B[l / 16][l % 16];
//   accumulator register v of lane l holds C[row(l, v)][l % 16], where the
//   FP64 form interleaves rows (row = 4 v + l / 16) and the FP32 form blocks
//   them (row = 4 (l / 16) + v).  abdf_selftest checks both on the device.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    using acc_t = f64x4;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mfma<float> {
    using acc_t = f32x4;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kPanelStride = 17;   // LDS row stride of the 16-column panel
constexpr int kStrip = 4;          // 16x16 tiles per wave per trailing-update step

// LDS needed by lu_factor_wg for size NP and element type T.
template <typename T>
__host__ __device__ constexpr size_t lu_lds_bytes(int NP) {
    return size_t(NP) * kPanelStride * sizeof(T) + size_t(16) * NP * sizeof(T) + size_t(NP) * sizeof(int32_t) +
           kWaves * (sizeof(double) + sizeof(int32_t));
}

// Factors A (NP x NP, row-major, global) in place.  perm[i] receives the
// original row of row i of P A; *info receives 0 or the 1-based index of the
// first zero pivot.  smem must hold lu_lds_bytes<T>(NP).
template <typename T>
__device__ void lu_factor_wg(T *A, int NP, int32_t *perm, int32_t *info, unsigned char *smem) {
    using M = Mfma<T>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int PS = kPanelStride;
    T *P = reinterpret_cast<T *>(smem);
    T *U = P + size_t(NP) * PS;
    int32_t *piv = reinterpret_cast<int32_t *>(U + size_t(16) * NP);
    double *redv = reinterpret_cast<double *>(piv + NP);
    int32_t *redi = reinterpret_cast<int32_t *>(redv + kWaves);
    int first_zero = 0;

    for (int kb = 0; kb < NP; kb += 16) {
        const int m = NP - kb;
        for (int e = tid; e < m * 16; e += kBlock) {
            const int i = e >> 4, j = e & 15;
            P[i * PS + j] = A[size_t(kb + i) * NP + kb + j];
        }
        __syncthreads();
        for (int j = 0; j < 16; ++j) {
            double bv = -1.0;
            int bi = j;
            for (int i = j + tid; i < m; i += kBlock) {
                const double v = fabs(double(P[i * PS + j]));
                if (v > bv) { bv = v; bi = i; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { redv[wave] = bv; redi[wave] = bi; }
            __syncthreads();
            double fv = redv[0];
            int fi = redi[0];
            for (int w = 1; w < kWaves; ++w)
                if (redv[w] > fv || (redv[w] == fv && redi[w] < fi)) { fv = redv[w]; fi = redi[w]; }
            if (fi != j && tid < 16) {
                const T a = P[j * PS + tid];
                P[j * PS + tid] = P[fi * PS + tid];
                P[fi * PS + tid] = a;
            }
            if (tid == 0) piv[kb + j] = kb + fi;
            __syncthreads();
            const T pv = P[j * PS + j];
            if (tid == 0 && pv == T(0) && first_zero == 0) first_zero = kb + j + 1;
            for (int i = j + 1 + tid; i < m; i += kBlock) {
                T l = P[i * PS + j];
                if (pv != T(0)) l = l / pv;
                P[i * PS + j] = l;
                for (int jj = j + 1; jj < 16; ++jj) P[i * PS + jj] -= l * P[j * PS + jj];
            }
            __syncthreads();
        }
        for (int e = tid; e < m * 16; e += kBlock) {
            const int i = e >> 4, j = e & 15;
            A[size_t(kb + i) * NP + kb + j] = P[i * PS + j];
        }
        // this panel's interchanges on every other column, in order
        for (int c = tid; c < NP - 16; c += kBlock) {
            const int col = c < kb ? c : c + 16;
            for (int j = 0; j < 16; ++j) {
                const int r2 = piv[kb + j];
                if (r2 != kb + j) {
                    const T a = A[size_t(kb + j) * NP + col];
                    A[size_t(kb + j) * NP + col] = A[size_t(r2) * NP + col];
                    A[size_t(r2) * NP + col] = a;
                }
            }
        }
        __syncthreads();
        if (kb + 16 < NP) {
            const int nc = NP - kb - 16;
            // U12 = L11^{-1} A12
            for (int c = tid; c < nc; c += kBlock) {
                T u[16];
                for (int r = 0; r < 16; ++r) u[r] = A[size_t(kb + r) * NP + kb + 16 + c];
                for (int r = 1; r < 16; ++r)
                    for (int s = 0; s < r; ++s) u[r] -= P[r * PS + s] * u[s];
                for (int r = 0; r < 16; ++r) {
                    A[size_t(kb + r) * NP + kb + 16 + c] = u[r];
                    U[r * NP + c] = u[r];
                }
            }
            __syncthreads();
            // A22 -= L21 U12 on the matrix cores
            const int nt = nc / 16;
            const int nstrips = nt * ((nt + kStrip - 1) / kStrip);
            const int spr = (nt + kStrip - 1) / kStrip;   // strips per tile row
            for (int st = wave; st < nstrips; st += kWaves) {
                const int ti = st / spr, tj0 = (st % spr) * kStrip;
                const int r0 = kb + 16 + 16 * ti;
                typename M::acc_t acc[kStrip];
                for (int q = 0; q < kStrip; ++q) {
                    const int tj = tj0 + q;
                    if (tj < nt) {
                        const int c0 = kb + 16 + 16 * tj;
                        for (int v = 0; v < 4; ++v)
                            acc[q][v] = A[size_t(r0 + M::row(lane, v)) * NP + c0 + (lane & 15)];
                    }
                }
                T a[4];
                for (int s = 0; s < 4; ++s) a[s] = -P[(16 + 16 * ti + (lane & 15)) * PS + 4 * s + (lane >> 4)];
                for (int q = 0; q < kStrip; ++q) {
                    const int tj = tj0 + q;
                    if (tj < nt) {
                        for (int s = 0; s < 4; ++s) {
                            const T b = U[(4 * s + (lane >> 4)) * NP + 16 * tj + (lane & 15)];
                            acc[q] = M::mma(a[s], b, acc[q]);
                        }
                    }
                }
                for (int q = 0; q < kStrip; ++q) {
                    const int tj = tj0 + q;
                    if (tj < nt) {
                        const int c0 = kb + 16 + 16 * tj;
                        for (int v = 0; v < 4; ++v)
                            A[size_t(r0 + M::row(lane, v)) * NP + c0 + (lane & 15)] = acc[q][v];
                    }
                }
            }
            __syncthreads();
        }
    }
    // row interchanges -> permutation
    if (tid == 0) {
        for (int i = 0; i < NP; ++i) perm[i] = i;
        for (int i = 0; i < NP; ++i) {
            const int p = piv[i];
            const int t = perm[i];
            perm[i] = perm[p];
            perm[p] = t;
        }
        if (info) *info = first_zero;
    }
    __syncthreads();
}

// Solves (P^T L U) z = b for one system: b[NP] in LDS (FP64), factors in
// global memory as T, z returned in y[NP] (LDS).  red: 16 doubles of LDS.
template <typename T>
__device__ void lu_solve_wg(const T *__restrict__ A, const int32_t *__restrict__ perm, int NP, const double *b,
                            double *y, double *red) {
    const int tid = threadIdx.x;
    for (int i = tid; i < NP; i += kBlock) y[i] = b[perm[i]];
    __syncthreads();
    const int NT = NP / 16;
    const int rl = tid >> 4, cl = tid & 15;
    // forward substitution, unit lower triangle
    for (int tb = 0; tb < NT; ++tb) {
        const T *Arow = A + size_t(16 * tb + rl) * NP;
        double acc = 0.0;
        for (int j = cl; j < 16 * tb; j += 16) acc += double(Arow[j]) * y[j];
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (cl == 0) red[rl] = acc;
        __syncthreads();
        if (tid < 16) {
            const int r = 16 * tb + tid;
            double l[16];
            for (int jj = 0; jj < 16; ++jj) l[jj] = double(A[size_t(r) * NP + 16 * tb + jj]);
            double v = y[r] - red[tid];
            for (int jj = 0; jj < 16; ++jj) {
                const double yj = __shfl(v, jj);
                if (tid > jj) v -= l[jj] * yj;
            }
            y[r] = v;
        }
        __syncthreads();
    }
    // back substitution, upper triangle
    for (int tb = NT - 1; tb >= 0; --tb) {
        const T *Arow = A + size_t(16 * tb + rl) * NP;
        double acc = 0.0;
        for (int j = 16 * (tb + 1) + cl; j < NP; j += 16) acc += double(Arow[j]) * y[j];
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (cl == 0) red[rl] = acc;
        __syncthreads();
        if (tid < 16) {
            const int r = 16 * tb + tid;
            double u[16];
            for (int jj = 0; jj < 16; ++jj) u[jj] = double(A[size_t(r) * NP + 16 * tb + jj]);
            double v = y[r] - red[tid];
            for (int jj = 15; jj >= 0; --jj) {
                if (tid == jj) v = v / u[jj];
                const double zj = __shfl(v, jj);
                if (tid < jj) v -= u[jj] * zj;
            }
            y[r] = v;
        }
        __syncthreads();
    }
}

}  // namespace abdf
