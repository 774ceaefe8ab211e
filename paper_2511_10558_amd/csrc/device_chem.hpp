// Rate coefficients, right-hand side and Newton-matrix rows for one cell,
// evaluated cooperatively by one workgroup.
#pragma once

#include "device_common.hpp"
#include "network.hpp"

namespace abdf {

// k_r for one cell (paper Sec. 2 Kooij-Arrhenius and direct cosmic-ray forms,
// App. B.1 photo form and the cosmic-ray-induced photon form
// alpha (T/300)^beta E zeta / (1 - omega), E the reaction's efficiency kept in
// its gamma field, omega the network's dust albedo); two-body coefficients carry the factor n_H of the
// fractional-abundance state.  Written to global memory, coalesced over r.
__device__ inline void cell_rates(const DeviceNet &n, const double *phi, double *k) {
    const double T = phi[0], nH = phi[1], Av = phi[2], zeta = phi[3], G0 = phi[4];
    const double T300 = T / 300.0;
    for (int r = threadIdx.x; r < n.R; r += kBlock) {
        const int t = n.rx_type[r];
        const double a = n.alpha[r];
        double v;
        if (t == kTwoBody) v = a * pow(T300, n.beta[r]) * exp(-n.gamma[r] / T) * nH;
        else if (t == kCosmicRay) v = a * zeta;
        else if (t == kCrPhoton) v = a * pow(T300, n.beta[r]) * (n.gamma[r] / (1.0 - n.albedo)) * zeta;
        else v = a * G0 * exp(-n.gamma[r] * Av);
        k[r] = v;
    }
}

// out_i = sum_r nu_ir v_r for per-reaction values v (LDS), in the wave layout
// of DeviceNet::sg_ent: each wave takes groups of 64 lanes; a lane sums its
// entries in order from zero, then the lanes of each species are added
// pairwise within the wave and the species' first lane writes out_i.
// Deterministic: the order of every sum is fixed by the layout, whichever
// wave takes a group.  The entries are loaded eight at a time before any is
// used, so the loads are in flight together.  Ends with a barrier.
template <int NT = kBlock>
__device__ __forceinline__ void species_gather(const DeviceNet &n, const double *v, double *out) {
    constexpr int kB = 8;
    const int lane = threadIdx.x & 63;
    for (int g = threadIdx.x >> 6; g < n.n_sgroup; g += NT / 64) {
        const int mine = n.sg_lane[g * 64 + lane];
        const int lw = n.sg_len[g];
        const int L = lw & 0xffffff, steps = lw >> 24;
        const int32_t *ent = n.sg_ent + n.sg_base[g] + lane;
        double acc = 0.0;
        for (int jb = 0; jb < L; jb += kB) {
            int w[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) w[u] = jb + u < mine ? ent[(jb + u) * 64] : 4;   // 4: coefficient 0, entry 0
            double vv[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) vv[u] = v[w[u] >> 3];
#pragma unroll
            for (int u = 0; u < kB; ++u)
                if (jb + u < mine) acc += double((w[u] & 7) - 4) * vv[u];
        }
        // the species' lanes pairwise; steps is the same for the whole wave
        const int red = n.sg_red[g * 64 + lane];
        const int q = red < 0 ? 0 : (red >> 7) & 127, m = red < 0 ? 1 : red & 127;
        for (int t = 0; t < steps; ++t) {
            const int off = 1 << t;
            const double o = __shfl_down(acc, off);
            if ((q & (2 * off - 1)) == 0 && q + off < m) acc += o;
        }
        if (red >= 0 && q == 0) out[red >> 14] = acc;
    }
    __syncthreads();
}

// f = nu . rate(x) for one cell.  x in LDS; k in global memory (one coalesced
// pass); rate[R] is LDS scratch; f may be LDS or global.
// Deterministic: every sum runs in a fixed order.
// kWide: more loads in flight per thread, for kernels with registers to spare.
template <int NT = kBlock, bool kWide = false>
__device__ __forceinline__ void cell_rhs(const DeviceNet &n, const double *__restrict__ k, const double *x,
                                double *rate, double *f) {
    // kU reactions per thread per pass, their loads issued before any use
    constexpr int kU = kWide ? 6 : 4;
    for (int r0 = threadIdx.x; r0 < n.R; r0 += kU * NT) {
        int ab[kU];
        double kr[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = r0 + u * NT;
            ab[u] = r < n.R ? n.rx_ab[r] : 0;
            kr[u] = r < n.R ? k[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = r0 + u * NT;
            const int a = ab[u] & 0xffff, b = (ab[u] >> 16) & 0xffff;
            double v = kr[u] * x[a];
            if (b != 0xffff) v *= x[b];
            if (r < n.R) rate[r] = v;
        }
    }
    __syncthreads();
    species_gather<NT>(n, rate, f);
}

// J(x) y = nu . (d rate / dx) y for one cell: per reaction
// k_r (y_a x_b + x_a y_b) (k_r y_a for one reactant; the same expression gives
// 2 k_r x_a y_a for A + A), then the species sums of cell_rhs.  x, y in LDS;
// drate[R] LDS scratch.
__device__ __forceinline__ void cell_jvp(const DeviceNet &n, const double *__restrict__ k, const double *x,
                                         const double *y, double *drate, double *out) {
    for (int r0 = threadIdx.x; r0 < n.R; r0 += 4 * kBlock) {
        int ab[4];
        double kr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * kBlock;
            ab[u] = r < n.R ? n.rx_ab[r] : 0;
            kr[u] = r < n.R ? k[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * kBlock;
            const int a = ab[u] & 0xffff, b = (ab[u] >> 16) & 0xffff;
            const double v = b == 0xffff ? kr[u] * y[a] : kr[u] * (y[a] * x[b] + x[a] * y[b]);
            if (r < n.R) drate[r] = v;
        }
    }
    __syncthreads();
    species_gather(n, drate, out);
}

// The Jacobian nonzeros J_e(x) of one cell into jv[nnzJ] (global, written
// coalesced): each nonzero's terms summed in the order of its term list.  x in
// LDS, k in global memory.  Cooperative.
template <int NT>
__device__ __forceinline__ void jacobian_values(const DeviceNet &n, const double *__restrict__ k, const double *x,
                                                double *jv) {
    // a nonzero's terms are loaded four at a time before any is used; the sum
    // still runs term by term in order
    for (int e = threadIdx.x; e < n.nnzJ; e += NT) {
        double v = 0.0;
        const int t0 = n.jterm_ptr[e], t1 = n.jterm_ptr[e + 1];
        for (int tb = t0; tb < t1; tb += 4) {
            int w[4];
            double cf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool in = tb + u < t1;
                w[u] = in ? n.jt_rx_other[tb + u] : 0;
                cf[u] = in ? n.jt_coef[tb + u] : 0.0;
            }
            double kv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int other = (w[u] & 0xffff) - 1;
                kv[u] = k[w[u] >> 16];
                xv[u] = x[other >= 0 ? other : 0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (tb + u < t1) {
                    double term = cf[u] * kv[u];
                    if ((w[u] & 0xffff) != 0) term *= xv[u];
                    v += term;
                }
            }
        }
        jv[e] = v;
    }
}

// Entries of M = I - c J of one cell where the factorisation gathers them:
// the 64-column words of the Jacobian's pattern give the nonzero of (i, j)
// (one word and one base per row and block column, shared by the lanes of a
// row); rows and columns beyond S are the identity's.
template <typename T>
struct NewtonMatrixSource {
    const uint64_t *jmask;   // [NP][nbw] pattern words
    const int32_t *jbase;    // [NP][nbw] index of the first nonzero of each word
    int nbw;
    const double *jv;        // the entries' values
    double c;
    // Entries are read in two passes, every row's word first and then every
    // value, so that no load waits behind a condition on an earlier one;
    // structural zeros load nothing.
    struct Row { uint64_t m; int32_t base; };
    __device__ __forceinline__ Row row(int i, int c0) const {
        const size_t w = size_t(i) * nbw + (c0 >> 6);
        return {jmask[w], jbase[w]};
    }
    __device__ __forceinline__ T entry(const Row &w, int i, int j) const {
        const int bit = j & 63;
        const bool nz = (w.m >> bit) & 1ull;
        const double jvv = nz ? jv[w.base + __popcll(w.m & ((1ull << bit) - 1ull))] : 0.0;
        return T((i == j ? 1.0 : 0.0) - c * jvv);
    }
};

}  // namespace abdf
