// Tall-skinny FP64 kernels of the Davidson solvers (single and batched):
// basis updates Out = beta Out + alpha A B and the fused Ritz vector /
// residual / preconditioner step.  Both are plain HBM streams over column
// blocks of the basis.
//
// Lane layout: a column block of KB columns stores one 8*KB-byte row per
// determinant, read by LPN = KB/2 lanes as 16-byte pieces (one lane of 8 or
// 16 bytes for KB = 1, 2), the layout the sigma kernel uses for X.  Each row
// group issues the loads of several column blocks before using them, so
// many independent requests are in flight per lane and no barrier is
// needed; the per-row sums are combined with a butterfly of shuffles inside
// the group.  Each row is read completely before it is written, so an
// in-place update (Out aliasing A) is safe.
#pragma once

#include "common.hpp"

namespace hinqs {

template <int KB>
struct RowLanes {
    static constexpr int EPL = KB >= 2 ? 2 : 1;  // doubles per lane and column block
    static constexpr int LPN = KB / EPL;         // lanes per row
    static constexpr int BATCH = 6;              // column blocks loaded together
};

template <int EPL>
__device__ __forceinline__ void load_piece(const double *p, double (&x)[EPL]) {
    if constexpr (EPL == 2) {
        const double2 v = *(const double2 *)p;
        x[0] = v.x;
        x[1] = v.y;
    } else {
        x[0] = *p;
    }
}

// acc[c] += sum over the columns j < m of row i of A (A.kb == KB) of
// A(i, j) * sB[j * NC + c]; sB (LDS) holds ceil(m / KB) * KB rows, zero for
// j >= m.  q = lane within the row group.  Returns the per-lane partial sums
// (the group's lanes cover different columns j).
template <int KB, int NC>
__device__ __forceinline__ void row_times_small(int64_t i, int m, const Mat &A, const double *sB, int q,
                                                double (&acc)[NC]) {
    using L = RowLanes<KB>;
    const int nbk = (m + KB - 1) / KB;
    for (int b0 = 0; b0 < nbk; b0 += L::BATCH) {
        double x[L::BATCH][L::EPL];
#pragma unroll
        for (int u = 0; u < L::BATCH; ++u) {
            const int b = b0 + u < nbk ? b0 + u : nbk - 1;  // clamped, not predicated
            load_piece<L::EPL>(A.p + (int64_t)b * A.bs + i * KB + q * L::EPL, x[u]);
        }
#pragma unroll
        for (int u = 0; u < L::BATCH; ++u) {
            if (b0 + u >= nbk) break;
            const double *brow = sB + ((b0 + u) * KB + q * L::EPL) * NC;
#pragma unroll
            for (int e = 0; e < L::EPL; ++e)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += x[u][e] * brow[e * NC + c];
        }
    }
}

// Sum over the LPN lanes of a row group; every lane receives the totals.
template <int LPN, int NC>
__device__ __forceinline__ void group_sum(double (&acc)[NC]) {
#pragma unroll
    for (int off = 1; off < LPN; off <<= 1)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += __shfl_xor(acc[c], off, LPN);
}

// Out(i, c) = beta Out(i, c) + alpha * sum_{j<m} A(i, j) B[j][c] for c < nc
// (B staged in LDS as sB, see row_times_small).  Column c of Out is written
// by lane (c % KB) / EPL of the group, so with Out.kb == KB each lane stores
// its own 16-byte piece of every output block.
template <int KB, int NC>
__device__ __forceinline__ void tsmm_row(int64_t i, int m, const Mat &A, const double *sB, int nc, double alpha,
                                         double beta, const Mat &Out, int q) {
    using L = RowLanes<KB>;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    row_times_small<KB, NC>(i, m, A, sB, q, acc);
    group_sum<L::LPN, NC>(acc);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= nc || ((c % KB) / L::EPL) != q) continue;
        double *o = Out.at(i, c);
        *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * acc[c];
    }
}

// Ritz vectors, residuals and preconditioned corrections of row i for the
// first nroots of KB roots:
//   x_c = V y_c,  w_c = W y_c,  r_c = w_c - theta_c x_c,
//   T[i][c] = r_c / clamp(theta_c - d_i),
// with V, W sharing the column layout (kb == KB), sY = Y staged as in
// row_times_small, th = theta.  Adds r_c^2 and T[i][c]^2 of the lane's own
// columns (c = q * EPL + e) to rn2[e], tn2[e].
template <int KB>
__device__ __forceinline__ void ritz_row(int64_t i, int m, const Mat &V, const Mat &W, const double *sY,
                                         const double *th, double d, double floor_, int nroots,
                                         double *__restrict__ T, int q, double (&rn2)[RowLanes<KB>::EPL],
                                         double (&tn2)[RowLanes<KB>::EPL]) {
    using L = RowLanes<KB>;
    double ax[KB], aw[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) ax[c] = aw[c] = 0.0;
    row_times_small<KB, KB>(i, m, V, sY, q, ax);
    row_times_small<KB, KB>(i, m, W, sY, q, aw);
    group_sum<L::LPN, KB>(ax);
    group_sum<L::LPN, KB>(aw);
    double out[L::EPL];
#pragma unroll
    for (int e = 0; e < L::EPL; ++e) out[e] = 0.0;
#pragma unroll
    for (int c = 0; c < KB; ++c) {
        const int e = c % L::EPL;
        if (c / L::EPL != q || c >= nroots) continue;
        const double res = aw[c] - th[c] * ax[c];
        double den = th[c] - d;
        if (fabs(den) < floor_) den = den < 0.0 ? -floor_ : floor_;
        const double t = res / den;
        rn2[e] += res * res;
        tn2[e] += t * t;
        out[e] = t;
    }
    if constexpr (L::EPL == 2) {
        *(double2 *)(T + i * KB + q * 2) = double2{out[0], out[1]};
    } else {
        T[i * KB + q] = out[0];
    }
}

// Workgroup totals of the per-lane sums of ritz_row: root c gathers the
// lanes with c / EPL == lane % LPN.  red: 2 * blockDim.x doubles of LDS.
// Thread c < KB returns (sum r_c^2, sum T_c^2).
template <int KB>
__device__ __forceinline__ void ritz_block_sums(const double (&rn2)[RowLanes<KB>::EPL],
                                                const double (&tn2)[RowLanes<KB>::EPL], double *red,
                                                double &rs, double &ts) {
    using L = RowLanes<KB>;
    const int nt = blockDim.x;
    rs = ts = 0.0;
#pragma unroll
    for (int e = 0; e < L::EPL; ++e) {
        __syncthreads();
        red[threadIdx.x] = rn2[e];
        red[nt + threadIdx.x] = tn2[e];
        __syncthreads();
        if ((int)threadIdx.x < KB && (int)threadIdx.x % L::EPL == e) {
            const int q = (int)threadIdx.x / L::EPL;
            for (int l = q; l < nt; l += L::LPN) {
                rs += red[l];
                ts += red[nt + l];
            }
        }
    }
}

}  // namespace hinqs
