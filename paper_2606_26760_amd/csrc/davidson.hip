// Block Davidson eigensolver for the lowest eigenpair of H_B (paper Sec. 2.2,
// Step 3: Davidson diagonalization of H_B, warm-started from the previous
// eigenvector).
//
// Storage.  The basis V and its images W = H V live in HBM column-blocked:
// block b holds columns [bK, bK+K) as a contiguous ndet x K row-major array
// (K = Davidson block size), in sorted determinant order.  New directions are
// formed in a contiguous ndet x K array T, so every sigma product reads one
// 64-byte row per coupling from a compact 8*K*ndet-byte array that stays in
// the caches, and its output Wn is appended to W afterwards.
//
// Per iteration:
//   Rayleigh-Ritz on G = V^T W         host Householder + implicit QL (cyclic
//                                      Jacobi if QL does not converge), m <= 96
//   T = (W y - theta V y) / (theta - H_ii)   fused Ritz/residual/preconditioner
//                                      (V y, W y on FP64 MFMA, like every
//                                      tall-skinny product of the solver)
//   classical Gram-Schmidt of T against V (a second pass only when the first
//   removed most of a column), then symmetric orthonormalization of T
//   (eigendecomposition of T^T T; nearly dependent directions dropped)
//   Wn = H T                           sigma kernel
//   G[:, new] = V^T Wn                 FP64 MFMA (v_mfma_f64_16x16x4f64) partials
//                                      reduced in a fixed order (deterministic)
// Restart (GD+k): when the space is full it is replaced by an orthonormal
// basis of the current Ritz vectors and those of the previous iteration,
// which keeps the convergence of the unrestarted method far better than a
// restart on the Ritz vectors alone.
// MIXED precision: FP32 off-diagonal sigma products (diagonal term added in
// FP64) while the residual is above a switch threshold (or until it stalls for
// three iterations below 1e-4 |theta|, near the FP32 rounding floor; or for
// eight anywhere), then a restart on the Ritz vectors, W recomputed with FP64
// sigma, and FP64 iterations to the requested tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "common.hpp"

namespace hinqs {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_BLOCK = 256;
constexpr int GRAM_MAX_BLOCKS = 512;
constexpr int GRAM_UNROLL = 4;

// partial[blk][a][b] = sum over this block's rows of A(i, a) * B(i, b)
// (a < ma <= 16*MT, b < nb <= 16).  MFMA operand layout (16x16x4 f64):
// lane l supplies A_mat[l%16][l/16] and B_mat[l/16][l%16] and receives
// D[l/16 + 4r][l%16] in element r of its 4-wide accumulator.  Loads for
// GRAM_UNROLL steps are issued before their MFMAs to keep loads in flight.
template <int MT>
__global__ __launch_bounds__(GRAM_BLOCK) void k_gram(int64_t nrows, Mat A, int ma, Mat B, int nb,
                                                     int64_t rows_per_wave, double *__restrict__ partial,
                                                     const int *__restrict__ gate) {
    if (gate && *gate == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * (GRAM_BLOCK / 64) + wave;
    const int64_t r0 = gw * rows_per_wave;
    const int64_t r1 = min(nrows, r0 + rows_per_wave);
    const int col = lane & 15, kk = lane >> 4;
    dbl4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    const bool bok = col < nb;
    for (int64_t i = r0; i < r1; i += 4 * GRAM_UNROLL) {
        double bv[GRAM_UNROLL], av[GRAM_UNROLL][MT];
#pragma unroll
        for (int u = 0; u < GRAM_UNROLL; ++u) {
            const int64_t row = i + 4 * u + kk;
            const bool rok = row < r1;
            bv[u] = (rok && bok) ? *B.at(row, col) : 0.0;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int a = t * 16 + col;
                av[u][t] = (rok && a < ma) ? *A.at(row, a) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < GRAM_UNROLL; ++u)
#pragma unroll
            for (int t = 0; t < MT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[u], acc[t], 0, 0, 0);
    }
    __shared__ double red[GRAM_BLOCK / 64][MT][64][4];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave][t][lane][r] = acc[t][r];
    __syncthreads();
    for (int e = threadIdx.x; e < MT * 256; e += GRAM_BLOCK) {
        const int t = e / 256, rem = e % 256, ln = rem / 4, r = rem % 4;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < GRAM_BLOCK / 64; ++w) s += red[w][t][ln][r];
        const int a = t * 16 + (ln >> 4) + 4 * r;
        const int b = ln & 15;
        if (a < ma && b < nb) partial[(int64_t)blockIdx.x * ma * nb + a * nb + b] = s;
    }
}

// out[e] = sum_blk partial[blk][e]: one workgroup per output, fixed-shape tree.
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partial, int nblk,
                                                         int n, double *__restrict__ out,
                                                         const int *__restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ double red[256];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)b * n + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

// Fused Ritz vector, residual, norm and diagonal preconditioner for the
// first nroots of KB roots:
//   r_c = W y_c - theta_c V y_c,   T[:, c] = r_c / clamp(theta_c - H_ii)
// (T[:, c] = 0 for c >= nroots).  V Y and W Y run on FP64 MFMA with the
// operand layout of k_tsmm (16-row tiles, Y held in registers, m <= 4 STEPS);
// the elementwise part works on the accumulators, whose element r of lane l is
// row r0 + l/16 + 4r, column l%16.  partial[blk][c] = sum over the block's
// rows of r_c^2 and partial[blk][KB + c] the same for T[:, c]^2.
template <int KB, int STEPS>
__global__ __launch_bounds__(256) void k_ritz(int64_t nrows, int m, Mat V, Mat W, const double *__restrict__ Y,
                                              const double *__restrict__ theta, const double *__restrict__ diag,
                                              double floor_, int nroots, double *__restrict__ T,
                                              double *__restrict__ partial) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    double yv[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        const int j = 4 * s + kk;
        yv[s] = (j < m && col < KB) ? Y[j * KB + col] : 0.0;
    }
    const bool live = col < nroots;
    const double th = col < KB ? theta[col] : 0.0;
    const int nsteps = (m + 3) / 4;
    const int64_t ntiles = (nrows + 15) / 16;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double rn2 = 0.0, tn2 = 0.0;
    for (int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; tile < ntiles; tile += nwaves) {
        const int64_t r0 = tile * 16, ra = r0 + col;
        const bool rok = ra < nrows;
        dbl4 ax = dbl4{0.0, 0.0, 0.0, 0.0}, aw = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s0 = 0; s0 < STEPS; s0 += 4) {
            if (s0 >= nsteps) break;
            double xv[4], wv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 4 * (s0 + u) + kk;
                const bool ok = rok && j < m;
                xv[u] = ok ? *V.at(ra, j) : 0.0;
                wv[u] = ok ? *W.at(ra, j) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ax = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[u], yv[s0 + u], ax, 0, 0, 0);
                aw = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[u], yv[s0 + u], aw, 0, 0, 0);
            }
        }
        if (col < KB) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + kk + 4 * r;
                if (row >= nrows) continue;
                double t = 0.0;
                if (live) {
                    const double res = aw[r] - th * ax[r];
                    double den = th - diag[row];
                    if (fabs(den) < floor_) den = den < 0.0 ? -floor_ : floor_;
                    t = res / den;
                    rn2 += res * res;
                    tn2 += t * t;
                }
                T[row * KB + col] = t;
            }
        }
    }
    // block sums per column: the lanes of column c are c, c + 16, c + 32, c + 48 in every wave
    __shared__ double red[2][4][64];
    red[0][wave][lane] = rn2;
    red[1][wave][lane] = tn2;
    __syncthreads();
    if ((int)threadIdx.x < KB) {
        const int c = threadIdx.x;
        double rs = 0.0, ts = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int q = 0; q < 4; ++q) {
                rs += red[0][w][c + 16 * q];
                ts += red[1][w][c + 16 * q];
            }
        partial[(int64_t)blockIdx.x * 2 * KB + c] = rs;
        partial[(int64_t)blockIdx.x * 2 * KB + KB + c] = ts;
    }
}

// gate[0] = 1 when the projection T -= V (V^T T) needs a second pass: some
// column q (tn2[q] = ||T_q||^2 > 0 before the first pass) kept less than half
// of its norm, ||T_q||^2 - ||(V^T T)_q||^2 < ||T_q||^2 / 4 (NaN counts as
// less); else 0.  C is the first pass's m x nc product V^T T; one wave.
__global__ void k_proj_gate(const double *__restrict__ C, int m, int nc, const double *__restrict__ tn2,
                            int *__restrict__ gate, int *__restrict__ count) {
    const int q = threadIdx.x;
    bool need = false;
    if (q < nc && tn2[q] > 0.0) {
        double c2 = 0.0;
        for (int a = 0; a < m; ++a) c2 += C[a * nc + q] * C[a * nc + q];
        need = !(tn2[q] - c2 >= 0.25 * tn2[q]);
    }
    const bool any = __ballot(need) != 0ull;
    if (threadIdx.x == 0) {
        *gate = any ? 1 : 0;
        *count += any ? 1 : 0;  // second passes run in this solve
    }
}

// Out(i, c) = beta Out(i, c) + alpha sum_{j<m} A(i, j) B[j][c] for c < nc <= 16 NT, m <= 4 STEPS,
// with FP64 MFMA (16x16x4): each wave takes 16-row tiles in turn; for k-step s lane l supplies
// A(r0 + l%16, 4s + l/16), holds B[4s + l/16][16t + l%16] for every step in registers, and
// receives rows r0 + l/16 + 4r of output column 16t + l%16.  A tile's rows are all read before
// any is written, so Out may alias A.  B is m x nc row-major.
template <int NT, int STEPS>
__global__ __launch_bounds__(256) void k_tsmm(int64_t nrows, int m, Mat A, const double *__restrict__ B, int nc,
                                              double alpha, double beta, Mat Out, const int *__restrict__ gate) {
    if (gate && *gate == 0) return;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
    double bv[STEPS][NT];
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 4 * s + kk, c = 16 * t + col;
            bv[s][t] = (j < m && c < nc) ? B[j * nc + c] : 0.0;
        }
    const int nsteps = (m + 3) / 4;
    const int64_t ntiles = (nrows + 15) / 16;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; tile < ntiles; tile += nwaves) {
        const int64_t r0 = tile * 16, ra = r0 + col;
        const bool rok = ra < nrows;
        dbl4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s0 = 0; s0 < STEPS; s0 += 4) {
            if (s0 >= nsteps) break;
            double av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 4 * (s0 + u) + kk;
                av[u] = (rok && j < m) ? *A.at(ra, j) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[s0 + u][t], acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + col;
            if (c >= nc) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + kk + 4 * r;
                if (row >= nrows) continue;
                double *o = Out.at(row, c);
                *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * acc[t][r];
            }
        }
    }
}

// dst(i, c0 + c) = src[i * K + c] for c < nc.
__global__ void k_put_columns(int64_t nrows, const double *src, int K, int nc, Mat dst, int c0) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * K) return;
    const int64_t i = t / K;
    const int c = (int)(t % K);
    if (c < nc) *dst.at(i, c0 + c) = src[t];
}

// Columns [c0, c0+nc) of a row-major ndet x K array: unit entries at rows idx[c].
__global__ void k_unit_columns(int64_t nrows, double *T, int K, int c0, int nc, const int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int c = 0; c < nc; ++c) T[i * K + c0 + c] = (idx[c] == i) ? 1.0 : 0.0;
}

__global__ void k_copy_column(int64_t nrows, const double *src, double *T, int K, int c) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    T[i * K + c] = src[i];
}

// Lexicographic (value, index) minimum of diag over rows not in excl[0..nex).
__global__ void k_argmin_partial(int64_t nrows, const double *diag, const int32_t *excl, int nex,
                                 double *pv, int64_t *pi) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double best = INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool skip = false;
        for (int e = 0; e < nex; ++e) skip |= (excl[e] == i);
        if (skip) continue;
        double v = diag[i];
        if (v < best || (v == best && i < bi)) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double v = sv[threadIdx.x + s];
            int64_t j = si[threadIdx.x + s];
            if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x])) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { pv[blockIdx.x] = sv[0]; pi[blockIdx.x] = si[0]; }
}

__global__ void k_argmin_final(int nblk, const double *pv, const int64_t *pi, int32_t *excl, int slot) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double best = INFINITY;
    int64_t bi = INT64_MAX;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        double v = pv[b];
        int64_t j = pi[b];
        if (v < best || (v == best && j < bi)) { best = v; bi = j; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double v = sv[threadIdx.x + s];
            int64_t j = si[threadIdx.x + s];
            if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x])) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) excl[slot] = (int32_t)si[0];
}

// Largest |x_i| (lowest index on ties), per block then final.
__global__ void k_absmax_partial(int64_t nrows, const double *x, double *pv, int64_t *pi) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = fabs(x[i]);
        if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double v = sv[threadIdx.x + s];
            int64_t j = si[threadIdx.x + s];
            if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x])) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = j;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { pv[blockIdx.x] = sv[0]; pi[blockIdx.x] = si[0]; }
}

__global__ void k_absmax_final(int nblk, const double *pv, const int64_t *pi, const double *x,
                               double *sign_out) {
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int b = 0; b < nblk; ++b) {
        if (pv[b] > best || (pv[b] == best && pi[b] < bi)) { best = pv[b]; bi = pi[b]; }
    }
    *sign_out = (bi != INT64_MAX && x[bi] < 0.0) ? -1.0 : 1.0;
}

// out[perm[i]] = x[i] * scale * (*sign)   (perm null: out[i])
__global__ void k_finalize(int64_t nrows, const double *x, double scale, const double *sign,
                           const int32_t *perm, double *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    double v = x[i] * scale * (*sign);
    out[perm ? perm[i] : i] = v;
}

__global__ void k_to_f32(int64_t n, const double *x, float *y) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = (float)x[t];
}

// W = (double)S32 + diag * X: the FP32 product covers the off-diagonal part only, and the
// diagonal term (whose magnitude is the total energy, ~1e2 Ha) is applied in FP64 to the FP64
// vector, so FP32 rounding no longer scales with |H_ii| and the FP32 phase can reach a far smaller
// residual before the FP64 refinement.
__global__ void k_fp32_finish(int64_t n, int K, const float *s32, const double *diag, const double *x,
                              double *w) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) w[t] = (double)s32[t] + diag[t / K] * x[t];
}

// ------------------------------------------------------------ host helpers

int gram_blocks_for(int64_t nrows) {
    int64_t waves = (nrows + 63) / 64;
    return (int)std::min<int64_t>(GRAM_MAX_BLOCKS, std::max<int64_t>(1, (waves + 3) / 4));
}

// G (ma x nb) = A^T B over nrows rows: MFMA partials per block, then a
// fixed-order reduction.  partial must hold nblk * ma * nb doubles.
void launch_gram(hipStream_t s, int64_t nrows, int nblk, Mat A, int ma, Mat B, int nb, double *partial,
                 double *out, const int *gate = nullptr) {
    if (nb > 16 || ma > 96 || ma < 1 || nb < 1) throw Error(HINQS_E_UNSUPPORTED, "Gram block shape");
    int64_t waves = (int64_t)nblk * (GRAM_BLOCK / 64);
    int64_t rpw = (nrows + waves - 1) / waves;
    rpw = (rpw + 3) / 4 * 4;
    const int mt = (ma + 15) / 16;
    dim3 g(nblk), b(GRAM_BLOCK);
    switch (mt) {
        case 1: hipLaunchKernelGGL(k_gram<1>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
        case 2: hipLaunchKernelGGL(k_gram<2>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
        case 3: hipLaunchKernelGGL(k_gram<3>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
        case 4: hipLaunchKernelGGL(k_gram<4>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
        case 5: hipLaunchKernelGGL(k_gram<5>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
        default: hipLaunchKernelGGL(k_gram<6>, g, b, 0, s, nrows, A, ma, B, nb, rpw, partial, gate); break;
    }
    HQ_LAUNCH_CHECK();
    const int n = ma * nb;
    hipLaunchKernelGGL(k_reduce_partials, dim3(n), dim3(256), 0, s, partial, nblk, n, out, gate);
    HQ_LAUNCH_CHECK();
}

// Cyclic Jacobi eigendecomposition of a symmetric n x n matrix (row-major).
// Eigenvalues ascending in w; eigenvectors as columns of Z (row-major n x n).
void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z) {
    std::vector<double> V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    double fro = 0.0;
    for (double x : A) fro += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
        if (off <= 1e-32 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = cs * akp - sn * akq;
                    a(k, q) = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = cs * apk - sn * aqk;
                    a(q, k) = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
        }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
    w.resize(n);
    Z.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        w[c] = a(ord[c], ord[c]);
        for (int k = 0; k < n; ++k) Z[(size_t)k * n + c] = V[(size_t)k * n + ord[c]];
    }
}

// Symmetric eigendecomposition by Householder reduction to tridiagonal form
// followed by the implicit-shift QL iteration (the classic tridiagonal
// eigenvalue method of Bowdler, Martin, Reinsch and Wilkinson), with the
// transformations accumulated into the eigenvectors: O(n^3) with a small
// constant, several times faster than cyclic Jacobi at the subspace sizes of
// the solver.  Same outputs as jacobi_eig; returns false if an eigenvalue
// needs more than 60 QL iterations (the caller then falls back to Jacobi).
bool tridiag_ql_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z) {
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    // QT holds Q transposed (row j = column j of Q), so the updates below run
    // along contiguous rows
    std::vector<double> QT((size_t)n * n, 0.0), v(n), pv(n), d(n), e(n, 0.0), tq(n);
    for (int i = 0; i < n; ++i) QT[(size_t)i * n + i] = 1.0;
    // Householder: A <- H A H column by column, Q <- Q H
    for (int k = 0; k + 2 < n; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += a(i, k) * a(i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        if (a(k + 1, k) > 0.0) alpha = -alpha;  // v = x - alpha e1 without cancellation
        double vv = 0.0;
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
        v[k + 1] -= alpha;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // p = beta A v, q = p - (beta/2)(v.p) v, A <- A - v q^T - q v^T
        double vp = 0.0;
        for (int i = k; i < n; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += a(i, j) * v[j];
            pv[i] = beta * t;
        }
        for (int i = k + 1; i < n; ++i) vp += v[i] * pv[i];
        const double kk = 0.5 * beta * vp;
        for (int i = k; i < n; ++i) pv[i] -= kk * v[i];
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) a(i, j) -= v[i] * pv[j] + pv[i] * v[j];
        // Q <- Q (I - beta v v^T): t_i = beta sum_j Q[i][j] v[j], Q[i][j] -= t_i v[j]
        for (int i = 0; i < n; ++i) tq[i] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const double *qj = &QT[(size_t)j * n];
            const double vj = v[j];
            for (int i = 0; i < n; ++i) tq[i] += qj[i] * vj;
        }
        for (int i = 0; i < n; ++i) tq[i] *= beta;
        for (int j = k + 1; j < n; ++j) {
            double *qj = &QT[(size_t)j * n];
            const double vj = v[j];
            for (int i = 0; i < n; ++i) qj[i] -= tq[i] * vj;
        }
    }
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
    // implicit QL on (d, e); columns of Q follow the rotations
    for (int l = 0; l < n; ++l) {
        int iter = 0, m;
        do {
            for (m = l; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) + dd == dd) break;
            }
            if (m != l) {
                if (++iter > 60) return false;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = std::sqrt(g * g + 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? std::fabs(r) : -std::fabs(r)));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i];
                    const double b = c * e[i];
                    // plain sqrt instead of hypot: the entries of these Gram matrices
                    // are far from overflow, and a norm that underflows to zero takes
                    // the exact-zero branch below
                    r = std::sqrt(f * f + g * g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    double *zi = &QT[(size_t)i * n], *zi1 = &QT[(size_t)(i + 1) * n];
                    for (int k = 0; k < n; ++k) {
                        const double fk = zi1[k];
                        zi1[k] = s * zi[k] + c * fk;
                        zi[k] = c * zi[k] - s * fk;
                    }
                }
                if (r == 0.0 && i >= l) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    for (double x : d)
        if (!std::isfinite(x)) return false;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
    w.resize(n);
    Z.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        w[c] = d[ord[c]];
        const double *qc = &QT[(size_t)ord[c] * n];
        for (int k = 0; k < n; ++k) Z[(size_t)k * n + c] = qc[k];
    }
    return true;
}

// Eigenpairs of a small symmetric matrix: tridiagonal QL, Jacobi as fallback.
void small_sym_eig(int n, const std::vector<double> &A, std::vector<double> &w, std::vector<double> &Z) {
    if (n >= 3 && tridiag_ql_eig(n, A, w, Z)) return;
    jacobi_eig(n, A, w, Z);
}

// Orthonormal basis (modified Gram-Schmidt, twice) of the columns of the
// m x q row-major matrix M; columns whose remaining norm falls below `drop`
// times their original norm are dropped.  Returns m x qk row-major.
std::vector<double> small_orth(int m, int q, const std::vector<double> &M, double drop, int &qk) {
    std::vector<std::vector<double>> cols;
    for (int c = 0; c < q; ++c) {
        std::vector<double> v(m);
        double n0 = 0.0;
        for (int a = 0; a < m; ++a) { v[a] = M[(size_t)a * q + c]; n0 += v[a] * v[a]; }
        n0 = std::sqrt(n0);
        if (!(n0 > 0.0)) continue;
        for (int pass = 0; pass < 2; ++pass)
            for (const auto &u : cols) {
                double d = 0.0;
                for (int a = 0; a < m; ++a) d += u[a] * v[a];
                for (int a = 0; a < m; ++a) v[a] -= d * u[a];
            }
        double n1 = 0.0;
        for (int a = 0; a < m; ++a) n1 += v[a] * v[a];
        n1 = std::sqrt(n1);
        if (n1 <= drop * n0) continue;
        for (int a = 0; a < m; ++a) v[a] /= n1;
        cols.push_back(v);
    }
    qk = (int)cols.size();
    std::vector<double> Q((size_t)m * qk);
    for (int c = 0; c < qk; ++c)
        for (int a = 0; a < m; ++a) Q[(size_t)a * qk + c] = cols[c][a];
    return Q;
}

struct Solver {
    Ctx &c;
    hipStream_t s;
    int64_t D;
    int K;        // block size (compile-time kernel variant)
    int mmax;     // largest subspace
    int nblocks;  // column blocks of V and W
    // workspace kept in the context between solves
    DBuf<double> &Vb, &Wb, &T, &Wn, &small, &partial, &nrm;
    Mat V{}, W{}, Tm{}, Wnm{};
    // Tm / Wnm: where the next new directions and their images are formed.
    // When they start a column block of V (m a multiple of K, with a block
    // left), that block of V and of W directly, so nothing is copied after
    // the product; otherwise the separate T and Wn arrays.
    bool direct = false;
    DBuf<float> &X32, &S32;
    DBuf<int32_t> &guess_idx;
    DBuf<double> &argv;
    DBuf<int64_t> &argi;
    DBuf<double> &xfin, &signbuf;
    int nblk_gram = 1;
    std::vector<hipEvent_t> evs;  // start/stop pairs around every sigma product, read at the end
    double ms_sigma = 0.0;
    int sigma_blocks = 0, sigma_columns = 0;
    // pinned staging ring for small host -> device uploads (no sync per upload)
    static constexpr int SLOTS = 16;
    static constexpr size_t SLOT_DOUBLES = 96 * 96;
    double *pinned = nullptr;
    double *pinned_dl = nullptr;  // small downloads land here (pinned, so the copy is asynchronous)
    int upload_count = 0;

    Solver(Ctx &cc, int k, int m_max)
        : c(cc), s(cc.stream), D(cc.ndet), K(k), mmax(m_max), Vb(cc.dw.Vb), Wb(cc.dw.Wb), T(cc.dw.T),
          Wn(cc.dw.Wn), small(cc.dw.small), partial(cc.dw.partial), nrm(cc.dw.nrm), X32(cc.dw.X32),
          S32(cc.dw.S32), guess_idx(cc.dw.guess_idx), argv(cc.dw.argv), argi(cc.dw.argi), xfin(cc.dw.xfin),
          signbuf(cc.dw.signbuf) {
        nblocks = (mmax + K - 1) / K;
        const size_t bsz = (size_t)D * K;
        Vb.ensure(bsz * nblocks);
        Wb.ensure(bsz * nblocks);
        T.ensure(bsz);
        Wn.ensure(bsz);
        V = Mat{Vb.p, K, (int64_t)bsz};
        W = Mat{Wb.p, K, (int64_t)bsz};
        Tm = Mat{T.p, K, (int64_t)bsz};
        Wnm = Mat{Wn.p, K, (int64_t)bsz};
        small.ensure(96 * 96 * 2 + 4096);
        nblk_gram = gram_blocks_for(D);
        partial.ensure(std::max<size_t>((size_t)nblk_gram * 96 * 16, 2048 * 2 * 16) + 4096);  // gram / k_ritz partials
        nrm.ensure(64);
        HQ_CHECK(hipMemsetAsync(Vb.p, 0, sizeof(double) * bsz * nblocks, s));
        HQ_CHECK(hipMemsetAsync(Wb.p, 0, sizeof(double) * bsz * nblocks, s));
        HQ_CHECK(hipMemsetAsync(T.p, 0, sizeof(double) * bsz, s));
        HQ_CHECK(hipMemsetAsync(Wn.p, 0, sizeof(double) * bsz, s));
        if (!c.dw.pinned)
            HQ_CHECK(hipHostMalloc((void **)&c.dw.pinned, sizeof(double) * SLOTS * SLOT_DOUBLES,
                                   hipHostMallocDefault));
        pinned = c.dw.pinned;
        if (!c.dw.pinned_dl)
            HQ_CHECK(hipHostMalloc((void **)&c.dw.pinned_dl, sizeof(double) * SLOT_DOUBLES, hipHostMallocDefault));
        pinned_dl = c.dw.pinned_dl;
    }
    ~Solver() {
        (void)hipStreamSynchronize(s);  // the staging ring is free for the next solve
        for (auto e : evs) (void)hipEventDestroy(e);
    }

    // small.p regions: [0, 96*96) gram outputs / Y, [96*96, 2*96*96) coefficient uploads
    double *scratch_a() { return small.p; }
    double *scratch_b() { return small.p + 96 * 96; }
    double *scratch_c() { return small.p + 2 * 96 * 96; }  // [0, 16) column norms, [64] gate flag
    int *pass2_count() { return reinterpret_cast<int *>(scratch_c() + 65); }

    void gram(Mat A, int ma, Mat B, int nb, double *out, const int *gate = nullptr) {
        launch_gram(s, D, nblk_gram, A, ma, B, nb, partial.p, out, gate);
    }

    std::vector<double> gram_host(Mat A, int ma, Mat B, int nb) {
        gram(A, ma, B, nb, scratch_a());
        return download(scratch_a(), (size_t)ma * nb);
    }

    // n doubles of device memory to the host (through the pinned landing area;
    // the wait polls the stream)
    std::vector<double> download(const double *src, size_t n) {
        if (n > SLOT_DOUBLES) throw Error(HINQS_E_UNSUPPORTED, "small download too large");
        HQ_CHECK(hipMemcpyAsync(pinned_dl, src, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        wait_stream(s);
        return std::vector<double>(pinned_dl, pinned_dl + n);
    }

    // Out[:, 0:nc] = beta Out + alpha A[:, 0:m] Bs (m x nc row-major, device);
    // A has K columns per block.
    void tsmm(Mat A, int m, const double *Bs, int nc, double alpha, double beta, Mat Out,
              const int *gate = nullptr) {
        if (m <= 0 || nc <= 0) return;
        if (nc > 32) throw Error(HINQS_E_UNSUPPORTED, "tsmm width");
        if (m > 96) throw Error(HINQS_E_UNSUPPORTED, "tsmm depth");
        if (A.kb != K) throw Error(HINQS_E_UNSUPPORTED, "tsmm column block");
        const int64_t ntiles = (D + 15) / 16;
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((ntiles + 3) / 4, 2048));
        dim3 g(grid), b(256);
        if (nc <= 16) {
            if (m <= 48) hipLaunchKernelGGL((k_tsmm<1, 12>), g, b, 0, s, D, m, A, Bs, nc, alpha, beta, Out, gate);
            else hipLaunchKernelGGL((k_tsmm<1, 24>), g, b, 0, s, D, m, A, Bs, nc, alpha, beta, Out, gate);
        } else {
            if (m <= 48) hipLaunchKernelGGL((k_tsmm<2, 12>), g, b, 0, s, D, m, A, Bs, nc, alpha, beta, Out, gate);
            else hipLaunchKernelGGL((k_tsmm<2, 24>), g, b, 0, s, D, m, A, Bs, nc, alpha, beta, Out, gate);
        }
        HQ_LAUNCH_CHECK();
    }

    // Copied through a pinned staging slot, so the host vector may be released
    // on return without waiting; a slot is reused only after SLOTS further
    // uploads, and every SLOTS-th upload waits for the stream first.
    void upload_small(const std::vector<double> &h, double *dst) {
        if (h.size() > SLOT_DOUBLES) throw Error(HINQS_E_UNSUPPORTED, "small upload too large");
        if (++upload_count % SLOTS == 0) wait_stream(s);
        double *slot = pinned + (size_t)(upload_count % SLOTS) * SLOT_DOUBLES;
        std::copy(h.begin(), h.end(), slot);
        HQ_CHECK(hipMemcpyAsync(dst, slot, sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
    }

    // Sum of the sigma launch times recorded so far (waits for the last one).
    void collect_sigma_times() {
        if (evs.empty()) return;
        HQ_CHECK(hipEventSynchronize(evs.back()));
        for (size_t i = 0; i + 1 < evs.size(); i += 2) {
            float ms = 0.f;
            HQ_CHECK(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
            ms_sigma += ms;
        }
        for (auto e : evs) (void)hipEventDestroy(e);
        evs.clear();
    }

    // Point Tm / Wnm at the place for new columns [m, m + K).
    void bind_new(int m) {
        const size_t bsz = (size_t)D * K;
        direct = m % K == 0 && m / K < nblocks;
        if (direct) {
            Tm = Mat{V.p + (size_t)(m / K) * bsz, K, (int64_t)bsz};
            Wnm = Mat{W.p + (size_t)(m / K) * bsz, K, (int64_t)bsz};
        } else {
            Tm = Mat{T.p, K, (int64_t)bsz};
            Wnm = Mat{Wn.p, K, (int64_t)bsz};
        }
    }
    // After Tm and Wnm hold kept new columns: move them to columns
    // [m, m + kept) of V and W unless they were formed there.
    void place_new(int kept, int m) {
        if (direct && Tm.p == V.p + (size_t)(m / K) * D * K && m % K == 0) return;
        put_columns(Tm.p, kept, V, m);
        put_columns(Wnm.p, kept, W, m);
    }

    void put_columns(const double *src, int nc, Mat dst, int c0) {
        const int64_t n = D * K;
        hipLaunchKernelGGL(k_put_columns, dim3(grid_for(n, 256)), dim3(256), 0, s, D, src, K, nc, dst, c0);
        HQ_LAUNCH_CHECK();
    }

    // out = H X for a contiguous ndet x K block X (columns >= nc are zero).
    void apply_h(const double *X, int nc, bool fp32, double *out) {
        hipEvent_t e0, e1;
        HQ_CHECK(hipEventCreate(&e0));
        evs.push_back(e0);
        HQ_CHECK(hipEventCreate(&e1));
        evs.push_back(e1);
        HQ_CHECK(hipEventRecord(e0, s));
        if (!fp32) {
            sigma_sorted(c, K, X, K, out, K, HINQS_FP64, s);
        } else {
            X32.ensure((size_t)D * K);
            S32.ensure((size_t)D * K);
            const int64_t n = D * K;
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, n, X, X32.p);
            HQ_LAUNCH_CHECK();
            sigma_offdiag_fp32(c, K, X32.p, S32.p, s);
            hipLaunchKernelGGL(k_fp32_finish, dim3(grid_for(n, 256)), dim3(256), 0, s, n, K, S32.p, c.diag.p, X,
                               out);
            HQ_LAUNCH_CHECK();
        }
        HQ_CHECK(hipEventRecord(e1, s));
        ++sigma_blocks;
        sigma_columns += nc;
    }

    // Symmetric orthonormalization of T[:, 0:kept] in place: S T^T T S = Z
    // diag(w) Z^T (S = diag(sc)), T <- T S Z_k w_k^(-1/2) over the eigenvalues
    // w_k > drop, largest first; the unused columns of T are cleared.  Returns
    // the number kept (0: none) and their smallest eigenvalue in wmin.
    int sym_orth(int kept, const std::vector<double> &sc, double drop, double &wmin) {
        double *Zd = scratch_b();  // K x K
        std::vector<double> g = gram_host(Tm, kept, Tm, kept);
        for (int a = 0; a < kept; ++a)
            for (int b = a; b < kept; ++b) {
                const double v = sc[a] * sc[b] * 0.5 * (g[(size_t)a * kept + b] + g[(size_t)b * kept + a]);
                g[(size_t)a * kept + b] = g[(size_t)b * kept + a] = v;
            }
        std::vector<double> w, Z;
        small_sym_eig(kept, g, w, Z);
        std::vector<int> keep;
        for (int j = kept - 1; j >= 0; --j)  // largest first
            if (std::isfinite(w[j]) && w[j] > drop) keep.push_back(j);
        const int nk = (int)keep.size();
        if (nk == 0) return 0;
        wmin = w[keep.back()];
        // K x K transform: rows >= kept and columns >= nk are zero
        std::vector<double> Zk((size_t)K * K, 0.0);
        for (int a = 0; a < kept; ++a)
            for (int q = 0; q < nk; ++q)
                Zk[(size_t)a * K + q] = sc[a] * Z[(size_t)a * kept + keep[q]] / std::sqrt(w[keep[q]]);
        upload_small(Zk, Zd);
        tsmm(Tm, K, Zd, K, 1.0, 0.0, Tm);
        return nk;
    }

    // Orthonormalize the columns of T against V[:, 0:m] and within T; returns
    // the number of kept directions, left in T[:, 0:kept] (other columns
    // zeroed).  scale[q] (host, K entries) is 1/||T[:, q]|| for the columns to
    // keep and 0 for those to discard; nullptr = the initial block (the first
    // n columns, scales from T^T T).  One projection pass against V, a second
    // only when the first left less than half of some column's norm (decided
    // on the device), so T is orthogonal to V to a few ulps; then symmetric
    // orthonormalization of the unit-scaled block.  Corrections drop
    // eigen-directions with eigenvalue <= ORTH_DROP (less than a tenth of
    // their norm outside span(V) and the other new directions): the transform
    // then amplifies rounding at most tenfold and needs no second round.  The
    // initial block keeps everything above 1e-14 instead, since a warm-start
    // guess can lie almost inside the span of the unit vectors that join it
    // and its own direction must survive, and repeats the orthonormalization
    // (eigenvalues > 1e-4) when the first kept one below 1e-2.
    int orthonormalize(int m, int n, const double *scale) {
        double *C = scratch_a();  // m x K
        const bool initial = scale == nullptr;
        std::vector<double> sc(K, 0.0);
        if (!initial) {
            for (int q = 0; q < K; ++q) sc[q] = scale[q];
        } else {
            std::vector<double> g = gram_host(Tm, n, Tm, n);
            for (int q = 0; q < n; ++q) {
                const double d = g[(size_t)q * n + q];
                if (std::isfinite(d) && d > 0.0) sc[q] = 1.0 / std::sqrt(d);
            }
        }
        int kept = 0;  // columns that may hold a direction
        for (int q = 0; q < K; ++q)
            if (sc[q] > 0.0) kept = q + 1;
        if (kept == 0) return 0;
        if (m > 0) {
            gram(V, m, Tm, kept, C);
            tsmm(V, m, C, kept, -1.0, 1.0, Tm);
            // the second pass runs only when the device gate asks for it
            std::vector<double> tn2(K, 0.0);
            for (int q = 0; q < kept; ++q)
                if (sc[q] > 0.0) tn2[q] = 1.0 / (sc[q] * sc[q]);
            upload_small(tn2, scratch_c());
            int *gate = reinterpret_cast<int *>(scratch_c() + 64);
            hipLaunchKernelGGL(k_proj_gate, dim3(1), dim3(64), 0, s, (const double *)C, m, kept,
                               (const double *)scratch_c(), gate, pass2_count());
            HQ_LAUNCH_CHECK();
            gram(V, m, Tm, kept, C, gate);
            tsmm(V, m, C, kept, -1.0, 1.0, Tm, gate);
        }
        double wmin = 0.0;
        int nk = sym_orth(kept, sc, initial ? 1e-14 : ORTH_DROP, wmin);
        if (nk > 0 && initial && wmin < 1e-2) nk = sym_orth(nk, std::vector<double>(K, 1.0), 1e-4, wmin);
        return nk;
    }

    void lowest_diag_indices(int n, int32_t *dev_idx) {
        unsigned nblk = (unsigned)std::min<int64_t>(grid_for(D, 256), 1024);
        argv.ensure(nblk);
        argi.ensure(nblk);
        for (int r = 0; r < n; ++r) {
            hipLaunchKernelGGL(k_argmin_partial, dim3(nblk), dim3(256), 0, s, D, c.diag.p, dev_idx, r,
                               argv.p, argi.p);
            HQ_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_argmin_final, dim3(1), dim3(256), 0, s, (int)nblk, argv.p, argi.p,
                               dev_idx, r);
            HQ_LAUNCH_CHECK();
        }
    }

    // x = V y0 -> normalized, gauge-fixed, scattered to caller order (or sorted).
    void finalize(int m, const std::vector<double> &y0, double *out, bool sorted) {
        xfin.ensure(D);
        signbuf.ensure(1);
        upload_small(y0, scratch_b());
        Mat X{xfin.p, 1, (int64_t)D};
        tsmm(V, m, scratch_b(), 1, 1.0, 0.0, X);
        std::vector<double> nn = gram_host(X, 1, X, 1);
        double scale = nn[0] > 0 ? 1.0 / std::sqrt(nn[0]) : 1.0;
        unsigned nblk = (unsigned)std::min<int64_t>(grid_for(D, 256), 1024);
        argv.ensure(nblk);
        argi.ensure(nblk);
        hipLaunchKernelGGL(k_absmax_partial, dim3(nblk), dim3(256), 0, s, D, xfin.p, argv.p, argi.p);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(64), 0, s, (int)nblk, argv.p, argi.p, xfin.p,
                           signbuf.p);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_finalize, dim3(grid_for(D, 256)), dim3(256), 0, s, D, xfin.p, scale,
                           signbuf.p, sorted ? (const int32_t *)nullptr : c.perm.p, out);
        HQ_LAUNCH_CHECK();
        HQ_CHECK(hipStreamSynchronize(s));
    }
};

template <int KK>
void launch_ritz(Solver &S, int m, const double *Yd, const double *thd, double floor_, int nroots,
                 unsigned grid) {
    if (m <= 48)
        hipLaunchKernelGGL((k_ritz<KK, 12>), dim3(grid), dim3(256), 0, S.s, S.D, m, S.V, S.W, Yd, thd, S.c.diag.p,
                           floor_, nroots, S.Tm.p, S.partial.p);
    else
        hipLaunchKernelGGL((k_ritz<KK, 24>), dim3(grid), dim3(256), 0, S.s, S.D, m, S.V, S.W, Yd, thd, S.c.diag.p,
                           floor_, nroots, S.Tm.p, S.partial.p);
    HQ_LAUNCH_CHECK();
}

}  // namespace

int davidson(Ctx &c, const hinqs_opts &o, const double *guess, double *energy, double *coeffs,
             hinqs_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t D = c.ndet;
    const int K = o.block;
    if (K != 1 && K != 2 && K != 4 && K != 8 && K != 16)
        throw Error(HINQS_E_UNSUPPORTED, "block size must be 1, 2, 4, 8 or 16");
    int mmax = o.max_space > 0 ? o.max_space : 6 * K;
    if (mmax < 3 * K) mmax = 3 * K;
    if (mmax > 96) throw Error(HINQS_E_UNSUPPORTED, "max_space must be <= 96 (and >= 3 * block)");
    const bool sorted = (o.flags & HINQS_SORTED_ORDER) != 0;
    const int kroots = (int)std::min<int64_t>(K, D);  // roots tracked
    if (o.flags & HINQS_AUTOTUNE) {
        autotune_sigma(c, K, HINQS_FP64);
        if (o.precision == HINQS_SOLVE_MIXED) autotune_sigma(c, K, HINQS_FP32);
    }
    Solver S(c, K, mmax);
    HQ_CHECK(hipMemsetAsync(S.pass2_count(), 0, sizeof(int), S.s));
    hipStream_t s = c.stream;
    bool fp32 = (o.precision == HINQS_SOLVE_MIXED);
    int it_fp32 = 0, restarts = 0, iters = 0;
    const int maxit = o.max_iter > 0 ? o.max_iter : 200;
    const char *vb = std::getenv("HINQS_VERBOSE");
    const bool verbose = vb && vb[0] && vb[0] != '0';

    // ---- initial block: warm start + lowest-diagonal unit vectors
    S.bind_new(0);  // formed in place as the first column block of V
    S.guess_idx.ensure(K + 1);
    const int nunit = guess ? kroots - 1 : kroots;
    S.lowest_diag_indices(nunit, S.guess_idx.p);
    int n0 = 0;
    if (guess) {
        if (sorted) {
            hipLaunchKernelGGL(k_copy_column, dim3(grid_for(D, 256)), dim3(256), 0, s, D, guess, S.Tm.p, K, 0);
            HQ_LAUNCH_CHECK();
        } else {
            DBuf<double> tmp;
            tmp.ensure(D);
            gather_rows(s, guess, tmp.p, c.perm.p, D, 8);
            hipLaunchKernelGGL(k_copy_column, dim3(grid_for(D, 256)), dim3(256), 0, s, D, tmp.p, S.Tm.p, K, 0);
            HQ_LAUNCH_CHECK();
            HQ_CHECK(hipStreamSynchronize(s));
        }
        n0 = 1;
    }
    if (nunit > 0) {
        hipLaunchKernelGGL(k_unit_columns, dim3(grid_for(D, 256)), dim3(256), 0, s, D, S.Tm.p, K, n0, nunit,
                           S.guess_idx.p);
        HQ_LAUNCH_CHECK();
    }
    int m = S.orthonormalize(0, n0 + nunit, nullptr);
    if (m == 0) throw Error(HINQS_E_INVALID_ARG, "initial guess is zero");
    S.apply_h(S.Tm.p, m, fp32, S.Wnm.p);
    S.place_new(m, 0);

    std::vector<double> G((size_t)96 * 96, 0.0);  // host copy, leading dimension 96
    // G[0:mrows, c0:c0+nc] = V[:, 0:mrows]^T B with B holding those nc columns
    auto load_g_cols = [&](int c0, int nc, int mrows, Mat B) {
        std::vector<double> g = S.gram_host(S.V, mrows, B, nc);
        for (int a = 0; a < mrows; ++a)
            for (int b = 0; b < nc; ++b) G[(size_t)a * 96 + c0 + b] = g[(size_t)a * nc + b];
        // mirror into rows; symmetrize the new-new block
        for (int a = 0; a < mrows; ++a)
            for (int b = c0; b < c0 + nc; ++b) {
                if (a >= c0 && a < b) {
                    double v = 0.5 * (G[(size_t)a * 96 + b] + G[(size_t)b * 96 + a]);
                    G[(size_t)a * 96 + b] = G[(size_t)b * 96 + a] = v;
                } else if (a < c0) {
                    G[(size_t)b * 96 + a] = G[(size_t)a * 96 + b];
                }
            }
    };
    // full G of the current V, W (after a restart)
    auto load_g_all = [&](int mm) {
        std::fill(G.begin(), G.end(), 0.0);
        for (int b0 = 0; b0 < mm; b0 += K) {
            const int nb = std::min(K, mm - b0);
            std::vector<double> g = S.gram_host(S.V, mm, S.W.cols(b0), nb);
            for (int a = 0; a < mm; ++a)
                for (int b = 0; b < nb; ++b) G[(size_t)a * 96 + b0 + b] = g[(size_t)a * nb + b];
        }
        for (int a = 0; a < mm; ++a)
            for (int b = a + 1; b < mm; ++b) {
                double v = 0.5 * (G[(size_t)a * 96 + b] + G[(size_t)b * 96 + a]);
                G[(size_t)a * 96 + b] = G[(size_t)b * 96 + a] = v;
            }
    };
    // Replace the basis by V Q (m x q, host), recompute W and G.
    auto rotate_basis = [&](const std::vector<double> &Q, int q) {
        S.upload_small(Q, S.scratch_b());
        S.tsmm(S.V, m, S.scratch_b(), q, 1.0, 0.0, S.V);
        S.tsmm(S.W, m, S.scratch_b(), q, 1.0, 0.0, S.W);
        m = q;
        load_g_all(m);
        ++restarts;
    };
    load_g_cols(0, m, m, S.Wnm);

    std::vector<double> theta, Y, Yprev;  // Y: m x K row-major; Yprev: previous Ritz coefficients
    int mprev = 0;
    double res0 = INFINITY;
    double best_res_fp32 = INFINITY;
    int stall = 0;
    bool force_switch = false;
    bool converged = false;
    std::vector<double> y0;
    int nroots_eff = std::min(kroots, m);
    for (;;) {
        // ---- Rayleigh-Ritz
        std::vector<double> Gm((size_t)m * m);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) Gm[(size_t)a * m + b] = G[(size_t)a * 96 + b];
        std::vector<double> w, Z;
        small_sym_eig(m, Gm, w, Z);
        nroots_eff = std::min(kroots, m);
        theta.assign(K, 0.0);
        Y.assign((size_t)m * K, 0.0);
        for (int q = 0; q < nroots_eff; ++q) {
            theta[q] = w[q];
            for (int a = 0; a < m; ++a) Y[(size_t)a * K + q] = Z[(size_t)a * m + q];
        }
        y0.assign(m, 0.0);
        for (int a = 0; a < m; ++a) y0[a] = Z[(size_t)a * m + 0];
        // ---- residuals + preconditioned corrections (T, formed where V's new columns go)
        S.bind_new(m);
        double *Yd = S.scratch_a();
        double *thd = S.scratch_a() + 96 * 16;
        S.upload_small(Y, Yd);
        S.upload_small(theta, thd);
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(((D + 15) / 16 + 3) / 4, 2048));
        switch (K) {
            case 1: launch_ritz<1>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 2: launch_ritz<2>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 4: launch_ritz<4>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 8: launch_ritz<8>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            default: launch_ritz<16>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
        }
        hipLaunchKernelGGL(k_reduce_partials, dim3(2 * K), dim3(256), 0, s, S.partial.p, (int)grid, 2 * K,
                           S.nrm.p, (const int *)nullptr);
        HQ_LAUNCH_CHECK();
        std::vector<double> rt = S.download(S.nrm.p, 2 * K);
        std::vector<double> rn(rt.begin(), rt.begin() + K), tn2(rt.begin() + K, rt.end());
        for (double &x : rn) x = std::sqrt(std::max(0.0, x));
        res0 = rn[0];
        ++iters;
        if (fp32) ++it_fp32;
        if (verbose)
            std::fprintf(stderr, "[hinqs] it %3d m %2d %s theta0 %.14f |r0| %.3e |r1| %.3e\n", iters, m,
                         fp32 ? "fp32" : "fp64", theta[0], rn[0], nroots_eff > 1 ? rn[1] : 0.0);
        if (!fp32 && res0 <= o.tol) { converged = true; break; }
        if (!fp32 && m >= D) { converged = true; break; }  // whole space: Ritz pairs are exact
        if (iters >= maxit) break;
        // ---- mixed precision: switch to FP64 products
        bool do_switch = false;
        if (fp32) {
            if (res0 < best_res_fp32 * 0.7) { best_res_fp32 = res0; stall = 0; }
            else ++stall;
            // three iterations without progress mean the FP32 floor only once the
            // residual is small next to |theta|: far above it, Davidson residuals
            // also rise for a few iterations after a restart
            const bool near_floor = res0 < 1e-4 * std::max(1.0, std::fabs(theta[0]));
            if (res0 <= std::max(o.mixed_switch, o.tol) || (stall >= 3 && near_floor) || stall >= 8 ||
                force_switch || m >= D)
                do_switch = true;
        }
        if (do_switch) {
            // basis := current and previous Ritz vectors (as at a GD+k restart,
            // so the FP64 phase keeps the last step's direction); images
            // recomputed with FP64 products, one block product per K columns
            const int nprev = (mprev > 0 && !Yprev.empty()) ? nroots_eff : 0;
            const int qq = nroots_eff + nprev;
            std::vector<double> M((size_t)m * qq, 0.0);
            for (int a = 0; a < m; ++a) {
                for (int r = 0; r < nroots_eff; ++r) M[(size_t)a * qq + r] = Y[(size_t)a * K + r];
                if (a < mprev)
                    for (int r = 0; r < nprev; ++r)
                        M[(size_t)a * qq + nroots_eff + r] = Yprev[(size_t)a * nroots_eff + r];
            }
            int q = 0;
            std::vector<double> Q = small_orth(m, qq, M, 1e-8, q);
            S.upload_small(Q, S.scratch_b());
            S.tsmm(S.V, m, S.scratch_b(), q, 1.0, 0.0, S.V);
            m = q;
            fp32 = false;
            // V's first column blocks now hold the q <= 2K basis vectors
            const size_t bsz = (size_t)D * K;
            for (int b0 = 0; b0 < q; b0 += K)
                S.apply_h(S.V.p + (size_t)(b0 / K) * bsz, std::min(K, q - b0), false, S.W.p + (size_t)(b0 / K) * bsz);
            load_g_all(m);
            ++restarts;
            Yprev.clear();
            mprev = 0;
            continue;  // fresh Rayleigh-Ritz with FP64 images
        }
        // ---- which roots get a correction (the others are scaled to zero)
        std::vector<double> tscale(K, 0.0);
        int nadd = 0;
        for (int q = 0; q < nroots_eff; ++q)
            if (rn[q] > o.tol && tn2[q] > 0.0 && std::isfinite(tn2[q])) {
                tscale[q] = 1.0 / std::sqrt(tn2[q]);
                ++nadd;
            }
        if (nadd == 0 && tn2[0] > 0.0 && std::isfinite(tn2[0])) {
            tscale[0] = 1.0 / std::sqrt(tn2[0]);
            nadd = 1;
        }
        nadd = std::max(nadd, 1);
        // ---- restart (GD+k): keep current and previous Ritz vectors
        std::vector<double> Ycur((size_t)m * nroots_eff);
        for (int a = 0; a < m; ++a)
            for (int r = 0; r < nroots_eff; ++r) Ycur[(size_t)a * nroots_eff + r] = Y[(size_t)a * K + r];
        if (m + nadd > mmax) {
            const int nprev = (mprev > 0 && !Yprev.empty()) ? nroots_eff : 0;
            const int qq = nroots_eff + nprev;
            std::vector<double> M((size_t)m * qq, 0.0);
            for (int a = 0; a < m; ++a) {
                for (int r = 0; r < nroots_eff; ++r) M[(size_t)a * qq + r] = Ycur[(size_t)a * nroots_eff + r];
                if (a < mprev)
                    for (int r = 0; r < nprev; ++r)
                        M[(size_t)a * qq + nroots_eff + r] = Yprev[(size_t)a * nroots_eff + r];
            }
            int q = 0;
            std::vector<double> Q = small_orth(m, qq, M, 1e-8, q);
            const int qfull = q;
            if (q + nadd > mmax) q = std::max(nroots_eff, mmax - nadd);  // keep the current Ritz vectors
            std::vector<double> Qk((size_t)m * q);
            for (int a = 0; a < m; ++a)
                for (int r = 0; r < q; ++r) Qk[(size_t)a * q + r] = Q[(size_t)a * qfull + r];
            // current Ritz coefficients in the new basis: Q^T Ycur
            std::vector<double> Yn((size_t)q * nroots_eff, 0.0);
            for (int r = 0; r < q; ++r)
                for (int cc = 0; cc < nroots_eff; ++cc) {
                    double d = 0.0;
                    for (int a = 0; a < m; ++a) d += Qk[(size_t)a * q + r] * Ycur[(size_t)a * nroots_eff + cc];
                    Yn[(size_t)r * nroots_eff + cc] = d;
                }
            rotate_basis(Qk, q);
            Ycur.swap(Yn);
        }
        int kept = S.orthonormalize(m, K, tscale.data());
        if (kept == 0) {
            if (!fp32) break;  // no new direction: report the current Ritz pair, not converged
            force_switch = true;  // FP32 images cannot resolve further directions: refine in FP64
            --iters;
            if (it_fp32 > 0) --it_fp32;
            continue;
        }
        S.apply_h(S.Tm.p, kept, fp32, S.Wnm.p);
        S.place_new(kept, m);
        load_g_cols(m, kept, m + kept, S.Wnm);
        Yprev.swap(Ycur);
        mprev = m;
        m += kept;
    }
    *energy = theta.empty() ? 0.0 : theta[0];
    S.finalize(m, y0, coeffs, sorted);
    if (st) {
        st->iterations = iters;
        st->iterations_fp32 = it_fp32;
        st->sigma_blocks = S.sigma_blocks;
        st->sigma_columns = S.sigma_columns;
        st->restarts = restarts;
        st->residual = res0;
        S.collect_sigma_times();
        st->ms_sigma = S.ms_sigma;
        st->nnz = c.nnz;
        int np2 = 0;
        HQ_CHECK(hipMemcpyAsync(&np2, S.pass2_count(), sizeof(int), hipMemcpyDeviceToHost, S.s));
        HQ_CHECK(hipStreamSynchronize(S.s));
        st->second_passes = np2;
        st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? HINQS_OK : HINQS_E_NOT_CONVERGED;
}

void gram_product(Ctx &c, int64_t nrows, const double *A, int lda, int ma, const double *B, int ldb,
                  int nb, double *G) {
    const int nblk = gram_blocks_for(nrows);
    DBuf<double> partial;
    partial.ensure((size_t)nblk * ma * nb);
    launch_gram(c.stream, nrows, nblk, Mat{const_cast<double *>(A), lda, 0}, ma,
                Mat{const_cast<double *>(B), ldb, 0}, nb, partial.p, G);
    HQ_CHECK(hipStreamSynchronize(c.stream));
}

}  // namespace hinqs
