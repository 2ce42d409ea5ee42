// Block Davidson eigensolver for the lowest eigenpair of H_B (paper Sec. 2.2,
// Step 3: "diagonalized with a Davidson eigensolver", warm-started from the
// previous eigenvector).
//
// Basis V and images W = H V live in HBM as ndet x ld row-major arrays (one
// determinant's coefficients contiguous), in sorted determinant order, so a
// block of new columns is directly the strided X of the sigma kernel.
// Per iteration:
//   G[:, new] = V^T W_new          FP64 MFMA (v_mfma_f64_16x16x4f64) partials,
//                                  reduced in a fixed order (deterministic)
//   Rayleigh-Ritz on G             host cyclic Jacobi (m <= 96)
//   T = (W y - theta V y) / (theta - H_ii)   fused Ritz/residual/preconditioner
//   CGS2 of T against V, then symmetric orthonormalization of T (eigen-
//   decomposition of T^T T, nearly dependent directions dropped)
//   W_new = H T                    sigma kernel
// with a thick restart to the current Ritz vectors when the space is full.
// MIXED precision: FP32 sigma products while the residual is above a switch
// threshold (or stalls), then a restart on the Ritz vectors, W recomputed
// with FP64 sigma, and FP64 iterations to the requested tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "common.hpp"

namespace hinqs {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_BLOCK = 256;
constexpr int GRAM_MAX_BLOCKS = 1024;

// partial[blk][a][b] = sum over this block's rows of A[i][a] * B[i][b]
// (a < ma <= 16*MT, b < nb <= 16).  MFMA operand layout (16x16x4 f64):
// lane l supplies A_mat[l%16][l/16] and B_mat[l/16][l%16] and receives
// D[l/16 + 4r][l%16] in element r of its 4-wide accumulator.
template <int MT>
__global__ __launch_bounds__(GRAM_BLOCK) void k_gram(int64_t nrows, const double *__restrict__ A,
                                                     int lda, int ma, const double *__restrict__ B,
                                                     int ldb, int nb, int64_t rows_per_wave,
                                                     double *__restrict__ partial) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * (GRAM_BLOCK / 64) + wave;
    const int64_t r0 = gw * rows_per_wave;
    const int64_t r1 = min(nrows, r0 + rows_per_wave);
    const int col = lane & 15, kk = lane >> 4;
    dbl4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    const bool bok = col < nb;

    for (int64_t i = r0; i < r1; i += 4) {
        const int64_t row = i + kk;
        const bool rok = row < r1;
        const double bv = (rok && bok) ? B[row * ldb + col] : 0.0;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const int a = t * 16 + col;
            const double av = (rok && a < ma) ? A[row * lda + a] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
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

// out[e] = sum_blk partial[blk][e], fixed order.
__global__ void k_sum_partials(const double *partial, int nblk, int n, double *out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * n + e];
    out[e] = s;
}

// Fused Ritz vector, residual, norm and diagonal preconditioner for KK roots:
//   r_c = W y_c - theta_c V y_c,   T[:, c] = r_c / clamp(theta_c - H_ii)
// partial[blk][c] = sum over the block's rows of r_c^2.  Rows of V and W are
// staged through LDS in 16-column chunks (coalesced loads); thread (r, c)
// owns row r of the tile and root c.
constexpr int JC = 16;

template <int KK>
__global__ __launch_bounds__(256) void k_ritz(int64_t nrows, int m, const double *__restrict__ V,
                                              const double *__restrict__ W, int ld,
                                              const double *__restrict__ Y,
                                              const double *__restrict__ theta,
                                              const double *__restrict__ diag, double floor_,
                                              int nroots, double *__restrict__ T, int ldt,
                                              double *__restrict__ partial) {
    constexpr int ROWS = 256 / KK;
    __shared__ double sV[ROWS * JC];
    __shared__ double sW[ROWS * JC];
    __shared__ double sY[96 * KK];
    __shared__ double red[256];
    for (int t = threadIdx.x; t < m * KK; t += 256) sY[t] = Y[t];
    const int r = threadIdx.x / KK, c = threadIdx.x % KK;
    const double th = theta[c];
    double nrm = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * ROWS; i0 < nrows; i0 += (int64_t)gridDim.x * ROWS) {
        double x = 0.0, w = 0.0;
        for (int j0 = 0; j0 < m; j0 += JC) {
            const int jn = min(JC, m - j0);
            __syncthreads();
            for (int f = threadIdx.x; f < ROWS * JC; f += 256) {
                const int rr = f / JC, j = f % JC;
                const int64_t row = i0 + rr;
                const bool ok = row < nrows && j < jn;
                sV[f] = ok ? V[row * ld + j0 + j] : 0.0;
                sW[f] = ok ? W[row * ld + j0 + j] : 0.0;
            }
            __syncthreads();
            for (int j = 0; j < jn; ++j) {
                const double y = sY[(j0 + j) * KK + c];
                x += sV[r * JC + j] * y;
                w += sW[r * JC + j] * y;
            }
        }
        const int64_t row = i0 + r;
        if (row < nrows && c < nroots) {
            const double res = w - th * x;
            nrm += res * res;
            double den = th - diag[row];
            if (fabs(den) < floor_) den = den < 0.0 ? -floor_ : floor_;
            T[row * ldt + c] = res / den;
        }
    }
    __syncthreads();
    red[threadIdx.x] = nrm;
    __syncthreads();
    if (threadIdx.x < KK) {
        double s = 0.0;
        for (int q = 0; q < ROWS; ++q) s += red[q * KK + threadIdx.x];
        partial[(int64_t)blockIdx.x * KK + threadIdx.x] = s;
    }
}

// Out[i, c] = beta * Out[i, c] + alpha * sum_j A[i, j] B[j, c],  c < nc <= NC, j < m <= 96.
// Every global read of a tile's A rows precedes (across a barrier) every
// write of the tile, so Out may alias A (in-place basis rotation, nc <= m).
template <int NC>
__global__ __launch_bounds__(256) void k_tsmm(int64_t nrows, int m, const double *A, int lda,
                                              const double *__restrict__ B, int nc, double alpha,
                                              double beta, double *Out, int ldo) {
    constexpr int ROWS = 256 / NC;
    __shared__ double sA[ROWS * JC];
    __shared__ double sB[96 * NC];
    for (int t = threadIdx.x; t < m * NC; t += 256) {
        const int j = t / NC, cc = t % NC;
        sB[t] = cc < nc ? B[j * nc + cc] : 0.0;
    }
    const int r = threadIdx.x / NC, c = threadIdx.x % NC;
    for (int64_t i0 = (int64_t)blockIdx.x * ROWS; i0 < nrows; i0 += (int64_t)gridDim.x * ROWS) {
        double acc = 0.0;
        for (int j0 = 0; j0 < m; j0 += JC) {
            const int jn = min(JC, m - j0);
            __syncthreads();
            for (int f = threadIdx.x; f < ROWS * JC; f += 256) {
                const int rr = f / JC, j = f % JC;
                const int64_t row = i0 + rr;
                sA[f] = (row < nrows && j < jn) ? A[row * lda + j0 + j] : 0.0;
            }
            __syncthreads();
            for (int j = 0; j < jn; ++j) acc += sA[r * JC + j] * sB[(j0 + j) * NC + c];
        }
        __syncthreads();  // all reads of this tile's A rows are done
        const int64_t row = i0 + r;
        if (row < nrows && c < nc) {
            double *o = Out + row * ldo + c;
            *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * acc;
        }
    }
}

// Columns [c0, c0+nc) of an ndet x ld array set to zero, except unit entries
// at rows idx[c] (idx may be null).
__global__ void k_unit_columns(int64_t nrows, double *V, int ld, int c0, int nc, const int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int c = 0; c < nc; ++c) V[i * ld + c0 + c] = (idx && idx[c] == i) ? 1.0 : 0.0;
}

__global__ void k_copy_column(int64_t nrows, const double *src, double *V, int ld, int c) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    V[i * ld + c] = src[i];
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
        if (threadIdx.x < s) {
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
        if (threadIdx.x < s) {
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
        if (threadIdx.x < s) {
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

// X32[i, c] = (float) V[i, c0 + c] for c < nc, zero for nc <= c < K32.
__global__ void k_to_f32(int64_t nrows, const double *V, int ld, int c0, int nc, float *X, int K32) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * K32) return;
    int64_t i = t / K32;
    int c = (int)(t % K32);
    X[t] = c < nc ? (float)V[i * ld + c0 + c] : 0.0f;
}

__global__ void k_from_f32(int64_t nrows, const float *S, int K32, double *W, int ld, int c0, int nc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * K32) return;
    int64_t i = t / K32;
    int c = (int)(t % K32);
    if (c < nc) W[i * ld + c0 + c] = (double)S[t];
}

// G (ma x nb) = A^T B over nrows rows: MFMA partials per block, then a
// fixed-order reduction.  partial must hold nblk * ma * nb doubles.
void launch_gram(hipStream_t s, int64_t nrows, int nblk, const double *A, int lda, int ma,
                 const double *B, int ldb, int nb, double *partial, double *out) {
    if (nb > 16 || ma > 96 || ma < 1 || nb < 1) throw Error(HINQS_E_UNSUPPORTED, "Gram block shape");
    int64_t waves = (int64_t)nblk * (GRAM_BLOCK / 64);
    int64_t rpw = (nrows + waves - 1) / waves;
    rpw = (rpw + 3) / 4 * 4;
    const int mt = (ma + 15) / 16;
    dim3 g(nblk), b(GRAM_BLOCK);
    switch (mt) {
        case 1: hipLaunchKernelGGL(k_gram<1>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
        case 2: hipLaunchKernelGGL(k_gram<2>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
        case 3: hipLaunchKernelGGL(k_gram<3>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
        case 4: hipLaunchKernelGGL(k_gram<4>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
        case 5: hipLaunchKernelGGL(k_gram<5>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
        default: hipLaunchKernelGGL(k_gram<6>, g, b, 0, s, nrows, A, lda, ma, B, ldb, nb, rpw, partial); break;
    }
    HQ_LAUNCH_CHECK();
    const int n = ma * nb;
    hipLaunchKernelGGL(k_sum_partials, dim3((n + 255) / 256), dim3(256), 0, s, partial, nblk, n, out);
    HQ_LAUNCH_CHECK();
}

int gram_blocks_for(int64_t nrows) {
    int64_t waves = (nrows + 63) / 64;
    return (int)std::min<int64_t>(GRAM_MAX_BLOCKS, std::max<int64_t>(1, (waves + 3) / 4));
}

// ------------------------------------------------------------ host helpers

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

struct Solver {
    Ctx &c;
    hipStream_t s;
    int64_t D;
    int K;        // block size (compile-time kernel variant)
    int mmax;     // largest subspace
    int ld;       // leading dimension of V, W
    DBuf<double> V, W, T, small, partial, nrm;
    DBuf<float> X32, S32;
    DBuf<int32_t> guess_idx;
    DBuf<double> argv;
    DBuf<int64_t> argi;
    DBuf<double> xfin, signbuf;
    int nblk_gram = 1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double ms_sigma = 0.0;
    int sigma_blocks = 0, sigma_columns = 0;

    Solver(Ctx &cc, int k, int m_max) : c(cc), s(cc.stream), D(cc.ndet), K(k), mmax(m_max) {
        ld = mmax + K;
        if (ld % 2) ++ld;
        V.ensure((size_t)D * ld);
        W.ensure((size_t)D * ld);
        T.ensure((size_t)D * K);
        small.ensure(96 * 96 + 4096);
        nblk_gram = gram_blocks_for(D);
        partial.ensure(std::max<size_t>((size_t)nblk_gram * 96 * 16, 2048 * 16) + 4096);
        nrm.ensure(64);
        HQ_CHECK(hipMemsetAsync(V.p, 0, sizeof(double) * (size_t)D * ld, s));
        HQ_CHECK(hipMemsetAsync(W.p, 0, sizeof(double) * (size_t)D * ld, s));
        HQ_CHECK(hipMemsetAsync(T.p, 0, sizeof(double) * (size_t)D * K, s));
        HQ_CHECK(hipEventCreate(&ev0));
        HQ_CHECK(hipEventCreate(&ev1));
    }
    ~Solver() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    // G (ma x nb, row-major, device `out`) = A^T B over all rows.
    void gram(const double *A, int lda, int ma, const double *B, int ldb, int nb, double *out) {
        launch_gram(s, D, nblk_gram, A, lda, ma, B, ldb, nb, partial.p, out);
    }

    std::vector<double> gram_host(const double *A, int lda, int ma, const double *B, int ldb, int nb) {
        gram(A, lda, ma, B, ldb, nb, small.p);
        std::vector<double> h((size_t)ma * nb);
        HQ_CHECK(hipMemcpyAsync(h.data(), small.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        HQ_CHECK(hipStreamSynchronize(s));
        return h;
    }

    // Out[:, 0:nc] = beta Out + alpha A[:, 0:m] Bsmall (m x nc, device)
    void tsmm(const double *A, int lda, int m, const double *Bs, int nc, double alpha, double beta,
              double *Out, int ldo) {
        if (m <= 0 || nc <= 0) return;
        int NC = nc <= 1 ? 1 : nc <= 2 ? 2 : nc <= 4 ? 4 : nc <= 8 ? 8 : 16;
        if (nc > 16) throw Error(HINQS_E_UNSUPPORTED, "tsmm width");
        if (m > 96) throw Error(HINQS_E_UNSUPPORTED, "tsmm depth");
        const size_t lds = 0;
        int rows = 256 / NC;
        int64_t tiles = (D + rows - 1) / rows;
        unsigned grid = (unsigned)std::min<int64_t>(tiles, 4096);
        dim3 g(grid), b(256);
        switch (NC) {
            case 1: hipLaunchKernelGGL(k_tsmm<1>, g, b, lds, s, D, m, A, lda, Bs, nc, alpha, beta, Out, ldo); break;
            case 2: hipLaunchKernelGGL(k_tsmm<2>, g, b, lds, s, D, m, A, lda, Bs, nc, alpha, beta, Out, ldo); break;
            case 4: hipLaunchKernelGGL(k_tsmm<4>, g, b, lds, s, D, m, A, lda, Bs, nc, alpha, beta, Out, ldo); break;
            case 8: hipLaunchKernelGGL(k_tsmm<8>, g, b, lds, s, D, m, A, lda, Bs, nc, alpha, beta, Out, ldo); break;
            default: hipLaunchKernelGGL(k_tsmm<16>, g, b, lds, s, D, m, A, lda, Bs, nc, alpha, beta, Out, ldo); break;
        }
        HQ_LAUNCH_CHECK();
    }

    // Synchronous so the host vector may be released on return.
    void upload_small(const std::vector<double> &h, double *dst) {
        HQ_CHECK(hipMemcpyAsync(dst, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
        HQ_CHECK(hipStreamSynchronize(s));
    }

    // W[:, c0:c0+nc] = H V[:, c0:c0+nc]
    void apply_h(int c0, int nc, bool fp32) {
        HQ_CHECK(hipEventRecord(ev0, s));
        if (!fp32) {
            sigma_sorted(c, K, V.p + c0, ld, W.p + c0, ld, HINQS_FP64, s);
        } else {
            X32.ensure((size_t)D * K);
            S32.ensure((size_t)D * K);
            int64_t n = D * K;
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, D, V.p, ld, c0, nc,
                               X32.p, K);
            HQ_LAUNCH_CHECK();
            sigma_sorted(c, K, X32.p, K, S32.p, K, HINQS_FP32, s);
            hipLaunchKernelGGL(k_from_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, D, S32.p, K, W.p, ld,
                               c0, nc);
            HQ_LAUNCH_CHECK();
        }
        HQ_CHECK(hipEventRecord(ev1, s));
        HQ_CHECK(hipEventSynchronize(ev1));
        float ms = 0.f;
        HQ_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
        ms_sigma += ms;
        ++sigma_blocks;
        sigma_columns += nc;
    }

    // Orthonormalize T[:, 0:n] against V[:, 0:m] and within itself; returns the
    // number of kept directions, written to V[:, m : m+kept].  Columns are first
    // scaled to unit norm, so the thresholds below are relative: a direction is
    // dropped when less than 1e-7 of it lies outside span(V) and the other
    // new directions.
    int orthonormalize_into_v(int m, int n) {
        const int ldt = K;
        double *C = small.p;                   // m x n
        double *Zd = small.p + 96 * 96;        // n x n
        int kept = 0;
        {
            std::vector<double> g = gram_host(T.p, ldt, n, T.p, ldt, n);
            std::vector<int> nz;
            for (int q = 0; q < n; ++q) {
                double d = g[(size_t)q * n + q];
                if (std::isfinite(d) && d > 0.0) nz.push_back(q);
            }
            kept = (int)nz.size();
            if (kept == 0) return 0;
            std::vector<double> Dg((size_t)n * kept, 0.0);
            for (int q = 0; q < kept; ++q) Dg[(size_t)nz[q] * kept + q] = 1.0 / std::sqrt(g[(size_t)nz[q] * n + nz[q]]);
            upload_small(Dg, Zd);
            tsmm(T.p, ldt, n, Zd, kept, 1.0, 0.0, T.p, ldt);
        }
        for (int round = 0; round < 2; ++round) {
            if (m > 0) {
                for (int pass = 0; pass < 2; ++pass) {
                    gram(V.p, ld, m, T.p, ldt, kept, C);
                    tsmm(V.p, ld, m, C, kept, -1.0, 1.0, T.p, ldt);
                }
            }
            std::vector<double> g = gram_host(T.p, ldt, kept, T.p, ldt, kept);
            for (int a = 0; a < kept; ++a)
                for (int b = a + 1; b < kept; ++b) {
                    double v = 0.5 * (g[(size_t)a * kept + b] + g[(size_t)b * kept + a]);
                    g[(size_t)a * kept + b] = g[(size_t)b * kept + a] = v;
                }
            std::vector<double> w, Z;
            jacobi_eig(kept, g, w, Z);
            const double thresh = round == 0 ? 1e-14 : 1e-4;
            std::vector<int> keep;
            for (int j = kept - 1; j >= 0; --j)  // largest first
                if (std::isfinite(w[j]) && w[j] > thresh) keep.push_back(j);
            const int nk = (int)keep.size();
            if (nk == 0) return 0;
            std::vector<double> Zk((size_t)kept * nk);
            for (int a = 0; a < kept; ++a)
                for (int q = 0; q < nk; ++q)
                    Zk[(size_t)a * nk + q] = Z[(size_t)a * kept + keep[q]] / std::sqrt(w[keep[q]]);
            upload_small(Zk, Zd);
            tsmm(T.p, ldt, kept, Zd, nk, 1.0, 0.0, T.p, ldt);
            kept = nk;
        }
        // append
        std::vector<double> eye((size_t)kept * kept, 0.0);
        for (int q = 0; q < kept; ++q) eye[(size_t)q * kept + q] = 1.0;
        upload_small(eye, Zd);
        tsmm(T.p, ldt, kept, Zd, kept, 1.0, 0.0, V.p + m, ld);
        return kept;
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
        upload_small(y0, small.p);
        tsmm(V.p, ld, m, small.p, 1, 1.0, 0.0, xfin.p, 1);
        std::vector<double> nn = gram_host(xfin.p, 1, 1, xfin.p, 1, 1);
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
    hipLaunchKernelGGL(k_ritz<KK>, dim3(grid), dim3(256), 0, S.s, S.D, m, S.V.p, S.W.p, S.ld, Yd, thd,
                       S.c.diag.p, floor_, nroots, S.T.p, S.K, S.partial.p);
    HQ_LAUNCH_CHECK();
}

}  // namespace

int davidson(Ctx &c, const hinqs_opts &o, const double *guess, double *energy, double *coeffs,
             hinqs_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t D = c.ndet;
    int K = o.block;
    if (K != 1 && K != 2 && K != 4 && K != 8 && K != 16)
        throw Error(HINQS_E_UNSUPPORTED, "block size must be 1, 2, 4, 8 or 16");
    int mmax = o.max_space > 0 ? o.max_space : 4 * K;
    if (mmax < 2 * K) mmax = 2 * K;
    if (mmax + K > 96) throw Error(HINQS_E_UNSUPPORTED, "max_space + block must be <= 96");
    const bool sorted = (o.flags & HINQS_SORTED_ORDER) != 0;
    const int kroots = (int)std::min<int64_t>(K, D);  // roots tracked
    Solver S(c, K, mmax);
    hipStream_t s = c.stream;
    bool fp32 = (o.precision == HINQS_SOLVE_MIXED);
    int it_fp32 = 0, restarts = 0, iters = 0;

    // ---- initial block: warm start + lowest-diagonal unit vectors
    S.guess_idx.ensure(K + 1);
    int nunit = guess ? kroots - 1 : kroots;
    S.lowest_diag_indices(nunit, S.guess_idx.p);
    int n0 = 0;
    if (guess) {
        if (sorted) hipLaunchKernelGGL(k_copy_column, dim3(grid_for(D, 256)), dim3(256), 0, s, D, guess, S.T.p, K, 0);
        else {
            // gather caller-order guess into sorted order: T[i, 0] = guess[perm[i]]
            DBuf<double> tmp;
            tmp.ensure(D);
            gather_rows(s, guess, tmp.p, c.perm.p, D, 8);
            hipLaunchKernelGGL(k_copy_column, dim3(grid_for(D, 256)), dim3(256), 0, s, D, tmp.p, S.T.p, K, 0);
            HQ_CHECK(hipStreamSynchronize(s));
        }
        HQ_LAUNCH_CHECK();
        n0 = 1;
    }
    if (nunit > 0) {
        hipLaunchKernelGGL(k_unit_columns, dim3(grid_for(D, 256)), dim3(256), 0, s, D, S.T.p, K, n0, nunit,
                           S.guess_idx.p);
        HQ_LAUNCH_CHECK();
    }
    int m = S.orthonormalize_into_v(0, n0 + nunit);
    if (m == 0) throw Error(HINQS_E_INVALID_ARG, "initial guess is zero");
    S.apply_h(0, m, fp32);
    std::vector<double> G((size_t)96 * 96, 0.0);  // host copy, leading dimension 96
    auto load_g_block = [&](int c0, int nc, int mrows) {
        for (int b0 = c0; b0 < c0 + nc; b0 += 16) {
            int nb = std::min(16, c0 + nc - b0);
            std::vector<double> g = S.gram_host(S.V.p, S.ld, mrows, S.W.p + b0, S.ld, nb);
            for (int a = 0; a < mrows; ++a)
                for (int b = 0; b < nb; ++b) {
                    G[(size_t)a * 96 + b0 + b] = g[(size_t)a * nb + b];
                }
        }
        // mirror: new columns -> rows; symmetrize the new-new block
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
    load_g_block(0, m, m);

    std::vector<double> theta, Y;  // Y: m x K row-major
    double res0 = INFINITY;
    double best_res_fp32 = INFINITY;
    int stall = 0;
    bool converged = false;
    std::vector<double> y0;
    const int maxit = o.max_iter > 0 ? o.max_iter : 200;
    int nroots_eff = std::min(kroots, m);
    for (;;) {
        // ---- Rayleigh-Ritz
        std::vector<double> Gm((size_t)m * m);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) Gm[(size_t)a * m + b] = G[(size_t)a * 96 + b];
        std::vector<double> w, Z;
        jacobi_eig(m, Gm, w, Z);
        nroots_eff = std::min(kroots, m);
        theta.assign(K, 0.0);
        Y.assign((size_t)m * K, 0.0);
        for (int q = 0; q < nroots_eff; ++q) {
            theta[q] = w[q];
            for (int a = 0; a < m; ++a) Y[(size_t)a * K + q] = Z[(size_t)a * m + q];
        }
        y0.assign(m, 0.0);
        for (int a = 0; a < m; ++a) y0[a] = Z[(size_t)a * m + 0];
        // ---- residuals + preconditioned corrections
        double *Yd = S.small.p;
        double *thd = S.small.p + 96 * 16;
        S.upload_small(Y, Yd);
        S.upload_small(theta, thd);
        unsigned grid = (unsigned)std::min<int64_t>(grid_for(D, 256 / K), 2048);
        switch (K) {
            case 1: launch_ritz<1>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 2: launch_ritz<2>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 4: launch_ritz<4>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            case 8: launch_ritz<8>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
            default: launch_ritz<16>(S, m, Yd, thd, o.precond_floor, nroots_eff, grid); break;
        }
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, S.partial.p, (int)grid, K, S.nrm.p);
        HQ_LAUNCH_CHECK();
        std::vector<double> rn(K);
        HQ_CHECK(hipMemcpyAsync(rn.data(), S.nrm.p, sizeof(double) * K, hipMemcpyDeviceToHost, s));
        HQ_CHECK(hipStreamSynchronize(s));
        for (double &x : rn) x = std::sqrt(std::max(0.0, x));
        res0 = rn[0];
        ++iters;
        if (fp32) ++it_fp32;
        if (!fp32 && res0 <= o.tol) { converged = true; break; }
        if (m >= D) {  // the subspace is the whole space: Ritz pairs are exact
            converged = true;
            break;
        }
        if (iters >= maxit) break;
        // ---- mixed precision: switch to FP64 products
        bool do_switch = false;
        if (fp32) {
            if (res0 < best_res_fp32 * 0.7) { best_res_fp32 = res0; stall = 0; }
            else ++stall;
            if (res0 <= std::max(o.mixed_switch, o.tol) || stall >= 3) do_switch = true;
        }
        // ---- restart / switch: rotate V, W onto the current Ritz vectors
        int nadd = 0;
        std::vector<int> add;
        for (int q = 0; q < nroots_eff; ++q)
            if (rn[q] > o.tol) add.push_back(q);
        if (add.empty()) add.push_back(0);
        nadd = (int)add.size();
        if (do_switch || m + nadd > mmax) {
            int kk = nroots_eff;
            std::vector<double> Yk((size_t)m * kk);
            for (int a = 0; a < m; ++a)
                for (int q = 0; q < kk; ++q) Yk[(size_t)a * kk + q] = Y[(size_t)a * K + q];
            S.upload_small(Yk, S.small.p + 96 * 96);
            S.tsmm(S.V.p, S.ld, m, S.small.p + 96 * 96, kk, 1.0, 0.0, S.V.p, S.ld);
            if (do_switch) {
                fp32 = false;
                S.apply_h(0, kk, false);
            } else {
                S.tsmm(S.W.p, S.ld, m, S.small.p + 96 * 96, kk, 1.0, 0.0, S.W.p, S.ld);
            }
            m = kk;
            std::fill(G.begin(), G.end(), 0.0);
            load_g_block(0, m, m);
            ++restarts;
            if (do_switch) continue;  // fresh Rayleigh-Ritz with FP64 images
        }
        // compact T's columns to the unconverged roots
        if (nadd < nroots_eff) {
            std::vector<double> P((size_t)K * nadd, 0.0);
            for (int q = 0; q < nadd; ++q) P[(size_t)add[q] * nadd + q] = 1.0;
            S.upload_small(P, S.small.p + 96 * 96);
            S.tsmm(S.T.p, K, K, S.small.p + 96 * 96, nadd, 1.0, 0.0, S.T.p, K);
        }
        int kept = S.orthonormalize_into_v(m, nadd);
        if (kept == 0) {
            if (!fp32) break;  // no new direction: report the current Ritz pair, not converged
            // FP32 images cannot resolve further directions: refine in FP64
            std::vector<double> Yk((size_t)m * nroots_eff);
            for (int a = 0; a < m; ++a)
                for (int q = 0; q < nroots_eff; ++q) Yk[(size_t)a * nroots_eff + q] = Y[(size_t)a * K + q];
            S.upload_small(Yk, S.small.p + 96 * 96);
            S.tsmm(S.V.p, S.ld, m, S.small.p + 96 * 96, nroots_eff, 1.0, 0.0, S.V.p, S.ld);
            fp32 = false;
            m = nroots_eff;
            S.apply_h(0, m, false);
            std::fill(G.begin(), G.end(), 0.0);
            load_g_block(0, m, m);
            ++restarts;
            continue;
        }
        S.apply_h(m, kept, fp32);
        load_g_block(m, kept, m + kept);
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
        st->ms_sigma = S.ms_sigma;
        st->nnz = c.nnz;
        st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? HINQS_OK : HINQS_E_NOT_CONVERGED;
}

void gram_product(Ctx &c, int64_t nrows, const double *A, int lda, int ma, const double *B, int ldb,
                  int nb, double *G) {
    const int nblk = gram_blocks_for(nrows);
    DBuf<double> partial;
    partial.ensure((size_t)nblk * ma * nb);
    launch_gram(c.stream, nrows, nblk, A, lda, ma, B, ldb, nb, partial.p, G);
    HQ_CHECK(hipStreamSynchronize(c.stream));
}

}  // namespace hinqs
