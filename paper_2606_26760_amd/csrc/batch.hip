// Batched lowest-eigenpair solves of many independent instances: a family of
// problems such as the points of a potential-energy scan, each with its own
// orbital count, electron count, integrals and determinant set.  The paper
// (Sec. 2.2, Step 3) solves one instance by Davidson; its outlook names bond
// scans as the next use.  Every instance is solved by the same block Davidson
// method as the single-instance path (FP64, GD+k restart, CGS2 plus symmetric
// orthonormalization), but all of them advance together.
//
// Layout.  The instances are concatenated into one block-diagonal coupling
// matrix: instance b owns global rows inst_row[b] .. inst_row[b+1] (in its own
// sorted order) and its couplings point only inside that range, so one launch
// of the persistent sigma kernel applies every instance's H_B at once, with
// the coupling-balanced XCD row ranges recomputed on the device from the
// instances still running; rows of finished instances are skipped.  Dense
// tall-skinny work (Gram products, basis updates, Ritz vectors) runs over a
// chunk list: a chunk is a run of at most CH rows of one instance and one
// workgroup handles one chunk, so a single launch covers all instances however
// uneven their sizes.  The small dense problems (Rayleigh-Ritz eigenproblem,
// restart basis, block orthonormalization) run on the device, one workgroup
// per instance, so an iteration needs no host round trip.
//
// Schedule.  All instances use the same subspace size m at every iteration
// (K, 2K, ..., m_max, then a restart to 2K), so the launches of an iteration
// depend only on m: each distinct m is captured once as a hipGraph and
// replayed.  Converged instances raise a flag that every kernel checks; the
// host reads one counter per iteration to learn when all have finished.
#include <algorithm>
#include <map>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace hinqs {

struct BatchState {
    struct Meta {
        int norb, na, nb;
        int64_t ndet, nnz;
    };
    std::vector<Meta> meta;
    std::vector<int64_t> row_off{0}, nz_off{0};  // row / coupling offsets of the instances (host)
    Ctx scratch;            // per-instance build; its buffers are reused by the next instance
    Ctx g;                  // block-diagonal couplings of all instances (arrays grow geometrically)
    DBuf<int32_t> perm;     // global sorted row -> caller index inside its instance
    DBuf<int32_t> row_inst; // global row -> instance
    DBuf<int64_t> inst_row; // row offsets (ninst + 1), device copy
    bool dirty = true;      // inst_row and the XCD row ranges need a refresh
    // launch shape of the batched iteration (chunk rows of the tall-skinny
    // kernels, threads of the Rayleigh-Ritz kernel), per block-size index;
    // tuned[k] says the shape was timed for the current instances
    struct Shape {
        int chunk = 2048;
        int rr_threads = 1024;
        double ms_per_it = 0.0;
    };
    Shape shape[5];
    std::string tuned_key[5];
};

namespace {

constexpr int MS = 64;             // largest subspace
constexpr int KB = 16;             // largest block; leading dimension of per-instance K-wide arrays
constexpr int PSTRIDE = MS * KB;   // doubles per chunk of a Gram partial
constexpr int RSTRIDE = KB;        // doubles per chunk of a residual partial
constexpr int NT = 256;            // threads of the per-instance kernels
constexpr int GRAM_UNROLL_B = 4;

struct Chunk {
    int64_t r0;
    int32_t n;
    int32_t inst;
};

// Per-instance solver state in device memory (passed by value).
struct BDev {
    int nb;
    const int32_t *inst_chunk;  // chunks of instance b: inst_chunk[b] .. inst_chunk[b+1]
    int32_t *done;              // 0 running, 1 converged, 2 no new direction
    int32_t *skip2;             // done, or the first projection pass left every column at least half its norm
    int32_t *iters, *mfin, *valid;  // valid: [b][MS] basis columns in use
    double *G;                  // [b][MS][MS] V^T H V
    double *Y;                  // [b][MS][KB] Ritz coefficients of the current basis
    double *theta;              // [b][KB]
    double *Q;                  // [b][MS][2K] restart transform (leading dimension 2K)
    double *C;                  // [b][MS][KB] projection coefficients
    double *Z;                  // [b][KB][KB] block orthonormalization transform
    double *scl;                // [b][KB] column scales of the new block
    double *energy, *resid;     // [b]
};

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Sum over a workgroup of B threads; every thread receives the same value.
template <int B = NT>
__device__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < B / 64; ++w) s += red[w];
    return s;
}

// Sum over one wave, broadcast from lane 0 so every lane holds the same value.
__device__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return __shfl(v, 0);
}

// Parallel cyclic Jacobi eigensolver for the symmetric n x n matrix A (LDS,
// leading dimension LD, n <= MAXN <= 64).  Rotations follow a round-robin
// pairing: each round pairs every index once, the n/2 disjoint rotations are
// computed from the current matrix and applied together (columns, then
// rows); each thread steps through its elements' (pair, index) positions
// by a fixed stride, so a round costs only LDS traffic and one rotation per
// pair.  Sweeps stop when the off-diagonal mass falls below 1e-32 of the
// Frobenius norm.  On return A's diagonal holds the eigenvalues and row j of
// ZT the eigenvector belonging to A[j][j].
template <int LD, int MAXN, int B = NT>
__device__ void block_jacobi(int n, double *A, double *ZT, int *pp, int *pq, double *pc, double *ps,
                             double *red) {
    constexpr int MAXE = ((MAXN + 1) / 2 * MAXN + B - 1) / B;  // elements per thread and phase
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += B) {
        const int i = e / n, j = e % n;
        ZT[i * LD + j] = i == j ? 1.0 : 0.0;
    }
    double f = 0.0;
    for (int e = tid; e < n * n; e += B) {
        const double x = A[(e / n) * LD + e % n];
        f += x * x;
    }
    const double fro = block_sum<B>(f, red);
    if (n < 2) return;
    const int ne = n + (n & 1), np = ne / 2, nr = ne - 1;
    // element e = tid + u B of a phase: column phase (pair e % np, row e / np,
    // so neighbouring threads hit different banks), row phase (pair e / n,
    // column e % n, contiguous rows); both advance by B per slot
    const int ck0 = tid % np, cj0 = tid / np, cstep_k = B % np, cstep_j = B / np;
    const int rj0 = tid % n, rk0 = tid / n, rstep_j = B % n, rstep_k = B / n;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double o = 0.0;
        for (int e = tid; e < n * n; e += B) {
            const int i = e / n, j = e % n;
            if (i < j) o += A[i * LD + j] * A[i * LD + j];
        }
        const double off = block_sum<B>(o, red);
        if (off == 0.0 || off <= 1e-32 * fro) break;
        for (int r = 0; r < nr; ++r) {
            if (tid < np) {
                int a, b;
                if (tid == 0) {
                    a = r;
                    b = ne - 1;
                } else {
                    a = r + tid;
                    if (a >= nr) a -= nr;
                    b = r - tid;
                    if (b < 0) b += nr;
                }
                const int p = min(a, b), q = max(a, b);
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * LD + q];
                    if (apq != 0.0) {
                        const double th = (A[q * LD + q] - A[p * LD + p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                pp[tid] = p;
                pq[tid] = (q < n && s != 0.0) ? q : -1;  // -1: nothing to rotate
                pc[tid] = c;
                ps[tid] = s;
            }
            __syncthreads();
            for (int u = 0, k = ck0, j = cj0; u < MAXE && j < n; ++u) {  // columns p, q
                const int q = pq[k];
                if (q >= 0) {
                    const int o1 = j * LD + pp[k], o2 = j * LD + q;
                    const double c = pc[k], s = ps[k];
                    const double x1 = A[o1], x2 = A[o2];
                    A[o1] = c * x1 - s * x2;
                    A[o2] = s * x1 + c * x2;
                }
                k += cstep_k;
                j += cstep_j;
                if (k >= np) {
                    k -= np;
                    ++j;
                }
            }
            __syncthreads();
            for (int u = 0, k = rk0, j = rj0; u < MAXE && k < np; ++u) {  // rows p, q and eigenvector rows
                const int q = pq[k];
                if (q >= 0) {
                    const int o1 = pp[k] * LD + j, o2 = q * LD + j;
                    const double c = pc[k], s = ps[k];
                    const double x1 = A[o1], x2 = A[o2], z1 = ZT[o1], z2 = ZT[o2];
                    A[o1] = c * x1 - s * x2;
                    A[o2] = s * x1 + c * x2;
                    ZT[o1] = c * z1 - s * z2;
                    ZT[o2] = s * z1 + c * z2;
                }
                j += rstep_j;
                k += rstep_k;
                if (j >= n) {
                    j -= n;
                    ++k;
                }
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------- chunked dense kernels

// partial[chunk][a * nb + b] = sum over the chunk's rows of A(i, a) B(i, b),
// a < ma <= 16 MT, b < nb <= 16, with FP64 MFMA (16x16x4): lane l supplies
// A_mat[l%16][l/16] and B_mat[l/16][l%16] and receives D[l/16 + 4r][l%16].
// The four waves split the chunk's rows.
template <int MT>
__global__ __launch_bounds__(256) void k_bgram(const Chunk *__restrict__ chunks, const int32_t *__restrict__ done,
                                               Mat A, int ma, Mat B, int nb, double *__restrict__ partial) {
    const Chunk ch = chunks[blockIdx.x];
    if (done[ch.inst]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = ((ch.n + 3) / 4 + 3) / 4 * 4;  // rows per wave, a multiple of 4
    const int64_t end = ch.r0 + ch.n;
    const int64_t r0 = ch.r0 + (int64_t)wave * per;
    const int64_t r1 = min(end, r0 + per);
    const int col = lane & 15, kk = lane >> 4;
    dbl4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    const bool bok = col < nb;
    for (int64_t i = r0; i < r1; i += 4 * GRAM_UNROLL_B) {
        double bv[GRAM_UNROLL_B], av[GRAM_UNROLL_B][MT];
#pragma unroll
        for (int u = 0; u < GRAM_UNROLL_B; ++u) {
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
        for (int u = 0; u < GRAM_UNROLL_B; ++u)
#pragma unroll
            for (int t = 0; t < MT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[u], acc[t], 0, 0, 0);
    }
    __shared__ double red[4][MT][64][4];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave][t][lane][r] = acc[t][r];
    __syncthreads();
    for (int e = threadIdx.x; e < MT * 256; e += 256) {
        const int t = e / 256, rem = e % 256, ln = rem / 4, r = rem % 4;
        const double s = red[0][t][ln][r] + red[1][t][ln][r] + red[2][t][ln][r] + red[3][t][ln][r];
        const int a = t * 16 + (ln >> 4) + 4 * r;
        const int b = ln & 15;
        if (a < ma && b < nb) partial[(int64_t)blockIdx.x * PSTRIDE + a * nb + b] = s;
    }
}

// Out(i, c) = beta Out(i, c) + alpha sum_{j<m} A(i, j) B_inst[j][c] for the
// rows of each chunk, with B_inst = Bs + inst * bstride (leading dimension
// ldb), c < nc <= 16 NT, m <= 4 STEPS.  FP64 MFMA (16x16x4) on 16-row tiles of
// the chunk, the four waves taking every fourth tile: for k-step s lane l
// supplies A(r0 + l%16, 4s + l/16), holds B_inst[4s + l/16][16t + l%16] in
// registers and receives rows r0 + l/16 + 4r of column 16t + l%16.  A tile's
// rows are all read before any is written, so Out may alias A.
template <int NT, int STEPS>
__global__ __launch_bounds__(256) void k_btsmm(const Chunk *__restrict__ chunks, const int32_t *__restrict__ done,
                                               int m, Mat A, const double *__restrict__ Bs, int bstride, int ldb,
                                               int nc, double alpha, double beta, Mat Out) {
    const Chunk ch = chunks[blockIdx.x];
    if (done[ch.inst]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    const double *B = Bs + (int64_t)ch.inst * bstride;
    double bv[STEPS][NT];
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 4 * s + kk, c = 16 * t + col;
            bv[s][t] = (j < m && c < nc) ? B[j * ldb + c] : 0.0;
        }
    const int nsteps = (m + 3) / 4;
    const int64_t end = ch.r0 + ch.n;
    for (int64_t r0 = ch.r0 + 16 * wave; r0 < end; r0 += 64) {
        const int64_t ra = r0 + col;
        const bool rok = ra < end;
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
                if (row >= end) continue;
                double *o = Out.at(row, c);
                *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * acc[t][r];
            }
        }
    }
}

// Ritz vectors, residuals and preconditioned corrections of every root of
// each chunk's instance, with per-chunk partial sums of r_c^2:
//   r_c = W y_c - theta_c V y_c,  T[:, c] = r_c / clamp(theta_c - H_ii),
// V y and W y on FP64 MFMA with the tile layout of k_btsmm (m <= 4 STEPS).
template <int KK, int STEPS>
__global__ __launch_bounds__(256) void k_britz(const Chunk *__restrict__ chunks, BDev st, int m, Mat V, Mat W,
                                               const double *__restrict__ diag, double floor_,
                                               double *__restrict__ T, double *__restrict__ rpart) {
    const Chunk ch = chunks[blockIdx.x];
    if (st.done[ch.inst]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kk = lane >> 4;
    const double *Yb = st.Y + (int64_t)ch.inst * MS * KB;
    double yv[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        const int j = 4 * s + kk;
        yv[s] = (j < m && col < KK) ? Yb[j * KB + col] : 0.0;
    }
    const double th = col < KK ? st.theta[ch.inst * KB + col] : 0.0;
    const int nsteps = (m + 3) / 4;
    const int64_t end = ch.r0 + ch.n;
    double rn2 = 0.0;
    for (int64_t r0 = ch.r0 + 16 * wave; r0 < end; r0 += 64) {
        const int64_t ra = r0 + col;
        const bool rok = ra < end;
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
        if (col < KK) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + kk + 4 * r;
                if (row >= end) continue;
                const double res = aw[r] - th * ax[r];
                double den = th - diag[row];
                if (fabs(den) < floor_) den = den < 0.0 ? -floor_ : floor_;
                rn2 += res * res;
                T[row * KK + col] = res / den;
            }
        }
    }
    __shared__ double red[4][64];
    red[wave][lane] = rn2;
    __syncthreads();
    if ((int)threadIdx.x < KK) {
        const int c = threadIdx.x;
        double rs = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int q = 0; q < 4; ++q) rs += red[w][c + 16 * q];
        rpart[(int64_t)blockIdx.x * RSTRIDE + c] = rs;
    }
}

// ------------------------------------------------------- per-instance kernels

// Sum of the chunk partials of instance b, element e (fixed order).
__device__ inline double chunk_sum(const double *__restrict__ part, int stride, int c0, int c1, int e) {
    // eight independent loads in flight (a plain loop waits for each load in
    // turn); fixed order, so the sum is reproducible
    constexpr int U = 8;
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    int ch = c0;
    for (; ch + U <= c1; ch += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = part[(int64_t)(ch + u) * stride + e];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += v[u];
    }
    for (; ch < c1; ++ch) acc[0] += part[(int64_t)ch * stride + e];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

constexpr int RR_LD = MS + 1;
// Threads of the Rayleigh-Ritz kernel (RR_NT in {256, 512, 1024}, chosen by
// the batch tuner): its Jacobi rounds are bound by LDS traffic and latency,
// so a full 16-wave workgroup per instance usually beats fewer waves despite
// the barriers (at m = 48: 1024 threads 0.55 ms, 256 threads 0.82 ms, one
// wave 3.0 ms).
constexpr size_t rr_lds_bytes(int nt) {
    return sizeof(double) * (2 * MS * RR_LD + 2 * MS * KB + 2 * KB * KB + KB + nt / 64 + MS) +
           sizeof(int) * (2 * MS + 2 * MS);
}

// Rayleigh-Ritz of instance b at subspace size m: the last K columns of
// G = V^T W arrive as chunk partials (gpart) and are folded into G; the valid
// columns are diagonalized; theta and Y receive the lowest K Ritz pairs.
// restart (m == m_max): the basis is replaced by an orthonormal basis Q of
// the current and the previous Ritz vectors (GD+k); Q (for the tall update),
// Q^T G Q, Q^T Y and the validity of the new columns are written.
template <int KK, int RR_NT>
__global__ __launch_bounds__(RR_NT) void k_brr(BDev st, int m, int restart, const double *__restrict__ gpart) {
    const int b = blockIdx.x;
    if (st.done[b]) return;
    extern __shared__ double lds[];
    double *A = lds;                       // MS x RR_LD
    double *ZT = A + MS * RR_LD;           // MS x RR_LD
    double *gn = ZT + MS * RR_LD;          // MS x KK: new columns, rows 0..m-1
    double *Yn = gn + MS * KB;             // MS x KK
    double *Y2 = Yn + MS * KB;             // 2KK x KK
    double *th = Y2 + 2 * KB * KB;         // KK
    double *red = th + KB;                 // RR_NT/64
    double *pc = red + RR_NT / 64;            // MS/2
    double *ps = pc + MS / 2;              // MS/2
    int *pp = (int *)(ps + MS / 2);        // MS/2
    int *pq = pp + MS / 2;                 // MS/2
    int *vidx = pq + MS / 2;               // MS
    int *misc = vidx + MS;                 // [0] nv, [1] kept mask
    const int tid = threadIdx.x;
    const int base = m - KK;
    const int c0 = st.inst_chunk[b], c1 = st.inst_chunk[b + 1];
    for (int e = tid; e < m * KK; e += RR_NT) gn[e] = chunk_sum(gpart, PSTRIDE, c0, c1, e);
    if (tid < 64) {  // valid columns, ascending, by one wave (m <= MS = 64)
        const bool ok = tid < m && st.valid[b * MS + tid] != 0;
        const uint64_t bal = __ballot(ok);
        if (ok) vidx[__popcll(bal & ((1ull << tid) - 1ull))] = tid;
        if (tid == 0) misc[0] = __popcll(bal);
    }
    __syncthreads();
    const int nv = misc[0];
    double *Gb = st.G + (int64_t)b * MS * MS;
    // element (r, c) of the current G: old block from memory, new columns from gn
    auto gval = [&](int r, int c) -> double {
        if (r < base && c < base) return Gb[r * MS + c];
        if (r < base) return gn[r * KK + (c - base)];
        if (c < base) return gn[c * KK + (r - base)];
        return 0.5 * (gn[r * KK + (c - base)] + gn[c * KK + (r - base)]);
    };
    for (int e = tid; e < nv * nv; e += RR_NT) {
        const int i = e / nv, j = e % nv;
        A[i * RR_LD + j] = gval(vidx[i], vidx[j]);
    }
    __syncthreads();
    block_jacobi<RR_LD, MS, RR_NT>(nv, A, ZT, pp, pq, pc, ps, red);
    __syncthreads();
    for (int e = tid; e < MS * KK; e += RR_NT) Yn[e] = 0.0;
    if (tid < KK) th[tid] = 0.0;
    __syncthreads();
    // lowest KK eigenpairs in ascending order (ties: lower index first)
    for (int j = tid; j < nv; j += RR_NT) {
        const double d = A[j * RR_LD + j];
        int rank = 0;
        for (int i = 0; i < nv; ++i) {
            const double x = A[i * RR_LD + i];
            rank += (x < d || (x == d && i < j)) ? 1 : 0;
        }
        if (rank < KK) {
            th[rank] = d;
            for (int i = 0; i < nv; ++i) Yn[vidx[i] * KK + rank] = ZT[j * RR_LD + i];
        }
    }
    __syncthreads();
    double *Yb = st.Y + (int64_t)b * MS * KB;
    if (tid < KB) st.theta[b * KB + tid] = tid < KK ? th[tid] : 0.0;
    if (!restart) {
        for (int e = tid; e < MS * KB; e += RR_NT) {
            const int a = e / KB, q = e % KB;
            Yb[e] = (a < m && q < KK) ? Yn[a * KK + q] : 0.0;
        }
        for (int e = tid; e < m * KK; e += RR_NT) {
            const int r = e / KK, c = base + e % KK;
            const double v = gval(r, c);
            Gb[r * MS + c] = v;
            if (r < base) Gb[c * MS + r] = v;
        }
        return;
    }
    // ---- GD+k restart
    constexpr int Q2 = 2 * KK;
    double *Qs = A;            // m x Q2
    double *GQ = A + MS * Q2;  // m x Q2
    double *Gs = ZT;           // m x m, leading dimension RR_LD
    for (int e = tid; e < m * m; e += RR_NT) {
        const int r = e / m, c = e % m;
        Gs[r * RR_LD + c] = gval(r, c);
    }
    if (tid < 64) {  // modified Gram-Schmidt, twice, by wave 0; lane a owns row a
        const int a = tid;
        unsigned kept = 0u;
        for (int c = 0; c < Q2; ++c) {
            double v = 0.0;
            if (a < m) v = c < KK ? Yn[a * KK + c] : Yb[a * KB + (c - KK)];
            const double n0 = sqrt(wave_sum(v * v));
            bool keep = n0 > 0.0;
            if (keep) {
                for (int pass = 0; pass < 2; ++pass)
                    for (int u = 0; u < c; ++u) {
                        if (!((kept >> u) & 1u)) continue;
                        const double qu = a < m ? Qs[a * Q2 + u] : 0.0;
                        const double d = wave_sum(qu * v);
                        v -= d * qu;
                    }
                const double n1 = sqrt(wave_sum(v * v));
                keep = n1 > 1e-8 * n0;
                if (keep) v /= n1;
            }
            if (a < m) Qs[a * Q2 + c] = keep ? v : 0.0;
            if (keep) kept |= 1u << c;
        }
        if (a == 0) misc[1] = (int)kept;
    }
    __syncthreads();
    const unsigned kept = (unsigned)misc[1];
    for (int e = tid; e < Q2 * KK; e += RR_NT) {  // Ritz coefficients in the new basis
        const int i = e / KK, q = e % KK;
        double s = 0.0;
        for (int a = 0; a < m; ++a) s += Qs[a * Q2 + i] * Yn[a * KK + q];
        Y2[e] = s;
    }
    for (int e = tid; e < m * Q2; e += RR_NT) {
        const int r = e / Q2, j = e % Q2;
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += Gs[r * RR_LD + c] * Qs[c * Q2 + j];
        GQ[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < Q2 * Q2; e += RR_NT) {
        const int i = e / Q2, j = e % Q2;
        double s1 = 0.0, s2 = 0.0;
        for (int a = 0; a < m; ++a) {
            s1 += Qs[a * Q2 + i] * GQ[a * Q2 + j];
            s2 += Qs[a * Q2 + j] * GQ[a * Q2 + i];
        }
        Gb[i * MS + j] = 0.5 * (s1 + s2);
    }
    double *Qb = st.Q + (int64_t)b * MS * 2 * KB;
    for (int e = tid; e < m * Q2; e += RR_NT) Qb[e] = Qs[e];
    for (int c = tid; c < MS; c += RR_NT) st.valid[b * MS + c] = (c < Q2 && ((kept >> c) & 1u)) ? 1 : 0;
    for (int e = tid; e < MS * KB; e += RR_NT) {
        const int a = e / KB, q = e % KB;
        Yb[e] = (a < Q2 && q < KK) ? Y2[a * KK + q] : 0.0;
    }
}

// After the Ritz step and the first Gram product [V T]^T T: residual norms,
// convergence of the lowest root, the projection coefficients C = V^T T and
// the unit scales of the corrections that are kept (roots with ||r|| > tol).
template <int KK>
__global__ __launch_bounds__(NT) void k_bpost_first(BDev st, int m, double tol, const double *__restrict__ rpart,
                                                    const double *__restrict__ gpart) {
    const int b = blockIdx.x;
    if (st.done[b]) {
        if (threadIdx.x == 0) st.skip2[b] = 1;
        return;
    }
    __shared__ double rn2[KK];
    __shared__ double g1[MS * KK];
    const int tid = threadIdx.x;
    const int c0 = st.inst_chunk[b], c1 = st.inst_chunk[b + 1];
    if (tid < KK) rn2[tid] = chunk_sum(rpart, RSTRIDE, c0, c1, tid);
    for (int e = tid; e < (m + KK) * KK; e += NT) g1[e] = chunk_sum(gpart, PSTRIDE, c0, c1, e);
    __syncthreads();
    const double r0 = sqrt(fmax(0.0, rn2[0]));
    if (tid == 0) {
        st.iters[b] += 1;
        st.resid[b] = r0;
        st.skip2[b] = 1;
        if (r0 <= tol) {
            st.done[b] = 1;
            st.energy[b] = st.theta[b * KB];
            st.mfin[b] = m;
        }
    }
    if (r0 <= tol) return;
    if (tid < 64) {  // wave 0: column scales, and whether the projection needs a second pass
        bool need = false;
        if (tid < KK) {
            const double rq = sqrt(fmax(0.0, rn2[tid]));
            const double nq = g1[(m + tid) * KK + tid];
            const bool keep = rq > tol && nq > 0.0 && isfinite(nq);
            st.scl[b * KB + tid] = keep ? 1.0 / sqrt(nq) : 0.0;
            if (keep) {  // ||T_q||^2 - ||(V^T T)_q||^2 < ||T_q||^2 / 4 (NaN counts as less)
                double c2 = 0.0;
                for (int a = 0; a < m; ++a) c2 += g1[a * KK + tid] * g1[a * KK + tid];
                need = !(nq - c2 >= 0.25 * nq);
            }
        }
        const bool any = __ballot(need) != 0ull;
        if (tid == 0) st.skip2[b] = any ? 0 : 1;
    }
    double *Cb = st.C + (int64_t)b * MS * KB;
    for (int e = tid; e < m * KK; e += NT) Cb[(e / KK) * KB + e % KK] = g1[e];
}

// C = V^T T from the chunk partials.
template <int KK>
__global__ __launch_bounds__(NT) void k_bpost_proj(BDev st, const int32_t *__restrict__ gate, int m,
                                                   const double *__restrict__ gpart) {
    const int b = blockIdx.x;
    if (gate[b]) return;
    const int c0 = st.inst_chunk[b], c1 = st.inst_chunk[b + 1];
    double *Cb = st.C + (int64_t)b * MS * KB;
    for (int e = threadIdx.x; e < m * KK; e += NT) Cb[(e / KK) * KB + e % KK] = chunk_sum(gpart, PSTRIDE, c0, c1, e);
}

// Symmetric orthonormalization of the new block T from g = T^T T: with
// S = diag(scl) (unit columns, dropped roots zero), S g S = Z diag(w) Z^T and
// T <- T S Z_k w_k^(-1/2) over the eigenvalues w_k > ORTH_DROP, largest
// first (the transform amplifies what is left of span(V) at most tenfold, so
// one round suffices).  No kept direction: the instance stops (its current
// Ritz pair is the result).  The new basis columns are marked valid.
template <int KK>
__global__ __launch_bounds__(NT) void k_bpost_orth(BDev st, const int32_t *__restrict__ gate, int m,
                                                   const double *__restrict__ gpart) {
    constexpr double thresh = ORTH_DROP;
    const int b = blockIdx.x;
    if (gate[b]) return;
    constexpr int LD = KK + 1;
    __shared__ double A[KK * LD], ZT[KK * LD], sc[KK], red[NT / 64];
    __shared__ double pc[KK], ps[KK];
    __shared__ int pp[KK], pq[KK], nk_s;
    const int tid = threadIdx.x;
    const int c0 = st.inst_chunk[b], c1 = st.inst_chunk[b + 1];
    if (tid < KK) sc[tid] = st.scl[b * KB + tid];
    for (int e = tid; e < KK * KK; e += NT) ZT[(e / KK) * LD + e % KK] = chunk_sum(gpart, PSTRIDE, c0, c1, e);
    __syncthreads();
    for (int e = tid; e < KK * KK; e += NT) {
        const int i = e / KK, j = e % KK;
        A[i * LD + j] = sc[i] * sc[j] * 0.5 * (ZT[i * LD + j] + ZT[j * LD + i]);
    }
    __syncthreads();
    block_jacobi<LD, KK>(KK, A, ZT, pp, pq, pc, ps, red);
    __syncthreads();
    double *Zb = st.Z + (int64_t)b * KB * KB;
    for (int e = tid; e < KB * KB; e += NT) Zb[e] = 0.0;
    if (tid == 0) {
        int n = 0;
        for (int j = 0; j < KK; ++j) {
            const double w = A[j * LD + j];
            n += (isfinite(w) && w > thresh) ? 1 : 0;
        }
        nk_s = n;
    }
    __syncthreads();
    if (tid < KK) {
        const int j = tid;
        const double w = A[j * LD + j];
        if (isfinite(w) && w > thresh) {
            int rank = 0;
            for (int i = 0; i < KK; ++i) {
                const double x = A[i * LD + i];
                if (isfinite(x) && x > thresh && (x > w || (x == w && i < j))) ++rank;
            }
            const double inv = 1.0 / sqrt(w);
            for (int a = 0; a < KK; ++a) Zb[a * KB + rank] = sc[a] * ZT[j * LD + a] * inv;
        }
    }
    const int nk = nk_s;
    if (tid == 0) {
        if (nk == 0) {
            st.done[b] = 2;
            st.energy[b] = st.theta[b * KB];
            st.mfin[b] = m;
        }
    }
    if (tid < KK) st.valid[b * MS + m + tid] = tid < nk ? 1 : 0;
}

// Coupling-balanced XCD row ranges over the instances still running: range x
// starts at the first row whose running-coupling prefix reaches x/8 of the
// total.  One wave: the instances' coupling counts are read 64 at a time and
// summed with shuffles, lane x (1..7) finds the instance where its target is
// crossed from the chunk's prefix sums, then binary-searches the row in it.
__global__ void k_bbalance(int nb, const int64_t *__restrict__ inst_row, const int64_t *__restrict__ rowptr,
                           const int32_t *__restrict__ done, int64_t *__restrict__ ranges) {
    const int lane = threadIdx.x;  // 64 threads
    const int64_t N = inst_row[nb];
    auto count = [&](int b) -> int64_t {
        return (b < nb && !done[b]) ? rowptr[inst_row[b + 1]] - rowptr[inst_row[b]] : 0;
    };
    int64_t tot = 0;
    for (int b0 = 0; b0 < nb; b0 += 64) {
        int64_t v = count(b0 + lane);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        tot += v;
    }
    const int64_t t = tot / 8 * lane + (tot % 8) * lane / 8;  // used by lanes 1..7
    int bsel = -1;
    int64_t before = 0, acc = 0;
    for (int b0 = 0; b0 < nb; b0 += 64) {
        const int64_t nz = count(b0 + lane);
        int64_t incl = nz;  // inclusive prefix over the chunk
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        int k = -1;  // first instance of the chunk that crosses this lane's target
        for (int q = 0; q < 64; ++q) {
            const int64_t iq = __shfl(incl, q), nq = __shfl(nz, q);
            if (k < 0 && nq > 0 && acc + iq > t) k = q;
        }
        const int ks = k < 0 ? 0 : k;
        const int64_t ik = __shfl(incl, ks), nk = __shfl(nz, ks);
        if (bsel < 0 && k >= 0) {
            bsel = b0 + k;
            before = acc + ik - nk;
        }
        acc += __shfl(incl, 63);
    }
    if (lane >= 1 && lane <= 7) {
        int64_t res = N;
        if (bsel >= 0) {
            int64_t lo = inst_row[bsel], hi = inst_row[bsel + 1];
            const int64_t want = t - before + rowptr[inst_row[bsel]];
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (rowptr[mid] < want) lo = mid + 1;
                else hi = mid;
            }
            res = lo;
        }
        ranges[lane] = res;
    }
    if (lane == 0) ranges[0] = 0;
    if (lane == 8) ranges[8] = N;
}

__global__ void k_bcount(int nb, const int32_t *__restrict__ done, int32_t *__restrict__ out) {
    __shared__ int red[256];
    int n = 0;
    for (int b = threadIdx.x; b < nb; b += 256) n += done[b] != 0 ? 1 : 0;
    red[threadIdx.x] = n;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_bvalid_init(int nb, int K, int32_t *valid) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)nb * MS) valid[t] = (int)(t % MS) < K ? 1 : 0;
}

// Initial block of instance b: unit vectors at its K lowest diagonal elements
// (lexicographic (value, row) order), written into V's first column block
// (which is zero on entry).
template <int KK>
__global__ __launch_bounds__(256) void k_binit(const int64_t *__restrict__ inst_row, const double *__restrict__ diag,
                                               double *__restrict__ V0) {
    // one pass: each thread keeps the KK smallest (value, row) pairs of its
    // strided rows in ascending order, then KK block-wide minima pop them
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = inst_row[b], r1 = inst_row[b + 1];
    __shared__ int64_t chosen[KK];
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    __shared__ int owner;
    auto less = [](double v, int64_t i, double w, int64_t j) { return v < w || (v == w && i < j); };
    double tv[KK];
    int64_t ti[KK];
#pragma unroll
    for (int u = 0; u < KK; ++u) {
        tv[u] = INFINITY;
        ti[u] = INT64_MAX;
    }
    for (int64_t i = r0 + tid; i < r1; i += 256) {
        const double v = diag[i];
        if (!less(v, i, tv[KK - 1], ti[KK - 1])) continue;
#pragma unroll
        for (int u = KK - 1; u >= 0; --u) {  // insert, shifting larger entries down
            if (less(v, i, tv[u], ti[u])) {
                if (u == 0 || !less(v, i, tv[u - 1], ti[u - 1])) {
                    tv[u] = v;
                    ti[u] = i;
                } else {
                    tv[u] = tv[u - 1];
                    ti[u] = ti[u - 1];
                }
            }
        }
    }
    for (int r = 0; r < KK; ++r) {
        sv[tid] = tv[0];
        si[tid] = ti[0];
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st && less(sv[tid + st], si[tid + st], sv[tid], si[tid])) {
                sv[tid] = sv[tid + st];
                si[tid] = si[tid + st];
            }
            __syncthreads();
        }
        if (tid == 0) chosen[r] = si[0];
        if (ti[0] == si[0] && si[0] != INT64_MAX) owner = tid;  // rows are distinct: one owner
        __syncthreads();
        if (si[0] != INT64_MAX && tid == owner) {  // pop the head
#pragma unroll
            for (int u = 0; u + 1 < KK; ++u) {
                tv[u] = tv[u + 1];
                ti[u] = ti[u + 1];
            }
            tv[KK - 1] = INFINITY;
            ti[KK - 1] = INT64_MAX;
        }
        __syncthreads();
    }
    if (tid < KK && chosen[tid] >= r0 && chosen[tid] < r1) V0[chosen[tid] * KK + tid] = 1.0;
}

// Final vector of every instance: x = V y_0 over the instance's final
// subspace, with per-chunk partials of ||x||^2 and of the largest |x_i|
// (lowest row on ties).
__global__ __launch_bounds__(256) void k_bfinal_x(const Chunk *__restrict__ chunks, BDev st, int m_last, Mat V,
                                                  double *__restrict__ x, double *__restrict__ fpart,
                                                  int64_t *__restrict__ ipart) {
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.inst, tid = threadIdx.x;
    const int mu = st.done[b] ? st.mfin[b] : m_last;
    __shared__ double sy[MS];
    __shared__ double sv[256], sn[256];
    __shared__ int64_t si[256];
    for (int j = tid; j < mu; j += 256) sy[j] = st.Y[(int64_t)b * MS * KB + j * KB];
    __syncthreads();
    const int64_t end = ch.r0 + ch.n;
    double n2 = 0.0, best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = ch.r0 + tid; i < end; i += 256) {
        double s = 0.0;
        for (int j = 0; j < mu; ++j) s += *V.at(i, j) * sy[j];
        x[i] = s;
        n2 += s * s;
        const double a = fabs(s);
        if (a > best || (a == best && i < bi)) {
            best = a;
            bi = i;
        }
    }
    sn[tid] = n2;
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sn[tid] += sn[tid + s];
            const double v = sv[tid + s];
            const int64_t j = si[tid + s];
            if (v > sv[tid] || (v == sv[tid] && j < si[tid])) {
                sv[tid] = v;
                si[tid] = j;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        fpart[blockIdx.x * 2] = sn[0];
        fpart[blockIdx.x * 2 + 1] = sv[0];
        ipart[blockIdx.x] = si[0];
    }
}

// Per instance: norm and gauge of the final vector (largest component
// positive), and the energy of instances that did not converge.
__global__ void k_bfinal_red(BDev st, const double *__restrict__ fpart, const int64_t *__restrict__ ipart,
                             const double *__restrict__ x, double *__restrict__ ss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= st.nb) return;
    double n2 = 0.0, best = -1.0;
    int64_t bi = INT64_MAX;
    for (int ch = st.inst_chunk[b]; ch < st.inst_chunk[b + 1]; ++ch) {
        n2 += fpart[ch * 2];
        const double v = fpart[ch * 2 + 1];
        const int64_t j = ipart[ch];
        if (v > best || (v == best && j < bi)) {
            best = v;
            bi = j;
        }
    }
    ss[b * 2] = n2 > 0.0 ? 1.0 / sqrt(n2) : 1.0;
    ss[b * 2 + 1] = (bi != INT64_MAX && x[bi] < 0.0) ? -1.0 : 1.0;
    if (!st.done[b]) st.energy[b] = st.theta[b * KB];
}

__global__ void k_bscatter(int64_t N, const double *__restrict__ x, const int32_t *__restrict__ row_inst,
                           const int64_t *__restrict__ inst_row, const int32_t *__restrict__ perm,
                           const double *__restrict__ ss, int sorted, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = row_inst[i];
    const int64_t r0 = inst_row[b];
    const int64_t dst = r0 + (sorted ? (i - r0) : (int64_t)perm[i]);
    out[dst] = x[i] * ss[b * 2] * ss[b * 2 + 1];
}

// ----------------------------------------------------------- concatenation

__global__ void k_cat_rowptr(int64_t n, const int64_t *__restrict__ src, int64_t *__restrict__ dst, int64_t nz0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) dst[i] = src[i] + nz0;
}

__global__ void k_cat_col(int64_t n, const int32_t *__restrict__ src, int32_t *__restrict__ dst, int32_t row0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] + row0;
}

__global__ void k_fill_i32(int64_t n, int32_t *__restrict__ dst, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

// ------------------------------------------------------------- host side

int env_or(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

template <typename T>
void copy_d2d(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n > 0) HQ_CHECK(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
}

// Capacity of b raised to at least `need` elements, keeping the first `used`
// (geometric growth, so appending instances one by one copies O(total)).
template <typename T>
void grow_keep(DBuf<T> &b, size_t used, size_t need, hipStream_t s) {
    if (b.p && need <= b.n) return;
    DBuf<T> nbuf;
    nbuf.ensure(std::max(need, 2 * b.n));
    copy_d2d(nbuf.p, b.p, (int64_t)used, s);
    wait_stream(s);
    b.swap(nbuf);
}

// Per-solve tables of the concatenated matrix: instance row offsets on the
// device and the coupling-balanced XCD row ranges.
void batch_layout(Ctx &c, BatchState &B) {
    if (!B.dirty) return;
    const int nb = (int)B.meta.size();
    B.g.device = c.device;
    B.g.stream = c.stream;
    B.g.have_elements = true;
    for (auto &row : B.g.sigma_cfg)
        for (auto &cfg : row) cfg = SigmaCfg{};
    compute_xcd_rows(B.g);
    B.inst_row.ensure(nb + 1);
    HQ_CHECK(hipMemcpyAsync(B.inst_row.p, B.row_off.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice,
                            c.stream));
    wait_stream(c.stream);
    B.dirty = false;
}

struct Resources {  // released on every exit path
    hipStream_t bs = nullptr;
    hipEvent_t ev = nullptr;
    int32_t *pinned = nullptr;  // landing word of the per-iteration finished-instance count
    std::vector<hipGraphExec_t> ex;
    bool capturing = false;
    ~Resources() {
        if (capturing && bs) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(bs, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        for (auto e : ex)
            if (e) (void)hipGraphExecDestroy(e);
        if (bs) (void)hipStreamSynchronize(bs);
        if (pinned) (void)hipHostFree(pinned);
        if (ev) (void)hipEventDestroy(ev);
        if (bs) (void)hipStreamDestroy(bs);
    }
};

template <int KK>
int batch_solve_k(Ctx &c, BatchState &B, const hinqs_opts &o, int mmax, const BatchState::Shape &shape,
                  double *energies, double *coeffs, int *status, int *iters_out, hinqs_batch_stats *stats,
                  std::chrono::steady_clock::time_point t0) {
    const int nb = (int)B.meta.size();
    const int64_t N = B.g.ndet;
    const int maxit = o.max_iter > 0 ? o.max_iter : 200;
    const bool use_graph = !(o.flags & HINQS_NO_GRAPH);
    const bool sorted = (o.flags & HINQS_SORTED_ORDER) != 0;
    if (o.flags & HINQS_AUTOTUNE) autotune_sigma(B.g, KK, HINQS_FP64);
    const SigmaCfg scfg = sigma_config(B.g, KK, HINQS_FP64);

    // ---- chunk list: runs of at most CH rows of one instance
    const int CH = std::max(64, env_or("HINQS_BATCH_CHUNK", shape.chunk));
    const int RRT = env_or("HINQS_BATCH_RR_THREADS", shape.rr_threads);
    if (RRT != 256 && RRT != 512 && RRT != 1024)
        throw Error(HINQS_E_INVALID_ARG, "Rayleigh-Ritz threads must be 256, 512 or 1024");
    std::vector<Chunk> chunks;
    std::vector<int32_t> inst_chunk(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        inst_chunk[b] = (int32_t)chunks.size();
        for (int64_t r = B.row_off[b]; r < B.row_off[b + 1]; r += CH)
            chunks.push_back(Chunk{r, (int32_t)std::min<int64_t>(CH, B.row_off[b + 1] - r), b});
    }
    inst_chunk[nb] = (int32_t)chunks.size();
    const int nch = (int)chunks.size();

    // buffers, all allocated before any capture (declared before R: R's
    // destructor drains the stream before they are freed)
    DBuf<double> Vb, Wb, gpart, gpart_u, rpart, state, xfin, fpart, ss;
    DBuf<int32_t> istate, d_ndone, d_inst_chunk;
    DBuf<int64_t> ranges, ipart;
    DBuf<Chunk> d_chunks;
    Resources R;
    HQ_CHECK(hipStreamCreateWithFlags(&R.bs, hipStreamNonBlocking));
    HQ_CHECK(hipHostMalloc((void **)&R.pinned, sizeof(int32_t), hipHostMallocDefault));
    HQ_CHECK(hipEventCreateWithFlags(&R.ev, hipEventDisableTiming));
    HQ_CHECK(hipEventRecord(R.ev, c.stream));  // work queued on the caller's stream comes first
    HQ_CHECK(hipStreamWaitEvent(R.bs, R.ev, 0));
    hipStream_t s = R.bs;

    const int nblocks = mmax / KK;
    const size_t bsz = (size_t)N * KK;
    Vb.ensure(bsz * nblocks);
    Wb.ensure(bsz * nblocks);
    gpart.ensure((size_t)nch * PSTRIDE);
    gpart_u.ensure((size_t)nch * PSTRIDE);
    rpart.ensure((size_t)nch * RSTRIDE);
    const size_t n_state = (size_t)nb * (MS * MS + MS * KB + KB + MS * 2 * KB + MS * KB + KB * KB + KB + 2);
    state.ensure(n_state);
    istate.ensure((size_t)nb * (4 + MS));
    d_ndone.ensure(1);
    ranges.ensure(9);
    d_chunks.ensure(nch);
    d_inst_chunk.ensure(nb + 1);
    xfin.ensure(N);
    fpart.ensure((size_t)nch * 2);
    ipart.ensure(nch);
    ss.ensure((size_t)nb * 2);
    HQ_CHECK(hipMemcpyAsync(d_chunks.p, chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
    HQ_CHECK(hipMemcpyAsync(d_inst_chunk.p, inst_chunk.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, s));
    HQ_CHECK(hipMemsetAsync(Vb.p, 0, sizeof(double) * bsz * nblocks, s));
    HQ_CHECK(hipMemsetAsync(Wb.p, 0, sizeof(double) * bsz * nblocks, s));
    HQ_CHECK(hipMemsetAsync(state.p, 0, sizeof(double) * n_state, s));
    HQ_CHECK(hipMemsetAsync(istate.p, 0, sizeof(int32_t) * nb * (4 + MS), s));
    BDev st{};
    st.nb = nb;
    st.inst_chunk = d_inst_chunk.p;
    st.done = istate.p;
    st.iters = st.done + nb;
    st.mfin = st.iters + nb;
    st.valid = st.mfin + nb;  // nb * MS
    st.skip2 = st.valid + (size_t)nb * MS;
    {
        double *p = state.p;
        st.G = p;      p += (size_t)nb * MS * MS;
        st.Y = p;      p += (size_t)nb * MS * KB;
        st.theta = p;  p += (size_t)nb * KB;
        st.Q = p;      p += (size_t)nb * MS * 2 * KB;
        st.C = p;      p += (size_t)nb * MS * KB;
        st.Z = p;      p += (size_t)nb * KB * KB;
        st.scl = p;    p += (size_t)nb * KB;
        st.energy = p; p += nb;
        st.resid = p;  p += nb;
    }
    wait_stream(s);
    const auto t_buf = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_bvalid_init, dim3(grid_for((int64_t)nb * MS, 256)), dim3(256), 0, s, nb, KK, st.valid);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipFuncSetAttribute((const void *)k_brr<KK, 256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)rr_lds_bytes(256)));
    HQ_CHECK(hipFuncSetAttribute((const void *)k_brr<KK, 512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)rr_lds_bytes(512)));
    HQ_CHECK(hipFuncSetAttribute((const void *)k_brr<KK, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)rr_lds_bytes(1024)));

    const Mat V{Vb.p, KK, (int64_t)bsz}, W{Wb.p, KK, (int64_t)bsz};
    SigmaMask mk;
    mk.ranges = ranges.p;
    mk.row_inst = B.row_inst.p;
    mk.inst_row = B.inst_row.p;
    mk.done = st.done;
    const Chunk *dch = d_chunks.p;
    const dim3 gch(nch), gin(nb), b256(256);

    auto gram = [&](Mat A, int ma, Mat Bm, double *part, const int32_t *gate) {
        const int mt = (ma + 15) / 16;
        switch (mt) {
            case 1: hipLaunchKernelGGL(k_bgram<1>, gch, b256, 0, s, dch, gate, A, ma, Bm, KK, part); break;
            case 2: hipLaunchKernelGGL(k_bgram<2>, gch, b256, 0, s, dch, gate, A, ma, Bm, KK, part); break;
            case 3: hipLaunchKernelGGL(k_bgram<3>, gch, b256, 0, s, dch, gate, A, ma, Bm, KK, part); break;
            default: hipLaunchKernelGGL(k_bgram<4>, gch, b256, 0, s, dch, gate, A, ma, Bm, KK, part); break;
        }
        HQ_LAUNCH_CHECK();
    };
    // Out = beta Out + alpha A[:, 0:m] B_inst (nc columns)
    auto tsmm = [&](Mat A, int m, const double *Bs, int bstride, int ldb, auto ncc, double alpha, double beta,
                    Mat Out, const int32_t *gate) {
        constexpr int NC = decltype(ncc)::value;
        hipLaunchKernelGGL((k_btsmm<(NC + 15) / 16, MS / 4>), gch, b256, 0, s, dch, gate, m, A, Bs, bstride, ldb,
                           NC, alpha, beta, Out);
        HQ_LAUNCH_CHECK();
    };
    using NK = std::integral_constant<int, KK>;
    using N2K = std::integral_constant<int, 2 * KK>;
    Ctx &g = B.g;
    auto sigma = [&](const double *X, double *S) {
        hipLaunchKernelGGL(k_bbalance, dim3(1), dim3(64), 0, s, nb, B.inst_row.p, g.rowptr.p, st.done, ranges.p);
        HQ_LAUNCH_CHECK();
        sigma_masked_fp64(g, KK, X, S, mk, s);
    };

    // ---- initial block (unit vectors at the lowest diagonal elements), its images and G
    hipLaunchKernelGGL(k_binit<KK>, gin, b256, 0, s, (const int64_t *)B.inst_row.p, (const double *)g.diag.p, Vb.p);
    HQ_LAUNCH_CHECK();
    sigma(V.p, W.p);
    const int32_t *dn = st.done, *g2 = st.skip2;
    gram(V, KK, W, gpart_u.p, dn);

    // ---- one iteration at subspace size m (m - KK columns old, KK new);
    // returns the subspace size after the optional restart
    const double tol = o.tol, floor_ = o.precond_floor;
    auto phase = [&](int m) -> int {
        const int restart = (m == mmax) ? 1 : 0;
        const int mp = restart ? 2 * KK : m;
        if (RRT == 1024)
            hipLaunchKernelGGL((k_brr<KK, 1024>), gin, dim3(1024), rr_lds_bytes(1024), s, st, m, restart,
                               (const double *)gpart_u.p);
        else if (RRT == 512)
            hipLaunchKernelGGL((k_brr<KK, 512>), gin, dim3(512), rr_lds_bytes(512), s, st, m, restart,
                               (const double *)gpart_u.p);
        else
            hipLaunchKernelGGL((k_brr<KK, 256>), gin, dim3(256), rr_lds_bytes(256), s, st, m, restart,
                               (const double *)gpart_u.p);
        HQ_LAUNCH_CHECK();
        if (restart) {
            tsmm(V, m, st.Q, MS * 2 * KB, 2 * KK, N2K{}, 1.0, 0.0, V, dn);
            tsmm(W, m, st.Q, MS * 2 * KB, 2 * KK, N2K{}, 1.0, 0.0, W, dn);
        }
        const Mat T = V.cols(mp);
        hipLaunchKernelGGL((k_britz<KK, MS / 4>), gch, b256, 0, s, dch, st, mp, V, W, (const double *)g.diag.p,
                           floor_, T.p, rpart.p);
        HQ_LAUNCH_CHECK();
        // projection against the basis, with T^T T from the first product; a
        // second pass only for instances whose first pass left some column
        // less than half its norm
        gram(V, mp + KK, T, gpart.p, dn);
        hipLaunchKernelGGL(k_bpost_first<KK>, gin, dim3(NT), 0, s, st, mp, tol, (const double *)rpart.p,
                           (const double *)gpart.p);
        HQ_LAUNCH_CHECK();
        tsmm(V, mp, st.C, MS * KB, KB, NK{}, -1.0, 1.0, T, dn);
        gram(V, mp, T, gpart.p, g2);
        hipLaunchKernelGGL(k_bpost_proj<KK>, gin, dim3(NT), 0, s, st, g2, mp, (const double *)gpart.p);
        HQ_LAUNCH_CHECK();
        tsmm(V, mp, st.C, MS * KB, KB, NK{}, -1.0, 1.0, T, g2);
        // symmetric orthonormalization within the block (unit columns first)
        const Mat Tm{T.p, KK, (int64_t)bsz};
        gram(Tm, KK, Tm, gpart.p, dn);
        hipLaunchKernelGGL(k_bpost_orth<KK>, gin, dim3(NT), 0, s, st, dn, mp, (const double *)gpart.p);
        HQ_LAUNCH_CHECK();
        tsmm(Tm, KK, st.Z, KB * KB, KB, NK{}, 1.0, 0.0, Tm, dn);
        // images and the new columns of G
        const Mat Wn = W.cols(mp);
        sigma(T.p, Wn.p);
        gram(V, mp + KK, Wn, gpart_u.p, dn);
        hipLaunchKernelGGL(k_bcount, dim3(1), b256, 0, s, nb, (const int32_t *)st.done, d_ndone.p);
        HQ_LAUNCH_CHECK();
        return mp;
    };

    wait_stream(s);
    const auto t1 = std::chrono::steady_clock::now();
    const bool verbose = env_or("HINQS_VERBOSE", 0) != 0;
    if (verbose)
        std::fprintf(stderr, "[hinqs] batch setup %.2f ms (buffers ready %.2f ms)\n",
                     std::chrono::duration<double, std::milli>(t1 - t0).count(),
                     std::chrono::duration<double, std::milli>(t_buf - t0).count());
    R.ex.assign(mmax / KK + 1, nullptr);
    int m = KK, it = 0, m_last = KK, ngraphs = 0;
    int32_t ndone = 0;
    double ms_capture = 0.0;
    while (it < maxit) {
        int mp;
        if (use_graph) {
            hipGraphExec_t &ex = R.ex[m / KK];
            if (!ex) {
                const auto tc = std::chrono::steady_clock::now();
                HQ_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                R.capturing = true;
                phase(m);
                hipGraph_t graph = nullptr;
                R.capturing = false;
                HQ_CHECK(hipStreamEndCapture(s, &graph));
                const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                HQ_CHECK(e);
                ++ngraphs;
                ms_capture += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc).count();
            }
            HQ_CHECK(hipGraphLaunch(ex, s));
            mp = (m == mmax) ? 2 * KK : m;
        } else {
            mp = phase(m);
        }
        ++it;
        m_last = mp;
        // pinned landing word, polled wait: the next graph launch waits on this read
        HQ_CHECK(hipMemcpyAsync(R.pinned, d_ndone.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        wait_stream(s);
        ndone = *R.pinned;
        if (ndone >= nb) break;
        m = mp + KK;
    }
    const auto t2 = std::chrono::steady_clock::now();
    if (verbose)
        std::fprintf(stderr, "[hinqs] batch loop %.2f ms (capture %.2f ms, %d iterations)\n",
                     std::chrono::duration<double, std::milli>(t2 - t1).count(), ms_capture, it);

    // ---- final vectors: x = V y_0, normalized, largest component positive, caller order
    hipLaunchKernelGGL(k_bfinal_x, gch, b256, 0, s, dch, st, m_last, V, xfin.p, fpart.p, ipart.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bfinal_red, dim3((nb + 63) / 64), dim3(64), 0, s, st, (const double *)fpart.p,
                       (const int64_t *)ipart.p, (const double *)xfin.p, ss.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bscatter, dim3(grid_for(N, 256)), b256, 0, s, N, (const double *)xfin.p,
                       (const int32_t *)B.row_inst.p, (const int64_t *)B.inst_row.p, (const int32_t *)B.perm.p,
                       (const double *)ss.p, sorted ? 1 : 0, coeffs);
    HQ_LAUNCH_CHECK();
    std::vector<double> e_h(nb), r_h(nb);
    std::vector<int32_t> done_h(nb), it_h(nb);
    HQ_CHECK(hipMemcpyAsync(e_h.data(), st.energy, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(r_h.data(), st.resid, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(done_h.data(), st.done, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(it_h.data(), st.iters, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    wait_stream(s);
    HQ_CHECK(hipEventRecord(R.ev, s));  // the caller's stream sees the outputs
    HQ_CHECK(hipStreamWaitEvent(c.stream, R.ev, 0));
    int nconv = 0;
    double maxres = 0.0;
    double elements = 0.0;
    for (int b = 0; b < nb; ++b) {
        // sigma products that carried instance b: the initial block plus one per
        // iteration that did not end it
        const int nsig = it_h[b] + ((done_h[b] == 1 || done_h[b] == 2) ? 0 : 1);
        elements += (double)(B.meta[b].nnz + B.meta[b].ndet) * KK * nsig;
    }
    for (int b = 0; b < nb; ++b) {
        energies[b] = e_h[b];
        const bool ok = done_h[b] == 1;
        nconv += ok ? 1 : 0;
        if (status) status[b] = ok ? HINQS_OK : HINQS_E_NOT_CONVERGED;
        if (iters_out) iters_out[b] = it_h[b];
        maxres = std::max(maxres, r_h[b]);
    }
    if (stats) {
        stats->instances = nb;
        stats->converged = nconv;
        stats->iterations = it;
        stats->graphs = ngraphs;
        stats->ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count() + ms_capture;
        stats->ms_iterations = std::chrono::duration<double, std::milli>(t2 - t1).count() - ms_capture;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        stats->max_residual = maxres;
        stats->ndet = N;
        stats->nnz = g.nnz;
        stats->sigma_team = scfg.team;
        stats->sigma_unroll = scfg.unr;
        stats->sigma_occupancy = scfg.occ;
        stats->sigma_elements = elements;
        stats->chunk_rows = CH;
        stats->rr_threads = RRT;
    }
    return nconv == nb ? HINQS_OK : HINQS_E_NOT_CONVERGED;
}

}  // namespace

namespace {

// Batch launch shapes tuned in this process, keyed by device architecture,
// block size, subspace limit, instance count and problem-size class.
std::mutex g_bshape_mutex;
std::map<std::string, BatchState::Shape> g_bshape_cache;

std::string batch_shape_key(const Ctx &c, const BatchState &B, int K, int mmax) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) arch = prop.gcnArchName;
    const int64_t n = B.g.ndet, z = B.g.nnz;
    const int dbucket = n > 0 ? (int)std::lround(2.0 * std::log2((double)n)) : 0;
    const int nbucket = n > 0 ? (int)std::lround((double)z / (double)n / 16.0) : 0;
    return arch + "|batch|k" + std::to_string(K) + "|m" + std::to_string(mmax) + "|i" +
           std::to_string(B.meta.size()) + "|d" + std::to_string(dbucket) + "|n" + std::to_string(nbucket);
}

bool batch_shape_cached(const std::string &key, BatchState::Shape &out) {
    std::lock_guard<std::mutex> lk(g_bshape_mutex);
    auto it = g_bshape_cache.find(key);
    if (it == g_bshape_cache.end()) return false;
    out = it->second;
    return true;
}

void batch_shape_store(const std::string &key, const BatchState::Shape &sh) {
    std::lock_guard<std::mutex> lk(g_bshape_mutex);
    g_bshape_cache[key] = sh;
}

// Times `iters` iterations of the batched solve for each candidate shape
// (chunk rows 1024..8192, Rayleigh-Ritz threads 512 or 1024; every candidate
// starts from the same initial block) and returns the fastest per iteration.
template <typename F>
BatchState::Shape tune_batch_shape(const BatchState &B, int iters, F &&time_it) {
    static const int chunks[] = {1024, 2048, 4096, 8192};
    static const int threads[] = {512, 1024};
    BatchState::Shape best;
    best.ms_per_it = 1e30;
    for (int ch : chunks) {
        if (ch > 2 * B.g.ndet / std::max<size_t>(1, B.meta.size()) && ch != chunks[0]) continue;
        for (int nt : threads) {
            BatchState::Shape sh;
            sh.chunk = ch;
            sh.rr_threads = nt;
            sh.ms_per_it = time_it(sh, iters);
            if (env_or("HINQS_VERBOSE", 0))
                std::fprintf(stderr, "[hinqs] batch shape chunk %d rr_threads %d: %.3f ms per iteration\n", ch, nt,
                             sh.ms_per_it);
            if (sh.ms_per_it < best.ms_per_it) best = sh;
        }
    }
    return best;
}

}  // namespace

void batch_clear(Ctx &c) {
    if (!c.batch) return;
    BatchState &B = *c.batch;  // device buffers are kept for the next instances
    B.meta.clear();
    B.row_off.assign(1, 0);
    B.nz_off.assign(1, 0);
    B.g.ndet = 0;
    B.g.nnz = 0;
    B.dirty = true;
}

int batch_add(Ctx &c, int norb, const double *h, const double *eri, double ecore, int64_t ndet,
              const uint64_t *alpha, const uint64_t *beta, int na, int nb) {
    if (!c.batch) c.batch = std::make_shared<BatchState>();
    BatchState &B = *c.batch;
    if (B.row_off.back() + ndet >= ((int64_t)1 << 31) - 1)
        throw Error(HINQS_E_UNSUPPORTED, "a batch holds fewer than 2^31 determinants");
    Ctx &p = B.scratch;
    p.device = c.device;
    p.stream = c.stream;
    p.have_ints = p.have_dets = p.have_elements = false;
    {
        struct Grow {
            Grow() { g_dbuf_grow = true; }
            ~Grow() { g_dbuf_grow = false; }
        } grow;
        build_integrals(p, norb, h, eri, ecore);
        build_determinants(p, ndet, alpha, beta, na, nb, false);
        build_connectivity(p, false);
        build_elements(p);
    }
    // append to the concatenated arrays
    hipStream_t s = c.stream;
    const int bi = (int)B.meta.size();
    const int64_t r0 = B.row_off.back(), z0 = B.nz_off.back();
    const int64_t r1 = r0 + p.ndet, z1 = z0 + p.nnz;
    grow_keep(B.g.rowptr, (size_t)(bi ? r0 + 1 : 0), (size_t)(r1 + 1), s);
    grow_keep(B.g.col, (size_t)z0, (size_t)std::max<int64_t>(z1, 1), s);
    grow_keep(B.g.val, (size_t)z0, (size_t)std::max<int64_t>(z1, 1), s);
    grow_keep(B.g.diag, (size_t)r0, (size_t)r1, s);
    grow_keep(B.perm, (size_t)r0, (size_t)r1, s);
    grow_keep(B.row_inst, (size_t)r0, (size_t)r1, s);
    hipLaunchKernelGGL(k_cat_rowptr, dim3(grid_for(p.ndet + 1, 256)), dim3(256), 0, s, p.ndet, p.rowptr.p,
                       B.g.rowptr.p + r0, z0);
    HQ_LAUNCH_CHECK();
    if (p.nnz > 0) {
        hipLaunchKernelGGL(k_cat_col, dim3(grid_for(p.nnz, 256)), dim3(256), 0, s, p.nnz, p.col.p, B.g.col.p + z0,
                           (int32_t)r0);
        HQ_LAUNCH_CHECK();
        copy_d2d(B.g.val.p + z0, p.val.p, p.nnz, s);
    }
    copy_d2d(B.g.diag.p + r0, p.diag.p, p.ndet, s);
    copy_d2d(B.perm.p + r0, p.perm.p, p.ndet, s);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(p.ndet, 256)), dim3(256), 0, s, p.ndet, B.row_inst.p + r0,
                       (int32_t)bi);
    HQ_LAUNCH_CHECK();
    // no wait: the next instance's build reuses the scratch buffers in stream order
    B.g.ndet = r1;
    B.g.nnz = z1;
    B.meta.push_back({norb, na, nb, p.ndet, p.nnz});
    B.row_off.push_back(r1);
    B.nz_off.push_back(z1);
    B.dirty = true;
    return bi;
}

void batch_info(Ctx &c, int *ninst, int64_t *offsets, int64_t *nnz) {
    const int nb = c.batch ? (int)c.batch->meta.size() : 0;
    if (ninst) *ninst = nb;
    if (offsets)
        for (int b = 0; b <= nb; ++b) offsets[b] = c.batch ? c.batch->row_off[b] : 0;
    if (nnz) *nnz = c.batch ? c.batch->nz_off[nb] : 0;
}

int batch_solve(Ctx &c, const hinqs_opts &o, double *energies, double *coeffs, int *status, int *iters_out,
                hinqs_batch_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!c.batch || c.batch->meta.empty()) throw Error(HINQS_E_NOT_READY, "the batch holds no instance");
    BatchState &B = *c.batch;
    const int K = o.block;
    if (K != 1 && K != 2 && K != 4 && K != 8 && K != 16)
        throw Error(HINQS_E_UNSUPPORTED, "block size must be 1, 2, 4, 8 or 16");
    int mmax = o.max_space > 0 ? o.max_space : 6 * K;
    mmax = std::min(mmax, MS) / K * K;
    if (mmax < 3 * K) throw Error(HINQS_E_UNSUPPORTED, "batched solves need 3 * block <= max_space <= 64");
    const int nb = (int)B.meta.size();
    for (int b = 0; b < nb; ++b)
        if (B.meta[b].ndet < mmax)
            throw Error(HINQS_E_UNSUPPORTED, "instance " + std::to_string(b) +
                                                 " has fewer determinants than the subspace size; solve it alone");
    batch_layout(c, B);
    auto run = [&](const BatchState::Shape &sh, const hinqs_opts &oo, double *e, double *x, int *st_,
                   int *it_, hinqs_batch_stats *bs, std::chrono::steady_clock::time_point tt) {
        switch (K) {
            case 1: return batch_solve_k<1>(c, B, oo, mmax, sh, e, x, st_, it_, bs, tt);
            case 2: return batch_solve_k<2>(c, B, oo, mmax, sh, e, x, st_, it_, bs, tt);
            case 4: return batch_solve_k<4>(c, B, oo, mmax, sh, e, x, st_, it_, bs, tt);
            case 8: return batch_solve_k<8>(c, B, oo, mmax, sh, e, x, st_, it_, bs, tt);
            default: return batch_solve_k<16>(c, B, oo, mmax, sh, e, x, st_, it_, bs, tt);
        }
    };
    const int ki = K <= 1 ? 0 : K <= 2 ? 1 : K <= 4 ? 2 : K <= 8 ? 3 : 4;
    const std::string key = batch_shape_key(c, B, K, mmax);
    double ms_tune = 0.0;
    if ((o.flags & HINQS_AUTOTUNE) && B.tuned_key[ki] != key) {
        const auto tt0 = std::chrono::steady_clock::now();
        if (!batch_shape_cached(key, B.shape[ki])) {
            B.shape[ki] = tune_batch_shape(B, mmax / K * 2, [&](const BatchState::Shape &sh, int iters) {
                hinqs_opts oo = o;
                oo.max_iter = iters;
                std::vector<double> e(nb);
                DBuf<double> x;
                x.ensure((size_t)B.g.ndet);
                hinqs_batch_stats bs{};
                (void)run(sh, oo, e.data(), x.p, nullptr, nullptr, &bs, std::chrono::steady_clock::now());
                return bs.iterations > 0 ? bs.ms_iterations / bs.iterations : 1e30;
            });
            batch_shape_store(key, B.shape[ki]);
        }
        B.tuned_key[ki] = key;
        ms_tune = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tt0).count();
    }
    const int rc = run(B.shape[ki], o, energies, coeffs, status, iters_out, stats, t0);
    if (stats) stats->ms_tune = ms_tune;
    return rc;
}

}  // namespace hinqs
