// Block sigma product S = H_B X over the stored couplings (paper Sec. 2.2,
// Step 3: the product the Davidson iteration repeats).
//
// Layout: CSR over sorted rows (rowptr int64, col int32, val fp64/fp32) plus
// the diagonal; X and S are ndet x K row-major with leading dimensions, so a
// row of X for K = 8 doubles is one 64-byte segment.  A team of TEAM lanes
// owns one row: lanes stride over the row's couplings (coalesced, streamed
// with non-temporal loads so the CSR does not evict X from the caches),
// gather X rows with 16-byte vector loads, accumulate K sums in registers and
// combine them with a butterfly of cross-lane shuffles.  Every row is written
// by exactly one team, so the result is deterministic and atomic-free.
//
// Workgroups are remapped so each XCD (8 on MI355X, round-robin dispatch)
// receives a contiguous range of rows: rows with the same alpha string gather
// the same X rows, and keeping them on one XCD keeps those X rows in its L2.
#include "common.hpp"

namespace hinqs {

namespace {

constexpr int SIGMA_BLOCK = 256;
constexpr int NUM_XCD = 8;

template <typename T>
struct Vec2;
template <>
struct Vec2<double> { using type = double2; static constexpr int n = 2; };
template <>
struct Vec2<float> { using type = float4; static constexpr int n = 4; };

template <typename T, int K>
__device__ inline void load_row(const T *p, T (&x)[K]) {
    using V = typename Vec2<T>::type;
    constexpr int W = Vec2<T>::n;
    if constexpr (K % W == 0) {
#pragma unroll
        for (int c = 0; c < K; c += W) {
            V v = *(const V *)(p + c);
            if constexpr (W == 2) {
                x[c] = v.x;
                x[c + 1] = v.y;
            } else {
                x[c] = v.x;
                x[c + 1] = v.y;
                x[c + 2] = v.z;
                x[c + 3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c) x[c] = p[c];
    }
}

template <typename T, int K, int TEAM>
__global__ __launch_bounds__(SIGMA_BLOCK) void k_sigma(int64_t nrows, const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ X, int ldx,
                                                       T *__restrict__ S, int lds) {
    // XCD-aware block order: hardware block b runs on XCD b % 8.
    const unsigned per_xcd = gridDim.x / NUM_XCD;
    const unsigned lb = (blockIdx.x % NUM_XCD) * per_xcd + blockIdx.x / NUM_XCD;
    const int sub = threadIdx.x % TEAM;
    const int64_t row = ((int64_t)lb * SIGMA_BLOCK + threadIdx.x) / TEAM;
    if (row >= nrows) return;  // uniform across the team
    T acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = T(0);
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    for (int64_t e = beg + sub; e < end; e += TEAM) {
        const int32_t j = __builtin_nontemporal_load(col + e);
        const T v = __builtin_nontemporal_load(val + e);
        T x[K];
        load_row<T, K>(X + (int64_t)j * ldx, x);
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] += v * x[c];
    }
#pragma unroll
    for (int off = TEAM / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] += __shfl_xor(acc[c], off, TEAM);
    }
    const T d = diag[row];
    const T *xr = X + row * ldx;
    T *sr = S + row * lds;
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (c % TEAM == sub) sr[c] = acc[c] + d * xr[c];
}

template <typename T, int K, int TEAM>
void launch_sigma(const Ctx &c, const T *val, const T *diag, const T *X, int ldx, T *S, int lds,
                  hipStream_t s) {
    int64_t teams_per_block = SIGMA_BLOCK / TEAM;
    int64_t nblk = (c.ndet + teams_per_block - 1) / teams_per_block;
    nblk = (nblk + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    hipLaunchKernelGGL((k_sigma<T, K, TEAM>), dim3((unsigned)nblk), dim3(SIGMA_BLOCK), 0, s, c.ndet,
                       c.rowptr.p, c.col.p, val, diag, X, ldx, S, lds);
    HQ_LAUNCH_CHECK();
}

template <typename T, int K>
void dispatch_team(const Ctx &c, const T *val, const T *diag, const T *X, int ldx, T *S, int lds,
                   hipStream_t s) {
    double avg = c.ndet > 0 ? (double)c.nnz / (double)c.ndet : 0.0;
    if (avg <= 24) launch_sigma<T, K, 4>(c, val, diag, X, ldx, S, lds, s);
    else if (avg <= 64) launch_sigma<T, K, 8>(c, val, diag, X, ldx, S, lds, s);
    else if (avg <= 256) launch_sigma<T, K, 16>(c, val, diag, X, ldx, S, lds, s);
    else launch_sigma<T, K, 32>(c, val, diag, X, ldx, S, lds, s);
}

template <typename T>
void dispatch_k(const Ctx &c, int k, const T *val, const T *diag, const T *X, int ldx, T *S, int lds,
                hipStream_t s) {
    switch (k) {
        case 1: dispatch_team<T, 1>(c, val, diag, X, ldx, S, lds, s); break;
        case 2: dispatch_team<T, 2>(c, val, diag, X, ldx, S, lds, s); break;
        case 4: dispatch_team<T, 4>(c, val, diag, X, ldx, S, lds, s); break;
        case 8: dispatch_team<T, 8>(c, val, diag, X, ldx, S, lds, s); break;
        case 16: dispatch_team<T, 16>(c, val, diag, X, ldx, S, lds, s); break;
        default: throw Error(HINQS_E_UNSUPPORTED, "sigma block size must be 1, 2, 4, 8 or 16");
    }
}

}  // namespace

// X, S in sorted order; k in {1,2,4,8,16}; leading dimensions keep 16-byte
// alignment of every row (ldx, lds multiples of 16 / sizeof(T) when k >= that).
void sigma_sorted(Ctx &c, int k, const void *X, int ldx, void *S, int lds, int precision,
                  hipStream_t s) {
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
    if (precision == HINQS_FP64)
        dispatch_k<double>(c, k, c.val.p, c.diag.p, (const double *)X, ldx, (double *)S, lds, s);
    else if (precision == HINQS_FP32)
        dispatch_k<float>(c, k, c.val32.p, c.diag32.p, (const float *)X, ldx, (float *)S, lds, s);
    else
        throw Error(HINQS_E_INVALID_ARG, "precision must be HINQS_FP64 or HINQS_FP32");
}

}  // namespace hinqs
