// Block sigma product S = H_B X over the stored couplings (paper Sec. 2.2,
// Step 3: the product the Davidson iteration repeats).
//
// Layout: CSR over sorted rows (rowptr int64, col int32, val fp64/fp32) plus
// the diagonal; X and S are ndet x K row-major with leading dimensions, so a
// row of X for K = 8 doubles is one 64-byte segment.  A team of lanes owns
// one row; groups of lanes inside the team share one coupling and gather its
// X row as one contiguous segment (16 bytes per lane), while the CSR stream is
// read with non-temporal loads so it does not evict X from the caches.  The
// partial sums are combined with a butterfly of cross-lane shuffles.  Every
// row is written by exactly one team, so the result is deterministic and
// atomic-free.
//
// Workgroups are remapped so each XCD (8 on MI355X, round-robin dispatch)
// receives a contiguous range of rows: rows with the same alpha string gather
// the same X rows, and keeping them on one XCD keeps those X rows in its L2.
#include "common.hpp"

namespace hinqs {

namespace {

constexpr int SIGMA_BLOCK = 256;
constexpr int NUM_XCD = 8;

// One 16-byte vector of T (2 doubles or 4 floats).
template <typename T>
struct Vec16;
template <>
struct Vec16<double> { using type = double2; static constexpr int n = 2; };
template <>
struct Vec16<float> { using type = float4; static constexpr int n = 4; };

template <typename T, int N>
__device__ inline void load_vec(const T *p, T (&x)[N]) {
    if constexpr (N * sizeof(T) == 16) {
        using V = typename Vec16<T>::type;
        V v = *(const V *)p;
        if constexpr (N == 2) { x[0] = v.x; x[1] = v.y; }
        else { x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w; }
    } else {
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] = p[c];
    }
}

template <typename T, int N>
__device__ inline void store_vec(T *p, const T (&x)[N]) {
    if constexpr (N * sizeof(T) == 16) {
        using V = typename Vec16<T>::type;
        V v;
        if constexpr (N == 2) { v.x = x[0]; v.y = x[1]; }
        else { v.x = x[0]; v.y = x[1]; v.z = x[2]; v.w = x[3]; }
        *(V *)p = v;
    } else {
#pragma unroll
        for (int c = 0; c < N; ++c) p[c] = x[c];
    }
}

// A team of TEAM lanes owns one row.  LPN lanes share one coupling: each loads
// EPL consecutive entries (16 bytes) of the gathered X row, so one load
// instruction touches 64 / LPN distinct rows and every row is read as one
// contiguous segment.  Each lane keeps UNR couplings in flight.
template <typename T, int K, int TEAM>
__global__ __launch_bounds__(SIGMA_BLOCK) void k_sigma(int64_t nrows, const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ X, int ldx,
                                                       T *__restrict__ S, int lds) {
    constexpr int VW = Vec16<T>::n;
    constexpr int LPN = (K >= VW) ? K / VW : 1;   // lanes per coupling
    constexpr int EPL = K / LPN;                   // entries of X per lane
    constexpr int NPT = TEAM / LPN;                // couplings per team step
    constexpr int UNR = 2;
    static_assert(TEAM % LPN == 0 && TEAM <= 64, "team shape");
    // XCD-aware block order: hardware block b runs on XCD b % 8.
    const unsigned per_xcd = gridDim.x / NUM_XCD;
    const unsigned lb = (blockIdx.x % NUM_XCD) * per_xcd + blockIdx.x / NUM_XCD;
    const int sub = threadIdx.x % TEAM;
    const int q = sub % LPN, g = sub / LPN;
    const int64_t row = ((int64_t)lb * SIGMA_BLOCK + threadIdx.x) / TEAM;
    if (row >= nrows) return;  // uniform across the team
    T acc[EPL];
#pragma unroll
    for (int c = 0; c < EPL; ++c) acc[c] = T(0);
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    const T *Xq = X + q * EPL;
    int64_t e = beg + g;
    for (; e + (UNR - 1) * NPT < end; e += UNR * NPT) {
        int32_t j[UNR];
        T v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            j[u] = __builtin_nontemporal_load(col + e + u * NPT);
            v[u] = __builtin_nontemporal_load(val + e + u * NPT);
        }
        T x[UNR][EPL];
#pragma unroll
        for (int u = 0; u < UNR; ++u) load_vec<T, EPL>(Xq + (int64_t)j[u] * ldx, x[u]);
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int c = 0; c < EPL; ++c) acc[c] += v[u] * x[u][c];
    }
    for (; e < end; e += NPT) {
        const int32_t j = __builtin_nontemporal_load(col + e);
        const T v = __builtin_nontemporal_load(val + e);
        T x[EPL];
        load_vec<T, EPL>(Xq + (int64_t)j * ldx, x);
#pragma unroll
        for (int c = 0; c < EPL; ++c) acc[c] += v * x[c];
    }
#pragma unroll
    for (int off = LPN; off < TEAM; off <<= 1) {
#pragma unroll
        for (int c = 0; c < EPL; ++c) acc[c] += __shfl_xor(acc[c], off, TEAM);
    }
    if (g == 0) {
        const T d = diag[row];
        T xr[EPL];
        load_vec<T, EPL>(Xq + row * ldx, xr);
#pragma unroll
        for (int c = 0; c < EPL; ++c) acc[c] += d * xr[c];
        store_vec<T, EPL>(S + row * lds + q * EPL, acc);
    }
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
    // lanes per coupling times couplings in flight per row, sized to the mean row length
    constexpr int VW = Vec16<T>::n;
    constexpr int LPN = (K >= VW) ? K / VW : 1;
    const double avg = c.ndet > 0 ? (double)c.nnz / (double)c.ndet : 0.0;
    const double per_step = avg / 4.0;  // aim at >= 4 team steps (x2 unroll) per row
    if constexpr (LPN <= 2) {
        if (per_step <= 4) launch_sigma<T, K, 8>(c, val, diag, X, ldx, S, lds, s);
        else if (per_step <= 8 * 2 / LPN) launch_sigma<T, K, 16>(c, val, diag, X, ldx, S, lds, s);
        else if (per_step <= 16 * 2 / LPN) launch_sigma<T, K, 32>(c, val, diag, X, ldx, S, lds, s);
        else launch_sigma<T, K, 64>(c, val, diag, X, ldx, S, lds, s);
    } else if constexpr (LPN == 4) {
        if (per_step <= 4) launch_sigma<T, K, 16>(c, val, diag, X, ldx, S, lds, s);
        else if (per_step <= 8) launch_sigma<T, K, 32>(c, val, diag, X, ldx, S, lds, s);
        else launch_sigma<T, K, 64>(c, val, diag, X, ldx, S, lds, s);
    } else {
        if (per_step <= 4) launch_sigma<T, K, 32>(c, val, diag, X, ldx, S, lds, s);
        else launch_sigma<T, K, 64>(c, val, diag, X, ldx, S, lds, s);
    }
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
