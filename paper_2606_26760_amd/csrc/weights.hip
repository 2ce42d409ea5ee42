// Spin-marginal teacher weights of the eigenvector (Sec. 2.2, Step 4,
// Eqs. 5-6): p_alpha(s) = sum of c_j^2 over the determinants of B whose alpha
// string is s, p_beta likewise over beta strings, and for every determinant
// x = (s_a, s_b) of B the weight w(x) = p_alpha(s_a) p_beta(s_b) / Z with Z
// the sum of those products over B.
//
// The marginals are segmented sums over the groups of the determinant store:
// an alpha group is a contiguous run of the sorted order, a beta group a run
// of the beta-major listing.  One wave per group sums lane-strided partials
// and combines them with a fixed butterfly, and Z is a two-level fixed-order
// reduction, so the weights are bitwise reproducible.
#include "common.hpp"

namespace hinqs {

namespace {

constexpr int W_NT = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// p[g] = sum of c[idx(u)]^2 over u in [off[g], off[g+1]); idx = perm[u] when
// perm is given, else u.  Non-finite coefficients raise the flag.
__global__ __launch_bounds__(W_NT) void k_marginal(const double *c, const int32_t *off, const int32_t *perm,
                                                   int32_t ngroups, double *p, unsigned *bad) {
    const int lane = threadIdx.x & 63;
    const int32_t g = (int32_t)((blockIdx.x * (int64_t)W_NT + threadIdx.x) >> 6);
    if (g >= ngroups) return;
    const int32_t lo = off[g], hi = off[g + 1];
    double acc = 0.0;
    for (int32_t u = lo + lane; u < hi; u += 64) {
        const double x = c[perm ? perm[u] : u];
        if (!isfinite(x)) atomicOr(bad, 1u);
        acc += x * x;
    }
    acc = wave_sum(acc);
    if (lane == 0) p[g] = acc;
}

// Unnormalized products of the sorted rows and per-workgroup partial sums.
__global__ __launch_bounds__(W_NT) void k_products(const double *pa, const double *pb, const int32_t *aidx,
                                                   const int32_t *bidx, int64_t n, double *wu, double *part) {
    __shared__ double red[W_NT / 64];
    const int64_t j = (int64_t)blockIdx.x * W_NT + threadIdx.x;
    double v = 0.0;
    if (j < n) {
        v = pa[aidx[j]] * pb[bidx[j]];
        wu[j] = v;
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < W_NT / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

// z[0] = sum of part[0..n) in a fixed order (one workgroup).
__global__ __launch_bounds__(W_NT) void k_total(const double *part, int64_t n, double *z) {
    __shared__ double red[W_NT / 64];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += W_NT) v += part[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < W_NT / 64; ++w) s += red[w];
        z[0] = s;
    }
}

// w[dst(j)] = wu[j] / z; dst = perm (sorted position -> caller index) or identity.
__global__ void k_normalize(const double *wu, const double *z, const int32_t *perm, int64_t n, double *w) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    w[perm ? perm[j] : j] = wu[j] / z[0];
}

__global__ void k_widen(const uint32_t *in, int64_t n, uint64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace

void teacher_weights(Ctx &c, const double *coeffs, bool sorted, double *w, double *p_alpha, double *p_beta) {
    hipStream_t s = c.stream;
    const int64_t n = c.ndet;
    // the alpha marginal reads c in sorted order; the beta marginal goes through bperm
    DBuf<double> cs;
    const double *csp = coeffs;
    if (!sorted) {
        cs.ensure(n);
        gather_rows(s, coeffs, cs.p, c.perm.p, n, 8);
        csp = cs.p;
    }
    DBuf<double> pa, pb, wu, part, z;
    DBuf<unsigned> bad;
    pa.ensure(c.nua);
    pb.ensure(c.nub);
    const int64_t nblk = (n + W_NT - 1) / W_NT;
    wu.ensure(n);
    part.ensure(nblk);
    z.ensure(1);
    bad.ensure(1);
    HQ_CHECK(hipMemsetAsync(bad.p, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_marginal, dim3(grid_for((int64_t)c.nua * 64, W_NT)), dim3(W_NT), 0, s, csp, c.ga.p,
                       (const int32_t *)nullptr, c.nua, pa.p, bad.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_marginal, dim3(grid_for((int64_t)c.nub * 64, W_NT)), dim3(W_NT), 0, s, csp, c.gb.p,
                       c.bperm.p, c.nub, pb.p, bad.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_products, dim3((unsigned)nblk), dim3(W_NT), 0, s, pa.p, pb.p, c.aidx.p, c.bidx.p, n, wu.p,
                       part.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_total, dim3(1), dim3(W_NT), 0, s, part.p, nblk, z.p);
    HQ_LAUNCH_CHECK();
    double hz = 0.0;
    unsigned hbad = 0;
    HQ_CHECK(hipMemcpyAsync(&hz, z.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&hbad, bad.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (hbad) throw Error(HINQS_E_NONFINITE, "coefficients contain NaN/Inf");
    if (!(hz > 0.0)) throw Error(HINQS_E_INVALID_ARG, "the weights sum to zero (all coefficients vanish)");
    if (w) {
        hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, 256)), dim3(256), 0, s, wu.p, z.p,
                           sorted ? (const int32_t *)nullptr : (const int32_t *)c.perm.p, n, w);
        HQ_LAUNCH_CHECK();
    }
    if (p_alpha) HQ_CHECK(hipMemcpyAsync(p_alpha, pa.p, sizeof(double) * c.nua, hipMemcpyDeviceToDevice, s));
    if (p_beta) HQ_CHECK(hipMemcpyAsync(p_beta, pb.p, sizeof(double) * c.nub, hipMemcpyDeviceToDevice, s));
    HQ_CHECK(hipStreamSynchronize(s));
}

void distinct_strings(Ctx &c, uint64_t *alpha, uint64_t *beta) {
    hipStream_t s = c.stream;
    if (alpha) {
        hipLaunchKernelGGL(k_widen, dim3(grid_for(c.nua, 256)), dim3(256), 0, s, c.ua.p, (int64_t)c.nua, alpha);
        HQ_LAUNCH_CHECK();
    }
    if (beta) {
        hipLaunchKernelGGL(k_widen, dim3(grid_for(c.nub, 256)), dim3(256), 0, s, c.ub.p, (int64_t)c.nub, beta);
        HQ_LAUNCH_CHECK();
    }
    HQ_CHECK(hipStreamSynchronize(s));
}

}  // namespace hinqs
