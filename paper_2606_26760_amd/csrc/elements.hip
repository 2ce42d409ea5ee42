// Integral staging and Slater-Condon matrix elements.
//
// The Hamiltonian of Sec. 2.2 enters through h_pq and the chemists' (pq|rs).
// With real orbitals (pq|rs) has 8-fold symmetry, so the library keeps one
// value per unordered pair of orbital pairs (9,316 doubles = 74.5 KB at
// norb = 16), small enough to sit in the LDS of a gfx950 workgroup next to h.
//
// The element rules are in slater.hpp.
#include <chrono>
#include <cmath>

#include "common.hpp"
#include "slater.hpp"

namespace hinqs {

namespace {

__global__ void k_pack_eri(const double *eri, int norb, double *packed, float *packed32) {
    // one thread per packed entry: decode (a >= b) pair-of-pairs, then (p >= q), (r >= s)
    int m = norb * (norb + 1) / 2;
    int64_t total = (int64_t)m * (m + 1) / 2;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int a = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
    while ((int64_t)a * (a + 1) / 2 > t) --a;
    while ((int64_t)(a + 1) * (a + 2) / 2 <= t) ++a;
    int b = (int)(t - (int64_t)a * (a + 1) / 2);
    int p = (int)((sqrt(8.0 * a + 1.0) - 1.0) / 2.0);
    while (p * (p + 1) / 2 > a) --p;
    while ((p + 1) * (p + 2) / 2 <= a) ++p;
    int q = a - p * (p + 1) / 2;
    int r = (int)((sqrt(8.0 * b + 1.0) - 1.0) / 2.0);
    while (r * (r + 1) / 2 > b) --r;
    while ((r + 1) * (r + 2) / 2 <= b) ++r;
    int s = b - r * (r + 1) / 2;
    double v = eri[(((int64_t)p * norb + q) * norb + r) * norb + s];
    packed[t] = v;
    packed32[t] = (float)v;
}

struct ElemArgs {
    int64_t ndet;
    int norb;
    int npack;
    double ecore;
    const uint32_t *sa, *sb;
    const int64_t *rowptr;
    const uint32_t *desc;
    const double *eri;   // packed
    const double *h;
    double *val;
    float *val32;
    double *diag;
    float *diag32;
    const int64_t *skip;  // per row: leading entries whose values are already set (or null)
};

// One wave per row; lanes stride over the row's couplings.  Integrals in LDS
// (USE_LDS) or read through the caches for orbital counts whose packed tensor
// exceeds the LDS.
template <bool USE_LDS>
__global__ __launch_bounds__(256) void k_elements(ElemArgs a) {
    extern __shared__ double smem[];
    const double *eri = a.eri;
    const double *h = a.h;
    if (USE_LDS) {
        for (int t = threadIdx.x; t < a.npack; t += blockDim.x) smem[t] = a.eri[t];
        for (int t = threadIdx.x; t < a.norb * a.norb; t += blockDim.x) smem[a.npack + t] = a.h[t];
        __syncthreads();
        eri = smem;
        h = smem + a.npack;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int64_t row = (int64_t)blockIdx.x * nw + wave; row < a.ndet; row += (int64_t)gridDim.x * nw) {
        const uint32_t ai = a.sa[row], bi = a.sb[row];
        const int64_t beg = a.rowptr[row] + (a.skip ? a.skip[row] : 0), end = a.rowptr[row + 1];
        for (int64_t e = beg + lane; e < end; e += 64) {
            const double v = coupling_value(eri, h, a.norb, a.desc[e], ai, bi);
            a.val[e] = v;
            a.val32[e] = (float)v;
        }
    }
}

template <bool USE_LDS>
__global__ __launch_bounds__(256) void k_diag(ElemArgs a) {
    extern __shared__ double smem[];
    const double *eri = a.eri;
    const double *h = a.h;
    if (USE_LDS) {
        for (int t = threadIdx.x; t < a.npack; t += blockDim.x) smem[t] = a.eri[t];
        for (int t = threadIdx.x; t < a.norb * a.norb; t += blockDim.x) smem[a.npack + t] = a.h[t];
        __syncthreads();
        eri = smem;
        h = smem + a.npack;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.ndet;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = diag_value(eri, h, a.norb, a.ecore, a.sa[i], a.sb[i]);
        a.diag[i] = v;
        a.diag32[i] = (float)v;
    }
}

}  // namespace

void build_integrals(Ctx &c, int norb, const double *h, const double *eri, double ecore) {
    const int64_t n2 = (int64_t)norb * norb, n4 = n2 * n2;
    double hmax = 0.0, gmax = 0.0;
    for (int64_t t = 0; t < n2; ++t) {
        if (!std::isfinite(h[t])) throw Error(HINQS_E_NONFINITE, "h contains NaN/Inf");
        hmax = std::fmax(hmax, std::fabs(h[t]));
    }
    for (int64_t t = 0; t < n4; ++t) {
        if (!std::isfinite(eri[t])) throw Error(HINQS_E_NONFINITE, "eri contains NaN/Inf");
        gmax = std::fmax(gmax, std::fabs(eri[t]));
    }
    if (!std::isfinite(ecore)) throw Error(HINQS_E_NONFINITE, "e_core is NaN/Inf");
    const double htol = 1e-12 * (hmax > 0 ? hmax : 1.0), gtol = 1e-12 * (gmax > 0 ? gmax : 1.0);
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            if (std::fabs(h[p * norb + q] - h[q * norb + p]) > htol)
                throw Error(HINQS_E_ASYMMETRIC, "h is not symmetric");
    auto G = [&](int p, int q, int r, int s) { return eri[((int64_t)(p * norb + q) * norb + r) * norb + s]; };
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            for (int r = 0; r < norb; ++r)
                for (int s = 0; s < norb; ++s) {
                    double v = G(p, q, r, s);
                    if (std::fabs(v - G(q, p, r, s)) > gtol || std::fabs(v - G(p, q, s, r)) > gtol ||
                        std::fabs(v - G(r, s, p, q)) > gtol)
                        throw Error(HINQS_E_ASYMMETRIC, "eri lacks 8-fold real-orbital symmetry");
                }
    c.norb = norb;
    c.ecore = ecore;
    c.h_host.assign(h, h + n2);
    c.eri_host.assign(eri, eri + n4);
    hipStream_t s = c.stream;
    c.d_h.ensure(n2);
    HQ_CHECK(hipMemcpyAsync(c.d_h.p, h, sizeof(double) * n2, hipMemcpyHostToDevice, s));
    auto &full = c.bs.eri_full;
    full.ensure(n4);
    HQ_CHECK(hipMemcpyAsync(full.p, eri, sizeof(double) * n4, hipMemcpyHostToDevice, s));
    const int np = neri_packed(norb);
    c.d_eri.ensure(np);
    c.d_eri32.ensure(np);
    hipLaunchKernelGGL(k_pack_eri, dim3(grid_for(np, 256)), dim3(256), 0, s, full.p, norb, c.d_eri.p,
                       c.d_eri32.p);
    HQ_LAUNCH_CHECK();
    wait_stream(s);
    c.have_ints = true;
}

void build_elements(Ctx &c) { build_elements_after(c, nullptr); }

void build_elements_after(Ctx &c, const int64_t *skip) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c.stream;
    const int np = neri_packed(c.norb);
    c.val.ensure(c.nnz);
    c.val32.ensure(c.nnz);
    c.diag.ensure(c.ndet);
    c.diag32.ensure(c.ndet);
    ElemArgs a{c.ndet, c.norb, np, c.ecore, c.sa.p, c.sb.p, c.rowptr.p, c.desc.p, c.d_eri.p, c.d_h.p,
               c.val.p, c.val32.p, c.diag.p, c.diag32.p, skip};
    const size_t lds = sizeof(double) * ((size_t)np + (size_t)c.norb * c.norb);
    const bool use_lds = lds <= 150 * 1024;
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c.device);
    unsigned grid_rows = (unsigned)std::min<int64_t>((c.ndet + 3) / 4, (int64_t)dev_cus * 8);
    unsigned grid_diag = (unsigned)std::min<int64_t>((c.ndet + 255) / 256, (int64_t)dev_cus * 8);
    if (grid_rows < 1) grid_rows = 1;
    if (grid_diag < 1) grid_diag = 1;
    if (use_lds) {
        HQ_CHECK(hipFuncSetAttribute((const void *)k_elements<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        HQ_CHECK(hipFuncSetAttribute((const void *)k_diag<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        if (c.nnz > 0) {
            hipLaunchKernelGGL(k_elements<true>, dim3(grid_rows), dim3(256), lds, s, a);
            HQ_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_diag<true>, dim3(grid_diag), dim3(256), lds, s, a);
        HQ_LAUNCH_CHECK();
    } else {
        if (c.nnz > 0) {
            hipLaunchKernelGGL(k_elements<false>, dim3(grid_rows), dim3(256), 0, s, a);
            HQ_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_diag<false>, dim3(grid_diag), dim3(256), 0, s, a);
        HQ_LAUNCH_CHECK();
    }
    wait_stream(s);
    c.have_elements = true;
    c.ms_elements =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hinqs
