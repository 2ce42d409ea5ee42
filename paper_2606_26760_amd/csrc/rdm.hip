// One- and two-particle density matrices of a vector over B, and the energy
// gradient with respect to the integrals built from them.
//
//   rdm1[p,q]     = sum_s  <c| a+_{ps} a_{qs} |c>
//   rdm2[p,q,r,s] = sum_st <c| a+_{ps} a+_{rt} a_{st} a_{qs} |c>
//
// Every stored coupling (i <- j) contributes c_i c_j times its canonical sign
// to a few entries; the diagonal contributes c_i^2 times occupation products.
// Work is split so that only the double-excitation entries need scattered
// updates of the norb^4 tensor:
//   * diagonal:  Psame[k][l] = sum c_i^2 (n_ka n_la + n_kb n_lb), Pab[k][l] =
//     sum c_i^2 n_ka n_lb, occ[k] = sum c_i^2 (n_ka + n_kb)  (LDS, norb^2)
//   * singles q -> p: rdm1[p][q] += w;  Sc[p][q][k] += w for every electron k
//     the two determinants share (Coulomb-like terms rdm2[p,q,k,k] and
//     rdm2[k,k,p,q]); Sx[p][q][k] += w for the same-spin ones (exchange-like
//     rdm2[p,k,k,q], rdm2[k,q,p,k] with a minus sign)  (LDS, norb^3)
//   * doubles:  rdm2 entries atomically added into one of NCOPY global copies
//     chosen by workgroup, to spread contention.  A double adds the same
//     weight to rdm2[p,q,r,s] and to its pair swap rdm2[r,s,p,q], so only the
//     first of each such pair is accumulated (one entry for an alpha-beta
//     double, two for a same-spin one) and the assembly adds the swap.
// The coupling set is symmetric and the vector real, so the coupling (j <- i)
// contributes to the index-transposed entries exactly what (i <- j) does
// (rdm2[p,q,r,s] -> rdm2[q,p,s,r], rdm1[p,q] -> rdm1[q,p], Sc/Sx[p][q][k] ->
// [q][p][k]): only entries with j < i are visited, and the assembly adds the
// transposes.  A final kernel assembles rdm1/rdm2 from the tables and sums
// the copies in a fixed order.  The floating-point atomics make the result
// reproducible to rounding, not bitwise.
#include "common.hpp"

namespace hinqs {

namespace {

constexpr int NCOPY = 32;

struct RdmArgs {
    int64_t ndet;
    int norb;
    const uint32_t *sa, *sb;
    const int64_t *rowptr;
    const int32_t *col;
    const uint32_t *desc;
    const double *c;
    double *g2;      // NCOPY x norb^4
    double *tab;     // per-copy tables when not in LDS: NCOPY x ntab
    int ntab;        // doubles per table set
};

// Table layout (one set): Sc[norb^3] | Sx[norb^3] | rdm1[norb^2] | Psame[norb^2] | Pab[norb^2] | occ[norb]
__host__ __device__ inline int tab_size(int n) { return 2 * n * n * n + 3 * n * n + n; }

template <bool LDS>
__global__ __launch_bounds__(256) void k_rdm(RdmArgs a) {
    extern __shared__ double sm[];
    const int n = a.norb, n2 = n * n, n3 = n2 * n;
    const int copy = blockIdx.x % NCOPY;
    double *tab = LDS ? sm : a.tab + (int64_t)copy * a.ntab;
    if (LDS) {
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) tab[t] = 0.0;
        __syncthreads();
    }
    double *Sc = tab, *Sx = tab + n3, *g1 = tab + 2 * n3, *Ps = g1 + n2, *Pab = Ps + n2, *occ = Pab + n2;
    double *g2 = a.g2 + (int64_t)copy * n2 * n2;
    auto G2 = [&](int p, int q, int r, int s, double v) {
        atomicAdd(&g2[((p * n + q) * n + r) * n + s], v);
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t row = (int64_t)blockIdx.x * nw + wave; row < a.ndet; row += (int64_t)gridDim.x * nw) {
        const double ci = a.c[row];
        const uint32_t ai = a.sa[row], bi = a.sb[row];
        if (ci != 0.0) {
            // diagonal: occupied pairs spread over lanes
            const double w = ci * ci;
            const int na = popc32(ai), nb = popc32(bi);
            const int ntot = na + nb;
            for (int t = lane; t < ntot * ntot; t += 64) {
                const int x = t / ntot, y = t % ntot;
                // x-th and y-th occupied spin-orbital (alpha first)
                uint32_t sx = x < na ? ai : bi, sy = y < na ? ai : bi;
                int ix = x < na ? x : x - na, iy = y < na ? y : y - na;
                for (int q = 0; q < ix; ++q) sx &= sx - 1;
                for (int q = 0; q < iy; ++q) sy &= sy - 1;
                const int k = lowbit(sx), l = lowbit(sy);
                const bool xa = x < na, ya = y < na;
                if (x == y) {
                    atomicAdd(&occ[k], w);
                } else if (xa == ya) {
                    atomicAdd(&Ps[k * n + l], w);
                } else if (xa) {
                    atomicAdd(&Pab[k * n + l], w);
                }
            }
        }
        const int64_t beg = a.rowptr[row], end = a.rowptr[row + 1];
        for (int64_t e = beg + lane; e < end; e += 64) {
            const int32_t j = a.col[e];
            if (j > row) continue;  // its mirror (row <- j) is the transpose
            const double cj = a.c[j];
            const uint32_t d = a.desc[e];
            double w = ci * cj;
            if (w == 0.0) continue;
            if (desc_neg(d)) w = -w;
            const uint32_t type = desc_type(d);
            const int h1 = desc_h1(d), h2 = desc_h2(d), p1 = desc_p1(d), p2 = desc_p2(d);
            if (type == HINQS_EXC_1A || type == HINQS_EXC_1B) {
                const int p = p1, q = h1;
                const uint32_t same = (type == HINQS_EXC_1A ? ai : bi) & ~(1u << p);
                const uint32_t other = (type == HINQS_EXC_1A ? bi : ai);
                atomicAdd(&g1[p * n + q], w);
                for (uint32_t m = same; m; m &= m - 1) {
                    const int k = lowbit(m);
                    atomicAdd(&Sc[(p * n + q) * n + k], w);
                    atomicAdd(&Sx[(p * n + q) * n + k], w);
                }
                for (uint32_t m = other; m; m &= m - 1) {
                    const int k = lowbit(m);
                    atomicAdd(&Sc[(p * n + q) * n + k], w);
                }
            } else if (type == HINQS_EXC_2AB) {
                G2(p1, h1, p2, h2, w);  // + pair swap (p2, h2, p1, h1) at assembly
            } else {
                G2(p1, h1, p2, h2, w);  // + (p2, h2, p1, h1)
                G2(p1, h2, p2, h1, -w);  // + (p2, h1, p1, h2)
            }
        }
    }
    if (LDS) {
        __syncthreads();
        double *dst = a.tab + (int64_t)copy * a.ntab;
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) atomicAdd(&dst[t], tab[t]);
    }
}

// rdm1 / rdm2 from the copies and tables (fixed summation order over copies).
__global__ void k_rdm_assemble(int norb, const double *g2c, const double *tabc, int ntab, double *rdm1,
                               double *rdm2) {
    const int n = norb, n2 = n * n, n3 = n2 * n;
    const int64_t n4 = (int64_t)n2 * n2;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const int s = (int)(t % n), r = (int)((t / n) % n), q = (int)((t / n2) % n), p = (int)(t / n3);
    const int64_t tt = ((int64_t)(q * n + p) * n + s) * n + r;  // transpose (q, p, s, r)
    const int64_t tp = ((int64_t)(r * n + s) * n + p) * n + q;  // pair swap (r, s, p, q)
    const int64_t tq = ((int64_t)(s * n + r) * n + q) * n + p;  // both (s, r, q, p)
    double v = 0.0;
    for (int cpy = 0; cpy < NCOPY; ++cpy) {
        const double *g = g2c + (int64_t)cpy * n4;
        v += (g[t] + g[tt]) + (g[tp] + g[tq]);
    }
    double sc1 = 0, sc2 = 0, sx1 = 0, sx2 = 0, ps = 0, pab = 0, pba = 0, pex = 0;
    for (int cpy = 0; cpy < NCOPY; ++cpy) {
        const double *tb = tabc + (int64_t)cpy * ntab;
        const double *Sc = tb, *Sx = tb + n3, *Ps = tb + 2 * n3 + n2, *Pab = Ps + n2;
        if (r == s) sc1 += Sc[(p * n + q) * n + r] + Sc[(q * n + p) * n + r];
        if (p == q) sc2 += Sc[(r * n + s) * n + p] + Sc[(s * n + r) * n + p];
        if (q == r) sx1 += Sx[(p * n + s) * n + q] + Sx[(s * n + p) * n + q];
        if (p == s) sx2 += Sx[(r * n + q) * n + p] + Sx[(q * n + r) * n + p];
        if (p == q && r == s) {
            if (p != r) ps += Ps[p * n + r];
            pab += Pab[p * n + r];
            pba += Pab[r * n + p];
        }
        if (q == r && p == s && p != q) pex += Ps[p * n + q];
    }
    v += sc1 + sc2 - sx1 - sx2 + ps + pab + pba - pex;
    rdm2[t] = v;
    if (t < n2) {
        const int pp = (int)(t / n), qq = (int)(t % n);
        double g = 0.0;
        for (int cpy = 0; cpy < NCOPY; ++cpy) {
            const double *tb = tabc + (int64_t)cpy * ntab;
            g += tb[2 * n3 + pp * n + qq] + tb[2 * n3 + qq * n + pp];
            if (pp == qq) g += tb[2 * n3 + 3 * n2 + pp];
        }
        rdm1[t] = g;
    }
}

__global__ void k_grad(int norb, const double *rdm1, const double *rdm2, double scale, double *gh,
                       double *geri) {
    const int n = norb, n2 = n * n, n3 = n2 * n;
    const int64_t n4 = (int64_t)n2 * n2;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const int s = (int)(t % n), r = (int)((t / n) % n), q = (int)((t / n2) % n), p = (int)(t / n3);
    auto R = [&](int a, int b, int c, int d) { return rdm2[((a * n + b) * n + c) * n + d]; };
    double v = R(p, q, r, s) + R(q, p, r, s) + R(p, q, s, r) + R(q, p, s, r) + R(r, s, p, q) +
               R(s, r, p, q) + R(r, s, q, p) + R(s, r, q, p);
    geri[t] = scale * 0.5 * v / 8.0;
    if (t < n2) {
        const int pp = (int)(t / n), qq = (int)(t % n);
        gh[t] = scale * 0.5 * (rdm1[pp * n + qq] + rdm1[qq * n + pp]);
    }
}

}  // namespace

void rdm12_sorted(Ctx &c, const double *cs, double *rdm1, double *rdm2) {
    hipStream_t s = c.stream;
    const int n = c.norb;
    const int64_t n4 = (int64_t)n * n * n * n;
    const int ntab = tab_size(n);
    // accumulation copies in the context's call scratch (slots 2 and 3; slot
    // 0 may hold the gathered coefficients), kept for the next call
    double *g2c = c.cs.get<double>(2, (size_t)NCOPY * n4);
    double *tabc = c.cs.get<double>(3, (size_t)NCOPY * ntab);
    HQ_CHECK(hipMemsetAsync(g2c, 0, sizeof(double) * NCOPY * n4, s));
    HQ_CHECK(hipMemsetAsync(tabc, 0, sizeof(double) * NCOPY * ntab, s));
    RdmArgs a{c.ndet, n, c.sa.p, c.sb.p, c.rowptr.p, c.col.p, c.desc.p, cs, g2c, tabc, ntab};
    const size_t lds = sizeof(double) * (size_t)ntab;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
    unsigned grid = (unsigned)std::min<int64_t>((c.ndet + 3) / 4, (int64_t)cus * 4);
    if (grid < 1) grid = 1;
    if (lds <= 150 * 1024) {
        HQ_CHECK(hipFuncSetAttribute((const void *)k_rdm<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
        hipLaunchKernelGGL(k_rdm<true>, dim3(grid), dim3(256), lds, s, a);
    } else {
        hipLaunchKernelGGL(k_rdm<false>, dim3(grid), dim3(256), 0, s, a);
    }
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rdm_assemble, dim3(grid_for(n4, 256)), dim3(256), 0, s, n, g2c, tabc, ntab,
                       rdm1, rdm2);
    HQ_LAUNCH_CHECK();
}

void integral_grad_sorted(Ctx &c, const double *cs, double scale, double *gh, double *geri) {
    hipStream_t s = c.stream;
    const int n = c.norb;
    const int64_t n4 = (int64_t)n * n * n * n;
    double *r1 = c.cs.get<double>(4, (size_t)n * n + (size_t)n4);  // rdm1, then rdm2
    double *r2 = r1 + (size_t)n * n;
    rdm12_sorted(c, cs, r1, r2);
    hipLaunchKernelGGL(k_grad, dim3(grid_for(n4, 256)), dim3(256), 0, s, n, r1, r2, scale, gh, geri);
    HQ_LAUNCH_CHECK();
}

}  // namespace hinqs
