// Slater-Condon matrix elements of the Hamiltonian of Sec. 2.2 from a pair
// descriptor and the bra's strings, and the diagonal element of a
// determinant, with the integrals in the packed 8-fold layout (LDS or
// global).  Shared by the element builder and the selection kernels.
//
// Element rules for <x_i|H|x_j> (x_i the bra; holes occupied in x_j,
// particles in x_i; s the canonical sign stored in the descriptor):
//   diagonal        E_core + sum_k h_kk + 1/2 sum_{k,l}[(kk|ll) - delta_spin (kl|lk)]
//   single q -> p   s [h_pq + sum_{k in common, same spin} ((pq|kk) - (pk|kq))
//                        + sum_{k, other spin} (pq|kk)]
//   same-spin double  s [(p1 h1|p2 h2) - (p1 h2|p2 h1)]
//   opposite-spin     s (pa ha|pb hb)
#pragma once

#include "common.hpp"

namespace hinqs {

__device__ inline double single_value(const double *eri, const double *h, int norb, int p, int q,
                                      uint32_t common_same, uint32_t other) {
    double v = h[p * norb + q];
    for (uint32_t m = common_same; m; m &= m - 1) {
        int k = lowbit(m);
        v += eri[eri_index(p, q, k, k)] - eri[eri_index(p, k, k, q)];
    }
    for (uint32_t m = other; m; m &= m - 1) {
        int k = lowbit(m);
        v += eri[eri_index(p, q, k, k)];
    }
    return v;
}

// <x_i|H|x_j> for the pair with descriptor d; (ai, bi) are the bra's strings.
__device__ inline double coupling_value(const double *eri, const double *h, int norb, uint32_t d, uint32_t ai,
                                        uint32_t bi) {
    const uint32_t type = desc_type(d);
    const int h1 = desc_h1(d), h2 = desc_h2(d), p1 = desc_p1(d), p2 = desc_p2(d);
    double v;
    if (type == HINQS_EXC_1A) {
        v = single_value(eri, h, norb, p1, h1, ai & ~(1u << p1), bi);
    } else if (type == HINQS_EXC_1B) {
        v = single_value(eri, h, norb, p1, h1, bi & ~(1u << p1), ai);
    } else if (type == HINQS_EXC_2AB) {
        v = eri[eri_index(p1, h1, p2, h2)];
    } else {
        v = eri[eri_index(p1, h1, p2, h2)] - eri[eri_index(p1, h2, p2, h1)];
    }
    return desc_neg(d) ? -v : v;
}

// <x|H|x> for the determinant with strings (a, b).
__device__ inline double diag_value(const double *eri, const double *h, int norb, double ecore, uint32_t a,
                                    uint32_t b) {
    double e1 = 0.0, e2 = 0.0;
    for (uint32_t m = a; m; m &= m - 1) {
        int k = lowbit(m);
        e1 += h[k * norb + k];
        for (uint32_t n = a; n; n &= n - 1) {
            int l = lowbit(n);
            e2 += eri[eri_index(k, k, l, l)] - eri[eri_index(k, l, l, k)];
        }
        for (uint32_t n = b; n; n &= n - 1) {
            int l = lowbit(n);
            e2 += 2.0 * eri[eri_index(k, k, l, l)];
        }
    }
    for (uint32_t m = b; m; m &= m - 1) {
        int k = lowbit(m);
        e1 += h[k * norb + k];
        for (uint32_t n = b; n; n &= n - 1) {
            int l = lowbit(n);
            e2 += eri[eri_index(k, k, l, l)] - eri[eri_index(k, l, l, k)];
        }
    }
    return ecore + e1 + 0.5 * e2;
}

}  // namespace hinqs
