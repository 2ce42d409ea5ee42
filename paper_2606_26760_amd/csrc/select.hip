// Selection steps around the subspace solve (Sec. 2.2): the classical
// expansion of Eq. 2 (every determinant outside B that H connects to one of
// the largest-|c| determinants of B), the PT2 importance of Eq. 3 (the
// numerator sum_i c_i <x|H|x_i> of a candidate x over B, its diagonal H_xx
// and the score), and a stable top-k over a vector of scores, used both for
// the cold-start ranking by H_xx and for keeping the best-scored candidates.
//
// Both the expansion and the PT2 numerator reach into B only through its
// sorted string tables: alpha groups (distinct alpha strings ua, rows
// ga[g] .. ga[g+1] with ascending beta strings sb) and beta groups (distinct
// beta strings ub, entries gb[g] .. gb[g+1] of the beta-major listing bperm
// with their alpha strings bm_alpha).  A determinant is found by two binary
// searches; every partner of a candidate is found by scanning at most
// 2 + na (norb - na) groups.  Matrix elements follow slater.hpp, with the
// packed integrals in LDS when they fit.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "slater.hpp"

namespace hinqs {

namespace {

constexpr int EX_NT = 256;  // expansion: one workgroup per chosen determinant at a time
constexpr int PT_NT = 1024; // PT2: one wave per candidate at a time
constexpr int NPAIR32 = 32 * 31 / 2;

struct BTables {
    int32_t nua, nub;
    const uint32_t *ua, *ub;      // distinct strings, ascending
    const uint32_t *sa, *sb;      // strings in sorted order
    const int32_t *ga, *gb;       // group offsets
    const int32_t *bperm;         // beta-major listing of sorted positions
    const uint32_t *bm_alpha;     // alpha string of bperm[u]
};

BTables tables_of(const Ctx &c) {
    return BTables{c.nua, c.nub, c.ua.p, c.ub.p, c.sa.p, c.sb.p, c.ga.p, c.gb.p, c.bperm.p, c.bm_alpha.p};
}

// Index of x in the ascending array v[0..n), or -1.
__device__ inline int32_t find_u32(const uint32_t *v, int32_t n, uint32_t x) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (v[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && v[lo] == x) ? lo : -1;
}

// Sorted position of the determinant (a, b) in B, or -1.
__device__ inline int64_t find_det(const BTables &t, uint32_t a, uint32_t b) {
    const int32_t g = find_u32(t.ua, t.nua, a);
    if (g < 0) return -1;
    const int32_t lo = t.ga[g], hi = t.ga[g + 1];
    const int32_t r = find_u32(t.sb + lo, hi - lo, b);
    return r < 0 ? -1 : (int64_t)lo + r;
}

// Orbital of the n-th set bit (from the lowest) of m; m has more than n bits.
__device__ inline int nth_bit(uint32_t m, int n) {
    for (int i = 0; i < n; ++i) m &= m - 1;
    return lowbit(m);
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Stage the packed integrals and h in LDS (USE_LDS) or point at them.
template <bool USE_LDS>
__device__ inline void stage_integrals(double *smem, const double *eri_g, const double *h_g, int npack, int norb,
                                       const double *&eri, const double *&h) {
    eri = eri_g;
    h = h_g;
    if (USE_LDS) {
        for (int t = threadIdx.x; t < npack; t += blockDim.x) smem[t] = eri_g[t];
        for (int t = threadIdx.x; t < norb * norb; t += blockDim.x) smem[npack + t] = h_g[t];
        __syncthreads();
        eri = smem;
        h = smem + npack;
    }
}

// ------------------------------------------------------------ top-k keys
// Order-preserving unsigned image of a double (ascending values give
// ascending keys; -0 is taken as +0, so equal values tie); with `largest`
// the order is reversed.  NaN raises the flag.
__global__ void k_order_keys(const double *v, int64_t n, bool largest, uint64_t *keys, int32_t *vals,
                             unsigned *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = v[i];
    if (x != x) atomicOr(bad, 1u);
    if (x == 0.0) x = 0.0;
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    uint64_t k = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    keys[i] = largest ? ~k : k;
    vals[i] = (int32_t)i;
}

// Keys ordering |c| descending; non-finite c raises the flag.
__global__ void k_mag_keys(const double *c, int64_t n, uint64_t *keys, int32_t *vals, unsigned *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = c[i];
    if (!isfinite(x)) atomicOr(bad, 1u);
    keys[i] = 0x7fffffffffffffffull - (uint64_t)__double_as_longlong(fabs(x));
    vals[i] = (int32_t)i;
}

// top_out[t] = vals[t] (index in the caller's order of the vector); pos[t] =
// its sorted position.
__global__ void k_take_top(const int32_t *vals, int64_t ntop, const int32_t *inv, int32_t *top_out,
                           int32_t *pos) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntop) return;
    const int32_t v = vals[t];
    if (top_out) top_out[t] = v;
    if (pos) pos[t] = inv ? inv[v] : v;
}

// ------------------------------------------------------ classical expansion
struct ExpArgs {
    BTables B;
    int norb, npack, na, nb;
    int64_t ntop;
    const int32_t *pos;  // sorted positions of the chosen determinants
    const double *eri, *h;
    uint64_t *keys;      // ntop * (excitations per determinant) entries
    unsigned long long *count;
};

// Every single and double excitation y of a chosen determinant x, indexed
// r = 0 .. nexc-1 in five ranges: alpha singles, beta singles, alpha-alpha
// doubles, beta-beta doubles, alpha-beta doubles.  y is kept when
// <y|H|x> != 0 and y is not in B; kept keys (alpha << norb | beta) are
// appended with one atomic per wave.
template <bool USE_LDS>
__global__ __launch_bounds__(EX_NT) void k_expand(ExpArgs a) {
    extern __shared__ double smem[];
    __shared__ uint16_t pairs[NPAIR32];      // k = j (j - 1) / 2 + i  ->  i | j << 8, i < j
    __shared__ uint8_t occ[2][32], vir[2][32];
    const double *eri, *h;
    stage_integrals<USE_LDS>(smem, a.eri, a.h, a.npack, a.norb, eri, h);
    for (int k = threadIdx.x; k < NPAIR32; k += blockDim.x) {
        int j = 1;
        while ((j + 1) * j / 2 <= k) ++j;
        pairs[k] = (uint16_t)((k - j * (j - 1) / 2) | (j << 8));
    }
    const int norb = a.norb, na = a.na, nb = a.nb, nva = norb - na, nvb = norb - nb;
    const uint32_t full = norb >= 32 ? 0xffffffffu : ((1u << norb) - 1u);
    const int64_t sA = (int64_t)na * nva, sB = (int64_t)nb * nvb;
    const int64_t cva = (int64_t)nva * (nva - 1) / 2, cvb = (int64_t)nvb * (nvb - 1) / 2;
    const int64_t dAA = (int64_t)na * (na - 1) / 2 * cva, dBB = (int64_t)nb * (nb - 1) / 2 * cvb;
    const int64_t total = sA + sB + dAA + dBB + sA * sB;
    const int lane = threadIdx.x & 63;
    for (int64_t t = blockIdx.x; t < a.ntop; t += gridDim.x) {
        const int32_t p = a.pos[t];
        const uint32_t xa = a.B.sa[p], xb = a.B.sb[p];
        __syncthreads();  // the previous determinant's lists are no longer read
        if (threadIdx.x < 2) {
            const uint32_t s = threadIdx.x == 0 ? xa : xb;
            int no = 0, nv = 0;
            for (int q = 0; q < norb; ++q) {
                if ((s >> q) & 1u)
                    occ[threadIdx.x][no++] = (uint8_t)q;
                else
                    vir[threadIdx.x][nv++] = (uint8_t)q;
            }
        }
        __syncthreads();
        for (int64_t r0 = 0; r0 < total; r0 += EX_NT) {
            int64_t r = r0 + threadIdx.x;
            bool keep = false;
            uint64_t key = 0;
            if (r < total) {
                uint32_t ya = xa, yb = xb;
                if (r < sA) {
                    ya ^= (1u << occ[0][r / nva]) | (1u << vir[0][r % nva]);
                } else if ((r -= sA) < sB) {
                    yb ^= (1u << occ[1][r / nvb]) | (1u << vir[1][r % nvb]);
                } else if ((r -= sB) < dAA) {
                    const int po = pairs[r / cva], pv = pairs[r % cva];
                    ya ^= (1u << occ[0][po & 255]) | (1u << occ[0][po >> 8]) | (1u << vir[0][pv & 255]) |
                          (1u << vir[0][pv >> 8]);
                } else if ((r -= dAA) < dBB) {
                    const int po = pairs[r / cvb], pv = pairs[r % cvb];
                    yb ^= (1u << occ[1][po & 255]) | (1u << occ[1][po >> 8]) | (1u << vir[1][pv & 255]) |
                          (1u << vir[1][pv >> 8]);
                } else {
                    r -= dBB;
                    const int64_t s1 = r / sB, s2 = r % sB;
                    ya ^= (1u << occ[0][s1 / nva]) | (1u << vir[0][s1 % nva]);
                    yb ^= (1u << occ[1][s2 / nvb]) | (1u << vir[1][s2 % nvb]);
                }
                const double v = coupling_value(eri, h, norb, pair_desc(ya, yb, xa, xb), ya, yb);
                if (v != 0.0 && find_det(a.B, ya, yb) < 0) {
                    keep = true;
                    key = ((uint64_t)ya << norb) | (uint64_t)(yb & full);
                }
            }
            const uint64_t m = __ballot(keep);
            if (m) {
                const int leader = __builtin_ctzll(m);
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(a.count, (unsigned long long)__popcll(m));
                base = __shfl(base, leader, 64);
                if (keep) a.keys[base + __popcll(m & ((1ull << lane) - 1ull))] = key;
            }
        }
    }
}

__global__ void k_unique_flags(const uint64_t *keys, int64_t n, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_unique_write(const uint64_t *keys, const int32_t *flag, const int32_t *pos, int64_t n,
                               int norb, int64_t cap, uint64_t *out_a, uint64_t *out_b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int64_t p = pos[i];
    if (p >= cap) return;
    const uint64_t lo = norb >= 64 ? ~0ull : ((1ull << norb) - 1ull);
    out_a[p] = keys[i] >> norb;
    out_b[p] = keys[i] & lo;
}

// ------------------------------------------------------------------- PT2
struct Pt2Args {
    BTables B;
    int norb, npack, na, nb;
    int alink_max;
    const int32_t *alink_ptr, *alink;  // single alpha moves between strings of B
    double ecore, e0;
    int64_t ncand;
    const uint64_t *ca, *cb;
    const double *cs;  // coefficients in sorted order
    const double *eri, *h;
    double *numer, *hxx, *score;
    unsigned *bad;
};

constexpr int SCAN_U = 8;  // group entries in flight per lane

// acc += c_j <x|H|x_j> over the rows j in [lo, hi) of one alpha group (alpha
// string aj) whose beta string differs from xb by a number of electrons in
// the accepted set: SAME_ALPHA accepts 0 (the diagonal d), 1 or 2 electrons,
// otherwise exactly one.
template <bool SAME_ALPHA>
__device__ inline void scan_alpha_group(const Pt2Args &a, const double *eri, const double *h, int32_t lo,
                                        int32_t hi, uint32_t xa, uint32_t xb, uint32_t aj, double d, int lane,
                                        double &acc) {
    for (int32_t j0 = lo + lane; j0 < hi; j0 += 64 * SCAN_U) {
        uint32_t bj[SCAN_U];
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            const int32_t j = j0 + 64 * u;
            bj[u] = j < hi ? a.B.sb[j] : ~xb;
        }
        uint32_t m = 0, m0 = 0;  // entries needing a coupling value / the diagonal
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            const int db = popc32(xb ^ bj[u]);
            if (SAME_ALPHA) {
                m0 |= db == 0 ? 1u << u : 0u;
                m |= (db != 0 && db <= 4) ? 1u << u : 0u;
            } else {
                m |= db == 2 ? 1u << u : 0u;
            }
        }
        // the hits in ascending order, so every lane sums its entries in group order
        for (uint32_t mm = m | m0; mm; mm &= mm - 1) {
            const int u = lowbit(mm);
            const int32_t j = j0 + 64 * u;
            const double v =
                (m0 >> u) & 1u ? d : coupling_value(eri, h, a.norb, pair_desc(xa, xb, aj, a.B.sb[j]), xa, xb);
            acc += a.cs[j] * v;
        }
    }
}

// Linked alpha groups of at most PT2_GL * SCAN_U rows are scanned 64 / PT2_GL
// at a time, PT2_GL lanes each and in a single step, so the chain of
// dependent loads per candidate runs over a few batches of groups instead of
// every group one after another.
constexpr int PT2_GL = 32;
constexpr int PT2_SMALL = PT2_GL * SCAN_U;

// acc += c_j <x|H|x_j> over the rows j in [lo, hi) (at most PT2_SMALL of them)
// of one alpha group (alpha string aj) whose beta string is one electron from
// xb; sl is this lane's index among the PT2_GL lanes sharing the group.
__device__ inline void scan_small_group(const Pt2Args &a, const double *eri, const double *h, int32_t lo,
                                        int32_t hi, uint32_t xa, uint32_t xb, uint32_t aj, int sl, double &acc) {
    uint32_t bj[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
        const int32_t j = lo + sl + PT2_GL * u;
        bj[u] = j < hi ? a.B.sb[j] : ~xb;
    }
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) m |= popc32(xb ^ bj[u]) == 2 ? 1u << u : 0u;
    for (; m; m &= m - 1) {
        const int32_t j = lo + sl + PT2_GL * lowbit(m);
        acc += a.cs[j] * coupling_value(eri, h, a.norb, pair_desc(xa, xb, aj, a.B.sb[j]), xa, xb);
    }
}

// Candidate order for PT2: key (alpha << norb | beta) of each candidate
// (0 for a malformed one; the main kernel checks every candidate itself).
__global__ void k_pt2_keys(const uint64_t *ca, const uint64_t *cb, int64_t n, int norb, uint64_t *keys,
                           int32_t *vals) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint64_t a = ca[t], b = cb[t];
    keys[t] = ((a >> norb) | (b >> norb)) ? 0ull : ((a << norb) | b);
    vals[t] = (int32_t)t;
}

// Groups of each candidate (in key order): its alpha group and beta group in
// B, or -1.  One thread per candidate, so the searches overlap.
__global__ void k_pt2_groups(const BTables B, const uint64_t *ca, const uint64_t *cb, const int32_t *order, int64_t n,
                             int norb, int32_t *ga_of, int32_t *gb_of) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int32_t t = order[u];
    const uint64_t a = ca[t], b = cb[t];
    const bool ok = ((a >> norb) | (b >> norb)) == 0;
    ga_of[u] = ok ? find_u32(B.ua, B.nua, (uint32_t)a) : -1;
    gb_of[u] = ok ? find_u32(B.ub, B.nub, (uint32_t)b) : -1;
}

// Waves take runs of PT2_RUN consecutive candidates in key order from a
// shared counter (every wave stops once the counter passes ncand), one
// candidate at a time.  Its partners in B fall into three disjoint classes, each read from
// one kind of group:
//   same alpha string        the alpha group of xa (beta differs by 0, 1 or 2)
//   same beta string         the beta group of xb (alpha differs by 1 or 2)
//   one move in each spin    the alpha groups of the strings one move from xa
//                            (link table when xa is an alpha string of B, else
//                            searched), keeping beta strings one move from xb
// The diagonal enters through the first class when x lies in B.  Candidates
// of a run mostly share xa, so the bounds of its alpha groups are loaded once
// per distinct xa and kept in the lanes (slot r of lane l: move 64 r + l;
// SLOTS * 64 >= na (norb - na)).
constexpr int PT2_RUN = 16;

template <bool USE_LDS, int SLOTS>
__global__ __launch_bounds__(PT_NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_pt2(
    Pt2Args a, const int32_t *order, const int32_t *ga_of, const int32_t *gb_of, unsigned long long *next) {
    extern __shared__ double smem[];
    const double *eri, *h;
    stage_integrals<USE_LDS>(smem, a.eri, a.h, a.npack, a.norb, eri, h);
    const int lane = threadIdx.x & 63;
    const int norb = a.norb, nva = norb - a.na, nmov = a.na * nva;
    const uint32_t full = norb >= 32 ? 0xffffffffu : ((1u << norb) - 1u);
    uint32_t cur_a = 0;
    bool have = false;
    int nlink = 0;
    int32_t lo_m[SLOTS], hi_m[SLOTS];
    uint32_t aj_m[SLOTS];
    int64_t u = 0, u_end = 0;
    for (;;) {
        if (u == u_end) {  // next run of PT2_RUN candidates from the shared counter
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(next, (unsigned long long)PT2_RUN);
            base = __shfl(base, 0, 64);
            if ((int64_t)base >= a.ncand) break;
            u = (int64_t)base;
            u_end = min(a.ncand, u + PT2_RUN);
        }
        const int32_t t = order[u];
        const uint64_t a64 = a.ca[t], b64 = a.cb[t];
        const int32_t g = ga_of[u], gbx = gb_of[u];
        ++u;
        if ((a64 >> norb) != 0 || (b64 >> norb) != 0 || (int)__popcll(a64) != a.na || (int)__popcll(b64) != a.nb) {
            if (lane == 0) {
                atomicOr(a.bad, 1u);
                const double nan = __longlong_as_double(0x7ff8000000000000ll);
                if (a.numer) a.numer[t] = nan;
                if (a.hxx) a.hxx[t] = nan;
                if (a.score) a.score[t] = nan;
            }
            continue;
        }
        const uint32_t xa = (uint32_t)a64, xb = (uint32_t)b64;
        if (!have || xa != cur_a) {  // alpha groups one move from xa
            have = true;
            cur_a = xa;
            nlink = g >= 0 ? a.alink_ptr[g] : nmov;
#pragma unroll
            for (int r = 0; r < SLOTS; ++r) {
                const int m = 64 * r + lane;
                int32_t gm = -1;
                if (m < nlink) {
                    if (g >= 0) {
                        gm = a.alink[(int64_t)g * a.alink_max + m];
                    } else {
                        const uint32_t am =
                            xa ^ (1u << nth_bit(xa, m / nva)) ^ (1u << nth_bit(~xa & full, m % nva));
                        gm = find_u32(a.B.ua, a.B.nua, am);
                    }
                }
                lo_m[r] = gm >= 0 ? a.B.ga[gm] : 0;
                hi_m[r] = gm >= 0 ? a.B.ga[gm + 1] : 0;
                aj_m[r] = gm >= 0 ? a.B.ua[gm] : 0u;
            }
        }
        const double d = diag_value(eri, h, norb, a.ecore, xa, xb);
        double acc = 0.0;
        if (g >= 0) scan_alpha_group<true>(a, eri, h, a.B.ga[g], a.B.ga[g + 1], xa, xb, xa, d, lane, acc);
        if (gbx >= 0) {
            const int32_t end = a.B.gb[gbx + 1];
            for (int32_t u0 = a.B.gb[gbx] + lane; u0 < end; u0 += 64 * SCAN_U) {
                uint32_t aj[SCAN_U];
#pragma unroll
                for (int v = 0; v < SCAN_U; ++v) {
                    const int32_t q = u0 + 64 * v;
                    aj[v] = q < end ? a.B.bm_alpha[q] : xa;
                }
                uint32_t m = 0;
#pragma unroll
                for (int v = 0; v < SCAN_U; ++v) {
                    const int da = popc32(xa ^ aj[v]);
                    m |= (da != 0 && da <= 4) ? 1u << v : 0u;
                }
                for (; m; m &= m - 1) {
                    const int32_t q = u0 + 64 * lowbit(m);
                    acc += a.cs[a.B.bperm[q]] *
                           coupling_value(eri, h, norb, pair_desc(xa, xb, a.B.bm_alpha[q], xb), xa, xb);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
            const int32_t sz = hi_m[r] - lo_m[r];
            uint64_t found = __ballot(sz > PT2_SMALL);  // large groups: the whole wave, one at a time
            while (found) {
                const int src = __builtin_ctzll(found);
                found &= found - 1;
                const int32_t lo = __shfl(lo_m[r], src, 64), hi = __shfl(hi_m[r], src, 64);
                const uint32_t aj = (uint32_t)__shfl((int)aj_m[r], src, 64);
                scan_alpha_group<false>(a, eri, h, lo, hi, xa, xb, aj, d, lane, acc);
            }
            found = __ballot(sz > 0 && sz <= PT2_SMALL);  // small groups: 64 / PT2_GL at a time
            while (found) {
                int src = -1;
#pragma unroll
                for (int k = 0; k < 64 / PT2_GL; ++k) {
                    if (found) {
                        const int f = __builtin_ctzll(found);
                        found &= found - 1;
                        if (k == lane / PT2_GL) src = f;
                    }
                }
                const int sidx = src < 0 ? 0 : src;
                const int32_t lo = __shfl(lo_m[r], sidx, 64), hi = __shfl(hi_m[r], sidx, 64);
                const uint32_t aj = (uint32_t)__shfl((int)aj_m[r], sidx, 64);
                scan_small_group(a, eri, h, lo, src < 0 ? lo : hi, xa, xb, aj, lane % PT2_GL, acc);
            }
        }
        acc = wave_sum_d(acc);
        if (lane == 0) {
            if (a.numer) a.numer[t] = acc;
            if (a.hxx) a.hxx[t] = d;
            if (a.score) a.score[t] = acc * acc / fabs(a.e0 - d);
        }
    }
}

int device_cus(const Ctx &c) {
    int n = 256;
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, c.device);
    return n;
}

size_t integral_lds(const Ctx &c) {
    return sizeof(double) * ((size_t)neri_packed(c.norb) + (size_t)c.norb * c.norb);
}

}  // namespace

int64_t excitations_per_det(int norb, int na, int nb) {
    const int64_t nva = norb - na, nvb = norb - nb;
    const int64_t sA = na * nva, sB = nb * nvb;
    return sA + sB + (int64_t)na * (na - 1) / 2 * (nva * (nva - 1) / 2) +
           (int64_t)nb * (nb - 1) / 2 * (nvb * (nvb - 1) / 2) + sA * sB;
}

void top_k(Ctx &c, int64_t n, const double *v, int64_t k, bool largest, int32_t *idx) {
    hipStream_t s = c.stream;
    uint64_t *keys = c.cs.get<uint64_t>(0, n);
    int32_t *vals = c.cs.get<int32_t>(1, n);
    unsigned *bad = (unsigned *)c.cs.words(1);
    HQ_CHECK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, v, n, largest, keys, vals, bad);
    HQ_LAUNCH_CHECK();
    radix_sort_u64(s, keys, vals, n, 64, c.work);
    unsigned hbad = 0;
    HQ_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (hbad) throw Error(HINQS_E_NONFINITE, "values contain NaN");
    hipLaunchKernelGGL(k_take_top, dim3(grid_for(k, 256)), dim3(256), 0, s, vals, k, (const int32_t *)nullptr,
                       idx, (int32_t *)nullptr);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipStreamSynchronize(s));
}

int64_t expand(Ctx &c, const double *coeffs, bool sorted, int64_t ntop, int64_t capacity, uint64_t *out_a,
               uint64_t *out_b, int32_t *top) {
    hipStream_t s = c.stream;
    const int64_t n = c.ndet;
    if (ntop > n) ntop = n;
    // the ntop largest |c| (stable: ties keep the lower index first).  Scratch
    // slots 0 and 1 hold the sort keys and values, then (stream-ordered after
    // the top ntop have been taken) the raw excitations and their sort values.
    uint64_t *keys = c.cs.get<uint64_t>(0, n);
    int32_t *vals = c.cs.get<int32_t>(1, n);
    int32_t *pos = c.cs.get<int32_t>(2, ntop);
    unsigned long long *words = c.cs.words(2);
    unsigned *bad = (unsigned *)words;
    unsigned long long *cnt = words + 1;
    HQ_CHECK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_mag_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, coeffs, n, keys, vals, bad);
    HQ_LAUNCH_CHECK();
    radix_sort_u64(s, keys, vals, n, 63, c.work);
    unsigned hbad = 0;
    HQ_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (hbad) throw Error(HINQS_E_NONFINITE, "coefficients contain NaN/Inf");
    hipLaunchKernelGGL(k_take_top, dim3(grid_for(ntop, 256)), dim3(256), 0, s, vals, ntop,
                       sorted ? (const int32_t *)nullptr : (const int32_t *)c.inv.p, top, pos);
    HQ_LAUNCH_CHECK();

    // every single and double of the chosen determinants, kept when coupled and outside B
    const int64_t nexc = excitations_per_det(c.norb, c.na, c.nb);
    const int64_t cap = ntop * nexc;
    if (cap >= ((int64_t)1 << 31))
        throw Error(HINQS_E_UNSUPPORTED, "expansion of " + std::to_string(ntop) +
                                             " determinants exceeds 2^31 excitations; expand fewer at once");
    uint64_t *raw = c.cs.get<uint64_t>(0, cap);
    HQ_CHECK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    ExpArgs ea{tables_of(c), c.norb, neri_packed(c.norb), c.na, c.nb, ntop, pos, c.d_eri.p, c.d_h.p, raw, cnt};
    const size_t lds = integral_lds(c);
    const int cus = device_cus(c);
    if (lds <= 150 * 1024) {
        HQ_CHECK(hipFuncSetAttribute((const void *)k_expand<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
        const unsigned grid = (unsigned)std::min<int64_t>(ntop, (int64_t)cus * 2);
        hipLaunchKernelGGL(k_expand<true>, dim3(grid), dim3(EX_NT), lds, s, ea);
    } else {
        const unsigned grid = (unsigned)std::min<int64_t>(ntop, (int64_t)cus * 8);
        hipLaunchKernelGGL(k_expand<false>, dim3(grid), dim3(EX_NT), 0, s, ea);
    }
    HQ_LAUNCH_CHECK();
    unsigned long long hcnt = 0;
    HQ_CHECK(hipMemcpyAsync(&hcnt, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    const int64_t nraw = (int64_t)hcnt;
    if (nraw == 0) return 0;

    // sort and drop repeats: ascending (alpha, beta)
    int32_t *rv = c.cs.get<int32_t>(1, nraw);
    radix_sort_u64(s, raw, rv, nraw, 2 * c.norb, c.work);
    int32_t *flag = c.cs.get<int32_t>(3, nraw);
    int32_t *fpos = c.cs.get<int32_t>(4, nraw);
    hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(nraw, 256)), dim3(256), 0, s, raw, nraw, flag);
    HQ_LAUNCH_CHECK();
    exclusive_scan_i32(s, flag, fpos, nraw, c.work);
    int32_t last[2] = {0, 0};
    HQ_CHECK(hipMemcpyAsync(&last[0], fpos + nraw - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&last[1], flag + nraw - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (capacity > 0) {
        hipLaunchKernelGGL(k_unique_write, dim3(grid_for(nraw, 256)), dim3(256), 0, s, raw, flag, fpos,
                           nraw, c.norb, capacity, out_a, out_b);
        HQ_LAUNCH_CHECK();
    }
    HQ_CHECK(hipStreamSynchronize(s));
    return (int64_t)last[0] + last[1];
}

void pt2(Ctx &c, const double *coeffs, bool sorted, double e0, int64_t ncand, const uint64_t *ca,
         const uint64_t *cb, double *numer, double *hxx, double *score) {
    hipStream_t s = c.stream;
    const double *csp = coeffs;
    if (!sorted) {
        double *cs = c.cs.get<double>(0, c.ndet);
        gather_rows(s, coeffs, cs, c.perm.p, c.ndet, 8);
        csp = cs;
    }
    unsigned long long *words = c.cs.words(2);
    unsigned *bad = (unsigned *)words;
    unsigned long long *next = words + 1;
    HQ_CHECK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    Pt2Args pa{tables_of(c), c.norb, neri_packed(c.norb), c.na, c.nb, c.alink_max, c.alink_ptr.p, c.alink.p,
               c.ecore, e0, ncand, ca, cb, csp, c.d_eri.p, c.d_h.p, numer, hxx, score, bad};
    // candidates in key order, and their groups in B
    uint64_t *keys = c.cs.get<uint64_t>(1, ncand);
    int32_t *order = c.cs.get<int32_t>(2, ncand);
    int32_t *ga_of = c.cs.get<int32_t>(3, ncand);
    int32_t *gb_of = c.cs.get<int32_t>(4, ncand);
    hipLaunchKernelGGL(k_pt2_keys, dim3(grid_for(ncand, 256)), dim3(256), 0, s, ca, cb, ncand, c.norb, keys,
                       order);
    HQ_LAUNCH_CHECK();
    radix_sort_u64(s, keys, order, ncand, 2 * c.norb, c.work);
    hipLaunchKernelGGL(k_pt2_groups, dim3(grid_for(ncand, 256)), dim3(256), 0, s, pa.B, ca, cb, order, ncand,
                       c.norb, ga_of, gb_of);
    HQ_LAUNCH_CHECK();
    const size_t lds = integral_lds(c);
    const int cus = device_cus(c);
    const bool use_lds = lds <= 150 * 1024;
    // resident workgroups only (two per CU); they share the candidates through a counter
    const int64_t runs = (ncand + PT2_RUN - 1) / PT2_RUN;
    const unsigned grid =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 2, (runs + PT_NT / 64 - 1) / (PT_NT / 64)));
    HQ_CHECK(hipMemsetAsync(next, 0, sizeof(unsigned long long), s));
    const int moves = c.na * (c.norb - c.na);
    auto launch = [&](auto lds_tag, auto slots_tag) {
        constexpr bool L = decltype(lds_tag)::value;
        constexpr int S = decltype(slots_tag)::value;
        if (L)
            HQ_CHECK(hipFuncSetAttribute((const void *)k_pt2<L, S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds));
        hipLaunchKernelGGL((k_pt2<L, S>), dim3(grid), dim3(PT_NT), L ? lds : 0, s, pa, order, ga_of, gb_of, next);
    };
    using T = std::true_type;
    using F = std::false_type;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    using S4 = std::integral_constant<int, 4>;
    if (use_lds) {
        if (moves <= 64) launch(T{}, S1{});
        else if (moves <= 128) launch(T{}, S2{});
        else launch(T{}, S4{});
    } else {
        if (moves <= 64) launch(F{}, S1{});
        else if (moves <= 128) launch(F{}, S2{});
        else launch(F{}, S4{});
    }
    HQ_LAUNCH_CHECK();
    unsigned hbad = 0;
    HQ_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (hbad)
        throw Error(HINQS_E_BAD_OCCUPATION,
                    "a candidate has bits at or above norb or the wrong electron count (its outputs are NaN)");
}

namespace {

// PT2 quantities of the members of B from (H_B c) in sorted order (diagonal
// included); outputs in caller order through perm (null: sorted order).
__global__ void k_pt2_members(int64_t n, const double *hc, const double *diag, double e0, const int32_t *perm,
                              double *numer, double *hxx, double *score) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm ? (int64_t)perm[i] : i;
    const double v = hc[i], d = diag[i];
    if (numer) numer[o] = v;
    if (hxx) hxx[o] = d;
    if (score) score[o] = v * v / fabs(e0 - d);
}

}  // namespace

void pt2_members(Ctx &c, const double *coeffs, bool sorted, double e0, double *numer, double *hxx,
                 double *score) {
    hipStream_t s = c.stream;
    const int64_t n = c.ndet;
    const double *cs = coeffs;
    if (!sorted) {
        double *g = c.cs.get<double>(0, n);
        gather_rows(s, coeffs, g, c.perm.p, n, 8);
        cs = g;
    }
    double *hc = c.cs.get<double>(1, n);
    sigma_sorted(c, 1, cs, 1, hc, 1, HINQS_FP64, s);
    hipLaunchKernelGGL(k_pt2_members, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const double *)hc,
                       (const double *)c.diag.p, e0, sorted ? (const int32_t *)nullptr : (const int32_t *)c.perm.p,
                       numer, hxx, score);
    HQ_LAUNCH_CHECK();
}

}  // namespace hinqs

// ------------------------------------------------------------ product space
namespace hinqs {
namespace {

// missing[g] = number of distinct beta strings absent from alpha group g.
__global__ void k_missing_counts(const int32_t *ga, int32_t nua, int32_t nub, int64_t *missing) {
    const int32_t g = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g < nua) missing[g] = (int64_t)nub - (ga[g + 1] - ga[g]);
}

// One wave per alpha group: the distinct beta strings absent from the group,
// ascending, written as (alpha, beta) pairs from off[g] (first `cap` only).
__global__ void k_missing_list(const uint32_t *ua, const uint32_t *ub, const uint32_t *sb, const int32_t *ga,
                               int32_t nua, int32_t nub, const int64_t *off, int64_t cap, uint64_t *oa,
                               uint64_t *ob) {
    const int lane = threadIdx.x & 63;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (g >= nua) return;
    const int32_t lo = ga[g], n = ga[g + 1] - lo;
    int64_t pos = off[g];
    for (int32_t t0 = 0; t0 < nub; t0 += 64) {
        const int32_t t = t0 + lane;
        bool miss = false;
        uint32_t b = 0;
        if (t < nub) {
            b = ub[t];
            int32_t l = 0, h = n;  // is b among the group's beta strings?
            while (l < h) {
                const int32_t m = (l + h) >> 1;
                if (sb[lo + m] < b)
                    l = m + 1;
                else
                    h = m;
            }
            miss = !(l < n && sb[lo + l] == b);
        }
        const uint64_t m = __ballot(miss);
        if (miss) {
            const int64_t k = pos + __popcll(m & ((1ull << lane) - 1ull));
            if (k < cap) {
                oa[k] = ua[g];
                ob[k] = b;
            }
        }
        pos += __popcll(m);
    }
}

}  // namespace

int64_t product_closure(Ctx &c, int64_t cap, uint64_t *out_a, uint64_t *out_b) {
    hipStream_t s = c.stream;
    const int64_t total = (int64_t)c.nua * c.nub - c.ndet;
    if (cap <= 0 || total <= 0) return total;
    int64_t *miss = c.cs.get<int64_t>(0, c.nua + 1);
    int64_t *off = c.cs.get<int64_t>(1, c.nua + 1);
    HQ_CHECK(hipMemsetAsync(miss + c.nua, 0, sizeof(int64_t), s));
    hipLaunchKernelGGL(k_missing_counts, dim3(grid_for(c.nua, 256)), dim3(256), 0, s, c.ga.p, c.nua, c.nub, miss);
    HQ_LAUNCH_CHECK();
    exclusive_scan_i64(s, miss, off, c.nua + 1, c.work);
    hipLaunchKernelGGL(k_missing_list, dim3(grid_for((int64_t)c.nua * 64, 256)), dim3(256), 0, s, c.ua.p, c.ub.p,
                       c.sb.p, c.ga.p, c.nua, c.nub, off, cap, out_a, out_b);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipStreamSynchronize(s));
    return total;
}

}  // namespace hinqs
