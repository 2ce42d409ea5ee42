// Coupling enumeration: for every determinant x_i of B, every x_j of B that
// differs from it by one or two electrons, i.e. every pair with a possibly
// nonzero <x_i|H|x_j> (Slater-Condon rules; paper Sec. 2.2, Step 3 builds
// [H_B]_ij over exactly these pairs).
//
// The three classes are found without an O(|B|^2) scan:
//   alpha-only moves   x_j shares beta_i: scan the beta group of beta_i;
//   beta-only moves    x_j shares alpha_i: scan the alpha group of alpha_i;
//   alpha+beta moves   alpha_j is a single move of alpha_i present in B (alpha
//                      link table): scan that alpha group for beta strings one
//                      move away or, in groups of at least lookup_min rows
//                      (dense sets, e.g. product spaces), look each beta
//                      string one move away up by binary search.
// Each candidate is tested with XOR + popcount; the sign comes from masked
// popcounts (common.hpp).  The alpha-only class runs one thread per entry of
// the beta-major listing and the other two one thread per sorted row, so in
// both kernels neighbouring threads share the string whose groups they walk,
// which turns the string loads into broadcasts.  A counting pass sizes each
// row; a fill pass writes (col, desc), alpha-only entries first.
#include <chrono>
#include <cstdlib>

#include "common.hpp"

namespace hinqs {

namespace {

// Group scans test SCAN_W candidates without branching, then emit the hits of
// that step from a bit mask: the emission code (descriptor and two stores)
// then runs about once per step instead of on every candidate where some lane
// of the wave happens to hit.  Entries keep their order.
struct ConnArgs {
    int64_t ndet;
    const uint32_t *sb;
    const int32_t *aidx, *bidx, *ga, *gb, *bperm;
    const uint32_t *bm_alpha;
    const int32_t *alink_cnt, *alink;
    const uint32_t *alink_info;
    int alink_max;
    int norb;
    int32_t lookup_min;  // alpha groups at least this long are searched, not scanned
};

// Alpha+beta couplings of a row with beta string bi into the alpha group
// [g0, g1) (rows sorted by beta string) by lookup: every beta string one move
// away from bi, generated in ascending order, is located by binary search in
// the part of the group not passed yet, so the hits come out with j ascending,
// as from the scan.  Ascending order: first the moves that lower the value
// (hole h from the highest occupied orbital down, then particle p < h
// upwards), then those that raise it (particle p from the lowest empty
// orbital up, then hole h < p downwards).
template <typename Emit>
__device__ inline void ab_lookup(const uint32_t *__restrict__ sb, int32_t g0, int32_t g1, uint32_t bi, int norb,
                                 Emit &&emit) {
    const uint32_t full = norb >= 32 ? 0xffffffffu : ((1u << norb) - 1u);
    const uint32_t emp = ~bi & full;
    int32_t lo = g0;
    auto find = [&](uint32_t v) {
        int32_t l = lo, h = g1;  // first position in [lo, g1) with sb >= v
        while (l < h) {
            const int32_t m = (l + h) >> 1;
            if (sb[m] < v) l = m + 1;
            else h = m;
        }
        lo = l;
        if (l < g1 && sb[l] == v) {
            emit(l);
            lo = l + 1;
        }
    };
    for (uint32_t hs = bi; hs;) {
        const int h = 31 - __builtin_clz(hs);
        hs &= ~(1u << h);
        for (uint32_t ps = emp & ((1u << h) - 1u); ps; ps &= ps - 1) find(bi ^ (1u << h) ^ (1u << lowbit(ps)));
    }
    for (uint32_t ps = emp; ps; ps &= ps - 1) {
        const int p = lowbit(ps);
        for (uint32_t hs = bi & ((1u << p) - 1u); hs;) {
            const int h = 31 - __builtin_clz(hs);
            hs &= ~(1u << h);
            find(bi ^ (1u << h) ^ (1u << p));
        }
    }
}

// Alpha-only moves (x_j shares beta_i), one thread per entry of the
// beta-major listing: neighbouring threads share beta_i and scan the same
// beta group in lock step (broadcast loads), where one thread per sorted row
// would scan a different beta group on every lane.  Counting pass: n1[i];
// filling pass: the row's first n1[i] entries.
template <bool FILL>
__global__ __launch_bounds__(256) void k_connect_beta(ConnArgs a, int32_t *n1, const int64_t *rowptr,
                                                      int32_t *col, uint32_t *desc) {
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 >= a.ndet) return;
    const int32_t i = a.bperm[t0];
    const uint32_t ai = a.bm_alpha[t0];
    const int32_t bg = a.bidx[i];
    int64_t out = FILL ? rowptr[i] : 0;
    int32_t n = 0;
    for (int32_t t0 = a.gb[bg], e = a.gb[bg + 1]; t0 < e; t0 += SCAN_W) {
        uint32_t m = 0;
#pragma unroll
        for (int u = 0; u < SCAN_W; ++u) {
            const uint32_t aj = t0 + u < e ? a.bm_alpha[t0 + u] : ai;
            const int d = popc32(ai ^ aj);
            m |= (d == 2 || d == 4) ? 1u << u : 0u;
        }
        if (FILL) {
            for (; m; m &= m - 1) {
                const int32_t t = t0 + lowbit(m);
                col[out] = a.bperm[t];
                desc[out] = same_spin_desc(ai, a.bm_alpha[t], HINQS_EXC_1A, HINQS_EXC_2AA);
                ++out;
            }
        } else {
            n += popc32(m);
        }
    }
    if (!FILL) n1[i] = n;
}

// Beta-only and alpha+beta moves, one thread per sorted row (neighbouring
// rows share alpha_i, so their group scans are broadcast loads).  Counting
// pass: counts[i] = n1[i] + these; filling pass: after the row's n1[i]
// alpha-only entries.
template <bool FILL>
__global__ __launch_bounds__(256) void k_connect(ConnArgs a, const int32_t *n1, int64_t *counts,
                                                 const int64_t *rowptr, int32_t *col, uint32_t *desc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ndet) return;
    const uint32_t bi = a.sb[i];
    const int32_t ag = a.aidx[i];
    int64_t out = FILL ? rowptr[i] + n1[i] : 0;
    int64_t n = 0;
    // beta-only: determinants with the same alpha string
    for (int32_t j0 = a.ga[ag], e = a.ga[ag + 1]; j0 < e; j0 += SCAN_W) {
        uint32_t m = 0;
#pragma unroll
        for (int u = 0; u < SCAN_W; ++u) {
            const uint32_t bj = j0 + u < e ? a.sb[j0 + u] : bi;
            const int d = popc32(bi ^ bj);
            m |= (d == 2 || d == 4) ? 1u << u : 0u;
        }
        if (FILL) {
            for (; m; m &= m - 1) {
                const int32_t j = j0 + lowbit(m);
                col[out] = j;
                desc[out] = same_spin_desc(bi, a.sb[j], HINQS_EXC_1B, HINQS_EXC_2BB);
                ++out;
            }
        } else {
            n += popc32(m);
        }
    }
    // alpha + beta: alpha string one move away, beta string one move away
    const int64_t lbase = (int64_t)ag * a.alink_max;
    for (int32_t l = 0, le = a.alink_cnt[ag]; l < le; ++l) {
        const int32_t tgt = a.alink[lbase + l];
        const uint32_t info = a.alink_info[lbase + l];
        const int ha = info & 31, pa = (info >> 5) & 31;
        const uint32_t npar = (info >> 10) & 1u;
        if (a.ga[tgt + 1] - a.ga[tgt] >= a.lookup_min) {
            ab_lookup(a.sb, a.ga[tgt], a.ga[tgt + 1], bi, a.norb, [&](int32_t j) {
                if (FILL) {
                    col[out] = j;
                    desc[out] = ab_desc(ha, pa, npar, bi, a.sb[j]);
                    ++out;
                } else {
                    ++n;
                }
            });
            continue;
        }
        for (int32_t j0 = a.ga[tgt], e = a.ga[tgt + 1]; j0 < e; j0 += SCAN_W) {
            uint32_t m = 0;
#pragma unroll
            for (int u = 0; u < SCAN_W; ++u) {
                const uint32_t bj = j0 + u < e ? a.sb[j0 + u] : bi;
                m |= popc32(bi ^ bj) == 2 ? 1u << u : 0u;
            }
            if (FILL) {
                for (; m; m &= m - 1) {
                    const int32_t j = j0 + lowbit(m);
                    col[out] = j;
                    desc[out] = ab_desc(ha, pa, npar, bi, a.sb[j]);
                    ++out;
                }
            } else {
                n += popc32(m);
            }
        }
    }
    if (!FILL) counts[i] = n1[i] + n;
}

// bounds[x] = first row whose couplings start at or after x * total / 8 (x = 0..8).
__global__ void k_balance_bounds(int64_t n, const int64_t *rowptr, int64_t *bounds) {
    const int x = threadIdx.x;
    if (x > 8) return;
    const int64_t total = rowptr[n];
    if (x == 8) { bounds[8] = n; return; }
    const int64_t target = (total / 8) * x + (total % 8) * x / 8;
    int64_t lo = 0, hi = n;  // smallest r in [0, n] with rowptr[r] >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (rowptr[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bounds[x] = lo;
}

__global__ void k_caller_counts(int64_t n, const int64_t *rowptr, const int32_t *perm, int64_t *counts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    counts[perm[i]] = rowptr[i + 1] - rowptr[i];
}

// One wave per sorted row: copy its couplings to the caller-order position,
// translating column indices to caller indices.
__global__ void k_caller_copy(int64_t n, const int64_t *rowptr, const int32_t *col, const uint32_t *desc,
                              const int32_t *perm, const int64_t *rowptr_c, int32_t *col_c,
                              uint32_t *desc_c) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n) return;
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    const int64_t dst = rowptr_c[perm[row]];
    for (int64_t e = beg + lane; e < end; e += 64) {
        if (col_c) col_c[dst + (e - beg)] = perm[col[e]];
        if (desc_c) desc_c[dst + (e - beg)] = desc[e];
    }
}

int32_t env_i32(const char *name, int32_t dflt) {
    const char *v = std::getenv(name);
    return (v && *v) ? (int32_t)std::atoi(v) : dflt;
}

}  // namespace

void export_connectivity(Ctx &c, int64_t *rowptr_c, int32_t *col_c, uint32_t *desc_c) {
    hipStream_t s = c.stream;
    const int64_t n = c.ndet;
    DBuf<int64_t> counts;
    counts.ensure(n + 1);
    HQ_CHECK(hipMemsetAsync(counts.p + n, 0, sizeof(int64_t), s));
    hipLaunchKernelGGL(k_caller_counts, dim3(grid_for(n, 256)), dim3(256), 0, s, n, c.rowptr.p, c.perm.p,
                       counts.p);
    HQ_LAUNCH_CHECK();
    exclusive_scan_i64(s, counts.p, rowptr_c, n + 1, c.work);
    if (col_c || desc_c) {
        hipLaunchKernelGGL(k_caller_copy, dim3(grid_for(n * 64, 256)), dim3(256), 0, s, n, c.rowptr.p,
                           c.col.p, c.desc.p, c.perm.p, rowptr_c, col_c, desc_c);
        HQ_LAUNCH_CHECK();
    }
    wait_stream(s);
}

void compute_xcd_rows(Ctx &c) {
    hipStream_t s = c.stream;
    DBuf<int64_t> bnd;
    bnd.ensure(9);
    hipLaunchKernelGGL(k_balance_bounds, dim3(1), dim3(64), 0, s, c.ndet, c.rowptr.p, bnd.p);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipMemcpyAsync(c.xcd_rows, bnd.p, sizeof(c.xcd_rows), hipMemcpyDeviceToHost, s));
    wait_stream(s);
}

void build_connectivity(Ctx &c, bool xcd_rows) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c.stream;
    const int64_t n = c.ndet;
    // lookups replace the scan only where a group is very long next to the
    // number of beta moves: a lookup is a binary search whose loads differ
    // from lane to lane, while a scan step tests 16 candidates with loads that
    // neighbouring threads share (measured: lookups in every group 4x slower
    // on the sampled 1e6 set, and no faster on product spaces with groups of
    // 1,716 and 3,432 rows)
    const int32_t nmoves = c.nb * (c.norb - c.nb);
    const int32_t lookup_min = env_i32("HINQS_CONNECT_LOOKUP_MIN", std::max<int32_t>(4096, 64 * nmoves));
    ConnArgs a{n,          c.sb.p,        c.aidx.p,  c.bidx.p,
               c.ga.p,     c.gb.p,        c.bperm.p, c.bm_alpha.p,  c.alink_ptr.p,
               c.alink.p,  c.alink_info.p, c.alink_max, c.norb, lookup_min};
    auto &counts = c.bs.counts;
    auto &n1 = c.bs.gidx;  // alpha-only couplings per row (free once the tables are built)
    counts.ensure(n + 1);
    n1.ensure(n);
    dim3 g(grid_for(n, 256)), b(256);
    hipLaunchKernelGGL(k_connect_beta<false>, g, b, 0, s, a, n1.p, (const int64_t *)nullptr, (int32_t *)nullptr,
                       (uint32_t *)nullptr);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_connect<false>, g, b, 0, s, a, (const int32_t *)n1.p, counts.p, (const int64_t *)nullptr,
                       (int32_t *)nullptr, (uint32_t *)nullptr);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipMemsetAsync(counts.p + n, 0, sizeof(int64_t), s));
    c.rowptr.ensure(n + 1);
    exclusive_scan_i64(s, counts.p, c.rowptr.p, n + 1, c.work);
    int64_t nnz = 0;
    HQ_CHECK(hipMemcpyAsync(&nnz, c.rowptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    wait_stream(s);
    if (nnz >= ((int64_t)1 << 40)) throw Error(HINQS_E_UNSUPPORTED, "too many couplings");
    c.nnz = nnz;
    c.col.ensure(nnz);
    c.desc.ensure(nnz);
    hipLaunchKernelGGL(k_connect_beta<true>, g, b, 0, s, a, (int32_t *)nullptr, c.rowptr.p, c.col.p, c.desc.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_connect<true>, g, b, 0, s, a, (const int32_t *)n1.p, (int64_t *)nullptr, c.rowptr.p,
                       c.col.p, c.desc.p);
    HQ_LAUNCH_CHECK();
    if (xcd_rows) compute_xcd_rows(c);
    for (auto &row : c.sigma_cfg)
        for (auto &g : row) g = SigmaCfg{};
    c.ms_connect =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hinqs
