// Incremental basis update (Sec. 2.2: Step 2 appends the best-scored new
// candidates to B and evicts the lowest-scored entries beyond a cap; Step 3
// keeps its diagonalization state across iterations and warm-starts from the
// previous eigenvector).
//
// B' = (B without the evicted determinants, in their caller order) followed
// by the appended determinants A.  The string tables of B' are rebuilt (a
// sort of |B'| keys), but the couplings are patched, not re-enumerated:
//   row of a kept determinant  its old couplings to kept determinants, copied
//                              with remapped columns and their stored values,
//                              then its couplings to A, found through A's own
//                              string tables;
//   row of an appended one     a full enumeration against B'.
// Only the new entries get Slater-Condon values.  Within a row the entries
// are in a fixed order (kept ones first), so products stay deterministic;
// the row sets equal those of a fresh build.
#include <chrono>

#include "common.hpp"

namespace hinqs {

namespace {

__global__ void k_fill_i32v(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// keep[i] = 0 for every listed caller index; bad: 1 out of range, 2 repeated.
// (Listed sorted positions are first turned into caller indices by perm.)
__global__ void k_mark_evict(const int32_t *evict, int64_t ne, int64_t n, const int32_t *perm, int32_t *keep,
                             unsigned *bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    int32_t i = evict[t];
    if (i < 0 || i >= n) {
        atomicOr(bad, 1u);
        return;
    }
    if (perm) i = perm[i];
    if (atomicSub(&keep[i], 1) != 1) atomicOr(bad, 2u);
}

// The new caller list: kept determinants (caller order) then the appended ones.
__global__ void k_new_list(const int32_t *keep, const int32_t *newidx, const int32_t *inv_old, const uint32_t *sa,
                           const uint32_t *sb, int64_t n_old, const uint64_t *add_a, const uint64_t *add_b,
                           int64_t n_add, int64_t n_keep, uint64_t *out_a, uint64_t *out_b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_old) {
        if (keep[i]) {
            const int32_t p = inv_old[i];
            out_a[newidx[i]] = sa[p];
            out_b[newidx[i]] = sb[p];
        }
    } else if (i < n_old + n_add) {
        out_a[n_keep + (i - n_old)] = add_a[i - n_old];
        out_b[n_keep + (i - n_old)] = add_b[i - n_old];
    }
}

// o2n[old sorted position] = new sorted position or -1; n2o the inverse (-1
// for appended rows, filled beforehand).
__global__ void k_maps(const int32_t *perm_old, const int32_t *keep, const int32_t *newidx, const int32_t *inv_new,
                       int64_t n_old, int32_t *o2n, int32_t *n2o) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_old) return;
    const int32_t ci = perm_old[p];
    const int32_t r = keep[ci] ? inv_new[newidx[ci]] : -1;
    o2n[p] = r;
    if (r >= 0) n2o[r] = (int32_t)p;
}

// Sorted positions in B' of A's sorted entries (ascending).
__global__ void k_amap(const int32_t *perm_a, const int32_t *inv_new, int64_t n_add, int64_t n_keep, int32_t *amap) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_add) amap[p] = inv_new[n_keep + perm_a[p]];
}

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

// For each distinct string of B': its group in A (same string) and, for
// alpha, the A groups one single move away.
__global__ void k_cross_alpha(const uint32_t *ua, int32_t nua, const uint32_t *ua_a, int32_t nua_a, int norb,
                              int maxl, int32_t *same, int32_t *xcnt, int32_t *xlink) {
    const int32_t g = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= nua) return;
    const uint32_t s = ua[g];
    same[g] = find_u32(ua_a, nua_a, s);
    const uint32_t full = norb >= 32 ? 0xffffffffu : ((1u << norb) - 1u);
    int n = 0;
    for (uint32_t ho = s; ho; ho &= ho - 1) {
        const int h = lowbit(ho);
        for (uint32_t pe = ~s & full; pe; pe &= pe - 1) {
            const int32_t t = find_u32(ua_a, nua_a, s ^ (1u << h) ^ (1u << lowbit(pe)));
            if (t >= 0) xlink[(int64_t)g * maxl + n++] = t;
        }
    }
    xcnt[g] = n;
}

__global__ void k_cross_beta(const uint32_t *ub, int32_t nub, const uint32_t *ub_a, int32_t nub_a, int32_t *same) {
    const int32_t g = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g < nub) same[g] = find_u32(ub_a, nub_a, ub[g]);
}

struct CrossArgs {
    int64_t n;                    // rows of B'
    const int32_t *n2o;           // B' row -> old sorted position, -1 for appended rows
    const uint32_t *sa, *sb;      // B' strings (sorted)
    const int32_t *aidx, *bidx;   // B' row -> distinct alpha / beta string
    const int32_t *asame, *bsame, *xcnt, *xlink;
    int maxl;
    // A's tables (has_a false: nothing is appended)
    bool has_a;
    const uint32_t *ua_a, *sb_a, *bm_alpha_a;
    const int32_t *ga_a, *gb_a, *bperm_a;
    const int32_t *amap;          // A sorted position -> B' sorted position
};

// Counting pass (FILL = false): for each kept row, cnt[r] = kept[r] (its old
// entries whose column survives) + its couplings to A.  Filling pass: the
// couplings to A, written after the kept entries.
template <bool FILL>
__global__ __launch_bounds__(256) void k_cross(CrossArgs a, int64_t *cnt, int64_t *kept, const int64_t *rowptr,
                                               int32_t *col, uint32_t *desc) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const int32_t p = a.n2o[r];
    if (p < 0) return;
    const int64_t nk = kept[r];
    int64_t out = FILL ? rowptr[r] + nk : 0;
    int64_t n = 0;
    if (!a.has_a) {
        if (!FILL) cnt[r] = nk;
        return;
    }
    const uint32_t ai = a.sa[r], bi = a.sb[r];
    const int32_t gbA = a.bsame[a.bidx[r]];
    // group scans: SCAN_W candidates tested branch-free, hits emitted from the mask
    if (gbA >= 0) {  // same beta string, alpha one or two moves away
        for (int32_t u0 = a.gb_a[gbA], e = a.gb_a[gbA + 1]; u0 < e; u0 += SCAN_W) {
            uint32_t m = 0;
#pragma unroll
            for (int v = 0; v < SCAN_W; ++v) {
                const uint32_t aj = u0 + v < e ? a.bm_alpha_a[u0 + v] : ai;
                const int d = popc32(ai ^ aj);
                m |= (d == 2 || d == 4) ? 1u << v : 0u;
            }
            if (FILL) {
                for (; m; m &= m - 1) {
                    const int32_t u = u0 + lowbit(m);
                    col[out] = a.amap[a.bperm_a[u]];
                    desc[out] = same_spin_desc(ai, a.bm_alpha_a[u], HINQS_EXC_1A, HINQS_EXC_2AA);
                    ++out;
                }
            } else {
                n += popc32(m);
            }
        }
    }
    const int32_t ag = a.aidx[r];
    const int32_t gaA = a.asame[ag];
    if (gaA >= 0) {  // same alpha string, beta one or two moves away
        for (int32_t j0 = a.ga_a[gaA], e = a.ga_a[gaA + 1]; j0 < e; j0 += SCAN_W) {
            uint32_t m = 0;
#pragma unroll
            for (int v = 0; v < SCAN_W; ++v) {
                const uint32_t bj = j0 + v < e ? a.sb_a[j0 + v] : bi;
                const int d = popc32(bi ^ bj);
                m |= (d == 2 || d == 4) ? 1u << v : 0u;
            }
            if (FILL) {
                for (; m; m &= m - 1) {
                    const int32_t j = j0 + lowbit(m);
                    col[out] = a.amap[j];
                    desc[out] = same_spin_desc(bi, a.sb_a[j], HINQS_EXC_1B, HINQS_EXC_2BB);
                    ++out;
                }
            } else {
                n += popc32(m);
            }
        }
    }
    for (int32_t l = 0, le = a.xcnt[ag]; l < le; ++l) {  // one move in each spin
        const int32_t tg = a.xlink[(int64_t)ag * a.maxl + l];
        const uint32_t aj = a.ua_a[tg];
        const int ha = lowbit(aj & ~ai), pa = lowbit(ai & ~aj);  // the alpha move of this group
        const uint32_t npar = single_parity(aj, ha, pa);
        for (int32_t j0 = a.ga_a[tg], e = a.ga_a[tg + 1]; j0 < e; j0 += SCAN_W) {
            uint32_t m = 0;
#pragma unroll
            for (int v = 0; v < SCAN_W; ++v) {
                const uint32_t bj = j0 + v < e ? a.sb_a[j0 + v] : bi;
                m |= popc32(bi ^ bj) == 2 ? 1u << v : 0u;
            }
            if (FILL) {
                for (; m; m &= m - 1) {
                    const int32_t j = j0 + lowbit(m);
                    col[out] = a.amap[j];
                    desc[out] = ab_desc(ha, pa, npar, bi, a.sb_a[j]);
                    ++out;
                }
            } else {
                n += popc32(m);
            }
        }
    }
    if (!FILL) cnt[r] = nk + n;
}

// One wave per old row: kept[o2n[p]] = number of its entries whose column survives.
__global__ void k_kept_count(int64_t n_old, const int32_t *o2n, const int64_t *rowptr_old, const int32_t *col_old,
                             int64_t *kept) {
    const int lane = threadIdx.x & 63;
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= n_old) return;
    const int32_t r = o2n[p];
    if (r < 0) return;
    int64_t n = 0;
    for (int64_t q = rowptr_old[p] + lane, e = rowptr_old[p + 1]; q < e; q += 64) n += o2n[col_old[q]] >= 0;
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if (lane == 0) kept[r] = n;
}

struct RowArgs {
    const int32_t *rows;  // rows to enumerate (sorted positions, ascending)
    int64_t nrows;
    const uint32_t *sa, *sb, *bm_alpha, *alink_info;
    const int32_t *aidx, *bidx, *ga, *gb, *bperm, *alink_cnt, *alink;
    int alink_max;
};

// Ballot-compacted append of the lanes with `keep` set, in lane order.
struct WaveOut {
    int64_t pos;  // next output slot (uniform)
    int64_t n;    // entries so far (uniform)
};

template <bool FILL>
__device__ inline void wave_emit(bool keep, int32_t colv, uint32_t descv, int lane, WaveOut &o, int32_t *col,
                                 uint32_t *desc) {
    const uint64_t m = __ballot(keep);
    if (FILL && keep) {
        const int64_t k = o.pos + __popcll(m & ((1ull << lane) - 1ull));
        col[k] = colv;
        desc[k] = descv;
    }
    o.pos += __popcll(m);
    o.n += __popcll(m);
}

// Couplings of the listed rows against the whole set, one wave per row
// (lanes stride each group), in the same order as the one-thread-per-row
// enumerator: beta group, alpha group, then the linked alpha groups.  Used
// for appended rows, which are too scattered for rows sharing alpha strings
// in one wave.
template <bool FILL>
__global__ __launch_bounds__(256) void k_rows_wave(RowArgs a, int64_t *counts, const int64_t *rowptr, int32_t *col,
                                                   uint32_t *desc) {
    const int lane = threadIdx.x & 63;
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (t >= a.nrows) return;
    const int64_t i = a.rows[t];
    const uint32_t ai = a.sa[i], bi = a.sb[i];
    const int32_t ag = a.aidx[i], bg = a.bidx[i];
    WaveOut o{FILL ? rowptr[i] : 0, 0};
    for (int32_t u0 = a.gb[bg], e = a.gb[bg + 1]; u0 < e; u0 += 64) {
        const int32_t u = u0 + lane;
        const uint32_t aj = u < e ? a.bm_alpha[u] : ai;
        const int d = popc32(ai ^ aj);
        const bool k = d == 2 || d == 4;
        wave_emit<FILL>(k, k ? a.bperm[u] : 0, k ? same_spin_desc(ai, aj, HINQS_EXC_1A, HINQS_EXC_2AA) : 0u, lane, o,
                        col, desc);
    }
    for (int32_t j0 = a.ga[ag], e = a.ga[ag + 1]; j0 < e; j0 += 64) {
        const int32_t j = j0 + lane;
        const uint32_t bj = j < e ? a.sb[j] : bi;
        const int d = popc32(bi ^ bj);
        const bool k = d == 2 || d == 4;
        wave_emit<FILL>(k, j, k ? same_spin_desc(bi, bj, HINQS_EXC_1B, HINQS_EXC_2BB) : 0u, lane, o, col, desc);
    }
    const int64_t lbase = (int64_t)ag * a.alink_max;
    for (int32_t l = 0, le = a.alink_cnt[ag]; l < le; ++l) {
        const int32_t tgt = a.alink[lbase + l];
        const uint32_t info = a.alink_info[lbase + l];
        const int ha = info & 31, pa = (info >> 5) & 31;
        const uint32_t npar = (info >> 10) & 1u;
        for (int32_t j0 = a.ga[tgt], e = a.ga[tgt + 1]; j0 < e; j0 += 64) {
            const int32_t j = j0 + lane;
            const uint32_t bj = j < e ? a.sb[j] : bi;
            const bool k = popc32(bi ^ bj) == 2;
            wave_emit<FILL>(k, j, k ? ab_desc(ha, pa, npar, bi, bj) : 0u, lane, o, col, desc);
        }
    }
    if (!FILL && lane == 0) counts[i] = o.n;
}

// One wave per old row: copy its entries whose column survives (order kept)
// into the B' row, with remapped columns and their values.
__global__ void k_copy_kept(int64_t n_old, const int32_t *o2n, const int64_t *rowptr_old, const int32_t *col_old,
                            const uint32_t *desc_old, const double *val_old, const float *val32_old,
                            const int64_t *rowptr, int32_t *col, uint32_t *desc, double *val, float *val32) {
    const int lane = threadIdx.x & 63;
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= n_old) return;
    const int32_t r = o2n[p];
    if (r < 0) return;
    int64_t dst = rowptr[r];
    const int64_t b = rowptr_old[p], e = rowptr_old[p + 1];
    for (int64_t q0 = b; q0 < e; q0 += 64) {
        const int64_t q = q0 + lane;
        const int32_t nc = q < e ? o2n[col_old[q]] : -1;
        const uint64_t m = __ballot(nc >= 0);
        if (nc >= 0) {
            const int64_t k = dst + __popcll(m & ((1ull << lane) - 1ull));
            col[k] = nc;
            desc[k] = desc_old[q];
            val[k] = val_old[q];
            val32[k] = val32_old[q];
        }
        dst += __popcll(m);
    }
}

__global__ void k_zero(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_carry_scatter(const double *c_old, int64_t n_old, const int32_t *map, const int32_t *keep,
                                double *c_new) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_old) return;
    if (keep && !keep[i]) return;
    const int32_t d = map[i];
    if (d >= 0) c_new[d] = c_old[i];
}

// ---------------------------------------------------------- selection policy
// flag[v] = 1 for every chosen index v (a position in a combined list).
__global__ void k_flag_chosen(const int32_t *idx, int64_t k, int32_t *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < k) flag[idx[t]] = 1;
}

// comb[0..nb) = bscore, comb[nb + t] = cscore[list[t]] (list may be null: identity).
__global__ void k_combine(const double *bscore, int64_t nb, const double *cscore, const int32_t *list, int64_t nl,
                          double *comb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb)
        comb[i] = bscore[i];
    else if (i < nb + nl)
        comb[i] = cscore[list ? list[i - nb] : i - nb];
}

// Ordered compaction: out[pos[i]] = val(i) for the i < n with flag[i] == want.
__global__ void k_compact_i32(const int32_t *flag, const int32_t *pos, int64_t n, int32_t want, const int32_t *src,
                              int64_t shift, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || flag[i] != want) return;
    out[pos[i]] = src ? src[i] - (int32_t)shift : (int32_t)i;
}

// Appended strings and scores from the ordered candidate list.
__global__ void k_gather_cand(const int32_t *list, int64_t n, const uint64_t *ca, const uint64_t *cb,
                              const double *cscore, uint64_t *oa, uint64_t *ob, double *os) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t v = list[t];
    oa[t] = ca[v];
    ob[t] = cb[v];
    if (os) os[t] = cscore[v];
}

// out[i] = 1 - f[i]
__global__ void k_invert_flags(const int32_t *f, int64_t n, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = 1 - f[i];
}

// flag[t] = 1 when the chosen combined index list[t] is a candidate (>= nb).
__global__ void k_is_candidate(const int32_t *list, int64_t n, int64_t nb, int32_t *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) flag[t] = list[t] >= nb ? 1 : 0;
}

// Scores of B': kept basis scores (caller order), then the appended ones.
__global__ void k_new_scores(const double *bscore, const int32_t *keepb, const int32_t *posb, int64_t nb,
                             const double *app, int64_t na, int64_t nkeep, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        if (keepb[i]) out[posb[i]] = bscore[i];
    } else if (i < nb + na) {
        out[nkeep + (i - nb)] = app[i - nb];
    }
}

// Swap the determinant store (strings, permutations, tables) of two contexts.
void swap_tables(Ctx &x, Ctx &y) {
    std::swap(x.ndet, y.ndet);
    std::swap(x.na, y.na);
    std::swap(x.nb, y.nb);
    x.sa.swap(y.sa);
    x.sb.swap(y.sb);
    x.perm.swap(y.perm);
    x.inv.swap(y.inv);
    std::swap(x.nua, y.nua);
    std::swap(x.nub, y.nub);
    x.ua.swap(y.ua);
    x.ub.swap(y.ub);
    x.ga.swap(y.ga);
    x.aidx.swap(y.aidx);
    x.bidx.swap(y.bidx);
    x.gb.swap(y.gb);
    x.bperm.swap(y.bperm);
    x.bm_alpha.swap(y.bm_alpha);
    std::swap(x.alink_max, y.alink_max);
    x.alink_ptr.swap(y.alink_ptr);
    x.alink.swap(y.alink);
    x.alink_info.swap(y.alink_info);
    std::swap(x.have_dets, y.have_dets);
}

void scratch_ctx(const Ctx &c, Ctx &t) {
    t.device = c.device;
    t.stream = c.stream;
    t.norb = c.norb;
}

}  // namespace

void update_determinants(Ctx &c, int64_t n_evict, const int32_t *evict, int64_t n_add, const uint64_t *add_a,
                         const uint64_t *add_b, const double *c_old, double *c_new, bool sorted,
                         double *ms_out) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c.stream;
    const int64_t n_old = c.ndet;
    const int norb = c.norb;

    // ---- the new caller list (no state changes until every check passed)
    DBuf<int32_t> keep, newidx;
    DBuf<unsigned> bad;
    keep.ensure(n_old);
    newidx.ensure(n_old);
    bad.ensure(1);
    HQ_CHECK(hipMemsetAsync(bad.p, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(n_old, 256)), dim3(256), 0, s, keep.p, n_old, 1);
    HQ_LAUNCH_CHECK();
    if (n_evict > 0) {
        hipLaunchKernelGGL(k_mark_evict, dim3(grid_for(n_evict, 256)), dim3(256), 0, s, evict, n_evict, n_old,
                           sorted ? (const int32_t *)c.perm.p : (const int32_t *)nullptr, keep.p, bad.p);
        HQ_LAUNCH_CHECK();
    }
    exclusive_scan_i32(s, keep.p, newidx.p, n_old, c.work);
    unsigned hbad = 0;
    int32_t last[2] = {0, 0};
    HQ_CHECK(hipMemcpyAsync(&hbad, bad.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&last[0], newidx.p + n_old - 1, 4, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&last[1], keep.p + n_old - 1, 4, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (hbad & 1u) throw Error(HINQS_E_INVALID_ARG, "an evicted index is outside [0, ndet)");
    if (hbad & 2u) throw Error(HINQS_E_INVALID_ARG, "an evicted index is listed twice");
    const int64_t n_keep = (int64_t)last[0] + last[1];
    const int64_t n_new = n_keep + n_add;
    if (n_new < 1) throw Error(HINQS_E_INVALID_ARG, "the update would leave no determinant");
    if (n_new >= ((int64_t)1 << 31)) throw Error(HINQS_E_UNSUPPORTED, "more than 2^31 - 1 determinants");

    DBuf<uint64_t> la, lb;
    la.ensure(n_new);
    lb.ensure(n_new);
    hipLaunchKernelGGL(k_new_list, dim3(grid_for(n_old + n_add, 256)), dim3(256), 0, s, keep.p, newidx.p, c.inv.p,
                       c.sa.p, c.sb.p, n_old, add_a, add_b, n_add, n_keep, la.p, lb.p);
    HQ_LAUNCH_CHECK();
    Ctx t;  // tables of B' (validates the appended strings and rejects repeats)
    scratch_ctx(c, t);
    build_determinants(t, n_new, la.p, lb.p, c.na, c.nb, true);
    la.release();
    lb.release();
    Ctx ta;  // tables of A alone
    if (n_add > 0) {
        scratch_ctx(c, ta);
        build_determinants(ta, n_add, add_a, add_b, c.na, c.nb, true);
    }

    // ---- commit: B' tables into c; old tables and couplings kept aside
    c.have_elements = false;
    swap_tables(c, t);  // t now holds the old tables
    DBuf<int64_t> rowptr_old;
    DBuf<int32_t> col_old;
    DBuf<uint32_t> desc_old;
    DBuf<double> val_old;
    DBuf<float> val32_old;
    rowptr_old.swap(c.rowptr);
    col_old.swap(c.col);
    desc_old.swap(c.desc);
    val_old.swap(c.val);
    val32_old.swap(c.val32);

    DBuf<int32_t> o2n, n2o;
    o2n.ensure(n_old);
    n2o.ensure(n_new);
    hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(n_new, 256)), dim3(256), 0, s, n2o.p, n_new, -1);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_maps, dim3(grid_for(n_old, 256)), dim3(256), 0, s, t.perm.p, keep.p, newidx.p, c.inv.p,
                       n_old, o2n.p, n2o.p);
    HQ_LAUNCH_CHECK();

    // ---- counts: kept rows (old entries + couplings to A), appended rows (full)
    DBuf<int64_t> cnt, kept, rowptr;
    cnt.ensure(n_new + 1);
    kept.ensure(n_new);
    HQ_CHECK(hipMemsetAsync(kept.p, 0, sizeof(int64_t) * n_new, s));
    HQ_CHECK(hipMemsetAsync(cnt.p + n_new, 0, sizeof(int64_t), s));
    DBuf<int32_t> asame, bsame, xcnt, xlink, amap;
    const int maxl = std::max(1, c.na * (norb - c.na));
    CrossArgs ca{};
    ca.n = n_new;
    ca.n2o = n2o.p;
    ca.sa = c.sa.p;
    ca.sb = c.sb.p;
    ca.aidx = c.aidx.p;
    ca.bidx = c.bidx.p;
    ca.maxl = maxl;
    ca.has_a = n_add > 0;
    if (n_add > 0) {
        asame.ensure(c.nua);
        xcnt.ensure(c.nua);
        xlink.ensure((size_t)c.nua * maxl);
        bsame.ensure(c.nub);
        amap.ensure(n_add);
        hipLaunchKernelGGL(k_cross_alpha, dim3(grid_for(c.nua, 128)), dim3(128), 0, s, c.ua.p, c.nua, ta.ua.p,
                           ta.nua, norb, maxl, asame.p, xcnt.p, xlink.p);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cross_beta, dim3(grid_for(c.nub, 256)), dim3(256), 0, s, c.ub.p, c.nub, ta.ub.p,
                           ta.nub, bsame.p);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_amap, dim3(grid_for(n_add, 256)), dim3(256), 0, s, ta.perm.p, c.inv.p, n_add, n_keep,
                           amap.p);
        HQ_LAUNCH_CHECK();
        ca.asame = asame.p;
        ca.bsame = bsame.p;
        ca.xcnt = xcnt.p;
        ca.xlink = xlink.p;
        ca.ua_a = ta.ua.p;
        ca.sb_a = ta.sb.p;
        ca.bm_alpha_a = ta.bm_alpha.p;
        ca.ga_a = ta.ga.p;
        ca.gb_a = ta.gb.p;
        ca.bperm_a = ta.bperm.p;
        ca.amap = amap.p;
    }
    hipLaunchKernelGGL(k_kept_count, dim3(grid_for(n_old * 64, 256)), dim3(256), 0, s, n_old, o2n.p, rowptr_old.p,
                       col_old.p, kept.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cross<false>, dim3(grid_for(n_new, 256)), dim3(256), 0, s, ca, cnt.p, kept.p,
                       (const int64_t *)nullptr, (int32_t *)nullptr, (uint32_t *)nullptr);
    HQ_LAUNCH_CHECK();
    // appended rows in ascending sorted position (amap is ascending: A and B' share the key order)
    const RowArgs ra{amap.p,    n_add,     c.sa.p,    c.sb.p,   c.bm_alpha.p, c.alink_info.p, c.aidx.p,
                     c.bidx.p,  c.ga.p,    c.gb.p,    c.bperm.p, c.alink_ptr.p, c.alink.p,    c.alink_max};
    if (n_add > 0) {
        hipLaunchKernelGGL(k_rows_wave<false>, dim3(grid_for(n_add * 64, 256)), dim3(256), 0, s, ra, cnt.p,
                           (const int64_t *)nullptr, (int32_t *)nullptr, (uint32_t *)nullptr);
        HQ_LAUNCH_CHECK();
    }
    rowptr.ensure(n_new + 1);
    exclusive_scan_i64(s, cnt.p, rowptr.p, n_new + 1, c.work);
    int64_t nnz = 0;
    HQ_CHECK(hipMemcpyAsync(&nnz, rowptr.p + n_new, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipStreamSynchronize(s));
    if (nnz >= ((int64_t)1 << 40)) throw Error(HINQS_E_UNSUPPORTED, "too many couplings");

    // ---- fill: kept entries with their values, couplings to A, appended rows
    c.rowptr.swap(rowptr);
    c.nnz = nnz;
    c.col.ensure(nnz);
    c.desc.ensure(nnz);
    c.val.ensure(nnz);
    c.val32.ensure(nnz);
    hipLaunchKernelGGL(k_copy_kept, dim3(grid_for(n_old * 64, 256)), dim3(256), 0, s, n_old, o2n.p, rowptr_old.p,
                       col_old.p, desc_old.p, val_old.p, val32_old.p, c.rowptr.p, c.col.p, c.desc.p, c.val.p,
                       c.val32.p);
    HQ_LAUNCH_CHECK();
    if (n_add > 0) {
        hipLaunchKernelGGL(k_cross<true>, dim3(grid_for(n_new, 256)), dim3(256), 0, s, ca, (int64_t *)nullptr,
                           kept.p, c.rowptr.p, c.col.p, c.desc.p);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_rows_wave<true>, dim3(grid_for(n_add * 64, 256)), dim3(256), 0, s, ra,
                           (int64_t *)nullptr, c.rowptr.p, c.col.p, c.desc.p);
        HQ_LAUNCH_CHECK();
    }
    build_elements_after(c, kept.p);  // new entries' values, every diagonal element
    compute_xcd_rows(c);
    for (auto &row : c.sigma_cfg)
        for (auto &g : row) g = SigmaCfg{};

    // ---- warm start: kept coefficients carried over, appended ones zero
    if (c_old && c_new) {
        hipLaunchKernelGGL(k_zero, dim3(grid_for(n_new, 256)), dim3(256), 0, s, c_new, n_new);
        HQ_LAUNCH_CHECK();
        if (sorted) {
            hipLaunchKernelGGL(k_carry_scatter, dim3(grid_for(n_old, 256)), dim3(256), 0, s, c_old, n_old, o2n.p,
                               (const int32_t *)nullptr, c_new);
        } else {
            hipLaunchKernelGGL(k_carry_scatter, dim3(grid_for(n_old, 256)), dim3(256), 0, s, c_old, n_old,
                               newidx.p, keep.p, c_new);
        }
        HQ_LAUNCH_CHECK();
    }
    HQ_CHECK(hipStreamSynchronize(s));
    c.have_elements = true;
    if (ms_out)
        *ms_out = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// The basis-update rules of Sec. 2.2, Step 2, on top of update_determinants:
//   GROW_APPEND   append the K best-scored candidates (highest score first);
//                 when |B| + K exceeds bmax (> 0), drop the lowest-scored of B
//                 and of those K until bmax remain;
//   GROW_REBUILD  keep the K best-scored of B and the candidates together
//                 (B's survivors in their order, then the chosen candidates,
//                 highest score first); no cap.
// Ties go to the lower index of the list [B (caller order); candidates].
int64_t grow_basis(Ctx &c, int mode, int64_t ncand, const uint64_t *ca, const uint64_t *cb, const double *cscore,
                   int64_t k, const double *bscore, int64_t bmax, const double *c_old, double *c_new,
                   double *score_new, double *ms_out) {
    hipStream_t s = c.stream;
    const int64_t nb = c.ndet;
    DBuf<int32_t> order, flag, pos, evict, applist;
    DBuf<double> comb, app_score;
    DBuf<uint64_t> app_a, app_b;
    int64_t n_app = 0, n_ev = 0;
    auto count_flags = [&](const int32_t *f, const int32_t *p, int64_t n) {
        int32_t last[2] = {0, 0};
        HQ_CHECK(hipMemcpyAsync(&last[0], p + n - 1, 4, hipMemcpyDeviceToHost, s));
        HQ_CHECK(hipMemcpyAsync(&last[1], f + n - 1, 4, hipMemcpyDeviceToHost, s));
        HQ_CHECK(hipStreamSynchronize(s));
        return (int64_t)last[0] + last[1];
    };
    // flag[0..nb) marks B entries to keep (1); the appended candidates are listed in applist
    flag.ensure(nb);
    pos.ensure(nb);
    if (mode == HINQS_GROW_APPEND) {
        const int64_t kk = std::min(k, ncand);
        order.ensure(std::max<int64_t>(kk, 1));
        if (kk > 0) top_k(c, ncand, cscore, kk, true, order.p);
        hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nb, 256)), dim3(256), 0, s, flag.p, nb, 1);
        HQ_LAUNCH_CHECK();
        DBuf<int32_t> aflag, apos;
        aflag.ensure(std::max<int64_t>(kk, 1));
        apos.ensure(std::max<int64_t>(kk, 1));
        hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(kk, 256)), dim3(256), 0, s, aflag.p, kk, 1);
        HQ_LAUNCH_CHECK();
        if (bmax > 0 && nb + kk > bmax) {
            const int64_t m = nb + kk - bmax;
            comb.ensure(nb + kk);
            hipLaunchKernelGGL(k_combine, dim3(grid_for(nb + kk, 256)), dim3(256), 0, s, bscore, nb, cscore,
                               order.p, kk, comb.p);
            HQ_LAUNCH_CHECK();
            DBuf<int32_t> low, dropped;
            low.ensure(m);
            top_k(c, nb + kk, comb.p, m, false, low.p);
            dropped.ensure(nb + kk);
            hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nb + kk, 256)), dim3(256), 0, s, dropped.p, nb + kk, 0);
            HQ_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_flag_chosen, dim3(grid_for(m, 256)), dim3(256), 0, s, low.p, m, dropped.p);
            HQ_LAUNCH_CHECK();
            // keep = 1 - dropped, for B and for the K chosen candidates
            hipLaunchKernelGGL(k_invert_flags, dim3(grid_for(nb, 256)), dim3(256), 0, s, dropped.p, nb, flag.p);
            HQ_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_invert_flags, dim3(grid_for(kk, 256)), dim3(256), 0, s, dropped.p + nb, kk, aflag.p);
            HQ_LAUNCH_CHECK();
        }
        if (kk > 0) {
            exclusive_scan_i32(s, aflag.p, apos.p, kk, c.work);
            n_app = count_flags(aflag.p, apos.p, kk);
            applist.ensure(std::max<int64_t>(n_app, 1));
            hipLaunchKernelGGL(k_compact_i32, dim3(grid_for(kk, 256)), dim3(256), 0, s, aflag.p, apos.p, kk, 1,
                               order.p, 0, applist.p);
            HQ_LAUNCH_CHECK();
        }
    } else if (mode == HINQS_GROW_REBUILD) {
        const int64_t nt = nb + ncand;
        const int64_t kk = std::min(k, nt);
        comb.ensure(nt);
        hipLaunchKernelGGL(k_combine, dim3(grid_for(nt, 256)), dim3(256), 0, s, bscore, nb, cscore,
                           (const int32_t *)nullptr, ncand, comb.p);
        HQ_LAUNCH_CHECK();
        order.ensure(kk);
        top_k(c, nt, comb.p, kk, true, order.p);
        DBuf<int32_t> chosen, tflag, tpos;
        chosen.ensure(nt);
        hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nt, 256)), dim3(256), 0, s, chosen.p, nt, 0);
        HQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_flag_chosen, dim3(grid_for(kk, 256)), dim3(256), 0, s, order.p, kk, chosen.p);
        HQ_LAUNCH_CHECK();
        HQ_CHECK(hipMemcpyAsync(flag.p, chosen.p, sizeof(int32_t) * nb, hipMemcpyDeviceToDevice, s));
        // the chosen candidates, in the order of the top list
        tflag.ensure(kk);
        tpos.ensure(kk);
        hipLaunchKernelGGL(k_is_candidate, dim3(grid_for(kk, 256)), dim3(256), 0, s, order.p, kk, nb, tflag.p);
        HQ_LAUNCH_CHECK();
        exclusive_scan_i32(s, tflag.p, tpos.p, kk, c.work);
        n_app = count_flags(tflag.p, tpos.p, kk);
        applist.ensure(std::max<int64_t>(n_app, 1));
        hipLaunchKernelGGL(k_compact_i32, dim3(grid_for(kk, 256)), dim3(256), 0, s, tflag.p, tpos.p, kk, 1, order.p,
                           nb, applist.p);
        HQ_LAUNCH_CHECK();
    } else {
        throw Error(HINQS_E_INVALID_ARG, "unknown update mode");
    }
    // evicted = B entries with flag 0
    exclusive_scan_i32(s, flag.p, pos.p, nb, c.work);
    const int64_t n_keep = count_flags(flag.p, pos.p, nb);
    n_ev = nb - n_keep;
    DBuf<int32_t> epos, eflag;
    if (n_ev > 0) {
        evict.ensure(n_ev);
        eflag.ensure(nb);
        epos.ensure(nb);
        hipLaunchKernelGGL(k_invert_flags, dim3(grid_for(nb, 256)), dim3(256), 0, s, flag.p, nb, eflag.p);
        HQ_LAUNCH_CHECK();
        exclusive_scan_i32(s, eflag.p, epos.p, nb, c.work);
        hipLaunchKernelGGL(k_compact_i32, dim3(grid_for(nb, 256)), dim3(256), 0, s, eflag.p, epos.p, nb, 1,
                           (const int32_t *)nullptr, 0, evict.p);
        HQ_LAUNCH_CHECK();
    }
    if (n_app > 0) {
        app_a.ensure(n_app);
        app_b.ensure(n_app);
        app_score.ensure(n_app);
        hipLaunchKernelGGL(k_gather_cand, dim3(grid_for(n_app, 256)), dim3(256), 0, s, applist.p, n_app, ca, cb,
                           cscore, app_a.p, app_b.p, app_score.p);
        HQ_LAUNCH_CHECK();
    }
    update_determinants(c, n_ev, evict.p, n_app, app_a.p, app_b.p, c_old, c_new, false, ms_out);
    if (score_new) {
        hipLaunchKernelGGL(k_new_scores, dim3(grid_for(nb + n_app, 256)), dim3(256), 0, s, bscore, flag.p, pos.p, nb,
                           app_score.p, n_app, n_keep, score_new);
        HQ_LAUNCH_CHECK();
        HQ_CHECK(hipStreamSynchronize(s));
    }
    return n_keep + n_app;
}

namespace {
__global__ void k_caller_strings(const uint32_t *sa, const uint32_t *sb, const int32_t *perm, int64_t n,
                                 uint64_t *oa, uint64_t *ob) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (oa) oa[perm[p]] = sa[p];
    if (ob) ob[perm[p]] = sb[p];
}
}  // namespace

void caller_strings(Ctx &c, uint64_t *alpha, uint64_t *beta) {
    hipLaunchKernelGGL(k_caller_strings, dim3(grid_for(c.ndet, 256)), dim3(256), 0, c.stream, c.sa.p, c.sb.p,
                       c.perm.p, c.ndet, alpha, beta);
    HQ_LAUNCH_CHECK();
    HQ_CHECK(hipStreamSynchronize(c.stream));
}

}  // namespace hinqs
