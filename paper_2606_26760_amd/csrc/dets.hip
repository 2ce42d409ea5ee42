// Determinant store: validation, sort, string tables and single-move links.
//
// B (the sampled basis of Sec. 2.2, Steps 1-3) is kept sorted alpha-major,
// then beta, as pairs of uint32 strings.  Around it sit:
//   ua / ga / aidx      distinct alpha strings, their groups (contiguous runs
//                       of the sorted order), and each determinant's group;
//   ub / gb / bperm     the same for beta, over a beta-major listing;
//   alink               for every distinct alpha string, the single moves that
//                       land on another distinct alpha string of B.
// The duplicate check follows the paper's removal of repeated configurations
// (Step 1): a repeated pair is rejected instead of silently merged.
#include <chrono>

#include "common.hpp"

namespace hinqs {

namespace {

__global__ void k_make_keys(const uint32_t *a, const uint32_t *b, int64_t n, int norb, uint64_t *keys,
                            int32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = ((uint64_t)a[i] << norb) | (uint64_t)b[i];
    vals[i] = (int32_t)i;
}

__global__ void k_unpack_sorted(const uint64_t *keys, const int32_t *vals, int64_t n, int norb,
                                uint32_t *sa, uint32_t *sb, int32_t *perm, int32_t *inv,
                                int32_t *flag_a, int32_t *dup) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t mask = (norb >= 32) ? 0xffffffffull : ((1ull << norb) - 1ull);
    uint64_t k = keys[i];
    uint32_t a = (uint32_t)(k >> norb), b = (uint32_t)(k & mask);
    sa[i] = a;
    sb[i] = b;
    perm[i] = vals[i];
    inv[vals[i]] = (int32_t)i;
    bool first = (i == 0) || ((keys[i - 1] >> norb) != (k >> norb));
    flag_a[i] = first ? 1 : 0;
    if (i > 0 && keys[i - 1] == k) *dup = 1;
}

// From exclusive scan of first-of-group flags: group index, distinct string, offsets.
__global__ void k_groups(const uint32_t *s, const int32_t *flag, const int32_t *scan, int64_t n,
                         int32_t *gidx, uint32_t *uniq, int32_t *goff) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t g = scan[i] + flag[i] - 1;
    gidx[i] = g;
    if (flag[i]) {
        uniq[g] = s[i];
        goff[g] = (int32_t)i;
    }
}

__global__ void k_set_last(int32_t *goff, const int32_t *scan, const int32_t *flag, int64_t n) {
    // number of groups = scan[n-1] + flag[n-1]; goff[ngroups] = n
    int32_t ng = scan[n - 1] + flag[n - 1];
    goff[ng] = (int32_t)n;
}

__global__ void k_unpack_beta_major(const uint64_t *keys, const int32_t *vals, int64_t n, int norb,
                                    uint32_t *sbm, int32_t *bperm, uint32_t *bm_alpha,
                                    int32_t *flag_b) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint64_t mask = (norb >= 32) ? 0xffffffffull : ((1ull << norb) - 1ull);
    uint64_t k = keys[t];
    sbm[t] = (uint32_t)(k >> norb);
    bm_alpha[t] = (uint32_t)(k & mask);
    bperm[t] = vals[t];
    bool first = (t == 0) || ((keys[t - 1] >> norb) != (k >> norb));
    flag_b[t] = first ? 1 : 0;
}

__global__ void k_bidx(const int32_t *bperm, const int32_t *gidx_bm, int64_t n, int32_t *bidx) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    bidx[bperm[t]] = gidx_bm[t];
}

// Binary search of `key` in ascending `u[0..n)`; -1 if absent.
__device__ inline int32_t find_string(const uint32_t *u, int32_t n, uint32_t key) {
    int32_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int32_t mid = (lo + hi) >> 1;
        uint32_t v = u[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// For each distinct alpha string s = ua[u] and each move r -> q (r occupied, q empty),
// the string t = s - r + q if it is also in B.  For a coupled pair whose bra has
// alpha string s and ket alpha string t, the alpha hole (occupied in t) is q and
// the alpha particle (occupied in s) is r.
__global__ void k_alpha_links(const uint32_t *ua, int32_t nua, int norb, int maxl, int32_t *cnt,
                              int32_t *link, uint32_t *info) {
    int32_t u = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (u >= nua) return;
    uint32_t s = ua[u];
    uint32_t full = (norb >= 32) ? 0xffffffffu : ((1u << norb) - 1u);
    int c = 0;
    for (uint32_t occ = s; occ; occ &= occ - 1) {
        int r = lowbit(occ);
        for (uint32_t emp = ~s & full; emp; emp &= emp - 1) {
            int q = lowbit(emp);
            uint32_t t = s ^ (1u << r) ^ (1u << q);
            int32_t v = find_string(ua, nua, t);
            if (v >= 0) {
                int64_t at = (int64_t)u * maxl + c;
                link[at] = v;
                info[at] = (uint32_t)q | ((uint32_t)r << 5) | (single_parity(t, q, r) << 10);
                ++c;
            }
        }
    }
    cnt[u] = c;
}

template <int ROWBYTES>
__global__ void k_gather_rows(const char *src, char *dst, const int32_t *idx, int64_t n) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const char *s = src + (int64_t)idx[r] * ROWBYTES;
    char *d = dst + r * ROWBYTES;
    if constexpr (ROWBYTES % 16 == 0) {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 16) *(uint4 *)(d + b) = *(const uint4 *)(s + b);
    } else if constexpr (ROWBYTES % 8 == 0) {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 8) *(uint2 *)(d + b) = *(const uint2 *)(s + b);
    } else {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 4) *(uint32_t *)(d + b) = *(const uint32_t *)(s + b);
    }
}

template <int ROWBYTES>
__global__ void k_scatter_rows(const char *src, char *dst, const int32_t *idx, int64_t n) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const char *s = src + r * ROWBYTES;
    char *d = dst + (int64_t)idx[r] * ROWBYTES;
    if constexpr (ROWBYTES % 16 == 0) {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 16) *(uint4 *)(d + b) = *(const uint4 *)(s + b);
    } else if constexpr (ROWBYTES % 8 == 0) {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 8) *(uint2 *)(d + b) = *(const uint2 *)(s + b);
    } else {
#pragma unroll
        for (int b = 0; b < ROWBYTES; b += 4) *(uint32_t *)(d + b) = *(const uint32_t *)(s + b);
    }
}

void row_copy(hipStream_t s, const void *src, void *dst, const int32_t *idx, int64_t n, int rowbytes,
              bool gather) {
    if (n <= 0) return;
    dim3 g(grid_for(n, 256)), b(256);
    const char *S = (const char *)src;
    char *D = (char *)dst;
#define HQ_ROWCASE(RB)                                                                  \
    case RB:                                                                            \
        if (gather) hipLaunchKernelGGL(k_gather_rows<RB>, g, b, 0, s, S, D, idx, n);   \
        else hipLaunchKernelGGL(k_scatter_rows<RB>, g, b, 0, s, S, D, idx, n);         \
        break;
    switch (rowbytes) {
        HQ_ROWCASE(4) HQ_ROWCASE(8) HQ_ROWCASE(16) HQ_ROWCASE(24) HQ_ROWCASE(32) HQ_ROWCASE(40)
        HQ_ROWCASE(48) HQ_ROWCASE(56) HQ_ROWCASE(64) HQ_ROWCASE(72) HQ_ROWCASE(80) HQ_ROWCASE(88)
        HQ_ROWCASE(96) HQ_ROWCASE(104) HQ_ROWCASE(112) HQ_ROWCASE(120) HQ_ROWCASE(128)
        default:
            throw Error(HINQS_E_UNSUPPORTED, "row size " + std::to_string(rowbytes));
    }
#undef HQ_ROWCASE
    HQ_LAUNCH_CHECK();
}

}  // namespace

void gather_rows(hipStream_t s, const void *src, void *dst, const int32_t *idx, int64_t n,
                 int rowbytes) {
    row_copy(s, src, dst, idx, n, rowbytes, true);
}
void scatter_rows(hipStream_t s, const void *src, void *dst, const int32_t *idx, int64_t n,
                  int rowbytes) {
    row_copy(s, src, dst, idx, n, rowbytes, false);
}

namespace {

// Checks every determinant (electron counts, no orbital >= norb) and narrows the
// strings to uint32.  bad[0] receives the lowest offending index (INT64_MAX if
// none), bad[1] a bit set: 1 = orbital >= norb, 2 = wrong electron count.
__global__ void k_validate(const uint64_t *a64, const uint64_t *b64, int64_t n, int norb, int na, int nb,
                           uint32_t *a32, uint32_t *b32, unsigned long long *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t full = (norb >= 64) ? ~0ull : ((1ull << norb) - 1ull);
    const uint64_t a = a64[i], b = b64[i];
    unsigned long long kind = 0;
    if ((a & ~full) || (b & ~full)) kind |= 1ull;
    if (__popcll(a) != na || __popcll(b) != nb) kind |= 2ull;
    if (kind) {
        atomicMin(&bad[0], (unsigned long long)i);
        atomicOr(&bad[1], kind);
    }
    a32[i] = (uint32_t)a;
    b32[i] = (uint32_t)b;
}

}  // namespace

void build_determinants(Ctx &c, int64_t ndet, const uint64_t *alpha, const uint64_t *beta, int na,
                        int nb, bool on_device) {
    const int norb = c.norb;
    auto t0 = std::chrono::steady_clock::now();
    c.have_dets = false;
    c.have_elements = false;
    hipStream_t s = c.stream;
    auto &up_a = c.bs.up_a, &up_b = c.bs.up_b;
    const uint64_t *da64 = alpha, *db64 = beta;
    if (!on_device) {
        up_a.ensure(ndet);
        up_b.ensure(ndet);
        HQ_CHECK(hipMemcpyAsync(up_a.p, alpha, 8 * ndet, hipMemcpyHostToDevice, s));
        HQ_CHECK(hipMemcpyAsync(up_b.p, beta, 8 * ndet, hipMemcpyHostToDevice, s));
        da64 = up_a.p;
        db64 = up_b.p;
    }
    auto &da = c.bs.da, &db = c.bs.db;
    da.ensure(ndet);
    db.ensure(ndet);
    auto &bad = c.bs.bad;
    bad.ensure(2);
    unsigned long long init[2] = {~0ull, 0ull};
    HQ_CHECK(hipMemcpyAsync(bad.p, init, sizeof(init), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_validate, dim3(grid_for(ndet, 256)), dim3(256), 0, s, da64, db64, ndet, norb, na,
                       nb, da.p, db.p, bad.p);
    HQ_LAUNCH_CHECK();
    unsigned long long hbad[2];
    HQ_CHECK(hipMemcpyAsync(hbad, bad.p, sizeof(hbad), hipMemcpyDeviceToHost, s));
    wait_stream(s);
    if (hbad[1] & 1ull)
        throw Error(HINQS_E_BAD_OCCUPATION, "determinant " + std::to_string(hbad[0]) +
                                                " (or another) has an occupied orbital >= norb");
    if (hbad[1] & 2ull)
        throw Error(HINQS_E_BAD_OCCUPATION,
                    "determinant " + std::to_string(hbad[0]) + " (or another) has the wrong electron count");
    c.ndet = ndet;
    c.na = na;
    c.nb = nb;

    auto &keys = c.bs.keys;
    auto &vals = c.bs.vals, &flag = c.bs.flag, &scan = c.bs.scan, &dup = c.bs.dup;
    keys.ensure(ndet);
    vals.ensure(ndet);
    flag.ensure(ndet);
    scan.ensure(ndet);
    dup.ensure(1);
    HQ_CHECK(hipMemsetAsync(dup.p, 0, sizeof(int32_t), s));
    dim3 g(grid_for(ndet, 256)), b(256);
    hipLaunchKernelGGL(k_make_keys, g, b, 0, s, da.p, db.p, ndet, norb, keys.p, vals.p);
    HQ_LAUNCH_CHECK();
    radix_sort_u64(s, keys.p, vals.p, ndet, 2 * norb, c.work, c.bs.sort);

    c.sa.ensure(ndet);
    c.sb.ensure(ndet);
    c.perm.ensure(ndet);
    c.inv.ensure(ndet);
    hipLaunchKernelGGL(k_unpack_sorted, g, b, 0, s, keys.p, vals.p, ndet, norb, c.sa.p, c.sb.p,
                       c.perm.p, c.inv.p, flag.p, dup.p);
    HQ_LAUNCH_CHECK();
    int32_t hdup = 0;
    HQ_CHECK(hipMemcpyAsync(&hdup, dup.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    wait_stream(s);
    if (hdup) throw Error(HINQS_E_DUPLICATE, "the determinant set contains a duplicate");

    // ---- alpha groups
    exclusive_scan_i32(s, flag.p, scan.p, ndet, c.work);
    int32_t last[2];
    HQ_CHECK(hipMemcpyAsync(&last[0], scan.p + ndet - 1, 4, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&last[1], flag.p + ndet - 1, 4, hipMemcpyDeviceToHost, s));
    wait_stream(s);
    c.nua = last[0] + last[1];
    c.ua.ensure(c.nua);
    c.ga.ensure(c.nua + 1);
    c.aidx.ensure(ndet);
    hipLaunchKernelGGL(k_groups, g, b, 0, s, c.sa.p, flag.p, scan.p, ndet, c.aidx.p, c.ua.p, c.ga.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, c.ga.p, scan.p, flag.p, ndet);
    HQ_LAUNCH_CHECK();

    // ---- beta-major listing: keys (beta << norb | alpha), values = sorted position
    hipLaunchKernelGGL(k_make_keys, g, b, 0, s, c.sb.p, c.sa.p, ndet, norb, keys.p, vals.p);
    HQ_LAUNCH_CHECK();
    radix_sort_u64(s, keys.p, vals.p, ndet, 2 * norb, c.work, c.bs.sort);
    auto &sbm = c.bs.sbm;
    sbm.ensure(ndet);
    c.bperm.ensure(ndet);
    c.bm_alpha.ensure(ndet);
    hipLaunchKernelGGL(k_unpack_beta_major, g, b, 0, s, keys.p, vals.p, ndet, norb, sbm.p, c.bperm.p,
                       c.bm_alpha.p, flag.p);
    HQ_LAUNCH_CHECK();
    exclusive_scan_i32(s, flag.p, scan.p, ndet, c.work);
    HQ_CHECK(hipMemcpyAsync(&last[0], scan.p + ndet - 1, 4, hipMemcpyDeviceToHost, s));
    HQ_CHECK(hipMemcpyAsync(&last[1], flag.p + ndet - 1, 4, hipMemcpyDeviceToHost, s));
    wait_stream(s);
    c.nub = last[0] + last[1];
    c.ub.ensure(c.nub);
    c.gb.ensure(c.nub + 1);
    auto &gidx_bm = c.bs.gidx;
    gidx_bm.ensure(ndet);
    hipLaunchKernelGGL(k_groups, g, b, 0, s, sbm.p, flag.p, scan.p, ndet, gidx_bm.p, c.ub.p, c.gb.p);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, c.gb.p, scan.p, flag.p, ndet);
    HQ_LAUNCH_CHECK();
    c.bidx.ensure(ndet);
    hipLaunchKernelGGL(k_bidx, g, b, 0, s, c.bperm.p, gidx_bm.p, ndet, c.bidx.p);
    HQ_LAUNCH_CHECK();

    // ---- alpha single-move links between distinct strings of B
    int maxl = na * (norb - na);
    if (maxl < 1) maxl = 1;
    c.alink_max = maxl;
    c.alink_ptr.ensure(c.nua);
    c.alink.ensure((size_t)c.nua * maxl);
    c.alink_info.ensure((size_t)c.nua * maxl);
    hipLaunchKernelGGL(k_alpha_links, dim3(grid_for(c.nua, 128)), dim3(128), 0, s, c.ua.p, c.nua, norb,
                       maxl, c.alink_ptr.p, c.alink.p, c.alink_info.p);
    HQ_LAUNCH_CHECK();
    wait_stream(s);
    c.ms_sort = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c.have_dets = true;
}

}  // namespace hinqs
