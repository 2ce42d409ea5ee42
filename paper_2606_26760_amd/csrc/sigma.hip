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
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

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

// A value known to be equal on all lanes of the wave, moved to a scalar register
// so that loops over it branch on the scalar unit.
template <bool UNIFORM>
__device__ inline int64_t uniform_if(int64_t v) {
    if constexpr (UNIFORM) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    } else {
        return v;
    }
}

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

// Persistent teams: TEAM lanes own one row at a time and walk a strided list
// of rows.  Rows are split into 8 contiguous ranges holding equal numbers of
// couplings, one per XCD (hardware block b runs on XCD b % 8; the coupling
// count per row varies several-fold along the sorted order, so equal row
// counts would leave most XCDs idle behind the densest one), and inside a
// range consecutive teams take
// consecutive rows, so the rows in flight on an XCD are neighbours in the
// sorted order and gather overlapping X rows from that XCD's L2.  LPN lanes
// share one coupling: each loads EPL consecutive entries (16 bytes) of the
// gathered X row, so one load instruction touches 64 / LPN distinct rows and
// every row is read as one contiguous segment.
// The CSR stream is software-pipelined: while the X rows of one step (UNR
// couplings per lane) are in flight, the (col, val) of the next step and the
// bounds of the team's next row are already being fetched, so the dependent
// load chain rowptr -> col -> X costs one memory latency per step, not three.
struct XcdRows {
    int64_t b[NUM_XCD + 1];
};

// MASK (batched instances): the XCD row ranges come from device memory and the
// rows of finished instances are skipped; a team jumps over a finished
// instance in one step, so the cost does not grow with its size.
// Row counters (ctr, not for MASK): instead of a fixed stride, the team
// leader takes the XCD's next run of `run` rows from a counter, so the teams of an XCD stay
// on neighbouring rows however unequal the rows are; with fixed strides the
// teams drift apart and the X rows in flight no longer share the XCD's L2
// (a trace-driven model of the gathers gives 53 % L2 hits for strides and
// 80 % for a shared counter).  The next run is requested when a run starts,
// so the atomic's latency hides behind the current rows; runs of several
// rows keep the counters from becoming a hot spot in their L2 channels.  The
// last team of an XCD to finish puts its counters back to zero for the next
// launch.  ctr: CTR_STRIDE words per XCD, word 0 = next row, word
// CTR_DONE = teams finished.
constexpr int CTR_STRIDE = SIGMA_CTR_WORDS / NUM_XCD;
constexpr int CTR_DONE = 16;

template <typename T, int K, int TEAM, int UNR, bool MASK>
__global__ __launch_bounds__(SIGMA_BLOCK) void k_sigma(XcdRows ranges, SigmaMask mk, int xcd_map,
                                                       const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ X, int ldx,
                                                       T *__restrict__ S, int lds,
                                                       unsigned long long *ctr, int run) {
    constexpr int VW = Vec16<T>::n;
    constexpr int LPN = (K >= VW) ? K / VW : 1;   // lanes per coupling
    constexpr int EPL = K / LPN;                   // entries of X per lane
    constexpr int NPT = TEAM / LPN;                // couplings per team per unrolled slot
    constexpr int STEP = UNR * NPT;                // couplings per team step
    constexpr int TPB = SIGMA_BLOCK / TEAM;        // teams per block
    static_assert(TEAM % LPN == 0 && TEAM <= 64, "team shape");
    const int64_t blocks_per_xcd = gridDim.x / NUM_XCD;
    const int xcd = xcd_map ? blockIdx.x % NUM_XCD : blockIdx.x / blocks_per_xcd;
    const int64_t bix = xcd_map ? blockIdx.x / NUM_XCD : blockIdx.x % blocks_per_xcd;
    const int64_t team0 = bix * TPB + threadIdx.x / TEAM;
    const int64_t nteams = blocks_per_xcd * TPB;
    const int64_t r0 = MASK ? mk.ranges[xcd] : ranges.b[xcd];
    const int64_t r1 = MASK ? mk.ranges[xcd + 1] : ranges.b[xcd + 1];
    const int sub = threadIdx.x % TEAM;
    const int q = sub % LPN, g = sub / LPN;
    const T *Xq = X + q * EPL;
    // MASK: instance of the last row looked up (rows only increase)
    int64_t inst_end = -1;
    bool inst_done = false;
    auto live_row = [&](int64_t rw) -> int64_t {
        if constexpr (MASK) {
            while (rw < r1) {
                if (rw >= inst_end) {
                    const int32_t b = mk.row_inst[rw];
                    inst_end = mk.inst_row[b + 1];
                    inst_done = mk.done[b] != 0;
                }
                if (!inst_done) break;
                rw += (inst_end - rw + nteams - 1) / nteams * nteams;
            }
        }
        return rw;
    };
    const bool dyn = !MASK && ctr != nullptr;
    unsigned long long *const myctr = dyn ? ctr + xcd * CTR_STRIDE : nullptr;
    auto take = [&]() -> unsigned long long {  // result valid on the team leader only
        unsigned long long v = 0;
        if (sub == 0) v = atomicAdd(myctr, (unsigned long long)run);
        return v;
    };
    auto first_row = [&](unsigned long long v) -> int64_t { return r0 + (int64_t)__shfl(v, 0, TEAM); };
    int64_t run_end = 0;  // end of the run of rows taken last
    auto finish = [&]() {
        if (dyn && sub == 0) {
            const unsigned long long d = atomicAdd(myctr + CTR_DONE, 1ull);
            if (d + 1 == (unsigned long long)nteams) {
                atomicExch(myctr, 0ull);
                atomicExch(myctr + CTR_DONE, 0ull);
            }
        }
    };
    unsigned long long pend = 0;
    int64_t row;
    if (dyn) {
        row = first_row(take());
        run_end = min(row + run, r1);
        if (row < r1) pend = take();
    } else {
        row = live_row(r0 + team0);
    }
    if (row >= r1) {  // uniform across the team
        finish();
        return;
    }
    int64_t beg = uniform_if<TEAM == 64>(rowptr[row]), end = uniform_if<TEAM == 64>(rowptr[row + 1]);
    for (;;) {
        int64_t nrow;
        if (dyn) {
            if (row + 1 < run_end) {
                nrow = row + 1;
            } else {
                nrow = first_row(pend);
                run_end = min(nrow + run, r1);
                if (nrow < r1) pend = take();
            }
        } else {
            nrow = live_row(row + nteams);
        }
        // next row's bounds, in flight during this row (clamped, not predicated)
        const int64_t nrc = nrow < r1 ? nrow : row;
        const int64_t nbeg = rowptr[nrc], nend = rowptr[nrc + 1];
        T acc[EPL];
#pragma unroll
        for (int c = 0; c < EPL; ++c) acc[c] = T(0);
        // Software pipeline with two register sets (a, b): while the X rows of
        // one step are in flight, the (col, val) of the next step are fetched
        // into the other set, so no loop-carried copy has to wait for a load.
        // Loads are never predicated: indices past the row are clamped to a
        // valid entry and their value is replaced by 0 at the point of use.
        const int64_t last = end > 0 ? end - 1 : 0;
        int32_t ja[UNR], jb[UNR];
        T va[UNR], vb[UNR];
        bool oka[UNR], okb[UNR];
        auto fetch = [&](int64_t eb, int32_t (&jj)[UNR], T (&vv)[UNR], bool (&ok)[UNR]) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t idx = eb + g + u * NPT;
                ok[u] = idx < end;
                const int64_t idc = ok[u] ? idx : last;
                jj[u] = __builtin_nontemporal_load(col + idc);
                vv[u] = __builtin_nontemporal_load(val + idc);
            }
        };
        auto step = [&](const int32_t (&jj)[UNR], const T (&vv)[UNR], const bool (&ok)[UNR],
                        int64_t eb_next, int32_t (&jn)[UNR], T (&vn)[UNR], bool (&okn)[UNR]) {
            T x[UNR][EPL];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int32_t jr = ok[u] ? jj[u] : (int32_t)row;
                load_vec<T, EPL>(Xq + (int64_t)jr * ldx, x[u]);
            }
            fetch(eb_next, jn, vn, okn);
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const T w = ok[u] ? vv[u] : T(0);
#pragma unroll
                for (int c = 0; c < EPL; ++c) acc[c] += w * x[u][c];
            }
        };
        int64_t eb = beg;
        fetch(eb, ja, va, oka);
        while (eb < end) {  // same trip count on every lane of the team
            step(ja, va, oka, eb + STEP, jb, vb, okb);
            eb += STEP;
            if (eb >= end) break;
            step(jb, vb, okb, eb + STEP, ja, va, oka);
            eb += STEP;
        }
#pragma unroll
        for (int off = LPN; off < TEAM; off <<= 1) {
#pragma unroll
            for (int c = 0; c < EPL; ++c) acc[c] += __shfl_xor(acc[c], off, TEAM);
        }
        if (g == 0) {
            if (diag) {   // null: off-diagonal part only (the caller adds the diagonal itself)
                const T d = diag[row];
                T xr[EPL];
                load_vec<T, EPL>(Xq + row * ldx, xr);
#pragma unroll
                for (int c = 0; c < EPL; ++c) acc[c] += d * xr[c];
            }
            store_vec<T, EPL>(S + row * lds + q * EPL, acc);
        }
        if (nrow >= r1) break;
        row = nrow;
        beg = uniform_if<TEAM == 64>(nbeg);
        end = uniform_if<TEAM == 64>(nend);
    }
    finish();
}

// Cross-row pipelined variant.  A team walks its rows as one stream of steps
// (UNR * TEAM / LPN couplings of one row per step; an empty row is one step
// with none), and four register sets rotate through the stages of a step:
//   stage t:  fetch (col, val) of step t+2;  gather the X rows of step t+1;
//             accumulate step t-1 (and finish its row if it is the row's last)
// so two steps of X gathers are in flight while a third is accumulated, with
// no bubble at row boundaries.  Every step also fetches its row's diagonal
// element and X row (used by the row's last step), so each stage issues the
// same loads in the same order and the hardware's in-order load counter never
// forces a wait on younger gathers.
template <typename T, int K, int TEAM, int UNR, bool MASK>
__global__ __launch_bounds__(SIGMA_BLOCK) void k_sigma_xr(XcdRows ranges, SigmaMask mk, int xcd_map,
                                                          const int64_t *__restrict__ rowptr,
                                                          const int32_t *__restrict__ col,
                                                          const T *__restrict__ val,
                                                          const T *__restrict__ diag,
                                                          const T *__restrict__ X, int ldx,
                                                          T *__restrict__ S, int lds) {
    constexpr int VW = Vec16<T>::n;
    constexpr int LPN = (K >= VW) ? K / VW : 1;   // lanes per coupling
    constexpr int EPL = K / LPN;                   // entries of X per lane
    constexpr int NPT = TEAM / LPN;                // couplings per team per unrolled slot
    constexpr int STEP = UNR * NPT;                // couplings per team step
    constexpr int TPB = SIGMA_BLOCK / TEAM;        // teams per block
    constexpr bool UNI = TEAM == 64;
    static_assert(TEAM % LPN == 0 && TEAM <= 64, "team shape");
    const int64_t blocks_per_xcd = gridDim.x / NUM_XCD;
    const int xcd = xcd_map ? blockIdx.x % NUM_XCD : blockIdx.x / blocks_per_xcd;
    const int64_t bix = xcd_map ? blockIdx.x / NUM_XCD : blockIdx.x % blocks_per_xcd;
    const int64_t team0 = bix * TPB + threadIdx.x / TEAM;
    const int64_t nteams = blocks_per_xcd * TPB;
    const int64_t r0 = MASK ? mk.ranges[xcd] : ranges.b[xcd];
    const int64_t r1 = MASK ? mk.ranges[xcd + 1] : ranges.b[xcd + 1];
    const int sub = threadIdx.x % TEAM;
    const int q = sub % LPN, g = sub / LPN;
    const T *Xq = X + q * EPL;
    int64_t inst_end = -1;
    bool inst_done = false;
    auto live_row = [&](int64_t rw) -> int64_t {
        if constexpr (MASK) {
            while (rw < r1) {
                if (rw >= inst_end) {
                    const int32_t b = mk.row_inst[rw];
                    inst_end = mk.inst_row[b + 1];
                    inst_done = mk.done[b] != 0;
                }
                if (!inst_done) break;
                rw += (inst_end - rw + nteams - 1) / nteams * nteams;
            }
        }
        return rw;
    };
    // step generator (the same on every lane of a team)
    int64_t g_row = live_row(r0 + team0);
    if (g_row >= r1) return;
    const int64_t safe_row = g_row;  // an in-range row for clamped loads
    int64_t g_eb = uniform_if<UNI>(rowptr[g_row]), g_end = uniform_if<UNI>(rowptr[g_row + 1]);
    int64_t n_row = live_row(g_row + nteams);
    int64_t n_beg, n_end;
    {
        const int64_t c = n_row < r1 ? n_row : safe_row;
        n_beg = rowptr[c];
        n_end = rowptr[c + 1];
    }
    struct Slot {
        int32_t j[UNR];
        T v[UNR];
        bool ok[UNR];
        T x[UNR][EPL];
        T dx[EPL];
        T dd;
        int64_t row;
        bool last, valid;
    };
    Slot s0, s1, s2, s3;
    auto emit = [&](Slot &sl) {
        sl.valid = g_row < r1;
        sl.row = sl.valid ? g_row : safe_row;
        sl.last = g_eb + STEP >= g_end;
        const int64_t lastidx = g_end > 0 ? g_end - 1 : 0;
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t idx = g_eb + g + u * NPT;
            sl.ok[u] = sl.valid && idx < g_end;
            const int64_t idc = sl.ok[u] ? idx : lastidx;
            sl.j[u] = __builtin_nontemporal_load(col + idc);
            sl.v[u] = __builtin_nontemporal_load(val + idc);
        }
        if (sl.valid) {
            g_eb += STEP;
            if (g_eb >= g_end) {
                g_row = n_row;
                g_eb = uniform_if<UNI>(n_beg);
                g_end = uniform_if<UNI>(n_end);
                n_row = live_row(g_row + nteams);
                const int64_t c = n_row < r1 ? n_row : safe_row;
                n_beg = rowptr[c];
                n_end = rowptr[c + 1];
            }
        }
    };
    auto gather = [&](Slot &sl) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int32_t jr = sl.ok[u] ? sl.j[u] : (int32_t)safe_row;
            load_vec<T, EPL>(Xq + (int64_t)jr * ldx, sl.x[u]);
        }
        sl.dd = diag ? diag[sl.row] : T(0);
        load_vec<T, EPL>(Xq + sl.row * ldx, sl.dx);
    };
    T acc[EPL];
#pragma unroll
    for (int c = 0; c < EPL; ++c) acc[c] = T(0);
    auto accumulate = [&](Slot &sl) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const T w = sl.ok[u] ? sl.v[u] : T(0);
#pragma unroll
            for (int c = 0; c < EPL; ++c) acc[c] += w * sl.x[u][c];
        }
        if (sl.last) {
#pragma unroll
            for (int off = LPN; off < TEAM; off <<= 1) {
#pragma unroll
                for (int c = 0; c < EPL; ++c) acc[c] += __shfl_xor(acc[c], off, TEAM);
            }
            if (g == 0) {
                T o[EPL];
#pragma unroll
                for (int c = 0; c < EPL; ++c) o[c] = acc[c] + sl.dd * sl.dx[c];
                store_vec<T, EPL>(S + sl.row * lds + q * EPL, o);
            }
#pragma unroll
            for (int c = 0; c < EPL; ++c) acc[c] = T(0);
        }
    };
    emit(s0);
    emit(s1);
    gather(s0);
    emit(s2);
    gather(s1);
    for (;;) {
        emit(s3);
        gather(s2);
        accumulate(s0);
        if (!s1.valid) break;
        emit(s0);
        gather(s3);
        accumulate(s1);
        if (!s2.valid) break;
        emit(s1);
        gather(s0);
        accumulate(s2);
        if (!s3.valid) break;
        emit(s2);
        gather(s1);
        accumulate(s3);
        if (!s0.valid) break;
    }
}

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

int kindex(int k) { return k <= 1 ? 0 : k <= 2 ? 1 : k <= 4 ? 2 : k <= 8 ? 3 : 4; }

template <typename T, int K>
constexpr int lanes_per_coupling() {
    return (K >= Vec16<T>::n) ? K / Vec16<T>::n : 1;
}

template <typename T, int K, int TEAM, int UNR, bool MASK>
void launch_sigma_u(const Ctx &c, const SigmaCfg &cfg, const SigmaMask &mk, const T *val, const T *diag,
                    const T *X, int ldx, T *S, int lds, hipStream_t s, unsigned long long *ctr) {
    static int cus = 0;
    if (!cus) {
        cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
    }
    // workgroups resident per CU (4 waves each), capped by the number of row teams
    int64_t nblk = (int64_t)cus * std::max(1, cfg.occ);
    const int64_t max_blk = (c.ndet + SIGMA_BLOCK / TEAM - 1) / (SIGMA_BLOCK / TEAM);
    nblk = std::min(nblk, std::max<int64_t>(max_blk, 1));
    nblk = (nblk + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    XcdRows ranges;
    for (int x = 0; x <= NUM_XCD; ++x) ranges.b[x] = c.xcd_rows[x];
    const int xmap = env_int("HINQS_SIGMA_XCDMAP", 1);
    if (cfg.pipe)
        hipLaunchKernelGGL((k_sigma_xr<T, K, TEAM, UNR, MASK>), dim3((unsigned)nblk), dim3(SIGMA_BLOCK), 0, s,
                           ranges, mk, xmap, c.rowptr.p, c.col.p, val, diag, X, ldx, S, lds);
    else
        hipLaunchKernelGGL((k_sigma<T, K, TEAM, UNR, MASK>), dim3((unsigned)nblk), dim3(SIGMA_BLOCK), 0, s,
                           ranges, mk, xmap, c.rowptr.p, c.col.p, val, diag, X, ldx, S, lds,
                           MASK ? (unsigned long long *)nullptr : (ctr ? ctr : c.sigma_ctr.p),
                           std::max(1, cfg.run));
    HQ_LAUNCH_CHECK();
}

template <typename T, int K, int TEAM, bool MASK>
void launch_sigma(const Ctx &c, const SigmaCfg &cfg, const SigmaMask &mk, const T *val, const T *diag,
                  const T *X, int ldx, T *S, int lds, hipStream_t s, unsigned long long *ctr) {
    if (cfg.unr <= 2) launch_sigma_u<T, K, TEAM, 2, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr);
    else if (cfg.unr <= 4) launch_sigma_u<T, K, TEAM, 4, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr);
    else launch_sigma_u<T, K, TEAM, 8, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr);
}

template <typename T, int K, bool MASK>
void dispatch_team(const Ctx &c, const SigmaCfg &cfg, const SigmaMask &mk, const T *val, const T *diag,
                   const T *X, int ldx, T *S, int lds, hipStream_t s, unsigned long long *ctr) {
    constexpr int LPN = lanes_per_coupling<T, K>();
    const int team = std::max(cfg.team, LPN);
#define HQ_TEAM(n) launch_sigma<T, K, n, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr)
    switch (team) {
        case 1: if constexpr (LPN <= 1) { HQ_TEAM(1); break; } [[fallthrough]];
        case 2: if constexpr (LPN <= 2) { HQ_TEAM(2); break; } [[fallthrough]];
        case 4: if constexpr (LPN <= 4) { HQ_TEAM(4); break; } [[fallthrough]];
        case 8: if constexpr (LPN <= 8) { HQ_TEAM(8); break; } [[fallthrough]];
        case 16: HQ_TEAM(16); break;
        case 32: HQ_TEAM(32); break;
        default: HQ_TEAM(64); break;
    }
#undef HQ_TEAM
}

template <typename T, bool MASK = false>
void dispatch_k(const Ctx &c, int k, const SigmaCfg &cfg, const T *val, const T *diag, const T *X, int ldx,
                T *S, int lds, hipStream_t s, const SigmaMask &mk = SigmaMask{},
                unsigned long long *ctr = nullptr) {
    switch (k) {
        case 1: dispatch_team<T, 1, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr); break;
        case 2: dispatch_team<T, 2, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr); break;
        case 4: dispatch_team<T, 4, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr); break;
        case 8: dispatch_team<T, 8, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr); break;
        case 16: dispatch_team<T, 16, MASK>(c, cfg, mk, val, diag, X, ldx, S, lds, s, ctr); break;
        default: throw Error(HINQS_E_UNSUPPORTED, "sigma block size must be 1, 2, 4, 8 or 16");
    }
}


}  // namespace

// Default shape before tuning: team sized to about four unrolled steps per mean row.
SigmaCfg default_cfg(const Ctx &c, int k, int precision) {
    const int vw = precision == HINQS_FP64 ? 2 : 4;
    const int lpn = k >= vw ? k / vw : 1;
    const double avg = c.ndet > 0 ? (double)c.nnz / (double)c.ndet : 0.0;
    const double want = avg / 8.0 * lpn;
    SigmaCfg g;
    g.team = want <= 8 ? 8 : want <= 16 ? 16 : want <= 32 ? 32 : 64;
    g.unr = 2;
    g.occ = 4;
    return g;
}

SigmaCfg sigma_config(const Ctx &c, int k, int precision) {
    SigmaCfg g = c.sigma_cfg[precision == HINQS_FP64 ? 0 : 1][kindex(k)];
    if (g.team == 0) g = default_cfg(c, k, precision);
    // explicit overrides for experiments
    g.team = env_int("HINQS_SIGMA_TEAM", g.team);
    g.unr = env_int("HINQS_SIGMA_UNR", g.unr);
    g.occ = env_int("HINQS_SIGMA_OCC", g.occ);
    g.pipe = env_int("HINQS_SIGMA_PIPE", g.pipe);
    g.run = env_int("HINQS_SIGMA_RUN", g.run);
    return g;
}

// X, S in sorted order; k in {1,2,4,8,16}; leading dimensions keep 16-byte
// alignment of every row (ldx, lds multiples of 16 / sizeof(T) when k >= that).
void sigma_sorted(Ctx &c, int k, const void *X, int ldx, void *S, int lds, int precision,
                  hipStream_t s, unsigned long long *ctr) {
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
    const SigmaCfg cfg = sigma_config(c, k, precision);
    if (precision == HINQS_FP64)
        dispatch_k<double>(c, k, cfg, c.val.p, c.diag.p, (const double *)X, ldx, (double *)S, lds, s,
                           SigmaMask{}, ctr);
    else if (precision == HINQS_FP32)
        dispatch_k<float>(c, k, cfg, c.val32.p, c.diag32.p, (const float *)X, ldx, (float *)S, lds, s,
                          SigmaMask{}, ctr);
    else
        throw Error(HINQS_E_INVALID_ARG, "precision must be HINQS_FP64 or HINQS_FP32");
}

void sigma_offdiag_fp32(const Ctx &c, int k, const float *X, float *S, hipStream_t s) {
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
    const SigmaCfg cfg = sigma_config(c, k, HINQS_FP32);
    dispatch_k<float>(c, k, cfg, c.val32.p, (const float *)nullptr, X, k, S, k, s);
}

void sigma_masked_fp64(const Ctx &c, int k, const double *X, double *S, const SigmaMask &mk, hipStream_t s) {
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
    const SigmaCfg cfg = sigma_config(c, k, HINQS_FP64);
    dispatch_k<double, true>(c, k, cfg, c.val.p, c.diag.p, X, k, S, k, s, mk);
}

void sigma_launch(const Ctx &c, int k, int precision, const SigmaCfg &cfg, const void *X, int ldx, void *S,
                  int lds, hipStream_t s) {
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
    if (precision == HINQS_FP64)
        dispatch_k<double>(c, k, cfg, c.val.p, c.diag.p, (const double *)X, ldx, (double *)S, lds, s);
    else if (precision == HINQS_FP32)
        dispatch_k<float>(c, k, cfg, c.val32.p, c.diag32.p, (const float *)X, ldx, (float *)S, lds, s);
    else
        throw Error(HINQS_E_INVALID_ARG, "precision must be HINQS_FP64 or HINQS_FP32");
}

}  // namespace hinqs
