// Shared definitions of the gfx950 selected-CI library: error handling, device
// buffers, the context, and the bit-string rules (excitation degree, holes,
// particles and fermionic signs) used by every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <utility>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hinqs.h"

namespace hinqs {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HQ_CHECK(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::hinqs::Error(e_ == hipErrorOutOfMemory ? HINQS_E_OOM : HINQS_E_HIP,   \
                                 std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define HQ_LAUNCH_CHECK() HQ_CHECK(hipGetLastError())

// ---------------------------------------------------------- device buffer
// Where device memory comes from: the allocator callbacks given to
// hinqs_create (a framework's caching allocator), or hipMalloc when none were
// given.  Each entry point installs its context's allocator for the duration
// of the call; a buffer remembers the allocator it came from and returns its
// memory there.
struct Allocator {
    hinqs_alloc_fn alloc = nullptr;
    hinqs_free_fn free = nullptr;
    void *user = nullptr;
    hipStream_t stream = nullptr;
};
inline thread_local const Allocator *g_alloc = nullptr;

// While set, any device allocation on this thread is an internal error (the
// no-allocation entry point runs under it).
inline thread_local bool g_no_alloc = false;

// While set, buffers (re)allocated on this thread get twice the requested
// capacity, so a context rebuilt for a sequence of growing problems (the
// instances of a batch) reallocates rarely.
inline thread_local bool g_dbuf_grow = false;

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    Allocator src;   // allocator p came from (alloc == nullptr: hipMalloc)
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) {
            if (src.free) src.free(p, src.stream, src.user);
            else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        src = Allocator{};
    }
    // (Re)allocate to hold at least `count` elements; contents undefined.
    void ensure(size_t count) {
        if (count <= n && p) return;
        if (g_no_alloc) throw Error(HINQS_E_HIP, "internal: device allocation in the no-allocation path");
        release();
        if (g_dbuf_grow) count *= 2;
        size_t bytes = (count ? count : 1) * sizeof(T);
        if (g_alloc && g_alloc->alloc) {
            p = (T *)g_alloc->alloc(bytes, (void *)g_alloc->stream, g_alloc->user);
            if (!p) throw Error(HINQS_E_OOM, "the context's allocator returned no memory for " +
                                                 std::to_string(bytes) + " bytes");
            src = *g_alloc;
        } else {
            hipError_t e = hipMalloc((void **)&p, bytes);
            if (e != hipSuccess) {
                p = nullptr;
                throw Error(HINQS_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                             hipGetErrorString(e));
            }
        }
        n = count ? count : 1;
    }
    size_t bytes() const { return n * sizeof(T); }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(src, o.src);
    }
    operator T *() const { return p; }
};

// Waits for the stream by polling it: the solver's loop waits for a few small
// results each iteration, and a blocking wait adds the wake-up latency of the
// sleeping host thread to every one of those round trips.
inline void wait_stream(hipStream_t s) {
    hipError_t e;
    while ((e = hipStreamQuery(s)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) throw Error(HINQS_E_HIP, std::string("stream wait: ") + hipGetErrorString(e));
}

// Installs an allocator for the current thread until the end of the scope.
struct AllocScope {
    const Allocator *prev;
    explicit AllocScope(const Allocator *a) : prev(g_alloc) { g_alloc = a; }
    ~AllocScope() { g_alloc = prev; }
};

// --------------------------------------------------------- bit-string rules
// Strings are uint32 (norb <= 32); bit p = spatial orbital p.

__host__ __device__ inline int popc32(uint32_t x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __popc(x);
#else
    return __builtin_popcount(x);
#endif
}

__host__ __device__ inline int lowbit(uint32_t x) {  // index of lowest set bit, x != 0
#ifdef __HIP_DEVICE_COMPILE__
    return __ffs(x) - 1;
#else
    return __builtin_ctz(x);
#endif
}

// Candidates tested per step of a group scan before the hits are emitted.
constexpr int SCAN_W = 16;

// Davidson: a new direction is kept when the eigenvalue of its unit-scaled
// block Gram exceeds this (more than a tenth of its norm lies outside the
// span of the basis and of the other new directions), so the orthonormalizing
// transform amplifies rounding at most tenfold and needs no second round.
constexpr double ORTH_DROP = 1e-2;

__host__ __device__ inline int highbit(uint32_t x) {  // index of highest set bit, x != 0
#ifdef __HIP_DEVICE_COMPILE__
    return 31 - __clz(x);
#else
    return 31 - __builtin_clz(x);
#endif
}

// Bits strictly between orbitals a and b (a != b, both < 32).
__host__ __device__ inline uint32_t between(int a, int b) {
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return ((hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u))) & ~((2u << lo) - 1u);
}

// Parity (0 = +, 1 = -) of a+_p a_h |s>: occupied orbitals strictly between h and p.
// The same-spin string of the other spin, and every orbital outside (h, p),
// contribute an even count and drop out.
__host__ __device__ inline uint32_t single_parity(uint32_t s, int h, int p) {
    return (uint32_t)popc32(s & between(h, p)) & 1u;
}

// Parity of a+_p1 a+_p2 a_h2 a_h1 |s> with h1 < h2 (occupied in s) and p1 < p2
// (empty in s).  The string equals -(a+_p1 a_h2)(a+_p2 a_h1): the move h1 -> p2
// acts on s, the move h2 -> p1 on the intermediate string.
__host__ __device__ inline uint32_t double_parity(uint32_t s, int h1, int h2, int p1, int p2) {
    uint32_t s1 = s ^ (1u << h1) ^ (1u << p2);
    return 1u ^ single_parity(s, h1, p2) ^ single_parity(s1, h2, p1);
}

// Descriptor layout (see hinqs_connectivity).
__host__ __device__ inline uint32_t make_desc(uint32_t type, uint32_t neg, int h1, int h2, int p1,
                                              int p2) {
    return type | (neg << 3) | ((uint32_t)h1 << 4) | ((uint32_t)h2 << 9) | ((uint32_t)p1 << 14) |
           ((uint32_t)p2 << 19);
}
__host__ __device__ inline uint32_t desc_type(uint32_t d) { return d & 7u; }
__host__ __device__ inline uint32_t desc_neg(uint32_t d) { return (d >> 3) & 1u; }
__host__ __device__ inline int desc_h1(uint32_t d) { return (d >> 4) & 31; }
__host__ __device__ inline int desc_h2(uint32_t d) { return (d >> 9) & 31; }
__host__ __device__ inline int desc_p1(uint32_t d) { return (d >> 14) & 31; }
__host__ __device__ inline int desc_p2(uint32_t d) { return (d >> 19) & 31; }

// Same-spin pair (bra string si, ket string sj) differing by one or two
// electrons: class `type1` or `type2` descriptor.
__host__ __device__ inline uint32_t same_spin_desc(uint32_t si, uint32_t sj, uint32_t type1,
                                                   uint32_t type2) {
    uint32_t holes = sj & ~si, parts = si & ~sj;
    if (popc32(holes) == 1) {
        int h = lowbit(holes), p = lowbit(parts);
        return make_desc(type1, single_parity(sj, h, p), h, 0, p, 0);
    }
    int h1 = lowbit(holes), h2 = highbit(holes), p1 = lowbit(parts), p2 = highbit(parts);
    return make_desc(type2, double_parity(sj, h1, h2, p1, p2), h1, h2, p1, p2);
}

// Opposite-spin double from an alpha move (ha -> pa on alpha string aj, parity na)
// and a beta move (beta strings bi <- bj).
__host__ __device__ inline uint32_t ab_desc(int ha, int pa, uint32_t na, uint32_t bi, uint32_t bj) {
    uint32_t hb_m = bj & ~bi, pb_m = bi & ~bj;
    int hb = lowbit(hb_m), pb = lowbit(pb_m);
    return make_desc(HINQS_EXC_2AB, na ^ single_parity(bj, hb, pb), ha, hb, pa, pb);
}

// Descriptor of the pair bra (ai, bi) <- ket (aj, bj), or 0 when they differ
// by more than two electrons or not at all.
__host__ __device__ inline uint32_t pair_desc(uint32_t ai, uint32_t bi, uint32_t aj, uint32_t bj) {
    const int da = popc32(ai ^ aj), db = popc32(bi ^ bj);
    if (da + db == 0 || da + db > 4) return 0u;
    if (db == 0) return same_spin_desc(ai, aj, HINQS_EXC_1A, HINQS_EXC_2AA);
    if (da == 0) return same_spin_desc(bi, bj, HINQS_EXC_1B, HINQS_EXC_2BB);
    const int ha = lowbit(aj & ~ai), pa = lowbit(ai & ~aj);  // one alpha and one beta move
    return ab_desc(ha, pa, single_parity(aj, ha, pa), bi, bj);
}

// ------------------------------------------------- packed integral indexing
// Pair index of (p, q) with p >= q: p(p+1)/2 + q; 8-fold symmetric (pq|rs) is
// stored once per unordered pair of pair indices.
__host__ __device__ inline int pair_index(int p, int q) {
    return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
}
__host__ __device__ inline int eri_index(int p, int q, int r, int s) {
    int a = pair_index(p, q), b = pair_index(r, s);
    return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
}
inline int npair(int norb) { return norb * (norb + 1) / 2; }
inline int neri_packed(int norb) { int m = npair(norb); return m * (m + 1) / 2; }

// Words of the sigma kernel's row counters: 32 per XCD (8 XCDs).
constexpr int SIGMA_CTR_WORDS = 8 * 32;

// Launch shape of the sigma kernel: lanes per row team, couplings in flight per
// lane, resident workgroups per CU.
struct SigmaCfg {
    int team = 0, unr = 0, occ = 0;
    int pipe = 0;     // 0: one step of gathers in flight per team; 1: cross-row four-stage pipeline
    int run = 4;      // rows a team takes from its XCD's row counter at a time (pipe 0)
    double ms = 0.0;  // measured time of one launch when chosen by the tuner
};

// Row mask of the sigma kernel for batched instances (rows of instance b are
// inst_row[b] .. inst_row[b+1]); ranges holds 9 row bounds, one range per XCD.
struct SigmaMask {
    const int64_t *ranges = nullptr;
    const int32_t *row_inst = nullptr;
    const int64_t *inst_row = nullptr;
    const int32_t *done = nullptr;
};

// Column-blocked tall matrix: element (i, j) at p[(j / kb) * bs + i * kb + j % kb].
// A plain row-major array with leading dimension ld is {p, ld, 0} with j < ld.
struct Mat {
    double *p;
    int kb;
    int64_t bs;
    __host__ __device__ double *at(int64_t i, int j) const {
        return p + (int64_t)(j / kb) * bs + i * kb + (j % kb);
    }
    __host__ __device__ Mat cols(int c0) const {  // view from column c0 (c0 % kb == 0)
        return Mat{p + (int64_t)(c0 / kb) * bs, kb, bs};
    }
};

// ------------------------------------------------------------- context
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
};

struct BatchState;  // batched instances (batch.hip)

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Allocator alloc;   // device memory of every buffer below
    std::string err;

    // integrals
    int norb = 0;
    bool have_ints = false;
    double ecore = 0.0;
    std::vector<double> h_host, eri_host;   // as given (norb^2, norb^4)
    DBuf<double> d_h;                      // norb^2
    DBuf<double> d_eri;                    // packed 8-fold
    DBuf<float> d_eri32;                   // packed, FP32 copy

    // determinants (sorted: alpha-major, then beta)
    bool have_dets = false;
    int na = 0, nb = 0;
    int64_t ndet = 0;
    DBuf<uint32_t> sa, sb;     // strings in sorted order
    DBuf<int32_t> perm;        // sorted position -> caller index
    DBuf<int32_t> inv;         // caller index -> sorted position
    int32_t nua = 0, nub = 0;
    DBuf<uint32_t> ua, ub;     // distinct alpha / beta strings, ascending
    DBuf<int32_t> ga;          // alpha group offsets (nua+1) into sorted order
    DBuf<int32_t> aidx, bidx;  // per determinant: index into ua / ub
    DBuf<int32_t> gb;          // beta group offsets (nub+1) into bperm
    DBuf<int32_t> bperm;       // beta-major listing of sorted positions
    DBuf<uint32_t> bm_alpha;   // alpha string of bperm[t]
    int alink_max = 0;         // row length of the padded link table
    DBuf<int32_t> alink_ptr;   // per distinct alpha string: number of single moves to strings of B
    DBuf<int32_t> alink;       // [nua][alink_max] target index into ua
    DBuf<uint32_t> alink_info; // hole | particle << 5 | parity << 10

    // couplings (sorted order, diagonal not stored)
    int64_t nnz = 0;
    DBuf<int64_t> rowptr;
    DBuf<int32_t> col;
    DBuf<uint32_t> desc;
    DBuf<double> val;
    DBuf<float> val32;
    DBuf<double> diag;
    DBuf<float> diag32;
    bool have_elements = false;
    // row ranges with equal coupling counts, one per XCD (rows xcd_rows[x] .. xcd_rows[x+1])
    int64_t xcd_rows[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // tuned sigma launch shapes, [precision][log2 k]
    SigmaCfg sigma_cfg[2][5];
    // row counters of the sigma kernel (SIGMA_CTR_WORDS; zero between launches; set up with the context)
    DBuf<unsigned long long> sigma_ctr;

    // timings (ms)
    double ms_sort = 0, ms_connect = 0, ms_elements = 0;

    // workspace shared by calls
    DBuf<char> work;
    // temporaries of building a set (kept between builds, so rebuilding, or
    // building the instances of a batch one after another, allocates rarely)
    struct BuildScratch {
        DBuf<uint64_t> up_a, up_b, keys;
        DBuf<uint32_t> da, db, sbm;
        DBuf<int32_t> vals, flag, scan, dup, gidx;
        DBuf<unsigned long long> bad;
        DBuf<int64_t> counts;
        DBuf<double> eri_full;
        DBuf<char> sort;
    } bs;
    // temporaries of calls that stage data (caller-order sigma, RDMs and
    // gradients, top-k, expansion, PT2, product closure), kept between calls:
    // once a size has been seen, repeating the call allocates nothing and has
    // no buffer to release, so it need not wait for the stream
    struct CallScratch {
        DBuf<char> b[5];
        DBuf<unsigned long long> flags;  // small counters and error flags
        template <typename T>
        T *get(int i, size_t count) {
            b[i].ensure(count * sizeof(T));
            return (T *)b[i].p;
        }
        unsigned long long *words(int n) {
            flags.ensure(n);
            return flags.p;
        }
    } cs;
    // Davidson workspace (basis, images, staging), kept between solves
    struct DavidsonWork {
        DBuf<double> Vb, Wb, T, Wn, small, partial, nrm, argv, xfin, signbuf;
        DBuf<float> X32, S32;
        DBuf<int32_t> guess_idx;
        DBuf<int64_t> argi;
        double *pinned = nullptr;  // host staging ring (hipHostMalloc)
        double *pinned_dl = nullptr;  // host landing area of small device results
        DavidsonWork() = default;
        DavidsonWork(const DavidsonWork &) = delete;
        DavidsonWork &operator=(const DavidsonWork &) = delete;
        ~DavidsonWork() {
            if (pinned) (void)hipHostFree(pinned);
            if (pinned_dl) (void)hipHostFree(pinned_dl);
        }
    } dw;

    // independent instances solved together (hinqs_batch_*)
    std::shared_ptr<BatchState> batch;

    size_t device_bytes() const;
};

// ------------------------------------------------------ internal entry points
void build_integrals(Ctx &c, int norb, const double *h, const double *eri, double ecore);
void build_determinants(Ctx &c, int64_t ndet, const uint64_t *alpha, const uint64_t *beta, int na,
                        int nb, bool on_device);
// xcd_rows: also split the rows over the XCDs for sigma (a host read; not
// needed for a set that is only an instance of a batch being assembled).
void build_connectivity(Ctx &c, bool xcd_rows = true);
void build_elements(Ctx &c);
// Values of the entries of each row after its first skip[row] (whose values
// are already in place), and every diagonal element.
void build_elements_after(Ctx &c, const int64_t *skip);

void export_connectivity(Ctx &c, int64_t *rowptr_c, int32_t *col_c, uint32_t *desc_c);
// Row ranges with equal coupling counts, one per XCD, from c.rowptr.
void compute_xcd_rows(Ctx &c);

// Scan / sort utilities (scan.hip).  All on c.stream.
void exclusive_scan_i64(hipStream_t s, const int64_t *in, int64_t *out, int64_t n, DBuf<char> &tmp);
void exclusive_scan_i32(hipStream_t s, const int32_t *in, int32_t *out, int64_t n, DBuf<char> &tmp);
// Stable LSD radix sort of `keys` (nbits significant low bits) carrying `vals`.
void radix_sort_u64(hipStream_t s, uint64_t *keys, int32_t *vals, int64_t n, int nbits,
                    DBuf<char> &tmp);
// The same with the sort's own buffers in `own` (kept by the caller; no
// synchronization at the end).
void radix_sort_u64(hipStream_t s, uint64_t *keys, int32_t *vals, int64_t n, int nbits, DBuf<char> &tmp,
                    DBuf<char> &own);

// Sigma (sigma.hip): S = H X in sorted order with leading dimensions.
// ctr: the kernel's row counters (SIGMA_CTR_WORDS, zero on entry, left at
// zero); nullptr = the context's own.
void sigma_sorted(Ctx &c, int k, const void *X, int ldx, void *S, int lds, int precision,
                  hipStream_t s, unsigned long long *ctr = nullptr);

// No-allocation sigma (noalloc.hip).  noalloc_setup: once per device, with
// that device current (hinqs_create calls it).  sigma_noalloc: the whole
// product with counters and staging in the static array; arguments already
// validated as for hinqs_sigma.
void noalloc_setup(int device);
void sigma_noalloc(Ctx &c, int k, const void *X, void *S, int precision, bool sorted);
// S = H X for X, S in caller order (sorted = false) or sorted order, any k in
// [1, 16]: X gathered and padded to K columns into xs, the sorted product into
// ss (both ndet x K of the precision's type), S scattered back.  ctr: as for
// sigma_sorted.
void sigma_staged(Ctx &c, int k, const void *X, void *S, int precision, bool sorted, void *xs, void *ss,
                  unsigned long long *ctr);
// Time the candidate launch shapes on c's couplings, keep the fastest in c
// (and in a process-wide cache keyed by problem shape).  Returns it.
SigmaCfg autotune_sigma(Ctx &c, int k, int precision);
// Shape the next sigma launch will use for (k, precision), and the shape
// used before any tuning.
SigmaCfg sigma_config(const Ctx &c, int k, int precision);
SigmaCfg default_cfg(const Ctx &c, int k, int precision);
// S = H X in sorted order with an explicit launch shape.
void sigma_launch(const Ctx &c, int k, int precision, const SigmaCfg &cfg, const void *X, int ldx, void *S,
                  int lds, hipStream_t s);
// FP32 off-diagonal product S = (H - diag(H)) X (X, S with leading dimension k); the caller adds the
// diagonal term in FP64.
void sigma_offdiag_fp32(const Ctx &c, int k, const float *X, float *S, hipStream_t s);
// FP64 sigma over the rows that mk leaves live (X, S with leading dimension k).
void sigma_masked_fp64(const Ctx &c, int k, const double *X, double *S, const SigmaMask &mk, hipStream_t s);

// Batched instances (batch.hip)
void batch_clear(Ctx &c);
int batch_add(Ctx &c, int norb, const double *h, const double *eri, double ecore, int64_t ndet,
              const uint64_t *alpha, const uint64_t *beta, int na, int nb);
void batch_info(Ctx &c, int *ninst, int64_t *offsets, int64_t *nnz);
int batch_solve(Ctx &c, const hinqs_opts &o, double *energies, double *coeffs, int *status, int *iters,
                hinqs_batch_stats *st);

// Selection (select.hip): c in caller order unless `sorted`.
int64_t excitations_per_det(int norb, int na, int nb);
void top_k(Ctx &c, int64_t n, const double *v, int64_t k, bool largest, int32_t *idx);
int64_t expand(Ctx &c, const double *coeffs, bool sorted, int64_t ntop, int64_t capacity, uint64_t *out_a,
               uint64_t *out_b, int32_t *top);
void pt2(Ctx &c, const double *coeffs, bool sorted, double e0, int64_t ncand, const uint64_t *ca,
         const uint64_t *cb, double *numer, double *hxx, double *score);
// PT2 quantities (Eq. 3) of every member of B: numer = (H_B c)_x (one sigma
// product, the diagonal included), hxx = H_xx, score = numer^2 / |e0 - hxx|;
// outputs ndet each, caller order unless sorted.
void pt2_members(Ctx &c, const double *coeffs, bool sorted, double e0, double *numer, double *hxx,
                 double *score);

// Determinants of (distinct alpha strings) x (distinct beta strings) that are
// not in the set, ascending; the first cap are written; returns how many.
int64_t product_closure(Ctx &c, int64_t cap, uint64_t *out_a, uint64_t *out_b);

// Teacher weights (weights.hip): c in caller order unless `sorted`.
void teacher_weights(Ctx &c, const double *coeffs, bool sorted, double *w, double *p_alpha, double *p_beta);
void distinct_strings(Ctx &c, uint64_t *alpha, uint64_t *beta);

// Incremental basis update (update.hip): evict (caller indices, or sorted
// positions when `sorted`), append (device strings), carry c_old over.
void update_determinants(Ctx &c, int64_t n_evict, const int32_t *evict, int64_t n_add, const uint64_t *add_a,
                         const uint64_t *add_b, const double *c_old, double *c_new, bool sorted, double *ms_out);

// The basis-growth rules (update.hip); returns the new ndet.
int64_t grow_basis(Ctx &c, int mode, int64_t ncand, const uint64_t *ca, const uint64_t *cb, const double *cscore,
                   int64_t k, const double *bscore, int64_t bmax, const double *c_old, double *c_new,
                   double *score_new, double *ms_out);
// Strings of the current set in caller order (device uint64; either may be null).
void caller_strings(Ctx &c, uint64_t *alpha, uint64_t *beta);

// Davidson (davidson.hip)
int davidson(Ctx &c, const hinqs_opts &o, const double *guess, double *energy, double *coeffs,
             hinqs_stats *st);

// Tall-skinny Gram product G = A^T B (FP64 MFMA), A: nrows x ma, B: nrows x nb.
void gram_product(Ctx &c, int64_t nrows, const double *A, int lda, int ma, const double *B, int ldb,
                  int nb, double *G);

// RDMs (rdm.hip): c in sorted order.
void rdm12_sorted(Ctx &c, const double *cs, double *rdm1, double *rdm2);
void integral_grad_sorted(Ctx &c, const double *cs, double scale, double *gh, double *geri);

// permutation helpers (dets.hip)
void gather_rows(hipStream_t s, const void *src, void *dst, const int32_t *idx, int64_t n,
                 int rowbytes);   // dst[r] = src[idx[r]]
void scatter_rows(hipStream_t s, const void *src, void *dst, const int32_t *idx, int64_t n,
                  int rowbytes);  // dst[idx[r]] = src[r]

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace hinqs
