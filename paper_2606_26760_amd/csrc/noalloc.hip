// Sigma product S = H_B X without any device allocation (the repeated product
// of the Davidson iteration, Sec. 2.2, Step 3), for callers that cannot
// allocate: the kernel's row counters and the sorted-order staging of X and S
// live in one static device array per GPU instead of context buffers.  The
// staging kernels (caller order and k padded to K in one pass each way) serve
// hinqs_sigma too, with the context's buffers.
//
// Layout of the array: [0, 4096) row counters (SIGMA_CTR_WORDS words, cleared
// by a fill kernel on every call; no memset, so the call can be captured in a
// graph); [4096, 4096 + B) staged X; [4096 + B, 4096 + 2B) staged S, where
// B = ndet * K * element size rounded up to 256 bytes.
#include <mutex>

#include "common.hpp"

namespace hinqs {

constexpr size_t NOALLOC_BYTES = HINQS_NOALLOC_SCRATCH_BYTES;
constexpr size_t NOALLOC_CTR_BYTES = 4096;
static_assert(SIGMA_CTR_WORDS * sizeof(unsigned long long) <= NOALLOC_CTR_BYTES, "counter region");

// In host code `scratch` only names the host-side shadow of the array; its
// device address comes from hipGetSymbolAddress (noalloc_setup) and only that
// address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_ptr[MAX_DEVICES] = {};

unsigned char *device_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= MAX_DEVICES || !g_ptr[device])
        throw Error(HINQS_E_NOT_READY, "the no-allocation scratch of this device is not set up");
    return g_ptr[device];
}

__global__ void k_clear_words(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// xs (sorted order, K wide) from X (k wide; caller order through perm, or
// sorted when perm is null); columns k..K-1 are zero.
template <typename T>
__global__ void k_stage_in(const T *__restrict__ X, int k, const int32_t *__restrict__ perm, int64_t D, int K,
                           T *__restrict__ xs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= D * K) return;
    const int64_t i = t / K;
    const int col = (int)(t - i * K);
    const int64_t r = perm ? (int64_t)perm[i] : i;
    xs[t] = col < k ? X[r * k + col] : T(0);
}

// S (k wide, caller order through perm or sorted) from ss (sorted, K wide).
template <typename T>
__global__ void k_stage_out(const T *__restrict__ ss, int K, const int32_t *__restrict__ perm, int64_t D, int k,
                            T *__restrict__ S) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= D * k) return;
    const int64_t i = t / k;
    const int col = (int)(t - i * k);
    const int64_t r = perm ? (int64_t)perm[i] : i;
    S[r * k + col] = ss[i * K + col];
}

template <typename T>
void staged(Ctx &c, int k, int K, const void *X, void *S, bool sorted, T *xs, T *ss, unsigned long long *ctr) {
    hipStream_t s = c.stream;
    const int64_t D = c.ndet;
    const int32_t *perm = sorted ? nullptr : c.perm.p;
    hipLaunchKernelGGL(k_stage_in<T>, dim3(grid_for(D * K, 256)), dim3(256), 0, s, (const T *)X, k, perm, D, K,
                       xs);
    HQ_LAUNCH_CHECK();
    sigma_sorted(c, K, xs, K, ss, K, sizeof(T) == 8 ? HINQS_FP64 : HINQS_FP32, s, ctr);
    hipLaunchKernelGGL(k_stage_out<T>, dim3(grid_for(D * k, 256)), dim3(256), 0, s, ss, K, perm, D, k, (T *)S);
    HQ_LAUNCH_CHECK();
}

}  // namespace

void sigma_staged(Ctx &c, int k, const void *X, void *S, int precision, bool sorted, void *xs, void *ss,
                  unsigned long long *ctr) {
    const int K = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
    if (precision == HINQS_FP64) staged<double>(c, k, K, X, S, sorted, (double *)xs, (double *)ss, ctr);
    else staged<float>(c, k, K, X, S, sorted, (float *)xs, (float *)ss, ctr);
}

void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= MAX_DEVICES) throw Error(HINQS_E_UNSUPPORTED, "device index above 63");
    if (g_ptr[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        throw Error(HINQS_E_HIP, std::string("hipGetSymbolAddress of the no-allocation scratch failed: ") +
                                     hipGetErrorString(e));
    g_ptr[device] = (unsigned char *)p;
}

void sigma_noalloc(Ctx &c, int k, const void *X, void *S, int precision, bool sorted) {
    struct Forbid {  // any device allocation below is an internal error
        bool prev = g_no_alloc;
        Forbid() { g_no_alloc = true; }
        ~Forbid() { g_no_alloc = prev; }
    } forbid;
    unsigned char *base = device_scratch(c.device);
    const size_t esz = precision == HINQS_FP64 ? 8 : 4;
    const int K = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
    const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)S % 16 == 0);
    const bool direct = sorted && K == k && aligned;
    const size_t blk = ((size_t)c.ndet * K * esz + 255) / 256 * 256;
    const size_t need = NOALLOC_CTR_BYTES + (direct ? 0 : 2 * blk);
    if (need > NOALLOC_BYTES)
        throw Error(HINQS_E_UNSUPPORTED, "the no-allocation sigma needs " + std::to_string(need) +
                                             " bytes of scratch for ndet = " + std::to_string(c.ndet) +
                                             " and k = " + std::to_string(k) + "; its limit is " +
                                             std::to_string(NOALLOC_BYTES) +
                                             " (sorted-order, 16-byte aligned X and S with k in {1,2,4,8,16} "
                                             "need no staging)");
    hipStream_t s = c.stream;
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(SIGMA_CTR_WORDS), 0, s, (unsigned long long *)base,
                       SIGMA_CTR_WORDS);
    HQ_LAUNCH_CHECK();
    if (direct)
        sigma_sorted(c, K, X, K, S, K, precision, s, (unsigned long long *)base);
    else
        sigma_staged(c, k, X, S, precision, sorted, base + NOALLOC_CTR_BYTES, base + NOALLOC_CTR_BYTES + blk,
                     (unsigned long long *)base);
}

}  // namespace hinqs
