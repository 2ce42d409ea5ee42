// Device prefix sums and a stable LSD radix sort for 64-bit keys.
//
// The radix sort orders determinant keys for the sorted determinant store:
// 8-bit digits, one histogram pass and one scatter pass per digit.  Inside a
// 4096-item tile each wave owns a contiguous 1024-item chunk; ranks among
// equal digits come from eight wave ballots (one per digit bit), so the sort
// is stable without any LDS sorting network.
#include "common.hpp"

namespace hinqs {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Exclusive scan of one value per thread across the block; returns the block total.
template <typename T>
__device__ T block_exclusive_scan(T v, T *lds_wave, T &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    T incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) lds_wave[wave] = incl;
    __syncthreads();
    T wave_off = 0, tot = 0;
    for (int w = 0; w < nwaves; ++w) {
        T x = lds_wave[w];
        if (w < wave) wave_off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return wave_off + incl - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums(const T *in, int64_t n, T *sums) {
    __shared__ T lds[SCAN_BLOCK / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
        if (base + j < n) s += in[base + j];
    T total;
    (void)block_exclusive_scan<T>(s, lds, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans `n` values in place-safe fashion (in may equal out), exclusive.
template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_single(const T *in, T *out, int64_t n,
                                                            T *total_out) {
    __shared__ T lds[SCAN_BLOCK / 64];
    T carry = 0;
    for (int64_t tile = 0; tile < n; tile += SCAN_TILE) {
        int64_t base = tile + (int64_t)threadIdx.x * SCAN_ITEMS;
        T v[SCAN_ITEMS];
        T s = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            v[j] = (base + j < n) ? in[base + j] : T(0);
            s += v[j];
        }
        T total;
        T ex = block_exclusive_scan<T>(s, lds, total);
        T run = carry + ex;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (base + j < n) out[base + j] = run;
            run += v[j];
        }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan(const T *in, T *out, int64_t n,
                                                          const T *offsets) {
    __shared__ T lds[SCAN_BLOCK / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        v[j] = (base + j < n) ? in[base + j] : T(0);
        s += v[j];
    }
    T total;
    T run = offsets[blockIdx.x] + block_exclusive_scan<T>(s, lds, total);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

template <typename T>
void exclusive_scan(hipStream_t s, const T *in, T *out, int64_t n, DBuf<char> &tmp) {
    if (n <= 0) return;
    int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 1) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, n,
                           (T *)nullptr);
        HQ_LAUNCH_CHECK();
        return;
    }
    tmp.ensure(sizeof(T) * (size_t)ntiles * 2 + 64);
    T *sums = (T *)tmp.p;
    T *offs = sums + ntiles;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, offs, ntiles,
                       (T *)nullptr);
    HQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, s, in, out, n,
                       offs);
    HQ_LAUNCH_CHECK();
}

// ------------------------------------------------------------- radix sort
constexpr int RS_WAVES = 4;
constexpr int RS_BLOCK = 64 * RS_WAVES;
constexpr int RS_STEPS = 16;                         // 64-item steps per wave
constexpr int RS_CHUNK = 64 * RS_STEPS;              // items per wave
constexpr int RS_TILE = RS_CHUNK * RS_WAVES;         // items per block

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                      int ntiles, int32_t *counts) {
    __shared__ int32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = threadIdx.x; j < RS_TILE; j += RS_BLOCK) {
        int64_t idx = base + j;
        if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t *keys, const int32_t *vals,
                                                         int64_t n, int shift, int ntiles,
                                                         const int32_t *offsets, uint64_t *okeys,
                                                         int32_t *ovals) {
    __shared__ int32_t whist[RS_WAVES][256];
    __shared__ int32_t woff[RS_WAVES][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < RS_WAVES * 256; j += RS_BLOCK) (&whist[0][0])[j] = 0;
    __syncthreads();
    const int64_t cbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)wave * RS_CHUNK;
    for (int st = 0; st < RS_STEPS; ++st) {
        int64_t idx = cbase + st * 64 + lane;
        if (idx < n) atomicAdd(&whist[wave][(keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    {
        int d = threadIdx.x;  // RS_BLOCK == 256 digits
        int32_t run = offsets[(int64_t)d * ntiles + blockIdx.x];
        for (int w = 0; w < RS_WAVES; ++w) {
            woff[w][d] = run;
            run += whist[w][d];
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int st = 0; st < RS_STEPS; ++st) {
        int64_t idx = cbase + st * 64 + lane;
        bool valid = idx < n;
        uint64_t key = valid ? keys[idx] : 0ull;
        int32_t val = valid ? vals[idx] : 0;
        uint32_t digit = (uint32_t)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (digit >> b) & 1u;
            uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        int32_t start = 0;
        if (valid) start = woff[wave][digit];
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            int32_t pos = start + __popcll(peers & lt);
            okeys[pos] = key;
            ovals[pos] = val;
            if ((peers & lt) == 0ull) woff[wave][digit] = start + __popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

void exclusive_scan_i64(hipStream_t s, const int64_t *in, int64_t *out, int64_t n, DBuf<char> &tmp) {
    exclusive_scan<int64_t>(s, in, out, n, tmp);
}
void exclusive_scan_i32(hipStream_t s, const int32_t *in, int32_t *out, int64_t n, DBuf<char> &tmp) {
    exclusive_scan<int32_t>(s, in, out, n, tmp);
}

void radix_sort_u64(hipStream_t s, uint64_t *keys, int32_t *vals, int64_t n, int nbits,
                    DBuf<char> &tmp) {
    DBuf<char> own;
    radix_sort_u64(s, keys, vals, n, nbits, tmp, own);
    HQ_CHECK(hipStreamSynchronize(s));  // `own` is released on return
}

void radix_sort_u64(hipStream_t s, uint64_t *keys, int32_t *vals, int64_t n, int nbits, DBuf<char> &tmp,
                    DBuf<char> &own) {
    if (n <= 1) return;
    if (n >= (int64_t)1 << 31) throw Error(HINQS_E_UNSUPPORTED, "radix sort limited to 2^31 items");
    const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    const int64_t ncount = 256LL * ntiles;
    // layout of tmp: counts | offsets | key buffer | val buffer | scan workspace
    size_t off_counts = 0;
    size_t off_offsets = off_counts + sizeof(int32_t) * ncount;
    size_t off_keys = (off_offsets + sizeof(int32_t) * ncount + 255) & ~(size_t)255;
    size_t off_vals = off_keys + sizeof(uint64_t) * n;
    size_t total = off_vals + sizeof(int32_t) * n + 256;
    own.ensure(total);
    int32_t *counts = (int32_t *)(own.p + off_counts);
    int32_t *offsets = (int32_t *)(own.p + off_offsets);
    uint64_t *k2 = (uint64_t *)(own.p + off_keys);
    int32_t *v2 = (int32_t *)(own.p + off_vals);
    uint64_t *kin = keys, *kout = k2;
    int32_t *vin = vals, *vout = v2;
    int passes = (nbits + 7) / 8;
    if (passes < 1) passes = 1;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(RS_BLOCK), 0, s, kin, n, shift, ntiles,
                           counts);
        HQ_LAUNCH_CHECK();
        exclusive_scan_i32(s, counts, offsets, ncount, tmp);
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(RS_BLOCK), 0, s, kin, vin, n, shift,
                           ntiles, offsets, kout, vout);
        HQ_LAUNCH_CHECK();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (kin != keys) {
        HQ_CHECK(hipMemcpyAsync(keys, kin, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        HQ_CHECK(hipMemcpyAsync(vals, vin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace hinqs
