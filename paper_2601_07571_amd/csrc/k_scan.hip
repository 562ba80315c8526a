// k_scan.hip -- exact integer prefix sums (reduce, scan of block totals, scan
// with offsets).  Integer addition is associative, so the result does not depend
// on the blocking.  Used for the triangle-weight scan (uint64, inclusive) and for
// the spatial-bucket offsets of the sample sort (uint32, exclusive).
#include <hip/hip_runtime.h>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // elements per block

template <typename T>
__device__ __forceinline__ T wave_inclusive(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive prefix over the block's threads; returns the block total in *total.
template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T* total)
{
    __shared__ T wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const T inc = wave_inclusive(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_block_totals(const T* __restrict__ in, int64_t n, T* __restrict__ totals)
{
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) s += in[base + i];
    T tot;
    (void)block_exclusive(s, &tot);
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// One block scans the block totals (exclusive) with a running carry.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_totals(T* __restrict__ totals, int64_t nb)
{
    T carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        const int64_t i = b0 + threadIdx.x;
        const T v = i < nb ? totals[i] : T(0);
        T tot;
        const T ex = block_exclusive(v, &tot);
        if (i < nb) totals[i] = carry + ex;
        carry += tot;
    }
}

template <typename T, bool Inclusive>
__global__ void __launch_bounds__(kThreads) k_block_scan(const T* __restrict__ in, T* __restrict__ out, int64_t n,
                                                         const T* __restrict__ offsets)
{
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < n ? in[base + i] : T(0);
        s += v[i];
    }
    T tot;
    T run = block_exclusive(s, &tot) + offsets[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (Inclusive) run += v[i];
        if (base + i < n) out[base + i] = run;
        if (!Inclusive) run += v[i];
    }
}

template <typename T, bool Inclusive>
void scan(const T* in, T* out, int64_t n, void* tmp, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t nb = (n + kTile - 1) / kTile;
    T* totals = static_cast<T*>(tmp);
    k_block_totals<T><<<(unsigned)nb, kThreads, 0, s>>>(in, n, totals);
    k_scan_totals<T><<<1, kThreads, 0, s>>>(totals, nb);
    k_block_scan<T, Inclusive><<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, totals);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n)
{
    const int64_t nb = (n + kTile - 1) / kTile;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(unsigned long long);
}

void launch_inclusive_scan_u64(const unsigned long long* in, unsigned long long* out, int64_t n, void* tmp,
                               hipStream_t s)
{
    scan<unsigned long long, true>(in, out, n, tmp, s);
}

void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t s)
{
    scan<uint32_t, false>(in, out, n, tmp, s);
}

}  // namespace gm
