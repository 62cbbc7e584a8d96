// Exclusive scans shared by the node lists, the sessile-segment lists and
// the near-pair lists: one workgroup for short arrays, three launches over
// blocks of SCAN_BLOCK counts for long ones.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dd {

// Exclusive scan of cnt[0..n) into ptr[0..n] by one workgroup of 1024
// threads, 4096 counts per round: each thread takes 4 consecutive counts,
// wavefront prefix sums by shuffles, the 16 wavefront totals through LDS, and
// a running carry from round to round.
template <class T>
__global__ __launch_bounds__(1024) void k_scan(const T *cnt, int64_t n, T *ptr)
{
    __shared__ T wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    T carry = 0;
    for (int64_t base = 0; base < n; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)tid;
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (i0 + k < n) ? cnt[i0 + k] : 0;
        const T t = v[0] + v[1] + v[2] + v[3];
        T s = t;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T u = __shfl_up(s, off, 64);
            if (lane >= off) s += u;
        }
        if (lane == 63) wsum[w] = s;
        __syncthreads();
        T before = carry, total = carry;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            before += k < w ? wsum[k] : 0;
            total += wsum[k];
        }
        T run = before + s - t;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < n) ptr[i0 + k] = run;
            run += v[k];
        }
        carry = total;
        __syncthreads();
    }
    if (tid == 0) ptr[n] = carry;
}

constexpr int64_t SCAN_BLOCK = 4096;   // counts per workgroup round

// Entries of scratch launch_scan needs for n counts.
inline int64_t scan_scratch_len(int64_t n) { return 2 * ((n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1); }

// Workgroup b: the exclusive scan of counts b SCAN_BLOCK .. + SCAN_BLOCK - 1
// within the block into ptr, and the block's total into bsum[b].
template <class T>
__global__ __launch_bounds__(1024) void k_scan_blocks(const T *cnt, int64_t n, T *ptr, T *bsum)
{
    __shared__ T wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t i0 = blockIdx.x * SCAN_BLOCK + 4 * (int64_t)tid;
    T v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i0 + k < n) ? cnt[i0 + k] : 0;
    const T t = v[0] + v[1] + v[2] + v[3];
    T s = t;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T u = __shfl_up(s, off, 64);
        if (lane >= off) s += u;
    }
    if (lane == 63) wsum[w] = s;
    __syncthreads();
    T before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        before += k < w ? wsum[k] : 0;
        total += wsum[k];
    }
    T run = before + s - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) ptr[i0 + k] = run;
        run += v[k];
    }
    if (tid == 0) bsum[blockIdx.x] = total;
}

// ptr[i] += boff[i / SCAN_BLOCK] for i < n; ptr[n] = the grand total boff[nb].
template <class T>
__global__ __launch_bounds__(256) void k_scan_add(T *ptr, int64_t n, const T *boff)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) ptr[i] += boff[i / SCAN_BLOCK];
    if (i == 0) ptr[n] = boff[(n + SCAN_BLOCK - 1) / SCAN_BLOCK];
}

// Exclusive scan of cnt[0..n) into ptr[0..n] (ptr[n] = the total) on st.
// With scratch (scan_scratch_len(n) entries) and more than 8 blocks of
// counts: block scans, a scan of the block totals and the offsets added,
// each launch spread over the chip; otherwise one workgroup.  The same
// integer sums either way.
template <class T>
void launch_scan(const T *cnt, int64_t n, T *ptr, T *scratch, hipStream_t st)
{
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (!scratch || nb <= 8) {
        hipLaunchKernelGGL(k_scan<T>, dim3(1), dim3(1024), 0, st, cnt, n, ptr);
        return;
    }
    T *bsum = scratch, *boff = scratch + nb;
    hipLaunchKernelGGL(k_scan_blocks<T>, dim3((unsigned)nb), dim3(1024), 0, st, cnt, n, ptr, bsum);
    hipLaunchKernelGGL(k_scan<T>, dim3(1), dim3(1024), 0, st, (const T *)bsum, nb, boff);
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ptr, n,
                       (const T *)boff);
}

}  // namespace dd
