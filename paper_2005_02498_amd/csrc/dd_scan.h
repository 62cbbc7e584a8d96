// Single-workgroup exclusive scan shared by the node lists and the near-pair
// lists.
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

}  // namespace dd
