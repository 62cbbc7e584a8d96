// Measured vector-ALU peak (dd_vector_peak): the FMA throughput this device
// reaches in the instruction forms the pair kernels use (FP64 FMA, and FP32
// FMA without packed FP32 instructions, which every build disables), with one
// operand from a scalar register or all operands from vector registers.  A
// reference point for the all-pairs kernels' roofline next to the published
// peaks.
#include "dd_common.h"

namespace dd {

constexpr int PROBE_CHAINS = 8;      // independent FMA chains per lane
constexpr int PROBE_ITERS = 4096;    // chain steps per launch
constexpr int PROBE_BLOCKS = 4096;   // 16 workgroups of 256 lanes per CU

// VEC = false: a <- x y + a with x, y the same for every lane (one operand
// comes from a scalar register, as in the FP64 pair kernel); VEC = true:
// a <- b d + a with b, d per lane (every operand in a vector register, as in
// the FP32 quadrature).
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_fma_peak(T x, T y, T *__restrict__ out)
{
    T a[PROBE_CHAINS], b[PROBE_CHAINS], d[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) {
        a[k] = (T)(threadIdx.x + k);
        b[k] = x + (T)(threadIdx.x * (k + 1)) * (T)1e-9;
        d[k] = y - (T)k * (T)1e-9;
    }
    for (int i = 0; i < PROBE_ITERS; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) a[k] = VEC ? fma(b[k], d[k], a[k]) : fma(x, y, a[k]);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += a[k];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename T, bool VEC>
int probe(int reps, double *tflops, hipStream_t st)
{
    Workspace *ws;
    int rc;
    if ((rc = workspace(&ws))) return rc;
    void *p;
    if ((rc = ensure(ws, WS_PROBE, sizeof(T) * 256 * PROBE_BLOCKS, &p))) return rc;
    // small x * y: the chains grow by 1e-6 per step, far from overflow
    const T x = (T)0.001, y = (T)0.001;
    hipEvent_t e0, e1;
    DD_HIP(hipEventCreate(&e0));
    DD_HIP(hipEventCreate(&e1));
    for (int r = 0; r < 3; ++r)   // warm-up: clocks ramp up under load
        hipLaunchKernelGGL((k_fma_peak<T, VEC>), dim3(PROBE_BLOCKS), dim3(256), 0, st, x, y, (T *)p);
    DD_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL((k_fma_peak<T, VEC>), dim3(PROBE_BLOCKS), dim3(256), 0, st, x, y, (T *)p);
    DD_HIP(hipEventRecord(e1, st));
    DD_HIP(hipGetLastError());
    DD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DD_HIP(hipEventElapsedTime(&ms, e0, e1));
    DD_HIP(hipEventDestroy(e0));
    DD_HIP(hipEventDestroy(e1));
    const double flop = 2.0 * PROBE_CHAINS * PROBE_ITERS * 256.0 * PROBE_BLOCKS * reps;
    *tflops = flop / (ms * 1e-3) / 1e12;
    return DD_OK;
}

}  // namespace dd

extern "C" int dd_vector_peak(int kind, int reps, double *tflops, void *stream)
{
    ::dd::Range range_("dd_vector_peak");
    dd::clear_error();
    if (!tflops) return dd::set_error(DD_EINVAL, "tflops is null");
    if (reps < 1 || reps > 1000) return dd::set_error(DD_EINVAL, "reps must be in 1..1000");
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
    case 0: return dd::probe<double, false>(reps, tflops, st);
    case 1: return dd::probe<float, false>(reps, tflops, st);
    case 2: return dd::probe<double, true>(reps, tflops, st);
    case 3: return dd::probe<float, true>(reps, tflops, st);
    default: return dd::set_error(DD_EINVAL, "kind must be 0..3");
    }
}
