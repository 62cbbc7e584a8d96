// Slip-rate surrogate of libdd.so: an ensemble of MLPs 36 -> 256 -> 256 ->
// 256 -> 12 (ReLU hidden layers) trained and evaluated with hand-written
// bfloat16 matrix-core (MFMA) kernels, float32 accumulation, float32 master
// weights and Adam moments.
//
// Every product of the forward and backward passes is one launch of the
// batched GEMM kernel below (blockIdx.z = ensemble member), with the bias,
// activation and ReLU-derivative work fused into its epilogue.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dd_common.h"

namespace dd {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int IN = DD_MLP_IN, HID = DD_MLP_HIDDEN, OUT = DD_MLP_OUT;
constexpr int INP = 64;    // input width padded for K steps of 32
constexpr int OUTP = 16;   // output width padded to one MFMA tile
constexpr int64_t P = DD_MLP_PARAMS;
// offsets of the flat master parameters (see dd.h)
constexpr int64_t OW1 = 0, OB1 = OW1 + HID * IN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID,
                  OW3 = OB2 + HID, OB3 = OW3 + HID * HID, OW4 = OB3 + HID, OB4 = OW4 + OUT * HID;
static_assert(OB4 + OUT == P, "parameter layout");

__device__ __forceinline__ __bf16 to_bf16(float v) { return __float2bfloat16(v); }
__device__ __forceinline__ float from_bf16(__bf16 v) { return __bfloat162float(v); }

// ------------------------------------------------------------------ GEMM --
// C[m][n] = sum_k A(m, k) B(n, k) for one ensemble member (blockIdx.z):
//   A(m, k) = TA ? A[k lda + m] : A[m lda + k]      (bf16)
//   B(n, k) = TB ? B[k ldb + n] : B[n ldb + k]      (bf16)
// Workgroup tile 64 x 64, K step 32, four waves in a 2 x 2 arrangement each
// owning 32 x 32 = 2 x 2 tiles of v_mfma_f32_16x16x32_bf16.  Operand layout
// of that instruction: lane l holds row (A) / column (B) l % 16 and the eight
// k values 8 (l / 16) .. 8 (l / 16) + 7; the accumulator holds column l % 16,
// rows 4 (l / 16) .. 4 (l / 16) + 3.
enum Epi {
    EPI_BIAS_RELU_BF16 = 0,   // out_h = bf16(relu(acc + bias))
    EPI_BIAS_F32 = 1,         // out_f = acc + bias
    EPI_F32 = 2,              // out_f = acc
    EPI_MASK = 3,             // g = acc * (mask_h > 0): out_h = bf16(g), out_f = g
};

struct GemmArgs {
    const __bf16 *A; int64_t lda, sA;       // sA: member stride (elements)
    const __bf16 *B; int64_t ldb, sB;
    int M, N, K;
    const float *bias; int64_t sbias; int nbias;
    const __bf16 *mask; int64_t ldmask, smask;
    __bf16 *out_h; float *out_f; int64_t ldo, so_h, so_f;
};

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

template <bool TA, bool TB>
__device__ __forceinline__ void stage(const GemmArgs &g, int member, int m0, int n0, int k0,
                                      __bf16 (*As)[LDSK], __bf16 (*Bs)[LDSK])
{
    const int t = threadIdx.x;
    const __bf16 *A = g.A + member * g.sA;
    const __bf16 *B = g.B + member * g.sB;
    const __bf16 zero = to_bf16(0.f);
    if (!TA) {   // row r, k offset 8 (t % 4)
        const int r = t / 4, kk = (t % 4) * 8, m = m0 + r;
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + kk + i;
            As[r][kk + i] = (m < g.M && k < g.K) ? A[(int64_t)m * g.lda + k] : zero;
        }
    } else {     // k row t / 8, m offset 8 (t % 8)
        const int kr = t / 8, mm = (t % 8) * 8, k = k0 + kr;
        for (int i = 0; i < 8; ++i) {
            const int m = m0 + mm + i;
            As[mm + i][kr] = (m < g.M && k < g.K) ? A[(int64_t)k * g.lda + m] : zero;
        }
    }
    if (!TB) {
        const int r = t / 4, kk = (t % 4) * 8, n = n0 + r;
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + kk + i;
            Bs[r][kk + i] = (n < g.N && k < g.K) ? B[(int64_t)n * g.ldb + k] : zero;
        }
    } else {
        const int kr = t / 8, nn = (t % 8) * 8, k = k0 + kr;
        for (int i = 0; i < 8; ++i) {
            const int n = n0 + nn + i;
            Bs[nn + i][kr] = (n < g.N && k < g.K) ? B[(int64_t)k * g.ldb + n] : zero;
        }
    }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __bf16 As[BM][LDSK];
    __shared__ __bf16 Bs[BN][LDSK];
    const int member = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += BK) {
        __syncthreads();
        stage<TA, TB>(g, member, m0, n0, k0, As, Bs);
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i)
            for (int e = 0; e < 8; ++e) a[i][e] = As[wm + 16 * i + lr][lk + e];
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 8; ++e) b[j][e] = Bs[wn + 16 * j + lr][lk + e];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }

    // epilogue: lane owns column n, rows r .. r+3 of each 16 x 16 tile
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + lr;
            if (n >= g.N) continue;
            float bias = 0.f;
            if (EPI == EPI_BIAS_RELU_BF16 || EPI == EPI_BIAS_F32)
                bias = (n < g.nbias) ? g.bias[member * g.sbias + n] : 0.f;
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + e;
                if (m >= g.M) continue;
                const float v = acc[i][j][e];
                const int64_t o = (int64_t)m * g.ldo + n;
                if (EPI == EPI_BIAS_RELU_BF16) {
                    g.out_h[member * g.so_h + o] = to_bf16(fmaxf(v + bias, 0.f));
                } else if (EPI == EPI_BIAS_F32) {
                    g.out_f[member * g.so_f + o] = v + bias;
                } else if (EPI == EPI_F32) {
                    g.out_f[member * g.so_f + o] = v;
                } else {
                    const float h = from_bf16(g.mask[member * g.smask + (int64_t)m * g.ldmask + n]);
                    const float d = h > 0.f ? v : 0.f;
                    g.out_h[member * g.so_h + o] = to_bf16(d);
                    g.out_f[member * g.so_f + o] = d;
                }
            }
        }
}

template <bool TA, bool TB, int EPI>
static void gemm(const GemmArgs &g, int members, hipStream_t st)
{
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, members);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, g);
}

// ------------------------------------------------------- small kernels --
// X0[r][k] = bf16((f - shift[k]) * scale[k]) for k < 36 (0 up to 64), with
// f = log10(max(feat, 0) * dens_scale + dens_floor) for the density features
// 12..35 when dens_floor > 0, f = feat otherwise.
constexpr int SCAL = 2 * IN + 2 * OUT + 3;   // shifts/scales, dens_scale, dens_floor, spread floor

__global__ void k_standardize(const float *__restrict__ feat, int64_t n, const float *__restrict__ scal,
                              __bf16 *__restrict__ X0)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * INP) return;
    const int64_t r = i / INP;
    const int k = (int)(i % INP);
    float v = 0.f;
    if (k < IN) {
        float f = feat[r * IN + k];
        const float dfloor = scal[2 * IN + 2 * OUT + 1];
        if (k >= 12 && dfloor > 0.f) f = log10f(fmaxf(f, 0.f) * scal[2 * IN + 2 * OUT] + dfloor);
        v = (f - scal[k]) * scal[IN + k];
    }
    X0[i] = to_bf16(v);
}

// Loss and output gradient, one workgroup per member:
//   T'[r][o] = (target[r][o] - out_shift[o]) / out_scale[o]
//   dY[r][o] = 2 (Y[r][o] - T'[r][o]) / (n 12) (0 in the padding columns)
//   loss = mean over r, o of (Y - T')^2, summed in a fixed tree order.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ Y, int64_t sY, const float *__restrict__ target,
                                              int64_t n, const float *__restrict__ scal, float *__restrict__ dYf,
                                              __bf16 *__restrict__ dYh, int64_t sdY, float *loss_out)
{
    __shared__ double red[256];
    const int member = blockIdx.x;
    const float *Ym = Y + member * sY;
    double acc = 0.0;
    const float inv = 2.f / (float)(n * OUT);
    for (int64_t i = threadIdx.x; i < n * OUTP; i += blockDim.x) {
        const int64_t r = i / OUTP;
        const int o = (int)(i % OUTP);
        float d = 0.f;
        if (o < OUT) {
            const float tt = (target[r * OUT + o] - scal[2 * IN + o]) / scal[2 * IN + OUT + o];
            const float e = Ym[r * OUTP + o] - tt;
            acc += (double)e * e;
            d = inv * e;
        }
        dYf[member * sdY + i] = d;
        dYh[member * sdY + i] = to_bf16(d);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_out) loss_out[member] = (float)(red[0] / (double)(n * OUT));
}

// Column sums (bias gradients): out[member][c] = sum_r G[member][r][c].
// Workgroup = 64 columns x 4 row lanes of one member; each lane sums rows
// r = lane_row, lane_row + 4, ... in order, then the 4 partials are added in
// a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ G, int64_t sG, int64_t n, int ld,
                                                int ncols, float *__restrict__ out, int64_t sout)
{
    __shared__ float part[4][64];
    const int member = blockIdx.y;
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
    const float *g = G + member * sG;
    float s = 0.f;
    if (c < ncols)
        for (int64_t r = rl; r < n; r += 4) s += g[r * ld + c];
    part[rl][threadIdx.x & 63] = s;
    __syncthreads();
    if (rl == 0 && c < ncols)
        out[member * sout + c] = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) +
                                 part[3][threadIdx.x];
}

// Adam on the flat master parameters; gradients are read from the padded
// GEMM layouts (dW1 [256][64], dW4 [16][256], biases).
struct GradPtrs {
    const float *dW1, *dW2, *dW3, *dW4, *db1, *db2, *db3, *db4;
    int64_t s1, s2, s3, s4, sb;   // member strides
};

__device__ __forceinline__ float grad_at(const GradPtrs &G, int member, int64_t p)
{
    if (p < OB1) { int64_t o = p / IN, i = p % IN; return G.dW1[member * G.s1 + o * INP + i]; }
    if (p < OW2) return G.db1[member * G.sb + (p - OB1)];
    if (p < OB2) return G.dW2[member * G.s2 + (p - OW2)];
    if (p < OW3) return G.db2[member * G.sb + (p - OB2)];
    if (p < OB3) return G.dW3[member * G.s3 + (p - OW3)];
    if (p < OW4) return G.db3[member * G.sb + (p - OB3)];
    if (p < OB4) return G.dW4[member * G.s4 + (p - OW4)];
    return G.db4[member * G.sb + (p - OB4)];
}

__global__ void k_gather_grads(GradPtrs G, int members, float *__restrict__ out)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= members * P) return;
    out[i] = grad_at(G, (int)(i / P), i % P);
}

// Adam with (1 - beta1), (1 - beta2) and the bias corrections 1 - beta^t all
// formed in double on the host and rounded once, so that the first step is
// exactly the normalised gradient.
__global__ void k_adam(GradPtrs G, int members, float *__restrict__ w, float *__restrict__ m1,
                       float *__restrict__ m2, float lr, float b1, float b2, float omb1, float omb2, float eps,
                       float c1, float c2)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= members * P) return;
    const float g = grad_at(G, (int)(i / P), i % P);
    const float a = b1 * m1[i] + omb1 * g;
    const float v = b2 * m2[i] + omb2 * g * g;
    m1[i] = a;
    m2[i] = v;
    w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// bf16 weight copies in the GEMM layouts: W1p [256][64] (zero padded), W2,
// W3 [256][256], W4p [16][256] (rows 12..15 zero); bias4 padded to 16.
__global__ void k_refresh(const float *__restrict__ w, int members, __bf16 *__restrict__ W1p,
                          __bf16 *__restrict__ W2, __bf16 *__restrict__ W3, __bf16 *__restrict__ W4p)
{
    const int64_t per = (int64_t)HID * INP + 2 * (int64_t)HID * HID + (int64_t)OUTP * HID;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= members * per) return;
    const int member = (int)(i / per);
    int64_t j = i % per;
    const float *wm = w + member * P;
    if (j < (int64_t)HID * INP) {
        const int64_t o = j / INP, k = j % INP;
        W1p[member * (int64_t)HID * INP + j] = to_bf16(k < IN ? wm[OW1 + o * IN + k] : 0.f);
        return;
    }
    j -= (int64_t)HID * INP;
    if (j < (int64_t)HID * HID) { W2[member * (int64_t)HID * HID + j] = to_bf16(wm[OW2 + j]); return; }
    j -= (int64_t)HID * HID;
    if (j < (int64_t)HID * HID) { W3[member * (int64_t)HID * HID + j] = to_bf16(wm[OW3 + j]); return; }
    j -= (int64_t)HID * HID;
    const int64_t o = j / HID;
    W4p[member * (int64_t)OUTP * HID + j] = to_bf16(o < OUT ? wm[OW4 + j] : 0.f);
}

// Ensemble reduction per point: rates = member mean (unstandardised),
// spread = |population std|_2 / max(|mean|_2, 1e-30), needs_dd = spread > tol.
__global__ void k_ensemble(const float *__restrict__ Y, int64_t sY, int members, int64_t n,
                           const float *__restrict__ scal, float tol, float *__restrict__ rates,
                           float *__restrict__ spread, uint8_t *__restrict__ needs_dd)
{
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    float mean[OUT], var[OUT];
    for (int o = 0; o < OUT; ++o) mean[o] = var[o] = 0.f;
    for (int m = 0; m < members; ++m)
        for (int o = 0; o < OUT; ++o)
            mean[o] += Y[m * sY + r * OUTP + o] * scal[2 * IN + OUT + o] + scal[2 * IN + o];
    const float im = 1.f / members;
    for (int o = 0; o < OUT; ++o) mean[o] *= im;
    for (int m = 0; m < members; ++m)
        for (int o = 0; o < OUT; ++o) {
            const float d = Y[m * sY + r * OUTP + o] * scal[2 * IN + OUT + o] + scal[2 * IN + o] - mean[o];
            var[o] += d * d;
        }
    float s2 = 0.f, m2 = 0.f;
    for (int o = 0; o < OUT; ++o) {
        s2 += var[o] * im;
        m2 += mean[o] * mean[o];
        rates[r * OUT + o] = mean[o];
    }
    const float sp = sqrtf(s2) / fmaxf(sqrtf(m2), scal[2 * IN + 2 * OUT + 2]);
    spread[r] = sp;
    needs_dd[r] = sp > tol ? 1 : 0;
}


// ------------------------------------------------- fused inference kernel --
constexpr int HSTR = HID + 8;   // LDS row stride of the activations (bf16)

__device__ __forceinline__ bf16x8 lds_frag(const __bf16 *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ bf16x8 glb_frag(const __bf16 *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

// One workgroup (RG x CG waves) carries WROWS = 64 RG rows of one member
// (blockIdx.y) through all four layers in one LDS buffer: the standardised
// inputs, then each hidden layer's activations overwrite the previous ones
// (every wave holds its output tile in registers until all waves have read
// the layer's input).  Rows are padded by 8 bf16 so that the 16-byte fragment
// reads of 16 consecutive rows fall in distinct banks.  Hidden layers: wave w
// owns rows 64 (w / CG) .. +63 and output columns 16 JT (w % CG) .. +16 JT - 1
// (4 x JT tiles of v_mfma_f32_16x16x32_bf16); bias + ReLU are applied when
// the accumulators are written back.  The layer's weights come through LDS
// one K step (32 inputs x 256 outputs) at a time, loaded once per workgroup
// and read by the RG waves of every column group, so each weight reaches the
// CU once per WROWS rows: the L2-to-CU weight traffic, which bounds a
// workgroup of 64 rows that streams every wave's own weights, falls by RG.
// The next slice is fetched into registers one step ahead; two barriers per
// step guard the one slice buffer (a second does not fit beside the
// activations).  Output layer: its weights also go through LDS, and the waves
// split the WROWS rows in tiles of 16.
constexpr int WRG = 4;                  // row groups of 64
constexpr int WJT = 4;                  // 16-column tiles per wave
constexpr int WCG = HID / (16 * WJT);   // column groups
constexpr int WROWS = 64 * WRG;
constexpr int WTHREADS = 64 * WRG * WCG;
constexpr int WSTR = 32;                // LDS row stride of a weight slice (bf16)
constexpr int WSLICE = HID * WSTR;      // one slice buffer (bf16)
constexpr int WCHUNKS = HID * 32 / 8;   // 16-byte chunks per slice
constexpr int WPER = (WCHUNKS + WTHREADS - 1) / WTHREADS;

// Position of 16-byte chunk c (0..3) of output row o in a slice buffer: the
// chunk index is XOR-ed with bits 1-2 of the row, so that both the fragment
// reads (16 rows, one chunk) and the stores (4 rows, 4 chunks) of 16 lanes
// spread over all banks.
__device__ __forceinline__ int slice_pos(int o, int c)
{
    return o * WSTR + ((c ^ ((o >> 1) & 3)) << 3);
}

template <int K>
__device__ __forceinline__ void hidden_layer(__bf16 *__restrict__ H, __bf16 *__restrict__ Ws,
                                             const __bf16 *__restrict__ W, const float *__restrict__ bias,
                                             int wave, int lane, int tid)
{
    // W: [HID][K] (out, in), K contiguous
    constexpr int NS = K / 32;
    f32x4 acc[4][WJT];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < WJT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const int rg = wave / WCG, cg = wave % WCG;
    // this thread's chunks of a slice: chunk c = output row c / 4, inputs 8 (c % 4) .. +7
    bf16x8 pre[WPER];
#pragma unroll
    for (int u = 0; u < WPER; ++u) {
        const int c = tid + u * WTHREADS;
        if (c < WCHUNKS) pre[u] = glb_frag(W + (int64_t)(c >> 2) * K + (c & 3) * 8);
    }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        if (st > 0) __syncthreads();   // slice st - 1 read by every wave
#pragma unroll
        for (int u = 0; u < WPER; ++u) {
            const int c = tid + u * WTHREADS;
            if (c < WCHUNKS) *reinterpret_cast<bf16x8 *>(Ws + slice_pos(c >> 2, c & 3)) = pre[u];
        }
        if (st + 1 < NS) {
#pragma unroll
            for (int u = 0; u < WPER; ++u) {
                const int c = tid + u * WTHREADS;
                if (c < WCHUNKS) pre[u] = glb_frag(W + (int64_t)(c >> 2) * K + 32 * (st + 1) + (c & 3) * 8);
            }
        }
        __syncthreads();   // slice st (and, at st = 0, the layer input) in place
        const int k0 = 32 * st;
        bf16x8 a[4], b[WJT];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = lds_frag(H + (64 * rg + 16 * i + lr) * HSTR + k0 + lk);
#pragma unroll
        for (int j = 0; j < WJT; ++j) b[j] = lds_frag(Ws + slice_pos(16 * WJT * cg + 16 * j + lr, lane >> 4));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < WJT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();   // every wave has read the layer input and the last slice
    for (int j = 0; j < WJT; ++j) {
        const int n = 16 * WJT * cg + 16 * j + lr;
        const float bn_ = bias[n];
        for (int i = 0; i < 4; ++i)
            for (int e = 0; e < 4; ++e) {
                const int r = 64 * rg + 16 * i + (lane >> 4) * 4 + e;
                H[r * HSTR + n] = to_bf16(fmaxf(acc[i][j][e] + bn_, 0.f));
            }
    }
}

__global__ __launch_bounds__(WTHREADS) void k_mlp_infer(const float *__restrict__ feat, int64_t n,
                                                             const float *__restrict__ scal,
                                                             const __bf16 *__restrict__ W1p,
                                                             const __bf16 *__restrict__ W2,
                                                             const __bf16 *__restrict__ W3,
                                                             const __bf16 *__restrict__ W4p,
                                                             const float *__restrict__ w, float *__restrict__ Y,
                                                             int64_t sY)
{
    __shared__ __attribute__((aligned(16))) __bf16 H[WROWS * HSTR];
    __shared__ __attribute__((aligned(16))) __bf16 Ws[WSLICE];
    const int member = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * WROWS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float dfloor = scal[2 * IN + 2 * OUT + 1], dscale = scal[2 * IN + 2 * OUT];
    // standardised input tile (rows beyond n and columns beyond IN are zero)
    for (int i = tid; i < WROWS * INP; i += WTHREADS) {
        const int r = i / INP, k = i % INP;
        float v = 0.f;
        if (k < IN && r0 + r < n) {
            float f = feat[(r0 + r) * IN + k];
            if (k >= 12 && dfloor > 0.f) f = log10f(fmaxf(f, 0.f) * dscale + dfloor);
            v = (f - scal[k]) * scal[IN + k];
        }
        H[r * HSTR + k] = to_bf16(v);
    }
    const float *wm = w + member * P;
    hidden_layer<INP>(H, Ws, W1p + (int64_t)member * HID * INP, wm + OB1, wave, lane, tid);
    hidden_layer<HID>(H, Ws, W2 + (int64_t)member * HID * HID, wm + OB2, wave, lane, tid);
    hidden_layer<HID>(H, Ws, W3 + (int64_t)member * HID * HID, wm + OB3, wave, lane, tid);
    // the output layer's weights [16][256] to the slice buffer, row stride HSTR
    // (every wave has finished reading the last slice inside hidden_layer)
    static_assert(OUTP * HSTR <= WSLICE, "output weights fit the slice buffer");
    const __bf16 *W4m = W4p + (int64_t)member * OUTP * HID;
    for (int c = tid; c < OUTP * HID / 8; c += WTHREADS)
        *reinterpret_cast<bf16x8 *>(Ws + (c / (HID / 8)) * HSTR + (c % (HID / 8)) * 8) = glb_frag(W4m + 8 * c);
    __syncthreads();   // last hidden activations and output weights in place
    // output layer: wave owns WROWS / (waves) rows in tiles of 16, 16 padded columns
    constexpr int OT = WROWS / 16 / (WRG * WCG);   // row tiles per wave
    {
        const int lr = lane & 15, lk = (lane >> 4) * 8;
        f32x4 acc[OT];
        for (int t = 0; t < OT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < HID; k0 += 32) {
            const bf16x8 b = lds_frag(Ws + lr * HSTR + k0 + lk);
#pragma unroll
            for (int t = 0; t < OT; ++t) {
                const bf16x8 a = lds_frag(H + (16 * (OT * wave + t) + lr) * HSTR + k0 + lk);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
        const int o = lr;
        const float bo = o < OUT ? wm[OB4 + o] : 0.f;
        for (int t = 0; t < OT; ++t)
            for (int e = 0; e < 4; ++e) {
                const int64_t r = r0 + 16 * (OT * wave + t) + (lane >> 4) * 4 + e;
                if (r < n) Y[member * sY + r * OUTP + o] = acc[t][e] + bo;
            }
    }
}

}  // namespace mlp
}  // namespace dd

// ============================================================= host side ==
using namespace dd;
using namespace dd::mlp;

struct dd_mlp {
    int members = 0;
    int device = -1;
    float *w = nullptr, *m1 = nullptr, *m2 = nullptr;   // [members][P]
    int64_t t = 0;                                        // Adam steps taken
    __bf16 *W1p = nullptr, *W2 = nullptr, *W3 = nullptr, *W4p = nullptr;
    float *scal = nullptr;                                // device [2*36 + 2*12]
    float h_scal[SCAL];                                   // host copy
    float *dW1 = nullptr, *dW2 = nullptr, *dW3 = nullptr, *dW4 = nullptr, *db = nullptr;
    // row workspace, sized for `cap` rows
    int64_t cap = 0;
    bool cap_train = false;
    __bf16 *X0 = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *dYh = nullptr;
    __bf16 *Dh[2] = {nullptr, nullptr};
    float *Y = nullptr, *dYf = nullptr;
    float *Df[2] = {nullptr, nullptr};
};

namespace {

constexpr int64_t INFER_CHUNK = 262144;   // rows per inference pass
constexpr int64_t TRAIN_MAX = 65536;

void free_rows(dd_mlp *h)
{
    void *ps[] = {h->X0, h->H1, h->H2, h->H3, h->dYh, h->Dh[0], h->Dh[1], h->Y, h->dYf, h->Df[0], h->Df[1]};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    h->X0 = h->H1 = h->H2 = h->H3 = h->dYh = h->Dh[0] = h->Dh[1] = nullptr;
    h->Y = h->dYf = h->Df[0] = h->Df[1] = nullptr;
    h->cap = 0;
    h->cap_train = false;
}

int dev_alloc(void **p, size_t bytes)
{
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(DD_ENOMEM, "surrogate allocation of %zu bytes failed", bytes);
    }
    return DD_OK;
}

int ensure_rows(dd_mlp *h, int64_t rows, bool training)
{
    if (rows <= h->cap && (!training || h->cap_train)) return DD_OK;
    DD_HIP(hipDeviceSynchronize());
    const bool train = training || h->cap_train;
    rows = std::max(rows, h->cap);
    free_rows(h);
    const int64_t M = h->members;
    int rc;
    if ((rc = dev_alloc((void **)&h->X0, sizeof(__bf16) * rows * INP))) return rc;
    if ((rc = dev_alloc((void **)&h->H1, sizeof(__bf16) * M * rows * HID))) return rc;
    if ((rc = dev_alloc((void **)&h->H2, sizeof(__bf16) * M * rows * HID))) return rc;
    if ((rc = dev_alloc((void **)&h->H3, sizeof(__bf16) * M * rows * HID))) return rc;
    if ((rc = dev_alloc((void **)&h->Y, sizeof(float) * M * rows * OUTP))) return rc;
    if (train) {
        if ((rc = dev_alloc((void **)&h->dYh, sizeof(__bf16) * M * rows * OUTP))) return rc;
        if ((rc = dev_alloc((void **)&h->dYf, sizeof(float) * M * rows * OUTP))) return rc;
        for (int k = 0; k < 2; ++k) {
            if ((rc = dev_alloc((void **)&h->Dh[k], sizeof(__bf16) * M * rows * HID))) return rc;
            if ((rc = dev_alloc((void **)&h->Df[k], sizeof(float) * M * rows * HID))) return rc;
        }
    }
    h->cap = rows;
    h->cap_train = train;
    return DD_OK;
}

// host RNG for the initial weights: splitmix64, top 53 bits -> [0, 1)
uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int refresh(dd_mlp *h, hipStream_t st)
{
    const int64_t per = (int64_t)HID * INP + 2 * (int64_t)HID * HID + (int64_t)OUTP * HID;
    const int64_t tot = per * h->members;
    hipLaunchKernelGGL(k_refresh, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, h->w, h->members,
                       h->W1p, h->W2, h->W3, h->W4p);
    DD_HIP(hipGetLastError());
    return DD_OK;
}

int check_model(const dd_mlp *h)
{
    if (!h) return set_error(DD_EINVAL, "null surrogate handle");
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    if (dev != h->device) return set_error(DD_EINVAL, "surrogate used on device %d, created on %d", dev, h->device);
    return DD_OK;
}

// Forward pass of all members on rows [0, n) of X0 (already standardised).
void forward(dd_mlp *h, int64_t n, hipStream_t st)
{
    const int M = h->members;
    GemmArgs g{};
    g.A = h->X0; g.lda = INP; g.sA = 0;                 // the members share the inputs
    g.B = h->W1p; g.ldb = INP; g.sB = (int64_t)HID * INP;
    g.M = (int)n; g.N = HID; g.K = INP;
    g.bias = h->w + OB1; g.sbias = P; g.nbias = HID;
    g.out_h = h->H1; g.ldo = HID; g.so_h = n * HID;
    gemm<false, false, EPI_BIAS_RELU_BF16>(g, M, st);
    const __bf16 *ins[2] = {h->H1, h->H2};
    __bf16 *outs[2] = {h->H2, h->H3};
    const __bf16 *Ws[2] = {h->W2, h->W3};
    const int64_t bo[2] = {OB2, OB3};
    for (int l = 0; l < 2; ++l) {
        g = GemmArgs{};
        g.A = ins[l]; g.lda = HID; g.sA = n * HID;
        g.B = Ws[l]; g.ldb = HID; g.sB = (int64_t)HID * HID;
        g.M = (int)n; g.N = HID; g.K = HID;
        g.bias = h->w + bo[l]; g.sbias = P; g.nbias = HID;
        g.out_h = outs[l]; g.ldo = HID; g.so_h = n * HID;
        gemm<false, false, EPI_BIAS_RELU_BF16>(g, M, st);
    }
    g = GemmArgs{};
    g.A = h->H3; g.lda = HID; g.sA = n * HID;
    g.B = h->W4p; g.ldb = HID; g.sB = (int64_t)OUTP * HID;
    g.M = (int)n; g.N = OUTP; g.K = HID;
    g.bias = h->w + OB4; g.sbias = P; g.nbias = OUT;
    g.out_f = h->Y; g.ldo = OUTP; g.so_f = n * OUTP;
    gemm<false, false, EPI_BIAS_F32>(g, M, st);
}

GradPtrs grad_ptrs(const dd_mlp *h)
{
    GradPtrs G;
    G.dW1 = h->dW1; G.dW2 = h->dW2; G.dW3 = h->dW3; G.dW4 = h->dW4;
    G.db1 = h->db; G.db2 = h->db + HID; G.db3 = h->db + 2 * HID; G.db4 = h->db + 3 * HID;
    G.s1 = (int64_t)HID * INP; G.s2 = G.s3 = (int64_t)HID * HID; G.s4 = (int64_t)OUTP * HID;
    G.sb = 4 * HID;
    return G;
}

void colsum(const float *G, int64_t sG, int64_t n, int ld, int ncols, float *out, int members, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((ncols + 63) / 64, members), dim3(256), 0, st, G, sG, n, ld, ncols, out,
                       (int64_t)4 * HID);
}

// Forward + backward on n rows.  Gradients land in dW1..dW4 (padded GEMM
// layouts) and db; per-member losses in loss_out (nullable).
int gradients(dd_mlp *h, int64_t n, const float *feat, const float *target, float *loss_out, hipStream_t st)
{
    const int M = h->members;
    int rc;
    if ((rc = ensure_rows(h, n, true))) return rc;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n * INP + 255) / 256)), dim3(256), 0, st, feat, n,
                       h->scal, h->X0);
    forward(h, n, st);
    hipLaunchKernelGGL(k_loss, dim3(M), dim3(256), 0, st, h->Y, n * OUTP, target, n, h->scal, h->dYf, h->dYh,
                       n * OUTP, loss_out);
    GemmArgs g{};
    // output layer: dW4 [16][256] = dY^T H3, db4 = colsum(dY)
    g.A = h->dYh; g.lda = OUTP; g.sA = n * OUTP;
    g.B = h->H3; g.ldb = HID; g.sB = n * HID;
    g.M = OUTP; g.N = HID; g.K = (int)n;
    g.out_f = h->dW4; g.ldo = HID; g.so_f = (int64_t)OUTP * HID;
    gemm<true, true, EPI_F32>(g, M, st);
    colsum(h->dYf, n * OUTP, n, OUTP, OUTP, h->db + 3 * HID, M, st);
    // dZ3 = (dY W4p) * (H3 > 0)  -> buffer 0
    g = GemmArgs{};
    g.A = h->dYh; g.lda = OUTP; g.sA = n * OUTP;
    g.B = h->W4p; g.ldb = HID; g.sB = (int64_t)OUTP * HID;
    g.M = (int)n; g.N = HID; g.K = OUTP;
    g.mask = h->H3; g.ldmask = HID; g.smask = n * HID;
    g.out_h = h->Dh[0]; g.out_f = h->Df[0]; g.ldo = HID; g.so_h = n * HID; g.so_f = n * HID;
    gemm<false, true, EPI_MASK>(g, M, st);
    // hidden layers 3 and 2: dW = dZ^T H_prev, db = colsum(dZ),
    // dZ_prev = (dZ W) * (H_prev > 0) into the other buffer
    const __bf16 *Hprev[2] = {h->H2, h->H1};
    float *dWs[2] = {h->dW3, h->dW2};
    const __bf16 *Ws[2] = {h->W3, h->W2};
    const int dbo[2] = {2 * HID, 1 * HID};
    int cur = 0;
    for (int l = 0; l < 2; ++l) {
        g = GemmArgs{};
        g.A = h->Dh[cur]; g.lda = HID; g.sA = n * HID;
        g.B = Hprev[l]; g.ldb = HID; g.sB = n * HID;
        g.M = HID; g.N = HID; g.K = (int)n;
        g.out_f = dWs[l]; g.ldo = HID; g.so_f = (int64_t)HID * HID;
        gemm<true, true, EPI_F32>(g, M, st);
        colsum(h->Df[cur], n * HID, n, HID, HID, h->db + dbo[l], M, st);
        g = GemmArgs{};
        g.A = h->Dh[cur]; g.lda = HID; g.sA = n * HID;
        g.B = Ws[l]; g.ldb = HID; g.sB = (int64_t)HID * HID;   // B(n = i, k = o) = W[o][i]
        g.M = (int)n; g.N = HID; g.K = HID;
        g.mask = Hprev[l]; g.ldmask = HID; g.smask = n * HID;
        g.out_h = h->Dh[1 - cur]; g.out_f = h->Df[1 - cur]; g.ldo = HID; g.so_h = n * HID; g.so_f = n * HID;
        gemm<false, true, EPI_MASK>(g, M, st);
        cur = 1 - cur;
    }
    // first layer: dW1 [256][64] = dZ1^T X0, db1
    g = GemmArgs{};
    g.A = h->Dh[cur]; g.lda = HID; g.sA = n * HID;
    g.B = h->X0; g.ldb = INP; g.sB = 0;
    g.M = HID; g.N = INP; g.K = (int)n;
    g.out_f = h->dW1; g.ldo = INP; g.so_f = (int64_t)HID * INP;
    gemm<true, true, EPI_F32>(g, M, st);
    colsum(h->Df[cur], n * HID, n, HID, HID, h->db, M, st);
    DD_HIP(hipGetLastError());
    return DD_OK;
}

int train_checks(const dd_mlp *h, int64_t n, const float *feat, const float *target)
{
    int rc;
    if ((rc = check_model(h))) return rc;
    if (n < 1 || n > TRAIN_MAX) return set_error(DD_EINVAL, "batch size must be in 1..65536");
    if (!feat || !target) return set_error(DD_EINVAL, "null feature or target array");
    return DD_OK;
}

}  // namespace

extern "C" int dd_mlp_create(int n_members, uint64_t seed, dd_mlp **out)
{
    clear_error();
    if (!out) return set_error(DD_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (n_members < 1 || n_members > 8) return set_error(DD_EINVAL, "n_members must be in 1..8");
    dd_mlp *h = new dd_mlp();
    h->members = n_members;
    int rc = DD_OK;
    if (hipGetDevice(&h->device) != hipSuccess) rc = set_error(DD_EHIP, "hipGetDevice failed");
    const int64_t M = n_members;
    if (!rc) rc = dev_alloc((void **)&h->w, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->m1, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->m2, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->W1p, sizeof(__bf16) * M * HID * INP);
    if (!rc) rc = dev_alloc((void **)&h->W2, sizeof(__bf16) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->W3, sizeof(__bf16) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->W4p, sizeof(__bf16) * M * OUTP * HID);
    if (!rc) rc = dev_alloc((void **)&h->scal, sizeof(float) * SCAL);
    if (!rc) rc = dev_alloc((void **)&h->dW1, sizeof(float) * M * HID * INP);
    if (!rc) rc = dev_alloc((void **)&h->dW2, sizeof(float) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->dW3, sizeof(float) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->dW4, sizeof(float) * M * OUTP * HID);
    if (!rc) rc = dev_alloc((void **)&h->db, sizeof(float) * M * 4 * HID);
    if (rc) {
        dd_mlp_destroy(h);
        return rc;
    }
    // He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases
    std::vector<float> p((size_t)(M * P), 0.f);
    for (int m = 0; m < n_members; ++m) {
        uint64_t s = seed + (uint64_t)m;
        float *pm = p.data() + m * P;
        auto fill = [&](int64_t off, int64_t count, int fan_in) {
            const double lim = std::sqrt(6.0 / fan_in);
            for (int64_t i = 0; i < count; ++i) {
                const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
                pm[off + i] = (float)((2.0 * u - 1.0) * lim);
            }
        };
        fill(OW1, (int64_t)HID * IN, IN);
        fill(OW2, (int64_t)HID * HID, HID);
        fill(OW3, (int64_t)HID * HID, HID);
        fill(OW4, (int64_t)OUT * HID, HID);
    }
    for (int k = 0; k < IN; ++k) { h->h_scal[k] = 0.f; h->h_scal[IN + k] = 1.f; }
    for (int k = 0; k < OUT; ++k) { h->h_scal[2 * IN + k] = 0.f; h->h_scal[2 * IN + OUT + k] = 1.f; }
    h->h_scal[2 * IN + 2 * OUT] = 1.f;
    h->h_scal[2 * IN + 2 * OUT + 1] = 0.f;
    h->h_scal[2 * IN + 2 * OUT + 2] = 1e-30f;
    if (hipMemcpy(h->w, p.data(), sizeof(float) * M * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->m1, 0, sizeof(float) * M * P) != hipSuccess ||
        hipMemset(h->m2, 0, sizeof(float) * M * P) != hipSuccess ||
        hipMemcpy(h->scal, h->h_scal, sizeof h->h_scal, hipMemcpyHostToDevice) != hipSuccess) {
        dd_mlp_destroy(h);
        return set_error(DD_EHIP, "initialising the surrogate failed");
    }
    if ((rc = refresh(h, nullptr)) || hipDeviceSynchronize() != hipSuccess) {
        dd_mlp_destroy(h);
        return rc ? rc : set_error(DD_EHIP, "initialising the surrogate failed");
    }
    *out = h;
    return DD_OK;
}

extern "C" int dd_mlp_destroy(dd_mlp *h)
{
    if (!h) return DD_OK;
    (void)hipDeviceSynchronize();
    free_rows(h);
    void *ps[] = {h->w, h->m1, h->m2, h->W1p, h->W2, h->W3, h->W4p, h->scal, h->dW1, h->dW2, h->dW3, h->dW4, h->db};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete h;
    return DD_OK;
}

extern "C" int dd_mlp_set_params(dd_mlp *h, int member, const float *host_params)
{
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (member < 0 || member >= h->members) return set_error(DD_EINVAL, "member out of range");
    if (!host_params) return set_error(DD_EINVAL, "null parameter array");
    for (int64_t i = 0; i < P; ++i)
        if (!std::isfinite(host_params[i])) return set_error(DD_EINVAL, "non-finite parameter %lld", (long long)i);
    DD_HIP(hipDeviceSynchronize());
    DD_HIP(hipMemcpy(h->w + member * P, host_params, sizeof(float) * P, hipMemcpyHostToDevice));
    DD_HIP(hipMemset(h->m1 + member * P, 0, sizeof(float) * P));
    DD_HIP(hipMemset(h->m2 + member * P, 0, sizeof(float) * P));
    h->t = 0;
    if ((rc = refresh(h, nullptr))) return rc;
    DD_HIP(hipDeviceSynchronize());
    return DD_OK;
}

extern "C" int dd_mlp_get_params(const dd_mlp *h, int member, float *host_params)
{
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (member < 0 || member >= h->members) return set_error(DD_EINVAL, "member out of range");
    if (!host_params) return set_error(DD_EINVAL, "null parameter array");
    DD_HIP(hipDeviceSynchronize());
    DD_HIP(hipMemcpy(host_params, h->w + member * P, sizeof(float) * P, hipMemcpyDeviceToHost));
    return DD_OK;
}

extern "C" int dd_mlp_set_scaling(dd_mlp *h, const float *in_shift, const float *in_scale,
                                  const float *out_shift, const float *out_scale)
{
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (!in_shift || !in_scale || !out_shift || !out_scale) return set_error(DD_EINVAL, "null scaling array");
    float s[SCAL];
    std::memcpy(s, h->h_scal, sizeof s);
    std::memcpy(s, in_shift, sizeof(float) * IN);
    std::memcpy(s + IN, in_scale, sizeof(float) * IN);
    std::memcpy(s + 2 * IN, out_shift, sizeof(float) * OUT);
    std::memcpy(s + 2 * IN + OUT, out_scale, sizeof(float) * OUT);
    for (float v : s)
        if (!std::isfinite(v)) return set_error(DD_EINVAL, "non-finite scaling value");
    for (int k = 0; k < OUT; ++k)
        if (!(s[2 * IN + OUT + k] != 0.f)) return set_error(DD_EINVAL, "out_scale must be non-zero");
    DD_HIP(hipDeviceSynchronize());
    std::memcpy(h->h_scal, s, sizeof s);
    DD_HIP(hipMemcpy(h->scal, s, sizeof s, hipMemcpyHostToDevice));
    return DD_OK;
}

extern "C" int dd_mlp_set_log_densities(dd_mlp *h, float dens_scale, float dens_floor)
{
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (!(dens_floor >= 0.f) || !std::isfinite(dens_floor) || !(dens_scale > 0.f) || !std::isfinite(dens_scale))
        return set_error(DD_EINVAL, "need dens_scale > 0 and dens_floor >= 0");
    DD_HIP(hipDeviceSynchronize());
    h->h_scal[2 * IN + 2 * OUT] = dens_scale;
    h->h_scal[2 * IN + 2 * OUT + 1] = dens_floor;
    DD_HIP(hipMemcpy(h->scal, h->h_scal, sizeof h->h_scal, hipMemcpyHostToDevice));
    return DD_OK;
}

extern "C" int dd_mlp_set_spread_floor(dd_mlp *h, float floor)
{
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (!(floor >= 0.f) || !std::isfinite(floor)) return set_error(DD_EINVAL, "spread floor must be >= 0");
    DD_HIP(hipDeviceSynchronize());
    h->h_scal[2 * IN + 2 * OUT + 2] = std::max(floor, 1e-30f);
    DD_HIP(hipMemcpy(h->scal, h->h_scal, sizeof h->h_scal, hipMemcpyHostToDevice));
    return DD_OK;
}

extern "C" int dd_mlp_gradients(dd_mlp *h, int64_t n, const float *feat, const float *target,
                                float *grad_out, float *loss_out, void *stream)
{
    clear_error();
    int rc;
    if ((rc = train_checks(h, n, feat, target))) return rc;
    if (!grad_out) return set_error(DD_EINVAL, "null gradient output");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = gradients(h, n, feat, target, loss_out, st))) return rc;
    const int64_t tot = h->members * P;
    hipLaunchKernelGGL(k_gather_grads, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, grad_ptrs(h),
                       h->members, grad_out);
    DD_HIP(hipGetLastError());
    return DD_OK;
}

extern "C" int dd_mlp_train_step(dd_mlp *h, int64_t n, const float *feat, const float *target, float lr,
                                 float *loss_out, void *stream)
{
    clear_error();
    int rc;
    if ((rc = train_checks(h, n, feat, target))) return rc;
    if (!(lr > 0.f) || !std::isfinite(lr)) return set_error(DD_EINVAL, "lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = gradients(h, n, feat, target, loss_out, st))) return rc;
    h->t += 1;
    const double B1 = 0.9, B2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(B1, (double)h->t));
    const float c2 = (float)(1.0 - std::pow(B2, (double)h->t));
    const int64_t tot = h->members * P;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, grad_ptrs(h), h->members,
                       h->w, h->m1, h->m2, lr, (float)B1, (float)B2, (float)(1.0 - B1), (float)(1.0 - B2), 1e-8f,
                       c1, c2);
    return refresh(h, st);
}

extern "C" int dd_surrogate_rates(const dd_mlp *hc, int64_t n, const float *feat, float *rates, float *spread,
                                  uint8_t *needs_dd, float spread_tol, void *stream)
{
    clear_error();
    dd_mlp *h = const_cast<dd_mlp *>(hc);   // the handle's workspace grows; the model is unchanged
    int rc;
    if ((rc = check_model(h))) return rc;
    if (n < 0) return set_error(DD_EINVAL, "n < 0");
    if (n == 0) return DD_OK;
    if (!feat || !rates || !spread || !needs_dd) return set_error(DD_EINVAL, "null array");
    if (!(spread_tol >= 0.f)) return set_error(DD_EINVAL, "spread_tol must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    const int64_t chunk = std::min<int64_t>(n, INFER_CHUNK);
    if ((rc = ensure_rows(h, chunk, false))) return rc;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t m = std::min(chunk, n - r0);
        dim3 grid((unsigned)((m + WROWS - 1) / WROWS), h->members);
        hipLaunchKernelGGL(k_mlp_infer, grid, dim3(WTHREADS), 0, st, feat + r0 * IN, m, h->scal, h->W1p, h->W2,
                           h->W3, h->W4p, h->w, h->Y, m * OUTP);
        hipLaunchKernelGGL(k_ensemble, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, h->Y, m * OUTP,
                           h->members, m, h->scal, spread_tol, rates + r0 * OUT, spread + r0, needs_dd + r0);
    }
    DD_HIP(hipGetLastError());
    return DD_OK;
}
