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
#include <cstdio>
#include <cstring>
#include <string>
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
    // split K (EPI_F32 only): nsp splits, blockIdx.z = split * members +
    // member; split s covers k in [s kc, min(K, (s + 1) kc)) and writes its
    // partial product at out_f + s ssplit.  kc is a multiple of BK; one
    // split: kc >= K.
    int kc, nsp; int64_t ssplit;
};

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

// Eight consecutive bf16 of a row of P (elements c .. c + 7 of row `row`,
// leading dimension ld), zero where c + i >= lim or the row is out of range:
// one 16-byte load when the eight lie inside and the address is 16-byte
// aligned, else element by element.
__device__ __forceinline__ bf16x8 load8(const __bf16 *P, int64_t ld, int row, bool row_ok, int c, int lim)
{
    bf16x8 v;
    const __bf16 zero = to_bf16(0.f);
    const __bf16 *q = P + (int64_t)row * ld + c;
    if (row_ok && c + 8 <= lim && ((uintptr_t)q & 15) == 0) {
        v = *reinterpret_cast<const bf16x8 *>(q);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (row_ok && c + i < lim) ? q[i] : zero;
    }
    return v;
}

template <bool TA, bool TB>
__device__ __forceinline__ void stage(const GemmArgs &g, int member, int m0, int n0, int k0, int ke,
                                      __bf16 (*As)[LDSK], __bf16 (*Bs)[LDSK])
{
    const int t = threadIdx.x;
    const __bf16 *A = g.A + member * g.sA;
    const __bf16 *B = g.B + member * g.sB;
    if (!TA) {   // row r, k offset 8 (t % 4): eight k of one row
        const int r = t / 4, kk = (t % 4) * 8, m = m0 + r;
        const bf16x8 v = load8(A, g.lda, m, m < g.M, k0 + kk, ke);
#pragma unroll
        for (int i = 0; i < 8; ++i) As[r][kk + i] = v[i];
    } else {     // k row t / 8, m offset 8 (t % 8): eight m of one k row, stored transposed
        const int kr = t / 8, mm = (t % 8) * 8, k = k0 + kr;
        const bf16x8 v = load8(A, g.lda, k, k < ke, m0 + mm, g.M);
#pragma unroll
        for (int i = 0; i < 8; ++i) As[mm + i][kr] = v[i];
    }
    if (!TB) {
        const int r = t / 4, kk = (t % 4) * 8, n = n0 + r;
        const bf16x8 v = load8(B, g.ldb, n, n < g.N, k0 + kk, ke);
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[r][kk + i] = v[i];
    } else {
        const int kr = t / 8, nn = (t % 8) * 8, k = k0 + kr;
        const bf16x8 v = load8(B, g.ldb, k, k < ke, n0 + nn, g.N);
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[nn + i][kr] = v[i];
    }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    // rows of LDSK = 40 bf16 (80 bytes): every 16-byte fragment at k = 8 q is aligned
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][LDSK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][LDSK];
    const int members = (int)gridDim.z / g.nsp;
    const int member = (int)blockIdx.z % members, split = (int)blockIdx.z / members;
    const int kb = split * g.kc, ke = min(g.K, kb + g.kc);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
        stage<TA, TB>(g, member, m0, n0, k0, ke, As, Bs);
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + lr][lk]);
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * j + lr][lk]);
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
                    g.out_f[split * g.ssplit + member * g.so_f + o] = v;
                } else {
                    const float h = from_bf16(g.mask[member * g.smask + (int64_t)m * g.ldmask + n]);
                    const float d = h > 0.f ? v : 0.f;
                    g.out_h[member * g.so_h + o] = to_bf16(d);
                    g.out_f[member * g.so_f + o] = d;
                }
            }
        }
}

// Returns the number of K splits launched (at most `splits`).
template <bool TA, bool TB, int EPI>
static int gemm(const GemmArgs &g0, int members, hipStream_t st, int splits = 1)
{
    GemmArgs g = g0;
    g.kc = splits <= 1 ? std::max(g.K, 1) : (g.K + splits * BK - 1) / (splits * BK) * BK;
    g.nsp = std::max(1, (g.K + g.kc - 1) / g.kc);
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, members * g.nsp);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, g);
    return g.nsp;
}

// K splits of a weight-gradient GEMM (K = batch rows) with `tiles` output
// tiles per member: enough workgroups for two per compute unit of a 256-CU
// device, at least four BK steps per split, at most KSPLIT_MAX splits.  A
// function of the shapes alone, so the summation order does not depend on
// the device.
constexpr int KSPLIT_MAX = 32;
// output tiles per member of the weight-gradient GEMMs: dW1 [256][64],
// dW2 and dW3 [256][256], dW4 [16][256]
constexpr int TILES_W1 = (HID / BM) * (INP / BN), TILES_W23 = (HID / BM) * (HID / BN), TILES_W4 = HID / BN;
static int ksplit(int tiles, int members, int64_t K)
{
    const int64_t want = (512 + (int64_t)tiles * members - 1) / ((int64_t)tiles * members);
    const int64_t most = std::max<int64_t>(1, K / (4 * BK));
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, most, (int64_t)KSPLIT_MAX}));
}

// ------------------------------------------------------- small kernels --
// X0[r][k] = bf16((f - shift[k]) * scale[k]) for k < 36 (0 up to 64), with
// f = log10(max(feat, 0) * dens_scale + dens_floor) for the density features
// 12..35 when dens_floor > 0, f = feat otherwise.
constexpr int SCAL = 2 * IN + 2 * OUT + 3;   // shifts/scales, dens_scale, dens_floor, spread floor
constexpr float LOG10_2 = 0.30102999566398120f;

// The standardization as one multiply-add, identical in training and
// inference: bf16(std_in(f, a, b)) with a = scale[k] (times log10(2) for a
// density input, whose f is then log2 of its argument) and b = -shift[k]
// scale[k].  log2 is v_log_f32, the hardware's transcendental; its argument
// max(feat, 0) dens_scale + dens_floor is at least dens_floor > 0.
__device__ __forceinline__ float dens_log2(float f, float dscale, float dfloor)
{
    return __builtin_amdgcn_logf(fmaf(fmaxf(f, 0.f), dscale, dfloor));
}
__device__ __forceinline__ float std_in(float f, float a, float b) { return fmaf(f, a, b); }

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
        const float dfloor = scal[2 * IN + 2 * OUT + 1], sc = scal[IN + k];
        float a = sc;
        if (k >= 12 && dfloor > 0.f) {
            f = dens_log2(f, scal[2 * IN + 2 * OUT], dfloor);
            a = sc * LOG10_2;
        }
        v = std_in(f, a, -scal[k] * sc);
    }
    X0[i] = to_bf16(v);
}

// Loss and output gradient on one block of LOSS_ROWS rows of one member:
//   T'[r][o] = (target[r][o] - out_shift[o]) / out_scale[o]
//   dY[r][o] = 2 (Y[r][o] - T'[r][o]) / (n 12) (0 in the padding columns)
// in f32 and bf16, and the block's sum of (Y - T')^2 in fp64 into
// lpart[member][block]; k_loss_fin turns the block sums into the mean.
constexpr int LOSS_ROWS = 64;
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ Y, int64_t sY, const float *__restrict__ target,
                                              int64_t n, const float *__restrict__ scal, float *__restrict__ dYf,
                                              __bf16 *__restrict__ dYh, int64_t sdY, double *__restrict__ lpart,
                                              int64_t slp)
{
    __shared__ double red[256];
    const int member = blockIdx.y;
    const float *Ym = Y + member * sY;
    double acc = 0.0;
    const float inv = 2.f / (float)(n * OUT);
    const int64_t i0 = (int64_t)blockIdx.x * LOSS_ROWS * OUTP, i1 = min(i0 + LOSS_ROWS * OUTP, n * OUTP);
#pragma unroll
    for (int k = 0; k < LOSS_ROWS * OUTP / 256; ++k) {
        const int64_t i = i0 + threadIdx.x + 256 * k;
        if (i >= i1) break;
        const int64_t r = i / OUTP;
        const int o = (int)(i % OUTP);
        float d = 0.f;
        if (o < OUT) {
            const float tt = (target[r * OUT + o] - scal[2 * IN + o]) / scal[2 * IN + OUT + o];
            const float e = Ym[i] - tt;
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
    if (threadIdx.x == 0) lpart[member * slp + blockIdx.x] = red[0];
}

// Per-member loss = (sum of the nb block sums) / (n OUT); lanes take blocks
// lane, lane + 64, ... in order, then a fixed tree adds the 64 lanes.
__global__ __launch_bounds__(64) void k_loss_fin(const double *__restrict__ lpart, int64_t slp, int nb, int64_t n,
                                                 float *__restrict__ loss_out)
{
    __shared__ double red[64];
    const int member = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) s += lpart[member * slp + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_out[member] = (float)(red[0] / (double)(n * OUT));
}

// Column sums (bias gradients): out[member][c] = sum_r G[member][r][c], in
// two passes so that the whole device takes part.  k_colsum_part: workgroup
// = 64 columns x 4 row lanes over one block of CS_ROWS rows; lane l adds rows
// l, l + 4, ... of the block in order, the 4 lanes are added in a fixed order
// into part[member][block][c].  k_colsum_fin then adds the blocks of each
// column: lane l takes blocks l, l + 4, ... in order, again 4 lanes in a
// fixed order.  The result depends on n only, not on the launch.
constexpr int CS_ROWS = 64;
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ G, int64_t sG, int64_t n, int ld,
                                                     int ncols, float *__restrict__ part, int64_t spm)
{
    __shared__ float p4[4][64];
    const int member = blockIdx.y;
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.z * CS_ROWS;
    const float *g = G + member * sG;
    float s = 0.f;
    if (c < ncols) {
        float v[CS_ROWS / 4];
#pragma unroll
        for (int k = 0; k < CS_ROWS / 4; ++k) {
            const int64_t r = r0 + rl + 4 * k;
            v[k] = r < n ? g[r * ld + c] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < CS_ROWS / 4; ++k) s += v[k];
    }
    p4[rl][threadIdx.x & 63] = s;
    __syncthreads();
    if (rl == 0 && c < ncols)
        part[member * spm + blockIdx.z * (int64_t)ncols + c] =
            ((p4[0][threadIdx.x] + p4[1][threadIdx.x]) + p4[2][threadIdx.x]) + p4[3][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_colsum_fin(const float *__restrict__ part, int64_t spm, int nb, int ncols,
                                                    float *__restrict__ out, int64_t sout)
{
    __shared__ float p4[4][64];
    const int member = blockIdx.y;
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
    const float *p = part + member * spm;
    float s = 0.f;
    if (c < ncols)
        for (int b = rl; b < nb; b += 4) s += p[(int64_t)b * ncols + c];
    p4[rl][threadIdx.x & 63] = s;
    __syncthreads();
    if (rl == 0 && c < ncols)
        out[member * sout + c] = ((p4[0][threadIdx.x] + p4[1][threadIdx.x]) + p4[2][threadIdx.x]) +
                                 p4[3][threadIdx.x];
}

// Adam on the flat master parameters; gradients are read from the padded
// GEMM layouts (dW1 [256][64], dW4 [16][256], biases).
// A weight gradient is the sum of its K-split partial products, added in
// split order.
struct GradPtrs {
    const float *dW1, *dW2, *dW3, *dW4, *db1, *db2, *db3, *db4;
    int64_t s1, s2, s3, s4, sb;   // member strides
    int k1, k2, k3, k4;           // K splits of dW1 .. dW4
    int64_t ss1, ss2, ss3, ss4;   // split strides
};

__device__ __forceinline__ float split_sum(const float *q, int k, int64_t ss)
{
    float v = q[0];
    for (int s = 1; s < k; ++s) v += q[s * ss];
    return v;
}

__device__ __forceinline__ float grad_at(const GradPtrs &G, int member, int64_t p)
{
    if (p < OB1) {
        const int64_t o = p / IN, i = p % IN;
        return split_sum(G.dW1 + member * G.s1 + o * INP + i, G.k1, G.ss1);
    }
    if (p < OW2) return G.db1[member * G.sb + (p - OB1)];
    if (p < OB2) return split_sum(G.dW2 + member * G.s2 + (p - OW2), G.k2, G.ss2);
    if (p < OW3) return G.db2[member * G.sb + (p - OB2)];
    if (p < OB3) return split_sum(G.dW3 + member * G.s3 + (p - OW3), G.k3, G.ss3);
    if (p < OW4) return G.db3[member * G.sb + (p - OB3)];
    if (p < OB4) return split_sum(G.dW4 + member * G.s4 + (p - OW4), G.k4, G.ss4);
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
// spread = |population std|_2 / max(|mean|_2, spread floor), needs_dd =
// spread > tol.  A member's 12 outputs are the first three float4s of its
// 64-byte row of Y; VEC: rates rows as float4s too (16-byte aligned rates).
template <bool VEC>
__global__ __launch_bounds__(256) void k_ensemble(const float *__restrict__ Y, int64_t sY, int members, int64_t n,
                                                  const float *__restrict__ scal, float tol,
                                                  float *__restrict__ rates, float *__restrict__ spread,
                                                  uint8_t *__restrict__ needs_dd)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    float mean[OUT], var[OUT];
#pragma unroll
    for (int o = 0; o < OUT; ++o) mean[o] = var[o] = 0.f;
    const float *osh = scal + 2 * IN, *osc = scal + 2 * IN + OUT;
    for (int m = 0; m < members; ++m) {
        const float4 *y = reinterpret_cast<const float4 *>(Y + m * sY + r * OUTP);
#pragma unroll
        for (int q = 0; q < OUT / 4; ++q) {
            const float4 v = y[q];
            mean[4 * q] += v.x * osc[4 * q] + osh[4 * q];
            mean[4 * q + 1] += v.y * osc[4 * q + 1] + osh[4 * q + 1];
            mean[4 * q + 2] += v.z * osc[4 * q + 2] + osh[4 * q + 2];
            mean[4 * q + 3] += v.w * osc[4 * q + 3] + osh[4 * q + 3];
        }
    }
    const float im = 1.f / members;
#pragma unroll
    for (int o = 0; o < OUT; ++o) mean[o] *= im;
    for (int m = 0; m < members; ++m) {
        const float4 *y = reinterpret_cast<const float4 *>(Y + m * sY + r * OUTP);
#pragma unroll
        for (int q = 0; q < OUT / 4; ++q) {
            const float4 v = y[q];
            const float d[4] = {v.x * osc[4 * q] + osh[4 * q] - mean[4 * q],
                                v.y * osc[4 * q + 1] + osh[4 * q + 1] - mean[4 * q + 1],
                                v.z * osc[4 * q + 2] + osh[4 * q + 2] - mean[4 * q + 2],
                                v.w * osc[4 * q + 3] + osh[4 * q + 3] - mean[4 * q + 3]};
#pragma unroll
            for (int e = 0; e < 4; ++e) var[4 * q + e] += d[e] * d[e];
        }
    }
    float s2 = 0.f, m2 = 0.f;
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
        s2 += var[o] * im;
        m2 += mean[o] * mean[o];
    }
    if (VEC) {
        float4 *ro = reinterpret_cast<float4 *>(rates + r * OUT);
#pragma unroll
        for (int q = 0; q < OUT / 4; ++q) ro[q] = float4{mean[4 * q], mean[4 * q + 1], mean[4 * q + 2], mean[4 * q + 3]};
    } else {
#pragma unroll
        for (int o = 0; o < OUT; ++o) rates[r * OUT + o] = mean[o];
    }
    const float sp = sqrtf(s2) / fmaxf(sqrtf(m2), scal[2 * IN + 2 * OUT + 2]);
    spread[r] = sp;
    needs_dd[r] = sp > tol ? 1 : 0;
}

// ------------------------------------------------- fused inference kernel --
// A persistent workgroup of four waves carries tiles of IP = 128 points of
// one member (blockIdx.y) through all four layers; workgroup x of G takes the
// tiles x, x + G, ...  The hidden-layer products are taken transposed,
// out^T = W x^T, on v_mfma_f32_32x32x16_bf16: the weights are the A operand
// (32 output features x 16 inputs per tile), the activations the B operand
// (16 inputs x 32 points).  Operand layout of that instruction: lane l holds
// row (A) or column (B) l % 32 and the eight k values 8 (l / 32) .. +7; the
// accumulator of lane l holds column (point) l % 32 and the 16 rows
// (features) 8 (i / 4) + 4 (l / 32) + (i % 4), i = 0..15.
//
// * Weights stay in registers: wave w computes the output features 64 w ..
//   64 w + 63 (two 32-row tiles) of every hidden layer for all the tile's
//   points, so it holds its 2 x 16 weight fragments of a layer (128 VGPRs)
//   and, as soon as a K step's fragments have been used, loads the next
//   layer's fragments for that K step into them: each layer's weights arrive
//   while the previous layer computes, and layer 2's of the next tile while
//   layer 3 and the output layer compute.  Layer 1's 24 registers stay.
// * Activations go through LDS in the B-operand layout [K step][point tile]
//   [lane][8 bf16] (128 KB for two buffers): every wave reads each 16-byte
//   fragment once per layer, 64 B per clock per CU at the matrix cores' rate.
// * No data movement between layers beyond that: a lane's accumulator holds
//   16 features of one point, exactly the 8 + 8 bf16 a lane supplies as the
//   B operand of two K steps of the next layer, provided the next layer's
//   weight columns are stored in the matching order.  So the layer inputs of
//   layers 2-4 use the K order
//     K step t, lane half h, slot s  <->  input 32 (t / 2) + 16 (t % 2) + 8 (s / 4) + 4 h + (s % 4)
//   (the sum over K does not depend on the order), and k_refresh_infer
//   writes the weights in it; layer 1 reads the 36 inputs in natural order,
//   padded to 48.
// * The bias enters as the accumulator's initial value (the C operand of a
//   layer's first K step); the epilogue is conversion to bf16 and ReLU only.
// * The output layer (12 outputs padded to 16) runs on
//   v_mfma_f32_16x16x32_bf16, wave w taking point tile w as two halves of 16
//   points.
// * The next tile's inputs are loaded into registers during layer 2 and
//   standardized into an LDS buffer of their own during layer 3.
constexpr int IP = 128;                  // points per tile
constexpr int IWAVES = 4;
constexpr int IK1 = 3;                   // K steps of 16 of the first layer (36 inputs)
constexpr int IKS = HID / 16;            // K steps of 16 of layers 2 and 3
constexpr int IK4 = HID / 32;            // K steps of 32 of the output layer
constexpr int IMT = HID / 32 / IWAVES;   // 32-row tiles per wave in the hidden layers (2)
constexpr int INT = IP / 32;             // point tiles (4)
// bf16 fragments of one member's inference weights, per layer
constexpr int64_t WI1 = (int64_t)IWAVES * IK1 * IMT * 64 * 8;
constexpr int64_t WI2 = (int64_t)IWAVES * IKS * IMT * 64 * 8;
constexpr int64_t WI4 = (int64_t)IK4 * 64 * 8;
constexpr int64_t WI_PER = WI1 + 2 * WI2 + WI4;
static_assert(WI2 == (int64_t)HID * HID, "hidden-layer fragments cover the matrix");
static_assert(WI4 == (int64_t)OUTP * HID, "output fragments cover the padded rows");
static_assert(IK4 <= IKS, "output fragments fit in the hidden-layer weight registers");

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Input index of slot s in lane half h of K step t, for layers 2-4.
__host__ __device__ __forceinline__ int perm_k(int t, int h, int s)
{
    return 32 * (t / 2) + 16 * (t % 2) + 8 * (s / 4) + 4 * h + (s % 4);
}

// Inference weight fragments from the float32 master weights: element e of
// the member's copy, laid out [wave][K step][row tile][lane][slot] (layers
// 1-3; row = 64 wave + 32 tile + lane % 32) and [K step of 32][lane][slot]
// (layer 4, the A operand of v_mfma_f32_16x16x32_bf16: row lane % 16, k
// values 8 (lane / 16) + slot, which are the B fragments of K steps
// 2 T + (lane / 32) and lane half (lane / 16) % 2 of the 32 x 32 layout; rows
// 12..15 zero).
__global__ void k_refresh_infer(const float *__restrict__ w, int members, __bf16 *__restrict__ Wi)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= members * WI_PER) return;
    const int member = (int)(i / WI_PER);
    int64_t e = i % WI_PER;
    const float *wm = w + member * P;
    float v = 0.f;
    if (e < WI1 + 2 * WI2) {
        int layer = 1, T = IK1;
        int64_t base = 0;
        if (e >= WI1) {
            layer = e < WI1 + WI2 ? 2 : 3;
            base = layer == 2 ? WI1 : WI1 + WI2;
            T = IKS;
        }
        int64_t q = e - base;
        const int s = (int)(q % 8); q /= 8;
        const int lane = (int)(q % 64); q /= 64;
        const int jj = (int)(q % IMT); q /= IMT;
        const int t = (int)(q % T); q /= T;
        const int wv = (int)q;
        const int row = 64 * wv + 32 * jj + lane % 32, h = lane / 32;
        if (layer == 1) {
            const int k = 16 * t + 8 * h + s;
            v = k < IN ? wm[OW1 + row * IN + k] : 0.f;
        } else {
            v = wm[(layer == 2 ? OW2 : OW3) + row * HID + perm_k(t, h, s)];
        }
    } else {
        int64_t q = e - (WI1 + 2 * WI2);
        const int s = (int)(q % 8); q /= 8;
        const int lane = (int)(q % 64); q /= 64;
        const int T = (int)q;
        const int o = lane % 16, c = lane / 16;
        v = o < OUT ? wm[OW4 + o * HID + perm_k(2 * T + c / 2, c % 2, s)] : 0.f;
    }
    Wi[i] = to_bf16(v);
}

// Fragment f (1 KB) of the weight block starting at element `block` of a
// member's fragments, through a buffer descriptor of them (scalar registers):
// the lane's byte offset 16 lane is the one vector register all these loads
// share, the block and fragment offset a scalar one.
typedef __attribute__((address_space(3))) bf16x8 lds_frag;

// The LDS address of p as a base register of its own: the empty asm hides
// the constant part from the compiler, so that accesses p[c] take c as the
// instruction's offset (up to 64 KB) instead of one address add per access.
__device__ __forceinline__ lds_frag *lds_base(bf16x8 *p)
{
    unsigned a = (unsigned)(uintptr_t)(lds_frag *)p;
    asm volatile("" : "+v"(a));
    return (lds_frag *)(uintptr_t)a;
}

__device__ __forceinline__ bf16x8 ldfrag(__amdgpu_buffer_rsrc_t rs, int block, int f, unsigned lane16)
{
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane16, 2 * (block + 512 * f), 0));
}

// The bias of a hidden layer in the accumulator layout of row tile J:
// element i of lane half h is feature 32 J + 8 (i / 4) + 4 h + i % 4.
__device__ __forceinline__ void load_bias(f32x16 &bc, const float *bias, int J, int h)
{
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 b = *reinterpret_cast<const float4 *>(bias + 32 * J + 8 * g + 4 * h);
        bc[4 * g] = b.x;
        bc[4 * g + 1] = b.y;
        bc[4 * g + 2] = b.z;
        bc[4 * g + 3] = b.w;
    }
}

// bf16(max(a, 0)), bf16(max(b, 0)) as one packed pair: rounded to bf16 first,
// then an integer max with 0 clears the negative values (sign bit set, so
// negative as int16).  Rounding is monotonic and keeps the sign, so this is
// the same pair (a negative zero becomes +0).
__device__ __forceinline__ unsigned relu_pk(float a, float b)
{
    const bf16x2 p = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const s16x2 q = __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), s16x2{0, 0});
    return __builtin_bit_cast(unsigned, q);
}

// Unit u (0..15) of the epilogue of one phase's accumulators ga[jj][i]
// (point tile 2 gph + i): features 32 J + 8 g + 4 h + e, J = J0 + jj, of
// accumulator a = u / 4 (jj = a / 2, i = a % 2), register group g = u % 4:
// ReLU and bf16, collected in frag; groups 0-1 form the B fragment of the
// next layer's K step 2 J and groups 2-3 that of K step 2 J + 1, each
// written to LDS once complete.
// dst: the fragment of K step 2 J0, point tile 2 gph and this lane.
__device__ __forceinline__ void epi_unit(const f32x16 (&ga)[IMT][2], int u, lds_frag *dst, u32x4 &frag)
{
    const int a = u / 4, jj = a / 2, i = a % 2, g = u % 4;
    frag[2 * (g % 2)] = relu_pk(ga[jj][i][4 * g], ga[jj][i][4 * g + 1]);
    frag[2 * (g % 2) + 1] = relu_pk(ga[jj][i][4 * g + 2], ga[jj][i][4 * g + 3]);
    if (g % 2 == 1) dst[((2 * jj + g / 2) * INT + i) * 64] = __builtin_bit_cast(bf16x8, frag);
}

// One phase of a layer: its NK K steps for point tiles 2 ph and 2 ph + 1 into
// acc, starting from the bias bc.  Every step, in this order (kept by a
// scheduling barrier): the LDS reads of the next step's B fragments, this
// step's four MFMAs, 16 / NK units of the guest epilogue (GUEST: the other
// phase's accumulators ga, of this or the previous layer; VALU work that runs
// while the matrix core works), and loads into the weight registers the step
// has used:
//   NEXT = 1: the next hidden layer's fragments of this step (both row tiles,
//             from block wn of the descriptor rs);
//   NEXT = 2: row tile 1 <- layer 2 (block wn2); row tile 0 <- the output
//             layer's fragment t (block wn) for t < IK4, layer 2 after that.
// At the last step, bc <- the bias of the next phase (nbias), which its step
// 0 reads.  extra(t) runs after the step's epilogue units (more VALU work
// under the MFMAs).
struct NoExtra {
    __device__ void operator()(int) const {}
};
template <int NK, bool GUEST, int NEXT, int NW, class Extra = NoExtra>
__device__ __forceinline__ void run_phase(bf16x8 (&Wr)[NW][IMT], bf16x8 (*src)[INT][64], int ph, int lane,
                                          f32x16 (&acc)[IMT][2], f32x16 (&bc)[IMT], const float *nbias,
                                          const f32x16 (&ga)[IMT][2], bf16x8 (*gdst)[INT][64], int gph, int J0,
                                          int h, __amdgpu_buffer_rsrc_t rs, int wn, int wn2,
                                          const Extra &extra = Extra())
{
    bf16x8 b[NK][2];
    u32x4 frag{};
    lds_frag *sb = lds_base(&src[0][2 * ph][lane]);
    lds_frag *db = GUEST ? lds_base(&gdst[2 * J0][2 * gph][lane]) : nullptr;
    b[0][0] = sb[0];
    b[0][1] = sb[64];
#pragma unroll
    for (int t = 0; t < NK; ++t) {
        if (t + 1 < NK) {
            b[t + 1][0] = sb[(t + 1) * INT * 64];
            b[t + 1][1] = sb[(t + 1) * INT * 64 + 64];
        }
#pragma unroll
        for (int jj = 0; jj < IMT; ++jj)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                acc[jj][i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wr[t][jj], b[t][i], t == 0 ? bc[jj] : acc[jj][i],
                                                                      0, 0, 0);
        if (GUEST) {   // units t 16 / NK .. (t + 1) 16 / NK - 1 of the guest epilogue
#pragma unroll
            for (int u = t * 16 / NK; u < (t + 1) * 16 / NK; ++u) epi_unit(ga, u, db, frag);
        }
        extra(t);
        if (t == NK - 1) {
#pragma unroll
            for (int jj = 0; jj < IMT; ++jj) load_bias(bc[jj], nbias, J0 + jj, h);
        }
        if (NEXT == 1) {
#pragma unroll
            for (int jj = 0; jj < IMT; ++jj) Wr[t][jj] = ldfrag(rs, wn, t * IMT + jj, 16u * lane);
        } else if (NEXT == 2) {
            Wr[t][1] = ldfrag(rs, wn2, t * IMT + 1, 16u * lane);
            Wr[t][0] = t < IK4 ? ldfrag(rs, wn, t, 16u * lane) : ldfrag(rs, wn2, t * IMT, 16u * lane);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Inputs of one tile, loaded during the previous tile: thread tid takes point
// p = tid % IP of the tile and the groups of eight inputs g = g0, g0 + 2,
// g0 + 4 (g0 = tid / IP): group g holds inputs 8 g .. 8 g + 7 (group 4:
// 32..35 and padding; group 5: padding only).  Two float4s per group (one for
// group 4); a row of 36 floats is nine float4s.  Rows at or beyond n read row
// n - 1 instead (their outputs are not stored); threads with g0 = 1 read a
// fifth float4 of their own row that they do not use.
__device__ __forceinline__ void load_inputs(float4 (&fv)[5], const float4 *__restrict__ f4, int64_t row, int64_t n,
                                            int g0)
{
    const float4 *q = f4 + (row < n ? row : n - 1) * 9 + 2 * g0;
    fv[0] = q[0];
    fv[1] = q[1];
    fv[2] = q[4];
    fv[3] = q[5];
    fv[4] = q[8 - 8 * g0];
}

// Group G of the point's inputs, standardized (std_in with the coefficients
// a = coef[k], b = coef[IN + k]), to LDS as one bf16 fragment: dst is the
// fragment of group 0 of the point (K step 0, lane p % 32 of point tile
// p / 32); group G is K step G / 2, lane half G % 2.  Inputs 36..47 are zero.
template <int G>
__device__ __forceinline__ void scatter_group(float4 f0, float4 f1, lds_frag *dst, const float *coef, bool dlog,
                                              float dscale, float dfloor)
{
    bf16x8 o{};
    if (G < 5) {
        const float v[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
        if (dlog && G >= 1) {   // groups holding density inputs (k >= 12)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * G + e;
                if (k < IN) o[e] = to_bf16(std_in(k >= 12 ? dens_log2(v[e], dscale, dfloor) : v[e], coef[k], coef[IN + k]));
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * G + e;
                if (k < IN) o[e] = to_bf16(std_in(v[e], coef[k], coef[IN + k]));
            }
        }
    }
    dst[(G / 2) * INT * 64 + 32 * (G % 2)] = o;
}

// Group j (0..2) of this thread's inputs: g = g0 + 2 j.
__device__ __forceinline__ void scatter_item(int j, int g0, const float4 (&fv)[5], lds_frag *dst, const float *coef,
                                             bool dlog, float dscale, float dfloor)
{
    const float4 z = {0.f, 0.f, 0.f, 0.f};
    if (g0 == 0) {
        if (j == 0) scatter_group<0>(fv[0], fv[1], dst, coef, dlog, dscale, dfloor);
        if (j == 1) scatter_group<2>(fv[2], fv[3], dst, coef, dlog, dscale, dfloor);
        if (j == 2) scatter_group<4>(fv[4], z, dst, coef, dlog, dscale, dfloor);
    } else {
        if (j == 0) scatter_group<1>(fv[0], fv[1], dst, coef, dlog, dscale, dfloor);
        if (j == 1) scatter_group<3>(fv[2], fv[3], dst, coef, dlog, dscale, dfloor);
        if (j == 2) scatter_group<5>(z, z, dst, coef, dlog, dscale, dfloor);
    }
}

// The scatter of the next tile's inputs as extra work of a layer-3 phase:
// items 0 and 1 at steps 5 and 11 of the first phase, item 2 at step 5 of
// the second.
struct ScatterExtra {
    int first_item, g0;
    const float4 (&fv)[5];
    lds_frag *dst;
    const float *coef;
    bool dlog;
    float dscale, dfloor;
    __device__ void operator()(int t) const
    {
        if (t == 5) scatter_item(first_item, g0, fv, dst, coef, dlog, dscale, dfloor);
        if (t == 11 && first_item == 0) scatter_item(1, g0, fv, dst, coef, dlog, dscale, dfloor);
    }
};

__global__ __launch_bounds__(64 * IWAVES, 1) void k_mlp_infer(const float *__restrict__ feat, int64_t n,
                                                              int ntiles, const float *__restrict__ scal,
                                                              const __bf16 *__restrict__ Wi,
                                                              const float *__restrict__ w, float *__restrict__ Y,
                                                              int64_t sY)
{
    // activations: [buffer][K step][point tile][lane] of 8 bf16
    __shared__ bf16x8 act[2][IKS][INT][64];
    // the standardized inputs of a tile, layer 1's B operand (12 KB)
    __shared__ bf16x8 xin[IK1][INT][64];
    // the biases of layers 1-3 and of the output layer (padded to 16)
    __shared__ __attribute__((aligned(16))) float bias_s[3 * HID + OUTP];
    // standardization coefficients a[k], b[k] (std_in)
    __shared__ __attribute__((aligned(16))) float coef_s[2 * IN];
    static_assert(HID == 64 * IWAVES, "one bias of each layer per thread");
    static_assert(IP == 128 && 64 * IWAVES == 2 * IP, "two threads per point for the inputs");
    const int member = blockIdx.y, G = gridDim.x;
    const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wave
    const unsigned lane16 = 16u * lane;
    const int p_in = tid % IP, g0 = __builtin_amdgcn_readfirstlane(tid / IP);   // uniform in the wave
    const __bf16 *wi = Wi + member * WI_PER;
    const float *wm = w + member * P;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16 *>(wi), 0,
                                                                         (int)(2 * WI_PER), 0x00020000);
    // element offsets of this wave's weight blocks of layers 1-3 and of the output layer's
    const int w1 = (int)(wv * IK1 * IMT * 512);
    const int w2 = (int)(WI1 + wv * IKS * IMT * 512), w3 = (int)(WI1 + WI2 + wv * IKS * IMT * 512);
    const int w4 = (int)(WI1 + 2 * WI2);
    const float4 *f4 = reinterpret_cast<const float4 *>(feat);
    const float dfloor = scal[2 * IN + 2 * OUT + 1], dscale = scal[2 * IN + 2 * OUT];
    const bool dlog = dfloor > 0.f;
    bf16x8 W1r[IK1][IMT], Wr[IKS][IMT];   // weight fragments in registers (layer 1; layers 2-4)
    float4 fv[5];                         // the next tile's inputs
    // Start: the first tile's inputs, the standardization coefficients and
    // the biases to LDS; then the weights of layers 1 and 2 (arriving while
    // the inputs are standardized).
    int tile = blockIdx.x;
    load_inputs(fv, f4, (int64_t)tile * IP + p_in, n, g0);
    float ca = 0.f, cb = 0.f;
    if (tid < IN) {
        const float sh = scal[tid], sc = scal[IN + tid];
        ca = tid >= 12 && dlog ? sc * LOG10_2 : sc;
        cb = -sh * sc;
    }
    const float bl1 = wm[OB1 + tid], bl2 = wm[OB2 + tid], bl3 = wm[OB3 + tid];
    const float bl4 = tid < OUT ? wm[OB4 + tid] : 0.f;
    if (tid < IN) {
        coef_s[tid] = ca;
        coef_s[IN + tid] = cb;
    }
    bias_s[tid] = bl1;
    bias_s[HID + tid] = bl2;
    bias_s[2 * HID + tid] = bl3;
    if (tid < OUTP) bias_s[3 * HID + tid] = bl4;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < IK1; ++t)
#pragma unroll
        for (int jj = 0; jj < IMT; ++jj) W1r[t][jj] = ldfrag(rs, w1, t * IMT + jj, lane16);
#pragma unroll
    for (int t = 0; t < IKS; ++t)
#pragma unroll
        for (int jj = 0; jj < IMT; ++jj) Wr[t][jj] = ldfrag(rs, w2, t * IMT + jj, lane16);
    lds_frag *xdst = lds_base(&xin[0][p_in / 32][p_in % 32]);   // this thread's group-0 fragment
#pragma unroll
    for (int j = 0; j < 3; ++j) scatter_item(j, g0, fv, xdst, coef_s, dlog, dscale, dfloor);
    f32x16 bc[IMT];   // the bias of the layer being computed, in accumulator layout
    const int J0 = IMT * wv;
#pragma unroll
    for (int jj = 0; jj < IMT; ++jj) load_bias(bc[jj], bias_s, J0 + jj, h);
    __syncthreads();
    // Per tile, layers 1-3 in two phases each (point tiles 0-1, then 2-3),
    // one barrier between phases.  Layer l + 1's phase p needs only layer l's
    // phase-p outputs, so each phase's epilogue runs inside the next phase:
    //   L1.0 | L1.1 + epi L1.0 | bar | L2.0 + epi L1.1 | bar | L2.1 + epi L2.0 | bar
    //   L3.0 + epi L2.1 | bar | L3.1 + epi L3.0, epi L3.1 | bar | output layer | bar
    // Buffers: layer 1 reads xin and writes act 1, layer 2 reads 1 and writes
    // 0, layer 3 reads 0 and writes 1, the output layer reads 1.  An epilogue
    // writes point tiles of its own phase only, which no wave reads until the
    // next barrier, and the tiles it overwrites were last read two barriers
    // earlier.  The next tile's inputs are loaded during layer 2 and written
    // to xin during layer 3 (layer 1 has read xin two barriers before).
    f32x16 acc[2][IMT][2];   // [phase][row tile][point tile within the phase]
    for (; tile < ntiles; tile += G) {
        run_phase<IK1, false, 0>(W1r, xin, 0, lane, acc[0], bc, bias_s, acc[1], act[1], 1, J0, h, rs, 0, 0);
        run_phase<IK1, true, 0>(W1r, xin, 1, lane, acc[1], bc, bias_s + HID, acc[0], act[1], 0, J0, h, rs, 0, 0);
        __syncthreads();
        // the next tile's inputs, two phases ahead of their standardization;
        // loaded after the last tile too (rows clamped to n - 1), so that the
        // waits for the weights can count the loads issued after them exactly
        load_inputs(fv, f4, (int64_t)(tile + G) * IP + p_in, n, g0);
        run_phase<IKS, true, 0>(Wr, act[1], 0, lane, acc[0], bc, bias_s + HID, acc[1], act[1], 1, J0, h, rs, 0, 0);
        __syncthreads();
        run_phase<IKS, true, 1>(Wr, act[1], 1, lane, acc[1], bc, bias_s + 2 * HID, acc[0], act[0], 0, J0, h, rs,
                                w3, 0);
        __syncthreads();
        // (after the last tile the scatter writes stale inputs that are never read)
        run_phase<IKS, true, 0>(Wr, act[0], 0, lane, acc[0], bc, bias_s + 2 * HID, acc[1], act[0], 1, J0, h, rs, 0,
                                0, ScatterExtra{0, g0, fv, xdst, coef_s, dlog, dscale, dfloor});
        __syncthreads();
        run_phase<IKS, true, 2>(Wr, act[0], 1, lane, acc[1], bc, bias_s, acc[0], act[1], 0, J0, h, rs, w4, w2,
                                ScatterExtra{2, g0, fv, xdst, coef_s, dlog, dscale, dfloor});
        {
            u32x4 frag{};
            lds_frag *db = lds_base(&act[1][2 * J0][2][lane]);
#pragma unroll
            for (int u = 0; u < 16; ++u) epi_unit(acc[1], u, db, frag);
        }
        __syncthreads();
        // ---- output layer: wave wv takes point tile wv (reads buffer 1) as
        // two halves of 16 points on v_mfma_f32_16x16x32_bf16; lane l reads
        // the fragment of K step 2 T + l / 32, lane half (l / 16) % 2
        {
            const int c = lane >> 4;
            lds_frag *ob = lds_base(&act[1][c >> 1][wv][32 * (c & 1) + (lane & 15)]);
            f32x4 o0 = {}, o1 = {};
            bf16x8 b[IK4][2];
#pragma unroll
            for (int T = 0; T < 2; ++T) {
                b[T][0] = ob[2 * T * INT * 64];
                b[T][1] = ob[2 * T * INT * 64 + 16];
            }
#pragma unroll
            for (int T = 0; T < IK4; ++T) {
                if (T + 2 < IK4) {
                    b[T + 2][0] = ob[2 * (T + 2) * INT * 64];
                    b[T + 2][1] = ob[2 * (T + 2) * INT * 64 + 16];
                }
                o0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wr[T][0], b[T][0], o0, 0, 0, 0);
                o1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wr[T][0], b[T][1], o1, 0, 0, 0);
                Wr[T][0] = ldfrag(rs, w2, T * IMT, lane16);   // (after the last tile: unused)
                __builtin_amdgcn_sched_barrier(0);
            }
            // accumulator of lane l: point l % 16 of the half, outputs 4 c .. 4 c + 3
            const float4 bb = *reinterpret_cast<const float4 *>(bias_s + 3 * HID + 4 * c);
            const int64_t r = (int64_t)tile * IP + 32 * wv + (lane & 15);
            float *y = Y + member * sY + r * OUTP + 4 * c;
            if (r < n) *reinterpret_cast<float4 *>(y) = float4{o0[0] + bb.x, o0[1] + bb.y, o0[2] + bb.z, o0[3] + bb.w};
            if (r + 16 < n)
                *reinterpret_cast<float4 *>(y + 16 * OUTP) =
                    float4{o1[0] + bb.x, o1[1] + bb.y, o1[2] + bb.z, o1[3] + bb.w};
        }
        __syncthreads();
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
    int cus = 1;                                          // compute units of that device
    float *w = nullptr, *m1 = nullptr, *m2 = nullptr;   // [members][P]
    int64_t t = 0;                                        // Adam steps taken
    __bf16 *W1p = nullptr, *W2 = nullptr, *W3 = nullptr, *W4p = nullptr;
    __bf16 *Wi = nullptr;                                 // inference fragments [members][WI_PER]
    float *scal = nullptr;                                // device [2*36 + 2*12]
    float h_scal[SCAL];                                   // host copy
    float *dW1 = nullptr, *dW2 = nullptr, *dW3 = nullptr, *dW4 = nullptr, *db = nullptr;
    int ks[4] = {1, 1, 1, 1};                             // K splits of dW1 .. dW4 in the last backward
    // row workspace, sized for `cap` rows
    int64_t cap = 0;
    bool cap_train = false;
    __bf16 *X0 = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *dYh = nullptr;
    __bf16 *Dh[2] = {nullptr, nullptr};
    float *Y = nullptr, *dYf = nullptr;
    float *Df[2] = {nullptr, nullptr};
    float *part = nullptr;                                // column-sum block partials
    double *lpart = nullptr;                              // loss block partials
};

namespace {

constexpr int64_t INFER_CHUNK = 262144;   // rows per inference pass
constexpr int64_t TRAIN_MAX = 65536;

void free_rows(dd_mlp *h)
{
    void *ps[] = {h->X0, h->H1, h->H2, h->H3, h->dYh, h->Dh[0], h->Dh[1], h->Y, h->dYf, h->Df[0], h->Df[1],
                  h->part, h->lpart};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    h->X0 = h->H1 = h->H2 = h->H3 = h->dYh = h->Dh[0] = h->Dh[1] = nullptr;
    h->Y = h->dYf = h->Df[0] = h->Df[1] = h->part = nullptr;
    h->lpart = nullptr;
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
        const int64_t nb = (rows + CS_ROWS - 1) / CS_ROWS, nbl = (rows + LOSS_ROWS - 1) / LOSS_ROWS;
        if ((rc = dev_alloc((void **)&h->part, sizeof(float) * M * nb * HID))) return rc;
        if ((rc = dev_alloc((void **)&h->lpart, sizeof(double) * M * nbl))) return rc;
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
    const int64_t ti = WI_PER * h->members;
    hipLaunchKernelGGL(k_refresh_infer, dim3((unsigned)((ti + 255) / 256)), dim3(256), 0, st, h->w, h->members,
                       h->Wi);
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
    G.k1 = h->ks[0]; G.k2 = h->ks[1]; G.k3 = h->ks[2]; G.k4 = h->ks[3];
    G.ss1 = h->members * G.s1; G.ss2 = h->members * G.s2; G.ss3 = h->members * G.s3; G.ss4 = h->members * G.s4;
    return G;
}

// Two passes; part holds members x ceil(n / CS_ROWS) x ncols floats.
void colsum(const float *G, int64_t sG, int64_t n, int ld, int ncols, float *out, int members, float *part,
            hipStream_t st)
{
    const int nb = (int)((n + CS_ROWS - 1) / CS_ROWS);
    const int64_t spm = (int64_t)nb * ncols;
    hipLaunchKernelGGL(k_colsum_part, dim3((ncols + 63) / 64, members, nb), dim3(256), 0, st, G, sG, n, ld, ncols,
                       part, spm);
    hipLaunchKernelGGL(k_colsum_fin, dim3((ncols + 63) / 64, members), dim3(256), 0, st, part, spm, nb, ncols, out,
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
    const int nbl = (int)((n + LOSS_ROWS - 1) / LOSS_ROWS);
    hipLaunchKernelGGL(k_loss, dim3(nbl, M), dim3(256), 0, st, h->Y, n * OUTP, target, n, h->scal, h->dYf,
                       h->dYh, n * OUTP, h->lpart, (int64_t)nbl);
    if (loss_out)
        hipLaunchKernelGGL(k_loss_fin, dim3(M), dim3(64), 0, st, h->lpart, (int64_t)nbl, nbl, n, loss_out);
    GemmArgs g{};
    // output layer: dW4 [16][256] = dY^T H3, db4 = colsum(dY)
    g.A = h->dYh; g.lda = OUTP; g.sA = n * OUTP;
    g.B = h->H3; g.ldb = HID; g.sB = n * HID;
    g.M = OUTP; g.N = HID; g.K = (int)n;
    g.out_f = h->dW4; g.ldo = HID; g.so_f = (int64_t)OUTP * HID; g.ssplit = M * g.so_f;
    h->ks[3] = gemm<true, true, EPI_F32>(g, M, st, ksplit(TILES_W4, M, n));
    colsum(h->dYf, n * OUTP, n, OUTP, OUTP, h->db + 3 * HID, M, h->part, st);
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
        g.out_f = dWs[l]; g.ldo = HID; g.so_f = (int64_t)HID * HID; g.ssplit = M * g.so_f;
        h->ks[2 - l] = gemm<true, true, EPI_F32>(g, M, st, ksplit(TILES_W23, M, n));
        colsum(h->Df[cur], n * HID, n, HID, HID, h->db + dbo[l], M, h->part, st);
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
    g.out_f = h->dW1; g.ldo = INP; g.so_f = (int64_t)HID * INP; g.ssplit = M * g.so_f;
    h->ks[0] = gemm<true, true, EPI_F32>(g, M, st, ksplit(TILES_W1, M, n));
    colsum(h->Df[cur], n * HID, n, HID, HID, h->db, M, h->part, st);
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
    if (!rc && hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess)
        rc = set_error(DD_EHIP, "hipDeviceGetAttribute failed");
    const int64_t M = n_members;
    if (!rc) rc = dev_alloc((void **)&h->w, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->m1, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->m2, sizeof(float) * M * P);
    if (!rc) rc = dev_alloc((void **)&h->W1p, sizeof(__bf16) * M * HID * INP);
    if (!rc) rc = dev_alloc((void **)&h->W2, sizeof(__bf16) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->W3, sizeof(__bf16) * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->W4p, sizeof(__bf16) * M * OUTP * HID);
    if (!rc) rc = dev_alloc((void **)&h->Wi, sizeof(__bf16) * M * WI_PER);
    if (!rc) rc = dev_alloc((void **)&h->scal, sizeof(float) * SCAL);
    // weight gradients hold one partial product per K split
    const int64_t k1 = ksplit(TILES_W1, n_members, TRAIN_MAX), k23 = ksplit(TILES_W23, n_members, TRAIN_MAX),
                  k4 = ksplit(TILES_W4, n_members, TRAIN_MAX);
    if (!rc) rc = dev_alloc((void **)&h->dW1, sizeof(float) * k1 * M * HID * INP);
    if (!rc) rc = dev_alloc((void **)&h->dW2, sizeof(float) * k23 * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->dW3, sizeof(float) * k23 * M * HID * HID);
    if (!rc) rc = dev_alloc((void **)&h->dW4, sizeof(float) * k4 * M * OUTP * HID);
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
    void *ps[] = {h->w, h->m1, h->m2, h->W1p, h->W2, h->W3, h->W4p, h->Wi, h->scal, h->dW1, h->dW2, h->dW3, h->dW4,
                  h->db};
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

// ---------------------------------------------------------- persistence --
// File layout (host byte order, which is little-endian on every ROCm host):
//   char   magic[8]           "DDMLP\0\0\1" (the last byte is the version)
//   int32  members, in, hidden, out, params per member, scaling entries
//   int64  Adam steps taken
//   float  scaling[SCAL]      shifts, scales, dens_scale, dens_floor, spread floor
//   float  w[members][P], m1[members][P], m2[members][P]
//   uint64 FNV-1a hash of every byte before it
namespace {

constexpr char MAGIC[8] = {'D', 'D', 'M', 'L', 'P', 0, 0, 1};
constexpr int HDR_INTS = 6;

struct Fnv {
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const void *p, size_t n)
    {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    }
};

struct File {
    FILE *f = nullptr;
    ~File()
    {
        if (f) std::fclose(f);
    }
};

bool put(FILE *f, Fnv &fnv, const void *p, size_t n)
{
    fnv.add(p, n);
    return std::fwrite(p, 1, n, f) == n;
}

bool get(FILE *f, Fnv &fnv, void *p, size_t n)
{
    if (std::fread(p, 1, n, f) != n) return false;
    fnv.add(p, n);
    return true;
}

}  // namespace

extern "C" int dd_mlp_save(const dd_mlp *h, const char *path)
{
    ::dd::Range range_("dd_mlp_save");
    clear_error();
    int rc;
    if ((rc = check_model(h))) return rc;
    if (!path || !*path) return set_error(DD_EINVAL, "null or empty path");
    const int64_t MP = h->members * P;
    std::vector<float> buf((size_t)(3 * MP));
    DD_HIP(hipDeviceSynchronize());
    DD_HIP(hipMemcpy(buf.data(), h->w, sizeof(float) * MP, hipMemcpyDeviceToHost));
    DD_HIP(hipMemcpy(buf.data() + MP, h->m1, sizeof(float) * MP, hipMemcpyDeviceToHost));
    DD_HIP(hipMemcpy(buf.data() + 2 * MP, h->m2, sizeof(float) * MP, hipMemcpyDeviceToHost));
    // written to a temporary name and renamed, so that a reader never sees a
    // partial file under `path`
    const std::string tmp = std::string(path) + ".tmp";
    File out;
    if (!(out.f = std::fopen(tmp.c_str(), "wb"))) return set_error(DD_EIO, "cannot open %s for writing", tmp.c_str());
    Fnv fnv;
    const int32_t hdr[HDR_INTS] = {h->members, IN, HID, OUT, (int32_t)P, SCAL};
    bool ok = put(out.f, fnv, MAGIC, sizeof MAGIC) && put(out.f, fnv, hdr, sizeof hdr) &&
              put(out.f, fnv, &h->t, sizeof h->t) && put(out.f, fnv, h->h_scal, sizeof h->h_scal) &&
              put(out.f, fnv, buf.data(), sizeof(float) * buf.size());
    const uint64_t sum = fnv.h;
    ok = ok && std::fwrite(&sum, 1, sizeof sum, out.f) == sizeof sum;
    ok = (std::fclose(out.f) == 0) && ok;
    out.f = nullptr;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return set_error(DD_EIO, "writing %s failed", path);
    }
    return DD_OK;
}

extern "C" int dd_mlp_load(const char *path, dd_mlp **out)
{
    ::dd::Range range_("dd_mlp_load");
    clear_error();
    if (!out) return set_error(DD_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (!path || !*path) return set_error(DD_EINVAL, "null or empty path");
    // the whole file is read and checked before any device call
    File in;
    if (!(in.f = std::fopen(path, "rb"))) return set_error(DD_EIO, "cannot open %s", path);
    Fnv fnv;
    char magic[8];
    int32_t hdr[HDR_INTS];
    int64_t t = 0;
    float scal[SCAL];
    if (!get(in.f, fnv, magic, sizeof magic) || std::memcmp(magic, MAGIC, sizeof magic) != 0)
        return set_error(DD_EIO, "%s is not a surrogate file of this version", path);
    if (!get(in.f, fnv, hdr, sizeof hdr)) return set_error(DD_EIO, "%s: truncated header", path);
    if (hdr[0] < 1 || hdr[0] > 8 || hdr[1] != IN || hdr[2] != HID || hdr[3] != OUT || hdr[4] != (int32_t)P ||
        hdr[5] != SCAL)
        return set_error(DD_EIO, "%s: network shape (%d members, %d-%d-%d, %d parameters, %d scaling) does not "
                                 "match this library's", path, hdr[0], hdr[1], hdr[2], hdr[3], hdr[4], hdr[5]);
    const int64_t MP = (int64_t)hdr[0] * P;
    std::vector<float> buf((size_t)(3 * MP));
    if (!get(in.f, fnv, &t, sizeof t) || !get(in.f, fnv, scal, sizeof scal) ||
        !get(in.f, fnv, buf.data(), sizeof(float) * buf.size()))
        return set_error(DD_EIO, "%s: truncated", path);
    uint64_t sum = 0;
    char extra;
    if (std::fread(&sum, 1, sizeof sum, in.f) != sizeof sum || sum != fnv.h)
        return set_error(DD_EIO, "%s: checksum mismatch (corrupted or truncated)", path);
    if (std::fread(&extra, 1, 1, in.f) != 0) return set_error(DD_EIO, "%s: trailing bytes", path);
    if (t < 0) return set_error(DD_EIO, "%s: negative Adam step count", path);
    for (float v : scal)
        if (!std::isfinite(v)) return set_error(DD_EIO, "%s: non-finite scaling value", path);
    for (float v : buf)
        if (!std::isfinite(v)) return set_error(DD_EIO, "%s: non-finite parameter or moment", path);

    dd_mlp *h = nullptr;
    int rc = dd_mlp_create(hdr[0], 0, &h);
    if (rc) return rc;
    auto fail = [&](int code) {
        dd_mlp_destroy(h);
        return code;
    };
    if (hipMemcpy(h->w, buf.data(), sizeof(float) * MP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->m1, buf.data() + MP, sizeof(float) * MP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->m2, buf.data() + 2 * MP, sizeof(float) * MP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->scal, scal, sizeof scal, hipMemcpyHostToDevice) != hipSuccess)
        return fail(set_error(DD_EHIP, "copying the loaded surrogate to the device failed"));
    std::memcpy(h->h_scal, scal, sizeof scal);
    h->t = t;
    if ((rc = refresh(h, nullptr))) return fail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return fail(set_error(DD_EHIP, "loading the surrogate failed"));
    *out = h;
    return DD_OK;
}

extern "C" int dd_mlp_info(const dd_mlp *h, int *n_members, int64_t *adam_steps)
{
    clear_error();
    if (!h) return set_error(DD_EINVAL, "null surrogate handle");
    if (n_members) *n_members = h->members;
    if (adam_steps) *adam_steps = h->t;
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
    ::dd::Range range_("dd_mlp_gradients");
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
    ::dd::Range range_("dd_mlp_train_step");
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
    ::dd::Range range_("dd_surrogate_rates");
    clear_error();
    dd_mlp *h = const_cast<dd_mlp *>(hc);   // the handle's workspace grows; the model is unchanged
    int rc;
    if ((rc = check_model(h))) return rc;
    if (n < 0) return set_error(DD_EINVAL, "n < 0");
    if (n == 0) return DD_OK;
    if (!feat || !rates || !spread || !needs_dd) return set_error(DD_EINVAL, "null array");
    if (!(spread_tol >= 0.f)) return set_error(DD_EINVAL, "spread_tol must be >= 0");
    if ((uintptr_t)feat % 16 != 0) return set_error(DD_EINVAL, "feat must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int64_t chunk = std::min<int64_t>(n, INFER_CHUNK);
    if ((rc = ensure_rows(h, chunk, false))) return rc;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t m = std::min(chunk, n - r0);
        const int ntiles = (int)((m + IP - 1) / IP);
        dim3 grid((unsigned)std::min(ntiles, std::max(1, h->cus / h->members)), h->members);
        hipLaunchKernelGGL(k_mlp_infer, grid, dim3(64 * IWAVES), 0, st, feat + r0 * IN, m, ntiles, h->scal, h->Wi,
                           h->w, h->Y, m * OUTP);
        float *ro = rates + r0 * OUT;
        if ((uintptr_t)ro % 16 == 0)
            hipLaunchKernelGGL(k_ensemble<true>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, h->Y,
                               m * OUTP, h->members, m, h->scal, spread_tol, ro, spread + r0, needs_dd + r0);
        else
            hipLaunchKernelGGL(k_ensemble<false>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, h->Y,
                               m * OUTP, h->members, m, h->scal, spread_tol, ro, spread + r0, needs_dd + r0);
    }
    DD_HIP(hipGetLastError());
    return DD_OK;
}
