// Surrogate network: n_in (<= 32) -> 4 x 256 (GELU) -> n_out (<= 16).
//
// Forward: one work-group of 8 waves per 64 rows (each wave all 64 rows x
// 32 output columns); every layer is a [64 x K] x [K x 256] product on the
// bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation). Weights are bf16; the
// activations are kept in LDS split into bf16 hi + lo parts (two MFMAs per
// tile), so the product sees the activations to ~16 significant bits. In "precise" mode the
// weights are split as well (three MFMAs: a_hi w_hi + a_lo w_hi + a_hi w_lo),
// which reproduces FP32 weights for gradient checks. Bias and GELU are fused
// into the epilogue; the layer output stays in LDS for the next layer.
//
// Training: FP32 backward (64 x 64-tiled GEMMs on the FP32 matrix cores for
// dA = dZ W and dW = dZ^T A, column sums for db), weighted MSE on normalized outputs, Adam on FP32
// master weights with refreshed bf16 copies after each step.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <random>
#include <type_traits>
#include <vector>

#include "mlp.h"
#include "runtime.h"

// Per-network outputs of the allocation-free ensemble inference. One copy per
// GPU, at that GPU's own address: host code never passes this name to a
// kernel, only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[HOM_STATIC_SCRATCH_FLOATS];

namespace hom {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int MROWS = 64;             // rows per forward work-group
constexpr int FWD_WAVES = 8;          // waves per forward work-group
constexpr int NRB = MROWS / 16;       // 16-row tiles per wave (every wave spans all rows)
constexpr int NCB = MLP_W / (16 * FWD_WAVES);  // 16-column tiles per wave
constexpr int AST = 264;              // LDS row stride of the bf16 activation tiles (16-byte aligned rows)

// erf by Abramowitz and Stegun's rational approximation 7.1.26 (Handbook of
// Mathematical Functions, 1964): erf(x) = 1 - t (a1 + t (a2 + ... + t a5))
// exp(-x^2), t = 1 / (1 + p x) for x >= 0, odd extension; absolute error
// below 1.5e-7 (2e-7 with the hardware reciprocal), about a third of the
// instructions of the library erf. The network's forward and backward passes
// both use it, so training sees one consistent activation function.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));  // v_rcp_f32, 1 ulp
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  const float e = __expf(-ax * ax);
  return copysignf(fmaf(-p * t, e, 1.0f), x);
}
__device__ __forceinline__ float gelu_prime_f(float z) {
  return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) + z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// The same approximation arranged for the forward pass: with x = z / sqrt 2,
// Phi(z) = 1 - q / 2 for z >= 0 and q / 2 below, q = p(t) t exp(-x^2), so
// GELU(z) = z Phi(z) = max(z, 0) - |z| q / 2 (no cancellation for negative z);
// the 1 / sqrt 2 and the 1 / 2 are folded into the constants.
__device__ __forceinline__ float gelu_fwd(float z) {
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.2316418883f, az, 1.0f));
  float p = fmaf(0.5307027145f, t, -0.7265760135f);
  p = fmaf(p, t, 0.7107068705f);
  p = fmaf(p, t, -0.142248368f);
  p = fmaf(p, t, 0.127414796f);
  const float e = __builtin_amdgcn_exp2f(z * z * -0.7213475204f);  // exp(-z^2 / 2)
  return fmaf(-az, p * t * e, fmaxf(z, 0.0f));
}

// bf16 weight copies in fragment order: the 16 x 32 block of output rows
// 16 cb .. 16 cb + 15 and inputs 32 s .. 32 s + 31 is one contiguous 1 KiB
// fragment, lane-major (lane = 16 (k / 8 mod 4) + output mod 16, then 8
// consecutive inputs), so a wave's B operand of one k-step is a single
// coalesced 1 KiB load. Offset of the lane's 8 values in a layer with inner
// dimension K:
__host__ __device__ __forceinline__ long long frag_offset(int cb, int s, int K, int lane) {
  return (((long long)cb * (K / 32) + s) * 64 + lane) * 8;
}

struct FwdArgs {
  const float* x;
  long long n;
  int n_in, n_out;
  const float* xmean;
  const float* xinv;
  const float* ymean;
  const float* ystd;
  const float* skip;  // G [16][MLP_GATES][32], c [16]
  const __bf16* skip_hi;  // G rounded to bf16
  const __bf16* skip_lo;  // the remainder G - hi, rounded to bf16
  int g0, g1, g2;     // gate input indices
  const __bf16* whi[MLP_LAYERS];
  const __bf16* wlo[MLP_LAYERS];
  const float* bias[MLP_LAYERS];
  float* y;      // [n][n_out] outputs in physical units (optional)
  float* yhat;   // [n][16] normalized outputs (optional)
  float* xs;     // [n][32] normalized inputs (optional, training)
  float* zs[MLP_LAYERS - 1];  // [n][256] pre-activations (optional)
  float* as[MLP_LAYERS - 1];  // [n][256] activations (optional)
};

// SAVE: keep the normalized inputs, pre-activations, activations and
// normalized outputs for the backward pass (training); inference writes y only
template <int PRECISE, bool SAVE>
__global__ void __launch_bounds__(FWD_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4))) k_mlp_fwd(FwdArgs a) {
  // The tile's activations live in LDS already split into bf16 hi + lo: each
  // value is split once, by the lane that produced it, and every wave reads
  // its MFMA fragments directly.
  __shared__ __attribute__((aligned(16))) __bf16 ahi[MROWS * AST];
  __shared__ __attribute__((aligned(16))) __bf16 alo[MROWS * AST];
  __shared__ float xin[MROWS * (MLP_IN + 1)];  // normalized inputs, kept for the skip
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const long long row0 = (long long)blockIdx.x * MROWS;
  for (int i = tid; i < MROWS * MLP_IN; i += FWD_WAVES * 64) {
    const int r = i / MLP_IN, k = i % MLP_IN;
    const long long gr = row0 + r;
    float v = 0.0f;
    if (gr < a.n && k < a.n_in) v = (a.x[gr * a.n_in + k] - a.xmean[k]) * a.xinv[k];
    const __bf16 h = (__bf16)v;
    ahi[r * AST + k] = h;
    alo[r * AST + k] = (__bf16)(v - (float)h);
    xin[r * (MLP_IN + 1) + k] = v;
    if (SAVE && gr < a.n) a.xs[gr * MLP_IN + k] = v;
  }
  __syncthreads();
  const int lrow = lane & 15;
  const int kq = (lane >> 4) * 8;
#pragma unroll 1
  for (int l = 0; l < MLP_LAYERS - 1; ++l) {
    const int K = l == 0 ? MLP_IN : MLP_W;
    const __bf16* whi = a.whi[l];
    const __bf16* wlo = a.wlo[l];
    // lane: row m = rb 16 + lrow, outputs nn0 .. nn0 + 3 of tile cb; the
    // bias enters as the first product's accumulator input
    floatx4_t bv[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      bv[cb] = *reinterpret_cast<const floatx4_t*>(a.bias[l] + wave * (16 * NCB) + cb * 16 + (lane >> 4) * 4);
    floatx4_t acc[NRB][NCB];
    bf16x8_t bh[NCB], bl[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const long long f = frag_offset(wave * NCB + cb, 0, K, lane);
      bh[cb] = *reinterpret_cast<const bf16x8_t*>(whi + f);
      if constexpr (PRECISE) bl[cb] = *reinterpret_cast<const bf16x8_t*>(wlo + f);
    }
    const auto step = [&](int k0, auto first) {
      constexpr bool FIRST = decltype(first)::value;
      bf16x8_t xh[NRB], xl[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        const int o = (rb * 16 + lrow) * AST + k0 + kq;
        xh[rb] = *reinterpret_cast<const bf16x8_t*>(ahi + o);
        xl[rb] = *reinterpret_cast<const bf16x8_t*>(alo + o);
      }
      // weights of the next k-step in flight during this step's products
      const int k1 = k0 + 32 < K ? k0 + 32 : k0;
      bf16x8_t nh[NCB], nl[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const long long f = frag_offset(wave * NCB + cb, k1 / 32, K, lane);
        nh[cb] = *reinterpret_cast<const bf16x8_t*>(whi + f);
        if constexpr (PRECISE) nl[cb] = *reinterpret_cast<const bf16x8_t*>(wlo + f);
      }
      // the transposed tile Z^T = W A^T (weights as the first operand): each
      // lane's four accumulator values are four consecutive outputs of one
      // row, stored as one 8-byte LDS write per part in the epilogue. hi and
      // lo passes over all of the wave's tiles: no product waits on the
      // previous one into the same accumulator
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          if constexpr (FIRST)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[cb], xh[rb], bv[cb], 0, 0, 0);
          else
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[cb], xh[rb], acc[rb][cb], 0, 0, 0);
        }
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[cb], xl[rb], acc[rb][cb], 0, 0, 0);
      if constexpr (PRECISE) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[cb], xh[rb], acc[rb][cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bh[cb] = nh[cb];
        if constexpr (PRECISE) bl[cb] = nl[cb];
      }
    };
    step(0, std::true_type{});
    for (int k0 = 32; k0 < K; k0 += 32) step(k0, std::false_type{});
    __syncthreads();  // all waves done reading this layer's input
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int m = rb * 16 + lrow;
        const int nn0 = wave * (16 * NCB) + cb * 16 + (lane >> 4) * 4;
        floatx4_t z, g;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          z[i] = acc[rb][cb][i];
          g[i] = gelu_fwd(z[i]);
        }
        unsigned hp[2], lp[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const bf16x2_t hh = {(__bf16)g[2 * j], (__bf16)g[2 * j + 1]};
          hp[j] = __builtin_bit_cast(unsigned, hh);
          const float h0 = __builtin_bit_cast(float, hp[j] << 16);
          const float h1 = __builtin_bit_cast(float, hp[j] & 0xffff0000u);
          const bf16x2_t ll = {(__bf16)(g[2 * j] - h0), (__bf16)(g[2 * j + 1] - h1)};
          lp[j] = __builtin_bit_cast(unsigned, ll);
        }
        *reinterpret_cast<uint2*>(ahi + m * AST + nn0) = make_uint2(hp[0], hp[1]);
        *reinterpret_cast<uint2*>(alo + m * AST + nn0) = make_uint2(lp[0], lp[1]);
        if constexpr (SAVE) {
          const long long gr = row0 + m;
          if (gr < a.n) {
            *reinterpret_cast<floatx4_t*>(a.zs[l] + gr * MLP_W + nn0) = z;
            *reinterpret_cast<floatx4_t*>(a.as[l] + gr * MLP_W + nn0) = g;
          }
        }
      }
    __syncthreads();
  }
  // output layer: each wave 16 rows x 16 outputs
  if (wave < MROWS / 16) {
    const int l = MLP_LAYERS - 1;
    const __bf16* whi = a.whi[l];
    const __bf16* wlo = a.wlo[l];
    floatx4_t acc = floatx4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < MLP_W; k0 += 32) {
      const int o = (wave * 16 + lrow) * AST + k0 + kq;
      const bf16x8_t xh = *reinterpret_cast<const bf16x8_t*>(ahi + o);
      const bf16x8_t xl = *reinterpret_cast<const bf16x8_t*>(alo + o);
      const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(whi + frag_offset(0, k0 / 32, MLP_W, lane));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, bh, acc, 0, 0, 0);
      if constexpr (PRECISE) {
        const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(wlo + frag_offset(0, k0 / 32, MLP_W, lane));
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bl, acc, 0, 0, 0);
      }
    }
    // gated cubic skip, sk = c + sum_g s_g(x) (G_g . x), on the matrix cores:
    // for every gate polynomial s_g the 16 rows x 16 outputs of G_g . x in one
    // tile whose layout matches acc (x and G split into bf16 hi + lo parts,
    // three products: about 16 significant bits)
    floatx4_t sk = floatx4_t{0.f, 0.f, 0.f, 0.f};
    if (a.y) {  // uniform over the work-group
      bf16x8_t xh, xl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float v = xin[(wave * 16 + lrow) * (MLP_IN + 1) + kq + j];
        xh[j] = (__bf16)v;
        xl[j] = (__bf16)(v - (float)xh[j]);
      }
      float sg[4][MLP_GATES];  // the gate polynomials of this lane's four rows
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float* xr = xin + (wave * 16 + (lane >> 4) * 4 + i) * (MLP_IN + 1);
        const float va = xr[a.g0], vb = xr[a.g1], vc = xr[a.g2];
        const float s[MLP_GATES] = {1.f, va, va * va, va * va * va, vb, vb * vb, vb * vb * vb,
                                    vc, vc * vc, vc * vc * vc};
#pragma unroll
        for (int gi = 0; gi < MLP_GATES; ++gi) sg[i][gi] = s[gi];
      }
      const size_t gb = (size_t)lrow * MLP_GATES * MLP_IN + kq;  // output lrow, inputs kq ..
#pragma unroll
      for (int gi = 0; gi < MLP_GATES; ++gi) {
        const bf16x8_t gh = *reinterpret_cast<const bf16x8_t*>(a.skip_hi + gb + gi * MLP_IN);
        const bf16x8_t gl = *reinterpret_cast<const bf16x8_t*>(a.skip_lo + gb + gi * MLP_IN);
        floatx4_t t = floatx4_t{0.f, 0.f, 0.f, 0.f};
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gh, t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, gh, t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gl, t, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) sk[i] += sg[i][gi] * t[i];
      }
      const float c = a.skip[MLP_OUT * MLP_GATES * MLP_IN + lrow];
#pragma unroll
      for (int i = 0; i < 4; ++i) sk[i] += c;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = wave * 16 + (lane >> 4) * 4 + i;
      const long long gr = row0 + m;
      if (gr >= a.n) continue;
      const float z = acc[i] + a.bias[l][lrow];
      if (SAVE) a.yhat[gr * MLP_OUT + lrow] = z;
      if (a.y && lrow < a.n_out) a.y[gr * a.n_out + lrow] = z * a.ystd[lrow] + a.ymean[lrow] + sk[i];
    }
  }
}

// C[M][N] = op(A) op(B) (+ beta C), row-major, FP32. op(A) = A (M x K, lda)
// or A^T (A stored K x M); op(B) = B (K x N, ldb) or B^T (B stored N x K).
// C = op(A) op(B) (+ beta C), 64 x 64 tiles. With gridDim.z > 1 the inner
// dimension is split in chunks of kc: work-group z takes rows z kc .. of A
// and B (A, B stored [k][*], the weight-gradient form) and writes its own
// partial C + z M ldc.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              float beta, int kc = 0) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  if (gridDim.z > 1) {
    const int k0 = blockIdx.z * kc;
    K = min(kc, K - k0);
    A += (long long)k0 * lda;
    B += (long long)k0 * ldb;
    C += (long long)blockIdx.z * M * ldc;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // the wave's 32 x 32 quarter of the tile
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  // FP32 matrix cores (v_mfma_f32_16x16x4_f32: exact products, FP32
  // accumulation): lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16] of a
  // 16 x 4 x 16 step and holds C rows 4 (l / 16) .. + 3 of column l % 16
  floatx4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int i = tid; i < 16 * 64; i += 256) {
      const int kk = i / 64, mm = i % 64;
      const int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < M && gk < K) va = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
      As[kk][mm] = va;
      const int gn = n0 + mm;
      float vb = 0.f;
      if (gn < N && gk < K) vb = TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn];
      Bs[kk][mm] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      float av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = As[kk][wm + t * 16 + (lane & 15)];
        bv[t] = Bs[kk][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + (lane >> 4) * 4 + r, gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          float* c = C + (long long)gm * ldc + gn;
          *c = beta == 0.f ? acc[i][j][r] : beta * *c + acc[i][j][r];
        }
      }
}

// column sums: out[j] = sum_r in[r][j], one thread per column (fixed order)
// Column sums (bias gradients) in two fixed-order stages: blocks of 64
// columns x 4 row lanes over row chunks into FP64 partials, then the chunks.
constexpr int COLSUM_CHUNK = 256;
__global__ void __launch_bounds__(256) k_colsum_part(const float* in, long long rows, int cols, double* part) {
  __shared__ double red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int lane = threadIdx.x >> 6;
  const long long r0 = (long long)blockIdx.y * COLSUM_CHUNK;
  const long long r1 = min(rows, r0 + COLSUM_CHUNK);
  double s = 0.0;
  if (c < cols)
    for (long long r = r0 + lane; r < r1; r += 4) s += in[r * cols + c];
  red[lane][threadIdx.x & 63] = s;
  __syncthreads();
  if (lane == 0 && c < cols)
    part[(long long)blockIdx.y * cols + c] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                             red[3][threadIdx.x];
}

__global__ void __launch_bounds__(256) k_colsum_final(const double* part, int chunks, int cols, float* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += part[(long long)k * cols + c];
  out[c] = (float)s;
}

// dz = da * gelu'(z)
__global__ void k_gelu_back(const float* da, const float* z, float* dz, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dz[i] = da[i] * gelu_prime_f(z[i]);
}

// weighted MSE on normalized outputs: dyhat = 2 w (yhat - t) / B, loss partials
// weighted mean squared error: output weights w [16], row weights rw [B] (or null)
__global__ void k_loss(const float* yhat, const float* t, const float* w, const float* rw, long long B, int n_out,
                       float* dy, double* part) {
  __shared__ double red[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < B * MLP_OUT) {
    const int j = (int)(i % MLP_OUT);
    float g = 0.f;
    if (j < n_out) {
      const float d = yhat[i] - t[i];
      const float wj = w[j] * (rw ? rw[i / MLP_OUT] : 1.0f);
      g = 2.0f * wj * d / (float)B;
      l = (double)wj * (double)d * (double)d / (double)B;
    }
    dy[i] = g;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, long long count, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct LayerSpans {
  long long off[MLP_LAYERS];
  int n[MLP_LAYERS], k[MLP_LAYERS];
};

// master FP32 weights -> bf16 hi / lo copies (weight matrices in fragment
// order) and the effective FP32 weights the forward pass uses (hi, or hi + lo
// in precise mode)
__global__ void k_split(const float* w, __bf16* hi, __bf16* lo, float* eff_bf, float* eff_pr, long long count,
                        LayerSpans ls) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float v = w[i];
  const __bf16 h = (__bf16)v;
  const __bf16 l = (__bf16)(v - (float)h);
  long long d = i;  // biases and padding keep their place
#pragma unroll
  for (int L = 0; L < MLP_LAYERS; ++L) {
    const long long r = i - ls.off[L];
    if (r >= 0 && r < (long long)ls.n[L] * ls.k[L]) {
      const int nn = (int)(r / ls.k[L]), k = (int)(r % ls.k[L]);
      d = ls.off[L] + frag_offset(nn >> 4, k >> 5, ls.k[L], ((k & 31) >> 3) * 16 + (nn & 15)) + (k & 7);
    }
  }
  hi[d] = h;
  lo[d] = l;
  eff_bf[i] = (float)h;
  eff_pr[i] = (float)h + (float)l;
}

__global__ void k_gather(const float* src, int cols, const int* idx, long long count, float* dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count * cols) return;
  const long long r = i / cols;
  const int c = (int)(i % cols);
  dst[i] = src[(long long)idx[r] * cols + c];
}

// M networks: y = mean, spread = RMS pairwise distance of the stress outputs
// (sqrt(2 / (M - 1) sum_m |s_m - s_mean|^2), |s_a - s_b| for two networks)
// over max(|s_mean|, floor_scale)
__global__ void k_accept_n(const float* ys /* [M][n][n_out] */, int M, long long n, int n_out, float* y,
                           float* spread, uint8_t* accept, float thr, float floor_scale) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float inv = 1.f / (float)M;
  float d2 = 0.f, m2 = 0.f;
  for (int j = 0; j < n_out; ++j) {
    float mean = 0.f;
    for (int m = 0; m < M; ++m) mean += ys[((long long)m * n + r) * n_out + j];
    mean *= inv;
    y[r * n_out + j] = mean;
    if (j < 6) {
      for (int m = 0; m < M; ++m) {
        const float d = ys[((long long)m * n + r) * n_out + j] - mean;
        d2 += d * d;
      }
      m2 += mean * mean;
    }
  }
  const float s = sqrtf(2.f * d2 / (float)(M - 1)) / fmaxf(sqrtf(m2), floor_scale);
  spread[r] = s;
  accept[r] = s <= thr ? 1 : 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int lay_k(int l) { return l == 0 ? MLP_IN : MLP_W; }
static int lay_n(int l) { return l == MLP_LAYERS - 1 ? MLP_OUT : MLP_W; }

Mlp::Mlp(int n_in_, int n_out_, uint64_t seed) : n_in(n_in_), n_out(n_out_) {
  if (n_in < 1 || n_in > MLP_IN || n_out < 1 || n_out > MLP_OUT) fail(HOM_E_ARG, "network size out of range");
  size_t off = 0;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    woff[l] = off;
    off += (size_t)lay_n(l) * lay_k(l);
    boff[l] = off;
    off += lay_n(l);
  }
  npad = off;
  auto alloc = [&](void** p, size_t b) {
    HIPCHK(hipMalloc(p, b));
    HIPCHK(hipMemset(*p, 0, b));
    allocs.push_back(*p);
  };
  alloc((void**)&w, npad * 4);
  alloc((void**)&g, npad * 4);
  alloc((void**)&m, npad * 4);
  alloc((void**)&v, npad * 4);
  alloc((void**)&eff_bf, npad * 4);
  alloc((void**)&eff_pr, npad * 4);
  alloc((void**)&hi, npad * 2);
  alloc((void**)&lo, npad * 2);
  alloc((void**)&scal, 5 * MLP_OUT * 4 + 2 * MLP_IN * 4);
  // G and c in FP32, then G's bf16 hi and lo parts
  alloc((void**)&skip, (MLP_OUT * MLP_GATES * MLP_IN + MLP_OUT) * 4 + 2 * MLP_OUT * MLP_GATES * MLP_IN * 2);
  // He initialization (normal, std sqrt(2 / fan_in)), seeded; biases zero
  std::vector<float> hw(npad, 0.f);
  std::mt19937_64 gen(seed);
  for (int l = 0; l < MLP_LAYERS; ++l) {
    const int K = lay_k(l), N = lay_n(l);
    const int kin = l == 0 ? n_in : K;
    const int nout = l == MLP_LAYERS - 1 ? n_out : N;
    std::normal_distribution<double> nd(0.0, std::sqrt((l == MLP_LAYERS - 1 ? 1.0 : 2.0) / kin));
    for (int i = 0; i < nout; ++i)
      for (int k = 0; k < kin; ++k) hw[woff[l] + (size_t)i * K + k] = (float)nd(gen);
  }
  HIPCHK(hipMemcpy(w, hw.data(), npad * 4, hipMemcpyHostToDevice));
  std::vector<float> s(5 * MLP_OUT + 2 * MLP_IN, 0.f);
  for (int j = 0; j < MLP_IN; ++j) s[MLP_IN + j] = 1.f;            // xinv
  for (int j = 0; j < MLP_OUT; ++j) s[2 * MLP_IN + MLP_OUT + j] = 1.f;  // ystd
  for (int j = 0; j < MLP_OUT; ++j) s[2 * MLP_IN + 2 * MLP_OUT + j] = 1.f;  // loss weights
  HIPCHK(hipMemcpy(scal, s.data(), s.size() * 4, hipMemcpyHostToDevice));
  hx_mean.assign(n_in, 0.f);
  hx_inv.assign(n_in, 1.f);
  hy_mean.assign(n_out, 0.f);
  hy_std.assign(n_out, 1.f);
  refresh(nullptr);
  HIPCHK(hipDeviceSynchronize());
}

Mlp::~Mlp() {
  free_work();
  for (void* p : allocs) (void)hipFree(p);
  if (splitk) (void)hipFree(splitk);
  if (csum) (void)hipFree(csum);
}

void Mlp::free_work() {
  for (void* p : work) (void)hipFree(p);
  work.clear();
  work_rows = 0;
}

void Mlp::refresh(hipStream_t s) {
  const long long n = (long long)npad;
  LayerSpans ls;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    ls.off[l] = (long long)woff[l];
    ls.n[l] = lay_n(l);
    ls.k[l] = lay_k(l);
  }
  hipLaunchKernelGGL(k_split, dim3((n + 255) / 256), dim3(256), 0, s, w, hi, lo, eff_bf, eff_pr, n, ls);
}

void Mlp::set_scaling(const float* xmean, const float* xstd, const float* ymean, const float* ystd,
                      const float* lw) {
  std::vector<float> s(5 * MLP_OUT + 2 * MLP_IN, 0.f);
  for (int j = 0; j < MLP_IN; ++j) {
    s[j] = j < n_in ? xmean[j] : 0.f;
    s[MLP_IN + j] = j < n_in ? 1.f / xstd[j] : 1.f;
    if (j < n_in && !(xstd[j] > 0.f)) fail(HOM_E_ARG, "input scale must be positive");
  }
  for (int j = 0; j < MLP_OUT; ++j) {
    s[2 * MLP_IN + j] = j < n_out ? ymean[j] : 0.f;
    s[2 * MLP_IN + MLP_OUT + j] = j < n_out ? ystd[j] : 1.f;
    s[2 * MLP_IN + 2 * MLP_OUT + j] = j < n_out ? (lw ? lw[j] : 1.f) : 0.f;
    if (j < n_out && !(ystd[j] > 0.f)) fail(HOM_E_ARG, "output scale must be positive");
  }
  HIPCHK(hipMemcpy(scal, s.data(), s.size() * 4, hipMemcpyHostToDevice));
  for (int j = 0; j < n_in; ++j) {
    hx_mean[j] = xmean[j];
    hx_inv[j] = 1.f / xstd[j];
  }
  for (int j = 0; j < n_out; ++j) {
    hy_mean[j] = ymean[j];
    hy_std[j] = ystd[j];
  }
}

void Mlp::normalized_targets(const float* X, const float* T, long long n, float* out) const {
  std::vector<double> xn(n_in);
  for (long long r = 0; r < n; ++r) {
    if (!hskip.empty()) normalize_row(X + r * n_in, xn.data());
    for (int j = 0; j < MLP_OUT; ++j) {
      float v = 0.f;
      if (j < n_out) {
        const double sk = hskip.empty() ? 0.0 : skip_value(xn.data(), j);
        v = (float)((T[r * n_out + j] - sk - hy_mean[j]) / hy_std[j]);
      }
      out[r * MLP_OUT + j] = v;
    }
  }
}

void Mlp::set_skip(const int* gates, const float* G, const float* c) {
  for (int i = 0; i < 3; ++i) {
    if (gates[i] < 0 || gates[i] >= n_in) fail(HOM_E_ARG, "gate index out of range");
    gate[i] = gates[i];
  }
  std::vector<float> f(MLP_OUT * MLP_GATES * MLP_IN + MLP_OUT, 0.f);
  hskip.assign((size_t)n_out * MLP_GATES * n_in + n_out, 0.0);
  for (int j = 0; j < n_out; ++j) {
    for (int g = 0; g < MLP_GATES; ++g)
      for (int k = 0; k < n_in; ++k) {
        const float v = G[((size_t)j * MLP_GATES + g) * n_in + k];
        f[((size_t)j * MLP_GATES + g) * MLP_IN + k] = v;
        hskip[((size_t)j * MLP_GATES + g) * n_in + k] = v;
      }
    f[MLP_OUT * MLP_GATES * MLP_IN + j] = c[j];
    hskip[(size_t)n_out * MLP_GATES * n_in + j] = c[j];
  }
  HIPCHK(hipMemcpy(skip, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  // bf16 hi + lo parts of G (round to nearest even; G is finite)
  const auto bf16_bits = [](float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  };
  constexpr size_t NG = (size_t)MLP_OUT * MLP_GATES * MLP_IN;
  std::vector<uint16_t> parts(2 * NG);
  for (size_t i = 0; i < NG; ++i) {
    parts[i] = bf16_bits(f[i]);
    const uint32_t hu = (uint32_t)parts[i] << 16;
    float h;
    std::memcpy(&h, &hu, 4);
    parts[NG + i] = bf16_bits(f[i] - h);
  }
  HIPCHK(hipMemcpy(skip + f.size(), parts.data(), parts.size() * 2, hipMemcpyHostToDevice));
}

void Mlp::normalize_row(const float* x, double* xn) const {
  for (int k = 0; k < n_in; ++k) xn[k] = ((double)x[k] - hx_mean[k]) * hx_inv[k];
}

double Mlp::skip_value(const double* xn, int j) const {
  if (hskip.empty()) return 0.0;
  const double va = xn[gate[0]], vb = xn[gate[1]], vc = xn[gate[2]];
  const double s[MLP_GATES] = {1, va, va * va, va * va * va, vb, vb * vb, vb * vb * vb, vc, vc * vc, vc * vc * vc};
  double y = hskip[(size_t)n_out * MLP_GATES * n_in + j];
  for (int g = 0; g < MLP_GATES; ++g) {
    double t = 0.0;
    for (int k = 0; k < n_in; ++k) t += hskip[((size_t)j * MLP_GATES + g) * n_in + k] * xn[k];
    y += s[g] * t;
  }
  return y;
}

// Host-side least squares in FP64: normal equations of the design
// [1, xhat * s_g(xhat)] with a tiny ridge, solved by Cholesky.
void Mlp::fit_skip(const float* X, const float* Y, long long n, const int* gates, const float* lw,
                   const float* rw) {
  if (n < 2) fail(HOM_E_ARG, "need rows to fit");
  for (int i = 0; i < 3; ++i)
    if (gates[i] < 0 || gates[i] >= n_in) fail(HOM_E_ARG, "gate index out of range");
  // input scaling from the rows
  std::vector<double> xm(n_in, 0.0), xv(n_in, 0.0);
  for (long long r = 0; r < n; ++r)
    for (int k = 0; k < n_in; ++k) xm[k] += X[r * n_in + k];
  for (int k = 0; k < n_in; ++k) xm[k] /= (double)n;
  for (long long r = 0; r < n; ++r)
    for (int k = 0; k < n_in; ++k) {
      const double d = X[r * n_in + k] - xm[k];
      xv[k] += d * d;
    }
  std::vector<float> xmf(n_in), xsf(n_in);
  for (int k = 0; k < n_in; ++k) {
    const double sd = std::sqrt(xv[k] / (double)n);
    xmf[k] = (float)xm[k];
    xsf[k] = sd > 1e-12 ? (float)sd : 1.f;
  }
  hx_mean.assign(xmf.begin(), xmf.end());
  hx_inv.resize(n_in);
  for (int k = 0; k < n_in; ++k) hx_inv[k] = 1.f / xsf[k];
  const int P = 1 + MLP_GATES * n_in;
  std::vector<double> AtA((size_t)P * P, 0.0), AtY((size_t)P * n_out, 0.0), phi(P), xn(n_in);
  for (long long r = 0; r < n; ++r) {
    normalize_row(X + r * n_in, xn.data());
    const double va = xn[gates[0]], vb = xn[gates[1]], vc = xn[gates[2]];
    const double s[MLP_GATES] = {1, va, va * va, va * va * va, vb, vb * vb, vb * vb * vb, vc, vc * vc, vc * vc * vc};
    phi[0] = 1.0;
    for (int g = 0; g < MLP_GATES; ++g)
      for (int k = 0; k < n_in; ++k) phi[1 + g * n_in + k] = s[g] * xn[k];
    const double wr = rw ? (double)rw[r] : 1.0;  // weighted least squares
    for (int a = 0; a < P; ++a) {
      const double pa = wr * phi[a];
      double* row = &AtA[(size_t)a * P];
      for (int b = 0; b <= a; ++b) row[b] += pa * phi[b];
      for (int j = 0; j < n_out; ++j) AtY[(size_t)a * n_out + j] += pa * Y[r * n_out + j];
    }
  }
  double tr = 0.0;
  for (int a = 0; a < P; ++a) tr += AtA[(size_t)a * P + a];
  // Cholesky (lower, in place) with a small ridge; the cubic gate features
  // make the normal equations ill-conditioned, so the ridge grows until the
  // factorization succeeds in FP64
  const std::vector<double> A0(AtA);
  bool ok = false;
  for (double ridge : {1e-12, 1e-10, 1e-8, 1e-6}) {
    AtA = A0;
    for (int a = 0; a < P; ++a) AtA[(size_t)a * P + a] += ridge * tr / P;
    ok = true;
    for (int j = 0; j < P && ok; ++j) {
      double d = AtA[(size_t)j * P + j];
      for (int k = 0; k < j; ++k) d -= AtA[(size_t)j * P + k] * AtA[(size_t)j * P + k];
      if (!(d > 0.0)) {
        ok = false;
        break;
      }
      d = std::sqrt(d);
      AtA[(size_t)j * P + j] = d;
      for (int i = j + 1; i < P; ++i) {
        double v = AtA[(size_t)i * P + j];
        for (int k = 0; k < j; ++k) v -= AtA[(size_t)i * P + k] * AtA[(size_t)j * P + k];
        AtA[(size_t)i * P + j] = v / d;
      }
    }
    if (ok) break;
  }
  if (!ok) fail(HOM_E_NAN, "skip fit: normal equations not positive definite");
  std::vector<float> G((size_t)n_out * MLP_GATES * n_in), c(n_out);
  std::vector<double> z(P);
  for (int j = 0; j < n_out; ++j) {
    for (int i = 0; i < P; ++i) {
      double v = AtY[(size_t)i * n_out + j];
      for (int k = 0; k < i; ++k) v -= AtA[(size_t)i * P + k] * z[k];
      z[i] = v / AtA[(size_t)i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
      double v = z[i];
      for (int k = i + 1; k < P; ++k) v -= AtA[(size_t)k * P + i] * z[k];
      z[i] = v / AtA[(size_t)i * P + i];
    }
    c[j] = (float)z[0];
    for (int g = 0; g < MLP_GATES; ++g)
      for (int k = 0; k < n_in; ++k) G[((size_t)j * MLP_GATES + g) * n_in + k] = (float)z[1 + g * n_in + k];
  }
  set_skip(gates, G.data(), c.data());
  // residual scaling
  std::vector<double> rm(n_out, 0.0), rv(n_out, 0.0);
  std::vector<double> res((size_t)n * n_out);
  for (long long r = 0; r < n; ++r) {
    normalize_row(X + r * n_in, xn.data());
    for (int j = 0; j < n_out; ++j) {
      const double v = Y[r * n_out + j] - skip_value(xn.data(), j);
      res[r * n_out + j] = v;
      rm[j] += v;
    }
  }
  for (int j = 0; j < n_out; ++j) rm[j] /= (double)n;
  for (long long r = 0; r < n; ++r)
    for (int j = 0; j < n_out; ++j) rv[j] += (res[r * n_out + j] - rm[j]) * (res[r * n_out + j] - rm[j]);
  std::vector<float> rmf(n_out), rsf(n_out);
  for (int j = 0; j < n_out; ++j) {
    const double sd = std::sqrt(rv[j] / (double)n);
    rmf[j] = (float)rm[j];
    rsf[j] = sd > 1e-12 ? (float)sd : 1.f;
  }
  set_scaling(xmf.data(), xsf.data(), rmf.data(), rsf.data(), lw);
}

void Mlp::ensure_work(long long rows) {
  if (rows <= work_rows) return;
  free_work();
  auto alloc = [&](float** p, size_t count) {
    HIPCHK(hipMalloc((void**)p, count * 4));
    work.push_back(*p);
  };
  alloc(&xs, rows * MLP_IN);
  for (int l = 0; l < MLP_LAYERS - 1; ++l) {
    alloc(&zs[l], rows * MLP_W);
    alloc(&as[l], rows * MLP_W);
  }
  alloc(&yhat, rows * MLP_OUT);
  alloc(&dy, rows * MLP_OUT);
  alloc(&da, rows * MLP_W);
  alloc(&dz, rows * MLP_W);
  alloc(&xb, rows * MLP_IN);
  alloc(&tb, rows * MLP_OUT);
  alloc(&rwb, rows);
  alloc(&lpart, (rows * MLP_OUT + 255) / 256 * 2);
  work_rows = rows;
}

void Mlp::forward(const float* x, float* y, long long n, bool precise, bool save, hipStream_t s) {
  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.n = n;
  a.n_in = n_in;
  a.n_out = n_out;
  a.xmean = scal;
  a.xinv = scal + MLP_IN;
  a.ymean = scal + 2 * MLP_IN;
  a.ystd = scal + 2 * MLP_IN + MLP_OUT;
  a.skip = skip;
  a.skip_hi = reinterpret_cast<const __bf16*>(skip + MLP_OUT * MLP_GATES * MLP_IN + MLP_OUT);
  a.skip_lo = a.skip_hi + MLP_OUT * MLP_GATES * MLP_IN;
  a.g0 = gate[0];
  a.g1 = gate[1];
  a.g2 = gate[2];
  for (int l = 0; l < MLP_LAYERS; ++l) {
    a.whi[l] = hi + woff[l];
    a.wlo[l] = lo + woff[l];
    a.bias[l] = w + boff[l];
  }
  a.y = y;
  if (save) {
    a.yhat = yhat;
    a.xs = xs;
    for (int l = 0; l < MLP_LAYERS - 1; ++l) {
      a.zs[l] = zs[l];
      a.as[l] = as[l];
    }
  }
  const unsigned blocks = (unsigned)((n + MROWS - 1) / MROWS);
  if (save) {
    if (precise)
      hipLaunchKernelGGL((k_mlp_fwd<1, true>), dim3(blocks), dim3(FWD_WAVES * 64), 0, s, a);
    else
      hipLaunchKernelGGL((k_mlp_fwd<0, true>), dim3(blocks), dim3(FWD_WAVES * 64), 0, s, a);
  } else {
    if (precise)
      hipLaunchKernelGGL((k_mlp_fwd<1, false>), dim3(blocks), dim3(FWD_WAVES * 64), 0, s, a);
    else
      hipLaunchKernelGGL((k_mlp_fwd<0, false>), dim3(blocks), dim3(FWD_WAVES * 64), 0, s, a);
  }
}

// C = sum_s P[s] over the split-K partials, in a fixed order
__global__ void __launch_bounds__(256) k_sum_splits(const float* P, int splits, int M, int N, float* C, int ldc) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  float v = 0.f;
  for (int k = 0; k < splits; ++k) v += P[(long long)k * M * N + i];
  C[(long long)m * ldc + n] = v;
}

static void colsum(Mlp& net, const float* in, long long rows, int cols, float* out, hipStream_t s) {
  const int chunks = (int)((rows + COLSUM_CHUNK - 1) / COLSUM_CHUNK);
  const size_t need = (size_t)chunks * cols;
  if (need > net.csum_n) {
    if (net.csum) HIPCHK(hipFree(net.csum));
    net.csum = nullptr;
    HIPCHK(hipMalloc((void**)&net.csum, need * sizeof(double)));
    net.csum_n = need;
  }
  hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, chunks), dim3(256), 0, s, in, rows, cols, net.csum);
  hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, s, net.csum, chunks, cols, out);
}

static void gemm(Mlp& net, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                 float* C, int ldc, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  // weight gradients: a small M x N output over a long K (the batch) gets
  // few work-groups; split K over more of them and sum the partials
  if (ta && !tb && grid.x * grid.y < 128 && K >= 1024) {
    const int splits = std::min(64, K / 256);
    const int kc = (K + splits - 1) / splits;
    const size_t need = (size_t)splits * M * N;
    if (need > net.splitk_n) {
      if (net.splitk) HIPCHK(hipFree(net.splitk));
      net.splitk = nullptr;
      HIPCHK(hipMalloc((void**)&net.splitk, need * sizeof(float)));
      net.splitk_n = need;
    }
    const int nsp = (K + kc - 1) / kc;  // every split has at least one row
    hipLaunchKernelGGL((k_gemm<true, false>), dim3(grid.x, grid.y, nsp), dim3(256), 0, s, M, N, K, A, lda, B, ldb,
                       net.splitk, N, 0.f, kc);
    const long long cnt = (long long)M * N;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, net.splitk, nsp, M, N,
                       C, ldc);
    return;
  }
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, 0.f);
  if (ta && !tb) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, 0.f);
  if (!ta && tb) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, 0.f);
  if (ta && tb) hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, 0.f);
}

// loss and gradient of the rows (x, t normalized targets already in xb / tb
// layout: x raw [B][n_in], t normalized [B][16])
// Fixed-order sum of the loss partials of one step into a device accumulator
// (training reads the losses back once, at the end, not after every step).
__global__ void __launch_bounds__(256) k_loss_accumulate(const double* part, int n, double* acc) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

double Mlp::loss_grad(const float* x, const float* tnorm, long long B, bool precise, hipStream_t s,
                      const float* rw) {
  const int lb = grad_only(x, tnorm, B, precise, s, rw);
  std::vector<double> lp(lb);
  HIPCHK(hipMemcpyAsync(lp.data(), lpart, lb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double L = 0.0;
  for (double v : lp) L += v;
  return L;
}

int Mlp::grad_only(const float* x, const float* tnorm, long long B, bool precise, hipStream_t s, const float* rw) {
  ensure_work(B);
  forward(x, nullptr, B, precise, true, s);
  const long long cnt = B * MLP_OUT;
  const int lb = (int)((cnt + 255) / 256);
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, s, yhat, tnorm, scal + 2 * MLP_IN + 2 * MLP_OUT, rw, B, n_out, dy,
                     reinterpret_cast<double*>(lpart));
  const float* eff = precise ? eff_pr : eff_bf;
  const float* dcur = dy;
  int ncur = MLP_OUT;
  for (int l = MLP_LAYERS - 1; l >= 0; --l) {
    const int K = lay_k(l), N = lay_n(l);
    const float* ain = l == 0 ? xs : as[l - 1];
    // dW[N][K] = dZ^T (B x N) . A (B x K)
    gemm(*this, true, false, N, K, (int)B, dcur, ncur, ain, K, g + woff[l], K, s);
    colsum(*this, dcur, B, N, g + boff[l], s);
    if (l > 0) {
      // dA (B x K) = dZ (B x N) . W (N x K), then dZ_prev = dA * gelu'(Z_prev)
      gemm(*this, false, false, (int)B, K, N, dcur, ncur, eff + woff[l], K, da, K, s);
      const long long c = B * K;
      hipLaunchKernelGGL(k_gelu_back, dim3((c + 255) / 256), dim3(256), 0, s, da, zs[l - 1], dz, c);
      // dz is read by the next layer's dW / dA products before its own
      // gelu' step overwrites it (stream order), so one pair of buffers suffices
      dcur = dz;
      ncur = K;
    }
  }
  return lb;
}

void Mlp::get_params(float* out) const {
  std::vector<float> hw(npad);
  HIPCHK(hipMemcpy(hw.data(), w, npad * 4, hipMemcpyDeviceToHost));
  size_t o = 0;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    const int K = lay_k(l);
    const int kin = l == 0 ? n_in : K;
    const int nout = l == MLP_LAYERS - 1 ? n_out : lay_n(l);
    for (int i = 0; i < nout; ++i)
      for (int k = 0; k < kin; ++k) out[o++] = hw[woff[l] + (size_t)i * K + k];
    for (int i = 0; i < nout; ++i) out[o++] = hw[boff[l] + i];
  }
}

void Mlp::get_grads(float* out) const {
  std::vector<float> hg(npad);
  HIPCHK(hipMemcpy(hg.data(), g, npad * 4, hipMemcpyDeviceToHost));
  size_t o = 0;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    const int K = lay_k(l);
    const int kin = l == 0 ? n_in : K;
    const int nout = l == MLP_LAYERS - 1 ? n_out : lay_n(l);
    for (int i = 0; i < nout; ++i)
      for (int k = 0; k < kin; ++k) out[o++] = hg[woff[l] + (size_t)i * K + k];
    for (int i = 0; i < nout; ++i) out[o++] = hg[boff[l] + i];
  }
}

void Mlp::set_params(const float* in) {
  std::vector<float> hw(npad, 0.f);
  size_t o = 0;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    const int K = lay_k(l);
    const int kin = l == 0 ? n_in : K;
    const int nout = l == MLP_LAYERS - 1 ? n_out : lay_n(l);
    for (int i = 0; i < nout; ++i)
      for (int k = 0; k < kin; ++k) hw[woff[l] + (size_t)i * K + k] = in[o++];
    for (int i = 0; i < nout; ++i) hw[boff[l] + i] = in[o++];
  }
  HIPCHK(hipMemcpy(w, hw.data(), npad * 4, hipMemcpyHostToDevice));
  refresh(nullptr);
  HIPCHK(hipDeviceSynchronize());
}

size_t Mlp::param_count() const {
  size_t c = 0;
  for (int l = 0; l < MLP_LAYERS; ++l) {
    const int kin = l == 0 ? n_in : lay_k(l);
    const int nout = l == MLP_LAYERS - 1 ? n_out : lay_n(l);
    c += (size_t)nout * kin + nout;
  }
  return c;
}

void Mlp::train(const float* X, const float* T, long long n, int epochs, int batch, double lr0, uint64_t seed,
                const float* row_weight, float* loss_out) {
  if (n < batch || batch < 1) fail(HOM_E_ARG, "need at least one full batch");
  // a stream of this call (default priority): networks trained from several
  // host threads overlap on the device
  hipStream_t s = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sguard{s};
  float *dX = nullptr, *dT = nullptr, *dW = nullptr;
  int* didx = nullptr;
  HIPCHK(hipMalloc((void**)&dX, n * n_in * 4));
  HIPCHK(hipMalloc((void**)&dT, n * MLP_OUT * 4));
  HIPCHK(hipMalloc((void**)&didx, n * 4));
  if (row_weight) HIPCHK(hipMalloc((void**)&dW, n * 4));
  struct Guard {  // destroyed before sguard: waits for the stream, then frees
    hipStream_t s;
    std::vector<void*> p;
    ~Guard() {
      (void)hipStreamSynchronize(s);
      for (void* q : p)
        if (q) (void)hipFree(q);
    }
  } guard{s, {dX, dT, didx, dW}};
  std::vector<float> tn((size_t)n * MLP_OUT);
  normalized_targets(X, T, n, tn.data());
  HIPCHK(hipMemcpy(dX, X, n * n_in * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dT, tn.data(), tn.size() * 4, hipMemcpyHostToDevice));
  if (row_weight) {  // scaled to mean 1, so the learning rate keeps its meaning
    double sum = 0.0;
    for (long long r = 0; r < n; ++r) sum += row_weight[r];
    if (!(sum > 0.0)) fail(HOM_E_ARG, "row weights sum to zero");
    std::vector<float> rw(row_weight, row_weight + n);
    for (float& x : rw) x = (float)(x * (double)n / sum);
    HIPCHK(hipMemcpy(dW, rw.data(), n * 4, hipMemcpyHostToDevice));
  }
  ensure_work(batch);
  std::mt19937_64 gen(seed);
  std::vector<int> perm(n);
  const long long steps_per_epoch = n / batch;
  double* dloss = nullptr;  // per-epoch loss sums on the device
  HIPCHK(hipMalloc((void**)&dloss, std::max(epochs, 1) * sizeof(double)));
  guard.p.push_back(dloss);
  HIPCHK(hipMemsetAsync(dloss, 0, std::max(epochs, 1) * sizeof(double), s));
  // the clears of freshly allocated work buffers ran on the null stream, which
  // this non-blocking stream does not wait for
  HIPCHK(hipStreamSynchronize(nullptr));
  const long long total = steps_per_epoch * epochs;
  long long step = 0;
  const float b1 = 0.9f, b2 = 0.999f;
  for (int e = 0; e < epochs; ++e) {
    for (long long i = 0; i < n; ++i) perm[i] = (int)i;
    std::shuffle(perm.begin(), perm.end(), gen);
    HIPCHK(hipStreamSynchronize(s));  // the last epoch's gathers have read didx
    HIPCHK(hipMemcpy(didx, perm.data(), n * 4, hipMemcpyHostToDevice));
    for (long long sidx = 0; sidx < steps_per_epoch; ++sidx) {
      const int* bi = didx + sidx * batch;
      const long long cx = (long long)batch * n_in, ct = (long long)batch * MLP_OUT;
      hipLaunchKernelGGL(k_gather, dim3((cx + 255) / 256), dim3(256), 0, s, dX, n_in, bi, (long long)batch, xb);
      hipLaunchKernelGGL(k_gather, dim3((ct + 255) / 256), dim3(256), 0, s, dT, MLP_OUT, bi, (long long)batch, tb);
      if (dW)
        hipLaunchKernelGGL(k_gather, dim3((batch + 255) / 256), dim3(256), 0, s, dW, 1, bi, (long long)batch, rwb);
      const int lb = grad_only(xb, tb, batch, false, s, dW ? rwb : nullptr);
      hipLaunchKernelGGL(k_loss_accumulate, dim3(1), dim3(256), 0, s, reinterpret_cast<const double*>(lpart), lb,
                         dloss + e);
      ++step;
      // cosine decay to 1 % with a short warm-up
      const double prog = (double)step / (double)total;
      double lr = lr0 * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(3.14159265358979 * prog)));
      if (step < 200) lr *= (double)step / 200.0;
      const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
      const long long np = (long long)npad;
      hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, w, g, m, v, np, (float)lr, b1, b2, c1, c2,
                         1e-8f);
      refresh(s);
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (loss_out && epochs > 0) {
    std::vector<double> hl(epochs);
    HIPCHK(hipMemcpy(hl.data(), dloss, epochs * sizeof(double), hipMemcpyDeviceToHost));
    for (int e = 0; e < epochs; ++e) loss_out[e] = (float)(hl[e] / steps_per_epoch);
  }
}

void Mlp::reset_optimizer() {
  HIPCHK(hipMemset(m, 0, npad * 4));
  HIPCHK(hipMemset(v, 0, npad * 4));
  HIPCHK(hipDeviceSynchronize());
}

void ensemble_accept(const Mlp* const* nets, int M, const float* x, float* y, float* ys, float* spread,
                        uint8_t* accept, long long n, float thr, float floor_scale, hipStream_t s) {
  const int n_out = nets[0]->n_out;
  for (int m = 0; m < M; ++m)
    const_cast<Mlp*>(nets[m])->forward(x, ys + (size_t)m * n * n_out, n, false, false, s);
  hipLaunchKernelGGL(k_accept_n, dim3((n + 255) / 256), dim3(256), 0, s, ys, M, n, n_out, y, spread, accept, thr,
                     floor_scale);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device
}  // namespace

// address of the static array on the current device, looked up once per device
static float* static_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(HOM_E_DEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  return g_scratch_ptr[dev];
}

void ensemble_accept_static(const Mlp* const* nets, int M, const float* x, float* y, float* spread, uint8_t* accept,
                            long long n, float thr, float floor_scale, hipStream_t s) {
  const unsigned long long need = (unsigned long long)n * (unsigned long long)M * (unsigned long long)nets[0]->n_out;
  if (need > (unsigned long long)HOM_STATIC_SCRATCH_FLOATS)
    fail(HOM_E_ARG, "rows x networks x outputs = " + std::to_string(need) + " exceeds the static scratch of " +
                        std::to_string(HOM_STATIC_SCRATCH_FLOATS) + " floats");
  ensemble_accept(nets, M, x, y, static_scratch(), spread, accept, n, thr, floor_scale, s);
}

}  // namespace hom
