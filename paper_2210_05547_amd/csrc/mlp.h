// Thermochemistry surrogate network for gfx950: BF16 matrix-core (MFMA) inference with
// FP32 accumulation, FP32 backward pass and Adam.
//
// The paper closes (Sec. 5) by pointing at machine learning as a way to replace the
// expensive calls of its thermochemical library.  The network maps standardised inputs
//   x = (log10 rho, ln T_c, Y_1..Y_5),   T_c = (e - sum_s Y_s h0_s/M_s) / sum_s Y_s c_s,
// (c_s = (3/2 + 2 r_s) R_s: every mode fully excited, so T_c is a closed-form lower bound
// of T) to standardised residuals of y = (ln T, ln mu, ln kappa, ln(rho D_1..5)) about a
// linear function of x (fitted on the training set): y = m + s net(x) + L [1, x],
// with three hidden layers of 64 units: 7 -> 64 -> 64 -> 64 -> 8, 9352 parameters,
// flat order [W1 (64x7, row = output), b1, W2, b2, W3, b3, W4 (8x64), b4].
//
// Matrix-core mapping (v_mfma_f32_32x32x16_bf16, one wavefront of 64 lanes):
//   A (32x16, weights):     lane l holds A[l%32][8(l/32) + q], q = 0..7
//   B (16x32, activations): lane l holds B[8(l/32) + q][l%32]
//   D (32x32, FP32):        lane l, register r holds D[(r%4) + 8(r/4) + 4(l/32)][l%32]
// A wavefront evaluates 64 points as two 32-point column tiles.  The hidden layers'
// K order is permuted so that the B operand of a layer is exactly what the lane holds
// in its accumulators of the previous layer: K step t, lane half h, element q is
// hidden unit 32(t/2) + 4h + (r%4) + 8(r/4) with r = 8(t%2) + q.  Hidden activations
// therefore stay in registers; only the network's inputs (hi + lo BF16 pairs, see
// mlp_wave64) and its 8 outputs pass through a small per-wave LDS buffer.  Biases
// initialise the accumulators.  Weights are stored once, pre-swizzled so that each
// lane's A operand is 16 contiguous bytes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hrx {

constexpr int MLP_NIN = 7, MLP_NH = 64, MLP_NOUT = 8;
constexpr int MLP_NPARAM = 64 * 7 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 8 * 64 + 8;  // 9352
// offsets of each layer's W and b in the flat parameter vector
constexpr int MLP_OFF_W[4] = {0, 64 * 7 + 64, 64 * 7 + 64 + 64 * 64 + 64,
                              64 * 7 + 64 + 2 * (64 * 64 + 64)};
constexpr int MLP_OFF_B[4] = {64 * 7, 64 * 7 + 64 + 64 * 64, 64 * 7 + 64 + 2 * 64 * 64 + 64,
                              64 * 7 + 64 + 2 * (64 * 64 + 64) + 8 * 64};
constexpr int MLP_NIN_L[4] = {7, 64, 64, 64};
constexpr int MLP_NOUT_L[4] = {64, 64, 64, 8};
// MFMA tiling per layer: M tiles of 32 outputs, K steps of 16 inputs
constexpr int MLP_MT[4] = {2, 2, 2, 1};
constexpr int MLP_KS[4] = {1, 4, 4, 4};
// offsets (in BF16 elements) of each layer's swizzled weights
constexpr int MLP_SW_OFF[4] = {0, 1024, 1024 + 4096, 1024 + 2 * 4096};
constexpr int MLP_SW_SIZE = 1024 + 2 * 4096 + 2048;  // 11264
constexpr int MLP_NBIAS = 64 + 64 + 64 + 8;
constexpr int MLP_HPITCH = 16;  // BF16 elements per point row of the input/output buffer

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8_t;

// hidden unit carried by K index (step t, lane half h, element q) of layers 2..4
__host__ __device__ __forceinline__ int mlp_hidden_unit(int t, int h, int q) {
  const int r = 8 * (t & 1) + q;
  return 32 * (t >> 1) + 4 * h + (r & 3) + 8 * (r >> 2);
}

// float -> bfloat16 bits, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}
// value of an input as the first layer sees it: bf16(x) + bf16(x - bf16(x))
__device__ __forceinline__ float split_bf(float x) {
  const float hi = bf2f(f2bf(x));
  return hi + bf2f(f2bf(x - hi));
}

// Hidden activation: the squared rectifier max(z, 0)^2 (continuously differentiable,
// derivative 2 max(z, 0) = 2 sqrt(a) for the output a).  Two full-rate VALU operations
// per value, where tanh (no instruction on gfx950) needs an exponential and a
// reciprocal at a quarter of the rate; on this regression it is also the more accurate
// of the two at equal width.
// The rectifier is one integer max on the bit pattern (negative floats, -0 included,
// are negative integers), which skips the NaN canonicalisation a float max carries.
__device__ __forceinline__ float mlp_act(float z) {
  const float r = __builtin_bit_cast(float, max(__builtin_bit_cast(int, z), 0));
  return r * r;
}

// The same activation for eight values at once, straight to the next layer's BF16
// operand: z |z| (one multiply: the square with z's sign), rounded to BF16 pairs, then
// the rectifier as a packed 16-bit integer max with 0 (negative BF16 values, -0
// included, are negative integers).  Bit-identical to rounding mlp_act(z) to BF16, at
// two operations per value instead of two and a half.
__device__ __forceinline__ bf16x8_t mlp_act_bf16x8(const float* z) {
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef short s16x2_t __attribute__((ext_vector_type(2)));
  bf16x8_t out;
#pragma unroll
  for (int q = 0; q < 8; q += 2) {
    const f32x2_t v = {z[q] * __builtin_fabsf(z[q]), z[q + 1] * __builtin_fabsf(z[q + 1])};
    const s16x2_t h = __builtin_bit_cast(s16x2_t, __builtin_convertvector(v, bf16x2_t));
    const bf16x2_t r = __builtin_bit_cast(bf16x2_t, __builtin_elementwise_max(h, (s16x2_t)0));
    out[q] = r[0];
    out[q + 1] = r[1];
  }
  return out;
}

// Swizzled weight index of element (row o, column k) of layer L (padded with zeros).
__host__ __device__ __forceinline__ int mlp_sw_index(int L, int m, int t, int lane, int q) {
  return MLP_SW_OFF[L] + ((m * MLP_KS[L] + t) * 64 + lane) * 8 + q;
}

// Evaluate the network for the 64 points of one wavefront.  Lane l owns point l:
// x[7] standardised inputs in, y[8] standardised outputs out.  sW: swizzled BF16
// weights (LDS), sB: biases (LDS), sH: this wave's staging buffer (LDS, 64 x
// MLP_HPITCH BF16).  If save != nullptr the FP32 post-activations of the three hidden
// layers are written to save[(L*ldn + point)*64 + unit] for training, with
// point = base + lane and only for points below ldn.
__device__ __forceinline__ void mlp_wave64(const uint16_t* __restrict__ sW,
                                           const float* __restrict__ sB, uint16_t* sH,
                                           const float* x, float* y, float* save, long base,
                                           long ldn, bool valid) {
  const int lane = threadIdx.x & 63;
  const int hl = lane >> 5;    // which half of the wave
  const int col = lane & 31;   // column (point) within a 32-point tile
  // inputs -> BF16 row of this lane's point as hi/lo pairs: columns 0..6 hold
  // bf16(x), columns 7..13 hold bf16(x - bf16(x)) (the first layer's weights are
  // repeated for both halves), 14..15 are zero: the first layer sees its inputs to
  // about 16 significant bits at no extra matrix-core work (K is padded to 16 anyway)
  {
    uint16_t* row = sH + lane * MLP_HPITCH;
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) {
      const uint16_t hi = f2bf(x[k]);
      row[k] = hi;
      row[MLP_NIN + k] = f2bf(x[k] - bf2f(hi));
    }
    row[14] = 0;
    row[15] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  bf16x8_t b[2][4];   // B operands of the current layer: [point tile][K step]
#pragma unroll
  for (int pt = 0; pt < 2; ++pt)
    b[pt][0] = *reinterpret_cast<const bf16x8_t*>(sH + (32 * pt + col) * MLP_HPITCH + 8 * hl);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int L = 0; L < 4; ++L) {
    const int MT = MLP_MT[L], KS = MLP_KS[L];
    const float* bias = sB + (L == 0 ? 0 : (L == 1 ? 64 : (L == 2 ? 128 : 192)));
    f32x16_t acc[2][2];  // [point tile][M tile]
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      f32x16_t c;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int u = 32 * m + (r & 3) + 8 * (r >> 2) + 4 * hl;
        c[r] = (L < 3 || u < MLP_NOUT) ? bias[u] : 0.0f;
      }
#pragma unroll
      for (int pt = 0; pt < 2; ++pt) acc[pt][m] = c;
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(sW + mlp_sw_index(L, m, t, lane, 0));
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
          acc[pt][m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[pt][t], acc[pt][m], 0, 0, 0);
      }
    if (L < 3) {
      // activations in registers; the next layer's B operand for K step t is the
      // BF16 image of registers 8(t%2) .. 8(t%2)+7 of M tile t/2
#pragma unroll
      for (int pt = 0; pt < 2; ++pt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (!save) {
            float z[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) z[q] = acc[pt][t >> 1][8 * (t & 1) + q];
            b[pt][t] = mlp_act_bf16x8(z);
            continue;
          }
          f32x8_t v;
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = mlp_act(acc[pt][t >> 1][8 * (t & 1) + q]);
          b[pt][t] = __builtin_convertvector(v, bf16x8_t);
          {
            const long gp = base + 32 * pt + col;
            if (gp < ldn) {
#pragma unroll
              for (int g = 0; g < 2; ++g) {
                const int i0 = 32 * (t >> 1) + 8 * (2 * (t & 1) + g) + 4 * hl;
                *reinterpret_cast<float4*>(save + ((long)L * ldn + gp) * 64 + i0) =
                    make_float4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
              }
            }
          }
        }
    } else {
      // outputs 0..7 live in registers r = 0..3 of both halves; stage through LDS as FP32
      float* sO = reinterpret_cast<float*>(sH);
#pragma unroll
      for (int pt = 0; pt < 2; ++pt)
#pragma unroll
        for (int r = 0; r < 4; ++r) sO[(32 * pt + col) * 8 + r + 4 * hl] = acc[pt][0][r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int o = 0; o < MLP_NOUT; ++o) y[o] = sO[lane * 8 + o];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  (void)valid;
}

// Cooperative copy of the swizzled weights and biases into LDS (whole block).
__device__ __forceinline__ void mlp_load_lds(const uint16_t* __restrict__ gW,
                                             const float* __restrict__ gB, uint16_t* sW,
                                             float* sB) {
  const uint4* src = reinterpret_cast<const uint4*>(gW);
  uint4* dst = reinterpret_cast<uint4*>(sW);
  for (int i = threadIdx.x; i < MLP_SW_SIZE / 8; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < MLP_NBIAS; i += blockDim.x) sB[i] = gB[i];
}

// Standardisation statistics, linear output baseline and training-domain bounds of the
// surrogate (device).
struct MlpNorm {
  float in_mean[MLP_NIN], in_istd[MLP_NIN];   // mean and 1/std of the raw features
  float out_mean[MLP_NOUT], out_std[MLP_NOUT];
  float out_lin[MLP_NOUT][MLP_NIN + 1];  // y_o += L[o][0] + sum_k L[o][1 + k] x_k
  double log10rho_min, log10rho_max;   // kg/m^3
  double e_lo[5], e_hi[5];             // species energies at the T bounds (J/kg)
  double xiN_min, xiN_max;             // mass fraction of the element N
};

}  // namespace hrx
