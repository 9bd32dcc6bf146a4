// Learned proposal on the matrix cores: a 6-64-64-64-40 ReLU MLP evaluated
// by one wavefront for 64 rows at a time with BF16 operands and FP32
// accumulation (v_mfma_f32_16x16x32_bf16 for the 64-wide layers,
// v_mfma_f32_16x16x16bf16_1k for the zero-padded 16-wide input), and the
// 8-lobe von Mises-Fisher mixture it parameterises (addition beyond the
// paper, which leaves better importance sampling of the residual integrand
// to future work, Sec. 7).
#pragma once

#include "rpi_device.h"

namespace rpi {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 6, kMlpH = 64, kMlpOut = 40, kLobes = 8;
// flat parameter vector, row-major [in][out]:
// W1[6][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][40] b4[40]
constexpr int OFF_W1 = 0, OFF_B1 = 384, OFF_W2 = 448, OFF_B2 = 4544, OFF_W3 = 4608, OFF_B3 = 8704,
              OFF_W4 = 8768, OFF_B4 = 11328;
static_assert(OFF_B4 + kMlpOut == kMlpNParam, "parameter layout");
// BF16 block of a proposal (element offsets): forward layouts then backward layouts
constexpr int H_WT1 = 0, H_WT2 = H_WT1 + 64 * 16, H_WT3 = H_WT2 + 64 * 64, H_WT4 = H_WT3 + 64 * 64,
              H_W2 = H_WT4 + 48 * 64, H_W3 = H_W2 + 64 * 64, H_W4 = H_W3 + 64 * 64, H_TOTAL = H_W4 + 64 * 48;
static_assert(H_TOTAL == kMlpHalfElems, "BF16 block layout");
constexpr int kActStride = 72;   // bf16 per LDS activation row (64 + 8 padding against bank conflicts)
constexpr int kOutStride = 48;   // fp32 per LDS output row (40 used)
constexpr int kMlpLdsBytes = 64 * kOutStride * 4;  // 12288: the traversal stack's LDS holds one forward pass
static_assert(kMlpLdsBytes >= 64 * kActStride * 2, "activation rows fit the output block");

DEV uint16_t f2bf(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// MFMA 16x16x16 operand layout (lane l, r = l % 16, g = l / 16):
//   A (16 x K16):  lane holds A[r][4g .. 4g+3]
//   B (K16 x 16):  lane holds B[4g .. 4g+3][r]
//   D (16 x 16):   lane holds D[4g .. 4g+3][r]
DEV f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
// MFMA 16x16x32 (gfx950), twice the depth per instruction:
//   A (16 x K32):  lane holds A[r][8g .. 8g+7]
//   B (K32 x 16):  lane holds B[8g .. 8g+7][r]
//   D (16 x 16):   as above
// (the product needs only that both operands use the same order of k)
DEV f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c, 0,
                                                  0, 0);
}

// Rows mt*16 .. mt*16 + 15 of a dense layer (16 accumulators per lane; the
// layer is described below).
template <int K, int NT, bool LAST, int IS = kActStride>
DEV void mlp_tile(const uint16_t* in, uint16_t* out, const uint16_t* __restrict__ wt, const float* __restrict__ bias,
                  float* outf, int mt) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  f32x4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (K % 32 == 0) {
#pragma unroll
    for (int kt = 0; kt < K / 32; ++kt) {
      const bf16x8 aa = *reinterpret_cast<const bf16x8*>(in + (mt * 16 + r) * IS + kt * 32 + 8 * g);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[nt] = mfma32(aa, *reinterpret_cast<const bf16x8*>(wt + (nt * 16 + r) * K + kt * 32 + 8 * g), acc[nt]);
    }
  } else {
#pragma unroll
    for (int kt = 0; kt < K / 16; ++kt) {
      const bf16x4 aa = *reinterpret_cast<const bf16x4*>(in + (mt * 16 + r) * IS + kt * 16 + 4 * g);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[nt] = mfma(aa, *reinterpret_cast<const bf16x4*>(wt + (nt * 16 + r) * K + kt * 16 + 4 * g), acc[nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int col = nt * 16 + r;
    const float bv = bias[col];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = mt * 16 + 4 * g + e;
      const float v = acc[nt][e] + bv;
      if (LAST) outf[row * kOutStride + col] = v;
      else out[row * kActStride + col] = f2bf(fmaxf(v, 0.0f));
    }
  }
}

// One dense layer over the 64 rows in LDS: in [64][IS] bf16 (K columns)
// times W (transposed in wt [NT*16][K]) + bias; ReLU and bf16 into out
// [64][kActStride], or fp32 into outf [64][kOutStride] for the last layer.
// One 16-row tile at a time, last tile first.
// out / outf may alias in (one wave owns the rows): a tile's input rows are
// read only by that tile's products, which its writes depend on, and the
// fp32 output rows of tile mt (bytes [3072 mt, 3072 mt + 3072)) overlap only
// input rows >= 21 mt, i.e. tiles already consumed or being consumed.
template <int K, int NT, bool LAST, int IS = kActStride>
DEV void mlp_layer(const uint16_t* in, uint16_t* out, const uint16_t* __restrict__ wt, const float* __restrict__ bias,
                   float* outf) {
#pragma unroll 1
  for (int mt = 3; mt >= 0; --mt) mlp_tile<K, NT, LAST, IS>(in, out, wt, bias, outf, mt);
  __syncthreads();
}

// Forward pass of the wave's 64 rows (lane l supplies row l).  All 64 lanes
// must execute this call.  lds: kMlpLdsBytes of workgroup memory (one wave
// per workgroup).  Returns this lane's 40 raw outputs in LDS (valid until the
// region is reused).
DEV const float* mlp_forward_wave(const MlpDev& M, const float x[6], void* lds) {
  uint16_t* act = reinterpret_cast<uint16_t*>(lds);
  float* outf = reinterpret_cast<float*>(lds);
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < 16; ++c) act[l * kActStride + c] = c < 6 ? f2bf(x[c]) : (uint16_t)0;
  __syncthreads();
  mlp_layer<16, 4, false>(act, act, M.wt1, M.b1, nullptr);
  mlp_layer<64, 4, false>(act, act, M.wt2, M.b2, nullptr);
  mlp_layer<64, 4, false>(act, act, M.wt3, M.b3, nullptr);
  mlp_layer<64, 3, true>(act, nullptr, M.wt4, M.b4, outf);
  return outf + l * kOutStride;
}

DEV void mlp_input(const MlpDev& M, vec3 p_obj, vec3 n_obj, float x[6]) {
  x[0] = (p_obj.x - M.center.x) * M.inv_half.x;
  x[1] = (p_obj.y - M.center.y) * M.inv_half.y;
  x[2] = (p_obj.z - M.center.z) * M.inv_half.z;
  x[3] = n_obj.x;
  x[4] = n_obj.y;
  x[5] = n_obj.z;
}

// ------------------------------------------------------------------ vMF mixture
DEV float softplusf_(float x) { return x > 20.0f ? x : log1pf(expf(x)); }

// Lobe l of raw outputs: mean = normalize(raw xyz), kappa = softplus + 0.01
// (<= 1e4), weight = softmax over lobes (mx = max raw weight logit, es = sum).
DEV void lobe(const float* raw, int l, vec3& mu, float& kappa) {
  float x = raw[5 * l], y = raw[5 * l + 1], z = raw[5 * l + 2];
  float n = sqrtf(x * x + y * y + z * z);
  if (!(n > 0.0f)) {
    x = 0.0f;
    y = 0.0f;
    z = 1.0f;
    n = 1.0f;
  }
  mu = v3(x / n, y / n, z / n);
  kappa = fminf(softplusf_(raw[5 * l + 3]) + 0.01f, 1e4f);
}
DEV void lobe_weights(const float* raw, float w[kLobes]) {
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) mx = fmaxf(mx, raw[5 * l + 4]);
  float sum = 0.0f;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) {
    w[l] = expf(raw[5 * l + 4] - mx);
    sum += w[l];
  }
#pragma unroll
  for (int l = 0; l < kLobes; ++l) w[l] /= sum;
}
// Mixture density: kappa / (2 pi (1 - e^{-2 kappa})) exp(kappa (mu.w - 1)).
DEV float vmf_mix_pdf(const float* raw, vec3 w) {
  float wl[kLobes];
  lobe_weights(raw, wl);
  float q = 0.0f;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) {
    vec3 mu;
    float k;
    lobe(raw, l, mu, k);
    q += wl[l] * k / (2.0f * kPi * (-expm1f(-2.0f * k))) * expf(k * (dot(mu, w) - 1.0f));
  }
  return q;
}
// Jakob 2012, numerically stable vMF sampling on S^2.
DEV vec3 vmf_mix_sample(const float* raw, float u0, float u1, float u2) {
  float wl[kLobes];
  lobe_weights(raw, wl);
  int l = 0;
  float run = 0.0f;
  for (; l < kLobes - 1; ++l) {
    run += wl[l];
    if (u0 < run) break;
  }
  vec3 mu;
  float k;
  lobe(raw, l, mu, k);
  // u1 = 0 with e^{-2 kappa} below the float range makes the argument 0:
  // the formula's limit there is c = -1, the antipode of the mean
  const float a = u1 + (1.0f - u1) * expf(-2.0f * k);
  const float c = a > 0.0f ? 1.0f + logf(a) / k : -1.0f;
  const float s = sqrtf(fmaxf(0.0f, 1.0f - c * c));
  float sp, cp;
  sincosf(2.0f * kPi * u2, &sp, &cp);
  vec3 t, b;
  onb(mu, t, b);
  return unit(t * (s * cp) + b * (s * sp) + mu * c);
}

// Technique (8)'s direction sampler, a defensive mixture (Hesterberg 1995):
// with probability kT8Uniform a uniform direction on the sphere, else the
// learned lobes, so the technique keeps full support where the lobes'
// densities underflow.
constexpr float kT8Uniform = 0.25f;
DEV vec3 t8_dir_sample(const float* raw, float u0, float u1, float u2) {
  if (u0 < kT8Uniform) return sphere_dir(u1, u2);
  return vmf_mix_sample(raw, (u0 - kT8Uniform) / (1.0f - kT8Uniform), u1, u2);
}
DEV float t8_dir_pdf(const float* raw, vec3 w) {
  return kT8Uniform / (4.0f * kPi) + (1.0f - kT8Uniform) * vmf_mix_pdf(raw, w);
}

}  // namespace rpi
