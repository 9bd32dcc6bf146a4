// Learned proposal kernels (addition beyond the paper; the paper
// leaves better sampling of the residual integrand to future work, Sec. 7):
// batched MLP inference, the gradient of the weighted negative log-likelihood
// of the vMF mixture (the Monte Carlo KL objective of neural importance
// sampling, Mueller et al. 2019) by back-propagation on the matrix cores, and
// Adam.  BF16 operands, FP32 accumulation, 64 rows per pass (inference: one
// wavefront per workgroup; the gradient: four).
#include "rpi_mlp.h"

namespace rpi {

MlpDev mlp_view(const MlpBufs& B, vec3 center, vec3 inv_half) {
  MlpDev M;
  M.wt1 = B.h + H_WT1;
  M.wt2 = B.h + H_WT2;
  M.wt3 = B.h + H_WT3;
  M.wt4 = B.h + H_WT4;
  M.w2 = B.h + H_W2;
  M.w3 = B.h + H_W3;
  M.w4 = B.h + H_W4;
  M.b1 = B.bias;
  M.b2 = B.bias + 64;
  M.b3 = B.bias + 128;
  M.b4 = B.bias + 192;
  M.center = center;
  M.inv_half = inv_half;
  return M;
}

// Write the copies the kernels read of flat parameter p (value x): BF16 in
// the forward ([out][in]) and backward ([in][out]) layouts, FP32 biases.
DEV void pack_one(const MlpBufs& B, int p, float x) {
  const uint16_t h = f2bf(x);
  if (p < OFF_B1) {
    B.h[H_WT1 + (p % 64) * 16 + p / 64] = h;
  } else if (p < OFF_W2) {
    B.bias[p - OFF_B1] = x;
  } else if (p < OFF_B2) {
    const int q = p - OFF_W2, i = q / 64, o = q % 64;
    B.h[H_WT2 + o * 64 + i] = h;
    B.h[H_W2 + i * 64 + o] = h;
  } else if (p < OFF_W3) {
    B.bias[64 + p - OFF_B2] = x;
  } else if (p < OFF_B3) {
    const int q = p - OFF_W3, i = q / 64, o = q % 64;
    B.h[H_WT3 + o * 64 + i] = h;
    B.h[H_W3 + i * 64 + o] = h;
  } else if (p < OFF_W4) {
    B.bias[128 + p - OFF_B3] = x;
  } else if (p < OFF_B4) {
    const int q = p - OFF_W4, i = q / 40, o = q % 40;
    B.h[H_WT4 + o * 64 + i] = h;
    B.h[H_W4 + i * 48 + o] = h;
  } else {
    B.bias[192 + p - OFF_B4] = x;
  }
}

__global__ void mlp_pack_kernel(MlpBufs B) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpNParam) pack_one(B, p, B.master[p]);
}

__global__ __launch_bounds__(64) void mlp_forward_kernel(MlpDev M, const float* __restrict__ x, int64_t n,
                                                         float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float lds[kMlpLdsBytes / 4];
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t r = base + threadIdx.x;
    float in[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (r < n)
#pragma unroll
      for (int c = 0; c < 6; ++c) in[c] = x[r * 6 + c];
    const float* raw = mlp_forward_wave(M, in, lds);
    if (r < n)
      for (int c = 0; c < kMlpOut; ++c) out[r * kMlpOut + c] = raw[c];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ training
constexpr int kA0Stride = 24;  // bf16 per row of the (16-wide, zero-padded) input block
constexpr int kGradWaves = 4;  // waves per 64-row tile of the gradient kernel

// Gradient of -log q(w) with respect to the 40 raw outputs (one row).
// Mixture terms in log space: log f_l = log kappa - log(2 pi (1 - e^{-2 kappa}))
// + kappa (mu.w - 1); the loss uses kappa = softplus + 0.01 without the
// sampler's upper clamp.
DEV float nll_grad(const float* raw, vec3 w, float g[kMlpOut]) {
  float mx = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) mx = fmaxf(mx, raw[5 * l + 4]);
  float es = 0.0f;
  float lw[kLobes], lf[kLobes], kap[kLobes], c[kLobes], nrm[kLobes], sg[kLobes];
  vec3 mu[kLobes];
#pragma unroll
  for (int l = 0; l < kLobes; ++l) {
    const vec3 v = v3(raw[5 * l], raw[5 * l + 1], raw[5 * l + 2]);
    nrm[l] = fmaxf(sqrtf(dot(v, v)), 1e-20f);
    mu[l] = v * (1.0f / nrm[l]);
    const float t = raw[5 * l + 3];
    kap[l] = (t > 30.0f ? t : log1pf(expf(t))) + 0.01f;
    sg[l] = 1.0f / (1.0f + expf(-t));
    lw[l] = raw[5 * l + 4] - mx;
    es += expf(lw[l]);
  }
  const float les = logf(es);
  float lq = -INFINITY;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) {
    lw[l] -= les;
    c[l] = dot(mu[l], w);
    lf[l] = logf(kap[l]) - logf(2.0f * kPi) - logf(-expm1f(-2.0f * kap[l])) + kap[l] * (c[l] - 1.0f);
    lq = fmaxf(lq, lw[l] + lf[l]);
  }
  float sq = 0.0f;
#pragma unroll
  for (int l = 0; l < kLobes; ++l) sq += expf(lw[l] + lf[l] - lq);
  lq += logf(sq);
#pragma unroll
  for (int l = 0; l < kLobes; ++l) {
    const float rl = expf(lw[l] + lf[l] - lq);  // responsibility of lobe l
    const float dk = 1.0f / kap[l] - 2.0f / expm1f(2.0f * kap[l]) + (c[l] - 1.0f);
    const float s = -rl * kap[l] / nrm[l];
    g[5 * l + 0] = s * (w.x - c[l] * mu[l].x);
    g[5 * l + 1] = s * (w.y - c[l] * mu[l].y);
    g[5 * l + 2] = s * (w.z - c[l] * mu[l].z);
    g[5 * l + 3] = -rl * dk * sg[l];
    g[5 * l + 4] = -(rl - expf(lw[l]));
  }
  return -lq;
}

// Tile (mt, nt) of a weight gradient: dst[i][j] (+)= sum over the 64 rows of
// X[row][i] G[row][j] for i in mt*16 .. +15, j in nt*16 .. +15 (the matrix
// cores reduce over rows: A = X^T, B = G).  X: bf16 rows of stride xs; G:
// bf16 rows of stride gs, or fp32 rows when GF32.
template <bool GF32>
DEV void grad_tile(const uint16_t* X, int xs, const void* G, int gs, float* dst, int ldd, int ni, int nj, bool first,
                   int mt, int nt) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = kt * 32 + 8 * g + e;
      a[e] = (short)X[row * xs + mt * 16 + r];
      if (GF32) b[e] = (short)f2bf(reinterpret_cast<const float*>(G)[row * gs + nt * 16 + r]);
      else b[e] = (short)reinterpret_cast<const uint16_t*>(G)[row * gs + nt * 16 + r];
    }
    acc = mfma32(a, b, acc);
  }
  const int j = nt * 16 + r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = mt * 16 + 4 * g + e;
    if (i < ni && j < nj) {
      float* d = dst + i * ldd + j;
      *d = first ? acc[e] : *d + acc[e];
    }
  }
}

// Back-propagated signal into features nt*16 .. nt*16 + 15 of a 64-wide
// layer: Gin[row][i] = [A[row][i] > 0] sum_o Gout[row][o] W[i][o] (W in
// [in][out] layout, ldw per row, KT*16 outputs), stored bf16; returns the
// column sums (the layer's bias gradient), valid in lanes 0..15 for columns
// nt*16 + lane.
template <int KT, bool GF32>
DEV float back_tile(const void* Gout, int gs, const uint16_t* __restrict__ w, int ldw, const uint16_t* A,
                    uint16_t* Gin, int nt) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  float cs = 0.0f;
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int row = mt * 16 + r;
#pragma unroll
    for (int kt = 0; kt < KT / 2; ++kt) {  // 32 outputs at a time
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int o = kt * 32 + 8 * g + e;
        if (GF32) a[e] = (short)f2bf(reinterpret_cast<const float*>(Gout)[row * gs + o]);
        else a[e] = (short)reinterpret_cast<const uint16_t*>(Gout)[row * gs + o];
      }
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(w + (nt * 16 + r) * ldw + kt * 32 + 8 * g);
      acc = mfma32(a, b, acc);
    }
    if constexpr (KT % 2 == 1) {  // the last 16 outputs
      bf16x4 a;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = (KT - 1) * 16 + 4 * g + e;
        if (GF32) a[e] = (short)f2bf(reinterpret_cast<const float*>(Gout)[row * gs + o]);
        else a[e] = (short)reinterpret_cast<const uint16_t*>(Gout)[row * gs + o];
      }
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(w + (nt * 16 + r) * ldw + (KT - 1) * 16 + 4 * g);
      acc = mfma(a, b, acc);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = mt * 16 + 4 * g + e, col = nt * 16 + r;
      const float v = A[row * kActStride + col] != 0 && !(A[row * kActStride + col] & 0x8000u) ? acc[e] : 0.0f;
      Gin[row * kActStride + col] = f2bf(v);
      cs += v;
    }
  }
  cs += __shfl_xor(cs, 16, 64);
  cs += __shfl_xor(cs, 32, 64);
  return cs;
}

// Gradient partials of the weighted NLL: block b accumulates the tiles
// b, b + grid, ... of 64 rows into partial[b][kMlpPartial] (the first tile
// overwrites); the last two words are the weighted loss and the weight sum.
// Records: {x[6], w_obj[3], weight} (10 floats).  Four waves share a tile:
// wave w runs the forward products of rows 16w .. 16w + 15, and in the
// backward pass the weight-gradient tiles of input features 16w .. 16w + 15
// and the signal into features 16w .. 16w + 15 (the first layer's output
// tile w); wave 0 alone does the per-row loss.  Every word of the partial
// has one writer, and the sums are those of one wave doing all the tiles.
__global__ __launch_bounds__(64 * kGradWaves) void mlp_grad_kernel(MlpDev M, const float* __restrict__ rec,
                                                                   int64_t nrec, int64_t rows, int sampled,
                                                                   uint32_t k0, uint32_t k1, uint32_t step,
                                                                   float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t A0[64 * kA0Stride];
  __shared__ __attribute__((aligned(16))) uint16_t A1[64 * kActStride];
  __shared__ __attribute__((aligned(16))) uint16_t A2[64 * kActStride];
  __shared__ __attribute__((aligned(16))) uint16_t A3[64 * kActStride];
  __shared__ __attribute__((aligned(16))) uint16_t GA[64 * kActStride];
  __shared__ __attribute__((aligned(16))) uint16_t GB[64 * kActStride];
  __shared__ __attribute__((aligned(16))) float OUT[64 * kOutStride];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* P = partial + (size_t)blockIdx.x * kMlpPartial;
  const int64_t ntiles = (rows + 63) / 64;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const bool first = tile == (int64_t)blockIdx.x;
    const int64_t row = tile * 64 + l;
    float wt = 0.0f;
    vec3 om = v3(0.f, 0.f, 1.f);
    if (wv == 0) {
      float x[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (row < rows) {
        int64_t ri = row;
        if (sampled)
          ri = (int64_t)(((uint64_t)philox((uint32_t)row, step, 0x5eedu, 0u, k0, k1).x * (uint64_t)nrec) >> 32);
        const float* R = rec + ri * 10;
#pragma unroll
        for (int c = 0; c < 6; ++c) x[c] = R[c];
        om = v3(R[6], R[7], R[8]);
        wt = R[9];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) A0[l * kA0Stride + c] = c < 6 ? f2bf(x[c]) : (uint16_t)0;
    }
    __syncthreads();
    mlp_tile<16, 4, false, kA0Stride>(A0, A1, M.wt1, M.b1, nullptr, wv);
    __syncthreads();
    mlp_tile<64, 4, false>(A1, A2, M.wt2, M.b2, nullptr, wv);
    __syncthreads();
    mlp_tile<64, 4, false>(A2, A3, M.wt3, M.b3, nullptr, wv);
    __syncthreads();
    mlp_tile<64, 3, true>(A3, nullptr, M.wt4, M.b4, OUT, wv);
    __syncthreads();
    if (wv == 0) {
      // output signal, weighted (normalised by the total weight at the reduction)
      float gr[kMlpOut];
      float loss = 0.0f;
      if (wt != 0.0f) loss = wt * nll_grad(OUT + l * kOutStride, om, gr);
      else
#pragma unroll
        for (int c = 0; c < kMlpOut; ++c) gr[c] = 0.0f;
#pragma unroll
      for (int c = 0; c < kOutStride; ++c) OUT[l * kOutStride + c] = c < kMlpOut ? wt * gr[c] : 0.0f;
      // loss and weight sums
      float ls = loss, ws = wt;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        ls += __shfl_xor(ls, off, 64);
        ws += __shfl_xor(ws, off, 64);
      }
      if (l == 0) {
        P[kMlpNParam] = first ? ls : P[kMlpNParam] + ls;
        P[kMlpNParam + 1] = first ? ws : P[kMlpNParam + 1] + ws;
      }
    }
    __syncthreads();
    // layer 4: db4 = column sums of the output signal, dW4 = A3^T G4
    if (wv == 0 && l < kMlpOut) {
      float cs = 0.0f;
      for (int q = 0; q < 64; ++q) cs += OUT[q * kOutStride + l];
      P[OFF_B4 + l] = first ? cs : P[OFF_B4 + l] + cs;
    }
#pragma unroll 1
    for (int nt = 0; nt < 3; ++nt)
      grad_tile<true>(A3, kActStride, OUT, kOutStride, P + OFF_W4, kMlpOut, 64, kMlpOut, first, wv, nt);
    float db = back_tile<3, true>(OUT, kOutStride, M.w4, 48, A3, GA, wv);
    if (l < 16) P[OFF_B3 + wv * 16 + l] = first ? db : P[OFF_B3 + wv * 16 + l] + db;
    __syncthreads();
    // layer 3
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt)
      grad_tile<false>(A2, kActStride, GA, kActStride, P + OFF_W3, 64, 64, 64, first, wv, nt);
    db = back_tile<4, false>(GA, kActStride, M.w3, 64, A2, GB, wv);
    if (l < 16) P[OFF_B2 + wv * 16 + l] = first ? db : P[OFF_B2 + wv * 16 + l] + db;
    __syncthreads();
    // layer 2
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt)
      grad_tile<false>(A1, kActStride, GB, kActStride, P + OFF_W2, 64, 64, 64, first, wv, nt);
    db = back_tile<4, false>(GB, kActStride, M.w2, 64, A1, GA, wv);
    if (l < 16) P[OFF_B1 + wv * 16 + l] = first ? db : P[OFF_B1 + wv * 16 + l] + db;
    __syncthreads();
    // layer 1 (inputs 0..5 of the padded 16): output tile wv
    grad_tile<false>(A0, kA0Stride, GA, kActStride, P + OFF_W1, 64, kMlpIn, 64, first, 0, wv);
    __syncthreads();
  }
}

// Sums over the blocks' partials.  A workgroup of kRedWaves waves owns the 64
// entries p0 .. p0 + 63 (lane l: entry p0 + l); wave w adds the blocks
// b = w, w + kRedWaves, ... in increasing order, then the wave sums are added
// in wave order.  The weight sum W (entry kMlpNParam + 1), which every entry
// divides by, is formed in every workgroup in the same fixed order (thread t
// adds the blocks t, t + 512, ...; a butterfly over each wave, whose lanes all
// end with the same value; the wave sums in wave order).  The result does not
// depend on scheduling.  Returns the entry's sum to the lanes of wave 0.
constexpr int kRedWaves = 8;
constexpr int kRedThreads = 64 * kRedWaves;
constexpr int kRedEntries = kMlpPartial;  // parameters, loss, weight sum

DEV float sum_blocks(const float* __restrict__ partial, int blocks, int p, float* lds, float& W) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  float s = 0.0f;
  if (p < kRedEntries) {
#pragma unroll 8
    for (int b = w; b < blocks; b += kRedWaves) s += partial[(size_t)b * kMlpPartial + p];
  }
  float ws = 0.0f;
  for (int b = threadIdx.x; b < blocks; b += kRedThreads) ws += partial[(size_t)b * kMlpPartial + kMlpNParam + 1];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ws += __shfl_xor(ws, off, 64);
  lds[w * 64 + l] = s;
  if (l == 0) lds[kRedThreads + w] = ws;
  __syncthreads();
  W = 0.0f;
#pragma unroll
  for (int k = 0; k < kRedWaves; ++k) W += lds[kRedThreads + k];
  float t = 0.0f;
  if (w == 0)
#pragma unroll
    for (int k = 0; k < kRedWaves; ++k) t += lds[k * 64 + l];
  return t;
}

__global__ __launch_bounds__(kRedThreads) void mlp_reduce_kernel(const float* __restrict__ partial, int blocks,
                                                                 float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ float lds[kRedThreads + kRedWaves];
  const int p = blockIdx.x * 64 + (threadIdx.x & 63);
  float W;
  const float s = sum_blocks(partial, blocks, p, lds, W);
  if (threadIdx.x >= 64) return;
  const float inv = W > 0.0f ? 1.0f / W : 0.0f;
  if (p < kMlpNParam) grad[p] = s * inv;
  else if (p == kMlpNParam && loss) *loss = s * inv;
}

// Adam (Kingma and Ba 2015) on the FP32 masters, then the kernels' copies.
__global__ __launch_bounds__(kRedThreads) void mlp_adam_kernel(const float* __restrict__ partial, int blocks, MlpBufs B,
                                                               float lr, float beta1, float beta2, float eps, int t,
                                                               float* __restrict__ loss_out) {
  __shared__ float lds[kRedThreads + kRedWaves];
  const int p = blockIdx.x * 64 + (threadIdx.x & 63);
  float W;
  const float s = sum_blocks(partial, blocks, p, lds, W);
  if (threadIdx.x >= 64 || !(W > 0.0f)) return;
  if (p == kMlpNParam) {
    if (loss_out) *loss_out = s / W;
    return;
  }
  if (p > kMlpNParam) return;
  const float g = s / W;
  const float m = beta1 * B.adam_m[p] + (1.0f - beta1) * g;
  const float v = beta2 * B.adam_v[p] + (1.0f - beta2) * g * g;
  B.adam_m[p] = m;
  B.adam_v[p] = v;
  const float mh = m / (1.0f - powf(beta1, (float)t)), vh = v / (1.0f - powf(beta2, (float)t));
  const float x = B.master[p] - lr * mh / (sqrtf(vh) + eps);
  B.master[p] = x;
  pack_one(B, p, x);
}

// ------------------------------------------------------------------ launchers
void launch_mlp_pack(const MlpBufs& B, hipStream_t st) {
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((kMlpNParam + 255) / 256), dim3(256), 0, st, B);
}
void launch_mlp_forward(const MlpDev& M, const float* x, int64_t n, float* out, hipStream_t st) {
  const int64_t tiles = (n + 63) / 64;
  const int blocks = (int)std::min<int64_t>(tiles, 4096);
  if (blocks > 0) hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(64), 0, st, M, x, n, out);
}
void launch_mlp_grad(const MlpDev& M, const float* rec, int64_t nrec, int64_t rows, int sampled, uint32_t k0,
                     uint32_t k1, uint32_t step, float* partial, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(64 * kGradWaves), 0, st, M, rec, nrec, rows, sampled, k0, k1,
                     step, partial);
}
void launch_mlp_reduce(const float* partial, int blocks, float* grad, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kRedEntries + 63) / 64), dim3(kRedThreads), 0, st, partial, blocks, grad,
                     loss);
}
void launch_mlp_adam(const float* partial, int blocks, const MlpBufs& B, float lr, float beta1, float beta2, float eps,
                     int t, float* loss_out, hipStream_t st) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kRedEntries + 63) / 64), dim3(kRedThreads), 0, st, partial, blocks, B, lr,
                     beta1, beta2, eps, t, loss_out);
}

}  // namespace rpi
