// Residual-aware denoising of a residual image (gfx950, wave64).
//
// The paper attributes its remaining artefacts to the noise of the
// residual around the edit and leaves denoising to an external tool
// (Sec. 6, limitations; Sec. 7).  This is the library's own filter: an
// edge-avoiding a-trous wavelet transform (Dammertz et al. 2010) with the
// variance-guided luminance weight of spatiotemporal variance-guided
// filtering (Schied et al. 2017), applied to the residual rather than to a
// frame.  Its variance comes from two independent half estimates a, b of
// the residual (R = a + b, Var R ~ (a - b)^2), so pixels that no dynamic
// path reached (a = b = 0) have zero variance and keep their exact zero:
// the filter does not smear the edit into the static image.
//
//   gbuffer_kernel   one camera ray per pixel centre in the new frame:
//                    geometric normal facing the camera, hit distance
//   denoise_init     R = a + b, v = mean over channels of (a - b)^2
//   atrous_kernel    one 5x5 B3-spline pass at stride 2^i with normal,
//                    depth and luminance edge-stopping weights; the
//                    variance goes through with squared weights
#include "rpi_device.h"

namespace rpi {

__global__ __launch_bounds__(kTraceBlock) void gbuffer_kernel(DevScene S, DevFrame F, float4* g) {
  __shared__ __attribute__((aligned(16))) int stk[kStackDepth * kTraceBlock];
  const DevCamera& C = S.cam;
  const int P = C.W * C.H;
  const int pixel = blockIdx.x * kTraceBlock + threadIdx.x;
  if (pixel >= P) return;
  WorkCount wc{};
  const vec3 w = camera_dir(C, pixel, 0.5f, 0.5f);
  const Hit h = closest<false>(S, F, C.eye, w, stk, wc);
  if (!h.ok) {
    g[pixel] = make_float4(0.f, 0.f, 0.f, -1.f);
    return;
  }
  vec3 p, n;
  uint32_t md;
  hit_vertex(S, F.pose, h, C.eye, w, p, n, md);
  if (dot(n, w) > 0.0f) n = v3(-n.x, -n.y, -n.z);
  g[pixel] = make_float4(n.x, n.y, n.z, h.t);
}

__global__ __launch_bounds__(256) void denoise_init(const float* a, const float* b, float4* x, int P) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= P) return;
  const float ar = a[3 * i], ag = a[3 * i + 1], ab = a[3 * i + 2];
  const float br = b[3 * i], bg = b[3 * i + 1], bb = b[3 * i + 2];
  const float dr = ar - br, dg = ag - bg, db = ab - bb;
  x[i] = make_float4(ar + br, ag + bg, ab + bb, (dr * dr + dg * dg + db * db) * (1.0f / 3.0f));
}

struct AtrousArgs {
  const float4* in;   // rgb + variance
  float4* out;
  const float4* g;    // normal + distance (< 0: no hit)
  float* image;       // last pass: rgb out (H x W x 3), else null
  int W, H, stride;
  float sigma_n, sigma_z, sigma_l;
};

DEV float b3(int k) { return k == 0 ? 0.375f : (k == 1 || k == -1 ? 0.25f : 0.0625f); }

__global__ __launch_bounds__(256) void atrous_kernel(AtrousArgs A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.W * A.H) return;
  const int px = i % A.W, py = i / A.W;
  const float4 c = A.in[i];
  const float4 gc = A.g[i];
  // the variance that scales the luminance weight: a 3x3 Gaussian of it
  float vb = 0.0f, vw = 0.0f;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int qx = px + dx, qy = py + dy;
      if (qx < 0 || qx >= A.W || qy < 0 || qy >= A.H) continue;
      const float k = (dx == 0 ? 0.5f : 0.25f) * (dy == 0 ? 0.5f : 0.25f);
      vb += k * A.in[qy * A.W + qx].w;
      vw += k;
    }
  const float sd = sqrtf(fmaxf(vb / vw, 0.0f));
  const float lc = (c.x + c.y + c.z) * (1.0f / 3.0f);
  float sw = 0.0f, sr = 0.0f, sg = 0.0f, sbl = 0.0f, sv = 0.0f;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      const int qx = px + dx * A.stride, qy = py + dy * A.stride;
      if (qx < 0 || qx >= A.W || qy < 0 || qy >= A.H) continue;
      const int q = qy * A.W + qx;
      const float4 x = A.in[q];
      const float4 gq = A.g[q];
      float w = b3(dx) * b3(dy);
      if (dx != 0 || dy != 0) {
        // geometry: both rays miss, or both hit with similar normals and distances
        if ((gc.w < 0.0f) != (gq.w < 0.0f)) continue;
        if (gc.w >= 0.0f) {
          const float nd = fmaxf(0.0f, gc.x * gq.x + gc.y * gq.y + gc.z * gq.z);
          w *= powf(nd, A.sigma_n);
          w *= expf(-fabsf(gc.w - gq.w) / (A.sigma_z * gc.w + 1e-6f));
        }
        // residual value: differences beyond sigma_l standard deviations of
        // the centre's estimate are edges (zero variance: only equal values)
        const float lq = (x.x + x.y + x.z) * (1.0f / 3.0f);
        const float dl = fabsf(lc - lq);
        if (dl > 0.0f) w = sd > 0.0f ? w * expf(-dl / (A.sigma_l * sd)) : 0.0f;
      }
      sw += w;
      sr += w * x.x;
      sg += w * x.y;
      sbl += w * x.z;
      sv += w * w * x.w;
    }
  const float inv = 1.0f / sw;  // the centre tap alone gives sw >= 0.140625
  const float4 o = make_float4(sr * inv, sg * inv, sbl * inv, sv * inv * inv);
  A.out[i] = o;
  if (A.image) {
    A.image[3 * i] = o.x;
    A.image[3 * i + 1] = o.y;
    A.image[3 * i + 2] = o.z;
  }
}

void launch_gbuffer(const DevScene& S, const DevFrame& F, float4* g, hipStream_t st) {
  const int P = S.cam.W * S.cam.H;
  hipLaunchKernelGGL(gbuffer_kernel, dim3((P + kTraceBlock - 1) / kTraceBlock), dim3(kTraceBlock), 0, st, S, F, g);
}

void launch_denoise(const float* a, const float* b, const float4* g, float4* buf0, float4* buf1, int W, int H,
                    int iterations, float sigma_n, float sigma_z, float sigma_l, float* out, hipStream_t st) {
  const int P = W * H;
  const dim3 grid((P + 255) / 256);
  hipLaunchKernelGGL(denoise_init, grid, dim3(256), 0, st, a, b, buf0, P);
  float4* in = buf0;
  float4* o = buf1;
  for (int it = 0; it < iterations; ++it) {
    AtrousArgs A{in, o, g, it + 1 == iterations ? out : nullptr, W, H, 1 << it, sigma_n, sigma_z, sigma_l};
    hipLaunchKernelGGL(atrous_kernel, grid, dim3(256), 0, st, A);
    float4* t = in;
    in = o;
    o = t;
  }
}

}  // namespace rpi
