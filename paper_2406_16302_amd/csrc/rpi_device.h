// Device-side building blocks of the residual path estimator for gfx950:
// counter-based RNG, BSDFs, pinhole camera, light sampling (guide-table CDF
// picks), 4-wide BVH traversal with a per-lane LDS stack, ghost-crossing records.
#pragma once

#include "rpi_internal.h"

namespace rpi {

#define DEV __device__ __forceinline__

constexpr int kWave = 64;       // wavefront width on CDNA
constexpr int kTraceBlock = 64; // one wave per workgroup for the trace-heavy kernels
constexpr float kPi = 3.14159265358979323846f;

// ------------------------------------------------------------------ Philox4x32-10
// Salmon et al., SC'11.  Counter = (sample, tech<<24 | dir<<23 | side<<22 |
// bounce<<8 | slot, job, 0); key = seed.
struct Rng {
  uint32_t k0, k1, sample, hi, job;
};
DEV uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}
DEV void draw(const Rng& g, uint32_t side, uint32_t bounce, uint32_t slot, float u[4]) {
  const uint4 x = philox(g.sample, g.hi | (side << 22) | (bounce << 8) | slot, g.job, 0u, g.k0, g.k1);
  const float s = 1.0f / 16777216.0f;
  u[0] = (float)(x.x >> 8) * s;
  u[1] = (float)(x.y >> 8) * s;
  u[2] = (float)(x.z >> 8) * s;
  u[3] = (float)(x.w >> 8) * s;
}

// ------------------------------------------------------------------ materials
// Vertex material word: bit 31 = on the object, low bits = material index.
constexpr uint32_t kDynBit = 0x80000000u;

DEV Material load_mat(const float* m) {
  Material r;
  r.type = (int)m[0];
  r.albedo = v3(m[1], m[2], m[3]);
  r.rough = m[4];
  r.emit = v3(m[5], m[6], m[7]);
  return r;
}
DEV Material vmat(const DevScene& S, const DevFrame& F, uint32_t md) {
  return (md & kDynBit) ? F.objmat : load_mat(S.mats + 8 * (md & ~kDynBit));
}
DEV float roughness(const Material& m) { return m.type == MAT_GGX ? m.rough : 1.0f; }

// Duff et al. 2017, "Building an orthonormal basis, revisited".
DEV void onb(vec3 n, vec3& t, vec3& b) {
  const float sign = copysignf(1.0f, n.z);
  const float a = -1.0f / (sign + n.z);
  const float c = n.x * n.y * a;
  t = v3(1.0f + sign * n.x * n.x * a, sign * c, -sign * n.x);
  b = v3(c, sign + n.y * n.y * a, -n.y);
}

DEV float ggx_D(float a, float nh) {
  const float a2 = a * a;
  const float k = nh * nh * (a2 - 1.0f) + 1.0f;
  return a2 / (kPi * k * k);
}
DEV float ggx_G1(float a, float c) {
  c = fabsf(c);
  const float t2 = (1.0f - c * c) / (c * c);
  return 2.0f / (1.0f + sqrtf(1.0f + a * a * t2));
}

// rho(wi <-> wo): two-sided, reflection only (Lambertian or GGX conductor
// with Smith G and Schlick F); wi, wo unit directions away from the surface.
DEV vec3 bsdf_eval(const Material& m, vec3 n, vec3 wi, vec3 wo) {
  const float ci = dot(n, wi), co = dot(n, wo);
  if (!(ci * co > 0.0f)) return v3(0, 0, 0);
  if (m.type == MAT_DIFFUSE) return m.albedo * (1.0f / kPi);
  if (m.type != MAT_GGX) return v3(0, 0, 0);
  const vec3 ns = ci > 0.0f ? n : -n;
  const vec3 h = unit(wi + wo);
  const float nh = dot(ns, h), ih = fabsf(dot(wi, h));
  const float D = ggx_D(m.rough, nh);
  const float G = ggx_G1(m.rough, ci) * ggx_G1(m.rough, co);
  const float s1 = 1.0f - ih, s2 = s1 * s1, s5 = s2 * s2 * s1;
  const float k = D * G / (4.0f * fabsf(ci) * fabsf(co));
  return v3((m.albedo.x + (1.0f - m.albedo.x) * s5) * k, (m.albedo.y + (1.0f - m.albedo.y) * s5) * k,
            (m.albedo.z + (1.0f - m.albedo.z) * s5) * k);
}
// Solid-angle pdf of sampling wo given wi.
DEV float bsdf_pdf(const Material& m, vec3 n, vec3 wi, vec3 wo) {
  const float ci = dot(n, wi), co = dot(n, wo);
  if (!(ci * co > 0.0f)) return 0.0f;
  if (m.type == MAT_DIFFUSE) return fabsf(co) * (1.0f / kPi);
  if (m.type != MAT_GGX) return 0.0f;
  const vec3 ns = ci > 0.0f ? n : -n;
  const vec3 h = unit(wi + wo);
  const float nh = dot(ns, h);
  return ggx_D(m.rough, nh) * nh / (4.0f * fabsf(dot(wo, h)));
}
// Cosine lobe (Lambertian) or GGX half-vector sampling (Walter et al. 2007)
// on the side of wi.
DEV bool bsdf_sample(const Material& m, vec3 n, vec3 wi, float u0, float u1, vec3& wo) {
  const float ci = dot(n, wi);
  if (ci == 0.0f || m.type == MAT_EMITTER) return false;
  const vec3 ns = ci > 0.0f ? n : -n;
  vec3 t, b;
  onb(ns, t, b);
  const float ph = 2.0f * kPi * u1;
  float sp, cp;
  sincosf(ph, &sp, &cp);
  if (m.type == MAT_DIFFUSE) {
    const float r = sqrtf(u0);
    const float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
    wo = t * (r * cp) + b * (r * sp) + ns * z;
    return dot(wo, ns) > 0.0f;
  }
  const float a = m.rough;
  const float t2 = a * a * u0 / (1.0f - u0);
  const float ct = 1.0f / sqrtf(1.0f + t2);
  const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  const vec3 h = t * (st * cp) + b * (st * sp) + ns * ct;
  const float ih = dot(wi, h);
  wo = h * (2.0f * ih) - wi;
  return dot(wo, ns) > 0.0f;
}

DEV vec3 cosine_dir(vec3 n, float u0, float u1) {
  vec3 t, b;
  onb(n, t, b);
  float sp, cp;
  sincosf(2.0f * kPi * u1, &sp, &cp);
  const float r = sqrtf(u0), z = sqrtf(fmaxf(0.0f, 1.0f - u0));
  return t * (r * cp) + b * (r * sp) + n * z;
}
DEV vec3 sphere_dir(float u0, float u1) {
  const float z = 1.0f - 2.0f * u0;
  const float r = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  float sp, cp;
  sincosf(2.0f * kPi * u1, &sp, &cp);
  return v3(r * cp, r * sp, z);
}

// ------------------------------------------------------------------ camera
DEV int raster(const DevCamera& C, vec3 p) {
  const vec3 d = p - C.eye;
  const float z = dot(d, C.fwd);
  if (!(z > 0.0f)) return -1;
  const float sx = dot(d, C.right) / z, sy = dot(d, C.up) / z;
  const float fx = (sx / (C.aspect * C.tan_half) + 1.0f) * 0.5f * (float)C.W;
  const float fy = (1.0f - sy / C.tan_half) * 0.5f * (float)C.H;
  if (!(fx >= 0.0f && fx < (float)C.W && fy >= 0.0f && fy < (float)C.H)) return -1;
  const int px = min((int)fx, C.W - 1), py = min((int)fy, C.H - 1);
  return py * C.W + px;
}
DEV vec3 camera_dir(const DevCamera& C, int pixel, float u0, float u1) {
  const int px = pixel % C.W, py = pixel / C.W;
  const float sx = (2.0f * (((float)px + u0) / (float)C.W) - 1.0f) * C.aspect * C.tan_half;
  const float sy = (1.0f - 2.0f * (((float)py + u1) / (float)C.H)) * C.tan_half;
  return unit(C.fwd + C.right * sx + C.up * sy);
}
// W_j G(x0, x1) = P / (A_film cos^3) * |cos_1| / r^2 and the whole-image
// sampling pdf of x1 (area measure): the same with P replaced by 1.
DEV float camera_geo(const DevCamera& C, vec3 x1, vec3 n1) {
  const vec3 d = x1 - C.eye;
  const float r2 = len2(d);
  const vec3 w = unit(d);
  const float cc = dot(w, C.fwd);
  return fabsf(dot(n1, w)) / (C.a_film * cc * cc * cc * r2);
}
DEV float camera_geo_dir(const DevCamera& C, vec3 w) {
  const float cc = dot(w, C.fwd);
  return 1.0f / (C.a_film * cc * cc * cc);
}

// ------------------------------------------------------------------ offsets
DEV vec3 spawn(const DevScene& S, vec3 p, vec3 n, vec3 towards) {
  const float s = dot(n, towards - p) >= 0.0f ? 1.0f : -1.0f;
  return p + n * (s * S.eps);
}
DEV vec3 spawn_dir(const DevScene& S, vec3 p, vec3 n, vec3 dir) {
  const float s = dot(n, dir) >= 0.0f ? 1.0f : -1.0f;
  return p + n * (s * S.eps);
}

// A ray from point p on the object (geometric normal n) in direction dir
// leaves the object for good when the object is convex and dir points to the
// outer side of the face, the side away from a point inside (its centre at
// this pose): the object's BVH can be skipped for it.
DEV bool leaves_convex(const DevScene& S, const Pose& pose, vec3 p, vec3 n, vec3 dir) {
  if (!S.obj_convex) return false;
  const vec3 c = pose_apply(pose, S.obj_center);
  return dot(n, p - c) * dot(n, dir) > 0.0f;
}

// A ray or segment from point p on a sealed object (below) into the object's
// inner side: blocked by the object, or into its inside for good.
DEV bool into_sealed(const DevScene& S, const DevFrame& F, vec3 p, vec3 n, vec3 dir) {
  if (!F.sealed) return false;
  const vec3 c = pose_apply(F.pose, S.obj_center);
  return dot(n, p - c) * dot(n, dir) < 0.0f;
}

// A hit q on a sealed object (closed, convex, camera and emitters outside)
// whose ray came from the inner side of q's face (from: the ray's start)
// is inside the object for good: every later vertex of its walk is too, and
// no path through them can reach the camera or an emitter.  Walks stop there.
DEV bool interior_hit(const DevScene& S, const DevFrame& F, vec3 q, vec3 qn, uint32_t qmd, vec3 from) {
  if (!F.sealed || !(qmd & kDynBit)) return false;
  const vec3 c = pose_apply(F.pose, S.obj_center);
  return dot(qn, from - q) * dot(qn, c - q) > 0.0f;
}

// x lies inside a sealed object (in the ball about its centre that the
// object contains): a ray from outside must cross the object before x, and
// rays from x cannot leave it.
DEV bool deep_inside(const DevScene& S, const DevFrame& F, vec3 x) {
  if (!F.sealed) return false;
  const vec3 d = x - pose_apply(F.pose, S.obj_center);
  return dot(d, d) < S.obj_rin * S.obj_rin;
}

// ------------------------------------------------------------------ triangles

// Scene arrays are reached through pointers read from the job table, which
// the compiler would load with flat instructions; these go through the
// global address space.
typedef float gf4 __attribute__((ext_vector_type(4)));
typedef int gi4 __attribute__((ext_vector_type(4)));
DEV float4 gld(const float4* p, size_t i) {
  const gf4 v = ((const __attribute__((address_space(1))) gf4*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
DEV int4 gld(const int4* p, size_t i) {
  const gi4 v = ((const __attribute__((address_space(1))) gi4*)p)[i];
  return make_int4(v.x, v.y, v.z, v.w);
}
DEV void load_tri(const float4* __restrict__ T, int i, vec3& v0, vec3& e1, vec3& e2, int& id, int& mat) {
  const float4 a = gld(T, 3 * (size_t)i), b = gld(T, 3 * (size_t)i + 1), c = gld(T, 3 * (size_t)i + 2);
  v0 = v3(a.x, a.y, a.z);
  e1 = v3(b.x, b.y, b.z);
  e2 = v3(c.x, c.y, c.z);
  id = __float_as_int(a.w);
  mat = __float_as_int(b.w);
}
// Moller-Trumbore; t > 0 or -1.
DEV float tri_t(vec3 o, vec3 d, vec3 v0, vec3 e1, vec3 e2) {
  const vec3 p = cross(d, e2);
  const float det = dot(e1, p);
  if (det == 0.0f) return -1.0f;
  const float inv = 1.0f / det;
  const vec3 s = o - v0;
  const float u = dot(s, p) * inv;
  if (u < 0.0f || u > 1.0f) return -1.0f;
  const vec3 q = cross(s, e1);
  const float v = dot(d, q) * inv;
  if (v < 0.0f || u + v > 1.0f) return -1.0f;
  const float t = dot(e2, q) * inv;
  return t > 0.0f ? t : -1.0f;
}

// ------------------------------------------------------------------ BVH traversal
// Work counters of the instrumented kernel variants (CW = true).
enum { RAY_CLOSEST = 0, RAY_SHADOW = 1, RAY_CAMERA = 2, RAY_GHOST = 3, RAY_RETRACE = 4, RAY_MAPVIS = 5 };
struct WorkCount {
  uint32_t nodes, tris, bytes;
  uint32_t rays[6];
};

// Slab test of one box; fminf/fmaxf drop the NaNs of 0 * inf.  The host pads
// every box, so FMA contraction here can only widen the accepted set.
DEV bool slab(float lx, float ly, float lz, float hx, float hy, float hz, vec3 inv, vec3 oi, float tlim,
              float& tnear) {
#pragma clang fp contract(fast)
  const float ax = lx * inv.x - oi.x, bx = hx * inv.x - oi.x;
  const float ay = ly * inv.y - oi.y, by = hy * inv.y - oi.y;
  const float az = lz * inv.z - oi.z, bz = hz * inv.z - oi.z;
  const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
  const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tlim));
  tnear = t0;
  return t0 <= t1;
}

// A ray with a NaN in its origin or direction meets no triangle (every
// comparison of its hit tests is false) but every box (the slab test's
// min/max drop the NaNs), so its traversal would visit the whole BVH to find
// nothing: the traversals end it before the first node, with the same
// result.
DEV bool ray_ok(vec3 o, vec3 d) {
  return (o.x == o.x) & (o.y == o.y) & (o.z == o.z) & (d.x == d.x) & (d.y == d.y) & (d.z == d.z);
}

// One visit of a 4-wide node: test(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, tnear)
// says whether the ray meets a child's box.  ORDER: the nearest child met is
// returned and the others go on the lane's stack, the farthest first
// (deepest), so the next nearest is popped first (closest-hit queries find
// their hit sooner and cull more); without ORDER the children are taken in
// slot order: all-hit queries visit every box met anyway, and so does an
// any-hit query whose segment is clear (any_in; for the blocked ones the
// sort costs more than it saves).  With no child met the next entry is
// popped (kDone once the stack is empty).  At most (children - 1) entries
// are pushed.
constexpr int kDone = 0x7fffffff;  // no node left (inner node indices stay below it)
template <bool ORDER = true, class Test>
DEV int visit4(const float4* __restrict__ N, int node, int* __restrict__ stk, int& sp, Test&& test) {
  const size_t b = (size_t)kNodeF4 * (size_t)node;
  const float4 lx = gld(N, b), hx = gld(N, b + 1), ly = gld(N, b + 2), hy = gld(N, b + 3), lz = gld(N, b + 4),
               hz = gld(N, b + 5);
  const int4 e = gld(reinterpret_cast<const int4*>(N), b + 6);
  const int lane = threadIdx.x;
  const float inf = __builtin_inff();
  // entry distance of each child met, +inf for the others (a box met has a
  // finite entry distance); no branch per child
  auto key = [&](float lox, float loy, float loz, float hix, float hiy, float hiz, int link) {
    float t;
    const bool h = test(lox, loy, loz, hix, hiy, hiz, t) & (link != kEmptyLink);
    return h ? t : inf;
  };
  float d0 = key(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, e.x);
  float d1 = key(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, e.y);
  float d2 = key(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, e.z);
  float d3 = key(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, e.w);
  int c0 = e.x, c1 = e.y, c2 = e.z, c3 = e.w;
  if constexpr (ORDER) {
    // sorting network on (distance, link): 0-1, 2-3, 0-2, 1-3, 1-2
    auto cas = [](float& da, int& ca, float& db, int& cb) {
      const bool sw = db < da;
      const float td = sw ? db : da;
      db = sw ? da : db;
      da = td;
      const int tc = sw ? cb : ca;
      cb = sw ? ca : cb;
      ca = tc;
    };
    cas(d0, c0, d1, c1);
    cas(d2, c2, d3, c3);
    cas(d0, c0, d2, c2);
    cas(d1, c1, d3, c3);
    cas(d1, c1, d2, c2);
  }
  if (d3 < inf) stk[sp++ * kTraceBlock + lane] = c3;
  if (d2 < inf) stk[sp++ * kTraceBlock + lane] = c2;
  if (d1 < inf) stk[sp++ * kTraceBlock + lane] = c1;
  if (d0 < inf) return c0;
  return sp > 0 ? stk[--sp * kTraceBlock + lane] : kDone;
}

// Visit every leaf whose box the ray (o, d) meets before tlim (read through
// a reference, so closest-hit leaves tighten it).  leaf(code) returns true to
// stop.  The stack lives in LDS: entry k of lane l at stk[k * kTraceBlock + l];
// it holds inner nodes and leaves alike.
// While-while traversal with speculative node visits (Aila and Laine 2009):
// a lane that meets its first leaf postpones it and keeps visiting inner
// nodes until every lane of the wave holds a leaf (or a lane meets a second
// one); then the wave tests its leaves together.  The triangle loop runs
// with the lanes of all leaves instead of one branch per node visit, and
// lanes that found a leaf early do useful node work meanwhile.  A
// closest-hit query may visit a few nodes that the postponed leaf's hit
// would have culled; the hit found is the same.  ORDER: nearest child first
// (false for any-hit and all-hit queries).
template <bool CW, bool ORDER = true, class Leaf>
DEV void bvh_walk(const float4* __restrict__ N, vec3 o, vec3 d, const float& tlim, int* __restrict__ stk,
                     WorkCount& wc, Leaf&& leaf) {
  const vec3 inv = v3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
  const vec3 oi = v3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
  const int lane = threadIdx.x;
  int sp = 0;
  int node = ray_ok(o, d) ? 0 : kDone;  // >= 0: inner node to visit next; < 0: a leaf code; kDone
  int pl = 0;    // postponed leaf code, 0: none
  auto test = [&](float lx, float ly, float lz, float hx, float hy, float hz, float& tn) {
    return slab(lx, ly, lz, hx, hy, hz, inv, oi, tlim, tn);
  };
  while (node != kDone) {
    while ((uint32_t)node < (uint32_t)kDone) {
      if (CW) wc.nodes++;
      node = visit4<ORDER>(N, node, stk, sp, test);
      if (node < 0 && pl == 0) {  // postpone the first leaf and go on with the stack
        pl = node;
        node = sp > 0 ? stk[--sp * kTraceBlock + lane] : kDone;
      }
      if (__ballot(pl == 0) == 0ull) break;  // every lane still here holds a leaf
    }
    while (pl < 0) {
      if (leaf(pl)) return;
      pl = 0;
      if (node < 0) {
        pl = node;
        node = sp > 0 ? stk[--sp * kTraceBlock + lane] : kDone;
      }
    }
  }
}

DEV int leaf_first(int code) { return (int)(((uint32_t)code & 0x7fffffffu) >> 4); }
DEV int leaf_count(int code) { return code & 15; }

DEV bool box_hit(vec3 lo, vec3 hi, vec3 o, vec3 d, float tlim) {
  const vec3 inv = v3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
  const vec3 oi = v3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
  float tn;
  return slab(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, inv, oi, tlim, tn);
}

// Whether the segment o + t d, 0 < t < tlim, comes within radius r of c
// (a cheap cull before an object's BVH; the sphere is padded).
DEV bool sphere_near(vec3 c, float r, vec3 o, vec3 d, float tlim) {
  const vec3 oc = c - o;
  const float dd = dot(d, d);
  float t = dot(oc, d) / dd;
  t = fminf(fmaxf(t, 0.0f), tlim);
  const vec3 x = o + d * t - c;
  return dot(x, x) <= r * r;
}

struct Hit {
  float t;
  int id;    // input triangle index
  int idx;   // index in its BVH's triangle array
  int dyn;   // 1: on the object
  int ok;
};

template <bool CW>
DEV void closest_in(const DevBvh& B, vec3 o, vec3 d, Hit& h, int dyn, int* stk, WorkCount& wc, float tstop) {
  bvh_walk<CW>(B.nodes, o, d, h.t, stk, wc, [&](int code) {
    const int f = leaf_first(code), n = leaf_count(code);
    for (int i = f; i < f + n; ++i) {
      vec3 v0, e1, e2;
      int id, mat;
      load_tri(B.tris, i, v0, e1, e2, id, mat);
      if (CW) wc.tris++;
      const float t = tri_t(o, d, v0, e1, e2);
      if (t > 0.0f && (t < h.t || (t == h.t && id < h.id))) {
        h.t = t;
        h.id = id;
        h.idx = i;
        h.dyn = dyn;
        h.ok = 1;
      }
    }
    return h.t <= tstop;
  });
}

// Whether a ray may meet the object of frame F: its padded box and
// bounding sphere, both tested against o + t d, 0 < t < tlim.
DEV bool near_object(const DevFrame& F, vec3 o, vec3 d, float tlim) {
  return box_hit(F.olo, F.ohi, o, d, tlim) && sphere_near(F.oc, F.orad, o, d, tlim);
}
DEV bool near_ghost(const DevFrame& F, vec3 o, vec3 d, float tlim) {
  return box_hit(F.glo, F.ghi, o, d, tlim) && sphere_near(F.gc, F.orad, o, d, tlim);
}

// Closest hit in scene_f: static geometry plus the object at F's pose.
// noobj: the ray leaves the convex object it starts on (leaves_convex).
// tstop: the caller rejects any hit at t <= tstop, so the search may end
// as soon as it has one (the hit returned is then not the closest).
template <bool CW>
DEV Hit closest(const DevScene& S, const DevFrame& F, vec3 o, vec3 d, int* stk, WorkCount& wc,
                int ray_type = RAY_CLOSEST, bool noobj = false, float tstop = -1.0f) {
  const Pose& pose = F.pose;
  if (CW) wc.rays[ray_type]++;
  Hit h;
  h.t = INFINITY;
  h.id = 0x7fffffff;
  h.idx = -1;
  h.dyn = 0;
  h.ok = 0;
  closest_in<CW>(S.stat, o, d, h, 0, stk, wc, tstop);
  if (!noobj && h.t > tstop && near_object(F, o, d, h.t))
    closest_in<CW>(S.obj, pose_inv_apply(pose, o), pose_inv_rot(pose, d), h, 1, stk, wc, tstop);
  return h;
}

// Both closest hits of the line o + t d: hf along d (t > 0) and hb along -d
// (t < 0, hb.t = -t), in one traversal.  tri_t and the slab test are odd in
// d (every product and sum in them changes sign exactly), so hf and hb are
// bit for bit the hits of two closest-hit queries along d and -d.
DEV bool slab_line(float lx, float ly, float lz, float hx, float hy, float hz, vec3 inv, vec3 oi, float tf, float tb,
                   float& tnear) {
#pragma clang fp contract(fast)
  const float ax = lx * inv.x - oi.x, bx = hx * inv.x - oi.x;
  const float ay = ly * inv.y - oi.y, by = hy * inv.y - oi.y;
  const float az = lz * inv.z - oi.z, bz = hz * inv.z - oi.z;
  const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), -tb));
  const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tf));
  tnear = fabsf(t0) < fabsf(t1) ? fabsf(t0) : fabsf(t1);
  return t0 <= t1;
}

// tri_t without the sign test: the line parameter of the hit, or NaN.
DEV float tri_line(vec3 o, vec3 d, vec3 v0, vec3 e1, vec3 e2) {
  const vec3 p = cross(d, e2);
  const float det = dot(e1, p);
  if (det == 0.0f) return __builtin_nanf("");
  const float inv = 1.0f / det;
  const vec3 s = o - v0;
  const float u = dot(s, p) * inv;
  if (u < 0.0f || u > 1.0f) return __builtin_nanf("");
  const vec3 q = cross(s, e1);
  const float v = dot(d, q) * inv;
  if (v < 0.0f || u + v > 1.0f) return __builtin_nanf("");
  return dot(e2, q) * inv;
}

// bvh_walk over the line: leaves whose box meets o + t d, -tb < t < tf.
template <bool CW, class Leaf>
DEV void bvh_walk_line(const float4* __restrict__ N, vec3 o, vec3 d, const float& tf, const float& tb,
                       int* __restrict__ stk, WorkCount& wc, Leaf&& leaf) {
  const vec3 inv = v3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
  const vec3 oi = v3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
  const int lane = threadIdx.x;
  int sp = 0;
  int node = ray_ok(o, d) ? 0 : kDone;
  int pl = 0;
  auto test = [&](float lx, float ly, float lz, float hx, float hy, float hz, float& tn) {
    return slab_line(lx, ly, lz, hx, hy, hz, inv, oi, tf, tb, tn);
  };
  while (node != kDone) {
    while ((uint32_t)node < (uint32_t)kDone) {
      if (CW) wc.nodes++;
      node = visit4(N, node, stk, sp, test);
      if (node < 0 && pl == 0) {
        pl = node;
        node = sp > 0 ? stk[--sp * kTraceBlock + lane] : kDone;
      }
      if (__ballot(pl == 0) == 0ull) break;
    }
    while (pl < 0) {
      leaf(pl);
      pl = 0;
      if (node < 0) {
        pl = node;
        node = sp > 0 ? stk[--sp * kTraceBlock + lane] : kDone;
      }
    }
  }
}

template <bool CW>
DEV void closest_line_in(const DevBvh& B, vec3 o, vec3 d, Hit& hf, Hit& hb, int dyn, int* stk, WorkCount& wc) {
  bvh_walk_line<CW>(B.nodes, o, d, hf.t, hb.t, stk, wc, [&](int code) {
    const int f = leaf_first(code), n = leaf_count(code);
    for (int i = f; i < f + n; ++i) {
      vec3 v0, e1, e2;
      int id, mat;
      load_tri(B.tris, i, v0, e1, e2, id, mat);
      if (CW) wc.tris++;
      const float t = tri_line(o, d, v0, e1, e2);
      if (t > 0.0f && (t < hf.t || (t == hf.t && id < hf.id))) {
        hf.t = t;
        hf.id = id;
        hf.idx = i;
        hf.dyn = dyn;
        hf.ok = 1;
      }
      if (-t > 0.0f && (-t < hb.t || (-t == hb.t && id < hb.id))) {
        hb.t = -t;
        hb.id = id;
        hb.idx = i;
        hb.dyn = dyn;
        hb.ok = 1;
      }
    }
  });
}

// closest(o, d) and closest(o, -d) of scene_f as one line query (one
// traversal, counted as one ray query).
template <bool CW>
DEV void closest_line(const DevScene& S, const DevFrame& F, vec3 o, vec3 d, Hit& hf, Hit& hb, int* stk,
                      WorkCount& wc) {
  const Pose& pose = F.pose;
  if (CW) wc.rays[RAY_CLOSEST]++;
  hf.t = INFINITY;
  hf.id = 0x7fffffff;
  hf.idx = -1;
  hf.dyn = 0;
  hf.ok = 0;
  hb = hf;
  closest_line_in<CW>(S.stat, o, d, hf, hb, 0, stk, wc);
  if (near_object(F, o, d, hf.t) || near_object(F, o, -d, hb.t))
    closest_line_in<CW>(S.obj, pose_inv_apply(pose, o), pose_inv_rot(pose, d), hf, hb, 1, stk, wc);
}

template <bool CW>
DEV bool any_in(const DevBvh& B, vec3 o, vec3 d, float tmax, int* stk, WorkCount& wc) {
  bool hit = false;
  bvh_walk<CW, false>(B.nodes, o, d, tmax, stk, wc, [&](int code) {
    const int f = leaf_first(code), n = leaf_count(code);
    for (int i = f; i < f + n; ++i) {
      vec3 v0, e1, e2;
      int id, mat;
      load_tri(B.tris, i, v0, e1, e2, id, mat);
      if (CW) wc.tris++;
      const float t = tri_t(o, d, v0, e1, e2);
      if (t > 0.0f && t < tmax) {
        hit = true;
        return true;
      }
    }
    return false;
  });
  return hit;
}

// Any hit of scene_f on o + t d, 0 < t < tmax.
template <bool CW>
DEV bool occluded(const DevScene& S, const DevFrame& F, vec3 o, vec3 d, float tmax, int* stk, WorkCount& wc,
                  bool noobj = false) {
  const Pose& pose = F.pose;
  if (any_in<CW>(S.stat, o, d, tmax, stk, wc)) return true;
  if (noobj || !near_object(F, o, d, tmax)) return false;
  return any_in<CW>(S.obj, pose_inv_apply(pose, o), pose_inv_rot(pose, d), tmax, stk, wc);
}

// Hit point, geometric normal and material word of a closest hit.
DEV void hit_vertex(const DevScene& S, const Pose& pose, const Hit& h, vec3 o, vec3 d, vec3& p, vec3& n,
                    uint32_t& md) {
  const DevBvh& B = h.dyn ? S.obj : S.stat;
  vec3 v0, e1, e2;
  int id, mat;
  load_tri(B.tris, h.idx, v0, e1, e2, id, mat);
  p = o + d * h.t;
  n = unit(cross(e1, e2));
  if (h.dyn) n = pose_rot(pose, n);
  md = (uint32_t)mat | (h.dyn ? kDynBit : 0u);
}

// ------------------------------------------------------------------ path ends and edges
// A path end: the pinhole, a surface vertex, an area-light point or an
// environment direction (n = direction towards the environment).
enum { END_EYE = 0, END_SURF = 1, END_LIGHT = 2, END_ENV = 3 };
struct End {
  vec3 p, n;
  int kind;
};
DEV End end_eye(const DevScene& S) { return End{S.cam.eye, S.cam.fwd, END_EYE}; }
DEV End end_surf(vec3 p, vec3 n) { return End{p, n, END_SURF}; }

// Canonical edge segment: ends offset by eps along their normals (the
// pinhole is not offset), open interval 0 < t < tmax (1, or inf for rays to
// the environment).
struct Seg {
  vec3 o, d;
  float tmax;
};
DEV Seg canon(const DevScene& S, const End& A, const End& B) {
  Seg s;
  if (B.kind == END_ENV) {
    s.o = A.kind == END_EYE ? A.p : spawn_dir(S, A.p, A.n, B.n);
    s.d = B.n;
    s.tmax = INFINITY;
    return s;
  }
  s.o = A.kind == END_EYE ? A.p : spawn(S, A.p, A.n, B.p);
  const vec3 e = spawn(S, B.p, B.n, A.p);
  s.d = e - s.o;
  s.tmax = 1.0f;
  return s;
}

// Ghost crossings of an edge A-B (A the end nearer the camera): count and
// sums of 1/|cos_g|, |g - A|^2/|cos_g| and |g - B'|^2/|cos_g|, where g lies on
// the line along which a ghost-started technique generates the edge
// (pinhole -> x_1, offset light point B' -> x_{k-2}, or x_a -> x_{a+1}).
struct Cross {
  float n, s0, sa, sb;
};
DEV Cross no_cross() { return Cross{0.f, 0.f, 0.f, 0.f}; }

template <bool CW>
DEV Cross edge_cross(const DevScene& S, const DevFrame& F, const End& A, const End& B, int* stk, WorkCount& wc) {
  Cross c = no_cross();
  if (!F.ghosts) return c;
  if (CW) wc.rays[RAY_GHOST]++;
  const Seg s = canon(S, A, B);
  if (!near_ghost(F, s.o, s.d, s.tmax)) return c;
  const bool env = B.kind == END_ENV;
  const vec3 a = A.p;
  const vec3 b = env ? A.p : (B.kind == END_LIGHT ? spawn(S, B.p, B.n, A.p) : B.p);
  const vec3 go = pose_inv_apply(F.ghost, s.o), gd = pose_inv_rot(F.ghost, s.d);
  const vec3 la = pose_inv_apply(F.ghost, a), ld = pose_inv_rot(F.ghost, b - a);
  const vec3 u = env ? unit(s.d) : unit(b - a);
  const float tmax = s.tmax;
  bvh_walk<CW, false>(S.obj.nodes, go, gd, tmax, stk, wc, [&](int code) {
    const int f = leaf_first(code), n = leaf_count(code);
    for (int i = f; i < f + n; ++i) {
      vec3 v0, e1, e2;
      int id, mat;
      load_tri(S.obj.tris, i, v0, e1, e2, id, mat);
      if (CW) wc.tris++;
      const float t = tri_t(go, gd, v0, e1, e2);
      if (!(t > 0.0f && t < tmax)) continue;
      vec3 g = s.o + s.d * t;
      c.n += 1.0f;
      if (!env) {
        // density only where the generating line itself crosses the triangle
        // between the ends (the ghost techniques generate the edge along it)
        const float tl = tri_t(la, ld, v0, e1, e2);
        if (!(tl > 0.0f && tl < 1.0f)) continue;
        g = a + (b - a) * tl;
      }
      const vec3 ng = pose_rot(F.ghost, unit(cross(e1, e2)));
      const float cg = fabsf(dot(ng, u));
      c.s0 += 1.0f / cg;
      c.sa += len2(g - a) / cg;
      c.sb += env ? 0.0f : len2(g - b) / cg;
    }
    return false;
  });
  return c;
}

template <bool CW>
DEV bool edge_visible(const DevScene& S, const DevFrame& F, const End& A, const End& B, int* stk, WorkCount& wc,
                      int ray_type, bool noobj = false) {
  if (CW) wc.rays[ray_type]++;
  const Seg s = canon(S, A, B);
  return !occluded<CW>(S, F, s.o, s.d, s.tmax, stk, wc, noobj);
}

// ------------------------------------------------------------------ light sampling
struct LightEnd {
  vec3 p, n;    // area: point and normal; env: n = direction
  uint32_t mat; // emitter material index
  int env;
};
// The first CDF entry strictly above u (clamped to n - 1): a binary search
// over the range the guide table gives for u (g[j] .. g[j + 1], j = the
// table slot of u), which returns the same index as a search over the whole
// CDF with one or two loads instead of log2(n) dependent ones.
DEV int cdf_find(const float* __restrict__ cdf, const int32_t* __restrict__ g, int bits, int n, float u) {
  const int M = 1 << bits;
  const int j = min((int)(u * (float)M), M - 1);  // u * 2^bits is exact
  int lo = g[max(j, 0)], hi = g[max(j, 0) + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cdf[mid] <= u) lo = mid + 1;
    else hi = mid;
  }
  return min(lo, n - 1);
}

DEV bool sample_light(const DevScene& S, const float u[4], LightEnd& L) {
  // every branch writes the fields in the same order, which lets the
  // compiler keep a LightEnd in registers
  if (u[0] < S.p_env) {
    L.p = v3(0, 0, 0);
    L.n = sphere_dir(u[2], u[3]);
    L.mat = 0;
    L.env = 1;
    return true;
  }
  if (S.nlights == 0) return false;
  const int k = cdf_find(S.light_cdf, S.light_guide, S.light_gbits, S.nlights, u[1]);
  vec3 v0, e1, e2;
  int id, mat;
  load_tri(S.light_tris, k, v0, e1, e2, id, mat);
  const float su = sqrtf(u[2]);
  const float b1 = 1.0f - su, b2 = u[3] * su;
  const vec3 va = v0, vb = v0 + e1, vc = v0 + e2;
  L.p = va * (1.0f - b1 - b2) + vb * b1 + vc * b2;
  L.n = unit(cross(e1, e2));
  L.mat = (uint32_t)mat;
  L.env = 0;
  return true;
}
DEV float light_pdf(const DevScene& S, int env) {
  return env ? S.p_env * (1.0f / (4.0f * kPi)) : (1.0f - S.p_env) * S.inv_light_area;
}
DEV vec3 light_Le(const DevScene& S, const LightEnd& L) {
  return L.env ? S.env : v3(S.mats[8 * L.mat + 5], S.mats[8 * L.mat + 6], S.mats[8 * L.mat + 7]);
}
DEV End end_light(const LightEnd& L) { return End{L.p, L.n, L.env ? END_ENV : END_LIGHT}; }

// Uniform-by-area point on the object at `pose`.
DEV void object_point(const DevScene& S, const Pose& pose, const float u[4], vec3& p, vec3& n, uint32_t& md,
                      int& tri) {
  const int k = cdf_find(S.obj_cdf, S.obj_guide, S.obj_gbits, S.nobj, u[0]);
  vec3 v0, e1, e2;
  int id, mat;
  load_tri(S.obj_tris, k, v0, e1, e2, id, mat);
  const float su = sqrtf(u[1]);
  const float b1 = 1.0f - su, b2 = u[2] * su;
  const vec3 va = v0, vb = v0 + e1, vc = v0 + e2;
  p = pose_apply(pose, va * (1.0f - b1 - b2) + vb * b1 + vc * b2);
  n = pose_rot(pose, unit(cross(e1, e2)));
  md = (uint32_t)mat | kDynBit;
  tri = k;
}

}  // namespace rpi
