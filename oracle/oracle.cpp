// Residual path integral oracle: plain, slow CPU reference.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the CPU
// baseline leg of bench.py may load this library.  It shares no code with the
// HIP library (no headers, helpers or tables); both read the same seeded
// input arrays.
//
// What it computes (Xu et al., "Residual path integrals for re-rendering",
// EGSR 2024):
//   * the primal path integral, Sec. 3.1 eq. (pathIntegral)/(pathcontribution)
//     with Veach's full measurement contribution (pinhole importance, G on
//     every edge, box pixel filter): render_frame;
//   * the residual I2 - I1, Sec. 3.2 eq. (twointegral)/(shiftmapped), by the
//     dynamic-path sampling techniques (1)-(6) of Sec. 4.1-4.2 plus path
//     tracing with static paths rejected (Sec. 4.3), combined with the
//     balance heuristic over N_D + N_G + 1 strategies (Sec. 4.3), path mapping
//     and rejection (Sec. 5) and two-way mapping (Sec. 5, path rejection).
//
// Precision: every quantity that decides an integer outcome (which triangle a
// ray hits, which side of a surface a direction lies on, which pixel a point
// projects to, whether a mapped path is rejected) is computed in fp32, the
// precision the GPU kernel takes those decisions in.  Contributions, pdfs,
// MIS sums and the image are computed and accumulated in fp64.
//
// Where the paper is silent it takes one reading and keeps it: depth counts
// segments, c = 1/2 two-way weights, one technique-independent map, uniform
// sphere for technique (6), outward cosine lobe for technique (3), etc.
//
// Parity pins: tests/test_oracle_*.py (identity edit, white furnace closed
// form, depth-2 quadrature, convergence to the difference of two frames,
// strategy-subset agreement, generation-pdf == MIS-term consistency, mapping
// involution, BSDF normalisation, BVH == brute force, Philox KAT vectors).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- vectors
struct V3 {
  float x, y, z;
};
static inline V3 mk(float x, float y, float z) { return V3{x, y, z}; }
static inline V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline V3 operator*(V3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline V3 operator-(V3 a) { return mk(-a.x, -a.y, -a.z); }
static inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline float length(V3 a) { return std::sqrt(dot(a, a)); }
static inline V3 normalize(V3 a) {
  float l = length(a);
  return mk(a.x / l, a.y / l, a.z / l);
}

struct D3 {
  double x, y, z;
};
static inline D3 dmk(double x, double y, double z) { return D3{x, y, z}; }
static inline D3 operator+(D3 a, D3 b) { return dmk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline D3 operator-(D3 a, D3 b) { return dmk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline D3 operator*(D3 a, double s) { return dmk(a.x * s, a.y * s, a.z * s); }
static inline D3 mul(D3 a, D3 b) { return dmk(a.x * b.x, a.y * b.y, a.z * b.z); }
static inline D3 dd(V3 a) { return dmk(a.x, a.y, a.z); }
static inline double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline double dlen2(D3 a) { return ddot(a, a); }
static inline D3 dnorm(D3 a) {
  double l = std::sqrt(dlen2(a));
  return dmk(a.x / l, a.y / l, a.z / l);
}

static const double PI = 3.14159265358979323846;
static const float PIf = 3.14159265358979323846f;

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11: ten rounds of two 32x32->64 multiplies with Weyl key increments.
struct U4 {
  uint32_t v[4];
};
static U4 philox(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * c.v[0];
    uint64_t p1 = (uint64_t)M1 * c.v[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    U4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}
static inline float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// Counter layout: (sample, tech<<24 | dir<<23 | side<<22 | bounce<<8 | slot, job, 0).
struct Rng {
  uint32_t k0, k1, sample, tech, dir, job;
  void draw(uint32_t side, uint32_t bounce, uint32_t slot, float u[4]) const {
    U4 c;
    c.v[0] = sample;
    c.v[1] = (tech << 24) | (dir << 23) | (side << 22) | (bounce << 8) | slot;
    c.v[2] = job;
    c.v[3] = 0;
    U4 r = philox(c, k0, k1);
    for (int i = 0; i < 4; ++i) u[i] = u01(r.v[i]);
  }
};

// ---------------------------------------------------------------- scene
enum { MAT_DIFFUSE = 0, MAT_GGX = 1, MAT_EMITTER = 2 };
struct Material {
  int type;
  float albedo[3];
  float rough;
  float emit[3];
};

struct Tri {
  V3 v0, e1, e2, n;  // n = normalize(cross(e1, e2))
  int mat;
  int id;  // index in the input triangle list
  double area;
};

struct Pose {  // world = R * p + t, R row-major
  float r[9];
  float t[3];
};
static inline V3 pose_apply(const Pose& P, V3 p) {
  return mk(P.r[0] * p.x + P.r[1] * p.y + P.r[2] * p.z + P.t[0],
            P.r[3] * p.x + P.r[4] * p.y + P.r[5] * p.z + P.t[1],
            P.r[6] * p.x + P.r[7] * p.y + P.r[8] * p.z + P.t[2]);
}
static inline V3 pose_rot(const Pose& P, V3 v) {
  return mk(P.r[0] * v.x + P.r[1] * v.y + P.r[2] * v.z, P.r[3] * v.x + P.r[4] * v.y + P.r[5] * v.z,
            P.r[6] * v.x + P.r[7] * v.y + P.r[8] * v.z);
}
static inline V3 pose_inv_rot(const Pose& P, V3 v) {
  return mk(P.r[0] * v.x + P.r[3] * v.y + P.r[6] * v.z, P.r[1] * v.x + P.r[4] * v.y + P.r[7] * v.z,
            P.r[2] * v.x + P.r[5] * v.y + P.r[8] * v.z);
}
static inline V3 pose_inv_apply(const Pose& P, V3 p) {
  return pose_inv_rot(P, p - mk(P.t[0], P.t[1], P.t[2]));
}
static Pose pose_from(const float* m) {
  Pose P;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P.r[3 * i + j] = m[4 * i + j];
    P.t[i] = m[4 * i + 3];
  }
  return P;
}

// Simple object-median BVH: an acceleration only; closest hits are defined
// by the brute-force rule (smallest t, then smallest triangle id).
struct BNode {
  float lo[3], hi[3];
  int left, right;  // children, or -1
  int first, count;
};
struct Bvh {
  std::vector<BNode> nodes;
  std::vector<int> order;  // triangle indices in leaf order
};

static void bvh_build(Bvh& B, const std::vector<Tri>& tris) {
  B.nodes.clear();
  B.order.resize(tris.size());
  for (size_t i = 0; i < tris.size(); ++i) B.order[i] = (int)i;
  if (tris.empty()) return;
  std::vector<V3> cen(tris.size());
  for (size_t i = 0; i < tris.size(); ++i) {
    const Tri& t = tris[i];
    V3 a = t.v0, b = t.v0 + t.e1, c = t.v0 + t.e2;
    cen[i] = mk((a.x + b.x + c.x) / 3, (a.y + b.y + c.y) / 3, (a.z + b.z + c.z) / 3);
  }
  struct Job {
    int node, first, count;
  };
  std::vector<Job> stack;
  B.nodes.push_back(BNode{});
  stack.push_back({0, 0, (int)tris.size()});
  while (!stack.empty()) {
    Job j = stack.back();
    stack.pop_back();
    BNode nd;
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = INFINITY;
      nd.hi[a] = -INFINITY;
    }
    for (int i = j.first; i < j.first + j.count; ++i) {
      const Tri& t = tris[B.order[i]];
      V3 p[3] = {t.v0, t.v0 + t.e1, t.v0 + t.e2};
      for (auto& q : p) {
        float c[3] = {q.x, q.y, q.z};
        for (int a = 0; a < 3; ++a) {
          nd.lo[a] = std::min(nd.lo[a], c[a]);
          nd.hi[a] = std::max(nd.hi[a], c[a]);
        }
      }
    }
    // conservative padding so that box culling never drops a true hit
    for (int a = 0; a < 3; ++a) {
      float pad = 1e-5f * (nd.hi[a] - nd.lo[a]) + 1e-6f * (std::fabs(nd.lo[a]) + std::fabs(nd.hi[a])) + 1e-7f;
      nd.lo[a] -= pad;
      nd.hi[a] += pad;
    }
    nd.first = j.first;
    nd.count = j.count;
    nd.left = nd.right = -1;
    if (j.count > 4) {
      int axis = 0;
      float ext[3] = {nd.hi[0] - nd.lo[0], nd.hi[1] - nd.lo[1], nd.hi[2] - nd.lo[2]};
      if (ext[1] > ext[axis]) axis = 1;
      if (ext[2] > ext[axis]) axis = 2;
      int* beg = B.order.data() + j.first;
      int mid = j.count / 2;
      std::nth_element(beg, beg + mid, beg + j.count, [&](int x, int y) {
        float cx = axis == 0 ? cen[x].x : axis == 1 ? cen[x].y : cen[x].z;
        float cy = axis == 0 ? cen[y].x : axis == 1 ? cen[y].y : cen[y].z;
        return cx < cy || (cx == cy && x < y);
      });
      int l = (int)B.nodes.size();
      B.nodes.push_back(BNode{});
      B.nodes.push_back(BNode{});
      nd.left = l;
      nd.right = l + 1;
      stack.push_back({l, j.first, mid});
      stack.push_back({l + 1, j.first + mid, j.count - mid});
    }
    B.nodes[j.node] = nd;
  }
}

// Slab test in double (conservative).
static bool box_hit(const BNode& n, const double o[3], const double inv[3], double tmax) {
  double t0 = 0.0, t1 = tmax;
  for (int a = 0; a < 3; ++a) {
    double lo = (n.lo[a] - o[a]) * inv[a];
    double hi = (n.hi[a] - o[a]) * inv[a];
    if (std::isnan(lo) || std::isnan(hi)) {  // 0 * inf: ray parallel and on the slab plane
      if (o[a] < n.lo[a] || o[a] > n.hi[a]) return false;
      continue;
    }
    if (lo > hi) std::swap(lo, hi);
    t0 = std::max(t0, lo);
    t1 = std::min(t1, hi);
    if (t0 > t1) return false;
  }
  return true;
}

// Moller-Trumbore in fp32.  Returns t (ray parameter) or -1 for a miss.
static float tri_t(V3 o, V3 d, const Tri& t) {
  V3 p = cross(d, t.e2);
  float det = dot(t.e1, p);
  if (det == 0.0f) return -1.0f;
  float inv = 1.0f / det;
  V3 s = o - t.v0;
  float u = dot(s, p) * inv;
  if (u < 0.0f || u > 1.0f) return -1.0f;
  V3 q = cross(s, t.e1);
  float v = dot(d, q) * inv;
  if (v < 0.0f || u + v > 1.0f) return -1.0f;
  float tt = dot(t.e2, q) * inv;
  return tt > 0.0f ? tt : -1.0f;
}

struct Camera {
  V3 eye, fwd, right, up;
  float tan_half, aspect;
  int W, H;
  double a_film;
};

struct Scene {
  std::vector<Tri> stat, obj;  // obj in object space (= input coordinates)
  Bvh bstat, bobj;
  bool brute;
  std::vector<Material> mats;
  D3 env;
  bool has_env;
  std::vector<int> lights;  // indices into stat of emitter triangles
  std::vector<float> light_cdf;
  double light_area;
  std::vector<float> obj_cdf;
  double obj_area;
  float obj_lo[3], obj_hi[3];  // bounding box of the object's vertices as given
  Camera cam;
  float eps;
  int ntri;
};

// ---------------------------------------------------------------- frames
struct Frame {
  Pose pose;       // object pose in this frame
  Pose ghost;      // object pose in the other frame
  bool ghosts;     // motion edits: the other frame's object is a ghost here
  Material objmat; // material of the object in this frame
};

struct Hit {
  bool ok;
  float t;
  int id;     // input triangle index
  bool dyn;   // on the object
  V3 p, n;
  int mat;
};

static void closest_in(const Scene& S, const std::vector<Tri>& tris, const Bvh& B, V3 o, V3 d,
                       float& best_t, int& best_id, int& best_k) {
  if (tris.empty()) return;
  auto test = [&](int k) {
    float t = tri_t(o, d, tris[k]);
    if (t > 0.0f && (t < best_t || (t == best_t && tris[k].id < best_id))) {
      best_t = t;
      best_id = tris[k].id;
      best_k = k;
    }
  };
  if (S.brute) {
    for (size_t k = 0; k < tris.size(); ++k) test((int)k);
    return;
  }
  double od[3] = {o.x, o.y, o.z}, inv[3] = {1.0 / d.x, 1.0 / d.y, 1.0 / d.z};
  std::vector<int> st;
  st.push_back(0);
  while (!st.empty()) {
    const BNode& n = B.nodes[st.back()];
    st.pop_back();
    if (!box_hit(n, od, inv, best_t == INFINITY ? 1e30 : (double)best_t * (1.0 + 1e-6) + 1e-30)) continue;
    if (n.left < 0) {
      for (int i = n.first; i < n.first + n.count; ++i) test(B.order[i]);
    } else {
      st.push_back(n.left);
      st.push_back(n.right);
    }
  }
}

static void all_in(const Scene& S, const std::vector<Tri>& tris, const Bvh& B, V3 o, V3 d, float tmax,
                   std::vector<std::pair<float, int>>& out) {
  if (tris.empty()) return;
  auto test = [&](int k) {
    float t = tri_t(o, d, tris[k]);
    if (t > 0.0f && t < tmax) out.push_back({t, k});
  };
  if (S.brute) {
    for (size_t k = 0; k < tris.size(); ++k) test((int)k);
    return;
  }
  double od[3] = {o.x, o.y, o.z}, inv[3] = {1.0 / d.x, 1.0 / d.y, 1.0 / d.z};
  std::vector<int> st;
  st.push_back(0);
  double tm = std::isinf(tmax) ? 1e30 : (double)tmax * (1.0 + 1e-6) + 1e-30;
  while (!st.empty()) {
    const BNode& n = B.nodes[st.back()];
    st.pop_back();
    if (!box_hit(n, od, inv, tm)) continue;
    if (n.left < 0) {
      for (int i = n.first; i < n.first + n.count; ++i) test(B.order[i]);
    } else {
      st.push_back(n.left);
      st.push_back(n.right);
    }
  }
}

// Ray queries made by the calling thread (closest hits, any-hit tests and
// ghost all-hit enumerations), for the CPU baseline's rays/s.
static thread_local int64_t t_ray_queries = 0;

// Closest hit in scene_f = static geometry + object at pose.
static Hit closest(const Scene& S, const Pose& pose, V3 o, V3 d) {
  ++t_ray_queries;
  float bt = INFINITY;
  int bid = 0x7fffffff, bk = -1, ok = -1;
  closest_in(S, S.stat, S.bstat, o, d, bt, bid, bk);
  int sk = bk;
  V3 oo = pose_inv_apply(pose, o), dd_ = pose_inv_rot(pose, d);
  closest_in(S, S.obj, S.bobj, oo, dd_, bt, bid, ok);
  Hit h;
  h.ok = bt < INFINITY;
  if (!h.ok) return h;
  h.t = bt;
  h.id = bid;
  h.p = o + d * bt;
  if (ok >= 0 && S.obj[ok].id == bid) {
    h.dyn = true;
    h.n = pose_rot(pose, S.obj[ok].n);
    h.mat = S.obj[ok].mat;
  } else {
    h.dyn = false;
    h.n = S.stat[sk].n;
    h.mat = S.stat[sk].mat;
  }
  return h;
}

// Any hit of scene_f on the open segment o + t (e - o), 0 < t < 1 (tmax = inf for rays).
static bool blocked(const Scene& S, const Pose& pose, V3 o, V3 d, float tmax) {
  ++t_ray_queries;
  std::vector<std::pair<float, int>> hits;
  all_in(S, S.stat, S.bstat, o, d, tmax, hits);
  if (!hits.empty()) return true;
  all_in(S, S.obj, S.bobj, pose_inv_apply(pose, o), pose_inv_rot(pose, d), tmax, hits);
  return !hits.empty();
}

// ---------------------------------------------------------------- materials
static Material vertex_material(const Scene& S, const Frame& F, int mat, bool dyn) {
  return dyn ? F.objmat : S.mats[mat];
}

static void onb(V3 n, V3& t, V3& b) {  // Duff et al. 2017, "Building an orthonormal basis, revisited"
  float sign = std::copysign(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float c = n.x * n.y * a;
  t = mk(1.0f + sign * n.x * n.x * a, sign * c, -sign * n.x);
  b = mk(c, sign + n.y * n.y * a, -n.y);
}

// GGX (Walter et al. 2007) with Smith uncorrelated G1 and Schlick Fresnel.
static double ggx_D(double a, double nh) {
  double a2 = a * a;
  double k = nh * nh * (a2 - 1.0) + 1.0;
  return a2 / (PI * k * k);
}
static double ggx_G1(double a, double c) {
  c = std::fabs(c);
  double t2 = (1.0 - c * c) / (c * c);
  return 2.0 / (1.0 + std::sqrt(1.0 + a * a * t2));
}

// BSDF value rho(wi <-> wo) at a surface with geometric normal n (two-sided,
// reflection only).  wi, wo: unit directions away from the surface.
static D3 bsdf_eval(const Material& m, D3 n, D3 wi, D3 wo) {
  double ci = ddot(n, wi), co = ddot(n, wo);
  if (!(ci * co > 0.0)) return dmk(0, 0, 0);
  if (m.type == MAT_DIFFUSE) return dmk(m.albedo[0] / PI, m.albedo[1] / PI, m.albedo[2] / PI);
  if (m.type == MAT_GGX) {
    D3 ns = ci > 0 ? n : n * -1.0;
    D3 h = dnorm(wi + wo);
    double nh = ddot(ns, h), ih = std::fabs(ddot(wi, h));
    double a = m.rough;
    double D = ggx_D(a, nh);
    double G = ggx_G1(a, ci) * ggx_G1(a, co);
    double s = std::pow(1.0 - ih, 5.0);
    double k = D * G / (4.0 * std::fabs(ci) * std::fabs(co));
    return dmk((m.albedo[0] + (1.0 - m.albedo[0]) * s) * k, (m.albedo[1] + (1.0 - m.albedo[1]) * s) * k,
               (m.albedo[2] + (1.0 - m.albedo[2]) * s) * k);
  }
  return dmk(0, 0, 0);
}

// Solid-angle pdf of sampling wo given wi.
static double bsdf_pdf(const Material& m, D3 n, D3 wi, D3 wo) {
  double ci = ddot(n, wi), co = ddot(n, wo);
  if (!(ci * co > 0.0)) return 0.0;
  if (m.type == MAT_DIFFUSE) return std::fabs(co) / PI;
  if (m.type == MAT_GGX) {
    D3 ns = ci > 0 ? n : n * -1.0;
    D3 h = dnorm(wi + wo);
    double nh = ddot(ns, h);
    return ggx_D(m.rough, nh) * nh / (4.0 * std::fabs(ddot(wo, h)));
  }
  return 0.0;
}

// Sample wo given wi (fp32: the direction decides the next hit).
static bool bsdf_sample(const Material& m, V3 n, V3 wi, float u0, float u1, V3& wo) {
  float ci = dot(n, wi);
  if (ci == 0.0f || m.type == MAT_EMITTER) return false;
  V3 ns = ci > 0.0f ? n : -n;
  V3 t, b;
  onb(ns, t, b);
  if (m.type == MAT_DIFFUSE) {
    float r = std::sqrt(u0), ph = 2.0f * PIf * u1;
    float z = std::sqrt(std::max(0.0f, 1.0f - u0));
    wo = t * (r * std::cos(ph)) + b * (r * std::sin(ph)) + ns * z;
    return dot(wo, ns) > 0.0f;
  }
  float a = m.rough;
  float t2 = a * a * u0 / (1.0f - u0);
  float ct = 1.0f / std::sqrt(1.0f + t2);
  float st = std::sqrt(std::max(0.0f, 1.0f - ct * ct));
  float ph = 2.0f * PIf * u1;
  V3 h = t * (st * std::cos(ph)) + b * (st * std::sin(ph)) + ns * ct;
  float ih = dot(wi, h);
  wo = h * (2.0f * ih) - wi;
  return dot(wo, ns) > 0.0f;
}

// ---------------------------------------------------------------- camera
// Pinhole at distance-1 film, box pixel filter.  raster() < 0: off image.
static int raster(const Camera& C, V3 p) {
  V3 d = p - C.eye;
  float z = dot(d, C.fwd);
  if (!(z > 0.0f)) return -1;
  float sx = dot(d, C.right) / z, sy = dot(d, C.up) / z;
  float fx = (sx / (C.aspect * C.tan_half) + 1.0f) * 0.5f * (float)C.W;
  float fy = (1.0f - sy / C.tan_half) * 0.5f * (float)C.H;
  if (!(fx >= 0.0f && fx < (float)C.W && fy >= 0.0f && fy < (float)C.H)) return -1;
  int px = std::min((int)fx, C.W - 1), py = std::min((int)fy, C.H - 1);
  return py * C.W + px;
}

static V3 camera_dir(const Camera& C, int pixel, float u0, float u1) {
  int px = pixel % C.W, py = pixel / C.W;
  float sx = (2.0f * (((float)px + u0) / (float)C.W) - 1.0f) * C.aspect * C.tan_half;
  float sy = (1.0f - 2.0f * (((float)py + u1) / (float)C.H)) * C.tan_half;
  return normalize(C.fwd + C.right * sx + C.up * sy);
}

// W_j(x0 -> x1) G(x0, x1): importance P / (A_film cos^4) times cos_c |cos_1| / r^2.
static double camera_factor(const Camera& C, V3 x1, V3 n1) {
  D3 d = dd(x1) - dd(C.eye);
  double r2 = dlen2(d);
  D3 w = dnorm(d);
  double cc = ddot(w, dd(C.fwd));
  double c1 = std::fabs(ddot(dd(n1), w));
  double P = (double)C.W * C.H;
  return P / (C.a_film * cc * cc * cc) * c1 / r2;
}

// Whole-image pinhole sampling, area pdf of x1.
static double camera_pdf(const Camera& C, V3 x1, V3 n1) {
  D3 d = dd(x1) - dd(C.eye);
  double r2 = dlen2(d);
  D3 w = dnorm(d);
  double cc = ddot(w, dd(C.fwd));
  double c1 = std::fabs(ddot(dd(n1), w));
  return 1.0 / (C.a_film * cc * cc * cc) * c1 / r2;
}

// ---------------------------------------------------------------- sampling helpers
static int cdf_pick(const std::vector<float>& cdf, float u) {
  int n = (int)cdf.size();
  int i = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
  return std::min(i, n - 1);
}
static V3 tri_point(const Tri& t, float u1, float u2) {
  float su = std::sqrt(u1);
  float b1 = 1.0f - su, b2 = u2 * su;
  V3 a = t.v0, b = t.v0 + t.e1, c = t.v0 + t.e2;
  return a * (1.0f - b1 - b2) + b * b1 + c * b2;
}
static V3 sphere_dir(float u0, float u1) {
  float z = 1.0f - 2.0f * u0;
  float r = std::sqrt(std::max(0.0f, 1.0f - z * z));
  float ph = 2.0f * PIf * u1;
  return mk(r * std::cos(ph), r * std::sin(ph), z);
}

// Light end point x_{k-1}: an area-emitter point or an environment direction.
struct LightPt {
  bool env;
  V3 p, n;   // area: point and normal; env: p unused, n = direction towards the environment
  D3 Le;
};

static double env_select_prob(const Scene& S) {
  if (!S.has_env) return 0.0;
  return S.lights.empty() ? 1.0 : 0.5;
}
// Light-selection pdf p_L: area measure for area emitters, solid angle for the environment.
static double light_pdf(const Scene& S, const LightPt& L) {
  double pe = env_select_prob(S);
  if (L.env) return pe / (4.0 * PI);
  return (1.0 - pe) / S.light_area;
}
static bool sample_light(const Scene& S, const float u[4], LightPt& L) {
  double pe = env_select_prob(S);
  if ((double)u[0] < pe) {
    L.env = true;
    L.n = sphere_dir(u[2], u[3]);
    L.p = mk(0, 0, 0);
    L.Le = S.env;
    return true;
  }
  if (S.lights.empty()) return false;
  const Tri& t = S.stat[S.lights[cdf_pick(S.light_cdf, u[1])]];
  L.env = false;
  L.p = tri_point(t, u[2], u[3]);
  L.n = t.n;
  const Material& m = S.mats[t.mat];
  L.Le = dmk(m.emit[0], m.emit[1], m.emit[2]);
  return true;
}

// Spawn point: offset eps along the normal on the side of `towards`.
static V3 spawn(const Scene& S, V3 p, V3 n, V3 towards) {
  float s = dot(n, towards - p) >= 0.0f ? 1.0f : -1.0f;
  return p + n * (s * S.eps);
}
static V3 spawn_dir(const Scene& S, V3 p, V3 n, V3 dir) {
  float s = dot(n, dir) >= 0.0f ? 1.0f : -1.0f;
  return p + n * (s * S.eps);
}

// ---------------------------------------------------------------- paths
struct PV {
  V3 p, n;
  int mat;
  bool dyn;  // on the object in the frame the path lives in
};
enum { MAXV = 10 };
struct Path {
  int k;        // vertices x_0 .. x_{k-1}
  PV v[MAXV];   // v[1..k-2] scattering vertices (v[0] unused: the pinhole)
  LightPt L;    // x_{k-1}
  int tech, i, j;
  double p_gen; // product of the densities actually used to generate it
  int start;    // index of the start vertex / crossing edge (diagnostics)
};

// Canonical edge segment between path vertices a and a+1 (Sec. 6.1 visibility
// and ghost records): ends offset by eps along their normals (the pinhole is
// not offset), open interval 0 < t < 1; an environment end is a ray.
struct Seg {
  V3 o, d;
  float tmax;
};
static Seg edge_seg(const Scene& S, const Path& P, int a) {
  V3 A = a == 0 ? S.cam.eye : P.v[a].p;
  Seg s;
  if (a + 1 == P.k - 1 && P.L.env) {
    s.o = a == 0 ? A : spawn_dir(S, A, P.v[a].n, P.L.n);
    s.d = P.L.n;
    s.tmax = INFINITY;
    return s;
  }
  V3 B = a + 1 == P.k - 1 ? P.L.p : P.v[a + 1].p;
  V3 nB = a + 1 == P.k - 1 ? P.L.n : P.v[a + 1].n;
  V3 o = a == 0 ? A : spawn(S, A, P.v[a].n, B);
  V3 e = spawn(S, B, nB, A);
  s.o = o;
  s.d = e - o;
  s.tmax = 1.0f;
  return s;
}

// Ghost crossings of an edge: count (canonical segment) and, over the
// crossings of the generating line, sums of 1/|cos_g|, |g-A|^2/|cos_g|, |g-B|^2/|cos_g|.
struct Cross {
  int n;
  double s0, sa, sb;
};
static Cross crossings(const Scene& S, const Frame& F, const Path& P, int a) {
  Cross c{0, 0, 0, 0};
  if (!F.ghosts) return c;
  ++t_ray_queries;
  Seg s = edge_seg(S, P, a);
  std::vector<std::pair<float, int>> hits;
  all_in(S, S.obj, S.bobj, pose_inv_apply(F.ghost, s.o), pose_inv_rot(F.ghost, s.d), s.tmax, hits);
  V3 A = a == 0 ? S.cam.eye : P.v[a].p;
  bool envB = (a + 1 == P.k - 1) && P.L.env;
  V3 B = envB ? A : (a + 1 == P.k - 1 ? spawn(S, P.L.p, P.L.n, A) : P.v[a + 1].p);
  // |cos_g| against the line the ghost-started technique generates this edge
  // along: pinhole -> x_1, offset light point -> x_{k-2}, or x_a -> x_{a+1}.
  D3 u = envB ? dnorm(dd(s.d)) : dnorm(dd(B) - dd(A));
  for (auto& h : hits) {
    // crossing point on the generating line where it meets that triangle
    V3 g = s.o + s.d * h.first;
    c.n += 1;
    if (!envB) {
      // a ghost technique generates this edge from a point of that triangle
      // only if the generating line itself crosses it between the ends: other
      // crossings of the canonical segment (near an end, where it leaves the
      // line by the offsets) mark the edge dynamic but carry no density
      float tl = tri_t(pose_inv_apply(F.ghost, A), pose_inv_rot(F.ghost, B - A), S.obj[h.second]);
      if (!(tl > 0.0f && tl < 1.0f)) continue;
      g = A + (B - A) * tl;
    }
    double cg = std::fabs(ddot(dd(pose_rot(F.ghost, S.obj[h.second].n)), u));
    c.s0 += 1.0 / cg;
    c.sa += dlen2(dd(g) - dd(A)) / cg;
    c.sb += envB ? 0.0 : dlen2(dd(g) - dd(B)) / cg;
  }
  return c;
}

static V3 pos(const Scene& S, const Path& P, int i) {
  if (i == 0) return S.cam.eye;
  if (i == P.k - 1) return P.L.p;
  return P.v[i].p;
}

// Unit direction from vertex i towards vertex j (j may be the light end).
static D3 dir_to(const Scene& S, const Path& P, int i, int j) {
  if (j == P.k - 1 && P.L.env) return dd(P.L.n);
  if (i == P.k - 1 && P.L.env) return dd(P.L.n) * -1.0;
  return dnorm(dd(pos(S, P, j)) - dd(pos(S, P, i)));
}

// Origin of the ray that generates vertex j from vertex i: the pinhole, or
// the surface point offset by eps towards j (exactly where a walk ray starts).
static V3 origin(const Scene& S, const Path& P, int i, int j) {
  if (i == 0) return S.cam.eye;
  V3 to = pos(S, P, j);
  if (i == P.k - 1) return spawn(S, P.L.p, P.L.n, to);
  return spawn(S, P.v[i].p, P.v[i].n, to);
}

// Unit direction of the ray generating vertex j from vertex i.
static D3 gen_dir(const Scene& S, const Path& P, int i, int j) {
  if (j == P.k - 1 && P.L.env) return dd(P.L.n);
  return dnorm(dd(pos(S, P, j)) - dd(origin(S, P, i, j)));
}

// Area-measure conversion factor |cos at j| / r^2 for generating vertex j
// from vertex i, measured from the generating ray's origin (1 for an
// environment end: solid-angle measure).
static double to_area(const Scene& S, const Path& P, int i, int j) {
  if (j == P.k - 1 && P.L.env) return 1.0;
  D3 d = dd(pos(S, P, j)) - dd(origin(S, P, i, j));
  D3 nj = dd(j == P.k - 1 ? P.L.n : P.v[j].n);
  return std::fabs(ddot(nj, dnorm(d))) / dlen2(d);
}

// Geometry term G between vertices i and j = i+1.
static double geom(const Scene& S, const Path& P, int i, int j) {
  D3 w = dir_to(S, P, i, j);
  double ci = i == 0 ? 1.0 : std::fabs(ddot(dd(P.v[i].n), w));
  if (j == P.k - 1 && P.L.env) return ci;
  D3 nj = dd(j == P.k - 1 ? P.L.n : P.v[j].n);
  double cj = std::fabs(ddot(nj, w));
  return ci * cj / dlen2(dd(pos(S, P, j)) - dd(pos(S, P, i)));
}

// Path contribution without the camera factor (eq. pathcontribution, Veach's
// full form): prod_{i=1}^{k-2} rho(x_{i-1} -> x_i -> x_{i+1}) G(x_i, x_{i+1}) * L_e.
static D3 contribution_rest(const Scene& S, const Frame& F, const Path& P) {
  D3 f = dmk(1, 1, 1);
  for (int i = 1; i <= P.k - 2; ++i) {
    Material m = vertex_material(S, F, P.v[i].mat, P.v[i].dyn);
    D3 rho = bsdf_eval(m, dd(P.v[i].n), dir_to(S, P, i, i - 1), dir_to(S, P, i, i + 1));
    f = mul(f, rho) * geom(S, P, i, i + 1);
  }
  return mul(f, P.L.Le);
}

// Support (geometric validity apart from visibility): reflection at every
// scattering vertex, emitter facing the last scattering vertex, no emitter
// inside the path, first vertex projecting into the image.
static bool supported(const Scene& S, const Frame& F, const Path& P, bool check_raster = true) {
  if (P.k < 2) return false;
  for (int i = 1; i <= P.k - 2; ++i) {
    Material m = vertex_material(S, F, P.v[i].mat, P.v[i].dyn);
    if (m.type == MAT_EMITTER) return false;
    V3 a = i - 1 == 0 ? S.cam.eye - P.v[i].p : pos(S, P, i - 1) - P.v[i].p;
    V3 b = (i + 1 == P.k - 1 && P.L.env) ? P.L.n : pos(S, P, i + 1) - P.v[i].p;
    if (!(dot(P.v[i].n, a) * dot(P.v[i].n, b) > 0.0f)) return false;
  }
  if (!P.L.env) {
    V3 prev = pos(S, P, P.k - 2);
    if (!(dot(P.L.n, prev - P.L.p) > 0.0f)) return false;
  }
  if (!check_raster) return true;
  V3 x1 = P.k == 2 ? P.L.p : P.v[1].p;
  if (P.k == 2 && P.L.env) return false;
  return raster(S.cam, x1) >= 0;
}

// ---------------------------------------------------------------- learned proposal
// A small MLP maps a surface point of the object (position normalised to the
// object's bounding box, geometric normal; object space) to a mixture of 8
// von Mises-Fisher lobes over directions (addition beyond the paper: the paper
// names better importance sampling of the residual integrand as future work,
// Sec. 7).  Layers 6 -> 64 -> 64 -> 64 -> 40 with ReLU; parameters in one
// flat vector: W1[6][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
// W4[64][40], b4[40] (row-major [in][out]).
enum { MLP_IN = 6, MLP_H = 64, MLP_OUT = 40, MLP_LOBES = 8 };
static const int MLP_NPARAM = 6 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 40 + 40;
static const int OFF_W1 = 0, OFF_B1 = 384, OFF_W2 = 448, OFF_B2 = 4544, OFF_W3 = 4608, OFF_B3 = 8704,
                 OFF_W4 = 8768, OFF_B4 = 11328;

// Round to the nearest bfloat16 (ties to even), returned as float.
static float bf16r(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

// Forward pass in fp64 arithmetic.  bf16 = true rounds weights and every
// layer input to bfloat16 (the precision of the matrix-core kernels; biases,
// accumulation and outputs stay wide).  acts (optional) receives the inputs
// of the four layers for back-propagation: [6 | 64 | 64 | 64] values.
static void mlp_forward(const float* P, const double* x, bool bf16, double* out, double* acts = nullptr) {
  double a0[MLP_IN], a1[MLP_H], a2[MLP_H], a3[MLP_H];
  auto w = [&](int off, int i) { return bf16 ? (double)bf16r(P[off + i]) : (double)P[off + i]; };
  auto in = [&](double v) { return bf16 ? (double)bf16r((float)v) : v; };
  for (int i = 0; i < MLP_IN; ++i) a0[i] = in(x[i]);
  auto layer = [&](const double* a, int n_in, int n_out, int ow, int ob, double* z, bool relu) {
    for (int j = 0; j < n_out; ++j) {
      double acc = 0.0;
      for (int i = 0; i < n_in; ++i) acc += a[i] * w(ow, i * n_out + j);
      acc += P[ob + j];
      z[j] = relu ? (acc > 0.0 ? acc : 0.0) : acc;
    }
  };
  double z1[MLP_H], z2[MLP_H], z3[MLP_H];
  layer(a0, MLP_IN, MLP_H, OFF_W1, OFF_B1, z1, true);
  for (int j = 0; j < MLP_H; ++j) a1[j] = in(z1[j]);
  layer(a1, MLP_H, MLP_H, OFF_W2, OFF_B2, z2, true);
  for (int j = 0; j < MLP_H; ++j) a2[j] = in(z2[j]);
  layer(a2, MLP_H, MLP_H, OFF_W3, OFF_B3, z3, true);
  for (int j = 0; j < MLP_H; ++j) a3[j] = in(z3[j]);
  layer(a3, MLP_H, MLP_OUT, OFF_W4, OFF_B4, out, false);
  if (acts) {
    std::memcpy(acts, a0, sizeof a0);
    std::memcpy(acts + 6, a1, sizeof a1);
    std::memcpy(acts + 70, a2, sizeof a2);
    std::memcpy(acts + 134, a3, sizeof a3);
  }
}

// Lobe parameters from the raw outputs (fp32, as the sampler uses them):
// mean = normalize(raw xyz), kappa = softplus(raw) + 0.01 (<= 1e4),
// weight = softmax over lobes.
struct Lobes {
  float mu[MLP_LOBES][3], kappa[MLP_LOBES], w[MLP_LOBES];
};
static float softplusf(float x) { return x > 20.0f ? x : std::log1p(std::exp(x)); }
static Lobes lobes_of(const double* raw) {
  Lobes L;
  float mx = -INFINITY;
  for (int l = 0; l < MLP_LOBES; ++l) mx = std::max(mx, (float)raw[5 * l + 4]);
  float sum = 0.0f;
  for (int l = 0; l < MLP_LOBES; ++l) {
    float x = (float)raw[5 * l], y = (float)raw[5 * l + 1], z = (float)raw[5 * l + 2];
    float n = std::sqrt(x * x + y * y + z * z);
    if (!(n > 0.0f)) {
      x = 0.0f;
      y = 0.0f;
      z = 1.0f;
      n = 1.0f;
    }
    L.mu[l][0] = x / n;
    L.mu[l][1] = y / n;
    L.mu[l][2] = z / n;
    L.kappa[l] = std::min(softplusf((float)raw[5 * l + 3]) + 0.01f, 1e4f);
    L.w[l] = std::exp((float)raw[5 * l + 4] - mx);
    sum += L.w[l];
  }
  for (int l = 0; l < MLP_LOBES; ++l) L.w[l] /= sum;
  return L;
}
// vMF density on the unit sphere: kappa / (2 pi (1 - e^{-2 kappa})) exp(kappa (mu.w - 1)).
static double vmf_pdf(const Lobes& L, D3 w) {
  double q = 0.0;
  for (int l = 0; l < MLP_LOBES; ++l) {
    const double k = L.kappa[l];
    const double c = L.mu[l][0] * w.x + L.mu[l][1] * w.y + L.mu[l][2] * w.z;
    q += L.w[l] * k / (2.0 * PI * (-std::expm1(-2.0 * k))) * std::exp(k * (c - 1.0));
  }
  return q;
}
// Jakob 2012, numerically stable vMF sampling on S^2 (fp32: it decides hits).
static V3 vmf_sample(const Lobes& L, float u0, float u1, float u2) {
  int l = 0;
  float run = 0.0f;
  for (; l < MLP_LOBES - 1; ++l) {
    run += L.w[l];
    if (u0 < run) break;
  }
  const float k = L.kappa[l];
  // u1 = 0 with e^{-2 kappa} below the float range makes the argument 0:
  // the formula's limit there is c = -1, the antipode of the mean
  const float a = u1 + (1.0f - u1) * std::exp(-2.0f * k);
  const float c = a > 0.0f ? 1.0f + std::log(a) / k : -1.0f;
  const float s = std::sqrt(std::max(0.0f, 1.0f - c * c));
  const float ph = 2.0f * PIf * u2;
  V3 mu = mk(L.mu[l][0], L.mu[l][1], L.mu[l][2]);
  V3 t, b;
  onb(mu, t, b);
  return normalize(t * (s * std::cos(ph)) + b * (s * std::sin(ph)) + mu * c);
}

// Technique (8)'s direction sampler is a defensive mixture (Hesterberg
// 1995): with probability T8_UNIFORM a uniform direction on the sphere, else
// the learned lobes.  The technique keeps full support where the lobes'
// densities underflow, so it can stand in for techniques (2) and (3).
static const float T8_UNIFORM = 0.25f;
static V3 sphere_dir(float u0, float u1);
static V3 t8_sample(const Lobes& L, float u0, float u1, float u2) {
  if (u0 < T8_UNIFORM) return sphere_dir(u1, u2);
  return vmf_sample(L, (u0 - T8_UNIFORM) / (1.0f - T8_UNIFORM), u1, u2);
}
static double t8_pdf(const Lobes& L, D3 w) {
  return (double)T8_UNIFORM / (4.0 * PI) + (1.0 - (double)T8_UNIFORM) * vmf_pdf(L, w);
}

struct Proposal {
  const float* params;  // MLP_NPARAM floats, or null (technique 8 off)
  V3 center, inv_half;  // object-space bounding box normalisation
};
static void proposal_input(const Proposal& Pr, V3 p_obj, V3 n_obj, double* x) {
  x[0] = (p_obj.x - Pr.center.x) * Pr.inv_half.x;
  x[1] = (p_obj.y - Pr.center.y) * Pr.inv_half.y;
  x[2] = (p_obj.z - Pr.center.z) * Pr.inv_half.z;
  x[3] = n_obj.x;
  x[4] = n_obj.y;
  x[5] = n_obj.z;
}
static Lobes proposal_lobes(const Proposal& Pr, V3 p_obj, V3 n_obj) {
  double x[MLP_IN], raw[MLP_OUT];
  proposal_input(Pr, p_obj, n_obj, x);
  mlp_forward(Pr.params, x, true, raw);
  return lobes_of(raw);
}

// Weighted negative log-likelihood of directions (the Monte Carlo KL
// estimator of neural importance sampling) and its gradient, fp64, for
// records {x[6], w_obj[3], weight}.
static double mlp_loss_grad(const float* P, const float* rec, int n, bool bf16, double* grad) {
  std::fill(grad, grad + MLP_NPARAM, 0.0);
  double wsum = 0.0, loss = 0.0;
  for (int r = 0; r < n; ++r) wsum += rec[10 * r + 9];
  if (!(wsum > 0.0)) return 0.0;
  for (int r = 0; r < n; ++r) {
    const float* R = rec + 10 * r;
    const double wt = R[9] / wsum;
    if (wt == 0.0) continue;
    double x[MLP_IN], raw[MLP_OUT], acts[198];
    for (int i = 0; i < 6; ++i) x[i] = R[i];
    mlp_forward(P, x, bf16, raw, acts);
    D3 om = dmk(R[6], R[7], R[8]);
    // mixture terms in fp64 from the raw outputs
    double mu[MLP_LOBES][3], nrm[MLP_LOBES], kap[MLP_LOBES], sp_d[MLP_LOBES], wl[MLP_LOBES], f[MLP_LOBES];
    double mx = -1e300;
    for (int l = 0; l < MLP_LOBES; ++l) mx = std::max(mx, raw[5 * l + 4]);
    double es = 0.0;
    for (int l = 0; l < MLP_LOBES; ++l) {
      nrm[l] = std::sqrt(raw[5 * l] * raw[5 * l] + raw[5 * l + 1] * raw[5 * l + 1] + raw[5 * l + 2] * raw[5 * l + 2]);
      for (int a = 0; a < 3; ++a) mu[l][a] = raw[5 * l + a] / nrm[l];
      const double t = raw[5 * l + 3];
      const double sp = t > 30.0 ? t : std::log1p(std::exp(t));
      sp_d[l] = 1.0 / (1.0 + std::exp(-t));
      kap[l] = sp + 0.01;
      wl[l] = std::exp(raw[5 * l + 4] - mx);
      es += wl[l];
    }
    double q = 0.0;
    for (int l = 0; l < MLP_LOBES; ++l) {
      wl[l] /= es;
      const double k = kap[l];
      const double c = mu[l][0] * om.x + mu[l][1] * om.y + mu[l][2] * om.z;
      f[l] = k / (2.0 * PI * (-std::expm1(-2.0 * k))) * std::exp(k * (c - 1.0));
      q += wl[l] * f[l];
    }
    loss += -wt * std::log(q);
    // d(-log q)/d raw
    double draw_[MLP_OUT];
    for (int l = 0; l < MLP_LOBES; ++l) {
      const double k = kap[l];
      const double c = mu[l][0] * om.x + mu[l][1] * om.y + mu[l][2] * om.z;
      const double r_l = wl[l] * f[l] / q;  // responsibility
      // d log f / d kappa = 1/k - 2 e^{-2k}/(1 - e^{-2k}) + (c - 1)
      const double e2 = std::exp(-2.0 * k);
      const double dlogf_dk = 1.0 / k - 2.0 * e2 / (1.0 - e2) + (c - 1.0);
      // d log f / d mu_raw = k (om - c mu) / |raw|
      for (int a = 0; a < 3; ++a) {
        const double oa = a == 0 ? om.x : a == 1 ? om.y : om.z;
        draw_[5 * l + a] = -r_l * k * (oa - c * mu[l][a]) / nrm[l];
      }
      draw_[5 * l + 3] = -r_l * dlogf_dk * sp_d[l];
      draw_[5 * l + 4] = -(r_l - wl[l]);
    }
    // back-propagation
    double g3[MLP_H], g2[MLP_H], g1[MLP_H];
    const double* a0 = acts;
    const double* a1 = acts + 6;
    const double* a2 = acts + 70;
    const double* a3 = acts + 134;
    auto w = [&](int off, int i) { return bf16 ? (double)bf16r(P[off + i]) : (double)P[off + i]; };
    for (int j = 0; j < MLP_OUT; ++j) {
      grad[OFF_B4 + j] += wt * draw_[j];
      for (int i = 0; i < MLP_H; ++i) grad[OFF_W4 + i * MLP_OUT + j] += wt * a3[i] * draw_[j];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0.0;
      for (int j = 0; j < MLP_OUT; ++j) acc += w(OFF_W4, i * MLP_OUT + j) * draw_[j];
      g3[i] = a3[i] > 0.0 ? acc : 0.0;
    }
    auto back = [&](const double* a_in, const double* g_out, int n_in, int ow, int ob, double* g_in, const double* a_prev) {
      for (int j = 0; j < MLP_H; ++j) {
        grad[ob + j] += wt * g_out[j];
        for (int i = 0; i < n_in; ++i) grad[ow + i * MLP_H + j] += wt * a_in[i] * g_out[j];
      }
      if (g_in)
        for (int i = 0; i < n_in; ++i) {
          double acc = 0.0;
          for (int j = 0; j < MLP_H; ++j) acc += w(ow, i * MLP_H + j) * g_out[j];
          g_in[i] = a_prev[i] > 0.0 ? acc : 0.0;
        }
    };
    back(a2, g3, MLP_H, OFF_W3, OFF_B3, g2, a2);
    back(a1, g2, MLP_H, OFF_W2, OFF_B2, g1, a1);
    back(a0, g1, MLP_IN, OFF_W1, OFF_B1, nullptr, nullptr);
  }
  return loss;
}

// ---------------------------------------------------------------- MIS (Sec. 4.3)
struct MisOpts {
  uint32_t mask;   // bit t-1: technique t enabled
  bool ghosts;
  double p_dir;    // technique (6) direction pdf, uniform sphere
  const Proposal* prop;  // technique (8): learned lobes (null: off)
  const Frame* frame;
  // samples of technique t relative to the base count N: the balance
  // heuristic over unequal sample counts n_t weighs density p_t by n_t
  // (Veach 1997, Sec. 9.2), and the image divides by N
  double ratio[9];
};

// Forward pdf a_i (1 <= i <= k-3): x_i generated from x_{i+1} by BSDF
// sampling with the other neighbour x_{i+2} as incoming, area measure at x_i.
static double pdf_a(const Scene& S, const Frame& F, const Path& P, int i) {
  Material m = vertex_material(S, F, P.v[i + 1].mat, P.v[i + 1].dyn);
  double ps = bsdf_pdf(m, dd(P.v[i + 1].n), dir_to(S, P, i + 1, i + 2), gen_dir(S, P, i + 1, i));
  return ps * to_area(S, P, i + 1, i);
}
// Backward pdf b_i (2 <= i <= k-2): x_i generated from x_{i-1} with incoming x_{i-2}.
static double pdf_b(const Scene& S, const Frame& F, const Path& P, int i) {
  Material m = vertex_material(S, F, P.v[i - 1].mat, P.v[i - 1].dyn);
  double ps = bsdf_pdf(m, dd(P.v[i - 1].n), dir_to(S, P, i - 1, i - 2), gen_dir(S, P, i - 1, i));
  return ps * to_area(S, P, i - 1, i);
}
static double prod_a(const Scene& S, const Frame& F, const Path& P, int lo, int hi) {
  double r = 1.0;
  for (int i = lo; i <= hi; ++i) r *= pdf_a(S, F, P, i);
  return r;
}
static double prod_b(const Scene& S, const Frame& F, const Path& P, int lo, int hi) {
  double r = 1.0;
  for (int i = lo; i <= hi; ++i) r *= pdf_b(S, F, P, i);
  return r;
}

// Cosine-lobe pdf about the outward normal (technique (3)), area measure at x_{m+1}.
static double pdf_cos_out(const Scene& S, const Path& P, int m) {
  D3 w = gen_dir(S, P, m, m + 1);
  double c = ddot(dd(P.v[m].n), w);
  if (c <= 0.0) return 0.0;
  return c / PI * to_area(S, P, m, m + 1);
}

static double cam_pdf(const Scene& S, const Path& P);

struct MisTerms {
  double total;
  double by_tech[9];
};

// Technique (8)'s density of x_{m+1} given x_m: the learned lobes at x_m
// (object space) for the direction from the offset origin, in area measure.
static double t8_dir_pdf(const Scene& S, const Path& P, const MisOpts& O, int m) {
  const Pose& pose = O.frame->pose;
  Lobes Lb = proposal_lobes(*O.prop, pose_inv_apply(pose, P.v[m].p), pose_inv_rot(pose, P.v[m].n));
  V3 wg = normalize(P.v[m + 1].p - origin(S, P, m, m + 1));
  D3 wo = dnorm(dd(pose_inv_rot(pose, wg)));
  return t8_pdf(Lb, wo) * to_area(S, P, m, m + 1);
}

// Sum over every strategy able to produce the path: one per dynamic vertex
// (techniques 1/2/3 by position), one per ghost crossing (4/5/6 by edge),
// plus path tracing (7).  Each strategy pdf is written out as the full
// product of its vertex densities (no prefix tables).
static MisTerms mis_terms(const Scene& S, const Frame& F, const Path& P, const MisOpts& O) {
  MisTerms r;
  std::memset(&r, 0, sizeof r);
  int k = P.k;
  double pL = light_pdf(S, P.L);
  double pD = 1.0 / S.obj_area;
  auto on = [&](int t) { return (O.mask >> (t - 1)) & 1u; };
  if (on(7)) {
    double p = cam_pdf(S, P);
    if (k >= 3) p *= prod_b(S, F, P, 2, k - 2) * pL;
    r.by_tech[7] += p;
  }
  for (int m = 1; m <= k - 2; ++m) {
    if (!P.v[m].dyn) continue;
    if (m == k - 2) {
      if (on(1)) r.by_tech[1] += pL * pD * prod_a(S, F, P, 1, m - 1);
    } else if (m == 1) {
      if (on(2) && k >= 4) r.by_tech[2] += pD * prod_b(S, F, P, 2, k - 2) * pL;
      if (on(8) && O.prop && O.prop->params) r.by_tech[8] += pD * t8_dir_pdf(S, P, O, 1) * prod_b(S, F, P, 3, k - 2) * pL;
    } else {
      if (on(3)) r.by_tech[3] += pD * pdf_cos_out(S, P, m) * prod_a(S, F, P, 1, m - 1) *
                                 prod_b(S, F, P, m + 2, k - 2) * pL;
      if (on(8) && O.prop && O.prop->params)
        r.by_tech[8] += pD * t8_dir_pdf(S, P, O, m) * prod_a(S, F, P, 1, m - 1) * prod_b(S, F, P, m + 2, k - 2) * pL;
    }
  }
  if (O.ghosts && k >= 3) {
    double pG = pD;
    for (int a = 0; a <= k - 2; ++a) {
      Cross c = crossings(S, F, P, a);
      if (c.n == 0) continue;
      if (a + 1 == k - 1) {
        if (on(4) && !P.L.env) {
          // eq. (vertex1pdf): ghost area pdf -> solid angle at x_L -> area at x_{k-2}
          D3 w = gen_dir(S, P, k - 1, k - 2);
          double ck = std::fabs(ddot(dd(P.v[k - 2].n), w));
          double r2 = dlen2(dd(P.v[k - 2].p) - dd(origin(S, P, k - 1, k - 2)));
          r.by_tech[4] += pL * pG * c.sb * ck / r2 * prod_a(S, F, P, 1, k - 3);
        }
      } else if (a == 0) {
        if (on(5)) {
          D3 w = dir_to(S, P, 0, 1);
          double c1 = std::fabs(ddot(dd(P.v[1].n), w));
          double r2 = dlen2(dd(P.v[1].p) - dd(S.cam.eye));
          r.by_tech[5] += pG * c.sa * c1 / r2 * prod_b(S, F, P, 2, k - 2) * pL;
        }
      } else {
        if (on(6)) {
          // g_{G,x1,x2}: line measure through the ghost point
          double G = geom(S, P, a, a + 1);
          r.by_tech[6] += pG * O.p_dir * G * c.s0 * prod_a(S, F, P, 1, a - 1) *
                          prod_b(S, F, P, a + 2, k - 2) * pL;
        }
      }
    }
  }
  for (int t = 1; t <= 8; ++t) r.total += O.ratio[t] * r.by_tech[t];
  return r;
}

static bool is_dynamic(const Scene& S, const Frame& F, const Path& P) {
  for (int i = 1; i <= P.k - 2; ++i)
    if (P.v[i].dyn) return true;
  if (!F.ghosts) return false;
  for (int a = 0; a <= P.k - 2; ++a)
    if (crossings(S, F, P, a).n > 0) return true;
  return false;
}

static bool path_visible(const Scene& S, const Pose& pose, const Path& P, int a) {
  Seg s = edge_seg(S, P, a);
  return !blocked(S, pose, s.o, s.d, s.tmax);
}

}  // namespace orc

namespace orc {

// First-vertex camera terms, including an environment direction seen directly (k = 2).
static double cam_factor(const Scene& S, const Path& P) {
  if (P.k == 2 && P.L.env) {
    double cc = ddot(dd(P.L.n), dd(S.cam.fwd));
    return (double)S.cam.W * S.cam.H / (S.cam.a_film * cc * cc * cc);
  }
  V3 x1 = P.k == 2 ? P.L.p : P.v[1].p;
  V3 n1 = P.k == 2 ? P.L.n : P.v[1].n;
  return camera_factor(S.cam, x1, n1);
}
static double cam_pdf(const Scene& S, const Path& P) {
  if (P.k == 2 && P.L.env) {
    double cc = ddot(dd(P.L.n), dd(S.cam.fwd));
    return 1.0 / (S.cam.a_film * cc * cc * cc);
  }
  V3 x1 = P.k == 2 ? P.L.p : P.v[1].p;
  V3 n1 = P.k == 2 ? P.L.n : P.v[1].n;
  return camera_pdf(S.cam, x1, n1);
}
static int path_pixel(const Scene& S, const Path& P) {
  if (P.k == 2 && P.L.env) return raster(S.cam, S.cam.eye + P.L.n);
  return raster(S.cam, P.k == 2 ? P.L.p : P.v[1].p);
}
static bool path_ok(const Scene& S, const Frame& F, const Path& P) {
  if (P.k == 2) {
    if (P.L.env) return path_pixel(S, P) >= 0;
    return dot(P.L.n, S.cam.eye - P.L.p) > 0.0f && path_pixel(S, P) >= 0;
  }
  return supported(S, F, P);
}

// ---------------------------------------------------------------- path mapping (Sec. 5)
enum { ACCEPT = 0, R1 = 1, R2 = 2, R3 = 3, R4 = 4, R5 = 5, R6 = 6, REJECT_UNMAPPED = 7 };

struct MapParams {
  float alpha_min, d_min, jac_max;
};

static float roughness_of(const Material& m) { return m.type == MAT_GGX ? m.rough : 1.0f; }

// T_{f->f'}: camera-ray re-trace for x_1 (dynamic/ghost pair operator), rigid
// object transform for dynamic x_i (i >= 2), identity ("keep the vertex the
// same") elsewhere.  Rejection rules R1-R6 are symmetric in f <-> f'.
static int map_path(const Scene& S, const Frame& F, const Frame& Fp, const Path& X, Path& Y,
                    const MapParams& M) {
  Y = X;
  int k = X.k;
  if (k <= 2) return R1;
  if (std::memcmp(&F.pose, &Fp.pose, sizeof(Pose)) == 0) {
    // both frames place the object identically: the scenes coincide and T is the identity
    for (int a = 0; a <= k - 2; ++a)
      if (F.ghosts && crossings(S, F, X, a).n > 0) return R5;
    return ACCEPT;
  }
  // y_1
  bool retrace = X.v[1].dyn || (F.ghosts && crossings(S, F, X, 0).n > 0);
  {
    int mv = retrace ? 1 : 0;
    for (int i = 2; i <= k - 2; ++i) mv += X.v[i].dyn ? 1 : 0;
    if (mv > 1) return R2;
  }
  if (retrace) {
    V3 w = normalize(X.v[1].p - S.cam.eye);
    Hit h = closest(S, Fp.pose, S.cam.eye, w);
    if (!h.ok) return R1;
    if (!h.dyn && S.mats[h.mat].type == MAT_EMITTER) return R1;
    Y.v[1] = PV{h.p, h.n, h.mat, h.dyn};
  } else {
    Y.v[1].dyn = false;
  }
  for (int i = 2; i <= k - 2; ++i) {
    if (X.v[i].dyn) {
      V3 q = pose_inv_apply(F.pose, X.v[i].p);
      Y.v[i].p = pose_apply(Fp.pose, q);
      Y.v[i].n = pose_rot(Fp.pose, pose_inv_rot(F.pose, X.v[i].n));
      Y.v[i].dyn = true;
    }
  }
  // A vertex counts as moved when a moving operator was applied to it (the
  // camera re-trace for x_1, the rigid transform for dynamic x_i); this is
  // symmetric in f <-> f' even where the re-traced point coincides with x_1
  // (object faces coplanar across the two poses).
  int moved = 0, istar = -1;
  for (int i = 1; i <= k - 2; ++i)
    if (i == 1 ? retrace : X.v[i].dyn) {
      ++moved;
      istar = i;
    }
  if (moved > 1) return R2;
  if (moved == 1) {
    Material mx = vertex_material(S, F, X.v[istar].mat, X.v[istar].dyn);
    Material my = vertex_material(S, Fp, Y.v[istar].mat, Y.v[istar].dyn);
    for (int j = istar - 1; j <= istar + 1; j += 2) {
      if (j < 1) continue;  // the pinhole: same camera ray, no reconnection
      bool light = j == k - 1;
      if (!light && (X.v[j].dyn || Y.v[j].dyn)) return R3;
      float aj = light ? 1.0f : roughness_of(vertex_material(S, F, X.v[j].mat, X.v[j].dyn));
      if (std::min(std::min(roughness_of(mx), roughness_of(my)), aj) < M.alpha_min) return R3;
      if (light && X.L.env) continue;
      V3 xj = light ? X.L.p : X.v[j].p;
      V3 nj = light ? X.L.n : X.v[j].n;
      V3 dy = Y.v[istar].p - xj, dx = X.v[istar].p - xj;
      float ly2 = dot(dy, dy), lx2 = dot(dx, dx);
      if (std::min(std::sqrt(ly2), std::sqrt(lx2)) < M.d_min) return R3;
      // eq. (path_reconnection_jacobian)
      float jac = (std::fabs(dot(nj, dy)) / std::sqrt(ly2)) / (std::fabs(dot(nj, dx)) / std::sqrt(lx2)) *
                  (lx2 / ly2);
      if (!(jac <= M.jac_max && jac >= 1.0f / M.jac_max)) return R4;
    }
  }
  if (!supported(S, Fp, Y, false)) return R6;
  for (int a = 0; a <= k - 2; ++a) {
    bool touches = moved == 1 && (a == istar - 1 || a == istar);
    if (touches) {
      if (a == 0) continue;  // re-traced camera edge: visible by construction
      if (!path_visible(S, Fp.pose, Y, a)) return R5;
    } else if (F.ghosts && crossings(S, F, X, a).n > 0) {
      return R5;  // shared edge blocked in f' exactly when it crosses the ghost in f
    }
  }
  return ACCEPT;
}

// ---------------------------------------------------------------- techniques (Sec. 4)
struct Gen {
  const Scene& S;
  const Frame& F;
  Rng rng;
  int depth;
  int tech;
  std::vector<Path>& out;
};

static PV obj_point(const Scene& S, const Pose& pose, const float u[4], int* tri = nullptr) {
  int ti = cdf_pick(S.obj_cdf, u[0]);
  if (tri) *tri = ti;
  const Tri& t = S.obj[ti];
  PV v;
  v.p = pose_apply(pose, tri_point(t, u[1], u[2]));
  v.n = pose_rot(pose, t.n);
  v.mat = t.mat;
  v.dyn = true;
  return v;
}

// One BSDF-sampled extension of a random walk from v, whose other neighbour
// lies in direction wi.  Returns the generation pdf (area measure) or 0.
static double extend(const Gen& g, const PV& v, V3 wi, const float u[4], PV& out) {
  Material m = vertex_material(g.S, g.F, v.mat, v.dyn);
  V3 wo;
  if (!bsdf_sample(m, v.n, wi, u[0], u[1], wo)) return 0.0;
  V3 o = spawn_dir(g.S, v.p, v.n, wo);
  Hit h = closest(g.S, g.F.pose, o, wo);
  if (!h.ok) return 0.0;
  if (!h.dyn && g.S.mats[h.mat].type == MAT_EMITTER) return 0.0;
  out = PV{h.p, h.n, h.mat, h.dyn};
  double ps = bsdf_pdf(m, dd(v.n), dd(wi), dd(wo));
  D3 d = dd(out.p) - dd(o);
  return ps * std::fabs(ddot(dd(out.n), dnorm(d))) / dlen2(d);
}

// A ghost-started sample generates its path only if its ghost point is one
// of the crossings recorded on the generated edge (strictly inside the
// canonical segment); otherwise the sample fails.  This keeps generation
// consistent with the strategy set counted by MIS when ghost and object
// surfaces coincide (e.g. coplanar faces under translation).
static bool ghost_on_edge(const Gen& g, const Path& Q, int a, int tri) {
  Seg s = edge_seg(g.S, Q, a);
  float t = tri_t(pose_inv_apply(g.F.ghost, s.o), pose_inv_rot(g.F.ghost, s.d), g.S.obj[tri]);
  return t > 0.0f && t < s.tmax;
}

static V3 towards(const LightPt& L, V3 from) { return L.env ? L.n : normalize(L.p - from); }

// Assemble x_0, eye[i..0], [mid], light[0..j] and the light end.
static bool assemble(const Gen& g, const PV* eye, int i, const PV* mid, const PV* light, int j,
                     const LightPt& L, double p_gen, int start, Path& P) {
  int n = 0;
  P.v[0] = PV{g.S.cam.eye, g.S.cam.fwd, -1, false};
  for (int a = i; a >= 0; --a) P.v[++n] = eye[a];
  if (mid) P.v[++n] = *mid;
  for (int b = 0; b <= j; ++b) P.v[++n] = light[b];
  P.k = n + 2;
  if (P.k - 1 > g.depth || P.k > MAXV) return false;
  P.L = L;
  P.tech = g.tech;
  P.p_gen = p_gen;
  P.start = start;
  P.i = i;
  P.j = j;
  return true;
}

// Camera connection of the assembled path's first edge (light tracing).
static bool camera_edge_ok(const Gen& g, const Path& P) {
  if (raster(g.S.cam, P.v[1].p) < 0) return false;
  return path_visible(g.S, g.F.pose, P, 0);
}
static bool light_edge_ok(const Gen& g, const Path& P) {
  if (!P.L.env && !(dot(P.L.n, P.v[P.k - 2].p - P.L.p) > 0.0f)) return false;
  return path_visible(g.S, g.F.pose, P, P.k - 2);
}

static void emit(const Gen& g, Path& P) {
  if (path_ok(g.S, g.F, P)) g.out.push_back(P);
}

// (1) Dynamic from emitter.
static void tech1(const Gen& g) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  PV xd = obj_point(g.S, g.F.pose, u);
  g.rng.draw(0, 0, 1, u);
  LightPt L;
  if (!sample_light(g.S, u, L)) return;
  double p = (1.0 / g.S.obj_area) * light_pdf(g.S, L);
  PV eye[MAXV];
  eye[0] = xd;
  V3 wi = towards(L, xd.p);
  Path P;
  for (int i = 0; i + 2 <= g.depth; ++i) {
    if (assemble(g, eye, i, nullptr, nullptr, -1, L, p, 0, P)) {
      if (i == 0 && !light_edge_ok(g, P)) return;  // blocked first connection: the sample fails
      if (camera_edge_ok(g, P)) emit(g, P);
    }
    if (i + 3 > g.depth) break;
    g.rng.draw(1, i + 1, 0, u);
    double pe = extend(g, eye[i], wi, u, eye[i + 1]);
    if (pe == 0.0) break;
    p *= pe;
    wi = normalize(eye[i].p - eye[i + 1].p);
  }
}

// Walk towards the light with next-event estimation at each walk vertex.
// light[0] is given; nee(j) produces the path ending at light[j].
template <class Fn>
static void light_walk(const Gen& g, PV* light, V3 wi0, double p0, int jmax, Fn&& nee) {
  float u[4];
  V3 wi = wi0;
  double p = p0;
  for (int j = 0; j <= jmax; ++j) {
    g.rng.draw(0, j + 1, 1, u);
    LightPt L;
    bool ok = sample_light(g.S, u, L);
    nee(j, ok, L, ok ? p * light_pdf(g.S, L) : 0.0);
    if (j == jmax) break;
    g.rng.draw(0, j + 1, 0, u);
    double pe = extend(g, light[j], wi, u, light[j + 1]);
    if (pe == 0.0) break;
    p *= pe;
    wi = normalize(light[j].p - light[j + 1].p);
  }
}

// (2) Dynamic from sensor.
static void tech2(const Gen& g) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  PV xd = obj_point(g.S, g.F.pose, u);
  if (g.depth < 3) return;
  Path P;
  P.v[0] = PV{g.S.cam.eye, g.S.cam.fwd, -1, false};
  P.v[1] = xd;
  P.k = 3;
  P.L.env = false;
  P.L.p = xd.p;  // placeholder end for the camera-edge test
  P.L.n = xd.n;
  if (raster(g.S.cam, xd.p) < 0 || !path_visible(g.S, g.F.pose, P, 0)) return;
  PV light[MAXV];
  V3 wi = normalize(g.S.cam.eye - xd.p);
  g.rng.draw(0, 0, 2, u);
  double pe = extend(g, xd, wi, u, light[0]);
  if (pe == 0.0) return;
  double p0 = (1.0 / g.S.obj_area) * pe;
  light_walk(g, light, normalize(xd.p - light[0].p), p0, g.depth - 3, [&](int j, bool ok, const LightPt& L, double p) {
    Path Q;
    if (!ok) return;
    if (!assemble(g, nullptr, -1, &xd, light, j, L, p, 1, Q)) return;
    if (light_edge_ok(g, Q)) emit(g, Q);
  });
}

// Walk towards the sensor with a camera connection at each walk vertex.
template <class Fn>
static void eye_walk(const Gen& g, PV* eye, V3 wi0, double p0, int imax, Fn&& cam) {
  float u[4];
  V3 wi = wi0;
  double p = p0;
  for (int i = 0; i <= imax; ++i) {
    cam(i, p);
    if (i == imax) break;
    g.rng.draw(1, i + 1, 0, u);
    double pe = extend(g, eye[i], wi, u, eye[i + 1]);
    if (pe == 0.0) break;
    p *= pe;
    wi = normalize(eye[i].p - eye[i + 1].p);
  }
}

// Lists of sub-path prefixes for the two-ended techniques (3), (6), (8).
struct SubPath {
  PV v[MAXV];
  double p[MAXV];        // density of the prefix ending at v[i]
  int n;
  bool conn[MAXV];       // endpoint connection valid at v[i]
  LightPt L[MAXV];       // light end for NEE at v[i]
  double pl[MAXV];       // light pdf of L[i]
};

// Paths of a sample with a light-side vertex l0 and (eye = true) a
// sensor-side vertex e0 on either side of the start (mid: x_D, or none for
// a ghost start): light walk from l0 with next-event estimation, eye walk
// from e0 with a camera connection at each vertex, every valid pairing.
// mid_cam: the sensor sees the start vertex directly, which adds the paths
// x_0 -> x_D -> l0 ... (the light walk then goes one bounce further).
static void two_ended(const Gen& g, const PV* mid, bool eye, PV e0, double pe0, V3 wie, PV l0, double pl0, V3 wil,
                      double pstart, int start, bool mid_cam = false) {
  // light side: l[0..], NEE at each vertex
  SubPath Ls, Es;
  Ls.n = 0;
  Es.n = 0;
  int extra = mid ? 1 : 0;
  int jmax = g.depth - 3 - extra + (mid_cam ? 1 : 0);  // i = 0 partner, or the sensor at x_D
  int imax = g.depth - 3 - extra;
  Ls.v[0] = l0;
  light_walk(g, Ls.v, wil, pl0, jmax, [&](int j, bool ok, const LightPt& L, double p) {
    Ls.n = j + 1;
    Ls.L[j] = L;
    Ls.pl[j] = p;
    Ls.conn[j] = ok;
  });
  if (mid_cam)
    for (int j = 0; j < Ls.n; ++j) {
      if (!Ls.conn[j]) continue;
      Path Q;
      if (!assemble(g, nullptr, -1, mid, Ls.v, j, Ls.L[j], pstart * Ls.pl[j], start, Q)) continue;
      if (light_edge_ok(g, Q)) emit(g, Q);
    }
  if (!eye) return;
  Es.v[0] = e0;
  eye_walk(g, Es.v, wie, pe0, imax, [&](int i, double p) {
    Es.n = i + 1;
    Es.p[i] = p;
  });
  for (int i = 0; i < Es.n; ++i) {
    // camera connection at eye[i]
    Path Pc;
    if (!assemble(g, Es.v, i, mid, Ls.v, 0, Ls.L[0], 0, start, Pc)) continue;
    if (!camera_edge_ok(g, Pc)) continue;
    for (int j = 0; j < Ls.n; ++j) {
      if (!Ls.conn[j]) continue;
      Path Q;
      double p = pstart * Es.p[i] * Ls.pl[j];
      if (!assemble(g, Es.v, i, mid, Ls.v, j, Ls.L[j], p, start, Q)) continue;
      if (light_edge_ok(g, Q)) emit(g, Q);
    }
  }
}

// (3) Dynamic two ends: cosine lobe about the outward normal towards the
// light side, then a BSDF direction towards the sensor.
static void tech3(const Gen& g) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  PV xd = obj_point(g.S, g.F.pose, u);
  if (g.depth < 4) return;
  g.rng.draw(0, 0, 2, u);
  V3 t, b;
  onb(xd.n, t, b);
  float r = std::sqrt(u[0]), ph = 2.0f * PIf * u[1];
  float z = std::sqrt(std::max(0.0f, 1.0f - u[0]));
  V3 wl = t * (r * std::cos(ph)) + b * (r * std::sin(ph)) + xd.n * z;
  if (!(dot(wl, xd.n) > 0.0f)) return;
  V3 ol = spawn_dir(g.S, xd.p, xd.n, wl);
  Hit hl = closest(g.S, g.F.pose, ol, wl);
  if (!hl.ok || (!hl.dyn && g.S.mats[hl.mat].type == MAT_EMITTER)) return;
  PV l0{hl.p, hl.n, hl.mat, hl.dyn};
  g.rng.draw(0, 0, 3, u);
  Material m = vertex_material(g.S, g.F, xd.mat, xd.dyn);
  // the sensor-side BSDF sample sees the light-side neighbour x_{m+1} as its
  // incoming direction (vertex to vertex, as the MIS tables evaluate it)
  const V3 wi = normalize(l0.p - xd.p);
  V3 we;
  if (!bsdf_sample(m, xd.n, wi, u[0], u[1], we)) return;
  V3 oe = spawn_dir(g.S, xd.p, xd.n, we);
  Hit he = closest(g.S, g.F.pose, oe, we);
  if (!he.ok || (!he.dyn && g.S.mats[he.mat].type == MAT_EMITTER)) return;
  PV e0{he.p, he.n, he.mat, he.dyn};
  D3 dl = dd(l0.p) - dd(ol), de = dd(e0.p) - dd(oe);
  double pl = ddot(dd(xd.n), dd(wl)) / PI * std::fabs(ddot(dd(l0.n), dnorm(dl))) / dlen2(dl);
  double pe = bsdf_pdf(m, dd(xd.n), dd(wi), dd(we)) * std::fabs(ddot(dd(e0.n), dnorm(de))) / dlen2(de);
  two_ended(g, &xd, true, e0, pe, normalize(xd.p - e0.p), l0, pl, normalize(xd.p - l0.p), 1.0 / g.S.obj_area, 0);
}

// (8) Learned proposal: a start x_D on the object whose light-side direction
// is drawn from the MLP's vMF mixture at x_D (object space), made defensive
// by a uniform-sphere component.  On the sensor
// side x_D is either seen by the camera directly (the paths of technique
// (2), whose BSDF direction the mixture replaces) or followed, as in
// technique (3), by a BSDF direction towards the sensor and an eye walk.
static void tech8(const Gen& g, const Proposal& Pr) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  PV xd = obj_point(g.S, g.F.pose, u);
  if (g.depth < 3 || !Pr.params) return;
  Lobes Lb = proposal_lobes(Pr, pose_inv_apply(g.F.pose, xd.p), pose_inv_rot(g.F.pose, xd.n));
  g.rng.draw(0, 0, 2, u);
  V3 wobj = t8_sample(Lb, u[0], u[1], u[2]);
  V3 wl = normalize(pose_rot(g.F.pose, wobj));
  V3 ol = spawn_dir(g.S, xd.p, xd.n, wl);
  Hit hl = closest(g.S, g.F.pose, ol, wl);
  if (!hl.ok || (!hl.dyn && g.S.mats[hl.mat].type == MAT_EMITTER)) return;
  PV l0{hl.p, hl.n, hl.mat, hl.dyn};
  D3 dl = dd(l0.p) - dd(ol);
  D3 wq = dnorm(dd(pose_inv_rot(g.F.pose, normalize(l0.p - ol))));
  double pl = t8_pdf(Lb, wq) * std::fabs(ddot(dd(l0.n), dnorm(dl))) / dlen2(dl);
  // the sensor sees x_D (the support test of the assembled paths checks the sides)
  Path C;
  C.v[0] = PV{g.S.cam.eye, g.S.cam.fwd, -1, false};
  C.v[1] = xd;
  C.k = 3;
  C.L.env = false;
  C.L.p = xd.p;  // placeholder end for the camera-edge test
  C.L.n = xd.n;
  const bool cam = raster(g.S.cam, xd.p) >= 0 && path_visible(g.S, g.F.pose, C, 0);
  // or a BSDF direction towards the sensor: its incoming direction is the
  // light-side neighbour x_{m+1} (vertex to vertex, as the MIS tables evaluate it)
  bool eye = false;
  PV e0{};
  double pe = 0.0;
  V3 oe{};
  if (g.depth >= 4) {
    g.rng.draw(0, 0, 3, u);
    Material m = vertex_material(g.S, g.F, xd.mat, xd.dyn);
    const V3 wi = normalize(l0.p - xd.p);
    V3 we;
    if (bsdf_sample(m, xd.n, wi, u[0], u[1], we)) {
      oe = spawn_dir(g.S, xd.p, xd.n, we);
      Hit he = closest(g.S, g.F.pose, oe, we);
      if (he.ok && !(!he.dyn && g.S.mats[he.mat].type == MAT_EMITTER)) {
        e0 = PV{he.p, he.n, he.mat, he.dyn};
        D3 de = dd(e0.p) - dd(oe);
        pe = bsdf_pdf(m, dd(xd.n), dd(wi), dd(we)) * std::fabs(ddot(dd(e0.n), dnorm(de))) / dlen2(de);
        eye = true;
      }
    }
  }
  two_ended(g, &xd, eye, e0, pe, eye ? normalize(xd.p - e0.p) : V3{}, l0, pl, normalize(xd.p - l0.p),
            1.0 / g.S.obj_area, 0, cam);
}

// (4) Ghost from emitter: the ray x_L -> x_G gives x_1 (eq. vertex1pdf).
static void tech4(const Gen& g) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  int gt;
  PV xg = obj_point(g.S, g.F.ghost, u, &gt);
  g.rng.draw(0, 0, 1, u);
  LightPt L;
  if (!sample_light(g.S, u, L) || L.env) return;
  if (!(dot(L.n, xg.p - L.p) > 0.0f)) return;
  V3 o = spawn(g.S, L.p, L.n, xg.p);
  V3 w = normalize(xg.p - o);
  float tg = length(xg.p - o);
  Hit h = closest(g.S, g.F.pose, o, w);
  if (!h.ok || !(h.t > tg)) return;
  if (!h.dyn && g.S.mats[h.mat].type == MAT_EMITTER) return;
  PV eye[MAXV];
  eye[0] = PV{h.p, h.n, h.mat, h.dyn};
  {
    Path Q;
    Q.k = 3;
    Q.v[1] = eye[0];
    Q.L = L;
    if (!ghost_on_edge(g, Q, 1, gt)) return;
  }
  D3 wg = dnorm(dd(eye[0].p) - dd(o));
  double cg = std::fabs(ddot(dd(xg.n), wg)), c1 = std::fabs(ddot(dd(eye[0].n), wg));
  double p = light_pdf(g.S, L) * (1.0 / g.S.obj_area) * dlen2(dd(xg.p) - dd(o)) / cg * c1 /
             dlen2(dd(eye[0].p) - dd(o));
  eye_walk(g, eye, normalize(L.p - eye[0].p), p, g.depth - 2, [&](int i, double pp) {
    Path P;
    if (!assemble(g, eye, i, nullptr, nullptr, -1, L, pp, 0, P)) return;
    if (camera_edge_ok(g, P)) emit(g, P);
  });
}

// (5) Ghost from sensor: the camera ray through x_G gives x_1.
static void tech5(const Gen& g) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  int gt;
  PV xg = obj_point(g.S, g.F.ghost, u, &gt);
  if (g.depth < 2) return;
  V3 w = normalize(xg.p - g.S.cam.eye);
  float tg = length(xg.p - g.S.cam.eye);
  Hit h = closest(g.S, g.F.pose, g.S.cam.eye, w);
  if (!h.ok || !(h.t > tg)) return;
  if (!h.dyn && g.S.mats[h.mat].type == MAT_EMITTER) return;
  PV light[MAXV];
  light[0] = PV{h.p, h.n, h.mat, h.dyn};
  if (raster(g.S.cam, light[0].p) < 0) return;
  {
    Path Q;
    Q.k = 3;
    Q.v[1] = light[0];
    Q.L.env = false;
    Q.L.p = light[0].p;
    Q.L.n = light[0].n;
    if (!ghost_on_edge(g, Q, 0, gt)) return;
  }
  D3 wg = dnorm(dd(light[0].p) - dd(g.S.cam.eye));
  double cg = std::fabs(ddot(dd(xg.n), wg)), c1 = std::fabs(ddot(dd(light[0].n), wg));
  double p0 = (1.0 / g.S.obj_area) * dlen2(dd(xg.p) - dd(g.S.cam.eye)) / cg * c1 /
              dlen2(dd(light[0].p) - dd(g.S.cam.eye));
  light_walk(g, light, normalize(g.S.cam.eye - light[0].p), p0, g.depth - 2,
             [&](int j, bool ok, const LightPt& L, double p) {
               Path Q;
               if (!ok) return;
               if (!assemble(g, nullptr, -1, nullptr, light, j, L, p, 0, Q)) return;
               if (light_edge_ok(g, Q)) emit(g, Q);
             });
}

// (6) Ghost two ends: a uniform direction through x_G, rays both ways.
static void tech6(const Gen& g, double p_dir) {
  float u[4];
  g.rng.draw(0, 0, 0, u);
  int gt;
  PV xg = obj_point(g.S, g.F.ghost, u, &gt);
  if (g.depth < 3) return;
  g.rng.draw(0, 0, 2, u);
  V3 w = sphere_dir(u[0], u[1]);
  Hit hl = closest(g.S, g.F.pose, xg.p, w);
  if (!hl.ok || (!hl.dyn && g.S.mats[hl.mat].type == MAT_EMITTER)) return;
  Hit he = closest(g.S, g.F.pose, xg.p, -w);
  if (!he.ok || (!he.dyn && g.S.mats[he.mat].type == MAT_EMITTER)) return;
  PV l0{hl.p, hl.n, hl.mat, hl.dyn}, e0{he.p, he.n, he.mat, he.dyn};
  {
    Path Q;
    Q.k = 4;
    Q.v[1] = e0;
    Q.v[2] = l0;
    Q.L.env = false;
    Q.L.p = l0.p;
    Q.L.n = l0.n;
    if (!ghost_on_edge(g, Q, 1, gt)) return;
  }
  D3 d = dd(l0.p) - dd(e0.p);
  D3 wu = dnorm(d);
  double G = std::fabs(ddot(dd(e0.n), wu)) * std::fabs(ddot(dd(l0.n), wu)) / dlen2(d);
  double pg = (1.0 / g.S.obj_area) * p_dir * G / std::fabs(ddot(dd(xg.n), wu));
  two_ended(g, nullptr, true, e0, 1.0, normalize(l0.p - e0.p), l0, 1.0, normalize(e0.p - l0.p), pg, 0);
}

// Camera path: jittered pixel ray; emission at x_1; NEE at every vertex.
// tech = 7: residual technique (7); tech = 0: plain frame rendering.
static void camera_path(const Gen& g, uint32_t sample) {
  const Camera& C = g.S.cam;
  int P = C.W * C.H;
  int pixel = (int)(sample % (uint32_t)P);
  float u[4];
  g.rng.draw(0, 0, 0, u);
  V3 w = camera_dir(C, pixel, u[0], u[1]);
  Hit h = closest(g.S, g.F.pose, C.eye, w);
  Path Q;
  Q.v[0] = PV{C.eye, C.fwd, -1, false};
  Q.tech = g.tech;
  Q.start = 0;
  Q.i = Q.j = -1;
  if (!h.ok) {
    if (g.S.has_env) {
      Q.k = 2;
      Q.L.env = true;
      Q.L.n = w;
      Q.L.p = mk(0, 0, 0);
      Q.L.Le = g.S.env;
      Q.p_gen = cam_pdf(g.S, Q);
      emit(g, Q);
    }
    return;
  }
  if (!h.dyn && g.S.mats[h.mat].type == MAT_EMITTER) {
    const Material& m = g.S.mats[h.mat];
    Q.k = 2;
    Q.L.env = false;
    Q.L.p = h.p;
    Q.L.n = h.n;
    Q.L.Le = dmk(m.emit[0], m.emit[1], m.emit[2]);
    Q.p_gen = cam_pdf(g.S, Q);
    emit(g, Q);
    return;
  }
  PV light[MAXV];
  light[0] = PV{h.p, h.n, h.mat, h.dyn};
  double p0 = camera_pdf(C, light[0].p, light[0].n);
  light_walk(g, light, -w, p0, g.depth - 2, [&](int j, bool ok, const LightPt& L, double p) {
    Path R;
    if (!ok) return;
    if (!assemble(g, nullptr, -1, nullptr, light, j, L, p, 0, R)) return;
    if (light_edge_ok(g, R)) emit(g, R);
  });
}

// ---------------------------------------------------------------- drivers
struct Params {
  int spp, depth;
  uint32_t mask;
  int two_way;
  uint64_t seed;
  uint32_t job;
  float alpha_min, d_min, jac_max, c_weight;
  int64_t s0, s1;
  int threads;
  int material_mode;
  int no_mapping;  // the path-mapping ablation: every pair is rejected
  int32_t tech_spp[8];  // samples per pixel of technique t (index t-1); 0: spp
  int balance;          // accepted pairs weighted by the balance heuristic over both directions
};

struct Record {
  int32_t dir, tech;
  uint32_t sample;
  int32_t k, pixel, reason, n_starts, pad;
  double val[3];
  double mis_total, mis_tech, p_gen;
  // techniques (2)/(3): proposal training record {x[6], w_obj[3], weight}
  double train[10];
  double mis_by_tech[9];  // every strategy's term of mis_total
};

struct Stats {
  int64_t paths, accepted, rejected[7], by_tech[9], zero_mis, samples, rays;
};

static int n_starts_for(const Scene& S, const Frame& F, const Path& P, int tech) {
  int k = P.k, n = 0;
  if ((tech >= 1 && tech <= 3) || tech == 8) {
    for (int m = 1; m <= k - 2; ++m)
      if (P.v[m].dyn && ((tech == 1 && m == k - 2) || (tech == 2 && m == 1 && m != k - 2) ||
                         (tech == 3 && m >= 2 && m <= k - 3) || (tech == 8 && m <= k - 3)))
        ++n;
  } else if (tech >= 4 && tech <= 6) {
    for (int a = 0; a <= k - 2; ++a) {
      int c = crossings(S, F, P, a).n;
      if ((tech == 4 && a == k - 2) || (tech == 5 && a == 0 && a != k - 2) ||
          (tech == 6 && a >= 1 && a <= k - 3))
        n += c;
    }
  } else {
    n = 1;
  }
  return n;
}

// Training record of a path generated by technique (2) or (3) at x_m,
// m = i + 2 (m = 1 for technique (2)):
// the proposal input at x_m, the direction to x_{m+1} (from the offset
// origin, in object space) and the path's mean absolute residual
// contribution over its generation density -- a sample of the directional
// distribution of residual energy at x_m that technique (8) learns.
static void train_record(const Scene& S, const Frame& F, const Proposal& Pr, const Path& X, D3 val, double* out) {
  const int m = X.i + 2;
  double x[MLP_IN];
  proposal_input(Pr, pose_inv_apply(F.pose, X.v[m].p), pose_inv_rot(F.pose, X.v[m].n), x);
  for (int a = 0; a < MLP_IN; ++a) out[a] = x[a];
  const V3 w = pose_inv_rot(F.pose, normalize(X.v[m + 1].p - origin(S, X, m, m + 1)));
  out[6] = w.x;
  out[7] = w.y;
  out[8] = w.z;
  out[9] = (std::fabs(val.x) + std::fabs(val.y) + std::fabs(val.z)) / 3.0 / X.p_gen;
}

static void residual_range(const Scene& S, const Frame& F, const Frame& Fp, int dir, int tech, double sigma,
                           const Params& Pm, int64_t s0, int64_t s1, double N, double* img, double* tech_img,
                           Stats& st, std::vector<Record>* recs, const Proposal* prop) {
  MisOpts O{Pm.mask, F.ghosts, 1.0 / (4.0 * PI), prop, &F, {}};
  for (int t = 0; t <= 8; ++t) O.ratio[t] = 1.0;
  for (int t = 1; t <= 8; ++t)
    if (Pm.tech_spp[t - 1] > 0) O.ratio[t] = (double)Pm.tech_spp[t - 1] / (double)Pm.spp;
  MapParams M{Pm.alpha_min, Pm.d_min, Pm.jac_max};
  double c = Pm.material_mode ? 1.0 : (double)Pm.c_weight;
  int P = S.cam.W * S.cam.H;
  std::vector<Path> paths;
  for (int64_t s = s0; s < s1; ++s) {
    paths.clear();
    Rng rng{(uint32_t)Pm.seed, (uint32_t)(Pm.seed >> 32), (uint32_t)s, (uint32_t)tech, (uint32_t)dir, Pm.job};
    Gen g{S, F, rng, Pm.depth, tech, paths};
    switch (tech) {
      case 1: tech1(g); break;
      case 2: tech2(g); break;
      case 3: tech3(g); break;
      case 4: tech4(g); break;
      case 5: tech5(g); break;
      case 6: tech6(g, 1.0 / (4.0 * PI)); break;
      case 7: camera_path(g, (uint32_t)s); break;
      case 8: tech8(g, *prop); break;
      default: break;
    }
    st.samples++;
    for (Path& X : paths) {
      if (tech == 7 && !is_dynamic(S, F, X)) continue;
      MisTerms mt = mis_terms(S, F, X, O);
      if (!(mt.total > 0.0)) {
        st.zero_mis++;
        continue;
      }
      int pix = path_pixel(S, X);
      double cf = cam_factor(S, X);
      D3 fx = contribution_rest(S, F, X) * cf;
      Path Y = X;
      // Without the mapping (the paper's path-mapping ablation) every path is
      // rejected: it keeps its own frame's term with weight 1.
      int reason = Pm.material_mode ? ACCEPT : (Pm.no_mapping ? REJECT_UNMAPPED : map_path(S, F, Fp, X, Y, M));
      D3 val;
      double total = mt.total;
      if (reason == ACCEPT) {
        D3 fy = contribution_rest(S, Fp, Y) * cf;
        if (Pm.balance && !Pm.material_mode) {
          // The other direction samples the same pair through Y = T(X), with
          // the strategy densities of its own frame; in X's measure their sum
          // is Sigma_f'(Y) |T'|, and the balance heuristic over the strategies
          // of both directions divides the pair's value by both sums.
          MisOpts Oy = O;
          Oy.ghosts = Fp.ghosts;
          Oy.frame = &Fp;
          MisTerms my = mis_terms(S, Fp, Y, Oy);
          const double jac = cam_pdf(S, X) / cam_pdf(S, Y);  // 1 unless x_1 was re-traced
          total = mt.total + my.total * jac;
          val = fx - fy;
        } else {
          val = (fx - fy) * c;
        }
        st.accepted++;
      } else {
        val = fx;
        st.rejected[reason == REJECT_UNMAPPED ? 0 : reason]++;
      }
      const D3 unweighted = val;
      val = val * (sigma / total / N);
      st.paths++;
      st.by_tech[tech]++;
      img[3 * pix + 0] += val.x;
      img[3 * pix + 1] += val.y;
      img[3 * pix + 2] += val.z;
      if (tech_img) {
        double* ti = tech_img + (size_t)(tech - 1) * 3 * P;
        ti[3 * pix + 0] += val.x;
        ti[3 * pix + 1] += val.y;
        ti[3 * pix + 2] += val.z;
      }
      if (recs) {
        Record r;
        std::memset(&r, 0, sizeof r);
        r.dir = dir;
        r.tech = tech;
        r.sample = (uint32_t)s;
        r.k = X.k;
        r.pixel = pix;
        r.reason = reason;
        r.n_starts = n_starts_for(S, F, X, tech);
        r.pad = ((X.i + 1) << 4) | (X.j + 1);
        r.val[0] = val.x;
        r.val[1] = val.y;
        r.val[2] = val.z;
        r.mis_total = total;
        r.mis_tech = mt.by_tech[tech];
        for (int t = 0; t < 9; ++t) r.mis_by_tech[t] = mt.by_tech[t];
        r.p_gen = X.p_gen;
        if (tech == 2 || tech == 3) train_record(S, F, *prop, X, unweighted, r.train);
        recs->push_back(r);
      }
    }
  }
}

static void frame_range(const Scene& S, const Frame& F, int dir, const Params& Pm, int64_t s0, int64_t s1,
                        double N, double* img, Stats& st) {
  std::vector<Path> paths;
  for (int64_t s = s0; s < s1; ++s) {
    paths.clear();
    Rng rng{(uint32_t)Pm.seed, (uint32_t)(Pm.seed >> 32), (uint32_t)s, 0u, (uint32_t)dir, Pm.job};
    Gen g{S, F, rng, Pm.depth, 0, paths};
    camera_path(g, (uint32_t)s);
    st.samples++;
    for (Path& X : paths) {
      int pix = path_pixel(S, X);
      D3 v = contribution_rest(S, F, X) * (cam_factor(S, X) / X.p_gen / N);
      img[3 * pix + 0] += v.x;
      img[3 * pix + 1] += v.y;
      img[3 * pix + 2] += v.z;
      st.paths++;
    }
  }
}

template <class Fn>
static void parallel(int threads, int64_t s0, int64_t s1, int npix, double* img, double* tech_img, int ntech,
                     Stats& st, Fn&& body) {
  if (threads <= 1 || s1 - s0 < 2 * threads) {
    const int64_t r0 = t_ray_queries;
    body(s0, s1, img, tech_img, st);
    st.rays += t_ray_queries - r0;
    return;
  }
  std::vector<std::vector<double>> imgs(threads, std::vector<double>((size_t)3 * npix, 0.0));
  std::vector<std::vector<double>> timgs(threads);
  std::vector<Stats> sts(threads);
  std::vector<std::thread> th;
  int64_t n = s1 - s0;
  for (int t = 0; t < threads; ++t) {
    std::memset(&sts[t], 0, sizeof(Stats));
    if (tech_img) timgs[t].assign((size_t)3 * npix * ntech, 0.0);
    int64_t a = s0 + n * t / threads, b = s0 + n * (t + 1) / threads;
    th.emplace_back([&, t, a, b] {
      const int64_t r0 = t_ray_queries;
      body(a, b, imgs[t].data(), tech_img ? timgs[t].data() : nullptr, sts[t]);
      sts[t].rays = t_ray_queries - r0;
    });
  }
  for (auto& x : th) x.join();
  for (int t = 0; t < threads; ++t) {
    for (size_t i = 0; i < imgs[t].size(); ++i) img[i] += imgs[t][i];
    if (tech_img)
      for (size_t i = 0; i < timgs[t].size(); ++i) tech_img[i] += timgs[t][i];
    st.paths += sts[t].paths;
    st.accepted += sts[t].accepted;
    st.zero_mis += sts[t].zero_mis;
    st.samples += sts[t].samples;
    st.rays += sts[t].rays;
    for (int r = 0; r < 7; ++r) st.rejected[r] += sts[t].rejected[r];
    for (int r = 0; r < 9; ++r) st.by_tech[r] += sts[t].by_tech[r];
  }
}

static Material mat_from(const float* m) {
  Material r;
  r.type = (int)m[0];
  for (int i = 0; i < 3; ++i) {
    r.albedo[i] = m[1 + i];
    r.emit[i] = m[5 + i];
  }
  r.rough = m[4];
  return r;
}

static Material object_material(const Scene& S) {
  return S.obj.empty() ? Material{} : S.mats[S.obj[0].mat];
}

}  // namespace orc

// ---------------------------------------------------------------- C entry points (ctypes)
using namespace orc;

extern "C" {

int orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U4 c;
  for (int i = 0; i < 4; ++i) c.v[i] = ctr[i];
  U4 r = philox(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = r.v[i];
  return 0;
}

void* orc_scene_create(const float* pos, int nv, const int* idx, int nf, const int* tri_mat, const int* tri_obj,
                       const float* mats, int nm, const float* env, const float* cam, int brute) {
  Scene* S = new Scene();
  S->ntri = nf;
  for (int i = 0; i < nm; ++i) S->mats.push_back(mat_from(mats + 8 * i));
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = 0; i < nv; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)pos[3 * i + a]);
      hi[a] = std::max(hi[a], (double)pos[3 * i + a]);
    }
  double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
  S->eps = (float)(1e-4 * diag);
  std::vector<double> la, oa;
  for (int ax = 0; ax < 3; ++ax) {
    S->obj_lo[ax] = INFINITY;
    S->obj_hi[ax] = -INFINITY;
  }
  for (int f = 0; f < nf; ++f) {
    Tri t;
    V3 a = mk(pos[3 * idx[3 * f]], pos[3 * idx[3 * f] + 1], pos[3 * idx[3 * f] + 2]);
    V3 b = mk(pos[3 * idx[3 * f + 1]], pos[3 * idx[3 * f + 1] + 1], pos[3 * idx[3 * f + 1] + 2]);
    V3 c = mk(pos[3 * idx[3 * f + 2]], pos[3 * idx[3 * f + 2] + 1], pos[3 * idx[3 * f + 2] + 2]);
    t.v0 = a;
    t.e1 = b - a;
    t.e2 = c - a;
    t.n = normalize(cross(t.e1, t.e2));
    t.mat = tri_mat[f];
    t.id = f;
    D3 cr = dmk((double)t.e1.y * t.e2.z - (double)t.e1.z * t.e2.y, (double)t.e1.z * t.e2.x - (double)t.e1.x * t.e2.z,
                (double)t.e1.x * t.e2.y - (double)t.e1.y * t.e2.x);
    t.area = 0.5 * std::sqrt(dlen2(cr));
    if (tri_obj[f]) {
      S->obj.push_back(t);
      oa.push_back(t.area);
      for (V3 q : {a, b, c}) {
        const float cq[3] = {q.x, q.y, q.z};
        for (int ax = 0; ax < 3; ++ax) {
          S->obj_lo[ax] = std::min(S->obj_lo[ax], cq[ax]);
          S->obj_hi[ax] = std::max(S->obj_hi[ax], cq[ax]);
        }
      }
    } else {
      if (S->mats[t.mat].type == MAT_EMITTER) {
        S->lights.push_back((int)S->stat.size());
        la.push_back(t.area);
      }
      S->stat.push_back(t);
    }
  }
  auto cdf = [](const std::vector<double>& a, std::vector<float>& out, double& tot) {
    tot = 0;
    for (double x : a) tot += x;
    double run = 0;
    out.clear();
    for (double x : a) {
      run += x;
      out.push_back((float)(run / tot));
    }
  };
  cdf(la, S->light_cdf, S->light_area);
  cdf(oa, S->obj_cdf, S->obj_area);
  S->env = dmk(env[0], env[1], env[2]);
  S->has_env = env[0] > 0 || env[1] > 0 || env[2] > 0;
  Camera& C = S->cam;
  C.eye = mk(cam[0], cam[1], cam[2]);
  C.fwd = normalize(mk(cam[3], cam[4], cam[5]) - C.eye);
  C.right = normalize(cross(C.fwd, mk(cam[6], cam[7], cam[8])));
  C.up = cross(C.right, C.fwd);
  C.W = (int)cam[10];
  C.H = (int)cam[11];
  C.aspect = (float)C.W / (float)C.H;
  C.tan_half = std::tan(cam[9] * 0.5f * PIf / 180.0f);
  C.a_film = 4.0 * (double)C.aspect * (double)C.tan_half * (double)C.tan_half;
  S->brute = brute != 0;
  if (!S->brute) {
    bvh_build(S->bstat, S->stat);
    bvh_build(S->bobj, S->obj);
  }
  return S;
}

void orc_scene_destroy(void* s) { delete (Scene*)s; }

double orc_scene_eps(void* s) { return ((Scene*)s)->eps; }
double orc_object_area(void* s) { return ((Scene*)s)->obj_area; }

// Closest hit for a batch of rays in the frame whose object pose is `pose`.
int orc_trace(void* sp, const float* pose, const float* rays, int n, float* t_out, int* id_out) {
  Scene& S = *(Scene*)sp;
  Pose P = pose_from(pose);
  for (int i = 0; i < n; ++i) {
    V3 o = mk(rays[6 * i], rays[6 * i + 1], rays[6 * i + 2]);
    V3 d = mk(rays[6 * i + 3], rays[6 * i + 4], rays[6 * i + 5]);
    Hit h = closest(S, P, o, d);
    t_out[i] = h.ok ? h.t : -1.0f;
    id_out[i] = h.ok ? h.id : -1;
  }
  return 0;
}

// GGX terms on their own, for the microfacet pins (normalisation of D, the
// weak white furnace of Smith G1 with D).
double orc_ggx_D(double a, double nh) { return ggx_D(a, nh); }
double orc_ggx_G1(double a, double c) { return ggx_G1(a, c); }

// BSDF helpers for the normalisation pins (Lambertian/GGX).
double orc_bsdf_eval(const float* m, const double* n, const double* wi, const double* wo, double* rgb) {
  D3 r = bsdf_eval(mat_from(m), dmk(n[0], n[1], n[2]), dmk(wi[0], wi[1], wi[2]), dmk(wo[0], wo[1], wo[2]));
  rgb[0] = r.x;
  rgb[1] = r.y;
  rgb[2] = r.z;
  return bsdf_pdf(mat_from(m), dmk(n[0], n[1], n[2]), dmk(wi[0], wi[1], wi[2]), dmk(wo[0], wo[1], wo[2]));
}
int orc_bsdf_sample(const float* m, const float* n, const float* wi, float u0, float u1, float* wo) {
  V3 w;
  bool ok = bsdf_sample(mat_from(m), mk(n[0], n[1], n[2]), mk(wi[0], wi[1], wi[2]), u0, u1, w);
  wo[0] = w.x;
  wo[1] = w.y;
  wo[2] = w.z;
  return ok ? 1 : 0;
}

// Plain path tracing of one frame: which = 1 (old) or 2 (new), on the Philox
// streams of direction `dir` (the frame's own: 0 for the new frame, 1 for the
// old; tracing both frames on one direction's streams correlates them).
int orc_render_frame_dir(void* sp, const float* pose_old, const float* pose_new, const float* new_mat, int which,
                         int dir, const Params* pm, double* img, int64_t* stats_out) {
  Scene& S = *(Scene*)sp;
  Frame F;
  F.ghosts = false;
  F.pose = pose_from(which == 2 ? pose_new : pose_old);
  F.ghost = F.pose;
  F.objmat = (which == 2 && new_mat) ? mat_from(new_mat) : object_material(S);
  int P = S.cam.W * S.cam.H;
  int64_t N = (int64_t)pm->spp * P;
  int64_t s0 = pm->s0, s1 = pm->s1 < 0 ? N : pm->s1;
  Stats st;
  std::memset(&st, 0, sizeof st);
  parallel(pm->threads, s0, s1, P, img, nullptr, 0, st,
           [&](int64_t a, int64_t b, double* im, double*, Stats& s) { frame_range(S, F, dir, *pm, a, b, (double)N, im, s); });
  if (stats_out) {
    stats_out[0] = st.samples;
    stats_out[1] = st.paths;
  }
  return 0;
}
int orc_render_frame(void* sp, const float* pose_old, const float* pose_new, const float* new_mat, int which,
                     const Params* pm, double* img, int64_t* stats_out) {
  return orc_render_frame_dir(sp, pose_old, pose_new, new_mat, which, which == 2 ? 0 : 1, pm, img, stats_out);
}

// Residual I2 - I1.  Motion edits: pose_old/pose_new are the object poses of
// the two frames.  Material edits (pm->material_mode): new_mat replaces the
// object's material in the new frame; the poses must coincide.
static Proposal make_proposal(const Scene& S, const float* mlp) {
  Proposal Pr;
  Pr.params = mlp;
  const float* lo = S.obj_lo;
  const float* hi = S.obj_hi;
  Pr.center = mk(0.5f * (lo[0] + hi[0]), 0.5f * (lo[1] + hi[1]), 0.5f * (lo[2] + hi[2]));
  Pr.inv_half = mk(2.0f / std::max(hi[0] - lo[0], 1e-6f), 2.0f / std::max(hi[1] - lo[1], 1e-6f),
                   2.0f / std::max(hi[2] - lo[2], 1e-6f));
  return Pr;
}

int orc_mlp_forward(const float* params, const double* x, int n, int bf16, double* out) {
  for (int i = 0; i < n; ++i) mlp_forward(params, x + 6 * i, bf16 != 0, out + MLP_OUT * i);
  return MLP_NPARAM;
}
double orc_mlp_loss_grad(const float* params, const float* rec, int n, int bf16, double* grad) {
  return mlp_loss_grad(params, rec, n, bf16 != 0, grad);
}
double orc_vmf_pdf(const double* raw, const double* w) {
  Lobes L = lobes_of(raw);
  return vmf_pdf(L, dmk(w[0], w[1], w[2]));
}
int orc_vmf_sample(const double* raw, float u0, float u1, float u2, float* w) {
  Lobes L = lobes_of(raw);
  V3 v = vmf_sample(L, u0, u1, u2);
  w[0] = v.x;
  w[1] = v.y;
  w[2] = v.z;
  return 0;
}
int orc_proposal_input(void* sp, const float* p_obj, const float* n_obj, double* x) {
  Proposal Pr = make_proposal(*(Scene*)sp, nullptr);
  proposal_input(Pr, mk(p_obj[0], p_obj[1], p_obj[2]), mk(n_obj[0], n_obj[1], n_obj[2]), x);
  return 0;
}

int orc_render_residual(void* sp, const float* pose_old, const float* pose_new, const float* new_mat,
                        const Params* pm, double* img, double* tech_img, int64_t* stats_out, Record* recs,
                        int64_t rec_cap, int64_t* rec_count, const float* mlp) {
  Scene& S = *(Scene*)sp;
  const Proposal prop = make_proposal(S, mlp);
  Frame F2, F1;
  F2.pose = pose_from(pose_new);
  F1.pose = pose_from(pose_old);
  F2.ghost = F1.pose;
  F1.ghost = F2.pose;
  F2.ghosts = F1.ghosts = !pm->material_mode;
  F1.objmat = object_material(S);
  F2.objmat = pm->material_mode && new_mat ? mat_from(new_mat) : F1.objmat;
  int P = S.cam.W * S.cam.H;
  int64_t N = (int64_t)pm->spp * P;
  int64_t s0 = pm->s0, s1 = pm->s1 < 0 ? N : pm->s1;
  Stats st;
  std::memset(&st, 0, sizeof st);
  std::vector<Record> rv;
  bool want = recs != nullptr && pm->threads <= 1;
  int ndir = (pm->two_way && !pm->material_mode) ? 2 : 1;
  for (int d = 0; d < ndir; ++d) {
    const Frame& F = d == 0 ? F2 : F1;
    const Frame& Fp = d == 0 ? F1 : F2;
    double sigma = d == 0 ? 1.0 : -1.0;
    for (int t = 1; t <= 8; ++t) {
      if (!((pm->mask >> (t - 1)) & 1u)) continue;
      if (pm->material_mode && t >= 4 && t <= 6) continue;
      if (t == 8 && !mlp) continue;
      // technique t's own sample count (the full stream only): tech_spp x pixels
      const int64_t s1t = pm->tech_spp[t - 1] > 0 ? (int64_t)pm->tech_spp[t - 1] * P : s1;
      parallel(pm->threads, s0, s1t, P, img, tech_img, 8, st,
               [&](int64_t a, int64_t b, double* im, double* ti, Stats& s) {
                 residual_range(S, F, Fp, d, t, sigma, *pm, a, b, (double)N, im, ti, s, want ? &rv : nullptr,
                                &prop);
               });
    }
  }
  if (stats_out) {
    stats_out[0] = st.samples;
    stats_out[1] = st.paths;
    stats_out[2] = st.accepted;
    for (int r = 1; r <= 6; ++r) stats_out[2 + r] = st.rejected[r];
    stats_out[9] = st.zero_mis;
    for (int t = 1; t <= 8; ++t) stats_out[9 + t] = st.by_tech[t];
    stats_out[18] = st.rejected[0];
    stats_out[19] = st.rays;
  }
  if (rec_count) {
    *rec_count = (int64_t)rv.size();
    if (recs)
      for (int64_t i = 0; i < (int64_t)rv.size() && i < rec_cap; ++i) recs[i] = rv[(size_t)i];
  }
  return 0;
}

// Mapping symmetry check (Sec. 5, two-way mapping): for every path generated
// in frame f whose mapped path is itself a valid dynamic path of f', map back
// and compare.  out[0] = checked pairs, out[1] = acceptance disagreements,
// out[2] = accepted round trips that do not return to x, out[3] = accepted.
int orc_map_check(void* sp, const float* pose_old, const float* pose_new, const Params* pm, int64_t* out) {
  Scene& S = *(Scene*)sp;
  Frame F2, F1;
  F2.pose = pose_from(pose_new);
  F1.pose = pose_from(pose_old);
  F2.ghost = F1.pose;
  F1.ghost = F2.pose;
  F2.ghosts = F1.ghosts = true;
  F1.objmat = F2.objmat = object_material(S);
  MapParams M{pm->alpha_min, pm->d_min, pm->jac_max};
  int64_t N = (int64_t)pm->spp * S.cam.W * S.cam.H;
  int64_t s1 = pm->s1 < 0 ? N : pm->s1;
  for (int i = 0; i < 4; ++i) out[i] = 0;
  std::vector<Path> paths;
  for (int d = 0; d < 2; ++d) {
    const Frame& F = d == 0 ? F2 : F1;
    const Frame& Fp = d == 0 ? F1 : F2;
    for (int t = 1; t <= 7; ++t) {
      for (int64_t smp = pm->s0; smp < s1; ++smp) {
        paths.clear();
        Rng rng{(uint32_t)pm->seed, (uint32_t)(pm->seed >> 32), (uint32_t)smp, (uint32_t)t, (uint32_t)d, pm->job};
        Gen g{S, F, rng, pm->depth, t, paths};
        switch (t) {
          case 1: tech1(g); break;
          case 2: tech2(g); break;
          case 3: tech3(g); break;
          case 4: tech4(g); break;
          case 5: tech5(g); break;
          case 6: tech6(g, 1.0 / (4.0 * PI)); break;
          default: camera_path(g, (uint32_t)smp); break;
        }
        for (Path& X : paths) {
          if (!is_dynamic(S, F, X)) continue;
          Path Y;
          int rx = map_path(S, F, Fp, X, Y, M);
          if (rx == R1 || rx == R5 || rx == R6) continue;  // y is not a valid path of f'
          if (!supported(S, Fp, Y, false)) continue;
          bool vis = true;
          for (int a = 0; a <= Y.k - 2 && vis; ++a) vis = path_visible(S, Fp.pose, Y, a);
          if (!vis || !is_dynamic(S, Fp, Y)) continue;
          Path Z;
          int ry = map_path(S, Fp, F, Y, Z, M);
          out[0]++;
          if ((rx == ACCEPT) != (ry == ACCEPT)) out[1]++;
          if (rx == ACCEPT && ry == ACCEPT) {
            out[3]++;
            for (int i = 1; i <= X.k - 2; ++i)
              if (length(Z.v[i].p - X.v[i].p) > 10.0f * S.eps) {
                out[2]++;
                break;
              }
          }
        }
      }
    }
  }
  return 0;
}

}  // extern "C"
