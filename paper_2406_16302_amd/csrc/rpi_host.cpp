// Host runtime of librpi: validation, binned-SAH BVH construction, area CDFs,
// upload, chunk planning and the launch sequence of the residual estimator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rpi.h"
#include "rpi_internal.h"

using namespace rpi;

static thread_local std::string g_err;

static rpi_status fail(rpi_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(e_ == hipErrorOutOfMemory ? RPI_ERR_OUT_OF_MEMORY : RPI_ERR_DEVICE, \
                                      std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// ------------------------------------------------------------------ BVH build (host)
namespace {

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int a = 0; a < 3; ++a) {
      lo[a] = INFINITY;
      hi[a] = -INFINITY;
    }
  }
  void grow(const float p[3]) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  float area() const {
    const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (!(dx >= 0)) return 0.0f;
    return 2.0f * (dx * dy + dy * dz + dz * dx);
  }
};

struct HostTri {
  float v0[3], v1[3], v2[3];
  int id, mat;
};

struct BuiltBvh {
  std::vector<float4> nodes;
  std::vector<float4> tris;
  int max_depth = 0;
};

constexpr int kLeafMax = 4;
constexpr int kBins = 16;
constexpr int kMedianDepth = 24;  // below this depth splits are object medians (bounded stack use)

// Binned SAH (16 bins per axis) with object-median splits from depth 24 on;
// children's boxes are stored in their parent (64-byte nodes).
class Builder {
 public:
  explicit Builder(const std::vector<HostTri>& t) : tris_(t) {
    const size_t n = t.size();
    cen_.resize(n);
    box_.resize(n);
    order_.resize(n);
    for (size_t i = 0; i < n; ++i) {
      box_[i].reset();
      box_[i].grow(t[i].v0);
      box_[i].grow(t[i].v1);
      box_[i].grow(t[i].v2);
      for (int a = 0; a < 3; ++a) cen_[i][a] = 0.5f * (box_[i].lo[a] + box_[i].hi[a]);
      order_[i] = (int)i;
    }
  }

  bool build(BuiltBvh& out, std::string& err) {
    out.nodes.clear();
    out.tris.clear();
    const int n = (int)tris_.size();
    if (n == 0) {
      err = "empty triangle set";
      return false;
    }
    // root node holds the two children of the full range
    out.nodes.resize(4);
    struct Job {
      int node, slot, first, count, depth;
    };
    std::vector<Job> st;
    int l, r;
    split(0, n, 0, l);
    r = n - l;
    if (n <= kLeafMax) {
      l = n;
      r = 0;
    }
    st.push_back({0, 0, 0, l, 1});
    st.push_back({0, 1, l, r, 1});
    while (!st.empty()) {
      Job j = st.back();
      st.pop_back();
      Box b;
      range_box(j.first, j.count, b);
      int32_t link;
      if (j.count <= kLeafMax) {
        const int first = (int)out.tris.size() / 3;
        for (int i = j.first; i < j.first + j.count; ++i) push_tri(out, tris_[order_[i]]);
        if (first >= (1 << 27)) {
          err = "too many triangles for the leaf encoding";
          return false;
        }
        link = (int32_t)(0x80000000u | ((uint32_t)first << 4) | (uint32_t)j.count);
        out.max_depth = std::max(out.max_depth, j.depth);
      } else {
        if (j.depth + 1 >= kStackDepth) {
          err = "BVH deeper than the traversal stack";
          return false;
        }
        const int node = (int)out.nodes.size() / 4;
        out.nodes.resize(out.nodes.size() + 4);
        int cl;
        split(j.first, j.count, j.depth, cl);
        st.push_back({node, 1, j.first + cl, j.count - cl, j.depth + 1});
        st.push_back({node, 0, j.first, cl, j.depth + 1});
        link = node;
      }
      set_child(out, j.node, j.slot, b, link, j.count == 0);
    }
    return true;
  }

 private:
  void range_box(int first, int count, Box& b) {
    b.reset();
    for (int i = first; i < first + count; ++i) b.grow(box_[order_[i]]);
  }

  // Partition [first, first+count) and return the left count.
  void split(int first, int count, int depth, int& left) {
    if (count <= 1) {
      left = count;
      return;
    }
    Box cb;
    cb.reset();
    for (int i = first; i < first + count; ++i) cb.grow(cen_[order_[i]].data());
    int best_axis = -1, best_bin = -1;
    float best_cost = INFINITY;
    if (depth < kMedianDepth) {
      for (int a = 0; a < 3; ++a) {
        const float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0)) continue;
        Box bb[kBins];
        int bc[kBins] = {0};
        for (auto& x : bb) x.reset();
        for (int i = first; i < first + count; ++i) {
          const int t = order_[i];
          int k = (int)((cen_[t][a] - cb.lo[a]) / ext * kBins);
          k = std::min(std::max(k, 0), kBins - 1);
          bc[k]++;
          bb[k].grow(box_[t]);
        }
        float rarea[kBins];
        int rcnt[kBins];
        Box acc;
        acc.reset();
        int c = 0;
        for (int k = kBins - 1; k > 0; --k) {
          acc.grow(bb[k]);
          c += bc[k];
          rarea[k] = acc.area();
          rcnt[k] = c;
        }
        acc.reset();
        c = 0;
        for (int k = 0; k < kBins - 1; ++k) {
          acc.grow(bb[k]);
          c += bc[k];
          if (c == 0 || rcnt[k + 1] == 0) continue;
          const float cost = acc.area() * c + rarea[k + 1] * rcnt[k + 1];
          if (cost < best_cost) {
            best_cost = cost;
            best_axis = a;
            best_bin = k;
          }
        }
      }
    }
    int* beg = order_.data() + first;
    if (best_axis >= 0) {
      const int a = best_axis;
      const float ext = cb.hi[a] - cb.lo[a];
      int* mid = std::partition(beg, beg + count, [&](int t) {
        int k = (int)((cen_[t][a] - cb.lo[a]) / ext * kBins);
        k = std::min(std::max(k, 0), kBins - 1);
        return k <= best_bin;
      });
      left = (int)(mid - beg);
      if (left > 0 && left < count) return;
    }
    // object median on the widest centroid axis
    int a = 0;
    for (int q = 1; q < 3; ++q)
      if (cb.hi[q] - cb.lo[q] > cb.hi[a] - cb.lo[a]) a = q;
    left = count / 2;
    std::nth_element(beg, beg + left, beg + count, [&](int x, int y) {
      return cen_[x][a] < cen_[y][a] || (cen_[x][a] == cen_[y][a] && x < y);
    });
  }

  static void push_tri(BuiltBvh& out, const HostTri& t) {
    float e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = t.v1[a] - t.v0[a];
      e2[a] = t.v2[a] - t.v0[a];
    }
    float id, mat;
    std::memcpy(&id, &t.id, 4);
    std::memcpy(&mat, &t.mat, 4);
    out.tris.push_back(make_float4(t.v0[0], t.v0[1], t.v0[2], id));
    out.tris.push_back(make_float4(e1[0], e1[1], e1[2], mat));
    out.tris.push_back(make_float4(e2[0], e2[1], e2[2], 0.0f));
  }

  static void set_child(BuiltBvh& out, int node, int slot, const Box& b0, int32_t link, bool empty) {
    Box b = b0;
    if (empty) {  // an empty leaf: an inverted box no ray can enter
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = 1e30f;
        b.hi[a] = -1e30f;
      }
    } else {
      for (int a = 0; a < 3; ++a) {  // conservative padding against rounding in the slab test
        const float pad = 1e-5f * (b.hi[a] - b.lo[a]) + 1e-6f * (std::fabs(b.lo[a]) + std::fabs(b.hi[a])) + 1e-7f;
        b.lo[a] -= pad;
        b.hi[a] += pad;
      }
    }
    float* f = reinterpret_cast<float*>(&out.nodes[4 * node]);
    int32_t* iv = reinterpret_cast<int32_t*>(&out.nodes[4 * node + 3]);
    if (slot == 0) {
      f[0] = b.lo[0];
      f[1] = b.lo[1];
      f[2] = b.lo[2];
      f[3] = b.hi[0];
      f[4] = b.hi[1];
      f[5] = b.hi[2];
      iv[0] = link;
    } else {
      f[6] = b.lo[0];
      f[7] = b.lo[1];
      f[8] = b.lo[2];
      f[9] = b.hi[0];
      f[10] = b.hi[1];
      f[11] = b.hi[2];
      iv[1] = link;
    }
    iv[2] = 0;
    iv[3] = 0;
  }

  const std::vector<HostTri>& tris_;
  std::vector<std::array<float, 3>> cen_;
  std::vector<Box> box_;
  std::vector<int> order_;
};

template <class T>
rpi_status upload(const std::vector<T>& v, T** out) {
  *out = nullptr;
  if (v.empty()) return RPI_OK;
  HIP_OK(hipMalloc((void**)out, v.size() * sizeof(T)));
  HIP_OK(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return RPI_OK;
}

Pose pose_of(const float* m) {
  Pose P;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P.r[3 * i + j] = m[4 * i + j];
    P.t[i] = m[4 * i + 3];
  }
  return P;
}
const float kIdentity[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};

Material mat_of(const float* m) {
  Material r;
  r.type = (int)m[0];
  r.albedo = v3(m[1], m[2], m[3]);
  r.rough = m[4];
  r.emit = v3(m[5], m[6], m[7]);
  return r;
}

}  // namespace

// ------------------------------------------------------------------ scene / edit objects
struct rpi_scene {
  DevScene dev;
  std::vector<void*> allocs;
  float obj_lo[3], obj_hi[3];  // object bounds in object space (= old pose)
  Material obj_mat;
  float diag;
  int W, H;
  int bvh_depth_static, bvh_depth_obj;
  // last records (RPI_FLAG_RECORDS)
  std::vector<uint32_t> rec_host;
  std::mutex mu;
};

struct rpi_edit {
  int kind;
  float pose_old[12], pose_new[12];
  Material new_mat;
};

static bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

extern "C" const char* rpi_last_error(void) { return g_err.c_str(); }
extern "C" const char* rpi_version(void) { return "rpi 0.1 (gfx950)"; }

extern "C" rpi_status rpi_build_scene(const rpi_scene_desc* d, rpi_scene** out) {
  if (!d || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->num_vertices <= 0 || d->num_triangles <= 0 || !d->positions || !d->indices || !d->tri_material ||
      !d->tri_object || !d->materials || d->num_materials <= 0 || !d->camera)
    return fail(RPI_ERR_INVALID_ARG, "missing scene arrays");
  for (int i = 0; i < d->num_vertices; ++i)
    if (!finite3(d->positions + 3 * i)) return fail(RPI_ERR_INVALID_ARG, "non-finite vertex " + std::to_string(i));
  for (int m = 0; m < d->num_materials; ++m) {
    const float* r = d->materials + 8 * m;
    const int t = (int)r[0];
    if (!(t == MAT_DIFFUSE || t == MAT_GGX || t == MAT_EMITTER) || (float)t != r[0])
      return fail(RPI_ERR_INVALID_ARG, "bad material type in row " + std::to_string(m));
    if (t == MAT_GGX && !(r[4] > 0.0f && r[4] <= 1.0f))
      return fail(RPI_ERR_INVALID_ARG, "GGX roughness must be in (0, 1]");
  }
  const float* cam = d->camera;
  if (!finite3(cam) || !finite3(cam + 3) || !finite3(cam + 6) || !(cam[9] > 0.0f && cam[9] < 179.0f) ||
      !(cam[10] >= 1.0f && cam[11] >= 1.0f) || cam[10] != std::floor(cam[10]) || cam[11] != std::floor(cam[11]))
    return fail(RPI_ERR_INVALID_ARG, "bad camera");
  std::unique_ptr<rpi_scene> S(new rpi_scene());
  std::vector<HostTri> stat, obj;
  std::vector<double> la, oa;
  std::vector<float4> obj_flat, light_flat;
  for (int f = 0; f < d->num_triangles; ++f) {
    HostTri t;
    const int* ix = d->indices + 3 * f;
    for (int c = 0; c < 3; ++c)
      if (ix[c] < 0 || ix[c] >= d->num_vertices)
        return fail(RPI_ERR_INVALID_ARG, "index out of range in triangle " + std::to_string(f));
    std::memcpy(t.v0, d->positions + 3 * ix[0], 12);
    std::memcpy(t.v1, d->positions + 3 * ix[1], 12);
    std::memcpy(t.v2, d->positions + 3 * ix[2], 12);
    t.id = f;
    t.mat = d->tri_material[f];
    if (t.mat < 0 || t.mat >= d->num_materials) return fail(RPI_ERR_INVALID_ARG, "material id out of range");
    const int type = (int)d->materials[8 * t.mat];
    double e1[3], e2[3];
    float fe1[3], fe2[3];
    for (int a = 0; a < 3; ++a) {
      fe1[a] = t.v1[a] - t.v0[a];
      fe2[a] = t.v2[a] - t.v0[a];
      e1[a] = fe1[a];
      e2[a] = fe2[a];
    }
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    float idf, matf;
    std::memcpy(&idf, &t.id, 4);
    std::memcpy(&matf, &t.mat, 4);
    if (d->tri_object[f]) {
      if (type == MAT_EMITTER) return fail(RPI_ERR_UNSUPPORTED, "emissive dynamic object");
      obj.push_back(t);
      oa.push_back(area);
      obj_flat.push_back(make_float4(t.v0[0], t.v0[1], t.v0[2], idf));
      obj_flat.push_back(make_float4(fe1[0], fe1[1], fe1[2], matf));
      obj_flat.push_back(make_float4(fe2[0], fe2[1], fe2[2], 0.0f));
    } else {
      if (type == MAT_EMITTER) {
        if (!(area > 0)) return fail(RPI_ERR_INVALID_ARG, "zero-area emitter triangle");
        la.push_back(area);
        light_flat.push_back(make_float4(t.v0[0], t.v0[1], t.v0[2], idf));
        light_flat.push_back(make_float4(fe1[0], fe1[1], fe1[2], matf));
        light_flat.push_back(make_float4(fe2[0], fe2[1], fe2[2], 0.0f));
      }
      stat.push_back(t);
    }
  }
  if (obj.empty()) return fail(RPI_ERR_UNSUPPORTED, "no dynamic triangles (tri_object == 1)");
  if (stat.empty()) return fail(RPI_ERR_UNSUPPORTED, "no static triangles");
  // area CDFs, built in double, stored as float
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
  std::vector<float> lcdf, ocdf;
  double ltot = 0, otot = 0;
  cdf(la, lcdf, ltot);
  cdf(oa, ocdf, otot);
  if (!(otot > 0)) return fail(RPI_ERR_INVALID_ARG, "zero-area object");
  const bool has_env = d->env && (d->env[0] > 0 || d->env[1] > 0 || d->env[2] > 0);
  if (la.empty() && !has_env) return fail(RPI_ERR_UNSUPPORTED, "scene has no emitter");
  // BVHs
  BuiltBvh bs, bo;
  std::string err;
  {
    Builder b(stat);
    if (!b.build(bs, err)) return fail(RPI_ERR_UNSUPPORTED, "static BVH: " + err);
  }
  {
    Builder b(obj);
    if (!b.build(bo, err)) return fail(RPI_ERR_UNSUPPORTED, "object BVH: " + err);
  }
  S->bvh_depth_static = bs.max_depth;
  S->bvh_depth_obj = bo.max_depth;
  // scene diagonal and ray offset
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = 0; i < d->num_vertices; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)d->positions[3 * i + a]);
      hi[a] = std::max(hi[a], (double)d->positions[3 * i + a]);
    }
  const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                (hi[2] - lo[2]) * (hi[2] - lo[2]));
  S->diag = (float)diag;
  for (int a = 0; a < 3; ++a) {
    S->obj_lo[a] = INFINITY;
    S->obj_hi[a] = -INFINITY;
  }
  for (const auto& t : obj)
    for (const float* p : {t.v0, t.v1, t.v2})
      for (int a = 0; a < 3; ++a) {
        S->obj_lo[a] = std::min(S->obj_lo[a], p[a]);
        S->obj_hi[a] = std::max(S->obj_hi[a], p[a]);
      }
  S->obj_mat = mat_of(d->materials + 8 * obj[0].mat);
  for (const auto& t : obj)
    if (t.mat != obj[0].mat) return fail(RPI_ERR_UNSUPPORTED, "the dynamic object must use a single material");

  DevScene& D = S->dev;
  std::memset(&D, 0, sizeof D);
  std::vector<float> mats(d->materials, d->materials + 8 * d->num_materials);
  rpi_status rc;
  auto up = [&](auto& v, auto** p) -> rpi_status {
    rpi_status r = upload(v, p);
    if (r == RPI_OK && *p) S->allocs.push_back((void*)*p);
    return r;
  };
  float4 *sn, *stt, *on, *ot, *of, *lf;
  float *oc, *lc, *mt;
  if ((rc = up(bs.nodes, &sn)) || (rc = up(bs.tris, &stt)) || (rc = up(bo.nodes, &on)) || (rc = up(bo.tris, &ot)) ||
      (rc = up(obj_flat, &of)) || (rc = up(light_flat, &lf)) || (rc = up(ocdf, &oc)) || (rc = up(lcdf, &lc)) ||
      (rc = up(mats, &mt))) {
    for (void* p : S->allocs) (void)hipFree(p);
    return rc;
  }
  D.stat = DevBvh{sn, stt, (int)stat.size()};
  D.obj = DevBvh{on, ot, (int)obj.size()};
  D.obj_tris = of;
  D.obj_cdf = oc;
  D.nobj = (int)obj.size();
  D.light_tris = lf;
  D.light_cdf = lc;
  D.nlights = (int)la.size();
  D.mats = mt;
  D.nmats = d->num_materials;
  D.inv_obj_area = (float)(1.0 / otot);
  D.inv_light_area = la.empty() ? 0.0f : (float)(1.0 / ltot);
  D.p_env = has_env ? (la.empty() ? 1.0f : 0.5f) : 0.0f;
  D.env = has_env ? v3(d->env[0], d->env[1], d->env[2]) : v3(0, 0, 0);
  DevCamera& C = D.cam;
  C.eye = v3(cam[0], cam[1], cam[2]);
  C.fwd = unit(v3(cam[3], cam[4], cam[5]) - C.eye);
  C.right = unit(cross(C.fwd, v3(cam[6], cam[7], cam[8])));
  C.up = cross(C.right, C.fwd);
  C.W = (int)cam[10];
  C.H = (int)cam[11];
  C.aspect = (float)C.W / (float)C.H;
  C.tan_half = std::tan(cam[9] * 0.5f * 3.14159265358979323846f / 180.0f);
  C.a_film = (float)(4.0 * (double)C.aspect * (double)C.tan_half * (double)C.tan_half);
  if (!(std::fabs(dot(C.right, C.right) - 1.0f) < 1e-3f)) return fail(RPI_ERR_INVALID_ARG, "camera up parallel to view");
  D.eps = (float)(1e-4 * diag);
  S->W = C.W;
  S->H = C.H;
  *out = S.release();
  return RPI_OK;
}

extern "C" rpi_status rpi_destroy_scene(rpi_scene* s) {
  if (!s) return RPI_OK;
  for (void* p : s->allocs) (void)hipFree(p);
  delete s;
  return RPI_OK;
}

static rpi_status check_rigid(const float* m) {
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(m[i])) return fail(RPI_ERR_INVALID_ARG, "non-finite transform");
  double R[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = m[4 * i + j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += R[i][k] * R[j][k];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-4) return fail(RPI_ERR_INVALID_ARG, "transform is not orthonormal");
    }
  const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                     R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
  if (!(det > 0)) return fail(RPI_ERR_INVALID_ARG, "transform is mirrored (det <= 0)");
  return RPI_OK;
}

extern "C" rpi_status rpi_apply_edit(rpi_scene* s, const rpi_edit_desc* d, rpi_edit** out) {
  if (!s || !d || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<rpi_edit> e(new rpi_edit());
  e->kind = d->kind;
  std::memcpy(e->pose_old, kIdentity, sizeof kIdentity);
  if (d->kind == RPI_EDIT_RIGID) {
    rpi_status rc = check_rigid(d->old_to_new);
    if (rc) return rc;
    std::memcpy(e->pose_new, d->old_to_new, sizeof e->pose_new);
    e->new_mat = s->obj_mat;
  } else if (d->kind == RPI_EDIT_MATERIAL) {
    std::memcpy(e->pose_new, kIdentity, sizeof kIdentity);
    const float* m = d->new_material;
    const int t = (int)m[0];
    if (t == MAT_EMITTER) return fail(RPI_ERR_UNSUPPORTED, "emissive new material");
    if (!(t == MAT_DIFFUSE || t == MAT_GGX) || (float)t != m[0]) return fail(RPI_ERR_INVALID_ARG, "bad material type");
    if (t == MAT_GGX && !(m[4] > 0.0f && m[4] <= 1.0f)) return fail(RPI_ERR_INVALID_ARG, "GGX roughness must be in (0, 1]");
    e->new_mat = mat_of(m);
  } else {
    return fail(RPI_ERR_INVALID_ARG, "unknown edit kind");
  }
  *out = e.release();
  return RPI_OK;
}

extern "C" rpi_status rpi_destroy_edit(rpi_edit* e) {
  delete e;
  return RPI_OK;
}

// ------------------------------------------------------------------ rendering
static void world_box(const rpi_scene* s, const Pose& P, vec3& lo, vec3& hi, float pad) {
  lo = v3(INFINITY, INFINITY, INFINITY);
  hi = v3(-INFINITY, -INFINITY, -INFINITY);
  for (int c = 0; c < 8; ++c) {
    const vec3 p = pose_apply(P, v3((c & 1) ? s->obj_hi[0] : s->obj_lo[0], (c & 2) ? s->obj_hi[1] : s->obj_lo[1],
                                    (c & 4) ? s->obj_hi[2] : s->obj_lo[2]));
    lo = v3(std::min(lo.x, p.x), std::min(lo.y, p.y), std::min(lo.z, p.z));
    hi = v3(std::max(hi.x, p.x), std::max(hi.y, p.y), std::max(hi.z, p.z));
  }
  lo = lo - v3(pad, pad, pad);
  hi = hi + v3(pad, pad, pad);
}

static DevFrame make_frame(const rpi_scene* s, const float* pose, const float* ghost, const Material& m, bool ghosts) {
  DevFrame F;
  std::memset(&F, 0, sizeof F);
  F.pose = pose_of(pose);
  F.ghost = pose_of(ghost);
  F.objmat = m;
  const float pad = 1e-3f * s->diag;
  world_box(s, F.pose, F.olo, F.ohi, pad);
  world_box(s, F.ghost, F.glo, F.ghi, pad);
  F.ghosts = ghosts ? 1 : 0;
  F.same_pose = std::memcmp(pose, ghost, 12 * sizeof(float)) == 0 ? 1 : 0;
  return F;
}

static rpi_status check_params(const rpi_scene* s, const rpi_render_params* p) {
  if (!p) return fail(RPI_ERR_INVALID_ARG, "null params");
  if (p->spp <= 0) return fail(RPI_ERR_INVALID_ARG, "spp must be positive");
  if (p->max_depth < 2 || p->max_depth > 7) return fail(RPI_ERR_INVALID_ARG, "max_depth must be in [2, 7]");
  if (p->strategy_mask == 0 || (p->strategy_mask & ~0x7Fu)) return fail(RPI_ERR_INVALID_ARG, "strategy_mask must be a non-empty subset of bits 0..6");
  if (!(p->jac_max > 1.0f) || !(p->alpha_min >= 0.0f) || !(p->c_weight > 0.0f && p->c_weight < 1.0f))
    return fail(RPI_ERR_INVALID_ARG, "bad rejection / weight parameters");
  const int64_t N = (int64_t)p->spp * s->W * s->H;
  const int64_t e = p->sample_end < 0 ? N : p->sample_end;
  if (p->sample_begin < 0 || e > N || p->sample_begin > e) return fail(RPI_ERR_INVALID_ARG, "bad sample range");
  if (N > 0xffffffffLL) return fail(RPI_ERR_UNSUPPORTED, "more than 2^32 samples per technique stream");
  return RPI_OK;
}

namespace {
// Per-call device workspace from the stream-ordered allocator.
struct Ws {
  void* mem = nullptr;
  Workspace W{};
  DevStats* stats = nullptr;
  uint32_t *tcount, *toff, *hist;
  float4* binned;
  size_t bytes = 0;
};

int max_pairs_per_sample(int tech, int d) {
  switch (tech) {
    case 1:
    case 4: return d - 1;
    case 2: return std::max(d - 2, 0);
    case 5: return d - 1;
    case 7: return d;
    case 3: {
      int c = 0;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) c += (i + j + 4 <= d);
      return c;
    }
    default: {
      int c = 0;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) c += (i + j + 3 <= d);
      return c;
    }
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kSplatBlocks = 256;

rpi_status ws_alloc(Ws& w, int Q, int depth, int64_t pair_cap, int ntiles, bool keep, hipStream_t st) {
  const int nslot = depth;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align_up(b);
    return o;
  };
  const size_t o_eye = take((size_t)nslot * kEyeFields * Q * sizeof(float4));
  const size_t o_light = take((size_t)nslot * kLightFields * Q * sizeof(float4));
  const size_t o_start = take((size_t)kStartFields * Q * sizeof(float4));
  const size_t o_counts = take((size_t)Q * 4);
  const size_t o_pairs = take((size_t)pair_cap * 4);
  const size_t o_np = take(256);
  const size_t o_rec = take((size_t)pair_cap * sizeof(float4));
  const size_t o_keys = keep ? take((size_t)pair_cap * 4) : 0;
  const size_t o_ks = keep ? take((size_t)pair_cap * 4) : 0;
  const size_t o_stats = take(sizeof(DevStats));
  const size_t o_tc = take((size_t)ntiles * 4);
  const size_t o_to = take((size_t)(ntiles + 1) * 4);
  const size_t o_tu = take((size_t)ntiles * kSplatBlocks * 4);
  const size_t o_bin = take((size_t)pair_cap * sizeof(float4));
  w.bytes = off;
  HIP_OK(hipMallocAsync(&w.mem, off, st));
  char* b = (char*)w.mem;
  w.W.eye = (float4*)(b + o_eye);
  w.W.light = (float4*)(b + o_light);
  w.W.start = (float4*)(b + o_start);
  w.W.counts = (uint32_t*)(b + o_counts);
  w.W.pairs = (uint32_t*)(b + o_pairs);
  w.W.npairs = (uint32_t*)(b + o_np);
  w.W.records = (float4*)(b + o_rec);
  w.W.rec_keys = keep ? (uint32_t*)(b + o_keys) : nullptr;
  w.W.rec_sample = keep ? (uint32_t*)(b + o_ks) : nullptr;
  w.W.Q = Q;
  w.W.pair_cap = pair_cap;
  w.W.nslot = nslot;
  w.stats = (DevStats*)(b + o_stats);
  w.tcount = (uint32_t*)(b + o_tc);
  w.toff = (uint32_t*)(b + o_to);
  w.hist = (uint32_t*)(b + o_tu);
  w.binned = (float4*)(b + o_bin);
  return RPI_OK;
}
}  // namespace

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// The residual of one job into `out`, given both frames' poses and materials.
static rpi_status residual_job(const rpi_scene* s, const float* pose_old, const float* pose_new, const Material& mat_old,
                               const Material& mat_new, bool material_mode, const rpi_render_params* p, uint32_t job,
                               float* out, rpi_stats* stats, hipStream_t st, std::vector<uint32_t>* rec_out) {
  const int W = s->W, H = s->H, P = W * H;
  const int64_t N = (int64_t)p->spp * P;
  const int64_t s0 = p->sample_begin, s1 = p->sample_end < 0 ? N : p->sample_end;
  const bool keep = (p->flags & RPI_FLAG_RECORDS) != 0;
  const bool cw = (p->flags & RPI_FLAG_COUNT_WORK) != 0;
  const bool time_k = stats != nullptr && (p->flags & RPI_FLAG_TIME_KERNELS) != 0;
  const bool want_stats = stats != nullptr || cw;
  struct Timed {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Timed> evs;
  auto timed = [&](int kid, auto&& launch) -> rpi_status {
    if (!time_k) {
      launch();
      return RPI_OK;
    }
    Timed t{kid, nullptr, nullptr};
    HIP_OK(hipEventCreate(&t.a));
    HIP_OK(hipEventCreate(&t.b));
    HIP_OK(hipEventRecord(t.a, st));
    launch();
    HIP_OK(hipEventRecord(t.b, st));
    evs.push_back(t);
    return RPI_OK;
  };
  int Q = p->queue_cap > 0 ? p->queue_cap : (1 << 20);
  Q = (int)std::min<int64_t>(Q, std::max<int64_t>(s1 - s0, 1));
  Q = std::min(Q, 1 << 24);
  const int d = p->max_depth;
  const int tilesx = (W + 15) / 16, ntiles = tilesx * ((H + 15) / 16);
  if (ntiles > 16384) return fail(RPI_ERR_UNSUPPORTED, "image larger than 2048x2048");
  int maxp = 0;
  for (int t = 1; t <= 7; ++t) maxp = std::max(maxp, max_pairs_per_sample(t, d) + (t == 7 ? 1 : 0));
  const int64_t pair_cap = (int64_t)Q * maxp;
  Ws w;
  rpi_status rc = ws_alloc(w, Q, d, pair_cap, ntiles, keep, st);
  if (rc) return rc;
  if (!(p->flags & RPI_FLAG_ACCUMULATE)) launch_zero_f32(out, (int64_t)P * 3, st);
  if (want_stats) launch_zero_u32((uint32_t*)w.stats, sizeof(DevStats) / 4, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, st));
  }
  const bool two_way = !material_mode && (p->flags & RPI_FLAG_TWO_WAY);
  const Material m2 = material_mode ? mat_new : mat_old;
  DevFrame F2 = make_frame(s, pose_new, pose_old, m2, !material_mode);
  DevFrame F1 = make_frame(s, pose_old, pose_new, mat_old, !material_mode);
  WalkArgs A;
  std::memset(&A, 0, sizeof A);
  A.S = s->dev;
  A.W = w.W;
  A.stats = want_stats ? w.stats : nullptr;
  A.k0 = (uint32_t)p->seed;
  A.k1 = (uint32_t)(p->seed >> 32);
  A.job = job;
  A.depth = d;
  A.material_mode = material_mode ? 1 : 0;
  A.mask = p->strategy_mask;
  A.cweight = material_mode ? 1.0f : p->c_weight;
  A.inv_n = (float)(1.0 / (double)N);
  A.alpha_min = p->alpha_min;
  A.d_min = p->d_min < 0 ? (float)(0.01 * (double)s->diag) : p->d_min;
  A.jac_max = p->jac_max;
  A.count_work = cw ? 1 : 0;
  A.keep_records = keep ? 1 : 0;
  SplatArgs sa;
  sa.records = w.W.records;
  sa.nrec = w.W.npairs;
  sa.cap = pair_cap;
  sa.tcount = w.tcount;
  sa.toff = w.toff;
  sa.hist = w.hist;
  sa.nblk = kSplatBlocks;
  sa.binned = w.binned;
  sa.image = out;
  sa.W = W;
  sa.H = H;
  sa.tilesx = tilesx;
  sa.ntiles = ntiles;
  const int cblocks = device_cus() * 16;
  const int ndir = two_way ? 2 : 1;
  for (int dir = 0; dir < ndir; ++dir) {
    A.F = dir == 0 ? F2 : F1;
    A.Fp = dir == 0 ? F1 : F2;
    A.dir = dir;
    A.sigma = dir == 0 ? 1.0f : -1.0f;
    for (int t = 1; t <= 7; ++t) {
      if (!((p->strategy_mask >> (t - 1)) & 1u)) continue;
      if (material_mode && t >= 4 && t <= 6) continue;
      A.tech = t;
      for (int64_t c0 = s0; c0 < s1; c0 += Q) {
        A.sample0 = c0;
        A.nsamples = (int)std::min<int64_t>(Q, s1 - c0);
        launch_zero_u32(w.W.npairs, 1, st);
        rpi_status r1 = timed(t, [&] { launch_walk(A, st); });
        if (r1) return r1;
        r1 = timed(8, [&] { launch_connect(A, cblocks, st); });
        if (r1) return r1;
        r1 = timed(9, [&] { launch_splat(sa, st); });
        if (r1) return r1;
        if (keep && rec_out) {
          // host copies of this chunk's records (debug path; synchronous)
          uint32_t n = 0;
          HIP_OK(hipMemcpyAsync(&n, w.W.npairs, 4, hipMemcpyDeviceToHost, st));
          HIP_OK(hipStreamSynchronize(st));
          n = (uint32_t)std::min<int64_t>(n, pair_cap);
          std::vector<float4> rec(n);
          std::vector<uint32_t> keys(n), smp(n);
          if (n) {
            HIP_OK(hipMemcpy(rec.data(), w.W.records, n * sizeof(float4), hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(keys.data(), w.W.rec_keys, n * 4, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(smp.data(), w.W.rec_sample, n * 4, hipMemcpyDeviceToHost));
          }
          for (uint32_t r = 0; r < n; ++r) {
            uint32_t o[8];
            o[0] = keys[r] & 1u;
            o[1] = (keys[r] >> 1) & 127u;
            o[2] = smp[r];
            o[3] = (keys[r] >> 8) & 0xffu;
            std::memcpy(&o[4], &rec[r], 16);
            rec_out->insert(rec_out->end(), o, o + 8);
          }
        }
      }
    }
  }
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  if (stats || cw) {
    DevStats ds;
    if (stats) HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipMemcpyAsync(&ds, w.stats, sizeof ds, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (stats) {
      std::memset(stats, 0, sizeof *stats);
      stats->paths = (int64_t)ds.paths;
      stats->accepted = (int64_t)ds.accepted;
      for (int r = 0; r < 7; ++r) stats->rejected[r] = (int64_t)ds.rejected[r];
      for (int t = 0; t < 9; ++t) stats->by_tech[t] = (int64_t)ds.by_tech[t];
      stats->nodes_visited = (int64_t)ds.nodes;
      stats->tris_tested = (int64_t)ds.tris;
      for (int q = 0; q < 6; ++q) stats->rays[q] = (int64_t)ds.rays[q];
      for (int q = 0; q < 16; ++q) {
        stats->kernel_nodes[q] = (int64_t)ds.knodes[q];
        stats->kernel_tris[q] = (int64_t)ds.ktris[q];
        stats->kernel_bytes_written[q] = (int64_t)ds.kbytes[q];
      }
      for (const Timed& t : evs) {
        float kms = 0;
        HIP_OK(hipEventElapsedTime(&kms, t.a, t.b));
        stats->kernel_ms[t.kid] += kms;
        stats->kernel_launches[t.kid] += 1;
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
      }
      stats->samples = (s1 - s0) * ndir * __builtin_popcount(p->strategy_mask & (material_mode ? 0x47u : 0x7Fu));
      float ms = 0;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      stats->milliseconds = ms;
      hipEventDestroy(e0);
      hipEventDestroy(e1);
    }
  }
  HIP_OK(hipFreeAsync(w.mem, st));
  return RPI_OK;
}

extern "C" rpi_status rpi_render_residual(const rpi_scene* s, const rpi_edit* e, const rpi_render_params* p, float* out,
                                          rpi_stats* stats, void* stream) {
  if (!s || !e || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_status rc = check_params(s, p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const bool mm = e->kind == RPI_EDIT_MATERIAL;
  std::vector<uint32_t> recs;
  rc = residual_job(s, e->pose_old, e->pose_new, s->obj_mat, e->new_mat, mm, p, p->job, out, stats, st,
                    (p->flags & RPI_FLAG_RECORDS) ? &recs : nullptr);
  if (rc) return rc;
  if (p->flags & RPI_FLAG_RECORDS) {
    std::lock_guard<std::mutex> lk(const_cast<rpi_scene*>(s)->mu);
    const_cast<rpi_scene*>(s)->rec_host.swap(recs);
  }
  return RPI_OK;
}

extern "C" rpi_status rpi_get_records(const rpi_scene* s, void* host_out, int64_t cap, int64_t* count) {
  if (!s || !count) return fail(RPI_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(const_cast<rpi_scene*>(s)->mu);
  const int64_t n = (int64_t)s->rec_host.size() / 8;
  *count = n;
  if (host_out) std::memcpy(host_out, s->rec_host.data(), (size_t)std::min(n, cap) * 32);
  return RPI_OK;
}

extern "C" rpi_status rpi_render_frame(const rpi_scene* s, const rpi_edit* e, int32_t which, const rpi_render_params* p,
                                       float* out, void* stream) {
  if (!s || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (which != 1 && which != 2) return fail(RPI_ERR_INVALID_ARG, "which must be 1 (old) or 2 (new)");
  if (!p || p->spp <= 0 || p->max_depth < 2 || p->max_depth > 7) return fail(RPI_ERR_INVALID_ARG, "bad params");
  const int64_t N = (int64_t)p->spp * s->W * s->H;
  FrameArgs A;
  std::memset(&A, 0, sizeof A);
  A.S = s->dev;
  const float* pose = (e && which == 2) ? e->pose_new : kIdentity;
  const Material m = (e && which == 2) ? e->new_mat : s->obj_mat;
  A.F = make_frame(s, pose, pose, m, false);
  A.image = out;
  A.k0 = (uint32_t)p->seed;
  A.k1 = (uint32_t)(p->seed >> 32);
  A.job = p->job;
  A.dir = which == 2 ? 0 : 1;
  A.depth = p->max_depth;
  A.spp = p->spp;
  A.accumulate = (p->flags & RPI_FLAG_ACCUMULATE) ? 1 : 0;
  A.s0 = p->sample_begin;
  A.s1 = p->sample_end < 0 ? N : p->sample_end;
  launch_frame(A, (hipStream_t)stream);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

extern "C" rpi_status rpi_render_residual_batch(const rpi_scene* s, const rpi_job* jobs, int32_t n,
                                                const rpi_render_params* p, rpi_stats* stats, void* stream) {
  if (!s || !jobs || n <= 0) return fail(RPI_ERR_INVALID_ARG, "null argument");
  (void)p;
  (void)stats;
  (void)stream;
  return fail(RPI_ERR_UNSUPPORTED, "batch path not built yet");
}
