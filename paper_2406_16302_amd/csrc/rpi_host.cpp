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
#include <atomic>
#include <thread>
#include <random>
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
  std::vector<float4> nodes;  // binary while building, 4-wide after collapse4
  std::vector<float4> tris;
  int max_depth = 0;
  int max_stack = 0;          // traversal stack entries a ray can need (4-wide)
};

constexpr int kLeafMax = 2;  // leaves of 2 triangles traced faster than 1, 3, 4 or 8 (measured)
constexpr int kBins = 16;
constexpr int kMedianDepth = 24;  // from this depth on splits are object medians (bounded stack use)

// Binned SAH (16 bins per axis) with object-median splits from depth 24 on.
// The binary tree it builds keeps both children's boxes and links in their
// parent (4 float4: c0.lo.xyz, c0.hi.xyz, c1.lo.xyz, c1.hi.xyz, then the two
// links); collapse4 turns it into the device's 4-wide nodes.
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
    // Object medians halve a node's triangles per level, so starting them at
    // depth D leaves every leaf within D + ceil(log2(n / kLeafMax)) levels:
    // D is chosen to keep that under the traversal stack depth.
    int halvings = 0;
    while (((int64_t)kLeafMax << halvings) < (int64_t)n) ++halvings;
    median_depth_ = std::max(1, std::min(kMedianDepth, kStackDepth - 2 - halvings));
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
    if (depth < median_depth_) {
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
  int median_depth_ = kMedianDepth;
};

// Collapse the binary BVH into 4-wide nodes (kNodeF4 float4 per node: the
// children's lo.x, hi.x, lo.y, hi.y, lo.z, hi.z planes, then their links;
// unused slots hold kEmptyLink).  A 4-wide visit tests up to four boxes
// with one dependent fetch, and the traversal of a ray takes about half as
// many dependent steps.  A node visit pushes up to (children - 1) entries,
// so wider nodes need more stack: each binary subtree v gets a budget b(v)
// of entries, a node widens (replacing its largest-area inner child by that
// child's two children) only while every resulting child c keeps
// h(c) <= b - (children - 1), where h is the binary height (the entries a
// binary traversal below c can push), and its children inherit
// b - (children - 1).  With b(root) = kStackDepth - 1 >= h(root) (the binary
// builder's guarantee) no path can push more than kStackDepth - 1 entries.
bool collapse4(BuiltBvh& bvh, std::string& err) {
  const std::vector<float4>& in = bvh.nodes;
  const int n2 = (int)in.size() / 4;
  struct Child {
    float lo[3], hi[3];
    int32_t link;
  };
  auto child = [&](int node, int slot) {
    const float* f = reinterpret_cast<const float*>(&in[4 * (size_t)node]);
    const int32_t* iv = reinterpret_cast<const int32_t*>(&in[4 * (size_t)node + 3]);
    Child c;
    for (int a = 0; a < 3; ++a) {
      c.lo[a] = f[6 * slot + a];
      c.hi[a] = f[6 * slot + 3 + a];
    }
    c.link = iv[slot];
    return c;
  };
  // binary heights, children after their parent in the array
  std::vector<int> h(n2, 0);
  for (int i = n2 - 1; i >= 0; --i) {
    int m = 0;
    for (int slot = 0; slot < 2; ++slot) {
      const int32_t l = child(i, slot).link;
      if (l >= 0) {
        if (l <= i || l >= n2) {
          err = "binary BVH link out of order";
          return false;
        }
        m = std::max(m, h[l]);
      }
    }
    h[i] = 1 + m;
  }
  auto hc = [&](const Child& c) { return c.link >= 0 ? h[c.link] : 0; };
  auto area = [](const Child& c) {
    const float dx = c.hi[0] - c.lo[0], dy = c.hi[1] - c.lo[1], dz = c.hi[2] - c.lo[2];
    return dx * dy + dy * dz + dz * dx;
  };
  const int root_budget = kStackDepth - 1;
  if (h[0] > root_budget) {
    err = "BVH deeper than the traversal stack";
    return false;
  }
  std::vector<float4> out;
  struct Job {
    int bin, budget, wide, depth;  // binary node, its budget, its 4-wide node, stack entries above it
  };
  std::vector<Job> st;
  out.resize(kNodeF4);
  st.push_back({0, root_budget, 0, 0});
  int max_stack = 0;
  while (!st.empty()) {
    const Job j = st.back();
    st.pop_back();
    std::vector<Child> C = {child(j.bin, 0), child(j.bin, 1)};
    while (C.size() < 4) {
      int best = -1;
      float best_area = -1.0f;
      for (int k = 0; k < (int)C.size(); ++k) {
        if (C[k].link < 0) continue;
        // children after expanding C[k]: all must fit the budget left to them
        const int cost = (int)C.size();  // (size + 1) children -> size entries
        bool ok = true;
        for (int q = 0; q < (int)C.size() && ok; ++q)
          if (q != k) ok = hc(C[q]) <= j.budget - cost;
        for (int slot = 0; slot < 2 && ok; ++slot) ok = hc(child(C[k].link, slot)) <= j.budget - cost;
        if (ok && area(C[k]) > best_area) {
          best_area = area(C[k]);
          best = k;
        }
      }
      if (best < 0) break;
      const int b = C[best].link;
      C[best] = child(b, 0);
      C.push_back(child(b, 1));
    }
    const int pushes = (int)C.size() - 1;
    max_stack = std::max(max_stack, j.depth + pushes);
    float* f = reinterpret_cast<float*>(&out[(size_t)kNodeF4 * j.wide]);
    int32_t* links = reinterpret_cast<int32_t*>(&out[(size_t)kNodeF4 * j.wide + 6]);
    for (int k = 0; k < 4; ++k) {
      if (k < (int)C.size()) {
        for (int a = 0; a < 3; ++a) {
          f[8 * a + k] = C[k].lo[a];
          f[8 * a + 4 + k] = C[k].hi[a];
        }
        if (C[k].link < 0) {
          links[k] = C[k].link;
        } else {
          const int w = (int)(out.size() / kNodeF4);
          out.resize(out.size() + kNodeF4);
          f = reinterpret_cast<float*>(&out[(size_t)kNodeF4 * j.wide]);  // the resize moved the array
          links = reinterpret_cast<int32_t*>(&out[(size_t)kNodeF4 * j.wide + 6]);
          links[k] = w;
          st.push_back({C[k].link, j.budget - pushes, w, j.depth + pushes});
        }
      } else {
        for (int a = 0; a < 3; ++a) {
          f[8 * a + k] = 0.0f;
          f[8 * a + 4 + k] = 0.0f;
        }
        links[k] = kEmptyLink;
      }
    }
    float* pad = reinterpret_cast<float*>(&out[(size_t)kNodeF4 * j.wide + 7]);
    for (int k = 0; k < 4; ++k) pad[k] = 0.0f;
  }
  if (max_stack > kStackDepth) {
    err = "4-wide BVH exceeds the traversal stack";
    return false;
  }
  // every link inside the arrays
  const int n4 = (int)(out.size() / kNodeF4);
  const int ntri = (int)(bvh.tris.size() / 3);
  for (int i = 0; i < n4; ++i) {
    const int32_t* links = reinterpret_cast<const int32_t*>(&out[(size_t)kNodeF4 * i + 6]);
    for (int k = 0; k < 4; ++k) {
      const int32_t l = links[k];
      if (l >= 0 ? (l <= i || l >= n4)
                 : (int)(((uint32_t)l & 0x7fffffffu) >> 4) + (int)(l & 15) > ntri) {
        err = "4-wide BVH link out of range";
        return false;
      }
    }
  }
  bvh.nodes.swap(out);
  bvh.max_stack = max_stack;
  return true;
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
struct BatchCache;
static void destroy_batch_cache(BatchCache* c);

struct rpi_scene {
  DevScene dev;
  // device-memory hook (rpi_build_scene); without one: hipMalloc / hipMallocAsync
  rpi_allocator al{};
  bool has_al = false;
  // autotuned launch configuration (0 = not tuned)
  int tuned_Q = 0, tuned_walk = 0, tuned_conn = 0;
  BatchCache* batch = nullptr;
  std::vector<void*> allocs;
  float obj_lo[3], obj_hi[3];  // object bounds in object space (= old pose)
  float obj_sc[3], obj_sr;     // bounding sphere in object space: centre, radius
  // A closed convex object: its outward face planes in object space (n, d:
  // n.x - d > 0 outside), the emitter triangles (world) and whether it is sealed
  bool obj_sealed = false;
  std::vector<std::array<double, 4>> obj_planes;
  std::vector<std::array<float, 9>> light_host;
  Material obj_mat;
  float diag;
  float lmax = 1.0f;  // largest emission of the scene (emitters, environment): the fixed-point splat's scale
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

struct rpi_proposal {
  MlpBufs B{};
  void* mem = nullptr;
  vec3 center, inv_half;  // input normalisation: the object's bounding box in object space
  int steps = 0;          // Adam steps taken
  MlpDev view() const { return mlp_view(B, center, inv_half); }
};

// The library's own stream-ordered pool per device.  It keeps the memory
// handed back (release threshold: unlimited) so that the per-call workspace
// (tens of GB at the large rounds) is not unmapped and mapped again at every
// synchronisation, as the default pool would do; rpi_destroy_scene trims it.
static std::mutex g_pool_mu;
static hipMemPool_t g_pool[64];
static bool g_pool_tried[64];

static hipMemPool_t lib_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (!g_pool_tried[dev]) {
    g_pool_tried[dev] = true;
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
      uint64_t keep = ~(uint64_t)0;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      g_pool[dev] = pool;
    }
  }
  return g_pool[dev];
}

// Device memory of a scene and of the calls on it: through the caller's hook
// when one was given, else from the library's pool on the stream (async; the
// default pool if the library's could not be made) or hipMalloc.
static rpi_status dev_alloc(const rpi_scene* s, size_t bytes, hipStream_t st, bool async, void** out) {
  *out = nullptr;
  if (bytes == 0) return RPI_OK;
  if (s->has_al) {
    *out = s->al.allocate(s->al.ctx, bytes, (void*)st);
    if (!*out) return fail(RPI_ERR_OUT_OF_MEMORY, "the allocator hook returned no memory for " + std::to_string(bytes) + " bytes");
    return RPI_OK;
  }
  hipMemPool_t pool = async ? lib_pool() : nullptr;
  hipError_t e = async ? (pool ? hipMallocFromPoolAsync(out, bytes, pool, st) : hipMallocAsync(out, bytes, st))
                       : hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(e == hipErrorOutOfMemory ? RPI_ERR_OUT_OF_MEMORY : RPI_ERR_DEVICE,
                std::string("device allocation of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  }
  return RPI_OK;
}
static void dev_free(const rpi_scene* s, void* p, hipStream_t st, bool async) {
  if (!p) return;
  if (s->has_al) s->al.deallocate(s->al.ctx, p, (void*)st);
  else if (async) (void)hipFreeAsync(p, st);
  else (void)hipFree(p);
}

// Guide table of a CDF (the cutpoint method of Chen and Asau 1974): with
// M = 2^bits (the power of two >= n, at most 2^22), g[j] is the first index
// whose CDF value exceeds j / M (j = 0..M; j / M is exact in float).  The
// first index above any u in [j / M, (j + 1) / M) lies in [g[j], g[j + 1]],
// so a search over that range returns what a search over the whole CDF
// returns.
static void cdf_guide(const std::vector<float>& cdf, std::vector<int32_t>& g, int& bits) {
  const int n = (int)cdf.size();
  bits = 0;
  while ((1 << bits) < n && bits < 22) ++bits;
  const int M = 1 << bits;
  g.assign(M + 1, 0);
  int i = 0;
  for (int j = 0; j <= M; ++j) {
    const float x = (float)j / (float)M;
    while (i < n && cdf[i] <= x) ++i;
    g[j] = i;
  }
}

template <class T>
static rpi_status upload(const rpi_scene* s, const std::vector<T>& v, T** out) {
  *out = nullptr;
  if (v.empty()) return RPI_OK;
  void* p = nullptr;
  rpi_status rc = dev_alloc(s, v.size() * sizeof(T), nullptr, false, &p);
  if (rc) return rc;
  *out = (T*)p;
  HIP_OK(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return RPI_OK;
}

static bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

// Whether the object's triangles bound a convex solid: every vertex lies on
// the inner side (the side of the vertex mean c) of every face plane, within
// tol.  A face whose plane passes through c (within tol) makes it non-convex.
// Rays leaving a convex object through its surface cannot meet it again,
// which lets the kernels skip its BVH for them.  O(faces x vertices), on
// host threads.
static bool object_convex(const std::vector<HostTri>& obj, double tol, vec3& center,
                          std::vector<std::array<double, 4>>* planes, bool* closed) {
  std::vector<std::array<float, 3>> v;
  v.reserve(3 * obj.size());
  for (const auto& t : obj)
    for (const float* p : {t.v0, t.v1, t.v2}) v.push_back({p[0], p[1], p[2]});
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  // closed: with vertices welded by position, every edge borders exactly two triangles
  {
    auto id = [&](const float* p) {
      const std::array<float, 3> k{p[0], p[1], p[2]};
      return (int64_t)(std::lower_bound(v.begin(), v.end(), k) - v.begin());
    };
    std::vector<int64_t> edges;
    edges.reserve(3 * obj.size());
    for (const auto& t : obj) {
      const int64_t a = id(t.v0), b = id(t.v1), c = id(t.v2);
      for (auto e : {std::make_pair(a, b), std::make_pair(b, c), std::make_pair(c, a)})
        edges.push_back(std::min(e.first, e.second) * (int64_t)v.size() + std::max(e.first, e.second));
    }
    std::sort(edges.begin(), edges.end());
    bool ok = true;
    for (size_t i = 0; i < edges.size() && ok;) {
      size_t j = i;
      while (j < edges.size() && edges[j] == edges[i]) ++j;
      ok = j - i == 2;
      i = j;
    }
    *closed = ok;
  }
  double c[3] = {0, 0, 0};
  for (const auto& p : v)
    for (int a = 0; a < 3; ++a) c[a] += p[a];
  for (int a = 0; a < 3; ++a) c[a] /= (double)v.size();
  center = v3((float)c[0], (float)c[1], (float)c[2]);
  const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<bool> ok{true};
  planes->assign(obj.size(), {0, 0, 0, 0});
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      for (size_t f = w; f < obj.size() && ok.load(std::memory_order_relaxed); f += nt) {
        const HostTri& t = obj[f];
        double e1[3], e2[3], n[3];
        for (int a = 0; a < 3; ++a) {
          e1[a] = (double)t.v1[a] - t.v0[a];
          e2[a] = (double)t.v2[a] - t.v0[a];
        }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0)) {
          ok = false;
          return;
        }
        const double d = (n[0] * t.v0[0] + n[1] * t.v0[1] + n[2] * t.v0[2]) / len;
        const double sc = (n[0] * c[0] + n[1] * c[1] + n[2] * c[2]) / len - d;
        if (!(std::fabs(sc) > tol)) {
          ok = false;
          return;
        }
        const double s = sc > 0 ? 1.0 : -1.0;
        // outward plane: n.x - d > 0 on the side away from the centre
        (*planes)[f] = {-s * n[0] / len, -s * n[1] / len, -s * n[2] / len, -s * d};
        for (const auto& p : v)
          if (s * ((n[0] * p[0] + n[1] * p[1] + n[2] * p[2]) / len - d) < -tol) {
            ok = false;
            return;
          }
      }
    });
  for (auto& x : th) x.join();
  return ok.load();
}

extern "C" const char* rpi_last_error(void) { return g_err.c_str(); }
extern "C" const char* rpi_version(void) { return "rpi 0.2 (gfx950)"; }

extern "C" rpi_status rpi_sync_status(void* stream) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(e));
  return RPI_OK;
}

extern "C" rpi_status rpi_build_scene(const rpi_scene_desc* d, const rpi_allocator* al, rpi_scene** out) {
  if (!d || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (al && (!al->allocate || !al->deallocate)) return fail(RPI_ERR_INVALID_ARG, "allocator hook without functions");
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
    if (d->tri_object[f] < 0) return fail(RPI_ERR_INVALID_ARG, "negative tri_object in triangle " + std::to_string(f));
    if (d->tri_object[f] > 1)  // every dynamic triangle moves with the one pose pair of an edit
      return fail(RPI_ERR_UNSUPPORTED, "several independently moving objects (tri_object > 1)");
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
    if (!b.build(bs, err) || !collapse4(bs, err)) return fail(RPI_ERR_UNSUPPORTED, "static BVH: " + err);
  }
  {
    Builder b(obj);
    if (!b.build(bo, err) || !collapse4(bo, err)) return fail(RPI_ERR_UNSUPPORTED, "object BVH: " + err);
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
  // bounding sphere: centre of the bounds, radius to the farthest vertex (double)
  {
    double r2 = 0;
    for (int a = 0; a < 3; ++a) S->obj_sc[a] = 0.5f * (S->obj_lo[a] + S->obj_hi[a]);
    for (const auto& t : obj)
      for (const float* p : {t.v0, t.v1, t.v2}) {
        double q = 0;
        for (int a = 0; a < 3; ++a) q += ((double)p[a] - S->obj_sc[a]) * ((double)p[a] - S->obj_sc[a]);
        r2 = std::max(r2, q);
      }
    S->obj_sr = (float)(std::sqrt(r2) * (1.0 + 1e-6));
  }
  S->obj_mat = mat_of(d->materials + 8 * obj[0].mat);
  for (const auto& t : obj)
    if (t.mat != obj[0].mat) return fail(RPI_ERR_UNSUPPORTED, "the dynamic object must use a single material");

  DevScene& D = S->dev;
  std::memset(&D, 0, sizeof D);
  std::vector<float> mats(d->materials, d->materials + 8 * d->num_materials);
  rpi_status rc;
  if (al) {
    S->al = *al;
    S->has_al = true;
  }
  auto up = [&](auto& v, auto** p) -> rpi_status {
    rpi_status r = upload(S.get(), v, p);
    if (*p) S->allocs.push_back((void*)*p);
    return r;
  };
  std::vector<int32_t> ogd, lgd;
  int ogb, lgb;
  cdf_guide(ocdf, ogd, ogb);
  cdf_guide(lcdf, lgd, lgb);
  float4 *sn, *stt, *on, *ot, *of, *lf;
  float *oc, *lc, *mt;
  int32_t *og, *lg;
  if ((rc = up(bs.nodes, &sn)) || (rc = up(bs.tris, &stt)) || (rc = up(bo.nodes, &on)) || (rc = up(bo.tris, &ot)) ||
      (rc = up(obj_flat, &of)) || (rc = up(light_flat, &lf)) || (rc = up(ocdf, &oc)) || (rc = up(lcdf, &lc)) ||
      (rc = up(mats, &mt)) || (rc = up(ogd, &og)) || (rc = up(lgd, &lg))) {
    for (void* p : S->allocs) dev_free(S.get(), p, nullptr, false);
    return rc;
  }
  D.stat = DevBvh{sn, stt, (int)stat.size()};
  D.obj = DevBvh{on, ot, (int)obj.size()};
  D.obj_tris = of;
  D.obj_cdf = oc;
  D.nobj = (int)obj.size();
  D.obj_guide = og;
  D.obj_gbits = ogb;
  D.light_tris = lf;
  D.light_cdf = lc;
  D.nlights = (int)la.size();
  D.light_guide = lg;
  D.light_gbits = lgb;
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
  bool closed = false;
  D.obj_convex = object_convex(obj, 1e-6 * diag, D.obj_center, &S->obj_planes, &closed) ? 1 : 0;
  S->obj_sealed = D.obj_convex && closed;
  if (!S->obj_sealed) S->obj_planes.clear();
  D.obj_rin = 0.0f;
  if (S->obj_sealed) {  // the nearest face plane bounds a ball about the centre inside the object
    double rin = INFINITY;
    for (const auto& pl : S->obj_planes)
      rin = std::min(rin, pl[3] - (pl[0] * D.obj_center.x + pl[1] * D.obj_center.y + pl[2] * D.obj_center.z));
    D.obj_rin = rin > 0 ? (float)(0.999 * rin) : 0.0f;
  }
  S->light_host.clear();
  for (size_t i = 0; i < light_flat.size(); i += 3) {
    const float4 a = light_flat[i], e1 = light_flat[i + 1], e2 = light_flat[i + 2];
    S->light_host.push_back({a.x, a.y, a.z, a.x + e1.x, a.y + e1.y, a.z + e1.z, a.x + e2.x, a.y + e2.y, a.z + e2.z});
  }
  S->W = C.W;
  S->H = C.H;
  {
    double lm = 0.0;
    for (int m = 0; m < d->num_materials; ++m)
      if ((int)d->materials[8 * m] == MAT_EMITTER)
        for (int c = 0; c < 3; ++c) lm = std::max(lm, (double)std::fabs(d->materials[8 * m + 5 + c]));
    if (has_env)
      for (int c = 0; c < 3; ++c) lm = std::max(lm, (double)std::fabs(d->env[c]));
    S->lmax = lm > 0.0 && std::isfinite(lm) ? (float)lm : 1.0f;
  }
  *out = S.release();
  return RPI_OK;
}

extern "C" rpi_status rpi_destroy_scene(rpi_scene* s) {
  if (!s) return RPI_OK;
  destroy_batch_cache(s->batch);
  s->batch = nullptr;
  (void)hipDeviceSynchronize();  // no call on the scene may still be running
  for (void* p : s->allocs) dev_free(s, p, nullptr, false);
  if (!s->has_al)
    if (hipMemPool_t pool = lib_pool()) (void)hipMemPoolTrimTo(pool, 0);  // hand the pooled workspace back
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
  if (!d || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  // the description is checked first, on its own (no device work, no scene state)
  if (d->kind == RPI_EDIT_RIGID) {
    rpi_status rc = check_rigid(d->old_to_new);
    if (rc) return rc;
  } else if (d->kind == RPI_EDIT_MATERIAL) {
    const float* m = d->new_material;
    const int t = (int)m[0];
    if (t == MAT_EMITTER) return fail(RPI_ERR_UNSUPPORTED, "emissive new material");
    if (!(t == MAT_DIFFUSE || t == MAT_GGX) || (float)t != m[0]) return fail(RPI_ERR_INVALID_ARG, "bad material type");
    if (t == MAT_GGX && !(m[4] > 0.0f && m[4] <= 1.0f)) return fail(RPI_ERR_INVALID_ARG, "GGX roughness must be in (0, 1]");
    for (int i = 1; i < 8; ++i)
      if (!std::isfinite(m[i])) return fail(RPI_ERR_INVALID_ARG, "non-finite material parameter");
  } else {
    return fail(RPI_ERR_INVALID_ARG, "unknown edit kind");
  }
  if (!s) return fail(RPI_ERR_INVALID_ARG, "null scene");
  std::unique_ptr<rpi_edit> e(new rpi_edit());
  e->kind = d->kind;
  std::memcpy(e->pose_old, kIdentity, sizeof kIdentity);
  if (d->kind == RPI_EDIT_RIGID) {
    std::memcpy(e->pose_new, d->old_to_new, sizeof e->pose_new);
    e->new_mat = s->obj_mat;
  } else {
    std::memcpy(e->pose_new, kIdentity, sizeof kIdentity);
    e->new_mat = mat_of(d->new_material);
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
  const vec3 sc = v3(s->obj_sc[0], s->obj_sc[1], s->obj_sc[2]);
  F.oc = pose_apply(F.pose, sc);
  F.gc = pose_apply(F.ghost, sc);
  F.orad = s->obj_sr + pad;
  F.ghosts = ghosts ? 1 : 0;
  F.same_pose = std::memcmp(pose, ghost, 12 * sizeof(float)) == 0 ? 1 : 0;
  // Sealed: the object is closed and convex and, at this pose, the camera and
  // every emitter lie outside it (a face plane separates each of them).  Then
  // no path that reaches the object's inside can leave it again to connect.
  if (s->obj_sealed) {
    const double tol = 1e-5 * s->diag;
    auto separated = [&](const float* pts, int n) {
      vec3 q[3];
      for (int i = 0; i < n; ++i) q[i] = pose_inv_apply(F.pose, v3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]));
      for (const auto& pl : s->obj_planes) {
        bool all = true;
        for (int i = 0; i < n && all; ++i) all = pl[0] * q[i].x + pl[1] * q[i].y + pl[2] * q[i].z - pl[3] > tol;
        if (all) return true;
      }
      return false;
    };
    const float eye[3] = {s->dev.cam.eye.x, s->dev.cam.eye.y, s->dev.cam.eye.z};
    bool ok = separated(eye, 1);
    for (size_t i = 0; ok && i < s->light_host.size(); ++i) ok = separated(s->light_host[i].data(), 3);
    F.sealed = ok ? 1 : 0;
  }
  return F;
}

// Flags that apply to motion edits only.
static rpi_status check_edit_flags(const rpi_edit* e, const rpi_render_params* p) {
  if (e->kind != RPI_EDIT_MATERIAL) return RPI_OK;
  if (p->flags & RPI_FLAG_NO_MAPPING) return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_NO_MAPPING applies to motion edits only");
  if (p->flags & RPI_FLAG_BALANCE) return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_BALANCE applies to motion edits only");
  return RPI_OK;
}

static rpi_status check_params(const rpi_scene* s, const rpi_render_params* p) {
  if (!p) return fail(RPI_ERR_INVALID_ARG, "null params");
  if (p->spp <= 0) return fail(RPI_ERR_INVALID_ARG, "spp must be positive");
  if (p->max_depth < 2 || p->max_depth > 7) return fail(RPI_ERR_INVALID_ARG, "max_depth must be in [2, 7]");
  if (p->strategy_mask == 0 || (p->strategy_mask & ~0xFFu)) return fail(RPI_ERR_INVALID_ARG, "strategy_mask must be a non-empty subset of bits 0..7");
  if ((p->strategy_mask & 0x80u) && !p->proposal) return fail(RPI_ERR_INVALID_ARG, "technique 8 needs a proposal");
  if (p->d_train_records && p->train_capacity < 0) return fail(RPI_ERR_INVALID_ARG, "negative train_capacity");
  if (p->train_weighting != 0 && p->train_weighting != 1) return fail(RPI_ERR_INVALID_ARG, "train_weighting must be 0 or 1");
  if (p->tile != 0 && p->tile != 16 && p->tile != 32) return fail(RPI_ERR_INVALID_ARG, "tile must be 0, 16 or 32");
  if ((p->flags & RPI_FLAG_PER_TECHNIQUE) && !p->d_technique_images)
    return fail(RPI_ERR_INVALID_ARG, "RPI_FLAG_PER_TECHNIQUE needs d_technique_images");
  if ((p->flags & RPI_FLAG_NO_MAPPING) && !(p->flags & RPI_FLAG_TWO_WAY))
    return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_NO_MAPPING needs RPI_FLAG_TWO_WAY (a motion edit sampled in both frames)");
  if ((p->flags & RPI_FLAG_BALANCE) && !(p->flags & RPI_FLAG_TWO_WAY))
    return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_BALANCE needs RPI_FLAG_TWO_WAY (a motion edit sampled in both frames)");
  if ((p->flags & RPI_FLAG_BALANCE) && (p->strategy_mask & 0x80u))
    return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_BALANCE does not combine with technique 8");
  bool uneq = false;
  for (int t = 0; t < kTechs; ++t) {
    if (p->technique_spp[t] < 0) return fail(RPI_ERR_INVALID_ARG, "negative technique_spp");
    if ((int64_t)p->technique_spp[t] * s->W * s->H > 0xffffffffLL)
      return fail(RPI_ERR_UNSUPPORTED, "more than 2^32 samples per technique stream");
    uneq |= p->technique_spp[t] > 0;
  }
  if (uneq && (p->sample_begin != 0 || p->sample_end >= 0))
    return fail(RPI_ERR_INVALID_ARG, "technique_spp needs the full sample range");
  if (!(p->jac_max > 1.0f) || !(p->alpha_min >= 0.0f) || !(p->c_weight > 0.0f && p->c_weight < 1.0f))
    return fail(RPI_ERR_INVALID_ARG, "bad rejection / weight parameters");
  const int64_t N = (int64_t)p->spp * s->W * s->H;
  const int64_t e = p->sample_end < 0 ? N : p->sample_end;
  if (p->sample_begin < 0 || e > N || p->sample_begin > e) return fail(RPI_ERR_INVALID_ARG, "bad sample range");
  if (N > 0xffffffffLL) return fail(RPI_ERR_UNSUPPORTED, "more than 2^32 samples per technique stream");
  if ((int64_t)s->W * s->H >= (1 << 24)) return fail(RPI_ERR_UNSUPPORTED, "image of 2^24 pixels or more");
  return RPI_OK;
}

namespace {
int max_pairs_per_sample(int tech, int d) {
  switch (tech) {
    case 1:
    case 4: return d - 1;
    case 2: return std::max(d - 2, 0);
    case 5: return d - 1;
    case 7: return d + 1;
    case 3:
    case 8: {
      int c = tech == 8 ? std::max(d - 2, 0) : 0;  // technique 8: the camera sees x_D
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
constexpr int kMaxTiles = 16384;   // one LDS histogram of kMaxTiles words per splat workgroup

// One residual job as the host plans it.
struct JobSpec {
  float pose_old[12], pose_new[12];
  Material mat_old, mat_new;
  int W, H;
  float* out;
  float* tech = nullptr;  // RPI_FLAG_PER_TECHNIQUE: 8 images of W x H x 3
};

// Launch configuration (chosen by the autotuner or defaults).
struct Tuning {
  int Q = 1 << 20;      // samples per round
  int walk_bpc = 16;    // persistent walk workgroups per compute unit
  int conn_bpc = 16;    // connect workgroups per compute unit
};

// Device workspace for rounds of Q samples over a batch of jobs.
struct Ws {
  void* mem = nullptr;
  const rpi_scene* owner = nullptr;  // whose allocator holds mem
  bool async = true;
  Workspace W{};
  DevStats* stats = nullptr;
  uint32_t *tcount, *toff, *cpre, *hist, *item_counter, *train_count;
  float4* binned;
  DevJob* jobs;
  int64_t* prefix;  // [kTechs][2 * njobs + 1]
  int32_t* tile_job;
  unsigned long long* acc;  // fixed-point images of the jobs
  size_t bytes = 0;
};

// Byte offsets of the workspace parts for rounds of Q samples.
struct WsLayout {
  size_t eye, light, start, counts, pairs, pairs2, np, rec, keys, ks, t8, stats, tc, to, cp, hist, bin, jobs, pre, tj,
      ic, tc2, task, nt, acc, order, okey, bytes;
};

static WsLayout ws_layout(int Q, int depth, int64_t pair_cap, int ntiles, int njobs, bool keep, bool t8,
                          int64_t acc_elems) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align_up(b);
    return o;
  };
  const int nslot = depth;
  L.eye = take((size_t)nslot * kEyeFields * Q * sizeof(float4));
  L.light = take((size_t)nslot * kLightFields * Q * sizeof(float4));
  L.start = take((size_t)kStartFields * Q * sizeof(float4));
  L.counts = take((size_t)Q * 4);
  L.pairs = take((size_t)pair_cap * 4);
  L.pairs2 = take((size_t)pair_cap * 4);
  L.np = take(256);
  L.rec = take((size_t)pair_cap * sizeof(float4));
  L.keys = keep ? take((size_t)pair_cap * 4) : 0;
  L.ks = keep ? take((size_t)pair_cap * 4) : 0;
  L.t8 = t8 ? take((size_t)pair_cap * 2 * sizeof(float4)) : 0;
  L.stats = take(sizeof(DevStats));
  L.tc = take((size_t)ntiles * 4);
  L.to = take((size_t)(ntiles + 1) * 4);
  L.cp = take((size_t)(ntiles + 1) * 4);
  L.hist = take((size_t)ntiles * kSplatBlocks * 4);
  L.bin = take((size_t)pair_cap * sizeof(float4));
  L.jobs = take((size_t)njobs * sizeof(DevJob));
  L.pre = take((size_t)kTechs * (2 * njobs + 1) * sizeof(int64_t));
  L.tj = take((size_t)ntiles * 4);
  L.ic = take(256);
  L.tc2 = take(256);
  L.task = take((size_t)kTaskFields * Q * sizeof(float4));
  L.nt = take(256);
  L.acc = take((size_t)acc_elems * 8);
  L.order = take((size_t)Q * 4);
  L.okey = take((size_t)Q * 2);
  L.bytes = off;
  return L;
}

// Point the workspace views into `mem` (L.bytes bytes of device memory).
static void ws_bind(Ws& w, const WsLayout& L, void* mem, int Q, int depth, int64_t pair_cap, bool keep, bool t8) {
  w.mem = mem;
  w.bytes = L.bytes;
  char* b = (char*)mem;
  w.W.eye = (float4*)(b + L.eye);
  w.W.light = (float4*)(b + L.light);
  w.W.start = (float4*)(b + L.start);
  w.W.counts = (uint32_t*)(b + L.counts);
  w.W.pairs = (uint32_t*)(b + L.pairs);
  w.W.pairs2 = (uint32_t*)(b + L.pairs2);
  w.W.order = (uint32_t*)(b + L.order);
  w.W.okey = (uint16_t*)(b + L.okey);
  w.W.npairs = (uint32_t*)(b + L.np);
  w.W.records = (float4*)(b + L.rec);
  w.W.rec_keys = keep ? (uint32_t*)(b + L.keys) : nullptr;
  w.W.rec_sample = keep ? (uint32_t*)(b + L.ks) : nullptr;
  w.W.t8q = t8 ? (float4*)(b + L.t8) : nullptr;
  w.W.task = (float4*)(b + L.task);
  w.W.ntasks = (uint32_t*)(b + L.nt);
  w.W.fetch = w.W.ntasks + 16;
  w.W.kbins = w.W.ntasks + 32;
  w.W.Q = Q;
  w.W.pair_cap = pair_cap;
  w.W.nslot = depth;
  w.stats = (DevStats*)(b + L.stats);
  w.tcount = (uint32_t*)(b + L.tc);
  w.toff = (uint32_t*)(b + L.to);
  w.cpre = (uint32_t*)(b + L.cp);
  w.hist = (uint32_t*)(b + L.hist);
  w.binned = (float4*)(b + L.bin);
  w.jobs = (DevJob*)(b + L.jobs);
  w.prefix = (int64_t*)(b + L.pre);
  w.tile_job = (int32_t*)(b + L.tj);
  w.item_counter = (uint32_t*)(b + L.ic);
  w.train_count = (uint32_t*)(b + L.tc2);
  w.acc = (unsigned long long*)(b + L.acc);
}


rpi_status ws_alloc(const rpi_scene* s, Ws& w, int Q, int depth, int64_t pair_cap, int ntiles, int njobs, bool keep,
                    bool t8, int64_t acc_elems, hipStream_t st, bool async) {
  const WsLayout L = ws_layout(Q, depth, pair_cap, ntiles, njobs, keep, t8, acc_elems);
  w.async = async;
  w.owner = s;
  void* mem = nullptr;
  rpi_status rc = dev_alloc(s, L.bytes, st, async, &mem);
  if (rc) return rc;
  ws_bind(w, L, mem, Q, depth, pair_cap, keep, t8);
  return RPI_OK;
}

void ws_free(Ws& w, hipStream_t st) {
  if (!w.mem) return;
  dev_free(w.owner, w.mem, st, w.async);
  w.mem = nullptr;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// Host-side plan of a batch: job table, item prefix tables, tile map.
struct Plan {
  std::vector<DevJob> jobs;
  std::vector<int64_t> prefix;  // [kTechs][2 * njobs + 1]
  std::vector<int32_t> tile_job;
  int ntiles = 0;
  int ts = 16;  // splat tile edge
  int64_t pair_cap = 0;
  int Q = 0;
  bool material_mode = false;
  std::vector<int64_t> acc_off;  // per job: first element of its fixed-point image
  int64_t acc_elems = 0;
  vec3 obj_center, obj_inv_half;  // training-record input normalisation
};

// Point every job of the plan at its part of the workspace's fixed-point image.
static void bind_jobs(Plan& pl, const Ws& w) {
  for (size_t j = 0; j < pl.jobs.size(); ++j) pl.jobs[j].acc = w.acc + pl.acc_off[j];
}

}  // namespace

static DevScene job_scene_impl(const DevScene& base, int W, int H) {
  DevScene S = base;
  S.cam.W = W;
  S.cam.H = H;
  S.cam.aspect = (float)W / (float)H;
  S.cam.a_film = (float)(4.0 * (double)S.cam.aspect * (double)S.cam.tan_half * (double)S.cam.tan_half);
  return S;
}

// Proposal input normalisation: centre and inverse half-extent of the
// object's bounding box in object space.
static void object_normalisation(const rpi_scene* s, vec3& center, vec3& inv_half) {
  center = v3(0.5f * (s->obj_lo[0] + s->obj_hi[0]), 0.5f * (s->obj_lo[1] + s->obj_hi[1]),
              0.5f * (s->obj_lo[2] + s->obj_hi[2]));
  inv_half = v3(2.0f / std::max(s->obj_hi[0] - s->obj_lo[0], 1e-6f), 2.0f / std::max(s->obj_hi[1] - s->obj_lo[1], 1e-6f),
                2.0f / std::max(s->obj_hi[2] - s->obj_lo[2], 1e-6f));
}

static rpi_status make_plan(const rpi_scene* s, const std::vector<JobSpec>& js, bool material_mode,
                            const rpi_render_params* p, const Tuning& tu, Plan& pl) {
  const int nj = (int)js.size();
  pl.material_mode = material_mode;
  object_normalisation(s, pl.obj_center, pl.obj_inv_half);
  pl.jobs.resize(nj);
  pl.ntiles = 0;
  pl.tile_job.clear();
  pl.acc_off.assign(nj, 0);
  pl.acc_elems = 0;
  for (int j = 0; j < nj; ++j) {
    pl.acc_off[j] = pl.acc_elems;
    pl.acc_elems += (int64_t)js[j].W * js[j].H * 3;
  }
  // 16x16 tiles unless the batch needs more than kMaxTiles of them (or the
  // caller asks for a tile edge)
  int64_t t16 = 0;
  for (const JobSpec& q : js) t16 += (int64_t)((q.W + 15) / 16) * ((q.H + 15) / 16);
  pl.ts = p->tile ? p->tile : (t16 <= kMaxTiles ? 16 : 32);
  const int kTileSize = pl.ts;
  for (int j = 0; j < nj; ++j) {
    const JobSpec& q = js[j];
    DevJob& J = pl.jobs[j];
    std::memset(&J, 0, sizeof J);
    J.S = job_scene_impl(s->dev, q.W, q.H);
    J.F[0] = make_frame(s, q.pose_new, q.pose_old, material_mode ? q.mat_new : q.mat_old, !material_mode);
    J.F[1] = make_frame(s, q.pose_old, q.pose_new, q.mat_old, !material_mode);
    J.image = q.out;
    J.tech_images = q.tech;
    J.fx_scale = (float)(1099511627776.0 / (double)s->lmax);  // 2^40 / largest emission
    J.fx_unit = (double)s->lmax / 1099511627776.0;
    for (int t = 0; t < kTechs; ++t)
      J.tech_ratio[t] = p->technique_spp[t] > 0 ? (float)((double)p->technique_spp[t] / (double)p->spp) : 1.0f;
    const int64_t N = (int64_t)p->spp * q.W * q.H;
    if (N > 0xffffffffLL) return fail(RPI_ERR_UNSUPPORTED, "more than 2^32 samples per technique stream");
    J.s0 = p->sample_begin;
    J.s1 = p->sample_end < 0 ? N : std::min<int64_t>(p->sample_end, N);
    if (J.s0 < 0 || J.s0 > J.s1) return fail(RPI_ERR_INVALID_ARG, "bad sample range");
    J.inv_n = (float)(1.0 / (double)N);
    J.W = q.W;
    J.H = q.H;
    J.tilesx = (q.W + kTileSize - 1) / kTileSize;
    J.tile0 = pl.ntiles;
    const int nt = J.tilesx * ((q.H + kTileSize - 1) / kTileSize);
    for (int t = 0; t < nt; ++t) pl.tile_job.push_back(j);
    pl.ntiles += nt;
  }
  if (pl.ntiles > kMaxTiles)
    return fail(RPI_ERR_UNSUPPORTED, "images exceed 16384 tiles of " + std::to_string(kTileSize) + "x" +
                                         std::to_string(kTileSize) + " pixels");
  const bool two_way = !material_mode && (p->flags & RPI_FLAG_TWO_WAY);
  pl.prefix.assign((size_t)kTechs * (2 * nj + 1), 0);
  for (int t = 1; t <= kTechs; ++t) {
    int64_t* pre = pl.prefix.data() + (size_t)(t - 1) * (2 * nj + 1);
    const bool on = ((p->strategy_mask >> (t - 1)) & 1u) && !(material_mode && t >= 4 && t <= 6) &&
                    (t != 8 || p->proposal);
    int64_t run = 0;
    for (int j = 0; j < nj; ++j)
      for (int d = 0; d < 2; ++d) {
        pre[2 * j + d] = run;
        const int64_t n = p->technique_spp[t - 1] > 0 ? (int64_t)p->technique_spp[t - 1] * js[j].W * js[j].H
                                                       : pl.jobs[j].s1 - pl.jobs[j].s0;
        if (on && (d == 0 || two_way)) run += (n + kItem - 1) / kItem;
      }
    pre[2 * nj] = run;
  }
  int maxp = 0;
  for (int t = 1; t <= kTechs; ++t) maxp = std::max(maxp, max_pairs_per_sample(t, p->max_depth));
  int64_t total = 0;
  for (int j = 0; j < nj; ++j) {
    total = std::max(total, pl.jobs[j].s1 - pl.jobs[j].s0);
    for (int t = 0; t < kTechs; ++t) total = std::max(total, (int64_t)p->technique_spp[t] * js[j].W * js[j].H);
  }
  int64_t Q = std::min<int64_t>(tu.Q, std::max<int64_t>(total * nj * 2, kItem));
  Q = (Q + kItem - 1) / kItem * kItem;
  Q = std::min<int64_t>(Q, kMaxRound);
  pl.Q = (int)Q;
  pl.pair_cap = Q * maxp;
  return RPI_OK;
}

// Enqueue the launch sequence of a planned batch on `st` (graph-capturable:
// kernels only).  Records/timing hooks only on the direct path.
struct RunOpts {
  bool count_work = false, keep = false, time_k = false, accumulate = false, stats = false;
  Tuning tu;
};

struct Timed {
  int kid;
  int tech;  // the technique whose round launched it
  hipEvent_t a, b;
};

static rpi_status enqueue(const Plan& pl, const Ws& w, const rpi_render_params* p, const RunOpts& o, hipStream_t st,
                          std::vector<Timed>* evs, std::vector<uint32_t>* rec_out) {
  const int nj = (int)pl.jobs.size();
  const bool per_tech = (p->flags & RPI_FLAG_PER_TECHNIQUE) != 0;
  launch_zero_images(w.jobs, nj, st);  // the fixed-point images (and technique images)
  WalkArgs A;
  std::memset(&A, 0, sizeof A);
  A.jobs = w.jobs;
  A.njobs = nj;
  A.item_counter = w.item_counter;
  A.W = w.W;
  A.stats = (o.count_work || o.stats) ? w.stats : nullptr;
  A.k0 = (uint32_t)p->seed;
  A.k1 = (uint32_t)(p->seed >> 32);
  A.job_base = p->job;
  A.depth = p->max_depth;
  A.material_mode = pl.material_mode ? 1 : 0;
  A.mask = p->strategy_mask;
  A.cweight = pl.material_mode ? 1.0f : p->c_weight;
  A.alpha_min = p->alpha_min;
  A.d_min = p->d_min;
  A.jac_max = p->jac_max;
  A.no_mapping = (p->flags & RPI_FLAG_NO_MAPPING) ? 1 : 0;
  A.balance = (p->flags & RPI_FLAG_BALANCE) ? 1 : 0;
  A.tech_spp = 0;
  A.count_work = o.count_work ? 1 : 0;
  A.keep_records = o.keep ? 1 : 0;
  const bool t8 = (p->strategy_mask & 0x80u) && p->proposal;
  if (p->proposal) A.mlp = p->proposal->view();
  if (p->d_train_records) {
    if (!p->proposal) {
      // the records carry the proposal's input: normalise by the object's bounds
      // even without a proposal attached
      MlpDev M;
      std::memset(&M, 0, sizeof M);
      M.center = pl.obj_center;
      M.inv_half = pl.obj_inv_half;
      A.mlp = M;
    }
    A.train = p->d_train_records;
    A.train_cap = p->train_capacity;
    A.train_count = w.train_count;
    A.train_weighting = p->train_weighting;
  }
  SplatArgs sa;
  std::memset(&sa, 0, sizeof sa);
  sa.records = w.W.records;
  sa.nrec = w.W.npairs;
  sa.cap = pl.pair_cap;
  sa.jobs = w.jobs;
  sa.tile_job = w.tile_job;
  sa.hist = w.hist;
  sa.tcount = w.tcount;
  sa.toff = w.toff;
  sa.cpre = w.cpre;
  sa.binned = w.binned;
  sa.ntiles = pl.ntiles;
  sa.nblk = kSplatBlocks;
  sa.ts = pl.ts;
  const int wblocks = device_cus() * o.tu.walk_bpc;
  const int cblocks = device_cus() * o.tu.conn_bpc;
  const int R = pl.Q / kItem;
  auto timed = [&](int kid, auto&& launch) -> rpi_status {
    if (!evs) {
      launch();
      return RPI_OK;
    }
    Timed t{kid, A.tech, nullptr, nullptr};
    HIP_OK(hipEventCreate(&t.a));
    HIP_OK(hipEventCreate(&t.b));
    HIP_OK(hipEventRecord(t.a, st));
    launch();
    HIP_OK(hipEventRecord(t.b, st));
    evs->push_back(t);
    return RPI_OK;
  };
  for (int t = 1; t <= kTechs; ++t) {
    const int64_t* pre_h = pl.prefix.data() + (size_t)(t - 1) * (2 * nj + 1);
    const int64_t T = pre_h[2 * nj];
    if (T == 0) continue;
    A.tech = t;
    A.tech_spp = p->technique_spp[t - 1];
    A.item_prefix = w.prefix + (size_t)(t - 1) * (2 * nj + 1);
    for (int64_t i0 = 0; i0 < T; i0 += R) {
      A.item0 = i0;
      A.nitems = (int)std::min<int64_t>(R, T - i0);
      launch_zero_u32(w.W.npairs, 1, st);
      launch_zero_u32(w.item_counter, 1, st);
      launch_zero_u32(w.W.ntasks, 64, st);  // the task count, the fetch counters, the length bins
      const int blocks = std::min<int64_t>(wblocks, A.nitems);
      rpi_status r;
      // samples ordered by where they start (on the object or the ghost;
      // path tracing: pixel tiles)
      A.W.order = w.W.order;
      r = timed(kKidStartOrder, [&] { launch_start_order(A, st); });
      if (r) return r;
      if (t == 8) {
        r = timed(kKidT8Start, [&] { launch_t8_start(A, std::min<int64_t>(cblocks, A.nitems), st); });
        if (r) return r;
      }
      r = timed(kid_start(t), [&] { launch_walk(A, blocks, st); });
      if (r) return r;
      if (split_walks(t)) {
        r = timed(kid_walk(t), [&] { launch_walk_tasks(A, blocks, st); });
        if (r) return r;
      }
      // the path queue sorted by path length, so that a wave's paths loop over
      // the same number of vertices, then within windows by pixel tile (back
      // into W.pairs), so that a wave's mapping rays start close together
      launch_sort_pairs(A, st);
      WalkArgs As = A;
      As.W.pairs = w.W.pairs;  // the queue ordered by path length, then by pixel tile within windows
      if (t8) {
        r = timed(kKidProposalPdf, [&] { launch_proposal_pdf(As, cblocks, st); });
        if (r) return r;
      }
      r = timed(kKidConnect, [&] { launch_connect(As, cblocks, st); });
      if (r) return r;
      r = timed(kKidSplat, [&] { launch_splat(sa, st); });
      if (r) return r;
      if (o.keep && rec_out) {
        uint32_t n = 0;
        HIP_OK(hipMemcpyAsync(&n, w.W.npairs, 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        n = (uint32_t)std::min<int64_t>(n, pl.pair_cap);
        std::vector<float4> rec(n);
        std::vector<uint32_t> keys(n), smp(n);
        if (n) {
          HIP_OK(hipMemcpy(rec.data(), w.W.records, n * sizeof(float4), hipMemcpyDeviceToHost));
          HIP_OK(hipMemcpy(keys.data(), w.W.rec_keys, n * 4, hipMemcpyDeviceToHost));
          HIP_OK(hipMemcpy(smp.data(), w.W.rec_sample, n * 4, hipMemcpyDeviceToHost));
        }
        for (uint32_t r2 = 0; r2 < n; ++r2) {
          uint32_t q[8];
          q[0] = keys[r2] & 1u;
          q[1] = (keys[r2] >> 1) & 127u;
          q[2] = smp[r2];
          q[3] = (keys[r2] >> 8) & 0xffu;
          float4 rr = rec[r2];
          int code = 0;
          std::memcpy(&code, &rr.x, 4);
          const int pix = code < 0 ? -1 : (code & 0xffffff);
          std::memcpy(&rr.x, &pix, 4);
          std::memcpy(&q[4], &rr, 16);
          rec_out->insert(rec_out->end(), q, q + 8);
        }
      }
    }
    // this technique's share into its own image
    if (per_tech) launch_flush_acc(w.jobs, nj, t, false, st);
  }
  // the total of the technique images, added in technique order
  if (per_tech) launch_sum_technique_images(w.jobs, nj, o.accumulate, st);
  else launch_flush_acc(w.jobs, nj, 0, o.accumulate, st);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

static rpi_status upload_plan(const Plan& pl, const Ws& w, hipStream_t st) {
  HIP_OK(hipMemcpyAsync(w.jobs, pl.jobs.data(), pl.jobs.size() * sizeof(DevJob), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(w.prefix, pl.prefix.data(), pl.prefix.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(w.tile_job, pl.tile_job.data(), pl.tile_job.size() * 4, hipMemcpyHostToDevice, st));
  // the host vectors are pageable: make the copies complete before they can go away
  HIP_OK(hipStreamSynchronize(st));
  return RPI_OK;
}

static void fill_stats(rpi_stats* stats, const DevStats& ds, const Plan& pl, const rpi_render_params* p) {
  std::memset(stats, 0, sizeof *stats);
  stats->paths = (int64_t)ds.paths;
  stats->accepted = (int64_t)ds.accepted;
  for (int r = 0; r < 7; ++r) stats->rejected[r] = (int64_t)ds.rejected[r];
  for (int t = 0; t < 9; ++t) stats->by_tech[t] = (int64_t)ds.by_tech[t];
  stats->nodes_visited = (int64_t)ds.nodes;
  stats->tris_tested = (int64_t)ds.tris;
  for (int q = 0; q < 6; ++q) stats->rays[q] = (int64_t)ds.rays[q];
  for (int q = 0; q < kKernelSlots; ++q) {
    stats->kernel_nodes[q] = (int64_t)ds.knodes[q];
    stats->kernel_tris[q] = (int64_t)ds.ktris[q];
    stats->kernel_bytes_written[q] = (int64_t)ds.kbytes[q];
  }
  const int nj = (int)pl.jobs.size();
  for (int t = 1; t <= kTechs; ++t) {
    const int64_t* pre = pl.prefix.data() + (size_t)(t - 1) * (2 * nj + 1);
    for (int j = 0; j < nj; ++j)
      for (int d = 0; d < 2; ++d)
        if (pre[2 * j + d + 1] > pre[2 * j + d])
          stats->samples += p->technique_spp[t - 1] > 0
                                ? (int64_t)p->technique_spp[t - 1] * pl.jobs[j].W * pl.jobs[j].H
                                : pl.jobs[j].s1 - pl.jobs[j].s0;
  }
}

// Direct (non-graph) execution of a batch of jobs with optional statistics.
static rpi_status run_jobs(const rpi_scene* s, const std::vector<JobSpec>& js, bool material_mode,
                           const rpi_render_params* p, const Tuning& tu, rpi_stats* stats, hipStream_t st,
                           std::vector<uint32_t>* rec_out) {
  Plan pl;
  rpi_status rc = make_plan(s, js, material_mode, p, tu, pl);
  if (rc) return rc;
  RunOpts o;
  o.count_work = (p->flags & RPI_FLAG_COUNT_WORK) != 0;
  o.keep = (p->flags & RPI_FLAG_RECORDS) != 0;
  o.time_k = stats != nullptr && (p->flags & RPI_FLAG_TIME_KERNELS) != 0;
  o.accumulate = (p->flags & RPI_FLAG_ACCUMULATE) != 0;
  o.stats = stats != nullptr;
  o.tu = tu;
  Ws w;
  const bool t8 = (p->strategy_mask & 0x80u) && p->proposal;
  rc = ws_alloc(s, w, pl.Q, p->max_depth, pl.pair_cap, pl.ntiles, (int)pl.jobs.size(), o.keep, t8, pl.acc_elems, st,
                true);
  if (rc) return rc;
  bind_jobs(pl, w);
  rc = upload_plan(pl, w, st);
  if (rc) {
    ws_free(w, st);
    return rc;
  }
  const bool want = stats != nullptr || o.count_work;
  if (want) launch_zero_u32((uint32_t*)w.stats, sizeof(DevStats) / 4, st);
  if (p->d_train_records) launch_zero_u32(w.train_count, 1, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, st));
  }
  std::vector<Timed> evs;
  rc = enqueue(pl, w, p, o, st, o.time_k ? &evs : nullptr, rec_out);
  if (rc) {
    ws_free(w, st);
    return rc;
  }
  if (want) {
    DevStats ds;
    uint32_t ntrain = 0;
    if (stats) HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipMemcpyAsync(&ds, w.stats, sizeof ds, hipMemcpyDeviceToHost, st));
    if (p->d_train_records) HIP_OK(hipMemcpyAsync(&ntrain, w.train_count, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (stats) {
      fill_stats(stats, ds, pl, p);
      stats->train_records = ntrain;
      float ms = 0;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      stats->milliseconds = ms;
      for (const Timed& t : evs) {
        float kms = 0;
        HIP_OK(hipEventElapsedTime(&kms, t.a, t.b));
        stats->kernel_ms[t.kid] += kms;
        stats->kernel_launches[t.kid] += 1;
        stats->technique_ms[t.tech] += kms;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
  }
  ws_free(w, st);
  return RPI_OK;
}

static Tuning scene_tuning(const rpi_scene* s, const rpi_render_params* p);

extern "C" rpi_status rpi_render_residual(const rpi_scene* s, const rpi_edit* e, const rpi_render_params* p, float* out,
                                          rpi_stats* stats, void* stream) {
  if (!s || !e || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_status rc = check_params(s, p);
  if (rc) return rc;
  if (p->d_train_records && !stats) return fail(RPI_ERR_INVALID_ARG, "training-record collection needs stats");
  rc = check_edit_flags(e, p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  JobSpec j;
  std::memcpy(j.pose_old, e->pose_old, sizeof j.pose_old);
  std::memcpy(j.pose_new, e->pose_new, sizeof j.pose_new);
  j.mat_old = s->obj_mat;
  j.mat_new = e->new_mat;
  j.W = s->W;
  j.H = s->H;
  j.out = out;
  j.tech = (p->flags & RPI_FLAG_PER_TECHNIQUE) ? p->d_technique_images : nullptr;
  std::vector<uint32_t> recs;
  rpi_render_params q = *p;
  if (q.d_min < 0) q.d_min = (float)(0.01 * (double)s->diag);
  rc = run_jobs(s, {j}, e->kind == RPI_EDIT_MATERIAL, &q, scene_tuning(s, p), stats, st,
                (p->flags & RPI_FLAG_RECORDS) ? &recs : nullptr);
  if (rc) return rc;
  if (p->flags & RPI_FLAG_RECORDS) {
    std::lock_guard<std::mutex> lk(const_cast<rpi_scene*>(s)->mu);
    const_cast<rpi_scene*>(s)->rec_host.swap(recs);
  }
  return RPI_OK;
}

// ------------------------------------------------------------------ residual-aware sample allocation
extern "C" rpi_status rpi_allocate_samples(const rpi_scene* s, const rpi_edit* e, const rpi_render_params* p,
                                           int32_t pilot_spp, int32_t* out, void* stream) {
  if (!s || !e || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_status rc = check_params(s, p);
  if (rc) return rc;
  if (pilot_spp < 2) return fail(RPI_ERR_INVALID_ARG, "pilot_spp must be at least 2");
  if (p->d_train_records) return fail(RPI_ERR_INVALID_ARG, "no training records in an allocation pilot");
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = (int64_t)s->W * s->H;
  const int64_t N = (int64_t)pilot_spp * P;
  if (N > 0xffffffffLL) return fail(RPI_ERR_UNSUPPORTED, "pilot of more than 2^32 samples per stream");
  // two independent halves of the pilot, each with its per-technique images
  void* mem = nullptr;
  const size_t img = (size_t)P * 3;
  rc = dev_alloc(s, (2 * kTechs + 1) * img * sizeof(float), st, true, &mem);
  if (rc) return rc;
  float* ta = (float*)mem;
  float* tb = ta + kTechs * img;
  float* tot = tb + kTechs * img;
  rpi_render_params q = *p;
  q.spp = pilot_spp;
  for (int t = 0; t < kTechs; ++t) q.technique_spp[t] = 0;
  q.flags &= ~(uint32_t)(RPI_FLAG_ACCUMULATE | RPI_FLAG_RECORDS | RPI_FLAG_COUNT_WORK);
  q.flags |= RPI_FLAG_PER_TECHNIQUE | RPI_FLAG_TIME_KERNELS;
  double ms[kTechs + 1] = {0};
  for (int h = 0; h < 2; ++h) {
    q.sample_begin = h ? N / 2 : 0;
    q.sample_end = h ? N : N / 2;
    q.d_technique_images = h ? tb : ta;
    rpi_stats stt;
    rc = rpi_render_residual(s, e, &q, tot, &stt, stream);
    if (rc) {
      dev_free(s, mem, st, true);
      return rc;
    }
    for (int t = 1; t <= kTechs; ++t) ms[t] += stt.technique_ms[t];
  }
  std::vector<float> ha(kTechs * img), hb(kTechs * img);
  hipError_t e1 = hipMemcpyAsync(ha.data(), ta, ha.size() * sizeof(float), hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipMemcpyAsync(hb.data(), tb, hb.size() * sizeof(float), hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  dev_free(s, mem, st, true);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
    return fail(RPI_ERR_DEVICE, "copying the pilot's technique images failed");
  // Var of technique t's share of the pilot ~ sum over pixels of (a_t - b_t)^2;
  // its cost per sample from its launches' device time.  Treating the
  // techniques as strata, the variance with n_t samples is V_t N / n_t at a
  // cost c_t n_t, minimised for a fixed cost by n_t ~ sqrt(V_t / c_t)
  // (Neyman allocation); the total cost is kept at that of equal counts.
  double x[kTechs + 1] = {0}, c[kTechs + 1] = {0};
  double sc = 0.0, scx = 0.0;
  for (int t = 1; t <= kTechs; ++t) {
    if (!(ms[t] > 0.0)) continue;
    double v = 0.0;
    const float* a = ha.data() + (size_t)(t - 1) * img;
    const float* b = hb.data() + (size_t)(t - 1) * img;
    for (size_t i = 0; i < img; ++i) v += ((double)a[i] - b[i]) * ((double)a[i] - b[i]);
    c[t] = ms[t] / (double)N;
    x[t] = std::sqrt(v / c[t]);
    sc += c[t];
    scx += c[t] * x[t];
  }
  for (int t = 1; t <= kTechs; ++t) {
    if (!(c[t] > 0.0)) {
      out[t - 1] = 0;
      continue;
    }
    const double n = scx > 0.0 ? (double)p->spp * P * sc / scx * x[t] : (double)p->spp * P;
    const double spp_t = std::round(n / (double)P);
    out[t - 1] = (int32_t)std::min<double>(std::max<double>(spp_t, 1.0), 64.0 * p->spp);
  }
  return RPI_OK;
}

// ------------------------------------------------------------------ residual denoiser
extern "C" rpi_status rpi_render_gbuffer(const rpi_scene* s, const rpi_edit* e, int32_t which, float* d_gbuf,
                                         void* stream) {
  if (!s || !d_gbuf) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (which != 0 && which != 1) return fail(RPI_ERR_INVALID_ARG, "which must be 0 (old frame) or 1 (new frame)");
  const float* pose = (e && which == 1) ? e->pose_new : kIdentity;
  const Material m = (e && which == 1) ? e->new_mat : s->obj_mat;
  const DevFrame F = make_frame(s, pose, pose, m, false);
  launch_gbuffer(s->dev, F, (float4*)d_gbuf, (hipStream_t)stream);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

extern "C" rpi_status rpi_denoise_residual(const rpi_scene* s, const rpi_edit* e, const float* d_a, const float* d_b,
                                           const rpi_denoise_params* dp, float* d_out, void* stream) {
  if (!s || !e || !d_a || !d_b || !d_out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_denoise_params q{3, 64.0f, 0.1f, 2.0f};
  if (dp) {
    if (dp->iterations) q.iterations = dp->iterations;
    if (dp->sigma_normal > 0) q.sigma_normal = dp->sigma_normal;
    if (dp->sigma_depth > 0) q.sigma_depth = dp->sigma_depth;
    if (dp->sigma_value > 0) q.sigma_value = dp->sigma_value;
    if (dp->iterations < 0 || dp->iterations > 10 || !std::isfinite(dp->sigma_normal) ||
        !std::isfinite(dp->sigma_depth) || !std::isfinite(dp->sigma_value) || dp->sigma_normal < 0 ||
        dp->sigma_depth < 0 || dp->sigma_value < 0)
      return fail(RPI_ERR_INVALID_ARG, "bad denoise parameters");
  }
  hipStream_t st = (hipStream_t)stream;
  const int W = s->W, H = s->H;
  const size_t px = (size_t)W * H;
  void* mem = nullptr;
  rpi_status rc = dev_alloc(s, 3 * px * sizeof(float4), st, true, &mem);
  if (rc) return rc;
  float4* g = (float4*)mem;
  const DevFrame F = make_frame(s, e->pose_new, e->pose_new, e->new_mat, false);
  launch_gbuffer(s->dev, F, g, st);
  launch_denoise(d_a, d_b, g, g + px, g + 2 * px, W, H, q.iterations, q.sigma_normal, q.sigma_depth, q.sigma_value,
                 d_out, st);
  dev_free(s, mem, st, true);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

// ------------------------------------------------------------------ allocation-free variant
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the workspace of rpi_render_residual_noalloc lives in
// one static device array per GPU.  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static rpi_status scratch_address(void** out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RPI_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RPI_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RPI_OK;
}

extern "C" rpi_status rpi_render_residual_noalloc(const rpi_scene* s, const rpi_edit* e, const rpi_render_params* p,
                                                  float* out, void* stream) {
  if (!s || !e || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_status rc = check_params(s, p);
  if (rc) return rc;
  if (p->d_train_records || (p->flags & (RPI_FLAG_RECORDS | RPI_FLAG_COUNT_WORK | RPI_FLAG_TIME_KERNELS)))
    return fail(RPI_ERR_UNSUPPORTED, "records, work counting, kernel timing and training records need "
                                     "rpi_render_residual");
  rc = check_edit_flags(e, p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  JobSpec j;
  std::memcpy(j.pose_old, e->pose_old, sizeof j.pose_old);
  std::memcpy(j.pose_new, e->pose_new, sizeof j.pose_new);
  j.mat_old = s->obj_mat;
  j.mat_new = e->new_mat;
  j.W = s->W;
  j.H = s->H;
  j.out = out;
  j.tech = (p->flags & RPI_FLAG_PER_TECHNIQUE) ? p->d_technique_images : nullptr;
  rpi_render_params q = *p;
  if (q.d_min < 0) q.d_min = (float)(0.01 * (double)s->diag);
  const bool material = e->kind == RPI_EDIT_MATERIAL;
  Plan pl;
  rc = make_plan(s, {j}, material, &q, scene_tuning(s, p), pl);
  if (rc) return rc;
  // the largest round (a multiple of 64 samples, at most the planned one)
  // whose workspace fits the scratch array
  const bool t8 = (q.strategy_mask & 0x80u) && q.proposal;
  const int64_t maxp = pl.pair_cap / pl.Q;
  auto need = [&](int64_t Q) {
    return ws_layout((int)Q, q.max_depth, Q * maxp, pl.ntiles, 1, false, t8, pl.acc_elems).bytes;
  };
  if (need(kItem) > kScratchBytes)
    return fail(RPI_ERR_UNSUPPORTED, "the workspace of this image (" + std::to_string(need(kItem)) +
                                         " bytes for the smallest round) exceeds the " +
                                         std::to_string(kScratchBytes >> 20) + " MiB static scratch array");
  int64_t lo = 1, hi = pl.Q / kItem;  // in items of 64 samples: need(lo) fits
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (need(mid * kItem) <= kScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  pl.Q = (int)(lo * kItem);
  pl.pair_cap = (int64_t)pl.Q * maxp;
  void* ptr = nullptr;
  rc = scratch_address(&ptr);
  if (rc) return rc;
  Ws w;
  w.owner = s;
  ws_bind(w, ws_layout(pl.Q, q.max_depth, pl.pair_cap, pl.ntiles, 1, false, t8, pl.acc_elems), ptr, pl.Q, q.max_depth,
          pl.pair_cap, false, t8);
  bind_jobs(pl, w);
  rc = upload_plan(pl, w, st);
  if (rc) return rc;
  RunOpts o;
  o.accumulate = (q.flags & RPI_FLAG_ACCUMULATE) != 0;
  o.tu = scene_tuning(s, p);
  return enqueue(pl, w, &q, o, st, nullptr, nullptr);
}

extern "C" rpi_status rpi_get_records(const rpi_scene* s, void* host_out, int64_t cap, int64_t* count) {
  if (!s || !count) return fail(RPI_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(const_cast<rpi_scene*>(s)->mu);
  const int64_t n = (int64_t)s->rec_host.size() / 8;
  *count = n;
  if (host_out) std::memcpy(host_out, s->rec_host.data(), (size_t)std::min(n, cap) * 32);
  return RPI_OK;
}

static rpi_status frame_common(const rpi_scene* s, const rpi_render_params* p, float* out, FrameArgs& A) {
  if (!s || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (!p || p->spp <= 0 || p->max_depth < 2 || p->max_depth > 7) return fail(RPI_ERR_INVALID_ARG, "bad params");
  const int64_t N = (int64_t)p->spp * s->W * s->H;
  if (N > 0xffffffffLL) return fail(RPI_ERR_UNSUPPORTED, "more than 2^32 samples per stream");
  const int64_t e = p->sample_end < 0 ? N : p->sample_end;
  if (p->sample_begin < 0 || e > N || p->sample_begin > e) return fail(RPI_ERR_INVALID_ARG, "bad sample range");
  std::memset(&A, 0, sizeof A);
  A.S = s->dev;
  A.image = out;
  A.k0 = (uint32_t)p->seed;
  A.k1 = (uint32_t)(p->seed >> 32);
  A.job = p->job;
  A.depth = p->max_depth;
  A.spp = p->spp;
  A.accumulate = (p->flags & RPI_FLAG_ACCUMULATE) ? 1 : 0;
  A.s0 = p->sample_begin;
  A.s1 = e;
  return RPI_OK;
}

extern "C" rpi_status rpi_render_frame(const rpi_scene* s, const rpi_edit* e, int32_t which, const rpi_render_params* p,
                                       float* out, void* stream) {
  if (which != 0 && which != 1) return fail(RPI_ERR_INVALID_ARG, "which must be 0 (old frame) or 1 (new frame)");
  FrameArgs A;
  rpi_status rc = frame_common(s, p, out, A);
  if (rc) return rc;
  const float* pose = (e && which == 1) ? e->pose_new : kIdentity;
  const Material m = (e && which == 1) ? e->new_mat : s->obj_mat;
  A.F = make_frame(s, pose, pose, m, false);
  A.dir = which == 1 ? 0 : 1;  // the residual's direction index of that frame
  A.mode = 0;
  launch_frame(A, (hipStream_t)stream);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

extern "C" rpi_status rpi_render_frame_difference(const rpi_scene* s, const rpi_edit* e, int32_t correlated,
                                                  const rpi_render_params* p, float* out, void* stream) {
  if (!e) return fail(RPI_ERR_INVALID_ARG, "null edit");
  if (correlated != 0 && correlated != 1) return fail(RPI_ERR_INVALID_ARG, "correlated must be 0 or 1");
  FrameArgs A;
  rpi_status rc = frame_common(s, p, out, A);
  if (rc) return rc;
  A.F = make_frame(s, e->pose_new, e->pose_new, e->new_mat, false);
  A.F2 = make_frame(s, kIdentity, kIdentity, s->obj_mat, false);
  A.dir = 0;
  A.mode = correlated ? 1 : 2;
  launch_frame(A, (hipStream_t)stream);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

static Tuning scene_tuning(const rpi_scene* s, const rpi_render_params* p) {
  Tuning t;
  if (s->tuned_Q > 0) {
    t.Q = s->tuned_Q;
    t.walk_bpc = s->tuned_walk;
    t.conn_bpc = s->tuned_conn;
  }
  if (p->queue_cap > 0) t.Q = p->queue_cap;
  return t;
}

// Autotuner: time candidate (round size, persistent walk grid, connect grid)
// on a sample range of a representative job and keep the fastest.
static rpi_status autotune_job(rpi_scene* s, const JobSpec& j, bool material_mode, const rpi_render_params* p,
                               hipStream_t st, rpi_tuning* out) {
  rpi_render_params q = *p;
  q.flags &= ~(uint32_t)(RPI_FLAG_RECORDS | RPI_FLAG_COUNT_WORK | RPI_FLAG_ACCUMULATE | RPI_FLAG_PER_TECHNIQUE);
  q.flags |= RPI_FLAG_ACCUMULATE;
  for (int t = 0; t < kTechs; ++t) q.technique_spp[t] = 0;
  const int64_t N = (int64_t)p->spp * j.W * j.H;
  q.sample_begin = 0;
  // up to 2^24 samples per stream: the largest round holds that many samples
  // of both directions, so the window shows what rounds of each size cost
  q.sample_end = std::min<int64_t>(N, 1 << 24);
  if (q.d_min < 0) q.d_min = (float)(0.01 * (double)s->diag);
  const int Qs[3] = {1 << 23, 1 << 24, kMaxRound};
  const int walks[2] = {16, 32};
  double best = 1e300;
  Tuning bt;
  for (int qi = 0; qi < 3; ++qi)
    for (int wi = 0; wi < 2; ++wi) {
      Tuning t;
      t.Q = Qs[qi];
      t.walk_bpc = walks[wi];
      t.conn_bpc = 16;
      rpi_stats stt;
      rpi_status rc = run_jobs(s, {j}, material_mode, &q, t, &stt, st, nullptr);
      if (rc) return rc;
      if (stt.milliseconds < best) {
        best = stt.milliseconds;
        bt = t;
      }
    }
  s->tuned_Q = bt.Q;
  s->tuned_walk = bt.walk_bpc;
  s->tuned_conn = bt.conn_bpc;
  if (out) {
    out->queue_cap = bt.Q;
    out->walk_blocks_per_cu = bt.walk_bpc;
    out->connect_blocks_per_cu = bt.conn_bpc;
    out->ms_per_msample = best / ((double)(q.sample_end - q.sample_begin) * 14.0 / 1e6);
  }
  return RPI_OK;
}

extern "C" rpi_status rpi_autotune(rpi_scene* s, const rpi_edit* e, const rpi_render_params* p, rpi_tuning* out,
                                   void* stream) {
  if (!s || !e) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_status rc = check_params(s, p);
  if (rc) return rc;
  JobSpec j;
  std::memcpy(j.pose_old, e->pose_old, sizeof j.pose_old);
  std::memcpy(j.pose_new, e->pose_new, sizeof j.pose_new);
  j.mat_old = s->obj_mat;
  j.mat_new = e->new_mat;
  j.W = s->W;
  j.H = s->H;
  void* tmp = nullptr;
  rc = dev_alloc(s, (size_t)s->W * s->H * 3 * sizeof(float), (hipStream_t)stream, true, &tmp);
  if (rc) return rc;
  j.out = (float*)tmp;
  j.tech = nullptr;
  rc = autotune_job(s, j, e->kind == RPI_EDIT_MATERIAL, p, (hipStream_t)stream, out);
  dev_free(s, tmp, (hipStream_t)stream, true);
  return rc;
}

extern "C" rpi_status rpi_set_tuning(rpi_scene* s, const rpi_tuning* t) {
  if (!s || !t) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (t->queue_cap <= 0 || t->queue_cap % kItem || t->queue_cap > kMaxRound || t->walk_blocks_per_cu < 1 ||
      t->walk_blocks_per_cu > 64 || t->connect_blocks_per_cu < 1 || t->connect_blocks_per_cu > 64)
    return fail(RPI_ERR_INVALID_ARG, "bad tuning");
  s->tuned_Q = t->queue_cap;
  s->tuned_walk = t->walk_blocks_per_cu;
  s->tuned_conn = t->connect_blocks_per_cu;
  return RPI_OK;
}

extern "C" rpi_status rpi_get_tuning(const rpi_scene* s, rpi_tuning* t) {
  if (!s || !t) return fail(RPI_ERR_INVALID_ARG, "null argument");
  rpi_render_params p;
  std::memset(&p, 0, sizeof p);
  const Tuning tu = scene_tuning(s, &p);
  t->queue_cap = tu.Q;
  t->walk_blocks_per_cu = tu.walk_bpc;
  t->connect_blocks_per_cu = tu.conn_bpc;
  t->ms_per_msample = 0.0;
  return RPI_OK;
}

// A captured batch: persistent workspace, job table staging, graph.
struct BatchCache {
  std::vector<int> sizes;      // W, H per job
  rpi_render_params params;    // everything the graph bakes in
  Plan plan;
  Ws ws;
  DevJob* pinned = nullptr;    // host staging of the job table
  hipEvent_t staged = nullptr; // the last job-table upload has been consumed
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void destroy_batch_cache(BatchCache* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->staged) (void)hipEventDestroy(c->staged);
  if (c->pinned) (void)hipHostFree(c->pinned);
  ws_free(c->ws, nullptr);
  delete c;
}

static bool same_params(const rpi_render_params& a, const rpi_render_params& b) {
  return a.spp == b.spp && a.max_depth == b.max_depth && a.seed == b.seed && a.strategy_mask == b.strategy_mask &&
         a.flags == b.flags && a.alpha_min == b.alpha_min && a.d_min == b.d_min && a.jac_max == b.jac_max &&
         a.c_weight == b.c_weight && a.sample_begin == b.sample_begin && a.sample_end == b.sample_end &&
         a.queue_cap == b.queue_cap && a.job == b.job && a.proposal == b.proposal && a.tile == b.tile;
}

extern "C" rpi_status rpi_render_residual_batch(const rpi_scene* cs, const rpi_job* jobs, int32_t n,
                                                const rpi_render_params* p, rpi_stats* stats, void* stream) {
  rpi_scene* s = const_cast<rpi_scene*>(cs);
  if (!s || !jobs || n <= 0 || !p) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (n > 127) return fail(RPI_ERR_UNSUPPORTED, "at most 127 jobs per batch");
  if (p->spp <= 0 || p->max_depth < 2 || p->max_depth > 7 || p->strategy_mask == 0 || (p->strategy_mask & ~0xFFu) ||
      ((p->strategy_mask & 0x80u) && !p->proposal))
    return fail(RPI_ERR_INVALID_ARG, "bad params");
  if (p->d_train_records) return fail(RPI_ERR_UNSUPPORTED, "training-record collection is not available for batches");
  for (int t = 0; t < kTechs; ++t)
    if (p->technique_spp[t] != 0) return fail(RPI_ERR_UNSUPPORTED, "technique_spp is not available for batches");
  if (p->flags & (RPI_FLAG_RECORDS | RPI_FLAG_PER_TECHNIQUE))
    return fail(RPI_ERR_UNSUPPORTED, "records and per-technique images are not available for batches");
  if (p->tile != 0 && p->tile != 16 && p->tile != 32) return fail(RPI_ERR_INVALID_ARG, "tile must be 0, 16 or 32");
  if ((p->flags & RPI_FLAG_NO_MAPPING) && !(p->flags & RPI_FLAG_TWO_WAY))
    return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_NO_MAPPING needs RPI_FLAG_TWO_WAY");
  if ((p->flags & RPI_FLAG_BALANCE) && (!(p->flags & RPI_FLAG_TWO_WAY) || (p->strategy_mask & 0x80u)))
    return fail(RPI_ERR_UNSUPPORTED, "RPI_FLAG_BALANCE needs RPI_FLAG_TWO_WAY and no technique 8");
  hipStream_t st = (hipStream_t)stream;
  rpi_render_params q = *p;
  if (q.d_min < 0) q.d_min = (float)(0.01 * (double)s->diag);
  std::vector<JobSpec> js(n);
  std::vector<int> sizes;
  for (int i = 0; i < n; ++i) {
    const rpi_job& jb = jobs[i];
    if (jb.width <= 0 || jb.height <= 0 || !jb.d_out || (int64_t)jb.width * jb.height >= (1 << 24))
      return fail(RPI_ERR_INVALID_ARG, "bad job image");
    rpi_status rc = check_rigid(jb.pose_old);
    if (rc) return rc;
    rc = check_rigid(jb.pose_new);
    if (rc) return rc;
    std::memcpy(js[i].pose_old, jb.pose_old, 48);
    std::memcpy(js[i].pose_new, jb.pose_new, 48);
    js[i].mat_old = js[i].mat_new = s->obj_mat;
    js[i].W = jb.width;
    js[i].H = jb.height;
    js[i].out = jb.d_out;
    sizes.push_back(jb.width);
    sizes.push_back(jb.height);
  }
  if (q.flags & (RPI_FLAG_COUNT_WORK | RPI_FLAG_TIME_KERNELS)) {
    // instrumented or per-kernel-timed: the same plan and kernels launched
    // directly instead of through the captured graph
    if (s->tuned_Q == 0 && p->queue_cap <= 0) return fail(RPI_ERR_INVALID_ARG, "tune the scene first");
    return run_jobs(s, js, false, &q, scene_tuning(s, &q), stats, st, nullptr);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  BatchCache* c = s->batch;
  if (!c || c->sizes != sizes || !same_params(c->params, q)) {
    destroy_batch_cache(c);
    s->batch = nullptr;
    if (s->tuned_Q == 0 && p->queue_cap <= 0) {
      // tune on the largest job of the batch
      int big = 0;
      for (int i = 1; i < n; ++i)
        if ((int64_t)js[i].W * js[i].H > (int64_t)js[big].W * js[big].H) big = i;
      rpi_render_params tq = q;
      tq.sample_begin = 0;
      tq.sample_end = -1;
      rpi_status rc = autotune_job(s, js[big], false, &tq, st, nullptr);
      if (rc) return rc;
    }
    c = new BatchCache();
    c->sizes = sizes;
    c->params = q;
    rpi_status rc = make_plan(s, js, false, &q, scene_tuning(s, &q), c->plan);
    if (!rc)
      rc = ws_alloc(s, c->ws, c->plan.Q, q.max_depth, c->plan.pair_cap, c->plan.ntiles, n, false,
                    (q.strategy_mask & 0x80u) && q.proposal, c->plan.acc_elems, st, false);
    if (!rc) bind_jobs(c->plan, c->ws);
    if (rc) {
      destroy_batch_cache(c);
      return rc;
    }
    if (hipHostMalloc((void**)&c->pinned, sizeof(DevJob) * n, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      destroy_batch_cache(c);
      return fail(RPI_ERR_DEVICE, "batch setup failed");
    }
    rc = upload_plan(c->plan, c->ws, c->cap_stream);
    if (rc) {
      destroy_batch_cache(c);
      return rc;
    }
    RunOpts o;
    o.accumulate = (q.flags & RPI_FLAG_ACCUMULATE) != 0;
    o.stats = true;
    o.tu = scene_tuning(s, &q);
    // statistics are always counted inside the graph (cheap per-workgroup atomics)
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      destroy_batch_cache(c);
      return fail(RPI_ERR_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    launch_zero_u32((uint32_t*)c->ws.stats, sizeof(DevStats) / 4, c->cap_stream);
    rc = enqueue(c->plan, c->ws, &q, o, c->cap_stream, nullptr, nullptr);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &c->graph);
    if (rc || e2 != hipSuccess) {
      destroy_batch_cache(c);
      return rc ? rc : fail(RPI_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    }
    e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      destroy_batch_cache(c);
      return fail(RPI_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    s->batch = c;
  } else {
    // same shapes and parameters: refresh the job table (poses, output pointers)
    Plan pl;
    rpi_status rc = make_plan(s, js, false, &q, scene_tuning(s, &q), pl);
    if (rc) return rc;
    HIP_OK(hipEventSynchronize(c->staged));
    c->plan.jobs = pl.jobs;
    bind_jobs(c->plan, c->ws);
  }
  std::memcpy(c->pinned, c->plan.jobs.data(), sizeof(DevJob) * n);
  HIP_OK(hipMemcpyAsync(c->ws.jobs, c->pinned, sizeof(DevJob) * n, hipMemcpyHostToDevice, st));
  HIP_OK(hipEventRecord(c->staged, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, st));
  }
  HIP_OK(hipGraphLaunch(c->exec, st));
  if (stats) {
    HIP_OK(hipEventRecord(e1, st));
    DevStats ds;
    HIP_OK(hipMemcpyAsync(&ds, c->ws.stats, sizeof ds, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    fill_stats(stats, ds, c->plan, &q);
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    stats->milliseconds = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return RPI_OK;
}

// ------------------------------------------------------------------ learned proposal
static rpi_status upload_params(rpi_proposal* pr, const float* params) {
  for (int i = 0; i < kMlpNParam; ++i)
    if (!std::isfinite(params[i])) return fail(RPI_ERR_INVALID_ARG, "non-finite proposal parameter");
  HIP_OK(hipMemcpy(pr->B.master, params, kMlpNParam * sizeof(float), hipMemcpyHostToDevice));
  HIP_OK(hipMemset(pr->B.adam_m, 0, 2 * kMlpNParam * sizeof(float)));
  launch_mlp_pack(pr->B, nullptr);
  HIP_OK(hipGetLastError());
  HIP_OK(hipDeviceSynchronize());
  pr->steps = 0;
  return RPI_OK;
}

extern "C" rpi_status rpi_proposal_create(const rpi_scene* s, const float* params, uint64_t seed, rpi_proposal** out) {
  if (!s || !out) return fail(RPI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<rpi_proposal> pr(new rpi_proposal());
  object_normalisation(s, pr->center, pr->inv_half);
  // masters, Adam m and v, biases (4 x 64, the last 8 padding), BF16 block
  const size_t nf = 3 * (size_t)kMlpNParam + 256;
  const size_t bytes = nf * sizeof(float) + (size_t)kMlpHalfElems * sizeof(uint16_t);
  if (hipMalloc(&pr->mem, bytes) != hipSuccess) return fail(RPI_ERR_OUT_OF_MEMORY, "proposal allocation failed");
  HIP_OK(hipMemset(pr->mem, 0, bytes));  // padding rows / columns stay zero
  float* f = (float*)pr->mem;
  pr->B.master = f;
  pr->B.adam_m = f + kMlpNParam;
  pr->B.adam_v = f + 2 * kMlpNParam;
  pr->B.bias = f + 3 * kMlpNParam;
  pr->B.h = (uint16_t*)(f + nf);
  std::vector<float> init;
  if (!params) {
    // He-uniform weights, zero biases
    init.assign(kMlpNParam, 0.0f);
    std::mt19937_64 rng(seed);
    const int fan_in[4] = {6, 64, 64, 64}, off[4] = {0, 448, 4608, 8768}, cnt[4] = {384, 4096, 4096, 2560};
    for (int L = 0; L < 4; ++L) {
      std::uniform_real_distribution<float> U(-std::sqrt(6.0f / fan_in[L]), std::sqrt(6.0f / fan_in[L]));
      for (int i = 0; i < cnt[L]; ++i) init[off[L] + i] = U(rng);
    }
    params = init.data();
  }
  rpi_status rc = upload_params(pr.get(), params);
  if (rc) {
    (void)hipFree(pr->mem);
    return rc;
  }
  *out = pr.release();
  return RPI_OK;
}

extern "C" rpi_status rpi_proposal_destroy(rpi_proposal* pr) {
  if (!pr) return RPI_OK;
  (void)hipDeviceSynchronize();
  if (pr->mem) (void)hipFree(pr->mem);
  delete pr;
  return RPI_OK;
}

extern "C" rpi_status rpi_proposal_set_weights(rpi_proposal* pr, const float* params) {
  if (!pr || !params) return fail(RPI_ERR_INVALID_ARG, "null argument");
  HIP_OK(hipDeviceSynchronize());
  return upload_params(pr, params);
}

extern "C" rpi_status rpi_proposal_get_weights(const rpi_proposal* pr, float* params) {
  if (!pr || !params) return fail(RPI_ERR_INVALID_ARG, "null argument");
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(params, pr->B.master, kMlpNParam * sizeof(float), hipMemcpyDeviceToHost));
  return RPI_OK;
}

extern "C" rpi_status rpi_proposal_forward(const rpi_proposal* pr, const float* x, int64_t n, float* out,
                                          void* stream) {
  if (!pr || (n > 0 && (!x || !out))) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (n < 0) return fail(RPI_ERR_INVALID_ARG, "negative row count");
  if (n == 0) return RPI_OK;
  launch_mlp_forward(pr->view(), x, n, out, (hipStream_t)stream);
  HIP_OK(hipGetLastError());
  return RPI_OK;
}

namespace {
constexpr int kMaxGradBlocks = 1024;
int grad_blocks(int64_t rows) { return (int)std::min<int64_t>((rows + 63) / 64, kMaxGradBlocks); }
}  // namespace

extern "C" rpi_status rpi_proposal_loss_grad(const rpi_proposal* pr, const float* rec, int64_t n, float* grad,
                                            float* loss, void* stream) {
  if (!pr || !rec || !grad) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (n < 1) return fail(RPI_ERR_INVALID_ARG, "need at least one record");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = grad_blocks(n);
  float* partial = nullptr;
  HIP_OK(hipMallocAsync((void**)&partial, (size_t)blocks * kMlpPartial * sizeof(float), st));
  launch_mlp_grad(pr->view(), rec, n, n, 0, 0u, 0u, 0u, partial, blocks, st);
  launch_mlp_reduce(partial, blocks, grad, loss, st);
  hipError_t le = hipGetLastError();
  (void)hipFreeAsync(partial, st);
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}

extern "C" rpi_status rpi_proposal_train(rpi_proposal* pr, const float* rec, int64_t n, const rpi_train_params* tp,
                                        float* losses, void* stream) {
  if (!pr || !rec || !tp) return fail(RPI_ERR_INVALID_ARG, "null argument");
  if (n < 1 || n > 0xffffffffLL) return fail(RPI_ERR_INVALID_ARG, "record count must be in [1, 2^32)");
  if (tp->steps < 0 || tp->batch < 64 || tp->batch % 64 || tp->batch > (1 << 20))
    return fail(RPI_ERR_INVALID_ARG, "batch must be a positive multiple of 64 up to 2^20");
  if (!(tp->lr > 0.0f) || !(tp->beta1 >= 0.0f && tp->beta1 < 1.0f) || !(tp->beta2 >= 0.0f && tp->beta2 < 1.0f) ||
      !(tp->eps > 0.0f))
    return fail(RPI_ERR_INVALID_ARG, "bad Adam parameters");
  if (tp->steps == 0) return RPI_OK;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = grad_blocks(tp->batch);
  float* partial = nullptr;
  HIP_OK(hipMallocAsync((void**)&partial, (size_t)blocks * kMlpPartial * sizeof(float), st));
  const MlpDev M = pr->view();
  for (int t = 1; t <= tp->steps; ++t) {
    const int step = pr->steps + t;
    launch_mlp_grad(M, rec, n, tp->batch, 1, (uint32_t)tp->seed, (uint32_t)(tp->seed >> 32), (uint32_t)step, partial,
                    blocks, st);
    launch_mlp_adam(partial, blocks, pr->B, tp->lr, tp->beta1, tp->beta2, tp->eps, step,
                    losses ? losses + (t - 1) : nullptr, st);
  }
  pr->steps += tp->steps;
  hipError_t le = hipGetLastError();
  (void)hipFreeAsync(partial, st);
  if (le != hipSuccess) return fail(RPI_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(le));
  return RPI_OK;
}
