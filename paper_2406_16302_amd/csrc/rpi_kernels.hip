// HIP kernels of the residual path estimator (gfx950, wave64).
//
// Pipeline per (technique, round of samples of both directions), all on one
// stream:
//   start_order_kernel   the round's samples ordered by where they start (a
//                        counting sort by grid cell of x_D / x_G, or by pixel
//                        tile), so that the lanes of a wave start close
//                        together;
//   walk_kernel<TECH>    one lane per sample: start sampling (Sec. 4.1/4.2) and
//                        the start's ray queries (path tracing, 7, also walks
//                        here); samples whose walks go on are queued as tasks;
//   walk_task_kernel<TECH>  the queued walks, each lane stepping its own task
//                        through one traversal loop shared by the wave: random
//                        walks with BVH traversal, next-event and camera
//                        connections, ghost-crossing records (Sec. 4.3, 6.1).
//                        Sub-path vertices go to SoA records in HBM and every
//                        connected path is appended to a queue with one atomic
//                        per wave (ballot/prefix compaction);
//   pair_hist/pair_sort/pair_order  the path queue sorted by path length,
//                        then within windows by the pixel tile of x_1;
//   connect_kernel       one lane per connected path: MIS over N_D + N_G + 1
//                        strategies from forward/backward pdf prefix tables
//                        (Sec. 4.3), path mapping and rejection (Sec. 5),
//                        evaluation in both frames (eq. shiftmapped), one
//                        signed splat record per path;
//   splat kernels        counting sort of the records by tile (16x16 or
//                        32x32), then workgroups take chunks of a tile's
//                        records and sum them per pixel in LDS in fixed point;
//                        the sums go to a fixed-point image that is turned into
//                        the float image at the end of the call (no float
//                        atomics: the image is the same bit for bit whatever
//                        the order).
// Technique 8 adds t8_start_kernel (the learned proposal at x_D and the
// direction drawn from it) and proposal_pdf_kernel (its density at the queued
// paths' dynamic vertices, for the MIS sums).  frame_kernel renders a frame by
// plain path tracing (Sec. 3.1).
#include "rpi_device.h"
#include "rpi_mlp.h"

namespace rpi {

constexpr int kMaxK = 8;  // vertices per path: max_depth <= 7
constexpr int kTileMax = 32;  // splat tile edge is 16 or 32 (SplatArgs::ts)

// ------------------------------------------------------------------ SoA records
DEV float4 f4(vec3 a, float w) { return make_float4(a.x, a.y, a.z, w); }
DEV float4 f4u(vec3 a, uint32_t w) { return make_float4(a.x, a.y, a.z, __uint_as_float(w)); }
DEV vec3 xyz(float4 a) { return v3(a.x, a.y, a.z); }

DEV float4& EYE(const Workspace& W, int slot, int field, int s) {
  return W.eye[((size_t)slot * kEyeFields + field) * W.Q + s];
}
DEV float4& LIT(const Workspace& W, int slot, int field, int s) {
  return W.light[((size_t)slot * kLightFields + field) * W.Q + s];
}
DEV float4& STA(const Workspace& W, int field, int s) { return W.start[(size_t)field * W.Q + s]; }

// reflection-only support at vertex p: both neighbours on one side
DEV bool same_side(vec3 n, vec3 p, vec3 a, vec3 b) { return dot(n, a - p) * dot(n, b - p) > 0.0f; }
DEV bool same_side_dir(vec3 n, vec3 p, vec3 a, vec3 dir) { return dot(n, a - p) * dot(n, dir) > 0.0f; }

DEV bool is_emitter(const DevScene& S, uint32_t md) {
  return !(md & kDynBit) && S.mats[8 * (md & ~kDynBit)] == (float)MAT_EMITTER;
}

// What a walk of one work item sees: its job's scene and frame, the workspace.
struct Ctx {
  const DevScene& S;
  const DevFrame& F;
  const Workspace& W;
  int depth;
};

// A random walk the start phase of a technique hands to its walk phase:
// start vertex, crossings of the edge into it, the neighbour on the other
// side (towards the camera for a light walk, towards the light for an eye
// walk) and the last slot.
struct WalkStart {
  vec3 p, n;
  uint32_t md;
  Cross pred;
  End end;
  int lim;
};

struct Lane {
  const Ctx& A;
  Rng g;
  int s;
  int* stk;
  WorkCount wc;
  int nE, nL;
  uint32_t camok, neeok, dynpre;
  int k2;  // path tracing saw an emitter / the environment at x_1; technique 8: the camera sees x_D
  int64_t sample;  // sample index within its (technique, direction) stream
  uint32_t defer;  // walks left for the walk phase: bit 0 light, bit 1 eye
  WalkStart lw, ew;
};

DEV void defer_light(Lane& L, vec3 p0, vec3 n0, uint32_t md0, Cross pred0, End prev0, int jmax) {
  if (jmax < 0) return;
  L.lw = WalkStart{p0, n0, md0, pred0, prev0, jmax};
  L.defer |= 1u;
}
DEV void defer_eye(Lane& L, vec3 p0, vec3 n0, uint32_t md0, Cross pred0, End next0, int imax) {
  if (imax < 0) return;
  L.ew = WalkStart{p0, n0, md0, pred0, next0, imax};
  L.defer |= 2u;
}

// Extend a walk from (p, n, md) whose other neighbour lies in direction wi.
template <bool CW>
DEV bool extend(Lane& L, vec3 p, vec3 n, uint32_t md, vec3 wi, const float u[4], vec3& q, vec3& qn,
                uint32_t& qmd) {
  const Material m = vmat(L.A.S, L.A.F, md);
  vec3 wo;
  if (!bsdf_sample(m, n, wi, u[0], u[1], wo)) return false;
  const vec3 o = spawn_dir(L.A.S, p, n, wo);
  const bool noobj = (md & kDynBit) && leaves_convex(L.A.S, L.A.F.pose, p, n, wo);
  const Hit h = closest<CW>(L.A.S, L.A.F, o, wo, L.stk, L.wc, RAY_CLOSEST, noobj);
  if (!h.ok) return false;
  hit_vertex(L.A.S, L.A.F.pose, h, o, wo, q, qn, qmd);
  return !is_emitter(L.A.S, qmd) && !interior_hit(L.A.S, L.A.F, q, qn, qmd, p);
}

DEV uint32_t light_word(const LightEnd& E) { return E.mat | (E.env ? 0x40000000u : 0u); }

// Light-side walk.  Slot 0 vertex (p0, n0, md0) with its predecessor edge
// crossing pred0; prev0 = the neighbour towards the camera.  Next-event
// estimation at each vertex.  dyn0: path-tracing dynamic state before slot 0.
template <bool CW>
// dyn_only: only paths with a dynamic vertex or ghost crossing count (path
// tracing with static paths rejected), so a light connection from a static
// prefix is traced only if it may cross the ghost.
DEV void light_walk(Lane& L, vec3 p0, vec3 n0, uint32_t md0, Cross pred0, End prev0, int jmax, bool dyn0,
                    bool dyn_only) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  vec3 p = p0, n = n0;
  uint32_t md = md0;
  Cross pred = pred0;
  End prev = prev0;
  bool dyn = dyn0;
  for (int j = 0; j <= jmax; ++j) {
    dyn = dyn || (md & kDynBit) || pred.n > 0.0f;
    // next-event estimation
    float u[4];
    draw(L.g, 0, j + 1, 1, u);
    LightEnd E;
    bool ok = sample_light(S, u, E);
    Cross nee = no_cross();
    if (ok) {
      const End eL = end_light(E);
      ok = E.env ? same_side_dir(n, p, prev.p, E.n)
                 : (dot(E.n, p - E.p) > 0.0f && same_side(n, p, prev.p, E.p));
      if (ok && dyn_only && !dyn) {
        const Seg sg = canon(S, end_surf(p, n), eL);
        ok = A.F.ghosts && near_ghost(A.F, sg.o, sg.d, sg.tmax);
      }
      if (ok) {
        const End cur = end_surf(p, n);
        const bool noobj = (md & kDynBit) && leaves_convex(S, A.F.pose, p, n, E.env ? E.n : E.p - p);
        ok = edge_visible<CW>(S, A.F, cur, eL, L.stk, L.wc, RAY_SHADOW, noobj);
        if (ok) nee = edge_cross<CW>(S, A.F, cur, eL, L.stk, L.wc);
      }
    }
    LIT(A.W, j, 0, L.s) = f4u(p, md);
    LIT(A.W, j, 1, L.s) = f4(n, pred.n);
    LIT(A.W, j, 2, L.s) = make_float4(pred.s0, pred.sa, pred.sb, 0.0f);
    LIT(A.W, j, 3, L.s) = f4u(E.p, light_word(E));
    LIT(A.W, j, 4, L.s) = f4(E.n, nee.n);
    LIT(A.W, j, 5, L.s) = make_float4(nee.s0, nee.sa, nee.sb, 0.0f);
    if (CW) L.wc.bytes += kLightFields * 16;
    L.nL = j + 1;
    if (ok) L.neeok |= 1u << j;
    if (dyn || nee.n > 0.0f) L.dynpre |= 1u << j;
    if (j == jmax) break;
    draw(L.g, 0, j + 1, 0, u);
    vec3 q, qn;
    uint32_t qmd;
    if (!extend<CW>(L, p, n, md, unit(prev.p - p), u, q, qn, qmd)) break;
    pred = edge_cross<CW>(S, A.F, end_surf(p, n), end_surf(q, qn), L.stk, L.wc);
    prev = end_surf(p, n);
    p = q;
    n = qn;
    md = qmd;
  }
}

// Eye-side walk.  Slot 0 vertex with predecessor crossing pred0 (the edge to
// next0, its neighbour towards the light); camera connection at each vertex.
template <bool CW>
DEV void eye_walk(Lane& L, vec3 p0, vec3 n0, uint32_t md0, Cross pred0, End next0, int imax) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  vec3 p = p0, n = n0;
  uint32_t md = md0;
  Cross pred = pred0;
  End next = next0;
  for (int i = 0; i <= imax; ++i) {
    const vec3 nxt = next.kind == END_ENV ? p + next.n : next.p;
    bool ok = raster(S.cam, p) >= 0 && same_side(n, p, S.cam.eye, nxt);
    Cross cam = no_cross();
    if (ok) {
      const End e0 = end_eye(S), cur = end_surf(p, n);
      const bool noobj = (md & kDynBit) && leaves_convex(S, A.F.pose, p, n, S.cam.eye - p);
      ok = edge_visible<CW>(S, A.F, e0, cur, L.stk, L.wc, RAY_CAMERA, noobj);
      if (ok) cam = edge_cross<CW>(S, A.F, e0, cur, L.stk, L.wc);
    }
    EYE(A.W, i, 0, L.s) = f4u(p, md);
    EYE(A.W, i, 1, L.s) = f4(n, pred.n);
    EYE(A.W, i, 2, L.s) = make_float4(pred.s0, pred.sa, pred.sb, 0.0f);
    EYE(A.W, i, 3, L.s) = make_float4(cam.n, cam.s0, cam.sa, cam.sb);
    if (CW) L.wc.bytes += kEyeFields * 16;
    L.nE = i + 1;
    if (ok) L.camok |= 1u << i;
    if (i == imax) break;
    float u[4];
    draw(L.g, 1, i + 1, 0, u);
    vec3 q, qn;
    uint32_t qmd;
    if (!extend<CW>(L, p, n, md, unit(nxt - p), u, q, qn, qmd)) break;
    pred = edge_cross<CW>(S, A.F, end_surf(q, qn), end_surf(p, n), L.stk, L.wc);
    next = end_surf(p, n);
    p = q;
    n = qn;
    md = qmd;
  }
}

DEV void store_xl(const Lane& L, const LightEnd& E) {
  STA(L.A.W, 3, L.s) = f4u(E.p, light_word(E));
  STA(L.A.W, 4, L.s) = f4(E.n, 0.0f);
}
DEV void store_mid(const Lane& L, vec3 p, vec3 n, uint32_t md, Cross cam, uint32_t flags) {
  STA(L.A.W, 0, L.s) = f4u(p, md);
  STA(L.A.W, 1, L.s) = f4(n, cam.n);
  STA(L.A.W, 2, L.s) = make_float4(cam.s0, cam.sa, cam.sb, __uint_as_float(flags));
}

// A ghost-started sample generates its path only if its ghost triangle is
// crossed strictly inside the generated edge's canonical segment.
DEV bool ghost_on_edge(const Lane& L, const End& A, const End& B, int tri) {
  const DevScene& S = L.A.S;
  const Seg s = canon(S, A, B);
  vec3 v0, e1, e2;
  int id, mat;
  load_tri(S.obj_tris, tri, v0, e1, e2, id, mat);
  const float t = tri_t(pose_inv_apply(L.A.F.ghost, s.o), pose_inv_rot(L.A.F.ghost, s.d), v0, e1, e2);
  return t > 0.0f && t < s.tmax;
}

// (1) dynamic from emitter
template <bool CW>
DEV void tech1(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 p, n;
  uint32_t md;
  int tri;
  object_point(S, A.F.pose, u, p, n, md, tri);
  draw(L.g, 0, 0, 1, u);
  LightEnd E;
  if (!sample_light(S, u, E)) return;
  const End eL = end_light(E);
  if (!E.env && !(dot(E.n, p - E.p) > 0.0f)) return;
  if (into_sealed(S, A.F, p, n, E.env ? E.n : E.p - p)) return;  // the object itself blocks the light
  if (!edge_visible<CW>(S, A.F, end_surf(p, n), eL, L.stk, L.wc, RAY_SHADOW,
                        leaves_convex(S, A.F.pose, p, n, E.env ? E.n : E.p - p)))
    return;
  const Cross c = edge_cross<CW>(S, A.F, end_surf(p, n), eL, L.stk, L.wc);
  store_xl(L, E);
  defer_eye(L, p, n, md, c, eL, A.depth - 2);
}

// (2) dynamic from sensor
template <bool CW>
DEV void tech2(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  if (A.depth < 3) return;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 p, n;
  uint32_t md;
  int tri;
  object_point(S, A.F.pose, u, p, n, md, tri);
  if (raster(S.cam, p) < 0) return;
  const End e0 = end_eye(S), xd = end_surf(p, n);
  if (into_sealed(S, A.F, p, n, S.cam.eye - p)) return;  // x_D faces away from the camera
  if (!edge_visible<CW>(S, A.F, e0, xd, L.stk, L.wc, RAY_CAMERA, leaves_convex(S, A.F.pose, p, n, S.cam.eye - p)))
    return;
  const Cross cam = edge_cross<CW>(S, A.F, e0, xd, L.stk, L.wc);
  draw(L.g, 0, 0, 2, u);
  vec3 q, qn;
  uint32_t qmd;
  if (!extend<CW>(L, p, n, md, unit(S.cam.eye - p), u, q, qn, qmd)) return;
  store_mid(L, p, n, md, cam, 1u);
  const Cross pred = edge_cross<CW>(S, A.F, xd, end_surf(q, qn), L.stk, L.wc);
  defer_light(L, q, qn, qmd, pred, xd, A.depth - 3);
}

// (3) dynamic two ends: cosine lobe about the outward normal towards the
// light side, then a BSDF direction towards the sensor.
template <bool CW>
DEV void tech3(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  if (A.depth < 4) return;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 p, n;
  uint32_t md;
  int tri;
  object_point(S, A.F.pose, u, p, n, md, tri);
  draw(L.g, 0, 0, 2, u);
  const vec3 wl = cosine_dir(n, u[0], u[1]);
  if (!(dot(wl, n) > 0.0f)) return;
  if (into_sealed(S, A.F, p, n, wl)) return;  // into the object: the light side would start inside
  const vec3 ol = spawn_dir(S, p, n, wl);
  const Hit hl = closest<CW>(S, A.F, ol, wl, L.stk, L.wc, RAY_CLOSEST,
                             leaves_convex(S, A.F.pose, p, n, wl));
  if (!hl.ok) return;
  vec3 l0, l0n;
  uint32_t l0md;
  hit_vertex(S, A.F.pose, hl, ol, wl, l0, l0n, l0md);
  if (is_emitter(S, l0md)) return;
  if (interior_hit(S, A.F, l0, l0n, l0md, p)) return;  // the light side starts inside the object
  draw(L.g, 0, 0, 3, u);
  const Material m = vmat(S, A.F, md);
  // the sensor-side BSDF sample sees x_{m+1} as its incoming direction
  vec3 we;
  if (!bsdf_sample(m, n, unit(l0 - p), u[0], u[1], we)) return;
  if (into_sealed(S, A.F, p, n, we)) return;
  const vec3 oe = spawn_dir(S, p, n, we);
  const Hit he = closest<CW>(S, A.F, oe, we, L.stk, L.wc, RAY_CLOSEST,
                             leaves_convex(S, A.F.pose, p, n, we));
  if (!he.ok) return;
  vec3 e0, e0n;
  uint32_t e0md;
  hit_vertex(S, A.F.pose, he, oe, we, e0, e0n, e0md);
  if (is_emitter(S, e0md)) return;
  if (interior_hit(S, A.F, e0, e0n, e0md, p)) return;  // the sensor side starts inside the object
  const End xd = end_surf(p, n);
  store_mid(L, p, n, md, no_cross(), 1u);
  const Cross ce = edge_cross<CW>(S, A.F, end_surf(e0, e0n), xd, L.stk, L.wc);
  const Cross cl = edge_cross<CW>(S, A.F, xd, end_surf(l0, l0n), L.stk, L.wc);
  defer_light(L, l0, l0n, l0md, cl, xd, A.depth - 4);
  defer_eye(L, e0, e0n, e0md, ce, xd, A.depth - 4);
}

// (8) learned proposal: x_D and its light-side direction come from the start
// kernel (the MLP's vMF mixture at x_D, start records 0, 1, 3).  The sensor
// side is the camera seeing x_D directly (technique (2)'s paths) and, as in
// technique (3), a BSDF direction towards the sensor and an eye walk.
template <bool CW>
DEV void tech8(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  if (A.depth < 3) return;
  const float4 a = STA(A.W, 0, L.s), b = STA(A.W, 1, L.s), c = STA(A.W, 3, L.s);
  const vec3 p = xyz(a), n = xyz(b), wl = xyz(c);
  const uint32_t md = __float_as_uint(a.w);
  if (into_sealed(S, A.F, p, n, wl)) return;  // into the object: the light side would start inside
  const vec3 ol = spawn_dir(S, p, n, wl);
  const Hit hl = closest<CW>(S, A.F, ol, wl, L.stk, L.wc, RAY_CLOSEST,
                             leaves_convex(S, A.F.pose, p, n, wl));
  if (!hl.ok) return;
  vec3 l0, l0n;
  uint32_t l0md;
  hit_vertex(S, A.F.pose, hl, ol, wl, l0, l0n, l0md);
  if (is_emitter(S, l0md)) return;
  if (interior_hit(S, A.F, l0, l0n, l0md, p)) return;  // the light side starts inside the object
  const End xd = end_surf(p, n);
  // the camera sees x_D, on the side of l0
  Cross cam = no_cross();
  if (raster(S.cam, p) >= 0 && same_side(n, p, S.cam.eye, l0) && !into_sealed(S, A.F, p, n, S.cam.eye - p)) {
    const End e0 = end_eye(S);
    if (edge_visible<CW>(S, A.F, e0, xd, L.stk, L.wc, RAY_CAMERA, leaves_convex(S, A.F.pose, p, n, S.cam.eye - p))) {
      cam = edge_cross<CW>(S, A.F, e0, xd, L.stk, L.wc);
      L.k2 = 1;
    }
  }
  store_mid(L, p, n, md, cam, 1u);
  const Cross cl = edge_cross<CW>(S, A.F, xd, end_surf(l0, l0n), L.stk, L.wc);
  // one bounce further when the camera sees x_D (paths x_0 x_D l_0 .. l_j)
  defer_light(L, l0, l0n, l0md, cl, xd, L.k2 ? A.depth - 3 : A.depth - 4);
  // a BSDF direction towards the sensor; its incoming direction is x_{m+1}
  if (A.depth < 4) return;
  float u[4];
  draw(L.g, 0, 0, 3, u);
  const Material m = vmat(S, A.F, md);
  vec3 we;
  if (!bsdf_sample(m, n, unit(l0 - p), u[0], u[1], we)) return;
  if (into_sealed(S, A.F, p, n, we)) return;
  const vec3 oe = spawn_dir(S, p, n, we);
  const Hit he = closest<CW>(S, A.F, oe, we, L.stk, L.wc, RAY_CLOSEST,
                             leaves_convex(S, A.F.pose, p, n, we));
  if (!he.ok) return;
  vec3 e0, e0n;
  uint32_t e0md;
  hit_vertex(S, A.F.pose, he, oe, we, e0, e0n, e0md);
  if (is_emitter(S, e0md)) return;
  if (interior_hit(S, A.F, e0, e0n, e0md, p)) return;  // the sensor side starts inside the object
  const Cross ce = edge_cross<CW>(S, A.F, end_surf(e0, e0n), xd, L.stk, L.wc);
  defer_eye(L, e0, e0n, e0md, ce, xd, A.depth - 4);
}

// (4) ghost from emitter: the ray x_L -> x_G gives the first vertex.
template <bool CW>
DEV void tech4(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 xg, ng;
  uint32_t gmd;
  int tri;
  object_point(S, A.F.ghost, u, xg, ng, gmd, tri);
  if (deep_inside(S, A.F, xg)) return;  // x_G inside the object: no path of this start
  draw(L.g, 0, 0, 1, u);
  LightEnd E;
  if (!sample_light(S, u, E) || E.env) return;
  if (!(dot(E.n, xg - E.p) > 0.0f)) return;
  const vec3 o = spawn(S, E.p, E.n, xg);
  const vec3 w = unit(xg - o);
  const float tg = sqrtf(len2(xg - o));
  const Hit h = closest<CW>(S, A.F, o, w, L.stk, L.wc, RAY_CLOSEST, false, tg);
  if (!h.ok || !(h.t > tg)) return;
  vec3 q, qn;
  uint32_t qmd;
  hit_vertex(S, A.F.pose, h, o, w, q, qn, qmd);
  if (is_emitter(S, qmd)) return;
  const End eL = end_light(E), x1 = end_surf(q, qn);
  if (!ghost_on_edge(L, x1, eL, tri)) return;
  const Cross c = edge_cross<CW>(S, A.F, x1, eL, L.stk, L.wc);
  store_xl(L, E);
  defer_eye(L, q, qn, qmd, c, eL, A.depth - 2);
}

// (5) ghost from sensor: the camera ray through x_G gives x_1.
template <bool CW>
DEV void tech5(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  if (A.depth < 2) return;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 xg, ng;
  uint32_t gmd;
  int tri;
  object_point(S, A.F.ghost, u, xg, ng, gmd, tri);
  if (deep_inside(S, A.F, xg)) return;  // x_G inside the object: no path of this start
  const vec3 w = unit(xg - S.cam.eye);
  const float tg = sqrtf(len2(xg - S.cam.eye));
  const Hit h = closest<CW>(S, A.F, S.cam.eye, w, L.stk, L.wc, RAY_CLOSEST, false, tg);
  if (!h.ok || !(h.t > tg)) return;
  vec3 q, qn;
  uint32_t qmd;
  hit_vertex(S, A.F.pose, h, S.cam.eye, w, q, qn, qmd);
  if (is_emitter(S, qmd)) return;
  if (raster(S.cam, q) < 0) return;
  const End e0 = end_eye(S), x1 = end_surf(q, qn);
  if (!ghost_on_edge(L, e0, x1, tri)) return;
  const Cross c = edge_cross<CW>(S, A.F, e0, x1, L.stk, L.wc);
  defer_light(L, q, qn, qmd, c, e0, A.depth - 2);
}

// (6) ghost two ends: a uniform direction through x_G, rays both ways.
template <bool CW>
DEV void tech6(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  if (A.depth < 3) return;
  float u[4];
  draw(L.g, 0, 0, 0, u);
  vec3 xg, ng;
  uint32_t gmd;
  int tri;
  object_point(S, A.F.ghost, u, xg, ng, gmd, tri);
  if (deep_inside(S, A.F, xg)) return;  // x_G inside the object: no path of this start
  draw(L.g, 0, 0, 2, u);
  const vec3 w = sphere_dir(u[0], u[1]);
  Hit hl, he;  // the closest hits along w and -w, in one line query
  closest_line<CW>(S, A.F, xg, w, hl, he, L.stk, L.wc);
  if (!hl.ok) return;
  vec3 l0, l0n;
  uint32_t l0md;
  hit_vertex(S, A.F.pose, hl, xg, w, l0, l0n, l0md);
  if (is_emitter(S, l0md)) return;
  if (interior_hit(S, A.F, l0, l0n, l0md, xg)) return;  // x_G inside the object: no path leaves it
  if (!he.ok) return;
  vec3 e0, e0n;
  uint32_t e0md;
  hit_vertex(S, A.F.pose, he, xg, -w, e0, e0n, e0md);
  if (is_emitter(S, e0md)) return;
  if (interior_hit(S, A.F, e0, e0n, e0md, xg)) return;
  const End ee = end_surf(e0, e0n), el = end_surf(l0, l0n);
  if (!ghost_on_edge(L, ee, el, tri)) return;
  const Cross c = edge_cross<CW>(S, A.F, ee, el, L.stk, L.wc);
  defer_light(L, l0, l0n, l0md, c, ee, A.depth - 3);
  defer_eye(L, e0, e0n, e0md, c, el, A.depth - 3);
}

// (7) path tracing with static paths rejected (and tech 0: plain frames).
template <bool CW>
DEV void tech7(Lane& L) {
  const Ctx& A = L.A;
  const DevScene& S = A.S;
  const int P = S.cam.W * S.cam.H;
  const int pixel = (int)((uint32_t)L.sample % (uint32_t)P);  // streams hold < 2^32 samples
  float u[4];
  draw(L.g, 0, 0, 0, u);
  const vec3 w = camera_dir(S.cam, pixel, u[0], u[1]);
  const Hit h = closest<CW>(S, A.F, S.cam.eye, w, L.stk, L.wc);
  const End e0 = end_eye(S);
  if (!h.ok) {
    if (S.p_env > 0.0f) {
      LightEnd E;
      E.env = 1;
      E.n = w;
      E.p = v3(0, 0, 0);
      E.mat = 0;
      if (raster(S.cam, S.cam.eye + w) < 0) return;
      const Cross c = edge_cross<CW>(S, A.F, e0, end_light(E), L.stk, L.wc);
      store_xl(L, E);
      store_mid(L, v3(0, 0, 0), v3(0, 0, 0), 0u, c, 0u);
      L.k2 = c.n > 0.0f ? 1 : 0;
    }
    return;
  }
  vec3 q, qn;
  uint32_t qmd;
  hit_vertex(S, A.F.pose, h, S.cam.eye, w, q, qn, qmd);
  if (is_emitter(S, qmd)) {
    LightEnd E;
    E.env = 0;
    E.p = q;
    E.n = qn;
    E.mat = qmd & ~kDynBit;
    if (!(dot(qn, S.cam.eye - q) > 0.0f) || raster(S.cam, q) < 0) return;
    const Cross c = edge_cross<CW>(S, A.F, e0, end_light(E), L.stk, L.wc);
    store_xl(L, E);
    store_mid(L, v3(0, 0, 0), v3(0, 0, 0), 0u, c, 0u);
    L.k2 = c.n > 0.0f ? 1 : 0;
    return;
  }
  if (raster(S.cam, q) < 0) return;
  const Cross c = edge_cross<CW>(S, A.F, e0, end_surf(q, qn), L.stk, L.wc);
  defer_light(L, q, qn, qmd, c, e0, A.depth - 2);
}

// Number of connected paths of a sample and the i-th of them.
template <int TECH, class LaneT>
DEV int pair_count(const LaneT& L, int depth) {
  int c = 0;
  if (TECH == 1 || TECH == 4) {
    c = __popc(L.camok);
  } else if (TECH == 2 || TECH == 5) {
    c = __popc(L.neeok);
  } else if (TECH == 7) {
    c = __popc(L.neeok & L.dynpre) + L.k2;
  } else {
    if (TECH == 8 && L.k2) c = __popc(L.neeok);  // the camera sees x_D: one path per light vertex
    const int extra = (TECH == 3 || TECH == 8) ? 4 : 3;
    for (int i = 0; i < L.nE; ++i)
      if (L.camok >> i & 1u)
        for (int j = 0; j < L.nL; ++j)
          if ((L.neeok >> j & 1u) && i + j + extra <= depth) ++c;
  }
  return c;
}
// Connected path code: sample slot << 6 | (i + 1) << 3 | (j + 1) (slots below
// 2^26; i + 1 and j + 1 below 8 since paths have at most 8 vertices).
DEV uint32_t pair_code(int s, int i, int j) { return ((uint32_t)s << 6) | ((uint32_t)(i + 1) << 3) | (uint32_t)(j + 1); }
DEV int code_slot(uint32_t code) { return (int)(code >> 6); }
DEV int code_i(uint32_t code) { return (int)((code >> 3) & 7u) - 1; }
DEV int code_j(uint32_t code) { return (int)(code & 7u) - 1; }

template <int TECH, class LaneT>
DEV void write_pairs(const LaneT& L, uint32_t* out, int depth) {
  int w = 0;
  if (TECH == 1 || TECH == 4) {
    for (int i = 0; i < L.nE; ++i)
      if (L.camok >> i & 1u) out[w++] = pair_code(L.s, i, -1);
  } else if (TECH == 2 || TECH == 5 || TECH == 7) {
    if (TECH == 7 && L.k2) out[w++] = pair_code(L.s, -1, -1);
    const uint32_t m = TECH == 7 ? (L.neeok & L.dynpre) : L.neeok;
    for (int j = 0; j < L.nL; ++j)
      if (m >> j & 1u) out[w++] = pair_code(L.s, -1, j);
  } else {
    if (TECH == 8 && L.k2)
      for (int j = 0; j < L.nL; ++j)
        if (L.neeok >> j & 1u) out[w++] = pair_code(L.s, -1, j);
    const int extra = (TECH == 3 || TECH == 8) ? 4 : 3;
    for (int i = 0; i < L.nE; ++i)
      if (L.camok >> i & 1u)
        for (int j = 0; j < L.nL; ++j)
          if ((L.neeok >> j & 1u) && i + j + extra <= depth) out[w++] = pair_code(L.s, i, j);
  }
}

// Wave-level exclusive prefix sum with one queue reservation per wave.
DEV uint32_t wave_reserve(uint32_t* counter, int c, int& total) {
  const int lane = threadIdx.x & (kWave - 1);
  int x = c;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  total = __shfl(x, kWave - 1, kWave);
  uint32_t base = 0;
  if (lane == kWave - 1 && total > 0) base = atomicAdd(counter, (uint32_t)total);
  base = __shfl(base, kWave - 1, kWave);
  return base + (uint32_t)(x - c);
}

// Instrumented variants: wave-reduced work counters, one atomic per wave and field.
DEV unsigned long long wave_sum(uint32_t x) {
  unsigned long long v = x;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
DEV void flush_work(DevStats* st, int kid, const WorkCount& wc) {
  const bool lead = (threadIdx.x & (kWave - 1)) == 0;
  const unsigned long long n = wave_sum(wc.nodes), t = wave_sum(wc.tris), b = wave_sum(wc.bytes);
  unsigned long long r[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) r[q] = wave_sum(wc.rays[q]);
  if (lead) {
    atomicAdd(&st->nodes, n);
    atomicAdd(&st->tris, t);
    atomicAdd(&st->knodes[kid], n);
    atomicAdd(&st->ktris[kid], t);
    atomicAdd(&st->kbytes[kid], b);
#pragma unroll
    for (int q = 0; q < 6; ++q) atomicAdd(&st->rays[q], r[q]);
  }
}

// The next 64 entries of a queue for this wave (one wave per workgroup):
// waves take work as they finish, which balances uneven per-entry cost.
DEV uint32_t next_batch(uint32_t* counter) {
  uint32_t b = 0;
  if (threadIdx.x == 0) b = atomicAdd(counter, (uint32_t)kTraceBlock);
  return __builtin_amdgcn_readfirstlane(__shfl(b, 0, kWave));
}

// Work item g -> (job, direction) by binary search of the item prefix table.
DEV int find_jd(const int64_t* pre, int n, int64_t g) {
  int lo = 0, hi = n;  // pre[lo] <= g < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The sample a slot of the round holds.  Slots are in item order (item it,
// lane l -> slot it * 64 + l, the sample's index following from the item's
// place in its stream) unless start_order_kernel permuted the round; its
// permutation stays within one (job, direction) stream, so a slot and the
// slot whose sample it holds belong to the same stream.
DEV int64_t slot_sample(const WalkArgs& A, const DevJob& J, int jd, int s) {
  const int so = A.W.order ? (int)A.W.order[s] : s;
  return J.s0 + (A.item0 + so / kItem - A.item_prefix[jd]) * kItem + so % kItem;
}

// Start order: within windows of order_items<t>() items of one (job,
// direction) stream, the round's samples are counting-sorted by a key of
// where they start, so that the lanes of a wave start close together and
// their first rays take similar paths through the BVH.
//   techniques 1-6 and 8: the cell of the start point (x_D on the object, x_G on
//     the ghost, from the sample's first draw as its technique takes it) in a
//     16 x 16 x 16 grid over that object's bounds, cells in Morton order
//     (technique 3: an 8 x 8 x 8 grid under the octant of its first ray's
//     direction);
//   path tracing (7): the pixel, in 8-pixel column groups by row within the
//     window, so that a wave covers an 8 x 8 tile.
// Only the assignment of samples to slots changes: every sample keeps its
// random numbers, and slot_sample follows the permutation.  Windows that
// hold more than one stream keep the item order.  Samples past their
// stream's end go last.  Pass 1 counts the keys (LDS) and keeps them in
// W.okey, then the counts become each key's first place in the window, and
// pass 2 places the slots.
#ifndef RPI_ORDER_ITEMS
#define RPI_ORDER_ITEMS 1024
#endif
constexpr int kOrderBins = 4096;
constexpr int kOrderThreads = 1024;  // one workgroup per window
template <int TECH>
constexpr int order_items() { return TECH == 7 ? 64 : RPI_ORDER_ITEMS; }
DEV uint32_t spread4(uint32_t c) { return (c & 1u) | ((c & 2u) << 2) | ((c & 4u) << 4) | ((c & 8u) << 6); }
DEV uint32_t grid_cell16(float v, float a, float b) {
  const float t = (v - a) / fmaxf(b - a, 1e-30f) * 16.0f;
  return (uint32_t)min(15, max(0, (int)t));
}
template <int TECH>
__global__ __launch_bounds__(kOrderThreads) void start_order_kernel(WalkArgs A) {
  __shared__ uint32_t cnt[kOrderBins], part[kOrderThreads];
  constexpr int kPerThread = kOrderBins / kOrderThreads;
  constexpr int kOrderItems = order_items<TECH>();
  const int nwin = (A.nitems + kOrderItems - 1) / kOrderItems;
  for (int w = blockIdx.x; w < nwin; w += gridDim.x) {
    const int i0 = w * kOrderItems, i1 = min(i0 + kOrderItems, A.nitems);
    const int p0 = i0 * kItem, p1 = i1 * kItem;
    const int jd = find_jd(A.item_prefix, 2 * A.njobs, A.item0 + i0);
    if (find_jd(A.item_prefix, 2 * A.njobs, A.item0 + i1 - 1) != jd) {
      for (int p = p0 + (int)threadIdx.x; p < p1; p += kOrderThreads) A.W.order[p] = (uint32_t)p;
      continue;  // the same for the whole workgroup
    }
    for (int b = threadIdx.x; b < kOrderBins; b += kOrderThreads) cnt[b] = 0u;
    __syncthreads();
    const DevJob& J = A.jobs[jd >> 1];
    const int dir = jd & 1;
    const DevFrame& F = J.F[dir];
    const bool ghost = TECH >= 4 && TECH <= 6;
    const vec3 lo = ghost ? F.glo : F.olo, hi = ghost ? F.ghi : F.ohi;
    const int64_t lim = A.tech_spp ? (int64_t)A.tech_spp * J.W * J.H : J.s1;
    const uint32_t P = (uint32_t)(J.W * J.H);
    const int64_t smp0 = J.s0 + (A.item0 + i0 - A.item_prefix[jd]) * kItem;
    const int y0 = (int)(((uint32_t)smp0 % P) / (uint32_t)J.W);
    const int rows = (kOrderItems * kItem + J.W - 1) / J.W + 1;
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kOrderThreads) {
      const int64_t smp = J.s0 + (A.item0 + p / kItem - A.item_prefix[jd]) * kItem + p % kItem;
      uint32_t kk = kOrderBins - 1;
      if (smp < lim && TECH == 7) {
        const uint32_t pixel = (uint32_t)smp % P;
        const int x = (int)(pixel % (uint32_t)J.W), y = (int)(pixel / (uint32_t)J.W);
        kk = (uint32_t)min((x >> 3) * rows + (y - y0 + J.H) % J.H, kOrderBins - 2);
      } else if (smp < lim) {
        const Rng g{A.k0, A.k1, (uint32_t)smp, ((uint32_t)TECH << 24) | ((uint32_t)dir << 23),
                    A.job_base + (uint32_t)(jd >> 1)};
        float u[4];
        draw(g, 0, 0, 0, u);
        vec3 x, n;
        uint32_t md;
        int tri;
        object_point(J.S, ghost ? F.ghost : F.pose, u, x, n, md, tri);
        kk = spread4(grid_cell16(x.x, lo.x, hi.x)) | (spread4(grid_cell16(x.y, lo.y, hi.y)) << 1) |
             (spread4(grid_cell16(x.z, lo.z, hi.z)) << 2);
        if (TECH == 3) {
          // technique 3's first ray leaves x_D in a cosine-lobe direction:
          // its octant above an 8 x 8 x 8 grid
          draw(g, 0, 0, 2, u);
          const vec3 wd = cosine_dir(n, u[0], u[1]);
          const uint32_t oct = (wd.x < 0.0f ? 1u : 0u) | (wd.y < 0.0f ? 2u : 0u) | (wd.z < 0.0f ? 4u : 0u);
          kk = (oct << 9) | spread4(grid_cell16(x.x, lo.x, hi.x) >> 1) |
               (spread4(grid_cell16(x.y, lo.y, hi.y) >> 1) << 1) | (spread4(grid_cell16(x.z, lo.z, hi.z) >> 1) << 2);
        }
      }
      atomicAdd(&cnt[kk], 1u);
      A.W.okey[p] = (uint16_t)kk;
    }
    __syncthreads();
    {  // exclusive prefix sums: each key's first place in the window (kPerThread keys per thread)
      const int t = threadIdx.x;
      uint32_t sum = 0u;
      for (int q = 0; q < kPerThread; ++q) sum += cnt[kPerThread * t + q];
      part[t] = sum;
      __syncthreads();
      for (int off = 1; off < kOrderThreads; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
      }
      uint32_t run = part[t] - sum;
      for (int q = 0; q < kPerThread; ++q) {
        const uint32_t c = cnt[kPerThread * t + q];
        cnt[kPerThread * t + q] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kOrderThreads)
      A.W.order[p0 + atomicAdd(&cnt[A.W.okey[p]], 1u)] = (uint32_t)p;
    __syncthreads();
  }
}

// Occupancy targets of the trace-heavy kernels (waves per SIMD; 0 leaves the
// register allocation to the compiler).  The 10 KB LDS stack per wave lets a
// compute unit hold 16 waves, four per SIMD.  The start kernels fit four
// without spills.
#ifndef RPI_START_WAVES_PER_EU
#define RPI_START_WAVES_PER_EU 4
#endif
#if RPI_START_WAVES_PER_EU > 0
#define RPI_START_OCCUPANCY __attribute__((amdgpu_waves_per_eu(RPI_START_WAVES_PER_EU)))
#else
#define RPI_START_OCCUPANCY
#endif
// the walk-phase state machine keeps a query and a walk per lane: at 3 waves
// per SIMD (168 VGPRs) it spills less, which pays for the lower occupancy
#ifndef RPI_WALK_WAVES_PER_EU
#define RPI_WALK_WAVES_PER_EU 3
#endif
// the walk phases of techniques 1 and 4 (eye walks only) measure faster at
// 4 waves per SIMD
#ifndef RPI_WALK_WAVES_T14
#define RPI_WALK_WAVES_T14 4
#endif
#define RPI_WALK_OCCUPANCY(T) \
  __attribute__((amdgpu_waves_per_eu((T) == 1 || (T) == 4 ? RPI_WALK_WAVES_T14 : RPI_WALK_WAVES_PER_EU)))
// connect holds a whole path (vertices, crossing sums, pdf tables) in
// registers: 3 waves per SIMD gives it 168 VGPRs and leaves a few spills
#ifndef RPI_CONNECT_WAVES_PER_EU
#define RPI_CONNECT_WAVES_PER_EU 3
#endif
#define RPI_CONNECT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(RPI_CONNECT_WAVES_PER_EU)))

// ------------------------------------------------------------------ walk tasks

DEV float4& TSK(const Workspace& W, int field, uint32_t t) { return W.task[(size_t)field * W.Q + t]; }

DEV void store_walk(const Workspace& W, int f0, uint32_t t, const WalkStart& w) {
  TSK(W, f0, t) = f4u(w.p, w.md);
  TSK(W, f0 + 1, t) = f4u(w.n, (uint32_t)w.lim);
  TSK(W, f0 + 2, t) = make_float4(w.pred.n, w.pred.s0, w.pred.sa, w.pred.sb);
  TSK(W, f0 + 3, t) = f4u(w.end.p, (uint32_t)w.end.kind);
  TSK(W, f0 + 4, t) = f4(w.end.n, 0.0f);
}
DEV WalkStart load_walk(const Workspace& W, int f0, uint32_t t) {
  const float4 a = TSK(W, f0, t), b = TSK(W, f0 + 1, t), c = TSK(W, f0 + 2, t), d = TSK(W, f0 + 3, t),
               e = TSK(W, f0 + 4, t);
  return WalkStart{xyz(a), xyz(b), __float_as_uint(a.w), Cross{c.x, c.y, c.z, c.w},
                   End{xyz(d), xyz(e), (int)__float_as_uint(d.w)}, (int)__float_as_uint(b.w)};
}

// Start phase: persistent waves pull 64-slot work items (job, direction,
// sample range) from a round counter until the round is drained, which
// balances jobs of uneven image size and uneven per-sample cost.  Each lane
// takes the sample its slot holds (slot_sample: in the order the ordering
// pass chose) and draws its technique's start; samples whose walks remain
// are compacted into the task queue (one atomic per wave), so the walk phase
// runs full waves instead of the few lanes whose starts succeeded.
template <int TECH, bool CW>
__global__ __launch_bounds__(kTraceBlock) RPI_START_OCCUPANCY void walk_kernel(WalkArgs A) {
  __shared__ __attribute__((aligned(16))) int stk[kStackDepth * kTraceBlock];
  for (;;) {
    uint32_t it = 0;
    if (threadIdx.x == 0) it = atomicAdd(A.item_counter, 1u);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, kWave));
    if (it >= (uint32_t)A.nitems) break;
    const int64_t g = A.item0 + it;
    const int jd = __builtin_amdgcn_readfirstlane(find_jd(A.item_prefix, 2 * A.njobs, g));
    const DevJob& J = A.jobs[jd >> 1];
    const int dir = jd & 1;
    const int s = (int)it * kItem + threadIdx.x;
    const int64_t smp = slot_sample(A, J, jd, s);
    const bool active = smp < (A.tech_spp ? (int64_t)A.tech_spp * J.W * J.H : J.s1);
    const Ctx C{J.S, J.F[dir], A.W, A.depth};
    Lane L{C, Rng{A.k0, A.k1, (uint32_t)smp, ((uint32_t)TECH << 24) | ((uint32_t)dir << 23), A.job_base + (uint32_t)(jd >> 1)},
           s, stk, WorkCount{}, 0, 0, 0u, 0u, 0u, 0, smp, 0u};
    if (active) {
      if (TECH == 1) tech1<CW>(L);
      if (TECH == 2) tech2<CW>(L);
      if (TECH == 3) tech3<CW>(L);
      if (TECH == 4) tech4<CW>(L);
      if (TECH == 5) tech5<CW>(L);
      if (TECH == 6) tech6<CW>(L);
      if (TECH == 7) tech7<CW>(L);
      if (TECH == 8) tech8<CW>(L);
    }
    // samples with walks left go to the task queue (techniques whose starts
    // fail often), or walk here (those whose walks follow most starts)
    if (!split_walks(TECH) && active) {
      if (L.defer & 1u) light_walk<CW>(L, L.lw.p, L.lw.n, L.lw.md, L.lw.pred, L.lw.end, L.lw.lim, false, TECH == 7);
      if (L.defer & 2u) eye_walk<CW>(L, L.ew.p, L.ew.n, L.ew.md, L.ew.pred, L.ew.end, L.ew.lim);
      L.defer = 0u;
      A.W.counts[s] = (uint32_t)L.nE | ((uint32_t)L.nL << 8);
    }
    const int want = split_walks(TECH) && active && L.defer ? 1 : 0;
    int ntask;
    const uint32_t t = wave_reserve(A.W.ntasks, want, ntask);
    if (want) {
      TSK(A.W, 0, t) = make_float4(__uint_as_float((uint32_t)s), __uint_as_float(L.defer),
                                   __uint_as_float((uint32_t)L.k2), 0.0f);
      if (L.defer & 1u) store_walk(A.W, 1, t, L.lw);
      if (L.defer & 2u) store_walk(A.W, 6, t, L.ew);
    }
    // the others are complete: their paths go out now
    if (split_walks(TECH) && active && !want) A.W.counts[s] = 0u;
    const int c = active && !want ? pair_count<TECH>(L, A.depth) : 0;
    int total;
    const uint32_t at = wave_reserve(A.W.npairs, c, total);
    if (c > 0 && at + (uint32_t)c <= (uint32_t)A.W.pair_cap) write_pairs<TECH>(L, A.W.pairs + at, A.depth);
    if (CW) {
      L.wc.bytes += 4u * (uint32_t)c + (active && !want ? 4u : 0u) +
                    (want ? 16u * (1u + 5u * (uint32_t)__popc(L.defer)) : 0u);
      flush_work(A.stats, kid_start(TECH), L.wc);
    }
  }
}

// ------------------------------------------------------------------ walk phase
// Every lane of a wave runs its own task through a small state machine
// (next-event or camera connection, extension, vertex records) that issues
// one compound ray query at a time:
//   visibility: any hit in the static scene, then in the object at its pose
//     (when the segment meets its box), then, if nothing blocks, the ghost
//     crossings of the same segment;
//   extension: closest hit in the static scene and the object, then the
//     ghost crossings of the new edge.
// One traversal loop serves the queries of all lanes together whatever their
// kind and stage, so lanes whose walk has no query of a given kind do not sit
// out that query, and a lane whose task is done takes the next one from the
// queue.  The arithmetic of each query is that of edge_visible, closest and
// edge_cross.
enum : int { QS_NONE = 0, QS_STAT = 1, QS_OBJ = 2, QS_GHOST = 3 };
enum : int { QK_VIS = 0, QK_EXT = 1 };
enum : int {
  PH_IDLE = 0, PH_LNEE, PH_LNEE_RES, PH_LREC, PH_LEXTEND, PH_LEXT_RES,
  PH_ESTART, PH_ECAM, PH_ECAM_RES, PH_EREC, PH_EEXTEND, PH_EEXT_RES, PH_FIN
};

struct SmQuery {
  int stage, kind;
  int node, sp, pl;
  const float4* nodes;  // BVH of the stage
  const float4* tris;
  vec3 o, d;      // world ray; in the ghost stage the canonical segment
  float tmax;     // segment end, or the closest t so far (extension)
  vec3 ro, rd, inv, oi;  // ray in the frame of the stage's BVH
  int hit;        // visibility: occluded; extension: a closest hit exists
  int noobj;      // the ray leaves the (convex) object it starts on: no object stage
  Cross c;        // ghost crossings; before them, an extension's closest hit
                  // (bits of its id, triangle index and object flag in s0, sa, sb)
};

struct SmLane {
  uint32_t s, defer;
  int jd, ph, j, lim;
  uint32_t smp;      // sample index in its (technique, direction) stream
  vec3 p, n;
  uint32_t md;
  Cross pred;        // crossings into the vertex
  vec3 other;        // light walk: the neighbour towards the camera; eye walk: the point towards the light
  int dyn, ok;
  LightEnd E;        // the light end of the connection; from an extension on, its hit
                     // (p, n and material word in p, n, mat)
  int nE, nL, k2;
  uint32_t camok, neeok, dynpre;
  // Two-sided tasks (techniques 3 and 6): 1 = the eye vertex 0 goes first,
  // 2 = then the light walk, 3 = then the rest of the eye walk; elim: the eye
  // walk's last slot.  A vertex is added only if some connected path could
  // still use it (the pairs need i + j + extra <= depth).
  int order, elim;
};

template <int TECH>
DEV constexpr bool sm_two_sided() {
  return TECH == 3 || TECH == 6;
}
DEV constexpr int pair_extra(int tech) { return (tech == 3 || tech == 8) ? 4 : 3; }
// light vertex j1: an eye vertex i <= depth - extra - j1 that connects (e_0
// is known; later ones might)
DEV bool light_useful(const SmLane& L, int j1, int depth, int extra) {
  const int imax = depth - extra - j1;
  if (imax < 0) return false;
  return (L.camok & 1u) || (imax >= 1 && L.elim >= 1);
}
// eye vertex i1: a light vertex j with a successful connection and i1 + j + extra <= depth
DEV bool eye_useful(const SmLane& L, int i1, int depth, int extra) {
  for (int j = 0; j < L.nL; ++j)
    if ((L.neeok >> j & 1u) && i1 + j + extra <= depth) return true;
  return false;
}

DEV void sm_stage(SmQuery& q, int stage, const DevBvh& B, vec3 ro, vec3 rd) {
  q.stage = stage;
  q.node = ray_ok(ro, rd) ? 0 : kDone;
  q.sp = 0;
  q.pl = 0;
  q.nodes = B.nodes;
  q.tris = B.tris;
  q.ro = ro;
  q.rd = rd;
  q.inv = v3(1.0f / rd.x, 1.0f / rd.y, 1.0f / rd.z);
  q.oi = v3(ro.x * q.inv.x, ro.y * q.inv.y, ro.z * q.inv.z);
}

template <bool CW>
DEV void sm_visibility(SmQuery& q, const DevScene& S, const End& A, const End& B, int ray_type, bool noobj,
                       WorkCount& wc) {
  if (CW) wc.rays[ray_type]++;
  const Seg sg = canon(S, A, B);
  q.kind = QK_VIS;
  q.noobj = noobj ? 1 : 0;
  q.o = sg.o;
  q.d = sg.d;
  q.tmax = sg.tmax;
  q.hit = 0;
  q.c = no_cross();
  sm_stage(q, QS_STAT, S.stat, sg.o, sg.d);
}

template <bool CW>
DEV void sm_extension(SmQuery& q, const DevScene& S, vec3 o, vec3 d, bool noobj, WorkCount& wc) {
  if (CW) wc.rays[RAY_CLOSEST]++;
  q.kind = QK_EXT;
  q.noobj = noobj ? 1 : 0;
  q.o = o;
  q.d = d;
  q.tmax = INFINITY;
  q.hit = 0;
  q.c = Cross{0.0f, __int_as_float(0x7fffffff), __int_as_float(-1), __int_as_float(0)};
  sm_stage(q, QS_STAT, S.stat, o, d);
}

// The next stage of a lane's query once the traversal of its current stage
// has ended (QS_NONE: the query is answered).
template <bool CW>
DEV void sm_next(SmQuery& q, SmLane& L, const DevScene& S, const DevFrame& F, WorkCount& wc) {
  if (q.stage == QS_GHOST) {
    q.stage = QS_NONE;
    return;
  }
  if (q.kind == QK_VIS && q.hit) {  // blocked
    q.stage = QS_NONE;
    return;
  }
  if (q.stage == QS_STAT && !q.noobj && near_object(F, q.o, q.d, q.tmax)) {
    sm_stage(q, QS_OBJ, S.obj, pose_inv_apply(F.pose, q.o), pose_inv_rot(F.pose, q.d));
    return;
  }
  if (q.kind == QK_VIS) {  // visible: the ghost crossings of the same segment
    if (F.ghosts) {
      if (CW) wc.rays[RAY_GHOST]++;
      if (near_ghost(F, q.o, q.d, q.tmax)) {
        sm_stage(q, QS_GHOST, S.obj, pose_inv_apply(F.ghost, q.o), pose_inv_rot(F.ghost, q.d));
        return;
      }
    }
    q.stage = QS_NONE;
    return;
  }
  // extension: the new vertex, then the ghost crossings of the new edge (its
  // end nearer the camera first)
  q.stage = QS_NONE;
  q.noobj = 0;
  if (!q.hit) return;
  const Hit h{q.tmax, __float_as_int(q.c.s0), __float_as_int(q.c.sa), __float_as_int(q.c.sb), 1};
  q.c = no_cross();
  hit_vertex(S, F.pose, h, q.o, q.d, L.E.p, L.E.n, L.E.mat);
  if (interior_hit(S, F, L.E.p, L.E.n, L.E.mat, L.p)) {  // the walk ends inside the object
    q.hit = 0;
    return;
  }
  if (is_emitter(S, L.E.mat) || !F.ghosts) return;
  if (CW) wc.rays[RAY_GHOST]++;
  const bool light = L.ph == PH_LEXT_RES;
  const End A = light ? end_surf(L.p, L.n) : end_surf(L.E.p, L.E.n);
  const End B = light ? end_surf(L.E.p, L.E.n) : end_surf(L.p, L.n);
  const Seg sg = canon(S, A, B);
  if (!near_ghost(F, sg.o, sg.d, sg.tmax)) return;
  q.o = sg.o;
  q.d = sg.d;
  q.tmax = sg.tmax;
  sm_stage(q, QS_GHOST, S.obj, pose_inv_apply(F.ghost, sg.o), pose_inv_rot(F.ghost, sg.d));
}

// Ends a, b of the line along which a ghost-started technique generates the
// edge of the lane's query (as edge_cross takes them from the edge's ends).
DEV void sm_line(const SmLane& L, const DevScene& S, vec3& a, vec3& b, int& env) {
  env = 0;
  if (L.ph == PH_LNEE_RES) {  // x_j -> light point (offset) or environment
    a = L.p;
    env = L.E.env;
    b = env ? L.p : spawn(S, L.E.p, L.E.n, L.p);
  } else if (L.ph == PH_ECAM_RES) {  // pinhole -> x_i
    a = S.cam.eye;
    b = L.p;
  } else if (L.ph == PH_LEXT_RES) {  // x_j -> new vertex
    a = L.p;
    b = L.E.p;
  } else {  // new vertex -> x_i
    a = L.E.p;
    b = L.p;
  }
}

// Triangle i of a leaf for the lane's query; true ends the stage (any hit).
template <bool CW>
DEV bool sm_triangle(SmQuery& q, const SmLane& L, const DevScene& S, const DevFrame& F, int i, WorkCount& wc) {
  vec3 v0, e1, e2;
  int id, mat;
  load_tri(q.tris, i, v0, e1, e2, id, mat);
  if (CW) wc.tris++;
  const float t = tri_t(q.ro, q.rd, v0, e1, e2);
  if (q.stage == QS_GHOST) {
    if (!(t > 0.0f && t < q.tmax)) return false;
    vec3 g = q.o + q.d * t;
    q.c.n += 1.0f;
    vec3 a, b;
    int env;
    sm_line(L, S, a, b, env);
    if (!env) {
      // density only where the generating line itself crosses the triangle
      const vec3 la = pose_inv_apply(F.ghost, a), ld = pose_inv_rot(F.ghost, b - a);
      const float tl = tri_t(la, ld, v0, e1, e2);
      if (!(tl > 0.0f && tl < 1.0f)) return false;
      g = a + (b - a) * tl;
    }
    const vec3 u = env ? unit(q.d) : unit(b - a);
    const vec3 ng = pose_rot(F.ghost, unit(cross(e1, e2)));
    const float cg = fabsf(dot(ng, u));
    q.c.s0 += 1.0f / cg;
    q.c.sa += len2(g - a) / cg;
    q.c.sb += env ? 0.0f : len2(g - b) / cg;
    return false;
  }
  if (q.kind == QK_VIS) {
    if (t > 0.0f && t < q.tmax) {
      q.hit = 1;
      return true;
    }
    return false;
  }
  if (t > 0.0f && (t < q.tmax || (t == q.tmax && id < __float_as_int(q.c.s0)))) {
    q.tmax = t;
    q.c.s0 = __int_as_float(id);
    q.c.sa = __int_as_float(i);
    q.c.sb = __int_as_float(q.stage == QS_OBJ ? 1 : 0);
    q.hit = 1;
  }
  return false;
}

DEV Rng sm_rng(const WalkArgs& A, const SmLane& L, int tech) {
  return Rng{A.k0, A.k1, L.smp, ((uint32_t)tech << 24) | ((uint32_t)(L.jd & 1) << 23),
             A.job_base + (uint32_t)(L.jd >> 1)};
}

template <int TECH>
DEV void sm_begin(const WalkArgs& A, SmLane& L, uint32_t t) {
  const float4 h = TSK(A.W, 0, t);
  L.s = __float_as_uint(h.x);
  L.defer = __float_as_uint(h.y);
  L.k2 = (int)__float_as_uint(h.z);
  const int64_t g = A.item0 + L.s / kItem;
  L.jd = find_jd(A.item_prefix, 2 * A.njobs, g);
  L.smp = (uint32_t)slot_sample(A, A.jobs[L.jd >> 1], L.jd, (int)L.s);
  L.nE = L.nL = 0;
  L.camok = L.neeok = L.dynpre = 0u;
  L.ph = PH_ESTART;
  L.order = 0;
  L.elim = 0;
  if (sm_two_sided<TECH>() && (L.defer & 3u) == 3u) {
    L.order = 1;  // the eye vertex 0 first
    return;
  }
  if (L.defer & 1u) {
    const WalkStart w = load_walk(A.W, 1, t);
    L.p = w.p;
    L.n = w.n;
    L.md = w.md;
    L.pred = w.pred;
    L.other = w.end.p;
    L.lim = w.lim;
    L.j = 0;
    L.dyn = 0;
    L.ph = PH_LNEE;
  }
}

// One pass of a lane's walk: it takes its query's answer, moves to the next
// vertex or walk, and issues its next query, or finishes.  Each block below
// runs once per pass for all lanes that need it (one random draw, one light
// sample, one BSDF sample per pass), so lanes in different parts of their
// walks share the code instead of taking one branch each.
template <int TECH, bool CW>
DEV void sm_step(const WalkArgs& A, SmLane& L, SmQuery& q, uint32_t t, WorkCount& wc) {
  const DevJob& J = A.jobs[L.jd >> 1];
  const DevScene& S = J.S;
  const DevFrame& F = J.F[L.jd & 1];
  const Workspace& W = A.W;
  const int s = (int)L.s;
  // answers: visibility of a connection, or the next vertex of a walk
  if (L.ph == PH_LNEE_RES || L.ph == PH_ECAM_RES) {
    L.ok = q.hit ? 0 : 1;
    if (q.hit) q.c = no_cross();
    L.ph = L.ph == PH_LNEE_RES ? PH_LREC : PH_EREC;
  } else if (L.ph == PH_LEXT_RES || L.ph == PH_EEXT_RES) {
    const bool light = L.ph == PH_LEXT_RES;
    if (!q.hit || is_emitter(S, L.E.mat)) {
      L.ph = light ? PH_ESTART : PH_FIN;
      if (light && L.order == 2) L.order = 3;
    } else {
      L.pred = q.c;
      // component copies: a struct copy inside the lane state keeps the
      // compiler from holding it in registers
      L.other.x = L.p.x;
      L.other.y = L.p.y;
      L.other.z = L.p.z;
      L.p.x = L.E.p.x;
      L.p.y = L.E.p.y;
      L.p.z = L.E.p.z;
      L.n.x = L.E.n.x;
      L.n.y = L.E.n.y;
      L.n.z = L.E.n.z;
      L.md = L.E.mat;
      L.j += 1;
      L.ph = light ? PH_LNEE : PH_ECAM;
    }
  }
  if (L.ph == PH_ESTART) {
    L.ph = PH_FIN;
    if (L.defer & 2u) {
      const WalkStart w = load_walk(W, 6, t);
      L.p = w.p;
      L.n = w.n;
      L.md = w.md;
      L.pred = w.pred;
      // the point towards the light: the neighbour, or a point along the
      // environment direction
      L.other = w.end.kind == END_ENV ? L.p + w.end.n : w.end.p;
      L.lim = w.lim;
      L.elim = w.lim;
      L.j = 0;
      // resumed after the light walk: its vertex 0 is connected and recorded
      L.ph = L.order == 3 ? PH_EEXTEND : PH_ECAM;
    }
  }
  // connections: next-event estimation (light walk), camera (eye walk)
  if (L.ph == PH_LNEE || L.ph == PH_ECAM) {
    q.c = no_cross();  // the connection's crossings (none unless it is traced)
    L.ok = 0;
    bool go, noobj = false;
    End ea, eb;
    int rt;
    if (L.ph == PH_LNEE) {
      L.dyn = L.dyn || (L.md & kDynBit) || L.pred.n > 0.0f;
      float u[4];
      draw(sm_rng(A, L, TECH), 0, L.j + 1, 1, u);
      L.E = LightEnd{v3(0, 0, 0), v3(0, 0, 0), 0u, 0};
      go = sample_light(S, u, L.E);
      if (go)
        go = L.E.env ? same_side_dir(L.n, L.p, L.other, L.E.n)
                     : (dot(L.E.n, L.p - L.E.p) > 0.0f && same_side(L.n, L.p, L.other, L.E.p));
      ea = end_surf(L.p, L.n);
      eb = end_light(L.E);
      rt = RAY_SHADOW;
      if (go && (L.md & kDynBit))
        noobj = leaves_convex(S, F.pose, L.p, L.n, L.E.env ? L.E.n : L.E.p - L.p);
      L.ph = go ? PH_LNEE_RES : PH_LREC;
    } else {
      go = raster(S.cam, L.p) >= 0 && same_side(L.n, L.p, S.cam.eye, L.other);
      ea = end_eye(S);
      eb = end_surf(L.p, L.n);
      rt = RAY_CAMERA;
      if (go && (L.md & kDynBit)) noobj = leaves_convex(S, F.pose, L.p, L.n, S.cam.eye - L.p);
      L.ph = go ? PH_ECAM_RES : PH_EREC;
    }
    if (go) {
      sm_visibility<CW>(q, S, ea, eb, rt, noobj, wc);
      return;
    }
  }
  // vertex records, then the extension
  if (L.ph == PH_LREC || L.ph == PH_EREC) {
    const bool light = L.ph == PH_LREC;
    const int j = L.j;
    if (light) {
      LIT(W, j, 0, s) = f4u(L.p, L.md);
      LIT(W, j, 1, s) = f4(L.n, L.pred.n);
      LIT(W, j, 2, s) = make_float4(L.pred.s0, L.pred.sa, L.pred.sb, 0.0f);
      LIT(W, j, 3, s) = f4u(L.E.p, light_word(L.E));
      LIT(W, j, 4, s) = f4(L.E.n, q.c.n);
      LIT(W, j, 5, s) = make_float4(q.c.s0, q.c.sa, q.c.sb, 0.0f);
      if (CW) wc.bytes += kLightFields * 16;
      if (L.dyn || q.c.n > 0.0f) L.dynpre |= 1u << j;
    } else {
      EYE(W, j, 0, s) = f4u(L.p, L.md);
      EYE(W, j, 1, s) = f4(L.n, L.pred.n);
      EYE(W, j, 2, s) = make_float4(L.pred.s0, L.pred.sa, L.pred.sb, 0.0f);
      EYE(W, j, 3, s) = make_float4(q.c.n, q.c.s0, q.c.sa, q.c.sb);
      if (CW) wc.bytes += kEyeFields * 16;
    }
    // (selects rather than branches: a store through a chosen field keeps
    // the lane state out of registers)
    const uint32_t bit = L.ok ? 1u << j : 0u;
    L.nL = light ? j + 1 : L.nL;
    L.nE = light ? L.nE : j + 1;
    L.neeok |= light ? bit : 0u;
    L.camok |= light ? 0u : bit;
    L.ph = light ? PH_LEXTEND : PH_EEXTEND;
  }
  // the extension, if a connected path could use the next vertex
  if (L.ph == PH_LEXTEND || L.ph == PH_EEXTEND) {
    const bool light = L.ph == PH_LEXTEND;
    const int j = L.j;
    if (!light && L.order == 1) {  // eye vertex 0 done: now the light walk
      const WalkStart w = load_walk(W, 1, t);
      L.p = w.p;
      L.n = w.n;
      L.md = w.md;
      L.pred = w.pred;
      L.other = w.end.p;
      L.lim = w.lim;
      L.j = 0;
      L.dyn = 0;
      L.order = 2;
      L.ph = PH_LNEE;
      return;
    }
    bool ext = j < L.lim;
    if (sm_two_sided<TECH>() && ext) {
      if (light && L.order == 2) ext = light_useful(L, j + 1, A.depth, pair_extra(TECH));
      if (!light && L.order == 3) ext = eye_useful(L, j + 1, A.depth, pair_extra(TECH));
    }
    L.ph = light ? PH_ESTART : PH_FIN;
    if (ext) {
      float u[4];
      draw(sm_rng(A, L, TECH), light ? 0u : 1u, j + 1, 0, u);
      vec3 wo;
      if (bsdf_sample(vmat(S, F, L.md), L.n, unit(L.other - L.p), u[0], u[1], wo)) {
        sm_extension<CW>(q, S, spawn_dir(S, L.p, L.n, wo), wo,
                         (L.md & kDynBit) && leaves_convex(S, F.pose, L.p, L.n, wo), wc);
        L.ph = light ? PH_LEXT_RES : PH_EEXT_RES;
      }
    }
    if (L.ph == PH_ESTART && L.order == 2) L.order = 3;  // the light walk ends here
  }
}

#ifndef RPI_SM_REFILL
#define RPI_SM_REFILL 32
#endif

// Walk phase: persistent waves; see the state machine above.  Lanes hand the
// wave their finished tasks' connected paths with one queue reservation per
// wave and take new tasks with one counter update per wave.
template <int TECH, bool CW>
__global__ __launch_bounds__(kTraceBlock) RPI_WALK_OCCUPANCY(TECH) void walk_task_kernel(WalkArgs A) {
  __shared__ __attribute__((aligned(16))) int stk[kStackDepth * kTraceBlock];
  const int lane = threadIdx.x;
  const uint32_t n = min(*A.W.ntasks, (uint32_t)A.W.Q);
  WorkCount wc{};
  SmLane L;
  L.ph = PH_IDLE;
  SmQuery q;
  q.stage = QS_NONE;
  q.node = kDone;
  q.pl = 0;
  uint32_t t = 0;
  bool drained = false;
  for (;;) {
    // connected paths of the finished tasks
    const unsigned long long fin = __ballot(L.ph == PH_FIN);
    if (fin) {
      const bool f = L.ph == PH_FIN;
      const int c = f ? pair_count<TECH>(L, A.depth) : 0;
      int total;
      const uint32_t at = wave_reserve(A.W.npairs, c, total);
      if (c > 0 && at + (uint32_t)c <= (uint32_t)A.W.pair_cap) write_pairs<TECH>(L, A.W.pairs + at, A.depth);
      if (f) {
        A.W.counts[L.s] = (uint32_t)L.nE | ((uint32_t)L.nL << 8);
        if (CW) wc.bytes += 4u * (uint32_t)c + 4u;
        L.ph = PH_IDLE;
      }
    }
    // idle lanes take the next tasks
    if (!drained) {
      const unsigned long long idle = __ballot(L.ph == PH_IDLE);
      if (idle) {
        const uint32_t k = (uint32_t)__popcll(idle);
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&A.W.fetch[0], k);
        base = __builtin_amdgcn_readfirstlane(__shfl(base, 0, kWave));
        if (base + k >= n) drained = true;
        if (L.ph == PH_IDLE) {
          t = base + (uint32_t)__popcll(idle & ((1ull << lane) - 1ull));
          if (t < n) sm_begin<TECH>(A, L, t);
        }
      }
    }
    // every lane steps its walk until it has a query pending or its task is done
    while (L.ph != PH_IDLE && L.ph != PH_FIN && q.stage == QS_NONE) sm_step<TECH, CW>(A, L, q, t, wc);
    if (__ballot(q.stage != QS_NONE) == 0ull) {
      if (drained && __ballot(L.ph != PH_IDLE) == 0ull) break;
      continue;
    }
    // the queries of all lanes, stage by stage, until every one is answered
    for (;;) {
      if (q.stage != QS_NONE && q.node == kDone && q.pl == 0) {
        const DevJob& J = A.jobs[L.jd >> 1];
        sm_next<CW>(q, L, J.S, J.F[L.jd & 1], wc);
      }
      // back to the walks when few lanes still trace, so that the others
      // can take their next queries (all of them once the queue is drained)
      if (__popcll(__ballot(q.stage != QS_NONE)) <= (drained ? 0 : RPI_SM_REFILL)) break;
      while (q.stage != QS_NONE && (uint32_t)q.node < (uint32_t)kDone) {
        if (CW) wc.nodes++;
        q.node = visit4(q.nodes, q.node, stk, q.sp, [&](float lx, float ly, float lz, float hx, float hy, float hz,
                                                        float& tn) {
          return slab(lx, ly, lz, hx, hy, hz, q.inv, q.oi, q.tmax, tn);
        });
        if (q.node < 0 && q.pl == 0) {  // postpone the first leaf and go on with the stack
          q.pl = q.node;
          q.node = q.sp > 0 ? stk[--q.sp * kTraceBlock + lane] : kDone;
        }
        if (__ballot(q.pl == 0) == 0ull) break;  // every lane still here holds a leaf
      }
      while (q.pl < 0) {
        const DevJob& J = A.jobs[L.jd >> 1];
        const DevScene& S = J.S;
        const DevFrame& F = J.F[L.jd & 1];
        const int f0 = leaf_first(q.pl), cnt = leaf_count(q.pl);
        bool stop = false;
        for (int i = f0; i < f0 + cnt; ++i)
          if (sm_triangle<CW>(q, L, S, F, i, wc)) {
            stop = true;
            break;
          }
        q.pl = 0;
        if (stop) {
          q.node = kDone;
          break;
        }
        if (q.node < 0) {
          q.pl = q.node;
          q.node = q.sp > 0 ? stk[--q.sp * kTraceBlock + lane] : kDone;
        }
      }
    }
  }
  if (CW) flush_work(A.stats, kid_walk(TECH), wc);
}

// Technique (8), first half: x_D by area, the proposal at x_D (one MLP pass
// per wave on the matrix cores) and the light-side direction drawn from its
// vMF mixture (made defensive by a uniform-sphere component), into start records 0 (x_D, material), 1 (normal) and 3 (the
// direction) of the sample's slot; walk_kernel<8> continues from there.
// Slots hold the samples slot_sample gives them, as in the walk kernel.
__global__ __launch_bounds__(kTraceBlock) void t8_start_kernel(WalkArgs A) {
  __shared__ __attribute__((aligned(16))) float lds[kMlpLdsBytes / 4];
  for (uint32_t it = blockIdx.x; it < (uint32_t)A.nitems; it += gridDim.x) {
    const int64_t g = A.item0 + it;
    const int jd = __builtin_amdgcn_readfirstlane(find_jd(A.item_prefix, 2 * A.njobs, g));
    const DevJob& J = A.jobs[jd >> 1];
    const int dir = jd & 1;
    const DevFrame& F = J.F[dir];
    const int s = (int)it * kItem + threadIdx.x;
    const int64_t smp = slot_sample(A, J, jd, s);
    const bool active = smp < (A.tech_spp ? (int64_t)A.tech_spp * J.W * J.H : J.s1);
    const Rng rng{A.k0, A.k1, (uint32_t)smp, (8u << 24) | ((uint32_t)dir << 23), A.job_base + (uint32_t)(jd >> 1)};
    float x[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    vec3 p = v3(0.f, 0.f, 0.f), n = v3(0.f, 0.f, 1.f);
    uint32_t md = 0u;
    float u[4];
    if (active) {
      draw(rng, 0, 0, 0, u);
      int tri;
      object_point(J.S, F.pose, u, p, n, md, tri);
      mlp_input(A.mlp, pose_inv_apply(F.pose, p), pose_inv_rot(F.pose, n), x);
    }
    const float* raw = mlp_forward_wave(A.mlp, x, lds);
    if (active) {
      draw(rng, 0, 0, 2, u);
      const vec3 wl = unit(pose_rot(F.pose, t8_dir_sample(raw, u[0], u[1], u[2])));
      STA(A.W, 0, s) = f4u(p, md);
      STA(A.W, 1, s) = f4(n, 0.0f);
      STA(A.W, 3, s) = f4(wl, 0.0f);
    }
    __syncthreads();  // the next item's pass overwrites the outputs
  }
}

// ------------------------------------------------------------------ connect
struct PV {
  vec3 p, n;
  uint32_t md;
};

DEV vec3 lpos(const LightEnd& E, vec3 from) { return E.env ? from + E.n : E.p; }

// Component selects.  A conditional over two lvalues selects an address; over
// the vertex array that keeps the array in scratch memory.
DEV vec3 pick(bool c, const vec3& a, const vec3& b) { return v3(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z); }
DEV PV pick(bool c, const PV& a, const PV& b) { return PV{pick(c, a.p, b.p), pick(c, a.n, b.n), c ? a.md : b.md}; }


// Path vertex q (1 <= q <= number of scattering vertices) of connected path
// (s, i, j): eye slots i..0, then the start vertex x_D (techniques 2, 3, 8),
// then light slots 0..j.
DEV PV path_vertex(const Workspace& W, int s, int i, bool mid, int q) {
  float4 a, b;
  if (q <= i + 1) {
    a = EYE(W, i + 1 - q, 0, s);
    b = EYE(W, i + 1 - q, 1, s);
  } else if (mid && q == i + 2) {
    a = STA(W, 0, s);
    b = STA(W, 1, s);
  } else {
    const int bb = q - (i + 1) - (mid ? 1 : 0) - 1;
    a = LIT(W, bb, 0, s);
    b = LIT(W, bb, 1, s);
  }
  return PV{xyz(a), xyz(b), __float_as_uint(a.w)};
}
DEV bool has_mid(int tech) { return tech == 2 || tech == 3 || tech == 8; }

// Proposal training record of a technique-(3) path: the MLP input at x_D, the
// light-side direction in object space, and |residual contribution| / p_gen.
struct TrainRec {
  float x[6], w[3], weight;
};

// What the evaluation of one connected path sees.
struct CCtx {
  const DevScene& S;
  const DevFrame& F;
  const DevFrame& Fp;
  const Workspace& W;
  int tech, material_mode;
  uint32_t mask;
  float sigma, cweight, inv_n, alpha_min, d_min, jac_max;
  int job;
  const MlpDev* mlp;  // training-record input normalisation (collection on), else null
  int train_weighting;
  int no_mapping;     // the path-mapping ablation: every pair rejected
  const float* ratio; // [8]: samples of technique t / the base count (balance heuristic over unequal counts)
};

// q8a, q8b: the proposal's densities at x_1..x_4 and x_5 (technique (8) in the mask).
// BAL: accepted pairs weighted by the balance heuristic over the strategies of
// both directions (the mapped path's strategy sum in the other frame) instead
// of the fixed two-way weight.
template <bool CW, bool BAL>
DEV void connect_one(const CCtx& A, uint32_t code, float4 q8a, float4 q8b, int* stk, WorkCount& wc, float4& rec,
                     int& reason, TrainRec& tr) {
  const DevScene& S = A.S;
  const Workspace& W = A.W;
  const int s = code_slot(code);
  const int i = code_i(code);
  const int j = code_j(code);
  const int T = A.tech;
  const bool mid = has_mid(T);
  const int nsc = (i + 1) + (mid ? 1 : 0) + (j + 1);  // scattering vertices
  const int k = nsc + 2;
  reason = 0;
  rec = make_float4(__int_as_float(-1), 0.f, 0.f, 0.f);
  tr.weight = 0.0f;

  // ---- assemble x_0 .. x_{k-1}
  PV v[kMaxK] = {};  // entries past the last scattering vertex stay zero (the
                     // selects below read them and never take them)
  // edge crossings: bit a of exm marks a crossed edge a; exw[a] is the one sum
  // the ghost densities of that edge use (s_b at the light end, s_a at the eye
  // edge, s_0 between)
  float exw[kMaxK];
  uint32_t exm = 0u;
  v[0] = PV{S.cam.eye, S.cam.fwd, 0u};
#pragma unroll
  for (int q = 1; q < kMaxK - 1; ++q) {
    if (q > nsc) break;
    v[q] = path_vertex(W, s, i, mid, q);
  }
  LightEnd E;
  {
    float4 a, b;
    if (j >= 0) {
      a = LIT(W, j, 3, s);
      b = LIT(W, j, 4, s);
    } else {
      a = STA(W, 3, s);
      b = STA(W, 4, s);
    }
    const uint32_t w = __float_as_uint(a.w);
    E.p = xyz(a);
    E.n = xyz(b);
    E.env = (w & 0x40000000u) ? 1 : 0;
    E.mat = w & 0x3fffffffu;
  }
  // edge crossing records in path order
  const bool motion = !A.material_mode;
#pragma unroll
  for (int a = 0; a < kMaxK - 1; ++a) {
    exw[a] = 0.0f;
    if (a > k - 2 || !motion) continue;
    float4 r1, r2;  // crossing record: count in r1.w, sums in r2.xyz
    if (a == 0 && k == 2) {
      r1 = STA(W, 1, s);
      r2 = STA(W, 2, s);
    } else if (a == 0) {
      if (i >= 0) {
        const float4 c = EYE(W, i, 3, s);
        exw[a] = a == k - 2 ? c.w : c.z;
        exm |= c.x > 0.0f ? 1u : 0u;
        continue;
      } else if (mid) {
        r1 = STA(W, 1, s);
        r2 = STA(W, 2, s);
      } else {
        r1 = LIT(W, 0, 1, s);
        r2 = LIT(W, 0, 2, s);
      }
    } else if (a == k - 2) {
      if (j >= 0) {
        r1 = LIT(W, j, 4, s);
        r2 = LIT(W, j, 5, s);
      } else {
        r1 = EYE(W, 0, 1, s);
        r2 = EYE(W, 0, 2, s);
      }
    } else if (a <= i + 1) {
      r1 = EYE(W, i + 1 - a, 1, s);
      r2 = EYE(W, i + 1 - a, 2, s);
    } else if (mid && a == i + 2) {
      r1 = LIT(W, 0, 1, s);
      r2 = LIT(W, 0, 2, s);
    } else {
      const int bb = a - (i + 1) - (mid ? 1 : 0);  // edge (light[bb-1], light[bb])
      r1 = LIT(W, bb, 1, s);
      r2 = LIT(W, bb, 2, s);
    }
    exw[a] = a == k - 2 ? r2.z : (a == 0 ? r2.y : r2.x);
    exm |= r1.w > 0.0f ? 1u << a : 0u;
  }
  // records read: the path code, two float4 per scattering vertex, two for
  // the light end, up to two per edge's crossing record
  if (CW) wc.bytes += 4u + 32u * (uint32_t)nsc + 32u + (motion ? 32u * (uint32_t)(k - 1) : 0u);

  const DevCamera& C = S.cam;
  const float P = (float)(C.W * C.H);
  // ---- pixel and camera factor W_j G(x0, x1) (shared by the mapped path)
  int pixel;
  float camf, pcam;
  if (k == 2) {
    if (E.env) {
      pixel = raster(C, C.eye + E.n);
      pcam = camera_geo_dir(C, E.n);
    } else {
      pixel = raster(C, E.p);
      pcam = camera_geo(C, E.p, E.n);
    }
  } else {
    pixel = raster(C, v[1].p);
    pcam = camera_geo(C, v[1].p, v[1].n);
  }
  camf = P * pcam;
  if (pixel < 0) {
    reason = 7;
    return;
  }
  const vec3 Le = light_Le(S, E);


  // ---- f in frame F with vertex `sub` replaced by y (sub = 0: none)
  auto rest = [&](const DevFrame& F, int sub, const PV& y) -> vec3 {
    vec3 f = v3(1.f, 1.f, 1.f);
#pragma unroll
    for (int q = 1; q < kMaxK - 1; ++q) {
      if (q > k - 2) break;
      const PV cur = pick(q == sub, y, v[q]);
      const vec3 pp = pick(q - 1 == sub, y.p, v[q - 1].p);
      const bool last = q + 1 == k - 1;
      const PV nx = pick(q + 1 == sub, y, v[q + 1]);
      const bool envn = last && E.env;
      const vec3 pn = pick(last, lpos(E, cur.p), nx.p);
      const vec3 nn = pick(last, E.n, nx.n);
      const Material m = vmat(S, F, cur.md);
      const vec3 wi = unit(pp - cur.p), wo = envn ? E.n : unit(pn - cur.p);
      const vec3 rho = bsdf_eval(m, cur.n, wi, wo);
      float g;
      if (envn) {
        g = fabsf(dot(cur.n, wo));
      } else {
        const vec3 d = pn - cur.p;
        const vec3 w = unit(d);
        g = fabsf(dot(cur.n, w)) * fabsf(dot(nn, w)) / len2(d);
      }
      f = vmul(f, rho) * g;
    }
    return vmul(f, Le);
  };

  const vec3 fx = (k == 2 ? Le : rest(A.F, 0, v[0])) * camf;

  // ---- MIS (Sec. 4.3): forward/backward pdf tables
  const float pL = light_pdf(S, E.env);
  const float pD = S.inv_obj_area;
  // the last scattering vertex x_{k-2}, picked with constant indices (an index
  // that depends on k would keep the vertex array in scratch memory)
  PV vl = v[0];
#pragma unroll
  for (int q = 1; q < kMaxK - 1; ++q)
    if (q == k - 2) vl = v[q];
  auto origin = [&](int r, int q) -> vec3 {  // ray origin generating q from r
    const vec3 to = q == k - 1 ? lpos(E, vl.p) : v[q].p;
    if (r == 0) return C.eye;
    if (r == k - 1) return spawn(S, E.p, E.n, to);
    return spawn(S, v[r].p, v[r].n, to);
  };
  auto to_area = [&](int r, int q, vec3 o) -> float {
    if (q == k - 1 && E.env) return 1.0f;
    const vec3 d = pick(q == k - 1, E.p, v[q].p) - o;
    const vec3 nq = pick(q == k - 1, E.n, v[q].n);
    return fabsf(dot(nq, unit(d))) / len2(d);
  };
  auto dir_from = [&](int r, int q) -> vec3 {  // unit direction r -> q between path vertices
    if (q == k - 1 && E.env) return E.n;
    if (r == k - 1 && E.env) return -E.n;
    const vec3 a = pick(r == 0, C.eye, pick(r == k - 1, E.p, v[r].p));
    const vec3 b = pick(q == 0, C.eye, pick(q == k - 1, E.p, v[q].p));
    return unit(b - a);
  };
  // vertex-generation pdf: vertex q from r by BSDF sampling at r, incoming from o
  auto gen = [&](int r, int q, int inc) -> float {
    const Material m = vmat(S, A.F, v[r].md);
    vec3 og = origin(r, q);
    const vec3 wo = (q == k - 1 && E.env) ? E.n : unit(pick(q == k - 1, E.p, v[q].p) - og);
    return bsdf_pdf(m, v[r].n, dir_from(r, inc), wo) * to_area(r, q, og);
  };
  // The strategy densities of the path in v[] (crossing records exm/exw,
  // camera density pcam): the forward/backward tables and the MIS sum.
  float pgen = 0.0f;  // techniques (2), (3): density of the generating strategy
  auto mis_sum = [&](bool first) -> float {
    float Apre[kMaxK], Bsuf[kMaxK + 1];
    Apre[0] = 1.0f;
  #pragma unroll
    for (int q = 1; q < kMaxK; ++q) Apre[q] = Apre[q - 1];
  #pragma unroll
    for (int q = 1; q <= kMaxK - 3; ++q)
      if (q <= k - 3) Apre[q] = Apre[q - 1] * gen(q + 1, q, q + 2);
  #pragma unroll
    for (int q = kMaxK; q >= 0; --q) Bsuf[q] = 1.0f;
  #pragma unroll
    for (int q = kMaxK - 2; q >= 2; --q) Bsuf[q] = (q <= k - 2) ? Bsuf[q + 1] * gen(q - 1, q, q - 2) : 1.0f;
    auto on = [&](int t) { return (A.mask >> (t - 1)) & 1u; };
    // each strategy's density weighs by its sample count relative to the base
    // count (the balance heuristic over unequal counts; 1 when they are equal)
    const float* rt = A.ratio;
    float sum = 0.0f;
    if (on(7)) sum += rt[6] * (k == 2 ? pcam : pcam * Bsuf[2] * pL);
  #pragma unroll
    for (int m = 1; m < kMaxK - 1; ++m) {
      if (m > k - 2 || !(v[m].md & kDynBit)) continue;
      if (m == k - 2) {
        if (on(1)) sum += rt[0] * (pL * pD * Apre[m - 1]);
      } else if (m == 1) {
        if (on(2) && k >= 4) {
          const float t2 = pD * Bsuf[2] * pL;
          sum += rt[1] * t2;
          if (first && T == 2) pgen = t2;
        }
        if (on(8)) sum += rt[7] * (pD * q8a.x * to_area(1, 2, origin(1, 2)) * Bsuf[3] * pL);
      } else if (on(3) || on(8)) {
        const vec3 o = origin(m, m + 1);
        const vec3 w = unit(v[m + 1].p - o);
        const float rest3 = to_area(m, m + 1, o) * Apre[m - 1] * Bsuf[m + 2] * pL;
        const float c = dot(v[m].n, w);
        if (on(3) && c > 0.0f) {
          const float t3 = pD * (c / kPi) * rest3;
          sum += rt[2] * t3;
          if (first && T == 3 && m == i + 2) pgen = t3;
        }
        if (on(8)) sum += rt[7] * (pD * (m == 2 ? q8a.y : m == 3 ? q8a.z : m == 4 ? q8a.w : q8b.x) * rest3);
      }
    }
    if (motion && k >= 3) {
      const float pG = pD;
      const float pdir = 1.0f / (4.0f * kPi);
  #pragma unroll
      for (int a = 0; a < kMaxK - 1; ++a) {
        if (a > k - 2 || !((exm >> a) & 1u)) continue;
        if (a == k - 2) {
          if (on(4) && !E.env) {
            const vec3 o = spawn(S, E.p, E.n, vl.p);  // the offset light point generating x_{k-2}
            const vec3 d = vl.p - o;
            float ak = Apre[0];
  #pragma unroll
            for (int q = 1; q < kMaxK; ++q)
              if (q == k - 3) ak = Apre[q];
            sum += rt[3] * (pL * pG * exw[a] * fabsf(dot(vl.n, unit(d))) / len2(d) * ak);
          }
        } else if (a == 0) {
          if (on(5)) {
            const vec3 d = v[1].p - C.eye;
            sum += rt[4] * (pG * exw[a] * fabsf(dot(v[1].n, unit(d))) / len2(d) * Bsuf[2] * pL);
          }
        } else if (on(6)) {
          const vec3 d = v[a + 1].p - v[a].p;
          const vec3 w = unit(d);
          const float G = fabsf(dot(v[a].n, w)) * fabsf(dot(v[a + 1].n, w)) / len2(d);
          sum += rt[5] * (pG * pdir * G * exw[a] * Apre[a > 0 ? a - 1 : 0] * Bsuf[a + 2] * pL);
        }
      }
    }
    return sum;
  };
  const float sum = mis_sum(true);
  float denom = sum;  // the balance heuristic's denominator of this path's value
  if (!(sum > 0.0f)) {
    reason = 8;
    return;
  }

  // ---- path mapping and rejection (Sec. 5)
  vec3 val;
  if (A.material_mode) {
    val = (fx - (k == 2 ? Le : rest(A.Fp, 0, v[0])) * camf) * A.cweight;
  } else {
    int rej = 0;
    PV y = v[0];
    int istar = 0;
    const DevFrame& Fp = A.Fp;
    if (A.no_mapping) {
      rej = 9;  // the path-mapping ablation: every path keeps its own frame's term
    } else if (k <= 2) {
      rej = 1;
    } else if (A.F.same_pose) {
#pragma unroll
      for (int a = 0; a < kMaxK - 1; ++a)
        if (a <= k - 2 && ((exm >> a) & 1u)) rej = 5;
    } else {
      const bool retrace = (v[1].md & kDynBit) || (exm & 1u);
      int moved = retrace ? 1 : 0;
      istar = retrace ? 1 : 0;
#pragma unroll
      for (int q = 2; q < kMaxK - 1; ++q)
        if (q <= k - 2 && (v[q].md & kDynBit)) {
          ++moved;
          istar = q;
        }
      if (moved > 1) rej = 2;
      if (!rej && moved == 1) {
        if (istar == 1) {
          const vec3 w = unit(v[1].p - C.eye);
          const Hit h = closest<CW>(S, Fp, C.eye, w, stk, wc, RAY_RETRACE);
          if (!h.ok) {
            rej = 1;
          } else {
            hit_vertex(S, Fp.pose, h, C.eye, w, y.p, y.n, y.md);
            if (is_emitter(S, y.md)) rej = 1;
          }
        } else {
          PV x = v[1];
#pragma unroll
          for (int q = 2; q < kMaxK - 1; ++q)
            if (q == istar) x = v[q];
          y.p = pose_apply(Fp.pose, pose_inv_apply(A.F.pose, x.p));
          y.n = pose_rot(Fp.pose, pose_inv_rot(A.F.pose, x.n));
          y.md = x.md;
        }
      }
      // R3 / R4 at the reconnection neighbours of the moved vertex
      if (!rej && moved == 1) {
        PV xs = v[1];
#pragma unroll
        for (int q = 2; q < kMaxK - 1; ++q)
          if (q == istar) xs = v[q];
        const float ax = roughness(vmat(S, A.F, xs.md)), ay = roughness(vmat(S, Fp, y.md));
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int jn = side == 0 ? istar - 1 : istar + 1;
          if (jn < 1 || rej) continue;
          const bool light = jn == k - 1;
          PV xj = v[1];
#pragma unroll
          for (int q = 1; q < kMaxK - 1; ++q)
            if (q == jn) xj = v[q];
          if (!light && (xj.md & kDynBit)) rej = 3;
          const float aj = light ? 1.0f : roughness(vmat(S, A.F, xj.md));
          if (fminf(fminf(ax, ay), aj) < A.alpha_min) rej = rej ? rej : 3;
          if (rej || (light && E.env)) continue;
          const vec3 pj = pick(light, E.p, xj.p), nj = pick(light, E.n, xj.n);
          const vec3 dy = y.p - pj, dxv = xs.p - pj;
          const float ly2 = dot(dy, dy), lx2 = dot(dxv, dxv);
          if (fminf(sqrtf(ly2), sqrtf(lx2)) < A.d_min) {
            rej = 3;
            continue;
          }
          const float jac = (fabsf(dot(nj, dy)) / sqrtf(ly2)) / (fabsf(dot(nj, dxv)) / sqrtf(lx2)) * (lx2 / ly2);
          if (!(jac <= A.jac_max && jac >= 1.0f / A.jac_max)) rej = 4;
        }
      }
      // R6: support of the mapped path in f'
      if (!rej) {
#pragma unroll
        for (int q = 1; q < kMaxK - 1; ++q) {
          if (q > k - 2 || rej) continue;
          const PV cur = pick(q == istar, y, v[q]);
          if (is_emitter(S, cur.md)) rej = 6;
          const vec3 a = pick(q - 1 == 0, C.eye, pick(q - 1 == istar, y.p, v[q - 1].p));
          const vec3 b = pick(q + 1 == k - 1, lpos(E, cur.p), pick(q + 1 == istar, y.p, v[q + 1].p));
          if (!same_side(cur.n, cur.p, a, b)) rej = 6;
        }
        if (!rej && !E.env) {
          const vec3 prv = pick(k - 2 == istar, y.p, vl.p);
          if (!(dot(E.n, prv - E.p) > 0.0f)) rej = 6;
        }
      }
      // R5: visibility in f' (edges at the moved vertex), ghost records elsewhere
      if (!rej) {
#pragma unroll
        for (int a = 0; a < kMaxK - 1; ++a) {
          if (a > k - 2 || rej) continue;
          const bool touches = moved == 1 && (a == istar - 1 || a == istar);
          if (touches) {
            if (a == 0) continue;
            const PV pa = pick(a == istar, y, v[a]);
            const End EA = end_surf(pa.p, pa.n);
            const bool last = a + 1 == k - 1;
            const PV pb = pick(a + 1 == istar, y, v[a + 1]);
            const End EB{pick(last, E.p, pb.p), pick(last, E.n, pb.n),
                         last ? (E.env ? END_ENV : END_LIGHT) : END_SURF};
            if (!edge_visible<CW>(S, Fp, EA, EB, stk, wc, RAY_MAPVIS)) rej = 5;
          } else if ((exm >> a) & 1u) {
            rej = 5;
          }
        }
      }
    }
    if (!rej) {
      const vec3 fy = rest(Fp, istar, y) * camf;
      if constexpr (BAL) {
        // The other direction samples this pair through y = T(x) with its own
        // frame's strategies.  Their densities: the tables of the mapped path
        // (x with vertex istar replaced by y), its dynamic vertex y, and its
        // ghost crossings in f' (the object at this frame's pose): only the
        // two edges at y can cross it, since x's other edges are unoccluded in
        // this frame.  In x's measure the sum carries |T'| = pcam_x / pcam_y
        // (1 unless x_1 was re-traced).  With no vertex moved (the frames
        // coincide, or x has no dynamic vertex and no crossing) the mapped
        // path is x and its strategies are x's.
        float sum_y = sum;
        if (istar > 0) {
          PV ym = v[0], yp = v[0];  // the neighbours of the moved vertex
#pragma unroll
          for (int q = 0; q < kMaxK - 1; ++q) {
            if (q == istar - 1) ym = v[q];
            if (q == istar + 1) yp = v[q];
          }
          const End ey = end_surf(y.p, y.n);
          const Cross c1 = edge_cross<CW>(S, Fp, istar == 1 ? end_eye(S) : end_surf(ym.p, ym.n), ey, stk, wc);
          const bool last = istar + 1 == k - 1;
          const Cross c2 = edge_cross<CW>(S, Fp, ey, last ? end_light(E) : end_surf(yp.p, yp.n), stk, wc);
          const float w1 = istar == 1 ? c1.sa : c1.s0, w2 = last ? c2.sb : c2.s0;
          // swap the mapped path in, take its sum, swap x back
          float exw_x[kMaxK];
#pragma unroll
          for (int q = 0; q < kMaxK; ++q) {
            exw_x[q] = exw[q];
            exw[q] = q == istar - 1 ? w1 : (q == istar ? w2 : 0.0f);
          }
          const uint32_t exm_x = exm;
          exm = ((c1.n > 0.0f ? 1u : 0u) << (istar - 1)) | ((c2.n > 0.0f ? 1u : 0u) << istar);
          PV xs = v[0];
#pragma unroll
          for (int q = 1; q < kMaxK - 1; ++q)
            if (q == istar) {
              xs = v[q];
              v[q] = y;
            }
          const PV vl_x = vl;
          if (istar == k - 2) vl = y;
          const float pcam_x = pcam;
          if (istar == 1) pcam = camera_geo(C, y.p, y.n);
          sum_y = mis_sum(false) * (pcam_x / pcam);
#pragma unroll
          for (int q = 1; q < kMaxK - 1; ++q)
            if (q == istar) v[q] = xs;
          vl = vl_x;
          pcam = pcam_x;
          exm = exm_x;
#pragma unroll
          for (int q = 0; q < kMaxK; ++q) exw[q] = exw_x[q];
        }
        val = fx - fy;
        denom = sum + sum_y;
      } else {
        val = (fx - fy) * A.cweight;
      }
    } else {
      val = fx;
    }
    reason = rej;
  }
  const float sc = A.sigma / denom * A.inv_n;
  rec = make_float4(__int_as_float(pixel | (A.job << 24)), val.x * sc, val.y * sc, val.z * sc);
  if (A.mlp && (T == 2 || T == 3) && pgen > 0.0f) {
    // x_m = x_D (m = i + 2) and its light-side neighbour, by constant indices
    const int m = i + 2;
    PV xm = v[0], xn = v[0];
#pragma unroll
    for (int q = 1; q < kMaxK - 1; ++q) {
      if (q == m) xm = v[q];
      if (q == m + 1) xn = v[q];
    }
    const vec3 to = m + 1 == k - 1 ? lpos(E, vl.p) : xn.p;
    const vec3 o = spawn(S, xm.p, xm.n, to);  // the ray origin generating x_{m+1} from x_m
    const vec3 w = pose_inv_rot(A.F.pose, unit(xn.p - o));
    mlp_input(*A.mlp, pose_inv_apply(A.F.pose, xm.p), pose_inv_rot(A.F.pose, xm.n), tr.x);
    tr.w[0] = w.x;
    tr.w[1] = w.y;
    tr.w[2] = w.z;
    const float fa = (fabsf(val.x) + fabsf(val.y) + fabsf(val.z)) * (1.0f / 3.0f);
    tr.weight = A.train_weighting == 1 ? fa / pgen * (fa / sum) : fa / pgen;
  }
}

template <bool CW, bool BAL>
__global__ __launch_bounds__(kTraceBlock) RPI_CONNECT_OCCUPANCY void connect_kernel(WalkArgs A) {
  __shared__ __attribute__((aligned(16))) int stk[kStackDepth * kTraceBlock];
  __shared__ unsigned long long cnt[16];
  if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = min((uint32_t)A.W.pair_cap, *A.W.npairs);
  WorkCount wc{};
  // wave-uniform trip count (one wave per workgroup): the training-record
  // queue reservation below is a wave-wide prefix sum
  for (;;) {
    const uint32_t base = next_batch(&A.W.fetch[1]);
    if (base >= n) break;
    const uint32_t idx = base + threadIdx.x;
    const bool act = idx < n;
    TrainRec tr;
    tr.weight = 0.0f;
    if (act) {
      const uint32_t code = A.W.pairs[idx];
      const int s = code_slot(code);
      const int64_t g = A.item0 + s / kItem;
      const int jd = find_jd(A.item_prefix, 2 * A.njobs, g);
      const DevJob& J = A.jobs[jd >> 1];
      const int dir = jd & 1;
      const CCtx C{J.S, J.F[dir], J.F[1 - dir], A.W, A.tech, A.material_mode, A.mask, dir ? -1.0f : 1.0f,
                   A.cweight, J.inv_n, A.alpha_min, A.d_min, A.jac_max, jd >> 1, A.train ? &A.mlp : nullptr,
                   A.train_weighting, A.no_mapping, J.tech_ratio};
      const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 q8a = A.W.t8q ? A.W.t8q[2 * (size_t)idx] : z4, q8b = A.W.t8q ? A.W.t8q[2 * (size_t)idx + 1] : z4;
      float4 rec;
      int reason;
      connect_one<CW, BAL>(C, code, q8a, q8b, stk, wc, rec, reason, tr);
      A.W.records[idx] = rec;
      if (CW) wc.bytes += 16u;
      if (A.keep_records) {
        // debug key: the pair as (i + 1) << 4 | (j + 1)
        const uint32_t pr = ((uint32_t)(code_i(code) + 1) << 4) | (uint32_t)(code_j(code) + 1);
        A.W.rec_keys[idx] = (uint32_t)dir | ((uint32_t)A.tech << 1) | (pr << 8);
        A.W.rec_sample[idx] = (uint32_t)slot_sample(A, J, jd, s);
      }
      if (A.stats && (reason <= 6 || reason == 9)) atomicAdd(&cnt[reason == 9 ? 7 : reason], 1ull);
    }
    if (A.train) {
      const int c = tr.weight > 0.0f ? 1 : 0;
      int total;
      const uint32_t at = wave_reserve(A.train_count, c, total);
      if (c && (int64_t)at < A.train_cap) {
        float* o = A.train + (size_t)at * 10;
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = tr.x[q];
        o[6] = tr.w[0];
        o[7] = tr.w[1];
        o[8] = tr.w[2];
        o[9] = tr.weight;
      }
    }
  }
  __syncthreads();
  if (A.stats && threadIdx.x < 8) {
    const unsigned long long c = cnt[threadIdx.x];
    if (c) {
      if (threadIdx.x == 0) atomicAdd(&A.stats->accepted, c);
      else atomicAdd(&A.stats->rejected[threadIdx.x == 7 ? 0 : threadIdx.x], c);
      atomicAdd(&A.stats->paths, c);
      atomicAdd(&A.stats->by_tech[A.tech], c);
    }
  }
  if (CW) flush_work(A.stats, kKidConnect, wc);
}

// Technique (8)'s MIS term needs the proposal at every dynamic vertex x_m
// with 1 <= m <= k-3 of every queued path: one MLP pass per vertex
// position over the wave's 64 paths (matrix cores), then the mixture density
// of the object-space direction x_m -> x_{m+1} (from the offset origin, as
// the other MIS terms measure it).
__global__ __launch_bounds__(kTraceBlock) void proposal_pdf_kernel(WalkArgs A) {
  __shared__ __attribute__((aligned(16))) float lds[kMlpLdsBytes / 4];
  const uint32_t n = min((uint32_t)A.W.pair_cap, *A.W.npairs);
  const MlpDev& M = A.mlp;
  for (uint32_t base = blockIdx.x * kTraceBlock; base < n; base += gridDim.x * kTraceBlock) {
    const uint32_t idx = base + threadIdx.x;
    const bool act = idx < n;
    int s = 0, i = 0, k = 0, dir = 0;
    const DevJob* J = A.jobs;
    if (act) {
      const uint32_t code = A.W.pairs[idx];
      s = code_slot(code);
      i = code_i(code);
      const int j = code_j(code);
      k = (i + 1) + (has_mid(A.tech) ? 1 : 0) + (j + 1) + 2;
      const int jd = find_jd(A.item_prefix, 2 * A.njobs, A.item0 + s / kItem);
      J = A.jobs + (jd >> 1);
      dir = jd & 1;
    }
    const Pose& pose = J->F[dir].pose;
    float q[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int m = 1; m <= kMaxK - 3; ++m) {
      PV x = PV{v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 1.f), 0u}, y = x;
      bool need = act && m <= k - 3;
      if (need) {
        x = path_vertex(A.W, s, i, has_mid(A.tech), m);
        need = (x.md & kDynBit) != 0u;
        if (need) y = path_vertex(A.W, s, i, has_mid(A.tech), m + 1);
      }
      if (__ballot(need) == 0ull) continue;  // wave-uniform
      float in[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (need) mlp_input(M, pose_inv_apply(pose, x.p), pose_inv_rot(pose, x.n), in);
      const float* raw = mlp_forward_wave(M, in, lds);
      if (need) {
        const vec3 o = spawn(J->S, x.p, x.n, y.p);
        q[m - 1] = t8_dir_pdf(raw, pose_inv_rot(pose, unit(y.p - o)));
      }
      __syncthreads();  // the next pass overwrites the outputs
    }
    if (act) {
      A.W.t8q[2 * (size_t)idx] = make_float4(q[0], q[1], q[2], q[3]);
      A.W.t8q[2 * (size_t)idx + 1] = make_float4(q[4], 0.f, 0.f, 0.f);
    }
  }
}

// ------------------------------------------------------------------ splat
// Batch-wide tile of a record and the pixel's index inside the tile.
DEV int tile_of(const SplatArgs& a, int code, int& local) {
  const DevJob& J = a.jobs[code >> 24];
  const int pixel = code & 0xffffff;
  const int px = pixel % J.W, py = pixel / J.W;
  local = (py % a.ts) * a.ts + (px % a.ts);
  return J.tile0 + (py / a.ts) * J.tilesx + px / a.ts;
}

__global__ void zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}
__global__ void zero_f32(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}

// Counting sort of the records by tile without global atomics: block b owns
// the contiguous record slice [b*len, (b+1)*len) and histograms it in LDS;
// hist[tile * nblk + b] is then scanned tile-major, and the same block
// scatters its slice with LDS cursors.
DEV void slice(const SplatArgs& a, uint32_t n, uint32_t& b0, uint32_t& b1) {
  const uint32_t len = (n + a.nblk - 1) / a.nblk;
  b0 = min(n, blockIdx.x * len);
  b1 = min(n, b0 + len);
}

__global__ __launch_bounds__(256) void splat_count(SplatArgs a) {
  extern __shared__ uint32_t lh[];  // [ntiles]
  const uint32_t n = (uint32_t)min((int64_t)*a.nrec, a.cap);
  for (int t = threadIdx.x; t < a.ntiles; t += 256) lh[t] = 0u;
  __syncthreads();
  uint32_t b0, b1;
  slice(a, n, b0, b1);
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const int code = __float_as_int(a.records[i].x);
    int local;
    if (code >= 0) atomicAdd(&lh[tile_of(a, code, local)], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < a.ntiles; t += 256) a.hist[(size_t)t * a.nblk + blockIdx.x] = lh[t];
}

// One workgroup per tile: exclusive scan of its nblk block counts (in place)
// and the tile total.
__global__ __launch_bounds__(256) void splat_scan_blocks(SplatArgs a) {
  __shared__ uint32_t part[256];
  const int t = blockIdx.x;
  uint32_t* h = a.hist + (size_t)t * a.nblk;
  const int per = (a.nblk + 255) / 256;
  uint32_t sum = 0;
  for (int i = threadIdx.x * per; i < min(a.nblk, (int)(threadIdx.x + 1) * per); ++i) sum += h[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int i = threadIdx.x * per; i < min(a.nblk, (int)(threadIdx.x + 1) * per); ++i) {
    const uint32_t c = h[i];
    h[i] = run;
    run += c;
  }
  if (threadIdx.x == 255) a.tcount[t] = part[255];
}

// Exclusive scans of the tile totals and of the tiles' chunk counts
// (ceil(total / kSplatChunk)) by one workgroup.
__global__ __launch_bounds__(1024) void splat_scan_tiles(SplatArgs a) {
  __shared__ uint32_t part[1024], cpart[1024];
  const int t = threadIdx.x;
  const int per = (a.ntiles + 1023) / 1024;
  uint32_t sum = 0, csum = 0;
  for (int i = t * per; i < min(a.ntiles, (t + 1) * per); ++i) {
    sum += a.tcount[i];
    csum += (a.tcount[i] + kSplatChunk - 1) / kSplatChunk;
  }
  part[t] = sum;
  cpart[t] = csum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t x = t >= off ? part[t - off] : 0u, y = t >= off ? cpart[t - off] : 0u;
    __syncthreads();
    part[t] += x;
    cpart[t] += y;
    __syncthreads();
  }
  uint32_t run = part[t] - sum, crun = cpart[t] - csum;
  for (int i = t * per; i < min(a.ntiles, (t + 1) * per); ++i) {
    a.toff[i] = run;
    a.cpre[i] = crun;
    run += a.tcount[i];
    crun += (a.tcount[i] + kSplatChunk - 1) / kSplatChunk;
  }
  if (t == 1023) {
    a.toff[a.ntiles] = part[1023];
    a.cpre[a.ntiles] = cpart[1023];
  }
}

__global__ __launch_bounds__(256) void splat_scatter(SplatArgs a) {
  extern __shared__ uint32_t cur[];  // [ntiles] write cursors of this block
  const uint32_t n = (uint32_t)min((int64_t)*a.nrec, a.cap);
  for (int t = threadIdx.x; t < a.ntiles; t += 256) cur[t] = a.toff[t] + a.hist[(size_t)t * a.nblk + blockIdx.x];
  __syncthreads();
  uint32_t b0, b1;
  slice(a, n, b0, b1);
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const float4 r = a.records[i];
    const int code = __float_as_int(r.x);
    if (code < 0) continue;
    int local;
    const int t = tile_of(a, code, local);
    const uint32_t at = atomicAdd(&cur[t], 1u);
    a.binned[at] = make_float4(__int_as_float(local), r.y, r.z, r.w);
  }
}

// Record value -> fixed point (units of 2^-40 of the scene's largest
// emission).  Clamped to +-2^56 units so that sums of many records cannot
// wrap; rintf of a float already holding an integer is exact.
constexpr float kFxClamp = 72057594037927936.0f;  // 2^56
DEV unsigned long long to_fixed(float v, float scale) {
  const float x = fminf(fmaxf(v * scale, -kFxClamp), kFxClamp);
  return (unsigned long long)(long long)rintf(x);
}

// Workgroups take chunks of at most kSplatChunk binned records of one tile
// (a few tiles near the edit hold most records, so one workgroup per tile
// would leave the chip idle behind them) and sum them per pixel in LDS in
// fixed point; the tile's sums go to the job's fixed-point image: a plain
// read-modify-write when the tile has one chunk, integer adds when several
// chunks share it.  Integer addition is associative, so the image does not
// depend on the order in which records, chunks or rounds arrive, and no
// floating-point atomic is used.
__global__ __launch_bounds__(256) void splat_tiles(SplatArgs a) {
  __shared__ unsigned long long acc[kTileMax * kTileMax * 3];
  const uint32_t nch = a.cpre[a.ntiles];
  const int tp = a.ts * a.ts;
  for (uint32_t g = blockIdx.x; g < nch; g += gridDim.x) {
    int lo = 0, hi = a.ntiles;  // cpre[lo] <= g < cpre[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.cpre[mid] <= g) lo = mid;
      else hi = mid;
    }
    const int t = lo;
    const uint32_t b = a.toff[t] + (g - a.cpre[t]) * kSplatChunk;
    const uint32_t e = min(b + kSplatChunk, a.toff[t + 1]);
    const bool shared = a.cpre[t + 1] - a.cpre[t] > 1;
    const DevJob& J = a.jobs[a.tile_job[t]];
    const float scale = J.fx_scale;
    for (int i = threadIdx.x; i < tp * 3; i += 256) acc[i] = 0ull;
    __syncthreads();
    for (uint32_t i = b + threadIdx.x; i < e; i += 256) {
      const float4 r = a.binned[i];
      const int l = __float_as_int(r.x);
      atomicAdd(&acc[3 * l + 0], to_fixed(r.y, scale));
      atomicAdd(&acc[3 * l + 1], to_fixed(r.z, scale));
      atomicAdd(&acc[3 * l + 2], to_fixed(r.w, scale));
    }
    __syncthreads();
    const int lt = t - J.tile0;
    const int tx = lt % J.tilesx, ty = lt / J.tilesx;
    for (int l = threadIdx.x; l < tp; l += 256) {
      const int px = tx * a.ts + (l % a.ts), py = ty * a.ts + (l / a.ts);
      if (px < J.W && py < J.H) {
        unsigned long long* o = J.acc + 3 * ((size_t)py * J.W + px);
        if (shared) {
          atomicAdd(o + 0, acc[3 * l]);
          atomicAdd(o + 1, acc[3 * l + 1]);
          atomicAdd(o + 2, acc[3 * l + 2]);
        } else {
          o[0] += acc[3 * l];
          o[1] += acc[3 * l + 1];
          o[2] += acc[3 * l + 2];
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void zero_images(const DevJob* jobs, int njobs) {
  for (int j = 0; j < njobs; ++j) {
    const int64_t n = (int64_t)jobs[j].W * jobs[j].H * 3;
    unsigned long long* f = jobs[j].acc;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) f[i] = 0ull;
    float* q = jobs[j].tech_images;
    if (q)
      for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < kTechs * n; i += (int64_t)gridDim.x * 256) q[i] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void flush_acc(const DevJob* jobs, int njobs, int tech, int accumulate) {
  for (int j = 0; j < njobs; ++j) {
    const DevJob& J = jobs[j];
    const int64_t n = (int64_t)J.W * J.H * 3;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
      const float v = (float)((double)(long long)J.acc[i] * J.fx_unit);
      J.acc[i] = 0ull;
      if (tech) J.tech_images[(size_t)(tech - 1) * n + i] = v;
      else J.image[i] = accumulate ? J.image[i] + v : v;
    }
  }
}

// The total of the technique images, pixel by pixel in technique order, so
// that it equals their sum taken in that order bit for bit.
__global__ __launch_bounds__(256) void sum_technique_images(const DevJob* jobs, int njobs, int accumulate) {
  for (int j = 0; j < njobs; ++j) {
    const int64_t n = (int64_t)jobs[j].W * jobs[j].H * 3;
    float* p = jobs[j].image;
    const float* q = jobs[j].tech_images;
    if (!q) continue;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
      float acc = accumulate ? p[i] : 0.0f;
#pragma unroll
      for (int t = 0; t < kTechs; ++t) acc += q[(size_t)t * n + i];
      p[i] = acc;
    }
  }
}

// ------------------------------------------------------------------ frames
// One camera sample of plain path tracing in frame F (Sec. 3.1): next-event
// estimation at every vertex and emission seen directly from the camera.
// The Philox stream is that of sample smp of technique 7 in direction dir.
DEV vec3 frame_sample(const FrameArgs& A, const DevFrame& F, int dir, int pixel, int64_t smp, int* stk, WorkCount& wc) {
  const DevScene& S = A.S;
  const DevCamera& C = S.cam;
  const int P = C.W * C.H;
  const float Pf = (float)P;
  const float invN = 1.0f / ((float)A.spp * Pf);
  vec3 sum = v3(0, 0, 0);
  Rng g{A.k0, A.k1, (uint32_t)smp, (uint32_t)dir << 23, A.job};
  float u[4];
  draw(g, 0, 0, 0, u);
  const vec3 w = camera_dir(C, pixel, u[0], u[1]);
  const Hit h = closest<false>(S, F, C.eye, w, stk, wc);
  if (!h.ok) {
    if (S.p_env > 0.0f && raster(C, C.eye + w) >= 0) sum = sum + S.env * (Pf * invN);
    return sum;
  }
  vec3 p, n;
  uint32_t md;
  hit_vertex(S, F.pose, h, C.eye, w, p, n, md);
  const int pix1 = raster(C, p);
  if (pix1 < 0) return sum;
  if (is_emitter(S, md)) {
    if (dot(n, C.eye - p) > 0.0f) {
      const float* em = S.mats + 8 * (md & ~kDynBit) + 5;
      sum = sum + v3(em[0], em[1], em[2]) * (Pf * invN);
    }
    return sum;
  }
  // throughput f / p up to the current vertex (camera factor / camera pdf = P)
  vec3 beta = v3(Pf, Pf, Pf);
  vec3 prev = C.eye;
  for (int b = 0; b + 2 <= A.depth; ++b) {
    const Material mt = vmat(S, F, md);
    draw(g, 0, b + 1, 1, u);
    LightEnd E;
    if (sample_light(S, u, E)) {
      const bool face = E.env ? true : dot(E.n, p - E.p) > 0.0f;
      const vec3 lp = E.env ? p + E.n : E.p;
      if (face && same_side(n, p, prev, lp) &&
          edge_visible<false>(S, F, end_surf(p, n), end_light(E), stk, wc, RAY_SHADOW)) {
        const vec3 wl = E.env ? E.n : unit(E.p - p);
        const vec3 rho = bsdf_eval(mt, n, unit(prev - p), wl);
        float gg;
        if (E.env) {
          gg = fabsf(dot(n, wl));
        } else {
          const vec3 d = E.p - p;
          gg = fabsf(dot(n, wl)) * fabsf(dot(E.n, wl)) / len2(d);
        }
        const vec3 c = vmul(vmul(beta, rho), light_Le(S, E)) * (gg / light_pdf(S, E.env));
        sum = sum + c * invN;
      }
    }
    if (b + 3 > A.depth) break;
    draw(g, 0, b + 1, 0, u);
    vec3 wo;
    if (!bsdf_sample(mt, n, unit(prev - p), u[0], u[1], wo)) break;
    const vec3 o = spawn_dir(S, p, n, wo);
    const Hit h2 = closest<false>(S, F, o, wo, stk, wc);
    if (!h2.ok) break;
    vec3 q, qn;
    uint32_t qmd;
    hit_vertex(S, F.pose, h2, o, wo, q, qn, qmd);
    if (is_emitter(S, qmd)) break;
    // f/p update: rho G / (pdf_w * cos_q / r^2 from the offset origin)
    const vec3 wi = unit(prev - p);
    const vec3 rho = bsdf_eval(mt, n, wi, unit(q - p));
    const vec3 d = q - p;
    const vec3 du = unit(d);
    const float G = fabsf(dot(n, du)) * fabsf(dot(qn, du)) / len2(d);
    const vec3 dq = q - o;
    const float pa = bsdf_pdf(mt, n, wi, wo) * fabsf(dot(qn, unit(dq))) / len2(dq);
    if (!(pa > 0.0f)) break;  // a direction of zero density (rounding at grazing angles) ends the walk
    beta = vmul(beta, rho) * (G / pa);
    prev = p;
    p = q;
    n = qn;
    md = qmd;
  }
  return sum;
}

// One lane per pixel; samples s = pixel + m * P (the residual technique (7)
// uses the same pixel-of-sample rule).  mode 0: frame F in stream direction
// A.dir; 1: the difference F - F2 with the same random numbers in both
// frames (correlated path tracing); 2: F - F2 from independent streams
// (direction 0 for F, 1 for F2: path tracing each frame from scratch).
__global__ __launch_bounds__(kTraceBlock) void frame_kernel(FrameArgs A) {
  __shared__ __attribute__((aligned(16))) int stk[kStackDepth * kTraceBlock];
  const DevCamera& C = A.S.cam;
  const int P = C.W * C.H;
  const int pixel = blockIdx.x * kTraceBlock + threadIdx.x;
  if (pixel >= P) return;
  WorkCount wc{};
  vec3 sum = v3(0, 0, 0);
  for (int m = 0; m < A.spp; ++m) {
    const int64_t smp = (int64_t)pixel + (int64_t)m * P;
    if (smp < A.s0 || smp >= A.s1) continue;
    if (A.mode == 0) {
      sum = sum + frame_sample(A, A.F, A.dir, pixel, smp, stk, wc);
    } else {
      const vec3 a = frame_sample(A, A.F, 0, pixel, smp, stk, wc);
      const vec3 b = frame_sample(A, A.F2, A.mode == 1 ? 0 : 1, pixel, smp, stk, wc);
      sum = sum + (a - b);
    }
  }
  float* o = A.image + 3 * (size_t)pixel;
  if (A.accumulate) {
    o[0] += sum.x;
    o[1] += sum.y;
    o[2] += sum.z;
  } else {
    o[0] = sum.x;
    o[1] = sum.y;
    o[2] = sum.z;
  }
}

// ------------------------------------------------------------------ launchers
template <int T, bool CW>
static void launch_walk_t(const WalkArgs& A, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((walk_kernel<T, CW>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
}
template <bool CW>
static void launch_walk_cw(const WalkArgs& A, int blocks, hipStream_t st) {
  switch (A.tech) {
    case 1: launch_walk_t<1, CW>(A, blocks, st); break;
    case 2: launch_walk_t<2, CW>(A, blocks, st); break;
    case 3: launch_walk_t<3, CW>(A, blocks, st); break;
    case 4: launch_walk_t<4, CW>(A, blocks, st); break;
    case 5: launch_walk_t<5, CW>(A, blocks, st); break;
    case 6: launch_walk_t<6, CW>(A, blocks, st); break;
    case 8: launch_walk_t<8, CW>(A, blocks, st); break;
    default: launch_walk_t<7, CW>(A, blocks, st); break;
  }
}

void launch_walk(const WalkArgs& A, int blocks, hipStream_t st) {
  if (A.count_work) launch_walk_cw<true>(A, blocks, st);
  else launch_walk_cw<false>(A, blocks, st);
}
template <int T, bool CW>
static void launch_walk_task_t(const WalkArgs& A, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((walk_task_kernel<T, CW>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
}
template <bool CW>
static void launch_walk_task_cw(const WalkArgs& A, int blocks, hipStream_t st) {
  switch (A.tech) {
    case 1: launch_walk_task_t<1, CW>(A, blocks, st); break;
    case 2: launch_walk_task_t<2, CW>(A, blocks, st); break;
    case 3: launch_walk_task_t<3, CW>(A, blocks, st); break;
    case 4: launch_walk_task_t<4, CW>(A, blocks, st); break;
    case 5: launch_walk_task_t<5, CW>(A, blocks, st); break;
    case 6: launch_walk_task_t<6, CW>(A, blocks, st); break;
    case 8: launch_walk_task_t<8, CW>(A, blocks, st); break;
    default: launch_walk_task_t<7, CW>(A, blocks, st); break;
  }
}
void launch_walk_tasks(const WalkArgs& A, int blocks, hipStream_t st) {
  if (A.count_work) launch_walk_task_cw<true>(A, blocks, st);
  else launch_walk_task_cw<false>(A, blocks, st);
}
void launch_sum_technique_images(const DevJob* jobs, int njobs, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(sum_technique_images, dim3(1024), dim3(256), 0, st, jobs, njobs, accumulate ? 1 : 0);
}
void launch_flush_acc(const DevJob* jobs, int njobs, int tech, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(flush_acc, dim3(1024), dim3(256), 0, st, jobs, njobs, tech, accumulate ? 1 : 0);
}
void launch_zero_images(const DevJob* jobs, int njobs, hipStream_t st) {
  hipLaunchKernelGGL(zero_images, dim3(1024), dim3(256), 0, st, jobs, njobs);
}
void launch_t8_start(const WalkArgs& A, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(t8_start_kernel, dim3(blocks), dim3(kTraceBlock), 0, st, A);
}
void launch_proposal_pdf(const WalkArgs& A, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(proposal_pdf_kernel, dim3(blocks), dim3(kTraceBlock), 0, st, A);
}

// Counting sort of the path queue by path length k (vertices), in two
// passes: histogram, then each block reserves its slice's places per k and
// scatters.  The order within one k is not kept.
DEV int path_len(uint32_t code, int tech) {
  const int i = code_i(code), j = code_j(code);
  return min((i + 1) + (has_mid(tech) ? 1 : 0) + (j + 1) + 2, 15);
}
__global__ __launch_bounds__(256) void pair_hist_kernel(WalkArgs A) {
  __shared__ uint32_t h[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t n = min((uint32_t)A.W.pair_cap, *A.W.npairs);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    atomicAdd(&h[path_len(A.W.pairs[i], A.tech)], 1u);
  __syncthreads();
  if (threadIdx.x < 16 && h[threadIdx.x]) atomicAdd(&A.W.kbins[threadIdx.x], h[threadIdx.x]);
}
__global__ __launch_bounds__(256) void pair_sort_kernel(WalkArgs A) {
  __shared__ uint32_t h[16], base[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t n = min((uint32_t)A.W.pair_cap, *A.W.npairs);
  const uint32_t len = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t b0 = min(n, blockIdx.x * len), b1 = min(n, b0 + len);
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += 256) atomicAdd(&h[path_len(A.W.pairs[i], A.tech)], 1u);
  __syncthreads();
  if (threadIdx.x < 16) {
    uint32_t pre = 0;
    for (int k = 0; k < (int)threadIdx.x; ++k) pre += A.W.kbins[k];
    base[threadIdx.x] = pre + (h[threadIdx.x] ? atomicAdd(&A.W.kbins[16 + threadIdx.x], h[threadIdx.x]) : 0u);
    h[threadIdx.x] = 0u;
  }
  __syncthreads();
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const uint32_t code = A.W.pairs[i];
    const int k = path_len(code, A.tech);
    A.W.pairs2[base[k] + atomicAdd(&h[k], 1u)] = code;
  }
}
void launch_start_order(const WalkArgs& A, hipStream_t st) {
  const int items = A.tech == 7 ? order_items<7>() : order_items<1>();
  const dim3 grid((unsigned)std::min((A.nitems + items - 1) / items, 2048));
  switch (A.tech) {
    case 1: hipLaunchKernelGGL(start_order_kernel<1>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 2: hipLaunchKernelGGL(start_order_kernel<2>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 3: hipLaunchKernelGGL(start_order_kernel<3>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 4: hipLaunchKernelGGL(start_order_kernel<4>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 5: hipLaunchKernelGGL(start_order_kernel<5>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 6: hipLaunchKernelGGL(start_order_kernel<6>, grid, dim3(kOrderThreads), 0, st, A); break;
    case 7: hipLaunchKernelGGL(start_order_kernel<7>, grid, dim3(kOrderThreads), 0, st, A); break;
    default: hipLaunchKernelGGL(start_order_kernel<8>, grid, dim3(kOrderThreads), 0, st, A); break;
  }
}
// Path order: within windows of kOrderWindow entries of the length-sorted
// queue (pairs2), the paths are counting-sorted by (length, the tile of
// their pixel in a 16 x 16 grid over the image) into pairs, so that the
// connect kernel's camera re-traces and the mapped edges' visibility rays of
// a wave start from nearby points.
constexpr int kOrderWindow = 65536;
__global__ __launch_bounds__(kOrderThreads) void pair_order_kernel(WalkArgs A) {
  __shared__ uint32_t cnt[kOrderBins], part[kOrderThreads];
  constexpr int kPerThread = kOrderBins / kOrderThreads;
  const int n = (int)min((uint32_t)A.W.pair_cap, *A.W.npairs);
  // the keys: the splat records' space (pair_cap float4), free until connect writes them
  uint32_t* key = reinterpret_cast<uint32_t*>(A.W.records);
  for (int w = blockIdx.x; w * kOrderWindow < n; w += gridDim.x) {
    const int p0 = w * kOrderWindow, p1 = min(p0 + kOrderWindow, n);
    for (int b = threadIdx.x; b < kOrderBins; b += kOrderThreads) cnt[b] = 0u;
    __syncthreads();
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kOrderThreads) {
      const uint32_t code = A.W.pairs2[p];
      const int s = code_slot(code), i = code_i(code), j = code_j(code);
      const bool mid = has_mid(A.tech);
      const int nsc = (i + 1) + (mid ? 1 : 0) + (j + 1);
      uint32_t tile = 0u;
      if (nsc > 0) {
        const int jd = find_jd(A.item_prefix, 2 * A.njobs, A.item0 + s / kItem);
        const DevCamera& C = A.jobs[jd >> 1].S.cam;
        const int px = raster(C, path_vertex(A.W, s, i, mid, 1).p);
        if (px >= 0) tile = (uint32_t)(((px / C.W) * 16 / C.H) * 16 + (px % C.W) * 16 / C.W);
      }
      const uint32_t kk = ((uint32_t)min(nsc + 2, 15) << 8) | tile;
      atomicAdd(&cnt[kk], 1u);
      key[p] = kk;
    }
    __syncthreads();
    {  // exclusive prefix sums: each key's first place in the window
      const int t = threadIdx.x;
      uint32_t sum = 0u;
      for (int q = 0; q < kPerThread; ++q) sum += cnt[kPerThread * t + q];
      part[t] = sum;
      __syncthreads();
      for (int off = 1; off < kOrderThreads; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
      }
      uint32_t run = part[t] - sum;
      for (int q = 0; q < kPerThread; ++q) {
        const uint32_t c = cnt[kPerThread * t + q];
        cnt[kPerThread * t + q] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kOrderThreads)
      A.W.pairs[p0 + atomicAdd(&cnt[key[p]], 1u)] = A.W.pairs2[p];
    __syncthreads();
  }
}

void launch_sort_pairs(const WalkArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(pair_hist_kernel, dim3(1024), dim3(256), 0, st, A);
  hipLaunchKernelGGL(pair_sort_kernel, dim3(1024), dim3(256), 0, st, A);
  hipLaunchKernelGGL(pair_order_kernel,
                     dim3((unsigned)std::min<int64_t>((A.W.pair_cap + kOrderWindow - 1) / kOrderWindow, 2048)),
                     dim3(kOrderThreads), 0, st, A);
}

void launch_connect(const WalkArgs& A, int blocks, hipStream_t st) {
  if (A.count_work && A.balance)
    hipLaunchKernelGGL((connect_kernel<true, true>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
  else if (A.count_work)
    hipLaunchKernelGGL((connect_kernel<true, false>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
  else if (A.balance)
    hipLaunchKernelGGL((connect_kernel<false, true>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
  else
    hipLaunchKernelGGL((connect_kernel<false, false>), dim3(blocks), dim3(kTraceBlock), 0, st, A);
}
void launch_splat(const SplatArgs& a, hipStream_t st) {
  const size_t lds = (size_t)a.ntiles * sizeof(uint32_t);
  hipLaunchKernelGGL(splat_count, dim3(a.nblk), dim3(256), lds, st, a);
  hipLaunchKernelGGL(splat_scan_blocks, dim3(a.ntiles), dim3(256), 0, st, a);
  hipLaunchKernelGGL(splat_scan_tiles, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(splat_scatter, dim3(a.nblk), dim3(256), lds, st, a);
  // chunks: at most one per tile plus one per kSplatChunk records
  const int64_t chunks = (int64_t)a.ntiles + a.cap / kSplatChunk + 1;
  hipLaunchKernelGGL(splat_tiles, dim3((unsigned)std::min<int64_t>(chunks, 8192)), dim3(256), 0, st, a);
}
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u32, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256 + 1)), dim3(256), 0, st, p, n);
}
void launch_zero_f32(float* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_f32, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256 + 1)), dim3(256), 0, st, p, n);
}
void launch_frame(const FrameArgs& A, hipStream_t st) {
  const int P = A.S.cam.W * A.S.cam.H;
  hipLaunchKernelGGL(frame_kernel, dim3((P + kTraceBlock - 1) / kTraceBlock), dim3(kTraceBlock), 0, st, A);
}

}  // namespace rpi
