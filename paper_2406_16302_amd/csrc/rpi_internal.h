// Internal types shared by the host runtime (rpi_host.cpp) and the kernels
// (rpi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RPI_HD __host__ __device__ __forceinline__

namespace rpi {

// ------------------------------------------------------------------ vectors
struct vec3 {
  float x, y, z;
};
RPI_HD vec3 v3(float x, float y, float z) { return vec3{x, y, z}; }
RPI_HD vec3 operator+(vec3 a, vec3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
RPI_HD vec3 operator-(vec3 a, vec3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
RPI_HD vec3 operator-(vec3 a) { return v3(-a.x, -a.y, -a.z); }
RPI_HD vec3 operator*(vec3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
RPI_HD vec3 vmul(vec3 a, vec3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
RPI_HD float dot(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
RPI_HD vec3 cross(vec3 a, vec3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
RPI_HD float len2(vec3 a) { return dot(a, a); }
RPI_HD vec3 unit(vec3 a) {
  float l = sqrtf(dot(a, a));
  return v3(a.x / l, a.y / l, a.z / l);
}

// Rigid pose: world = R p + t (R row-major).
struct Pose {
  float r[9];
  float t[3];
};
RPI_HD vec3 pose_apply(const Pose& P, vec3 p) {
  return v3(P.r[0] * p.x + P.r[1] * p.y + P.r[2] * p.z + P.t[0],
            P.r[3] * p.x + P.r[4] * p.y + P.r[5] * p.z + P.t[1],
            P.r[6] * p.x + P.r[7] * p.y + P.r[8] * p.z + P.t[2]);
}
RPI_HD vec3 pose_rot(const Pose& P, vec3 v) {
  return v3(P.r[0] * v.x + P.r[1] * v.y + P.r[2] * v.z, P.r[3] * v.x + P.r[4] * v.y + P.r[5] * v.z,
            P.r[6] * v.x + P.r[7] * v.y + P.r[8] * v.z);
}
RPI_HD vec3 pose_inv_rot(const Pose& P, vec3 v) {
  return v3(P.r[0] * v.x + P.r[3] * v.y + P.r[6] * v.z, P.r[1] * v.x + P.r[4] * v.y + P.r[7] * v.z,
            P.r[2] * v.x + P.r[5] * v.y + P.r[8] * v.z);
}
RPI_HD vec3 pose_inv_apply(const Pose& P, vec3 p) {
  return pose_inv_rot(P, p - v3(P.t[0], P.t[1], P.t[2]));
}

// ------------------------------------------------------------------ scene on the device
enum { MAT_DIFFUSE = 0, MAT_GGX = 1, MAT_EMITTER = 2 };

// 4-wide BVH node (128 B, kNodeF4 float4): the boxes of children 0..3 as
// planes, then their links:
//   f4[0] = lo.x of c0..c3   f4[1] = hi.x   f4[2] = lo.y   f4[3] = hi.y
//   f4[4] = lo.z             f4[5] = hi.z   f4[6] = links (int bits)   f4[7] = 0
// A child link >= 0 is an inner node; a negative link is a leaf
// 0x80000000 | first << 4 | count (count <= 15) into the triangle array;
// unused slots hold kEmptyLink and are never entered.  The root is node 0.
// Triangle (48 B): f4[0] = v0.xyz, id; f4[1] = e1.xyz, material; f4[2] = e2.xyz, 0.
constexpr int kNodeF4 = 8;
constexpr int32_t kEmptyLink = (int32_t)0x80000000;  // a leaf of no triangles
struct DevBvh {
  const float4* nodes;
  const float4* tris;
  int32_t ntris;
};

// Traversal stack entries per lane (LDS: kStackDepth * 256 B per wave).  At
// 40 a compute unit holds 16 waves of the trace kernels, four per SIMD; the
// builder bounds the entries any ray can push by kStackDepth - 1.
#ifndef RPI_STACK_DEPTH
#define RPI_STACK_DEPTH 40
#endif
constexpr int kStackDepth = RPI_STACK_DEPTH;

struct DevCamera {
  vec3 eye, fwd, right, up;
  float tan_half, aspect;
  int32_t W, H;
  float a_film;  // 4 aspect tan^2: film area at distance 1
};

struct DevScene {
  DevBvh stat, obj;
  const float4* obj_tris;  // object triangles in input order (area sampling), 3 float4 each
  const float* obj_cdf;
  int32_t nobj;
  const int32_t* obj_guide;  // guide table of obj_cdf: 2^obj_gbits + 1 entries
  int32_t obj_gbits;
  const float4* light_tris;  // emitter triangles in input order
  const float* light_cdf;
  int32_t nlights;
  const int32_t* light_guide;
  int32_t light_gbits;
  const float* mats;  // 8 floats per material
  int32_t nmats;
  float inv_obj_area;   // p_D = p_G
  float inv_light_area;
  float p_env;          // probability of selecting the environment
  vec3 env;
  DevCamera cam;
  float eps;            // ray offset: 1e-4 of the scene diagonal
  int32_t obj_convex;   // the object bounds a convex solid (every vertex on the inner side of every face)
  vec3 obj_center;      // a point inside it (object space): the mean of its vertices
  float obj_rin;        // closed convex object: radius of a ball about obj_center inside it (else 0)
};

struct Material {
  int32_t type;
  vec3 albedo;
  float rough;
  vec3 emit;
};

struct DevFrame {
  Pose pose;       // object pose in this frame
  Pose ghost;      // object pose in the other frame (the ghost)
  Material objmat; // object material in this frame
  vec3 olo, ohi;   // padded world bounds of the object at pose
  vec3 glo, ghi;   // padded world bounds of the ghost
  vec3 oc, gc;     // padded bounding spheres of the object at pose and of the ghost:
  float orad;      //   centres and radius (the same for both)
  int32_t ghosts;  // 1 for motion edits
  int32_t same_pose;  // the two frames place the object identically
  int32_t sealed;  // closed convex object with the camera and the emitters outside it
};

// ------------------------------------------------------------------ workspace
// Sub-path vertex records, SoA: record r of slot v of sample s is at
// base[(v * FIELDS + r) * Q + s] (float4), so a wave's lanes touch
// consecutive 16-byte words.
constexpr int kEyeFields = 4;    // pos+md, nrm+pred.n, pred sums+flags, camera-edge crossings
constexpr int kLightFields = 6;  // pos+md, nrm+pred.n, pred sums+flags, light pos+md, light nrm+nee.n, nee sums+ok
constexpr int kStartFields = 5;  // mid pos+md, mid nrm+cam.n, cam sums, x_L pos+md, x_L nrm
constexpr int kTaskFields = 11;  // slot+flags, light walk start (5), eye walk start (5)

struct Workspace {
  float4* eye;
  float4* light;
  float4* start;
  uint32_t* counts;    // per sample: nE | nL << 8
  uint32_t* pairs;     // queue of connected paths: slot << 6 | (i+1) << 3 | (j+1)
  uint32_t* npairs;    // [1] queue length
  float4* records;     // per queued path: pixel (int bits), rgb
  uint32_t* rec_keys;  // optional: dir | tech << 1 | pair << 8  (debug records)
  uint32_t* rec_sample;
  float4* task;        // walk tasks (start phase -> walk phase), SoA: task[field * Q + t]
  uint32_t* ntasks;    // [1] task queue length
  uint32_t* fetch;     // [2] work counters of the walk phase (tasks) and the connect kernel (paths)
  uint32_t* kbins;     // [32] paths per length k, then the sort's cursors per k
  uint32_t* pairs2;    // [pair_cap] the path queue sorted by path length (then ordered back into pairs)
  uint32_t* order;     // [Q] or null: slot s of the round holds the sample of item-order slot order[s]
  uint16_t* okey;      // [Q] the ordering pass's keys
  float4* t8q;         // technique (8) on: per queued path (2 float4), the proposal's
                       // solid-angle density at vertices x_1 .. x_5 (0 where not used)
  int32_t Q;           // samples per chunk
  int64_t pair_cap;
  int32_t nslot;       // vertex slots per side
};

// One residual job: the scene as seen by this job's camera (resolution), the
// two frames (F[0]: new frame with the old pose as ghost, sign +1; F[1]: old
// frame, sign -1), the output image and the sample range of every
// (technique, direction) stream.
struct DevJob {
  DevScene S;
  DevFrame F[2];
  float* image;
  float* tech_images;  // per-technique images (8 x W x H x 3) or null
  // Fixed-point accumulation image (W x H x 3, two's complement in units of
  // fx_unit): the splat adds integers, whose sum does not depend on the
  // order of the additions, so the image is the same bit for bit whatever
  // the scheduling, the round size or the tile size.
  unsigned long long* acc;
  float fx_scale;   // fixed-point units per unit of radiance: 2^40 / (largest emission of the scene)
  double fx_unit;   // 1 / fx_scale
  // samples of technique t (index t-1) relative to the base count N: the
  // weight of its density in the MIS sums (balance heuristic over unequal
  // sample counts; all 1 by default)
  float tech_ratio[8];
  int64_t s0, s1;
  float inv_n;      // 1 / (spp * W * H)
  int32_t tile0;    // first tile of this job in the batch-wide tile index space
  int32_t tilesx;   // tiles per image row
  int32_t W, H;
};

constexpr int kItem = 64;  // samples per work item (one wave)
constexpr int kMaxRound = 1 << 25;  // samples per round: the path code holds slots below 2^26

// Kernel slots of the per-kernel statistics: 1..8 start phase of technique
// t, 17..24 its walk phase, then connect, splat, frame, the proposal's
// densities and technique 8's MLP starts.
constexpr int kKernelSlots = 32;
constexpr int kKidConnect = 9, kKidSplat = 10, kKidFrame = 11, kKidProposalPdf = 12, kKidT8Start = 13,
              kKidStartOrder = 14;
RPI_HD constexpr int kid_start(int t) { return t; }
RPI_HD constexpr int kid_walk(int t) { return 16 + t; }
// Techniques whose walks run in a separate phase over the compacted task
// queue: all but path tracing (7), whose camera rays start a walk in most
// lanes and which runs faster in one kernel (measured).
RPI_HD constexpr bool split_walks(int t) { return t != 7; }
constexpr int kTechs = 8;  // techniques 1..6 of Sec. 4, 7 = path tracing, 8 = learned proposal

// Device view of a learned proposal (technique 8): the MLP's BF16 weights in
// the two layouts its kernels read, FP32 biases, and the normalisation of its
// position input to the object's bounding box in object space.
struct MlpDev {
  const uint16_t* wt1;  // [64][16]  layer 1 transposed ([out][in], inputs 6..15 zero)
  const uint16_t* wt2;  // [64][64]  transposed
  const uint16_t* wt3;  // [64][64]  transposed
  const uint16_t* wt4;  // [48][64]  transposed (outputs 40..47 zero)
  const uint16_t* w2;   // [64][64]  [in][out]
  const uint16_t* w3;   // [64][64]  [in][out]
  const uint16_t* w4;   // [64][48]  [in][out] (outputs 40..47 zero)
  const float* b1;      // [64]
  const float* b2;      // [64]
  const float* b3;      // [64]
  const float* b4;      // [48]
  vec3 center, inv_half;
};

struct DevStats {
  unsigned long long paths, accepted, rejected[7], by_tech[9], rays[6], nodes, tris, samples;
  unsigned long long knodes[kKernelSlots], ktris[kKernelSlots], kbytes[kKernelSlots];
};

// One round of the estimator for one technique: work items g in
// [item0, item0 + nitems) of the batch-wide item list, where
// item_prefix[2 j + d] .. item_prefix[2 j + d + 1] are the items of job j,
// direction d.  Workspace slot of item g, lane l: (g - item0) * 64 + l.
struct WalkArgs {
  const DevJob* jobs;
  int32_t njobs;
  const int64_t* item_prefix;  // [2 * njobs + 1]
  int64_t item0;
  int32_t nitems;
  uint32_t* item_counter;      // work-pulling counter of the persistent walk kernel
  Workspace W;
  DevStats* stats;
  uint32_t k0, k1, job_base;   // Philox key; counter word 2 = job_base + job
  int32_t tech, depth;
  int32_t material_mode;
  uint32_t mask;
  float cweight;
  float alpha_min, d_min, jac_max;
  int32_t no_mapping;          // every path rejected (the path-mapping ablation)
  int32_t balance;             // accepted pairs: balance heuristic over both directions' strategies
  int32_t tech_spp;            // this technique's samples per pixel (0: the job's sample range)
  int32_t count_work;
  int32_t keep_records;
  MlpDev mlp;                  // technique (8) and its MIS term (mask bit 7)
  float* train;                // technique (3) paths -> proposal training records (or null)
  uint32_t* train_count;
  int64_t train_cap;
  int32_t train_weighting;     // 0: |f| / p_gen, 1: |f|^2 / (p_gen * MIS sum)
};

// Tile-binned splat of one record queue.  ntiles * 4 bytes of LDS per
// workgroup hold a tile histogram (ntiles <= 16384).
constexpr uint32_t kSplatChunk = 2048;  // binned records per splat workgroup pass

struct SplatArgs {
  const float4* records;  // x: job << 24 | pixel (int bits), or -1; yzw: rgb
  const uint32_t* nrec;
  int64_t cap;
  const DevJob* jobs;
  const int32_t* tile_job;  // [ntiles]: job of each batch-wide tile
  uint32_t* hist;     // [ntiles * nblk], then its per-tile exclusive scan
  uint32_t* tcount;   // [ntiles]
  uint32_t* toff;     // [ntiles + 1]
  uint32_t* cpre;     // [ntiles + 1]: exclusive scan of the tiles' chunk counts
  float4* binned;     // [cap]
  int ntiles, nblk;
  int ts;             // tile edge in pixels: 16 or 32
};

struct FrameArgs {
  DevScene S;
  DevFrame F;
  DevFrame F2;  // mode 1, 2: the frame subtracted
  float* image;
  uint32_t k0, k1, job;
  int dir, depth, spp, accumulate;
  int mode;     // 0 frame F; 1 F - F2 on the same streams; 2 F - F2 on independent streams
  int64_t s0, s1;
  DevStats* stats;
};

// launchers (rpi_kernels.hip)
void launch_walk(const WalkArgs& A, int blocks, hipStream_t st);        // start phase (persistent over items)
void launch_walk_tasks(const WalkArgs& A, int blocks, hipStream_t st);  // walk phase (over the task queue)
void launch_connect(const WalkArgs& A, int blocks, hipStream_t st);
void launch_sort_pairs(const WalkArgs& A, hipStream_t st);
void launch_start_order(const WalkArgs& A, hipStream_t st);  // fills A.W.order for the round
// zero the jobs' technique images (if any) and fixed-point accumulation images
void launch_zero_images(const DevJob* jobs, int njobs, hipStream_t st);
// fixed-point accumulation -> float: tech = 0: into the job's image (added to
// it with `accumulate`), else into technique image tech - 1; the accumulation
// image is zeroed
void launch_flush_acc(const DevJob* jobs, int njobs, int tech, bool accumulate, hipStream_t st);
// image = (accumulate ? image : 0) + technique image 1 + ... + technique image 8
void launch_sum_technique_images(const DevJob* jobs, int njobs, bool accumulate, hipStream_t st);
void launch_splat(const SplatArgs& a, hipStream_t st);
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st);
void launch_zero_f32(float* p, int64_t n, hipStream_t st);
void launch_frame(const FrameArgs& A, hipStream_t st);
void launch_proposal_pdf(const WalkArgs& A, int blocks, hipStream_t st);
void launch_t8_start(const WalkArgs& A, int blocks, hipStream_t st);

// residual denoiser (rpi_denoise.hip)
void launch_gbuffer(const DevScene& S, const DevFrame& F, float4* g, hipStream_t st);
void launch_denoise(const float* a, const float* b, const float4* g, float4* buf0, float4* buf1, int W, int H,
                    int iterations, float sigma_n, float sigma_z, float sigma_l, float* out, hipStream_t st);

// learned proposal (rpi_train.hip)
constexpr int kMlpNParam = 11368;
constexpr int kMlpHalfElems = 64 * 16 + 64 * 64 + 64 * 64 + 48 * 64 + 64 * 64 + 64 * 64 + 64 * 48;  // BF16 block
constexpr int kMlpPartial = kMlpNParam + 2;  // per-block gradient partial: params, weighted loss, weight sum
struct MlpBufs {  // one device allocation per proposal
  float* master;  // [kMlpNParam] FP32 parameters (flat layout)
  float* adam_m;  // [kMlpNParam]
  float* adam_v;  // [kMlpNParam]
  float* bias;    // b1[64] b2[64] b3[64] b4[48]
  uint16_t* h;    // wt1 wt2 wt3 wt4 w2 w3 w4 (BF16)
};
MlpDev mlp_view(const MlpBufs& B, vec3 center, vec3 inv_half);
void launch_mlp_pack(const MlpBufs& B, hipStream_t st);
void launch_mlp_forward(const MlpDev& M, const float* x, int64_t n, float* out, hipStream_t st);
// Gradient partials of the weighted NLL over `rows` rows into partial[blocks][kMlpPartial]
// (zeroed here).  sampled = 0: row r is record r; else row r draws its record
// uniformly from [0, nrec) by Philox (key k0,k1; counter (r, step)).
void launch_mlp_grad(const MlpDev& M, const float* rec, int64_t nrec, int64_t rows, int sampled, uint32_t k0,
                     uint32_t k1, uint32_t step, float* partial, int blocks, hipStream_t st);
void launch_mlp_reduce(const float* partial, int blocks, float* grad, float* loss, hipStream_t st);
void launch_mlp_adam(const float* partial, int blocks, const MlpBufs& B, float lr, float beta1, float beta2,
                     float eps, int t, float* loss_out, hipStream_t st);

}  // namespace rpi
