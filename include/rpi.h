/*
 * rpi.h -- C ABI of librpi: the residual path estimator of
 * "Residual path integrals for re-rendering" (Xu, Li, Georgiev, Hedstrom,
 * Ramamoorthi, EGSR 2024) on one AMD Instinct MI355X (gfx950).
 *
 * All entry points return an rpi_status (0 = success, negative = error) and
 * never throw across the ABI.  A human-readable message for the last failing
 * call on the calling thread is available from rpi_last_error().
 *
 * Device pointers are plain HIP device addresses (for example the data_ptr
 * of a torch CUDA tensor on ROCm); streams are hipStream_t passed as void*.
 * Rendering calls are asynchronous on the given stream unless they are asked
 * to return statistics, in which case they synchronise that stream.
 *
 * Shared input conventions (see rpi_scene_desc):
 *   - geometry is a triangle soup; triangles of the dynamic / edited object
 *     carry tri_object = 1 and are given at the OLD pose;
 *   - materials are rows of 8 floats: type (0 Lambertian, 1 GGX conductor,
 *     2 one-sided emitter), albedo rgb (GGX: F0), roughness (GGX alpha),
 *     emission rgb;
 *   - images are H x W x 3 float32, row-major, row 0 at the top.
 */
#ifndef RPI_H
#define RPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rpi_status;
#define RPI_OK 0
#define RPI_ERR_INVALID_ARG (-1)   /* malformed input; nothing was launched */
#define RPI_ERR_UNSUPPORTED (-2)   /* well-formed but outside what the library handles */
#define RPI_ERR_OUT_OF_MEMORY (-3) /* a device allocation failed */
#define RPI_ERR_DEVICE (-4)        /* a HIP runtime call failed (sticky device errors included) */

#define RPI_EDIT_RIGID 0
#define RPI_EDIT_MATERIAL 1

/* rpi_render_params.flags */
#define RPI_FLAG_TWO_WAY 1u    /* sample both frames, two-way mapping (motion edits) */
#define RPI_FLAG_ACCUMULATE 2u /* add into the output instead of overwriting it */
#define RPI_FLAG_COUNT_WORK 4u /* count BVH node visits and triangle tests (slower kernels) */
#define RPI_FLAG_RECORDS 8u    /* keep per-path splat records for inspection (rpi_get_records) */
#define RPI_FLAG_TIME_KERNELS 16u /* time every launch with HIP events (per-kernel durations in rpi_stats) */
/* Path mapping off: the ablation of the paper's fig. ablat_pathmapping.
 * Every connected path is treated as rejected (Sec. 5, path rejection), so
 * each frame's dynamic paths keep weight 1 in their own frame and the
 * residual becomes the difference of the two frames' dynamic parts (still
 * unbiased, without the correlation the mapping buys).  Motion edits with
 * RPI_FLAG_TWO_WAY only; anything else is UNSUPPORTED. */
#define RPI_FLAG_NO_MAPPING 32u
/* Per-technique images (the decomposition of the paper's fig.
 * importance_sample): technique t's MIS-weighted share of the residual goes
 * to image t-1 of params.d_technique_images, and d_out receives their sum,
 * added pixel by pixel in technique order 1..8 (onto d_out's contents with
 * RPI_FLAG_ACCUMULATE, else onto zero).  The technique images are always
 * overwritten (zero for techniques that did not run). */
#define RPI_FLAG_PER_TECHNIQUE 64u
/* Balance heuristic across the two directions of the two-way mapping
 * (Sec. 5, two-way path mapping; Sec. 4.3, technique combination).  An
 * accepted pair (x, y = T(x)) is weighted by the balance heuristic over the
 * strategies of both frames instead of the fixed weight c_weight: its value
 * f(x) - f'(y)|T'| is divided by Sigma_f(x) + Sigma_f'(y)|T'|, the sums of
 * the strategy densities that generate x in its own frame and y in the
 * other (|T'| = 1 except for a re-traced x_1, where it is the ratio of the
 * two camera densities).  Rejected paths keep their own frame's sum.  Still
 * unbiased: the two directions' weights of a pair sum to one.  Motion edits
 * with RPI_FLAG_TWO_WAY, without technique 8; anything else is UNSUPPORTED.
 * c_weight is then unused. */
#define RPI_FLAG_BALANCE 128u

typedef struct rpi_scene rpi_scene;
typedef struct rpi_edit rpi_edit;
typedef struct rpi_proposal rpi_proposal;

/* Device-memory hook.  allocate returns `bytes` of device memory (256-byte
 * aligned) or NULL; deallocate returns it.  Both receive the HIP stream the
 * memory is used on (NULL for the scene's own arrays).  deallocate may be
 * called as soon as the work that uses the memory has been enqueued on that
 * stream, before it has run: the allocator must hand the memory out again
 * only in stream order (as hipFreeAsync and PyTorch's caching allocator do).
 * The hook and ctx must stay valid until rpi_destroy_scene returns. */
typedef struct {
  void* (*allocate)(void* ctx, size_t bytes, void* hip_stream);
  void (*deallocate)(void* ctx, void* ptr, void* hip_stream);
  void* ctx;
} rpi_allocator;

/* Scene description.  Every array is host memory, copied by rpi_build_scene;
 * the caller may free it on return. */
typedef struct {
  const float* positions;      /* [3 * num_vertices] */
  int32_t num_vertices;
  const int32_t* indices;      /* [3 * num_triangles], counter-clockwise around the normal */
  int32_t num_triangles;
  const int32_t* tri_material; /* [num_triangles], < num_materials */
  const int32_t* tri_object;   /* [num_triangles], 0 static, 1 dynamic/edited object (one object:
                                  values above 1 are UNSUPPORTED, negative ones INVALID_ARG) */
  const float* materials;      /* [8 * num_materials] */
  int32_t num_materials;
  const float* env;            /* [3] constant environment radiance (0 = none) */
  const float* camera;         /* [12] eye xyz, target xyz, up xyz, vfov_deg, width, height */
} rpi_scene_desc;

/* An edit between the old frame (the scene as given) and the new frame.
 * RIGID: the object moves by old_to_new, a 3x4 row-major rigid transform
 *   (R orthonormal, det +1: the vertex map of Sec. 5 has unit Jacobian).
 * MATERIAL: the object's material becomes new_material in the new frame. */
typedef struct {
  int32_t kind;
  float old_to_new[12];
  float new_material[8];
} rpi_edit_desc;

typedef struct {
  int32_t spp;            /* samples per pixel per technique per direction */
  int32_t max_depth;      /* maximum number of path segments (>= 2) */
  uint64_t seed;          /* Philox key */
  uint32_t strategy_mask; /* bit t-1 enables technique t: 1..6 of Sec. 4, 7 = path tracing,
                             8 = learned proposal (needs proposal) */
  uint32_t flags;         /* RPI_FLAG_* */
  float alpha_min;        /* reconnection roughness threshold (Sec. 5), default 0.2 */
  float d_min;            /* reconnection distance threshold; < 0: 1% of the scene diagonal */
  float jac_max;          /* Jacobian rejection threshold, default 10 */
  float c_weight;         /* two-way weight of accepted pairs, default 0.5 */
  int64_t sample_begin;   /* sample-index range of every (technique, direction) stream */
  int64_t sample_end;     /* < 0: spp * width * height */
  int32_t queue_cap;      /* samples per round, rounded up to a multiple of 64 and
                             capped at 2^25 (0: the tuned or default size) */
  uint32_t job;           /* third Philox counter word (distinct jobs get independent streams) */
  /* Learned proposal (addition beyond the paper): with a non-NULL
   * proposal, strategy_mask bit 7 enables technique 8 -- a start x_D on the
   * object whose light-side direction is drawn from the proposal's lobes,
   * seen by the camera directly (the paths of technique 2) or followed by a
   * BSDF direction and an eye walk (those of technique 3) -- and its term in
   * every path's MIS sum.  The proposal's weights are read when the kernels
   * run (a training step enqueued before the call is seen by it). */
  const rpi_proposal* proposal;
  /* Training-record collection: every path generated by technique 2 or 3 appends
   * one record {x[6], w_obj[3], weight} (10 float32) to d_train_records
   * (device memory, train_capacity records): the proposal input at x_D, the
   * direction x_D -> x_{D+1} in object space, and the mean absolute residual
   * contribution of the path divided by its generation density.  Requires
   * stats (the count is returned in rpi_stats.train_records, records beyond
   * the capacity are dropped).  NULL: off. */
  float* d_train_records;
  int64_t train_capacity;
  /* Record weight: 0 = |f| / p_gen (the directional distribution of residual
   * energy at x_D); 1 = |f|^2 / (p_gen * sum of the path's strategy
   * densities) (its second-moment contribution under the MIS combination:
   * directions the other strategies sample poorly weigh more). */
  int32_t train_weighting;
  /* RPI_FLAG_PER_TECHNIQUE: 8 x H x W x 3 float32 device memory (technique
   * t in image t-1); ignored without the flag. */
  float* d_technique_images;
  /* Splat tile edge in pixels: 16 or 32, 0 = automatic (16 unless the images
   * need more than 16384 tiles).  The image does not depend on it beyond
   * float rounding. */
  int32_t tile;
  /* Samples per pixel of technique t (index t-1); 0: spp.  Techniques then
   * draw unequal sample counts n_t = technique_spp[t-1] * W * H, and every
   * strategy density enters the MIS sums weighted by n_t / (spp * W * H):
   * the balance heuristic over unequal counts (Veach 1997, Sec. 9.2), which
   * keeps the estimator unbiased.  Needs the full sample range
   * (sample_begin 0, sample_end < 0); not available for batches.  See
   * rpi_allocate_samples. */
  int32_t technique_spp[8];
} rpi_render_params;

typedef struct {
  int64_t samples;        /* technique samples drawn */
  int64_t paths;          /* connected paths evaluated and splatted (residual paths) */
  int64_t accepted;       /* paths whose mapped path was accepted */
  int64_t rejected[7];    /* by rule R1..R6 of Sec. 5; index 0: mapping off (RPI_FLAG_NO_MAPPING) */
  int64_t by_tech[9];     /* paths by technique (index 1..8) */
  int64_t rays[6];        /* with RPI_FLAG_COUNT_WORK: closest, shadow, camera, ghost all-hit,
                             mapping re-trace, mapping visibility */
  int64_t nodes_visited;  /* with RPI_FLAG_COUNT_WORK */
  int64_t tris_tested;    /* with RPI_FLAG_COUNT_WORK */
  double milliseconds;    /* device time of the call (when stats are requested) */
  /* Per kernel: index t = 1..8 start phase of technique t, 16 + t its walk
   * phase, 9 connect, 10 splat (all splat kernels of a chunk), 11 frame,
   * 12 proposal densities for the MIS sums, 13 technique-8 starts (MLP),
   * 14 the coherent sample-order pass before each start phase.
   * ms/launches with RPI_FLAG_TIME_KERNELS; node/triangle fetches and bytes
   * written with RPI_FLAG_COUNT_WORK. */
  double kernel_ms[32];
  int64_t kernel_launches[32];
  int64_t kernel_nodes[32];
  int64_t kernel_tris[32];
  int64_t kernel_bytes_written[32];
  int64_t train_records;  /* training records produced (may exceed train_capacity) */
  double technique_ms[9];  /* with RPI_FLAG_TIME_KERNELS: device time of each technique's launches
                              (start and walk phases, connect, splat of its rounds), index 1..8 */
} rpi_stats;

/* Copy, validate and upload a scene: the static geometry and the object
 * of both frames (Sec. 3.2: the inputs are the old frame and the new frame,
 * which differ only by the edited object), with binned-SAH BVHs for the
 * static geometry and for the object in object space, and the area CDFs of
 * the object and the emitters.  allocator: NULL for hipMalloc /
 * hipMallocAsync, else every device allocation of the scene and of the
 * calls made on it goes through it (learned proposals keep their own).
 * Errors: INVALID_ARG (NaN/inf vertex, index out of range, bad material id
 * or type, negative tri_object, zero-area object or emitter, bad camera),
 * UNSUPPORTED (emissive object, object with several materials, several
 * objects (tri_object > 1), no dynamic triangles, no emitter),
 * OUT_OF_MEMORY, DEVICE.  Validation happens before any device work. */
rpi_status rpi_build_scene(const rpi_scene_desc* desc, const rpi_allocator* allocator, rpi_scene** out);
rpi_status rpi_destroy_scene(rpi_scene* scene);

/* Record an edit of the scene's object: a rigid motion (Sec. 5, transform
 * with object movement) or a material change (Sec. 6.2, material editing).
 * The description is validated before the scene is used.  Errors:
 * INVALID_ARG (unknown kind, non-finite, non-orthonormal or mirrored
 * transform, bad or non-finite material, null scene), UNSUPPORTED (emissive
 * new material). */
rpi_status rpi_apply_edit(rpi_scene* scene, const rpi_edit_desc* desc, rpi_edit** out);
rpi_status rpi_destroy_edit(rpi_edit* edit);

/* The residual I2 - I1 (Sec. 3.2, eq. shiftmapped) into d_out
 * (H*W*3 float32, caller-owned device memory), by the dynamic-path
 * techniques of Sec. 4, MIS (Sec. 4.3), path mapping and rejection (Sec. 5).
 * Material edits use techniques 1-3 (and 7 if enabled), one-way.
 * stats may be NULL; when given, the call synchronises hip_stream. */
rpi_status rpi_render_residual(const rpi_scene* scene, const rpi_edit* edit, const rpi_render_params* params,
                               float* d_out, rpi_stats* stats, void* hip_stream);

/* rpi_render_residual for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same estimator, same result up to float rounding (the rounds
 * are smaller); the call allocates nothing: its workspace is a static device
 * array of 128 MiB that each GPU the library runs on holds until the process
 * ends, and rounds are sized to fit it.  The caller still passes the output
 * (and, with RPI_FLAG_PER_TECHNIQUE, the technique images).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race on it and must be serialised by the caller.
 * The call synchronises hip_stream once before its kernels (the round plan
 * is copied from host memory); the kernels then run asynchronously.
 * Errors: as rpi_render_residual; UNSUPPORTED for RPI_FLAG_RECORDS,
 * RPI_FLAG_COUNT_WORK, RPI_FLAG_TIME_KERNELS, training records, and images
 * whose smallest round does not fit the array. */
rpi_status rpi_render_residual_noalloc(const rpi_scene* scene, const rpi_edit* edit, const rpi_render_params* params,
                                       float* d_out, void* hip_stream);

/* Plain path tracing (next-event estimation, emission seen directly) of one
 * frame (Sec. 3.1, eq. pathIntegral): which = 0 old frame, 1 new frame (edit
 * may be NULL: the scene as given).  Sample s of a stream goes to pixel
 * s mod (W*H); the Philox streams are those of technique 7 of
 * rpi_render_residual in the same frame. */
rpi_status rpi_render_frame(const rpi_scene* scene, const rpi_edit* edit, int32_t which,
                            const rpi_render_params* params, float* d_out, void* hip_stream);

/* The baselines the paper compares against (Sec. 6.2, incremental
 * re-rendering): the difference I_new - I_old of two path-traced frames
 * (as rpi_render_frame) into d_out.  correlated = 1: both frames use the
 * same random numbers per sample (correlated path tracing; paths that miss
 * the object's old and new poses cancel exactly); correlated = 0: each frame
 * from its own streams (path tracing from scratch).  Errors as
 * rpi_render_frame; edit must not be NULL. */
rpi_status rpi_render_frame_difference(const rpi_scene* scene, const rpi_edit* edit, int32_t correlated,
                                       const rpi_render_params* params, float* d_out, void* hip_stream);

/* One job of a batch: a rigid edit given by the object's poses in the two
 * frames (3x4 row-major, relative to the scene as given), its own image. */
typedef struct {
  float pose_old[12];
  float pose_new[12];
  int32_t width, height;
  float* d_out;            /* height * width * 3 float32 device memory */
} rpi_job;

/* Many residual jobs (e.g. consecutive frames of an animation) with uneven
 * image sizes (addition beyond the paper, which leaves batching to future work,
 * Sec. 6.3).  The launch sequence (persistent walk kernels pulling 64-sample
 * work items of all jobs, connect, batch-wide tile splat) is captured once
 * into a hipGraph on a library stream and replayed on hip_stream; later calls
 * with the same image sizes and parameters only upload the new poses and
 * output pointers.  Runs the autotuner on the largest job first if the scene
 * is not tuned.  Job j uses Philox counter word params->job + j.  Up to 127
 * jobs and 16384 tiles of 32x32 pixels in total.  stats may be NULL.
 * With RPI_FLAG_COUNT_WORK or RPI_FLAG_TIME_KERNELS the same plan and kernels
 * run without the graph (instrumented or timed per launch; the scene must be
 * tuned).  Errors as above; records and per-technique images are UNSUPPORTED. */
rpi_status rpi_render_residual_batch(const rpi_scene* scene, const rpi_job* jobs, int32_t num_jobs,
                                     const rpi_render_params* params, rpi_stats* stats, void* hip_stream);

/* Residual-aware sample allocation (addition beyond the paper, which
 * gives every technique the same sample count).  A pilot of pilot_spp
 * samples per pixel, in two independent halves with per-technique images,
 * measures for each enabled technique t the variance V_t of its MIS-weighted
 * share of the residual (the squared difference of the halves, summed over
 * pixels) and its device time per sample c_t; technique_spp_out[t-1]
 * receives n_t / (W*H) with n_t ~ sqrt(V_t / c_t) (Neyman allocation over
 * the techniques taken as strata), scaled so that the total cost equals that
 * of params->spp for every technique, rounded, and kept in [1, 64 spp]
 * (0 for techniques that do not run).  Pass the result in
 * params.technique_spp: the balance heuristic over the unequal counts keeps
 * the estimator unbiased.  Synchronises hip_stream.  Errors as
 * rpi_render_residual; INVALID_ARG for pilot_spp < 2. */
rpi_status rpi_allocate_samples(const rpi_scene* scene, const rpi_edit* edit, const rpi_render_params* params,
                                int32_t pilot_spp, int32_t* technique_spp_out, void* hip_stream);

/* Residual-aware denoising (addition beyond the paper, which leaves the
 * residual's noise around the edit to an external denoiser, Sec. 6,
 * limitations).  d_a and d_b are two independent estimates of the residual
 * (rpi_render_residual on the sample ranges [0, N/2) and [N/2, N) of every
 * stream, each divided by the full N, so that R = a + b); d_out (H x W x 3
 * float32, may alias neither input) receives R filtered by an
 * edge-avoiding a-trous wavelet transform (Dammertz et al. 2010): 5x5
 * B3-spline taps at strides 1, 2, 4, ..., weighted by the new frame's
 * normals and hit distances (one camera ray per pixel centre) and by the
 * luminance difference in units of the residual's standard deviation, which
 * is estimated per pixel as (a - b)^2 and carried through the passes with
 * squared weights (Schied et al. 2017).  Pixels no dynamic path reached
 * (a = b = 0) have zero variance and keep their zero.  The filter trades
 * bias for variance: its output is not an unbiased estimate.  Workspace
 * (48 bytes per pixel) comes from the scene's allocator.  Asynchronous.
 * Errors: INVALID_ARG (null pointers, iterations outside 0..10, negative or
 * non-finite sigmas). */
typedef struct {
  int32_t iterations;  /* a-trous passes (strides 1, 2, 4, ...), 0: 3 */
  float sigma_normal;  /* exponent of the normal weight max(0, n_p . n_q)^sigma, 0: 64 */
  float sigma_depth;   /* hit-distance tolerance relative to the centre's distance, 0: 0.1 */
  float sigma_value;   /* luminance tolerance in standard deviations of the centre's residual, 0: 2 */
} rpi_denoise_params;

rpi_status rpi_denoise_residual(const rpi_scene* scene, const rpi_edit* edit, const float* d_a, const float* d_b,
                                const rpi_denoise_params* params, float* d_out, void* hip_stream);

/* The guide of rpi_denoise_residual: per pixel (row-major, H x W x 4 float32)
 * the geometric normal facing the camera and the hit distance of the ray
 * through the pixel centre in frame `which` (0 old, 1 new); (0, 0, 0, -1)
 * where the ray leaves the scene.  Asynchronous. */
rpi_status rpi_render_gbuffer(const rpi_scene* scene, const rpi_edit* edit, int32_t which, float* d_gbuf,
                              void* hip_stream);

/* Launch configuration chosen by the autotuner. */
typedef struct {
  int32_t queue_cap;              /* samples per round */
  int32_t walk_blocks_per_cu;     /* persistent walk workgroups per compute unit */
  int32_t connect_blocks_per_cu;  /* connect workgroups per compute unit */
  double ms_per_msample;          /* measured device time per million technique samples */
} rpi_tuning;

/* Time a small grid of launch configurations (round size 2^23, 2^24 or 2^25,
 * persistent walk grid 16 or 32 blocks per CU) on the first 2^24 samples of
 * every stream of this edit and keep the fastest for later calls on this
 * scene whose queue_cap is 0.
 * Synchronises hip_stream.  out may be NULL. */
rpi_status rpi_autotune(rpi_scene* scene, const rpi_edit* edit, const rpi_render_params* params, rpi_tuning* out,
                        void* hip_stream);

/* Use a launch configuration measured earlier (for example by rpi_autotune
 * in another process) for later calls on this scene whose queue_cap is 0.
 * Errors: INVALID_ARG (queue_cap not a positive multiple of 64 or above
 * 2^25, the most samples a round's path codes can address, or blocks per CU
 * outside [1, 64]). */
rpi_status rpi_set_tuning(rpi_scene* scene, const rpi_tuning* tuning);

/* The launch configuration later calls on this scene with queue_cap 0 use
 * (the tuned one, else the defaults: rounds of 2^20 samples, 16 walk and 16
 * connect workgroups per CU); ms_per_msample is 0. */
rpi_status rpi_get_tuning(const rpi_scene* scene, rpi_tuning* out);

/* Per-path records of the last rpi_render_residual call on this scene made
 * with RPI_FLAG_RECORDS (host copy): each record is 8 int32/float words
 * {dir, tech, sample, pair(i<<8|j), pixel, r, g, b}.  Returns the count in
 * *count; copies at most cap records. */
rpi_status rpi_get_records(const rpi_scene* scene, void* host_out, int64_t cap, int64_t* count);

/* ------------------------------------------------------------------------
 * Learned proposal (addition beyond the paper, which names better sampling of
 * the residual integrand as future work, Sec. 7).  An MLP with inputs
 * (position of a point on the object normalised to the object's bounding box
 * in object space, its object-space normal), three hidden layers of 64 ReLU
 * units and 40 outputs parameterises a mixture of 8 von Mises-Fisher lobes
 * over object-space directions: lobe l has mean normalize(out[5l..5l+2]),
 * concentration softplus(out[5l+3]) + 0.01 (sampling clamps it at 1e4) and
 * weight softmax(out[5l+4]).  Parameters are one float32 vector of
 * RPI_PROPOSAL_NPARAM values: W1[6][64] b1[64] W2[64][64] b2[64] W3[64][64]
 * b3[64] W4[64][40] b4[40], weights row-major [in][out].  Kernels compute in
 * BF16 x BF16 -> FP32 on the matrix cores; FP32 masters and Adam state stay
 * on the device.  A proposal belongs to the device current at creation; calls
 * on one proposal must not overlap.
 * ---------------------------------------------------------------------- */
#define RPI_PROPOSAL_NPARAM 11368
#define RPI_PROPOSAL_INPUTS 6
#define RPI_PROPOSAL_OUTPUTS 40
#define RPI_TRAIN_RECORD_FLOATS 10

typedef struct {
  int32_t steps;  /* Adam steps */
  int32_t batch;  /* records per step, drawn uniformly with replacement (multiple of 64, <= 1<<20) */
  float lr, beta1, beta2, eps;
  uint64_t seed;  /* Philox key of the record draws */
} rpi_train_params;

/* Create a proposal for the scene's object.  params: host float32
 * [RPI_PROPOSAL_NPARAM], or NULL for He-uniform initial weights (zero
 * biases) drawn from seed.  Errors: INVALID_ARG (null scene/out, non-finite
 * parameter), OUT_OF_MEMORY, DEVICE. */
rpi_status rpi_proposal_create(const rpi_scene* scene, const float* params, uint64_t seed, rpi_proposal** out);
rpi_status rpi_proposal_destroy(rpi_proposal* proposal);

/* Replace / read the float32 parameters (host memory, RPI_PROPOSAL_NPARAM
 * values); set_weights also resets the Adam moments and step.  Both
 * synchronise the device. */
rpi_status rpi_proposal_set_weights(rpi_proposal* proposal, const float* params);
rpi_status rpi_proposal_get_weights(const rpi_proposal* proposal, float* params);

/* Raw outputs for n inputs: d_x float32 [n][6] (already normalised), d_out
 * float32 [n][40]; device memory.  Asynchronous on hip_stream. */
rpi_status rpi_proposal_forward(const rpi_proposal* proposal, const float* d_x, int64_t n, float* d_out,
                                void* hip_stream);

/* Weighted mean negative log-likelihood of n records (device float32
 * [n][10]: x[6], w_obj[3], weight) and its gradient: d_grad float32
 * [RPI_PROPOSAL_NPARAM], d_loss float32 [1] (may be NULL), both divided by
 * the sum of the weights (0 if it is not positive).  Asynchronous. */
rpi_status rpi_proposal_loss_grad(const rpi_proposal* proposal, const float* d_records, int64_t n, float* d_grad,
                                  float* d_loss, void* hip_stream);

/* Adam on the records (device float32 [n][10]); d_losses (may be NULL)
 * receives the loss of every step (float32 [steps]).  Asynchronous on
 * hip_stream; later renders on that stream use the updated weights.
 * Errors: INVALID_ARG (n < 1, bad train params). */
rpi_status rpi_proposal_train(rpi_proposal* proposal, const float* d_records, int64_t n,
                              const rpi_train_params* train, float* d_losses, void* hip_stream);

/* Wait for the work enqueued on hip_stream and report a device error that
 * it raised (kernel faults are sticky in HIP and would otherwise surface in
 * a later call).  Returns RPI_OK or DEVICE. */
rpi_status rpi_sync_status(void* hip_stream);

/* Thread-local message of the last error. */
const char* rpi_last_error(void);

/* Library version string. */
const char* rpi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPI_H */
