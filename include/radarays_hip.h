/*
 * radarays_hip.h -- C ABI of the MI355X radar-scan library.
 *
 * The library simulates a rotating FMCW radar the way RadaRays does (Mock,
 * Magnusson, Hertzberg, Sec. III): for every azimuth of the spinning sensor
 * it draws rays from a Gaussian beam cone, traces them through a triangle
 * mesh with reflection and refraction (Snell + Fresnel), returns part of
 * the energy of every hit to the sensor through the paper's standard BRDF,
 * and sums the returns into an azimuth x range polar image.
 *
 * Conventions
 *  - All functions return an rr_status (0 = success).  On failure nothing has
 *    been enqueued on the stream and outputs are untouched, except where a
 *    function says otherwise.  rr_last_error() gives a message.
 *  - Pointers named *_dev are device pointers on the context's GPU; all
 *    other pointers are host pointers.  The library copies every host input
 *    before returning; the caller keeps ownership of its buffers.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Scan calls are
 *    asynchronous on that stream unless a stats pointer is passed.
 *  - A context is not thread-safe; use one per host thread or lock.  A
 *    context's internal workspace is shared by its scans: scans of one
 *    context on different streams must not overlap in time (use
 *    rr_radar_scan_ws with separate workspaces, or separate contexts).
 *  - Triangle ids in records and statistics are the caller's original
 *    indices into `indices`.
 */
#ifndef RADARAYS_HIP_H
#define RADARAYS_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rr_status;
#define RR_OK 0
#define RR_EINVAL (-1)    /* invalid argument; nothing launched */
#define RR_ENOMEM (-2)    /* device/host allocation failed or over budget */
#define RR_EDEVICE (-3)   /* HIP runtime error */
#define RR_ESTATE (-4)    /* call order violated (e.g. scan before bvh_build) */
#define RR_EOVERFLOW (-5) /* a ray-queue capacity invariant was violated */

/* sensor flags */
#define RR_BEAM_GAIN 1u      /* weight returns by the receive gain exp(-z^2/2) */
#define RR_FIXED_PATTERN 2u  /* every azimuth uses the same cone offsets */
#define RR_MIRROR_PAIRS 4u   /* odd rays mirror the azimuth offset of ray i-1 */
#define RR_RETURN_ALL 8u     /* return all reflected energy (w = 1; lidar-like) */
/* Also return along the air path (Sec. III-A, multi-path reflection): from
 * every hit at depth >= 1 of a ray in air, straight back to the sensor when
 * the sensor is on the incoming side of the surface and no triangle blocks
 * the segment (one visibility ray each).  Window angle between the mean
 * reflection and the direction to the sensor; energy taken from the
 * reflected share (at most what the retrace return left); range = half the
 * round trip; receive gain (with RR_BEAM_GAIN) from the angle between the
 * beam axis and the arrival direction.  Needs a four-wide BVH and the
 * level-by-level launches (EINVAL otherwise).  The visibility rays of every
 * level are traced together in one launch after the last level; the
 * workspace grows by 48 bytes per possible hit at depth >= 1,
 * N_p (2^B - 2). */
#define RR_AIR_PATH 16u

/* material kinds */
#define RR_DIELECTRIC 0u /* Fresnel reflection + Snell refraction, lossless */
#define RR_METAL 1u      /* reflects `reflectance`, absorbs the rest */
#define RR_LAMBERTIAN 2u
#define RR_COOK_TORRANCE 3u /* reflects `reflectance` (albedo), absorbs the rest */

/* limits */
#define RR_MAX_BOUNCES 8u
#define RR_MAX_MATERIALS 255u
#define RR_MAX_AZIMUTH 65535u
#define RR_MAX_RAYS_PER_BEAM (1u << 20)
#define RR_MAX_BINS 65535u
#define RR_MAX_PRIMARIES (1u << 26) /* n_azimuth * rays_per_beam */

typedef struct rr_context rr_context;
typedef struct rr_scene rr_scene;

/* Sensor pose in the world frame.  Sensor frame: +x = azimuth 0, +z = the
 * rotation axis; azimuth k points at angle 2*pi*k/n_azimuth counter-clockwise
 * about +z (Sec. III-B).  The quaternion (w, x, y, z) is normalised by the
 * library and rejected if its norm is off by more than 1e-3. */
typedef struct {
  float position[3];
  float quat_wxyz[4];
} rr_pose;

/* Per-scan sensor parameters (Sec. III-A, III-B, IV).
 *  n_azimuth      columns of the polar image, 1..65535
 *  rays_per_beam  N_s primary rays per azimuth, 1..2^20 (each carries 1/N_s
 *                 of the azimuth's unit emitted energy, Sec. III-A)
 *  max_bounces    B: interactions per path, 1..8; returns are computed at
 *                 every interaction, children spawn while depth + 1 < B
 *  n_bins         rows of the image, 1..65535
 *  bin_size_m     range bin width; a return lands in floor(range/bin_size)
 *                 where range is the one-way optical path length; returns
 *                 at or beyond n_bins * bin_size are dropped
 *  beam_width_rad b in [0, pi): beam width of Eq. 2 and the window of Eq. 4
 *  beam_prob      P in (0, 1): probability of a ray inside b/2 (Eq. 2)
 *  energy_cutoff  children whose energy is <= this are not traced (>= 0)
 *  seed, scan_id  key of the counter-based generator of the ray samples
 *  flags          RR_* sensor flags
 *  beam_stretch_az, beam_stretch_inc
 *                 elliptic beam (Sec. III-A): the drawn cone offsets are
 *                 scaled by these factors along azimuth and inclination,
 *                 0..100 (0 = 1, the circular cone); the receive gain keeps
 *                 the drawn radius */
typedef struct {
  uint32_t n_azimuth, rays_per_beam, max_bounces, n_bins;
  float bin_size_m, beam_width_rad, beam_prob, energy_cutoff;
  uint64_t seed;
  uint32_t scan_id, flags;
  float beam_stretch_az, beam_stretch_inc;
} rr_sensor_params;

/* Material (Sec. III-A; Eq. 5 parameters, S = 1 - A - B).
 *  kind        RR_DIELECTRIC / RR_METAL / RR_LAMBERTIAN / RR_COOK_TORRANCE
 *  n           refractive index of a dielectric (> 0), ignored otherwise
 *  reflectance reflected share for metal and Lambertian, in [0, 1]
 *  A, B, C     lobe parameters: A, B in [0, 1], A + B <= 1, C >= 0
 * RR_COOK_TORRANCE (a user-defined BRDF as in Sec. IV): Cook-Torrance with
 * the GGX distribution and separable Smith masking (Walter et al. 2007),
 *   f = A / pi + (1 - A) D(h) F(v.h) G1(n.l) G1(n.v) / (4 (n.l)(n.v)),
 * A = diffuse amount in [0, 1], B = roughness alpha in [1e-4, 1], n = index
 * of the Fresnel factor (> 0, also the index of refraction of the
 * transmitted share), reflectance = reflected share (1 - transmittance), C
 * ignored.  The share returned into the beam window around a return
 * direction v is f (n.v) 2 pi (1 - cos(b/2)), at most 1; the transmitted
 * share refracts by Snell's law. */
typedef struct {
  uint32_t kind;
  float n, reflectance, A, B, C;
} rr_material;

/* BVH build options (all zero = defaults). */
typedef struct {
  uint32_t max_leaf_size; /* triangles per leaf, 1..16 (1..4 for width 8), default 2 */
  uint32_t sah_bins;      /* SAH bins per axis, 4..64, default 16 */
  uint32_t n_threads;     /* host build threads, 0 = all cores */
  uint32_t split_pct;     /* early split clipping: extra triangle references, in
                             percent of the triangle count, 0..200 (0 = none) */
  uint32_t width;         /* children per node: 4 (default) or 8 (compressed
                             eight-wide nodes, leaves of at most 4 triangles) */
  uint32_t merge_leaves;  /* 0: default (1); 1: the binary build goes down to
                             single triangles and the wide collapse forms
                             leaves of at most max_leaf_size references
                             (always so for width 8); 2: leaves are those of
                             the binary SAH build */
  uint32_t builder;       /* 0: binned SAH on the host (default); 1: linear BVH
                             built on the GPU (Morton-sorted triangles, binary
                             radix tree, collapsed to four-wide nodes; leaves are
                             subtrees of at most max_leaf_size triangles; width 4
                             and split_pct 0 only) -- about ten times faster to
                             build, slower to trace; either builder's four-wide
                             tree can be refitted (rr_bvh_refit) */
  uint32_t collapse;      /* host builder, width 4: how the binary SAH tree is
                             collapsed into four-wide nodes.  0: default (2);
                             1: greedy, each node opens its largest-area inner
                             child until it has four; 2: cost-optimal, a
                             dynamic program over the binary tree minimises
                             the expected surface-area cost of node steps and
                             triangle tests.  Ignored by the GPU builder and
                             for width 8. */
  int32_t spatial_pct;    /* host builder: spatial splits (a reference that
                             straddles a split plane goes to both sides,
                             bounded by its triangle's part on each side,
                             where the surface-area cost says so), extra
                             triangle references allowed, in percent of the
                             triangle count: 0 default (10), 1..200, -1 none.
                             The build takes about four times as long (2 M
                             triangles: ~2 s on 16 cores), more on meshes of
                             long triangles crossing one another (200 k random
                             slivers: 9.6 s instead of 0.3 s).  The GPU builder
                             takes 0 or -1. */
} rr_bvh_options;

typedef struct {
  uint32_t n_tris;        /* triangles in the scene */
  uint32_t n_hittable;    /* non-degenerate triangles placed in the BVH */
  uint32_t n_nodes;       /* wide inner nodes */
  uint32_t n_leaves;
  uint32_t max_depth;     /* deepest inner node (root = 0) */
  uint32_t max_stack;     /* worst-case traversal stack entries */
  uint64_t device_bytes;  /* nodes + triangles resident on the GPU */
  double sah_cost;
  double build_ms;
} rr_bvh_info;

/* Filled when a scan is given a stats pointer (the call then waits for the
 * stream).  segments = closest-hit queries traced (misses included). */
typedef struct {
  uint64_t segments;
  uint64_t rays_per_depth[RR_MAX_BOUNCES];
  uint32_t overflow; /* nonzero: a ray queue overflowed (a library bug) */
  uint32_t air_rays; /* air-path visibility rays traced (RR_AIR_PATH) */
} rr_scan_stats;

/* One scan of a batch. */
typedef struct {
  rr_pose pose;
  rr_sensor_params params;
  float* image_dev; /* n_azimuth * n_bins floats, row-major [azimuth][bin] */
  /* Optional (NULL: every primary): n_azimuth * rays_per_beam bytes in device
   * memory, primary k * rays_per_beam + i traced only if its byte is nonzero
   * (parity sampling, as the primary_mask of rr_radar_scan_records).  The
   * image then holds the returns of the traced primaries only.  Read on the
   * stream when the scans run; the caller keeps it valid until then. */
  const uint8_t* primary_mask_dev;
} rr_scan_desc;

/* ---------------------------------------------------------------- context */
const char* rr_status_str(rr_status s);

/* Create a context on HIP device `device` (>= 0).  ENOMEM/EDEVICE on failure. */
rr_status rr_create(int device, rr_context** out);
/* Waits for the device, frees everything the context owns.  NULL is a no-op. */
rr_status rr_destroy(rr_context* ctx);
/* Message of the last failure on this context (or of the last context-less
 * failure when ctx is NULL).  Never NULL. */
const char* rr_last_error(const rr_context* ctx);

/* ---------------------------------------------------------------- scene */
/* The scene is the triangle mesh every ray of a scan is traced against (Sec.
 * III-A: rays travel through a triangle mesh of the environment; Sec. III-D:
 * the ray-tracing engine holds the mesh in an acceleration structure on the
 * device that computes the scan).
 * Copy a triangle mesh into the library (host side).  vertices: nv x 3 float
 * (finite, |x| <= 1e7); indices: nt x 3 (each < nv); tri_material: nt ids
 * (checked against the material table at scan time).  nt may be 0.
 * Zero-area triangles are kept but can never be hit (no normal).  ctx may
 * be NULL: the scene then lives on the host only (BVH build and the host
 * self-check work; scans need a scene created with a context). */
rr_status rr_scene_upload(rr_context* ctx, const float* vertices, uint32_t nv,
                          const uint32_t* indices, uint32_t nt, const uint16_t* tri_material,
                          rr_scene** out);

/* Build the bounding-volume hierarchy on the host (binned SAH, collapsed to
 * four-wide nodes with 8-bit quantised child boxes) and copy nodes and
 * triangles to the context's GPU.  This is the acceleration structure of the
 * ray-tracing engine (Sec. III-D, whose run time grows with the logarithm of
 * the triangle count).  Synchronous.  After it
 * the scene is immutable and may be shared by concurrent scans.  opt may be
 * NULL.  Calling it again rebuilds, which frees the previous device copies:
 * ESTATE while a graph (rr_graph_create) or a server (rr_server_create) of
 * this scene exists, since their launches point at those copies. */
rr_status rr_bvh_build(rr_context* ctx, rr_scene* scene, const rr_bvh_options* opt);

rr_status rr_bvh_get_info(const rr_scene* scene, rr_bvh_info* out);

/* Moves the vertices of a scene with a four-wide BVH on the device:
 * vertices_dev holds nv x 3 floats in device memory, nv equal to the count
 * uploaded, indices and materials unchanged (for moving objects).  The tree
 * keeps its structure and leaf order; triangles, normals, child boxes and
 * node frames are recomputed on the GPU, one launch per tree depth, deepest
 * first, stream-ordered on `stream`, so scans issued after it on that stream
 * see the new geometry.  The caller keeps vertices_dev valid and unchanged
 * until the refit has run on `stream` (it is read there, not copied on the
 * call), and orders it after scans of this scene on other streams (the tree
 * is rewritten in place).  Either builder's tree can be refitted (a host SAH
 * tree keeps its better structure while objects move a little).  A tree
 * built on the GPU refits with no allocation; the first refit of a
 * host-built tree sets up its refit state synchronously (device copies of
 * indices and materials, the nodes grouped by depth and a box per node: 14
 * bytes per triangle and 28 per node), later ones allocate nothing.  Triangles that were degenerate at
 * build time stay out of the tree; child boxes of split references grow to
 * whole triangles, so a tree built with spatial or early splits loses their
 * tightness and keeps their extra references (urban block: 2.06 ms per scan
 * after a refit back to the built vertices, 1.83 before): build trees meant
 * for refitting with spatial_pct = -1.  The host copy of the mesh is not
 * changed, so
 * rr_bvh_build afterwards builds from the uploaded vertices.  ESTATE
 * without a device BVH; EINVAL for a NULL pointer, an eight-wide tree or a
 * vertex count other than the uploaded one (coordinates in device memory
 * are not checked). */
rr_status rr_bvh_refit(rr_context* ctx, rr_scene* scene, const float* vertices_dev, uint32_t nv,
                       void* stream);

/* Host check of the built hierarchy: traces n_rays random rays (origins in
 * the scene bounds, seeded) through it on the CPU and through a brute-force
 * loop over all triangles, and counts closest hits that differ. */
rr_status rr_bvh_selfcheck(const rr_scene* scene, uint32_t n_rays, uint64_t seed,
                           uint64_t* mismatches);

/* Frees the scene (host and device copies).  The caller must have waited for
 * scans that use it.  ESTATE (nothing freed) while a graph or a server of this
 * scene exists. */
rr_status rr_scene_release(rr_context* ctx, rr_scene* scene);

/* ---------------------------------------------------------------- scans */
/* Exact device bytes one scan with these parameters needs as workspace in
 * the default launch mode, for memory admission of scan requests.  The sizes
 * follow the ray tree of Sec. III-A: N_p = n_azimuth * rays_per_beam primaries
 * (Sec. III-A/B, rays sampled per azimuth), and every interaction may spawn a
 * reflected and a refracted child until max_bounces interactions, so bounce
 * level d holds at most N_p * 2^d rays.  Contents: two ray queues of N_p * 2^(B-1) rays, the hit
 * buffer, the fixed-point accumulator, the counters and the traversal-stack
 * spill area.  With rr_tuning.fused = 1 a context also reserves a child pool
 * and hit ring per trace wave (about 1.2 GB) in its own workspace; a
 * caller-provided workspace of this size is then too small (EINVAL).
 * EINVAL if the parameters are out of range. */
rr_status rr_workspace_query(const rr_sensor_params* params, size_t* bytes);

/* One polar image (Sec. III-A, III-B).  image_dev receives n_azimuth x n_bins
 * floats, row-major [azimuth][bin]: the energy returned into each range bin
 * as a fraction of the azimuth's unit emitted energy (linear, no dB).  The
 * image is fully overwritten.  Accumulation uses 64-bit fixed-point integer
 * atomics, so results are bit-identical from run to run.  The workspace is
 * owned by the context and grown on demand. */
rr_status rr_radar_scan(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                        const rr_sensor_params* params, const rr_material* materials,
                        uint32_t n_materials, float* image_dev, rr_scan_stats* stats,
                        void* stream);

/* As rr_radar_scan with a caller-provided workspace of at least
 * rr_workspace_query() bytes (device memory, 256-byte aligned).  Scans on
 * different workspaces may overlap on different streams. */
rr_status rr_radar_scan_ws(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                           const rr_sensor_params* params, const rr_material* materials,
                           uint32_t n_materials, float* image_dev, void* workspace_dev,
                           size_t workspace_bytes, rr_scan_stats* stats, void* stream);

/* Allocation-free variant of rr_radar_scan, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same kernels and the same image,
 * bit for bit; the workspace is a fixed device array of rr_scratch_bytes()
 * bytes (64 MiB) that the library holds on every device it runs on, from
 * its load to the end of the process, instead of the context's workspace.
 * The call makes no hipMalloc, hipFree or other device allocation.  The
 * traversal-stack spill area in it is sized for the scene's tree (none for
 * a tree whose worst-case stack fits the 16 LDS entries per lane), so the
 * scans that fit are those of modest size: a 400 x 64 ray, three-bounce
 * scan of a small scene needs about 15 MB.  ENOMEM (nothing launched) when
 * the scan's workspace exceeds the array; EINVAL for an eight-wide tree or
 * the one-launch mode (rr_tuning.fused = 1).  Every call on one device
 * shares that device's array, which keeps the last call's contents (each
 * call's first kernel clears the counters and the accumulator it uses):
 * calls that overlap on one device, on any streams or contexts, race, so
 * the caller orders them.  Profiling (rr_profile_enable) is ignored. */
rr_status rr_radar_scan_noalloc(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                                const rr_sensor_params* params, const rr_material* materials,
                                uint32_t n_materials, float* image_dev, rr_scan_stats* stats,
                                void* stream);
/* Size of the array rr_radar_scan_noalloc works in, bytes. */
rr_status rr_scratch_bytes(size_t* bytes);

/* Debug/parity variant of rr_radar_scan.  Optional outputs (NULL = skip):
 *  records_dev  int32 [n_azimuth * rays_per_beam][2^B - 1], heap order per
 *               primary (slot h-1 for heap id h; 1 = primary, 2h = reflected
 *               child, 2h+1 = refracted child): original triangle id of the
 *               segment's hit, -1 for a miss, -2 for a segment never spawned.
 *               With RR_AIR_PATH each primary has 2 (2^B - 1) entries; the
 *               second half holds the air-path outcome of each segment's
 *               hit: -2 none, 0 returned, 1 blocked, 2 beyond the last bin.
 *               EINVAL if n_azimuth * rays_per_beam * entries >= 2^32.
 *  accum_dev    uint64 [n_azimuth * n_bins]: the fixed-point accumulator
 *               (energy * 2^56) the image is converted from
 * primary_mask_dev (optional) uint8 [n_azimuth * rays_per_beam]: primaries
 * with a zero byte are not traced at all. */
rr_status rr_radar_scan_records(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                                const rr_sensor_params* params, const rr_material* materials,
                                uint32_t n_materials, const uint8_t* primary_mask_dev,
                                float* image_dev, int32_t* records_dev, uint64_t* accum_dev,
                                rr_scan_stats* stats, void* stream);

/* Many scans (poses, azimuth counts, rays per beam and bounce limits may all
 * differ; the beam width must be shared) traced together: per group of
 * scans one ray-generation launch, one trace and one shade launch per bounce
 * level over the rays of every scan of the group, one finalize.  Groups are
 * consecutive scans whose workspace fits the context's batch budget
 * (rr_tuning.batch_budget_mb, default 24 GiB).  Each image equals what
 * rr_radar_scan gives for that scan, bit for bit.  stats (optional) sums
 * over the batch. */
rr_status rr_radar_scan_batch(rr_context* ctx, const rr_scene* scene, const rr_scan_desc* scans,
                              uint32_t n_scans, const rr_material* materials,
                              uint32_t n_materials, rr_scan_stats* stats, void* stream);

/* Workspace bytes rr_radar_scan_batch needs for these scans. */
rr_status rr_batch_workspace_query(const rr_scan_desc* scans, uint32_t n_scans, size_t* bytes);

/* ---------------------------------------------------------------- epilogue */
/* Polar-image epilogue (Sec. III-B "Polar Image", Sec. III-C "Noise"), in
 * float64, in this order for each pixel (azimuth k, bin b) of an image E:
 *  1. measurement noise: E is blurred along range with a Gaussian of
 *     blur_sigma_bins bins: taps |m| <= ceil(3 sigma), weights
 *     exp(-m^2 / (2 sigma^2)) normalised to sum 1, zero beyond the column
 *     ends (sigma = 0: no blur);
 *  2. system noise: + uniform_amp * u, u in [0, 1) from word (b mod 4) of
 *     Philox4x64-10 with key (seed, scan_id) and counter (k, b div 4, 1, 0),
 *     u = (word >> 11) * 2^-53;
 *  3. ambient noise: + perlin_amp * (1 + n) / 2, n in [-1, 1] the 2-D
 *     gradient noise of Perlin (SIGGRAPH 2002, quintic fade) at
 *     (k / perlin_cell_az, b / perlin_cell_bins); the gradient of lattice
 *     point (i, j) is entry (top 3 bits of word 0 of Philox with counter
 *     (i, j, 2, 0)) of (1,1), (-1,1), (1,-1), (-1,-1), (1,0), (-1,0), (0,1),
 *     (0,-1);
 *  4. L = 10 log10(E) dB (the image is a fraction of the emitted energy, so
 *     E_0 = 1), -inf for E <= 0;
 *  5. pixel = floor(max_value * (L - db_floor) / (0 - db_floor) + 1/2),
 *     clamped to [0, max_value]: 0 dB and above give max_value. */
typedef struct {
  float blur_sigma_bins;  /* 0..16 */
  float uniform_amp;      /* >= 0 (0 = no system noise) */
  float perlin_amp;       /* >= 0 (0 = no ambient noise) */
  float perlin_cell_az;   /* lattice spacing in azimuth columns, >= 1 when perlin_amp > 0 */
  float perlin_cell_bins; /* lattice spacing in range bins, >= 1 when perlin_amp > 0 */
  float db_floor;         /* dB that maps to pixel 0, finite and < 0 (e.g. -100) */
  uint32_t max_value;     /* pixel value at 0 dB, 1..255 */
  uint32_t reserved0;     /* must be 0 */
  uint64_t seed;
  uint32_t scan_id;       /* image i of a call uses scan_id + i */
  uint32_t reserved1;     /* must be 0 */
} rr_post_params;

/* Epilogue of n_images float images of n_azimuth x n_bins, contiguous,
 * row-major [image][azimuth][bin], in device memory (images_dev).  Outputs
 * (device memory, same layout, either may be NULL but not both): db_dev
 * float32 dB (step 4), u8_dev 8-bit pixels (step 5).  The outputs must not
 * overlap the input.  n_images, n_azimuth, n_bins in 0..65535 (0 = nothing
 * to do).  Stream-ordered on `stream` (NULL = the default stream); no
 * allocation.  EINVAL for out-of-range parameters or NULL pointers. */
rr_status rr_postprocess(rr_context* ctx, const float* images_dev, uint32_t n_images, uint32_t n_azimuth,
                         uint32_t n_bins, const rr_post_params* post, float* db_dev, uint8_t* u8_dev,
                         void* stream);

/* rr_radar_scan with the epilogue fused into the scan's last launch: the
 * fixed-point accumulator is converted to the float image (written to
 * image_dev unless NULL) and steps 1-5 run on it in the same launch.  The
 * outputs equal rr_radar_scan followed by rr_postprocess of its image with
 * the same post parameters, bit for bit.  At least one of image_dev, db_dev
 * and u8_dev must be non-NULL. */
rr_status rr_radar_scan_post(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                             const rr_sensor_params* params, const rr_material* materials,
                             uint32_t n_materials, const rr_post_params* post, float* image_dev,
                             float* db_dev, uint8_t* u8_dev, rr_scan_stats* stats, void* stream);

/* ---------------------------------------------------------------- serving */
/* A server owns a context and a resident scene and turns a stream of scan
 * requests into batches (continuous batching).  Requests wait in arrival
 * order; whenever one of the server's slots is free, the dispatcher admits
 * the oldest waiting requests whose combined workspace fits the slot's
 * memory budget (and that share the beam width of the first), and launches
 * them as one batch on the slot's stream.  Slots run concurrently, so
 * requests that arrive while others are on the GPU start as soon as a slot
 * frees up.  Each image is bit-identical to a lone rr_radar_scan of the same
 * request.  While a server exists, only the server may use its context. */
typedef struct rr_server rr_server;

typedef struct {
  uint32_t n_slots;         /* batches in flight, one stream each (1..8, default 2) */
  uint32_t max_batch_scans; /* requests per batch (1..65535, default 256) */
  uint64_t memory_budget;   /* workspace bytes over all slots (default 32 GiB) */
  uint32_t reserved[4];
} rr_server_options;

typedef struct {
  uint64_t submitted, completed, rejected, batches, segments;
  double latency_p50_ms, latency_p99_ms, latency_mean_ms, latency_max_ms;
  double wall_s;      /* first submission to last completion since the last reset */
  double scans_per_s; /* completed / wall_s */
  double mseg_per_s;  /* segments / wall_s / 1e6 */
} rr_server_stats;

/* The material table is copied; the scene must outlive the server, and
 * rr_bvh_build / rr_scene_release of it return ESTATE until the server is
 * destroyed. */
rr_status rr_server_create(rr_context* ctx, const rr_scene* scene, const rr_material* materials,
                           uint32_t n_materials, const rr_server_options* opt, rr_server** out);
/* Thread-safe, non-blocking.  image_dev (n_azimuth x n_bins floats) is
 * written when the request completes.  ENOMEM if the request alone exceeds
 * a slot's budget (counted as rejected); EINVAL for invalid parameters. */
rr_status rr_server_submit(rr_server* srv, const rr_pose* pose, const rr_sensor_params* params,
                           float* image_dev, uint64_t* ticket);
/* Blocks until the request is done; latency = completion - submission. */
rr_status rr_server_wait(rr_server* srv, uint64_t ticket, double* latency_ms);
/* Non-blocking: *done = 1 once finished (the ticket is then released). */
rr_status rr_server_poll(rr_server* srv, uint64_t ticket, int* done, double* latency_ms);
rr_status rr_server_get_stats(rr_server* srv, rr_server_stats* out);
rr_status rr_server_reset_stats(rr_server* srv);
/* Finishes every submitted request, then frees the server. */
rr_status rr_server_destroy(rr_server* srv);

/* ---------------------------------------------------------------- tuning */
/* Launch parameters of the traversal kernel (all zero = defaults).  They
 * change speed only, never results. */
typedef struct {
  uint32_t refill_lanes;   /* a wave takes new rays once this many lanes are
                              idle (1..64, default 8) */
  uint32_t trace_waves_per_cu; /* persistent trace waves per compute unit in
                              the grid (1..32, default 24) */
  uint32_t pool_rays;      /* rays a trace wave claims per atomic (64..4096,
                              default 64) */
  uint32_t batch_budget_mb; /* workspace budget of one batch group, MiB (>= 64,
                              default 24 GiB) */
  uint32_t tri_batch;      /* leaves a trace wave queues before it tests their
                             triangles in one step, one leaf per lane (1..64,
                             default 6) */
  uint32_t fused;          /* 0: default (2); 1: every bounce level in one
                             persistent launch, each wave tracing and shading
                             its own rays' children; 2: one trace and one shade
                             launch per bounce level */
  uint32_t shade_batch;    /* fused: finished rays a wave queues before it
                             shades them in one step (1..64) */
  uint32_t tail_help;      /* a bounce level whose ray bound is at most
                             this many rays per lane of the trace grid
                             (1..1024, default 12) is traced with tail
                             helping: once a wave has no rays left to claim,
                             its idle lanes walk subtrees of its unfinished
                             rays.  The air-path visibility launch always
                             uses it.  RR_TAIL_HELP_OFF: never */
} rr_tuning;
#define RR_TAIL_HELP_OFF 0xffffffffu

/* Zero fields take their defaults.  EINVAL for a field out of its range,
 * and then no field changes.  rr_get_tuning returns the values in effect. */
rr_status rr_set_tuning(rr_context* ctx, const rr_tuning* t);
rr_status rr_get_tuning(const rr_context* ctx, rr_tuning* out);

/* Autotuner: scans the given workload with candidate launch parameters
 * (coordinate descent over refill_lanes, trace_waves_per_cu, pool_rays,
 * tri_batch, fused, shade_batch and tail_help, each candidate timed with HIP events over `reps` scans
 * on `stream`), keeps the fastest in the context and returns it in *best
 * with its time per scan.  Every candidate produces the same image.  The
 * one-launch mode (fused = 1) is not a candidate for an air-path scan or an
 * eight-wide tree, which it does not trace. */
rr_status rr_autotune(rr_context* ctx, const rr_scene* scene, const rr_pose* pose,
                      const rr_sensor_params* params, const rr_material* materials,
                      uint32_t n_materials, float* image_dev, uint32_t reps, rr_tuning* best,
                      double* best_ms, void* stream);

/* As rr_autotune for a batch (the many-pose use of Sec. IV): each candidate
 * is timed on rr_radar_scan_batch over these scans, so the parameters suit
 * the batched launch rather than one of its scans (a launch-bound scan
 * alone prefers fewer trace waves than a batch of them).  *best_ms is the
 * time per batch.  The images of the descriptors are overwritten; the scans
 * must be valid for rr_radar_scan_batch (EINVAL otherwise, nothing kept). */
rr_status rr_autotune_batch(rr_context* ctx, const rr_scene* scene, const rr_scan_desc* scans,
                            uint32_t n_scans, const rr_material* materials, uint32_t n_materials,
                            uint32_t reps, rr_tuning* best, double* best_ms, void* stream);

/* ---------------------------------------------------------------- graphs */
/* A HIP graph holding the complete launch sequence of a batch of scans
 * (clear, ray generation, trace and shade per level, finalize) with its own
 * workspace.  rr_graph_launch uploads the per-scan constants (poses, seeds,
 * scan ids and image pointers may change; azimuths, rays per beam, bounces,
 * bins, bin size, beam width and flags must match the scans the graph was
 * created with) and replays the graph on `stream`.  The captured launches
 * point at the scene's device copies: rr_bvh_build and rr_scene_release of
 * the scene return ESTATE until the graph is destroyed (rr_bvh_refit, which
 * rewrites the copies in place, stays allowed). */
typedef struct rr_graph rr_graph;
rr_status rr_graph_create(rr_context* ctx, const rr_scene* scene, const rr_scan_desc* scans,
                          uint32_t n_scans, const rr_material* materials, uint32_t n_materials,
                          rr_graph** out);
/* scans may be NULL to replay the scans given at creation. */
rr_status rr_graph_launch(rr_graph* g, const rr_scan_desc* scans, void* stream);
rr_status rr_graph_destroy(rr_graph* g);

/* ---------------------------------------------------------------- profiling */
#define RR_PROFILE_TIME 1u  /* bracket every kernel launch of a scan with HIP events */
#define RR_PROFILE_COUNT 2u /* use the counting kernels: node visits, triangle tests */
#define RR_PROFILE_TRACE_TIME 4u /* bracket only the trace launches with HIP events */

typedef struct {
  uint64_t trace_launches;     /* closest-hit (trace) launches recorded */
  double trace_ms;             /* summed event time of those launches */
  double trace_level_ms[RR_MAX_BOUNCES];
  double shade_ms;             /* interaction / binning / child launches */
  double raygen_ms;            /* primary generation launches */
  uint64_t node_visits;        /* inner nodes fetched (RR_PROFILE_COUNT) */
  uint64_t tri_tests;          /* ray-triangle tests (RR_PROFILE_COUNT) */
  uint64_t rays;               /* rays traced by the counted launches */
  uint64_t hits;               /* rays that hit a triangle */
  /* SIMD occupancy of the trace loop per bounce level (RR_PROFILE_COUNT):
   * wave iterations, and lanes holding a ray summed over those iterations;
   * the tail_ pair counts only iterations after the level's queue ran dry. */
  uint64_t wave_iters[RR_MAX_BOUNCES];
  uint64_t active_lanes[RR_MAX_BOUNCES];
  uint64_t tail_wave_iters[RR_MAX_BOUNCES];
  uint64_t tail_active_lanes[RR_MAX_BOUNCES];
  uint64_t max_ray_iters[RR_MAX_BOUNCES]; /* most loop iterations of one ray */
  double shadow_ms;            /* air-path visibility launches (RR_PROFILE_TIME) */
} rr_profile;

/* Measurement hooks for benchmarks (not needed for scans).  Enabling with
 * flags = 0 disables.  The counting kernel is slower; its results are the
 * same images. */
rr_status rr_profile_enable(rr_context* ctx, uint32_t flags);
/* Waits for the recorded events, returns the totals since the last read and
 * resets them. */
rr_status rr_profile_read(rr_context* ctx, rr_profile* out);

/* Bandwidth probe for the roofline: random 64-byte row gathers (the access
 * pattern of node and triangle fetches) over a device working set of
 * `working_set_bytes` (>= 64 KiB, <= 16 GiB), `reads_mb` MiB read in total;
 * returns the achieved read rate in GB/s.  Allocates and frees its buffers
 * and synchronizes the device. */
rr_status rr_measure_gather(rr_context* ctx, uint64_t working_set_bytes, uint32_t reads_mb, double* gbs);

#ifdef __cplusplus
}
#endif
#endif /* RADARAYS_HIP_H */
