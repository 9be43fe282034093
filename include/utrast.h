/*
 * utrast.h -- C-ABI of the MI355X (gfx950) unscented-transform Gaussian rasterizer for
 * arbitrary cameras and spinning LiDAR (SimULi, arXiv 2510.12901).
 *
 * The library renders a set of 3D Gaussian particles (Sec. 3.1) seen by a sensor
 * (Sec. 3.2 camera models; Sec. 3.3 spinning LiDAR, Eq. 3) along given rays
 * r(t) = o + t d (Sec. 3.2, "Volume Rendering").  The hot path is five calls:
 *
 *   ut_project            sigma-point projection, tile rect, LiDAR ray-based culling
 *   ut_bin_and_sort       depth sort and super-tile bins; each tile's (depth, index)-ordered
 *                         list is the super-tile list filtered by the particle's tile rect
 *   ut_composite_camera   front-to-back compositing of the 3D response (Eq. 1)
 *   ut_composite_lidar    the same over azimuth-elevation tiles, plus LiDAR outputs
 *   ut_composite_backward adjoint of the above with respect to every particle parameter
 *                         (walking the super-tile bins backwards)
 *
 * plus host set-up (ut_lidar_tiling = Alg. 1, ut_sensor_build = ray mask / summed-area
 * table of Appendix B), a batched composite for serving, and the scene graph's
 * rigid actor transforms (ut_actor_transform and its adjoint) that bring dynamic objects'
 * particles to the world frame before projection.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers marked "device" are HIP device pointers (hipMalloc or torch CUDA tensors);
 *   "host" pointers are ordinary CPU memory.  The caller owns every buffer; the library
 *   never allocates or frees device memory and keeps no mutable global state (the one
 *   exception is the fixed per-GPU queue of ut_composite_batch_noalloc), so calls on
 *   different streams with disjoint buffers are independent.
 * - All work is enqueued on the given stream (ut_stream = hipStream_t, NULL = the null
 *   stream).  Only ut_bin_and_sort with a non-NULL n_pairs pointer synchronises that stream.
 * - Errors: host-side argument checks return UT_ERR_ARG before anything is enqueued;
 *   HIP launch or copy failures return UT_ERR_DEVICE; a tile-list capacity overflow returns
 *   UT_ERR_CAPACITY.  Non-finite or degenerate particles are not errors: they are culled
 *   (tile count 0) and counted.  No C++ exception crosses this ABI.
 * - Particle arrays are float32 structure-of-arrays, component-major: mean[3][n] means
 *   mean[c * n + i].
 */
#ifndef UTRAST_H
#define UTRAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int ut_status;
enum { UT_OK = 0, UT_ERR_ARG = -1, UT_ERR_CAPACITY = -2, UT_ERR_DEVICE = -3, UT_ERR_UNSUPPORTED = -4 };

/* Sensor kinds and feature kinds. */
enum { UT_PINHOLE = 0, UT_FISHEYE = 1, UT_LIDAR = 2, UT_ORTHO = 3 };
enum { UT_FEAT_CAMERA = 0, UT_FEAT_LIDAR = 1 };

#define UT_RECORD_BYTES 128     /* per-particle compositing record written by ut_project */
#define UT_MAX_ELEV_TILES 256   /* largest N_phi accepted */
#define UT_CAMERA_TILE 16       /* camera tiles are 16 x 16 pixels */
#define UT_SUPER_TILE 8         /* binning super-tiles are 8 x 8 tiles */
#define UT_MAX_LIDAR_TILE_RAYS 512   /* ut_composite_batch and the adjoint take up to 256 */
#define UT_ACC_FLOATS 13        /* per-particle adjoint accumulator width (doubles) */

typedef void* ut_stream; /* hipStream_t */

/* Particles (Sec. 3.1): mean mu, rotation quaternion q = (w,x,y,z) (any non-zero norm; the
 * library normalises), log_scale (S = diag(exp(log_scale)), Sigma = R S S^T R^T),
 * opacity_logit (sigma = sigmoid), feat = SH coefficients feat[K][3][n] with
 * K = (sh_degree+1)^2, coefficient k of channel c of particle i at feat[(k*3+c)*n + i],
 * real SH with the Condon-Shortley phase ordered by l then m = -l..l.
 * feat_kind UT_FEAT_CAMERA: colour = max(0, SH(dir) + 0.5); UT_FEAT_LIDAR: the three
 * features (intensity, hit logit, drop logit) of Sec. 3.2 are SH(dir) raw.  dir is the
 * unit vector from the sensor origin to the particle mean.  All device, read-only. */
typedef struct {
  const float* mean;
  const float* quat;
  const float* log_scale;
  const float* opacity_logit;
  const float* feat;
  int32_t n;
  int32_t sh_degree;   /* 0..3 */
  int32_t feat_kind;
} ut_gaussians;

/* Sensor.  R_sw (row-major) maps world axes to sensor axes, origin is the sensor position
 * in the world (both float32, host fields).  Camera axes x right, y down, z forward;
 * LiDAR axes x forward, y left, z up.
 *   UT_PINHOLE : (u,v) = (fx x/z + cx, fy y/z + cy), valid iff z > near
 *   UT_FISHEYE : equidistant, theta = atan2(|xy|, z), theta_d = theta(1 + k1 t^2 + k2 t^4
 *                + k3 t^6 + k4 t^8), (u,v) = (cx,cy) + (fx,fy) theta_d xy/|xy|,
 *                valid iff |x| > near and theta <= theta_max
 *   UT_LIDAR   : Eq. 3, azimuth atan2(y,x) in [0, 2pi), elevation asin(z/r), valid iff r > near
 *   UT_ORTHO   : (fx x + cx, fy y + cy), valid iff z > near (affine; used to test the UT)
 * ray_dir: device float32 [3][R] world-frame directions.  Camera ray y*width + x goes
 * through the pixel centre (x+0.5, y+0.5); LiDAR ray b*n_az + a is beam b (elevations
 * sorted ascending) at azimuth 2 pi a / n_az.  An all-zero direction marks "no ray"
 * (its outputs are zero).  tables: device buffer of ut_sensor_table_bytes() bytes filled
 * by ut_sensor_build (LiDAR only; may be NULL for cameras). */
typedef struct {
  int32_t kind;
  float R_sw[9];
  float origin[3];
  double near_;
  /* cameras */
  int32_t width, height;
  double fx, fy, cx, cy, k[4], theta_max;
  /* spinning LiDAR */
  int32_t n_beams, n_az;
  int32_t n_phi;          /* elevation tiles N_phi */
  int32_t max_per_tile;   /* M of Alg. 1 */
  int32_t cull;           /* ray-based culling on/off */
  int32_t cull_az, cull_el; /* culling grid: azimuth cells over 360 deg, elevation cells */
  int32_t n_theta;        /* azimuth tiles, set by ut_sensor_build */
  int32_t max_tile_rays;  /* largest ray count of one tile, set by ut_sensor_build */
  int32_t n_units;        /* LiDAR compositing units (runs of adjacent azimuth tiles of one
                             elevation tile packed into one workgroup), set by ut_sensor_build */
  int32_t unit_rays;      /* rays per unit at most (64, 128 or 256; 0 = no units), set by
                             ut_sensor_build */
  int32_t n_units_wide;   /* units of up to 256 rays for the batched composite (0 = none), set
                             by ut_sensor_build */
  const float* beam_elev_host; /* host [n_beams] radians, sorted ascending (LiDAR set-up only) */
  const float* ray_dir;   /* device [3][R] */
  void* tables;           /* device, LiDAR tiling + summed-area table */
  /* Time-dependent sensor (Sec. 3.2 and its appendix on time-dependent effects: sensor motion
   * inside the projection, each ray at its own time).  moving = 0: a static sensor, the rest
   * is ignored.  moving = 1: (R_sw, origin) is the pose at frame time 0 and (R_sw1, origin1)
   * at time 1; in between the origin moves linearly and the rotation by spherical linear
   * interpolation (shorter arc).  Camera row v is read out at t = v / height (rolling
   * shutter), LiDAR azimuth phi at t = phi / (2 pi).  A sigma point is projected with the pose
   * at t = 1/2, then rs_iters - 1 more times with the pose at the time of its previous
   * projection.  ray_org (device [3][R]) holds every ray's origin o(t_i); ray_dir its
   * direction at t_i.  Not for UT_ORTHO. */
  int32_t moving;
  float R_sw1[9];
  float origin1[3];
  const float* ray_org;   /* device [3][R], moving sensors only */
  int32_t rs_iters;       /* 1..64 */
  /* LiDAR beam divergence (Sec. 3.2, LiDAR appendix: the beam is a cone, not a line).  Full
   * cone angle in radians, 0 <= beam_divergence < pi; 0 = off.  Each particle is smoothed
   * across the beam at its range r = |mu - origin| before projection:
   * Sigma_hat = Sigma + (r tan(beam_divergence / 2))^2 (I - d d^T), d = (mu - origin) / r,
   * with the opacity left unscaled; the UT's sigma points use the lower Cholesky factor L of
   * Sigma_hat and the compositing record holds Sigma_hat^{-1}.  origin is the frame-start origin for moving
   * sensors.  Must be 0 for cameras (UT_ERR_ARG otherwise).  The adjoint differentiates
   * the filter too (the mean moves the smoothing term). */
  double beam_divergence;
} ut_sensor;

/* Compositing cut-offs (Eq. 1 practice): skip alpha < alpha_min, clamp alpha at
 * alpha_max, stop after the particle that brings transmittance below t_min. */
typedef struct {
  double alpha_min, alpha_max, t_min;
} ut_render_params;

/* Projection output, all device buffers sized for n particles (caller-allocated). */
typedef struct {
  void* records;       /* [n] UT_RECORD_BYTES each (layout private to the library); written only
                          for particles with count > 0, the rest are left untouched */
  int32_t* rect;       /* [4][n] tile rect x0,y0,x1,y1 inclusive; LiDAR x = azimuth tile,
                          x1 may exceed n_theta-1 where the rect wraps through 0 */
  uint32_t* key;       /* [n] depth key: float32 bits of |mu - o|^2 computed
                          (dx*dx + dy*dy) + dz*dz in float32 without fused multiply-add */
  uint32_t* count;     /* [n] tiles touched; 0 = culled */
  uint32_t* trect;     /* [n][2] the same rect packed (x0 | y0 << 16, x1 | y1 << 16) */
  float* moments;      /* [5][n] UT mean (u, v) and covariance (uu, uv, vv); may be NULL */
  uint32_t* n_culled;  /* [2] invalid particles, LiDAR ray-culled particles (set by the call) */
} ut_projected;

/* Super-tile bins (what the compositing consumes).  Tiles are grouped in super-tiles of
 * UT_SUPER_TILE x UT_SUPER_TILE tiles (super id = (ty / 8) * super_x + tx / 8,
 * super_x = ceil(tiles_x / 8)); gauss[0..n_pairs) holds, per super-tile, every particle
 * whose rect touches it, ordered by (super-tile, depth key, particle index); ranges[2][n_super]
 * = [start, end).  A tile's list -- its particles ordered by (depth key, index) -- is its
 * super-tile's list filtered by "the particle's rect contains the tile".  Device,
 * caller-allocated. */
typedef struct {
  uint32_t* gauss;
  uint32_t* ranges;
  uint64_t max_pairs;  /* capacity of gauss */
} ut_bin_lists;

/* Per-tile lists, materialised from the bins (for the adjoint and for checking the order):
 * gauss[0..n_pairs) ordered by (tile, depth key, particle index), ranges[2][n_tiles]. */
typedef struct {
  uint32_t* gauss;
  uint32_t* ranges;
  uint64_t max_pairs;
  uint64_t* n_pairs_dev;  /* device [1]: total written by ut_tile_lists_count */
} ut_tile_lists;

/* Per-ray outputs, device, R = rays of the sensor.
 * feat[3][R]: premultiplied colour sum w c (camera) or LiDAR features zeta (channel 0 =
 * intensity); depth[R] = sum w t* (unnormalised); alpha[R] = omega = 1 - T_final;
 * drop[R] = ray-drop probability softmax(zeta_1, zeta_2)[drop] (LiDAR only, may be NULL);
 * t_final[R], n_proc[R] (list entries visited) are the state the adjoint replays
 * (may be NULL when no backward follows).
 * n_visit[R], n_pass[R] (optional, may be NULL; written by ut_composite_camera/_lidar, not by
 * ut_composite_batch): work counters -- list entries the ray actually evaluated (entries that
 * no ray of the tile can reach are dropped before the rays see them) and, of those, entries
 * that passed the alpha_min pre-test.
 * tile_end[n_tiles] (optional, adjoint state, may be NULL; written by ut_composite_camera/_lidar,
 * not by ut_composite_batch): per tile, the index in the super-tile bin (bins->gauss) just past
 * the last entry any ray of the tile processed, so the adjoint can walk the bin backwards from
 * there without materialised per-tile lists. */
typedef struct {
  float* feat;
  float* depth;
  float* alpha;
  float* drop;
  double* t_final;
  uint32_t* n_proc;
  uint32_t* n_visit;
  uint32_t* n_pass;
  uint32_t* tile_end;
} ut_render_out;

/* Upstream gradients dL/d(output), device float32 arrays shaped like ut_render_out;
 * any member may be NULL (= zero). */
typedef struct {
  const float* feat;
  const float* depth;
  const float* alpha;
  const float* drop;
} ut_upstream;

/* Gradients with respect to the particle parameters, device float32, same shapes as
 * ut_gaussians (feat: [K][3][n]).  Overwritten by the call. */
typedef struct {
  float* mean;
  float* quat;
  float* log_scale;
  float* opacity_logit;
  float* feat;
} ut_gaussian_grads;

const char* ut_status_str(ut_status s);
int32_t ut_record_bytes(void);

/* Alg. 1 (ElevationTiling), host only.  beam_elev: host [n_beams] radians sorted
 * ascending; n_az azimuth steps per revolution; n_phi elevation tiles; M rays per tile
 * bound.  Writes bounds[n_phi+1] (radians), beam_start[n_phi+1] (first beam of each
 * elevation tile; beams of tile k are [beam_start[k], beam_start[k+1])) and *n_theta. */
ut_status ut_lidar_tiling(const float* beam_elev, int32_t n_beams, int32_t n_az, int32_t n_phi,
                          int32_t M, double* bounds, int32_t* beam_start, int32_t* n_theta);

/* Bytes of the device tables of a sensor (0 for cameras). */
ut_status ut_sensor_table_bytes(const ut_sensor* s, size_t* bytes);

/* Sensor set-up, once per sensor definition (Sec. 3.3: the tiling is reused across calls).
 * LiDAR: runs Alg. 1, builds the ray mask over the culling grid and its summed-area
 * table (Appendix B) and the compositing units, and copies them to s->tables (device,
 * ut_sensor_table_bytes bytes); sets s->n_theta, s->max_tile_rays, s->n_units,
 * s->unit_rays and s->n_units_wide (a second packing of up to 256 rays per unit, which
 * ut_composite_batch uses).  A unit is a run of adjacent azimuth tiles of one elevation tile within one
 * super-tile column whose rays fit one workgroup of unit_rays lanes (the smallest of 64, 128,
 * 256 that holds the largest tile); the tiles stay the binning units and every ray still walks
 * its own tile's list, so units change which rays share a wavefront, not any result.
 * Cameras: sets max_tile_rays = 256 (no units).  Camera ray tables are not built here: the
 * rays are an input of the problem (r(t) = o + t d), so the caller supplies ray_dir (and
 * ray_org for moving sensors), e.g. its own unprojection of the pixel centres.
 * Synchronises the stream (the host tables are freed on return). */
ut_status ut_sensor_build(ut_sensor* s, ut_stream stream);

/* Number of tiles of a (built) sensor. */
int32_t ut_sensor_tiles(const ut_sensor* s);
/* Number of rays of a sensor. */
int64_t ut_sensor_rays(const ut_sensor* s);

/* Sigma-point projection (Sec. 3.2; LiDAR Eq. 3 and ray-based culling, Alg. 2 and 3).
 * Per particle: normalise q, build R, s = exp(log_scale), sigma = sigmoid(logit); project
 * the 7 sigma points mu +- sqrt(3 + lambda) s_j R[:,j] with the scaled unscented transform
 * (ut_abk = alpha, beta, kappa; lambda = alpha^2 (3 + kappa) - 3); UT mean and covariance;
 * 3-sigma extent of the covariance diagonal -> tile rect; for LiDAR with culling on, the
 * count is zero when no ray falls in the extent on the culling grid; depth key; SH
 * features; compositing record.  Any invalid sigma point culls the particle.
 * ut_abk: host [3].  out: device buffers sized g->n. */
ut_status ut_project(const ut_gaussians* g, const ut_sensor* s, const double* ut_abk,
                     ut_projected* out, ut_stream stream);

/* Workspace sizes of the binning stage.  The count workspace depends on the particle count
 * only; the pair workspace on the super-tile pair total P reported by ut_bin_count, so a
 * scheduler can reserve it after counting.  ut_workspace_bytes = count + pair bytes for
 * max_pairs (one buffer, as ut_bin_and_sort takes it). */
size_t ut_count_workspace_bytes(int32_t n_gaussians);
size_t ut_pair_workspace_bytes(uint64_t n_pairs);
size_t ut_workspace_bytes(uint64_t max_pairs, int32_t n_tiles, int32_t n_gaussians);
/* Number of super-tiles of a (built) sensor. */
int32_t ut_sensor_super_tiles(const ut_sensor* s);

/* Binning and depth sort (Sec. 3.2, tiling as in 3DGS, binned per super-tile).  The output
 * is one list per super-tile of 8 x 8 tiles, not per tile: the compositing kernels filter a
 * super-tile list by each particle's rect on chip, which yields each tile's exact
 * (depth, index)-ordered list without writing it to memory; ut_tile_lists_count / _fill
 * materialise the per-tile lists when a caller needs them.
 * Step 1 (ut_bin_count, asynchronous): stable radix sort of the particles by depth key,
 * exclusive scan of their super-tile counts in that order; the pair total P stays in the
 * count workspace ws and, if n_pairs_host is non-NULL, is copied there asynchronously
 * (pinned memory; read it after the stream is synchronised).  Step 2 (ut_bin_sort,
 * asynchronous, same ws untouched in between): emit the (super-tile, particle) pairs in
 * depth order, stable radix sort them by super-tile id (pair_ws of at least
 * ut_pair_workspace_bytes(n_pairs) bytes), write bins->gauss[0..P) and bins->ranges.
 * UT_ERR_CAPACITY if P > bins->max_pairs or a workspace is too small (nothing enqueued).
 * ut_bin_and_sort runs both with one buffer ws (count part first, pair part after it) and
 * synchronises the stream in between; *n_pairs (host, may be NULL) receives P. */
ut_status ut_bin_count(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws,
                       size_t ws_bytes, uint64_t* n_pairs_host, ut_stream stream);
ut_status ut_bin_sort(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws,
                      size_t ws_bytes, void* pair_ws, size_t pair_ws_bytes, uint64_t n_pairs,
                      ut_bin_lists* bins, ut_stream stream);
ut_status ut_bin_and_sort(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws,
                          size_t ws_bytes, ut_bin_lists* bins, uint64_t* n_pairs,
                          ut_stream stream);

/* Step 2 without the host round trip: like ut_bin_sort, but the pair total P is read on the
 * device from ws (as ut_bin_count left it), and every launch is sized for a capacity
 * max_pairs chosen by the caller (bins->max_pairs >= max_pairs, pair_ws of at least
 * ut_pair_workspace_bytes(max_pairs) bytes, max_pairs < 2^30).  If P > max_pairs nothing
 * is emitted, every super-tile range is left empty (a composite then renders nothing) and
 * *overflow (device uint32, may be NULL) is set to 1; it is never cleared by the library, so
 * one flag can guard several calls: check it after the stream has completed and render
 * again with a larger capacity.  The result is bit-identical to ut_bin_sort whenever P fits.
 * Nothing is synchronised, so a whole frame (projection, count, this call, compositing) can
 * be enqueued, or captured in a graph, without a host round trip. */
ut_status ut_bin_sort_device(const ut_projected* p, int32_t n, const ut_sensor* s, void* ws,
                             size_t ws_bytes, void* pair_ws, size_t pair_ws_bytes, uint64_t max_pairs,
                             ut_bin_lists* bins, uint32_t* overflow, ut_stream stream);

/* Per-tile lists from the bins.  ut_tile_lists_count writes each tile's list length into
 * lists->ranges and turns it into [start, end) ranges; the total (the number of (tile,
 * particle) pairs) is copied to *n_pairs_host (pinned, asynchronous) if non-NULL.
 * ut_tile_lists_fill then writes lists->gauss (capacity lists->max_pairs >= total). */
ut_status ut_tile_lists_count(const ut_projected* p, const ut_sensor* s, const ut_bin_lists* bins,
                              ut_tile_lists* lists, uint64_t* n_pairs_host, ut_stream stream);
ut_status ut_tile_lists_fill(const ut_projected* p, const ut_sensor* s, const ut_bin_lists* bins,
                             ut_tile_lists* lists, ut_stream stream);

/* Front-to-back compositing (Eq. 1) of every ray of a camera over its tile's list (the
 * workgroup of a tile compacts that list from its super-tile bin with wavefront ballots and
 * prefix sums while it composites, so per-tile lists never go through HBM): for
 * each particle, t* = argmax of its 3D response along the ray (d^T B v / d^T B d with
 * B = Sigma^{-1}, v = mu - o), rho = exp(-D^2/2) at t*, alpha = min(sigma rho, alpha_max),
 * skipped when alpha < alpha_min or t* < near; w = alpha T; feat += w c; depth += w t*;
 * T *= 1 - alpha; the ray stops after T < t_min.  Deterministic (no atomics). */
ut_status ut_composite_camera(const ut_projected* p, const ut_bin_lists* bins,
                              const ut_sensor* s, const ut_render_params* prm,
                              ut_render_out* out, ut_stream stream);

/* The same over the azimuth-elevation tiles of a spinning LiDAR; additionally
 * drop = sigmoid(zeta_2 - zeta_1) (the softmax of Sec. 3.2 over hit/drop). */
ut_status ut_composite_lidar(const ut_projected* p, const ut_bin_lists* bins,
                             const ut_sensor* s, const ut_render_params* prm,
                             ut_render_out* out, ut_stream stream);

/* Bytes of the per-particle accumulator workspace of the adjoint (the call takes it as an
 * argument, acc_ws, because the per-pair partials are summed in float64 per particle before
 * the chain rule, and the library allocates nothing). */
size_t ut_backward_workspace_bytes(int32_t n_gaussians);

/* Adjoint of ut_composite_* with the discrete structure of the forward held fixed (lists,
 * culls, alpha_min skips, alpha_max clamps, colour clamps, the termination index).
 * bins: the forward's super-tile bins.  Each tile walks its super-tile bin backwards from
 * fwd->tile_end, keeping the entries whose rect covers the tile (and that the tile's ray cone
 * can reach), and replays each ray's list in reverse from fwd->n_proc, recovering
 * T_i = T_{i+1}/(1 - alpha_i) from fwd->t_final; per-pair gradients are reduced per wavefront
 * and added atomically into per-particle float64 accumulators (acc_ws, zeroed by the call),
 * then a per-particle kernel applies the chain rule to (mean, quat, log_scale, opacity_logit,
 * feat) including the SH direction's dependence on the mean.  fwd must hold feat, t_final,
 * n_proc and tile_end of the forward call with the same arguments.  Gradients are
 * accumulated in float64 but their summation order is not fixed (atomics).  Sensors whose
 * tiles hold more than 256 rays (LiDAR with large M) return UT_ERR_UNSUPPORTED. */
ut_status ut_composite_backward(const ut_gaussians* g, const ut_projected* p,
                                const ut_bin_lists* bins, const ut_sensor* s,
                                const ut_render_params* prm, const ut_render_out* fwd,
                                const ut_upstream* up, void* acc_ws, size_t acc_ws_bytes,
                                ut_gaussian_grads* grads, ut_stream stream);

/* Batched compositing for serving.  One launch composites the tiles of several independent
 * render requests (any mix of camera and LiDAR sensors, each with its own projection, lists
 * and outputs) as (request, tile) work items.  Per-ray arithmetic is the
 * same as ut_composite_camera / ut_composite_lidar, so every ray's output is bit-identical
 * to the single-request call.  items: host array [n_items]; queue_ws: device workspace of
 * ut_batch_workspace_bytes(n_items) bytes.  n_workgroups > 0: that many persistent workgroups
 * loop over the items; n_workgroups == 0: one workgroup per (request, tile) item, the
 * hardware dispatcher handing them out in item order (no loop, so the kernel keeps the
 * single-request kernel's register budget; the faster mode on MI355X).  Sensors whose tiles
 * hold more than 256 rays return UT_ERR_UNSUPPORTED (n_visit, n_pass and tile_end are not
 * written on this path). */
typedef struct {
  const ut_projected* proj;
  const ut_bin_lists* bins;
  const ut_sensor* sensor;
  ut_render_out* out;
} ut_batch_item;

size_t ut_batch_workspace_bytes(int32_t n_items);
ut_status ut_composite_batch(const ut_batch_item* items, int32_t n_items,
                             const ut_render_params* prm, void* queue_ws, size_t ws_bytes,
                             int32_t n_workgroups, ut_stream stream);

/* ut_composite_batch without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The queue lives in a library-owned device array of fixed size, one per GPU, held until the
 * process ends; the call allocates nothing.  Same items, arithmetic and outputs as
 * ut_composite_batch (bit-identical).  n_items > UT_BATCH_NOALLOC_MAX_ITEMS returns
 * UT_ERR_CAPACITY before anything is enqueued.  Every call on one GPU uses that GPU's single
 * queue, which keeps the last call's contents (the counters are cleared at the start of each
 * call): calls that overlap on one GPU (different streams, or a graph replayed while another
 * call runs) race and must be serialised by the caller. */
#define UT_BATCH_NOALLOC_MAX_ITEMS 64
ut_status ut_composite_batch_noalloc(const ut_batch_item* items, int32_t n_items,
                                     const ut_render_params* prm, int32_t n_workgroups, ut_stream stream);

/* Spatial order of a resident particle set.  Results never depend on the particles' order
 * (every list is ordered by depth key, ties by index), but memory traffic does: stored along a
 * Z-order curve of their means, the particles one view sees share cache lines.  A one-time
 * reorder for a resident scene:
 *   ut_spatial_order   perm (device uint32 [n], caller-allocated) = the particle indices in
 *                      order of the 30-bit Morton code of the mean inside the bounding box of
 *                      the finite means (10 bits per axis; non-finite means last; ties by
 *                      index).  ws: device, ut_spatial_order_workspace_bytes(n) bytes.
 *   ut_gather_gaussians writes the reordered set, dst[:, j] = src[:, perm[j]], into caller
 *                      arrays of the source's shapes (must not overlap the source).
 * A reordered set renders the same images; its gradients are in the new order (row j belongs
 * to source particle perm[j]).  UT_ERR_ARG for NULL pointers or n < 0; UT_ERR_CAPACITY for a
 * short workspace. */
size_t ut_spatial_order_workspace_bytes(int32_t n_gaussians);
ut_status ut_spatial_order(const ut_gaussians* g, uint32_t* perm, void* ws, size_t ws_bytes, ut_stream stream);
ut_status ut_gather_gaussians(const ut_gaussians* src, const uint32_t* perm, float* mean, float* quat,
                              float* log_scale, float* opacity_logit, float* feat, ut_stream stream);

/* Scene graph: rigid actor transforms (Sec. 3.1, scene representation).  Every particle
 * belongs to the static background or to one dynamic object (actor); an actor's particles
 * keep their means and covariances in the actor's own frame, and at render time the actor's
 * SE(3) pose for the timestamp maps them to the world:
 *   mu_w = R_a mu + t_a,   Sigma_w = R_a Sigma R_a^T,   i.e. q_w = q_a * q (Hamilton product),
 * with R_a = R(q_a / |q_a|).  Scale, opacity and features are not changed, so the world-frame
 * ut_gaussians shares those arrays with the object-frame one.  A moving sensor still sees
 * each actor at the one pose given for the frame. */
typedef struct {
  float q[4];     /* rotation object -> world, (w, x, y, z); normalised by the kernels */
  float t[3];     /* translation (world position of the object's origin) */
  float pad_;     /* unused; keeps the record 32 bytes */
} ut_actor_pose;

/* Forward: mean_world[3][n], quat_world[4][n] (device, caller-allocated, must not overlap
 * g->mean / g->quat) receive the world-frame means and quaternions of g (object-frame
 * particles; only mean, quat and n are read).  actor: device int32 [n], the actor of each
 * particle; an id outside [0, n_actors) is background and is copied unchanged.  poses:
 * device [n_actors] (may be NULL when n_actors == 0).  FP64 arithmetic, float32 results.
 * UT_ERR_ARG: NULL pointers, n < 0 or n_actors < 0. */
ut_status ut_actor_transform(const ut_gaussians* g, const int32_t* actor, const ut_actor_pose* poses,
                             int32_t n_actors, float* mean_world, float* quat_world, ut_stream stream);

/* Adjoint of ut_actor_transform.  d_mean_world[3][n], d_quat_world[4][n]: device gradients
 * with respect to the world-frame means and quaternions (for instance from
 * ut_composite_backward on the transformed set).  Writes d_mean[3][n], d_quat[4][n] (device;
 * may be the same buffers as d_mean_world / d_quat_world) with respect to the object-frame
 * parameters in g, and, when d_pose is not NULL, d_pose: device float64 [n_actors][7] =
 * gradient with respect to (q_w, q_x, q_y, q_z, t_x, t_y, t_z) of each pose (raw quaternion,
 * through its normalisation), zeroed by the call and accumulated with atomics (summation
 * order not fixed).  Background particles pass their gradients through.  UT_ERR_ARG as for
 * the forward. */
ut_status ut_actor_transform_backward(const ut_gaussians* g, const int32_t* actor,
                                      const ut_actor_pose* poses, int32_t n_actors,
                                      const float* d_mean_world, const float* d_quat_world,
                                      float* d_mean, float* d_quat, double* d_pose, ut_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* UTRAST_H */
