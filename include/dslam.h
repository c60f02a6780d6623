/*
 * dslam.h -- C ABI of the MI355X dense RGB-D-inertial tracking library.
 *
 * The library implements the per-frame tracking step of Laidlow, Bloesch, Li
 * and Leutenegger, "Dense RGB-D-Inertial SLAM with Map Deformations"
 * (Section IV): projective association against a predicted model view,
 * photometric (eq. (3)) and point-to-plane ICP (eq. (4)) residuals with
 * inverse-covariance and Huber weights, reduction into Gauss-Newton normal
 * equations per pyramid level, the IMU preintegration factor (Section IV-C,
 * eq. (5)), the joint solve over pose, velocity, IMU biases and gravity
 * direction (eqs. (6)-(7)) and the Schur-complement marginalisation into a
 * prior with its first-order correction (eqs. (8)-(9)).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns a dslam_status; DSLAM_OK (0) on success.  Outputs are
 *   written only on success.  No C++ exception and no abort crosses the ABI.
 * - "device pointer" means memory allocated on the session's GPU (for example
 *   a torch CUDA tensor's data_ptr()); "host pointer" means ordinary CPU memory.
 * - Streams are hipStream_t passed as void*; NULL means the default stream.
 *   All calls on one session must be issued on one stream (or be externally
 *   ordered): the session's device state is updated in stream order.
 * - Images are row-major with a pitch given in elements.  Depth is float32
 *   metres, 0 (or non-finite, or negative) meaning invalid.  Intensity is uint8.
 * - Quaternions are Hamilton unit quaternions stored (w, x, y, z) (Section II).
 *   Orientation perturbations are on the left: q [+] da = exp(da) (x) q
 *   (Section IV-A).
 * - Per-frame tangent order is [dr, dalpha, dv, dbg, dba] (15); the gravity
 *   orientation q_IW has its own 3-vector dg.  The paper keeps q_IW in every
 *   state (eq. (1)); this library keeps one q_IW shared by the previous and
 *   the current state, so the joint system is 33-d and the prior 18-d.
 * - Matrices are row-major doubles unless stated otherwise.
 */
#ifndef DSLAM_H
#define DSLAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSLAM_OK = 0,
  DSLAM_ERR_INVALID = 1,     /* bad argument: size, null pointer, non-unit quaternion, unsorted IMU ... */
  DSLAM_ERR_NO_CAPACITY = 2, /* the context's HBM budget cannot hold the session */
  DSLAM_ERR_SINGULAR = 3,    /* the normal equations were not positive definite; state left unchanged */
  DSLAM_ERR_DEVICE = 4,      /* a HIP runtime error */
  DSLAM_ERR_BUSY = 5,        /* the session has work in flight that the call would race with */
  DSLAM_ERR_NOT_READY = 6    /* a required input (for example the model view) has not been supplied */
} dslam_status;

enum { DSLAM_MAX_LEVELS = 4, DSLAM_MAX_IMU_SAMPLES = 32 };

/* tracking modes: RGB-D-inertial (the paper's system), RGB-D only (its baseline), gyro only */
enum { DSLAM_MODE_RGBDI = 0, DSLAM_MODE_RGBD = 1, DSLAM_MODE_GYRO = 2 };

/* how the residual pass stores Jacobian rows and contracts J^T J (see DESIGN notes in the source) */
enum {
  DSLAM_JAC_FP32 = 0,      /* FP32 rows, wavefront-shuffle + LDS block reduction on the vector ALUs */
  DSLAM_JAC_FP32_MFMA = 1, /* FP32 rows contracted on matrix cores (v_mfma_f32_16x16x4_f32) */
  DSLAM_JAC_FP16 = 2,      /* FP16 rows (power-of-two column scales) on v_mfma_f32_16x16x32_f16 */
  DSLAM_JAC_BF16 = 3       /* BF16 rows on v_mfma_f32_16x16x32_bf16 */
};

enum { DSLAM_PYR_CURRENT = 0, DSLAM_PYR_MODEL = 1 };

/* pyramid channels for dslam_copy_pyramid */
enum {
  DSLAM_CH_VX = 0, DSLAM_CH_VY, DSLAM_CH_VZ, DSLAM_CH_NX, DSLAM_CH_NY, DSLAM_CH_NZ,
  DSLAM_CH_I, DSLAM_CH_GX, DSLAM_CH_GY
};

/* State of one camera frame (eq. (1) without q_IW): camera position r_WC,
 * orientation q_WC, IMU velocity v_IS expressed in I, gyro and accelerometer biases. */
typedef struct {
  double r[3];
  double q[4];
  double v[3];
  double bg[3];
  double ba[3];
} dslam_frame_state;

/* Pinhole camera at pyramid level 0; pixel centres sit at integer coordinates. */
typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
} dslam_camera;

/* IMU noise model and extrinsics (Table I).  Noise densities: white noise of
 * density sigma gives the held value of a sub-interval of length dt the
 * variance sigma^2/dt; bias random walks add sigma_rw^2 * Dt per frame. */
typedef struct {
  double sigma_g;      /* gyro noise density, rad/s/sqrt(Hz) */
  double sigma_a;      /* accelerometer noise density, m/s^2/sqrt(Hz) */
  double sigma_bg_rw;  /* gyro drift density, rad/s^2/sqrt(Hz) */
  double sigma_ba_rw;  /* accelerometer drift density, m/s^3/sqrt(Hz) */
  double gravity;      /* |g|, m/s^2; g_I = (0, 0, -gravity) */
  double R_CS[9];      /* rotation S -> C */
  double t_CS[3];      /* origin of S expressed in C */
} dslam_imu_params;

/* Tracking parameters.  levels in [1, 4]; iters[l] Gauss-Newton iterations at
 * level l (level 0 = full resolution), run coarse to fine (Section IV-D). */
typedef struct {
  int32_t levels;
  int32_t iters[DSLAM_MAX_LEVELS];
  double icp_dist;   /* association distance gate, metres (0.10) */
  double icp_cos;    /* optional normal-compatibility gate as a cosine; < -1 disables it (default) */
  double sigma_I;    /* photometric noise; W_RGB = 1/sigma_I^2 */
  double depth_k;    /* depth noise sigma_z = depth_k * z^2; W_ICP = 1/sigma_z^2 */
  double huber_k;    /* Huber threshold on the whitened residual; 0 = no robust weight */
  int32_t jac_format;
  int32_t mode;
  /* health checks of a tracked frame (dslam_track_result.health); 0 disables each */
  double min_inlier_frac; /* LOW_INLIERS below this fraction of 2 x (level-0 pixels) inliers of both terms */
  double max_cost_rise;   /* COST_UP when the finest level's visual cost rises by more than this fraction */
  /* 1 (RGB-D-inertial mode only): a frame that ends with tracking lost
   * (LOW_INLIERS, NONFINITE or COST_UP) is re-estimated without its visual
   * terms: one Gauss-Newton step of the prior and the IMU factor alone
   * (Sections IV-C, IV-E) from the frame's start state and its IMU
   * prediction, marginalised at the result; health gains IMU_ONLY.  0: the
   * joint estimate stands, flagged.  Costs one extra launch per frame, which
   * returns at once unless the frame was lost. */
  int32_t imu_fallback;
} dslam_track_params;

typedef struct {
  double t;        /* seconds; the sample is held over [t, next t) */
  double gyro[3];  /* rad/s in S */
  double acc[3];   /* m/s^2 in S (specific force) */
} dslam_imu_sample;

/* Preintegrated IMU measurement between two frames (Section IV-C). */
typedef struct {
  double dR[9], dv[3], dp[3];
  double dt;
  double bg[3], ba[3];  /* linearisation biases */
  double J[54];         /* 9x6: d(dphi, dv, dp)/d(bg, ba); dR(b) ~ dR Exp(J[0:3] db) */
  double Sigma[81];     /* 9x9 noise covariance of (dphi, dv, dp), dR <- dR Exp(dphi) */
} dslam_preint;

/* Marginal prior on (x0, q_IW) (eqs. (6), (8)): cost (d - H^-1 b)^T H (d - H^-1 b)
 * with d = [x0 [-] xbar ; q_IW [-] q_IW_bar]. */
typedef struct {
  double H[324];
  double b[18];
  dslam_frame_state xbar;
  double q_IW_bar[4];
} dslam_prior;

/* Health flags of a tracked frame (dslam_track_result.health).  A frame
 * with any flag set is reported as tracking lost: the estimate is returned
 * as computed, and the caller decides whether to trust it (the paper's
 * estimator has no failure detection of its own; these are the checks that
 * a failed dense alignment shows, Section VI). */
enum {
  DSLAM_HEALTH_LOW_INLIERS = 1, /* level-0 inliers (ICP + photometric) < min_inlier_frac x 2 x pixels */
  DSLAM_HEALTH_NONFINITE = 2,   /* a cost or an updated state entry is not finite */
  DSLAM_HEALTH_COST_UP = 4,     /* finest level: last visual cost > (1 + max_cost_rise) x first */
  DSLAM_HEALTH_SINGULAR = 8,    /* a Gauss-Newton system was not positive definite (status SINGULAR) */
  DSLAM_HEALTH_IMU_ONLY = 16    /* the estimate is the inertial-only fallback (dslam_track_params.imu_fallback) */
};

/* Result of one tracked frame. */
typedef struct {
  int32_t status;       /* dslam_status of the frame */
  int32_t frame_index;  /* frames tracked by the session so far */
  int32_t health;       /* DSLAM_HEALTH_* flags */
  int32_t tracking_lost; /* 1 if any health flag is set, else 0 (a result flag, not an error) */
  dslam_frame_state x0; /* refined previous state */
  dslam_frame_state x1; /* current state */
  double q_IW[4];
  double cost_icp, cost_rgb, cost_imu, cost_prior; /* weighted costs at the last linearisation */
  int64_t n_icp[DSLAM_MAX_LEVELS]; /* ICP inliers at the last iteration of each level */
  int64_t n_rgb[DSLAM_MAX_LEVELS]; /* photometric inliers at the last iteration of each level */
  double last_step_norm;           /* |dz| of the last iteration */
  dslam_prior prior;               /* prior handed to the next frame */
} dslam_track_result;

/* Visual normal equations of one residual pass, lifted to the world frame
 * over [dr0, da0, dr1, da1] (12) and split per term, b = -sum w J^T e.
 * raw[] holds the pass's own sums before lifting: per term (ICP then RGB)
 * the 21 upper-triangular entries of sum w j j^T (row-major upper triangle of
 * 6x6), the 6 entries of sum w j e, sum w e^2 and the inlier count (29). */
typedef struct {
  double H_icp[144], b_icp[12], cost_icp;
  int64_t n_icp;
  double H_rgb[144], b_rgb[12], cost_rgb;
  int64_t n_rgb;
  double raw[58];
} dslam_linear_system;

typedef struct dslam_context dslam_context;
typedef struct dslam_session dslam_session;
typedef struct dslam_batch dslam_batch;

/* Maximum sessions in one batched step and distinct resolutions within it. */
#define DSLAM_MAX_BATCH 256
#define DSLAM_MAX_BATCH_RESOLUTIONS 16

/* One session's inputs for dslam_track_frame or a batched step: the new
 * frame and the model view predicted for it (device images, height x width,
 * row pitch in elements), the model-view pose T_WM (4x4 row-major, host) and
 * the frame's IMU samples (host, sorted by time, the first stamped at or
 * before t0; ignored in DSLAM_MODE_RGBD).  dslam_track_frame accepts
 * model_depth = NULL (reuse the session's MODEL pyramid); a batched step
 * needs the model view. */
typedef struct {
  const float* depth;
  const uint8_t* intensity;
  int32_t pitch;
  const float* model_depth;
  const uint8_t* model_intensity;
  int32_t model_pitch;
  double T_WM[16];
  const dslam_imu_sample* imu;
  int32_t n_imu;
  double t0, t1;
} dslam_frame_input;

/* One result of the launch-shape autotuner: the residual pass of `level` of
 * a width x height camera with `jac_format` runs fastest with `ppt` pixels per
 * thread and, with xcd_banded = 1, its tiles dealt to the GPU's 8
 * accelerator dies (XCDs, each with its own L2 cache) in contiguous bands
 * rather than round-robin (us: its measured time per pass and reduction of
 * its partials). */
typedef struct {
  int32_t width, height, level, jac_format, ppt;
  float us;
  int32_t xcd_banded;
} dslam_tune_entry;

/* Human-readable name of a status code (static string). */
const char* dslam_status_string(dslam_status s);

/* Library build tag: target, compiler and options (static string). */
const char* dslam_build_info(void);

/* Create a context on GPU `device` that admits sessions while their summed
 * device footprint (dslam_session_bytes) stays within hbm_budget_bytes
 * (0 = no limit).  *out is owned by the caller; release with dslam_context_destroy. */
dslam_status dslam_context_create(int32_t device, uint64_t hbm_budget_bytes, dslam_context** out);
dslam_status dslam_context_destroy(dslam_context* ctx);
/* Bytes currently admitted on the context. */
uint64_t dslam_context_used_bytes(const dslam_context* ctx);

/* Tile-shape autotuner for the residual pass.  For each camera cams[0..n) and
 * each of its `levels` pyramid levels, times the pass (jac_format's kernel)
 * followed by the reduction of its block partials (as the Gauss-Newton step
 * starts with it) with 1, 2 and 4 pixels per thread, each with the tiles in round-robin and in
 * XCD-banded order, on a synthetic slanted, textured plane (best of three
 * rounds of 20 launch pairs) and records the first shape in that order within 2%
 * of the fastest in the context; sessions opened on the context afterwards with the
 * same resolution and format use it (a session keeps its tile shape for life,
 * so its results do not depend on batching; the tile order never changes a
 * result, only which die computes each tile).  Runs
 * synchronously on `stream`, with temporary device memory counted against
 * the budget while it runs.  out (nullable, capacity max_out) receives the
 * chosen entries, *n_out their number. */
dslam_status dslam_context_autotune(dslam_context* ctx, const dslam_camera* cams, int32_t n, int32_t levels,
                                    int32_t jac_format, void* stream, dslam_tune_entry* out, int32_t max_out,
                                    int32_t* n_out);
/* Record launch shapes in the context as if the autotuner had chosen them
 * (e.g. entries saved from an earlier dslam_context_autotune run on the same
 * kind of GPU); each replaces the context's entry of the same resolution,
 * level and format.  entries: host, n of them; `us` is kept but not used.
 * Errors: INVALID (ppt not 1, 2 or 4, xcd_banded not 0 or 1, level outside
 * [0, DSLAM_MAX_LEVELS), unknown format, width or height < 1); nothing is
 * recorded then. */
dslam_status dslam_context_set_tune(dslam_context* ctx, const dslam_tune_entry* entries, int32_t n);

/* Device bytes a session of this camera and pyramid depth holds for its lifetime. */
uint64_t dslam_session_bytes(const dslam_camera* cam, int32_t levels);

/* Open a tracking session.  All device memory is allocated here; nothing is
 * allocated per frame.  x0/q_IW/prior give the initial state and its prior
 * (prior may be NULL in DSLAM_MODE_RGBD).  Errors: INVALID (levels outside
 * [1,4], width or height not divisible by 2^(levels-1), non-unit quaternion,
 * unknown mode or format), NO_CAPACITY (budget), DEVICE. */
dslam_status dslam_session_open(dslam_context* ctx, const dslam_camera* cam, const dslam_track_params* tp,
                                const dslam_imu_params* ip, const dslam_frame_state* x0, const double q_IW[4],
                                const dslam_prior* prior, dslam_session** out);
/* Wait for the session's last enqueued work (its own completion event, not
 * the whole device), free its memory and return its bytes to the context.
 * BUSY (nothing freed) while a dslam_server still holds queued or unreturned
 * requests of the session: poll them out, or destroy the server, first. */
dslam_status dslam_session_close(dslam_session* s);

/* Build the session's CURRENT or MODEL pyramid (Section IV-D) from device
 * images: depth_dev (float32, metres) and intensity_dev (uint8), both
 * height x width with row pitch `pitch_elems`.  For MODEL, T_W_ref (4x4,
 * host) is the pose at which the model view was predicted.  Enqueued on
 * `stream`; the caller keeps the inputs alive until the stream passes it. */
dslam_status dslam_build_pyramid(dslam_session* s, int32_t which, const float* depth_dev,
                                 const uint8_t* intensity_dev, int32_t pitch_elems, const double T_W_ref[16],
                                 void* stream);

/* Host float64 IMU preintegration (Section IV-C) over [t0, t1) at the
 * linearisation biases bg, ba.  Samples (host) must be sorted by time, the
 * first stamped at or before t0, and hold the zero-order-hold values.  Noise
 * covariance and bias Jacobians are propagated analytically. */
dslam_status dslam_preintegrate_imu(const dslam_imu_sample* samples, int32_t n, double t0, double t1,
                                    const double bg[3], const double ba[3], const dslam_imu_params* p,
                                    dslam_preint* out);

/* Host float64 Gauss-Newton step (eqs. (6)-(9)) from the raw sums of one
 * residual pass (`raw`, the layout of dslam_linear_system.raw) taken at the
 * states x0, x1 with the model-view pose T_WM (4x4): lift the visual terms,
 * add the IMU factor and the prior (DSLAM_MODE_RGBDI), solve, and update
 * x0, x1 and q_IW in place.  dz_out (33, nullable) receives the increment; if
 * marg_out is not NULL the Schur-complement prior of x0 is written there.
 * SINGULAR leaves the states untouched.  Same arithmetic as the device solve. */
dslam_status dslam_solve_step(const double raw[58], const double T_WM[16], const dslam_preint* pre,
                              const dslam_imu_params* ip, const dslam_track_params* tp, const dslam_prior* prior,
                              dslam_frame_state* x0, dslam_frame_state* x1, double q_IW[4], double dz_out[33],
                              dslam_prior* marg_out);

/* Track one frame (Section IV-A: at the arrival of a frame the current state
 * x1 is estimated while the previous state x0 is refined).  `in` gives the
 * frame (device depth and intensity, host IMU samples covering [t0, t1),
 * n_imu in [1, 32], ignored in DSLAM_MODE_RGBD) and, optionally, the model
 * view it is tracked against (model_depth / model_intensity device images and
 * the pose T_WM at which the view was predicted); with model_depth NULL the
 * MODEL pyramid of an earlier call or of dslam_build_pyramid is used
 * (NOT_READY if there is none).  Builds the CURRENT pyramid (and the MODEL
 * one) in the frame's first launch, beside the device preintegration of the
 * IMU samples at the session's bias estimates and the IMU prediction of x1,
 * then runs the coarse-to-fine Gauss-Newton iterations entirely on the device
 * (Section IV-D), marginalises x0 into the next frame's prior (Section IV-E)
 * and shifts the state.  Asynchronous: returns after enqueueing on `stream`.
 * If `out` is not NULL the frame's result is copied there asynchronously; it
 * is valid once `stream` has passed the frame (dslam_session_result also
 * waits for it).  `out` should be pinned host memory (hipHostMalloc): with
 * pageable memory the copy, and so this call, waits for the frame.  The
 * caller owns the images until the stream passes the frame.  Errors (nothing
 * is enqueued): INVALID (null or short images, IMU samples unsorted, not
 * covering t0 or more than 32, non-finite T_WM, no iterations), NOT_READY,
 * DEVICE. */
dslam_status dslam_track_frame(dslam_session* s, const dslam_frame_input* in, dslam_track_result* out,
                               void* stream);

/* dslam_track_frame, then wait for the frame and copy its result to `out`
 * (host, required).  The result is copied in stream order to pinned memory
 * the session owns, and the wait polls the frame's completion (the calling
 * thread stays busy until the frame ends).  Returns the enqueue error, or
 * DSLAM_OK with the frame's own status (a failed solve) in out->status. */
dslam_status dslam_track_frame_sync(dslam_session* s, const dslam_frame_input* in, dslam_track_result* out,
                                    void* stream);

/* How dslam_track_frame issues a frame's
 * Gauss-Newton launches after the first.  enable = 1: each level's
 * iterations (residual pass, step) are captured in a HIP graph at the first
 * frame that needs them and replayed from then on, one graph launch per
 * level; the first launch stores the frame's inputs in device memory for
 * them.  enable = 0 (the default, faster while the host keeps ahead of the
 * device): every launch is issued on its own.  Both give the same results bit
 * for bit.  Errors: INVALID (enable not 0 or 1); a failed capture makes the
 * tracking call return DEVICE. */
dslam_status dslam_session_set_graphs(dslam_session* s, int32_t enable);

/* Surfel map: the dense model the tracker aligns to (the mapping step the
 * paper keeps from its RGB-D base system, Sections III and V).  A map holds
 * up to `capacity` surfels (world position, unit normal, intensity, radius,
 * confidence) for one camera; dslam_map_fuse adds a tracked frame to it and
 * dslam_map_predict renders the model view the next frame is tracked
 * against.  All of the map's memory is allocated at creation and counted
 * against the context's budget (NO_CAPACITY).  Calls on one map are ordered
 * by the caller's stream; the map's arrays are reproducible bit for bit (the
 * float32 operations are fixed and every surfel is written by at most one
 * thread per call). */
typedef struct dslam_map dslam_map;

typedef struct {
  int32_t capacity;  /* surfels, >= 1 */
  float assoc_dist;  /* metres: a frame pixel joins the surfel of its cell when their depths differ by at most this */
  float assoc_cos;   /* ... and the cosine between their world normals is at least this, in [-1, 1] */
  float render_band; /* metres, >= 0: surfels this far behind a pixel's nearest one still count as its front
                        surface, of which the most central is shown */
} dslam_map_params;

/* Field indices of dslam_map_copy. */
enum {
  DSLAM_MAP_PX = 0, DSLAM_MAP_PY, DSLAM_MAP_PZ, DSLAM_MAP_NX, DSLAM_MAP_NY, DSLAM_MAP_NZ,
  DSLAM_MAP_INTENSITY, DSLAM_MAP_RADIUS, DSLAM_MAP_CONFIDENCE
};

/* Create an empty map for `cam` (level-0 intrinsics; sessions that fuse into
 * or predict from it must use the same camera and context).  Errors:
 * INVALID (arguments), NO_CAPACITY (budget or allocation), DEVICE. */
dslam_status dslam_map_create(dslam_context* ctx, const dslam_camera* cam, const dslam_map_params* p,
                              dslam_map** out);
/* Wait for the map's work and free it. */
dslam_status dslam_map_destroy(dslam_map* m);
/* Empty the map (asynchronous on `stream`). */
dslam_status dslam_map_reset(dslam_map* m, void* stream);
/* Fuse the session's current frame (level 0 of its CURRENT pyramid, i.e. the
 * frame last tracked or built) into the map at its pose T_WC (camera to world,
 * 4x4 row-major, host): each surfel in front of the camera marks the pixel of
 * its projected centre (nearest, then lowest index); a valid pixel (level-0
 * depth, and the normal of its parent pixel at level 1 of a deeper pyramid)
 * whose cell
 * holds a surfel within assoc_dist in depth and assoc_cos in normal updates it
 * with confidence-weighted averages (pixel weight 1 / (1 + g^2), g the
 * distance from the image centre relative to the centre's own distance from
 * the corner); every other valid pixel becomes a new surfel unless one of its
 * 8 neighbouring cells holds a surfel within assoc_dist of its depth,
 * appended in pixel order while the capacity lasts (the rest are counted as
 * dropped).
 * Asynchronous on `stream`.  Errors: INVALID (arguments, camera mismatch),
 * DEVICE. */
dslam_status dslam_map_fuse(dslam_map* m, dslam_session* s, const double T_WC[16], void* stream);
/* Predict the model view at T_WM (4x4 row-major, host) by splatting the
 * surfels (each covers the pixels of its disk; of the surfels within
 * render_band of a pixel's nearest, the one whose centre projects closest to
 * the pixel is shown) and build the
 * session's MODEL pyramid from it, as dslam_build_pyramid(MODEL) would from
 * caller images, except that its level-0 normals are the shown surfels'
 * (camera frame; zero where no surfel covers the pixel).  Asynchronous on
 * `stream`.  Errors as dslam_map_fuse. */
dslam_status dslam_map_predict(dslam_map* m, dslam_session* s, const double T_WM[16], void* stream);
/* The same prediction into caller device images (height x width, pitch =
 * width): depth in metres (0 where no surfel covers the pixel) and intensity.
 * Asynchronous on `stream`. */
dslam_status dslam_map_render(dslam_map* m, const double T_WM[16], float* depth_dev, uint8_t* intensity_dev,
                              void* stream);
/* Deform the map by a solved deformation graph (dslam_deform_solve): each
 * surfel moves to phi(p) over its 4 nearest of the n_nodes (5..256) nodes
 * (host, 3 doubles each) with the node parameters `params` (host, 12 per
 * node: A row-major, then t), and its normal to the normalised
 * sum_k w_k A_k n; evaluated in float64, rounded once to the map's float32.
 * Waits for the device.  Errors: INVALID (arguments, non-finite input),
 * DEVICE. */
dslam_status dslam_map_deform(dslam_map* m, int32_t n_nodes, const double* nodes, const double* params,
                              void* stream);
/* Wait for the map's last call and read its surfel count and the number of
 * new surfels dropped so far for lack of capacity (nullable). */
dslam_status dslam_map_count(dslam_map* m, int32_t* count, int32_t* dropped);
/* Wait for the map's last call and copy one field (DSLAM_MAP_*) of its
 * surfels, in index order, to host memory (at most max_surfels floats;
 * INVALID if the map holds more). */
dslam_status dslam_map_copy(dslam_map* m, int32_t field, float* host_out, int32_t max_surfels);

/* Deformation graph with the gravity term (Section V, eqs. (10)-(17)): the
 * non-rigid correction the paper applies to its map on a loop closure.
 * Nodes l sit at positions g_l and carry a 3x3 matrix A_l and a translation
 * t_l; a point v deforms as phi(v) = sum_k w_k (A_k (v - g_k) + g_k + t_k)
 * over its 4 nearest nodes, w_k = (1 - |v - g_k| / d_max)^2 normalised, d_max
 * the distance of the 5th nearest.  The cost is
 * E = 1 E_rot + 10 E_reg + 100 (E_con + E_pin [+ E_rel]) + 100 E_imu with
 * E_rot = sum |A^T A - I|_F^2, E_reg over each node's 4 nearest other nodes,
 * E_con = sum |phi(source) - destination|^2, E_pin = sum |phi(d) - d|^2 over
 * pinned points, E_rel = sum |phi(source) - phi(destination)|^2 over earlier
 * registrations (global closures only) and E_imu = sum |A g_W - g_W|^2. */
typedef struct dslam_deform dslam_deform;

typedef struct {
  int32_t n_nodes;     /* >= 6 */
  const double* nodes; /* host, 3 per node */
  int32_t n_con;
  const double* con;   /* host, source xyz then destination xyz per constraint */
  int32_t n_pin;
  const double* pin;   /* host, xyz per pinned point */
  int32_t n_rel;
  const double* rel;   /* host, source xyz then destination xyz per earlier registration */
  int32_t global;      /* 1: global closure (E_rel included), 0: local */
  double g_W[3];       /* gravity in the vision-world frame */
} dslam_deform_problem;

/* Allocate a solver for up to max_nodes (6..256) nodes and max_points
 * constraint points (con + pin + rel) on the context's device (counted
 * against its budget).  The system is held dense: with n = 12 max_nodes
 * unknowns and m = 24 max_nodes + 3 max_points residual rows (both rounded
 * up to 16), about 8 (m (n + 1) + 2 (n + 1)^2) + 612 m bytes ([J r], the
 * normal matrix, its factor, the per-tile row lists): 328 MB at 256 nodes
 * and 256 points.  Errors: INVALID, NO_CAPACITY. */
dslam_status dslam_deform_create(dslam_context* ctx, int32_t max_nodes, int32_t max_points, dslam_deform** out);
dslam_status dslam_deform_destroy(dslam_deform* d);
/* Minimise E by `iters` (1..63) Gauss-Newton steps from A = I, t = 0 on the
 * device (each step: residuals and Jacobians, the normal equations, a
 * Cholesky solve) and copy the node parameters to params_out (host, 12 per
 * node: A row-major, then t) and, if cost_out is not NULL, the cost before
 * each step (iters values).  Waits for the device.  Errors: INVALID
 * (arguments, sizes, non-finite input), SINGULAR (the normal equations were
 * not positive definite: too few constraints), DEVICE. */
dslam_status dslam_deform_solve(dslam_deform* d, const dslam_deform_problem* p, int32_t iters, double* params_out,
                                double* cost_out, void* stream);

/* Wait for the session's last tracked frame and copy its result to host memory. */
dslam_status dslam_session_result(dslam_session* s, dslam_track_result* out);

/* One residual pass at `level` with caller-chosen float32 transforms:
 * (Ra, ta) map current-camera points into the model-view camera (ICP
 * association) and (Rb, tb) into the reference camera of x0 (photometric
 * warp), each rotation given as its offset from the identity, R - I,
 * rounded to float32 from float64 (a point maps as p + ((R - I) p + t));
 * x0, x1 (host) give the float64 poses used to lift the sums to the world
 * frame.  If mask_dev (device, width_l x height_l bytes) is not NULL, each
 * pixel gets bit 0 = ICP inlier, bit 1 = photometric inlier.  Synchronous. */
dslam_status dslam_linearize(dslam_session* s, int32_t level, const float Ra[9], const float ta[3],
                             const float Rb[9], const float tb[3], const dslam_frame_state* x0,
                             const dslam_frame_state* x1, uint8_t* mask_dev, dslam_linear_system* out,
                             void* stream);

/* Launch the residual pass of `level` `reps` times back to back on `stream`
 * with the session's current transforms, writing only its scratch partials
 * (the estimator state is untouched).  For timing the pass with events on
 * the caller's stream.  Asynchronous.  NOT_READY without both pyramids. */
dslam_status dslam_profile_residual(dslam_session* s, int32_t level, int32_t reps, void* stream);

/* Copy one channel of one pyramid level to host memory (width_l*height_l floats). Synchronous. */
dslam_status dslam_copy_pyramid(dslam_session* s, int32_t which, int32_t level, int32_t channel, float* host_out);

/* Batched tracking (serving form): one step tracks one frame of each of n
 * sessions with shared launches, so that many sessions fill the GPU.  Every
 * session's arithmetic is the same as in dslam_track_frame (same pixel
 * partition, order of sums and solve), so its result does not depend on the
 * other sessions of the batch.
 *
 * dslam_batch_create allocates the staging memory for up to max_sessions
 * (<= DSLAM_MAX_BATCH) sessions (device and pinned host; counted against the
 * context's budget, NO_CAPACITY otherwise). */
dslam_status dslam_batch_create(dslam_context* ctx, int32_t max_sessions, dslam_batch** out);
/* Wait for the batch's work and free it. */
dslam_status dslam_batch_destroy(dslam_batch* b);
/* Enqueue one tracking step for sessions[0..n) with frames[0..n) on `stream`
 * (Section IV, as dslam_track_frame, plus both pyramids of each session built
 * from frames[i]).  The sessions must belong to the batch's context, be
 * distinct, share the pyramid depth and iteration counts, and use at most
 * DSLAM_MAX_BATCH_RESOLUTIONS distinct resolutions.  Waits first for the
 * batch's previous step (its staging memory is reused).  The caller keeps the
 * device images alive until the step completes.  Asynchronous; errors:
 * INVALID (arguments), DEVICE. */
dslam_status dslam_batch_track(dslam_batch* b, int32_t n, dslam_session* const* sessions,
                               const dslam_frame_input* frames, void* stream);
/* Wait for the batch's last step and copy its n results, in call order. */
dslam_status dslam_batch_results(dslam_batch* b, dslam_track_result* out);
/* Tile order of the batch's residual passes (see dslam_tune_entry): 1 = dealt
 * to the XCDs in contiguous bands (the default: at batch scale neighbouring
 * tiles read the same model-view rows, and banding lets them share an L2
 * instead of fetching those rows once per die), 0 = round-robin, -1 = the
 * order tuned for the batch's largest sessions.  The order never changes a
 * result.  Applies to later steps and to dslam_batch_profile_residual.  Waits
 * for the batch's last step.  Errors: INVALID (order outside [-1, 1]). */
dslam_status dslam_batch_set_tile_order(dslam_batch* b, int32_t order);
/* enable = 1: the batch's later steps replay their kernel launches from HIP
 * graphs (Section IV's per-frame schedule for the whole batch: both
 * pyramids, the initialisation, every level's residual passes and
 * Gauss-Newton steps, the marginalisation and the gathering of the results).
 * One graph is captured per plan of launches, i.e. per batch composition
 * (sessions per resolution and launch shape, in slot order) and schedule, at
 * the first step with that plan, and replayed by later steps with the same
 * plan; the batch keeps the 32 most recent.  The staging copies stay outside
 * the graphs.  Results are bit for bit those of the launches issued one by
 * one (enable = 0, the default; disabling frees the graphs).  Waits for the
 * batch's last step.  Errors: INVALID (enable not 0 or 1), DEVICE. */
dslam_status dslam_batch_set_graphs(dslam_batch* b, int32_t enable);

/* The batched step for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step as dslam_batch_track followed by dslam_batch_results, with the same
 * results bit for bit (XCD-banded tile order), but no dslam_batch is needed
 * and nothing is allocated.
 * The slot records and results live in a static device array of 1.8 MiB
 * (DSLAM_MAX_BATCH sessions' records; each GPU the library runs on holds its
 * own copy until the process ends, its address resolved by
 * dslam_context_create) and static host staging.  Every call on a GPU shares
 * that GPU's array, which keeps the last call's contents (every record the
 * step reads is written by the call first, so nothing needs clearing); calls
 * are serialised by the library and each waits for its step, so calls that
 * would overlap on one GPU run one after the other.  Sessions as for
 * dslam_batch_track (all of one context); results (host, n entries) in call
 * order.  Errors: INVALID (arguments, n > DSLAM_MAX_BATCH), DEVICE. */
dslam_status dslam_batch_track_noalloc(int32_t n, dslam_session* const* sessions, const dslam_frame_input* frames,
                                       dslam_track_result* results, void* stream);
/* Launch the batched residual pass of `level` of the batch's last step `reps`
 * times back to back on `stream` (same sessions, transforms and work split;
 * only the sessions' scratch partials are written, no estimator state
 * changes).  *pixels (nullable) receives the pixels one launch processes.  For
 * timing the pass with events on the caller's stream.  Asynchronous once the
 * last step has completed. */
dslam_status dslam_batch_profile_residual(dslam_batch* b, int32_t level, int32_t reps, void* stream,
                                          uint64_t* pixels);

/* Serving loop with continuous batching.  Frames of many sessions are
 * submitted as requests; each poll retires finished batched steps and
 * launches new ones from the pending requests: every session with a pending
 * frame joins the next step with its oldest one (up to max_batch sessions
 * with the same pyramid schedule), and up to pipeline_depth steps are in
 * flight at once on the server's own streams, so requests that arrive while
 * others are on the GPU are admitted as soon as a step slot frees up.  A
 * session's next frame may join a step while its previous frame is still
 * running; the device orders the two.  Sessions are admitted by the context's HBM budget at
 * dslam_session_open (NO_CAPACITY when it is exhausted).  A session's frames
 * are tracked in submission order.  Not thread-safe: one thread drives a
 * server. */
typedef struct dslam_server dslam_server;

typedef struct {
  int32_t max_batch;       /* sessions per batched step, 1..DSLAM_MAX_BATCH */
  int32_t pipeline_depth;  /* batched steps in flight at once, 1..8 */
  int32_t use_graphs;      /* 1: the steps replay their launches from graphs (dslam_batch_set_graphs), 0: not */
} dslam_server_params;

/* A finished request.  submit_s / done_s are host steady-clock seconds (the
 * same clock as dslam_server_clock) at submission and at the poll that
 * retired it; device_ms is the GPU time of the batched step that ran it
 * (from the end of its sessions' earlier work to its own end). */
typedef struct {
  uint64_t request_id;
  dslam_session* session;
  double submit_s, launch_s, done_s;
  float device_ms;
  int32_t batch_size;
  dslam_track_result result;
} dslam_request_done;

dslam_status dslam_server_create(dslam_context* ctx, const dslam_server_params* p, dslam_server** out);
/* Wait for in-flight steps and free the server (pending requests are dropped). */
dslam_status dslam_server_destroy(dslam_server* sv);
/* Queue one frame of `session` (opened on the server's context).  The frame
 * input is copied, IMU samples included; its device images must stay valid
 * until the request is returned by dslam_server_poll.  *request_id receives a
 * server-unique id.  Errors: INVALID (arguments, IMU samples). */
dslam_status dslam_server_submit(dslam_server* sv, dslam_session* session, const dslam_frame_input* frame,
                                 uint64_t* request_id);
/* Retire finished steps, launch new ones, and copy up to max_out finished
 * requests to out (*n_out of them).  With wait != 0 and nothing finished yet,
 * blocks until the oldest in-flight step completes.  Returns the first error
 * met while launching or retiring a step; the requests of that step are
 * returned with the error in result.status. */
dslam_status dslam_server_poll(dslam_server* sv, int32_t wait, dslam_request_done* out, int32_t max_out,
                               int32_t* n_out);
/* Requests queued but not launched, and launched but not yet returned. */
dslam_status dslam_server_counts(const dslam_server* sv, int32_t* pending, int32_t* in_flight);
/* The server's clock (steady clock, seconds). */
double dslam_server_clock(void);

/* Session checkpoint as an opaque, versioned byte blob in caller host memory:
 * everything the session's later frames depend on -- the estimator state
 * (x0, q_IW, the marginal prior of Section IV-E, the frame counter), the
 * model-view pose and MODEL pyramid (so that frames tracked against the
 * previous model view continue), and the camera and tracking parameters it
 * was taken under.  dslam_session_checkpoint with buf NULL writes the size
 * to *size; otherwise buf must hold at least dslam_session_checkpoint's size
 * (INVALID otherwise).  Waits for the session's work.  dslam_session_restore
 * loads a blob into a session opened with the same camera, pyramid depth and
 * tracking parameters (INVALID for a foreign, truncated, corrupted or
 * mismatched blob; the session is unchanged then); frames tracked after a
 * restore give the same results, bit for bit, as frames tracked after the
 * checkpoint by the session it was taken from.  BUSY while a server holds
 * requests of the session. */
dslam_status dslam_session_checkpoint(dslam_session* s, void* buf, uint64_t capacity, uint64_t* size);
dslam_status dslam_session_restore(dslam_session* s, const void* buf, uint64_t size);

/* The estimator state alone (x0, q_IW, prior, frame counter) through host
 * memory, to start a session over from a known state; the pyramids are not
 * part of it.  Waits for the session's work. */
dslam_status dslam_session_get_state(dslam_session* s, dslam_frame_state* x0, double q_IW[4], dslam_prior* prior,
                                     int32_t* frame_index);
dslam_status dslam_session_set_state(dslam_session* s, const dslam_frame_state* x0, const double q_IW[4],
                                     const dslam_prior* prior, int32_t frame_index);

#ifdef __cplusplus
}
#endif

#endif /* DSLAM_H */
