// Host side of the C ABI declared in include/dslam.h: contexts, sessions,
// argument checking, launch sequencing of the tracking step and the host
// float64 entry points (preintegration and Gauss-Newton step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "host.h"


using namespace dslam;

// ---- static scratch of the allocation-free batched step ---------------------
// One batched step's slot records and results (the memory a dslam_batch
// allocates) for up to DSLAM_MAX_BATCH sessions, in a file-scope device array:
// every GPU the library runs on holds its own copy until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in), resolved
// once per device by dslam_context_create.
static constexpr size_t al256(size_t n) { return (n + 255) & ~size_t(255); }
static constexpr size_t kScratchVis = al256(sizeof(dslam::SlotVis) * DSLAM_MAX_BATCH);
static constexpr size_t kScratchSolve = al256(sizeof(dslam::SlotSolve) * DSLAM_MAX_BATCH);
static constexpr size_t kScratchRes = al256(sizeof(dslam_track_result) * DSLAM_MAX_BATCH);
static constexpr size_t kScratchBytes = kScratchVis + kScratchSolve + kScratchRes;
static_assert(kScratchBytes <= (4u << 20), "the static scratch stays within 4 MiB");
static __device__ __attribute__((aligned(256))) unsigned char scratch[kScratchBytes];

namespace {

const char* kStatus[] = {"ok", "invalid argument", "no capacity", "singular system", "device error", "busy",
                         "not ready"};

#define HIP_OK(expr)                           \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return DSLAM_ERR_DEVICE; \
  } while (0)

bool quat_ok(const double* q) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  return std::isfinite(n) && std::fabs(n - 1.0) <= 1e-6;
}

bool state_ok(const dslam_frame_state* x) {
  if (!x || !quat_ok(x->q)) return false;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(x->r[i]) || !std::isfinite(x->v[i]) || !std::isfinite(x->bg[i]) || !std::isfinite(x->ba[i]))
      return false;
  return true;
}

bool params_ok(const dslam_camera* cam, const dslam_track_params* tp) {
  if (!cam || !tp) return false;
  if (tp->levels < 1 || tp->levels > DSLAM_MAX_LEVELS) return false;
  int div = 1 << (tp->levels - 1);
  if (cam->width < 8 || cam->height < 8 || cam->width % div || cam->height % div) return false;
  if ((cam->width >> (tp->levels - 1)) < 4 || (cam->height >> (tp->levels - 1)) < 4) return false;
  if ((int64_t)cam->width * cam->height > (1 << 26)) return false;
  if (!(cam->fx > 0) || !(cam->fy > 0) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy)) return false;
  for (int l = 0; l < tp->levels; ++l)
    if (tp->iters[l] < 0 || tp->iters[l] > 1000) return false;
  if (tp->mode != DSLAM_MODE_RGBDI && tp->mode != DSLAM_MODE_RGBD && tp->mode != DSLAM_MODE_GYRO) return false;
  if (tp->jac_format < DSLAM_JAC_FP32 || tp->jac_format > DSLAM_JAC_BF16) return false;
  if (!(tp->icp_dist > 0) || !(tp->icp_cos <= 1) || !(tp->sigma_I > 0) ||
      !(tp->depth_k > 0) || !(tp->huber_k >= 0))
    return false;
  if (!(tp->min_inlier_frac >= 0 && tp->min_inlier_frac <= 1) || !(tp->max_cost_rise >= 0) ||
      !std::isfinite(tp->max_cost_rise) || (tp->imu_fallback != 0 && tp->imu_fallback != 1))
    return false;
  return true;
}

void level_intrinsics(const dslam_camera& c, int l, LevelPtrs* L) {
  double s = std::ldexp(1.0, -l);
  L->W = c.width >> l;
  L->H = c.height >> l;
  L->fx = (float)(c.fx * s);
  L->fy = (float)(c.fy * s);
  L->cx = (float)((c.cx + 0.5) * s - 0.5);
  L->cy = (float)((c.cy + 0.5) * s - 0.5);
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct Layout {
  size_t planes, partial_floats, total;
  int max_blocks;
};

Layout layout_for(const dslam_camera& c, int levels) {
  Layout lo{0, 0, 0, 0};
  size_t planes = 0;
  for (int l = 0; l < levels; ++l) {
    size_t n = (size_t)(c.width >> l) * (c.height >> l);
    // current: V (3), N (3) float32 + I uint16; model: the same + G (2) int16
    planes += 12 * align256(n * sizeof(float)) + 4 * align256(n * sizeof(uint16_t));
  }
  int nb = residual_blocks(c.width * c.height, 1);
  lo.planes = planes;
  lo.max_blocks = nb;
  lo.partial_floats = (size_t)nb * PARTIAL_STRIDE;
  lo.total = planes + align256(lo.partial_floats * sizeof(float)) + align256(sizeof(SessionDev)) +
             align256(64 * sizeof(double)) + align256(24 * sizeof(float)) + align256(sizeof(SolveParams));
  return lo;
}

ImuParamsD imu_params_d(const dslam_imu_params& ip) {
  ImuParamsD d;
  d.gravity = ip.gravity;
  d.sigma_bg_rw = ip.sigma_bg_rw;
  d.sigma_ba_rw = ip.sigma_ba_rw;
  for (int i = 0; i < 9; ++i) d.R_CS[i] = ip.R_CS[i];
  for (int i = 0; i < 3; ++i) d.t_CS[i] = ip.t_CS[i];
  return d;
}

// Nearest depth (metres) for which the FP16 row scales keep every entry in range.
constexpr double kFp16MinDepth = 0.25;

int default_ppt(int npix) { return npix >= 600000 ? 4 : (npix >= 150000 ? 2 : 1); }

ResidualArgs residual_args(dslam_session* s, int l, const float* xf, uint8_t* mask) {
  const LevelPtrs& c = s->cur[l];
  const LevelPtrs& m = s->model[l];
  ResidualArgs a;
  a.cV0 = c.V[0]; a.cV1 = c.V[1]; a.cV2 = c.V[2];
  a.cN0 = c.N[0]; a.cN1 = c.N[1]; a.cN2 = c.N[2];
  a.cI = c.I;
  a.mV0 = m.V[0]; a.mV1 = m.V[1]; a.mV2 = m.V[2];
  a.mN0 = m.N[0]; a.mN1 = m.N[1]; a.mN2 = m.N[2];
  a.mI = m.I; a.mG0 = m.G[0]; a.mG1 = m.G[1];
  a.W = c.W; a.H = c.H; a.npix = c.W * c.H;
  a.fx = c.fx; a.fy = c.fy; a.cx = c.cx; a.cy = c.cy;
  a.dist2 = (float)(s->tp.icp_dist * s->tp.icp_dist);
  a.cosmin = (float)s->tp.icp_cos;
  a.depth_k = (float)s->tp.depth_k;
  a.sigma_I = (float)s->tp.sigma_I;
  a.huber_k = (float)s->tp.huber_k;
  a.xf = xf;
  a.partials = s->partials;
  a.mask = mask;
  a.jac = s->tp.jac_format;
  a.col_scale[0] = a.col_scale[1] = 1.0f;
  a.banded = s->banded[l];
  if (a.jac == DSLAM_JAC_FP16) {
    // Power-of-two scales that bring each term's largest possible row entry
    // to about 2^14 (FP16 overflows above 65504), from bounds at the nearest
    // depth the scales are sized for (entries beyond saturate):
    //   ICP: sqrt(W) = 1/(k z^2), |j| <= max(1, |p|) with |p| <= 1.5 z;
    //   photometric: sqrt(W) = 1/sigma_I, |j| <= 255 fx_l / z (gradient times
    //   projection Jacobian; the rotational part is bounded by the same).
    const double zmin = kFp16MinDepth;
    const double b_icp = std::max(1.0, 1.5 * zmin) / (s->tp.depth_k * zmin * zmin);
    const double b_rgb = 255.0 * c.fx / (s->tp.sigma_I * zmin);
    a.col_scale[0] = (float)std::ldexp(1.0, 14 - (int)std::ceil(std::log2(b_icp)));
    a.col_scale[1] = (float)std::ldexp(1.0, 14 - (int)std::ceil(std::log2(b_rgb)));
  }
  return a;
}

int last_level_of(const dslam_track_params& tp);

SolveParams solve_params(dslam_session* s) {
  SolveParams sp;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) sp.R_WM[3 * r + c] = s->T_WM[4 * r + c];
    sp.t_WM[r] = s->T_WM[4 * r + 3];
  }
  sp.imu = imu_params_d(s->ip);
  sp.mode = s->tp.mode;
  sp.marginalise = 1;  // the device solve marginalises on the frame's last step only
  // health thresholds: inliers of both terms at the frame's finest level
  const int fl = last_level_of(s->tp);
  const double npix = fl >= 0 ? (double)s->cur[fl].W * (double)s->cur[fl].H : 0.0;
  sp.min_inliers = s->tp.min_inlier_frac > 0.0 ? s->tp.min_inlier_frac * 2.0 * npix : 0.0;
  sp.max_cost_rise = s->tp.max_cost_rise > 0.0 ? s->tp.max_cost_rise : 0.0;
  sp.imu_fallback = s->tp.imu_fallback == 1 && s->tp.mode == DSLAM_MODE_RGBDI ? 1 : 0;
  return sp;
}

// The launch shape the autotuner chose for this resolution, level and format
// (ppt 0: none).
dslam_tune_entry tuned_shape(dslam_context* ctx, int W, int H, int level, int jac) {
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  for (const dslam_tune_entry& e : ctx->tuned)
    if (e.width == W && e.height == H && e.level == level && e.jac_format == jac) return e;
  dslam_tune_entry none{W, H, level, jac, 0, 0.0f, 0};
  return none;
}

// Validates the frame's IMU samples and packs them for the device.
dslam_status pack_imu(const dslam_session* s, const dslam_imu_sample* imu, int32_t n_imu, double t0, double t1,
                      ImuBatch* batch) {
  std::memset(batch, 0, sizeof(*batch));
  if (s->tp.mode == DSLAM_MODE_RGBD) return DSLAM_OK;
  if (!imu || n_imu < 1 || n_imu > DSLAM_MAX_IMU_SAMPLES || !(t1 > t0)) return DSLAM_ERR_INVALID;
  if (!(imu[0].t <= t0)) return DSLAM_ERR_INVALID;
  for (int k = 1; k < n_imu; ++k)
    if (!(imu[k].t > imu[k - 1].t)) return DSLAM_ERR_INVALID;
  batch->n = n_imu;
  batch->t0 = t0;
  batch->t1 = t1;
  for (int k = 0; k < n_imu; ++k) batch->s[k] = imu[k];
  return DSLAM_OK;
}

FrameArgs frame_args(dslam_session* s, const SolveParams& sp) {
  FrameArgs fa;
  fa.imu = imu_params_d(s->ip);
  fa.sigma_g = s->ip.sigma_g;
  fa.sigma_a = s->ip.sigma_a;
  for (int i = 0; i < 9; ++i) fa.R_WM[i] = sp.R_WM[i];
  for (int i = 0; i < 3; ++i) fa.t_WM[i] = sp.t_WM[i];
  fa.mode = s->tp.mode;
  fa.imu_fallback = sp.imu_fallback;
  return fa;
}

int last_level_of(const dslam_track_params& tp) {
  int last = -1;
  for (int l = tp.levels - 1; l >= 0; --l)
    if (tp.iters[l] > 0) last = l;
  return last;
}

bool finite16(const double* T) {
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  return true;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: the device address of its scratch copy, once.
hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

// host staging of the same records (static, pageable: their copies complete
// before the call returns); one host thread uses them at a time
SlotVis g_hvis[DSLAM_MAX_BATCH];
SlotSolve g_hsolve[DSLAM_MAX_BATCH];
dslam_track_result g_hres[DSLAM_MAX_BATCH];
std::mutex g_noalloc_mu;

}  // namespace

extern "C" {

const char* dslam_status_string(dslam_status s) {
  int i = (int)s;
  return (i >= 0 && i < (int)(sizeof(kStatus) / sizeof(kStatus[0]))) ? kStatus[i] : "unknown status";
}

const char* dslam_build_info(void) {
  return "dslam gfx950 HIP " DSLAM_BUILD_TAG;
}

dslam_status dslam_context_create(int32_t device, uint64_t hbm_budget_bytes, dslam_context** out) {
  if (!out) return DSLAM_ERR_INVALID;
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(device));
  HIP_OK(resolve_scratch(device));  // the static batch scratch of this device (dslam_batch_track_noalloc)
  dslam_context* c = new (std::nothrow) dslam_context;
  if (!c) return DSLAM_ERR_NO_CAPACITY;
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return DSLAM_OK;
}

dslam_status dslam_context_destroy(dslam_context* ctx) {
  if (!ctx) return DSLAM_ERR_INVALID;
  if (ctx->used.load() != 0) return DSLAM_ERR_BUSY;
  delete ctx;
  return DSLAM_OK;
}

uint64_t dslam_context_used_bytes(const dslam_context* ctx) { return ctx ? ctx->used.load() : 0; }

uint64_t dslam_session_bytes(const dslam_camera* cam, int32_t levels) {
  if (!cam || levels < 1 || levels > DSLAM_MAX_LEVELS || cam->width <= 0 || cam->height <= 0) return 0;
  return layout_for(*cam, levels).total;
}

dslam_status dslam_session_open(dslam_context* ctx, const dslam_camera* cam, const dslam_track_params* tp,
                                const dslam_imu_params* ip, const dslam_frame_state* x0, const double q_IW[4],
                                const dslam_prior* prior, dslam_session** out) {
  if (!ctx || !out || !params_ok(cam, tp) || !ip || !state_ok(x0) || !q_IW || !quat_ok(q_IW)) return DSLAM_ERR_INVALID;
  if (tp->mode != DSLAM_MODE_RGBD && !prior) return DSLAM_ERR_INVALID;
  Layout lo = layout_for(*cam, tp->levels);
  uint64_t prev = ctx->used.fetch_add(lo.total);
  if (ctx->budget && prev + lo.total > ctx->budget) {
    ctx->used.fetch_sub(lo.total);
    return DSLAM_ERR_NO_CAPACITY;
  }
  dslam_session* s = new (std::nothrow) dslam_session;
  if (!s) {
    ctx->used.fetch_sub(lo.total);
    return DSLAM_ERR_NO_CAPACITY;
  }
  s->ctx = ctx;
  s->cam = *cam;
  s->tp = *tp;
  s->ip = *ip;
  s->levels = tp->levels;
  s->bytes = lo.total;
  s->have_model = false;
  s->cur_normals_ok = true;
  s->max_blocks = lo.max_blocks;
  s->use_graphs = false;
  s->capture = nullptr;
  for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) s->graph[l] = nullptr;
  for (int i = 0; i < 16; ++i) s->T_WM[i] = (i % 5 == 0) ? 1.0 : 0.0;
  auto fail = [&](dslam_status st) {
    if (s->arena) (void)hipFree(s->arena);
    if (s->h_result) (void)hipHostFree(s->h_result);
    ctx->used.fetch_sub(lo.total);
    delete s;
    return st;
  };
  s->arena = nullptr;
  s->h_result = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  if (hipMalloc(&s->arena, lo.total) != hipSuccess) {
    s->arena = nullptr;
    return fail(DSLAM_ERR_NO_CAPACITY);
  }
  char* p = (char*)s->arena;
  for (int l = 0; l < s->levels; ++l) {
    const size_t npx = (size_t)(cam->width >> l) * (cam->height >> l);
    const size_t b32 = align256(npx * sizeof(float)), b16 = align256(npx * sizeof(uint16_t));
    LevelPtrs* C = &s->cur[l];
    LevelPtrs* M = &s->model[l];
    level_intrinsics(*cam, l, C);
    level_intrinsics(*cam, l, M);
    for (LevelPtrs* L : {C, M}) {
      for (int k = 0; k < 3; ++k) { L->V[k] = (float*)p; p += b32; }
      for (int k = 0; k < 3; ++k) { L->N[k] = (float*)p; p += b32; }
      L->I = (uint16_t*)p; p += b16;
    }
    C->G[0] = C->G[1] = nullptr;
    for (int k = 0; k < 2; ++k) { M->G[k] = (int16_t*)p; p += b16; }
    const dslam_tune_entry tuned = tuned_shape(ctx, cam->width, cam->height, l, tp->jac_format);
    s->ppt[l] = tuned.ppt ? tuned.ppt : default_ppt(C->W * C->H);
    s->banded[l] = tuned.ppt ? tuned.xcd_banded : 0;
  }
  s->partials = (float*)p; p += align256(lo.partial_floats * sizeof(float));
  s->sd = (SessionDev*)p; p += align256(sizeof(SessionDev));
  s->red_out = (double*)p; p += align256(64 * sizeof(double));
  s->xf_scratch = (float*)p; p += align256(24 * sizeof(float));
  s->sp_dev = (SolveParams*)p;
  s->last_stream = nullptr;
  s->enqueued = false;
  SessionDev init;
  std::memset(&init, 0, sizeof(init));
  init.x0 = *x0;
  init.x1 = *x0;
  for (int i = 0; i < 4; ++i) init.qIW[i] = q_IW[i];
  if (prior) init.prior = *prior;
  if (hipMemset(s->arena, 0, lo.total) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  if (hipHostMalloc((void**)&s->h_result, sizeof(dslam_track_result), hipHostMallocDefault) != hipSuccess) {
    s->h_result = nullptr;
    return fail(DSLAM_ERR_NO_CAPACITY);
  }
  if (hipMemcpy(s->sd, &init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  s->own_done = std::make_shared<DoneEvent>();
  if (hipEventCreateWithFlags(&s->own_done->ev, hipEventDisableTiming) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  s->done = s->own_done;
  *out = s;
  return DSLAM_OK;
}

dslam_status dslam_context_set_tune(dslam_context* ctx, const dslam_tune_entry* entries, int32_t n) {
  if (!ctx || n < 0 || (n > 0 && !entries)) return DSLAM_ERR_INVALID;
  for (int i = 0; i < n; ++i) {
    const dslam_tune_entry& e = entries[i];
    if ((e.ppt != 1 && e.ppt != 2 && e.ppt != 4) || (e.xcd_banded != 0 && e.xcd_banded != 1) || e.level < 0 ||
        e.level >= DSLAM_MAX_LEVELS || e.jac_format < DSLAM_JAC_FP32 || e.jac_format > DSLAM_JAC_BF16 ||
        e.width < 1 || e.height < 1)
      return DSLAM_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  for (int i = 0; i < n; ++i) {
    const dslam_tune_entry& f = entries[i];
    bool replaced = false;
    for (dslam_tune_entry& e : ctx->tuned)
      if (e.width == f.width && e.height == f.height && e.level == f.level && e.jac_format == f.jac_format) {
        e = f;
        replaced = true;
      }
    if (!replaced) ctx->tuned.push_back(f);
  }
  return DSLAM_OK;
}

dslam_status dslam_context_autotune(dslam_context* ctx, const dslam_camera* cams, int32_t n, int32_t levels,
                                    int32_t jac_format, void* stream, dslam_tune_entry* out, int32_t max_out,
                                    int32_t* n_out) {
  if (!ctx || !cams || n < 1 || levels < 1 || levels > DSLAM_MAX_LEVELS || max_out < 0 || (max_out > 0 && !out))
    return DSLAM_ERR_INVALID;
  dslam_track_params tp;
  std::memset(&tp, 0, sizeof(tp));
  tp.levels = levels;
  for (int l = 0; l < levels; ++l) tp.iters[l] = 1;
  tp.icp_dist = 0.10;
  tp.icp_cos = -2.0;
  tp.sigma_I = 4.0;
  tp.depth_k = 1e-3;
  tp.huber_k = 1.345;
  tp.jac_format = jac_format;
  tp.mode = DSLAM_MODE_RGBD;
  for (int c = 0; c < n; ++c)
    if (!params_ok(&cams[c], &tp)) return DSLAM_ERR_INVALID;
  dslam_imu_params ip;
  std::memset(&ip, 0, sizeof(ip));
  dslam_frame_state x0;
  std::memset(&x0, 0, sizeof(x0));
  x0.q[0] = 1.0;
  const double q[4] = {1.0, 0.0, 0.0, 0.0};
  double T[16];
  for (int i = 0; i < 16; ++i) T[i] = (i % 5 == 0) ? 1.0 : 0.0;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  std::vector<dslam_tune_entry> found;
  dslam_status rc = DSLAM_OK;
  for (int c = 0; c < n && rc == DSLAM_OK; ++c) {
    const dslam_camera& cam = cams[c];
    dslam_session* s = nullptr;
    rc = dslam_session_open(ctx, &cam, &tp, &ip, &x0, q, nullptr, &s);
    if (rc != DSLAM_OK) break;
    void* img = nullptr;
    const size_t npx = (size_t)cam.width * cam.height;
    if (hipMalloc(&img, npx * 5) != hipSuccess) {
      (void)dslam_session_close(s);
      rc = DSLAM_ERR_NO_CAPACITY;
      break;
    }
    float* depth = (float*)img;
    uint8_t* inten = (uint8_t*)img + npx * 4;
    auto run = [&]() -> dslam_status {
      if (launch_tune_scene(depth, inten, cam.width, cam.height, st) != hipSuccess) return DSLAM_ERR_DEVICE;
      dslam_status b = dslam_build_pyramid(s, DSLAM_PYR_MODEL, depth, inten, cam.width, T, st);
      if (b == DSLAM_OK) b = dslam_build_pyramid(s, DSLAM_PYR_CURRENT, depth, inten, cam.width, nullptr, st);
      if (b != DSLAM_OK) return b;
      // identity transforms: every valid pixel associates with itself
      if (hipMemsetAsync(s->sd->xf, 0, sizeof(s->sd->xf), st) != hipSuccess) return DSLAM_ERR_DEVICE;
      for (int l = 0; l < levels; ++l) {
        ResidualArgs ra = residual_args(s, l, s->sd->xf, nullptr);
        // a shape is timed as the pass plus the fixed-order reduction of its block
        // partials that the Gauss-Newton step starts with (fewer pixels per
        // thread make a faster pass but more partials to add); each shape's time
        // is the best of three rounds of back-to-back launches, and the first
        // shape (in the order below) within 2% of the fastest wins, so that
        // shapes whose times differ by noise alone do not flip between runs
        const int shapes[6][2] = {{1, 0}, {1, 1}, {2, 0}, {2, 1}, {4, 0}, {4, 1}};
        float t[6];
        for (int c = 0; c < 6; ++c) {
          ra.banded = shapes[c][1];
          const int ppt = shapes[c][0], reps = 20;
          t[c] = 0.0f;
          for (int round = 0; round < 3; ++round) {
            const int nb = residual_blocks(ra.npix, ppt);
            auto pass = [&]() {
              return launch_residual(ra, ppt, st) == hipSuccess &&
                     launch_reduce(s->partials, nb, s->red_out, st) == hipSuccess;
            };
            for (int r = 0; r < 2; ++r)
              if (!pass()) return DSLAM_ERR_DEVICE;
            if (hipEventRecord(e0, st) != hipSuccess) return DSLAM_ERR_DEVICE;
            for (int r = 0; r < reps; ++r)
              if (!pass()) return DSLAM_ERR_DEVICE;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
              return DSLAM_ERR_DEVICE;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return DSLAM_ERR_DEVICE;
            const float us = ms * 1000.0f / reps;
            if (round == 0 || us < t[c]) t[c] = us;
          }
        }
        float fastest = t[0];
        for (int c = 1; c < 6; ++c) fastest = std::min(fastest, t[c]);
        int pick = 0;
        while (t[pick] > 1.02f * fastest) ++pick;
        dslam_tune_entry best{cam.width, cam.height, l, jac_format, shapes[pick][0], t[pick], shapes[pick][1]};
        found.push_back(best);
      }
      return DSLAM_OK;
    };
    rc = run();
    (void)hipStreamSynchronize(st);
    (void)hipFree(img);
    (void)dslam_session_close(s);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DSLAM_OK) return rc;
  {
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const dslam_tune_entry& f : found) {
      bool replaced = false;
      for (dslam_tune_entry& e : ctx->tuned)
        if (e.width == f.width && e.height == f.height && e.level == f.level && e.jac_format == f.jac_format) {
          e = f;
          replaced = true;
        }
      if (!replaced) ctx->tuned.push_back(f);
    }
  }
  int k = 0;
  for (; k < (int)found.size() && k < max_out; ++k) out[k] = found[k];
  if (n_out) *n_out = k;
  return DSLAM_OK;
}

static void drop_graphs(dslam_session* s) {
  for (int l = 0; l < DSLAM_MAX_LEVELS; ++l)
    if (s->graph[l]) {
      (void)hipGraphExecDestroy(s->graph[l]);
      s->graph[l] = nullptr;
    }
}

dslam_status dslam_session_close(dslam_session* s) {
  if (!s) return DSLAM_ERR_INVALID;
  if (s->server_refs.load() > 0) return DSLAM_ERR_BUSY;
  (void)hipSetDevice(s->ctx->device);
  if (s->enqueued) (void)hipEventSynchronize(session_done(s));
  drop_graphs(s);
  if (s->capture) (void)hipStreamDestroy(s->capture);
  (void)hipFree(s->arena);
  (void)hipHostFree(s->h_result);
  s->ctx->used.fetch_sub(s->bytes);
  delete s;
  return DSLAM_OK;
}

// One pyramid launch of the session's CURRENT or MODEL planes.
static PyrArgs pyr_args(const dslam_session* s, int which, const float* depth, const uint8_t* inten, int pitch) {
  PyrArgs a;
  a.src = PyrSrc{depth, inten, pitch};
  const LevelPtrs* P = which == DSLAM_PYR_MODEL ? s->model : s->cur;
  for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) a.L[l] = P[l < s->levels ? l : 0];
  a.levels = s->levels;
  a.with_grad = which == DSLAM_PYR_MODEL;
  return a;
}

dslam_status dslam_build_pyramid(dslam_session* s, int32_t which, const float* depth_dev,
                                 const uint8_t* intensity_dev, int32_t pitch_elems, const double T_W_ref[16],
                                 void* stream) {
  if (!s || !depth_dev || !intensity_dev || pitch_elems < s->cam.width) return DSLAM_ERR_INVALID;
  if (which != DSLAM_PYR_CURRENT && which != DSLAM_PYR_MODEL) return DSLAM_ERR_INVALID;
  if (which == DSLAM_PYR_MODEL) {
    if (!T_W_ref) return DSLAM_ERR_INVALID;
    for (int i = 0; i < 16; ++i)
      if (!std::isfinite(T_W_ref[i])) return DSLAM_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(order_after_session(s, st));
  HIP_OK(launch_pyramid(pyr_args(s, which, depth_dev, intensity_dev, pitch_elems), st));
  HIP_OK(mark_session(s, st));
  if (which == DSLAM_PYR_CURRENT) s->cur_normals_ok = true;
  if (which == DSLAM_PYR_MODEL) {
    std::memcpy(s->T_WM, T_W_ref, sizeof(s->T_WM));
    s->have_model = true;
  }
  return DSLAM_OK;
}

dslam_status dslam_preintegrate_imu(const dslam_imu_sample* samples, int32_t n, double t0, double t1,
                                    const double bg[3], const double ba[3], const dslam_imu_params* p,
                                    dslam_preint* out) {
  if (!samples || !bg || !ba || !p || !out) return DSLAM_ERR_INVALID;
  PreintWork* w = new (std::nothrow) PreintWork;
  if (!w) return DSLAM_ERR_NO_CAPACITY;
  dslam_preint r;
  int st = preintegrate(Par{0, 1}, samples, n, t0, t1, bg, ba, p->sigma_g, p->sigma_a, w, &r);
  delete w;
  if (st != DSLAM_OK) return (dslam_status)st;
  *out = r;
  return DSLAM_OK;
}

dslam_status dslam_solve_step(const double raw[58], const double T_WM[16], const dslam_preint* pre,
                              const dslam_imu_params* ip, const dslam_track_params* tp, const dslam_prior* prior,
                              dslam_frame_state* x0, dslam_frame_state* x1, double q_IW[4], double dz_out[33],
                              dslam_prior* marg_out) {
  if (!raw || !T_WM || !ip || !tp || !x0 || !x1 || !q_IW) return DSLAM_ERR_INVALID;
  if (tp->mode != DSLAM_MODE_RGBD && tp->mode != DSLAM_MODE_RGBDI && tp->mode != DSLAM_MODE_GYRO)
    return DSLAM_ERR_INVALID;
  if (tp->mode != DSLAM_MODE_RGBD && (!pre || !prior)) return DSLAM_ERR_INVALID;
  if (!state_ok(x0) || !state_ok(x1) || !quat_ok(q_IW)) return DSLAM_ERR_INVALID;
  SolveWork* w = new (std::nothrow) SolveWork;
  if (!w) return DSLAM_ERR_NO_CAPACITY;
  SolveParams sp;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) sp.R_WM[3 * r + c] = T_WM[4 * r + c];
    sp.t_WM[r] = T_WM[4 * r + 3];
  }
  sp.imu = imu_params_d(*ip);
  sp.mode = tp->mode;
  sp.marginalise = marg_out != nullptr;
  dslam_frame_state a = *x0, b = *x1;
  double q[4] = {q_IW[0], q_IW[1], q_IW[2], q_IW[3]};
  dslam_prior m;
  dslam_preint dummy_pre;
  dslam_prior dummy_prior;
  if (!pre) { std::memset(&dummy_pre, 0, sizeof(dummy_pre)); pre = &dummy_pre; }
  if (!prior) { std::memset(&dummy_prior, 0, sizeof(dummy_prior)); prior = &dummy_prior; }
  int st = solve_step(Par{0, 1}, w, raw, sp, pre, prior, &a, &b, q, &m);
  if (st == DSLAM_OK) {
    *x0 = a;
    *x1 = b;
    for (int i = 0; i < 4; ++i) q_IW[i] = q[i];
    if (dz_out) {
      int n = tp->mode == DSLAM_MODE_RGBD ? 6 : NZ;
      for (int i = 0; i < NZ; ++i) dz_out[i] = i < n ? w->dz[i] : 0.0;
    }
    if (marg_out && tp->mode != DSLAM_MODE_RGBD) *marg_out = m;
  }
  delete w;
  return (dslam_status)st;
}

// STEP_* flags of iteration `it` of level l.
static int step_flags(const dslam_track_params& tp, int l, int it) {
  const int fl = last_level_of(tp);
  int f = 0;
  if (l == fl && it == 0) f |= STEP_FIRST;
  if (l == fl && it == tp.iters[l] - 1) f |= STEP_LAST;
  return f;
}

// One level's Gauss-Newton iterations (each: the residual pass, then the
// step).  With sp == nullptr (graph capture) the step reads the frame's solve
// parameters from device memory, written by the frame's first launch: every
// argument of these launches is then fixed for the session (device pointers,
// sizes, the level's schedule), so the same launches serve every frame.
static hipError_t enqueue_level(dslam_session* s, int l, const SolveParams* sp, hipStream_t st) {
  const ResidualArgs ra = residual_args(s, l, s->sd->xf, nullptr);
  const int nb = residual_blocks(ra.npix, s->ppt[l]);
  for (int it = 0; it < s->tp.iters[l]; ++it) {
    hipError_t e = launch_residual(ra, s->ppt[l], st);
    if (e != hipSuccess) return e;
    const int flags = step_flags(s->tp, l, it);
    if (sp) {
      SolveArgs sa;
      sa.sp = *sp;
      sa.level = l;
      sa.flags = flags;
      sa.nblocks = nb;
      e = launch_solve(s->sd, s->partials, sa, st);
    } else {
      e = launch_solve_graph(s->sd, s->partials, s->sp_dev, l, flags, nb, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Captures, once per session, each level's launches into a graph on a private
// stream (see enqueue_level).
static dslam_status capture_graphs(dslam_session* s) {
  bool complete = true;
  for (int l = 0; l < s->levels; ++l) complete = complete && (s->tp.iters[l] <= 0 || s->graph[l]);
  if (complete) return DSLAM_OK;
  if (!s->capture) HIP_OK(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking));
  for (int l = 0; l < s->levels; ++l) {
    if (s->tp.iters[l] <= 0 || s->graph[l]) continue;
    HIP_OK(hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_level(s, l, nullptr, s->capture);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s->capture, &g);
    if (e == hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&s->graph[l], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      s->graph[l] = nullptr;
      drop_graphs(s);
      return DSLAM_ERR_DEVICE;
    }
  }
  return DSLAM_OK;
}

// Enqueues one frame; with a model view (mdepth != nullptr) its pyramid is
// built in the same launch as the current frame's and the frame's
// initialisation.  Arguments validated by the callers.
static dslam_status track_enqueue(dslam_session* s, const float* depth, const uint8_t* inten, int32_t pitch,
                                  const float* mdepth, const uint8_t* minten, int32_t mpitch, const double* T_WM,
                                  const ImuBatch& batch, dslam_track_result* out, hipStream_t st) {
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (mdepth) std::memcpy(s->T_WM, T_WM, sizeof(s->T_WM));
  const SolveParams sp = solve_params(s);
  const FrameArgs fa = frame_args(s, sp);
  const PyrArgs cur = pyr_args(s, DSLAM_PYR_CURRENT, depth, inten, pitch);
  s->cur_normals_ok = true;  // the frame's first launch builds the current pyramid with its normals
  PyrArgs model;
  if (mdepth) model = pyr_args(s, DSLAM_PYR_MODEL, mdepth, minten, mpitch);
  if (s->use_graphs) {
    dslam_status gs = capture_graphs(s);
    if (gs != DSLAM_OK) return gs;
  }
  HIP_OK(order_after_session(s, st));
  HIP_OK(launch_frame_init_pyramid(s->sd, batch, fa, sp, cur, mdepth ? &model : nullptr, s->sp_dev, st));
  if (mdepth) s->have_model = true;
  for (int l = s->levels - 1; l >= 0; --l) {
    if (s->tp.iters[l] <= 0) continue;
    if (s->use_graphs) HIP_OK(hipGraphLaunch(s->graph[l], st));
    else HIP_OK(enqueue_level(s, l, &sp, st));
  }
  if (sp.imu_fallback) {  // the inertial-only re-estimate of a lost frame (returns at once otherwise)
    const int fl = last_level_of(s->tp);
    if (s->use_graphs) {
      HIP_OK(launch_solve_graph(s->sd, s->partials, s->sp_dev, fl, STEP_LAST | STEP_INERTIAL, 0, st));
    } else {
      SolveArgs sa;
      sa.sp = sp;
      sa.level = fl;
      sa.flags = STEP_LAST | STEP_INERTIAL;
      sa.nblocks = 0;
      HIP_OK(launch_solve(s->sd, s->partials, sa, st));
    }
  }
  if (out) HIP_OK(hipMemcpyAsync(out, &s->sd->result, sizeof(dslam_track_result), hipMemcpyDeviceToHost, st));
  HIP_OK(mark_session(s, st));
  return DSLAM_OK;
}

dslam_status dslam_session_set_graphs(dslam_session* s, int32_t enable) {
  if (!s || (enable != 0 && enable != 1)) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  s->use_graphs = enable == 1;
  return DSLAM_OK;
}

dslam_status dslam_track_frame(dslam_session* s, const dslam_frame_input* f, dslam_track_result* out, void* stream) {
  if (!s || !f || !f->depth || !f->intensity || f->pitch < s->cam.width) return DSLAM_ERR_INVALID;
  const bool model = f->model_depth != nullptr;
  if (model && (!f->model_intensity || f->model_pitch < s->cam.width || !finite16(f->T_WM))) return DSLAM_ERR_INVALID;
  ImuBatch batch;
  dslam_status sti = pack_imu(s, f->imu, f->n_imu, f->t0, f->t1, &batch);
  if (sti != DSLAM_OK) return sti;
  if (last_level_of(s->tp) < 0) return DSLAM_ERR_INVALID;
  if (!model && !s->have_model) return DSLAM_ERR_NOT_READY;
  return track_enqueue(s, f->depth, f->intensity, f->pitch, model ? f->model_depth : nullptr,
                       model ? f->model_intensity : nullptr, f->model_pitch, f->T_WM, batch, out, (hipStream_t)stream);
}

dslam_status dslam_track_frame_sync(dslam_session* s, const dslam_frame_input* f, dslam_track_result* out,
                                    void* stream) {
  if (!out) return DSLAM_ERR_INVALID;
  // the result is copied in stream order into the session's pinned mirror, and
  // the frame's end is polled, so nothing is left to do between the frame's
  // end on the device and the return (no sleep, no separate copy)
  dslam_status st = dslam_track_frame(s, f, s ? s->h_result : nullptr, stream);
  if (st != DSLAM_OK) return st;
  hipError_t e;
  while ((e = hipEventQuery(session_done(s))) == hipErrorNotReady) {
  }
  if (e != hipSuccess) return DSLAM_ERR_DEVICE;
  *out = *s->h_result;
  return DSLAM_OK;
}

static void drop_batch_graphs(dslam_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

dslam_status dslam_batch_create(dslam_context* ctx, int32_t max_sessions, dslam_batch** out) {
  if (!ctx || !out || max_sessions < 1 || max_sessions > MAX_BATCH) return DSLAM_ERR_INVALID;
  const size_t vis = align256(sizeof(SlotVis) * max_sessions);
  const size_t sol = align256(sizeof(SlotSolve) * max_sessions);
  const size_t res = align256(sizeof(dslam_track_result) * max_sessions);
  const uint64_t bytes = vis + sol + res;
  uint64_t prev = ctx->used.fetch_add(bytes);
  if (ctx->budget && prev + bytes > ctx->budget) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  dslam_batch* b = new (std::nothrow) dslam_batch;
  if (!b) {
    ctx->used.fetch_sub(bytes);
    return DSLAM_ERR_NO_CAPACITY;
  }
  b->ctx = ctx;
  b->max_n = max_sessions;
  b->bytes = bytes;
  b->dev = nullptr;
  b->host = nullptr;
  b->pending = false;
  b->n = 0;
  b->tile_order = 1;
  auto fail = [&](dslam_status st) {
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    ctx->used.fetch_sub(bytes);
    delete b;
    return st;
  };
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  if (hipMalloc(&b->dev, bytes) != hipSuccess) {
    b->dev = nullptr;
    return fail(DSLAM_ERR_NO_CAPACITY);
  }
  if (hipHostMalloc(&b->host, bytes, hipHostMallocDefault) != hipSuccess) {
    b->host = nullptr;
    return fail(DSLAM_ERR_NO_CAPACITY);
  }
  char* d = (char*)b->dev;
  char* h = (char*)b->host;
  b->d_vis = (SlotVis*)d;
  b->d_solve = (SlotSolve*)(d + vis);
  b->d_res = (dslam_track_result*)(d + vis + sol);
  b->h_vis = (SlotVis*)h;
  b->h_solve = (SlotSolve*)(h + vis);
  b->h_res = (dslam_track_result*)(h + vis + sol);
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) return fail(DSLAM_ERR_DEVICE);
  *out = b;
  return DSLAM_OK;
}

dslam_status dslam_batch_destroy(dslam_batch* b) {
  if (!b) return DSLAM_ERR_INVALID;
  (void)hipSetDevice(b->ctx->device);
  if (b->pending) (void)hipEventSynchronize(b->done);
  drop_batch_graphs(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  (void)hipEventDestroy(b->done);
  (void)hipFree(b->dev);
  (void)hipHostFree(b->host);
  b->ctx->used.fetch_sub(b->bytes);
  delete b;
  return DSLAM_OK;
}

}  // extern "C"

namespace {

// Host and device memory of one batched step: staging of the slot records
// (pinned or static host memory) and their device copies, plus the results.
struct BatchMem {
  SlotVis* h_vis;
  SlotSolve* h_solve;
  dslam_track_result* h_res;
  SlotVis* d_vis;
  SlotSolve* d_solve;
  dslam_track_result* d_res;
};

constexpr int kMaxBatchGraphs = 32;  // graphs kept per batch object

// Sessions of one class share a batched launch's work split: same image size
// and the same launch shape (pixels per thread) at every level.
bool same_class(const dslam_session* a, const dslam_session* b) {
  if (a->cam.width != b->cam.width || a->cam.height != b->cam.height) return false;
  for (int l = 0; l < a->levels; ++l)
    if (a->ppt[l] != b->ppt[l]) return false;
  return true;
}

// Slot order of the classes: larger images first, then wider, then by launch shape.
bool class_before(const dslam_session* a, const dslam_session* b) {
  const int pa = a->cam.width * a->cam.height, pb = b->cam.width * b->cam.height;
  if (pa != pb) return pa > pb;
  if (a->cam.width != b->cam.width) return a->cam.width > b->cam.width;
  for (int l = 0; l < a->levels; ++l)
    if (a->ppt[l] != b->ppt[l]) return a->ppt[l] < b->ppt[l];
  return false;
}

// The launches of one batched step: everything its kernels take besides the
// staging memory (whose device pointers are fixed per batch object), so that
// equal plans on one batch object issue identical launches.
struct BatchPlan {
  int n, levels, jac;
  int iters[DSLAM_MAX_LEVELS];
  dslam_track_params tp;  // the schedule (levels, iterations) of the step flags
  BatchGrid pyr_grid;
  int fallback;  // some session re-estimates a lost frame without its visual terms
  int max_ppt[DSLAM_MAX_LEVELS];
  int banded[DSLAM_MAX_LEVELS];  // tile order of the level's batched residual pass
  BatchGrid res_grid[DSLAM_MAX_LEVELS];
  uint64_t pixels[DSLAM_MAX_LEVELS];
};

void push_grid(std::vector<int32_t>* k, const BatchGrid& g) {
  k->push_back(g.nclass);
  for (int c = 0; c <= g.nclass; ++c) k->push_back(g.first_block[c]);
  for (int c = 0; c < g.nclass; ++c) {
    k->push_back(g.blocks_per_slot[c]);
    k->push_back(g.first_slot[c]);
  }
}

// Everything a batched step's launches depend on, as a key of its graph.
std::vector<int32_t> plan_key(const BatchPlan& p) {
  std::vector<int32_t> k{p.n, p.levels, p.jac, p.fallback};
  for (int l = 0; l < p.levels; ++l) k.push_back(p.iters[l]);
  push_grid(&k, p.pyr_grid);
  for (int l = 0; l < p.levels; ++l) {
    k.push_back(p.max_ppt[l]);
    k.push_back(p.banded[l]);
    push_grid(&k, p.res_grid[l]);
  }
  return k;
}

// Validates a batched step's arguments without touching any state.
dslam_status batch_validate(const dslam_context* ctx, int32_t n, dslam_session* const* sessions,
                            const dslam_frame_input* frames) {
  const dslam_session* s0 = sessions[0];
  if (!s0) return DSLAM_ERR_INVALID;
  for (int i = 0; i < n; ++i) {
    const dslam_session* s = sessions[i];
    const dslam_frame_input& f = frames[i];
    if (!s || s->ctx != ctx || s->levels != s0->levels || s->tp.jac_format != s0->tp.jac_format)
      return DSLAM_ERR_INVALID;
    for (int l = 0; l < s->levels; ++l)
      if (s->tp.iters[l] != s0->tp.iters[l]) return DSLAM_ERR_INVALID;
    for (int j = 0; j < i; ++j)
      if (sessions[j] == s) return DSLAM_ERR_INVALID;
    if (!f.depth || !f.intensity || f.pitch < s->cam.width) return DSLAM_ERR_INVALID;
    if (!f.model_depth || !f.model_intensity || f.model_pitch < s->cam.width) return DSLAM_ERR_INVALID;
    if (!finite16(f.T_WM)) return DSLAM_ERR_INVALID;
    ImuBatch probe;
    const dslam_status sti = pack_imu(s, f.imu, f.n_imu, f.t0, f.t1, &probe);
    if (sti != DSLAM_OK) return sti;
  }
  if (last_level_of(s0->tp) < 0) return DSLAM_ERR_INVALID;
  int nres = 0;
  for (int i = 0; i < n; ++i) {
    bool known = false;
    for (int j = 0; j < i; ++j) known = known || same_class(sessions[j], sessions[i]);
    nres += known ? 0 : 1;
  }
  return nres > MAX_CLASSES ? DSLAM_ERR_INVALID : DSLAM_OK;
}

// Stages one validated batched step: the slot order (sessions grouped by
// class, larger images first; order[k] = caller index of slot k), the slot
// records and their copy to the device on `st`, and the plan of its launches.
dslam_status batch_stage(const BatchMem& m, int32_t n, dslam_session* const* sessions,
                         const dslam_frame_input* frames, int tile_order, hipStream_t st, int* order,
                         BatchPlan* plan, hipEvent_t start = nullptr) {
  const dslam_session* s0 = sessions[0];
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order, order + n, [&](int a, int c) { return class_before(sessions[a], sessions[c]); });
  int nclass = 0, cls_first[MAX_BATCH + 1];
  for (int k = 0; k < n; ++k)
    if (k == 0 || !same_class(sessions[order[k]], sessions[order[k - 1]])) cls_first[nclass++] = k;
  if (nclass > MAX_CLASSES) return DSLAM_ERR_INVALID;
  cls_first[nclass] = n;
  ImuBatch imu;
  for (int k = 0; k < n; ++k) {
    dslam_session* s = sessions[order[k]];
    const dslam_frame_input& f = frames[order[k]];
    (void)pack_imu(s, f.imu, f.n_imu, f.t0, f.t1, &imu);
    std::memcpy(s->T_WM, f.T_WM, sizeof(s->T_WM));
    SlotVis& v = m.h_vis[k];
    SlotSolve& o = m.h_solve[k];
    for (int l = 0; l < s->levels; ++l) {
      v.res[l] = residual_args(s, l, s->sd->xf, nullptr);
      v.cur[l] = s->cur[l];
      v.model[l] = s->model[l];
      v.ppt[l] = s->ppt[l];
      o.nblocks[l] = residual_blocks(v.res[l].npix, s->ppt[l]);
    }
    v.depth = f.depth;
    v.inten = f.intensity;
    v.pitch = f.pitch;
    v.mdepth = f.model_depth;
    v.minten = f.model_intensity;
    v.mpitch = f.model_pitch;
    // the current frame's normals are read only through the normal gate;
    // otherwise the step leaves them out (ensure_cur_normals fills them on demand)
    v.cur_normals = s->tp.icp_cos >= -1.0 ? 1 : 0;
    s->cur_normals_ok = v.cur_normals != 0;
    o.sd = s->sd;
    o.partials = s->partials;
    o.imu = imu;
    o.sp = solve_params(s);
    o.fa = frame_args(s, o.sp);
  }
  // the staging copies write only this step's staging memory: they go ahead of
  // the waits for the sessions' earlier work (which may still be running on
  // another stream), and the step's launches follow the waits
  HIP_OK(hipMemcpyAsync(m.d_vis, m.h_vis, sizeof(SlotVis) * n, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(m.d_solve, m.h_solve, sizeof(SlotSolve) * n, hipMemcpyHostToDevice, st));
  // one wait per distinct completion event: the sessions of an earlier batched
  // step share that step's event
  const DoneEvent* waited[MAX_BATCH];
  int nw = 0;
  for (int k = 0; k < n; ++k) {
    dslam_session* s = sessions[k];
    if (!s->enqueued || s->last_stream == st) continue;
    bool dup = false;
    for (int w = 0; w < nw; ++w) dup = dup || waited[w] == s->done.get();
    if (dup) continue;
    HIP_OK(hipStreamWaitEvent(st, s->done->ev, 0));
    waited[nw++] = s->done.get();
  }
  if (start) HIP_OK(hipEventRecord(start, st));
  // work split of each launch: one class per resolution and launch shape
  auto grid = [&](auto blocks_of) {
    BatchGrid g;
    g.nclass = nclass;
    int blk = 0;
    for (int c = 0; c < nclass; ++c) {
      const int per = blocks_of(sessions[order[cls_first[c]]]);
      g.first_block[c] = blk;
      g.blocks_per_slot[c] = per;
      g.first_slot[c] = cls_first[c];
      blk += per * (cls_first[c + 1] - cls_first[c]);
    }
    g.first_block[nclass] = blk;
    return g;
  };
  plan->n = n;
  plan->levels = s0->levels;
  plan->jac = s0->tp.jac_format;
  plan->tp = s0->tp;
  plan->fallback = 0;
  for (int k = 0; k < n; ++k) plan->fallback |= m.h_solve[k].sp.imu_fallback;
  plan->pyr_grid = grid([&](const dslam_session* s) { return 2 * PyrTileBatch::tiles(s->cam.width, s->cam.height); });
  for (int l = 0; l < s0->levels; ++l) {
    int max_ppt = 1;
    uint64_t px = 0;
    for (int k = 0; k < n; ++k) {
      max_ppt = std::max(max_ppt, sessions[k]->ppt[l]);
      px += (uint64_t)sessions[k]->cur[l].W * sessions[k]->cur[l].H;
    }
    plan->iters[l] = s0->tp.iters[l];
    plan->res_grid[l] =
        grid([&](const dslam_session* s) { return residual_blocks(s->cur[l].W * s->cur[l].H, s->ppt[l]); });
    plan->max_ppt[l] = max_ppt;
    // tile order < 0: the first class's (it holds the largest images)
    plan->banded[l] = tile_order < 0 ? sessions[order[0]]->banded[l] : tile_order;
    plan->pixels[l] = px;
  }
  return DSLAM_OK;
}

// Every kernel of one staged batched step (Section IV for each session, with
// shared launches): both pyramids of every session, the frames'
// initialisation, each level's Gauss-Newton iterations and the gathering of
// the results.  Their arguments are the plan and the fixed staging pointers,
// so the same launches can be captured once and replayed.
hipError_t batch_launches(const BatchMem& m, const BatchPlan& p, hipStream_t st) {
  hipError_t e = launch_pyramid_batch(m.d_vis, p.levels, p.pyr_grid, st);
  if (e == hipSuccess) e = launch_frame_init_batch(m.d_solve, p.n, st);
  for (int l = p.levels - 1; l >= 0 && e == hipSuccess; --l)
    for (int it = 0; it < p.iters[l] && e == hipSuccess; ++it) {
      e = launch_residual_batch(m.d_vis, p.res_grid[l], l, p.max_ppt[l], p.jac, p.banded[l], st);
      if (e == hipSuccess) e = launch_solve_batch(m.d_solve, p.n, l, step_flags(p.tp, l, it), st);
    }
  if (e == hipSuccess && p.fallback)
    e = launch_solve_batch(m.d_solve, p.n, last_level_of(p.tp), STEP_LAST | STEP_INERTIAL, st);
  if (e == hipSuccess) e = launch_gather_results(m.d_solve, p.n, m.d_res, st);
  return e;
}

// The results' copy to the host staging (m.h_res, slot order) and the
// sessions' completion marks, after the step's launches on `st`: one record of
// `shared` for all of them, or (null) a record of each session's own event.
dslam_status batch_finish(const BatchMem& m, int32_t n, dslam_session* const* sessions, const int* order,
                          hipStream_t st, const DoneRef* shared) {
  HIP_OK(hipMemcpyAsync(m.h_res, m.d_res, sizeof(dslam_track_result) * n, hipMemcpyDeviceToHost, st));
  if (shared) HIP_OK(hipEventRecord((*shared)->ev, st));
  for (int k = 0; k < n; ++k) {
    dslam_session* s = sessions[order[k]];
    s->have_model = true;
    if (shared) mark_session_shared(s, st, *shared);
    else HIP_OK(mark_session(s, st));
  }
  return DSLAM_OK;
}

// A completion event for the batch's next step: one that no session holds any
// more (its earlier records are no longer waited for), or a new one.
DoneRef step_done_event(dslam_batch* b, hipError_t* err) {
  *err = hipSuccess;
  for (const DoneRef& d : b->step_done)
    if (d.use_count() == 1) return d;
  DoneRef d = std::make_shared<DoneEvent>();
  *err = hipEventCreateWithFlags(&d->ev, hipEventDisableTiming);
  if (*err != hipSuccess) return nullptr;
  b->step_done.push_back(d);
  return d;
}

// The executable graph of a plan on this batch object: found in the cache or
// captured (on a private stream) and instantiated.  Called with no step of the
// batch in flight.  nullptr with *err set on failure.
hipGraphExec_t batch_graph(dslam_batch* b, const BatchMem& m, const BatchPlan& p, hipError_t* err) {
  std::vector<int32_t> key = plan_key(p);
  for (auto& g : b->graphs)
    if (g.first == key) return g.second;
  *err = hipSuccess;
  if (!b->capture) {
    *err = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (*err != hipSuccess) {
      b->capture = nullptr;
      return nullptr;
    }
  }
  if ((int)b->graphs.size() >= kMaxBatchGraphs) {  // the oldest plan makes room
    (void)hipGraphExecDestroy(b->graphs.front().second);
    b->graphs.erase(b->graphs.begin());
  }
  *err = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
  if (*err != hipSuccess) return nullptr;
  hipError_t e = batch_launches(m, p, b->capture);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->capture, &g);
  if (e == hipSuccess) e = ee;
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  b->graphs.emplace_back(std::move(key), exec);
  return exec;
}

}  // namespace

extern "C" {

dslam_status dslam_batch_track(dslam_batch* b, int32_t n, dslam_session* const* sessions,
                               const dslam_frame_input* frames, void* stream) {
  return batch_track_timed(b, n, sessions, frames, (hipStream_t)stream, nullptr);
}

}  // extern "C"

dslam_status batch_track_timed(dslam_batch* b, int32_t n, dslam_session* const* sessions,
                               const dslam_frame_input* frames, hipStream_t st, hipEvent_t start) {
  if (!b || !sessions || !frames || n < 1 || n > b->max_n) return DSLAM_ERR_INVALID;
  const dslam_status v = batch_validate(b->ctx, n, sessions, frames);
  if (v != DSLAM_OK) return v;
  HIP_OK(hipSetDevice(b->ctx->device));
  if (b->pending) HIP_OK(hipEventSynchronize(b->done));  // staging memory is reused
  b->pending = false;
  const BatchMem m{b->h_vis, b->h_solve, b->h_res, b->d_vis, b->d_solve, b->d_res};
  BatchPlan plan;
  const dslam_status e = batch_stage(m, n, sessions, frames, b->tile_order, st, b->order, &plan, start);
  if (e != DSLAM_OK) return e;
  if (b->use_graphs) {
    hipError_t ge = hipSuccess;
    hipGraphExec_t exec = batch_graph(b, m, plan, &ge);
    if (!exec) return DSLAM_ERR_DEVICE;
    HIP_OK(hipGraphLaunch(exec, st));
  } else {
    HIP_OK(batch_launches(m, plan, st));
  }
  hipError_t de = hipSuccess;
  const DoneRef sd = step_done_event(b, &de);
  HIP_OK(de);
  const dslam_status f = batch_finish(m, n, sessions, b->order, st, &sd);
  if (f != DSLAM_OK) return f;
  HIP_OK(hipEventRecord(b->done, st));
  b->levels = plan.levels;
  b->jac = plan.jac;
  for (int l = 0; l < plan.levels; ++l) {
    b->max_ppt[l] = plan.max_ppt[l];
    b->banded[l] = plan.banded[l];
    b->res_grid[l] = plan.res_grid[l];
    b->pixels[l] = plan.pixels[l];
  }
  b->n = n;
  b->pending = true;
  return DSLAM_OK;
}

extern "C" {

dslam_status dslam_batch_set_tile_order(dslam_batch* b, int32_t order) {
  if (!b || order < -1 || order > 1) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(b->ctx->device));
  if (b->pending) HIP_OK(hipEventSynchronize(b->done));
  b->tile_order = order;
  if (order >= 0)  // dslam_batch_profile_residual relaunches the last step's pass in the new order
    for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) b->banded[l] = order;
  return DSLAM_OK;
}

dslam_status dslam_batch_set_graphs(dslam_batch* b, int32_t enable) {
  if (!b || (enable != 0 && enable != 1)) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(b->ctx->device));
  if (b->pending) HIP_OK(hipEventSynchronize(b->done));
  if (!enable) drop_batch_graphs(b);
  b->use_graphs = enable == 1;
  return DSLAM_OK;
}

dslam_status dslam_batch_track_noalloc(int32_t n, dslam_session* const* sessions, const dslam_frame_input* frames,
                                       dslam_track_result* results, void* stream) {
  if (!sessions || !frames || !results || n < 1 || !sessions[0]) return DSLAM_ERR_INVALID;
  if (n > DSLAM_MAX_BATCH) return DSLAM_ERR_INVALID;  // the scratch holds DSLAM_MAX_BATCH slots
  dslam_context* ctx = sessions[0]->ctx;
  const dslam_status v = batch_validate(ctx, n, sessions, frames);
  if (v != DSLAM_OK) return v;
  unsigned char* base = (unsigned char*)scratch_ptr(ctx->device);
  if (!base) return DSLAM_ERR_DEVICE;
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // every slot the step reads is written first: nothing in the scratch needs clearing
  const BatchMem m{g_hvis, g_hsolve, g_hres, (SlotVis*)base, (SlotSolve*)(base + kScratchVis),
                   (dslam_track_result*)(base + kScratchVis + kScratchSolve)};
  int order[MAX_BATCH];
  BatchPlan plan;
  const dslam_status e = batch_stage(m, n, sessions, frames, 1, st, order, &plan);
  if (e != DSLAM_OK) return e;
  HIP_OK(batch_launches(m, plan, st));
  const dslam_status f = batch_finish(m, n, sessions, order, st, nullptr);
  if (f != DSLAM_OK) return f;
  HIP_OK(hipStreamSynchronize(st));
  for (int k = 0; k < n; ++k) results[order[k]] = g_hres[k];
  return DSLAM_OK;
}

dslam_status dslam_batch_profile_residual(dslam_batch* b, int32_t level, int32_t reps, void* stream,
                                          uint64_t* pixels) {
  if (!b || !b->pending || level < 0 || level >= b->levels || reps < 1 || reps > 100000) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(b->ctx->device));
  HIP_OK(hipEventSynchronize(b->done));
  hipStream_t st = (hipStream_t)stream;
  for (int r = 0; r < reps; ++r)
    HIP_OK(launch_residual_batch(b->d_vis, b->res_grid[level], level, b->max_ppt[level], b->jac, b->banded[level],
                                 st));
  if (pixels) *pixels = b->pixels[level];
  return DSLAM_OK;
}

dslam_status dslam_batch_results(dslam_batch* b, dslam_track_result* out) {
  if (!b || !out || !b->pending) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(b->ctx->device));
  HIP_OK(hipEventSynchronize(b->done));
  for (int k = 0; k < b->n; ++k) out[b->order[k]] = b->h_res[k];
  return DSLAM_OK;
}

dslam_status dslam_session_result(dslam_session* s, dslam_track_result* out) {
  if (!s || !out) return DSLAM_ERR_INVALID;
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  HIP_OK(hipMemcpy(out, &s->sd->result, sizeof(dslam_track_result), hipMemcpyDeviceToHost));
  return DSLAM_OK;
}

dslam_status dslam_linearize(dslam_session* s, int32_t level, const float Ra[9], const float ta[3],
                             const float Rb[9], const float tb[3], const dslam_frame_state* x0,
                             const dslam_frame_state* x1, uint8_t* mask_dev, dslam_linear_system* out,
                             void* stream) {
  if (!s || !Ra || !ta || !Rb || !tb || !state_ok(x0) || !state_ok(x1) || !out) return DSLAM_ERR_INVALID;
  if (level < 0 || level >= s->levels) return DSLAM_ERR_INVALID;
  if (!s->have_model) return DSLAM_ERR_NOT_READY;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(order_after_session(s, st));
  float xf[24];
  for (int i = 0; i < 9; ++i) { xf[i] = Ra[i]; xf[12 + i] = Rb[i]; }
  for (int i = 0; i < 3; ++i) { xf[9 + i] = ta[i]; xf[21 + i] = tb[i]; }
  HIP_OK(hipMemcpyAsync(s->xf_scratch, xf, sizeof(xf), hipMemcpyHostToDevice, st));
  ResidualArgs ra = residual_args(s, level, s->xf_scratch, mask_dev);
  HIP_OK(launch_residual(ra, s->ppt[level], st));
  HIP_OK(launch_reduce(s->partials, residual_blocks(ra.npix, s->ppt[level]), s->red_out, st));
  double raw[64];
  HIP_OK(hipMemcpyAsync(raw, s->red_out, 58 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(mark_session(s, st));
  HIP_OK(hipStreamSynchronize(st));
  SolveParams sp = solve_params(s);
  dslam_linear_system r;
  lift_visual(raw, sp.R_WM, *x0, *x1, r.H_icp, r.b_icp, r.H_rgb, r.b_rgb);
  r.cost_icp = raw[27];
  r.cost_rgb = raw[29 + 27];
  r.n_icp = (int64_t)raw[28];
  r.n_rgb = (int64_t)raw[57];
  for (int i = 0; i < 58; ++i) r.raw[i] = raw[i];
  *out = r;
  return DSLAM_OK;
}

dslam_status dslam_profile_residual(dslam_session* s, int32_t level, int32_t reps, void* stream) {
  if (!s || level < 0 || level >= s->levels || reps < 1 || reps > 100000) return DSLAM_ERR_INVALID;
  if (!s->have_model) return DSLAM_ERR_NOT_READY;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(order_after_session(s, st));
  ResidualArgs ra = residual_args(s, level, s->sd->xf, nullptr);
  for (int r = 0; r < reps; ++r) HIP_OK(launch_residual(ra, s->ppt[level], st));
  HIP_OK(mark_session(s, st));
  return DSLAM_OK;
}

dslam_status dslam_copy_pyramid(dslam_session* s, int32_t which, int32_t level, int32_t channel, float* host_out) {
  if (!s || !host_out || level < 0 || level >= s->levels) return DSLAM_ERR_INVALID;
  if (which != DSLAM_PYR_CURRENT && which != DSLAM_PYR_MODEL) return DSLAM_ERR_INVALID;
  const LevelPtrs& L = which == DSLAM_PYR_MODEL ? s->model[level] : s->cur[level];
  const bool grad = channel == DSLAM_CH_GX || channel == DSLAM_CH_GY;
  if (channel < DSLAM_CH_VX || channel > DSLAM_CH_GY || (grad && which != DSLAM_PYR_MODEL)) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  const size_t n = (size_t)L.W * L.H;
  if (which == DSLAM_PYR_CURRENT && channel >= DSLAM_CH_NX && channel <= DSLAM_CH_NZ && !s->cur_normals_ok) {
    HIP_OK(ensure_cur_normals(s, nullptr));  // the null stream: the copy below waits for it
    HIP_OK(mark_session(s, nullptr));
  }
  if (channel >= DSLAM_CH_NX && channel <= DSLAM_CH_NZ) {
    HIP_OK(hipMemcpy(host_out, L.N[channel - DSLAM_CH_NX], n * sizeof(float), hipMemcpyDeviceToHost));
  } else if (channel >= DSLAM_CH_VX && channel <= DSLAM_CH_VZ) {
    HIP_OK(hipMemcpy(host_out, L.V[channel - DSLAM_CH_VX], n * sizeof(float), hipMemcpyDeviceToHost));
  } else {
    std::vector<uint16_t> tmp(n);
    const void* src = channel == DSLAM_CH_I ? (const void*)L.I : (const void*)L.G[channel - DSLAM_CH_GX];
    HIP_OK(hipMemcpy(tmp.data(), src, n * sizeof(uint16_t), hipMemcpyDeviceToHost));
    for (size_t q = 0; q < n; ++q)
      host_out[q] = channel == DSLAM_CH_I ? (float)tmp[q] / kIntensityScale
                                          : (float)(int16_t)tmp[q] / kGradientScale;
  }
  return DSLAM_OK;
}

// ---- checkpoint / restore ------------------------------------------------
// Blob: CkptHeader, then the device state record (SessionDev), then each
// level's MODEL planes in order (V x3, N x3 float32, I uint16, G x2 int16).
namespace {

constexpr char kCkptMagic[8] = {'D', 'S', 'L', 'A', 'M', 'C', 'K', 'P'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
  char magic[8];
  uint32_t version, header_bytes;
  uint64_t total_bytes, state_bytes, model_bytes;
  uint64_t checksum;  // FNV-1a over the blob with this field zero
  int32_t width, height, levels, mode, jac_format, have_model;
  int32_t iters[DSLAM_MAX_LEVELS];
  int32_t ppt[DSLAM_MAX_LEVELS];
  double fx, fy, cx, cy;
  double icp_dist, icp_cos, sigma_I, depth_k, huber_k, min_inlier_frac, max_cost_rise;
  double T_WM[16];
};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const uint8_t* b = (const uint8_t*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t model_plane_bytes(const dslam_session* s) {
  uint64_t n = 0;
  for (int l = 0; l < s->levels; ++l) n += (uint64_t)s->model[l].W * s->model[l].H * (6 * 4 + 3 * 2);
  return n;
}

uint64_t ckpt_bytes(const dslam_session* s) { return sizeof(CkptHeader) + sizeof(SessionDev) + model_plane_bytes(s); }

// Copies every MODEL plane between the session and host memory (to_host:
// device -> p, else p -> device).
hipError_t copy_model_planes(dslam_session* s, uint8_t* p, bool to_host) {
  for (int l = 0; l < s->levels; ++l) {
    const LevelPtrs& L = s->model[l];
    const size_t n = (size_t)L.W * L.H;
    void* planes[9] = {L.V[0], L.V[1], L.V[2], L.N[0], L.N[1], L.N[2], L.I, L.G[0], L.G[1]};
    for (int k = 0; k < 9; ++k) {
      const size_t bytes = n * (k < 6 ? 4 : 2);
      hipError_t e = to_host ? hipMemcpy(p, planes[k], bytes, hipMemcpyDeviceToHost)
                             : hipMemcpy(planes[k], p, bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) return e;
      p += bytes;
    }
  }
  return hipSuccess;
}

void fill_header(const dslam_session* s, CkptHeader* h) {
  std::memset(h, 0, sizeof(*h));
  std::memcpy(h->magic, kCkptMagic, 8);
  h->version = kCkptVersion;
  h->header_bytes = sizeof(CkptHeader);
  h->total_bytes = ckpt_bytes(s);
  h->state_bytes = sizeof(SessionDev);
  h->model_bytes = model_plane_bytes(s);
  h->width = s->cam.width;
  h->height = s->cam.height;
  h->levels = s->levels;
  h->mode = s->tp.mode;
  h->jac_format = s->tp.jac_format;
  h->have_model = s->have_model ? 1 : 0;
  for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) {
    h->iters[l] = l < s->levels ? s->tp.iters[l] : 0;
    h->ppt[l] = l < s->levels ? s->ppt[l] : 0;
  }
  h->fx = s->cam.fx;
  h->fy = s->cam.fy;
  h->cx = s->cam.cx;
  h->cy = s->cam.cy;
  h->icp_dist = s->tp.icp_dist;
  h->icp_cos = s->tp.icp_cos;
  h->sigma_I = s->tp.sigma_I;
  h->depth_k = s->tp.depth_k;
  h->huber_k = s->tp.huber_k;
  h->min_inlier_frac = s->tp.min_inlier_frac;
  h->max_cost_rise = s->tp.max_cost_rise;
  std::memcpy(h->T_WM, s->T_WM, sizeof(h->T_WM));
}

bool ppt_ok(int p) { return p == 1 || p == 2 || p == 4; }

}  // namespace

dslam_status dslam_session_checkpoint(dslam_session* s, void* buf, uint64_t capacity, uint64_t* size) {
  if (!s || (!buf && !size)) return DSLAM_ERR_INVALID;
  const uint64_t need = ckpt_bytes(s);
  if (!buf) {
    *size = need;
    return DSLAM_OK;
  }
  if (capacity < need) return DSLAM_ERR_INVALID;
  if (s->server_refs.load() > 0) return DSLAM_ERR_BUSY;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  uint8_t* p = (uint8_t*)buf;
  CkptHeader h;
  fill_header(s, &h);
  HIP_OK(hipMemcpy(p + sizeof(CkptHeader), s->sd, sizeof(SessionDev), hipMemcpyDeviceToHost));
  HIP_OK(copy_model_planes(s, p + sizeof(CkptHeader) + sizeof(SessionDev), true));
  std::memcpy(p, &h, sizeof(h));
  h.checksum = fnv1a(14695981039346656037ull, p, need);
  std::memcpy(p, &h, sizeof(h));
  if (size) *size = need;
  return DSLAM_OK;
}

dslam_status dslam_session_restore(dslam_session* s, const void* buf, uint64_t size) {
  if (!s || !buf || size < sizeof(CkptHeader)) return DSLAM_ERR_INVALID;
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion || h.header_bytes != sizeof(CkptHeader))
    return DSLAM_ERR_INVALID;
  if (h.state_bytes != sizeof(SessionDev) || h.model_bytes != model_plane_bytes(s) || h.total_bytes != ckpt_bytes(s) ||
      size < h.total_bytes)
    return DSLAM_ERR_INVALID;
  {  // checksum over the blob with the checksum field zero
    CkptHeader z = h;
    z.checksum = 0;
    uint64_t c = fnv1a(14695981039346656037ull, &z, sizeof(z));
    c = fnv1a(c, (const uint8_t*)buf + sizeof(CkptHeader), h.total_bytes - sizeof(CkptHeader));
    if (c != h.checksum) return DSLAM_ERR_INVALID;
  }
  // the session must match the one the blob was taken from (the tile shape is adopted)
  CkptHeader mine;
  fill_header(s, &mine);
  bool same = h.width == mine.width && h.height == mine.height && h.levels == mine.levels && h.mode == mine.mode &&
              h.jac_format == mine.jac_format && h.fx == mine.fx && h.fy == mine.fy && h.cx == mine.cx &&
              h.cy == mine.cy && h.icp_dist == mine.icp_dist && h.icp_cos == mine.icp_cos &&
              h.sigma_I == mine.sigma_I && h.depth_k == mine.depth_k && h.huber_k == mine.huber_k &&
              h.min_inlier_frac == mine.min_inlier_frac && h.max_cost_rise == mine.max_cost_rise;
  for (int l = 0; l < DSLAM_MAX_LEVELS; ++l) {
    same = same && h.iters[l] == mine.iters[l];
    if (l < s->levels) same = same && ppt_ok(h.ppt[l]);
  }
  if (!same || (h.have_model != 0 && h.have_model != 1)) return DSLAM_ERR_INVALID;
  if (s->server_refs.load() > 0) return DSLAM_ERR_BUSY;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  const uint8_t* p = (const uint8_t*)buf;
  HIP_OK(hipMemcpy(s->sd, p + sizeof(CkptHeader), sizeof(SessionDev), hipMemcpyHostToDevice));
  HIP_OK(copy_model_planes(s, const_cast<uint8_t*>(p) + sizeof(CkptHeader) + sizeof(SessionDev), false));
  std::memcpy(s->T_WM, h.T_WM, sizeof(s->T_WM));
  s->have_model = h.have_model == 1;
  bool retile = false;
  for (int l = 0; l < s->levels; ++l) {
    retile = retile || s->ppt[l] != h.ppt[l];
    s->ppt[l] = h.ppt[l];
  }
  if (retile) drop_graphs(s);  // captured with the old tile shape
  return DSLAM_OK;
}

dslam_status dslam_session_get_state(dslam_session* s, dslam_frame_state* x0, double q_IW[4], dslam_prior* prior,
                                     int32_t* frame_index) {
  if (!s) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  SessionDev d;
  HIP_OK(hipMemcpy(&d, s->sd, sizeof(d), hipMemcpyDeviceToHost));
  if (x0) *x0 = d.x0;
  if (q_IW) for (int i = 0; i < 4; ++i) q_IW[i] = d.qIW[i];
  if (prior) *prior = d.prior;
  if (frame_index) *frame_index = d.frame_index;
  return DSLAM_OK;
}

dslam_status dslam_session_set_state(dslam_session* s, const dslam_frame_state* x0, const double q_IW[4],
                                     const dslam_prior* prior, int32_t frame_index) {
  if (!s || !state_ok(x0) || !q_IW || !quat_ok(q_IW)) return DSLAM_ERR_INVALID;
  if (s->tp.mode != DSLAM_MODE_RGBD && !prior) return DSLAM_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  HIP_OK(hipSetDevice(s->ctx->device));
  if (s->enqueued) HIP_OK(hipEventSynchronize(session_done(s)));
  SessionDev d;
  HIP_OK(hipMemcpy(&d, s->sd, sizeof(d), hipMemcpyDeviceToHost));
  d.x0 = *x0;
  d.x1 = *x0;
  for (int i = 0; i < 4; ++i) d.qIW[i] = q_IW[i];
  if (prior) d.prior = *prior;
  d.frame_index = frame_index;
  d.status = DSLAM_OK;
  HIP_OK(hipMemcpy(s->sd, &d, sizeof(d), hipMemcpyHostToDevice));
  return DSLAM_OK;
}

}  // extern "C"
