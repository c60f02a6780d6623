// Serving loop with continuous batching over the batched tracking step.
//
// Requests (one frame of one session each) wait in one queue in submission
// order.  A poll first retires the batched steps whose completion event has
// fired, then fills every free step slot with a new batch: it scans the queue
// from the front and takes the first request of every session not taken yet,
// as long as the session shares the pyramid schedule of the batch's first
// request and the batch stays within the batched step's limits (sessions,
// distinct resolutions).  Later frames of a session wait for the earlier ones,
// so each session's frames are tracked in order.  A session's next frame may
// join a step while its previous one is still running: the new step is staged
// and launched at once, and on the device its launches wait for the sessions'
// earlier work (one wait per earlier step: the sessions of a step share its
// completion event), so when every session is in every step
// (saturation) the next step starts as soon as the previous one ends, with no
// host round trip in between.  Each slot owns a batch's staging memory, a
// stream and a pair of timing events, so up to pipeline_depth steps are in
// flight.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_set>
#include <vector>

#include "host.h"

namespace {

double steady_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id;
  dslam_session* s;
  dslam_frame_input in;
  dslam_imu_sample imu[DSLAM_MAX_IMU_SAMPLES];
  double submit_s;
};

struct StepSlot {
  dslam_batch* batch = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  bool busy = false;
  double launch_s = 0.0;
  std::vector<Request> reqs;
};

bool same_schedule(const dslam_session* a, const dslam_session* b) {
  if (a->levels != b->levels || a->tp.jac_format != b->tp.jac_format) return false;
  for (int l = 0; l < a->levels; ++l)
    if (a->tp.iters[l] != b->tp.iters[l]) return false;
  return true;
}

bool frame_ok(const dslam_session* s, const dslam_frame_input* f) {
  if (!f->depth || !f->intensity || f->pitch < s->cam.width) return false;
  if (!f->model_depth || !f->model_intensity || f->model_pitch < s->cam.width) return false;
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(f->T_WM[i])) return false;
  if (s->tp.mode == DSLAM_MODE_RGBD) return true;
  if (!f->imu || f->n_imu < 1 || f->n_imu > DSLAM_MAX_IMU_SAMPLES || !(f->t1 > f->t0)) return false;
  if (!(f->imu[0].t <= f->t0)) return false;
  for (int k = 1; k < f->n_imu; ++k)
    if (!(f->imu[k].t > f->imu[k - 1].t)) return false;
  return true;
}

}  // namespace

struct dslam_server {
  dslam_context* ctx;
  dslam_server_params p;
  std::vector<StepSlot> slots;
  std::deque<Request> pending;
  std::deque<dslam_request_done> finished;
  uint64_t next_id = 1;
  int launched = 0;  // requests launched and not yet returned
};

namespace {

void release(dslam_server* sv) {
  for (StepSlot& st : sv->slots) {
    if (st.stream) (void)hipStreamSynchronize(st.stream);
    if (st.batch) (void)dslam_batch_destroy(st.batch);
    if (st.t0) (void)hipEventDestroy(st.t0);
    if (st.t1) (void)hipEventDestroy(st.t1);
    if (st.stream) (void)hipStreamDestroy(st.stream);
    for (Request& r : st.reqs) r.s->server_refs.fetch_sub(1);  // dropped with the server
  }
  for (Request& r : sv->pending) r.s->server_refs.fetch_sub(1);
  for (dslam_request_done& d : sv->finished) d.session->server_refs.fetch_sub(1);
  delete sv;
}

// Moves a finished step's requests to the finished queue.
dslam_status retire(dslam_server* sv, StepSlot& st) {
  const double t = steady_seconds();
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, st.t0, st.t1) != hipSuccess) ms = -1.0f;
  std::vector<dslam_track_result> res(st.reqs.size());
  dslam_status rs = dslam_batch_results(st.batch, res.data());
  for (size_t i = 0; i < st.reqs.size(); ++i) {
    dslam_request_done d;
    std::memset(&d, 0, sizeof(d));
    d.request_id = st.reqs[i].id;
    d.session = st.reqs[i].s;
    d.submit_s = st.reqs[i].submit_s;
    d.launch_s = st.launch_s;
    d.done_s = t;
    d.device_ms = ms;
    d.batch_size = (int32_t)st.reqs.size();
    if (rs == DSLAM_OK) d.result = res[i];
    else d.result.status = rs;
    sv->finished.push_back(d);
  }
  sv->launched -= (int)st.reqs.size();
  st.reqs.clear();
  st.busy = false;
  return rs;
}

// Takes the next batch from the queue (see the file comment).
void take_batch(dslam_server* sv, std::vector<Request>* out) {
  std::deque<Request> rest;
  std::unordered_set<const dslam_session*> seen;
  std::vector<std::pair<int, int>> res;  // distinct resolutions in the batch
  const dslam_session* first = nullptr;
  for (Request& r : sv->pending) {
    bool take = (int)out->size() < sv->p.max_batch && !seen.count(r.s);
    if (take && first && !same_schedule(first, r.s)) take = false;
    if (take) {
      std::pair<int, int> wh{r.s->cam.width, r.s->cam.height};
      bool known = false;
      for (auto& x : res) known = known || x == wh;
      if (!known && (int)res.size() >= DSLAM_MAX_BATCH_RESOLUTIONS) take = false;
      else if (!known) res.push_back(wh);
    }
    seen.insert(r.s);  // later frames of this session wait for this one
    if (take) {
      if (!first) first = r.s;
      out->push_back(r);
    } else {
      rest.push_back(r);
    }
  }
  sv->pending.swap(rest);
}

dslam_status launch(dslam_server* sv, StepSlot& st) {
  st.reqs.clear();
  take_batch(sv, &st.reqs);
  if (st.reqs.empty()) return DSLAM_OK;
  const int n = (int)st.reqs.size();
  std::vector<dslam_session*> ss(n);
  std::vector<dslam_frame_input> fs(n);
  for (int i = 0; i < n; ++i) {
    ss[i] = st.reqs[i].s;
    fs[i] = st.reqs[i].in;
    fs[i].imu = st.reqs[i].imu;
  }
  st.launch_s = steady_seconds();
  dslam_status rc = DSLAM_OK;
  // t0 is recorded once the step's earlier work is waited for: device_ms is the
  // step's own time, not its wait behind the previous step
  rc = batch_track_timed(st.batch, n, ss.data(), fs.data(), st.stream, st.t0);
  if (rc == DSLAM_OK && hipEventRecord(st.t1, st.stream) != hipSuccess) rc = DSLAM_ERR_DEVICE;
  if (rc != DSLAM_OK) {  // the step never ran: return its requests with the error
    const double t = steady_seconds();
    for (Request& r : st.reqs) {
      dslam_request_done d;
      std::memset(&d, 0, sizeof(d));
      d.request_id = r.id;
      d.session = r.s;
      d.submit_s = r.submit_s;
      d.launch_s = st.launch_s;
      d.done_s = t;
      d.device_ms = -1.0f;
      d.batch_size = n;
      d.result.status = rc;
      sv->finished.push_back(d);
    }
    st.reqs.clear();
    return rc;
  }
  sv->launched += n;
  st.busy = true;
  return DSLAM_OK;
}

}  // namespace

extern "C" {

double dslam_server_clock(void) { return steady_seconds(); }

dslam_status dslam_server_create(dslam_context* ctx, const dslam_server_params* p, dslam_server** out) {
  if (!ctx || !p || !out || p->max_batch < 1 || p->max_batch > DSLAM_MAX_BATCH || p->pipeline_depth < 1 ||
      p->pipeline_depth > 8 || (p->use_graphs != 0 && p->use_graphs != 1))
    return DSLAM_ERR_INVALID;
  dslam_server* sv = new (std::nothrow) dslam_server;
  if (!sv) return DSLAM_ERR_NO_CAPACITY;
  sv->ctx = ctx;
  sv->p = *p;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete sv;
    return DSLAM_ERR_DEVICE;
  }
  sv->slots.resize(p->pipeline_depth);
  for (StepSlot& st : sv->slots) {
    dslam_status bs = dslam_batch_create(ctx, p->max_batch, &st.batch);
    if (bs != DSLAM_OK) {
      st.batch = nullptr;
      release(sv);
      return bs;
    }
    if (p->use_graphs && dslam_batch_set_graphs(st.batch, 1) != DSLAM_OK) {
      release(sv);
      return DSLAM_ERR_DEVICE;
    }
    if (hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&st.t0) != hipSuccess || hipEventCreate(&st.t1) != hipSuccess) {
      release(sv);
      return DSLAM_ERR_DEVICE;
    }
  }
  *out = sv;
  return DSLAM_OK;
}

dslam_status dslam_server_destroy(dslam_server* sv) {
  if (!sv) return DSLAM_ERR_INVALID;
  (void)hipSetDevice(sv->ctx->device);
  release(sv);
  return DSLAM_OK;
}

dslam_status dslam_server_submit(dslam_server* sv, dslam_session* session, const dslam_frame_input* frame,
                                 uint64_t* request_id) {
  if (!sv || !session || !frame || session->ctx != sv->ctx || !frame_ok(session, frame)) return DSLAM_ERR_INVALID;
  Request r;
  r.id = sv->next_id++;
  r.s = session;
  r.in = *frame;
  std::memset(r.imu, 0, sizeof(r.imu));
  if (session->tp.mode != DSLAM_MODE_RGBD)
    std::memcpy(r.imu, frame->imu, sizeof(dslam_imu_sample) * frame->n_imu);
  r.in.imu = nullptr;
  r.submit_s = steady_seconds();
  sv->pending.push_back(r);
  session->server_refs.fetch_add(1);  // the session cannot close while the server holds the request
  if (request_id) *request_id = r.id;
  return DSLAM_OK;
}

dslam_status dslam_server_poll(dslam_server* sv, int32_t wait, dslam_request_done* out, int32_t max_out,
                               int32_t* n_out) {
  if (!sv || (max_out > 0 && !out) || max_out < 0) return DSLAM_ERR_INVALID;
  if (hipSetDevice(sv->ctx->device) != hipSuccess) return DSLAM_ERR_DEVICE;
  dslam_status first_err = DSLAM_OK;
  for (;;) {
    for (StepSlot& st : sv->slots)
      if (st.busy && hipEventQuery(st.t1) == hipSuccess) {
        dslam_status rs = retire(sv, st);
        if (first_err == DSLAM_OK) first_err = rs;
      }
    for (StepSlot& st : sv->slots)
      if (!st.busy && !sv->pending.empty()) {
        dslam_status ls = launch(sv, st);
        if (first_err == DSLAM_OK) first_err = ls;
      }
    if (!wait || !sv->finished.empty() || sv->launched == 0) break;
    // block on the step launched first
    StepSlot* oldest = nullptr;
    for (StepSlot& st : sv->slots)
      if (st.busy && (!oldest || st.launch_s < oldest->launch_s)) oldest = &st;
    if (!oldest) break;
    if (hipEventSynchronize(oldest->t1) != hipSuccess) return DSLAM_ERR_DEVICE;
  }
  int n = 0;
  while (n < max_out && !sv->finished.empty()) {
    out[n++] = sv->finished.front();
    sv->finished.pop_front();
    out[n - 1].session->server_refs.fetch_sub(1);
  }
  if (n_out) *n_out = n;
  return first_err;
}

dslam_status dslam_server_counts(const dslam_server* sv, int32_t* pending, int32_t* in_flight) {
  if (!sv) return DSLAM_ERR_INVALID;
  if (pending) *pending = (int32_t)sv->pending.size();
  if (in_flight) *in_flight = sv->launched + (int32_t)sv->finished.size();
  return DSLAM_OK;
}

}  // extern "C"
