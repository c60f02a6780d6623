// Host-side objects behind the opaque handles of the C ABI (contexts,
// sessions, batches), shared by the library's host sources.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <vector>

#include "step.h"

struct dslam_context {
  int device;
  uint64_t budget;
  std::atomic<uint64_t> used{0};
  std::mutex tune_mu;
  std::vector<dslam_tune_entry> tuned;  // autotuned pixels per thread (dslam_context_autotune)
};

using dslam::LevelPtrs;
using dslam::SessionDev;

// A completion event that several sessions can share: one record at the end of
// a batched step marks that step's end for every session in it (one record
// and, for the next step on another stream, one wait instead of one per
// session).  Destroyed with its last holder.
struct DoneEvent {
  hipEvent_t ev = nullptr;
  ~DoneEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};
using DoneRef = std::shared_ptr<DoneEvent>;

struct dslam_session {
  dslam_context* ctx;
  dslam_camera cam;
  dslam_track_params tp;
  dslam_imu_params ip;
  int levels;
  uint64_t bytes;
  void* arena;
  LevelPtrs cur[DSLAM_MAX_LEVELS], model[DSLAM_MAX_LEVELS];
  SessionDev* sd;
  float* partials;
  int max_blocks;
  double* red_out;   // device, 64 doubles
  float* xf_scratch; // device, 24 floats (dslam_linearize)
  dslam_track_result* h_result;  // pinned host mirror of the result record (dslam_track_frame_sync)
  DoneRef own_done;         // the session's own completion event
  DoneRef done;             // the event recorded after the last enqueue of its work (own, or a batched step's)
  hipStream_t last_stream;  // stream of the last enqueue (a later enqueue on another stream waits for done)
  bool enqueued;            // done has been recorded at least once
  std::atomic<int> server_refs{0};  // requests of the session held by servers (queued or not yet returned)
  bool have_model;
  bool cur_normals_ok;  // the current pyramid's normal planes belong to its vertex planes (a batched step
                        // without the normal gate leaves them out; ensure_cur_normals fills them)
  double T_WM[16];
  int ppt[DSLAM_MAX_LEVELS];
  int banded[DSLAM_MAX_LEVELS];  // tile order of each level's residual pass (tile_of)
  // a frame's Gauss-Newton launches after the first, one graph per level,
  // captured at the first frame that uses them (null: not captured yet)
  dslam::SolveParams* sp_dev;  // device: the frame's solve parameters
  bool use_graphs;
  hipStream_t capture;
  hipGraphExec_t graph[DSLAM_MAX_LEVELS];
  std::mutex mu;
};

// Orders new work of the session on `st` after its earlier work when that was
// enqueued on another stream (the session's device state is updated in stream
// order, so a change of stream must not let two frames overlap).
inline hipError_t order_after_session(dslam_session* s, hipStream_t st) {
  if (s->enqueued && s->last_stream != st) return hipStreamWaitEvent(st, s->done->ev, 0);
  return hipSuccess;
}

// Marks the end of the session's work enqueued on `st` with its own event.
inline hipError_t mark_session(dslam_session* s, hipStream_t st) {
  hipError_t e = hipEventRecord(s->own_done->ev, st);
  if (e == hipSuccess) {
    s->done = s->own_done;
    s->last_stream = st;
    s->enqueued = true;
  }
  return e;
}

// Marks the end of the session's work enqueued on `st` with `d`, already
// recorded on `st` after that work.
inline void mark_session_shared(dslam_session* s, hipStream_t st, const DoneRef& d) {
  s->done = d;
  s->last_stream = st;
  s->enqueued = true;
}

// Fills the current pyramid's normal planes on `st` where a batched step left
// them out (the caller orders `st` after the session's work).
inline hipError_t ensure_cur_normals(dslam_session* s, hipStream_t st) {
  if (s->cur_normals_ok) return hipSuccess;
  for (int l = 0; l < s->levels; ++l) {
    const hipError_t e = dslam::launch_normals(s->cur[l], st);
    if (e != hipSuccess) return e;
  }
  s->cur_normals_ok = true;
  return hipSuccess;
}

// The session's completion event (valid once enqueued).
inline hipEvent_t session_done(const dslam_session* s) { return s->done->ev; }

struct dslam_batch {
  dslam_context* ctx;
  int max_n;
  uint64_t bytes;
  void* dev;                   // SlotVis[max_n] | SlotSolve[max_n] | dslam_track_result[max_n]
  dslam::SlotVis* d_vis;
  dslam::SlotSolve* d_solve;
  dslam_track_result* d_res;
  void* host;                  // pinned mirror of the same layout
  dslam::SlotVis* h_vis;
  dslam::SlotSolve* h_solve;
  dslam_track_result* h_res;
  hipEvent_t done;
  std::vector<DoneRef> step_done;  // shared completion events of its steps (reused once no session holds one)
  bool pending;
  int n;
  int order[dslam::MAX_BATCH];        // slot -> caller index
  int levels;                         // of the last step
  int jac;
  int max_ppt[DSLAM_MAX_LEVELS];
  int banded[DSLAM_MAX_LEVELS];
  dslam::BatchGrid res_grid[DSLAM_MAX_LEVELS];  // residual work split of the last step
  uint64_t pixels[DSLAM_MAX_LEVELS];            // pixels per residual pass of the last step
  // the step's launches replayed from graphs, one per plan of launches (batch
  // composition and schedule), captured at the first step with that plan
  int tile_order = 1;  // batched residual passes: 1 XCD-banded, 0 round-robin, -1 the first class's tuned order
  bool use_graphs = false;
  hipStream_t capture = nullptr;
  std::vector<std::pair<std::vector<int32_t>, hipGraphExec_t>> graphs;
};

// dslam_batch_track with `start` (nullable) recorded on `st` once the step's
// staging is enqueued and its sessions' earlier work is waited for, i.e. where
// the step's own device time begins.
dslam_status batch_track_timed(dslam_batch* b, int32_t n, dslam_session* const* sessions,
                               const dslam_frame_input* frames, hipStream_t st, hipEvent_t start);
