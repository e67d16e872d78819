// Launch timing (a measurement aid, not part of the method): HIP events bracket the timed launches
// on the stream they are launched on, so that durations are measured without synchronising the
// caller. The record is host-side and process-wide.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace invdft {

namespace {
struct TimedLaunch {
  hipEvent_t start, stop;
  int kind;       // an fe_prec for applies, kTimedSweep + pass for the MINRES sweeps
  double bytes;
  double cols;
};
struct LaunchTiming {
  bool on = false;
  std::vector<TimedLaunch> rec;     // launches of the current measurement
  std::vector<hipEvent_t> spare;    // events of earlier measurements, reused
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!spare.empty()) {
      e = spare.back();
      spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  void clear() {
    for (auto& t : rec) {
      spare.push_back(t.start);
      spare.push_back(t.stop);
    }
    rec.clear();
  }
};
LaunchTiming g_timing;

// sums of the recorded launches of one kind
fe_status timing_sum(int kind, int64_t* launches, double* ms, double* bytes, double* columns) {
  int64_t n = 0;
  double t = 0.0, b = 0.0, cl = 0.0;
  for (auto& r : g_timing.rec) {
    if (r.kind != kind) continue;
    INVDFT_HIP(hipEventSynchronize(r.stop));
    float e = 0.0f;
    INVDFT_HIP(hipEventElapsedTime(&e, r.start, r.stop));
    ++n;
    t += e;
    b += r.bytes;
    cl += r.cols;
  }
  if (launches) *launches = n;
  if (ms) *ms = t;
  if (bytes) *bytes = b;
  if (columns) *columns = cl;
  return FE_OK;
}
}  // namespace

fe_status apply_timing(int enable) {
  if (enable) g_timing.clear();
  g_timing.on = enable != 0;
  return FE_OK;
}

fe_status apply_timing_read(fe_prec prec, int64_t* launches, double* ms, double* bytes, double* columns) {
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16)
    return fail(FE_EINVAL, "fe_apply_timing_read: prec must be FE_F64, FE_F32 or FE_BF16");
  return timing_sum((int)prec, launches, ms, bytes, columns);
}

fe_status sweep_timing_read(int pass, int64_t* launches, double* ms, double* bytes, double* columns) {
  if (pass < 0 || pass > 2) return fail(FE_EINVAL, "fe_sweep_timing_read: pass must be 0 (A), 1 (B) or 2 (C)");
  return timing_sum(kTimedSweep + pass, launches, ms, bytes, columns);
}

fe_status timed_begin(int kind, double bytes, double cols, hipStream_t s, int* slot) {
  *slot = -1;
  if (!g_timing.on) return FE_OK;
  TimedLaunch t{g_timing.take(), g_timing.take(), kind, bytes, cols};
  if (!t.start || !t.stop) return fail(FE_EDEVICE, "launch timing: hipEventCreate failed");
  INVDFT_HIP(hipEventRecord(t.start, s));
  *slot = (int)g_timing.rec.size();
  g_timing.rec.push_back(t);
  return FE_OK;
}

fe_status timed_end(int slot, hipStream_t s) {
  if (slot < 0) return FE_OK;
  INVDFT_HIP(hipEventRecord(g_timing.rec[slot].stop, s));
  return FE_OK;
}

}  // namespace invdft
