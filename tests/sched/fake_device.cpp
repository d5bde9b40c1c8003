// A recording stand-in for the device side of libdgrtm, for CPU tests of the host driver.
//
// The host driver (csrc/api.cpp) and the host set-up (csrc/setup.cpp) are linked against this
// file instead of the HIP kernels and the HIP runtime.  "Device" memory is host memory handed in
// by the caller, so copies are plain memcpy; a kernel launch computes nothing and appends one
// record per launch (per slot for the step kernel) to a log that the test reads back.  The log
// holds what the host decided: modes, active prefixes, local steps, physical times, segment
// windows, checkpoint copies, receiver and boundary recording.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "../../paper_1506_00907_amd/csrc/kernels.hpp"

namespace {

constexpr int kRecWords = 24;
struct Rec {
  int64_t v[kRecWords];
};
std::vector<Rec> g_log;

// record kinds
enum : int64_t {
  R_STEP = 1, R_RECORD = 2, R_COPY = 3, R_TRACE_INIT = 4, R_SEG_INIT = 5, R_FILL = 6, R_BND = 7,
  R_REPLAY_HIST = 8, R_OTHER = 9
};

Rec &push(int64_t kind) {
  g_log.push_back(Rec{});
  Rec &r = g_log.back();
  r.v[0] = kind;
  return r;
}

int64_t ip(const void *p) { return (int64_t)(intptr_t)p; }

}  // namespace

extern "C" {

int64_t fake_log_size(void) { return (int64_t)g_log.size(); }
int fake_log_words(void) { return kRecWords; }
void fake_log_read(int64_t *out) {
  for (size_t i = 0; i < g_log.size(); ++i) std::memcpy(out + i * kRecWords, g_log[i].v, sizeof(Rec));
}
void fake_log_clear(void) { g_log.clear(); }

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  if (bytes) std::memmove(dst, src, bytes);
  Rec &r = push(R_COPY);
  r.v[1] = (int64_t)kind;
  r.v[2] = ip(dst);
  r.v[3] = ip(src);
  r.v[4] = (int64_t)bytes;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t *e) {
  *e = reinterpret_cast<hipEvent_t>(new int(0));
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<int *>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "fake device"; }

}  // extern "C"

namespace dgrtm {

hipError_t launch_step(int, const StepArgs &a, hipStream_t) {
  for (int i = 0; i < a.nslots; ++i) {
    const SlotArgs &s = a.slot[i];
    Rec &r = push(R_STEP);
    r.v[1] = a.mode;
    r.v[2] = a.k_end;
    r.v[3] = a.tau_sign < 0.0f ? 1 : 0;
    r.v[4] = i;
    r.v[5] = a.nslots;
    r.v[6] = s.tau;
    r.v[7] = s.data_j;
    r.v[8] = s.g0;
    r.v[9] = s.g1;
    r.v[10] = s.image_from;
    r.v[11] = s.img_rule;
    r.v[12] = s.amp_mode;
    r.v[13] = s.src_scale < 0.0f ? 1 : 0;
    r.v[14] = a.precision;
    r.v[15] = ip(s.q);
    r.v[16] = s.NG;
    r.v[17] = s.C;
    r.v[18] = a.n_local;
    r.v[19] = s.n_t;
    r.v[20] = ip(s.rhs_out);
    r.v[21] = s.condition;
  }
  return hipSuccess;
}

hipError_t launch_record(int, const float *q, int64_t, const int64_t *, const float *, int64_t n_rec, float *out,
                         int64_t out_stride, hipStream_t) {
  Rec &r = push(R_RECORD);
  r.v[1] = ip(q);
  r.v[2] = ip(out);
  r.v[3] = n_rec;
  r.v[4] = out_stride;
  return hipSuccess;
}

hipError_t launch_trace_init(int, const TraceInitArgs &a, hipStream_t) {
  Rec &r = push(R_TRACE_INIT);
  r.v[1] = ip(a.q);
  r.v[2] = a.tau;
  return hipSuccess;
}

hipError_t launch_seg_init(int, const SegInitArgs &a, hipStream_t) {
  Rec &r = push(R_SEG_INIT);
  r.v[1] = a.history_before_start;
  r.v[2] = a.L;
  for (int l = 0; l < a.L && l < kMaxLevels; ++l) r.v[3 + l] = a.seg_m0[l];
  r.v[12] = ip(a.ring);
  return hipSuccess;
}

hipError_t launch_bnd_record(int, const BndRecArgs &a, hipStream_t) {
  Rec &r = push(R_BND);
  r.v[1] = a.tau;
  r.v[2] = a.n_active;
  return hipSuccess;
}

hipError_t launch_replay_history(int, const float *, const float *, const float *, float *ring, int64_t, int,
                                 const int64_t *, hipStream_t) {
  Rec &r = push(R_REPLAY_HIST);
  r.v[1] = ip(ring);
  return hipSuccess;
}

hipError_t launch_fill_f32(float *p, int64_t n, float, hipStream_t) {
  Rec &r = push(R_FILL);
  r.v[1] = ip(p);
  r.v[2] = n;
  r.v[3] = 32;
  return hipSuccess;
}

hipError_t launch_fill_f64(double *p, int64_t n, double, hipStream_t) {
  Rec &r = push(R_FILL);
  r.v[1] = ip(p);
  r.v[2] = n;
  r.v[3] = 64;
  return hipSuccess;
}

hipError_t launch_to_device_layout(int, int, const float *, float *, const int64_t *, int64_t, hipStream_t) {
  push(R_OTHER).v[1] = 1;
  return hipSuccess;
}
hipError_t launch_to_user_layout(int, int, const float *, float *, const int64_t *, int64_t, hipStream_t) {
  push(R_OTHER).v[1] = 2;
  return hipSuccess;
}
hipError_t launch_image_to_user(int, const double *, double *, const int64_t *, int64_t, int, hipStream_t) {
  push(R_OTHER).v[1] = 3;
  return hipSuccess;
}
hipError_t launch_residual(const float *, const float *, int64_t, double *, hipStream_t) {
  push(R_OTHER).v[1] = 4;
  return hipSuccess;
}

// operator fragments: the driver only sizes, fills and uploads them
int64_t op_fragment_floats(int) { return 64; }
int64_t op_fragment_bf16_words(int) { return 64; }
void build_op_fragments(int, const float *, const float *, const float *, const float *, float *out) {
  std::memset(out, 0, 64 * sizeof(float));
}
void build_op_fragments_bf16(int, const double *, const double *, const double *, const double *, uint32_t *out) {
  std::memset(out, 0, 64 * sizeof(uint32_t));
}

}  // namespace dgrtm
