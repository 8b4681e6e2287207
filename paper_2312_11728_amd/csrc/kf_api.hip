// C interface of libkf: argument validation, contexts and kernel dispatch.
// Every entry point validates its scalar arguments and pointers before it
// touches the device, so a bad call fails with KF_ERR_ARG and a message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kf.h"
#include "kf_backward.hpp"
#include "kf_dedup.hpp"
#include "kf_kernels.hpp"
#include "kf_plane_launch.hpp"
#include "kf_search_launch.hpp"

// A named roctx range around one call of the interface, so that a profiler's
// timeline groups each call's kernels and copies under the entry point's name
// (rocprofv3 --marker-trace).  Without a profiler attached the push and pop
// cost a few tens of nanoseconds.
struct KfRange {
  explicit KfRange(const char* name) { roctxRangePushA(name); }
  ~KfRange() { roctxRangePop(); }
  KfRange(const KfRange&) = delete;
  KfRange& operator=(const KfRange&) = delete;
};
#define KF_RANGE() KfRange kf_range_(__func__)

struct kf_ctx {
  int device = 0;
  int n_cu = 256;
  int32_t* d_counter = nullptr;      // persistent-kernel tile counter
  kf::FitLaunch fit[2] = {{256, 0, 4, 1, 0}, {256, 0, 4, 1, 0}};  // per precision
  // graph cache for kf_fit_tracks (one entry per precision)
  bool use_graph[2] = {false, false};
  hipStream_t capture = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<unsigned char> key[2];   // launch arguments the graph was captured with
  // workspace of the packed hit layout (kf_reserve)
  void* work_mem = nullptr;
  kf::PackWork work{};
  // block partials of the alignment-gradient reduction (grown on demand)
  void* red_mem = nullptr;
  size_t red_bytes = 0;
  // device address of this device's fixed scratch array (kf_fit_adjoint_noalloc)
  void* scratch = nullptr;
  // workspace of the candidate search (grown on demand) and the identity of
  // the pool its bins were built from
  void* search_mem = nullptr;
  size_t search_bytes = 0;
  std::vector<unsigned char> bins_key;
  // workspace of duplicate removal (grown on demand)
  void* dedup_mem = nullptr;
  size_t dedup_bytes = 0;
  // workspace of the final fit's rounds (grown on demand)
  void* final_mem = nullptr;
  size_t final_bytes = 0;
  int32_t* final_counts = nullptr;   // pinned host copy of a round's open-track count
  // event pairs around the fit kernel of direct launches (kf_set_kernel_timing)
  bool timing = false;
  std::vector<hipEvent_t> t_start, t_stop;
  int t_used = 0;
  int64_t t_dropped = 0;
};

// Fixed device scratch of kf_fit_adjoint_noalloc: the block partials of the
// alignment-gradient reduction, for callers that cannot allocate.  Each device
// the library runs on holds its own copy until the process ends.  Host code
// never passes `scratch` itself to a kernel (on the host it is only a stand-in
// for the symbol): it uses the device address hipGetSymbolAddress returns,
// looked up once per device by kf_create with that device current.
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

constexpr int32_t kMaxTimedLaunches = 4096;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return KF_OK;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(KF_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Device address of the scratch array on `device`, which must be current;
// looked up on the first call for that device and kept.
int scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(KF_ERR_DEVICE, "device %d outside the scratch table", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(KF_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return KF_OK;
}

int check_geometry(const kf_geometry* g, kf::GeomArgs* out) {
  if (!g) return fail(KF_ERR_ARG, "geometry is NULL");
  if (g->n_layers < 1 || g->n_layers > KF_MAX_LAYERS)
    return fail(KF_ERR_ARG, "geometry.n_layers = %d outside [1, %d]", g->n_layers, KF_MAX_LAYERS);
  if (!g->kind || !g->pos || !g->lo || !g->hi || !g->x_over_x0) return fail(KF_ERR_ARG, "geometry array is NULL");
  if (!std::isfinite(g->bz_tesla) || g->bz_tesla == 0.0) return fail(KF_ERR_ARG, "geometry.bz_tesla must be finite and != 0");
  if (!std::isfinite(g->particle_mass_gev) || !(g->particle_mass_gev > 0.0))
    return fail(KF_ERR_ARG, "geometry.particle_mass_gev must be > 0");
  std::memset(out, 0, sizeof(*out));
  out->n_layers = g->n_layers;
  for (int i = 0; i < g->n_layers; ++i) {
    if (g->kind[i] != 0 && g->kind[i] != 1) return fail(KF_ERR_ARG, "geometry.kind[%d] = %d (0 barrel, 1 disk)", i, g->kind[i]);
    if (!std::isfinite(g->pos[i]) || (g->kind[i] == 0 && !(g->pos[i] > 0.0)))
      return fail(KF_ERR_ARG, "geometry.pos[%d] invalid", i);
    if (!std::isfinite(g->lo[i]) || !std::isfinite(g->hi[i]) || !(g->lo[i] <= g->hi[i]))
      return fail(KF_ERR_ARG, "geometry.lo/hi[%d] invalid", i);
    if (!std::isfinite(g->x_over_x0[i]) || g->x_over_x0[i] < 0.0) return fail(KF_ERR_ARG, "geometry.x_over_x0[%d] invalid", i);
    out->kind[i] = g->kind[i];
    out->pos[i] = g->pos[i];
    out->x0[i] = g->x_over_x0[i];
  }
  out->bz = g->bz_tesla;
  out->mass = g->particle_mass_gev;
  return KF_OK;
}

int check_sizes(int64_t n, int64_t ld) {
  if (n < 0) return fail(KF_ERR_ARG, "n = %lld < 0", (long long)n);
  if (ld < n) return fail(KF_ERR_ARG, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (ld > (int64_t(1) << 40)) return fail(KF_ERR_ARG, "ld too large");
  return KF_OK;
}

int check_prec(int prec) {
  if (prec != KF_F32 && prec != KF_F64) return fail(KF_ERR_ARG, "precision %d unknown", prec);
  return KF_OK;
}

#define KF_REQUIRE(ptr)                                                   \
  do {                                                                    \
    if (!(ptr)) return fail(KF_ERR_ARG, "%s is NULL", #ptr);              \
  } while (0)

void drop_timing_events(kf_ctx* ctx) {
  for (hipEvent_t ev : ctx->t_start) hipEventDestroy(ev);
  for (hipEvent_t ev : ctx->t_stop) hipEventDestroy(ev);
  ctx->t_start.clear();
  ctx->t_stop.clear();
  ctx->t_used = 0;
  ctx->t_dropped = 0;
}

#define KF_TRY(expr)                 \
  do {                               \
    int rc_ = (expr);                \
    if (rc_ != KF_OK) return rc_;    \
  } while (0)

}  // namespace

extern "C" {

const char* kf_last_error(void) { return g_err.c_str(); }

int kf_create(kf_ctx** out, int hip_device) {
  KF_REQUIRE(out);
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return fail(KF_ERR_DEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= count) return fail(KF_ERR_ARG, "hip_device %d outside [0, %d)", hip_device, count);
  int prev = 0;
  hipGetDevice(&prev);
  if ((e = hipSetDevice(hip_device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  kf_ctx* c = new kf_ctx();
  c->device = hip_device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  e = hipMalloc(&c->d_counter, 64);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
  const int rc = e == hipSuccess ? scratch_address(hip_device, &c->scratch) : int(KF_OK);
  hipSetDevice(prev);
  if (e != hipSuccess || rc != KF_OK) {
    if (c->capture) hipStreamDestroy(c->capture);
    if (c->d_counter) hipFree(c->d_counter);
    delete c;
    return e != hipSuccess ? hip_fail(e, "kf_create") : rc;
  }
  *out = c;
  return ok();
}

int kf_destroy(kf_ctx* c) {
  if (!c) return ok();
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(c->device);
  for (int i = 0; i < 2; ++i)
    if (c->exec[i]) hipGraphExecDestroy(c->exec[i]);
  drop_timing_events(c);
  if (c->capture) hipStreamDestroy(c->capture);
  if (c->d_counter) hipFree(c->d_counter);
  if (c->work_mem) hipFree(c->work_mem);
  if (c->red_mem) hipFree(c->red_mem);
  if (c->search_mem) hipFree(c->search_mem);
  if (c->dedup_mem) hipFree(c->dedup_mem);
  if (c->final_mem) hipFree(c->final_mem);
  if (c->final_counts) hipHostFree(c->final_counts);
  hipSetDevice(prev);
  delete c;
  return ok();
}

int kf_make_seeds(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const int32_t* hit_offsets,
                  const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, double bz_tesla, int32_t mode,
                  void* seed_state, void* seed_cov, int8_t* seed_charge, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (mode != 0 && mode != 1) return fail(KF_ERR_ARG, "seed mode %d unknown (0 first three, 1 spaced)", mode);
  if (!std::isfinite(bz_tesla) || bz_tesla == 0.0) return fail(KF_ERR_ARG, "bz_tesla must be finite and != 0");
  if (n == 0) return ok();
  KF_REQUIRE(hit_offsets);
  KF_REQUIRE(hit_valid);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(seed_state);
  KF_REQUIRE(seed_cov);
  KF_REQUIRE(seed_charge);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == KF_F32) {
    kf::SeedArgs<float> a{n, ld, n_hits, hit_offsets, hit_valid, (const float*)hit_pos, bz_tesla, mode,
                          (float*)seed_state, (float*)seed_cov, seed_charge, trk_status};
    e = kf::launch_seeds(a, s);
  } else {
    kf::SeedArgs<double> a{n, ld, n_hits, hit_offsets, hit_valid, (const double*)hit_pos, bz_tesla, mode,
                           (double*)seed_state, (double*)seed_cov, seed_charge, trk_status};
    e = kf::launch_seeds(a, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_make_seeds");
  return ok();
}

int kf_propagate(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* state_in, const void* cov_in,
                 const int8_t* charge, const int16_t* target_layer, const int16_t* from_layer, const kf_geometry* geom,
                 int32_t apply_material, void* state_out, void* cov_out, void* path_len, uint32_t* trk_status,
                 void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n == 0) return ok();
  KF_REQUIRE(state_in);
  KF_REQUIRE(cov_in);
  KF_REQUIRE(charge);
  KF_REQUIRE(target_layer);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == KF_F32) {
    kf::PropArgs<float> a{n, ld, (const float*)state_in, (const float*)cov_in, charge, target_layer, from_layer,
                          apply_material, (float*)state_out, (float*)cov_out, (float*)path_len, trk_status};
    e = kf::launch_propagate(a, g, s);
  } else {
    kf::PropArgs<double> a{n, ld, (const double*)state_in, (const double*)cov_in, charge, target_layer, from_layer,
                           apply_material, (double*)state_out, (double*)cov_out, (double*)path_len, trk_status};
    e = kf::launch_propagate(a, g, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_propagate");
  return ok();
}

int kf_update(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, void* state, void* cov, int8_t* charge,
              const void* hit_pos, const void* hit_cov, void* chi2, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  if (n == 0) return ok();
  KF_REQUIRE(state);
  KF_REQUIRE(cov);
  KF_REQUIRE(charge);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(hit_cov);
  KF_REQUIRE(chi2);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == KF_F32) {
    kf::UpdArgs<float> a{n, ld, (float*)state, (float*)cov, charge, (const float*)hit_pos, (const float*)hit_cov,
                         (float*)chi2, trk_status};
    e = kf::launch_update(a, s);
  } else {
    kf::UpdArgs<double> a{n, ld, (double*)state, (double*)cov, charge, (const double*)hit_pos,
                          (const double*)hit_cov, (double*)chi2, trk_status};
    e = kf::launch_update(a, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_update");
  return ok();
}

}  // extern "C"

namespace {

template <typename T>
kf::FitArgs<T> make_fit_args(int64_t n, int64_t ld, const void* seed_state, const void* seed_cov,
                             const int8_t* seed_charge, const int32_t* hit_offsets, const int16_t* hit_layer,
                             const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, const void* hit_cov,
                             const void* align, void* state_out, void* cov_out, int8_t* charge_out, void* chi2,
                             int32_t* ndf, void* ckpt, int32_t seg, int32_t n_seg, uint32_t* trk_status,
                             int32_t* counter) {
  kf::FitArgs<T> a;
  std::memset(&a, 0, sizeof(a));   // padding too: the bytes key the graph cache
  a.n = n;
  a.ld = ld;
  a.n_hits = n_hits;
  a.seed_state = (const T*)seed_state;
  a.seed_cov = (const T*)seed_cov;
  a.seed_charge = seed_charge;
  a.hit_offsets = hit_offsets;
  a.hit_layer = hit_layer;
  a.hit_valid = hit_valid;
  a.hit_pos = (const T*)hit_pos;
  a.hit_cov = (const T*)hit_cov;
  a.align = (const T*)align;
  a.state_out = (T*)state_out;
  a.cov_out = (T*)cov_out;
  a.charge_out = charge_out;
  a.chi2 = (T*)chi2;
  a.ndf = ndf;
  a.ckpt = (T*)ckpt;
  a.seg = seg;
  a.n_seg = n_seg;
  a.trk_status = trk_status;
  a.tile_counter = counter;
  a.n_tiles = 0;
  a.max_len = kf::kMaxLen;
  a.packed = 0;
  a.pk = kf::PackedHits<T>{};
  return a;
}

// The launch sequence of one fit: the optional sort / pack passes, then the
// fit kernel (with the tile-counter reset of the persistent form).
template <typename T>
hipError_t run_fit(kf_ctx* ctx, kf::FitArgs<T> a, const kf::GeomArgs& g, const kf::FitLaunch& l, int layout,
                   hipStream_t s, bool may_time = true) {
  if (layout == 1 || layout == 2 || layout == 4) {
    hipError_t e = kf::launch_pack(a, ctx->work, layout, &a.pk, s);
    if (e != hipSuccess) return e;
  }
  a.packed = layout;
  // graph captures (on the context's capture stream) carry no timing events
  const bool timed = may_time && ctx->timing && s != ctx->capture;
  if (timed && ctx->t_used >= int(ctx->t_start.size())) ++ctx->t_dropped;
  const int slot = timed && ctx->t_used < int(ctx->t_start.size()) ? ctx->t_used++ : -1;
  if (slot >= 0) {
    hipError_t e = hipEventRecord(ctx->t_start[slot], s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = kf::launch_fit(a, g, l, ctx->n_cu, s);
  if (e == hipSuccess && slot >= 0) e = hipEventRecord(ctx->t_stop[slot], s);
  return e;
}


// With graphs enabled, the sequence is captured once on the context's
// capture stream and replayed on the caller's stream while every launch
// argument stays the same (any change re-captures).  The sequence clears its
// counters with kernels, so a replay needs no host-side work.
template <typename T>
hipError_t run_fit_graph(kf_ctx* ctx, int pi, const kf::FitArgs<T>& a, const kf::GeomArgs& g,
                         const kf::FitLaunch& l, int layout, hipStream_t s) {
  std::vector<unsigned char> key(sizeof(a) + sizeof(g) + sizeof(l) + sizeof(layout));
  unsigned char* k = key.data();
  std::memcpy(k, &a, sizeof(a));
  std::memcpy(k + sizeof(a), &g, sizeof(g));
  std::memcpy(k + sizeof(a) + sizeof(g), &l, sizeof(l));
  std::memcpy(k + sizeof(a) + sizeof(g) + sizeof(l), &layout, sizeof(layout));
  if (!ctx->exec[pi] || key != ctx->key[pi]) {
    if (ctx->exec[pi]) hipGraphExecDestroy(ctx->exec[pi]);
    ctx->exec[pi] = nullptr;
    ctx->key[pi].clear();
    hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t er = run_fit(ctx, a, g, l, layout, ctx->capture);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture, &graph);
    if (er == hipSuccess) er = e;
    if (er == hipSuccess) er = hipGraphInstantiate(&ctx->exec[pi], graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (er != hipSuccess) {
      ctx->exec[pi] = nullptr;
      return er;
    }
    ctx->key[pi] = key;
  }
  return hipGraphLaunch(ctx->exec[pi], s);
}

}  // namespace

extern "C" {

int kf_set_fit_graph(kf_ctx* ctx, int32_t enable) {
  KF_REQUIRE(ctx);
  if (enable != 0 && enable != 1) return fail(KF_ERR_ARG, "enable must be 0 or 1");
  for (int i = 0; i < 2; ++i) {
    ctx->use_graph[i] = enable != 0;
    if (!enable && ctx->exec[i]) {
      hipGraphExecDestroy(ctx->exec[i]);
      ctx->exec[i] = nullptr;
      ctx->key[i].clear();
    }
  }
  return ok();
}

int kf_set_kernel_timing(kf_ctx* ctx, int32_t max_launches) {
  KF_REQUIRE(ctx);
  if (max_launches < 0 || max_launches > kMaxTimedLaunches)
    return fail(KF_ERR_ARG, "max_launches = %d outside [0, %d]", max_launches, kMaxTimedLaunches);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(ctx->device);
  drop_timing_events(ctx);
  ctx->timing = max_launches > 0;
  hipError_t e = hipSuccess;
  for (int i = 0; i < max_launches && e == hipSuccess; ++i) {
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (a) ctx->t_start.push_back(a);
    if (b) ctx->t_stop.push_back(b);
    if (e == hipSuccess && (!a || !b)) e = hipErrorInvalidValue;
  }
  if (e != hipSuccess) {
    drop_timing_events(ctx);
    ctx->timing = false;
  }
  hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(e, "kf_set_kernel_timing");
  return ok();
}

int kf_fit_kernel_time(kf_ctx* ctx, double* total_ms, int64_t* launches, int64_t* dropped) {
  KF_REQUIRE(ctx);
  KF_REQUIRE(total_ms);
  KF_REQUIRE(launches);
  double sum = 0.0;
  for (int i = 0; i < ctx->t_used; ++i) {
    hipError_t e = hipEventSynchronize(ctx->t_stop[i]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->t_start[i], ctx->t_stop[i]);
    if (e != hipSuccess) return hip_fail(e, "kf_fit_kernel_time");
    sum += double(ms);
  }
  *total_ms = sum;
  *launches = ctx->t_used;
  if (dropped) *dropped = ctx->t_dropped;
  ctx->t_used = 0;
  ctx->t_dropped = 0;
  return ok();
}

}  // extern "C"

namespace {

// The fit call shared by kf_fit_tracks (given seeds) and kf_seed_fit_tracks
// (seed_mode >= 0: every track seeded from its hits inside the fit kernel).
int fit_tracks_impl(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                    const void* seed_cov, const int8_t* seed_charge, int32_t seed_mode, void* seed_state_out,
                    void* seed_cov_out, int8_t* seed_charge_out, const int32_t* hit_offsets,
                    const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                    const void* hit_cov, const kf_geometry* geom, const void* align, void* state_out, void* cov_out,
                    int8_t* charge_out, void* chi2, int32_t* ndf, void* checkpoints, int32_t seg, int32_t max_len,
                    uint32_t* trk_status, void* stream) {
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (checkpoints && seg < 1) return fail(KF_ERR_ARG, "seg = %d < 1", seg);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  if (seed_mode < -1 || seed_mode > 1) return fail(KF_ERR_ARG, "seed mode %d unknown (0 first three, 1 spaced)", seed_mode);
  if (n == 0) return ok();
  if (seed_mode < 0) {
    KF_REQUIRE(seed_state);
    KF_REQUIRE(seed_cov);
    KF_REQUIRE(seed_charge);
  }
  KF_REQUIRE(hit_offsets);
  KF_REQUIRE(hit_layer);
  KF_REQUIRE(hit_valid);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(hit_cov);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(charge_out);
  KF_REQUIRE(chi2);
  KF_REQUIRE(ndf);
  KF_REQUIRE(trk_status);
  int32_t n_seg = 0;
  if (checkpoints) {
    n_seg = (max_len - 1 + seg - 1) / seg;
    if (n_seg < 1) n_seg = 1;
  }
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  const int pi = prec == KF_F32 ? 0 : 1;
  const kf::FitLaunch l = ctx->fit[pi];
  const bool room = ctx->work.cap > 0 && n <= ctx->work.max_tracks && max_len <= ctx->work.max_len;
  const int layout = room || l.layout == 3 ? l.layout : (l.layout == 4 ? 3 : 0);
  hipError_t e;
  if (prec == KF_F32) {
    auto a = make_fit_args<float>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, n_hits,
                                  hit_pos, hit_cov, align, state_out, cov_out, charge_out, chi2, ndf, checkpoints, seg,
                                  n_seg, trk_status, ctx->d_counter);
    a.max_len = max_len;
    a.make_seeds = seed_mode + 1;
    a.seed_state_out = (float*)seed_state_out;
    a.seed_cov_out = (float*)seed_cov_out;
    a.seed_charge_out = seed_charge_out;
    e = ctx->use_graph[pi] && !ctx->timing ? run_fit_graph(ctx, pi, a, g, l, layout, s)
                                           : run_fit(ctx, a, g, l, layout, s);
  } else {
    auto a = make_fit_args<double>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid,
                                   n_hits, hit_pos, hit_cov, align, state_out, cov_out, charge_out, chi2, ndf,
                                   checkpoints, seg, n_seg, trk_status, ctx->d_counter);
    a.max_len = max_len;
    a.make_seeds = seed_mode + 1;
    a.seed_state_out = (double*)seed_state_out;
    a.seed_cov_out = (double*)seed_cov_out;
    a.seed_charge_out = seed_charge_out;
    e = ctx->use_graph[pi] && !ctx->timing ? run_fit_graph(ctx, pi, a, g, l, layout, s)
                                           : run_fit(ctx, a, g, l, layout, s);
  }
  if (e != hipSuccess) return hip_fail(e, seed_mode < 0 ? "kf_fit_tracks" : "kf_seed_fit_tracks");
  return ok();
}

}  // namespace

extern "C" {

int kf_fit_tracks(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state, const void* seed_cov,
                  const int8_t* seed_charge, const int32_t* hit_offsets, const int16_t* hit_layer,
                  const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, const void* hit_cov,
                  const kf_geometry* geom, const void* align, void* state_out, void* cov_out, int8_t* charge_out,
                  void* chi2, int32_t* ndf, void* checkpoints, int32_t seg, int32_t max_len, uint32_t* trk_status,
                  void* stream) {
  KF_RANGE();
  return fit_tracks_impl(ctx, prec, n, ld, seed_state, seed_cov, seed_charge, -1, nullptr, nullptr, nullptr,
                         hit_offsets, hit_layer, hit_valid, n_hits, hit_pos, hit_cov, geom, align, state_out, cov_out,
                         charge_out, chi2, ndf, checkpoints, seg, max_len, trk_status, stream);
}

int kf_seed_fit_tracks(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, int32_t seed_mode,
                       const int32_t* hit_offsets, const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits,
                       const void* hit_pos, const void* hit_cov, const kf_geometry* geom, const void* align,
                       void* seed_state_out, void* seed_cov_out, int8_t* seed_charge_out, void* state_out,
                       void* cov_out, int8_t* charge_out, void* chi2, int32_t* ndf, void* checkpoints, int32_t seg,
                       int32_t max_len, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  if (seed_mode != 0 && seed_mode != 1) return fail(KF_ERR_ARG, "seed mode %d unknown (0 first three, 1 spaced)", seed_mode);
  return fit_tracks_impl(ctx, prec, n, ld, nullptr, nullptr, nullptr, seed_mode, seed_state_out, seed_cov_out,
                         seed_charge_out, hit_offsets, hit_layer, hit_valid, n_hits, hit_pos, hit_cov, geom, align,
                         state_out, cov_out, charge_out, chi2, ndf, checkpoints, seg, max_len, trk_status, stream);
}

}  // extern "C"

namespace {

// kf_backward_fit and kf_smooth_tracks (fwd_checkpoints and the smooth_*
// outputs set).
int backward_impl(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* state_in, const void* cov_in,
                  const int8_t* charge_in, const uint32_t* fwd_status, const void* fwd_checkpoints,
                  const int32_t* hit_offsets, const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits,
                  const void* hit_pos, const void* hit_cov, const kf_geometry* geom, double cov_scale,
                  int32_t max_len, void* state_out, void* cov_out, int8_t* charge_out, void* chi2, int32_t* ndf,
                  uint32_t* trk_status, void* smooth_state, void* smooth_cov, const char* name, void* stream) {
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  if (!std::isfinite(cov_scale) || !(cov_scale >= 1.0)) return fail(KF_ERR_ARG, "cov_scale must be finite and >= 1");
  if (n == 0) return ok();
  KF_REQUIRE(state_in);
  KF_REQUIRE(cov_in);
  KF_REQUIRE(charge_in);
  KF_REQUIRE(hit_offsets);
  KF_REQUIRE(hit_layer);
  KF_REQUIRE(hit_valid);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(hit_cov);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(charge_out);
  KF_REQUIRE(chi2);
  KF_REQUIRE(ndf);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  if (state_out == state_in || cov_out == cov_in || (const void*)charge_out == (const void*)charge_in)
    return fail(KF_ERR_ARG, "the outputs must not alias the inputs");
  const bool smooth = fwd_checkpoints != nullptr || smooth_state != nullptr || smooth_cov != nullptr;
  if (smooth) {
    KF_REQUIRE(fwd_checkpoints);
    KF_REQUIRE(smooth_state);
    KF_REQUIRE(smooth_cov);
    if (smooth_state == smooth_cov || smooth_state == state_out || smooth_cov == cov_out)
      return fail(KF_ERR_ARG, "the smoothed outputs must not alias each other or the outputs");
  }
  const int32_t n_seg_f = max_len > 1 ? max_len - 1 : 1;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == KF_F32) {
    kf::BwdArgs<float> b;
    b.f = make_fit_args<float>(n, ld, state_in, cov_in, charge_in, hit_offsets, hit_layer, hit_valid, n_hits, hit_pos,
                               hit_cov, nullptr, state_out, cov_out, charge_out, chi2, ndf, nullptr, 1, 0, trk_status,
                               ctx->d_counter);
    b.f.max_len = max_len;
    b.fwd_status = fwd_status;
    b.cov_scale = float(cov_scale);
    b.fwd_ckpt = (const float*)fwd_checkpoints;
    b.n_seg_f = n_seg_f;
    b.smooth_state = (float*)smooth_state;
    b.smooth_cov = (float*)smooth_cov;
    e = kf::launch_backward(b, g, s);
  } else {
    kf::BwdArgs<double> b;
    b.f = make_fit_args<double>(n, ld, state_in, cov_in, charge_in, hit_offsets, hit_layer, hit_valid, n_hits,
                                hit_pos, hit_cov, nullptr, state_out, cov_out, charge_out, chi2, ndf, nullptr, 1, 0,
                                trk_status, ctx->d_counter);
    b.f.max_len = max_len;
    b.fwd_status = fwd_status;
    b.cov_scale = cov_scale;
    b.fwd_ckpt = (const double*)fwd_checkpoints;
    b.n_seg_f = n_seg_f;
    b.smooth_state = (double*)smooth_state;
    b.smooth_cov = (double*)smooth_cov;
    e = kf::launch_backward(b, g, s);
  }
  if (e != hipSuccess) return hip_fail(e, name);
  return ok();
}

}  // namespace

extern "C" {

int kf_backward_fit(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* state_in,
                    const void* cov_in, const int8_t* charge_in, const uint32_t* fwd_status,
                    const int32_t* hit_offsets, const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits,
                    const void* hit_pos, const void* hit_cov, const kf_geometry* geom, double cov_scale,
                    int32_t max_len, void* state_out, void* cov_out, int8_t* charge_out, void* chi2, int32_t* ndf,
                    uint32_t* trk_status, void* stream) {
  KF_RANGE();
  return backward_impl(ctx, prec, n, ld, state_in, cov_in, charge_in, fwd_status, nullptr, hit_offsets, hit_layer,
                       hit_valid, n_hits, hit_pos, hit_cov, geom, cov_scale, max_len, state_out, cov_out, charge_out,
                       chi2, ndf, trk_status, nullptr, nullptr, "kf_backward_fit", stream);
}

int kf_smooth_tracks(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* state_in,
                     const void* cov_in, const int8_t* charge_in, const uint32_t* fwd_status,
                     const void* fwd_checkpoints, const int32_t* hit_offsets, const int16_t* hit_layer,
                     const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, const void* hit_cov,
                     const kf_geometry* geom, double cov_scale, int32_t max_len, void* state_out, void* cov_out,
                     int8_t* charge_out, void* chi2, int32_t* ndf, uint32_t* trk_status, void* smooth_state,
                     void* smooth_cov, void* stream) {
  KF_RANGE();
  if (!fwd_checkpoints || !smooth_state || !smooth_cov)
    return fail(KF_ERR_ARG, "kf_smooth_tracks needs fwd_checkpoints, smooth_state and smooth_cov");
  return backward_impl(ctx, prec, n, ld, state_in, cov_in, charge_in, fwd_status, fwd_checkpoints, hit_offsets,
                       hit_layer, hit_valid, n_hits, hit_pos, hit_cov, geom, cov_scale, max_len, state_out, cov_out,
                       charge_out, chi2, ndf, trk_status, smooth_state, smooth_cov, "kf_smooth_tracks", stream);
}

int kf_remove_duplicates(kf_ctx* ctx, int64_t n, const int32_t* track_hits, int64_t hit_stride, int32_t n_layers,
                         const float* score, int64_t score_stride, float frac, uint8_t* keep, int32_t* dup_of,
                         void* stream) {
  KF_RANGE();
  if (n < 0) return fail(KF_ERR_ARG, "n = %lld < 0", (long long)n);
  if (n_layers < 1 || n_layers > 64) return fail(KF_ERR_ARG, "n_layers = %d outside [1, 64]", n_layers);
  if (hit_stride < n_layers) return fail(KF_ERR_ARG, "hit_stride = %lld < n_layers", (long long)hit_stride);
  if (score_stride < 1) return fail(KF_ERR_ARG, "score_stride = %lld < 1", (long long)score_stride);
  if (!(frac > 0.0f && frac <= 1.0f)) return fail(KF_ERR_ARG, "frac must be in (0, 1]");
  if (n * int64_t(n_layers) >= (int64_t(1) << 31)) return fail(KF_ERR_ARG, "n * n_layers must be < 2^31");
  if (n == 0) return ok();
  KF_REQUIRE(ctx);
  KF_REQUIRE(track_hits);
  KF_REQUIRE(score);
  KF_REQUIRE(keep);
  const size_t need = kf::dedup_workspace_bytes(n, n_layers);
  if (need > ctx->dedup_bytes) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    if (ctx->dedup_mem) hipFree(ctx->dedup_mem);
    ctx->dedup_mem = nullptr;
    ctx->dedup_bytes = 0;
    hipError_t e = hipMalloc(&ctx->dedup_mem, need);
    hipSetDevice(prev);
    if (e != hipSuccess) {
      ctx->dedup_mem = nullptr;
      return fail(KF_ERR_NOMEM, "kf_remove_duplicates: %zu bytes: %s", need, hipGetErrorString(e));
    }
    ctx->dedup_bytes = need;
  }
  kf::DedupArgs a{n, track_hits, hit_stride, n_layers, score, score_stride, frac, keep, dup_of};
  hipError_t e = kf::launch_dedup(a, ctx->dedup_mem, ctx->dedup_bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "kf_remove_duplicates");
  return ok();
}

int kf_reserve(kf_ctx* ctx, int64_t max_tracks, int32_t max_len) {
  KF_RANGE();
  if (max_tracks < 0) return fail(KF_ERR_ARG, "max_tracks = %lld < 0", (long long)max_tracks);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  KF_REQUIRE(ctx);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(ctx->device);
  // captured fit graphs point into the old workspace
  for (int i = 0; i < 2; ++i) {
    if (ctx->exec[i]) hipGraphExecDestroy(ctx->exec[i]);
    ctx->exec[i] = nullptr;
    ctx->key[i].clear();
  }
  if (ctx->work_mem) {
    hipFree(ctx->work_mem);
    ctx->work_mem = nullptr;
  }
  ctx->work = kf::PackWork{};
  if (max_tracks == 0) {
    hipSetDevice(prev);
    return ok();
  }
  const int64_t n_tiles = (max_tracks + kf::kTile - 1) / kf::kTile;
  const int64_t cap = n_tiles * kf::kTile * max_len;
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t b_hist = up(int64_t(kf::kMaxLen + 2) * 4), b_order = up(max_tracks * 4);
  const int64_t b_tiles = up((n_tiles + 1) * 8), b_lv = up(cap * 4), b_hit = up(cap * 9 * 8);
  const int64_t total = 2 * b_hist + 2 * b_order + b_tiles + b_lv + b_hit;
  hipError_t e = hipMalloc(&ctx->work_mem, size_t(total));
  hipSetDevice(prev);
  if (e != hipSuccess) {
    ctx->work_mem = nullptr;
    return fail(KF_ERR_NOMEM, "kf_reserve: %lld bytes: %s", (long long)total, hipGetErrorString(e));
  }
  char* p = (char*)ctx->work_mem;
  kf::PackWork& w = ctx->work;
  w.hist = (int32_t*)p;
  p += b_hist;
  w.cursor = (int32_t*)p;
  p += b_hist;
  w.order = (int32_t*)p;
  p += b_order;
  w.slot_of = (int32_t*)p;
  p += b_order;
  w.tile_base = (int64_t*)p;
  p += b_tiles;
  w.lv = (int32_t*)p;
  p += b_lv;
  w.hit = (void*)p;
  w.cap = cap;
  w.max_tracks = max_tracks;
  w.max_len = max_len;
  return ok();
}

int kf_set_fit_launch(kf_ctx* ctx, kf_precision prec, int32_t block, int32_t persistent, int32_t blocks_per_cu,
                      int32_t waves, int32_t layout) {
  KF_TRY(check_prec(prec));
  if (waves != 1 && waves != 2) return fail(KF_ERR_ARG, "waves = %d (1 or 2)", waves);
  if (layout < 0 || layout > 4) return fail(KF_ERR_ARG, "layout = %d (0 to 4)", layout);
  if (block < 64 || block > 256 || block % 64 != 0) return fail(KF_ERR_ARG, "block = %d (64, 128, 192 or 256)", block);
  if (persistent != 0 && persistent != 1) return fail(KF_ERR_ARG, "persistent must be 0 or 1");
  if (blocks_per_cu < 1 || blocks_per_cu > 32) return fail(KF_ERR_ARG, "blocks_per_cu = %d outside [1, 32]", blocks_per_cu);
  KF_REQUIRE(ctx);
  ctx->fit[prec == KF_F32 ? 0 : 1] = kf::FitLaunch{block, persistent, blocks_per_cu, waves, layout};
  return ok();
}

int kf_get_fit_launch(const kf_ctx* ctx, kf_precision prec, int32_t* block, int32_t* persistent,
                      int32_t* blocks_per_cu, int32_t* waves, int32_t* layout) {
  KF_TRY(check_prec(prec));
  KF_REQUIRE(ctx);
  KF_REQUIRE(block);
  KF_REQUIRE(persistent);
  KF_REQUIRE(blocks_per_cu);
  KF_REQUIRE(waves);
  KF_REQUIRE(layout);
  const kf::FitLaunch& l = ctx->fit[prec == KF_F32 ? 0 : 1];
  *block = l.block;
  *persistent = l.persistent;
  *blocks_per_cu = l.blocks_per_cu;
  *waves = l.waves;
  *layout = l.layout;
  return ok();
}

int kf_device_cu_count(const kf_ctx* ctx, int32_t* n_cu) {
  KF_REQUIRE(ctx);
  KF_REQUIRE(n_cu);
  *n_cu = ctx->n_cu;
  return ok();
}

int kf_score_hits(kf_ctx* ctx, int64_t n, int64_t ld, const float* seed_state, const float* seed_cov,
                  const int8_t* seed_charge, const int16_t* seed_layer, const int16_t* layer_plan, int32_t plan_len,
                  const kf_geometry* geom, const kf_search_params* prm, const int32_t* pool_layer_offsets,
                  int64_t n_pool, const float* pool_pos, const float* pool_cov, const int32_t* pool_hit_id,
                  const int32_t* pool_module, int32_t* cand_hits, int32_t* cand_overlap, float* cand_score,
                  float* cand_state, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  KF_REQUIRE(prm);
  if (prm->beam < 1 || prm->beam > kf::kMaxBeam) return fail(KF_ERR_ARG, "beam = %d outside [1, %d]", prm->beam, kf::kMaxBeam);
  if (!(prm->chi2_max > 0.f) || !std::isfinite(prm->chi2_max)) return fail(KF_ERR_ARG, "chi2_max must be finite and > 0");
  if (!(prm->n_sigma > 0.f) || !std::isfinite(prm->n_sigma)) return fail(KF_ERR_ARG, "n_sigma must be finite and > 0");
  if (!std::isfinite(prm->hit_bonus)) return fail(KF_ERR_ARG, "hit_bonus must be finite");
  if (!(prm->miss_penalty >= 0.f) || !std::isfinite(prm->miss_penalty)) return fail(KF_ERR_ARG, "miss_penalty must be >= 0");
  if (prm->max_miss < 0 || prm->max_miss > 100) return fail(KF_ERR_ARG, "max_miss = %d outside [0, 100]", prm->max_miss);
  if (!(prm->sigma_rphi >= 0.f) || !(prm->sigma_z >= 0.f)) return fail(KF_ERR_ARG, "sigma_rphi / sigma_z must be >= 0");
  if (prm->overlap != 0 && prm->overlap != 1) return fail(KF_ERR_ARG, "overlap = %d (0 off, 1 on)", prm->overlap);
  if (prm->overlap && !std::isfinite(prm->overlap_bonus)) return fail(KF_ERR_ARG, "overlap_bonus must be finite");
  KF_REQUIRE(prm->win_min_rphi);
  KF_REQUIRE(prm->win_max_rphi);
  KF_REQUIRE(prm->win_min_z);
  KF_REQUIRE(prm->win_max_z);
  const int nl = geom->n_layers;
  for (int l = 0; l < nl; ++l) {
    if (!(prm->win_min_rphi[l] > 0.f) || !(prm->win_min_rphi[l] <= prm->win_max_rphi[l]) ||
        !std::isfinite(prm->win_max_rphi[l]) || !(prm->win_min_z[l] > 0.f) ||
        !(prm->win_min_z[l] <= prm->win_max_z[l]) || !std::isfinite(prm->win_max_z[l]))
      return fail(KF_ERR_ARG, "window limits of layer %d invalid (need 0 < min <= max)", l);
  }
  if (plan_len < 1 || plan_len > 64) return fail(KF_ERR_ARG, "plan_len = %d outside [1, 64]", plan_len);
  KF_REQUIRE(layer_plan);
  for (int k = 0; k < plan_len; ++k) {
    const int L = layer_plan[k];
    if (L < 0 || L >= nl) return fail(KF_ERR_ARG, "layer_plan[%d] = %d is not a layer", k, L);
    if (g.kind[L] != 0) return fail(KF_ERR_ARG, "layer_plan[%d] = %d is not a barrel layer", k, L);
  }
  KF_REQUIRE(pool_layer_offsets);
  if (n_pool < 0 || n_pool >= (int64_t(1) << 31)) return fail(KF_ERR_ARG, "n_pool = %lld outside [0, 2^31)", (long long)n_pool);
  if (pool_layer_offsets[0] != 0 || pool_layer_offsets[nl] != n_pool)
    return fail(KF_ERR_ARG, "pool_layer_offsets must start at 0 and end at n_pool");
  for (int l = 0; l < nl; ++l)
    if (pool_layer_offsets[l + 1] < pool_layer_offsets[l]) return fail(KF_ERR_ARG, "pool_layer_offsets decrease at %d", l);
  KF_REQUIRE(ctx);
  if (n == 0) return ok();
  KF_REQUIRE(seed_state);
  KF_REQUIRE(seed_cov);
  KF_REQUIRE(seed_charge);
  KF_REQUIRE(seed_layer);
  KF_REQUIRE(cand_hits);
  KF_REQUIRE(cand_score);
  KF_REQUIRE(trk_status);
  if (n_pool > 0) {
    KF_REQUIRE(pool_pos);
    KF_REQUIRE(pool_cov);
    KF_REQUIRE(pool_hit_id);
    if (prm->overlap) KF_REQUIRE(pool_module);
  }
  // bins of every layer
  kf::BinTable t;
  std::memset(&t, 0, sizeof(t));
  t.n_layers = nl;
  int64_t n_bins = 0;
  for (int l = 0; l <= nl; ++l) t.off[l] = pool_layer_offsets[l];
  for (int l = 0; l < nl; ++l) {
    int64_t np = 1, nz = 1;
    const bool used = pool_layer_offsets[l + 1] > pool_layer_offsets[l];
    if (g.kind[l] == 0 && used) {
      np = std::max<int64_t>(1, int64_t(std::ceil(2.0 * M_PI * geom->pos[l] / kf::kBinArc)));
      nz = std::max<int64_t>(1, int64_t(std::ceil((geom->hi[l] - geom->lo[l]) / kf::kBinZ)));
    }
    t.base[l] = int32_t(n_bins);
    t.nphi[l] = int32_t(np);
    t.nz[l] = int32_t(nz);
    t.lo[l] = float(geom->lo[l]);
    t.hi[l] = float(geom->hi[l]);
    if (!(t.hi[l] > t.lo[l])) t.hi[l] = t.lo[l] + 1.f;
    n_bins += np * nz;
    if (n_bins >= (int64_t(1) << 31)) return fail(KF_ERR_ARG, "too many pool bins (layer %d)", l);
  }
  // workspace
  const int64_t S = n * prm->beam, P = plan_len;
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t nsum = n_bins / 2048 + 2;
  const int64_t b_bins = up(n_bins * 4), b_pool4 = up(n_pool * 4), b_sum = up(nsum * 4) + 256;
  const int64_t b_pool = up(n_pool * int64_t(sizeof(kf::PoolHit))) + up((n_bins + 1) * 4);
  const int64_t b_slot = up(P * S) + 2 * up(P * S * 4) +
                         up(P * int64_t(sizeof(kf::SearchLayer)));
  const int64_t total = b_bins + 2 * b_pool4 + b_sum + b_pool + b_slot;
  if (size_t(total) > ctx->search_bytes) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    if (ctx->search_mem) hipFree(ctx->search_mem);
    ctx->search_mem = nullptr;
    ctx->search_bytes = 0;
    ctx->bins_key.clear();
    hipError_t e = hipMalloc(&ctx->search_mem, size_t(total));
    hipSetDevice(prev);
    if (e != hipSuccess) {
      ctx->search_mem = nullptr;
      return fail(KF_ERR_NOMEM, "kf_score_hits: %lld bytes: %s", (long long)total, hipGetErrorString(e));
    }
    ctx->search_bytes = size_t(total);
  }
  // identity of the binned pool: pointers, sizes, layer offsets, bin table
  const int32_t* module = prm->overlap ? pool_module : nullptr;
  std::vector<unsigned char> key(4 * sizeof(void*) + sizeof(n_pool) + sizeof(t));
  {
    unsigned char* k = key.data();
    const void* ptrs[4] = {pool_pos, pool_cov, pool_hit_id, module};
    std::memcpy(k, ptrs, sizeof(ptrs));
    std::memcpy(k + sizeof(ptrs), &n_pool, sizeof(n_pool));
    std::memcpy(k + sizeof(ptrs) + sizeof(n_pool), &t, sizeof(t));
  }
  const bool rebin = !(prm->reuse_bins == 1 && key == ctx->bins_key);
  char* q = (char*)ctx->search_mem;
  auto take = [&q](int64_t b) {
    char* r = q;
    q += b;
    return (void*)r;
  };
  kf::SearchWork w;
  w.count = (int32_t*)take(b_bins);
  w.bin_of = (int32_t*)take(b_pool4);
  w.rank = (int32_t*)take(b_pool4);
  w.block_sum = (int32_t*)take(up(nsum * 4));
  w.total = (int32_t*)take(256);
  w.pool.hits = (kf::PoolHit*)take(up(n_pool * int64_t(sizeof(kf::PoolHit))));
  w.pool.bin_off = (int32_t*)take(up((n_bins + 1) * 4));
  kf::SearchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.ld = ld;
  a.beam = prm->beam;
  a.plan_len = plan_len;
  a.seed_state = seed_state;
  a.seed_cov = seed_cov;
  a.seed_charge = seed_charge;
  a.seed_layer = seed_layer;
  a.chi2_max = prm->chi2_max;
  a.n_sigma = prm->n_sigma;
  a.hit_bonus = prm->hit_bonus;
  a.miss_penalty = prm->miss_penalty;
  a.max_miss = prm->max_miss;
  a.bz = float(geom->bz_tesla);
  a.mass = float(geom->particle_mass_gev);
  a.pool = w.pool.hits;
  a.bin_off = w.pool.bin_off;
  a.n_pool = n_pool;
  a.hist_parent = (int8_t*)take(up(P * S));
  a.hist_id = (int32_t*)take(up(P * S * 4));
  a.hist_ovl = (int32_t*)take(up(P * S * 4));
  kf::SearchLayer* d_layers = (kf::SearchLayer*)take(up(P * int64_t(sizeof(kf::SearchLayer))));
  a.overlap = prm->overlap;
  a.overlap_bonus = prm->overlap_bonus;
  a.cand_ovl = cand_overlap;
  a.status = trk_status;
  a.cand_hits = cand_hits;
  a.cand_score = cand_score;
  a.cand_state = cand_state;
  std::vector<kf::SearchLayer> layers(plan_len);
  for (int k = 0; k < plan_len; ++k) {
    const int L = layer_plan[k];
    kf::SearchLayer& sl = layers[k];
    sl.layer = L;
    sl.prev_layer = k > 0 ? layer_plan[k - 1] : -1;
    sl.R = float(geom->pos[L]);
    sl.x0 = float(geom->x_over_x0[L]);
    sl.base = t.base[L];
    sl.nphi = t.nphi[L];
    sl.nz = t.nz[L];
    sl.lo = t.lo[L];
    sl.hi = t.hi[L];
    sl.wmin_r = prm->win_min_rphi[L];
    sl.wmax_r = prm->win_max_rphi[L];
    sl.wmin_z = prm->win_min_z[L];
    sl.wmax_z = prm->win_max_z[L];
    sl.sig_r = prm->sigma_rphi;
    sl.sig_z = prm->sigma_z;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (rebin) {
    ctx->bins_key.clear();
    e = kf::launch_bin_pool(t, pool_pos, pool_cov, pool_hit_id, module, n_pool, n_bins, w, s);
    if (e == hipSuccess) ctx->bins_key = key;
  }
  if (e == hipSuccess) e = kf::launch_search(a, layers.data(), d_layers, s);
  if (e != hipSuccess) return hip_fail(e, "kf_score_hits");
  return ok();
}

}  // extern "C"

namespace {

// Sub-buffers of the final fit's workspace, 256-byte aligned.
struct FinalWork {
  void *f_state, *f_cov, *f_chi2, *b_state, *b_cov, *b_chi2, *ckpt, *sm_state, *sm_cov, *seed_state, *chi2_work;
  int32_t *f_ndf, *b_ndf;
  uint32_t *f_status, *b_status;
  int8_t *f_charge, *b_charge, *seed_charge;
  uint8_t *used, *open;
  // the sub-batch of the open tracks after the first round
  int32_t *flag, *len, *pos, *epos, *map, *sub_offsets, *counts;
  int16_t* sub_layer;
  uint8_t* sub_used;
  void *sub_pos, *sub_cov, *scan_temp;
  size_t scan_bytes;
};

size_t final_layout(int64_t n, int64_t n_hits, int32_t max_len, size_t esz, unsigned char* base, FinalWork* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  const size_t N = size_t(n), nseg = size_t(max_len > 1 ? max_len - 1 : 1);
  FinalWork x;
  x.f_state = take(6 * N * esz);
  x.f_cov = take(21 * N * esz);
  x.f_chi2 = take(N * esz);
  x.b_state = take(6 * N * esz);
  x.b_cov = take(21 * N * esz);
  x.b_chi2 = take(N * esz);
  x.ckpt = take(28 * N * nseg * esz);
  x.sm_state = take(6 * N * size_t(max_len) * esz);
  x.sm_cov = take(21 * N * size_t(max_len) * esz);
  x.seed_state = take(6 * N * esz);
  x.chi2_work = take(size_t(n_hits) * esz);
  x.f_ndf = (int32_t*)take(N * 4);
  x.b_ndf = (int32_t*)take(N * 4);
  x.f_status = (uint32_t*)take(N * 4);
  x.b_status = (uint32_t*)take(N * 4);
  x.f_charge = (int8_t*)take(N);
  x.b_charge = (int8_t*)take(N);
  x.seed_charge = (int8_t*)take(N);
  x.used = (uint8_t*)take(size_t(n_hits));
  x.open = (uint8_t*)take(N);
  x.flag = (int32_t*)take(N * 4);
  x.len = (int32_t*)take(N * 4);
  x.pos = (int32_t*)take(N * 4);
  x.epos = (int32_t*)take(N * 4);
  x.map = (int32_t*)take(N * 4);
  x.sub_offsets = (int32_t*)take((N + 1) * 4);
  x.counts = (int32_t*)take(2 * 4);
  x.sub_layer = (int16_t*)take(size_t(n_hits) * 2);
  x.sub_used = (uint8_t*)take(size_t(n_hits));
  x.sub_pos = take(3 * size_t(n_hits) * esz);
  x.sub_cov = take(6 * size_t(n_hits) * esz);
  // hipCUB's exclusive scan over n int32 (its storage does not depend on T)
  kf::GatherArgs<float> q{};
  q.n = n;
  kf::launch_final_gather(q, nullptr);
  x.scan_bytes = q.scan_bytes;
  x.scan_temp = take(x.scan_bytes > 0 ? x.scan_bytes : 1);
  if (w) *w = x;
  return off;
}

// The rounds of kf_final_fit in type T: set-up, then per round the fused
// seeding and forward fit over the used hits (with its seeds and its filtered
// state after every entry), the backward fit storing its prediction at every
// entry, the unbiased chi2 of every used hit (entry-parallel) and the
// round's decisions.
// The first round runs on the caller's batch.  After each round the tracks
// still open are gathered, with their used hits, into a compact sub-batch
// (the map keeps each one's index in the caller's batch, where the round's
// decisions and outputs are written), and the host waits for the stream to
// read their count: the next round is launched on that many tracks only, and
// none when the count is 0.
template <typename T>
hipError_t final_rounds(kf_ctx* ctx, int pi, int64_t n, int64_t ld, int32_t seed_mode, const int32_t* hit_offsets,
                        const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                        const void* hit_cov, const kf::GeomArgs& g, double cov_scale, double chi2_cut,
                        int32_t max_reject, int32_t min_keep, int32_t max_len, void* state_out, void* cov_out,
                        int8_t* charge_out, void* chi2, int32_t* ndf, uint32_t* trk_status, uint8_t* outlier,
                        void* hit_chi2, const FinalWork& w, hipStream_t s) {
  kf::FinalRoundArgs<T> r;
  std::memset(&r, 0, sizeof(r));
  r.n = n;
  r.ld = ld;
  r.hit_offsets = hit_offsets;
  r.hit_layer = hit_layer;
  r.hit_valid = hit_valid;
  r.hit_pos = (const T*)hit_pos;
  r.hit_cov = (const T*)hit_cov;
  r.n_hits = n_hits;
  r.max_len = max_len;
  r.max_reject = max_reject;
  r.min_keep = min_keep;
  r.chi2_cut = chi2_cut;
  r.used = w.used;
  r.open = w.open;
  r.outlier = outlier;
  r.hit_chi2 = (T*)hit_chi2;
  r.chi2_work = (T*)w.chi2_work;
  r.seed_state = (const T*)w.seed_state;
  r.seed_charge = w.seed_charge;
  r.ckpt = (const T*)w.ckpt;
  r.pred_state = (const T*)w.sm_state;
  r.pred_cov = (const T*)w.sm_cov;
  r.b_state = (const T*)w.b_state;
  r.b_cov = (const T*)w.b_cov;
  r.b_charge = w.b_charge;
  r.b_chi2 = (const T*)w.b_chi2;
  r.b_ndf = w.b_ndf;
  r.b_status = w.b_status;
  r.state_out = (T*)state_out;
  r.cov_out = (T*)cov_out;
  r.charge_out = charge_out;
  r.chi2_out = (T*)chi2;
  r.ndf_out = ndf;
  r.status_out = trk_status;
  r.map = nullptr;
  r.orig_offsets = hit_offsets;
  r.used_orig = w.used;
  r.open_orig = w.open;
  hipError_t e = kf::launch_final_init(r, s);
  const kf::FitLaunch l = ctx->fit[pi];
  const int32_t n_seg = max_len > 1 ? max_len - 1 : 1;
  // the batch a round runs on: the caller's tracks in the first round, then
  // the sub-batch of those still open (the same hits, compacted)
  int64_t nb = n;
  const int32_t* b_off = hit_offsets;
  const int16_t* b_lay = hit_layer;
  uint8_t* b_used = w.used;
  const void* b_pos = hit_pos;
  const void* b_cov = hit_cov;
  for (int32_t round = 0; round <= max_reject && e == hipSuccess; ++round) {
    const bool room = ctx->work.cap > 0 && nb <= ctx->work.max_tracks && max_len <= ctx->work.max_len;
    const int layout = room || l.layout == 3 ? l.layout : (l.layout == 4 ? 3 : 0);
    auto f = make_fit_args<T>(nb, nb, nullptr, nullptr, nullptr, b_off, b_lay, b_used, n_hits, b_pos, b_cov,
                              nullptr, w.f_state, w.f_cov, w.f_charge, w.f_chi2, w.f_ndf, w.ckpt, 1, n_seg,
                              w.f_status, ctx->d_counter);
    f.max_len = max_len;
    f.make_seeds = seed_mode + 1;
    f.seed_state_out = (T*)w.seed_state;
    f.seed_charge_out = w.seed_charge;
    // the later rounds' few open tracks: one wave per block (here and in the
    // backward pass), so that each wave has a compute unit to itself
    kf::FitLaunch lr = l;
    if (round > 0 && !l.persistent) lr.block = 64;
    e = run_fit(ctx, f, g, lr, layout, s, false);
    if (e != hipSuccess) break;
    kf::BwdArgs<T> b;
    b.f = make_fit_args<T>(nb, nb, w.f_state, w.f_cov, w.f_charge, b_off, b_lay, b_used, n_hits, b_pos, b_cov,
                           nullptr, w.b_state, w.b_cov, w.b_charge, w.b_chi2, w.b_ndf, nullptr, 1, 0, w.b_status,
                           ctx->d_counter);
    b.f.max_len = max_len;
    b.fwd_status = w.f_status;
    b.cov_scale = T(cov_scale);
    b.fwd_ckpt = (const T*)w.ckpt;
    b.n_seg_f = n_seg;
    b.smooth_state = (T*)w.sm_state;
    b.smooth_cov = (T*)w.sm_cov;
    e = kf::launch_backward_predictions(b, g, s, round > 0 ? 64 : 256);
    if (e != hipSuccess) break;
    r.n = nb;
    r.hit_offsets = b_off;
    r.hit_layer = b_lay;
    r.hit_pos = (const T*)b_pos;
    r.hit_cov = (const T*)b_cov;
    r.used = b_used;
    r.round = round;
    e = kf::launch_final_chi2(r, g, s);
    if (e != hipSuccess) break;
    e = kf::launch_final_round(r, s);
    if (e != hipSuccess || round == max_reject) break;
    // the tracks still open, gathered for the next round (the host needs
    // their count to size the next round's launches)
    kf::GatherArgs<T> ga{};
    ga.n = n;
    ga.hit_offsets = hit_offsets;
    ga.hit_layer = hit_layer;
    ga.used = w.used;
    ga.hit_pos = (const T*)hit_pos;
    ga.hit_cov = (const T*)hit_cov;
    ga.n_hits = n_hits;
    ga.open = w.open;
    ga.flag = w.flag;
    ga.len = w.len;
    ga.pos = w.pos;
    ga.epos = w.epos;
    ga.map = w.map;
    ga.sub_offsets = w.sub_offsets;
    ga.sub_layer = w.sub_layer;
    ga.sub_used = w.sub_used;
    ga.sub_pos = (T*)w.sub_pos;
    ga.sub_cov = (T*)w.sub_cov;
    ga.counts = w.counts;
    ga.scan_temp = w.scan_temp;
    ga.scan_bytes = w.scan_bytes;
    e = kf::launch_final_gather(ga, s);
    if (e != hipSuccess) break;
    int32_t* counts = ctx->final_counts;
    e = hipMemcpyAsync(counts, w.counts, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || counts[0] == 0) break;
    nb = counts[0];
    b_off = w.sub_offsets;
    b_lay = w.sub_layer;
    b_used = w.sub_used;
    b_pos = w.sub_pos;
    b_cov = w.sub_cov;
    r.open = nullptr;   // every track of the sub-batch is open
    r.map = w.map;
  }
  return e;
}

}  // namespace

extern "C" {

int kf_final_fit(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, int32_t seed_mode, const int32_t* hit_offsets,
                 const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                 const void* hit_cov, const kf_geometry* geom, double cov_scale, double chi2_cut, int32_t max_reject,
                 int32_t min_keep, int32_t max_len, void* state_out, void* cov_out, int8_t* charge_out, void* chi2,
                 int32_t* ndf, uint32_t* trk_status, uint8_t* outlier, void* hit_chi2, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (seed_mode != 0 && seed_mode != 1) return fail(KF_ERR_ARG, "seed mode %d unknown (0 first three, 1 spaced)", seed_mode);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  if (!std::isfinite(cov_scale) || !(cov_scale >= 1.0)) return fail(KF_ERR_ARG, "cov_scale must be finite and >= 1");
  if (!(chi2_cut > 0.0)) return fail(KF_ERR_ARG, "chi2_cut must be > 0");
  if (max_reject < 0 || max_reject > kf::kMaxLen) return fail(KF_ERR_ARG, "max_reject = %d outside [0, %d]", max_reject, kf::kMaxLen);
  if (min_keep < 3 || min_keep > kf::kMaxLen) return fail(KF_ERR_ARG, "min_keep = %d outside [3, %d]", min_keep, kf::kMaxLen);
  if (n == 0) return ok();
  KF_REQUIRE(ctx);
  KF_REQUIRE(hit_offsets);
  KF_REQUIRE(hit_layer);
  KF_REQUIRE(hit_valid);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(hit_cov);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(charge_out);
  KF_REQUIRE(chi2);
  KF_REQUIRE(ndf);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(outlier);
  const size_t esz = prec == KF_F32 ? 4 : 8;
  const size_t need = final_layout(n, n_hits, max_len, esz, nullptr, nullptr);
  if (need > ctx->final_bytes) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    if (ctx->final_mem) hipFree(ctx->final_mem);
    ctx->final_mem = nullptr;
    ctx->final_bytes = 0;
    hipError_t e = hipMalloc(&ctx->final_mem, need);
    hipSetDevice(prev);
    if (e != hipSuccess) {
      ctx->final_mem = nullptr;
      return fail(KF_ERR_NOMEM, "kf_final_fit: %zu bytes: %s", need, hipGetErrorString(e));
    }
    ctx->final_bytes = need;
  }
  if (!ctx->final_counts) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    hipError_t e = hipHostMalloc((void**)&ctx->final_counts, 2 * sizeof(int32_t), hipHostMallocDefault);
    hipSetDevice(prev);
    if (e != hipSuccess) {
      ctx->final_counts = nullptr;
      return fail(KF_ERR_NOMEM, "kf_final_fit: pinned count: %s", hipGetErrorString(e));
    }
  }
  FinalWork w;
  final_layout(n, n_hits, max_len, esz, (unsigned char*)ctx->final_mem, &w);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = prec == KF_F32
                     ? final_rounds<float>(ctx, 0, n, ld, seed_mode, hit_offsets, hit_layer, hit_valid, n_hits,
                                           hit_pos, hit_cov, g, cov_scale, chi2_cut, max_reject, min_keep, max_len,
                                           state_out, cov_out, charge_out, chi2, ndf, trk_status, outlier, hit_chi2,
                                           w, s)
                     : final_rounds<double>(ctx, 1, n, ld, seed_mode, hit_offsets, hit_layer, hit_valid, n_hits,
                                            hit_pos, hit_cov, g, cov_scale, chi2_cut, max_reject, min_keep, max_len,
                                            state_out, cov_out, charge_out, chi2, ndf, trk_status, outlier, hit_chi2,
                                            w, s);
  if (e != hipSuccess) return hip_fail(e, "kf_final_fit");
  return ok();
}

}  // extern "C"

namespace {

// kf_fit_adjoint and kf_fit_adjoint_noalloc: the block partials of the
// alignment reduction go to the context-owned buffer (grown on demand) or to
// the fixed scratch array (no allocation, bounded size).
int fit_adjoint_impl(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                   const void* seed_cov, const int8_t* seed_charge, const int32_t* hit_offsets,
                   const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                   const void* hit_cov, const kf_geometry* geom, const void* align, const void* checkpoints,
                   int32_t seg, int32_t max_len, const void* dL_dchi2, void* grad_seed, void* grad_hit_pos,
                   void* grad_align, const uint32_t* trk_status, void* stream, bool no_alloc) {
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (seg < 1) return fail(KF_ERR_ARG, "seg = %d < 1", seg);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  KF_REQUIRE(ctx);
  if (n > 0) {
    KF_REQUIRE(seed_state);
    KF_REQUIRE(seed_cov);
    KF_REQUIRE(seed_charge);
    KF_REQUIRE(hit_offsets);
    KF_REQUIRE(hit_layer);
    KF_REQUIRE(hit_valid);
    KF_REQUIRE(hit_pos);
    KF_REQUIRE(hit_cov);
    KF_REQUIRE(checkpoints);
    KF_REQUIRE(grad_seed);
    KF_REQUIRE(grad_hit_pos);
    KF_REQUIRE(trk_status);
  } else if (!grad_align) {
    return ok();
  }
  if (grad_align && n_hits > 0) {
    KF_REQUIRE(hit_layer);
    KF_REQUIRE(hit_valid);
    KF_REQUIRE(hit_pos);
    KF_REQUIRE(grad_hit_pos);
  }
  int32_t n_seg = (max_len - 1 + seg - 1) / seg;
  if (n_seg < 1) n_seg = 1;
  hipStream_t s = (hipStream_t)stream;
  const size_t esz = prec == KF_F32 ? 4 : 8;
  void* partial = nullptr;
  if (grad_align && no_alloc) {
    const size_t need = size_t(kf::adjoint_partial_blocks(n_hits)) * 2 * kf::kMaxLayers * esz;
    if (need > kScratchBytes)
      return fail(KF_ERR_ARG,
                  "kf_fit_adjoint_noalloc: n_hits = %lld needs %zu bytes of scratch, more than its fixed %zu "
                  "(at most %lld hits in %s)",
                  (long long)n_hits, need, kScratchBytes,
                  (long long)(kScratchBytes / (2 * kf::kMaxLayers * esz)) * kf::kAlignPerBlock,
                  prec == KF_F32 ? "FP32" : "FP64");
    if (!ctx->scratch) return fail(KF_ERR_DEVICE, "kf_fit_adjoint_noalloc: no scratch address for this context");
    partial = ctx->scratch;
  }
  void* seg_buf = nullptr;
  if (!no_alloc) {
    // the alignment partials, then (seg > 1) the buffer of one checkpoint
    // segment's states per track
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t need_part = grad_align ? up(size_t(kf::adjoint_partial_blocks(n_hits)) * 2 * kf::kMaxLayers * esz) : 0;
    const size_t need_seg = seg > 1 && max_len > 1 ? up(size_t(n) * size_t(max_len - 1) * kf::kSegVals * esz) : 0;
    const size_t need = need_part + need_seg;
    if (need > ctx->red_bytes) {
      int prev = 0;
      hipGetDevice(&prev);
      hipSetDevice(ctx->device);
      if (ctx->red_mem) hipFree(ctx->red_mem);
      ctx->red_mem = nullptr;
      ctx->red_bytes = 0;
      hipError_t e = hipMalloc(&ctx->red_mem, need);
      hipSetDevice(prev);
      if (e != hipSuccess) {
        ctx->red_mem = nullptr;
        return fail(KF_ERR_NOMEM, "kf_fit_adjoint: %zu bytes: %s", need, hipGetErrorString(e));
      }
      ctx->red_bytes = need;
    }
    if (grad_align) partial = ctx->red_mem;
    if (need_seg) seg_buf = (char*)ctx->red_mem + need_part;
  }
  hipError_t e;
  if (prec == KF_F32) {
    kf::AdjArgs<float> a;
    a.f = make_fit_args<float>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, n_hits,
                               hit_pos, hit_cov, align, nullptr, nullptr, nullptr, nullptr, nullptr,
                               const_cast<void*>(checkpoints), seg, n_seg, nullptr, nullptr);
    a.f.max_len = max_len;
    a.w = (const float*)dL_dchi2;
    a.fwd_status = trk_status;
    a.grad_seed = (float*)grad_seed;
    a.grad_hit = (float*)grad_hit_pos;
    a.grad_align = (float*)grad_align;
    a.partial = (float*)partial;
    a.seg_buf = (float*)seg_buf;
    e = kf::launch_adjoint(a, g, s);
  } else {
    kf::AdjArgs<double> a;
    a.f = make_fit_args<double>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, n_hits,
                                hit_pos, hit_cov, align, nullptr, nullptr, nullptr, nullptr, nullptr,
                                const_cast<void*>(checkpoints), seg, n_seg, nullptr, nullptr);
    a.f.max_len = max_len;
    a.w = (const double*)dL_dchi2;
    a.fwd_status = trk_status;
    a.grad_seed = (double*)grad_seed;
    a.grad_hit = (double*)grad_hit_pos;
    a.grad_align = (double*)grad_align;
    a.partial = (double*)partial;
    a.seg_buf = (double*)seg_buf;
    e = kf::launch_adjoint(a, g, s);
  }
  if (e != hipSuccess) return hip_fail(e, no_alloc ? "kf_fit_adjoint_noalloc" : "kf_fit_adjoint");
  return ok();
}

}  // namespace

extern "C" {

int kf_fit_adjoint(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                   const void* seed_cov, const int8_t* seed_charge, const int32_t* hit_offsets,
                   const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                   const void* hit_cov, const kf_geometry* geom, const void* align, const void* checkpoints,
                   int32_t seg, int32_t max_len, const void* dL_dchi2, void* grad_seed, void* grad_hit_pos,
                   void* grad_align, const uint32_t* trk_status, void* stream) {
  KF_RANGE();
  return fit_adjoint_impl(ctx, prec, n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid,
                          n_hits, hit_pos, hit_cov, geom, align, checkpoints, seg, max_len, dL_dchi2, grad_seed,
                          grad_hit_pos, grad_align, trk_status, stream, false);
}

int kf_fit_adjoint_noalloc(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                           const void* seed_cov, const int8_t* seed_charge, const int32_t* hit_offsets,
                           const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                           const void* hit_cov, const kf_geometry* geom, const void* align, const void* checkpoints,
                           int32_t seg, int32_t max_len, const void* dL_dchi2, void* grad_seed, void* grad_hit_pos,
                           void* grad_align, const uint32_t* trk_status, void* stream) {
  KF_RANGE();
  return fit_adjoint_impl(ctx, prec, n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid,
                          n_hits, hit_pos, hit_cov, geom, align, checkpoints, seg, max_len, dL_dchi2, grad_seed,
                          grad_hit_pos, grad_align, trk_status, stream, true);
}

}  // extern "C"

// ---- tilted planar modules ---------------------------------------------------

namespace {

template <typename T>
int check_plane_geometry(const kf_plane_geometry* g, kf::PlaneGeomArgs<T>* out) {
  if (!g) return fail(KF_ERR_ARG, "plane geometry is NULL");
  if (g->n_modules < 1 || g->n_modules >= (int64_t(1) << 31))
    return fail(KF_ERR_ARG, "plane geometry.n_modules = %lld outside [1, 2^31)", (long long)g->n_modules);
  if (!g->modules) return fail(KF_ERR_ARG, "plane geometry.modules is NULL");
  if (!std::isfinite(g->bz_tesla) || g->bz_tesla == 0.0)
    return fail(KF_ERR_ARG, "plane geometry.bz_tesla must be finite and != 0");
  if (!std::isfinite(g->particle_mass_gev) || !(g->particle_mass_gev > 0.0))
    return fail(KF_ERR_ARG, "plane geometry.particle_mass_gev must be > 0");
  *out = kf::PlaneGeomArgs<T>{(const T*)g->modules, g->n_modules, g->bz_tesla, g->particle_mass_gev};
  return KF_OK;
}

// one launch covers at most 2^31 lanes (the grid's x dimension)
int check_lanes(int64_t n, const char* what) {
  if (n >= (int64_t(1) << 31)) return fail(KF_ERR_ARG, "%s = %lld must be < 2^31", what, (long long)n);
  return KF_OK;
}

template <typename T>
int propagate_plane_impl(int64_t n, int64_t ld, const void* state_in, const void* cov_in, const int8_t* charge,
                         const int32_t* target_module, const kf_plane_geometry* geom, int32_t apply_material,
                         void* state_out, void* cov_out, void* path_len, uint32_t* trk_status, hipStream_t s) {
  kf::PlaneGeomArgs<T> g;
  KF_TRY(check_plane_geometry(geom, &g));
  kf::PlanePropArgs<T> a{n, ld, (const T*)state_in, (const T*)cov_in, charge, target_module, apply_material,
                         (T*)state_out, (T*)cov_out, (T*)path_len, trk_status};
  const hipError_t e = kf::launch_propagate_plane(a, g, s);
  if (e != hipSuccess) return hip_fail(e, "kf_propagate_plane");
  return ok();
}

template <typename T>
int update_plane_impl(int64_t n, int64_t ld, void* state, void* cov, int8_t* charge, const int32_t* module,
                      const void* hit_uv, const void* hit_cov_uv, const kf_plane_geometry* geom, void* chi2,
                      uint32_t* trk_status, hipStream_t s) {
  kf::PlaneGeomArgs<T> g;
  KF_TRY(check_plane_geometry(geom, &g));
  kf::PlaneUpdArgs<T> a{n, ld, (T*)state, (T*)cov, charge, module, (const T*)hit_uv, (const T*)hit_cov_uv,
                        (T*)chi2, trk_status};
  const hipError_t e = kf::launch_update_plane(a, g, s);
  if (e != hipSuccess) return hip_fail(e, "kf_update_plane");
  return ok();
}

template <typename T>
int fit_plane_impl(int64_t n, int64_t ld, const void* seed_state, const void* seed_cov, const int8_t* seed_charge,
                   const int32_t* hit_offsets, const int32_t* hit_module, const uint8_t* hit_valid, int64_t n_hits,
                   const void* hit_uv, const void* hit_cov_uv, const kf_plane_geometry* geom, void* state_out,
                   void* cov_out, int8_t* charge_out, void* chi2, int32_t* ndf, uint32_t* trk_status,
                   hipStream_t s) {
  kf::PlaneGeomArgs<T> g;
  KF_TRY(check_plane_geometry(geom, &g));
  kf::PlaneFitArgs<T> a{n, ld, n_hits, (const T*)seed_state, (const T*)seed_cov, seed_charge, hit_offsets,
                        hit_module, hit_valid, (const T*)hit_uv, (const T*)hit_cov_uv, (T*)state_out, (T*)cov_out,
                        charge_out, (T*)chi2, ndf, trk_status};
  const hipError_t e = kf::launch_fit_plane(a, g, s);
  if (e != hipSuccess) return hip_fail(e, "kf_fit_plane_tracks");
  return ok();
}

}  // namespace

extern "C" {

int kf_propagate_plane(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* state_in,
                       const void* cov_in, const int8_t* charge, const int32_t* target_module,
                       const kf_plane_geometry* geom, int32_t apply_material, void* state_out, void* cov_out,
                       void* path_len, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  KF_TRY(check_lanes(n, "n"));
  if (n == 0) return ok();
  KF_REQUIRE(state_in);
  KF_REQUIRE(cov_in);
  KF_REQUIRE(charge);
  KF_REQUIRE(target_module);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  return prec == KF_F32 ? propagate_plane_impl<float>(n, ld, state_in, cov_in, charge, target_module, geom,
                                                      apply_material, state_out, cov_out, path_len, trk_status, s)
                        : propagate_plane_impl<double>(n, ld, state_in, cov_in, charge, target_module, geom,
                                                       apply_material, state_out, cov_out, path_len, trk_status, s);
}

int kf_update_plane(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, void* state, void* cov, int8_t* charge,
                    const int32_t* module, const void* hit_uv, const void* hit_cov_uv, const kf_plane_geometry* geom,
                    void* chi2, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  KF_TRY(check_lanes(n, "n"));
  if (n == 0) return ok();
  KF_REQUIRE(state);
  KF_REQUIRE(cov);
  KF_REQUIRE(charge);
  KF_REQUIRE(module);
  KF_REQUIRE(hit_uv);
  KF_REQUIRE(hit_cov_uv);
  KF_REQUIRE(chi2);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  return prec == KF_F32 ? update_plane_impl<float>(n, ld, state, cov, charge, module, hit_uv, hit_cov_uv, geom, chi2,
                                                   trk_status, s)
                        : update_plane_impl<double>(n, ld, state, cov, charge, module, hit_uv, hit_cov_uv, geom,
                                                    chi2, trk_status, s);
}

int kf_fit_plane_tracks(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                        const void* seed_cov, const int8_t* seed_charge, const int32_t* hit_offsets,
                        const int32_t* hit_module, const uint8_t* hit_valid, int64_t n_hits, const void* hit_uv,
                        const void* hit_cov_uv, const kf_plane_geometry* geom, void* state_out, void* cov_out,
                        int8_t* charge_out, void* chi2, int32_t* ndf, uint32_t* trk_status, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  KF_TRY(check_lanes(n, "n"));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  KF_TRY(check_lanes(n_hits, "n_hits"));
  if (n == 0) return ok();
  KF_REQUIRE(seed_state);
  KF_REQUIRE(seed_cov);
  KF_REQUIRE(seed_charge);
  KF_REQUIRE(hit_offsets);
  KF_REQUIRE(hit_module);
  KF_REQUIRE(hit_valid);
  KF_REQUIRE(hit_uv);
  KF_REQUIRE(hit_cov_uv);
  KF_REQUIRE(state_out);
  KF_REQUIRE(cov_out);
  KF_REQUIRE(charge_out);
  KF_REQUIRE(chi2);
  KF_REQUIRE(ndf);
  KF_REQUIRE(trk_status);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  return prec == KF_F32
             ? fit_plane_impl<float>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_module, hit_valid,
                                     n_hits, hit_uv, hit_cov_uv, geom, state_out, cov_out, charge_out, chi2, ndf,
                                     trk_status, s)
             : fit_plane_impl<double>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_module, hit_valid,
                                      n_hits, hit_uv, hit_cov_uv, geom, state_out, cov_out, charge_out, chi2, ndf,
                                      trk_status, s);
}

int kf_plane_to_global(kf_ctx* ctx, kf_precision prec, int64_t n_hits, const int32_t* module, const void* hit_uv,
                       const kf_plane_geometry* geom, void* hit_pos, void* stream) {
  KF_RANGE();
  KF_TRY(check_prec(prec));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  KF_TRY(check_lanes(n_hits, "n_hits"));
  if (n_hits == 0) return ok();
  KF_REQUIRE(module);
  KF_REQUIRE(hit_uv);
  KF_REQUIRE(hit_pos);
  KF_REQUIRE(ctx);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == KF_F32) {
    kf::PlaneGeomArgs<float> g;
    KF_TRY(check_plane_geometry(geom, &g));
    e = kf::launch_plane_to_global(n_hits, module, (const float*)hit_uv, g, (float*)hit_pos, s);
  } else {
    kf::PlaneGeomArgs<double> g;
    KF_TRY(check_plane_geometry(geom, &g));
    e = kf::launch_plane_to_global(n_hits, module, (const double*)hit_uv, g, (double*)hit_pos, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_plane_to_global");
  return ok();
}

}  // extern "C"
