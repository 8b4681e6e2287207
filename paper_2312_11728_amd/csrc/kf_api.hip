// C interface of libkf: argument validation, contexts and kernel dispatch.
// Every entry point validates its scalar arguments and pointers before it
// touches the device, so a bad call fails with KF_ERR_ARG and a message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "kf.h"
#include "kf_kernels.hpp"

struct kf_ctx {
  int device = 0;
  int n_cu = 256;
  int32_t* d_counter = nullptr;      // persistent-kernel tile counter
  kf::FitLaunch fit[2] = {{256, 0, 4, 1, 0}, {256, 0, 4, 1, 0}};  // per precision
  // graph cache for kf_fit_tracks (one entry per precision)
  bool use_graph[2] = {false, false};
  hipStream_t capture = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::string key[2];
  // workspace of the packed hit layout (kf_reserve)
  void* work_mem = nullptr;
  kf::PackWork work{};
  // block partials of the alignment-gradient reduction (grown on demand)
  void* red_mem = nullptr;
  size_t red_bytes = 0;
};

namespace {

thread_local std::string g_err;

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
  hipSetDevice(prev);
  if (e != hipSuccess) {
    if (c->d_counter) hipFree(c->d_counter);
    delete c;
    return hip_fail(e, "kf_create");
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
  if (c->capture) hipStreamDestroy(c->capture);
  if (c->d_counter) hipFree(c->d_counter);
  if (c->work_mem) hipFree(c->work_mem);
  if (c->red_mem) hipFree(c->red_mem);
  hipSetDevice(prev);
  delete c;
  return ok();
}

int kf_make_seeds(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const int32_t* hit_offsets,
                  const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, double bz_tesla, int32_t mode,
                  void* seed_state, void* seed_cov, int8_t* seed_charge, uint32_t* trk_status, void* stream) {
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

}  // namespace

extern "C" {

int kf_fit_tracks(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state, const void* seed_cov,
                  const int8_t* seed_charge, const int32_t* hit_offsets, const int16_t* hit_layer,
                  const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos, const void* hit_cov,
                  const kf_geometry* geom, const void* align, void* state_out, void* cov_out, int8_t* charge_out,
                  void* chi2, int32_t* ndf, void* checkpoints, int32_t seg, int32_t max_len, uint32_t* trk_status,
                  void* stream) {
  KF_TRY(check_prec(prec));
  KF_TRY(check_sizes(n, ld));
  kf::GeomArgs g;
  KF_TRY(check_geometry(geom, &g));
  if (n_hits < 0) return fail(KF_ERR_ARG, "n_hits < 0");
  if (checkpoints && seg < 1) return fail(KF_ERR_ARG, "seg = %d < 1", seg);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  if (n == 0) return ok();
  KF_REQUIRE(seed_state);
  KF_REQUIRE(seed_cov);
  KF_REQUIRE(seed_charge);
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
  const int layout = room ? l.layout : 0;
  const bool packed = layout != 0;
  hipError_t e;
  if (prec == KF_F32) {
    auto a = make_fit_args<float>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, n_hits,
                                  hit_pos, hit_cov, align, state_out, cov_out, charge_out, chi2, ndf, checkpoints, seg,
                                  n_seg, trk_status, ctx->d_counter);
    a.max_len = max_len;
    if (packed && (e = kf::launch_pack(a, ctx->work, layout, &a.pk, s)) != hipSuccess) return hip_fail(e, "kf_fit_tracks");
    a.packed = layout;
    e = kf::launch_fit(a, g, l, ctx->n_cu, s);
  } else {
    auto a = make_fit_args<double>(n, ld, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid,
                                   n_hits, hit_pos, hit_cov, align, state_out, cov_out, charge_out, chi2, ndf,
                                   checkpoints, seg, n_seg, trk_status, ctx->d_counter);
    a.max_len = max_len;
    if (packed && (e = kf::launch_pack(a, ctx->work, layout, &a.pk, s)) != hipSuccess) return hip_fail(e, "kf_fit_tracks");
    a.packed = layout;
    e = kf::launch_fit(a, g, l, ctx->n_cu, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_fit_tracks");
  return ok();
}

int kf_reserve(kf_ctx* ctx, int64_t max_tracks, int32_t max_len) {
  if (max_tracks < 0) return fail(KF_ERR_ARG, "max_tracks = %lld < 0", (long long)max_tracks);
  if (max_len < 1 || max_len > kf::kMaxLen) return fail(KF_ERR_ARG, "max_len = %d outside [1, %d]", max_len, kf::kMaxLen);
  KF_REQUIRE(ctx);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(ctx->device);
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
  if (layout < 0 || layout > 2) return fail(KF_ERR_ARG, "layout = %d (0, 1 or 2)", layout);
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

int kf_score_hits(kf_ctx*, int64_t, int64_t, const float*, const float*, const int8_t*, const int16_t*, int32_t,
                  const kf_geometry*, const kf_search_params*, const int32_t*, int64_t, const float*, const float*,
                  const int32_t*, int32_t*, float*, float*, uint32_t*, void*) {
  return fail(KF_ERR_UNSUPPORTED, "kf_score_hits: not built yet");
}

int kf_fit_adjoint(kf_ctx* ctx, kf_precision prec, int64_t n, int64_t ld, const void* seed_state,
                   const void* seed_cov, const int8_t* seed_charge, const int32_t* hit_offsets,
                   const int16_t* hit_layer, const uint8_t* hit_valid, int64_t n_hits, const void* hit_pos,
                   const void* hit_cov, const kf_geometry* geom, const void* align, const void* checkpoints,
                   int32_t seg, int32_t max_len, const void* dL_dchi2, void* grad_seed, void* grad_hit_pos,
                   void* grad_align, const uint32_t* trk_status, void* stream) {
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
  if (grad_align) {
    const size_t need = size_t(kf::adjoint_partial_blocks(n_hits)) * 2 * kf::kMaxLayers * esz;
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
    a.partial = (float*)ctx->red_mem;
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
    a.partial = (double*)ctx->red_mem;
    e = kf::launch_adjoint(a, g, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kf_fit_adjoint");
  return ok();
}

}  // extern "C"
