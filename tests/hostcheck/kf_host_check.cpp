// Host build of the per-track code of the HIP path, for runs under the
// address and undefined-behaviour sanitizers on the CPU.  The functions the
// kernels call with one track per lane (seeding inside the forward fit, the
// forward fit with checkpoints, the adjoint's reverse sweep with and without
// its state buffer, the forward fit over tilted modules) are host-device
// functions; this program calls them track by track on host memory.  It is a
// test of the device code's memory accesses and arithmetic, not a product
// path: nothing in the library calls it.
//
// Usage: kf_host_check <dir> <32|64>
// <dir>/meta.txt holds "key value" lines; the arrays are raw little-endian
// files in <dir> (layouts as in the C interface: [component][index]).  The
// outputs go to <dir>/out<prec>_<name>.bin as float64 (statuses as uint32,
// charges and ndf as float64).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "kf_adjoint.hpp"
#include "kf_plane_fit.hpp"

namespace {

std::string g_dir;
std::map<std::string, double> g_meta;

[[noreturn]] void die(const char* what, const std::string& name) {
  std::fprintf(stderr, "kf_host_check: %s %s\n", what, name.c_str());
  std::exit(2);
}

void read_meta() {
  FILE* f = std::fopen((g_dir + "/meta.txt").c_str(), "r");
  if (!f) die("cannot open", g_dir + "/meta.txt");
  char key[64];
  double v;
  while (std::fscanf(f, "%63s %lf", key, &v) == 2) g_meta[key] = v;
  std::fclose(f);
}

double meta(const char* k) {
  auto it = g_meta.find(k);
  if (it == g_meta.end()) die("missing meta key", k);
  return it->second;
}

template <typename V>
std::vector<V> load(const std::string& name, size_t count) {
  std::vector<V> v(count);
  FILE* f = std::fopen((g_dir + "/" + name).c_str(), "rb");
  if (!f) die("cannot open", name);
  if (count && std::fread(v.data(), sizeof(V), count, f) != count) die("short file", name);
  std::fclose(f);
  return v;
}

template <typename V>
void save(const std::string& tag, const std::string& name, const V* p, size_t count) {
  const std::string path = g_dir + "/out" + tag + "_" + name + ".bin";
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) die("cannot write", path);
  if (count && std::fwrite(p, sizeof(V), count, f) != count) die("short write", path);
  std::fclose(f);
}

template <typename T>
void save_f64(const std::string& tag, const std::string& name, const std::vector<T>& v) {
  std::vector<double> d(v.begin(), v.end());
  save(tag, name, d.data(), d.size());
}

template <typename T>
std::vector<T> as(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// Seeding, forward fit with checkpoints every `seg` entries, then the reverse
// sweep twice: with the state buffer and recomputing each state from its
// checkpoint.  Both sweeps must give the same bits.
template <typename T>
int run_fit(const std::string& tag) {
  const int64_t n = int64_t(meta("n")), nh = int64_t(meta("n_hits"));
  const int nl = int(meta("n_layers")), seg = int(meta("seg")), max_len = int(meta("max_len"));
  const int seed_mode = int(meta("seed_mode"));
  const bool use_align = meta("align") != 0;
  const auto off = load<int32_t>("hit_offsets.i32", n + 1);
  const auto layer = load<int16_t>("hit_layer.i16", nh);
  const auto valid = load<uint8_t>("hit_valid.u8", nh);
  const auto pos = as<T>(load<double>("hit_pos.f64", 3 * nh));
  const auto cov = as<T>(load<double>("hit_cov.f64", 6 * nh));
  const auto kind = load<int32_t>("layer_kind.i32", nl);
  const auto lpos = as<T>(load<double>("layer_pos.f64", nl));
  const auto lx0 = as<T>(load<double>("layer_x0.f64", nl));
  std::vector<T> align, sal(2 * kf::kMaxLayers, T(0));
  if (use_align) {
    align = as<T>(load<double>("align.f64", 2 * nl));
    for (int i = 0; i < nl; ++i) {
      sal[i] = align[i];
      sal[kf::kMaxLayers + i] = align[nl + i];
    }
  }
  const kf::TrackGeom<T> g{kind.data(), lpos.data(), lx0.data(), nl, T(meta("bz")), T(meta("mass"))};
  int32_t n_seg = (max_len - 1 + seg - 1) / seg;
  if (n_seg < 1) n_seg = 1;

  std::vector<T> seed_state(6 * n), seed_cov(21 * n), state(6 * n), C(21 * n), chi2(n), ckpt(28 * n * n_seg);
  std::vector<int8_t> seed_q(n), q(n);
  std::vector<int32_t> ndf(n);
  std::vector<uint32_t> status(n, 0u);
  kf::FitArgs<T> a{};
  a.n = n;
  a.ld = n;
  a.n_hits = nh;
  a.max_len = max_len;
  a.hit_offsets = off.data();
  a.hit_layer = layer.data();
  a.hit_valid = valid.data();
  a.hit_pos = pos.data();
  a.hit_cov = cov.data();
  a.align = use_align ? align.data() : nullptr;
  a.state_out = state.data();
  a.cov_out = C.data();
  a.charge_out = q.data();
  a.chi2 = chi2.data();
  a.ndf = ndf.data();
  a.ckpt = ckpt.data();
  a.seg = seg;
  a.n_seg = n_seg;
  a.trk_status = status.data();
  a.make_seeds = 1 + seed_mode;
  a.seed_state_out = seed_state.data();
  a.seed_cov_out = seed_cov.data();
  a.seed_charge_out = seed_q.data();
  T bk[28];
  for (int64_t t = 0; t < n; ++t) kf::fit_slot<T, 0>(a, g, use_align ? sal.data() : nullptr, t, bk, 1);

  // the reverse sweep from the seeds the fit made (per-track chi2 weights w)
  const auto w = as<T>(load<double>("weights.f64", n));
  kf::AdjArgs<T> r{};
  r.f = a;
  r.f.make_seeds = 0;
  r.f.seed_state = seed_state.data();
  r.f.seed_cov = seed_cov.data();
  r.f.seed_charge = seed_q.data();
  r.w = w.data();
  r.fwd_status = status.data();
  std::vector<T> gs(6 * n), gh(3 * nh), gs2(6 * n), gh2(3 * nh),
      segbuf(size_t(max_len > 1 ? max_len - 1 : 1) * kf::kSegVals * n);
  for (int pass = 0; pass < 2; ++pass) {
    r.grad_seed = pass ? gs2.data() : gs.data();
    r.grad_hit = pass ? gh2.data() : gh.data();
    r.seg_buf = (pass == 0 && seg > 1) ? segbuf.data() : nullptr;
    if (r.seg_buf)
      for (int64_t t = 0; t < n; ++t) {
        kf::CsrTrack<T> acc{r.f, off[t]};
        kf::refill_track(r, g, use_align ? sal.data() : nullptr, t, acc, int(off[t + 1] - off[t]));
      }
    for (int64_t t = 0; t < n; ++t) {
      const int64_t e0 = off[t];
      kf::CsrTrack<T> acc{r.f, e0};
      kf::adjoint_track(r, g, use_align ? sal.data() : nullptr, t, acc, int(off[t + 1] - e0), e0);
    }
  }
  const bool same = std::memcmp(gs.data(), gs2.data(), gs.size() * sizeof(T)) == 0 &&
                    std::memcmp(gh.data(), gh2.data(), gh.size() * sizeof(T)) == 0;

  save_f64(tag, "seed_state", seed_state);
  save_f64(tag, "seed_cov", seed_cov);
  save_f64(tag, "seed_charge", seed_q);
  save_f64(tag, "state", state);
  save_f64(tag, "cov", C);
  save_f64(tag, "charge", q);
  save_f64(tag, "chi2", chi2);
  save_f64(tag, "ndf", ndf);
  save(tag, "status", status.data(), status.size());
  save_f64(tag, "grad_seed", gs);
  save_f64(tag, "grad_hit", gh);
  std::printf("fit%s: %lld tracks, adjoint with and without the state buffer %s\n", tag.c_str(), (long long)n,
              same ? "identical" : "DIFFERENT");
  return same ? 0 : 1;
}

// Forward fit over tilted modules from the given seeds.
template <typename T>
int run_planes(const std::string& tag) {
  const int64_t n = int64_t(meta("pn")), nh = int64_t(meta("pn_hits")), M = int64_t(meta("pn_modules"));
  const auto off = load<int32_t>("p_offsets.i32", n + 1);
  const auto mod = load<int32_t>("p_module.i32", nh);
  const auto valid = load<uint8_t>("p_valid.u8", nh);
  const auto uv = as<T>(load<double>("p_uv.f64", 2 * nh));
  const auto cuv = as<T>(load<double>("p_cov.f64", 3 * nh));
  const auto tab = as<T>(load<double>("p_table.f64", 10 * M));
  const auto sp = as<T>(load<double>("p_seed_state.f64", 6 * n));
  const auto sc = as<T>(load<double>("p_seed_cov.f64", 21 * n));
  const auto sq = load<int8_t>("p_seed_charge.i8", n);
  std::vector<T> state(6 * n), C(21 * n), chi2(n);
  std::vector<int8_t> q(n);
  std::vector<int32_t> ndf(n);
  std::vector<uint32_t> status(n, 0u);
  kf::PlaneFitArgs<T> a{};
  a.n = n;
  a.ld = n;
  a.n_hits = nh;
  a.seed_state = sp.data();
  a.seed_cov = sc.data();
  a.seed_charge = sq.data();
  a.hit_offsets = off.data();
  a.hit_module = mod.data();
  a.hit_valid = valid.data();
  a.hit_uv = uv.data();
  a.hit_cov_uv = cuv.data();
  a.state_out = state.data();
  a.cov_out = C.data();
  a.charge_out = q.data();
  a.chi2 = chi2.data();
  a.ndf = ndf.data();
  a.trk_status = status.data();
  const kf::PlaneGeomArgs<T> g{tab.data(), M, meta("pbz"), meta("pmass")};
  for (int64_t t = 0; t < n; ++t) kf::fit_plane_track(a, g, t);
  save_f64(tag, "p_state", state);
  save_f64(tag, "p_cov", C);
  save_f64(tag, "p_charge", q);
  save_f64(tag, "p_chi2", chi2);
  save_f64(tag, "p_ndf", ndf);
  save(tag, "p_status", status.data(), status.size());
  std::printf("planes%s: %lld tracks\n", tag.c_str(), (long long)n);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3 || (std::strcmp(argv[2], "32") != 0 && std::strcmp(argv[2], "64") != 0)) {
    std::fprintf(stderr, "usage: %s <dir> <32|64>\n", argv[0]);
    return 2;
  }
  g_dir = argv[1];
  read_meta();
  const std::string tag = argv[2];
  int rc = 0;
  if (tag == "32") {
    rc |= run_fit<float>(tag);
    rc |= run_planes<float>(tag);
  } else {
    rc |= run_fit<double>(tag);
    rc |= run_planes<double>(tag);
  }
  return rc;
}
