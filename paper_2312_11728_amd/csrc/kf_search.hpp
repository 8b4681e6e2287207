// Combinatorial candidate search (forward search of the paper's track finding,
// Sec. 2.2; layers and layer plans, Sec. 3.1): per-slot and per-seed steps,
// callable from device and host code.
//
// A seed owns `beam` candidate slots.  At every layer of the plan:
//   extend (one thread per slot): apply the update with the hit the slot's
//     candidate took at the previous layer, propagate to the layer with its
//     material, open the window, compute chi2 for every pool hit inside it
//     and keep the slot's best `beam` children (a child per accepted hit, or
//     one miss child when none is accepted and the miss budget allows, or
//     else one stop child: a candidate that stops -- no crossing, or no hit
//     within its miss budget -- keeps its score and the state it entered the
//     layer with, and from then on is carried from layer to layer unchanged);
//   select (every slot of the seed, at the start of the next layer's
//     extend or before the final pass): merge the slots' sorted child lists
//     into the seed's best `beam` children, which become the next layer's
//     slots;
//   overlap (with the overlap step on; at the next layer's extend, or in the
//     final pass): right after a kept child's update with its hit, the best
//     hit of a higher-numbered module of the same layer inside the window
//     around the updated state (smallest chi2 <= chi2_max, lower id first)
//     is taken as its overlap hit -- a second update, and a score term
//     overlap_bonus - chi2 that counts from the next ranking on.
// Children are ranked by (score descending; hit id ascending, a miss after
// every hit and a stop after a miss; parent rank ascending) -- a total order,
// so the result does not depend on the order in which hits are visited.
#pragma once

#include "kf_kernels.hpp"
#include "kf_math.hpp"

namespace kf {

constexpr int kMaxBeam = 8;
// threads (slots) of a search block: one wave
#ifndef KF_SEARCH_BLOCK
#define KF_SEARCH_BLOCK 64
#endif
constexpr int kSearchBlock = KF_SEARCH_BLOCK;
// waves per SIMD the search kernel's register allocation must allow
#ifndef KF_SEARCH_WAVES
#define KF_SEARCH_WAVES 2
#endif
constexpr int kSearchWaves = KF_SEARCH_WAVES;
static_assert(kSearchBlock >= kMaxBeam && kSearchBlock <= 1024, "search block size");
constexpr float kBinArc = 0.5f;   // pool bin size along r-phi (cm)
constexpr float kBinZ = 1.0f;     // pool bin size along z (cm)
constexpr int32_t kMissKey = 0x7ffffffe;   // ranking keys of a miss and a stop
constexpr int32_t kStopKey = 0x7fffffff;
constexpr int32_t kMissIdx = -1;           // hit codes of a miss and a stop
constexpr int32_t kStopIdx = -3;

// Per-layer binning of the hit pool: the hits of layer l sit in bins
// base[l] + pb * nz[l] + zb, pb in [0, nphi[l]) over phi in [-pi, pi),
// zb in [0, nz[l]) over z in [lo[l], hi[l]] (hits beyond clamp to the edge
// bins).  off: the caller's pool CSR by layer.
struct BinTable {
  int32_t n_layers;
  int32_t off[kMaxLayers + 1];
  int32_t base[kMaxLayers];
  int32_t nphi[kMaxLayers];
  int32_t nz[kMaxLayers];
  float lo[kMaxLayers];
  float hi[kMaxLayers];
};

// bin of a coordinate mapped to f in bin units, clamped to [0, n) (NaN -> 0)
KF_HD inline int32_t clamp_bin(float f, int32_t n) {
  if (!(f >= 0.f)) return 0;
  if (f >= float(n)) return n - 1;
  return int32_t(f);
}

KF_HD inline int32_t phi_bin(float phi, int32_t nphi) {
  return clamp_bin((phi + float(kPi)) * (float(nphi) * float(0.5 / kPi)), nphi);
}

KF_HD inline int32_t z_bin(float z, float lo, float hi, int32_t nz) {
  return clamp_bin((z - lo) * (float(nz) / (hi - lo)), nz);
}

// One hit of the binned pool, 48 bytes: the window test reads the first 16,
// the chi2 the rest.
struct alignas(16) PoolHit {
  float x, y, z, phi;
  float cov[6];
  int32_t id;
  int32_t module;   // detector module (-1 if the caller gave none)
};

// Scalars of the layer being searched (one launch per layer).
struct SearchLayer {
  int32_t layer;       // layer id
  int32_t prev_layer;  // layer of the previous plan step (-1: the seeds' own)
  float R, x0;         // radius, x / X0
  int32_t base, nphi, nz;
  float lo, hi;
  float wmin_r, wmax_r, wmin_z, wmax_z, sig_r, sig_z;
};

struct SearchArgs {
  int64_t n, ld;                 // seeds, leading dimension of the seed arrays
  int32_t beam, plan_len;
  const float* seed_state;       // [6][ld]
  const float* seed_cov;         // [21][ld]
  const int8_t* seed_charge;     // [n]
  const int16_t* seed_layer;     // [n]
  float chi2_max, n_sigma, hit_bonus, miss_penalty;
  int32_t max_miss;
  float bz, mass;
  // binned pool
  const PoolHit* pool;           // [n_pool] in bin order
  const int32_t* bin_off;        // [n_bins + 1]
  int64_t n_pool;
  // slots (S = n * beam; slot = seed * beam + rank); what a seed's slots
  // hand on from layer to layer lives in LDS (SlotExchange), the histories
  // in global memory
  int8_t* hist_parent;           // [plan_len][S]
  int32_t* hist_id;              // [plan_len][S] caller's hit id, -1 = miss, -3 = stopped
  uint32_t* status;              // [n]
  int32_t* cand_hits;            // [n][beam][plan_len]
  float* cand_score;             // [n][beam]
  float* cand_state;             // [6][S] or null
  // overlap step
  int32_t overlap;               // 0 off, 1 on
  float overlap_bonus;
  int32_t* hist_ovl;             // [plan_len][S] overlap hit id of the slot's candidate, -1 none
  int32_t* cand_ovl;             // [n][beam][plan_len] or null
};

// a better than b in the ranking of children
KF_HD inline bool child_before(float sa, int32_t ka, int32_t pa, float sb, int32_t kb, int32_t pb) {
  if (sa != sb) return sa > sb;
  if (ka != kb) return ka < kb;
  return pa < pb;
}

KF_HD inline void load_pool_hit(const SearchArgs& a, int32_t h, float m[3], float V[6]) {
  const PoolHit& ph = a.pool[h];
  m[0] = ph.x;
  m[1] = ph.y;
  m[2] = ph.z;
#pragma unroll
  for (int i = 0; i < 6; ++i) V[i] = ph.cov[i];
}

// chi2 = r^T (C_pos + V)^-1 r of the predicted state (p, c) and hit (m, V);
// reads the position p[0..2] and its covariance block c[0..5] only.
KF_HD inline float hit_chi2(const float* p, const float* c, const float m[3], const float V[6], uint32_t& st) {
  float S[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) S[sym(i, j)] = c[sym(i, j)] + V[sym(i, j)];
  float Si[6];
  inverse_checked<float>(S, Si, st);
  const float r[3] = {m[0] - p[0], m[1] - p[1], m[2] - p[2]};
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) acc += r[i] * (Si[sym(i, 0)] * r[0] + Si[sym(i, 1)] * r[1] + Si[sym(i, 2)] * r[2]);
  return acc;
}

// A slot's window at a layer (step 2 of the search): phi_p +- dphi and
// zp +- w_z around the predicted position, covering the phi bins [b0, b1]
// (taken modulo nphi) and the z bins [z0, z1] of the layer's binned pool,
// slightly widened so that the exact test (in_window) decides.  scan is
// false when the window covers nothing (a non-finite prediction).
struct ScanWindow {
  bool scan;
  float phi_p, dphi, zp, w_z;
  int32_t b0, b1, z0, z1;
};

KF_HD inline ScanWindow open_window(const SearchArgs& a, const SearchLayer& L, const float p[6], const float c[21]) {
  ScanWindow w;
  w.phi_p = k_atan2(p[1], p[0]);
  const float ir = 1.f / k_sqrt(p[0] * p[0] + p[1] * p[1]);
  const float sp = p[1] * ir, cp = p[0] * ir;
  const float var_r = sp * sp * c[sym(0, 0)] - 2.f * sp * cp * c[sym(1, 0)] + cp * cp * c[sym(1, 1)];
  float w_r = a.n_sigma * k_sqrt(var_r + L.sig_r * L.sig_r);
  w_r = w_r < L.wmin_r ? L.wmin_r : (w_r > L.wmax_r ? L.wmax_r : w_r);
  float w_z = a.n_sigma * k_sqrt(c[sym(2, 2)] + L.sig_z * L.sig_z);
  w.w_z = w_z < L.wmin_z ? L.wmin_z : (w_z > L.wmax_z ? L.wmax_z : w_z);
  w.dphi = w_r / L.R;
  w.zp = p[2];
  const float bw = float(L.nphi) * float(0.5 / kPi);
  const float fb0 = k_floor((w.phi_p - w.dphi - 1e-5f + float(kPi)) * bw);
  const float fb1 = k_floor((w.phi_p + w.dphi + 1e-5f + float(kPi)) * bw);
  w.scan = fb0 >= -float(L.nphi) && fb1 <= 2.f * float(L.nphi) && fb1 >= fb0 && k_finite(w.zp) && k_finite(w.w_z);
  w.b0 = w.b1 = w.z0 = w.z1 = 0;
  if (w.scan) {
    w.b0 = int32_t(fb0);
    w.b1 = int32_t(fb1);
    if (w.b1 - w.b0 + 1 > L.nphi) {
      w.b0 = 0;
      w.b1 = L.nphi - 1;
    }
    w.z0 = z_bin(w.zp - w.w_z - 1e-4f, L.lo, L.hi, L.nz);
    w.z1 = z_bin(w.zp + w.w_z + 1e-4f, L.lo, L.hi, L.nz);
  }
  return w;
}

// The run of the binned pool that phi bin b of the window covers: every phi
// bin's z range [z0, z1] is one contiguous run [lo, hi).
KF_HD inline void bin_run(const SearchArgs& a, const SearchLayer& L, int32_t z0, int32_t z1, int32_t b, int32_t& lo,
                          int32_t& hi) {
  const int32_t pb = b < 0 ? b + L.nphi : (b >= L.nphi ? b - L.nphi : b);
  lo = a.bin_off[L.base + pb * L.nz + z0];
  hi = a.bin_off[L.base + pb * L.nz + z1 + 1];
}

// the exact window test of a pool hit
KF_HD inline bool in_window(float phi_p, float dphi, float zp, float w_z, const PoolHit& ph) {
  float d = ph.phi - phi_p;
  d = d > float(kPi) ? d - float(2 * kPi) : (d < -float(kPi) ? d + float(2 * kPi) : d);
  return k_abs(d) <= dphi && k_abs(ph.z - zp) <= w_z;
}

// The overlap step for a candidate that took binned pool hit h on layer L
// and has just been updated with it (p, c, q): among the hits of L on a
// module with a higher id than h's inside the window around the updated
// state (the extend step's window formulas with the updated covariance), the
// one with the smallest chi2 <= chi2_max (the lower id among equals).  The
// module order counts each pair of overlapping hits once.  If there is
// one, the state gets a second update with it and its id is returned with
// its chi2 in c2_out; else -1.
KF_HD inline int32_t pick_overlap(const SearchArgs& a, const SearchLayer& L, int32_t h, float p[6], float c[21],
                                  int& q, float& c2_out, uint32_t& st) {
  const int32_t mod = a.pool[h].module;
  const ScanWindow w = open_window(a, L, p, c);
  int32_t best = -1, best_id = 0;
  float best_c2 = 0.f;
  if (w.scan) {
    for (int32_t b = w.b0; b <= w.b1; ++b) {
      int32_t h0, h1;
      bin_run(a, L, w.z0, w.z1, b, h0, h1);
      for (int32_t k = h0; k < h1; ++k) {
        const PoolHit ph = a.pool[k];
        if (ph.module <= mod) continue;
        if (!in_window(w.phi_p, w.dphi, w.zp, w.w_z, ph)) continue;
        const float m[3] = {ph.x, ph.y, ph.z};
        const float c2 = hit_chi2(p, c, m, ph.cov, st);
        if (!(c2 <= a.chi2_max)) continue;
        if (best < 0 || c2 < best_c2 || (c2 == best_c2 && ph.id < best_id)) {
          best = k;
          best_id = ph.id;
          best_c2 = c2;
        }
      }
    }
  }
  if (best < 0) return -1;
  float m[3], V[6], c2u;
  load_pool_hit(a, best, m, V);
  update(p, c, q, m, V, c2u, st);
  c2_out = best_c2;
  return best_id;
}

// What the slots of a block's seeds hand on from one layer to the next,
// in LDS, indexed by the slot's place in the block: the state its candidate
// goes on with (the predicted state, or the state it entered the layer with
// if it stops there; p, c, then the charge), its child list at the layer
// (best first) and its candidate's misses.
template <int B>
struct SlotExchange {
  float state[28][kSearchBlock];
  float kid_score[B][kSearchBlock];
  int32_t kid_id[B][kSearchBlock];
  int32_t kid_idx[B][kSearchBlock];
  int32_t kid_n[kSearchBlock];
  int32_t miss[kSearchBlock];
};

// A slot's candidate for the next layer, as the selection leaves it.
struct Cand {
  bool live;        // the slot has a candidate
  int32_t idx;      // binned pool index of its hit on the layer it left, kMissIdx, kStopIdx
  float score;
  int miss;
  int q;
  float p[6], c[21];
};

// The seed's own candidate at the first layer (rank 0 only): its state, no
// hit to apply.
KF_HD inline void seed_candidate(const SearchArgs& a, int64_t s, Cand& k) {
  const int64_t seed = s / a.beam;
  k.live = s % a.beam == 0;
  if (!k.live) return;
#pragma unroll
  for (int i = 0; i < 6; ++i) k.p[i] = a.seed_state[i * a.ld + seed];
#pragma unroll
  for (int i = 0; i < 21; ++i) k.c[i] = a.seed_cov[i * a.ld + seed];
  k.q = a.seed_charge[seed];
  k.idx = kMissIdx;
  k.score = 0.f;
  k.miss = 0;
}

// The selection of plan step `step` for the slot at place i of its block
// (slot s): the child lists of the seed's slots are merged into the seed's
// next candidates, and the slot takes the one of its rank, with its
// parent's state; its history entry of the step goes to global memory.
// Every slot of a seed runs the same merge, each keeps its own result.
template <int B>
KF_HD inline void select_slot(const SearchArgs& a, const SlotExchange<B>& X, int step, int64_t s, int i, Cand& k) {
  const int64_t S = a.n * a.beam;
  const int i0 = (i / a.beam) * a.beam;
  const int me = i - i0;
  // The heads of the seed's child lists (each sorted best first, only its
  // first `beam` entries choosable) compete, ties by child id, then by the
  // parent's rank; the chosen list's next entry, read from LDS, becomes its
  // head.
  int cnt[B], taken[B];
  float hs[B];
  int32_t hk[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    cnt[r] = r < a.beam ? X.kid_n[r < a.beam ? i0 + r : i0] : 0;
    if (cnt[r] > a.beam) cnt[r] = a.beam;
    taken[r] = 0;
    // (an empty list reads a valid place and discards it)
    hs[r] = cnt[r] > 0 ? X.kid_score[0][cnt[r] > 0 ? i0 + r : i0] : -k_inf<float>();
    hk[r] = cnt[r] > 0 ? X.kid_id[0][cnt[r] > 0 ? i0 + r : i0] : kStopKey;
  }
  // outputs 0 .. me in turn; the last one chosen is this slot's
  int par = -1, pos = 0;
  float score = 0.f;
  int32_t key = 0;
  bool open = true;   // every output so far had a child
#pragma unroll
  for (int out = 0; out < B; ++out) {
    if (out > me || !open) continue;
    int best = -1, bpos = 0;
    float bs = 0.f;
    int32_t bk = 0;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (taken[r] < cnt[r] && (best < 0 || child_before(hs[r], hk[r], r, bs, bk, best))) {
        best = r;
        bpos = taken[r];
        bs = hs[r];
        bk = hk[r];
      }
    }
    if (best < 0) {
      open = false;
      continue;
    }
    if (out == me) {
      par = best;
      pos = bpos;
      score = bs;
      key = bk;
    }
    int nc = 0;
#pragma unroll
    for (int r = 0; r < B; ++r)
      if (r == best) nc = cnt[r];
    const bool more = bpos + 1 < nc;
    const int jr = more ? bpos + 1 : 0;
    const float ns = more ? X.kid_score[jr][i0 + best] : -k_inf<float>();
    const int32_t nk = more ? X.kid_id[jr][i0 + best] : kStopKey;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r == best) {
        hs[r] = ns;
        hk[r] = nk;
        ++taken[r];
      }
    }
  }
  k.live = par >= 0;
  if (!k.live) return;
  const int32_t idx = X.kid_idx[pos][i0 + par];
  k.idx = idx;
  k.score = score;
  k.miss = X.miss[i0 + par] + (idx == kMissIdx ? 1 : 0);
#pragma unroll
  for (int v = 0; v < 6; ++v) k.p[v] = X.state[v][i0 + par];
#pragma unroll
  for (int v = 0; v < 21; ++v) k.c[v] = X.state[6 + v][i0 + par];
  k.q = int(X.state[27][i0 + par]);
  a.hist_parent[int64_t(step) * S + s] = int8_t(par);
  a.hist_id[int64_t(step) * S + s] = idx >= 0 ? key : idx;
  if (a.overlap) a.hist_ovl[int64_t(step) * S + s] = kMissIdx;
}

// A slot's child list at a layer, best first (empty entries rank last), and
// the number of hits it accepted.
template <int B>
struct Kids {
  float s[B];
  int32_t key[B], idx[B];
  int n;
};

template <int B>
KF_HD inline void kids_init(Kids<B>& K) {
#pragma unroll
  for (int j = 0; j < B; ++j) {
    K.s[j] = -k_inf<float>();
    K.key[j] = kMissKey;
    K.idx[j] = -2;
  }
  K.n = 0;
}

// an accepted hit (child score ns, hit id key, binned pool index idx) into
// the sorted list; the last entry drops out
template <int B>
KF_HD inline void kids_add(const SearchArgs& a, Kids<B>& K, float ns, int32_t key, int32_t idx) {
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (j < a.beam && child_before(ns, key, 0, K.s[j], K.key[j], 0)) {
      const float ts = K.s[j];
      const int32_t tk = K.key[j], ti = K.idx[j];
      K.s[j] = ns;
      K.key[j] = key;
      K.idx[j] = idx;
      ns = ts;
      key = tk;
      idx = ti;
    }
  }
  ++K.n;
}

// Extend of candidate k of the slot at place i of its block (slot s) to
// layer L (see the file comment), in three parts: extend_open, the scan of
// its window (scan_window), extend_close.
//
// extend_open: the update with the hit the candidate took at the previous
// layer (and the overlap step), the state it enters L with (left in X, kept
// if it stops here), the propagation to L and its window.  Returns false
// when the slot has nothing to scan: no candidate, or one that stops (its
// stop child is then written).  score: the candidate's score with the
// overlap term; st collects the status bits.
template <int B>
KF_HD inline bool extend_open(const SearchArgs& a, SlotExchange<B>& X, const SearchLayer& L, const SearchLayer& Lp,
                              int step, int64_t s, int i, Cand& k, float& score, ScanWindow& w, uint32_t& st) {
  const int64_t S = a.n * a.beam;
  X.kid_n[i] = 0;
  w.scan = false;
  score = 0.f;
  if (!k.live) return false;
  float* const p = k.p;
  float* const c = k.c;
  float ovl = 0.f;
  if (k.idx >= 0) {
    float m[3], V[6], c2;
    load_pool_hit(a, k.idx, m, V);
    update(p, c, k.q, m, V, c2, st);
    if (a.overlap) {
      float oc2 = 0.f;
      const int32_t oid = pick_overlap(a, Lp, k.idx, p, c, k.q, oc2, st);
      a.hist_ovl[int64_t(step - 1) * S + s] = oid;
      if (oid >= 0) ovl = a.overlap_bonus - oc2;
    }
  }
  const int prev = step == 0 ? a.seed_layer[s / a.beam] : L.prev_layer;
  score = k.score + ovl;
  const bool stopped = k.idx == kStopIdx;   // carried unchanged
  // the state entering the layer, kept if the candidate stops here
#pragma unroll
  for (int v = 0; v < 6; ++v) X.state[v][i] = p[v];
#pragma unroll
  for (int v = 0; v < 21; ++v) X.state[6 + v][i] = c[v];
  X.state[27][i] = float(k.q);
  X.miss[i] = k.miss;
  if (stopped || !propagate(p, c, k.q, 0, L.R, L.x0, prev == L.layer, true, a.bz, a.mass, st)) {
    X.kid_score[0][i] = score;
    X.kid_id[0][i] = kStopKey;
    X.kid_idx[0][i] = kStopIdx;
    X.kid_n[i] = 1;
    return false;
  }
  w = open_window(a, L, p, c);
  return true;
}

// The scan of one slot's window by its own thread: chi2 of every pool hit
// inside it, each accepted one (chi2 <= chi2_max) added to K with the child
// score score + hit_bonus - chi2.  Reads run one step ahead, so that a load
// is in flight while the previous hit is scored: the next bin's run bounds
// while a bin is scanned, the next hit while a hit is scored (the index is
// clamped to the run, the last read repeats the current hit and is not used;
// an empty run reads nothing).
template <int B>
KF_HD inline void scan_window(const SearchArgs& a, const SearchLayer& L, const ScanWindow& w, const float p[6],
                              const float c[21], float score, Kids<B>& K, uint32_t& st) {
  if (!w.scan) return;
  int32_t h0, h1;
  bin_run(a, L, w.z0, w.z1, w.b0, h0, h1);
  for (int32_t b = w.b0; b <= w.b1; ++b) {
    int32_t n0 = 0, n1 = 0;
    if (b < w.b1) bin_run(a, L, w.z0, w.z1, b + 1, n0, n1);
    PoolHit cur;
    if (h0 < h1) cur = a.pool[h0];
    for (int32_t h = h0; h < h1; ++h) {
      const PoolHit ph = cur;
      cur = a.pool[h + 1 < h1 ? h + 1 : h];
      if (!in_window(w.phi_p, w.dphi, w.zp, w.w_z, ph)) continue;
      const float m[3] = {ph.x, ph.y, ph.z};
      const float c2 = hit_chi2(p, c, m, ph.cov, st);
      if (c2 <= a.chi2_max) kids_add(a, K, score + a.hit_bonus - c2, ph.id, h);
    }
    h0 = n0;
    h1 = n1;
  }
}

// extend_close: the slot's child list after its scan (a miss child when no
// hit was accepted and the miss budget allows, else a stop child) and the
// predicted state the candidate goes on with, into X.
template <int B>
KF_HD inline void extend_close(const SearchArgs& a, SlotExchange<B>& X, int i, const Cand& k, float score,
                               Kids<B>& K) {
  if (K.n == 0) {
    const bool can_miss = k.miss < a.max_miss;
    K.s[0] = can_miss ? score - a.miss_penalty : score;
    K.key[0] = can_miss ? kMissKey : kStopKey;
    K.idx[0] = can_miss ? kMissIdx : kStopIdx;
    K.n = 1;
  }
  if (K.idx[0] != kStopIdx) {
    // the candidate goes on from the predicted state
#pragma unroll
    for (int v = 0; v < 6; ++v) X.state[v][i] = k.p[v];
#pragma unroll
    for (int v = 0; v < 21; ++v) X.state[6 + v][i] = k.c[v];
    X.state[27][i] = float(k.q);
  }
  const int n_out = K.n < a.beam ? K.n : a.beam;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (j < n_out) {
      X.kid_score[j][i] = K.s[j];
      X.kid_id[j][i] = K.key[j];
      X.kid_idx[j][i] = K.idx[j];
    }
  }
  X.kid_n[i] = n_out;
}

// After the last layer and its selection: candidate k's final state
// (update with its last hit), score and hit list (backtracked through the
// parents; every slot of the seed must have written its histories).
KF_HD inline uint32_t finish_candidate(const SearchArgs& a, const SearchLayer& Llast, int64_t s, Cand& k) {
  const int64_t S = a.n * a.beam;
  const int64_t seed = s / a.beam;
  const int r = int(s % a.beam);
  const int P = a.plan_len;
  int32_t* out = a.cand_hits + s * P;
  uint32_t st = 0;
  int32_t* ovl_out = a.cand_ovl ? a.cand_ovl + s * P : nullptr;
  if (!k.live) {
    for (int j = 0; j < P; ++j) out[j] = -2;
    if (ovl_out)
      for (int j = 0; j < P; ++j) ovl_out[j] = -2;
    a.cand_score[s] = -k_inf<float>();
    if (a.cand_state)
#pragma unroll
      for (int v = 0; v < 6; ++v) a.cand_state[v * S + s] = k_nan<float>();
    return 0;
  }
  {
    float* const p = k.p;
    float* const c = k.c;
    int q = k.q;
    const int32_t h = k.idx;
    float ovl = 0.f;
    if (h >= 0) {
      float m[3], V[6], c2;
      load_pool_hit(a, h, m, V);
      update(p, c, q, m, V, c2, st);
      if (a.overlap) {
        float oc2 = 0.f;
        const int32_t oid = pick_overlap(a, Llast, h, p, c, q, oc2, st);
        a.hist_ovl[int64_t(P - 1) * S + s] = oid;
        if (oid >= 0) ovl = a.overlap_bonus - oc2;
      }
    }
    if (a.cand_state)
#pragma unroll
      for (int v = 0; v < 6; ++v) a.cand_state[v * S + s] = p[v];
    a.cand_score[s] = k.score + ovl;
  }
  int rr = r;
  for (int j = P - 1; j >= 0; --j) {
    const int64_t hs = int64_t(j) * S + seed * a.beam + rr;
    out[j] = a.hist_id[hs];
    if (ovl_out) ovl_out[j] = a.overlap ? a.hist_ovl[hs] : kMissIdx;
    rr = a.hist_parent[hs];
  }
  return st;
}

}  // namespace kf
