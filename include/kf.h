/*
 * kf.h -- C interface of the MI355X Kalman-filter track-fit library (libkf.so).
 *
 * The library runs the per-layer step of Kalman-filter track reconstruction
 * over many tracks at once: propagation of each track to its next detector
 * layer, the covariance propagation C' = F C F^T + Q with multiple scattering,
 * the residual-covariance inverse, the gain and state/covariance update, and
 * chi2 scoring of candidate hits.  The paper (Sec. 2.2 "Track finding
 * algorithm") names these as the processing steps of track finding and
 * (Sec. 3.1 "Geometry & detector description") as the vectorised key
 * computations: track-candidate propagation, hit selection and Kalman-filter
 * calculations.  A seed is a list of hits plus an initial parameter estimate
 * (Sec. 2.2); a layer is an r-z bounding box in global cylindrical coordinates
 * with its material (Sec. 3.1); configuration carries no global state
 * (Sec. 3, opening paragraphs, and Sec. 3.2).
 *
 * Conventions (all entry points)
 *   Units: cm, GeV/c, tesla, radians.
 *   Track state p = (x, y, z, ipt, phi, theta), ipt = 1/pT >= 0, phi in
 *   (-pi, pi], theta in (0, pi); the charge q = +-1 is a separate int8.
 *   Symmetric matrices are packed lower-triangular, row-major:
 *   idx(i, j) = i*(i+1)/2 + j for j <= i (6x6 -> 21 entries, 3x3 -> 6).
 *   Array pointers named *_state, *_cov, hit_*, chi2, ... are DEVICE pointers
 *   owned by the caller.  Structure-of-arrays: element (i, t) of a [k][ld]
 *   array is at base[i*ld + t]; ld >= n.  Float arrays hold float (KF_F32) or
 *   double (KF_F64) as selected by the precision argument.
 *   `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *   and return; none synchronises the stream.
 *   Device memory: kf_create allocates a few bytes of counters and
 *   kf_reserve the packed-layout workspace.  kf_score_hits, kf_fit_adjoint
 *   (its alignment reduction), kf_final_fit and kf_remove_duplicates keep a context-owned
 *   workspace that they grow on demand (hipMalloc, which can synchronise the
 *   device and must not happen under graph capture); a call with sizes no
 *   larger than an earlier call's on the same context allocates nothing.
 *   kf_set_kernel_timing creates events and kf_set_fit_graph captures graphs.
 *   No other call allocates device memory.
 *   n = 0 is a no-op (array pointers may then be NULL).
 *   Errors: every call returns a kf_status.  KF_ERR_ARG is returned before any
 *   device work for a null pointer, n < 0, ld < n, a bad geometry or another
 *   invalid scalar argument; KF_ERR_DEVICE wraps a HIP error.  kf_last_error()
 *   gives a message for the last non-OK return on the calling thread.
 *   Per-track numerical trouble never fails a call: it sets bits in the
 *   per-track status word and leaves finite outputs.
 *   Concurrency: one kf_ctx may be used by one host thread / one stream at a
 *   time (it owns a small device work counter); separate contexts are
 *   independent.
 */
#ifndef KF_H
#define KF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KF_OK = 0,
  KF_ERR_ARG = -1,
  KF_ERR_DEVICE = -2,
  KF_ERR_NOMEM = -3,
  KF_ERR_UNSUPPORTED = -4
} kf_status;

typedef enum { KF_F32 = 0, KF_F64 = 1 } kf_precision;

/* Per-track status bits (OR-ed). */
enum {
  KF_TRK_NO_CROSSING = 1u,   /* the helix does not reach the target surface; track frozen */
  KF_TRK_GRAZING = 2u,       /* |cos(incidence)| < 0.05 at a crossing; material clamped there */
  KF_TRK_NONFINITE = 4u,     /* a step produced a non-finite value; track frozen before it */
  KF_TRK_FP64_FALLBACK = 8u, /* a 3x3 inverse was recomputed in FP64 (FP32 path only) */
  KF_TRK_CHARGE_FLIP = 16u,  /* an update turned 1/pT negative; charge flipped */
  KF_TRK_COV_NOT_PSD = 32u,  /* a variance became negative after an update (FP32: beyond the rounding of the prior) */
  KF_TRK_BAD_INPUT = 64u,    /* layer id out of range or fewer than 3 valid hits for seeding */
  KF_TRK_OUTLIER = 128u      /* kf_final_fit: at least one hit was rejected as an outlier */
};

/* Detector description.  HOST struct and HOST arrays, read during the call
 * (copied into the kernel arguments), so it may be freed when the call returns.
 * A layer is a barrel cylinder r = pos with z in [lo, hi] or an endcap disk
 * z = pos with r in [lo, hi] (an r-z box).  x_over_x0 is its thickness in
 * radiation lengths at normal incidence.  1 <= n_layers <= KF_MAX_LAYERS. */
#define KF_MAX_LAYERS 64
typedef struct {
  int32_t n_layers;
  const int8_t *kind;       /* 0 = barrel cylinder, 1 = endcap disk */
  const double *pos;        /* R (barrel) or Z (disk) */
  const double *lo, *hi;    /* barrel: zmin, zmax; disk: rmin, rmax */
  const double *x_over_x0;  /* material per crossing at normal incidence */
  double bz_tesla;          /* uniform solenoidal field, != 0 */
  double particle_mass_gev; /* mass hypothesis for the scattering angle, > 0 */
} kf_geometry;

typedef struct kf_ctx kf_ctx;

/* Create a context on HIP device `hip_device` (allocates a few bytes of device
 * work counters).  Returns KF_ERR_DEVICE if the device cannot be used. */
int kf_create(kf_ctx **out, int hip_device);
/* Destroy a context (NULL is a no-op).  Waits for nothing: the caller must not
 * destroy a context with work still queued. */
int kf_destroy(kf_ctx *ctx);
/* Message for the last non-OK return on the calling thread ("" if none). */
const char *kf_last_error(void);

/* Seed every track from three of its valid hits (helix through three points:
 * transverse Menger curvature, then the polar angle from the arc length;
 * position = the first chosen hit).  mode 0: the first three valid hits.
 * mode 1: the first valid hit, then each next valid hit at least 2.5 cm away
 * (transverse) from the previously chosen one -- a longer lever arm for tracks
 * whose first hits are close in the transverse plane.  The seed covariance is
 * diag(1, 1, 1, 1, 0.01, 0.01) (a diffuse prior).
 * Inputs: hit_offsets[n+1] (CSR into the hit arrays), hit_valid[n_hits],
 * hit_pos[3][n_hits].  Outputs: seed_state[6][ld], seed_cov[21][ld],
 * seed_charge[n], trk_status[n] (overwritten; KF_TRK_BAD_INPUT if fewer than
 * three hits qualify, the seed is then zero with the prior covariance). */
int kf_make_seeds(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                  const int32_t *hit_offsets, const uint8_t *hit_valid, int64_t n_hits,
                  const void *hit_pos, double bz_tesla, int32_t mode,
                  void *seed_state, void *seed_cov, int8_t *seed_charge,
                  uint32_t *trk_status, void *stream);

/* Propagate n tracks to their target layers (the track-candidate propagation
 * the paper names as a vectorised key computation, Sec. 3.1, and the
 * propagation step of track finding, Sec. 2.2):
 * exact helix in the uniform field to the first admissible crossing of the
 * target surface, the surface-to-surface Jacobian F (including the dependence
 * of the path length on the state), C' = F C F^T, and, if apply_material, the
 * multiple-scattering noise Q of the target layer evaluated at the propagated
 * state (Highland angle, rank 2 in (ipt, phi, theta)).
 * Crossing rule: the first root with path s > -1 cm, or s > 0.01 cm when
 * from_layer[t] == target_layer[t] (a looper re-crossing the layer it sits on).
 * from_layer may be NULL (never the same layer).
 * state_in/out [6][ld], cov_in/out [21][ld] (in and out may alias),
 * charge[n], target_layer[n], path_len[n] (transverse path, may be NULL),
 * trk_status[n] (bits OR-ed in).  A track with no crossing is copied
 * unchanged and gets KF_TRK_NO_CROSSING. */
int kf_propagate(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                 const void *state_in, const void *cov_in, const int8_t *charge,
                 const int16_t *target_layer, const int16_t *from_layer,
                 const kf_geometry *geom, int32_t apply_material,
                 void *state_out, void *cov_out, void *path_len,
                 uint32_t *trk_status, void *stream);

/* Kalman update with one 3-D hit per track (the Kalman-filter calculations of
 * Sec. 2.2 and Sec. 3.1; the chi2 is the one the per-iteration cuts of
 * Sec. 3.2 apply to): r = m - (x, y, z),
 * S = C_pos + V, S^-1 (FP32: cofactors, recomputed in FP64 when the condition
 * estimate ||S||inf ||S^-1||inf exceeds 1e6, det <= 0 or non-finite),
 * chi2 = r^T S^-1 r, K = C H^T S^-1, p += K r, symmetrised Joseph form
 * C = (I-KH) C (I-KH)^T + K V K^T; if ipt turns negative the charge flips
 * (ipt, q and row/column 3 of C change sign); phi wrapped to (-pi, pi].
 * state[6][ld], cov[21][ld], charge[n] updated in place; hit_pos[3][ld],
 * hit_cov[6][ld]; chi2[n] out; trk_status[n] bits OR-ed in. */
int kf_update(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
              void *state, void *cov, int8_t *charge,
              const void *hit_pos, const void *hit_cov,
              void *chi2, uint32_t *trk_status, void *stream);

/* Forward Kalman fit of n tracks with uneven hit lists (the layer-by-layer
 * propagate-and-update loop of Sec. 2.2 run over the hits of each track; a seed
 * carries an estimate, Sec. 2.2, and layers are r-z boxes, Sec. 3.1).
 * Track t owns entries [hit_offsets[t], hit_offsets[t+1]) of the hit arrays,
 * in crossing order: hit_layer[e] (layer id), hit_valid[e] (0 = hole: the
 * layer's material is applied but no update), hit_pos[3][n_hits],
 * hit_cov[6][n_hits].  The seed (seed_state[6][ld], seed_cov[21][ld],
 * seed_charge[n]) sits on the track's first valid entry; the material of that
 * layer is added there, then every later entry is propagated to (with the
 * crossing rule of kf_propagate, from = the previous entry's layer), gets its
 * layer's material and, if valid, an update.  align (device, [2][n_layers] or
 * NULL) corrects barrel hits: rotation about z by align[0][l]/R_l and a z
 * shift align[1][l]; disk hits are not corrected.
 * Outputs: state_out[6][ld], cov_out[21][ld], charge_out[n], chi2[n] (sum),
 * ndf[n] (= 2 * used hits - 5), trk_status[n] (overwritten).
 * checkpoints: NULL, or a [28][ld * n_seg] buffer receiving (state, cov,
 * charge) before entry 1 + j*seg of each track's fit (j = 0..n_seg-1,
 * n_seg = ceil((max_len - 1) / seg)); used by kf_fit_adjoint.
 * max_len (1..64) bounds the entries used per track: entries beyond it are
 * ignored and the track gets KF_TRK_BAD_INPUT.
 * Layout (a tuning choice, see kf_set_fit_launch): with a workspace from
 * kf_reserve large enough for n tracks and max_len, the call can first sort
 * the tracks by entry count (longest first, so that the lanes of a wave run
 * similar loops) and optionally copy the hits into a tile-transposed layout
 * (entry k of 64 tracks contiguous, every hit load of a wave one coalesced
 * read); the fit can also stage the CSR entries of each wave's 64 tracks
 * through LDS itself, a few entries per track at a time (no pass before the
 * fit; with the sort, if a workspace is there).  Without a workspace the fit
 * reads the CSR arrays in track order.  Results are bit-identical within each
 * family of layouts (direct reads: 0-2; LDS staging: 3, 4) and agree to
 * rounding across the two (see kf_set_fit_launch).  The order of the tracks
 * changes no result, but in a geometry of barrel cylinders and disks, tracks
 * given in order of direction (and length) run faster: the lanes of a wave
 * then cross the same kind of layer at the same step. */
int kf_fit_tracks(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                  const void *seed_state, const void *seed_cov, const int8_t *seed_charge,
                  const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                  int64_t n_hits, const void *hit_pos, const void *hit_cov,
                  const kf_geometry *geom, const void *align,
                  void *state_out, void *cov_out, int8_t *charge_out,
                  void *chi2, int32_t *ndf,
                  void *checkpoints, int32_t seg, int32_t max_len,
                  uint32_t *trk_status, void *stream);

/* Seeding and fit in one launch: every track is seeded from its own hits
 * exactly as kf_make_seeds does in seed_mode (0: the first three valid hits;
 * 1: spaced by >= 2.5 cm in the transverse plane), with geom->bz_tesla as the
 * field and the same wide diagonal covariance, then fitted as kf_fit_tracks
 * fits it; results are bit-identical to kf_make_seeds followed by
 * kf_fit_tracks with the same arguments, except that trk_status[t] holds
 * the seeding bits (KF_TRK_BAD_INPUT: fewer than three usable hits) and the
 * fit's together.  seed_state_out [6][ld], seed_cov_out [21][ld] and
 * seed_charge_out [n] (device, each may be NULL) receive the seeds, for a
 * later kf_fit_adjoint.  The other arguments, the layout and launch choices
 * of the context, graph replay and kernel timing are those of kf_fit_tracks;
 * KF_ERR_ARG for a seed_mode other than 0 or 1. */
int kf_seed_fit_tracks(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld, int32_t seed_mode,
                       const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                       int64_t n_hits, const void *hit_pos, const void *hit_cov,
                       const kf_geometry *geom, const void *align,
                       void *seed_state_out, void *seed_cov_out, int8_t *seed_charge_out,
                       void *state_out, void *cov_out, int8_t *charge_out,
                       void *chi2, int32_t *ndf,
                       void *checkpoints, int32_t seg, int32_t max_len,
                       uint32_t *trk_status, void *stream);

/* Backward fit (the paper's Sec. 2.2, step 4: each found track is traversed
 * again backwards and its parameters refitted).  Input: the result of
 * kf_fit_tracks / kf_seed_fit_tracks on the same hits (state_in[6][ld],
 * cov_in[21][ld], charge_in[n]: the state on each track's last entry) and its
 * fwd_status[n] (may be NULL: every track is taken as complete).  The
 * covariance is multiplied by cov_scale (>= 1; 100 is the value the tests and
 * the benchmark use), the surface of the last entry's layer imposed on it
 * again (its normal made a null vector, as after every propagation), the
 * direction of motion reversed (phi + pi, pi - theta, -q; the theta terms of
 * the covariance change sign), and the entries are
 * taken in reverse order, from the last one down to the first valid one, with
 * kf_fit_tracks's rules per entry (the first adds its layer's material at the
 * current state; every later one is propagated to, gets its layer's material
 * and, if valid, an update; a failed crossing or a non-finite step freezes
 * the track).  The result, on the track's first valid entry, is turned back
 * to the outward direction.
 * Outputs: state_out[6][ld], cov_out[21][ld], charge_out[n] (must not alias
 * the inputs), chi2[n] (sum over the backward pass), ndf[n] (= 2 * used
 * hits - 5), trk_status[n] (overwritten with the backward pass's bits).
 * Tracks the forward fit stopped (KF_TRK_NO_CROSSING, KF_TRK_NONFINITE or
 * KF_TRK_BAD_INPUT in fwd_status) or with no valid entry are not refitted:
 * the input is copied out, chi2 = 0, ndf = -5, trk_status = KF_TRK_BAD_INPUT.
 * max_len (1..64) as in kf_fit_tracks.  Hit arrays, layout and precision as
 * in kf_fit_tracks; no alignment correction.  The hits of each wave's 64
 * tracks are staged through LDS.  KF_ERR_ARG for cov_scale < 1 or not finite,
 * aliased outputs, or the argument errors of kf_fit_tracks. */
int kf_backward_fit(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                    const void *state_in, const void *cov_in, const int8_t *charge_in,
                    const uint32_t *fwd_status,
                    const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                    int64_t n_hits, const void *hit_pos, const void *hit_cov,
                    const kf_geometry *geom, double cov_scale, int32_t max_len,
                    void *state_out, void *cov_out, int8_t *charge_out,
                    void *chi2, int32_t *ndf, uint32_t *trk_status, void *stream);

/* Backward fit with smoothing (the backward fit of kf_backward_fit, completed
 * by a two-filter smoother): in addition to the backward fit's outputs (the
 * same arguments and rules), the smoothed state of every entry of a refitted
 * track from its first valid entry to its last.  At each entry the forward
 * filtered state (from fwd_checkpoints) and the backward pass's state on
 * arriving there, before that layer's material (turned outward), both
 * describe the track just outside the layer; they are combined on the five
 * directions the state can move in on the surface:
 *   x = x_f + C_f (C_f + C_b)^+ (x_b - x_f),  C = C_f - C_f (C_f + C_b)^+ C_f
 * (the 5x5 system solved by Cholesky in FP64).  The last entry's smoothed
 * state is its forward filtered state (state_in).  The backward pass adds
 * each layer's material after the combination (the same arithmetic as
 * kf_backward_fit, apart from rounding).
 * fwd_checkpoints: the [28][ld * (max_len - 1)] checkpoints written by the
 * forward fit (kf_fit_tracks / kf_seed_fit_tracks) of the same tracks with
 * seg = 1 and the same max_len (slot m holds the filtered state after the
 * track's first valid entry + m).  smooth_state [6][ld * max_len],
 * smooth_cov [21][ld * max_len] (device, caller-owned): the smoothed state of
 * entry r (0-based within track t) at [i][r * ld + t].  Entries before the
 * first valid one, beyond max_len or of tracks not refitted are not written;
 * entries of a refitted track that its backward pass did not reach (it
 * stopped), or whose 5x5 system is not positive definite (the track then
 * gets KF_TRK_COV_NOT_PSD), hold NaN in smooth_state[0].  The smoothing runs
 * as two launches: the backward pass stores its prediction at every entry,
 * then one thread per (entry, track) combines it with the filtered state.
 * KF_ERR_ARG as kf_backward_fit, and for a missing or aliased smoothing
 * buffer. */
int kf_smooth_tracks(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                     const void *state_in, const void *cov_in, const int8_t *charge_in,
                     const uint32_t *fwd_status, const void *fwd_checkpoints,
                     const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                     int64_t n_hits, const void *hit_pos, const void *hit_cov,
                     const kf_geometry *geom, double cov_scale, int32_t max_len,
                     void *state_out, void *cov_out, int8_t *charge_out,
                     void *chi2, int32_t *ndf, uint32_t *trk_status,
                     void *smooth_state, void *smooth_cov, void *stream);

/* Final fit with outlier rejection (the final fit the paper names in Sec. 2.2,
 * step 4, and Sec. 4 as the next target of the method, where outlier
 * rejection is part of it; the rejection rule is this library's reading, the
 * paper gives none).  Rounds of refit and reject-the-worst on the hits of
 * each track:
 *   round i = 0 .. max_reject, for every track still open: the seeding and
 *   forward fit of kf_seed_fit_tracks (seed_mode) over the track's used hits
 *   (its valid hits not yet rejected), then the backward fit with smoothing
 *   of kf_smooth_tracks (cov_scale); every used hit gets its unbiased chi2,
 *   its chi2 against the estimate of the track made from its other hits:
 *   the forward prediction at the hit's entry (the hits before it) combined
 *   with the backward pass's prediction there (the hits after it), or the
 *   forward prediction alone at the last used entry; with (x, C) that
 *   estimate, r = m - H x, S = V + H C H^T, chi2 = r^T S^-1 r (FP64
 *   arithmetic; NaN where the combination is not positive definite or the
 *   entry was not reached).  In the linear model it equals the smoothed
 *   residual's r_s^T (V - H C_s H^T)^-1 r_s, but keeps its digits where the
 *   hit dominates the smoothed state.  If i < max_reject,
 *   the track was refitted, its worst used hit (largest chi2; the first entry
 *   among equals; NaN never counts) has chi2 > chi2_cut and the track keeps
 *   at least min_keep used hits without it, that hit is rejected and the
 *   track stays open; otherwise the track is closed with the round's
 *   backward-fit result.
 * Outputs (device, caller-owned): state_out [6][ld], cov_out [21][ld],
 * charge_out [n] -- the backward fit's state on the track's first used entry
 * -- chi2 [n] and ndf [n] of that backward pass (ndf = 2 * used hits - 5),
 * trk_status [n] (its status, plus KF_TRK_OUTLIER if a hit was rejected;
 * KF_TRK_BAD_INPUT for a track the forward fit could not seed or finish);
 * outlier [n_hits] (required): 1 for every rejected entry of the n tracks,
 * else 0; hit_chi2 [n_hits] (may be NULL): a used hit's unbiased chi2 in the
 * round its track closed, a rejected hit's in the round it was rejected,
 * NaN for holes, for entries not reached and for every hit of a track whose
 * forward fit stopped or could not be seeded in that round (the backward
 * pass did not refit it: there is no estimate from its other hits).  Entries outside the n tracks'
 * ranges are not written.
 * The rounds run on a context-owned workspace (about (34 + 55 * max_len)
 * values of the precision and 40 bytes per track, 10 values and 4 bytes per
 * hit; grown on demand, KF_ERR_NOMEM if that fails).  At most max_reject + 1
 * rounds: the first runs on all n tracks; after each round the tracks still
 * open are gathered (their hits with them) into a compact sub-batch that the
 * next round runs on, and the call waits for the stream once per round to
 * read that count into 8 bytes of pinned host memory the context allocates
 * at its first final fit (it returns once the last round is enqueued, or at
 * once when no track is left open).  The
 * forward fit runs in the context's launch shape for the precision (never in
 * a graph, never timed).
 * KF_ERR_ARG for chi2_cut not > 0 (NaN included), max_reject outside
 * [0, 64], min_keep outside [3, 64], a seed_mode other than 0 or 1, and the
 * argument errors of kf_seed_fit_tracks. */
int kf_final_fit(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld, int32_t seed_mode,
                 const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                 int64_t n_hits, const void *hit_pos, const void *hit_cov, const kf_geometry *geom,
                 double cov_scale, double chi2_cut, int32_t max_reject, int32_t min_keep, int32_t max_len,
                 void *state_out, void *cov_out, int8_t *charge_out, void *chi2, int32_t *ndf,
                 uint32_t *trk_status, uint8_t *outlier, void *hit_chi2, void *stream);

/* Duplicate removal among found tracks (the end of track finding, Sec. 2.2:
 * each seed is represented by its best candidate, and tracks found from
 * different seeds that share their hits are duplicates).  Track t carries one
 * hit id per layer of the plan, track_hits[t * hit_stride + l] for
 * l < n_layers (-1 a miss, -2 no candidate; ids >= 0 as kf_score_hits reports
 * them), and score[t * score_stride] (-inf: no candidate).  The best
 * candidates of kf_score_hits are rank 0: hit_stride = beam * plan_len,
 * score_stride = beam.  n(t) is the number of ids >= 0 of t; shared(t, u) the
 * number of layers at which t and u carry the same id >= 0.  t and u are
 * duplicates iff shared >= 1 and shared >= frac * min(n(t), n(u)) (exact: frac
 * as the float given, no rounding of the product); u outranks
 * t iff score(u) > score(t), or the scores are equal and u < t; t is removed
 * iff an outranking track is its duplicate (whether or not that one is
 * removed itself).  keep[n] (device, caller-owned): 1 kept, 0 removed (also
 * for a track without a candidate).  dup_of[n] (device, may be NULL): the
 * highest-ranked outranking duplicate of a removed track, else -1.  No two
 * kept tracks are duplicates.  The call sorts (hit id, track) pairs in a
 * context-owned workspace (about 16 bytes per track and layer plus the
 * sort's own; grown on demand, KF_ERR_NOMEM if that fails).  n = 0 is a
 * no-op.  KF_ERR_ARG for n < 0, n_layers outside [1, 64], hit_stride <
 * n_layers, score_stride < 1, frac outside (0, 1], n * n_layers >= 2^31, or
 * a missing pointer. */
int kf_remove_duplicates(kf_ctx *ctx, int64_t n, const int32_t *track_hits, int64_t hit_stride,
                         int32_t n_layers, const float *score, int64_t score_stride, float frac,
                         uint8_t *keep, int32_t *dup_of, void *stream);

/* Parameters of the combinatorial candidate search (kf_score_hits).  The
 * paper makes the window, the chi2 cut, the missed-layer limit and the
 * candidate score per-iteration parameters and standard functions (Sec. 3.2,
 * 3.3); these are the ones this search takes. */
typedef struct {
  int32_t beam;          /* candidates kept per seed, 1..8 */
  float chi2_max;        /* a hit is accepted iff its chi2 <= chi2_max (> 0) */
  float n_sigma;         /* window half-width in predicted standard deviations (> 0) */
  float hit_bonus;       /* child score = parent score + hit_bonus - chi2 */
  float miss_penalty;    /* miss child score = parent score - miss_penalty (>= 0) */
  int32_t max_miss;      /* a candidate with this many misses gets no miss child (0..100) */
  float sigma_rphi, sigma_z;  /* nominal hit resolution added to the window (cm, >= 0) */
  const float *win_min_rphi, *win_max_rphi, *win_min_z, *win_max_z; /* [n_layers] cm, HOST, 0 < min <= max */
  int32_t reuse_bins;    /* 1: the caller promises the pool's contents are unchanged since the last
                            call on this context; the pool is then binned again only if its
                            pointers, sizes, layer offsets or the geometry differ.  0: always bin. */
  int32_t overlap;       /* 1: each kept candidate picks up one detector-overlap hit per layer
                            (needs pool_module); 0: off */
  float overlap_bonus;   /* score of an overlap hit: + overlap_bonus - its chi2 (finite) */
} kf_search_params;

/* Combinatorial candidate search with chi2 scoring of the candidate hits
 * (the forward search of Sec. 2.2 over a layer plan, Sec. 3.1, with the
 * chi2 cut and candidate score of Sec. 3.2 and 3.3), FP32.
 * Every seed starts with one candidate (score 0).  For each layer L of
 * layer_plan (barrel layers), each live candidate is propagated to L with its
 * material (kf_propagate's crossing rule; a candidate without a crossing ends)
 * and opens the window
 *   w_rphi = clamp(n_sigma sqrt(t^T C_pos t + sigma_rphi^2), win_min_rphi[L], win_max_rphi[L]),
 *   w_z    = clamp(n_sigma sqrt(C_zz + sigma_z^2), win_min_z[L], win_max_z[L]),
 * t the transverse tangent of the layer at the predicted point; a pool hit of
 * L is inside iff |wrap(phi_hit - phi_pred)| <= w_rphi / R_L and
 * |z_hit - z_pred| <= w_z.  Each hit inside with chi2 <= chi2_max (the update's
 * chi2) gives a child scored parent + hit_bonus - chi2; a candidate with no
 * accepted hit gives one miss child scored parent - miss_penalty unless it has
 * max_miss misses already.  Per seed the children are ranked by (score
 * descending, hit id ascending with a miss after every hit, parent rank
 * ascending), the first `beam` are kept (their order is their rank) and the
 * kept ones with a hit get the Kalman update (kf_update) with it.
 * Overlap hits (params->overlap = 1; the single additional detector-overlap
 * hit a candidate may add on a layer, Sec. 2.2, picked from overlapping
 * modules of the layer, Sec. 3.1): right after a kept candidate's update
 * with its hit h, the hits of the same layer on a module with a higher id
 * than h's (pool_module; the order counts each pair of overlapping hits
 * once) inside the window around the updated state (the window
 * formulas above with the updated covariance) with chi2 <= chi2_max are its
 * overlap candidates; the one with the smallest chi2 (the lower hit id among
 * equals) is taken: a second update with it, and the candidate's score
 * gains overlap_bonus - chi2, which counts from the next layer's ranking on
 * (and in cand_score).
 * Seeds: seed_state[6][ld], seed_cov[21][ld], seed_charge[n], seed_layer[n]
 * (the layer each seed state is on; device).  layer_plan[plan_len] (HOST,
 * 1 <= plan_len <= 64).
 * Pool: pool_layer_offsets[n_layers + 1] (HOST; layer l owns hits
 * [off[l], off[l+1]), off[0] = 0, off[n_layers] = n_pool < 2^31),
 * pool_pos[3][n_pool], pool_cov[6][n_pool], pool_hit_id[n_pool] (device; the
 * ids, which must be distinct, are what the output reports and what breaks
 * ties), pool_module[n_pool] (device, the detector module of each hit; may
 * be NULL when params->overlap is 0).  The call bins the pool by (layer, phi, z) into a context-owned
 * workspace (about 64 bytes per pool hit and 9 bytes per candidate slot and plan layer; grown on
 * demand, KF_ERR_NOMEM if that fails), unless params->reuse_bins allows the
 * bins of the previous call to be used.  The per-layer parameters of the
 * plan are copied from host memory into that workspace on `stream` (a
 * host-to-device copy, synchronous with respect to the host) before the
 * search, which then runs as one kernel launch.
 * Outputs: cand_hits[n][beam][plan_len] (hit id, -1 = miss; -2 for every
 * entry of a rank the seed has no candidate for), cand_overlap
 * [n][beam][plan_len] (may be NULL: the overlap hit id of each layer, -1 for
 * none, -2 where cand_hits has -2), cand_score[n][beam]
 * (-inf for none), cand_state[6][n*beam] (column seed*beam + rank; the final
 * state after the last update; NaN for none; may be NULL), trk_status[n]
 * (overwritten: OR of the status bits of the seed's propagations and
 * updates).  n = 0 is a no-op. */
int kf_score_hits(kf_ctx *ctx, int64_t n, int64_t ld,
                  const float *seed_state, const float *seed_cov, const int8_t *seed_charge,
                  const int16_t *seed_layer,
                  const int16_t *layer_plan, int32_t plan_len,
                  const kf_geometry *geom, const kf_search_params *params,
                  const int32_t *pool_layer_offsets, int64_t n_pool,
                  const float *pool_pos, const float *pool_cov, const int32_t *pool_hit_id,
                  const int32_t *pool_module,
                  int32_t *cand_hits, int32_t *cand_overlap, float *cand_score, float *cand_state,
                  uint32_t *trk_status, void *stream);

/* Gradient of L = sum_t w_t chi2_t of kf_fit_tracks with respect to the seed
 * states, the hit positions and the per-layer alignment offsets, by a
 * hand-written reverse pass.  The paper has no such pass: it is an addition
 * built on the fit of Sec. 2.2, for alignment and for training code that
 * consumes the fit's chi2.  Every entry is reversed in three parts:
 * the update (whose Joseph form has the short form's derivative at the
 * optimal gain), the material noise Q(p), and the transport p' = g(p),
 * C' = F C F^T, where the path length s(p) enters by the implicit-function
 * rule ds/dp = d, so the crossing solve is not differentiated.  The forward
 * states are recomputed segment by segment from the checkpoints written by
 * kf_fit_tracks (same prec, seg, max_len and inputs) instead of being stored
 * for every entry.  The seed covariance and the hit covariances are
 * constants of L.
 * dL_dchi2[n] = w (NULL = all ones).  Outputs (overwritten):
 * grad_seed[6][ld]; grad_hit_pos[3][n_hits] (0 for holes, entries beyond
 * max_len and entries after the track stopped); grad_align[2][n_layers] or
 * NULL: a deterministic sum over barrel hits of (h_x g_y - h_y g_x)/R_l
 * (r-phi) and g_z (z), with g the hit gradient (disk layers get 0; with
 * align NULL it is the gradient at zero offsets).
 * trk_status[n]: the status kf_fit_tracks returned; tracks it stopped
 * (NO_CROSSING, NONFINITE, bad layer id) contribute only up to the entry
 * where they stopped.  Uses a context-owned buffer of 2 * 64 * ceil(n / 64)
 * values for the alignment reduction and, for seg > 1, n * (max_len - 1) * 29
 * values into which a pass before the reverse sweep recomputes the state
 * before every entry, each checkpoint segment once from its checkpoint
 * (allocated on first need, grown on demand, KF_ERR_NOMEM if that fails);
 * the checkpoints alone are what the caller keeps between the forward fit
 * and this call. */
int kf_fit_adjoint(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                   const void *seed_state, const void *seed_cov, const int8_t *seed_charge,
                   const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                   int64_t n_hits, const void *hit_pos, const void *hit_cov,
                   const kf_geometry *geom, const void *align,
                   const void *checkpoints, int32_t seg, int32_t max_len,
                   const void *dL_dchi2,
                   void *grad_seed, void *grad_hit_pos, void *grad_align,
                   const uint32_t *trk_status, void *stream);

/* kf_fit_adjoint for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, reverse kernel and results (to rounding: see below), but
 * the block partials of the alignment reduction live in a fixed device array
 * of this library (4 MiB per device, held until the process ends) instead of
 * the context's growing workspace, and each state of a checkpoint segment is
 * recomputed from the segment's checkpoint inside the reverse kernel when it
 * is needed, instead of being read from a buffer a refill kernel fills.  The
 * two run the same forward steps on the same values, compiled in two
 * kernels, so at seg > 1 the gradients can differ in the last bits of the
 * recomputed states (at seg 1 nothing is recomputed).  No hipMalloc, hipFree or other allocating call is made.
 * Limit: with grad_align != NULL, n_hits <= 16,777,216 (FP32) or 8,388,608
 * (FP64); larger batches get KF_ERR_ARG (grad_align == NULL needs no
 * scratch and has no limit).  Every call on one device shares that device's
 * array, which keeps the last call's contents (each call writes every
 * partial it reads, so nothing needs clearing): calls that overlap on one
 * device -- on two streams, two contexts or two host threads -- race and
 * must be serialised by the caller. */
int kf_fit_adjoint_noalloc(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                           const void *seed_state, const void *seed_cov, const int8_t *seed_charge,
                           const int32_t *hit_offsets, const int16_t *hit_layer, const uint8_t *hit_valid,
                           int64_t n_hits, const void *hit_pos, const void *hit_cov,
                           const kf_geometry *geom, const void *align,
                           const void *checkpoints, int32_t seg, int32_t max_len,
                           const void *dL_dchi2,
                           void *grad_seed, void *grad_hit_pos, void *grad_align,
                           const uint32_t *trk_status, void *stream);

/* ---- tilted planar modules ----------------------------------------------------
 * The Phase-2 layout of Sec. 3.1 describes each detector module by its
 * position, its normal vector and its phi-direction vector, and needs
 * propagation to such modules and Kalman updates on them.  A module here is
 * the plane through its centre c with unit normal n; its local frame is u
 * (the unit phi-direction, lying in the plane) and v = n x u.  A hit on a
 * module is the pair of local coordinates (m_u, m_v) = ((x - c).u, (x - c).v)
 * of its position x, with a 2x2 covariance packed (uu, vu, vv).
 * Module table: DEVICE array [10][n_modules] of the call's float type, rows
 * cx cy cz nx ny nz ux uy uz x_over_x0 (x/X0 at normal incidence); n and u
 * must be unit vectors with u.n = 0 (not checked: the table is on the device).
 * The struct itself is a HOST struct read during the call. */
typedef struct {
  int64_t n_modules;        /* >= 1; module ids are 0 .. n_modules - 1 */
  const void *modules;      /* DEVICE [10][n_modules] */
  double bz_tesla;          /* uniform solenoidal field, != 0 */
  double particle_mass_gev; /* mass hypothesis for the scattering angle, > 0 */
} kf_plane_geometry;

/* Propagate n tracks to the planes of their target modules: the helix of
 * kf_propagate to the root s > -1 cm of n.(x(s) - c) = 0 (Newton's method from
 * the straight-line estimate; accepted within 1e-9 cm of the plane in FP64,
 * within 64 * 2^-23 * (|cx| + |cy| + |cz| + 1) cm in FP32), the
 * surface-to-surface Jacobian F = G + g (ds/dp) with
 * ds/dp = -(n^T G_pos) / (n . g_pos), C' = F C F^T (the plane normal, in
 * position, is then a null vector and is imposed as one), and, if
 * apply_material, the Highland noise of x/X0 / |n . d| at the crossing (d the
 * unit direction).  target_module[n] (device); the other arrays as in
 * kf_propagate.  A track with no crossing is copied unchanged and gets
 * KF_TRK_NO_CROSSING; one whose module id is out of range, KF_TRK_BAD_INPUT. */
int kf_propagate_plane(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                       const void *state_in, const void *cov_in, const int8_t *charge,
                       const int32_t *target_module, const kf_plane_geometry *geom,
                       int32_t apply_material, void *state_out, void *cov_out, void *path_len,
                       uint32_t *trk_status, void *stream);

/* Kalman update with one local 2-D hit per track on its module (Sec. 3.1's
 * updates on tilted modules): H = [u^T 0; v^T 0] (2 x 6),
 * r = m - H (x - c), S = H C H^T + V (2 x 2), chi2 = r^T S^-1 r,
 * K = C H^T S^-1, p += K r, C = (I-KH) C (I-KH)^T + K V K^T (symmetric by
 * construction), then the charge flip and phi wrap of kf_update.  FP32 lanes
 * whose projected prior exceeds the hit covariance by more than 1e4
 * (tr(V^-1 H C H^T) > 1e4) are updated in FP64, and S^-1 is taken in FP64
 * when det S <= 0 or its condition estimate exceeds 1e6
 * (KF_TRK_FP64_FALLBACK).  state[6][ld], cov[21][ld], charge[n] in place;
 * module[n], hit_uv[2][ld], hit_cov_uv[3][ld] (uu, vu, vv); chi2[n] out;
 * trk_status[n] bits OR-ed in (KF_TRK_BAD_INPUT for a module id out of
 * range: the track is left unchanged with chi2 0). */
int kf_update_plane(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                    void *state, void *cov, int8_t *charge, const int32_t *module,
                    const void *hit_uv, const void *hit_cov_uv, const kf_plane_geometry *geom,
                    void *chi2, uint32_t *trk_status, void *stream);

/* Forward fit over tilted modules: the rules of kf_fit_tracks with a module
 * per entry.  Track t owns entries [hit_offsets[t], hit_offsets[t+1]):
 * hit_module[e] (int32), hit_valid[e] (0 = hole: propagation and material,
 * no update), hit_uv[2][n_hits], hit_cov_uv[3][n_hits].  The fit starts at
 * the first valid entry, where the seed sits on the hit; every entry, that
 * one included (a step of length ~0 onto the plane, which removes the seed
 * covariance's component along the normal), is propagated to with its
 * module's material (kf_propagate_plane) and, if valid, gets the local update
 * (kf_update_plane).  A failed crossing, a module id out of range
 * (KF_TRK_BAD_INPUT) or a step that turns the state non-finite (rolled back,
 * KF_TRK_NONFINITE) stops the track.  Outputs as in kf_fit_tracks:
 * state_out[6][ld], cov_out[21][ld], charge_out[n], chi2[n], ndf[n]
 * (= 2 * used hits - 5), trk_status[n] (overwritten; KF_TRK_BAD_INPUT also
 * for a track without a valid entry).  Seeds can be made with kf_make_seeds
 * from the hits' global positions (kf_plane_to_global). */
int kf_fit_plane_tracks(kf_ctx *ctx, kf_precision prec, int64_t n, int64_t ld,
                        const void *seed_state, const void *seed_cov, const int8_t *seed_charge,
                        const int32_t *hit_offsets, const int32_t *hit_module, const uint8_t *hit_valid,
                        int64_t n_hits, const void *hit_uv, const void *hit_cov_uv,
                        const kf_plane_geometry *geom, void *state_out, void *cov_out, int8_t *charge_out,
                        void *chi2, int32_t *ndf, uint32_t *trk_status, void *stream);

/* Global positions c + m_u u + m_v v of n_hits local hits (module[n_hits],
 * hit_uv[2][n_hits], device) into hit_pos[3][n_hits] (device), e.g. for
 * kf_make_seeds.  A module id out of range gives NaN coordinates. */
int kf_plane_to_global(kf_ctx *ctx, kf_precision prec, int64_t n_hits, const int32_t *module,
                       const void *hit_uv, const kf_plane_geometry *geom, void *hit_pos, void *stream);

/* Reserve the workspace of kf_fit_tracks' packed hit layout for up to
 * max_tracks tracks of up to max_len (1..64) entries (about
 * 80 * max_tracks * max_len bytes; replaces an earlier reservation;
 * max_tracks = 0 releases it).  KF_ERR_NOMEM if the allocation fails. */
int kf_reserve(kf_ctx *ctx, int64_t max_tracks, int32_t max_len);

/* ---- execution tuning (no effect on results) --------------------------------
 * Launch shape of kf_fit_tracks for one precision: threads per block (64, 128,
 * 192 or 256), persistent (1: a fixed grid of n_cu * blocks_per_cu blocks that
 * pull tiles of `block` tracks from a device counter; 0: one thread per
 * track), blocks_per_cu (1..32), waves (1 or 2: the kernel variant whose
 * register allocation allows at least that many waves per SIMD) and layout
 * (0: CSR in track order; 1: CSR in length-sorted order; 2: length-sorted
 * and packed; 3: CSR in track order staged through LDS by each wave; 4: CSR
 * in length-sorted order staged through LDS -- 1, 2 and 4 need a workspace
 * from kf_reserve, else 0 is used for 1 and 2 and 3 for 4).
 * Within a family of layouts (0-2 read the hits directly, 3-4 stage them
 * through LDS) every launch shape computes bit-identical results.  The two
 * families run the same arithmetic compiled into different loops, where the
 * compiler fuses different multiply-adds, so across them results agree to
 * rounding (FP64: about 1e-12 relative) and each meets the same accuracy
 * against the FP64 reference.  The choice is made by the autotuner of the
 * Python package for speed.  Stored in the context. */
int kf_set_fit_launch(kf_ctx *ctx, kf_precision prec, int32_t block, int32_t persistent, int32_t blocks_per_cu,
                      int32_t waves, int32_t layout);
int kf_get_fit_launch(const kf_ctx *ctx, kf_precision prec, int32_t *block, int32_t *persistent,
                      int32_t *blocks_per_cu, int32_t *waves, int32_t *layout);
/* Graph replay of kf_fit_tracks (enable = 1; 0 turns it off and frees the
 * cached graphs).  The first call with a given set of arguments (pointers,
 * sizes, precision, launch shape, layout) captures its whole launch sequence
 * -- sort and pack passes, counter reset, fit kernel -- into a hipGraph on a
 * context-owned stream; later calls with the same arguments replay it on the
 * caller's stream as one graph launch.  Any change of an argument captures
 * again; kf_reserve drops the cached graphs.  Results are identical to the
 * direct launches. */
int kf_set_fit_graph(kf_ctx *ctx, int32_t enable);

/* Kernel timing of kf_fit_tracks.  max_launches > 0 creates that many HIP
 * event pairs (at most 4096) and, from then on, records one pair on the
 * caller's stream around the fit kernel of each kf_fit_tracks call -- the
 * sort and pack passes are outside the pair; the persistent form's one-thread
 * tile-counter reset is inside -- until the pairs are used up (further calls
 * count as dropped).  While timing is on, kf_fit_tracks launches directly
 * even with graph replay enabled (the results are the same).  0 turns timing
 * off and frees the events.  Creating the events allocates; call it before a
 * timed region. */
int kf_set_kernel_timing(kf_ctx *ctx, int32_t max_launches);
/* Waits for the recorded fit kernels, returns the sum of their durations in
 * milliseconds and their number (dropped: the calls past the last pair; may
 * be NULL), and starts a new count with the same events. */
int kf_fit_kernel_time(kf_ctx *ctx, double *total_ms, int64_t *launches, int64_t *dropped);

/* Number of compute units of the context's device. */
int kf_device_cu_count(const kf_ctx *ctx, int32_t *n_cu);

#ifdef __cplusplus
}
#endif

#endif /* KF_H */
