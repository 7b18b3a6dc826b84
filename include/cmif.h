/*
 * cmif.h -- C ABI of libcmif, a gfx950 (MI355X) implementation of the
 * cross-mutual-information function (CMIF) and of MI-maximising global
 * alignment over rotations and displacements.
 *
 * What is computed (Ofverstedt, Lindblad, Sladoje, "Fast computation of
 * mutual information in the frequency domain with applications to global
 * multimodal image alignment"):
 *   - Sec. 2, Eq. 1-4: mutual information of two label images over their
 *     common domain, in bits, I = H_A + H_B - H_AB;
 *   - Eq. 5: CMIF(chi; A, B) = I(A, T_chi[B]) with T_chi[B](x) = B(x + chi);
 *   - Sec. 3.2, Eq. 8-12: joint counts C_ab(chi) are cross-correlations
 *     (Eq. 7) of masked level-set indicators, computed with FFTs; counts are
 *     rounded to integers, so the result equals the direct method's
 *     (Sec. 3.4); entropies of the relative histograms give the map;
 *   - Sec. 3.6, Alg. 1: global alignment; for every transform in the set,
 *     the displacement with the largest CMIF among those whose valid-point
 *     count N reaches gamma * max N, and across transforms a strictly larger
 *     value wins.
 *
 * Conventions that every entry point shares:
 *   - Images are row-major, uint8 labels in [0, Q) wherever their mask is
 *     set; masks are uint8 0/1 (a NULL mask means all ones).
 *   - Displacements: by default the full set of chi with a non-empty
 *     rectangle overlap, chi_y in [-(h_a-1), h_b-1], chi_x in [-(w_a-1),
 *     w_b-1]; a plan may restrict each image pair to a window [y0, y1] x
 *     [x0, x1] inside that set (the padded search window of Alg. 1).  A map
 *     has S_h x S_w entries, S_h = y1 - y0 + 1, S_w = x1 - x0 + 1 (full set:
 *     h_a + h_b - 1 and w_a + w_b - 1, y0 = -(h_a-1), x0 = -(w_a-1)), and
 *     entry [i][j] holds chi = (y0 + i, x0 + j).
 *   - Marginal counts and N are the exact integer sums of the rounded joint
 *     counts (identical to Eq. 10-11 in exact arithmetic).
 *   - MI is in bits, 0 where N = 0, with 0 log 0 = 0.
 *   - Rotation (the transform set Omega): B and M_B are resampled by
 *     nearest neighbour (Sec. 3.6) about B's centre with a fixed-point rule:
 *     c = round(cos(theta) 2^16), s = round(sin(theta) 2^16); output pixel
 *     (y, x) reads B at the source obtained by rotating the doubled centred
 *     coordinates (2x-(w_b-1), 2y-(h_b-1)) by [[c, -s], [s, c]] and rounding
 *     half up; a source outside B or on M_B = 0 gives mask 0.  theta = 0 is
 *     exactly the identity.  A result (angle, chi) means: A's pixel x
 *     corresponds to B's pixel src_theta(x + chi).
 *
 * Ownership and execution:
 *   - The caller owns every device buffer (inputs, outputs, workspaces).
 *     The library owns only host-side plan state.
 *   - Device pointers are HIP device addresses on the plan's device.  The
 *     stream argument is a hipStream_t passed as void* (NULL = the null
 *     stream).  Every call only enqueues work on that stream and returns;
 *     results are valid once the stream has been synchronised.
 *   - Host-detectable errors (bad arguments, unsupported sizes, workspace
 *     too small, wrong device) are returned before anything is enqueued.
 *     Conditions seen on the device (labels >= Q inside a mask, rounding
 *     residuals, fallbacks, non-finite soft inputs) are reported in
 *     cmif_stats.
 *   - No C++ exception crosses the ABI.  A plan is not safe for concurrent
 *     calls; calls of distinct plans may run concurrently on distinct
 *     streams with distinct workspaces.
 */
#ifndef CMIF_H
#define CMIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cmif_status {
  CMIF_OK = 0,
  CMIF_ERR_INVALID_ARGUMENT = 1,  /* NULL where required, bad sizes, Q, gamma */
  CMIF_ERR_UNSUPPORTED = 2,       /* valid but not supported (size too big) */
  CMIF_ERR_WORKSPACE_TOO_SMALL = 3,
  CMIF_ERR_DEVICE = 4,            /* a HIP runtime call failed */
  CMIF_ERR_WRONG_MODE = 5,        /* e.g. cmif_backward on a HARD plan */
  CMIF_ERR_NO_DEVICE = 6,         /* no usable gfx950 device */
  CMIF_ERR_HOST_MEMORY = 7
} cmif_status;

/* precision of the FFT stages (Sec. 3.2 "rounding ... to integers") */
enum {
  CMIF_PREC_FP32_ROUNDED = 0, /* FP32 FFTs, counts rounded, residual check,
                                 FP64 re-run of flagged label pairs: each
                                 pass of angles lists the (angle, a, b) whose
                                 residual reached 0.25 (up to the plan's
                                 fallback capacity, in angle-major pair
                                 order), recomputes their joint counts from
                                 FP64 spectra and reduces those angles
                                 again with the exact counts */
  CMIF_PREC_FP64 = 1          /* every FFT stage in FP64 (no re-run) */
};

enum {
  CMIF_MODE_HARD = 0, /* categorical labels (Eq. 8 level sets) */
  CMIF_MODE_SOFT = 1  /* real memberships in place of level sets */
};

enum {
  /* FP32_ROUNDED: list every label pair for the FP64 re-run, whatever its
     residual (pairs beyond the capacity are counted as overflow) */
  CMIF_FLAG_FORCE_FALLBACK = 1u << 0,
  /* keep the schedule host-visible: one kernel per stage and angle, no
     graph capture (a debugging aid; results are identical) */
  CMIF_FLAG_NO_GRAPH = 1u << 1,
  /* SOFT: keep what cmif_backward needs in the persistent workspace */
  CMIF_FLAG_SAVE_FOR_BACKWARD = 1u << 2,
  /* HARD + FP64 only: the paper-shaped schedule (Sec. 3.2, Eq. 15 transform
     count), kept as the comparator for the fused path: per angle, every
     level set and mask of A and B transformed on its own, then for each of
     the 1 + Q_A + Q_B + Q_A*Q_B correlations (Eq. 9-11) a product kernel, a
     column and a row inverse transform writing the real map to memory, one
     entropy kernel over all maps, and a host synchronisation before the next
     angle.  Same results; emits mi, n, best and per_angle (counts and
     digests are rejected) */
  CMIF_FLAG_PLAIN_SCHEDULE = 1u << 3,
  /* HARD, fused schedule: the first cmif_compute / cmif_align call times
     the candidate launch shapes of the pair row kernel (map rows per
     workgroup 1, 2, 4 x labels of B per team 4, 8, 16 where they fit: the
     row pass's pair blocking over B) and of the pair column kernel
     (XCD-grouped workgroup order on / off; FP32 also x the whole or half
     the default tile of columns per workgroup x radix cap 16 or 8 (the
     radix split of the column transform, e.g. 16x16x4 or 8x8x8x2 at 1024
     points) x one or two labels of A per workgroup (pair blocking over A:
     each F_B column read serves both products)): one untimed eager pass,
     then eager passes on the call's own buffers until every candidate of
     both kernels ran once; keeps the fastest per kernel, then runs the
     call.  With
     tune_cache_path the choice is read at cmif_plan when the file holds it
     (no timing) and written after timing.  Every candidate gives the same
     counts; MI may differ in the last bits (summation order).  Ignored for
     SOFT and the plain schedule */
  CMIF_FLAG_AUTOTUNE = 1u << 4
};

/* Plan description.  Every pointer is a host pointer read during cmif_plan
   only. */
typedef struct cmif_plan_desc {
  int32_t n_pairs;           /* image pairs handled by one call, >= 1 */
  const int32_t* h_a;        /* [n_pairs] heights of A, 1..4096 */
  const int32_t* w_a;        /* [n_pairs] widths of A, 1..4096 */
  const int32_t* h_b;        /* [n_pairs] heights of B, 1..4096 */
  const int32_t* w_b;        /* [n_pairs] widths of B, 1..4096 */
  int32_t q_a;               /* labels of A, 1..64 */
  int32_t q_b;               /* labels of B, 1..64 */
  int32_t n_angles;          /* rotation angles applied to B, >= 1 */
  const double* angles_rad;  /* [n_angles]; NULL means the single angle 0 */
  double gamma;              /* overlap fraction of Alg. 1, in [0, 1] */
  int32_t precision;         /* CMIF_PREC_* */
  int32_t mode;              /* CMIF_MODE_* */
  uint32_t flags;            /* CMIF_FLAG_* */
  int32_t device;            /* HIP device ordinal */
  int32_t angle_batch;       /* angles per pipeline pass, 0 = automatic */
  int32_t fallback_capacity; /* FP32_ROUNDED: label pairs per pass that the
                                FP64 re-run can take, 0 = min(64, pairs per
                                pass), at most 4096; sizes scratch */
  const char* tune_cache_path; /* CMIF_FLAG_AUTOTUNE: text file of tuned
                                  shapes, one line per plan key:
                                  "cmif-tune v1 gfx950 <Ph>x<Pw>:<S_h>x<S_w>...
                                  qa=<Q_A> qb=<Q_B> prec=<precision>
                                  batch=<angle batch> rows_per_wg=<1..8>
                                  bpw=<0|4|8|16> xcd=<0|1> half=<0|1>
                                  maxr=<16|8> ba=<1|2>" (FFT and map
                                  sizes of each image pair; the last three
                                  fields may be absent: defaults 0 16 1);
                                  unreadable or malformed lines are ignored,
                                  an unwritable file only skips the write;
                                  NULL = no file */
  const int32_t* window;     /* [n_pairs][4] displacement windows y0, y1,
                                x0, x1 (inclusive), each inside the full
                                set: -(h_a-1) <= y0 <= y1 <= h_b-1 and the
                                same for x; NULL = the full set for every
                                pair.  Maps, counts, digests, N, the gamma
                                threshold (gamma * max N over the window)
                                and the argmax cover the window only, and
                                the FFT side per axis is the smallest
                                supported length (see cmif_plan) >=
                                max(y1 + h_a, h_b - y0, h_a, h_b): the
                                least that keeps the window free of
                                circular aliasing and holds both images.
                                HARD mode, fused
                                schedule only (otherwise
                                CMIF_ERR_UNSUPPORTED) */
} cmif_plan_desc;

typedef struct cmif_plan_s* cmif_plan_t;

/* Device-side diagnostics, accumulated by every call that is given one
   (the caller zero-fills it before the first call it wants counted). */
typedef struct cmif_stats {
  uint32_t label_errors;      /* pixels inside a mask whose label is >= Q */
  uint32_t flagged_pairs;     /* (angle, image pair, label pair) items whose
                                 FP32 rounding residual reached 0.25 */
  uint32_t fallback_pairs;    /* items recomputed in FP64 */
  uint32_t fallback_overflow; /* flagged items beyond the re-run capacity */
  float max_residual;         /* max |y - rint(y)| over used displacements of
                                 the FP32 stages (before any re-run) */
  uint32_t nonfinite_inputs;  /* SOFT: NaN/Inf memberships seen */
  uint32_t unresolved_pairs;  /* items whose residual reached 0.25 but that
                                 the FP64 re-run did not take (beyond its
                                 capacity): their counts, and the MI of their
                                 angle, are not guaranteed exact.  0 means
                                 every count of the call is exact */
  uint32_t reserved;
} cmif_stats;

/* One alignment result (Alg. 1 output): the angle index into the plan's
   angle list, the displacement, its MI (bits) and its valid-point count. */
typedef struct cmif_best {
  int32_t angle_index;
  int32_t dy;
  int32_t dx;
  int32_t reserved;
  double angle_rad;
  double mi;
  int64_t n;
} cmif_best;

/* Inputs: host arrays with one DEVICE pointer per image pair. */
typedef struct cmif_inputs {
  const uint8_t* const* labels_a; /* HARD: [h_a][w_a] labels of A */
  const uint8_t* const* mask_a;   /* array may be NULL; entries may be NULL */
  const uint8_t* const* labels_b; /* HARD: [h_b][w_b] labels of B */
  const uint8_t* const* mask_b;
  const float* const* memb_a;     /* SOFT: [q_a][h_a][w_a] memberships of A */
  const float* const* memb_b;     /* SOFT: [q_b][h_b][w_b] memberships of B */
} cmif_inputs;

/* Outputs of cmif_compute: host arrays (or NULL) with one DEVICE pointer per
   image pair; each output is written for every angle of the plan. */
typedef struct cmif_outputs {
  double* const* mi;       /* [n_angles][S_h][S_w] MI map in bits */
  int32_t* const* n;       /* [n_angles][S_h][S_w] valid-point count N
                              (HARD: sum of the joint counts; SOFT: the
                              mask overlap M_A corr M_B, exact, which is
                              also the gamma threshold's N) */
  int32_t* const* counts;  /* HARD: [n_angles][q_a][q_b][S_h][S_w] joint */
  uint64_t* const* digest; /* HARD: [n_angles][q_a][q_b] order-free
                              fingerprint of each joint count map:
                              sum_chi C_ab(chi) * splitmix64(i*S_w + j)
                              modulo 2^64 (splitmix64 = Vigna's mixer
                              applied once to the map index) */
  cmif_best* best;         /* [n_pairs] Alg. 1 result over all angles */
  cmif_best* per_angle;    /* [n_pairs][n_angles] best per angle */
  cmif_stats* stats;       /* one struct, accumulated */
} cmif_outputs;

/* Builds a plan: validates the description, chooses FFT sizes (per axis
   the smallest of 128, 256, 512, 768, 1024, 1536, 2048, 4096 -- lengths
   2^k and 3 * 2^k -- that reaches S = h_a + h_b - 1, or with a window the
   alias-free size of the window and both image sides; above 4096
   CMIF_ERR_UNSUPPORTED: image sides above 2048 need a window, as in the
   paper's template-matching runs of Sec. 5.1 with a 4096 reference and a
   floating image of half its side; 4096-point sides are for
   CMIF_PREC_FP32_ROUNDED HARD plans without CMIF_FLAG_PLAIN_SCHEDULE, else
   CMIF_ERR_UNSUPPORTED),
   workspace layout and angle batching, and computes
   the fixed-point rotation coefficients.  Touches no device memory.  On
   success *out owns host memory released by cmif_plan_free.  Errors:
   CMIF_ERR_INVALID_ARGUMENT (NULL desc/out/size arrays, n_pairs < 1, sizes
   out of range, Q out of range, gamma outside [0, 1] or NaN, unknown
   precision/mode/flags, a window not inside the full set or empty),
   CMIF_ERR_UNSUPPORTED, CMIF_ERR_NO_DEVICE, CMIF_ERR_HOST_MEMORY. */
cmif_status cmif_plan(const cmif_plan_desc* desc, cmif_plan_t* out);

/* Releases host state; never frees caller memory.  NULL is ignored. */
void cmif_plan_free(cmif_plan_t plan);

/* Device workspace the caller must provide to cmif_compute / cmif_align /
   cmif_backward: `persistent` bytes that keep their content between calls
   of this plan (twiddle and log tables; SOFT forward state for
   cmif_backward) and `scratch` bytes that the call may overwrite.  Both
   buffers must be 256-byte aligned device memory of at least these sizes;
   every call receives the sizes it was given and rejects smaller ones with
   CMIF_ERR_WORKSPACE_TOO_SMALL before enqueuing anything. */
cmif_status cmif_workspace_size(cmif_plan_t plan, size_t* persistent,
                                size_t* scratch);

/* Launch sequence: unless the plan has CMIF_FLAG_NO_GRAPH (or the plain
   schedule, or stage profiling is on), cmif_compute and cmif_align record
   their whole launch sequence into a HIP graph on a private stream the first
   time and launch the graph on `stream`; later calls with the same device
   pointers (inputs, outputs, workspace, stream) replay it, new pointers
   capture again.  Results are identical either way; the contents behind the
   pointers may change freely between calls.

   CMIF maps (Eq. 5, Sec. 3.2) for every image pair and angle, plus the
   Alg. 1 results when out->best / out->per_angle are given.  Any output may
   be NULL.  HARD plans read labels/masks, SOFT plans memberships/masks (and
   ignore counts and digest).  SOFT maps are real-valued joints (no
   rounding, marginals and N of the MI from the joint sums, FP64 entropy
   sums); with CMIF_FLAG_SAVE_FOR_BACKWARD the call keeps N, log2 N - MI and
   the log2 marginals per displacement in the persistent workspace for
   cmif_backward (valid until the next cmif_compute of the plan). */
cmif_status cmif_compute(cmif_plan_t plan, const cmif_inputs* in,
                         const cmif_outputs* out, void* persistent,
                         size_t persistent_bytes, void* scratch,
                         size_t scratch_bytes, void* stream);

/* Global alignment (Alg. 1, lines 3-9): best[p] is the result for image
   pair p over all angles; per_angle (nullable) is [n_pairs][n_angles].
   No map is written.  stats is nullable. */
cmif_status cmif_align(cmif_plan_t plan, const cmif_inputs* in,
                       cmif_best* best, cmif_best* per_angle,
                       cmif_stats* stats, void* persistent,
                       size_t persistent_bytes, void* scratch,
                       size_t scratch_bytes, void* stream);

/* Global rigid alignment run twice (Sec. 3.6): (i) Alg. 1 over the plan's
   angles (the grid Omega), then (ii) for each image pair p Alg. 1 over the
   n_refine angles theta*_p + u_k * 2 pi / |Omega|, k < n_refine, around the
   grid's best angle theta*_p (0 when the grid kept the identity), with
   u_k = refine_offsets[k] in [-1, 1] (host array; the paper samples the
   interval uniformly at random, so the caller draws the u_k).  Across the
   stages a refinement result replaces the grid's only with a strictly
   larger MI (the refinement angles follow the grid in Alg. 1's order).
   HARD plans only.  best (device, [n_pairs]) receives the final result:
   angle_index < n_angles is a grid angle, n_angles + k the k-th refinement
   angle, -1 the identity; grid_best and refine_best (device, [n_pairs],
   nullable) receive the two stage results (refine_best's angle_index
   indexes the refinement angles).  stats (nullable) accumulates both
   stages.  The same workspaces as cmif_align.  Unlike the other calls this
   one waits for stage (i) on `stream` before it enqueues stage (ii), whose
   angles depend on theta*; results are valid once the stream has been
   synchronised.  Errors: as cmif_align, CMIF_ERR_WRONG_MODE for SOFT
   plans, CMIF_ERR_INVALID_ARGUMENT for n_refine outside 1..4096, NULL or
   out-of-range offsets. */
cmif_status cmif_align_two_stage(cmif_plan_t plan, const cmif_inputs* in,
                                 int32_t n_refine, const double* refine_offsets,
                                 cmif_best* best, cmif_best* grid_best,
                                 cmif_best* refine_best, cmif_stats* stats,
                                 void* persistent, size_t persistent_bytes,
                                 void* scratch, size_t scratch_bytes,
                                 void* stream);

/* The success measure of the paper's alignment experiments (Sec. 5.2): the
   mean Euclidean distance, in reference-image pixels, between the four
   corners of the reference image A taken as landmarks and the positions the
   alignment result recovers for them, against a known true transform.  An
   alignment counts as successful when this is below 2 % of the image
   width.  result (host) is an Alg. 1 result for images of sides h_a x w_a
   (A) and h_b x w_b (B); its correspondence maps A's pixel x to B's pixel
   R(theta)(x + chi - c_B) + c_B (the identity for angle_index -1), with
   c_B = ((w_b - 1)/2, (h_b - 1)/2) and R(theta) the rotation of cmif_plan's
   resampling rule in exact arithmetic.  truth (host, 6 doubles) is the true
   correspondence as an affine map of A's pixel (x, y) to B's:
   (truth[0] x + truth[1] y + truth[2], truth[3] x + truth[4] y + truth[5]).
   Both maps are rigid, so distances between the mapped corners in B equal
   those between the recovered and the true landmark positions in A.  Writes
   the mean distance to *error_px.  Host only, no device work.  Errors:
   CMIF_ERR_INVALID_ARGUMENT (NULL pointers, sides < 1). */
cmif_status cmif_corner_error(const cmif_best* result, int32_t h_a, int32_t w_a,
                              int32_t h_b, int32_t w_b, const double* truth,
                              double* error_px);

/* SOFT plans with CMIF_FLAG_SAVE_FOR_BACKWARD (which cmif_plan accepts for
   the single angle 0 only), after cmif_compute on the same inputs: given
   dL/dMI (grad_mi[p], device [n_angles][S_h][S_w] double), writes
   dL/dmemb_a (grad_a[p], [q_a][h_a][w_a] float) and dL/dmemb_b (grad_b[p],
   [q_b][h_b][w_b] float), overwriting them; masked-out pixels get 0.
   Either output array may be NULL to skip it.  Derivative: with G_ab(chi) =
   dL/dMI(chi) (log2(C_ab N / (C_a C_b)) - MI(chi)) / N(chi) (0 where C_ab
   or N is not positive), dL/dp_a(x) = sum_b sum_chi G_ab(chi) q_b(x + chi)
   and dL/dq_b(y) = sum_a sum_chi G_ab(chi) p_a(y - chi), evaluated by FFTs
   on the same grid as the forward.  Errors: CMIF_ERR_WRONG_MODE (HARD plan
   or no SAVE_FOR_BACKWARD), CMIF_ERR_INVALID_ARGUMENT (NULL memberships or
   grad_mi), workspace errors as cmif_compute. */
cmif_status cmif_backward(cmif_plan_t plan, const cmif_inputs* in,
                          const double* const* grad_mi, float* const* grad_a,
                          float* const* grad_b, void* persistent,
                          size_t persistent_bytes, void* scratch,
                          size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   cmif_compute with both workspaces placed in a library-owned device array
   of CMIF_NOALLOC_BYTES per GPU instead of caller buffers.  The caller
   still passes inputs and outputs exactly as for cmif_compute, and the
   results are the same.  The call allocates nothing: the array is a
   file-scope device variable that each GPU the library runs on holds from
   its first such call until the process ends; it is launched eagerly (no
   graph capture, no launch-shape tuning, no stage profiling).  Every call
   on one GPU shares that GPU's array and the array keeps the last call's
   contents (each call rebuilds its tables and clears its counters before
   use), so calls whose execution overlaps on one GPU race: order them on
   one stream or synchronise.  Errors: as cmif_compute, plus
   CMIF_ERR_UNSUPPORTED when the plan's persistent plus scratch workspace
   (256-byte rounded) exceeds CMIF_NOALLOC_BYTES or the plan is SOFT with
   CMIF_FLAG_SAVE_FOR_BACKWARD (no state is kept for cmif_backward). */
#define CMIF_NOALLOC_BYTES ((size_t)128 << 20)
cmif_status cmif_compute_noalloc(cmif_plan_t plan, const cmif_inputs* in,
                                 const cmif_outputs* out, void* stream);

/* Stage timing (a tracing aid).  While enabled on a plan, every kernel that
   a call enqueues is bracketed by two hipEvents recorded on the call's
   stream; cmif_profile_read waits for the recorded events and returns, per
   stage, the launch count, the summed event-to-event milliseconds and the
   algorithmic HBM bytes of those launches (the bytes the stage must move at
   minimum: its inputs read once and its outputs written once), then clears
   the records.  Stages: "check_labels", "fwd_rows", "fwd_cols",
   "pair_cols", "pair_rows", "pair_counts", "argmax", "fill", "tables",
   "fb_list", "fb_forward", "fb_pairs", "fb_rows" (FP64 re-run), "soft_grad"
   (adjoint), "plain" (plain schedule).  While profiling is enabled the
   calls launch eagerly (no graph).
   Disabled by default; enabling costs two event records per launch. */
typedef struct cmif_stage_time {
  char name[24];
  int32_t launches;
  int32_t reserved;
  double total_ms;
  double bytes;
} cmif_stage_time;

cmif_status cmif_profile_enable(cmif_plan_t plan, int32_t enable);

/* Writes up to `capacity` entries to `out` (host memory) and their number to
   *count. */
cmif_status cmif_profile_read(cmif_plan_t plan, cmif_stage_time* out,
                              int32_t capacity, int32_t* count);

/* What a plan chose, and how its calls ran so far. */
typedef struct cmif_plan_info {
  int32_t angle_batch;        /* angles per pipeline pass */
  int32_t fallback_capacity;  /* FP64 re-run slots per pass (0: none) */
  int32_t graph_captures;     /* launch sequences captured into HIP graphs */
  int32_t graph_replays;      /* calls that replayed a captured graph */
  int32_t fft_h, fft_w;       /* FFT lengths of image pair 0 */
  int32_t rows_per_wg;        /* pair row kernel: map rows per workgroup */
  int32_t labels_per_team;    /* pair row kernel: labels of B per team (0:
                                 the default shape) */
  int32_t xcd_grouping;       /* pair column kernel: XCD-grouped order (1,
                                 the default when every column length is a
                                 power of two) or launch order (0) */
  int32_t tuned;              /* 0 default shapes, 1 timed, 2 from the cache */
  int32_t tune_runs;          /* eager passes spent timing candidates */
  int32_t cols_half;          /* pair column kernel: half the default columns
                                 per workgroup (1) or the default (0) */
  int32_t cols_maxr;          /* pair column kernel: radix cap, 16 or 8 */
  int32_t cols_ba;            /* pair column kernel: labels of A per
                                 workgroup (pair blocking), 1 or 2 */
  int32_t reserved;
} cmif_plan_info;

/* Fills *info (host memory).  Errors: CMIF_ERR_INVALID_ARGUMENT on NULL. */
cmif_status cmif_plan_query(cmif_plan_t plan, cmif_plan_info* info);

/* Mini-batch k-means quantisation of an image into k labels: the QUANTIZE
   step of Alg. 1 (Sec. 3.6), with the mini-batch algorithm of Sculley
   (2010) that the paper uses.  Pixels are rows of `channels` FP32 values
   (device image[n_pixels][channels]); arithmetic is FP64.  Initial centres:
   the pixels init_idx[k] (device int32; Sculley's random examples), or,
   with init_idx NULL, the values already in `centers`.  Iteration t takes
   the batch batches[t][0..batch) (device int32 pixel indices, drawn by the
   caller), assigns each to its nearest centre under the centres at the
   start of the iteration, then applies the samples in batch order: the
   centre's count v increases by one and the centre moves to
   (1 - 1/v) c + (1/v) x, so every centre is the running mean of the
   samples assigned to it (no random reassignment of small clusters).
   Then every pixel gets the index of its nearest centre (squared
   Euclidean distance summed over channels in order, ties to the lowest
   index) in labels[n_pixels] (device uint8), 0 where mask (device uint8,
   NULL = all ones) is 0.  centers: device double[k][channels], in (without
   init_idx) and out.  bad_indices: device uint32 or NULL; each init or
   batch index outside [0, n_pixels) adds 1 there and is otherwise skipped
   (an initial centre from one is 0).  Enqueued on `stream` on the current
   device.  Errors: CMIF_ERR_INVALID_ARGUMENT (NULL image/centers/labels,
   batches NULL with iters > 0, n_pixels < 1, k outside 1..64, channels
   outside 1..8, batch outside 1..8192 with iters > 0, iters outside
   0..100000), CMIF_ERR_NO_DEVICE, CMIF_ERR_DEVICE. */
cmif_status cmif_kmeans(const float* image, const uint8_t* mask,
                        int64_t n_pixels, int32_t channels, int32_t k,
                        const int32_t* init_idx, const int32_t* batches,
                        int32_t iters, int32_t batch, double* centers,
                        uint8_t* labels, uint32_t* bad_indices, void* stream);

/* 3-D label volumes.  The paper's discussion states that the method
   carries over to nD: the correlations of Eq. 7 over three axes and the
   entropies of Eq. 12 per displacement chi = (dz, dy, dx) give the CMIF of
   two volumes A [d_a][h_a][w_a] and B [d_b][h_b][w_b] (row-major, z
   slowest) over every displacement with a non-empty box overlap, dz in
   [-(d_a-1), d_b-1] and likewise for y and x (translations only; the
   rotation set of Alg. 1 is not taken to 3-D).  FFT sides: in-plane the
   smallest of cmif_plan's lengths reaching h_a + h_b - 1 and w_a + w_b - 1,
   along depth the smallest of 32, 64, 128, 256, 512 reaching d_a + d_b - 1
   (otherwise CMIF_ERR_UNSUPPORTED). */
typedef struct cmif_volume_desc {
  int32_t d_a, h_a, w_a;  /* sides of A, 1..2048 */
  int32_t d_b, h_b, w_b;  /* sides of B, 1..2048 */
  int32_t q_a, q_b;       /* labels, 1..64 */
  double gamma;           /* overlap fraction of Alg. 1, in [0, 1] */
  int32_t precision;      /* CMIF_PREC_*: FP32_ROUNDED has no FP64 re-run
                             for volumes; label pairs whose rounding residual
                             reached 0.25 count in stats.unresolved_pairs */
  int32_t device;         /* HIP device ordinal */
} cmif_volume_desc;

/* Alg. 1 over a volume map: the eligible displacement with the largest
   MI, or the identity (0, 0, 0) with mi = 0 when none is positive. */
typedef struct cmif_best3d {
  int32_t dz, dy, dx, reserved;
  double mi;
  int64_t n;
} cmif_best3d;

/* Device workspace bytes of cmif_compute_volume for this description.
   Errors: CMIF_ERR_INVALID_ARGUMENT, CMIF_ERR_UNSUPPORTED as above. */
cmif_status cmif_volume_workspace_size(const cmif_volume_desc* desc,
                                       size_t* bytes);

/* The volume CMIF (one call, eager launches on `stream`): labels_a and
   labels_b are device uint8 volumes, masks device uint8 or NULL (all ones).
   Outputs, each device memory or NULL: mi and n [S_d][S_h][S_w] (S_d =
   d_a + d_b - 1, ...; entry [k][i][j] holds chi = (k - (d_a-1), i - (h_a-1),
   j - (w_a-1))), digest [q_a][q_b] (sum over the map of the joint count
   times splitmix64 of the row-major map index, modulo 2^64), best (Alg. 1,
   gamma * max N over the whole map), stats (accumulated).  workspace: at
   least cmif_volume_workspace_size bytes of 256-byte aligned device memory,
   overwritten.  Errors: those of the description, CMIF_ERR_INVALID_ARGUMENT
   (NULL labels or workspace), CMIF_ERR_WORKSPACE_TOO_SMALL,
   CMIF_ERR_NO_DEVICE, CMIF_ERR_DEVICE. */
cmif_status cmif_compute_volume(const cmif_volume_desc* desc,
                                const uint8_t* labels_a, const uint8_t* mask_a,
                                const uint8_t* labels_b, const uint8_t* mask_b,
                                double* mi, int32_t* n, uint64_t* digest,
                                cmif_best3d* best, cmif_stats* stats,
                                void* workspace, size_t workspace_bytes,
                                void* stream);

/* Static description of a status code. */
const char* cmif_status_string(cmif_status status);

/* Detail message of the last error returned to this thread ("" if none). */
const char* cmif_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CMIF_H */
