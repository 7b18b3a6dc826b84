// Launch interfaces of the libcmif kernels (host side).  Every launcher
// enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "internal.h"

namespace cmif {

template <typename T>
struct FwdRowsArgs {
  const uint8_t* lab;  // nullable: every in-mask pixel has label 0
  const uint8_t* msk;  // nullable
  const float* memb;   // nullable: soft memberships [Q][H][W] replace lab
  cmif_stats* stats;   // nullable (soft: non-finite memberships)
  int H, W, Q, nb;
  int label0;          // hard: labels label0 .. label0+Q-1 are transformed
  RotArgs rot;
  C2<T>* xrow;
  long long angle_stride;
  const C2<T>* tw;  // P_w-entry table
  const uint32_t* gate;  // nullable: angle beta runs only if gate[beta] != 0
  long long src_stride;  // != 0: batch entry beta reads lab/msk + beta *
                         // src_stride (hard labels; volume slices)
};

template <typename T>
struct FwdColsArgs {
  const C2<T>* xrow;
  int H, tiles, Q, nb;
  long long x_angle_stride, x_label_stride;
  C2<T>* F;
  long long f_angle_stride, f_label_stride;
  const C2<T>* tw;  // P_h-entry table
  const uint32_t* gate;  // nullable: angle beta runs only if gate[beta] != 0
  // circular mode (circ_ha > 0): the H = S_h input rows are map rows of an
  // (h_a, h_b) displacement map, placed at their circular positions
  int circ_ha, circ_hb;
};

template <typename T>
struct PairColsArgs {
  const C2<T>* FA;     // nullable: FB already holds the product spectra
  long long fa_label_stride;
  const C2<T>* FB;
  long long fb_angle_stride, fb_label_stride;
  int QA, QB, ha, hb, sh, tiles, nb;
  C2<T>* Z;
  long long z_angle_stride, z_pair_stride;
  const C2<T>* tw;  // P_h-entry table
  int zg;           // Z layout group of the row kernels: z_group_rt<T>(P_w)
  // item mode (nullable): one (angle, a, b) per item, Z slot = item index
  const int4* items;
  const uint32_t* n_items;  // device count of valid items
  int max_items;            // grid size in item mode
  int xcd;                  // XCD-grouped workgroup order: 0 off, 1 on
  // launch shape (FP32 fused passes; 0 = default): half the default
  // columns per workgroup, radix cap 8 instead of 16, two labels of A per
  // workgroup (each F_B column read serves both products)
  int cpw_half, maxr, ba;
};

template <typename T>
struct PairRowsArgs {
  const C2<T>* Z;
  long long z_angle_stride, z_pair_stride;
  int QA, QB, ha, wa, hb, wb, sh, sw, ph, nb;
  const C2<T>* tw;       // P_w-entry table
  const double* logtab;  // 512 entries: log2(1 + j/256), 1/(1 + j/256)
  const double* xlogtab; // kXlogN entries: c log2 c
  int rows_per_wg;       // map rows handled by one workgroup
  int bpw;               // labels of B per team, 0 = pair_rows_config's choice
  int full_x;            // x displacements are the full set (wa, wb are the
                         // image widths): every lag outside the map has no
                         // overlap
  double* mi;            // nullable, [nb][sh][sw]
  long long mi_angle_stride;
  int32_t* n;            // nullable, [nb][sh][sw]
  long long n_angle_stride;
  uint32_t* maxn;        // [nb]
  uint32_t* flags;       // nullable, [nb][QA*QB]
  cmif_stats* stats;     // nullable
  // FP64 re-run (all nullable): angle beta runs only if gate[beta] != 0;
  // pair slot s = ovr[beta*QA*QB + pair] >= 0 takes its exact joint counts
  // from ovc[s][sh][sw] instead of the rounded transform.
  const uint32_t* gate;
  const int32_t* ovr;
  const int32_t* ovc;
};

template <typename T>
struct PairCountsArgs {
  const C2<T>* Z;
  long long z_angle_stride, z_pair_stride;
  int QA, QB, wa, wb, sh, sw, ph, nb;
  const C2<T>* tw;       // P_w-entry table
  int32_t* counts;       // nullable, [nb][QA*QB][sh][sw]
  long long counts_angle_stride;
  uint64_t* digest;      // nullable, [nb][QA*QB], accumulated (zero first)
  long long digest_index0;  // added to the map index of the digest weights
                            // (a slice of a larger map)
  double* values;        // nullable, [nb][QA*QB][sh][sw] unrounded values
  // item mode (nullable): Z holds one pair per item slot (no angle stride);
  // item s = (angle, a, b) writes to the (angle, a*QB+b) outputs above and,
  // when item_counts is given, to item_counts[s][sh][sw]
  const int4* items;
  const uint32_t* n_items;
  int32_t* item_counts;
};

// Soft row pass (real joints, no rounding).
template <typename T>
struct SoftRowsArgs {
  const C2<T>* Z;
  long long z_angle_stride, z_pair_stride;
  int QA, QB, wa, wb, sh, sw, ph, nb;
  const C2<T>* tw;       // P_w-entry table
  double* mi;            // nullable, [nb][sh][sw]
  long long mi_angle_stride;
  T* save;               // nullable, [nb][QA+QB+2][sh][sw] adjoint state
  long long save_angle_stride;
};

// Soft adjoint passes (one angle).
template <typename T>
struct SoftGradRowsArgs {
  const C2<T>* Z;        // pair columns of the forward pass
  long long z_pair_stride;
  int QA, QB, wa, wb, sh, sw, ph;
  const C2<T>* tw;       // P_w-entry table
  const double* grad_mi; // [sh][sw] dL/dMI
  const T* save;         // [QA+QB+2][sh][sw]
  C2<T>* ZG;             // out: half spectra of G, layout of Z
};

template <typename T>
struct SoftGradColsArgs {
  const C2<T>* GH;       // [QA*QB][P_w/2][P_h] 2D spectra of G
  const C2<T>* FO;       // other side's spectra [Q][P_w/2][P_h]
  long long f_label_stride;
  int QA, QB, H, tiles, side;  // side 0: gradient of A, 1: of B
  C2<T>* GX;             // out: [Q_side][tile][H][TW] row spectra
  long long gx_label_stride;
  const C2<T>* tw;       // P_h-entry table
};

template <typename T>
struct SoftGradOutArgs {
  const C2<T>* GX;
  long long gx_label_stride;
  int Q, H, W, ph;
  const uint8_t* msk;    // nullable
  const C2<T>* tw;       // P_w-entry table
  float* grad;           // out: [Q][H][W]
};

// Compaction of the pairs that need the FP64 re-run (one workgroup).
struct FbListArgs {
  const uint32_t* flags;  // [nb][QA*QB]
  int nb, QA, QB, force, capacity;
  int4* items;            // [capacity] (angle, a, b, 0), flag order
  uint32_t* n_items;      // min(#flagged, capacity)
  int32_t* ovr;           // [nb][QA*QB] item slot or -1
  uint32_t* gate;         // [nb + 1]: angle has items; [nb]: any item
  uint32_t* maxn;         // [nb], cleared for gated angles
  uint64_t* digest;       // nullable [nb][QA*QB], cleared for listed pairs
  cmif_stats* stats;      // nullable
};

struct ArgmaxArgs {
  const double* mi;      // [nb][sh][sw]
  const int32_t* n;      // [nb][sh][sw]
  long long angle_stride;
  const uint32_t* maxn;  // [nb]
  int sh, sw, nb, rows_per_chunk, nchunks;
  double gamma;
  ArgPartial* partial;   // [nb][nchunks]
};

struct ArgmaxFinalArgs {
  const ArgPartial* partial;
  int nb, nchunks, sw, ha, wa;
  int angle0;            // global index of the batch's first angle
  double angles[kMaxBatch];  // angle values of the batch (radians)
  cmif_best* per_angle;  // nullable, [n_angles] for this pair
  cmif_best* running;    // running best over batches
  int first_batch;
  cmif_best* best_out;   // nullable: final copy target
  int last_batch;
};

// Block shape of the pair row kernel: `bpw` labels of B per team, `nteams`
// teams, the launch bound `ntmax` >= nteams * team_for(P), and its LDS bytes.
struct PairRowsConfig {
  int bpw, nteams, ntmax;
  size_t lds;
};

// LDS of the row kernel: exchange buffers, log tables, S_A and N per x, the
// C_a slots and (FP32 two-wave teams) the split transform's two exchange
// buffers per team.
inline size_t pair_rows_lds(size_t elem_real, int P, int nteams) {
  const bool split = elem_real == sizeof(float) && team_for(P) == 128;
  const size_t px = (size_t)(P / lag_parts(P));  // lags of one workgroup
  return (size_t)nteams * lds_elems(P) * 2 * elem_real +
         (512 + kXlogN) * sizeof(double) + px * sizeof(double) +
         (1 + 2 * kFoldA) * px * sizeof(uint32_t) +
         (split ? (size_t)nteams * 2 * P * 2 * elem_real : 0);
}

// Default shape (the launch-shape tuner may pick another).  The labels per
// team set the per-lane state (BPW counters per point) and, through the
// team count, the launch bound and so the register budget per lane; the
// default takes the smallest bpw whose workgroup stays within a lane cap:
// FP32 512 lanes (two waves per SIMD, 256 registers), FP64 128 lanes (its
// state needs the 512 registers of one wave per SIMD; more teams spill).
// Without such a bpw, the one with the fewest lanes.  Measured: FP32 at
// P = 2048 with 8 labels per team 3.4x faster than with 4 (1024 lanes,
// 128 registers, 368 bytes of spills); FP64 at P = 1024 and 2048 with 16
// 2.4x faster than with 4.  false when no supported shape fits (LDS above
// 160 KiB or > 1024 lanes).
inline bool pair_rows_config(size_t elem_real, int P, int QB, PairRowsConfig* c) {
  const int team = team_for(P);
  const int cap = elem_real == sizeof(float) ? 512 : 128;
  bool found = false;
  for (int bpw : {4, 8, 16}) {
    const int nteams = (QB + bpw - 1) / bpw;
    const int nt = nteams * team;
    if (nt > 1024) continue;
    const size_t lds = pair_rows_lds(elem_real, P, nteams);
    if (lds > 160 * 1024) continue;
    // keep the first fit, replace it while it is above the cap
    if (found && c->nteams * team <= cap) break;
    if (found && nteams >= c->nteams) continue;
    c->bpw = bpw;
    c->nteams = nteams;
    c->ntmax = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
    c->lds = lds;
    found = true;
    if (nt <= cap) break;
  }
  return found;
}

// The shape for a given bpw (4, 8 or 16); false if it does not fit.
inline bool pair_rows_config_bpw(size_t elem_real, int P, int QB, int bpw,
                                 PairRowsConfig* c) {
  const int team = team_for(P);
  const int nteams = (QB + bpw - 1) / bpw;
  const int nt = nteams * team;
  if (nt > 1024 || (bpw != 4 && bpw != 8 && bpw != 16)) return false;
  const size_t lds = pair_rows_lds(elem_real, P, nteams);
  if (lds > 160 * 1024) return false;
  c->bpw = bpw;
  c->nteams = nteams;
  c->ntmax = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
  c->lds = lds;
  return true;
}

// Block shape of the soft row kernel (bpw 4 or 8, double accumulators).
struct SoftRowsConfig {
  int bpw, nteams, ntmax;
  size_t lds;
};

inline bool soft_rows_config(size_t elem_real, int P, int QB, SoftRowsConfig* c) {
  const int team = team_for(P);
  for (int bpw : {4, 8}) {
    const int nteams = (QB + bpw - 1) / bpw;
    const int nt = nteams * team;
    if (nt > 1024) continue;
    const size_t lds = (size_t)nteams * lds_elems(P) * 2 * elem_real +
                       2 * (size_t)P * sizeof(double);
    if (lds > 160 * 1024) continue;
    c->bpw = bpw;
    c->nteams = nteams;
    c->ntmax = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
    c->lds = lds;
    return true;
  }
  return false;
}

template <typename T>
hipError_t launch_fwd_rows(int P, const FwdRowsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_fwd_cols(int P, const FwdColsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_pair_cols(int P, const PairColsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_pair_rows(int P, const PairRowsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_pair_counts(int P, const PairCountsArgs<T>& a, hipStream_t st);

template <typename T>
hipError_t launch_soft_rows(int P, const SoftRowsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_soft_grad_rows(int P, const SoftGradRowsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_soft_grad_cols(int P, const SoftGradColsArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_soft_grad_out(int P, const SoftGradOutArgs<T>& a, hipStream_t st);

hipError_t launch_init_tables(void* tw32, void* tw64, int P, double* logtab,
                              double* xlogtab, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st);
hipError_t launch_check_labels(const uint8_t* lab, const uint8_t* msk,
                               long long n, int Q, cmif_stats* stats,
                               hipStream_t st);
hipError_t launch_argmax(const ArgmaxArgs& a, hipStream_t st);
hipError_t launch_fb_list(const FbListArgs& a, hipStream_t st);

// Plain schedule: conjugate spectral product of one pair of 2D half
// spectra, and the per-displacement entropy reduction over materialised
// count maps.
hipError_t launch_plain_product(const C2<double>* fa, const C2<double>* fb,
                                C2<double>* y, int half, int ph, hipStream_t st);
struct PlainEntropyArgs {
  const double* joint;   // [QA*QB][S]
  const double* marg_a;  // [QA][S]
  const double* marg_b;  // [QB][S]
  const double* nmap;    // [S]
  long long S;
  int QA, QB;
  double* mi;            // [S]
  int32_t* n;            // [S]
  uint32_t* maxn;        // [1]
};
hipError_t launch_plain_entropy(const PlainEntropyArgs& a, hipStream_t st);
hipError_t launch_argmax_final(const ArgmaxFinalArgs& a, hipStream_t st);
// Volumes (k_volume.hip): depth transforms of the slice spectra, and the
// per-pair product with the inverse depth transform.
template <typename T>
struct ZfftArgs {
  const C2<T>* F2;          // [z][label][pos], z < D
  long long z_stride;       // elements between slices
  long long label_stride2;  // elements between labels of one slice
  int D, Q, npos;           // slices, labels, positions (P_w/2 * P_h)
  C2<T>* F3;                // [label][k_z][pos]
  const C2<T>* tw;          // P_d-entry table
};
template <typename T>
struct ZpairArgs {
  const C2<T>* F3A;
  const C2<T>* F3B;
  int QA, QB, npos, ph, DA, DB;
  C2<T>* G;                 // [dz][pair][pos], dz < DA + DB - 1
  const C2<T>* tw;          // P_d-entry table
};
template <typename T>
hipError_t launch_zfft(int PD, const ZfftArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_zpair(int PD, const ZpairArgs<T>& a, hipStream_t st);
hipError_t launch_count_flags(const uint32_t* flags, int n, cmif_stats* stats,
                              hipStream_t st);
hipError_t launch_best3d(const cmif_best* b2, cmif_best3d* out, int sh, int da,
                         int ha, hipStream_t st);

hipError_t launch_two_stage_combine(const cmif_best& grid, cmif_best* best,
                                    cmif_best* grid_out, cmif_best* refine_out,
                                    int n_grid, hipStream_t st);

// Host-side hooks of the plan object for the allocation-free entry point
// (noalloc.hip): the plan's device and workspace sizes, and one eager
// cmif_compute pass on caller-placed workspaces (no graph capture, no
// tuning, no stage profiling: nothing that creates runtime objects).
cmif_status plan_noalloc_info(cmif_plan_t plan, int* device,
                              size_t* persistent, size_t* scratch,
                              uint32_t* flags, int32_t* mode);
cmif_status compute_eager(cmif_plan_t plan, const cmif_inputs* in,
                          const cmif_outputs* out, void* persistent,
                          void* scratch, hipStream_t st);
cmif_status set_error(cmif_status s, const char* msg);

// Mini-batch k-means quantisation (k_kmeans.hip).
struct KmeansArgs {
  const float* img;         // [n][m] pixels x channels
  const uint8_t* mask;      // [n] or nullptr (labels 0 outside)
  int64_t n;
  int m, k;
  const int32_t* init_idx;  // [k] pixels that seed the centres, or nullptr
  const int32_t* batches;   // [iters][batch] pixel indices
  int iters, batch;
  double* centers;          // [k][m] in (without init_idx) / out
  uint8_t* labels;          // [n]
  uint32_t* bad;            // out-of-range indices seen (may be nullptr)
};
hipError_t launch_kmeans(const KmeansArgs& a, hipStream_t st);

}  // namespace cmif
