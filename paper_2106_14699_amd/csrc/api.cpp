// C ABI of libcmif: plan construction, workspace layout, host validation and
// the per-pair schedule of kernels (hard labels, FP32-rounded or FP64).
//
// Schedule for one image pair (all on the caller's stream):
//   tables      twiddles exp(2 pi i t/P) for each FFT length, log2 table
//   check       labels >= Q inside a mask -> stats.label_errors
//   A forward   rows (identity resampling) -> columns: F_A[label][c][k_y]
//   per batch of angles:
//     B forward rows (fixed-point NN rotation fused) -> columns
//     pair columns   conj(F_A,a) F_B,b and inverse FFT along y -> Z
//     pair rows      inverse FFT along x, rounding, residual check, fused
//                    entropy sums -> MI map, N map, max N, flags
//     FP64 re-run    (FP32 plans) list of flagged pairs -> gated FP64
//                    forward transforms, pair columns and counts of the
//                    listed pairs -> pair rows again for the gated angles,
//                    the listed pairs entering with exact counts
//     argmax         gamma-eligible argmax per angle, running best (Alg. 1)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"

using namespace cmif;

namespace {

thread_local std::string g_err;

cmif_status fail(cmif_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// FFT side: the smallest compiled length (2^k or 3 * 2^k, >= 128) that
// reaches v, or 0 when none does
int fft_size_at_least(int v) {
  for (int p : kFftSizes)
    if (p >= v) return p;
  return 0;
}

// Geometry of one image pair: image sides, map size (the displacement
// window), FFT sides, and the window's extents on either side of zero
// (e_a = 1 - y0, e_b = y1 + 1; the image sides for the full set), which the
// kernels take wherever they map circular lags to map rows and columns.
struct PairPlan {
  int ha, wa, hb, wb, sh, sw, ph, pw;
  int eha, ehb, ewa, ewb;
};

struct ScratchLayout {
  size_t xa, fa, xb, fb, z, mi, n, maxn, flags, partial, running, stats;
  // FP64 re-run (FP32 HARD plans only)
  size_t xa64, fa64, xb64, fb64, z64, cnt64, items, n_items, ovr, gate;
  // SOFT: FP64 mask-overlap pass (one "label" per image) and the adjoint
  size_t ov_xa, ov_fa, ov_xb, ov_fb, ov_z, zg, gh, gxa, gxb;
  // plain schedule: one row-spectrum buffer, Q_A+1 and Q_B+1 2D spectra, the
  // product, one pair's columns and all 1+Q_A+Q_B+Q_A*Q_B real maps
  size_t pl_x, pl_fa, pl_fb, pl_y, pl_z, pl_maps;
  size_t end;
};

enum Stage {
  ST_CHECK, ST_FWD_ROWS, ST_FWD_COLS, ST_PAIR_COLS, ST_PAIR_ROWS,
  ST_PAIR_COUNTS, ST_ARGMAX, ST_FILL, ST_TABLES, ST_FB_LIST, ST_FB_FWD,
  ST_FB_PAIR, ST_FB_ROWS, ST_SOFT_GRAD, ST_PLAIN, ST_COUNT
};
const char* const kStageNames[ST_COUNT] = {
    "check_labels", "fwd_rows", "fwd_cols", "pair_cols", "pair_rows",
    "pair_counts", "argmax", "fill", "tables", "fb_list", "fb_forward",
    "fb_pairs", "fb_rows", "soft_grad", "plain"};

struct ProfRec {
  int stage;
  hipEvent_t a, b;
  double bytes;
};

struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// One captured launch sequence, replayed while the call's pointers repeat.
struct GraphCache {
  bool valid = false;
  bool refused = false;      // the runtime refused a capture: stay eager
  std::vector<uintptr_t> key;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = nullptr;  // private capture stream (default priority)
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    valid = false;
    key.clear();
  }
  ~GraphCache() {
    reset();
    if (cs) (void)hipStreamDestroy(cs);
  }
};

}  // namespace

struct cmif_plan_s {
  cmif_plan_desc d;
  std::vector<PairPlan> pairs;
  std::vector<double> angles;
  std::vector<int32_t> rc, rs;
  int batch = 1;
  int fb_cap = 0;               // FP64 re-run items per pass (FP32 plans)
  std::vector<size_t> save_off; // SOFT + SAVE_FOR_BACKWARD: per pair
  std::vector<int> plens;       // distinct FFT lengths
  std::vector<size_t> tw_off;   // per plens entry: FP32 table, FP64 follows
  size_t logtab_off = 0;
  size_t xlog_off = 0;
  size_t persistent_bytes = 0;
  ScratchLayout lay{};
  size_t scratch_bytes = 0;
  int nchunks_max = 1;
  bool device_checked = false;
  bool windowed = false;        // built with per-pair displacement windows
  Profiler prof;
  GraphCache graphs[2];  // [0] cmif_compute, [1] cmif_align
  int graph_captures = 0;
  int graph_replays = 0;
  // launch shapes (defaults, or the autotuner's choice)
  int rows_per_wg = 1;   // pair row kernel: map rows per workgroup
  int bpw = 0;           // pair row kernel: labels of B per team (0: default)
  int xcd = 0;           // pair column kernel: XCD-grouped order
  int pc_half = 0;       // pair column kernel: half the default columns
  int pc_maxr = 16;      // pair column kernel: radix cap 16 or 8
  int pc_ba = 1;         // pair column kernel: labels of A per workgroup
  int def_xcd = 0;       // the default order (set by cmif_plan)
  int def_rpw = 1;       // the default rows per workgroup (set by cmif_plan)
  int tuned = 0;         // 0 default, 1 timed, 2 read from the cache
  int tune_runs = 0;
  std::string tune_path;
  std::string tune_key;
};

namespace {

size_t elem_bytes(const cmif_plan_s& P) {
  return P.d.precision == CMIF_PREC_FP64 ? sizeof(double2) : sizeof(float2);
}

// argmax chunks: about 256 per angle (a few map rows each)
int rows_per_chunk(int sh) { return (sh + 255) / 256; }

ScratchLayout layout_for(const cmif_plan_s& P, const PairPlan& g) {
  const size_t E = elem_bytes(P);
  const size_t qa = P.d.q_a, qb = P.d.q_b, nb = P.batch;
  const size_t half = g.pw / 2;
  ScratchLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up256(bytes); return r; };
  L.xa = take(qa * half * g.ha * E);
  L.fa = take(qa * half * g.ph * E);
  L.xb = take(nb * qb * half * g.hb * E);
  L.fb = take(nb * qb * half * g.ph * E);
  L.z = take(nb * z_pair_slots(qa * qb) * half * g.sh * E);
  L.mi = take(nb * (size_t)g.sh * g.sw * sizeof(double));
  L.n = take(nb * (size_t)g.sh * g.sw * sizeof(int32_t));
  L.maxn = take(nb * sizeof(uint32_t));
  L.flags = take(nb * qa * qb * sizeof(uint32_t));
  const int nchunks = (g.sh + rows_per_chunk(g.sh) - 1) / rows_per_chunk(g.sh);
  L.partial = take(nb * nchunks * sizeof(ArgPartial));
  L.running = take(sizeof(cmif_best));
  L.stats = take(sizeof(cmif_stats));
  if (P.fb_cap > 0) {
    const size_t E64 = sizeof(double2), cap = P.fb_cap;
    L.xa64 = take(qa * half * g.ha * E64);
    L.fa64 = take(qa * half * g.ph * E64);
    L.xb64 = take(nb * qb * half * g.hb * E64);
    L.fb64 = take(nb * qb * half * g.ph * E64);
    L.z64 = take(z_pair_slots(cap) * half * g.sh * E64);
    L.cnt64 = take(cap * (size_t)g.sh * g.sw * sizeof(int32_t));
    L.items = take(cap * sizeof(int4));
    L.n_items = take(sizeof(uint32_t));
    L.ovr = take(nb * qa * qb * sizeof(int32_t));
    L.gate = take((nb + 1) * sizeof(uint32_t));
  }
  if (P.d.flags & CMIF_FLAG_PLAIN_SCHEDULE) {
    const size_t E64 = sizeof(double2);
    L.pl_x = take(half * std::max(g.ha, g.hb) * E64);
    L.pl_fa = take((qa + 1) * half * g.ph * E64);
    L.pl_fb = take((qb + 1) * half * g.ph * E64);
    L.pl_y = take(half * g.ph * E64);
    L.pl_z = take(z_pair_slots(1) * half * g.sh * E64);
    L.pl_maps = take((1 + qa + qb + qa * qb) * (size_t)g.sh * g.sw * sizeof(double));
  }
  if (P.d.mode == CMIF_MODE_SOFT) {
    const size_t E64 = sizeof(double2);
    L.ov_xa = take(half * g.ha * E64);
    L.ov_fa = take(half * g.ph * E64);
    L.ov_xb = take(nb * half * g.hb * E64);
    L.ov_fb = take(nb * half * g.ph * E64);
    L.ov_z = take(nb * z_pair_slots(1) * half * g.sh * E64);
    if (P.d.flags & CMIF_FLAG_SAVE_FOR_BACKWARD) {
      L.zg = take(qa * qb * half * g.sh * E);
      L.gh = take(qa * qb * half * g.ph * E);
      L.gxa = take(qa * half * g.ha * E);
      L.gxb = take(qb * half * g.hb * E);
    }
  }
  L.end = o;
  return L;
}

int find_plen(const cmif_plan_s& P, int p) {
  for (size_t i = 0; i < P.plens.size(); ++i)
    if (P.plens[i] == p) return (int)i;
  return -1;
}

cmif_status check_device(cmif_plan_s* P) {
  if (P->device_checked) return CMIF_OK;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(CMIF_ERR_NO_DEVICE, "no HIP device");
  if (P->d.device < 0 || P->d.device >= n)
    return fail(CMIF_ERR_NO_DEVICE, "device ordinal out of range");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, P->d.device) != hipSuccess)
    return fail(CMIF_ERR_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CMIF_ERR_NO_DEVICE,
                std::string("libcmif is built for gfx950, device is ") +
                    prop.gcnArchName);
  P->device_checked = true;
  return CMIF_OK;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess) {
      ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

#define HIP_TRY(expr)                                                       \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess)                                                   \
      return fail(CMIF_ERR_DEVICE, std::string(#expr) + ": " +              \
                                       hipGetErrorString(_e));              \
  } while (0)

// Runs one launch; with profiling on, brackets it with events on `st`.
template <class F>
cmif_status launch_stage(cmif_plan_s& P, hipStream_t st, int stage,
                         double bytes, const char* what, F&& launch) {
  hipEvent_t ea = nullptr, eb = nullptr;
  if (P.prof.on) {
    ea = P.prof.take();
    eb = P.prof.take();
    if (!ea || !eb) return fail(CMIF_ERR_DEVICE, "hipEventCreate failed");
    if (hipEventRecord(ea, st) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventRecord failed");
  }
  const hipError_t e = launch();
  if (e != hipSuccess)
    return fail(CMIF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  if (P.prof.on) {
    if (hipEventRecord(eb, st) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventRecord failed");
    P.prof.recs.push_back(ProfRec{stage, ea, eb, bytes});
  }
  return CMIF_OK;
}

#define STAGE(stage, bytes, call)                                            \
  do {                                                                       \
    cmif_status _s = launch_stage(P, st, (stage), (double)(bytes), #call,   \
                                  [&]() { return (call); });                 \
    if (_s != CMIF_OK) return _s;                                            \
  } while (0)

struct CallOutputs {
  double* mi = nullptr;          // caller map for this pair or null
  int32_t* n = nullptr;
  int32_t* counts = nullptr;
  uint64_t* digest = nullptr;
  cmif_best* best = nullptr;
  cmif_best* per_angle = nullptr;  // [n_angles] for this pair
  cmif_stats* stats = nullptr;
};

template <typename T>
const C2<T>* twiddles(const cmif_plan_s& P, const uint8_t* pers, int len) {
  const size_t off = P.tw_off[find_plen(P, len)] +
                     (sizeof(T) == 8 ? (size_t)len * sizeof(float2) : 0);
  return reinterpret_cast<const C2<T>*>(pers + off);
}

// Forward transforms of the level sets (or soft memberships, when memb is
// given) of one image for `nb` angles (rotation r[b]); gate (nullable) skips
// angles with gate[b] == 0.
template <typename T>
cmif_status forward(cmif_plan_s& P, hipStream_t st, int stage_rows,
                     int stage_cols, const uint8_t* lab, const uint8_t* msk,
                     int H, int W, int Q, int nb, const int32_t* rc,
                     const int32_t* rs, const PairPlan& g, const uint8_t* pers,
                     C2<T>* x, C2<T>* f, const uint32_t* gate,
                     const float* memb = nullptr, cmif_stats* stats = nullptr,
                     int label0 = 0) {
  using CT = C2<T>;
  const int half = g.pw / 2;
  FwdRowsArgs<T> r{};
  r.lab = lab; r.msk = msk; r.memb = memb; r.stats = stats;
  r.H = H; r.W = W; r.Q = Q; r.nb = nb; r.label0 = label0;
  for (int b = 0; b < nb; ++b) { r.rot.c[b] = rc[b]; r.rot.s[b] = rs[b]; }
  r.xrow = x; r.angle_stride = (long long)Q * half * H;
  r.tw = twiddles<T>(P, pers, g.pw); r.gate = gate;
  const double in_bytes = memb ? (4.0 * Q + 1.0) * H * W : 2.0 * H * W;
  STAGE(stage_rows, nb * (in_bytes + (double)Q * half * H * sizeof(CT)),
        launch_fwd_rows<T>(g.pw, r, st));
  FwdColsArgs<T> c{};
  c.xrow = x; c.H = H; c.tiles = half / tile_width<T>(); c.Q = Q; c.nb = nb;
  c.x_angle_stride = (long long)Q * half * H;
  c.x_label_stride = (long long)half * H;
  c.F = f; c.f_angle_stride = (long long)Q * half * g.ph;
  c.f_label_stride = (long long)half * g.ph; c.tw = twiddles<T>(P, pers, g.ph);
  c.gate = gate;
  STAGE(stage_cols, nb * (double)Q * half * (H + g.ph) * sizeof(CT),
        launch_fwd_cols<T>(g.ph, c, st));
  return CMIF_OK;
}

// Saved soft state of pair p: [n_angles][Q_A+Q_B+2][S_h][S_w] in the
// transform precision.
size_t save_angle_elems(const cmif_plan_s& P, const PairPlan& g) {
  return (size_t)(P.d.q_a + P.d.q_b + 2) * g.sh * g.sw;
}

// Mask overlap N(chi) = sum_x M_A(x) M_B'(x + chi) in FP64 (one level set
// per image): the eligibility count of SOFT plans.  Writes n and maxn.
cmif_status overlap_pass(cmif_plan_s& P, const PairPlan& g, const ScratchLayout& L,
                         const uint8_t* ma, const uint8_t* mb, int a0, int nb,
                         bool first, int32_t* n_ptr, uint32_t* maxn,
                         uint32_t* flags, uint8_t* pers, uint8_t* scr,
                         hipStream_t st) {
  using C64 = C2<double>;
  const int half = g.pw / 2;
  C64* xa = reinterpret_cast<C64*>(scr + L.ov_xa);
  C64* fa = reinterpret_cast<C64*>(scr + L.ov_fa);
  C64* xb = reinterpret_cast<C64*>(scr + L.ov_xb);
  C64* fb = reinterpret_cast<C64*>(scr + L.ov_fb);
  C64* z = reinterpret_cast<C64*>(scr + L.ov_z);
  const int32_t id_c = 65536, id_s = 0;
  cmif_status s;
  if (first) {
    s = forward<double>(P, st, ST_FWD_ROWS, ST_FWD_COLS, nullptr, ma, g.ha,
                        g.wa, 1, 1, &id_c, &id_s, g, pers, xa, fa, nullptr);
    if (s != CMIF_OK) return s;
  }
  s = forward<double>(P, st, ST_FWD_ROWS, ST_FWD_COLS, nullptr, mb, g.hb, g.wb,
                      1, nb, &P.rc[a0], &P.rs[a0], g, pers, xb, fb, nullptr);
  if (s != CMIF_OK) return s;
  PairColsArgs<double> pc{};
  pc.FA = fa; pc.fa_label_stride = (long long)half * g.ph;
  pc.FB = fb; pc.fb_angle_stride = (long long)half * g.ph;
  pc.fb_label_stride = (long long)half * g.ph;
  pc.QA = 1; pc.QB = 1; pc.ha = g.eha; pc.hb = g.ehb; pc.sh = g.sh;
  pc.tiles = half / tile_width<double>(); pc.nb = nb; pc.Z = z;
  pc.z_angle_stride = (long long)z_pair_slots(1) * half * g.sh;
  pc.z_pair_stride = (long long)half * g.sh;
  pc.tw = twiddles<double>(P, pers, g.ph); pc.xcd = P.xcd;
  pc.zg = z_group_rt<double>(g.pw);
  STAGE(ST_PAIR_COLS, nb * (double)half * (g.ph + g.sh) * sizeof(C64),
        launch_pair_cols<double>(g.ph, pc, st));
  STAGE(ST_FILL, 4.0 * nb, launch_fill_u32(maxn, 0u, nb, st));
  STAGE(ST_FILL, 4.0 * nb, launch_fill_u32(flags, 0u, nb, st));
  PairRowsArgs<double> pr{};
  pr.Z = z; pr.z_angle_stride = pc.z_angle_stride; pr.z_pair_stride = pc.z_pair_stride;
  pr.QA = 1; pr.QB = 1; pr.wa = g.ewa; pr.wb = g.ewb;
  pr.sh = g.sh; pr.sw = g.sw; pr.ph = g.ph; pr.nb = nb;
  pr.tw = twiddles<double>(P, pers, g.pw);
  pr.logtab = reinterpret_cast<const double*>(pers + P.logtab_off);
  pr.xlogtab = reinterpret_cast<const double*>(pers + P.xlog_off);
  pr.rows_per_wg = 2; pr.mi = nullptr; pr.n = n_ptr;
  pr.full_x = g.ewa == g.wa && g.ewb == g.wb;
  pr.n_angle_stride = (long long)g.sh * g.sw; pr.maxn = maxn; pr.flags = flags;
  STAGE(ST_PAIR_ROWS, nb * ((double)half * g.sh * sizeof(C64) + 4.0 * g.sh * g.sw),
        launch_pair_rows<double>(g.pw, pr, st));
  return CMIF_OK;
}

template <typename T>
cmif_status run_pair(cmif_plan_s& P, int p, const uint8_t* la,
                     const uint8_t* ma, const uint8_t* lb, const uint8_t* mb,
                     const float* pa, const float* pb, const CallOutputs& o,
                     uint8_t* pers, uint8_t* scr, hipStream_t st) {
  const bool soft = P.d.mode == CMIF_MODE_SOFT;
  using CT = C2<T>;
  const PairPlan& g = P.pairs[p];
  const ScratchLayout L = layout_for(P, g);
  const int qa = P.d.q_a, qb = P.d.q_b;
  const int half = g.pw / 2;
  const int TW = tile_width<T>();
  const int tiles = half / TW;
  const bool fp64 = sizeof(T) == 8;
  const int iw = find_plen(P, g.pw), ih = find_plen(P, g.ph);
  const CT* tw_w = reinterpret_cast<const CT*>(
      pers + P.tw_off[iw] + (fp64 ? (size_t)g.pw * sizeof(float2) : 0));
  const CT* tw_h = reinterpret_cast<const CT*>(
      pers + P.tw_off[ih] + (fp64 ? (size_t)g.ph * sizeof(float2) : 0));
  const double* logtab = reinterpret_cast<const double*>(pers + P.logtab_off);
  const double* xlogtab = reinterpret_cast<const double*>(pers + P.xlog_off);
  CT* xa = reinterpret_cast<CT*>(scr + L.xa);
  CT* fa = reinterpret_cast<CT*>(scr + L.fa);
  CT* xb = reinterpret_cast<CT*>(scr + L.xb);
  CT* fb = reinterpret_cast<CT*>(scr + L.fb);
  CT* z = reinterpret_cast<CT*>(scr + L.z);
  double* mi_s = reinterpret_cast<double*>(scr + L.mi);
  int32_t* n_s = reinterpret_cast<int32_t*>(scr + L.n);
  uint32_t* maxn = reinterpret_cast<uint32_t*>(scr + L.maxn);
  uint32_t* flags = reinterpret_cast<uint32_t*>(scr + L.flags);
  ArgPartial* partial = reinterpret_cast<ArgPartial*>(scr + L.partial);
  cmif_best* running = reinterpret_cast<cmif_best*>(scr + L.running);
  cmif_stats* stats = o.stats;

  if (stats && !soft) {
    STAGE(ST_CHECK, 2.0 * g.ha * g.wa,
          launch_check_labels(la, ma, (long long)g.ha * g.wa, qa, stats, st));
    STAGE(ST_CHECK, 2.0 * g.hb * g.wb,
          launch_check_labels(lb, mb, (long long)g.hb * g.wb, qb, stats, st));
  }

  // forward transforms of A's level sets (identity resampling)
  const int32_t id_c = 65536, id_s = 0;
  {
    cmif_status s = forward<T>(P, st, ST_FWD_ROWS, ST_FWD_COLS, la, ma, g.ha,
                               g.wa, qa, 1, &id_c, &id_s, g, pers, xa, fa,
                               nullptr, pa, stats);
    if (s != CMIF_OK) return s;
  }
  const int nang = (int)P.angles.size();
  const long long map_stride = (long long)g.sh * g.sw;
  const int rpc = rows_per_chunk(g.sh);
  const int nchunks = (g.sh + rpc - 1) / rpc;
  const bool want_best = o.best != nullptr || o.per_angle != nullptr;
  for (int a0 = 0; a0 < nang; a0 += P.batch) {
    const int nb = std::min(P.batch, nang - a0);
    {
      cmif_status s = forward<T>(P, st, ST_FWD_ROWS, ST_FWD_COLS, lb, mb, g.hb,
                                 g.wb, qb, nb, &P.rc[a0], &P.rs[a0], g, pers, xb,
                                 fb, nullptr, pb, stats);
      if (s != CMIF_OK) return s;
    }

    STAGE(ST_FILL, 4.0 * nb, launch_fill_u32(maxn, 0u, nb, st));
    STAGE(ST_FILL, 4.0 * nb * qa * qb,
          launch_fill_u32(flags, 0u, (long long)nb * qa * qb, st));

    PairColsArgs<T> pc{};
    pc.FA = fa; pc.fa_label_stride = (long long)half * g.ph;
    pc.FB = fb; pc.fb_angle_stride = (long long)qb * half * g.ph;
    pc.fb_label_stride = (long long)half * g.ph;
    pc.QA = qa; pc.QB = qb; pc.ha = g.eha; pc.hb = g.ehb; pc.sh = g.sh;
    pc.tiles = tiles; pc.nb = nb; pc.Z = z;
    pc.z_angle_stride = (long long)z_pair_slots(qa * qb) * half * g.sh;
    pc.z_pair_stride = (long long)half * g.sh; pc.tw = tw_h; pc.xcd = P.xcd;
    pc.zg = z_group_rt<T>(g.pw);
    pc.cpw_half = P.pc_half; pc.maxr = P.pc_maxr; pc.ba = P.pc_ba;
    // A's spectra once per launch, B's once per angle, every pair's columns
    STAGE(ST_PAIR_COLS,
          (double)qa * half * g.ph * sizeof(CT) +
              nb * ((double)qb * half * g.ph + (double)qa * qb * half * g.sh) * sizeof(CT),
          launch_pair_cols<T>(g.ph, pc, st));

    double* mi_ptr = o.mi ? o.mi + a0 * map_stride : mi_s;
    int32_t* n_ptr = o.n ? o.n + a0 * map_stride : n_s;
    if (soft) {
      SoftRowsArgs<T> sr{};
      sr.Z = z; sr.z_angle_stride = pc.z_angle_stride; sr.z_pair_stride = pc.z_pair_stride;
      sr.QA = qa; sr.QB = qb; sr.wa = g.ewa; sr.wb = g.ewb; sr.sh = g.sh; sr.sw = g.sw;
      sr.ph = g.ph; sr.nb = nb; sr.tw = tw_w;
      sr.mi = mi_ptr; sr.mi_angle_stride = map_stride;
      const bool save = (P.d.flags & CMIF_FLAG_SAVE_FOR_BACKWARD) != 0;
      const size_t sae = save_angle_elems(P, g);
      sr.save = save ? reinterpret_cast<T*>(pers + P.save_off[p]) + a0 * sae : nullptr;
      sr.save_angle_stride = (long long)sae;
      STAGE(ST_PAIR_ROWS,
            nb * ((double)qa * qb * half * g.sh * sizeof(CT) + 8.0 * g.sh * g.sw +
                  (save ? (double)sizeof(T) * sae : 0.0)),
            launch_soft_rows<T>(g.pw, sr, st));
      if (o.n || want_best) {
        cmif_status s = overlap_pass(P, g, L, ma, mb, a0, nb, a0 == 0, n_ptr,
                                     maxn, flags, pers, scr, st);
        if (s != CMIF_OK) return s;
      }
    }
    PairRowsArgs<T> pr{};
    pr.Z = z; pr.z_angle_stride = pc.z_angle_stride; pr.z_pair_stride = pc.z_pair_stride;
    pr.QA = qa; pr.QB = qb; pr.wa = g.ewa; pr.wb = g.ewb;
    pr.sh = g.sh; pr.sw = g.sw; pr.ph = g.ph; pr.nb = nb; pr.tw = tw_w;
    pr.logtab = logtab; pr.xlogtab = xlogtab; pr.rows_per_wg = P.rows_per_wg;
    pr.bpw = P.bpw;
    pr.full_x = g.ewa == g.wa && g.ewb == g.wb;
    pr.mi = mi_ptr; pr.mi_angle_stride = map_stride;
    pr.n = n_ptr; pr.n_angle_stride = map_stride; pr.maxn = maxn; pr.flags = flags;
    pr.stats = stats;
    // every pair's columns read once, MI and N maps written once
    if (!soft)
      STAGE(ST_PAIR_ROWS,
            nb * ((double)qa * qb * half * g.sh * sizeof(CT) + 12.0 * g.sh * g.sw),
            launch_pair_rows<T>(g.pw, pr, st));
    if (!soft && (o.counts || o.digest)) {
      PairCountsArgs<T> pk{};
      pk.Z = z; pk.z_angle_stride = pc.z_angle_stride; pk.z_pair_stride = pc.z_pair_stride;
      pk.QA = qa; pk.QB = qb; pk.wa = g.ewa; pk.wb = g.ewb; pk.sh = g.sh; pk.sw = g.sw;
      pk.ph = g.ph; pk.nb = nb; pk.tw = tw_w;
      pk.counts = o.counts ? o.counts + (long long)a0 * qa * qb * map_stride : nullptr;
      pk.counts_angle_stride = (long long)qa * qb * map_stride;
      pk.digest = o.digest ? o.digest + (long long)a0 * qa * qb : nullptr;
      STAGE(ST_PAIR_COUNTS,
            nb * (double)qa * qb * (half * g.sh * sizeof(CT) + (o.counts ? 4.0 * g.sh * g.sw : 0.0)),
            launch_pair_counts<T>(g.pw, pk, st));
    }

    if (!soft && !fp64 && P.fb_cap > 0) {
      // FP64 re-run of the flagged pairs (everything stays on the device:
      // the list decides, the gates skip, nothing returns to the host)
      using C64 = C2<double>;
      C64* xa64 = reinterpret_cast<C64*>(scr + L.xa64);
      C64* fa64 = reinterpret_cast<C64*>(scr + L.fa64);
      C64* xb64 = reinterpret_cast<C64*>(scr + L.xb64);
      C64* fb64 = reinterpret_cast<C64*>(scr + L.fb64);
      C64* z64 = reinterpret_cast<C64*>(scr + L.z64);
      int32_t* cnt64 = reinterpret_cast<int32_t*>(scr + L.cnt64);
      int4* items = reinterpret_cast<int4*>(scr + L.items);
      uint32_t* n_items = reinterpret_cast<uint32_t*>(scr + L.n_items);
      int32_t* ovr = reinterpret_cast<int32_t*>(scr + L.ovr);
      uint32_t* gate = reinterpret_cast<uint32_t*>(scr + L.gate);
      uint64_t* dig = o.digest ? o.digest + (long long)a0 * qa * qb : nullptr;
      FbListArgs fl{};
      fl.flags = flags; fl.nb = nb; fl.QA = qa; fl.QB = qb;
      fl.force = (P.d.flags & CMIF_FLAG_FORCE_FALLBACK) ? 1 : 0;
      fl.capacity = P.fb_cap; fl.items = items; fl.n_items = n_items;
      fl.ovr = ovr; fl.gate = gate; fl.maxn = maxn; fl.digest = dig;
      fl.stats = stats;
      STAGE(ST_FB_LIST, 4.0 * nb * qa * qb * 2, launch_fb_list(fl, st));
      cmif_status s = forward<double>(P, st, ST_FB_FWD, ST_FB_FWD, la, ma, g.ha,
                                      g.wa, qa, 1, &id_c, &id_s, g, pers, xa64,
                                      fa64, gate + nb);
      if (s != CMIF_OK) return s;
      s = forward<double>(P, st, ST_FB_FWD, ST_FB_FWD, lb, mb, g.hb, g.wb, qb, nb,
                          &P.rc[a0], &P.rs[a0], g, pers, xb64, fb64, gate);
      if (s != CMIF_OK) return s;
      const int tiles64 = half / tile_width<double>();
      PairColsArgs<double> qc{};
      qc.FA = fa64; qc.fa_label_stride = (long long)half * g.ph;
      qc.FB = fb64; qc.fb_angle_stride = (long long)qb * half * g.ph;
      qc.fb_label_stride = (long long)half * g.ph;
      qc.QA = qa; qc.QB = qb; qc.ha = g.eha; qc.hb = g.ehb; qc.sh = g.sh;
      qc.tiles = tiles64; qc.nb = nb; qc.Z = z64; qc.z_angle_stride = 0;
      qc.z_pair_stride = (long long)half * g.sh;
      qc.tw = twiddles<double>(P, pers, g.ph); qc.zg = z_group_rt<double>(g.pw);
      qc.items = items; qc.n_items = n_items; qc.max_items = P.fb_cap;
      STAGE(ST_FB_PAIR, 0.0, launch_pair_cols<double>(g.ph, qc, st));
      PairCountsArgs<double> qk{};
      qk.Z = z64; qk.z_angle_stride = 0; qk.z_pair_stride = qc.z_pair_stride;
      qk.QA = qa; qk.QB = qb; qk.wa = g.ewa; qk.wb = g.ewb; qk.sh = g.sh;
      qk.sw = g.sw; qk.ph = g.ph; qk.nb = 1;
      qk.tw = twiddles<double>(P, pers, g.pw);
      qk.counts = o.counts ? o.counts + (long long)a0 * qa * qb * map_stride : nullptr;
      qk.counts_angle_stride = (long long)qa * qb * map_stride;
      qk.digest = dig; qk.items = items; qk.n_items = n_items;
      qk.item_counts = cnt64;
      STAGE(ST_FB_PAIR, 0.0, launch_pair_counts<double>(g.pw, qk, st));
      PairRowsArgs<T> rr = pr;
      rr.flags = nullptr;
      rr.stats = nullptr;
      rr.gate = gate; rr.ovr = ovr; rr.ovc = cnt64;
      STAGE(ST_FB_ROWS, 0.0, launch_pair_rows<T>(g.pw, rr, st));
    }

    if (want_best) {
      ArgmaxArgs am{};
      am.mi = mi_ptr; am.n = n_ptr; am.angle_stride = map_stride; am.maxn = maxn;
      am.sh = g.sh; am.sw = g.sw; am.nb = nb; am.rows_per_chunk = rpc;
      am.nchunks = nchunks; am.gamma = P.d.gamma; am.partial = partial;
      STAGE(ST_ARGMAX, nb * 12.0 * g.sh * g.sw, launch_argmax(am, st));
      ArgmaxFinalArgs af{};
      af.partial = partial; af.nb = nb; af.nchunks = nchunks; af.sw = g.sw;
      af.ha = g.eha; af.wa = g.ewa; af.angle0 = a0;
      for (int b = 0; b < nb; ++b) af.angles[b] = P.angles[a0 + b];
      af.per_angle = o.per_angle; af.running = running;
      af.first_batch = a0 == 0; af.best_out = o.best;
      af.last_batch = a0 + nb >= nang;
      STAGE(ST_ARGMAX, nb * (double)nchunks * sizeof(ArgPartial),
            launch_argmax_final(af, st));
    }
  }
  return CMIF_OK;
}

// The paper-shaped comparator (CMIF_FLAG_PLAIN_SCHEDULE): per angle, each
// of the Q_A + Q_B + 2 forward transforms (level sets and masks, Eq. 8) and
// each of the 1 + Q_A + Q_B + Q_A Q_B correlations (Eq. 9-11) runs as its own
// launches (product, column inverse, row inverse writing the real map), then
// one entropy kernel reads every map (Eq. 12) and the host waits for the
// angle before starting the next.
cmif_status run_pair_plain(cmif_plan_s& P, int p, const uint8_t* la,
                           const uint8_t* ma, const uint8_t* lb,
                           const uint8_t* mb, const CallOutputs& o,
                           uint8_t* pers, uint8_t* scr, hipStream_t st) {
  using C64 = C2<double>;
  const PairPlan& g = P.pairs[p];
  const ScratchLayout L = layout_for(P, g);
  const int qa = P.d.q_a, qb = P.d.q_b;
  const int half = g.pw / 2;
  const long long S = (long long)g.sh * g.sw;
  const long long fstride = (long long)half * g.ph;
  C64* x = reinterpret_cast<C64*>(scr + L.pl_x);
  C64* fa = reinterpret_cast<C64*>(scr + L.pl_fa);  // [qa] level sets, [qa] = mask
  C64* fb = reinterpret_cast<C64*>(scr + L.pl_fb);
  C64* y = reinterpret_cast<C64*>(scr + L.pl_y);
  C64* z = reinterpret_cast<C64*>(scr + L.pl_z);
  double* maps = reinterpret_cast<double*>(scr + L.pl_maps);
  double* joint = maps;                        // [qa*qb][S]
  double* marg_a = maps + (long long)qa * qb * S;
  double* marg_b = marg_a + (long long)qa * S;
  double* nmap = marg_b + (long long)qb * S;
  double* mi_s = reinterpret_cast<double*>(scr + L.mi);
  int32_t* n_s = reinterpret_cast<int32_t*>(scr + L.n);
  uint32_t* maxn = reinterpret_cast<uint32_t*>(scr + L.maxn);
  ArgPartial* partial = reinterpret_cast<ArgPartial*>(scr + L.partial);
  cmif_best* running = reinterpret_cast<cmif_best*>(scr + L.running);
  const int32_t id_c = 65536, id_s = 0;
  const int nang = (int)P.angles.size();
  const int rpc = rows_per_chunk(g.sh);
  const int nchunks = (g.sh + rpc - 1) / rpc;
  const bool want_best = o.best != nullptr || o.per_angle != nullptr;
  if (o.stats) {
    STAGE(ST_CHECK, 2.0 * g.ha * g.wa,
          launch_check_labels(la, ma, (long long)g.ha * g.wa, qa, o.stats, st));
    STAGE(ST_CHECK, 2.0 * g.hb * g.wb,
          launch_check_labels(lb, mb, (long long)g.hb * g.wb, qb, o.stats, st));
  }
  // one correlation: product, column inverse, row inverse -> real map
  auto correlate = [&](const C64* f1, const C64* f2, double* out) -> cmif_status {
    STAGE(ST_PLAIN, 3.0 * fstride * sizeof(C64),
          launch_plain_product(f1, f2, y, half, g.ph, st));
    PairColsArgs<double> pc{};
    pc.FA = nullptr; pc.FB = y; pc.fb_angle_stride = 0; pc.fb_label_stride = fstride;
    pc.QA = 1; pc.QB = 1; pc.ha = g.eha; pc.hb = g.ehb; pc.sh = g.sh;
    pc.tiles = half / tile_width<double>(); pc.nb = 1; pc.Z = z;
    pc.z_angle_stride = 0; pc.z_pair_stride = (long long)half * g.sh;
    pc.tw = twiddles<double>(P, pers, g.ph); pc.zg = z_group_rt<double>(g.pw);
    STAGE(ST_PLAIN, ((double)fstride + (double)half * g.sh) * sizeof(C64),
          launch_pair_cols<double>(g.ph, pc, st));
    PairCountsArgs<double> pk{};
    pk.Z = z; pk.z_angle_stride = 0; pk.z_pair_stride = pc.z_pair_stride;
    pk.QA = 1; pk.QB = 1; pk.wa = g.ewa; pk.wb = g.ewb; pk.sh = g.sh; pk.sw = g.sw;
    pk.ph = g.ph; pk.nb = 1; pk.tw = twiddles<double>(P, pers, g.pw);
    pk.values = out; pk.counts_angle_stride = S;
    STAGE(ST_PLAIN, (double)half * g.sh * sizeof(C64) + 8.0 * S,
          launch_pair_counts<double>(g.pw, pk, st));
    return CMIF_OK;
  };
  for (int ang = 0; ang < nang; ++ang) {
    cmif_status s;
    // forward transforms, one level set (or mask) per launch pair
    for (int a = 0; a <= qa; ++a) {
      s = forward<double>(P, st, ST_PLAIN, ST_PLAIN, a < qa ? la : nullptr, ma,
                          g.ha, g.wa, 1, 1, &id_c, &id_s, g, pers, x,
                          fa + a * fstride, nullptr, nullptr, nullptr,
                          a < qa ? a : 0);
      if (s != CMIF_OK) return s;
    }
    for (int b = 0; b <= qb; ++b) {
      s = forward<double>(P, st, ST_PLAIN, ST_PLAIN, b < qb ? lb : nullptr, mb,
                          g.hb, g.wb, 1, 1, &P.rc[ang], &P.rs[ang], g, pers, x,
                          fb + b * fstride, nullptr, nullptr, nullptr,
                          b < qb ? b : 0);
      if (s != CMIF_OK) return s;
    }
    // Eq. 9: joint; Eq. 10: marginals (level set against the other mask);
    // Eq. 11: N (mask against mask)
    for (int a = 0; a < qa; ++a)
      for (int b = 0; b < qb; ++b) {
        s = correlate(fa + a * fstride, fb + b * fstride, joint + (long long)(a * qb + b) * S);
        if (s != CMIF_OK) return s;
      }
    for (int a = 0; a < qa; ++a) {
      s = correlate(fa + a * fstride, fb + qb * fstride, marg_a + a * S);
      if (s != CMIF_OK) return s;
    }
    for (int b = 0; b < qb; ++b) {
      s = correlate(fa + qa * fstride, fb + b * fstride, marg_b + b * S);
      if (s != CMIF_OK) return s;
    }
    s = correlate(fa + qa * fstride, fb + qb * fstride, nmap);
    if (s != CMIF_OK) return s;
    STAGE(ST_FILL, 4.0, launch_fill_u32(maxn, 0u, 1, st));
    double* mi_ptr = o.mi ? o.mi + ang * S : mi_s;
    int32_t* n_ptr = o.n ? o.n + ang * S : n_s;
    PlainEntropyArgs pe{};
    pe.joint = joint; pe.marg_a = marg_a; pe.marg_b = marg_b; pe.nmap = nmap;
    pe.S = S; pe.QA = qa; pe.QB = qb; pe.mi = mi_ptr; pe.n = n_ptr; pe.maxn = maxn;
    STAGE(ST_PLAIN, 8.0 * S * (1 + qa + qb + qa * qb) + 12.0 * S,
          launch_plain_entropy(pe, st));
    if (want_best) {
      ArgmaxArgs am{};
      am.mi = mi_ptr; am.n = n_ptr; am.angle_stride = S; am.maxn = maxn;
      am.sh = g.sh; am.sw = g.sw; am.nb = 1; am.rows_per_chunk = rpc;
      am.nchunks = nchunks; am.gamma = P.d.gamma; am.partial = partial;
      STAGE(ST_ARGMAX, 12.0 * S, launch_argmax(am, st));
      ArgmaxFinalArgs af{};
      af.partial = partial; af.nb = 1; af.nchunks = nchunks; af.sw = g.sw;
      af.ha = g.eha; af.wa = g.ewa; af.angle0 = ang;
      af.angles[0] = P.angles[ang];
      af.per_angle = o.per_angle; af.running = running;
      af.first_batch = ang == 0; af.best_out = o.best;
      af.last_batch = ang + 1 >= nang;
      STAGE(ST_ARGMAX, (double)nchunks * sizeof(ArgPartial),
            launch_argmax_final(af, st));
    }
    // the host waits for every angle before it starts the next
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess)
      return fail(CMIF_ERR_DEVICE, std::string("hipStreamSynchronize: ") +
                                       hipGetErrorString(e));
  }
  return CMIF_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the launch shapes (CMIF_FLAG_AUTOTUNE)
// ---------------------------------------------------------------------------

bool tunable(const cmif_plan_s* P) {
  return (P->d.flags & CMIF_FLAG_AUTOTUNE) && P->d.mode == CMIF_MODE_HARD &&
         !(P->d.flags & CMIF_FLAG_PLAIN_SCHEDULE);
}

std::string tune_key(const cmif_plan_s* P) {
  std::ostringstream k;
  k << "cmif-tune v1 gfx950";
  for (const PairPlan& g : P->pairs)
    k << " " << g.ph << "x" << g.pw << ":" << g.sh << "x" << g.sw;
  k << " qa=" << P->d.q_a << " qb=" << P->d.q_b << " prec=" << P->d.precision
    << " batch=" << P->batch;
  return k.str();
}

// Reads "<key> rows_per_wg=R bpw=B xcd=X half=H maxr=M ba=A" lines (the
// last three optional, defaults 0 16 1); true if the key is found.
bool tune_read(cmif_plan_s* P) {
  std::ifstream f(P->tune_path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    const size_t at = line.find(" rows_per_wg=");
    if (at == std::string::npos || line.substr(0, at) != P->tune_key) continue;
    int r = 0, b = 0, x = 0, h = 0, m = 16, a = 1;
    const int got = std::sscanf(line.c_str() + at,
                                " rows_per_wg=%d bpw=%d xcd=%d half=%d maxr=%d ba=%d",
                                &r, &b, &x, &h, &m, &a);
    if (got != 3 && got != 6) continue;
    if (r < 1 || r > 8 || (b != 0 && b != 4 && b != 8 && b != 16) || x < 0 || x > 1 ||
        h < 0 || h > 1 || (m != 8 && m != 16) || a < 1 || a > 2)
      continue;
    P->rows_per_wg = r;
    P->bpw = b;
    P->xcd = x;
    P->pc_half = h;
    P->pc_maxr = m;
    P->pc_ba = a;
    return true;
  }
  return false;
}

void tune_write(const cmif_plan_s* P) {
  std::vector<std::string> lines;
  {
    std::ifstream f(P->tune_path);
    std::string line;
    while (f && std::getline(f, line)) {
      const size_t at = line.find(" rows_per_wg=");
      if (at != std::string::npos && line.substr(0, at) == P->tune_key) continue;
      if (!line.empty()) lines.push_back(line);
    }
  }
  std::ostringstream e;
  e << P->tune_key << " rows_per_wg=" << P->rows_per_wg << " bpw=" << P->bpw
    << " xcd=" << P->xcd << " half=" << P->pc_half << " maxr=" << P->pc_maxr
    << " ba=" << P->pc_ba;
  lines.push_back(e.str());
  const std::string tmp = P->tune_path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return;  // the cache is an optimisation: an unwritable path is ignored
    for (const std::string& l : lines) f << l << "\n";
  }
  (void)std::rename(tmp.c_str(), P->tune_path.c_str());
}

// Stage milliseconds of the recorded launches; clears the records and hands
// their events back to the pool above `base`.
cmif_status stage_ms(cmif_plan_s* P, double* ms, size_t base) {
  for (int s = 0; s < ST_COUNT; ++s) ms[s] = 0.0;
  for (const ProfRec& r : P->prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventSynchronize failed");
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventElapsedTime failed");
    ms[r.stage] += t;
  }
  P->prof.recs.clear();
  P->prof.used = base;
  return CMIF_OK;
}

// Times one eager pass per candidate (the call's own inputs and outputs;
// no stats), keeps the fastest row shape and column shape.  Pass k runs
// row candidate k mod |rows| and column candidate k mod |columns|, so every
// candidate of both kernels is timed at least once.  The caller's
// stage-profiler records are set aside meanwhile.
template <class F>
cmif_status autotune(cmif_plan_s* P, hipStream_t st, F&& pass) {
  if (P->tuned || !tunable(P)) return CMIF_OK;
  std::vector<ProfRec> saved;
  saved.swap(P->prof.recs);
  const bool was_on = P->prof.on;
  const size_t used0 = P->prof.used;
  P->prof.on = true;
  struct RowCand { int rpw, bpw; };
  struct ColCand { int xcd, half, maxr, ba; };
  std::vector<RowCand> rows;
  std::vector<ColCand> cols;
  const bool fp32 = P->d.precision != CMIF_PREC_FP64;
  const size_t er = fp32 ? sizeof(float) : sizeof(double);
  PairRowsConfig def;
  const bool have_def = pair_rows_config(er, P->pairs[0].pw, P->d.q_b, &def);
  for (int bpw : {0, 4, 8, 16}) {
    if (bpw != 0) {
      bool fits = true;
      for (const PairPlan& g : P->pairs) {
        PairRowsConfig c;
        fits = fits && pair_rows_config_bpw(er, g.pw, P->d.q_b, bpw, &c);
      }
      if (!fits || (have_def && def.bpw == bpw)) continue;
    }
    for (int rpw : {1, 2, 4}) rows.push_back({rpw, bpw});
  }
  // column shapes: workgroup order, and for FP32 half the columns per
  // workgroup, radix cap 8 and two labels of A per workgroup
  for (int xcd : {0, 1})
    for (int half : {0, 1})
      for (int maxr : {16, 8})
        for (int ba : {1, 2}) {
          if (!fp32 && (half || maxr != 16 || ba != 1)) continue;
          cols.push_back({xcd, half, maxr, ba});
        }
  double best_rows = 1e300, best_cols = 1e300;
  RowCand rpick{P->def_rpw, 0};
  ColCand cpick{P->def_xcd, 0, 16, 1};
  // an untimed pass first: code loading and cold caches stay out of the choice
  cmif_status s = pass(st);
  if (s == CMIF_OK) {
    double ms[ST_COUNT];
    s = stage_ms(P, ms, used0);
  }
  const size_t npass = std::max(rows.size(), cols.size());
  for (size_t k = 0; s == CMIF_OK && k < npass; ++k) {
    const RowCand& rc = rows[k % rows.size()];
    const ColCand& cc = cols[k % cols.size()];
    P->rows_per_wg = rc.rpw;
    P->bpw = rc.bpw;
    P->xcd = cc.xcd;
    P->pc_half = cc.half;
    P->pc_maxr = cc.maxr;
    P->pc_ba = cc.ba;
    s = pass(st);
    if (s != CMIF_OK) break;
    double ms[ST_COUNT];
    s = stage_ms(P, ms, used0);
    if (s != CMIF_OK) break;
    ++P->tune_runs;
    if (k < rows.size() && ms[ST_PAIR_ROWS] < best_rows) {
      best_rows = ms[ST_PAIR_ROWS];
      rpick = rc;
    }
    if (k < cols.size() && ms[ST_PAIR_COLS] < best_cols) {
      best_cols = ms[ST_PAIR_COLS];
      cpick = cc;
    }
  }
  P->prof.on = was_on;
  P->prof.recs.swap(saved);
  P->prof.used = used0;
  if (s != CMIF_OK) {
    P->rows_per_wg = P->def_rpw;
    P->bpw = 0;
    P->xcd = P->def_xcd;
    P->pc_half = 0;
    P->pc_maxr = 16;
    P->pc_ba = 1;
    return s;
  }
  P->rows_per_wg = rpick.rpw;
  P->bpw = rpick.bpw;
  P->xcd = cpick.xcd;
  P->pc_half = cpick.half;
  P->pc_maxr = cpick.maxr;
  P->pc_ba = cpick.ba;
  P->tuned = 1;
  if (!P->tune_path.empty()) tune_write(P);
  return CMIF_OK;
}

cmif_status validate_ws(const cmif_plan_s* P, void* pers, size_t pers_bytes,
                        void* scr, size_t scr_bytes) {
  if (pers_bytes < P->persistent_bytes || scr_bytes < P->scratch_bytes)
    return fail(CMIF_ERR_WORKSPACE_TOO_SMALL,
                "workspace too small: need persistent " +
                    std::to_string(P->persistent_bytes) + ", scratch " +
                    std::to_string(P->scratch_bytes));
  if ((P->persistent_bytes && pers == nullptr) ||
      (P->scratch_bytes && scr == nullptr))
    return fail(CMIF_ERR_INVALID_ARGUMENT, "workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(pers) & 255) ||
      (reinterpret_cast<uintptr_t>(scr) & 255))
    return fail(CMIF_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  return CMIF_OK;
}

cmif_status init_tables(cmif_plan_s* P, uint8_t* pb, hipStream_t st) {
  cmif_plan_s& PP = *P;
  for (size_t i = 0; i < P->plens.size(); ++i) {
    const int L = P->plens[i];
    cmif_status s = launch_stage(
        PP, st, ST_TABLES, 24.0 * L, "launch_init_tables", [&]() {
          return launch_init_tables(
              pb + P->tw_off[i], pb + P->tw_off[i] + (size_t)L * sizeof(float2), L,
              i == 0 ? reinterpret_cast<double*>(pb + P->logtab_off) : nullptr,
              i == 0 ? reinterpret_cast<double*>(pb + P->xlog_off) : nullptr, st);
        });
    if (s != CMIF_OK) return s;
  }
  return CMIF_OK;
}

cmif_status check_inputs(const cmif_plan_s* P, const cmif_inputs* in) {
  const int np = P->d.n_pairs;
  if (P->d.mode == CMIF_MODE_SOFT) {
    if (in->memb_a == nullptr || in->memb_b == nullptr)
      return fail(CMIF_ERR_INVALID_ARGUMENT, "membership arrays are NULL");
    for (int p = 0; p < np; ++p)
      if (in->memb_a[p] == nullptr || in->memb_b[p] == nullptr)
        return fail(CMIF_ERR_INVALID_ARGUMENT,
                    "membership pointer of a pair is NULL");
    return CMIF_OK;
  }
  if (in->labels_a == nullptr || in->labels_b == nullptr)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "labels arrays are NULL");
  for (int p = 0; p < np; ++p)
    if (in->labels_a[p] == nullptr || in->labels_b[p] == nullptr)
      return fail(CMIF_ERR_INVALID_ARGUMENT, "label pointer of a pair is NULL");
  return CMIF_OK;
}

cmif_status run_calls(cmif_plan_s* P, const cmif_inputs* in,
                      const cmif_outputs* out, cmif_best* best,
                      cmif_best* per_angle, cmif_stats* stats, void* pers,
                      void* scr, hipStream_t st) {
  const int np = P->d.n_pairs;
  const bool soft = P->d.mode == CMIF_MODE_SOFT;
  cmif_status s = check_inputs(P, in);
  if (s != CMIF_OK) return s;
  uint8_t* pb = static_cast<uint8_t*>(pers);
  uint8_t* sb = static_cast<uint8_t*>(scr);
  if ((P->d.flags & CMIF_FLAG_PLAIN_SCHEDULE) && out &&
      (out->counts || out->digest))
    return fail(CMIF_ERR_INVALID_ARGUMENT,
                "the plain schedule emits mi, n, best and per_angle only");
  s = init_tables(P, pb, st);
  if (s != CMIF_OK) return s;
  cmif_plan_s& PP = *P;
  const int nang = (int)P->angles.size();
  if (!soft && out && out->digest) {
    for (int p = 0; p < np; ++p)
      if (out->digest[p]) {
        const long long nw = 2LL * nang * P->d.q_a * P->d.q_b;
        s = launch_stage(PP, st, ST_FILL, 4.0 * nw, "fill digest", [&]() {
          return launch_fill_u32(reinterpret_cast<uint32_t*>(out->digest[p]), 0u, nw, st);
        });
        if (s != CMIF_OK) return s;
      }
  }
  for (int p = 0; p < np; ++p) {
    CallOutputs o;
    if (out) {
      o.mi = out->mi ? out->mi[p] : nullptr;
      o.n = out->n ? out->n[p] : nullptr;
      if (!soft) {
        o.counts = out->counts ? out->counts[p] : nullptr;
        o.digest = out->digest ? out->digest[p] : nullptr;
      }
    }
    o.best = best ? best + p : nullptr;
    o.per_angle = per_angle ? per_angle + (size_t)p * nang : nullptr;
    o.stats = stats;
    const uint8_t* ma = in->mask_a ? in->mask_a[p] : nullptr;
    const uint8_t* mb = in->mask_b ? in->mask_b[p] : nullptr;
    const uint8_t* la = soft ? nullptr : in->labels_a[p];
    const uint8_t* lb = soft ? nullptr : in->labels_b[p];
    const float* pa = soft ? in->memb_a[p] : nullptr;
    const float* pbm = soft ? in->memb_b[p] : nullptr;
    if (P->d.flags & CMIF_FLAG_PLAIN_SCHEDULE)
      s = run_pair_plain(*P, p, la, ma, lb, mb, o, pb, sb, st);
    else if (P->d.precision == CMIF_PREC_FP64)
      s = run_pair<double>(*P, p, la, ma, lb, mb, pa, pbm, o, pb, sb, st);
    else
      s = run_pair<float>(*P, p, la, ma, lb, mb, pa, pbm, o, pb, sb, st);
    if (s != CMIF_OK) return s;
  }
  return CMIF_OK;
}

// Adjoint of the soft forward for one pair (single angle 0): the joint is
// recomputed from the memberships, G_ab formed per displacement from the
// saved state, transformed, summed against the other side's spectra and
// transformed back.
template <typename T>
cmif_status run_backward_pair(cmif_plan_s& P, int p, const uint8_t* ma,
                              const uint8_t* mb, const float* pa,
                              const float* pbm, const double* grad_mi,
                              float* grad_a, float* grad_b, uint8_t* pers,
                              uint8_t* scr, hipStream_t st) {
  using CT = C2<T>;
  const PairPlan& g = P.pairs[p];
  const ScratchLayout L = layout_for(P, g);
  const int qa = P.d.q_a, qb = P.d.q_b;
  const int half = g.pw / 2;
  const int tiles = half / tile_width<T>();
  CT* xa = reinterpret_cast<CT*>(scr + L.xa);
  CT* fa = reinterpret_cast<CT*>(scr + L.fa);
  CT* xb = reinterpret_cast<CT*>(scr + L.xb);
  CT* fb = reinterpret_cast<CT*>(scr + L.fb);
  CT* z = reinterpret_cast<CT*>(scr + L.z);
  CT* zg = reinterpret_cast<CT*>(scr + L.zg);
  CT* gh = reinterpret_cast<CT*>(scr + L.gh);
  CT* gxa = reinterpret_cast<CT*>(scr + L.gxa);
  CT* gxb = reinterpret_cast<CT*>(scr + L.gxb);
  const T* save = reinterpret_cast<const T*>(pers + P.save_off[p]);
  const int32_t id_c = 65536, id_s = 0;
  cmif_status s = forward<T>(P, st, ST_FWD_ROWS, ST_FWD_COLS, nullptr, ma, g.ha,
                             g.wa, qa, 1, &id_c, &id_s, g, pers, xa, fa,
                             nullptr, pa, nullptr);
  if (s != CMIF_OK) return s;
  s = forward<T>(P, st, ST_FWD_ROWS, ST_FWD_COLS, nullptr, mb, g.hb, g.wb, qb, 1,
                 &P.rc[0], &P.rs[0], g, pers, xb, fb, nullptr, pbm, nullptr);
  if (s != CMIF_OK) return s;
  PairColsArgs<T> pc{};
  pc.FA = fa; pc.fa_label_stride = (long long)half * g.ph;
  pc.FB = fb; pc.fb_angle_stride = (long long)qb * half * g.ph;
  pc.fb_label_stride = (long long)half * g.ph;
  pc.QA = qa; pc.QB = qb; pc.ha = g.eha; pc.hb = g.ehb; pc.sh = g.sh;
  pc.tiles = tiles; pc.nb = 1; pc.Z = z;
  pc.z_angle_stride = (long long)z_pair_slots(qa * qb) * half * g.sh;
  pc.z_pair_stride = (long long)half * g.sh; pc.tw = twiddles<T>(P, pers, g.ph);
  pc.xcd = P.xcd; pc.zg = z_group_rt<T>(g.pw);
  const double zbytes = (double)qa * qb * half * g.sh * sizeof(CT);
  STAGE(ST_PAIR_COLS,
        (double)(qa + qb) * half * g.ph * sizeof(CT) + zbytes,
        launch_pair_cols<T>(g.ph, pc, st));
  SoftGradRowsArgs<T> gr{};
  gr.Z = z; gr.z_pair_stride = pc.z_pair_stride; gr.QA = qa; gr.QB = qb;
  gr.wa = g.ewa; gr.wb = g.ewb; gr.sh = g.sh; gr.sw = g.sw; gr.ph = g.ph;
  gr.tw = twiddles<T>(P, pers, g.pw); gr.grad_mi = grad_mi; gr.save = save;
  gr.ZG = zg;
  STAGE(ST_SOFT_GRAD,
        2.0 * zbytes + (8.0 + (double)sizeof(T) * (qa + qb + 2)) * g.sh * g.sw,
        launch_soft_grad_rows<T>(g.pw, gr, st));
  FwdColsArgs<T> gc{};
  gc.xrow = zg; gc.H = g.sh; gc.tiles = tiles; gc.Q = qa * qb; gc.nb = 1;
  gc.x_angle_stride = 0; gc.x_label_stride = (long long)half * g.sh;
  gc.F = gh; gc.f_angle_stride = 0; gc.f_label_stride = (long long)half * g.ph;
  gc.tw = twiddles<T>(P, pers, g.ph); gc.circ_ha = g.eha; gc.circ_hb = g.ehb;
  STAGE(ST_SOFT_GRAD, zbytes + (double)qa * qb * half * g.ph * sizeof(CT),
        launch_fwd_cols<T>(g.ph, gc, st));
  for (int side = 0; side < 2; ++side) {
    float* grad = side == 0 ? grad_a : grad_b;
    if (grad == nullptr) continue;
    const int q = side == 0 ? qa : qb;
    const int H = side == 0 ? g.ha : g.hb, W = side == 0 ? g.wa : g.wb;
    CT* gx = side == 0 ? gxa : gxb;
    SoftGradColsArgs<T> sc{};
    sc.GH = gh; sc.FO = side == 0 ? fb : fa;
    sc.f_label_stride = (long long)half * g.ph; sc.QA = qa; sc.QB = qb;
    sc.H = H; sc.tiles = tiles; sc.side = side; sc.GX = gx;
    sc.gx_label_stride = (long long)half * H; sc.tw = twiddles<T>(P, pers, g.ph);
    STAGE(ST_SOFT_GRAD,
          ((double)qa * qb + (side == 0 ? qb : qa)) * half * g.ph * sizeof(CT) +
              (double)q * half * H * sizeof(CT),
          launch_soft_grad_cols<T>(g.ph, sc, st));
    SoftGradOutArgs<T> so{};
    so.GX = gx; so.gx_label_stride = (long long)half * H; so.Q = q; so.H = H;
    so.W = W; so.ph = g.ph; so.msk = side == 0 ? ma : mb;
    so.tw = twiddles<T>(P, pers, g.pw); so.grad = grad;
    STAGE(ST_SOFT_GRAD,
          (double)q * half * H * sizeof(CT) + (4.0 * q + 1.0) * H * W,
          launch_soft_grad_out<T>(g.pw, so, st));
  }
  return CMIF_OK;
}

// Stage profiling brackets every launch with events on the stream, so it
// launches eagerly.
bool graph_allowed(const cmif_plan_s* P) {
  return !(P->d.flags & (CMIF_FLAG_NO_GRAPH | CMIF_FLAG_PLAIN_SCHEDULE)) &&
         !P->prof.on;
}

void key_ptrs(std::vector<uintptr_t>& k, const void* const* arr, int n) {
  k.push_back(arr ? 1u : 0u);
  if (arr)
    for (int p = 0; p < n; ++p) k.push_back(reinterpret_cast<uintptr_t>(arr[p]));
}

std::vector<uintptr_t> call_key(const cmif_plan_s* P, int op,
                                const cmif_inputs* in, const cmif_outputs* out,
                                const void* best, const void* per_angle,
                                const void* stats, const void* pers,
                                const void* scr, hipStream_t st) {
  const int n = P->d.n_pairs;
  std::vector<uintptr_t> k;
  k.push_back((uintptr_t)op);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->labels_a), n);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->mask_a), n);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->labels_b), n);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->mask_b), n);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->memb_a), n);
  key_ptrs(k, reinterpret_cast<const void* const*>(in->memb_b), n);
  if (out) {
    key_ptrs(k, reinterpret_cast<const void* const*>(out->mi), n);
    key_ptrs(k, reinterpret_cast<const void* const*>(out->n), n);
    key_ptrs(k, reinterpret_cast<const void* const*>(out->counts), n);
    key_ptrs(k, reinterpret_cast<const void* const*>(out->digest), n);
  }
  for (const void* p : {best, per_angle, stats, pers, scr, (const void*)st})
    k.push_back(reinterpret_cast<uintptr_t>(p));
  return k;
}

// Runs `body` through a captured graph: replays the cached one when the
// call's pointers match, otherwise captures the launch sequence on a
// private stream, instantiates it and launches it on `st` (ordered after the
// caller's earlier work on `st`).  A capture the runtime refuses falls back
// to launching eagerly on `st`.
template <class F>
cmif_status run_graph(cmif_plan_s* P, int op, std::vector<uintptr_t> key,
                      hipStream_t st, F&& body) {
  GraphCache& G = P->graphs[op];
  if (G.refused) return body(st);
  if (G.valid && G.key == key) {
    const hipError_t e = hipGraphLaunch(G.exec, st);
    if (e != hipSuccess)
      return fail(CMIF_ERR_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    ++P->graph_replays;
    return CMIF_OK;
  }
  G.reset();
  if (!G.cs && hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking) != hipSuccess) {
    G.cs = nullptr;
    G.refused = true;
    return body(st);
  }
  if (hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    G.refused = true;
    return body(st);
  }
  const cmif_status s = body(G.cs);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(G.cs, &graph);
  if (s != CMIF_OK || e != hipSuccess || graph == nullptr) {
    // the runtime refused part of the sequence under capture: launch
    // eagerly from now on (a genuine launch error shows up there too)
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    G.reset();
    G.refused = true;
    g_err.clear();
    return body(st);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    (void)hipGetLastError();
    G.reset();
    G.refused = true;
    return body(st);
  }
  G.exec = exec;
  G.key = std::move(key);
  G.valid = true;
  ++P->graph_captures;
  const hipError_t el = hipGraphLaunch(G.exec, st);
  if (el != hipSuccess)
    return fail(CMIF_ERR_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(el));
  return CMIF_OK;
}

}  // namespace

namespace cmif {

cmif_status set_error(cmif_status s, const char* msg) { return fail(s, msg); }

cmif_status plan_noalloc_info(cmif_plan_t plan, int* device, size_t* persistent,
                              size_t* scratch, uint32_t* flags, int32_t* mode) {
  if (!plan) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan");
  *device = plan->d.device;
  *persistent = plan->persistent_bytes;
  *scratch = plan->scratch_bytes;
  *flags = plan->d.flags;
  *mode = plan->d.mode;
  return CMIF_OK;
}

cmif_status compute_eager(cmif_plan_t plan, const cmif_inputs* in,
                          const cmif_outputs* out, void* persistent,
                          void* scratch, hipStream_t st) {
  cmif_status s = check_inputs(plan, in);
  if (s != CMIF_OK) return s;
  s = check_device(plan);
  if (s != CMIF_OK) return s;
  DeviceGuard dg(plan->d.device);
  if (!dg.ok) return fail(CMIF_ERR_DEVICE, "cannot select the plan's device");
  // the stage profiler records events: off for this call
  const bool prof = plan->prof.on;
  plan->prof.on = false;
  s = run_calls(plan, in, out, out ? out->best : nullptr,
                out ? out->per_angle : nullptr, out ? out->stats : nullptr,
                persistent, scratch, st);
  plan->prof.on = prof;
  return s;
}

}  // namespace cmif

extern "C" {

const char* cmif_status_string(cmif_status s) {
  switch (s) {
    case CMIF_OK: return "success";
    case CMIF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case CMIF_ERR_UNSUPPORTED: return "unsupported configuration";
    case CMIF_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case CMIF_ERR_DEVICE: return "HIP runtime error";
    case CMIF_ERR_WRONG_MODE: return "call does not match the plan's mode";
    case CMIF_ERR_NO_DEVICE: return "no usable gfx950 device";
    case CMIF_ERR_HOST_MEMORY: return "host memory allocation failed";
  }
  return "unknown status";
}

const char* cmif_last_error(void) { return g_err.c_str(); }

cmif_status cmif_plan_query(cmif_plan_t plan, cmif_plan_info* info) {
  g_err.clear();
  if (!plan || !info) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->angle_batch = plan->batch;
  info->fallback_capacity = plan->fb_cap;
  info->graph_captures = plan->graph_captures;
  info->graph_replays = plan->graph_replays;
  info->fft_h = plan->pairs[0].ph;
  info->fft_w = plan->pairs[0].pw;
  info->rows_per_wg = plan->rows_per_wg;
  info->labels_per_team = plan->bpw;
  info->xcd_grouping = plan->xcd;
  info->tuned = plan->tuned;
  info->tune_runs = plan->tune_runs;
  info->cols_half = plan->pc_half;
  info->cols_maxr = plan->pc_maxr;
  info->cols_ba = plan->pc_ba;
  return CMIF_OK;
}

cmif_status cmif_profile_enable(cmif_plan_t plan, int32_t enable) {
  g_err.clear();
  if (!plan) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan");
  plan->prof.on = enable != 0;
  return CMIF_OK;
}

cmif_status cmif_profile_read(cmif_plan_t plan, cmif_stage_time* out,
                              int32_t capacity, int32_t* count) {
  g_err.clear();
  if (!plan || !count || (capacity > 0 && !out))
    return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL argument");
  cmif_stage_time acc[ST_COUNT];
  std::memset(acc, 0, sizeof(acc));
  for (int s = 0; s < ST_COUNT; ++s)
    std::snprintf(acc[s].name, sizeof(acc[s].name), "%s", kStageNames[s]);
  for (const ProfRec& r : plan->prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventSynchronize failed");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return fail(CMIF_ERR_DEVICE, "hipEventElapsedTime failed");
    acc[r.stage].launches += 1;
    acc[r.stage].total_ms += ms;
    acc[r.stage].bytes += r.bytes;
  }
  plan->prof.recs.clear();
  plan->prof.used = 0;
  int n = 0;
  for (int s = 0; s < ST_COUNT; ++s) {
    if (acc[s].launches == 0) continue;
    if (n < capacity) out[n] = acc[s];
    ++n;
  }
  *count = n < capacity ? n : capacity;
  return CMIF_OK;
}

cmif_status cmif_plan(const cmif_plan_desc* d, cmif_plan_t* out) {
  g_err.clear();
  if (out == nullptr) return fail(CMIF_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (d == nullptr) return fail(CMIF_ERR_INVALID_ARGUMENT, "desc is NULL");
  if (d->n_pairs < 1)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "n_pairs must be >= 1");
  if (!d->h_a || !d->w_a || !d->h_b || !d->w_b)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "size arrays must not be NULL");
  if (d->q_a < 1 || d->q_a > 64 || d->q_b < 1 || d->q_b > 64)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "q_a and q_b must be in [1, 64]");
  if (!(d->gamma >= 0.0 && d->gamma <= 1.0))
    return fail(CMIF_ERR_INVALID_ARGUMENT, "gamma must be in [0, 1]");
  if (d->precision != CMIF_PREC_FP32_ROUNDED && d->precision != CMIF_PREC_FP64)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "unknown precision");
  if (d->mode != CMIF_MODE_HARD && d->mode != CMIF_MODE_SOFT)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "unknown mode");
  const uint32_t known = CMIF_FLAG_FORCE_FALLBACK | CMIF_FLAG_NO_GRAPH |
                         CMIF_FLAG_SAVE_FOR_BACKWARD | CMIF_FLAG_PLAIN_SCHEDULE |
                         CMIF_FLAG_AUTOTUNE;
  if (d->flags & ~known) return fail(CMIF_ERR_INVALID_ARGUMENT, "unknown flags");
  if ((d->flags & CMIF_FLAG_PLAIN_SCHEDULE) &&
      (d->mode != CMIF_MODE_HARD || d->precision != CMIF_PREC_FP64))
    return fail(CMIF_ERR_UNSUPPORTED, "the plain schedule is HARD and FP64 only");
  if (d->window && (d->mode != CMIF_MODE_HARD || (d->flags & CMIF_FLAG_PLAIN_SCHEDULE)))
    return fail(CMIF_ERR_UNSUPPORTED,
                "displacement windows are HARD mode, fused schedule only");
  if (d->n_angles < 1)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "n_angles must be >= 1");
  if (d->angles_rad == nullptr && d->n_angles != 1)
    return fail(CMIF_ERR_INVALID_ARGUMENT,
                "angles_rad may be NULL only with n_angles = 1");
  if (d->angle_batch < 0)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "angle_batch must be >= 0");
  if (d->fallback_capacity < 0 || d->fallback_capacity > 4096)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "fallback_capacity must be in [0, 4096]");
  if (d->mode == CMIF_MODE_SOFT && (d->flags & CMIF_FLAG_SAVE_FOR_BACKWARD)) {
    const bool identity = d->n_angles == 1 &&
                          (d->angles_rad == nullptr || d->angles_rad[0] == 0.0);
    if (!identity)
      return fail(CMIF_ERR_UNSUPPORTED,
                  "SAVE_FOR_BACKWARD supports the single angle 0 only");
  }

  cmif_plan_s* P = new (std::nothrow) cmif_plan_s();
  if (!P) return fail(CMIF_ERR_HOST_MEMORY, "plan allocation failed");
  P->d = *d;
  P->d.h_a = P->d.w_a = P->d.h_b = P->d.w_b = nullptr;
  P->d.angles_rad = nullptr;
  P->d.window = nullptr;
  P->windowed = d->window != nullptr;
  if (d->tune_cache_path) P->tune_path = d->tune_cache_path;
  P->d.tune_cache_path = nullptr;
  for (int p = 0; p < d->n_pairs; ++p) {
    PairPlan g{};
    g.ha = d->h_a[p]; g.wa = d->w_a[p]; g.hb = d->h_b[p]; g.wb = d->w_b[p];
    if (g.ha < 1 || g.wa < 1 || g.hb < 1 || g.wb < 1 || g.ha > kMaxP ||
        g.wa > kMaxP || g.hb > kMaxP || g.wb > kMaxP) {
      delete P;
      return fail(CMIF_ERR_INVALID_ARGUMENT, "image sides must be in [1, 4096]");
    }
    // displacement window (default: the full set) and its alias-free FFT
    // sides: lag chi and chi +- P must not both lie in the full set
    int y0 = 1 - g.ha, y1 = g.hb - 1, x0 = 1 - g.wa, x1 = g.wb - 1;
    if (d->window) {
      const int32_t* w = d->window + 4 * p;
      if (w[0] < y0 || w[1] > y1 || w[0] > w[1] || w[2] < x0 || w[3] > x1 ||
          w[2] > w[3]) {
        delete P;
        return fail(CMIF_ERR_INVALID_ARGUMENT,
                    "window of pair " + std::to_string(p) +
                        " is empty or outside the displacement set");
      }
      y0 = w[0]; y1 = w[1]; x0 = w[2]; x1 = w[3];
    }
    g.eha = 1 - y0; g.ehb = y1 + 1; g.ewa = 1 - x0; g.ewb = x1 + 1;
    g.sh = y1 - y0 + 1;
    g.sw = x1 - x0 + 1;
    // the transforms hold whole images (the forward kernels zero-pad, they
    // do not fold), so the side also covers both image sides
    g.ph = fft_size_at_least(std::max({y1 + g.ha, g.hb - y0, g.ha, g.hb}));
    g.pw = fft_size_at_least(std::max({x1 + g.wa, g.wb - x0, g.wa, g.wb}));
    if (g.ph == 0 || g.pw == 0) {
      delete P;
      return fail(CMIF_ERR_UNSUPPORTED, "FFT length above 4096");
    }
    // 4096-point transforms: the FP32-rounded HARD path of the fused
    // schedule (with its FP64 re-run); the FP64 and soft row kernels'
    // per-position state does not fit the LDS at that length
    if (std::max(g.ph, g.pw) > kMaxSoftP &&
        (d->mode != CMIF_MODE_HARD || d->precision != CMIF_PREC_FP32_ROUNDED ||
         (d->flags & CMIF_FLAG_PLAIN_SCHEDULE))) {
      delete P;
      return fail(CMIF_ERR_UNSUPPORTED,
                  "FFT lengths above 2048 are for FP32_ROUNDED HARD plans of the "
                  "fused schedule only");
    }
    PairRowsConfig rc;
    SoftRowsConfig sc;
    const size_t er = d->precision == CMIF_PREC_FP64 ? sizeof(double) : sizeof(float);
    const bool fits = d->mode == CMIF_MODE_SOFT
                          ? soft_rows_config(er, g.pw, d->q_b, &sc) &&
                                pair_rows_config(sizeof(double), g.pw, 1, &rc)
                          : pair_rows_config(er, g.pw, d->q_b, &rc);
    if (!fits) {
      delete P;
      return fail(CMIF_ERR_UNSUPPORTED,
                  "q_b too large for the row kernel at this FFT length");
    }
    P->pairs.push_back(g);
    for (int len : {g.ph, g.pw})
      if (find_plen(*P, len) < 0) P->plens.push_back(len);
  }
  for (int a = 0; a < d->n_angles; ++a) {
    const double th = d->angles_rad ? d->angles_rad[a] : 0.0;
    if (!std::isfinite(th)) {
      delete P;
      return fail(CMIF_ERR_INVALID_ARGUMENT, "angles must be finite");
    }
    P->angles.push_back(th);
    P->rc.push_back((int32_t)std::llround(std::cos(th) * 65536.0));
    P->rs.push_back((int32_t)std::llround(std::sin(th) * 65536.0));
  }
  // angle batch: keep the pair intermediates of one pass within 8 GiB
  size_t zmax = 0;
  const size_t E = elem_bytes(*P);
  for (const auto& g : P->pairs) {
    const size_t zb = (size_t)d->q_a * d->q_b * (g.pw / 2) * g.sh * E;
    zmax = std::max(zmax, zb);
  }
  int batch = d->angle_batch;
  if (batch == 0) {
    const size_t budget = size_t(8) << 30;
    batch = (int)std::max<size_t>(1, budget / std::max<size_t>(zmax, 1));
  }
  batch = std::min(batch, kMaxBatch);
  batch = std::min(batch, d->n_angles);
  if (d->flags & CMIF_FLAG_PLAIN_SCHEDULE) batch = 1;
  P->batch = std::max(batch, 1);
  if (d->precision == CMIF_PREC_FP32_ROUNDED && d->mode == CMIF_MODE_HARD) {
    const int per_pass = P->batch * d->q_a * d->q_b;
    const int cap = d->fallback_capacity > 0 ? d->fallback_capacity : 64;
    P->fb_cap = std::min(cap, per_pass);
  }
  // persistent: per FFT length FP32 + FP64 twiddles, then the log table
  size_t o = 0;
  for (int len : P->plens) {
    P->tw_off.push_back(o);
    o += up256((size_t)len * (sizeof(float2) + sizeof(double2)));
  }
  P->logtab_off = o;
  o += up256(512 * sizeof(double));
  P->xlog_off = o;
  o += up256(kXlogN * sizeof(double));
  if (d->mode == CMIF_MODE_SOFT && (d->flags & CMIF_FLAG_SAVE_FOR_BACKWARD)) {
    for (const auto& g : P->pairs) {
      P->save_off.push_back(o);
      const size_t er = d->precision == CMIF_PREC_FP64 ? sizeof(double) : sizeof(float);
      o += up256(save_angle_elems(*P, g) * P->angles.size() * er);
    }
  }
  P->persistent_bytes = o;
  size_t smax = 0;
  for (const auto& g : P->pairs) smax = std::max(smax, layout_for(*P, g).end);
  P->scratch_bytes = smax;
  // default column order: XCD-grouped (each tile's label-a workgroups on
  // one XCD, reading its F_B columns from that L2 in rotated label order)
  // where every column length is a power of two; measured against launch
  // order per call: 0.90 (512 points), 0.91-0.98 (1024, FP64 / FP32),
  // 0.99-1.00 (2048).  At 3 * 2^k lengths launch order stays the default
  // (the XCD order measured 1.5-2.4 % slower at 768).  The tuner times both.
  bool pow2_cols = true;
  for (const PairPlan& g : P->pairs) pow2_cols = pow2_cols && is_pow2(g.ph);
  P->def_xcd = pow2_cols ? 1 : 0;
  P->xcd = P->def_xcd;
  // rows per workgroup: 2 for FP32 1024-point rows (2-4 % faster there), 1
  // elsewhere (FP64 and 2048-point rows measured 2-5 % slower with 2, and
  // smaller maps need the workgroups: 35 % faster at 512 points)
  P->def_rpw = (d->precision != CMIF_PREC_FP64 && P->pairs[0].pw == 1024) ? 2 : 1;
  P->rows_per_wg = P->def_rpw;
  if (tunable(P)) {
    P->tune_key = tune_key(P);
    if (!P->tune_path.empty() && tune_read(P)) P->tuned = 2;
  }
  *out = P;
  return CMIF_OK;
}

void cmif_plan_free(cmif_plan_t plan) { delete plan; }

cmif_status cmif_workspace_size(cmif_plan_t plan, size_t* persistent,
                                 size_t* scratch) {
  g_err.clear();
  if (!plan || !persistent || !scratch)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL argument");
  *persistent = plan->persistent_bytes;
  *scratch = plan->scratch_bytes;
  return CMIF_OK;
}

cmif_status cmif_compute(cmif_plan_t plan, const cmif_inputs* in,
                         const cmif_outputs* out, void* persistent,
                         size_t persistent_bytes, void* scratch,
                         size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!plan || !in) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan or inputs");
  cmif_status s = validate_ws(plan, persistent, persistent_bytes, scratch,
                              scratch_bytes);
  if (s != CMIF_OK) return s;
  s = check_inputs(plan, in);
  if (s != CMIF_OK) return s;
  s = check_device(plan);
  if (s != CMIF_OK) return s;
  DeviceGuard dg(plan->d.device);
  if (!dg.ok) return fail(CMIF_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  cmif_best* best = out ? out->best : nullptr;
  cmif_best* per_angle = out ? out->per_angle : nullptr;
  cmif_stats* stats = out ? out->stats : nullptr;
  auto body = [&](hipStream_t s) {
    return run_calls(plan, in, out, best, per_angle, stats, persistent, scratch, s);
  };
  s = autotune(plan, st, [&](hipStream_t s2) {
    return run_calls(plan, in, out, best, per_angle, nullptr, persistent, scratch, s2);
  });
  if (s != CMIF_OK) return s;
  if (!graph_allowed(plan)) return body(st);
  return run_graph(plan, 0,
                   call_key(plan, 0, in, out, best, per_angle, stats, persistent,
                            scratch, st),
                   st, body);
}

cmif_status cmif_align(cmif_plan_t plan, const cmif_inputs* in,
                       cmif_best* best, cmif_best* per_angle,
                       cmif_stats* stats, void* persistent,
                       size_t persistent_bytes, void* scratch,
                       size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!plan || !in) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan or inputs");
  if (!best) return fail(CMIF_ERR_INVALID_ARGUMENT, "best is NULL");
  cmif_status s = validate_ws(plan, persistent, persistent_bytes, scratch,
                              scratch_bytes);
  if (s != CMIF_OK) return s;
  s = check_inputs(plan, in);
  if (s != CMIF_OK) return s;
  s = check_device(plan);
  if (s != CMIF_OK) return s;
  DeviceGuard dg(plan->d.device);
  if (!dg.ok) return fail(CMIF_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto body = [&](hipStream_t s) {
    return run_calls(plan, in, nullptr, best, per_angle, stats, persistent,
                     scratch, s);
  };
  s = autotune(plan, st, [&](hipStream_t s2) {
    return run_calls(plan, in, nullptr, best, per_angle, nullptr, persistent,
                     scratch, s2);
  });
  if (s != CMIF_OK) return s;
  if (!graph_allowed(plan)) return body(st);
  return run_graph(plan, 1,
                   call_key(plan, 1, in, nullptr, best, per_angle, stats,
                            persistent, scratch, st),
                   st, body);
}

cmif_status cmif_backward(cmif_plan_t plan, const cmif_inputs* in,
                          const double* const* grad_mi, float* const* grad_a,
                          float* const* grad_b, void* persistent,
                          size_t persistent_bytes, void* scratch,
                          size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!plan) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan");
  if (plan->d.mode != CMIF_MODE_SOFT ||
      !(plan->d.flags & CMIF_FLAG_SAVE_FOR_BACKWARD))
    return fail(CMIF_ERR_WRONG_MODE,
                "cmif_backward needs a SOFT plan with SAVE_FOR_BACKWARD");
  if (!in || !grad_mi) return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL inputs or grad_mi");
  cmif_status s = validate_ws(plan, persistent, persistent_bytes, scratch,
                              scratch_bytes);
  if (s != CMIF_OK) return s;
  s = check_inputs(plan, in);
  if (s != CMIF_OK) return s;
  for (int p = 0; p < plan->d.n_pairs; ++p)
    if (grad_mi[p] == nullptr)
      return fail(CMIF_ERR_INVALID_ARGUMENT, "grad_mi pointer of a pair is NULL");
  s = check_device(plan);
  if (s != CMIF_OK) return s;
  DeviceGuard dg(plan->d.device);
  if (!dg.ok) return fail(CMIF_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint8_t* pb = static_cast<uint8_t*>(persistent);
  uint8_t* sb = static_cast<uint8_t*>(scratch);
  s = init_tables(plan, pb, st);
  if (s != CMIF_OK) return s;
  for (int p = 0; p < plan->d.n_pairs; ++p) {
    const uint8_t* ma = in->mask_a ? in->mask_a[p] : nullptr;
    const uint8_t* mb = in->mask_b ? in->mask_b[p] : nullptr;
    float* ga = grad_a ? grad_a[p] : nullptr;
    float* gb = grad_b ? grad_b[p] : nullptr;
    if (!ga && !gb) continue;
    if (plan->d.precision == CMIF_PREC_FP64)
      s = run_backward_pair<double>(*plan, p, ma, mb, in->memb_a[p], in->memb_b[p],
                                    grad_mi[p], ga, gb, pb, sb, st);
    else
      s = run_backward_pair<float>(*plan, p, ma, mb, in->memb_a[p], in->memb_b[p],
                                   grad_mi[p], ga, gb, pb, sb, st);
    if (s != CMIF_OK) return s;
  }
  return CMIF_OK;
}

cmif_status cmif_align_two_stage(cmif_plan_t plan, const cmif_inputs* in,
                                 int32_t n_refine, const double* refine_offsets,
                                 cmif_best* best, cmif_best* grid_best,
                                 cmif_best* refine_best, cmif_stats* stats,
                                 void* persistent, size_t persistent_bytes,
                                 void* scratch, size_t scratch_bytes,
                                 void* stream) {
  g_err.clear();
  if (!plan || !in || !best)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL plan, inputs or best");
  if (plan->d.mode != CMIF_MODE_HARD)
    return fail(CMIF_ERR_WRONG_MODE, "the two-stage alignment takes HARD plans");
  if (n_refine < 1 || n_refine > 4096 || refine_offsets == nullptr)
    return fail(CMIF_ERR_INVALID_ARGUMENT,
                "n_refine must be in [1, 4096] with its offsets given");
  for (int k = 0; k < n_refine; ++k)
    if (!(std::fabs(refine_offsets[k]) <= 1.0))
      return fail(CMIF_ERR_INVALID_ARGUMENT, "refinement offsets must lie in [-1, 1]");
  cmif_status s = check_inputs(plan, in);
  if (s != CMIF_OK) return s;
  // stage (i): Alg. 1 over the plan's angle grid, into best
  s = cmif_align(plan, in, best, nullptr, stats, persistent, persistent_bytes,
                 scratch, scratch_bytes, stream);
  if (s != CMIF_OK) return s;
  DeviceGuard dg(plan->d.device);
  if (!dg.ok) return fail(CMIF_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int np = plan->d.n_pairs;
  std::vector<cmif_best> grid((size_t)np);
  HIP_TRY(hipMemcpyAsync(grid.data(), best, np * sizeof(cmif_best),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // stage (ii), per image pair: Alg. 1 over theta* + u_k 2 pi / |Omega|
  const double half = 2.0 * M_PI / (double)plan->angles.size();
  std::vector<double> ang((size_t)n_refine);
  for (int p = 0; p < np; ++p) {
    const PairPlan& g = plan->pairs[p];
    const double th0 = grid[p].angle_index >= 0 ? grid[p].angle_rad : 0.0;
    for (int k = 0; k < n_refine; ++k) ang[k] = th0 + refine_offsets[k] * half;
    cmif_plan_desc d = plan->d;
    d.n_pairs = 1;
    d.h_a = &g.ha; d.w_a = &g.wa; d.h_b = &g.hb; d.w_b = &g.wb;
    d.n_angles = n_refine;
    d.angles_rad = ang.data();
    d.flags = (plan->d.flags & ~(uint32_t)CMIF_FLAG_AUTOTUNE) | CMIF_FLAG_NO_GRAPH;
    // no more angles per pass than the grid plan: the workspace it was
    // given then fits this plan too
    d.angle_batch = plan->batch;
    d.tune_cache_path = nullptr;
    const int32_t win[4] = {1 - g.eha, g.ehb - 1, 1 - g.ewa, g.ewb - 1};
    d.window = plan->windowed ? win : nullptr;
    cmif_plan_t p2 = nullptr;
    s = cmif_plan(&d, &p2);
    if (s != CMIF_OK) return s;
    p2->rows_per_wg = plan->rows_per_wg;
    p2->bpw = plan->bpw;
    p2->xcd = plan->xcd;
    p2->pc_half = plan->pc_half;
    p2->pc_maxr = plan->pc_maxr;
    p2->pc_ba = plan->pc_ba;
    const uint8_t* la = in->labels_a[p];
    const uint8_t* lb = in->labels_b[p];
    const uint8_t* ma = in->mask_a ? in->mask_a[p] : nullptr;
    const uint8_t* mb = in->mask_b ? in->mask_b[p] : nullptr;
    cmif_inputs one{};
    one.labels_a = &la; one.labels_b = &lb; one.mask_a = &ma; one.mask_b = &mb;
    s = cmif_align(p2, &one, best + p, nullptr, stats, persistent,
                   persistent_bytes, scratch, scratch_bytes, stream);
    cmif_plan_free(p2);
    if (s != CMIF_OK) return s;
    HIP_TRY(launch_two_stage_combine(grid[p], best + p,
                                     grid_best ? grid_best + p : nullptr,
                                     refine_best ? refine_best + p : nullptr,
                                     (int)plan->angles.size(), st));
  }
  return CMIF_OK;
}

cmif_status cmif_corner_error(const cmif_best* result, int32_t h_a, int32_t w_a,
                              int32_t h_b, int32_t w_b, const double* truth,
                              double* error_px) {
  g_err.clear();
  if (!result || !truth || !error_px)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (h_a < 1 || w_a < 1 || h_b < 1 || w_b < 1)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "image sides must be >= 1");
  // the result's correspondence A -> B: x -> R(theta)(x + chi - c_B) + c_B
  // (the identity when Alg. 1 kept it)
  const double th = result->angle_index >= 0 ? result->angle_rad : 0.0;
  const double ct = std::cos(th), sn = std::sin(th);
  const double cx = 0.5 * (w_b - 1), cy = 0.5 * (h_b - 1);
  const double cxs[4] = {0.0, (double)(w_a - 1), 0.0, (double)(w_a - 1)};
  const double cys[4] = {0.0, 0.0, (double)(h_a - 1), (double)(h_a - 1)};
  double sum = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double vx = cxs[k] + result->dx - cx, vy = cys[k] + result->dy - cy;
    const double rx = ct * vx - sn * vy + cx, ry = sn * vx + ct * vy + cy;
    const double tx = truth[0] * cxs[k] + truth[1] * cys[k] + truth[2];
    const double ty = truth[3] * cxs[k] + truth[4] * cys[k] + truth[5];
    sum += std::hypot(rx - tx, ry - ty);
  }
  *error_px = 0.25 * sum;
  return CMIF_OK;
}

cmif_status cmif_kmeans(const float* image, const uint8_t* mask,
                        int64_t n_pixels, int32_t channels, int32_t k,
                        const int32_t* init_idx, const int32_t* batches,
                        int32_t iters, int32_t batch, double* centers,
                        uint8_t* labels, uint32_t* bad_indices, void* stream) {
  if (!image || !centers || !labels)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "image, centers and labels are required");
  if (n_pixels < 1) return fail(CMIF_ERR_INVALID_ARGUMENT, "n_pixels must be >= 1");
  if (k < 1 || k > 64) return fail(CMIF_ERR_INVALID_ARGUMENT, "k must be in [1, 64]");
  if (channels < 1 || channels > 8)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "channels must be in [1, 8]");
  if (iters < 0 || iters > 100000)
    return fail(CMIF_ERR_INVALID_ARGUMENT, "iters must be in [0, 100000]");
  if (iters > 0 && (!batches || batch < 1 || batch > 8192))
    return fail(CMIF_ERR_INVALID_ARGUMENT,
                "iters > 0 needs batches and batch in [1, 8192]");
  int ndev = 0, dev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(CMIF_ERR_NO_DEVICE, "no HIP device");
  if (hipGetDevice(&dev) != hipSuccess) return fail(CMIF_ERR_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(CMIF_ERR_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CMIF_ERR_NO_DEVICE,
                std::string("libcmif is built for gfx950, device is ") + prop.gcnArchName);
  KmeansArgs ka{};
  ka.img = image; ka.mask = mask; ka.n = n_pixels; ka.m = channels; ka.k = k;
  ka.init_idx = init_idx; ka.batches = iters > 0 ? batches : nullptr;
  ka.iters = iters; ka.batch = iters > 0 ? batch : 1;
  ka.centers = centers; ka.labels = labels; ka.bad = bad_indices;
  const hipError_t e = launch_kmeans(ka, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(CMIF_ERR_DEVICE, std::string("k-means launch: ") + hipGetErrorString(e));
  return CMIF_OK;
}

}  // extern "C"
