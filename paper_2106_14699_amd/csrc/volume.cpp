// CMIF of 3-D label volumes (cmif_compute_volume): the correlations of
// Eq. 7 over three axes and the entropies of Eq. 12 per 3-D displacement,
// with the 2-D kernels for the in-plane axes and the depth kernels of
// k_volume.hip.  Schedule (caller's stream):
//   tables       twiddles for P_w, P_h, P_d; log tables
//   check        labels >= Q inside a mask -> stats.label_errors
//   A, B         2-D forward transforms of the level sets, slice by slice
//                (batches of up to 16 slices) -> F2; depth transform -> F3
//   G            per pair: conj(F3_a) F3_b, inverse depth transform, the
//                depth displacements' 2-D spectra
//   per dz       pair column pass (products given) and pair row pass with
//                the fused entropy sums -> MI and N slice dz; count digests;
//                FP32: flagged pairs counted as unresolved
//   argmax       Alg. 1 over the whole (dz, dy, dx) map
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "kernels.h"

using namespace cmif;

namespace {

constexpr int kZSizes[] = {32, 64, 128, 256, 512};

int zsize_at_least(int v) {
  for (int p : kZSizes)
    if (p >= v) return p;
  return 0;
}

// in-plane lengths: those of cmif_plan up to 2048 points
int fft_size_at_least_v(int v) {
  for (int p : kFftSizes)
    if (p >= v && p <= kMaxSoftP) return p;
  return 0;
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

cmif_status err(cmif_status s, const std::string& m) { return set_error(s, m.c_str()); }

struct VolGeom {
  int da, ha, wa, db, hb, wb, qa, qb, sd, sh, sw, pd, ph, pw, half, npos;
  size_t E;  // complex element bytes
};

struct VolLayout {
  size_t tw_w, tw_h, tw_d, logtab, xlog, xa, f2a, f2b, f3a, f3b, g, z, mi, n,
      maxn, flags, partial, running, best2, end;
};

constexpr int kSliceBatch = kMaxBatch;

int rows_per_chunk_v(long long rows) { return (int)((rows + 255) / 256); }

cmif_status geometry(const cmif_volume_desc* d, VolGeom* g) {
  if (!d) return err(CMIF_ERR_INVALID_ARGUMENT, "desc is NULL");
  const int s[6] = {d->d_a, d->h_a, d->w_a, d->d_b, d->h_b, d->w_b};
  for (int v : s)
    if (v < 1 || v > kMaxSoftP)
      return err(CMIF_ERR_INVALID_ARGUMENT, "volume sides must be in [1, 2048]");
  if (d->q_a < 1 || d->q_a > 64 || d->q_b < 1 || d->q_b > 64)
    return err(CMIF_ERR_INVALID_ARGUMENT, "q_a and q_b must be in [1, 64]");
  if (!(d->gamma >= 0.0 && d->gamma <= 1.0))
    return err(CMIF_ERR_INVALID_ARGUMENT, "gamma must be in [0, 1]");
  if (d->precision != CMIF_PREC_FP32_ROUNDED && d->precision != CMIF_PREC_FP64)
    return err(CMIF_ERR_INVALID_ARGUMENT, "unknown precision");
  g->da = d->d_a; g->ha = d->h_a; g->wa = d->w_a;
  g->db = d->d_b; g->hb = d->h_b; g->wb = d->w_b;
  g->qa = d->q_a; g->qb = d->q_b;
  g->sd = g->da + g->db - 1; g->sh = g->ha + g->hb - 1; g->sw = g->wa + g->wb - 1;
  g->pd = zsize_at_least(g->sd);
  g->ph = fft_size_at_least_v(g->sh);
  g->pw = fft_size_at_least_v(g->sw);
  if (g->pd == 0 || g->ph == 0 || g->pw == 0)
    return err(CMIF_ERR_UNSUPPORTED,
               "transform above 512 along depth or 2048 in-plane");
  PairRowsConfig rc;
  const size_t er = d->precision == CMIF_PREC_FP64 ? sizeof(double) : sizeof(float);
  if (!pair_rows_config(er, g->pw, g->qb, &rc))
    return err(CMIF_ERR_UNSUPPORTED, "q_b too large for the row kernel");
  g->half = g->pw / 2;
  g->npos = g->half * g->ph;
  g->E = 2 * er;
  return CMIF_OK;
}

VolLayout layout(const VolGeom& g) {
  VolLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += up256(b); return r; };
  const size_t tw = sizeof(float2) + sizeof(double2);
  L.tw_w = take((size_t)g.pw * tw);
  L.tw_h = take((size_t)g.ph * tw);
  L.tw_d = take((size_t)g.pd * tw);
  L.logtab = take(512 * sizeof(double));
  L.xlog = take(kXlogN * sizeof(double));
  const int qmax = std::max(g.qa, g.qb), hmax = std::max(g.ha, g.hb);
  L.xa = take((size_t)kSliceBatch * qmax * g.half * hmax * g.E);
  L.f2a = take((size_t)g.da * g.qa * g.npos * g.E);
  L.f2b = take((size_t)g.db * g.qb * g.npos * g.E);
  L.f3a = take((size_t)g.qa * g.pd * g.npos * g.E);
  L.f3b = take((size_t)g.qb * g.pd * g.npos * g.E);
  const size_t npairs = (size_t)g.qa * g.qb;
  L.g = take((size_t)g.sd * npairs * g.npos * g.E);
  L.z = take((size_t)z_pair_slots((int)npairs) * g.half * g.sh * g.E);
  const size_t map = (size_t)g.sd * g.sh * g.sw;
  L.mi = take(map * sizeof(double));
  L.n = take(map * sizeof(int32_t));
  L.maxn = take(sizeof(uint32_t));
  L.flags = take(npairs * sizeof(uint32_t));
  const long long rows = (long long)g.sd * g.sh;
  const int rpc = rows_per_chunk_v(rows);
  L.partial = take((size_t)((rows + rpc - 1) / rpc) * sizeof(ArgPartial));
  L.running = take(sizeof(cmif_best));
  L.best2 = take(sizeof(cmif_best));
  L.end = o;
  return L;
}

#define VTRY(expr)                                                           \
  do {                                                                       \
    const hipError_t _e = (expr);                                            \
    if (_e != hipSuccess)                                                    \
      return err(CMIF_ERR_DEVICE, std::string(#expr) + ": " +                \
                                      hipGetErrorString(_e));                \
  } while (0)

template <typename T>
const C2<T>* twp(const uint8_t* base, size_t off, int len) {
  return reinterpret_cast<const C2<T>*>(
      base + off + (sizeof(T) == 8 ? (size_t)len * sizeof(float2) : 0));
}

// 2-D spectra of every slice of one volume (labels 0..Q-1), then its depth
// transform.
template <typename T>
cmif_status forward_volume(const VolGeom& g, const VolLayout& L, uint8_t* ws,
                           const uint8_t* lab, const uint8_t* msk, int D, int H,
                           int W, int Q, size_t f2_off, size_t f3_off,
                           cmif_stats* stats, hipStream_t st) {
  using CT = C2<T>;
  CT* xrow = reinterpret_cast<CT*>(ws + L.xa);
  CT* f2 = reinterpret_cast<CT*>(ws + f2_off);
  for (int z0 = 0; z0 < D; z0 += kSliceBatch) {
    const int nb = std::min(kSliceBatch, D - z0);
    FwdRowsArgs<T> r{};
    r.lab = lab + (size_t)z0 * H * W;
    r.msk = msk ? msk + (size_t)z0 * H * W : nullptr;
    r.stats = stats;
    r.H = H; r.W = W; r.Q = Q; r.nb = nb;
    for (int b = 0; b < nb; ++b) { r.rot.c[b] = 65536; r.rot.s[b] = 0; }
    r.xrow = xrow;
    r.angle_stride = (long long)Q * g.half * H;
    r.tw = twp<T>(ws, L.tw_w, g.pw);
    r.src_stride = (long long)H * W;
    VTRY(launch_fwd_rows<T>(g.pw, r, st));
    FwdColsArgs<T> c{};
    c.xrow = xrow; c.H = H; c.tiles = g.half / tile_width<T>(); c.Q = Q; c.nb = nb;
    c.x_angle_stride = (long long)Q * g.half * H;
    c.x_label_stride = (long long)g.half * H;
    c.F = f2 + (size_t)z0 * Q * g.npos;
    c.f_angle_stride = (long long)Q * g.npos;
    c.f_label_stride = g.npos;
    c.tw = twp<T>(ws, L.tw_h, g.ph);
    VTRY(launch_fwd_cols<T>(g.ph, c, st));
  }
  ZfftArgs<T> zf{};
  zf.F2 = f2; zf.z_stride = (long long)Q * g.npos; zf.label_stride2 = g.npos;
  zf.D = D; zf.Q = Q; zf.npos = g.npos;
  zf.F3 = reinterpret_cast<CT*>(ws + f3_off);
  zf.tw = twp<T>(ws, L.tw_d, g.pd);
  VTRY(launch_zfft<T>(g.pd, zf, st));
  return CMIF_OK;
}

template <typename T>
cmif_status run_volume(const VolGeom& g, const VolLayout& L, uint8_t* ws,
                       const cmif_volume_desc* d, const uint8_t* la,
                       const uint8_t* ma, const uint8_t* lb, const uint8_t* mb,
                       double* mi_out, int32_t* n_out, uint64_t* digest,
                       cmif_best3d* best, cmif_stats* stats, hipStream_t st) {
  using CT = C2<T>;
  const bool fp64 = sizeof(T) == 8;
  const int qa = g.qa, qb = g.qb, npairs = qa * qb;
  for (auto [off, len] : {std::pair<size_t, int>{L.tw_w, g.pw}, {L.tw_h, g.ph},
                          {L.tw_d, g.pd}}) {
    const bool first = off == L.tw_w;
    VTRY(launch_init_tables(ws + off, ws + off + (size_t)len * sizeof(float2), len,
                            first ? reinterpret_cast<double*>(ws + L.logtab) : nullptr,
                            first ? reinterpret_cast<double*>(ws + L.xlog) : nullptr,
                            st));
  }
  if (stats) {
    VTRY(launch_check_labels(la, ma, (long long)g.da * g.ha * g.wa, qa, stats, st));
    VTRY(launch_check_labels(lb, mb, (long long)g.db * g.hb * g.wb, qb, stats, st));
  }
  cmif_status s = forward_volume<T>(g, L, ws, la, ma, g.da, g.ha, g.wa, qa, L.f2a,
                                    L.f3a, stats, st);
  if (s != CMIF_OK) return s;
  s = forward_volume<T>(g, L, ws, lb, mb, g.db, g.hb, g.wb, qb, L.f2b, L.f3b, stats,
                        st);
  if (s != CMIF_OK) return s;
  CT* G = reinterpret_cast<CT*>(ws + L.g);
  ZpairArgs<T> zp{};
  zp.F3A = reinterpret_cast<CT*>(ws + L.f3a);
  zp.F3B = reinterpret_cast<CT*>(ws + L.f3b);
  zp.QA = qa; zp.QB = qb; zp.npos = g.npos; zp.ph = g.ph; zp.DA = g.da; zp.DB = g.db;
  zp.G = G; zp.tw = twp<T>(ws, L.tw_d, g.pd);
  VTRY(launch_zpair<T>(g.pd, zp, st));

  const long long slice = (long long)g.sh * g.sw;
  double* mi = mi_out ? mi_out : reinterpret_cast<double*>(ws + L.mi);
  int32_t* n = n_out ? n_out : reinterpret_cast<int32_t*>(ws + L.n);
  uint32_t* maxn = reinterpret_cast<uint32_t*>(ws + L.maxn);
  uint32_t* flags = reinterpret_cast<uint32_t*>(ws + L.flags);
  CT* Z = reinterpret_cast<CT*>(ws + L.z);
  VTRY(launch_fill_u32(maxn, 0u, 1, st));
  if (digest) VTRY(launch_fill_u32(reinterpret_cast<uint32_t*>(digest), 0u,
                                   2LL * npairs, st));
  for (int k = 0; k < g.sd; ++k) {
    if (!fp64) VTRY(launch_fill_u32(flags, 0u, npairs, st));
    PairColsArgs<T> pc{};
    pc.FA = nullptr;
    pc.FB = G + (size_t)k * npairs * g.npos;
    pc.fb_angle_stride = 0; pc.fb_label_stride = g.npos;
    pc.QA = qa; pc.QB = qb; pc.ha = g.ha; pc.hb = g.hb; pc.sh = g.sh;
    pc.tiles = g.half / tile_width<T>(); pc.nb = 1; pc.Z = Z;
    pc.z_angle_stride = 0; pc.z_pair_stride = (long long)g.half * g.sh;
    pc.tw = twp<T>(ws, L.tw_h, g.ph); pc.zg = z_group_rt<T>(g.pw);
    VTRY(launch_pair_cols<T>(g.ph, pc, st));
    PairRowsArgs<T> pr{};
    pr.Z = Z; pr.z_angle_stride = 0; pr.z_pair_stride = pc.z_pair_stride;
    pr.QA = qa; pr.QB = qb; pr.wa = g.wa; pr.wb = g.wb; pr.sh = g.sh; pr.sw = g.sw;
    pr.ph = g.ph; pr.nb = 1; pr.tw = twp<T>(ws, L.tw_w, g.pw);
    pr.logtab = reinterpret_cast<const double*>(ws + L.logtab);
    pr.xlogtab = reinterpret_cast<const double*>(ws + L.xlog);
    pr.rows_per_wg = 1; pr.bpw = 0; pr.full_x = 1;
    pr.mi = mi + k * slice; pr.mi_angle_stride = slice;
    pr.n = n + k * slice; pr.n_angle_stride = slice;
    pr.maxn = maxn; pr.flags = fp64 ? nullptr : flags; pr.stats = stats;
    VTRY(launch_pair_rows<T>(g.pw, pr, st));
    if (digest) {
      PairCountsArgs<T> pk{};
      pk.Z = Z; pk.z_angle_stride = 0; pk.z_pair_stride = pc.z_pair_stride;
      pk.QA = qa; pk.QB = qb; pk.wa = g.wa; pk.wb = g.wb; pk.sh = g.sh; pk.sw = g.sw;
      pk.ph = g.ph; pk.nb = 1; pk.tw = twp<T>(ws, L.tw_w, g.pw);
      pk.digest = digest; pk.digest_index0 = k * slice;
      VTRY(launch_pair_counts<T>(g.pw, pk, st));
    }
    if (!fp64 && stats) VTRY(launch_count_flags(flags, npairs, stats, st));
  }
  if (best) {
    const long long rows = (long long)g.sd * g.sh;
    const int rpc = rows_per_chunk_v(rows);
    const int nchunks = (int)((rows + rpc - 1) / rpc);
    ArgmaxArgs am{};
    am.mi = mi; am.n = n; am.angle_stride = (long long)g.sd * slice; am.maxn = maxn;
    am.sh = (int)rows; am.sw = g.sw; am.nb = 1; am.rows_per_chunk = rpc;
    am.nchunks = nchunks; am.gamma = d->gamma;
    am.partial = reinterpret_cast<ArgPartial*>(ws + L.partial);
    VTRY(launch_argmax(am, st));
    ArgmaxFinalArgs af{};
    af.partial = am.partial; af.nb = 1; af.nchunks = nchunks; af.sw = g.sw;
    af.ha = 1;  // the flattened (dz, dy) row is decoded below
    af.wa = g.wa; af.angle0 = 0; af.angles[0] = 0.0; af.per_angle = nullptr;
    af.running = reinterpret_cast<cmif_best*>(ws + L.running);
    af.first_batch = 1; af.last_batch = 1;
    af.best_out = reinterpret_cast<cmif_best*>(ws + L.best2);
    VTRY(launch_argmax_final(af, st));
    VTRY(launch_best3d(af.best_out, best, g.sh, g.da, g.ha, st));
  }
  return CMIF_OK;
}

}  // namespace

extern "C" {

cmif_status cmif_volume_workspace_size(const cmif_volume_desc* desc,
                                       size_t* bytes) {
  if (!bytes) return err(CMIF_ERR_INVALID_ARGUMENT, "bytes is NULL");
  VolGeom g{};
  const cmif_status s = geometry(desc, &g);
  if (s != CMIF_OK) return s;
  *bytes = layout(g).end;
  return CMIF_OK;
}

cmif_status cmif_compute_volume(const cmif_volume_desc* desc,
                                const uint8_t* labels_a, const uint8_t* mask_a,
                                const uint8_t* labels_b, const uint8_t* mask_b,
                                double* mi, int32_t* n, uint64_t* digest,
                                cmif_best3d* best, cmif_stats* stats,
                                void* workspace, size_t workspace_bytes,
                                void* stream) {
  VolGeom g{};
  cmif_status s = geometry(desc, &g);
  if (s != CMIF_OK) return s;
  if (!labels_a || !labels_b)
    return err(CMIF_ERR_INVALID_ARGUMENT, "labels are NULL");
  const VolLayout L = layout(g);
  if (workspace_bytes < L.end)
    return err(CMIF_ERR_WORKSPACE_TOO_SMALL,
               "workspace too small: need " + std::to_string(L.end));
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return err(CMIF_ERR_INVALID_ARGUMENT, "workspace NULL or not 256-byte aligned");
  int ndev = 0, prev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return err(CMIF_ERR_NO_DEVICE, "no HIP device");
  if (desc->device < 0 || desc->device >= ndev)
    return err(CMIF_ERR_NO_DEVICE, "device ordinal out of range");
  if (hipGetDevice(&prev) != hipSuccess) return err(CMIF_ERR_DEVICE, "hipGetDevice failed");
  if (prev != desc->device && hipSetDevice(desc->device) != hipSuccess)
    return err(CMIF_ERR_NO_DEVICE, "cannot select the device");
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  s = desc->precision == CMIF_PREC_FP64
          ? run_volume<double>(g, L, ws, desc, labels_a, mask_a, labels_b, mask_b, mi,
                               n, digest, best, stats, st)
          : run_volume<float>(g, L, ws, desc, labels_a, mask_a, labels_b, mask_b, mi,
                              n, digest, best, stats, st);
  if (prev != desc->device) (void)hipSetDevice(prev);
  return s;
}

}  // extern "C"
