// Forward 2D real-to-complex transforms of the masked level-set indicators
// (Sec. 3.1, Eq. 8) of A (once) and of the rotated B (per angle).
//
// k_fwd_rows: one workgroup per image row (and angle).  Each lane resamples
//   its pixels of the row by the fixed-point nearest-neighbour rotation
//   (Sec. 3.6), then every team transforms two level sets (or, for soft
//   memberships, two membership channels times the mask) at once: the
//   complex input L_a + i L_{a+1} (zero-padded to P_w) goes through one
//   forward FFT and the two real spectra are separated with the Hermitian
//   mirror X(P - k).  Output: X[label][tile][y][TW], k_x in [0, P_w/2) with
//   the k_x = 0 and k_x = P_w/2 values packed in slot 0.
// k_fwd_cols: one workgroup per (tile of TW columns, label, angle); the tile
//   (H rows x 64 B) is read coalesced into LDS, each team transforms one
//   column along y (zero-padded to P_h) and writes it contiguously as
//   F[label][c][k_y].  In circular mode the H rows are displacement-map rows
//   and go to their circular positions (the soft adjoint transforms its
//   per-displacement weights this way).
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"

namespace cmif {

__device__ __forceinline__ int floordiv_pos_pow2(long long a, int shift) {
  // floor(a / 2^shift) for any sign (arithmetic shift)
  return (int)(a >> shift);
}

// Lanes of the forward row kernel: up to four teams, at most 512 (at 1024
// lanes the launch bound leaves 128 registers per lane and the 2048-point
// FP64 kernel spilled).
constexpr int fwd_rows_lanes(int team) { return 4 * team <= 512 ? 4 * team : 512; }

template <typename T, int P, int TEAM>
__global__ void __launch_bounds__(fwd_rows_lanes(TEAM))
k_fwd_rows(const uint8_t* __restrict__ lab, const uint8_t* __restrict__ msk,
           const float* __restrict__ memb, int H, int W, int Q, int label0,
           RotArgs rot,
           C2<T>* __restrict__ xrow, long long angle_stride,
           const C2<T>* __restrict__ tw, const uint32_t* __restrict__ gate,
           cmif_stats* __restrict__ stats, long long src_stride) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* smem = reinterpret_cast<C2<T>*>(smem_raw);
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  const int y = blockIdx.x;
  const int beta = blockIdx.y;
  if (gate != nullptr && gate[beta] == 0u) return;  // nothing to redo here
  // batch entry beta reads its own image (the slices of a volume) when
  // src_stride is set, else the one image under rotation beta
  if (src_stride != 0) {
    if (lab) lab += beta * src_stride;
    if (msk) msk += beta * src_stride;
  }
  const int nteams = blockDim.x / TEAM;
  static_assert(TEAM % 64 == 0, "teams of whole waves");
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / TEAM);  // wave-uniform
  const int lane = threadIdx.x % TEAM;
  C2<T>* lds = smem + team * lds_elems(P);

  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  const long long c = rot.c[beta], s = rot.s[beta];
  const long long one = 65536;
  // per pixel of the row: source index in the unrotated image inside the
  // mask, or -1; hard labels resolve it to the label (255 = no level set)
  int srci[R];
  uint8_t lv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int x = lane + TEAM * q;
    int si = -1;
    if (x < W) {
      const long long X = 2LL * x - (W - 1);
      const long long Y = 2LL * y - (H - 1);
      const long long xs2 = c * X - s * Y;
      const long long ys2 = s * X + c * Y;
      const int xs = floordiv_pos_pow2(xs2 + (long long)(W - 1) * one + one, 17);
      const int ys = floordiv_pos_pow2(ys2 + (long long)(H - 1) * one + one, 17);
      if (xs >= 0 && xs < W && ys >= 0 && ys < H) {
        const int src = ys * W + xs;
        if (msk == nullptr || msk[src]) si = src;
      }
    }
    srci[q] = si;
    uint8_t l = 255;
    if (memb == nullptr && si >= 0) {
      // no label image: every in-mask pixel is label 0 (mask overlap counts);
      // labels label0 .. label0+Q-1 become level sets 0 .. Q-1
      const int v = lab ? (int)lab[si] : 0;
      if (v >= label0 && v < label0 + Q) l = (uint8_t)(v - label0);
    }
    lv[q] = l;
  }

  const int npacks = (Q + 1) / 2;
  const int iters = (npacks + nteams - 1) / nteams;
  const long long plane = (long long)(P / 2) * H;  // elements per label
  const long long hw = (long long)H * W;
  C2<T>* out = xrow + beta * angle_stride;
  uint32_t bad = 0u;
  for (int it = 0; it < iters; ++it) {
    const int pk = team + it * nteams;
    const bool active = pk < npacks;
    const int a0 = 2 * pk, a1 = 2 * pk + 1;
    C2<T> v[R];
    if (memb == nullptr) {
#pragma unroll
      for (int q = 0; q < R; ++q)
        v[q] = mk<T>(lv[q] == a0 ? (T)1 : (T)0, lv[q] == a1 ? (T)1 : (T)0);
    } else {
      // soft memberships in place of the indicators (non-finite -> 0)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        float m0 = 0.0f, m1 = 0.0f;
        if (active && srci[q] >= 0) {
          m0 = memb[(long long)a0 * hw + srci[q]];
          if (a1 < Q) m1 = memb[(long long)a1 * hw + srci[q]];
          if (!isfinite(m0)) { m0 = 0.0f; ++bad; }
          if (!isfinite(m1)) { m1 = 0.0f; ++bad; }
        }
        v[q] = mk<T>((T)m0, (T)m1);
      }
    }
    team_fft<T, P, TEAM, -1>(v, lds, ftw, lane);
#pragma unroll
    for (int q = 0; q < R; ++q) lds[lpad(lane + TEAM * q)] = v[q];
    team_sync<TEAM>();
    C2<T> vm[R / 2];
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      const int k = lane + TEAM * q;
      vm[q] = lds[lpad(k == 0 ? 0 : P - k)];
    }
    team_sync<TEAM>();
    if (active) {
#pragma unroll
      for (int q = 0; q < R / 2; ++q) {
        const int k = lane + TEAM * q;
        C2<T> f0, f1;
        if (k == 0) {
          // X(0) and X(P/2) of each real sequence are real: pack them
          f0 = mk<T>(v[0].x, v[R / 2].x);
          f1 = mk<T>(v[0].y, v[R / 2].y);
        } else {
          f0 = mk<T>((v[q].x + vm[q].x) * (T)0.5, (v[q].y - vm[q].y) * (T)0.5);
          f1 = mk<T>((v[q].y + vm[q].y) * (T)0.5, (vm[q].x - v[q].x) * (T)0.5);
        }
        const long long o = ((long long)(k / TW) * H + y) * TW + (k % TW);
        out[(long long)a0 * plane + o] = f0;
        if (a1 < Q) out[(long long)a1 * plane + o] = f1;
      }
    }
  }
  if (memb != nullptr && stats != nullptr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x % 64) == 0 && bad) atomicAdd(&stats->nonfinite_inputs, bad);
  }
}

// CPW columns of the tile per workgroup (one team each): the whole tile
// (TW) up to 2048 points; at 4096 points a tile's columns would need 278 KB
// of LDS, so each workgroup takes CPW of them and reads its 16-byte pieces
// of every row segment.
template <typename T, int P, int TEAM, int CPW>
__global__ void __launch_bounds__(CPW * TEAM)
k_fwd_cols(const C2<T>* __restrict__ xrow, int H, long long x_angle_stride,
           long long x_label_stride, C2<T>* __restrict__ F,
           long long f_angle_stride, long long f_label_stride,
           const C2<T>* __restrict__ tw, const uint32_t* __restrict__ gate,
           int circ_ha, int circ_hb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* smem = reinterpret_cast<C2<T>*>(smem_raw);
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  constexpr int NPART = TW / CPW;
  constexpr int EV = 16 / (int)sizeof(C2<T>);  // elements per 16-byte vector
  static_assert(TW % CPW == 0 && CPW % EV == 0, "column split");
  const int t = blockIdx.x / NPART, part = blockIdx.x % NPART;
  const int lbl = blockIdx.y, beta = blockIdx.z;
  if (gate != nullptr && gate[beta] == 0u) return;
  static_assert(TEAM % 64 == 0, "teams of whole waves");
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / TEAM);  // wave-uniform
  const int lane = threadIdx.x % TEAM;
  const C2<T>* src = xrow + beta * x_angle_stride + lbl * x_label_stride +
                     (long long)t * H * TW;
  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  // tile load (H rows: the workgroup's CPW columns of each 64-byte segment,
  // 16-byte vectors) into LDS, column-swizzled when the whole segment is
  // loaded, for the column reads below
  {
    const float4* s4 = reinterpret_cast<const float4*>(src);
    constexpr int VR = CPW / EV;  // vectors per row
    for (int e = threadIdx.x; e < H * VR; e += blockDim.x) {
      const int y = e / VR, col = (e % VR) * EV;
      const int dcol = NPART == 1 ? (col ^ stage_swz<TW>(y)) : col;
      *reinterpret_cast<float4*>(&smem[y * CPW + dcol]) =
          s4[(y * TW + part * CPW + col) / EV];
    }
  }
  __syncthreads();
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int y = lane + TEAM * q;
    // source row of position y: the row itself, or (circular mode) the map
    // row whose displacement is y mod P_h
    const int sr = circ_ha > 0 ? circ_to_map(y, P, circ_ha, circ_hb) : (y < H ? y : -1);
    const int scol = NPART == 1 ? (team ^ stage_swz<TW>(sr)) : team;
    v[q] = sr >= 0 ? smem[sr * CPW + scol] : mk<T>((T)0, (T)0);
  }
  __syncthreads();
  team_fft<T, P, TEAM, -1>(v, smem + team * lds_elems(P), ftw, lane);
  C2<T>* dst = F + beta * f_angle_stride + lbl * f_label_stride +
               (long long)(t * TW + part * CPW + team) * P;
#pragma unroll
  for (int q = 0; q < R; ++q) dst[lane + TEAM * q] = v[q];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int P>
static hipError_t launch_rows_p(const FwdRowsArgs<T>& a, hipStream_t st) {
  // FP32: one-wave teams up to P = 1024; FP64 keeps P/8 lanes above 512
  // (16 double points per lane do not fit the registers)
  constexpr int TEAM = sizeof(T) == 4 ? pair_col_team<T>(P) : team_for(P);
  const int npacks = (a.Q + 1) / 2;
  const size_t per_team = (size_t)lds_elems(P) * sizeof(C2<T>);
  int nteams = npacks;
  const int max_teams_lds = (int)(65536 / per_team) > 0 ? (int)(65536 / per_team) : 1;
  if (nteams > max_teams_lds) nteams = max_teams_lds;
  if (nteams > fwd_rows_lanes(TEAM) / TEAM) nteams = fwd_rows_lanes(TEAM) / TEAM;
  if (nteams < 1) nteams = 1;
  const size_t shm = per_team * nteams;
  auto fn = k_fwd_rows<T, P, TEAM>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  dim3 grid(a.H, a.nb);
  hipLaunchKernelGGL(fn, grid, dim3(nteams * TEAM), shm, st, a.lab, a.msk,
                     a.memb, a.H, a.W, a.Q, a.label0, a.rot, a.xrow,
                     a.angle_stride, a.tw, a.gate, a.stats, a.src_stride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fwd_rows(int P, const FwdRowsArgs<T>& a, hipStream_t st) {
  switch (P) {
    case 128: return launch_rows_p<T, 128>(a, st);
    case 256: return launch_rows_p<T, 256>(a, st);
    case 512: return launch_rows_p<T, 512>(a, st);
    case 768: return launch_rows_p<T, 768>(a, st);
    case 1024: return launch_rows_p<T, 1024>(a, st);
    case 1536: return launch_rows_p<T, 1536>(a, st);
    case 2048: return launch_rows_p<T, 2048>(a, st);
    case 4096: return launch_rows_p<T, 4096>(a, st);
  }
  return hipErrorInvalidValue;
}

template <typename T, int P>
static hipError_t launch_cols_p(const FwdColsArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = pair_col_team<T>(P);
  constexpr int TW = tile_width<T>();
  // the whole tile per workgroup up to 2048 points, 512 lanes' worth of
  // columns above
  constexpr int CPW = P <= 2048 ? TW : (512 / TEAM < TW ? 512 / TEAM : TW);
  const size_t shm = (size_t)CPW * lds_elems(P) * sizeof(C2<T>);
  auto fn = k_fwd_cols<T, P, TEAM, CPW>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  dim3 grid(a.tiles * (TW / CPW), a.Q, a.nb);
  hipLaunchKernelGGL(fn, grid, dim3(CPW * TEAM), shm, st, a.xrow, a.H,
                     a.x_angle_stride, a.x_label_stride, a.F, a.f_angle_stride,
                     a.f_label_stride, a.tw, a.gate, a.circ_ha, a.circ_hb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fwd_cols(int P, const FwdColsArgs<T>& a, hipStream_t st) {
  switch (P) {
    case 128: return launch_cols_p<T, 128>(a, st);
    case 256: return launch_cols_p<T, 256>(a, st);
    case 512: return launch_cols_p<T, 512>(a, st);
    case 768: return launch_cols_p<T, 768>(a, st);
    case 1024: return launch_cols_p<T, 1024>(a, st);
    case 1536: return launch_cols_p<T, 1536>(a, st);
    case 2048: return launch_cols_p<T, 2048>(a, st);
    case 4096: return launch_cols_p<T, 4096>(a, st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_fwd_rows<float>(int, const FwdRowsArgs<float>&, hipStream_t);
template hipError_t launch_fwd_rows<double>(int, const FwdRowsArgs<double>&, hipStream_t);
template hipError_t launch_fwd_cols<float>(int, const FwdColsArgs<float>&, hipStream_t);
template hipError_t launch_fwd_cols<double>(int, const FwdColsArgs<double>&, hipStream_t);

}  // namespace cmif
