// Soft-membership CMIF: forward row pass and the adjoint (gradient) passes.
//
// The soft variant replaces the level-set indicators of Eq. 8 by real
// memberships p_a(x) = M_A(x) m_a(x), q_b(y) = M_B(y) n_b(y), so the joint
// C_ab(chi) = sum_x p_a(x) q_b(x + chi) of Eq. 9 is real-valued.  The
// marginals and N are sums of the joint (C_a = sum_b C_ab, C_b = sum_a C_ab,
// N = sum_ab C_ab), and Eq. 12 gives
//   MI = log2 N + (sum C_ab log2 C_ab - sum C_a log2 C_a - sum C_b log2 C_b) / N
// with 0 log 0 = 0 and no rounding.  Spatial weights in place of binary masks
// (Sec. 3.3, Eq. 13) are the nearest relative in the paper.
//
// Derivative (from the formula above, every C being a function of C_ab):
//   dMI/dC_ab = (log2(C_ab N / (C_a C_b)) - MI) / N,
// so with upstream weights w(chi) = dL/dMI(chi) and G_ab = w dMI/dC_ab:
//   dL/dp_a(x) = sum_b sum_chi G_ab(chi) q_b(x + chi)   (correlation)
//   dL/dq_b(y) = sum_a sum_chi G_ab(chi) p_a(y - chi)   (convolution)
// In the frequency domain (F = forward DFT, P_h x P_w grid, G placed at
// chi mod P): F[dL/dp_a] = sum_b conj(F G_ab) F q_b and
// F[dL/dq_b] = sum_a F p_a F G_ab.
//
// Kernels:
//   k_soft_rows       forward row pass (one workgroup per map row and angle):
//                     real joints, FP64 entropy sums, MI map; optionally the
//                     state the adjoint needs: N, log2 N - MI, log2 C_a,
//                     log2 C_b per displacement (float planes)
//   k_soft_grad_rows  joints again, G_ab per displacement, forward transform
//                     along x -> half spectra of G in the pair-column layout
//   (k_fwd_cols in circular mode then transforms G along y)
//   k_soft_grad_cols  per (tile, channel): spectral sum over the partner
//                     channels and inverse transform along y -> row spectra
//   k_soft_grad_out   inverse transform along x, times the mask -> gradient
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"
#include "rows_common.h"

namespace cmif {

__device__ __forceinline__ double xlog2x_real(double c) {
  return c > 0.0 ? c * log2(c) : 0.0;
}

// Saved-state planes per angle: [0] N, [1] log2 N - MI, [2 + a] log2 C_a,
// [2 + Q_A + b] log2 C_b, each [S_h][S_w] in the transform precision T.
template <typename T, int P, int TEAM, int BPW, int NTMAX>
__global__ void __launch_bounds__(NTMAX)
k_soft_rows(const C2<T>* __restrict__ Z, long long z_angle_stride,
            long long z_pair_stride, int QA, int QB, int wa, int wb, int sh,
            int sw, int ph, const C2<T>* __restrict__ tw,
            double* __restrict__ mi_out, long long mi_angle_stride,
            T* __restrict__ save, long long save_angle_stride) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nteams = blockDim.x / TEAM;
  const int NT = blockDim.x;
  C2<T>* exch = reinterpret_cast<C2<T>*>(smem_raw);
  double* sa_l = reinterpret_cast<double*>(exch + (size_t)nteams * lds_elems(P));
  double* n_l = sa_l + P;
  const int i = blockIdx.x, beta = blockIdx.y;
  const int tid = threadIdx.x, team = tid / TEAM, lane = tid % TEAM;
  C2<T>* lds = exch + team * lds_elems(P);
  double* part = reinterpret_cast<double*>(lds);  // team partial, between FFTs

  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  const T scale = (T)1 / ((T)ph * (T)P);
  const int tile_stride = z_tile_stride<T, P>(sh);
  const int b_first = team * BPW;
  const long long plane = (long long)sh * sw;
  const long long mrow = (long long)i * sw;
  T* sv = save ? save + beta * save_angle_stride : nullptr;
  const C2<T>* zrow = Z + beta * z_angle_stride + z_row_offset<T, P>(i);

  // the fold loops below give every x to the same thread: no barrier needed
  for (int x = tid; x < P; x += NT) { sa_l[x] = 0.0; n_l[x] = 0.0; }

  double cb[BPW][R], sab[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    sab[q] = 0.0;
#pragma unroll
    for (int bb = 0; bb < BPW; ++bb) cb[bb][q] = 0.0;
  }
  for (int a = 0; a < QA; ++a) {
    double ca[R];
#pragma unroll
    for (int q = 0; q < R; ++q) ca[q] = 0.0;
#pragma unroll
    for (int pk = 0; pk < BPW / 2; ++pk) {
      const int b0 = b_first + 2 * pk, b1 = b0 + 1;
      const bool has0 = b0 < QB, has1 = b1 < QB;
      C2<T> w[R];
      if (has0) {
        load_pack<T, P, TEAM>(zrow + z_pair_offset<T, P>(a * QB + b0, z_pair_stride),
                              zrow + z_pair_offset<T, P>(a * QB + b1, z_pair_stride),
                              has1, tile_stride, lane, w);
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) w[q] = mk<T>((T)0, (T)0);
      }
      team_fft<T, P, TEAM, +1>(w, lds, ftw, lane);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if (circ_to_map(lane + TEAM * q, P, wa, wb) >= 0) {
          const double c0 = fmax((double)(w[q].x * scale), 0.0);
          const double c1 = has1 ? fmax((double)(w[q].y * scale), 0.0) : 0.0;
          cb[2 * pk][q] += c0;
          cb[2 * pk + 1][q] += c1;
          ca[q] += c0 + c1;
          sab[q] += xlog2x_real(c0) + xlog2x_real(c1);
        }
      }
    }
    // C_a: team partials through the exchange buffers, fixed-order sum
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) part[lane + TEAM * q] = ca[q];
    __syncthreads();
    for (int x = tid; x < P; x += NT) {
      const int j = circ_to_map(x, P, wa, wb);
      if (j >= 0) {
        double c = 0.0;
        for (int g = 0; g < nteams; ++g)
          c += reinterpret_cast<const double*>(exch + g * lds_elems(P))[x];
        sa_l[x] += xlog2x_real(c);
        n_l[x] += c;
        if (sv) sv[(2 + a) * plane + mrow + j] = c > 0.0 ? (T)log2(c) : (T)0;
      }
    }
    __syncthreads();  // the exchange buffers are the next FFT's
  }
  // S_AB - S_B per team (and log2 C_b), then the fixed-order team sum
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = circ_to_map(lane + TEAM * q, P, wa, wb);
    double sb = 0.0;
#pragma unroll
    for (int bb = 0; bb < BPW; ++bb) {
      const double c = cb[bb][q];
      sb += xlog2x_real(c);
      const int b = b_first + bb;
      if (sv && j >= 0 && b < QB)
        sv[(2 + QA + b) * plane + mrow + j] = c > 0.0 ? (T)log2(c) : (T)0;
    }
    sab[q] -= sb;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) part[lane + TEAM * q] = sab[q];
  __syncthreads();
  for (int x = tid; x < P; x += NT) {
    const int j = circ_to_map(x, P, wa, wb);
    if (j >= 0) {
      double tsum = 0.0;
      for (int g = 0; g < nteams; ++g)
        tsum += reinterpret_cast<const double*>(exch + g * lds_elems(P))[x];
      const double nn = n_l[x];
      const double l2n = nn > 0.0 ? log2(nn) : 0.0;
      const double mi = nn > 0.0 ? l2n + (tsum - sa_l[x]) / nn : 0.0;
      if (mi_out) mi_out[beta * mi_angle_stride + mrow + j] = mi;
      if (sv) {
        sv[mrow + j] = (T)nn;
        sv[plane + mrow + j] = (T)(l2n - mi);
      }
    }
  }
}

// Adjoint, row pass: workgroup = map row i; teams take pairs two at a time.
// For every used displacement j of the row:
//   G_ab = w / N * (log2 C_ab - log2 C_a - log2 C_b + log2 N - MI)
// (0 where w = 0, N <= 0 or C_ab <= 0), then G0 + i G1 goes through one
// forward transform along x and the two half spectra are written to
// ZG[pair][tile][i][TW] with slot 0 packing k_x = 0 and k_x = P_w/2.
template <typename T, int P, int TEAM>
__global__ void __launch_bounds__(4 * TEAM)
k_soft_grad_rows(const C2<T>* __restrict__ Z, long long z_pair_stride, int QA,
                 int QB, int wa, int wb, int sh, int sw, int ph,
                 const C2<T>* __restrict__ tw, const double* __restrict__ grad_mi,
                 const T* __restrict__ save, C2<T>* __restrict__ ZG) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* exch = reinterpret_cast<C2<T>*>(smem_raw);
  const int nteams = blockDim.x / TEAM;
  const int i = blockIdx.x;
  const int tid = threadIdx.x, team = tid / TEAM, lane = tid % TEAM;
  C2<T>* lds = exch + team * lds_elems(P);
  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  const T scale = (T)1 / ((T)ph * (T)P);
  const long long plane = (long long)sh * sw;
  const long long mrow = (long long)i * sw;
  const int nq = QA * QB;
  const int npk = (nq + 1) / 2;
  const int iters = (npk + nteams - 1) / nteams;

  // per position of the row: w / N and log2 N - MI (0 where unused)
  T wn[R], kk[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int j = circ_to_map(lane + TEAM * q, P, wa, wb);
    wn[q] = (T)0;
    kk[q] = (T)0;
    if (j >= 0) {
      const T nn = save[mrow + j];
      const double g = grad_mi[mrow + j];
      if (nn > (T)0 && g != 0.0) {
        wn[q] = (T)(g / (double)nn);
        kk[q] = save[plane + mrow + j];
      }
    }
  }
  const T* lca = save + 2 * plane + mrow;
  const T* lcb = save + (2 + QA) * plane + mrow;
  for (int it = 0; it < iters; ++it) {
    const int pk = team + it * nteams;
    const int p0 = 2 * pk, p1 = p0 + 1;
    const bool has0 = p0 < nq, has1 = p1 < nq;
    C2<T> w[R];
    if (has0) {
      load_pack<T, P, TEAM>(Z + z_pair_offset<T, P>(p0, z_pair_stride) + z_row_offset<T, P>(i),
                            Z + z_pair_offset<T, P>(p1, z_pair_stride) + z_row_offset<T, P>(i),
                            has1, z_tile_stride<T, P>(sh), lane, w);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) w[q] = mk<T>((T)0, (T)0);
    }
    team_fft<T, P, TEAM, +1>(w, lds, ftw, lane);
    const int a0 = p0 / QB, b0 = p0 % QB, a1 = p1 / QB, b1 = p1 % QB;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = circ_to_map(lane + TEAM * q, P, wa, wb);
      T g0 = (T)0, g1 = (T)0;
      if (has0 && j >= 0 && wn[q] != (T)0) {
        const T c0 = w[q].x * scale;
        if (c0 > (T)0)
          g0 = wn[q] * (log2(c0) - lca[a0 * plane + j] - lcb[b0 * plane + j] + kk[q]);
        if (has1) {
          const T c1 = w[q].y * scale;
          if (c1 > (T)0)
            g1 = wn[q] * (log2(c1) - lca[a1 * plane + j] - lcb[b1 * plane + j] + kk[q]);
        }
      }
      w[q] = mk<T>(g0, g1);
    }
    team_fft<T, P, TEAM, -1>(w, lds, ftw, lane);
#pragma unroll
    for (int q = 0; q < R; ++q) lds[lpad(lane + TEAM * q)] = w[q];
    team_sync<TEAM>();
    C2<T> wm[R / 2];
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      const int k = lane + TEAM * q;
      wm[q] = lds[lpad(k == 0 ? 0 : P - k)];
    }
    team_sync<TEAM>();
    if (has0) {
#pragma unroll
      for (int q = 0; q < R / 2; ++q) {
        const int k = lane + TEAM * q;
        C2<T> f0, f1;
        if (k == 0) {
          f0 = mk<T>(w[0].x, w[R / 2].x);
          f1 = mk<T>(w[0].y, w[R / 2].y);
        } else {
          f0 = mk<T>((w[q].x + wm[q].x) * (T)0.5, (w[q].y - wm[q].y) * (T)0.5);
          f1 = mk<T>((w[q].y + wm[q].y) * (T)0.5, (wm[q].x - w[q].x) * (T)0.5);
        }
        const long long o = ((long long)(k / TW) * sh + i) * TW + (k % TW);
        ZG[(long long)p0 * z_pair_stride + o] = f0;
        if (has1) ZG[(long long)p1 * z_pair_stride + o] = f1;
      }
    }
  }
}

// Adjoint, column pass: workgroup = (tile of TW columns, channel ch of side
// SIDE); team = column c.  SIDE 0 (A): acc = sum_b conj(GH_{ch,b}) F_B,b;
// SIDE 1 (B): acc = sum_a F_A,a GH_{a,ch}.  Column 0 holds two packed
// Hermitian columns, separated and re-packed around the product.  The
// inverse transform along y gives rows y in [0, H) of the side's image,
// stored as GX[ch][tile][y][TW].
template <typename T, int P, int TEAM, int SIDE>
__global__ void __launch_bounds__(tile_width<T>() * TEAM)
k_soft_grad_cols(const C2<T>* __restrict__ GH, const C2<T>* __restrict__ FO,
                 long long f_label_stride, int QA, int QB, int H,
                 C2<T>* __restrict__ GX, long long gx_label_stride,
                 const C2<T>* __restrict__ tw) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* smem = reinterpret_cast<C2<T>*>(smem_raw);
  const int t = blockIdx.x, ch = blockIdx.y;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int c = t * TW + team;
  C2<T>* lds = smem + team * lds_elems(P);
  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  const int npart = SIDE == 0 ? QB : QA;
  C2<T> acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = mk<T>((T)0, (T)0);
  for (int o = 0; o < npart; ++o) {
    const int pair = SIDE == 0 ? ch * QB + o : o * QB + ch;
    const C2<T>* g = GH + (long long)pair * f_label_stride + (long long)c * P;
    const C2<T>* f = FO + (long long)o * f_label_stride + (long long)c * P;
    if (c != 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int k = lane + TEAM * q;
        const C2<T> y = SIDE == 0 ? cmulc<T>(g[k], f[k]) : cmul<T>(f[k], g[k]);
        acc[q] = mk<T>(acc[q].x + y.x, acc[q].y + y.y);
      }
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int k = lane + TEAM * q;
        const int km = k == 0 ? 0 : P - k;
        C2<T> g0, g1, f0, f1;
        unpack0<T>(g[k], g[km], g0, g1);
        unpack0<T>(f[k], f[km], f0, f1);
        const C2<T> y0 = SIDE == 0 ? cmulc<T>(g0, f0) : cmul<T>(f0, g0);
        const C2<T> y1 = SIDE == 0 ? cmulc<T>(g1, f1) : cmul<T>(f1, g1);
        acc[q] = mk<T>(acc[q].x + y0.x - y1.y, acc[q].y + y0.y + y1.x);
      }
    }
  }
  team_fft<T, P, TEAM, +1>(acc, lds, ftw, lane);
  // rows y < H leave through a swizzled LDS tile as 16-byte vectors
  constexpr int EV = 16 / (int)sizeof(C2<T>);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int y = lane + TEAM * q;
    if (y < H) smem[y * TW + (team ^ stage_swz<TW>(y))] = acc[q];
  }
  __syncthreads();
  float4* z4 = reinterpret_cast<float4*>(GX + (long long)ch * gx_label_stride +
                                         (long long)t * H * TW);
  for (int e = threadIdx.x; e < H * TW / EV; e += blockDim.x) {
    const int y = (e * EV) / TW, col = (e * EV) % TW;
    z4[e] = *reinterpret_cast<const float4*>(&smem[y * TW + (col ^ stage_swz<TW>(y))]);
  }
}

// Adjoint, output pass: workgroup = image row y; teams take channels two at
// a time: the two half-spectrum rows form one packed sequence, one inverse
// transform along x gives both real gradient rows, scaled by 1/(P_h P_w)
// and multiplied by the mask.
template <typename T, int P, int TEAM>
__global__ void __launch_bounds__(4 * TEAM)
k_soft_grad_out(const C2<T>* __restrict__ GX, long long gx_label_stride, int Q,
                int H, int W, int ph, const uint8_t* __restrict__ msk,
                const C2<T>* __restrict__ tw, float* __restrict__ grad) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* exch = reinterpret_cast<C2<T>*>(smem_raw);
  const int nteams = blockDim.x / TEAM;
  const int y = blockIdx.x;
  const int tid = threadIdx.x, team = tid / TEAM, lane = tid % TEAM;
  C2<T>* lds = exch + team * lds_elems(P);
  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  const T scale = (T)1 / ((T)ph * (T)P);
  const int npk = (Q + 1) / 2;
  const int iters = (npk + nteams - 1) / nteams;
  const long long hw = (long long)H * W;
  for (int it = 0; it < iters; ++it) {
    const int pk = team + it * nteams;
    const int c0 = 2 * pk, c1 = c0 + 1;
    const bool has0 = c0 < Q, has1 = c1 < Q;
    C2<T> w[R];
    if (has0) {
      load_pack<T, P, TEAM>(GX + (long long)c0 * gx_label_stride + (long long)y * TW,
                            GX + (long long)c1 * gx_label_stride + (long long)y * TW,
                            has1, H * TW, lane, w);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) w[q] = mk<T>((T)0, (T)0);
    }
    team_fft<T, P, TEAM, +1>(w, lds, ftw, lane);
    if (has0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int x = lane + TEAM * q;
        if (x < W) {
          const bool in = msk == nullptr || msk[(long long)y * W + x] != 0;
          grad[(long long)c0 * hw + (long long)y * W + x] =
              in ? (float)(w[q].x * scale) : 0.0f;
          if (has1)
            grad[(long long)c1 * hw + (long long)y * W + x] =
                in ? (float)(w[q].y * scale) : 0.0f;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int P, int BPW, int NTMAX>
static hipError_t launch_sr_cfg(const SoftRowsArgs<T>& a, int nteams, size_t shm,
                                hipStream_t st) {
  constexpr int TEAM = team_for(P);
  auto fn = k_soft_rows<T, P, TEAM, BPW, NTMAX>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(a.sh, a.nb), dim3(nteams * TEAM), shm, st, a.Z,
                     a.z_angle_stride, a.z_pair_stride, a.QA, a.QB, a.wa, a.wb,
                     a.sh, a.sw, a.ph, a.tw, a.mi, a.mi_angle_stride, a.save,
                     a.save_angle_stride);
  return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_sr_p(const SoftRowsArgs<T>& a, hipStream_t st) {
  SoftRowsConfig c;
  if (!soft_rows_config(sizeof(T), P, a.QB, &c)) return hipErrorInvalidValue;
  if (c.bpw == 4) {
    if (c.ntmax <= 256) return launch_sr_cfg<T, P, 4, 256>(a, c.nteams, c.lds, st);
    if (c.ntmax <= 512) return launch_sr_cfg<T, P, 4, 512>(a, c.nteams, c.lds, st);
    return launch_sr_cfg<T, P, 4, 1024>(a, c.nteams, c.lds, st);
  }
  if (c.ntmax <= 256) return launch_sr_cfg<T, P, 8, 256>(a, c.nteams, c.lds, st);
  if (c.ntmax <= 512) return launch_sr_cfg<T, P, 8, 512>(a, c.nteams, c.lds, st);
  return launch_sr_cfg<T, P, 8, 1024>(a, c.nteams, c.lds, st);
}

// teams of a row-pass workgroup without an LDS table: up to 4, within 64 KiB
template <typename T, int P>
static int row_teams() {
  const size_t per_team = (size_t)lds_elems(P) * sizeof(C2<T>);
  int nteams = 4;
  while (nteams > 1 && per_team * nteams > 64 * 1024) --nteams;
  return nteams;
}

template <typename T, int P>
static hipError_t launch_sgr_p(const SoftGradRowsArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = team_for(P);
  const int nteams = row_teams<T, P>();
  const size_t shm = (size_t)nteams * lds_elems(P) * sizeof(C2<T>);
  auto fn = k_soft_grad_rows<T, P, TEAM>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(a.sh), dim3(nteams * TEAM), shm, st, a.Z,
                     a.z_pair_stride, a.QA, a.QB, a.wa, a.wb, a.sh, a.sw, a.ph,
                     a.tw, a.grad_mi, a.save, a.ZG);
  return hipGetLastError();
}

template <typename T, int P, int SIDE>
static hipError_t launch_sgc_side(const SoftGradColsArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = col_team_for<T>(P);
  constexpr int TW = tile_width<T>();
  const size_t shm = (size_t)TW * lds_elems(P) * sizeof(C2<T>);
  auto fn = k_soft_grad_cols<T, P, TEAM, SIDE>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  const int nch = SIDE == 0 ? a.QA : a.QB;
  hipLaunchKernelGGL(fn, dim3(a.tiles, nch), dim3(TW * TEAM), shm, st, a.GH,
                     a.FO, a.f_label_stride, a.QA, a.QB, a.H, a.GX,
                     a.gx_label_stride, a.tw);
  return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_sgc_p(const SoftGradColsArgs<T>& a, hipStream_t st) {
  return a.side == 0 ? launch_sgc_side<T, P, 0>(a, st) : launch_sgc_side<T, P, 1>(a, st);
}

template <typename T, int P>
static hipError_t launch_sgo_p(const SoftGradOutArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = team_for(P);
  const int nteams = row_teams<T, P>();
  const size_t shm = (size_t)nteams * lds_elems(P) * sizeof(C2<T>);
  auto fn = k_soft_grad_out<T, P, TEAM>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(a.H), dim3(nteams * TEAM), shm, st, a.GX,
                     a.gx_label_stride, a.Q, a.H, a.W, a.ph, a.msk, a.tw, a.grad);
  return hipGetLastError();
}

// The build compiles this file once per precision (CMIF_SOFT_T = float or
// double) so that the two halves compile in parallel.
#ifndef CMIF_SOFT_T
#define CMIF_SOFT_T float
#endif

#define CMIF_SOFT_DISPATCH(NAME, IMPL, ARGS)                        \
  template <typename T>                                             \
  hipError_t NAME(int P, const ARGS<T>& a, hipStream_t st) {        \
    switch (P) {                                                    \
      case 128: return IMPL<T, 128>(a, st);                         \
      case 256: return IMPL<T, 256>(a, st);                         \
      case 512: return IMPL<T, 512>(a, st);                         \
      case 768: return IMPL<T, 768>(a, st);                         \
      case 1024: return IMPL<T, 1024>(a, st);                       \
      case 1536: return IMPL<T, 1536>(a, st);                       \
      case 2048: return IMPL<T, 2048>(a, st);                       \
    }                                                               \
    return hipErrorInvalidValue;                                    \
  }                                                                 \
  template hipError_t NAME<CMIF_SOFT_T>(int, const ARGS<CMIF_SOFT_T>&, hipStream_t);

CMIF_SOFT_DISPATCH(launch_soft_rows, launch_sr_p, SoftRowsArgs)
CMIF_SOFT_DISPATCH(launch_soft_grad_rows, launch_sgr_p, SoftGradRowsArgs)
CMIF_SOFT_DISPATCH(launch_soft_grad_cols, launch_sgc_p, SoftGradColsArgs)
CMIF_SOFT_DISPATCH(launch_soft_grad_out, launch_sgo_p, SoftGradOutArgs)
#undef CMIF_SOFT_DISPATCH

}  // namespace cmif
