// Kernels of the 3-D (volume) CMIF: the method of Sec. 3 with the
// correlations of Eq. 7 over three axes, which the paper's discussion
// states carries over to nD.  Volumes are transformed slice by slice in 2-D
// (the forward row and column kernels, one batch entry per slice), then
// along depth here; each pair's product is transformed back along depth
// here, and every depth displacement's 2-D spectra then go through the
// pair column and row passes of the 2-D path.
//
// Layouts (complex<T>; pos = c * P_h + k_y indexes the 2-D half spectrum,
// npos = (P_w / 2) P_h positions, TW = 64 B / sizeof(complex<T>)):
//   F2 [z][label][pos]     2-D spectra of the slices (forward column kernel)
//   F3 [label][k_z][pos]   3-D spectra
//   G  [dz][pair][pos]     per depth displacement (map slice), the 2-D
//                          spectrum of every pair's correlation
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"
#include "rows_common.h"

namespace cmif {

// Lanes per depth transform: PD / 2 up to 128 points (two points per lane,
// sub-wave teams), 64 above.
constexpr int zteam(int pd) { return pd <= 128 ? pd / 2 : 64; }

// Depth transform of one label's slice spectra: workgroup = TW consecutive
// positions x one label; the [D][TW] tile is read row by row (64-byte
// segments), each team transforms one position's depth column (zero-padded
// from D to PD) and the [PD][TW] result leaves row by row.
template <typename T, int PD>
__global__ void __launch_bounds__(tile_width<T>() * zteam(PD))
k_zfft(const C2<T>* __restrict__ F2, long long z_stride, long long label_stride2,
       int D, int npos, C2<T>* __restrict__ F3, const C2<T>* __restrict__ tw) {
  constexpr int TEAM = zteam(PD);
  constexpr int R = PD / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* tile = reinterpret_cast<C2<T>*>(smem_raw);  // [PD][TW]
  C2<T>* exch = tile + PD * TW;
  const int pos0 = blockIdx.x * TW, lbl = blockIdx.y;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const C2<T>* src = F2 + lbl * label_stride2 + pos0;
  for (int e = threadIdx.x; e < D * TW; e += blockDim.x) {
    const int z = e / TW, p = e % TW;
    tile[e] = src[z * z_stride + p];
  }
  __syncthreads();
  FftTw<T, PD, TEAM> ftw;
  fft_load_twiddles<T, PD, TEAM>(ftw, tw, lane);
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int z = lane + TEAM * q;
    v[q] = z < D ? tile[z * TW + team] : mk<T>((T)0, (T)0);
  }
  team_fft<T, PD, TEAM, -1>(v, exch + team * lds_elems(PD), ftw, lane);
  __syncthreads();  // every team has read its column of the tile
#pragma unroll
  for (int q = 0; q < R; ++q) tile[(lane + TEAM * q) * TW + team] = v[q];
  __syncthreads();
  C2<T>* dst = F3 + (long long)lbl * PD * npos + pos0;
  for (int e = threadIdx.x; e < PD * TW; e += blockDim.x) {
    const int kz = e / TW, p = e % TW;
    dst[(long long)kz * npos + p] = tile[e];
  }
}

// Per pair (a, b) and TW positions: conj(F3_a) F3_b along k_z, inverse
// depth transform (scaled by 1/PD), and the depth lags that carry a
// displacement (dz in [-(DA-1), DB-1]) written to G[dz map index][pair].
// Positions of column 0 hold the packed k_x = 0 and k_x = P_w/2 planes,
// each Hermitian in (k_z, k_y) together: they are separated with the mirror
// (-k_z, -k_y), multiplied, and packed again, as the 2-D pair kernel does
// along k_y alone.
template <typename T, int PD>
__global__ void __launch_bounds__(tile_width<T>() * zteam(PD))
k_zpair(const C2<T>* __restrict__ F3A, const C2<T>* __restrict__ F3B, int QB,
        int npos, int ph, int DA, int DB, int npairs, C2<T>* __restrict__ G,
        const C2<T>* __restrict__ tw) {
  constexpr int TEAM = zteam(PD);
  constexpr int R = PD / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* ta = reinterpret_cast<C2<T>*>(smem_raw);  // [PD][TW]
  C2<T>* tb = ta + PD * TW;
  C2<T>* exch = tb + PD * TW;
  const int pos0 = blockIdx.x * TW, pair = blockIdx.y;
  const int a = pair / QB, b = pair % QB;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const C2<T>* fa = F3A + (long long)a * PD * npos;
  const C2<T>* fb = F3B + (long long)b * PD * npos;
  for (int e = threadIdx.x; e < PD * TW; e += blockDim.x) {
    const int kz = e / TW, p = e % TW;
    ta[e] = fa[(long long)kz * npos + pos0 + p];
    tb[e] = fb[(long long)kz * npos + pos0 + p];
  }
  __syncthreads();
  FftTw<T, PD, TEAM> ftw;
  fft_load_twiddles<T, PD, TEAM>(ftw, tw, lane);
  const int pos = pos0 + team;
  C2<T> v[R];
  if (pos >= ph) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int kz = lane + TEAM * q;
      v[q] = cmulc<T>(ta[kz * TW + team], tb[kz * TW + team]);
    }
  } else {
    // column 0: k_y = pos, mirror (-k_z, -k_y)
    const int kym = pos == 0 ? 0 : ph - pos;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int kz = lane + TEAM * q;
      const int kzm = kz == 0 ? 0 : PD - kz;
      C2<T> ga0, ga1, gb0, gb1;
      unpack0<T>(ta[kz * TW + team], fa[(long long)kzm * npos + kym], ga0, ga1);
      unpack0<T>(tb[kz * TW + team], fb[(long long)kzm * npos + kym], gb0, gb1);
      const C2<T> y0 = cmulc<T>(ga0, gb0);
      const C2<T> y1 = cmulc<T>(ga1, gb1);
      v[q] = mk<T>(y0.x - y1.y, y0.y + y1.x);  // y0 + i y1
    }
  }
  team_fft<T, PD, TEAM, +1>(v, exch + team * lds_elems(PD), ftw, lane);
  const T inv = (T)1 / (T)PD;
  __syncthreads();  // every team is done with the tiles
#pragma unroll
  for (int q = 0; q < R; ++q) ta[(lane + TEAM * q) * TW + team] = cscale<T>(v[q], inv);
  __syncthreads();
  for (int e = threadIdx.x; e < PD * TW; e += blockDim.x) {
    const int kz = e / TW, p = e % TW;
    const int k = circ_to_map(kz, PD, DA, DB);
    if (k >= 0) G[((long long)k * npairs + pair) * npos + pos0 + p] = ta[e];
  }
}

// Flagged label pairs of one map slice (residual >= 0.25 in the FP32 row
// pass) are not recomputed for volumes: they count as unresolved.
__global__ void k_count_flags(const uint32_t* __restrict__ flags, int n,
                              cmif_stats* __restrict__ stats) {
  uint32_t c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += flags[i] != 0u ? 1u : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x % 64) == 0 && c) atomicAdd(&stats->unresolved_pairs, c);
}

// The Alg. 1 result over the flattened (dz, dy) x dx map (dy field = the
// flattened row) as a 3-D displacement.
__global__ void k_best3d(const cmif_best* __restrict__ b2, cmif_best3d* __restrict__ out,
                         int sh, int da, int ha) {
  if (threadIdx.x != 0) return;
  const cmif_best b = *b2;
  cmif_best3d r{};
  if (b.angle_index >= 0) {
    r.dz = b.dy / sh - (da - 1);
    r.dy = b.dy % sh - (ha - 1);
    r.dx = b.dx;
  }
  r.mi = b.mi;
  r.n = b.n;
  *out = r;
}

template <typename T, int PD>
static hipError_t launch_zfft_p(const ZfftArgs<T>& a, hipStream_t st) {
  constexpr int TW = tile_width<T>();
  const size_t shm = ((size_t)PD * TW + (size_t)TW * lds_elems(PD)) * sizeof(C2<T>);
  auto fn = k_zfft<T, PD>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(a.npos / TW, a.Q), dim3(TW * zteam(PD)), shm, st, a.F2,
                     a.z_stride, a.label_stride2, a.D, a.npos, a.F3, a.tw);
  return hipGetLastError();
}

template <typename T, int PD>
static hipError_t launch_zpair_p(const ZpairArgs<T>& a, hipStream_t st) {
  constexpr int TW = tile_width<T>();
  const size_t shm = ((size_t)2 * PD * TW + (size_t)TW * lds_elems(PD)) * sizeof(C2<T>);
  auto fn = k_zpair<T, PD>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(a.npos / TW, a.QA * a.QB), dim3(TW * zteam(PD)), shm, st,
                     a.F3A, a.F3B, a.QB, a.npos, a.ph, a.DA, a.DB, a.QA * a.QB, a.G,
                     a.tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zfft(int PD, const ZfftArgs<T>& a, hipStream_t st) {
  if (a.npos % tile_width<T>() != 0) return hipErrorInvalidValue;
  switch (PD) {
    case 32: return launch_zfft_p<T, 32>(a, st);
    case 64: return launch_zfft_p<T, 64>(a, st);
    case 128: return launch_zfft_p<T, 128>(a, st);
    case 256: return launch_zfft_p<T, 256>(a, st);
    case 512: return launch_zfft_p<T, 512>(a, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_zpair(int PD, const ZpairArgs<T>& a, hipStream_t st) {
  if (a.npos % tile_width<T>() != 0) return hipErrorInvalidValue;
  switch (PD) {
    case 32: return launch_zpair_p<T, 32>(a, st);
    case 64: return launch_zpair_p<T, 64>(a, st);
    case 128: return launch_zpair_p<T, 128>(a, st);
    case 256: return launch_zpair_p<T, 256>(a, st);
    case 512: return launch_zpair_p<T, 512>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_count_flags(const uint32_t* flags, int n, cmif_stats* stats,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_count_flags, dim3(1), dim3(256), 0, st, flags, n, stats);
  return hipGetLastError();
}

hipError_t launch_best3d(const cmif_best* b2, cmif_best3d* out, int sh, int da,
                         int ha, hipStream_t st) {
  hipLaunchKernelGGL(k_best3d, dim3(1), dim3(64), 0, st, b2, out, sh, da, ha);
  return hipGetLastError();
}

template hipError_t launch_zfft<float>(int, const ZfftArgs<float>&, hipStream_t);
template hipError_t launch_zfft<double>(int, const ZfftArgs<double>&, hipStream_t);
template hipError_t launch_zpair<float>(int, const ZpairArgs<float>&, hipStream_t);
template hipError_t launch_zpair<double>(int, const ZpairArgs<double>&, hipStream_t);

}  // namespace cmif
