// Device helpers shared by the pair and row passes: separation of the
// packed column 0, loads of two stored half-spectrum rows and their
// Hermitian extension into one packed complex sequence.
#pragma once

#include "fft_core.h"
#include "internal.h"

namespace cmif {

// Separate the packed column 0: W = G0 + i G1 with G0, G1 Hermitian in k.
template <typename T>
__device__ __forceinline__ void unpack0(C2<T> w, C2<T> wm, C2<T>& g0, C2<T>& g1) {
  // g0 = (w + conj(wm)) / 2,  g1 = (w - conj(wm)) / (2i)
  g0 = mk<T>((w.x + wm.x) * (T)0.5, (w.y - wm.y) * (T)0.5);
  g1 = mk<T>((w.y + wm.y) * (T)0.5, (wm.x - w.x) * (T)0.5);
}

template <typename T>
__device__ __forceinline__ T round_half_even(T v);
template <>
__device__ __forceinline__ float round_half_even<float>(float v) { return rintf(v); }
template <>
__device__ __forceinline__ double round_half_even<double>(double v) { return rint(v); }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sequence index held by (lane, q) on input to a row transform: lane +
// TEAM q, or (SPLIT: two-wave decimation-in-time transform, TEAM = 128) the
// even samples in wave 0 and the odd ones in wave 1.
template <int TEAM, bool SPLIT>
__device__ __forceinline__ int row_in_pos(int lane, int q) {
  if constexpr (SPLIT) return 2 * ((lane & 63) + 64 * q) + (lane >> 6);
  else return lane + TEAM * q;
}

// Output index held by (lane, q) after the row transform.
template <int P, int TEAM, bool SPLIT>
__device__ __forceinline__ int row_out_pos(int lane, int q) {
  if constexpr (SPLIT) return (lane >> 6) * (P / 2) + (lane & 63) + 64 * q;
  else return lane + TEAM * q;
}

// Both input layouts (lane + TEAM q, and the split one) are q-major: the
// positions k < P/2 are exactly those with q < R/2, k = 0 can only occur at
// q = 0 and k = P/2 only at q = R/2.  The helpers below branch on q (a
// compile-time constant after unrolling) and select per lane only at those
// two positions, so no lane-divergent branch is left.

// Raw loads of row i of pairs p0 (and p1 when has1): element k of the half
// spectrum that sequence index k (row_in_pos) needs (its mirror P - k in the
// upper half; slot 0 for k = 0 and k = P/2).
template <typename T, int P, int TEAM, bool SPLIT = false>
__device__ __forceinline__ void load_raw(const C2<T>* __restrict__ z0,
                                         const C2<T>* __restrict__ z1,
                                         bool has1, int tile_stride, int lane,
                                         C2<T> (&u0)[P / TEAM],
                                         C2<T> (&u1)[P / TEAM]) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  constexpr int HALF = P / 2;
  static_assert(R % 2 == 0, "two halves of positions per lane");
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = row_in_pos<TEAM, SPLIT>(lane, q);
    int e = q < R / 2 ? k : P - k;              // k <= P/2 - 1, or its mirror
    if (q == R / 2) e = e == HALF ? 0 : e;      // k = P/2 sits in slot 0
    const int off = (e / TW) * tile_stride + (e % TW);
    u0[q] = z0[off];
    u1[q] = has1 ? z1[off] : mk<T>((T)0, (T)0);
  }
}

// Packed complex sequence W(k) = Z_p0(k) + i Z_p1(k) from the raw loads
// (Hermitian extension of both half spectra).
template <typename T, int P, int TEAM, bool SPLIT = false>
__device__ __forceinline__ void build_pack(const C2<T> (&u0)[P / TEAM],
                                           const C2<T> (&u1)[P / TEAM], int lane,
                                           C2<T> (&w)[P / TEAM]) {
  constexpr int R = P / TEAM;
  constexpr int HALF = P / 2;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (q < R / 2) {
      // u0 + i u1 (k = 0: the real k_x = 0 values packed in slot 0)
      C2<T> g = mk<T>(u0[q].x - u1[q].y, u0[q].y + u1[q].x);
      if (q == 0 && row_in_pos<TEAM, SPLIT>(lane, q) == 0) g = mk<T>(u0[q].x, u1[q].x);
      w[q] = g;
    } else {
      // conj(u0) + i conj(u1) (k = P/2: the k_x = P/2 values of slot 0)
      C2<T> g = mk<T>(u0[q].x + u1[q].y, u1[q].x - u0[q].y);
      if (q == R / 2 && row_in_pos<TEAM, SPLIT>(lane, q) == HALF)
        g = mk<T>(u0[q].y, u1[q].y);
      w[q] = g;
    }
  }
}

template <typename T, int P, int TEAM>
__device__ __forceinline__ void load_pack(const C2<T>* __restrict__ z0,
                                          const C2<T>* __restrict__ z1,
                                          bool has1, int tile_stride, int lane,
                                          C2<T> (&w)[P / TEAM]) {
  C2<T> u0[P / TEAM], u1[P / TEAM];
  load_raw<T, P, TEAM>(z0, z1, has1, tile_stride, lane, u0, u1);
  build_pack<T, P, TEAM>(u0, u1, lane, w);
}

}  // namespace cmif
