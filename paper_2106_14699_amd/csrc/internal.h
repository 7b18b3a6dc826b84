// Internal definitions shared by the kernels and the host scheduler of
// libcmif.  Not part of the public ABI.
//
// HBM layouts (per image pair; complex<T> = float2 or double2):
//   row spectra  X[label][tile][y][TW]      tile = k_x / TW, y in [0, H)
//   2D spectra   F[label][c][k_y]           c in [0, P_w/2), k_y in [0, P_h)
//   pair columns Z: pair p = a*Q_B+b, tile, map row i in [0, S_h), with
//                pairs stored two by two (see z_pair_offset)
// where TW = 64 B / sizeof(complex<T>) (8 for FP32, 4 for FP64), so one
// (tile, row) record is one 64-byte segment.  Column c = 0 holds the two
// real-input special frequencies packed as one complex value: the k_x = 0
// and k_x = P_w/2 row values are real for real input, so slot 0 stores
// X(y, 0) + i X(y, P_w/2); the column transform of that packed column yields
// G0(k_y) + i G1(k_y) with both G0 and G1 Hermitian, which the pair kernel
// separates again.
#pragma once

#include <stdint.h>

#include "../../include/cmif.h"

namespace cmif {

constexpr int kMaxBatch = 16;  // angles per pipeline pass (kernel argument)
constexpr int kMinP = 128;
constexpr int kXlogN = 2048;   // c log2 c tabulated for integer c < kXlogN
constexpr int kMaxP = 4096;
// Row pass: labels of A whose exact marginals C_a are folded into S_A and N
// together (one workgroup barrier per group)
constexpr int kFoldA = 2;
// Row pass: workgroups per map row.  At 4096 points the per-position state
// of one row (C_b of every label of B for 4096 lags) does not fit one
// workgroup's registers, so two workgroups each transform the whole row and
// keep the state of one half of the lags.
__host__ __device__ constexpr int lag_parts(int p) { return p >= 4096 ? 2 : 1; }
// FFT lengths with compiled kernels, ascending (the plan takes the smallest
// one that reaches the alias-free size).  4096 points: FP32-rounded HARD
// plans of the fused schedule only (their FP64 re-run included).
constexpr int kFftSizes[] = {128, 256, 512, 768, 1024, 1536, 2048, 4096};
constexpr int kMaxSoftP = 2048;  // SOFT, FP64-precision and plain plans

struct RotArgs {
  int32_t c[kMaxBatch];  // round(cos(theta) * 2^16)
  int32_t s[kMaxBatch];  // round(sin(theta) * 2^16)
};

// Argmax partial for one (angle, row block): best eligible MI and its flat
// map index, -1 when the block had no eligible entry.
struct ArgPartial {
  double mi;
  int64_t idx;
  int64_t n;
};

template <typename T>
constexpr int tile_width() { return 64 / (2 * (int)sizeof(T)); }

// Z layout (FP32 up to P = 1024): pairs are stored two by two, interleaved
// per (tile, map row): the 64-byte segment (tile t, row i) of pair p sits at
//   (p / 2) * 2 * pair_elems + t * 2 S_h TW + i * 2 TW + (p % 2) * TW
// (pair_elems = (P_w / 2) S_h elements), so one 128-byte line holds row i
// of both pairs that a row transform packs together.  Elsewhere (FP64, and
// FP32 at 2048 points, where the column kernel writes a tile as 32-byte
// pieces and the interleave measured slower) one pair after the other:
//   p * pair_elems + t * S_h TW + i * TW.
// Z buffers and per-angle strides hold an even number of pair slots
// (z_pair_slots).  The row kernels that read Z decide the layout by their
// length P_w (z_group, a compile-time constant there); the column kernel,
// whose length P_h may be another, writes the layout it is given at run time
// (the _rt forms, group z_group_rt(P_w)).
template <typename T>
__host__ __device__ constexpr int z_group_rt(int ph) {
  return sizeof(T) == 4 && ph <= 1024 ? 2 : 1;
}
template <typename T>
__host__ __device__ constexpr long long z_row_offset_rt(int i, int zg) {
  return (long long)i * zg * tile_width<T>();
}
template <typename T>
__host__ __device__ constexpr long long z_pair_offset_rt(int p, long long pair_elems, int zg) {
  // zg = 2: (p / 2) * 2 * pair_elems + (p % 2) * TW; zg = 1: p * pair_elems
  return (long long)(p >> (zg - 1)) * zg * pair_elems +
         (long long)(p & (zg - 1)) * tile_width<T>();
}
template <typename T>
__host__ __device__ constexpr int z_tile_stride_rt(int sh, int zg) {
  return sh * zg * tile_width<T>();
}
template <typename T, int P>
__host__ __device__ constexpr int z_group() {
  return z_group_rt<T>(P);
}
template <typename T, int P>
__host__ __device__ constexpr long long z_row_offset(int i) {
  return (long long)i * z_group<T, P>() * tile_width<T>();
}
template <typename T, int P>
__host__ __device__ constexpr long long z_pair_offset(int p, long long pair_elems) {
  return z_group<T, P>() == 2
             ? (long long)(p >> 1) * 2 * pair_elems + (long long)(p & 1) * tile_width<T>()
             : (long long)p * pair_elems;
}
template <typename T, int P>
__host__ __device__ constexpr int z_tile_stride(int sh) {
  return sh * z_group<T, P>() * tile_width<T>();
}
__host__ __device__ constexpr int z_pair_slots(int n) { return (n + 1) & ~1; }

// FFT lengths: 2^k or 3 * 2^k (radix-3 through the 12-point butterfly).
constexpr bool is_pow2(int p) { return (p & (p - 1)) == 0; }

// Lanes per FFT team: at most 8 points per lane (radix-8 stages), so a
// 1024-point transform is spread over two waves and 2048 over four; 3 * 2^k
// lengths take 12 points per lane (a 12-point first stage), so 768 points
// fill one wave and 1536 two.
constexpr int team_for(int p) {
  return is_pow2(p) ? (p <= 512 ? 64 : p / 8) : p / 12;
}

// Team size of the column kernels, whose workgroup holds one team per column
// of a TW-wide tile: capped so that TW teams fit in 1024 lanes.
template <typename T>
constexpr int col_team_for(int p) {
  return team_for(p) * tile_width<T>() <= 1024 ? team_for(p)
                                               : 1024 / tile_width<T>();
}

// Team size of the pair column kernel: one wave per column up to P = 1024
// (16 points per lane: radix 16, 16, 4 with two LDS exchanges and wave-level
// barriers only), P/16 lanes above, capped so that TW teams fit 1024 lanes.
// At 4096 points the column kernels run fewer columns than a tile per
// workgroup, and the teams keep 16 FP32 points per lane (256 lanes) or 8
// FP64 points (512 lanes: 16 double points with the operand registers of
// the pair kernel do not fit).
template <typename T>
constexpr int pair_col_team_raw(int p) {
  return is_pow2(p) ? (p <= 1024 ? 64 : p / 16) : p / 12;
}
template <typename T>
constexpr int pair_col_team(int p) {
  return p >= 4096 ? (sizeof(T) == 4 ? p / 16 : p / 8)
         : pair_col_team_raw<T>(p) * tile_width<T>() <= 1024
             ? pair_col_team_raw<T>(p)
             : 1024 / tile_width<T>();
}

// Column swizzle of a [rows][TW] LDS staging tile: element (row, col) lives
// at row*TW + (col ^ stage_swz(row)).  The swizzle is a multiple of
// 16 B / sizeof(element) so 16-byte vectors of a row stay contiguous, and
// writing one column for consecutive rows spreads over the banks (at most
// 2-way conflicts instead of TW-way).
template <int TW>
__host__ __device__ constexpr int stage_swz(int row) {
  return TW == 8 ? ((row >> 1) & 3) << 1 : (row >> 1) & (TW - 1);
}

// Map row (or column) of circular correlation lag y (P periodic) in a
// displacement window chi in [1 - e_a, e_b - 1]; -1 if lag y carries no
// displacement of the window.  e_a, e_b are the window's extents on either
// side of zero: the image sides h_a, h_b for the full set, 1 - y0 and
// y1 + 1 for a window [y0, y1] (either may be <= 0 when the window does not
// contain 0).  With P alias-free for the window, lag y holds chi = y for
// y <= e_b - 1 and chi = y - P otherwise.
__host__ __device__ inline int circ_to_map(int y, int p, int e_a, int e_b) {
  const int chi = y <= e_b - 1 ? y : y - p;
  return chi >= 1 - e_a && chi <= e_b - 1 ? chi + e_a - 1 : -1;
}

}  // namespace cmif
