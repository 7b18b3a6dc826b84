// Pair column pass: conjugate spectral products and the inverse transform
// along y for every label pair (Sec. 3.2, Eq. 9; Eq. 7 in the frequency
// domain: sum_x f(x) g(x + k) has spectrum conj(F) G).
//
// One workgroup per (tile of TW spectrum columns, label a of A, angle); each
// team owns one column c and keeps conj(F_A,a(:, c)) in registers while it
// loops over all labels b of B: product, inverse FFT along y (length P_h),
// then the TW columns are transposed through LDS so that every map row i of
// the tile leaves as one 64-byte segment of Z[a*Q_B+b][tile][i][TW].  Rows
// of the circular correlation that map to no displacement are not stored.
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"
#include "rows_common.h"

namespace cmif {

// Columns per workgroup (one team each), by default: the whole TW-wide
// tile, or part of it where TW teams would exceed 512 lanes (FP32) or 256
// lanes (FP64) — at 1024 lanes the launch bound leaves 128 registers per
// lane and the 2048-point kernel spilled.  A part writes its columns of
// every 64-byte row segment as 32-byte (or smaller) pieces.  At 4096 points
// 512 lanes' worth of columns (two FP32 columns, one FP64 column).  The
// launch-shape tuner may also take half of the default.
template <typename T, int P>
constexpr int pair_cols_cpw() {
  constexpr int cap = sizeof(T) == 4 ? 512 : 256;
  constexpr int team = pair_col_team<T>(P);
  if constexpr (P >= 4096) return 512 / team >= 1 ? 512 / team : 1;
  return tile_width<T>() * team <= cap ? tile_width<T>()
                                       : (cap / team >= 2 ? cap / team : 2);
}

// LDS of the column kernel: the teams' exchange buffers (re-used as the
// staging tile) and, when it fits, the twiddle table (otherwise every lane
// keeps its twiddles in registers).
template <typename T, int P, int CPW>
constexpr size_t pair_cols_exch_bytes() {
  return (size_t)CPW * lds_elems(P) * sizeof(C2<T>);
}
template <typename T, int P, int CPW>
constexpr size_t pair_cols_stage_bytes() {
  return (size_t)P * CPW * sizeof(C2<T>);
}
// A staging tile of its own (instead of the exchange buffers) when it fits:
// one barrier less per label b, and the copy-out of b overlaps the next FFT.
template <typename T, int P, int CPW>
constexpr bool pair_cols_sep_staging() {
  return pair_cols_exch_bytes<T, P, CPW>() + pair_cols_stage_bytes<T, P, CPW>() +
             (size_t)P * sizeof(C2<T>) <= 160 * 1024;
}
template <typename T, int P, int CPW>
constexpr size_t pair_cols_table_offset() {
  return pair_cols_exch_bytes<T, P, CPW>() +
         (pair_cols_sep_staging<T, P, CPW>() ? pair_cols_stage_bytes<T, P, CPW>() : 0);
}
template <typename T, int P, int CPW>
constexpr bool pair_cols_lds_twiddles() {
  return pair_cols_table_offset<T, P, CPW>() + (size_t)P * sizeof(C2<T>) <= 160 * 1024;
}

// Streaming 16-byte store: Z is written once here and read once by the row
// pass after the whole column pass, so its lines need not stay in the
// caches (non-temporal; measured 67.2 -> 57.7 ms per sweep for this pass).
__device__ __forceinline__ void store_stream16(float4* dst, float4 v) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v w;
  w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
  __builtin_nontemporal_store(w, reinterpret_cast<f4v*>(dst));
}

// Column swizzle of the [rows][CPW] staging tile: a multiple of the 16-byte
// vector's EV elements (vectors of a row stay whole), varying with the row
// so that one column written for consecutive rows spreads over the banks.
template <int CPW, int EV>
__device__ __forceinline__ int pc_swz(int row) {
  return CPW / EV > 1 ? ((row >> 1) & (CPW / EV - 1)) * EV : 0;
}

// Staging + store of one pair's CPW columns (columns part*CPW .. of the
// tile): rows i leave as 16-byte vectors into Z[pair][tile][i][TW] (layout
// group zg of the row kernels that read it).
template <typename T, int P, int TEAM, int CPW>
__device__ __forceinline__ void pair_cols_store(C2<T> (&v)[P / TEAM], C2<T>* smem,
                                                C2<T>* __restrict__ zp, int ha,
                                                int hb, int sh, int team,
                                                int part, int lane, int zg) {
  constexpr int R = P / TEAM;
  constexpr int EV = 16 / (int)sizeof(C2<T>);
  constexpr bool SEP = pair_cols_sep_staging<T, P, CPW>();
  C2<T>* stage = SEP ? reinterpret_cast<C2<T>*>(reinterpret_cast<unsigned char*>(smem) +
                                                 pair_cols_exch_bytes<T, P, CPW>())
                     : smem;
  // separate tile: the previous copy-out has finished reading it; aliased
  // tile: every team is done with its exchange buffer
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = circ_to_map(lane + TEAM * q, P, ha, hb);
    if (i >= 0) stage[i * CPW + (team ^ pc_swz<CPW, EV>(i))] = v[q];
  }
  __syncthreads();
  float4* z4 = reinterpret_cast<float4*>(zp);
  for (int e = threadIdx.x; e < sh * CPW / EV; e += blockDim.x) {
    const int i = (e * EV) / CPW, col = (e * EV) % CPW;
    store_stream16(z4 + (z_row_offset_rt<T>(i, zg) + part * CPW + col) / EV,
                   *reinterpret_cast<const float4*>(
                       &stage[i * CPW + (col ^ pc_swz<CPW, EV>(i))]));
  }
  if constexpr (!SEP) __syncthreads();  // the exchange buffers are reused next
}

// Runs labels b in [b_begin, b_end) of B against labels a0 .. a0 + BA - 1
// of A (those below QA; pair blocking: each F_B column read serves BA
// products); the output slot of (a, b) is a * QB + b, or zpair0 for the one
// pair of an item (BA = 1).  The b loop starts at b_begin + rot and wraps
// (every pair is computed on its own, so the order changes no result).
template <typename T, int P, int TEAM, int CPW, int BA, class TWS>
__device__ __forceinline__ void pair_cols_run(
    const C2<T>* __restrict__ fa_col, long long fa_label_stride, int a0, int QA,
    int QB, const C2<T>* __restrict__ fb_base, long long fb_label_stride,
    int b_begin, int b_end, int rot, int zpair0, int ha, int hb, int sh,
    C2<T>* __restrict__ z_base, long long z_pair_stride, const TWS& ftw,
    C2<T>* smem, int c, int team, int part, int lane, int zg) {
  constexpr int R = P / TEAM;
  C2<T>* lds = smem + team * lds_elems(P);
  auto slot = [&](int ab, int b) {
    return zpair0 >= 0 ? zpair0 : (a0 + ab) * QB + b;
  };
  const int nbl = b_end - b_begin;
  auto b_at = [&](int k) {  // k-th label of the rotated order
    const int j = k + rot;
    return b_begin + (j >= nbl ? j - nbl : j);
  };
  if (fa_col == nullptr) {
    // the B operand already holds the product spectra of every pair,
    // [pair][c][k_y] (plain schedule, volumes)
    for (int b = b_begin; b < b_end; ++b) {
      const C2<T>* fb_col = fb_base + (long long)(a0 * QB + b) * fb_label_stride;
      C2<T> v[R];
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = fb_col[lane + TEAM * q];
      team_fft<T, P, TEAM, +1>(v, lds, ftw, lane);
      pair_cols_store<T, P, TEAM, CPW>(
          v, smem, z_base + z_pair_offset_rt<T>(slot(0, b), z_pair_stride, zg), ha, hb,
          sh, team, part, lane, zg);
    }
    return;
  }
  C2<T> fa[BA][R];
#pragma unroll
  for (int ab = 0; ab < BA; ++ab) {
    const C2<T>* col = fa_col + (a0 + ab < QA ? ab : 0) * fa_label_stride;
#pragma unroll
    for (int q = 0; q < R; ++q) fa[ab][q] = col[lane + TEAM * q];
  }
  if (c != 0) {
    // software pipeline: the next b's column is in flight during this FFT
    C2<T> fbn[R];
    {
      const C2<T>* fb0 = fb_base + b_at(0) * fb_label_stride;
#pragma unroll
      for (int q = 0; q < R; ++q) fbn[q] = fb0[lane + TEAM * q];
    }
    for (int k = 0; k < nbl; ++k) {
      const int b = b_at(k);
      C2<T> fb[R];
#pragma unroll
      for (int q = 0; q < R; ++q) fb[q] = fbn[q];
      if (k + 1 < nbl) {
        const C2<T>* fb_next = fb_base + b_at(k + 1) * fb_label_stride;
#pragma unroll
        for (int q = 0; q < R; ++q) fbn[q] = fb_next[lane + TEAM * q];
      }
#pragma unroll
      for (int ab = 0; ab < BA; ++ab) {
        if (a0 + ab >= QA) break;
        C2<T> v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = cmulc<T>(fa[ab][q], fb[q]);
        team_fft<T, P, TEAM, +1>(v, lds, ftw, lane);
        pair_cols_store<T, P, TEAM, CPW>(
            v, smem, z_base + z_pair_offset_rt<T>(slot(ab, b), z_pair_stride, zg), ha,
            hb, sh, team, part, lane, zg);
      }
    }
  } else {
    // slot 0 packs the k_x = 0 and k_x = P_w/2 columns (both Hermitian)
    for (int k = 0; k < nbl; ++k) {
      const int b = b_at(k);
      const C2<T>* fb_col = fb_base + b * fb_label_stride;
#pragma unroll
      for (int ab = 0; ab < BA; ++ab) {
        if (a0 + ab >= QA) break;
        const C2<T>* fa_c = fa_col + ab * fa_label_stride;
        C2<T> v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int k = lane + TEAM * q;
          const int km = k == 0 ? 0 : P - k;
          C2<T> ga0, ga1, gb0, gb1;
          unpack0<T>(fa[ab][q], fa_c[km], ga0, ga1);
          unpack0<T>(fb_col[k], fb_col[km], gb0, gb1);
          const C2<T> y0 = cmulc<T>(ga0, gb0);     // Hermitian in k
          const C2<T> y1 = cmulc<T>(ga1, gb1);     // Hermitian in k
          v[q] = mk<T>(y0.x - y1.y, y0.y + y1.x);  // y0 + i y1
        }
        team_fft<T, P, TEAM, +1>(v, lds, ftw, lane);
        pair_cols_store<T, P, TEAM, CPW>(
            v, smem, z_base + z_pair_offset_rt<T>(slot(ab, b), z_pair_stride, zg), ha,
            hb, sh, team, part, lane, zg);
      }
    }
  }
}

// CPW columns per workgroup (a tile of TW columns takes TW / CPW of them),
// radix cap MAXR of the column transforms, BA labels of A per workgroup.
template <typename T, int P, int TEAM, int CPW, int MAXR, int BA>
__global__ void __launch_bounds__((CPW * TEAM))
k_pair_cols(const C2<T>* __restrict__ FA, long long fa_label_stride,
            const C2<T>* __restrict__ FB, long long fb_angle_stride,
            long long fb_label_stride, int QA, int QB, int ha, int hb, int sh,
            C2<T>* __restrict__ Z, long long z_angle_stride,
            long long z_pair_stride, const C2<T>* __restrict__ tw,
            const int4* __restrict__ items, const uint32_t* __restrict__ n_items,
            int xcd_groups, int zg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* smem = reinterpret_cast<C2<T>*>(smem_raw);
  constexpr int TW = tile_width<T>();
  constexpr int NPART = TW / CPW;  // workgroups per tile
  int t = blockIdx.x;  // tile part: tile t / NPART, part t % NPART
  int ablk, beta, b_begin, b_end, zpair0, rot = 0;
  C2<T>* z_base;
  if (items == nullptr) {
    // all pairs: workgroup (tile, block of BA labels of A, angle) runs every b
    ablk = blockIdx.y;
    beta = blockIdx.z;
    if (xcd_groups) {
      // consecutive workgroup ids go to consecutive XCDs (8): give each XCD
      // whole (angle, tile) groups, so that the workgroups that read one
      // tile's F_B columns share that XCD's L2
      const int L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      const int s = L >> 3;
      const int grp = (L & 7) + 8 * (s / (int)gridDim.y);
      ablk = s % (int)gridDim.y;
      t = grp % (int)gridDim.x;
      beta = grp / (int)gridDim.x;
    }
    b_begin = 0;
    b_end = QB;
    // XCD-grouped order: the Q_A workgroups of a tile run at the same time
    // on one XCD; each starts its b loop at its own label, so that they read
    // different F_B columns of the tile (all of it stays in that L2) rather
    // than the same lines at once
    rot = xcd_groups ? ablk % QB : 0;
    zpair0 = -1;
    z_base = Z + beta * z_angle_stride + (long long)(t / NPART) * z_tile_stride_rt<T>(sh, zg);
  } else {
    // item list: workgroup (tile, item) runs one pair (angle, a, b) of the
    // list into slot `item` of Z
    const int it = blockIdx.y;
    if ((uint32_t)it >= *n_items) return;
    const int4 e = items[it];
    beta = e.x;
    ablk = e.y;  // BA = 1 in item mode
    b_begin = e.z;
    b_end = e.z + 1;
    zpair0 = it;
    z_base = Z + (long long)(t / NPART) * z_tile_stride_rt<T>(sh, zg);
  }
  const int a0 = ablk * BA;
  static_assert(TEAM % 64 == 0, "teams of whole waves");
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / TEAM);  // wave-uniform
  const int lane = threadIdx.x % TEAM;
  const int part = t % NPART;
  const int c = (t / NPART) * TW + part * CPW + team;
  const C2<T>* fa_col = FA ? FA + a0 * fa_label_stride + (long long)c * P : nullptr;
  const C2<T>* fb_base = FB + beta * fb_angle_stride + (long long)c * P;
  if constexpr (pair_cols_lds_twiddles<T, P, CPW>()) {
    C2<T>* twl = reinterpret_cast<C2<T>*>(reinterpret_cast<unsigned char*>(smem) +
                                          pair_cols_table_offset<T, P, CPW>());
    for (int x = threadIdx.x; x < P; x += blockDim.x) twl[x] = tw[x];
    __syncthreads();
    const FftTwTable<T, P, TEAM, MAXR> ftw{twl};
    pair_cols_run<T, P, TEAM, CPW, BA>(fa_col, fa_label_stride, a0, QA, QB, fb_base,
                                       fb_label_stride, b_begin, b_end, rot, zpair0, ha, hb,
                                       sh, z_base, z_pair_stride, ftw, smem, c, team,
                                       part, lane, zg);
  } else {
    FftTw<T, P, TEAM, MAXR> ftw;
    fft_load_twiddles<T, P, TEAM, 1, MAXR>(ftw, tw, lane);
    pair_cols_run<T, P, TEAM, CPW, BA>(fa_col, fa_label_stride, a0, QA, QB, fb_base,
                                       fb_label_stride, b_begin, b_end, rot, zpair0, ha, hb,
                                       sh, z_base, z_pair_stride, ftw, smem, c, team,
                                       part, lane, zg);
  }
}

template <typename T, int P, int CPW, int MAXR, int BA>
static hipError_t launch_pc_cfg(const PairColsArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = pair_col_team<T>(P);
  constexpr int NPART = tile_width<T>() / CPW;
  const size_t shm = pair_cols_table_offset<T, P, CPW>() +
                     (pair_cols_lds_twiddles<T, P, CPW>() ? (size_t)P * sizeof(C2<T>) : 0);
  auto fn = k_pair_cols<T, P, TEAM, CPW, MAXR, BA>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  const int parts = a.tiles * NPART;
  // the layout group of the row kernels: 2 (pairs interleaved) for FP32 rows
  // up to 1024 points, else 1
  if (a.zg != 1 && !(a.zg == 2 && sizeof(T) == 4)) return hipErrorInvalidValue;
  const int ablocks = (a.QA + BA - 1) / BA;
  dim3 grid = a.items ? dim3(parts, a.max_items, 1) : dim3(parts, ablocks, a.nb);
  const int xcd_groups =
      !a.items && a.xcd != 0 && ((long long)parts * a.nb) % 8 == 0;
  hipLaunchKernelGGL(fn, grid, dim3(CPW * TEAM), shm, st, a.FA, a.fa_label_stride,
                     a.FB, a.fb_angle_stride, a.fb_label_stride, a.QA, a.QB, a.ha,
                     a.hb, a.sh, a.Z, a.z_angle_stride, a.z_pair_stride, a.tw,
                     a.items, a.n_items, xcd_groups, a.zg);
  return hipGetLastError();
}

// Launch shape: the default (the whole tile or the default part, radix cap
// 16, one label of A per workgroup) or, for FP32 fused passes, the tuner's
// choice of half the columns per workgroup, radix cap 8 and two labels of A
// per workgroup.  Item mode and the plain schedule take the default.
template <typename T, int P>
static hipError_t launch_pc_p(const PairColsArgs<T>& a, hipStream_t st) {
  constexpr int DEF = pair_cols_cpw<T, P>();
  if constexpr (sizeof(T) == 4 && DEF >= 4) {
    const bool tuned = a.items == nullptr && a.FA != nullptr;
    const bool half = tuned && a.cpw_half != 0;
    const bool r8 = tuned && a.maxr == 8;
    const bool ba2 = tuned && a.ba == 2;
    if (half) {
      if (r8) return ba2 ? launch_pc_cfg<T, P, DEF / 2, 8, 2>(a, st)
                         : launch_pc_cfg<T, P, DEF / 2, 8, 1>(a, st);
      return ba2 ? launch_pc_cfg<T, P, DEF / 2, 16, 2>(a, st)
                 : launch_pc_cfg<T, P, DEF / 2, 16, 1>(a, st);
    }
    if (r8) return ba2 ? launch_pc_cfg<T, P, DEF, 8, 2>(a, st)
                       : launch_pc_cfg<T, P, DEF, 8, 1>(a, st);
    if (ba2) return launch_pc_cfg<T, P, DEF, 16, 2>(a, st);
  }
  return launch_pc_cfg<T, P, DEF, 16, 1>(a, st);
}

template <typename T>
hipError_t launch_pair_cols(int P, const PairColsArgs<T>& a, hipStream_t st) {
  switch (P) {
    case 128: return launch_pc_p<T, 128>(a, st);
    case 256: return launch_pc_p<T, 256>(a, st);
    case 512: return launch_pc_p<T, 512>(a, st);
    case 768: return launch_pc_p<T, 768>(a, st);
    case 1024: return launch_pc_p<T, 1024>(a, st);
    case 1536: return launch_pc_p<T, 1536>(a, st);
    case 2048: return launch_pc_p<T, 2048>(a, st);
    case 4096: return launch_pc_p<T, 4096>(a, st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_pair_cols<float>(int, const PairColsArgs<float>&, hipStream_t);
template hipError_t launch_pair_cols<double>(int, const PairColsArgs<double>&, hipStream_t);

}  // namespace cmif
