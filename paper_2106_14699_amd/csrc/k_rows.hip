// Pair row pass with the fused entropy reduction (Sec. 3.2, Eq. 9-12), and
// the count-emission variant of the same row pass.
//
// k_pair_rows: one workgroup owns one map row i (displacement chi_y) of one
// angle and walks ALL label pairs for it, so the per-displacement histogram
// state never leaves the chip:
//   * teams split the labels of B: team g handles b in [g*BPW, (g+1)*BPW);
//   * two pairs (a, b0), (a, b1) share one complex inverse FFT along x:
//     W = Z_ab0 + i Z_ab1 (Hermitian extension of each half spectrum), so
//     the real part is C_ab0 and the imaginary part C_ab1 on the circular
//     x axis;
//   * counts = rint(value / (P_h P_w)); |value - count| >= 0.25 at a used
//     displacement flags the pair for the FP64 re-run; negatives clamp to 0;
//   * per displacement and lane: C_b for the team's labels (exact uint32)
//     and S_AB accumulated in FP64; the joint counts are also added into an
//     LDS C_a accumulator (integer atomics, exact and order-free);
//   * after each a, C_a is folded into S_A and N per displacement;
//   * at the end S_B is subtracted per team, the team partials are summed in
//     a fixed order, and MI = log2 N + (S_AB - S_A - S_B) / N is written;
//   * at 4096 points two workgroups share a row: each transforms the whole
//     row and keeps the state of one half of the lags (lag_parts).
// k_pair_counts: the same row transforms, writing the rounded joint counts
// and/or their order-free digests instead of entropies.
#include <type_traits>

#include "entropy.h"
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"
#include "rows_common.h"

namespace cmif {

// RERUN selects the FP64 re-run variant (angle gates, count overrides): a
// kernel of its own so that the main pass carries none of that code.
// ALLPOS (plans whose x displacements are the full set): every circular lag
// enters the per-position sums, with no branch per position.  The lags that
// carry no displacement are then displacements without overlap, whose exact
// correlation is 0: their rounded counts are 0 (their residual is transform
// noise like any other) and nothing derived from them is written.
template <typename T, int P, int TEAM, int BPW, int NTMAX, bool RERUN,
          bool ALLPOS = false>
__global__ void __launch_bounds__(NTMAX)
k_pair_rows(const C2<T>* __restrict__ Z, long long z_angle_stride,
            long long z_pair_stride, int QA, int QB, int wa, int wb, int sh,
            int sw, int ph, int rpw, const C2<T>* __restrict__ tw,
            const double* __restrict__ logtab_g,
            const double* __restrict__ xlogtab_g, double* __restrict__ mi_out,
            long long mi_angle_stride, int32_t* __restrict__ n_out,
            long long n_angle_stride, uint32_t* __restrict__ maxn,
            uint32_t* __restrict__ flags, cmif_stats* __restrict__ stats,
            const uint32_t* __restrict__ gate, const int32_t* __restrict__ ovr,
            const int32_t* __restrict__ ovc) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  constexpr int LP = lag_parts(P);  // workgroups per row
  constexpr int PX = P / LP;        // lags of this workgroup
  constexpr int RP = R / LP;        // of them per lane
  static_assert(LP == 1 || LP == 2, "one or two lag parts");
  if constexpr (RERUN) {
    if (gate[blockIdx.y] == 0u) return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nteams = blockDim.x / TEAM;
  const int NT = blockDim.x;
  C2<T>* exch = reinterpret_cast<C2<T>*>(smem_raw);
  double* ltab = reinterpret_cast<double*>(exch + (size_t)nteams * lds_elems(P));
  double* xlt = ltab + 512;                               // c log2 c, c < kXlogN
  double* sa_l = xlt + kXlogN;                             // S_A per x
  uint32_t* n_l = reinterpret_cast<uint32_t*>(sa_l + PX);  // N per x
  uint32_t* slot = n_l + PX;                    // [2 kFoldA][PX] C_a

  const int beta = blockIdx.y;  // angle within batch
  const int tid = threadIdx.x;
  // a team spans whole waves: its index is wave-uniform, and saying so
  // keeps the per-pack label tests (has0, has1) scalar branches instead of
  // exec-masked blocks around every load
  static_assert(TEAM % 64 == 0, "teams of whole waves");
  const int team = __builtin_amdgcn_readfirstlane(tid / TEAM);
  const int lane = tid % TEAM;
  C2<T>* lds = exch + team * lds_elems(P);

  for (int x = tid; x < 512; x += NT) ltab[x] = logtab_g[x];
  for (int x = tid; x < kXlogN; x += NT) xlt[x] = xlogtab_g[x];
  // SPLIT (FP32, two-wave teams): each row transform is two one-wave
  // half-length transforms joined by one exchange, so it takes one
  // workgroup barrier instead of one per Stockham exchange
  constexpr bool SPLIT = TEAM == 128 && sizeof(T) == 4;
  FftTw<T, SPLIT ? P / 2 : P, SPLIT ? 64 : TEAM> ftw;
  C2<T> wm[SPLIT ? R : 1];
  if constexpr (SPLIT) {
    fft_load_twiddles<T, P / 2, 64, 2>(ftw, tw, lane & 63);
#pragma unroll
    for (int q = 0; q < R; ++q) wm[q] = tw[(lane & 63) + 64 * q];
  } else {
    fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  }
  C2<T>* lds_w = lds + (lane >> 6) * lds_elems(P / 2);  // SPLIT: per wave
  C2<T>* cross = reinterpret_cast<C2<T>*>(slot + 2 * kFoldA * PX) + team * 2 * P;
  // lag half of this workgroup (LP = 2): lane positions q = lpart * RP + qq
  const int lpart = LP > 1 ? (int)(blockIdx.x % LP) : 0;
  const int chunk = LP > 1 ? (int)(blockIdx.x / LP) : (int)blockIdx.x;
  const int x0 = lpart * PX;
  auto pos_of = [&](int qq) {
    return row_out_pos<P, TEAM, SPLIT>(lane, lpart * RP + qq);
  };
  int nfft = 0;  // alternates the exchange buffers of consecutive transforms
  auto row_fft = [&](C2<T> (&v)[R]) {
    if constexpr (SPLIT) {
      team2_fft<T, P, +1>(v, lds_w, cross + (nfft & 1) * P, ftw, wm, lane >> 6,
                          lane & 63);
      ++nfft;
    } else {
      team_fft<T, P, TEAM, +1>(v, lds, ftw, lane);
    }
  };

  const T scale = (T)1 / ((T)ph * (T)P);
  const int tile_stride = z_tile_stride<T, P>(sh);
  const int b_first = team * BPW;
  const int nq = QA * QB;
  float maxres = 0.0f;
  uint32_t nmax = 0u;

  const int i_end = min(sh, (chunk + 1) * rpw);
  for (int i = chunk * rpw; i < i_end; ++i) {
    for (int x = tid; x < 2 * kFoldA * PX; x += NT) slot[x] = 0u;
    for (int x = tid; x < PX; x += NT) { sa_l[x] = 0.0; n_l[x] = 0u; }
    __syncthreads();
    const C2<T>* zrow = Z + beta * z_angle_stride + z_row_offset<T, P>(i);

    uint32_t cb[BPW][RP];
    double sab[RP];
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      sab[q] = 0.0;
#pragma unroll
      for (int bb = 0; bb < BPW; ++bb) cb[bb][q] = 0u;
    }

    // software pipeline: the raw loads of the next pack are in flight while
    // the current pack is transformed and reduced (not at 4096 points: the
    // registers of the loads in flight would spill there)
    constexpr bool PIPE = LP == 1;
    C2<T> nu0[R], nu1[R];
    if constexpr (PIPE) {
      const int b0 = b_first, b1 = b0 + 1;
      if (b0 < QB)
        load_raw<T, P, TEAM, SPLIT>(zrow + z_pair_offset<T, P>(b0, z_pair_stride),
                                    zrow + z_pair_offset<T, P>(b1, z_pair_stride), b1 < QB,
                                    tile_stride, lane, nu0, nu1);
    }
    for (int a = 0; a < QA; ++a) {
      uint32_t* sl = slot + (a % (2 * kFoldA)) * PX;
      uint32_t ca[RP];
#pragma unroll
      for (int q = 0; q < RP; ++q) ca[q] = 0u;
#pragma unroll
      for (int pk = 0; pk < BPW / 2; ++pk) {
        const int b0 = b_first + 2 * pk, b1 = b0 + 1;
        const bool has0 = b0 < QB, has1 = b1 < QB;
        C2<T> w[R];
        if constexpr (!PIPE) {
          if (has0)
            load_raw<T, P, TEAM, SPLIT>(
                zrow + z_pair_offset<T, P>(a * QB + b0, z_pair_stride),
                zrow + z_pair_offset<T, P>(a * QB + b1, z_pair_stride), has1,
                tile_stride, lane, nu0, nu1);
        }
        if (has0) {
          build_pack<T, P, TEAM, SPLIT>(nu0, nu1, lane, w);
        } else {
#pragma unroll
          for (int q = 0; q < R; ++q) w[q] = mk<T>((T)0, (T)0);
        }
        if constexpr (PIPE) {
          // next pack: (a, pk + 1), or (a + 1, 0)
          const int na = pk + 1 < BPW / 2 ? a : a + 1;
          const int nb0 = pk + 1 < BPW / 2 ? b0 + 2 : b_first;
          if (na < QA && nb0 < QB)
            load_raw<T, P, TEAM, SPLIT>(
                zrow + z_pair_offset<T, P>(na * QB + nb0, z_pair_stride),
                zrow + z_pair_offset<T, P>(na * QB + nb0 + 1, z_pair_stride),
                nb0 + 1 < QB, tile_stride, lane, nu0, nu1);
        }
        row_fft(w);
        // this workgroup's lags (one loop per half, so that every index
        // stays a compile-time register index)
        C2<T> wp[RP];
        if (LP > 1 && lpart) {
#pragma unroll
          for (int qq = 0; qq < RP; ++qq) wp[qq] = w[(LP - 1) * RP + qq];
        } else {
#pragma unroll
          for (int qq = 0; qq < RP; ++qq) wp[qq] = w[qq];
        }
        if constexpr (RERUN) {
          // re-run: pairs recomputed in FP64 enter with their exact counts
          // (count * P_h P_w is exact, so the rounding below returns it)
          const int o0 = has0 ? ovr[beta * nq + a * QB + b0] : -1;
          const int o1 = has1 ? ovr[beta * nq + a * QB + b1] : -1;
          if (o0 >= 0 || o1 >= 0) {
            const T unscale = (T)ph * (T)P;
            const long long mrow = (long long)i * sw;
            const long long mstride = (long long)sh * sw;
#pragma unroll
            for (int q = 0; q < RP; ++q) {
              const int j = circ_to_map(pos_of(q), P, wa, wb);
              if (j >= 0) {
                if (o0 >= 0) wp[q].x = (T)ovc[o0 * mstride + mrow + j] * unscale;
                if (o1 >= 0) wp[q].y = (T)ovc[o1 * mstride + mrow + j] * unscale;
              }
            }
          }
        }

        float e0max = 0.0f, e1max = 0.0f;
        uint32_t big = 0u;
#pragma unroll
        for (int q = 0; q < RP; ++q) {
          if (ALLPOS || circ_to_map(pos_of(q), P, wa, wb) >= 0) {
            const T v0 = wp[q].x * scale, v1 = wp[q].y * scale;
            const T r0 = round_half_even<T>(v0), r1 = round_half_even<T>(v1);
            e0max = fmaxf(e0max, (float)fabs(v0 - r0));
            e1max = fmaxf(e1max, (float)fabs(v1 - r1));
            const uint32_t n0 = (uint32_t)fmax(r0, (T)0);
            // an odd Q_B leaves the last pack without a second pair: its
            // imaginary part is transform noise and counts nothing
            const uint32_t n1 = has1 ? (uint32_t)fmax(r1, (T)0) : 0u;
            cb[2 * pk][q] += n0;
            cb[2 * pk + 1][q] += n1;
            ca[q] += n0 + n1;
            big |= n0 | n1;
            sab[q] += xlt[min(n0, (uint32_t)(kXlogN - 1))] +
                      xlt[min(n1, (uint32_t)(kXlogN - 1))];
          }
        }
        if (big >= (uint32_t)kXlogN) {
          // rare: counts beyond the table, replace the clamped entries
#pragma unroll
          for (int q = 0; q < RP; ++q) {
            if (ALLPOS || circ_to_map(pos_of(q), P, wa, wb) >= 0) {
              const uint32_t n0 = (uint32_t)fmax(round_half_even<T>(wp[q].x * scale), (T)0);
              const uint32_t n1 =
                  has1 ? (uint32_t)fmax(round_half_even<T>(wp[q].y * scale), (T)0) : 0u;
              if (n0 >= (uint32_t)kXlogN)
                sab[q] += xlog2x_u32(n0, ltab) - xlt[kXlogN - 1];
              if (n1 >= (uint32_t)kXlogN)
                sab[q] += xlog2x_u32(n1, ltab) - xlt[kXlogN - 1];
            }
          }
        }
        if (!has1) e1max = 0.0f;
        maxres = fmaxf(maxres, fmaxf(e0max, e1max));
        if (!RERUN && flags != nullptr) {
          if (__ballot(has0 && e0max >= 0.25f) != 0ull && (tid % 64) == 0) {
            const uint32_t old = atomicOr(&flags[beta * nq + a * QB + b0], 1u);
            if (old == 0u && stats) atomicAdd(&stats->flagged_pairs, 1u);
          }
          if (__ballot(has1 && e1max >= 0.25f) != 0ull && (tid % 64) == 0) {
            const uint32_t old = atomicOr(&flags[beta * nq + a * QB + b1], 1u);
            if (old == 0u && stats) atomicAdd(&stats->flagged_pairs, 1u);
          }
        }
      }
      // exact C_a = sum over all teams' b of C_ab (integer atomics; adding
      // a zero costs less than the lane-divergent branch that would skip it)
#pragma unroll
      for (int q = 0; q < RP; ++q) atomicAdd(&sl[pos_of(q) - x0], ca[q]);
      // every kFoldA labels of A (and after the last): their C_a are
      // complete, fold them into S_A and N.  The planes of consecutive
      // groups alternate, so the next group's atomics need no second
      // barrier.
      if ((a + 1) % kFoldA == 0 || a + 1 == QA) {
        __syncthreads();
        const int a0 = a - a % kFoldA;
        for (int x = tid; x < PX; x += NT) {
          for (int g = a0; g <= a; ++g) {
            uint32_t* sg = slot + (g % (2 * kFoldA)) * PX;
            const uint32_t cv = sg[x];
            if (cv != 0u) {
              sg[x] = 0u;
              sa_l[x] += cv < (uint32_t)kXlogN ? xlt[cv] : xlog2x_u32(cv, ltab);
              n_l[x] += cv;
            }
          }
        }
      }
    }

    // S_AB - S_B per team, then a fixed-order sum over teams
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      double sb = 0.0;
#pragma unroll
      for (int bb = 0; bb < BPW; ++bb) {
        const uint32_t v = cb[bb][q];
        sb += v < (uint32_t)kXlogN ? xlt[v] : xlog2x_u32(v, ltab);
      }
      sab[q] -= sb;
    }
    __syncthreads();
    double* part = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int q = 0; q < RP; ++q) part[pos_of(q) - x0] = sab[q];
    __syncthreads();

    for (int x = tid; x < PX; x += NT) {
      const int j = circ_to_map(x0 + x, P, wa, wb);
      if (j >= 0) {
        double tsum = 0.0;
        for (int g = 0; g < nteams; ++g)
          tsum += reinterpret_cast<const double*>(exch + g * lds_elems(P))[x];
        const uint32_t nn = n_l[x];
        // MI >= 0 for any joint histogram, and one label on either side
        // gives H_AB = H_B (or H_A) term by term, so MI = 0 exactly; the
        // identity form can round to a few ulps on either side of those
        double mi = 0.0;
        if (nn > 0u && QA > 1 && QB > 1)
          mi = fmax(log2_u32(nn, ltab) + (tsum - sa_l[x]) / (double)nn, 0.0);
        if (mi_out) mi_out[beta * mi_angle_stride + (long long)i * sw + j] = mi;
        if (n_out) n_out[beta * n_angle_stride + (long long)i * sw + j] = (int32_t)nn;
        nmax = nn > nmax ? nn : nmax;
      }
    }
    __syncthreads();  // part[] and the tables are reused by the next row
  }
  // wave max of N and of the residual, one atomic per wave
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t on = __shfl_xor(nmax, o, 64);
    nmax = on > nmax ? on : nmax;
    maxres = fmaxf(maxres, __shfl_xor(maxres, o, 64));
  }
  if ((tid % 64) == 0) {
    atomicMax(&maxn[beta], nmax);
    if (stats)
      atomicMax(reinterpret_cast<unsigned int*>(&stats->max_residual),
                __float_as_uint(maxres));
  }
}

// Lanes of the count kernel's workgroup: up to four teams, at most 512 lanes
// (two waves per SIMD keep 256 registers per lane; at 1024 lanes the
// 2048-point kernel spilled; team_for gives at most 256 lanes, a divisor of 512).
// 3 * 2^k lengths (12 points per lane) keep two teams: with 512 lanes the
// 1536-point kernel spilled.
constexpr int counts_lanes(int team, int p) {
  return !is_pow2(p) ? 2 * team : (4 * team <= 512 ? 4 * team : 512);
}

// Count emission: workgroup (map row, angle); each team takes label pairs
// two at a time (a-major order) and writes rint(count) to
// counts[beta][pair][i][j] and/or adds sum_j count * splitmix64(i*S_w + j)
// into digest[beta][pair] (64-bit wrap-around, order-free).  In item mode
// the slots of Z are list items (angle, a, b) and the grid has one angle.
template <typename T, int P, int TEAM>
__global__ void __launch_bounds__(counts_lanes(TEAM, P))
k_pair_counts(const C2<T>* __restrict__ Z, long long z_angle_stride,
              long long z_pair_stride, int QA, int QB, int wa, int wb, int sh,
              int sw, int ph, const C2<T>* __restrict__ tw,
              int32_t* __restrict__ counts, long long counts_angle_stride,
              uint64_t* __restrict__ digest, double* __restrict__ values,
              const int4* __restrict__ items,
              const uint32_t* __restrict__ n_items,
              int32_t* __restrict__ item_counts, long long digest_index0) {
  constexpr int R = P / TEAM;
  constexpr int TW = tile_width<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<T>* exch = reinterpret_cast<C2<T>*>(smem_raw);
  const int nteams = blockDim.x / TEAM;
  const int i = blockIdx.x, beta = blockIdx.y;
  static_assert(TEAM % 64 == 0, "teams of whole waves");
  const int tid = threadIdx.x, lane = tid % TEAM;
  const int team = __builtin_amdgcn_readfirstlane(tid / TEAM);  // wave-uniform
  C2<T>* lds = exch + team * lds_elems(P);
  const T scale = (T)1 / ((T)ph * (T)P);
  const C2<T>* zrow = Z + beta * z_angle_stride + z_row_offset<T, P>(i);
  const int npairs = QA * QB;
  const int nq = items ? (int)*n_items : npairs;  // slots of Z to emit
  if (nq == 0) return;
  const int npk = (nq + 1) / 2;
  const int iters = (npk + nteams - 1) / nteams;
  FftTw<T, P, TEAM> ftw;
  fft_load_twiddles<T, P, TEAM>(ftw, tw, lane);
  for (int it = 0; it < iters; ++it) {
    const int pk = team + it * nteams;
    const int p0 = 2 * pk, p1 = p0 + 1;
    const bool has0 = p0 < nq, has1 = p1 < nq;
    C2<T> w[R];
    if (has0) {
      load_pack<T, P, TEAM>(zrow + z_pair_offset<T, P>(p0, z_pair_stride),
                            zrow + z_pair_offset<T, P>(p1, z_pair_stride), has1,
                            z_tile_stride<T, P>(sh), lane, w);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) w[q] = mk<T>((T)0, (T)0);
    }
    team_fft<T, P, TEAM, +1>(w, lds, ftw, lane);
    // output angle and pair of slots p0, p1
    int g0 = beta, t0 = p0, g1 = beta, t1 = p1;
    if (items != nullptr) {
      if (has0) { const int4 e = items[p0]; g0 = e.x; t0 = e.y * QB + e.z; }
      if (has1) { const int4 e = items[p1]; g1 = e.x; t1 = e.y * QB + e.z; }
    }
    int32_t* cbase0 = counts ? counts + g0 * counts_angle_stride : nullptr;
    int32_t* cbase1 = counts ? counts + g1 * counts_angle_stride : nullptr;
    uint64_t d0 = 0, d1 = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int j = circ_to_map(lane + TEAM * q, P, wa, wb);
      if (has0 && j >= 0) {
        const T r0 = round_half_even<T>(w[q].x * scale);
        const T r1 = round_half_even<T>(w[q].y * scale);
        const uint32_t n0 = r0 > (T)0 ? (uint32_t)r0 : 0u;
        const uint32_t n1 = r1 > (T)0 ? (uint32_t)r1 : 0u;
        const long long o = (long long)i * sw + j;
        if (counts) {
          cbase0[(long long)t0 * sh * sw + o] = (int32_t)n0;
          if (has1) cbase1[(long long)t1 * sh * sw + o] = (int32_t)n1;
        }
        if (item_counts) {
          item_counts[(long long)p0 * sh * sw + o] = (int32_t)n0;
          if (has1) item_counts[(long long)p1 * sh * sw + o] = (int32_t)n1;
        }
        if (values) {
          double* vb = values + beta * counts_angle_stride;
          vb[(long long)p0 * sh * sw + o] = (double)(w[q].x * scale);
          if (has1) vb[(long long)p1 * sh * sw + o] = (double)(w[q].y * scale);
        }
        const uint64_t wgt = splitmix64((uint64_t)(digest_index0 + o));
        d0 += (uint64_t)n0 * wgt;
        d1 += (uint64_t)n1 * wgt;
      }
    }
    if (digest) {
      d0 = wave_sum_u64(d0);
      d1 = wave_sum_u64(d1);
      if ((tid % 64) == 0 && has0) {
        atomicAdd((unsigned long long*)&digest[(long long)g0 * npairs + t0],
                  (unsigned long long)d0);
        if (has1)
          atomicAdd((unsigned long long*)&digest[(long long)g1 * npairs + t1],
                    (unsigned long long)d1);
      }
    }
  }
}

template <typename T, int P, int BPW, int NTMAX, bool RERUN, bool ALLPOS = false>
static hipError_t launch_pr_cfg(const PairRowsArgs<T>& a, int nteams, size_t shm,
                                hipStream_t st) {
  constexpr int TEAM = team_for(P);
  auto fn = k_pair_rows<T, P, TEAM, BPW, NTMAX, RERUN, ALLPOS>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  const int rpw = a.rows_per_wg > 0 ? a.rows_per_wg : 1;
  dim3 grid((a.sh + rpw - 1) / rpw * lag_parts(P), a.nb);
  hipLaunchKernelGGL(fn, grid, dim3(nteams * TEAM), shm, st, a.Z,
                     a.z_angle_stride, a.z_pair_stride, a.QA, a.QB, a.wa, a.wb,
                     a.sh, a.sw, a.ph, rpw, a.tw, a.logtab, a.xlogtab, a.mi,
                     a.mi_angle_stride, a.n, a.n_angle_stride, a.maxn, a.flags,
                     a.stats, a.gate, a.ovr, a.ovc);
  return hipGetLastError();
}

template <typename T, int P, int BPW, bool RERUN, bool ALLPOS>
static hipError_t launch_pr_nt(const PairRowsArgs<T>& a, const PairRowsConfig& c,
                               hipStream_t st) {
  if (c.ntmax <= 256) return launch_pr_cfg<T, P, BPW, 256, RERUN, ALLPOS>(a, c.nteams, c.lds, st);
  if (c.ntmax <= 512) return launch_pr_cfg<T, P, BPW, 512, RERUN, ALLPOS>(a, c.nteams, c.lds, st);
  return launch_pr_cfg<T, P, BPW, 1024, RERUN, ALLPOS>(a, c.nteams, c.lds, st);
}

template <typename T, int P, int BPW, bool RERUN>
static hipError_t launch_pr_rr(const PairRowsArgs<T>& a, const PairRowsConfig& c,
                               hipStream_t st) {
  // every lag outside the map is a displacement without overlap when the x
  // displacements are the full set (window extents = image widths)
  if constexpr (!RERUN) {
    if (a.full_x) return launch_pr_nt<T, P, BPW, false, true>(a, c, st);
  }
  return launch_pr_nt<T, P, BPW, RERUN, false>(a, c, st);
}

template <typename T, int P, int BPW>
static hipError_t launch_pr_bpw(const PairRowsArgs<T>& a, const PairRowsConfig& c,
                                hipStream_t st) {
  // the FP64 re-run exists for the FP32 pass only
  if constexpr (std::is_same<T, float>::value) {
    if (a.ovr != nullptr) {
      if (a.gate == nullptr || a.ovc == nullptr) return hipErrorInvalidValue;
      return launch_pr_rr<T, P, BPW, true>(a, c, st);
    }
  } else {
    if (a.ovr != nullptr) return hipErrorInvalidValue;
  }
  return launch_pr_rr<T, P, BPW, false>(a, c, st);
}

// One (precision, FFT length) per object file: the build compiles this file
// once per pair with CMIF_ROWS_T / CMIF_ROWS_P set, and once without them
// for the dispatchers below, which only reference these.
template <typename T, int P>
hipError_t launch_pair_rows_p(const PairRowsArgs<T>& a, hipStream_t st) {
  // FP64 rows at 4096 points do not fit the LDS (plans reject them); the
  // 4096-point FP64 object holds the count kernel of the re-run only
  if constexpr (sizeof(T) == 8 && P >= 4096) {
    (void)a;
    (void)st;
    return hipErrorInvalidValue;
  } else {
  PairRowsConfig c;
  const bool ok = a.bpw > 0 ? pair_rows_config_bpw(sizeof(T), P, a.QB, a.bpw, &c)
                            : pair_rows_config(sizeof(T), P, a.QB, &c);
  if (!ok) return hipErrorInvalidValue;
  if (c.bpw == 4) return launch_pr_bpw<T, P, 4>(a, c, st);
  if (c.bpw == 8) return launch_pr_bpw<T, P, 8>(a, c, st);
  return launch_pr_bpw<T, P, 16>(a, c, st);
  }
}

template <typename T, int P>
hipError_t launch_pair_counts_p(const PairCountsArgs<T>& a, hipStream_t st) {
  constexpr int TEAM = team_for(P);
  const size_t per_team = (size_t)lds_elems(P) * sizeof(C2<T>);
  int nteams = counts_lanes(TEAM, P) / TEAM;
  while (nteams > 1 && per_team * nteams > 64 * 1024) --nteams;
  const size_t shm = per_team * nteams;
  auto fn = k_pair_counts<T, P, TEAM>;
  hipError_t e = hipFuncSetAttribute((const void*)fn,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  dim3 grid(a.sh, a.items ? 1 : a.nb);
  hipLaunchKernelGGL(fn, grid, dim3(nteams * TEAM), shm, st, a.Z,
                     a.z_angle_stride, a.z_pair_stride, a.QA, a.QB, a.wa, a.wb,
                     a.sh, a.sw, a.ph, a.tw, a.counts, a.counts_angle_stride,
                     a.digest, a.values, a.items, a.n_items, a.item_counts,
                     a.digest_index0);
  return hipGetLastError();
}

#if defined(CMIF_ROWS_T) && defined(CMIF_ROWS_P)

template hipError_t launch_pair_rows_p<CMIF_ROWS_T, CMIF_ROWS_P>(
    const PairRowsArgs<CMIF_ROWS_T>&, hipStream_t);
template hipError_t launch_pair_counts_p<CMIF_ROWS_T, CMIF_ROWS_P>(
    const PairCountsArgs<CMIF_ROWS_T>&, hipStream_t);

#else

#define CMIF_ROWS_EXTERN(T, P)                                                  \
  extern template hipError_t launch_pair_rows_p<T, P>(const PairRowsArgs<T>&,   \
                                                      hipStream_t);             \
  extern template hipError_t launch_pair_counts_p<T, P>(const PairCountsArgs<T>&, \
                                                        hipStream_t);
CMIF_ROWS_EXTERN(float, 128)
CMIF_ROWS_EXTERN(float, 256)
CMIF_ROWS_EXTERN(float, 512)
CMIF_ROWS_EXTERN(float, 768)
CMIF_ROWS_EXTERN(float, 1024)
CMIF_ROWS_EXTERN(float, 1536)
CMIF_ROWS_EXTERN(float, 2048)
CMIF_ROWS_EXTERN(float, 4096)
CMIF_ROWS_EXTERN(double, 128)
CMIF_ROWS_EXTERN(double, 256)
CMIF_ROWS_EXTERN(double, 512)
CMIF_ROWS_EXTERN(double, 768)
CMIF_ROWS_EXTERN(double, 1024)
CMIF_ROWS_EXTERN(double, 1536)
CMIF_ROWS_EXTERN(double, 2048)
CMIF_ROWS_EXTERN(double, 4096)
#undef CMIF_ROWS_EXTERN

template <typename T>
hipError_t launch_pair_rows(int P, const PairRowsArgs<T>& a, hipStream_t st) {
  switch (P) {
    case 128: return launch_pair_rows_p<T, 128>(a, st);
    case 256: return launch_pair_rows_p<T, 256>(a, st);
    case 512: return launch_pair_rows_p<T, 512>(a, st);
    case 768: return launch_pair_rows_p<T, 768>(a, st);
    case 1024: return launch_pair_rows_p<T, 1024>(a, st);
    case 1536: return launch_pair_rows_p<T, 1536>(a, st);
    case 2048: return launch_pair_rows_p<T, 2048>(a, st);
    case 4096: return launch_pair_rows_p<T, 4096>(a, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pair_counts(int P, const PairCountsArgs<T>& a, hipStream_t st) {
  switch (P) {
    case 128: return launch_pair_counts_p<T, 128>(a, st);
    case 256: return launch_pair_counts_p<T, 256>(a, st);
    case 512: return launch_pair_counts_p<T, 512>(a, st);
    case 768: return launch_pair_counts_p<T, 768>(a, st);
    case 1024: return launch_pair_counts_p<T, 1024>(a, st);
    case 1536: return launch_pair_counts_p<T, 1536>(a, st);
    case 2048: return launch_pair_counts_p<T, 2048>(a, st);
    case 4096: return launch_pair_counts_p<T, 4096>(a, st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_pair_rows<float>(int, const PairRowsArgs<float>&, hipStream_t);
template hipError_t launch_pair_rows<double>(int, const PairRowsArgs<double>&, hipStream_t);
template hipError_t launch_pair_counts<float>(int, const PairCountsArgs<float>&, hipStream_t);
template hipError_t launch_pair_counts<double>(int, const PairCountsArgs<double>&, hipStream_t);

#endif

}  // namespace cmif
