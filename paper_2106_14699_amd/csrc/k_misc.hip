// Small kernels: twiddle / log tables, fills, label-range check, and the
// Alg. 1 argmax (per angle over eligible displacements, then across angles).
#include "entropy.h"
#include "fft_core.h"
#include "internal.h"
#include "kernels.h"

namespace cmif {

// tw[t] = exp(+2 pi i t / P) evaluated in FP64 with sincospi (exact argument
// reduction of t/P), stored in FP32 and FP64; logtab[j] = log2(1 + j/256),
// logtab[256 + j] = 1 / (1 + j/256); xlogtab[c] = c log2 c for c < kXlogN
// (0 for c = 0, 1).
__global__ void k_init_tables(float2* tw32, double2* tw64, int P, double* logtab,
                              double* xlogtab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < P) {
    double s, c;
    sincospi(2.0 * (double)t / (double)P, &s, &c);
    if (tw64) tw64[t] = make_double2(c, s);
    if (tw32) tw32[t] = make_float2((float)c, (float)s);
  }
  if (logtab && t < 256) {
    const double m = 1.0 + (double)t / 256.0;
    logtab[t] = log2(m);
    logtab[256 + t] = 1.0 / m;
  }
  if (xlogtab && t < kXlogN) xlogtab[t] = t <= 1 ? 0.0 : (double)t * log2((double)t);
}

hipError_t launch_init_tables(void* tw32, void* tw64, int P, double* logtab,
                              double* xlogtab, hipStream_t st) {
  const int n = P > kXlogN ? P : kXlogN;
  hipLaunchKernelGGL(k_init_tables, dim3((n + 255) / 256), dim3(256), 0, st,
                     (float2*)tw32, (double2*)tw64, P, logtab, xlogtab);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// Counts pixels inside the mask whose label is >= Q (they belong to no
// level set; the direct method would have no histogram bin for them).
__global__ void k_check_labels(const uint8_t* lab, const uint8_t* msk,
                               long long n, int Q, cmif_stats* stats) {
  uint32_t bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if ((msk == nullptr || msk[i]) && lab[i] >= Q) ++bad;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
  if ((threadIdx.x % 64) == 0 && bad) atomicAdd(&stats->label_errors, bad);
}

hipError_t launch_check_labels(const uint8_t* lab, const uint8_t* msk,
                               long long n, int Q, cmif_stats* stats,
                               hipStream_t st) {
  if (stats == nullptr || n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_check_labels, dim3((unsigned)blocks), dim3(256), 0, st,
                     lab, msk, n, Q, stats);
  return hipGetLastError();
}

// (mi, idx) ordering of Alg. 1 inside one transform: larger MI wins, equal
// MI goes to the smaller row-major index; idx < 0 means "none".
__device__ __forceinline__ bool better(double m1, long long i1, double m2,
                                       long long i2) {
  if (i2 < 0) return i1 >= 0;
  if (i1 < 0) return false;
  return m1 > m2 || (m1 == m2 && i1 < i2);
}

// Per (row chunk, angle): best eligible entry, N >= gamma * max N compared
// in FP64.
__global__ void __launch_bounds__(256)
k_argmax_partial(const double* __restrict__ mi, const int32_t* __restrict__ nmap,
                 long long angle_stride, const uint32_t* __restrict__ maxn,
                 int sh, int sw, int rows_per_chunk, int nchunks, double gamma,
                 ArgPartial* __restrict__ partial) {
  const int chunk = blockIdx.x, beta = blockIdx.y;
  const double thr = gamma * (double)maxn[beta];
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(sh, r0 + rows_per_chunk);
  const long long lo = (long long)r0 * sw, hi = (long long)r1 * sw;
  const double* m = mi + beta * angle_stride;
  const int32_t* nn = nmap + beta * angle_stride;
  double bm = 0.0;
  long long bi = -1;
  int bn = 0;
  for (long long k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    const int n = nn[k];
    if ((double)n >= thr) {
      const double v = m[k];
      if (better(v, k, bm, bi)) { bm = v; bi = k; bn = n; }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double om = __shfl_xor(bm, o, 64);
    const long long oi = __shfl_xor(bi, o, 64);
    const int on = __shfl_xor(bn, o, 64);
    if (better(om, oi, bm, bi)) { bm = om; bi = oi; bn = on; }
  }
  __shared__ double sm[4];
  __shared__ long long si[4];
  __shared__ int sn[4];
  const int w = threadIdx.x / 64;
  if ((threadIdx.x % 64) == 0) { sm[w] = bm; si[w] = bi; sn[w] = bn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x / 64); ++k)
      if (better(sm[k], si[k], bm, bi)) { bm = sm[k]; bi = si[k]; bn = sn[k]; }
    ArgPartial p;
    p.mi = bm;
    p.idx = bi;
    p.n = bn;
    partial[beta * nchunks + chunk] = p;
  }
}

// FP64 re-run list (Sec. 3.2: a transform whose rounding residual is too
// large is recomputed in double precision).  One workgroup walks the batch's
// (angle, pair) flags in order and keeps the first `capacity` flagged ones:
// items[s] = (angle, a, b), ovr[angle][pair] = s (else -1), gate[angle] = 1
// for angles with an item and gate[nb] = 1 if there is any.  The gated
// angles' max-N is cleared (their rows are reduced again) and so are the
// digests of listed pairs (their exact counts are emitted again).
__global__ void __launch_bounds__(1024)
k_fb_list(const uint32_t* __restrict__ flags, int nb, int QA, int QB, int force,
          int capacity, int4* __restrict__ items, uint32_t* __restrict__ n_items,
          int32_t* __restrict__ ovr, uint32_t* __restrict__ gate,
          uint32_t* __restrict__ maxn, uint64_t* __restrict__ digest,
          cmif_stats* __restrict__ stats) {
  __shared__ uint32_t wave_cnt[16];
  __shared__ uint32_t gate_l[kMaxBatch];
  const int tid = threadIdx.x, wave = tid / 64, wl = tid % 64;
  const int nwaves = blockDim.x / 64;
  const int nq = QA * QB;
  const int total = nb * nq;
  for (int b = tid; b < kMaxBatch; b += blockDim.x) gate_l[b] = 0u;
  __syncthreads();
  uint32_t base = 0;  // flagged items before this chunk (uniform)
  for (int c0 = 0; c0 < total; c0 += blockDim.x) {
    const int idx = c0 + tid;
    const bool f = idx < total && (force != 0 || flags[idx] != 0u);
    const uint64_t bal = __ballot(f);
    const uint32_t below = (uint32_t)__popcll(bal & ((1ull << wl) - 1ull));
    if (wl == 0) wave_cnt[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0, chunk = 0;
    for (int w = 0; w < nwaves; ++w) {
      if (w < wave) before += wave_cnt[w];
      chunk += wave_cnt[w];
    }
    if (idx < total) {
      int32_t slot = -1;
      const uint32_t pos = base + before + below;
      if (f && pos < (uint32_t)capacity) {
        const int beta = idx / nq, pr = idx % nq;
        items[pos] = make_int4(beta, pr / QB, pr % QB, 0);
        slot = (int32_t)pos;
        gate_l[beta] = 1u;
        if (digest) digest[idx] = 0ull;
      } else if (flags[idx] != 0u && stats) {
        // its residual reached 0.25 and it is not recomputed: its counts
        // may be off by one
        atomicAdd(&stats->unresolved_pairs, 1u);
      }
      ovr[idx] = slot;
    }
    base += chunk;
    __syncthreads();  // wave_cnt is rewritten by the next chunk
  }
  const uint32_t kept = base < (uint32_t)capacity ? base : (uint32_t)capacity;
  uint32_t any = 0u;
  for (int b = 0; b < nb; ++b) any |= gate_l[b];
  for (int b = tid; b < nb; b += blockDim.x) {
    gate[b] = gate_l[b];
    if (gate_l[b]) maxn[b] = 0u;
  }
  if (tid == 0) {
    gate[nb] = any;
    *n_items = kept;
    if (stats) {
      atomicAdd(&stats->fallback_pairs, kept);
      atomicAdd(&stats->fallback_overflow, base - kept);
    }
  }
}

// Alg. 1 across the two stages of Sec. 3.6 for one image pair: the
// refinement result (in *best, angle index into the refinement list)
// replaces the grid's only with a strictly larger MI, its angle index then
// counted after the n_grid grid angles.  Copies of both stage results go to
// grid_out and refine_out when given.
__global__ void k_two_stage_combine(cmif_best grid, cmif_best* __restrict__ best,
                                    cmif_best* __restrict__ grid_out,
                                    cmif_best* __restrict__ refine_out,
                                    int n_grid) {
  if (threadIdx.x != 0) return;
  cmif_best r = *best;
  if (refine_out) *refine_out = r;
  if (grid_out) *grid_out = grid;
  if (r.mi > grid.mi) {
    r.angle_index = n_grid + r.angle_index;
    *best = r;
  } else {
    *best = grid;
  }
}

hipError_t launch_two_stage_combine(const cmif_best& grid, cmif_best* best,
                                    cmif_best* grid_out, cmif_best* refine_out,
                                    int n_grid, hipStream_t st) {
  hipLaunchKernelGGL(k_two_stage_combine, dim3(1), dim3(64), 0, st, grid, best,
                     grid_out, refine_out, n_grid);
  return hipGetLastError();
}

hipError_t launch_fb_list(const FbListArgs& a, hipStream_t st) {
  if (a.nb < 1 || a.nb > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fb_list, dim3(1), dim3(1024), 0, st, a.flags, a.nb, a.QA,
                     a.QB, a.force, a.capacity, a.items, a.n_items, a.ovr,
                     a.gate, a.maxn, a.digest, a.stats);
  return hipGetLastError();
}

// Plain schedule (the paper-shaped comparator): Y = conj(F_a) F_b as its
// own kernel, element (c, k_y) per thread.  Column 0 packs the k_x = 0 and
// k_x = P_w/2 columns (both Hermitian in k_y): they are separated, multiplied
// and packed again, as the fused pair kernel does.
__global__ void k_plain_product(const double2* __restrict__ fa,
                                const double2* __restrict__ fb,
                                double2* __restrict__ y, int half, int ph) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)half * ph) return;
  const int c = (int)(e / ph), k = (int)(e % ph);
  const double2 a = fa[e], b = fb[e];
  if (c != 0) {
    y[e] = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
    return;
  }
  const int km = k == 0 ? 0 : ph - k;
  const double2 am = fa[km], bm = fb[km];
  // separate W = G0 + i G1 (G0, G1 Hermitian): G0 = (W + conj(Wm))/2,
  // G1 = (W - conj(Wm))/(2i)
  const double2 a0 = make_double2((a.x + am.x) * 0.5, (a.y - am.y) * 0.5);
  const double2 a1 = make_double2((a.y + am.y) * 0.5, (am.x - a.x) * 0.5);
  const double2 b0 = make_double2((b.x + bm.x) * 0.5, (b.y - bm.y) * 0.5);
  const double2 b1 = make_double2((b.y + bm.y) * 0.5, (bm.x - b.x) * 0.5);
  const double2 y0 = make_double2(a0.x * b0.x + a0.y * b0.y, a0.x * b0.y - a0.y * b0.x);
  const double2 y1 = make_double2(a1.x * b1.x + a1.y * b1.y, a1.x * b1.y - a1.y * b1.x);
  y[e] = make_double2(y0.x - y1.y, y0.y + y1.x);
}

hipError_t launch_plain_product(const C2<double>* fa, const C2<double>* fb,
                                C2<double>* y, int half, int ph, hipStream_t st) {
  const long long n = (long long)half * ph;
  hipLaunchKernelGGL(k_plain_product, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, st, reinterpret_cast<const double2*>(fa),
                     reinterpret_cast<const double2*>(fb),
                     reinterpret_cast<double2*>(y), half, ph);
  return hipGetLastError();
}

// Plain schedule: Eq. 12 per displacement from separately transformed and
// materialised maps (joint, both marginals, N; Eq. 9-11), each rounded to
// the nearest integer (Sec. 3.2).  One thread per displacement.
__device__ __forceinline__ double plain_xlog(double v) {
  const double c = fmax(rint(v), 0.0);
  return c > 1.0 ? c * log2(c) : 0.0;
}

__global__ void k_plain_entropy(const double* __restrict__ joint,
                                const double* __restrict__ marg_a,
                                const double* __restrict__ marg_b,
                                const double* __restrict__ nmap, long long S,
                                int QA, int QB, double* __restrict__ mi,
                                int32_t* __restrict__ n_out,
                                uint32_t* __restrict__ maxn) {
  const long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  uint32_t nn = 0u;
  if (o < S) {
    const double nr = fmax(rint(nmap[o]), 0.0);
    nn = (uint32_t)nr;
    double v = 0.0;
    // MI >= 0, and exactly 0 with one label on either side (as in the
    // fused row pass)
    if (nn > 0u && QA > 1 && QB > 1) {
      double sab = 0.0, sa = 0.0, sb = 0.0;
      for (int p = 0; p < QA * QB; ++p) sab += plain_xlog(joint[p * S + o]);
      for (int a = 0; a < QA; ++a) sa += plain_xlog(marg_a[a * S + o]);
      for (int b = 0; b < QB; ++b) sb += plain_xlog(marg_b[b * S + o]);
      v = fmax(log2(nr) + (sab - sa - sb) / nr, 0.0);
    }
    mi[o] = v;
    n_out[o] = (int32_t)nn;
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    const uint32_t t = __shfl_xor(nn, s, 64);
    nn = t > nn ? t : nn;
  }
  if ((threadIdx.x % 64) == 0) atomicMax(maxn, nn);
}

hipError_t launch_plain_entropy(const PlainEntropyArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_plain_entropy, dim3((unsigned)((a.S + 255) / 256)), dim3(256),
                     0, st, a.joint, a.marg_a, a.marg_b, a.nmap, a.S, a.QA, a.QB,
                     a.mi, a.n, a.maxn);
  return hipGetLastError();
}

hipError_t launch_argmax(const ArgmaxArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_argmax_partial, dim3(a.nchunks, a.nb), dim3(256), 0, st,
                     a.mi, a.n, a.angle_stride, a.maxn, a.sh, a.sw,
                     a.rows_per_chunk, a.nchunks, a.gamma, a.partial);
  return hipGetLastError();
}

// One thread: per angle of the batch reduce the chunk partials, then fold
// the angles in order into the running best.  As in Alg. 1 the best starts
// as the identity with I = 0 (angle_index -1, chi = 0) and only a strictly
// larger MI replaces it, so the earliest angle wins ties.
struct AngleVals {
  double v[kMaxBatch];
};

__global__ void __launch_bounds__(64 * kMaxBatch)
k_argmax_final(const ArgPartial* __restrict__ partial, int nb, int nchunks,
               int sw, int ha, int wa, int angle0, AngleVals angles,
               cmif_best* __restrict__ per_angle, cmif_best* __restrict__ running,
               int first_batch, cmif_best* __restrict__ best_out,
               int last_batch) {
  __shared__ cmif_best res[kMaxBatch];
  // wave b reduces angle b's chunk partials (the order of a max with the
  // smaller-index tie rule does not matter)
  const int b = threadIdx.x / 64, l = threadIdx.x % 64;
  if (b < nb) {
    double bm = 0.0;
    long long bi = -1;
    long long bn = 0;
    for (int c = l; c < nchunks; c += 64) {
      const ArgPartial p = partial[b * nchunks + c];
      if (better(p.mi, p.idx, bm, bi)) { bm = p.mi; bi = p.idx; bn = p.n; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double om = __shfl_xor(bm, o, 64);
      const long long oi = __shfl_xor(bi, o, 64);
      const long long on = __shfl_xor(bn, o, 64);
      if (better(om, oi, bm, bi)) { bm = om; bi = oi; bn = on; }
    }
    if (l == 0) {
      cmif_best r;
      r.angle_index = angle0 + b;
      r.angle_rad = angles.v[b];
      r.reserved = 0;
      if (bi >= 0) {
        r.dy = (int)(bi / sw) - (ha - 1);
        r.dx = (int)(bi % sw) - (wa - 1);
        r.mi = bm;
        r.n = bn;
      } else {
        r.dy = 0;
        r.dx = 0;
        r.mi = 0.0;
        r.n = 0;
      }
      res[b] = r;
      if (per_angle) per_angle[angle0 + b] = r;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  cmif_best run = *running;
  if (first_batch) {
    run.angle_index = -1;
    run.dy = 0;
    run.dx = 0;
    run.reserved = 0;
    run.angle_rad = 0.0;
    run.mi = 0.0;
    run.n = 0;
  }
  // angles in order: I starts at 0 with the identity, a strictly larger MI
  // replaces the best (the earliest angle wins ties)
  for (int k = 0; k < nb; ++k)
    if (res[k].mi > run.mi) run = res[k];
  *running = run;
  if (last_batch && best_out) *best_out = run;
}

hipError_t launch_argmax_final(const ArgmaxFinalArgs& a, hipStream_t st) {
  AngleVals av;
  for (int b = 0; b < kMaxBatch; ++b) av.v[b] = a.angles[b];
  if (a.nb < 1 || a.nb > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(64 * a.nb), 0, st, a.partial, a.nb,
                     a.nchunks, a.sw, a.ha, a.wa, a.angle0, av,
                     a.per_angle, a.running, a.first_batch, a.best_out,
                     a.last_batch);
  return hipGetLastError();
}

}  // namespace cmif
