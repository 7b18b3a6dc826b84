// Team-level Stockham FFT for gfx950 (wave64).
//
// A "team" of TEAM lanes (one wave, or several waves of one workgroup)
// transforms one complex sequence of length N = TEAM * R held in registers:
// lane l owns elements l + TEAM*q, q in [0, R), on entry and on exit
// (natural order).  Each radix stage does R/r radix-r butterflies per lane in
// registers; consecutive stages exchange data through a padded LDS buffer.
// The stage formula is the Stockham autosort recurrence: butterfly j reads
// elements j + m*N/r, multiplies by w^(m*(j mod Ns)*N/(Ns*r)), and writes
// output m to (j - j mod Ns)*r + (j mod Ns) + m*Ns.  With the lane mapping
// above, the reads of every stage are exactly the lane's own registers, and
// the last stage lands in natural order without an exchange.
//
// Lengths are 2^k or 3 * 2^k.  Radices are chosen greedily: the largest r in
// {16, 12, 8, 4, 3, 2} that divides both R = N/TEAM (points per lane) and
// the length still to be split, N/Ns; e.g. N = 1024 over 128 lanes runs as
// 8 x 8 x 8 x 2 with three LDS exchanges, N = 768 over 64 lanes as
// 12 x 4 x 4 x 4 (the stage formula above holds for any sequence of
// radices, with Ns the product of the radices before the stage).  Twiddles
// come from a table tw[t] = exp(+2 pi i t / N) computed in FP64 (no
// recurrences); each lane keeps the entries it needs in registers; DIR = -1
// (forward) uses their conjugates.  Transforms are unnormalised both ways.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmif {

template <typename T> struct c2t;
template <> struct c2t<float> { using type = float2; };
template <> struct c2t<double> { using type = double2; };
template <typename T> using C2 = typename c2t<T>::type;

template <typename T>
__device__ __forceinline__ C2<T> mk(T x, T y) { C2<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ C2<T> conjc(C2<T> a) { return mk<T>(a.x, -a.y); }
// a * (S * i), S = +1 or -1
template <typename T, int S>
__device__ __forceinline__ C2<T> mul_si(C2<T> a) {
  return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// Small DFTs in registers, natural order in and out, sign S of the exponent.
// ---------------------------------------------------------------------------
template <typename T, int S>
__device__ __forceinline__ void dft2(C2<T>* a) {
  C2<T> t = a[0];
  a[0] = cadd<T>(t, a[1]);
  a[1] = csub<T>(t, a[1]);
}

template <typename T, int S>
__device__ __forceinline__ void dft4(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3) {
  C2<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2);
  C2<T> t2 = cadd<T>(a1, a3), t3 = mul_si<T, S>(csub<T>(a1, a3));
  a0 = cadd<T>(t0, t2);
  a2 = csub<T>(t0, t2);
  a1 = cadd<T>(t1, t3);
  a3 = csub<T>(t1, t3);
}

template <typename T, int S>
__device__ __forceinline__ void dft4a(C2<T>* a) { dft4<T, S>(a[0], a[1], a[2], a[3]); }

template <typename T, int S>
__device__ __forceinline__ void dft8(C2<T>* a) {
  // even / odd halves, then w8^k combine
  C2<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  C2<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<T, S>(e0, e1, e2, e3);
  dft4<T, S>(o0, o1, o2, o3);
  const T h = (T)0.70710678118654752440;
  // w^1 = h(1 + S i), w^2 = S i, w^3 = h(-1 + S i)
  C2<T> w1o = mk<T>(h * (o1.x - S * o1.y), h * (o1.y + S * o1.x));
  C2<T> w2o = mul_si<T, S>(o2);
  C2<T> w3o = mk<T>(h * (-o3.x - S * o3.y), h * (-o3.y + S * o3.x));
  a[0] = cadd<T>(e0, o0); a[4] = csub<T>(e0, o0);
  a[1] = cadd<T>(e1, w1o); a[5] = csub<T>(e1, w1o);
  a[2] = cadd<T>(e2, w2o); a[6] = csub<T>(e2, w2o);
  a[3] = cadd<T>(e3, w3o); a[7] = csub<T>(e3, w3o);
}

template <typename T, int S>
__device__ __forceinline__ void dft16(C2<T>* a) {
  C2<T> e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
  dft8<T, S>(e);
  dft8<T, S>(o);
  const T c1 = (T)0.92387953251128675613;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977173;  // sin(pi/8)
  const T h = (T)0.70710678118654752440;
  // w16^k = (cos(k pi/8), S sin(k pi/8))
  const T wr[8] = {(T)1, c1, h, s1, (T)0, -s1, -h, -c1};
  const T wi[8] = {(T)0, s1, h, c1, (T)1, c1, h, s1};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    C2<T> w = mk<T>(wr[k], (T)S * wi[k]);
    C2<T> t = (k == 0) ? o[k] : (k == 4 ? mul_si<T, S>(o[k]) : cmul<T>(w, o[k]));
    a[k] = cadd<T>(e[k], t);
    a[k + 8] = csub<T>(e[k], t);
  }
}

// DFT of length 3: with w = exp(S 2 pi i / 3) = -1/2 + S i sqrt(3)/2,
// X1,2 = x0 - (x1 + x2)/2 +- S i (sqrt(3)/2)(x1 - x2).
template <typename T, int S>
__device__ __forceinline__ void dft3(C2<T>& a0, C2<T>& a1, C2<T>& a2) {
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  const C2<T> t1 = cadd<T>(a1, a2), t2 = csub<T>(a1, a2);
  const C2<T> m = mk<T>(a0.x - (T)0.5 * t1.x, a0.y - (T)0.5 * t1.y);
  const C2<T> r = mul_si<T, S>(cscale<T>(t2, h));
  a0 = cadd<T>(a0, t1);
  a1 = cadd<T>(m, r);
  a2 = csub<T>(m, r);
}

template <typename T, int S>
__device__ __forceinline__ void dft3a(C2<T>* a) { dft3<T, S>(a[0], a[1], a[2]); }

// DFT of length 12 as 3 x 4 (Cooley-Tukey, n = 4 n1 + n2, k = k1 + 3 k2):
// four length-3 DFTs over n1, twiddles w12^(n2 k1), three length-4 DFTs
// over n2.
template <typename T, int S>
__device__ __forceinline__ void dft12(C2<T>* a) {
  C2<T> y[4][3];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = a[n2];
    y[n2][1] = a[4 + n2];
    y[n2][2] = a[8 + n2];
    dft3<T, S>(y[n2][0], y[n2][1], y[n2][2]);
  }
  // w12^e = (cos(pi e / 6), S sin(pi e / 6)) for e = n2 k1 in 1..6
  const T c1 = (T)0.86602540378443864676, s1 = (T)0.5;
  const T wr[7] = {(T)1, c1, s1, (T)0, -s1, -c1, (T)-1};
  const T wi[7] = {(T)0, s1, c1, (T)1, c1, s1, (T)0};
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 3; ++k1) {
      const int e = n2 * k1;
      if (e == 3) y[n2][k1] = mul_si<T, S>(y[n2][k1]);
      else if (e == 6) y[n2][k1] = mk<T>(-y[n2][k1].x, -y[n2][k1].y);
      else y[n2][k1] = cmul<T>(mk<T>(wr[e], (T)S * wi[e]), y[n2][k1]);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    dft4<T, S>(y[0][k1], y[1][k1], y[2][k1], y[3][k1]);
    a[k1] = y[0][k1];
    a[k1 + 3] = y[1][k1];
    a[k1 + 6] = y[2][k1];
    a[k1 + 9] = y[3][k1];
  }
}

template <typename T, int S, int RADIX>
__device__ __forceinline__ void dft_r(C2<T>* a) {
  if constexpr (RADIX == 2) dft2<T, S>(a);
  else if constexpr (RADIX == 3) dft3a<T, S>(a);
  else if constexpr (RADIX == 4) dft4a<T, S>(a);
  else if constexpr (RADIX == 8) dft8<T, S>(a);
  else if constexpr (RADIX == 12) dft12<T, S>(a);
  else if constexpr (RADIX == 16) dft16<T, S>(a);
}

// padded LDS index: one spare element after every 16 (bank spreading)
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_elems(int n) { return n + n / 16; }

template <int TEAM>
__device__ __forceinline__ void team_sync() {
  if constexpr (TEAM <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// Stage plan: radix of the stage with Ns = ns (the largest supported radix
// dividing both the points per lane and the length left to split), and how
// many twiddles one lane needs for all stages (R/r butterflies x (r - 1)
// twiddles per stage with Ns > 1).  The twiddles of a lane are the same for
// every transform it does, so kernels load them once (fft_load_twiddles)
// and keep them in registers.
// maxr (16 or 8) caps the radix: a transform tuned for fewer, cheaper
// stages (16) or for fewer registers per butterfly (8).
constexpr int stage_radix(int n, int team, int ns, int maxr = 16) {
  return maxr >= 16 && cgcd(n / team, n / ns) % 16 == 0   ? 16
         : maxr >= 12 && cgcd(n / team, n / ns) % 12 == 0 ? 12
         : cgcd(n / team, n / ns) % 8 == 0                 ? 8
         : cgcd(n / team, n / ns) % 4 == 0                 ? 4
         : cgcd(n / team, n / ns) % 3 == 0                 ? 3
         : cgcd(n / team, n / ns) % 2 == 0                 ? 2
                                                           : 1;
}

// true when the greedy radices split n completely over a team
constexpr bool fft_plan_ok(int n, int team, int ns = 1, int maxr = 16) {
  return ns == n ? true
                 : (stage_radix(n, team, ns, maxr) < 2
                        ? false
                        : fft_plan_ok(n, team, ns * stage_radix(n, team, ns, maxr), maxr));
}

// supported transform lengths: 2^k or 3 * 2^k
constexpr bool fft_len_ok(int n) {
  return n >= 2 && ((n & (n - 1)) == 0 || (n % 3 == 0 && ((n / 3) & (n / 3 - 1)) == 0));
}

constexpr int fft_tw_count_from(int n, int team, int ns, int maxr) {
  return ns >= n ? 0
                 : (ns > 1 ? (n / team / stage_radix(n, team, ns, maxr)) *
                                 (stage_radix(n, team, ns, maxr) - 1)
                           : 0) +
                       fft_tw_count_from(n, team, ns * stage_radix(n, team, ns, maxr),
                                         maxr);
}

template <int N, int TEAM, int MAXR = 16>
constexpr int fft_tw_count() { return fft_tw_count_from(N, TEAM, 1, MAXR); }

// A lane's twiddles in registers; MAXR is the transform's radix cap.
template <typename T, int N, int TEAM, int MAXR = 16>
struct FftTw {
  static constexpr int kMaxR = MAXR;
  C2<T> w[fft_tw_count<N, TEAM, MAXR>() > 0 ? fft_tw_count<N, TEAM, MAXR>() : 1];
};

template <typename T, int N, int TEAM, int NS, int OFF, int MUL, int MAXR>
__device__ __forceinline__ void fft_tw_stage(FftTw<T, N, TEAM, MAXR>& f,
                                             const C2<T>* __restrict__ tw,
                                             int lane) {
  constexpr int R = N / TEAM;
  constexpr int RAD = stage_radix(N, TEAM, NS, MAXR);
  constexpr bool LAST = (NS * RAD == N);
  constexpr int BPL = R / RAD;
  constexpr int TSTRIDE = N / (NS * RAD);
  if constexpr (NS > 1) {
#pragma unroll
    for (int t = 0; t < BPL; ++t) {
      const int k = (lane + TEAM * t) % NS;
#pragma unroll
      for (int m = 1; m < RAD; ++m)
        f.w[OFF + t * (RAD - 1) + (m - 1)] = tw[m * k * TSTRIDE * MUL];
    }
  }
  if constexpr (!LAST)
    fft_tw_stage<T, N, TEAM, NS * RAD,
                 OFF + (NS > 1 ? BPL * (RAD - 1) : 0), MUL, MAXR>(f, tw, lane);
}

// Fills a lane's twiddles from the table tw[t] = exp(+2 pi i t / (N MUL))
// (MUL > 1: the table of a longer transform, every MUL-th entry used).
template <typename T, int N, int TEAM, int MUL = 1, int MAXR = 16>
__device__ __forceinline__ void fft_load_twiddles(FftTw<T, N, TEAM, MAXR>& f,
                                                  const C2<T>* __restrict__ tw,
                                                  int lane) {
  fft_tw_stage<T, N, TEAM, 1, 0, MUL, MAXR>(f, tw, lane);
}

// Twiddle source reading the N-entry table exp(+2 pi i t/N) from LDS (or any
// memory) at every stage, for kernels whose register budget is tight.
template <typename T, int N, int TEAM, int MAXR = 16>
struct FftTwTable {
  static constexpr int kMaxR = MAXR;
  const C2<T>* tab;
};

template <typename T, int N, int TEAM, int NS, int RAD, int OFF, int MAXR>
__device__ __forceinline__ C2<T> tw_get(const FftTw<T, N, TEAM, MAXR>& f, int t,
                                        int m, int k) {
  (void)k;
  return f.w[OFF + t * (RAD - 1) + (m - 1)];
}

template <typename T, int N, int TEAM, int NS, int RAD, int OFF, int MAXR>
__device__ __forceinline__ C2<T> tw_get(const FftTwTable<T, N, TEAM, MAXR>& f,
                                        int t, int m, int k) {
  (void)t;
  return f.tab[m * k * (N / (NS * RAD))];
}

// One Stockham stage with Ns = NS (twiddles from offset OFF), then the next.
template <typename T, int N, int TEAM, int DIR, int NS, int OFF, class TWS>
__device__ __forceinline__ void fft_stage(C2<T> (&v)[N / TEAM], C2<T>* lds,
                                          const TWS& f, int lane) {
  constexpr int R = N / TEAM;
  constexpr int RAD = stage_radix(N, TEAM, NS, TWS::kMaxR);
  constexpr bool LAST = (NS * RAD == N);
  constexpr int BPL = R / RAD;
#pragma unroll
  for (int t = 0; t < BPL; ++t) {
    const int j = lane + TEAM * t;
    const int k = j % NS;
    C2<T> x[RAD];
#pragma unroll
    for (int m = 0; m < RAD; ++m) x[m] = v[t + m * BPL];
    if constexpr (NS > 1) {
#pragma unroll
      for (int m = 1; m < RAD; ++m) {
        C2<T> w = tw_get<T, N, TEAM, NS, RAD, OFF, TWS::kMaxR>(f, t, m, k);
        if constexpr (DIR < 0) w.y = -w.y;
        x[m] = cmul<T>(x[m], w);
      }
    }
    dft_r<T, DIR, RAD>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < RAD; ++m) v[t + m * BPL] = x[m];
    } else {
      const int base = (j - k) * RAD + k;
#pragma unroll
      for (int m = 0; m < RAD; ++m) lds[lpad(base + m * NS)] = x[m];
    }
  }
  if constexpr (!LAST) {
    team_sync<TEAM>();
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = lds[lpad(lane + TEAM * q)];
    team_sync<TEAM>();
    fft_stage<T, N, TEAM, DIR, NS * RAD, OFF + (NS > 1 ? BPL * (RAD - 1) : 0),
              TWS>(v, lds, f, lane);
  }
}

// In-place unnormalised DFT of length N over a team: DIR = -1 forward
// (exp(-2 pi i jk/N)), +1 inverse.  lds: lds_elems(N) elements private to
// the team; f: the lane's twiddles in registers (FftTw, fft_load_twiddles)
// or the N-entry table (FftTwTable).
template <typename T, int N, int TEAM, int DIR, class TWS>
__device__ __forceinline__ void team_fft(C2<T> (&v)[N / TEAM], C2<T>* lds,
                                         const TWS& f, int lane) {
  static_assert(N % TEAM == 0 && N / TEAM >= 2, "team too large for N");
  static_assert(fft_len_ok(N), "lengths 2^k or 3 * 2^k only");
  static_assert(fft_plan_ok(N, TEAM, 1, TWS::kMaxR),
                "no radix split of N over this team");
  fft_stage<T, N, TEAM, DIR, 1, 0, TWS>(v, lds, f, lane);
}

// Length-P transform over two waves (TEAM = 128, R = P/128 points per
// lane) with a single workgroup barrier: the decimation-in-time split of
// the sequence into even and odd samples.  Wave w (0 or 1) holds x[2n + w]
// at n = l + 64 q (l = lane in the wave, q < R), transforms them at length
// P/2 alone (one-wave Stockham: wave-level barriers only), and one exchange
// through `cross` (2 x P/2 elements, distinct from the buffer of the previous
// call) joins the halves:
//   X[m] = E[m] + W^m O[m],  X[m + P/2] = E[m] - W^m O[m],  W = exp(DIR 2 pi i / P).
// On return wave w holds X[w P/2 + l + 64 q].  wm[q] = exp(+2 pi i m / P) at
// m = l + 64 q; f_half: twiddles of the length-P/2 transform.  Every lane of
// the workgroup must call it (it contains __syncthreads).
template <typename T, int P, int DIR, class TWS>
__device__ __forceinline__ void team2_fft(C2<T> (&v)[P / 128], C2<T>* lds_w,
                                          C2<T>* cross, const TWS& f_half,
                                          const C2<T> (&wm)[P / 128], int wave,
                                          int l) {
  constexpr int R = P / 128;
  team_fft<T, P / 2, 64, DIR>(v, lds_w, f_half, l);
  // the wave index is uniform: one branch per wave instead of per-lane
  // selects between the two halves' formulas
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  C2<T>* mine = cross + wv * (P / 2);
  const C2<T>* other = cross + (1 - wv) * (P / 2);
#pragma unroll
  for (int q = 0; q < R; ++q) mine[l + 64 * q] = v[q];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      C2<T> w = wm[q];
      if constexpr (DIR < 0) w.y = -w.y;
      v[q] = cadd<T>(v[q], cmul<T>(w, other[l + 64 * q]));
    }
  } else {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      C2<T> w = wm[q];
      if constexpr (DIR < 0) w.y = -w.y;
      v[q] = csub<T>(other[l + 64 * q], cmul<T>(w, v[q]));
    }
  }
}

}  // namespace cmif
