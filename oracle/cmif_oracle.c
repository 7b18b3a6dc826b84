/*
 * CPU oracle for the cross-mutual-information function (CMIF).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or table with the GPU library, and the GPU library never calls it.
 *
 * What it computes is the plain definition, by the direct method the paper
 * describes in Sec. 2.2: for every displacement chi considered on its own,
 * walk the overlap of A and the displaced B, increment the joint histogram
 * bin of each pair of labels found where both masks are set, then form the
 * relative histograms and the entropies.
 *
 *   Eq. 1-4  I(A,B) = H_A + H_B - H_AB, entropies in bits over the overlap.
 *   Eq. 5    CMIF(chi; A, B) = I(A, T_chi[B]),  T_chi[B](x) = B(x + chi).
 *   Eq. 7    the pairing A(x) <-> B(x + chi) (cross-correlation sign).
 *   Eq. 11   N(chi) = number of points where both masks are set.
 *   Eq. 12   H_A(chi) = -sum_a (C_a/N) log2 (C_a/N), likewise H_B, H_AB;
 *            0/0 = 0 and 0 log 0 = 0; MI = 0 where N = 0.
 *   Alg. 1   per transform: threshold gamma * max N, argmax of CMIF over the
 *            displacements whose N reaches it; across transforms a strictly
 *            larger value replaces the current best.
 *   Sec. 3.3 / Sec. 3.6: the soft variant weights each point by real-valued
 *            memberships (spatially weighted MI generalised to per-label
 *            weights); nearest-neighbour warping of the categorical image.
 *
 * Readings taken where the paper is silent (stated again beside the code):
 *   - displacement set: every chi whose rectangles overlap at all,
 *     chi_y in [-(H_A-1), H_B-1], chi_x in [-(W_A-1), W_B-1]; map index
 *     [i][j] <-> chi = (i - (H_A-1), j - (W_A-1));
 *   - marginals are overlap-restricted (Eq. 12 governs);
 *   - ties inside one transform: smallest row-major map index;
 *   - NN rotation: fixed-point rule (c, s = round(cos, sin * 2^16)), doubled
 *     centred coordinates, round half up, points whose source falls outside
 *     B or on M_B = 0 get M' = 0.
 *
 * parity pinned by: brute-force enumeration, scipy correlate2d of indicator
 * images, numpy FFT + rint, sklearn mutual_info_score, closed-form N for
 * all-ones masks, invariants (tests/test_oracle_pins.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_LABEL 2

/* Vigna's splitmix64 output function, applied to a counter (order-free
 * digest weights). */
static uint64_t or_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t or_digest_weight(uint64_t idx) { return or_splitmix64(idx); }

int or_version(void) { return 1; }

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Entropy term of Eq. 12: -(c/n) log2(c/n), with 0 log 0 = 0. */
static double or_hterm(double c, double n) {
  if (c <= 0.0) return 0.0;
  double p = c / n;
  return -p * log2(p);
}

/* Eq. 2 with Eq. 12: MI from a joint table of counts (or weights).
 * joint is [qa][qb]; returns 0 when the total is 0 (0/0 = 0). */
static double or_mi_from_joint(const double* joint, int qa, int qb,
                               double* n_out) {
  double n = 0.0;
  for (int i = 0; i < qa * qb; ++i) n += joint[i];
  if (n_out) *n_out = n;
  if (n <= 0.0) return 0.0;
  double ha = 0.0, hb = 0.0, hab = 0.0;
  for (int a = 0; a < qa; ++a) {
    double ca = 0.0;
    for (int b = 0; b < qb; ++b) ca += joint[a * qb + b];
    ha += or_hterm(ca, n);
  }
  for (int b = 0; b < qb; ++b) {
    double cb = 0.0;
    for (int a = 0; a < qa; ++a) cb += joint[a * qb + b];
    hb += or_hterm(cb, n);
  }
  for (int i = 0; i < qa * qb; ++i) hab += or_hterm(joint[i], n);
  return ha + hb - hab;
}

/* Label range check: inside the mask every label must be < q. */
static int or_check_labels(const uint8_t* lab, const uint8_t* msk, int h,
                           int w, int q) {
  for (int i = 0; i < h * w; ++i)
    if ((msk == NULL || msk[i]) && lab[i] >= q) return OR_ERR_LABEL;
  return OR_OK;
}

/*
 * Joint histogram at one displacement (direct method, Sec. 2.2): pairs
 * A(y, x) with B(y + dy, x + dx) wherever both lie inside their images and
 * both masks are set.  joint is [qa][qb] int64, zeroed here.
 */
static void or_joint_at(const uint8_t* A, const uint8_t* MA, int ha, int wa,
                        const uint8_t* B, const uint8_t* MB, int hb, int wb,
                        int qa, int qb, int dy, int dx, int64_t* joint) {
  memset(joint, 0, sizeof(int64_t) * (size_t)qa * qb);
  int y0 = dy < 0 ? -dy : 0;
  int y1 = ha < hb - dy ? ha : hb - dy;
  int x0 = dx < 0 ? -dx : 0;
  int x1 = wa < wb - dx ? wa : wb - dx;
  for (int y = y0; y < y1; ++y) {
    const uint8_t* ar = A + (size_t)y * wa;
    const uint8_t* mar = MA ? MA + (size_t)y * wa : NULL;
    const uint8_t* br = B + (size_t)(y + dy) * wb + dx;
    const uint8_t* mbr = MB ? MB + (size_t)(y + dy) * wb + dx : NULL;
    for (int x = x0; x < x1; ++x) {
      if (mar && !mar[x]) continue;
      if (mbr && !mbr[x]) continue;
      joint[(size_t)ar[x] * qb + br[x]] += 1;
    }
  }
}

/*
 * CMIF at one displacement chi = (dy, dx).  Writes MI (bits), N and, when
 * joint_out is non-NULL, the [qa][qb] joint counts.
 */
int or_cmif_at(const uint8_t* A, const uint8_t* MA, int ha, int wa,
               const uint8_t* B, const uint8_t* MB, int hb, int wb, int qa,
               int qb, int dy, int dx, double* mi, int64_t* n,
               int64_t* joint_out) {
  if (qa < 1 || qb < 1 || qa > 256 || qb > 256) return OR_ERR_ARG;
  if (or_check_labels(A, MA, ha, wa, qa) || or_check_labels(B, MB, hb, wb, qb))
    return OR_ERR_LABEL;
  int64_t* joint = (int64_t*)malloc(sizeof(int64_t) * (size_t)qa * qb);
  double* jd = (double*)malloc(sizeof(double) * (size_t)qa * qb);
  or_joint_at(A, MA, ha, wa, B, MB, hb, wb, qa, qb, dy, dx, joint);
  for (int i = 0; i < qa * qb; ++i) jd[i] = (double)joint[i];
  double nn;
  double v = or_mi_from_joint(jd, qa, qb, &nn);
  if (mi) *mi = v;
  if (n) *n = (int64_t)nn;
  if (joint_out) memcpy(joint_out, joint, sizeof(int64_t) * (size_t)qa * qb);
  free(joint);
  free(jd);
  return OR_OK;
}

/*
 * Full CMIF map over every displacement with a non-empty rectangle overlap.
 *   mi      [SH][SW] double or NULL
 *   n       [SH][SW] int64 or NULL
 *   counts  [qa][qb][SH][SW] int64 or NULL
 *   digest  [qa][qb] uint64 or NULL: sum over chi of count * w(idx(chi)),
 *           modulo 2^64, with w the splitmix64 output of the row-major map
 *           index (an order-free fingerprint of the whole count array).
 * SH = ha + hb - 1, SW = wa + wb - 1.  MA/MB may be NULL (all ones).
 */
int or_cmif_direct(const uint8_t* A, const uint8_t* MA, int ha, int wa,
                   const uint8_t* B, const uint8_t* MB, int hb, int wb, int qa,
                   int qb, double* mi, int64_t* n, int64_t* counts,
                   uint64_t* digest, int nthreads) {
  if (ha < 1 || wa < 1 || hb < 1 || wb < 1) return OR_ERR_ARG;
  if (qa < 1 || qb < 1 || qa > 256 || qb > 256) return OR_ERR_ARG;
  if (or_check_labels(A, MA, ha, wa, qa) || or_check_labels(B, MB, hb, wb, qb))
    return OR_ERR_LABEL;
  const int sh = ha + hb - 1, sw = wa + wb - 1;
  const size_t npix = (size_t)sh * sw;
  const int nq = qa * qb;
  uint64_t* dig_all = NULL;
  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  if (digest) dig_all = (uint64_t*)calloc((size_t)nt * nq, sizeof(uint64_t));

#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int64_t* joint = (int64_t*)malloc(sizeof(int64_t) * nq);
    double* jd = (double*)malloc(sizeof(double) * nq);
    uint64_t* dig = dig_all ? dig_all + (size_t)tid * nq : NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int i = 0; i < sh; ++i) {
      int dy = i - (ha - 1);
      for (int j = 0; j < sw; ++j) {
        int dx = j - (wa - 1);
        or_joint_at(A, MA, ha, wa, B, MB, hb, wb, qa, qb, dy, dx, joint);
        size_t idx = (size_t)i * sw + j;
        for (int k = 0; k < nq; ++k) jd[k] = (double)joint[k];
        double nn;
        double v = or_mi_from_joint(jd, qa, qb, &nn);
        if (mi) mi[idx] = v;
        if (n) n[idx] = (int64_t)nn;
        if (counts)
          for (int k = 0; k < nq; ++k) counts[(size_t)k * npix + idx] = joint[k];
        if (dig) {
          uint64_t wgt = or_splitmix64((uint64_t)idx);
          for (int k = 0; k < nq; ++k) dig[k] += (uint64_t)joint[k] * wgt;
        }
      }
    }
    free(joint);
    free(jd);
  }
  if (digest) {
    for (int k = 0; k < nq; ++k) {
      uint64_t s = 0;
      for (int t = 0; t < nt; ++t) s += dig_all[(size_t)t * nq + k];
      digest[k] = s;
    }
    free(dig_all);
  }
  return OR_OK;
}

/*
 * Alg. 1, one transform: max of N over the map, threshold gamma * maxN
 * (compared in FP64), argmax of MI over the eligible displacements; ties go
 * to the smallest row-major index.  Returns the index, or -1 for an empty
 * map.
 */
int64_t or_argmax(const double* mi, const int64_t* n, int64_t npix,
                  double gamma, double* best_mi, int64_t* best_n) {
  int64_t maxn = 0;
  for (int64_t i = 0; i < npix; ++i)
    if (n[i] > maxn) maxn = n[i];
  double thr = gamma * (double)maxn;
  int64_t best = -1;
  double bv = 0.0;
  for (int64_t i = 0; i < npix; ++i) {
    if ((double)n[i] >= thr) {
      if (best < 0 || mi[i] > bv) {
        best = i;
        bv = mi[i];
      }
    }
  }
  if (best_mi) *best_mi = best >= 0 ? bv : 0.0;
  if (best_n) *best_n = best >= 0 ? n[best] : 0;
  return best;
}

/* Fixed-point rotation coefficients: round(cos, sin * 2^16). */
void or_rot_coeffs(double theta, int64_t* c, int64_t* s) {
  *c = llround(cos(theta) * 65536.0);
  *s = llround(sin(theta) * 65536.0);
}

static int64_t or_floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

/*
 * Nearest-neighbour rotation of B and its mask about B's centre (Sec. 3.6:
 * NN interpolation keeps labels categorical).  Output (y, x) reads B at the
 * source point obtained by rotating the doubled centred coordinates
 * (2x-(W-1), 2y-(H-1)) with the fixed-point matrix [[c, -s], [s, c]] and
 * rounding half up; a source outside B or on M_B = 0 gives M' = 0, B' = 0.
 * MB may be NULL (all ones).
 */
void or_warp_nn(const uint8_t* B, const uint8_t* MB, int h, int w, int64_t c,
                int64_t s, uint8_t* outB, uint8_t* outM) {
  const int64_t one = 65536;
  for (int y = 0; y < h; ++y) {
    for (int x = 0; x < w; ++x) {
      int64_t X = 2 * (int64_t)x - (w - 1);
      int64_t Y = 2 * (int64_t)y - (h - 1);
      int64_t xs2 = c * X - s * Y;
      int64_t ys2 = s * X + c * Y;
      int64_t xs = or_floordiv(xs2 + (int64_t)(w - 1) * one + one, 2 * one);
      int64_t ys = or_floordiv(ys2 + (int64_t)(h - 1) * one + one, 2 * one);
      size_t o = (size_t)y * w + x;
      if (xs >= 0 && xs < w && ys >= 0 && ys < h &&
          (MB == NULL || MB[(size_t)ys * w + xs])) {
        outB[o] = B[(size_t)ys * w + xs];
        outM[o] = 1;
      } else {
        outB[o] = 0;
        outM[o] = 0;
      }
    }
  }
}

/*
 * Soft CMIF, direct method in FP64: joint weight
 *   J_ab(chi) = sum_x M_A(x) p_a(x) M_B(x+chi) q_b(x+chi),
 * marginals and N taken as sums of J, MI by Eq. 2 / Eq. 12 with real
 * weights.  pa is [qa][ha][wa], pb is [qb][hb][wb] (float32 memberships).
 * joint_out, when non-NULL, is [qa][qb][SH][SW] double.
 */
int or_soft_direct(const float* pa, const uint8_t* MA, int ha, int wa,
                   const float* pb, const uint8_t* MB, int hb, int wb, int qa,
                   int qb, double* mi, double* n, double* joint_out,
                   int nthreads) {
  if (ha < 1 || wa < 1 || hb < 1 || wb < 1 || qa < 1 || qb < 1)
    return OR_ERR_ARG;
  const int sh = ha + hb - 1, sw = wa + wb - 1;
  const size_t npix = (size_t)sh * sw;
  const int nq = qa * qb;
  const size_t plane_a = (size_t)ha * wa, plane_b = (size_t)hb * wb;
  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    double* jd = (double*)malloc(sizeof(double) * nq);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int i = 0; i < sh; ++i) {
      int dy = i - (ha - 1);
      for (int j = 0; j < sw; ++j) {
        int dx = j - (wa - 1);
        for (int k = 0; k < nq; ++k) jd[k] = 0.0;
        int y0 = dy < 0 ? -dy : 0;
        int y1 = ha < hb - dy ? ha : hb - dy;
        int x0 = dx < 0 ? -dx : 0;
        int x1 = wa < wb - dx ? wa : wb - dx;
        for (int y = y0; y < y1; ++y) {
          for (int x = x0; x < x1; ++x) {
            size_t ia = (size_t)y * wa + x;
            size_t ib = (size_t)(y + dy) * wb + (x + dx);
            if (MA && !MA[ia]) continue;
            if (MB && !MB[ib]) continue;
            for (int a = 0; a < qa; ++a) {
              double va = (double)pa[a * plane_a + ia];
              for (int b = 0; b < qb; ++b)
                jd[a * qb + b] += va * (double)pb[b * plane_b + ib];
            }
          }
        }
        size_t idx = (size_t)i * sw + j;
        double nn;
        double v = or_mi_from_joint(jd, qa, qb, &nn);
        if (mi) mi[idx] = v;
        if (n) n[idx] = nn;
        if (joint_out)
          for (int k = 0; k < nq; ++k) joint_out[(size_t)k * npix + idx] = jd[k];
      }
    }
    free(jd);
  }
  return OR_OK;
}

/* MI (Eq. 2 / Eq. 12) of one explicit joint table of real weights. */
double or_mi_of_joint(const double* joint, int qa, int qb) {
  return or_mi_from_joint(joint, qa, qb, NULL);
}

/*
 * 3-D CMIF by the direct method (the nD generalisation of Sec. 2.2 that the
 * paper's discussion states): volumes A [da][ha][wa] and B [db][hb][wb]
 * (row-major, z slowest), masks optional.  For every displacement
 * chi = (dz, dy, dx) with a non-empty box overlap, dz in [-(da-1), db-1]
 * and likewise for y and x, the joint histogram pairs A(z, y, x) with
 * B(z + dz, y + dy, x + dx) where both masks are set; MI by Eq. 2 / Eq. 12.
 * Map index [k][i][j] <-> chi = (k - (da-1), i - (ha-1), j - (wa-1)).
 * digest[a][b] = sum over the map of count * splitmix64(flat map index).
 */
int or_cmif_direct3d(const uint8_t* A, const uint8_t* MA, int da, int ha,
                     int wa, const uint8_t* B, const uint8_t* MB, int db,
                     int hb, int wb, int qa, int qb, double* mi, int64_t* n,
                     uint64_t* digest, int nthreads) {
  if (da < 1 || ha < 1 || wa < 1 || db < 1 || hb < 1 || wb < 1) return OR_ERR_ARG;
  if (qa < 1 || qb < 1 || qa > 256 || qb > 256) return OR_ERR_ARG;
  if (or_check_labels(A, MA, da * ha, wa, qa) ||
      or_check_labels(B, MB, db * hb, wb, qb))
    return OR_ERR_LABEL;
  const int sd = da + db - 1, sh = ha + hb - 1, sw = wa + wb - 1;
  const int nq = qa * qb;
  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  uint64_t* dig_all = digest ? (uint64_t*)calloc((size_t)nt * nq, sizeof(uint64_t)) : NULL;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int64_t* joint = (int64_t*)malloc(sizeof(int64_t) * nq);
    int64_t* jt = (int64_t*)malloc(sizeof(int64_t) * nq);
    double* jd = (double*)malloc(sizeof(double) * nq);
    uint64_t* dig = dig_all ? dig_all + (size_t)tid * nq : NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int kk = 0; kk < sd * sh; ++kk) {
      const int k = kk / sh, i = kk % sh;
      const int dz = k - (da - 1), dy = i - (ha - 1);
      const int z0 = dz < 0 ? -dz : 0, z1 = da < db - dz ? da : db - dz;
      for (int j = 0; j < sw; ++j) {
        const int dx = j - (wa - 1);
        memset(joint, 0, sizeof(int64_t) * nq);
        for (int z = z0; z < z1; ++z) {
          /* one slice pair: the 2-D overlap walk of or_joint_at */
          const uint8_t* As = A + (size_t)z * ha * wa;
          const uint8_t* MAs = MA ? MA + (size_t)z * ha * wa : NULL;
          const uint8_t* Bs = B + (size_t)(z + dz) * hb * wb;
          const uint8_t* MBs = MB ? MB + (size_t)(z + dz) * hb * wb : NULL;
          or_joint_at(As, MAs, ha, wa, Bs, MBs, hb, wb, qa, qb, dy, dx, jt);
          for (int q = 0; q < nq; ++q) joint[q] += jt[q];
        }
        const size_t idx = ((size_t)k * sh + i) * sw + j;
        for (int q = 0; q < nq; ++q) jd[q] = (double)joint[q];
        double nn;
        const double v = or_mi_from_joint(jd, qa, qb, &nn);
        if (mi) mi[idx] = v;
        if (n) n[idx] = (int64_t)nn;
        if (dig) {
          const uint64_t wgt = or_splitmix64((uint64_t)idx);
          for (int q = 0; q < nq; ++q) dig[q] += (uint64_t)joint[q] * wgt;
        }
      }
    }
    free(joint);
    free(jt);
    free(jd);
  }
  if (digest) {
    for (int q = 0; q < nq; ++q) {
      uint64_t s = 0;
      for (int t = 0; t < nt; ++t) s += dig_all[(size_t)t * nq + q];
      digest[q] = s;
    }
    free(dig_all);
  }
  return OR_OK;
}
