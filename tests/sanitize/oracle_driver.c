/* Exercises the C oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (host build): every entry point on small random inputs,
 * ragged and degenerate sizes, masks on and off, label errors, and the
 * NN rotation at several angles.  Any sanitizer report aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_cmif_direct(const uint8_t*, const uint8_t*, int, int, const uint8_t*,
                   const uint8_t*, int, int, int, int, double*, int64_t*,
                   int64_t*, uint64_t*, int);
int or_cmif_at(const uint8_t*, const uint8_t*, int, int, const uint8_t*,
               const uint8_t*, int, int, int, int, int, int, double*, int64_t*,
               int64_t*);
int64_t or_argmax(const double*, const int64_t*, int64_t, double, double*,
                  int64_t*);
void or_rot_coeffs(double, int64_t*, int64_t*);
void or_warp_nn(const uint8_t*, const uint8_t*, int, int, int64_t, int64_t,
                uint8_t*, uint8_t*);
int or_soft_direct(const float*, const uint8_t*, int, int, const float*,
                   const uint8_t*, int, int, int, int, double*, double*,
                   double*, int);
double or_mi_of_joint(const double*, int, int);

static uint64_t st = 88172645463325252ull;
static uint32_t rnd(void) {
  st ^= st << 13; st ^= st >> 7; st ^= st << 17;
  return (uint32_t)st;
}

static uint8_t* labels(int n, int q) {
  uint8_t* a = malloc((size_t)n);
  for (int i = 0; i < n; ++i) a[i] = (uint8_t)(rnd() % (uint32_t)q);
  return a;
}

int main(void) {
  const int sizes[][4] = {{1, 1, 1, 1}, {1, 7, 3, 1}, {5, 4, 6, 9},
                          {13, 11, 2, 17}, {9, 9, 9, 9}, {20, 3, 4, 21}};
  for (int s = 0; s < 6; ++s) {
    const int ha = sizes[s][0], wa = sizes[s][1], hb = sizes[s][2], wb = sizes[s][3];
    for (int q = 1; q <= 5; q += 2) {
      uint8_t* A = labels(ha * wa, q);
      uint8_t* B = labels(hb * wb, q + 1);
      uint8_t* MA = labels(ha * wa, 2);
      uint8_t* MB = labels(hb * wb, 2);
      const int sh = ha + hb - 1, sw = wa + wb - 1;
      double* mi = malloc(sizeof(double) * sh * sw);
      int64_t* n = malloc(sizeof(int64_t) * sh * sw);
      int64_t* cnt = malloc(sizeof(int64_t) * sh * sw * q * (q + 1));
      uint64_t* dig = malloc(sizeof(uint64_t) * q * (q + 1));
      for (int m = 0; m < 2; ++m) {
        if (or_cmif_direct(A, m ? MA : NULL, ha, wa, B, m ? MB : NULL, hb, wb, q,
                           q + 1, mi, n, cnt, dig, 2) != 0)
          return 1;
        double bm;
        int64_t bn;
        (void)or_argmax(mi, n, (int64_t)sh * sw, 0.5, &bm, &bn);
        double v;
        int64_t nn;
        int64_t joint[64];
        if (or_cmif_at(A, MA, ha, wa, B, MB, hb, wb, q, q + 1, hb - 1, -(wa - 1),
                       &v, &nn, joint) != 0)
          return 2;
      }
      /* a label out of range inside the mask is an error, not a write */
      A[0] = (uint8_t)q;
      if (or_cmif_direct(A, NULL, ha, wa, B, NULL, hb, wb, q, q + 1, mi, n, NULL,
                         NULL, 1) == 0)
        return 3;
      uint8_t* ob = malloc((size_t)hb * wb);
      uint8_t* om = malloc((size_t)hb * wb);
      for (int k = 0; k < 8; ++k) {
        int64_t c, sn;
        or_rot_coeffs(-3.0 + 0.9 * k, &c, &sn);
        or_warp_nn(B, MB, hb, wb, c, sn, ob, om);
      }
      float* pa = malloc(sizeof(float) * q * ha * wa);
      float* pb = malloc(sizeof(float) * (q + 1) * hb * wb);
      for (int i = 0; i < q * ha * wa; ++i) pa[i] = (float)(rnd() % 1000) / 999.0f;
      for (int i = 0; i < (q + 1) * hb * wb; ++i) pb[i] = (float)(rnd() % 1000) / 999.0f;
      double* nr = malloc(sizeof(double) * sh * sw);
      double* jo = malloc(sizeof(double) * sh * sw * q * (q + 1));
      if (or_soft_direct(pa, MA, ha, wa, pb, MB, hb, wb, q, q + 1, mi, nr, jo, 2) != 0)
        return 4;
      double jt[6] = {0, 1, 2, 3, 0, 5};
      if (!isfinite(or_mi_of_joint(jt, 2, 3))) return 5;
      free(A); free(B); free(MA); free(MB); free(mi); free(n); free(cnt);
      free(dig); free(ob); free(om); free(pa); free(pb); free(nr); free(jo);
    }
  }
  puts("oracle sanitizer driver ok");
  return 0;
}
