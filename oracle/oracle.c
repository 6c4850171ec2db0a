/*
 * FP64 CPU oracle for the block-floating-point FFT / range-Doppler SAR path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the GPU
 * path (no headers, tables or helpers).
 *
 * What it computes is the plain mathematical definition of each operation
 * (paper, Sec. III-B "The overflow mechanism" and Eq. (1) in Sec. IV-A):
 *
 *   forward   X[k] = sum_n x[n] exp(-2 pi i n k / N)              (unscaled)
 *   inverse   IDFT(Z)[n] = (1/N) sum_k Z[k] exp(+2 pi i n k / N)
 *             realised as conj(FFT(conj(Z))) / N, the conj-FFT-conj form
 *             the paper uses to reuse the forward butterfly;
 *   compress  y = IDFT(FFT(x) . H) per row (matched filtering);
 *   SAR       image = A_az( transpose( A_r(echo) ) ), A(v) = IDFT(DFT(v) H).
 *
 * The block-floating-point shift of Eq. (1) is a mathematical no-op (the
 * paper states the 1/N factor commutes with the transform), so the oracle has
 * no BFP step: it evaluates the exact linear map in double precision.
 *
 * The FFT is a textbook recursive radix-2 decimation-in-time transform; the
 * direct O(N^2) DFT is provided so the FFT can be pinned against brute force.
 * Roots of unity are evaluated in FP64 with exact integer argument reduction
 * (never by recurrence; Sec. III-A attributes the "42 dB" folklore to
 * recurrence-built tables).
 *
 * Layout: interleaved complex doubles (re, im), rows contiguous, row-major.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double re, im;
} cplx;

/* exp(-2 pi i k / n) for integer k, n > 0, with the argument reduced exactly
 * in integers to the first octant before any floating-point operation.
 * Symmetry makes k = 0, n/4, n/2, 3n/4 exact (1, -i, -1, +i). */
static cplx root_of_unity(long long k, long long n) {
  long long m = k % n;
  if (m < 0) m += n;
  /* angle = 2 pi m / n = 2 pi A / (8 n) with A = 8 m in [0, 8n) */
  long long a = 8 * m, full = 8 * n;
  double sgn_s = 1.0, sgn_c = 1.0;
  int swap = 0;
  if (2 * a > full) { a = full - a; sgn_s = -1.0; }          /* 2pi - t   */
  if (4 * a > full) { a = full / 2 - a; sgn_c = -1.0; }      /* pi - t    */
  if (8 * a > full) { a = full / 4 - a; swap = 1; }          /* pi/2 - t  */
  /* now t = 2 pi a / (8 n) in [0, pi/4] */
  double t = (2.0 * M_PI * (double)a) / (double)full;
  double c = cos(t), s = sin(t);
  if (a == 0) { c = 1.0; s = 0.0; }
  if (swap) { double tmp = c; c = s; s = tmp; }
  c *= sgn_c;
  s *= sgn_s;
  cplx w = {c, -s}; /* exp(-i angle) */
  return w;
}

static inline cplx cmul(cplx a, cplx b) {
  cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  return r;
}

/* Recursive radix-2 DIT: X = DFT_n of the strided sequence x[0], x[s], ...
 * tw[j] = exp(-2 pi i j / n_top) for j < n_top/2; a sub-transform of size n
 * uses tw[k * (n_top / n)].  scratch holds n elements. */
static void fft_rec(const cplx *x, long s, cplx *X, long n, const cplx *tw,
                    long n_top, cplx *scratch) {
  if (n == 1) {
    X[0] = x[0];
    return;
  }
  long h = n / 2;
  cplx *E = scratch, *O = scratch + h;
  /* E = FFT(even samples), O = FFT(odd samples); X is free as scratch here */
  fft_rec(x, 2 * s, E, h, tw, n_top, X);
  fft_rec(x + s, 2 * s, O, h, tw, n_top, X + h);
  long step = n_top / n;
  for (long k = 0; k < h; ++k) {
    cplx t = cmul(tw[k * step], O[k]);
    cplx e = E[k];
    X[k].re = e.re + t.re;
    X[k].im = e.im + t.im;
    X[k + h].re = e.re - t.re;
    X[k + h].im = e.im - t.im;
  }
}

static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

static cplx *make_table(long n) {
  long h = n / 2 > 0 ? n / 2 : 1;
  cplx *tw = (cplx *)malloc(sizeof(cplx) * h);
  for (long j = 0; j < h; ++j) tw[j] = root_of_unity(j, n);
  return tw;
}

/* One forward transform of length n (power of two). */
static void fft_one(const cplx *x, cplx *X, long n, const cplx *tw) {
  cplx *scratch = (cplx *)malloc(sizeof(cplx) * n);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * n);
  /* scratch layout requirement: the recursion writes X as scratch for the
   * children, so stage through tmp when x and X alias */
  fft_rec(x, 1, tmp, n, tw, n, scratch);
  memcpy(X, tmp, sizeof(cplx) * n);
  free(tmp);
  free(scratch);
}

/* IDFT(Z) = conj(FFT(conj Z)) / N */
static void ifft_one(const cplx *Z, cplx *z, long n, const cplx *tw) {
  cplx *c = (cplx *)malloc(sizeof(cplx) * n);
  for (long i = 0; i < n; ++i) { c[i].re = Z[i].re; c[i].im = -Z[i].im; }
  fft_one(c, c, n, tw);
  double inv = 1.0 / (double)n;
  for (long i = 0; i < n; ++i) { z[i].re = c[i].re * inv; z[i].im = -c[i].im * inv; }
  free(c);
}

/* ---------------------------------------------------------------- API --- */

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* rows independent transforms of length n; inverse != 0 gives the
 * normalised IDFT.  in and out may alias.  Returns 0, or -1 for bad n. */
int oracle_fft_rows(const double *in, double *out, long rows, long n, int inverse) {
  if (!is_pow2(n)) return -1;
  cplx *tw = make_table(n);
#pragma omp parallel for schedule(static)
  for (long r = 0; r < rows; ++r) {
    const cplx *x = (const cplx *)in + r * n;
    cplx *X = (cplx *)out + r * n;
    if (inverse) ifft_one(x, X, n, tw); else fft_one(x, X, n, tw);
  }
  free(tw);
  return 0;
}

/* Direct O(N^2) DFT of one vector of any length n >= 1 (brute force). */
int oracle_dft_direct(const double *in, double *out, long n, int inverse) {
  if (n < 1) return -1;
  const cplx *x = (const cplx *)in;
  cplx *X = (cplx *)malloc(sizeof(cplx) * n);
  for (long k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (long j = 0; j < n; ++j) {
      cplx w = root_of_unity((j * k) % n, n);
      if (inverse) w.im = -w.im;
      sr += x[j].re * w.re - x[j].im * w.im;
      si += x[j].re * w.im + x[j].im * w.re;
    }
    if (inverse) { sr /= (double)n; si /= (double)n; }
    X[k].re = sr;
    X[k].im = si;
  }
  memcpy(out, X, sizeof(cplx) * n);
  free(X);
  return 0;
}

/* exp(-2 pi i k / n) as seen by the oracle (exposed for tests). */
void oracle_root(long long k, long long n, double *re, double *im) {
  cplx w = root_of_unity(k, n);
  *re = w.re;
  *im = w.im;
}

/* Matched filter from a replica h of length len (len <= n), zero-padded:
 * H = conj(DFT_n(h)) / max_k |DFT_n(h)|, so |H| <= 1 (Sec. III-B). */
int oracle_matched_filter(const double *h, long len, long n, double *H) {
  if (!is_pow2(n) || len < 1 || len > n) return -1;
  cplx *x = (cplx *)calloc(n, sizeof(cplx));
  memcpy(x, h, sizeof(cplx) * len);
  cplx *tw = make_table(n);
  fft_one(x, x, n, tw);
  double m = 0.0;
  for (long k = 0; k < n; ++k) {
    double a = hypot(x[k].re, x[k].im);
    if (a > m) m = a;
  }
  cplx *Ho = (cplx *)H;
  for (long k = 0; k < n; ++k) {
    Ho[k].re = x[k].re / m;
    Ho[k].im = -x[k].im / m;
  }
  free(tw);
  free(x);
  return 0;
}

/* y = IDFT(DFT(x) . H) per row; H has n entries and is shared by all rows.
 * conj_filter != 0 uses conj(H) (the adjoint of the same chain). */
int oracle_compress_rows(const double *in, double *out, const double *H, long rows,
                         long n, int conj_filter) {
  if (!is_pow2(n)) return -1;
  cplx *tw = make_table(n);
  const cplx *Hc = (const cplx *)H;
#pragma omp parallel
  {
    cplx *buf = (cplx *)malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
    for (long r = 0; r < rows; ++r) {
      const cplx *x = (const cplx *)in + r * n;
      fft_one(x, buf, n, tw);
      for (long k = 0; k < n; ++k) {
        cplx hk = Hc[k];
        if (conj_filter) hk.im = -hk.im;
        buf[k] = cmul(buf[k], hk);
      }
      ifft_one(buf, (cplx *)out + r * n, n, tw);
    }
    free(buf);
  }
  free(tw);
  return 0;
}

/* out[c][r] = in[r][c]; in is rows x cols. */
void oracle_transpose(const double *in, double *out, long rows, long cols) {
  const cplx *a = (const cplx *)in;
  cplx *b = (cplx *)out;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < cols; ++c)
    for (long r = 0; r < rows; ++r) b[c * rows + r] = a[r * cols + c];
}

/* Per-pulse phase correction of range-compressed data laid out
 * [range][pulse]: z[r][m] = rc_t[r][m] * exp(i phi[m]). */
void oracle_apply_phase(const double *rc_t, double *z, const double *phi,
                        long n_range, long n_pulse) {
#pragma omp parallel for schedule(static)
  for (long r = 0; r < n_range; ++r) {
    for (long m = 0; m < n_pulse; ++m) {
      cplx e = {cos(phi[m]), sin(phi[m])};
      cplx v = ((const cplx *)rc_t)[r * n_pulse + m];
      ((cplx *)z)[r * n_pulse + m] = cmul(v, e);
    }
  }
}

/* Range-Doppler image of an echo laid out [pulse][range]:
 *   rc   = A_r(echo)            rows = pulses, length n_range
 *   rc_t = transpose(rc)        [range][pulse]
 *   z    = rc_t . exp(i phi_m)  (skipped when phi == NULL)
 *   img  = A_az(z)              rows = range bins, length n_pulse
 * rc_t_out (optional) receives rc_t.  img is [range][azimuth]. */
int oracle_sar_image(const double *echo, long n_pulse, long n_range, const double *Hr,
                     const double *Ha, const double *phi, double *img, double *rc_t_out) {
  if (!is_pow2(n_pulse) || !is_pow2(n_range)) return -1;
  size_t tot = (size_t)n_pulse * (size_t)n_range * 2;
  double *rc = (double *)malloc(sizeof(double) * tot);
  double *rct = (double *)malloc(sizeof(double) * tot);
  oracle_compress_rows(echo, rc, Hr, n_pulse, n_range, 0);
  oracle_transpose(rc, rct, n_pulse, n_range);
  if (rc_t_out) memcpy(rc_t_out, rct, sizeof(double) * tot);
  if (phi) oracle_apply_phase(rct, rct, phi, n_range, n_pulse);
  oracle_compress_rows(rct, img, Ha, n_range, n_pulse, 0);
  free(rc);
  free(rct);
  return 0;
}

/* Image entropy E = -sum p ln p, p = |I|^2 / S, S = sum |I|^2 (0 ln 0 = 0).
 * grad (optional) receives dE/dRe I + i dE/dIm I = -(2/S)(ln p + E) I. */
double oracle_entropy(const double *img, long count, double *grad) {
  const cplx *I = (const cplx *)img;
  double S = 0.0;
  for (long i = 0; i < count; ++i) S += I[i].re * I[i].re + I[i].im * I[i].im;
  double E = 0.0;
  for (long i = 0; i < count; ++i) {
    double p = (I[i].re * I[i].re + I[i].im * I[i].im) / S;
    if (p > 0.0) E -= p * log(p);
  }
  if (grad) {
    cplx *G = (cplx *)grad;
    for (long i = 0; i < count; ++i) {
      double p = (I[i].re * I[i].re + I[i].im * I[i].im) / S;
      double f = p > 0.0 ? -(2.0 / S) * (log(p) + E) : 0.0;
      G[i].re = f * I[i].re;
      G[i].im = f * I[i].im;
    }
  }
  return E;
}

/* Autofocus objective and its analytic gradient with respect to the
 * per-pulse phase vector phi (length n_pulse), for range-compressed data
 * rc_t laid out [range][pulse]:
 *   z = rc_t . exp(i phi_m),  I = A_az(z),  E = entropy(I)
 *   G_I = dE/dI (real-pair gradient), G_z = A_az^H(G_I) (same chain with
 *   conj(H_a)),  g_m = sum_r Im(G_z[r][m] conj(z[r][m])).
 * img_out (optional) receives I.  Returns E. */
double oracle_autofocus(const double *rc_t, long n_range, long n_pulse, const double *Ha,
                        const double *phi, double *g, double *img_out) {
  size_t tot = (size_t)n_range * (size_t)n_pulse * 2;
  double *z = (double *)malloc(sizeof(double) * tot);
  double *I = (double *)malloc(sizeof(double) * tot);
  double *G = (double *)malloc(sizeof(double) * tot);
  oracle_apply_phase(rc_t, z, phi, n_range, n_pulse);
  oracle_compress_rows(z, I, Ha, n_range, n_pulse, 0);
  double E = oracle_entropy(I, n_range * n_pulse, g ? G : NULL);
  if (g) {
    oracle_compress_rows(G, G, Ha, n_range, n_pulse, 1);
    const cplx *Gz = (const cplx *)G, *zc = (const cplx *)z;
    for (long m = 0; m < n_pulse; ++m) g[m] = 0.0;
    for (long r = 0; r < n_range; ++r)
      for (long m = 0; m < n_pulse; ++m) {
        cplx a = Gz[r * n_pulse + m], b = zc[r * n_pulse + m];
        /* Im(a * conj(b)) */
        g[m] += a.im * b.re - a.re * b.im;
      }
  }
  if (img_out) memcpy(img_out, I, sizeof(double) * tot);
  free(z);
  free(I);
  free(G);
  return E;
}
