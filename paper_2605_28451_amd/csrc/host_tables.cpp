// Host-side FP64 tables: twiddles and matched filters, rounded once to the
// storage type.  Roots of unity are evaluated with the argument reduced
// exactly in integers to the first octant (so W^0, W^{N/4}, W^{N/2} and
// W^{3N/4} are exact in every format) and never by recurrence (Sec. III-A).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <complex>
#include <vector>

#include "bfpfft.h"
#include "host_tables.hpp"

namespace bfp {

// exp(-2 pi i k / n): reduce k/n to an angle t in [0, pi/4] by the
// symmetries of the circle, all in integer arithmetic on 8k vs 8n.
std::complex<double> unit_root(long long k, long long n) {
  long long m = k % n;
  if (m < 0) m += n;
  const long long full = 8 * n;
  long long a = 8 * m;
  bool neg_sin = false, neg_cos = false, swap = false;
  if (a > full / 2) { a = full - a; neg_sin = true; }   // angle > pi
  if (a > full / 4) { a = full / 2 - a; neg_cos = true; } // angle > pi/2
  if (a > full / 8) { a = full / 4 - a; swap = true; }   // angle > pi/4
  double c = 1.0, s = 0.0;
  if (a != 0) {
    const double t = 2.0 * M_PI * (double)a / (double)full;
    c = cos(t);
    s = sin(t);
  }
  if (swap) { double tmp = c; c = s; s = tmp; }
  if (neg_cos) c = -c;
  if (neg_sin) s = -s;
  return std::complex<double>(c, -s);
}

// ------------------------------------------------------- rounding ---------
uint16_t f64_to_f16_bits(double x) {
  // round to nearest-even IEEE binary16, overflow to inf, subnormals kept
  uint64_t u;
  memcpy(&u, &x, 8);
  const uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
  const double a = fabs(x);
  if (a != a) return sign | 0x7E00u;
  if (a >= 65520.0) return sign | 0x7C00u;  // rounds to inf
  if (a < 6.103515625e-05) {
    // subnormal (or zero): quantum 2^-24
    const double q = nearbyint(a * 16777216.0);  // ldexp(a, 24), RNE (default mode)
    return sign | (uint16_t)q;                   // q == 1024 is the smallest normal
  }
  int e;
  const double f = frexp(a, &e);                 // a = f 2^e, f in [0.5, 1)
  double q = nearbyint(ldexp(f, 11));            // 11 significant bits
  if (q >= 2048.0) { q /= 2.0; e += 1; }
  const uint16_t ef = (uint16_t)(e - 1 + 15);
  const uint16_t mf = (uint16_t)((uint32_t)q - 1024u);
  return sign | (uint16_t)(ef << 10) | mf;
}

uint8_t f64_to_fp8_bits(double x, int mant, int bias) {
  const uint8_t sign = signbit(x) ? 0x80 : 0;
  double a = fabs(x);
  const int emax_field = (mant == 3) ? 15 : 30;
  const int mmax = (mant == 3) ? 6 : 3;
  const double vmax = ldexp(1.0 + mmax / (double)(1 << mant), emax_field - bias);
  if (a != a) return sign | 0x7F;
  if (a > vmax) a = vmax;
  if (a == 0.0) return sign;
  int e;
  (void)frexp(a, &e);  // a = f 2^e, f in [0.5, 1)
  int ue = e - 1;                 // a in [2^ue, 2^(ue+1))
  const int emin = 1 - bias;
  if (ue < emin) ue = emin;
  double q = nearbyint(ldexp(a, mant - ue));
  if (q >= (double)(2 << mant)) { q /= 2.0; ue += 1; }
  const int qi = (int)q;
  if (qi < (1 << mant)) return sign | (uint8_t)qi;  // subnormal
  return sign | (uint8_t)(((ue + bias) << mant) | (qi - (1 << mant)));
}

static inline uint32_t f32_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

void encode_complex(const std::complex<double> *src, size_t count, int fmt, void *dst) {
  switch (fmt) {
    case BFP_FMT_F32: {
      float *d = static_cast<float *>(dst);
      for (size_t i = 0; i < count; ++i) {
        d[2 * i] = (float)src[i].real();
        d[2 * i + 1] = (float)src[i].imag();
      }
      break;
    }
    case BFP_FMT_F16: {
      uint16_t *d = static_cast<uint16_t *>(dst);
      for (size_t i = 0; i < count; ++i) {
        d[2 * i] = f64_to_f16_bits(src[i].real());
        d[2 * i + 1] = f64_to_f16_bits(src[i].imag());
      }
      break;
    }
    case BFP_FMT_E4M3:
    case BFP_FMT_E5M2: {
      const int mant = fmt == BFP_FMT_E4M3 ? 3 : 2, bias = fmt == BFP_FMT_E4M3 ? 7 : 15;
      uint8_t *d = static_cast<uint8_t *>(dst);
      for (size_t i = 0; i < count; ++i) {
        d[2 * i] = f64_to_fp8_bits(src[i].real(), mant, bias);
        d[2 * i + 1] = f64_to_fp8_bits(src[i].imag(), mant, bias);
      }
      break;
    }
  }
  (void)f32_bits;
}

// --------------------------------------------------------- twiddles -------
// Pass p of a size with radices R_0..R_{P-1}: span NS_p = R_0 ... R_{p-1};
// entries W_{NS R}^{m r} = W_N^{m r N / (NS R)} for m < NS, r < R, stored
// row-major by m, passes with NS > 1 concatenated in order.
std::vector<std::complex<double>> twiddle_table(int log2n, const int *radix, int passes) {
  const long long n = 1ll << log2n;
  std::vector<std::complex<double>> t;
  long long ns = radix[0];
  for (int p = 1; p < passes; ++p) {
    const int r_p = radix[p];
    const long long stride = n / (ns * r_p);
    for (long long m = 0; m < ns; ++m)
      for (int r = 0; r < r_p; ++r) t.push_back(unit_root(m * r * stride, n));
    ns *= r_p;
  }
  return t;
}

// ---------------------------------------------------- host FFT (FP64) -----
// Iterative radix-2 decimation-in-frequency with bit reversal at the end;
// used only to build matched filters on the host.
void host_fft(std::vector<std::complex<double>> &a) {
  const size_t n = a.size();
  for (size_t len = n; len >= 2; len >>= 1) {
    const size_t h = len / 2;
    const size_t step = n / len;
    for (size_t i = 0; i < n; i += len) {
      for (size_t j = 0; j < h; ++j) {
        const std::complex<double> u = a[i + j], v = a[i + j + h];
        a[i + j] = u + v;
        a[i + j + h] = (u - v) * unit_root((long long)(j * step), (long long)n);
      }
    }
  }
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
}

}  // namespace bfp

namespace bfp {

// Table of the N = 4096 matrix-core path (FP16 bit patterns):
//  [0, 1024): per lane l = c + 16 g (64 lanes), 8 halves of A_lo then 8 of
//             A_hi: A[2q+s][2r+u] of the DFT16 (q over {0,1,4,5,8,9,12,13}
//             for A_lo, +2 for A_hi; r = 4g + k/2, u = k % 2);
//  [1024, 2048): the same slices times 2^-12 (first pass of a BFP inverse);
//  then the inter-pass twiddles of the passes of span 16 and 256, entry
//  (m, r) = W_{16 NS}^{m r} stored as the two dot-product operands
//  (Re w, -Im w) and (Im w, Re w).
std::vector<uint16_t> mfma4096_table() {
  std::vector<uint16_t> t;
  t.reserve(2048 + 4 * (256 + 4096));
  // scale 0: F16; scale 1: F16 . 2^-12 (every nonzero entry has magnitude
  // >= sin(pi/8), so the scaled value stays a normal FP16 number)
  for (int scale = 0; scale < 2; ++scale)
    for (int l = 0; l < 64; ++l) {
      const int row = l & 15, g = l >> 4, idx = row >> 1, s = row & 1;
      const int q_lo = ((idx >> 1) << 2) + (idx & 1);
      for (int half = 0; half < 2; ++half) {
        const int q = q_lo + 2 * half;
        for (int k = 0; k < 8; ++k) {
          const int r = 4 * g + (k >> 1), u = k & 1;
          const std::complex<double> w = unit_root((long long)q * r, 16);  // cos - i sin
          const double cs = w.real(), sn = -w.imag();
          double v;
          if (s == 0) v = (u == 0) ? cs : sn;
          else v = (u == 0) ? -sn : cs;
          t.push_back(f64_to_f16_bits(scale ? ldexp(v, -12) : v));
        }
      }
    }
  for (int ns : {16, 256}) {
    const long long stride = 4096 / (ns * 16);
    for (int m = 0; m < ns; ++m)
      for (int r = 0; r < 16; ++r) {
        const std::complex<double> w = unit_root((long long)m * r * stride, 4096);
        t.push_back(f64_to_f16_bits(w.real()));
        t.push_back(f64_to_f16_bits(-w.imag()));
        t.push_back(f64_to_f16_bits(w.imag()));
        t.push_back(f64_to_f16_bits(w.real()));
      }
  }
  return t;
}


// Tapers for weighted apertures (Sec. VIII, limitations: deeply
// weighted apertures aiming at -40 dB sidelobes).  Positions are centred on
// the middle of the aperture, x_n = (n - (len - 1) / 2) / len.
//
// Hamming: 0.54 - 0.46 cos(2 pi n / (len - 1)).
//
// Taylor (nbar, SLL): with eta = 10^(SLL / 20), A = acosh(eta) / pi and the
// dilation s^2 = nbar^2 / (A^2 + (nbar - 1/2)^2), the coefficients
//   F_m = (-1)^(m+1) prod_{i<nbar} (1 - m^2 / (s^2 (A^2 + (i - 1/2)^2)))
//         / (2 prod_{i<nbar, i != m} (1 - m^2 / i^2)),   m = 1 .. nbar - 1,
// give w(x) = 1 + 2 sum_m F_m cos(2 pi m x), scaled to 1 at x = 0.  Its
// first nbar - 1 sidelobes sit near -SLL dB; beyond them they fall as for
// a uniform aperture.
bool taper(int kind, int len, int nbar, double sll_db, double *out) {
  if (!out || len < 1) return false;
  if (kind == 0) {
    for (int n = 0; n < len; ++n) out[n] = 1.0;
    return true;
  }
  if (kind == 1) {
    if (len == 1) {
      out[0] = 1.0;
      return true;
    }
    const double pi = 3.14159265358979323846;
    for (int n = 0; n < len; ++n) out[n] = 0.54 - 0.46 * std::cos(2.0 * pi * n / (len - 1));
    return true;
  }
  if (kind != 2 || nbar < 1 || !(sll_db > 0.0) || sll_db > 300.0) return false;
  const double pi = 3.14159265358979323846;
  const double eta = std::pow(10.0, sll_db / 20.0);
  const double A = std::acosh(eta) / pi;
  const double s2 = double(nbar) * nbar / (A * A + (nbar - 0.5) * (nbar - 0.5));
  std::vector<double> F((size_t)nbar, 0.0);
  for (int m = 1; m < nbar; ++m) {
    double num = 1.0, den = 1.0;
    for (int i = 1; i < nbar; ++i) {
      num *= 1.0 - double(m) * m / (s2 * (A * A + (i - 0.5) * (i - 0.5)));
      if (i != m) den *= 1.0 - double(m) * m / (double(i) * i);
    }
    F[m] = ((m % 2) ? 1.0 : -1.0) * num / (2.0 * den);
  }
  double centre = 1.0;
  for (int m = 1; m < nbar; ++m) centre += 2.0 * F[m];
  for (int n = 0; n < len; ++n) {
    const double x = (n - 0.5 * (len - 1)) / len;
    double w = 1.0;
    for (int m = 1; m < nbar; ++m) w += 2.0 * F[m] * std::cos(2.0 * pi * m * x);
    out[n] = w / centre;
  }
  return true;
}
}  // namespace bfp
