// Host FP64 table builders (twiddles, matched filters) and storage encoders.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <complex>
#include <vector>

namespace bfp {

std::complex<double> unit_root(long long k, long long n);
uint16_t f64_to_f16_bits(double x);
uint8_t f64_to_fp8_bits(double x, int mant, int bias);
void encode_complex(const std::complex<double> *src, size_t count, int fmt, void *dst);
std::vector<std::complex<double>> twiddle_table(int log2n, const int *radix, int passes);
void host_fft(std::vector<std::complex<double>> &a);
std::vector<uint16_t> mfma4096_table();
// Amplitude taper of `len` points for weighted matched filters (kind: 0
// rectangular, 1 Hamming, 2 Taylor with nbar terms and peak sidelobe level
// -sll_db); returns false on invalid arguments.
bool taper(int kind, int len, int nbar, double sll_db, double *out);

}  // namespace bfp
