// Host check of the register DFTs against the O(N^2) definition in double:
// prints "N max_err_fwd max_err_inv" (errors scaled by 1/sqrt(N)) for every
// length used as a factor of a compiled transform length.
#include <cmath>
#include <complex>
#include <cstdio>

#include "../../paper_2003_07504_amd/csrc/fft_reg.hpp"

using ilsk::cf;

template <int N, int DIR>
double check() {
  cf x[N];
  std::complex<double> in[N];
  for (int i = 0; i < N; ++i) {
    in[i] = {std::sin(1.3 * i + 0.2), std::cos(0.7 * i * i + 1.0)};
    x[i] = {(float)in[i].real(), (float)in[i].imag()};
  }
  ilsk::dft<N, DIR>(x);
  double e = 0.0;
  for (int k = 0; k < N; ++k) {
    std::complex<double> ref = 0.0;
    for (int n = 0; n < N; ++n) ref += in[n] * std::polar(1.0, DIR * 2.0 * M_PI * double((long long)n * k % N) / N);
    e = std::fmax(e, std::abs(std::complex<double>(x[k].x, x[k].y) - ref));
  }
  return e / std::sqrt((double)N);
}

template <int... Ns>
void run() {
  ((std::printf("%d %.3e %.3e\n", Ns, check<Ns, -1>(), check<Ns, 1>())), ...);
}

int main() {
  run<1, 2, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 30, 32, 36, 40, 45, 48, 64>();
  return 0;
}
