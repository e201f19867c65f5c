// Register-resident small DFTs for gfx950, fully specialised at compile time.
//
// dft<N, DIR>(x) transforms N complex values held in registers, natural
// order in and natural order out:  X[k] = sum_n x[n] exp(DIR * 2 pi i n k / N)
// (DIR = -1 forward, +1 inverse, unnormalised).  A length with two or more
// distinct prime factors is split N = N1 * N2 with coprime factors by the
// prime-factor (Good-Thomas) mapping, which needs no twiddle factors; a prime
// power is split N = R * L (R = 4, 2, 3 or 5) Cooley-Tukey style: L
// interleaved R-point DFTs, a twiddle by exp(DIR 2 pi i n2 k1 / N), then R
// L-point DFTs.  Every index and every twiddle is a compile-time constant, so
// after inlining the whole transform is straight-line register code; twiddle
// constants are evaluated in double precision at compile time and rounded
// once to float.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace ilsk {

struct cf {
  float x, y;
};

__host__ __device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
// a * w
__host__ __device__ __forceinline__ cf cmul(cf a, cf w) {
  return {fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x)};
}
// a * conj(w)
__host__ __device__ __forceinline__ cf cmulc(cf a, cf w) {
  return {fmaf(a.x, w.x, a.y * w.y), fmaf(a.y, w.x, -(a.x * w.y))};
}
__host__ __device__ __forceinline__ cf mul_i(cf a) { return {-a.y, a.x}; }   // i * a
__host__ __device__ __forceinline__ cf mul_mi(cf a) { return {a.y, -a.x}; }  // -i * a
__host__ __device__ __forceinline__ cf cneg(cf a) { return {-a.x, -a.y}; }
__host__ __device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- static_for
template <class F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------ compile-time trigonometry
struct dcs {
  double c, s;
};
constexpr double kPi = 3.14159265358979323846264338327950288;

// cos and sin of |x| <= pi/4 by their Taylor series (error < 1e-17).
constexpr dcs cs_small(double x) {
  double x2 = x * x;
  double ts = x, s = x, tc = 1.0, c = 1.0;
  for (int i = 1; i < 14; ++i) {
    ts *= -x2 / double((2 * i) * (2 * i + 1));
    s += ts;
    tc *= -x2 / double((2 * i - 1) * (2 * i));
    c += tc;
  }
  return {c, s};
}

// cos and sin of 2 pi m / n, with the argument reduced exactly in integers to
// the nearest quarter turn, so the multiples of pi/2 come out exact.
constexpr dcs cossin_turn(long long m, long long n) {
  m %= n;
  if (m < 0) m += n;
  long long k = (8 * m + n) / (2 * n);  // nearest integer to 4m/n
  long long num = 4 * m - k * n;        // remainder, |num| <= n/2
  dcs b = cs_small(2.0 * kPi * double(num) / (4.0 * double(n)));
  switch (k & 3) {
    case 0: return b;
    case 1: return {-b.s, b.c};
    case 2: return {-b.c, -b.s};
    default: return {b.s, -b.c};
  }
}

// a * exp(DIR * 2 pi i M / N), with the trivial angles done without multiplies.
template <long long M, long long N, int DIR>
__host__ __device__ __forceinline__ cf twiddle_c(cf a) {
  constexpr long long m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (2 * m == N) {
    return cneg(a);
  } else if constexpr (4 * m == N) {
    return DIR > 0 ? mul_i(a) : mul_mi(a);
  } else if constexpr (4 * m == 3 * N) {
    return DIR > 0 ? mul_mi(a) : mul_i(a);
  } else {
    constexpr dcs w = cossin_turn(m, N);
    constexpr float c = float(w.c);
    constexpr float s = float(DIR * w.s);
    return cmul(a, cf{c, s});
  }
}

// ------------------------------------------------------------ small kernels
template <int DIR>
__host__ __device__ __forceinline__ void dft2(cf& a, cf& b) {
  cf t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__host__ __device__ __forceinline__ void dft3(cf& a, cf& b, cf& c) {
  constexpr float s = float(DIR) * 0.86602540378443864676f;  // DIR * sin(2 pi / 3)
  cf t1 = cadd(b, c);
  cf t2 = {fmaf(-0.5f, t1.x, a.x), fmaf(-0.5f, t1.y, a.y)};
  cf d = csub(b, c);
  cf t3 = {s * d.x, s * d.y};
  a = cadd(a, t1);
  b = {t2.x - t3.y, t2.y + t3.x};  // t2 + i t3
  c = {t2.x + t3.y, t2.y - t3.x};  // t2 - i t3
}

template <int DIR>
__host__ __device__ __forceinline__ void dft4(cf& a, cf& b, cf& c, cf& d) {
  cf t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d);
  cf bd = csub(b, d);
  cf t3 = DIR > 0 ? mul_i(bd) : mul_mi(bd);  // (DIR i)(b - d)
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}

template <int DIR>
__host__ __device__ __forceinline__ void dft5(cf& a, cf& b, cf& c, cf& d, cf& e) {
  constexpr dcs w1 = cossin_turn(1, 5), w2 = cossin_turn(2, 5);
  constexpr float c1 = float(w1.c), c2 = float(w2.c);
  constexpr float s1 = float(DIR * w1.s), s2 = float(DIR * w2.s);
  cf t1 = cadd(b, e), t2 = cadd(c, d), t3 = csub(b, e), t4 = csub(c, d);
  cf r1 = {fmaf(c1, t1.x, fmaf(c2, t2.x, a.x)), fmaf(c1, t1.y, fmaf(c2, t2.y, a.y))};
  cf r2 = {fmaf(c2, t1.x, fmaf(c1, t2.x, a.x)), fmaf(c2, t1.y, fmaf(c1, t2.y, a.y))};
  cf i1 = {fmaf(s1, t3.x, s2 * t4.x), fmaf(s1, t3.y, s2 * t4.y)};   // s1 t3 + s2 t4
  cf i2 = {fmaf(s2, t3.x, -s1 * t4.x), fmaf(s2, t3.y, -s1 * t4.y)};  // s2 t3 - s1 t4
  a = cadd(a, cadd(t1, t2));
  b = {r1.x - i1.y, r1.y + i1.x};  // r1 + i i1
  e = {r1.x + i1.y, r1.y - i1.x};  // r1 - i i1
  c = {r2.x - i2.y, r2.y + i2.x};
  d = {r2.x + i2.y, r2.y - i2.x};
}

constexpr int pick_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : 5;
}

constexpr bool is_235_smooth(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

// Prime-factor split of n: the prime-power part of n for its largest prime
// (N1), if n has another prime factor too; 0 when n is a prime power.
constexpr int pfa_split(int n) {
  int part = 1;
  for (int p : {2, 3, 5}) {
    int q = 1;
    while (n % (q * p) == 0) q *= p;
    if (q > 1) part = q;
  }
  return (part > 1 && part < n) ? part : 0;
}

constexpr int inverse_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <int N, int DIR>
__host__ __device__ __forceinline__ void dft(cf (&x)[N]);

// Good-Thomas: input n = (N2 n1 + N1 n2) mod N, output k = (N2 t2 k1 + N1 t1 k2)
// mod N with t2 = N2^-1 mod N1, t1 = N1^-1 mod N2; then exp(2 pi i n k / N)
// factors into exp(2 pi i n1 k1 / N1) exp(2 pi i n2 k2 / N2).
template <int N1, int N2, int DIR>
__host__ __device__ __forceinline__ void dft_pfa(cf (&x)[N1 * N2]) {
  constexpr int N = N1 * N2;
  constexpr int t2 = inverse_mod(N2 % N1, N1), t1 = inverse_mod(N1 % N2, N2);
  cf a[N1][N2];
  static_for<N2>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    cf t[N1];
    static_for<N1>([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      t[n1] = x[(N2 * n1 + N1 * n2) % N];
    });
    dft<N1, DIR>(t);
    static_for<N1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      a[k1][n2] = t[k1];
    });
  });
  static_for<N1>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    dft<N2, DIR>(a[k1]);
    static_for<N2>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      x[(N2 * t2 * k1 + N1 * t1 * k2) % N] = a[k1][k2];
    });
  });
}

template <int N, int DIR>
__host__ __device__ __forceinline__ void dft(cf (&x)[N]) {
  static_assert(is_235_smooth(N), "register DFT length must be 2/3/5-smooth");
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    dft2<DIR>(x[0], x[1]);
  } else if constexpr (N == 3) {
    dft3<DIR>(x[0], x[1], x[2]);
  } else if constexpr (N == 4) {
    dft4<DIR>(x[0], x[1], x[2], x[3]);
  } else if constexpr (N == 5) {
    dft5<DIR>(x[0], x[1], x[2], x[3], x[4]);
  } else if constexpr (pfa_split(N) != 0) {
    dft_pfa<pfa_split(N), N / pfa_split(N), DIR>(x);
  } else {
    constexpr int R = pick_radix(N);
    constexpr int L = N / R;
    cf a[R][L];
    static_for<L>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cf t[R];
      static_for<R>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        t[n1] = x[L * n1 + n2];
      });
      dft<R, DIR>(t);
      static_for<R>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        a[k1][n2] = twiddle_c<(long long)n2 * k1, N, DIR>(t[k1]);
      });
    });
    static_for<R>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      dft<L, DIR>(a[k1]);
      static_for<L>([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        x[k1 + R * k2] = a[k1][k2];
      });
    });
  }
}

}  // namespace ilsk
