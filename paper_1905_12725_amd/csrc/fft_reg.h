// In-register DFTs of small 2-3-5-smooth sizes and the two-step transform
// of a line of length N = N1 N2 used for the grid sizes that are not powers
// of two.
//
// Two-step (Cooley-Tukey with one transpose):
//   step 1: thread j < N2 holds x[N2 n1 + j] (n1 < N1), does an N1-point
//           DFT in registers, multiplies by w_N^(j k1) and writes Y[k1][j]
//           to LDS;
//   step 2: thread j' < N1 reads Y[j'][n2] (n2 < N2) and does an N2-point
//           DFT: register k2 then holds X[j' + N1 k2].
// The input distribution of plan (N1, N2) equals the output distribution
// of plan (N2, N1), so a forward transform with the swapped plan takes the
// inverse transform's output where it lies.
#pragma once

#include <utility>

#include "fft_common.h"

namespace dbfft {

// ---------------------------------------------------------------- compile-time twiddles
namespace ctw {
constexpr double kQuarterPi = 0.78539816339744830962;
constexpr double sin_series(double x) {  // |x| <= pi/4
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {  // |x| <= pi/4
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / R through the octant of the angle (exact
// rational reduction, series on at most pi/4)
constexpr double cos2pi(int m, int R) {
  m %= R;
  const int o = (8 * m) / R, r = 8 * m - o * R;
  const double phi = kQuarterPi * r / R, psi = kQuarterPi - phi;
  switch (o) {
    case 0: return cos_series(phi);
    case 1: return sin_series(psi);
    case 2: return -sin_series(phi);
    case 3: return -cos_series(psi);
    case 4: return -cos_series(phi);
    case 5: return -sin_series(psi);
    case 6: return sin_series(phi);
    default: return cos_series(psi);
  }
}
constexpr double sin2pi(int m, int R) {
  m %= R;
  const int o = (8 * m) / R, r = 8 * m - o * R;
  const double phi = kQuarterPi * r / R, psi = kQuarterPi - phi;
  switch (o) {
    case 0: return sin_series(phi);
    case 1: return cos_series(psi);
    case 2: return cos_series(phi);
    case 3: return sin_series(psi);
    case 4: return -sin_series(phi);
    case 5: return -cos_series(psi);
    case 6: return -cos_series(phi);
    default: return -sin_series(psi);
  }
}
}  // namespace ctw

template <int R, int M>
struct Twiddle {
  static constexpr double c = ctw::cos2pi(M, R);
  static constexpr double s = ctw::sin2pi(M, R);
};

// compile-time loop: f(std::integral_constant<int, i>) for i < N
template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int reg_first_factor(int R) {
  return (R % 4 == 0 && R != 4 && R != 8) ? 4 : (R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : 5));
}

// R-point DFT of v in registers, exponent sign d (-1 forward, +1 inverse),
// R a product of 2, 3 and 5 up to 16, or 7
template <typename T, int R>
__device__ __forceinline__ void reg_dft(cpx<T>* v, T d) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2 || R == 3 || R == 4 || R == 5 || R == 7 || R == 8) {
    dftR<T, R>(v, d);
  } else {
    constexpr int A = reg_first_factor(R);
    constexpr int B = R / A;
    cpx<T> tmp[R];
    sfor<B>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cpx<T> u[A];
      sfor<A>([&](auto n1c) { u[decltype(n1c)::value] = v[B * decltype(n1c)::value + n2]; });
      reg_dft<T, A>(u, d);
      sfor<A>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        constexpr int m = (n2 * k1) % R;
        if constexpr (m != 0) u[k1] = mul(u[k1], mk<T>((T)Twiddle<R, m>::c, d * (T)Twiddle<R, m>::s));
        tmp[k1 * B + n2] = u[k1];
      });
    });
    sfor<A>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      cpx<T> u2[B];
      sfor<B>([&](auto n2c) { u2[decltype(n2c)::value] = tmp[k1 * B + decltype(n2c)::value]; });
      reg_dft<T, B>(u2, d);
      sfor<B>([&](auto k2c) { v[k1 + A * decltype(k2c)::value] = u2[decltype(k2c)::value]; });
    });
  }
}

// Two-step transform of one line per thread group.  v[] holds EM =
// max(N1, N2) registers; on entry thread j (< N2) holds its N1 inputs in
// v[0..N1), on exit thread j (< N1) holds its N2 outputs in v[0..N2).
// Position p of Y[k1][j] = k1 * (N2 + RP) + j in LDS, at lds[p * pitch +
// off]; tw[m] = exp(-2 pi i m / N).  Synchronizes the block (twice).
template <typename T, int N1, int N2, int RP>
__device__ __forceinline__ void two_step_fft(cpx<T>* v, int j, cpx<T>* lds, int pitch, int off,
                                             const cpx<T>* __restrict__ tw, T d) {
  constexpr int N = N1 * N2;
  if (j < N2) {
    reg_dft<T, N1>(v, d);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      cpx<T> w = tw[(j * k1) % N];
      w.y *= -d;
      v[k1] = mul(v[k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) lds[(k1 * (N2 + RP) + j) * pitch + off] = v[k1];
  }
  __syncthreads();
  if (j < N1) {
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) v[n2] = lds[(j * (N2 + RP) + n2) * pitch + off];
    reg_dft<T, N2>(v, d);
  }
  __syncthreads();
}

// factor pairs (N1 <= N2 <= 16) of the supported lengths that are not powers
// of two; 0 when the length has none
constexpr int two_step_n1(int n) {
  switch (n) {
    case 12: return 3;
    case 15: return 3;
    case 18: return 3;
    case 20: return 4;
    case 24: return 4;
    case 25: return 5;
    case 27: return 3;
    case 30: return 5;
    case 36: return 6;
    case 40: return 5;
    case 45: return 5;
    case 48: return 6;
    case 50: return 5;
    case 54: return 6;
    case 60: return 6;
    case 63: return 7;
    case 72: return 8;
    case 80: return 8;
    case 90: return 9;
    case 96: return 8;
    default: return 0;
  }
}

}  // namespace dbfft
