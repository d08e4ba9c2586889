// Single-cell x/y passes for 2-3-5-smooth line lengths that are not powers
// of two: two-step register transforms (fft_reg.h, fft_mixed.h) over tiles
// of flattened (other index, k3) pairs, tiles grouped per XCD as in the
// power-of-two passes.
#include "fft_mixed.h"

namespace dbfft {

template <typename T, int N, int MODE>
__global__ __launch_bounds__(MixedShape<N>::NT) void k_strided_mixed(const cpx<T>* in, cpx<T>* out, StridedGeom sg,
                                                                     Geom g, const cpx<T>* __restrict__ twg, T d,
                                                                     double* __restrict__ dc_out,
                                                                     const int* __restrict__ stop, AlphaTask at) {
  using S = MixedShape<N>;
  if (at.sc != nullptr && blockIdx.x == 0 && blockIdx.z == 0) alpha_task_wave(at.sc, at.eparts, at.neparts);
  if (stop != nullptr && *stop) return;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[N * S::PITCH];
  for (int i = threadIdx.x; i < N; i += S::NT) tw[i] = twg[i];
  __syncthreads();
  const int nb = gridDim.x;
  const int per = nb >> 3;
  const int b = blockIdx.x;
  const int tile = (b < (per << 3)) ? (b & 7) * per + (b >> 3) : b;
  // plain: grid z is the component; small-strain gradient and divergence:
  // grid z is the part (three)
  constexpr bool parts = MODE == SP_GRAD_SMALL || MODE == SP_DIV_SMALL;
  const long long cz = parts ? 0 : blockIdx.z;
  mixed_strided_tile<T, N, MODE, parts>(in + cz * sg.cstride_in, out + cz * sg.cstride_out, sg, g, tw, lds, d,
                                        dc_out, tile, threadIdx.x, (int)blockIdx.z);
}

bool mixed_strided_supported(int n) { return two_step_n1(n) != 0; }

template <typename T, int N, int MODE>
static void launch_mixed_nm(const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                            const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                            const AlphaTask& at) {
  using S = MixedShape<N>;
  const long long npair = (long long)sg.nother * sg.ncols;
  const int ntiles = (int)((npair + S::TZ - 1) / S::TZ);
  const int nz = MODE == SP_PLAIN ? ncomp_plain : ((MODE == SP_GRAD_SMALL || MODE == SP_DIV_SMALL) ? 3 : 1);
  dim3 grid(ntiles, 1, nz);
  DB_LAUNCH((k_strided_mixed<T, N, MODE>), grid, dim3(S::NT), 0, st, static_cast<const cpx<T>*>(in),
                     static_cast<cpx<T>*>(out), sg, g, static_cast<const cpx<T>*>(tw), (T)dir, dc_out, stop, at);
}

template <typename T, int N>
static void launch_mixed_n(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg,
                           const Geom& g, const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                           const AlphaTask& at) {
  switch (mode) {
    case SP_PLAIN: launch_mixed_nm<T, N, SP_PLAIN>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    case SP_GRAD_SMALL:
      launch_mixed_nm<T, N, SP_GRAD_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at);
      break;
    case SP_GRAD_FINITE:
      launch_mixed_nm<T, N, SP_GRAD_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at);
      break;
    case SP_DIV_SMALL: launch_mixed_nm<T, N, SP_DIV_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    default: launch_mixed_nm<T, N, SP_DIV_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
  }
}

template <typename T>
void launch_strided_mixed(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                          const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                          const AlphaTask& at) {
  switch (sg.nline) {
#define DBFFT_MIX(NN) \
  case NN: launch_mixed_n<T, NN>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    DBFFT_MIX(12) DBFFT_MIX(15) DBFFT_MIX(18) DBFFT_MIX(20) DBFFT_MIX(24) DBFFT_MIX(25) DBFFT_MIX(27)
    DBFFT_MIX(30) DBFFT_MIX(36) DBFFT_MIX(40) DBFFT_MIX(45) DBFFT_MIX(48) DBFFT_MIX(50) DBFFT_MIX(54)
    DBFFT_MIX(60) DBFFT_MIX(63) DBFFT_MIX(72) DBFFT_MIX(80) DBFFT_MIX(90) DBFFT_MIX(96)
#undef DBFFT_MIX
    default: break;
  }
}
template void launch_strided_mixed<double>(int, const void*, void*, int, const StridedGeom&, const Geom&,
                                           const void*, int, double*, hipStream_t, const int*, const AlphaTask&);
template void launch_strided_mixed<float>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                          int, double*, hipStream_t, const int*, const AlphaTask&);

// ---------------------------------------------------------------- z pass
template <typename T, int M, int KIN, int ISO>
__global__ __launch_bounds__(64) void k_line_mixed(const cpx<T>* in, cpx<T>* out, Geom g, const cpx<T>* __restrict__ twg,
                                                   const cpx<T>* __restrict__ rtwg, TangentArgs<T> tn,
                                                   const double* __restrict__ macro_dev, double* __restrict__ partials,
                                                   const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  using L = MixedLine<M>;
  __shared__ cpx<T> tw[M];
  __shared__ cpx<T> rtw[M + 1];
  __shared__ cpx<T> lds[L::LB * L::PITCH];
  for (int i = threadIdx.x; i < M; i += 64) tw[i] = twg[i];
  for (int i = threadIdx.x; i <= M; i += 64) rtw[i] = rtwg[i];
  __syncthreads();
  // isotropic: grid y splits the normal (0) and shear (1) components
  const double e = mixed_line_fused<T, M, KIN, ISO>(in, out, g, tw, rtw, lds, tn, macro_dev, blockIdx.x, threadIdx.x,
                                                    ISO ? (int)blockIdx.y : -1);
  if (partials != nullptr && threadIdx.x == 0) partials[blockIdx.x + (long long)blockIdx.y * gridDim.x] = e;
}

// z pass of the anisotropic and finite-strain tangents in FP32: the four
// waves of a block share one line group, whose components are staged in LDS
// (mixed_line_staged); one energy partial per block.
template <typename T, int M, int KIN, int LAW>
__global__ __launch_bounds__(256) void k_line_staged(const cpx<T>* in, cpx<T>* out, Geom g,
                                                     const cpx<T>* __restrict__ twg, const cpx<T>* __restrict__ rtwg,
                                                     TangentArgs<T> tn, const double* __restrict__ macro_dev,
                                                     double* __restrict__ partials, const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  using L = MixedLine<M>;
  constexpr int NW = 4, NC = (KIN == KIN_SMALL) ? 6 : 9;
  __shared__ cpx<T> tw[M];
  __shared__ cpx<T> rtw[M + 1];
  __shared__ cpx<T> lds[NW * L::LB * L::PITCH];
  __shared__ cpx<T> X[NC * L::LB * M];
  __shared__ double ew[NW];
  for (int i = threadIdx.x; i < M; i += NW * 64) tw[i] = twg[i];
  for (int i = threadIdx.x; i <= M; i += NW * 64) rtw[i] = rtwg[i];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double e = mixed_line_staged<T, M, KIN, LAW, NW>(in, out, g, tw, rtw, lds + w * L::LB * L::PITCH, X, tn, macro_dev,
                                                    blockIdx.x, w, lane);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
  if (lane == 0) ew[w] = e;
  __syncthreads();
  if (threadIdx.x == 0 && partials != nullptr) partials[blockIdx.x] = (ew[0] + ew[1]) + (ew[2] + ew[3]);
}

static int mixed_lines_per_wave(int M) {
  const int n1 = mixed_n1(M), n2 = M / n1;
  return 64 / (n1 > n2 ? n1 : n2);
}

bool mixed_line_supported(int n3, int elem_bytes, bool iso) {
  if (n3 % 2 != 0 || two_step_n1(n3 / 2) == 0) return false;
  return iso || elem_bytes == 8;
}

int mixed_line_blocks(const Geom& g) {
  const int lb = mixed_lines_per_wave(g.n3 / 2);
  return (int)(((long long)g.n1 * g.n2 + lb - 1) / lb);
}

int mixed_line_energy_blocks(const Geom& g, bool iso) { return mixed_line_blocks(g) * (iso ? 2 : 1); }

template <typename T, int M>
static void launch_line_mixed_m(int kin, bool iso, const void* in, void* out, const Geom& g, const void* tw,
                                const void* rtw, const TangentArgs<T>& tan, const double* macro_dev, double* partials,
                                hipStream_t st, const int* stop) {
  const int nb = mixed_line_blocks(g);
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
  if (iso)
    DB_LAUNCH((k_line_mixed<T, M, KIN_SMALL, 1>), dim3(nb, 2), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                       partials, stop);
  else if constexpr (sizeof(T) == 4) {
    // one line group per block of four waves (as many blocks as there are
    // line groups, so the energy partials count as for one wave per group)
    if (kin == KIN_SMALL)
      DB_LAUNCH((k_line_staged<T, M, KIN_SMALL, 0>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
                partials, stop);
    else if (finite_law(tan.kind) == 2)
      DB_LAUNCH((k_line_staged<T, M, KIN_FINITE, 2>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
                partials, stop);
    else
      DB_LAUNCH((k_line_staged<T, M, KIN_FINITE, 0>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
                partials, stop);
  }
}

template <typename T>
void launch_line_mixed(int kin, bool iso, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                       const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                       const int* stop) {
  switch (g.n3 / 2) {
#define DBFFT_ZM(MM) \
  case MM: launch_line_mixed_m<T, MM>(kin, iso, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
    DBFFT_ZM(12) DBFFT_ZM(15) DBFFT_ZM(18) DBFFT_ZM(20) DBFFT_ZM(24) DBFFT_ZM(25) DBFFT_ZM(27) DBFFT_ZM(30)
    DBFFT_ZM(36) DBFFT_ZM(40) DBFFT_ZM(45) DBFFT_ZM(48) DBFFT_ZM(50) DBFFT_ZM(54) DBFFT_ZM(60) DBFFT_ZM(63) DBFFT_ZM(72)
    DBFFT_ZM(80) DBFFT_ZM(90) DBFFT_ZM(96)
#undef DBFFT_ZM
    default: break;
  }
}
// Anisotropic and finite-strain tangents on power-of-two lines: the staged
// z pass (a block of four waves per line group) instead of the register
// kernel, whose one-wave blocks hold every component of their lines (up to
// 256 VGPRs, one wave per SIMD; on grids of 64^3 and below they also leave
// SIMDs idle).  The staging buffer and the exchange buffers fit the 64 KB
// of a block's LDS up to n3 = 64 in FP64 and n3 = 128 in FP32.  FP32
// finite-strain lines of 128 keep the register kernel (measured faster
// there: 60 against 67 us at 128^3).
bool staged_line_supported(int n3, int elem_bytes, bool iso, bool finite) {
  if (iso) return false;
  if (n3 == 32 || n3 == 64) return true;
  return elem_bytes == 8 && n3 == 128 && !finite;
}

int staged_line_blocks(const Geom& g) { return mixed_line_blocks(g); }

template <typename T, int M>
static void launch_staged_m(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                            const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                            const int* stop) {
  const int nb = staged_line_blocks(g);
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
  if (kin == KIN_SMALL)
    DB_LAUNCH((k_line_staged<T, M, KIN_SMALL, 0>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
              partials, stop);
  else if (finite_law(tan.kind) == 2)
    DB_LAUNCH((k_line_staged<T, M, KIN_FINITE, 2>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
              partials, stop);
  else
    DB_LAUNCH((k_line_staged<T, M, KIN_FINITE, 0>), dim3(nb), dim3(256), 0, st, i, o, g, t, r, tan, macro_dev,
              partials, stop);
}

template <typename T>
void launch_line_staged(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                        const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                        const int* stop) {
  if (g.n3 == 32) launch_staged_m<T, 16>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
  else if (g.n3 == 64) launch_staged_m<T, 32>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
  else if constexpr (sizeof(T) == 4) launch_staged_m<T, 64>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
}
template void launch_line_staged<double>(int, const void*, void*, const Geom&, const void*, const void*,
                                         const TangentArgs<double>&, const double*, double*, hipStream_t, const int*);
template void launch_line_staged<float>(int, const void*, void*, const Geom&, const void*, const void*,
                                        const TangentArgs<float>&, const double*, double*, hipStream_t, const int*);

template void launch_line_mixed<double>(int, bool, const void*, void*, const Geom&, const void*, const void*,
                                        const TangentArgs<double>&, const double*, double*, hipStream_t, const int*);
template void launch_line_mixed<float>(int, bool, const void*, void*, const Geom&, const void*, const void*,
                                       const TangentArgs<float>&, const double*, double*, hipStream_t, const int*);

// ---------------------------------------------------------------- real z transforms
// Inverse (C2R, + macro) or forward (R2C, scaled 1/N) real transforms of
// one component per grid y, LB lines per wave, even n3 with n3/2 in the
// two-step set (powers of two included): the strain fields and stress
// residuals of the Newton steps.
template <typename T, int M>
__global__ __launch_bounds__(64) void k_line_c2r(const cpx<T>* in, T* out, Geom g, const cpx<T>* __restrict__ twg,
                                                 const cpx<T>* __restrict__ rtwg, const double* __restrict__ mac_a,
                                                 const double* __restrict__ mac_b) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM, TL = L::TL, LB = L::LB, PITCH = L::PITCH;
  __shared__ cpx<T> tw[M];
  __shared__ cpx<T> rtw[M + 1];
  __shared__ cpx<T> lds[LB * PITCH];
  for (int i = threadIdx.x; i < M; i += 64) tw[i] = twg[i];
  for (int i = threadIdx.x; i <= M; i += 64) rtw[i] = rtwg[i];
  __syncthreads();
  const int lane = threadIdx.x, line = lane / TL, t = lane % TL;
  const bool active = line < LB;
  const long long gl = (long long)blockIdx.x * LB + line;
  const bool valid = active && gl < (long long)g.n1 * g.n2;
  const int tj = active ? t : TL;
  const int partner = active ? line * TL + ((t < N2) ? (N2 - t) % N2 : t) : lane;
  const int off = (active ? line : 0) * PITCH;
  const int c = blockIdx.y;
  const T mc = (T)((mac_a ? mac_a[c] : 0.0) + (mac_b ? mac_b[c] : 0.0));
  cpx<T> e[EM];
  mixed_line_inverse<T, M>(in + (long long)c * g.nh + (valid ? gl : 0) * g.nh3, valid, t, tj, partner, lds, off, tw,
                           rtw, e);
  if (valid && t < N1) {
    T* o = out + (long long)c * g.nvox + gl * g.n3;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int n = t + N1 * k2;
      o[2 * n] = e[k2].x + mc;
      o[2 * n + 1] = e[k2].y + mc;
    }
  }
}

template <typename T, int M>
__global__ __launch_bounds__(64) void k_line_r2c(const T* in, cpx<T>* out, Geom g, const cpx<T>* __restrict__ twg,
                                                 const cpx<T>* __restrict__ rtwg) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM, TL = L::TL, LB = L::LB, PITCH = L::PITCH;
  __shared__ cpx<T> tw[M];
  __shared__ cpx<T> rtw[M + 1];
  __shared__ cpx<T> lds[LB * PITCH];
  for (int i = threadIdx.x; i < M; i += 64) tw[i] = twg[i];
  for (int i = threadIdx.x; i <= M; i += 64) rtw[i] = rtwg[i];
  __syncthreads();
  const int lane = threadIdx.x, line = lane / TL, t = lane % TL;
  const bool active = line < LB;
  const long long gl = (long long)blockIdx.x * LB + line;
  const bool valid = active && gl < (long long)g.n1 * g.n2;
  const int tj = active ? t : TL;
  const int partner = active ? line * TL + ((t < N2) ? (N2 - t) % N2 : t) : lane;
  const int off = (active ? line : 0) * PITCH;
  const int c = blockIdx.y;
  cpx<T> e[EM];
#pragma unroll
  for (int k2 = 0; k2 < EM; ++k2) e[k2] = mk<T>(0, 0);
  if (valid && t < N1) {
    const T* x = in + (long long)c * g.nvox + gl * g.n3;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int n = t + N1 * k2;
      e[k2] = mk<T>(x[2 * n], x[2 * n + 1]);
    }
  }
  mixed_line_forward<T, M>(out + (long long)c * g.nh + (valid ? gl : 0) * g.nh3, valid, t, tj, partner, lds, off, tw,
                           rtw, e, (T)g.inv_nvox);
}

bool real_line_supported(int n3) {
  switch (n3 / 2) {
    case 12: case 15: case 16: case 18: case 20: case 24: case 25: case 27: case 30: case 32: case 36: case 40:
    case 45: case 48: case 50: case 54: case 60: case 63: case 64: case 72: case 80: case 90: case 96:
      return n3 % 2 == 0;
    default: return false;
  }
}

template <typename T, int M>
static void launch_line_real_m(int mode, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                               const double* mac_a, const double* mac_b, int ncomp, hipStream_t st) {
  const int lb = MixedLine<M>::LB;
  const int nb = (int)(((long long)g.n1 * g.n2 + lb - 1) / lb);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
  if (mode == LP_C2R)
    DB_LAUNCH((k_line_c2r<T, M>), dim3(nb, ncomp), dim3(64), 0, st, static_cast<const cpx<T>*>(in),
              static_cast<T*>(out), g, t, r, mac_a, mac_b);
  else
    DB_LAUNCH((k_line_r2c<T, M>), dim3(nb, ncomp), dim3(64), 0, st, static_cast<const T*>(in),
              static_cast<cpx<T>*>(out), g, t, r);
}

template <typename T>
void launch_line_real(int mode, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                      const double* mac_a, const double* mac_b, int ncomp, hipStream_t st) {
  switch (g.n3 / 2) {
#define DBFFT_ZR(MM) \
  case MM: launch_line_real_m<T, MM>(mode, in, out, g, tw, rtw, mac_a, mac_b, ncomp, st); break;
    DBFFT_ZR(12) DBFFT_ZR(15) DBFFT_ZR(16) DBFFT_ZR(18) DBFFT_ZR(20) DBFFT_ZR(24) DBFFT_ZR(25) DBFFT_ZR(27)
    DBFFT_ZR(30) DBFFT_ZR(32) DBFFT_ZR(36) DBFFT_ZR(40) DBFFT_ZR(45) DBFFT_ZR(48) DBFFT_ZR(50) DBFFT_ZR(54)
    DBFFT_ZR(60) DBFFT_ZR(63) DBFFT_ZR(64) DBFFT_ZR(72) DBFFT_ZR(80) DBFFT_ZR(90) DBFFT_ZR(96)
#undef DBFFT_ZR
    default: break;
  }
}
template void launch_line_real<double>(int, const void*, void*, const Geom&, const void*, const void*, const double*,
                                       const double*, int, hipStream_t);
template void launch_line_real<float>(int, const void*, void*, const Geom&, const void*, const void*, const double*,
                                      const double*, int, hipStream_t);

// ---------------------------------------------------------------- odd z pass
// Fused z pass for an odd length N = n3 (two-step N1 x N2), isotropic
// small-strain tangent.  A line's samples are real, so two components ride
// in one complex transform (z_a + i z_b) and come apart by conjugate
// symmetry on the way back: S_a(k) = (Y(k) + conj Y(N-k))/2, S_b(k) =
// (Y(k) - conj Y(N-k))/(2i).  The stored half spectrum k = 0..(N-1)/2 is
// extended by X(N-k) = conj X(k).  One wave handles LB lines; grid y splits
// the components: part 0 the pairs (11, 22) and (33, 23), part 1 (13, 12).
template <int N>
struct OddLine {
  static constexpr int N1 = two_step_n1(N);
  static constexpr int N2 = N / N1;
  static constexpr int TL = N1 > N2 ? N1 : N2;
  static constexpr int LB = 64 / TL;
  static constexpr int NH = (N + 1) / 2;
  static constexpr int PITCH = N + TL + 1;
};

template <typename T, int N>
__global__ __launch_bounds__(64) void k_line_odd(const cpx<T>* in, cpx<T>* out, Geom g,
                                                 const cpx<T>* __restrict__ twg, TangentArgs<T> tn,
                                                 const double* __restrict__ macro_dev, double* __restrict__ partials,
                                                 const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  using L = OddLine<N>;
  constexpr int N1 = L::N1, N2 = L::N2, TL = L::TL, LB = L::LB, NH = L::NH, PITCH = L::PITCH;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[LB * PITCH];
  __shared__ cpx<T> ybuf[LB * N];
  for (int i = threadIdx.x; i < N; i += 64) tw[i] = twg[i];
  __syncthreads();
  const int lane = threadIdx.x, line = lane / TL, t = lane % TL;
  const bool active = line < LB;
  const long long nlines = (long long)g.n1 * g.n2;
  const long long gl = (long long)blockIdx.x * LB + line;
  const bool valid = active && gl < nlines;
  const int tj = active ? t : TL;  // lanes past the last line take no part
  const int off = (active ? line : 0) * PITCH;
  const int part = blockIdx.y;
  const T scale = (T)g.inv_nvox;
  double mac[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) mac[c] = macro_dev ? macro_dev[c] : 0.0;
  const cpx<T>* inl = in + (valid ? gl : 0) * NH;
  cpx<T>* outl = out + (valid ? gl : 0) * NH;
  cpx<T>* yb = ybuf + (active ? line : 0) * N;

  // inverse: z_a + i z_b from the half spectra of components ca, cb;
  // thread t < N1 then holds the samples n = t + N1 k2 (k2 < N2)
  auto inverse_pair = [&](int ca, int cb, cpx<T>* Z) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int k = N2 * n1 + t;
      cpx<T> xa = mk<T>(0, 0), xb = mk<T>(0, 0);
      if (valid && t < N2) {
        if (k < NH) {
          xa = inl[ca * g.nh + k];
          xb = inl[cb * g.nh + k];
        } else {
          xa = conj(inl[ca * g.nh + (N - k)]);
          xb = conj(inl[cb * g.nh + (N - k)]);
        }
      }
      Z[n1] = add(xa, muli(xb, (T)1));
    }
    two_step_fft<T, N1, N2, 1>(Z, tj, lds, 1, off, tw, (T)1);
  };
  // forward of the pair held as z = s_a + i s_b (thread t < N1, samples
  // t + N1 k2), separated and stored scaled
  auto forward_pair = [&](int ca, int cb, cpx<T>* Z) {
    two_step_fft<T, N2, N1, 1>(Z, tj, lds, 1, off, tw, (T)-1);
    // thread t < N2 holds Y(t + N2 m), m < N1
    if (active && t < N2) {
#pragma unroll
      for (int m = 0; m < N1; ++m) yb[t + N2 * m] = Z[m];
    }
    __syncthreads();
    if (valid && t < N2) {
#pragma unroll
      for (int m = 0; m < N1; ++m) {
        const int k = t + N2 * m;
        if (k < NH) {
          const cpx<T> Yk = Z[m];
          const cpx<T> Ym = conj(yb[(N - k) % N]);
          const cpx<T> Sa = scl(add(Yk, Ym), (T)0.5);
          const cpx<T> Sb = muli(scl(sub(Yk, Ym), (T)0.5), (T)-1);
          outl[ca * g.nh + k] = scl(Sa, scale);
          outl[cb * g.nh + k] = scl(Sb, scale);
        }
      }
    }
    __syncthreads();
  };

  double energy = 0.0;
  const bool lt = valid && t < N1;
  if (part == 0) {
    cpx<T> P[N2 > N1 ? N2 : N1], Q[N2 > N1 ? N2 : N1];
    inverse_pair(0, 1, P);  // 11 + i 22
    inverse_pair(2, 3, Q);  // 33 + i 23
    if (lt) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const long long vox = gl * N + t + N1 * k2;
        T lam, mu;
        if (tn.kind == TAN_ISO_PHASE) {
          const int p = tn.phase[vox];
          lam = (T)tn.lam[p];
          mu = (T)tn.mu[p];
        } else {
          const T E = tn.field[vox];
          lam = (T)tn.lam1 * E;
          mu = (T)tn.mu1 * E;
        }
        const T m2 = mu + mu;
        const T e11 = P[k2].x + (T)mac[0], e22 = P[k2].y + (T)mac[1];
        const T e33 = Q[k2].x + (T)mac[2], e23 = Q[k2].y + (T)mac[3];
        const T tr = e11 + e22 + e33;
        const T s11 = lam * tr + m2 * e11, s22 = lam * tr + m2 * e22, s33 = lam * tr + m2 * e33;
        const T s23 = m2 * e23;
        energy += (double)(e11 * s11 + e22 * s22 + e33 * s33) + 2.0 * (double)(e23 * s23);
        P[k2] = mk<T>(s11, s22);
        Q[k2] = mk<T>(s33, s23);
      }
    }
    forward_pair(0, 1, P);
    forward_pair(2, 3, Q);
  } else {
    cpx<T> P[N2 > N1 ? N2 : N1];
    inverse_pair(4, 5, P);  // 13 + i 12
    if (lt) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const long long vox = gl * N + t + N1 * k2;
        T mu;
        if (tn.kind == TAN_ISO_PHASE) mu = (T)tn.mu[tn.phase[vox]];
        else mu = (T)tn.mu1 * tn.field[vox];
        const T m2 = mu + mu;
        const T e13 = P[k2].x + (T)mac[4], e12 = P[k2].y + (T)mac[5];
        const T s13 = m2 * e13, s12 = m2 * e12;
        energy += 2.0 * (double)(e13 * s13 + e12 * s12);
        P[k2] = mk<T>(s13, s12);
      }
    }
    forward_pair(4, 5, P);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) energy += __shfl_xor(energy, o, 64);
  if (partials != nullptr && threadIdx.x == 0)
    partials[blockIdx.x + (long long)blockIdx.y * gridDim.x] = energy * g.inv_nvox;
}

// the odd lengths of the two-step set
bool odd_line_supported(int n3) { return n3 == 15 || n3 == 25 || n3 == 27 || n3 == 45 || n3 == 63; }

static int odd_lines_per_wave(int n3) {
  switch (n3) {
    case 15: return OddLine<15>::LB;
    case 25: return OddLine<25>::LB;
    case 27: return OddLine<27>::LB;
    case 45: return OddLine<45>::LB;
    default: return OddLine<63>::LB;
  }
}

int odd_line_energy_blocks(const Geom& g) {
  const int lb = odd_lines_per_wave(g.n3);
  return 2 * (int)(((long long)g.n1 * g.n2 + lb - 1) / lb);
}

template <typename T>
void launch_line_odd(const void* in, void* out, const Geom& g, const void* tw, const TangentArgs<T>& tan,
                     const double* macro_dev, double* partials, hipStream_t st, const int* stop) {
  const int nb = odd_line_energy_blocks(g) / 2;
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  switch (g.n3) {
#define DBFFT_ZO(NN) \
  case NN: DB_LAUNCH((k_line_odd<T, NN>), dim3(nb, 2), dim3(64), 0, st, i, o, g, t, tan, macro_dev, partials, stop); break;
    DBFFT_ZO(15) DBFFT_ZO(25) DBFFT_ZO(27) DBFFT_ZO(45) DBFFT_ZO(63)
#undef DBFFT_ZO
    default: break;
  }
}
template void launch_line_odd<double>(const void*, void*, const Geom&, const void*, const TangentArgs<double>&,
                                      const double*, double*, hipStream_t, const int*);
template void launch_line_odd<float>(const void*, void*, const Geom&, const void*, const TangentArgs<float>&,
                                     const double*, double*, hipStream_t, const int*);

}  // namespace dbfft
