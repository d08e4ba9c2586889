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
                                                                     const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  using S = MixedShape<N>;
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
                            const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop) {
  using S = MixedShape<N>;
  const long long npair = (long long)sg.nother * sg.ncols;
  const int ntiles = (int)((npair + S::TZ - 1) / S::TZ);
  const int nz = MODE == SP_PLAIN ? ncomp_plain : ((MODE == SP_GRAD_SMALL || MODE == SP_DIV_SMALL) ? 3 : 1);
  dim3 grid(ntiles, 1, nz);
  DB_LAUNCH((k_strided_mixed<T, N, MODE>), grid, dim3(S::NT), 0, st, static_cast<const cpx<T>*>(in),
                     static_cast<cpx<T>*>(out), sg, g, static_cast<const cpx<T>*>(tw), (T)dir, dc_out, stop);
}

template <typename T, int N>
static void launch_mixed_n(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg,
                           const Geom& g, const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop) {
  switch (mode) {
    case SP_PLAIN: launch_mixed_nm<T, N, SP_PLAIN>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case SP_GRAD_SMALL: launch_mixed_nm<T, N, SP_GRAD_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case SP_GRAD_FINITE: launch_mixed_nm<T, N, SP_GRAD_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case SP_DIV_SMALL: launch_mixed_nm<T, N, SP_DIV_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    default: launch_mixed_nm<T, N, SP_DIV_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
  }
}

template <typename T>
void launch_strided_mixed(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                          const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop) {
  switch (sg.nline) {
#define DBFFT_MIX(NN) \
  case NN: launch_mixed_n<T, NN>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    DBFFT_MIX(12) DBFFT_MIX(15) DBFFT_MIX(18) DBFFT_MIX(20) DBFFT_MIX(24) DBFFT_MIX(25) DBFFT_MIX(27)
    DBFFT_MIX(30) DBFFT_MIX(36) DBFFT_MIX(40) DBFFT_MIX(45) DBFFT_MIX(48) DBFFT_MIX(50) DBFFT_MIX(54)
    DBFFT_MIX(60) DBFFT_MIX(63) DBFFT_MIX(72) DBFFT_MIX(80) DBFFT_MIX(90) DBFFT_MIX(96)
#undef DBFFT_MIX
    default: break;
  }
}
template void launch_strided_mixed<double>(int, const void*, void*, int, const StridedGeom&, const Geom&,
                                           const void*, int, double*, hipStream_t, const int*);
template void launch_strided_mixed<float>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                          int, double*, hipStream_t, const int*);

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
    if (kin == KIN_SMALL)
      DB_LAUNCH((k_line_mixed<T, M, KIN_SMALL, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                         partials, stop);
    else if (finite_law(tan.kind) == 2)
      DB_LAUNCH((k_line_mixed<T, M, KIN_FINITE, 2>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                partials, stop);
    else
      DB_LAUNCH((k_line_mixed<T, M, KIN_FINITE, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
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
template void launch_line_mixed<double>(int, bool, const void*, void*, const Geom&, const void*, const void*,
                                        const TangentArgs<double>&, const double*, double*, hipStream_t, const int*);
template void launch_line_mixed<float>(int, bool, const void*, void*, const Geom&, const void*, const void*,
                                       const TangentArgs<float>&, const double*, double*, hipStream_t, const int*);

}  // namespace dbfft
