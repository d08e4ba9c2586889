// FFT passes of the DBFFT operator application.
//
// Inverse direction (Fourier -> real):   x pass (+ gradient) -> y pass -> z C2R
// Forward direction (real -> Fourier):   z R2C -> y pass -> x pass (+ divergence)
// The gradient of Sec. 2.2 eq. symgrad (or the full gradient of Sec. 2.4) is
// applied on the fly while the x pass loads the displacement coefficients,
// and the divergence of eq. diver is applied while the last x pass stores,
// so the 3-component unknown is never expanded to a tensor in HBM outside
// the intermediate workspace.  The z pass carries the pointwise tangent:
// inverse real transform, sigma = C(x):eps, forward real transform, for all
// tensor components of a group of z lines held in LDS.
#include "fft_generic.h"

namespace dbfft {

// ------------------------------------------------------------------ x/y passes
// Block = (column tile of TZ consecutive k3, one value of the other index,
// [component]).  The tile's lines are loaded with k3 fastest so each row of
// the tile is one contiguous run in HBM.
template <typename T, int MODE>
__global__ __launch_bounds__(kStridedThreads) void k_strided(const cpx<T>* in, cpx<T>* out, StridedGeom sg, Geom g,
                                                             FftPlan plan, const cpx<T>* __restrict__ twg,
                                                             T d, int TZ, double* __restrict__ dc_out,
                                                             const int* __restrict__ stop, AlphaTask at) {
  if (at.sc != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0)
    alpha_task_wave(at.sc, at.eparts, at.neparts);
  if (stop != nullptr && *stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  strided_core<T, MODE>(in, out, sg, g, plan, twg, d, TZ, dc_out, blockIdx.x, blockIdx.y, blockIdx.z, smem_raw);
}

static int strided_tile(int nline, int elem_bytes, int fused) {
  // contiguous run of >= 128 B per row; fused modes keep n*TZ within the
  // per-thread register budget.
  int tz = (elem_bytes == 16) ? 8 : 16;
  if (fused) {
    while (tz > 1 && nline * tz > kStridedQ * kStridedThreads) tz >>= 1;
  }
  while (tz > 1 && nline * tz * elem_bytes * 2 + nline * elem_bytes > 64 * 1024) tz >>= 1;
  return tz;
}

template <typename T>
void launch_strided(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                    const FftPlan& plan, const void* tw, int dir, double* dc_out, hipStream_t st,
                    const int* stop, const AlphaTask& at) {
  if (fast_strided_supported(sg.nline)) {
    launch_strided_fast<T>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at);
    return;
  }
  if (mixed_strided_supported(sg.nline)) {
    launch_strided_mixed<T>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at);
    return;
  }
  const int eb = (int)sizeof(cpx<T>);
  const int TZ = strided_tile(sg.nline, eb, mode != SP_PLAIN);
  const int ntiles = (sg.ncols + TZ - 1) / TZ;
  dim3 grid(ntiles, sg.nother, mode == SP_PLAIN ? ncomp_plain : 1);
  const size_t shm = (size_t)(sg.nline + 2 * sg.nline * TZ) * eb;
  const T d = (T)dir;
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  switch (mode) {
    case SP_PLAIN:
      DB_LAUNCH((k_strided<T, SP_PLAIN>), grid, dim3(kStridedThreads), shm, st, i, o, sg, g, plan, t, d, TZ, dc_out, stop, at);
      break;
    case SP_GRAD_SMALL:
      DB_LAUNCH((k_strided<T, SP_GRAD_SMALL>), grid, dim3(kStridedThreads), shm, st, i, o, sg, g, plan, t, d, TZ, dc_out, stop, at);
      break;
    case SP_GRAD_FINITE:
      DB_LAUNCH((k_strided<T, SP_GRAD_FINITE>), grid, dim3(kStridedThreads), shm, st, i, o, sg, g, plan, t, d, TZ, dc_out, stop, at);
      break;
    case SP_DIV_SMALL:
      DB_LAUNCH((k_strided<T, SP_DIV_SMALL>), grid, dim3(kStridedThreads), shm, st, i, o, sg, g, plan, t, d, TZ, dc_out, stop, at);
      break;
    default:
      DB_LAUNCH((k_strided<T, SP_DIV_FINITE>), grid, dim3(kStridedThreads), shm, st, i, o, sg, g, plan, t, d, TZ, dc_out, stop, at);
      break;
  }
}

template void launch_strided<double>(int, const void*, void*, int, const StridedGeom&, const Geom&, const FftPlan&,
                                     const void*, int, double*, hipStream_t, const int*, const AlphaTask&);
template void launch_strided<float>(int, const void*, void*, int, const StridedGeom&, const Geom&, const FftPlan&,
                                    const void*, int, double*, hipStream_t, const int*, const AlphaTask&);

// ------------------------------------------------------------------ z pass
// Block = L consecutive (x, y) lines.  A real transform of even length n3 is
// done as a complex transform of length n3/2 on z[n] = f[2n] + i f[2n+1] with
// the standard even/odd split before (C2R) or after (R2C); an odd n3 takes
// the full-length complex transform of the real samples.
template <typename T, int MODE, int KIN, int LAW>
__global__ __launch_bounds__(kLineThreads) void k_line(const void* in_v, void* out_v, Geom g, FftPlan plan,
                                                       const cpx<T>* __restrict__ twg,
                                                       const cpx<T>* __restrict__ rtwg, TangentArgs<T> tn,
                                                       const double* __restrict__ macro_dev,
                                                       const double* __restrict__ macro_add,
                                                       double* __restrict__ partials, int L, int ncomp,
                                                       const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  line_core<T, MODE, KIN, LAW>(in_v, out_v, g, plan, twg, rtwg, tn, macro_dev, macro_add, partials, L, ncomp,
                          (long long)blockIdx.x, smem_raw);
}

int line_lines_per_block(const Geom& g, int ncomp, int elem_bytes) {
  // about 512 voxels per block, bounded by LDS (64 KiB budget)
  int L = 512 / g.n3;
  if (L < 1) L = 1;
  if (L > 16) L = 16;
  while (L > 1 && line_smem_bytes(g, L, ncomp, elem_bytes) > 64 * 1024) --L;
  return L;
}

template <typename T>
void launch_line(int mode, int kin, const void* in, void* out, const Geom& g, const FftPlan& plan, const void* tw,
                 const void* rtw, const TangentArgs<T>& tan, const double* macro_dev, const double* macro_add,
                 double* partials, int ncomp, hipStream_t st, int* nblocks_out, const int* stop) {
  const bool iso = kin == KIN_SMALL && (tan.kind == TAN_ISO_PHASE || tan.kind == TAN_ISO_FIELD);
  if (mode == LP_FUSED && macro_add == nullptr &&
      staged_line_supported(g.n3, (int)sizeof(cpx<T>), iso, kin == KIN_FINITE)) {
    if (nblocks_out) *nblocks_out = staged_line_blocks(g);
    launch_line_staged<T>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
    return;
  }
  if (mode == LP_FUSED && macro_add == nullptr && fast_line_supported(g.n3)) {
    if (nblocks_out) *nblocks_out = fast_line_blocks(g, (int)sizeof(cpx<T>));
    launch_line_fast<T>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
    return;
  }
  if ((mode == LP_C2R || mode == LP_R2C) && ncomp <= 9 && real_line_supported(g.n3)) {
    if (nblocks_out) *nblocks_out = 0;
    launch_line_real<T>(mode, in, out, g, tw, rtw, macro_dev, macro_add, ncomp, st);
    return;
  }
  if (mode == LP_FUSED && macro_add == nullptr && iso && odd_line_supported(g.n3)) {
    if (nblocks_out) *nblocks_out = odd_line_energy_blocks(g);
    launch_line_odd<T>(in, out, g, tw, tan, macro_dev, partials, st, stop);
    return;
  }
  if (mode == LP_FUSED && macro_add == nullptr && mixed_line_supported(g.n3, (int)sizeof(cpx<T>), iso)) {
    if (nblocks_out) *nblocks_out = mixed_line_energy_blocks(g, iso);
    launch_line_mixed<T>(kin, iso, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop);
    return;
  }
  const int eb = (int)sizeof(cpx<T>);
  const int L = line_lines_per_block(g, ncomp, eb);
  const long long nlines = (long long)g.n1 * g.n2;
  const int nblk = (int)((nlines + L - 1) / L);
  if (nblocks_out) *nblocks_out = nblk;
  const size_t shm = line_smem_bytes(g, L, ncomp, eb);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
#define DBFFT_LINE(MD, KN, LW)                                                                                   \
  DB_LAUNCH((k_line<T, MD, KN, LW>), dim3(nblk), dim3(kLineThreads), shm, st, in, out, g, plan, t, r, tan,      \
            macro_dev, macro_add, partials, L, ncomp, stop)
  if (kin == KIN_SMALL) {
    switch (mode) {
      case LP_FUSED: DBFFT_LINE(LP_FUSED, KIN_SMALL, 0); break;
      case LP_C2R: DBFFT_LINE(LP_C2R, KIN_SMALL, 0); break;
      case LP_R2C: DBFFT_LINE(LP_R2C, KIN_SMALL, 0); break;
      case LP_STRESS: DBFFT_LINE(LP_STRESS, KIN_SMALL, 0); break;
      default: DBFFT_LINE(LP_CONST, KIN_SMALL, 0); break;
    }
  } else if (finite_law(tan.kind) == 2) {
    switch (mode) {
      case LP_FUSED: DBFFT_LINE(LP_FUSED, KIN_FINITE, 2); break;
      case LP_C2R: DBFFT_LINE(LP_C2R, KIN_FINITE, 2); break;
      case LP_R2C: DBFFT_LINE(LP_R2C, KIN_FINITE, 2); break;
      case LP_STRESS: DBFFT_LINE(LP_STRESS, KIN_FINITE, 2); break;
      default: DBFFT_LINE(LP_CONST, KIN_FINITE, 2); break;
    }
  } else {
    switch (mode) {
      case LP_FUSED: DBFFT_LINE(LP_FUSED, KIN_FINITE, 0); break;
      case LP_C2R: DBFFT_LINE(LP_C2R, KIN_FINITE, 0); break;
      case LP_R2C: DBFFT_LINE(LP_R2C, KIN_FINITE, 0); break;
      case LP_STRESS: DBFFT_LINE(LP_STRESS, KIN_FINITE, 0); break;
      default: DBFFT_LINE(LP_CONST, KIN_FINITE, 0); break;
    }
  }
#undef DBFFT_LINE
}

template void launch_line<double>(int, int, const void*, void*, const Geom&, const FftPlan&, const void*,
                                  const void*, const TangentArgs<double>&, const double*, const double*, double*,
                                  int, hipStream_t, int*, const int*);
template void launch_line<float>(int, int, const void*, void*, const Geom&, const FftPlan&, const void*,
                                 const void*, const TangentArgs<float>&, const double*, const double*, double*,
                                 int, hipStream_t, int*, const int*);

int fused_line_blocks(const Geom& g, int ncomp, int elem_bytes, int tan_kind) {
  const bool iso = (ncomp == 6) && (tan_kind == TAN_ISO_PHASE || tan_kind == TAN_ISO_FIELD);
  if (staged_line_supported(g.n3, elem_bytes, iso, ncomp == 9)) return staged_line_blocks(g);
  if (fast_line_supported(g.n3)) return fast_line_blocks(g, elem_bytes);
  if (iso && odd_line_supported(g.n3)) return odd_line_energy_blocks(g);
  if (mixed_line_supported(g.n3, elem_bytes, iso)) return mixed_line_energy_blocks(g, iso);
  const int L = line_lines_per_block(g, ncomp, elem_bytes);
  return (int)(((long long)g.n1 * g.n2 + L - 1) / L);
}

int line_block_count(const Geom& g) {
  const int L = line_lines_per_block(g, 9, 16);
  return (int)(((long long)g.n1 * g.n2 + L - 1) / L);
}

}  // namespace dbfft
