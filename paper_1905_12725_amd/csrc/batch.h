// Per-cell descriptors and launch plan of the batched PCG (batch.hip).
#pragma once

#include "fft_common.h"

namespace dbfft {

enum BatchBuf : int { BUF_W = 0, BUF_X = 1, BUF_R = 2, BUF_P = 3, BUF_Q = 4 };

template <typename T>
struct CellDesc {
  Geom g;
  FftPlan p1, p2, p3;
  const cpx<T>* tw1;
  const cpx<T>* tw2;
  const cpx<T>* tw3;
  const cpx<T>* rtw;
  cpx<T>* W;
  cpx<T>* x;
  cpx<T>* r;
  cpx<T>* p;
  cpx<T>* q;
  TangentArgs<T> tan;
  PrecondArgs pa;
  PcgConst pc;
  PcgScalars* sc;
  double* partA;  // energy partials of the z pass
  double* partB;  // update partials
  double* dc;     // average stress of the direction (DC bin of the divergence pass)
  int tzx, tzy;   // column tile widths of the x and y passes (autotuned)
  int L;          // z lines per block
  int mx, my;     // x / y pass with the two-step register transform
  int mz;         // z pass: 0 LDS engine, 1 two-step isotropic, 2 two-step general (FP32)
};

// flattened grids of one batched iteration (block offsets per cell are
// device arrays of ncell + 1 entries)
struct BatchLaunch {
  int ncell, kin, ncomp;
  int law;  // finite strains: 2 Saint Venant-Kirchhoff, 0 neo-Hookean
  int nbx_f, nby, nbz, nbv;
  const int* boff_xf;
  const int* boff_y;
  const int* boff_z;
  const int* boff_v;
  size_t lds_x, lds_y, lds_z;
  int gen_x, gen_y, gen_z;  // 1: some cell needs the LDS Stockham engine on this axis
};

// line lengths the batched two-step kernels are compiled for (x/y: n; z: n3/2)
constexpr bool batch_two_step_xy(int n) {
  switch (n) {
    case 12: case 16: case 18: case 20: case 24: case 30: case 32: case 36: case 40: case 48: case 50: case 54:
    case 60: case 64: case 72: case 80: case 90: case 96: return true;
    default: return false;
  }
}
constexpr bool batch_two_step_z(int m) {
  switch (m) {
    case 12: case 16: case 18: case 20: case 24: case 25: case 27: case 30: case 32: case 36: case 40: case 45:
    case 48: case 50: case 54: case 60: case 64: return true;
    default: return false;
  }
}

template <typename T>
void launch_batch_iteration(const BatchLaunch& bl, const void* desc, hipStream_t st);
template <typename T>
void launch_batch_flags(const void* desc, int ncell, int* flags, hipStream_t st);
template <typename T>
float tune_strided_ms(const CellDesc<T>& R, int axis, int TZ, hipStream_t st, int reps);

}  // namespace dbfft
