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
  int pad;
};

// flattened grids of one batched iteration (block offsets per cell are
// device arrays of ncell + 1 entries)
struct BatchLaunch {
  int ncell, kin, ncomp;
  int nbx_f, nby, nbz, nbv;
  const int* boff_xf;
  const int* boff_y;
  const int* boff_z;
  const int* boff_v;
  size_t lds_x, lds_y, lds_z;
};

template <typename T>
void launch_batch_iteration(const BatchLaunch& bl, const void* desc, hipStream_t st);
template <typename T>
void launch_batch_flags(const void* desc, int ncell, int* flags, hipStream_t st);
template <typename T>
float tune_strided_ms(const CellDesc<T>& R, int axis, int TZ, hipStream_t st, int reps);

}  // namespace dbfft
