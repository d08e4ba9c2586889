// Batched PCG over many cells of uneven grid sizes.
//
// One launch per pass covers every cell of the batch: the flattened grid is
// cut into consecutive block ranges, one per cell, and each block finds its
// cell in a device table of per-cell descriptors (geometry, FFT plans,
// twiddles, vectors, tangent, preconditioner, scalars).  Every cell keeps
// its own CG scalars and convergence flag; blocks of converged cells exit at
// once, so a fixed chunk of iterations can be captured in a HIP graph and
// replayed until every cell has converged.
#include "batch.h"
#include "fft_generic.h"
#include "fft_mixed.h"
#include "pcg_core.h"

namespace dbfft {

__device__ __forceinline__ int find_cell(const int* __restrict__ boff, int ncell, int b) {
  // last r with boff[r] <= b (boff is non-decreasing, boff[0] = 0)
  int lo = 0, hi = ncell - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Blocks are dispatched to the 8 XCDs round robin, and consecutive tiles
// of a pass share cache lines where rows are not line-aligned.  The blocks
// [b0, b1) of a cell are renumbered so that the tiles of each XCD are
// consecutive: the cell's blocks on XCD 0 take the first tiles, then those
// on XCD 1, and so on (a bijection onto 0 .. b1 - b0 - 1).
__device__ __forceinline__ int xcd_local(int b, int b0, int b1) {
  const int x = b & 7;
  int before = 0;
  for (int y = 0; y < x; ++y) {
    const int f = b0 + ((y - b0) & 7);  // first block of XCD y in the range
    if (f < b1) before += (b1 - 1 - f) / 8 + 1;
  }
  const int fx = b0 + ((x - b0) & 7);
  return before + (b - fx) / 8;
}

template <typename T>
__device__ __forceinline__ cpx<T>* buf_of(const CellDesc<T>& R, int which) {
  switch (which) {
    case BUF_W: return R.W;
    case BUF_X: return R.x;
    case BUF_R: return R.r;
    case BUF_P: return R.p;
    default: return R.q;
  }
}

// two-step tile of a cell's x or y pass; lb = component * tiles + tile
template <typename T, int N, int MODE>
__device__ __forceinline__ void batch_mixed_tile(const cpx<T>* in, cpx<T>* out, const StridedGeom& sg, const Geom& g,
                                                 const cpx<T>* twg, T d, double* dc, int lb,
                                                 unsigned char* smem_raw) {
  using S = MixedShape<N>;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* lds = tw + N;
  for (int i = threadIdx.x; i < N; i += kStridedThreads) tw[i] = twg[i];
  __syncthreads();
  const long long npair = (long long)sg.nother * sg.ncols;
  const long long ntile = (npair + S::TZ - 1) / S::TZ;
  const long long c = lb / ntile;
  const long long tile = lb - c * ntile;
  mixed_strided_tile<T, N, MODE>(in + c * sg.cstride_in, out + c * sg.cstride_out, sg, g, tw, lds, d, dc, tile,
                                 threadIdx.x);
}

// x pass (axis 0) or y pass (axis 1) of every cell.  GEN = false: every
// cell takes the two-step register transform on this axis, and the LDS
// Stockham engine (which needs more registers than the two-step tiles of
// the plain passes) is left out of the kernel.
template <typename T, int MODE, bool GEN>
__global__ __launch_bounds__(kStridedThreads) void kb_strided(const CellDesc<T>* __restrict__ D,
                                                              const int* __restrict__ boff, int ncell, int axis,
                                                              int src, int dst, int ncomp, T d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int r = find_cell(boff, ncell, blockIdx.x);
  const CellDesc<T>& R = D[r];
  if (R.sc->converged) return;
  const int lb = xcd_local(blockIdx.x, boff[r], boff[r + 1]);
  const Geom& g = R.g;
  StridedGeom sg;
  int tile, o, c, TZ;
  const FftPlan* plan;
  const cpx<T>* tw;
  if (axis == 0) {
    sg.nline = g.n1;
    sg.lstride = (long long)g.n2 * g.nh3;
    sg.ostride = g.nh3;
    sg.nother = g.n2;
    TZ = R.tzx;
    const int nt = (g.nh3 + TZ - 1) / TZ;
    tile = lb % nt;
    o = (lb / nt) % g.n2;
    c = lb / (nt * g.n2);
    plan = &R.p1;
    tw = R.tw1;
  } else {
    sg.nline = g.n2;
    sg.lstride = g.nh3;
    sg.ostride = (long long)g.n2 * g.nh3;
    sg.nother = g.n1;
    TZ = R.tzy;
    const int nt = (g.nh3 + TZ - 1) / TZ;
    tile = lb % nt;
    o = (lb / nt) % g.n1;
    c = lb / (nt * g.n1);
    plan = &R.p2;
    tw = R.tw2;
  }
  sg.ncols = g.nh3;
  sg.cstride_in = g.nh;
  sg.cstride_out = g.nh;
  (void)ncomp;
  double* dc = (MODE == SP_DIV_SMALL || MODE == SP_DIV_FINITE) ? R.dc : nullptr;
  if (axis == 0 ? R.mx : R.my) {
    switch (sg.nline) {
#define DBFFT_BM(NN) \
  case NN: batch_mixed_tile<T, NN, MODE>(buf_of(R, src), buf_of(R, dst), sg, g, tw, d, dc, lb, smem_raw); return;
      DBFFT_BM(12) DBFFT_BM(16) DBFFT_BM(18) DBFFT_BM(20) DBFFT_BM(24) DBFFT_BM(30) DBFFT_BM(32) DBFFT_BM(36)
      DBFFT_BM(40) DBFFT_BM(48) DBFFT_BM(50) DBFFT_BM(54) DBFFT_BM(60) DBFFT_BM(64) DBFFT_BM(72) DBFFT_BM(80)
      DBFFT_BM(90) DBFFT_BM(96)
#undef DBFFT_BM
      default: return;
    }
  }
  if constexpr (GEN) strided_core<T, MODE>(buf_of(R, src), buf_of(R, dst), sg, g, *plan, tw, d, TZ, dc, tile, o, c, smem_raw);
  else (void)plan;
}

// two-step z pass of a cell: four waves per block (each a line group of its
// own for isotropic tangents, else one line group for the block), one
// energy partial per block
template <typename T, int M, int KIN, int LAW>
__device__ __forceinline__ void batch_mixed_line(const CellDesc<T>& R, int lb, unsigned char* smem_raw) {
  using L = MixedLine<M>;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* rtw = tw + M;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cpx<T>* lds = rtw + M + 1 + w * L::LB * L::PITCH;
  __shared__ double ew[kLineThreads / 64];
  for (int i = threadIdx.x; i < M; i += kLineThreads) tw[i] = R.tw3[i];
  for (int i = threadIdx.x; i <= M; i += kLineThreads) rtw[i] = R.rtw[i];
  __syncthreads();
  const long long blk = (long long)lb * (kLineThreads / 64) + w;
  double e = 0.0;
  if (KIN == KIN_SMALL && R.mz == 1) {
    e = mixed_line_fused<T, M, KIN_SMALL, 1>(R.W, R.W, R.g, tw, rtw, lds, R.tan, R.sc->pmac, blk, lane);
  } else if constexpr (sizeof(T) == 4) {
    // anisotropic or finite-strain tangents: the block's four waves share
    // one line group
    cpx<T>* X = rtw + M + 1 + (kLineThreads / 64) * L::LB * L::PITCH;
    e = mixed_line_staged<T, M, KIN, LAW, kLineThreads / 64>(R.W, R.W, R.g, tw, rtw, lds, X, R.tan, R.sc->pmac, lb,
                                                              w, lane);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
  }
  if (lane == 0) ew[w] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kLineThreads / 64; ++i) s += ew[i];
    R.partA[lb] = s;
  }
}

// GEN = false: every cell takes the two-step z pass (no LDS engine in the kernel)
template <typename T, int KIN, int LAW, bool GEN>
__global__ __launch_bounds__(kLineThreads) void kb_line(const CellDesc<T>* __restrict__ D, const int* __restrict__ boff,
                                                        int ncell, int ncomp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int r = find_cell(boff, ncell, blockIdx.x);
  const CellDesc<T>& R = D[r];
  if (R.sc->converged) return;
  const int lb = blockIdx.x - boff[r];
  if (R.mz) {
    switch (R.g.n3 / 2) {
#define DBFFT_BZ(MM) \
  case MM: batch_mixed_line<T, MM, KIN, LAW>(R, lb, smem_raw); return;
      DBFFT_BZ(12) DBFFT_BZ(16) DBFFT_BZ(18) DBFFT_BZ(20) DBFFT_BZ(24) DBFFT_BZ(25) DBFFT_BZ(27) DBFFT_BZ(30)
      DBFFT_BZ(32) DBFFT_BZ(36) DBFFT_BZ(40) DBFFT_BZ(45) DBFFT_BZ(48) DBFFT_BZ(50) DBFFT_BZ(54) DBFFT_BZ(60)
      DBFFT_BZ(64)
#undef DBFFT_BZ
      default: return;
    }
  }
  if constexpr (GEN)
    line_core<T, LP_FUSED, KIN, LAW>(R.W, R.W, R.g, R.p3, R.tw3, R.rtw, R.tan, R.sc->pmac, nullptr, R.partA, R.L,
                                     ncomp, (long long)lb, smem_raw);
}

// r -= alpha q and the partial sums of beta (x is updated by kb_xp)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void kb_update(const CellDesc<T>* __restrict__ D, const int* __restrict__ boff,
                                                         int ncell) {
  const int r = find_cell(boff, ncell, blockIdx.x);
  const CellDesc<T>& R = D[r];
  const int lb = blockIdx.x - boff[r];
  update_core<T>(nullptr, R.r, R.p, R.q, R.sc, R.pa, R.g, R.partB, lb, boff[r + 1] - boff[r]);
}

// x += alpha p (the step alpha_core left pending), then p = M r + beta p
template <typename T>
__global__ __launch_bounds__(kVecThreads) void kb_xp(const CellDesc<T>* __restrict__ D, const int* __restrict__ boff,
                                                     int ncell) {
  const int r = find_cell(boff, ncell, blockIdx.x);
  const CellDesc<T>& R = D[r];
  const int lb = blockIdx.x - boff[r];
  xp_core<T>(R.x, R.p, R.r, R.sc, R.pa, R.g, lb, boff[r + 1] - boff[r]);
}

// one block per cell
template <typename T>
__global__ __launch_bounds__(kVecThreads) void kb_alpha(const CellDesc<T>* __restrict__ D, const int* __restrict__ bz) {
  const int r = blockIdx.x;
  const CellDesc<T>& R = D[r];
  alpha_core(R.sc, R.partA, bz[r + 1] - bz[r], R.dc, R.pc);
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void kb_beta(const CellDesc<T>* __restrict__ D, const int* __restrict__ bv) {
  const int r = blockIdx.x;
  const CellDesc<T>& R = D[r];
  beta_core(R.sc, R.partB, bv[r + 1] - bv[r], R.pc, 0);
}

template <typename T>
__global__ void kb_flags(const CellDesc<T>* __restrict__ D, int ncell, int* __restrict__ flags) {
  for (int r = threadIdx.x; r < ncell; r += blockDim.x) flags[r] = D[r].sc->converged;
}

template <typename T, int MODE>
static void launch_kb_strided(const BatchLaunch& bl, const CellDesc<T>* D, int axis, int src, int dst, T d,
                              hipStream_t st) {
  const dim3 ts(kStridedThreads);
  const int nb = axis == 0 ? bl.nbx_f : bl.nby;
  const int* boff = axis == 0 ? bl.boff_xf : bl.boff_y;
  const size_t lds = axis == 0 ? bl.lds_x : bl.lds_y;
  if (axis == 0 ? bl.gen_x : bl.gen_y)
    hipLaunchKernelGGL((kb_strided<T, MODE, true>), dim3(nb), ts, lds, st, D, boff, bl.ncell, axis, src, dst, bl.ncomp, d);
  else
    hipLaunchKernelGGL((kb_strided<T, MODE, false>), dim3(nb), ts, lds, st, D, boff, bl.ncell, axis, src, dst, bl.ncomp,
                       d);
}

template <typename T, int KIN, int LAW>
static void launch_kb_line(const BatchLaunch& bl, const CellDesc<T>* D, hipStream_t st) {
  const dim3 ls(kLineThreads);
  if (bl.gen_z)
    hipLaunchKernelGGL((kb_line<T, KIN, LAW, true>), dim3(bl.nbz), ls, bl.lds_z, st, D, bl.boff_z, bl.ncell, bl.ncomp);
  else
    hipLaunchKernelGGL((kb_line<T, KIN, LAW, false>), dim3(bl.nbz), ls, bl.lds_z, st, D, bl.boff_z, bl.ncell, bl.ncomp);
}

template <typename T>
void launch_batch_iteration(const BatchLaunch& bl, const void* desc, hipStream_t st) {
  auto D = static_cast<const CellDesc<T>*>(desc);
  const dim3 vs(kVecThreads);
  // x inverse + gradient: a = p -> W
  if (bl.kin == KIN_SMALL) launch_kb_strided<T, SP_GRAD_SMALL>(bl, D, 0, BUF_P, BUF_W, (T)1, st);
  else launch_kb_strided<T, SP_GRAD_FINITE>(bl, D, 0, BUF_P, BUF_W, (T)1, st);
  // y inverse, all components
  launch_kb_strided<T, SP_PLAIN>(bl, D, 1, BUF_W, BUF_W, (T)1, st);
  // z: C2R, tangent, R2C
  if (bl.kin == KIN_SMALL) launch_kb_line<T, KIN_SMALL, 0>(bl, D, st);
  else if (bl.law == 2) launch_kb_line<T, KIN_FINITE, 2>(bl, D, st);
  else launch_kb_line<T, KIN_FINITE, 0>(bl, D, st);
  // y forward
  launch_kb_strided<T, SP_PLAIN>(bl, D, 1, BUF_W, BUF_W, (T)-1, st);
  // x forward + divergence: W -> q
  if (bl.kin == KIN_SMALL) launch_kb_strided<T, SP_DIV_SMALL>(bl, D, 0, BUF_W, BUF_Q, (T)-1, st);
  else launch_kb_strided<T, SP_DIV_FINITE>(bl, D, 0, BUF_W, BUF_Q, (T)-1, st);
  hipLaunchKernelGGL((kb_alpha<T>), dim3(bl.ncell), vs, 0, st, D, bl.boff_z);
  hipLaunchKernelGGL((kb_update<T>), dim3(bl.nbv), vs, 0, st, D, bl.boff_v, bl.ncell);
  hipLaunchKernelGGL((kb_beta<T>), dim3(bl.ncell), vs, 0, st, D, bl.boff_v);
  hipLaunchKernelGGL((kb_xp<T>), dim3(bl.nbv), vs, 0, st, D, bl.boff_v, bl.ncell);
}

template <typename T>
void launch_batch_flags(const void* desc, int ncell, int* flags, hipStream_t st) {
  hipLaunchKernelGGL((kb_flags<T>), dim3(1), dim3(256), 0, st, static_cast<const CellDesc<T>*>(desc), ncell, flags);
}

template void launch_batch_iteration<double>(const BatchLaunch&, const void*, hipStream_t);
template void launch_batch_iteration<float>(const BatchLaunch&, const void*, hipStream_t);
template void launch_batch_flags<double>(const void*, int, int*, hipStream_t);
template void launch_batch_flags<float>(const void*, int, int*, hipStream_t);

// timing helper of the tile autotuner: one plain y or x pass of a cell
template <typename T>
__global__ __launch_bounds__(kStridedThreads) void kb_tune(CellDesc<T> R, int axis, int TZ, T d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Geom& g = R.g;
  StridedGeom sg;
  int tile, o;
  const int nt = (g.nh3 + TZ - 1) / TZ;
  tile = blockIdx.x % nt;
  o = blockIdx.x / nt;
  if (axis == 0) {
    sg.nline = g.n1;
    sg.lstride = (long long)g.n2 * g.nh3;
    sg.ostride = g.nh3;
    sg.nother = g.n2;
  } else {
    sg.nline = g.n2;
    sg.lstride = g.nh3;
    sg.ostride = (long long)g.n2 * g.nh3;
    sg.nother = g.n1;
  }
  sg.ncols = g.nh3;
  sg.cstride_in = g.nh;
  sg.cstride_out = g.nh;
  strided_core<T, SP_PLAIN>(R.W, R.W, sg, g, axis == 0 ? R.p1 : R.p2, axis == 0 ? R.tw1 : R.tw2, d, TZ, nullptr, tile,
                            o, 0, smem_raw);
}

template <typename T>
float tune_strided_ms(const CellDesc<T>& R, int axis, int TZ, hipStream_t st, int reps) {
  const Geom& g = R.g;
  const int n = axis == 0 ? g.n1 : g.n2;
  const int nother = axis == 0 ? g.n2 : g.n1;
  const int nt = (g.nh3 + TZ - 1) / TZ;
  const size_t shm = (size_t)(n + 2 * n * TZ) * sizeof(cpx<T>);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.f;
  }
  hipLaunchKernelGGL((kb_tune<T>), dim3(nt * nother), dim3(kStridedThreads), shm, st, R, axis, TZ, (T)1);
  (void)hipEventRecord(e0, st);
  for (int i = 0; i < reps; ++i)
    hipLaunchKernelGGL((kb_tune<T>), dim3(nt * nother), dim3(kStridedThreads), shm, st, R, axis, TZ, (T)1);
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  float ms = -1.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}
template float tune_strided_ms<double>(const CellDesc<double>&, int, int, hipStream_t, int);
template float tune_strided_ms<float>(const CellDesc<float>&, int, int, hipStream_t, int);

}  // namespace dbfft
