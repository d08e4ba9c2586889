// Register-resident FFT passes for power-of-two transform lengths.
//
// A length-N transform is spread over TL = N/8 threads that hold 8 elements
// each.  Every Stockham stage (radix 8, 4 or 2) is done in registers; LDS is
// used only to exchange elements between stages, in place.  The element
// distribution is fixed at compile time:
//   stage-0 input  : register r of thread t holds index t + TL*r
//   last output    : register q*R + r holds index t + TL*(q + NB*r),
//                    R the last radix and NB = 8/R butterflies per thread.
// The inverse transform's output distribution equals the forward
// transform's input distribution after a register renaming, so the z pass
// applies the pointwise tangent with no data movement at all.
#include "fft_common.h"
#include "fft_generic.h"
#include "pcg_core.h"

namespace dbfft {

// Radices of the stages: 8, then 4, then 2 (no radix above E).
template <int N, int E>
constexpr int fast_nstages() {
  int m = N, s = 0;
  if (E >= 8)
    while (m % 8 == 0) { m /= 8; ++s; }
  while (m % 4 == 0) { m /= 4; ++s; }
  while (m % 2 == 0) { m /= 2; ++s; }
  return s;
}
template <int N, int E>
constexpr int fast_radix(int st) {
  int m = N, s = 0;
  if (E >= 8)
    while (m % 8 == 0) { if (s == st) return 8; m /= 8; ++s; }
  while (m % 4 == 0) { if (s == st) return 4; m /= 4; ++s; }
  while (m % 2 == 0) { if (s == st) return 2; m /= 2; ++s; }
  return 1;
}
template <int N, int E>
constexpr int fast_ns(int st) {
  int p = 1;
  for (int s = 0; s < st; ++s) p *= fast_radix<N, E>(s);
  return p;
}

// radix-R butterflies of stage ST on the E registers of thread t
template <typename T, int N, int E, int ST>
__device__ __forceinline__ void fast_stage(cpx<T>* v, int t, const cpx<T>* __restrict__ tw, T d) {
  constexpr int R = fast_radix<N, E>(ST);
  constexpr int NS = fast_ns<N, E>(ST);
  constexpr int TL = N / E;
  constexpr int NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cpx<T>* b = v + q * R;
    if constexpr (NS > 1) {
      const int j = t + TL * q;
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[k * r * (N / (NS * R))];
        w.y *= -d;
        b[r] = mul(b[r], w);
      }
    }
    dftR<T, R>(b, d);
  }
}

// padded position of element i: one empty slot after every 2^PS elements
// (PS = 0: no padding), so strided exchange patterns spread over the banks
template <int PS>
__device__ __forceinline__ constexpr int fast_pad(int i) {
  return PS > 0 ? i + (i >> PS) : i;
}

// write the outputs of stage ST to LDS and read the inputs of stage ST+1;
// element index i of a sequence lives at lds[pad(i) * pitch + lane_off]
template <typename T, int N, int E, int ST, int PS = 0>
__device__ __forceinline__ void fast_exchange(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off) {
  constexpr int R = fast_radix<N, E>(ST), NS = fast_ns<N, E>(ST), NB = E / R;
  constexpr int R2 = fast_radix<N, E>(ST + 1), NB2 = E / R2;
  constexpr int TL = N / E;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + TL * q;
    const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[fast_pad<PS>(base + r * NS) * pitch + off] = v[q * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB2; ++q) {
    const int j = t + TL * q;
#pragma unroll
    for (int r = 0; r < R2; ++r) v[q * R2 + r] = lds[fast_pad<PS>(j + r * (N / R2)) * pitch + off];
  }
  __syncthreads();
}

template <typename T, int N, int E, int ST, int PS>
__device__ __forceinline__ void fast_fft_from(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off,
                                              const cpx<T>* __restrict__ tw, T d) {
  fast_stage<T, N, E, ST>(v, t, tw, d);
  if constexpr (ST + 1 < fast_nstages<N, E>()) {
    fast_exchange<T, N, E, ST, PS>(v, t, lds, pitch, off);
    fast_fft_from<T, N, E, ST + 1, PS>(v, t, lds, pitch, off, tw, d);
  }
}

// full transform of the E registers (stage-0 input -> last-stage output)
template <typename T, int N, int E, int PS = 0>
__device__ __forceinline__ void fast_fft(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off,
                                         const cpx<T>* __restrict__ tw, T d) {
  fast_fft_from<T, N, E, 0, PS>(v, t, lds, pitch, off, tw, d);
}

// index of output register g (= q*R + r) of thread t
template <int N, int E>
__device__ __forceinline__ constexpr int fast_out_pos(int g) {
  constexpr int R = fast_radix<N, E>(fast_nstages<N, E>() - 1);
  constexpr int NB = E / R;
  return (g / R) + NB * (g % R);  // q + NB r, times TL plus t
}

// ------------------------------------------------------------------ x / y passes
// Elements per thread: 4 for the passes that keep several vectors live
// (gradient, divergence), 8 for the plain ones.
template <typename T, int N, int MODE>
constexpr int strided_E() {
  return (MODE != SP_PLAIN && N <= 128) ? 4 : 8;
}
template <int N, int E>
struct StridedShape {
  static constexpr int TL = N / E;
  // at most 256 threads, at most 32 columns unless needed for one full wave
  static constexpr int TZ = (256 / TL) < 32 ? (256 / TL) : ((64 / TL) > 32 ? (64 / TL) : 32);
  static constexpr int NT = TL * TZ;
  static constexpr int PITCH = TZ + 1;
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__((StridedShape<N, strided_E<T, N, MODE>()>::NT)) void k_strided_fast(const cpx<T>* in, cpx<T>* out, StridedGeom sg,
                                                                      Geom g, const cpx<T>* __restrict__ twg, T d,
                                                                      double* __restrict__ dc_out,
                                                                      const int* __restrict__ stop,
                                                                      PcgScalars* alpha_sc, const double* eparts,
                                                                      int neparts) {
  if (alpha_sc != nullptr && blockIdx.x == 0 && blockIdx.z == 0)
    alpha_task<StridedShape<N, strided_E<T, N, MODE>()>::NT>(alpha_sc, eparts, neparts);
  if (stop != nullptr && *stop) return;
  constexpr int E = strided_E<T, N, MODE>();
  using S = StridedShape<N, E>;
  constexpr int TL = S::TL, TZ = S::TZ, NT = S::NT, PITCH = S::PITCH;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[N * PITCH];
  const int tid = threadIdx.x;
  const int s = tid % TZ, t = tid / TZ;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();
  // The (other index, column) pairs are numbered with the column fastest
  // and cut into tiles of TZ consecutive pairs, so every tile is full (the
  // half-spectrum column count n3/2 + 1 is not a multiple of TZ).  Tiles
  // are renumbered so that consecutive tiles, which share cache lines when
  // rows are not line-aligned, run on the same XCD (blocks are dispatched
  // to the 8 XCDs round robin).
  const int nb = gridDim.x;
  const int per = nb >> 3;
  const int b = blockIdx.x;
  const int tile = (b < (per << 3)) ? (b & 7) * per + (b >> 3) : b;
  const long long npair = (long long)sg.nother * sg.ncols;
  const long long pr = (long long)tile * TZ + s;
  const bool valid = pr < npair;
  const int o = valid ? (int)(pr / sg.ncols) : 0;
  const int col = valid ? (int)(pr - (long long)o * sg.ncols) : 0;
  const long long base = (long long)o * sg.ostride + col;
  const long long ls = sg.lstride;

  auto loadv = [&](const cpx<T>* src, cpx<T>* v) {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = valid ? src[base + (long long)(t + TL * r) * ls] : mk<T>(0, 0);
  };
  auto storev = [&](cpx<T>* dst, const cpx<T>* v) {
    if (!valid) return;
#pragma unroll
    for (int gq = 0; gq < E; ++gq) dst[base + (long long)(t + TL * fast_out_pos<N, E>(gq)) * ls] = v[gq];
  };

  if constexpr (MODE == SP_PLAIN) {
    const int c = blockIdx.z;
    cpx<T> v[E];
    loadv(in + c * sg.cstride_in, v);
    fast_fft<T, N, E>(v, t, lds, PITCH, s, tw, d);
    storev(out + c * sg.cstride_out, v);
  } else if constexpr (MODE == SP_GRAD_SMALL) {
    // x pass, line = k1, other = k2, column = k3: each strain component
    // eps_ij = i/2 (xi_j a_i + xi_i a_j) is formed on the coefficients (xi1
    // varies along the line) and transformed on its own; the three
    // displacement components are loaded once, up front.
    const T xi2 = (T)xi_of(o, g.n2, g.il2);
    const T xi3 = (T)xi_of(col, g.n3, g.il3);
    const long long co = sg.cstride_out;
    cpx<T> A0[E], A1[E], A2[E];
    loadv(in, A0);
    loadv(in + sg.cstride_in, A1);
    loadv(in + 2 * sg.cstride_in, A2);
    auto emit = [&](int c, auto&& form) {
      cpx<T> v[E];
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = form(r, (T)xi_of(t + TL * r, g.n1, g.il1));
      fast_fft<T, N, E>(v, t, lds, PITCH, s, tw, d);
      storev(out + c * co, v);
    };
    // stored order 11 22 33 23 13 12
    emit(0, [&](int r, T x1) { return muli(scl(A0[r], x1), (T)1); });
    emit(1, [&](int r, T) { return muli(scl(A1[r], xi2), (T)1); });
    emit(2, [&](int r, T) { return muli(scl(A2[r], xi3), (T)1); });
    emit(3, [&](int r, T) { return muli(scl(add(scl(A1[r], xi3), scl(A2[r], xi2)), (T)0.5), (T)1); });
    emit(4, [&](int r, T x1) { return muli(scl(add(scl(A0[r], xi3), scl(A2[r], x1)), (T)0.5), (T)1); });
    emit(5, [&](int r, T x1) { return muli(scl(add(scl(A0[r], xi2), scl(A1[r], x1)), (T)0.5), (T)1); });
  } else if constexpr (MODE == SP_GRAD_FINITE) {
    // With T_i = FFT(a_i) and U_i = FFT(xi1 a_i): H_i1 = i U_i,
    // H_i2 = i xi2 T_i, H_i3 = i xi3 T_i (six transforms for nine outputs).
    const T xi2 = (T)xi_of(o, g.n2, g.il2);
    const T xi3 = (T)xi_of(col, g.n3, g.il3);
    T xi1[E];
#pragma unroll
    for (int r = 0; r < E; ++r) xi1[r] = (T)xi_of(t + TL * r, g.n1, g.il1);
    const long long co = sg.cstride_out;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> Ti[E], U[E];
      loadv(in + i * sg.cstride_in, Ti);
#pragma unroll
      for (int r = 0; r < E; ++r) U[r] = scl(Ti[r], xi1[r]);
      fast_fft<T, N, E>(Ti, t, lds, PITCH, s, tw, d);
      fast_fft<T, N, E>(U, t, lds, PITCH, s, tw, d);
      cpx<T> w[E];
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = muli(U[r], (T)1);
      storev(out + (3 * i + 0) * co, w);
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = muli(scl(Ti[r], xi2), (T)1);
      storev(out + (3 * i + 1) * co, w);
#pragma unroll
      for (int r = 0; r < E; ++r) w[r] = muli(scl(Ti[r], xi3), (T)1);
      storev(out + (3 * i + 2) * co, w);
    }
  } else if constexpr (MODE == SP_DIV_SMALL) {
    // r_i = -i sum_j xi_j s_ij after the forward x transform; three row
    // accumulators, the next stress component loaded while the current one
    // is transformed.
    const T xi2 = (T)xi_of(o, g.n2, g.il2);
    const T xi3 = (T)xi_of(col, g.n3, g.il3);
    cpx<T> a0[E], a1[E], a2[E];
#pragma unroll
    for (int r = 0; r < E; ++r) a0[r] = a1[r] = a2[r] = mk<T>(0, 0);
    cpx<T> nx[E];
    loadv(in, nx);
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
      cpx<T> v[E];
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = nx[r];
      if (c + 1 < 6) loadv(in + (c + 1) * sg.cstride_in, nx);
      fast_fft<T, N, E>(v, t, lds, PITCH, s, tw, d);
      if (dc_out != nullptr && valid && o == 0 && col == 0 && t == 0) dc_out[c] = (double)v[0].x;
      // stored order 11 22 33 23 13 12
      const int ii = (c < 3) ? c : (c == 3 ? 1 : 0);
      const int jj = (c < 3) ? c : (c == 5 ? 1 : 2);
#pragma unroll
      for (int gq = 0; gq < E; ++gq) {
        const T x1 = (T)xi_of(t + TL * fast_out_pos<N, E>(gq), g.n1, g.il1);
        const T xj = (jj == 0) ? x1 : (jj == 1 ? xi2 : xi3);
        const T xi_ = (ii == 0) ? x1 : (ii == 1 ? xi2 : xi3);
        const cpx<T> t1 = scl(v[gq], xj);
        if (ii == 0) a0[gq] = add(a0[gq], t1);
        else if (ii == 1) a1[gq] = add(a1[gq], t1);
        else a2[gq] = add(a2[gq], t1);
        if (ii != jj) {
          const cpx<T> t2 = scl(v[gq], xi_);
          if (jj == 0) a0[gq] = add(a0[gq], t2);
          else if (jj == 1) a1[gq] = add(a1[gq], t2);
          else a2[gq] = add(a2[gq], t2);
        }
      }
    }
#pragma unroll
    for (int gq = 0; gq < E; ++gq) {
      a0[gq] = muli(a0[gq], (T)-1);
      a1[gq] = muli(a1[gq], (T)-1);
      a2[gq] = muli(a2[gq], (T)-1);
    }
    storev(out, a0);
    storev(out + sg.cstride_out, a1);
    storev(out + 2 * sg.cstride_out, a2);
  } else {
    // SP_DIV_FINITE, row by row: r_i = -i (xi1 F[P_i1] + F[xi2 P_i2 + xi3 P_i3])
    // (xi2, xi3 are constant along the line, so they are applied before the
    // transform): six transforms for the nine components, one row live, the
    // next row's components loaded while the current row is transformed.
    const T xi2 = (T)xi_of(o, g.n2, g.il2);
    const T xi3 = (T)xi_of(col, g.n3, g.il3);
    const bool dcl = dc_out != nullptr && valid && o == 0 && col == 0;
    cpx<T> P1[E], P2[E], P3[E];
    loadv(in, P1);
    loadv(in + sg.cstride_in, P2);
    loadv(in + 2 * sg.cstride_in, P3);
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      cpx<T> C[E], A[E];
      T dsum[3] = {0, 0, 0};
#pragma unroll
      for (int r = 0; r < E; ++r) {
        C[r] = add(scl(P2[r], xi2), scl(P3[r], xi3));
        A[r] = P1[r];
        if (dcl) {
          dsum[0] += P1[r].x;
          dsum[1] += P2[r].x;
          dsum[2] += P3[r].x;
        }
      }
      if (dcl) {
        // line sums (the k1 = 0 coefficient) of P_i1, P_i2, P_i3: the 16
        // threads of the line reduce through the exchange buffer
#pragma unroll
        for (int j = 0; j < 3; ++j) lds[t * PITCH + j] = mk<T>(dsum[j], 0);
      }
      if (i + 1 < 3) {
        loadv(in + (3 * i + 3) * sg.cstride_in, P1);
        loadv(in + (3 * i + 4) * sg.cstride_in, P2);
        loadv(in + (3 * i + 5) * sg.cstride_in, P3);
      }
      if (dc_out != nullptr && blockIdx.x == 0) {
        __syncthreads();
        if (dcl && t == 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int u = 0; u < TL; ++u) acc += (double)lds[u * PITCH + j].x;
            dc_out[3 * i + j] = acc;
          }
        }
        __syncthreads();
      }
      fast_fft<T, N, E>(C, t, lds, PITCH, s, tw, d);
      fast_fft<T, N, E>(A, t, lds, PITCH, s, tw, d);
#pragma unroll
      for (int gq = 0; gq < E; ++gq) {
        const T x1 = (T)xi_of(t + TL * fast_out_pos<N, E>(gq), g.n1, g.il1);
        A[gq] = muli(add(scl(A[gq], x1), C[gq]), (T)-1);
      }
      storev(out + i * sg.cstride_out, A);
    }
  }
}

// Fused CG step in the last forward pass (small strains).
//  * alpha is already in the scalars (computed by the first block of the
//    preceding y pass, or by the alpha kernel).
//  * The divergence q = -i xi . sigma_hat stays in registers and
//    r -= alpha q is applied at once.
//  * The first tiles take the self-conjugate columns k3 = 0 and n3/2 with
//    the k2 lines ordered 0, n2/2, 1, n2-1, 2, n2-2, ..., so the Hermitian
//    partner line (-k2) of every plane line sits in the neighbouring tile
//    column (or is the line itself); these plane tiles project r onto
//    Hermitian pairs through LDS before storing it.  The other tiles take
//    the (k2, k3) pairs in their natural order (line-aligned) and leave the
//    self-conjugate columns out.
//  * Block partial sums of <r, M r> and <r, r> (weight 2 off the planes, 1 on
//    them, where both points of a pair are counted).
template <int TZ>
__host__ __device__ __forceinline__ long long div_plane_pad(int n2) {
  return (2LL * n2 + TZ - 1) / TZ * TZ;
}

template <int TZ>
__device__ __forceinline__ void div_pair(long long pr, int n2, int nh3, bool& valid, int& o, int& col,
                                         int& sp_xor) {
  const long long Pp = div_plane_pad<TZ>(n2);
  valid = true;
  sp_xor = 0;
  if (pr >= Pp) {
    // interior tile: natural (k2, k3) order, self-conjugate columns left out
    const long long q = pr - Pp;
    o = (int)(q / nh3);
    col = (int)(q - (long long)o * nh3);
    if (o >= n2 || col == 0 || col == nh3 - 1) valid = false;
    if (o >= n2) o = 0;
    return;
  }
  if (pr >= 2LL * n2) {
    valid = false;
    o = 0;
    col = 0;
    return;
  }
  const int plane = (int)(pr / n2), j = (int)(pr - (long long)plane * n2);
  col = plane ? nh3 - 1 : 0;
  if (j == 0) o = 0;
  else if (j == 1) o = n2 / 2;
  else {
    o = (j & 1) ? n2 - j / 2 : j / 2;
    sp_xor = 1;
  }
}

// Row of the divergence a stored stress component (11 22 33 23 13 12)
// enters through its first index, and the row it enters through its second.
__host__ __device__ constexpr int div_row_i(int c) { return c < 3 ? c : (c == 3 ? 1 : 0); }
__host__ __device__ constexpr int div_row_j(int c) { return c < 3 ? c : (c == 5 ? 1 : 2); }

template <typename T, int N>
__global__ __launch_bounds__((StridedShape<N, strided_E<T, N, SP_DIV_SMALL>()>::NT)) void k_div_update_fast(
    const cpx<T>* in, cpx<T>* r, StridedGeom sg, Geom g, const cpx<T>* __restrict__ twg,
    const PcgScalars* __restrict__ sc, PrecondArgs pa, double* __restrict__ dc_out, double* __restrict__ partials) {
  constexpr int E = strided_E<T, N, SP_DIV_SMALL>();
  using S = StridedShape<N, E>;
  constexpr int TL = S::TL, TZ = S::TZ, NT = S::NT, PITCH = S::PITCH;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> lds[N * PITCH];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  if (sc->converged) return;
  const int s = tid % TZ, t = tid / TZ;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();
  const int nb = gridDim.x;
  const int per = nb >> 3;
  const int b = blockIdx.x;
  const int tile = (b < (per << 3)) ? (b & 7) * per + (b >> 3) : b;
  const bool plane_tile = (long long)tile * TZ < div_plane_pad<TZ>(sg.nother);
  bool valid;
  int o, col, sp_xor;
  div_pair<TZ>((long long)tile * TZ + s, sg.nother, sg.ncols, valid, o, col, sp_xor);
  const long long base = (long long)o * sg.ostride + col;
  const long long ls = sg.lstride;
  const T d = (T)-1;
  auto loadv = [&](const cpx<T>* src, cpx<T>* v) {
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = valid ? src[base + (long long)(t + TL * q) * ls] : mk<T>(0, 0);
  };
  const T xi2 = (T)xi_of(o, g.n2, g.il2);
  const T xi3 = (T)xi_of(col, g.n3, g.il3);
  // a_i = sum_j xi_j s_ij on the output distribution of the transform
  cpx<T> acc[3][E];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int q = 0; q < E; ++q) acc[i][q] = mk<T>(0, 0);
  cpx<T> nx[E];
  loadv(in, nx);
  // Six stress components in a rolled loop: the next one is loaded while
  // this one is transformed, then it is added to every row with its
  // coefficient (zero for the rows it does not enter), so no accumulator is
  // selected at run time.
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
    cpx<T> v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = nx[q];
    if (c + 1 < 6) loadv(in + (c + 1) * sg.cstride_in, nx);
    fast_fft<T, N, E>(v, t, lds, PITCH, s, tw, d);
    if (dc_out != nullptr && valid && o == 0 && col == 0 && t == 0) dc_out[c] = (double)v[0].x;
    const int ii = div_row_i(c), jj = div_row_j(c);
#pragma unroll
    for (int gq = 0; gq < E; ++gq) {
      const T x1 = (T)xi_of(t + TL * fast_out_pos<N, E>(gq), g.n1, g.il1);
      const T xj = (jj == 0) ? x1 : (jj == 1 ? xi2 : xi3);
      const T xi_ = (ii == 0) ? x1 : (ii == 1 ? xi2 : xi3);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T cf = (k == ii ? xj : (T)0) + ((k == jj && ii != jj) ? xi_ : (T)0);
        acc[k][gq] = add(acc[k][gq], scl(v[gq], cf));
      }
    }
  }

  const long long cs = sg.cstride_out;
  const double alpha = sc->alpha;
  // r -= alpha q with q = -i a, rounded to the storage precision
  cpx<T> rn[3][E];
#pragma unroll
  for (int gq = 0; gq < E; ++gq) {
    const long long off = base + (long long)(t + TL * fast_out_pos<N, E>(gq)) * ls;
    const cpx<T> qv[3] = {muli(acc[0][gq], (T)-1), muli(acc[1][gq], (T)-1), muli(acc[2][gq], (T)-1)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cpx<T> rv0 = valid ? r[off + c * cs] : mk<T>(0, 0);
      rn[c][gq] = valid ? down<T>(sub(up(rv0), scl(up(qv[c]), alpha))) : mk<T>(0, 0);
    }
  }
  if (plane_tile) {
    // Hermitian projection: element (k1, line) pairs with (-k1, partner line)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      __syncthreads();
#pragma unroll
      for (int gq = 0; gq < E; ++gq) lds[(t + TL * fast_out_pos<N, E>(gq)) * PITCH + s] = rn[c][gq];
      __syncthreads();
#pragma unroll
      for (int gq = 0; gq < E; ++gq) {
        const int k1 = t + TL * fast_out_pos<N, E>(gq);
        const int k1p = (k1 == 0) ? 0 : N - k1;
        const cpx<T> pv = lds[k1p * PITCH + (s ^ sp_xor)];
        rn[c][gq] = down<T>(scl(add(up(rn[c][gq]), conj(up(pv))), 0.5));
      }
    }
  }
  double rz = 0.0, rr = 0.0;
  const double w = plane_tile ? 1.0 : 2.0;
#pragma unroll
  for (int gq = 0; gq < E; ++gq) {
    const int k1 = t + TL * fast_out_pos<N, E>(gq);
    const long long off = base + (long long)k1 * ls;
    if (!valid) continue;
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[off + c * cs] = rn[c][gq];
      rv[c] = up(rn[c][gq]);
    }
    precond(pa, xi_of(k1, g.n1, g.il1), xi_of(o, g.n2, g.il2), xi_of(col, g.n3, g.il3), rv, zv);
    double a = 0.0, bb = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
      bb += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
    }
    rz += w * a;
    rr += w * bb;
  }
  const double s1 = block_sum<NT>(rz, red);
  const double s2 = block_sum<NT>(rr, red);
  if (tid == 0) {
    partials[2 * blockIdx.x] = s1;
    partials[2 * blockIdx.x + 1] = s2;
  }
}

template <typename T, int N>
static int launch_div_update_n(const void* W, void* r, const StridedGeom& sg, const Geom& g, const void* tw,
                               const PcgScalars* sc, const PrecondArgs& pa, double* dc_out, double* partials,
                               hipStream_t st) {
  using S = StridedShape<N, strided_E<T, N, SP_DIV_SMALL>()>;
  const long long npair = div_plane_pad<S::TZ>(sg.nother) + (long long)sg.nother * sg.ncols;
  const int ntiles = (int)((npair + S::TZ - 1) / S::TZ);
  DB_LAUNCH((k_div_update_fast<T, N>), dim3(ntiles), dim3(S::NT), 0, st, static_cast<const cpx<T>*>(W),
                     static_cast<cpx<T>*>(r), sg, g, static_cast<const cpx<T>*>(tw), sc, pa, dc_out, partials);
  return ntiles;
}

template <typename T>
int launch_div_update_fast(const void* W, void* r, const StridedGeom& sg, const Geom& g, const void* tw,
                           const PcgScalars* sc, const PrecondArgs& pa, double* dc_out, double* partials,
                           hipStream_t st) {
  switch (sg.nline) {
    case 8: return launch_div_update_n<T, 8>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
    case 16: return launch_div_update_n<T, 16>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
    case 32: return launch_div_update_n<T, 32>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
    case 64: return launch_div_update_n<T, 64>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
    case 128: return launch_div_update_n<T, 128>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
    default: return launch_div_update_n<T, 256>(W, r, sg, g, tw, sc, pa, dc_out, partials, st);
  }
}
template int launch_div_update_fast<double>(const void*, void*, const StridedGeom&, const Geom&, const void*,
                                            const PcgScalars*, const PrecondArgs&, double*, double*, hipStream_t);
template int launch_div_update_fast<float>(const void*, void*, const StridedGeom&, const Geom&, const void*,
                                           const PcgScalars*, const PrecondArgs&, double*, double*, hipStream_t);

bool fast_strided_supported(int n) { return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

template <typename T, int N, int MODE>
static void launch_fast_nm(const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                           const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                           PcgScalars* alpha_sc = nullptr, const double* eparts = nullptr, int neparts = 0) {
  using S = StridedShape<N, strided_E<T, N, MODE>()>;
  const long long npair = (long long)sg.nother * sg.ncols;
  const int ntiles = (int)((npair + S::TZ - 1) / S::TZ);
  dim3 grid(ntiles, 1, MODE == SP_PLAIN ? ncomp_plain : 1);
  DB_LAUNCH((k_strided_fast<T, N, MODE>), grid, dim3(S::NT), 0, st, static_cast<const cpx<T>*>(in),
                     static_cast<cpx<T>*>(out), sg, g, static_cast<const cpx<T>*>(tw), (T)dir, dc_out, stop, alpha_sc,
                     eparts, neparts);
}

template <typename T, int N>
static void launch_fast_n(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg,
                          const Geom& g, const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                          const AlphaTask& at) {
  PcgScalars* a = at.sc;
  const double* e = at.eparts;
  const int ne = at.neparts;
  switch (mode) {
    case SP_PLAIN: launch_fast_nm<T, N, SP_PLAIN>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, a, e, ne); break;
    case SP_GRAD_SMALL:
      launch_fast_nm<T, N, SP_GRAD_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, a, e, ne);
      break;
    case SP_GRAD_FINITE:
      launch_fast_nm<T, N, SP_GRAD_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, a, e, ne);
      break;
    case SP_DIV_SMALL:
      launch_fast_nm<T, N, SP_DIV_SMALL>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, a, e, ne);
      break;
    default: launch_fast_nm<T, N, SP_DIV_FINITE>(in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, a, e, ne); break;
  }
}

template <typename T>
void launch_strided_fast(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                         const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                         const AlphaTask& at) {
  switch (sg.nline) {
    case 8: launch_fast_n<T, 8>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    case 16: launch_fast_n<T, 16>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    case 32: launch_fast_n<T, 32>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    case 64: launch_fast_n<T, 64>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    case 128: launch_fast_n<T, 128>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
    default: launch_fast_n<T, 256>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop, at); break;
  }
}
template void launch_strided_fast<double>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                          int, double*, hipStream_t, const int*, const AlphaTask&);
template void launch_strided_fast<float>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                         int, double*, hipStream_t, const int*, const AlphaTask&);

// ------------------------------------------------------------------ z pass (fused tangent)
// One wave per block; TL = M/8 threads per z line, 64/TL lines per wave.
// Thread t of a line holds, for every tensor component, the packed pairs
// z[n] = f[2n] + i f[2n+1] at n = t + TL*m (m = 0..7): the inverse real
// transform's output and the forward real transform's input.
template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> v, int src) {
  return mk<T>(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// Value of lane (TL - t) mod TL of the same line (lines of TL = 8 or 16
// lanes sit in DPP rows): row mirror (half-row mirror for 8) then row shift
// right by one; lane t = 0 of a line gets a value it does not use.
template <int TL>
__device__ __forceinline__ int partner_b32(int v, int partner) {
  if constexpr (TL == 16) {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
    return __builtin_amdgcn_update_dpp(0, m, 0x111, 0xF, 0xF, false);
  } else if constexpr (TL == 8) {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
    return __builtin_amdgcn_update_dpp(0, m, 0x111, 0xF, 0xF, false);
  } else {
    return __shfl(v, partner, 64);
  }
}
template <int TL>
__device__ __forceinline__ double partner_f64(double x, int partner) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = partner_b32<TL>((int)b, partner);
  const int hi = partner_b32<TL>((int)(b >> 32), partner);
  return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}
template <int TL, typename T>
__device__ __forceinline__ cpx<T> shfl_partner(cpx<T> v, int partner) {
  if constexpr (sizeof(T) == 8) {
    return mk<T>(partner_f64<TL>(v.x, partner), partner_f64<TL>(v.y, partner));
  } else {
    return mk<T>(__builtin_bit_cast(float, partner_b32<TL>(__builtin_bit_cast(int, v.x), partner)),
                 __builtin_bit_cast(float, partner_b32<TL>(__builtin_bit_cast(int, v.y), partner)));
  }
}

// Exchange padding of the z pass: one slot per 256 bytes of a line.
template <typename T>
constexpr int line_pad() {
  return sizeof(T) == 8 ? 4 : 5;
}

// Elements per thread of the z pass.
template <typename T>
constexpr int line_E() {
  return 4;
}
template <typename T, int M, int E>
struct LineCtx {
  static constexpr int TL = M / E;
  static constexpr int LB = 64 / TL;
  static constexpr int PITCH = M + (M >> line_pad<T>()) + 1;
};

// inverse real transform of component c for the 8 lines of the wave:
// e[m] = packed pair at position t + TL m
template <typename T, int M, int E>
__device__ __forceinline__ void line_inverse(const cpx<T>* src, bool valid, int t, int partner, cpx<T>* lds, int off,
                                             const cpx<T>* tw, const cpx<T>* rtw, cpx<T>* e) {
  constexpr int TL = M / E;
  cpx<T> X[E];
#pragma unroll
  for (int r = 0; r < E; ++r) X[r] = valid ? src[t + TL * r] : mk<T>(0, 0);
  const cpx<T> XN = (valid && t == 0) ? src[M] : mk<T>(0, 0);
  cpx<T> Z[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    // X[M - k] for k = t + TL r: lane (TL - t), register 7 - r; for t = 0 own register 8 - r (XN when r = 0)
    const cpx<T> sh = shfl_partner<M / E>(X[E - 1 - r], partner);
    const cpx<T> own = (r == 0) ? XN : X[(E - r) & (E - 1)];
    const cpx<T> Xm = conj((t == 0) ? own : sh);
    const cpx<T> Ev = add(X[r], Xm);
    const cpx<T> Od = mul(sub(X[r], Xm), conj(rtw[t + TL * r]));
    Z[r] = add(Ev, muli(Od, (T)1));
  }
  fast_fft<T, M, E, line_pad<T>()>(Z, t, lds, 1, off, tw, (T)1);
#pragma unroll
  for (int gq = 0; gq < E; ++gq) e[fast_out_pos<M, E>(gq)] = Z[gq];
}

// forward real transform of packed pairs e (positions t + TL m), scaled, stored
template <typename T, int M, int E>
__device__ __forceinline__ void line_forward(cpx<T>* dst, bool valid, int t, int partner, cpx<T>* lds, int off,
                                             const cpx<T>* tw, const cpx<T>* rtw, const cpx<T>* e, T scale) {
  constexpr int TL = M / E;
  cpx<T> Z[E];
#pragma unroll
  for (int m = 0; m < E; ++m) Z[m] = e[m];
  fast_fft<T, M, E, line_pad<T>()>(Z, t, lds, 1, off, tw, (T)-1);
  cpx<T> Zp[E];
#pragma unroll
  for (int gq = 0; gq < E; ++gq) Zp[fast_out_pos<M, E>(gq)] = Z[gq];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + TL * m;
    const cpx<T> sh = shfl_partner<M / E>(Zp[E - 1 - m], partner);
    const cpx<T> own = Zp[(E - m) & (E - 1)];
    const cpx<T> Zm = conj((t == 0) ? own : sh);
    const cpx<T> Ev = scl(add(Zp[m], Zm), (T)0.5);
    const cpx<T> Od = mul(rtw[k], scl(sub(Zp[m], Zm), (T)0.5));
    if (valid) dst[k] = scl(sub(Ev, muli(Od, (T)1)), scale);
  }
  if (valid && t == 0) {
    const cpx<T> Z0 = Zp[0], Zm = conj(Zp[0]);
    const cpx<T> Ev = scl(add(Z0, Zm), (T)0.5);
    const cpx<T> Od = mul(rtw[M], scl(sub(Z0, Zm), (T)0.5));
    dst[M] = scl(sub(Ev, muli(Od, (T)1)), scale);
  }
}

template <typename T>
__device__ __forceinline__ void iso_coeffs(const TangentArgs<T>& tn, long long vox, T& lam, T& mu2) {
  if (tn.kind == TAN_ISO_PHASE) {
    const int p = tn.phase[vox];
    lam = (T)tn.lam[p];
    mu2 = (T)(2.0 * tn.mu[p]);
  } else {
    const T E = tn.field[vox];
    lam = (T)tn.lam1 * E;
    mu2 = (T)(2.0 * tn.mu1) * E;
  }
}

// ISO = 1: isotropic tangent; only the three normal components couple
// (through the trace), so they are transformed together and every shear
// component on its own, which keeps at most three components in registers.
template <typename T, int M, int KIN, int ISO>
__global__ __launch_bounds__(64) void k_line_fast(const cpx<T>* in, cpx<T>* out, Geom g, const cpx<T>* __restrict__ twg,
                                                  const cpx<T>* __restrict__ rtwg, TangentArgs<T> tn,
                                                  const double* __restrict__ macro_dev, double* __restrict__ partials,
                                                  const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  constexpr int E = line_E<T>();
  using LC = LineCtx<T, M, E>;
  constexpr int TL = LC::TL, LB = LC::LB, PITCH = LC::PITCH;
  constexpr int NC = (KIN == KIN_SMALL) ? 6 : 9;
  __shared__ cpx<T> tw[M];
  __shared__ cpx<T> rtw[M + 1];
  __shared__ cpx<T> lds[LB * PITCH];
  const int lane = threadIdx.x;
  const int line = lane / TL, t = lane % TL;
  for (int i = lane; i < M; i += 64) tw[i] = twg[i];
  for (int i = lane; i <= M; i += 64) rtw[i] = rtwg[i];
  __syncthreads();
  const int nh3 = g.nh3, n3 = g.n3;
  const long long nlines = (long long)g.n1 * g.n2;
  const long long gl = (long long)blockIdx.x * LB + line;
  const bool valid = gl < nlines;
  const int partner = line * TL + ((TL - t) % TL);
  const int off = line * PITCH;
  const T scale = (T)g.inv_nvox;
  double mac[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) mac[c] = macro_dev ? macro_dev[c] : 0.0;
  double energy = 0.0;
  const cpx<T>* inl = in + gl * nh3;
  cpx<T>* outl = out + gl * nh3;

  if constexpr (ISO == 1) {
    // normal components 11 22 33
    cpx<T> e[3][E];
#pragma unroll
    for (int c = 0; c < 3; ++c) line_inverse<T, M, E>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c]);
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int n = t + TL * m;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long long vox = gl * n3 + 2 * n + h;
          T lam, mu2;
          iso_coeffs<T>(tn, vox, lam, mu2);
          T ev[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) ev[c] = (h == 0 ? e[c][m].x : e[c][m].y) + (T)mac[c];
          const T tr = ev[0] + ev[1] + ev[2];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T sv = lam * tr + mu2 * ev[c];
            energy += (double)(ev[c] * sv);
            if (h == 0) e[c][m].x = sv;
            else e[c][m].y = sv;
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) line_forward<T, M, E>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c], scale);
    // shear components 23 13 12, one at a time: sigma = 2 mu eps
#pragma unroll 1
    for (int c = 3; c < 6; ++c) {
      cpx<T> e1[E];
      line_inverse<T, M, E>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e1);
      if (valid) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int n = t + TL * m;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const long long vox = gl * n3 + 2 * n + h;
            T lam, mu2;
            iso_coeffs<T>(tn, vox, lam, mu2);
            const T ev = (h == 0 ? e1[m].x : e1[m].y) + (T)mac[c];
            const T sv = mu2 * ev;
            energy += 2.0 * (double)(ev * sv);
            if (h == 0) e1[m].x = sv;
            else e1[m].y = sv;
          }
        }
      }
      line_forward<T, M, E>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e1, scale);
    }
  } else {
    cpx<T> e[NC][E];
#pragma unroll
    for (int c = 0; c < NC; ++c) line_inverse<T, M, E>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c]);
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int n = t + TL * m;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long long vox = gl * n3 + 2 * n + h;
          T ev[NC], sv[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) ev[c] = (h == 0 ? e[c][m].x : e[c][m].y) + (T)mac[c];
          if constexpr (KIN == KIN_SMALL) {
            const T r2 = (T)1.41421356237309504880, ir2 = (T)0.70710678118654752440;
            const T vv[6] = {ev[0], ev[1], ev[2], r2 * ev[3], r2 * ev[4], r2 * ev[5]};
            T o6[6] = {0, 0, 0, 0, 0, 0};
            int idx = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
              for (int b = a; b < 6; ++b) {
                const T cab = (tn.kind == TAN_ANISO_FIELD) ? tn.field[(long long)idx * g.nvox + vox]
                                                           : (T)tn.grain_table[(long long)tn.grain[vox] * 21 + idx];
                o6[a] += cab * vv[b];
                if (b != a) o6[b] += cab * vv[a];
                ++idx;
              }
            sv[0] = o6[0];
            sv[1] = o6[1];
            sv[2] = o6[2];
            sv[3] = o6[3] * ir2;
            sv[4] = o6[4] * ir2;
            sv[5] = o6[5] * ir2;
            energy += (double)(ev[0] * sv[0] + ev[1] * sv[1] + ev[2] * sv[2]) +
                      2.0 * (double)(ev[3] * sv[3] + ev[4] * sv[4] + ev[5] * sv[5]);
          } else {
            tangent_finite<T, ISO>(tn, vox, g.nvox, ev, sv);
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc += (double)(ev[c] * sv[c]);
            energy += acc;
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            if (h == 0) e[c][m].x = sv[c];
            else e[c][m].y = sv[c];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) line_forward<T, M, E>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c], scale);
  }
  if (partials != nullptr) {
#pragma unroll
    for (int offs = 32; offs > 0; offs >>= 1) energy += __shfl_xor(energy, offs, 64);
    if (lane == 0) partials[blockIdx.x] = energy * g.inv_nvox;
  }
}

bool fast_line_supported(int n3) { return n3 == 16 || n3 == 32 || n3 == 64 || n3 == 128 || n3 == 256; }

int fast_line_blocks(const Geom& g, int elem_bytes) {
  (void)elem_bytes;  // four elements per thread in both precisions
  const int M = g.n3 / 2;
  const int E = 4;
  const int LB = 64 / (M / E);
  return (int)(((long long)g.n1 * g.n2 + LB - 1) / LB);
}

template <typename T, int M>
static void launch_line_fast_m(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                               const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                               const int* stop) {
  const int nb = fast_line_blocks(g, (int)sizeof(cpx<T>));
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
  if (kin == KIN_SMALL && (tan.kind == TAN_ISO_PHASE || tan.kind == TAN_ISO_FIELD))
    DB_LAUNCH((k_line_fast<T, M, KIN_SMALL, 1>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                       partials, stop);
  else if (kin == KIN_SMALL)
    DB_LAUNCH((k_line_fast<T, M, KIN_SMALL, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                       partials, stop);
  else
    if (finite_law(tan.kind) == 2)
      DB_LAUNCH((k_line_fast<T, M, KIN_FINITE, 2>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                         partials, stop);
    else
      DB_LAUNCH((k_line_fast<T, M, KIN_FINITE, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                         partials, stop);
}

template <typename T>
void launch_line_fast(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                      const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                      const int* stop) {
  switch (g.n3) {
    case 16: launch_line_fast_m<T, 8>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
    case 32: launch_line_fast_m<T, 16>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
    case 64: launch_line_fast_m<T, 32>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
    case 128: launch_line_fast_m<T, 64>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
    default: launch_line_fast_m<T, 128>(kin, in, out, g, tw, rtw, tan, macro_dev, partials, st, stop); break;
  }
}
template void launch_line_fast<double>(int, const void*, void*, const Geom&, const void*, const void*,
                                       const TangentArgs<double>&, const double*, double*, hipStream_t, const int*);
template void launch_line_fast<float>(int, const void*, void*, const Geom&, const void*, const void*,
                                      const TangentArgs<float>&, const double*, double*, hipStream_t, const int*);

}  // namespace dbfft
