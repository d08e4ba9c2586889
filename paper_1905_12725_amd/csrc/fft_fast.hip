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

namespace dbfft {

template <int N>
constexpr int fast_nstages() {
  int m = N, s = 0;
  while (m % 8 == 0) { m /= 8; ++s; }
  while (m % 4 == 0) { m /= 4; ++s; }
  while (m % 2 == 0) { m /= 2; ++s; }
  return s;
}
template <int N>
constexpr int fast_radix(int st) {
  int m = N, s = 0;
  while (m % 8 == 0) { if (s == st) return 8; m /= 8; ++s; }
  while (m % 4 == 0) { if (s == st) return 4; m /= 4; ++s; }
  while (m % 2 == 0) { if (s == st) return 2; m /= 2; ++s; }
  return 1;
}
template <int N>
constexpr int fast_ns(int st) {
  int p = 1;
  for (int s = 0; s < st; ++s) p *= fast_radix<N>(s);
  return p;
}

// radix-R butterflies of stage ST on the 8 registers of thread t
template <typename T, int N, int ST>
__device__ __forceinline__ void fast_stage(cpx<T>* v, int t, const cpx<T>* __restrict__ tw, T d) {
  constexpr int R = fast_radix<N>(ST);
  constexpr int NS = fast_ns<N>(ST);
  constexpr int TL = N / 8;
  constexpr int NB = 8 / R;
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

// write the outputs of stage ST to LDS and read the inputs of stage ST+1;
// element index i of a sequence lives at lds[i * pitch + lane_off]
template <typename T, int N, int ST>
__device__ __forceinline__ void fast_exchange(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off) {
  constexpr int R = fast_radix<N>(ST), NS = fast_ns<N>(ST), NB = 8 / R;
  constexpr int R2 = fast_radix<N>(ST + 1), NB2 = 8 / R2;
  constexpr int TL = N / 8;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + TL * q;
    const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[(base + r * NS) * pitch + off] = v[q * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB2; ++q) {
    const int j = t + TL * q;
#pragma unroll
    for (int r = 0; r < R2; ++r) v[q * R2 + r] = lds[(j + r * (N / R2)) * pitch + off];
  }
  __syncthreads();
}

template <typename T, int N, int ST>
__device__ __forceinline__ void fast_fft_from(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off,
                                              const cpx<T>* __restrict__ tw, T d) {
  fast_stage<T, N, ST>(v, t, tw, d);
  if constexpr (ST + 1 < fast_nstages<N>()) {
    fast_exchange<T, N, ST>(v, t, lds, pitch, off);
    fast_fft_from<T, N, ST + 1>(v, t, lds, pitch, off, tw, d);
  }
}

// full transform of the 8 registers (stage-0 input -> last-stage output)
template <typename T, int N>
__device__ __forceinline__ void fast_fft(cpx<T>* v, int t, cpx<T>* lds, int pitch, int off,
                                         const cpx<T>* __restrict__ tw, T d) {
  fast_fft_from<T, N, 0>(v, t, lds, pitch, off, tw, d);
}

// index of output register g (= q*R + r) of thread t
template <int N>
__device__ __forceinline__ constexpr int fast_out_pos(int g) {
  constexpr int R = fast_radix<N>(fast_nstages<N>() - 1);
  constexpr int NB = 8 / R;
  return (g / R) + NB * (g % R);  // q + NB r, times TL plus t
}

// ------------------------------------------------------------------ x / y passes
template <int N>
struct StridedShape {
  static constexpr int TL = N / 8;
  static constexpr int TZ = (N >= 256) ? 8 : (N >= 128 ? 16 : 32);
  static constexpr int NT = TL * TZ;
  static constexpr int PITCH = TZ + 1;
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__(StridedShape<N>::NT) void k_strided_fast(const cpx<T>* in, cpx<T>* out, StridedGeom sg,
                                                                      Geom g, const cpx<T>* __restrict__ twg, T d,
                                                                      double* __restrict__ dc_out,
                                                                      const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  using S = StridedShape<N>;
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

  auto load8 = [&](const cpx<T>* src, cpx<T>* v) {
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = valid ? src[base + (long long)(t + TL * r) * ls] : mk<T>(0, 0);
  };
  auto store8 = [&](cpx<T>* dst, const cpx<T>* v) {
    if (!valid) return;
#pragma unroll
    for (int gq = 0; gq < 8; ++gq) dst[base + (long long)(t + TL * fast_out_pos<N>(gq)) * ls] = v[gq];
  };

  if constexpr (MODE == SP_PLAIN) {
    const int c = blockIdx.z;
    cpx<T> v[8];
    load8(in + c * sg.cstride_in, v);
    fast_fft<T, N>(v, t, lds, PITCH, s, tw, d);
    store8(out + c * sg.cstride_out, v);
  } else if constexpr (MODE == SP_GRAD_SMALL || MODE == SP_GRAD_FINITE) {
    // x pass, line = k1, other = k2, column = k3.  With T_i = FFT(a_i) and
    // U_i = FFT(xi1 a_i):  eps_11 = i U_1, eps_22 = i xi2 T_2, eps_33 = i xi3 T_3,
    // eps_12 = i/2 (U_2 + xi2 T_1), eps_13 = i/2 (U_3 + xi3 T_1),
    // eps_23 = i/2 (xi3 T_2 + xi2 T_3);  H_i1 = i U_i, H_i2 = i xi2 T_i, H_i3 = i xi3 T_i.
    const T xi2 = (T)xi_of(o, g.n2);
    const T xi3 = (T)xi_of(col, g.n3);
    T xi1[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) xi1[r] = (T)xi_of(t + TL * r, g.n1);
    const long long co = sg.cstride_out;
    cpx<T> T1[8], T2[8], Tc[8], U[8];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T>* Ti = (i == 0) ? T1 : (i == 1 ? T2 : Tc);
      load8(in + i * sg.cstride_in, Ti);
#pragma unroll
      for (int r = 0; r < 8; ++r) U[r] = scl(Ti[r], xi1[r]);
      fast_fft<T, N>(Ti, t, lds, PITCH, s, tw, d);
      fast_fft<T, N>(U, t, lds, PITCH, s, tw, d);
      cpx<T> w[8];
      if constexpr (MODE == SP_GRAD_FINITE) {
#pragma unroll
        for (int r = 0; r < 8; ++r) w[r] = muli(U[r], (T)1);
        store8(out + (3 * i + 0) * co, w);
#pragma unroll
        for (int r = 0; r < 8; ++r) w[r] = muli(scl(Ti[r], xi2), (T)1);
        store8(out + (3 * i + 1) * co, w);
#pragma unroll
        for (int r = 0; r < 8; ++r) w[r] = muli(scl(Ti[r], xi3), (T)1);
        store8(out + (3 * i + 2) * co, w);
      } else {
        // stored order 11 22 33 23 13 12
        if (i == 0) {
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(U[r], (T)1);
          store8(out + 0 * co, w);
        } else if (i == 1) {
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(scl(T2[r], xi2), (T)1);
          store8(out + 1 * co, w);
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(scl(add(U[r], scl(T1[r], xi2)), (T)0.5), (T)1);
          store8(out + 5 * co, w);
        } else {
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(scl(Tc[r], xi3), (T)1);
          store8(out + 2 * co, w);
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(scl(add(U[r], scl(T1[r], xi3)), (T)0.5), (T)1);
          store8(out + 4 * co, w);
#pragma unroll
          for (int r = 0; r < 8; ++r) w[r] = muli(scl(add(scl(T2[r], xi3), scl(Tc[r], xi2)), (T)0.5), (T)1);
          store8(out + 3 * co, w);
        }
      }
    }
  } else {
    // SP_DIV_*: r_i = -i sum_j xi_j s_ij after the forward x transform
    const T xi2 = (T)xi_of(o, g.n2);
    const T xi3 = (T)xi_of(col, g.n3);
    T xi1[8];
#pragma unroll
    for (int gq = 0; gq < 8; ++gq) xi1[gq] = (T)xi_of(t + TL * fast_out_pos<N>(gq), g.n1);
    cpx<T> a0[8], a1[8], a2[8];  // rows of -i xi_j s_ij before the factor -i
#pragma unroll
    for (int r = 0; r < 8; ++r) a0[r] = a1[r] = a2[r] = mk<T>(0, 0);
    constexpr int NC = (MODE == SP_DIV_SMALL) ? 6 : 9;
    // one component live at a time (keeps the three accumulators the only
    // long-lived registers)
#pragma unroll 1
    for (int c = 0; c < NC; ++c) {
      cpx<T> v[8];
      load8(in + c * sg.cstride_in, v);
      fast_fft<T, N>(v, t, lds, PITCH, s, tw, d);
      if (dc_out != nullptr && valid && o == 0 && col == 0 && t == 0) dc_out[c] = (double)v[0].x;
      int ii, jj;
      if constexpr (MODE == SP_DIV_SMALL) {
        ii = (c < 3) ? c : (c == 3 ? 1 : 0);
        jj = (c < 3) ? c : (c == 5 ? 1 : 2);
      } else {
        ii = c / 3;
        jj = c % 3;
      }
#pragma unroll
      for (int gq = 0; gq < 8; ++gq) {
        const T xj = (jj == 0) ? xi1[gq] : (jj == 1 ? xi2 : xi3);
        const cpx<T> t1 = scl(v[gq], xj);
        if (ii == 0) a0[gq] = add(a0[gq], t1);
        else if (ii == 1) a1[gq] = add(a1[gq], t1);
        else a2[gq] = add(a2[gq], t1);
        if (MODE == SP_DIV_SMALL && ii != jj) {
          const T xi_ = (ii == 0) ? xi1[gq] : (ii == 1 ? xi2 : xi3);
          const cpx<T> t2 = scl(v[gq], xi_);
          if (jj == 0) a0[gq] = add(a0[gq], t2);
          else if (jj == 1) a1[gq] = add(a1[gq], t2);
          else a2[gq] = add(a2[gq], t2);
        }
      }
    }
#pragma unroll
    for (int gq = 0; gq < 8; ++gq) {
      a0[gq] = muli(a0[gq], (T)-1);
      a1[gq] = muli(a1[gq], (T)-1);
      a2[gq] = muli(a2[gq], (T)-1);
    }
    store8(out, a0);
    store8(out + sg.cstride_out, a1);
    store8(out + 2 * sg.cstride_out, a2);
  }
}

bool fast_strided_supported(int n) { return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

template <typename T, int N>
static void launch_fast_n(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg,
                          const Geom& g, const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop) {
  using S = StridedShape<N>;
  const long long npair = (long long)sg.nother * sg.ncols;
  const int ntiles = (int)((npair + S::TZ - 1) / S::TZ);
  dim3 grid(ntiles, 1, mode == SP_PLAIN ? ncomp_plain : 1);
  const T d = (T)dir;
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  switch (mode) {
    case SP_PLAIN:
      hipLaunchKernelGGL((k_strided_fast<T, N, SP_PLAIN>), grid, dim3(S::NT), 0, st, i, o, sg, g, t, d, dc_out, stop);
      break;
    case SP_GRAD_SMALL:
      hipLaunchKernelGGL((k_strided_fast<T, N, SP_GRAD_SMALL>), grid, dim3(S::NT), 0, st, i, o, sg, g, t, d, dc_out, stop);
      break;
    case SP_GRAD_FINITE:
      hipLaunchKernelGGL((k_strided_fast<T, N, SP_GRAD_FINITE>), grid, dim3(S::NT), 0, st, i, o, sg, g, t, d, dc_out, stop);
      break;
    case SP_DIV_SMALL:
      hipLaunchKernelGGL((k_strided_fast<T, N, SP_DIV_SMALL>), grid, dim3(S::NT), 0, st, i, o, sg, g, t, d, dc_out, stop);
      break;
    default:
      hipLaunchKernelGGL((k_strided_fast<T, N, SP_DIV_FINITE>), grid, dim3(S::NT), 0, st, i, o, sg, g, t, d, dc_out, stop);
      break;
  }
}

template <typename T>
void launch_strided_fast(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                         const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop) {
  switch (sg.nline) {
    case 8: launch_fast_n<T, 8>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case 16: launch_fast_n<T, 16>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case 32: launch_fast_n<T, 32>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case 64: launch_fast_n<T, 64>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    case 128: launch_fast_n<T, 128>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
    default: launch_fast_n<T, 256>(mode, in, out, ncomp_plain, sg, g, tw, dir, dc_out, st, stop); break;
  }
}
template void launch_strided_fast<double>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                          int, double*, hipStream_t, const int*);
template void launch_strided_fast<float>(int, const void*, void*, int, const StridedGeom&, const Geom&, const void*,
                                         int, double*, hipStream_t, const int*);

// ------------------------------------------------------------------ z pass (fused tangent)
// One wave per block; TL = M/8 threads per z line, 64/TL lines per wave.
// Thread t of a line holds, for every tensor component, the packed pairs
// z[n] = f[2n] + i f[2n+1] at n = t + TL*m (m = 0..7): the inverse real
// transform's output and the forward real transform's input.
template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> v, int src) {
  return mk<T>(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

template <typename T, int M>
struct LineCtx {
  static constexpr int TL = M / 8;
  static constexpr int LB = 64 / TL;
  static constexpr int PITCH = M + 1;
};

// inverse real transform of component c for the 8 lines of the wave:
// e[m] = packed pair at position t + TL m
template <typename T, int M>
__device__ __forceinline__ void line_inverse(const cpx<T>* src, bool valid, int t, int partner, cpx<T>* lds, int off,
                                             const cpx<T>* tw, const cpx<T>* rtw, cpx<T>* e) {
  constexpr int TL = M / 8;
  cpx<T> X[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) X[r] = valid ? src[t + TL * r] : mk<T>(0, 0);
  const cpx<T> XN = (valid && t == 0) ? src[M] : mk<T>(0, 0);
  cpx<T> Z[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    // X[M - k] for k = t + TL r: lane (TL - t), register 7 - r; for t = 0 own register 8 - r (XN when r = 0)
    const cpx<T> sh = shfl_c(X[7 - r], partner);
    const cpx<T> own = (r == 0) ? XN : X[(8 - r) & 7];
    const cpx<T> Xm = conj((t == 0) ? own : sh);
    const cpx<T> Ev = add(X[r], Xm);
    const cpx<T> Od = mul(sub(X[r], Xm), conj(rtw[t + TL * r]));
    Z[r] = add(Ev, muli(Od, (T)1));
  }
  fast_fft<T, M>(Z, t, lds, 1, off, tw, (T)1);
#pragma unroll
  for (int gq = 0; gq < 8; ++gq) e[fast_out_pos<M>(gq)] = Z[gq];
}

// forward real transform of packed pairs e (positions t + TL m), scaled, stored
template <typename T, int M>
__device__ __forceinline__ void line_forward(cpx<T>* dst, bool valid, int t, int partner, cpx<T>* lds, int off,
                                             const cpx<T>* tw, const cpx<T>* rtw, const cpx<T>* e, T scale) {
  constexpr int TL = M / 8;
  cpx<T> Z[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) Z[m] = e[m];
  fast_fft<T, M>(Z, t, lds, 1, off, tw, (T)-1);
  cpx<T> Zp[8];
#pragma unroll
  for (int gq = 0; gq < 8; ++gq) Zp[fast_out_pos<M>(gq)] = Z[gq];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int k = t + TL * m;
    const cpx<T> sh = shfl_c(Zp[7 - m], partner);
    const cpx<T> own = Zp[(8 - m) & 7];
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
  using LC = LineCtx<T, M>;
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
    cpx<T> e[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) line_inverse<T, M>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c]);
    if (valid) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
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
    for (int c = 0; c < 3; ++c) line_forward<T, M>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c], scale);
    // shear components 23 13 12, one at a time: sigma = 2 mu eps
#pragma unroll 1
    for (int c = 3; c < 6; ++c) {
      cpx<T> e1[8];
      line_inverse<T, M>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e1);
      if (valid) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
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
      line_forward<T, M>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e1, scale);
    }
  } else {
    cpx<T> e[NC][8];
#pragma unroll
    for (int c = 0; c < NC; ++c) line_inverse<T, M>(inl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c]);
    if (valid) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
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
            T Fi[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) Fi[i] = tn.field[(long long)i * g.nvox + vox];
            const T lnJ = tn.field[9LL * g.nvox + vox];
            const int p = tn.phase[vox];
            const T mu = (T)tn.mu[p], lam = (T)tn.lam[p];
            T tr = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int J = 0; J < 3; ++J) tr += Fi[J * 3 + i] * ev[i * 3 + J];
            T T1[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int J = 0; J < 3; ++J) {
                T acc = 0;
#pragma unroll
                for (int b = 0; b < 3; ++b) acc += ev[b * 3 + a] * Fi[J * 3 + b];
                T1[a * 3 + J] = acc;
              }
            const T c2 = mu - lam * lnJ;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int J = 0; J < 3; ++J) {
                T acc = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) acc += Fi[a * 3 + i] * T1[a * 3 + J];
                sv[i * 3 + J] = mu * ev[i * 3 + J] + c2 * acc + lam * tr * Fi[J * 3 + i];
              }
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
    for (int c = 0; c < NC; ++c) line_forward<T, M>(outl + c * g.nh, valid, t, partner, lds, off, tw, rtw, e[c], scale);
  }
  if (partials != nullptr) {
#pragma unroll
    for (int offs = 32; offs > 0; offs >>= 1) energy += __shfl_xor(energy, offs, 64);
    if (lane == 0) partials[blockIdx.x] = energy * g.inv_nvox;
  }
}

bool fast_line_supported(int n3) { return n3 == 16 || n3 == 32 || n3 == 64 || n3 == 128 || n3 == 256; }

int fast_line_blocks(const Geom& g) {
  const int M = g.n3 / 2;
  const int LB = 64 / (M / 8);
  return (int)(((long long)g.n1 * g.n2 + LB - 1) / LB);
}

template <typename T, int M>
static void launch_line_fast_m(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                               const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                               const int* stop) {
  const int nb = fast_line_blocks(g);
  auto i = static_cast<const cpx<T>*>(in);
  auto o = static_cast<cpx<T>*>(out);
  auto t = static_cast<const cpx<T>*>(tw);
  auto r = static_cast<const cpx<T>*>(rtw);
  if (kin == KIN_SMALL && (tan.kind == TAN_ISO_PHASE || tan.kind == TAN_ISO_FIELD))
    hipLaunchKernelGGL((k_line_fast<T, M, KIN_SMALL, 1>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                       partials, stop);
  else if (kin == KIN_SMALL)
    hipLaunchKernelGGL((k_line_fast<T, M, KIN_SMALL, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
                       partials, stop);
  else
    hipLaunchKernelGGL((k_line_fast<T, M, KIN_FINITE, 0>), dim3(nb), dim3(64), 0, st, i, o, g, t, r, tan, macro_dev,
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
