// Two-step register transforms of the x/y passes and of the z pass for
// line lengths that factor into two 2-3-5-smooth factors of at most 16
// (fft_reg.h).  The block bodies are shared by the single-cell kernels
// (fft_mixed.hip) and the batched ones (batch.hip).
#pragma once

#include "dbfft_internal.h"
#include "fft_generic.h"
#include "fft_reg.h"

namespace dbfft {

// factor pair of a line length (powers of two included, for the batched
// kernels); 0 when the length is not supported
constexpr int mixed_n1(int n) {
  switch (n) {
    case 16: return 4;
    case 32: return 4;
    case 64: return 8;
    case 128: return 8;
    default: return two_step_n1(n);
  }
}

template <int N>
struct MixedShape {
  static constexpr int N1 = mixed_n1(N);
  static constexpr int N2 = N / N1;
  static constexpr int EM = N1 > N2 ? N1 : N2;  // registers per vector
  static constexpr int TL = EM;                  // threads per line
  static constexpr int TZ = (256 / TL) < 32 ? (256 / TL) : 32;
  static constexpr int NT = TL * TZ;
  static constexpr int PITCH = TZ + 1;
  static constexpr size_t lds_elems = (size_t)N * PITCH + N;  // exchange + twiddles
};

// x/y pass of one tile (TZ (other index, k3) pairs) of a line length N.
// Threads: tid < NT; s = tid % TZ the tile column, t = tid / TZ the thread of
// the line.  Inputs in the step-1 distribution (thread t < N2, register n1:
// row N2 n1 + t), outputs in the step-2 one (thread t < N1, register k2:
// row t + N1 k2).  `tw` is the N-point twiddle table in LDS, `lds` the
// exchange buffer (N * PITCH elements).  PARTS (SP_GRAD_SMALL, SP_DIV_SMALL
// only): the small-strain gradient and divergence in three parts, so that
// fewer vectors are live; `part` = i: the gradient writes the components
// (i, i) and (i, i+1 mod 3) from a_i and a_(i+1), the divergence writes r_i
// from the stress row i.  Without PARTS one call does everything.
template <typename T, int N, int MODE, bool PARTS = false>
__device__ __forceinline__ void mixed_strided_tile(const cpx<T>* in, cpx<T>* out, const StridedGeom& sg,
                                                   const Geom& g, const cpx<T>* tw, cpx<T>* lds, T d,
                                                   double* __restrict__ dc_out, long long tile, int tid,
                                                   int part = 0) {
  using S = MixedShape<N>;
  constexpr int N1 = S::N1, N2 = S::N2, EM = S::EM, TZ = S::TZ, PITCH = S::PITCH;
  const int s = tid % TZ, t = tid / TZ;
  const long long npair = (long long)sg.nother * sg.ncols;
  const long long pr = tile * TZ + s;
  const bool valid = pr < npair && t < S::TL;
  const int o = valid ? (int)(pr / sg.ncols) : 0;
  const int col = valid ? (int)(pr - (long long)o * sg.ncols) : 0;
  const long long base = (long long)o * sg.ostride + col;
  const long long ls = sg.lstride;
  const bool lin = valid && t < N2, lout = valid && t < N1;
  auto loadv = [&](const cpx<T>* src, cpx<T>* v) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = lin ? src[base + (long long)(N2 * n1 + t) * ls] : mk<T>(0, 0);
  };
  auto storev = [&](cpx<T>* dst, const cpx<T>* v) {
    if (!lout) return;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) dst[base + (long long)(t + N1 * k2) * ls] = v[k2];
  };
  auto fft = [&](cpx<T>* v) { two_step_fft<T, N1, N2, 0>(v, t, lds, PITCH, s, tw, d); };

  if constexpr (MODE == SP_PLAIN) {
    cpx<T> v[EM];
    loadv(in, v);
    fft(v);
    storev(out, v);
  } else if constexpr (MODE == SP_GRAD_SMALL) {
    const T xi2 = (T)xi_of(o, g.n2, g.il2), xi3 = (T)xi_of(col, g.n3, g.il3);
    const long long co = sg.cstride_out;
    if constexpr (PARTS) {
      // components (i, i) and (i, j), j = i + 1 mod 3: stored 11 22 33 23 13 12
      const int i = part, j = (part + 1) % 3;
      const int cij = (i == 0) ? 5 : (i == 1 ? 3 : 4);
      auto xa = [&](int a, T x1) { return a == 0 ? x1 : (a == 1 ? xi2 : xi3); };
      cpx<T> Ai[N1], Aj[N1];
      loadv(in + i * sg.cstride_in, Ai);
      loadv(in + j * sg.cstride_in, Aj);
      {
        cpx<T> v[EM];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = muli(scl(Ai[n1], xa(i, (T)xi_of(N2 * n1 + t, g.n1, g.il1))), (T)1);
        fft(v);
        storev(out + i * co, v);
      }
      {
        cpx<T> v[EM];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
          const T x1 = (T)xi_of(N2 * n1 + t, g.n1, g.il1);
          v[n1] = muli(scl(add(scl(Ai[n1], xa(j, x1)), scl(Aj[n1], xa(i, x1))), (T)0.5), (T)1);
        }
        fft(v);
        storev(out + cij * co, v);
      }
    } else {
    cpx<T> A0[N1], A1[N1], A2[N1];
    loadv(in, A0);
    loadv(in + sg.cstride_in, A1);
    loadv(in + 2 * sg.cstride_in, A2);
    auto emit = [&](int c, auto&& form) {
      cpx<T> v[EM];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) v[n1] = form(n1, (T)xi_of(N2 * n1 + t, g.n1, g.il1));
      fft(v);
      storev(out + c * co, v);
    };
    // stored order 11 22 33 23 13 12: eps_ij = i/2 (xi_j a_i + xi_i a_j)
    emit(0, [&](int r, T x1) { return muli(scl(A0[r], x1), (T)1); });
    emit(1, [&](int r, T) { return muli(scl(A1[r], xi2), (T)1); });
    emit(2, [&](int r, T) { return muli(scl(A2[r], xi3), (T)1); });
    emit(3, [&](int r, T) { return muli(scl(add(scl(A1[r], xi3), scl(A2[r], xi2)), (T)0.5), (T)1); });
    emit(4, [&](int r, T x1) { return muli(scl(add(scl(A0[r], xi3), scl(A2[r], x1)), (T)0.5), (T)1); });
    emit(5, [&](int r, T x1) { return muli(scl(add(scl(A0[r], xi2), scl(A1[r], x1)), (T)0.5), (T)1); });
    }
  } else if constexpr (MODE == SP_GRAD_FINITE) {
    // T_i = FFT(a_i), U_i = FFT(xi1 a_i): H_i1 = i U_i, H_i2 = i xi2 T_i, H_i3 = i xi3 T_i
    const T xi2 = (T)xi_of(o, g.n2, g.il2), xi3 = (T)xi_of(col, g.n3, g.il3);
    const long long co = sg.cstride_out;
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      cpx<T> Ti[EM], U[EM];
      loadv(in + i * sg.cstride_in, Ti);
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) U[n1] = scl(Ti[n1], (T)xi_of(N2 * n1 + t, g.n1, g.il1));
      fft(Ti);
      fft(U);
      cpx<T> w[EM];
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) w[k2] = muli(U[k2], (T)1);
      storev(out + (3 * i + 0) * co, w);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) w[k2] = muli(scl(Ti[k2], xi2), (T)1);
      storev(out + (3 * i + 1) * co, w);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) w[k2] = muli(scl(Ti[k2], xi3), (T)1);
      storev(out + (3 * i + 2) * co, w);
    }
  } else if constexpr (MODE == SP_DIV_SMALL) {
    // r_i = -i sum_j xi_j s_ij after the forward x transform
    const T xi2 = (T)xi_of(o, g.n2, g.il2), xi3 = (T)xi_of(col, g.n3, g.il3);
    if constexpr (PARTS) {
      // row i: s_i1, s_i2, s_i3 as stored components
      const int i = part;
      // stored index of (i, j): i for i = j, else 3 / 4 / 5 for the pairs summing to 3 / 2 / 1
      auto comp = [&](int j) { return (i == j) ? i : 6 - (i + j); };
      cpx<T> a[N2];
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) a[k2] = mk<T>(0, 0);
      cpx<T> nx[N1];
      loadv(in + comp(0) * sg.cstride_in, nx);
#pragma unroll 1
      for (int jj = 0; jj < 3; ++jj) {
        const int c = comp(jj);
        cpx<T> v[EM];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = nx[n1];
        if (jj + 1 < 3) loadv(in + comp(jj + 1) * sg.cstride_in, nx);
        fft(v);
        // the row whose first index is the component's writes its mean
        const int first = (c < 3) ? c : (c == 3 ? 1 : 0);
        if (dc_out != nullptr && first == i && lout && o == 0 && col == 0 && t == 0) dc_out[c] = (double)v[0].x;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const T x1 = (T)xi_of(t + N1 * k2, g.n1, g.il1);
          const T xj = (jj == 0) ? x1 : (jj == 1 ? xi2 : xi3);
          a[k2] = add(a[k2], scl(v[k2], xj));
        }
      }
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) a[k2] = muli(a[k2], (T)-1);
      storev(out + i * sg.cstride_out, a);
    } else {
    cpx<T> a0[N2], a1[N2], a2[N2];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) a0[k2] = a1[k2] = a2[k2] = mk<T>(0, 0);
    cpx<T> nx[N1];
    loadv(in, nx);
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
      cpx<T> v[EM];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) v[n1] = nx[n1];
      if (c + 1 < 6) loadv(in + (c + 1) * sg.cstride_in, nx);
      fft(v);
      if (dc_out != nullptr && lout && o == 0 && col == 0 && t == 0) dc_out[c] = (double)v[0].x;
      // stored order 11 22 33 23 13 12
      const int ii = (c < 3) ? c : (c == 3 ? 1 : 0);
      const int jj = (c < 3) ? c : (c == 5 ? 1 : 2);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const T x1 = (T)xi_of(t + N1 * k2, g.n1, g.il1);
        const T xj = (jj == 0) ? x1 : (jj == 1 ? xi2 : xi3);
        const T xi_ = (ii == 0) ? x1 : (ii == 1 ? xi2 : xi3);
        const cpx<T> t1 = scl(v[k2], xj);
        if (ii == 0) a0[k2] = add(a0[k2], t1);
        else if (ii == 1) a1[k2] = add(a1[k2], t1);
        else a2[k2] = add(a2[k2], t1);
        if (ii != jj) {
          const cpx<T> t2 = scl(v[k2], xi_);
          if (jj == 0) a0[k2] = add(a0[k2], t2);
          else if (jj == 1) a1[k2] = add(a1[k2], t2);
          else a2[k2] = add(a2[k2], t2);
        }
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      a0[k2] = muli(a0[k2], (T)-1);
      a1[k2] = muli(a1[k2], (T)-1);
      a2[k2] = muli(a2[k2], (T)-1);
    }
    storev(out, a0);
    storev(out + sg.cstride_out, a1);
    storev(out + 2 * sg.cstride_out, a2);
    }
  } else {
    // SP_DIV_FINITE, row by row: r_i = -i (xi1 F[P_i1] + F[xi2 P_i2 + xi3 P_i3])
    const T xi2 = (T)xi_of(o, g.n2, g.il2), xi3 = (T)xi_of(col, g.n3, g.il3);
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      cpx<T> P1[N1], P2[N1], P3[N1];
      loadv(in + (3 * i) * sg.cstride_in, P1);
      loadv(in + (3 * i + 1) * sg.cstride_in, P2);
      loadv(in + (3 * i + 2) * sg.cstride_in, P3);
      cpx<T> C[EM], A[EM];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        C[n1] = add(scl(P2[n1], xi2), scl(P3[n1], xi3));
        A[n1] = P1[n1];
      }
      if (dc_out != nullptr && tile == 0) {
        // the k1 = 0 coefficients of the line (k2, k3) = (0, 0) are the line
        // sums; C is zero there (xi2 = xi3 = 0), so P_i2 and P_i3 are summed
        // directly (column s = 0 of the first tile, through the exchange buffer)
        if (s == 0 && lin) {
          double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1) {
            a1 += (double)P1[n1].x;
            a2 += (double)P2[n1].x;
            a3 += (double)P3[n1].x;
          }
          lds[3 * t] = mk<T>((T)a1, 0);
          lds[3 * t + 1] = mk<T>((T)a2, 0);
          lds[3 * t + 2] = mk<T>((T)a3, 0);
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int u = 0; u < N2; ++u) acc += (double)lds[3 * u + j].x;
            dc_out[3 * i + j] = acc;
          }
        }
        __syncthreads();
      }
      fft(C);
      fft(A);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const T x1 = (T)xi_of(t + N1 * k2, g.n1, g.il1);
        A[k2] = muli(add(scl(A[k2], x1), C[k2]), (T)-1);
      }
      storev(out + i * sg.cstride_out, A);
    }
  }
}

// ---------------------------------------------------------------- z pass
// One wave handles LB = 64 / TL z lines of M = n3/2 complex points (the
// real transform of length n3 as a complex one of length M with the
// even/odd split).  Inverse with plan (N1, N2), forward with plan (N2, N1):
// the forward transform's input distribution is the inverse's output one,
// so the tangent is applied where the values lie, and the forward output
// lands in the inverse's input distribution (thread t < N2, register m:
// coefficient N2 m + t), where the split pairs it with coefficient M - k
// on lane (N2 - t) mod N2.
template <int M>
struct MixedLine {
  static constexpr int N1 = mixed_n1(M);
  static constexpr int N2 = M / N1;
  static constexpr int EM = N1 > N2 ? N1 : N2;
  static constexpr int TL = EM;
  static constexpr int LB = 64 / TL;
  static constexpr int PITCH = M + TL + 1;  // both plans' padded exchange rows fit
};

template <typename T>
__device__ __forceinline__ cpx<T> shfl_cx(cpx<T> v, int src) {
  return mk<T>(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// inverse real transform of one component: coefficients src[0..M] of the
// lane's line -> packed pairs at n = t + N1 k2 in e[k2] (t < N1).  NSUM > 1
// transforms the sum of NSUM components `sstride` apart (the transform is
// linear).
template <typename T, int M, int NSUM = 1>
__device__ __forceinline__ void mixed_line_inverse(const cpx<T>* src, bool valid, int t, int tj, int partner,
                                                   cpx<T>* lds, int off, const cpx<T>* tw, const cpx<T>* rtw,
                                                   cpx<T>* e, long long sstride = 0) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM;
  const bool lin = valid && t < N2;
  cpx<T> X[N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
    X[n1] = lin ? src[N2 * n1 + t] : mk<T>(0, 0);
#pragma unroll
    for (int s = 1; s < NSUM; ++s)
      if (lin) X[n1] = add(X[n1], src[s * sstride + N2 * n1 + t]);
  }
  cpx<T> XN = (valid && t == 0) ? src[M] : mk<T>(0, 0);
#pragma unroll
  for (int s = 1; s < NSUM; ++s)
    if (valid && t == 0) XN = add(XN, src[s * sstride + M]);
  cpx<T> Z[EM];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
    const cpx<T> sh = shfl_cx(X[N1 - 1 - n1], partner);
    const cpx<T> own = (n1 == 0) ? XN : X[(N1 - n1) % N1];
    const cpx<T> Xm = conj((t == 0) ? own : sh);
    const int k = (t < N2) ? N2 * n1 + t : 0;
    const cpx<T> Ev = add(X[n1], Xm);
    const cpx<T> Od = mul(sub(X[n1], Xm), conj(rtw[k]));
    Z[n1] = add(Ev, muli(Od, (T)1));
  }
  two_step_fft<T, N1, N2, 1>(Z, tj, lds, 1, off, tw, (T)1);
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) e[k2] = Z[k2];
}

// forward real transform of packed pairs e[k2] (n = t + N1 k2), scaled,
// stored to dst[0..M]
template <typename T, int M>
__device__ __forceinline__ void mixed_line_forward(cpx<T>* dst, bool valid, int t, int tj, int partner,
                                                   cpx<T>* lds, int off, const cpx<T>* tw, const cpx<T>* rtw,
                                                   const cpx<T>* e, T scale) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM;
  cpx<T> Z[EM];
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) Z[k2] = e[k2];
  two_step_fft<T, N2, N1, 1>(Z, tj, lds, 1, off, tw, (T)-1);
  // thread t < N2 now holds coefficient N2 m + t in Z[m], m < N1
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    const cpx<T> sh = shfl_cx(Z[N1 - 1 - m], partner);
    const cpx<T> own = Z[(N1 - m) % N1];
    const cpx<T> Zm = conj((t == 0) ? own : sh);
    const int k = (t < N2) ? N2 * m + t : 0;
    const cpx<T> Ev = scl(add(Z[m], Zm), (T)0.5);
    const cpx<T> Od = mul(rtw[k], scl(sub(Z[m], Zm), (T)0.5));
    if (valid && t < N2) dst[k] = scl(sub(Ev, muli(Od, (T)1)), scale);
  }
  if (valid && t == 0) {
    const cpx<T> Z0 = Z[0], Zm = conj(Z[0]);
    const cpx<T> Ev = scl(add(Z0, Zm), (T)0.5);
    const cpx<T> Od = mul(rtw[M], scl(sub(Z0, Zm), (T)0.5));
    dst[M] = scl(sub(Ev, muli(Od, (T)1)), scale);
  }
}

// fused z pass of one wave (LB lines): inverse real transforms, tangent
// (ISO: one component at a time after the trace; otherwise all
// components), energy, forward real transforms.  Returns the wave's energy
// sum (1/N of sum eps : sigma) in every lane.  ISO only: part 0 does the
// normal components, part 1 the shear ones, -1 all six.
template <typename T, int M, int KIN, int ISO>
__device__ __forceinline__ double mixed_line_fused(const cpx<T>* in, cpx<T>* out, const Geom& g,
                                                   const cpx<T>* tw, const cpx<T>* rtw, cpx<T>* lds,
                                                   const TangentArgs<T>& tn, const double* __restrict__ macro_dev,
                                                   long long block, int lane, int part = -1) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM, TL = L::TL, LB = L::LB, PITCH = L::PITCH;
  constexpr int NC = (KIN == KIN_SMALL) ? 6 : 9;
  const int line = lane / TL, t = lane % TL;
  const long long nlines = (long long)g.n1 * g.n2;
  const long long gl = block * LB + line;
  const bool active = line < LB;
  const bool valid = active && gl < nlines;
  const int tj = active ? t : TL;  // lanes past the last line take no part
  const int partner = active ? line * TL + ((t < N2) ? (N2 - t) % N2 : t) : lane;
  const int off = (active ? line : 0) * PITCH;
  const T scale = (T)g.inv_nvox;
  const int nh3 = g.nh3, n3 = g.n3;
  double mac[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) mac[c] = macro_dev ? macro_dev[c] : 0.0;
  double energy = 0.0;
  const cpx<T>* inl = in + (valid ? gl : 0) * nh3;
  cpx<T>* outl = out + (valid ? gl : 0) * nh3;
  const bool lt = valid && t < N1;

  if constexpr (ISO == 1) {
    // The normal components couple only through the trace: one inverse
    // transform of their summed coefficients gives tr(eps), and every
    // component is then transformed, updated (lam tr + 2 mu eps_c, or
    // 2 mu eps_c for shear) and written back on its own, so at most two
    // components are in registers.
    cpx<T> tr[EM];
    if (part != 1) mixed_line_inverse<T, M, 3>(inl, valid, t, tj, partner, lds, off, tw, rtw, tr, g.nh);
    const T trmac = (T)(mac[0] + mac[1] + mac[2]);
    const int cbeg = (part == 1) ? 3 : 0, cend = (part == 0) ? 3 : 6;
#pragma unroll 1
    for (int c = cbeg; c < cend; ++c) {
      cpx<T> e1[EM];
      mixed_line_inverse<T, M>(inl + c * g.nh, valid, t, tj, partner, lds, off, tw, rtw, e1);
      const T mc = (T)mac[c];
      if (lt) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const int n = t + N1 * k2;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const long long vox = gl * n3 + 2 * n + h;
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
            const T ev = (h == 0 ? e1[k2].x : e1[k2].y) + mc;
            T sv;
            if (c < 3) {
              const T trv = (h == 0 ? tr[k2].x : tr[k2].y) + trmac;
              sv = lam * trv + (mu + mu) * ev;
              energy += (double)(ev * sv);
            } else {
              sv = (mu + mu) * ev;
              energy += 2.0 * (double)(ev * sv);
            }
            if (h == 0) e1[k2].x = sv;
            else e1[k2].y = sv;
          }
        }
      }
      mixed_line_forward<T, M>(outl + c * g.nh, valid, t, tj, partner, lds, off, tw, rtw, e1, scale);
    }
  } else {
    cpx<T> e[NC][EM];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      mixed_line_inverse<T, M>(inl + c * g.nh, valid, t, tj, partner, lds, off, tw, rtw, e[c]);
    if (lt) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int n = t + N1 * k2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long long vox = gl * n3 + 2 * n + h;
          T ev[NC], sv[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) ev[c] = (h == 0 ? e[c][k2].x : e[c][k2].y) + (T)mac[c];
          if constexpr (KIN == KIN_SMALL) {
            if (tn.kind == TAN_ANISO_FIELD) tangent_small_field<T>(tn, vox, g.nvox, ev, sv);
            else tangent_small<T>(tn, vox, ev, sv);
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
            if (h == 0) e[c][k2].x = sv[c];
            else e[c][k2].y = sv[c];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
      mixed_line_forward<T, M>(outl + c * g.nh, valid, t, tj, partner, lds, off, tw, rtw, e[c], scale);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) energy += __shfl_xor(energy, o, 64);
  return energy * g.inv_nvox;
}

// z pass of one line group (LB lines) by the NW waves of a block, for
// tangents that couple every component (anisotropic small-strain tangents,
// finite strains): wave w transforms
// the components w, w + NW, ... one at a time and stages their real values
// in LDS (X: [c][line][n], packed pairs n = 0..M-1), the block applies the
// tangent voxel by voxel from there, and every wave transforms its
// components back.  Only one component is in registers at a time, so the
// pass does not hold all nine (the register-resident version needs 256
// VGPRs and spills).  X holds NC = 6 (small strains) or 9 components.
// `lds` is the wave's own exchange buffer.  Returns
// this thread's share of the energy (1/N of sum eps : sigma); the caller
// sums over the block.  Every thread of the block must call it: the
// transforms and the staging use block barriers.
template <typename T, int M, int KIN, int LAW, int NW>
__device__ __forceinline__ double mixed_line_staged(const cpx<T>* in, cpx<T>* out, const Geom& g,
                                                    const cpx<T>* tw, const cpx<T>* rtw, cpx<T>* lds,
                                                    cpx<T>* __restrict__ X, const TangentArgs<T>& tn,
                                                    const double* __restrict__ macro_dev, long long group,
                                                    int wave, int lane) {
  using L = MixedLine<M>;
  constexpr int N1 = L::N1, N2 = L::N2, EM = L::EM, TL = L::TL, LB = L::LB, PITCH = L::PITCH;
  constexpr int NC = (KIN == KIN_SMALL) ? 6 : 9;
  const int line = lane / TL, t = lane % TL;
  const long long nlines = (long long)g.n1 * g.n2;
  const long long gl = group * LB + line;
  const bool active = line < LB;
  const bool valid = active && gl < nlines;
  const int tj = active ? t : TL;  // lanes past the last line take no part
  const int partner = active ? line * TL + ((t < N2) ? (N2 - t) % N2 : t) : lane;
  const int off = (active ? line : 0) * PITCH;
  const int nh3 = g.nh3, n3 = g.n3;
  const cpx<T>* inl = in + (valid ? gl : 0) * nh3;
  cpx<T>* outl = out + (valid ? gl : 0) * nh3;
  const bool lt = valid && t < N1;
  // The transforms exchange through LDS behind block barriers, so every
  // wave runs the same number of rounds; a wave with no component left in
  // the last round transforms zeros and stores nothing.
  constexpr int NR = (NC + NW - 1) / NW;
#pragma unroll 1
  for (int j = 0; j < NR; ++j) {
    const int c = wave + NW * j;
    const bool has = c < NC;
    cpx<T> e[EM];
    mixed_line_inverse<T, M>(inl + (has ? c : 0) * g.nh, valid && has, t, tj, partner, lds, off, tw, rtw, e);
    if (lt && has) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) X[(c * LB + line) * M + t + N1 * k2] = e[k2];
    }
  }
  __syncthreads();
  double mac[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) mac[c] = macro_dev ? macro_dev[c] : 0.0;
  double energy = 0.0;
  for (int idx = (int)threadIdx.x; idx < LB * M; idx += NW * 64) {
    const int ln = idx / M, n = idx - ln * M;
    const long long gln = group * LB + ln;
    if (gln >= nlines) continue;
    cpx<T> v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = X[(c * LB + ln) * M + n];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long long vox = gln * n3 + 2 * n + h;
      T ev[NC], sv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) ev[c] = (h == 0 ? v[c].x : v[c].y) + (T)mac[c];
      if constexpr (KIN == KIN_SMALL) {
        if (tn.kind == TAN_ANISO_FIELD) tangent_small_field<T>(tn, vox, g.nvox, ev, sv);
        else tangent_small<T>(tn, vox, ev, sv);
        energy += (double)(ev[0] * sv[0] + ev[1] * sv[1] + ev[2] * sv[2]) +
                  2.0 * (double)(ev[3] * sv[3] + ev[4] * sv[4] + ev[5] * sv[5]);
      } else {
        tangent_finite<T, LAW>(tn, vox, g.nvox, ev, sv);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc += (double)(ev[c] * sv[c]);
        energy += acc;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (h == 0) v[c].x = sv[c];
        else v[c].y = sv[c];
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) X[(c * LB + ln) * M + n] = v[c];
  }
  __syncthreads();
  const T scale = (T)g.inv_nvox;
#pragma unroll 1
  for (int j = 0; j < NR; ++j) {
    const int c = wave + NW * j;
    const bool has = c < NC;
    cpx<T> e[EM];
#pragma unroll
    for (int k2 = 0; k2 < EM; ++k2)
      e[k2] = (lt && has && k2 < N2) ? X[(c * LB + line) * M + t + N1 * k2] : mk<T>(0, 0);
    mixed_line_forward<T, M>(outl + (has ? c : 0) * g.nh, valid && has, t, tj, partner, lds, off, tw, rtw, e, scale);
  }
  return energy * g.inv_nvox;
}

}  // namespace dbfft
