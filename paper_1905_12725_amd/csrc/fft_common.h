// Device-side complex arithmetic and the LDS-resident Stockham engine.
//
// A block transforms S independent sequences of length n held in LDS with
// layout [n][S] (sequence index fastest).  Each stage of radix R reads R
// elements spaced n/R apart, applies the twiddles of the sub-transform
// length Ns*R, does a radix-R DFT and writes R elements spaced Ns apart
// (Stockham autosort: natural order in and out, ping-pong buffers).
#pragma once

#include "dbfft_internal.h"

namespace dbfft {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> add(cpx<T> a, cpx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> sub(cpx<T> a, cpx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> scl(cpx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cpx<T> mul(cpx<T> a, cpx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk<T>(a.x, -a.y); }
// multiply by (d * i), d = +-1
template <typename T>
__device__ __forceinline__ cpx<T> muli(cpx<T> a, T d) { return mk<T>(-d * a.y, d * a.x); }

// frequency 2 pi m / L of DFT index k on an axis of n points and length L
// (Sec. 2.1; inv_len = 1/L), m the signed index; the even-grid Nyquist index
// gets 0.
__device__ __forceinline__ double xi_of(int k, int n, double inv_len) {
  int m = (2 * k < n) ? k : k - n;
  if (2 * k == n) m = 0;
  return (double)m * (kTwoPi * inv_len);  // 2 pi / L is the same for every call of a pass
}

// radix-R DFT in registers, exponent sign d (-1 forward, +1 inverse)
template <typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = add(a, b);
  v[1] = sub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3, T d) {
  cpx<T> t0 = add(a0, a2), t1 = sub(a0, a2), t2 = add(a1, a3), t3 = muli(sub(a1, a3), d);
  a0 = add(t0, t2);
  a2 = sub(t0, t2);
  a1 = add(t1, t3);
  a3 = sub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft3(cpx<T>* v, T d) {
  const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
  cpx<T> s = add(v[1], v[2]), df = sub(v[1], v[2]);
  cpx<T> y0 = add(v[0], s);
  cpx<T> m = sub(v[0], scl(s, (T)0.5));
  cpx<T> t = muli(scl(df, h), d);
  v[0] = y0;
  v[1] = add(m, t);
  v[2] = sub(m, t);
}

template <typename T>
__device__ __forceinline__ void dft5(cpx<T>* v, T d) {
  const T c1 = (T)0.30901699437494742410;   // cos(2 pi/5)
  const T c2 = (T)-0.80901699437494742410;  // cos(4 pi/5)
  const T s1 = (T)0.95105651629515357212;   // sin(2 pi/5)
  const T s2 = (T)0.58778525229247312917;   // sin(4 pi/5)
  cpx<T> s14 = add(v[1], v[4]), d14 = sub(v[1], v[4]);
  cpx<T> s23 = add(v[2], v[3]), d23 = sub(v[2], v[3]);
  cpx<T> a = v[0];
  cpx<T> m1 = add(a, add(scl(s14, c1), scl(s23, c2)));
  cpx<T> m2 = add(a, add(scl(s14, c2), scl(s23, c1)));
  cpx<T> t1 = muli(add(scl(d14, s1), scl(d23, s2)), d);
  cpx<T> t2 = muli(sub(scl(d14, s2), scl(d23, s1)), d);
  v[0] = add(a, add(s14, s23));
  v[1] = add(m1, t1);
  v[4] = sub(m1, t1);
  v[2] = add(m2, t2);
  v[3] = sub(m2, t2);
}

// 7 points: the six non-zero inputs in conjugate pairs (1,6), (2,5), (3,4);
// output m gathers sum_k s_k cos(2 pi k m/7) and d i sum_k d_k sin(2 pi k m/7)
template <typename T>
__device__ __forceinline__ void dft7(cpx<T>* v, T d) {
  const T c[3] = {(T)0.62348980185873359439, (T)-0.22252093395631433737, (T)-0.90096886790241903498};
  const T sn[3] = {(T)0.78183148246802980363, (T)0.97492791218182361934, (T)0.43388373911755823142};
  const cpx<T> a = v[0];
  cpx<T> sp[3], dm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sp[k] = add(v[k + 1], v[6 - k]);
    dm[k] = sub(v[k + 1], v[6 - k]);
  }
  v[0] = add(a, add(sp[0], add(sp[1], sp[2])));
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    cpx<T> re = a, im = mk<T>(0, 0);
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
      const int j = (k * m) % 7;  // cos and sin of 2 pi j / 7 through the pair index
      const int q = (j <= 3) ? j : 7 - j;
      const T sg = (j <= 3) ? (T)1 : (T)-1;
      re = add(re, scl(sp[k - 1], c[q - 1]));
      im = add(im, scl(dm[k - 1], sg * sn[q - 1]));
    }
    const cpx<T> t = muli(im, d);
    v[m] = add(re, t);
    v[7 - m] = sub(re, t);
  }
}

template <typename T>
__device__ __forceinline__ void dft8(cpx<T>* v, T d) {
  const T r = (T)0.70710678118654752440;
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, d);
  dft4(o0, o1, o2, o3, d);
  // W8 = (1 + d i)/sqrt2, W8^2 = d i, W8^3 = (-1 + d i)/sqrt2
  cpx<T> w1 = scl(add(o1, muli(o1, d)), r);
  cpx<T> w2 = muli(o2, d);
  cpx<T> w3 = scl(sub(muli(o3, d), o3), r);
  v[0] = add(e0, o0);
  v[4] = sub(e0, o0);
  v[1] = add(e1, w1);
  v[5] = sub(e1, w1);
  v[2] = add(e2, w2);
  v[6] = sub(e2, w2);
  v[3] = add(e3, w3);
  v[7] = sub(e3, w3);
}

template <typename T, int R>
__device__ __forceinline__ void dftR(cpx<T>* v, T d) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v, d);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3], d);
  else if constexpr (R == 5) dft5(v, d);
  else if constexpr (R == 7) dft7(v, d);
  else if constexpr (R == 8) dft8(v, d);
}

// One Stockham stage over S sequences of length n.  tw[t] = exp(-2 pi i t / n).
template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                               const cpx<T>* __restrict__ tw, int n, int S, int Ns, T d,
                                               int tid, int nthr) {
  const int nr = n / R;
  const int step = n / (Ns * R);
  const int total = nr * S;
  for (int b = tid; b < total; b += nthr) {
    const int s = b % S;
    const int j = b / S;
    const int k = j % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nr) * S + s];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[k * r * step];
        w.y *= -d;  // forward table; conjugate for the inverse (d = +1)
        v[r] = mul(v[r], w);
      }
    }
    dftR<T, R>(v, d);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * S + s] = v[r];
  }
}

// Full transform; returns the buffer holding the result.  Ends with a barrier.
template <typename T>
__device__ cpx<T>* fft_lds(cpx<T>* A, cpx<T>* B, const cpx<T>* tw, const FftPlan& plan, int S, T d, int tid,
                           int nthr) {
  cpx<T>* src = A;
  cpx<T>* dst = B;
  const int n = plan.n;
  for (int st = 0; st < plan.nstages; ++st) {
    const int R = plan.radix[st], Ns = plan.ns[st];
    switch (R) {
      case 2: stockham_stage<T, 2>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
      case 3: stockham_stage<T, 3>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
      case 4: stockham_stage<T, 4>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
      case 5: stockham_stage<T, 5>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
      case 7: stockham_stage<T, 7>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
      default: stockham_stage<T, 8>(src, dst, tw, n, S, Ns, d, tid, nthr); break;
    }
    __syncthreads();
    cpx<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Block-wide FP64 sum (NT threads, result valid in thread 0).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  }
  return s;
}

// alpha = <r, M r> / <p, K p> from the z pass's energy partials
// (fixed-order sum), done by the first block of a following pass (every
// thread of that block calls it); marks the step pending for the direction
// kernel, or flags a breakdown.  A converged iteration clears the pending
// step.  The macroscopic part of the step is taken by the beta kernel.
template <int NT>
__device__ __forceinline__ void alpha_task(PcgScalars* sc, const double* __restrict__ eparts, int neparts) {
  __shared__ double red[NT / 64];
  if (sc->converged) {
    if (threadIdx.x == 0) sc->pending = 0;
    return;
  }
  double e = 0.0;
  for (int i = threadIdx.x; i < neparts; i += NT) e += eparts[i];
  const double pq = block_sum<NT>(e, red);
  if (threadIdx.x == 0) {
    sc->pq = pq;
    if (!(pq > 0.0)) {
      sc->converged = 2;
      sc->pending = 0;
    } else {
      sc->alpha = sc->rz / pq;
      sc->pending = 1;
    }
  }
}

// alpha_task by the first wave of a block alone (fixed-order sum over its
// lanes, then across them), for blocks whose size is not a multiple of 64;
// the other threads return at once and nothing waits on a barrier.
__device__ __forceinline__ void alpha_task_wave(PcgScalars* sc, const double* __restrict__ eparts, int neparts) {
  if (threadIdx.x >= 64) return;
  if (sc->converged) {
    if (threadIdx.x == 0) sc->pending = 0;
    return;
  }
  // eight loads in flight per lane (the partials of a large grid number a
  // few thousand), summed in a fixed order
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 7 * 64 < neparts; i += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += eparts[i + u * 64];
  }
  for (; i < neparts; i += 64) a[0] += eparts[i];
  double e = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (threadIdx.x == 0) {
    sc->pq = e;
    if (!(e > 0.0)) {
      sc->converged = 2;
      sc->pending = 0;
    } else {
      sc->alpha = sc->rz / e;
      sc->pending = 1;
    }
  }
}

}  // namespace dbfft
