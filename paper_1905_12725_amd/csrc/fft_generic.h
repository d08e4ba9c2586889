// Generic (runtime-plan) FFT pass bodies, shared by the single-cell and the
// batched kernels.  See fft_passes.hip for the pass structure.
#pragma once

#include "fft_common.h"

namespace dbfft {

constexpr int kStridedThreads = 256;
constexpr int kStridedQ = 8;  // max elements per thread in fused modes

template <typename T, int MODE>
__device__ __forceinline__ void strided_core(const cpx<T>* in, cpx<T>* out, const StridedGeom& sg, const Geom& g,
                                             const FftPlan& plan, const cpx<T>* __restrict__ twg, T d, int TZ,
                                             double* __restrict__ dc_out, int tile, int o, int c,
                                             unsigned char* smem_raw) {
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = sg.nline;
  cpx<T>* A = tw + n;
  cpx<T>* B = A + n * TZ;
  const int tid = threadIdx.x;
  constexpr int NT = kStridedThreads;

  const int col0 = tile * TZ;
  const int ncol = min(TZ, sg.ncols - col0);
  const long long base = (long long)o * sg.ostride + col0;
  const int total = n * TZ;

  for (int t = tid; t < n; t += NT) tw[t] = twg[t];

  if constexpr (MODE == SP_PLAIN) {
    const cpx<T>* src = in + c * sg.cstride_in + base;
    cpx<T>* dstp = out + c * sg.cstride_out + base;
    for (int e = tid; e < total; e += NT) {
      const int ln = e / TZ, s = e - ln * TZ;
      A[e] = (s < ncol) ? src[ln * sg.lstride + s] : mk<T>(0, 0);
    }
    __syncthreads();
    cpx<T>* res = fft_lds<T>(A, B, tw, plan, TZ, d, tid, NT);
    for (int e = tid; e < total; e += NT) {
      const int ln = e / TZ, s = e - ln * TZ;
      if (s < ncol) dstp[ln * sg.lstride + s] = res[e];
    }
  } else {
    // x pass with a fused pointwise operator: line index = k1, other = k2, column = k3
    const T xi2 = (T)xi_of(o, g.n2, g.il2);
    if constexpr (MODE == SP_GRAD_SMALL || MODE == SP_GRAD_FINITE) {
      cpx<T> a0[kStridedQ], a1[kStridedQ], a2[kStridedQ];
#pragma unroll
      for (int q = 0; q < kStridedQ; ++q) {
        const int e = tid + q * NT;
        a0[q] = a1[q] = a2[q] = mk<T>(0, 0);
        if (e < total) {
          const int ln = e / TZ, s = e - ln * TZ;
          if (s < ncol) {
            const long long off = base + ln * sg.lstride + s;
            a0[q] = in[off];
            a1[q] = in[off + sg.cstride_in];
            a2[q] = in[off + 2 * sg.cstride_in];
          }
        }
      }
      constexpr int NC = (MODE == SP_GRAD_SMALL) ? 6 : 9;
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int q = 0; q < kStridedQ; ++q) {
          const int e = tid + q * NT;
          if (e < total) {
            const int ln = e / TZ, s = e - ln * TZ;
            const T x1 = (T)xi_of(ln, g.n1, g.il1);
            const T x3 = (T)xi_of(col0 + s, g.n3, g.il3);
            const T xi[3] = {x1, xi2, x3};
            const cpx<T> a[3] = {a0[q], a1[q], a2[q]};
            cpx<T> v;
            if constexpr (MODE == SP_GRAD_SMALL) {
              // stored order 11 22 33 23 13 12: eps_ij = i/2 (xi_j a_i + xi_i a_j)
              const int ii = (c < 3) ? c : (c == 3 ? 1 : 0);
              const int jj = (c < 3) ? c : (c == 5 ? 1 : 2);
              v = add(scl(a[ii], xi[jj]), scl(a[jj], xi[ii]));
              v = muli(scl(v, (T)0.5), (T)1);
            } else {
              // H_iJ = i xi_J a_i, row-major
              const int ii = c / 3, jj = c % 3;
              v = muli(scl(a[ii], xi[jj]), (T)1);
            }
            A[e] = v;
          }
        }
        __syncthreads();
        cpx<T>* res = fft_lds<T>(A, B, tw, plan, TZ, d, tid, NT);
        cpx<T>* dstp = out + c * sg.cstride_out + base;
        for (int e = tid; e < total; e += NT) {
          const int ln = e / TZ, s = e - ln * TZ;
          if (s < ncol) dstp[ln * sg.lstride + s] = res[e];
        }
        __syncthreads();
      }
    } else {
      // SP_DIV_*: forward x transform of each stress component, then
      // r_i = -i xi_j s_ij accumulated per owned element.
      cpx<T> acc0[kStridedQ], acc1[kStridedQ], acc2[kStridedQ];
#pragma unroll
      for (int q = 0; q < kStridedQ; ++q) acc0[q] = acc1[q] = acc2[q] = mk<T>(0, 0);
      constexpr int NC = (MODE == SP_DIV_SMALL) ? 6 : 9;
      for (int c = 0; c < NC; ++c) {
        const cpx<T>* src = in + c * sg.cstride_in + base;
        for (int e = tid; e < total; e += NT) {
          const int ln = e / TZ, s = e - ln * TZ;
          A[e] = (s < ncol) ? src[ln * sg.lstride + s] : mk<T>(0, 0);
        }
        __syncthreads();
        cpx<T>* res = fft_lds<T>(A, B, tw, plan, TZ, d, tid, NT);
        if (dc_out != nullptr && o == 0 && tile == 0 && tid == 0) dc_out[c] = (double)res[0].x;
#pragma unroll
        for (int q = 0; q < kStridedQ; ++q) {
          const int e = tid + q * NT;
          if (e < total) {
            const int ln = e / TZ, s = e - ln * TZ;
            const T x1 = (T)xi_of(ln, g.n1, g.il1);
            const T x3 = (T)xi_of(col0 + s, g.n3, g.il3);
            const T xi[3] = {x1, xi2, x3};
            const cpx<T> v = res[e];
            int ii, jj;
            if constexpr (MODE == SP_DIV_SMALL) {
              ii = (c < 3) ? c : (c == 3 ? 1 : 0);
              jj = (c < 3) ? c : (c == 5 ? 1 : 2);
            } else {
              ii = c / 3;
              jj = c % 3;
            }
            // row ii gets xi_jj s; for a symmetric off-diagonal pair row jj gets xi_ii s too
            const cpx<T> t1 = scl(v, xi[jj]);
            if (ii == 0) acc0[q] = add(acc0[q], t1);
            else if (ii == 1) acc1[q] = add(acc1[q], t1);
            else acc2[q] = add(acc2[q], t1);
            if (MODE == SP_DIV_SMALL && ii != jj) {
              const cpx<T> t2 = scl(v, xi[ii]);
              if (jj == 0) acc0[q] = add(acc0[q], t2);
              else if (jj == 1) acc1[q] = add(acc1[q], t2);
              else acc2[q] = add(acc2[q], t2);
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < kStridedQ; ++q) {
        const int e = tid + q * NT;
        if (e < total) {
          const int ln = e / TZ, s = e - ln * TZ;
          if (s < ncol) {
            const long long off = base + ln * sg.lstride + s;
            out[off] = muli(acc0[q], (T)-1);
            out[off + sg.cstride_out] = muli(acc1[q], (T)-1);
            out[off + 2 * sg.cstride_out] = muli(acc2[q], (T)-1);
          }
        }
      }
    }
  }
}

constexpr int kLineThreads = 256;

template <typename T>
__device__ __forceinline__ void tangent_small(const TangentArgs<T>& tn, long long vox, const T* e, T* s) {
  if (tn.kind == TAN_ISO_PHASE || tn.kind == TAN_ISO_FIELD) {
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
    const T tr = e[0] + e[1] + e[2];
    const T m2 = mu + mu;
    s[0] = lam * tr + m2 * e[0];
    s[1] = lam * tr + m2 * e[1];
    s[2] = lam * tr + m2 * e[2];
    s[3] = m2 * e[3];
    s[4] = m2 * e[4];
    s[5] = m2 * e[5];
  } else {
    // Mandel: v = (e11, e22, e33, r2 e23, r2 e13, r2 e12); upper triangle row-major
    const T r2 = (T)1.41421356237309504880;
    const T v[6] = {e[0], e[1], e[2], r2 * e[3], r2 * e[4], r2 * e[5]};
    T c[21];
    const double* gt = tn.grain_table + (long long)tn.grain[vox] * 21;
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = (T)gt[i];
    T o[6];
    int idx = 0;
    T Cm[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) {
        Cm[a][b] = c[idx];
        Cm[b][a] = c[idx];
        ++idx;
      }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) acc += Cm[a][b] * v[b];
      o[a] = acc;
    }
    const T ir2 = (T)0.70710678118654752440;
    s[0] = o[0];
    s[1] = o[1];
    s[2] = o[2];
    s[3] = o[3] * ir2;
    s[4] = o[4] * ir2;
    s[5] = o[5] * ir2;
  }
}

// 21-coefficient per-voxel field read (layout [21][nvox])
template <typename T>
__device__ __forceinline__ void tangent_small_field(const TangentArgs<T>& tn, long long vox, long long nvox,
                                                    const T* e, T* s) {
  const T r2 = (T)1.41421356237309504880;
  const T v[6] = {e[0], e[1], e[2], r2 * e[3], r2 * e[4], r2 * e[5]};
  T Cm[6][6];
  int idx = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b) {
      const T c = tn.field[(long long)idx * nvox + vox];
      Cm[a][b] = c;
      Cm[b][a] = c;
      ++idx;
    }
  T o[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    T acc = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc += Cm[a][b] * v[b];
    o[a] = acc;
  }
  const T ir2 = (T)0.70710678118654752440;
  s[0] = o[0];
  s[1] = o[1];
  s[2] = o[2];
  s[3] = o[3] * ir2;
  s[4] = o[4] * ir2;
  s[5] = o[5] * ir2;
}

// finite strain neo-Hookean tangent applied to H (row-major 3x3):
// dP = mu H + (mu - lam lnJ) F^-T H^T F^-T + lam (F^-T : H) F^-T
template <typename T>
__device__ __forceinline__ void tangent_neo(const TangentArgs<T>& tn, long long vox, long long nvox, const T* H,
                                            T* P) {
  T Fi[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Fi[i] = tn.field[(long long)i * nvox + vox];
  const T lnJ = tn.field[9LL * nvox + vox];
  const int p = tn.phase[vox];
  const T mu = (T)tn.mu[p], lam = (T)tn.lam[p];
  // FiT[i][J] = Fi[J][i]
  T tr = 0;  // F^-T : H = sum_iJ Fi[J][i] H[i][J]
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) tr += Fi[J * 3 + i] * H[i * 3 + J];
  // T1[a][J] = sum_b H[b][a] Fi[J][b]
  T T1[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) acc += H[b * 3 + a] * Fi[J * 3 + b];
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
      P[i * 3 + J] = mu * H[i * 3 + J] + c2 * acc + lam * tr * Fi[J * 3 + i];
    }
}

// finite strain Saint Venant-Kirchhoff tangent applied to H (row-major 3x3),
// from the per-voxel F and S: with C = F^T H,
// dP = H S + F (lam tr(C) I + mu (C + C^T))
template <typename T>
__device__ __forceinline__ void tangent_svk(const TangentArgs<T>& tn, long long vox, long long nvox, const T* H,
                                            T* P) {
  T F[9], S6[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = tn.field[(long long)i * nvox + vox];
#pragma unroll
  for (int a = 0; a < 6; ++a) S6[a] = tn.field[(long long)(9 + a) * nvox + vox];
  const T S[9] = {S6[0], S6[5], S6[4], S6[5], S6[1], S6[3], S6[4], S6[3], S6[2]};
  const int p = tn.phase[vox];
  const T mu = (T)tn.mu[p], lam = (T)tn.lam[p];
  T C[9];
#pragma unroll
  for (int K = 0; K < 3; ++K)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      T acc = 0;
#pragma unroll
      for (int m = 0; m < 3; ++m) acc += F[m * 3 + K] * H[m * 3 + J];
      C[K * 3 + J] = acc;
    }
  const T tr = C[0] + C[4] + C[8];
  T dS[9];
#pragma unroll
  for (int K = 0; K < 3; ++K)
#pragma unroll
    for (int J = 0; J < 3; ++J) dS[K * 3 + J] = mu * (C[K * 3 + J] + C[J * 3 + K]) + ((K == J) ? lam * tr : (T)0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      T acc = 0;
#pragma unroll
      for (int K = 0; K < 3; ++K) acc += H[i * 3 + K] * S[K * 3 + J] + F[i * 3 + K] * dS[K * 3 + J];
      P[i * 3 + J] = acc;
    }
}

// finite-strain tangent applied to H; LAW (a template parameter, so each
// kernel holds the registers of one law only): 2 Saint Venant-Kirchhoff,
// otherwise neo-Hookean
template <typename T, int LAW>
__device__ __forceinline__ void tangent_finite(const TangentArgs<T>& tn, long long vox, long long nvox, const T* H,
                                               T* P) {
  if constexpr (LAW == 2) tangent_svk<T>(tn, vox, nvox, H, P);
  else tangent_neo<T>(tn, vox, nvox, H, P);
}

// law selector of the finite-strain kernels for a tangent kind
inline int finite_law(int tan_kind) { return tan_kind == TAN_SVK_FIELD ? 2 : 0; }

template <typename T, int MODE, int KIN, int LAW = 0>
__device__ __forceinline__ void line_core(const void* in_v, void* out_v, const Geom& g, const FftPlan& plan,
                                          const cpx<T>* __restrict__ twg, const cpx<T>* __restrict__ rtwg,
                                          const TangentArgs<T>& tn, const double* __restrict__ macro_dev,
                                          const double* __restrict__ macro_add, double* __restrict__ partials,
                                          int L, int ncomp, long long lineblock, unsigned char* smem_raw) {
  constexpr int NT = kLineThreads;
  const int tid = threadIdx.x;
  // even n3: complex transforms of length Z = n3/2 on packed sample pairs;
  // odd n3: complex transforms of length Z = n3 on the samples themselves
  const int n3 = g.n3, M = n3 / 2, nh3 = g.nh3, Z = z_length(n3);
  const bool odd = (n3 & 1) != 0;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);  // Z
  cpx<T>* rtw = tw + Z;                               // M + 1
  cpx<T>* FA = rtw + (M + 1);                         // Z * L
  cpx<T>* FB = FA + Z * L;                            // Z * L
  cpx<T>* XB = FB + Z * L;                            // (M + 1) * L
  T* RB = reinterpret_cast<T*>(XB + (M + 1) * L);     // ncomp * L * n3
  __shared__ double red[NT / 64];

  const long long nlines = (long long)g.n1 * g.n2;
  const long long line0 = lineblock * L;
  const int nl = (int)min((long long)L, nlines - line0);

  for (int t = tid; t < Z; t += NT) tw[t] = twg[t];
  for (int t = tid; t <= M; t += NT) rtw[t] = rtwg[t];
  __syncthreads();

  const cpx<T>* inc = static_cast<const cpx<T>*>(in_v);
  const T* inr = static_cast<const T*>(in_v);
  cpx<T>* outc = static_cast<cpx<T>*>(out_v);
  T* outr = static_cast<T*>(out_v);

  // ---------------- inverse real transforms into RB
  if constexpr (MODE == LP_FUSED || MODE == LP_C2R || MODE == LP_STRESS) {
    for (int c = 0; c < ncomp; ++c) {
      const cpx<T>* src = inc + c * g.nh + line0 * nh3;
      for (int e = tid; e < nh3 * L; e += NT) {
        const int s = e / nh3, k = e - s * nh3;
        XB[k * L + s] = (s < nl) ? src[(long long)s * nh3 + k] : mk<T>(0, 0);
      }
      __syncthreads();
      if (odd) {
        // full spectrum from the half spectrum: X(n3 - k) = conj X(k)
        for (int e = tid; e < Z * L; e += NT) {
          const int k = e / L, s = e - k * L;
          FA[k * L + s] = (k < nh3) ? XB[k * L + s] : conj(XB[(n3 - k) * L + s]);
        }
      } else {
        for (int e = tid; e < M * L; e += NT) {
          const int k = e / L, s = e - k * L;
          const cpx<T> Xk = XB[k * L + s];
          const cpx<T> Xm = conj(XB[(M - k) * L + s]);
          const cpx<T> E = add(Xk, Xm);
          const cpx<T> O = mul(sub(Xk, Xm), conj(rtw[k]));
          FA[k * L + s] = add(E, muli(O, (T)1));
        }
      }
      __syncthreads();
      cpx<T>* res = fft_lds<T>(FA, FB, tw, plan, L, (T)1, tid, NT);
      T* rb = RB + (long long)c * L * n3;
      if (odd) {
        for (int e = tid; e < Z * L; e += NT) {
          const int nn = e / L, s = e - nn * L;
          rb[s * n3 + nn] = res[nn * L + s].x;
        }
      } else {
        for (int e = tid; e < M * L; e += NT) {
          const int nn = e / L, s = e - nn * L;
          const cpx<T> z = res[nn * L + s];
          rb[s * n3 + 2 * nn] = z.x;
          rb[s * n3 + 2 * nn + 1] = z.y;
        }
      }
      __syncthreads();
    }
  } else if constexpr (MODE == LP_R2C) {
    for (int c = 0; c < ncomp; ++c) {
      const T* src = inr + c * g.nvox + line0 * n3;
      T* rb = RB + (long long)c * L * n3;
      for (int e = tid; e < L * n3; e += NT) {
        const int s = e / n3;
        rb[e] = (s < nl) ? src[e] : (T)0;
      }
    }
    __syncthreads();
  }

  // ---------------- macro strain add / pointwise tangent
  double energy = 0.0;
  if constexpr (MODE == LP_FUSED || MODE == LP_CONST || MODE == LP_C2R || MODE == LP_STRESS) {
    T mac[9];
    constexpr int NC = (KIN == KIN_SMALL) ? 6 : 9;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      double m = 0.0;
      if (macro_dev) m += macro_dev[c];
      if (macro_add) m += macro_add[c];
      mac[c] = (T)m;
    }
    for (int v = tid; v < L * n3; v += NT) {
      const int s = v / n3, z = v - s * n3;
      if (s >= nl) continue;
      const long long vox = (line0 + s) * n3 + z;
      if constexpr (MODE == LP_C2R) {
        for (int c = 0; c < ncomp && c < 9; ++c) RB[((long long)c * L + s) * n3 + z] += mac[c];
      } else {
        T e[NC], sg[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const T base = (MODE == LP_CONST) ? (T)0 : RB[((long long)c * L + s) * n3 + z];
          e[c] = base + mac[c];
        }
        if constexpr (KIN == KIN_SMALL) {
          if (tn.kind == TAN_ANISO_FIELD) tangent_small_field<T>(tn, vox, g.nvox, e, sg);
          else tangent_small<T>(tn, vox, e, sg);
          energy += (double)(e[0] * sg[0] + e[1] * sg[1] + e[2] * sg[2]) +
                    2.0 * (double)(e[3] * sg[3] + e[4] * sg[4] + e[5] * sg[5]);
        } else {
          tangent_finite<T, LAW>(tn, vox, g.nvox, e, sg);
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < 9; ++c) acc += (double)(e[c] * sg[c]);
          energy += acc;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) RB[((long long)c * L + s) * n3 + z] = sg[c];
      }
    }
    __syncthreads();
  }

  if constexpr (MODE == LP_C2R || MODE == LP_STRESS) {
    for (int c = 0; c < ncomp; ++c) {
      T* dst = outr + c * g.nvox + line0 * n3;
      const T* rb = RB + (long long)c * L * n3;
      for (int e = tid; e < L * n3; e += NT) {
        const int s = e / n3;
        if (s < nl) dst[e] = rb[e];
      }
    }
    return;
  } else {
    // ---------------- forward real transforms of RB, scaled by 1/N
    const T scale = (T)g.inv_nvox;
    for (int c = 0; c < ncomp; ++c) {
      const T* rb = RB + (long long)c * L * n3;
      if (odd) {
        for (int e = tid; e < Z * L; e += NT) {
          const int nn = e / L, s = e - nn * L;
          FA[nn * L + s] = mk<T>(rb[s * n3 + nn], (T)0);
        }
      } else {
        for (int e = tid; e < M * L; e += NT) {
          const int nn = e / L, s = e - nn * L;
          FA[nn * L + s] = mk<T>(rb[s * n3 + 2 * nn], rb[s * n3 + 2 * nn + 1]);
        }
      }
      __syncthreads();
      cpx<T>* res = fft_lds<T>(FA, FB, tw, plan, L, (T)-1, tid, NT);
      cpx<T>* dst = outc + c * g.nh + line0 * nh3;
      if (odd) {
        for (int e = tid; e < nh3 * L; e += NT) {
          const int s = e / nh3, k = e - s * nh3;
          if (s < nl) dst[(long long)s * nh3 + k] = scl(res[k * L + s], scale);
        }
        __syncthreads();
        continue;
      }
      for (int e = tid; e < nh3 * L; e += NT) {
        const int s = e / nh3, k = e - s * nh3;
        if (s >= nl) continue;
        const int k0 = (k == M) ? 0 : k;
        const int km = (k == 0) ? 0 : M - k;
        const cpx<T> Zk = res[k0 * L + s];
        const cpx<T> Zm = conj(res[km * L + s]);
        const cpx<T> Ev = scl(add(Zk, Zm), (T)0.5);
        const cpx<T> Od = mul(rtw[k], scl(sub(Zk, Zm), (T)0.5));
        const cpx<T> X = sub(Ev, muli(Od, (T)1));
        dst[(long long)s * nh3 + k] = scl(X, scale);
      }
      __syncthreads();
    }
    if constexpr (MODE == LP_FUSED) {
      if (partials != nullptr) {
        const double tot = block_sum<NT>(energy, red);
        if (tid == 0) partials[lineblock] = tot * g.inv_nvox;
      }
    }
  }
}


}  // namespace dbfft
