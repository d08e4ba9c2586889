// Device bodies of the PCG kernels (complex CG with the per-frequency
// preconditioner of Sec. 2.5 eqs. pred2/pred3), shared by the single-cell and
// the batched kernels.
#pragma once

#include "fft_common.h"

namespace dbfft {

constexpr int kVecThreads = 256;

struct FreqIdx {
  int k1, k2, k3;
};

__device__ __forceinline__ FreqIdx decode(long long k, const Geom& g) {
  FreqIdx f;
  f.k3 = (int)(k % g.nh3);
  const long long t = k / g.nh3;
  f.k2 = (int)(t % g.n2);
  f.k1 = (int)(t / g.n2);
  return f;
}

__device__ __forceinline__ double half_weight(int k3, int n3) {
  return (k3 == 0 || 2 * k3 == n3) ? 1.0 : 2.0;
}

// z = [xi.Cbar.xi]^-1 r; zero on the null set (xi = 0).
__device__ __forceinline__ void precond(const PrecondArgs& pa, double x1, double x2, double x3,
                                        const cpx<double>* r, cpx<double>* z) {
  if (x1 == 0.0 && x2 == 0.0 && x3 == 0.0) {
    z[0] = z[1] = z[2] = mk<double>(0, 0);
    return;
  }
  const double pr[6] = {x1 * x1, x2 * x2, x3 * x3, x2 * x3, x1 * x3, x1 * x2};
  double A[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += pr[q] * pa.G[q][m];
    A[m] = acc;
  }
  // A = [[a d e], [d b f], [e f c]] with storage 00 11 22 12 02 01
  const double a = A[0], b = A[1], c = A[2], f = A[3], e = A[4], d = A[5];
  const double c00 = b * c - f * f, c01 = e * f - d * c, c02 = d * f - b * e;
  const double c11 = a * c - e * e, c12 = d * e - a * f, c22 = a * b - d * d;
  const double inv = 1.0 / (a * c00 + d * c01 + e * c02);
  const double M[3][3] = {{c00 * inv, c01 * inv, c02 * inv}, {c01 * inv, c11 * inv, c12 * inv},
                          {c02 * inv, c12 * inv, c22 * inv}};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      zr += M[i][k] * r[k].x;
      zi += M[i][k] * r[k].y;
    }
    z[i] = mk<double>(zr, zi);
  }
}

template <typename T>
__device__ __forceinline__ cpx<double> up(cpx<T> a) {
  return mk<double>((double)a.x, (double)a.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> down(cpx<double> a) {
  return mk<T>((T)a.x, (T)a.y);
}

// Index of the Hermitian partner (-k1, -k2, k3) of a point on a
// self-conjugate plane (k3 = 0 or k3 = n3/2) of the half spectrum.
__device__ __forceinline__ long long partner_index(const FreqIdx& f, const Geom& g) {
  const int p1 = (f.k1 == 0) ? 0 : g.n1 - f.k1;
  const int p2 = (f.k2 == 0) ? 0 : g.n2 - f.k2;
  return ((long long)p1 * g.n2 + p2) * g.nh3 + f.k3;
}

__device__ __forceinline__ bool conj_plane(int k3, int n3) { return k3 == 0 || 2 * k3 == n3; }

// x += alpha p (x == nullptr: x is left to the direction kernel, xp_core);
// r -= alpha q; partial <r, M r> and <r, r>.
// On the planes k3 = 0 and k3 = n3/2 the coefficients of a real field are
// Hermitian, a(-k1, -k2) = conj a(k1, k2), and the real inverse transform
// sees only that part.  Rounding in the transforms leaves a small
// anti-Hermitian part in q = K p that K can never remove again, so the
// residual is projected back: the thread of the lower index of each pair
// updates both entries of the pair (the other one skips it).
template <typename T>
__device__ __forceinline__ void update_core(cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                            const cpx<T>* __restrict__ p, const cpx<T>* __restrict__ q,
                                            const PcgScalars* __restrict__ sc, const PrecondArgs& pa, const Geom& g,
                                            double* __restrict__ partials, int chunk, int nchunks) {
  __shared__ double red[kVecThreads / 64];
  if (sc->converged) return;
  const double alpha = sc->alpha;
  double rz = 0.0, rr = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)chunk * kVecThreads + threadIdx.x; k < nh;
       k += (long long)nchunks * kVecThreads) {
    const FreqIdx f = decode(k, g);
    long long kp = k;
    if (conj_plane(f.k3, g.n3)) {
      kp = partner_index(f, g);
      if (kp < k) continue;
    }
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o = c * nh + k;
      cpx<double> rc = sub(up(r[o]), scl(up(q[o]), alpha));
      if (conj_plane(f.k3, g.n3)) {
        const long long op = c * nh + kp;
        const cpx<double> rp = sub(up(r[op]), scl(up(q[op]), alpha));
        rc = scl(add(rc, conj(rp)), 0.5);
        if (kp != k) r[op] = down<T>(conj(rc));
        if (x != nullptr) {
          const cpx<double> xc = scl(add(add(up(x[o]), scl(up(p[o]), alpha)),
                                         conj(add(up(x[op]), scl(up(p[op]), alpha)))), 0.5);
          if (kp != k) x[op] = down<T>(conj(xc));
          x[o] = down<T>(xc);
        }
      } else if (x != nullptr) {
        x[o] = down<T>(add(up(x[o]), scl(up(p[o]), alpha)));
      }
      r[o] = down<T>(rc);
      rv[c] = up(down<T>(rc));
    }
    precond(pa, xi_of(f.k1, g.n1, g.il1), xi_of(f.k2, g.n2, g.il2), xi_of(f.k3, g.n3, g.il3), rv, zv);
    // a pair counts twice (weight 1 per entry), other points with the
    // half-spectrum weight
    const double w = (kp != k) ? 2.0 : half_weight(f.k3, g.n3);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
      b += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
    }
    rz += w * a;
    rr += w * b;
  }
  const double s1 = block_sum<kVecThreads>(rz, red);
  const double s2 = block_sum<kVecThreads>(rr, red);
  if (threadIdx.x == 0) {
    partials[2 * chunk] = s1;
    partials[2 * chunk + 1] = s2;
  }
}

// p = M r + beta p
template <typename T>
__device__ __forceinline__ void pupdate_core(cpx<T>* __restrict__ p, const cpx<T>* __restrict__ r,
                                             const PcgScalars* __restrict__ sc, const PrecondArgs& pa, const Geom& g,
                                             int chunk, int nchunks) {
  if (sc->converged) return;
  const double beta = sc->beta;
  const long long nh = g.nh;
  for (long long k = (long long)chunk * kVecThreads + threadIdx.x; k < nh;
       k += (long long)nchunks * kVecThreads) {
    const FreqIdx f = decode(k, g);
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = up(r[c * nh + k]);
    precond(pa, xi_of(f.k1, g.n1, g.il1), xi_of(f.k2, g.n2, g.il2), xi_of(f.k3, g.n3, g.il3), rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o = c * nh + k;
      p[o] = down<T>(add(zv[c], scl(up(p[o]), beta)));
    }
  }
}

// p = M r; partial <r, M r> and <r, r>.  r is first projected onto
// Hermitian pairs on the self-conjugate planes (as in update_core).
// WRITE_P = false: the projection and the partial sums only (p untouched).
template <typename T, bool WRITE_P = true>
__device__ __forceinline__ void pinit_core(cpx<T>* __restrict__ p, cpx<T>* __restrict__ r,
                                           const PrecondArgs& pa, const Geom& g, double* __restrict__ partials,
                                           int chunk, int nchunks) {
  __shared__ double red[kVecThreads / 64];
  double rz = 0.0, rr = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)chunk * kVecThreads + threadIdx.x; k < nh;
       k += (long long)nchunks * kVecThreads) {
    const FreqIdx f = decode(k, g);
    long long kp = k;
    const bool plane = conj_plane(f.k3, g.n3);
    if (plane) {
      kp = partner_index(f, g);
      if (kp < k) continue;
    }
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cpx<double> rc = up(r[c * nh + k]);
      if (plane) {
        rc = scl(add(rc, conj(up(r[c * nh + kp]))), 0.5);
        r[c * nh + k] = down<T>(rc);
        if (kp != k) r[c * nh + kp] = down<T>(conj(rc));
      }
      rv[c] = up(down<T>(rc));
    }
    precond(pa, xi_of(f.k1, g.n1, g.il1), xi_of(f.k2, g.n2, g.il2), xi_of(f.k3, g.n3, g.il3), rv, zv);
    const double w = (kp != k) ? 2.0 : half_weight(f.k3, g.n3);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (WRITE_P) {
        p[c * nh + k] = down<T>(zv[c]);
        if (kp != k) p[c * nh + kp] = down<T>(conj(zv[c]));
      }
      a += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
      b += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
    }
    rz += w * a;
    rr += w * b;
  }
  const double s1 = block_sum<kVecThreads>(rz, red);
  const double s2 = block_sum<kVecThreads>(rr, red);
  if (threadIdx.x == 0) {
    partials[2 * chunk] = s1;
    partials[2 * chunk + 1] = s2;
  }
}

// fixed-order sum of strided partials, result in thread 0
static __device__ double reduce_fixed(const double* partials, int nparts, int stride, int off, double* red) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) s += partials[(long long)b * stride + off];
  return block_sum<kVecThreads>(s, red);
}

__device__ __forceinline__ double frob_stored(const double* t, int ncomp) {
  double s = 0.0;
  if (ncomp == 6) {
    for (int c = 0; c < 3; ++c) s += t[c] * t[c];
    for (int c = 3; c < 6; ++c) s += 2.0 * t[c] * t[c];
  } else {
    for (int c = 0; c < 9; ++c) s += t[c] * t[c];
  }
  return sqrt(s);
}

// macroscopic part of the step: x_e += alpha p_e, r_e -= alpha B:<sigma(p)>,
// tracked average stress += alpha <sigma(p)> (thread 0)
__device__ __forceinline__ void macro_step(PcgScalars* __restrict__ sc, double alpha, const double* __restrict__ dc,
                                           const PcgConst& pc) {
  for (int a = 0; a < pc.nmacro; ++a) {
    double qe = 0.0;
    for (int c = 0; c < pc.ncomp; ++c) qe += pc.basis[a][c] * (pc.ncomp == 6 && c >= 3 ? 2.0 : 1.0) * dc[c];
    sc->qe[a] = qe;
    sc->xe[a] += alpha * sc->pe[a];
    sc->re[a] -= alpha * qe;
  }
  for (int c = 0; c < pc.ncomp; ++c) sc->sig[c] += alpha * dc[c];
}

// alpha = <r,z>/<p,Kp>; macro block of x and r; tracked average stress.
// partials: energy sums of the z pass (one per block) = <p, K p>.  The
// field part of x takes alpha p in the direction kernel (`pending`, as in
// the fused iteration) unless the update kernel is given x.
__device__ __forceinline__ void alpha_core(PcgScalars* __restrict__ sc, const double* __restrict__ partials,
                                           int nparts, const double* __restrict__ dc, const PcgConst& pc) {
  __shared__ double red[kVecThreads / 64];
  // state staged in LDS while the partials are read (as in beta_core)
  __shared__ PcgScalars s;
  __shared__ double sdc[9];
  constexpr int kWords = (int)(sizeof(PcgScalars) / sizeof(int));
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += blockDim.x)
    reinterpret_cast<int*>(&s)[i] = reinterpret_cast<const int*>(sc)[i];
  if (tid < 9) sdc[tid] = dc[tid];
  double pv = 0.0;
  for (int i = tid; i < nparts; i += blockDim.x) pv += partials[i];
  const double pq = block_sum<kVecThreads>(pv, red);
  if (s.converged) {
    if (tid == 0) sc->pending = 0;
    return;
  }
  if (tid == 0) {
    s.pq = pq;
    if (!(pq > 0.0)) {
      s.converged = 2;
      s.pending = 0;
    } else {
      const double alpha = s.rz / pq;
      s.alpha = alpha;
      s.pending = 1;
      macro_step(&s, alpha, sdc, pc);
    }
  }
  __syncthreads();
  for (int i = tid; i < kWords; i += blockDim.x)
    reinterpret_cast<int*>(sc)[i] = reinterpret_cast<const int*>(&s)[i];
}

// beta, macro block of p, convergence.  first == 1: initial call after
// p = M r (no beta, iteration counter stays 0).  first == 2: the residual
// was replaced by a recomputed one and the iteration goes on with the same
// direction: beta = <r, M r> / rho with rho the <r, M r> the direction was
// formed with (left in sc->rz by the host), counter unchanged.
// dc != nullptr (fused CG): the macroscopic step of this iteration is taken
// first, with the average stress of the direction from the divergence pass.
__device__ __forceinline__ void beta_core(PcgScalars* __restrict__ sc, const double* __restrict__ partials,
                                          int nparts, const PcgConst& pc, int first,
                                          const double* __restrict__ dc = nullptr) {
  __shared__ double red[kVecThreads / 64];
  // The scalar state is copied to LDS by the first threads while every
  // thread reads its partial sums, so the single thread that finishes the
  // step reads no global memory; the block writes the state back.
  __shared__ PcgScalars s;
  __shared__ double sdc[9];
  constexpr int kWords = (int)(sizeof(PcgScalars) / sizeof(int));
  static_assert(sizeof(PcgScalars) % sizeof(int) == 0, "PcgScalars is copied word by word");
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += blockDim.x)
    reinterpret_cast<int*>(&s)[i] = reinterpret_cast<const int*>(sc)[i];
  if (dc != nullptr && tid < 9) sdc[tid] = dc[tid];
  // fixed order: thread t sums partials t, t + blockDim, ... (as reduce_fixed)
  double pa_ = 0.0, pb_ = 0.0;
  for (int i = tid; i < nparts; i += blockDim.x) {
    pa_ += partials[2 * (long long)i];
    pb_ += partials[2 * (long long)i + 1];
  }
  const double rz_a = block_sum<kVecThreads>(pa_, red);
  const double rr = block_sum<kVecThreads>(pb_, red);
  if (s.converged) return;
  if (tid == 0) {
    if (dc != nullptr) macro_step(&s, s.alpha, sdc, pc);
    double ze[kMaxMacro];
    double rz = rz_a, re2 = 0.0;
    for (int a = 0; a < pc.nmacro; ++a) {
      double z = 0.0;
      for (int b = 0; b < pc.nmacro; ++b) z += pc.Me[a][b] * s.re[b];
      ze[a] = z;
      rz += s.re[a] * z;
      re2 += s.re[a] * s.re[a];
    }
    double beta = 0.0;
    if (first == 1) {
      s.iter = 0;
    } else {
      beta = rz / s.rz;
      if (first == 0) s.iter += 1;
    }
    s.beta = beta;
    s.rz = rz;
    s.rr = rr;
    s.re2 = re2;
    const double nrm = pc.scale > 0.0 ? pc.scale : frob_stored(s.sig, pc.ncomp);
    const double ra = sqrt(rr > 0.0 ? rr : 0.0), rl = sqrt(re2);
    double eq, ld;
    if (nrm == 0.0) {
      eq = (ra == 0.0) ? 0.0 : INFINITY;
      ld = (rl == 0.0) ? 0.0 : INFINITY;
    } else {
      eq = ra / nrm;
      ld = rl / nrm;
    }
    s.eq_res = eq;
    s.load_res = ld;
    if (eq < pc.tol && ld < pc.tol_load) s.converged = 1;
    else if (s.iter >= pc.max_iter) s.converged = 3;
    // Macro block of the next direction, p_e = z_e + beta p_e, and its
    // tensor for the next operator application.  Once stopped, p_e (like the
    // field part of p, which the direction kernels leave alone then) keeps
    // the last direction, from which an iteration with a replaced residual
    // goes on.
    if (!s.converged || first == 1) {
      for (int a = 0; a < pc.nmacro; ++a) s.pe[a] = ze[a] + beta * s.pe[a];
      for (int c = 0; c < 9; ++c) {
        double m = 0.0;
        for (int a = 0; a < pc.nmacro; ++a) m += s.pe[a] * pc.basis[a][c];
        s.pmac[c] = m;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < kWords; i += blockDim.x)
    reinterpret_cast<int*>(sc)[i] = reinterpret_cast<const int*>(&s)[i];
}

// fused CG: x += alpha p (if this iteration's step is pending), then
// p = M r + beta p (unless converged)
template <typename T>
__device__ __forceinline__ void xp_core(cpx<T>* __restrict__ x, cpx<T>* __restrict__ p, const cpx<T>* __restrict__ r,
                                        const PcgScalars* __restrict__ sc, const PrecondArgs& pa, const Geom& g,
                                        int chunk, int nchunks) {
  const int pending = sc->pending;
  const int conv = sc->converged;
  if (!pending && conv) return;
  const double alpha = sc->alpha, beta = sc->beta;
  const long long nh = g.nh;
  for (long long k = (long long)chunk * kVecThreads + threadIdx.x; k < nh;
       k += (long long)nchunks * kVecThreads) {
    const FreqIdx f = decode(k, g);
    cpx<double> pv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[c] = up(p[c * nh + k]);
    if (pending) {
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c * nh + k] = down<T>(add(up(x[c * nh + k]), scl(pv[c], alpha)));
    }
    if (!conv) {
      cpx<double> rv[3], zv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) rv[c] = up(r[c * nh + k]);
      precond(pa, xi_of(f.k1, g.n1, g.il1), xi_of(f.k2, g.n2, g.il2), xi_of(f.k3, g.n3, g.il3), rv, zv);
#pragma unroll
      for (int c = 0; c < 3; ++c) p[c * nh + k] = down<T>(add(zv[c], scl(pv[c], beta)));
    }
  }
}

}  // namespace dbfft
