// Preconditioned conjugate gradient kernels (complex CG with the
// per-frequency preconditioner of Sec. 2.5 eqs. pred2/pred3).
//
// Vector kernels stream the 3-component half spectrum once per call and
// emit per-block FP64 partial sums; single-block scalar kernels reduce the
// partials in a fixed order (bitwise reproducible), update the scalars and
// the macroscopic block of the unknown, and test convergence on the device,
// so a whole iteration is enqueued with no host round trip.
#include "fft_common.h"

namespace dbfft {

constexpr int kVecThreads = 256;
constexpr int kMaxVecBlocks = 2048;

int pcg_block_count(const Geom& g) {
  long long b = (g.nh + kVecThreads - 1) / kVecThreads;
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

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

// x += alpha p; r -= alpha q; partial <r, M r> and <r, r>
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_update(cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                                        const cpx<T>* __restrict__ p, const cpx<T>* __restrict__ q,
                                                        const PcgScalars* __restrict__ sc, PrecondArgs pa, Geom g,
                                                        double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  if (sc->converged) return;
  const double alpha = sc->alpha;
  double rz = 0.0, rr = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const FreqIdx f = decode(k, g);
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o = c * nh + k;
      cpx<double> xc = up(x[o]), pc = up(p[o]), rc = up(r[o]), qc = up(q[o]);
      xc = add(xc, scl(pc, alpha));
      rc = sub(rc, scl(qc, alpha));
      x[o] = down<T>(xc);
      r[o] = down<T>(rc);
      rv[c] = up(down<T>(rc));
    }
    precond(pa, xi_of(f.k1, g.n1), xi_of(f.k2, g.n2), xi_of(f.k3, g.n3), rv, zv);
    const double w = half_weight(f.k3, g.n3);
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
    partials[2 * blockIdx.x] = s1;
    partials[2 * blockIdx.x + 1] = s2;
  }
}

// p = M r + beta p
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pupdate(cpx<T>* __restrict__ p, const cpx<T>* __restrict__ r,
                                                         const PcgScalars* __restrict__ sc, PrecondArgs pa, Geom g) {
  if (sc->converged) return;
  const double beta = sc->beta;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const FreqIdx f = decode(k, g);
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = up(r[c * nh + k]);
    precond(pa, xi_of(f.k1, g.n1), xi_of(f.k2, g.n2), xi_of(f.k3, g.n3), rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long o = c * nh + k;
      p[o] = down<T>(add(zv[c], scl(up(p[o]), beta)));
    }
  }
}

// p = M r; partial <r, M r> and <r, r>
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pinit(cpx<T>* __restrict__ p, const cpx<T>* __restrict__ r,
                                                       PrecondArgs pa, Geom g, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  double rz = 0.0, rr = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const FreqIdx f = decode(k, g);
    cpx<double> rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = up(r[c * nh + k]);
    precond(pa, xi_of(f.k1, g.n1), xi_of(f.k2, g.n2), xi_of(f.k3, g.n3), rv, zv);
    const double w = half_weight(f.k3, g.n3);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p[c * nh + k] = down<T>(zv[c]);
      a += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
      b += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
    }
    rz += w * a;
    rr += w * b;
  }
  const double s1 = block_sum<kVecThreads>(rz, red);
  const double s2 = block_sum<kVecThreads>(rr, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s1;
    partials[2 * blockIdx.x + 1] = s2;
  }
}

// fixed-order sum of strided partials, result in thread 0
__device__ double reduce_fixed(const double* partials, int nparts, int stride, int off, double* red) {
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

// alpha = <r,z>/<p,Kp>; macro block of x and r; tracked average stress.
// partials: energy sums of the z pass (one per block) = <p, K p>.
__global__ __launch_bounds__(kVecThreads) void k_alpha(PcgScalars* __restrict__ sc, const double* __restrict__ partials,
                                                       int nparts, const double* __restrict__ dc, PcgConst pc) {
  __shared__ double red[kVecThreads / 64];
  if (sc->converged) return;
  const double pq = reduce_fixed(partials, nparts, 1, 0, red);
  if (threadIdx.x != 0) return;
  sc->pq = pq;
  if (!(pq > 0.0)) {
    sc->converged = 2;
    return;
  }
  const double alpha = sc->rz / pq;
  sc->alpha = alpha;
  for (int a = 0; a < pc.nmacro; ++a) {
    double qe = 0.0;
    for (int c = 0; c < pc.ncomp; ++c) qe += pc.basis[a][c] * (pc.ncomp == 6 && c >= 3 ? 2.0 : 1.0) * dc[c];
    sc->qe[a] = qe;
    sc->xe[a] += alpha * sc->pe[a];
    sc->re[a] -= alpha * qe;
  }
  for (int c = 0; c < pc.ncomp; ++c) sc->sig[c] += alpha * dc[c];
}

// beta, macro block of p, convergence.  first != 0: initial call after
// p = M r (no beta, iteration counter stays 0).
__global__ __launch_bounds__(kVecThreads) void k_beta(PcgScalars* __restrict__ sc, const double* __restrict__ partials,
                                                      int nparts, PcgConst pc, int first) {
  __shared__ double red[kVecThreads / 64];
  if (sc->converged) return;
  const double rz_a = reduce_fixed(partials, nparts, 2, 0, red);
  const double rr = reduce_fixed(partials, nparts, 2, 1, red);
  if (threadIdx.x != 0) return;
  double ze[kMaxMacro];
  double rz = rz_a, re2 = 0.0;
  for (int a = 0; a < pc.nmacro; ++a) {
    double z = 0.0;
    for (int b = 0; b < pc.nmacro; ++b) z += pc.Me[a][b] * sc->re[b];
    ze[a] = z;
    rz += sc->re[a] * z;
    re2 += sc->re[a] * sc->re[a];
  }
  if (first) {
    for (int a = 0; a < pc.nmacro; ++a) sc->pe[a] = ze[a];
    sc->iter = 0;
  } else {
    const double beta = rz / sc->rz;
    sc->beta = beta;
    for (int a = 0; a < pc.nmacro; ++a) sc->pe[a] = ze[a] + beta * sc->pe[a];
    sc->iter += 1;
  }
  sc->rz = rz;
  sc->rr = rr;
  sc->re2 = re2;
  const double nrm = frob_stored(sc->sig, pc.ncomp);
  const double ra = sqrt(rr > 0.0 ? rr : 0.0), rl = sqrt(re2);
  double eq, ld;
  if (nrm == 0.0) {
    eq = (ra == 0.0) ? 0.0 : INFINITY;
    ld = (rl == 0.0) ? 0.0 : INFINITY;
  } else {
    eq = ra / nrm;
    ld = rl / nrm;
  }
  sc->eq_res = eq;
  sc->load_res = ld;
  // macro tensor of p for the next operator application
  for (int c = 0; c < 9; ++c) {
    double m = 0.0;
    for (int a = 0; a < pc.nmacro; ++a) m += sc->pe[a] * pc.basis[a][c];
    sc->pmac[c] = m;
  }
  if (eq < pc.tol && ld < pc.tol_load) sc->converged = 1;
  else if (sc->iter >= pc.max_iter) sc->converged = 3;
}

template <typename T>
void launch_pcg_update(void* x, void* r, const void* p, const void* q, const PcgScalars* sc, const PrecondArgs& pa,
                       const Geom& g, double* partials, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_update<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(x),
                     static_cast<cpx<T>*>(r), static_cast<const cpx<T>*>(p), static_cast<const cpx<T>*>(q), sc, pa, g,
                     partials);
}
template <typename T>
void launch_pcg_pupdate(void* p, const void* r, const PcgScalars* sc, const PrecondArgs& pa, const Geom& g,
                        int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_pupdate<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(p),
                     static_cast<const cpx<T>*>(r), sc, pa, g);
}
template <typename T>
void launch_precond_init(void* p, const void* r, const PrecondArgs& pa, const Geom& g, double* partials, int nblocks,
                         hipStream_t st) {
  hipLaunchKernelGGL((k_pinit<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(p),
                     static_cast<const cpx<T>*>(r), pa, g, partials);
}
void launch_pcg_alpha(PcgScalars* sc, const double* partials, int nparts, const double* dc, const PcgConst& pc,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kVecThreads), 0, st, sc, partials, nparts, dc, pc);
}
void launch_pcg_beta(PcgScalars* sc, const double* partials, int nparts, const PcgConst& pc, int first,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_beta, dim3(1), dim3(kVecThreads), 0, st, sc, partials, nparts, pc, first);
}

template void launch_pcg_update<double>(void*, void*, const void*, const void*, const PcgScalars*,
                                        const PrecondArgs&, const Geom&, double*, int, hipStream_t);
template void launch_pcg_update<float>(void*, void*, const void*, const void*, const PcgScalars*,
                                       const PrecondArgs&, const Geom&, double*, int, hipStream_t);
template void launch_pcg_pupdate<double>(void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                         hipStream_t);
template void launch_pcg_pupdate<float>(void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                        hipStream_t);
template void launch_precond_init<double>(void*, const void*, const PrecondArgs&, const Geom&, double*, int,
                                          hipStream_t);
template void launch_precond_init<float>(void*, const void*, const PrecondArgs&, const Geom&, double*, int,
                                         hipStream_t);

// ------------------------------------------------------------- vector utilities
template <typename T>
__global__ void k_axpby(T* y, const T* x, double a, double b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}
template <typename T>
void launch_axpby(void* y, const void* x, double a, double b, long long n, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_axpby<T>), dim3((int)nb), dim3(256), 0, st, static_cast<T*>(y), static_cast<const T*>(x), a, b, n);
}
template void launch_axpby<double>(void*, const void*, double, double, long long, hipStream_t);
template void launch_axpby<float>(void*, const void*, double, double, long long, hipStream_t);

template <typename Tin, typename Tout>
__global__ void k_convert(Tout* __restrict__ out, const Tin* __restrict__ in, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (Tout)in[i];
}
template <typename Tin, typename Tout>
void launch_convert(void* out, const void* in, long long n, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3((int)nb), dim3(256), 0, st, static_cast<Tout*>(out),
                     static_cast<const Tin*>(in), n);
}
template void launch_convert<double, float>(void*, const void*, long long, hipStream_t);
template void launch_convert<float, double>(void*, const void*, long long, hipStream_t);
template void launch_convert<double, double>(void*, const void*, long long, hipStream_t);

// weighted inner product of two 3-component half-spectrum vectors
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_dotw(const cpx<T>* __restrict__ u, const cpx<T>* __restrict__ v,
                                                      Geom g, double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  double acc = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const int k3 = (int)(k % g.nh3);
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cpx<T> x = u[c * nh + k], y = v[c * nh + k];
      a += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
    }
    acc += half_weight(k3, g.n3) * a;
  }
  const double s = block_sum<kVecThreads>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
void launch_dot_w(const void* u, const void* v, int isf32, const Geom& g, double* partials, int nblocks,
                  hipStream_t st) {
  if (isf32)
    hipLaunchKernelGGL((k_dotw<float>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<const cpx<float>*>(u),
                       static_cast<const cpx<float>*>(v), g, partials);
  else
    hipLaunchKernelGGL((k_dotw<double>), dim3(nblocks), dim3(kVecThreads), 0, st,
                       static_cast<const cpx<double>*>(u), static_cast<const cpx<double>*>(v), g, partials);
}

__global__ __launch_bounds__(kVecThreads) void k_reduce(const double* __restrict__ partials, int nparts, int nvals,
                                                        double* __restrict__ out) {
  __shared__ double red[kVecThreads / 64];
  for (int v = 0; v < nvals; ++v) {
    const double s = reduce_fixed(partials, nparts, nvals, v, red);
    if (threadIdx.x == 0) out[v] = s;
    __syncthreads();
  }
}
void launch_reduce(const double* partials, int nparts, int nvals, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kVecThreads), 0, st, partials, nparts, nvals, out);
}

}  // namespace dbfft
