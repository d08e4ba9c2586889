// Preconditioned conjugate gradient kernels (complex CG with the
// per-frequency preconditioner of Sec. 2.5 eqs. pred2/pred3).
//
// Vector kernels stream the 3-component half spectrum once per call and
// emit per-block FP64 partial sums; single-block scalar kernels reduce the
// partials in a fixed order (bitwise reproducible), update the scalars and
// the macroscopic block of the unknown, and test convergence on the device,
// so a whole iteration is enqueued with no host round trip.
#include "pcg_core.h"

namespace dbfft {

constexpr int kMaxVecBlocks = 2048;

int pcg_block_count(const Geom& g) {
  long long b = (g.nh + kVecThreads - 1) / kVecThreads;
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_update(cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                                        const cpx<T>* __restrict__ p, const cpx<T>* __restrict__ q,
                                                        const PcgScalars* __restrict__ sc, PrecondArgs pa, Geom g,
                                                        double* __restrict__ partials) {
  update_core<T>(x, r, p, q, sc, pa, g, partials, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pupdate(cpx<T>* __restrict__ p, const cpx<T>* __restrict__ r,
                                                         const PcgScalars* __restrict__ sc, PrecondArgs pa, Geom g) {
  pupdate_core<T>(p, r, sc, pa, g, blockIdx.x, gridDim.x);
}

template <typename T, bool WRITE_P>
__global__ __launch_bounds__(kVecThreads) void k_pinit(cpx<T>* __restrict__ p, cpx<T>* __restrict__ r,
                                                       PrecondArgs pa, Geom g, double* __restrict__ partials) {
  pinit_core<T, WRITE_P>(p, r, pa, g, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kVecThreads) void k_beta(PcgScalars* __restrict__ sc, const double* __restrict__ partials,
                                                      int nparts, PcgConst pc, int first) {
  beta_core(sc, partials, nparts, pc, first);
}

__global__ __launch_bounds__(kVecThreads) void k_beta_step(PcgScalars* __restrict__ sc,
                                                           const double* __restrict__ partials, int nparts,
                                                           const double* __restrict__ dc, PcgConst pc) {
  beta_core(sc, partials, nparts, pc, 0, dc);
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_xp(cpx<T>* __restrict__ x, cpx<T>* __restrict__ p,
                                                    const cpx<T>* __restrict__ r, const PcgScalars* __restrict__ sc,
                                                    PrecondArgs pa, Geom g) {
  xp_core<T>(x, p, r, sc, pa, g, blockIdx.x, gridDim.x);
}

void launch_pcg_beta_step(PcgScalars* sc, const double* partials, int nparts, const double* dc, const PcgConst& pc,
                          hipStream_t st) {
  DB_LAUNCH(k_beta_step, dim3(1), dim3(kVecThreads), 0, st, sc, partials, nparts, dc, pc);
}
template <typename T>
void launch_pcg_xp(void* x, void* p, const void* r, const PcgScalars* sc, const PrecondArgs& pa, const Geom& g,
                   int nblocks, hipStream_t st) {
  DB_LAUNCH((k_xp<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(x),
                     static_cast<cpx<T>*>(p), static_cast<const cpx<T>*>(r), sc, pa, g);
}
template void launch_pcg_xp<double>(void*, void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                    hipStream_t);
template void launch_pcg_xp<float>(void*, void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                   hipStream_t);

int fused_cg_partials(const Geom& g) {
  // divergence tiles (at least 2 columns each): all (k2, k3) pairs, padding,
  // then the two plane columns again; two sums each
  return 2 * (int)(((long long)g.n2 * (g.nh3 + 2) + 1) / 2 + 2);
}

template <typename T>
void launch_pcg_update(void* x, void* r, const void* p, const void* q, const PcgScalars* sc, const PrecondArgs& pa,
                       const Geom& g, double* partials, int nblocks, hipStream_t st) {
  DB_LAUNCH((k_update<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(x),
                     static_cast<cpx<T>*>(r), static_cast<const cpx<T>*>(p), static_cast<const cpx<T>*>(q), sc, pa, g,
                     partials);
}
template <typename T>
void launch_pcg_pupdate(void* p, const void* r, const PcgScalars* sc, const PrecondArgs& pa, const Geom& g,
                        int nblocks, hipStream_t st) {
  DB_LAUNCH((k_pupdate<T>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(p),
                     static_cast<const cpx<T>*>(r), sc, pa, g);
}
template <typename T>
void launch_precond_init(void* p, void* r, const PrecondArgs& pa, const Geom& g, double* partials, int nblocks,
                         hipStream_t st) {
  DB_LAUNCH((k_pinit<T, true>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(p),
                     static_cast<cpx<T>*>(r), pa, g, partials);
}
template <typename T>
void launch_precond_dots(void* r, const PrecondArgs& pa, const Geom& g, double* partials, int nblocks,
                         hipStream_t st) {
  DB_LAUNCH((k_pinit<T, false>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<cpx<T>*>(nullptr),
                     static_cast<cpx<T>*>(r), pa, g, partials);
}
template void launch_precond_dots<double>(void*, const PrecondArgs&, const Geom&, double*, int, hipStream_t);
template void launch_precond_dots<float>(void*, const PrecondArgs&, const Geom&, double*, int, hipStream_t);
void launch_pcg_beta(PcgScalars* sc, const double* partials, int nparts, const PcgConst& pc, int first,
                     hipStream_t st) {
  DB_LAUNCH(k_beta, dim3(1), dim3(kVecThreads), 0, st, sc, partials, nparts, pc, first);
}

template void launch_pcg_update<double>(void*, void*, const void*, const void*, const PcgScalars*,
                                        const PrecondArgs&, const Geom&, double*, int, hipStream_t);
template void launch_pcg_update<float>(void*, void*, const void*, const void*, const PcgScalars*,
                                       const PrecondArgs&, const Geom&, double*, int, hipStream_t);
template void launch_pcg_pupdate<double>(void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                         hipStream_t);
template void launch_pcg_pupdate<float>(void*, const void*, const PcgScalars*, const PrecondArgs&, const Geom&, int,
                                        hipStream_t);
template void launch_precond_init<double>(void*, void*, const PrecondArgs&, const Geom&, double*, int,
                                          hipStream_t);
template void launch_precond_init<float>(void*, void*, const PrecondArgs&, const Geom&, double*, int,
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
  DB_LAUNCH((k_axpby<T>), dim3((int)nb), dim3(256), 0, st, static_cast<T*>(y), static_cast<const T*>(x), a, b, n);
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
  DB_LAUNCH((k_convert<Tin, Tout>), dim3((int)nb), dim3(256), 0, st, static_cast<Tout*>(out),
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
    DB_LAUNCH((k_dotw<float>), dim3(nblocks), dim3(kVecThreads), 0, st, static_cast<const cpx<float>*>(u),
                       static_cast<const cpx<float>*>(v), g, partials);
  else
    DB_LAUNCH((k_dotw<double>), dim3(nblocks), dim3(kVecThreads), 0, st,
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
  DB_LAUNCH(k_reduce, dim3(1), dim3(kVecThreads), 0, st, partials, nparts, nvals, out);
}

// ------------------------------------------------------------- block PCG
// Inner products of two blocks of 3-component half-spectrum vectors (FP64):
// partials[b * na * nb + i * nb + j] = block b's part of
// sum_k w(k3) Re(conj(A_i(k)) B_j(k)), the weighted real inner product.
__global__ __launch_bounds__(kVecThreads) void k_block_dot(BlockVecs A, BlockVecs B, int na, int nb, Geom g,
                                                           double* __restrict__ partials) {
  __shared__ double red[kVecThreads / 64];
  double acc[kMaxBlock][kMaxBlock];
#pragma unroll
  for (int i = 0; i < kMaxBlock; ++i)
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) acc[i][j] = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const double w = half_weight((int)(k % g.nh3), g.n3);
    cpx<double> a[kMaxBlock][3];
#pragma unroll
    for (int i = 0; i < kMaxBlock; ++i)
      if (i < na)
#pragma unroll
        for (int c = 0; c < 3; ++c) a[i][c] = static_cast<const cpx<double>*>(A.v[i])[c * nh + k];
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) {
      if (j >= nb) break;
      cpx<double> bv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) bv[c] = static_cast<const cpx<double>*>(B.v[j])[c * nh + k];
#pragma unroll
      for (int i = 0; i < kMaxBlock; ++i)
        if (i < na) {
          double t = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) t += a[i][c].x * bv[c].x + a[i][c].y * bv[c].y;
          acc[i][j] += w * t;
        }
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxBlock; ++i)
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j)
      if (i < na && j < nb) {
        const double sum = block_sum<kVecThreads>(acc[i][j], red);
        if (threadIdx.x == 0) partials[(long long)blockIdx.x * na * nb + i * nb + j] = sum;
      }
}

// Y_j = ybeta Y_j + sum_i X_i C[i][j] (j < ny, i < nx), FP64.  norms != null:
// block partials of the weighted squared norm of every Y_j after the update,
// partials[b * ny + j].
__global__ __launch_bounds__(kVecThreads) void k_block_comb(BlockVecs X, BlockVecs Y, int nx, int ny, BlockCoef C,
                                                            double ybeta, Geom g, double* __restrict__ norms) {
  __shared__ double red[kVecThreads / 64];
  double nrm[kMaxBlock];
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) nrm[j] = 0.0;
  const long long nh = g.nh;
  for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < nh;
       k += (long long)gridDim.x * kVecThreads) {
    const double w = half_weight((int)(k % g.nh3), g.n3);
    cpx<double> x[kMaxBlock][3];
#pragma unroll
    for (int i = 0; i < kMaxBlock; ++i)
      if (i < nx)
#pragma unroll
        for (int c = 0; c < 3; ++c) x[i][c] = static_cast<const cpx<double>*>(X.v[i])[c * nh + k];
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) {
      if (j >= ny) break;
      cpx<double>* y = static_cast<cpx<double>*>(const_cast<void*>(Y.v[j]));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cpx<double> v = (ybeta != 0.0) ? scl(y[c * nh + k], ybeta) : mk<double>(0, 0);
#pragma unroll
        for (int i = 0; i < kMaxBlock; ++i)
          if (i < nx) v = add(v, scl(x[i][c], C.c[i][j]));
        y[c * nh + k] = v;
        nrm[j] += w * (v.x * v.x + v.y * v.y);
      }
    }
  }
  if (norms == nullptr) return;
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j)
    if (j < ny) {
      const double sum = block_sum<kVecThreads>(nrm[j], red);
      if (threadIdx.x == 0) norms[(long long)blockIdx.x * ny + j] = sum;
    }
}

// Coarse unknowns of a two-level preconditioner: for point p (linear
// half-spectrum index idx[p]) and component c, out[6p + 2c] = sqrt(2) Re v,
// out[6p + 2c + 1] = sqrt(2) Im v (the coordinates along the orthonormal
// coarse basis).
__global__ void k_coarse_gather(const cpx<double>* __restrict__ v, const long long* __restrict__ idx, int npts,
                                long long nh, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 3 * npts) return;
  const int p = j / 3, c = j % 3;
  const cpx<double> a = v[c * nh + idx[p]];
  const double s = 1.4142135623730951;
  out[6 * p + 2 * c] = s * a.x;
  out[6 * p + 2 * c + 1] = s * a.y;
}

// v(k) = (y_re + i y_im) / sqrt(2) at every coarse point, and its conjugate at
// the partner point (-k) on the self-conjugate planes (partner[p] >= 0)
__global__ void k_coarse_scatter(cpx<double>* __restrict__ v, const long long* __restrict__ idx,
                                 const long long* __restrict__ partner, int npts, long long nh,
                                 const double* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 3 * npts) return;
  const int p = j / 3, c = j % 3;
  const double s = 0.7071067811865476;
  const cpx<double> a = mk<double>(s * y[6 * p + 2 * c], s * y[6 * p + 2 * c + 1]);
  v[c * nh + idx[p]] = a;
  if (partner[p] >= 0) v[c * nh + partner[p]] = conj(a);
}

void launch_coarse_gather(const void* v, const long long* idx, int npts, long long nh, double* out, hipStream_t st) {
  const int n = 3 * npts;
  DB_LAUNCH(k_coarse_gather, dim3((n + 255) / 256), dim3(256), 0, st, static_cast<const cpx<double>*>(v), idx, npts,
            nh, out);
}
void launch_coarse_scatter(void* v, const long long* idx, const long long* partner, int npts, long long nh,
                           const double* y, hipStream_t st) {
  const int n = 3 * npts;
  DB_LAUNCH(k_coarse_scatter, dim3((n + 255) / 256), dim3(256), 0, st, static_cast<cpx<double>*>(v), idx, partner,
            npts, nh, y);
}

// ------------------------------------------------------------- error estimates
// Compatibility measure of Sec. 3 (eq. chedckcomp; its finite-strain form in
// Sec. 3.3) on the normalized coefficients of a strain field, in place.
// With A v = xi x v (A_il = e_ikl xi_k): small strains (6 stored components
// 11 22 33 23 13 12) eta = curl curl eps becomes -A eps A^T; finite strains
// (9 components H_il, row-major) the row-wise curl (curl H)_ij = e_jkl d_k H_il
// becomes i (H A^T).  xi is that of the gradient (Nyquist zeroed).
__global__ __launch_bounds__(kVecThreads) void k_incompat(cpx<double>* __restrict__ w, Geom g, int finite) {
  const long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x;
  if (k >= g.nh) return;
  const FreqIdx f = decode(k, g);
  const double x1 = xi_of(f.k1, g.n1, g.il1), x2 = xi_of(f.k2, g.n2, g.il2), x3 = xi_of(f.k3, g.n3, g.il3);
  const double A[3][3] = {{0.0, -x3, x2}, {x3, 0.0, -x1}, {-x2, x1, 0.0}};
  const long long nh = g.nh;
  if (finite) {
    cpx<double> H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int l = 0; l < 3; ++l) H[i][l] = w[(i * 3 + l) * nh + k];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cpx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
        for (int l = 0; l < 3; ++l) s = add(s, scl(H[i][l], A[j][l]));
        w[(i * 3 + j) * nh + k] = mk<double>(-s.y, s.x);  // i s
      }
    return;
  }
  constexpr int ci[6] = {0, 1, 2, 1, 0, 0}, cj[6] = {0, 1, 2, 2, 2, 1};
  cpx<double> e[3][3];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const cpx<double> v = w[c * nh + k];
    e[ci[c]][cj[c]] = v;
    e[cj[c]][ci[c]] = v;
  }
  cpx<double> B[3][3];  // eps A^T
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
      for (int n = 0; n < 3; ++n) s = add(s, scl(e[l][n], A[j][n]));
      B[l][j] = s;
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    cpx<double> s = mk<double>(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < 3; ++l) s = add(s, scl(B[l][cj[c]], A[ci[c]][l]));
    w[c * nh + k] = scl(s, -1.0);
  }
}

void launch_incompat(void* w, const Geom& g, int finite, hipStream_t st) {
  DB_LAUNCH(k_incompat, dim3((unsigned)((g.nh + kVecThreads - 1) / kVecThreads)), dim3(kVecThreads), 0, st,
            static_cast<cpx<double>*>(w), g, finite);
}

void launch_block_dot(const BlockVecs& A, const BlockVecs& B, int na, int nb, const Geom& g, double* partials,
                      int nblocks, hipStream_t st) {
  DB_LAUNCH(k_block_dot, dim3(nblocks), dim3(kVecThreads), 0, st, A, B, na, nb, g, partials);
}
void launch_block_comb(const BlockVecs& X, const BlockVecs& Y, int nx, int ny, const BlockCoef& C, double ybeta,
                       const Geom& g, double* norms, int nblocks, hipStream_t st) {
  DB_LAUNCH(k_block_comb, dim3(nblocks), dim3(kVecThreads), 0, st, X, Y, nx, ny, C, ybeta, g, norms);
}

}  // namespace dbfft
