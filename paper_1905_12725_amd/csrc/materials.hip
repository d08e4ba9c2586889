// Per-voxel constitutive updates and field reductions.
//
//  * rate-dependent J2 viscoplasticity with anisotropic (rotated cubic)
//    elasticity, backward Euler with unknowns (sigma, y = ln dp):
//      R1 = S sigma - (eps - eps_p_n) + exp(y) n(sigma),
//      R2 = m ln(s_eq / s0) - y + ln(edot0 dt),
//    started from a scalar estimate and finished by a 7x7 Newton; the
//    consistent tangent is [S + dp dn/dsigma + dp (m / s_eq) n n^T]^-1;
//  * compressible neo-Hookean first Piola-Kirchhoff stress, plus the
//    per-voxel data (F^-1, ln J) the fused operator needs for K:H;
//  * Saint Venant-Kirchhoff first Piola-Kirchhoff stress (Sec. 3.3), plus
//    the per-voxel data (F, S) the fused operator needs for K:H;
//  * voxel averages of the tangent (the preconditioner's mean stiffness,
//    Sec. 2.5), max-norm of a field difference (Newton stop, Sec. 2.4),
//    adjoint gradient density.
#include "fft_common.h"

namespace dbfft {

constexpr int kMatThreads = 256;
constexpr double kR2 = 1.41421356237309504880;

// Gaussian elimination with partial pivoting on an n x n system (n <= 7),
// in place; solution written to b.
template <int NMAX>
__device__ bool gauss_solve(double (*A)[NMAX], double* b, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = fabs(A[k][k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        piv = i;
      }
    if (!(best > 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        const double t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      const double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    const double inv = 1.0 / A[k][k];
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i][k] * inv;
      if (f != 0.0) {
        for (int j = k; j < n; ++j) A[i][j] -= f * A[k][j];
        b[i] -= f * b[k];
      }
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k][j] * b[j];
    b[k] = s / A[k][k];
  }
  return true;
}

// inverse of a 6x6 matrix via column-by-column solves
__device__ bool inv6(const double (*A)[6], double (*X)[6]) {
  for (int c = 0; c < 6; ++c) {
    double W[6][6];
    double e[6];
    for (int i = 0; i < 6; ++i) {
      for (int j = 0; j < 6; ++j) W[i][j] = A[i][j];
      e[i] = (i == c) ? 1.0 : 0.0;
    }
    if (!gauss_solve<6>(W, e, 6)) return false;
    for (int i = 0; i < 6; ++i) X[i][c] = e[i];
  }
  return true;
}

__device__ __forceinline__ void seq_n(const double* sg, double& seq, double* n) {
  const double p = (sg[0] + sg[1] + sg[2]) / 3.0;
  double s[6] = {sg[0] - p, sg[1] - p, sg[2] - p, sg[3], sg[4], sg[5]};
  double ss = 0.0;
  for (int a = 0; a < 6; ++a) ss += s[a] * s[a];
  seq = sqrt(1.5 * ss);
  for (int a = 0; a < 6; ++a) n[a] = 1.5 * s[a] / seq;
}

// Cholesky factor of a symmetric positive definite 6x6 matrix (lower
// triangle of A used), all indices compile-time so nothing leaves registers
__device__ __forceinline__ bool chol6(const double (&A)[6][6], double (&L)[6][6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return false;
    const double ljj = sqrt(d);
    L[j][j] = ljj;
    const double inv = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double v = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v * inv;
    }
  }
  return true;
}

// solves L L^T x = b in place
__device__ __forceinline__ void chol6_solve(const double (&L)[6][6], double (&b)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[i][k] * b[k];
    b[i] = v / L[i][i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double v = b[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) v -= L[k][i] * b[k];
    b[i] = v / L[i][i];
  }
}

// M = S + c1 (P_dev - (2/3) n n^T) + c2 n n^T, S the grain's compliance
__device__ __forceinline__ void flow_matrix(const double* __restrict__ S36, const double (&n)[6], double c1, double c2,
                                            double (&M)[6][6]) {
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const double pd = ((a == b) ? 1.0 : 0.0) - ((a < 3 && b < 3) ? 1.0 / 3.0 : 0.0);
      M[a][b] = S36[a * 6 + b] + c1 * (pd - (2.0 / 3.0) * n[a] * n[b]) + c2 * n[a] * n[b];
    }
}

// Backward-Euler J2 viscoplastic update in (sigma, y = ln dp).  The 7x7
// Newton system [[A, e^y n], [(m/s_eq) n^T, -1]] is reduced to its 6x6 Schur
// complement A + e^y (m/s_eq) n n^T (symmetric positive definite: A = S +
// e^y (3/(2 s_eq)) (P_dev - (2/3) n n^T)), solved by Cholesky; the
// consistent tangent is the inverse of the same form at the converged state.
__global__ __launch_bounds__(kMatThreads) void k_j2_update(const double* __restrict__ eps,
                                                          const double* __restrict__ epsp_n,
                                                          const int32_t* __restrict__ grain,
                                                          const double* __restrict__ gC, const double* __restrict__ gS,
                                                          double s0, double m, double edot0, double dt, long long nvox,
                                                          double* __restrict__ sig_out, double* __restrict__ tan21,
                                                          double* __restrict__ epsp_new, int* __restrict__ fail) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  const int gid = grain[v];
  const double* C36 = gC + (long long)gid * 36;
  const double* S36 = gS + (long long)gid * 36;
  double ee[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const double e = eps[(long long)a * nvox + v];
    ee[a] = ((a < 3) ? e : kR2 * e) - epsp_n[(long long)a * nvox + v];
  }
  double str[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc += C36[a * 6 + b] * ee[b];
    str[a] = acc;
  }
  double seq_tr, ntr[6];
  {
    const double p = (str[0] + str[1] + str[2]) / 3.0;
    const double s[6] = {str[0] - p, str[1] - p, str[2] - p, str[3], str[4], str[5]};
    double ss = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) ss += s[a] * s[a];
    seq_tr = sqrt(1.5 * ss);
#pragma unroll
    for (int a = 0; a < 6; ++a) ntr[a] = (seq_tr > 0.0) ? 1.5 * s[a] / seq_tr : 0.0;
  }
  double sg[6], dp = 0.0, n[6];
  bool elastic = !(seq_tr > 1e-12 * s0);
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    n[a] = 0.0;
    sg[a] = str[a];
  }
  if (!elastic) {
    const double logc = log(edot0 * dt);
    double Cn[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) acc += C36[a * 6 + b] * ntr[b];
      Cn[a] = acc;
    }
    double h = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) h += ntr[a] * Cn[a];
    double lo = fmin(log(0.5 * seq_tr / h), logc + m * log(0.5 * seq_tr / s0));
    double hi = log(seq_tr / h);
    double y = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
      const double ey = exp(y), ep = exp((y - logc) / m);
      const double gv = seq_tr - h * ey - s0 * ep;
      const double dg = -h * ey - (s0 / m) * ep;
      if (gv > 0.0) lo = y;
      else hi = y;
      double yn = y - gv / dg;
      if (yn <= lo || yn >= hi) yn = 0.5 * (lo + hi);
      const bool done = fabs(yn - y) <= 1e-14 * fmax(1.0, fabs(y));
      y = yn;
      if (done) break;
    }
    {
      const double ey = exp(y);
#pragma unroll
      for (int a = 0; a < 6; ++a) sg[a] = str[a] - ey * Cn[a];
    }
    for (int it = 0; it < 100; ++it) {
      double seq;
      seq_n(sg, seq, n);
      const double ey = exp(y);
      double R[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) acc += S36[a * 6 + b] * sg[b];
        R[a] = -(acc - ee[a] + ey * n[a]);
      }
      const double R6 = -(m * log(seq / s0) - y + logc);
      double A[6][6], L[6][6];
      flow_matrix(S36, n, ey * 1.5 / seq, ey * m / seq, A);
#pragma unroll
      for (int a = 0; a < 6; ++a) R[a] += ey * R6 * n[a];
      if (!chol6(A, L)) {
        ok = false;
        break;
      }
      chol6_solve(L, R);
      double nd = 0.0, dmax = 0.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        nd += n[a] * R[a];
        sg[a] += R[a];
        dmax = fmax(dmax, fabs(R[a]));
      }
      const double dy = (m / seq) * nd - R6;
      y += dy;
      if (dmax <= 1e-11 * s0 && fabs(dy) <= 1e-11) break;
    }
    double seq;
    seq_n(sg, seq, n);
    dp = exp(y);
  }
  // outputs: stress in stored tensor order, tangent upper triangle, plastic strain (Mandel)
#pragma unroll
  for (int a = 0; a < 6; ++a) sig_out[(long long)a * nvox + v] = (a < 3) ? sg[a] : sg[a] / kR2;
  if (elastic) {
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) tan21[(long long)(idx++) * nvox + v] = 0.5 * (C36[a * 6 + b] + C36[b * 6 + a]);
  } else {
    // consistent tangent: inverse of S + dp (3/(2 s_eq)) (P_dev - (2/3) n n^T) + dp (m/s_eq) n n^T
    double seq;
    {
      double nn[6];
      seq_n(sg, seq, nn);
    }
    double A[6][6], L[6][6];
    flow_matrix(S36, n, dp * 1.5 / seq, dp * m / seq, A);
    if (!chol6(A, L)) ok = false;
    double Ct[6][6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double e[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) e[i] = (i == c) ? 1.0 : 0.0;
      chol6_solve(L, e);
#pragma unroll
      for (int i = 0; i < 6; ++i) Ct[i][c] = e[i];
    }
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) tan21[(long long)(idx++) * nvox + v] = 0.5 * (Ct[a][b] + Ct[b][a]);
  }
  if (!ok || !(dp == dp)) atomicOr(fail, 1);
#pragma unroll
  for (int a = 0; a < 6; ++a) epsp_new[(long long)a * nvox + v] = epsp_n[(long long)a * nvox + v] + dp * n[a];
}

void launch_j2_update(const double* eps, const double* epsp_n, const int32_t* grain, const double* grain_C,
                      const double* grain_S, double s0, double m, double edot0, double dt, long long nvox,
                      double* sig, double* tangent21, double* epsp_new, int* fail, hipStream_t st) {
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_j2_update, dim3(nb), dim3(kMatThreads), 0, st, eps, epsp_n, grain, grain_C, grain_S, s0, m,
                     edot0, dt, nvox, sig, tangent21, epsp_new, fail);
}

// neo-Hookean: P = mu (F - F^-T) + lam ln J F^-T; data = (F^-1 row-major, ln J)
__global__ __launch_bounds__(kMatThreads) void k_neo_update(const double* __restrict__ H,
                                                           const uint8_t* __restrict__ phase, NeoParams np,
                                                           long long nvox, double* __restrict__ P,
                                                           double* __restrict__ data, int* __restrict__ fail) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double F[9];
  for (int i = 0; i < 9; ++i) F[i] = H[(long long)i * nvox + v] + ((i % 4 == 0) ? 1.0 : 0.0);
  const double c00 = F[4] * F[8] - F[5] * F[7];
  const double c01 = F[5] * F[6] - F[3] * F[8];
  const double c02 = F[3] * F[7] - F[4] * F[6];
  const double J = F[0] * c00 + F[1] * c01 + F[2] * c02;
  if (!(J > 0.0)) {
    atomicOr(fail, 1);
  }
  const double iJ = 1.0 / J;
  double Fi[9];  // inverse, row-major: Fi = adj(F)^T... adj_ij = cofactor_ji
  Fi[0] = c00 * iJ;
  Fi[1] = (F[2] * F[7] - F[1] * F[8]) * iJ;
  Fi[2] = (F[1] * F[5] - F[2] * F[4]) * iJ;
  Fi[3] = c01 * iJ;
  Fi[4] = (F[0] * F[8] - F[2] * F[6]) * iJ;
  Fi[5] = (F[2] * F[3] - F[0] * F[5]) * iJ;
  Fi[6] = c02 * iJ;
  Fi[7] = (F[1] * F[6] - F[0] * F[7]) * iJ;
  Fi[8] = (F[0] * F[4] - F[1] * F[3]) * iJ;
  const double lnJ = log(J);
  const int p = phase[v];
  const double mu = np.mu[p], lam = np.lam[p];
  for (int i = 0; i < 3; ++i)
    for (int Jc = 0; Jc < 3; ++Jc) {
      const double FiT = Fi[Jc * 3 + i];
      P[(long long)(i * 3 + Jc) * nvox + v] = mu * (F[i * 3 + Jc] - FiT) + lam * lnJ * FiT;
    }
  for (int i = 0; i < 9; ++i) data[(long long)i * nvox + v] = Fi[i];
  data[9LL * nvox + v] = lnJ;
}

void launch_neo_update(const double* H, const uint8_t* phase, const NeoParams& np, long long nvox, double* P,
                       double* data, int* fail, hipStream_t st) {
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_neo_update, dim3(nb), dim3(kMatThreads), 0, st, H, phase, np, nvox, P, data, fail);
}

// Saint Venant-Kirchhoff: E = (F^T F - I)/2, S = lam tr(E) I + 2 mu E,
// P = F S; data = (F row-major, S stored order 11 22 33 23 13 12).  No
// failure condition: the law is defined for every F.
__global__ __launch_bounds__(kMatThreads) void k_svk_update(const double* __restrict__ H,
                                                           const uint8_t* __restrict__ phase, NeoParams np,
                                                           long long nvox, double* __restrict__ P,
                                                           double* __restrict__ data) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double F[9];
  for (int i = 0; i < 9; ++i) F[i] = H[(long long)i * nvox + v] + ((i % 4 == 0) ? 1.0 : 0.0);
  double E[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double c = 0.0;
      for (int k = 0; k < 3; ++k) c += F[k * 3 + a] * F[k * 3 + b];
      E[a * 3 + b] = 0.5 * (c - (a == b ? 1.0 : 0.0));
    }
  const int p = phase[v];
  const double mu = np.mu[p], lam = np.lam[p];
  const double tr = E[0] + E[4] + E[8];
  double S[9];
  for (int a = 0; a < 9; ++a) S[a] = 2.0 * mu * E[a] + ((a % 4 == 0) ? lam * tr : 0.0);
  for (int i = 0; i < 3; ++i)
    for (int J = 0; J < 3; ++J) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += F[i * 3 + k] * S[k * 3 + J];
      P[(long long)(i * 3 + J) * nvox + v] = acc;
    }
  for (int i = 0; i < 9; ++i) data[(long long)i * nvox + v] = F[i];
  const int sidx[6] = {0, 4, 8, 5, 2, 1};
  for (int a = 0; a < 6; ++a) data[(long long)(9 + a) * nvox + v] = S[sidx[a]];
}

void launch_svk_update(const double* H, const uint8_t* phase, const NeoParams& np, long long nvox, double* P,
                       double* data, int* fail, hipStream_t st) {
  (void)fail;
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_svk_update, dim3(nb), dim3(kMatThreads), 0, st, H, phase, np, nvox, P, data);
}

// ------------------------------------------------------------ tangent mean
constexpr int kMeanBlocks = 512;
int tangent_mean_block_count(const Geom&) { return kMeanBlocks; }
int tangent_mean_nvals(int kin) { return kin == KIN_SMALL ? 21 : 81; }

// finite strains: all 81 components of a voxel from one read of its field
// entries; each component gets the same terms, in the same voxel order and
// with the same block sums, as a sweep of its own would give
template <typename T>
__global__ __launch_bounds__(kMatThreads) void k_tangent_mean_finite(TangentArgs<T> tn, Geom g,
                                                                    double* __restrict__ partials) {
  // finite strains: all 81 components of a voxel from one read of its
  // field entries; each component gets the same terms, in the same voxel
  // order, as a sweep of its own would give
  double acc[81];
#pragma unroll
  for (int c = 0; c < 81; ++c) acc[c] = 0.0;
  for (long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x; v < g.nvox;
       v += (long long)gridDim.x * kMatThreads) {
    const int p = tn.phase[v];
    const double mu = tn.mu[p], lam = tn.lam[p];
    if (tn.kind == TAN_SVK_FIELD) {
      // K_iJkL = d_ik S_LJ + lam F_iJ F_kL + mu (F_iL F_kJ + (F F^T)_ik d_JL)
      const int smap[9] = {0, 5, 4, 5, 1, 3, 4, 3, 2};  // (a, b) -> stored index
      double F[9], S[6];
#pragma unroll
      for (int q = 0; q < 9; ++q) F[q] = (double)tn.field[(long long)q * g.nvox + v];
#pragma unroll
      for (int q = 0; q < 6; ++q) S[q] = (double)tn.field[(long long)(9 + q) * g.nvox + v];
#pragma unroll
      for (int c = 0; c < 81; ++c) {
        const int L = c % 3, k = (c / 3) % 3, J = (c / 9) % 3, i = c / 27;
        double FFt = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) FFt += F[i * 3 + q] * F[k * 3 + q];
        acc[c] += ((i == k) ? S[smap[L * 3 + J]] : 0.0) + lam * F[i * 3 + J] * F[k * 3 + L] +
                  mu * (F[i * 3 + L] * F[k * 3 + J] + ((J == L) ? FFt : 0.0));
      }
    } else {
      // K_iJkL = mu d_ik d_JL + (mu - lam ln J) Finv_Li Finv_Jk + lam Finv_Ji Finv_Lk
      double Fi[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) Fi[q] = (double)tn.field[(long long)q * g.nvox + v];
      const double lnJ = (double)tn.field[9LL * g.nvox + v];
#pragma unroll
      for (int c = 0; c < 81; ++c) {
        const int L = c % 3, k = (c / 3) % 3, J = (c / 9) % 3, i = c / 27;
        acc[c] += ((i == k && J == L) ? mu : 0.0) + (mu - lam * lnJ) * Fi[L * 3 + i] * Fi[J * 3 + k] +
                  lam * Fi[J * 3 + i] * Fi[L * 3 + k];
      }
    }
  }
  // block sums as block_sum forms them (wave shuffles, then the waves in
  // order), all components at once
  __shared__ double wred[81][kMatThreads / 64];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < 81; ++c) {
    double s = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (ln == 0) wred[c][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 81) {
    double s = 0.0;
    for (int w = 0; w < kMatThreads / 64; ++w) s += wred[threadIdx.x][w];
    partials[(long long)blockIdx.x * 81 + threadIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kMatThreads) void k_tangent_mean(TangentArgs<T> tn, int kin, Geom g,
                                                             double* __restrict__ partials) {
  // small strains: the 21 Mandel upper-triangle components, one sweep each
  __shared__ double red[kMatThreads / 64];
  (void)kin;
  constexpr int nv = 21;
  for (int c = 0; c < nv; ++c) {
    double acc = 0.0;
    // Mandel upper-triangle index c -> (a, b)
    int a = 0, b = 0, idx = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) {
        if (idx == c) {
          a = i;
          b = j;
        }
        ++idx;
      }
    for (long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x; v < g.nvox;
         v += (long long)gridDim.x * kMatThreads) {
      double val;
      if (tn.kind == TAN_ISO_PHASE || tn.kind == TAN_ISO_FIELD) {
        double lam, mu;
        if (tn.kind == TAN_ISO_PHASE) {
          lam = tn.lam[tn.phase[v]];
          mu = tn.mu[tn.phase[v]];
        } else {
          const double E = (double)tn.field[v];
          lam = tn.lam1 * E;
          mu = tn.mu1 * E;
        }
        val = ((a < 3 && b < 3) ? lam : 0.0) + ((a == b) ? 2.0 * mu : 0.0);
      } else if (tn.kind == TAN_ANISO_GRAIN) {
        val = tn.grain_table[(long long)tn.grain[v] * 21 + c];
      } else {
        val = (double)tn.field[(long long)c * g.nvox + v];
      }
      acc += val;
    }
    const double s = block_sum<kMatThreads>(acc, red);
    if (threadIdx.x == 0) partials[(long long)blockIdx.x * nv + c] = s;
    __syncthreads();
  }
}

template <typename T>
void launch_tangent_mean(const TangentArgs<T>& tan, int kin, const Geom& g, double* partials, int nblocks,
                         hipStream_t st) {
  if (kin == KIN_SMALL)
    hipLaunchKernelGGL((k_tangent_mean<T>), dim3(nblocks), dim3(kMatThreads), 0, st, tan, kin, g, partials);
  else
    hipLaunchKernelGGL((k_tangent_mean_finite<T>), dim3(nblocks), dim3(kMatThreads), 0, st, tan, g, partials);
}
template void launch_tangent_mean<double>(const TangentArgs<double>&, int, const Geom&, double*, int, hipStream_t);
template void launch_tangent_mean<float>(const TangentArgs<float>&, int, const Geom&, double*, int, hipStream_t);

// ------------------------------------------------------------ misc reductions
__global__ __launch_bounds__(kMatThreads) void k_max_abs_diff(const double* __restrict__ a,
                                                             const double* __restrict__ b, long long n,
                                                             double* __restrict__ partials) {
  __shared__ double red[kMatThreads];
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * kMatThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kMatThreads)
    m = fmax(m, fabs(b != nullptr ? a[i] - b[i] : a[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kMatThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}
void launch_max_abs_diff(const double* a, const double* b, long long n, double* partials, int nblocks,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_max_abs_diff, dim3(nblocks), dim3(kMatThreads), 0, st, a, b, n, partials);
}

// g(x) = scale * eta : C1 : eps with isotropic unit-modulus C1 (stored order)
__global__ __launch_bounds__(kMatThreads) void k_adjoint_density(const double* __restrict__ eps,
                                                                const double* __restrict__ eta, double lam1,
                                                                double mu1, long long nvox, double* __restrict__ grad,
                                                                double scale) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double e[6], h[6];
  for (int c = 0; c < 6; ++c) {
    e[c] = eps[(long long)c * nvox + v];
    h[c] = eta[(long long)c * nvox + v];
  }
  const double tre = e[0] + e[1] + e[2], trh = h[0] + h[1] + h[2];
  const double dd = h[0] * e[0] + h[1] * e[1] + h[2] * e[2] + 2.0 * (h[3] * e[3] + h[4] * e[4] + h[5] * e[5]);
  grad[v] = scale * (lam1 * trh * tre + 2.0 * mu1 * dd);
}
void launch_adjoint_density(const double* eps, const double* eta, double lam1, double mu1, long long nvox,
                            double* grad, double scale, hipStream_t st) {
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_adjoint_density, dim3(nb), dim3(kMatThreads), 0, st, eps, eta, lam1, mu1, nvox, grad, scale);
}

// g(x) = scale * sum_c A_c(x) B_c(x) over nc component-major fields
// ------------------------------------------------------------------ J2 adjoint
__device__ __forceinline__ void load_sym21(const double* __restrict__ t21, long long nvox, long long v,
                                           double (*K)[6]) {
  int idx = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b) {
      const double x = t21[(long long)(idx++) * nvox + v];
      K[a][b] = x;
      K[b][a] = x;
    }
}

__device__ __forceinline__ void matvec6(const double (*A)[6], const double* x, double* y) {
  for (int a = 0; a < 6; ++a) {
    double acc = 0.0;
    for (int b = 0; b < 6; ++b) acc += A[a][b] * x[b];
    y[a] = acc;
  }
}

__device__ __forceinline__ void grain_matvec6(const double* __restrict__ M36, const double* x, double* y) {
  for (int a = 0; a < 6; ++a) {
    double acc = 0.0;
    for (int b = 0; b < 6; ++b) acc += M36[a * 6 + b] * x[b];
    y[a] = acc;
  }
}

struct EU6 {
  double v[6];
};

__global__ __launch_bounds__(kMatThreads) void k_j2_adj_prestress(const double* __restrict__ lam,
                                                                 const double* __restrict__ tan21,
                                                                 const int32_t* __restrict__ grain,
                                                                 const double* __restrict__ gS, EU6 eu,
                                                                 long long nvox, double* __restrict__ sig0) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double K[6][6], l[6], sl[6], u[6], out[6];
  load_sym21(tan21, nvox, v, K);
  for (int a = 0; a < 6; ++a) l[a] = lam[(long long)a * nvox + v];
  grain_matvec6(gS + (long long)grain[v] * 36, l, sl);
  // u = EU - S lam, so K u + lam = K EU + lam - K S lam
  for (int a = 0; a < 6; ++a) u[a] = ((a < 3) ? eu.v[a] : kR2 * eu.v[a]) - sl[a];
  matvec6(K, u, out);
  for (int a = 0; a < 6; ++a) {
    const double m = out[a] + l[a];
    sig0[(long long)a * nvox + v] = (a < 3) ? m : m / kR2;
  }
}

void launch_j2_adj_prestress(const double* lam, const double* tan21, const int32_t* grain, const double* grain_S,
                             const double EU_st[6], long long nvox, double* sig0, hipStream_t st) {
  EU6 eu;
  for (int a = 0; a < 6; ++a) eu.v[a] = EU_st[a];
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_j2_adj_prestress, dim3(nb), dim3(kMatThreads), 0, st, lam, tan21, grain, grain_S, eu, nvox,
                     sig0);
}

__global__ __launch_bounds__(kMatThreads) void k_j2_adj_back(double* __restrict__ lam,
                                                            const double* __restrict__ tan21,
                                                            const int32_t* __restrict__ grain,
                                                            const double* __restrict__ gS,
                                                            const double* __restrict__ eps_star,
                                                            const double* __restrict__ p_new,
                                                            const double* __restrict__ p_old, double scale,
                                                            long long nvox, double* __restrict__ grad) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double K[6][6], l[6], sl[6], u[6], ln[6];
  load_sym21(tan21, nvox, v, K);
  for (int a = 0; a < 6; ++a) l[a] = lam[(long long)a * nvox + v];
  grain_matvec6(gS + (long long)grain[v] * 36, l, sl);
  for (int a = 0; a < 6; ++a) {
    const double e = eps_star[(long long)a * nvox + v];
    u[a] = sl[a] - ((a < 3) ? e : kR2 * e);
  }
  matvec6(K, u, ln);
  double acc = 0.0;
  for (int a = 0; a < 6; ++a) {
    acc += (p_new[(long long)a * nvox + v] - p_old[(long long)a * nvox + v]) * ln[a];
    lam[(long long)a * nvox + v] = ln[a];
  }
  grad[v] += scale * acc;
}

void launch_j2_adj_back(double* lam, const double* tan21, const int32_t* grain, const double* grain_S,
                        const double* eps_star, const double* p_new, const double* p_old, double scale, long long nvox,
                        double* grad, hipStream_t st) {
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_j2_adj_back, dim3(nb), dim3(kMatThreads), 0, st, lam, tan21, grain, grain_S, eps_star, p_new,
                     p_old, scale, nvox, grad);
}

__global__ __launch_bounds__(kMatThreads) void k_contract(const double* __restrict__ A, const double* __restrict__ B,
                                                         int nc, long long nvox, double* __restrict__ grad,
                                                         double scale) {
  const long long v = (long long)blockIdx.x * kMatThreads + threadIdx.x;
  if (v >= nvox) return;
  double acc = 0.0;
  for (int c = 0; c < nc; ++c) acc += A[(long long)c * nvox + v] * B[(long long)c * nvox + v];
  grad[v] = scale * acc;
}
void launch_contract(const double* A, const double* B, int nc, long long nvox, double* grad, double scale,
                     hipStream_t st) {
  const int nb = (int)((nvox + kMatThreads - 1) / kMatThreads);
  hipLaunchKernelGGL(k_contract, dim3(nb), dim3(kMatThreads), 0, st, A, B, nc, nvox, grad, scale);
}

}  // namespace dbfft
