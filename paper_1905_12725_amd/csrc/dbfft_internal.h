// Internal declarations shared by the HIP kernels and the host engine.
//
// Layouts (all device arrays, C order):
//   half spectrum  [c][k1][k2][k3]   k3 = 0 .. n3/2   (complex, T2 = float2/double2)
//   real field     [c][x][y][z]      z fastest        (T)
// A vector of the Krylov space is 3 half-spectrum components plus a small
// FP64 macro block kept separately.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

namespace dbfft {

// Per-kernel timing: when the engine times a PCG kernel it leaves a pair of
// events here before the launch; DB_LAUNCH then launches through
// hipExtLaunchKernelGGL, which records them at the kernel's own start and
// end (the kernel's execution time, without the gap to the previous
// kernel), and counts the launches so the engine knows whether the pair
// covered the only kernel of the timed step.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  int consumed = 0;
  long long launches = 0;
};
extern thread_local LaunchTiming g_launch_timing;
#define DB_LAUNCH(K, GRID, BLOCK, SHM, ST, ...)                                                            \
  do {                                                                                                    \
    ::dbfft::LaunchTiming& lt_ = ::dbfft::g_launch_timing;                                                \
    if (lt_.start != nullptr) {                                                                           \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, lt_.start, lt_.stop, 0u, __VA_ARGS__);               \
      lt_.start = lt_.stop = nullptr;                                                                     \
      lt_.consumed = 1;                                                                                   \
    } else {                                                                                              \
      hipLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, __VA_ARGS__);                                           \
    }                                                                                                     \
    ++lt_.launches;                                                                                       \
  } while (0)

constexpr int kMaxStages = 12;
constexpr int kMaxPhases = 8;
constexpr int kMaxMacro = 9;
constexpr double kTwoPi = 6.283185307179586;  // nearest double to 2*pi

// Stockham plan of one complex transform of length n = prod(radix).
struct FftPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int ns[kMaxStages];  // length of the sub-transforms combined before the stage
};

struct Geom {
  int n1, n2, n3, nh3;  // nh3 = n3/2 + 1
  long long nh;         // n1*n2*nh3
  long long nvox;       // n1*n2*n3
  double inv_nvox;
  double il1, il2, il3;  // 1 / cell side length per axis (frequencies 2 pi m / L)
};

enum Kin : int { KIN_SMALL = 0, KIN_FINITE = 1 };

// Pointwise tangent used inside the fused z pass.
enum TanKind : int {
  TAN_ISO_PHASE = 0,   // uint8 phase id -> (lambda, mu)
  TAN_ISO_FIELD = 1,   // per-voxel modulus scaling unit-modulus (lambda1, mu1)
  TAN_ANISO_GRAIN = 2, // int32 grain id -> 21 Mandel coefficients (table)
  TAN_ANISO_FIELD = 3, // 21 Mandel coefficients per voxel, [21][nvox]
  TAN_NEO_FIELD = 4,   // finite strain: per-voxel F^-1 (9) and ln J, [10][nvox]; phase -> (mu, lambda)
  TAN_SVK_FIELD = 5,   // finite strain: per-voxel F (9) and S (11 22 33 23 13 12), [15][nvox]; phase -> (mu, lambda)
};

template <typename T>
struct TangentArgs {
  int kind;
  int nphase;
  double lam[kMaxPhases];
  double mu[kMaxPhases];
  double lam1, mu1;             // TAN_ISO_FIELD
  const uint8_t* phase;         // TAN_ISO_PHASE, TAN_NEO_FIELD
  const T* field;               // TAN_ISO_FIELD: [nvox]; ANISO_FIELD: [21][nvox]; NEO: [10][nvox]
  const int32_t* grain;         // TAN_ANISO_GRAIN
  const double* grain_table;    // TAN_ANISO_GRAIN: [ngrain][21]
};

// Preconditioner M(xi) = [xi.Cbar.xi]^-1: A_ik = sum_{j<=l} xi_j xi_l G[jl][ik]
// (symmetric 3x3 stored as 6: 00 11 22 12 02 01).
struct PrecondArgs {
  double G[6][6];
};

// Device-resident scalars of one PCG solve.
struct PcgScalars {
  double rz;          // <r, z>
  double pq;          // <p, K p>
  double alpha, beta;
  double rr;          // <r_a, r_a> (full-spectrum norm^2 of the displacement part)
  double re2;         // |r_e|^2
  double sig[9];      // average stress (or nominal stress) of the current iterate
  double xe[kMaxMacro], re[kMaxMacro], pe[kMaxMacro], qe[kMaxMacro];
  double pmac[9];     // macro strain tensor of p (stored component order), read by the z pass
  double eq_res, load_res;
  int iter;
  int converged;      // 1 converged, 2 breakdown, 3 iteration cap
  int pending;        // fused CG: alpha of this iteration still to be added to x
  int pad;
};

struct PcgConst {
  double tol, tol_load;
  int max_iter;
  int nmacro;                         // |S|
  int ncomp;                          // 6 or 9
  double Me[kMaxMacro][kMaxMacro];    // macro preconditioner
  double basis[kMaxMacro][9];         // B_a as row-major 3x3 (stress-controlled set only)
  double scale;                       // > 0: fixed scale of the residual test; 0: ||<sigma>||
};

// ---------------------------------------------------------------- launchers
// All launches are asynchronous on `st`.  T is float or double.

// x/y passes over lines with element stride `lstride`, `nother` lines per
// column tile (other index stride `ostride`), contiguous k3 columns.
struct StridedGeom {
  int nline;          // transform length
  long long lstride;  // element stride along the line
  long long ostride;  // stride of the other (non-transformed, non-k3) index
  int nother;         // count of the other index
  int ncols;          // nh3
  long long cstride_in, cstride_out;  // component strides
};

enum StridedMode : int {
  SP_PLAIN = 0,       // C independent components (grid z = component)
  SP_GRAD_SMALL = 1,  // in: 3 comps a -> out: 6 comps i/2 (xi_j a_i + xi_i a_j), then inverse FFT along x
  SP_GRAD_FINITE = 2, // in: 3 comps a -> out: 9 comps i xi_j a_i, inverse FFT along x
  SP_DIV_SMALL = 3,   // in: 6 comps, forward FFT along x, out: 3 comps -i xi_j s_ij
  SP_DIV_FINITE = 4,  // in: 9 comps, forward FFT along x, out: 3 comps
};

// alpha of a PCG iteration, computed by the first block of a pass (the
// fused iteration's y forward pass, the separate iteration's x forward
// pass) from the energy partials of the z pass before it
struct AlphaTask {
  PcgScalars* sc = nullptr;
  const double* eparts = nullptr;
  int neparts = 0;
};

template <typename T>
void launch_strided(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg,
                    const Geom& g, const FftPlan& plan, const void* tw, int dir, double* dc_out,
                    hipStream_t st, const int* stop, const AlphaTask& at = AlphaTask());

enum LineMode : int {
  LP_FUSED = 0,       // C2R -> (+ macro) -> tangent -> R2C (scaled 1/N); energy partials
  LP_C2R = 1,         // C2R (+ macro) -> real out
  LP_R2C = 2,         // real in -> R2C scaled 1/N
  LP_CONST = 3,       // constant field (macro only) -> tangent -> R2C scaled 1/N
  LP_STRESS = 4,      // C2R (+ macro) -> tangent -> real out
};

template <typename T>
void launch_line(int mode, int kin, const void* in, void* out, const Geom& g, const FftPlan& plan,
                 const void* tw, const void* rtw, const TangentArgs<T>& tan, const double* macro_dev,
                 const double* macro_add, double* partials, int ncomp, hipStream_t st, int* nblocks_out,
                 const int* stop);

int line_block_count(const Geom& g);
// number of blocks (= energy partials) of the fused z pass for this grid
int fused_line_blocks(const Geom& g, int ncomp, int elem_bytes, int tan_kind);

// register-resident kernels for power-of-two transform lengths
bool fast_strided_supported(int n);
// two-step register z pass (fused tangent) for n3/2 a 2-3-5-smooth length
// that is not a power of two: isotropic tangents in both precisions, any
// tangent in FP32
bool mixed_line_supported(int n3, int elem_bytes, bool iso);
int mixed_line_blocks(const Geom& g);
// real z transforms (LP_C2R with macro_dev + macro_add, LP_R2C scaled 1/N),
// one component per grid y, for even n3 with n3/2 in the two-step set
bool real_line_supported(int n3);
template <typename T>
void launch_line_real(int mode, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                      const double* mac_a, const double* mac_b, int ncomp, hipStream_t st);
// fused z pass of the odd two-step lengths 15, 25, 27, 45, 63 (isotropic
// small strains), two parts
bool odd_line_supported(int n3);
int odd_line_energy_blocks(const Geom& g);
// staged z pass of anisotropic / finite-strain tangents on power-of-two
// lines (n3 = 32, 64; FP32 also 128)
bool staged_line_supported(int n3, int elem_bytes, bool iso, bool finite);
int staged_line_blocks(const Geom& g);
template <typename T>
void launch_line_staged(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                        const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                        const int* stop);
template <typename T>
void launch_line_odd(const void* in, void* out, const Geom& g, const void* tw, const TangentArgs<T>& tan,
                     const double* macro_dev, double* partials, hipStream_t st, const int* stop);
// energy partials of the two-step z pass (isotropic: two blocks per line group)
int mixed_line_energy_blocks(const Geom& g, bool iso);
template <typename T>
void launch_line_mixed(int kin, bool iso, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                       const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                       const int* stop);
// two-step register x/y passes for 2-3-5-smooth lengths that are not powers of two
bool mixed_strided_supported(int n);
template <typename T>
void launch_strided_mixed(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                          const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                          const AlphaTask& at = AlphaTask());
bool fast_line_supported(int n3);
int fast_line_blocks(const Geom& g, int elem_bytes);
template <typename T>
void launch_strided_fast(int mode, const void* in, void* out, int ncomp_plain, const StridedGeom& sg, const Geom& g,
                         const void* tw, int dir, double* dc_out, hipStream_t st, const int* stop,
                         const AlphaTask& at = AlphaTask());
template <typename T>
void launch_line_fast(int kin, const void* in, void* out, const Geom& g, const void* tw, const void* rtw,
                      const TangentArgs<T>& tan, const double* macro_dev, double* partials, hipStream_t st,
                      const int* stop);
int line_lines_per_block(const Geom& g, int ncomp, int elem_bytes);
// Length of the complex transform of one z line in the generic z pass: n3/2
// on packed pairs of real samples when n3 is even, n3 on the real samples
// (zero imaginary part) when it is odd.
__host__ __device__ constexpr inline int z_length(int n3) { return (n3 % 2 == 0) ? n3 / 2 : n3; }
// LDS bytes of a generic z-pass block of L lines: twiddles (z_length),
// split twiddles (n3/2 + 1), two transform buffers, the half-spectrum
// staging lines and the real samples of every component.
inline size_t line_smem_bytes(const Geom& g, int L, int ncomp, int elem_bytes) {
  const size_t Z = (size_t)z_length(g.n3), M = (size_t)(g.n3 / 2), l = (size_t)L, eb = (size_t)elem_bytes;
  return (Z + M + 1) * eb + 2 * Z * l * eb + (M + 1) * l * eb + (size_t)ncomp * l * g.n3 * (eb / 2);
}

// PCG vector kernels (3 half-spectrum components).
template <typename T>
void launch_pcg_update(void* x, void* r, const void* p, const void* q, const PcgScalars* sc,
                       const PrecondArgs& pa, const Geom& g, double* partials, int nblocks, hipStream_t st);
template <typename T>
void launch_pcg_pupdate(void* p, const void* r, const PcgScalars* sc, const PrecondArgs& pa,
                        const Geom& g, int nblocks, hipStream_t st);
template <typename T>
void launch_precond_init(void* p, void* r, const PrecondArgs& pa, const Geom& g, double* partials,
                         int nblocks, hipStream_t st);
// the Hermitian projection of r and the partial sums of <r, M r> and <r, r>
// (launch_precond_init without writing p)
template <typename T>
void launch_precond_dots(void* r, const PrecondArgs& pa, const Geom& g, double* partials, int nblocks,
                         hipStream_t st);
// Fused CG iteration (small strains, register-FFT x pass, n2 even): alpha
// after the z pass (first block of the y pass, or its own kernel); the
// divergence pass updates r in place, projects it onto Hermitian pairs on
// the self-conjugate planes and emits the partial sums of <r, M r> and
// <r, r>; beta takes the macroscopic step with the divergence pass's average
// stress; the direction kernel adds alpha p to x and forms the next p.
void launch_pcg_beta_step(PcgScalars* sc, const double* partials, int nparts, const double* dc, const PcgConst& pc,
                          hipStream_t st);
template <typename T>
void launch_pcg_xp(void* x, void* p, const void* r, const PcgScalars* sc, const PrecondArgs& pa, const Geom& g,
                   int nblocks, hipStream_t st);
// x forward transform + divergence + r -= alpha q + Hermitian planes
// (T = float or double; n2 even; alpha already in the scalars); returns the number of partial-sum
// pairs written to `partials`
template <typename T>
int launch_div_update_fast(const void* W, void* r, const StridedGeom& sg, const Geom& g, const void* tw,
                           const PcgScalars* sc, const PrecondArgs& pa, double* dc_out, double* partials,
                           hipStream_t st);
int fused_cg_partials(const Geom& g);
void launch_pcg_beta(PcgScalars* sc, const double* partials, int nparts, const PcgConst& pc, int first,
                     hipStream_t st);
int pcg_block_count(const Geom& g);

// block PCG (FP64): blocks of at most kMaxBlock 3-component half-spectrum vectors
constexpr int kMaxBlock = 6;
struct BlockVecs {
  const void* v[kMaxBlock];
};
struct BlockCoef {
  double c[kMaxBlock][kMaxBlock];
};
// partials[b][i * nb + j] of <A_i, B_j> over nblocks blocks
void launch_block_dot(const BlockVecs& A, const BlockVecs& B, int na, int nb, const Geom& g, double* partials,
                      int nblocks, hipStream_t st);
// Y_j = ybeta Y_j + sum_i X_i C[i][j]; norms (may be null): partials[b][j] of |Y_j|^2
void launch_block_comb(const BlockVecs& X, const BlockVecs& Y, int nx, int ny, const BlockCoef& C, double ybeta,
                       const Geom& g, double* norms, int nblocks, hipStream_t st);

// two-level preconditioner (FP64): coordinates of the coarse unknowns of a
// 3-component vector at the listed half-spectrum points, and their
// write-back (with the conjugate at plane partners, partner >= 0)
void launch_coarse_gather(const void* v, const long long* idx, int npts, long long nh, double* out, hipStream_t st);
void launch_coarse_scatter(void* v, const long long* idx, const long long* partner, int npts, long long nh,
                           const double* y, hipStream_t st);

// vector utilities
template <typename T>
void launch_axpby(void* y, const void* x, double a, double b, long long n2, hipStream_t st);  // y = a x + b y (n2 reals)
template <typename Tin, typename Tout>
void launch_convert(void* out, const void* in, long long n, hipStream_t st);
void launch_dot_w(const void* u, const void* v, int isf32, const Geom& g, double* partials, int nblocks,
                  hipStream_t st);
void launch_reduce(const double* partials, int nparts, int nvals, double* out, hipStream_t st);
// compatibility operator of the error estimate on 6 (small) or 9 (finite)
// half-spectrum FP64 components, in place
void launch_incompat(void* w, const Geom& g, int finite, hipStream_t st);

// materials / fields
template <typename T>
void launch_tangent_mean(const TangentArgs<T>& tan, int kin, const Geom& g, double* partials, int nblocks,
                         hipStream_t st);
int tangent_mean_block_count(const Geom& g);
int tangent_mean_nvals(int kin);

struct NeoParams {
  double mu[kMaxPhases];
  double lam[kMaxPhases];
};

void launch_j2_update(const double* eps, const double* epsp_n, const int32_t* grain, const double* grain_C,
                      const double* grain_S, double s0, double m, double edot0, double dt, long long nvox,
                      double* sig, double* tangent21, double* epsp_new, int* fail, hipStream_t st);
void launch_neo_update(const double* H, const uint8_t* phase, const NeoParams& np, long long nvox, double* P,
                       double* data, int* fail, hipStream_t st);
// Saint Venant-Kirchhoff: P = F S, S = lam tr(E) I + 2 mu E, E = (F^T F - I)/2;
// data = (F row-major, S in stored order) [15][nvox]
void launch_svk_update(const double* H, const uint8_t* phase, const NeoParams& np, long long nvox, double* P,
                       double* data, int* fail, hipStream_t st);
void launch_max_abs_diff(const double* a, const double* b, long long n, double* partials, int nblocks,
                         hipStream_t st);
void launch_adjoint_density(const double* eps, const double* eta, double lam1, double mu1, long long nvox,
                            double* grad, double scale, hipStream_t st);
// J2 adjoint, one increment (Mandel vectors; K from the 21-term upper
// triangle, S the grain's compliance [ngrain][36]):
//  prestress: sig0 = K : EU + lam - K S lam, written in stored tensor order
//  back:      lam <- K (S lam - eps*), grad += scale * (p_new - p_old) . lam
void launch_j2_adj_prestress(const double* lam, const double* tan21, const int32_t* grain, const double* grain_S,
                             const double EU_st[6], long long nvox, double* sig0, hipStream_t st);
void launch_j2_adj_back(double* lam, const double* tan21, const int32_t* grain, const double* grain_S,
                        const double* eps_star, const double* p_new, const double* p_old, double scale, long long nvox,
                        double* grad, hipStream_t st);
// grad(x) = scale * sum_c A_c(x) B_c(x) (component-major [nc][nvox] fields)
void launch_contract(const double* A, const double* B, int nc, long long nvox, double* grad, double scale,
                     hipStream_t st);

}  // namespace dbfft
